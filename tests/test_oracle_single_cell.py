"""The oracle's single-precision model of the DD cell (CELL_DD_SINGLE,
solve(cell_single=True)): the pure diamond-difference cell of the sweep
(paper section II.B; the scheme named in section IV) evaluated in IEEE
single precision, used to show how much single-precision rounding alone
moves a pure-DD solution.  Pins: it is the same cell as the double one up to
rounding, and its arithmetic is single precision."""
import numpy as np
import pytest

import oracle
from synthetic.workloads import SourceSpec, random_small_problem


def _omega(p):
    om, _ = oracle.lqn(p.sn_order)
    return om


def test_single_cell_of_one_voxel_is_the_float32_cell():
    """A one-voxel mesh has vacuum inflow, so psi = q / (sigma + c_x + c_y
    + c_z) with c_a = 2|Omega_a|/Delta_a: the single-precision mode must give
    exactly numpy's float32 evaluation of that expression, and 2 psi as
    outflows."""
    p = random_small_problem(41, n=(1, 1, 1), sn=4, L=0, G=1, n_mat=1)
    rng = np.random.default_rng(4)
    h = np.array([p.dx, p.dy, p.dz])
    for om in _omega(p)[:6]:
        q, sg = rng.uniform(0.1, 3.0, 2)
        psi, out, _ = oracle.sweep_mode(p, om, np.array([sg]), np.array([q]), oracle.CELL_DD_SINGLE)
        c = (2.0 * np.abs(om) / h).astype(np.float32)
        den = np.float32(sg) + c[0]
        den = den + c[1]
        den = den + c[2]
        want = np.float32(q) / den
        assert psi[0] == float(want)
        assert np.all(out[:, 0] == float(np.float32(2.0) * want))


def test_single_cell_sweep_is_single_precision_and_close_to_double():
    """Every cell result of a single-precision sweep is a float32 value, and
    on an optically thin problem with a positive source (no cancellation)
    it stays within float32 rounding of the double sweep."""
    p = random_small_problem(42, n=(7, 5, 6), sn=6, L=0, G=1, n_mat=2)
    rng = np.random.default_rng(5)
    sig = rng.uniform(0.05, 0.2, p.V)
    Q = rng.uniform(0.5, 1.5, p.V)
    for om in _omega(p)[::7]:
        ps, os_, _ = oracle.sweep_mode(p, om, sig, Q, oracle.CELL_DD_SINGLE)
        pd, od, _ = oracle.sweep_mode(p, om, sig, Q, oracle.CELL_DD)
        assert np.all(ps.astype(np.float32).astype(np.float64) == ps)
        assert np.all(os_.astype(np.float32).astype(np.float64) == os_)
        assert np.abs(ps - pd).max() / np.abs(pd).max() < 5e-6
        assert np.abs(ps - pd).max() > 0  # it really rounds


def test_single_cell_solve():
    """A whole pure-DD solve with single-precision cells agrees with the
    double solve to single-precision accuracy on a thin problem; the mode
    refuses the fixup."""
    p = random_small_problem(43, n=(9, 8, 7), sn=4, L=1, G=2, n_mat=2, fixup=0)
    s = SourceSpec(position=(-2.0, 3.1, 2.7), spectrum=np.array([1.0, 0.4]))
    a = oracle.solve(p, s, fixed_iters=[4, 4])["phi_total"]
    b = oracle.solve(p, s, fixed_iters=[4, 4], cell_single=True)["phi_total"]
    assert 0 < np.abs(a - b).max() < 1e-5 * np.abs(a).max()
    q = random_small_problem(43, n=(9, 8, 7), sn=4, L=1, G=2, n_mat=2, fixup=1)
    with pytest.raises(ValueError):
        oracle.solve(q, s, fixed_iters=[1, 1], cell_single=True)
