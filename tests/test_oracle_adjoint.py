"""Pins of the oracle's adjoint and density gradient (no GPU)."""
import numpy as np
import pytest

import oracle
from synthetic.workloads import SourceSpec, random_small_problem


def _sweep_matrix(p, om, sig):
    V = p.V
    A = np.zeros((V, V))
    for v in range(V):
        e = np.zeros(V)
        e[v] = 1.0
        A[:, v] = oracle.sweep(p, om, sig, e)[0]
    return A


def test_dd_sweep_transpose_is_reverse_sweep():
    p = random_small_problem(80, n=(3, 4, 2))
    rng = np.random.default_rng(2)
    sig = rng.uniform(0.1, 2.0, p.V)
    for om in ([0.3, -0.5, 0.81], [-0.6, 0.64, -0.48]):
        om = np.array(om) / np.linalg.norm(om)
        A = _sweep_matrix(p, om, sig)
        B = _sweep_matrix(p, -om, sig)
        assert np.abs(A.T - B).max() < 1e-15 * np.abs(A).max() * 10


def _problem():
    p = random_small_problem(81, n=(3, 4, 3), sn=4, L=1, G=2, n_mat=2, density=True)
    src = SourceSpec(position=(-2.0, 1.5, 1.7), axis=(1.0, 0.1, 0.0), half_angle=np.deg2rad(35),
                     spectrum=np.array([1.0, 0.4]))
    W = np.random.default_rng(3).uniform(0, 1, (p.G, p.V))
    return p, src, W


def test_reciprocity():
    p, src, W = _problem()
    r = oracle.adjoint(p, src, W, tol=1e-15)
    assert abs(r["J"] - r["recip"]) < 1e-12 * abs(r["J"])


def test_gradient_matches_central_differences():
    p, src, W = _problem()
    r = oracle.adjoint(p, src, W, tol=1e-15)
    g = r["grad"]
    h = 1e-3
    fd = np.zeros(p.V)
    for v in range(p.V):
        d = p.density.copy()
        d[v] += h
        jp = (W * oracle.solve(p.with_density(d), src, tol=1e-15)["phi_total"]).sum()
        d[v] -= 2 * h
        jm = (W * oracle.solve(p.with_density(d), src, tol=1e-15)["phi_total"]).sum()
        fd[v] = (jp - jm) / (2 * h)
    assert np.abs(g - fd).max() < 1e-5 * np.abs(fd).max()
    # both the ray back-projection and the scattering terms matter here
    assert np.abs(fd).max() > 0


def test_gradient_source_inside_mesh():
    p = random_small_problem(82, n=(4, 3, 3), sn=2, L=0, G=2, n_mat=2, density=True)
    src = SourceSpec(position=(2.1, 1.3, 1.45), spectrum=np.array([1.0, 0.2]))
    W = np.random.default_rng(4).uniform(0, 1, (p.G, p.V))
    g = oracle.adjoint(p, src, W, tol=1e-15)["grad"]
    h = 1e-3
    for v in (0, 7, 20, 35):
        d = p.density.copy(); d[v] += h
        jp = (W * oracle.solve(p.with_density(d), src, tol=1e-15)["phi_total"]).sum()
        d[v] -= 2 * h
        jm = (W * oracle.solve(p.with_density(d), src, tol=1e-15)["phi_total"]).sum()
        assert abs(g[v] - (jp - jm) / (2 * h)) < 1e-5 * np.abs(g).max()


# --- set-to-zero fixup: frozen-branch linearisation ---------------------------

def _thick(seed, n=(4, 4, 3), sn=4, L=1, G=2):
    """Optically thick cells (6x the generator's cross sections) next to a
    cone source: the pure DD sweep goes negative in many cells, so the fixup
    acts."""
    p = random_small_problem(seed, n=n, sn=sn, L=L, G=G, n_mat=2, density=True, fixup=1)
    p.sigma_t = p.sigma_t * 6.0
    p.sigma_s = p.sigma_s * 6.0
    src = SourceSpec(position=(-2.0, 1.5, 1.7), axis=(1.0, 0.1, 0.0), half_angle=np.deg2rad(35),
                     spectrum=np.array([1.0, 0.4][:G]))
    W = np.random.default_rng(seed).uniform(0, 1, (p.G, p.V))
    return p, src, W


def _spiky(p, seed):
    rng = np.random.default_rng(seed)
    sig = rng.uniform(0.5, 12.0, p.V)
    Q = np.where(rng.uniform(size=p.V) < 0.15, rng.uniform(1.0, 50.0, p.V), 0.0)
    return sig, Q


def test_frozen_cell_reproduces_the_fixup_sweep():
    p, _, _ = _thick(84)
    sig, Q = _spiky(p, 5)
    om = np.array([0.35, -0.6, 0.72]) / np.linalg.norm([0.35, -0.6, 0.72])
    psi, out, mask = oracle.sweep_mode(p, om, sig, Q, oracle.CELL_FIXUP)
    assert (mask != 0).sum() > 5  # the fixup acted in several cells
    psi_f, out_f, _ = oracle.sweep_mode(p, om, sig, Q, oracle.CELL_FROZEN, mask)
    assert np.array_equal(psi, psi_f) and np.array_equal(out, out_f)
    # and CELL_FIXUP equals the default sweep of a fixup problem
    assert np.array_equal(psi, oracle.sweep(p, om, sig, Q)[0])


def test_transposed_frozen_sweep_is_the_matrix_transpose():
    p, _, _ = _thick(84, n=(3, 4, 3))
    sig, Q = _spiky(p, 6)
    for om in ([0.35, -0.6, 0.72], [-0.8, 0.3, -0.52]):
        om = np.array(om) / np.linalg.norm(om)
        _, _, mask = oracle.sweep_mode(p, om, sig, Q, oracle.CELL_FIXUP)
        assert (mask != 0).sum() > 3
        V = p.V
        A = np.zeros((V, V))
        B = np.zeros((V, V))
        for v in range(V):
            e = np.zeros(V)
            e[v] = 1.0
            A[:, v] = oracle.sweep_mode(p, om, sig, e, oracle.CELL_FROZEN, mask)[0]
            B[:, v] = oracle.sweep_mode(p, -om, sig, e, oracle.CELL_TRANS, mask)[0]
        assert np.abs(A.T - B).max() < 1e-14 * np.abs(A).max()
        # the frozen map is not the pure DD map: the fixup matters here
        D = np.zeros((V, V))
        for v in range(V):
            e = np.zeros(V)
            e[v] = 1.0
            D[:, v] = oracle.sweep_mode(p, om, sig, e, oracle.CELL_DD)[0]
        assert np.abs(A - D).max() > 1e-3 * np.abs(D).max()


def test_reciprocity_with_fixup():
    p, src, W = _thick(84)
    r = oracle.adjoint(p, src, W, tol=1e-15)
    assert abs(r["J"] - r["recip"]) < 1e-12 * abs(r["J"])


def test_gradient_with_fixup_matches_central_differences():
    """The fixup is continuous (a fixed axis switches at zero outflow), so J
    is piecewise smooth in the density; central differences with a small
    step agree with the frozen-branch gradient away from switching points."""
    p, src, W = _thick(84)
    assert oracle.solve(p, src, tol=1e-15)["nneg"] > 100
    r = oracle.adjoint(p, src, W, tol=1e-15)
    g = r["grad"]
    h = 1e-6
    fd = np.zeros(p.V)
    for v in range(p.V):
        d = p.density.copy()
        d[v] += h
        jp = (W * oracle.solve(p.with_density(d), src, tol=1e-15)["phi_total"]).sum()
        d[v] -= 2 * h
        jm = (W * oracle.solve(p.with_density(d), src, tol=1e-15)["phi_total"]).sum()
        fd[v] = (jp - jm) / (2 * h)
    big = np.abs(fd) > 1e-3 * np.abs(fd).max()
    assert big.sum() > p.V // 2
    assert (np.abs(g - fd)[big] / np.abs(fd[big])).max() < 1e-5
