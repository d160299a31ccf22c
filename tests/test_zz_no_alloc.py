"""dsn_solve_noalloc: the one-source forward solve that allocates no device
memory (its working set lives in one fixed 64 MiB device array per GPU).

Host checks (no GPU): a problem too large for the array and combined
sources are rejected before any device call.  GPU checks: two calls in a
row through the C ABI, the second on a smaller problem, each equal to
dsn_solve's result bit for bit (same kernels, same launch shape) and to the
oracle within the parity bar; converged in the FP32 rule too; the device's
free memory and the handle's device state do not change."""
import ctypes as C

import numpy as np
import pytest

import oracle
from parity import parity_err
from synthetic.workloads import SourceSpec, config1, random_small_problem

dsn = pytest.importorskip("paper_1910_11335_amd")


def _cone(p, G):
    ext = np.array([p.nx * p.dx, p.ny * p.dy, p.nz * p.dz])
    return SourceSpec(position=(ext[0] + 7.0, 0.5 * ext[1], 0.5 * ext[2]), axis=(-1.0, 0.05, 0.0),
                      half_angle=np.deg2rad(25.0), spectrum=np.linspace(1.0, 0.3, G))


def test_noalloc_rejects_what_does_not_fit_before_device_work():
    # 64^3 S8 P3 G19: far above the fixed array
    p = random_small_problem(3, n=(64, 64, 64), d=(0.5, 0.5, 0.5), sn=8, L=3, G=19, n_mat=2, fixup=1)
    h = dsn.Problem(p, "fp32")
    lib = dsn.lib()
    st, keep = dsn.dsn._source_struct(_cone(p, 19), 19)
    o, _ = dsn.dsn._opts(19, 1e-5, 100, None, False, None)
    info = dsn.dsn.SolveInfo()
    assert lib.dsn_solve_noalloc(h.handle, C.byref(st), C.byref(o), C.c_void_p(8), None,
                                 C.byref(info)) == dsn.dsn.DSN_ERR_UNSUPPORTED
    assert "maximum" in dsn.last_error()
    h.close()
    q, s = config1()
    h = dsn.Problem(q, "fp64")
    st, keep = dsn.dsn._source_struct(s, 2)
    o, _ = dsn.dsn._opts(2, 1e-8, 100, None, False, None, combine=True)
    info = dsn.dsn.SolveInfo()
    assert lib.dsn_solve_noalloc(h.handle, C.byref(st), C.byref(o), C.c_void_p(8), None,
                                 C.byref(info)) == dsn.dsn.DSN_ERR_INVALID_ARG
    o, _ = dsn.dsn._opts(2, 1e-8, 100, None, False, None)
    assert lib.dsn_solve_noalloc(h.handle, C.byref(st), C.byref(o), None, None,
                                 C.byref(info)) == dsn.dsn.DSN_ERR_INVALID_ARG
    h.close()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_equals_solve_twice_second_smaller(precision):
    torch = pytest.importorskip("torch")
    big = random_small_problem(31, n=(21, 18, 24), sn=6, L=2, G=3, n_mat=3, fixup=1)
    small = random_small_problem(32, n=(9, 7, 11), sn=4, L=1, G=2, n_mat=2, fixup=0)
    tol = 1e-12 if precision == "fp64" else 1e-4
    # a first call loads the library's code objects (and with them the fixed
    # array) if nothing has yet
    q, s0 = config1()
    hq = dsn.Problem(q, precision)
    hq.solve_noalloc(s0, fixed_iters=[1, 1])
    hq.close()
    handles = []
    free = []
    for p in (big, small):
        s = _cone(p, p.G)
        fixed = [3] * p.G
        h = dsn.Problem(p, precision)
        handles.append(h)
        ref = h.solve([s], fixed_iters=fixed)["phi_total"][0]  # dsn_solve on this handle
        hn = dsn.Problem(p, precision)  # a fresh handle: the no-alloc call gives it no device state
        before = hn.workspace_bytes()
        out = torch.empty((p.G, p.V), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        free.append(torch.cuda.mem_get_info()[0])
        got = hn.solve_noalloc(s, fixed_iters=fixed, out=out)
        torch.cuda.synchronize()
        free.append(torch.cuda.mem_get_info()[0])
        assert hn.workspace_bytes() == before
        assert list(got["iters"]) == fixed
        assert torch.equal(got["phi_total"], ref), p.name
        want = oracle.solve(p, s, fixed_iters=fixed)["phi_total"]
        assert parity_err(got["phi_total"].cpu().numpy(), want, p, 1e-13 if precision == "fp64" else 1e-5) < tol
        # converged in the precision's rule: same iteration counts and result as dsn_solve
        rule = dsn.CONVERGED[precision]
        a = h.solve([s], **rule)
        b = hn.solve_noalloc(s, out=out, **rule)
        assert list(b["iters"]) == list(a["iters"][0])
        assert torch.equal(b["phi_total"], a["phi_total"][0])
        hn.close()
    # no device memory taken by the no-alloc calls
    assert free[0] == free[1] and free[2] == free[3]
    for h in handles:
        h.close()


@pytest.mark.gpu
def test_noalloc_on_a_column_relay_handle():
    """On a handle pinned to a column-relay sweep shape the no-allocation
    solve runs that shape (LDS handover included) and equals the handle's
    own dsn_solve bit for bit."""
    torch = pytest.importorskip("torch")
    p = random_small_problem(33, n=(17, 20, 12), sn=8, L=2, G=2, n_mat=3, fixup=1)
    s = _cone(p, p.G)
    h = dsn.Problem(p, "fp32")
    h.set_sweep_shape(1, 40, 0, 4)
    ref = h.solve([s], fixed_iters=[3, 2])["phi_total"][0]
    got = h.solve_noalloc(s, fixed_iters=[3, 2])
    assert got["sweep_shape"][3] == 4
    assert torch.equal(got["phi_total"], ref)
    h.close()
