"""Host-side checks of the C-ABI library (no GPU, no compute calls): it
loads, exports every function include/dsn.h declares, derives the same
quadrature as the oracle, and rejects invalid input before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from oracle.quadrature import lqn, SUPPORTED_ORDERS
from synthetic.workloads import SourceSpec, config1, random_small_problem

dsn = pytest.importorskip("paper_1910_11335_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "dsn.h")).read()
    declared = set(re.findall(r"\b(dsn_[a-z_]+)\s*\(", hdr))
    assert declared == set(dsn.dsn.EXPORTS)
    l = C.CDLL(dsn.LIB_PATH)
    for name in declared:
        assert hasattr(l, name), name


@pytest.mark.parametrize("N", SUPPORTED_ORDERS)
def test_library_quadrature_matches_oracle(N):
    om, w = dsn.quadrature(N)
    om2, w2 = lqn(N)
    assert np.abs(om - om2).max() < 2e-15
    assert np.abs(w - w2).max() < 2e-15


def test_unsupported_order_rejected():
    with pytest.raises(dsn.DsnError) as e:
        dsn.quadrature(14)
    assert e.value.status == dsn.dsn.DSN_ERR_INVALID_ARG


def _bad(fn):
    with pytest.raises(dsn.DsnError) as e:
        fn()
    return e.value.status


def test_create_validation():
    p = random_small_problem(1, n=(4, 5, 6), sn=4, L=1, G=3)
    dsn.Problem(p).close()
    q = random_small_problem(1, n=(4, 5, 6), sn=4, L=1, G=3)
    q.material = q.material.copy()
    q.material[3] = 7
    assert _bad(lambda: dsn.Problem(q)) == dsn.dsn.DSN_ERR_INVALID_ARG
    q = random_small_problem(1, n=(4, 5, 6), sn=4, L=1, G=3)
    q.sigma_s = q.sigma_s.copy()
    q.sigma_s[0, 0, 0, 2] = 0.1   # upscatter from group 2 into group 0
    assert _bad(lambda: dsn.Problem(q)) == dsn.dsn.DSN_ERR_INVALID_ARG
    q = random_small_problem(1, n=(4, 5, 6), sn=4, L=1, G=3)
    q.sn_order = 5
    assert _bad(lambda: dsn.Problem(q)) == dsn.dsn.DSN_ERR_INVALID_ARG
    q = random_small_problem(1, n=(4, 5, 6), sn=2, L=2, G=3)   # L > N - 1
    assert _bad(lambda: dsn.Problem(q)) == dsn.dsn.DSN_ERR_INVALID_ARG
    q = random_small_problem(1, n=(4, 5, 6), sn=4, L=1, G=3)
    q.sigma_t = q.sigma_t.copy()
    q.sigma_t[1, 1] = np.nan
    assert _bad(lambda: dsn.Problem(q)) == dsn.dsn.DSN_ERR_INVALID_ARG
    q = random_small_problem(1, n=(4, 5, 6), sn=4, L=1, G=3)
    q.density = q.density.copy()
    q.density[0] = -1
    assert _bad(lambda: dsn.Problem(q)) == dsn.dsn.DSN_ERR_INVALID_ARG
    assert "density" in dsn.last_error()


def test_solve_argument_checks_run_before_device():
    p, s = config1()
    h = dsn.Problem(p)
    # source exactly on a voxel centre
    bad = SourceSpec(position=(0.5, 0.5, 0.5), spectrum=np.array([1.0, 0.0]))
    lib = dsn.lib()
    st, keep = dsn.dsn._source_struct(bad, 2)
    o, _ = dsn.dsn._opts(2, 1e-8, 100, None, False, None)
    info = dsn.dsn.SolveInfo()
    r = lib.dsn_solve(h.handle, C.byref(st), 1, C.byref(o), C.c_void_p(8), None, C.byref(info))
    assert r == dsn.dsn.DSN_ERR_INVALID_ARG and "voxel centre" in dsn.last_error()
    # negative tolerance
    st, keep = dsn.dsn._source_struct(s, 2)
    o, _ = dsn.dsn._opts(2, -1.0, 100, None, False, None)
    r = lib.dsn_solve(h.handle, C.byref(st), 1, C.byref(o), C.c_void_p(8), None, C.byref(info))
    assert r == dsn.dsn.DSN_ERR_INVALID_ARG
    # negative wait limit
    o, _ = dsn.dsn._opts(2, 1e-8, 100, None, False, None, wait_limit=-1)
    r = lib.dsn_solve(h.handle, C.byref(st), 1, C.byref(o), C.c_void_p(8), None, C.byref(info))
    assert r == dsn.dsn.DSN_ERR_INVALID_ARG and "wait_limit" in dsn.last_error()
    # NULL output
    o, _ = dsn.dsn._opts(2, 1e-8, 100, None, False, None)
    r = lib.dsn_solve(h.handle, C.byref(st), 1, C.byref(o), None, None, C.byref(info))
    assert r == dsn.dsn.DSN_ERR_INVALID_ARG
    # an empty source list is a valid no-op (no device call, nothing written)
    r = lib.dsn_solve(h.handle, None, 0, C.byref(o), None, None, C.byref(info))
    assert r == dsn.dsn.DSN_OK and info.updates == 0
    r = lib.dsn_solve(h.handle, None, -1, C.byref(o), None, None, C.byref(info))
    assert r == dsn.dsn.DSN_ERR_INVALID_ARG
    oc, _ = dsn.dsn._opts(2, 1e-8, 100, None, False, None, combine=True)
    r = lib.dsn_solve(h.handle, None, 0, C.byref(oc), C.c_void_p(8), None, C.byref(info))
    assert r == dsn.dsn.DSN_ERR_INVALID_ARG and "combine" in dsn.last_error()
    assert h.workspace_bytes() > 0
    h.close()


def test_no_gpu_means_loud_failure():
    torch = pytest.importorskip("torch")
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    p, s = config1()
    h = dsn.Problem(p)
    lib = dsn.lib()
    st, keep = dsn.dsn._source_struct(s, 2)
    o, _ = dsn.dsn._opts(2, 1e-8, 100, None, False, None)
    info = dsn.dsn.SolveInfo()
    r = lib.dsn_solve(h.handle, C.byref(st), 1, C.byref(o), C.c_void_p(8), None, C.byref(info))
    assert r == dsn.dsn.DSN_ERR_DEVICE
    h.close()


def test_batch_rejects_a_problem_listed_twice():
    p, s = config1()
    h = dsn.Problem(p)
    lib = dsn.lib()
    st, keep = dsn.dsn._source_struct(s, 2)
    arr = (dsn.dsn.Source * 1)(st)
    parr = (C.POINTER(dsn.dsn.Source) * 2)(C.cast(arr, C.POINTER(dsn.dsn.Source)),
                                           C.cast(arr, C.POINTER(dsn.dsn.Source)))
    handles = (C.c_void_p * 2)(h.handle.value, h.handle.value)
    nsrc = (C.c_int32 * 2)(1, 1)
    outs = (C.c_void_p * 2)(8, 8)
    o, _ = dsn.dsn._opts(2, 1e-8, 100, None, False, None)
    info = dsn.dsn.SolveInfo()
    r = lib.dsn_solve_batch(handles, 2, parr, nsrc, C.byref(o), outs, C.byref(info))
    assert r == dsn.dsn.DSN_ERR_INVALID_ARG and "twice" in dsn.last_error()
    h.close()


def test_dose_argument_checks_run_before_device():
    p, s = config1()
    h = dsn.Problem(p)
    lib = dsn.lib()
    k = np.ones((h.nmat, h.G))
    r = lib.dsn_dose(h.handle, C.c_void_p(8), 1, k.ctypes.data_as(C.POINTER(C.c_double)), None, None)
    assert r == dsn.dsn.DSN_ERR_INVALID_ARG
    k[0, 1] = np.inf
    r = lib.dsn_dose(h.handle, C.c_void_p(8), 1, k.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(8), None)
    assert r == dsn.dsn.DSN_ERR_INVALID_ARG and "finite" in dsn.last_error()
    r = lib.dsn_dose(h.handle, C.c_void_p(8), -1, k.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(8), None)
    assert r == dsn.dsn.DSN_ERR_INVALID_ARG
    h.close()


def test_fan_source_checks_run_before_device():
    p, s = config1()
    h = dsn.Problem(p)
    lib = dsn.lib()
    o, _ = dsn.dsn._opts(2, 1e-8, 100, None, False, None)
    info = dsn.dsn.SolveInfo()
    fan = SourceSpec(position=(-3.0, 8.2, 8.1), axis=(1.0, 0.0, 0.0), half_angle=0.4,
                     spectrum=np.array([1.0, 0.0]), fan_normal=(2.0, 0.0, 0.0), fan_half_thickness=0.1)
    st, keep = dsn.dsn._source_struct(fan, 2)
    r = lib.dsn_solve(h.handle, C.byref(st), 1, C.byref(o), C.c_void_p(8), None, C.byref(info))
    assert r == dsn.dsn.DSN_ERR_INVALID_ARG and "parallel" in dsn.last_error()
    wide = SourceSpec(**{**fan.__dict__, "fan_normal": (0.0, 0.0, 1.0), "half_angle": 1.7})
    st, keep = dsn.dsn._source_struct(wide, 2)
    r = lib.dsn_solve(h.handle, C.byref(st), 1, C.byref(o), C.c_void_p(8), None, C.byref(info))
    assert r == dsn.dsn.DSN_ERR_INVALID_ARG and "pi/2" in dsn.last_error()
    h.close()


def test_c_client_compiles_links_and_runs(tmp_path):
    """The header compiles as C11 with warnings as errors, a C program links
    against the library and its host-side calls behave from C."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lib = dsn.dsn.LIB_PATH
    exe = str(tmp_path / "c_abi_check")
    subprocess.check_call([gcc, "-std=c11", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(root, "include"),
                           os.path.join(root, "tests", "c_abi_check.c"), "-o", exe, lib, "-lm",
                           "-Wl,-rpath," + os.path.dirname(lib)])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout + out.stderr


def test_sweep_shape_checks_run_before_device():
    """dsn_set_sweep_shape rejects shapes no sweep kernel is built for (S4:
    3 directions per octant, so 2 waves per block do not divide them; no
    column relay of 3 roles, none of 3 directions, none on per-XCD queues),
    block counts out of range and negative counts, with no device call."""
    p, s = config1()
    h = dsn.Problem(p)
    lib = dsn.lib()
    for w, b, x, r in [(2, 64, 0, 0), (7, 64, 0, 0), (0, 64, 0, 0), (1, 0, 0, 0), (1, (1 << 20) + 1, 0, 0),
                       (3, 64, -1, 0), (1, 64, 0, -1), (1, 64, 0, 3), (3, 64, 0, 2), (1, 64, 8, 2)]:
        assert lib.dsn_set_sweep_shape(h.handle, w, b, x, r) == dsn.dsn.DSN_ERR_INVALID_ARG, (w, b, x, r)
    assert lib.dsn_set_sweep_shape(None, 1, 64, 0, 0) == dsn.dsn.DSN_ERR_INVALID_ARG
    with pytest.raises(dsn.DsnError):
        h.set_sweep_shape(3, 64)  # a valid shape: needs the device, which this host lacks
    h.close()
