"""CPU FP64 oracle for the discrete-ordinates hot path (TEST INFRASTRUCTURE).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this package.  The product library never calls it, and it never calls
the product library.  The C part (oracle.c) is built by oracle/build.py into
oracle/liboracle.so.

Every entry point takes a synthetic.workloads.ProblemSpec / SourceSpec.
"""
import ctypes as C
import os

import numpy as np

from .quadrature import lqn

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_MEM, ERR_NOT_CONVERGED = 0, 1, 3, 5

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("material", C.POINTER(C.c_uint8)), ("density", _dp),
                ("n_mat", C.c_int), ("G", C.c_int), ("sigma_t", _dp),
                ("L", C.c_int), ("sigma_s", _dp),
                ("n_dir", C.c_int), ("omega", _dp), ("w", _dp), ("fixup", C.c_int)]


class _Source(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("axis", C.c_double * 3), ("half_angle", C.c_double),
                ("spectrum", _dp), ("q_vol", _dp), ("fan_normal", C.c_double * 3), ("fan_half_thickness", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iters", C.c_int), ("fixed_iters", _ip),
                ("sweep_order", C.c_int), ("verbose", C.c_int), ("stop_rule", C.c_int), ("cell_single", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build
            build()
        l = C.CDLL(LIB_PATH)
        l.orc_harmonics.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _dp]
        l.orc_plane_count.restype = C.c_long
        l.orc_plane_count.argtypes = [C.c_int] * 4
        l.orc_plane_enumerate.restype = C.c_long
        l.orc_plane_enumerate.argtypes = [C.c_int] * 4 + [_ip]
        l.orc_sweep.argtypes = [C.POINTER(_Problem), _dp, _dp, _dp, _dp, _dp, C.c_int, C.POINTER(C.c_long)]
        l.orc_sweep_mode.argtypes = [C.POINTER(_Problem), _dp, _dp, _dp, _dp, _dp, C.c_int, C.POINTER(C.c_uint8)]
        l.orc_raytrace.argtypes = [C.POINTER(_Problem), C.POINTER(_Source), _dp, _dp]
        l.orc_ray_material_path.argtypes = [C.POINTER(_Problem), _dp, _dp, _dp]
        l.orc_moment_matrices.argtypes = [C.POINTER(_Problem), _dp, _dp]
        l.orc_solve.argtypes = [C.POINTER(_Problem), C.POINTER(_Source), C.POINTER(_Opts), _dp, _dp, _dp,
                                _ip, _dp, C.POINTER(C.c_long)]
        l.orc_adjoint.argtypes = [C.POINTER(_Problem), C.POINTER(_Source), C.POINTER(_Opts), _dp, _dp, _dp,
                                  _dp, _ip, _ip]
        l.orc_num_threads.restype = C.c_int
        l.orc_set_num_threads.argtypes = [C.c_int]
        l.orc_set_num_threads.restype = None
        _lib = l
    return _lib


def _p(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


class _Keep:
    """Holds the numpy arrays a ctypes struct points into."""

    def __init__(self, prob, quad=None):
        om, w = quad if quad is not None else lqn(prob.sn_order)
        self.mat = np.ascontiguousarray(prob.material, dtype=np.uint8)
        self.dens = None if prob.density is None else np.ascontiguousarray(prob.density, dtype=np.float64)
        self.st = np.ascontiguousarray(prob.sigma_t, dtype=np.float64)
        self.ss = np.ascontiguousarray(prob.sigma_s, dtype=np.float64)
        self.om = np.ascontiguousarray(om, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        assert self.st.shape[0] == self.ss.shape[0] and self.ss.shape[1] == prob.legendre_order + 1
        self.s = _Problem(prob.nx, prob.ny, prob.nz, prob.dx, prob.dy, prob.dz,
                          _p(self.mat, C.POINTER(C.c_uint8)), _p(self.dens),
                          self.st.shape[0], self.st.shape[1], _p(self.st),
                          prob.legendre_order, _p(self.ss), len(self.w), _p(self.om), _p(self.w),
                          int(prob.fixup))


def _source(src, G, V):
    spec = np.ascontiguousarray(np.asarray(src.spectrum, dtype=np.float64).reshape(-1))
    if spec.size != G:
        raise ValueError("spectrum must have G entries")
    qv = None if src.q_vol is None else np.ascontiguousarray(src.q_vol, dtype=np.float64).reshape(G, V)
    s = _Source((C.c_double * 3)(*src.position), (C.c_double * 3)(*src.axis), float(src.half_angle),
                _p(spec), _p(qv), (C.c_double * 3)(*getattr(src, "fan_normal", (0.0, 0.0, 1.0))),
                float(getattr(src, "fan_half_thickness", 0.0)))
    return s, (spec, qv)


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    """Threads of later oracle calls (results do not depend on it)."""
    lib().orc_set_num_threads(int(n))


def harmonics(L, omega):
    """R_lm(omega) for every direction: [n][(L+1)^2]."""
    omega = np.atleast_2d(np.asarray(omega, dtype=np.float64))
    out = np.zeros((len(omega), (L + 1) ** 2))
    for n, (a, b, c) in enumerate(omega):
        buf = np.zeros((L + 1) ** 2)
        lib().orc_harmonics(L, a, b, c, _p(buf))
        out[n] = buf
    return out


def plane_count(S, nx, ny, nz):
    return lib().orc_plane_count(S, nx, ny, nz)


def plane_enumerate(S, nx, ny, nz):
    n = lib().orc_plane_enumerate(S, nx, ny, nz, None)
    buf = np.zeros(3 * max(n, 1), dtype=np.int32)
    lib().orc_plane_enumerate(S, nx, ny, nz, _p(buf, _ip))
    return buf[: 3 * n].reshape(n, 3)


def moment_matrices(prob, quad=None):
    k = _Keep(prob, quad)
    Nm, Nd = (prob.legendre_order + 1) ** 2, len(k.w)
    M = np.zeros((Nd, Nm))
    D = np.zeros((Nm, Nd))
    lib().orc_moment_matrices(C.byref(k.s), _p(M), _p(D))
    return M, D


def sweep(prob, omega, sig, Q, order=0):
    """One DD sweep along omega.  Returns psi [V], outflows [3][V], #negative."""
    k = _Keep(prob)
    V = prob.V
    om = np.ascontiguousarray(omega, dtype=np.float64)
    sig = np.ascontiguousarray(sig, dtype=np.float64)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    psi = np.zeros(V)
    o = np.zeros(3 * V)
    nneg = C.c_long(0)
    lib().orc_sweep(C.byref(k.s), _p(om), _p(sig), _p(Q), _p(psi), _p(o), int(order), C.byref(nneg))
    return psi, o.reshape(3, V), nneg.value


CELL_DD, CELL_FIXUP, CELL_FROZEN, CELL_TRANS, CELL_DD_SINGLE = 0, 1, 2, 3, 4


def sweep_mode(prob, omega, sig, Q, mode, mask=None):
    """One sweep along omega with an explicit cell mode (CELL_*): CELL_FIXUP
    records each cell's set of fixed axes (bit a = axis a) into the returned
    mask; CELL_FROZEN applies the fixup cell with the given sets frozen (a
    linear map); CELL_TRANS the transposed frozen cell (for a sweep along
    -omega); CELL_DD_SINGLE the pure DD cell in single precision.  Returns
    psi [V], outflows [3][V], mask [V] (uint8)."""
    k = _Keep(prob)
    V = prob.V
    om = np.ascontiguousarray(omega, dtype=np.float64)
    sig = np.ascontiguousarray(sig, dtype=np.float64)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    psi = np.zeros(V)
    o = np.zeros(3 * V)
    m = np.zeros(V, dtype=np.uint8) if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).copy()
    st = lib().orc_sweep_mode(C.byref(k.s), _p(om), _p(sig), _p(Q), _p(psi), _p(o), int(mode),
                              m.ctypes.data_as(C.POINTER(C.c_uint8)))
    if st != OK:
        raise ValueError("oracle sweep failed with status %d" % st)
    return psi, o.reshape(3, V), m


def ray_material_path(prob, xs, xe):
    k = _Keep(prob)
    lam = np.zeros(prob.n_mat)
    lib().orc_ray_material_path(C.byref(k.s), _p(np.asarray(xs, dtype=np.float64)),
                                _p(np.asarray(xe, dtype=np.float64)), _p(lam))
    return lam


def raytrace(prob, src):
    k = _Keep(prob)
    s, hold = _source(src, prob.G, prob.V)
    phiu = np.zeros((prob.G, prob.V))
    oms = np.zeros((prob.V, 3))
    st = lib().orc_raytrace(C.byref(k.s), C.byref(s), _p(phiu), _p(oms))
    if st:
        raise ValueError("oracle raytrace failed with status %d" % st)
    return phiu, oms


def _opts(tol, max_iters, fixed_iters, G, order, verbose=False, stop_rule=0, cell_single=False):
    fi = None if fixed_iters is None else np.ascontiguousarray(np.broadcast_to(fixed_iters, (G,)), dtype=np.int32)
    return _Opts(float(tol), int(max_iters), _p(fi, _ip), int(order), int(verbose), int(stop_rule),
                 int(bool(cell_single))), fi


def solve(prob, src, tol=1e-10, max_iters=10000, fixed_iters=None, sweep_order=0, moments=False, quad=None,
          verbose=False, stop_rule=0, cell_single=False):
    """Forward solve of one source.  Returns a dict with phi_total [G][V],
    phi_u [G][V], phi_c [G][Nm][V] (if moments), iters [G], resid [G],
    nneg (count of negative DD outflows met), status.  verbose: a line on
    stderr as each group ends.  cell_single (pure DD only): every DD cell in
    single precision, a model of single-precision rounding (moments stay
    double)."""
    k = _Keep(prob, quad)
    G, V, Nm = prob.G, prob.V, (prob.legendre_order + 1) ** 2
    s, hold = _source(src, G, V)
    o, fi = _opts(tol, max_iters, fixed_iters, G, sweep_order, verbose, stop_rule, cell_single)
    phit = np.zeros((G, V))
    phiu = np.zeros((G, V))
    phic = np.zeros((G, Nm, V)) if moments else None
    iters = np.zeros(G, dtype=np.int32)
    resid = np.zeros(G)
    nneg = C.c_long(0)
    st = lib().orc_solve(C.byref(k.s), C.byref(s), C.byref(o), _p(phit), _p(phiu), _p(phic),
                         _p(iters, _ip), _p(resid), C.byref(nneg))
    if st not in (OK, ERR_NOT_CONVERGED):
        raise ValueError("oracle solve failed with status %d" % st)
    return dict(phi_total=phit, phi_u=phiu, phi_c=phic, iters=iters, resid=resid, nneg=nneg.value,
                status=st)


def adjoint(prob, src, W, tol=1e-12, max_iters=10000, fixed_iters=None):
    """Gradient of J = sum W * phi_total with respect to per-voxel density
    (with the fixup on: of the solve linearised with every cell's fixed-axis
    set frozen at the converged solution).
    Returns dict(J, recip, grad [V], iters_fwd [G], iters_adj [G], status)."""
    k = _Keep(prob)
    G, V = prob.G, prob.V
    s, hold = _source(src, G, V)
    o, fi = _opts(tol, max_iters, fixed_iters, G, 0)
    W = np.ascontiguousarray(W, dtype=np.float64).reshape(G, V)
    J, rc = C.c_double(0), C.c_double(0)
    grad = np.zeros(V)
    itf = np.zeros(G, dtype=np.int32)
    ita = np.zeros(G, dtype=np.int32)
    st = lib().orc_adjoint(C.byref(k.s), C.byref(s), C.byref(o), _p(W), C.byref(J), C.byref(rc),
                           _p(grad), _p(itf, _ip), _p(ita, _ip))
    if st not in (OK, ERR_NOT_CONVERGED):
        raise ValueError("oracle adjoint failed with status %d" % st)
    return dict(J=J.value, recip=rc.value, grad=grad, iters_fwd=itf, iters_adj=ita, status=st)


def dose(prob, phi, k):
    """Absorbed dose from group fluences: for every fluence set s and voxel v,
    dose[s][v] = sum over groups g of phi[s][g][v] times k[m(v)][g], k being
    the fluence-to-dose factor of the voxel's material m(v) in group g (the
    use of the fluence named in the paper's sections I and IV).  phi [n][G][V]
    or [G][V]; returns [n][V] or [V].  Written as the plain double loop."""
    ph = np.asarray(phi, dtype=np.float64)
    single = ph.ndim == 2
    if single:
        ph = ph[None]
    n, G, V = ph.shape
    mat = np.asarray(prob.material, dtype=np.int64).reshape(-1)
    k = np.asarray(k, dtype=np.float64)
    out = np.zeros((n, V))
    for g in range(G):
        out += ph[:, g, :] * k[mat, g][None, :]
    return out[0] if single else out
