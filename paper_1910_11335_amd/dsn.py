"""ctypes binding of libdsn.so (include/dsn.h).  Argument marshalling only:
every step of the solve runs in the library's HIP kernels.  Torch supplies
the device output buffers and the stream.

There is no CPU fallback: if the library is missing or no gfx950 GPU is
usable, calls raise DsnError.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsn.so")

DSN_OK, DSN_ERR_INVALID_ARG, DSN_ERR_UNSUPPORTED, DSN_ERR_OUT_OF_MEMORY = 0, 1, 2, 3
DSN_ERR_DEVICE, DSN_ERR_NOT_CONVERGED, DSN_ERR_NUMERICAL = 4, 5, 6
DSN_FP64, DSN_FP32 = 0, 1

STATUS_NAMES = {0: "DSN_OK", 1: "DSN_ERR_INVALID_ARG", 2: "DSN_ERR_UNSUPPORTED", 3: "DSN_ERR_OUT_OF_MEMORY",
                4: "DSN_ERR_DEVICE", 5: "DSN_ERR_NOT_CONVERGED", 6: "DSN_ERR_NUMERICAL"}

# Converged-solve settings of the two precisions.  FP64: every group's
# relative L2 change of its scalar fluence below 1e-10 (stop rule 0).  FP32:
# the estimated per-voxel error left below 1e-5 (stop rule 1), or the FP32
# rounding floor (three non-decreasing changes) if that comes first, so the
# iteration error stays well inside a 1e-4 per-voxel budget beside the FP32
# rounding.
CONVERGED = {"fp64": {"tol": 1e-10, "stop_rule": 0, "stagnation_stop": False},
             "fp32": {"tol": 1e-5, "stop_rule": 1, "stagnation_stop": True}}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class DsnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class ProblemDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("material", C.POINTER(C.c_uint8)), ("density", _dp),
                ("n_materials", C.c_int32), ("n_groups", C.c_int32), ("sigma_t", _dp),
                ("legendre_order", C.c_int32), ("sigma_s", _dp), ("sn_order", C.c_int32),
                ("fixup", C.c_int32), ("precision", C.c_int32)]


class Source(C.Structure):
    _fields_ = [("position", C.c_double * 3), ("axis", C.c_double * 3), ("half_angle", C.c_double),
                ("spectrum", _dp), ("fan_normal", C.c_double * 3), ("fan_half_thickness", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iters", C.c_int32), ("fixed_iters", _ip),
                ("stagnation_stop", C.c_int32), ("profile", C.c_int32), ("wait_limit", C.c_int32),
                ("autotune", C.c_int32), ("combine_sources", C.c_int32), ("stream", C.c_void_p),
                ("stop_rule", C.c_int32), ("batch_mode", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", _ip), ("residual", _dp), ("updates", C.c_double), ("seconds", C.c_double),
                ("stage_ms", C.c_double * 4), ("stage_launches", C.c_int64 * 4), ("sweep_bytes", C.c_double),
                ("sweep_waves_per_block", C.c_int32), ("sweep_blocks", C.c_int32), ("sweep_xcd_queues", C.c_int32),
                ("sweep_relay", C.c_int32)]

    def stages(self):
        names = ("setup", "m2d", "sweep", "d2m")
        return {n: dict(ms=self.stage_ms[i], launches=int(self.stage_launches[i])) for i, n in enumerate(names)}


EXPORTS = ["dsn_create", "dsn_destroy", "dsn_workspace_bytes", "dsn_solve", "dsn_solve_adjoint",
           "dsn_set_density", "dsn_solve_batch", "dsn_dose", "dsn_quadrature", "dsn_sweep_tuning", "dsn_set_sweep_shape",
           "dsn_last_error", "dsn_solve_noalloc", "dsn_xcd_queues"]

_lib = None


def lib():
    """The loaded library (raises DsnError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DsnError(DSN_ERR_DEVICE, "libdsn.so is not built (run __graft_entry__.build())")
        l = C.CDLL(LIB_PATH)
        l.dsn_create.argtypes = [C.POINTER(ProblemDesc), C.POINTER(C.c_void_p)]
        l.dsn_create.restype = C.c_int
        l.dsn_destroy.argtypes = [C.c_void_p]
        l.dsn_destroy.restype = None
        l.dsn_workspace_bytes.argtypes = [C.c_void_p]
        l.dsn_workspace_bytes.restype = C.c_size_t
        l.dsn_solve.argtypes = [C.c_void_p, C.POINTER(Source), C.c_int32, C.POINTER(SolveOpts), C.c_void_p,
                                C.c_void_p, C.POINTER(SolveInfo)]
        l.dsn_solve.restype = C.c_int
        l.dsn_solve_adjoint.argtypes = [C.c_void_p, C.POINTER(Source), C.c_void_p, C.POINTER(SolveOpts),
                                        _dp, C.c_void_p, C.c_void_p, C.POINTER(SolveInfo)]
        l.dsn_solve_adjoint.restype = C.c_int
        l.dsn_solve_noalloc.argtypes = [C.c_void_p, C.POINTER(Source), C.POINTER(SolveOpts), C.c_void_p,
                                        C.c_void_p, C.POINTER(SolveInfo)]
        l.dsn_solve_noalloc.restype = C.c_int
        l.dsn_set_density.argtypes = [C.c_void_p, C.c_void_p]
        l.dsn_set_density.restype = C.c_int
        l.dsn_solve_batch.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.POINTER(Source)), _ip,
                                      C.POINTER(SolveOpts), C.POINTER(C.c_void_p), C.POINTER(SolveInfo)]
        l.dsn_solve_batch.restype = C.c_int
        l.dsn_quadrature.argtypes = [C.c_int32, _dp, _dp]
        l.dsn_quadrature.restype = C.c_int
        l.dsn_dose.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, _dp, C.c_void_p, C.c_void_p]
        l.dsn_dose.restype = C.c_int
        l.dsn_sweep_tuning.argtypes = [C.c_void_p, _ip, _ip, _ip, _ip, C.POINTER(C.c_float), C.c_int32]
        l.dsn_sweep_tuning.restype = C.c_int32
        l.dsn_set_sweep_shape.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        l.dsn_set_sweep_shape.restype = C.c_int
        l.dsn_xcd_queues.argtypes = [C.c_void_p]
        l.dsn_xcd_queues.restype = C.c_int32
        l.dsn_last_error.argtypes = []
        l.dsn_last_error.restype = C.c_char_p
        _lib = l
    return _lib


def last_error():
    return lib().dsn_last_error().decode()


def _check(st):
    if st not in (DSN_OK, DSN_ERR_NOT_CONVERGED):
        raise DsnError(st, last_error())
    return st


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def quadrature(sn_order):
    """The library's own level-symmetric set: (omega [N(N+2), 3], w [N(N+2)])."""
    n = sn_order * (sn_order + 2)
    om = np.zeros((max(n, 1), 3))
    w = np.zeros(max(n, 1))
    _check(lib().dsn_quadrature(int(sn_order), _ptr(om), _ptr(w)))
    return om[:n], w[:n]


def _source_struct(src, G):
    spec = np.ascontiguousarray(np.asarray(src.spectrum, dtype=np.float64).reshape(-1))
    if spec.size != G:
        raise ValueError("spectrum must have %d entries" % G)
    fan_n = getattr(src, "fan_normal", (0.0, 0.0, 1.0))
    s = Source((C.c_double * 3)(*[float(x) for x in src.position]),
               (C.c_double * 3)(*[float(x) for x in src.axis]), float(src.half_angle), _ptr(spec),
               (C.c_double * 3)(*[float(x) for x in fan_n]), float(getattr(src, "fan_half_thickness", 0.0)))
    return s, spec


def _opts(G, tol, max_iters, fixed_iters, stagnation_stop, stream, profile=False, wait_limit=0, autotune=False,
          combine=False, stop_rule=0, batch_mode=0):
    fi = None
    if fixed_iters is not None:
        fi = np.ascontiguousarray(np.broadcast_to(np.asarray(fixed_iters), (G,)), dtype=np.int32)
    o = SolveOpts(float(tol), int(max_iters), _ptr(fi, _ip), int(bool(stagnation_stop)), int(bool(profile)),
                  int(wait_limit), int(bool(autotune)), int(bool(combine)),
                  C.c_void_p(stream if stream is not None else 0), int(stop_rule), int(batch_mode))
    return o, fi


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Problem:
    """A problem handle.  `spec` is any object with the fields of the C
    problem description (nx, ny, nz, dx, dy, dz, material, density, sigma_t
    [M][G], sigma_s [M][L+1][G][G], sn_order, legendre_order, fixup)."""

    def __init__(self, spec, precision="fp64"):
        self.precision = DSN_FP32 if precision in ("fp32", DSN_FP32) else DSN_FP64
        self._mat = np.ascontiguousarray(spec.material, dtype=np.uint8).reshape(-1)
        self._dens = None if spec.density is None else np.ascontiguousarray(spec.density, dtype=np.float64)
        self._st = np.ascontiguousarray(spec.sigma_t, dtype=np.float64)
        self._ss = np.ascontiguousarray(spec.sigma_s, dtype=np.float64)
        self.nx, self.ny, self.nz = int(spec.nx), int(spec.ny), int(spec.nz)
        self.V = self.nx * self.ny * self.nz
        self.G = self._st.shape[1]
        self.nmat = self._st.shape[0]
        self.L = int(spec.legendre_order)
        self.N = int(spec.sn_order)
        self.Nd = self.N * (self.N + 2)
        if self._mat.size != self.V:
            raise ValueError("material must have nx*ny*nz entries")
        desc = ProblemDesc(self.nx, self.ny, self.nz, float(spec.dx), float(spec.dy), float(spec.dz),
                           _ptr(self._mat, C.POINTER(C.c_uint8)), _ptr(self._dens), self._st.shape[0], self.G,
                           _ptr(self._st), self.L, _ptr(self._ss), self.N, int(spec.fixup), self.precision)
        h = C.c_void_p(0)
        _check(lib().dsn_create(C.byref(desc), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().dsn_destroy(self.handle)
            self.handle = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self):
        return lib().dsn_workspace_bytes(self.handle)

    def set_density(self, density):
        """Replaces the per-voxel density: a cuda FP64 tensor [V] (natural
        order), a numpy array, or None (all ones)."""
        if density is None:
            _check(lib().dsn_set_density(self.handle, None))
            return
        if hasattr(density, "data_ptr"):
            d = density.to(dtype=__import__("torch").float64).contiguous()
            if d.numel() != self.V:
                raise ValueError("density must have V entries")
            _check(lib().dsn_set_density(self.handle, C.c_void_p(d.data_ptr())))
            return
        d = np.ascontiguousarray(density, dtype=np.float64).reshape(-1)
        if d.size != self.V:
            raise ValueError("density must have V entries")
        _check(lib().dsn_set_density(self.handle, d.ctypes.data_as(C.c_void_p)))

    def solve(self, sources, tol=1e-10, max_iters=10000, fixed_iters=None, stagnation_stop=False,
              uncollided=False, stream=None, out=None, profile=False, wait_limit=0, autotune=False, combine=False,
              stop_rule=0):
        """Solves every source; returns dict(phi_total [n_src][G][V] cuda
        FP64 tensor, phi_u (or None), iters [n_src][G], residual, updates,
        seconds, status, stages, sweep_bytes, sweep_shape = (waves per
        block, blocks, per-XCD queues, column-relay roles)).  autotune: time the sweep launch
        shapes at this call if the handle has not been tuned (see
        sweep_tuning(), set_sweep_shape()).
        combine: the sources act together in one solve (a CT ring); the
        outputs are then [1][G][V].
        stop_rule: 0 stops a group on the relative L2 change of its scalar
        fluence, 1 on the estimated per-voxel error (dsn_solve_opts)."""
        import torch
        if not isinstance(sources, (list, tuple)):
            sources = [sources]
        ns = len(sources)
        structs, keep = [], []
        for s in sources:
            st, sp = _source_struct(s, self.G)
            structs.append(st)
            keep.append(sp)
        arr = (Source * ns)(*structs)
        dev = torch.device("cuda", torch.cuda.current_device())
        no = 1 if combine else ns
        phit = out if out is not None else torch.empty((no, self.G, self.V), dtype=torch.float64, device=dev)
        if tuple(phit.shape) != (no, self.G, self.V) or phit.dtype != torch.float64 or not phit.is_cuda:
            raise ValueError("out must be a cuda float64 tensor of shape %s" % ((no, self.G, self.V),))
        phiu = torch.empty((no, self.G, self.V), dtype=torch.float64, device=dev) if uncollided else None
        o, fi = _opts(self.G, tol, max_iters, fixed_iters, stagnation_stop, _stream_handle(stream), profile,
                      wait_limit, autotune, combine, stop_rule)
        iters = np.zeros((no, self.G), dtype=np.int32)
        res = np.zeros((no, self.G))
        info = SolveInfo()
        info.iters, info.residual = _ptr(iters, _ip), _ptr(res)
        st = _check(lib().dsn_solve(self.handle, arr, ns, C.byref(o), C.c_void_p(phit.data_ptr()),
                                    C.c_void_p(phiu.data_ptr()) if phiu is not None else None, C.byref(info)))
        return dict(phi_total=phit, phi_u=phiu, iters=iters, residual=res, updates=info.updates,
                    seconds=info.seconds, status=st, stages=info.stages(), sweep_bytes=info.sweep_bytes,
                    sweep_shape=(info.sweep_waves_per_block, info.sweep_blocks, info.sweep_xcd_queues,
                                 info.sweep_relay))

    def solve_noalloc(self, source, tol=1e-10, max_iters=10000, fixed_iters=None, stagnation_stop=False,
                      uncollided=False, stream=None, out=None, wait_limit=0, stop_rule=0):
        """One source through dsn_solve_noalloc (no device allocation by the
        library: its working set lives in a fixed 64 MiB device array per
        GPU).  Returns dict(phi_total [G][V], phi_u (or None), iters [G],
        residual, updates, seconds, status, sweep_shape).  Output tensors are
        allocated here unless `out` is given."""
        import torch
        st_, sp = _source_struct(source, self.G)
        dev = torch.device("cuda", torch.cuda.current_device())
        phit = out if out is not None else torch.empty((self.G, self.V), dtype=torch.float64, device=dev)
        if tuple(phit.shape) != (self.G, self.V) or phit.dtype != torch.float64 or not phit.is_cuda:
            raise ValueError("out must be a cuda float64 tensor of shape %s" % ((self.G, self.V),))
        phiu = torch.empty((self.G, self.V), dtype=torch.float64, device=dev) if uncollided else None
        o, fi = _opts(self.G, tol, max_iters, fixed_iters, stagnation_stop, _stream_handle(stream), False,
                      wait_limit, False, False, stop_rule)
        iters = np.zeros(self.G, dtype=np.int32)
        res = np.zeros(self.G)
        info = SolveInfo()
        info.iters, info.residual = _ptr(iters, _ip), _ptr(res)
        st = _check(lib().dsn_solve_noalloc(self.handle, C.byref(st_), C.byref(o), C.c_void_p(phit.data_ptr()),
                                            C.c_void_p(phiu.data_ptr()) if phiu is not None else None,
                                            C.byref(info)))
        return dict(phi_total=phit, phi_u=phiu, iters=iters, residual=res, updates=info.updates,
                    seconds=info.seconds, status=st,
                    sweep_shape=(info.sweep_waves_per_block, info.sweep_blocks, info.sweep_xcd_queues,
                                 info.sweep_relay))

    def dose(self, phi, k, stream=None):
        """Absorbed dose sum_g phi[g] k[material][g]: phi a cuda FP64 tensor
        [n][G][V] or [G][V], k [n_materials][G] fluence-to-dose factors.
        Returns a cuda FP64 tensor [n][V] (or [V])."""
        import torch
        single = phi.dim() == 2
        ph = (phi.unsqueeze(0) if single else phi).to(torch.float64).contiguous()
        if ph.dim() != 3 or ph.shape[1] != self.G or ph.shape[2] != self.V or not ph.is_cuda:
            raise ValueError("phi must be a cuda tensor [n][G][V]")
        kk = np.ascontiguousarray(k, dtype=np.float64)
        if kk.shape != (self.nmat, self.G):
            raise ValueError("k must be [n_materials][G]")
        out = torch.empty((ph.shape[0], self.V), dtype=torch.float64, device=ph.device)
        _check(lib().dsn_dose(self.handle, C.c_void_p(ph.data_ptr()), int(ph.shape[0]), _ptr(kk),
                              C.c_void_p(out.data_ptr()), C.c_void_p(_stream_handle(stream))))
        return out[0] if single else out

    def sweep_tuning(self):
        """The launch shapes the autotune timed: list of (waves per block,
        blocks, per-XCD queues, column-relay roles, ms per sweep; negative
        ms: the shape's result differed from the default shape's and it was
        not used), empty before any autotune."""
        cap = 64
        w = np.zeros(cap, dtype=np.int32)
        b = np.zeros(cap, dtype=np.int32)
        x = np.zeros(cap, dtype=np.int32)
        r = np.zeros(cap, dtype=np.int32)
        ms = np.zeros(cap, dtype=np.float32)
        n = lib().dsn_sweep_tuning(self.handle, _ptr(w, _ip), _ptr(b, _ip), _ptr(x, _ip), _ptr(r, _ip),
                                   ms.ctypes.data_as(C.POINTER(C.c_float)), cap)
        return [(int(w[i]), int(b[i]), int(x[i]), int(r[i]), float(ms[i])) for i in range(min(n, cap))]

    def xcd_queues(self):
        """Per-XCD ticket queues the device allows (0: only the global
        queue); see dsn_xcd_queues."""
        n = lib().dsn_xcd_queues(self.handle)
        if n < 0:
            raise DsnError(DSN_ERR_DEVICE, last_error())
        return int(n)

    def set_sweep_shape(self, waves_per_block, blocks, xcd_queues=0, relay=0):
        """Pins the sweep launch shape (e.g. one from another handle's
        sweep_tuning()); the handle then counts as tuned.  relay > 0: the
        column-relay sweep with that many roles (dsn_set_sweep_shape)."""
        _check(lib().dsn_set_sweep_shape(self.handle, int(waves_per_block), int(blocks), int(xcd_queues),
                                         int(relay)))

    def adjoint(self, source, W, tol=1e-10, max_iters=10000, fixed_iters=None, stream=None, want_phi=False):
        """dJ/d(density) of J = sum W * phi_total.  W: cuda FP64 tensor [G][V].
        Returns dict(J, grad (cuda [V]), phi_total or None, iters, updates,
        seconds, status)."""
        import torch
        W = W.to(torch.float64).contiguous()
        if W.numel() != self.G * self.V or not W.is_cuda:
            raise ValueError("W must be a cuda tensor with G*V entries")
        st_, sp = _source_struct(source, self.G)
        grad = torch.empty(self.V, dtype=torch.float64, device=W.device)
        phit = torch.empty((self.G, self.V), dtype=torch.float64, device=W.device) if want_phi else None
        o, fi = _opts(self.G, tol, max_iters, fixed_iters, False, _stream_handle(stream))
        J = C.c_double(0.0)
        iters = np.zeros((2, self.G), dtype=np.int32)
        info = SolveInfo()
        info.iters = _ptr(iters, _ip)
        st = _check(lib().dsn_solve_adjoint(self.handle, C.byref(st_), C.c_void_p(W.data_ptr()), C.byref(o),
                                            C.byref(J), C.c_void_p(grad.data_ptr()),
                                            C.c_void_p(phit.data_ptr()) if phit is not None else None,
                                            C.byref(info)))
        return dict(J=J.value, grad=grad, phi_total=phit, iters=iters, updates=info.updates,
                    seconds=info.seconds, status=st)


BATCH_STREAMS, BATCH_FUSED = 0, 1


def solve_batch(problems, sources, tol=1e-10, max_iters=10000, fixed_iters=None, stagnation_stop=False,
                stream=None, stop_rule=0, batch_mode=BATCH_STREAMS, autotune=False, wait_limit=0):
    """Batched solve: sources[b] is the list of sources of problems[b].
    batch_mode: BATCH_STREAMS (a stream and host thread per problem, the
    default) or BATCH_FUSED (one sweep launch per source iteration over every
    (problem, source) pair).  Returns
    dict(phi_total: list of cuda tensors [n_src_b][G][V_b], iters
    [total_src][G], updates, seconds, status, sweep_shape (the fused launch's
    (waves per block, blocks), zeros for a stream per problem))."""
    import torch
    nb = len(problems)
    G = problems[0].G
    handles = (C.c_void_p * nb)(*[p.handle.value for p in problems])
    keep, arrs = [], []
    nsrc = np.zeros(nb, dtype=np.int32)
    for b, (p, srcs) in enumerate(zip(problems, sources)):
        structs = []
        for s in srcs:
            st, sp = _source_struct(s, G)
            structs.append(st)
            keep.append(sp)
        a = (Source * max(1, len(srcs)))(*structs)
        arrs.append(a)
        nsrc[b] = len(srcs)
    parr = (C.POINTER(Source) * nb)(*[C.cast(a, C.POINTER(Source)) for a in arrs])
    dev = torch.device("cuda", torch.cuda.current_device())
    outs = [torch.empty((int(nsrc[b]), G, p.V), dtype=torch.float64, device=dev) for b, p in enumerate(problems)]
    optr = (C.c_void_p * nb)(*[o.data_ptr() for o in outs])
    o, fi = _opts(G, tol, max_iters, fixed_iters, stagnation_stop, _stream_handle(stream), stop_rule=stop_rule,
                  batch_mode=batch_mode, autotune=autotune, wait_limit=wait_limit)
    iters = np.zeros((int(nsrc.sum()), G), dtype=np.int32)
    info = SolveInfo()
    info.iters = _ptr(iters, _ip)
    st = _check(lib().dsn_solve_batch(handles, nb, parr, _ptr(nsrc, _ip), C.byref(o), optr, C.byref(info)))
    return dict(phi_total=outs, iters=iters, updates=info.updates, seconds=info.seconds, status=st,
                sweep_shape=(info.sweep_waves_per_block, info.sweep_blocks))
