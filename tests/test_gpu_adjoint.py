"""GPU adjoint / density gradient (through the C ABI) against the oracle's
adjoint and against central finite differences of the forward solve."""
import numpy as np
import pytest

import oracle
from synthetic.workloads import SourceSpec, config4, detector_weights, random_small_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
dsn = pytest.importorskip("paper_1910_11335_amd")


def _grad_err(got, want, floor=1e-6):
    sel = np.abs(want) > floor * np.abs(want).max()
    return (np.abs(got - want)[sel] / np.abs(want[sel])).max()


SMALL = [
    # seed, mesh, sn, L, G, n_mat, source kind
    (81, (3, 4, 3), 4, 1, 2, 2, "cone"),
    (82, (9, 10, 7), 4, 1, 3, 3, "outside"),
    (83, (12, 9, 17), 8, 3, 2, 3, "inside"),
]


def _src(kind, p):
    ext = np.array([p.nx * p.dx, p.ny * p.dy, p.nz * p.dz])
    spec = np.linspace(1.0, 0.4, p.G)
    if kind == "cone":
        return SourceSpec(position=(-2.0, 1.5, 1.7), axis=(1.0, 0.1, 0.0), half_angle=np.deg2rad(35), spectrum=spec)
    if kind == "outside":
        return SourceSpec(position=(-3.0, 0.4 * ext[1], 0.6 * ext[2]), spectrum=spec)
    return SourceSpec(position=tuple(0.41 * ext + 0.013), spectrum=spec)


@pytest.mark.parametrize("case", SMALL, ids=[str(c[0]) for c in SMALL])
def test_adjoint_fp64_matches_oracle(case):
    seed, n, sn, L, G, nm, kind = case
    p = random_small_problem(seed, n=n, sn=sn, L=L, G=G, n_mat=nm, fixup=0, density=True)
    s = _src(kind, p)
    W = np.random.default_rng(seed).uniform(0, 1, (p.G, p.V))
    ref = oracle.adjoint(p, s, W, tol=1e-13)
    h = dsn.Problem(p, "fp64")
    out = h.adjoint(s, torch.tensor(W, device="cuda"), tol=1e-13)
    g = out["grad"].cpu().numpy()
    e = _grad_err(g, ref["grad"])
    print("case", seed, "J rel %.2e grad rel %.2e" % (abs(out["J"] / ref["J"] - 1), e), flush=True)
    assert abs(out["J"] / ref["J"] - 1) < 1e-12
    assert e < 1e-10
    assert list(out["iters"][0]) == list(ref["iters_fwd"])
    h.close()


def test_adjoint_fp32_vs_oracle():
    seed, n, sn, L, G, nm, kind = SMALL[1]
    p = random_small_problem(seed, n=n, sn=sn, L=L, G=G, n_mat=nm, fixup=0, density=True)
    s = _src(kind, p)
    W = np.random.default_rng(seed).uniform(0, 1, (p.G, p.V))
    ref = oracle.adjoint(p, s, W, tol=1e-13)
    h = dsn.Problem(p, "fp32")
    out = h.adjoint(s, torch.tensor(W, device="cuda"), tol=1e-7)
    e = _grad_err(out["grad"].cpu().numpy(), ref["grad"], floor=1e-3)
    print("fp32 grad rel %.2e" % e, flush=True)
    assert e < 1e-3
    h.close()


def test_config4_gradient_vs_central_differences():
    """64^3, S8 P3, G = 10, density ~ U(0.8, 1.2), exit-face detector loss:
    FP32 adjoint gradient against central differences (h = 1e-3) of the
    converged GPU-FP64 forward solve on 32 seeded voxels whose gradient is
    at least 1e-3 of the largest."""
    p, s = config4()
    W = detector_weights(p)
    Wt = torch.tensor(W, device="cuda")
    h32 = dsn.Problem(p, "fp32")
    r32 = h32.adjoint(s, Wt, tol=1e-7)
    g32 = r32["grad"].cpu().numpy()
    h64 = dsn.Problem(p, "fp64")
    r64 = h64.adjoint(s, Wt, tol=1e-12)
    g64 = r64["grad"].cpu().numpy()
    cand = np.flatnonzero(np.abs(g64) >= 1e-3 * np.abs(g64).max())
    pick = np.random.default_rng(4004).choice(cand, 32, replace=False)
    hstep = 1e-3
    fd = np.zeros(len(pick))
    dens = p.density.copy()
    for t, v in enumerate(pick):
        for sgn in (+1, -1):
            d = dens.copy()
            d[v] += sgn * hstep
            h64.set_density(d)
            phi = h64.solve([s], tol=1e-12)["phi_total"][0].cpu().numpy()
            fd[t] += sgn * (W * phi).sum() / (2 * hstep)
    e32 = np.abs(g32[pick] - fd) / np.abs(fd)
    e64 = np.abs(g64[pick] - fd) / np.abs(fd)
    print("config4 FD check: fp32 max rel %.2e, fp64 max rel %.2e" % (e32.max(), e64.max()), flush=True)
    assert e64.max() < 1e-4
    assert e32.max() < 1e-3
    h32.close()
    h64.close()


def test_autograd_function_matches_adjoint():
    seed, n, sn, L, G, nm, kind = SMALL[0]
    p = random_small_problem(seed, n=n, sn=sn, L=L, G=G, n_mat=nm, fixup=0, density=True)
    s = _src(kind, p)
    W = torch.tensor(np.random.default_rng(5).uniform(0, 1, (p.G, p.V)), device="cuda")
    h = dsn.Problem(p, "fp64")
    rho = torch.tensor(p.density, device="cuda", requires_grad=True)
    phi = dsn.fluence(rho, h, s, tol=1e-13)
    loss = (W * phi).sum()
    loss.backward()
    ref = oracle.adjoint(p, s, W.cpu().numpy(), tol=1e-13)
    assert abs(loss.item() / ref["J"] - 1) < 1e-12
    assert _grad_err(rho.grad.cpu().numpy(), ref["grad"]) < 1e-10
    h.close()


def _thick(seed, n, sn, L, G):
    """Optically thick cells (6x the generator's cross sections): with the
    fixup on, many cells of the converged solve have fixed axes."""
    p = random_small_problem(seed, n=n, sn=sn, L=L, G=G, n_mat=2, fixup=1, density=True)
    p.sigma_t = p.sigma_t * 6.0
    p.sigma_s = p.sigma_s * 6.0
    return p


FIXUP = [
    # seed, mesh, sn, L, G, source kind
    (84, (4, 4, 3), 4, 1, 2, "cone"),
    (85, (9, 10, 7), 4, 1, 3, "outside"),
    (86, (12, 9, 17), 8, 3, 2, "inside"),
]


@pytest.mark.parametrize("case", FIXUP, ids=[str(c[0]) for c in FIXUP])
def test_adjoint_with_fixup_fp64_matches_oracle(case):
    """Adjoint through the set-to-zero fixup (fixed-axis sets frozen at the
    converged solution, transposed frozen cell) against the oracle's."""
    seed, n, sn, L, G, kind = case
    p = _thick(seed, n, sn, L, G)
    s = _src(kind, p)
    assert oracle.solve(p, s, tol=1e-13)["nneg"] > 0
    W = np.random.default_rng(seed).uniform(0, 1, (p.G, p.V))
    ref = oracle.adjoint(p, s, W, tol=1e-13)
    h = dsn.Problem(p, "fp64")
    out = h.adjoint(s, torch.tensor(W, device="cuda"), tol=1e-13)
    e = _grad_err(out["grad"].cpu().numpy(), ref["grad"])
    print("fixup case", seed, "J rel %.2e grad rel %.2e" % (abs(out["J"] / ref["J"] - 1), e), flush=True)
    assert abs(out["J"] / ref["J"] - 1) < 1e-12
    assert e < 1e-10
    assert list(out["iters"][0]) == list(ref["iters_fwd"])
    assert list(out["iters"][1]) == list(ref["iters_adj"])
    h.close()


def test_adjoint_with_fixup_fp32_vs_oracle():
    seed, n, sn, L, G, kind = FIXUP[1]
    p = _thick(seed, n, sn, L, G)
    s = _src(kind, p)
    W = np.random.default_rng(seed).uniform(0, 1, (p.G, p.V))
    ref = oracle.adjoint(p, s, W, tol=1e-13)
    h = dsn.Problem(p, "fp32")
    out = h.adjoint(s, torch.tensor(W, device="cuda"), tol=1e-7)
    e = _grad_err(out["grad"].cpu().numpy(), ref["grad"], floor=1e-3)
    print("fixup fp32 grad rel %.2e" % e, flush=True)
    assert e < 1e-3
    h.close()


def test_adjoint_with_fixup_on_per_xcd_forward_shape():
    """FP32 with the fixup on a handle pinned to per-XCD queues: the forward
    sweeps use tagged face words, the fixed-axis recording sweeps of the
    adjoint sign-parity ones on the same buffers, so every adjoint switches
    between them.  Two adjoints in a row and a forward solve afterwards equal
    the default-shape handle's results (the forward one bit for bit; J and
    the gradient, whose back-projection sums with atomics, to 1e-12)."""
    seed, n, sn, L, G, kind = FIXUP[2]
    p = _thick(seed, n, sn, L, G)
    s = _src(kind, p)
    W = torch.tensor(np.random.default_rng(seed).uniform(0, 1, (p.G, p.V)), device="cuda")
    h0 = dsn.Problem(p, "fp32")
    ref = h0.adjoint(s, W, tol=1e-7)
    fwd = h0.solve([s], tol=1e-7, stagnation_stop=True)["phi_total"]
    h0.close()
    h = dsn.Problem(p, "fp32")
    nq = h.xcd_queues()
    if nq == 0:
        pytest.skip("the device probe saw no round-robin workgroup placement: no per-XCD queues")
    h.set_sweep_shape(2, 64, nq)
    for rep in range(2):
        out = h.adjoint(s, W, tol=1e-7)
        assert list(out["iters"][0]) == list(ref["iters"][0]) and list(out["iters"][1]) == list(ref["iters"][1])
        assert abs(out["J"] / ref["J"] - 1) < 1e-12, rep
        assert _grad_err(out["grad"].cpu().numpy(), ref["grad"].cpu().numpy()) < 1e-12, rep
    got = h.solve([s], tol=1e-7, stagnation_stop=True)
    assert got["sweep_shape"] == (2, 64, nq, 0)
    assert torch.equal(got["phi_total"], fwd)
    h.close()


@pytest.mark.parametrize("fixup", [0, 1])
def test_adjoint_on_a_column_relay_forward_shape(fixup):
    """A handle pinned to a column-relay sweep shape (rows of pencils with
    the y faces handed over in LDS): its forward sweeps use the relay
    kernel; the adjoint's reversed, recording and transposed sweeps use
    pencil items of as many directions per block, on the same face buffers
    (the relay leaves the y words stale, so every switch invalidates them).
    Two adjoints in a row and a forward solve afterwards equal the
    default-shape handle's results (the forward one bit for bit; J and the
    gradient, whose back-projection sums with atomics, to 1e-12)."""
    if fixup:
        seed, n, sn, L, G, kind = FIXUP[2]
        p = _thick(seed, n, sn, L, G)
    else:
        seed, n, sn, L, G, nm, kind = SMALL[2]
        p = random_small_problem(seed, n=n, sn=sn, L=L, G=G, n_mat=nm, fixup=0, density=True)
    s = _src(kind, p)
    W = torch.tensor(np.random.default_rng(seed).uniform(0, 1, (p.G, p.V)), device="cuda")
    h0 = dsn.Problem(p, "fp32")
    ref = h0.adjoint(s, W, tol=1e-7)
    fwd = h0.solve([s], tol=1e-7, stagnation_stop=True)["phi_total"]
    h0.close()
    h = dsn.Problem(p, "fp32")
    h.set_sweep_shape(1, 96, 0, 2)
    for rep in range(2):
        out = h.adjoint(s, W, tol=1e-7)
        assert list(out["iters"][0]) == list(ref["iters"][0]) and list(out["iters"][1]) == list(ref["iters"][1])
        assert abs(out["J"] / ref["J"] - 1) < 1e-12, rep
        assert _grad_err(out["grad"].cpu().numpy(), ref["grad"].cpu().numpy()) < 1e-12, rep
    got = h.solve([s], tol=1e-7, stagnation_stop=True)
    assert got["sweep_shape"] == (1, 96, 0, 2)
    assert torch.equal(got["phi_total"], fwd)
    h.close()
