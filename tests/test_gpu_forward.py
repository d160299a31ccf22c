"""GPU parity of the forward solve against the FP64 oracle (through the C ABI).

Bar: GPU-FP64 within 1e-12 relative and FP32 (FP64 reductions) within 1e-4
relative, per voxel, over voxels above 1e-6 of the group maximum, with the
same iteration counts on both sides (tests/parity.py: voxels next to a sign
change of a pure diamond-difference fluence against the group maximum)."""
import numpy as np
import pytest

import oracle
from parity import l2_rel, parity_err, rel_err
from synthetic.workloads import SourceSpec, config1, config2, config3, random_small_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
dsn = pytest.importorskip("paper_1910_11335_amd")


def test_config1_fp64_matches_oracle():
    p, s = config1()
    ref = oracle.solve(p, s, tol=1e-8)
    print("oracle iters", ref["iters"], flush=True)
    h = dsn.Problem(p, "fp64")
    out = h.solve([s], tol=1e-8, uncollided=True)
    got = out["phi_total"][0].cpu().numpy()
    assert list(out["iters"][0]) == list(ref["iters"])
    assert rel_err(got, ref["phi_total"]) < 1e-12
    assert l2_rel(got, ref["phi_total"]) < 1e-12
    assert rel_err(out["phi_u"][0].cpu().numpy(), ref["phi_u"]) < 1e-13
    h.close()


CASES = [
    # (seed, mesh, sn, L, G, n_mat, fixup, source)
    (1, (5, 7, 9), 2, 1, 2, 2, 0, "inside"),
    (2, (20, 19, 21), 4, 1, 3, 3, 1, "cone"),
    (3, (9, 17, 8), 6, 2, 2, 2, 0, "outside"),
    (4, (16, 16, 16), 8, 3, 2, 4, 1, "cone"),
    (5, (1, 1, 1), 4, 1, 1, 1, 0, "outside"),
    (6, (33, 3, 12), 12, 4, 2, 2, 1, "inside"),
    (15, (13, 11, 10), 10, 0, 3, 2, 1, "cone"),     # S10, isotropic scattering
    (16, (12, 9, 14), 6, 0, 2, 3, 0, "inside"),     # P0 with pure DD
    (18, (17, 10, 12), 10, 3, 2, 3, 0, "outside"),  # S10 P3
]


def _source(kind, p, G):
    ext = np.array([p.nx * p.dx, p.ny * p.dy, p.nz * p.dz])
    spec = np.linspace(1.0, 0.3, G)
    if kind == "inside":
        return SourceSpec(position=tuple(0.37 * ext + 0.011), spectrum=spec)
    if kind == "outside":
        return SourceSpec(position=(-2.3, 0.6 * ext[1], 0.45 * ext[2]), spectrum=spec)
    return SourceSpec(position=(ext[0] + 7.0, 0.5 * ext[1], 0.5 * ext[2]), axis=(-1.0, 0.05, 0.0),
                      half_angle=np.deg2rad(25.0), spectrum=spec)


@pytest.mark.parametrize("case", CASES, ids=[str(c[0]) for c in CASES])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_ragged_meshes(case, precision):
    seed, n, sn, L, G, nm, fixup, kind = case
    p = random_small_problem(seed, n=n, sn=sn, L=L, G=G, n_mat=nm, fixup=fixup)
    s = _source(kind, p, G)
    fixed = [4] * G
    ref = oracle.solve(p, s, fixed_iters=fixed)
    h = dsn.Problem(p, precision)
    out = h.solve([s], fixed_iters=fixed)
    got = out["phi_total"][0].cpu().numpy()
    tol = 1e-12 if precision == "fp64" else 1e-4
    e = parity_err(got, ref["phi_total"], p, 1e-13 if precision == "fp64" else 1e-5)
    print("case", case, precision, "max rel err %.3e" % e, flush=True)
    assert e < tol
    h.close()


def test_converged_iteration_counts_and_fp32_error():
    """Converged solves in the benchmark's stopping rules (dsn.CONVERGED)
    against the oracle converged much further (L2 change below 1e-13): GPU
    FP64 stops after the oracle's iteration counts at the same rule and
    matches it to 1e-12; FP32 (estimated per-voxel error below 1e-5, or the
    FP32 floor) is within 1e-4 of the converged solution at every voxel above
    1e-6 of its group's maximum.  The problem is pure DD with negative
    fluence, where the L2 stop at 1e-6 once left low-fluence voxels 1e-4 off."""
    p = random_small_problem(7, n=(18, 13, 11), sn=4, L=2 - 1, G=2, n_mat=2, fixup=0)
    s = _source("cone", p, 2)
    r64 = dsn.CONVERGED["fp64"]
    ref = oracle.solve(p, s, tol=r64["tol"], stop_rule=r64["stop_rule"])
    h = dsn.Problem(p, "fp64")
    out = h.solve([s], **r64)
    assert list(out["iters"][0]) == list(ref["iters"])
    assert parity_err(out["phi_total"][0].cpu().numpy(), ref["phi_total"], p) < 1e-12
    conv = oracle.solve(p, s, tol=1e-13)["phi_total"]
    h32 = dsn.Problem(p, "fp32")
    out32 = h32.solve([s], **dsn.CONVERGED["fp32"])
    got32 = out32["phi_total"][0].cpu().numpy()
    e = parity_err(got32, conv, p, 1e-5)
    print("fp32 converged err %.3e (every voxel against its own value: %.3e) iters %s (fp64 %s)" % (
        e, rel_err(got32, conv), out32["iters"][0].tolist(), out["iters"][0].tolist()), flush=True)
    assert e < 1e-4
    h.close()
    h32.close()


@pytest.mark.parametrize("fixup", [0, 1])
def test_pointwise_stop_rule_matches_oracle(fixup):
    """Stop rule 1 (estimated per-voxel error) on the GPU in FP64 stops after
    the same iteration counts as the oracle's rule 1 at the same tol, and
    the results agree to 1e-12."""
    p = random_small_problem(11 + fixup, n=(18, 13, 11), sn=4, L=1, G=2, n_mat=2, fixup=fixup)
    s = _source("cone", p, 2)
    h = dsn.Problem(p, "fp64")
    for tol in (1e-5, 1e-8):
        ref = oracle.solve(p, s, tol=tol, stop_rule=1)
        out = h.solve([s], tol=tol, stop_rule=1)
        print("rule 1 tol %g iters %s" % (tol, ref["iters"].tolist()), flush=True)
        assert list(out["iters"][0]) == list(ref["iters"])
        assert parity_err(out["phi_total"][0].cpu().numpy(), ref["phi_total"], p) < 1e-12
    h.close()


def test_multiple_sources_and_repeatability():
    p = random_small_problem(8, n=(10, 9, 8), sn=4, L=1, G=2, n_mat=2, fixup=1)
    srcs = [_source(k, p, 2) for k in ("inside", "outside", "cone")]
    h = dsn.Problem(p, "fp32")
    a = h.solve(srcs, fixed_iters=[3, 3])["phi_total"].cpu().numpy()
    b = h.solve(srcs, fixed_iters=[3, 3])["phi_total"].cpu().numpy()
    assert np.array_equal(a, b)  # no atomics in the forward path: bitwise repeatable
    for i, s in enumerate(srcs):
        ref = oracle.solve(p, s, fixed_iters=[3, 3])
        assert rel_err(a[i], ref["phi_total"]) < 1e-4
    h.close()


def test_empty_source_list_is_a_no_op():
    """No sources: an empty result and no device work; the handle then
    solves normally."""
    p = random_small_problem(10, n=(6, 5, 7), sn=4, L=1, G=2, n_mat=2, fixup=1)
    h = dsn.Problem(p, "fp32")
    out = h.solve([], fixed_iters=[2, 2])
    assert tuple(out["phi_total"].shape) == (0, 2, p.V) and out["updates"] == 0
    s = _source("inside", p, 2)
    got = h.solve([s], fixed_iters=[2, 2])["phi_total"][0].cpu().numpy()
    assert rel_err(got, oracle.solve(p, s, fixed_iters=[2, 2])["phi_total"]) < 1e-4
    h.close()


def test_streamed_and_cached_paths_agree():
    """48^3 S16 FP32 (128 MB of angular fluence per source): one source fits
    the last-level cache, so the kernels use ordinary loads and stores; three
    sources in one launch (382 MB) exceed it, so the streamed arrays go
    non-temporal.  The hint changes no arithmetic: each source's fluence is
    the same bit for bit, and equals the oracle's."""
    p = random_small_problem(21, n=(48, 48, 48), d=(0.5, 0.5, 0.5), sn=16, L=2, G=2, n_mat=3, fixup=1)
    srcs = [_source(k, p, 2) for k in ("cone", "inside", "outside")]
    fixed = [2, 1]
    h = dsn.Problem(p, "fp32")
    both = h.solve(srcs, fixed_iters=fixed)["phi_total"]
    for i, s in enumerate(srcs):
        one = h.solve([s], fixed_iters=fixed)["phi_total"][0]
        assert torch.equal(one, both[i]), i
    ref = oracle.solve(p, srcs[0], fixed_iters=fixed)
    assert rel_err(both[0].cpu().numpy(), ref["phi_total"]) < 1e-4
    h.close()


def test_not_converged_status():
    p, s = config1()
    h = dsn.Problem(p, "fp64")
    out = h.solve([s], tol=1e-14, max_iters=3)
    assert out["status"] == dsn.dsn.DSN_ERR_NOT_CONVERGED
    assert (out["iters"] == 3).all()
    ref = oracle.solve(p, s, fixed_iters=[3, 3])
    assert rel_err(out["phi_total"][0].cpu().numpy(), ref["phi_total"]) < 1e-12
    h.close()


_CFG2 = {}


def _cfg2_oracle():
    if not _CFG2:
        p, s = config2()
        _CFG2["r"] = (p, s, oracle.solve(p, s, fixed_iters=[2] * p.G))
    return _CFG2["r"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config2_full_size(precision):
    """64^3, S8 P3, G = 19, water cylinder, cone source, fixup on, two source
    iterations per group, in the autotuned launch shape the benchmark times,
    every voxel against the oracle; in FP32 also pinned to per-XCD queues,
    bit for bit equal to the tuned solve."""
    p, s, ref = _cfg2_oracle()
    fixed = [2] * p.G
    h = dsn.Problem(p, precision)
    out = h.solve([s], fixed_iters=fixed, autotune=True)
    got = out["phi_total"][0].cpu().numpy()
    e = rel_err(got, ref["phi_total"])
    print("config2", precision, "shape", out["sweep_shape"], "max rel err %.3e" % e, flush=True)
    nq = h.xcd_queues()
    if precision == "fp32" and nq > 0:  # per-XCD queues, where the device's workgroup placement allows them
        h.set_sweep_shape(2, 1024, nq)
        assert torch.equal(h.solve([s], fixed_iters=fixed)["phi_total"], out["phi_total"])
    assert e < (1e-12 if precision == "fp64" else 1e-4)
    h.close()


def test_dependency_timeout_reports_error_and_recovers():
    """A wait limit of one poll (forced from the host) makes every downstream
    pencil give up at its first stale face word: the sweeps abort, the call
    reports a device error, and the same problem then solves normally."""
    p = random_small_problem(9, n=(24, 20, 19), sn=8, L=1, G=2, n_mat=2, fixup=1)
    s = _source("cone", p, 2)
    h = dsn.Problem(p, "fp32")
    with pytest.raises(dsn.DsnError) as err:
        h.solve([s], fixed_iters=[1, 1], wait_limit=1)
    assert err.value.status == dsn.dsn.DSN_ERR_DEVICE
    out = h.solve([s], fixed_iters=[2, 2])
    ref = oracle.solve(p, s, fixed_iters=[2, 2])
    assert rel_err(out["phi_total"][0].cpu().numpy(), ref["phi_total"]) < 1e-4
    h.close()


_CFG3 = {}


def _cfg3_two_groups():
    """The benchmark workload (128^3 x 0.25 cm phantom, S16 P5, cone source,
    fixup on) restricted to its first two energy groups, which are exactly
    groups 0 and 1 of the 19-group solve (no upscatter)."""
    if not _CFG3:
        p, s = config3()
        p2 = type(p)(**{**p.__dict__, "sigma_t": p.sigma_t[:, :2].copy(), "sigma_s": p.sigma_s[:, :, :2, :2].copy()})
        s2 = type(s)(**{**s.__dict__, "spectrum": np.asarray(s.spectrum)[:2].copy()})
        _CFG3["r"] = (p2, s2, oracle.solve(p2, s2, fixed_iters=[2, 1]))
    return _CFG3["r"]


@pytest.mark.timeout(600)  # the oracle's three 128^3 S16 sweeps take about a minute
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_config3_full_size_first_groups(precision):
    """Full benchmark mesh, quadrature and scattering order in the launch
    configuration the benchmark times (the sweep shape picked by the same
    autotune at the first iteration of group 0), two source iterations in
    group 0 (in-group scattering) and one in group 1 (downscatter), every
    voxel against the oracle."""
    p, s, ref = _cfg3_two_groups()
    h = dsn.Problem(p, precision)
    out = h.solve([s], fixed_iters=[2, 1], autotune=True)
    got = out["phi_total"][0].cpu().numpy()
    e = rel_err(got, ref["phi_total"])
    print("config3 first groups", precision, "shape", out["sweep_shape"], "max rel err %.3e" % e, flush=True)
    assert all(ms > 0 for _, _, _, _, ms in h.sweep_tuning())
    assert e < (1e-12 if precision == "fp64" else 1e-4)
    h.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_graph_replays_match_direct_launches(precision):
    """Steady source iterations replay a captured HIP graph; with the stage
    timer on every kernel is launched directly.  Several graph-replayed solves
    in a row, with other work and synchronisations between them, must each
    equal the directly launched one bit for bit."""
    p = random_small_problem(12, n=(20, 17, 23), sn=6, L=2, G=3, n_mat=3, fixup=1)
    srcs = [_source(k, p, 3) for k in ("inside", "cone")]
    h = dsn.Problem(p, precision)
    tol = 1e-10 if precision == "fp64" else 1e-6
    eager = h.solve(srcs, tol=tol, stagnation_stop=precision == "fp32", profile=True)
    ref = eager["phi_total"].clone()
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated work between replays
        torch.cuda.synchronize()
        out = h.solve(srcs, tol=tol, stagnation_stop=precision == "fp32")
        assert (out["iters"] == eager["iters"]).all()
        assert torch.equal(out["phi_total"], ref), "replay %d differs" % rep
        del junk
    h.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_pinned_sweep_shapes_give_identical_results(precision):
    """Every built waves-per-block value that divides an octant's 10 S8
    directions, with one block, an odd count and more blocks than items, and
    in FP32 the per-XCD queues (one block per XCD upwards), and every
    column-relay shape (rows of pencils with the y faces handed over in LDS;
    one block, an odd count, more blocks than items), pinned with
    dsn_set_sweep_shape on one handle: each solve equals the default shape's
    bit for bit, and the default equals the oracle.  The fixup is on, so
    consecutive solves switch between sign-parity face words (global queue),
    tagged ones (per-XCD queues) and column-relay sweeps that leave the y
    words stale, on the same face buffers."""
    p = random_small_problem(17, n=(19, 22, 17), sn=8, L=3, G=2, n_mat=3, fixup=1)
    srcs = [_source("cone", p, 2), _source("inside", p, 2)]
    fixed = [3, 2]
    ref_h = dsn.Problem(p, precision)
    ref = ref_h.solve(srcs, fixed_iters=fixed)
    ref_h.close()
    tol = 1e-12 if precision == "fp64" else 1e-4
    for i, s in enumerate(srcs):
        o = oracle.solve(p, s, fixed_iters=fixed)
        assert parity_err(ref["phi_total"][i].cpu().numpy(), o["phi_total"], p,
                          1e-13 if precision == "fp64" else 1e-5) < tol
    wl = [1, 2, 5, 10] if precision == "fp32" else [1, 2, 5]
    shapes = [(w, b, 0, 0) for w in wl for b in (1, 7, 3000)]
    cols = [(1, 2), (1, 4), (2, 2), (2, 4)] if precision == "fp32" else [(1, 2), (1, 4)]
    shapes += [(w, b, 0, r) for w, r in cols for b in (1, 7, 3000)]
    h = dsn.Problem(p, precision)
    nq = h.xcd_queues()
    if precision == "fp32":
        shapes = [x for w in (1, 2) for x in ((w, 7, 0, 0),) + (((w, nq, nq, 0), (w, 520, nq, 0)) if nq else ())] \
            + shapes
    # pencil shapes again right after column-relay ones (whose sweeps leave the y words stale)
    shapes += [(2, 64, 0, 0), (1, 64, 0, 2), (1, 7, 0, 0)]
    for w, b, x, r in shapes:
        print("shape", (w, b, x, r), flush=True)
        h.set_sweep_shape(w, b, x, r)
        out = h.solve(srcs, fixed_iters=fixed)
        assert out["sweep_shape"] == (w, b, x, r)
        assert torch.equal(out["phi_total"], ref["phi_total"]), (w, b, x, r)
    with pytest.raises(dsn.DsnError):
        h.set_sweep_shape(10 if precision == "fp32" else 5, 64, max(nq, 8))  # per-XCD queues stop at 4 waves per block
    h.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_autotuned_sweep_shape_gives_identical_results(precision):
    """The autotune times every sweep launch shape (waves per block x grid,
    in FP32 the per-XCD-queue variants, and the column-relay shapes) on the
    first iteration's source,
    checks each shape's angular fluence against the default shape's by
    checksum, and keeps the fastest.  Each direction's arithmetic does not
    depend on the shape: every shape passes the check, and the tuned solve,
    and later solves (graph replays, a batch of sources) on the tuned handle,
    equal the default-shape solve bit for bit."""
    p = random_small_problem(13, n=(21, 18, 24), sn=16, L=3, G=2, n_mat=3, fixup=1)
    srcs = [_source("cone", p, 2), _source("inside", p, 2)]
    fixed = [3, 2]
    ref_h = dsn.Problem(p, precision)
    ref = ref_h.solve(srcs[:1], fixed_iters=fixed)
    ref2 = ref_h.solve(srcs, fixed_iters=fixed)
    ref_h.close()
    h = dsn.Problem(p, precision)
    out = h.solve(srcs[:1], fixed_iters=fixed, autotune=True)
    shapes = h.sweep_tuning()
    built = {1, 2, 3, 4, 5, 6, 9, 10, 12} if precision == "fp32" else {1, 2, 3, 4, 5, 6}
    wpbs = {w for w in built if 36 % w == 0}  # S16: 36 directions per octant
    plain = [x for x in shapes if x[2] == 0 and x[3] == 0]
    xcd = [x for x in shapes if x[2] > 0]
    col = [x for x in shapes if x[3] > 0]
    assert {w for w, _, _, _, _ in plain} == wpbs and len(plain) == 3 * len(wpbs)
    cols = {(1, 2), (1, 4), (2, 2), (2, 4)} if precision == "fp32" else {(1, 2), (1, 4)}
    assert {(w, r) for w, _, _, r, _ in col} == cols and len(col) == 3 * len(cols)
    nq = h.xcd_queues()  # the device probe's per-XCD queue count (0: placement not round robin)
    if precision == "fp32" and nq > 0:  # per-XCD queues: up to four waves per block
        assert {w for w, _, _, _, _ in xcd} == {w for w in wpbs if w <= 4} and {x[2] for x in xcd} == {nq}
    else:
        assert not xcd
    assert all(ms > 0 for _, _, _, _, ms in shapes), shapes  # every shape reproduced the default's fluence
    best = min(shapes, key=lambda x: x[4])
    assert out["sweep_shape"] == best[:4]
    assert torch.equal(out["phi_total"], ref["phi_total"])
    again = h.solve(srcs[:1], fixed_iters=fixed, autotune=True)  # already tuned: no new timing
    assert len(h.sweep_tuning()) == len(shapes) and again["sweep_shape"] == best[:4]
    assert torch.equal(again["phi_total"], ref["phi_total"])
    both = h.solve(srcs, fixed_iters=fixed)
    assert torch.equal(both["phi_total"], ref2["phi_total"])
    h.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fan_beam_matches_oracle(precision):
    """Fan-beam source (collimated to a slab of directions around a plane
    through the axis) against the oracle, fixup on, fixed iterations."""
    p = random_small_problem(14, n=(19, 15, 13), sn=6, L=2, G=3, n_mat=3, fixup=1)
    ext = np.array([p.nx * p.dx, p.ny * p.dy, p.nz * p.dz])
    s = SourceSpec(position=(-4.0, 0.45 * ext[1] + 0.013, 0.52 * ext[2] + 0.007), axis=(1.0, 0.05, 0.02),
                   half_angle=np.deg2rad(28.0), spectrum=np.linspace(1.0, 0.3, 3), fan_normal=(0.0, 0.1, 1.0),
                   fan_half_thickness=np.deg2rad(6.0))
    fixed = [4, 3, 3]
    ref = oracle.solve(p, s, fixed_iters=fixed)
    assert 0 < (ref["phi_u"][0] > 0).sum() < p.V // 2  # a genuine fan, not the whole mesh
    h = dsn.Problem(p, precision)
    out = h.solve([s], fixed_iters=fixed, uncollided=True)
    got_u = out["phi_u"][0].cpu().numpy()
    assert np.array_equal(got_u > 0, ref["phi_u"] > 0)
    e = rel_err(out["phi_total"][0].cpu().numpy(), ref["phi_total"])
    print("fan %s max rel %.2e" % (precision, e), flush=True)
    assert e < (1e-12 if precision == "fp64" else 1e-4)
    h.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_diverging_iteration_reports_numerical_error(precision):
    """Scattering cross sections above the total ones (a supercritical,
    non-physical medium: nothing in the argument checks forbids it) make
    source iteration grow until the fluence overflows; the residual then
    turns non-finite and the call returns DSN_ERR_NUMERICAL instead of
    running to max_iters.  Pure DD, so the face words accept any value."""
    p = random_small_problem(19, n=(9, 8, 10), sn=4, L=0, G=1, n_mat=1, fixup=0, density=False)
    p = type(p)(**{**p.__dict__, "sigma_s": 12.0 * p.sigma_t.reshape(1, 1, 1, 1).copy()})
    s = _source("inside", p, 1)
    h = dsn.Problem(p, precision)
    with pytest.raises(dsn.DsnError) as err:
        h.solve([s], tol=1e-10, max_iters=20000)
    assert err.value.status == dsn.dsn.DSN_ERR_NUMERICAL
    assert "NaN or infinite" in dsn.last_error()
    h.close()


def test_long_mesh_decodes_tickets_from_device_memory():
    """A 2 x 2064 x 8 mesh has 258 pencils along y: 258 pencil diagonals,
    more than a sweep block keeps in LDS, so its tickets are decoded against
    the diagonal table in device memory (binary search).  FP64 with the
    fixup against the oracle at fixed iterations."""
    p = random_small_problem(17, n=(2, 2064, 8), sn=4, L=1, G=2, n_mat=3, fixup=1)
    ext = np.array([p.nx * p.dx, p.ny * p.dy, p.nz * p.dz])
    s = SourceSpec(position=(0.5 * ext[0], -2.0, 0.5 * ext[2]), spectrum=np.array([1.0, 0.4]))
    fixed = [3, 2]
    ref = oracle.solve(p, s, fixed_iters=fixed)["phi_total"]
    h = dsn.Problem(p, "fp64")
    out = h.solve([s], fixed_iters=fixed)
    e = parity_err(out["phi_total"][0].cpu().numpy(), ref, p)
    print("long mesh max rel %.2e" % e, flush=True)
    assert e < 1e-12
    h.close()
