"""Batched solves (many sources, uneven phantoms) through the C ABI."""
import numpy as np
import pytest

import oracle
from synthetic.workloads import (ProblemSpec, SourceSpec, cone_source, ellipsoid_phantom, kramers_spectrum,
                                 water_cylinder, xs_tables)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
dsn = pytest.importorskip("paper_1910_11335_amd")


def _phantom(n, seed, G=3, L=1, sn=4, fixup=1):
    d = 0.5
    mat = ellipsoid_phantom(seed, (n, n, n), d, 5, [0, 1, 2, 3])
    st, ss = xs_tables(seed, G, ["air", "tissue", "bone", "metal"], L)
    return ProblemSpec(n, n, n, d, d, d, mat, None, st, ss, sn, L, fixup=fixup, name="phantom%d" % n)


def _ring(p, k, G):
    c = (p.nx * p.dx / 2, p.ny * p.dy / 2, p.nz * p.dz / 2)
    spec = kramers_spectrum(G)
    return [cone_source(c, 12.0, 2 * np.pi * s / k + 0.1, 40.0, spec) for s in range(k)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_sources_equal_separate_solves(precision):
    p = _phantom(20, 11)
    srcs = _ring(p, 5, p.G)
    h = dsn.Problem(p, precision)
    tol = 1e-10 if precision == "fp64" else 1e-6
    batch = h.solve(srcs, tol=tol, stagnation_stop=precision == "fp32")
    for i, s in enumerate(srcs):
        one = h.solve([s], tol=tol, stagnation_stop=precision == "fp32")
        assert list(one["iters"][0]) == list(batch["iters"][i])
        assert torch.equal(one["phi_total"][0], batch["phi_total"][i])
    h.close()


@pytest.mark.parametrize("mode", ["streams", "fused"])
def test_solve_batch_uneven_phantoms_matches_oracle(mode):
    probs = [_phantom(n, 20 + n) for n in (9, 16, 21)]
    srcs = [_ring(p, 3, p.G) for p in probs]
    handles = [dsn.Problem(p, "fp64") for p in probs]
    fixed = [3] * probs[0].G
    bm = dsn.BATCH_STREAMS if mode == "streams" else dsn.BATCH_FUSED
    out = dsn.solve_batch(handles, srcs, fixed_iters=fixed, batch_mode=bm)
    for b, (p, h) in enumerate(zip(probs, handles)):
        sep = h.solve(srcs[b], fixed_iters=fixed)["phi_total"]
        assert torch.equal(sep, out["phi_total"][b])
        ref = oracle.solve(p, srcs[b][1], fixed_iters=fixed)["phi_total"]
        got = out["phi_total"][b][1].cpu().numpy()
        m = np.abs(ref).max(axis=1, keepdims=True)
        sel = np.abs(ref) > 1e-6 * m
        assert (np.abs(got - ref)[sel] / np.abs(ref[sel])).max() < 1e-12
    for h in handles:
        h.close()


def test_solve_batch_with_per_xcd_queues_on_concurrent_streams():
    """FP32 with the fixup, S8 (10 directions per octant): the three uneven
    phantoms pinned to per-XCD-queue sweep shapes (their sweeps then run
    concurrently on different streams, each launch's blocks serving the
    queue of the XCD they land on) give the same fluence, bit for bit, as
    the default shape solving each phantom alone."""
    probs = [_phantom(n, 40 + n, L=3, sn=8) for n in (11, 17, 24)]
    srcs = [_ring(p, 3, p.G) for p in probs]
    fixed = [3] * probs[0].G
    refs = []
    for p, ss in zip(probs, srcs):
        h = dsn.Problem(p, "fp32")
        refs.append(h.solve(ss, fixed_iters=fixed)["phi_total"])
        h.close()
    handles = [dsn.Problem(p, "fp32") for p in probs]
    nq = handles[0].xcd_queues()
    if nq == 0:
        pytest.skip("the device probe saw no round-robin workgroup placement: no per-XCD queues")
    for h, (w, b) in zip(handles, [(1, nq), (2, 520), (2, 1024)]):
        h.set_sweep_shape(w, b, nq)
    for rep in range(2):
        out = dsn.solve_batch(handles, srcs, fixed_iters=fixed, batch_mode=dsn.BATCH_STREAMS)
        for b in range(len(probs)):
            assert torch.equal(out["phi_total"][b], refs[b]), (rep, b)
    for h in handles:
        h.close()


def test_opposite_sources_give_rotated_fluence():
    """A z-axis cylinder is invariant under the 180 degree rotation about its
    axis; the level-symmetric set and the DD scheme are too, so sources at
    theta and theta + pi give fluences related by (i, j) -> (nx-1-i, ny-1-j)."""
    n, d, G = 24, 0.5, 3
    mat = water_cylinder((n, n, n), d, 5.0, 9.0)
    st, ss = xs_tables(7, G, ["air", "tissue"], 1)
    p = ProblemSpec(n, n, n, d, d, d, mat, None, st, ss, 4, 1, fixup=1)
    c = (n * d / 2,) * 3
    spec = kramers_spectrum(G)
    a = cone_source(c, 15.0, 0.3, 30.0, spec)
    b = cone_source(c, 15.0, 0.3 + np.pi, 30.0, spec)
    h = dsn.Problem(p, "fp64")
    out = h.solve([a, b], tol=1e-11)["phi_total"].cpu().numpy().reshape(2, G, n, n, n)
    rot = out[0][:, :, ::-1, ::-1]
    assert np.abs(out[1] - rot).max() < 1e-12 * np.abs(out[0]).max()
    h.close()


def _ct_ring(p, k, G):
    """k cone beams of 30 degrees (full apex) on a ring around the phantom,
    the CT mode of the paper (section II.D)."""
    c = (p.nx * p.dx / 2, p.ny * p.dy / 2, p.nz * p.dz / 2)
    spec = kramers_spectrum(G)
    return [cone_source(c, 11.0, 2 * np.pi * s / k + 0.05, 30.0, spec) for s in range(k)]


def test_combined_ct_ring_equals_sum_of_oracle_solves():
    """Sources acting together in one solve (combine_sources) against the sum
    of the oracle's single-source solves.  With the fixup off and the same
    iteration counts, source iteration is linear in the source, so the sum is
    exact up to rounding: GPU-FP64 within 1e-12, the uncollided part too."""
    p = _phantom(14, 31, fixup=0)
    srcs = _ct_ring(p, 6, p.G)
    fixed = [3] * p.G
    h = dsn.Problem(p, "fp64")
    out = h.solve(srcs, fixed_iters=fixed, combine=True, uncollided=True)
    assert out["phi_total"].shape == (1, p.G, p.V) and out["iters"].shape == (1, p.G)
    refs = [oracle.solve(p, s, fixed_iters=fixed) for s in srcs]
    want = sum(r["phi_total"] for r in refs)
    want_u = sum(r["phi_u"] for r in refs)
    got = out["phi_total"][0].cpu().numpy()
    got_u = out["phi_u"][0].cpu().numpy()
    for g, w in zip((got, got_u), (want, want_u)):
        m = np.abs(w).max(axis=1, keepdims=True)
        sel = np.abs(w) > 1e-6 * m
        assert (np.abs(g - w)[sel] / np.abs(w[sel])).max() < 1e-12
    h.close()


def test_combined_ct_ring_fp32_and_fixup():
    """FP32 combined solve against the FP64 one (1e-4 over voxels above 1e-6
    of the group maximum), fixup on, converged."""
    p = _phantom(16, 32, fixup=1)
    srcs = _ct_ring(p, 8, p.G)
    h64 = dsn.Problem(p, "fp64")
    h32 = dsn.Problem(p, "fp32")
    r64 = h64.solve(srcs, tol=1e-10, combine=True)["phi_total"][0].cpu().numpy()
    r32 = h32.solve(srcs, tol=1e-6, stagnation_stop=True, combine=True)["phi_total"][0].cpu().numpy()
    m = np.abs(r64).max(axis=1, keepdims=True)
    sel = np.abs(r64) > 1e-6 * m
    assert (np.abs(r32 - r64)[sel] / np.abs(r64[sel])).max() < 1e-4
    h64.close()
    h32.close()


def test_dose_matches_oracle():
    """Absorbed dose (dsn_dose) against the oracle's: on given fluences
    (random, 3 sets) and end to end from an FP64 solve against the oracle's
    solve, both within 1e-12 relative."""
    from synthetic.workloads import dose_factors
    p = _phantom(12, 41)
    k = dose_factors(p.G, ["air", "tissue", "bone", "metal"])
    h = dsn.Problem(p, "fp64")
    rng = np.random.default_rng(5)
    phi = rng.uniform(0.0, 1.0, (3, p.G, p.V))
    got = h.dose(torch.from_numpy(phi).cuda(), k).cpu().numpy()
    want = oracle.dose(p, phi, k)
    assert (np.abs(got - want) / np.abs(want)).max() < 1e-12
    s = _ring(p, 1, p.G)[0]
    fixed = [3] * p.G
    phit = h.solve([s], fixed_iters=fixed)["phi_total"]
    got = h.dose(phit[0], k).cpu().numpy()
    want = oracle.dose(p, oracle.solve(p, s, fixed_iters=fixed)["phi_total"], k)
    sel = want > 1e-6 * want.max()
    assert (np.abs(got - want)[sel] / want[sel]).max() < 1e-12
    h.close()


def test_config5_phantoms_batched_against_oracle():
    """The batched CT workload's three phantoms (48^3, 80^3, 96^3 x 0.5 cm,
    S8 P3, G = 19, FP32) in one dsn_solve_batch call with two sources each
    (0 and 180 degrees on the 50 cm ring), one source iteration per group,
    a stream per phantom and fused (equal bit for bit);
    the 48^3 phantom's two sources and the 80^3 phantom's first against the
    FP64 oracle (1e-4 over voxels above 1e-6 of the group maximum), the 96^3
    phantom's against a separate dsn_solve call (bit for bit)."""
    import time
    from synthetic.workloads import config5_phantoms, config5_sources
    probs = config5_phantoms()
    srcs = [[config5_sources(p, 90)[0], config5_sources(p, 90)[45]] for p in probs]
    handles = [dsn.Problem(p, "fp32") for p in probs]
    fixed = [1] * probs[0].G
    out = dsn.solve_batch(handles, srcs, fixed_iters=fixed)
    alone = handles[2].solve(srcs[2], fixed_iters=fixed)["phi_total"]
    assert torch.equal(alone, out["phi_total"][2])
    # the fused form (one sweep launch over all six (phantom, source) pairs) gives the same bits
    fused = dsn.solve_batch(handles, srcs, fixed_iters=fixed, batch_mode=dsn.BATCH_FUSED, autotune=True)
    for b in range(3):
        assert torch.equal(fused["phi_total"][b], out["phi_total"][b]), b
    checks = [(0, 0), (0, 1), (1, 0)]
    for b, k in checks:
        t0 = time.perf_counter()
        ref = oracle.solve(probs[b], srcs[b][k], fixed_iters=fixed)["phi_total"]
        got = out["phi_total"][b][k].cpu().numpy()
        m = np.abs(ref).max(axis=1, keepdims=True)
        sel = np.abs(ref) > 1e-6 * m
        e = (np.abs(got - ref)[sel] / np.abs(ref[sel])).max()
        print("phantom %d^3 source %d: max rel %.2e (oracle %.1f s)" % (probs[b].nx, k, e,
                                                                       time.perf_counter() - t0), flush=True)
        assert e < 1e-4
    for h in handles:
        h.close()


def test_more_sources_than_one_batch_holds():
    """70 sources on a small mesh: the library advances them in batches of
    at most 64 (here 64 + 6); every result equals its own single-source
    solve bit for bit, the iteration counts included."""
    p = _phantom(10, 51, G=2)
    srcs = _ring(p, 70, p.G)
    h = dsn.Problem(p, "fp32")
    out = h.solve(srcs, tol=1e-6, stagnation_stop=True)
    assert out["phi_total"].shape == (70, p.G, p.V)
    for i in (0, 1, 63, 64, 69):
        one = h.solve([srcs[i]], tol=1e-6, stagnation_stop=True)
        assert list(one["iters"][0]) == list(out["iters"][i])
        assert torch.equal(one["phi_total"][0], out["phi_total"][i])
    h.close()


def test_beam_missing_the_mesh_gives_zero_fluence():
    """A cone aimed away from the phantom: no voxel is lit, the first-collision
    source is zero, the residual is 0/0 := 0, every group stops after one
    iteration and the fluence is exactly zero (no NaN)."""
    p = _phantom(8, 52)
    c = (p.nx * p.dx / 2, p.ny * p.dy / 2, p.nz * p.dz / 2)
    s = SourceSpec(position=(c[0] + 30.0, c[1], c[2]), axis=(1.0, 0.0, 0.0), half_angle=np.deg2rad(10.0),
                   spectrum=kramers_spectrum(p.G))
    for prec in ("fp64", "fp32"):
        h = dsn.Problem(p, prec)
        out = h.solve([s], tol=1e-8)
        assert out["status"] == 0 and (out["iters"] == 1).all()
        assert torch.count_nonzero(out["phi_total"]).item() == 0
        h.close()


def test_solve_batch_with_column_relay_shapes():
    """FP32 with the fixup, S8: the three uneven phantoms pinned to
    column-relay sweep shapes, batched on concurrent streams, give the same
    fluence bit for bit as the default shape solving each phantom alone."""
    probs = [_phantom(n, 50 + n, L=3, sn=8) for n in (11, 17, 24)]
    srcs = [_ring(p, 3, p.G) for p in probs]
    fixed = [3] * probs[0].G
    refs = []
    for p, ss in zip(probs, srcs):
        h = dsn.Problem(p, "fp32")
        refs.append(h.solve(ss, fixed_iters=fixed)["phi_total"])
        h.close()
    handles = [dsn.Problem(p, "fp32") for p in probs]
    for h, (w, b, r) in zip(handles, [(1, 7, 2), (2, 300, 2), (1, 1024, 4)]):
        h.set_sweep_shape(w, b, 0, r)
    for rep in range(2):
        out = dsn.solve_batch(handles, srcs, fixed_iters=fixed, batch_mode=dsn.BATCH_STREAMS)
        for b in range(len(probs)):
            assert torch.equal(out["phi_total"][b], refs[b]), (rep, b)
    for h in handles:
        h.close()


@pytest.mark.parametrize("precision,fixup", [("fp64", 0), ("fp32", 1), ("fp32", 0)])
def test_fused_batch_equals_separate_solves(precision, fixup):
    """One fused sweep launch per source iteration over every (phantom,
    source) pair: three uneven phantoms (one with no sources) with 3, 1 and 2
    sources, converged in the precision's rule, give the iteration counts
    and the fluence of separate dsn_solve calls bit for bit; twice in a row
    (the second call reuses the handles' buffers and face words)."""
    probs = [_phantom(n, 60 + n, L=2, sn=6, fixup=fixup) for n in (13, 10, 22, 17)]
    srcs = [_ring(probs[0], 3, probs[0].G), [], _ring(probs[2], 1, probs[2].G), _ring(probs[3], 2, probs[3].G)]
    rule = dsn.CONVERGED[precision]
    refs, counts = [], []
    for p, ss in zip(probs, srcs):
        if not ss:
            refs.append(None)
            counts.append(None)
            continue
        h = dsn.Problem(p, precision)
        r = h.solve(ss, **rule)
        refs.append(r["phi_total"])
        counts.append(r["iters"])
        h.close()
    handles = [dsn.Problem(p, precision) for p in probs]
    for rep in range(2):
        out = dsn.solve_batch(handles, srcs, batch_mode=dsn.BATCH_FUSED, **rule)
        assert out["sweep_shape"][0] > 0 and out["sweep_shape"][1] > 0
        row = 0
        for b in range(len(probs)):
            if not srcs[b]:
                assert out["phi_total"][b].shape[0] == 0
                continue
            k = len(srcs[b])
            assert (out["iters"][row:row + k] == counts[b]).all(), (rep, b)
            assert torch.equal(out["phi_total"][b], refs[b]), (rep, b)
            row += k
    for h in handles:
        h.close()


def test_fused_batch_autotune_and_later_single_solves():
    """FP32 pure DD (stamped face words, whose stamps come from the batch's
    own counter block): the fused batch with its launch shape autotuned
    gives the separate solves' fluence bit for bit, reports a shape it timed,
    and a single solve on the same handles afterwards is unchanged (the batch
    leaves face words that the next single sweep must not accept)."""
    probs = [_phantom(n, 70 + n, L=1, sn=8, fixup=0) for n in (9, 20, 14)]
    srcs = [_ring(p, 2, p.G) for p in probs]
    fixed = [4] * probs[0].G
    handles = [dsn.Problem(p, "fp32") for p in probs]
    refs = [h.solve(ss, fixed_iters=fixed)["phi_total"].clone() for h, ss in zip(handles, srcs)]
    out = dsn.solve_batch(handles, srcs, fixed_iters=fixed, batch_mode=dsn.BATCH_FUSED, autotune=True)
    assert out["sweep_shape"][0] in (1, 2, 5) and out["sweep_shape"][1] > 0
    for b in range(len(probs)):
        assert torch.equal(out["phi_total"][b], refs[b]), b
    for b, (h, ss) in enumerate(zip(handles, srcs)):
        assert torch.equal(h.solve(ss, fixed_iters=fixed)["phi_total"], refs[b]), b
    for h in handles:
        h.close()


def test_fused_batch_needs_one_cell_mode():
    """Problems that differ in the fixup cannot share a sweep launch:
    batch_mode FUSED is refused before any device work; the default runs them
    on a stream each, with the separate solves' results."""
    probs = [_phantom(11, 81, fixup=1), _phantom(12, 82, fixup=0)]
    srcs = [_ring(p, 2, p.G) for p in probs]
    fixed = [2] * probs[0].G
    handles = [dsn.Problem(p, "fp64") for p in probs]
    refs = [h.solve(ss, fixed_iters=fixed)["phi_total"].clone() for h, ss in zip(handles, srcs)]
    with pytest.raises(dsn.DsnError) as e:
        dsn.solve_batch(handles, srcs, fixed_iters=fixed, batch_mode=dsn.BATCH_FUSED)
    assert "fixup" in str(e.value)
    out = dsn.solve_batch(handles, srcs, fixed_iters=fixed)
    assert out["sweep_shape"] == (0, 0)
    for b in range(2):
        assert torch.equal(out["phi_total"][b], refs[b]), b
    for h in handles:
        h.close()


def test_fused_batch_with_more_segments_than_lds_holds():
    """Eight meshes of 40 pencils along y and one along z (40 pencil
    diagonals each): the fused launch's ticket order has 320 segments, more
    than its blocks keep in LDS, so tickets are decoded against the table in
    device memory.  FP32 with the fixup, bit for bit equal to the separate
    solves."""
    from synthetic.workloads import random_small_problem
    probs = [random_small_problem(90 + q, n=(2 + q, 320, 8), sn=4, L=1, G=2, n_mat=3, fixup=1) for q in range(8)]
    srcs = []
    for p in probs:
        ext = (p.nx * p.dx, p.ny * p.dy, p.nz * p.dz)
        srcs.append([SourceSpec(position=(-3.0, 0.3 * ext[1], 0.5 * ext[2]), spectrum=np.array([1.0, 0.5]))])
    fixed = [2, 2]
    refs = []
    for p, ss in zip(probs, srcs):
        h = dsn.Problem(p, "fp32")
        refs.append(h.solve(ss, fixed_iters=fixed)["phi_total"])
        h.close()
    handles = [dsn.Problem(p, "fp32") for p in probs]
    out = dsn.solve_batch(handles, srcs, fixed_iters=fixed, batch_mode=dsn.BATCH_FUSED)
    for b in range(len(probs)):
        assert torch.equal(out["phi_total"][b], refs[b]), b
    for h in handles:
        h.close()
