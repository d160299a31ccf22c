#!/usr/bin/env python3
"""Throughput benchmark of the discrete-ordinates hot path on one MI355X.

A step is one converged solve of the workload: ray trace + first-collision
source, then for every energy group source iteration (scattering source,
transport sweep of every direction, moment quadrature, residual) to
convergence, downscatter, output.  The workload is the 128^3 x 0.25 cm
phantom of 12 random ellipsoids over air/tissue/bone/metal, G = 19 groups
(10-120 keV), S16 (288 directions), P5 scattering, cone-beam point source,
FP32 sweeps and contractions with FP64 moments and residual, each group
stopped by the FP32 rule of dsn.CONVERGED (estimated per-voxel error below
1e-5, or the FP32 floor).  Inputs are synthetic and resident on the GPU before timing.

Prints one JSON line (metric: voxel*direction*group updates per second).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MI355X_HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1910_11335_amd", "csrc")
# committed rocprofv3 counter summaries: (summary, kernel source it was taken with)
TRAFFIC_SUMMARY = {"k_sweep": (os.path.join(ROOT, "profiles", "k_sweep_cfg3_fp32.md"), os.path.join(CSRC, "sweep.hip")),
                   "k_d2m": (os.path.join(ROOT, "profiles", "k_d2m_cfg3_fp32.md"), os.path.join(CSRC, "kernels.hip"))}


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from its committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when that
    summary does not cover this workload or the kernel source has changed
    since the counters were taken."""
    import re
    summary, source = TRAFFIC_SUMMARY[kernel]
    if workload != "cfg3" or precision != "fp32" or not os.path.exists(summary):
        return None
    text = open(summary).read()
    t = re.search(r"traffic_bytes_per_launch: ([0-9.eE+]+)", text)
    h = re.search(r"kernel_source_sha256_prefix: ([0-9a-f]+)", text)
    if not t or not h:
        return None
    return float(t.group(1)) if kernel_source_digest(source).startswith(h.group(1)) else None


def kernel_source_digest(path):
    """sha256 of a kernel source file with comments and white space removed,
    so only code changes invalidate the measured traffic."""
    import hashlib
    import re
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    text = re.sub(r"\s+", "", text)
    return hashlib.sha256(text.encode()).hexdigest()


def hbm_stream_leg(torch, gib=4):
    """The measured streaming ceiling: the plain read-only, write-only and
    copy kernels of libhbmstream.so (16 bytes per lane, non-temporal; 65536
    and 262144 workgroups of 256 lanes, the faster kept) over `gib` GiB
    buffers, ten timed launches each (HIP events on the stream)."""
    import ctypes as C
    path = os.path.join(ROOT, "paper_1910_11335_amd", "libhbmstream.so")
    lib = C.CDLL(path)
    lib.hbm_stream_run.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_int,
                                   C.c_void_p, C.POINTER(C.c_float)]
    nb = gib << 30
    a = torch.ones(nb, dtype=torch.uint8, device="cuda")
    b = torch.empty(nb, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    for kind, name, moved in ((0, "read", 1), (1, "write", 1), (2, "copy", 2)):
        best = 0.0
        for blocks in (65536, 262144):
            ms = C.c_float(0.0)
            rc = lib.hbm_stream_run(kind, 1, C.c_void_p(b.data_ptr()), C.c_void_p(a.data_ptr()), nb, blocks, 10,
                                    C.c_void_p(stream), C.byref(ms))
            if rc:
                raise RuntimeError("hbm_stream_run failed (%d)" % rc)
            best = max(best, moved * nb / (ms.value * 1e-3) / 1e9)
        out[name + "_GBs"] = best
    del a, b
    torch.cuda.empty_cache()
    out.update({"bytes": nb, "kernel": "libhbmstream.so: 16 B per lane, non-temporal, 65536 or 262144 x 256 lanes",
                "copy_frac_of_peak": out["copy_GBs"] / MI355X_HBM_PEAK_GBS})
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg3",
                    choices=["cfg1", "cfg2", "cfg3", "cfg4", "cfg5", "table2-coarse", "table2-fine",
                             "table2-coarse-ct", "table2-fine-ct"],
                    help="cfg5: the batched CT workload (three phantoms x --cfg5-sources sources in one "
                         "dsn_solve_batch call), reported against one dsn_solve call per (phantom, source); "
                         "cfg4: the density gradient (forward + adjoint + gradient per step); "
                         "table2-*: the paper's run-time shapes (S6 P0, 90 groups, water cylinder; -ct: 16 "
                         "cone beams acting together in one solve)")
    ap.add_argument("--cfg5-sources", type=int, default=90)
    ap.add_argument("--cfg5-seq-sample", type=int, default=6,
                    help="sources per phantom timed one call each; the sequential time is extrapolated")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fixed-iters", type=int, default=0,
                    help="run exactly this many source iterations per group instead of converging")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run the plain 1 GiB copy kernel of libhbmstream.so twice (the reference kernel for "
                         "the HBM byte counters)")
    ap.add_argument("--hbm-only", action="store_true",
                    help="run only the HBM streaming microbenchmark (read, write, copy) and print its line")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the GPU-FP64 solve and the batched-vs-sequential comparison")
    ap.add_argument("--vs-oracle", action="store_true",
                    help="cfg1 / cfg2 only: also solve with the oracle to convergence (FP64, tol 1e-10; "
                         "minutes at 64^3) and report the GPU results' error against it")
    return ap.parse_args()


def workload_problem(name):
    """(problem, sources, combine) of a single-solve workload: the sources
    act together in one solve when combine is set (the CT ring)."""
    from synthetic.workloads import config1, config2, config3, table2_ct_ring, table2_water
    if name.endswith("-ct"):
        p, _ = table2_water(name.startswith("table2-fine"))
        return p, table2_ct_ring(p), True
    p, s = {"cfg1": config1, "cfg2": config2, "cfg3": config3, "table2-coarse": lambda: table2_water(False),
            "table2-fine": lambda: table2_water(True)}[name]()
    return p, [s], False


def cpu_baseline(workload):
    """The oracle on a bounded sample of the workload.  The 16^3 S4 case is
    small enough for whole converged solves (tol 1e-8, both groups), repeated
    for about 2 s; otherwise: the same mesh, quadrature and scattering order,
    group 0 only, two source iterations (ray trace included), about 15 s on
    16 host threads at 128^3 S16.  The small meshes (16^3, 64^3) are also
    timed on one thread."""
    import numpy as np
    import oracle
    p, srcs, _ = workload_problem(workload)
    s = srcs[0]
    nd = p.sn_order * (p.sn_order + 2)
    if workload == "cfg1":
        oracle.solve(p, s, tol=1e-8)  # warm-up (thread pool)

        def run():
            reps, upd, t0 = 0, 0.0, time.perf_counter()
            while reps == 0 or time.perf_counter() - t0 < 2.0:
                r = oracle.solve(p, s, tol=1e-8)
                upd += float(p.V) * nd * float(np.sum(r["iters"]))
                reps += 1
            return upd, time.perf_counter() - t0, reps

        what = "converged solves (tol 1e-8, G = %d)" % p.G
    else:
        p1 = type(p)(**{**p.__dict__, "sigma_t": p.sigma_t[:, :1].copy(),
                        "sigma_s": p.sigma_s[:, :, :1, :1].copy()})
        s1 = type(s)(**{**s.__dict__, "spectrum": np.asarray(s.spectrum)[:1].copy()})
        iters = 2

        def run():
            t0 = time.perf_counter()
            oracle.solve(p1, s1, fixed_iters=[iters])
            return float(p.V) * nd * iters, time.perf_counter() - t0, 1

        what = "group 0 only, %d source iterations incl. ray trace" % iters
    upd, t, reps = run()
    extra = {}
    if workload in ("cfg1", "cfg2"):
        threads = oracle.num_threads()
        oracle.set_num_threads(1)
        u1, t1, _ = run()
        oracle.set_num_threads(threads)
        extra = {"one_thread": {"value": u1 / t1, "cores": 1, "seconds": t1}}
    return {"value": upd / t, "unit": "voxel*dir*group updates/s", "cores": oracle.num_threads(),
            **extra, "kind": "oracle",
            "sample": "%s mesh, S%d P%d, %s, x%d (%.3g updates), %.1f s; sweep parallel over the 8 octants"
                      % (workload, p.sn_order, p.legendre_order, what, reps, upd, t)}


def max_rel(a, b, floor=1e-6):
    """Largest |a - b| / |b| over voxels with |b| above `floor` of their
    group's maximum (a, b: [G][V] arrays)."""
    import numpy as np
    worst = 0.0
    for g in range(b.shape[0]):
        m = np.abs(b[g]).max()
        if m == 0:
            continue
        sel = np.abs(b[g]) > floor * m
        worst = max(worst, float((np.abs(a[g] - b[g])[sel] / np.abs(b[g][sel])).max()))
    return worst


def rmsd(a, b, floor=1e-6):
    """Root-mean-square relative deviation (the paper's eq. 23 measure) of a
    against b over voxels above `floor` of their group's maximum."""
    import numpy as np
    acc, n = 0.0, 0
    for g in range(b.shape[0]):
        m = np.abs(b[g]).max()
        if m == 0:
            continue
        sel = np.abs(b[g]) > floor * m
        acc += float((((a[g] - b[g])[sel] / b[g][sel]) ** 2).sum())
        n += int(sel.sum())
    return (acc / n) ** 0.5 if n else 0.0


def fp64_leg(dsn, torch, p, s, phi32):
    """The same converged solve on the GPU-FP64 path: seconds per solve and
    the FP32 result's error against it."""
    h = dsn.Problem(p, "fp64")
    kw = dict(max_iters=2000, **dsn.CONVERGED["fp64"])
    h.solve([s], autotune=True, **kw)  # warm-up: allocation, code load, sweep launch shape
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = h.solve([s], **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    phi64 = r["phi_total"][0].cpu().numpy()
    h.close()
    return {"s_per_solve": dt, "updates_per_s": r["updates"] / dt, "iterations": int(r["iters"][0].sum()),
            "tol": 1e-10, "fp32_vs_fp64_max_rel": max_rel(phi32, phi64),
            "fp32_vs_fp64_rmsd": rmsd(phi32, phi64),
            "fp32_vs_fp64_rel_l2": rel_l2(phi32, phi64)}, phi64


def rel_l2(a, b):
    import numpy as np
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def oracle_leg(p, s, results):
    """The oracle's converged FP64 solve (tol 1e-10) of the same problem:
    its wall time and each GPU result's error against it (results: name ->
    [G][V] array)."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    ref = oracle.solve(p, s, tol=1e-10, verbose=True)
    dt = time.perf_counter() - t0
    want = np.asarray(ref["phi_total"]).reshape(p.G, p.V)
    line = {"s_per_solve": dt, "cores": oracle.num_threads(), "iterations": int(np.sum(ref["iters"])), "tol": 1e-10,
            "kind": "oracle"}
    for name, got in results.items():
        line[name] = {"max_rel": max_rel(got, want), "rmsd": rmsd(got, want), "rel_l2": rel_l2(got, want)}
    return line


def batching_leg(dsn, torch, n_src=8):
    """Batching: n_src cone sources around the 48^3 phantom of the batched CT
    workload (S8 P3, G = 19, FP32), one call solving all of them against one
    call per source."""
    from synthetic.workloads import config5_phantoms, config5_sources
    p = config5_phantoms()[0]
    srcs = config5_sources(p, n_src)
    h = dsn.Problem(p, "fp32")
    kw = dict(max_iters=2000, **dsn.CONVERGED["fp32"])
    h.solve(srcs, autotune=True, **kw)  # warm-up: batch buffers, sweep launch shape
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rb = h.solve(srcs, **kw)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    for x in srcs:
        h.solve([x], **kw)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    h.close()
    return {"workload": "48^3 x 0.5 cm phantom, S8 P3, G=19, FP32, %d cone sources on a 50 cm circle" % n_src,
            "batched_s": tb, "sequential_s": ts, "speedup": ts / tb,
            "batched_updates_per_s": rb["updates"] / tb}


def cfg5_line(args, dsn, torch):
    """The batched CT workload: 48^3, 80^3 and 96^3 phantoms (0.5 cm, S8 P3,
    G = 19, FP32), n cone sources each on a 50 cm circle, all solved by one
    dsn_solve_batch call in the fused form (every source iteration one sweep
    launch over all 3n (phantom, source) pairs, its shape autotuned inside
    the timed call).  Beside it: the same call with a stream and host thread
    per phantom (the library's default form, faster on this GPU), and one
    dsn_solve call per (phantom, source), timed on a sample and extrapolated
    to all sources."""
    from synthetic.workloads import config5_phantoms, config5_sources
    probs = config5_phantoms()
    n = args.cfg5_sources
    srcs = [config5_sources(p, n) for p in probs]
    hs = [dsn.Problem(p, "fp32") for p in probs]
    kw = dict(max_iters=2000, **dsn.CONVERGED["fp32"])
    G = probs[0].G
    # untimed: each phantom's own sweep launch shape (the per-phantom streams
    # and the sequential solves use it), then the per-source buffers sized
    # for the batch (both batch forms use the same sizes)
    for h, ss in zip(hs, srcs):
        h.solve(ss, fixed_iters=[1] + [0] * (G - 1), autotune=True)
    dsn.solve_batch(hs, srcs, fixed_iters=[1] + [0] * (G - 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = dsn.solve_batch(hs, srcs, batch_mode=dsn.BATCH_FUSED, autotune=True, **kw)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    rs = dsn.solve_batch(hs, srcs, batch_mode=dsn.BATCH_STREAMS, **kw)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    same = all(torch.equal(x, y) for x, y in zip(r["phi_total"], rs["phi_total"]))
    per = []
    k = max(1, min(args.cfg5_seq_sample, n))
    for h, ss in zip(hs, srcs):
        pick = ss[::max(1, n // k)][:k]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for x in pick:
            h.solve([x], **kw)
        torch.cuda.synchronize()
        per.append((time.perf_counter() - t0) / len(pick))
    seq = sum(x * n for x in per)
    shapes = [h.sweep_tuning() for h in hs]
    for h in hs:
        h.close()
    return {
        "metric": "voxel*dir*group updates/s (converged solves, batched)",
        "value": r["updates"] / tb,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": 1e3 * tb,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cfg5: 48^3, 80^3, 96^3 x 0.5 cm phantoms, S8 (80 dirs), P3, G=19, %d cone sources "
                               "each, converged (FP32 rule: estimated per-voxel error < 1e-5), one dsn_solve_batch call, "
                               "fused: one sweep launch per source iteration over all (phantom, source) pairs" % n,
                   "solves": 3 * n,
                   "source_iterations": int(r["iters"].sum()),
                   "fused_sweep_shape": list(r["sweep_shape"])},
        "roofline": None,
        "batched_s": tb,
        "streams": {"s": ts, "updates_per_s": rs["updates"] / ts, "same_result_as_fused": same,
                    "speedup_vs_sequential": seq / ts,
                    "kind": "dsn_solve_batch with a stream and host thread per phantom (default batch form)",
                    "sweep_shape_per_phantom": [min((t for t in x if t[4] > 0), key=lambda t: t[4])[:4] if x else None
                                                for x in shapes]},
        "sequential": {"s_extrapolated": seq, "s_per_solve_by_phantom": per, "sample_per_phantom": k,
                       "kind": "one dsn_solve call per (phantom, source), timed on a sample, extrapolated"},
        "speedup_vs_sequential": seq / tb,
        "speedup_vs_streams": ts / tb,
    }


def cfg4_line(args, dsn, torch):
    """The differentiation workload: 64^3 x 0.5 cm, 6 ellipsoids, density ~
    U(0.8, 1.2), G = 10, S8 P3, fixup off, exit-face detector loss.  A step
    is one gradient: forward solve, adjoint solve and the density gradient
    (checkpointed recomputation), converged."""
    from synthetic.workloads import config4, detector_weights
    p, s = config4()
    W = torch.tensor(detector_weights(p), device="cuda")
    h = dsn.Problem(p, args.precision)
    tol = 1e-6 if args.precision == "fp32" else 1e-10
    h.adjoint(s, W, tol=tol)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates = 0.0
    for _ in range(args.steps):
        r = h.adjoint(s, W, tol=tol)
        updates += r["updates"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    h.close()
    return {
        "metric": "voxel*dir*group updates/s (forward + adjoint solve and density gradient)",
        "value": updates / dt, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": "cfg4: 64x64x64 voxels, S8 (80 dirs), P3, G=10, density gradient of an exit-face "
                               "detector loss, tol %g" % tol,
                   "iterations_forward": [int(x) for x in r["iters"][0]],
                   "iterations_adjoint": [int(x) for x in r["iters"][1]]},
        "roofline": None,
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU only (the solve is single-GPU); "
              "got --gpus %d, WORLD_SIZE %d" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1910_11335_amd as dsn
    torch.cuda.set_device(0)
    if args.hbm_only:
        print(json.dumps({"metric": "HBM streaming bandwidth (plain kernels)", "unit": "GB/s",
                          "peak": MI355X_HBM_PEAK_GBS, **hbm_stream_leg(torch)}), flush=True)
        return
    if args.workload == "cfg5":
        print(json.dumps(cfg5_line(args, dsn, torch)), flush=True)
        return
    if args.workload == "cfg4":
        print(json.dumps(cfg4_line(args, dsn, torch)), flush=True)
        return
    if args.calibrate_copy:
        # the plain copy kernel of libhbmstream.so over 1 GiB (one untimed and
        # one timed launch): the reference for the HBM byte counters
        import ctypes as C
        lib = C.CDLL(os.path.join(ROOT, "paper_1910_11335_amd", "libhbmstream.so"))
        lib.hbm_stream_run.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_int,
                                       C.c_void_p, C.POINTER(C.c_float)]
        src_buf = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        dst_buf = torch.empty_like(src_buf)
        ms = C.c_float(0.0)
        if lib.hbm_stream_run(2, 1, C.c_void_p(dst_buf.data_ptr()), C.c_void_p(src_buf.data_ptr()), 1 << 30, 65536,
                              1, C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(ms)):
            raise RuntimeError("calibration copy failed")
        torch.cuda.synchronize()
        del src_buf, dst_buf
    p, srcs, combine = workload_problem(args.workload)
    s = srcs[0]
    h = dsn.Problem(p, args.precision)
    kw = dict(max_iters=2000, **dsn.CONVERGED[args.precision])
    if args.fixed_iters:
        kw = dict(fixed_iters=[args.fixed_iters] * p.G)
    out = torch.empty((1, p.G, p.V), dtype=torch.float64, device="cuda")
    # untimed: time the sweep's launch shapes on group 0's first source iteration
    tuned = h.solve(srcs, out=out, fixed_iters=[1] + [0] * (p.G - 1), autotune=True, combine=combine)
    for _ in range(args.warmup):
        h.solve(srcs, out=out, combine=combine, **kw)
    torch.cuda.synchronize()
    updates = 0.0
    stage_ms = {}
    launches = {}
    sweep_bytes = 0.0
    iters = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = h.solve(srcs, out=out, profile=True, combine=combine, **kw)
        updates += r["updates"]
        sweep_bytes += r["sweep_bytes"]
        iters = r["iters"][0]
        for k, v in r["stages"].items():
            stage_ms[k] = stage_ms.get(k, 0.0) + v["ms"]
            launches[k] = launches.get(k, 0) + v["launches"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same solves with the steady iterations replayed as HIP graphs (no
    # stage timer): reported beside the timed steps, not in `value`
    t1 = time.perf_counter()
    for _ in range(args.steps):
        h.solve(srcs, out=out, combine=combine, **kw)
    torch.cuda.synchronize()
    dt_graphs = time.perf_counter() - t1
    sweep_s = stage_ms["sweep"] / 1e3
    traffic = measured_traffic("k_sweep", args.workload, args.precision)
    achieved = sweep_bytes / sweep_s / 1e9 if sweep_s > 0 else 0.0
    # k_d2m (moments, residual partials and the next directional source),
    # timed with its residual kernel (k_resid, about 1 % of the pair)
    ts = 4 if args.precision == "fp32" else 8
    nm, nd = (p.legendre_order + 1) ** 2, p.sn_order * (p.sn_order + 2)
    vp = ((p.ny + 7) // 8) * ((p.nz + 7) // 8) * p.nx * 64
    d2m_bpv = 2 * nd * ts + nm * (ts + 8) + 8 + (8 if kw.get("stop_rule") == 1 else 0)
    d2m_iters = launches["d2m"] // 2
    d2m_ms = stage_ms["d2m"] / max(1, d2m_iters)
    d2m_gb = d2m_bpv * vp / 1e9
    d2m_traffic = measured_traffic("k_d2m", args.workload, args.precision)
    line = {
        "metric": "voxel*dir*group updates/s (converged solve)",
        "value": updates / dt,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "ms_per_step_graph_replays": 1e3 * dt_graphs / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %dx%dx%d voxels, S%d (%d dirs), P%d, G=%d, %s, %s" % (
            args.workload, p.nx, p.ny, p.nz, p.sn_order, p.sn_order * (p.sn_order + 2), p.legendre_order, p.G,
            "%d cone beams in one solve" % len(srcs) if combine else
            "cone source" if s.half_angle < np.pi else "isotropic point source", "fixed %d iters/group" % args.fixed_iters if args.fixed_iters else "converged"),
            "source_iterations_per_group": [int(x) for x in iters],
            "stage_ms_per_step": {k: v / args.steps for k, v in stage_ms.items()},
            "launches_per_step": {k: v // args.steps for k, v in launches.items()},
            "sweep_shape": {"waves_per_block": tuned["sweep_shape"][0], "blocks": tuned["sweep_shape"][1],
                            "xcd_queues": tuned["sweep_shape"][2], "relay": tuned["sweep_shape"][3],
                            "timed_ms": {"%dx%d%s" % (w, b, "/xcd" if x else "/relay%d" % r if r else ""): round(ms, 4)
                                         for w, b, x, r, ms in h.sweep_tuning()}}},
        "roofline": {"kernel": "k_sweep", "bound": "hbm", "achieved": achieved, "peak": MI355X_HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / MI355X_HBM_PEAK_GBS,
                     "traffic": traffic / 1e9 if traffic else None, "traffic_unit": "GB per launch (HBM)",
                     "algorithmic_GB_per_launch": sweep_bytes / max(1, launches["sweep"]) / 1e9,
                     "avg_launch_ms": stage_ms["sweep"] / max(1, launches["sweep"]),
                     "bytes_per_update": 2 * (4 if args.precision == "fp32" else 8)},
        "roofline_d2m": {"kernel": "k_d2m", "bound": "hbm", "achieved": d2m_gb / d2m_ms * 1e3 if d2m_ms > 0 else 0.0,
                         "peak": MI355X_HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": d2m_gb / d2m_ms * 1e3 / MI355X_HBM_PEAK_GBS if d2m_ms > 0 else 0.0,
                         "traffic": d2m_traffic / 1e9 if d2m_traffic else None,
                         "traffic_unit": "GB per launch (HBM)", "algorithmic_GB_per_launch": d2m_gb,
                         "avg_launch_ms": d2m_ms, "bytes_per_voxel": d2m_bpv,
                         "note": "read psi and F, write the FP64 moments and the next Q, old phi_00 (and phi_u "
                                 "for the pointwise stop); time includes k_resid"},
    }
    results = {}
    if not args.fixed_iters:
        results["gpu_" + args.precision] = out[0].cpu().numpy()
    if not args.no_extras and not args.fixed_iters and args.precision == "fp32":
        phi32 = results["gpu_fp32"]
        line["fp32_s_per_solve"] = dt / args.steps
        h.close()
        def leg(name, fn):
            # an extra leg that fails is reported in the line, with its error,
            # and does not cost the main measurement
            try:
                line[name] = fn()
            except dsn.DsnError as e:
                line[name] = {"error": str(e)}
                print("bench: %s failed: %s" % (name, e), file=sys.stderr, flush=True)

        def fp64():
            out, results["gpu_fp64"] = fp64_leg(dsn, torch, p, s, phi32)
            return out

        def batched_ct():
            cfg = cfg5_line(args, dsn, torch)
            return {k: cfg[k] for k in ("metric", "value", "unit", "ms_per_step", "config", "batched_s", "streams",
                                        "sequential", "speedup_vs_sequential", "speedup_vs_streams")}

        leg("fp64", fp64)
        leg("batching", lambda: batching_leg(dsn, torch))
        if args.workload == "cfg3":
            leg("batched_ct", batched_ct)
        line["hbm_stream"] = hbm_stream_leg(torch)
    if args.vs_oracle and results:
        if args.workload not in ("cfg1", "cfg2"):
            raise SystemExit("--vs-oracle is for the cfg1 and cfg2 workloads (the oracle takes minutes at 64^3)")
        line["vs_oracle"] = oracle_leg(p, s, results)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload)
    h.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
