"""Writes the converged-solve goldens of the full-size workloads.

Each file tests/golden/converged_<case>.npz holds what the FP64 oracle (and
nothing else) computes for one workload of synthetic/workloads.py, solved by
source iteration until the relative L2 change of the collided scalar fluence
of every group drops below 1e-10 (the GPU-FP64 stopping rule):
  iters [G]     source iterations per group
  idx   [K]     sampled voxels (natural order v = i + nx (j + ny k)), drawn
                uniformly without replacement from a fixed seed
  phi   [G][K]  total fluence (uncollided + collided) at those voxels
  gmax  [G]     largest |total fluence| of each group over the whole mesh
  sc    [G][K]  the sampled voxel's fluence differs in sign from a face
                neighbour's (pure diamond difference can go negative; the
                parity measure treats such voxels apart)
  nneg  [G]     voxels of the whole mesh with negative fluence
  phi_single [G][K]  pure diamond difference only: the same solve (the same
                iteration counts) with every DD cell in single precision, at
                the sampled voxels - how far single-precision rounding alone
                moves the solution there
  info          a text line: case, tolerance, threads, seconds
The meshes are too large to store whole; the parity tests compare the GPU
solve at the sampled voxels.

Usage: python tests/golden/make_converged.py CASE [--threads T]
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synthetic import workloads as wl  # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from parity import sign_change_voxels  # noqa: E402

TOL = 1e-10


def _cfg5_48():
    p = wl.config5_phantoms()[0]
    return p, wl.config5_sources(p)[0]


CASES = {
    # name: (problem and source, sampled voxels)
    "cfg2": (wl.config2, 8192),
    "cfg3": (wl.config3, 8192),
    "cfg4": (wl.config4, 8192),
    "cfg5_48": (_cfg5_48, 8192),
    "table2_coarse": (lambda: wl.table2_water(False), 2048),
}


def path_of(case):
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "converged_%s.npz" % case)


def make(case, threads):
    build, k = CASES[case]
    p, s = build()
    if threads:
        oracle.set_num_threads(threads)
    t0 = time.time()
    ref = oracle.solve(p, s, tol=TOL, verbose=True)
    dt = time.time() - t0
    if ref["status"] != oracle.OK:
        raise SystemExit("oracle did not converge (status %d)" % ref["status"])
    phi = ref["phi_total"]
    rng = np.random.default_rng(7700)
    idx = np.sort(rng.choice(p.V, size=min(k, p.V), replace=False)).astype(np.int64)
    info = "case %s (%s), oracle FP64, relative L2 change of phi_00 < %g, %d threads, %.0f s" % (
        case, p.name, TOL, oracle.num_threads(), dt)
    sc = np.stack([sign_change_voxels(phi[g], (p.nx, p.ny, p.nz))[idx] for g in range(p.G)])
    extra = {}
    if not p.fixup:
        single = oracle.solve(p, s, fixed_iters=ref["iters"], cell_single=True)["phi_total"]
        extra["phi_single"] = np.ascontiguousarray(single[:, idx])
    np.savez_compressed(path_of(case), iters=ref["iters"].astype(np.int32), idx=idx,
                        phi=np.ascontiguousarray(phi[:, idx]), gmax=np.abs(phi).max(axis=1), sc=sc,
                        nneg=(phi < 0).sum(axis=1).astype(np.int64), info=np.array(info), **extra)
    print(info, "iters", ref["iters"].tolist(), flush=True)


def load(case):
    """The stored golden as a dict (no pickled objects)."""
    with np.load(path_of(case), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=sorted(CASES))
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    make(a.case, a.threads)
