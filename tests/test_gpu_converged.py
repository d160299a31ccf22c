"""Converged full-size solves against the FP64 oracle's converged solution.

The oracle's solutions of the full-size workloads take minutes to hours on
the host, so they are stored: tests/golden/converged_<case>.npz, written by
tests/golden/make_converged.py (which calls only the oracle): iteration
counts of the FP64 rule (relative L2 change below 1e-10), total fluence at a
fixed random sample of voxels and every group's largest |fluence|.

Each workload runs in the launch configuration the benchmark times (sweep
shape picked by the autotune) with the stopping rules of dsn.CONVERGED:
  GPU-FP64: the oracle's iteration count in every group, then every sampled
            voxel above 1e-6 of its group's maximum within 1e-12;
  FP32:     every such voxel within 1e-4, or, for the pure diamond-difference
            workload, within 4 times what single-precision cells alone
            (the oracle's model, stored in the golden) move that voxel;
voxels next to a sign change of a pure diamond-difference fluence against
their group's maximum (tests/parity.py).
"""
import os
import sys

import numpy as np
import pytest

from parity import sampled_fp32_excess, sampled_rel_err
from synthetic import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
dsn = pytest.importorskip("paper_1910_11335_amd")

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_converged  # noqa: E402


def _workload(case):
    return make_converged.CASES[case][0]()


CASES = ["cfg2", "cfg3", "cfg4", "cfg5_48", "table2_coarse"]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES)
def test_converged_full_size(case, precision):
    if not os.path.exists(make_converged.path_of(case)):
        pytest.skip("golden %s not written" % case)
    gold = make_converged.load(case)
    p, s = _workload(case)
    h = dsn.Problem(p, precision)
    rule = dsn.CONVERGED[precision]
    out = h.solve([s], autotune=True, max_iters=2000, **rule)
    got = out["phi_total"][0].cpu().numpy()
    e, n, e_sc = sampled_rel_err(got, gold)
    print("%s %s: iters %s (oracle %s), max err %.3e over %d sampled voxels (%.3e at voxels next to a sign "
          "change, %d negative in the oracle), shape %s" % (
              case, precision, out["iters"][0].tolist(), gold["iters"].tolist(), e, n, e_sc,
              int(gold["nneg"].sum()), out["sweep_shape"]), flush=True)
    assert np.isfinite(got).all()
    # the whole-mesh maxima agree too (the sample may miss a group's peak)
    gm = np.abs(got).max(axis=1)
    gm_err = float(np.max(np.abs(gm - gold["gmax"]) / gold["gmax"]))
    if precision == "fp64":
        assert list(out["iters"][0]) == list(gold["iters"])
        assert e < 1e-12 and gm_err < 1e-12
    else:
        x, _, n_wide = sampled_fp32_excess(got, gold)
        print("   fp32 error / allowance %.3f (%d voxels where the single-precision model allows more than 1e-4)"
              % (x, n_wide), flush=True)
        assert x < 1.0 and gm_err < 1e-4
    h.close()
