"""Builds libdsn.so (HIP for gfx950 + host C++) in-tree with hipcc."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libdsn.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["kernels.hip", "sweep.hip", "runtime.hip", "quadrature.cpp"]
# no packed FP32 instructions anywhere in the device code
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose=False, jobs=None):
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmd = [HIPCC] + COMMON
        if src.endswith(".hip"):
            cmd += DEVICE_FLAGS + ["-x", "hip"]
        cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, pr in procs:
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the packed-fp32 feature; that warning is expected
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if lines and (verbose or pr.returncode):
            print("\n".join(lines), file=sys.stderr)
        if pr.returncode:
            failed.append(src)
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    build_hbm_stream(verbose)
    return OUT


HBM_OUT = os.path.join(PKG, "libhbmstream.so")


def build_hbm_stream(verbose=False):
    """The HBM streaming microbenchmark (csrc/hbm_stream.hip), a library of
    its own: a measurement aid, not part of the solver."""
    tmp = HBM_OUT + ".tmp"
    cmd = [HIPCC] + COMMON + DEVICE_FLAGS + ["-x", "hip", "-shared", os.path.join(CSRC, "hbm_stream.hip"),
                                             "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    text = out.stdout.decode(errors="replace")
    lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if lines and (verbose or out.returncode):
        print("\n".join(lines), file=sys.stderr)
    if out.returncode:
        raise RuntimeError("hipcc failed for hbm_stream.hip")
    os.replace(tmp, HBM_OUT)
    return HBM_OUT


if __name__ == "__main__":
    print(build(verbose=True))
