"""Build liblbm.so for gfx950 with hipcc, in-tree.

The library is several HIP translation units: the host side and the
non-step kernels (lbm.hip), and one unit per storage form and rounding mode
holding that form's step-kernel instances (step_*.hip). They compile in
parallel into objects under _build/ and are linked into liblbm.so.

Every HIP translation unit is compiled with packed-FP32 instruction
selection disabled (-packed-fp32-ops); hipcc's host pass warns that it does
not know the feature, which is harmless.
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    """The translation units, the slowest to compile first."""
    steps = sorted(glob.glob(os.path.join(CSRC, "step_*.hip")))
    # FP64 and the stochastic-rounding units hold the largest kernels
    steps.sort(key=lambda p: (not p.endswith(("_f64.hip", "_sr.hip")), p))
    return steps + [os.path.join(CSRC, "lbm.hip")]


def _compile(src, extra, verbose):
    obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", "-o", obj + ".tmp", src]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        return obj, r.stdout + r.stderr
    os.replace(obj + ".tmp", obj)
    return obj, None


def build(verbose: bool = False, extra=(), jobs: int = 0) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = jobs or max(1, min(len(srcs), os.cpu_count() or 4, 16))
    objs, errors = [], []
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as pool:
        for obj, err in pool.map(lambda s: _compile(s, extra, verbose), srcs):
            objs.append(obj)
            if err:
                errors.append(err)
    if errors:
        sys.stderr.write("\n".join(errors))
        raise RuntimeError("hipcc failed building liblbm.so")
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("linking liblbm.so failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
