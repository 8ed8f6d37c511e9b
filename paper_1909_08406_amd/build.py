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


def resource_usage(out_md=None, jobs: int = 0) -> str:
    """The compiler's per-kernel resource usage of every step kernel (VGPRs,
    AGPRs, SGPRs, scratch, LDS, occupancy), from -Rpass-analysis remarks of
    a device-only compile of each step translation unit, as a markdown
    table; written to out_md when given."""
    import re
    import tempfile
    srcs = [s for s in sources() if os.path.basename(s).startswith("step_")]
    jobs = jobs or max(1, min(len(srcs), os.cpu_count() or 4, 16))

    def remarks(src):
        with tempfile.TemporaryDirectory() as tmp:
            cmd = [HIPCC, *FLAGS, "--cuda-device-only", "-Rpass-analysis=kernel-resource-usage", "-c", "-o",
                   os.path.join(tmp, "x.o"), src]
            r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(r.stdout + r.stderr)
        return r.stderr

    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as pool:
        texts = list(pool.map(remarks, srcs))
    fields = ("VGPRs", "AGPRs", "TotalSGPRs", "ScratchSize [bytes/lane]", "LDS Size [bytes/block]",
              "Occupancy [waves/SIMD]")
    rows = {}
    for text in texts:
        name = None
        for line in text.splitlines():
            m = re.search(r"remark:\s+Function Name: (\S+)", line)
            if m:
                name = m.group(1)
                rows.setdefault(name, {})
                continue
            m = re.search(r"remark:\s+([^:]+): (\S+)", line)
            if name and m and m.group(1).strip() in fields:
                rows[name][m.group(1).strip()] = m.group(2)
    demangled = subprocess.run(["c++filt"], input="\n".join(rows), capture_output=True, text=True).stdout.split("\n")
    md = ["| kernel | VGPR | AGPR | SGPR | scratch B/lane | LDS B/block | waves/SIMD |", "|---|---|---|---|---|---|---|"]
    for mangled, pretty in sorted(zip(rows, demangled), key=lambda kv: kv[1]):
        if "k_step" not in pretty and "k_stream_free" not in pretty:
            continue
        # the Newton count each storage form runs: 3 in FP64, 1 otherwise
        m = re.search(r"k_step\w*<lbm::Store(\w+), (\d+),", pretty)
        if m and int(m.group(2)) != (3 if m.group(1) == "F64" else 1):
            continue
        r = rows[mangled]
        md.append("| `%s` | %s |" % (pretty.split("(")[0], " | ".join(r.get(f, "") for f in fields)))
    text = "\n".join(md) + "\n"
    if out_md:
        with open(out_md, "w") as fh:
            fh.write("# Step-kernel resource usage (compiler, gfx950)\n\n"
                     "Command (from the repository root): `python3 -m paper_1909_08406_amd.build --resource-usage "
                     "%s`, a device-only compile of each step translation unit with "
                     "`-Rpass-analysis=kernel-resource-usage` and the library's flags.\n\n"
                     "Template arguments of `k_step` and `k_step_lds`: storage, Newton steps, block threads, hint "
                     "flags (1 non-temporal loads, 2 non-temporal stores, 4 LDS staging), stochastic rounding, "
                     "model (0 E2, 1 isothermal, 2 E1, 4 entropic path length, 8 walls, sums combine). Listed: "
                     "the Newton count each storage form runs (3 in FP64, 1 otherwise).\n\n"
                     % os.path.relpath(out_md, ROOT) + text)
    return text


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--resource-usage":
        print(resource_usage(sys.argv[2] if len(sys.argv) > 2 else None))
    else:
        print(build(verbose=True))
