"""Throughput of the fused RD3Q41 collide-and-stream step on one MI355X.

Workload: the precision-form acoustic pulse, 512^3 cells (2 nodes per cell,
268,435,456 nodes), Gaussian density bump of amplitude 1e-3 and half width
8 cells, u = 0, theta = theta0, tau_lb = 0.6. The headline form is FP16
holding f - w rho0 with stochastic rounding (FP32 arithmetic); FP32 storage
of f and the other forms are timed on the same grid. Each form is first
autotuned (launch configuration), then a step is one launch of the fused
kernel over all nodes, timed with HIP events on the context's stream; the
inputs are resident in HBM before timing starts.

Prints one JSON line. --gpus above 1 is refused: the library has no multi-GPU path.
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ALGO_VALUES_PER_NODE = 82  # 41 loads + 41 stores per node update
COUNTERS = os.path.join(ROOT, "profiles", "k_step_pulse512_hbm_counters.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=400,
                    help="untimed steps before tuning and timing: long enough (about 4 s of the FP16 step) for "
                         "the clock to settle under sustained load")
    ap.add_argument("--n", type=int, default=512, help="cells per edge of the periodic box")
    ap.add_argument("--forms", default="f16s+sr,f32,f16s,f32+sr,f32s,bf16s+sr,f16s+sr+e1,f32+e1,f16s+sr+elbm,f32+elbm,f64",
                    help="storage forms ('+sr': stochastic rounding, '+e1': series equilibrium E1 instead of "
                         "the entropic E2, '+elbm': entropic path length, '+walls': kinetic walls normal to y); "
                         "the first is the headline")
    ap.add_argument("--tau", type=float, default=0.6)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=128, help="cells per edge of the oracle sample")
    ap.add_argument("--cpu-steps", type=int, default=24)
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-box batch measurement")
    ap.add_argument("--batch-forms", default="f16s+sr,f32")
    ap.add_argument("--batch-steps", type=int, default=100, help="eager steps timed for the batch")
    ap.add_argument("--batch-graph-steps", type=int, default=1000,
                    help="steps of the captured graph the batch is timed with (one replay)")
    ap.add_argument("--copy-reference", type=float, default=0.0, metavar="GIB",
                    help="only time a plain device-to-device copy of GIB GiB (HBM counter reference)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="only print a markdown summary of rocprofv3 --pmc outputs (*_counter_collection.csv "
                         "under each DIR): per step-kernel instance, the median of each counter over its dispatches "
                         "and the figures derived from them")
    ap.add_argument("--kernel-filter", default="k_step", help="kernels summarized by --summarize-counters")
    ap.add_argument("--hbm-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="only write the HBM-traffic summary under profiles/ from four rocprofv3 --pmc outputs")
    ap.add_argument("--trace-summary", nargs=3, metavar=("TRACE_DIR", "BENCH_STDERR", "OUT_MD"),
                    help="only write a kernel-trace summary from a rocprofv3 --kernel-trace output of the "
                         "trace run (bench_log_cmd) and that run's stderr")
    return ap.parse_args()


# What the step kernels' HBM traffic depends on: their sources, their launch
# code and the buffer layout (not the rest of the host code).
STEP_SOURCES = ("device.hpp", "kernels.hpp", "lattice.hpp", "layout.hpp", "step_launch.hpp", "step_tu.hpp",
                "step_*.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1909_08406_amd", "csrc")
    for p in sorted({f for pat in STEP_SOURCES for f in glob.glob(os.path.join(csrc, pat))}):
        with open(p, "rb") as fh:
            h.update(os.path.basename(p).encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(form, block, hints, xcd_remap):
    """HBM bytes per launch of the launch variant (block size, cache hints,
    XCD remap) of a form from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    try:
        with open(COUNTERS) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256") != kernel_source_hash():
        return None
    rec = d.get("forms", {}).get(form, {}).get("%d,%d,%d" % (block, hints, xcd_remap))
    if not rec:
        return None
    return {"fetch_bytes": rec["fetch_bytes"], "write_bytes": rec["write_bytes"],
            "total_bytes": rec["fetch_bytes"] + rec["write_bytes"], "kernel": rec["kernel"],
            "scale": d.get("scale"), "source": os.path.relpath(COUNTERS, ROOT)}


def time_copy(torch, gib, reps=5, lbm=None):
    """A plain device-to-device copy of known size: bytes read = bytes
    written = GIB GiB. The runtime's copy, or with `lbm` the library's own
    copy kernel (16-byte words)."""
    n = int(gib * (1 << 30))
    a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    if lbm is None:
        copy = lambda: b.copy_(a)  # noqa: E731
    else:
        stream = torch.cuda.current_stream()
        copy = lambda: lbm.device_copy(a.data_ptr(), b.data_ptr(), n, stream)  # noqa: E731
    copy()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        copy()
    e.record()
    e.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_read": n, "bytes_written": n, "ms": ms, "gbs_read_plus_write": 2 * n / (ms * 1e-3) / 1e9}


def copy_reference(torch, gib, reps=5):
    r = time_copy(torch, gib, reps)
    print(json.dumps({"copy_reference_bytes_read": r["bytes_read"], "copy_reference_bytes_written": r["bytes_written"],
                      "ms": r["ms"], "gbs_read_plus_write": r["gbs_read_plus_write"]}), flush=True)


# MI355X: 256 CUs of 4 SIMDs in 8 XCDs (GRBM_GUI_ACTIVE is summed over the XCDs)
CUS, SIMDS_PER_CU, XCDS = 256, 4, 8


def summarize_counters(dirs, kernel_filter):
    """Median per dispatch of every counter of each matching kernel instance
    (rocprofv3 --pmc CSVs), with derived figures: instructions per wavefront,
    the clock (GRBM_GUI_ACTIVE per XCD over the dispatch duration), VALU issue
    share (a wave64 VALU instruction issues over 2 cycles of a SIMD), mean
    waves per SIMD (SQ_WAVE_CYCLES counts 4-cycle units), L2 hit rate."""
    import csv
    import statistics
    rows = []
    for d in dirs:
        for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
            with open(path) as fh:
                rows += list(csv.DictReader(fh))
    per = {}
    for r in rows:
        if kernel_filter not in r["Kernel_Name"]:
            continue
        k = r["Kernel_Name"].split("(")[0]
        disp = per.setdefault(k, {}).setdefault(r["Dispatch_Id"], {})
        disp[r["Counter_Name"]] = float(r["Counter_Value"])
        disp["_ns"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        disp["_vgpr"] = r.get("VGPR_Count")
    out = []
    for k, disps in sorted(per.items()):
        names = sorted({c for d in disps.values() for c in d if not c.startswith("_")})
        med = {c: statistics.median(d[c] for d in disps.values() if c in d) for c in names}
        ns = statistics.median(d["_ns"] for d in disps.values())
        out.append("### `%s`" % k)
        out.append("")
        out.append("%d dispatches, median duration %.3f ms" % (len(disps), ns * 1e-6))
        out.append("")
        out.append("| counter | median per dispatch |")
        out.append("|---|---|")
        for c in names:
            out.append("| %s | %.6g |" % (c, med[c]))
        derived = []
        w = med.get("SQ_WAVES")
        gui = med.get("GRBM_GUI_ACTIVE")
        if w:
            for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_INSTS_LDS"):
                if c in med:
                    derived.append(("%s per wavefront" % c, med[c] / w))
        if gui:
            cyc = gui / XCDS
            derived.append(("clock (GHz)", cyc / ns))
            simds = CUS * SIMDS_PER_CU
            if "SQ_INSTS_VALU" in med:
                derived.append(("VALU issue share (2 cycles per wave64 instruction)", 2 * med["SQ_INSTS_VALU"] / (simds * cyc)))
            if "SQ_ACTIVE_INST_VALU" in med:
                derived.append(("SQ_ACTIVE_INST_VALU per SIMD-cycle", med["SQ_ACTIVE_INST_VALU"] / (simds * cyc)))
            if "SQ_WAVE_CYCLES" in med:
                derived.append(("mean waves per SIMD (SQ_WAVE_CYCLES x 4)", 4 * med["SQ_WAVE_CYCLES"] / (simds * cyc)))
            for c in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VMEM"):
                if c in med and "SQ_WAVE_CYCLES" in med:
                    derived.append(("%s / SQ_WAVE_CYCLES" % c, med[c] / med["SQ_WAVE_CYCLES"]))
            if "TA_TA_BUSY_sum" in med:
                derived.append(("TA busy share (TA_TA_BUSY_sum per TA-cycle)", med["TA_TA_BUSY_sum"] / (CUS * cyc)))
        if gui and "TCC_BUSY_sum" in med:
            derived.append(("L2 channel busy share (TCC_BUSY_sum per channel-cycle, 16 channels per XCD)",
                            med["TCC_BUSY_sum"] / (16 * XCDS * gui / XCDS)))
        if w:
            for c in ("TCP_TCC_READ_REQ_sum", "TCP_TCC_WRITE_REQ_sum", "TCC_REQ_sum"):
                if c in med:
                    derived.append(("%s per wavefront" % c, med[c] / w))
        if "TCC_HIT_sum" in med and "TCC_MISS_sum" in med:
            derived.append(("L2 hit rate", med["TCC_HIT_sum"] / max(1.0, med["TCC_HIT_sum"] + med["TCC_MISS_sum"])))
        if derived:
            out.append("")
            out.append("| derived | value |")
            out.append("|---|---|")
            for name, v in derived:
                out.append("| %s | %.4g |" % (name, v))
        out.append("")
    print("\n".join(out))


# rocprofv3 recipes of the committed summaries (run from the repository root)
HBM_RUN = "python3 bench.py --steps 3 --warmup 10 --no-cpu-baseline --no-batch --forms f16s+sr,f32,f16s"
COPY_RUN = "python3 bench.py --copy-reference 4"
TUNE_ROUNDS, TUNE_REPS = 3, 4  # the autotuner: 3 rounds, each configuration timed with 1 + 3 dispatches


def _counter_rows(d):
    import csv
    rows = []
    for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        with open(path) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _per_dispatch(rows, counter):
    """{dispatch id: (kernel name, value)} for one counter, in dispatch order."""
    out = {}
    for r in rows:
        if r["Counter_Name"] == counter:
            out[int(r["Dispatch_Id"])] = (r["Kernel_Name"].split("(")[0].strip(), float(r["Counter_Value"]))
    return dict(sorted(out.items()))


def hbm_summary(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    """HBM bytes per launch of every launch configuration of the step
    kernels of HBM_RUN (FETCH_SIZE and WRITE_SIZE, KiB per dispatch, each
    in a run of its own), scaled by what the same counters read for the
    runtime's copy of 4 GiB (COPY_RUN). The dispatches of each form come in
    a fixed order: the warmup (10 steps), then the autotuner's rounds over
    (variant, XCD remap) pairs, TUNE_REPS dispatches each; each
    configuration keeps the median over its rounds. Writes COUNTERS (read
    by the bench) and its markdown beside it."""
    import re
    import statistics
    from paper_1909_08406_amd import lbm
    nvariants = lbm.num_variants()
    step_kernel = re.compile(r"lbm::k_step(_lds)?<")
    gib4 = 4 << 30
    cf = max(v for _, v in _per_dispatch(_counter_rows(copy_fetch_dir), "FETCH_SIZE").values())
    cw = max(v for _, v in _per_dispatch(_counter_rows(copy_write_dir), "WRITE_SIZE").values())
    scale_f, scale_w = gib4 / (cf * 1024), gib4 / (cw * 1024)
    fetch = _per_dispatch(_counter_rows(fetch_dir), "FETCH_SIZE")
    write = _per_dispatch(_counter_rows(write_dir), "WRITE_SIZE")
    forms = HBM_RUN.split("--forms ")[1].split(",")
    # the step dispatches of the run, form after form
    seq_f = [(k, v) for k, v in fetch.values() if step_kernel.search(k)]
    seq_w = [(k, v) for k, v in write.values() if step_kernel.search(k)]
    per_form = 10 + TUNE_ROUNDS * nvariants * 2 * TUNE_REPS + 10 + 3
    if len(seq_f) != per_form * len(forms) or len(seq_w) != len(seq_f):
        raise SystemExit("expected %d step dispatches, found %d fetch / %d write"
                         % (per_form * len(forms), len(seq_f), len(seq_w)))
    n = 512 ** 3 * 2
    out = {"source_sha256": kernel_source_hash(), "scale": {"fetch": scale_f, "write": scale_w},
           "commands": ["rocprofv3 --pmc FETCH_SIZE -f csv -d %s -o f -- %s" % (fetch_dir, HBM_RUN),
                        "rocprofv3 --pmc WRITE_SIZE -f csv -d %s -o w -- %s" % (write_dir, HBM_RUN),
                        "rocprofv3 --pmc FETCH_SIZE -f csv -d %s -o cf -- %s" % (copy_fetch_dir, COPY_RUN),
                        "rocprofv3 --pmc WRITE_SIZE -f csv -d %s -o cw -- %s" % (copy_write_dir, COPY_RUN)],
           "forms": {}}
    lines = []
    for i, form in enumerate(forms):
        base = i * per_form + 10
        eb = 2 if form.startswith(("f16s", "bf16s")) else 4 if form.startswith("f32") else 8
        algo = ALGO_VALUES_PER_NODE // 2 * eb * n
        recs = {}
        for v in range(nvariants):
            for x in (0, 1):
                idx = [base + rnd * nvariants * 2 * TUNE_REPS + (2 * v + x) * TUNE_REPS + k
                       for rnd in range(TUNE_ROUNDS) for k in range(TUNE_REPS)]
                names = {seq_f[j][0] for j in idx}
                if len(names) != 1:
                    raise SystemExit("dispatch order does not match the autotuner's for %s v%d r%d" % (form, v, x))
                fb = statistics.median(seq_f[j][1] for j in idx) * 1024 * scale_f
                wb = statistics.median(seq_w[j][1] for j in idx) * 1024 * scale_w
                blk, hints = None, None
                kname = names.pop()
                recs[(v, x)] = (kname, fb, wb)
        out["forms"][form] = {}
        for (v, x), (kname, fb, wb) in recs.items():
            targs = kname.split("<")[1].split(">")[0].split(",")
            blk, hints = int(targs[2]), int(targs[3])
            out["forms"][form]["%d,%d,%d" % (blk, hints, x)] = {"kernel": kname, "fetch_bytes": fb,
                                                                "write_bytes": wb, "variant": v}
            lines.append("| `%s` (XCD remap %s) | %s | %.2f | %.2f | %.2f | %.3f | %.3f |"
                         % (kname, "on" if x else "off", form, fb / 1e9, wb / 1e9, algo / 1e9, fb / algo, wb / algo))
    with open(COUNTERS, "w") as fh:
        json.dump(out, fh, indent=1)
    md = ["# HBM traffic of the fused step kernel, 512^3 acoustic pulse (rocprofv3 counters)", "",
          "Commands (from the repository root on one MI355X; each counter in a run of its own):", ""]
    md += ["    " + c for c in out["commands"]]
    md += ["", "Summary written by `python3 bench.py --hbm-summary %s %s %s %s`." % (fetch_dir, write_dir,
                                                                                   copy_fetch_dir, copy_write_dir),
           "",
           "Scale: the runtime's copy of 4 GiB reads FETCH_SIZE = %.0f KiB and WRITE_SIZE = %.0f KiB per dispatch, "
           "so bytes = FETCH_SIZE KiB x 1024 x %.3f and WRITE_SIZE KiB x 1024 x %.3f." % (cf, cw, scale_f, scale_w),
           "",
           "Algorithmic bytes per launch: 41 loads + 41 stores per node, %d nodes. Every launch variant with the XCD "
           "remap off and on (the autotuner's dispatches: %d rounds of %d, medians)." % (n, TUNE_ROUNDS, TUNE_REPS),
           "",
           "| kernel | form | fetched GB | written GB | algorithmic read = write GB | fetch / algorithmic | "
           "write / algorithmic |", "|---|---|---|---|---|---|---|"] + lines
    with open(COUNTERS.replace(".json", ".md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


def trace_summary(trace_dir, bench_log, steps, out_md):
    """Kernel-trace summary (rocprofv3 --kernel-trace CSV): per step-kernel
    instance, dispatches, mean duration over all and over the last `steps`
    (for the chosen configuration of a form: its timed steps); bench_log is
    the same run's stderr (the bench's own HIP-event figures)."""
    import csv
    rows = []
    for path in sorted(glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)):
        with open(path) as fh:
            rows += list(csv.DictReader(fh))
    per, res = {}, {}
    for r in sorted(rows, key=lambda r: int(r["Start_Timestamp"])):
        k = r["Kernel_Name"].split("(")[0].strip()
        if "k_step" in k or "k_stream_free" in k or "k_copy16" in k:
            per.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)
            res[k] = tuple(r.get(c, "") for c in ("VGPR_Count", "SGPR_Count", "LDS_Block_Size", "Scratch_Size",
                                                  "Workgroup_Size_X"))
    with open(bench_log) as fh:
        blog = [l.rstrip() for l in fh if l.startswith("#")]
    md = ["# Step kernels on the 512^3 acoustic pulse: rocprofv3 kernel trace of the default bench run", "",
          "Command (from the repository root on one MI355X):", "",
          "    rocprofv3 --kernel-trace --stats -f csv -d %s -o kt -- %s" % (trace_dir, bench_log_cmd(steps)), "",
          "Summary written by `python3 bench.py --steps %d --trace-summary %s <stderr of that run> %s`." % (
              steps, trace_dir, out_md), "",
          "bench.py's own HIP-event timing in the same run:", ""] + ["    " + l for l in blog] + [
          "", "The last columns are the trace's own fields per dispatch (`VGPR_Count` and `SGPR_Count` in the "
          "profiler's allocation units, not registers; LDS bytes per block, scratch bytes per lane, threads per "
          "block). The compiler's register counts are in `profiles/k_step_resources.md`.", "",
          "| kernel | dispatches | mean ms (all) | mean ms (last %d) | VGPR_Count | SGPR_Count | LDS | scratch | "
          "block |" % steps, "|---|---|---|---|---|---|---|---|---|"]
    for k, d in sorted(per.items(), key=lambda kv: -len(kv[1])):
        last = d[-steps:]
        md.append("| `%s` | %d | %.3f | %.3f | %s |" % (k, len(d), sum(d) / len(d), sum(last) / len(last),
                                                       " | ".join(res[k])))
    with open(out_md, "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


def bench_log_cmd(steps):
    """The traced command: the default bench run, with its step count."""
    return "python3 bench.py --steps %d" % steps


def parse_form(form):
    """'storage[+sr][+e1][+elbm][+walls]': storage form, stochastic rounding,
    series equilibrium E1 instead of the entropic E2, entropic path length,
    kinetic walls normal to y (at rest at theta0)."""
    storage, *flags = form.split("+")
    unknown = set(flags) - {"sr", "e1", "elbm", "walls"}
    if unknown:
        raise SystemExit("unknown form flag(s) %s in %r" % (sorted(unknown), form))
    return storage, "sr" in flags, "e1" in flags, "elbm" in flags, "walls" in flags


CHUNK = 10  # steps per event-timed chunk of the warmup


def run_chunks(torch, stream, fn, steps):
    """Run fn(CHUNK) repeatedly for `steps` steps; ms per step of each chunk."""
    nch = max(1, steps // CHUNK)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nch + 1)]
    ev[0].record(stream)
    for i in range(nch):
        fn(CHUNK)
        ev[i + 1].record(stream)
    ev[-1].synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) / CHUNK for i in range(nch)]


def time_steps(torch, stream, fn, steps):
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    fn(steps)
    end.record(stream)
    end.synchronize()
    torch.cuda.synchronize()
    return start.elapsed_time(end)


def time_form(lbm, torch, F, th, n, tau, form, steps, warmup, autotune, pattern=False):
    """Under sustained load the GPU lowers its clock (power limit) within a
    few seconds; kernels with much arithmetic per byte slow down with it. So
    the warmup runs first, at the default launch, timed in chunks (its first
    chunks give the rate before the clock drops, `burst_ms_per_step`); the
    autotuner then picks at the settled clock, and the timed steps follow."""
    storage, sr, e1, elbm, walls = parse_form(form)
    stream = torch.cuda.Stream()
    t0 = time.time()
    ctx = lbm.init([(n, n, n, tau)], *F.absolute(th), storage=storage, stream=stream, stochastic=sr, series=e1,
                   entropic=elbm, walls=walls)
    init_s = time.time() - t0
    chunks = run_chunks(torch, stream, ctx.step, warmup) if warmup > 0 else []
    burst = sum(chunks[1:6]) / len(chunks[1:6]) if len(chunks) > 1 else None
    settled = chunks[-5:]
    tune = None
    if autotune:
        best, table = ctx.autotune(reps=3)
        tune = {"variant": best[0], "xcd_remap": best[1]}
        ctx.step(CHUNK)
    info = ctx.info()
    tuning_now = ctx.tuning()
    if tune is not None:
        tune["block_threads"] = info["block_threads"]
    ms = time_steps(torch, stream, ctx.step, steps)
    status = ctx.status()
    pat = None
    if pattern:
        # the step's access pattern alone: collisionless streaming in the same
        # context, in the launch configuration fastest for it (a short timing
        # of each, then the full count in the best)
        cand = {}
        for v in range(lbm.num_variants()):
            for x in (0, 1):
                ctx.set_tuning(variant=v, xcd_remap=x)
                ctx.stream_free(2)
                cand[(v, x)] = time_steps(torch, stream, ctx.stream_free, 2 * CHUNK) / (2 * CHUNK)
        bv, bx = min(cand, key=cand.get)
        ctx.set_tuning(variant=bv, xcd_remap=bx)
        pat = {"ms": time_steps(torch, stream, ctx.stream_free, steps) / steps, "variant": bv, "xcd_remap": bx,
               "block_threads": lbm.variant_desc(bv)[0]}
    ctx.free()
    del ctx
    torch.cuda.empty_cache()
    nodes = info["nodes"]
    ms_step = ms / steps
    bytes_launch = ALGO_VALUES_PER_NODE * lbm.ELEM_BYTES[storage] * nodes
    # launch variant that was timed (the models other than E2 run 256 threads, no hints)
    blk, hints = lbm.variant_desc(info["variant"])
    if info["block_threads"] != blk:
        blk, hints = info["block_threads"], 0
    return {
        "form": form,
        "launch": [blk, hints, int(tuning_now["xcd_remap"])],
        "ms_per_step": ms_step,
        "mlups": nodes * steps / (ms * 1e-3) / 1e6,
        "gbs": bytes_launch / (ms_step * 1e-3) / 1e9,
        "bytes_per_launch": bytes_launch,
        "nodes": nodes,
        "status": status,
        "init_s": init_s,
        "shift_exp": info["shift_exp"],
        "newton_iters": info["newton_iters"],
        "tuning": tune,
        "burst_ms_per_step": burst,
        "warmup_last_chunks_ms": settled,
        "pattern": pat,
    }


def time_batch(lbm, torch, form, steps, graph_steps, warmup, autotune):
    """The 256-box batch of uneven periodic standing-wave boxes (edges from
    {16, 24, 32, 48, 64, 96}, seed 0) in one context: one launch per step
    over every (box, tile), timed eager (`steps` steps) and as one replay of
    a captured graph of `graph_steps` steps (after one untimed replay that
    also captures it)."""
    from paper_1909_08406_amd import workloads as wl

    storage, sr, e1, elbm, walls = parse_form(form)
    specs = wl.batch_specs()
    cat = wl.concat([wl.batch_fields(b) for b in specs])
    _, _, th = lbm.lattice()
    stream = torch.cuda.Stream()
    ctx = lbm.init([(b.nx, b.ny, b.nz, b.tau) for b in specs], cat[0], cat[1], cat[2], cat[3], cat[4] * th,
                   storage=storage, stream=stream, stochastic=sr, series=e1, entropic=elbm, walls=walls)
    del cat
    if autotune:
        ctx.autotune(reps=3)
    nodes = ctx.info()["nodes"]
    out = {"nodes": nodes, "tuning": ctx.tuning()}
    for mode, g in (("eager", 0), ("graph", graph_steps)):
        ctx.set_tuning(graph_steps=g)
        n = steps if g == 0 else g
        ctx.step(max(warmup, g))
        ctx.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        ctx.step(n)
        end.record(stream)
        end.synchronize()
        ms = start.elapsed_time(end) / n
        bytes_launch = ALGO_VALUES_PER_NODE * lbm.ELEM_BYTES[storage] * nodes
        out[mode] = {"ms_per_step": ms, "mlups": nodes / (ms * 1e-3) / 1e6, "gbs": bytes_launch / (ms * 1e-3) / 1e9,
                     "steps_timed": n, "graph_steps": g}
    out["status"] = ctx.status()
    ctx.free()
    torch.cuda.empty_cache()
    return out


def cpu_baseline(args):
    import oracle
    from paper_1909_08406_amd import workloads as wl

    n = args.cpu_n
    _, _, th = oracle.lattice()
    F = wl.gaussian_pulse(n, eps=1e-3, b=8.0)
    f = oracle.init(n, n, n, *F.absolute(th))
    t0 = time.time()
    oracle.run(n, n, n, 1.0 / args.tau, f, args.cpu_steps)
    dt = time.time() - t0
    nodes = 2 * n ** 3
    return {
        "value": nodes * args.cpu_steps / dt / 1e6,
        "unit": "MLUPS",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": "FP64 oracle (OpenMP over nodes), same pulse recipe (eps 1e-3, b 8, tau 0.6) on %d^3 cells "
                  "(%d nodes), %d steps, %.1f s" % (n, nodes, args.cpu_steps, dt),
    }


def pattern_ceiling(r):
    """The step's memory access pattern alone (lbm_stream_free in the same
    context, in its own fastest launch configuration): its rate, and the
    step's rate as a fraction of it."""
    pat = r.get("pattern")
    if pat is None:
        return None
    gbs = r["bytes_per_launch"] / (pat["ms"] * 1e-3) / 1e9
    return {"kernel": "lbm::k_stream_free", "ms_per_step": pat["ms"], "achieved": gbs, "frac": gbs / HBM_PEAK_GBS,
            "launch": [pat["block_threads"], pat["variant"], pat["xcd_remap"]],
            "step_over_pattern": pat["ms"] / r["ms_per_step"]}


DTYPE = {"f16s": "f16-shifted storage, f32 compute", "bf16s": "bf16-shifted storage, f32 compute",
         "f32": "f32", "f32s": "f32-shifted storage, f32 compute", "f64": "f64"}


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.kernel_filter)
        return
    if args.hbm_summary:
        hbm_summary(*args.hbm_summary)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary[0], args.trace_summary[1], args.steps, args.trace_summary[2])
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1909_08406_amd import lbm
    from paper_1909_08406_amd import workloads as wl

    torch.cuda.set_device(0)
    if args.copy_reference > 0:
        copy_reference(torch, args.copy_reference)
        return
    _, _, th = lbm.lattice()
    n = args.n
    t0 = time.time()
    F = wl.gaussian_pulse(n, eps=1e-3, b=8.0)
    print("# fields %d^3 generated in %.1f s" % (n, time.time() - t0), file=sys.stderr, flush=True)
    runs = []
    for i, form in enumerate(args.forms.split(",")):
        r = time_form(lbm, torch, F, th, n, args.tau, form, args.steps, args.warmup, not args.no_autotune,
                      pattern=(i == 0))
        print("# %s: %.3f ms/step, %.0f MLUPS, %.0f GB/s (first warmup steps %s ms/step; init %.1f s, tuning %s)"
              % (form, r["ms_per_step"], r["mlups"], r["gbs"],
                 "%.3f" % r["burst_ms_per_step"] if r["burst_ms_per_step"] else "-", r["init_s"], r["tuning"]),
              file=sys.stderr, flush=True)
        if r["pattern"] is not None:
            pc = pattern_ceiling(r)
            print("# %s access pattern alone (free streaming, launch %s): %.3f ms/step, %.0f GB/s; "
                  "step rate / pattern rate %.3f" % (form, pc["launch"], pc["ms_per_step"], pc["achieved"],
                                                      pc["step_over_pattern"]), file=sys.stderr, flush=True)
        runs.append(r)
    del F
    # what a plain copy reaches on this device: the achievable HBM rate
    # beside the published peak
    cp = time_copy(torch, 4, reps=20, lbm=lbm)
    copy_ceiling = {"kernel": "lbm::k_copy16, plain copy of 4 GiB (lbm_device_copy)", "ms": cp["ms"],
                    "achieved": cp["gbs_read_plus_write"], "frac": cp["gbs_read_plus_write"] / HBM_PEAK_GBS,
                    "step_over_copy": runs[0]["gbs"] / cp["gbs_read_plus_write"]}
    print("# plain copy of 4 GiB: %.0f GB/s read + write (%.3f of 8 TB/s); %s step at %.3f of it"
          % (cp["gbs_read_plus_write"], copy_ceiling["frac"], runs[0]["form"], copy_ceiling["step_over_copy"]),
          file=sys.stderr, flush=True)
    batch = None
    if not args.no_batch:
        batch = {"workload": "256 periodic standing-wave boxes, edges from {16,24,32,48,64,96}, k 1..4, "
                             "tau U[0.51,1), amplitude 10^U[-4,-2], seed 0; one launch per step over all boxes; "
                             "'graph' is one replay of a captured %d-step graph" % args.batch_graph_steps,
                 "forms": {}}
        for form in args.batch_forms.split(","):
            r = time_batch(lbm, torch, form, args.batch_steps, args.batch_graph_steps, args.warmup,
                           not args.no_autotune)
            batch["nodes"] = r.pop("nodes")
            batch["forms"][form] = r
            print("# batch %s: eager %.3f ms/step %.0f MLUPS %.0f GB/s; graph %.3f ms/step %.0f MLUPS %.0f GB/s (%s)"
                  % (form, r["eager"]["ms_per_step"], r["eager"]["mlups"], r["eager"]["gbs"],
                     r["graph"]["ms_per_step"], r["graph"]["mlups"], r["graph"]["gbs"], r["tuning"]),
                  file=sys.stderr, flush=True)
    head = runs[0]
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args)
        print("# cpu baseline: %s" % cpu["sample"], file=sys.stderr, flush=True)
    by = {r["form"]: {k: r[k] for k in ("mlups", "gbs", "ms_per_step", "burst_ms_per_step", "status", "shift_exp",
                                        "newton_iters", "tuning")} for r in runs}
    traffic = measured_traffic(head["form"], *head["launch"])
    out = {
        "metric": "MLUPS + achieved HBM GB/s, fused collide-stream, FP16-shifted vs FP32 storage",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[parse_form(head["form"])[0]] + (", stochastic rounding" if parse_form(head["form"])[1] else ""),
        "data": "synthetic",
        "config": {"workload": "periodic acoustic pulse %d^3 cells (%d nodes), eps 1e-3, b 8, tau 0.6, %s"
                               % (n, head["nodes"], head["form"]),
                   "nodes": head["nodes"], "form": head["form"]},
        "achieved_gbs": head["gbs"],
        "by_form": by,
        "roofline": {"bound": "hbm", "achieved": head["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["gbs"] / HBM_PEAK_GBS,
                     "traffic": traffic["total_bytes"] / (head["ms_per_step"] * 1e-3) / 1e9 if traffic else None,
                     "traffic_bytes_per_launch": traffic,
                     "kernel": "lbm::k_step (%s)" % head["form"],
                     "algorithmic_bytes_per_launch": head["bytes_per_launch"],
                     "pattern_ceiling": pattern_ceiling(head),
                     "copy_ceiling": copy_ceiling},
        "cpu_baseline": cpu,
        "batch": batch,
    }
    # FP32 storage that meets the thermal-mode accuracy bar is the one with
    # stochastic rounding (round to nearest biases the slow entropy mode)
    if "f32+sr" in by:
        out["speedup_vs_f32"] = head["mlups"] / by["f32+sr"]["mlups"]
        out["speedup_vs_f32_form"] = "f32+sr"
    if "f32" in by:
        out["speedup_vs_f32_round_to_nearest"] = head["mlups"] / by["f32"]["mlups"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
