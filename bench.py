"""Throughput of the fused RD3Q41 collide-and-stream step on one MI355X.

Workload: the precision-form acoustic pulse, 512^3 cells (2 nodes per cell,
268,435,456 nodes), Gaussian density bump of amplitude 1e-3 and half width
8 cells, u = 0, theta = theta0, tau_lb = 0.6. The headline storage is FP16
holding f - w rho0 (FP32 arithmetic); FP32 storage of f is timed on the
same grid for the speedup. A step is one launch of the fused kernel over
all nodes; inputs are resident in HBM before timing starts.

Prints one JSON line. --gpus above 1 is refused: this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ALGO_VALUES_PER_NODE = 82  # 41 loads + 41 stores per node update


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=512, help="cells per edge of the periodic box")
    ap.add_argument("--storages", default="f16s,f32", help="first one is the headline")
    ap.add_argument("--tau", type=float, default=0.6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=128, help="cells per edge of the oracle sample")
    ap.add_argument("--cpu-steps", type=int, default=24)
    ap.add_argument("--copy-reference", type=float, default=0.0, metavar="GIB",
                    help="only time a plain device-to-device copy of GIB GiB (HBM counter reference)")
    return ap.parse_args()


def copy_reference(torch, gib, reps=5):
    """A plain copy kernel of known size: bytes read = bytes written = GIB GiB."""
    n = int(gib * (1 << 30))
    a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    e.synchronize()
    ms = s.elapsed_time(e) / reps
    print(json.dumps({"copy_reference_bytes_read": n, "copy_reference_bytes_written": n, "ms": ms,
                      "gbs_read_plus_write": 2 * n / (ms * 1e-3) / 1e9}), flush=True)


def time_storage(lbm, torch, F, th, n, tau, storage, steps, warmup):
    stream = torch.cuda.Stream()
    t0 = time.time()
    ctx = lbm.init([(n, n, n, tau)], *F.absolute(th), storage=storage, stream=stream)
    init_s = time.time() - t0
    info = ctx.info()
    ctx.step(warmup)
    ctx.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    ctx.step(steps)
    end.record(stream)
    end.synchronize()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    status = ctx.status()
    tot = ctx.totals(check=False)[0]
    ctx.free()
    del ctx
    torch.cuda.empty_cache()
    nodes = info["nodes"]
    eb = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}[storage]
    ms_step = ms / steps
    bytes_launch = ALGO_VALUES_PER_NODE * eb * nodes
    return {
        "storage": storage,
        "ms_per_step": ms_step,
        "mlups": nodes * steps / (ms * 1e-3) / 1e6,
        "gbs": bytes_launch / (ms_step * 1e-3) / 1e9,
        "bytes_per_launch": bytes_launch,
        "nodes": nodes,
        "status": status,
        "mass": tot[0],
        "energy": tot[4],
        "init_s": init_s,
        "shift_exp": info["shift_exp"],
        "newton_iters": info["newton_iters"],
    }


def cpu_baseline(args):
    import numpy as np  # noqa: F401
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
        "sample": "FP64 oracle, same pulse recipe (eps 1e-3, b 8) on %d^3 cells (%d nodes), %d steps, %.1f s"
                  % (n, nodes, args.cpu_steps, dt),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
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
    gen_s = time.time() - t0
    print("# fields %d^3 generated in %.1f s" % (n, gen_s), file=sys.stderr, flush=True)
    runs = []
    for st in args.storages.split(","):
        r = time_storage(lbm, torch, F, th, n, args.tau, st, args.steps, args.warmup)
        print("# %s: %.3f ms/step, %.0f MLUPS, %.0f GB/s (init %.1f s)"
              % (st, r["ms_per_step"], r["mlups"], r["gbs"], r["init_s"]), file=sys.stderr, flush=True)
        runs.append(r)
    del F
    head = runs[0]
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args)
        print("# cpu baseline: %s" % cpu["sample"], file=sys.stderr, flush=True)
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
        "dtype": {"f16s": "f16-shifted storage, f32 compute", "bf16s": "bf16-shifted storage, f32 compute",
                  "f32": "f32", "f64": "f64"}[head["storage"]],
        "data": "synthetic",
        "config": {"workload": "periodic acoustic pulse %d^3 cells (%d nodes), eps 1e-3, b 8, tau 0.6, %s storage"
                               % (n, head["nodes"], head["storage"]),
                   "nodes": head["nodes"], "storage": head["storage"]},
        "achieved_gbs": head["gbs"],
        "by_storage": {r["storage"]: {"mlups": r["mlups"], "gbs": r["gbs"], "ms_per_step": r["ms_per_step"],
                                      "status": r["status"], "shift_exp": r["shift_exp"],
                                      "newton_iters": r["newton_iters"]} for r in runs},
        "roofline": {"bound": "hbm", "achieved": head["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["gbs"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_step<%s>" % head["storage"],
                     "algorithmic_bytes_per_launch": head["bytes_per_launch"]},
        "cpu_baseline": cpu,
    }
    if len(runs) > 1 and "f32" in out["by_storage"]:
        out["speedup_vs_f32"] = head["mlups"] / out["by_storage"]["f32"]["mlups"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
