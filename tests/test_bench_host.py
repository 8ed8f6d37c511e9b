"""Host logic of bench.py (no device): the one-GPU guard, the counter
summaries built from rocprofv3 CSV files, and the hash that ties the HBM
counter summary to the step kernels' sources."""
import csv
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def write_counters(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counter_summary_derived_figures(tmp_path, capsys):
    """Two dispatches of one kernel: medians per counter, then instructions
    per wavefront and the clock (GRBM_GUI_ACTIVE is summed over 8 XCDs)."""
    rows = []
    for d, (valu, gui) in enumerate([(1000.0, 8.0e6), (1200.0, 8.0e6)]):
        for name, v in (("SQ_WAVES", 10.0), ("SQ_INSTS_VALU", valu * 10), ("GRBM_GUI_ACTIVE", gui)):
            rows.append({"Dispatch_Id": d, "Kernel_Name": "void lbm::k_step<x>(args)", "Counter_Name": name,
                         "Counter_Value": v, "Start_Timestamp": 0, "End_Timestamp": 500000})
    write_counters(str(tmp_path / "a" / "a_counter_collection.csv"), rows)
    bench.summarize_counters([str(tmp_path / "a")], "k_step")
    out = capsys.readouterr().out
    assert "2 dispatches, median duration 0.500 ms" in out
    assert "| SQ_INSTS_VALU per wavefront | 1100 |" in out
    # 8e6 cycles over 8 XCDs in 0.5 ms: 2 GHz
    assert "| clock (GHz) | 2 |" in out


def test_hbm_summary_attributes_dispatches_to_configurations(tmp_path, monkeypatch):
    """Synthetic FETCH_SIZE and WRITE_SIZE runs in the bench's dispatch
    order (warmup, the autotuner's rounds over variant and remap, the timed
    steps): every (variant, remap) gets the median of its own dispatches,
    scaled by the copy reference."""
    from paper_1909_08406_amd import lbm
    nv = lbm.num_variants()
    forms = bench.HBM_RUN.split("--forms ")[1].split(",")
    store = {"f16s+sr": ("StoreF16S", "true"), "f32": ("StoreF32", "false"), "f16s": ("StoreF16S", "false")}

    def name(form, v):
        blk, fl = lbm.variant_desc(v)
        k = "k_step_lds" if fl & 4 else "k_step"
        return "void lbm::%s<lbm::%s, 1, %d, %d, %s, 0>(args)" % (k, store[form][0], blk, fl, store[form][1])

    def expected(form, v, x, counter):
        return 1000.0 * (1 + forms.index(form)) + 10.0 * v + x + (0.5 if counter == "WRITE_SIZE" else 0.0)

    for counter, d in (("FETCH_SIZE", "f"), ("WRITE_SIZE", "w")):
        rows, did = [], 0

        def add(kernel, value):
            nonlocal did
            rows.append({"Dispatch_Id": did, "Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": value,
                         "Start_Timestamp": 0, "End_Timestamp": 1})
            did += 1

        add("void lbm::k_init<x>(args)", 1.0)  # other kernels are skipped
        for form in forms:
            for _ in range(10):
                add(name(form, 0), 7.0)  # warmup
            for rnd in range(bench.TUNE_ROUNDS):
                for v in range(nv):
                    for x in (0, 1):
                        for k in range(bench.TUNE_REPS):
                            # one outlier per configuration; the median ignores it
                            add(name(form, v), expected(form, v, x, counter) + (500.0 if rnd == k == 0 else 0.0))
            for _ in range(13):
                add(name(form, 0), 9.0)  # the chosen configuration, then the timed steps
        write_counters(str(tmp_path / d / "x_counter_collection.csv"), rows)
    for counter, d, kib in (("FETCH_SIZE", "cf", 2097152.0), ("WRITE_SIZE", "cw", 4194304.0)):
        write_counters(str(tmp_path / d / "x_counter_collection.csv"),
                       [{"Dispatch_Id": 0, "Kernel_Name": "copy", "Counter_Name": counter, "Counter_Value": kib,
                         "Start_Timestamp": 0, "End_Timestamp": 1}])
    out_json = tmp_path / "hbm.json"
    monkeypatch.setattr(bench, "COUNTERS", str(out_json))
    bench.hbm_summary(*(str(tmp_path / d) for d in ("f", "w", "cf", "cw")))
    d = json.loads(out_json.read_text())
    assert d["scale"] == {"fetch": 2.0, "write": 1.0}
    assert d["source_sha256"] == bench.kernel_source_hash()
    for form in forms:
        assert len(d["forms"][form]) == 2 * nv
        for v in range(nv):
            blk, fl = lbm.variant_desc(v)
            for x in (0, 1):
                rec = d["forms"][form]["%d,%d,%d" % (blk, fl, x)]
                assert rec["variant"] == v
                assert rec["fetch_bytes"] == pytest.approx(expected(form, v, x, "FETCH_SIZE") * 1024 * 2.0)
                assert rec["write_bytes"] == pytest.approx(expected(form, v, x, "WRITE_SIZE") * 1024 * 1.0)
    assert (tmp_path / "hbm.md").exists()


def test_source_hash_follows_the_step_kernels_only(tmp_path, monkeypatch):
    """The hash that keys the HBM counters changes with a step-kernel
    source or the layout, not with the rest of the host code."""
    tree = tmp_path / "paper_1909_08406_amd" / "csrc"
    shutil.copytree(os.path.join(ROOT, "paper_1909_08406_amd", "csrc"), tree)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    with open(tree / "lbm.hip", "a") as fh:
        fh.write("\n// host-only change\n")
    assert bench.kernel_source_hash() == h0
    for f in ("kernels.hpp", "layout.hpp", "step_f16s_sr.hip"):
        with open(tree / f, "a") as fh:
            fh.write("\n// change\n")
        h1 = bench.kernel_source_hash()
        assert h1 != h0, f
        h0 = h1


def test_trace_summary_means_over_the_last_steps(tmp_path):
    """Per kernel instance: all dispatches and the last `steps` of them
    (the timed steps), the bench's own lines carried over; other kernels
    are left out."""
    rows = []
    t = 0
    for k, durs in (("void lbm::k_step<A>(x)", [2.0] * 5 + [1.0] * 3), ("void lbm::k_copy16(x)", [0.5, 0.5]),
                    ("void lbm::k_init<A>(x)", [9.0])):
        for d in durs:
            rows.append({"Kernel_Name": k, "Start_Timestamp": t, "End_Timestamp": t + int(d * 1e6),
                         "VGPR_Count": 8, "SGPR_Count": 16, "LDS_Block_Size": 0, "Scratch_Size": 0,
                         "Workgroup_Size_X": 256})
            t += int(d * 1e6) + 1000
    os.makedirs(tmp_path / "kt")
    with open(tmp_path / "kt" / "kt_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    log = tmp_path / "bench.err"
    log.write_text("# f16s+sr: 1.000 ms/step\nnoise\n")
    out = tmp_path / "kt.md"
    bench.trace_summary(str(tmp_path / "kt"), str(log), 3, str(out))
    md = out.read_text()
    assert "    # f16s+sr: 1.000 ms/step" in md and "noise" not in md
    assert "| `void lbm::k_step<A>` | 8 | 1.625 | 1.000 | 8 | 16 | 0 | 0 | 256 |" in md
    assert "| `void lbm::k_copy16` | 2 | 0.500 | 0.500 |" in md
    assert "k_init" not in md
