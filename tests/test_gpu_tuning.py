"""The autotuner's wider search and its cache (lbm_autotune_ex): a second
context with the same key takes the cached choice without timing anything,
the cache survives in a file, and every choice computes the same results
bit for bit."""
import numpy as np
import pytest

from paper_1909_08406_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    from paper_1909_08406_amd import lbm
    return lbm


def say(*a):
    print(*a, flush=True)


def _ctx(L, boxes, storage="f16s", sr=True, seed=4):
    _, _, th = L.lattice()
    fields = [wl.random_state(b[0], b[1], b[2], seed=seed + i, amp_u=0.03, amp_rho=1e-3, amp_theta=1e-3)
              for i, b in enumerate(boxes)]
    cat = wl.concat(fields)
    return L.init(boxes, cat[0], cat[1], cat[2], cat[3], cat[4] * th, storage=storage, stochastic=sr)


def test_cached_choice_is_reused_without_timing(L):
    L.tune_cache_file(None)
    L.tune_cache_clear()
    box = [(64, 16, 8, 0.6)]
    a = _ctx(L, box)
    ra = a.autotune_ex(reps=2)
    say("first context:", ra)
    assert not ra["from_cache"] and ra["timed"] > 0 and ra["best_ms"] > 0
    assert L.tune_cache_count() == 1
    b = _ctx(L, box)
    rb = b.autotune_ex(reps=2)
    say("second context:", rb)
    assert rb["from_cache"] and rb["timed"] == 0
    for k in ("variant", "xcd_remap", "schedule", "graph_steps"):
        assert rb[k] == ra[k], k
    assert b.tuning() == a.tuning()
    # another shape or storage is another key
    c = _ctx(L, [(32, 16, 8, 0.6)])
    assert not c.autotune_ex(reps=1)["from_cache"]
    d = _ctx(L, box, storage="f32", sr=False)
    assert not d.autotune_ex(reps=1)["from_cache"]
    assert L.tune_cache_count() == 3
    # the tuned and the cached contexts step identically
    a.step(20)
    b.step(20)
    assert np.array_equal(a.get_populations(), b.get_populations())
    for x in (a, b, c, d):
        x.free()


def test_cache_file_round_trip(L, tmp_path):
    path = tmp_path / "tune.txt"
    L.tune_cache_clear()
    L.tune_cache_file(path)
    box = [(48, 8, 8, 0.7)]
    a = _ctx(L, box, storage="bf16s")
    ra = a.autotune_ex(reps=1)
    a.free()
    assert not ra["from_cache"]
    lines = path.read_text().splitlines()
    say("cache file:", lines)
    assert len(lines) == 1 and len(lines[0].split()) == 5
    # a fresh in-process cache loads the file and hits
    L.tune_cache_file(None)
    L.tune_cache_clear()
    assert L.tune_cache_count() == 0
    with open(path, "a") as fh:
        fh.write("malformed line\n")
    L.tune_cache_file(path)
    assert L.tune_cache_count() == 1
    b = _ctx(L, box, storage="bf16s")
    rb = b.autotune_ex(reps=1)
    b.free()
    assert rb["from_cache"] and (rb["variant"], rb["xcd_remap"], rb["schedule"], rb["graph_steps"]) == \
        (ra["variant"], ra["xcd_remap"], ra["schedule"], ra["graph_steps"])
    L.tune_cache_file(None)
    L.tune_cache_clear()


@pytest.mark.parametrize("storage,sr", [("f32", False), ("f16s", True)])
def test_wider_search_keeps_results_bit_identical(L, storage, sr):
    """Schedule and graph length chosen by the search, on several uneven
    boxes: the tuned context steps bit for bit like one left at the
    default launch (per-box schedule, eager launches), and the held state
    is not changed by the timing itself."""
    L.tune_cache_clear()
    boxes = [(24, 16, 8, 0.6), (16, 8, 8, 0.8), (7, 5, 3, 0.52), (32, 8, 4, 0.95)]
    a = _ctx(L, boxes, storage, sr)
    b = _ctx(L, boxes, storage, sr)
    b.set_tuning(schedule="per_box", graph_steps=0, variant=0, xcd_remap=0)
    f0 = a.get_populations()
    r = a.autotune_ex(reps=2, cache=False)
    say("wider search:", r, a.tuning())
    assert np.array_equal(a.get_populations(), f0)
    assert r["schedule"] in ("per_box", "batched") and r["graph_steps"] in (0, 16, 64)
    a.step(70)
    b.step(70)
    assert np.array_equal(a.get_populations(), b.get_populations())
    assert L.tune_cache_count() == 0
    a.free()
    b.free()
