"""Many independent boxes in one context: the batched launch (one launch
per step over every (box, tile) pair) and graph replay of captured steps.

- The batched schedule and graph replays compute the same per-node
  arithmetic as one launch per box: populations bit-identical, for every
  storage form, with and without stochastic rounding.
- The 256-box batch of uneven standing-wave boxes (edges from
  {16, 24, 32, 48, 64, 96}, k = 1..4, tau in [0.51, 1), log-uniform
  amplitude, seed 0): every box checked against the oracle for one step on
  sampled nodes (FP32, FP16-shifted with stochastic rounding), and seeded
  boxes (smallest, extreme tau, shortest wavelength, largest) checked
  against full oracle runs, the whole batch stepping through graph replays.
"""
import numpy as np
import pytest

from paper_1909_08406_amd import workloads as wl

pytestmark = pytest.mark.gpu

STORAGE_FORMS = [("f64", False), ("f32", False), ("f32", True), ("f32s", False), ("f16s", False), ("f16s", True),
                 ("bf16s", False), ("bf16s", True)]

# ragged boxes: odd edges, a single cell, tails of every tile size
RAGGED = [(3, 5, 7, 0.62), (16, 16, 16, 0.55), (1, 1, 1, 0.9), (5, 2, 9, 0.51), (24, 16, 8, 0.7), (2, 3, 1, 0.8),
          (13, 7, 5, 0.58)]


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    from paper_1909_08406_amd import lbm
    return lbm


def say(*a):
    print(*a, flush=True)


def ragged_fields():
    fields = [wl.random_state(b[0], b[1], b[2], seed=70 + i, amp_u=0.03, amp_rho=1e-3, amp_theta=1e-3)
              for i, b in enumerate(RAGGED)]
    return wl.concat(fields)


def make(L, boxes, cat, storage, sr, **tuning):
    _, _, th = L.lattice()
    ctx = L.init(boxes, cat[0], cat[1], cat[2], cat[3], cat[4] * th, storage=storage, stochastic=sr)
    if tuning:
        ctx.set_tuning(**tuning)
    return ctx


@pytest.mark.parametrize("storage,sr", STORAGE_FORMS)
def test_batched_schedule_identical_to_per_box(L, storage, sr):
    say("batched vs per-box", storage, sr)
    cat = ragged_fields()
    ref_ctx = make(L, RAGGED, cat, storage, sr, schedule="per_box")
    assert ref_ctx.tuning()["schedule"] == "per_box"
    ref_ctx.step(9)
    ref = ref_ctx.get_populations()
    ref_ctx.free()
    for v, x in [(0, 1), (3, 0), (5, 1), (1, 0)]:
        ctx = make(L, RAGGED, cat, storage, sr, variant=v, xcd_remap=x)
        assert ctx.tuning()["schedule"] == "batched"  # the default for several boxes
        ctx.step(9)
        got = ctx.get_populations()
        assert ctx.status() == 0
        ctx.free()
        assert np.array_equal(got, ref), (v, x)


@pytest.mark.parametrize("storage,sr", [("f64", False), ("f32", True), ("f16s", True), ("bf16s", False)])
@pytest.mark.parametrize("schedule", ["batched", "per_box"])
def test_graph_replays_identical_to_eager(L, storage, sr, schedule):
    """Several replays, with the program's own eager work and host
    synchronisations between them; every replay checked against eager
    launches. The stochastic-rounding step count comes from a device
    counter in replays, so a stale count would show up here."""
    say("graph replay", storage, sr, schedule)
    cat = ragged_fields()
    eager = make(L, RAGGED, cat, storage, sr, schedule=schedule)
    graph = make(L, RAGGED, cat, storage, sr, schedule=schedule, graph_steps=4)
    for rnd, n in enumerate([4, 9, 1, 8, 6]):
        eager.step(n)
        graph.step(n)
        a = eager.get_populations()
        b = graph.get_populations()
        assert np.array_equal(a, b), (rnd, n)
        np.testing.assert_array_equal(eager.totals(), graph.totals())
        assert graph.info()["steps_done"] == eager.info()["steps_done"]
    # changing the tuning drops the captured graphs and captures anew
    graph.set_tuning(graph_steps=2, variant=3)
    eager.step(5)
    graph.step(5)
    assert np.array_equal(eager.get_populations(), graph.get_populations())
    eager.free()
    graph.free()


def test_graph_steps_validation(L):
    cat = ragged_fields()
    ctx = make(L, RAGGED, cat, "f32", False)
    for bad in [dict(graph_steps=3), dict(graph_steps=-2), dict(graph_steps=2048), dict(schedule=2)]:
        with pytest.raises(L.LbmError):
            ctx.set_tuning(**bad)
    ctx.free()


# ---------------------------------------------------------------------------
# The 256-box batch
# ---------------------------------------------------------------------------

def batch_fields():
    specs = wl.batch_specs()
    cat = wl.concat([wl.batch_fields(s) for s in specs])
    boxes = [(s.nx, s.ny, s.nz, s.tau) for s in specs]
    return specs, boxes, cat


def kq_shells(orc):
    """Storage exponent per velocity without the run-level part: the
    documented round(-log2 w_shell)."""
    _, w, _ = orc.lattice()
    return np.round(-np.log2(w)).astype(int)


def fp16_spacing(h):
    """Spacing of FP16 numbers at |h| (normal range and subnormals)."""
    a = np.maximum(np.abs(h), 2.0 ** -14)
    return 2.0 ** (np.floor(np.log2(a)) - 10)


@pytest.mark.parametrize("storage,sr", [("f32", False), ("f16s", True)])
def test_batch_256_sampled_step_every_box(L, orc, storage, sr):
    """Every box of the batch: after 5 steps (graph replays and an eager
    step), one more step on sampled nodes computed by the oracle from the
    GPU's held state (pulled by the oracle's own map), against the GPU."""
    specs, boxes, cat = batch_fields()
    say("256-box batch sampled step", storage, sr, "nodes", int(sum(2 * b[0] * b[1] * b[2] for b in boxes)))
    ctx = make(L, boxes, cat, storage, sr, graph_steps=2)
    ctx.step(5)
    kamp = ctx.info()["shift_exp"]
    kq = kq_shells(orc) + kamp
    rng = np.random.default_rng(5)
    q = np.arange(41, dtype=np.int64)
    pulled, nodes_all = [], []
    for bi, b in enumerate(boxes):
        N = 2 * b[0] * b[1] * b[2]
        nodes = np.concatenate([[0, N - 1], rng.integers(0, N, 14)]).astype(np.int64)
        src = orc.pull_sources(b[0], b[1], b[2], nodes)
        pulled.append(ctx.gather(bi, (q[None, :] * N + src).reshape(-1)).reshape(-1, 41))
        nodes_all.append(nodes)
    ctx.step(1)
    worst = 0.0
    for bi, b in enumerate(boxes):
        N = 2 * b[0] * b[1] * b[2]
        got = ctx.gather(bi, (q[None, :] * N + nodes_all[bi][:, None]).reshape(-1)).reshape(-1, 41)
        ref = np.stack([orc.collide_node(p, 1.0 / b[3]) for p in pulled[bi]])
        _, w, _ = orc.lattice()
        if storage == "f16s":
            # one FP16 spacing of the stored deviation (stochastic rounding)
            # plus the FP32 arithmetic
            quant = fp16_spacing((ref - w) * 2.0 ** kq) * 2.0 ** (-kq)
            bound = quant + 5e-6 * np.max(np.abs(ref))
        else:
            bound = 5e-6 * np.max(np.abs(ref))
        r = float(np.max(np.abs(got - ref) / bound))
        worst = max(worst, r)
        assert r <= 1.0, (bi, specs[bi], r)
    say("  worst error / bound %.3f over %d boxes" % (worst, len(boxes)))
    assert ctx.status() == 0
    ctx.free()


def seeded_boxes(specs):
    """(box index, steps): the two smallest boxes, the smallest tau, the two
    largest tau, the shortest wavelength among small boxes for 1000 steps;
    the largest box for 100 steps (the oracle's time)."""
    N = np.array([2 * s.nx * s.ny * s.nz for s in specs])
    tau = np.array([s.tau for s in specs])
    lam = np.array([s.nx / s.k for s in specs])
    order = np.argsort(N, kind="stable")
    pick = [int(order[0]), int(order[1]), int(np.argmin(tau))]
    for i in np.argsort(-tau, kind="stable")[:2]:
        pick.append(int(i))
    small = [i for i in order if N[i] <= 100_000 and i not in pick]
    pick.append(int(min(small, key=lambda i: (lam[i], N[i]))))
    # and the median-size box
    pick.append(int(order[len(order) // 2]))
    out = [(i, 1000) for i in dict.fromkeys(pick)]
    out.append((int(order[-1]), 100))
    return out


_BATCH_RUNS = {}
CHECKPOINTS = (50, 200, 1000)


def batch_run(L, storage, boxes_wanted):
    """The whole batch stepped through graph replays to each checkpoint;
    the per-node moments of the wanted boxes at every checkpoint."""
    if storage not in _BATCH_RUNS:
        specs, boxes, cat = batch_fields()
        ctx = make(L, boxes, cat, storage, False, graph_steps=50)
        offs = np.concatenate([[0], np.cumsum([2 * b[0] * b[1] * b[2] for b in boxes])])
        out, done = {}, 0
        for t in CHECKPOINTS:
            ctx.step(t - done)
            done = t
            m = ctx.moments()
            for i in boxes_wanted:
                out[(i, t)] = m[:, offs[i]:offs[i + 1]].copy()
            del m
        assert ctx.status() == 0
        ctx.free()
        _BATCH_RUNS[storage] = out
    return _BATCH_RUNS[storage]


_SEEDED = seeded_boxes(wl.batch_specs())
_ORACLE = {}


def oracle_moments(orc, box, steps):
    """Oracle moments of one box at every checkpoint up to `steps`."""
    if (box, steps) not in _ORACLE:
        s = wl.batch_specs()[box]
        F = wl.batch_fields(s)
        _, _, th = orc.lattice()
        f = orc.init(s.nx, s.ny, s.nz, *F.absolute(th))
        _ORACLE[(box, 0)] = orc.moment_fields(f)
        done = 0
        for t in CHECKPOINTS:
            if t > steps:
                break
            f = orc.run(s.nx, s.ny, s.nz, 1.0 / s.tau, f, t - done)
            done = t
            _ORACLE[(box, t)] = orc.moment_fields(f)
    return _ORACLE


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("box,steps", _SEEDED)
def test_batch_256_seeded_box_vs_oracle(L, orc, box, steps, storage, tol):
    """One box of the 256-box batch against a full oracle run of that box
    alone: normwise moment error at each checkpoint up to `steps` (1e-12
    FP64, 1e-5 FP32); the error relative to the initial perturbation is
    printed as well."""
    specs = wl.batch_specs()
    s = specs[box]
    say("batch box", box, s, steps, storage)
    runs = batch_run(L, storage, [b for b, _ in _SEEDED])
    ref = oracle_moments(orc, box, steps)
    m0 = ref[(box, 0)]
    pert0 = float(np.max(np.abs(m0 - m0.mean(axis=1, keepdims=True))))
    for t in CHECKPOINTS:
        if t > steps:
            break
        m_ref = ref[(box, t)]
        mg = runs[(box, t)]
        err = float(np.max(np.abs(mg - m_ref)) / np.max(np.abs(m_ref)))
        say("  step %4d: normwise moment error %.2e (%.2e of the initial perturbation)"
            % (t, err, err * np.max(np.abs(m_ref)) / pert0))
        assert err <= tol, t
