"""Parity of the HIP path (through the C-ABI) against the FP64 CPU oracle.

Bars: integer streaming maps bit-exact; moments after the run within 1e-12
relative (FP64) and 1e-5 relative (FP32), as the normwise relative error of
the moment vector (rho, jx, jy, jz, E): max|m_gpu - m_ref| / max|m_ref|
over all five fields and all nodes. A second, per-field gate measures each
field against the size of its own perturbation,
max|m_gpu - m_ref| / max|m_ref - mean(m_ref)| (the three momentum
components share the largest of their perturbations). Its floors are set by
rounding, not by the method: two FP64 computations that sum in different
orders differ by ~1e-16 of the populations per node and step, which over
200 steps is ~1e-14 absolute in j, i.e. ~1e-11 of an acoustic momentum of
~4e-4 (measured 1.7e-11, bar 2e-10); FP32 storage rounds each population to
~1e-9 per step, whose smooth-field accumulation over 200 steps reaches
~1e-7 absolute (measured 8.9e-5 of the momentum perturbation, bar 1e-3).

The GPU holds post-collision populations (pull scheme) while the oracle
holds pre-collision ones (collide then push); their conserved moments are
equal, and the oracle's collide_field() of its state gives the GPU's
populations, which are compared element by element.
"""
import os
import time

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


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def moment_errors(m_gpu, m_ref):
    """Per-field relative errors of rho, jx, jy, jz, E."""
    return [rel_err(m_gpu[k], m_ref[k]) if np.max(np.abs(m_ref[k])) > 0 else float(np.max(np.abs(m_gpu[k])))
            for k in range(5)]


def moment_error(m_gpu, m_ref, storage=None):
    """The gated figure: normwise relative error of the moment vector."""
    return rel_err(m_gpu, m_ref)


def perturbation_errors(m_gpu, m_ref, m_init=None):
    """Per field: max|m_gpu - m_ref| over the size of the field's
    perturbation max|m - mean(m)|, the larger of the reference's at the
    checkpoint and at the start (m_init: a wave's density perturbation
    passes through zero twice a period); jx, jy and jz share the largest
    momentum perturbation (a field may be uniformly zero)."""
    def pert(m):
        return [float(np.max(np.abs(m[k] - m[k].mean()))) for k in range(5)]
    p = pert(m_ref)
    if m_init is not None:
        p = [max(a, b) for a, b in zip(p, pert(m_init))]
    pj = max(p[1:4])
    den = [p[0], pj, pj, pj, p[4]]
    return [float(np.max(np.abs(m_gpu[k] - m_ref[k]))) / den[k] for k in range(5)]


def oracle_init_moments(orc, dims, F):
    _, _, th = orc.lattice()
    return orc.moment_fields(orc.init(*dims, *F.absolute(th)))


# per-field perturbation bars (see the module docstring)
PERT_BAR = {"f64": 2e-10, "f32": 1e-3}


def oracle_run(orc, dims, tau, F, steps):
    nx, ny, nz = dims
    _, _, th = orc.lattice()
    f = orc.init(nx, ny, nz, *F.absolute(th))
    return orc.run(nx, ny, nz, 1.0 / tau, f, steps)


def gpu_run(L, dims, tau, F, steps, storage, **kw):
    _, _, th = L.lattice()
    ctx = L.init([(*dims, tau)], *F.absolute(th), storage=storage, **kw)
    ctx.step(steps)
    return ctx


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 2, 2), (3, 2, 1), (5, 7, 3), (17, 9, 5), (32, 16, 16)])
def test_pull_map_bit_exact(L, orc, dims):
    say("pull map", dims)
    F = wl.standing_wave(*dims, amp=0.0)
    ctx = gpu_run(L, dims, 0.6, F, 0, "f32")
    got = ctx.debug_pull_map(0)
    ctx.free()
    assert np.array_equal(got, orc.pull_map(*dims))


@pytest.mark.parametrize("storage,sr", [("f64", False), ("f32", False), ("f16s", True), ("bf16s", False)])
def test_free_streaming_is_the_oracle_permutation(L, orc, storage, sr):
    """Collisionless streaming (lbm_stream_free) moves every held value along
    its link unchanged: after 3 steps the populations equal the oracle's pull
    map applied three times to the initial ones, bit for bit, on boxes with
    a ragged tail and x extents from 1 to 17; the tuned launch variant runs
    the same permutation."""
    boxes = [(17, 9, 5, 0.6), (5, 7, 3, 0.7), (1, 2, 3, 0.55)]
    _, _, th = L.lattice()
    fields = [wl.random_state(b[0], b[1], b[2], seed=50 + i) for i, b in enumerate(boxes)]
    cat = wl.concat(fields)
    for variant in (0, 1, 3):
        ctx = L.init(boxes, cat[0], cat[1], cat[2], cat[3], cat[4] * th, storage=storage, stochastic=sr)
        ctx.set_tuning(variant=variant, xcd_remap=1)
        f0 = ctx.get_populations()
        steps0 = ctx.info()["steps_done"]
        ctx.stream_free(3)
        f1 = ctx.get_populations()
        assert ctx.info()["steps_done"] == steps0
        ctx.free()
        off = 0
        for b in boxes:
            N = 2 * b[0] * b[1] * b[2]
            src = orc.pull_map(*b[:3]).reshape(41, N)
            g0 = f0[off * 41:(off + N) * 41].reshape(41, N)
            g1 = f1[off * 41:(off + N) * 41].reshape(41, N)
            want = g0
            for _ in range(3):
                want = np.take_along_axis(want, src, axis=1)
            assert np.array_equal(g1, want), (storage, variant, b)
            off += N


def test_device_copy(L):
    """lbm_device_copy (the measurement copy kernel) copies exactly the
    requested bytes, ragged tails included, and nothing beyond them; bad
    arguments are rejected before any launch."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(5)
    for nbytes in (16, 16 * 1023, 16 * (4 * 256 * 3 + 5)):
        a = torch.randint(0, 256, (nbytes + 256,), dtype=torch.uint8, device="cuda", generator=g)
        b = torch.zeros_like(a)
        L.device_copy(a.data_ptr(), b.data_ptr(), nbytes)
        torch.cuda.synchronize()
        assert torch.equal(b[:nbytes], a[:nbytes]), nbytes
        assert not bool(b[nbytes:].any()), nbytes
    for src, dst, n in ((a.data_ptr() + 8, b.data_ptr(), 16), (a.data_ptr(), b.data_ptr(), 24),
                        (a.data_ptr(), a.data_ptr() + 16, 32)):
        with pytest.raises(L.LbmError) as e:
            L.device_copy(src, dst, n)
        assert e.value.code == L.E_ARG


def test_init_equilibrium_matches_oracle(L, orc):
    """The closed-form partition-function Newton (GPU) and the generic 5x5
    Newton (oracle) give the same entropic equilibrium, up to Ma ~ 0.4."""
    dims = (7, 5, 3)
    say("init equilibrium", dims)
    F = wl.random_state(*dims, seed=21, amp_rho=0.2, amp_u=0.25, amp_theta=0.1)
    ctx = gpu_run(L, dims, 0.6, F, 0, "f64")
    g = ctx.get_populations().reshape(41, -1)
    ctx.free()
    _, _, th = orc.lattice()
    f = orc.init(*dims, *F.absolute(th))
    assert np.max(np.abs(g - f)) < 2e-15


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_standing_wave_32x16x16_200_steps(L, orc, storage, tol):
    """Plain method on a 32x16x16 box, rho = 1 + 1e-3 sin(2 pi x/32),
    tau = 0.6, 200 steps."""
    dims, tau, steps = (32, 16, 16), 0.6, 200
    say("standing wave", storage, dims, steps)
    F = wl.standing_wave(*dims, amp=1e-3)
    ctx = gpu_run(L, dims, tau, F, steps, storage)
    m_gpu = ctx.moments()
    g = ctx.get_populations().reshape(41, -1)
    ctx.free()
    f = oracle_run(orc, dims, tau, F, steps)
    m_ref = orc.moment_fields(f)
    errs = moment_errors(m_gpu, m_ref)
    # density error relative to the initial wave amplitude (stricter)
    drho = float(np.max(np.abs(m_gpu[0] - m_ref[0]))) / 1e-3
    g_ref = orc.collide_field(*dims, 1.0 / tau, f)
    perr = rel_err(g, g_ref)
    pe = perturbation_errors(m_gpu, m_ref, oracle_init_moments(orc, dims, F))
    say("  per-field moment errors", ["%.2e" % e for e in errs], "normwise %.2e" % rel_err(m_gpu, m_ref),
        "per-field / perturbation", ["%.2e" % e for e in pe],
        "density error / amplitude %.2e" % drho, "population error %.2e" % perr)
    assert moment_error(m_gpu, m_ref, storage) <= tol
    assert max(pe) <= PERT_BAR[storage], pe
    # measured: FP64 2.4e-11 and 1.5e-13, FP32 1.2e-4 and 1.7e-7
    assert drho <= (5e-10 if storage == "f64" else 1e-3)
    assert perr <= (5e-12 if storage == "f64" else 3e-6)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("amp_u", [0.05, 0.2])
def test_random_state_ragged_box(L, orc, storage, tol, amp_u):
    """Independent random nodes (up to |u| ~ 0.35, i.e. Ma ~ 0.5) on a
    13x7x5 box: 910 nodes, four tiles of 256 and a ragged tail."""
    dims, tau, steps = (13, 7, 5), 0.55, 30
    say("random state", storage, amp_u, dims)
    F = wl.random_state(*dims, seed=5, amp_u=amp_u)
    ctx = gpu_run(L, dims, tau, F, steps, storage)
    m_gpu = ctx.moments()
    g = ctx.get_populations().reshape(41, -1)
    assert ctx.status() == 0
    ctx.free()
    f = oracle_run(orc, dims, tau, F, steps)
    m_ref = orc.moment_fields(f)
    errs = moment_errors(m_gpu, m_ref)
    pe = perturbation_errors(m_gpu, m_ref, oracle_init_moments(orc, dims, F))
    say("  per-field moment errors", ["%.2e" % e for e in errs], "normwise %.2e" % rel_err(m_gpu, m_ref),
        "per-field / perturbation", ["%.2e" % e for e in pe])
    assert moment_error(m_gpu, m_ref, storage) <= tol
    # measured: FP64 <= 2.8e-13, FP32 <= 4.7e-6 of the perturbations
    assert max(pe) <= (5e-12 if storage == "f64" else 1e-4), pe
    assert rel_err(g, orc.collide_field(*dims, 1.0 / tau, f)) <= tol


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_several_boxes_in_one_context(L, orc, storage):
    boxes = [(5, 3, 2, 0.6), (8, 4, 4, 0.7), (3, 3, 3, 0.95), (1, 2, 3, 0.52)]
    say("multi-box", storage, boxes)
    _, _, th = L.lattice()
    fields = [wl.random_state(b[0], b[1], b[2], seed=30 + i) for i, b in enumerate(boxes)]
    cat = wl.concat(fields)
    ctx = L.init(boxes, cat[0], cat[1], cat[2], cat[3], cat[4] * th, storage=storage)
    ctx.step(12)
    m = ctx.moments()
    tot = ctx.totals()
    ctx.free()
    tol = 1e-12 if storage == "f64" else 1e-5
    off = 0
    for i, (b, F) in enumerate(zip(boxes, fields)):
        n = 2 * b[0] * b[1] * b[2]
        f = oracle_run(orc, b[:3], b[3], F, 12)
        m_ref = orc.moment_fields(f)
        assert moment_error(m[:, off:off + n], m_ref, storage) <= tol, i
        t_ref = orc.totals(f)
        assert abs(tot[i, 0] / t_ref[0] - 1) <= tol and abs(tot[i, 4] / t_ref[4] - 1) <= tol
        off += n


@pytest.mark.parametrize("case,tol", [("wave", 2e-15), ("random", 2e-15)])
def test_fp64_conservation_and_totals(L, orc, case, tol):
    """Exact conservation of mass, momentum and energy (Sec. V) shows as
    global FP64 totals that drift only by rounding over 200 steps: measured
    <= 1.2e-18 (wave) and 2.5e-16 (random state) of the totals; the bar is
    about ten units of the last place of a sum of 16384 values of order
    one."""
    dims, tau = (32, 16, 16), 0.6
    say("conservation fp64", case, dims)
    if case == "wave":
        F = wl.standing_wave(*dims, amp=1e-3)
    else:
        F = wl.random_state(*dims, seed=3, amp_u=0.05)
    _, _, th = L.lattice()
    ctx = L.init([(*dims, tau)], *F.absolute(th), storage="f64")
    t0 = ctx.totals()[0]
    ctx.step(200)
    t1 = ctx.totals()[0]
    ctx.free()
    scale = np.array([t0[0]] * 4 + [t0[4]])
    drift = np.abs(t1 - t0) / scale
    say("  drift", drift)
    assert np.max(drift) < tol
    _, _, tho = orc.lattice()
    f = orc.init(*dims, *F.absolute(tho))
    ref = orc.totals(f)
    assert np.max(np.abs(t0 - ref) / scale) < 1e-13


STORAGE_FORMS = [("f64", False), ("f32", False), ("f32", True), ("f32s", False), ("f16s", False), ("f16s", True),
                 ("bf16s", False), ("bf16s", True)]


@pytest.mark.parametrize("storage,sr", STORAGE_FORMS)
def test_checkpoint_resume_is_bit_identical(L, storage, sr):
    dims, tau = (9, 6, 4), 0.58
    say("checkpoint", storage, "stochastic rounding" if sr else "")
    F = wl.random_state(*dims, seed=12, amp_u=0.03, amp_rho=1e-3, amp_theta=1e-3)
    _, _, th = L.lattice()
    a = L.init([(*dims, tau)], *F.absolute(th), storage=storage, stochastic=sr)
    a.step(10)
    ref = a.get_populations()
    a.free()
    b = L.init([(*dims, tau)], *F.absolute(th), storage=storage, stochastic=sr)
    b.step(4)
    snap = b.get_populations()
    steps = b.info()["steps_done"]
    b.free()
    c = L.init([(*dims, tau)], *F.absolute(th), storage=storage, stochastic=sr)
    c.set_populations(snap)
    c.set_step_counter(steps)
    c.step(6)
    got = c.get_populations()
    c.free()
    assert np.array_equal(got, ref)


def test_uniform_equilibrium_fixed_point(L):
    dims = (6, 5, 4)
    n = 2 * 6 * 5 * 4
    one = np.ones(n)
    _, _, th = L.lattice()
    for storage, tol in (("f64", 1e-14), ("f32", 4e-6)):
        ctx = L.init([(*dims, 0.6)], 1.1 * one, 0.02 * one, -0.01 * one, 0.005 * one, 1.01 * th * one,
                     storage=storage)
        f0 = ctx.get_populations()
        ctx.step(10)
        f1 = ctx.get_populations()
        ctx.free()
        assert np.max(np.abs(f1 - f0)) <= tol * np.max(f0), storage


def test_zero_and_negative_step_counts(L):
    """Zero steps (eager or with graph replays set up) leave the held state
    and the step count as they are; a negative count is rejected before any
    launch, and the state is again unchanged."""
    boxes = [(5, 3, 2, 0.6), (1, 1, 1, 0.7)]
    F = [wl.random_state(*b[:3], seed=3 + i) for i, b in enumerate(boxes)]
    _, _, th = L.lattice()
    cat = wl.concat(F)
    ctx = L.init(boxes, cat[0], cat[1], cat[2], cat[3], cat[4] * th, storage="f16s", stochastic=True)
    done = 0
    for g, n in ((0, 3), (4, 5)):  # 5 steps with graphs of 4: one replay, one eager step
        ctx.set_tuning(graph_steps=g)
        ctx.step(n)
        done += n
        f0 = ctx.get_populations()
        ctx.step(0)
        ctx.stream_free(0)
        for call in (ctx.step, ctx.stream_free):
            with pytest.raises(L.LbmError) as e:
                call(-1)
            assert e.value.code == L.E_ARG
        assert ctx.info()["steps_done"] == done
        assert np.array_equal(ctx.get_populations(), f0), g
    assert ctx.status() == 0
    ctx.free()


def test_nonfinite_state_is_flagged(L):
    """Unrealisable populations set from the host make the step flag the
    node; the kernel itself completes normally."""
    dims = (4, 4, 4)
    F = wl.standing_wave(*dims, amp=0.0)
    _, _, th = L.lattice()
    ctx = L.init([(*dims, 0.6)], *F.absolute(th), storage="f32")
    assert ctx.status() == 0
    f = ctx.get_populations().reshape(41, -1)
    ctx.set_populations(-f)  # negative density at every node
    ctx.step(1)
    assert ctx.status() == L.E_NONFINITE
    with pytest.raises(L.LbmError) as e:
        ctx.totals()
    assert e.value.code == L.E_NONFINITE
    ctx.free()


@pytest.mark.parametrize("sr", [False, True])
def test_fp16_range_overflow_is_flagged(L, sr):
    """A stored FP16 value that would leave the FP16 range is reported as
    non-finite, also with stochastic rounding, whose pair conversion rounds
    toward zero and would otherwise saturate at 65504 silently.

    Standing wave on 32x4x4 (amplitude 1e-3, tau 0.6): the largest scaled
    deviation in the velocity phase is about 2.1 times that of the initial
    density phase (3/5 of the bump is acoustic; the |c| = 2 shell carries
    u.c/theta). The automatic shift exponent leaves 2^6 of headroom; six
    more bits leave 1.7x, so the wave overflows within its first quarter
    period (11 steps), while four more (6.7x) stay in range. Every kernel
    completes normally."""
    dims = (32, 4, 4)
    F = wl.standing_wave(*dims, amp=1e-3)
    _, _, th = L.lattice()
    ctx = L.init([(*dims, 0.6)], *F.absolute(th), storage="f16s", stochastic=sr)
    k_auto = ctx.info()["shift_exp"]
    ctx.free()
    for extra, expect in ((4, 0), (6, L.E_NONFINITE)):
        ctx = L.init([(*dims, 0.6)], *F.absolute(th), storage="f16s", stochastic=sr, shift_exp=k_auto + extra)
        assert ctx.status() == 0
        ctx.step(16)
        st = ctx.status()
        say("fp16 range: sr %s, shift %d (+%d): status %d" % (sr, k_auto + extra, extra, st))
        ctx.free()
        assert st == expect, (sr, extra, st)


@pytest.mark.parametrize("storage,sr", [("f16s", False), ("f16s", True), ("bf16s", False), ("bf16s", True),
                                       ("f32s", False), ("f32", True)])
def test_shifted_storage_error_vs_fp64(L, orc, storage, sr):
    """Shifted storage of f - w rho0 (and FP32 with stochastic rounding) with
    FP32 arithmetic, against the FP64 oracle on the 32x16x16 standing wave
    after 200 steps."""
    dims, tau, steps = (32, 16, 16), 0.6, 200
    F = wl.standing_wave(*dims, amp=1e-3)
    ctx = gpu_run(L, dims, tau, F, steps, storage, stochastic=sr)
    info = ctx.info()
    m_gpu = ctx.moments()
    ctx.free()
    f = oracle_run(orc, dims, tau, F, steps)
    m_ref = orc.moment_fields(f)
    errs = moment_errors(m_gpu, m_ref)
    drho = float(np.max(np.abs(m_gpu[0] - m_ref[0]))) / 1e-3
    say("shifted", storage, "SR" if sr else "RNE", "k_amp", info["shift_exp"], "per-field moment errors",
        ["%.2e" % e for e in errs], "normwise %.2e" % rel_err(m_gpu, m_ref), "density error / amplitude %.2e" % drho)
    pe = perturbation_errors(m_gpu, m_ref, oracle_init_moments(orc, dims, F))
    say("  per-field / perturbation", ["%.2e" % e for e in pe])
    assert rel_err(m_gpu, m_ref) <= 1e-5
    # measured density error / amplitude: f16s 6.5e-4 (RNE) and 3.2e-4 (SR),
    # bf16s 4.7e-3 and 2.9e-3, f32s 3.3e-6, f32 with SR 6.3e-5
    assert drho <= {"f16s": 1e-2, "bf16s": 3e-2, "f32s": 1e-4, "f32": 1e-3}[storage]
    # per field against the perturbation: the storage quantum (FP16 of the
    # scaled deviation 2^-11, BF16 2^-8, FP32 of the deviation 2^-24 of w)
    assert max(pe) <= {"f16s": 1e-2, "bf16s": 5e-2, "f32s": 2e-4, "f32": 2e-3}[storage], pe


def _sampled_step_check(L, orc, dims, tau, F, storage, warm, nsample, tol, seed=0, sr=False, autotune=False,
                        entropic=False):
    """At full size: after `warm` steps, compute one more step for sampled
    nodes with the oracle (pull by the oracle's own map, then collide) from
    the GPU's held state, and compare with the GPU's next state. With
    `autotune` the checked step runs in the launch configuration the
    autotuner picks."""
    _, _, th = L.lattice()
    ctx = L.init([(*dims, tau)], *F.absolute(th), storage=storage, stochastic=sr, entropic=entropic)
    assert bool(ctx.info()["flags"] & L.FLAG_ENTROPIC) == entropic
    if autotune:
        say("  autotuned:", ctx.autotune()[0])
    ctx.step(warm)
    N = 2 * dims[0] * dims[1] * dims[2]
    rng = np.random.default_rng(seed)
    nodes = np.concatenate([[0, N - 1, N // 2 - 1, N // 2], rng.integers(0, N, nsample)]).astype(np.int64)
    src = orc.pull_sources(*dims, nodes)                       # [k, 41]
    q = np.arange(41, dtype=np.int64)
    pulled = ctx.gather(0, (q[None, :] * N + src).reshape(-1)).reshape(-1, 41)
    ctx.step(1)
    got = ctx.gather(0, (q[None, :] * N + nodes[:, None]).reshape(-1)).reshape(-1, 41)
    status = ctx.status()
    ctx.free()
    ref = np.stack([orc.collide_node(p, 1.0 / tau, entropic=entropic) for p in pulled])
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    # conservation by the GPU collision itself: moments of its output
    # against the moments of the pulled input, per node
    m_in = np.stack([orc.node_moments(p) for p in pulled])
    m_out = np.stack([orc.node_moments(g) for g in got])
    cons = float(np.max(np.abs(m_out - m_in)) / np.max(np.abs(m_in)))
    say("  sampled step error %.2e over %d nodes, collision conservation error %.2e" % (err, nodes.size, cons))
    assert status == 0
    assert err <= tol
    assert cons <= tol


_C2_ORACLE = {}


@pytest.mark.parametrize("sr", [False, True])
def test_thermal_mode_128_full_field_200_steps(L, orc, sr):
    """Plain method at the thermal-mode size, 128^3, theta = theta0 (1 +
    1e-3 cos(2 pi z/128)) plus seeded density noise (uniform 1e-4, seed 0),
    tau 0.55: FP32 storage (round to nearest and stochastic rounding)
    against a full FP64 oracle run of the same 4,194,304 nodes over 200
    steps, every node and moment. The oracle run (~1.3e9 node updates) is
    shared by both forms."""
    n, tau, steps = 128, 0.55, 200
    F = wl.thermal_mode(n)
    if not _C2_ORACLE:
        say("C2 oracle: 128^3, %d steps on %d threads" % (steps, orc.threads()))
        f = oracle_run(orc, (n, n, n), tau, F, steps)
        _C2_ORACLE["m"] = orc.moment_fields(f)
        del f
    m_ref = _C2_ORACLE["m"]
    ctx = gpu_run(L, (n, n, n), tau, F, steps, "f32", stochastic=sr)
    m_gpu = ctx.moments()
    assert ctx.status() == 0
    ctx.free()
    err = rel_err(m_gpu, m_ref)
    pe = perturbation_errors(m_gpu, m_ref, oracle_init_moments(orc, (n, n, n), F))
    say("C2 full field f32%s: normwise %.2e, per-field / perturbation %s" % ("+SR" if sr else "", err,
                                                                             ["%.2e" % e for e in pe]))
    # measured normwise 6.2e-8 (RNE) and 8.6e-8 (SR); per field <= 8e-4 of
    # the perturbation (the density noise of 1e-4 is its smallest)
    assert err <= 1e-5
    assert max(pe) <= 1e-2, pe


def test_sampled_full_size_thermal_mode_128(L, orc):
    """Plain method, FP32, 128^3 thermal mode with seeded density noise."""
    say("sampled 128^3 fp32")
    F = wl.thermal_mode(128)
    _sampled_step_check(L, orc, (128, 128, 128), 0.55, F, "f32", 5, 2000, 5e-7)  # measured 4.4e-8


def test_sampled_full_size_taylor_green_256(L, orc):
    """Plain method, FP32, 256^3 Taylor-Green vortex at Ma = 0.3."""
    say("sampled 256^3 fp32 TGV")
    _, _, th = L.lattice()
    F = wl.taylor_green(256, 0.3 * np.sqrt(5.0 / 3.0 * th))
    _sampled_step_check(L, orc, (256, 256, 256), 0.51816, F, "f32", 3, 2000, 2e-6)  # measured 1.5e-7


def test_sampled_full_size_pulse_512_f16s(L, orc):
    """Precision form at full size: 512^3 acoustic pulse, FP16-shifted
    storage, one step checked against the oracle on sampled nodes (to the
    FP16 quantum of the stored deviations)."""
    say("sampled 512^3 f16s pulse")
    F = wl.gaussian_pulse(512, eps=1e-3, b=8.0)
    _sampled_step_check(L, orc, (512, 512, 512), 0.6, F, "f16s", 2, 1000, 5e-9)  # measured 2.6e-10


def test_sampled_full_size_pulse_512_f16s_sr_autotuned(L, orc):
    """The benchmarked configuration: 512^3 acoustic pulse, FP16-shifted
    storage with stochastic rounding, in the launch shape the autotuner
    picks. Stochastic rounding moves a stored value by less than one FP16
    quantum of its scaled deviation (round to nearest: half), so its error
    is about twice the round-to-nearest one (measured 9.5e-10 against
    2.6e-10)."""
    say("sampled 512^3 f16s+sr pulse, autotuned")
    F = wl.gaussian_pulse(512, eps=1e-3, b=8.0)
    _sampled_step_check(L, orc, (512, 512, 512), 0.6, F, "f16s", 2, 1000, 1e-8, sr=True, autotune=True)  # 9.5e-10


def test_sampled_full_size_pulse_512_f16s_sr_entropic(L, orc):
    """The benchmarked entropic form: as above with the entropic path length,
    against the oracle's exact root of the entropy condition. Near
    equilibrium the kernel's closed form differs from that root by O(x^2)
    (x below the pulse amplitude 1e-3 here), which moves a population by
    O(x^2) |f_eq - f|. At this amplitude the path length itself changes the
    stored values by less than their FP16 quantum (the sampled error equals
    the BGK run's), so this checks the entropic kernel's streaming, moments
    and relaxation at full size in its own launch shape; the path length is
    checked far from equilibrium on small boxes."""
    say("sampled 512^3 f16s+sr pulse, entropic, autotuned")
    F = wl.gaussian_pulse(512, eps=1e-3, b=8.0)
    _sampled_step_check(L, orc, (512, 512, 512), 0.6, F, "f16s", 2, 1000, 1e-8, sr=True, autotune=True,
                        entropic=True)  # measured 9.5e-10


@pytest.mark.parametrize("storage,sr", STORAGE_FORMS)
def test_results_identical_across_launch_configurations(L, storage, sr):
    """Every step-kernel variant and tile mapping computes the same per-node
    arithmetic: the held state after a few steps must be bit-identical.
    A race in the streaming (reading a buffer that is being written) would
    show up as a dependence on the launch configuration."""
    dims, tau = (19, 11, 7), 0.57
    say("launch invariance", storage, sr)
    F = wl.random_state(*dims, seed=41, amp_u=0.03, amp_rho=1e-3, amp_theta=1e-3)
    _, _, th = L.lattice()
    ref = None
    for v in range(L.num_variants()):
        for x in (0, 1):
            ctx = L.init([(*dims, tau)], *F.absolute(th), storage=storage, stochastic=sr)
            ctx.set_tuning(v, x)
            ctx.step(7)
            got = ctx.get_populations()
            ctx.free()
            if ref is None:
                ref = got
            assert np.array_equal(got, ref), (v, x)


def test_autotune_keeps_state(L):
    dims = (24, 16, 8)
    F = wl.random_state(*dims, seed=2, amp_u=0.02)
    _, _, th = L.lattice()
    ctx = L.init([(*dims, 0.6)], *F.absolute(th), storage="f32")
    ctx.step(3)
    before = ctx.get_populations()
    best, table = ctx.autotune(reps=2)
    say("autotune", best, {k: round(v, 4) for k, v in table.items()})
    assert ctx.get_tuning() == best
    assert np.array_equal(ctx.get_populations(), before)
    ctx.step(2)
    ref = L.init([(*dims, 0.6)], *F.absolute(th), storage="f32")
    ref.step(5)
    assert np.array_equal(ctx.get_populations(), ref.get_populations())
    ctx.free()
    ref.free()


INIT_FORMS = [("f64", False, False), ("f32", False, False), ("f16s", True, False), ("bf16s", True, False),
              ("f32", False, True)]


@pytest.mark.parametrize("storage,sr,iso", INIT_FORMS)
def test_init_device_identical_to_host_init(L, storage, sr, iso):
    """lbm_init_device (fields in device memory, no host staging) builds the
    same populations and the same shift exponent as lbm_init, and the runs
    stay identical."""
    import torch
    boxes = [(9, 5, 3, 0.6), (16, 4, 2, 0.7), (1, 1, 1, 0.55)]
    cat = wl.concat([wl.random_state(b[0], b[1], b[2], seed=80 + i, amp_u=0.05, amp_rho=2e-3, amp_theta=2e-3)
                     for i, b in enumerate(boxes)])
    _, _, th = L.lattice()
    host = L.init(boxes, cat[0], cat[1], cat[2], cat[3], cat[4] * th, storage=storage, stochastic=sr, isothermal=iso)
    dev_fields = [torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
                  for a in (cat[0], cat[1], cat[2], cat[3], cat[4] * th)]
    dev = L.init_device(boxes, *dev_fields, storage=storage, stochastic=sr, isothermal=iso)
    assert dev.info()["shift_exp"] == host.info()["shift_exp"]
    assert np.array_equal(dev.get_populations(), host.get_populations())
    host.step(5)
    dev.step(5)
    assert np.array_equal(dev.get_populations(), host.get_populations())
    host.free()
    dev.free()


def test_init_device_rejects_unrealisable_fields(L):
    import torch
    dims = (6, 4, 3)
    F = wl.random_state(*dims, seed=3, amp_u=0.02)
    _, _, th = L.lattice()
    base = [np.array(a, dtype=np.float64) for a in F.absolute(th)]
    for k, i, bad in [(0, 5, 0.0), (0, 7, -1.0), (4, 11, -0.1), (1, 3, np.nan), (3, 0, np.inf)]:
        arrs = [a.copy() for a in base]
        arrs[k][i] = bad
        t = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in arrs]
        with pytest.raises(L.LbmError) as e:
            L.init_device([(*dims, 0.6)], *t, storage="f32")
        assert e.value.code == L.E_DOMAIN, (k, i, bad)


def test_workspace_too_small_is_nomem(L):
    """A caller workspace below lbm_workspace_size is refused with
    LBM_E_NOMEM before any device work."""
    import ctypes
    import torch
    dims = (8, 4, 4)
    F = wl.random_state(*dims, seed=4, amp_u=0.02)
    _, _, th = L.lattice()
    boxes = [(*dims, 0.6)]
    need = L.workspace_size(boxes, "f32")
    ws = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in F.absolute(th)]
    h = ctypes.c_void_p()
    op = L._opts("f32", L.TAU_LB, 1.0, 0, None)
    rc = L.lib().lbm_init(ctypes.byref(h), L._boxes(boxes), 1, ctypes.byref(op),
                          *[a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs], None,
                          ws.data_ptr(), need - 256)
    assert rc == L.E_NOMEM and not h.value


_ORACLE_RUNS = {}


def cached_oracle_moments(orc, key, dims, tau, F, steps):
    """Oracle moments of a run, computed once per key for all storage forms;
    large runs go in chunks of about 6e8 node updates, each reported."""
    if key not in _ORACLE_RUNS:
        _, _, th = orc.lattice()
        f = orc.init(*dims, *F.absolute(th))
        chunk = max(1, int(6e8 // (2 * dims[0] * dims[1] * dims[2])))
        done, t0 = 0, time.time()
        while done < steps:
            k = min(chunk, steps - done)
            f = orc.run(*dims, 1.0 / tau, f, k)
            done += k
            if done < steps or chunk < steps:
                say("oracle %s: %d of %d steps, %.0f s" % (key, done, steps, time.time() - t0))
        _ORACLE_RUNS[key] = orc.moment_fields(f)
    return _ORACLE_RUNS[key]


# per-field bars of the Taylor-Green parity; measured at most 6.0e-12 (FP64)
# and 9.0e-5 (FP32, 1000 steps at Ma 0.3)
TGV_PERT_BAR = {"f64": 1e-10, "f32": 1e-3}


@pytest.mark.parametrize("ma,tau,steps", [(0.1, 0.50605, 200), (0.2, 0.51211, 200), (0.3, 0.51816, 1000)])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_taylor_green_64_vs_oracle(L, orc, ma, tau, steps, storage, tol):
    """The Taylor-Green problem at 64^3 with the 256^3 runs' Mach number and
    tau (so Re = 400) against the oracle: all 1000 steps of the 256^3 runs
    at Ma 0.3, where the collision works farthest from the rest state
    (|u| up to 0.21), and 200 steps at Ma 0.1 and 0.2. Normwise moment error
    (1e-12 FP64, 1e-5 FP32) and per field against that field's own
    perturbation. (An oracle run of the 256^3 problem itself takes about 9
    minutes per 100 steps on 16 host cores; at that size the GPU state is
    checked one step at a time on sampled nodes.)"""
    n = 64
    _, _, th = L.lattice()
    F = wl.taylor_green(n, ma * np.sqrt(5.0 / 3.0 * th))
    ctx = L.init([(n, n, n, tau)], *F.absolute(th), storage=storage)
    ctx.step(steps)
    m = ctx.moments()
    assert ctx.status() == 0
    ctx.free()
    m_ref = cached_oracle_moments(orc, ("tgv64", ma, steps), (n, n, n), tau, F, steps)
    err = moment_error(m, m_ref)
    pe = perturbation_errors(m, m_ref, oracle_init_moments(orc, (n, n, n), F))
    say("TGV 64^3 Ma %.1f %s, %d steps: normwise moment error %.2e, per field / perturbation %s"
        % (ma, storage, steps, err, ["%.2e" % e for e in pe]))
    assert err <= tol
    assert max(pe) <= TGV_PERT_BAR[storage], pe


@pytest.mark.skipif(os.environ.get("LBM_FULL_ORACLE") != "1",
                    reason="about 10 minutes of host time (the oracle at 256^3); run with LBM_FULL_ORACLE=1")
def test_taylor_green_256_100_steps_vs_oracle(L, orc):
    """The 256^3 Taylor-Green problem itself (Ma 0.1, tau 0.50605, Re 1600),
    FP32 storage and arithmetic, against a full FP64 oracle run of all
    33,554,432 nodes over 100 steps: normwise moment error (1e-5) and per
    field against its own perturbation (1e-3, the 64^3 runs' bar). Skipped
    in the default run for its host time."""
    n, tau, steps, chunk = 256, 0.50605, 100, 10
    _, _, th = L.lattice()
    F = wl.taylor_green(n, 0.1 * np.sqrt(5.0 / 3.0 * th))
    ctx = gpu_run(L, (n, n, n), tau, F, steps, "f32")
    m_gpu = ctx.moments()
    assert ctx.status() == 0
    ctx.free()
    _, _, th_o = orc.lattice()
    f = orc.init(n, n, n, *F.absolute(th_o))
    m_init = orc.moment_fields(f)
    t0 = time.time()
    for done in range(0, steps, chunk):
        f = orc.run(n, n, n, 1.0 / tau, f, chunk)
        say("C3 256^3 oracle: %d of %d steps, %.0f s" % (done + chunk, steps, time.time() - t0))
    m_ref = orc.moment_fields(f)
    del f
    err = moment_error(m_gpu, m_ref)
    pe = perturbation_errors(m_gpu, m_ref, m_init)
    say("C3 256^3 f32, %d steps: normwise moment error %.2e, per field / perturbation %s"
        % (steps, err, ["%.2e" % e for e in pe]))
    assert err <= 1e-5
    assert max(pe) <= TGV_PERT_BAR["f32"], pe


PULSE_FORMS = [("f64", False, 1e-12), ("f32", False, 1e-5), ("f16s", True, 1e-5), ("bf16s", True, 3e-5)]


def pulse_vs_oracle(L, orc, n, storage, sr, tol, steps=80, tau=0.6):
    """The acoustic pulse recipe (eps 1e-3, b = 8, tau 0.6) on n^3 cells
    against the oracle: normwise moment error, and the same over the
    pulse's own perturbation (printed)."""
    _, _, th = L.lattice()
    F = wl.gaussian_pulse(n, eps=1e-3, b=8.0)
    ctx = L.init([(n, n, n, tau)], *F.absolute(th), storage=storage, stochastic=sr)
    ctx.step(steps)
    m = ctx.moments()
    assert ctx.status() == 0
    ctx.free()
    m_ref = cached_oracle_moments(orc, ("pulse", n, steps), (n, n, n), tau, F, steps)
    err = moment_error(m, m_ref)
    pert = float(np.max(np.abs(m_ref - m_ref.mean(axis=1, keepdims=True))))
    say("pulse %d^3, %d steps, %s%s: normwise moment error %.2e (%.2e of the perturbation)"
        % (n, steps, storage, "+SR" if sr else "", err, err * np.max(np.abs(m_ref)) / pert))
    assert err <= tol


@pytest.mark.parametrize("storage,sr,tol", PULSE_FORMS)
def test_pulse_128_vs_oracle(L, orc, storage, sr, tol):
    """The pulse on 128^3 for 80 steps against the oracle (1e-12 FP64, 1e-5
    FP32 and FP16-shifted with stochastic rounding, whose stored deviations
    carry ~11 bits of an amplitude of 1e-3; 3e-5 BF16-shifted, 3 bits
    fewer: measured 2.3e-6)."""
    pulse_vs_oracle(L, orc, 128, storage, sr, tol)


@pytest.mark.skipif(os.environ.get("LBM_FULL_ORACLE") != "1",
                    reason="about 5 minutes of host time (the oracle at 256^3); run with LBM_FULL_ORACLE=1")
@pytest.mark.parametrize("storage,sr,tol", PULSE_FORMS)
def test_pulse_256_vs_oracle(L, orc, storage, sr, tol):
    """The pulse on 256^3 for 80 steps against the oracle, same bars.
    Skipped in the default run for its host time."""
    pulse_vs_oracle(L, orc, 256, storage, sr, tol)


def test_padded_and_unpadded_boxes_in_one_context(L, orc):
    """16-bit storage pads a box's q-block stride when the block is a
    multiple of 1 MiB (64^3 cells in FP16: 2^20 bytes) and not otherwise
    (32x32x64: 2^18 bytes). A context mixing both: populations written and
    read back exactly in the host order; the batched schedule and graph
    replays bit-identical to per-box launches; the padded box's moments
    after 20 steps against the oracle (1e-5 normwise, FP16-shifted+SR)."""
    boxes = [(64, 64, 64, 0.6), (32, 32, 64, 0.7), (16, 8, 4, 0.55)]
    _, _, th = L.lattice()
    fields = [wl.random_state(b[0], b[1], b[2], seed=90 + i, amp_u=0.01, amp_rho=2e-3, amp_theta=2e-3)
              for i, b in enumerate(boxes)]
    args = wl.concat(fields)
    ctx = L.init(boxes, args[0], args[1], args[2], args[3], args[4] * th, storage="f16s", stochastic=True)
    f0 = ctx.get_populations()
    ctx.set_populations(f0)
    assert np.array_equal(ctx.get_populations(), f0)
    ctx.free()
    out = {}
    for name, tune in (("per_box", dict(schedule="per_box", graph_steps=0)),
                       ("batched", dict(schedule="batched", graph_steps=0)),
                       ("graph", dict(schedule="batched", graph_steps=4))):
        ctx = L.init(boxes, args[0], args[1], args[2], args[3], args[4] * th, storage="f16s", stochastic=True)
        ctx.set_tuning(**tune)
        ctx.step(20)
        out[name] = (ctx.get_populations(), ctx.moments())
        assert ctx.status() == 0
        ctx.free()
    assert np.array_equal(out["per_box"][0], out["batched"][0])
    assert np.array_equal(out["per_box"][0], out["graph"][0])
    # the padded 64^3 box against the oracle
    nx, ny, nz, tau = boxes[0]
    F = fields[0]
    f = orc.run(nx, ny, nz, 1 / tau, orc.init(nx, ny, nz, *F.absolute(th)), 20)
    m_ref = orc.moment_fields(f)
    m = out["per_box"][1][:, :2 * nx * ny * nz]
    err = float(np.max(np.abs(m - m_ref)) / np.max(np.abs(m_ref)))
    say("padded 64^3 box, FP16-shifted+SR, 20 steps: moment error %.2e" % err)
    assert err <= 1e-5
