"""Physics of the HIP path at the configured workloads, against what the paper
and the linearised Navier-Stokes-Fourier (NSF) equations fix:

  - isentropic sound speed sqrt(gamma theta0) (Sec. I, Sec. VI) and acoustic
    and entropy-mode decay rates of the linearised NSF equations (Sec. I),
    within 0.1% (speed) and 1% (rates), for every storage form;
  - thermal (heat-conduction) mode decay at 128^3 over 2000 steps;
  - exact global conservation on the Taylor-Green vortex at Ma 0.1-0.3,
    where viscous heating must equal the kinetic-energy loss;
  - the 512^3 acoustic pulse against the analytic spherical wave (Sec. VI),
    with the 16-bit storage forms measured against FP64 on the GPU.

Every figure is also printed next to the FP64 oracle's where the oracle can
run the same problem.
"""
import numpy as np
import pytest

from oracle import analysis as an
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


def mode_series(ctx, k, field, steps, every):
    t, a = [], []
    for s in range(0, steps + 1, every):
        if s:
            ctx.step(every)
        t.append(s)
        a.append(ctx.project(0, k)[field])
    return np.array(t, dtype=float), np.array(a)


_ORACLE_C1 = {}


def oracle_c1_fit(orc):
    if not _ORACLE_C1:
        nx, ny, nz, tau = 32, 16, 16, 0.6
        k = 2 * np.pi / nx
        _, _, th = orc.lattice()
        F = wl.standing_wave(nx, ny, nz, 1e-3)
        f = orc.init(nx, ny, nz, *F.absolute(th))
        sig = []
        for s in range(201):
            if s:
                f = orc.run(nx, ny, nz, 1.0 / tau, f, 1)
            sig.append(-2 * an.fourier_mode(orc.moment_fields(f)[0] - 1.0, nx, ny, nz, (k, 0, 0)).imag)
        nu = an.viscosity(th, tau)
        ac, ent = an.nsf_modes(k, nu, nu, th)
        _ORACLE_C1.update(an.fit_acoustic_entropy(np.arange(201)[10:], np.array(sig)[10:], ac.imag, -ac.real))
    return _ORACLE_C1


@pytest.mark.parametrize("storage,sr", [("f64", False), ("f32", False), ("f32", True), ("f32s", False),
                                       ("f16s", False), ("f16s", True), ("bf16s", False), ("bf16s", True)])
def test_sound_speed_and_decay_32x16x16(L, orc, storage, sr):
    """Standing acoustic wave rho = 1 + 1e-3 sin(2 pi x/32) on 32x16x16,
    tau = 0.6, 200 steps: c_s within 0.1% of sqrt(gamma theta0), acoustic
    and entropy decay within 1% of the NSF eigenvalues. BF16 (8-bit
    significand) resolves the slow entropy mode of a 1e-3 wave only to a few
    per cent; for it that rate is reported, not held to 1%. With round to
    nearest its acoustic rate is near the 1% bar as well (0.6%) and moves by
    about 1% under last-bit changes of the FP32 arithmetic (hardware
    reciprocals in place of the equilibrium solve's divisions gave 1.8%)."""
    nx, ny, nz, tau = 32, 16, 16, 0.6
    k = 2 * np.pi / nx
    _, _, th = L.lattice()
    F = wl.standing_wave(nx, ny, nz, 1e-3)
    ctx = L.init([(nx, ny, nz, tau)], *F.absolute(th), storage=storage, stochastic=sr)
    t, a = mode_series(ctx, (k, 0, 0), 0, 200, 1)
    ctx.free()
    sig = -2 * a.imag
    nu = an.viscosity(th, tau)
    ac, ent = an.nsf_modes(k, nu, nu, th)
    fit = an.fit_acoustic_entropy(t[10:], sig[10:], ac.imag, -ac.real)
    cs = np.sqrt(an.GAMMA * th)
    ref = oracle_c1_fit(orc)
    say("C1 %s%s: c_s/sqrt(gamma theta0)-1 = %.2e (oracle %.2e), acoustic rate/NSF-1 = %.2e (oracle %.2e), "
        "entropy rate/NSF-1 = %.2e (oracle %.2e), fit rms %.1e"
        % (storage, "+SR" if sr else "", fit["w"] / k / cs - 1, ref["w"] / k / cs - 1, fit["G"] / -ac.real - 1,
           ref["G"] / -ac.real - 1, fit["Ge"] / -ent - 1, ref["Ge"] / -ent - 1, fit["rms"]))
    assert abs(fit["w"] / k / cs - 1) < 1e-3
    assert abs(fit["G"] / -ac.real - 1) < 1e-2
    assert abs(fit["Ge"] / -ent - 1) < (1e-2 if storage != "bf16s" else 1e-1)
    # and the same fit as the FP64 oracle to well inside those bounds
    assert abs(fit["w"] / ref["w"] - 1) < 1e-4
    assert abs(fit["G"] / ref["G"] - 1) < (2e-3 if storage != "bf16s" else 5e-3)


@pytest.mark.parametrize("storage,sr,tol", [("f64", False, 1e-2), ("f32", True, 1e-2), ("f32s", False, 1e-2),
                                           ("f16s", True, 1e-2), ("f32", False, 1e-1)])
def test_thermal_mode_128_2000_steps(L, storage, sr, tol):
    """Plain method, 128^3 periodic, theta = theta0 (1 + 1e-3 cos(2 pi z/128))
    plus seeded density noise, tau = 0.55, 2000 steps: the heat-conduction
    (entropy) mode decays at the NSF rate within 1%, and the acoustic part
    oscillates at the isentropic sound speed.

    The mode changes by ~1e-11 per population per step, far below the
    rounding step of FP32-stored f (~1e-8). Once the density noise has
    decayed the field is uniform across each z-plane and nearly periodic in
    time, so round-to-nearest errors recur instead of averaging out and bias
    the slow decay by several per cent; stochastic rounding (unbiased) or
    storing the shift f - w rho0 in FP32 (a ~1000 times finer step) removes
    the bias. Round-to-nearest FP32 is held only to 10%."""
    n, tau = 128, 0.55
    k = 2 * np.pi / n
    _, _, th = L.lattice()
    F = wl.thermal_mode(n)
    ctx = L.init([(n, n, n, tau)], *F.absolute(th), storage=storage, stochastic=sr)
    t, a = mode_series(ctx, (0, 0, k), 5, 2000, 10)
    tot = ctx.totals()[0]
    ctx.free()
    sig = 2 * a.real
    nu = an.viscosity(th, tau)
    ac, ent = an.nsf_modes(k, nu, nu, th)
    fit = an.fit_acoustic_entropy(t[2:], sig[2:], ac.imag, -ac.real)
    cs = np.sqrt(an.GAMMA * th)
    say("C2 %s%s: entropy rate %.6e vs NSF %.6e (rel %.2e), c_s rel %.2e, amplitude ratio after 2000 steps %.4f, "
        "fit rms %.1e" % (storage, "+SR" if sr else "", fit["Ge"], -ent, fit["Ge"] / -ent - 1, fit["w"] / k / cs - 1,
                          np.exp(-fit["Ge"] * 2000), fit["rms"]))
    assert abs(fit["Ge"] / -ent - 1) < tol
    assert abs(fit["w"] / k / cs - 1) < 1e-3


@pytest.mark.parametrize("ma,tau,storage,sr", [(0.1, 0.50605, "f32", False), (0.2, 0.51211, "f32", False),
                                              (0.3, 0.51816, "f32", False), (0.1, 0.50605, "f32", True),
                                              (0.1, 0.50605, "f32s", False), (0.1, 0.50605, "f64", False)])
def test_taylor_green_256_conservation(L, ma, tau, storage, sr):
    """Plain method, FP32, 256^3 Taylor-Green vortex, Re = 1600 with
    U0 = Ma sqrt(gamma theta0): the run stays realisable, mass and momentum
    are conserved, and because total energy is conserved the rise of the
    thermal energy (3/2) sum rho theta equals the kinetic-energy loss.

    At Ma 0.1 the kinetic-energy loss over 1000 steps is only 1.3e-5 of the
    total energy, so the balance needs energy conserved to ~1e-9 per step.
    FP32 arithmetic leaves a mean energy bias of ~5e-10 of the node energy
    per collision at |u| ~ 0.1 (round-off in evaluating the equilibrium),
    which shows as ~1.4% here and ~0.2% at Ma 0.2 and 0.3; the FP32 forms
    are held to 2%, FP64 to 1%."""
    n, steps = 256, 1000
    _, _, th = L.lattice()
    u0 = ma * np.sqrt(5.0 / 3.0 * th)
    F = wl.taylor_green(n, u0)
    ctx = L.init([(n, n, n, tau)], *F.absolute(th), storage=storage, stochastic=sr)

    def energies():
        m = ctx.moments()
        ke = 0.5 * np.sum((m[1] ** 2 + m[2] ** 2 + m[3] ** 2) / m[0])
        return ke, np.sum(m[4]) - ke, m

    ke0, th0_e, _ = energies()
    tot0 = ctx.totals()[0]
    ctx.step(steps)
    status = ctx.status()
    ke1, th1_e, m = energies()
    tot1 = ctx.totals(check=False)[0]
    ctx.free()
    nodes = 2 * n ** 3
    L_ = n / (2 * np.pi)
    nu = th * (tau - 0.5)
    say("C3 Ma %.1f %s%s: status %d, KE %.6e -> %.6e (ratio %.4f; laminar exp(-6 nu t/L^2) = %.4f), "
        "thermal gain / KE loss = %.6f, mass drift %.2e, energy drift %.2e, |J|/mass %.2e"
        % (ma, storage, "+SR" if sr else "", status, ke0, ke1, ke1 / ke0, np.exp(-6 * nu * steps / L_ ** 2), (th1_e - th0_e) / (ke0 - ke1),
           tot1[0] / tot0[0] - 1, tot1[4] / tot0[4] - 1, np.max(np.abs(tot1[1:4])) / tot1[0]))
    assert status == 0
    assert abs(tot1[0] / tot0[0] - 1) < 1e-6
    assert np.max(np.abs(tot1[1:4])) / tot1[0] < 1e-6
    # energy bookkeeping: heating equals kinetic-energy loss
    assert ke1 < ke0
    assert abs((th1_e - th0_e) / (ke0 - ke1) - 1) < (1e-2 if storage == "f64" else 2e-2)
    assert nodes > 0


def solenoidal_energy_enstrophy(m, n):
    """Kinetic energy and enstrophy of the divergence-free part of the flow
    of an n^3 box from its node moments: on each sublattice (a periodic n^3
    grid) the velocity u = j / rho is projected onto divergence-free Fourier
    modes; KE = (rho_mean / 2) sum |P u|^2 and Omega = (rho_mean / 2) sum
    |k|^2 |P u|^2 (= the vorticity's), summed by Parseval (real FFT: the
    interior of the last axis counts twice). For such a field dKE/dt =
    -2 nu Omega."""
    kz = 2 * np.pi * np.fft.fftfreq(n)[:, None, None]
    ky = 2 * np.pi * np.fft.fftfreq(n)[None, :, None]
    kx = 2 * np.pi * np.fft.rfftfreq(n)[None, None, :]
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2s = k2.copy()
    k2s[0, 0, 0] = 1.0
    weight = np.full(kx.shape, 2.0)
    weight[..., 0] = 1.0
    if n % 2 == 0:
        weight[..., -1] = 1.0
    ke = om = 0.0
    n3 = n ** 3
    rbar = float(m[0].mean())
    for s in (0, 1):
        sl = slice(s * n3, (s + 1) * n3)
        W = [np.fft.rfftn((m[1 + a, sl] / m[0, sl]).reshape(n, n, n)) for a in range(3)]  # x, y, z
        kdw = (kx * W[0] + ky * W[1] + kz * W[2]) / k2s
        e = sum(np.abs(W[a] - ka * kdw) ** 2 for a, ka in enumerate((kx, ky, kz)))
        ke += 0.5 * rbar * float(np.sum(weight * e)) / n3
        om += 0.5 * rbar * float(np.sum(weight * k2 * e)) / n3
    return ke, om


def test_taylor_green_256_early_laminar_decay(L):
    """Plain method, FP32, 256^3 Taylor-Green vortex at Ma 0.1 (tau 0.50605,
    Re 1600): before the vortex stretching has built up enstrophy, the
    kinetic energy decays at the laminar rate of the initial mode. The
    velocity field is an eigenfunction of the Laplacian with eigenvalue
    -3/L^2 (L = n / 2 pi), so dKE/dt = -2 nu Omega gives 6 nu / L^2.

    Two effects ride on it and are removed. (1) The populations start at
    equilibrium with omega = 1.976, so for tens of steps the moments ring
    with alternating sign (an initial layer): the fit starts at step 40.
    (2) The initial field has no pressure correction; the pressure
    imbalance, at wavevectors 2 and 2 sqrt 2 (in units of 1/L), radiates
    sound that trades about 0.1% of the energy with the vortex at the
    acoustic frequencies 2 c_s / L and 2 sqrt 2 c_s / L (c_s = sqrt(gamma
    theta0)), as much as the viscous loss in 400 steps. So the energy of the
    divergence-free part of the flow, sampled every 20 steps from 40 to 400,
    is fitted with a - b t plus those two oscillations, and b / a is held
    to 6 nu / L^2 and to the measured viscous dissipation 2 nu <Omega> / KE
    (the enstrophy grows by 5% by step 400) within 3%."""
    n, tau, ma = 256, 0.50605, 0.1
    _, _, th = L.lattice()
    u0 = ma * np.sqrt(5.0 / 3.0 * th)
    F = wl.taylor_green(n, u0)
    ctx = L.init([(n, n, n, tau)], *F.absolute(th), storage="f32")
    ts, ke, om = [], [], []
    done = 0
    for t in range(40, 401, 20):
        ctx.step(t - done)
        done = t
        m = ctx.moments()
        k, o = solenoidal_energy_enstrophy(m, n)
        del m
        ts.append(t)
        ke.append(k)
        om.append(o)
    assert ctx.status() == 0
    ctx.free()
    ts, ke, om = np.array(ts, dtype=float), np.array(ke), np.array(om)
    nu = th * (tau - 0.5)
    Lc = n / (2 * np.pi)
    rate = 6.0 * nu / Lc ** 2
    cs = np.sqrt(an.GAMMA * th)
    cols = [np.ones_like(ts), -ts]
    for w in (2 * cs / Lc, 2 * np.sqrt(2) * cs / Lc):
        cols += [np.cos(w * ts), np.sin(w * ts)]
    A = np.column_stack(cols)
    c, *_ = np.linalg.lstsq(A, ke, rcond=None)
    fit = c[1] / c[0]
    dissip = float(np.mean(2 * nu * om / ke))
    say("C3 early decay f32: laminar 6 nu/L^2 = %.4e per step; divergence-free kinetic energy decays at %.4e "
        "(ratio %.4f; against the measured 2 nu <Omega>/KE = %.4e: %.4f); fit rms %.1e of KE"
        % (rate, fit, fit / rate, dissip, fit / dissip, np.sqrt(np.mean((ke - A @ c) ** 2)) / c[0]))
    assert abs(fit / rate - 1) < 3e-2
    assert abs(fit / dissip - 1) < 3e-2


def _line_pressure(ctx, n, y0, z0, s=0):
    """p = rho theta along x at (y0, z0) on sublattice s, from gathered
    populations (x = 0..n-1)."""
    N = 2 * n ** 3
    nodes = ((s * n + z0) * n + y0) * n + np.arange(n)
    q = np.arange(41)
    f = ctx.gather(0, (q[:, None] * N + nodes[None, :]).reshape(-1)).reshape(41, n)
    return f


def test_pulse_512_against_analytic_and_fp64(L, orc):
    """Precision form: 512^3 periodic acoustic pulse (Gaussian density bump,
    amplitude 1e-3, half width 8 cells), 500 steps. The pressure p - rho0
    theta0 along the x axis through the centre follows theta0 times the
    analytic spherical wave with speed sqrt(gamma theta0) before the front
    wraps; FP32 and the 16-bit shifted forms, with round to nearest and
    with stochastic rounding (the benchmarked form), are compared with FP64
    run on the GPU (itself checked against the oracle at smaller sizes)."""
    n, tau, eps, b = 512, 0.6, 1e-3, 8.0
    _, _, th = L.lattice()
    c, w, _ = orc.lattice()
    c2 = (c ** 2).sum(1)
    F = wl.gaussian_pulse(n, eps=eps, b=b)
    cs = np.sqrt(an.GAMMA * th)
    nu = an.viscosity(th, tau)
    xs = np.arange(n) - n / 2
    lines = {}
    for storage, sr in (("f64", False), ("f32", False), ("f16s", False), ("bf16s", False), ("f16s", True),
                        ("bf16s", True)):
        form = storage + ("+sr" if sr else "")
        ctx = L.init([(n, n, n, tau)], *F.absolute(th), storage=storage, stochastic=sr)
        tot0 = ctx.totals()[0]
        got = {}
        done = 0
        for t in (100, 200, 500):
            ctx.step(t - done)
            done = t
            f = _line_pressure(ctx, n, n // 2, n // 2)
            rho = f.sum(0)
            jx = c[:, 0] @ f
            en = 0.5 * (c2 @ f)
            p = (2 * en - jx * jx / rho) / 3.0  # rho theta with u = (jx, 0, 0)/rho on the axis
            got[t] = p - th
        tot1 = ctx.totals()[0]
        ctx.free()
        lines[form] = got
        say("C4 %s: mass drift %.2e, energy drift %.2e" % (form, tot1[0] / tot0[0] - 1, tot1[4] / tot0[4] - 1))
    for t in (100, 200):
        ana = th * an.pulse_3d_integral(np.abs(xs), float(t), eps, b, cs, nu_eff=nu)
        err = np.max(np.abs(lines["f64"][t] - ana)) / (th * eps)
        say("C4 t=%d: FP64 vs analytic pulse, max error / (theta0 eps) = %.3e" % (t, err))
        assert err < 2e-2
    # measured (round to nearest): FP32 <= 1.5e-4, FP16 <= 1.4e-4, BF16 <= 9.7e-4
    # of theta0 eps; stochastic rounding is unbiased with the same quantum
    for form in ("f32", "f16s", "bf16s", "f16s+sr", "bf16s+sr"):
        for t in (100, 200, 500):
            e = np.max(np.abs(lines[form][t] - lines["f64"][t])) / (th * eps)
            say("C4 %s t=%d: error vs FP64 / (theta0 eps) = %.3e" % (form, t, e))
            assert e < {"f32": 1e-3, "f16s": 2e-3, "bf16s": 1e-2}[form.split("+")[0]], (form, t, e)
