"""The step kernel's per-node collision, run on the host through the C-ABI
(same templates, FP64 and FP32 arithmetic), against the FP64 oracle: the
collision of Sec. II towards the entropic equilibrium of Sec. V must match
and must conserve mass, momentum and energy to the rounding of the
arithmetic (no bias from how the weights round)."""
import numpy as np
import pytest

from paper_1909_08406_amd import lbm as L


def _moments(f, c):
    return np.array([f.sum(), *(f @ c), f @ (c ** 2).sum(1)])


def _cases(orc, n=12, seed=0):
    c, w, th = orc.lattice()
    rng = np.random.default_rng(seed)
    for i in range(n):
        amp = (1e-3, 1e-2, 0.1, 0.2)[i % 4]
        rho = 1 + rng.uniform(-0.01, 0.01)
        u = rng.uniform(-amp, amp, 3)
        eta = rng.uniform(-0.02, 0.02)
        feq = orc.equilibrium(rho, u, th * (1 + eta))[0]
        yield amp, feq * (1 + 1e-3 * rng.standard_normal(41))


@pytest.mark.parametrize("precision,newton,tol,cons_tol", [("f64", 3, 2e-15, 1e-15), ("f32", 1, 4e-8, 6e-8),
                                                            ("f32", 2, 4e-8, 6e-8)])
def test_host_collision_matches_oracle(orc, precision, newton, tol, cons_tol):
    c, _, _ = orc.lattice()
    for amp, f in _cases(orc):
        fin = f.astype(np.float32).astype(np.float64) if precision == "f32" else f
        g = L.collide_host(f, 1 / 0.6, precision, newton)
        ref = orc.collide_node(fin, 1 / 0.6)
        assert np.max(np.abs(g - ref)) < tol, amp
        assert np.max(np.abs(_moments(g, c) - _moments(fin, c))) < cons_tol, amp


def test_fp32_collision_has_no_drift_at_equilibrium(orc):
    """Repeated FP32 collisions of an equilibrium stay there to FP32 storage
    rounding: no systematic loss of mass or energy."""
    c, _, th = orc.lattice()
    f = orc.equilibrium(1.1, (0.02, -0.01, 0.005), th * 1.01)[0].astype(np.float32).astype(np.float64)
    g = f.copy()
    for _ in range(100):
        g = L.collide_host(g, 1 / 0.6, "f32", 1)
    m0, m1 = _moments(f, c), _moments(g, c)
    assert np.max(np.abs(g - f)) < 2e-8
    assert abs(m1[0] - m0[0]) < 5e-8 and abs(m1[4] - m0[4]) < 1e-7


@pytest.mark.parametrize("precision,newton,tol,cons_tol", [("f64", 3, 2e-15, 1e-15), ("f32", 1, 4e-8, 6e-8)])
def test_host_isothermal_collision_matches_oracle(orc, precision, newton, tol, cons_tol):
    """Isothermal model: the kernel's collision towards the equilibrium
    under mass and momentum only, against the oracle's; mass and momentum
    kept to the rounding of the arithmetic."""
    c, w, th = orc.lattice()
    for amp, f in _cases(orc, seed=3):
        fin = f.astype(np.float32).astype(np.float64) if precision == "f32" else f
        g = L.collide_host(f, 1 / 0.6, precision, newton, isothermal=True)
        ref = orc.collide_node(fin, 1 / 0.6, model="isothermal")
        assert np.max(np.abs(g - ref)) < tol, amp
        assert np.max(np.abs(_moments(g, c)[:4] - _moments(fin, c)[:4])) < cons_tol, amp
    # the rest state rho w is a fixed point
    g = L.collide_host(1.2 * w, 1 / 0.6, precision, newton, isothermal=True)
    assert np.max(np.abs(g - 1.2 * w)) < tol


@pytest.mark.parametrize("precision,newton,tol,cons_tol", [("f64", 0, 2e-15, 2e-15), ("f32", 0, 4e-8, 6e-8)])
def test_host_series_collision_matches_oracle(orc, precision, newton, tol, cons_tol):
    """Series equilibrium E1 (Sec. V): the kernel's collision against the
    oracle's for |u| <= 0.1 (the series' range); mass and energy kept to the
    rounding of the arithmetic, and the momentum change equal to the
    oracle's (E1 is not exactly momentum-conserving when theta differs from
    theta0)."""
    c, w, th = orc.lattice()
    for amp, f in _cases(orc, seed=4):
        if amp > 0.1:
            continue  # beyond the series' range: its own truncation error is ~u^4
        fin = f.astype(np.float32).astype(np.float64) if precision == "f32" else f
        g = L.collide_host(f, 1 / 0.6, precision, newton, series=True)
        ref = orc.collide_node(fin, 1 / 0.6, model="series")
        assert np.max(np.abs(g - ref)) < tol, amp
        m_in, m_g, m_ref = _moments(fin, c), _moments(g, c), _moments(ref, c)
        assert abs(m_g[0] - m_in[0]) < cons_tol and abs(m_g[4] - m_in[4]) < cons_tol, amp
        assert np.max(np.abs(m_g[1:4] - m_ref[1:4])) < cons_tol, amp


def _entropic_cases(orc, model="thermal"):
    """Nodes at increasing distance from equilibrium: both sides of the
    series range of the kernel's path length (FP32 and FP64), and a node
    where the positivity cap decides alpha."""
    c, w, th = orc.lattice()
    rng = np.random.default_rng(17)
    for amp in (1e-4, 1e-3, 0.01, 0.03, 0.1, 0.3):
        rho = 1 + rng.uniform(-0.01, 0.01)
        u = rng.uniform(-0.05, 0.05, 3)
        if model == "thermal":
            feq = orc.equilibrium(rho, u, th * (1 + rng.uniform(-0.02, 0.02)))[0]
        else:
            feq = orc.equilibrium_iso(rho, u)[0]
        yield amp, feq * (1 + amp * rng.uniform(-1, 1, 41))
    f = orc.equilibrium(1.0, np.array([0.02, 0.0, 0.01]), th)[0] * (1 + 0.05 * rng.uniform(-1, 1, 41))
    f[7] *= 40.0
    yield "cap", f


def _alpha_of(orc, f, out, omega, model="thermal"):
    """alpha from f* = f + alpha (omega/2) (f_eq - f) with the oracle's f_eq."""
    m = orc.node_moments(f)
    u = m[1:4] / m[0]
    if model == "thermal":
        feq = orc.equilibrium(m[0], u, (2 * m[4] / m[0] - u @ u) / 3)[0]
    else:
        feq = orc.equilibrium_iso(m[0], u)[0]
    d = feq - f
    return 2 * float((out - f) @ d) / (omega * float(d @ d)), feq


@pytest.mark.parametrize("model", ["thermal", "isothermal"])
@pytest.mark.parametrize("precision,newton,tol,atol", [("f64", 3, 2e-15, 1e-12), ("f32", 1, 6e-8, 2e-5)])
def test_host_entropic_collision_matches_oracle(orc, model, precision, newton, tol, atol):
    """Entropic path length (LBM_FLAG_ENTROPIC): the kernel's collision,
    series path near equilibrium and Newton on dH farther out, against the
    oracle's (bisection on the equal-entropy condition). Populations to the
    rounding of the arithmetic; alpha itself where f_eq - f is resolved."""
    c, w, th = orc.lattice()
    omega = 1 / 0.51
    for amp, f in _entropic_cases(orc, model):
        fin = f.astype(np.float32).astype(np.float64) if precision == "f32" else f
        g = L.collide_host(fin, omega, precision, newton, isothermal=(model == "isothermal"), entropic=True)
        ref = orc.collide_node(fin, omega, model=model, entropic=True)
        # the equilibrium solve's own error (one FP32 Newton step far from
        # the start) shows in the BGK collision of the same node as well
        bgk = L.collide_host(fin, omega, precision, newton, isothermal=(model == "isothermal"))
        bgk_err = np.max(np.abs(bgk - orc.collide_node(fin, omega, model=model)))
        assert np.max(np.abs(g - ref)) < max(tol, 1.5 * bgk_err), amp
        a_ref = orc.path_length(fin, _alpha_of(orc, fin, ref, omega, model)[1])
        a_gpu, feq = _alpha_of(orc, fin, g, omega, model)
        if amp == "cap" or amp >= 1e-3:
            # alpha resolved once f_eq - f is well above the rounding of f
            assert abs(a_gpu - a_ref) < atol / (1e-3 if amp == "cap" else amp), amp
        assert np.all(g > 0)
        k = 5 if model == "thermal" else 4
        cons = 1e-15 if precision == "f64" else 6e-8
        bgk_cons = np.max(np.abs(_moments(bgk, c)[:k] - _moments(fin, c)[:k]))
        assert np.max(np.abs(_moments(g, c)[:k] - _moments(fin, c)[:k])) < max(cons * 10, 1.5 * bgk_cons), amp


def test_host_entropic_matches_bgk_at_equilibrium():
    """At an equilibrium the path length is 2 and nothing moves."""
    import oracle as orc
    c, w, th = orc.lattice()
    f = orc.equilibrium(1.05, np.array([0.03, -0.02, 0.01]), th)[0]
    for precision in ("f64", "f32"):
        g = L.collide_host(f, 1.5, precision, entropic=True)
        b = L.collide_host(f, 1.5, precision)
        assert np.max(np.abs(g - b)) <= (1e-16 if precision == "f64" else 3e-8)


def test_host_entropic_rejects_series():
    f = np.full(41, 1.0 / 41)
    with pytest.raises(Exception):
        L.collide_host(f, 1.5, "f64", series=True, entropic=True)
