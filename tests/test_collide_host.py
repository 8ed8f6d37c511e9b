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
