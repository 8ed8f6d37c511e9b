"""Physics analysis for oracle and GPU runs (test infrastructure only).

Linearised Navier-Stokes-Fourier (NSF) modes (Sec. I, the linearised NSF
acoustic equations with Fourier heat conduction), Fourier-mode projection
on the two bcc sublattices (Sec. IV), damped-mode fits and the analytic
3D acoustic pulse (Sec. VI, spherical pulse source).

Nothing here is GPU code; numpy and scipy only.
"""
import numpy as np
from scipy import integrate, optimize

GAMMA = 5.0 / 3.0  # monatomic ideal gas (Sec. VI, specific heat ratio 5/3)


def viscosity(theta0, tau_lb):
    """Kinematic viscosity of BGK with omega = 1/tau_lb at rest temperature
    theta0: nu = theta0 (tau_lb - 1/2) in lattice units. Prandtl number 1
    (single relaxation time) gives the thermal diffusivity chi = nu."""
    return theta0 * (tau_lb - 0.5)


def nsf_matrix(k, nu, chi, theta0, gamma=GAMMA, rho0=1.0):
    """Generator of the linearised NSF equations for a plane wave exp(i k x),
    state (d rho, d u_parallel, d theta), zero bulk viscosity, c_v = 3/2:
        d/dt drho   = -i k rho0 du
        d/dt du     = -i k (theta0 drho + rho0 dtheta)/rho0 - (4/3) nu k^2 du
        d/dt dtheta = -(gamma - 1) theta0 i k du - gamma chi k^2 dtheta
    """
    ik = 1j * k
    return np.array([
        [0.0, -ik * rho0, 0.0],
        [-ik * theta0 / rho0, -(4.0 / 3.0) * nu * k * k, -ik],
        [0.0, -(gamma - 1.0) * theta0 * ik, -gamma * chi * k * k],
    ], dtype=complex)


def nsf_modes(k, nu, chi, theta0, gamma=GAMMA):
    """(acoustic eigenvalue with Im > 0, entropy eigenvalue) per time step."""
    ev = np.linalg.eigvals(nsf_matrix(k, nu, chi, theta0, gamma))
    ent = ev[np.argmin(np.abs(ev.imag))]
    ac = ev[np.argmax(ev.imag)]
    return ac, ent.real


def node_positions(nx, ny, nz):
    """Positions (x, y, z) of all nodes in [s][z][y][x] order: node
    (s, x, y, z) sits at (x, y, z) + s (1/2, 1/2, 1/2)."""
    s, z, y, x = np.meshgrid(np.arange(2), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    h = 0.5 * s
    return (x + h).reshape(-1).astype(float), (y + h).reshape(-1).astype(float), (z + h).reshape(-1).astype(float)


def fourier_mode(field, nx, ny, nz, kvec):
    """a_k = (1/N) sum_nodes field * exp(-i k.x_node) at the true node positions."""
    x, y, z = node_positions(nx, ny, nz)
    ph = np.exp(-1j * (kvec[0] * x + kvec[1] * y + kvec[2] * z))
    f = np.asarray(field, dtype=float).reshape(-1)
    return np.sum(f * ph) / f.size


def linear_step_matrix(c, w, kvec, omega, isothermal=False):
    """One step of the lattice BGK scheme, linearised about the rest state
    f_i = w_i (rho 1, u 0, theta theta0), acting on the amplitudes a_i of a
    Fourier mode a_i exp(i k.x) over the bcc node positions (Sec. II: relax
    with rate omega toward the equilibrium of Sec. V, then move along c_i).

    The equilibrium has the exponential form w_i exp(lambda.phi_i) with
    phi = (1, c, c^2) and lambda = 0 at the rest state, so its derivative is
    d f_eq = W Phi (Phi^T W Phi)^{-1} Phi^T d f: the w-weighted projection of
    d f onto span(1, c, c^2) that keeps the five conserved moments. Moving
    along c_i brings to x what was at x - c_i (a node of the bcc lattice for
    every c_i, half-integer ones included), i.e. multiplies a_i by
    exp(-i k.c_i). Returns the 41 x 41 complex matrix S (I + omega (J - I)).
    isothermal: the equilibrium keeps mass and momentum only (phi = (1, c)),
    the model with sound speed sqrt(theta0)."""
    c = np.asarray(c, dtype=float).reshape(-1, 3)
    w = np.asarray(w, dtype=float)
    q = w.size
    phi = np.column_stack([np.ones(q), c] if isothermal else [np.ones(q), c, np.sum(c * c, axis=1)])
    gram = phi.T @ (w[:, None] * phi)
    J = (w[:, None] * phi) @ np.linalg.solve(gram, phi.T)
    C = (1.0 - omega) * np.eye(q) + omega * J
    S = np.exp(-1j * (c @ np.asarray(kvec, dtype=float)))
    return S[:, None] * C


def linear_moment_series(c, w, kvec, omega, a0, steps, isothermal=False):
    """Amplitudes of (rho, jx, jy, jz, E) of the mode after t = 0..steps
    steps of the linearised scheme from population amplitudes a0:
    array (steps + 1, 5); E = sum_i f_i c_i^2 / 2."""
    c = np.asarray(c, dtype=float).reshape(-1, 3)
    M = linear_step_matrix(c, w, kvec, omega, isothermal)
    P = np.vstack([np.ones(len(c)), c.T, 0.5 * np.sum(c * c, axis=1)])
    a = np.asarray(a0, dtype=complex)
    out = np.empty((steps + 1, 5), dtype=complex)
    for t in range(steps + 1):
        out[t] = P @ a
        a = M @ a
    return out


def linear_modes(c, w, kvec, omega, isothermal=False):
    """Hydrodynamic eigenvalues of the linearised step for wavevector k, as
    rates per step: (acoustic log-eigenvalue with Im > 0, entropy rate).
    The acoustic pair and the entropy mode are the eigenvalues closest to
    exp(+-i c_s |k|) and 1 among those of modulus near 1. The isothermal
    model has no entropy mode (its rate is then that of the slowest
    non-propagating mode, a shear mode)."""
    ev = np.linalg.eigvals(linear_step_matrix(c, w, kvec, omega, isothermal))
    lg = np.log(ev.astype(complex))
    # slow modes, one per conserved moment: two acoustic, two shear and (with
    # energy conserved) one entropy; the acoustic ones have the largest |Im|
    slow = lg[np.argsort(-lg.real)[:4 if isothermal else 5]]
    ac = slow[np.argmax(slow.imag)]
    rest = [z for z in slow if abs(z.imag) < 0.5 * ac.imag]
    # entropy vs shear: for Prandtl 1 the shear rate nu k^2 and the entropy
    # rate gamma chi k^2 differ by the factor gamma, entropy decays faster
    ent = min(rest, key=lambda z: z.real) if rest else np.nan
    return ac, -float(np.real(ent))


def temperature(rho, jx, jy, jz, en):
    """theta from E = (rho u^2 + 3 rho theta)/2 (Sec. II)."""
    u2 = (jx * jx + jy * jy + jz * jz) / (rho * rho)
    return (2.0 * en / rho - u2) / 3.0


def fit_acoustic_entropy(t, a, omega0, rate0):
    """Least-squares fit of a(t) = A exp(-G t) cos(w t + p) + B exp(-Ge t).
    Returns dict(A, G, w, p, B, Ge, rms)."""
    t = np.asarray(t, dtype=float)
    a = np.asarray(a, dtype=float)
    scale = np.max(np.abs(a))

    def model(p):
        A, G, w, ph, B, Ge = p
        return A * np.exp(-G * t) * np.cos(w * t + ph) + B * np.exp(-Ge * t)

    p0 = [0.6 * a[0], rate0, omega0, 0.0, 0.4 * a[0], rate0]
    r = optimize.least_squares(lambda p: (model(p) - a) / scale, p0, xtol=1e-15, ftol=1e-15, gtol=1e-15,
                               x_scale=[scale, rate0, omega0, 1.0, scale, rate0], max_nfev=20000)
    A, G, w, ph, B, Ge = r.x
    if A < 0:
        A, ph = -A, ph + np.pi
    rms = float(np.sqrt(np.mean((model(r.x) - a) ** 2)) / scale)
    return dict(A=A, G=G, w=w, p=ph, B=B, Ge=Ge, rms=rms)


def fit_decay(t, a):
    """Exponential rate of a non-oscillating mode by log-linear least squares."""
    t = np.asarray(t, dtype=float)
    la = np.log(np.abs(np.asarray(a, dtype=float)))
    A = np.vstack([np.ones_like(t), -t]).T
    c, *_ = np.linalg.lstsq(A, la, rcond=None)
    return float(c[1])


def pulse_3d(r, t, eps, b, cs):
    """Spherical pulse eps exp(-alpha r^2), alpha = ln2/b^2, under the linear
    wave equation with speed cs (Sec. VI, 3D acoustic pulse source; the
    printed integral lacks its time factor, which is cos(cs xi t)). The
    integral has the closed d'Alembert form used here:
        rho'(r, t) = eps/(2 r) [(r + cs t) e^{-alpha (r + cs t)^2}
                                + (r - cs t) e^{-alpha (r - cs t)^2}],
    and eps exp(-alpha r^2) at r = 0 limits continuously."""
    alpha = np.log(2.0) / (b * b)
    r = np.asarray(r, dtype=float)
    ct = cs * t
    with np.errstate(invalid="ignore", divide="ignore"):
        v = eps / (2.0 * r) * ((r + ct) * np.exp(-alpha * (r + ct) ** 2) + (r - ct) * np.exp(-alpha * (r - ct) ** 2))
    # r -> 0 limit: eps (1 - 2 alpha c^2 t^2) exp(-alpha c^2 t^2)
    lim = eps * (1.0 - 2.0 * alpha * ct * ct) * np.exp(-alpha * ct * ct)
    return np.where(r < 1e-12, lim, v)


def pulse_2d(r, t, eps, b, cs, nu_eff=0.0):
    """Axisymmetric 2D pulse eps exp(-alpha r^2), alpha = ln2/b^2, under
    the linearised Euler equations with sound speed cs (Sec. VI, the 2D
    acoustic pulse): the Hankel-transform solution
        rho'(r, t) = eps/(2 alpha) int_0^inf e^{-xi^2/(4 alpha)} cos(cs xi t)
                     J0(xi r) xi d xi,
    with an optional viscous damping factor e^{-nu_eff xi^2 t} (nu_eff the
    acoustic attenuation coefficient Gamma/k^2)."""
    from scipy import special
    alpha = np.log(2.0) / (b * b)
    upper = 14.0 * np.sqrt(alpha)
    r = np.atleast_1d(np.asarray(r, dtype=float))

    def one(rr):
        fn = lambda xi: (np.exp(-xi * xi / (4.0 * alpha) - nu_eff * xi * xi * t) * np.cos(cs * xi * t)
                         * special.j0(xi * rr) * xi)
        val, _ = integrate.quad(fn, 0.0, upper, limit=400, epsabs=1e-14, epsrel=1e-11)
        return eps / (2.0 * alpha) * val

    return np.array([one(rr) for rr in r])


def pulse_3d_integral(r, t, eps, b, cs, nu_eff=0.0):
    """The same solution as the integral over wavenumbers xi,
        eps/(2 alpha sqrt(pi alpha)) int_0^inf e^{-xi^2/(4 alpha)} cos(cs xi t)
            e^{-nu_eff xi^2 t} sin(xi r)/(xi r) xi^2 d xi,
    with an optional viscous damping factor (nu_eff = acoustic attenuation
    coefficient Gamma/k^2)."""
    alpha = np.log(2.0) / (b * b)
    pref = eps / (2.0 * alpha * np.sqrt(np.pi * alpha))
    upper = 12.0 * np.sqrt(alpha)

    def one(rr):
        def fn(xi):
            if rr < 1e-12:
                kern = xi * xi
            else:
                kern = np.sin(xi * rr) / (xi * rr) * xi * xi
            return np.exp(-xi * xi / (4 * alpha) - nu_eff * xi * xi * t) * np.cos(cs * xi * t) * kern
        v, _ = integrate.quad(fn, 0.0, upper, limit=400, epsabs=1e-14, epsrel=1e-12)
        return pref * v

    return np.array([one(float(rr)) for rr in np.atleast_1d(r)])
