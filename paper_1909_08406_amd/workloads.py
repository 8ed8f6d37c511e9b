"""Seeded synthetic inputs for the RD3Q41 lattice Boltzmann path.

This module produces initial fields only. It holds none of the method's
arithmetic (no lattice constants, no equilibrium, no streaming), so both
the GPU path and the CPU oracle can be fed from it. Temperatures are
returned relative to the lattice reference temperature (``theta_rel`` =
theta/theta0); each consumer multiplies by its own theta0.

Fields are FP64 numpy arrays over all nodes in [s][z][y][x] order (x
fastest): nx*ny*nz cells with two nodes each, node (s, x, y, z) located at
(x, y, z) + s*(1/2, 1/2, 1/2).
"""
from dataclasses import dataclass

import numpy as np

BATCH_EDGES = (16, 24, 32, 48, 64, 96)


@dataclass
class Fields:
    nx: int
    ny: int
    nz: int
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    theta_rel: np.ndarray

    @property
    def nodes(self):
        return 2 * self.nx * self.ny * self.nz

    def absolute(self, theta0):
        """(rho, ux, uy, uz, theta) with theta = theta_rel * theta0."""
        return self.rho, self.ux, self.uy, self.uz, self.theta_rel * theta0


def positions(nx, ny, nz):
    """Node positions (x, y, z), each an FP64 array in [s][z][y][x] order."""
    s = np.arange(2).reshape(2, 1, 1, 1) * 0.5
    z = np.arange(nz, dtype=np.float64).reshape(1, nz, 1, 1)
    y = np.arange(ny, dtype=np.float64).reshape(1, 1, ny, 1)
    x = np.arange(nx, dtype=np.float64).reshape(1, 1, 1, nx)
    shape = (2, nz, ny, nx)
    return (np.broadcast_to(x + s, shape).reshape(-1),
            np.broadcast_to(y + s, shape).reshape(-1),
            np.broadcast_to(z + s, shape).reshape(-1))


def _rest(nx, ny, nz):
    n = 2 * nx * ny * nz
    return np.ones(n), np.zeros(n), np.zeros(n), np.zeros(n), np.ones(n)


def standing_wave(nx, ny, nz, amp=1e-3, k=1, axis=0):
    """rho = 1 + amp sin(2 pi k x_axis / n_axis), u = 0, theta = theta0."""
    rho, ux, uy, uz, th = _rest(nx, ny, nz)
    p = positions(nx, ny, nz)[axis]
    n_axis = (nx, ny, nz)[axis]
    rho = 1.0 + amp * np.sin(2.0 * np.pi * k * p / n_axis)
    return Fields(nx, ny, nz, rho, ux, uy, uz, th)


def thermal_mode(n=128, amp=1e-3, noise=1e-4, seed=0):
    """theta = theta0 (1 + amp cos(2 pi z / n)), rho = 1 + U(-noise, noise)
    drawn with numpy's default_rng(seed) in node order, u = 0."""
    rho, ux, uy, uz, th = _rest(n, n, n)
    z = positions(n, n, n)[2]
    th = 1.0 + amp * np.cos(2.0 * np.pi * z / n)
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-noise, noise, size=rho.size)
    return Fields(n, n, n, rho, ux, uy, uz, th)


def taylor_green(n, u0):
    """u = u0 sin X cos Y cos Z, v = -u0 cos X sin Y cos Z, w = 0 with
    X = 2 pi x / n at the node positions; rho = 1, theta = theta0."""
    rho, ux, uy, uz, th = _rest(n, n, n)
    x, y, z = positions(n, n, n)
    X, Y, Z = (2.0 * np.pi * v / n for v in (x, y, z))
    ux = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    uy = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    return Fields(n, n, n, rho, ux, uy, uz, th)


def kida_peltz(n, u0):
    """Kida-Peltz initial field (the periodic decaying-turbulence case):
    u_x = u0 sin X (cos 3Y cos Z - cos Y cos 3Z) and its cyclic permutations
    in (X, Y, Z) = 2 pi (x, y, z)/n at the node positions; rho = 1,
    theta = theta0."""
    rho, ux, uy, uz, th = _rest(n, n, n)
    x, y, z = positions(n, n, n)
    X, Y, Z = (2.0 * np.pi * v / n for v in (x, y, z))
    ux = u0 * np.sin(X) * (np.cos(3 * Y) * np.cos(Z) - np.cos(Y) * np.cos(3 * Z))
    uy = u0 * np.sin(Y) * (np.cos(3 * Z) * np.cos(X) - np.cos(Z) * np.cos(3 * X))
    uz = u0 * np.sin(Z) * (np.cos(3 * X) * np.cos(Y) - np.cos(X) * np.cos(3 * Y))
    return Fields(n, n, n, rho, ux, uy, uz, th)


def gaussian_pulse(nx, ny=None, nz=None, eps=1e-3, b=8.0):
    """rho = 1 + eps exp(-ln2 r^2 / b^2) (b = half width at half maximum)
    centred on the cell corner (nx/2, ny/2, nz/2), r by periodic minimum
    image; u = 0, theta = theta0."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    x, y, z = positions(nx, ny, nz)
    r2 = np.zeros_like(x)
    for p, n in ((x, nx), (y, ny), (z, nz)):
        d = p - 0.5 * n
        d = d - n * np.round(d / n)
        r2 += d * d
    rho = 1.0 + eps * np.exp(-np.log(2.0) * r2 / (b * b))
    _, ux, uy, uz, th = _rest(nx, ny, nz)
    return Fields(nx, ny, nz, rho, ux, uy, uz, th)


def gaussian_pulse_2d(nx, ny, nz=1, eps=1e-3, b=8.0):
    """2D pulse rho = 1 + eps exp(-ln2 r^2 / b^2) with r the distance in the
    x-y plane from (nx/2, ny/2) (periodic minimum image), the same at every
    z (one cell in z holds the two node layers of the bcc lattice); u = 0,
    theta = theta0."""
    x, y, z = positions(nx, ny, nz)
    r2 = np.zeros_like(x)
    for p, n in ((x, nx), (y, ny)):
        d = p - 0.5 * n
        d = d - n * np.round(d / n)
        r2 += d * d
    rho = 1.0 + eps * np.exp(-np.log(2.0) * r2 / (b * b))
    _, ux, uy, uz, th = _rest(nx, ny, nz)
    return Fields(nx, ny, nz, rho, ux, uy, uz, th)


def pulse_over_wall_2d(nx, ny, nz=1, eps=1e-4, b=20.0, height=100.0, u0=0.0):
    """2D pulse above a wall normal to y: rho = 1 + eps exp(-ln2 r^2 / b^2)
    with r the x-y distance from (nx/2, height - 1/4) (the wall lies a
    quarter cell below the first node layer; periodic minimum image in x),
    uniform velocity (u0, 0, 0), theta = theta0."""
    x, y, z = positions(nx, ny, nz)
    d = x - 0.5 * nx
    d = d - nx * np.round(d / nx)
    dy = y - (height - 0.25)
    rho = 1.0 + eps * np.exp(-np.log(2.0) * (d * d + dy * dy) / (b * b))
    _, ux, uy, uz, th = _rest(nx, ny, nz)
    ux = np.full_like(ux, u0)
    return Fields(nx, ny, nz, rho, ux, uy, uz, th)


def random_state(nx, ny, nz, seed=0, amp_rho=1e-2, amp_u=5e-2, amp_theta=2e-2):
    """Independent uniform perturbations per node (parity-test input):
    rho = 1 + U(-a, a), u_a = U(-b, b), theta/theta0 = 1 + U(-c, c)."""
    n = 2 * nx * ny * nz
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-amp_rho, amp_rho, n)
    ux = rng.uniform(-amp_u, amp_u, n)
    uy = rng.uniform(-amp_u, amp_u, n)
    uz = rng.uniform(-amp_u, amp_u, n)
    th = 1.0 + rng.uniform(-amp_theta, amp_theta, n)
    return Fields(nx, ny, nz, rho, ux, uy, uz, th)


@dataclass
class BoxSpec:
    nx: int
    ny: int
    nz: int
    k: int
    tau: float
    amp: float


def batch_specs(nboxes=256, seed=0):
    """Independent periodic boxes: for each box in turn, edges drawn with
    rng.choice over BATCH_EDGES (3 draws), wavenumber rng.integers(1, 5),
    tau = rng.uniform(0.51, 1.0), amplitude 10**rng.uniform(-4, -2)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nboxes):
        e = rng.choice(BATCH_EDGES, 3)
        k = int(rng.integers(1, 5))
        tau = float(rng.uniform(0.51, 1.0))
        amp = float(10.0 ** rng.uniform(-4.0, -2.0))
        out.append(BoxSpec(int(e[0]), int(e[1]), int(e[2]), k, tau, amp))
    return out


def batch_fields(spec):
    """Standing wave rho = 1 + A sin(2 pi k x / nx), u = 0, theta = theta0."""
    return standing_wave(spec.nx, spec.ny, spec.nz, amp=spec.amp, k=spec.k, axis=0)


def concat(fields_list):
    """Concatenate per-box fields box after box (the multi-box host layout)."""
    cat = lambda name: np.concatenate([getattr(f, name) for f in fields_list])
    return cat("rho"), cat("ux"), cat("uy"), cat("uz"), cat("theta_rel")
