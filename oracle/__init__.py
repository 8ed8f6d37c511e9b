"""Plain FP64 CPU oracle for the RD3Q41 energy-conserving lattice Boltzmann
method (Kolluru, Atif, Namburi, Ansumali, arXiv:1909.08406).

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package. It shares no code with the
GPU library (``paper_1909_08406_amd``) and never imports it.

The arithmetic lives in ``lbm_oracle.c`` (built by ``oracle/build.py``);
this module only marshals numpy arrays through ctypes.  Every function
cites the passage of the paper it follows in the C source.

Parity status of each function (what pins it, see tests/test_oracle_*.py):
  lattice, constraint_residuals  -- Table I weights and the seven weight
                                    constraints of Sec. III; cubic symmetry.
  equilibrium (E2)                -- residual of the Sec. V constraint system,
                                    u=0/theta=theta0 special case, H-minimum,
                                    cubic equivariance, agreement with E1.
  series_rest / series_errors     -- printed M2, M2', M3, M3' coefficients.
  equilibrium_series (E1)         -- exact mass and energy.
  pull_map / push_map             -- brute-force position search, bijection.
  run / collide_field             -- per-node conservation, uniform fixed
                                    point, sound speed and decay rates
                                    against linearised Navier-Stokes-Fourier.
  path_length (entropic step)     -- H(f + alpha (feq - f)) = H(f) with H
                                    evaluated directly from its definition,
                                    alpha -> 2 near equilibrium with the
                                    cubic-order correction, H decrease of the
                                    post-collision state, the positivity cap,
                                    a brute-force scan of the sign change.
"""
import ctypes
import os

import numpy as np

NQ = 41
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbm_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i, d, l = ctypes.c_int, ctypes.c_double, ctypes.c_int64
    sig = {
        "orc_lattice": (i, [_dp, _dp, _dp]),
        "orc_constraint_residuals": (None, [_dp]),
        "orc_node_moments": (None, [_dp, _dp]),
        "orc_entropy": (d, [_dp]),
        "orc_equilibrium": (i, [d, d, d, d, d, _dp, _dp, _dp, _ip]),
        "orc_series_rest": (None, [d, d, _dp]),
        "orc_series_errors": (None, [d, _dp]),
        "orc_equilibrium_series": (None, [d, d, d, d, d, _dp]),
        "orc_collide_node": (i, [_dp, d, _dp]),
        "orc_equilibrium_iso": (i, [d, d, d, d, _dp, _dp, _dp, _ip]),
        "orc_collide_node_model": (i, [_dp, d, i, _dp]),
        "orc_path_length": (d, [_dp, _dp]),
        "orc_path_dh": (d, [_dp, _dp, d]),
        "orc_init_model": (i, [i, i, i, _dp, _dp, _dp, _dp, _dp, i, _dp]),
        "orc_collide_field_model": (i, [i, i, i, d, i, _dp, _dp]),
        "orc_run_model": (i, [i, i, i, d, i, _dp, _dp, i]),
        "orc_run_walls": (i, [i, i, i, d, i, _dp, _dp, _dp, i]),
        "orc_run_walls_kind": (i, [i, i, i, d, i, _dp, _ip, _dp, _dp, i]),
        "orc_pull_map": (None, [i, i, i, _lp]),
        "orc_push_map": (None, [i, i, i, _lp]),
        "orc_pull_src_nodes": (None, [i, i, i, _lp, l, _lp]),
        "orc_init": (i, [i, i, i, _dp, _dp, _dp, _dp, _dp, _dp]),
        "orc_collide_field": (i, [i, i, i, d, _dp, _dp]),
        "orc_run": (i, [i, i, i, d, _dp, _dp, i]),
        "orc_moment_fields": (None, [l, _dp, _dp, _dp, _dp, _dp, _dp]),
        "orc_totals": (None, [l, _dp, _dp]),
        "orc_threads": (i, []),
        "orc_set_threads": (None, [i]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _pops(f, n=None, copy=False):
    """Populations as a C-contiguous FP64 (41, N) array; N checked when
    given (the C side trusts the sizes it is passed)."""
    a = np.array(f, dtype=np.float64, copy=True, order="C") if copy else _f64(f)
    if a.size % NQ or (n is not None and a.size != NQ * n):
        raise ValueError("populations of size %d do not hold 41 x %s values" % (a.size, n))
    return a.reshape(NQ, a.size // NQ)


def lattice():
    """(c[41,3], w[41], theta0) in the canonical velocity order."""
    lib = _load()
    c = np.zeros((NQ, 3))
    w = np.zeros(NQ)
    t = np.zeros(1)
    lib.orc_lattice(_d(c), _d(w), _d(t))
    return c, w, float(t[0])


def constraint_residuals():
    out = np.zeros(7)
    _load().orc_constraint_residuals(_d(out))
    return out


def node_moments(f):
    f = _f64(f)
    m = np.zeros(5)
    _load().orc_node_moments(_d(f), _d(m))
    return m


def entropy(f):
    f = _f64(f)
    return float(_load().orc_entropy(_d(f)))


def equilibrium(rho, u, theta):
    """E2: returns (feq[41], lam[5] = (alpha, beta_x, beta_y, beta_z, gamma),
    residual, newton iterations, status)."""
    feq = np.zeros(NQ)
    lam = np.zeros(5)
    res = np.zeros(1)
    it = ctypes.c_int(0)
    rc = _load().orc_equilibrium(float(rho), float(u[0]), float(u[1]), float(u[2]), float(theta),
                                 _d(feq), _d(lam), _d(res), ctypes.byref(it))
    return feq, lam, float(res[0]), it.value, rc


def equilibrium_iso(rho, u):
    """Isothermal equilibrium (mass and momentum constraints only): returns
    (feq[41], lam[5] = (alpha, beta_x, beta_y, beta_z, 0), residual,
    newton iterations, status)."""
    feq = np.zeros(NQ)
    lam = np.zeros(5)
    res = np.zeros(1)
    it = ctypes.c_int(0)
    rc = _load().orc_equilibrium_iso(float(rho), float(u[0]), float(u[1]), float(u[2]),
                                     _d(feq), _d(lam), _d(res), ctypes.byref(it))
    return feq, lam, float(res[0]), it.value, rc


# equilibrium models: 0 energy conserving (E2), 1 isothermal, 2 series (E1);
# ENTROPIC adds the entropic path length to the relaxation (E2, isothermal)
MODELS = {"thermal": 0, "isothermal": 1, "series": 2}
ENTROPIC = 4


def _model(model, entropic=False):
    m = MODELS[model] if isinstance(model, str) else int(model)
    if entropic:
        if m == MODELS["series"]:
            raise ValueError("the entropic path length needs an exact entropic equilibrium (thermal or isothermal)")
        m |= ENTROPIC
    return m


def path_length(f, feq):
    """Entropic path length alpha of one node: the nontrivial root of
    H(f + a (feq - f)) = H(f) in (1, a_cap] (a_cap = (1 - 2^-10) a_max, a_max
    the largest a that keeps f + a (feq - f) positive); 2 when f = feq."""
    f, feq = _f64(f), _f64(feq)
    if f.size != NQ or feq.size != NQ:
        raise ValueError("one node of 41 populations expected")
    return float(_load().orc_path_length(_d(f), _d(feq)))


def path_dh(f, feq, a):
    """H(f + a (feq - f)) - H(f) by the oracle's rewritten form."""
    f, feq = _f64(f), _f64(feq)
    if f.size != NQ or feq.size != NQ:
        raise ValueError("one node of 41 populations expected")
    return float(_load().orc_path_dh(_d(f), _d(feq), float(a)))


def series_rest(rho, eta):
    out = np.zeros(NQ)
    _load().orc_series_rest(float(rho), float(eta), _d(out))
    return out


def series_errors(eta):
    """(M2, M2', M3, M3') of the zero-velocity series at eta."""
    out = np.zeros(4)
    _load().orc_series_errors(float(eta), _d(out))
    return out


def equilibrium_series(rho, u, theta):
    out = np.zeros(NQ)
    _load().orc_equilibrium_series(float(rho), float(u[0]), float(u[1]), float(u[2]), float(theta), _d(out))
    return out


def collide_node(f, omega, model="thermal", entropic=False):
    f = _f64(f)
    if f.size != NQ:
        raise ValueError("one node of 41 populations expected")
    out = np.zeros(NQ)
    rc = _load().orc_collide_node_model(_d(f), float(omega), _model(model, entropic), _d(out))
    if rc != 0:
        raise RuntimeError("oracle equilibrium did not converge")
    return out


def pull_map(nx, ny, nz):
    n = 2 * nx * ny * nz
    out = np.zeros(NQ * n, dtype=np.int64)
    _load().orc_pull_map(nx, ny, nz, out.ctypes.data_as(_lp))
    return out.reshape(NQ, n)


def pull_sources(nx, ny, nz, nodes):
    """[len(nodes), 41] source node of each population arriving at each node."""
    nodes = np.ascontiguousarray(nodes, dtype=np.int64).reshape(-1)
    out = np.zeros(nodes.size * NQ, dtype=np.int64)
    _load().orc_pull_src_nodes(nx, ny, nz, nodes.ctypes.data_as(_lp), nodes.size, out.ctypes.data_as(_lp))
    return out.reshape(nodes.size, NQ)


def push_map(nx, ny, nz):
    n = 2 * nx * ny * nz
    out = np.zeros(NQ * n, dtype=np.int64)
    _load().orc_push_map(nx, ny, nz, out.ctypes.data_as(_lp))
    return out.reshape(NQ, n)


def init(nx, ny, nz, rho, ux, uy, uz, theta, model="thermal"):
    """Equilibrium populations [41, N] for FP64 node fields (theta absolute;
    ignored by the isothermal model)."""
    n = 2 * nx * ny * nz
    args = [_f64(a).reshape(-1) for a in (rho, ux, uy, uz, theta)]
    for a in args:
        if a.size != n:
            raise ValueError("field size %d != %d nodes" % (a.size, n))
    f = np.zeros((NQ, n))
    rc = _load().orc_init_model(nx, ny, nz, *[_d(a) for a in args], _model(model), _d(f))
    if rc != 0:
        raise RuntimeError("oracle equilibrium did not converge at init")
    return f


def collide_field(nx, ny, nz, omega, f, model="thermal", entropic=False):
    f = _pops(f, 2 * nx * ny * nz)
    out = np.zeros_like(f)
    rc = _load().orc_collide_field_model(nx, ny, nz, float(omega), _model(model, entropic), _d(f), _d(out))
    if rc != 0:
        raise RuntimeError("oracle equilibrium did not converge")
    return out


def run(nx, ny, nz, omega, f, nsteps, model="thermal", entropic=False):
    """Advance populations f [41, N] by nsteps collide+push steps (in place copy returned)."""
    f = _pops(f, 2 * nx * ny * nz, copy=True)
    tmp = np.empty_like(f)
    rc = _load().orc_run_model(nx, ny, nz, float(omega), _model(model, entropic), _d(f), _d(tmp), int(nsteps))
    if rc != 0:
        raise RuntimeError("oracle equilibrium did not converge during run")
    return f


def run_walls(nx, ny, nz, omega, f, nsteps, walls, model="thermal", entropic=False, kinds=(0, 0)):
    """Like run, with kinetic walls normal to y a quarter cell outside the
    first and last node layers (diffuse, mass-conserving reflection towards
    each wall's equilibrium). walls = ((ux, uy, uz, theta) lower,
    (ux, uy, uz, theta) upper), theta absolute (unused by the isothermal
    model). kinds: 0 diffuse, 1 specular (mirror image in y) per wall.
    Periodic in x and z."""
    if ny < 2:
        raise ValueError("walls need ny >= 2")
    f = _pops(f, 2 * nx * ny * nz, copy=True)
    tmp = np.empty_like(f)
    w = _f64(walls).reshape(-1)
    if w.size != 8:
        raise ValueError("walls: two (ux, uy, uz, theta)")
    k = (ctypes.c_int * 2)(int(kinds[0]), int(kinds[1]))
    rc = _load().orc_run_walls_kind(nx, ny, nz, float(omega), _model(model, entropic), _d(w),
                                    ctypes.cast(k, _ip), _d(f), _d(tmp), int(nsteps))
    if rc != 0:
        raise RuntimeError("oracle wall run failed (%d)" % rc)
    return f


def moment_fields(f):
    """(rho, jx, jy, jz, E) per node from populations [41, N]."""
    f = _pops(f)
    n = f.shape[-1]
    m = np.zeros((5, n))
    _load().orc_moment_fields(n, _d(f), *[_d(m[k]) for k in range(5)])
    return m


def totals(f):
    f = _pops(f)
    out = np.zeros(5)
    _load().orc_totals(f.shape[-1], _d(f), _d(out))
    return out


def threads():
    return int(_load().orc_threads())


def set_threads(n):
    _load().orc_set_threads(int(n))
