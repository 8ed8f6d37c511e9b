// The fused pull-collide step of the RD3Q41 library: per-node collision
// (moments, equilibrium, relaxation, path length, walls), storage encoding
// and the step kernels for one box and for a batch of boxes.
#pragma once

#include <type_traits>

#include "device.hpp"
#include "step_launch.hpp"

namespace lbm {

constexpr int BLOCK = 256;
constexpr int NXCD = 8;  // MI355X: 8 accelerator complex dies, blocks dispatched round-robin

// Map the dispatch-order block id to a tile id so that each XCD (block id
// mod 8) works on one contiguous range of tiles: neighbouring tiles share
// cache lines at their edges, and each XCD has its own L2.
__device__ inline uint32_t xcd_tile(uint32_t b, uint32_t G)
{
    const uint32_t per = G / NXCD, rem = G % NXCD;
    const uint32_t xcd = b % NXCD, idx = b / NXCD;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

template <typename R>
__device__ inline void flag_bad(const StepParams& p, R rho, R theta)
{
    if (__builtin_expect(!(rho > R(0)) || !(theta > R(0)) || !(theta < R(1e30)), 0))
        atomicOr(p.flag, 1u);
}

// ---------------------------------------------------------------------------
// Collision of one node (Sec. II: f* = f + omega (f_eq - f); Sec. V: f_eq the
// entropic equilibrium of the node's rho, j, E) on its stored values x_q:
// f_q for direct storage, h_q = (f_q - w_q rho0) 2^{k_q} for the shifted
// forms. Returns in y the new stored values h* for the shifted forms and
// the increment f* - f for direct storage (before rounding to the storage
// type), and rho and theta for the realisability flag.
//
// Moments are formed from deviations from the reference state w_q rho_ref:
// for direct storage d_q = f_q - w_q (exact in floating point while f_q is
// within a factor two of w_q), for shifted storage the stored h_q scaled
// per shell. The relaxation is folded into one or two fused multiply-adds
// per population with omega w_s rho_ref (and the storage scale) per shell.
// ---------------------------------------------------------------------------
template <typename R>
struct CollideConst {
    R om;            // omega
    R rho_ref;       // rho0 (shifted storage) or 1
    R inv_scale[6];  // 2^{-k_s} (shifted) or 1
    R omw[6];        // omega w_s rho_ref 2^{k_s} (shifted) or omega w_s
};

// Equilibrium models: the energy-conserving entropic equilibrium E2, the
// isothermal one (mass and momentum only) and the series equilibrium E1 (low
// two bits). MODEL_ENTROPIC adds the entropic path length to the relaxation
// (with E2 or the isothermal equilibrium, the exact minimisers of H).
constexpr int MODEL_E2 = 0;
constexpr int MODEL_ISO = 1;
constexpr int MODEL_SERIES = 2;
constexpr int MODEL_ENTROPIC = 4;
constexpr int MODEL_WALLS = 8;
constexpr int MODEL_BASE_MASK = 3;

// ---------------------------------------------------------------------------
// Entropic path length (Sec. IX.A: the relaxation f + alpha beta (f_eq - f)
// with beta = omega/2, where alpha = 2 is the BGK step and the entropic
// method chooses alpha by the H theorem; Sec. IX.D: alpha from
// x_q = f_eq,q/f_q - 1; H = sum f (log(f/w) - 1) of Sec. V).
//
// alpha is the nontrivial root of dH(a) = H(f + a (f_eq - f)) - H(f), the
// mirror state having the entropy of f. Because f_eq - f carries no conserved
// moment and log(f_eq/w) lies in their span,
//   dH(a) = sum_q f_q [(1 + a x_q) log(1 + a x_q) - a x_q] - a sum_q f_q x_q log(1 + x_q).
// dH is convex with its minimum at a = 1, so the root lies in (1, a_cap],
// a_cap = (1 - 2^-10) min_{x_q < 0} (-1/x_q) keeping the mirror state
// positive; alpha = a_cap when dH(a_cap) <= 0.
//
// Near equilibrium (max |x_q| <= XS) dH/a is a power series in x,
//   dH(a)/a = sum_{n >= 2} (-1)^n S_n (a^{n-1} - n) / (n (n-1)),  S_n = sum_q f_q x_q^n,
// truncated at order N (the truncated terms move alpha by less than the
// storage rounding moves f) and solved by Newton from a = 2: one pass over
// the populations for the S_n, then scalar work only. For 16-bit storage
// (COARSE) the root of the series to second order in x,
//   alpha = 2 + (S3 - 2 S4) / (3 S2 - 4 S3),
// is used for max |x_q| <= 1/32: its error in alpha is O(x^3), moving f* by
// at most ~3e-6 of f there, below the 16-bit storage quantum. Farther from
// equilibrium Newton runs on dH itself (a pass over the populations with
// log1p per iteration, at most ITMAX iterations).
// ---------------------------------------------------------------------------
template <typename R>
struct PathConst;
template <>
struct PathConst<float> {
    static constexpr int N = 7;
    static constexpr float XS = 0.0625f;
    static constexpr float XS_COARSE = 0.03125f;
    static constexpr int IT = 3;
    static constexpr int ITMAX = 40;
    static constexpr float TOL = 1e-6f;
};
template <>
struct PathConst<double> {
    static constexpr int N = 10;
    static constexpr double XS = 0.015625;
    static constexpr double XS_COARSE = 0.015625;
    static constexpr int IT = 4;
    static constexpr int ITMAX = 60;
    static constexpr double TOL = 1e-14;
};

// log(1 + y): FP32 from the hardware logarithm with the correction
// log(u) y / (u - 1), u = 1 + y rounded (accurate for small y as well);
// FP64 from the math library.
template <typename R>
__host__ __device__ inline R d_log1p(R y);
template <>
__host__ __device__ inline float d_log1p<float>(float y)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const float u = 1.0f + y;
    return u == 1.0f ? y : __logf(u) * (y * __builtin_amdgcn_rcpf(u - 1.0f));
#else
    return std::log1p(y);
#endif
}
template <>
__host__ __device__ inline double d_log1p<double>(double y)
{
    return log1p(y);
}

// Opaque to the optimiser (no instruction): values recomputed after it are
// not merged with copies computed before it, which would keep those live.
template <typename R>
__host__ __device__ inline void opaque(R& v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+v"(v));
#else
    (void)v;
#endif
}

// fd(q, f, d) gives f_q and d_q = f_eq,q - f_q of the node; fresh() makes
// the inputs of fd opaque before the far path recomputes them.
template <typename R, bool COARSE, class FD, class FRESH>
__host__ __device__ __forceinline__ R path_length(const FD& fd, const FRESH& fresh)
{
    using PC = PathConst<R>;
    constexpr int N = COARSE ? 4 : PC::N;
    constexpr R XS = COARSE ? PC::XS_COARSE : PC::XS;
    R S[N + 1];
#pragma unroll
    for (int n = 0; n <= N; ++n) S[n] = R(0);
    R xabs = R(0);
    static_for<Q>([&](auto qc) {
        R f, d;
        fd(qc, f, d);
        const R x = d * d_rcp<R>(f);
        xabs = fmax(xabs, fabs(x));
        R t = d * x;  // f x^2
#pragma unroll
        for (int n = 2; n <= N; ++n) {
            S[n] += t;
            t *= x;
        }
    });
    // the sums are complete here (not sunk into the branch that uses them,
    // which would keep the 41 x_q live across it)
#pragma unroll
    for (int n = 2; n <= N; ++n) opaque(S[n]);
    opaque(xabs);
    fresh();
    if (__builtin_expect(!(xabs <= XS), 0)) {
        // far from equilibrium (rare): Newton on dH itself from
        // a = min(2, a_cap), over f_q and x_q held in private memory
        // (volatile: read back in plain loops, not kept in registers)
        volatile R fb[Q], xb[Q];
        R xmin = R(0);
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            R f, d;
            fd(qc, f, d);
            const R x = d * d_rcp<R>(f);
            fb[q] = f;
            xb[q] = x;
            xmin = fmin(xmin, x);
        });
        const R acap = xmin < R(0) ? (R(1) - R(1.0 / 1024)) * (R(-1) / xmin) : R(1e30);
        R P = R(0);  // sum_q f_q x_q log(1 + x_q)
#pragma clang loop unroll(disable)
        for (int q = 0; q < Q; ++q) {
            const R f = fb[q], x = xb[q];
            P = fma(f * x, d_log1p<R>(x), P);
        }
        R a = fmin(R(2), acap);
#pragma clang loop unroll(disable)
        for (int it = 0; it < PC::ITMAX; ++it) {
            R g = R(0), gp = R(0);
#pragma clang loop unroll(disable)
            for (int q = 0; q < Q; ++q) {
                const R f = fb[q], x = xb[q];
                const R y = a * x;
                const R L = d_log1p<R>(y);
                g = fma(f, fma(R(1) + y, L, -y), g);
                gp = fma(f * x, L, gp);
            }
            g = fma(-a, P, g);
            gp -= P;
            if (!(gp > R(0))) break;
            const R an = fmin(fmax(a - g / gp, R(1)), acap);
            const bool done = fabs(an - a) <= R(PC::TOL) * a;
            a = an;
            if (done) break;
        }
        fresh();
        return a;
    }
    if constexpr (COARSE) {
        const R den = R(3) * S[2] - R(4) * S[3];
        const R a = R(2) + (S[3] - R(2) * S[4]) / den;
        return (den > R(0) && a > R(1) && a < R(4)) ? a : R(2);
    }
    // G(a) = dH(a)/a = sum_n c_n (a^{n-1} - n), c_n = (-1)^n S_n / (n (n-1))
    R c[N + 1];
#pragma unroll
    for (int n = 2; n <= N; ++n) c[n] = ((n & 1) ? -S[n] : S[n]) * R(1.0 / (n * (n - 1)));
    R a = R(2);
#pragma unroll
    for (int it = 0; it < PC::IT; ++it) {
        R G = R(0), Gp = R(0), p = R(1);  // p = a^{n-2}
#pragma unroll
        for (int n = 2; n <= N; ++n) {
            Gp = fma(c[n] * R(n - 1), p, Gp);
            G = fma(c[n], fma(a, p, R(-n)), G);
            p *= a;
        }
        if (Gp > R(0)) a -= G / Gp;
    }
    if (!(a > R(1) && a < R(4))) a = R(2);  // only where the S_n are rounding noise
    return a;
}

// For direct storage in FP64 x is overwritten by the deviations
// d_q = f_q - w_q (exact while f_q is within a factor two of w_q), so only d
// stays live through the equilibrium solve (214 instead of 256 registers:
// two wavefronts per SIMD) and the caller restores f_q = d_q + w_q. In FP32
// both are kept (measured marginally faster).
template <typename R>
constexpr bool DEV_IN_PLACE = std::is_same<R, double>::value;

// The relaxation reads the stored values again through xr(q) when one is
// given (a second decode of values the caller keeps in a compact form), so
// the decoded x need not stay live through the equilibrium solve.
struct NoReload {};

template <typename R, bool SHIFTED, int NEWTON, int MODEL = MODEL_E2, class XR = NoReload, bool COARSE = false>
__host__ __device__ __forceinline__ void collide(R x[Q], R y[Q], const CollideConst<R>& cc, R& rho_out, R& theta_out,
                                        const XR& xr = XR())
{
    ShellSums<R> SS;
    if constexpr (SHIFTED) {
        shell_sums<R>(x, SS);
    } else if constexpr (DEV_IN_PLACE<R>) {
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            x[q] = x[q] - R(weight(q));
        });
        shell_sums<R>(x, SS);
    } else {
        R d[Q];
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            d[q] = x[q] - R(weight(q));
        });
        shell_sums<R>(d, SS);
    }
    NodeDev<R> st;
    st.rho_ref = cc.rho_ref;
    R drho = R(0), jx = R(0), jy = R(0), jz = R(0), de2 = R(0);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const R s0 = cc.inv_scale[s] * SS.s0[s];
        drho += s0;
        if (s == 0) continue;
        de2 += R(SHELL_C2[s]) * s0;
        const R kc = cc.inv_scale[s] * R(SHELL_CA[s]);
        jx += kc * SS.sx[s];
        jy += kc * SS.sy[s];
        jz += kc * SS.sz[s];
    }
    st.drho = drho;
    st.j[0] = jx;
    st.j[1] = jy;
    st.j[2] = jz;
    st.de2 = de2;
    st.rho = st.rho_ref * R(SUM_W) + drho;
    st.irho = R(1) / st.rho;
    const R ux = jx * st.irho, uy = jy * st.irho, uz = jz * st.irho;
    const R K = (st.rho_ref * R(SUM_WC2) + de2) * st.irho;  // 2E/rho = u^2 + 3 theta
    const R theta = (K - (ux * ux + uy * uy + uz * uz)) * R(1.0 / 3.0);
    rho_out = st.rho;
    theta_out = theta;

    constexpr int BASE = MODEL & MODEL_BASE_MASK;
    static_assert(!(MODEL & MODEL_ENTROPIC) || BASE != MODEL_SERIES, "path length needs an exact minimiser of H");
    R om = cc.om, om1 = R(1) - om;
    R omw[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) omw[s] = cc.omw[s];
    // f_eq,q - w_q rho_ref = w_q rho_ref D_q; relaxation of population q
    auto relax = [&](auto qc, R D) {
        constexpr int q = decltype(qc)::value;
        constexpr int sh = VEL[q].shell;
        if constexpr (SHIFTED && !std::is_same<XR, NoReload>::value) y[q] = fma(om1, xr(qc), omw[sh] * D);
        else if constexpr (SHIFTED) y[q] = fma(om1, x[q], omw[sh] * D);          // h* = (1-w) h + w 2^k d_eq
        else if constexpr (DEV_IN_PLACE<R>) y[q] = fma(omw[sh], D, -om * x[q]);  // f* - f = w (f_eq - f)
        else y[q] = fma(omw[sh], D, -om * (x[q] - R(weight(q))));
    };
    if constexpr (BASE == MODEL_SERIES) {
        // 1 + D_q = (1 + eps_q) rho / (rho_ref sum_i w_i)
        // eta = theta/theta0 - 1 from the deviations of 2E and rho:
        // 3 theta0 rho eta = rho_ref (sum w c^2 - 3 theta0 sum w) + de2 - 3 theta0 drho - rho u^2
        constexpr double E2_OFF = SUM_WC2 - 3.0 * THETA0 * SUM_W;
        const R eta = (st.rho_ref * R(E2_OFF) + st.de2 - R(3.0 * THETA0) * st.drho -
                       st.rho * (ux * ux + uy * uy + uz * uz)) *
                      st.irho * R(1.0 / (3.0 * THETA0));
        SeriesCoef<R> sc;
        series_coef<R>(ux, uy, uz, eta, sc);
        const R kap = st.drho / (st.rho_ref * R(SUM_W));
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            relax(qc, dmul(series_eps<q, R>(sc), kap));
        });
        return;
    }
    Mult<R> m;
    if constexpr (BASE == MODEL_ISO) {
        // isothermal: g = 0, Maxwellian guess at theta0
        m.b[0] = ux * R(1.0 / THETA0);
        m.b[1] = uy * R(1.0 / THETA0);
        m.b[2] = uz * R(1.0 / THETA0);
        m.g = R(0);
#pragma unroll
        for (int it = 0; it < NEWTON; ++it) newton_step<R, false>(m, st);
    } else {
        const R ith = R(1) / theta;
        m.b[0] = ux * ith;
        m.b[1] = uy * ith;
        m.b[2] = uz * ith;
        m.g = R(0.5) * ith - R(0.5 / THETA0);
#pragma unroll
        for (int it = 0; it < NEWTON; ++it) newton_step<R>(m, st);
    }

    // 1 + D_q = (1 + eps_q)(1 + kappa)
    Shells<R> S;
    shells_at<R>(m, S);
    R kap = kappa_of<R>(st, S);
    // Entropic step in FP32 arithmetic: D_q is kept in y[q] from the path
    // length's pass to the relaxation (fits the occupancy the kernel has
    // anyway); in FP64 it is recomputed (keeping it would halve occupancy).
    constexpr bool KEEP_D = (MODEL & MODEL_ENTROPIC) != 0 && !std::is_same<R, double>::value;
    if constexpr ((MODEL & MODEL_ENTROPIC) != 0) {
        // f_q and f_eq,q - f_q from the stored values
        auto fd = [&](auto qc, R& f, R& d) {
            constexpr int q = decltype(qc)::value;
            constexpr int sh = VEL[q].shell;
            const R D = dmul(gibbs_dev<q, R>(S), kap);
            if constexpr (KEEP_D) y[q] = D;
            if constexpr (SHIFTED) {
                const R wr = R(weight(q)) * cc.rho_ref, h = x[q] * cc.inv_scale[sh];
                f = wr + h;
                d = fma(wr, D, -h);
            } else if constexpr (DEV_IN_PLACE<R>) {
                f = R(weight(q)) + x[q];
                d = fma(R(weight(q)), D, -x[q]);
            } else {
                f = x[q];
                d = fma(R(weight(q)), D, -(x[q] - R(weight(q))));
            }
        };
        // the relaxation and the far path recompute what they need rather
        // than keeping further values live
        auto fresh = [&]() {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                opaque(S.sh[a]);
                opaque(S.chm[a]);
                opaque(S.s1[a]);
                opaque(S.c1m[a]);
                opaque(S.s2[a]);
                opaque(S.c2m[a]);
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) opaque(S.tau[k]);
            opaque(kap);
#pragma unroll
            for (int q = 0; q < Q; ++q) opaque(x[q]);
        };
        // relaxation rate alpha omega / 2 (alpha = 2: BGK)
        const R ah = R(0.5) * path_length<R, COARSE>(fd, fresh);
        om = cc.om * ah;
        om1 = R(1) - om;
#pragma unroll
        for (int s = 0; s < 6; ++s) omw[s] = cc.omw[s] * ah;
    }
    if constexpr (KEEP_D) {
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            relax(qc, y[q]);
        });
    } else {
        // omw_s D_q = omw_s (e_q + kappa + e_q kappa) = A_s e_q + B_s with
        // e_q the Gibbs factor's deviation: one FMA per population
        R A[6], B[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            A[s] = omw[s] * (R(1) + kap);
            B[s] = omw[s] * kap;
        }
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int sh = VEL[q].shell;
            const R e = gibbs_dev<q, R>(S);
            if constexpr (SHIFTED && !std::is_same<XR, NoReload>::value) y[q] = fma(om1, xr(qc), fma(A[sh], e, B[sh]));
            else if constexpr (SHIFTED) y[q] = fma(om1, x[q], fma(A[sh], e, B[sh]));
            else if constexpr (DEV_IN_PLACE<R>) y[q] = fma(A[sh], e, fma(-om, x[q], B[sh]));
            else y[q] = fma(A[sh], e, fma(-om, x[q] - R(weight(q)), B[sh]));
        });
    }
}

// ---------------------------------------------------------------------------
// Fused step: pull the 41 populations of a node along the links (Sec. IV,
// periodic), form rho, j, E (Sec. II), solve the entropic equilibrium
// (Sec. V), relax with the BGK rate omega (Sec. II) and store the
// post-collision values at the node in the other buffer. One node per
// thread; every load and store is coalesced along x. Addresses are a
// per-q scalar base plus a 32-bit byte offset.
//
// ---------------------------------------------------------------------------
// Launch variants (block size, cache-policy hints FL_NT_*); the per-node
// arithmetic is the same in every variant, so results do not depend on the
// choice.

template <class T>
__device__ inline T ld_hint(const T* p, int nt)
{
    if (nt) {
        if constexpr (sizeof(T) == 2) {
            const uint16_t b = __builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p));
            return __builtin_bit_cast(T, b);
        } else {
            return __builtin_nontemporal_load(p);
        }
    }
    return *p;
}

template <class T>
__device__ inline void st_hint(T* p, T v, int nt)
{
    if (nt) {
        if constexpr (sizeof(T) == 2) {
            __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, v), reinterpret_cast<uint16_t*>(p));
        } else {
            __builtin_nontemporal_store(v, p);
        }
    } else {
        *p = v;
    }
}

// Collision of one node from its decoded stored values x, encoded to the
// storage type in out (round to nearest, or stochastic rounding with bits
// drawn for node `nid` of the context at the launch's step); raises the
// flag for an unrealisable node.
// x: decoded stored values (overwritten by the collision for direct storage).
template <class ST, int NEWTON, bool SR, int MODEL, class XR = NoReload>
__device__ __forceinline__ void collide_encode(typename ST::R x[Q], typename ST::T out[Q], const StepParams& p,
                                      uint32_t nid, const XR& xr = XR())
{
    using R = typename ST::R;
    CollideConst<R> cc;
    cc.om = R(p.omega);
    cc.rho_ref = ST::shifted ? R(p.rho_ref) : R(1);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        cc.inv_scale[s] = ST::unit_scale ? R(1) : R(p.inv_scale[s]);
        cc.omw[s] = ST::shifted ? R(p.omw[s]) : cc.om * R(SHELL_W[s]);
    }
    R y[Q], rho, theta;
    // 16-bit storage: the path length to its own resolution
    collide<R, ST::shifted, NEWTON, MODEL, XR, sizeof(typename ST::T) == 2>(x, y, cc, rho, theta, xr);
    flag_bad<R>(p, rho, theta);
    uint32_t rs = 0, rw = 0;
    if constexpr (SR) {
        // random bits per (node of the context, step): the step is the
        // launch's own count plus, in graph replays, a device-held base
        const uint32_t step = p.step + (p.step_base ? *p.step_base : 0u);
        rs = hash32(nid ^ hash32(step * WEYL_STEP + p.seed));
    }
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (SR) {
            if constexpr (q % 2 == 0) rw = weyl_word(rs, uint32_t(q / 2));
            const uint32_t rb = (q % 2 == 0) ? (rw & 0xffffu) : (rw >> 16);
            // 16-bit storage: populations in pairs sharing one random word
            // (measured 2-3% faster, except with the series equilibrium,
            // where it measured 1.7% slower and the single encoder stays)
            if constexpr (ST::shifted && sizeof(typename ST::T) == 2 && (MODEL & MODEL_BASE_MASK) != MODEL_SERIES) {
                if constexpr (q % 2 == 0 && q + 1 < Q) ST::encode_sr2(y[q], y[q + 1], rw, out[q], out[q + 1]);
                else if constexpr (q % 2 == 0) out[q] = ST::encode_sr(y[q], rb);
            } else if constexpr (ST::shifted) {
                out[q] = ST::encode_sr(y[q], rb);
            } else {
                out[q] = sr_add(x[q], y[q], rb);  // stochastic rounding exists for FP32 only
            }
        } else {
            if constexpr (ST::shifted) out[q] = ST::encode(y[q]);
            else if constexpr (DEV_IN_PLACE<R>) out[q] = ST::encode((x[q] + R(weight(q))) + y[q]);  // f = d + w
            else out[q] = ST::encode(x[q] + y[q]);
        }
    });
}

// ---------------------------------------------------------------------------
// Kinetic walls normal to y (Sec. VII.A: diffuse walls of given velocity and
// temperature). Node layers L = 2y + s sit at height L/2; the walls lie a
// quarter cell outside the first and the last layer. A population that would
// arrive from beyond a wall (source layer L - 2 c_y outside) is replaced:
// each wall returns to the node the mass the node sent through it in the
// previous step (its own post-collision populations -c_q, which no node
// pulls), re-emitted in the shape of the wall's equilibrium at unit density:
//   f_q = sigma f_w,q,  sigma = sum f*_{-q} / sum f_w,q  over the replaced q.
// In deviation form (dev = f - w rho_r; f_w,q = w_q (1 + Dw_q)) with
// dsigma = sigma - rho_r = sum (dev_{-q} - rho_r w_q Dw_q) / sum f_w,q, the
// new value is dev_q = w_q (dsigma + sigma Dw_q). Velocities with c_y > 0
// can only come through the lower wall, c_y < 0 through the upper one.
// A specular wall (the inviscid planar wall of Sec. VI.B) returns instead
// the node's own post-collision population (c_x, -c_y, c_z): same shell, so
// the stored value is taken as it is.
// ---------------------------------------------------------------------------
constexpr int WALL_STRIDE = Q + 1;  // per wall: 41 deviations, then the kind
template <class ST>
__device__ __forceinline__ void wall_pull(typename ST::R x[Q], const char* __restrict__ src, uint64_t qbytes,
                                          uint32_t n, int L, int top, const StepParams& p)
{
    using R = typename ST::R;
    using T = typename ST::T;
    const R rr = ST::shifted ? R(p.rho_ref) : R(1);
    const uint64_t nbytes = uint64_t(n) * sizeof(T);
    // deviation of a stored value of shell sh, and back
    auto dev_of = [&](R v, int sh, double w) { return ST::shifted ? v * R(p.inv_scale[sh]) : v - R(w); };
    auto stored_of = [&](R d, int sh, double w) { return ST::shifted ? d * R(p.scale[sh]) : d + R(w); };
    const bool spec[2] = {p.wall_dev[Q] != 0.0, p.wall_dev[WALL_STRIDE + Q] != 0.0};
    R num[2] = {R(0), R(0)}, den[2] = {R(0), R(0)};
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int vy = VEL[q].y;
        if constexpr (vy != 0) {
            constexpr int w = vy > 0 ? 0 : 1;
            constexpr int r = reverse_of(q);
            const bool beyond = vy > 0 ? L < vy : L > top + vy;
            if (beyond && !spec[w]) {
                const R dw = R(p.wall_dev[w * WALL_STRIDE + q]);
                const R out = ST::decode(*reinterpret_cast<const T*>(src + r * qbytes + nbytes));
                num[w] += dev_of(out, VEL[r].shell, weight(r)) - rr * R(weight(q)) * dw;
                den[w] += R(weight(q)) * (R(1) + dw);
            }
        }
    });
    R ds[2], sg[2];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        ds[w] = den[w] > R(0) ? num[w] / den[w] : R(0);
        sg[w] = rr + ds[w];
    }
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int vy = VEL[q].y;
        if constexpr (vy != 0) {
            constexpr int w = vy > 0 ? 0 : 1;
            const bool beyond = vy > 0 ? L < vy : L > top + vy;
            if (beyond) {
                if (spec[w]) {
                    constexpr int m = mirror_y_of(q);
                    x[q] = ST::decode(*reinterpret_cast<const T*>(src + m * qbytes + nbytes));
                } else {
                    const R dw = R(p.wall_dev[w * WALL_STRIDE + q]);
                    x[q] = stored_of(R(weight(q)) * fma(sg[w], dw, ds[w]), VEL[q].shell, weight(q));
                }
            }
        }
    });
}

// Stochastic rounding to FP16 saturates at the largest finite magnitude
// instead of overflowing (see StoreF16S::encode_sr2): a stored value of that
// magnitude is flagged when it is read back. One max of three magnitudes
// per pair of the decoded inputs (written out: the library's fmaxf would
// first quiet possible signalling NaNs of every input).
template <class ST, bool SR>
__device__ __forceinline__ void flag_saturated(const typename ST::R x[Q], const StepParams& p)
{
    if constexpr (SR && ST::SAT > 0.f) {
        float amax = 0.f;
#pragma unroll
        for (int k = 0; k + 1 < Q; k += 2) asm("v_max3_f32 %0, |%1|, |%2|, %0" : "+v"(amax) : "v"(x[k]), "v"(x[k + 1]));
        asm("v_max3_f32 %0, |%1|, |%1|, %0" : "+v"(amax) : "v"(x[Q - 1]));
        if (__builtin_expect(!(amax < ST::SAT), 0)) atomicOr(p.flag, 1u);
    }
}

// The step of node n of one box: src and dst are the box's first q-block
// in the current and the other population buffer.
template <class ST, int NEWTON, int FL, bool SR, int MODEL>
__device__ __forceinline__ void step_node(const char* __restrict__ src, char* __restrict__ dst, const StepParams& p,
                                 uint32_t n)
{
    using R = typename ST::R;
    using T = typename ST::T;
    const Coord c = decode(n, p.g);
    Nbr nb;
    make_nbr(p.g, c, nb, uint32_t(sizeof(T)));
    const uint64_t qbytes = uint64_t(p.g.qs) * sizeof(T);

    R x[Q];
    T out[Q];
    // 16-bit storage: the raw values are also kept two per 32-bit register
    // and decoded again for the relaxation (fewer live registers through the
    // equilibrium solve; the decode is exact, so results are unchanged).
    // Measured at 512^3: FP16-shifted+SR 8.69 -> 8.60 ms per step at the
    // unthrottled clock; at the clock a long run settles to, BF16-shifted+SR
    // 9.21 -> 9.11 ms (112 -> 87 VGPRs) and E1 with SR unchanged. The
    // entropic and wall steps, which need the decoded values again, keep
    // them.
    constexpr bool PACK = sizeof(T) == 2 && !(MODEL & (MODEL_ENTROPIC | MODEL_WALLS));
    if constexpr (PACK) {
        constexpr int QP = (Q + 1) / 2;
        uint32_t pk[QP];
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const T raw = ld_hint(reinterpret_cast<const T*>(src + q * qbytes + uint64_t(pull_src<q>(nb))),
                                  FL & FL_NT_LOAD);
            x[q] = ST::decode(raw);
            const uint32_t b = __builtin_bit_cast(uint16_t, raw);
            if constexpr (q % 2 == 0) pk[q / 2] = b;
            else pk[q / 2] |= b << 16;
        });
        flag_saturated<ST, SR>(x, p);
        // keep the packed words opaque, so the relaxation cannot reuse x
#pragma unroll
        for (int k = 0; k < QP; ++k) asm volatile("" : "+v"(pk[k]));
        auto xr = [&](auto qc) {
            constexpr int q = decltype(qc)::value;
            return ST::decode(__builtin_bit_cast(T, uint16_t(pk[q / 2] >> (16 * (q % 2)))));
        };
        collide_encode<ST, NEWTON, SR, MODEL>(x, out, p, p.node0 + n, xr);
    } else {
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            x[q] = ST::decode(ld_hint(reinterpret_cast<const T*>(src + q * qbytes + uint64_t(pull_src<q>(nb))),
                                      FL & FL_NT_LOAD));
        });
        flag_saturated<ST, SR>(x, p);
        if constexpr ((MODEL & MODEL_WALLS) != 0) {
            // the pulls above wrapped periodically (in bounds); the ones
            // from beyond a wall are replaced
            const int L = int(2 * c.y + c.s), top = int(2 * p.g.ny) - 1;
            if (L < 4 || L > top - 4) wall_pull<ST>(x, src, qbytes, n, L, top, p);
        }
        collide_encode<ST, NEWTON, SR, MODEL>(x, out, p, p.node0 + n);
    }
    const uint32_t nbytes = n * uint32_t(sizeof(T));
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        st_hint(reinterpret_cast<T*>(dst + q * qbytes + uint64_t(nbytes)), out[q], FL & FL_NT_STORE);
    });
}

// One box per launch; fin/fout point at the box's first q-block.
template <class ST, int NEWTON, int BLK, int FL, bool SR, int MODEL = MODEL_E2>
__global__ __launch_bounds__(BLK) void k_step(const typename ST::T* __restrict__ fin,
                                              typename ST::T* __restrict__ fout, StepParams p)
{
    const uint32_t blk = p.xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t n = blk * BLK + threadIdx.x;
    if (n >= p.g.N) return;
    step_node<ST, NEWTON, FL, SR, MODEL>(reinterpret_cast<const char*>(fin), reinterpret_cast<char*>(fout), p, n);
}

// LDS-staged step, 16-bit storage, for tiles of BLK nodes that lie within
// one x-row (BLK divides nx). Every node of such a tile pulls population q
// from the same source row (same sublattice, y and z moves), shifted along
// x by pull_dx<q> in [-2, 2]. The block first copies, for each q, that
// row's segment [x0 - 2, x0 + BLK + 2) (periodic in x) into LDS with
// aligned 32-bit loads: one load instruction covers the tile's span for two
// populations, and the first 2Q threads fetch one halo word each. All loads
// are issued before the first LDS write, so they are in flight together.
// Each node then reads its 41 values from LDS, and reads them again for the
// relaxation rather than keeping them in registers. The per-node arithmetic
// and the stores are step_node's.
template <class ST, int NEWTON, int BLK, int FL, bool SR, int MODEL = MODEL_E2>
__global__ __launch_bounds__(BLK) void k_step_lds(const typename ST::T* __restrict__ fin,
                                                  typename ST::T* __restrict__ fout, StepParams p)
{
    using R = typename ST::R;
    using T = typename ST::T;
    static_assert(sizeof(T) == 2 && (MODEL & MODEL_WALLS) == 0, "LDS staging: 16-bit storage, periodic boxes");
    static_assert(2 * Q <= BLK, "one halo word per thread");
    constexpr int BODY = BLK / 2;  // 32-bit words of the tile's own span of a row
    constexpr int SEG = BODY + 2;  // and one word (two elements) of halo on either side
    constexpr int NP = (Q + 1) / 2;  // passes of two populations
    __shared__ uint32_t stage[Q * SEG];
    const uint32_t blk = p.xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t n0 = blk * BLK;
    const Coord c0 = decode(n0, p.g);  // the tile's row; c0.x is a multiple of BLK
    Nbr nb;
    make_nbr(p.g, c0, nb, uint32_t(sizeof(T)));
    const char* src = reinterpret_cast<const char*>(fin);
    const uint64_t qbytes = uint64_t(p.g.qs) * sizeof(T);
    const uint32_t t = threadIdx.x;
    // byte offsets within a row: the body from x0, the halo words at x0 - 2 and x0 + BLK
    const uint32_t xb = c0.x * 2u;
    const uint32_t xlo = (c0.x == 0 ? p.g.nx - 2u : c0.x - 2u) * 2u;
    const uint32_t xhi = (c0.x + BLK == p.g.nx ? 0u : c0.x + BLK) * 2u;
    const uint32_t odd = t / BODY, w = t - odd * BODY;  // population of the pair, word of the body
    // bodies: pass j copies populations 2j (threads below BODY) and 2j + 1
    // (the last pass, with Q odd, copies population Q - 1 twice)
    uint32_t body[NP];
    static_for<NP>([&](auto jc) {
        constexpr int qa = 2 * decltype(jc)::value, qb = qa + 1 < Q ? qa + 1 : qa;
        const uint32_t q = odd ? uint32_t(qb) : uint32_t(qa);
        const uint32_t row = odd ? pull_row<qb>(nb) : pull_row<qa>(nb);
        body[decltype(jc)::value] = *reinterpret_cast<const uint32_t*>(src + q * qbytes + uint64_t(row + xb + 4 * w));
    });
    // halos: thread t < 2Q fetches the left (t even) or right word of population t / 2
    const uint32_t hq = t >> 1, right = t & 1u;
    uint32_t halo = 0;
    if (t < 2u * Q) {
        uint32_t row = pull_row<0>(nb);
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if constexpr (q > 0) row = hq == uint32_t(q) ? pull_row<q>(nb) : row;
        });
        halo = *reinterpret_cast<const uint32_t*>(src + hq * qbytes + uint64_t(row + (right ? xhi : xlo)));
    }
    static_for<NP>([&](auto jc) {
        constexpr int qa = 2 * decltype(jc)::value, qb = qa + 1 < Q ? qa + 1 : qa;
        stage[(odd ? qb : qa) * SEG + 1 + w] = body[decltype(jc)::value];
    });
    if (t < 2u * Q) stage[hq * SEG + (right ? SEG - 1 : 0)] = halo;
    __syncthreads();
    const uint16_t* st16 = reinterpret_cast<const uint16_t*>(stage);
    // element of population q for this node: segment index t + 2 + dx
    auto lds_val = [&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const int dx = c0.s ? pull_dx<q>(1u) : pull_dx<q>(0u);
        return ST::decode(__builtin_bit_cast(T, st16[q * 2 * SEG + int(t) + 2 + dx]));
    };
    R x[Q];
    T out[Q];
    static_for<Q>([&](auto qc) { x[decltype(qc)::value] = lds_val(qc); });
    flag_saturated<ST, SR>(x, p);
    const uint32_t n = n0 + t;
    collide_encode<ST, NEWTON, SR, MODEL>(x, out, p, p.node0 + n, lds_val);
    char* dst = reinterpret_cast<char*>(fout);
    const uint32_t nbytes = n * uint32_t(sizeof(T));
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        st_hint(reinterpret_cast<T*>(dst + q * qbytes + uint64_t(nbytes)), out[q], FL & FL_NT_STORE);
    });
}

// Collisionless streaming (free flight): every population moves along its
// link unchanged, the update of Sec. II without the collision term. The
// same pull addressing, loads and stores as k_step (T: the stored type), a
// pure permutation of the stored values.
template <class T, int BLK, int FL>
__global__ __launch_bounds__(BLK) void k_stream_free(const T* __restrict__ fin, T* __restrict__ fout, StepParams p)
{
    const uint32_t blk = p.xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t n = blk * BLK + threadIdx.x;
    if (n >= p.g.N) return;
    const Coord c = decode(n, p.g);
    Nbr nb;
    make_nbr(p.g, c, nb, uint32_t(sizeof(T)));
    const uint64_t qbytes = uint64_t(p.g.qs) * sizeof(T);
    const char* src = reinterpret_cast<const char*>(fin);
    char* dst = reinterpret_cast<char*>(fout);
    T v[Q];
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        v[q] = ld_hint(reinterpret_cast<const T*>(src + q * qbytes + uint64_t(pull_src<q>(nb))), FL & FL_NT_LOAD);
    });
    const uint32_t nbytes = n * uint32_t(sizeof(T));
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        st_hint(reinterpret_cast<T*>(dst + q * qbytes + uint64_t(nbytes)), v[q], FL & FL_NT_STORE);
    });
}

// ---------------------------------------------------------------------------
// Batched step: every box of a context in one launch. The grid is the list
// of (box, tile) pairs, box after box, each box cut into tiles of BLK nodes
// (its last tile ragged); a block reads its pair from `tiles`, the box's
// parameters from `boxes` (both uniform across the block, so they sit in
// scalar registers) and runs the same per-node step as k_step.
// ---------------------------------------------------------------------------
struct BatchBox {
    StepParams p;     // geometry, omega, storage scales and node0 of the box
    uint64_t offset;  // element offset of the box in a population buffer
};

template <class ST, int NEWTON, int BLK, int FL, bool SR, int MODEL = MODEL_E2>
__global__ __launch_bounds__(BLK) void k_step_batch(const typename ST::T* __restrict__ fin,
                                                    typename ST::T* __restrict__ fout,
                                                    const BatchBox* __restrict__ boxes,
                                                    const uint2* __restrict__ tiles, uint32_t xcd_remap,
                                                    uint32_t step, const uint32_t* __restrict__ step_base)
{
    const uint32_t t = xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint2 bt = tiles[t];  // (box, tile within the box)
    const BatchBox& B = boxes[bt.x];
    const uint32_t n = bt.y * BLK + threadIdx.x;
    if (n >= B.p.g.N) return;
    StepParams p = B.p;
    p.step = step;
    p.step_base = step_base;
    step_node<ST, NEWTON, FL, SR, MODEL>(reinterpret_cast<const char*>(fin + B.offset),
                                       reinterpret_cast<char*>(fout + B.offset), p, n);
}

}  // namespace lbm
