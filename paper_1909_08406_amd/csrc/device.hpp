// Device building blocks of the fused RD3Q41 update: node decoding and the
// periodic two-sublattice pull map (Sec. IV), moments (Sec. II), the exact
// entropic equilibrium through the closed-form shell partition function
// (Sec. V), and the storage encodings.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "lattice.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// Division by a run-time invariant divisor: n / d = (umulhi(n, m) + n) >> l
// with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1, exact for all
// 32-bit n (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994).
// ---------------------------------------------------------------------------
struct FastDiv {
    uint32_t d, m, l;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
    return FastDiv{d, uint32_t(m), l};
}

__host__ __device__ inline uint32_t umulhi32(uint32_t a, uint32_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umulhi(a, b);
#else
    return uint32_t((uint64_t(a) * b) >> 32);
#endif
}

__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f)
{
    uint32_t t = umulhi32(n, f.m);
    return uint32_t((uint64_t(t) + n) >> f.l);
}

// ---------------------------------------------------------------------------
// Box geometry and the pull map.
// ---------------------------------------------------------------------------
struct Geom {
    uint32_t nx, ny, nz;
    uint32_t nxy;    // nx*ny
    uint32_t plane;  // nx*ny*nz, nodes of one sublattice
    uint32_t N;      // 2*plane
    FastDiv dx, dy, dz;
};

inline Geom make_geom(uint32_t nx, uint32_t ny, uint32_t nz)
{
    Geom g;
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.nxy = nx * ny;
    g.plane = nx * ny * nz;
    g.N = 2 * g.plane;
    g.dx = make_fastdiv(nx);
    g.dy = make_fastdiv(ny);
    g.dz = make_fastdiv(nz);
    return g;
}

struct Coord {
    uint32_t x, y, z, s;
};

__device__ inline Coord decode(uint32_t n, const Geom& g)
{
    Coord c;
    uint32_t r = fdiv(n, g.dx);
    c.x = n - r * g.nx;
    uint32_t r2 = fdiv(r, g.dy);
    c.y = r - r2 * g.ny;
    c.s = fdiv(r2, g.dz);
    c.z = r2 - c.s * g.nz;
    return c;
}

// Wrapped neighbour offsets of one node, scaled by `unit` (1 for node ids,
// sizeof(element) for byte offsets into a q-block). For an integer move by d
// in [-2, 2] along an axis the source coordinate is (x - d) mod n, held in
// o[2 - d]; i.e. o[k] = ((x + k - 2) mod n) * stride. The half moves sigma/2
// (sigma = +-1) connect the sublattices: a node at x + s/2 receives from the
// other sublattice at x + s - (1 + sigma)/2, held in h[0] for sigma = +1 and
// h[1] for sigma = -1.
struct Nbr {
    uint32_t xo[5], yo[5], zo[5];
    uint32_t xh[2], yh[2], zh[2];
    uint32_t so, sh;  // own and opposite sublattice offsets
};

__device__ inline void axis_wrap(uint32_t x, uint32_t n, uint32_t stride, uint32_t s, uint32_t o[5], uint32_t h[2])
{
    uint32_t m1 = x == 0 ? n - 1 : x - 1;
    uint32_t m2 = m1 == 0 ? n - 1 : m1 - 1;
    uint32_t p1 = x + 1 == n ? 0 : x + 1;
    uint32_t p2 = p1 + 1 == n ? 0 : p1 + 1;
    o[0] = m2 * stride;
    o[1] = m1 * stride;
    o[2] = x * stride;
    o[3] = p1 * stride;
    o[4] = p2 * stride;
    h[0] = s ? o[2] : o[1];
    h[1] = s ? o[3] : o[2];
}

__device__ inline void make_nbr(const Geom& g, const Coord& c, Nbr& nb, uint32_t unit = 1)
{
    axis_wrap(c.x, g.nx, unit, c.s, nb.xo, nb.xh);
    axis_wrap(c.y, g.ny, g.nx * unit, c.s, nb.yo, nb.yh);
    axis_wrap(c.z, g.nz, g.nxy * unit, c.s, nb.zo, nb.zh);
    nb.so = c.s ? g.plane * unit : 0;
    nb.sh = c.s ? 0 : g.plane * unit;
}

// Offset (in the unit of make_nbr) of the node that population q is pulled
// from (Sec. IV: streaming along the links of the bcc lattice, periodic).
template <int q>
__device__ inline uint32_t pull_src(const Nbr& nb)
{
    constexpr HalfVel v = VEL[q];
    if constexpr (v.shell == 5) {
        return nb.sh + nb.zh[v.z > 0 ? 0 : 1] + nb.yh[v.y > 0 ? 0 : 1] + nb.xh[v.x > 0 ? 0 : 1];
    } else {
        return nb.so + nb.zo[2 - v.z / 2] + nb.yo[2 - v.y / 2] + nb.xo[2 - v.x / 2];
    }
}

// ---------------------------------------------------------------------------
// Arithmetic helpers per compute type.
// ---------------------------------------------------------------------------
template <typename R> __device__ inline R d_exp(R x);
template <> __device__ inline float d_exp<float>(float x) { return __expf(x); }
template <> __device__ inline double d_exp<double>(double x) { return exp(x); }

template <typename R> __device__ inline R d_rcp(R x);
template <> __device__ inline float d_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double d_rcp<double>(double x) { return 1.0 / x; }

// e^{h/2} and e^{-h/2}
template <typename R>
__device__ inline void half_exp_pair(R h, R& ep, R& em)
{
    ep = d_exp<R>(R(0.5) * h);
    if constexpr (sizeof(R) == 4) em = d_exp<R>(R(-0.5) * h);
    else em = d_rcp<R>(ep);
}

// ---------------------------------------------------------------------------
// Exact entropic equilibrium (Sec. V).
//
// With f_eq,i = rho w_i e^{b.c_i - g c_i^2} / Z(b, g) and
// Z = sum_i w_i e^{b.c_i - g c_i^2} (the paper's beta = -b, gamma = g,
// alpha = ln Z), mass holds by construction and momentum and energy require
//     d lnZ / d b = u,   -d lnZ / d g = u^2 + 3 theta = K.
// Z sums in closed form over the six shells with cosh/sinh of b_a/2, b_a,
// 2 b_a and powers of t = e^{-g/4}. Newton minimises the convex function
// lnZ - b.u + g K; its Hessian is the 4x4 covariance of (c, -c^2) under
// the equilibrium, symmetric positive definite. Start: the continuous
// Maxwellian, b = u/theta, g = 1/(2 theta) - 1/(2 theta0).
// ---------------------------------------------------------------------------
template <typename R>
struct Mult {
    R b[3];
    R g;
};

template <typename R>
__device__ inline void newton_step(Mult<R>& m, R ux, R uy, R uz, R K)
{
    const R w0 = R(W_REST), w1 = R(W_SC1), w2 = R(W_SC2), w3 = R(W_FCC), w4 = R(W_BCC), w5 = R(W_HALF);
    R Ch[3], Sh[3], C1[3], S1[3], C2[3], S2[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R ep, em;
        half_exp_pair<R>(m.b[a], ep, em);
        Ch[a] = R(0.5) * (ep + em);
        Sh[a] = R(0.5) * (ep - em);
        C1[a] = R(1) + R(2) * Sh[a] * Sh[a];
        S1[a] = R(2) * Sh[a] * Ch[a];
        C2[a] = R(1) + R(2) * S1[a] * S1[a];
        S2[a] = R(2) * S1[a] * C1[a];
    }
    const R t = d_exp<R>(R(-0.25) * m.g);
    const R t2 = t * t, t3 = t2 * t, t4 = t2 * t2, t8 = t4 * t4, t12 = t8 * t4, t16 = t8 * t8;
    const R T1 = w1 * t4, T2 = w2 * t16, T3 = w3 * t8, T4 = w4 * t12, T5 = w5 * t3;

    // pair products of the fcc shell and triple products of the bcc shells
    const R Pxy = C1[0] * C1[1], Pxz = C1[0] * C1[2], Pyz = C1[1] * C1[2];
    const R P3 = Pxy * C1[2];
    const R H3 = Ch[0] * Ch[1] * Ch[2];
    const R sc1 = R(2) * T1 * (C1[0] + C1[1] + C1[2]);
    const R sc2 = R(2) * T2 * (C2[0] + C2[1] + C2[2]);
    const R fcc = R(4) * T3 * (Pxy + Pxz + Pyz);
    const R bcc = R(8) * T4 * P3;
    const R hlf = R(8) * T5 * H3;

    const R Z = w0 + sc1 + sc2 + fcc + bcc + hlf;                               // <1>
    const R N2 = sc1 + R(4) * sc2 + R(2) * fcc + R(3) * bcc + R(0.75) * hlf;     // <c^2>
    const R N4 = sc1 + R(16) * sc2 + R(4) * fcc + R(9) * bcc + R(0.5625) * hlf;  // <c^4>

    R M[3], XX[3], XC[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int b = (a + 1) % 3, c = (a + 2) % 3;
        const R s1 = R(2) * T1 * S1[a];
        const R s2 = R(4) * T2 * S2[a];
        const R f = R(4) * T3 * S1[a] * (C1[b] + C1[c]);
        const R bb = R(8) * T4 * S1[a] * C1[b] * C1[c];
        const R hh = R(4) * T5 * Sh[a] * Ch[b] * Ch[c];
        M[a] = s1 + s2 + f + bb + hh;                                          // <c_a>
        XC[a] = s1 + R(4) * s2 + R(2) * f + R(3) * bb + R(0.75) * hh;          // <c_a c^2>
        XX[a] = R(2) * T1 * C1[a] + R(8) * T2 * C2[a] + R(4) * T3 * C1[a] * (C1[b] + C1[c]) + bcc + R(0.25) * hlf;  // <c_a^2>
    }
    // <c_a c_b>, a < b
    const R XYxy = R(4) * T3 * S1[0] * S1[1] + R(8) * T4 * S1[0] * S1[1] * C1[2] + R(2) * T5 * Sh[0] * Sh[1] * Ch[2];
    const R XYxz = R(4) * T3 * S1[0] * S1[2] + R(8) * T4 * S1[0] * S1[2] * C1[1] + R(2) * T5 * Sh[0] * Sh[2] * Ch[1];
    const R XYyz = R(4) * T3 * S1[1] * S1[2] + R(8) * T4 * S1[1] * S1[2] * C1[0] + R(2) * T5 * Sh[1] * Sh[2] * Ch[0];

    const R iz = d_rcp<R>(Z);
    const R mu0 = M[0] * iz, mu1 = M[1] * iz, mu2 = M[2] * iz, m2 = N2 * iz;
    // gradient of lnZ - b.u + g K
    const R r0 = mu0 - ux, r1 = mu1 - uy, r2 = mu2 - uz, r3 = K - m2;
    // Hessian (covariance of (c, -c^2))
    const R H00 = XX[0] * iz - mu0 * mu0, H11 = XX[1] * iz - mu1 * mu1, H22 = XX[2] * iz - mu2 * mu2;
    const R H10 = XYxy * iz - mu1 * mu0, H20 = XYxz * iz - mu2 * mu0, H21 = XYyz * iz - mu2 * mu1;
    const R H30 = m2 * mu0 - XC[0] * iz, H31 = m2 * mu1 - XC[1] * iz, H32 = m2 * mu2 - XC[2] * iz;
    const R H33 = N4 * iz - m2 * m2;

    // LDL^T factorisation and solve of H d = r
    const R D0 = H00, iD0 = d_rcp<R>(D0);
    const R l10 = H10 * iD0, l20 = H20 * iD0, l30 = H30 * iD0;
    const R D1 = H11 - l10 * H10, iD1 = d_rcp<R>(D1);
    const R l21 = (H21 - l20 * H10) * iD1, l31 = (H31 - l30 * H10) * iD1;
    const R D2 = H22 - l20 * H20 - l21 * l21 * D1, iD2 = d_rcp<R>(D2);
    const R l32 = (H32 - l30 * H20 - l31 * l21 * D1) * iD2;
    const R D3 = H33 - l30 * H30 - l31 * l31 * D1 - l32 * l32 * D2, iD3 = d_rcp<R>(D3);
    const R y0 = r0, y1 = r1 - l10 * y0, y2 = r2 - l20 * y0 - l21 * y1, y3 = r3 - l30 * y0 - l31 * y1 - l32 * y2;
    const R x3 = y3 * iD3;
    const R x2 = y2 * iD2 - l32 * x3;
    const R x1 = y1 * iD1 - l21 * x2 - l31 * x3;
    const R x0 = y0 * iD0 - l10 * x1 - l20 * x2 - l30 * x3;
    m.b[0] -= x0;
    m.b[1] -= x1;
    m.b[2] -= x2;
    m.g -= x3;
}

// Factors of the Gibbs terms w_q e^{b.c_q - g c_q^2}: per-axis powers
// e^{+-b/2}, e^{+-b}, e^{+-2b}, the shell prefactors w_s t^{4 |c_s|^2}
// (t = e^{-g/4}) and Z = sum_q w_q e^{...} in closed form over the shells.
template <typename R>
struct Gibbs {
    R p1[3], m1[3], p2[3], m2[3], p4[3], m4[3];
    R T[6];
    R Z;
};

template <typename R>
__device__ inline void gibbs_factors(const Mult<R>& m, Gibbs<R>& G)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        half_exp_pair<R>(m.b[a], G.p1[a], G.m1[a]);  // e^{+-b/2}
        G.p2[a] = G.p1[a] * G.p1[a];
        G.m2[a] = G.m1[a] * G.m1[a];                 // e^{+-b}
        G.p4[a] = G.p2[a] * G.p2[a];
        G.m4[a] = G.m2[a] * G.m2[a];                 // e^{+-2b}
    }
    const R t = d_exp<R>(R(-0.25) * m.g);
    const R t2 = t * t, t3 = t2 * t, t4 = t2 * t2, t8 = t4 * t4, t12 = t8 * t4, t16 = t8 * t8;
    G.T[0] = R(W_REST);
    G.T[1] = R(W_SC1) * t4;
    G.T[2] = R(W_SC2) * t16;
    G.T[3] = R(W_FCC) * t8;
    G.T[4] = R(W_BCC) * t12;
    G.T[5] = R(W_HALF) * t3;
    R C[3], D[3], H[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C[a] = G.p2[a] + G.m2[a];  // 2 cosh b
        D[a] = G.p4[a] + G.m4[a];  // 2 cosh 2b
        H[a] = G.p1[a] + G.m1[a];  // 2 cosh b/2
    }
    G.Z = G.T[0] + G.T[1] * (C[0] + C[1] + C[2]) + G.T[2] * (D[0] + D[1] + D[2]) +
          G.T[3] * (C[0] * C[1] + C[0] * C[2] + C[1] * C[2]) + G.T[4] * (C[0] * C[1] * C[2]) +
          G.T[5] * (H[0] * H[1] * H[2]);
}

// P_s times the velocity-dependent factor of term q: P_s e^{b.c_q} with
// P_s standing for (a multiple of) the shell prefactor.
template <int q, typename R>
__device__ inline R gibbs_term(const Gibbs<R>& G, const R P[6])
{
    constexpr HalfVel v = VEL[q];
    auto fac = [&](int a, int h) -> R {
        switch (h) {
            case 1: return G.p1[a];
            case -1: return G.m1[a];
            case 2: return G.p2[a];
            case -2: return G.m2[a];
            case 4: return G.p4[a];
            case -4: return G.m4[a];
            default: return R(1);
        }
    };
    R val = P[v.shell];
    if constexpr (v.x != 0) val *= fac(0, v.x);
    if constexpr (v.y != 0) val *= fac(1, v.y);
    if constexpr (v.z != 0) val *= fac(2, v.z);
    return val;
}

// ---------------------------------------------------------------------------
// Moments of 41 values by shell: for each shell s the plain sum and the sums
// signed by the sign of c_x, c_y, c_z (the magnitude |c_a| of a shell is
// applied by the caller). The two 8-velocity shells use a butterfly.
// ---------------------------------------------------------------------------
template <typename R>
struct ShellSums {
    R s0[6], sx[6], sy[6], sz[6];
};

template <typename R>
__device__ inline void cube8(const R* v, R& s0, R& sx, R& sy, R& sz)
{
    // order (+++), (++-), (+-+), (+--), (-++), (-+-), (--+), (---)
    const R a0 = v[0] + v[1], a1 = v[0] - v[1], a2 = v[2] + v[3], a3 = v[2] - v[3];
    const R a4 = v[4] + v[5], a5 = v[4] - v[5], a6 = v[6] + v[7], a7 = v[6] - v[7];
    const R b0 = a0 + a2, b1 = a0 - a2, b2 = a1 + a3;
    const R c0 = a4 + a6, c1 = a4 - a6, c2 = a5 + a7;
    s0 = b0 + c0;
    sx = b0 - c0;
    sy = b1 + c1;
    sz = b2 + c2;
}

// four values of one coordinate plane of the fcc shell: (+,+), (+,-), (-,+), (-,-)
template <typename R>
__device__ inline void plane4(R pp, R pm, R mp, R mm, R& s0, R& d1, R& d2)
{
    const R u1 = pp + pm, u2 = mp + mm, v1 = pp - pm, v2 = mp - mm;
    s0 = u1 + u2;
    d1 = u1 - u2;
    d2 = v1 + v2;
}

template <typename R>
__device__ inline void shell_sums(const R x[Q], ShellSums<R>& S)
{
    S.s0[0] = x[0];
    S.sx[0] = S.sy[0] = S.sz[0] = R(0);
    // sc-1 (q 1..6) and sc-2 (q 7..12): +x, +y, +z, -z, -y, -x
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const R* v = x + 1 + 6 * k;
        S.s0[1 + k] = (v[0] + v[5]) + (v[1] + v[4]) + (v[2] + v[3]);
        S.sx[1 + k] = v[0] - v[5];
        S.sy[1 + k] = v[1] - v[4];
        S.sz[1 + k] = v[2] - v[3];
    }
    // fcc-1 (q 13..24): (1,1,0) (1,0,1) (1,0,-1) (1,-1,0) (0,1,1) (0,1,-1)
    //                   (0,-1,1) (0,-1,-1) (-1,1,0) (-1,0,1) (-1,0,-1) (-1,-1,0)
    {
        const R* v = x + 13;
        R sxy, dxy_x, dxy_y, sxz, dxz_x, dxz_z, syz, dyz_y, dyz_z;
        plane4(v[0], v[3], v[8], v[11], sxy, dxy_x, dxy_y);
        plane4(v[1], v[2], v[9], v[10], sxz, dxz_x, dxz_z);
        plane4(v[4], v[5], v[6], v[7], syz, dyz_y, dyz_z);
        S.s0[3] = sxy + sxz + syz;
        S.sx[3] = dxy_x + dxz_x;
        S.sy[3] = dxy_y + dyz_y;
        S.sz[3] = dxz_z + dyz_z;
    }
    cube8(x + 25, S.s0[4], S.sx[4], S.sy[4], S.sz[4]);  // bcc-1
    cube8(x + 33, S.s0[5], S.sx[5], S.sy[5], S.sz[5]);  // bcc-1/2
}

// |c_a| of a nonzero component and |c|^2, per shell
constexpr double SHELL_CA[6] = {0.0, 1.0, 2.0, 1.0, 1.0, 0.5};

// ---------------------------------------------------------------------------
// Storage encodings. Every kernel works on deviations d_q = f_q - w_q rho_ref
// with rho_ref = rho0 for the shifted forms and 0 otherwise; the shifted
// forms hold h_q = d_q 2^{k_q} in 16 bits.
// ---------------------------------------------------------------------------
struct StoreF64 {
    using T = double;
    using R = double;
    static constexpr bool shifted = false;
    __device__ static R decode(T v) { return v; }
    __device__ static T encode(R v) { return v; }
    __device__ static R load(const T* p) { return *p; }
    __device__ static void store(T* p, R v) { *p = v; }
};

struct StoreF32 {
    using T = float;
    using R = float;
    static constexpr bool shifted = false;
    __device__ static R decode(T v) { return v; }
    __device__ static T encode(R v) { return v; }
    __device__ static R load(const T* p) { return *p; }
    __device__ static void store(T* p, R v) { *p = v; }
};

struct StoreF16S {
    using T = _Float16;
    using R = float;
    static constexpr bool shifted = true;
    __device__ static R decode(T v) { return float(v); }
    __device__ static T encode(R v) { return _Float16(v); }  // round to nearest even
    __device__ static R load(const T* p) { return float(*p); }
    __device__ static void store(T* p, R v) { *p = _Float16(v); }
};

// bfloat16 conversions on the host: decode by a 16-bit shift, encode with
// round-to-nearest-even on the dropped 16 bits (NaN kept quiet).
inline uint16_t host_f32_to_bf16_rne(float v)
{
    uint32_t u;
    std::memcpy(&u, &v, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
inline float host_bf16_to_f32(uint16_t b)
{
    const uint32_t u = uint32_t(b) << 16;
    float v;
    std::memcpy(&v, &u, 4);
    return v;
}

// On the device the conversion float -> __bf16 is the hardware
// round-to-nearest-even conversion of gfx950.
struct StoreBF16S {
    using T = __bf16;
    using R = float;
    static constexpr bool shifted = true;
    __device__ static R decode(T v) { return float(v); }
    __device__ static T encode(R v) { return __bf16(v); }
    __device__ static R load(const T* p) { return float(*p); }
    __device__ static void store(T* p, R v) { *p = __bf16(v); }
};

// Parameters of the step kernels (passed by value).
struct StepParams {
    Geom g;
    double omega;          // relaxation rate
    float scale[6];        // 2^{k_shell + k_amp}   (shifted storage)
    float inv_scale[6];    // 2^{-(k_shell + k_amp)}
    float cshift[6];       // -omega w_shell rho0 2^{k_shell + k_amp} (shifted storage)
    double rho_ref;        // rho0 (shifted) or 0: reference of the stored values
    double e2_ref;         // sum_q w_q rho_ref c_q^2 = 3 rho_ref theta0
    uint32_t* flag;        // set to 1 when a node has rho <= 0, theta <= 0 or NaN
    uint32_t xcd_remap;    // 1: group consecutive tiles per XCD
};

}  // namespace lbm
