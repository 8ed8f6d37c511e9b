// Kernels of the RD3Q41 library: the fused pull-collide step, equilibrium
// initialisation, moments, FP64 conservation totals, population I/O and the
// debug pull map.
#pragma once

#include "device.hpp"

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
// Fused step: pull the 41 populations of a node along the links (Sec. IV,
// periodic), form rho, j, E (Sec. II), solve the entropic equilibrium
// (Sec. V), relax with the BGK rate omega (Sec. II) and store the
// post-collision values at the node in the other buffer. One node per
// thread; every load and store is coalesced along x. Addresses are a
// per-q scalar base plus a 32-bit byte offset.
//
// Moments are formed from deviations from the reference state w_q rho_k:
// for direct storage d_q = f_q - w_q (exact in floating point while f_q is
// within a factor two of w_q), for shifted storage the stored h_q scaled
// per shell. Relaxation f* = (1 - omega) f + omega f_eq is folded into one
// fused multiply-add per population, with omega rho/Z (and the storage
// scale) folded into the six shell prefactors of f_eq.
// ---------------------------------------------------------------------------
// Launch variants (block size, cache-policy hints); the per-node arithmetic
// is the same in every variant, so results do not depend on the choice.
constexpr int FL_NT_LOAD = 1;   // non-temporal loads (streamed once)
constexpr int FL_NT_STORE = 2;  // non-temporal stores

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

template <class ST, int NEWTON, int BLK, int FL>
__global__ __launch_bounds__(BLK) void k_step(const typename ST::T* __restrict__ fin,
                                              typename ST::T* __restrict__ fout, StepParams p)
{
    using R = typename ST::R;
    using T = typename ST::T;
    const uint32_t blk = p.xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t n = blk * BLK + threadIdx.x;
    if (n >= p.g.N) return;
    const Coord c = decode(n, p.g);
    Nbr nb;
    make_nbr(p.g, c, nb, uint32_t(sizeof(T)));
    const uint64_t qbytes = uint64_t(p.g.N) * sizeof(T);
    const char* src = reinterpret_cast<const char*>(fin);
    char* dst = reinterpret_cast<char*>(fout);

    R x[Q];
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        x[q] = ST::decode(ld_hint(reinterpret_cast<const T*>(src + q * qbytes + uint64_t(pull_src<q>(nb))),
                                  FL & FL_NT_LOAD));
    });

    ShellSums<R> S;
    R rho_k, e2_k;
    if constexpr (ST::shifted) {
        shell_sums<R>(x, S);
        rho_k = R(p.rho_ref);
        e2_k = R(p.e2_ref);
    } else {
        R d[Q];
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            d[q] = x[q] - R(weight(q));
        });
        shell_sums<R>(d, S);
        rho_k = R(1);
        e2_k = R(3.0 * THETA0);
    }
    R drho = R(0), jx = R(0), jy = R(0), jz = R(0), de2 = R(0);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        R k = R(1);
        if constexpr (ST::shifted) k = R(p.inv_scale[s]);
        const R s0 = k * S.s0[s];
        drho += s0;
        if (s == 0) continue;
        de2 += R(SHELL_C2[s]) * s0;
        const R kc = k * R(SHELL_CA[s]);
        jx += kc * S.sx[s];
        jy += kc * S.sy[s];
        jz += kc * S.sz[s];
    }
    const R rho = rho_k + drho;
    const R irho = R(1) / rho;
    const R ux = jx * irho, uy = jy * irho, uz = jz * irho;
    const R K = (e2_k + de2) * irho;  // 2E/rho = u^2 + 3 theta
    const R u2 = ux * ux + uy * uy + uz * uz;
    const R theta = (K - u2) * R(1.0 / 3.0);
    flag_bad<R>(p, rho, theta);

    Mult<R> m;
    const R ith = R(1) / theta;
    m.b[0] = ux * ith;
    m.b[1] = uy * ith;
    m.b[2] = uz * ith;
    m.g = R(0.5) * ith - R(0.5 / THETA0);
#pragma unroll
    for (int it = 0; it < NEWTON; ++it) newton_step<R>(m, ux, uy, uz, K);

    Gibbs<R> G;
    gibbs_factors<R>(m, G);
    const R om = R(p.omega), om1 = R(1) - om;
    const R oa = om * rho / G.Z;
    R P[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        P[s] = oa * G.T[s];
        if constexpr (ST::shifted) P[s] *= R(p.scale[s]);
    }
    const uint32_t nbytes = n * uint32_t(sizeof(T));
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const R e = gibbs_term<q, R>(G, P);
        R v;
        if constexpr (ST::shifted) v = fma(om1, x[q], e + R(p.cshift[VEL[q].shell]));
        else v = fma(om1, x[q], e);
        st_hint(reinterpret_cast<T*>(dst + q * qbytes + uint64_t(nbytes)), ST::encode(v), FL & FL_NT_STORE);
    });
}

// ---------------------------------------------------------------------------
// Initialisation at equilibrium from FP64 fields (one chunk of nodes).
// mode 0: only measure max_q |f_q - w_q rho0| 2^{k_shell} (for the shifted
// storage exponent); mode 1: store the encoded populations.
// ---------------------------------------------------------------------------
constexpr int INIT_NEWTON = 6;

__device__ inline void equilibrium_f64(double rho, double ux, double uy, double uz, double theta, double e[Q],
                                       double& a)
{
    const double K = ux * ux + uy * uy + uz * uz + 3.0 * theta;
    Mult<double> m;
    m.b[0] = ux / theta;
    m.b[1] = uy / theta;
    m.b[2] = uz / theta;
    m.g = 0.5 / theta - 0.5 / THETA0;
    for (int it = 0; it < INIT_NEWTON; ++it) newton_step<double>(m, ux, uy, uz, K);
    Gibbs<double> G;
    gibbs_factors<double>(m, G);
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        e[q] = gibbs_term<q, double>(G, G.T);
    });
    a = rho / G.Z;
}

__device__ inline void block_max_float(float v, float* out)
{
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    __shared__ float sm[BLOCK / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sm[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = sm[0];
        for (int i = 1; i < BLOCK / 64; ++i) r = fmaxf(r, sm[i]);
        // non-negative floats order like their bit patterns
        atomicMax(reinterpret_cast<unsigned int*>(out), __float_as_uint(r));
    }
}

template <class ST>
__global__ __launch_bounds__(BLOCK) void k_init(typename ST::T* __restrict__ f, uint32_t N, uint32_t n0,
                                                uint32_t count, const double* __restrict__ fields, StepParams p,
                                                int mode, float* maxdev)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    float dev = 0.f;
    if (i < count) {
        const double rho = fields[i], ux = fields[count + i], uy = fields[2 * count + i],
                     uz = fields[3 * count + i], th = fields[4 * count + i];
        double e[Q], a;
        equilibrium_f64(rho, ux, uy, uz, th, e, a);
        bool bad = !(a > 0.0) || !(a < 1e300);
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int sh = VEL[q].shell;
            const double d = a * e[q] - SHELL_W[sh] * p.rho_ref;
            bad |= !(fabs(d) < 1e300);
            if (mode == 0) {
                dev = fmaxf(dev, float(fabs(d) * double(1u << SHELL_K[sh])));
            } else {
                double v = d;
                if constexpr (ST::shifted) v *= double(p.scale[sh]);
                ST::store(f + size_t(q) * N + n0 + i, typename ST::R(v));
            }
        });
        if (bad) atomicOr(p.flag, 1u);
    }
    if (mode == 0) block_max_float(dev, maxdev);
}

// ---------------------------------------------------------------------------
// FP64 decoding helpers for the diagnostics kernels.
// ---------------------------------------------------------------------------
template <class ST, int q>
__device__ inline double dev64(const typename ST::T* f, size_t N, uint32_t n, const StepParams& p)
{
    double v = double(ST::load(f + size_t(q) * N + n));
    if constexpr (ST::shifted) v *= double(p.inv_scale[VEL[q].shell]);
    return v;
}

// rho, jx, jy, jz, E of node n in FP64.
template <class ST>
__device__ inline void node_moments64(const typename ST::T* f, size_t N, uint32_t n, const StepParams& p,
                                      double m[5])
{
    double rd = 0, jx = 0, jy = 0, jz = 0, e4 = 0;
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr HalfVel v = VEL[q];
        const double d = dev64<ST, q>(f, N, n, p);
        rd += d;
        jx += double(v.x) * d;
        jy += double(v.y) * d;
        jz += double(v.z) * d;
        e4 += double(v.x * v.x + v.y * v.y + v.z * v.z) * d;
    });
    m[0] = p.rho_ref + rd;
    m[1] = 0.5 * jx;
    m[2] = 0.5 * jy;
    m[3] = 0.5 * jz;
    m[4] = 0.5 * (p.e2_ref + 0.25 * e4);
}

template <class ST>
__global__ __launch_bounds__(BLOCK) void k_moments(const typename ST::T* __restrict__ f, uint32_t N, uint32_t n0,
                                                   uint32_t count, StepParams p, double* __restrict__ out)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= count) return;
    double m[5];
    node_moments64<ST>(f, N, n0 + i, p, m);
#pragma unroll
    for (int k = 0; k < 5; ++k) out[size_t(k) * count + i] = m[k];
}

// Block-wide FP64 sum of 5 values: wavefront butterfly (64 lanes), then the
// 4 wave partials in LDS. Result valid in thread 0.
__device__ inline void block_sum5(double v[5], double out[5])
{
#pragma unroll
    for (int k = 0; k < 5; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    __shared__ double sm[BLOCK / 64][5];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 5; ++k) sm[wv][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) {
            double s = sm[0][k];
            for (int i = 1; i < BLOCK / 64; ++i) s += sm[i][k];
            out[k] = s;
        }
}

constexpr int TOTAL_BLOCKS = 1024;

// Per-block partial sums of the node moments (fixed assignment of nodes to
// threads, so the result does not depend on timing).
template <class ST>
__global__ __launch_bounds__(BLOCK) void k_totals(const typename ST::T* __restrict__ f, uint32_t N, StepParams p,
                                                  double* __restrict__ partials)
{
    double acc[5] = {0, 0, 0, 0, 0};
    for (uint32_t n = blockIdx.x * BLOCK + threadIdx.x; n < N; n += gridDim.x * BLOCK) {
        double m[5];
        node_moments64<ST>(f, N, n, p, m);
#pragma unroll
        for (int k = 0; k < 5; ++k) acc[k] += m[k];
    }
    double r[5];
    block_sum5(acc, r);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) partials[blockIdx.x * 5 + k] = r[k];
}

__global__ __launch_bounds__(BLOCK) void k_reduce_partials(const double* __restrict__ partials, uint32_t nblk,
                                                           double* __restrict__ out)
{
    double acc[5] = {0, 0, 0, 0, 0};
    for (uint32_t b = threadIdx.x; b < nblk; b += BLOCK)
        for (int k = 0; k < 5; ++k) acc[k] += partials[b * 5 + k];
    double r[5];
    block_sum5(acc, r);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) out[k] = r[k];
}

// ---------------------------------------------------------------------------
// Population I/O in FP64: one q-block chunk [n0, n0 + count) at a time.
// ---------------------------------------------------------------------------
template <class ST>
__global__ __launch_bounds__(BLOCK) void k_get(const typename ST::T* __restrict__ fq, uint32_t count, float inv_scale,
                                               double wref, double* __restrict__ out)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= count) return;
    double v = double(ST::load(fq + i));
    if constexpr (ST::shifted) v *= double(inv_scale);
    out[i] = wref + v;
}

template <class ST>
__global__ __launch_bounds__(BLOCK) void k_set(typename ST::T* __restrict__ fq, uint32_t count, float scale,
                                               double wref, const double* __restrict__ in)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= count) return;
    double v = in[i] - wref;
    if constexpr (ST::shifted) v *= double(scale);
    ST::store(fq + i, typename ST::R(v));
}

template <class ST>
__global__ __launch_bounds__(BLOCK) void k_gather(const typename ST::T* __restrict__ f, uint32_t N,
                                                  const int64_t* __restrict__ idx, uint32_t count, StepParams p,
                                                  double* __restrict__ out)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= count) return;
    const int64_t k = idx[i];
    const uint32_t q = uint32_t(k / N), n = uint32_t(k - int64_t(q) * N);
    const int sh = q == 0 ? 0 : q < 7 ? 1 : q < 13 ? 2 : q < 25 ? 3 : q < 33 ? 4 : 5;
    double v = double(ST::load(f + size_t(q) * N + n));
    if constexpr (ST::shifted) v *= double(p.inv_scale[sh]);
    out[i] = SHELL_W[sh] * p.rho_ref + v;
}

// Source node of every (q, node) of a chunk, by the same code as k_step.
__global__ __launch_bounds__(BLOCK) void k_pull_map(Geom g, uint32_t n0, uint32_t count, int64_t* __restrict__ out)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= count) return;
    const Coord c = decode(n0 + i, g);
    Nbr nb;
    make_nbr(g, c, nb);
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        out[size_t(q) * count + i] = int64_t(pull_src<q>(nb));
    });
}

}  // namespace lbm
