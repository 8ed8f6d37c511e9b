// Kernels of the RD3Q41 library besides the step: equilibrium
// initialisation, moments, FP64 conservation totals and Fourier
// projections, population I/O and the debug pull map. Included by the host
// side of the library only (lbm.hip).
#pragma once

#include "kernels.hpp"

namespace lbm {

// Device-held step counter read by graph replays (one vector store).
__global__ void k_set_counter(uint32_t* __restrict__ ctr, uint32_t v)
{
    if (threadIdx.x == 0) ctr[0] = v;
}

// ---------------------------------------------------------------------------
// Initialisation at equilibrium from FP64 fields (one chunk of nodes).
// mode 0: only measure max_q |f_q - w_q rho0| 2^{k_shell} (for the shifted
// storage exponent); mode 1: store the encoded populations.
// ---------------------------------------------------------------------------
constexpr int INIT_NEWTON = 6;

// Deviations D_q (f_eq,q = w_q rho_ref (1 + D_q)) of the equilibrium of
// (rho, u, theta) in FP64, relative to the reference state w_q rho_ref.
// model: MODEL_E2, MODEL_ISO (theta unused) or MODEL_SERIES.
__host__ __device__ inline void equilibrium_dev_f64(double rho, double ux, double uy, double uz, double theta,
                                                    double rho_ref, int model, double D[Q])
{
    NodeDev<double> st;
    st.rho_ref = rho_ref;
    st.rho = rho;
    st.irho = 1.0 / rho;
    st.drho = rho - rho_ref * SUM_W;
    st.j[0] = rho * ux;
    st.j[1] = rho * uy;
    st.j[2] = rho * uz;
    st.de2 = rho * (ux * ux + uy * uy + uz * uz + 3.0 * theta) - rho_ref * SUM_WC2;
    model &= MODEL_BASE_MASK;  // the path length plays no part in the equilibrium
    if (model == MODEL_SERIES) {
        SeriesCoef<double> sc;
        series_coef<double>(ux, uy, uz, theta / THETA0 - 1.0, sc);
        const double kap = st.drho / (rho_ref * SUM_W);
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            D[q] = dmul(series_eps<q, double>(sc), kap);
        });
        return;
    }
    Mult<double> m;
    if (model == MODEL_ISO) {
        m.b[0] = ux / THETA0;
        m.b[1] = uy / THETA0;
        m.b[2] = uz / THETA0;
        m.g = 0.0;
        for (int it = 0; it < INIT_NEWTON; ++it) newton_step<double, false>(m, st);
    } else {
        m.b[0] = ux / theta;
        m.b[1] = uy / theta;
        m.b[2] = uz / theta;
        m.g = 0.5 / theta - 0.5 / THETA0;
        for (int it = 0; it < INIT_NEWTON; ++it) newton_step<double>(m, st);
    }
    Shells<double> S;
    shells_at<double>(m, S);
    const double kap = kappa_of<double>(st, S);
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        D[q] = dmul(gibbs_dev<q, double>(S), kap);
    });
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

// Nodal FP64 fields of one chunk of nodes (host data staged on the device,
// or device arrays of the caller), element i for node n0 + i.
struct InitFields {
    const double* rho;
    const double* ux;
    const double* uy;
    const double* uz;
    const double* th;
};

template <class ST>
__global__ __launch_bounds__(BLOCK) void k_init(typename ST::T* __restrict__ f, uint32_t qs, uint32_t n0,
                                                uint32_t count, InitFields fields, StepParams p, int mode,
                                                float* maxdev)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    float dev = 0.f;
    if (i < count) {
        const double rho = fields.rho[i], ux = fields.ux[i], uy = fields.uy[i], uz = fields.uz[i], th = fields.th[i];
        // the domain: rho > 0, theta > 0 (checked but unused by the
        // isothermal model), all finite
        const bool in_domain = rho > 0.0 && th > 0.0 && fabs(rho) < 1e300 && fabs(th) < 1e300 &&
                               fabs(ux) < 1e300 && fabs(uy) < 1e300 && fabs(uz) < 1e300;
        // storage reference: rho0 for the shifted forms, the weights themselves otherwise
        const double rref = ST::shifted ? p.rho_ref : 1.0;
        double D[Q];
        equilibrium_dev_f64(rho, ux, uy, uz, th, rref, int(p.model), D);
        bool bad = false;
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int sh = VEL[q].shell;
            const double d = SHELL_W[sh] * rref * D[q];  // f_eq,q - w_q rref
            bad |= !(fabs(d) < 1e300) || !(SHELL_W[sh] * rref + d > 0.0);
            if (mode == 0) {
                dev = fmaxf(dev, float(fabs(d) * double(1u << SHELL_K[sh])));
            } else {
                double v;
                if constexpr (ST::shifted) v = d * double(p.scale[sh]);
                else v = SHELL_W[sh] + d;
                ST::store(f + size_t(q) * qs + n0 + i, typename ST::R(v));
            }
        });
        if (bad || !in_domain) atomicOr(p.flag, 1u);
    }
    if (mode == 0) block_max_float(dev, maxdev);
}

// ---------------------------------------------------------------------------
// FP64 decoding helpers for the diagnostics kernels.
// ---------------------------------------------------------------------------
template <class ST, int q>
__device__ inline double dev64(const typename ST::T* f, size_t qs, uint32_t n, const StepParams& p)
{
    double v = double(ST::load(f + size_t(q) * qs + n));
    if constexpr (ST::shifted) v *= double(p.inv_scale[VEL[q].shell]);
    return v;
}

// rho, jx, jy, jz, E of node n in FP64.
template <class ST>
__device__ inline void node_moments64(const typename ST::T* f, size_t qs, uint32_t n, const StepParams& p,
                                      double m[5])
{
    double rd = 0, jx = 0, jy = 0, jz = 0, e4 = 0;
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr HalfVel v = VEL[q];
        const double d = dev64<ST, q>(f, qs, n, p);
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
__global__ __launch_bounds__(BLOCK) void k_moments(const typename ST::T* __restrict__ f, uint32_t qs, uint32_t n0,
                                                   uint32_t count, StepParams p, double* __restrict__ out)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= count) return;
    double m[5];
    node_moments64<ST>(f, qs, n0 + i, p, m);
#pragma unroll
    for (int k = 0; k < 5; ++k) out[size_t(k) * count + i] = m[k];
}

// Block-wide FP64 sum of K values: wavefront butterfly (64 lanes), then the
// wave partials in LDS. Result valid in thread 0.
template <int K>
__device__ inline void block_sum(double v[K], double out[K])
{
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    __shared__ double sm[BLOCK / 64][K];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < K; ++k) sm[wv][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < K; ++k) {
            double s = sm[0][k];
            for (int i = 1; i < BLOCK / 64; ++i) s += sm[i][k];
            out[k] = s;
        }
}

__device__ inline void block_sum5(double v[5], double out[5]) { block_sum<5>(v, out); }

constexpr int TOTAL_BLOCKS = 1024;

// Per-block partial sums of the node moments (fixed assignment of nodes to
// threads, so the result does not depend on timing).
// sat_check: flag a stored magnitude at the saturation value of the
// stochastic-rounding FP16 encoder (contexts with stochastic rounding).
template <class ST>
__global__ __launch_bounds__(BLOCK) void k_totals(const typename ST::T* __restrict__ f, uint32_t N, StepParams p,
                                                  double* __restrict__ partials, uint32_t sat_check = 0)
{
    double acc[5] = {0, 0, 0, 0, 0};
    for (uint32_t n = blockIdx.x * BLOCK + threadIdx.x; n < N; n += gridDim.x * BLOCK) {
        double m[5];
        node_moments64<ST>(f, p.g.qs, n, p, m);
        if constexpr (ST::SAT > 0.f) {
            if (sat_check) {
                bool sat = false;
                for (int q = 0; q < Q; ++q) sat |= !(fabsf(float(f[size_t(q) * p.g.qs + n])) < ST::SAT);
                if (sat) atomicOr(p.flag, 1u);
            }
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) acc[k] += m[k];
    }
    double r[5];
    block_sum<5>(acc, r);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) partials[blockIdx.x * 5 + k] = r[k];
}

template <int K>
__global__ __launch_bounds__(BLOCK) void k_reduce_partials(const double* __restrict__ partials, uint32_t nblk,
                                                           double* __restrict__ out)
{
    double acc[K];
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (uint32_t b = threadIdx.x; b < nblk; b += BLOCK)
        for (int k = 0; k < K; ++k) acc[k] += partials[b * K + k];
    double r[K];
    block_sum<K>(acc, r);
    if (threadIdx.x == 0)
        for (int k = 0; k < K; ++k) out[k] = r[k];
}

// Fourier amplitudes (1/N) sum_n m(n) e^{-i k.x_n} of rho, jx, jy, jz, E and
// theta = (2E/rho - u^2)/3 at the true node positions (sublattice 1 at
// +1/2 in every direction): per-block partial sums of 12 values.
constexpr int PROJ_FIELDS = 6;

template <class ST>
__global__ __launch_bounds__(BLOCK) void k_project(const typename ST::T* __restrict__ f, StepParams p, double kx,
                                                   double ky, double kz, double* __restrict__ partials)
{
    const uint32_t N = p.g.N;
    double acc[2 * PROJ_FIELDS];
    for (int k = 0; k < 2 * PROJ_FIELDS; ++k) acc[k] = 0.0;
    for (uint32_t n = blockIdx.x * BLOCK + threadIdx.x; n < N; n += gridDim.x * BLOCK) {
        double m[5];
        node_moments64<ST>(f, p.g.qs, n, p, m);
        const Coord c = decode(n, p.g);
        const double h = 0.5 * double(c.s);
        const double ph = kx * (double(c.x) + h) + ky * (double(c.y) + h) + kz * (double(c.z) + h);
        double sn, cs;
        sincos(ph, &sn, &cs);
        const double u2 = (m[1] * m[1] + m[2] * m[2] + m[3] * m[3]) / (m[0] * m[0]);
        const double th = (2.0 * m[4] / m[0] - u2) / 3.0;
        const double v[PROJ_FIELDS] = {m[0], m[1], m[2], m[3], m[4], th};
        for (int k = 0; k < PROJ_FIELDS; ++k) {
            acc[2 * k] += v[k] * cs;
            acc[2 * k + 1] -= v[k] * sn;
        }
    }
    double r[2 * PROJ_FIELDS];
    block_sum<2 * PROJ_FIELDS>(acc, r);
    if (threadIdx.x == 0)
        for (int k = 0; k < 2 * PROJ_FIELDS; ++k) partials[blockIdx.x * 2 * PROJ_FIELDS + k] = r[k];
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
    double v = double(ST::load(f + size_t(q) * p.g.qs + n));
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

// ---------------------------------------------------------------------------
// Plain copy of n 16-byte words: reads and writes in equal amounts, fully
// coalesced, no arithmetic. Its rate is what a streaming kernel reaches on
// the device, reported beside the step's own rate. One word per lane in
// 256-lane blocks measured fastest on gfx950 (6.2 TB/s read + write on
// 4 GiB, against 5.6-5.8 with two or four words per lane, 4.2 with eight,
// 5.1-5.4 with 512- and 1024-lane blocks, 5.9 with non-temporal hints).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_copy16(const uint4* __restrict__ in, uint4* __restrict__ out, uint64_t n)
{
    const uint64_t i = uint64_t(blockIdx.x) * BLOCK + threadIdx.x;
    if (i < n) out[i] = in[i];
}

}  // namespace lbm
