// RD3Q41 lattice constants for the device path (Sec. IV, Table I).
//
// Velocities are held in half units so that every component is an integer:
// c = (hx, hy, hz)/2. Order: rest, sc-1, sc-2, fcc-1, bcc-1, bcc-1/2 (Table I
// order), each shell in descending lexicographic order of (cx, cy, cz).
#pragma once

#include <cstdint>
#include <utility>

namespace lbm {

constexpr int Q = 41;

struct HalfVel {
    int x, y, z;  // twice the velocity components
    int shell;    // 0 rest, 1 sc-1, 2 sc-2, 3 fcc-1, 4 bcc-1, 5 bcc-1/2
};

constexpr HalfVel VEL[Q] = {
    {0, 0, 0, 0},
    // sc-1: (+-1, 0, 0) and permutations
    {2, 0, 0, 1}, {0, 2, 0, 1}, {0, 0, 2, 1}, {0, 0, -2, 1}, {0, -2, 0, 1}, {-2, 0, 0, 1},
    // sc-2: (+-2, 0, 0) and permutations
    {4, 0, 0, 2}, {0, 4, 0, 2}, {0, 0, 4, 2}, {0, 0, -4, 2}, {0, -4, 0, 2}, {-4, 0, 0, 2},
    // fcc-1: (+-1, +-1, 0) and permutations
    {2, 2, 0, 3}, {2, 0, 2, 3}, {2, 0, -2, 3}, {2, -2, 0, 3},
    {0, 2, 2, 3}, {0, 2, -2, 3}, {0, -2, 2, 3}, {0, -2, -2, 3},
    {-2, 2, 0, 3}, {-2, 0, 2, 3}, {-2, 0, -2, 3}, {-2, -2, 0, 3},
    // bcc-1: (+-1, +-1, +-1)
    {2, 2, 2, 4}, {2, 2, -2, 4}, {2, -2, 2, 4}, {2, -2, -2, 4},
    {-2, 2, 2, 4}, {-2, 2, -2, 4}, {-2, -2, 2, 4}, {-2, -2, -2, 4},
    // bcc-1/2: (+-1/2, +-1/2, +-1/2)
    {1, 1, 1, 5}, {1, 1, -1, 5}, {1, -1, 1, 5}, {1, -1, -1, 5},
    {-1, 1, 1, 5}, {-1, 1, -1, 5}, {-1, -1, 1, 5}, {-1, -1, -1, 5},
};

// Table I weights per moving shell; the rest weight is fixed by sum w = 1.
constexpr double W_SC1 = 0.04743040745116578;
constexpr double W_SC2 = 0.00165687664501576;
constexpr double W_FCC = 0.00651175327832464;
constexpr double W_BCC = 0.00454087801154440;
constexpr double W_HALF = 0.04917980624482672;
constexpr double W_REST = 1.0 - (6.0 * W_SC1 + 6.0 * W_SC2 + 12.0 * W_FCC + 8.0 * W_BCC + 8.0 * W_HALF);

constexpr double SHELL_W[6] = {W_REST, W_SC1, W_SC2, W_FCC, W_BCC, W_HALF};
// |c|^2 of each shell
constexpr double SHELL_C2[6] = {0.0, 1.0, 4.0, 2.0, 3.0, 0.75};

constexpr double weight(int q) { return SHELL_W[VEL[q].shell]; }

// Index of the velocity (c_x, -c_y, c_z).
constexpr int mirror_y_of(int q)
{
    for (int r = 0; r < Q; ++r)
        if (VEL[r].x == VEL[q].x && VEL[r].y == -VEL[q].y && VEL[r].z == VEL[q].z) return r;
    return -1;
}

// Index of the velocity -c_q.
constexpr int reverse_of(int q)
{
    for (int r = 0; r < Q; ++r)
        if (VEL[r].x == -VEL[q].x && VEL[r].y == -VEL[q].y && VEL[r].z == -VEL[q].z) return r;
    return -1;
}

// theta0 = sum_i w_i c_ix^2 (Sec. III: the second weight constraint defines
// the reference temperature; the paper leaves it as an unknown of the system).
constexpr double theta0_value()
{
    double s = 0.0;
    for (int q = 0; q < Q; ++q) s += weight(q) * (0.25 * VEL[q].x * VEL[q].x);
    return s;
}
constexpr double THETA0 = theta0_value();

// sum_i w_i and sum_i w_i c_i^2 (= 1 and 3 theta0 up to rounding)
constexpr double sum_w_value()
{
    double s = 0.0;
    for (int q = 0; q < Q; ++q) s += weight(q);
    return s;
}
constexpr double sum_wc2_value()
{
    double s = 0.0;
    for (int q = 0; q < Q; ++q) s += weight(q) * 0.25 * (VEL[q].x * VEL[q].x + VEL[q].y * VEL[q].y + VEL[q].z * VEL[q].z);
    return s;
}
constexpr double SUM_W = sum_w_value();
constexpr double SUM_WC2 = sum_wc2_value();

// Per-shell sums of the series equilibrium (Sec. V): sum_{i in shell}
// w_i c_i^4 and sum_{i in shell} w_i c_ix^2 c_iy^2.
constexpr double shell_sum_c4(int s)
{
    double a = 0.0;
    for (int q = 0; q < Q; ++q) {
        if (VEL[q].shell != s) continue;
        const double c2 = 0.25 * (VEL[q].x * VEL[q].x + VEL[q].y * VEL[q].y + VEL[q].z * VEL[q].z);
        a += weight(q) * c2 * c2;
    }
    return a;
}
constexpr double shell_sum_cxcy(int s)
{
    double a = 0.0;
    for (int q = 0; q < Q; ++q)
        if (VEL[q].shell == s) a += weight(q) * 0.0625 * (VEL[q].x * VEL[q].x) * (VEL[q].y * VEL[q].y);
    return a;
}
constexpr double SHELL_C4[6] = {shell_sum_c4(0), shell_sum_c4(1), shell_sum_c4(2),
                                shell_sum_c4(3), shell_sum_c4(4), shell_sum_c4(5)};
constexpr double SHELL_CXCY[6] = {shell_sum_cxcy(0), shell_sum_cxcy(1), shell_sum_cxcy(2),
                                  shell_sum_cxcy(3), shell_sum_cxcy(4), shell_sum_cxcy(5)};

// Power-of-two exponent per shell used by the shifted storage so that
// (f - w rho0) 2^k has magnitude ~ (relative deviation) 2^k_amp:
// k_shell = round(-log2 w_shell).
constexpr int SHELL_K[6] = {2, 4, 9, 7, 8, 4};

// Compile-time loop over q = 0..Q-1 (or any N): f(std::integral_constant<int, q>).
template <class F, int... Is>
__host__ __device__ inline void static_for_impl(F&& f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__host__ __device__ inline void static_for(F&& f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

}  // namespace lbm
