/*
 * RD3Q41 energy-conserving lattice Boltzmann method: plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE. This is the slow, literal reference that the GPU
 * library is checked against. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it. It shares no code, header,
 * table or constant with the GPU library: the lattice below is enumerated
 * here from the shell definitions, and the equilibrium is solved with a
 * generic 5x5 Newton iteration over all 41 velocities (not the closed-form
 * shell partition function the GPU uses).
 *
 * Paper: P. K. Kolluru, M. Atif, M. Namburi, S. Ansumali, "Lattice Boltzmann
 * model for weakly compressible flows" (arXiv:1909.08406).
 *
 * Conventions (readings where the paper is silent):
 *  - Velocity order: rest, then the shells sc-1, sc-2, fcc-1, bcc-1, bcc-1/2
 *    in the order of Table I; inside a shell, descending lexicographic order
 *    on (cx, cy, cz).
 *  - Grid: nx*ny*nz cells of unit spacing, two nodes per cell (Sec. IV: two
 *    simple-cubic sublattices offset by half a spacing in each direction).
 *    Node (s, x, y, z) sits at (x + s/2, y + s/2, z + s/2), s in {0, 1}.
 *    Node id n = ((s*nz + z)*ny + y)*nx + x. Fully periodic.
 *  - Population arrays are [q][node] (41 blocks of N = 2*nx*ny*nz values).
 *  - Relaxation: f* = f + omega (f_eq - f), where omega is the paper's 2*beta
 *    (Sec. II, discrete BGK equation). The caller chooses omega.
 *  - Time step: collide every node, then push each post-collision value
 *    along its link (Sec. II, f_i(x + c_i dt, t + dt) = f_i + 2 beta (...)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 41

/* ------------------------------------------------------------------------ */
/* Lattice (Sec. IV, Table I)                                               */
/* ------------------------------------------------------------------------ */

/* Table I weights, per shell; shell 0 (rest) is fixed by normalisation. */
static const double TABLE_I_WEIGHT[6] = {
    0.0,                 /* rest: 1 - sum of the others (the paper does not print it) */
    0.04743040745116578, /* sc-1   (+-1, 0, 0) and permutations      */
    0.00165687664501576, /* sc-2   (+-2, 0, 0) and permutations      */
    0.00651175327832464, /* fcc-1  (+-1, +-1, 0) and permutations    */
    0.00454087801154440, /* bcc-1  (+-1, +-1, +-1)                   */
    0.04917980624482672, /* bcc-1/2 (+-1/2, +-1/2, +-1/2)            */
};

static double g_c[NQ][3];
static double g_w[NQ];
static int g_shell[NQ];
static double g_theta0;
static int g_ready = 0;

/* Shell of a velocity given in half units (hx, hy, hz), or -1 if none. */
static int shell_of(int hx, int hy, int hz)
{
    int a[3] = {abs(hx), abs(hy), abs(hz)};
    /* sort ascending */
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (a[j] < a[i]) { int t = a[i]; a[i] = a[j]; a[j] = t; }
    if (a[0] == 0 && a[1] == 0 && a[2] == 0) return 0;
    if (a[0] == 0 && a[1] == 0 && a[2] == 2) return 1; /* |c| = 1 on an axis  */
    if (a[0] == 0 && a[1] == 0 && a[2] == 4) return 2; /* |c| = 2 on an axis  */
    if (a[0] == 0 && a[1] == 2 && a[2] == 2) return 3; /* face diagonal        */
    if (a[0] == 2 && a[1] == 2 && a[2] == 2) return 4; /* body diagonal        */
    if (a[0] == 1 && a[1] == 1 && a[2] == 1) return 5; /* half body diagonal   */
    return -1;
}

static void lattice_build(void)
{
    if (g_ready) return;
    int q = 0;
    for (int s = 0; s < 6; ++s)
        for (int hx = 4; hx >= -4; --hx)
            for (int hy = 4; hy >= -4; --hy)
                for (int hz = 4; hz >= -4; --hz)
                    if (shell_of(hx, hy, hz) == s) {
                        g_c[q][0] = 0.5 * hx;
                        g_c[q][1] = 0.5 * hy;
                        g_c[q][2] = 0.5 * hz;
                        g_shell[q] = s;
                        ++q;
                    }
    /* q == 41 here: 1 + 6 + 6 + 12 + 8 + 8 */
    double moving = 0.0;
    for (int i = 0; i < NQ; ++i)
        if (g_shell[i] != 0) moving += TABLE_I_WEIGHT[g_shell[i]];
    for (int i = 0; i < NQ; ++i)
        g_w[i] = g_shell[i] == 0 ? 1.0 - moving : TABLE_I_WEIGHT[g_shell[i]];
    /* Reference temperature: second moment of the weights along one axis,
     * sum_i w_i c_ix^2 = theta0 (Sec. III, the seven weight constraints). */
    double th = 0.0;
    for (int i = 0; i < NQ; ++i) th += g_w[i] * g_c[i][0] * g_c[i][0];
    g_theta0 = th;
    g_ready = 1;
}

/* Velocities (41x3), weights (41) and theta0. Returns the number of velocities. */
int orc_lattice(double *c, double *w, double *theta0)
{
    lattice_build();
    for (int i = 0; i < NQ; ++i) {
        if (c) { c[3 * i] = g_c[i][0]; c[3 * i + 1] = g_c[i][1]; c[3 * i + 2] = g_c[i][2]; }
        if (w) w[i] = g_w[i];
    }
    if (theta0) *theta0 = g_theta0;
    return NQ;
}

/*
 * The seven weight constraints of Sec. III (the system that fixes the
 * weights and theta0), as relative residuals:
 *   sum w = 1, sum w cx^2 = theta0, sum w cx^4 = 3 theta0^2,
 *   sum w cx^2 cy^2 = theta0^2, sum w cx^4 c^2 = 21 theta0^3,
 *   sum w cx^2 c^4 = 35 theta0^3, sum w c^8 = 945 theta0^4.
 * The second holds by the definition of theta0 used here.
 */
void orc_constraint_residuals(double out[7])
{
    lattice_build();
    double s[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < NQ; ++i) {
        double cx = g_c[i][0], cy = g_c[i][1], cz = g_c[i][2];
        double c2 = cx * cx + cy * cy + cz * cz;
        s[0] += g_w[i];
        s[1] += g_w[i] * cx * cx;
        s[2] += g_w[i] * cx * cx * cx * cx;
        s[3] += g_w[i] * cx * cx * cy * cy;
        s[4] += g_w[i] * cx * cx * cx * cx * c2;
        s[5] += g_w[i] * cx * cx * c2 * c2;
        s[6] += g_w[i] * c2 * c2 * c2 * c2;
    }
    double t = g_theta0;
    out[0] = s[0] - 1.0;
    out[1] = s[1] / t - 1.0;
    out[2] = s[2] / (3.0 * t * t) - 1.0;
    out[3] = s[3] / (t * t) - 1.0;
    out[4] = s[4] / (21.0 * t * t * t) - 1.0;
    out[5] = s[5] / (35.0 * t * t * t) - 1.0;
    out[6] = s[6] / (945.0 * t * t * t * t) - 1.0;
}

/* ------------------------------------------------------------------------ */
/* Moments (Sec. II)                                                        */
/* ------------------------------------------------------------------------ */

/* rho = <f,1>, j = <f,c>, E = <f,c^2/2>; m = (rho, jx, jy, jz, E). */
void orc_node_moments(const double *f, double m[5])
{
    lattice_build();
    double r = 0, jx = 0, jy = 0, jz = 0, e = 0;
    for (int i = 0; i < NQ; ++i) {
        double cx = g_c[i][0], cy = g_c[i][1], cz = g_c[i][2];
        r += f[i];
        jx += f[i] * cx;
        jy += f[i] * cy;
        jz += f[i] * cz;
        e += f[i] * 0.5 * (cx * cx + cy * cy + cz * cz);
    }
    m[0] = r; m[1] = jx; m[2] = jy; m[3] = jz; m[4] = e;
}

/* Boltzmann H-function, Sec. V: H = sum f (log(f/w) - 1). */
double orc_entropy(const double *f)
{
    lattice_build();
    double h = 0.0;
    for (int i = 0; i < NQ; ++i) h += f[i] * (log(f[i] / g_w[i]) - 1.0);
    return h;
}

/* ------------------------------------------------------------------------ */
/* Exact entropic equilibrium E2 (Sec. V)                                   */
/* ------------------------------------------------------------------------ */

/* Solve A x = b (n x n, n <= 5, leading block of A) by Gaussian
 * elimination with partial pivoting. */
static int solve_n(int n, double A[5][5], double b[5], double x[5])
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i][k]) > fabs(A[p][k])) p = i;
        if (A[p][k] == 0.0) return -1;
        if (p != k) {
            for (int j = 0; j < n; ++j) { double t = A[k][j]; A[k][j] = A[p][j]; A[p][j] = t; }
            double t = b[k]; b[k] = b[p]; b[p] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double l = A[i][k] / A[k][k];
            for (int j = k; j < n; ++j) A[i][j] -= l * A[k][j];
            b[i] -= l * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < n; ++j) s -= A[i][j] * x[j];
        x[i] = s / A[i][i];
    }
    return 0;
}

/*
 * Residual of the multiplier system with rho factored out:
 *   F(lam) = sum_i w_i exp(-a - b.c_i - g c_i^2) (1, c_i, c_i^2)
 *            - (1, u, u^2 + 3 theta),
 * lam = (a, bx, by, bz, g) are the paper's (alpha, beta, gamma) for mass,
 * momentum and energy. With n = 4 only the first four constraints (mass and
 * momentum) are imposed and g stays as given (the isothermal equilibrium,
 * g = 0). Also fills the Jacobian J = dF/dlam when J != NULL.
 */
static double e2_residual(int n, const double lam[5], const double tgt[5], double F[5], double J[5][5])
{
    double phi[5];
    for (int k = 0; k < n; ++k) F[k] = -tgt[k];
    if (J) memset(J, 0, sizeof(double) * 25);
    for (int i = 0; i < NQ; ++i) {
        double cx = g_c[i][0], cy = g_c[i][1], cz = g_c[i][2];
        double c2 = cx * cx + cy * cy + cz * cz;
        double e = g_w[i] * exp(-lam[0] - lam[1] * cx - lam[2] * cy - lam[3] * cz - lam[4] * c2);
        phi[0] = 1.0; phi[1] = cx; phi[2] = cy; phi[3] = cz; phi[4] = c2;
        for (int k = 0; k < n; ++k) {
            F[k] += e * phi[k];
            if (J)
                for (int l = 0; l < n; ++l) J[k][l] -= e * phi[k] * phi[l];
        }
    }
    double r = 0.0;
    for (int k = 0; k < n; ++k) r = fmax(r, fabs(F[k]));
    return r;
}

/* Newton iteration from lam on the first n constraints; returns the final
 * max-norm residual. */
static double e2_newton(int n, double lam[5], const double tgt[5], int *iters)
{
    double F[5], J[5][5], d[5], mF[5];
    double r = e2_residual(n, lam, tgt, F, J);
    int it = 0;
    for (; it < 50 && r > 1e-15 && isfinite(r); ++it) {
        for (int k = 0; k < n; ++k) mF[k] = -F[k];
        if (solve_n(n, J, mF, d) != 0) break;
        for (int k = 0; k < n; ++k) lam[k] += d[k];
        double rn = e2_residual(n, lam, tgt, F, J);
        /* stop once rounding dominates: the residual no longer shrinks */
        if (!(rn < r) && r < 1e-12) { r = rn; ++it; break; }
        r = rn;
    }
    if (iters) *iters = it;
    return r;
}

/*
 * Equilibrium f_eq,i = rho w_i exp(-a - b.c_i - g c_i^2) that satisfies
 * <f_eq, {1, c, c^2}> = {rho, rho u, rho u^2 + 3 rho theta} (Sec. V, the
 * entropic equilibrium and its five-multiplier system). The multipliers are
 * found numerically, as the paper says is typical: Newton from the
 * Maxwellian guess b = -u/theta, g = 1/(2 theta) - 1/(2 theta0), and from
 * lam = 0 if that fails. Returns 0 on success, -1 if not converged.
 * lam_out (optional) receives (a, bx, by, bz, g); resid the residual.
 */
int orc_equilibrium(double rho, double ux, double uy, double uz, double theta,
                    double *feq, double *lam_out, double *resid, int *iters)
{
    lattice_build();
    double tgt[5] = {1.0, ux, uy, uz, ux * ux + uy * uy + uz * uz + 3.0 * theta};
    double lam[5];
    lam[1] = -ux / theta;
    lam[2] = -uy / theta;
    lam[3] = -uz / theta;
    lam[4] = 0.5 / theta - 0.5 / g_theta0;
    double z = 0.0;
    for (int i = 0; i < NQ; ++i) {
        double cx = g_c[i][0], cy = g_c[i][1], cz = g_c[i][2];
        z += g_w[i] * exp(-lam[1] * cx - lam[2] * cy - lam[3] * cz - lam[4] * (cx * cx + cy * cy + cz * cz));
    }
    lam[0] = log(z);
    double r = e2_newton(5, lam, tgt, iters);
    if (!(r <= 1e-13)) {
        for (int k = 0; k < 5; ++k) lam[k] = 0.0;
        r = e2_newton(5, lam, tgt, iters);
    }
    for (int i = 0; i < NQ; ++i) {
        double cx = g_c[i][0], cy = g_c[i][1], cz = g_c[i][2];
        double c2 = cx * cx + cy * cy + cz * cz;
        feq[i] = rho * g_w[i] * exp(-lam[0] - lam[1] * cx - lam[2] * cy - lam[3] * cz - lam[4] * c2);
    }
    if (lam_out) for (int k = 0; k < 5; ++k) lam_out[k] = lam[k];
    if (resid) *resid = r;
    return (r <= 1e-13) ? 0 : -1;
}

/*
 * Isothermal equilibrium (Sec. V: the usual construction, with mass and
 * momentum but not energy conserved; Sec. VI uses it for the isothermal
 * acoustic pulse): f_eq,i = rho w_i exp(-a - b.c_i), the minimiser of the
 * same H-function under the mass and momentum constraints alone, so that
 * g = 0 and the rest state is f = rho w at temperature theta0. Newton on
 * (a, bx, by, bz) from b = -u/theta0, then from lam = 0 if that fails.
 * Returns 0 on success, -1 if not converged.
 */
int orc_equilibrium_iso(double rho, double ux, double uy, double uz, double *feq, double *lam_out, double *resid,
                        int *iters)
{
    lattice_build();
    double tgt[5] = {1.0, ux, uy, uz, 0.0};
    double lam[5] = {0.0, -ux / g_theta0, -uy / g_theta0, -uz / g_theta0, 0.0};
    double z = 0.0;
    for (int i = 0; i < NQ; ++i)
        z += g_w[i] * exp(-lam[1] * g_c[i][0] - lam[2] * g_c[i][1] - lam[3] * g_c[i][2]);
    lam[0] = log(z);
    double r = e2_newton(4, lam, tgt, iters);
    if (!(r <= 1e-13)) {
        for (int k = 0; k < 5; ++k) lam[k] = 0.0;
        r = e2_newton(4, lam, tgt, iters);
    }
    for (int i = 0; i < NQ; ++i)
        feq[i] = rho * g_w[i] * exp(-lam[0] - lam[1] * g_c[i][0] - lam[2] * g_c[i][1] - lam[3] * g_c[i][2]);
    if (lam_out) for (int k = 0; k < 5; ++k) lam_out[k] = lam[k];
    if (resid) *resid = r;
    return (r <= 1e-13) ? 0 : -1;
}

/* ------------------------------------------------------------------------ */
/* Series equilibrium E1 (Sec. V), a cross-check of E2                      */
/* ------------------------------------------------------------------------ */

/*
 * Zero-velocity equilibrium to third order in eta = theta/theta0 - 1
 * (Sec. V, the series for f-tilde):
 *   f~_i = w_i rho [1 + eta/2 (c^2/t0 - 3) + eta^2/8 (c^4/t0^2 - 10 c^2/t0 + 15)
 *                   + eta^3/48 (c^6/t0^3 - 21 c^4/t0^2 + 105 c^2/t0 - 105)].
 */
void orc_series_rest(double rho, double eta, double *ft)
{
    lattice_build();
    double t0 = g_theta0;
    for (int i = 0; i < NQ; ++i) {
        double cx = g_c[i][0], cy = g_c[i][1], cz = g_c[i][2];
        double x = (cx * cx + cy * cy + cz * cz) / t0; /* c^2 / theta0 */
        double p1 = 0.5 * eta * (x - 3.0);
        double p2 = eta * eta / 8.0 * (x * x - 10.0 * x + 15.0);
        double p3 = eta * eta * eta / 48.0 * (x * x * x - 21.0 * x * x + 105.0 * x - 105.0);
        ft[i] = g_w[i] * rho * (1.0 + p1 + p2 + p3);
    }
}

/*
 * Error terms of the zero-velocity moments of f~ with respect to the
 * Maxwell-Boltzmann values (Sec. V, "error terms w.r.t. zero velocity
 * equilibrium moments"), read as
 *   sum f~ c^4          = 15 rho theta^2 (1 + M2),
 *   sum f~ cx^2 cy^2    =    rho theta^2 (1 + M2'),
 *   sum f~ c^6          = 105 rho theta^3 (1 + M3),
 *   sum f~ c^2 cx^2 cy^2 = 7 rho theta^3 (1 + M3'),
 * computed here from the lattice sums (m = M2, M2', M3, M3').
 */
void orc_series_errors(double eta, double m[4])
{
    lattice_build();
    double ft[NQ];
    orc_series_rest(1.0, eta, ft);
    double th = g_theta0 * (1.0 + eta);
    double s4 = 0, sxy = 0, s6 = 0, s2xy = 0;
    for (int i = 0; i < NQ; ++i) {
        double cx = g_c[i][0], cy = g_c[i][1], cz = g_c[i][2];
        double c2 = cx * cx + cy * cy + cz * cz;
        s4 += ft[i] * c2 * c2;
        sxy += ft[i] * cx * cx * cy * cy;
        s6 += ft[i] * c2 * c2 * c2;
        s2xy += ft[i] * c2 * cx * cx * cy * cy;
    }
    m[0] = s4 / (15.0 * th * th) - 1.0;
    m[1] = sxy / (th * th) - 1.0;
    m[2] = s6 / (105.0 * th * th * th) - 1.0;
    m[3] = s2xy / (7.0 * th * th * th) - 1.0;
}

/*
 * Series equilibrium to third order in velocity (Sec. V, f_eq as the
 * product of f~ and a cubic polynomial in u.c/theta with coefficients A1,
 * A2 built from M2 and M2'):
 *   A1 = (5/2) M2 / (1 + (5/2) M2),
 *   A2 = 5 A1 (1 - M2) - (3 + M2' - 5 M2).
 */
void orc_equilibrium_series(double rho, double ux, double uy, double uz, double theta, double *feq)
{
    lattice_build();
    double eta = theta / g_theta0 - 1.0;
    double m[4];
    orc_series_errors(eta, m);
    double M2 = m[0], M2p = m[1];
    double A1 = 2.5 * M2 / (1.0 + 2.5 * M2);
    double A2 = 5.0 * A1 * (1.0 - M2) - (3.0 + M2p - 5.0 * M2);
    double ft[NQ];
    orc_series_rest(rho, eta, ft);
    double u2 = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < NQ; ++i) {
        double cx = g_c[i][0], cy = g_c[i][1], cz = g_c[i][2];
        double c2 = cx * cx + cy * cy + cz * cz;
        double uc = (ux * cx + uy * cy + uz * cz) / theta; /* u.c / theta */
        double p = 1.0 + uc - u2 / (2.0 * theta) * (1.0 - A1) + 0.5 * uc * uc + uc * uc * uc / 6.0
                 - u2 * c2 / (6.0 * theta * theta) * A1
                 + u2 * uc / (6.0 * theta) * A2
                 - u2 * c2 * uc / (6.0 * theta * theta) * A1;
        feq[i] = ft[i] * p;
    }
}

/* ------------------------------------------------------------------------ */
/* Collision (Sec. II, discrete BGK)                                        */
/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* Entropic path length (Sec. IX.A and IX.D; H-function of Sec. V)          */
/* ------------------------------------------------------------------------ */

/*
 * Entropy change along the line through f and f_eq: with x_i = f_eq,i/f_i - 1
 * the state f + a (f_eq - f) has components f_i (1 + a x_i), and
 *   dH(a) = H(f + a (f_eq - f)) - H(f)
 *         = sum_i f_i (1 + a x_i) log(1 + a x_i) - a sum_i f_i x_i log(1 + x_i),
 * which follows from H = sum f (log(f/w) - 1) because f_eq - f carries no
 * mass, momentum or energy and log(f_eq/w) is a combination of 1, c and c^2
 * (Sec. V). The same expression with f_eq of the isothermal model holds with
 * 1 and c. p1 = sum_i f_i x_i log(1 + x_i) is passed in.
 */
static double path_dh(const double *f, const double *x, double p1, double a)
{
    double s = 0.0;
    for (int i = 0; i < NQ; ++i) {
        const double y = a * x[i];
        s += f[i] * ((1.0 + y) * log1p(y) - y);  /* - y: sum_i f_i x_i = 0 */
    }
    return s - a * p1;
}

/*
 * Path length alpha of the entropic step (Sec. IX.A: alpha = 2 is the
 * standard BGK step, the entropic method chooses alpha from the H theorem;
 * Sec. IX.D: computed from x_i = f_eq,i/f_i - 1). Reading: alpha is the
 * nontrivial root of dH(a) = 0, the mirror state f + alpha (f_eq - f) having
 * the entropy of f. dH is convex with dH(0) = 0 and its minimum at a = 1
 * (the equilibrium), so the root lies in (1, a_max), where a_max =
 * min_{x_i < 0} (-1/x_i) keeps the mirror state positive. The search is
 * limited to (1, a_cap], a_cap = (1 - 2^-10) a_max; if dH(a_cap) <= 0 the
 * path length is a_cap. f = f_eq gives alpha = 2 (also when rounding leaves
 * no x_i < 0, which in exact arithmetic means f = f_eq). Plain bisection.
 */
double orc_path_length(const double *f, const double *feq)
{
    double x[NQ], p1 = 0.0, xmin = 0.0;
    int any = 0;
    for (int i = 0; i < NQ; ++i) {
        x[i] = (feq[i] - f[i]) / f[i];
        p1 += f[i] * x[i] * log1p(x[i]);
        if (x[i] != 0.0) any = 1;
        if (x[i] < xmin) xmin = x[i];
    }
    /* f = f_eq: alpha = 2. Without a negative x_i, sum_i f_i x_i = 0 forces
     * every x_i to zero in exact arithmetic, so that case is f = f_eq up to
     * rounding, and takes the same value. */
    if (!any || !(xmin < 0.0)) return 2.0;
    const double acap = (-1.0 / xmin) * (1.0 - 1.0 / 1024.0);
    double lo = 1.0, hi = acap;
    if (!(path_dh(f, x, p1, hi) > 0.0)) return hi;
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (path_dh(f, x, p1, mid) > 0.0) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

/* dH(a) of the state f toward feq (as in orc_path_length), for tests. */
double orc_path_dh(const double *f, const double *feq, double a)
{
    double x[NQ], p1 = 0.0;
    for (int i = 0; i < NQ; ++i) {
        x[i] = (feq[i] - f[i]) / f[i];
        p1 += f[i] * x[i] * log1p(x[i]);
    }
    return path_dh(f, x, p1, a);
}

/* Equilibrium models (low two bits): 0 energy conserving (E2), 1 isothermal,
 * 2 series (E1); ORC_ENTROPIC adds the entropic path length (E2 and
 * isothermal only). */
#define ORC_ENTROPIC 4

/* f* = f + omega (f_eq - f) for one node (Sec. II), with the equilibrium of
 * the node's rho, u, theta (model 0, energy conserving, E2), of its rho, u
 * (model 1, isothermal) or the series equilibrium E1 of its rho, u, theta
 * (model 2). With ORC_ENTROPIC, f* = f + alpha (omega/2) (f_eq - f) with the
 * path length alpha of the node (Sec. IX.A: alpha beta with beta = omega/2). */
int orc_collide_node_model(const double *f, double omega, int model, double *out)
{
    double m[5], feq[NQ];
    const int entropic = (model & ORC_ENTROPIC) != 0;
    model &= 3;
    if (entropic && model == 2) return -2;
    orc_node_moments(f, m);
    double rho = m[0];
    double ux = m[1] / rho, uy = m[2] / rho, uz = m[3] / rho;
    int rc;
    if (model == 1) {
        rc = orc_equilibrium_iso(rho, ux, uy, uz, feq, NULL, NULL, NULL);
    } else if (model == 2) {
        double theta = (2.0 * m[4] / rho - (ux * ux + uy * uy + uz * uz)) / 3.0;
        orc_equilibrium_series(rho, ux, uy, uz, theta, feq);
        rc = 0;
    } else {
        /* E = (rho u^2 + 3 rho theta)/2 (Sec. II) */
        double theta = (2.0 * m[4] / rho - (ux * ux + uy * uy + uz * uz)) / 3.0;
        rc = orc_equilibrium(rho, ux, uy, uz, theta, feq, NULL, NULL, NULL);
    }
    const double om = entropic ? 0.5 * omega * orc_path_length(f, feq) : omega;
    for (int i = 0; i < NQ; ++i) out[i] = f[i] + om * (feq[i] - f[i]);
    return rc;
}

int orc_collide_node(const double *f, double omega, double *out)
{
    return orc_collide_node_model(f, omega, 0, out);
}

/* ------------------------------------------------------------------------ */
/* Grid, streaming maps and time stepping                                   */
/* ------------------------------------------------------------------------ */

static int64_t wrap(int64_t v, int64_t n)
{
    int64_t r = v % n;
    return r < 0 ? r + n : r;
}

static int64_t node_id(int64_t s, int64_t x, int64_t y, int64_t z, int64_t nx, int64_t ny, int64_t nz)
{
    return ((s * nz + z) * ny + y) * nx + x;
}

/*
 * Destination of the population that leaves node (s, x, y, z) along c_q.
 * Positions are doubled so that every coordinate is an integer: a node at
 * (x + s/2) has doubled coordinate 2x + s, and a move by c_q adds 2 c_q.
 * The arrival point lies on the sublattice given by its parity.
 */
static int64_t push_dest(int q, int64_t s, int64_t x, int64_t y, int64_t z, int64_t nx, int64_t ny, int64_t nz)
{
    int64_t X = 2 * x + s + (int64_t)lround(2.0 * g_c[q][0]);
    int64_t Y = 2 * y + s + (int64_t)lround(2.0 * g_c[q][1]);
    int64_t Z = 2 * z + s + (int64_t)lround(2.0 * g_c[q][2]);
    int64_t s2 = X & 1; /* X, Y and Z have equal parity on the bcc lattice */
    return node_id(s2, wrap((X - s2) / 2, nx), wrap((Y - s2) / 2, ny), wrap((Z - s2) / 2, nz), nx, ny, nz);
}

/* Same arithmetic for the source of the population arriving along c_q. */
static int64_t pull_src(int q, int64_t s, int64_t x, int64_t y, int64_t z, int64_t nx, int64_t ny, int64_t nz)
{
    int64_t X = 2 * x + s - (int64_t)lround(2.0 * g_c[q][0]);
    int64_t Y = 2 * y + s - (int64_t)lround(2.0 * g_c[q][1]);
    int64_t Z = 2 * z + s - (int64_t)lround(2.0 * g_c[q][2]);
    int64_t s2 = X & 1;
    return node_id(s2, wrap((X - s2) / 2, nx), wrap((Y - s2) / 2, ny), wrap((Z - s2) / 2, nz), nx, ny, nz);
}

/* src[q*N + n] = node whose population q arrives at node n in one step. */
void orc_pull_map(int nx, int ny, int nz, int64_t *src)
{
    lattice_build();
    int64_t N = 2LL * nx * ny * nz;
    for (int q = 0; q < NQ; ++q)
        for (int64_t n = 0; n < N; ++n) {
            int64_t x = n % nx, y = (n / nx) % ny, z = (n / ((int64_t)nx * ny)) % nz, s = n / ((int64_t)nx * ny * nz);
            src[q * N + n] = pull_src(q, s, x, y, z, nx, ny, nz);
        }
}

/* Sources of population q = 0..40 for a list of destination nodes:
 * src[i*41 + q] (sampled checks on grids too large for a full map). */
void orc_pull_src_nodes(int nx, int ny, int nz, const int64_t *nodes, int64_t count, int64_t *src)
{
    lattice_build();
    for (int64_t i = 0; i < count; ++i) {
        int64_t n = nodes[i];
        int64_t x = n % nx, y = (n / nx) % ny, z = (n / ((int64_t)nx * ny)) % nz, s = n / ((int64_t)nx * ny * nz);
        for (int q = 0; q < NQ; ++q) src[i * NQ + q] = pull_src(q, s, x, y, z, nx, ny, nz);
    }
}

/* dst[q*N + n] = node that population q leaving node n reaches in one step. */
void orc_push_map(int nx, int ny, int nz, int64_t *dst)
{
    lattice_build();
    int64_t N = 2LL * nx * ny * nz;
    for (int q = 0; q < NQ; ++q)
        for (int64_t n = 0; n < N; ++n) {
            int64_t x = n % nx, y = (n / nx) % ny, z = (n / ((int64_t)nx * ny)) % nz, s = n / ((int64_t)nx * ny * nz);
            dst[q * N + n] = push_dest(q, s, x, y, z, nx, ny, nz);
        }
}

/* Populations at equilibrium with the given fields (all [node], FP64);
 * model 0 E2, 1 isothermal (ignores theta), 2 series E1. */
int orc_init_model(int nx, int ny, int nz, const double *rho, const double *ux, const double *uy,
                   const double *uz, const double *theta, int model, double *f)
{
    lattice_build();
    int64_t N = 2LL * nx * ny * nz;
    int bad = 0;
    model &= 3; /* the initial state is the equilibrium; the path length plays no part */
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t n = 0; n < N; ++n) {
        double feq[NQ];
        int rc = 0;
        if (model == 1) rc = orc_equilibrium_iso(rho[n], ux[n], uy[n], uz[n], feq, NULL, NULL, NULL);
        else if (model == 2) orc_equilibrium_series(rho[n], ux[n], uy[n], uz[n], theta[n], feq);
        else rc = orc_equilibrium(rho[n], ux[n], uy[n], uz[n], theta[n], feq, NULL, NULL, NULL);
        if (rc != 0) bad = 1;
        for (int q = 0; q < NQ; ++q) f[q * N + n] = feq[q];
    }
    return bad ? -1 : 0;
}

int orc_init(int nx, int ny, int nz, const double *rho, const double *ux, const double *uy,
             const double *uz, const double *theta, double *f)
{
    return orc_init_model(nx, ny, nz, rho, ux, uy, uz, theta, 0, f);
}

/* Post-collision populations of every node, without streaming. */
int orc_collide_field_model(int nx, int ny, int nz, double omega, int model, const double *f, double *out)
{
    lattice_build();
    int64_t N = 2LL * nx * ny * nz;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t n = 0; n < N; ++n) {
        double a[NQ], b[NQ];
        for (int q = 0; q < NQ; ++q) a[q] = f[q * N + n];
        if (orc_collide_node_model(a, omega, model, b) != 0) bad = 1;
        for (int q = 0; q < NQ; ++q) out[q * N + n] = b[q];
    }
    return bad ? -1 : 0;
}

int orc_collide_field(int nx, int ny, int nz, double omega, const double *f, double *out)
{
    return orc_collide_field_model(nx, ny, nz, omega, 0, f, out);
}

/*
 * nsteps time steps: collide at every node, then push along the links.
 * f holds the state on entry and on exit; tmp is scratch of the same size.
 */
int orc_run_model(int nx, int ny, int nz, double omega, int model, double *f, double *tmp, int nsteps)
{
    lattice_build();
    int64_t N = 2LL * nx * ny * nz;
    int bad = 0;
    for (int t = 0; t < nsteps; ++t) {
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int64_t n = 0; n < N; ++n) {
            double a[NQ], b[NQ];
            int64_t x = n % nx, y = (n / nx) % ny, z = (n / ((int64_t)nx * ny)) % nz, s = n / ((int64_t)nx * ny * nz);
            for (int q = 0; q < NQ; ++q) a[q] = f[q * N + n];
            if (orc_collide_node_model(a, omega, model, b) != 0) bad = 1;
            for (int q = 0; q < NQ; ++q) tmp[q * N + push_dest(q, s, x, y, z, nx, ny, nz)] = b[q];
        }
        memcpy(f, tmp, sizeof(double) * (size_t)(NQ * N));
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Kinetic walls (Sec. VII.A: diffuse walls at fixed velocity and           */
/* temperature; reading of the multi-speed rule below)                      */
/* ------------------------------------------------------------------------ */

/*
 * Walls normal to y, a quarter cell outside the node layers: with the layer
 * index L = 2y + s (layer L at height L/2), the lower wall lies at -1/4 and
 * the upper one at ny - 1/4. Populations are pushed as in orc_run_model,
 * periodically in x and z. A post-collision population whose destination
 * layer L + 2 c_y lies beyond a wall is taken up by that wall, and the wall
 * gives the same mass back to the node it came from: the populations that
 * would arrive at that node from beyond the wall (the reverses of the ones
 * taken up) are set to sigma f_w,q, where f_w is the equilibrium of the
 * wall's velocity and temperature at unit density (the model's equilibrium)
 * and sigma = (mass taken up) / (sum of f_w,q over those populations): a
 * diffuse, mass-conserving reflection. A specular wall (kind 1; the inviscid
 * planar wall of Sec. VI.B) instead returns each population taken up as its
 * mirror image (c_x, -c_y, c_z) at the same node.
 * wall[8] = (ux, uy, uz, theta) of the lower wall, then of the upper wall;
 * kind[2] = 0 diffuse, 1 specular, for the lower and the upper wall.
 */
int orc_run_walls_kind(int nx, int ny, int nz, double omega, int model, const double *wall, const int *kind,
                       double *f, double *tmp, int nsteps)
{
    lattice_build();
    const int64_t N = 2LL * nx * ny * nz;
    double fw[2][NQ];
    int rev[NQ], mir[NQ];
    for (int w = 0; w < 2; ++w) {
        const double *p = wall + 4 * w;
        int rc = (model & 3) == 1 ? orc_equilibrium_iso(1.0, p[0], p[1], p[2], fw[w], NULL, NULL, NULL)
                                  : orc_equilibrium(1.0, p[0], p[1], p[2], p[3], fw[w], NULL, NULL, NULL);
        if (rc != 0 || (model & 3) == 2) return -2;
    }
    for (int q = 0; q < NQ; ++q)
        for (int r = 0; r < NQ; ++r)
        {
            if (g_c[r][0] == -g_c[q][0] && g_c[r][1] == -g_c[q][1] && g_c[r][2] == -g_c[q][2]) rev[q] = r;
            if (g_c[r][0] == g_c[q][0] && g_c[r][1] == -g_c[q][1] && g_c[r][2] == g_c[q][2]) mir[q] = r;
        }
    const int64_t top = 2LL * ny - 1; /* last layer */
    int bad = 0;
    for (int t = 0; t < nsteps; ++t) {
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int64_t n = 0; n < N; ++n) {
            double a[NQ], b[NQ];
            const int64_t x = n % nx, y = (n / nx) % ny, z = (n / ((int64_t)nx * ny)) % nz,
                          s = n / ((int64_t)nx * ny * nz);
            const int64_t L = 2 * y + s;
            for (int q = 0; q < NQ; ++q) a[q] = f[q * N + n];
            if (orc_collide_node_model(a, omega, model, b) != 0) bad = 1;
            double taken[2] = {0.0, 0.0}, norm[2] = {0.0, 0.0};
            int side[NQ];
            for (int q = 0; q < NQ; ++q) {
                const int64_t Ld = L + (int64_t)lround(2.0 * g_c[q][1]);
                side[q] = Ld < 0 ? 0 : Ld > top ? 1 : -1;
                if (side[q] < 0) {
                    tmp[q * N + push_dest(q, s, x, y, z, nx, ny, nz)] = b[q];
                } else {
                    taken[side[q]] += b[q];
                    norm[side[q]] += fw[side[q]][rev[q]];
                }
            }
            for (int q = 0; q < NQ; ++q)
                if (side[q] >= 0) {
                    const int w = side[q];
                    if (kind[w] == 1) tmp[mir[q] * N + n] = b[q];
                    else tmp[rev[q] * N + n] = taken[w] / norm[w] * fw[w][rev[q]];
                }
        }
        memcpy(f, tmp, sizeof(double) * (size_t)(NQ * N));
    }
    return bad ? -1 : 0;
}

int orc_run_walls(int nx, int ny, int nz, double omega, int model, const double *wall, double *f, double *tmp,
                  int nsteps)
{
    const int kind[2] = {0, 0};
    return orc_run_walls_kind(nx, ny, nz, omega, model, wall, kind, f, tmp, nsteps);
}

int orc_run(int nx, int ny, int nz, double omega, double *f, double *tmp, int nsteps)
{
    return orc_run_model(nx, ny, nz, omega, 0, f, tmp, nsteps);
}

/* Per-node rho, j, E fields. */
void orc_moment_fields(int64_t N, const double *f, double *rho, double *jx, double *jy, double *jz, double *en)
{
    lattice_build();
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double a[NQ], m[5];
        for (int q = 0; q < NQ; ++q) a[q] = f[q * N + n];
        orc_node_moments(a, m);
        rho[n] = m[0]; jx[n] = m[1]; jy[n] = m[2]; jz[n] = m[3]; en[n] = m[4];
    }
}

static double pairwise_sum(const double *v, int64_t n)
{
    if (n <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += v[i];
        return s;
    }
    int64_t h = n / 2;
    return pairwise_sum(v, h) + pairwise_sum(v + h, n - h);
}

/* Global mass, momentum and energy, pairwise-summed over the node fields. */
void orc_totals(int64_t N, const double *f, double out[5])
{
    double *m = (double *)malloc(sizeof(double) * (size_t)(5 * N));
    orc_moment_fields(N, f, m, m + N, m + 2 * N, m + 3 * N, m + 4 * N);
    for (int k = 0; k < 5; ++k) out[k] = pairwise_sum(m + k * N, N);
    free(m);
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
