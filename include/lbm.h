/*
 * liblbm: fused collide-and-stream update of the RD3Q41 energy-conserving
 * lattice Boltzmann method on one AMD Instinct MI355X (gfx950).
 *
 * Method: P. K. Kolluru, M. Atif, M. Namburi, S. Ansumali, "Lattice Boltzmann
 * model for weakly compressible flows" (arXiv:1909.08406).
 *   - State: 41 populations f_i per node (Sec. II), on the RD3Q41 velocity
 *     set of Table I (Sec. IV): rest, sc-1, sc-2, fcc-1, bcc-1, bcc-1/2.
 *   - Grid: a body-centred cubic lattice, i.e. two simple-cubic sublattices
 *     offset by half a spacing (Sec. IV). A box of nx*ny*nz cells has
 *     N = 2*nx*ny*nz nodes; node (s, x, y, z) sits at (x, y, z) + s/2*(1,1,1).
 *     Node id n = ((s*nz + z)*ny + y)*nx + x. All boxes are fully periodic.
 *   - Update: discrete BGK, f_i(x + c_i, t + 1) = f_i + omega (f_i^eq - f_i)
 *     (Sec. II; omega is the paper's 2*beta), with f^eq the exact entropic
 *     equilibrium w_i rho exp(-alpha - beta.c_i - gamma c_i^2) whose
 *     multipliers reproduce rho, rho u and rho u^2 + 3 rho theta (Sec. V).
 *     Mass, momentum and energy are conserved by every collision.
 *   - Observables: rho = <f,1>, j = <f,c>, E = <f,c^2/2> (Sec. II).
 *
 * Velocity order (shared by every array indexed by q): q = 0 rest, then the
 * shells in the order of Table I, each sorted in descending lexicographic
 * order of (cx, cy, cz). lbm_lattice() returns the table.
 *
 * Streaming is "pull": the populations held after a step are the
 * post-collision values at their node of origin, g = C[f]. Because the
 * collision conserves rho, j and E, the moments of g equal those of the
 * pre-collision state f of a collide-then-push description.
 *
 * Conventions for every entry point:
 *   - Host arrays are FP64, box after box; inside a box node fields are
 *     [s][z][y][x] (x fastest) and populations are [q][node].
 *   - The caller owns every host pointer and keeps it; the library copies
 *     what it needs before returning. Device memory is owned by the context
 *     (allocated by the library, or a caller-supplied workspace that must
 *     outlive the context).
 *   - Calls are asynchronous on the context stream unless stated otherwise.
 *   - Return value: LBM_OK (0) or a negative lbm_error. Nothing throws
 *     across this interface. lbm_strerror() is thread-safe. A context is
 *     not thread-safe: calls on one context must not overlap.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_Q 41

typedef enum {
    LBM_OK = 0,
    LBM_E_ARG = -1,         /* invalid argument (NULL pointer, bad size, tau <= 1/2, ...) */
    LBM_E_NOMEM = -2,       /* device or host allocation failed, or workspace too small */
    LBM_E_DOMAIN = -3,      /* unrealisable input: rho <= 0, theta <= 0 or non-finite field */
    LBM_E_NONFINITE = -4,   /* a step produced rho <= 0, theta <= 0 or a non-finite moment */
    LBM_E_HIP = -5,         /* a HIP runtime call failed */
    LBM_E_UNSUPPORTED = -6  /* valid request the library or device cannot serve */
} lbm_error;

/* How populations are held in device memory (arithmetic type in brackets). */
typedef enum {
    LBM_F64 = 0,        /* f in FP64                          [FP64] */
    LBM_F32 = 1,        /* f in FP32                          [FP32] */
    LBM_F16_SHIFT = 2,  /* FP16 of (f - w_q rho0) * 2^k_q     [FP32] */
    LBM_BF16_SHIFT = 3, /* BF16 of (f - w_q rho0) * 2^k_q     [FP32] */
    LBM_F32_SHIFT = 4   /* FP32 of (f - w_q rho0)              [FP32] */
} lbm_storage;

/* lbm_opts.flags */
#define LBM_FLAG_STOCHASTIC_ROUNDING 1u /* round stored values stochastically (unbiased):
                                           LBM_F32, LBM_F16_SHIFT, LBM_BF16_SHIFT only */
#define LBM_FLAG_ISOTHERMAL 2u          /* isothermal model (Sec. V, the usual construction
                                           without energy conservation; Sec. VI, isothermal
                                           acoustics): the same exponential equilibrium under
                                           the mass and momentum constraints only, i.e. no c^2
                                           multiplier and temperature theta0; sound speed
                                           sqrt(theta0). The theta field of lbm_init is
                                           checked but not used. Steps run the default
                                           launch shape (256 threads, no hints);
                                           lbm_tuning.variant is not used. */
#define LBM_FLAG_SERIES_EQUILIBRIUM 4u  /* the series equilibrium E1 (Sec. V): the zero-
                                           velocity series to third order in theta/theta0 - 1
                                           times the cubic velocity polynomial with A1, A2
                                           from the lattice's fourth-moment errors M2, M2';
                                           polynomial, no Newton solve. Mass and energy are
                                           conserved, momentum up to O(u eta^k) terms.
                                           Not with LBM_FLAG_ISOTHERMAL. Default launch
                                           shape, as for the isothermal model. */
#define LBM_FLAG_WALLS 16u              /* kinetic walls normal to y in every box (Sec. VII.A:
                                           walls of given velocity and temperature; the
                                           rule on this lattice is a reading): node layers
                                           L = 2y + s sit at height L/2 and the walls a
                                           quarter cell outside the first and last layer.
                                           A population that would come from beyond a wall
                                           is replaced: the wall returns to each node the
                                           mass that node sent through it in the previous
                                           step, re-emitted in the shape of the wall's
                                           equilibrium at unit density (diffuse, mass
                                           conserving). x and z stay periodic. Needs
                                           ny >= 2; with the energy-conserving or the
                                           isothermal equilibrium and optionally
                                           LBM_FLAG_ENTROPIC, not with
                                           LBM_FLAG_SERIES_EQUILIBRIUM
                                           (LBM_E_UNSUPPORTED). Walls start at rest at
                                           theta0; lbm_set_walls changes them. Default
                                           launch shape. */
#define LBM_FLAG_ENTROPIC 8u            /* entropic path length (Sec. IX.A: relaxation
                                           f + alpha beta (f_eq - f), beta = omega/2,
                                           alpha = 2 for BGK; Sec. IX.D: alpha from
                                           x_q = f_eq,q/f_q - 1; H of Sec. V): alpha per
                                           node is the nontrivial root of
                                           H(f + alpha (f_eq - f)) = H(f) in (1, a_cap],
                                           a_cap = (1 - 2^-10) min_{x_q<0} (-1/x_q) (the
                                           mirror state stays positive), a_cap when no root
                                           lies below it. With the energy-conserving or the
                                           isothermal equilibrium; not with
                                           LBM_FLAG_SERIES_EQUILIBRIUM. Default launch
                                           shape. */

/* Meaning of lbm_box.tau. */
typedef enum {
    LBM_TAU_LB = 0,     /* lattice relaxation time: omega = 1/tau, tau > 1/2           */
    LBM_TAU_PAPER = 1   /* the paper's mean free time (Sec. II): omega = 2/(2 tau + 1) */
} lbm_tau_conv;

/* One periodic box of nx*ny*nz cells (2 nodes per cell). */
typedef struct {
    int32_t nx, ny, nz;
    int32_t reserved;   /* must be 0 */
    double tau;         /* relaxation time, read per lbm_opts.tau_conv */
} lbm_box;

#define LBM_SHIFT_AUTO (-1000)

typedef struct {
    int32_t storage;      /* lbm_storage */
    int32_t tau_conv;     /* lbm_tau_conv */
    double rho0;          /* reference density of the shifted storage (0 means 1.0) */
    int32_t newton_iters; /* Newton steps of the equilibrium solve; 0 = default
                             (1 with FP32 arithmetic, 3 with FP64) */
    int32_t shift_exp;    /* k_amp of the shifted storage, k_q = k_shell(q) + k_amp;
                             LBM_SHIFT_AUTO picks it from the initial state */
    uint32_t flags;       /* LBM_FLAG_* */
    uint32_t seed;        /* seed of the stochastic rounding */
} lbm_opts;

/* Read-only facts about a context. */
typedef struct {
    int32_t storage;
    int32_t newton_iters;
    int32_t shift_exp;          /* k_amp in use (shifted storage), else 0 */
    int32_t nboxes;
    int64_t nodes;              /* total nodes over all boxes */
    int64_t bytes_per_step;     /* algorithmic HBM bytes of one step: 82 * nodes * sizeof(storage) */
    int32_t block_threads;      /* launch configuration of the step kernel */
    int32_t variant;            /* step-kernel variant id */
    uint64_t device_bytes;      /* device memory held by the context */
    uint32_t flags;             /* LBM_FLAG_* in effect */
    uint32_t steps_done;        /* step counter (seeds the stochastic rounding) */
} lbm_info;

typedef struct lbm_ctx lbm_ctx; /* opaque, owned by the library */

/*
 * Lattice constants of Table I (Sec. IV): velocities c[41][3], weights w[41]
 * (the rest weight is 1 - sum of the printed ones) and the reference
 * temperature theta0 = sum_i w_i c_ix^2 (Sec. III). Any pointer may be NULL.
 * No device needed.
 */
int lbm_lattice(double *c, double *w, double *theta0);

/*
 * Device bytes a context with these boxes and options needs (two population
 * buffers plus staging). No device needed. Errors: LBM_E_ARG.
 */
int lbm_workspace_size(const lbm_box *boxes, int32_t nboxes, const lbm_opts *opts, uint64_t *bytes);

/*
 * Create a context and set every node to the equilibrium of the given
 * fields, f = f^eq(rho, u, theta) (the fields are nodal FP64 arrays of the
 * total node count; theta in lattice units, e.g. theta0 for the rest
 * state). stream: a hipStream_t, or NULL for a stream the library creates.
 * workspace/workspace_bytes: device memory of at least lbm_workspace_size()
 * bytes for the context to use, or NULL/0 to let the library allocate it.
 * Synchronises the stream before returning.
 * Errors: LBM_E_ARG (NULL pointer, nboxes < 1, dimension < 1, tau out of
 * range, unknown storage, a q-block over 4 GiB), LBM_E_DOMAIN (rho <= 0,
 * theta <= 0 or non-finite), LBM_E_NOMEM, LBM_E_HIP.
 */
int lbm_init(lbm_ctx **out, const lbm_box *boxes, int32_t nboxes, const lbm_opts *opts,
             const double *rho, const double *ux, const double *uy, const double *uz,
             const double *theta, void *stream, void *workspace, uint64_t workspace_bytes);

/*
 * As lbm_init, with the five field arrays in device memory (FP64, all boxes
 * concatenated, the same layout): the equilibrium is built from them in
 * place, with no host copy. The caller keeps them alive until the call
 * returns. Unrealisable values (rho <= 0, theta <= 0, non-finite) are found
 * on the device and reported as LBM_E_DOMAIN. Errors as lbm_init.
 */
int lbm_init_device(lbm_ctx **out, const lbm_box *boxes, int32_t nboxes, const lbm_opts *opts,
                    const double *rho, const double *ux, const double *uy, const double *uz,
                    const double *theta, void *stream, void *workspace, uint64_t workspace_bytes);

/*
 * n >= 0 fused collide-and-stream steps of every box (Sec. II), queued on
 * the context stream without a host synchronisation. A step is one launch
 * per box or one launch over all boxes, optionally replayed from captured
 * graphs (see lbm_tuning); results do not depend on the choice.
 */
int lbm_step(lbm_ctx *ctx, int32_t n);

/*
 * n >= 0 collisionless streaming steps (free flight): every population moves
 * along its link unchanged, i.e. the update of Sec. II without the collision
 * term (the free-molecular limit). The held values are permuted exactly
 * (no rounding, any storage form), and mass, momentum and energy are kept.
 * It runs the step kernel's pull addressing, loads and stores in the
 * context's launch variant and tile mapping, so its rate is the ceiling of
 * the step's memory access pattern. Queued on the context stream; the
 * stochastic-rounding step counter is not advanced. Periodic boxes only:
 * LBM_E_UNSUPPORTED with LBM_FLAG_WALLS. Errors: LBM_E_ARG, LBM_E_HIP.
 */
int lbm_stream_free(lbm_ctx *ctx, int32_t n);

/*
 * Measurement helper, outside the method: copies `bytes` bytes from the
 * device pointer src to the device pointer dst with the library's plain
 * copy kernel (16-byte words, fully coalesced, no arithmetic). Its rate,
 * bytes read plus bytes written over the kernel's time, is what a
 * streaming kernel reaches on the device; the step's rate is reported
 * beside it and beside the published HBM peak. bytes: a multiple of 16
 * (0 does nothing); src and dst 16-byte aligned, not overlapping, both
 * owned by the caller. Queued on `stream` (a hipStream_t, NULL for the
 * null stream) without synchronising.
 * Errors: LBM_E_ARG (null or misaligned pointers, a size not a multiple of
 * 16 or above (2^31 - 1) x 4096, overlapping ranges), LBM_E_HIP.
 */
int lbm_device_copy(const void *src, void *dst, uint64_t bytes, void *stream);

/* Wait for all work queued on the context stream. */
int lbm_synchronize(lbm_ctx *ctx);

/*
 * Per-node FP64 moments rho, jx, jy, jz, E (arrays of the total node count;
 * any may be NULL). Synchronous. Errors: LBM_E_ARG, LBM_E_HIP.
 */
int lbm_moments(lbm_ctx *ctx, double *rho, double *jx, double *jy, double *jz, double *energy);

/*
 * Global conservation totals per box, summed in FP64 on the device:
 * out[5*b + k] = (mass, Jx, Jy, Jz, E)[k] of box b. Synchronous.
 * Returns LBM_E_NONFINITE if any step since init flagged a node with
 * rho <= 0, theta <= 0 or a non-finite moment (out is still written).
 */
int lbm_totals(lbm_ctx *ctx, double *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * conservation totals of lbm_totals for one box whose populations the
 * caller holds in device memory, with no context and no allocation.
 * f: device pointer to the box's first q-block, populations [q][node] in
 * the storage form `storage` (lbm_storage), consecutive q-blocks `qstride`
 * elements apart (qstride >= 2*nx*ny*nz; nodes ordered as in every host
 * array); box: its dimensions (tau unused). Shifted forms hold
 * (f - w_q rho0) 2^{k_q} with k_q = round(-log2 w_q) + shift_exp for
 * LBM_F16_SHIFT and LBM_BF16_SHIFT (shift_exp as reported by lbm_get_info)
 * and k_q = 0 for LBM_F32_SHIFT; rho0 = 0 means 1.0. out: device pointer to
 * 5 doubles, (mass, Jx, Jy, Jz, E) summed in FP64 as lbm_totals does (the
 * same result bit for bit). Queued on `stream` (a hipStream_t, NULL for the
 * null stream) without synchronising.
 * The per-block partial sums live in a fixed device array of the library
 * (1024 x 5 doubles, one per device, kept until the process ends); calls
 * that overlap on one device race on it. Largest input: fewer than 2^32
 * nodes and a q-stride below 2^32 elements (else LBM_E_ARG).
 * Errors: LBM_E_ARG, LBM_E_HIP, LBM_E_UNSUPPORTED (device index >= 64).
 */
int lbm_totals_noalloc(const void *f, int32_t storage, const lbm_box *box, uint64_t qstride, double rho0,
                       int32_t shift_exp, void *stream, double *out);

/*
 * Fourier amplitudes of the node fields of one box at wavevector k[3]
 * (radians per cell spacing): out[2f] + i out[2f+1] = (1/N) sum_n m_f(n)
 * exp(-i k.x_n) for m_f = rho, jx, jy, jz, E, theta (f = 0..5), with x_n the
 * node position (sublattice 1 offset by half a cell in every direction) and
 * theta = (2E/rho - u^2)/3 (Sec. II). Summed in FP64 on the device, without
 * copying fields to the host. Synchronous. Errors: LBM_E_ARG.
 */
int lbm_project(lbm_ctx *ctx, int32_t box, const double *k, double *out);

/* LBM_OK, or LBM_E_NONFINITE once a step has flagged a node. Synchronous. */
int lbm_status(lbm_ctx *ctx);

/*
 * Copy the held populations to the host as FP64, f[box][q][node] (shifted
 * storage decoded as w_q rho0 + h 2^-k_q, exactly). Synchronous.
 */
int lbm_get_populations(lbm_ctx *ctx, double *f);

/* Overwrite the held populations from FP64 host values (rounded to the
 * storage type, round-to-nearest-even). Synchronous. */
int lbm_set_populations(lbm_ctx *ctx, const double *f);

/*
 * Held populations at selected entries of one box: out[i] = f[q][node] for
 * idx[i] = q*N_box + node, decoded to FP64. Synchronous.
 * Errors: LBM_E_ARG for an index outside [0, 41*N_box).
 */
int lbm_gather(lbm_ctx *ctx, int32_t box, const int64_t *idx, int64_t count, double *out);

/*
 * Streaming map of one box as the step kernel computes it: src[q*N + n] is
 * the node whose population q the step pulls into node n. Synchronous.
 */
int lbm_debug_pull_map(lbm_ctx *ctx, int32_t box, int64_t *src);

/* Set the step counter that seeds the stochastic rounding (restore it with
 * the populations to resume a run bit for bit). */
int lbm_set_step_counter(lbm_ctx *ctx, uint32_t steps_done);

/* Facts about the context (see lbm_info). */
int lbm_get_info(lbm_ctx *ctx, lbm_info *info);

/* How a step is launched over the boxes of a context. */
typedef enum {
    LBM_SCHEDULE_PER_BOX = 0, /* one launch per box (default for one box) */
    LBM_SCHEDULE_BATCHED = 1  /* one launch over every (box, tile) pair (default for several boxes) */
} lbm_schedule;

/* Largest graph_steps of lbm_tuning. */
#define LBM_GRAPH_STEPS_MAX 1024

/*
 * Launch configuration of the step kernel. Every choice computes the same
 * per-node arithmetic, so results are identical across choices.
 * graph_steps: 0 launches every step from the host; an even value in
 * [2, LBM_GRAPH_STEPS_MAX] makes lbm_step capture that many steps once as a
 * hipGraph (per starting buffer) and replay it, leaving the remainder of n
 * to eager launches. A graph holds no memset node; the stochastic-rounding
 * step count of a replay is a device counter set by a one-thread kernel
 * before each replay.
 */
typedef struct {
    int32_t variant;     /* 0 .. lbm_num_variants()-1 (block size, cache hints) */
    int32_t xcd_remap;   /* 1: consecutive tiles on one XCD (L2 domain); 0: dispatch order */
    int32_t schedule;    /* lbm_schedule */
    int32_t graph_steps; /* 0, or even in [2, LBM_GRAPH_STEPS_MAX] */
} lbm_tuning;

/* Number of step-kernel variants. No device needed. */
int lbm_num_variants(void);

/* Block size and hint flags of a variant: 1 non-temporal loads, 2
 * non-temporal stores, 4 source rows staged in LDS (16-bit storage, per-box
 * launches of boxes whose nx is a multiple of the block size; elsewhere the
 * variant runs the plain kernel of its block size). No device needed.
 * Errors: LBM_E_ARG. */
int lbm_variant_desc(int32_t variant, int32_t *block_threads, uint32_t *flags);

/* Select / read the launch configuration of a context. */
int lbm_set_tuning(lbm_ctx *ctx, const lbm_tuning *t);
int lbm_get_tuning(lbm_ctx *ctx, lbm_tuning *t);

/*
 * Time every (variant, xcd_remap) pair with `reps` steps each on the
 * context's own boxes (with its current schedule), in three interleaved
 * rounds, and keep the pair whose fastest round is fastest. The held state
 * is unchanged (each timed launch reads the current buffer and writes the
 * other one). ms (optional) receives 2*lbm_num_variants() step times (the
 * fastest round's mean), index 2*variant + xcd_remap; best (optional) the
 * choice. Synchronous.
 */
int lbm_autotune(lbm_ctx *ctx, int32_t reps, float *ms, lbm_tuning *best);

/* lbm_autotune_ex flags */
#define LBM_TUNE_SCHEDULE 1u /* also choose the schedule (contexts with several boxes) */
#define LBM_TUNE_GRAPH 2u    /* also choose graph_steps among 0 (eager), 16 and 64 */
#define LBM_TUNE_CACHE 4u    /* take the choice from the tuning cache when it holds the context's key,
                                and record a new choice there */

/* Outcome of lbm_autotune_ex. */
typedef struct {
    lbm_tuning best;    /* the configuration now in use by the context */
    float best_ms;      /* its measured mean time per step (0 when taken from the cache) */
    int32_t from_cache; /* 1 when the choice came from the cache and nothing was timed */
    int32_t timed;      /* number of configurations timed (each in three rounds) */
} lbm_tune_result;

/*
 * Autotuner with a wider search and a cache (the tile shape, cache hints
 * and tile-to-XCD mapping of the step kernel, then optionally the schedule
 * and the graph length). Every (variant, xcd_remap) pair is timed with the
 * context's schedule and eager launches as in lbm_autotune; with
 * LBM_TUNE_SCHEDULE the two schedules, then with LBM_TUNE_GRAPH eager
 * launches against replays of captured 16- and 64-step graphs, are timed
 * with the chosen pair. Within 0.5% of the fastest, the configuration with
 * the XCD remap on (no HBM traffic beyond the algorithmic bytes), the
 * current schedule and eager launches are preferred. Timed launches never
 * change the held state. The choice is applied to the context.
 * With LBM_TUNE_CACHE the choice is looked up first under the context's
 * key (device architecture, storage, model and rounding flags, Newton
 * steps, the search flags and the box shapes), and a new choice is stored
 * under it; a hit times nothing. ms (optional) receives the
 * 2*lbm_num_variants() variant/remap times as in lbm_autotune (zeros for a
 * cache hit and for variants that a model does not use); res (optional)
 * the outcome. Synchronous. Errors: LBM_E_ARG (reps < 1, unknown flag),
 * LBM_E_HIP.
 */
int lbm_autotune_ex(lbm_ctx *ctx, int32_t reps, uint32_t flags, float *ms, lbm_tune_result *res);

/*
 * Back the tuning cache with a text file (one line per key: key, variant,
 * xcd_remap, schedule, graph_steps): its entries are loaded now (malformed
 * lines are skipped; the file is created if missing) and every new choice is
 * appended. NULL: keep the cache in this process only. The cache is shared
 * by every context of the process and thread-safe.
 * Errors: LBM_E_ARG (file cannot be opened). No device needed.
 */
int lbm_tune_cache_file(const char *path);

/* Forget every cached choice held in this process (a backing file is kept). */
int lbm_tune_cache_clear(void);

/* Number of choices held in the tuning cache of this process. */
int lbm_tune_cache_count(void);

/* The hipStream_t the context queues its work on. */
void *lbm_stream(lbm_ctx *ctx);

/* Release device memory the library allocated and the context itself. */
void lbm_free(lbm_ctx *ctx);

/* Static description of an error code. */
const char *lbm_strerror(int code);

/*
 * Velocity and temperature of the two kinetic walls of one box of a context
 * made with LBM_FLAG_WALLS (Sec. VII.A: a stationary wall and a moving wall
 * held at different temperatures). wall[8] = (ux, uy, uz, theta) of the
 * lower wall (below layer 0), then of the upper wall; theta absolute (not
 * used by the isothermal model, whose walls are at theta0). A wall-normal
 * velocity is accepted and enters only through the wall's equilibrium. The
 * wall equilibria are computed in FP64 on the host and copied to the
 * context's workspace, ordered after the steps already enqueued; the call
 * synchronises the context stream. Both walls are made diffuse
 * (lbm_set_walls_kind below chooses). Errors: LBM_E_ARG (no walls, bad box),
 * LBM_E_DOMAIN (non-finite values, theta <= 0), LBM_E_HIP.
 */
int lbm_set_walls(lbm_ctx *ctx, int32_t box, const double *wall);

/* Kinds of kinetic wall. */
#define LBM_WALL_DIFFUSE 0   /* re-emission in the shape of the wall's equilibrium (Sec. VII.A) */
#define LBM_WALL_SPECULAR 1  /* each population taken up returns as its mirror image (c_x, -c_y, c_z)
                                at the same node: the inviscid planar wall of Sec. VI.B; keeps mass,
                                energy and the momentum along the wall; the wall's velocity and
                                temperature play no part */

/*
 * As lbm_set_walls, with the kind of each wall: kind[2] = kind of the lower
 * and of the upper wall (LBM_WALL_DIFFUSE or LBM_WALL_SPECULAR; wall[8] is
 * checked in both cases). Errors as lbm_set_walls; LBM_E_ARG for an unknown
 * kind.
 */
int lbm_set_walls_kind(lbm_ctx *ctx, int32_t box, const double *wall, const int32_t *kind);

/*
 * Host-only self test of the library's integer helpers (division by
 * invariant integers used for node decoding). Returns LBM_OK or LBM_E_ARG.
 * No device needed.
 */
int lbm_selftest(void);

/*
 * The step kernel's per-node collision (Sec. II with the equilibrium of
 * Sec. V), run on the host with the same arithmetic in FP64 (precision 0)
 * or FP32 (precision 1) and `newton` Newton steps: f_out = C[f_in] for one
 * node's 41 populations (direct storage; inputs rounded to the precision).
 * flags: 0, LBM_FLAG_ISOTHERMAL or LBM_FLAG_SERIES_EQUILIBRIUM for the
 * isothermal or the series equilibrium, plus LBM_FLAG_ENTROPIC for the
 * entropic path length (not with the series equilibrium).
 * For testing the arithmetic without a device. Errors: LBM_E_ARG.
 */
int lbm_collide_host(int32_t precision, int32_t newton, uint32_t flags, double omega, const double *f_in,
                     double *f_out);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
