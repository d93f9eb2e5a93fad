/*
 * mtpt.h -- C-ABI of libmtpt.so: the per-time-step hot path of mass-transfer
 * particle tracking (MTPT) on one AMD Instinct MI355X (gfx950).
 *
 * The method (Schauer et al., arXiv 2204.03756, Sec. 3):
 *   1. random walk X_i += v dt + xi_i sqrt(2 D_RW dt), xi_i standard normal,
 *      with zero-flux walls as elastic reflection (the drift v dt is the
 *      advective term of the advection-dispersion equation, Sec. 2, which the
 *      paper's tests leave at zero; the jump is formed in FP64 as
 *      xi sqrt(2 D_RW dt) + v dt);
 *   2. neighbours within the search radius psi (Eq. (1));
 *   3. Gaussian weights K_ij = exp(-beta r_ij^2 / (4 D_MT dt)) (Eq. (2)-(3),
 *      the normalising prefactor cancels) and the symmetric normalisation
 *      W_ij = K_ij / (0.5 (s_i + s_j)), s_i = sum_k K_ik (self term included);
 *   4. explicit mass exchange M_i += beta sum_j W_ij (M_j - M_i) (Eq. (4)-(5)),
 *      every increment computed from the masses at time t.
 * An optional A+B->C reaction (three species) runs after the exchange.
 *
 * General rules for every function below:
 *   - Return MTPT_OK (0) or a negative MTPT_E_* code; mtpt_last_error() then
 *     holds a message (thread-local, valid until the next call on the thread).
 *   - Host pointers are plain host memory owned by the caller; the library
 *     copies inputs before returning and never keeps a host pointer.
 *   - All device memory is owned by the library and taken from the allocator
 *     passed at create (hipMalloc/hipFree when NULL).
 *   - Work is enqueued on the stream given at create (a new stream of default
 *     priority when NULL).  Only the functions marked "synchronises" wait.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Positions are exchanged as FP64 [n][dim], masses as FP64 [n_species][n],
 *     both in the caller's original particle order (pid = row index).
 *   - Determinism: the same params, inputs and seed give bit-identical
 *     results run to run, across a resume at start_step, and alone versus
 *     inside a pool.
 *   - Environment: MTPT_MIN_TILES (a whole number in [1, 2^20], default 256)
 *     is the fewest tiles a sim's mass-transfer passes are cut into, read at
 *     create and at admission; a sim whose throughput-sized tiles would be
 *     fewer gets smaller ones, so a small sim's step spreads over the chip.
 *     Positions, masses and pair counts do not depend on it; the FP64 totals
 *     only through the grouping of their partial sums.
 */
#ifndef MTPT_H
#define MTPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MTPT_ABI_VERSION 4

typedef struct mtpt_sim mtpt_sim;   /* opaque, library-owned */
typedef struct mtpt_pool mtpt_pool; /* opaque, library-owned */

enum {
    MTPT_OK = 0,
    MTPT_E_ARG = -1,       /* invalid argument or parameter */
    MTPT_E_NOMEM = -2,     /* device memory (or pool budget/slots) exhausted */
    MTPT_E_DEVICE = -3,    /* a HIP call failed; message has hipGetErrorString */
    MTPT_E_NONFINITE = -4, /* a mass total became NaN or infinite */
    MTPT_E_ABI = -5,       /* params.abi_version != MTPT_ABI_VERSION */
    MTPT_E_STATE = -6      /* call not valid in the object's current state */
};

/* Internal arithmetic.  FP64: positions, weights and masses in FP64.
 * FP32W_FP64ACC: positions and weights in FP32, masses and their increments
 * in FP64.  FP32_KAHAN: positions, weights and masses in FP32, each increment
 * summed with Kahan compensation.  In FP32 modes the input positions are
 * rounded to FP32 once at create and the walk runs in FP32; pairs whose FP32
 * squared distance lies within 1e-5 relative of psi^2 are re-tested in FP64,
 * so the neighbour sets equal those of an FP64 test on the FP32 positions. */
enum { MTPT_FP64 = 0, MTPT_FP32W_FP64ACC = 1, MTPT_FP32_KAHAN = 2 };

typedef struct {
    uint32_t abi_version; /* must be MTPT_ABI_VERSION */
    int32_t dim;          /* 2 or 3 */
    int64_t n;            /* particles, 0 <= n <= 2^31 - 256 */
    int32_t n_species;    /* 1, or 3 (A, B, C with the A+B->C reaction) */
    int32_t precision;    /* MTPT_FP64 / MTPT_FP32W_FP64ACC / MTPT_FP32_KAHAN */
    double lo[3], hi[3];  /* box [lo, hi]^dim, reflecting walls, hi > lo */
    double d_rw;          /* random-walk diffusivity, >= 0 (0 and vel = 0: static particles) */
    double d_mt;          /* mass-transfer diffusivity, > 0 */
    double dt;            /* time step, > 0 */
    double beta;          /* bandwidth/update coefficient, in (0, 1] */
    double psi;           /* search radius; <= 0 selects 3 sqrt(4 D_MT dt) */
    double k_react;       /* A+B->C rate constant (n_species == 3), >= 0 */
    uint64_t seed;        /* Philox key of the random walk */
    int64_t start_step;   /* index of the first step (resume), >= 0 */
    double vel[3];        /* drift velocity (advection), finite; 0 for pure dispersion */
    double disp[9];       /* shape tensor T of the dispersion, row-major [3][3]: D_RW = d_rw T,
                             D_MT = d_mt T; all zero for isotropic dispersion (T = I).
                             See the note below. */
} mtpt_params;

/* Dispersion tensor (Sec. 2: the advection-dispersion equation carries a
 * dispersion tensor D; Sec. 3, Eq. (2): the mass-transfer kernel written with
 * the tensor D_MT; the paper's runs take D = D I).  T must be symmetric and
 * positive definite in its leading dim x dim block (the rest is ignored).
 * With T = L L^T (Cholesky) and M = L^-1, everything runs in the caller's
 * frame and box:
 *   - jumps: X += v dt + sqrt(2 d_rw dt) L xi (covariance 2 dt D_RW);
 *   - kernel: K = exp(-beta q / (4 d_mt dt)) with the Mahalanobis distance
 *     q = dx^T T^-1 dx = |M dx|^2 (Eq. (2) prints D_MT in the exponent; its
 *     inverse is the dimensionally consistent reading);
 *   - cutoff: q <= psi^2, an ellipsoid, found through cells of side at least
 *     psi sqrt(T_kk) along axis k;
 *   - walls: the box's faces, mirrors as in the isotropic case.
 * L, M and q are formed in one fixed order (L00 = sqrt(T00), L10 = T10/L00,
 * L11 = sqrt(T11 - L10 L10), L20 = T20/L00, L21 = (T21 - L20 L10)/L11,
 * L22 = sqrt((T22 - L20 L20) - L21 L21); M by forward substitution;
 * y = M dx row by row in ascending column order, q = (y0 y0 + y1 y1) + y2 y2),
 * and with T = I they reduce to the isotropic forms bit for bit. */

typedef struct {
    void* (*alloc)(size_t bytes, void* ctx); /* returns device memory or NULL */
    void (*free)(void* ptr, void* ctx);
    void* ctx;
} mtpt_allocator;

typedef struct {
    int64_t steps_done;     /* steps taken since create */
    int64_t pairs_last;     /* ordered pairs i != j within psi at the last step */
    uint64_t pairs_total;   /* sum of pairs over all steps taken */
    double mass_total[3];   /* per-species FP64 mass totals after the last step */
    double mass_initial[3]; /* the same at create */
    double drift;           /* max |total - initial| / |initial| over the conserved
                               totals: each species, or A+C and B+C with A+B->C */
    int32_t nonfinite;      /* 1 if any total was ever NaN or infinite */
    int32_t n_cells;        /* cells of the binning grid (side >= psi) */
} mtpt_stats_t;

/* Create a simulation: the particle state of Sec. 3 (positions X_i and
 * masses M_i of N particles in the box, Sec. 2.1) and its parameters
 * (D_RW, D_MT, dt, beta, the search radius psi of Eq. (1)).
 * pos: host FP64 [n][dim], row-major, every coordinate within [lo, hi].
 * mass: host FP64 [n_species][n], species-major, finite.
 * hip_stream: a hipStream_t, or NULL for a library-owned stream.
 * alloc: device allocator, or NULL for hipMalloc/hipFree.
 * The library copies pos and mass (host staging, then device copies), bins
 * the particles into cells, computes the initial mass totals, and waits for
 * that work before returning; the sim owns all its device memory.
 * Errors: MTPT_E_ABI, MTPT_E_ARG (dim, n, species, precision, box, dt, d_mt,
 * d_rw, beta, k_react, vel or disp out of range, a position outside the box,
 * a non-finite mass), MTPT_E_NOMEM, MTPT_E_DEVICE.  *out is NULL on error. */
int mtpt_create(const mtpt_params* params, const double* pos, const double* mass,
                void* hip_stream, const mtpt_allocator* alloc, mtpt_sim** out);

/* Enqueue n_steps full steps of Sec. 3 on the sim's stream: the random walk
 * with reflecting walls, the neighbour search within psi (Eq. (1)), the
 * kernel weights and row sums (Eq. (2)-(3)), the symmetric normalisation
 * and the explicit mass exchange (Eq. (4)-(5)), the optional A+B->C
 * reaction, and the FP64 mass totals.  Returns without waiting; a later
 * synchronising call reports device errors.  n_steps >= 0, else
 * MTPT_E_ARG; MTPT_E_DEVICE if a launch fails. */
int mtpt_step(mtpt_sim* sim, int64_t n_steps);

/* Masses M_i after the last step (Eq. (5); with three species A, B, C after
 * the reaction), into the caller's host buffer out: FP64 [n_species][n] in
 * the original particle order.  Synchronises.  MTPT_E_NONFINITE (out still
 * written) if a mass total became NaN or infinite; MTPT_E_ARG for NULL. */
int mtpt_masses(mtpt_sim* sim, double* out);

/* Positions X_i after the last step's random walk (Sec. 3), into the
 * caller's host buffer out: FP64 [n][dim] in the original particle order
 * (FP32 state converted exactly in the FP32 modes).  Synchronises. */
int mtpt_positions(mtpt_sim* sim, double* out);

/* Counters and totals (see mtpt_stats_t): ordered pairs within psi per step
 * (Eq. (1)) and the FP64 mass totals, whose conservation follows from the
 * symmetry of W (Sec. 3).  Synchronises. */
int mtpt_stats(mtpt_sim* sim, mtpt_stats_t* out);

/* Neighbour sets at the current positions (Sec. 3, Eq. (1): r^2 <= psi^2,
 * inclusive, self included; the ellipsoid q <= psi^2 with a dispersion
 * tensor), found by a plain scan of the 3^d cells around each particle, as
 * CSR in original order with each row ascending: row_ptr[n+1] (host, always
 * written), col[nnz] (host) written only when nnz <= cap, *nnz_out = nnz.
 * Scratch device memory comes from the sim's allocator (MTPT_E_NOMEM).
 * Synchronises.  A debug/test export, not a step. */
int mtpt_neighbors(mtpt_sim* sim, int64_t* row_ptr, int64_t* col, int64_t cap, int64_t* nnz_out);

/* mtpt_neighbors for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result, with every byte of device scratch (row counts, scan
 * tiles, the device row offsets and columns) carved from one static array
 * of 64 MiB that each GPU the library runs on holds until the process ends.
 * It calls no hipMalloc, hipFree or allocator.  Sizes beyond the array are
 * rejected with MTPT_E_ARG: 16 n + 8 nnz bytes (plus scan padding) must fit,
 * checked before any device work for the rows and again, after row_ptr is
 * written, for the columns.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (other threads, other streams) race; the
 * call synchronises the sim's stream before it returns. */
int mtpt_neighbors_static(mtpt_sim* sim, int64_t* row_ptr, int64_t* col, int64_t cap, int64_t* nnz_out);

/* Neighbour sets exactly as a hot pass of the last step used them, in the
 * CSR format of mtpt_neighbors (pid order, rows ascending, self included):
 * which = 0: the row-sum pass (every candidate it found within the cutoff,
 * Sec. 3 Eq. (1), the sums s_i of the normalisation run over these);
 * which = 1: the transfer pass (every pair whose weight it applied, Eq. (5):
 * the neighbour bits the row-sum pass recorded, decoded over the same
 * (trimmed) candidate rows, or its own candidate loop where a wave has no
 * bits).  Re-runs that pass on the last step's state without storing
 * anything.  MTPT_E_STATE before the first step; MTPT_E_ARG for another
 * which.  Synchronises.  A debug/test export, not a step. */
int mtpt_step_neighbors(mtpt_sim* sim, int32_t which, int64_t* row_ptr, int64_t* col, int64_t cap,
                        int64_t* nnz_out);

/* Free the sim's device memory (and stream, if library-owned); the handle
 * is invalid afterwards.  NULL is a no-op.  Synchronises on the sim's
 * stream first. */
int mtpt_destroy(mtpt_sim* sim);

/* Message of the last error on this thread ("" if none). */
const char* mtpt_last_error(void);

/* MTPT_ABI_VERSION the library was built with. */
int mtpt_abi_version(void);

/* Per-phase device time (measurement, no passage of the paper): when
 * enabled, HIP events bracket every kernel the sim launches and their
 * durations are accumulated per phase.  names[k], ms[k] and launches[k],
 * k < min(*count, cap), receive the phase name (static string), total
 * milliseconds and launch count; any of the three may be NULL.
 * mtpt_phase_times synchronises and resets the accumulators. */
int mtpt_set_profiling(mtpt_sim* sim, int32_t on);
int mtpt_phase_times(mtpt_sim* sim, const char** names, double* ms, int64_t* launches,
                     int32_t cap, int32_t* count);

/* ---------------------------------------------------------------------
 * Serving (no passage of the paper: independent simulations of Sec. 3 run
 * side by side): a pool of simulations of any size and dimension, admitted
 * while device memory and slots allow, stepped together: one tick advances
 * every active sim by one step with one batched launch per phase.  Each
 * sim's result is bit-identical to the same sim run alone.
 * --------------------------------------------------------------------- */

/* hbm_budget: bytes of device memory the pool may hold (0: 90 % of free
 * memory at create).  max_slots: most sims active at once (>= 1, else
 * MTPT_E_ARG).  hip_stream and alloc as for mtpt_create. */
int mtpt_pool_create(size_t hbm_budget, int32_t max_slots, void* hip_stream,
                     const mtpt_allocator* alloc, mtpt_pool** out);

/* Admit a sim (params, pos and mass as for mtpt_create) that will run
 * n_steps (>= 1) steps; *ticket identifies it.  Its bytes are those of
 * mtpt_sim_bytes plus n_species * n * 8 of result staging.  pos and mass are
 * read before the call returns (into pinned staging owned by the pool); the
 * upload and the set-up binning are enqueued behind the ticks in flight and
 * the call does not wait for them (it waits only when all four staging
 * buffers still have copies in flight).  Returns MTPT_E_NOMEM when the slots
 * or the budget cannot hold it now (retry after a result has been
 * collected); other errors as mtpt_create (device errors of the enqueued
 * work surface at a later synchronising call). */
int mtpt_pool_admit(mtpt_pool* pool, const mtpt_params* params, const double* pos,
                    const double* mass, int64_t n_steps, int64_t* ticket);

/* Enqueue one step for every active sim that still has steps to take.
 * *n_completed receives the number of sims whose last step this tick was.
 * Returns without waiting. */
int mtpt_pool_tick(mtpt_pool* pool, int32_t* n_completed);

/* 1 in *done if the ticket's sim has taken all its steps on the device,
 * else 0 (a query of the event behind its last step: it does not wait).
 * MTPT_E_ARG for an unknown ticket. */
int mtpt_pool_done(mtpt_pool* pool, int64_t ticket, int32_t* done);

/* Counters and totals of an admitted sim (see mtpt_stats_t).  Synchronises:
 * for a finished sim only with its own last step (the copy runs on a second
 * stream of the pool), else with the pool's stream.  MTPT_E_ARG for an
 * unknown ticket. */
int mtpt_pool_stats(mtpt_pool* pool, int64_t ticket, mtpt_stats_t* out);

/* Copy a finished sim's masses (as mtpt_masses: host FP64 [n_species][n],
 * original order) into mass_out and free its slot and memory; the ticket is
 * invalid afterwards.  Synchronises with the sim's last step only (the
 * export runs on a second stream of the pool; the ticks of the other sims
 * keep running).  MTPT_E_STATE if its last step is not enqueued yet,
 * MTPT_E_ARG for an unknown ticket. */
int mtpt_pool_result(mtpt_pool* pool, int64_t ticket, double* mass_out);

/* Active sims, bytes held, budget (any pointer may be NULL). */
int mtpt_pool_usage(mtpt_pool* pool, int32_t* active, size_t* bytes_held, size_t* budget);

/* Bytes of device memory a sim with these params allocates at create (its
 * particle arrays, cell tables and scratch; for admission).  Errors as the
 * parameter checks of mtpt_create. */
int mtpt_sim_bytes(const mtpt_params* params, size_t* bytes);

/* Free every sim of the pool and the pool (synchronises first).  NULL is a
 * no-op. */
int mtpt_pool_destroy(mtpt_pool* pool);

#ifdef __cplusplus
}
#endif

#endif /* MTPT_H */
