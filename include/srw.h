/*
 * srw.h -- C ABI of libsrw.so: random-walk incomplete LDL^T preconditioning of
 * R-matrices and preconditioned conjugate gradient on one AMD Instinct MI355X
 * (gfx950).
 *
 * Method: H. Qian and S. S. Sapatnekar, "Stochastic Preconditioning for Iterative
 * Linear Equation Solvers".  An R-matrix (Section 1) is symmetric, has a positive
 * diagonal, non-positive off-diagonal entries and is irreducibly diagonally
 * dominant.  The preconditioner is built from random walks on the matrix graph
 * (Sections 2-3, 5.2) and applied inside PCG (Algorithm 1).
 *
 * Conventions shared by every entry point
 *   - Pointers marked "device" are HIP device pointers; "host" are host pointers.
 *     The caller owns every buffer it passes; the library owns an srw_factor from
 *     srw_build_factor until srw_factor_free.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on it;
 *     entry points that return host values (iteration counts, sizes, status found on
 *     the device) synchronise that stream before returning.
 *   - Every entry point returns an SRW_* status; no exception crosses the ABI.  On
 *     an error, outputs are unspecified and no srw_factor is returned.
 *   - Node labels are the caller's row indices 0..n-1 throughout.
 */
#ifndef SRW_H
#define SRW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------- */
#define SRW_OK 0
#define SRW_NOT_CONVERGED 1   /* PCG hit max_iter; x holds the last iterate        */
#define SRW_E_ARG (-1)        /* malformed arguments or CSR structure               */
#define SRW_E_NOT_RMATRIX (-2) /* values violate the R-matrix definition            */
#define SRW_E_SINGULAR (-3)   /* a connected component has no path to ground        */
#define SRW_E_WALK_LIMIT (-4) /* a walk exceeded srw_options.max_steps              */
#define SRW_E_NOMEM (-5)      /* device allocation failed                           */
#define SRW_E_HIP (-6)        /* a HIP runtime call failed                          */

#define SRW_ORDER_RANDOM 0    /* seeded random ordering (Section 5.4)               */
#define SRW_ORDER_GIVEN 1     /* caller-supplied ranks                              */

#define SRW_FP64 0            /* factor values and triangular solves in FP64        */
#define SRW_FP32 1            /* factor stored and solved in FP32 under FP64 PCG    */

/* ---- inputs ------------------------------------------------------------------ */

/* Square sparse matrix in CSR form, all arrays on the device.
 *   rowptr: int64[n+1], rowptr[0] = 0, rowptr[n] = nnz, non-decreasing;
 *   col:    int32[nnz], strictly increasing within each row, in [0, n);
 *   val:    float64[nnz].
 * Every row stores its diagonal exactly once; stored off-diagonal entries must be
 * strictly negative (a structural zero is not stored).  The matrix must be
 * symmetric with bitwise-equal mirrored values.  Limits: n < 2^31, nnz - n < 2^32. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int64_t* rowptr;
    const int32_t* col;
    const double* val;
} srw_csr;

/* Build options; srw_default_options() fills the defaults shown. */
typedef struct {
    int32_t ordering;          /* SRW_ORDER_RANDOM                                  */
    const int32_t* rank;       /* device int32[n], a permutation of 0..n-1, read
                                  when ordering == SRW_ORDER_GIVEN; rank 0 first     */
    const int32_t* walks;      /* device int32[n] per-row walk budgets, or NULL for
                                  the uniform walks_per_row; values < 1 count as 1  */
    int32_t factor_precision;  /* SRW_FP64                                          */
    uint64_t max_steps;        /* per-walk step cap, 0 = 2^22; exceeding it fails
                                  the build with SRW_E_WALK_LIMIT                    */
    int32_t keep;              /* 0 = keep only the factor; 1 = also keep the
                                  transition table and per-row tallies; 2 = also keep
                                  the per-walk records (for export / inspection)    */
    int32_t refill_period;     /* walk scheduling: idle lanes take new walks every
                                  this many steps (1, 2, 4 or 8); 0 = 8, which keeps
                                  every lane on the same random-number block phase  */
    int32_t profile;           /* 1 = time the build phases with HIP events on the
                                  build stream (see srw_factor_stats); 0 = off      */
    int32_t schedule;          /* walk order: 0 = all rows by rank (longest walks
                                  first); 1 (default) = rows ranked below n/256 by
                                  rank, then the rest in node-id slabs, one per XCD */
    int32_t solve_order;       /* order in which the triangular solves take rows:
                                  0 = rank; 1 (default) = dependency level, then rank
                                  (the build computes the levels once)              */
} srw_options;

void srw_default_options(srw_options* opt);

/* ---- the preconditioner ------------------------------------------------------ */

typedef struct srw_factor srw_factor;

/* Builds the random-walk incomplete LDL^T factor of the R-matrix A (Algorithm 1,
 * "Precondition"):
 *   1. checks that A is an R-matrix (Section 1) and that every connected component
 *      has a path to ground (Section 2.1);
 *   2. ranks the nodes: rank = position when sorted by (Philox4x64-10 key, node id),
 *      key = word 0 of the block with key (seed, 0), counter (0, 0, node, 1) -- the
 *      random ordering of Section 5.4 -- or takes opt->rank;
 *   3. builds the walk game of Section 2.1 as integer thresholds;
 *   4. runs walks_per_row walks from every row k that has a higher-ranked neighbour:
 *      the first step goes to a higher-ranked neighbour (Section 5.2), later steps
 *      follow the game, and the walk ends at ground or at a lower-ranked node
 *      ("creating homes", Section 2.2.1).  Draw t of walk w of row k is 32-bit word
 *      (t mod 8) of the Philox4x64-10 block with key (seed, 0) and counter
 *      (t div 8, w, k, 0);
 *   5. reduces the walks of each row to integer tallies M', H'_{k,i}, J'_k
 *      (Section 3.1);
 *   6. forms Y_ki = -(w_ki/a_k + tau_k H'_ki/M'_k) (eq. newy) and
 *      D_k = a_k / (1 + tau_k (J'_k/M'_k - 1)) (eqs. newz, d), with
 *      tau_k = (sum of A_kj over higher-ranked j) / -A_kk, and drops entries with
 *      |Y_ki| < drop_tol (Section 4, footnote);
 *   7. stores Y by rows and by columns for the two triangular solves.
 * Y is unit lower triangular in rank order; the preconditioner is (Y^T D Y)^{-1},
 * i.e. (L D L^T)^{-1} with L = rev(Y)^T of eq. y in the reversed ordering.
 * A must stay valid only during the call.  *out receives a new factor. */
int srw_build_factor(const srw_csr* A, int32_t walks_per_row, double drop_tol, uint64_t seed,
                     const srw_options* opt, srw_factor** out, void* stream);

void srw_factor_free(srw_factor* F);

/* Sizes and counters of a factor (host outputs; any pointer may be NULL):
 * n, nnz_y (strictly triangular entries kept), walks (simulated walks), walk_steps
 * (their total steps), levels_fwd / levels_bwd (length of the longest dependency
 * chain of the triangular solves, the same for both; -1 until srw_factor_depth has
 * computed it), precision (SRW_FP64 / SRW_FP32), keep (srw_options.keep). */
int srw_factor_info(const srw_factor* F, int64_t* n, int64_t* nnz_y, int64_t* walks,
                    int64_t* walk_steps, int32_t* levels_fwd, int32_t* levels_bwd,
                    int32_t* precision, int32_t* keep);

/* Build phases timed when srw_options.profile = 1, in this order. */
#define SRW_NUM_PHASES 8
/* validate, rank, table, schedule (record offsets and the walk queue), walk (the
 * walk kernel alone), tally, factor, plan (Y by columns; both triangles relabelled
 * by solve slot, with the dependency levels when the level order is asked for) */

typedef struct {
    int64_t n, nnz_a, nnz_y;
    int64_t walks;         /* simulated walks                                       */
    int64_t walk_steps;    /* their total steps                                     */
    int64_t walk_deg_sum;  /* sum over steps of the degree of the node left: the
                              walk kernel's algorithmic bytes are
                              12 * walk_steps + 8 * walk_deg_sum                     */
    int32_t levels_fwd, levels_bwd; /* dependency depth, -1 until srw_factor_depth  */
    int32_t precision, keep;
    double phase_ms[SRW_NUM_PHASES]; /* milliseconds, -1 when not profiled           */
} srw_stats;

/* Counters and (if profiled) phase times of a factor; host output. */
int srw_factor_stats(const srw_factor* F, srw_stats* out);

/* Length of the longest dependency chain of the triangular solves (the number of
 * levels a level-by-level substitution would need), computed on the device and cached
 * in the factor; *depth is a host output.  Not needed to solve. */
int srw_factor_depth(srw_factor* F, int32_t* depth, void* stream);

/* Copies the factor to caller device buffers: yptr int64[n+1], ycol int32[nnz_y]
 * (ascending node id per row), yval float64[nnz_y] (FP64 factor) or float32[nnz_y]
 * (FP32 factor), d (same type as yval)[n], rank int32[n].  Any pointer may be NULL. */
int srw_factor_export(const srw_factor* F, int64_t* yptr, int32_t* ycol, void* yval, void* d,
                      int32_t* rank, void* stream);

/* Transition table (needs keep >= 1), device buffers: nbr int32[nnz-n] and
 * thr / mthr uint32[nnz-n] over the off-diagonal entries of A in CSR order (entry q
 * of row v is at rowptr[v] - v + m), tau float64[n], grounded uint8[n].
 * thr = floor(2^32 c_m / a_v) of the running weight sum c_m; mthr the same over the
 * higher-ranked neighbours normalised by their total weight (zero width elsewhere).
 * Any pointer may be NULL. */
int srw_table_export(const srw_factor* F, int32_t* nbr, uint32_t* thr, uint32_t* mthr,
                     double* tau, uint8_t* grounded, void* stream);

/* Per-row tallies (needs keep >= 1), device buffers over nodes: walks uint32[n] (M',
 * 0 for rows without walks), J uint64[n] (sum of stays at the start, start
 * included), G uint32[n] (walks ended at ground), steps uint64[n], visits_sq
 * uint64[n], h_off int64[n] and hlen int32[n]: the distinct end nodes of row k and
 * their counts H'_{k,i} sit at h_end / h_cnt[h_off[k] .. h_off[k] + hlen[k]) in
 * ascending node id; h_end / h_cnt hold `walks` entries in total (see info).
 * Any pointer may be NULL. */
int srw_tally_export(const srw_factor* F, uint32_t* walks, uint64_t* J, uint32_t* G,
                     uint64_t* steps, uint64_t* visits_sq, int64_t* h_off, int32_t* hlen,
                     int32_t* h_end, uint32_t* h_cnt, void* stream);

/* Per-walk records (needs keep == 2): walk w of row k sits at rec_off[k] + w
 * (rec_off int64[n]); end int32 (-1 = ground), visits uint32, length uint32.
 * Any pointer may be NULL. */
int srw_walk_export(const srw_factor* F, int64_t* rec_off, int32_t* end, uint32_t* visits,
                    uint32_t* length, void* stream);

/* ---- the solve ---------------------------------------------------------------- */

/* Preconditioned conjugate gradient (Algorithm 1, "solve"; Barrett et al.,
 * Templates) on A x = b from x0 = 0 with the preconditioner of F.  Stops when the
 * recurrence residual satisfies ||r||_2 <= tol ||b||_2, then recomputes the true
 * residual b - Ax and restarts from it if the test fails.  b, x: device float64[n]
 * (x is overwritten).  Host outputs: iters (products with A inside the iteration),
 * rel_residual = ||b - Ax||_2 / ||b||_2 (0 when b = 0); either may be NULL.
 * Returns SRW_OK or SRW_NOT_CONVERGED (x = last iterate, iters = max_iter).
 * A must be the matrix F was built from. */
int srw_pcg_solve(const srw_csr* A, const srw_factor* F, const double* b, double tol,
                  int32_t max_iter, double* x, int32_t* iters, double* rel_residual,
                  void* stream);

/* z = (Y^T D Y)^{-1} r, one application of the preconditioner (device float64[n]
 * each; r is not modified). */
int srw_apply(const srw_factor* F, const double* r, double* z, void* stream);

/* Human-readable name of a status code (static storage). */
const char* srw_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* SRW_H */
