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
#define SRW_ORDER_NATURAL 2   /* rank = node id: the natural ordering 1..N the
                                 paper's derivations assume (Sections 2-3)          */

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
    int32_t ordering;          /* SRW_ORDER_RANDOM (or _GIVEN, _NATURAL)            */
    const int32_t* rank;       /* device int32[n], a permutation of 0..n-1, read
                                  when ordering == SRW_ORDER_GIVEN; rank 0 first     */
    const int32_t* walks;      /* device int32[n] per-row walk budgets, or NULL for
                                  the uniform walks_per_row; values < 1 count as 1;
                                  a budget above 8192 on a row that walks fails the
                                  build with SRW_E_ARG before any walk runs          */
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
                                  0 = rank; 1 = dependency level, then rank (the
                                  build computes the levels once); 2 (default) =
                                  level for batched builds, whose many-system solves
                                  need it, else rank (as fast there, and the build
                                  skips the levels)                                  */
    int32_t reuse;             /* 1 = walk reuse (Section 5.3, Algorithm "reuse"):
                                  every walk also counts, for their start nodes, the
                                  walks its two stacks extract (disjoint segments of
                                  at least two steps that end below their start);
                                  the tallies of a row then hold its own walks plus
                                  those.  Needs refill_period 0 or 8 and keep <= 1;
                                  not for batched builds.  A walk keeps at most 64
                                  open segments (else SRW_E_WALK_LIMIT, see
                                  srw_last_error).  0 (default) = off               */
    int32_t walk_waves;        /* waves per compute unit that the persistent walk
                                  kernel runs: 4..64, rounded down to a multiple of
                                  4 and capped at what the kernel's registers allow;
                                  0 = 8.  Fewer walks in flight than the chip can hold
                                  see shorter memory latency per step, which bounds
                                  the longest walks; results do not depend on it     */
    int32_t one_step_exact;    /* 1 (default): the exact one-step treatment of
                                  Section 5.2 (eqs. newy, newz: the first step goes
                                  to a higher-ranked neighbour, rows without one are
                                  exact and walk none); 0: the plain estimator of
                                  eqs. yzdetail and d -- every row walks, every step
                                  (the first included) follows the game, one-step
                                  walks count, Y_ki = -H'_ki / M' and
                                  D_k = M' A_kk / J'_k.  0 is a test mode (both reach
                                  the same limit); it needs reuse = 0 and is refused
                                  by the batched, two-game and adaptive entry points */
    int32_t head_rows;         /* the triangular solves' dense head: the lowest-ranked
                                  h rows, whose long chain of dependencies (their
                                  walks end at one another) would otherwise be solved
                                  level by level, get the explicit inverse of their
                                  diagonal block of Y (computed once by the build,
                                  2 x h(h+1)/2 values) and are solved by two dense
                                  products; the other rows are substituted as before.
                                  0 (default) = min(n, 4096); -1 = none; 1..16384 =
                                  min(n, that), lowered in steps of 64 rows where a
                                  workgroup's LDS cannot hold one column of the
                                  head's values (8 B per row), and where the head's
                                  rows times its entries pass 2^33 (long rows, e.g.
                                  from large per-row budgets).  Single builds only
                                  (batched and two-game builds take none).  Results
                                  agree with the substitution to rounding            */
} srw_options;

#define SRW_HEAD_MAX 16384  /* largest srw_options.head_rows */

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

/* The comparison preconditioner of the paper's ICCG columns (Section 6, Tables 1-2):
 * zero fill-in incomplete Cholesky of the R-matrix A in the same form as the
 * random-walk factor, A ~ Y^T D Y with Y unit lower triangular in rank order.  Nodes
 * are eliminated in decreasing rank and every update outside A's pattern is dropped,
 * so row k of Y holds exactly the lower-ranked neighbours of k:
 *   D_k = A_kk - sum_{j in Up(k)} D_j Y_jk^2,
 *   Y_ki = (A_ki - sum_{j in Up(k), j ~ i} D_j Y_jk Y_ji) / D_k,
 * Up(k) the higher-ranked neighbours of k (sums in row k's CSR order).  The ordering
 * comes from opt as for srw_build_factor (SRW_ORDER_NATURAL for the conventional
 * ICCG; the default is the random ordering of `seed`); walks, reuse and FP32 are
 * refused (SRW_E_ARG).  A is validated as by srw_build_factor.  The result is an
 * srw_factor: srw_pcg_solve, srw_apply, srw_factor_export and srw_factor_free take
 * it as they take a random-walk factor (its walk counters are zero). */
int srw_build_ic0(const srw_csr* A, uint64_t seed, const srw_options* opt, srw_factor** out,
                  void* stream);

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
    int64_t tallied_walks; /* walks in the tallies: = walks, or with walk reuse the
                              simulated walks plus the extracted ones              */
    int32_t reuse;         /* srw_options.reuse of the build                        */
    int32_t two_game;      /* 1 for a factor of srw_build_factor_ldu                */
    int32_t walk_waves;    /* waves per CU the walk kernel ran (0: no walks)        */
    int64_t head_rows;     /* rows of the solves' dense head (0: none)              */
    int32_t walk_lds;      /* 1 if the walk kernel read its records from a copy in
                              each workgroup's LDS (tables of at most the LDS one
                              workgroup can hold, the default refill period), 0
                              if from memory                                      */
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
 * ascending node id; h_end / h_cnt hold srw_stats.tallied_walks entries in total.
 * With walk reuse, `walks` counts the row's own walks and the extracted ones.
 * Any pointer may be NULL. */
int srw_tally_export(const srw_factor* F, uint32_t* walks, uint64_t* J, uint32_t* G,
                     uint64_t* steps, uint64_t* visits_sq, int64_t* h_off, int32_t* hlen,
                     int32_t* h_end, uint32_t* h_cnt, void* stream);

/* Per-row statistics of the walks behind the tallies (needs keep >= 1), device float64
 * outputs over nodes, either may be NULL: visit_var = sample variance of the stays at
 * the start node per walk, (sum v^2 - J'^2 / M') / (M' - 1) (NaN if M' < 2), the
 * spread behind D of eq. d; len_mean = mean walk length steps / M' (NaN if M' = 0), the
 * quantity the stopping rule of Section 5.1 averages.  The pilot statistics from which
 * per-row walk budgets are set. */
int srw_walk_stats(const srw_factor* F, double* visit_var, double* len_mean, void* stream);

/* Per-walk records (needs keep == 2): walk w of row k sits at rec_off[k] + w
 * (rec_off int64[n]); end int32 (-1 = ground), visits uint32, length uint32.
 * Any pointer may be NULL. */
int srw_walk_export(const srw_factor* F, int64_t* rec_off, int32_t* end, uint32_t* visits,
                    uint32_t* length, void* stream);

/* ---- asymmetric matrices (Section 7.1) -------------------------------------------- */

/* Builds the preconditioner of an asymmetric A from two walk games with one ordering:
 * the game of A gives Y_A and D (eqs. y2 and d), the game of A^T gives Y_T (eq. y3),
 * and in rank order A ~ Y_T^T D Y_A (the reversed LDU of rev(A)).  A must have a
 * positive diagonal, negative off-diagonal entries, a symmetric pattern (values may
 * differ: A_kj != A_jk), off-diagonal row sums and column sums both at most the
 * diagonal, and in every connected component a node with positive row excess and a
 * node with positive column excess; else SRW_E_NOT_RMATRIX / SRW_E_SINGULAR.  The
 * game of A^T is built from A^T (formed on the device) with the ordering of the game
 * of A (srw_options.ordering ignored for it) and the same seed, so for a symmetric A
 * both games give the same factor.  Options, limits and errors as srw_build_factor
 * (both builds honour keep, precision and reuse).  The handle owns both factors;
 * srw_factor_export / srw_*_export read the game of A, srw_factor_transpose_game gives
 * the other; srw_apply applies z = (Y_T^T D Y_A)^{-1} r.  Solve with
 * srw_bicgstab_solve (srw_pcg_solve rejects it: the preconditioner is not
 * symmetric). */
int srw_build_factor_ldu(const srw_csr* A, int32_t walks_per_row, double drop_tol,
                         uint64_t seed, const srw_options* opt, srw_factor** out,
                         void* stream);

/* The factor of the game of A^T inside a two-game handle (owned by F: do not free).
 * SRW_E_ARG if F is not a two-game factor. */
int srw_factor_transpose_game(const srw_factor* F, const srw_factor** G);

/* Preconditioned BiCGSTAB (Barrett et al., Templates) on A x = b from x0 = 0, with
 * the preconditioner of F (any factor of A: two-game or symmetric) or none (F NULL).
 * r~ = r0; each iteration applies the preconditioner twice.  Stops when a residual
 * (the half step's s or the full step's r) has ||.||_2 <= tol ||b||_2, then
 * recomputes b - Ax and restarts from it (r~ = r) if the test fails.  Breakdowns
 * (r~.r = 0, r~.v = 0, t.t = 0, omega = 0) return SRW_NOT_CONVERGED with the last
 * iterate.  b, x: device float64[n] (x overwritten); host outputs iters (iterations,
 * a converged half step counting as one) and rel_residual = ||b - Ax||_2 / ||b||_2;
 * either may be NULL.  Returns SRW_OK, SRW_NOT_CONVERGED, SRW_E_ARG, SRW_E_HIP. */
int srw_bicgstab_solve(const srw_csr* A, const srw_factor* F, const double* b, double tol,
                       int32_t max_iter, double* x, int32_t* iters, double* rel_residual,
                       void* stream);

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

/* srw_apply for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and
 * the same result bit for bit, with the triangular solves' work vectors and failure
 * flag in a static scratch array of the library (one per device, 32 MiB + 256 B, held
 * until the process ends) instead of stream-ordered allocations.  It calls no
 * allocating routine.  Limit: F's rows <= SRW_NOALLOC_MAX_N, else SRW_E_ARG (see
 * srw_last_error).  Every call on a device shares that device's scratch: calls that
 * overlap on one device (other streams, other threads) race and must be serialised by
 * the caller.  The call synchronises `stream` to read the solves' status (SRW_E_HIP if
 * a solve gave up waiting). */
#define SRW_NOALLOC_MAX_N (1 << 21)
int srw_apply_noalloc(const srw_factor* F, const double* r, double* z, void* stream);

/* Walks per row by the stopping rule of Section 5.1: walks run from row k one after
 * another until the relative error of their mean length is within delta at confidence
 * alpha, tested as delta * mean * sqrt(M) / sigma > z with z = Q^{-1}((1 - alpha) / 2)
 * (2.5758 for alpha = 99 %; sigma the sample standard deviation of the M lengths,
 * sigma = 0 passes), with at least min_walks (>= 2) and at most max_walks (<= 8192)
 * walks.  Walk w of row k is the walk srw_build_factor would run as walk w, so the
 * budget is exactly the sequential rule's.  walks int32[n] (device output): the budget
 * of every row, 0 for rows whose factor row is exact (no higher-ranked neighbour);
 * pass it as srw_options.walks to build with it.  opt as for srw_build_factor (the
 * ordering and the step cap matter; keep and profile are ignored).  Internally: rounds
 * of walks with doubling per-row targets and a prefix scan of their lengths. */
int srw_adaptive_budgets(const srw_csr* A, uint64_t seed, const srw_options* opt, double delta,
                         double z, int32_t min_walks, int32_t max_walks, int32_t* walks,
                         void* stream);

/* ---- batched builds and solves (an extension: the factor does not depend on b and
 * serves every right-hand side, Sections 2.2 and 6) --------------------------------- */

/* Builds nmat independent R-matrices (A: host array of nmat descriptors of device CSR
 * arrays) as one block-diagonal matrix: one walk launch for all of them.  Matrix i is
 * ordered at random with seeds[i] (host array) and its walks are keyed by its own node
 * ids and seeds[i], so rows off_i .. off_i + n_i - 1 of the result (off_i = n_0 + ... +
 * n_{i-1}) are the factor srw_build_factor gives for A[i] with seed seeds[i], with node
 * ids shifted by off_i.  opt as for srw_build_factor, except that the ordering must be
 * SRW_ORDER_RANDOM; opt->walks, if given, holds budgets over the stacked rows.  The
 * factor keeps a copy of the stacked matrix; export and srw_apply see the stacked
 * system. */
int srw_build_factor_batched(int32_t nmat, const srw_csr* A, int32_t walks_per_row,
                             double drop_tol, const uint64_t* seeds, const srw_options* opt,
                             srw_factor** out, void* stream);

/* Number of stacked matrices (0 for a factor of one matrix) and, if row_off is not
 * NULL, their first rows: row_off int64[nmat + 1] (host). */
int srw_batch_info(const srw_factor* F, int32_t* nmat, int64_t* row_off);

/* PCG on every (matrix, right-hand side) system of a batched factor at once.  B, X:
 * device float64 [N][nrhs] row-major over the stacked rows (1 <= nrhs <= 8); each
 * system (i, j) starts from x0 = 0 and stops when its recurrence residual satisfies
 * ||r|| <= tol ||b||; then its true residual is computed and a system that misses the
 * tolerance restarts from it (at most 3 restarts).  Dot products are reduced per
 * system in a fixed order; the triangular solves carry the nrhs values of a row
 * together.  use_graph = 1 captures one iteration in a HIP graph and replays it.  On
 * first use for a problem shape the solve schedule is picked by timing, and kept for
 * the process: the level-by-level substitutions (one launch per dependency level;
 * batched factors are level-ordered), then the sync-free ones at 2 and 1 blocks per CU
 * with 16, 32 and 64 rows per work claim, the sweep ending as soon as a sync-free
 * schedule is slower than the level-by-level one.
 * Host outputs (may be NULL): iters int32[nmat * nrhs] and rel_residual
 * float64[nmat * nrhs] (true residuals), system (i, j) at i * nrhs + j.  Returns SRW_OK
 * or SRW_NOT_CONVERGED (some system missed tol within max_iter). */
int srw_pcg_solve_batched(srw_factor* F, int32_t nrhs, const double* B, double tol,
                          int32_t max_iter, double* X, int32_t* iters, double* rel_residual,
                          int32_t use_graph, void* stream);

/* One application of the preconditioner to every system of a batched factor: for each
 * matrix i and right-hand side j, z = (Y^T D Y)^{-1} r (Algorithm 1's M applied by a
 * backward then a forward substitution, Section 2.2.2).  R, Z: device float64
 * [N][nrhs] row-major over the stacked rows (1 <= nrhs <= 8), caller-owned; R is read,
 * Z written.  schedule: 0 = the one srw_pcg_solve_batched tuned for this shape (else
 * level by level), 1 = the sync-free substitutions (2 blocks per CU, 16-row claims),
 * 2 = level by level.  Every schedule sums a row's entries in the same order, so all
 * give the same bits.  Allocates a workspace of 2 N nrhs factor values on the stream
 * and synchronises the stream.  Returns SRW_OK, SRW_E_ARG (not a batched factor, nrhs
 * or schedule out of range), or SRW_E_HIP (a sync-free solve gave up waiting). */
int srw_apply_batched(srw_factor* F, int32_t nrhs, const double* R, double* Z, int32_t schedule,
                      void* stream);

/* ---- learned walk budgets (an extension: the paper sets walks per row by a
 * stopping rule on walk lengths, Section 5.1) ------------------------------------ */

/* Random ordering of Section 5.4 alone: rank int32[n] (device), the same ranks
 * srw_build_factor computes for this seed with SRW_ORDER_RANDOM. */
int srw_ordering(int64_t n, uint64_t seed, int32_t* rank, void* stream);

/* Eight float32 features per row (device, row-major [n][8]) from A and the ranks:
 * 0 degree (off-diagonal entries), 1 log a_k, 2 e_k / a_k (excess e_k = a_k - sum of
 * the row's conductances w_kj = -A_kj), 3 tau_k (conductance to higher-ranked
 * neighbours over a_k, Section 5.2), 4 fraction of neighbours ranked above k,
 * 5 log(max w / min w) over the row, 6 log(n / (rank_k + 1)), 7 mean of e_j / a_j over
 * the neighbours (0 for the last three quantities without neighbours).  Computed in
 * float64.  A is not validated here. */
int srw_row_features(const srw_csr* A, const int32_t* rank, float* features, void* stream);

/* Per-walk variance of each row's estimates from the tallies of F (needs keep >= 1):
 * label float64[n] (device) = tau^2 sum_i p_i (1 - p_i) + (tau / (1 + tau (m - 1)))^2 s^2
 * with p_i = H'_{k,i} / M' (Section 3.1, ground excluded), m and s^2 the mean and sample
 * variance of the stays; the first term is the variance of one walk's contribution to
 * the entries of eq. newy, the second the first-order relative variance of eq. d.
 * per_step = 1 divides it by the row's mean walk length (steps per walk): the variance
 * bought per step.  NaN for rows without walks.  Budgets M_k = label_k / eps give every
 * row variance eps; M_k proportional to sqrt(label_k) with per_step = 1 minimise the
 * summed variance at a fixed number of steps. */
int srw_budget_labels(const srw_factor* F, int32_t per_step, double* label, void* stream);

/* The network: 8 -> 64 -> 64 -> 1, ReLU, one float32 array of SRW_MLP_PARAMS on the
 * device: W1 [8][64], b1 [64], W2 [64][64], b2 [64], W3 [64], b3 (row-major, x W).
 * mu_sd float32[16]: per-feature mean then standard deviation; inputs are
 * (feature - mean) / sd.  Inputs, weights and hidden activations enter the matrix
 * cores as bfloat16 (nearest, ties to even); sums are float32. */
#define SRW_MLP_PARAMS 4801

/* out float32[n] = the network's output (predicted log label) for n rows. */
int srw_mlp_forward(const float* params, const float* mu_sd, const float* features, int64_t n,
                    float* out, void* stream);

/* One step on the mean squared error over the n rows given (target float32[n]):
 * gradient by the backward pass (pre-activation gradients rounded to bfloat16 before
 * each product), summed in a fixed order; then, if adam_m and adam_v (float32
 * [SRW_MLP_PARAMS], zero before step 1) are not NULL, one Adam update of params
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias correction by step >= 1, learning rate lr).
 * grad (float32[SRW_MLP_PARAMS]) and loss (float32[1]) are device outputs and may be
 * NULL.  Work and outputs are ordered on the stream; no synchronisation. */
int srw_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t step, float lr,
                       const float* mu_sd, const float* features, const float* target,
                       int64_t n, float* grad, float* loss, void* stream);

/* srw_mlp_train_step on the rows rows[0..n) of features [n_rows][8] and target
 * [n_rows] (a minibatch drawn from the whole training set without copying it; a row may
 * appear more than once).  Returns SRW_E_ARG, with nothing queued, if a listed row lies
 * outside [0, n_rows); the check synchronises the stream. */
int srw_mlp_train_step_rows(float* params, float* adam_m, float* adam_v, int32_t step, float lr,
                            const float* mu_sd, const float* features, const float* target,
                            int64_t n_rows, const int32_t* rows, int64_t n, float* grad,
                            float* loss, void* stream);

/* Training set of the budget network from one matrix: the rows whose label (from
 * srw_budget_labels, float64[n], device) is finite and positive, in row order.
 * x_out float32 [count][8] = their features (srw_row_features), y_out float32[count] =
 * log(label), halved when half = 1 (the budgets exp(prediction) / eps then follow the
 * square root of the label: with labels per walk step, the least summed variance per
 * step).  x_out and y_out hold n rows; *count (host) receives the rows kept.
 * Synchronises the stream. */
int srw_budget_targets(const double* label, const float* features, int64_t n, int32_t half,
                       float* x_out, float* y_out, int64_t* count, void* stream);

/* Statistics of a training set of n >= 1 rows: mu_sd float32[16] = per-feature mean of
 * features [n][8], then the sample standard deviation (divisor n - 1; at least 1e-6; 1
 * when n = 1) -- the input scaling of the network; target_mean float32[1] = the mean of
 * target float32[n] (the output bias a fit starts from).  target and target_mean are
 * both given or both NULL.  Sums in float64 in a fixed order; device outputs, ordered on
 * the stream. */
int srw_mlp_standardize(const float* features, const float* target, int64_t n, float* mu_sd,
                        float* target_mean, void* stream);

/* walks int32[n] = clamp(ceil(exp(pred) / eps), lo, hi): per-row budgets for
 * srw_options.walks (rows with tau = 0 take no walks regardless). */
int srw_mlp_budgets(const float* pred, int64_t n, double eps, int32_t lo, int32_t hi,
                    int32_t* walks, void* stream);

/* The calling thread's last recorded failure: the failing step and HIP error name
 * (thread-local storage, valid until the thread's next failing call; "" if none). */
const char* srw_last_error(void);

/* Human-readable name of a status code (static storage). */
const char* srw_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* SRW_H */
