// Internal layout of srw_factor and the device-memory helpers of libsrw.
#pragma once

#include <vector>

#include "common.hpp"

// Library-owned preconditioner.  Node labels are the caller's row indices; Y is
// stored by rows (CSR, ascending node id per row, strictly lower in rank).  The
// triangular solves run over a solve plan: the rows of Y and of Y^T listed by slot --
// the position of a row in the order the solves take -- with columns given as slots.
struct srw_factor {
    int64_t n = 0;
    int64_t nnz_a = 0;
    int32_t precision = SRW_FP64;
    int32_t keep = 0;
    int64_t nnz_y = 0;
    int64_t walks_total = 0;       // simulated walks
    int64_t steps_total = 0;       // their steps
    int64_t tallied_total = 0;     // walks in the tallies (with walk reuse, the simulated
                                   // walks plus those extracted from them)
    int32_t reuse = 0;
    int32_t walk_waves = 0;  // waves per CU of the walk launch
    int32_t walk_lds = 0;    // 1: the walk kernel read the records from LDS
    int64_t deg_sum = 0;
    double phase_ms[SRW_NUM_PHASES] = {-1, -1, -1, -1, -1, -1, -1, -1};

    int32_t* rank = nullptr;     // [n]
    int32_t* by_rank = nullptr;  // [n] node of each rank
    int64_t* yptr = nullptr;     // [n+1]
    int32_t* ycol = nullptr;     // [nnz_y]
    void* yval = nullptr;        // [nnz_y] double or float
    void* d = nullptr;           // [n] double or float

    // solve plan: slots in increasing (level, rank) or increasing rank
    int32_t* slot_node = nullptr;  // [n] node of each slot
    int32_t* node_slot = nullptr;  // [n]
    int64_t* fptr = nullptr;       // [n+1] rows of Y by slot
    int32_t* fcol = nullptr;       // [nnz_y] slots, row order of Y kept
    void* fval = nullptr;          // [nnz_y]
    int64_t* bptr = nullptr;       // [n+1] rows of Y^T by slot
    int32_t* bcol = nullptr;       // [nnz_y] slots, source rank descending in a row
    void* bval = nullptr;          // [nnz_y]
    void* dslot = nullptr;         // [n] D by slot
    // dense head: the first `head` slots (the lowest ranks, in rank order) are solved
    // with X, the inverse of their diagonal block of Y (unit lower triangular), packed
    // by rows (row i: X[i][0..i] at i(i+1)/2), and its transpose packed by rows (row j:
    // X[j..head-1][j] at j head - j(j-1)/2)
    int64_t head = 0;
    void* hx = nullptr;
    void* hxt = nullptr;

    // longest dependency chain of the triangular solves, -1 until srw_factor_depth
    int32_t depth = -1;
    // level order: first slot of every dependency level past the head, and the end
    // ([depth + 1]; empty for the rank order)
    std::vector<int64_t> level_ptr;

    // asymmetric A (Section 7.1): the factor of the game of A^T with the same ordering
    // (owned); the preconditioner is then (Y_T^T D Y)^{-1}
    srw_factor* tgame = nullptr;

    // batched build: nmat matrices stacked block-diagonally (0 = one matrix)
    int32_t nmat = 0;
    std::vector<int64_t> mat_off_host;  // [nmat+1] first stacked row of every matrix
    int64_t* mat_off = nullptr;         // device copy
    int32_t* node_mat = nullptr;        // [n] matrix of every stacked row
    srw_csr Acat{0, 0, nullptr, nullptr, nullptr};  // the stacked matrix (owned)

    // kept on request (srw_options.keep)
    uint2* ent = nullptr;          // [nnz-n] {neighbour, threshold}
    uint32_t* mthr = nullptr;      // [nnz-n]
    double* tau = nullptr;         // [n]
    uint8_t* grounded = nullptr;   // [n]
    int32_t* budget = nullptr;     // [n] walks per row in the tallies (0 = exact row)
    int64_t* rec_off = nullptr;    // [n] first walk record of each row
    int64_t* h_off = nullptr;      // [n] first H-list entry of each row
    uint64_t* tJ = nullptr;        // [n]
    uint32_t* tG = nullptr;        // [n]
    uint64_t* tsteps = nullptr;    // [n]
    uint64_t* tvsq = nullptr;      // [n]
    int32_t* hlen = nullptr;       // [n]
    uint32_t* h_end = nullptr;     // [tallied_total]
    uint32_t* h_cnt = nullptr;     // [tallied_total]
    uint32_t* rec_end = nullptr;   // [walks_total]
    uint32_t* rec_vis = nullptr;   // [walks_total]
    uint32_t* rec_len = nullptr;   // [walks_total]

    // PCG workspace, allocated on first solve
    double* ws = nullptr;          // r, z, p, q  (4 n)
    void* ws_lo = nullptr;         // two low-precision work vectors for FP32 solves
    double* partials = nullptr;
    double* scalars = nullptr;
    double* host_scalars = nullptr;  // pinned

    std::vector<void*> allocations;       // device blocks owned by this factor (hipMalloc)
    std::vector<void*> pool_allocations;  // ... from the stream-ordered pool (hipMallocAsync)
};

namespace srw {

// rows of the triangular solves' dense head when srw_options.head_rows is 0
constexpr int64_t HEAD_DEFAULT = 4096;
// bound on head rows x head entries (the inverse's work grows with it): about six
// times that of the 128^3 grid's default head (4,096 rows, 0.32M entries, 1.6 ms)
constexpr int64_t HEAD_COST = (int64_t)8 << 30;

// Device allocation tracked by an owner list (freed together).  With a stream the
// blocks come from the stream-ordered pool (hipMallocAsync / hipFreeAsync), so the
// temporaries of repeated builds reuse pooled memory instead of being mapped anew.
// With a chunk size, requests up to half a chunk are carved out of shared chunks
// (256-byte aligned), larger ones get a block of their own: each runtime allocation
// and free costs tens to hundreds of microseconds, so a build makes few of them.
struct Arena {
    std::vector<void*> blocks;
    hipError_t last = hipSuccess;
    hipStream_t stream = nullptr;
    bool pooled = false;
    size_t chunk = 0;    // 0: every request is a block of its own
    char* cur = nullptr;  // free tail of the current chunk
    size_t left = 0;
    template <typename T>
    T* alloc(size_t count)
    {
        const size_t bytes = (((count ? count * sizeof(T) : sizeof(T)) + 255) & ~(size_t)255);
        if (bytes <= left) {
            void* r = cur;
            cur += bytes;
            left -= bytes;
            return (T*)r;
        }
        const bool own = bytes > chunk / 2;
        const size_t size = own ? bytes : chunk;
        void* p = nullptr;
        hipError_t e = pooled ? hipMallocAsync(&p, size, stream) : hipMalloc(&p, size);
        if (e != hipSuccess) {
            last = e;
            return nullptr;
        }
        blocks.push_back(p);
        if (!own) {
            cur = (char*)p + bytes;
            left = size - bytes;
        }
        return (T*)p;
    }
    void release()
    {
        for (void* p : blocks) (void)(pooled ? hipFreeAsync(p, stream) : hipFree(p));
        blocks.clear();
        cur = nullptr;
        left = 0;
    }
};

// Keeps freed stream-ordered allocations in the device's default pool (release
// threshold raised once per device), so they are reused by the next build.
void retain_pool_memory();

// Walk keys of a batched build: the matrix of every node of the block-diagonal
// matrix, the first node of every matrix and the matrix's seed.
struct BatchKeys {
    const int32_t* node_mat;
    const int64_t* mat_off;
    const uint64_t* mat_seed;
    // the slots in the order the dependency-level pass takes them: the matrices
    // interleaved (each in its own order), so that their chains advance together
    const int32_t* level_order;
};

// Walks-only build: apply the Section 5.1 stopping rule to every row's walks and
// write the verdict to found (see k_length_rule); no factor is made.
struct LengthRule {
    double delta, z;
    int32_t min_walks;
    int32_t* found;
};

// Internal status of a walks-only build (never returned by the C ABI).
constexpr int SRW_WALKS_ONLY = 100;

// asym: the matrix's values need not be symmetric (its pattern must be); used for
// each game of an asymmetric matrix
int build_factor_impl(const srw_csr* A, int32_t walks_per_row, double drop_tol, uint64_t seed,
                      const srw_options* opt, srw_factor** out, hipStream_t s,
                      const BatchKeys* batch = nullptr, const LengthRule* rule = nullptr,
                      bool asym = false, bool ic0 = false);
// Asymmetric A (Section 7.1): the game of A, then the game of A^T with its ordering.
int build_ldu_impl(const srw_csr* A, int32_t walks_per_row, double drop_tol, uint64_t seed,
                   const srw_options* opt, srw_factor** out, hipStream_t s);
// Preconditioned BiCGSTAB (F may be null: no preconditioner).
int bicgstab_impl(const srw_csr* A, srw_factor* F, const double* b, double tol, int32_t max_iter,
                  double* x, int32_t* iters, double* rel_residual, hipStream_t s);
// z = M^{-1} r for a factor (symmetric or two-game); work: 2 n doubles; err: one int.
hipError_t apply_factor(const srw_factor* F, const double* r, void* work, double* z, int* err,
                        hipStream_t s);
int adaptive_impl(const srw_csr* A, uint64_t seed, const srw_options* opt, double delta,
                  double z, int32_t min_walks, int32_t max_walks, int32_t* walks, hipStream_t s);
int pcg_impl(const srw_csr* A, srw_factor* F, const double* b, double tol, int32_t max_iter,
             double* x, int32_t* iters, double* rel_residual, hipStream_t s);
int apply_impl(srw_factor* F, const double* r, double* z, hipStream_t s);
// X and X^T of F's dense head (F->head > 0; F->hx, F->hxt allocated, the solve plan
// built).  err: device scratch; *err != 0 afterwards if a wait gave up.
hipError_t head_inverse_launch(const srw_factor* F, int* err, hipStream_t s);
// The largest head of at most h rows whose inverse this device can build (one column of
// the head's values must fit in a workgroup's LDS).
int64_t head_rows_fit(int64_t h);
// srw_apply with the library's static scratch instead of allocations.
int apply_noalloc_impl(const srw_factor* F, const double* r, double* z, hipStream_t s);
int dag_depth(srw_factor* F, int32_t* depth_out, hipStream_t s);
// Dependency level of every slot of the plan (lev, caller-allocated [n]) and the depth.
// order: the slots in the order the pass takes them (NULL: slot order); every slot's
// columns must precede it in that order
int dag_levels(srw_factor* F, int32_t* lev, int32_t* depth_out, hipStream_t s,
               const int32_t* order = nullptr);
void free_factor(srw_factor* F);
int ordering_impl(int64_t n, uint64_t seed, int32_t* rank, hipStream_t s);
int build_batched_impl(int32_t nmat, const srw_csr* A, int32_t walks_per_row, double drop_tol,
                       const uint64_t* seeds, const srw_options* opt, srw_factor** out,
                       hipStream_t s);
int pcg_batched_impl(srw_factor* F, int32_t nrhs, const double* B, double tol, int32_t max_iter,
                     double* X, int32_t* iters, double* rel, int32_t use_graph, hipStream_t s);
int apply_batched_impl(srw_factor* F, int32_t nrhs, const double* R, double* Z, int32_t schedule,
                       hipStream_t s);
int features_impl(const srw_csr* A, const int32_t* rank, float* feat, hipStream_t s);
int labels_impl(const srw_factor* F, int per_step, double* label, hipStream_t s);
int walk_stats_impl(const srw_factor* F, double* var, double* mean_len, hipStream_t s);
int mlp_forward_impl(const float* P, const float* musd, const float* feat, int64_t n, float* out,
                     hipStream_t s);
int mlp_train_impl(float* P, float* m, float* v, int32_t step, float lr, const float* musd,
                   const float* feat, const float* target, const int32_t* rows, int64_t n_rows,
                   int64_t n, float* grad, float* loss, hipStream_t s);
int budget_targets_impl(const double* label, const float* feat, int64_t n, int half, float* x_out,
                        float* y_out, int64_t* count, hipStream_t s);
int mlp_standardize_impl(const float* feat, const float* target, int64_t n, float* mu_sd,
                         float* target_mean, hipStream_t s);
int budgets_impl(const float* pred, int64_t n, double eps, int32_t lo, int32_t hi, int32_t* walks,
                 hipStream_t s);

}  // namespace srw
