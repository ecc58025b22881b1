// Batched builds and solves (an extension; the paper's factor is independent of b and is
// reused across right-hand sides, Sections 2.2 and 6): nmat independent R-matrices are
// stacked block-diagonally and built in one pass -- one walk launch for all of them,
// each walk keyed by its own matrix's node ids and seed, so block i of the factor is the
// factor srw_build_factor gives for matrix i alone.  PCG then advances every (matrix,
// right-hand side) system together: one product with the stacked matrix for all
// right-hand sides, dot products reduced per system, and triangular solves that carry
// the nrhs values of a row at once (one dependency chain serves every system).  One
// iteration is captured in a HIP graph and replayed.
//
// Layouts: right-hand sides and solutions are [rows][nrhs] row-major, matrices stacked
// in order.  A system's scalars (rho, alpha, ...) live on the device; a system stops
// moving once its recurrence residual meets the tolerance.
#include <algorithm>
#include <map>
#include <mutex>
#include <cstdio>
#include <cmath>
#include <cstring>

#include "factor.hpp"

namespace srw {

namespace {

constexpr int BLOCK = 256;
constexpr int MAXR = 8;          // right-hand sides per system group
constexpr int TILE_ROWS = 1024;  // rows of one reduction tile (never spans two matrices)

// ------------------------------------------------------------------- stacking
__global__ void k_stack_rowptr(int64_t n, const int64_t* __restrict__ src, int64_t row_off,
                               int64_t nnz_off, int64_t* __restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) dst[row_off + i] = src[i] + nnz_off;
}

__global__ void k_stack_col(int64_t nnz, const int32_t* __restrict__ src, int32_t row_off,
                            int32_t* __restrict__ dst)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) dst[q] = src[q] + row_off;
}

// The batch's orderings, all at once.  Stacked row v of matrix i = node_mat[v] is node
// v - off_i of A[i]; its sort key is the one a single-matrix build of A[i] with seed
// seeds[i] gives that node (Philox of the node id, ties by node id).
__global__ void k_batch_rank_keys(int64_t n, const int32_t* __restrict__ node_mat,
                                  const int64_t* __restrict__ off,
                                  const uint64_t* __restrict__ seed, uint64_t* __restrict__ keys,
                                  uint32_t* __restrict__ vals)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t i = node_mat[v];
    const u64x4 b = philox4x64_10(0, 0, (uint64_t)(v - off[i]), STREAM_ORDER, seed[i], 0);
    keys[v] = b.x0;
    vals[v] = (uint32_t)v;
}

// rows sorted by their key, keyed again by their matrix (a stable sort on it gives the
// rows of every matrix in its own order)
__global__ void k_batch_mat_keys(int64_t n, const uint32_t* __restrict__ rows,
                                 const int32_t* __restrict__ node_mat, uint32_t* __restrict__ keys,
                                 uint32_t* __restrict__ vals)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    keys[p] = (uint32_t)node_mat[rows[p]];
    vals[p] = rows[p];
}

// Position p of the (matrix, own order) list holds the row of local rank r = p - off_i,
// whose stacked rank is p.  For the dependency-level pass the matrices are
// interleaved: that row's key is floor(r 2^32 / n_i), then the matrix, so every
// matrix's rows keep their order and the passes over all matrices advance together
// (in stacked rank order one matrix's chain would hold up the next one's).
__global__ void k_batch_mix_keys(int64_t n, const uint32_t* __restrict__ rows,
                                 const int32_t* __restrict__ node_mat,
                                 const int64_t* __restrict__ off, uint64_t* __restrict__ keys,
                                 uint32_t* __restrict__ vals)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t v = rows[p];
    const int32_t i = node_mat[v];
    const uint64_t r = (uint64_t)(p - off[i]);
    const uint64_t ni = (uint64_t)(off[i + 1] - off[i]);
    keys[p] = ((r << 32) / ni) << 32 | (uint32_t)i;
    vals[p] = (uint32_t)p;  // the row's stacked rank, i.e. its slot in the rank order
}

__global__ void k_batch_rank_scatter(int64_t n, const uint32_t* __restrict__ rows,
                                     int32_t* __restrict__ rank)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) rank[rows[p]] = (int32_t)p;
}

__global__ void k_copy_u32_i32(int64_t n, const uint32_t* __restrict__ a, int32_t* __restrict__ b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (int32_t)a[i];
}

// matrix of every stacked row: the last matrix whose first row is <= the row
__global__ void k_node_mat(int64_t n, int32_t nmat, const int64_t* __restrict__ off,
                           int32_t* __restrict__ node_mat)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t lo = 0, hi = nmat - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) / 2;
        if (off[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    node_mat[v] = lo;
}

// ------------------------------------------------------------------ reductions
enum BOp : int { B_BB = 0, B_RHO0, B_ALPHA, B_RR, B_BETA, B_TRUE_RR };

// One system's scalars.
struct Sys {
    double rho, pq, alpha, rr, beta, bb;
    int32_t active, iters;
};

__device__ __forceinline__ double block_sum(double v, double* lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BLOCK / 64; ++w) s += lds[w];
    __syncthreads();
    return s;
}

struct Tiles {
    const int32_t* mat;   // [ntile] matrix of the tile
    const int64_t* row0;  // [ntile + 1] first row (tiles are contiguous)
};

// Partials over one tile: q = A p and p . q (OP_PQ), r . z (OP_DOT), r . r after the
// x / r update (OP_UPD), ||b - A x||^2 (OP_RES, r overwritten), b . b (OP_BB)
enum TOp : int { T_PQ = 0, T_DOT, T_UPD, T_RES, T_BB };

template <int OP>
__global__ __launch_bounds__(BLOCK) void k_tile(Tiles tl, int nrhs, const int64_t* __restrict__ rowptr,
                                                const int32_t* __restrict__ col,
                                                const double* __restrict__ val,
                                                const double* __restrict__ u,  // p, r, b
                                                const double* __restrict__ v,  // z, q, x
                                                double* __restrict__ w,        // q, x, r
                                                double* __restrict__ r2,       // r (T_UPD)
                                                const Sys* __restrict__ sys,
                                                double* __restrict__ partials)
{
    __shared__ double lds[BLOCK / 64];
    const int64_t t = blockIdx.x;
    const int32_t m = tl.mat[t];
    const int64_t r0 = tl.row0[t], r1 = tl.row0[t + 1];
    double acc[MAXR];
#pragma unroll
    for (int j = 0; j < MAXR; ++j) acc[j] = 0.0;
    // one thread per (row, right-hand side): the tile's nrhs-wide rows are contiguous,
    // so neighbouring threads touch neighbouring values
    const int64_t f0 = r0 * nrhs;
    const int nf = (int)((r1 - r0) * nrhs);  // <= TILE_ROWS * MAXR
    for (int fr = threadIdx.x; fr < nf; fr += BLOCK) {
        const int64_t f = f0 + fr;
        const int j = fr % nrhs;
        double add;
        if (OP == T_PQ || OP == T_RES) {
            const int64_t i = r0 + fr / nrhs;
            const double* src = OP == T_PQ ? u : v;  // p, or x
            double sum = 0.0;
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
                sum += val[e] * src[(int64_t)col[e] * nrhs + j];
            if (OP == T_PQ) {
                w[f] = sum;
                add = u[f] * sum;
            } else {
                const double rv = u[f] - sum;  // b - A x
                w[f] = rv;
                add = rv * rv;
            }
        } else if (OP == T_DOT || OP == T_BB) {
            add = u[f] * (OP == T_BB ? u[f] : v[f]);
        } else {  // T_UPD: x += alpha p, r -= alpha q (active systems)
            const Sys& S = sys[(int64_t)m * nrhs + j];
            double rv = r2[f];
            if (S.active) {
                w[f] = w[f] + S.alpha * u[f];
                rv = rv - S.alpha * v[f];
                r2[f] = rv;
            }
            add = rv * rv;
        }
#pragma unroll
        for (int jj = 0; jj < MAXR; ++jj)
            if (jj == j) acc[jj] += add;
    }
#pragma unroll
    for (int j = 0; j < MAXR; ++j) {
        if (j >= nrhs) continue;
        const double s = block_sum(acc[j], lds);
        if (threadIdx.x == 0) partials[t * nrhs + j] = s;
    }
}

// One thread per system: sum the partials of its matrix's tiles in order, then the
// scalar update of `op`.
__global__ void k_bfinal(int64_t nsys, int nrhs, const int64_t* __restrict__ mat_tile,
                         const double* __restrict__ partials, Sys* __restrict__ sys, int op,
                         double tol, int32_t max_iter, int* __restrict__ active_count)
{
    const int64_t sidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sidx >= nsys) return;
    const int64_t m = sidx / nrhs;
    const int j = (int)(sidx % nrhs);
    double s = 0.0;
    for (int64_t t = mat_tile[m]; t < mat_tile[m + 1]; ++t) s += partials[t * nrhs + j];
    Sys& S = sys[sidx];
    switch (op) {
        case B_BB:
            S.bb = s;
            S.active = s > 0.0 ? 1 : 0;
            S.iters = 0;
            break;
        case B_RHO0:
            if (S.active) S.rho = s;
            break;
        case B_ALPHA:
            if (S.active) {
                S.pq = s;
                S.alpha = S.rho / s;
            }
            break;
        case B_RR:
            if (S.active) {
                S.rr = s;
                S.iters += 1;
                if (sqrt(s) <= tol * sqrt(S.bb) || S.iters >= max_iter || !(s == s)) S.active = 0;
                else atomicAdd(active_count, 1);
            }
            break;
        case B_BETA:
            if (S.active) {
                S.beta = s / S.rho;
                S.rho = s;
            }
            break;
        case B_TRUE_RR:
            S.rr = s;
            // restart a system whose true residual misses the tolerance
            if (S.bb > 0.0 && sqrt(s) > tol * sqrt(S.bb) && S.iters < max_iter && s == s) {
                S.active = 1;
                atomicAdd(active_count, 1);
            } else {
                S.active = 0;
            }
            break;
    }
}

// p = z (restart) or p = z + beta p, active systems only
__global__ void k_bupdate_p(int64_t n, int nrhs, const int32_t* __restrict__ node_mat,
                            const double* __restrict__ z, double* __restrict__ p,
                            const Sys* __restrict__ sys, int restart)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    const int64_t row = i / nrhs;
    const int j = (int)(i % nrhs);
    const Sys& S = sys[(int64_t)node_mat[row] * nrhs + j];
    if (!S.active) return;
    p[i] = restart ? z[i] : z[i] + S.beta * p[i];
}

__global__ void k_copy_d(int64_t n, const double* __restrict__ a, double* __restrict__ b)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

__global__ void k_zero_d(int64_t n, double* __restrict__ a)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0;
}

__global__ void k_zero_i(int* a) { *a = 0; }

__global__ void k_zero_n(int* a, int n)
{
    if ((int)threadIdx.x < n) a[threadIdx.x] = 0;
}

// --------------------------------------------------- multi right-hand-side solves
// The substitutions of solve.hip with nrhs values per slot, stored [slot][nrhs]: a
// row's values are published by lane 0 with one device-scope store each, every value
// its own ready flag (signalling-NaN sentinel).  A waiting wave polls one address --
// the last value of its dependency that the order solves last -- then reloads its
// missing values.
//
// Work is claimed, not assigned: a wave takes the next `chunk` consecutive slots of the
// order from one counter (one atomic per claim) and solves them in order.  Claims are
// handed out in slot order, so every slot below the lowest unclaimed one belongs to a
// wave that is running.  The lowest unfinished slot therefore always has a running
// owner that has finished the earlier slots of its claim, and its dependencies (all
// lower slots) are finished: the solve progresses whether or not every wave of the
// grid is resident at once.  (A fixed cycle -- wave i takes slots i, i + W, ... --
// does not: a slot whose wave has not been dispatched yet can hold up the waves that
// occupy the chip.)
template <typename T>
struct MBits;
template <>
struct MBits<double> {
    using U = unsigned long long;
    static constexpr U sentinel = 0x7FF4DEADBEEF5A5Aull;
    static __device__ U nan_bits() { return 0x7FF8000000000000ull; }
};
template <>
struct MBits<float> {
    using U = unsigned int;
    static constexpr U sentinel = 0x7FA5A5A5u;
    static __device__ U nan_bits() { return 0x7FC00000u; }
};

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_mfill(int64_t n, T* x)
{
    using U = typename MBits<T>::U;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        ((U*)x)[i] = MBits<T>::sentinel;
}

template <typename U>
__device__ __forceinline__ U mload(const U* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Solve-claim counters, zeroed before every launch (a kernel, not a memset: the solves
// are captured in a graph).
__global__ void k_zero_u64(unsigned long long* a, int n)
{
    if ((int)threadIdx.x < n) a[threadIdx.x] = 0ull;
}

// A row of the multi-right-hand-side solves takes RG lanes: a wave solves 64 / RG rows
// at a time (the batch's rows are short, about nine entries), each lane summing the
// entries j, j + RG, ... of its row over all right-hand sides, the RG partial sums then
// added by a butterfly within the row's lanes.  A wave claims `chunk` consecutive slots
// (a multiple of 64 / RG) and solves them 64 / RG at a time, in order; within a round
// the rows wait and finish independently (a row may wait for another row of the same
// round).  A lane polls the values it is missing itself.
//
// In-order claims guarantee progress, not speed.  A wave cannot start a round before
// its earlier rounds are done, so with many waves each holding a long claim, rows whose
// values are ready queue behind rows that wait: the solve time grows steeply with
// waves x claim length (measured on 8.6 M slots, 8 right-hand sides, claims of 512
// slots: 108, 196 and 459 ms at 2, 4 and 5 blocks per CU, against 13 ms at 2 blocks
// per CU with 32-slot claims).  The tuner therefore tries only short claims on a
// grid of at most two blocks per CU (see pcg_batched_impl).
//
// wait_ticks: wall-clock ticks (constant-rate counter) after which a wait gives up --
// a guard against a defect, set far above the solve time of every schedule the tuner
// tries.
constexpr int RG = 8;
constexpr int RPW = 64 / RG;  // rows of a wave in flight

template <typename T, bool FWD>
__global__ __launch_bounds__(BLOCK) void k_trsv_multi(int64_t n, int nrhs, int32_t chunk,
                                                      const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ col,
                                                      const T* __restrict__ val,
                                                      const T* __restrict__ dslot,
                                                      const int32_t* __restrict__ slot_node,
                                                      const double* __restrict__ rhs,
                                                      const T* __restrict__ w, T* sol,
                                                      double* __restrict__ out, int* err,
                                                      unsigned long long* claim, int64_t wait_ticks)
{
    using U = typename MBits<T>::U;
    const int lane = threadIdx.x & 63;
    const int grp = lane / RG, j = lane % RG;
    for (;;) {
        // every lane executes the atomic (lane 0 adds the chunk) and the claim is read
        // from lane 0 as a scalar, so the loop exit below is a uniform branch
        const uint64_t base =
            lane0_u64(atomicAdd(claim, lane == 0 ? (unsigned long long)chunk : 0ull));
        if (base >= (uint64_t)n) break;
        const int64_t stop = std::min<int64_t>((int64_t)base + chunk, n);
        for (int64_t r0 = (int64_t)base; r0 < stop; r0 += RPW) {
            const int64_t i = r0 + grp;
            bool done = i >= stop;
            const int64_t s = done ? 0 : (FWD ? i : n - 1 - i);
            int64_t qc = done ? 0 : ptr[s];
            const int64_t q1 = done ? 0 : ptr[s + 1];
            T acc[MAXR];
#pragma unroll
            for (int jr = 0; jr < MAXR; ++jr) acc[jr] = T(0);
            U bits[MAXR];
            T a = T(0);
            int32_t c = 0;
            bool loaded = false;
            uint32_t spins = 0;
            const int64_t t0 = wall_clock64();
            while (ballot(!done) != 0) {
                const bool ok = !done && qc + j < q1;
                if (!done && !loaded) {
                    c = ok ? col[qc + j] : 0;
                    a = ok ? val[qc + j] : T(0);
                    const U* src = (const U*)sol + (int64_t)c * nrhs;
#pragma unroll
                    for (int jr = 0; jr < MAXR; ++jr)
                        bits[jr] = (ok && jr < nrhs) ? mload(src + jr) : U(0);
                    loaded = true;
                }
                bool miss = false;
#pragma unroll
                for (int jr = 0; jr < MAXR; ++jr)
                    miss = miss || (ok && jr < nrhs && bits[jr] == MBits<T>::sentinel);
                const uint64_t mb = ballot(miss);
                const bool gmiss = ((mb >> (grp * RG)) & ((1ull << RG) - 1)) != 0;
                bool finishing = false;
                if (!done && !gmiss) {  // the row's current entries are all there
#pragma unroll
                    for (int jr = 0; jr < MAXR; ++jr) acc[jr] += a * __builtin_bit_cast(T, bits[jr]);
                    qc += RG;
                    loaded = false;
                    finishing = qc >= q1;
                }
                if (ballot(finishing) != 0) {
                    const int32_t node = finishing ? slot_node[s] : 0;
                    const T dv = (FWD && finishing) ? dslot[s] : T(1);
#pragma unroll
                    for (int jr = 0; jr < MAXR; ++jr) {
                        T v = acc[jr];
                        v += __shfl_xor(v, 4, 64);
                        v += __shfl_xor(v, 2, 64);
                        v += __shfl_xor(v, 1, 64);
                        if (finishing && j == 0 && jr < nrhs) {
                            const T base_v = FWD ? w[s * nrhs + jr] / dv : (T)rhs[(int64_t)node * nrhs + jr];
                            const T x = base_v - v;
                            __hip_atomic_store((U*)sol + s * nrhs + jr, __builtin_bit_cast(U, x),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            if (out) out[(int64_t)node * nrhs + jr] = (double)x;
                        }
                    }
                    if (finishing) done = true;
                }
                if (!done && gmiss) {
                    // every 256 polls: give up past the time limit, or at once when
                    // another wave already gave up (a failed solve then drains)
                    if ((++spins & 255u) == 0) {
                        const bool failed =
                            __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
                        if (failed || wall_clock64() - t0 > wait_ticks) {
                            if (j == 0) {
                                atomicOr(err, 1);
                                // the first to give up records where it waited: err[2..6] =
                                // direction, slot, awaited slot, value absent, chunk
                                if (!failed && atomicCAS(err + 1, 0, 1) == 0) {
                                    err[2] = FWD ? 1 : 0;
                                    err[3] = (int)s;
                                    err[4] = c;
                                    err[5] = 1;
                                    err[6] = chunk;
                                }
                            }
#pragma unroll
                            for (int jr = 0; jr < MAXR; ++jr)
                                if (bits[jr] == MBits<T>::sentinel) bits[jr] = MBits<T>::nan_bits();
                        }
                    }
                    __builtin_amdgcn_s_sleep(2);
                    const U* src = (const U*)sol + (int64_t)c * nrhs;
#pragma unroll
                    for (int jr = 0; jr < MAXR; ++jr)
                        if (ok && jr < nrhs && bits[jr] == MBits<T>::sentinel) bits[jr] = mload(src + jr);
                }
            }
        }
    }
}

// The MAXR = 8 values of a row (64 or 32 bytes, aligned to their size) in 16-byte loads.
__device__ __forceinline__ void load_row8(const double* p, double (&x)[MAXR])
{
    const double2* q = (const double2*)p;
#pragma unroll
    for (int k = 0; k < MAXR / 2; ++k) {
        const double2 v = q[k];
        x[2 * k] = v.x;
        x[2 * k + 1] = v.y;
    }
}
__device__ __forceinline__ void load_row8(const float* p, float (&x)[MAXR])
{
    const float4* q = (const float4*)p;
#pragma unroll
    for (int k = 0; k < MAXR / 4; ++k) {
        const float4 v = q[k];
        x[4 * k] = v.x;
        x[4 * k + 1] = v.y;
        x[4 * k + 2] = v.z;
        x[4 * k + 3] = v.w;
    }
}

// Level-by-level substitution: one launch per dependency level of a level-ordered
// plan, over the level's slots [a, b).  Every value a row reads was written by an
// earlier launch, so there is no waiting and no flag.  A row takes RG lanes and its
// entries and partial sums go exactly as in k_trsv_multi (lane j: entries j, j + RG,
// ..., a zero product where a round runs past the row; then the butterfly), so both
// kernels give the same bits.  Lane j of a row writes right-hand side j.
template <typename T, bool FWD>
__global__ __launch_bounds__(BLOCK) void k_trsv_level(int64_t a, int64_t b, int nrhs,
                                                      const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ col,
                                                      const T* __restrict__ val,
                                                      const T* __restrict__ dslot,
                                                      const int32_t* __restrict__ slot_node,
                                                      const double* __restrict__ rhs,
                                                      const T* __restrict__ w, T* __restrict__ sol,
                                                      double* __restrict__ out)
{
    const int64_t s = a + ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / RG;
    const int j = (int)(threadIdx.x % RG);
    const bool row = s < b;
    T acc[MAXR];
#pragma unroll
    for (int jr = 0; jr < MAXR; ++jr) acc[jr] = T(0);
    if (row) {
        const int64_t q0 = ptr[s], q1 = ptr[s + 1];
        for (int64_t qb = q0; qb < q1; qb += RG) {
            const int64_t q = qb + j;
            const bool ok = q < q1;
            const int32_t c = ok ? col[q] : 0;
            const T av = ok ? val[q] : T(0);
            const T* src = sol + (int64_t)c * nrhs;
            T xv[MAXR];
            if (nrhs == MAXR) {
                load_row8(src, xv);  // a whole row of values in 16-byte loads
            } else {
#pragma unroll
                for (int jr = 0; jr < MAXR; ++jr) xv[jr] = jr < nrhs ? src[jr] : T(0);
            }
#pragma unroll
            for (int jr = 0; jr < MAXR; ++jr) {
                const T x = ok ? xv[jr] : T(0);
                acc[jr] += av * x;
            }
        }
    }
    T v = T(0);
#pragma unroll
    for (int jr = 0; jr < MAXR; ++jr) {
        T t = acc[jr];
        t += __shfl_xor(t, 4, 64);
        t += __shfl_xor(t, 2, 64);
        t += __shfl_xor(t, 1, 64);
        v = jr == j ? t : v;
    }
    if (row && j < nrhs) {
        const int32_t node = slot_node[s];
        const T base_v = FWD ? w[s * nrhs + j] / dslot[s] : (T)rhs[(int64_t)node * nrhs + j];
        const T x = base_v - v;
        sol[s * nrhs + j] = x;
        if (out) out[(int64_t)node * nrhs + j] = (double)x;
    }
}

int fill_grid(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>(grid_for(n, BLOCK), 1), 2048); }

}  // namespace

// -------------------------------------------------------------------- the build
int build_batched_impl(int32_t nmat, const srw_csr* A, int32_t walks_per_row, double drop_tol,
                       const uint64_t* seeds, const srw_options* opt_in, srw_factor** out,
                       hipStream_t s)
{
    std::vector<int64_t> off(nmat + 1, 0), nnz_off(nmat + 1, 0);
    for (int32_t i = 0; i < nmat; ++i) {
        off[i + 1] = off[i] + A[i].n;
        nnz_off[i + 1] = nnz_off[i] + A[i].nnz;
    }
    const int64_t N = off[nmat], NNZ = nnz_off[nmat];
    if (N >= (int64_t)0x7FFFFFFF) return SRW_E_ARG;
    Arena own;  // arrays the factor keeps
#define BALLOC(T, cnt) own.alloc<T>((size_t)(cnt))
    int64_t* rowptr = BALLOC(int64_t, N + 1);
    int32_t* col = BALLOC(int32_t, std::max<int64_t>(NNZ, 1));
    double* val = BALLOC(double, std::max<int64_t>(NNZ, 1));
    int32_t* rank = BALLOC(int32_t, std::max<int64_t>(N, 1));
    int32_t* node_mat = BALLOC(int32_t, std::max<int64_t>(N, 1));
    int64_t* mat_off = BALLOC(int64_t, nmat + 1);
    uint64_t* mat_seed = BALLOC(uint64_t, nmat);
#undef BALLOC
    auto fail = [&](int st) {
        (void)hipStreamSynchronize(s);
        own.release();
        return st;
    };
    if (!rowptr || !col || !val || !rank || !node_mat || !mat_off || !mat_seed) return fail(SRW_E_NOMEM);
    hipError_t e = hipSuccess;
    for (int32_t i = 0; i < nmat && e == hipSuccess; ++i) {
        const int64_t n = A[i].n, nnz = A[i].nnz;
        k_stack_rowptr<<<grid_for(n + 1, BLOCK), BLOCK, 0, s>>>(n, A[i].rowptr, off[i], nnz_off[i], rowptr);
        if (nnz > 0) {
            k_stack_col<<<grid_for(nnz, BLOCK), BLOCK, 0, s>>>(nnz, A[i].col, (int32_t)off[i], col + nnz_off[i]);
            e = hipMemcpyAsync(val + nnz_off[i], A[i].val, nnz * sizeof(double), hipMemcpyDeviceToDevice, s);
        }
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(mat_off, off.data(), (nmat + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(mat_seed, seeds, nmat * sizeof(uint64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && N > 0) {
        k_node_mat<<<grid_for(N, BLOCK), BLOCK, 0, s>>>(N, nmat, mat_off, node_mat);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return fail(hip_fail(e, "batched stacking"));
    // one random ordering per matrix (its own seed), shifted into the stacked order:
    // all rows sorted by their key, then stably by their matrix; then the matrices
    // interleaved for the dependency-level pass
    int32_t* level_order = nullptr;
    if (N > 0) {
        char* ws = nullptr;
        const size_t rt = radix_tmp_bytes(N);
        const size_t bytes = (size_t)N * (2 * sizeof(uint64_t) + 4 * sizeof(uint32_t)) + rt + 256;
        if ((e = hipMallocAsync((void**)&ws, bytes, s)) != hipSuccess)
            return fail(hip_fail(e, "batched ordering"));
        if ((e = hipMallocAsync((void**)&level_order, (size_t)N * sizeof(int32_t), s)) != hipSuccess) {
            (void)hipFreeAsync(ws, s);
            return fail(hip_fail(e, "batched ordering"));
        }
        uint64_t* k64 = (uint64_t*)ws;
        uint64_t* k64b = k64 + N;
        uint32_t* v1 = (uint32_t*)(k64b + N);
        uint32_t* v2 = v1 + N;
        uint32_t* k32 = v2 + N;
        uint32_t* k32b = k32 + N;
        void* tmp = (void*)(((uintptr_t)(k32b + N) + 255) & ~(uintptr_t)255);
        uint64_t* ko = nullptr;
        uint32_t* ko32 = nullptr;
        uint32_t* vo = nullptr;
        const int g = grid_for(N, BLOCK);
        int mbits = 1;
        while (mbits < 32 && ((int64_t)1 << mbits) < nmat) ++mbits;
        k_batch_rank_keys<<<g, BLOCK, 0, s>>>(N, node_mat, mat_off, mat_seed, k64, v1);
        e = hipGetLastError();
        if (e == hipSuccess) e = radix_sort_u64(k64, v1, k64b, v2, N, 64, tmp, &ko, &vo, s);
        if (e == hipSuccess) {
            uint32_t* rows = vo;
            uint32_t* other = rows == v1 ? v2 : v1;
            k_batch_mat_keys<<<g, BLOCK, 0, s>>>(N, rows, node_mat, k32, other);
            e = hipGetLastError();
            if (e == hipSuccess)
                e = radix_sort_u32(k32, other, k32b, rows, N, mbits, tmp, &ko32, &vo, s);
        }
        if (e == hipSuccess) {
            uint32_t* rows = vo;  // rows by (matrix, own order): position = stacked rank
            uint32_t* other = rows == v1 ? v2 : v1;
            k_batch_rank_scatter<<<g, BLOCK, 0, s>>>(N, rows, rank);
            k_batch_mix_keys<<<g, BLOCK, 0, s>>>(N, rows, node_mat, mat_off, k64, other);
            e = hipGetLastError();
            if (e == hipSuccess) e = radix_sort_u64(k64, other, k64b, rows, N, 64, tmp, &ko, &vo, s);
        }
        if (e == hipSuccess) {
            k_copy_u32_i32<<<g, BLOCK, 0, s>>>(N, vo, level_order);
            e = hipGetLastError();
        }
        (void)hipFreeAsync(ws, s);
        if (e != hipSuccess) {
            (void)hipFreeAsync(level_order, s);
            return fail(hip_fail(e, "batched ordering"));
        }
    }
    srw_options opt = *opt_in;
    opt.ordering = SRW_ORDER_GIVEN;
    opt.rank = rank;
    if (opt.solve_order == 2) opt.solve_order = 1;  // the batched solves need the levels
    srw_csr cat{N, NNZ, rowptr, col, val};
    BatchKeys keys{node_mat, mat_off, mat_seed, level_order};
    srw_factor* F = nullptr;
    const int st = build_factor_impl(&cat, walks_per_row, drop_tol, 0, &opt, &F, s, &keys);
    if (level_order) (void)hipFreeAsync(level_order, s);
    if (st != SRW_OK) return fail(st);
    F->nmat = nmat;
    F->mat_off_host = off;
    F->mat_off = mat_off;
    F->node_mat = node_mat;
    F->Acat = cat;
    for (void* p : own.blocks) F->allocations.push_back(p);
    own.blocks.clear();
    *out = F;
    return SRW_OK;
}

// -------------------------------------------------------------------- the solve
namespace {

struct BatchWork {
    int64_t N = 0, nsys = 0, ntile = 0;
    int nrhs = 0;
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *partials = nullptr;
    void* work = nullptr;  // 2 N nrhs values of the factor's precision
    Sys* sys = nullptr;
    int* active = nullptr;
    int* err = nullptr;
    unsigned long long* claim = nullptr;  // two solve-claim counters
    int64_t wait_ticks = 0;
    Tiles tiles{};
    int64_t* mat_tile = nullptr;
};

// Solve schedule: blocks per CU of the launch grid and slots per claim, or (level)
// one launch per dependency level.
struct Sched {
    int per_cu = 0;  // 0: not tuned
    int chunk = 0;
    int level = 0;
};

// Stream-ordered launch of a persistent grid of up to per_cu_cap blocks per CU (the
// occupancy the kernel allows, capped), no more than the work can use.  Progress does
// not depend on these blocks being resident together (see k_trsv_multi).
template <typename K>
hipError_t solve_launch(K kernel, int64_t rows, int chunk, int per_cu_cap, void** args, hipStream_t s)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, BLOCK, 0);
    if (e != hipSuccess) return e;
    if (per_cu_cap > 0) per_cu = std::min(per_cu, per_cu_cap);
    int64_t blocks = (int64_t)cus * std::max(1, per_cu);
    const int64_t claims = (rows + chunk - 1) / chunk;
    blocks = std::min<int64_t>(blocks, (claims + BLOCK / 64 - 1) / (BLOCK / 64));
    if (blocks < 1) blocks = 1;
    return hipLaunchKernel((const void*)kernel, dim3((unsigned)blocks), dim3(BLOCK), args, 0, s);
}

template <typename T>
hipError_t batch_apply(const srw_factor* F, BatchWork& W, const Sched& sc, hipStream_t s)
{
    int64_t n = F->n;
    int nrhs = W.nrhs;
    int32_t chunk = sc.chunk;
    int64_t ticks = W.wait_ticks;
    T* work = (T*)W.work;
    T* sol = work + n * nrhs;
    if (sc.level) {
        const std::vector<int64_t>& lp = F->level_ptr;
        const int L = (int)lp.size() - 1;
        const int64_t per_block = BLOCK / RG;
        for (int l = L - 1; l >= 0; --l) {  // backward: the levels in reverse
            const int64_t a = lp[l], b = lp[l + 1];
            if (b <= a) continue;
            k_trsv_level<T, false><<<(unsigned)((b - a + per_block - 1) / per_block), BLOCK, 0, s>>>(
                a, b, nrhs, F->bptr, F->bcol, (const T*)F->bval, nullptr, F->slot_node, W.r,
                nullptr, work, nullptr);
        }
        for (int l = 0; l < L; ++l) {
            const int64_t a = lp[l], b = lp[l + 1];
            if (b <= a) continue;
            k_trsv_level<T, true><<<(unsigned)((b - a + per_block - 1) / per_block), BLOCK, 0, s>>>(
                a, b, nrhs, F->fptr, F->fcol, (const T*)F->fval, (const T*)F->dslot, F->slot_node,
                nullptr, work, sol, W.z);
        }
        return hipGetLastError();
    }
    k_mfill<T><<<fill_grid(n * nrhs), BLOCK, 0, s>>>(n * nrhs, work);
    k_mfill<T><<<fill_grid(n * nrhs), BLOCK, 0, s>>>(n * nrhs, sol);
    k_zero_u64<<<1, 64, 0, s>>>(W.claim, 2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        const int64_t* ptr = F->bptr;
        const int32_t* col = F->bcol;
        const T* val = (const T*)F->bval;
        const T* dslot = nullptr;
        const int32_t* sn = F->slot_node;
        const double* rhs = W.r;
        const T* w = nullptr;
        T* o = work;
        double* out = nullptr;
        int* err = W.err;
        unsigned long long* claim = W.claim;
        void* args[] = {&n, &nrhs, &chunk, &ptr, &col, &val, &dslot, &sn, &rhs, &w, &o, &out, &err,
                        &claim, &ticks};
        e = solve_launch(k_trsv_multi<T, false>, n, chunk, sc.per_cu, args, s);
        if (e != hipSuccess) return e;
    }
    {
        const int64_t* ptr = F->fptr;
        const int32_t* col = F->fcol;
        const T* val = (const T*)F->fval;
        const T* dslot = (const T*)F->dslot;
        const int32_t* sn = F->slot_node;
        const double* rhs = nullptr;
        const T* w = work;
        T* o = sol;
        double* out = W.z;
        int* err = W.err;
        unsigned long long* claim = W.claim + 1;
        void* args[] = {&n, &nrhs, &chunk, &ptr, &col, &val, &dslot, &sn, &rhs, &w, &o, &out, &err,
                        &claim, &ticks};
        e = solve_launch(k_trsv_multi<T, true>, n, chunk, sc.per_cu, args, s);
    }
    return e;
}

hipError_t apply_b(const srw_factor* F, BatchWork& W, const Sched& sc, hipStream_t s)
{
    return F->precision == SRW_FP32 ? batch_apply<float>(F, W, sc, s) : batch_apply<double>(F, W, sc, s);
}

// z = M^{-1} r, then rho / p for the active systems (restart = 1: p = z)
hipError_t iteration(const srw_factor* F, BatchWork& W, const Sched& sc, double* X, double tol,
                     int32_t max_iter, hipStream_t s)
{
    const srw_csr& A = F->Acat;
    const int nrhs = W.nrhs;
    const int sg = (int)((W.nsys + 255) / 256);
    const int64_t nv = W.N * nrhs;
    hipError_t e;
    k_tile<T_PQ><<<(unsigned)W.ntile, BLOCK, 0, s>>>(W.tiles, nrhs, A.rowptr, A.col, A.val, W.p,
                                                     nullptr, W.q, nullptr, W.sys, W.partials);
    k_bfinal<<<sg, 256, 0, s>>>(W.nsys, nrhs, W.mat_tile, W.partials, W.sys, B_ALPHA, tol, max_iter, W.active);
    k_zero_i<<<1, 1, 0, s>>>(W.active);
    k_tile<T_UPD><<<(unsigned)W.ntile, BLOCK, 0, s>>>(W.tiles, nrhs, nullptr, nullptr, nullptr, W.p,
                                                      W.q, X, W.r, W.sys, W.partials);
    k_bfinal<<<sg, 256, 0, s>>>(W.nsys, nrhs, W.mat_tile, W.partials, W.sys, B_RR, tol, max_iter, W.active);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = apply_b(F, W, sc, s)) != hipSuccess) return e;
    k_tile<T_DOT><<<(unsigned)W.ntile, BLOCK, 0, s>>>(W.tiles, nrhs, nullptr, nullptr, nullptr, W.r,
                                                      W.z, nullptr, nullptr, W.sys, W.partials);
    k_bfinal<<<sg, 256, 0, s>>>(W.nsys, nrhs, W.mat_tile, W.partials, W.sys, B_BETA, tol, max_iter, W.active);
    k_bupdate_p<<<grid_for(nv, 256), 256, 0, s>>>(W.N, nrhs, F->node_mat, W.z, W.p, W.sys, 0);
    return hipGetLastError();
}

// Process-wide cache of tuned solve schedules.
struct TuneKey {
    int64_t n, nnz;
    int nrhs, precision;
    bool operator<(const TuneKey& o) const
    {
        if (n != o.n) return n < o.n;
        if (nnz != o.nnz) return nnz < o.nnz;
        if (nrhs != o.nrhs) return nrhs < o.nrhs;
        return precision < o.precision;
    }
};

std::mutex g_tune_mu;
std::map<TuneKey, Sched> g_tuned;

Sched tuned_schedule(const TuneKey& k)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(k);
    return it == g_tuned.end() ? Sched{} : it->second;
}

void remember_schedule(const TuneKey& k, const Sched& sc, float ms)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[k] = sc;
    (void)ms;
}

}  // namespace

// One application z = M^{-1} r to every system of a batched factor, on the schedule
// asked for (0: the one tuned for this shape, else level by level where the plan has
// levels, else the sync-free kernel; 1: the sync-free kernel, 2 blocks per CU and
// claims of 16 slots; 2: level by level).
int apply_batched_impl(srw_factor* F, int32_t nrhs, const double* R, double* Z, int32_t schedule,
                       hipStream_t s)
{
    const bool has_levels = !F->level_ptr.empty() && F->head == 0;
    if (schedule == 2 && !has_levels) {
        set_last_error("srw_apply_batched: the factor's plan has no dependency levels");
        return SRW_E_ARG;
    }
    BatchWork W;
    W.N = F->n;
    W.nrhs = nrhs;
    const int64_t nv = W.N * nrhs;
    const size_t vb = F->precision == SRW_FP32 ? sizeof(float) : sizeof(double);
    const size_t o_flag = ((2 * nv * vb) + 255) & ~(size_t)255;
    char* ws = nullptr;
    SRW_HIP(hipMallocAsync((void**)&ws, o_flag + 128, s));
    W.r = const_cast<double*>(R);
    W.z = Z;
    W.work = ws;
    W.active = (int*)(ws + o_flag);
    W.err = W.active + 1;
    W.claim = (unsigned long long*)(ws + o_flag + 64);
    W.wait_ticks = wait_ticks(5.0);
    Sched sc{2, RPW * 2, 0};
    if (schedule == 2) {
        sc = Sched{1, RPW, 1};
    } else if (schedule == 0) {
        const Sched t = tuned_schedule(TuneKey{F->n, F->nnz_y, nrhs, F->precision});
        if (t.per_cu) sc = t;
        else if (has_levels) sc = Sched{1, RPW, 1};
    }
    k_zero_n<<<1, 64, 0, s>>>(W.err, 8);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = apply_b(F, W, sc, s);
    int herr[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(herr, W.active, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    const hipError_t fe = hipFreeAsync(ws, s);
    if (e == hipSuccess) e = fe;
    if (e != hipSuccess) {
        set_last_error(hipGetErrorString(e));
        return SRW_E_HIP;
    }
    if (herr[1] != 0) {
        set_last_error("srw_apply_batched: a triangular solve gave up waiting");
        return SRW_E_HIP;
    }
    return SRW_OK;
}

int pcg_batched_impl(srw_factor* F, int32_t nrhs, const double* B, double tol, int32_t max_iter,
                     double* X, int32_t* iters, double* rel, int32_t use_graph, hipStream_t s)
{
    BatchWork W;
    W.N = F->n;
    W.nrhs = nrhs;
    W.nsys = (int64_t)F->nmat * nrhs;
    // reduction tiles: TILE_ROWS rows, never across a matrix boundary
    std::vector<int32_t> tmat;
    std::vector<int64_t> trow, mtile(F->nmat + 1, 0);
    for (int32_t m = 0; m < F->nmat; ++m) {
        mtile[m] = (int64_t)tmat.size();
        for (int64_t r = F->mat_off_host[m]; r < F->mat_off_host[m + 1]; r += TILE_ROWS) {
            tmat.push_back(m);
            trow.push_back(r);
        }
    }
    mtile[F->nmat] = (int64_t)tmat.size();
    trow.push_back(W.N);
    W.ntile = (int64_t)tmat.size();
    const int64_t nv = W.N * nrhs;
    const size_t vb = F->precision == SRW_FP32 ? sizeof(float) : sizeof(double);
    size_t bytes = 0;
    auto take = [&](size_t b) { size_t o = bytes; bytes += (b + 255) & ~(size_t)255; return o; };
    const size_t o_r = take(nv * 8), o_z = take(nv * 8), o_p = take(nv * 8), o_q = take(nv * 8);
    const size_t o_work = take(2 * nv * vb);
    const size_t o_part = take(std::max<int64_t>(W.ntile, 1) * nrhs * 8);
    const size_t o_sys = take(std::max<int64_t>(W.nsys, 1) * sizeof(Sys));
    const size_t o_flag = take(128);
    const size_t o_tm = take(std::max<int64_t>(W.ntile, 1) * 4), o_tr = take((W.ntile + 1) * 8);
    const size_t o_mt = take((F->nmat + 1) * 8);
    char* ws = nullptr;
    SRW_HIP(hipMallocAsync((void**)&ws, bytes, s));
    W.r = (double*)(ws + o_r);
    W.z = (double*)(ws + o_z);
    W.p = (double*)(ws + o_p);
    W.q = (double*)(ws + o_q);
    W.work = ws + o_work;
    W.partials = (double*)(ws + o_part);
    W.sys = (Sys*)(ws + o_sys);
    W.active = (int*)(ws + o_flag);
    W.err = W.active + 1;
    W.claim = (unsigned long long*)(ws + o_flag + 64);
    W.wait_ticks = wait_ticks(5.0);
    int32_t* d_tmat = (int32_t*)(ws + o_tm);
    int64_t* d_trow = (int64_t*)(ws + o_tr);
    W.mat_tile = (int64_t*)(ws + o_mt);
    W.tiles = Tiles{d_tmat, d_trow};
    Sys* host_sys = nullptr;
    int* host_flag = nullptr;
    hipError_t e = hipHostMalloc((void**)&host_sys, std::max<int64_t>(W.nsys, 1) * sizeof(Sys), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&host_flag, 16 * sizeof(int), hipHostMallocDefault);
    if (host_flag) std::memset(host_flag, 0, 16 * sizeof(int));
    Sched tuning{};  // schedule being timed when a solve failed (per_cu 0: not while tuning)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const int sg = (int)((W.nsys + 255) / 256);
    const srw_csr& A = F->Acat;
    auto sync_flags = [&]() -> hipError_t {
        hipError_t ee = hipMemcpyAsync(host_flag, W.active, 8 * sizeof(int), hipMemcpyDeviceToHost, s);
        if (ee == hipSuccess) ee = hipStreamSynchronize(s);
        return ee;
    };
    int status = SRW_OK;
    const char* where = "batched pcg";
    char diag[200] = "";
#define CK(call)                                    \
    do {                                            \
        if (e == hipSuccess) {                      \
            e = (call);                             \
            if (e == hipSuccess) e = hipGetLastError(); \
            if (e != hipSuccess) where = #call;     \
        }                                           \
    } while (0)
    CK(hipMemcpyAsync(d_tmat, tmat.data(), W.ntile * 4, hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(d_trow, trow.data(), (W.ntile + 1) * 8, hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(W.mat_tile, mtile.data(), (F->nmat + 1) * 8, hipMemcpyHostToDevice, s));
    if (e == hipSuccess) {
        k_zero_n<<<1, 64, 0, s>>>(W.err, 8);
        k_zero_d<<<fill_grid(nv), BLOCK, 0, s>>>(nv, X);
        k_copy_d<<<fill_grid(nv), BLOCK, 0, s>>>(nv, B, W.r);
        k_tile<T_BB><<<(unsigned)W.ntile, BLOCK, 0, s>>>(W.tiles, nrhs, nullptr, nullptr, nullptr, B,
                                                         nullptr, nullptr, nullptr, W.sys, W.partials);
        k_bfinal<<<sg, 256, 0, s>>>(W.nsys, nrhs, W.mat_tile, W.partials, W.sys, B_BB, tol, max_iter, W.active);
        e = hipGetLastError();
    }
    // the solve schedule: blocks per CU x slots per claim, timed once per problem shape
    // (rows, factor entries, right-hand sides, precision) and kept for the process
    const TuneKey key{F->n, F->nnz_y, nrhs, F->precision};
    Sched sched = tuned_schedule(key);
    if (e == hipSuccess && sched.per_cu == 0) {
        float best = 1e30f;
        Sched best_s{2, RPW * 2};
        hipEvent_t e0 = nullptr, e1 = nullptr;
        CK(hipEventCreate(&e0));
        CK(hipEventCreate(&e1));
        // level by level first, where the plan has levels; then the sync-free schedules,
        // from the one that was fastest on every batch measured (2 blocks per CU, 16-slot
        // claims): if even that one loses to the level-by-level solve, the rest are not
        // timed
        const bool levels = !F->level_ptr.empty() && F->head == 0;
        CK(apply_b(F, W, best_s, s));  // warm
        if (levels && e == hipSuccess) {
            const Sched cand{1, RPW, 1};
            CK(apply_b(F, W, cand, s));  // warm
            CK(hipEventRecord(e0, s));
            CK(apply_b(F, W, cand, s));
            CK(hipEventRecord(e1, s));
            CK(hipEventSynchronize(e1));
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess) {
                best = ms;
                best_s = cand;
            }
        }
        for (int cap : {2, 1}) {
            for (int chunk : {RPW * 2, RPW * 4, RPW * 8}) {
                if (e != hipSuccess) break;
                const Sched cand{cap, chunk};
                CK(hipEventRecord(e0, s));
                CK(apply_b(F, W, cand, s));
                CK(hipEventRecord(e1, s));
                CK(hipEventSynchronize(e1));
                CK(sync_flags());
                if (e == hipSuccess && host_flag[1] != 0) {
                    tuning = cand;
                    break;
                }
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess && ms < best) {
                    best = ms;
                    best_s = cand;
                }
                if (best_s.level) break;
            }
            if (tuning.per_cu || best_s.level) break;
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        sched = best_s;
        if (e == hipSuccess && !tuning.per_cu) remember_schedule(key, sched, best);
    }
    // a solve that failed while tuning stops the call (reported below)
    const bool stop = host_flag[1] != 0;
    // z = M^{-1} r, p = z, rho = r . z
    if (!stop) CK(apply_b(F, W, sched, s));
    if (e == hipSuccess && !stop) {
        k_bupdate_p<<<grid_for(nv, 256), 256, 0, s>>>(W.N, nrhs, F->node_mat, W.z, W.p, W.sys, 1);
        k_tile<T_DOT><<<(unsigned)W.ntile, BLOCK, 0, s>>>(W.tiles, nrhs, nullptr, nullptr, nullptr, W.r,
                                                          W.z, nullptr, nullptr, W.sys, W.partials);
        k_bfinal<<<sg, 256, 0, s>>>(W.nsys, nrhs, W.mat_tile, W.partials, W.sys, B_RHO0, tol, max_iter, W.active);
        e = hipGetLastError();
    }
    // one iteration captured once, replayed CHUNK times between host checks
    const int CHUNK = 8;
    // captured on a private stream (the caller's may be the null stream, which cannot
    // be captured) and replayed on the caller's stream
    hipStream_t cs = nullptr;
    if (e == hipSuccess && use_graph && !stop) {
        CK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        CK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        if (e == hipSuccess) {
            hipError_t ce = iteration(F, W, sched, X, tol, max_iter, cs);
            hipError_t ee = hipStreamEndCapture(cs, &graph);
            e = ce != hipSuccess ? ce : ee;
        }
        CK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    for (int outer = 0; e == hipSuccess && !stop && outer < 4; ++outer) {
        int done_iters = 0;
        while (e == hipSuccess && done_iters < max_iter) {
            for (int k = 0; k < CHUNK && e == hipSuccess; ++k) {
                if (use_graph) e = hipGraphLaunch(exec, s);
                else e = iteration(F, W, sched, X, tol, max_iter, s);
            }
            done_iters += CHUNK;
            if (e == hipSuccess) e = sync_flags();
            if (e == hipSuccess && (host_flag[1] != 0)) break;  // a solve gave up waiting
            if (e == hipSuccess && host_flag[0] == 0) break;    // every system stopped
        }
        if (e != hipSuccess || host_flag[1] != 0) break;
        // true residuals; systems that miss the tolerance restart from them
        k_zero_i<<<1, 1, 0, s>>>(W.active);
        k_tile<T_RES><<<(unsigned)W.ntile, BLOCK, 0, s>>>(W.tiles, nrhs, A.rowptr, A.col, A.val, B, X,
                                                          W.r, nullptr, W.sys, W.partials);
        k_bfinal<<<sg, 256, 0, s>>>(W.nsys, nrhs, W.mat_tile, W.partials, W.sys, B_TRUE_RR, tol, max_iter, W.active);
        e = hipGetLastError();
        if (e == hipSuccess) e = sync_flags();
        if (e != hipSuccess || host_flag[0] == 0) break;
        CK(apply_b(F, W, sched, s));
        if (e == hipSuccess) {
            k_bupdate_p<<<grid_for(nv, 256), 256, 0, s>>>(W.N, nrhs, F->node_mat, W.z, W.p, W.sys, 1);
            k_tile<T_DOT><<<(unsigned)W.ntile, BLOCK, 0, s>>>(W.tiles, nrhs, nullptr, nullptr, nullptr,
                                                              W.r, W.z, nullptr, nullptr, W.sys, W.partials);
            k_bfinal<<<sg, 256, 0, s>>>(W.nsys, nrhs, W.mat_tile, W.partials, W.sys, B_RHO0, tol, max_iter, W.active);
            e = hipGetLastError();
        }
    }
    CK(hipMemcpyAsync(host_sys, W.sys, W.nsys * sizeof(Sys), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (e == hipSuccess) {
        if (host_flag[1] != 0) {
            e = hipErrorLaunchFailure;  // a triangular solve gave up
            // host_flag[1 + i] = err[i]
            const Sched& at = tuning.per_cu ? tuning : sched;
            std::snprintf(diag, sizeof(diag),
                          "batched %s solve gave up waiting: slot %d for slot %d (value %s), "
                          "%d blocks per CU, %d slots per claim%s",
                          host_flag[3] ? "forward" : "backward", host_flag[4], host_flag[5],
                          host_flag[6] ? "absent" : "present", at.per_cu, host_flag[7],
                          tuning.per_cu ? " (while tuning)" : "");
            where = diag;
        }
        bool all = true;
        for (int64_t i = 0; i < W.nsys; ++i) {
            const Sys& S = host_sys[i];
            const double r = S.bb > 0.0 ? std::sqrt(S.rr) / std::sqrt(S.bb) : 0.0;
            if (iters) iters[i] = S.iters;
            if (rel) rel[i] = r;
            if (!(r <= tol)) all = false;
        }
        if (!all) status = SRW_NOT_CONVERGED;
    }
#undef CK
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
    (void)hipFreeAsync(ws, s);
    (void)hipStreamSynchronize(s);
    if (host_sys) (void)hipHostFree(host_sys);
    if (host_flag) (void)hipHostFree(host_flag);
    if (e != hipSuccess) return hip_fail(e, where);
    return status;
}

}  // namespace srw
