// Solve phase of the hybrid solver (Algorithm 1, "solve"): PCG with the
// preconditioner (Y^T D Y)^{-1} applied by two sync-free triangular solves over the
// slot-ordered solve plan.
//
// Reductions are deterministic: every dot product is summed per block of a fixed
// grid into partials and the partials are added by one block in a fixed order.
// The scalars of the iteration (rho, alpha, beta, ||r||^2) live on the device; the
// host reads ||r||^2 once per iteration for the stopping test.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <cmath>
#include <cstring>

#include "factor.hpp"

namespace srw {

namespace {

constexpr int BLOCK = 256;
constexpr int RED_GRID = 1024;  // blocks of every reducing kernel (grid-stride)

enum Scalar : int { S_RHO = 0, S_PQ, S_ALPHA, S_RR, S_RHO_NEW, S_BETA, S_BB, S_COUNT };
enum Op : int { OP_RHO0 = 0, OP_ALPHA, OP_RR, OP_BETA, OP_BB };

__device__ __forceinline__ double block_sum(double v, double* lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform (scalar)
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BLOCK / 64; ++w) s += lds[w];
    return s;
}

__global__ __launch_bounds__(BLOCK) void k_dot(int64_t n, const double* __restrict__ x,
                                               const double* __restrict__ y, double* partials)
{
    __shared__ double lds[BLOCK / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        s += x[i] * y[i];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(BLOCK) void k_finalize(const double* __restrict__ partials, int np,
                                                    double* sc, int op)
{
    __shared__ double lds[BLOCK / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += BLOCK) s += partials[i];
    s = block_sum(s, lds);
    if (threadIdx.x != 0) return;
    switch (op) {
        case OP_RHO0: sc[S_RHO] = s; break;
        case OP_ALPHA:
            sc[S_PQ] = s;
            sc[S_ALPHA] = sc[S_RHO] / s;
            break;
        case OP_RR: sc[S_RR] = s; break;
        case OP_BETA:
            sc[S_RHO_NEW] = s;
            sc[S_BETA] = s / sc[S_RHO];
            sc[S_RHO] = s;
            break;
        case OP_BB: sc[S_BB] = s; break;
    }
}

// q = A p (one thread per row, entries in CSR order) and partials of p . q
__global__ __launch_bounds__(BLOCK) void k_spmv_dot(int64_t n, const int64_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ p,
                                                    double* __restrict__ q, double* partials)
{
    __shared__ double lds[BLOCK / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        double acc = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) acc += val[e] * p[col[e]];
        q[i] = acc;
        s += p[i] * acc;
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// r = b - A x and partials of r . r
__global__ __launch_bounds__(BLOCK) void k_residual(int64_t n, const int64_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ b,
                                                    double* __restrict__ r, double* partials)
{
    __shared__ double lds[BLOCK / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        double acc = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) acc += val[e] * x[col[e]];
        const double ri = b[i] - acc;
        r[i] = ri;
        s += ri * ri;
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// x += alpha p, r -= alpha q, partials of r . r
__global__ __launch_bounds__(BLOCK) void k_update_xr(int64_t n, double* __restrict__ x,
                                                     double* __restrict__ r,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ q,
                                                     const double* __restrict__ sc,
                                                     double* partials)
{
    __shared__ double lds[BLOCK / 64];
    const double alpha = sc[S_ALPHA];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        x[i] = x[i] + alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        s += ri * ri;
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// p = z + beta p (beta = 0 with a null scalar pointer: p = z)
__global__ __launch_bounds__(BLOCK) void k_update_p(int64_t n, const double* __restrict__ z,
                                                    double* __restrict__ p,
                                                    const double* __restrict__ sc)
{
    const double beta = sc ? sc[S_BETA] : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        p[i] = sc ? z[i] + beta * p[i] : z[i];
}

__global__ __launch_bounds__(BLOCK) void k_copy(int64_t n, const double* __restrict__ a,
                                                double* __restrict__ b)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        b[i] = a[i];
}

// ----------------------------------------------------------- triangular solves
// Both substitutions run over the solve plan: the rows of Y (and of Y^T) stored by
// slot -- the position of the row in a topological order of Y z = v, increasing
// (level, rank) or increasing rank -- with every column replaced by its slot, so a
// row only depends on smaller slots going forward and on larger slots going backward.
//   backward  (Y^T w = r):   w_s = r_node(s) - sum_q Yt_sq w_q     (slots descending)
//   forward   (Y z = v):     z_s = w_s / D_s - sum_q Y_sq z_q       (slots ascending)
// A cooperative launch keeps every wave of the grid resident, and wave i takes the
// rows i, i + W, i + 2W, ... of the order (W waves): no counter is shared.  The wave
// that holds the first unfinished row has finished all its earlier rows and that
// row's dependencies are all done, so the solve always progresses.  The solution
// starts filled with a signalling-NaN pattern that arithmetic never produces; a
// row's value is published with one device-scope store and is its own ready flag.
// A waiting wave polls one address only -- that of its missing dependency which the
// order solves last -- and once that one is there reloads its other missing values,
// if any.
// The lane partial sums are added by a wave-wide butterfly, so the result does not
// depend on timing.
template <typename T>
struct Bits;
template <>
struct Bits<double> {
    using U = unsigned long long;
    static constexpr U sentinel = 0x7FF4DEADBEEF5A5Aull;
    static __device__ U nan_bits() { return 0x7FF8000000000000ull; }  // quiet NaN
};
template <>
struct Bits<float> {
    using U = unsigned int;
    static constexpr U sentinel = 0x7FA5A5A5u;
    static __device__ U nan_bits() { return 0x7FC00000u; }  // quiet NaN
};
template <>
struct Bits<int32_t> {
    using U = unsigned int;
    static constexpr U sentinel = 0xFFFFFFFFu;  // level -1: not yet known
    static __device__ U nan_bits() { return 0u; }
};

// A wait longer than wait_ticks of the wall clock marks the solve failed and proceeds
// with a NaN; the caller then reports the failure.  The limit guards against a defect
// (a wave waits at most for the chain of slots before its own); it is seconds, far
// above any legitimate wait.

#ifndef SRW_POLL_SLEEP
#define SRW_POLL_SLEEP 2  // s_sleep units (64 clocks) between polls of a missing value
#endif

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fill_sentinel(int64_t n, T* x)
{
    using U = typename Bits<T>::U;
    const int64_t i0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * BLOCK) ((U*)x)[i] = Bits<T>::sentinel;
}

__device__ __forceinline__ int wave_max_i32(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

template <typename U>
__device__ __forceinline__ U load_published(const U* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until no valid lane holds the sentinel in `bits` (each lane's value of slot
// c).  LATE_HIGH: the order solves higher slots later (forward), else lower slots.
// A wait that gives up raises *err and leaves a NaN in the missing lanes.
template <typename T, bool LATE_HIGH>
__device__ __forceinline__ void wait_published(typename Bits<T>::U& bits, const int32_t c,
                                               const bool valid, const T* sol, int* err,
                                               int64_t ticks)
{
    using U = typename Bits<T>::U;
    const int lane = threadIdx.x & 63;
    uint64_t miss = ballot(valid && bits == Bits<T>::sentinel);
    uint32_t spins = 0;
    const int64_t t0 = miss ? wall_clock64() : 0;
    while (miss != 0) {
        // every 256 polls: give up past the time limit, or at once when another wave
        // already gave up (a failed solve then drains instead of waiting at every row)
        bool give_up = false;
        if ((++spins & 255u) == 0)
            give_up = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                      wall_clock64() - t0 > ticks;
        if (give_up) {
            if (lane == 0) atomicOr(err, 1);
            if ((miss >> lane) & 1ull) bits = Bits<T>::nan_bits();
            break;
        }
        const bool mine = (miss >> lane) & 1ull;
        const int key = wave_max_i32(mine ? (LATE_HIGH ? c : -c) : INT_MIN);
        const int32_t lead = LATE_HIGH ? key : -key;
        const U lb = load_published((const U*)sol + lead);  // one address for the wave
        if (lb == Bits<T>::sentinel) {
            __builtin_amdgcn_s_sleep(SRW_POLL_SLEEP);
            continue;
        }
        // the lead's lane takes the polled value; only the other missing lanes reload
        // (often there are none, and the row goes on without another round trip)
        if (mine && c == lead) bits = lb;
        const bool other = mine && c != lead;
        if (ballot(other) != 0 && other) bits = load_published((const U*)sol + c);
        miss = ballot(valid && bits == Bits<T>::sentinel);
    }
}

// The substitution covers the slots h..n-1 (the first h slots are the dense head, done
// by the head kernels: before the forward rows, after the backward ones).
template <typename T, bool FWD>
__global__ __launch_bounds__(BLOCK) void k_trsv(int64_t n, int64_t h, const int64_t* __restrict__ ptr,
                                                const int32_t* __restrict__ col,
                                                const T* __restrict__ val,
                                                const T* __restrict__ dslot,
                                                const int32_t* __restrict__ slot_node,
                                                const double* __restrict__ rhs,
                                                const T* __restrict__ w, T* sol,
                                                double* __restrict__ out, int* err,
                                                int64_t ticks)
{
    using U = typename Bits<T>::U;
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (BLOCK / 64);
    const int64_t wid =
        (int64_t)blockIdx.x * (BLOCK / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t m = n - h;  // rows substituted
    if (wid >= m) return;  // whole wave
    // the wave's next row, loaded one row ahead: bounds and first 64 entries
    int64_t s = FWD ? h + wid : n - 1 - wid;
    int64_t q0 = ptr[s], q1 = ptr[s + 1];
    int32_t c = 0;
    T v = T(0);
    if (q0 + lane < q1) {
        c = col[q0 + lane];
        v = val[q0 + lane];
    }
    for (int64_t i = wid; i < m; i += nw) {
        const bool valid = q0 + lane < q1;
        U bits = valid ? load_published((const U*)sol + c) : U(0);
        const int32_t node = slot_node[s];
        const T base = FWD ? w[s] / dslot[s] : (T)rhs[node];
        const int64_t i2 = i + nw;
        int64_t s2 = 0, p0 = 0, p1 = 0;
        int32_t c2 = 0;
        T v2 = T(0);
        if (i2 < m) {
            s2 = FWD ? h + i2 : n - 1 - i2;
            p0 = ptr[s2];
            p1 = ptr[s2 + 1];
            if (p0 + lane < p1) {
                c2 = col[p0 + lane];
                v2 = val[p0 + lane];
            }
        }
        wait_published<T, FWD>(bits, c, valid, sol, err, ticks);
        T acc = v * __builtin_bit_cast(T, bits);
        for (int64_t qb = q0 + 64; qb < q1; qb += 64) {  // rows longer than 64 entries
            const int64_t q = qb + lane;
            const bool ok = q < q1;
            const int32_t cc = ok ? col[q] : 0;
            const T vv = ok ? val[q] : T(0);
            U bb = ok ? load_published((const U*)sol + cc) : U(0);
            wait_published<T, FWD>(bb, cc, ok, sol, err, ticks);
            acc += vv * __builtin_bit_cast(T, bb);
        }
        acc = wave_sum(acc);
        if (lane == 0) {
            const T x = base - acc;
            __hip_atomic_store((U*)sol + s, __builtin_bit_cast(U, x), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            if (out) out[node] = (double)x;
        }
        s = s2;
        q0 = p0;
        q1 = p1;
        c = c2;
        v = v2;
    }
}

// Dependency level of every slot over the forward plan: lev_s = 1 + the largest
// level among the row's columns, 0 for an empty row; the same scheme as k_trsv.  The
// waves take the slots order[0], order[1], ... in turn (slot order when order is
// NULL); every slot's columns precede it in that sequence.
// Each wave keeps the largest level it met; one atomic per wave gives the depth.
__global__ __launch_bounds__(BLOCK) void k_levels(int64_t n, const int32_t* __restrict__ order,
                                                  const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col, int32_t* lev,
                                                  int* depth, int* err, int64_t ticks)
{
    using U = Bits<int32_t>::U;
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (BLOCK / 64);
    const int64_t wid =
        (int64_t)blockIdx.x * (BLOCK / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int wmax = 0;
    for (int64_t i = wid; i < n; i += nw) {
        const int64_t s = order ? (int64_t)order[i] : i;
        int m = -1;
        for (int64_t qb = ptr[s]; qb < ptr[s + 1]; qb += 64) {
            const int64_t q = qb + lane;
            const bool ok = q < ptr[s + 1];
            const int32_t c = ok ? col[q] : 0;
            U bits = ok ? load_published((const U*)lev + c) : U(0);
            wait_published<int32_t, true>(bits, c, ok, lev, err, ticks);
            if (ok) m = max(m, (int)bits);
        }
        m = wave_max_i32(m) + 1;
        wmax = max(wmax, m + 1);
        if (lane == 0)
            __hip_atomic_store((U*)lev + s, (U)m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0 && wid < n) atomicMax(depth, wmax);
}

// ----------------------------------------------------------------- dense head
// The lowest-ranked rows carry most of the dependency chain (their walks end at one
// another): at 128^3 the first 4,096 ranks hold 402 of the 1,147 levels.  Those rows
// are solved with X, the inverse of their diagonal block of Y (unit lower triangular),
// by two dense products per application instead of level by level.
//   backward:  c_i = r_node(i) - sum over the row's Y^T entries on slots >= h of w,
//              w_head = X^T c
//   forward:   z_head = X (w_head / D_head)
// X is packed by rows (row i: X[i][0..i] at i(i+1)/2); X^T packed by rows too (row j:
// X[j..h-1][j] at j h - j(j-1)/2).
__host__ __device__ __forceinline__ int64_t head_roff(int64_t i) { return i * (i + 1) / 2; }
__host__ __device__ __forceinline__ int64_t head_toff(int64_t j, int64_t h)
{
    return j * h - j * (j - 1) / 2;
}

// X[i][j] = [i == j] - sum over the entries q of row i of Y: Y_iq X[q][j] (Y X = I).
// W consecutive columns of X are one workgroup's: it takes the rows c0..h-1 (the rows
// above are zero on these columns) in increasing order, dealt to its waves in turn,
// and keeps the columns' values of those rows in LDS.  A row waits for its dependency
// rows through flags in LDS; they are rows of the same workgroup, finished by waves
// that are all resident and take their rows in increasing order, so the lowest
// unfinished row can always finish.  The workgroups never wait for one another.
// A row's entries are summed lane by lane (64 at a time) and then across the wave by
// a butterfly: a fixed order.
constexpr int HINV_WAVES = 16;  // waves of a workgroup

template <typename T, int W>
__global__ __launch_bounds__(64 * HINV_WAVES) void k_head_inverse(int64_t h,
                                                                 const int64_t* __restrict__ ptr,
                                                                 const int32_t* __restrict__ col,
                                                                 const T* __restrict__ val, T* X,
                                                                 int* err, int64_t ticks)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int64_t c0 = (int64_t)W * blockIdx.x;
    const int64_t rows = h - c0;
    unsigned int* done = (unsigned int*)lds;              // bit r: row c0 + r finished
    const int64_t nwords = (rows + 31) / 32;
    T* xv = (T*)(lds + ((nwords * 4 + 15) & ~(int64_t)15));  // [rows][W]
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    for (int64_t k = threadIdx.x; k < nwords; k += blockDim.x) done[k] = 0u;
    __syncthreads();
    const int64_t t0 = wall_clock64();
    bool failed = false;
    for (int64_t i = c0 + wv; i < h; i += HINV_WAVES) {
        T acc[W];
#pragma unroll
        for (int k = 0; k < W; ++k) acc[k] = T(0);
        const int64_t q1 = ptr[i + 1];
        for (int64_t qb = ptr[i]; qb < q1; qb += 64) {
            const bool has = qb + lane < q1;
            const int32_t q = has ? col[qb + lane] : -1;
            const bool dep = q >= c0;  // rows below c0 are zero on these columns
            const int64_t r = dep ? (int64_t)q - c0 : 0;
            uint32_t spins = 0;
            while (ballot(dep && !failed &&
                          ((__hip_atomic_load(&done[r >> 5], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP) >> (r & 31)) & 1u) == 0u) != 0) {
                if ((++spins & 255u) == 0 && wall_clock64() - t0 > ticks) {
                    if (lane == 0) atomicOr(err, 1);
                    failed = true;  // finishes with what is there; the build fails
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            if (dep) {
                const T y = val[qb + lane];
#pragma unroll
                for (int k = 0; k < W; ++k) acc[k] = acc[k] + y * xv[r * W + k];
            }
        }
        T x[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int64_t j = c0 + k;
            const T sk = wave_sum(acc[k]);
            x[k] = j > i ? T(0) : (j == i ? T(1) : T(0)) - sk;
        }
        if (lane < W) {
            T mine = x[0];
#pragma unroll
            for (int k = 1; k < W; ++k) mine = lane == k ? x[k] : mine;
            const int64_t j = c0 + lane;
            xv[(i - c0) * W + lane] = mine;
            if (j <= i) X[head_roff(i) + j] = mine;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) atomicOr(&done[(i - c0) >> 5], 1u << ((i - c0) & 31));
    }
}

// LDS bytes of the workgroup that starts at column c0 (the first is the largest).
__host__ __device__ inline size_t head_inverse_lds(int64_t h, int W)
{
    const int64_t words = (h + 31) / 32;
    return (size_t)((words * 4 + 15) & ~(int64_t)15) + (size_t)h * W * 8;
}

// X^T from X through 64 x 64 tiles in LDS; one workgroup per tile (I, J), J <= I.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_head_transpose(int64_t h, const T* __restrict__ X,
                                                          T* __restrict__ XT)
{
    __shared__ T tile[64][65];
    int64_t b = blockIdx.x, I = 0;
    while ((I + 1) * (I + 2) / 2 <= b) ++I;  // tile row: the last I with I(I+1)/2 <= b
    const int64_t J = b - I * (I + 1) / 2;
    for (int k = threadIdx.x; k < 64 * 64; k += BLOCK) {
        const int r = k >> 6, c = k & 63;
        const int64_t i = 64 * I + r, j = 64 * J + c;
        tile[r][c] = (i < h && j <= i) ? X[head_roff(i) + j] : T(0);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 64 * 64; k += BLOCK) {
        const int c = k >> 6, r = k & 63;  // consecutive threads: consecutive i
        const int64_t i = 64 * I + r, j = 64 * J + c;
        if (i < h && j <= i) XT[head_toff(j, h) + (i - j)] = tile[r][c];
    }
}

// c_i (into c) for the head slots: one wave per slot.  w holds the backward solution
// on the slots >= h.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_head_rhs(int64_t h, const int64_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col,
                                                    const T* __restrict__ val,
                                                    const int32_t* __restrict__ slot_node,
                                                    const double* __restrict__ rhs,
                                                    const T* __restrict__ w, T* __restrict__ c)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    if (i >= h) return;  // whole wave
    T acc = T(0);
    for (int64_t q = ptr[i] + lane; q < ptr[i + 1]; q += 64) {
        const int32_t k = col[q];
        if (k >= h) acc += val[q] * w[k];
    }
    acc = wave_sum(acc);
    if (lane == 0) c[i] = (T)rhs[slot_node[i]] - acc;
}

// One wave per row r of the packed matrix M: FWD, row r of X times (w / D) over the
// head; otherwise row r of X^T times c[r..h-1].  Results to y (and by node to out).
template <typename T, bool FWD>
__global__ __launch_bounds__(BLOCK) void k_head_mv(int64_t h, const T* __restrict__ M,
                                                   const T* __restrict__ v,
                                                   const T* __restrict__ dslot,
                                                   const int32_t* __restrict__ slot_node,
                                                   T* __restrict__ y, double* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    if (r >= h) return;  // whole wave
    const T* row = M + (FWD ? head_roff(r) : head_toff(r, h));
    const int64_t len = FWD ? r + 1 : h - r;
    T acc = T(0);
    for (int64_t k = lane; k < len; k += 64)
        acc += row[k] * (FWD ? v[k] / dslot[k] : v[r + k]);
    acc = wave_sum(acc);
    if (lane == 0) {
        y[r] = acc;
        if (FWD && out) out[slot_node[r]] = (double)acc;
    }
}

// Grid of a cooperative launch: every block resident at once (occupancy x CUs),
// capped at the blocks the work can use.
template <typename K>
hipError_t coop_launch(K kernel, int64_t rows, void** args, hipStream_t s)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, BLOCK, 0);
    if (e != hipSuccess) return e;
    // The waits need every wave resident at once.  The runtime's occupancy is not
    // always met in full (a kernel reported at 8 workgroups per CU was measured running
    // 7 together), so the grid leaves one workgroup in eight unused.
    int64_t blocks = (int64_t)cus * std::max(1, per_cu * 7 / 8);
    blocks = std::min<int64_t>(blocks, (rows + BLOCK / 64 - 1) / (BLOCK / 64));
    if (blocks < 1) blocks = 1;
    return hipLaunchCooperativeKernel((const void*)kernel, dim3((unsigned)blocks), dim3(BLOCK),
                                      args, 0, s);
}

int fill_grid(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>(grid_for(n, BLOCK), 1), 2048); }

// work, sol: n values of T each; z (node order) receives the result as doubles.
template <typename T>
hipError_t apply_plan(const srw_factor* F, const double* r, T* work, T* sol, double* z, int* err,
                      hipStream_t s)
{
    int64_t n = F->n;
    int64_t h = F->head;
    int64_t ticks = wait_ticks(5.0);
    k_fill_sentinel<T><<<fill_grid(n), BLOCK, 0, s>>>(n, work);
    k_fill_sentinel<T><<<fill_grid(n), BLOCK, 0, s>>>(n, sol);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned hg = (unsigned)((h + BLOCK / 64 - 1) / (BLOCK / 64));
    if (n > h) {
        const int64_t* ptr = F->bptr;
        const int32_t* col = F->bcol;
        const T* val = (const T*)F->bval;
        const T* dslot = nullptr;
        const int32_t* slot_node = F->slot_node;
        const double* rhs = r;
        const T* w = nullptr;
        T* out_sol = work;
        double* out = nullptr;
        void* args[] = {&n, &h, &ptr, &col, &val, &dslot, &slot_node, &rhs, &w, &out_sol, &out, &err,
                        &ticks};
        e = coop_launch(k_trsv<T, false>, n - h, args, s);
        if (e != hipSuccess) return e;
    }
    if (h > 0) {
        // backward head (c in sol's head slots, then w_head), forward head
        k_head_rhs<T><<<hg, BLOCK, 0, s>>>(h, F->bptr, F->bcol, (const T*)F->bval, F->slot_node, r,
                                           work, sol);
        k_head_mv<T, false><<<hg, BLOCK, 0, s>>>(h, (const T*)F->hxt, sol, nullptr, nullptr, work,
                                                 nullptr);
        k_head_mv<T, true><<<hg, BLOCK, 0, s>>>(h, (const T*)F->hx, work, (const T*)F->dslot,
                                                F->slot_node, sol, z);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (n > h) {
        const int64_t* ptr = F->fptr;
        const int32_t* col = F->fcol;
        const T* val = (const T*)F->fval;
        const T* dslot = (const T*)F->dslot;
        const int32_t* slot_node = F->slot_node;
        const double* rhs = nullptr;
        const T* w = work;
        T* out_sol = sol;
        double* out = z;
        void* args[] = {&n, &h, &ptr, &col, &val, &dslot, &slot_node, &rhs, &w, &out_sol, &out, &err,
                        &ticks};
        e = coop_launch(k_trsv<T, true>, n - h, args, s);
    }
    return e;
}

// Two-game factor (Section 7.1): the backward solve runs over the plan of the game of
// A^T (its Y^T by slot) and writes its result by node into z; the result is gathered
// into the slot order of the game of A, whose forward solve (with D) finishes in z.
template <typename T>
__global__ void k_gather_slots(int64_t n, const int32_t* __restrict__ slot_node,
                               const double* __restrict__ x, T* __restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        y[i] = (T)x[slot_node[i]];
}

template <typename T>
hipError_t apply_ldu_plan(const srw_factor* F, const double* r, T* work, T* sol, double* z,
                          int* err, hipStream_t s)
{
    const srw_factor* G = F->tgame;
    int64_t n = F->n;
    int64_t h = 0;  // the games' factors take no dense head
    int64_t ticks = wait_ticks(5.0);
    k_fill_sentinel<T><<<fill_grid(n), BLOCK, 0, s>>>(n, work);
    k_fill_sentinel<T><<<fill_grid(n), BLOCK, 0, s>>>(n, sol);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        const int64_t* ptr = G->bptr;
        const int32_t* col = G->bcol;
        const T* val = (const T*)G->bval;
        const T* dslot = nullptr;
        const int32_t* slot_node = G->slot_node;
        const double* rhs = r;
        const T* w = nullptr;
        T* out_sol = work;
        double* out = z;
        void* args[] = {&n, &h, &ptr, &col, &val, &dslot, &slot_node, &rhs, &w, &out_sol, &out, &err,
                        &ticks};
        e = coop_launch(k_trsv<T, false>, n, args, s);
        if (e != hipSuccess) return e;
    }
    k_gather_slots<T><<<fill_grid(n), BLOCK, 0, s>>>(n, F->slot_node, z, work);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        const int64_t* ptr = F->fptr;
        const int32_t* col = F->fcol;
        const T* val = (const T*)F->fval;
        const T* dslot = (const T*)F->dslot;
        const int32_t* slot_node = F->slot_node;
        const double* rhs = nullptr;
        const T* w = work;
        T* out_sol = sol;
        double* out = z;
        void* args[] = {&n, &h, &ptr, &col, &val, &dslot, &slot_node, &rhs, &w, &out_sol, &out, &err,
                        &ticks};
        e = coop_launch(k_trsv<T, true>, n, args, s);
    }
    return e;
}

// work: 2 n doubles of scratch; err: one int (0 on entry).
hipError_t apply_any(const srw_factor* F, const double* r, void* work, double* z, int* err,
                     hipStream_t s)
{
    if (F->n == 0) return hipSuccess;
    if (F->tgame) {
        if (F->precision == SRW_FP32) {
            float* w = (float*)work;
            return apply_ldu_plan<float>(F, r, w, w + F->n, z, err, s);
        }
        double* w = (double*)work;
        return apply_ldu_plan<double>(F, r, w, w + F->n, z, err, s);
    }
    if (F->precision == SRW_FP32) {
        float* w = (float*)work;
        return apply_plan<float>(F, r, w, w + F->n, z, err, s);
    }
    double* w = (double*)work;
    return apply_plan<double>(F, r, w, w + F->n, z, err, s);
}

int red_grid(int64_t n)
{
    const int64_t g = (n + BLOCK - 1) / BLOCK;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, RED_GRID));
}

}  // namespace

int64_t wait_ticks(double seconds)
{
    static std::atomic<int> rate_khz[64];  // per device, 0 = not read yet
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    int khz = rate_khz[dev].load(std::memory_order_relaxed);
    if (khz == 0) {
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
            khz = 100000;  // the 100 MHz clock of this device family
        rate_khz[dev].store(khz, std::memory_order_relaxed);
    }
    return (int64_t)(seconds * 1000.0 * (double)khz);
}

int64_t head_rows_fit(int64_t h)
{
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    while (h > 0 && head_inverse_lds(h, 1) > (size_t)lds_max) h -= 64;
    return h > 0 ? h : 0;
}

hipError_t head_inverse_launch(const srw_factor* F, int* err, hipStream_t s)
{
    int64_t h = F->head;
    if (h <= 0) return hipSuccess;
    int64_t ticks = wait_ticks(10.0);
    hipError_t e = hipMemsetAsync(err, 0, sizeof(int), s);
    if (e != hipSuccess) return e;
    int dev = 0, lds_max = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) !=
        hipSuccess)
        return e;
    // the widest column group whose rows fit in one workgroup's LDS (sized for doubles)
    int W = 0;
    for (int w : {4, 2, 1})
        if (!W && head_inverse_lds(h, w) <= (size_t)lds_max) W = w;
    if (!W) return hipErrorInvalidValue;  // head_rows is capped so that one column fits
    const unsigned groups = (unsigned)((h + W - 1) / W);
    const size_t lds = head_inverse_lds(h, W);
    const int64_t nb = (h + 63) / 64;  // tile rows of the transpose
    const unsigned tiles = (unsigned)(nb * (nb + 1) / 2);
#define HEAD_INV(T, WW)                                                                            \
    do {                                                                                           \
        e = hipFuncSetAttribute((const void*)k_head_inverse<T, WW>,                               \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);            \
        if (e != hipSuccess) return e;                                                             \
        k_head_inverse<T, WW><<<groups, 64 * HINV_WAVES, lds, s>>>(                                \
            h, F->fptr, F->fcol, (const T*)F->fval, (T*)F->hx, err, ticks);                         \
    } while (0)
    if (F->precision == SRW_FP32) {
        if (W == 4) HEAD_INV(float, 4);
        else if (W == 2) HEAD_INV(float, 2);
        else HEAD_INV(float, 1);
        k_head_transpose<float><<<tiles, BLOCK, 0, s>>>(h, (const float*)F->hx, (float*)F->hxt);
    } else {
        if (W == 4) HEAD_INV(double, 4);
        else if (W == 2) HEAD_INV(double, 2);
        else HEAD_INV(double, 1);
        k_head_transpose<double><<<tiles, BLOCK, 0, s>>>(h, (const double*)F->hx, (double*)F->hxt);
    }
#undef HEAD_INV
    return hipGetLastError();
}

hipError_t apply_factor(const srw_factor* F, const double* r, void* work, double* z, int* err,
                        hipStream_t s)
{
    return apply_any(F, r, work, z, err, s);
}

int apply_impl(srw_factor* F, const double* r, double* z, hipStream_t s)
{
    const int64_t n = F->n;
    char* ws = nullptr;
    const size_t vec = (size_t)std::max<int64_t>(n, 1);
    SRW_HIP(hipMallocAsync((void**)&ws, 2 * vec * sizeof(double) + 64, s));
    int* err = (int*)(ws + 2 * vec * sizeof(double));
    hipError_t e = hipMemsetAsync(err, 0, sizeof(int), s);
    if (e == hipSuccess) e = apply_any(F, r, ws, z, err, s);
    int herr = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(ws, s);
    (void)hipStreamSynchronize(s);
    SRW_HIP(e);
    return herr ? SRW_E_HIP : SRW_OK;
}

// ------------------------------------------------------ allocation-free application
// Scratch of srw_apply_noalloc: the two work vectors of the triangular solves (up to
// SRW_NOALLOC_MAX_N values each, FP64 or FP32) and the solves' failure flag.  One copy
// per device, held until the process ends; every call on a device shares it.
constexpr size_t NOALLOC_WORK_BYTES = 2 * (size_t)SRW_NOALLOC_MAX_N * sizeof(double);
static __device__ __align__(256) unsigned char scratch[NOALLOC_WORK_BYTES + 256];

namespace {

// The device address of `scratch` on each device, looked up once per device with that
// device current (the array's name in host code is a host-side stand-in, not a device
// address).
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

hipError_t scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

__global__ void k_clear_flag(int* f) { *f = 0; }

}  // namespace

int apply_noalloc_impl(const srw_factor* F, const double* r, double* z, hipStream_t s)
{
    if (F->n > (int64_t)SRW_NOALLOC_MAX_N) {
        set_last_error("srw_apply_noalloc: the factor has more rows than SRW_NOALLOC_MAX_N");
        return SRW_E_ARG;
    }
    void* base = nullptr;
    SRW_HIP(scratch_address(&base));
    char* work = (char*)base;
    int* err = (int*)(work + NOALLOC_WORK_BYTES);
    k_clear_flag<<<1, 1, 0, s>>>(err);  // a kernel, not a memset
    SRW_HIP(hipGetLastError());
    SRW_HIP(apply_any(F, r, work, z, err, s));
    int herr = 0;
    SRW_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    SRW_HIP(hipStreamSynchronize(s));
    if (herr) {
        set_last_error("srw_apply_noalloc: a triangular solve gave up waiting");
        return SRW_E_HIP;
    }
    return SRW_OK;
}

int dag_levels(srw_factor* F, int32_t* lev, int32_t* depth_out, hipStream_t s,
               const int32_t* order)
{
    int64_t n = F->n;
    *depth_out = 0;
    if (n == 0) return SRW_OK;
    char* ws = nullptr;
    SRW_HIP(hipMallocAsync((void**)&ws, 64, s));
    int* depth = (int*)ws;
    int* err = depth + 1;
    hipError_t e = hipMemsetAsync(depth, 0, 2 * sizeof(int), s);
    if (e == hipSuccess) {
        k_fill_sentinel<int32_t><<<fill_grid(n), BLOCK, 0, s>>>(n, lev);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        const int64_t* ptr = F->fptr;
        const int32_t* col = F->fcol;
        int64_t ticks = wait_ticks(5.0);
        void* args[] = {&n, &order, &ptr, &col, &lev, &depth, &err, &ticks};
        e = coop_launch(k_levels, n, args, s);
    }
    int host[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(host, depth, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(ws, s);
    (void)hipStreamSynchronize(s);
    SRW_HIP(e);
    if (host[1]) return SRW_E_HIP;
    *depth_out = host[0];
    return SRW_OK;
}

int dag_depth(srw_factor* F, int32_t* depth_out, hipStream_t s)
{
    const int64_t n = F->n;
    *depth_out = 0;
    if (n == 0) return SRW_OK;
    int32_t* lev = nullptr;
    SRW_HIP(hipMallocAsync((void**)&lev, n * sizeof(int32_t), s));
    const int st = dag_levels(F, lev, depth_out, s);
    (void)hipFreeAsync(lev, s);
    (void)hipStreamSynchronize(s);
    return st;
}

int pcg_impl(const srw_csr* A, srw_factor* F, const double* b, double tol, int32_t max_iter,
             double* x, int32_t* iters_out, double* rel_out, hipStream_t s)
{
    const int64_t n = A->n;
    const int rg = red_grid(n);
    const int eg = rg;  // elementwise kernels share the fixed grid
    double* ws = nullptr;
    double* host = nullptr;
    const size_t vec = (size_t)std::max<int64_t>(n, 1);
    SRW_HIP(hipMallocAsync((void**)&ws, (6 * vec + RED_GRID + S_COUNT + 4) * sizeof(double), s));
    double *r = ws, *z = ws + vec, *p = ws + 2 * vec, *q = ws + 3 * vec, *work = ws + 4 * vec;
    double* partials = ws + 6 * vec;
    double* sc = partials + RED_GRID;
    int* err = (int*)(sc + S_COUNT);
    host = host_scratch() ? (double*)(host_scratch() + 8) : nullptr;
    hipError_t herr = host ? hipSuccess : hipErrorOutOfMemory;
    if (herr != hipSuccess) {
        (void)hipFreeAsync(ws, s);
        return hip_fail(herr, "hipHostMalloc");
    }
    int status = SRW_NOT_CONVERGED;
    bool gave_up = false;
    int32_t it = 0;
    double rel = 0.0;
    hipError_t e = hipSuccess;
    auto solve_failed = [&]() -> bool {
        int herr = 0;
        if (hipMemcpyAsync(host + 1, err, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return true;
        std::memcpy(&herr, host + 1, sizeof(int));
        return herr != 0;
    };
    auto read_scalar = [&](int idx, double* outv) -> hipError_t {
        hipError_t ee = hipMemcpyAsync(host, sc + idx, sizeof(double), hipMemcpyDeviceToHost, s);
        if (ee != hipSuccess) return ee;
        ee = hipStreamSynchronize(s);
        *outv = host[0];
        return ee;
    };
#define STEP(call)                      \
    do {                                \
        call;                           \
        e = hipGetLastError();          \
        if (e != hipSuccess) goto out;  \
    } while (0)
    {
        STEP(e = hipMemsetAsync(x, 0, vec * sizeof(double), s));
        STEP(e = hipMemsetAsync(err, 0, sizeof(int), s));
        STEP((k_dot<<<rg, BLOCK, 0, s>>>(n, b, b, partials)));
        STEP((k_finalize<<<1, BLOCK, 0, s>>>(partials, rg, sc, OP_BB)));
        double bb = 0.0;
        if ((e = read_scalar(S_BB, &bb)) != hipSuccess) goto out;
        const double bnorm = std::sqrt(bb);
        if (bnorm == 0.0) {
            status = SRW_OK;
            goto out;
        }
        STEP((k_copy<<<eg, BLOCK, 0, s>>>(n, b, r)));
        STEP(e = apply_any(F, r, work, z, err, s));
        STEP((k_update_p<<<eg, BLOCK, 0, s>>>(n, z, p, nullptr)));
        STEP((k_dot<<<rg, BLOCK, 0, s>>>(n, r, z, partials)));
        STEP((k_finalize<<<1, BLOCK, 0, s>>>(partials, rg, sc, OP_RHO0)));
        while (it < max_iter) {
            STEP((k_spmv_dot<<<rg, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, p, q, partials)));
            STEP((k_finalize<<<1, BLOCK, 0, s>>>(partials, rg, sc, OP_ALPHA)));
            STEP((k_update_xr<<<rg, BLOCK, 0, s>>>(n, x, r, p, q, sc, partials)));
            STEP((k_finalize<<<1, BLOCK, 0, s>>>(partials, rg, sc, OP_RR)));
            ++it;
            double rr = 0.0;
            if ((e = read_scalar(S_RR, &rr)) != hipSuccess) goto out;
            if (!std::isfinite(rr) || solve_failed()) {
                e = hipErrorLaunchFailure;  // a triangular solve gave up waiting
                gave_up = true;
                goto out;
            }
            if (std::sqrt(rr) <= tol * bnorm) {
                STEP((k_residual<<<rg, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, x, b, r, partials)));
                STEP((k_finalize<<<1, BLOCK, 0, s>>>(partials, rg, sc, OP_RR)));
                if ((e = read_scalar(S_RR, &rr)) != hipSuccess) goto out;
                if (std::sqrt(rr) <= tol * bnorm) {
                    status = SRW_OK;
                    break;
                }
                // restart from the true residual
                STEP(e = apply_any(F, r, work, z, err, s));
                STEP((k_update_p<<<eg, BLOCK, 0, s>>>(n, z, p, nullptr)));
                STEP((k_dot<<<rg, BLOCK, 0, s>>>(n, r, z, partials)));
                STEP((k_finalize<<<1, BLOCK, 0, s>>>(partials, rg, sc, OP_RHO0)));
                continue;
            }
            STEP(e = apply_any(F, r, work, z, err, s));
            STEP((k_dot<<<rg, BLOCK, 0, s>>>(n, r, z, partials)));
            STEP((k_finalize<<<1, BLOCK, 0, s>>>(partials, rg, sc, OP_BETA)));
            STEP((k_update_p<<<eg, BLOCK, 0, s>>>(n, z, p, sc)));
        }
        // true relative residual of the returned iterate
        STEP((k_residual<<<rg, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, x, b, r, partials)));
        STEP((k_finalize<<<1, BLOCK, 0, s>>>(partials, rg, sc, OP_RR)));
        double rr = 0.0;
        if ((e = read_scalar(S_RR, &rr)) != hipSuccess) goto out;
        rel = std::sqrt(rr) / bnorm;
        int herr = 0;
        if ((e = hipMemcpyAsync(host, err, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) goto out;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) goto out;
        std::memcpy(&herr, host, sizeof(int));
        if (herr) e = hipErrorLaunchFailure;
    }
out:
#undef STEP
    (void)hipFreeAsync(ws, s);
    (void)hipStreamSynchronize(s);
    if (gave_up) {
        set_last_error("pcg: a triangular solve gave up waiting, or the residual is not finite");
        return SRW_E_HIP;
    }
    if (e != hipSuccess) return hip_fail(e, "pcg");
    if (iters_out) *iters_out = it;
    if (rel_out) *rel_out = rel;
    return status;
}

}  // namespace srw
