// Solve phase of the hybrid solver (Algorithm 1, "solve"): PCG with the
// preconditioner (Y^T D Y)^{-1} applied by two sync-free triangular solves.
//
// Reductions are deterministic: every dot product is summed per block of a fixed
// grid into partials and the partials are added by one block in a fixed order.
// The scalars of the iteration (rho, alpha, beta, ||r||^2) live on the device; the
// host reads ||r||^2 once per iteration for the stopping test.
#include <algorithm>
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
// Sync-free substitution.  Rows are handed out as tickets in a topological order of
// Y z = v -- increasing (level, rank) or increasing rank -- and in the reverse order for
// Y^T w = r (a row's backward dependencies all have a higher level and rank): a wave
// takes one ticket at a time with a global atomic.  A row only waits on smaller tickets, and the
// smallest unfinished ticket always has all its dependencies done and is the current
// row of its wave, so the solve always progresses.  The
// solution vector starts filled with a signalling-NaN pattern that arithmetic never
// produces; a row's value is published with one device-scope store, and a consumer
// spins (device-scope loads) until the pattern is gone -- the value is its own ready
// flag, no fence is needed.  A wave-wide butterfly adds the lane partial sums, so the
// result does not depend on timing.
//   backward  (Y^T w = r):   w_k = r_k - sum_q Yt_kq w_q
//   forward   (Y z = v):     z_k = w_k / D_k - sum_q Y_kq z_q
template <typename T>
struct Bits;
template <>
struct Bits<double> {
    using U = unsigned long long;
    static constexpr U sentinel = 0x7FF4DEADBEEF5A5Aull;
};
template <>
struct Bits<float> {
    using U = unsigned int;
    static constexpr U sentinel = 0x7FA5A5A5u;
};

// A wait that outlives this many polls (about a second) marks the solve failed and
// proceeds with a NaN; the caller then reports the failure.
constexpr uint32_t SPIN_LIMIT = 1u << 20;

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fill_sentinel(int64_t n, T* x, unsigned long long* tickets)
{
    using U = typename Bits<T>::U;
    const int64_t i0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i0 == 0) tickets[0] = 0;
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * BLOCK) ((U*)x)[i] = Bits<T>::sentinel;
}

constexpr unsigned long long TICKETS_PER_WAVE = 1;

// First of the wave's next TICKETS_PER_WAVE tickets.  Every lane executes the atomic
// (lane 0 adds the batch, the others 0), so no lane-divergent branch precedes the
// scalar broadcast.
__device__ __forceinline__ unsigned long long wave_batch(unsigned long long* tickets)
{
    const bool l0 = (threadIdx.x & 63) == 0;
    return lane0_u64(atomicAdd(tickets, l0 ? TICKETS_PER_WAVE : 0ull));
}

#ifndef SRW_POLL_SLEEP
#define SRW_POLL_SLEEP 2  // s_sleep units (64 clocks) between polls of a missing value
#endif

// acc += sum over the entries [q0, q1) of val[q] * sol[col[q]], waiting for every
// sol value to be published.  Each 64-entry chunk issues all its loads at once; the
// wave then re-polls only the lanes still holding the sentinel, as one wave-uniform
// loop (no lane spins on its own), and gives up after SPIN_LIMIT polls.
template <typename T>
__device__ __forceinline__ T gather_published(const int64_t q0, const int64_t q1,
                                              const int32_t* __restrict__ col,
                                              const T* __restrict__ val, const T* sol, int* err)
{
    using U = typename Bits<T>::U;
    const int lane = threadIdx.x & 63;
    T acc = T(0);
    for (int64_t qb = q0; qb < q1; qb += 64) {
        const int64_t q = qb + lane;
        const bool valid = q < q1;
        const int32_t c = valid ? col[q] : 0;
        const T v = valid ? val[q] : T(0);
        const U* p = (const U*)sol + c;
        U bits = valid ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : U(0);
        uint32_t spins = 0;
        while (ballot(bits == Bits<T>::sentinel) != 0) {
            if (++spins > SPIN_LIMIT) {
                if (lane == 0) atomicOr(err, 1);
                if (bits == Bits<T>::sentinel) bits = __builtin_bit_cast(U, (T)NAN);
                break;
            }
            __builtin_amdgcn_s_sleep(SRW_POLL_SLEEP);
            if (bits == Bits<T>::sentinel)
                bits = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        acc += v * __builtin_bit_cast(T, bits);
    }
    return acc;
}

template <typename T, bool FWD>
__global__ __launch_bounds__(BLOCK) void k_trsv_syncfree(
    const int32_t* __restrict__ by_rank, int64_t n, const int64_t* __restrict__ ptr,
    const int32_t* __restrict__ col, const T* __restrict__ val, const T* __restrict__ dvec,
    const double* __restrict__ rhs, const T* __restrict__ w, T* sol, double* __restrict__ sol64,
    unsigned long long* tickets, int* err)
{
    using U = typename Bits<T>::U;
    const int lane = threadIdx.x & 63;
    for (;;) {
        const unsigned long long t = wave_batch(tickets);
        if (t >= (unsigned long long)n) break;
        const int32_t k = by_rank[FWD ? (int64_t)t : n - 1 - (int64_t)t];
        T acc = gather_published<T>(ptr[k], ptr[k + 1], col, val, sol, err);
        acc = wave_sum(acc);
        if (lane == 0) {
            const T v = FWD ? w[k] / dvec[k] - acc : (T)rhs[k] - acc;
            __hip_atomic_store((U*)sol + k, __builtin_bit_cast(U, v), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            if (sol64) sol64[k] = (double)v;
        }
    }
}

// Longest dependency chain of Y (the same for Y^T): lev_k = 1 + max over the row's
// entries, 0 for an empty row; rows in increasing rank, same publication scheme.
__global__ __launch_bounds__(BLOCK) void k_depth(const int32_t* __restrict__ by_rank, int64_t n,
                                                 const int64_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ col, int32_t* lev,
                                                 unsigned long long* tickets, int* depth, int* err)
{
    const int lane = threadIdx.x & 63;
    for (;;) {
        const unsigned long long base = wave_batch(tickets);
        if (base >= (unsigned long long)n) break;
        for (unsigned long long j = 0; j < TICKETS_PER_WAVE; ++j) {
        const unsigned long long t = base + j;
        if (t >= (unsigned long long)n) break;
        const int32_t k = by_rank[t];
        int32_t m = -1;
        for (int64_t q = ptr[k] + lane; q < ptr[k + 1]; q += 64) {
            const int32_t* p = lev + col[q];
            int32_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t spins = 0;
            while (v < 0) {
                if (++spins > SPIN_LIMIT) {
                    atomicOr(err, 1);
                    v = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            m = max(m, v);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
        if (lane == 0) {
            __hip_atomic_store(lev + k, m + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicMax(depth, m + 2);
        }
        }  // tickets of this wave
    }
}

__global__ void k_fill_i32(int64_t n, int32_t* x, int32_t v, unsigned long long* tickets)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) tickets[0] = 0;
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}

int persistent_blocks()
{
    static int blocks = 0;
    if (!blocks) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        blocks = cus * 8;
    }
    return blocks;
}

// w and z scratch: work (n values of T), ticket counters and an error flag.
// zlo receives z in the factor's precision; z (if not null) a double copy.
template <typename T>
hipError_t apply_syncfree(const srw_factor* F, const double* r, T* work, T* zlo, double* z,
                          unsigned long long* tickets, int* err, hipStream_t s)
{
    const int64_t n = F->n;
    const int fg = (int)std::min<int64_t>(grid_for(n, BLOCK), 2048);
    const int pb = persistent_blocks();
    k_fill_sentinel<T><<<fg, BLOCK, 0, s>>>(n, work, tickets);
    const int32_t* order = F->solve_order ? F->solve_order : F->by_rank;
    k_trsv_syncfree<T, false><<<pb, BLOCK, 0, s>>>(order, n, F->ytptr, F->ytcol,
                                                   (const T*)F->ytval, (const T*)F->d, r, nullptr,
                                                   work, nullptr, tickets, err);
    k_fill_sentinel<T><<<fg, BLOCK, 0, s>>>(n, zlo, tickets + 1);
    k_trsv_syncfree<T, true><<<pb, BLOCK, 0, s>>>(order, n, F->yptr, F->ycol,
                                                  (const T*)F->yval, (const T*)F->d, nullptr, work,
                                                  zlo, z, tickets + 1, err);
    return hipGetLastError();
}

// work: 2 n doubles of scratch; tickets: 2 counters; err: one int (0 on entry).
hipError_t apply_any(const srw_factor* F, const double* r, void* work, double* z,
                     unsigned long long* tickets, int* err, hipStream_t s)
{
    if (F->n == 0) return hipSuccess;
    if (F->precision == SRW_FP32) {
        float* w = (float*)work;
        return apply_syncfree<float>(F, r, w, w + F->n, z, tickets, err, s);
    }
    // FP64: the forward solve publishes straight into z
    return apply_syncfree<double>(F, r, (double*)work, z, nullptr, tickets, err, s);
}

int red_grid(int64_t n)
{
    const int64_t g = (n + BLOCK - 1) / BLOCK;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, RED_GRID));
}

}  // namespace

int apply_impl(srw_factor* F, const double* r, double* z, hipStream_t s)
{
    const int64_t n = F->n;
    char* ws = nullptr;
    const size_t vec = (size_t)std::max<int64_t>(n, 1);
    SRW_HIP(hipMallocAsync((void**)&ws, 2 * vec * sizeof(double) + 64, s));
    unsigned long long* tickets = (unsigned long long*)(ws + 2 * vec * sizeof(double));
    int* err = (int*)(tickets + 2);
    hipError_t e = hipMemsetAsync(err, 0, sizeof(int), s);
    if (e == hipSuccess) e = apply_any(F, r, ws, z, tickets, err, s);
    int herr = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(ws, s);
    (void)hipStreamSynchronize(s);
    SRW_HIP(e);
    return herr ? SRW_E_HIP : SRW_OK;
}

int dag_levels(srw_factor* F, int32_t* lev, int32_t* depth_out, hipStream_t s)
{
    const int64_t n = F->n;
    *depth_out = 0;
    if (n == 0) return SRW_OK;
    char* ws = nullptr;
    SRW_HIP(hipMallocAsync((void**)&ws, 64, s));
    unsigned long long* tickets = (unsigned long long*)ws;
    int* depth = (int*)(tickets + 1);
    int* err = depth + 1;
    hipError_t e = hipMemsetAsync(depth, 0, 2 * sizeof(int), s);
    if (e == hipSuccess) {
        k_fill_i32<<<(int)std::min<int64_t>(grid_for(n, BLOCK), 2048), BLOCK, 0, s>>>(n, lev, -1, tickets);
        k_depth<<<persistent_blocks(), BLOCK, 0, s>>>(F->by_rank, n, F->yptr, F->ycol, lev, tickets,
                                                      depth, err);
        e = hipGetLastError();
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
    unsigned long long* tickets = (unsigned long long*)(sc + S_COUNT);
    int* err = (int*)(tickets + 2);
    hipError_t herr = hipHostMalloc((void**)&host, 4 * sizeof(double), hipHostMallocDefault);
    if (herr != hipSuccess) {
        (void)hipFreeAsync(ws, s);
        return hip_fail(herr, "hipHostMalloc");
    }
    int status = SRW_NOT_CONVERGED;
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
        STEP(e = apply_any(F, r, work, z, tickets, err, s));
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
                STEP(e = apply_any(F, r, work, z, tickets, err, s));
                STEP((k_update_p<<<eg, BLOCK, 0, s>>>(n, z, p, nullptr)));
                STEP((k_dot<<<rg, BLOCK, 0, s>>>(n, r, z, partials)));
                STEP((k_finalize<<<1, BLOCK, 0, s>>>(partials, rg, sc, OP_RHO0)));
                continue;
            }
            STEP(e = apply_any(F, r, work, z, tickets, err, s));
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
    (void)hipHostFree(host);
    if (e != hipSuccess) return hip_fail(e, "pcg");
    if (iters_out) *iters_out = it;
    if (rel_out) *rel_out = rel;
    return status;
}

}  // namespace srw
