// Solve phase of the hybrid solver (Algorithm 1, "solve"): PCG with the
// preconditioner (Y^T D Y)^{-1} applied by two level-scheduled triangular solves.
//
// Reductions are deterministic: every dot product is summed per block of a fixed
// grid into partials and the partials are added by one block in a fixed order.
// The scalars of the iteration (rho, alpha, beta, ||r||^2) live on the device; the
// host reads ||r||^2 once per iteration for the stopping test.
#include <cmath>

#include "factor.hpp"

namespace srw {

namespace {

constexpr int BLOCK = 256;
constexpr int RED_GRID = 1024;  // blocks of every reducing kernel (grid-stride)
constexpr int TRSV_GROUP = 8;   // lanes per row in the triangular solves

enum Scalar : int { S_RHO = 0, S_PQ, S_ALPHA, S_RR, S_RHO_NEW, S_BETA, S_BB, S_COUNT };
enum Op : int { OP_RHO0 = 0, OP_ALPHA, OP_RR, OP_BETA, OP_BB };

__device__ __forceinline__ double block_sum(double v, double* lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
// One group of TRSV_GROUP lanes per row of the level; lane j sums entries j, j+G, ...
// then the group adds its lanes by a butterfly.
//   backward  (Y^T w = r):   w_k = r_k - sum_q Yt_kq w_q
//   forward   (Y z = v):     z_k = w_k / D_k - sum_q Y_kq z_q
template <typename T, typename In, bool FWD>
__global__ __launch_bounds__(BLOCK) void k_trsv_level(const int32_t* __restrict__ rows, int64_t count,
                                                      const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ col,
                                                      const T* __restrict__ val,
                                                      const T* __restrict__ dvec,
                                                      const In* __restrict__ rhs,
                                                      T* __restrict__ sol, double* __restrict__ sol64)
{
    const int64_t g = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / TRSV_GROUP;
    const int j = threadIdx.x % TRSV_GROUP;
    const bool valid = g < count;
    const int32_t k = valid ? rows[g] : 0;
    T acc = T(0);
    if (valid)
        for (int64_t q = ptr[k] + j; q < ptr[k + 1]; q += TRSV_GROUP) acc += val[q] * sol[col[q]];
#pragma unroll
    for (int off = TRSV_GROUP / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, TRSV_GROUP);
    if (valid && j == 0) {
        T v;
        if (FWD) v = sol[k] / dvec[k] - acc;  // sol[k] holds w_k from the backward solve
        else v = (T)rhs[k] - acc;
        sol[k] = v;
        if (sol64) sol64[k] = (double)v;
    }
}

template <typename T>
hipError_t apply_levels(const srw_factor* F, const double* r, T* work, double* z, hipStream_t s)
{
    // backward solve writes w into work; forward solve overwrites work with z
    for (size_t L = 0; L + 1 < F->bwd_lptr.size(); ++L) {
        const int64_t a = F->bwd_lptr[L], cnt = F->bwd_lptr[L + 1] - a;
        k_trsv_level<T, double, false><<<grid_for(cnt * TRSV_GROUP, BLOCK), BLOCK, 0, s>>>(
            F->bwd_rows + a, cnt, F->ytptr, F->ytcol, (const T*)F->ytval, (const T*)F->d, r, work,
            nullptr);
    }
    for (size_t L = 0; L + 1 < F->fwd_lptr.size(); ++L) {
        const int64_t a = F->fwd_lptr[L], cnt = F->fwd_lptr[L + 1] - a;
        k_trsv_level<T, double, true><<<grid_for(cnt * TRSV_GROUP, BLOCK), BLOCK, 0, s>>>(
            F->fwd_rows + a, cnt, F->yptr, F->ycol, (const T*)F->yval, (const T*)F->d, r, work, z);
    }
    return hipGetLastError();
}

hipError_t apply_any(const srw_factor* F, const double* r, void* work, double* z, hipStream_t s)
{
    if (F->n == 0) return hipSuccess;
    if (F->precision == SRW_FP32) return apply_levels<float>(F, r, (float*)work, z, s);
    return apply_levels<double>(F, r, (double*)work, z, s);
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
    void* work = nullptr;
    SRW_HIP(hipMallocAsync(&work, (size_t)std::max<int64_t>(n, 1) * sizeof(double), s));
    hipError_t e = apply_any(F, r, work, z, s);
    (void)hipFreeAsync(work, s);
    SRW_HIP(e);
    SRW_HIP(hipStreamSynchronize(s));
    return SRW_OK;
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
    SRW_HIP(hipMallocAsync((void**)&ws, (5 * vec + RED_GRID + S_COUNT) * sizeof(double), s));
    double *r = ws, *z = ws + vec, *p = ws + 2 * vec, *q = ws + 3 * vec, *work = ws + 4 * vec;
    double* partials = ws + 5 * vec;
    double* sc = partials + RED_GRID;
    hipError_t herr = hipHostMalloc((void**)&host, 4 * sizeof(double), hipHostMallocDefault);
    if (herr != hipSuccess) {
        (void)hipFreeAsync(ws, s);
        return hip_fail(herr, "hipHostMalloc");
    }
    int status = SRW_NOT_CONVERGED;
    int32_t it = 0;
    double rel = 0.0;
    hipError_t e = hipSuccess;
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
        STEP(e = apply_any(F, r, work, z, s));
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
            if (std::sqrt(rr) <= tol * bnorm) {
                STEP((k_residual<<<rg, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, x, b, r, partials)));
                STEP((k_finalize<<<1, BLOCK, 0, s>>>(partials, rg, sc, OP_RR)));
                if ((e = read_scalar(S_RR, &rr)) != hipSuccess) goto out;
                if (std::sqrt(rr) <= tol * bnorm) {
                    status = SRW_OK;
                    break;
                }
                // restart from the true residual
                STEP(e = apply_any(F, r, work, z, s));
                STEP((k_update_p<<<eg, BLOCK, 0, s>>>(n, z, p, nullptr)));
                STEP((k_dot<<<rg, BLOCK, 0, s>>>(n, r, z, partials)));
                STEP((k_finalize<<<1, BLOCK, 0, s>>>(partials, rg, sc, OP_RHO0)));
                continue;
            }
            STEP(e = apply_any(F, r, work, z, s));
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
