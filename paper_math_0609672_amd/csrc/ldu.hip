// Asymmetric matrices (Section 7.1): the walk game of A gives Y_A and D (eqs. y2, d),
// the game of A^T with the same ordering gives Y_T (eq. y3), and in rank order
// A ~ Y_T^T D Y_A, the reversed LDU of rev(A).  This file builds A^T, both factors,
// and solves with preconditioned BiCGSTAB (Barrett et al., Templates, preconditioned
// BiCGSTAB): the preconditioner is not symmetric, so conjugate gradients do not apply.
//
// Reductions are deterministic (fixed grid of partial sums, added in a fixed order);
// the iteration's scalars are formed on the host in FP64 from the reduced dots.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "factor.hpp"

namespace srw {

namespace {

constexpr int BLOCK = 256;
constexpr int RED = 1024;  // blocks of every reducing kernel (grid-stride)

// ------------------------------------------------------------------- transpose
__global__ void k_entry_rows(int64_t n, const int64_t* __restrict__ rowptr, uint32_t* __restrict__ row)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    for (int64_t p = rowptr[k]; p < rowptr[k + 1]; ++p) row[p] = (uint32_t)k;
}

// key of entry p of A as an entry of A^T: its column, then its row
__global__ void k_transpose_keys(int64_t nnz, const uint32_t* __restrict__ row,
                                 const int32_t* __restrict__ col, uint64_t* __restrict__ key,
                                 uint32_t* __restrict__ idx)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    key[p] = ((uint64_t)(uint32_t)col[p] << 32) | row[p];
    idx[p] = (uint32_t)p;
}

// row pointers of A^T: first sorted key of every column (binary search), k = 0..n
__global__ void k_transpose_ptr(int64_t n, const uint64_t* __restrict__ key, int64_t nnz,
                                int64_t* __restrict__ tptr)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > n) return;
    const uint64_t want = (uint64_t)k << 32;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (key[mid] < want) lo = mid + 1;
        else hi = mid;
    }
    tptr[k] = lo;
}

__global__ void k_transpose_fill(int64_t nnz, const uint64_t* __restrict__ key,
                                 const uint32_t* __restrict__ idx, const double* __restrict__ val,
                                 int32_t* __restrict__ tcol, double* __restrict__ tval)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    tcol[p] = (int32_t)(uint32_t)key[p];
    tval[p] = val[idx[p]];
}

int grid_of(int64_t n) { return (int)std::max<int64_t>(1, (n + BLOCK - 1) / BLOCK); }

// ------------------------------------------------------------------- BiCGSTAB
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

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < (n); i += (int64_t)gridDim.x * BLOCK)

// y = A x
__global__ __launch_bounds__(BLOCK) void k_spmv(int64_t n, const int64_t* __restrict__ rowptr,
                                                const int32_t* __restrict__ col,
                                                const double* __restrict__ val,
                                                const double* __restrict__ x, double* __restrict__ y)
{
    GRID_STRIDE(i, n)
    {
        double acc = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) acc += val[e] * x[col[e]];
        y[i] = acc;
    }
}

// partials of a . b, and of c . d when c is given (second half of `part`)
__global__ __launch_bounds__(BLOCK) void k_dots(int64_t n, const double* __restrict__ a,
                                                const double* __restrict__ b,
                                                const double* __restrict__ c,
                                                const double* __restrict__ d, double* part)
{
    __shared__ double lds[BLOCK / 64];
    double s1 = 0.0, s2 = 0.0;
    GRID_STRIDE(i, n)
    {
        s1 += a[i] * b[i];
        if (c) s2 += c[i] * d[i];
    }
    s1 = block_sum(s1, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s1;
    if (c) {
        s2 = block_sum(s2, lds);
        if (threadIdx.x == 0) part[RED + blockIdx.x] = s2;
    }
}

// out[0] = sum of part[0 .. np), out[1] = sum of part[RED .. RED + np) (when two)
__global__ __launch_bounds__(BLOCK) void k_sums(const double* __restrict__ part, int np, int two,
                                                double* out)
{
    __shared__ double lds[BLOCK / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += BLOCK) s += part[i];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[0] = s;
    if (two) {
        double t = 0.0;
        for (int i = threadIdx.x; i < np; i += BLOCK) t += part[RED + i];
        t = block_sum(t, lds);
        if (threadIdx.x == 0) out[1] = t;
    }
}

// p = r (first) or p = r + beta (p - omega v)
__global__ __launch_bounds__(BLOCK) void k_bicg_p(int64_t n, const double* __restrict__ r,
                                                  const double* __restrict__ v, double* __restrict__ p,
                                                  double beta, double omega, int first)
{
    GRID_STRIDE(i, n) { p[i] = first ? r[i] : r[i] + beta * (p[i] - omega * v[i]); }
}

// s = r - alpha v, partials of s . s
__global__ __launch_bounds__(BLOCK) void k_bicg_s(int64_t n, const double* __restrict__ r,
                                                  const double* __restrict__ v, double alpha,
                                                  double* __restrict__ s, double* part)
{
    __shared__ double lds[BLOCK / 64];
    double acc = 0.0;
    GRID_STRIDE(i, n)
    {
        const double si = r[i] - alpha * v[i];
        s[i] = si;
        acc += si * si;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// x += alpha ph
__global__ __launch_bounds__(BLOCK) void k_bicg_half(int64_t n, double* __restrict__ x,
                                                     const double* __restrict__ ph, double alpha)
{
    GRID_STRIDE(i, n) { x[i] = x[i] + alpha * ph[i]; }
}

// x += alpha ph + omega sh, r = s - omega t, partials of r . r
__global__ __launch_bounds__(BLOCK) void k_bicg_xr(int64_t n, double* __restrict__ x,
                                                   double* __restrict__ r,
                                                   const double* __restrict__ ph,
                                                   const double* __restrict__ sh,
                                                   const double* __restrict__ s,
                                                   const double* __restrict__ t, double alpha,
                                                   double omega, double* part)
{
    __shared__ double lds[BLOCK / 64];
    double acc = 0.0;
    GRID_STRIDE(i, n)
    {
        x[i] = x[i] + alpha * ph[i] + omega * sh[i];
        const double ri = s[i] - omega * t[i];
        r[i] = ri;
        acc += ri * ri;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// r = b - A x, partials of r . r
__global__ __launch_bounds__(BLOCK) void k_bicg_residual(int64_t n, const int64_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ b,
                                                         double* __restrict__ r, double* part)
{
    __shared__ double lds[BLOCK / 64];
    double acc = 0.0;
    GRID_STRIDE(i, n)
    {
        double q = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) q += val[e] * x[col[e]];
        const double ri = b[i] - q;
        r[i] = ri;
        acc += ri * ri;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// two copies of a
__global__ __launch_bounds__(BLOCK) void k_copy2(int64_t n, const double* __restrict__ a,
                                                 double* __restrict__ b, double* __restrict__ c)
{
    GRID_STRIDE(i, n)
    {
        b[i] = a[i];
        if (c) c[i] = a[i];
    }
}

#undef GRID_STRIDE

}  // namespace

int build_ldu_impl(const srw_csr* A, int32_t walks_per_row, double drop_tol, uint64_t seed,
                   const srw_options* opt_in, srw_factor** out, hipStream_t s)
{
    srw_options opt;
    srw_default_options(&opt);
    if (opt_in) opt = *opt_in;
    srw_factor* F = nullptr;
    int st = build_factor_impl(A, walks_per_row, drop_tol, seed, &opt, &F, s, nullptr, nullptr, true);
    if (st != SRW_OK) return st;
    const int64_t n = A->n, nnz = A->nnz;
    // A^T by a radix sort of the entries on (column, row)
    char* ws = nullptr;
    auto align = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t m = (size_t)std::max<int64_t>(nnz, 1);
    const size_t bytes = 2 * align(m * sizeof(uint64_t)) + 3 * align(m * sizeof(uint32_t)) +
                         align((size_t)(n + 1) * sizeof(int64_t)) + align(m * sizeof(int32_t)) +
                         align(m * sizeof(double)) + radix_tmp_bytes(nnz);
    hipError_t e = hipMallocAsync((void**)&ws, bytes, s);
    if (e != hipSuccess) {
        free_factor(F);
        return hip_fail(e, "hipMallocAsync");
    }
    char* p = ws;
    uint64_t* key = (uint64_t*)p; p += align(m * sizeof(uint64_t));
    uint64_t* key2 = (uint64_t*)p; p += align(m * sizeof(uint64_t));
    uint32_t* idx = (uint32_t*)p; p += align(m * sizeof(uint32_t));
    uint32_t* idx2 = (uint32_t*)p; p += align(m * sizeof(uint32_t));
    uint32_t* row = (uint32_t*)p; p += align(m * sizeof(uint32_t));
    int64_t* tptr = (int64_t*)p; p += align((size_t)(n + 1) * sizeof(int64_t));
    int32_t* tcol = (int32_t*)p; p += align(m * sizeof(int32_t));
    double* tval = (double*)p; p += align(m * sizeof(double));
    void* rt = p;
    int rbits = 1;
    while (rbits < 31 && ((int64_t)1 << rbits) < n) ++rbits;
    uint64_t* ko = key;
    uint32_t* vo = idx;
    k_entry_rows<<<grid_of(n), BLOCK, 0, s>>>(n, A->rowptr, row);
    k_transpose_keys<<<grid_of(nnz), BLOCK, 0, s>>>(nnz, row, A->col, key, idx);
    e = hipGetLastError();
    if (e == hipSuccess && nnz > 0)
        e = radix_sort_u64(key, idx, key2, idx2, nnz, 32 + rbits, rt, &ko, &vo, s);
    if (e == hipSuccess) {
        k_transpose_ptr<<<grid_of(n + 1), BLOCK, 0, s>>>(n, ko, nnz, tptr);
        k_transpose_fill<<<grid_of(nnz), BLOCK, 0, s>>>(nnz, ko, vo, A->val, tcol, tval);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        (void)hipFreeAsync(ws, s);
        free_factor(F);
        return hip_fail(e, "transpose");
    }
    // the game of A^T with the ordering of the game of A and the same walk draws
    srw_csr At{n, nnz, tptr, tcol, tval};
    srw_options ot = opt;
    ot.ordering = SRW_ORDER_GIVEN;
    ot.rank = F->rank;
    srw_factor* G = nullptr;
    st = build_factor_impl(&At, walks_per_row, drop_tol, seed, &ot, &G, s, nullptr, nullptr, true);
    (void)hipFreeAsync(ws, s);
    (void)hipStreamSynchronize(s);
    if (st != SRW_OK) {
        free_factor(F);
        return st;
    }
    F->tgame = G;
    *out = F;
    return SRW_OK;
}

int bicgstab_impl(const srw_csr* A, srw_factor* F, const double* b, double tol, int32_t max_iter,
                  double* x, int32_t* iters_out, double* rel_out, hipStream_t s)
{
    const int64_t n = A->n;
    const int rg = (int)std::max<int64_t>(1, std::min<int64_t>((n + BLOCK - 1) / BLOCK, RED));
    const size_t vec = (size_t)std::max<int64_t>(n, 1);
    double* ws = nullptr;
    // r, rt, p, v, ph, s, sh, t, 2 n of preconditioner scratch, partials, sums, err
    SRW_HIP(hipMallocAsync((void**)&ws, (10 * vec + 2 * RED + 4) * sizeof(double), s));
    double *r = ws, *rt = ws + vec, *p = ws + 2 * vec, *v = ws + 3 * vec, *ph = ws + 4 * vec;
    double *sv = ws + 5 * vec, *sh = ws + 6 * vec, *t = ws + 7 * vec, *work = ws + 8 * vec;
    double* part = ws + 10 * vec;
    double* sums = part + 2 * RED;
    int* err = (int*)(sums + 2);
    double* host = nullptr;
    host = host_scratch() ? (double*)(host_scratch() + 8) : nullptr;
    hipError_t e = host ? hipSuccess : hipErrorOutOfMemory;
    if (e != hipSuccess) {
        (void)hipFreeAsync(ws, s);
        return hip_fail(e, "hipHostMalloc");
    }
    int status = SRW_NOT_CONVERGED;
    bool gave_up = false;
    int32_t it = 0;
    double rel = 0.0;
    // sum the partials (one or two dots) and bring them to the host
    auto reduce = [&](int two, double* o) -> hipError_t {
        k_sums<<<1, BLOCK, 0, s>>>(part, rg, two, sums);
        hipError_t ee = hipGetLastError();
        if (ee == hipSuccess)
            ee = hipMemcpyAsync(host, sums, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
        if (ee == hipSuccess) ee = hipStreamSynchronize(s);
        o[0] = host[0];
        if (two) o[1] = host[1];
        return ee;
    };
    auto dots = [&](const double* a1, const double* b1, const double* c1, const double* d1,
                    double* o) -> hipError_t {
        k_dots<<<rg, BLOCK, 0, s>>>(n, a1, b1, c1, d1, part);
        hipError_t ee = hipGetLastError();
        return ee == hipSuccess ? reduce(c1 ? 1 : 0, o) : ee;
    };
    auto precond = [&](const double* src, double* dst) -> hipError_t {
        if (!F) {
            k_copy2<<<rg, BLOCK, 0, s>>>(n, src, dst, nullptr);
            return hipGetLastError();
        }
        return apply_factor(F, src, work, dst, err, s);
    };
    auto solve_failed = [&]() -> bool {
        int herr = 0;
        if (hipMemcpyAsync(host + 2, err, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return true;
        std::memcpy(&herr, host + 2, sizeof(int));
        return herr != 0;
    };
#define STEP(call)                      \
    do {                                \
        call;                           \
        if (e == hipSuccess) e = hipGetLastError(); \
        if (e != hipSuccess) goto out;  \
    } while (0)
    {
        double o[2] = {0.0, 0.0};
        STEP(e = hipMemsetAsync(x, 0, vec * sizeof(double), s));
        STEP(e = hipMemsetAsync(err, 0, sizeof(int), s));
        STEP(e = dots(b, b, nullptr, nullptr, o));
        const double bnorm = std::sqrt(o[0]);
        if (bnorm == 0.0) {
            status = SRW_OK;
            goto out;
        }
        STEP((k_copy2<<<rg, BLOCK, 0, s>>>(n, b, r, rt)));
        bool first = true;
        double rho_prev = 0.0, alpha = 0.0, omega = 0.0;
        while (it < max_iter) {
            STEP(e = dots(rt, r, nullptr, nullptr, o));
            const double rho = o[0];
            if (rho == 0.0) break;
            const double beta = first ? 0.0 : (rho / rho_prev) * (alpha / omega);
            STEP((k_bicg_p<<<rg, BLOCK, 0, s>>>(n, r, v, p, beta, omega, first ? 1 : 0)));
            first = false;
            STEP(e = precond(p, ph));
            STEP((k_spmv<<<rg, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, ph, v)));
            ++it;
            STEP(e = dots(rt, v, nullptr, nullptr, o));
            if (F && solve_failed()) {
                gave_up = true;
                e = hipErrorLaunchFailure;
                goto out;
            }
            const double rtv = o[0];
            if (rtv == 0.0) break;
            alpha = rho / rtv;
            STEP((k_bicg_s<<<rg, BLOCK, 0, s>>>(n, r, v, alpha, sv, part)));
            STEP(e = reduce(0, o));
            bool converged = false;
            if (std::sqrt(o[0]) <= tol * bnorm) {
                STEP((k_bicg_half<<<rg, BLOCK, 0, s>>>(n, x, ph, alpha)));
                converged = true;
            } else {
                STEP(e = precond(sv, sh));
                STEP((k_spmv<<<rg, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, sh, t)));
                STEP(e = dots(t, t, t, sv, o));
                const double tt = o[0], ts = o[1];
                if (tt == 0.0) break;
                omega = ts / tt;
                STEP((k_bicg_xr<<<rg, BLOCK, 0, s>>>(n, x, r, ph, sh, sv, t, alpha, omega, part)));
                STEP(e = reduce(0, o));
                rho_prev = rho;
                if (!std::isfinite(o[0])) break;
                if (std::sqrt(o[0]) <= tol * bnorm) converged = true;
                else if (omega == 0.0) break;
            }
            if (converged) {
                STEP((k_bicg_residual<<<rg, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, x, b, r, part)));
                STEP(e = reduce(0, o));
                if (std::sqrt(o[0]) <= tol * bnorm) {
                    status = SRW_OK;
                    break;
                }
                // restart from the true residual
                STEP((k_copy2<<<rg, BLOCK, 0, s>>>(n, r, rt, nullptr)));
                first = true;
            }
        }
        // true relative residual of the returned iterate
        STEP((k_bicg_residual<<<rg, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, x, b, r, part)));
        STEP(e = reduce(0, o));
        rel = std::sqrt(o[0]) / bnorm;
        if (F && solve_failed()) {
            gave_up = true;
            e = hipErrorLaunchFailure;
        }
    }
out:
#undef STEP
    (void)hipFreeAsync(ws, s);
    (void)hipStreamSynchronize(s);
    if (iters_out) *iters_out = it;
    if (rel_out) *rel_out = rel;
    if (gave_up) {
        set_last_error("bicgstab: a triangular solve of the preconditioner gave up waiting");
        return SRW_E_HIP;
    }
    if (e != hipSuccess) return hip_fail(e, "bicgstab");
    return status;
}

}  // namespace srw
