// extern "C" entry points of libsrw.so (declared in include/srw.h).
#include <cmath>
#include <new>

#include "factor.hpp"

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

bool csr_ok(const srw_csr* A)
{
    if (!A || A->n < 0 || A->nnz < A->n || A->n >= (int64_t)0x7FFFFFFF) return false;
    if (!A->rowptr) return false;
    if (A->nnz > 0 && (!A->col || !A->val)) return false;
    return true;
}

template <typename T>
int copy_out(T* dst, const void* src, size_t count, hipStream_t s)
{
    if (!dst || count == 0) return SRW_OK;
    if (!src) return SRW_E_ARG;
    SRW_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToDevice, s));
    return SRW_OK;
}

int options_ok(const srw_options* opt, int64_t n)
{
    if (!opt) return SRW_OK;
    if (opt->ordering != SRW_ORDER_RANDOM && opt->ordering != SRW_ORDER_GIVEN &&
        opt->ordering != SRW_ORDER_NATURAL)
        return SRW_E_ARG;
    if (opt->factor_precision != SRW_FP64 && opt->factor_precision != SRW_FP32) return SRW_E_ARG;
    if (opt->keep < 0 || opt->keep > 2) return SRW_E_ARG;
    const int rp = opt->refill_period;
    if (rp != 0 && rp != 1 && rp != 2 && rp != 4 && rp != 8) return SRW_E_ARG;
    if (opt->schedule != 0 && opt->schedule != 1) return SRW_E_ARG;
    if (opt->solve_order < 0 || opt->solve_order > 2) return SRW_E_ARG;
    if (opt->ordering == SRW_ORDER_GIVEN && !opt->rank && n > 0) return SRW_E_ARG;
    if (opt->reuse != 0 && opt->reuse != 1) return SRW_E_ARG;
    if (opt->reuse && (opt->keep == 2 || (rp != 0 && rp != 8))) return SRW_E_ARG;
    if (opt->walk_waves != 0 && (opt->walk_waves < 4 || opt->walk_waves > 64)) return SRW_E_ARG;
    if (opt->one_step_exact != 0 && opt->one_step_exact != 1) return SRW_E_ARG;
    if (!opt->one_step_exact && opt->reuse) return SRW_E_ARG;
    if (opt->head_rows < -1 || opt->head_rows > SRW_HEAD_MAX) return SRW_E_ARG;
    return SRW_OK;
}

}  // namespace

extern "C" {

void srw_default_options(srw_options* opt)
{
    if (!opt) return;
    opt->ordering = SRW_ORDER_RANDOM;
    opt->rank = nullptr;
    opt->walks = nullptr;
    opt->factor_precision = SRW_FP64;
    opt->max_steps = 0;
    opt->keep = 0;
    opt->refill_period = 0;
    opt->profile = 0;
    opt->schedule = 1;
    opt->solve_order = 2;
    opt->reuse = 0;
    opt->walk_waves = 0;
    opt->one_step_exact = 1;
    opt->head_rows = 0;
}


int srw_build_factor_batched(int32_t nmat, const srw_csr* A, int32_t walks_per_row,
                             double drop_tol, const uint64_t* seeds, const srw_options* opt,
                             srw_factor** out, void* stream)
{
    if (!out) return SRW_E_ARG;
    *out = nullptr;
    if (nmat < 1 || !A || !seeds) return SRW_E_ARG;
    int64_t total = 0;
    for (int32_t i = 0; i < nmat; ++i) {
        if (!csr_ok(&A[i])) return SRW_E_ARG;
        total += A[i].n;
    }
    if (total >= (int64_t)0x7FFFFFFF) return SRW_E_ARG;
    if (!(drop_tol >= 0.0) || !std::isfinite(drop_tol)) return SRW_E_ARG;
    if (options_ok(opt, total) != SRW_OK) return SRW_E_ARG;
    if (opt && opt->ordering != SRW_ORDER_RANDOM) return SRW_E_ARG;  // one ordering per matrix
    if (opt && !opt->one_step_exact) return SRW_E_ARG;                // the plain estimator: single builds
    if ((!opt || !opt->walks) && walks_per_row < 1) return SRW_E_ARG;
    if (walks_per_row > 8192 || walks_per_row < 0) return SRW_E_ARG;
    srw_options o;
    srw_default_options(&o);
    if (opt) o = *opt;
    try {
        return srw::build_batched_impl(nmat, A, walks_per_row, drop_tol, seeds, &o, out,
                                       as_stream(stream));
    } catch (const std::bad_alloc&) {
        return SRW_E_NOMEM;
    } catch (...) {
        return SRW_E_HIP;
    }
}

int srw_batch_info(const srw_factor* F, int32_t* nmat, int64_t* row_off)
{
    if (!F) return SRW_E_ARG;
    if (nmat) *nmat = F->nmat;
    if (row_off)
        for (int32_t i = 0; i <= F->nmat && F->nmat > 0; ++i) row_off[i] = F->mat_off_host[i];
    return SRW_OK;
}

int srw_pcg_solve_batched(srw_factor* F, int32_t nrhs, const double* B, double tol,
                          int32_t max_iter, double* X, int32_t* iters, double* rel_residual,
                          int32_t use_graph, void* stream)
{
    if (!F || F->nmat < 1 || nrhs < 1 || nrhs > 8) return SRW_E_ARG;
    if (!(tol >= 0.0) || max_iter < 0) return SRW_E_ARG;
    const int64_t nsys = (int64_t)F->nmat * nrhs;
    if (F->n == 0) {
        for (int64_t i = 0; i < nsys; ++i) {
            if (iters) iters[i] = 0;
            if (rel_residual) rel_residual[i] = 0.0;
        }
        return SRW_OK;
    }
    if (!B || !X) return SRW_E_ARG;
    try {
        return srw::pcg_batched_impl(F, nrhs, B, tol, max_iter, X, iters, rel_residual,
                                     use_graph ? 1 : 0, as_stream(stream));
    } catch (...) {
        return SRW_E_HIP;
    }
}

int srw_apply_batched(srw_factor* F, int32_t nrhs, const double* R, double* Z, int32_t schedule,
                      void* stream)
{
    if (!F || F->nmat < 1 || nrhs < 1 || nrhs > 8 || schedule < 0 || schedule > 2) return SRW_E_ARG;
    if (F->n == 0) return SRW_OK;
    if (!R || !Z) return SRW_E_ARG;
    try {
        return srw::apply_batched_impl(F, nrhs, R, Z, schedule, as_stream(stream));
    } catch (...) {
        return SRW_E_HIP;
    }
}

int srw_build_factor(const srw_csr* A, int32_t walks_per_row, double drop_tol, uint64_t seed,
                     const srw_options* opt, srw_factor** out, void* stream)
{
    if (!out) return SRW_E_ARG;
    *out = nullptr;
    if (!csr_ok(A)) return SRW_E_ARG;
    if (!(drop_tol >= 0.0) || !std::isfinite(drop_tol)) return SRW_E_ARG;
    if (options_ok(opt, A->n) != SRW_OK) return SRW_E_ARG;
    if ((!opt || !opt->walks) && walks_per_row < 1) return SRW_E_ARG;
    if (walks_per_row > 8192 || walks_per_row < 0) return SRW_E_ARG;
    try {
        return srw::build_factor_impl(A, walks_per_row, drop_tol, seed, opt, out, as_stream(stream));
    } catch (const std::bad_alloc&) {
        return SRW_E_NOMEM;
    } catch (...) {
        return SRW_E_HIP;
    }
}

int srw_build_ic0(const srw_csr* A, uint64_t seed, const srw_options* opt, srw_factor** out,
                  void* stream)
{
    if (!out) return SRW_E_ARG;
    *out = nullptr;
    if (!csr_ok(A)) return SRW_E_ARG;
    if (options_ok(opt, A->n) != SRW_OK) return SRW_E_ARG;
    if (opt && (opt->reuse || opt->factor_precision != SRW_FP64 || opt->walks)) return SRW_E_ARG;
    try {
        return srw::build_factor_impl(A, 1, 0.0, seed, opt, out, as_stream(stream), nullptr,
                                      nullptr, false, true);
    } catch (const std::bad_alloc&) {
        return SRW_E_NOMEM;
    } catch (...) {
        return SRW_E_HIP;
    }
}

void srw_factor_free(srw_factor* F) { srw::free_factor(F); }

int srw_build_factor_ldu(const srw_csr* A, int32_t walks_per_row, double drop_tol, uint64_t seed,
                         const srw_options* opt, srw_factor** out, void* stream)
{
    if (!out) return SRW_E_ARG;
    *out = nullptr;
    if (!csr_ok(A)) return SRW_E_ARG;
    if (!(drop_tol >= 0.0) || !std::isfinite(drop_tol)) return SRW_E_ARG;
    if (options_ok(opt, A->n) != SRW_OK) return SRW_E_ARG;
    if (opt && !opt->one_step_exact) return SRW_E_ARG;  // the plain estimator: single builds
    if ((!opt || !opt->walks) && walks_per_row < 1) return SRW_E_ARG;
    if (walks_per_row > 8192 || walks_per_row < 0) return SRW_E_ARG;
    try {
        return srw::build_ldu_impl(A, walks_per_row, drop_tol, seed, opt, out, as_stream(stream));
    } catch (const std::bad_alloc&) {
        return SRW_E_NOMEM;
    } catch (...) {
        return SRW_E_HIP;
    }
}

int srw_factor_transpose_game(const srw_factor* F, const srw_factor** G)
{
    if (!F || !G) return SRW_E_ARG;
    *G = F->tgame;
    return F->tgame ? SRW_OK : SRW_E_ARG;
}

int srw_bicgstab_solve(const srw_csr* A, const srw_factor* F, const double* b, double tol,
                       int32_t max_iter, double* x, int32_t* iters, double* rel_residual,
                       void* stream)
{
    if (!csr_ok(A)) return SRW_E_ARG;
    if (F && (A->n != F->n || A->nnz != F->nnz_a || F->nmat > 0)) return SRW_E_ARG;
    if (A->n > 0 && (!b || !x)) return SRW_E_ARG;
    if (!(tol >= 0.0) || max_iter < 0) return SRW_E_ARG;
    if (iters) *iters = 0;
    if (rel_residual) *rel_residual = 0.0;
    if (A->n == 0) return SRW_OK;
    try {
        return srw::bicgstab_impl(A, const_cast<srw_factor*>(F), b, tol, max_iter, x, iters,
                                  rel_residual, as_stream(stream));
    } catch (...) {
        return SRW_E_HIP;
    }
}

int srw_factor_info(const srw_factor* F, int64_t* n, int64_t* nnz_y, int64_t* walks,
                    int64_t* walk_steps, int32_t* levels_fwd, int32_t* levels_bwd,
                    int32_t* precision, int32_t* keep)
{
    if (!F) return SRW_E_ARG;
    if (n) *n = F->n;
    if (nnz_y) *nnz_y = F->nnz_y;
    if (walks) *walks = F->walks_total;
    if (walk_steps) *walk_steps = F->steps_total;
    if (levels_fwd) *levels_fwd = F->depth;
    if (levels_bwd) *levels_bwd = F->depth;
    if (precision) *precision = F->precision;
    if (keep) *keep = F->keep;
    return SRW_OK;
}

int srw_factor_stats(const srw_factor* F, srw_stats* out)
{
    if (!F || !out) return SRW_E_ARG;
    out->n = F->n;
    out->nnz_a = F->nnz_a;
    out->nnz_y = F->nnz_y;
    out->walks = F->walks_total;
    out->walk_steps = F->steps_total;
    out->walk_deg_sum = F->deg_sum;
    out->levels_fwd = F->depth;
    out->levels_bwd = F->depth;
    out->precision = F->precision;
    out->keep = F->keep;
    for (int i = 0; i < SRW_NUM_PHASES; ++i) out->phase_ms[i] = F->phase_ms[i];
    out->tallied_walks = F->tallied_total;
    out->reuse = F->reuse;
    out->two_game = F->tgame ? 1 : 0;
    out->walk_waves = F->walk_waves;
    out->head_rows = F->head;
    out->walk_lds = F->walk_lds;
    return SRW_OK;
}

int srw_factor_depth(srw_factor* F, int32_t* depth, void* stream)
{
    if (!F || !depth) return SRW_E_ARG;
    if (F->depth < 0) {
        int32_t d = 0;
        const int st = srw::dag_depth(F, &d, as_stream(stream));
        if (st != SRW_OK) return st;
        F->depth = d;
    }
    *depth = F->depth;
    return SRW_OK;
}

int srw_factor_export(const srw_factor* F, int64_t* yptr, int32_t* ycol, void* yval, void* d,
                      int32_t* rank, void* stream)
{
    if (!F) return SRW_E_ARG;
    hipStream_t s = as_stream(stream);
    const size_t vb = F->precision == SRW_FP32 ? sizeof(float) : sizeof(double);
    int st;
    if ((st = copy_out(yptr, F->yptr, (size_t)F->n + 1, s))) return st;
    if ((st = copy_out(ycol, F->ycol, (size_t)F->nnz_y, s))) return st;
    if ((st = copy_out((char*)yval, F->yval, (size_t)F->nnz_y * vb, s))) return st;
    if ((st = copy_out((char*)d, F->d, (size_t)F->n * vb, s))) return st;
    if ((st = copy_out(rank, F->rank, (size_t)F->n, s))) return st;
    SRW_HIP(hipStreamSynchronize(s));
    return SRW_OK;
}

int srw_table_export(const srw_factor* F, int32_t* nbr, uint32_t* thr, uint32_t* mthr,
                     double* tau, uint8_t* grounded, void* stream)
{
    if (!F) return SRW_E_ARG;
    if (F->keep < 1) return SRW_E_ARG;
    hipStream_t s = as_stream(stream);
    const int64_t m = F->nnz_a - F->n;
    if (m > 0 && (nbr || thr)) {
        // entries are stored as {neighbour, threshold} pairs
        if (nbr) SRW_HIP(hipMemcpy2DAsync(nbr, sizeof(int32_t), F->ent, sizeof(uint2), sizeof(int32_t),
                                          (size_t)m, hipMemcpyDeviceToDevice, s));
        if (thr) SRW_HIP(hipMemcpy2DAsync(thr, sizeof(uint32_t), (const char*)F->ent + sizeof(uint32_t),
                                          sizeof(uint2), sizeof(uint32_t), (size_t)m,
                                          hipMemcpyDeviceToDevice, s));
    }
    int st;
    if ((st = copy_out(mthr, F->mthr, (size_t)m, s))) return st;
    if ((st = copy_out(tau, F->tau, (size_t)F->n, s))) return st;
    if ((st = copy_out(grounded, F->grounded, (size_t)F->n, s))) return st;
    SRW_HIP(hipStreamSynchronize(s));
    return SRW_OK;
}

int srw_tally_export(const srw_factor* F, uint32_t* walks, uint64_t* J, uint32_t* G,
                     uint64_t* steps, uint64_t* visits_sq, int64_t* h_off, int32_t* hlen,
                     int32_t* h_end, uint32_t* h_cnt, void* stream)
{
    if (!F) return SRW_E_ARG;
    if (F->keep < 1) return SRW_E_ARG;
    hipStream_t s = as_stream(stream);
    const size_t n = (size_t)F->n, W = (size_t)F->tallied_total;
    int st;
    if ((st = copy_out((int32_t*)walks, F->budget, n, s))) return st;
    if ((st = copy_out(J, F->tJ, n, s))) return st;
    if ((st = copy_out(G, F->tG, n, s))) return st;
    if ((st = copy_out(steps, F->tsteps, n, s))) return st;
    if ((st = copy_out(visits_sq, F->tvsq, n, s))) return st;
    if ((st = copy_out(h_off, F->h_off, n, s))) return st;
    if ((st = copy_out(hlen, F->hlen, n, s))) return st;
    if ((st = copy_out((uint32_t*)h_end, F->h_end, W, s))) return st;
    if ((st = copy_out(h_cnt, F->h_cnt, W, s))) return st;
    SRW_HIP(hipStreamSynchronize(s));
    return SRW_OK;
}

int srw_walk_export(const srw_factor* F, int64_t* rec_off, int32_t* end, uint32_t* visits,
                    uint32_t* length, void* stream)
{
    if (!F) return SRW_E_ARG;
    if (F->keep < 2) return SRW_E_ARG;
    hipStream_t s = as_stream(stream);
    const size_t n = (size_t)F->n, W = (size_t)F->walks_total;
    int st;
    if ((st = copy_out(rec_off, F->rec_off, n, s))) return st;
    if ((st = copy_out((uint32_t*)end, F->rec_end, W, s))) return st;
    if ((st = copy_out(visits, F->rec_vis, W, s))) return st;
    if ((st = copy_out(length, F->rec_len, W, s))) return st;
    SRW_HIP(hipStreamSynchronize(s));
    return SRW_OK;
}

int srw_pcg_solve(const srw_csr* A, const srw_factor* F, const double* b, double tol,
                  int32_t max_iter, double* x, int32_t* iters, double* rel_residual, void* stream)
{
    if (!F || !csr_ok(A) || A->n != F->n || A->nnz != F->nnz_a) return SRW_E_ARG;
    if (F->tgame) return SRW_E_ARG;  // a two-game factor is not symmetric: srw_bicgstab_solve
    if (A->n > 0 && (!b || !x)) return SRW_E_ARG;
    if (!(tol >= 0.0) || max_iter < 0) return SRW_E_ARG;
    if (iters) *iters = 0;
    if (rel_residual) *rel_residual = 0.0;
    if (A->n == 0) return SRW_OK;
    try {
        return srw::pcg_impl(A, const_cast<srw_factor*>(F), b, tol, max_iter, x, iters,
                             rel_residual, as_stream(stream));
    } catch (...) {
        return SRW_E_HIP;
    }
}

int srw_apply(const srw_factor* F, const double* r, double* z, void* stream)
{
    if (!F) return SRW_E_ARG;
    if (F->n == 0) return SRW_OK;
    if (!r || !z) return SRW_E_ARG;
    return srw::apply_impl(const_cast<srw_factor*>(F), r, z, as_stream(stream));
}

int srw_apply_noalloc(const srw_factor* F, const double* r, double* z, void* stream)
{
    if (!F) return SRW_E_ARG;
    if (F->n == 0) return SRW_OK;
    if (!r || !z) return SRW_E_ARG;
    return srw::apply_noalloc_impl(F, r, z, as_stream(stream));
}

int srw_adaptive_budgets(const srw_csr* A, uint64_t seed, const srw_options* opt, double delta,
                         double z, int32_t min_walks, int32_t max_walks, int32_t* walks,
                         void* stream)
{
    if (!csr_ok(A) || (A->n > 0 && !walks)) return SRW_E_ARG;
    if (!(delta > 0.0) || !std::isfinite(delta) || !(z > 0.0) || !std::isfinite(z)) return SRW_E_ARG;
    if (min_walks < 2 || max_walks < min_walks || max_walks > 8192) return SRW_E_ARG;
    if (options_ok(opt, A->n) != SRW_OK) return SRW_E_ARG;
    if (opt && !opt->one_step_exact) return SRW_E_ARG;  // the Section 5.1 rule runs the exact-one-step walks
    srw_options o;
    srw_default_options(&o);
    if (opt) o = *opt;
    try {
        return srw::adaptive_impl(A, seed, &o, delta, z, min_walks, max_walks, walks,
                                  as_stream(stream));
    } catch (const std::bad_alloc&) {
        return SRW_E_NOMEM;
    } catch (...) {
        return SRW_E_HIP;
    }
}

int srw_ordering(int64_t n, uint64_t seed, int32_t* rank, void* stream)
{
    if (n < 0 || n >= (int64_t)0x7FFFFFFF || (n > 0 && !rank)) return SRW_E_ARG;
    return srw::ordering_impl(n, seed, rank, as_stream(stream));
}

int srw_row_features(const srw_csr* A, const int32_t* rank, float* features, void* stream)
{
    if (!csr_ok(A)) return SRW_E_ARG;
    if (A->n > 0 && (!rank || !features)) return SRW_E_ARG;
    return srw::features_impl(A, rank, features, as_stream(stream));
}

int srw_budget_labels(const srw_factor* F, int32_t per_step, double* label, void* stream)
{
    if (!F || F->keep < 1 || (per_step != 0 && per_step != 1)) return SRW_E_ARG;
    if (F->n > 0 && !label) return SRW_E_ARG;
    return srw::labels_impl(F, per_step, label, as_stream(stream));
}

int srw_walk_stats(const srw_factor* F, double* visit_var, double* len_mean, void* stream)
{
    if (!F || F->keep < 1) return SRW_E_ARG;
    return srw::walk_stats_impl(F, visit_var, len_mean, as_stream(stream));
}

int srw_mlp_forward(const float* params, const float* mu_sd, const float* features, int64_t n,
                    float* out, void* stream)
{
    if (n < 0) return SRW_E_ARG;
    if (n > 0 && (!params || !mu_sd || !features || !out)) return SRW_E_ARG;
    return srw::mlp_forward_impl(params, mu_sd, features, n, out, as_stream(stream));
}

int srw_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t step, float lr,
                       const float* mu_sd, const float* features, const float* target,
                       int64_t n, float* grad, float* loss, void* stream)
{
    if (n < 0) return SRW_E_ARG;
    if ((adam_m == nullptr) != (adam_v == nullptr)) return SRW_E_ARG;
    if (adam_m && (step < 1 || !(lr > 0.0f) || !std::isfinite(lr))) return SRW_E_ARG;
    if (n > 0 && (!params || !mu_sd || !features || !target)) return SRW_E_ARG;
    return srw::mlp_train_impl(params, adam_m, adam_v, step, lr, mu_sd, features, target, nullptr,
                               n, n, grad, loss, as_stream(stream));
}

int srw_mlp_train_step_rows(float* params, float* adam_m, float* adam_v, int32_t step, float lr,
                            const float* mu_sd, const float* features, const float* target,
                            int64_t n_rows, const int32_t* rows, int64_t n, float* grad,
                            float* loss, void* stream)
{
    if (n < 0 || n_rows < 0) return SRW_E_ARG;
    if ((adam_m == nullptr) != (adam_v == nullptr)) return SRW_E_ARG;
    if (adam_m && (step < 1 || !(lr > 0.0f) || !std::isfinite(lr))) return SRW_E_ARG;
    if (n > 0 && (!params || !mu_sd || !features || !target || !rows)) return SRW_E_ARG;
    return srw::mlp_train_impl(params, adam_m, adam_v, step, lr, mu_sd, features, target, rows,
                               n_rows, n, grad, loss, as_stream(stream));
}

int srw_budget_targets(const double* label, const float* features, int64_t n, int32_t half,
                       float* x_out, float* y_out, int64_t* count, void* stream)
{
    if (n < 0 || !count || (half != 0 && half != 1)) return SRW_E_ARG;
    if (n > 0 && (!label || !features || !x_out || !y_out)) return SRW_E_ARG;
    return srw::budget_targets_impl(label, features, n, half, x_out, y_out, count,
                                    as_stream(stream));
}

int srw_mlp_standardize(const float* features, const float* target, int64_t n, float* mu_sd,
                        float* target_mean, void* stream)
{
    if (n < 1 || !features || !mu_sd || (!target) != (!target_mean)) return SRW_E_ARG;
    return srw::mlp_standardize_impl(features, target, n, mu_sd, target_mean, as_stream(stream));
}

int srw_mlp_budgets(const float* pred, int64_t n, double eps, int32_t lo, int32_t hi,
                    int32_t* walks, void* stream)
{
    if (n < 0 || !(eps > 0.0) || !std::isfinite(eps) || lo < 1 || hi < lo || hi > 8192)
        return SRW_E_ARG;
    if (n > 0 && (!pred || !walks)) return SRW_E_ARG;
    return srw::budgets_impl(pred, n, eps, lo, hi, walks, as_stream(stream));
}

const char* srw_last_error(void) { return srw::get_last_error(); }

const char* srw_status_string(int status)
{
    switch (status) {
        case SRW_OK: return "SRW_OK";
        case SRW_NOT_CONVERGED: return "SRW_NOT_CONVERGED: PCG reached max_iter";
        case SRW_E_ARG: return "SRW_E_ARG: malformed arguments or CSR structure";
        case SRW_E_NOT_RMATRIX: return "SRW_E_NOT_RMATRIX: matrix values violate the R-matrix definition";
        case SRW_E_SINGULAR: return "SRW_E_SINGULAR: a connected component has no path to ground";
        case SRW_E_WALK_LIMIT: return "SRW_E_WALK_LIMIT: a walk exceeded max_steps";
        case SRW_E_NOMEM: return "SRW_E_NOMEM: device allocation failed";
        case SRW_E_HIP: return "SRW_E_HIP: a HIP runtime call failed";
        default: return "unknown srw status";
    }
}

}  // extern "C"
