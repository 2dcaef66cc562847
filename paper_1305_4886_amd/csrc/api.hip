// api.hip -- the C ABI declared in include/gpmi.h: argument checks,
// workspace layout and the host-side orchestration of the kernels.
//
// Blocked Cholesky (Section 2.1, Fig. 1; the h = 1 schedule of Section 2.2 is
// the same dependency graph on one device): for each panel of nb columns,
//   for each 64-column sub-panel d:   factor + invert the diagonal block (LDS),
//                                     solve the rows below on the matrix cores,
//                                     update the rest of the panel;
//   then the trailing SYRK/GEMM update of everything to the right (matrix cores).
// With lookahead the columns of panel k+1 are updated first and panel k+1 is
// factored on a second stream while the rest of panel k's trailing update
// runs, which keeps the diagonal-block chain (the critical path of Section 2.1)
// off the critical path of the device.
#include <math.h>
#include <string.h>

#include <new>

#include "internal.h"

// from k_cov.hip
int resid_chunks(int64_t n);

namespace {

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int64_t nblocks(int64_t n) { return (n + DB - 1) / DB; }

bool ok_handle(gp_handle_t h) { return h && h->magic == 0x67706d69; }

// theta check: log sigma^2 and log tau^2 may be -inf (an exact zero), never
// +inf or NaN; log rho must be finite.
int check_theta(const gp_theta_t &th) {
    if (th.kind < GP_EXP || th.kind > GP_MATERN52) return 1;
    if (isnan(th.log_sigma2) || th.log_sigma2 == INFINITY) return 2;
    if (!isfinite(th.log_rho)) return 2;
    if (isnan(th.log_tau2) || th.log_tau2 == INFINITY) return 2;
    return 0;
}

CovParams cov_params(const gp_theta_t &th, int dim) {
    CovParams p;
    p.kind = th.kind;
    p.dim = dim;
    p.s2 = exp(th.log_sigma2);
    p.inv_rho = exp(-th.log_rho);
    p.t2 = exp(th.log_tau2);
    return p;
}

// ---- workspace layouts ------------------------------------------------------
struct Layout {
    size_t dinv = 0, sync = 0, z = 0, vec2 = 0, vec3 = 0, part = 0, big1 = 0, big2 = 0, total = 0;
};

constexpr int GRAD_PARTS = 2048;

Layout layout(gp_op_t op, int64_t n, int64_t m, gp_prec_t prec) {
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += al256(bytes);
        return o;
    };
    const int64_t nb = nblocks(n);
    const size_t vec = sizeof(double) * (size_t)(n > 0 ? n : 1);
    switch (op) {
    case GP_OP_POTRF:
        L.dinv = take(sizeof(double) * DB * DB * (size_t)nb);
        break;
    case GP_OP_TRSV:
        L.dinv = take(sizeof(double) * DB * DB * (size_t)nb);
        L.sync = take(sizeof(int) * (size_t)(nb + 2));
        break;
    case GP_OP_TRSM:
        L.dinv = take(sizeof(double) * DB * DB * (size_t)nb);
        L.big1 = take(sizeof(double) * DB * (size_t)(m > 0 ? m : 1));
        break;
    case GP_OP_LOGLIK:
    case GP_OP_LOGLIK_GRAD:
        L.dinv = take(sizeof(double) * DB * DB * (size_t)nb);
        L.sync = take(sizeof(int) * (size_t)(nb + 2));
        L.z = take(vec);
        L.vec2 = take(vec);
        L.vec3 = take(vec);
        L.part = take(sizeof(double) * (size_t)(6 * GRAD_PARTS > 4 * (n + 8) ? 6 * GRAD_PARTS : 4 * (n + 8)));
        if (prec != GP_FP64) {
            // residual partials of the matrix-free FP64 residual
            L.big2 = take(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)resid_chunks(n > 0 ? n : 1));
        }
        if (op == GP_OP_LOGLIK_GRAD) {
            // W = L^{-1} (n x n) for the explicit inverse
            L.big1 = take(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1));
        }
        break;
    case GP_OP_KRIGE:
        L.dinv = take(sizeof(double) * DB * DB * (size_t)nb);
        L.big1 = take(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)(m > 0 ? m : 1));
        L.part = take(sizeof(double) * DB * (size_t)(m > 0 ? m : 1));
        break;
    default:
        break;
    }
    L.total = off < 256 ? 256 : off;
    return L;
}

template <typename T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) return GP_ERR_HIP;                                                   \
    } while (0)

// Trailing update, bracketed by events when the handle profiles.
hipError_t trailing(gp_handle_t h, hipStream_t s, gp_prec_t prec, const double *P, int64_t ldp, double *C,
                    int64_t ldc, int64_t M, int64_t N, int64_t K, const int32_t *info) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->prof) {
        while (h->prof_ev.size() < h->prof_used + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
            h->prof_ev.push_back(e);
        }
        e0 = h->prof_ev[h->prof_used];
        e1 = h->prof_ev[h->prof_used + 1];
        h->prof_used += 2;
        hipEventRecord(e0, s);
    }
    hipError_t e = launch_syrk_lower(s, prec, h->opt.band, P, ldp, C, ldc, M, N, K, info, 1);
    if (h->prof) {
        hipEventRecord(e1, s);
        h->prof_flops += syrk_flops(M, N, K);
        h->prof_launches += 1;
    }
    return e;
}

// ---- blocked Cholesky -------------------------------------------------------
int potrf_impl(gp_handle_t h, gp_prec_t prec, int64_t n, double *A, int64_t lda, int32_t *info,
               double *dinv) {
    hipStream_t s = h->stream;
    const int64_t NB = h->opt.nb > 0 ? h->opt.nb : 256;
    HIPCHK(launch_set_info(s, info));
    if (n <= 0) return GP_OK;

    auto factor_panel = [&](hipStream_t st, int64_t c0) -> int {
        const int64_t c1 = (c0 + NB < n) ? c0 + NB : n;
        for (int64_t d = c0; d < c1; d += DB) {
            const int jb = (int)((n - d) < DB ? (n - d) : DB);
            double *W = dinv + (d / DB) * DB * DB;
            HIPCHK(launch_diag_potrf(st, A + d + d * lda, lda, jb, W, info, d));
            const int64_t M = n - d - jb;
            if (M > 0) HIPCHK(launch_panel_solve(st, A + (d + jb) + d * lda, lda, W, M, jb, info));
            const int64_t nc = c1 - (d + jb);
            if (nc > 0 && M > 0)
                HIPCHK(launch_syrk_lower(st, GP_FP64, -1, A + (d + jb) + d * lda, lda,
                                         A + (d + jb) + (d + jb) * lda, lda, M, nc, jb, info, 2));
        }
        return GP_OK;
    };

    int rc = factor_panel(s, 0);
    if (rc) return rc;
    for (int64_t c0 = 0; c0 < n; c0 += NB) {
        const int64_t c1 = (c0 + NB < n) ? c0 + NB : n;
        if (c1 >= n) break;
        const int64_t K = c1 - c0;
        const int64_t c2 = (c1 + NB < n) ? c1 + NB : n;
        if (h->opt.lookahead) {
            // columns of the next panel first
            HIPCHK(trailing(h, s, prec, A + c1 + c0 * lda, lda, A + c1 + c1 * lda, lda, n - c1, c2 - c1, K,
                            info));
            HIPCHK(hipEventRecord(h->ev_cols, s));
            HIPCHK(hipStreamWaitEvent(h->side, h->ev_cols, 0));
            rc = factor_panel(h->side, c1);
            if (rc) return rc;
            HIPCHK(hipEventRecord(h->ev_panel, h->side));
            if (c2 < n)
                HIPCHK(trailing(h, s, prec, A + c2 + c0 * lda, lda, A + c2 + c2 * lda, lda, n - c2, n - c2,
                                K, info));
            HIPCHK(hipStreamWaitEvent(s, h->ev_panel, 0));
        } else {
            HIPCHK(trailing(h, s, prec, A + c1 + c0 * lda, lda, A + c1 + c1 * lda, lda, n - c1, n - c1, K,
                            info));
            rc = factor_panel(s, c1);
            if (rc) return rc;
        }
    }
    return GP_OK;
}

}  // namespace

// ============================================================================
extern "C" {

const char *gp_strerror(int code) {
    if (code == GP_OK) return "success";
    if (code == GP_ERR_NONFINITE) return "non-finite scalar argument";
    if (code == GP_ERR_WS_TOO_SMALL) return "workspace smaller than gp_workspace_size()";
    if (code == GP_ERR_HIP) return "HIP runtime error";
    if (code == GP_ERR_NOT_SUPPORTED) return "option combination not supported";
    if (code == GP_ERR_BAD_HANDLE) return "invalid handle";
    if (code < 0 && code > -100) return "invalid argument (index = -code)";
    return "unknown status";
}

static void default_options(gp_options_t *o) {
    memset(o, 0, sizeof(*o));
    o->nb = 256;
    o->lookahead = 1;
    o->band = 2;
    o->ir_max_iter = 20;
    o->ir_tol = 1e-10;
    o->reorder = 1;
}

int gp_create(gp_handle_t *h, void *stream) {
    if (!h) return -1;
    *h = nullptr;
    gp_handle_s *p = new (std::nothrow) gp_handle_s();
    if (!p) return GP_ERR_HIP;
    default_options(&p->opt);
    p->stream = (hipStream_t)stream;
    if (hipGetDevice(&p->device) != hipSuccess ||
        hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_cols, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_panel, hipEventDisableTiming) != hipSuccess) {
        if (p->side) hipStreamDestroy(p->side);
        if (p->ev_cols) hipEventDestroy(p->ev_cols);
        if (p->ev_panel) hipEventDestroy(p->ev_panel);
        delete p;
        return GP_ERR_HIP;
    }
    *h = p;
    return GP_OK;
}

int gp_profile(gp_handle_t h, int enable) {
    if (!ok_handle(h)) return -1;
    h->prof = enable ? 1 : 0;
    return GP_OK;
}

int gp_profile_read(gp_handle_t h, double *out3) {
    if (!ok_handle(h)) return -1;
    if (!out3) return -2;
    double ms = 0.0;
    for (size_t i = 0; i + 1 < h->prof_used; i += 2) {
        if (hipEventSynchronize(h->prof_ev[i + 1]) != hipSuccess) return GP_ERR_HIP;
        float t = 0.f;
        if (hipEventElapsedTime(&t, h->prof_ev[i], h->prof_ev[i + 1]) != hipSuccess) return GP_ERR_HIP;
        ms += t;
    }
    out3[0] = (double)h->prof_launches;
    out3[1] = ms;
    out3[2] = h->prof_flops;
    h->prof_used = 0;
    h->prof_launches = 0;
    h->prof_flops = 0.0;
    return GP_OK;
}

int gp_destroy(gp_handle_t h) {
    if (!ok_handle(h)) return -1;
    for (hipEvent_t e : h->prof_ev) hipEventDestroy(e);
    hipStreamSynchronize(h->side);
    hipStreamDestroy(h->side);
    hipEventDestroy(h->ev_cols);
    hipEventDestroy(h->ev_panel);
    h->magic = 0;
    delete h;
    return GP_OK;
}

int gp_set_stream(gp_handle_t h, void *stream) {
    if (!ok_handle(h)) return -1;
    h->stream = (hipStream_t)stream;
    return GP_OK;
}

int gp_set_options(gp_handle_t h, const gp_options_t *opt) {
    if (!ok_handle(h)) return -1;
    if (!opt) {
        default_options(&h->opt);
        return GP_OK;
    }
    if (opt->nb < 0 || opt->nb % DB != 0) return -2;
    if (opt->ir_max_iter < 0 || opt->band < -1) return -2;
    if (!(opt->ir_tol >= 0.0) || isinf(opt->ir_tol)) return GP_ERR_NONFINITE;
    h->opt = *opt;
    return GP_OK;
}

int gp_get_options(gp_handle_t h, gp_options_t *opt) {
    if (!ok_handle(h)) return -1;
    if (!opt) return -2;
    *opt = h->opt;
    return GP_OK;
}

int gp_workspace_size(gp_handle_t h, gp_op_t op, int64_t n, int64_t m, gp_prec_t prec, size_t *bytes) {
    if (!ok_handle(h)) return -1;
    if ((int)op < GP_OP_POTRF || (int)op > GP_OP_MORTON) return -2;
    if (n < 0) return -3;
    if (m < 0) return -4;
    if ((int)prec < GP_FP64 || (int)prec > GP_BF16_TRAIL) return -5;
    if (!bytes) return -6;
    *bytes = layout(op, n, m, prec).total;
    return GP_OK;
}

int gp_cov_build(gp_handle_t h, gp_theta_t th, int64_t n, int32_t dim, const double *X, double *C,
                 int64_t ldc) {
    if (!ok_handle(h)) return -1;
    if (int e = check_theta(th)) return e == 1 ? -2 : GP_ERR_NONFINITE;
    if (n < 0) return -3;
    if (dim < 1 || dim > 16) return -4;
    if (n > 0 && !X) return -5;
    if (n > 0 && !C) return -6;
    if (ldc < (n > 1 ? n : 1)) return -7;
    HIPCHK(launch_cov_lower(h->stream, cov_params(th, dim), n, X, C, ldc, nullptr));
    return GP_OK;
}

int gp_cross_cov_build(gp_handle_t h, gp_theta_t th, int64_t n, int64_t m, int32_t dim, const double *X,
                       const double *Xs, double *Cs, int64_t ldcs) {
    if (!ok_handle(h)) return -1;
    if (int e = check_theta(th)) return e == 1 ? -2 : GP_ERR_NONFINITE;
    if (n < 0) return -3;
    if (m < 0) return -4;
    if (dim < 1 || dim > 16) return -5;
    if (n > 0 && !X) return -6;
    if (m > 0 && !Xs) return -7;
    if (n > 0 && m > 0 && !Cs) return -8;
    if (ldcs < (n > 1 ? n : 1)) return -9;
    HIPCHK(launch_cross_cov(h->stream, cov_params(th, dim), n, m, X, Xs, Cs, ldcs));
    return GP_OK;
}

int gp_potrf(gp_handle_t h, gp_prec_t prec, int64_t n, double *A, int64_t lda, int32_t *info_dev,
             void *ws, size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if ((int)prec < GP_FP64 || (int)prec > GP_BF16_TRAIL) return -2;
    if (n < 0) return -3;
    if (n > 0 && !A) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (!info_dev) return -6;
    Layout L = layout(GP_OP_POTRF, n, 0, prec);
    if (!ws) return -7;
    if (ws_bytes < L.total) return GP_ERR_WS_TOO_SMALL;
    if (prec != GP_FP64) return GP_ERR_NOT_SUPPORTED;
    return potrf_impl(h, prec, n, A, lda, info_dev, at<double>(ws, L.dinv));
}

int gp_trsv(gp_handle_t h, gp_trans_t trans, int64_t n, const double *L, int64_t ldl, double *x, void *ws,
            size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (trans != GP_NOTRANS && trans != GP_TRANS) return -2;
    if (n < 0) return -3;
    if (n > 0 && !L) return -4;
    if (ldl < (n > 1 ? n : 1)) return -5;
    if (n > 0 && !x) return -6;
    Layout lay = layout(GP_OP_TRSV, n, 0, GP_FP64);
    if (!ws) return -7;
    if (ws_bytes < lay.total) return GP_ERR_WS_TOO_SMALL;
    if (n == 0) return GP_OK;
    double *dinv = at<double>(ws, lay.dinv);
    HIPCHK(launch_diag_inv(h->stream, L, ldl, n, dinv));
    HIPCHK(launch_trsv(h->stream, trans == GP_TRANS, L, ldl, x, n, dinv, at<int>(ws, lay.sync), nullptr));
    return GP_OK;
}

int gp_trsm(gp_handle_t h, gp_trans_t trans, int64_t n, int64_t nrhs, const double *L, int64_t ldl,
            double *B, int64_t ldb, void *ws, size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (trans != GP_NOTRANS && trans != GP_TRANS) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (n > 0 && !L) return -5;
    if (ldl < (n > 1 ? n : 1)) return -6;
    if (n > 0 && nrhs > 0 && !B) return -7;
    if (ldb < (n > 1 ? n : 1)) return -8;
    if (!ws) return -9;
    (void)ws_bytes;
    return GP_ERR_NOT_SUPPORTED;
}

int gp_loglik(gp_handle_t h, gp_theta_t th, gp_prec_t prec, int64_t n, int32_t dim, const double *X,
              const double *y, const double *mu, double *C, int64_t ldc, double *out3_dev,
              double *alpha_dev, int32_t *info_dev, double *ir_dev, void *ws, size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (int e = check_theta(th)) return e == 1 ? -2 : GP_ERR_NONFINITE;
    if ((int)prec < GP_FP64 || (int)prec > GP_BF16_TRAIL) return -3;
    if (n < 0) return -4;
    if (dim < 1 || dim > 16) return -5;
    if (n > 0 && !X) return -6;
    if (n > 0 && !y) return -7;
    if (n > 0 && !C) return -9;
    if (ldc < (n > 1 ? n : 1)) return -10;
    if (!out3_dev) return -11;
    if (!info_dev) return -13;
    Layout lay = layout(GP_OP_LOGLIK, n, 0, prec);
    if (!ws) return -15;
    if (ws_bytes < lay.total) return GP_ERR_WS_TOO_SMALL;
    if (prec != GP_FP64) return GP_ERR_NOT_SUPPORTED;
    (void)ir_dev;
    hipStream_t s = h->stream;
    double *dinv = at<double>(ws, lay.dinv);
    int *sync = at<int>(ws, lay.sync);
    double *z = at<double>(ws, lay.z);
    HIPCHK(launch_cov_lower(s, cov_params(th, dim), n, X, C, ldc, nullptr));
    int rc = potrf_impl(h, prec, n, C, ldc, info_dev, dinv);
    if (rc) return rc;
    HIPCHK(launch_sub_mu(s, n, y, mu, z));
    HIPCHK(launch_trsv(s, 0, C, ldc, z, n, dinv, sync, info_dev));
    HIPCHK(launch_loglik_reduce(s, n, C, ldc, z, out3_dev, info_dev, sync));
    if (alpha_dev) {
        HIPCHK(launch_copy_vec(s, n, z, alpha_dev));
        HIPCHK(launch_trsv(s, 1, C, ldc, alpha_dev, n, dinv, sync, info_dev));
    }
    return GP_OK;
}

int gp_loglik_grad(gp_handle_t h, gp_theta_t th, gp_prec_t prec, int64_t n, int32_t dim, const double *X,
                   const double *y, const double *mu, double *C, int64_t ldc, double *out3_dev,
                   double *grad3_dev, double *alpha_dev, int32_t *info_dev, double *ir_dev, void *ws,
                   size_t ws_bytes) {
    (void)h; (void)th; (void)prec; (void)n; (void)dim; (void)X; (void)y; (void)mu; (void)C; (void)ldc;
    (void)out3_dev; (void)grad3_dev; (void)alpha_dev; (void)info_dev; (void)ir_dev; (void)ws; (void)ws_bytes;
    return GP_ERR_NOT_SUPPORTED;
}

int gp_krige(gp_handle_t h, gp_theta_t th, int64_t n, int64_t m, int32_t dim, const double *X,
             const double *Xs, const double *L, int64_t ldl, const double *alpha, double mu,
             double *mean_dev, double *var_dev, int32_t include_nugget, void *ws, size_t ws_bytes) {
    (void)h; (void)th; (void)n; (void)m; (void)dim; (void)X; (void)Xs; (void)L; (void)ldl; (void)alpha;
    (void)mu; (void)mean_dev; (void)var_dev; (void)include_nugget; (void)ws; (void)ws_bytes;
    return GP_ERR_NOT_SUPPORTED;
}

int gp_loglik_batched(gp_handle_t h, int32_t nbatch, const gp_theta_t *th_host, const int64_t *n_host,
                      const int64_t *x_off_host, const int64_t *c_off_host, int32_t dim, const double *X,
                      const double *y, double *C_pool, double *out3_dev, int32_t *info_dev, void *ws,
                      size_t ws_bytes) {
    (void)h; (void)nbatch; (void)th_host; (void)n_host; (void)x_off_host; (void)c_off_host; (void)dim;
    (void)X; (void)y; (void)C_pool; (void)out3_dev; (void)info_dev; (void)ws; (void)ws_bytes;
    return GP_ERR_NOT_SUPPORTED;
}

int gp_morton_order(gp_handle_t h, int64_t n, int32_t dim, const double *X, int64_t *perm_dev, void *ws,
                    size_t ws_bytes) {
    (void)h; (void)n; (void)dim; (void)X; (void)perm_dev; (void)ws; (void)ws_bytes;
    return GP_ERR_NOT_SUPPORTED;
}

}  // extern "C"
