/*
 * gpmi.h -- C ABI of the MI355X (gfx950) Gaussian-process likelihood library.
 *
 * The library evaluates the hot path of maximum-likelihood fitting of a
 * Gaussian-process (geostatistical) model as set out in Section 1 of
 * Paciorek et al., "Parallelizing Gaussian Process Calculations in R"
 * (arXiv:1305.4886): build the covariance C(theta) from the locations, factor
 * it as L L^T = C, solve L^{-1}(y - mu), form the log-determinant and the
 * marginal log-likelihood, and predict (kriging mean and variance) at new
 * locations reusing the factor.  The paper's distributed block Cholesky
 * (Section 2.1-2.2, Fig. 1) is realised here on one GPU as a right-looking
 * blocked factorisation whose trailing updates run on the matrix cores.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - All matrices are column-major with an explicit leading dimension
 *    (element (i, j) at p[i + j * ld]) -- the column-wise block storage of the
 *    paper's Section 2.3.4.  Symmetric matrices use the lower triangle; the
 *    strict upper triangle is never read nor written.
 *  - Pointers marked [dev] are device pointers owned by the caller (e.g.
 *    torch.Tensor.data_ptr()); the library never allocates, frees or retains
 *    them past the call's stream position.  Pointers marked [host] are read
 *    during the call only.
 *  - Every call is asynchronous and ordered on the handle's stream.  The
 *    return value is a synchronous argument check:
 *        GP_OK (0)                        accepted and enqueued;
 *        -k  (k = 1..99)                  the k-th argument (1-based) is invalid;
 *        GP_ERR_* (below -1000)           see the list below.
 *    Numerical failure is reported on the device: *info_dev = 0, or the
 *    1-based index of the first column at which the matrix was found not to be
 *    positive definite (the LAPACK potrf convention; there is no pivoting, so a
 *    matrix that is not numerically positive definite fails -- Section 5), or
 *    -1 when one of the bounded waits between concurrently running workgroups
 *    gave up (a stall; never expected, but reported rather than hidden).  A
 *    failed evaluation writes NaN to its scalar outputs (and to alpha and the
 *    gradient where requested).
 *  - Workspace: the caller allocates `ws` (device memory, 256-byte aligned) of
 *    at least gp_workspace_size() bytes.  Its contents on entry are ignored.
 *  - theta is (log sigma^2, log rho, log tau^2); a log of -inf is an exact 0.
 *    Covariance (Section 1, C = C_y + C_g with diagonal C_y):
 *        C_ij = sigma^2 k(|x_i - x_j| / rho) + tau^2 [i == j]
 *    with k the exponential e^{-r}, Matern-3/2 (1 + sqrt3 r) e^{-sqrt3 r} or
 *    Matern-5/2 (1 + sqrt5 r + 5 r^2 / 3) e^{-sqrt5 r}; the nugget is attached
 *    to the index, not to coincident locations, and is absent from
 *    cross-covariances.
 */
#ifndef GPMI_H
#define GPMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GP_OK 0
#define GP_ERR_NONFINITE (-1001)    /* a host scalar (theta, mu, tolerance) is NaN/Inf where not allowed */
#define GP_ERR_WS_TOO_SMALL (-1002) /* ws_bytes < gp_workspace_size() */
#define GP_ERR_HIP (-1003)          /* a HIP runtime call failed (no device, launch failure, ...) */
#define GP_ERR_NOT_SUPPORTED (-1004)/* combination of options not implemented */
#define GP_ERR_BAD_HANDLE (-1005)
#define GP_ERR_SCRATCH_LIMIT (-1006)/* gp_loglik_noalloc: the problem's workspace exceeds GP_SCRATCH_BYTES */
#define GP_ERR_NO_CANDIDATE (-1007) /* an autotuner could time no candidate (each needs more workspace) */
#define GP_ERR_IO (-1008)           /* a tuning-table file could not be read, parsed or written */

/* Size of the static per-device workspace of gp_loglik_noalloc (128 MiB). */
#define GP_SCRATCH_BYTES (128u << 20)

typedef struct gp_handle_s *gp_handle_t;

/* Covariance families.  GP_SEP_MATERN2 is the family of the paper's spectral
 * example (Section 4.2): a point is (t, w, v) -- phase, log-wavelength and
 * the known noise variance of that observation (dim must be 3) -- and
 *     C_ij = sigma^2 M(|t_i - t_j| / rho) M(|w_i - w_j| / rho_w)
 *            + tau^2 [t_i == t_j] + v_i [i == j],
 *     M(r) = r^2 K_2(r) / 2   (Matern correlation of smoothness 2, range
 *                              scaling d / rho, K_2 the modified Bessel
 *                              function of the second kind),
 * i.e. a product of Matern correlations in phase and log-wavelength, a
 * random effect of variance tau^2 shared by the observations of one phase,
 * and heteroscedastic noise.  Cross-covariances carry the first term only.
 * Its gradient has four components (log sigma^2, log rho, log tau^2,
 * log rho_w).  gp_loglik_batched does not take it. */
typedef enum { GP_EXP = 0, GP_MATERN32 = 1, GP_MATERN52 = 2, GP_SEP_MATERN2 = 3 } gp_kernel_t;

/* Precision of the Cholesky trailing updates.  Diagonal-block factorisations,
 * panel solves, the log-determinant and all residuals stay in FP64 in every
 * mode; FP32_TRAIL / BF16_TRAIL run the trailing products on the FP32 / BF16
 * matrix cores with FP32 accumulation, added into FP64 storage. */
typedef enum { GP_FP64 = 0, GP_FP32_TRAIL = 1, GP_BF16_TRAIL = 2 } gp_prec_t;

typedef enum { GP_NOTRANS = 0, GP_TRANS = 1 } gp_trans_t;

typedef enum {
    GP_OP_POTRF = 0, GP_OP_TRSV = 1, GP_OP_TRSM = 2, GP_OP_LOGLIK = 3,
    GP_OP_LOGLIK_GRAD = 4, GP_OP_KRIGE = 5, GP_OP_BATCHED = 6, GP_OP_MORTON = 7,
    GP_OP_KRIGE_COV = 8, GP_OP_TRMM = 9, GP_OP_SIMULATE = 10
} gp_op_t;

typedef struct {
    int32_t kind;      /* gp_kernel_t */
    double log_sigma2; /* log of the spatial variance sigma^2  */
    double log_rho;    /* log of the range rho (> 0)           */
    double log_tau2;   /* log of the nugget variance tau^2 (GP_SEP_MATERN2: the per-phase
                          random-effect variance) */
    double log_rho2;   /* GP_SEP_MATERN2 only: log of the log-wavelength range rho_w */
} gp_theta_t;

typedef struct {
    int32_t nb;          /* outer panel width of the Cholesky, multiple of 64 (0 = automatic: 768 for FP64,
                            512 for FP32 trailing updates, 640 for BF16) */
    int32_t lookahead;   /* 1: factor panel k+1 on a side stream while the trailing update of k runs */
    int32_t band;        /* mixed modes: tiles within `band` 128-tile diagonals of the diagonal use FP64 */
    int32_t ir_max_iter; /* mixed modes: cap on iterative-refinement sweeps (0 = no refinement) */
    double ir_tol;       /* mixed modes: stop when |r - C x| / |r| <= ir_tol (FP64 residual) */
    int32_t reorder;     /* mixed modes: 1 = order the points along a Morton curve inside gp_loglik* */
    int32_t panel_cus;   /* compute units kept free of trailing updates for the lookahead chain
                            (0 = none: one shared stream pair without CU masks) */
    int32_t fused_panel; /* 1: each panel's diagonal block (factor, block inverses and, when rows
                            follow, its full inverse) in one launch of concurrent workgroups
                            (panels up to 1024 columns); 0: a chain of per-64-column launches */
    int32_t batch_grid;  /* gp_loglik_batched: 0 = one persistent launch with one workgroup per compute
                            unit; > 0 = a persistent launch of that many workgroups; -1 = level-synchronous
                            launches (three per tile column) */
    int32_t fail_inject; /* test hook, 0 in normal use.  Bit 0: the abort flag of the fused panel kernel
                            is raised before it starts; bit 1: that of every triangular solve inside
                            gp_loglik / gp_loglik_grad.  Every bounded wait then gives up at once and
                            the evaluation reports a stall (info = -1, NaN outputs) without any kernel
                            running into its time limit. */
    int32_t bf16_split;  /* GP_BF16_TRAIL: 1 (default) = each trailing product formed from hi and lo
                            BF16 parts of the panel (x = hi + lo, hi = bf16(x), lo = bf16(x - hi);
                            hi hi^T + hi lo^T + lo hi^T on the BF16 matrix cores: about 16 significant
                            bits per operand instead of 8); 0 = one BF16 product */
    int32_t syrk_slab;   /* FP64 trailing update, 128 x 128 tiles: K-slab shape staged through LDS per
                            barrier -- 16 columns in 2 stages (16, and 0 = default) or 8 columns in 4
                            stages (8).  Chosen per problem size by gp_tune_potrf. */
    int32_t batch_tile;  /* gp_loglik_batched, persistent launch: tile edge 64 or 128 (0 = automatic: the
                            tuning table's choice for the largest problem's size bucket, else 128).  The
                            level-synchronous launches (batch_grid = -1) always use 64. */
    int32_t tail_nb;     /* Cholesky: panel width once at most 24 x tail_nb columns remain to be factored,
                            where the chain of diagonal-block steps of a wide panel outlasts the trailing
                            update it overlaps (0 = automatic: 512; -1 = the outer width throughout).
                            Used only when narrower than the outer width; a multiple of 64 otherwise. */
} gp_options_t;

/* ---- handle ------------------------------------------------------------ */
/* Creates a handle bound to the current HIP device and to `stream` (a
 * hipStream_t; NULL = the null stream).  The handle owns one extra stream and
 * a few events for lookahead, but no device memory.  */
int gp_create(gp_handle_t *h, void *stream);
int gp_destroy(gp_handle_t h);
int gp_set_stream(gp_handle_t h, void *stream);
int gp_set_options(gp_handle_t h, const gp_options_t *opt); /* NULL restores defaults */
int gp_get_options(gp_handle_t h, gp_options_t *opt);
const char *gp_strerror(int code);

/* Kernel timing for measurement tools.  While enabled, every trailing-update
 * launch of the Cholesky (the matrix-core SYRK/GEMM that carries almost all of
 * its work, Section 2.1) is bracketed by events on the handle's stream.
 * gp_profile_read waits for those events and returns out4 [host, 4] =
 * {launches, total milliseconds, algorithmic flops, algorithmic bytes}
 * accumulated since the previous read, then resets the counters.  A launch
 * that updates E lower-triangle entries with a rank-K product counts 2 K E
 * flops and 16 E bytes (each entry read and written once in FP64). */
int gp_profile(gp_handle_t h, int enable);
int gp_profile_read(gp_handle_t h, double *out4);

/* Bytes of workspace the call `op` needs for problem size n (and m new points
 * for GP_OP_KRIGE, GP_OP_KRIGE_COV and GP_OP_SIMULATE (n = 0: no data) /
 * right-hand sides for GP_OP_TRSM and GP_OP_TRMM; for GP_OP_BATCHED, n is
 * the largest problem and m the number of problems).  The factorising calls
 * size a panel buffer by the handle's panel width: query after gp_set_options. */
int gp_workspace_size(gp_handle_t h, gp_op_t op, int64_t n, int64_t m, gp_prec_t prec,
                      size_t *bytes);

/* ---- covariance (Section 1: the entries of C(theta); Section 2.3.4) ------ */
/* Writes the lower triangle (i >= j) of the n x n covariance of the points X
 * [dev, n x dim row-major, 1 <= dim <= 16] into C [dev, ldc >= n]. */
int gp_cov_build(gp_handle_t h, gp_theta_t th, int64_t n, int32_t dim, const double *X,
                 double *C, int64_t ldc);

/* Cs[i + j*ldcs] = sigma^2 k(|X_i - Xs_j| / rho), n x m, no nugget. */
int gp_cross_cov_build(gp_handle_t h, gp_theta_t th, int64_t n, int64_t m, int32_t dim,
                       const double *X, const double *Xs, double *Cs, int64_t ldcs);

/* ---- blocked Cholesky (Section 2.1, Fig. 1; no pivoting, Section 5) ------ */
/* In place: the lower triangle of A [dev, lda >= n] is overwritten by L with
 * L L^T = A; the strict upper triangle is untouched.  *info_dev [dev] gets 0 or
 * the first failing 1-based column.  prec selects the trailing-update
 * arithmetic (gp_prec_t).  Right-looking by panels of opt.nb columns: the
 * panel's diagonal block is factored in 64-column steps and inverted, the rows
 * below it are multiplied by that inverse, then the trailing matrix is
 * updated; with opt.lookahead the next panel's diagonal block is factored on a
 * second stream during that update.  An even lda with A 16-byte aligned lets
 * the FP64 trailing updates stream the panel with 16-byte copies (the faster
 * form); with odd n those copies also read A's row n (inside the storage,
 * since lda > n), whose contents never reach L. */
int gp_potrf(gp_handle_t h, gp_prec_t prec, int64_t n, double *A, int64_t lda,
             int32_t *info_dev, void *ws, size_t ws_bytes);

/* Autotuner for gp_potrf's panel width, reserved compute units and (FP64)
 * trailing-update tile shape: for each pair (nb_cand[a], cu_cand[b]) [host
 * arrays; nb a positive multiple of 64, panel_cus >= 0] and, in FP64, each
 * K-slab shape of the 128 x 128 trailing-update tile (16 columns x 2 stages,
 * 8 x 4), it fills A [dev, lda >= n; overwritten] with a synthetic
 * positive-definite matrix of order n (exp(-8 |i - j| / n) + I), times
 * gp_potrf with lookahead on the handle's stream (HIP events, second of two
 * runs) and writes the milliseconds of the faster tile shape to
 * ms_out[a * n_cu + b] [host, may be NULL; -1 where the candidate's workspace
 * exceeds ws_bytes].  The fastest choice is stored in the handle's options
 * (nb, lookahead = 1, panel_cus, syrk_slab) and in its tuning table for
 * (prec, floor(log2 n)), which gp_potrf and every factorising call consult
 * when options.nb is 0 (automatic); on error the options are left
 * unchanged.  Returns GP_ERR_NO_CANDIDATE when no candidate fits in ws (it
 * must hold gp_workspace_size(GP_OP_POTRF, n)).  Synchronises the handle's
 * stream; info_dev [dev] is scratch. */
int gp_tune_potrf(gp_handle_t h, gp_prec_t prec, int64_t n, double *A, int64_t lda,
                  const int32_t *nb_cand, int32_t n_nb, const int32_t *cu_cand, int32_t n_cu,
                  int32_t *info_dev, double *ms_out, void *ws, size_t ws_bytes);

/* The factorisation's resolved choices for an n x n matrix at precision prec
 * under the handle's current options and tuning table (what gp_potrf and the
 * factorising calls would use): *nb = outer panel width, *panel_cus =
 * compute units reserved for the lookahead chain, *syrk_slab = K-slab shape
 * of the FP64 trailing-update tile (16 or 8), *tail_nb = width of the panels
 * that start where at most 24 x tail_nb columns remain (equal to *nb when the
 * width does not change) [host, each nullable].  No device work. */
int gp_potrf_plan(gp_handle_t h, gp_prec_t prec, int64_t n, int32_t *nb, int32_t *panel_cus, int32_t *syrk_slab,
                  int32_t *tail_nb);

/* ---- triangular solves with the lower factor (Section 1 "backsolve";
 *      the remoteForwardsolve / remoteBacksolve of Section 2.3.2) --------- */
/* x [dev, n] <- L^{-1} x (GP_NOTRANS) or L^{-T} x (GP_TRANS), in place. */
int gp_trsv(gp_handle_t h, gp_trans_t trans, int64_t n, const double *L, int64_t ldl, double *x,
            void *ws, size_t ws_bytes);
/* B [dev, n x nrhs, ldb >= n] <- L^{-1} B or L^{-T} B, in place. */
int gp_trsm(gp_handle_t h, gp_trans_t trans, int64_t n, int64_t nrhs, const double *L,
            int64_t ldl, double *B, int64_t ldb, void *ws, size_t ws_bytes);

/* ---- marginal log-likelihood (Section 1; Section 2.2.2: only scalars leave) */
/* Builds C(theta) into C [dev, ldc >= n], factors it in place, and writes
 * out3_dev [dev, 3] = {loglik, logdet, q} where
 *   logdet = log|C| = 2 sum log L_ii,  q = (y - mu)^T C^{-1} (y - mu),
 *   loglik = -1/2 (n log(2 pi) + logdet + q).
 * mu [dev, n] may be NULL (zero mean).  alpha_dev [dev, n] (nullable) receives
 * C^{-1}(y - mu) for reuse by gp_krige.  L stays in C.  In the mixed modes
 * q and alpha are refined in FP64 against the covariance regenerated from X
 * (ir_dev [dev, 3], nullable: {sweeps, final relative residual, converged}),
 * and, if options.reorder, the points are taken in Morton order internally:
 * L then belongs to the permuted points while alpha is returned in the
 * caller's order. */
int gp_loglik(gp_handle_t h, gp_theta_t th, gp_prec_t prec, int64_t n, int32_t dim,
              const double *X, const double *y, const double *mu, double *C, int64_t ldc,
              double *out3_dev, double *alpha_dev, int32_t *info_dev, double *ir_dev, void *ws,
              size_t ws_bytes);

/* gp_loglik for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): same
 * arguments, results and kernels as gp_loglik, without the workspace.  The
 * workspace is a static array of GP_SCRATCH_BYTES bytes that the library's
 * code object holds on every device it is loaded on until the process ends;
 * the call itself allocates nothing.  Returns GP_ERR_SCRATCH_LIMIT when
 * gp_workspace_size(GP_OP_LOGLIK, n, prec) exceeds GP_SCRATCH_BYTES (FP64
 * with the default panel width: n up to about 19,000) and
 * GP_ERR_NOT_SUPPORTED when options.panel_cus > 0 (that option creates
 * streams on first use).  The device current at the call must be the
 * handle's.  Every call on one device shares the array: calls that overlap
 * on one device (on different streams or handles) race and must be
 * serialised by the caller.  Nothing in the array needs to be cleared
 * between calls: every buffer in it is initialised by the call's own kernels. */
int gp_loglik_noalloc(gp_handle_t h, gp_theta_t th, gp_prec_t prec, int64_t n, int32_t dim,
                      const double *X, const double *y, const double *mu, double *C, int64_t ldc,
                      double *out3_dev, double *alpha_dev, int32_t *info_dev, double *ir_dev);

/* As gp_loglik, plus grad3_dev [dev, 3; 4 for GP_SEP_MATERN2, whose fourth
 * entry is d loglik / d log rho_w] = d loglik / d (log sigma^2, log rho,
 * log tau^2) by the adjoint 1/2 sum_ij (alpha_i alpha_j - (C^{-1})_ij) dC_ij /
 * dtheta (Rasmussen & Williams 2006, eq. 5.9), with C^{-1} formed from L on
 * the matrix cores and dC/dtheta regenerated from X.  On return C holds
 * C^{-1} (lower), not L. */
int gp_loglik_grad(gp_handle_t h, gp_theta_t th, gp_prec_t prec, int64_t n, int32_t dim,
                   const double *X, const double *y, const double *mu, double *C, int64_t ldc,
                   double *out3_dev, double *grad3_dev, double *alpha_dev, int32_t *info_dev,
                   double *ir_dev, void *ws, size_t ws_bytes);

/* ---- kriging (Section 1: prediction and its uncertainty; Section 2.2.2) -- */
/* Given the factor L [dev] and alpha = C^{-1}(y - mu) [dev] of the same
 * points X (as left by gp_loglik with reorder off), writes for the m new
 * points Xs [dev, m x dim]:
 *   mean_dev[j] = mu + c_j^T alpha,
 *   var_dev[j]  = sigma^2 - |L^{-1} c_j|^2 (+ tau^2 if include_nugget),
 * c_j the cross-covariance column.  var is not clamped at 0.  The m x n
 * cross-covariance is built transposed in the workspace and solved from the
 * right (C*^T L^{-T}) on the matrix cores; mean and variance are compensated
 * row sums. */
int gp_krige(gp_handle_t h, gp_theta_t th, int64_t n, int64_t m, int32_t dim, const double *X,
             const double *Xs, const double *L, int64_t ldl, const double *alpha, double mu,
             double *mean_dev, double *var_dev, int32_t include_nugget, void *ws,
             size_t ws_bytes);

/* Full prediction covariance at the m new points Xs [dev, m x dim] (Section 1:
 * the variance of the prediction; the full prediction variance matrix of the
 * kriging methods in Section 2.3.3, formed as the cross-product of
 * W = L^{-1} C* with itself, Section 2.3.2):
 *   S_ij = sigma^2 k(|s_i - s_j| / rho) (+ tau^2 [i == j] if include_nugget)
 *          - (W^T W)_ij,
 * written to the lower triangle of S [dev, m x m, lds >= m] (the strict upper
 * triangle is untouched).  L [dev] is the factor of the n data points X as
 * left by gp_loglik (reorder off).  With n = 0, S is the prior covariance of
 * the new points (X and L are not read).  W^T is built and solved from the
 * right in the workspace as in gp_krige; S -= W^T W is one SYRK on the matrix
 * cores.  Its diagonal equals gp_krige's variance. */
int gp_krige_cov(gp_handle_t h, gp_theta_t th, int64_t n, int64_t m, int32_t dim, const double *X,
                 const double *Xs, const double *L, int64_t ldl, int32_t include_nugget, double *S,
                 int64_t lds, void *ws, size_t ws_bytes);

/* Product with a lower-triangular matrix (the multiplication by the Cholesky
 * factor of Section 2.3.2 that turns independent normal draws into correlated
 * ones): out [dev, n x nrhs, ldo >= n] = L B, L [dev, n x n, ldl >= n] lower
 * (its strict upper triangle is not read), B [dev, n x nrhs, ldb >= n]; out
 * must not overlap B.  Workspace: gp_workspace_size(GP_OP_TRMM, n, nrhs). */
int gp_trmm(gp_handle_t h, int64_t n, int64_t nrhs, const double *L, int64_t ldl, const double *B,
            int64_t ldb, double *out, int64_t ldo, void *ws, size_t ws_bytes);

/* Realizations of the latent process at the m new points Xs (Section 1:
 * simulation of realizations, unconditional and conditional on the data;
 * the simulation method of Section 2.3.3):
 *   n = 0  (unconditional): mean_i = mu, S = prior covariance of the points;
 *   n > 0  (conditional on the data whose factor L and alpha = C^{-1}(y - mu)
 *           come from gp_loglik, reorder off): mean_i = mu + c_i^T alpha and
 *           S = the prediction covariance of gp_krige_cov;
 *   (+ tau^2 on the diagonal of S if include_nugget), then S = L_S L_S^T and
 *   out[:, r] = mean + L_S eps[:, r],   r = 0 .. nreal - 1.
 * eps [dev, m x nreal, ldeps >= m] holds the caller's standard normal draws;
 * out [dev, m x nreal, ldo >= m].  S [dev, m x m, lds >= m] is caller-owned
 * storage: on return it holds L_S with zeros above the diagonal.  The factor
 * has no pivoting (Section 5): when S is not numerically positive definite
 * (e.g. coincident new points without a nugget) *info_dev gets the failing
 * 1-based column and out is NaN.  Workspace: gp_workspace_size(GP_OP_SIMULATE,
 * n, m); the draws are multiplied 512 realizations at a time. */
int gp_simulate(gp_handle_t h, gp_theta_t th, int64_t n, int64_t m, int32_t dim, const double *X,
                const double *Xs, const double *L, int64_t ldl, const double *alpha, double mu,
                int32_t include_nugget, int64_t nreal, const double *eps, int64_t ldeps, double *out,
                int64_t ldo, double *S, int64_t lds, int32_t *info_dev, void *ws, size_t ws_bytes);

/* ---- many independent likelihoods in one call ------------------------------
 * Problem b has n_host[b] points starting at point x_off_host[b] of X [dev,
 * rows of dim doubles] and of y [dev]; its covariance/factor occupies
 * C_pool[c_off_host[b] + i + j * n_host[b]] (ld = n_b).  th_host[b] is its
 * parameter set.  Writes out3_dev[3 b + {0,1,2}] = {loglik, logdet, q} and
 * info_dev[b].  Same model and definitions as gp_loglik (FP64).  The
 * problems are factored together in square tiles (options batch_tile: 128
 * by default, or 64).  By default (options
 * batch_grid >= 0) one persistent launch takes every tile of every problem
 * as a task (covariance tile, left-looking update, then factor + inverse or
 * the product with the diagonal inverse), ordered so that each task's inputs
 * come from earlier tasks, with the forward solve and the reductions folded
 * into the diagonal tasks; a small launch before it resets the task flags.
 * batch_grid = -1 instead runs one tile column per step for all problems at
 * once (three launches per step plus one for the solves).  A stall of the
 * persistent launch (never expected) sets info_dev[b] = -1 and leaves NaN.
 * The workspace size query (GP_OP_BATCHED) covers every schedule and tile
 * edge unless batch_grid = -1 is set explicitly (the persistent launch keeps
 * a tile-major copy of the factors). */
int gp_loglik_batched(gp_handle_t h, int32_t nbatch, const gp_theta_t *th_host,
                      const int64_t *n_host, const int64_t *x_off_host, const int64_t *c_off_host,
                      int32_t dim, const double *X, const double *y, double *C_pool,
                      double *out3_dev, int32_t *info_dev, void *ws, size_t ws_bytes);

/* Autotuner for gp_loglik_batched's schedule: candidate c is the pair
 * (grid_cand[c], tile_cand[c]) [host; grid: -1 = level-synchronous launches,
 * 0 = one persistent workgroup per compute unit, > 0 = that many persistent
 * workgroups; tile: 64 or 128 = tile edge of the persistent launch, 0 = the
 * automatic choice; tile_cand may be NULL (every candidate keeps the
 * options' tile)].  Each candidate runs the batch given by the same arguments
 * as gp_loglik_batched twice on the handle's stream; ms_out[c] [host, may be
 * NULL] receives the milliseconds of the second run (-1 where the
 * candidate's workspace exceeds ws_bytes).  The fastest candidate is stored
 * in the handle's options (batch_grid, batch_tile) and in its tuning table
 * for the largest problem's size bucket; on error the options are left
 * unchanged (GP_ERR_NO_CANDIDATE: no candidate fits in ws).  C_pool, out3_dev
 * and info_dev are written as by gp_loglik_batched (they hold the last
 * candidate's results).  Synchronises the handle's stream.  Argument errors:
 * -13 grid_cand, -14 tile_cand, -15 n_cand, -17 ws. */
int gp_tune_batched(gp_handle_t h, int32_t nbatch, const gp_theta_t *th_host, const int64_t *n_host,
                    const int64_t *x_off_host, const int64_t *c_off_host, int32_t dim, const double *X,
                    const double *y, double *C_pool, double *out3_dev, int32_t *info_dev, const int32_t *grid_cand,
                    const int32_t *tile_cand, int32_t n_cand, double *ms_out, void *ws, size_t ws_bytes);

/* ---- the tuning table -------------------------------------------------------
 * The handle keeps the autotuners' choices per (operation, precision, size
 * bucket floor(log2 n)): panel width, reserved compute units and trailing-
 * update tile shape for the factorisation (used when options.nb = 0), the
 * schedule for the batched call (used when options.batch_grid = 0; bucket of
 * the largest problem).  gp_tune_save writes it to the text file `path` (one
 * line per entry, tagged with the device's architecture name);
 * gp_tune_load merges the entries of `path` that carry this device's
 * architecture (*loaded [host, nullable] = their count); gp_tune_clear
 * empties it.  File errors and malformed lines return GP_ERR_IO (nothing
 * merged). */
int gp_tune_save(gp_handle_t h, const char *path);
int gp_tune_load(gp_handle_t h, const char *path, int32_t *loaded);
int gp_tune_clear(gp_handle_t h);

/* ---- spatial ordering ----------------------------------------------------
 * perm_dev [dev, n] <- the permutation that sorts the points X [dev, n x 2]
 * by their 2 x 21-bit Morton (Z-order) code on the bounding box, ties broken
 * by index.  A symmetric permutation leaves loglik, its gradient and kriging
 * unchanged; it concentrates the large covariances near the diagonal. */
int gp_morton_order(gp_handle_t h, int64_t n, int32_t dim, const double *X, int64_t *perm_dev,
                    void *ws, size_t ws_bytes);

#ifdef __cplusplus
}
#endif
#endif /* GPMI_H */
