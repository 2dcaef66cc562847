/*
 * gp_oracle.c -- plain, slow CPU reference for the Gaussian-process
 * marginal-likelihood path (Paciorek et al., "Parallelizing Gaussian Process
 * Calculations in R", arXiv:1305.4886).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
 * compared against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares no
 * code, header, table or helper with the HIP library.
 *
 * Everything is IEEE double.  Matrices passed in or out are column-major with
 * an explicit leading dimension, lower triangle meaningful.  Build with
 *   gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC gp_oracle.c -lm
 * so that no fused multiply-add or reassociation changes the written order of
 * any sum.  OpenMP only splits independent rows of one column; the order of
 * every individual sum is fixed and ascending.
 *
 * Parameters theta are natural logs: th[0] = log sigma^2, th[1] = log rho,
 * th[2] = log tau^2 (the optimiser's coordinates of Section 1's marginal
 * likelihood).  A log of -inf gives an exact zero variance component.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t i64;

/* ------------------------------------------------------------------ */
/* Covariance functions (model of Section 1: C = C_y + C_g).           */
/* k(r) is the correlation at scaled distance r = |x_i - x_j| / rho;   */
/* g(r) = -r k'(r) is what d/d(log rho) of sigma^2 k(|d|/rho) needs.    */
/* ------------------------------------------------------------------ */
static double corr_k(int kind, double r)
{
    if (kind == 0) return exp(-r);                                 /* exponential   */
    if (kind == 1) { double a = sqrt(3.0) * r; return (1.0 + a) * exp(-a); }      /* Matern 3/2 */
    { double a = sqrt(5.0) * r; return (1.0 + a + a * a / 3.0) * exp(-a); }       /* Matern 5/2 */
}

static double corr_g(int kind, double r)
{
    if (kind == 0) return r * exp(-r);
    if (kind == 1) { double a = sqrt(3.0) * r; return 3.0 * r * r * exp(-a); }
    { double a = sqrt(5.0) * r; return (5.0 / 3.0) * r * r * (1.0 + a) * exp(-a); }
}

static double dist(int dim, const double *xi, const double *xj)
{
    double s = 0.0;
    for (int d = 0; d < dim; ++d) { double t = xi[d] - xj[d]; s += t * t; }
    return sqrt(s);
}

/* ------------------------------------------------------------------ */
/* The example's covariance family (Section 4.2): a Gaussian process    */
/* in phase t and log-wavelength w with a product of two Matern         */
/* correlations of smoothness 2, a random effect shared by all          */
/* observations of one phase, and known per-observation noise           */
/* variances.  A point is (t, w, v) with v its noise variance.  With    */
/* th[0] = log sigma^2, th[1] = log rho_t, th[2] = log tau^2 (the       */
/* random-effect variance), th[3] = log rho_w:                          */
/*   C_ij = sigma^2 M(|t_i - t_j|/rho_t) M(|w_i - w_j|/rho_w)           */
/*          + tau^2 [t_i == t_j] + v_i [i == j],                        */
/*   M(r) = 2^{1-nu} / Gamma(nu) r^nu K_nu(r) = r^2 K_2(r) / 2  (nu = 2), */
/* the Matern correlation as parameterised by the package the example   */
/* loads for it (range scaling d / rho, no sqrt(2 nu)).                 */
/* ------------------------------------------------------------------ */

/* exp(x) K_nu(x), x > 0, nu = 1 or 2, from the integral
 *   K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt
 * (Abramowitz & Stegun 9.6.24) by the trapezoidal rule, summed until the
 * terms fall below 1e-19 of the sum.  The integrand is analytic and decays
 * double-exponentially, so the rule converges geometrically in 1/step; for
 * large x the integrand is a peak of width about x^{-1/2} at t = 0 and the
 * error behaves like exp(-(2 pi / step)^2 / (2 x)), so the step is
 * min(1/16, 0.6 / sqrt(x)) (exponent below -54 for every x).  cosh t - 1 is
 * formed as 2 sinh^2(t/2).                                                 */
static double bessel_k_scaled(int nu, double x)
{
    const double h = fmin(1.0 / 16.0, 0.6 / sqrt(x));
    double s = 0.5;
    for (int k = 1; k < 20000; ++k) {
        double t = k * h, sh = sinh(0.5 * t);
        double e = exp(-x * 2.0 * sh * sh);
        double term = e * cosh(nu * t);
        s += term;
        if (term < 1e-19 * s && x * 2.0 * sh * sh > 1.0) break;
    }
    return h * s;
}

/* M(r) = r^2 K_2(r) / 2 and g(r) = -r M'(r) = r^3 K_1(r) / 2
 * (d/dr [r^2 K_2(r)] = -r^2 K_1(r), A&S 9.6.28).                        */
static double sep_m(double r)
{
    if (r == 0.0) return 1.0;
    return 0.5 * r * r * exp(-r) * bessel_k_scaled(2, r);
}
static double sep_g(double r)
{
    if (r == 0.0) return 0.0;
    return 0.5 * r * r * r * exp(-r) * bessel_k_scaled(1, r);
}

/* Covariance entry between points i and j (same_index: i == j) of any
 * family; cross-covariances (to new points) take neither nugget, random
 * effect nor noise. */
static double cov_entry(int kind, const double *th, int dim, const double *xi, const double *xj,
                        int same_index, int cross)
{
    const double s2 = exp(th[0]), rho = exp(th[1]), t2 = exp(th[2]);
    if (kind == 3) {
        const double rw = exp(th[3]);
        double v = s2 * sep_m(fabs(xi[0] - xj[0]) / rho) * sep_m(fabs(xi[1] - xj[1]) / rw);
        if (!cross) {
            if (xi[0] == xj[0]) v += t2;
            if (same_index) v += xi[2];
        }
        return v;
    }
    double r = dist(dim, xi, xj) / rho;
    return s2 * corr_k(kind, r) + ((same_index && !cross) ? t2 : 0.0);
}

/* Neumaier-compensated running sum. */
typedef struct { double s, c; } csum;
static void cs_add(csum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v; else a->c += (v - t) + a->s;
    a->s = t;
}
static double cs_val(const csum *a) { return a->s + a->c; }

/* C_ij = sigma^2 k(|x_i - x_j|/rho) + tau^2 [i == j]; full square written.
 * The nugget goes with the index (i == j), not with coincident locations. */
int orc_cov(int kind, const double th[4], i64 n, int dim, const double *X, double *C, i64 ldc)
{
    if (n < 0 || ldc < (n > 0 ? n : 1)) return -1;
#pragma omp parallel for schedule(static)
    for (i64 j = 0; j < n; ++j)
        for (i64 i = 0; i < n; ++i)
            C[i + j * ldc] = cov_entry(kind, th, dim, X + i * dim, X + j * dim, i == j, 0);
    return 0;
}

/* Cross-covariance between data points and new points, no nugget. n x m. */
int orc_cross_cov(int kind, const double th[4], i64 n, i64 m, int dim, const double *X,
                  const double *Xs, double *Cs, i64 ld)
{
    if (n < 0 || m < 0 || ld < (n > 0 ? n : 1)) return -1;
#pragma omp parallel for schedule(static)
    for (i64 j = 0; j < m; ++j)
        for (i64 i = 0; i < n; ++i)
            Cs[i + j * ld] = cov_entry(kind, th, dim, X + i * dim, Xs + j * dim, 0, 1);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Cholesky L L^T = A (Section 1; no pivoting, so a matrix that is not  */
/* numerically positive definite fails, as the Discussion notes).       */
/* Unblocked Cholesky-Crout, column by column:                          */
/*   s = A_jj - sum_{k<j} L_jk^2 ;  fail (return j+1) unless s > 0      */
/*   L_jj = sqrt(s);  L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj        */
/* The factor is held row-major internally so that each sum reads two   */
/* contiguous rows; sums run over ascending k.                          */
/* Returns 0, or the 1-based index of the first failing column (the     */
/* LAPACK convention).  Only the lower triangle of A is read/written.   */
/* ------------------------------------------------------------------ */
i64 orc_potrf(i64 n, double *A, i64 lda)
{
    if (n <= 0) return 0;
    double *R = (double *)malloc((size_t)n * (size_t)n * sizeof(double)); /* R[i*n+k] = L_ik */
    if (!R) return -1;
    for (i64 i = 0; i < n; ++i)
        for (i64 k = 0; k <= i; ++k) R[i * n + k] = A[i + k * lda];
    i64 info = 0;
    for (i64 j = 0; j < n; ++j) {
        const double *rj = R + j * n;
        double s = R[j * n + j];
        for (i64 k = 0; k < j; ++k) s -= rj[k] * rj[k];
        if (!(s > 0.0)) { info = j + 1; break; }
        const double ljj = sqrt(s);
        R[j * n + j] = ljj;
#pragma omp parallel for schedule(static)
        for (i64 i = j + 1; i < n; ++i) {
            const double *ri = R + i * n;
            double t = ri[j];
            for (i64 k = 0; k < j; ++k) t -= ri[k] * rj[k];
            R[i * n + j] = t / ljj;
        }
    }
    if (info == 0)
        for (i64 i = 0; i < n; ++i)
            for (i64 k = 0; k <= i; ++k) A[i + k * lda] = R[i * n + k];
    free(R);
    return info;
}

/* Triangular solves with the lower factor, in place on x.
 * trans = 0: forward substitution, x <- L^{-1} x (the "backsolve" of Section 1).
 * trans = 1: back substitution,    x <- L^{-T} x.                              */
void orc_trsv(int trans, i64 n, const double *L, i64 ldl, double *x)
{
    if (!trans) {
        for (i64 i = 0; i < n; ++i) {
            double t = x[i];
            for (i64 k = 0; k < i; ++k) t -= L[i + k * ldl] * x[k];
            x[i] = t / L[i + i * ldl];
        }
    } else {
        for (i64 i = n - 1; i >= 0; --i) {
            double t = x[i];
            for (i64 k = i + 1; k < n; ++k) t -= L[k + i * ldl] * x[k];
            x[i] = t / L[i + i * ldl];
        }
    }
}

/* log|C| = 2 sum log L_ii and q = z^T z, both compensated.  out = {logdet, q}. */
void orc_logdet_q(i64 n, const double *L, i64 ldl, const double *z, double out[2])
{
    csum ld = {0, 0}, q = {0, 0};
    for (i64 i = 0; i < n; ++i) {
        cs_add(&ld, log(L[i + i * ldl]));
        cs_add(&q, z[i] * z[i]);
    }
    out[0] = 2.0 * cs_val(&ld);
    out[1] = cs_val(&q);
}

/* Marginal log-likelihood of Section 1 with its constant:
 *   l = -1/2 (n log(2 pi) + log|C| + (y-mu)^T C^{-1} (y-mu)).
 * out = {l, logdet, q}.  L (n x n, ld n) receives the factor, alpha (nullable)
 * receives C^{-1}(y - mu).  mu may be NULL (zero mean).  Returns info.        */
i64 orc_loglik(int kind, const double th[4], i64 n, int dim, const double *X, const double *y,
               const double *mu, double *L, double out[3], double *alpha)
{
    orc_cov(kind, th, n, dim, X, L, n);
    i64 info = orc_potrf(n, L, n);
    if (info) { out[0] = out[1] = out[2] = NAN; return info; }
    double *z = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (i64 i = 0; i < n; ++i) z[i] = y[i] - (mu ? mu[i] : 0.0);
    orc_trsv(0, n, L, n, z);
    double lq[2];
    orc_logdet_q(n, L, n, z, lq);
    out[1] = lq[0];
    out[2] = lq[1];
    out[0] = -0.5 * ((double)n * log(2.0 * M_PI) + lq[0] + lq[1]);
    if (alpha) {
        memcpy(alpha, z, (size_t)n * sizeof(double));
        orc_trsv(1, n, L, n, alpha);
    }
    free(z);
    return 0;
}

/* W = L^{-1} by forward substitution on the unit vectors (lower result). */
void orc_inv_lower(i64 n, const double *L, i64 ldl, double *W, i64 ldw)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (i64 j = 0; j < n; ++j) {
        for (i64 i = 0; i < j; ++i) W[i + j * ldw] = 0.0;
        for (i64 i = j; i < n; ++i) {
            double t = (i == j) ? 1.0 : 0.0;
            for (i64 k = j; k < i; ++k) t -= L[i + k * ldl] * W[k + j * ldw];
            W[i + j * ldw] = t / L[i + i * ldl];
        }
    }
}

/* Gradient of l with respect to theta = (log sigma^2, log rho, log tau^2):
 *   dl/dtheta_k = 1/2 sum_ij (alpha_i alpha_j - (C^{-1})_ij) dC_ij/dtheta_k,
 * alpha = C^{-1}(y - mu), C^{-1} = L^{-T} L^{-1} (Rasmussen & Williams 2006,
 * eq. 5.9, the reference the paper gives for GP regression), with
 *   dC/dlog sigma^2 = sigma^2 k(r),  dC/dlog rho = sigma^2 g(r),
 *   dC/dlog tau^2   = tau^2 [i == j].
 * out = {l, logdet, q}; grad = 3 values.  Returns info.                       */
i64 orc_loglik_grad(int kind, const double th[4], i64 n, int dim, const double *X,
                    const double *y, const double *mu, double out[3], double grad[4])
{
    size_t nn = (size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1);
    double *L = (double *)malloc(nn * sizeof(double));
    double *alpha = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    i64 info = orc_loglik(kind, th, n, dim, X, y, mu, L, out, alpha);
    if (info) { grad[0] = grad[1] = grad[2] = grad[3] = NAN; free(L); free(alpha); return info; }
    double *W = (double *)malloc(nn * sizeof(double));
    orc_inv_lower(n, L, n, W, n);
    const double s2 = exp(th[0]), rho = exp(th[1]), t2 = exp(th[2]);
    /* Per-column compensated partial sums (rows i >= j of column j; the
     * symmetric pair (i, j), (j, i) is counted once with weight 1, the
     * diagonal with weight 1/2), then the columns are added in order j = 0..n-1,
     * so the result does not depend on the thread count. */
    double *part = (double *)malloc((size_t)(n > 0 ? n : 1) * 4 * sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
    for (i64 j = 0; j < n; ++j) {
        csum p0 = {0, 0}, p1 = {0, 0}, p2 = {0, 0}, p3 = {0, 0};
        for (i64 i = j; i < n; ++i) {
            double cinv = 0.0; /* (C^{-1})_ij = sum_{k >= i} W_ki W_kj */
            for (i64 k = i; k < n; ++k) cinv += W[k + i * n] * W[k + j * n];
            double a = alpha[i] * alpha[j] - cinv;
            double w = (i == j) ? 0.5 : 1.0;
            if (kind == 3) {
                /* dC/dlog sigma^2 = sigma^2 M_t M_w, dC/dlog rho_t = sigma^2 g_t M_w,
                 * dC/dlog tau^2 = tau^2 [t_i == t_j], dC/dlog rho_w = sigma^2 M_t g_w */
                const double *xi = X + i * dim, *xj = X + j * dim;
                double rt = fabs(xi[0] - xj[0]) / rho, rw = fabs(xi[1] - xj[1]) / exp(th[3]);
                double mt = sep_m(rt), mw = sep_m(rw);
                cs_add(&p0, w * a * s2 * mt * mw);
                cs_add(&p1, w * a * s2 * sep_g(rt) * mw);
                if (xi[0] == xj[0]) cs_add(&p2, w * a * t2);
                cs_add(&p3, w * a * s2 * mt * sep_g(rw));
            } else {
                double r = dist(dim, X + i * dim, X + j * dim) / rho;
                cs_add(&p0, w * a * s2 * corr_k(kind, r));
                cs_add(&p1, w * a * s2 * corr_g(kind, r));
                if (i == j) cs_add(&p2, w * a * t2);
            }
        }
        part[4 * j + 0] = cs_val(&p0);
        part[4 * j + 1] = cs_val(&p1);
        part[4 * j + 2] = cs_val(&p2);
        part[4 * j + 3] = cs_val(&p3);
    }
    csum g0 = {0, 0}, g1 = {0, 0}, g2 = {0, 0}, g3 = {0, 0};
    for (i64 j = 0; j < n; ++j) {
        cs_add(&g0, part[4 * j + 0]);
        cs_add(&g1, part[4 * j + 1]);
        cs_add(&g2, part[4 * j + 2]);
        cs_add(&g3, part[4 * j + 3]);
    }
    free(part);
    grad[0] = cs_val(&g0);
    grad[1] = cs_val(&g1);
    grad[2] = cs_val(&g2);
    grad[3] = cs_val(&g3);
    free(W); free(L); free(alpha);
    return 0;
}

/* Kriging (Section 1: prediction and its uncertainty) at m new points:
 *   c_j = sigma^2 k(|x_i - s_j|/rho),  mean_j = mu + c_j^T alpha,
 *   w_j = L^{-1} c_j,  var_j = sigma^2 - w_j^T w_j (+ tau^2 if include_nugget).
 * L and alpha come from orc_loglik.  No clamping of var.                      */
void orc_krige(int kind, const double th[4], i64 n, i64 m, int dim, const double *X,
               const double *Xs, const double *L, i64 ldl, const double *alpha, double mu,
               int include_nugget, double *mean, double *var)
{
    const double s2 = exp(th[0]), t2 = exp(th[2]);
#pragma omp parallel
    {
        double *c = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
#pragma omp for schedule(dynamic, 4)
        for (i64 j = 0; j < m; ++j) {
            for (i64 i = 0; i < n; ++i)
                c[i] = cov_entry(kind, th, dim, X + i * dim, Xs + j * dim, 0, 1);
            double mj = 0.0;
            for (i64 i = 0; i < n; ++i) mj += c[i] * alpha[i];
            mean[j] = mu + mj;
            orc_trsv(0, n, L, ldl, c);
            double ww = 0.0;
            for (i64 i = 0; i < n; ++i) ww += c[i] * c[i];
            if (kind == 3) /* prior variance of the point: sigma^2 (+ tau^2 + v_j) */
                var[j] = cov_entry(kind, th, dim, Xs + j * dim, Xs + j * dim, 1, !include_nugget) - ww;
            else
                var[j] = s2 - ww + (include_nugget ? t2 : 0.0);
        }
        free(c);
    }
}

/* Full prediction covariance at m new points (Section 1: the variance of the
 * prediction; the full prediction variance matrix among the kriging methods of
 * Section 2.3.3, built from the cross-product of W = L^{-1} C* with itself,
 * Section 2.3.2):
 *   S_ij = sigma^2 k(|s_i - s_j|/rho) (+ tau^2 [i == j] if include_nugget)
 *          - sum_k W_ki W_kj,        W_:j = L^{-1} c_j (forward substitution).
 * With n = 0 (no data) S is the prior covariance of the new points.
 * Lower triangle of S (m x m, ld lds) written; L from orc_loglik.            */
void orc_krige_cov(int kind, const double th[4], i64 n, i64 m, int dim, const double *X,
                   const double *Xs, const double *L, i64 ldl, int include_nugget,
                   double *S, i64 lds)
{
    double *W = (double *)malloc((size_t)(n > 0 ? n : 1) * (size_t)(m > 0 ? m : 1) * sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
    for (i64 j = 0; j < m; ++j) {
        double *w = W + j * n;
        for (i64 i = 0; i < n; ++i)
            w[i] = cov_entry(kind, th, dim, X + i * dim, Xs + j * dim, 0, 1);
        orc_trsv(0, n, L, ldl, w);
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (i64 j = 0; j < m; ++j)
        for (i64 i = j; i < m; ++i) {
            double t = cov_entry(kind, th, dim, Xs + i * dim, Xs + j * dim, i == j, !include_nugget);
            for (i64 k = 0; k < n; ++k) t -= W[k + i * n] * W[k + j * n];
            S[i + j * lds] = t;
        }
    free(W);
}

/* Product with a lower-triangular factor, B (n x r, ld ldb) <- L B: the
 * multiplication by the Cholesky factor that turns independent standard
 * normal draws into correlated ones (Section 2.3.2).  Rows are formed from
 * the bottom up so that each still reads the original entries above it.      */
void orc_trmm(i64 n, i64 r, const double *L, i64 ldl, double *B, i64 ldb)
{
#pragma omp parallel for schedule(static)
    for (i64 c = 0; c < r; ++c) {
        double *b = B + c * ldb;
        for (i64 i = n - 1; i >= 0; --i) {
            double t = 0.0;
            for (i64 k = 0; k <= i; ++k) t += L[i + k * ldl] * b[k];
            b[i] = t;
        }
    }
}

/* Realizations of the latent process at m new points (Section 1: simulate
 * realizations; unconditional simulation and simulation conditional on the
 * data among the methods listed there):
 *   unconditional (n = 0): mean_i = mu, S = sigma^2 k(|s_i - s_j|/rho);
 *   conditional (n > 0):   mean_i = mu + c_i^T alpha, S = orc_krige_cov;
 *   (+ tau^2 on the diagonal of S if include_nugget)
 *   S = L_S L_S^T (orc_potrf: no pivoting, so a singular S fails),
 *   out_:r = mean + L_S eps_:r   for r = 0 .. nreal - 1.
 * eps (m x nreal, ld ldeps) are the standard normal draws, supplied by the
 * caller.  Returns the factorisation's info; on failure out is NaN.
 * Ls (m x m, ld m, nullable) receives L_S.                                   */
i64 orc_simulate(int kind, const double th[4], i64 n, i64 m, int dim, const double *X,
                 const double *Xs, const double *L, i64 ldl, const double *alpha, double mu,
                 int include_nugget, i64 nreal, const double *eps, i64 ldeps, double *out,
                 i64 ldo, double *Ls)
{
    double *S = (double *)calloc((size_t)(m > 0 ? m : 1) * (size_t)(m > 0 ? m : 1), sizeof(double));
    double *mean = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    orc_krige_cov(kind, th, n, m, dim, X, Xs, L, ldl, include_nugget, S, m);
    for (i64 i = 0; i < m; ++i) {
        double t = 0.0;
        for (i64 k = 0; k < n; ++k)
            t += cov_entry(kind, th, dim, X + k * dim, Xs + i * dim, 0, 1) * alpha[k];
        mean[i] = mu + t;
    }
    i64 info = orc_potrf(m, S, m);
    for (i64 r = 0; r < nreal; ++r)
        for (i64 i = 0; i < m; ++i) out[i + r * ldo] = info ? NAN : eps[i + r * ldeps];
    if (!info) {
        for (i64 j = 0; j < m; ++j)
            for (i64 i = 0; i < j; ++i) S[i + j * m] = 0.0;
        orc_trmm(m, nreal, S, m, out, ldo);
        for (i64 r = 0; r < nreal; ++r)
            for (i64 i = 0; i < m; ++i) out[i + r * ldo] += mean[i];
        if (Ls) memcpy(Ls, S, (size_t)m * (size_t)m * sizeof(double));
    }
    free(S);
    free(mean);
    return info;
}
