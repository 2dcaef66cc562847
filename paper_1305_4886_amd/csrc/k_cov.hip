// k_cov.hip -- covariance-matrix kernels (Section 1: the entries of C(theta);
// the Discussion names covariance construction as the next bottleneck once the
// Cholesky is fast).  All are HBM-bound or exp-bound streaming kernels:
//   * lower-triangle build of C (writes n(n+1)/2 doubles),
//   * cross-covariance build (writes n m doubles),
//   * matrix-free FP64 residual r0 - C x for iterative refinement,
//   * gradient contraction sum_ij (a_i a_j - Cinv_ij) dC_ij/dtheta over the
//     lower triangle of C^{-1}, regenerating dC/dtheta from the points.
#include "internal.h"
#include <type_traits>

namespace {

constexpr int CT = 64;        // covariance tile edge
constexpr int MAXDIM = 16;

// Lower-triangular tile index t -> (bi, bj), bi >= bj, row-major order.
GP_DEV void tri_decode(int64_t t, int64_t &bi, int64_t &bj) {
    double f = (sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5;
    int64_t r = (int64_t)f;
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    bi = r;
    bj = t - r * (r + 1) / 2;
}

// |xi - xj| with the point dimension fixed at compile time (D > 0, the loop
// unrolled) or given at run time (D = 0); the same operations as point_dist.
template <int D>
GP_DEV double pdist(const double *xi, const double *xj, int dim) {
    if (D == 0) return point_dist(xi, xj, dim);
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double t = xi[d] - xj[d];
        s = fma(t, t, s);
    }
    return sqrt(s);
}

// Calls f(std::integral_constant<int, D>, std::integral_constant<int, K>) for
// the point dimension (1, 2, 3, else 0 = any) and covariance family of p.
template <typename F>
void by_dim_kind(const CovParams &p, F f) {
    auto k = [&](auto d) {
        if (p.kind == GP_EXP) f(d, std::integral_constant<int, GP_EXP>{});
        else if (p.kind == GP_MATERN32) f(d, std::integral_constant<int, GP_MATERN32>{});
        else f(d, std::integral_constant<int, GP_MATERN52>{});
    };
    switch (p.dim) {
    case 1: k(std::integral_constant<int, 1>{}); break;
    case 2: k(std::integral_constant<int, 2>{}); break;
    case 3: k(std::integral_constant<int, 3>{}); break;
    default: k(std::integral_constant<int, 0>{}); break;
    }
}

// One 64 x 64 tile of the lower triangle per workgroup of 256 threads.  Thread
// (row = tid % 64, cg = tid / 64) writes column entries j = cg, cg + 4, ...:
// each wave stores 64 consecutive rows of one column (512 B, coalesced).
template <int D, int K>
__global__ __launch_bounds__(256) void k_cov_lower(CovParams p, int64_t n, const double *__restrict__ X,
                                                   double *__restrict__ C, int64_t ldc) {
    __shared__ double sr[CT * MAXDIM];
    __shared__ double sc[CT * MAXDIM];
    int64_t bi, bj;
    tri_decode(blockIdx.x, bi, bj);
    const int dim = D > 0 ? D : p.dim;
    const int64_t i0 = bi * CT, j0 = bj * CT;
    for (int e = threadIdx.x; e < CT * dim; e += 256) {
        int64_t pi = i0 + e / dim, pj = j0 + e / dim;
        sr[e] = pi < n ? X[i0 * dim + e] : 0.0;
        sc[e] = pj < n ? X[j0 * dim + e] : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x & (CT - 1), cg = threadIdx.x >> 6;
    const int64_t i = i0 + r;
    if (i >= n) return;
    const double *xi = sr + r * dim;
    for (int c = cg; c < CT; c += 4) {
        const int64_t j = j0 + c;
        if (j > i) break;
        double d = pdist<D>(xi, sc + c * dim, dim);
        double v = p.s2 * cov_corr(K, d * p.inv_rho);
        if (i == j) v += p.t2;
        C[i + j * ldc] = v;
    }
}

template <int D, int K>
__global__ __launch_bounds__(256) void k_cross_cov(CovParams p, int64_t n, int64_t m,
                                                   const double *__restrict__ X,
                                                   const double *__restrict__ Xs,
                                                   double *__restrict__ Cs, int64_t ld) {
    __shared__ double sr[CT * MAXDIM];
    __shared__ double sc[CT * MAXDIM];
    const int dim = D > 0 ? D : p.dim;
    const int64_t i0 = (int64_t)blockIdx.x * CT, j0 = (int64_t)blockIdx.y * CT;
    for (int e = threadIdx.x; e < CT * dim; e += 256) {
        sr[e] = i0 + e / dim < n ? X[i0 * dim + e] : 0.0;
        sc[e] = j0 + e / dim < m ? Xs[j0 * dim + e] : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x & (CT - 1), cg = threadIdx.x >> 6;
    const int64_t i = i0 + r;
    if (i >= n) return;
    for (int c = cg; c < CT; c += 4) {
        const int64_t j = j0 + c;
        if (j >= m) break;
        double d = pdist<D>(sr + r * dim, sc + c * dim, dim);
        Cs[i + j * ld] = p.s2 * cov_corr(K, d * p.inv_rho);
    }
}

// Matrix-free residual, pass 1: partials[chunk][i] = sum_{j in chunk} C_ij x_j
// for a 256-row block and a 2048-column chunk (C regenerated from X, FP64).
// D > 0: the point dimension fixed at compile time (the distance loop fully
// unrolled); D = 0: any dimension up to MAXDIM.  K: the covariance family.
constexpr int RES_ROWS = 256, RES_COLS = 2048, RES_STAGE = 256;
template <int D, int K>
__global__ __launch_bounds__(256) void k_resid_partial(CovParams p, int64_t n,
                                                       const double *__restrict__ X,
                                                       const double *__restrict__ x,
                                                       double *__restrict__ partials,
                                                       const int32_t *skip) {
    if (skip && *skip) return;
    constexpr int ND = D > 0 ? D : MAXDIM;
    __shared__ double sp[RES_STAGE * ND];
    __shared__ double sx[RES_STAGE];
    const int dim = D > 0 ? D : p.dim;
    const int64_t i = (int64_t)blockIdx.x * RES_ROWS + threadIdx.x;
    const int64_t jc0 = (int64_t)blockIdx.y * RES_COLS;
    double xi[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) xi[d] = (d < dim && i < n) ? X[i * dim + d] : 0.0;
    double acc = 0.0;
    for (int64_t js = jc0; js < jc0 + RES_COLS && js < n; js += RES_STAGE) {
        __syncthreads();
        for (int e = threadIdx.x; e < RES_STAGE * dim; e += 256)
            sp[e] = js + e / dim < n ? X[js * dim + e] : 0.0;
        sx[threadIdx.x] = js + threadIdx.x < n ? x[js + threadIdx.x] : 0.0;
        __syncthreads();
        const int cnt = (int)((n - js) < RES_STAGE ? (n - js) : RES_STAGE);
        for (int c = 0; c < cnt; ++c) {
            double s = 0.0;
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                if (D > 0 || d < dim) {
                    double t = xi[d] - sp[c * dim + d];
                    s = fma(t, t, s);
                }
            }
            double v = p.s2 * cov_corr(K, sqrt(s) * p.inv_rho);
            if (js + c == i) v += p.t2;
            acc = fma(v, sx[c], acc);
        }
    }
    if (i < n) partials[(int64_t)blockIdx.y * n + i] = acc;
}

// Pass 2: res_i = r0_i - sum_chunks partials (fixed chunk order).
__global__ __launch_bounds__(256) void k_resid_finish(int64_t n, int nchunks,
                                                      const double *__restrict__ r0,
                                                      const double *__restrict__ partials,
                                                      double *__restrict__ res, const int32_t *skip) {
    if (skip && *skip) return;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += partials[(int64_t)c * n + i];
    res[i] = r0[i] - s;
}

// Gradient contraction over the lower triangle of Cinv, grid-stride over
// 64 x 64 tiles; each workgroup leaves 3 compensated partial sums (s, c).
__global__ __launch_bounds__(256) void k_grad_contract(CovParams p, int64_t n,
                                                       const double *__restrict__ X,
                                                       const double *__restrict__ Cinv, int64_t ldc,
                                                       const double *__restrict__ alpha,
                                                       double *__restrict__ partials,
                                                       const int32_t *info) {
    __shared__ double sr[CT * MAXDIM];
    __shared__ double sc[CT * MAXDIM];
    __shared__ double sar[CT], sac[CT];
    __shared__ double red[256 * 6];
    CSum acc0, acc1, acc2;
    const bool dead = info && *info;
    const int64_t T = (n + CT - 1) / CT;
    const int64_t ntiles = T * (T + 1) / 2;
    const int dim = p.dim;
    for (int64_t t = blockIdx.x; t < ntiles && !dead; t += gridDim.x) {
        int64_t bi, bj;
        tri_decode(t, bi, bj);
        const int64_t i0 = bi * CT, j0 = bj * CT;
        __syncthreads();
        for (int e = threadIdx.x; e < CT * dim; e += 256) {
            sr[e] = i0 + e / dim < n ? X[i0 * dim + e] : 0.0;
            sc[e] = j0 + e / dim < n ? X[j0 * dim + e] : 0.0;
        }
        if (threadIdx.x < CT) {
            sar[threadIdx.x] = i0 + threadIdx.x < n ? alpha[i0 + threadIdx.x] : 0.0;
            sac[threadIdx.x] = j0 + threadIdx.x < n ? alpha[j0 + threadIdx.x] : 0.0;
        }
        __syncthreads();
        const int r = threadIdx.x & (CT - 1), cg = threadIdx.x >> 6;
        const int64_t i = i0 + r;
        if (i < n) {
            for (int c = cg; c < CT; c += 4) {
                const int64_t j = j0 + c;
                if (j > i) break;
                double d = point_dist(sr + r * dim, sc + c * dim, dim);
                double k, g;
                cov_corr_g(p.kind, d * p.inv_rho, k, g);
                double a = sar[r] * sac[c] - Cinv[i + j * ldc];
                double w = (i == j) ? 0.5 : 1.0;
                acc0.add(w * a * p.s2 * k);
                acc1.add(w * a * p.s2 * g);
                if (i == j) acc2.add(w * a * p.t2);
            }
        }
    }
    // workgroup tree reduction of the (s, c) pairs
    red[threadIdx.x * 6 + 0] = acc0.s; red[threadIdx.x * 6 + 1] = acc0.c;
    red[threadIdx.x * 6 + 2] = acc1.s; red[threadIdx.x * 6 + 3] = acc1.c;
    red[threadIdx.x * 6 + 4] = acc2.s; red[threadIdx.x * 6 + 5] = acc2.c;
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if (threadIdx.x < stride) {
            for (int q = 0; q < 3; ++q) {
                CSum a, b;
                a.s = red[threadIdx.x * 6 + 2 * q]; a.c = red[threadIdx.x * 6 + 2 * q + 1];
                b.s = red[(threadIdx.x + stride) * 6 + 2 * q]; b.c = red[(threadIdx.x + stride) * 6 + 2 * q + 1];
                a.merge(b);
                red[threadIdx.x * 6 + 2 * q] = a.s; red[threadIdx.x * 6 + 2 * q + 1] = a.c;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partials[(int64_t)blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x];
}

}  // namespace

hipError_t launch_cov_lower(hipStream_t s, CovParams p, int64_t n, const double *X, double *C,
                            int64_t ldc, const int32_t *) {
    if (n <= 0) return hipSuccess;
    const int64_t T = (n + CT - 1) / CT;
    by_dim_kind(p, [&](auto d, auto k) {
        hipLaunchKernelGGL((k_cov_lower<decltype(d)::value, decltype(k)::value>), dim3((unsigned)(T * (T + 1) / 2)),
                           dim3(256), 0, s, p, n, X, C, ldc);
    });
    return hipGetLastError();
}

hipError_t launch_cross_cov(hipStream_t s, CovParams p, int64_t n, int64_t m, const double *X,
                            const double *Xs, double *Cs, int64_t ld) {
    if (n <= 0 || m <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + CT - 1) / CT), (unsigned)((m + CT - 1) / CT));
    by_dim_kind(p, [&](auto d, auto k) {
        hipLaunchKernelGGL((k_cross_cov<decltype(d)::value, decltype(k)::value>), grid, dim3(256), 0, s, p, n, m, X,
                           Xs, Cs, ld);
    });
    return hipGetLastError();
}

int resid_chunks(int64_t n) { return (int)((n + RES_COLS - 1) / RES_COLS); }

hipError_t launch_resid_matfree(hipStream_t s, CovParams p, int64_t n, const double *X,
                                const double *r0, const double *x, double *res, double *partials,
                                const int32_t *skip) {
    if (n <= 0) return hipSuccess;
    const int nch = resid_chunks(n);
    dim3 g1((unsigned)((n + RES_ROWS - 1) / RES_ROWS), (unsigned)nch);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, g1, dim3(256), 0, s, p, n, X, x, partials, skip); };
    auto by_kind = [&](auto d) {
        constexpr int D = decltype(d)::value;
        if (p.kind == GP_EXP) go(k_resid_partial<D, GP_EXP>);
        else if (p.kind == GP_MATERN32) go(k_resid_partial<D, GP_MATERN32>);
        else go(k_resid_partial<D, GP_MATERN52>);
    };
    switch (p.dim) {
    case 1: by_kind(std::integral_constant<int, 1>{}); break;
    case 2: by_kind(std::integral_constant<int, 2>{}); break;
    case 3: by_kind(std::integral_constant<int, 3>{}); break;
    default: by_kind(std::integral_constant<int, 0>{}); break;
    }
    hipLaunchKernelGGL(k_resid_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, nch, r0,
                       partials, res, skip);
    return hipGetLastError();
}

hipError_t launch_grad_contract(hipStream_t s, CovParams p, int64_t n, const double *X,
                                const double *Cinv, int64_t ldc, const double *alpha,
                                double *partials, int nparts, const int32_t *info) {
    hipLaunchKernelGGL(k_grad_contract, dim3((unsigned)nparts), dim3(256), 0, s, p, n, X, Cinv, ldc,
                       alpha, partials, info);
    return hipGetLastError();
}
