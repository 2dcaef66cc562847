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

// Matrix-free residual, pass 1 (C regenerated from X in FP64, each entry of
// the lower triangle once, used for its row and its column).  Workgroup-tile
// (I, J), I >= J, of 64 x 64: thread (tr, tc) = (tid % 16, tid / 16) takes
// rows 4 tr .. 4 tr + 3 and columns 4 tc .. 4 tc + 3.  The row sums
// sum_c C_rc x_c go to partial slot J of rows in block I, the column sums
// sum_r C_rc x_r to slot I of rows in block J; a diagonal tile puts both
// (entries strictly below its diagonal counted in each, the diagonal once)
// into slot I.  Every (row block, slot) pair is written by exactly one tile,
// and pass 2 adds the slots in a fixed order.  D > 0: the point dimension
// fixed at compile time; D = 0: any up to MAXDIM.  K: the covariance family.
constexpr int RT = 64;
template <int D, int K>
__global__ __launch_bounds__(256) void k_resid_sym(CovParams p, int64_t n, const double *__restrict__ X,
                                                   const double *__restrict__ x, double *__restrict__ partials,
                                                   const int32_t *skip) {
    if (skip && *skip) return;
    constexpr int ND = D > 0 ? D : MAXDIM;
    __shared__ double sr[RT * ND], sc[RT * ND], xr[RT], xc[RT];
    __shared__ double red_r[16][RT + 1], red_c[16][RT + 1];
    const int dim = D > 0 ? D : p.dim;
    const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
    const int64_t nb = (n + RT - 1) / RT, ntiles = nb * (nb + 1) / 2;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int64_t bi, bj;
        tri_decode(t, bi, bj);
        const int64_t i0 = bi * RT, j0 = bj * RT;
        const bool dg = bi == bj;
        __syncthreads();  // the previous tile's LDS reads are done
        for (int e = tid; e < RT * dim; e += 256) {
            sr[e] = i0 + e / dim < n ? X[i0 * dim + e] : 0.0;
            sc[e] = j0 + e / dim < n ? X[j0 * dim + e] : 0.0;
        }
        if (tid < RT) {
            xr[tid] = i0 + tid < n ? x[i0 + tid] : 0.0;
            xc[tid] = j0 + tid < n ? x[j0 + tid] : 0.0;
        }
        __syncthreads();
        double rs[4] = {0.0, 0.0, 0.0, 0.0}, cs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int r = 4 * tr + a;
            const int64_t gi = i0 + r;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = 4 * tc + b;
                const int64_t gj = j0 + c;
                if (gi >= n || gj >= n || (dg && c > r)) continue;
                double v = p.s2 * cov_corr(K, pdist<D>(sr + r * dim, sc + c * dim, dim) * p.inv_rho);
                if (gi == gj) {
                    v += p.t2;
                    rs[a] = fma(v, xc[c], rs[a]);  // the diagonal entry: its row only
                } else {
                    rs[a] = fma(v, xc[c], rs[a]);
                    cs[b] = fma(v, xr[r], cs[b]);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) red_r[tc][4 * tr + a] = rs[a];
#pragma unroll
        for (int b = 0; b < 4; ++b) red_c[tr][4 * tc + b] = cs[b];
        __syncthreads();
        if (tid < RT) {  // row sums of block I
            double s = 0.0;
            for (int q = 0; q < 16; ++q) s += red_r[q][tid];
            if (dg)
                for (int q = 0; q < 16; ++q) s += red_c[q][tid];
            if (i0 + tid < n) partials[bj * n + i0 + tid] = s;
        } else if (tid < 2 * RT && !dg) {  // column sums: rows of block J, slot I
            const int c = tid - RT;
            double s = 0.0;
            for (int q = 0; q < 16; ++q) s += red_c[q][c];
            if (j0 + c < n) partials[bi * n + j0 + c] = s;
        }
    }
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

int resid_chunks(int64_t n) { return (int)((n + RT - 1) / RT); }  // partial slots: one per 64-row block

hipError_t launch_resid_matfree(hipStream_t s, CovParams p, int64_t n, const double *X,
                                const double *r0, const double *x, double *res, double *partials,
                                const int32_t *skip) {
    if (n <= 0) return hipSuccess;
    const int nch = resid_chunks(n);
    const int64_t ntiles = (int64_t)nch * (nch + 1) / 2;
    const unsigned grid = (unsigned)(ntiles < 8192 ? ntiles : 8192);
    by_dim_kind(p, [&](auto d, auto k) {
        hipLaunchKernelGGL((k_resid_sym<decltype(d)::value, decltype(k)::value>), dim3(grid), dim3(256), 0, s, p, n,
                           X, x, partials, skip);
    });
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
