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

// ---- the spectral example's family (Section 4.2) ------------------------------
// Matern correlation of smoothness 2 with range scaling r = d / rho:
//   M(r) = r^2 K_2(r) / 2,   g(r) = -r M'(r) = r^3 K_1(r) / 2
// (d/dr [r^2 K_2(r)] = -r^2 K_1(r)).  Three regimes, each accurate to a few
// units in the last place:
//   r <= 2:      the power series of K_1, K_2 about 0 (Abramowitz & Stegun
//                9.6.11) in u = r^2 / 4, 14 terms;
//   2 < r < 20:  the integral exp(r) K_nu(r) = int_0^inf exp(-r (cosh t - 1))
//                cosh(nu t) dt (A&S 9.6.24) by the trapezoidal rule with
//                step 1/8 over the tabulated nodes below (error below e^-55
//                in this range: the integrand is analytic in a strip and
//                decays double-exponentially);
//   r >= 20:     the asymptotic expansion (A&S 9.7.2), summed to below
//                1e-17 of its first term (its smallest term is about e^-2r).
__constant__ double k_sep_nodes[41][3] = {  // {cosh(k/8) - 1, cosh(k/8), cosh(k/4)}
    {0.0, 1.0, 1.0},
    {0.007822677825710861, 1.0078226778257109, 1.0314130998795732},
    {0.03141309987957318, 1.0314130998795732, 1.1276259652063807},
    {0.07114034670458676, 1.0711403467045868, 1.2946832846768448},
    {0.12762596520638078, 1.1276259652063807, 1.5430806348152437},
    {0.2017536929756063, 1.2017536929756063, 1.8884238771610158},
    {0.2946832846768447, 1.2946832846768448, 2.352409615243247},
    {0.40786865682280316, 1.4078686568228032, 2.964188309728088},
    {0.5430806348152438, 1.5430806348152437, 3.7621956910836314},
    {0.7024346581381903, 1.7024346581381904, 4.796567530460195},
    {0.8884238771610156, 1.8884238771610158, 6.132289479663686},
    {1.1039581593626617, 2.1039581593626617, 7.853279872697439},
    {1.3524096152432474, 2.352409615243247, 10.067661995777765},
    {1.6376653561921377, 2.6376653561921377, 12.914557062512392},
    {1.9641883097280877, 2.964188309728088, 16.572824671057315},
    {2.337087043587521, 3.3370870435875206, 21.272299872959398},
    {2.762195691083631, 3.7621956910836314, 27.308232836016487},
    {3.2461652281969924, 4.246165228196992, 35.05983829029843},
    {3.7965675304601945, 4.796567530460195, 45.014120148530026},
    {4.422013837643509, 5.422013837643509, 57.796468111195395},
    {5.132289479663686, 6.132289479663686, 74.20994852478785},
    {5.938506971550673, 6.938506971550673, 95.28575798851459},
    {6.853279872697441, 7.853279872697439, 122.34800951782942},
    {7.8909201304827095, 8.89092013048271, 157.09692153324536},
    {9.067661995777764, 10.067661995777765, 201.7156361224559},
    {10.401916013575068, 11.401916013575068, 259.0073775612391},
    {11.914557062512394, 12.914557062512392, 332.5715682417774},
    {13.629250949773306, 14.629250949773304, 427.02996670288616},
    {15.57282467105731, 16.572824671057315, 548.317035155212},
    {17.77568612846868, 18.775686128468678, 704.0527791895422},
    {20.272299872959394, 21.272299872959398, 904.0214837702166},
    {23.101726314486257, 24.101726314486257, 1160.7864226767988},
    {26.30823283601649, 27.308232836016487, 1490.479161252178},
    {29.941986372478024, 30.941986372478024, 1913.8130413492318},
    {34.05983829029843, 35.05983829029843, 2457.384521883752},
    {38.72621384725188, 39.726213847251884, 3155.344133275175},
    {44.01412014853003, 45.014120148530026, 4051.5420254925943},
    {50.006288368867764, 51.00628836886776, 5202.282906336188},
    {56.79646811119539, 57.796468111195395, 6679.863452256852},
    {64.49089415251873, 65.49089415251873, 8577.114433792824},
    {73.20994852478785, 74.20994852478785, 11013.232920103324},
};

constexpr double EULER_GAMMA = 0.57721566490153286;

// M(r) and, if WANT_G, g(r).
template <bool WANT_G>
GP_DEV void matern2_eval(double r, double &k, double &g) {
    if (r <= 2.0) {
        if (r == 0.0) {
            k = 1.0;
            g = 0.0;
            return;
        }
        const double u = 0.25 * r * r, lg = log(0.5 * r);
        // A = sum u^j / (j! (j+2)!), B = sum (psi(j+1) + psi(j+3)) u^j / (j! (j+2)!),
        // A1, B1 the same over j! (j+1)! with psi(j+1) + psi(j+2); psi(j+1) = H_j - gamma
        double t2 = 0.5, t1 = 1.0, A = 0.0, B = 0.0, A1 = 0.0, B1 = 0.0, H = 0.0;
#pragma unroll
        for (int j = 0; j < 14; ++j) {
            const double h1 = H + 1.0 / (j + 1), h2 = h1 + 1.0 / (j + 2);  // H_{j+1}, H_{j+2}
            A += t2;
            B = fma(t2, H + h2 - 2.0 * EULER_GAMMA, B);
            if (WANT_G) {
                A1 += t1;
                B1 = fma(t1, H + h1 - 2.0 * EULER_GAMMA, B1);
                t1 *= u / ((j + 1) * (j + 2));
            }
            t2 *= u / ((j + 1) * (j + 3));
            H = h1;
        }
        const double u2 = u * u;
        k = (1.0 - u) + u2 * fma(-2.0 * lg, A, B);
        if (WANT_G) g = fma(2.0, u, u2 * fma(4.0 * lg, A1, -2.0 * B1));
        return;
    }
    const double er = exp(-r);
    if (r < 20.0) {
        double s2 = 0.5, s1 = 0.5;
        for (int j = 1; j <= 40; ++j) {
            const double x = r * k_sep_nodes[j][0];
            if (x > 50.0) break;
            const double e = exp(-x);
            s2 = fma(e, k_sep_nodes[j][2], s2);
            if (WANT_G) s1 = fma(e, k_sep_nodes[j][1], s1);
        }
        k = 0.0625 * r * r * er * s2;  // r^2 / 2 * (1/8) * s2 * e^-r
        if (WANT_G) g = 0.0625 * r * r * r * er * s1;
        return;
    }
    // sum_j a_j(nu) / r^j, a_j = a_{j-1} (4 nu^2 - (2j - 1)^2) / (8 j)
    const double pre = sqrt(1.5707963267948966 / r) * er;
    double a2 = 1.0, a1 = 1.0, S2 = 1.0, S1 = 1.0;
    const double ir = 1.0 / r;
    for (int j = 1; j < 60; ++j) {
        const double q = (double)(2 * j - 1) * (double)(2 * j - 1);
        a2 *= (16.0 - q) * ir / (8.0 * j);
        S2 += a2;
        if (WANT_G) {
            a1 *= (4.0 - q) * ir / (8.0 * j);
            S1 += a1;
        }
        if (fabs(a2) < 1e-17 && (!WANT_G || fabs(a1) < 1e-17)) break;
    }
    k = 0.5 * r * r * pre * S2;
    if (WANT_G) g = 0.5 * r * r * r * pre * S1;
}

GP_DEV double matern2(double r) {
    double k, g;
    matern2_eval<false>(r, k, g);
    return k;
}

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

// Covariance entry of family K between points xi and xj (same: i == j).
// Families 0-2: sigma^2 k(|xi - xj| / rho) + tau^2 [i == j].  Family 3, points
// (t, w, v): sigma^2 M(|t_i - t_j| / rho_t) M(|w_i - w_j| / rho_w) + tau^2
// [t_i == t_j] + v_i [i == j].  Cross-covariances (cross = true) carry only
// the first term.
template <int D, int K>
GP_DEV double cov_val(const CovParams &p, const double *xi, const double *xj, int dim, bool same, bool cross) {
    if constexpr (K == GP_SEP_MATERN2) {
        double v = p.s2 * matern2(fabs(xi[0] - xj[0]) * p.inv_rho) * matern2(fabs(xi[1] - xj[1]) * p.inv_rho2);
        if (!cross) {
            if (xi[0] == xj[0]) v += p.t2;
            if (same) v += xi[2];
        }
        return v;
    } else {
        const double v = p.s2 * cov_corr(K, pdist<D>(xi, xj, dim) * p.inv_rho);
        return (same && !cross) ? v + p.t2 : v;
    }
}

// Calls f(std::integral_constant<int, D>, std::integral_constant<int, K>) for
// the point dimension (1, 2, 3, else 0 = any) and covariance family of p.
template <typename F>
void by_dim_kind(const CovParams &p, F f) {
    if (p.kind == GP_SEP_MATERN2) {  // points (t, w, v): dimension 3 (checked at the entry points)
        f(std::integral_constant<int, 3>{}, std::integral_constant<int, GP_SEP_MATERN2>{});
        return;
    }
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
        C[i + j * ldc] = cov_val<D, K>(p, xi, sc + c * dim, dim, i == j, false);
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
        Cs[i + j * ld] = cov_val<D, K>(p, sr + r * dim, sc + c * dim, dim, false, true);
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
                const double v = cov_val<D, K>(p, sr + r * dim, sc + c * dim, dim, gi == gj, false);
                if (gi == gj) {
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
// 64 x 64 tiles; each workgroup leaves GRAD_NQ compensated partial sums
// (s, c): d/dlog sigma^2, d/dlog rho, d/dlog tau^2 and, for the separable
// family only (else 0), d/dlog rho_w.
__global__ __launch_bounds__(256) void k_grad_contract(CovParams p, int64_t n,
                                                       const double *__restrict__ X,
                                                       const double *__restrict__ Cinv, int64_t ldc,
                                                       const double *__restrict__ alpha,
                                                       double *__restrict__ partials,
                                                       const int32_t *info) {
    __shared__ double sr[CT * MAXDIM];
    __shared__ double sc[CT * MAXDIM];
    __shared__ double sar[CT], sac[CT];
    __shared__ double red[256 * 2 * GRAD_NQ];
    CSum acc0, acc1, acc2, acc3;
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
                double a = sar[r] * sac[c] - Cinv[i + j * ldc];
                double w = (i == j) ? 0.5 : 1.0;
                if (p.kind == GP_SEP_MATERN2) {
                    // dC/dlog sigma^2 = sigma^2 M_t M_w, dC/dlog rho_t = sigma^2 g_t M_w,
                    // dC/dlog tau^2 = tau^2 [t_i == t_j], dC/dlog rho_w = sigma^2 M_t g_w
                    const double *xi = sr + r * dim, *xj = sc + c * dim;
                    double kt, gt, kw, gw;
                    matern2_eval<true>(fabs(xi[0] - xj[0]) * p.inv_rho, kt, gt);
                    matern2_eval<true>(fabs(xi[1] - xj[1]) * p.inv_rho2, kw, gw);
                    acc0.add(w * a * p.s2 * kt * kw);
                    acc1.add(w * a * p.s2 * gt * kw);
                    if (xi[0] == xj[0]) acc2.add(w * a * p.t2);
                    acc3.add(w * a * p.s2 * kt * gw);
                } else {
                    double d = point_dist(sr + r * dim, sc + c * dim, dim);
                    double k, g;
                    cov_corr_g(p.kind, d * p.inv_rho, k, g);
                    acc0.add(w * a * p.s2 * k);
                    acc1.add(w * a * p.s2 * g);
                    if (i == j) acc2.add(w * a * p.t2);
                }
            }
        }
    }
    // workgroup tree reduction of the (s, c) pairs
    constexpr int W = 2 * GRAD_NQ;
    red[threadIdx.x * W + 0] = acc0.s; red[threadIdx.x * W + 1] = acc0.c;
    red[threadIdx.x * W + 2] = acc1.s; red[threadIdx.x * W + 3] = acc1.c;
    red[threadIdx.x * W + 4] = acc2.s; red[threadIdx.x * W + 5] = acc2.c;
    red[threadIdx.x * W + 6] = acc3.s; red[threadIdx.x * W + 7] = acc3.c;
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if (threadIdx.x < stride) {
            for (int q = 0; q < GRAD_NQ; ++q) {
                CSum a, b;
                a.s = red[threadIdx.x * W + 2 * q]; a.c = red[threadIdx.x * W + 2 * q + 1];
                b.s = red[(threadIdx.x + stride) * W + 2 * q]; b.c = red[(threadIdx.x + stride) * W + 2 * q + 1];
                a.merge(b);
                red[threadIdx.x * W + 2 * q] = a.s; red[threadIdx.x * W + 2 * q + 1] = a.c;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < W) partials[(int64_t)blockIdx.x * W + threadIdx.x] = red[threadIdx.x];
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
