// k_chol.hip -- latency-critical pieces of the blocked Cholesky and the solves.
//
//  * k_diag_potrf: factors one 64 x 64 diagonal block in LDS (right-looking,
//    column by column: pivot, scale, rank-1 update) and forms its inverse,
//    which the panel solve then applies on the matrix cores.  This is the
//    "Cholesky decomposition of the diagonal block" step on the critical path
//    of Section 2.1 / Fig. 1; a non-positive pivot stops the factorisation
//    and records the 1-based column (no pivoting -- Section 5).
//  * k_diag_inv: the same inverse for every diagonal block of a given L.
//  * k_trsv_fwd / k_trsv_trans: single-kernel blocked triangular solves
//    (forward L^{-1} b and backward L^{-T} b -- Section 1's backsolve and the
//    remoteForwardsolve / remoteBacksolve of Section 2.3.2).  Each workgroup
//    owns one 64-row block; it takes a ticket from an atomic counter (so the
//    blocks it depends on belong to workgroups already running), accumulates
//    the off-diagonal products as soon as each dependency's flag is released,
//    applies the block's inverse and releases its own flag.  L is read once,
//    64 contiguous doubles per load.
//  * k_loglik_reduce: compensated log|C| = 2 sum log L_ii, q = z^T z and the
//    log-likelihood (Section 1; only these scalars leave the device, as in
//    Section 2.2.2).
#include "internal.h"

namespace {

// Factor + invert one diagonal block (jb <= 64 valid rows, identity padding).
// One wave per block: rows in registers, 16-column panels with MFMA updates
// (wave_chol64), then the inverse on the matrix cores (wave_inv64_blocked).
// Winv is column-major 64 x 64.
__global__ __launch_bounds__(64) void k_diag_potrf(double *A, int64_t lda, int jb, double *Winv,
                                                   int32_t *info, int64_t col0) {
    __shared__ double Ls[DB][DB + 1];  // update buffer of the factorisation, then L
    __shared__ double Wl[DB][DB + 1];  // L^{-1}
    __shared__ union {
        double pn[DB][17];
        double t32[32][33];
    } U;
    __shared__ double rd[DB];
    if (*info) return;
    const int lane = threadIdx.x;
    double a[DB];
#pragma unroll
    for (int c = 0; c < DB; ++c) {
        double v;
        if (lane < jb && c < jb) v = (c <= lane) ? A[lane + (int64_t)c * lda] : 0.0;
        else v = (lane == c) ? 1.0 : 0.0;  // identity padding decouples unused rows
        a[c] = v;
    }
    const int fail = wave_chol64(a, lane, Ls, U.pn);
    if (fail) {
        if (lane == 0) *info = (int32_t)(col0 + fail);
        return;
    }
#pragma unroll
    for (int c = 0; c < DB; ++c) Ls[lane][c] = a[c];
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < DB; ++c)
        if (lane < jb && c < jb && c <= lane) A[lane + (int64_t)c * lda] = a[c];
    wave_inv64_blocked(Ls, Wl, U.t32, rd, lane);
#pragma unroll 4
    for (int c = 0; c < DB; ++c) Winv[lane + c * DB] = Wl[lane][c];
}

__global__ __launch_bounds__(64) void k_diag_inv(const double *L, int64_t ldl, int64_t n, double *dinv) {
    __shared__ double Ls[DB][DB + 1];
    __shared__ double Wl[DB][DB + 1];
    __shared__ double T32[32][33];
    __shared__ double rd[DB];
    const int64_t b0 = (int64_t)blockIdx.x * DB;
    const int jb = (int)((n - b0) < DB ? (n - b0) : DB);
    const int lane = threadIdx.x;
#pragma unroll 4
    for (int c = 0; c < DB; ++c) {
        double v;
        if (lane < jb && c < jb) v = (c <= lane) ? L[(b0 + lane) + (b0 + c) * ldl] : 0.0;
        else v = (lane == c) ? 1.0 : 0.0;
        Ls[lane][c] = v;
    }
    wave_lds_sync();
    wave_inv64_blocked(Ls, Wl, T32, rd, lane);
    double *W = dinv + (int64_t)blockIdx.x * DB * DB;
#pragma unroll 4
    for (int c = 0; c < DB; ++c) W[lane + c * DB] = Wl[lane][c];
}

// Cross-lane reduction of H register values: lanes l and l ^ H exchange the
// halves they do not keep, so after the steps H = 32, 16, ..., 1 lane l holds
// the sum over all lanes of the original p[l] (or p[l & 15] for 16 values).
template <int H>
GP_DEV void xr_step(double *p, int lane) {
    const bool hi = (lane & H) != 0;
#pragma unroll
    for (int c = 0; c < H; ++c) {
        const double keep = hi ? p[c + H] : p[c];
        const double send = hi ? p[c] : p[c + H];
        p[c] = keep + __shfl_xor(send, H, 64);
    }
}
GP_DEV double xr_reduce64(double *p, int lane) {
    xr_step<32>(p, lane);
    xr_step<16>(p, lane);
    xr_step<8>(p, lane);
    xr_step<4>(p, lane);
    xr_step<2>(p, lane);
    xr_step<1>(p, lane);
    return p[0];
}
GP_DEV double xr_reduce16(double *p, int lane) {
    xr_step<8>(p, lane);
    xr_step<4>(p, lane);
    xr_step<2>(p, lane);
    xr_step<1>(p, lane);
    double v = p[0];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// sync layout (ints): [0] ticket, [1] abort, [2 + b] flag of block b.
//
// Forward solve, block blk (rows i0 .. i0 + 63):
//   x_blk = Winv_blk (b_blk - sum_{j < blk} L[blk, j] x_j).
// Far blocks j < blk - 1 are split over the 4 waves (lane = row, 512-byte
// column loads).  The nearest block j = blk - 1, which decides the critical
// path, is prefetched into registers (16 columns per wave) together with the
// wave's 16 columns of Winv before any waiting starts.
__global__ __launch_bounds__(256) void k_trsv_fwd(const double *L, int64_t ldl, double *x, int64_t n,
                                                  const double *dinv, int *sync, const int32_t *info) {
    __shared__ int s_blk;
    __shared__ double part[4][DB];
    __shared__ double rhs[DB];
    __shared__ double sol[4][DB];
    if (info && *info) return;
    const int nblk = (int)((n + DB - 1) / DB);
    if (threadIdx.x == 0) s_blk = atomicAdd(&sync[0], 1);
    __syncthreads();
    const int blk = s_blk;
    if (blk >= nblk) return;
    int *abortf = &sync[1];
    int *flags = &sync[2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i0 = (int64_t)blk * DB;
    const int64_t i = i0 + lane;
    const bool rv = i < n;
    const double *W = dinv + (int64_t)blk * DB * DB;
    double wreg[16], lnear[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) wreg[q] = W[lane + (16 * w + q) * DB];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        lnear[q] = (rv && blk >= 1) ? L[i + ((int64_t)(blk - 1) * DB + 16 * w + q) * ldl] : 0.0;
    const double b = (rv && w == 0) ? x[i] : 0.0;
    double acc = 0.0;
    for (int jb = w; jb < blk - 1; jb += 4) {
        if (lane == 0) wait_flag(&flags[jb], abortf);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const double *Lc = L + i + (int64_t)jb * DB * ldl;
        const double *xj = x + (int64_t)jb * DB;
        if (rv) {
#pragma unroll 16
            for (int c = 0; c < DB; ++c) acc = fma(Lc[(int64_t)c * ldl], xj[c], acc);
        }
    }
    if (blk >= 1) {
        if (lane == 0) wait_flag(&flags[blk - 1], abortf);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const double *xj = x + (int64_t)(blk - 1) * DB + 16 * w;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc = fma(lnear[q], xj[q], acc);
    }
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0) rhs[lane] = rv ? b - (((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]) : 0.0;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) s = fma(wreg[q], rhs[16 * w + q], s);
    sol[w][lane] = s;
    __syncthreads();
    if (w == 0 && rv) x[i] = ((sol[0][lane] + sol[1][lane]) + sol[2][lane]) + sol[3][lane];
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) st_release_agent(&flags[blk], 1);
}

// Backward solve x <- L^{-T} x, block blk (columns c0 .. c0 + 63 of L):
//   x_blk = Winv_blk^T (b_blk - sum_{j > blk} L[j, blk]^T x_j).
// Lane = row of a row block j; each lane keeps 64 column partial sums, so
// every load is 64 contiguous rows of one column; a cross-lane exchange
// reduces them once per wave.  The nearest block j = blk + 1 is prefetched.
__global__ __launch_bounds__(256) void k_trsv_trans(const double *L, int64_t ldl, double *x, int64_t n,
                                                    const double *dinv, int *sync, const int32_t *info) {
    __shared__ int s_t;
    __shared__ double part[4][DB];
    __shared__ double nearp[DB];
    __shared__ double rhs[DB];
    __shared__ double sol[4][DB];
    if (info && *info) return;
    const int nblk = (int)((n + DB - 1) / DB);
    if (threadIdx.x == 0) s_t = atomicAdd(&sync[0], 1);
    __syncthreads();
    const int tk = s_t;
    if (tk >= nblk) return;
    const int blk = nblk - 1 - tk;
    int *abortf = &sync[1];
    int *flags = &sync[2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t c0 = (int64_t)blk * DB;
    const int64_t col = c0 + lane;
    const bool cv = col < n;
    const double *W = dinv + (int64_t)blk * DB * DB;
    double wreg[16], lnear[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) wreg[q] = W[(16 * w + q) + lane * DB];
    const bool has_near = blk + 1 < nblk;
    const int64_t rn = (int64_t)(blk + 1) * DB + lane;  // row of the nearest block held by this lane
    const bool rnv = has_near && rn < n;
#pragma unroll
    for (int q = 0; q < 16; ++q) lnear[q] = rnv ? L[rn + (c0 + 16 * w + q) * ldl] : 0.0;
    const double b = (cv && w == 0) ? x[col] : 0.0;
    // far blocks: full blocks of rows strictly below blk + 1; this block's
    // columns are then all < n
    double p[DB];
#pragma unroll
    for (int c = 0; c < DB; ++c) p[c] = 0.0;
    // visit far blocks in the order they complete (last block first)
    for (int jb = nblk - 1 - w; jb >= blk + 2; jb -= 4) {
        if (lane == 0) wait_flag(&flags[jb], abortf);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int64_t row = (int64_t)jb * DB + lane;
        if (row < n) {
            const double xv = x[row];
            const double *Lr = L + row + c0 * ldl;
#pragma unroll
            for (int c = 0; c < DB; ++c) p[c] = fma(Lr[(int64_t)c * ldl], xv, p[c]);
        }
    }
    part[w][lane] = xr_reduce64(p, lane);
    if (has_near) {
        if (lane == 0) wait_flag(&flags[blk + 1], abortf);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const double xv = rnv ? x[rn] : 0.0;
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = lnear[q] * xv;
        const double sv = xr_reduce16(v, lane);
        if (lane < 16) nearp[16 * w + lane] = sv;
    } else if (lane < 16) {
        nearp[16 * w + lane] = 0.0;
    }
    __syncthreads();
    if (w == 0)
        rhs[lane] = cv ? b - ((((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]) + nearp[lane]) : 0.0;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) s = fma(wreg[q], rhs[16 * w + q], s);
    sol[w][lane] = s;
    __syncthreads();
    if (w == 0 && cv) x[col] = ((sol[0][lane] + sol[1][lane]) + sol[2][lane]) + sol[3][lane];
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) st_release_agent(&flags[blk], 1);
}

__global__ void k_fill_u32(uint32_t *p, int64_t cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = 0u;
}

__global__ void k_set_info(int32_t *info) { *info = 0; }

__global__ void k_sub_mu(int64_t n, const double *y, const double *mu, double *z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = y[i] - (mu ? mu[i] : 0.0);
}

__global__ void k_copy_vec(int64_t n, const double *a, double *b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_loglik_reduce(int64_t n, const double *L, int64_t ldl,
                                                       const double *z, double *out3,
                                                       const int32_t *info, const int *sync) {
    __shared__ double red[256 * 4];
    CSum ld, q;
    const bool bad = (info && *info) || (sync && sync[1]);
    if (!bad) {
        for (int64_t i = threadIdx.x; i < n; i += 256) {
            ld.add(log(L[i + i * ldl]));
            q.add(z[i] * z[i]);
        }
    }
    red[threadIdx.x * 4 + 0] = ld.s; red[threadIdx.x * 4 + 1] = ld.c;
    red[threadIdx.x * 4 + 2] = q.s; red[threadIdx.x * 4 + 3] = q.c;
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if (threadIdx.x < stride) {
            for (int k = 0; k < 2; ++k) {
                CSum a, b;
                a.s = red[threadIdx.x * 4 + 2 * k]; a.c = red[threadIdx.x * 4 + 2 * k + 1];
                b.s = red[(threadIdx.x + stride) * 4 + 2 * k]; b.c = red[(threadIdx.x + stride) * 4 + 2 * k + 1];
                a.merge(b);
                red[threadIdx.x * 4 + 2 * k] = a.s; red[threadIdx.x * 4 + 2 * k + 1] = a.c;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (bad) {
            out3[0] = out3[1] = out3[2] = __builtin_nan("");
        } else {
            const double logdet = 2.0 * (red[0] + red[1]);
            const double qq = red[2] + red[3];
            out3[1] = logdet;
            out3[2] = qq;
            out3[0] = -0.5 * (((double)n * 1.8378770664093453 + logdet) + qq);
        }
    }
}

}  // namespace

hipError_t launch_diag_potrf(hipStream_t s, double *A, int64_t lda, int jb, double *Winv,
                             int32_t *info, int64_t col0) {
    hipLaunchKernelGGL(k_diag_potrf, dim3(1), dim3(64), 0, s, A, lda, jb, Winv, info, col0);
    return hipGetLastError();
}

hipError_t launch_diag_inv(hipStream_t s, const double *L, int64_t ldl, int64_t n, double *dinv) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_diag_inv, dim3((unsigned)((n + DB - 1) / DB)), dim3(64), 0, s, L, ldl, n, dinv);
    return hipGetLastError();
}

hipError_t launch_fill(hipStream_t s, void *p, size_t bytes) {
    const int64_t cnt = (int64_t)(bytes / 4);
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, (uint32_t *)p, cnt);
    return hipGetLastError();
}

hipError_t launch_trsv(hipStream_t s, int trans, const double *L, int64_t ldl, double *x, int64_t n,
                       const double *dinv, int *sync, const int32_t *info) {
    if (n <= 0) return hipSuccess;
    const int nblk = (int)((n + DB - 1) / DB);
    hipError_t e = launch_fill(s, sync, sizeof(int) * (size_t)(nblk + 2));
    if (e != hipSuccess) return e;
    if (trans)
        hipLaunchKernelGGL(k_trsv_trans, dim3((unsigned)nblk), dim3(256), 0, s, L, ldl, x, n, dinv, sync, info);
    else
        hipLaunchKernelGGL(k_trsv_fwd, dim3((unsigned)nblk), dim3(256), 0, s, L, ldl, x, n, dinv, sync, info);
    return hipGetLastError();
}

hipError_t launch_set_info(hipStream_t s, int32_t *info) {
    hipLaunchKernelGGL(k_set_info, dim3(1), dim3(1), 0, s, info);
    return hipGetLastError();
}

hipError_t launch_sub_mu(hipStream_t s, int64_t n, const double *y, const double *mu, double *z) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sub_mu, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, y, mu, z);
    return hipGetLastError();
}

hipError_t launch_copy_vec(hipStream_t s, int64_t n, const double *a, double *b) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_vec, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, b);
    return hipGetLastError();
}

hipError_t launch_loglik_reduce(hipStream_t s, int64_t n, const double *L, int64_t ldl,
                                const double *z, double *out3, const int32_t *info, const int *sync) {
    hipLaunchKernelGGL(k_loglik_reduce, dim3(1), dim3(256), 0, s, n, L, ldl, z, out3, info, sync);
    return hipGetLastError();
}
