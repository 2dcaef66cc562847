// k_aux.hip -- small streaming kernels around the matrix-core products:
// row reductions for kriging (c_j^T alpha and |w_j|^2, Section 1's
// prediction and its variance), block copies and transposes, the placement
// of diagonal-block inverses into the blocked triangular inverse, the
// iterative-refinement bookkeeping and the Morton ordering.
#include "internal.h"

namespace {

// dst[i + j ldd] = src[i + j lds], rows x cols.
__global__ __launch_bounds__(256) void k_copy2d(int64_t rows, int64_t cols, const double *src, int64_t lds,
                                                double *dst, int64_t ldd) {
    const int64_t j = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256)
        dst[i + j * ldd] = src[i + j * lds];
}

// Diagonal 64-blocks of W from the stored block inverses (column-major, ld DB).
__global__ __launch_bounds__(256) void k_place_dinv(int64_t n, const double *dinv, double *W, int64_t ldw,
                                                    int trans) {
    const int64_t b = blockIdx.x;
    const int64_t b0 = b * DB;
    const double *src = dinv + b * DB * DB;
    for (int e = threadIdx.x; e < DB * DB; e += 256) {
        const int i = e & (DB - 1), j = e >> 6;
        if (b0 + i < n && b0 + j < n) W[(b0 + i) + (b0 + j) * ldw] = trans ? src[j + i * DB] : src[i + j * DB];
    }
}

// dst[j + i ldd] = src[i + j lds] for i < rows, j < cols (batch z: strides
// sstr, dstr), 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void k_transpose_copy(int64_t rows, int64_t cols, const double *src, int64_t lds,
                                                        int64_t sstr, double *dst, int64_t ldd, int64_t dstr) {
    __shared__ double Tt[64][65];
    const double *S = src + (int64_t)blockIdx.z * sstr;
    double *D = dst + (int64_t)blockIdx.z * dstr;
    const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int c = ty; c < 64; c += 4) {
        const int64_t i = r0 + tx, j = c0 + c;
        Tt[c][tx] = (i < rows && j < cols) ? S[i + j * lds] : 0.0;
    }
    __syncthreads();
    for (int c = ty; c < 64; c += 4) {  // D(c0 + tx, r0 + c) = S(r0 + c, c0 + tx)
        const int64_t j = c0 + tx, i = r0 + c;
        if (i < rows && j < cols) D[j + i * ldd] = Tt[tx][c];
    }
}

// Final fixed-order combination of per-workgroup (s, c) partial sums of the
// gradient contraction: grad[q] = sum over parts.
__global__ __launch_bounds__(64) void k_grad_finish(int nparts, const double *partials, double *grad, int ngrad,
                                                    const int32_t *info) {
    if (threadIdx.x != 0) return;
    if (info && *info) {
        for (int q = 0; q < ngrad; ++q) grad[q] = __builtin_nan("");
        return;
    }
    for (int q = 0; q < ngrad; ++q) {
        CSum a;
        for (int p = 0; p < nparts; ++p) {
            CSum b;
            b.s = partials[p * 2 * GRAD_NQ + 2 * q];
            b.c = partials[p * 2 * GRAD_NQ + 2 * q + 1];
            a.merge(b);
        }
        grad[q] = a.value();
    }
}


// Synthetic SPD test matrix for the autotuner: the exponential covariance of
// n equispaced points on a line, exp(-8 |i - j| / n), plus the identity
// (lower triangle only).
__global__ void k_tune_fill(double *A, int64_t lda, int64_t n) {
    const double sc = 8.0 / (double)n;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        for (int64_t i = j + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            A[i + j * lda] = exp(-sc * (double)(i - j)) + (i == j ? 1.0 : 0.0);
}



// Row reductions of an m x n column-major matrix Y (ld ldy), in two passes
// with compensated sums: chunk c of RR_COLS columns gives partials
// (s, e)[c][j] for each row j (threads run along j, so every load is a
// contiguous run of a column); the finish pass adds the chunks in order.
//   mode 0: out_j = base + sum_i Y(j, i) v_i      mode 1: out_j = base - sum_i Y(j, i)^2
constexpr int RR_COLS = 512;
__global__ __launch_bounds__(256) void k_rowreduce_partial(int mode, int64_t m, int64_t n, const double *Y, int64_t ldy,
                                                           const double *v, double *partials) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (j >= m) return;
    const int64_t i1 = (c + 1) * RR_COLS < n ? (c + 1) * RR_COLS : n;
    CSum acc;
    for (int64_t i = c * RR_COLS; i < i1; ++i) {
        const double y = Y[j + i * ldy];
        acc.add(mode == 0 ? y * v[i] : y * y);
    }
    partials[2 * (c * m + j)] = acc.s;
    partials[2 * (c * m + j) + 1] = acc.c;
}

__global__ __launch_bounds__(256) void k_rowreduce_finish(int mode, int64_t m, int64_t nchunk, const double *partials,
                                                          double base, double *out) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    CSum acc;
    for (int64_t c = 0; c < nchunk; ++c) {
        CSum b;
        b.s = partials[2 * (c * m + j)];
        b.c = partials[2 * (c * m + j) + 1];
        acc.merge(b);
    }
    const double t = acc.value();
    out[j] = mode == 0 ? base + t : base - t;
}

}  // namespace

hipError_t launch_tune_fill(hipStream_t s, double *A, int64_t lda, int64_t n) {
    if (n <= 0) return hipSuccess;
    const int64_t gx = (n + 255) / 256 < 64 ? (n + 255) / 256 : 64;
    hipLaunchKernelGGL(k_tune_fill, dim3((unsigned)gx, (unsigned)(n < 8192 ? n : 8192)), dim3(256), 0, s, A, lda, n);
    return hipGetLastError();
}

int64_t rowreduce_chunks(int64_t n) { return (n + RR_COLS - 1) / RR_COLS; }

hipError_t launch_rowreduce(hipStream_t s, int mode, int64_t m, int64_t n, const double *Y, int64_t ldy,
                            const double *v, double base, double *partials, double *out) {
    if (m <= 0) return hipSuccess;
    const int64_t nch = n > 0 ? rowreduce_chunks(n) : 0;
    if (nch > 0)
        hipLaunchKernelGGL(k_rowreduce_partial, dim3((unsigned)((m + 255) / 256), (unsigned)nch), dim3(256), 0, s, mode,
                           m, n, Y, ldy, v, partials);
    hipLaunchKernelGGL(k_rowreduce_finish, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, mode, m, nch, partials,
                       base, out);
    return hipGetLastError();
}

hipError_t launch_copy2d(hipStream_t s, int64_t rows, int64_t cols, const double *src, int64_t lds, double *dst,
                         int64_t ldd) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const int64_t gx = (rows + 255) / 256 < 64 ? (rows + 255) / 256 : 64;
    hipLaunchKernelGGL(k_copy2d, dim3((unsigned)gx, (unsigned)cols), dim3(256), 0, s, rows, cols, src, lds, dst, ldd);
    return hipGetLastError();
}

hipError_t launch_place_dinv(hipStream_t s, int64_t n, const double *dinv, double *W, int64_t ldw, int trans) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_place_dinv, dim3((unsigned)((n + DB - 1) / DB)), dim3(256), 0, s, n, dinv, W, ldw, trans);
    return hipGetLastError();
}

hipError_t launch_transpose_copy(hipStream_t s, int64_t rows, int64_t cols, const double *src, int64_t lds,
                                 int64_t sstr, double *dst, int64_t ldd, int64_t dstr, int64_t batch) {
    if (rows <= 0 || cols <= 0 || batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_transpose_copy, dim3((unsigned)((rows + 63) / 64), (unsigned)((cols + 63) / 64), (unsigned)batch),
                       dim3(256), 0, s, rows, cols, src, lds, sstr, dst, ldd, dstr);
    return hipGetLastError();
}

hipError_t launch_grad_finish(hipStream_t s, int nparts, const double *partials, double *grad, int ngrad,
                              const int32_t *info) {
    hipLaunchKernelGGL(k_grad_finish, dim3(1), dim3(64), 0, s, nparts, partials, grad, ngrad, info);
    return hipGetLastError();
}

namespace {

// ---------------------------------------------------------------------------
// Iterative refinement of x = C^{-1} b with a low-precision factor; control
// lives on the device so no host synchronisation is needed.  state (doubles):
// [0] |b|, [1] previous relative residual, [2] last relative residual,
// [3] corrections applied, [4] converged (1) / not (0).  *done != 0 makes
// every later kernel of the refinement a no-op.
// ---------------------------------------------------------------------------
GP_DEV void block_norm2(int64_t n, const double *v, double *red, CSum &out) {
    CSum s;
    for (int64_t i = threadIdx.x; i < n; i += 256) s.add(v[i] * v[i]);
    red[2 * threadIdx.x] = s.s;
    red[2 * threadIdx.x + 1] = s.c;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            CSum a, b;
            a.s = red[2 * threadIdx.x]; a.c = red[2 * threadIdx.x + 1];
            b.s = red[2 * (threadIdx.x + st)]; b.c = red[2 * (threadIdx.x + st) + 1];
            a.merge(b);
            red[2 * threadIdx.x] = a.s; red[2 * threadIdx.x + 1] = a.c;
        }
        __syncthreads();
    }
    out.s = red[0];
    out.c = red[1];
}

__global__ __launch_bounds__(256) void k_ir_init(int64_t n, const double *b, double *state, int32_t *done,
                                                 const int32_t *info) {
    __shared__ double red[512];
    CSum s;
    block_norm2(n, b, red, s);
    if (threadIdx.x == 0) {
        state[0] = sqrt(s.value());
        state[1] = __builtin_inf();
        state[2] = __builtin_nan("");
        state[3] = 0.0;
        state[4] = 0.0;
        *done = (info && *info) ? 1 : 0;
    }
}

// Stop on convergence (rel <= tol), on the sweep cap, or when a sweep fails to
// halve the residual (stagnation).
__global__ __launch_bounds__(256) void k_ir_check(int64_t n, const double *res, double *state, int32_t *done,
                                                  int last, double tol) {
    __shared__ double red[512];
    if (*done) return;
    CSum s;
    block_norm2(n, res, red, s);
    if (threadIdx.x == 0) {
        const double nb = state[0];
        const double rel = nb > 0.0 ? sqrt(s.value()) / nb : 0.0;
        state[2] = rel;
        if (rel <= tol) {
            state[4] = 1.0;
            *done = 1;
        } else if (last || !(rel <= 0.5 * state[1])) {
            *done = 1;
        } else {
            state[1] = rel;
            state[3] += 1.0;
        }
    }
}

// A sweep whose check stopped the refinement computed no new correction, so
// every correction step of that sweep is skipped.
__global__ void k_axpy_skip(int64_t n, const double *dv, double *x, const int32_t *done) {
    if (*done) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += dv[i];
}

__global__ void k_copy_skip(int64_t n, const double *a, double *b, const int32_t *done) {
    if (*done) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// q = b^T x, log-likelihood, refinement report.
__global__ __launch_bounds__(256) void k_ir_finish(int64_t n, const double *b, const double *x, const double *state,
                                                   double *out3, double *ir, const int32_t *info) {
    __shared__ double red[512];
    CSum s;
    for (int64_t i = threadIdx.x; i < n; i += 256) s.add(b[i] * x[i]);
    red[2 * threadIdx.x] = s.s;
    red[2 * threadIdx.x + 1] = s.c;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            CSum a, c;
            a.s = red[2 * threadIdx.x]; a.c = red[2 * threadIdx.x + 1];
            c.s = red[2 * (threadIdx.x + st)]; c.c = red[2 * (threadIdx.x + st) + 1];
            a.merge(c);
            red[2 * threadIdx.x] = a.s; red[2 * threadIdx.x + 1] = a.c;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (info && *info) {
            out3[0] = out3[1] = out3[2] = __builtin_nan("");
        } else {
            const double q = red[0] + red[1];
            out3[2] = q;
            out3[0] = -0.5 * (((double)n * 1.8378770664093453 + out3[1]) + q);
        }
        if (ir) {
            ir[0] = state[3];
            ir[1] = state[2];
            ir[2] = state[4];
        }
    }
}

// ---------------------------------------------------------------------------
// Morton (Z-order) permutation.  Coordinates 0 and 1 of each point are scaled
// to 21-bit integers on the bounding box and bit-interleaved; the 42-bit code
// is shifted above a 22-bit point index, so keys are unique and ties resolve
// by index.  A bitonic network over the next power of two sorts the keys.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bbox(int64_t n, int dim, const double *X, double *box) {
    __shared__ double r[4][256];
    double lo0 = __builtin_inf(), hi0 = -__builtin_inf(), lo1 = __builtin_inf(), hi1 = -__builtin_inf();
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double a = X[i * dim];
        const double b = dim > 1 ? X[i * dim + 1] : 0.0;
        lo0 = fmin(lo0, a); hi0 = fmax(hi0, a);
        lo1 = fmin(lo1, b); hi1 = fmax(hi1, b);
    }
    r[0][threadIdx.x] = lo0; r[1][threadIdx.x] = hi0; r[2][threadIdx.x] = lo1; r[3][threadIdx.x] = hi1;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            r[0][threadIdx.x] = fmin(r[0][threadIdx.x], r[0][threadIdx.x + st]);
            r[1][threadIdx.x] = fmax(r[1][threadIdx.x], r[1][threadIdx.x + st]);
            r[2][threadIdx.x] = fmin(r[2][threadIdx.x], r[2][threadIdx.x + st]);
            r[3][threadIdx.x] = fmax(r[3][threadIdx.x], r[3][threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) box[threadIdx.x] = r[threadIdx.x][0];
}

GP_DEV uint64_t spread2_21(uint64_t v) {  // 21 bits -> even positions of 42 bits
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (2 * b);
    return r;
}

__global__ void k_morton_keys(int64_t n, int64_t npow, int dim, const double *X, const double *box,
                              uint64_t *keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npow) return;
    if (i >= n) {
        keys[i] = ~0ull;
        return;
    }
    const double q = 2097151.0;  // 2^21 - 1
    const double w0 = box[1] - box[0], w1 = box[3] - box[2];
    const double a = X[i * dim], b = dim > 1 ? X[i * dim + 1] : 0.0;
    const uint64_t qa = (uint64_t)(w0 > 0.0 ? fmin(fmax((a - box[0]) / w0, 0.0), 1.0) * q : 0.0);
    const uint64_t qb = (uint64_t)(w1 > 0.0 ? fmin(fmax((b - box[2]) / w1, 0.0), 1.0) * q : 0.0);
    const uint64_t code = spread2_21(qa) | (spread2_21(qb) << 1);
    keys[i] = (code << 22) | (uint64_t)i;
}

__global__ void k_bitonic_step(uint64_t *keys, int64_t npow, int64_t j, int64_t k) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npow) return;
    const int64_t l = i ^ j;
    if (l <= i) return;
    const uint64_t a = keys[i], b = keys[l];
    const bool up = (i & k) == 0;
    if ((a > b) == up) {
        keys[i] = b;
        keys[l] = a;
    }
}

__global__ void k_keys_to_perm(int64_t n, const uint64_t *keys, int64_t *perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) perm[i] = (int64_t)(keys[i] & ((1ull << 22) - 1));
}

// Xp[i] = X[perm[i]] (dim columns), yp, mup.
__global__ void k_gather_points(int64_t n, int dim, const int64_t *perm, const double *X, const double *y,
                                 const double *mu, double *Xp, double *yp, double *mup) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t p = perm[i];
    for (int d = 0; d < dim; ++d) Xp[i * dim + d] = X[p * dim + d];
    yp[i] = y[p];
    if (mu) mup[i] = mu[p];
}

__global__ void k_scatter_vec(int64_t n, const int64_t *perm, const double *src, double *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[perm[i]] = src[i];
}

}  // namespace

static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_ir_init(hipStream_t s, int64_t n, const double *b, double *state, int32_t *done,
                          const int32_t *info) {
    hipLaunchKernelGGL(k_ir_init, dim3(1), dim3(256), 0, s, n, b, state, done, info);
    return hipGetLastError();
}
hipError_t launch_ir_check(hipStream_t s, int64_t n, const double *res, double *state, int32_t *done, int last,
                           double tol) {
    hipLaunchKernelGGL(k_ir_check, dim3(1), dim3(256), 0, s, n, res, state, done, last, tol);
    return hipGetLastError();
}
hipError_t launch_copy_skip(hipStream_t s, int64_t n, const double *a, double *b, const int32_t *done) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_skip, dim3(nb256(n)), dim3(256), 0, s, n, a, b, done);
    return hipGetLastError();
}
hipError_t launch_axpy_skip(hipStream_t s, int64_t n, const double *dv, double *x, const int32_t *done) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpy_skip, dim3(nb256(n)), dim3(256), 0, s, n, dv, x, done);
    return hipGetLastError();
}
hipError_t launch_ir_finish(hipStream_t s, int64_t n, const double *b, const double *x, const double *state,
                            double *out3, double *ir, const int32_t *info) {
    hipLaunchKernelGGL(k_ir_finish, dim3(1), dim3(256), 0, s, n, b, x, state, out3, ir, info);
    return hipGetLastError();
}
hipError_t launch_morton(hipStream_t s, int64_t n, int dim, const double *X, int64_t *perm, uint64_t *keys,
                         double *box) {
    if (n <= 0) return hipSuccess;
    int64_t npow = 1;
    while (npow < n) npow <<= 1;
    hipLaunchKernelGGL(k_bbox, dim3(1), dim3(256), 0, s, n, dim, X, box);
    hipLaunchKernelGGL(k_morton_keys, dim3(nb256(npow)), dim3(256), 0, s, n, npow, dim, X, box, keys);
    for (int64_t k = 2; k <= npow; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_step, dim3(nb256(npow)), dim3(256), 0, s, keys, npow, j, k);
    hipLaunchKernelGGL(k_keys_to_perm, dim3(nb256(n)), dim3(256), 0, s, n, keys, perm);
    return hipGetLastError();
}
hipError_t launch_gather_points(hipStream_t s, int64_t n, int dim, const int64_t *perm, const double *X,
                                const double *y, const double *mu, double *Xp, double *yp, double *mup) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_points, dim3(nb256(n)), dim3(256), 0, s, n, dim, perm, X, y, mu, Xp, yp, mup);
    return hipGetLastError();
}
hipError_t launch_scatter_vec(hipStream_t s, int64_t n, const int64_t *perm, const double *src, double *dst) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_vec, dim3(nb256(n)), dim3(256), 0, s, n, perm, src, dst);
    return hipGetLastError();
}

// ---- product with the lower factor (simulation of realizations) -------------
namespace {

constexpr int TRMM_NC = 32;  // columns of E per workgroup

// Workgroup (block b, column chunk): the 128 x 32 slab of E staged in LDS;
// thread t owns row a = t % 128 and 16 of the 32 columns.  L is read down the
// block's columns (consecutive rows across threads), entries above the
// diagonal are never loaded.
__global__ __launch_bounds__(256) void k_trmm_diag(int64_t m, int64_t r, const double *L, int64_t ldl,
                                                   const double *E, int64_t lde, double *out, int64_t ldo,
                                                   const int32_t *info) {
    __shared__ double Es[TRMM_DB][TRMM_NC + 1];
    if (info && *info) return;
    const int64_t i0 = (int64_t)blockIdx.x * TRMM_DB, c0 = (int64_t)blockIdx.y * TRMM_NC;
    const int tid = threadIdx.x;
    for (int e = tid; e < TRMM_DB * TRMM_NC; e += 256) {
        const int bb = e % TRMM_DB, cc = e / TRMM_DB;
        const int64_t k = i0 + bb, c = c0 + cc;
        Es[bb][cc] = (k < m && c < r) ? E[k + c * lde] : 0.0;
    }
    __syncthreads();
    const int a = tid % TRMM_DB, h = tid / TRMM_DB;
    const int64_t i = i0 + a;
    const int bmax = (int)((m - i0) < TRMM_DB ? (m - i0) : TRMM_DB);
    double acc[TRMM_NC / 2];
#pragma unroll
    for (int q = 0; q < TRMM_NC / 2; ++q) acc[q] = 0.0;
    for (int b = 0; b < bmax; ++b) {
        const double l = (b <= a && i < m) ? L[i + (i0 + b) * ldl] : 0.0;
#pragma unroll
        for (int q = 0; q < TRMM_NC / 2; ++q) acc[q] = fma(l, Es[b][h * (TRMM_NC / 2) + q], acc[q]);
    }
    if (i >= m) return;
#pragma unroll
    for (int q = 0; q < TRMM_NC / 2; ++q) {
        const int64_t c = c0 + h * (TRMM_NC / 2) + q;
        if (c < r) out[i + c * ldo] += acc[q];
    }
}

__global__ __launch_bounds__(256) void k_bcast_rows(int64_t m, int64_t r, const double *mean, double mu, double *out,
                                                    int64_t ldo) {
    const int64_t c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
        out[i + c * ldo] = mean ? mean[i] : mu;
}

__global__ __launch_bounds__(256) void k_fail_fill(int64_t m, int64_t r, double *out, int64_t ldo, const int32_t *info) {
    if (*info == 0) return;
    const int64_t c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
        out[i + c * ldo] = __builtin_nan("");
}

// column j = j0 + blockIdx.y: rows 0 .. j - 1 set to zero
__global__ __launch_bounds__(256) void k_zero_upper(int64_t j0, double *A, int64_t lda) {
    const int64_t j = j0 + blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < j; i += (int64_t)gridDim.x * 256)
        A[i + j * lda] = 0.0;
}

// grid.y carries the columns: at most 65535 per launch
constexpr int64_t MAX_GRID_Y = 65535;

unsigned row_blocks(int64_t m) {
    const int64_t b = (m + 255) / 256;
    return (unsigned)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}

}  // namespace

hipError_t launch_trmm_diag(hipStream_t s, int64_t m, int64_t r, const double *L, int64_t ldl, const double *E,
                            int64_t lde, double *out, int64_t ldo, const int32_t *info) {
    if (m <= 0 || r <= 0) return hipSuccess;
    const int64_t nblk = (m + TRMM_DB - 1) / TRMM_DB, nch = (r + TRMM_NC - 1) / TRMM_NC;
    for (int64_t c0 = 0; c0 < nch; c0 += MAX_GRID_Y) {
        const int64_t cn = nch - c0 < MAX_GRID_Y ? nch - c0 : MAX_GRID_Y;
        hipLaunchKernelGGL(k_trmm_diag, dim3((unsigned)nblk, (unsigned)cn), dim3(256), 0, s, m, r - c0 * TRMM_NC, L,
                           ldl, E + c0 * TRMM_NC * lde, lde, out + c0 * TRMM_NC * ldo, ldo, info);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_bcast_rows(hipStream_t s, int64_t m, int64_t r, const double *mean, double mu, double *out,
                             int64_t ldo) {
    for (int64_t c0 = 0; c0 < r; c0 += MAX_GRID_Y) {
        const int64_t cn = r - c0 < MAX_GRID_Y ? r - c0 : MAX_GRID_Y;
        if (m <= 0) break;
        hipLaunchKernelGGL(k_bcast_rows, dim3(row_blocks(m), (unsigned)cn), dim3(256), 0, s, m, cn, mean, mu,
                           out + c0 * ldo, ldo);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fail_fill(hipStream_t s, int64_t m, int64_t r, double *out, int64_t ldo, const int32_t *info) {
    for (int64_t c0 = 0; c0 < r; c0 += MAX_GRID_Y) {
        const int64_t cn = r - c0 < MAX_GRID_Y ? r - c0 : MAX_GRID_Y;
        if (m <= 0) break;
        hipLaunchKernelGGL(k_fail_fill, dim3(row_blocks(m), (unsigned)cn), dim3(256), 0, s, m, cn, out + c0 * ldo, ldo,
                           info);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_zero_upper(hipStream_t s, int64_t m, double *A, int64_t lda) {
    for (int64_t c0 = 1; c0 < m; c0 += MAX_GRID_Y) {
        const int64_t cn = m - c0 < MAX_GRID_Y ? m - c0 : MAX_GRID_Y;
        // columns c0 .. c0 + cn - 1, rows 0 .. j - 1 (j the absolute column)
        hipLaunchKernelGGL(k_zero_upper, dim3(row_blocks(c0 + cn), (unsigned)cn), dim3(256), 0, s, c0, A, lda);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
