// k_batch.hip -- many independent Gaussian-process likelihoods, batched
// (the same model and quantities as the single-problem path: C(theta),
// L L^T = C, L^{-1} y, log|C|, loglik; Section 1).
//
// Level-synchronous tile Cholesky over the whole batch on 64 x 64 tiles.  For
// tile column j = 0, 1, ... two launches cover every problem at once:
//   diag(j):  C_jj - sum_{k<j} L_jk L_jk^T (left-looking, matrix cores), then
//             factor + invert it in one wave's registers (the diagonal-block
//             Cholesky of Section 2.1 / Fig. 1);
//   panel(j): for every tile i > j of every problem,
//             L_ij = (C_ij - sum_{k<j} L_ik L_jk^T) Winv_jj^T.
// Covariance tiles are generated from the points inside these kernels (C is
// never written as a whole).  A final launch runs, per problem, the forward
// solve z = L^{-1} y and the log-determinant / quadratic-form reductions.
// No workgroup ever waits on another: kernel boundaries order the steps.
#include "internal.h"

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

struct BProb {
    int64_t n, x_off, c_off, z_off, w_off;
    double s2, inv_rho, t2;
    int32_t kind, nt;
};
struct BTile {
    int32_t prob, i;
};

constexpr int T = 64;

// acc = sum_{k < j} L_ik L_jk^T for one 64 x 64 tile (4 waves, 32 x 32 each,
// f64 MFMA layout: row lane/16 + 4r, column lane%16).
GP_DEV void tile_update(const double *L, int64_t ld, int64_t n, int64_t i0, int64_t j0, int j,
                        double (*As)[T + 1], double (*Bs)[T + 1], v4d (&acc)[2][2]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[m][q] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < j; ++k) {
        const int64_t k0 = (int64_t)k * T;  // block k < j is a full block
        __syncthreads();
#pragma unroll
        for (int r = 0; r < (T * T) / 256; ++r) {
            const int e = r * 256 + tid;
            const int ii = e & (T - 1), kk = e >> 6;
            const int64_t gi = i0 + ii, gj = j0 + ii;
            const double va = L[gi < n ? gi + (k0 + kk) * ld : 0];
            const double vb = L[gj < n ? gj + (k0 + kk) * ld : 0];
            As[kk][ii] = gi < n ? va : 0.0;
            Bs[kk][ii] = gj < n ? vb : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < T; kk += 4) {
            double a[2], b[2];
#pragma unroll
            for (int m = 0; m < 2; ++m) a[m] = As[kk + (lane >> 4)][wm * 32 + m * 16 + (lane & 15)];
#pragma unroll
            for (int q = 0; q < 2; ++q) b[q] = Bs[kk + (lane >> 4)][wn * 32 + q * 16 + (lane & 15)];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    acc[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[q], acc[m][q], 0, 0, 0);
        }
    }
    __syncthreads();
}

// S = C_ij - acc with C regenerated from the points; identity padding of the
// last diagonal tile.
GP_DEV void tile_residual(const BProb &P, const double *Xb, int dim, int64_t i0, int64_t j0,
                          const v4d (&acc)[2][2], double (&sv)[2][2][4]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w & 1, wn = w >> 1;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = i0 + wm * 32 + m * 16 + (lane >> 4) + 4 * r;
                const int64_t gj = j0 + wn * 32 + q * 16 + (lane & 15);
                double c;
                if (gi < P.n && gj < P.n) {
                    const double d = point_dist(Xb + gi * dim, Xb + gj * dim, dim);
                    c = P.s2 * cov_corr(P.kind, d * P.inv_rho) + (gi == gj ? P.t2 : 0.0);
                } else {
                    c = (gi == gj) ? 1.0 : 0.0;
                }
                sv[m][q][r] = c - acc[m][q][r];
            }
}

__global__ __launch_bounds__(256, 1) void k_bdiag(const BProb *__restrict__ probs, const int32_t *__restrict__ plist,
                                                  int j, int dim, const double *__restrict__ X, double *C_pool,
                                                  double *wbuf, int32_t *info) {
    __shared__ double As[T][T + 1];
    __shared__ double Bs[T][T + 1];  // staging of the update, then the inverse
    __shared__ union {
        double pn[T][17];
        double t32[32][33];
    } U;
    __shared__ double rd[T];
    __shared__ int s_fail;
    const int b = plist[blockIdx.x];
    if (info[b] != 0) return;
    const BProb P = probs[b];
    const int64_t ld = P.n, j0 = (int64_t)j * T;
    double *L = C_pool + P.c_off;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    v4d acc[2][2];
    tile_update(L, ld, P.n, j0, j0, j, As, Bs, acc);
    double sv[2][2][4];
    tile_residual(P, X + P.x_off * dim, dim, j0, j0, acc, sv);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                As[wm * 32 + m * 16 + (lane >> 4) + 4 * r][wn * 32 + q * 16 + (lane & 15)] = sv[m][q][r];
    if (tid == 0) s_fail = 0;
    __syncthreads();
    if (w != 0) return;  // one wave factors and inverts the tile
    const int tj = (int)((P.n - j0) < T ? (P.n - j0) : T);
    double a[T];
#pragma unroll
    for (int c = 0; c < T; ++c) a[c] = As[lane][c];
    const int fail = wave_chol64(a, lane, As, U.pn);
    if (fail) {
        if (lane == 0) info[b] = (int32_t)(j0 + fail);
        return;
    }
#pragma unroll
    for (int c = 0; c < T; ++c) {
        As[lane][c] = a[c];
        if (lane < tj && c <= lane) L[(j0 + lane) + (j0 + c) * ld] = a[c];
    }
    wave_lds_sync();
    wave_inv64_blocked(As, Bs, U.t32, rd, lane);
    double *W = wbuf + P.w_off + (int64_t)j * T * T;
#pragma unroll 4
    for (int c = 0; c < T; ++c) W[lane + c * T] = Bs[lane][c];
}

__global__ __launch_bounds__(256, 2) void k_bpanel(const BProb *__restrict__ probs, const BTile *__restrict__ tlist,
                                                   int j, int dim, const double *__restrict__ X, double *C_pool,
                                                   const double *__restrict__ wbuf, const int32_t *__restrict__ info) {
    __shared__ double As[T][T + 1];
    __shared__ double Bs[T][T + 1];
    const BTile tk = tlist[blockIdx.x];
    if (info[tk.prob] != 0) return;
    const BProb P = probs[tk.prob];
    const int64_t ld = P.n, i0 = (int64_t)tk.i * T, j0 = (int64_t)j * T;
    double *L = C_pool + P.c_off;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    v4d acc[2][2];
    tile_update(L, ld, P.n, i0, j0, j, As, Bs, acc);
    double sv[2][2][4];
    tile_residual(P, X + P.x_off * dim, dim, i0, j0, acc, sv);
    // L_ij = S W_jj^T: A operand S staged k-major (As[kk][ii] = S[ii][kk]),
    // op(B)[kk][jj] = W_jj[jj][kk] = W[jj + kk T]
    const double *W = wbuf + P.w_off + (int64_t)j * T * T;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                As[wn * 32 + q * 16 + (lane & 15)][wm * 32 + m * 16 + (lane >> 4) + 4 * r] = sv[m][q][r];
#pragma unroll
    for (int r = 0; r < (T * T) / 256; ++r) {
        const int e = r * 256 + tid;
        Bs[e >> 6][e & (T - 1)] = W[e];
    }
    __syncthreads();
    v4d o[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q) o[m][q] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < T; kk += 4) {
        double a[2], bb[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) a[m] = As[kk + (lane >> 4)][wm * 32 + m * 16 + (lane & 15)];
#pragma unroll
        for (int q = 0; q < 2; ++q) bb[q] = Bs[kk + (lane >> 4)][wn * 32 + q * 16 + (lane & 15)];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int q = 0; q < 2; ++q)
                o[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], bb[q], o[m][q], 0, 0, 0);
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = i0 + wm * 32 + m * 16 + (lane >> 4) + 4 * r;
                const int64_t gj = j0 + wn * 32 + q * 16 + (lane & 15);
                if (gi < P.n && gj < P.n) L[gi + gj * ld] = o[m][q][r];
            }
}

// Per problem: z = L^{-1} y block by block (this workgroup only), then
// log|C| = 2 sum log L_ii, q = z^T z and the log-likelihood.
__global__ __launch_bounds__(256) void k_bsolve(const BProb *__restrict__ probs, const double *__restrict__ y,
                                                const double *__restrict__ C_pool, double *zbuf,
                                                const double *__restrict__ wbuf, double *out3, const int32_t *info) {
    __shared__ double red[4][T];
    __shared__ double rhs[T];
    __shared__ double r2[4 * 256];
    const int b = blockIdx.x;
    const BProb P = probs[b];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double *o = out3 + 3 * (int64_t)b;
    if (info[b] != 0) {
        if (tid == 0) o[0] = o[1] = o[2] = __builtin_nan("");
        return;
    }
    const int64_t n = P.n, ld = P.n;
    const double *L = C_pool + P.c_off;
    double *z = zbuf + P.z_off;
    for (int i = 0; i < P.nt; ++i) {
        const int64_t gi = (int64_t)i * T + lane;
        const bool rv = gi < n;
        double acc = 0.0;
        for (int k = w; k < i; k += 4) {
            const double *Lc = L + (rv ? gi : 0) + (int64_t)k * T * ld;
            const double *zk = z + (int64_t)k * T;
            if (rv) {
#pragma unroll 16
                for (int c = 0; c < T; ++c) acc = fma(Lc[(int64_t)c * ld], zk[c], acc);
            }
        }
        red[w][lane] = acc;
        __syncthreads();
        if (w == 0) rhs[lane] = rv ? y[P.x_off + gi] - (((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]) : 0.0;
        __syncthreads();
        const double *W = wbuf + P.w_off + (int64_t)i * T * T;
        double sacc = 0.0;
        for (int c = w * 16; c < w * 16 + 16; ++c) sacc = fma(W[lane + c * T], rhs[c], sacc);
        red[w][lane] = sacc;
        __syncthreads();
        if (w == 0 && rv) z[gi] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        __syncthreads();  // z_i (global, this workgroup) visible before the next block reads it
    }
    CSum sl, sq;
    for (int64_t q = tid; q < n; q += 256) {
        sl.add(log(L[q + q * ld]));
        sq.add(z[q] * z[q]);
    }
    r2[tid * 4 + 0] = sl.s; r2[tid * 4 + 1] = sl.c; r2[tid * 4 + 2] = sq.s; r2[tid * 4 + 3] = sq.c;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) {
            for (int h = 0; h < 2; ++h) {
                CSum a, c;
                a.s = r2[tid * 4 + 2 * h]; a.c = r2[tid * 4 + 2 * h + 1];
                c.s = r2[(tid + st) * 4 + 2 * h]; c.c = r2[(tid + st) * 4 + 2 * h + 1];
                a.merge(c);
                r2[tid * 4 + 2 * h] = a.s; r2[tid * 4 + 2 * h + 1] = a.c;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double logdet = 2.0 * (r2[0] + r2[1]);
        const double q = r2[2] + r2[3];
        o[1] = logdet;
        o[2] = q;
        o[0] = -0.5 * (((double)n * 1.8378770664093453 + logdet) + q);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side: per-step problem / tile lists, workspace layout, launches.
// ---------------------------------------------------------------------------
#include <algorithm>
#include <cmath>
#include <vector>

namespace {
inline size_t al256b(size_t x) { return (x + 255) & ~(size_t)255; }
}

size_t batch_ws_bytes(int64_t nmax, int64_t nbatch) {
    const int64_t nt = (nmax + T - 1) / T;
    size_t b = 0;
    b += al256b(sizeof(BProb) * (size_t)nbatch);
    b += al256b(sizeof(int32_t) * (size_t)nt * (size_t)nbatch);                  // diag lists
    b += al256b(sizeof(BTile) * (size_t)(nt * (nt + 1) / 2) * (size_t)nbatch);   // panel lists
    b += al256b(sizeof(double) * (size_t)nmax * (size_t)nbatch);                 // z
    b += al256b(sizeof(double) * (size_t)nt * T * T * (size_t)nbatch);           // diagonal inverses
    return b + 256;
}

struct BatchStaging {
    std::vector<BProb> probs;
    std::vector<int32_t> dlist;
    std::vector<BTile> tlist;
    hipEvent_t done = nullptr;
};

int batch_run(hipStream_t s, int num_cu, void *&staging_ptr, int32_t nb, const gp_theta_t *th, const int64_t *nh,
              const int64_t *xoff, const int64_t *coff, int32_t dim, const double *X, const double *y,
              double *C_pool, double *out3, int32_t *info, void *ws, size_t ws_bytes) {
    (void)num_cu;
    BatchStaging *st = static_cast<BatchStaging *>(staging_ptr);
    if (!st) {
        st = new BatchStaging();
        staging_ptr = st;
    }
    if (st->done) {
        if (hipEventSynchronize(st->done) != hipSuccess) return GP_ERR_HIP;  // host copy of the last call consumed
    } else if (hipEventCreateWithFlags(&st->done, hipEventDisableTiming) != hipSuccess) {
        return GP_ERR_HIP;
    }
    int64_t nmax = 1;
    for (int b = 0; b < nb; ++b) nmax = std::max(nmax, nh[b]);
    if (ws_bytes < batch_ws_bytes(nmax, nb)) return GP_ERR_WS_TOO_SMALL;
    const int64_t ntmax = (nmax + T - 1) / T;
    st->probs.assign(nb, BProb{});
    int64_t zoff = 0, woff = 0;
    for (int b = 0; b < nb; ++b) {
        BProb &p = st->probs[b];
        p.n = nh[b];
        p.x_off = xoff[b];
        p.c_off = coff[b];
        p.nt = (int32_t)((p.n + T - 1) / T);
        p.z_off = zoff;
        zoff += p.n;
        p.w_off = woff;
        woff += (int64_t)p.nt * T * T;
        p.kind = th[b].kind;
        p.s2 = std::exp(th[b].log_sigma2);
        p.inv_rho = std::exp(-th[b].log_rho);
        p.t2 = std::exp(th[b].log_tau2);
    }
    // step j: problems with nt > j (diagonal tile), tiles (b, i > j) (panel);
    // larger problems first within a step
    std::vector<int> order(nb);
    for (int b = 0; b < nb; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return nh[a] > nh[c]; });
    std::vector<int64_t> doff(ntmax + 1, 0), toff(ntmax + 1, 0);
    st->dlist.clear();
    st->tlist.clear();
    for (int64_t j = 0; j < ntmax; ++j) {
        doff[j] = (int64_t)st->dlist.size();
        toff[j] = (int64_t)st->tlist.size();
        for (int b : order)
            if (st->probs[b].nt > j) st->dlist.push_back(b);
        for (int b : order)
            for (int i = (int)j + 1; i < st->probs[b].nt; ++i) st->tlist.push_back(BTile{b, i});
    }
    doff[ntmax] = (int64_t)st->dlist.size();
    toff[ntmax] = (int64_t)st->tlist.size();

    char *base = static_cast<char *>(ws);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off += al256b(bytes);
        return p;
    };
    BProb *d_probs = reinterpret_cast<BProb *>(take(sizeof(BProb) * (size_t)nb));
    int32_t *d_dl = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)ntmax * (size_t)nb));
    BTile *d_tl = reinterpret_cast<BTile *>(take(sizeof(BTile) * (size_t)(ntmax * (ntmax + 1) / 2) * (size_t)nb));
    double *d_z = reinterpret_cast<double *>(take(sizeof(double) * (size_t)nmax * (size_t)nb));
    double *d_w = reinterpret_cast<double *>(take(sizeof(double) * (size_t)ntmax * T * T * (size_t)nb));

    if (hipMemcpyAsync(d_probs, st->probs.data(), sizeof(BProb) * (size_t)nb, hipMemcpyHostToDevice, s) != hipSuccess)
        return GP_ERR_HIP;
    if (!st->dlist.empty() &&
        hipMemcpyAsync(d_dl, st->dlist.data(), sizeof(int32_t) * st->dlist.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return GP_ERR_HIP;
    if (!st->tlist.empty() &&
        hipMemcpyAsync(d_tl, st->tlist.data(), sizeof(BTile) * st->tlist.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return GP_ERR_HIP;
    if (hipEventRecord(st->done, s) != hipSuccess) return GP_ERR_HIP;
    if (launch_fill(s, info, sizeof(int32_t) * (size_t)nb) != hipSuccess) return GP_ERR_HIP;
    for (int64_t j = 0; j < ntmax; ++j) {
        const int64_t nd = doff[j + 1] - doff[j], ntl = toff[j + 1] - toff[j];
        if (nd > 0)
            hipLaunchKernelGGL(k_bdiag, dim3((unsigned)nd), dim3(256), 0, s, d_probs, d_dl + doff[j], (int)j, dim, X,
                               C_pool, d_w, info);
        if (ntl > 0)
            hipLaunchKernelGGL(k_bpanel, dim3((unsigned)ntl), dim3(256), 0, s, d_probs, d_tl + toff[j], (int)j, dim, X,
                               C_pool, d_w, info);
        if (hipGetLastError() != hipSuccess) return GP_ERR_HIP;
    }
    hipLaunchKernelGGL(k_bsolve, dim3((unsigned)nb), dim3(256), 0, s, d_probs, y, C_pool, d_z, d_w, out3, info);
    return hipGetLastError() == hipSuccess ? GP_OK : GP_ERR_HIP;
}

void batch_staging_free(void *p) {
    BatchStaging *st = static_cast<BatchStaging *>(p);
    if (!st) return;
    if (st->done) {
        (void)hipEventSynchronize(st->done);
        (void)hipEventDestroy(st->done);
    }
    delete st;
}
