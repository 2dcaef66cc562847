// k_batch.hip -- many independent Gaussian-process likelihoods, batched
// (the same model and quantities as the single-problem path: C(theta),
// L L^T = C, L^{-1} y, log|C|, loglik; Section 1).
//
// Level-synchronous right-looking tile Cholesky over the whole batch on
// 64 x 64 tiles.  The covariance tiles of every problem are written once
// (lower triangle), then for tile column j = 0, 1, ... three launches cover
// every problem at once:
//   diag(j):   factor the (already updated) tile A_jj in one wave's registers
//              and invert it (the diagonal-block Cholesky of Section 2.1 /
//              Fig. 1);
//   panel(j):  L_ij = A_ij W_jj^T for every tile i > j;
//   update:    A_ik -= L_ij L_kj^T on the matrix cores, taken for two tile
//              columns at once (rank 128) after the column j + 1 alone has
//              been brought up to date for diag / panel(j + 1).
// Every launch of a level has the same short K, so a level costs the same
// whatever the problem sizes; problems are ordered largest first and each
// workgroup finds its problem and tile from per-level prefix counts.  The
// forward solve z = L^{-1} y rides along (diag: z_j = W_j y'_j; panel:
// y'_i -= L_ij z_j); a final launch forms, per problem, the log-determinant /
// quadratic-form reductions.  No workgroup ever waits on
// another: kernel boundaries order the steps.
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

GP_DEV void btri_decode(int64_t t, int64_t &r, int64_t &c) {  // t = r (r + 1) / 2 + c, c <= r
    double f = (sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5;
    r = (int64_t)f;
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    c = t - r * (r + 1) / 2;
}

// Largest q < cnt with off[q] <= t (off non-decreasing, off[0] = 0).
GP_DEV int find_prob(const int64_t *off, int cnt, int64_t t) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// acc (+)= X Y^T for two 64 x 64 blocks (rows past xr / yr read as zero): both
// staged k-major in LDS, 4 waves of 32 x 32 (f64 MFMA layout: row lane / 16 +
// 4 r, column lane % 16 within each 16 x 16 block).
GP_DEV void tile_nt(const double *X, int64_t ldx, int xr, const double *Y, int64_t ldy, int yr, double (*As)[T + 1],
                    double (*Bs)[T + 1], v4d (&acc)[2][2], bool accumulate = false) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    double va[(T * T) / 256], vb[(T * T) / 256];
    if (accumulate) __syncthreads();  // the previous product's LDS reads are done
#pragma unroll
    for (int r = 0; r < (T * T) / 256; ++r) {
        const int e = r * 256 + tid, ii = e & (T - 1), kk = e >> 6;
        va[r] = ii < xr ? X[ii + (int64_t)kk * ldx] : 0.0;
        vb[r] = ii < yr ? Y[ii + (int64_t)kk * ldy] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < (T * T) / 256; ++r) {
        const int e = r * 256 + tid, ii = e & (T - 1), kk = e >> 6;
        As[kk][ii] = va[r];
        Bs[kk][ii] = vb[r];
    }
    __syncthreads();
    if (!accumulate) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int q = 0; q < 2; ++q) acc[m][q] = v4d{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll 4
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

// Covariance tiles (i, k), k <= i, of every problem (full 64 x 64 squares,
// clipped to the problem).
__global__ __launch_bounds__(256) void k_bcov(const BProb *__restrict__ probs, const int32_t *__restrict__ order,
                                              const int64_t *__restrict__ off, int cnt, int dim,
                                              const double *__restrict__ X, const double *__restrict__ y,
                                              double *C_pool, double *zbuf) {
    const int q = find_prob(off, cnt, blockIdx.x);
    const BProb P = probs[order[q]];
    int64_t ti, tk;
    btri_decode(blockIdx.x - off[q], ti, tk);
    const int64_t i0 = ti * T, k0 = tk * T;
    double *C = C_pool + P.c_off;
    const double *Xb = X + P.x_off * dim;
    if (ti == 0 && tk == 0)  // the forward solve's right-hand side, updated in place by the levels
        for (int64_t e = threadIdx.x; e < P.n; e += 256) zbuf[P.z_off + e] = y[P.x_off + e];
    for (int e = threadIdx.x; e < T * T; e += 256) {
        const int64_t gi = i0 + (e & (T - 1)), gk = k0 + (e >> 6);
        if (gi < P.n && gk < P.n) {
            const double d = point_dist(Xb + gi * dim, Xb + gk * dim, dim);
            C[gi + gk * P.n] = P.s2 * cov_corr(P.kind, d * P.inv_rho) + (gi == gk ? P.t2 : 0.0);
        }
    }
}

// Factor + invert the diagonal tile j of problem order[blockIdx.x] (one wave).
__global__ __launch_bounds__(64) void k_bdiag(const BProb *__restrict__ probs, const int32_t *__restrict__ order,
                                              int j, double *C_pool, double *wbuf, double *zbuf, int32_t *info) {
    __shared__ double Ls[T][T + 1];
    __shared__ double Wl[T][T + 1];
    __shared__ union {
        double pn[T][17];
        double t32[32][33];
    } U;
    __shared__ double rd[T];
    const int b = order[blockIdx.x];
    if (info[b] != 0) return;
    const BProb P = probs[b];
    const int64_t ld = P.n, j0 = (int64_t)j * T;
    const int tj = (int)((P.n - j0) < T ? (P.n - j0) : T);
    double *D = C_pool + P.c_off + j0 + j0 * ld;
    const int lane = threadIdx.x;
    double a[T];
#pragma unroll
    for (int c = 0; c < T; ++c) {
        double v;
        if (lane < tj && c < tj) v = (c <= lane) ? D[lane + (int64_t)c * ld] : 0.0;
        else v = (lane == c) ? 1.0 : 0.0;  // identity padding decouples unused rows
        a[c] = v;
    }
    const int fail = wave_chol64(a, lane, Ls, U.pn);
    if (fail) {
        if (lane == 0) info[b] = (int32_t)(j0 + fail);
        return;
    }
#pragma unroll
    for (int c = 0; c < T; ++c) {
        Ls[lane][c] = a[c];
        if (lane < tj && c < tj && c <= lane) D[lane + (int64_t)c * ld] = a[c];
    }
    wave_lds_sync();
    wave_inv64_blocked(Ls, Wl, U.t32, rd, lane);
    double *W = wbuf + P.w_off + (int64_t)j * T * T;
#pragma unroll 4
    for (int c = 0; c < T; ++c) W[lane + c * T] = Wl[lane][c];
    // forward solve of this block: z_j = W_j y'_j (y'_j holds y_j minus the
    // products of the earlier blocks, subtracted by the panel steps)
    double *z = zbuf + P.z_off + j0;
    rd[lane] = lane < tj ? z[lane] : 0.0;
    wave_lds_sync();
    double zr = 0.0;
#pragma unroll 8
    for (int c = 0; c < T; ++c) zr = fma(Wl[lane][c], rd[c], zr);
    if (lane < tj) z[lane] = zr;
}

// L_ij = A_ij W_jj^T for tile i = j + 1 + (t - off[q]) of problem order[q].
__global__ __launch_bounds__(256, 2) void k_bpanel(const BProb *__restrict__ probs, const int32_t *__restrict__ order,
                                                   const int64_t *__restrict__ off, int cnt, int j, double *C_pool,
                                                   const double *__restrict__ wbuf, double *zbuf,
                                                   const int32_t *__restrict__ info) {
    __shared__ double As[T][T + 1];
    __shared__ double Bs[T][T + 1];
    const int q = find_prob(off, cnt, blockIdx.x);
    const int b = order[q];
    if (info[b] != 0) return;
    const BProb P = probs[b];
    const int64_t ld = P.n, i0 = (j + 1 + (blockIdx.x - off[q])) * (int64_t)T, j0 = (int64_t)j * T;
    const int ri = (int)((P.n - i0) < T ? (P.n - i0) : T);
    double *A = C_pool + P.c_off + i0 + j0 * ld;
    v4d acc[2][2];
    tile_nt(A, ld, ri, wbuf + P.w_off + (int64_t)j * T * T, T, T, As, Bs, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w & 1, wn = w >> 1;
    __syncthreads();  // As is reused for L_ij below
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int qq = 0; qq < 2; ++qq)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wm * 32 + m * 16 + (lane >> 4) + 4 * r, col = wn * 32 + qq * 16 + (lane & 15);
                As[row][col] = acc[m][qq][r];
                if (row < ri) A[row + (int64_t)col * ld] = acc[m][qq][r];
            }
    __syncthreads();
    // forward solve: y'_i -= L_ij z_j (this tile is the only writer of y'_i at this level)
    if (w == 0) {
        const double *zj = zbuf + P.z_off + j0;
        double u = 0.0;
#pragma unroll 8
        for (int c = 0; c < T; ++c) u = fma(As[lane][c], zj[c], u);
        if (lane < ri) zbuf[P.z_off + i0 + lane] -= u;
    }
}

// A_ik -= sum_{c < nk} L_{i,j+c} L_{k,j+c}^T for one trailing tile of problem
// order[q], u = t - off[q]: column mode (k = base, i = base + u) or triangle
// mode (base <= k <= i, (i - base, k - base) the u-th pair of the lower
// triangle).  nk = 2 applies two panel columns at once (rank 128), which
// halves the C traffic of the update.
__global__ __launch_bounds__(256, 2) void k_bupdate(const BProb *__restrict__ probs, const int32_t *__restrict__ order,
                                                    const int64_t *__restrict__ off, int cnt, int j, int nk, int base,
                                                    int column, double *C_pool, const int32_t *__restrict__ info) {
    __shared__ double As[T][T + 1];
    __shared__ double Bs[T][T + 1];
    const int q = find_prob(off, cnt, blockIdx.x);
    const int b = order[q];
    if (info[b] != 0) return;
    const BProb P = probs[b];
    int64_t ti, tk;
    const int64_t u = blockIdx.x - off[q];
    if (column) {
        ti = u;
        tk = 0;
    } else {
        btri_decode(u, ti, tk);
    }
    const int64_t ld = P.n, j0 = (int64_t)j * T;
    const int64_t i0 = (base + ti) * (int64_t)T, k0 = (base + tk) * (int64_t)T;
    const int ri = (int)((P.n - i0) < T ? (P.n - i0) : T), rk = (int)((P.n - k0) < T ? (P.n - k0) : T);
    double *L = C_pool + P.c_off;
    double *A = L + i0 + k0 * ld;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w & 1, wn = w >> 1;
    // the C tile's loads first, so their latency overlaps the operand product
    double cv[2][2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int qq = 0; qq < 2; ++qq)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wm * 32 + m * 16 + (lane >> 4) + 4 * r, col = wn * 32 + qq * 16 + (lane & 15);
                cv[m][qq][r] = (row < ri && col < rk) ? A[row + (int64_t)col * ld] : 0.0;
            }
    v4d acc[2][2];
    tile_nt(L + i0 + j0 * ld, ld, ri, L + k0 + j0 * ld, ld, rk, As, Bs, acc);
    if (nk == 2) tile_nt(L + i0 + (j0 + T) * ld, ld, ri, L + k0 + (j0 + T) * ld, ld, rk, As, Bs, acc, true);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int qq = 0; qq < 2; ++qq)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wm * 32 + m * 16 + (lane >> 4) + 4 * r, col = wn * 32 + qq * 16 + (lane & 15);
                if (row < ri && col < rk) A[row + (int64_t)col * ld] = cv[m][qq][r] - acc[m][qq][r];
            }
}

// Per problem: log|C| = 2 sum log L_ii, q = z^T z (z = L^{-1} y, formed by
// the levels) and the log-likelihood.
__global__ __launch_bounds__(256) void k_bsolve(const BProb *__restrict__ probs, const double *__restrict__ C_pool,
                                                const double *__restrict__ zbuf, double *out3, const int32_t *info) {
    __shared__ double r2[4 * 256];
    const int b = blockIdx.x;
    const BProb P = probs[b];
    const int tid = threadIdx.x;
    double *o = out3 + 3 * (int64_t)b;
    if (info[b] != 0) {
        if (tid == 0) o[0] = o[1] = o[2] = __builtin_nan("");
        return;
    }
    const int64_t n = P.n, ld = P.n;
    const double *L = C_pool + P.c_off;
    const double *z = zbuf + P.z_off;
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
    b += al256b(sizeof(int32_t) * (size_t)nbatch);                              // size order
    b += al256b(sizeof(int64_t) * (size_t)(2 * nt + 1) * (size_t)(nbatch + 1));  // per-level prefix counts
    b += al256b(sizeof(double) * (size_t)nmax * (size_t)nbatch);                 // z
    b += al256b(sizeof(double) * (size_t)nt * T * T * (size_t)nbatch);           // diagonal inverses
    return b + 256;
}

struct BatchStaging {
    std::vector<BProb> probs;
    std::vector<int32_t> order;
    std::vector<int64_t> offs;  // [level block][nb + 1]: covariance, then per level panel and update counts
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
    // problems largest first: at level j the first cnt[j] of them have a
    // diagonal tile; prefix counts of their covariance / panel / update tiles
    st->order.resize(nb);
    for (int b = 0; b < nb; ++b) st->order[b] = b;
    std::stable_sort(st->order.begin(), st->order.end(), [&](int a, int c) { return nh[a] > nh[c]; });
    const int64_t W = nb + 1;
    st->offs.assign((size_t)(2 * ntmax + 1) * (size_t)W, 0);
    std::vector<int> cnt(ntmax + 1, 0);
    auto tri = [](int64_t m) { return m > 0 ? m * (m + 1) / 2 : 0; };
    for (int q = 0; q < nb; ++q) st->offs[q + 1] = st->offs[q] + tri(st->probs[st->order[q]].nt);
    for (int64_t j = 0; j < ntmax; ++j) {
        int c = 0;
        while (c < nb && st->probs[st->order[c]].nt > j) ++c;
        cnt[j] = c;
        int64_t *po = &st->offs[(size_t)(1 + 2 * j) * W], *uo = &st->offs[(size_t)(2 + 2 * j) * W];
        for (int q = 0; q < c; ++q) {
            const int64_t m = st->probs[st->order[q]].nt - j - 1;
            po[q + 1] = po[q] + (m > 0 ? m : 0);
            uo[q + 1] = uo[q] + tri(m);
        }
    }

    char *base = static_cast<char *>(ws);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off += al256b(bytes);
        return p;
    };
    BProb *d_probs = reinterpret_cast<BProb *>(take(sizeof(BProb) * (size_t)nb));
    int32_t *d_order = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)nb));
    int64_t *d_offs = reinterpret_cast<int64_t *>(take(sizeof(int64_t) * st->offs.size()));
    double *d_z = reinterpret_cast<double *>(take(sizeof(double) * (size_t)nmax * (size_t)nb));
    double *d_w = reinterpret_cast<double *>(take(sizeof(double) * (size_t)ntmax * T * T * (size_t)nb));

    if (hipMemcpyAsync(d_probs, st->probs.data(), sizeof(BProb) * (size_t)nb, hipMemcpyHostToDevice, s) != hipSuccess)
        return GP_ERR_HIP;
    if (hipMemcpyAsync(d_order, st->order.data(), sizeof(int32_t) * (size_t)nb, hipMemcpyHostToDevice, s) != hipSuccess)
        return GP_ERR_HIP;
    if (hipMemcpyAsync(d_offs, st->offs.data(), sizeof(int64_t) * st->offs.size(), hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return GP_ERR_HIP;
    if (hipEventRecord(st->done, s) != hipSuccess) return GP_ERR_HIP;
    if (launch_fill(s, info, sizeof(int32_t) * (size_t)nb) != hipSuccess) return GP_ERR_HIP;
    const int64_t ncov = st->offs[nb];
    if (ncov > 0)
        hipLaunchKernelGGL(k_bcov, dim3((unsigned)ncov), dim3(256), 0, s, d_probs, d_order, d_offs, nb, dim, X, y, C_pool,
                           d_z);
    auto poff = [&](int64_t j) { return (size_t)(1 + 2 * j) * W; };
    auto uoff = [&](int64_t j) { return (size_t)(2 + 2 * j) * W; };
    auto diag_panel = [&](int64_t j) {
        const int c = cnt[j];
        const int64_t np = st->offs[poff(j) + c];
        if (c > 0)
            hipLaunchKernelGGL(k_bdiag, dim3((unsigned)c), dim3(64), 0, s, d_probs, d_order, (int)j, C_pool, d_w, d_z,
                               info);
        if (np > 0)
            hipLaunchKernelGGL(k_bpanel, dim3((unsigned)np), dim3(256), 0, s, d_probs, d_order, d_offs + poff(j), c,
                               (int)j, C_pool, d_w, d_z, info);
    };
    // Tile columns in pairs (j, j + 1): diag / panel of j, the update of
    // column j + 1 alone, diag / panel of j + 1, then one rank-128 update of
    // the tiles right of both (counts of those = the update counts of j + 1).
    for (int64_t j = 0; j < ntmax;) {
        diag_panel(j);
        if (j + 1 < ntmax) {
            const int c = cnt[j];
            const int64_t ncol = st->offs[poff(j) + c];  // tiles (i, j + 1), i > j: one per panel tile
            if (ncol > 0)
                hipLaunchKernelGGL(k_bupdate, dim3((unsigned)ncol), dim3(256), 0, s, d_probs, d_order, d_offs + poff(j),
                                   c, (int)j, 1, (int)j + 1, 1, C_pool, info);
            diag_panel(j + 1);
            const int c1 = cnt[j + 1];
            const int64_t nu = c1 > 0 ? st->offs[uoff(j + 1) + c1] : 0;
            if (nu > 0)
                hipLaunchKernelGGL(k_bupdate, dim3((unsigned)nu), dim3(256), 0, s, d_probs, d_order, d_offs + uoff(j + 1),
                                   c1, (int)j, 2, (int)j + 2, 0, C_pool, info);
            j += 2;
        } else {
            j += 1;  // the last tile column has nothing to its right
        }
        if (hipGetLastError() != hipSuccess) return GP_ERR_HIP;
    }
    hipLaunchKernelGGL(k_bsolve, dim3((unsigned)nb), dim3(256), 0, s, d_probs, C_pool, d_z, out3, info);
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
