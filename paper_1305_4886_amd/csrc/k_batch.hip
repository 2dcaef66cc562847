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
typedef double d2 __attribute__((ext_vector_type(2)));

namespace {

struct BProb {
    int64_t n, x_off, c_off, z_off, w_off;
    int64_t f_off, p_off;  // persistent launch: first tile flag, first per-tile partial pair
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

// ---------------------------------------------------------------------------
// Persistent dataflow variant: the whole batch in one launch.
//
// Task (p, i, k), i >= k, owns tile (i, k) of problem p.  It builds C_ik in
// registers (no covariance pass through memory), subtracts L_ij L_kj^T for
// j < k as those tiles become available (left-looking, the accumulator never
// leaves the registers), and then either factors and inverts the tile
// (i == k: L_kk, W_k = L_kk^{-1}, z_k = W_k (y_k - sum_j L_kj z_j) and the
// tile's log-determinant / quadratic-form partials) or forms L_ik = A_ik W_k^T
// once W_k is there.  The last diagonal task of a problem reduces its partials
// into (loglik, log|C|, q).
//
// Scheduling: the problems are spread over BQ task queues (one per XCD, by
// cost), each an ordered task list in which every task's inputs come earlier:
// tile column k of each of the queue's problems (largest first) before column
// k + 1, and within a problem's column the tiles below the diagonal top-down,
// with the next diagonal tile (k + 1, k + 1) right after (k + 1, k), its last
// input, so that it runs a column ahead of the tiles that wait for its
// inverse.  Workgroup w drains queue w mod BQ first (workgroups are dispatched
// to the XCDs round-robin, so a queue's problems share one L2), then takes
// from the other queues in turn.  A queue hands out its tasks in order
// through an atomic ticket, and a workgroup takes its next task while it
// works on the current one.  The launch always drains: of the tasks taken and
// not finished, the one taken first is being worked on (a prefetched task's
// holder took its current task earlier) and its inputs, taken earlier still
// from the same queue, are finished.
//
// Data that other workgroups read back (each L_ik in a tile-major copy, W_k,
// z_k, the partials) is written through to memory (agent-scope atomic
// stores), and a tile's flag is raised only after its publisher's stores have
// drained: 1 = ready, 2 = the problem failed (dependents skip their work and
// pass the 2 on).  The tile-major copy and W_k are then read with ordinary
// (cached, 16-byte) loads: each tile is written once per launch, occupies its
// own 32 KB, and is first read after its flag, so no XCD's caches can hold a
// line of it from before it was written (the caches start each launch clean
// of the previous one's data); z_k and the partials share cache lines across
// tiles and are read with agent-scope atomic loads.  Every wait
// is bounded: a stall raises the abort flag, every workgroup then leaves, and
// the problem that saw it reports info = -1 (its outputs stay NaN).
// ---------------------------------------------------------------------------
constexpr int BQ = 8;  // task queues
// flags: queue q's ticket at BF_TICKET + 32 q (own cache lines), the abort
// flag, then one flag per tile
constexpr int BF_TICKET = 0, BF_ABORT = 32 * BQ, BF_TILES = 32 * BQ + 32;

// Every buffer these touch is device memory: the global address space is
// stated, so that code the compiler cannot trace back to a kernel argument
// (the diagonal task's finish, a call of its own) still uses global rather
// than flat accesses, which would also count in lgkmcnt and make each LDS
// wait there wait for the stores in flight.
typedef __attribute__((address_space(1))) uint64_t gu64;
typedef __attribute__((address_space(1))) double gf64;
GP_DEV double bld(const double *p) {
    return __longlong_as_double(
        (long long)__hip_atomic_load((gu64 *)const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
GP_DEV void bst(double *p, double v) {
    __hip_atomic_store((gu64 *)p, (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
GP_DEV int bflag(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
GP_DEV int64_t tri64(int64_t r) { return r * (r + 1) / 2; }

struct alignas(16) PersistSmem {
    union {
        struct {  // operand ring: two stages of L_ij / L_kj (column-major, 16-byte aligned rows)
            double A[2][T][T + 2];
            double B[2][T][T + 2];
        } r;
        struct {  // diagonal task: the factor and its inverse
            double L[T][T + 1];
            double W[T][T + 1];
        } d;
    } u;
    union {
        double pn[T][17];
        double t32[32][33];
    } U;
    double rd[T];
    double zs[2][T];
    double tp[4][T];
    int64_t ticket;
    int ready, state;
};

// Wave 0 polls the flags of tile columns j .. j + 63 (those below k) of tile
// rows i and k until column j is published; returns the first column not yet
// published (the caller may take every column below it without waiting) and
// the state (1 ready, 2 the problem failed, 0 abort).  Block-uniform: every
// exit test of the poll loop is wave-uniform (ballots, readfirstlane).
template <typename SM>
GP_DEV void bensure(SM &sm, int *flags, const int *fl, int64_t ri_base, int64_t rk_base, int j, int k,
                    int &ready, int &state) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x, c = j + lane;
        const int cend = (k - j) < 64 ? k : j + 64;
        int r = cend, st = 1, spins = 0;
        for (;;) {
            int v = 1;
            if (c < cend) {
                const int a = bflag(fl + ri_base + c), d = bflag(fl + rk_base + c);
                v = (a == 0 || d == 0) ? 0 : ((a == 2 || d == 2) ? 2 : 1);
            }
            const uint64_t nr = __ballot(v == 0), fl2 = __ballot(v == 2);
            if (fl2) {
                st = 2;
                break;
            }
            r = nr ? j + (int)__builtin_ctzll(nr) : cend;
            if (r > j) break;
            if (__builtin_amdgcn_readfirstlane(bflag(flags + BF_ABORT))) {
                st = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            if (++spins > SPIN_LIMIT) {
                if (lane == 0) __hip_atomic_store(flags + BF_ABORT, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                st = 0;
                break;
            }
        }
        if (lane == 0) {
            sm.ready = r;
            sm.state = st;
        }
    }
    __syncthreads();
    ready = sm.ready;
    state = sm.state;
}

// Thread 0 waits for one flag; returns its value (1 / 2) or 0 on abort.  Block-uniform.
template <typename SM>
GP_DEV int bwait1(SM &sm, int *flags, const int *f) {
    if (threadIdx.x == 0) {
        int v, spins = 0;
        while ((v = bflag(f)) == 0) {
            if (bflag(flags + BF_ABORT)) break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins > SPIN_LIMIT) {
                __hip_atomic_store(flags + BF_ABORT, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        sm.state = v;
    }
    __syncthreads();
    return sm.state;
}

// Flags, info and outputs of a persistent launch to their initial state:
// flags (ticket, abort and one per tile) zero, info 0, out3 NaN (0 for an
// empty problem, whose log-likelihood is the empty sum).
__global__ __launch_bounds__(256) void k_binit(int *flags, int64_t nflags, const BProb *__restrict__ probs, int nb,
                                               double *out3, int32_t *info) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nflags; e += stride) flags[e] = 0;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += stride) {
        info[b] = 0;
        const double v = probs[b].n == 0 ? -0.0 : __builtin_nan("");
        out3[3 * b] = v;
        out3[3 * b + 1] = probs[b].n == 0 ? 0.0 : v;
        out3[3 * b + 2] = probs[b].n == 0 ? 0.0 : v;
    }
}

// tasks[t] = (problem, tile row | tile column << 16); queue q holds tasks
// qstart[q] .. qstart[q + 1] - 1.
__global__ __launch_bounds__(256, 1) void k_bpersist(const BProb *__restrict__ probs, const uint2 *__restrict__ tasks,
                                                     const int64_t *__restrict__ qstart, int dim,
                                                     const double *__restrict__ X,
                                                     const double *__restrict__ y, double *C_pool, double *lt,
                                                     double *wbuf, double *zbuf, double *part, int *flags,
                                                     double *out3, int32_t *info) {
    __shared__ PersistSmem sm;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w & 1, wn = w >> 1;
    const int64_t total = qstart[BQ];
    // thread 0: the queue it takes from and how many queues it has left behind
    int qx = blockIdx.x % BQ, qleft = 0;
    auto take = [&]() -> int64_t {
        while (qleft < BQ) {
            const int64_t a = atomicAdd(flags + BF_TICKET + 32 * qx, 1);
            if (a < qstart[qx + 1] - qstart[qx]) return qstart[qx] + a;
            qx = (qx + 1) % BQ;
            ++qleft;
        }
        return total;
    };
    if (tid == 0) sm.ticket = take();
    __syncthreads();
    int64_t t = sm.ticket;
    for (;; t = sm.ticket) {
        if (t >= total) break;
        const uint2 task = tasks[t];
        int64_t nxt = 0;  // thread 0: the next task, taken now and handed over at the end of this one
        if (tid == 0) nxt = take();
        const int b = (int)task.x, i = (int)(task.y & 0xffffu), k = (int)(task.y >> 16);
        const BProb P = probs[b];
        const bool diag = (i == k);
        const int64_t ld = P.n, i0 = (int64_t)i * T, k0 = (int64_t)k * T;
        const int ri = (int)((P.n - i0) < T ? (P.n - i0) : T), rk = (int)((P.n - k0) < T ? (P.n - k0) : T);
        double *L = C_pool + P.c_off;
        int *fl = flags + BF_TILES + P.f_off;  // flag of tile (r, c): fl[r (r + 1) / 2 + c]
        const int64_t fi = tri64(i), fk = tri64(k);
        const bool idle_wave = diag && wm == 0 && wn == 1;  // upper-right quarter of a diagonal tile: unused

        // 1. the covariance tile, in the D layout of v_mfma_f64_16x16x4.  For
        //    points in the plane the coordinates of this thread's 8 rows and
        //    2 columns are loaded first, before the operand tiles (the load
        //    counter drains in issue order), and the tile is built once the
        //    operand loads are on their way.
        v4d acc[2][2];
        const double *Xb = X + P.x_off * dim;
        double xr[8][2], xc[2][2];
        const bool planar = dim <= 2;
        if (planar) {
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wm * 32 + m * 16 + (lane >> 4) + 4 * r;
                    const double *p = Xb + (i0 + (row < ri ? row : 0)) * dim;
                    xr[4 * m + r][0] = p[0];
                    xr[4 * m + r][1] = dim == 2 ? p[1] : 0.0;
                }
#pragma unroll
            for (int qq = 0; qq < 2; ++qq) {
                const int col = wn * 32 + qq * 16 + (lane & 15);
                const double *p = Xb + (k0 + (col < rk ? col : 0)) * dim;
                xc[qq][0] = p[0];
                xc[qq][1] = dim == 2 ? p[1] : 0.0;
            }
        }
        auto gen_cov = [&]() {
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int qq = 0; qq < 2; ++qq)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wm * 32 + m * 16 + (lane >> 4) + 4 * r, col = wn * 32 + qq * 16 + (lane & 15);
                        double v = 0.0;
                        if (!idle_wave && row < ri && col < rk) {
                            const int64_t gi = i0 + row, gk = k0 + col;
                            double d;
                            if (planar) {
                                const double d0 = xr[4 * m + r][0] - xc[qq][0], d1 = xr[4 * m + r][1] - xc[qq][1];
                                d = sqrt(fma(d1, d1, d0 * d0));  // the rounding of point_dist
                            } else {
                                d = point_dist(Xb + gi * dim, Xb + gk * dim, dim);
                            }
                            v = P.s2 * cov_corr(P.kind, d * P.inv_rho) + (gi == gk ? P.t2 : 0.0);
                        }
                        acc[m][qq][r] = v;
                    }
        };
        // 2. A_ik -= sum_{j < k} L_ij L_kj^T, operands staged through registers
        //    (next column's loads in flight during this column's products)
        int ready = 0, state = 1;
        double tpart = 0.0;  // diagonal task: this wave's share of (sum_j L_kj z_j)[lane]
        if (k > 0) {
            // element pairs (rows 2 rp, 2 rp + 1 of column c) of the tile-major
            // copies of L_ij and L_kj (rows past the problem are stored as zeros)
            d2 va[(T * T) / 512], vb[(T * T) / 512];
            double zv = 0.0;
            auto stage = [&](int buf) {  // registers -> LDS stage buf
#pragma unroll
                for (int r = 0; r < (T * T) / 512; ++r) {
                    const int e = r * 256 + tid, rp = e & 31, kk = e >> 5;
                    *reinterpret_cast<d2 *>(&sm.u.r.A[buf][kk][2 * rp]) = va[r];
                    if (!diag) *reinterpret_cast<d2 *>(&sm.u.r.B[buf][kk][2 * rp]) = vb[r];
                }
                if (diag && tid < T) sm.zs[buf][tid] = zv;
            };
            bensure(sm, flags, fl, fi, fk, 0, k, ready, state);
            if (state == 1) {
                const d2 *Ai = reinterpret_cast<const d2 *>(lt + (P.f_off + fi) * (T * T));
                const d2 *Bk = reinterpret_cast<const d2 *>(lt + (P.f_off + fk) * (T * T));
#pragma unroll
                for (int r = 0; r < (T * T) / 512; ++r) {
                    va[r] = Ai[r * 256 + tid];
                    if (!diag) vb[r] = Bk[r * 256 + tid];
                }
                if (diag && tid < T) zv = bld(zbuf + P.z_off + tid);
            }
            gen_cov();  // overlaps the first operand loads
            if (state == 1) stage(0);
            __syncthreads();
            // One barrier per column: stage j & 1 is read while the registers
            // take column j + 1, which then goes to the other stage (last read
            // in column j - 1, before the previous barrier).
            for (int j = 0; j < k && state == 1; ++j) {
                const int cb = j & 1;
                const bool more = j + 1 < k;
                if (more) {
                    if (j + 1 >= ready) bensure(sm, flags, fl, fi, fk, j + 1, k, ready, state);
                    if (state != 1) break;
                }
                // The next column's loads go out one per step of the products
                // (a burst of them would hold up the matrix instructions); at the
                // last column the current tiles are fetched again (cached, unused).
                const int jn = more ? j + 1 : j;
                const d2 *An = reinterpret_cast<const d2 *>(lt + (P.f_off + fi + jn) * (T * T));
                const d2 *Bn = reinterpret_cast<const d2 *>(lt + (P.f_off + fk + jn) * (T * T));
                double(*Ao)[T + 2] = sm.u.r.A[cb];
                double(*Bo)[T + 2] = diag ? sm.u.r.A[cb] : sm.u.r.B[cb];
                double a[2], bb[2];
                if (!idle_wave) {
#pragma unroll
                    for (int m = 0; m < 2; ++m) a[m] = -Ao[lane >> 4][wm * 32 + m * 16 + (lane & 15)];
#pragma unroll
                    for (int qq = 0; qq < 2; ++qq) bb[qq] = Bo[lane >> 4][wn * 32 + qq * 16 + (lane & 15)];
                }
#pragma unroll
                for (int st = 0; st < T / 4; ++st) {
                    if (!idle_wave) {
                        // operands of the next step first: their LDS latency hides under these products
                        double an[2], bn[2];
                        if (st + 1 < T / 4) {
                            const int kn = 4 * (st + 1) + (lane >> 4);
#pragma unroll
                            for (int m = 0; m < 2; ++m) an[m] = -Ao[kn][wm * 32 + m * 16 + (lane & 15)];
#pragma unroll
                            for (int qq = 0; qq < 2; ++qq) bn[qq] = Bo[kn][wn * 32 + qq * 16 + (lane & 15)];
                        }
#pragma unroll
                        for (int m = 0; m < 2; ++m)
#pragma unroll
                            for (int qq = 0; qq < 2; ++qq)
                                acc[m][qq] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], bb[qq], acc[m][qq], 0, 0, 0);
                        if (st + 1 < T / 4) {
                            a[0] = an[0];
                            a[1] = an[1];
                            bb[0] = bn[0];
                            bb[1] = bn[1];
                        }
                    }
                    if ((st & 1) == 0) va[st >> 1] = An[(st >> 1) * 256 + tid];
                    else if (!diag) vb[st >> 1] = Bn[(st >> 1) * 256 + tid];
                    __builtin_amdgcn_sched_barrier(0);
                }
                if (diag) {
                    if (more && tid < T) zv = bld(zbuf + P.z_off + (int64_t)jn * T + tid);
#pragma unroll
                    for (int c = 16 * w; c < 16 * w + 16; ++c) tpart = fma(Ao[c][lane], sm.zs[cb][c], tpart);
                }
                if (more) stage(cb ^ 1);
                __syncthreads();
            }
        } else {
            gen_cov();
        }
        if (state == 0) {  // stalled: leave (the abort flag stops every workgroup)
            if (tid == 0) info[b] = -1;
            return;
        }

        if (!diag) {
            // 3a. L_ik = A_ik W_k^T once the diagonal task of column k has published W_k
            if (state == 1) state = bwait1(sm, flags, fl + fk + k);
            if (state == 0) {
                if (tid == 0) info[b] = -1;
                return;
            }
            if (state == 1) {
                // W_k's loads first, so their latency overlaps moving A_ik to LDS
                const d2 *Wk = reinterpret_cast<const d2 *>(wbuf + P.w_off + k0 * T);
                d2 wv[(T * T) / 512];
#pragma unroll
                for (int r = 0; r < (T * T) / 512; ++r) wv[r] = Wk[r * 256 + tid];
                __syncthreads();
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int qq = 0; qq < 2; ++qq)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = wm * 32 + m * 16 + (lane >> 4) + 4 * r, col = wn * 32 + qq * 16 + (lane & 15);
                            sm.u.r.A[0][col][row] = acc[m][qq][r];
                        }
#pragma unroll
                for (int r = 0; r < (T * T) / 512; ++r) {
                    const int e = r * 256 + tid, rp = e & 31, kk = e >> 5;
                    *reinterpret_cast<d2 *>(&sm.u.r.B[0][kk][2 * rp]) = wv[r];
                }
                __syncthreads();
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int qq = 0; qq < 2; ++qq) acc[m][qq] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
                for (int kk = 0; kk < T; kk += 4) {
                    double a[2], bb[2];
#pragma unroll
                    for (int m = 0; m < 2; ++m) a[m] = sm.u.r.A[0][kk + (lane >> 4)][wm * 32 + m * 16 + (lane & 15)];
#pragma unroll
                    for (int qq = 0; qq < 2; ++qq) bb[qq] = sm.u.r.B[0][kk + (lane >> 4)][wn * 32 + qq * 16 + (lane & 15)];
#pragma unroll
                    for (int m = 0; m < 2; ++m)
#pragma unroll
                        for (int qq = 0; qq < 2; ++qq)
                            acc[m][qq] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], bb[qq], acc[m][qq], 0, 0, 0);
                }
                __syncthreads();  // As / Bs reads of the product are done
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int qq = 0; qq < 2; ++qq)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = wm * 32 + m * 16 + (lane >> 4) + 4 * r, col = wn * 32 + qq * 16 + (lane & 15);
                            sm.u.r.A[0][col][row] = acc[m][qq][r];
                        }
                __syncthreads();
                double *Lik = L + i0 + k0 * ld;
                double *Lt = lt + (P.f_off + fi + k) * (T * T);
#pragma unroll
                for (int r = 0; r < (T * T) / 512; ++r) {
                    const int e = r * 256 + tid, rp = e & 31, c = e >> 5;
                    const double v0 = sm.u.r.A[0][c][2 * rp], v1 = sm.u.r.A[0][c][2 * rp + 1];
                    bst(Lt + 2 * rp + c * T, v0);
                    bst(Lt + 2 * rp + 1 + c * T, v1);
                    if (2 * rp < ri) Lik[2 * rp + (int64_t)c * ld] = v0;
                    if (2 * rp + 1 < ri) Lik[2 * rp + 1 + (int64_t)c * ld] = v1;
                }
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            if (tid == 0) {
                __hip_atomic_store(fl + fi + k, state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sm.ticket = bflag(flags + BF_ABORT) ? total : nxt;
            }
            __syncthreads();
            continue;
        }

        // 3b. diagonal tile: factor, invert, forward-solve block k, partials
        if (state == 1) {
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int qq = 0; qq < 2; ++qq)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wm * 32 + m * 16 + (lane >> 4) + 4 * r, col = wn * 32 + qq * 16 + (lane & 15);
                        if (!idle_wave) sm.u.d.L[row][col] = acc[m][qq][r];
                    }
            sm.tp[w][lane] = tpart;
            __syncthreads();
            if (w == 0) {
                double a[T];
#pragma unroll
                for (int c = 0; c < T; ++c) {
                    double v;
                    if (lane < rk && c < rk) v = (c <= lane) ? sm.u.d.L[lane][c] : 0.0;
                    else v = (lane == c) ? 1.0 : 0.0;  // identity padding decouples unused rows
                    a[c] = v;
                }
                const int fail = wave_chol64(a, lane, sm.u.d.W, sm.U.pn);
                if (fail) {
                    if (lane == 0) {
                        info[b] = (int32_t)(k0 + fail);
                        sm.state = 2;
                    }
                } else {
                    double *Lkk = L + k0 + k0 * ld;
#pragma unroll
                    for (int c = 0; c < T; ++c) {
                        sm.u.d.L[lane][c] = a[c];
                        if (lane < rk && c < rk && c <= lane) Lkk[lane + (int64_t)c * ld] = a[c];
                    }
                    wave_lds_sync();
                    wave_inv64_blocked(sm.u.d.L, sm.u.d.W, sm.U.t32, sm.rd, lane);
                    double *Wk = wbuf + P.w_off + k0 * T;
#pragma unroll 4
                    for (int c = 0; c < T; ++c) bst(Wk + lane + c * T, sm.u.d.W[lane][c]);
                    const double tsum = (sm.tp[0][lane] + sm.tp[1][lane]) + (sm.tp[2][lane] + sm.tp[3][lane]);
                    sm.zs[0][lane] = lane < rk ? y[P.x_off + k0 + lane] - tsum : 0.0;
                    wave_lds_sync();
                    double zr = 0.0;
#pragma unroll 8
                    for (int c = 0; c < T; ++c) zr = fma(sm.u.d.W[lane][c], sm.zs[0][c], zr);
                    if (lane < rk) bst(zbuf + P.z_off + k0 + lane, zr);
                    sm.tp[0][lane] = lane < rk ? log(sm.u.d.L[lane][lane]) : 0.0;
                    sm.tp[1][lane] = lane < rk ? zr * zr : 0.0;
                    wave_lds_sync();
                    if (lane == 0) {
                        CSum sl, sq;
                        for (int c = 0; c < T; ++c) {
                            sl.add(sm.tp[0][c]);
                            sq.add(sm.tp[1][c]);
                        }
                        bst(part + P.p_off + 2 * k, sl.value());
                        bst(part + P.p_off + 2 * k + 1, sq.value());
                        sm.state = 1;
                    }
                }
            }
            __syncthreads();
            state = sm.state;
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) {
            __hip_atomic_store(fl + fk + k, state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (k == P.nt - 1) {  // the last diagonal tile: every partial of the problem is published
                double *o = out3 + 3 * (int64_t)b;
                if (state == 1) {
                    CSum sl, sq;
                    for (int j = 0; j < P.nt; ++j) {
                        sl.add(bld(part + P.p_off + 2 * j));
                        sq.add(bld(part + P.p_off + 2 * j + 1));
                    }
                    const double logdet = 2.0 * sl.value(), qf = sq.value();
                    o[1] = logdet;
                    o[2] = qf;
                    o[0] = -0.5 * (((double)P.n * 1.8378770664093453 + logdet) + qf);
                }  // failed: the NaNs written at the start stay
            }
            sm.ticket = bflag(flags + BF_ABORT) ? total : nxt;
        }
        __syncthreads();
    }
}


// ---------------------------------------------------------------------------
// Persistent dataflow launch on 128 x 128 tiles.
//
// The task graph, queues, flags and publication rules of k_bpersist, with
// tiles twice as wide: one left-looking step moves two 128 KB operand tiles
// for 4.2 MFLOP (16 flop per byte against 8 with 64 x 64 tiles).  A
// workgroup has NW waves (eight by default: two per SIMD).  Task (p, i, k)
// first accumulates S = sum_{j<k} L_kj L_ij^T, 128 rows m (tile k) by 128
// columns r (tile i), each wave holding 128 / NW columns of every row; the
// operands arrive as K-slabs of 16 columns of the tiles' tile-major copies,
// copied straight into a four-stage LDS ring (three slabs in flight).  It
// then builds the covariance tile in the idle ring and forms
// G = A_ik^T = C_ki - S.  An off-diagonal task forms L_ik^T = W_k G on the
// matrix cores, taking G as the B operand straight from its accumulators:
// the D layout of v_mfma_f64_16x16x4 (lane l, register r: row l / 16 + 4 r,
// column l % 16) is the B layout of the K-step over rows 4 r .. 4 r + 3; it
// also publishes L_ik z_k for the diagonal task of row i.  A diagonal task
// (diag128_finish) factors its tile in LDS as a 2 x 2 matrix of 64 x 64
// blocks -- L11 and W11 = L11^{-1} by one wave, L21 = A21 W11^T and
// A22 - L21 L21^T on the matrix cores, L22 and W22 by one wave,
// W21 = -W22 (L21 W11) -- then forms z_k = W_k (y_k - sum_j L_kj z_j) and
// the tile's log-determinant / quadratic-form partials.
// ---------------------------------------------------------------------------
// K-slabs of BK2 columns through an NST-stage ring (NST - 1 slabs in flight);
// SPT slabs per 128-column step.  32-column slabs in two stages (half the
// barriers, one slab in flight) measured 1 % slower.
constexpr int T2 = 128, BK2 = 16, NST = 2048 / BK2 / 32, SPT = T2 / BK2;
static_assert(NST >= 2 && NST * BK2 == 64, "the ring holds 64 columns of both operands (128 KB)");
constexpr int BP_NW = 8;  // waves per workgroup of the 128-tile launch (two per SIMD)

struct alignas(16) P128Smem {
    union {
        double ring[NST][2][BK2][T2];  // [stage][operand: 0 = L_kj, 1 = L_ij][column][row]
        double Wt[T2][T2 + 2];       // off-diagonal task: W_k as [c][m] (row c at 1040 bytes: no bank conflicts)
        struct {                     // diagonal task: 64 x 64 blocks
            double B11[DB][DB + 1], B21[DB][DB + 1], B22[DB][DB + 1], Wb[DB][DB + 1];
        } d;
    } u;
    union {
        double pn[DB][17];
        double t32[32][33];
    } U;
    double px[2][T2][2];  // planar points: rows m (tile k), columns r (tile i)
    double rd[DB];
    double zk[T2];        // off-diagonal task: z_k
    double ys[T2];        // y_k - sum_j L_kj z_j
    double lg[T2];        // log L_mm
    double zq[T2];        // z_m^2
    int64_t ticket;
    int ready, state;
};

__shared__ P128Smem bp_sm;  // the 128-tile launch's LDS (shared with its diagonal-task finish)

template <typename Tp>
GP_DEV Tp *uni_ptr(Tp *p) {  // a pointer the compiler cannot prove wave-uniform, in scalar registers
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (Tp *)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

// x[mi][ni] += sum_{m < 64} A(32 wr + 16 mi + i, m) B(m, 32 wc + 16 ni + j) for
// one wave's 32 x 32 block of a 64 x 64 product, operands through callables.
template <typename FA, typename FB>
GP_DEV void blk32_mm(v4d (&x)[2][2], FA fa, FB fb, int wr, int wc, int lane) {
#pragma unroll 4
    for (int kk = 0; kk < DB; kk += 4) {
        double a[2], bb[2];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) a[mi] = fa(32 * wr + 16 * mi + (lane & 15), kk + (lane >> 4));
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) bb[ni] = fb(kk + (lane >> 4), 32 * wc + 16 * ni + (lane & 15));
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int ni = 0; ni < 2; ++ni)
                x[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mi], bb[ni], x[mi][ni], 0, 0, 0);
    }
}

// Element (row, column) of register r in block (mi, ni) of blk32_mm's result.
GP_DEV int blk_row(int wr, int mi, int lane, int r) { return 32 * wr + 16 * mi + (lane >> 4) + 4 * r; }
GP_DEV int blk_col(int wc, int ni, int lane) { return 32 * wc + 16 * ni + (lane & 15); }

// The diagonal task's finish, called once per diagonal tile with the tile G
// in the LDS blocks B11 / B21 / B22: y_k - sum_j L_kj z_j, the 2 x 2 block
// factorisation and inverse, W_k, z_k and the partials.  A call of its own
// (not inlined) so that its one-wave register factorisation is allocated
// apart from the accumulators and ring addresses of the persistent loop.
// Returns the tile's state (1 done, 2 not positive definite).
template <int NW>
__device__ __attribute__((noinline)) int diag128_finish(const BProb *__restrict__ probs, int b, int k, double *C_pool,
                                                        const double *__restrict__ y, double *wbuf, double *zbuf,
                                                        double *part, double *pbuf, int32_t *info) {
    constexpr int NT = 64 * NW;
    P128Smem &sm = bp_sm;
    auto &D = sm.u.d;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const BProb P = probs[b];
    const int64_t ld = P.n, k0 = (int64_t)k * T2, fk = tri64(k);
    const int rk = (int)((P.n - k0) < T2 ? (P.n - k0) : T2);
    double *L = C_pool + P.c_off;
    int state = 1;
    if (tid == 0) sm.state = 1;
    if (tid < T2) {  // y_k - sum_j L_kj z_j, the products published by the tasks (k, j)
        const double *pk = pbuf + (P.f_off + fk) * T2 + tid;
        double tsum = 0.0;
        int j = 0;
        for (; j + 8 <= k; j += 8) {  // eight loads in flight, summed in order
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = bld(pk + (int64_t)(j + u) * T2);
#pragma unroll
            for (int u = 0; u < 8; ++u) tsum += v[u];
        }
        for (; j < k; ++j) tsum += bld(pk + (int64_t)j * T2);
        sm.ys[tid] = tid < rk ? y[P.x_off + k0 + tid] - tsum : 0.0;
    }
    __syncthreads();
    double *Lkk = L + k0 + k0 * ld;
    const int wr = w & 1, wc = w >> 1;
    v4d x[2][2];
    // the two diagonal blocks in turn, through one copy of the
    // one-wave factor / inverse code: half 0 factors A11 into B11 and
    // inverts it into Wb; then L21 and A22 - L21 L21^T; half 1 factors
    // that into B22 and inverts it into B11 (L11 is stored by then)
#pragma nounroll
    for (int hb = 0; hb < 2 && state == 1; ++hb) {
        double(*Bd)[DB + 1] = hb ? D.B22 : D.B11;
        double(*Wo)[DB + 1] = hb ? D.B11 : D.Wb;
        const int o = 64 * hb;
        if (w == 0) {
            double a[DB];
#pragma unroll
            for (int c = 0; c < DB; ++c) a[c] = (c <= lane) ? Bd[lane][c] : 0.0;
            const int fail = wave_chol64(a, lane, Wo, sm.U.pn);
            if (fail) {
                if (lane == 0) {
                    info[b] = (int32_t)(k0 + o + fail);
                    sm.state = 2;
                }
            } else {
#pragma unroll
                for (int c = 0; c < DB; ++c) Bd[lane][c] = a[c];
                wave_lds_sync();
                sm.lg[o + lane] = Bd[lane][lane];  // its log is taken off the chain, below
                wave_inv64_blocked(Bd, Wo, sm.U.t32, sm.rd, lane);
            }
        }
        __syncthreads();
        state = sm.state;
        if (state == 1) {  // the factored block out of LDS by every wave (off the one-wave chain)
            gf64 *Lg = (gf64 *)Lkk;
            for (int e = tid; e < DB * DB; e += NT) {
                const int r = e & (DB - 1), c = e >> 6;
                if (c <= r && o + r < rk && o + c < rk) Lg[(o + r) + (int64_t)(o + c) * ld] = Bd[r][c];
            }
        }
        if (hb == 1 || state != 1) break;
        // L21 = A21 W11^T
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) x[mi][ni] = v4d{0.0, 0.0, 0.0, 0.0};
        if (w < 4)
            blk32_mm(x, [&](int r, int m) { return D.B21[r][m]; }, [&](int m, int c) { return D.Wb[c][m]; },
                     wr, wc, lane);
        __syncthreads();
        if (w < 4) {
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int rr = blk_row(wr, mi, lane, r), c = blk_col(wc, ni, lane);
                        D.B21[rr][c] = x[mi][ni][r];
                        if (64 + rr < rk && c < rk) ((gf64 *)Lkk)[(64 + rr) + (int64_t)c * ld] = x[mi][ni][r];
                    }
        }
        __syncthreads();
        if (w < 4 && wr >= wc) {  // A22 -= L21 L21^T, lower blocks
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        x[mi][ni][r] = D.B22[blk_row(wr, mi, lane, r)][blk_col(wc, ni, lane)];
            blk32_mm(x, [&](int r, int m) { return -D.B21[r][m]; }, [&](int m, int c) { return D.B21[c][m]; },
                     wr, wc, lane);
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        D.B22[blk_row(wr, mi, lane, r)][blk_col(wc, ni, lane)] = x[mi][ni][r];
        }
        __syncthreads();
    }
    if (state == 1) {  // W21 = -W22 (L21 W11): X = L21 W11 into B21, then W21 into B21
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) x[mi][ni] = v4d{0.0, 0.0, 0.0, 0.0};
        if (w < 4)
            blk32_mm(x, [&](int r, int m) { return D.B21[r][m]; }, [&](int m, int c) { return D.Wb[m][c]; },
                     wr, wc, lane);
        __syncthreads();
        if (w < 4) {
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        D.B21[blk_row(wr, mi, lane, r)][blk_col(wc, ni, lane)] = x[mi][ni][r];
        }
        __syncthreads();
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) x[mi][ni] = v4d{0.0, 0.0, 0.0, 0.0};
        if (w < 4)
            blk32_mm(x, [&](int r, int m) { return -D.B11[r][m]; }, [&](int m, int c) { return D.B21[m][c]; },
                     wr, wc, lane);
        __syncthreads();
        if (w < 4) {
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        D.B21[blk_row(wr, mi, lane, r)][blk_col(wc, ni, lane)] = x[mi][ni][r];
        }
        __syncthreads();
        // W_k = [[W11, 0], [W21, W22]] out, row-major (c, m) at c 128 + m
        double *Wk = wbuf + P.w_off + k0 * T2;
        for (int e = tid; e < T2 * T2; e += NT) {
            const int m = e & (T2 - 1), c = e >> 7;
            const double v = c < 64 ? (m < 64 ? D.Wb[c][m] : 0.0) : (m < 64 ? D.B21[c - 64][m] : D.B11[c - 64][m - 64]);
            bst(Wk + e, v);
        }
        // z_k = W_k (y_k - sum_j L_kj z_j); thread c < 128
        if (tid < T2) {
            const int c = tid;
            double zr = 0.0;
            if (c < 64) {
#pragma unroll 8
                for (int m = 0; m < 64; ++m) zr = fma(D.Wb[c][m], sm.ys[m], zr);
            } else {
#pragma unroll 8
                for (int m = 0; m < 64; ++m) zr = fma(D.B21[c - 64][m], sm.ys[m], zr);
#pragma unroll 8
                for (int m = 0; m < 64; ++m) zr = fma(D.B11[c - 64][m], sm.ys[64 + m], zr);
            }
            if (c < rk) bst(zbuf + P.z_off + k0 + c, zr);
            sm.zq[c] = c < rk ? zr * zr : 0.0;
            sm.lg[c] = c < rk ? log(sm.lg[c]) : 0.0;
        }
        __syncthreads();
        if (tid == 0 || tid == 64) {  // the two partials, one wave each
            const double *v = tid == 0 ? sm.lg : sm.zq;
            CSum acc_s;
            for (int c = 0; c < T2; ++c) acc_s.add(v[c]);
            bst(part + P.p_off + 2 * k + (tid == 0 ? 0 : 1), acc_s.value());
        }
    }
    return state;
}

template <int NW>
__global__ __launch_bounds__(64 * NW, 1) void k_bp128(const BProb *__restrict__ probs, const uint2 *__restrict__ tasks,
                                                  const int64_t *__restrict__ qstart, int dim,
                                                  const double *__restrict__ X, const double *__restrict__ y,
                                                  double *C_pool, double *lt, double *wbuf, double *zbuf, double *part,
                                                  double *pbuf, int *flags, double *out3, int32_t *info) {
    constexpr int NT = 64 * NW, RB = 8 / NW, CW = 16 * RB;  // threads, 16-column blocks and columns per wave
    P128Smem &sm = bp_sm;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t total = qstart[BQ];
    int qx = blockIdx.x % BQ, qleft = 0;
    auto take = [&]() -> int64_t {
        while (qleft < BQ) {
            const int64_t a = atomicAdd(flags + BF_TICKET + 32 * qx, 1);
            if (a < qstart[qx + 1] - qstart[qx]) return qstart[qx] + a;
            qx = (qx + 1) % BQ;
            ++qleft;
        }
        return total;
    };
    if (tid == 0) sm.ticket = take();
    __syncthreads();
    for (int64_t t = sm.ticket; t < total; t = sm.ticket) {
        const uint2 task = tasks[t];
        int64_t nxt = 0;  // thread 0: the next task, taken now and handed over at the end of this one
        if (tid == 0) nxt = take();
        const int b = __builtin_amdgcn_readfirstlane((int)task.x);
        const int i = __builtin_amdgcn_readfirstlane((int)(task.y & 0xffffu));
        const int k = __builtin_amdgcn_readfirstlane((int)(task.y >> 16));
        const BProb P = probs[b];
        const bool diag = (i == k);
        const int64_t ld = P.n, i0 = (int64_t)i * T2, k0 = (int64_t)k * T2;
        const int ri = (int)((P.n - i0) < T2 ? (P.n - i0) : T2), rk = (int)((P.n - k0) < T2 ? (P.n - k0) : T2);
        double *L = C_pool + P.c_off;
        int *fl = flags + BF_TILES + P.f_off;  // flag of tile (r, c): fl[r (r + 1) / 2 + c]
        const int64_t fi = tri64(i), fk = tri64(k);
        const double *Xb = X + P.x_off * dim;
        const bool planar = dim <= 2;

        // 1. points of the two tiles to LDS (planar), then the first slab's
        //    copies, then the covariance tile while they fly
        if (planar && tid < 2 * T2) {
            const int q = tid >> 7, e = tid & 127, cnt = q ? ri : rk;
            const double *p = Xb + ((q ? i0 : k0) + (e < cnt ? e : 0)) * dim;
            sm.px[q][e][0] = p[0];
            sm.px[q][e][1] = dim == 2 ? p[1] : 0.0;
        }
        if (tid == 0) sm.state = 1;
        __syncthreads();
        int ready = 0, state = 1;
        const int nsl = SPT * k;  // K-slabs of the left-looking update (SPT per tile column j < k)
        const double *LK = uni_ptr(lt + (P.f_off + fk) * (T2 * T2));  // tile (k, 0); (k, j) at + j T2^2
        const double *LI = uni_ptr(lt + (P.f_off + fi) * (T2 * T2));
        // copy c of this wave for slab s into stage st: column w + NW q of the
        // slab, operand op (c = 2 q + op; a diagonal task copies L_kj only, c = q)
        const int per = diag ? BK2 / NW : 2 * BK2 / NW;  // copies per wave and slab
        auto copy_slot = [&](int s, int st, int c) {
            const int q = diag ? c : (c >> 1), op = diag ? 0 : (c & 1);
            const int tt = w + NW * q;
            const int64_t col = (int64_t)(s / SPT) * T2 * T2 + (int64_t)(BK2 * (s % SPT) + tt) * T2;
            lds_dma_dwordx4(uni_ptr((op ? LI : LK) + col), 16u * lane,
                            __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)&sm.u.ring[st][op][tt][0]));
        };
        if (nsl > 0) {
            bensure(sm, flags, fl, fi, fk, 0, k, ready, state);
            if (state == 1) {
#pragma nounroll
                for (int s0 = 0; s0 < NST - 1 && s0 < nsl; ++s0) {
#pragma nounroll
                    for (int c = 0; c < per; ++c) copy_slot(s0, s0, c);
                }
            }
        }
        v4d acc[8][RB];  // sum_j L_kj L_ij^T, then C_ki minus that: G
#pragma unroll
        for (int mb = 0; mb < 8; ++mb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[mb][rb] = v4d{0.0, 0.0, 0.0, 0.0};

        // 2. sum_j L_kj L_ij^T over the slabs through the NST-stage ring: the
        //    copies of slab s + NST - 1 go out between the matrix instructions of
        //    slab s.  The ring's waits and barriers are explicit (vmcnt counts
        //    the copies; a __syncthreads would drain every copy in flight).
        for (int s = 0; s < nsl && state == 1; ++s) {
            const int st = s % NST, sn = s + NST - 1;
            const bool more = sn < nsl;
            if (more && sn / SPT >= ready) {
                bensure(sm, flags, fl, fi, fk, sn / SPT, k, ready, state);
                if (state != 1) {
                    wait_vmcnt<0>();  // no copy may land in LDS after this task
                    continue;         // (the loop condition ends the loop)
                }
            }
            // slabs after s already in flight
            const int later = nsl - 1 - s < NST - 2 ? nsl - 1 - s : NST - 2;
            if (diag)
                wait_slabs<BK2 / NW, NST - 2>(later);
            else
                wait_slabs<2 * BK2 / NW, NST - 2>(later);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();  // slab s is in stage st; stage (s - 1) % NST was last read in slab s - 1
            asm volatile("" ::: "memory");
            const double(*Rk)[T2] = sm.u.ring[st][0];
            const double(*Ri)[T2] = sm.u.ring[st][diag ? 0 : 1];
            double a[8], bb[RB];
#pragma unroll
            for (int mb = 0; mb < 8; ++mb) a[mb] = Rk[lane >> 4][16 * mb + (lane & 15)];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) bb[rb] = Ri[lane >> 4][CW * w + 16 * rb + (lane & 15)];
#pragma unroll
            for (int kk = 0; kk < BK2 / 4; ++kk) {
                double an[8], bn[RB];
                if (kk + 1 < BK2 / 4) {
                    const int kn = 4 * (kk + 1) + (lane >> 4);
#pragma unroll
                    for (int mb = 0; mb < 8; ++mb) an[mb] = Rk[kn][16 * mb + (lane & 15)];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) bn[rb] = Ri[kn][CW * w + 16 * rb + (lane & 15)];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int g = 0; g < 2; ++g) {
#pragma unroll
                    for (int mb = 4 * g; mb < 4 * g + 4; ++mb)
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb)
                            acc[mb][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mb], bb[rb], acc[mb][rb], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    // BK2 / 2 slots per slab, the copies spread over them
                    constexpr int NSLOT = BK2 / 2;
                    const int sl = 2 * kk + g;
                    if (more && (sl * per) / NSLOT != ((sl + 1) * per) / NSLOT)
                        copy_slot(sn, sn % NST, (sl * per) / NSLOT);
                    __builtin_amdgcn_sched_barrier(0);
                }
                if (kk + 1 < BK2 / 4) {
#pragma unroll
                    for (int mb = 0; mb < 8; ++mb) a[mb] = an[mb];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) bb[rb] = bn[rb];
                }
            }
        }
        // 3. the covariance tile, in two halves of 64 rows computed into the
        //    (now idle) ring, minus the accumulated products: G[m][c] = C(k0 + m,
        //    i0 + c), identity on the padded diagonal of a diagonal tile
        if (state == 1) {
            double(*GT)[T2] = reinterpret_cast<double(*)[T2]>(&sm.u.ring[0][0][0][0]);
            __syncthreads();  // every wave is past its ring reads
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
#pragma nounroll
                for (int e = tid; e < 64 * T2; e += NT) {
                    const int ml = e >> 7, c = e & (T2 - 1), m = 64 * hh + ml;
                    double v = 0.0;
                    if (m < rk && c < ri) {
                        const int64_t gm = k0 + m, gc = i0 + c;
                        double d;
                        if (planar) {
                            const double d0 = sm.px[1][c][0] - sm.px[0][m][0], d1 = sm.px[1][c][1] - sm.px[0][m][1];
                            d = sqrt(fma(d1, d1, d0 * d0));  // the rounding of point_dist
                        } else {
                            d = point_dist(Xb + gc * dim, Xb + gm * dim, dim);
                        }
                        v = P.s2 * cov_corr(P.kind, d * P.inv_rho) + (gm == gc ? P.t2 : 0.0);
                    } else if (diag && m == c) {
                        v = 1.0;  // identity padding decouples the rows past the problem
                    }
                    GT[ml][c] = v;
                }
                __syncthreads();
#pragma unroll
                for (int mb = 4 * hh; mb < 4 * hh + 4; ++mb)
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            acc[mb][rb][r] = GT[16 * (mb - 4 * hh) + (lane >> 4) + 4 * r][CW * w + 16 * rb + (lane & 15)] - acc[mb][rb][r];
                __syncthreads();
            }
        }
        if (state == 0) {  // stalled: leave (the abort flag stops every workgroup)
            if (tid == 0) info[b] = -1;
            return;
        }

        if (!diag) {
            // 3a. L_ik^T = W_k G once the diagonal task of column k has published W_k
            if (state == 1) state = bwait1(sm, flags, fl + fk + k);
            if (state == 0) {
                if (tid == 0) info[b] = -1;
                return;
            }
            if (state == 1) {
                __syncthreads();  // every wave is past its ring reads
                const double *Wk = uni_ptr(wbuf + P.w_off + k0 * T2);  // row-major: (c, m) at c T2 + m
#pragma nounroll
                for (int q = 0; q < T2 / NW; ++q) {
                    const int c = w + NW * q;
                    lds_dma_dwordx4(uni_ptr(Wk + (int64_t)c * T2), 16u * lane,
                                    __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)&sm.u.Wt[c][0]));
                }
                if (tid < T2) sm.zk[tid] = tid < rk ? bld(zbuf + P.z_off + k0 + tid) : 0.0;
                wait_vmcnt<0>();
                __syncthreads();
                // Four quarters of 32 output rows c: W_k is lower triangular, so
                // block (cb, mb) is zero for mb > cb.  A quarter's result goes to
                // the LDS rows of W_k it has just finished reading, then out as
                // whole 1 KB columns of L_ik (and its tile-major copy).
                double *Lt = lt + (P.f_off + fi + k) * (T2 * T2);
                double pz = 0.0;  // thread rr < 128: (L_ik z_k)(rr)
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    v4d o[2][RB];
#pragma unroll
                    for (int cq = 0; cq < 2; ++cq)
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb) o[cq][rb] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int mb = 0; mb < 2 * h + 2; ++mb)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int m = 16 * mb + 4 * r + (lane >> 4);
#pragma unroll
                            for (int cq = 0; cq < 2; ++cq) {
                                const int cb = 2 * h + cq;
                                if (mb > cb) continue;
                                const double wv = sm.u.Wt[16 * cb + (lane & 15)][m];
#pragma unroll
                                for (int rb = 0; rb < RB; ++rb)
                                    o[cq][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(wv, acc[mb][rb][r], o[cq][rb], 0,
                                                                                     0, 0);
                            }
                        }
                    __syncthreads();  // rows 32 h .. 32 h + 31 of W_k are read by every wave
#pragma unroll
                    for (int cq = 0; cq < 2; ++cq)
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                            for (int r = 0; r < 4; ++r)  // L_ik(rr, c) at row c
                                sm.u.Wt[16 * (2 * h + cq) + (lane >> 4) + 4 * r][CW * w + 16 * rb + (lane & 15)] =
                                    o[cq][rb][r];
                    __syncthreads();
#pragma nounroll
                    for (int e = tid; e < 32 * T2; e += NT) {
                        const int c = 32 * h + (e >> 7), rr = e & (T2 - 1);
                        const double v = sm.u.Wt[c][rr];
                        bst(Lt + rr + (int64_t)c * T2, v);
                        if (rr < ri && c < rk) L[(i0 + rr) + (k0 + c) * ld] = v;
                    }
                    if (tid < T2) {
#pragma unroll 8
                        for (int c = 32 * h; c < 32 * h + 32; ++c) pz = fma(sm.u.Wt[c][tid], sm.zk[c], pz);
                    }
                }
                // L_ik z_k (the diagonal task of tile row i sums these over k, in order)
                if (tid < T2) bst(pbuf + (P.f_off + fi + k) * T2 + tid, pz);
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            if (tid == 0) {
                __hip_atomic_store(fl + fi + k, state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sm.ticket = bflag(flags + BF_ABORT) ? total : nxt;
            }
            __syncthreads();
            continue;
        }

        // 3b. diagonal tile: factor, invert, forward-solve block k, partials
        if (state == 1) {
            __syncthreads();  // every wave is past its ring reads
            auto &D = sm.u.d;
#pragma unroll
            for (int mb = 0; mb < 8; ++mb)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int m = 16 * mb + (lane >> 4) + 4 * r, c = CW * w + 16 * rb + (lane & 15);
                        if (CW * w + 16 * rb < 64) {
                            if (mb < 4) D.B11[m][c] = acc[mb][rb][r];
                            else D.B21[m - 64][c] = acc[mb][rb][r];
                        } else if (mb >= 4) {
                            D.B22[m - 64][c - 64] = acc[mb][rb][r];
                        }
                    }
            state = diag128_finish<NW>(probs, b, k, C_pool, y, wbuf, zbuf, part, pbuf, info);
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) {
            __hip_atomic_store(fl + fk + k, state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (k == P.nt - 1) {  // the last diagonal tile: every partial of the problem is published
                double *o = out3 + 3 * (int64_t)b;
                if (state == 1) {
                    CSum sl, sq;
                    for (int j = 0; j < P.nt; ++j) {
                        sl.add(bld(part + P.p_off + 2 * j));
                        sq.add(bld(part + P.p_off + 2 * j + 1));
                    }
                    const double logdet = 2.0 * sl.value(), qf = sq.value();
                    o[1] = logdet;
                    o[2] = qf;
                    o[0] = -0.5 * (((double)P.n * 1.8378770664093453 + logdet) + qf);
                }  // failed: the NaNs written at the start stay
            }
            sm.ticket = bflag(flags + BF_ABORT) ? total : nxt;
        }
        __syncthreads();
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

size_t batch_ws_bytes(int64_t nmax, int64_t nbatch, bool persistent, int tile) {
    const int TT = persistent ? tile : T;  // the level-synchronous launches use 64 x 64 tiles
    const int64_t nt = (nmax + TT - 1) / TT;
    size_t b = 0;
    b += al256b(sizeof(BProb) * (size_t)nbatch);
    b += al256b(sizeof(int32_t) * (size_t)nbatch);                              // size order
    b += al256b(sizeof(int64_t) * (size_t)(2 * nt + 1) * (size_t)(nbatch + 1));  // per-level prefix counts
    b += al256b(sizeof(double) * (size_t)nmax * (size_t)nbatch);                 // z
    b += al256b(sizeof(double) * (size_t)nt * TT * TT * (size_t)nbatch);         // diagonal inverses
    b += al256b(sizeof(int) * ((size_t)BF_TILES + (size_t)(nt * (nt + 1) / 2) * (size_t)nbatch));  // tile flags
    b += al256b(sizeof(double) * 2 * (size_t)nt * (size_t)nbatch);               // per-tile partials
    b += al256b(8 * (size_t)(nt * (nt + 1) / 2) * (size_t)nbatch + 8 * (BQ + 1));  // task list, queue starts
    if (persistent) {  // tile-major copy of the factor's tiles, read back inside the launch, and L_ik z_k
        b += al256b(sizeof(double) * TT * TT * (size_t)(nt * (nt + 1) / 2) * (size_t)nbatch);
        b += al256b(sizeof(double) * TT * (size_t)(nt * (nt + 1) / 2) * (size_t)nbatch);
    }
    return b + 256;
}

struct BatchStaging {
    std::vector<BProb> probs;
    std::vector<int32_t> order;
    std::vector<int64_t> offs;  // [level block][nb + 1]: covariance, then per level panel and update counts
    void *pinned = nullptr;  // persistent launch: task list + queue starts (pinned host memory)
    size_t pinned_bytes = 0;
    hipEvent_t done = nullptr;
};

int batch_run(hipStream_t s, int num_cu, int grid, int tile, void *&staging_ptr, int32_t nb, const gp_theta_t *th,
              const int64_t *nh, const int64_t *xoff, const int64_t *coff, int32_t dim, const double *X,
              const double *y, double *C_pool, double *out3, int32_t *info, void *ws, size_t ws_bytes) {
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
    if (grid >= 0 && tile != T && tile != T2) return GP_ERR_NOT_SUPPORTED;
    const int TT = grid >= 0 ? tile : T;  // tile edge of this call
    if (ws_bytes < batch_ws_bytes(nmax, nb, grid >= 0, TT)) return GP_ERR_WS_TOO_SMALL;
    const int64_t ntmax = (nmax + TT - 1) / TT;
    st->probs.assign(nb, BProb{});
    int64_t zoff = 0, woff = 0, foff = 0, poff_ = 0;
    for (int b = 0; b < nb; ++b) {
        BProb &p = st->probs[b];
        p.n = nh[b];
        p.x_off = xoff[b];
        p.c_off = coff[b];
        p.nt = (int32_t)((p.n + TT - 1) / TT);
        p.z_off = zoff;
        zoff += p.n;
        p.w_off = woff;
        woff += (int64_t)p.nt * TT * TT;
        p.f_off = foff;
        foff += (int64_t)p.nt * (p.nt + 1) / 2;
        p.p_off = poff_;
        poff_ += 2 * (int64_t)p.nt;
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
    double *d_w = reinterpret_cast<double *>(take(sizeof(double) * (size_t)ntmax * TT * TT * (size_t)nb));

    if (grid >= 0) {
        // Persistent launch.  Problems go to the BQ queues largest first, each
        // to the queue with the least work so far (nt^3); a queue's task list
        // is, per tile column k and problem (largest first): for k = 0 the
        // tile (0, 0), then (1, 0), (1, 1), (2, 0), (3, 0), ...; for
        // 1 <= k <= nt - 2: (k + 1, k), (k + 1, k + 1), (k + 2, k), ....
        std::vector<int> qof(nb, 0);
        double qload[BQ] = {0.0};
        for (int q = 0; q < nb; ++q) {
            const int b = st->order[q];
            int x = 0;
            for (int c = 1; c < BQ; ++c)
                if (qload[c] < qload[x]) x = c;
            qof[b] = x;
            const double c3 = (double)st->probs[b].nt;
            qload[x] += c3 * c3 * c3;
            if (st->probs[b].nt >= 65536) return -4;  // tile indices are packed in 16 bits
        }
        const int64_t total = foff;  // one task per tile of the lower triangles
        const size_t tbytes = sizeof(uint2) * (size_t)(total > 0 ? total : 1), qbytes = sizeof(int64_t) * (BQ + 1);
        if (st->pinned_bytes < tbytes + qbytes) {
            if (st->pinned) (void)hipHostFree(st->pinned);
            st->pinned = nullptr;
            st->pinned_bytes = 0;
            if (hipHostMalloc(&st->pinned, tbytes + qbytes) != hipSuccess) return GP_ERR_HIP;
            st->pinned_bytes = tbytes + qbytes;
        }
        uint2 *tl = static_cast<uint2 *>(st->pinned);
        int64_t *qs = reinterpret_cast<int64_t *>(static_cast<char *>(st->pinned) + tbytes);
        int64_t nt_ = 0;
        auto emit = [&](int b, int64_t ti, int64_t tk) { tl[nt_++] = make_uint2((unsigned)b, (unsigned)(ti | (tk << 16))); };
        for (int x = 0; x < BQ; ++x) {
            qs[x] = nt_;
            int64_t ncol = 0;
            for (int q = 0; q < nb; ++q)
                if (qof[st->order[q]] == x) ncol = std::max<int64_t>(ncol, st->probs[st->order[q]].nt);
            for (int64_t k = 0; k < ncol; ++k)
                for (int q = 0; q < nb; ++q) {
                    const int b = st->order[q];
                    const int64_t ntq = st->probs[b].nt;
                    if (qof[b] != x || ntq == 0) continue;
                    if (k == 0) {
                        emit(b, 0, 0);
                        if (ntq >= 2) {
                            emit(b, 1, 0);
                            emit(b, 1, 1);
                        }
                        for (int64_t r = 2; r < ntq; ++r) emit(b, r, 0);
                    } else if (k <= ntq - 2) {
                        emit(b, k + 1, k);
                        emit(b, k + 1, k + 1);
                        for (int64_t r = k + 2; r < ntq; ++r) emit(b, r, k);
                    }
                }
        }
        qs[BQ] = nt_;
        if (nt_ != total) return GP_ERR_HIP;  // internal consistency
        const int64_t nflags = BF_TILES + foff;
        int *d_flags = reinterpret_cast<int *>(take(sizeof(int) * (size_t)nflags));
        double *d_part = reinterpret_cast<double *>(take(sizeof(double) * (size_t)(poff_ > 0 ? poff_ : 1)));
        uint2 *d_tasks = reinterpret_cast<uint2 *>(take(tbytes));
        int64_t *d_qs = reinterpret_cast<int64_t *>(take(qbytes));
        double *d_lt = reinterpret_cast<double *>(take(sizeof(double) * TT * TT * (size_t)(foff > 0 ? foff : 1)));
        double *d_pz = reinterpret_cast<double *>(take(sizeof(double) * TT * (size_t)(foff > 0 ? foff : 1)));
        if (off > ws_bytes) return GP_ERR_WS_TOO_SMALL;
        if (hipMemcpyAsync(d_probs, st->probs.data(), sizeof(BProb) * (size_t)nb, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(d_tasks, tl, tbytes, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(d_qs, qs, qbytes, hipMemcpyHostToDevice, s) != hipSuccess)
            return GP_ERR_HIP;
        if (hipEventRecord(st->done, s) != hipSuccess) return GP_ERR_HIP;
        const int64_t init_blocks = std::min<int64_t>(1024, std::max<int64_t>(nflags, nb) / 256 + 1);
        hipLaunchKernelGGL(k_binit, dim3((unsigned)init_blocks), dim3(256), 0, s, d_flags, nflags, d_probs, nb, out3,
                           info);
        if (total > 0) {
            int64_t g = grid > 0 ? grid : (int64_t)(num_cu > 0 ? num_cu : 1);
            if (g > total) g = total;
            if (TT == T2)
                hipLaunchKernelGGL(k_bp128<BP_NW>, dim3((unsigned)g), dim3(64 * BP_NW), 0, s, d_probs, d_tasks, d_qs, (int)dim, X, y,
                                   C_pool, d_lt, d_w, d_z, d_part, d_pz, d_flags, out3, info);
            else
                hipLaunchKernelGGL(k_bpersist, dim3((unsigned)g), dim3(256), 0, s, d_probs, d_tasks, d_qs, (int)dim, X,
                                   y, C_pool, d_lt, d_w, d_z, d_part, d_flags, out3, info);
        }
        return hipGetLastError() == hipSuccess ? GP_OK : GP_ERR_HIP;
    }

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
    if (st->pinned) (void)hipHostFree(st->pinned);
    delete st;
}
