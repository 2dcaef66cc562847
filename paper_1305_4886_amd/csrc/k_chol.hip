// k_chol.hip -- latency-critical pieces of the blocked Cholesky and the solves.
//
//  * k_diag_potrf: factors one 64 x 64 diagonal block in LDS (right-looking,
//    column by column: pivot, scale, rank-1 update) and forms its inverse,
//    which the panel solve then applies on the matrix cores.  This is the
//    "Cholesky decomposition of the diagonal block" step on the critical path
//    of Section 2.1 / Fig. 1; a non-positive pivot stops the factorisation
//    and records the 1-based column (no pivoting -- Section 5).
//  * k_diag_inv: the same inverse for every diagonal block of a given L.
//  * k_trsv2_fwd / k_trsv2_trans (k_trsv_fwd / k_trsv_trans for n <= 128):
//    single-kernel blocked triangular solves (forward L^{-1} b and backward
//    L^{-T} b -- Section 1's backsolve and the remoteForwardsolve /
//    remoteBacksolve of Section 2.3.2).  Each workgroup owns one 128-row
//    (64-row) block; it takes a ticket from an atomic counter (so the blocks
//    it depends on belong to workgroups already running), accumulates the
//    off-diagonal products as soon as each dependency's values are published
//    in the mailbox, applies the block's inverse and publishes its own
//    values.  L is read once, 64 contiguous doubles per load.
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

// ---------------------------------------------------------------------------
// k_panel_chol: the K x K diagonal block of one panel (K <= 64 PF_MAXB) in a
// single launch of NB = ceil(K / 64) workgroups that run concurrently and
// hand 64 x 64 blocks to each other through memory, instead of a chain of
// ~4 launches per 64 columns (factor, solve, update) plus the launches of
// the blocked inverse -- every one of which waits for a free slot behind the
// trailing update and pays a dispatch latency on the critical path.
//
// Phase 1 (workgroup b owns block row b; right-looking by block columns k):
//   when L_kk and W_k = L_kk^{-1} are published:
//     L_bk = S_bk W_k^T, published;  S_bj -= L_bk L_jk^T for k < j <= b
//     (L_jk from workgroup j as soon as it is published; S_bb is kept in
//     registers, S_bk is read before W_k is waited for);
//   after the last column: L_bb = chol(S_bb) and W_b (one wave, as in
//   k_diag_potrf), published.  Critical path per 64 columns: two 64^3
//   products, the 64 x 64 factor and inverse, and one flag round trip.
// Phase 2 (only when the rows below the panel follow, K % 64 == 0;
// workgroup b owns block column b of W = L^{-1}):
//   W_bb = W_b;  for k = b, b + 1, ...: T_sb += L_sk W_kb for s > k (in the
//   W buffer), then W_{k+1,b} = -W_{k+1} T_{k+1,b}.
//
// Every block another workgroup reads is written and read with relaxed
// agent-scope atomic accesses (coherent across XCDs, no cache-wide fence);
// a publisher waits for its stores (vmcnt 0, barrier) before it raises the
// block's flag.  Waits are bounded: on a timeout or a failed pivot the abort
// flag stops every workgroup.  Outputs: L in place, W_b into dinv (column-
// major 64 x 64 per block), W (ld ldw, zeros above the diagonal) if non-null.
// ---------------------------------------------------------------------------
constexpr int PF_ABORT = PF_MAXB * PF_MAXB;

GP_DEV double ld_coh(const double *p) {
    return __longlong_as_double((long long)__hip_atomic_load(
        reinterpret_cast<uint64_t *>(const_cast<double *>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
GP_DEV void st_coh(double *p, double v) {
    __hip_atomic_store(reinterpret_cast<uint64_t *>(p), (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// A bounded wait that gave up (timeout, or another workgroup's abort) turns
// info 0 into -1; a pivot failure already recorded (a positive column) stays.
GP_DEV void note_giveup(int32_t *info) {
    if (info) atomicCAS(info, 0, -1);
}

// Thread 0 waits for flags[idx] (bounded); every thread gets the outcome.  The
// abort flag is read beside the flag on every poll and takes precedence, so
// once it is raised every later wait gives up at once.  A give-up is recorded
// in info (note_giveup).
GP_DEV bool pf_wait(int *flags, int idx, int *s_ok, int32_t *info) {
    if (threadIdx.x == 0) {
        int ok = 1, spins = 0;
        for (;;) {
            const int f = __hip_atomic_load(&flags[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int ab = __hip_atomic_load(&flags[PF_ABORT], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ab) {
                ok = 0;
                break;
            }
            if (f) break;
            __builtin_amdgcn_s_sleep(2);
            if (++spins > SPIN_LIMIT) {
                __hip_atomic_store(&flags[PF_ABORT], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        if (!ok) note_giveup(info);
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// All of this workgroup's stores done, then flags[idx] = 1.
GP_DEV void pf_publish(int *flags, int idx) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&flags[idx], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// dst[r][c] = M[r + c ld] (T: dst[c][r] = M[r + c ld]) for r < rows, c < cols; 0 elsewhere.
template <bool T>
GP_DEV void pf_load(double (*dst)[DB + 1], const double *M, int64_t ld, int rows, int cols) {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = threadIdx.x + 256 * q, r = e & (DB - 1), c = e >> 6;
        v[q] = (r < rows && c < cols) ? ld_coh(M + r + (int64_t)c * ld) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = threadIdx.x + 256 * q, r = e & (DB - 1), c = e >> 6;
        if (T)
            dst[c][r] = v[q];
        else
            dst[r][c] = v[q];
    }
}

// The wave's A operand of a 64 x 64 x 64 product, X(row, m) for row = 16 w +
// lane % 16, m = 4 q + lane / 16 (q < 16): from LDS (Xs[row][m]) or from
// memory (Xg[row + m ldx]; rows >= xrows read row xrows - 1 and give zero).
GP_DEV void pf_xload(const double (*Xs)[DB + 1], const double *Xg, int64_t ldx, int xrows, double (&a)[16], int w,
                     int lane) {
    const int row = 16 * w + (lane & 15);
    if (Xs) {
#pragma unroll
        for (int q = 0; q < 16; ++q) a[q] = Xs[row][4 * q + (lane >> 4)];
    } else {
        const int rr = row < xrows ? row : xrows - 1;
#pragma unroll
        for (int q = 0; q < 16; ++q) a[q] = ld_coh(Xg + rr + (int64_t)(4 * q + (lane >> 4)) * ldx);
#pragma unroll
        for (int q = 0; q < 16; ++q) a[q] = row < xrows ? a[q] : 0.0;
    }
}

// acc[n][i] (+)= sum_m X(row, m) Y[col][m] over m < 64 with X from pf_xload,
// wave w: row = 16 w + lane / 16 + 4 i, col = 16 n + lane % 16 (the D layout
// of v_mfma_f64_16x16x4).  With accumulate, acc holds the addend on entry.
GP_DEV void pf_mm(const double (&a)[16], const double (*Y)[DB + 1], gp_v4d (&acc)[4], int lane,
                  bool accumulate = false) {
    if (!accumulate) {
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[n] = gp_v4d{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
    for (int q = 0; q < 16; ++q)
#pragma unroll
        for (int n = 0; n < 4; ++n)
            acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], Y[16 * n + (lane & 15)][4 * q + (lane >> 4)], acc[n], 0,
                                                          0, 0);
}

GP_DEV void pf_gemm(const double (*Xs)[DB + 1], const double *Xg, int64_t ldx, int xrows, const double (*Y)[DB + 1],
                    gp_v4d (&acc)[4], int w, int lane) {
    double a[16];
    pf_xload(Xs, Xg, ldx, xrows, a, w, lane);
    pf_mm(a, Y, acc, lane);
}

// M(row, col) += sgn acc for the wave's rows < rows and cols < cols (and col <= row
// if lower); loads first, then stores.
GP_DEV void pf_accum(double *M, int64_t ld, const gp_v4d (&acc)[4], double sgn, int rows, int cols, bool lower, int w,
                     int lane) {
    double v[16];
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * w + (lane >> 4) + 4 * i, c = 16 * n + (lane & 15);
            const bool ok = r < rows && c < cols && (!lower || c <= r);
            v[4 * n + i] = ok ? ld_coh(M + r + (int64_t)c * ld) : 0.0;
        }
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * w + (lane >> 4) + 4 * i, c = 16 * n + (lane & 15);
            const bool ok = r < rows && c < cols && (!lower || c <= r);
            if (ok) st_coh(M + r + (int64_t)c * ld, fma(sgn, acc[n][i], v[4 * n + i]));
        }
}

// With factor == 0 the block is already factored (L, and its 64 x 64 block
// inverses in dinv): only phase 2 runs, with nothing to wait for.  Launch
// dimension y batches independent blocks at strides sA (A), sD (dinv), sW (W)
// and sF (flags).
__global__ __launch_bounds__(256, 1) void k_panel_chol(double *A, int64_t lda, int K, double *dinv, double *W,
                                                       int64_t ldw, int *flags, int32_t *info, int64_t col0,
                                                       int factor, int64_t sA, int64_t sD, int64_t sW, int64_t sF) {
    // 74 KB, so that a workgroup fits beside one workgroup of the trailing
    // update; for the same reason its registers (VGPRs rounded to 8, plus
    // AGPRs) must stay within 288, the 512 of a SIMD less that workgroup's
    // two waves of 112
    __shared__ union {
        struct {
            double op[DB][DB + 1];  // B operand of the current product
            double lb[DB][DB + 1];  // L_bk of the current column (phase 1), W_kb^T (phase 2)
        } g;
        struct {
            double ls[DB][DB + 1];  // factor workspace, then L_bb
            double wl[DB][DB + 1];  // W_b
            union {
                double pn[DB][17];
                double t32[32][33];
            } u;
            double rd[DB];
        } d;
    } sm;
    __shared__ int s_ok;
    if (info && *info) return;
    A += (int64_t)blockIdx.y * sA;
    dinv += (int64_t)blockIdx.y * sD;
    if (W) W += (int64_t)blockIdx.y * sW;
    flags += (int64_t)blockIdx.y * sF;
    const int nb = (K + DB - 1) / DB;
    const int b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int rb = K - DB * b < DB ? K - DB * b : DB;  // rows (and columns) of block b
    double *Ab = A + DB * b;                           // block row b: Ab[r + c lda]
    double *Wc = W ? W + (int64_t)DB * b * ldw : nullptr;  // block column b of W: Wc[r + c ldw], r < K
    gp_v4d acc[4];
    // the rest of W's block column b first: zeros above the diagonal block and
    // T_sb = 0 below it (the stores drain while phase 1 waits)
    if (W) {
        for (int e = tid; e < DB * DB; e += 256) {
            const int r = e & (DB - 1), c = e >> 6;
            for (int s2 = 0; s2 < b; ++s2) Wc[DB * s2 + r + (int64_t)c * ldw] = 0.0;
            for (int s2 = b + 1; s2 < nb; ++s2) st_coh(Wc + DB * s2 + r + (int64_t)c * ldw, 0.0);
        }
    }

    // ---- phase 1 ----
    // S_bb stays in registers (the D layout of pf_mm) while the steps k < b
    // subtract L_bk L_bk^T from it; the other blocks of block row b are
    // updated in memory.
    gp_v4d sbb[4];
    if (factor) {
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * w + (lane >> 4) + 4 * i, c = 16 * n + (lane & 15);
                sbb[n][i] = ld_coh(Ab + (r < rb ? r : rb - 1) + (int64_t)(DB * b + (c < rb ? c : rb - 1)) * lda);
            }
    }
    for (int k = 0; factor && k < b; ++k) {
        double xa[16];  // S_bk: final once this workgroup's own updates of it are complete
        pf_xload(nullptr, Ab + (int64_t)DB * k * lda, lda, rb, xa, w, lane);
        if (!pf_wait(flags, k * PF_MAXB + k, &s_ok, info)) return;
        pf_load<false>(sm.g.op, dinv + (int64_t)k * DB * DB, DB, DB, DB);  // W_k
        __syncthreads();
        pf_mm(xa, sm.g.op, acc, lane);  // L_bk = S_bk W_k^T
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * w + (lane >> 4) + 4 * i, c = 16 * n + (lane & 15);
                sm.g.lb[r][c] = acc[n][i];
                if (r < rb) st_coh(Ab + r + (int64_t)(DB * k + c) * lda, acc[n][i]);
            }
        pf_publish(flags, b * PF_MAXB + k);  // its barrier also orders the lb writes
        {  // S_bb -= L_bk L_bk^T
            double nl[16];
            pf_xload(sm.g.lb, nullptr, 0, 0, nl, w, lane);
#pragma unroll
            for (int q = 0; q < 16; ++q) nl[q] = -nl[q];
            pf_mm(nl, sm.g.lb, sbb, lane, true);
        }
        for (int j = k + 1; j < b; ++j) {  // S_bj -= L_bk L_jk^T
            if (!pf_wait(flags, j * PF_MAXB + k, &s_ok, info)) return;
            pf_load<false>(sm.g.op, A + DB * j + (int64_t)DB * k * lda, lda, DB, DB);  // L_jk
            __syncthreads();
            pf_gemm(sm.g.lb, nullptr, 0, 0, sm.g.op, acc, w, lane);
            pf_accum(Ab + (int64_t)DB * j * lda, lda, acc, -1.0, rb, DB, false, w, lane);
            __syncthreads();  // op is reloaded next
        }
        // the S_bj stores complete before any of them is read back (by other
        // lanes of the same wave, at later steps); lb and op are rewritten next
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    }
    // diagonal block: one wave factors and inverts it (or, when it is
    // factored already, W_b is read back).  The four waves stage the updated
    // S_bb from their registers in LDS first (lower triangle; rows and
    // columns past the block replaced by the identity).
    double *D = Ab + (int64_t)DB * b * lda;
    if (factor) {
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * w + (lane >> 4) + 4 * i, c = 16 * n + (lane & 15);
                sm.d.ls[r][c] = (r < rb && c < rb) ? (c <= r ? sbb[n][i] : 0.0) : (r == c ? 1.0 : 0.0);
            }
        __syncthreads();
    }
    if (!factor) {
        for (int e = tid; e < DB * DB; e += 256) sm.d.wl[e & (DB - 1)][e >> 6] = dinv[(int64_t)b * DB * DB + e];
        if (tid == 0) s_ok = 1;
    } else if (w == 0) {
        double a[DB];
#pragma unroll
        for (int c = 0; c < DB; ++c) a[c] = sm.d.ls[lane][c];
        wave_lds_sync();
        const int fail = wave_chol64(a, lane, sm.d.ls, sm.d.u.pn);
        if (fail) {
            if (lane == 0) {
                __hip_atomic_store(info, (int32_t)(col0 + DB * b + fail), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&flags[PF_ABORT], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_ok = 0;
            }
        } else {
            if (lane == 0) s_ok = 1;
#pragma unroll
            for (int c = 0; c < DB; ++c) sm.d.ls[lane][c] = a[c];
            wave_lds_sync();
            wave_inv64_blocked(sm.d.ls, sm.d.wl, sm.d.u.t32, sm.d.rd, lane);
        }
    }
    __syncthreads();
    if (!s_ok) return;
    if (factor) {  // L_bb (lower triangle) and W_b out of LDS, 16 columns per wave
        double *Wb = dinv + (int64_t)b * DB * DB;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = 16 * w + q;
            if (lane < rb && c < rb && c <= lane) st_coh(D + lane + (int64_t)c * lda, sm.d.ls[lane][c]);
            st_coh(Wb + lane + c * DB, sm.d.wl[lane][c]);
        }
    }
    // phase 2 starts from W_b, written into its block column of W before the
    // publication, while it is still in LDS
    if (W) {
        for (int e = tid; e < DB * DB; e += 256) {
            const int r = e & (DB - 1), c = e >> 6;
            st_coh(Wc + DB * b + r + (int64_t)c * ldw, sm.d.wl[r][c]);  // W_bb
        }
    }
    pf_publish(flags, b * PF_MAXB + b);
    if (!W) return;

    // ---- phase 2: block column b of W = L^{-1} ----
    for (int k = b; k + 1 < nb; ++k) {
        pf_load<true>(sm.g.lb, Wc + DB * k, ldw, DB, DB);  // lb[c][m] = W_kb(m, c)
        __syncthreads();
        for (int s2 = k + 1; s2 < nb; ++s2) {
            if (factor && !pf_wait(flags, s2 * PF_MAXB + k, &s_ok, info)) return;
            pf_gemm(nullptr, A + DB * s2 + (int64_t)DB * k * lda, lda, DB, sm.g.lb, acc, w, lane);  // L_sk W_kb
            pf_accum(Wc + DB * s2, ldw, acc, 1.0, DB, DB, false, w, lane);                       // T_sb +=
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();  // T stores complete
        // W_{k+1} is published by workgroup k + 1; in inverse-only mode it is
        // an input (dinv) and this workgroup reads only its own blocks of W
        if (factor && !pf_wait(flags, (k + 1) * PF_MAXB + (k + 1), &s_ok, info)) return;
        pf_load<true>(sm.g.op, Wc + DB * (k + 1), ldw, DB, DB);  // op[c][m] = T(m, c)
        __syncthreads();
        pf_gemm(nullptr, dinv + (int64_t)(k + 1) * DB * DB, DB, DB, sm.g.op, acc, w, lane);  // W_{k+1} T
        double *Wk = Wc + DB * (k + 1);
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                st_coh(Wk + (16 * w + (lane >> 4) + 4 * i) + (int64_t)(16 * n + (lane & 15)) * ldw, -acc[n][i]);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();  // W_{k+1,b} complete before it is read as the next W_kb; lb and op free
    }
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

// Two doubles at 8-byte alignment (a column-major operand with odd leading
// dimension), read as one 16-byte load.
typedef double gp_d2u __attribute__((ext_vector_type(2), aligned(8)));

// Cross-lane reduction step: lanes l and l ^ H exchange the halves of p[0..2H)
// they do not keep.  After the steps H = 16, 8, 4, 2, 1 on 32 register values,
// lane l holds the sum of p[l % 32] over the 32 lanes of its half-wave.
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

// Work area of the solves: ints [0] ticket, [1] abort, then (at byte 256) a
// mailbox of one double per row.  A solved value is published by storing it
// into its mailbox slot, which holds a signalling-NaN sentinel until then;
// a reader polls the slots it needs (relaxed agent-scope atomics, which the
// hardware keeps coherent across XCDs), so each value carries its own ready
// signal and no flag or cache-wide fence sits on the dependency chain.
constexpr uint64_t MBOX_EMPTY = 0x7FF4DEADBEEF0000ull;

// The abort flag is read on every 32nd empty poll only: each read is a
// round trip to memory, and reading it on every iteration would double the
// time between two looks at the slot.
GP_DEV double mbox_poll(const double *slot, int *abortf) {
    const uint64_t *p = reinterpret_cast<const uint64_t *>(slot);
    uint64_t v;
    int spins = 0;
    while ((v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == MBOX_EMPTY) {
        if ((++spins & 31) == 0) {
            if (__hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (spins > SPIN_LIMIT) {
                __hip_atomic_store(abortf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return __longlong_as_double((long long)v);
}

GP_DEV void mbox_put(double *slot, double v) {
    __hip_atomic_store(reinterpret_cast<uint64_t *>(slot), (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Forward solve, block blk (rows i0 .. i0 + 63):
//   x_blk = Winv_blk (b_blk - sum_{j < blk} L[blk, j] x_j).
// Each workgroup takes a ticket (so the blocks it depends on belong to
// workgroups already running).  Waves 1-3 take the far blocks j < blk - 1
// (lane = row, 512-byte column loads, x_j broadcast by readlane) as their
// values appear; wave 0 has the nearest block's 64 x 64 tile and the rows of
// Winv in registers, so once the far sums are in, the critical path is one
// poll of x_{blk-1}, two 64-term dot products per lane and the store.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_trsv_fwd(const double *L, int64_t ldl, double *x, int64_t n,
                                                  const double *dinv, int *sync, double *mbox,
                                                  const int32_t *info) {
    __shared__ int s_blk;
    __shared__ double part[3][DB];
    __shared__ double Ws[DB][DB + 1];
    if (info && *info) return;
    const int nblk = (int)((n + DB - 1) / DB);
    if (threadIdx.x == 0) s_blk = atomicAdd(&sync[0], 1);
    __syncthreads();
    const int blk = s_blk;
    if (blk >= nblk) return;
    int *abortf = &sync[1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i0 = (int64_t)blk * DB;
    const int64_t i = i0 + lane;
    const bool rv = i < n;
    if (w > 0) {
        double acc = 0.0;
        for (int jb = w - 1; jb < blk - 1; jb += 3) {
            const double *Lc = L + i + (int64_t)jb * DB * ldl;
            const double xv = mbox_poll(&mbox[(int64_t)jb * DB + lane], abortf);
            if (rv) {  // all 64 loads of the tile in flight before the first product
                double v[DB];
#pragma unroll
                for (int c = 0; c < DB; ++c) v[c] = Lc[(int64_t)c * ldl];
                double a1 = 0.0;
#pragma unroll
                for (int c = 0; c < DB; c += 2) {
                    acc = fma(v[c], rdlane(xv, c), acc);
                    a1 = fma(v[c + 1], rdlane(xv, c + 1), a1);
                }
                acc += a1;
            }
        }
        part[w - 1][lane] = acc;
        __syncthreads();
        return;
    }
    const double *W = dinv + (int64_t)blk * DB * DB;
#pragma unroll 8
    for (int c = 0; c < DB; ++c) Ws[lane][c] = W[lane + c * DB];  // Ws[a][b] = Winv(a, b)
    double lnear[DB];
#pragma unroll
    for (int c = 0; c < DB; ++c)
        lnear[c] = (rv && blk >= 1) ? L[i + ((int64_t)(blk - 1) * DB + c) * ldl] : 0.0;
    const double b = rv ? x[i] : 0.0;
    __syncthreads();
    double rhs = b - ((part[0][lane] + part[1][lane]) + part[2][lane]);
    if (blk >= 1) {
        const double xv = mbox_poll(&mbox[(int64_t)(blk - 1) * DB + lane], abortf);
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int c = 0; c < DB; c += 2) {
            a0 = fma(lnear[c], rdlane(xv, c), a0);
            a1 = fma(lnear[c + 1], rdlane(xv, c + 1), a1);
        }
        rhs -= a0 + a1;
    }
    double z0 = 0.0, z1 = 0.0;
#pragma unroll
    for (int c = 0; c < DB; c += 2) {
        z0 = fma(Ws[lane][c], rdlane(rhs, c), z0);
        z1 = fma(Ws[lane][c + 1], rdlane(rhs, c + 1), z1);
    }
    const double z = z0 + z1;
    if (rv) {
        x[i] = z;
        mbox_put(&mbox[i], z);
    }
}

// Backward solve x <- L^{-T} x, block blk (columns c0 .. c0 + 63 of L):
//   x_blk = Winv_blk^T (b_blk - sum_{j > blk} L[j, blk]^T x_j).
// Waves 1-3: far row blocks j > blk + 1, last first (their completion order).
// Lane (h, r) with h = lane / 32, r = lane % 32 reads rows 2r, 2r + 1 of block
// j in columns 2q + h (q = 0..31) as 16-byte loads, so one instruction covers
// two full 512-byte column segments and all 32 loads of a tile are in flight
// before the products; 32 column partial sums per lane, one cross-lane
// exchange over each half-wave at the end.  Wave 0 (lane = column) keeps its
// column of the nearest row block and of Winv in registers.
__global__ __launch_bounds__(256) void k_trsv_trans(const double *L, int64_t ldl, double *x, int64_t n,
                                                    const double *dinv, int *sync, double *mbox,
                                                    const int32_t *info) {
    __shared__ int s_t;
    __shared__ double part[3][DB];
    __shared__ double Ws[DB][DB + 1];
    if (info && *info) return;
    const int nblk = (int)((n + DB - 1) / DB);
    if (threadIdx.x == 0) s_t = atomicAdd(&sync[0], 1);
    __syncthreads();
    const int tk = s_t;
    if (tk >= nblk) return;
    const int blk = nblk - 1 - tk;
    int *abortf = &sync[1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t c0 = (int64_t)blk * DB;
    const int64_t col = c0 + lane;
    const bool cv = col < n;
    if (w > 0) {
        // far blocks exist only when blk + 2 < nblk, so this block's 64
        // columns are all < n; only the last row block can be partial
        const int hh = lane >> 5, r2 = lane & 31;
        double p[DB / 2];
#pragma unroll
        for (int q = 0; q < DB / 2; ++q) p[q] = 0.0;
        for (int jb = nblk - w; jb >= blk + 2; jb -= 3) {
            const int64_t row = (int64_t)jb * DB + 2 * r2;
            const double *Lr = L + row + (c0 + hh) * ldl;
            if (row + 1 < n) {
                const double x0 = mbox_poll(&mbox[row], abortf);
                const double x1 = mbox_poll(&mbox[row + 1], abortf);
                gp_d2u v[DB / 2];
#pragma unroll
                for (int q = 0; q < DB / 2; ++q) v[q] = *reinterpret_cast<const gp_d2u *>(Lr + (int64_t)(2 * q) * ldl);
#pragma unroll
                for (int q = 0; q < DB / 2; ++q) p[q] = fma(v[q].y, x1, fma(v[q].x, x0, p[q]));
            } else if (row < n) {
                const double x0 = mbox_poll(&mbox[row], abortf);
#pragma unroll
                for (int q = 0; q < DB / 2; ++q) p[q] = fma(Lr[(int64_t)(2 * q) * ldl], x0, p[q]);
            }
        }
        // lane (h, r) ends with the half-wave sum of p[r]: column 2 r + h
        xr_step<16>(p, lane);
        xr_step<8>(p, lane);
        xr_step<4>(p, lane);
        xr_step<2>(p, lane);
        xr_step<1>(p, lane);
        part[w - 1][2 * r2 + hh] = p[0];
        __syncthreads();
        return;
    }
    const double *W = dinv + (int64_t)blk * DB * DB;
    const bool has_near = blk + 1 < nblk;
#pragma unroll 8
    for (int c = 0; c < DB; ++c) Ws[lane][c] = W[lane + c * DB];  // Ws[a][b] = Winv(a, b)
    double lcol[DB];
#pragma unroll
    for (int r = 0; r < DB; ++r) {
        const int64_t row = (int64_t)(blk + 1) * DB + r;
        lcol[r] = (has_near && row < n && cv) ? L[row + col * ldl] : 0.0;
    }
    const double b = cv ? x[col] : 0.0;
    __syncthreads();
    double rhs = b - ((part[0][lane] + part[1][lane]) + part[2][lane]);
    if (has_near) {
        const int64_t rn = (int64_t)(blk + 1) * DB + lane;
        const double xv = rn < n ? mbox_poll(&mbox[rn], abortf) : 0.0;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int r = 0; r < DB; r += 2) {
            a0 = fma(lcol[r], rdlane(xv, r), a0);
            a1 = fma(lcol[r + 1], rdlane(xv, r + 1), a1);
        }
        rhs -= a0 + a1;
    }
    double z0 = 0.0, z1 = 0.0;
#pragma unroll
    for (int r = 0; r < DB; r += 2) {  // (Winv^T rhs)[lane] = sum_r Winv(r, lane) rhs_r
        z0 = fma(Ws[r][lane], rdlane(rhs, r), z0);
        z1 = fma(Ws[r + 1][lane], rdlane(rhs, r + 1), z1);
    }
    const double z = z0 + z1;
    if (cv) {
        x[col] = z;
        mbox_put(&mbox[col], z);
    }
}

// Solves in 128-row steps.  The chain of the 64-row solves above pays one
// publish / poll round trip per 64 rows; here one workgroup of 8 waves takes
// a 128-row block B (64-blocks s0 = 2B, s1 = 2B + 1) with diagonal block
// D = [[L00, 0], [L10, L11]], W0 = L00^{-1}, W1 = L11^{-1}, and
// H = W1 L10 W0 (formed when the workgroup starts), so that
//   D^{-1} = [[W0, 0], [-H, W1]]:  both halves of the block come out of
// independent products once its right-hand side is known, and the chain
// pays one round trip per 128 rows.  Waves 4-7 take the far tiles as their
// values appear (wave 4 + h: row (or column) half h & 1, every other tile by
// h >> 1).  Waves 0-3 hold the quarters of the 128 x 128 near block in
// registers and form its product with the neighbouring block's values as
// they land; then wave 0 solves the first half and wave 1 the second.
// Vectors that every lane of a product needs are broadcast through LDS (one
// read per term, four accumulators), not by cross-lane reads.
constexpr int SB = 2 * DB;

struct Trsv2Smem {
    double W0s[DB][DB + 1], W1s[DB][DB + 1];
    double Ms[DB][DB + 1];  // L10, then H
    double Ts[DB][DB + 1];  // L10 W0
    double pf[4][DB], pn[4][DB], bv[2][DB], vb[4][DB];
    int blk;
};

// Waves 0-3: W0, W1 and L10 = L[s1 rows, s0 columns] into LDS, then
// H = W1 (L10 W0) (wave q: columns 16 q .. 16 q + 15).  Every wave of the
// workgroup passes the two barriers.
GP_DEV void trsv2_setup(Trsv2Smem &sm, const double *L, int64_t ldl, int64_t n, const double *dinv, int B,
                        bool has1) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t R0 = (int64_t)B * SB;
    if (w < 4) {
        const double *W0 = dinv + (int64_t)(2 * B) * DB * DB;
        for (int e = threadIdx.x; e < DB * DB; e += 256) {
            const int a = e & (DB - 1), c = e >> 6;
            sm.W0s[a][c] = W0[a + c * DB];
            if (has1) {
                sm.W1s[a][c] = dinv[(int64_t)(2 * B + 1) * DB * DB + a + c * DB];
                const int64_t r = R0 + DB + a;
                sm.Ms[a][c] = r < n ? L[r + (R0 + c) * ldl] : 0.0;
            }
        }
    }
    __syncthreads();
    if (w < 4 && has1) {  // T = L10 W0
        double t[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) t[c] = 0.0;
        for (int k = 0; k < DB; ++k) {
            const double l = sm.Ms[lane][k];
#pragma unroll
            for (int c = 0; c < 16; ++c) t[c] = fma(l, sm.W0s[k][16 * w + c], t[c]);
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) sm.Ts[lane][16 * w + c] = t[c];
    }
    __syncthreads();
    if (w < 4 && has1) {  // H = W1 T (overwrites L10)
        double t[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) t[c] = 0.0;
        for (int k = 0; k < DB; ++k) {
            const double a = sm.W1s[lane][k];
#pragma unroll
            for (int c = 0; c < 16; ++c) t[c] = fma(a, sm.Ts[k][16 * w + c], t[c]);
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) sm.Ms[lane][16 * w + c] = t[c];
    }
}

// Forward: x_B = D^{-1} (b_B - sum_{j < B} L[B, j] x_j): with r = the
// bracket, x_0 = W0 r_0 and x_1 = W1 r_1 - H r_0.
__global__ __launch_bounds__(512) void k_trsv2_fwd(const double *L, int64_t ldl, double *x, int64_t n,
                                                   const double *dinv, int *sync, double *mbox,
                                                   const int32_t *info) {
    __shared__ Trsv2Smem sm;
    if (info && *info) return;
    const int nsb = (int)((n + SB - 1) / SB), nblk = (int)((n + DB - 1) / DB);
    if (threadIdx.x == 0) sm.blk = atomicAdd(&sync[0], 1);
    __syncthreads();
    const int B = sm.blk;
    if (B >= nsb) return;
    int *abortf = &sync[1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t R0 = (int64_t)B * SB;
    const bool has1 = 2 * B + 1 < nblk;
    trsv2_setup(sm, L, ldl, n, dinv, B, has1);
    if (w >= 4) {
        // far tiles t < 2B - 2 (all full, all rows of them published before x_prev)
        const int h = w - 4, rh = h & 1;
        const int64_t i = R0 + DB * rh + lane;
        const bool rv = i < n;
        double acc = 0.0;
        for (int t = h >> 1; t < 2 * B - 2; t += 2) {
            // the tile's 64 loads go out before the poll: they do not depend on x
            const double *Lc = L + (rv ? i : R0) + (int64_t)t * DB * ldl;
            double v[DB];
#pragma unroll
            for (int c = 0; c < DB; ++c) v[c] = Lc[(int64_t)c * ldl];
            const double xv = mbox_poll(&mbox[(int64_t)t * DB + lane], abortf);
            if (rv) {
                double a1 = 0.0;
#pragma unroll
                for (int c = 0; c < DB; c += 2) {
                    acc = fma(v[c], rdlane(xv, c), acc);
                    a1 = fma(v[c + 1], rdlane(xv, c + 1), a1);
                }
                acc += a1;
            }
        }
        sm.pf[h][lane] = acc;
        __syncthreads();  // #1
        return;
    }
    const int rq = w >> 1, cq = w & 1;
    const int64_t row = R0 + DB * rq + lane;  // this lane's row of the block
    const bool rv = row < n;
    if (w < 2) sm.bv[w][lane] = R0 + DB * w + lane < n ? x[R0 + DB * w + lane] : 0.0;  // b of half w
    double part = 0.0;
    if (B >= 1) {
        // quarter (rq, cq) of the near block: rows of half rq, columns of 64-block 2 (B - 1) + cq
        const int64_t c0 = (int64_t)(2 * (B - 1) + cq) * DB;
        double nv[DB];
#pragma unroll
        for (int c = 0; c < DB; ++c) nv[c] = rv ? L[row + (c0 + c) * ldl] : 0.0;
        sm.vb[w][lane] = mbox_poll(&mbox[c0 + lane], abortf);
        wave_lds_sync();
        double a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int c = 0; c < DB; c += 4) {
            part = fma(nv[c], sm.vb[w][c], part);
            a1 = fma(nv[c + 1], sm.vb[w][c + 1], a1);
            a2 = fma(nv[c + 2], sm.vb[w][c + 2], a2);
            a3 = fma(nv[c + 3], sm.vb[w][c + 3], a3);
        }
        part += (a1 + a2) + a3;
    }
    sm.pn[w][lane] = part;
    __syncthreads();  // #1: far and near partials in
    if (w >= 2 || (w == 1 && !has1)) return;
    // r_0 into vb[0] (wave 0) or vb[2] (wave 1), r_1 into vb[1]
    const double r0 = sm.bv[0][lane] - ((sm.pf[0][lane] + sm.pf[2][lane]) + (sm.pn[0][lane] + sm.pn[1][lane]));
    double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
    if (w == 0) {
        sm.vb[0][lane] = r0;
        wave_lds_sync();
#pragma unroll
        for (int c = 0; c < DB; c += 4) {
            z0 = fma(sm.W0s[lane][c], sm.vb[0][c], z0);
            z1 = fma(sm.W0s[lane][c + 1], sm.vb[0][c + 1], z1);
            z2 = fma(sm.W0s[lane][c + 2], sm.vb[0][c + 2], z2);
            z3 = fma(sm.W0s[lane][c + 3], sm.vb[0][c + 3], z3);
        }
    } else {
        sm.vb[2][lane] = r0;
        sm.vb[1][lane] = sm.bv[1][lane] - ((sm.pf[1][lane] + sm.pf[3][lane]) + (sm.pn[2][lane] + sm.pn[3][lane]));
        wave_lds_sync();
#pragma unroll
        for (int c = 0; c < DB; c += 2) {
            z0 = fma(sm.W1s[lane][c], sm.vb[1][c], z0);
            z1 = fma(sm.W1s[lane][c + 1], sm.vb[1][c + 1], z1);
            z2 = fma(-sm.Ms[lane][c], sm.vb[2][c], z2);
            z3 = fma(-sm.Ms[lane][c + 1], sm.vb[2][c + 1], z3);
        }
    }
    const double z = (z0 + z1) + (z2 + z3);
    const int64_t i = R0 + DB * w + lane;
    if (i < n) {
        x[i] = z;
        mbox_put(&mbox[i], z);
    }
}

// Backward: x_B = D^{-T} (b_B - sum_{j > B} L[j, B]^T x_j), taken from the
// last block: with r = the bracket, x_1 = W1^T r_1 and x_0 = W0^T r_0 -
// H^T r_1.  Far waves: lane (hh, r2) reads rows 2 r2, 2 r2 + 1 of a tile in
// columns 2 q + hh as 16-byte loads (as in the 64-row backward solve).
__global__ __launch_bounds__(512) void k_trsv2_trans(const double *L, int64_t ldl, double *x, int64_t n,
                                                     const double *dinv, int *sync, double *mbox,
                                                     const int32_t *info) {
    __shared__ Trsv2Smem sm;
    if (info && *info) return;
    const int nsb = (int)((n + SB - 1) / SB), nblk = (int)((n + DB - 1) / DB);
    if (threadIdx.x == 0) sm.blk = atomicAdd(&sync[0], 1);
    __syncthreads();
    const int tk = sm.blk;
    if (tk >= nsb) return;
    const int B = nsb - 1 - tk;
    int *abortf = &sync[1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t C0 = (int64_t)B * SB;
    const bool has1 = 2 * B + 1 < nblk;
    trsv2_setup(sm, L, ldl, n, dinv, B, has1);
    if (w >= 4) {
        // far row tiles t >= 2 (B + 2), last first; they exist only when this
        // block is not one of the last two, so its 128 columns are all < n
        const int h = w - 4, ch = h & 1;
        const int hh = lane >> 5, r2 = lane & 31;
        const int64_t c0 = C0 + DB * ch;
        double p[DB / 2];
#pragma unroll
        for (int q = 0; q < DB / 2; ++q) p[q] = 0.0;
        for (int t = nblk - 1 - (h >> 1); t >= 2 * (B + 2); t -= 2) {
            const int64_t r = (int64_t)t * DB + 2 * r2;
            const double *Lr = L + r + (c0 + hh) * ldl;
            if (r + 1 < n) {
                // the tile's loads go out before the polls: they do not depend on x
                gp_d2u v[DB / 2];
#pragma unroll
                for (int q = 0; q < DB / 2; ++q) v[q] = *reinterpret_cast<const gp_d2u *>(Lr + (int64_t)(2 * q) * ldl);
                const double x0 = mbox_poll(&mbox[r], abortf);
                const double x1 = mbox_poll(&mbox[r + 1], abortf);
#pragma unroll
                for (int q = 0; q < DB / 2; ++q) p[q] = fma(v[q].y, x1, fma(v[q].x, x0, p[q]));
            } else if (r < n) {
                const double x0 = mbox_poll(&mbox[r], abortf);
#pragma unroll
                for (int q = 0; q < DB / 2; ++q) p[q] = fma(Lr[(int64_t)(2 * q) * ldl], x0, p[q]);
            }
        }
        xr_step<16>(p, lane);
        xr_step<8>(p, lane);
        xr_step<4>(p, lane);
        xr_step<2>(p, lane);
        xr_step<1>(p, lane);
        sm.pf[h][2 * r2 + hh] = p[0];
        __syncthreads();  // #1
        return;
    }
    const int rq = w >> 1, cq = w & 1;
    const int64_t col = C0 + DB * cq + lane;  // this lane's column of the block
    const bool cvq = col < n;
    if (w < 2) sm.bv[w][lane] = cvq ? x[col] : 0.0;
    double part = 0.0;
    if (B + 1 < nsb) {
        // quarter (rq, cq) of the block below: rows of 64-block 2 (B + 1) + rq, columns of half cq
        const int64_t r0 = (int64_t)(2 * (B + 1) + rq) * DB;
        double nv[DB];
#pragma unroll
        for (int r = 0; r < DB; ++r) nv[r] = (cvq && r0 + r < n) ? L[r0 + r + col * ldl] : 0.0;
        sm.vb[w][lane] = r0 + lane < n ? mbox_poll(&mbox[r0 + lane], abortf) : 0.0;
        wave_lds_sync();
        double a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int r = 0; r < DB; r += 4) {
            part = fma(nv[r], sm.vb[w][r], part);
            a1 = fma(nv[r + 1], sm.vb[w][r + 1], a1);
            a2 = fma(nv[r + 2], sm.vb[w][r + 2], a2);
            a3 = fma(nv[r + 3], sm.vb[w][r + 3], a3);
        }
        part += (a1 + a2) + a3;
    }
    sm.pn[w][lane] = part;
    __syncthreads();  // #1
    if (w >= 2 || (w == 1 && !has1)) return;
    const double r1 = has1 ? sm.bv[1][lane] - ((sm.pf[1][lane] + sm.pf[3][lane]) + (sm.pn[1][lane] + sm.pn[3][lane]))
                           : 0.0;
    double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
    if (w == 1) {
        sm.vb[1][lane] = r1;
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < DB; r += 4) {  // (W1^T r_1)[lane] = sum_r W1(r, lane) r_1[r]
            z0 = fma(sm.W1s[r][lane], sm.vb[1][r], z0);
            z1 = fma(sm.W1s[r + 1][lane], sm.vb[1][r + 1], z1);
            z2 = fma(sm.W1s[r + 2][lane], sm.vb[1][r + 2], z2);
            z3 = fma(sm.W1s[r + 3][lane], sm.vb[1][r + 3], z3);
        }
    } else {
        sm.vb[0][lane] = sm.bv[0][lane] - ((sm.pf[0][lane] + sm.pf[2][lane]) + (sm.pn[0][lane] + sm.pn[2][lane]));
        sm.vb[2][lane] = r1;
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < DB; r += 2) {  // W0^T r_0 - H^T r_1
            z0 = fma(sm.W0s[r][lane], sm.vb[0][r], z0);
            z1 = fma(sm.W0s[r + 1][lane], sm.vb[0][r + 1], z1);
            if (has1) {
                z2 = fma(-sm.Ms[r][lane], sm.vb[2][r], z2);
                z3 = fma(-sm.Ms[r + 1][lane], sm.vb[2][r + 1], z3);
            }
        }
    }
    const double z = (z0 + z1) + (z2 + z3);
    const int64_t i = C0 + DB * w + lane;
    if (i < n) {
        x[i] = z;
        mbox_put(&mbox[i], z);
    }
}

__global__ void k_fill_u64(uint64_t *p, int64_t cnt, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = v;
}

// Zero fill, grid-stride: a dispatch holds fewer than 2^32 work-items, so a
// buffer of n^2 doubles (n > 46341) cannot take one work-item per element.
// 16-byte stores over the aligned bulk, 4-byte stores for the rest.
__global__ void k_fill_zero(uint32_t *p, int64_t cnt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t head = (int64_t)((16 - ((uintptr_t)p & 15)) & 15) / 4;  // u32 before 16-byte alignment
    const int64_t h = head < cnt ? head : cnt;
    const int64_t nv = (cnt - h) / 4;
    uint4 *v = reinterpret_cast<uint4 *>(p + h);
    for (int64_t i = t0; i < nv; i += stride) v[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = t0; i < h; i += stride) p[i] = 0u;
    for (int64_t i = h + 4 * nv + t0; i < cnt; i += stride) p[i] = 0u;
}

__global__ void k_set_info(int32_t *info) { *info = 0; }

__global__ void k_raise_flag(int *p) { *p = 1; }

// After a solve: a wait of the solve that gave up (its abort flag, sync[1])
// turns info 0 into -1, so the evaluation reports the failure (the solved
// values then hold NaN sentinels).
__global__ void k_solve_status(const int *sync, int32_t *info) {
    if (sync[1] != 0 && *info == 0) *info = -1;
}

// A failed evaluation (info != 0): NaN scalars, NaN alpha and gradient.
__global__ __launch_bounds__(256) void k_fail_outputs(int64_t n, const int32_t *info, double *out3, double *alpha,
                                                      double *grad, int ngrad) {
    if (*info == 0) return;
    const double nan = __builtin_nan("");
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < 3 && out3) out3[i] = nan;
    if (i < ngrad && grad) grad[i] = nan;
    if (alpha && i < n) alpha[i] = nan;
}

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

hipError_t launch_panel_chol(hipStream_t s, double *A, int64_t lda, int K, double *dinv, double *W, int64_t ldw,
                             int *flags, int32_t *info, int64_t col0, int raise_abort) {
    if (K <= 0) return hipSuccess;
    if (K > DB * PF_MAXB || (W && (K % DB != 0 || ldw < K))) return hipErrorInvalidValue;
    hipError_t e = launch_fill(s, flags, panel_flags_bytes());
    if (e != hipSuccess) return e;
    if (raise_abort) hipLaunchKernelGGL(k_raise_flag, dim3(1), dim3(1), 0, s, flags + PF_ABORT);
    hipLaunchKernelGGL(k_panel_chol, dim3((unsigned)((K + DB - 1) / DB)), dim3(256), 0, s, A, lda, K, dinv, W, ldw,
                       flags, info, col0, 1, (int64_t)0, (int64_t)0, (int64_t)0, (int64_t)0);
    return hipGetLastError();
}

hipError_t launch_block_trtri(hipStream_t s, const double *L, int64_t ldl, int K, int64_t nblocks, const double *dinv,
                              double *W, int *flags, const int32_t *info) {
    if (K <= 0 || nblocks <= 0) return hipSuccess;
    if (K > DB * PF_MAXB || K % DB != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_panel_chol, dim3((unsigned)(K / DB), (unsigned)nblocks), dim3(256), 0, s,
                       const_cast<double *>(L), ldl, K, const_cast<double *>(dinv), W, (int64_t)K, flags,
                       const_cast<int32_t *>(info), (int64_t)0, 0, (int64_t)K * (ldl + 1), (int64_t)(K / DB) * DB * DB,
                       (int64_t)K * K, (int64_t)0);
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
    const int64_t want = (cnt / 4 + 255) / 256;
    const unsigned g = (unsigned)(want < 1 ? 1 : (want > 8192 ? 8192 : want));
    hipLaunchKernelGGL(k_fill_zero, dim3(g), dim3(256), 0, s, (uint32_t *)p, cnt);
    return hipGetLastError();
}

size_t trsv_work_bytes(int64_t n) { return 256 + sizeof(double) * (size_t)((n + DB - 1) / DB) * DB; }

hipError_t launch_trsv(hipStream_t s, int trans, const double *L, int64_t ldl, double *x, int64_t n,
                       const double *dinv, void *work, const int32_t *info, int raise_abort) {
    if (n <= 0) return hipSuccess;
    const int nblk = (int)((n + DB - 1) / DB);
    int *sync = static_cast<int *>(work);
    double *mbox = reinterpret_cast<double *>(static_cast<char *>(work) + 256);
    hipError_t e = launch_fill(s, sync, 256);
    if (e != hipSuccess) return e;
    if (raise_abort) hipLaunchKernelGGL(k_raise_flag, dim3(1), dim3(1), 0, s, sync + 1);
    const int64_t cnt = (int64_t)nblk * DB;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<uint64_t *>(mbox), cnt, MBOX_EMPTY);
    const int nsb = (int)((n + SB - 1) / SB);
    if (n <= SB) {  // one or two 64-blocks: the 64-row chain is as short
        if (trans)
            hipLaunchKernelGGL(k_trsv_trans, dim3((unsigned)nblk), dim3(256), 0, s, L, ldl, x, n, dinv, sync, mbox, info);
        else
            hipLaunchKernelGGL(k_trsv_fwd, dim3((unsigned)nblk), dim3(256), 0, s, L, ldl, x, n, dinv, sync, mbox, info);
    } else if (trans) {
        hipLaunchKernelGGL(k_trsv2_trans, dim3((unsigned)nsb), dim3(512), 0, s, L, ldl, x, n, dinv, sync, mbox, info);
    } else {
        hipLaunchKernelGGL(k_trsv2_fwd, dim3((unsigned)nsb), dim3(512), 0, s, L, ldl, x, n, dinv, sync, mbox, info);
    }
    return hipGetLastError();
}

hipError_t launch_solve_status(hipStream_t s, const void *work, int32_t *info) {
    hipLaunchKernelGGL(k_solve_status, dim3(1), dim3(1), 0, s, static_cast<const int *>(work), info);
    return hipGetLastError();
}

hipError_t launch_fail_outputs(hipStream_t s, int64_t n, const int32_t *info, double *out3, double *alpha,
                               double *grad, int ngrad) {
    const int64_t cnt = alpha && n > 4 ? n : 4;
    hipLaunchKernelGGL(k_fail_outputs, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, n, info, out3, alpha,
                       grad, ngrad);
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
