// internal.h -- shared declarations of the gfx950 GP-likelihood library.
// Device helpers, the handle, and the launchers each kernel file exports to
// the C-ABI layer (api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gpmi.h"

#define GP_DEV __device__ __forceinline__

// Diagonal-block edge of the inner Cholesky / inverse kernels and of the
// triangular-solve blocking.  Every diagonal inverse stored in workspace is a
// DB x DB column-major block.
constexpr int DB = 64;
// Edge of the trailing-update tiles (matrix-core kernels).
constexpr int TB = 128;

#include <vector>

// One tuned choice: for operation `op` (0 the factorisation, 1 the batched
// call) at precision `prec` and problem sizes n with floor(log2 n) == bucket.
struct TuneEntry {
    int32_t op, prec, bucket;
    int32_t nb, panel_cus, syrk_slab, batch_grid, batch_tile;
};

struct gp_handle_s {
    hipStream_t stream = nullptr;  // caller's stream
    hipStream_t side = nullptr;    // lookahead stream (default priority)
    hipEvent_t ev_cols = nullptr;  // main -> side: next panel's columns updated
    hipEvent_t ev_panel = nullptr; // side -> main: next panel factored
    hipEvent_t ev_in = nullptr;    // caller's stream -> masked main stream
    hipEvent_t ev_out = nullptr;   // masked main stream -> caller's stream
    // mixed modes: the FP64 band tiles of a trailing update run on `band`
    // (default priority) next to the low-precision tiles on the main stream
    hipStream_t band = nullptr;
    hipEvent_t ev_band_in = nullptr;   // main -> band: panel packed
    hipEvent_t ev_band_out = nullptr;  // band -> main: band tiles updated
    // With opt.panel_cus > 0 the factorisation runs on two streams of its own:
    // main_cu, masked to every compute unit but panel_cus reserved ones, and
    // side_cu, free to use all of them, so the lookahead chain always finds
    // room next to the trailing update.
    hipStream_t main_cu = nullptr;
    hipStream_t side_cu = nullptr;
    int masked_for = 0;            // panel_cus the masked streams were made for
    gp_options_t opt{};
    int device = 0;
    // optional timing of trailing updates (gp_profile)
    int prof = 0;
    std::vector<hipEvent_t> prof_ev;  // start/stop pairs
    size_t prof_used = 0;             // events in use
    double prof_flops = 0.0;
    double prof_bytes = 0.0;
    int64_t prof_launches = 0;
    int num_cu = 256;                 // compute units of the device
    void *batch_staging = nullptr;    // host staging of the batched task table
    void *scratch = nullptr;          // this device's static workspace (gp_loglik_noalloc), or null
    std::vector<TuneEntry> tune;      // tuned choices by (op, precision, size bucket)
    char arch[64] = {0};              // architecture name of the device (e.g. gfx950)
    int tuning = 0;                   // inside a tuner: explicit options only, no table lookups
    int magic = 0x67706d69;
};

// ---------------------------------------------------------------------------
// Covariance functions.  r = |x_i - x_j| / rho.
// k(r): exponential e^{-r}; Matern-3/2 (1 + a) e^{-a}, a = sqrt(3) r;
//       Matern-5/2 (1 + a + a^2/3) e^{-a}, a = sqrt(5) r.
// g(r) = -r k'(r): r e^{-r}; 3 r^2 e^{-a}; (5/3) r^2 (1 + a) e^{-a}.
// ---------------------------------------------------------------------------
struct CovParams {
    int kind;
    int dim;
    double s2, inv_rho, t2;
    double inv_rho2;  // GP_SEP_MATERN2: 1 / rho_w
};

// Components of the gradient contraction's partial sums (the separable
// family has four parameters, the others three).
constexpr int GRAD_NQ = 4;

GP_DEV double cov_corr(int kind, double r) {
    if (kind == GP_EXP) return exp(-r);
    if (kind == GP_MATERN32) {
        double a = 1.7320508075688772 * r;
        return (1.0 + a) * exp(-a);
    }
    double a = 2.23606797749979 * r;
    return (1.0 + a + a * a * (1.0 / 3.0)) * exp(-a);
}

// k(r) and g(r) together (one exp).
GP_DEV void cov_corr_g(int kind, double r, double &k, double &g) {
    if (kind == GP_EXP) {
        double e = exp(-r);
        k = e;
        g = r * e;
    } else if (kind == GP_MATERN32) {
        double a = 1.7320508075688772 * r, e = exp(-a);
        k = (1.0 + a) * e;
        g = 3.0 * r * r * e;
    } else {
        double a = 2.23606797749979 * r, e = exp(-a);
        k = (1.0 + a + a * a * (1.0 / 3.0)) * e;
        g = (5.0 / 3.0) * r * r * (1.0 + a) * e;
    }
}

GP_DEV double point_dist(const double *xi, const double *xj, int dim) {
    double s = 0.0;
    for (int d = 0; d < dim; ++d) {
        double t = xi[d] - xj[d];
        s = fma(t, t, s);
    }
    return sqrt(s);
}

// Neumaier / TwoSum helpers for compensated reductions.
GP_DEV void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
struct CSum {
    double s = 0.0, c = 0.0;
    GP_DEV void add(double v) {
        double t, e;
        two_sum(s, v, t, e);
        s = t;
        c += e;
    }
    GP_DEV void merge(const CSum &o) {
        double t, e;
        two_sum(s, o.s, t, e);
        s = t;
        c += o.c + e;
    }
    GP_DEV double value() const { return s + c; }
};

// Bounded wait used by every dependency spin in persistent kernels: about
// 2^22 polls (seconds), after which the waiter raises the abort flag and
// continues, so every wave always reaches its exit.
constexpr int SPIN_LIMIT = 1 << 22;

GP_DEV int ld_acquire_agent(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
GP_DEV void st_release_agent(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin (one lane) until *flag != 0 or abort; returns false on timeout/abort.
GP_DEV bool wait_flag(const int *flag, int *abortf) {
    int spins = 0;
    while (ld_acquire_agent(flag) == 0) {
        if (ld_acquire_agent(abortf)) return false;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > SPIN_LIMIT) {
            __hip_atomic_store(abortf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// Broadcast lane l's double (l a compile-time constant after unrolling).
GP_DEV double rdlane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// 1 / sqrt(x) to double precision: the hardware estimate (v_rsq_f64) refined
// by two Newton-Raphson steps y <- y (3 - x y^2) / 2, each of which doubles the
// number of correct bits.
GP_DEV double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}

// Orders LDS traffic between the lanes of one wave (LDS operations of a wave
// complete in order; this keeps the compiler from moving them across).
GP_DEV void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

typedef double gp_v4d __attribute__((ext_vector_type(4)));

// 16 x 16 x 16 product on the matrix cores, D = sum_k A(i, k) B(k, j) over
// k in [kbeg, kend) (multiples of 4), operands read through the callables.
// Operand layout of v_mfma_f64_16x16x4: lane l supplies A(l % 16, k0 + l / 16)
// and B(k0 + l / 16, l % 16); D lane l, register r is (l / 16 + 4 r, l % 16).
template <typename FA, typename FB>
GP_DEV gp_v4d wave_mm16(FA fa, FB fb, int kbeg, int kend, int lane) {
    gp_v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = kbeg; k0 < kend; k0 += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fa(lane & 15, k0 + (lane >> 4)), fb(k0 + (lane >> 4), lane & 15),
                                                   acc, 0, 0, 0);
    return acc;
}

// Cholesky of a 64 x 64 block held by one wave, lane r = row r (a[c] = A[r][c]).
// Right-looking in panels of 16 columns: inside a panel, column by column
// (pivot, 1 / sqrt by rsqrt_nr, scale, rank-1 update of the panel's columns to
// its right, with readlane broadcasts); then the columns right of the panel
// get A -= P P^T on the matrix cores (v_mfma_f64_16x16x4 on 16 x 16 tiles,
// operands from the panel staged in Pn, products returned through Us).  Only
// the lower triangle is meaningful on return: entries above the diagonal are
// updated without masks and hold garbage (they never feed a lower entry).
// Returns 0 or the first failing 1-based column (a non-positive or NaN
// pivot); later columns then hold garbage.  Us: 64 x 65, Pn: 64 x 17 doubles
// of LDS, used by this wave only.
GP_DEV int wave_chol64(double (&a)[DB], int lane, double (*Us)[DB + 1], double (*Pn)[17]) {
    int fail = 0;
#pragma unroll
    for (int p = 0; p < DB; p += 16) {
#pragma unroll
        for (int j = p; j < p + 16; ++j) {
            const double piv = rdlane(a[j], j);
            if (!(piv > 0.0) && fail == 0) fail = j + 1;
            const double inv = rsqrt_nr(piv);
            a[j] = (lane == j) ? piv * inv : a[j] * inv;
#pragma unroll
            for (int c = j + 1; c < p + 16; ++c) a[c] = fma(-a[j], rdlane(a[j], c), a[c]);
        }
        if (p + 16 < DB) {
#pragma unroll
            for (int k = 0; k < 16; ++k) Pn[lane][k] = a[p + k];
            wave_lds_sync();
            const int t0 = p + 16;
#pragma unroll
            for (int ti = 0; ti < (DB - p - 16) / 16; ++ti)
#pragma unroll
                for (int tj = 0; tj <= ti; ++tj) {
                    // D layout of v_mfma_f64_16x16x4: lane l, register r holds
                    // row l / 16 + 4 r, column l % 16
                    gp_v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int k0 = 0; k0 < 16; k0 += 4) {
                        const double av = Pn[t0 + 16 * ti + (lane & 15)][k0 + (lane >> 4)];
                        const double bv = Pn[t0 + 16 * tj + (lane & 15)][k0 + (lane >> 4)];
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        Us[t0 + 16 * ti + (lane >> 4) + 4 * r][t0 + 16 * tj + (lane & 15)] = acc[r];
                }
            wave_lds_sync();
#pragma unroll
            for (int c = p + 16; c < DB; ++c) a[c] -= Us[lane][c];
            wave_lds_sync();
        }
    }
    return fail;
}

// W = L^{-1} for the 64 x 64 lower factor in LDS (Ls[i][k] = L_ik for k <= i;
// entries above the diagonal are not read), one wave, blocked by 16:
// (1) the four 16 x 16 diagonal blocks by forward substitution, lane 16 b + c
//     solving column c of block b (W_cc = 1 / L_cc, W_ic = -(sum L_ik W_kc) / L_ii);
// (2) recursive doubling on the matrix cores, W21 = -W22 (L21 W11): first the
//     16-blocks (1,0) and (3,2), then the 32 x 32 block (rows 32.., cols ..31).
// The result, zeros above the diagonal included, is left in Wl.
// Scratch: T32 (32 x 33) and rd (64) doubles of LDS.
GP_DEV void wave_inv64_blocked(const double (*Ls)[DB + 1], double (*Wl)[DB + 1], double (*T32)[33], double *rd,
                               int lane) {
    rd[lane] = 1.0 / Ls[lane][lane];
    wave_lds_sync();
    {
        const int o = 16 * (lane >> 4), c = lane & 15;
        double w[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < i; ++k) s = fma(-Ls[o + i][o + k], w[k], s);
            w[i] = s * rd[o + i];
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) Wl[o + i][o + c] = w[i];
#pragma unroll
        for (int i = 0; i < DB; ++i)
            if ((i >> 4) != (lane >> 4)) Wl[i][lane] = 0.0;
    }
    wave_lds_sync();
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {  // T = L(b1, b0) W(b0, b0)
        const int o0 = 32 * pr, o1 = o0 + 16;
        const gp_v4d t = wave_mm16([&](int i, int k) { return Ls[o1 + i][o0 + k]; },
                                   [&](int k, int j) { return Wl[o0 + k][o0 + j]; }, 0, 16, lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) T32[16 * pr + (lane >> 4) + 4 * r][lane & 15] = t[r];
    }
    wave_lds_sync();
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {  // W(b1, b0) = -W(b1, b1) T
        const int o0 = 32 * pr, o1 = o0 + 16;
        const gp_v4d u = wave_mm16([&](int i, int k) { return Wl[o1 + i][o1 + k]; },
                                   [&](int k, int j) { return T32[16 * pr + k][j]; }, 0, 16, lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) Wl[o1 + (lane >> 4) + 4 * r][o0 + (lane & 15)] = -u[r];
    }
    wave_lds_sync();
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {  // T = L21 W11; block (kb, tj) of W11 is zero for kb < tj
            const gp_v4d t = wave_mm16([&](int i, int k) { return Ls[32 + 16 * ti + i][k]; },
                                       [&](int k, int j) { return Wl[k][16 * tj + j]; }, 16 * tj, 32, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) T32[16 * ti + (lane >> 4) + 4 * r][16 * tj + (lane & 15)] = t[r];
        }
    wave_lds_sync();
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {  // W21 = -W22 T; block (ti, kb) of W22 is zero for kb > ti
            const gp_v4d u = wave_mm16([&](int i, int k) { return Wl[32 + 16 * ti + i][32 + k]; },
                                       [&](int k, int j) { return T32[k][16 * tj + j]; }, 0, 16 * ti + 16, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) Wl[32 + 16 * ti + (lane >> 4) + 4 * r][16 * tj + (lane & 15)] = -u[r];
        }
    wave_lds_sync();
}

// Direct-to-LDS copies and the explicit waits that order them.
template <int N>
GP_DEV void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit field");
    // s_waitcnt vmcnt(N), expcnt and lgkmcnt left unconstrained (gfx9 encoding)
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Wait until at most j (0 <= j <= J) slabs of PER copies each are outstanding.
template <int PER, int J>
GP_DEV void wait_slabs(int j) {
    if constexpr (J == 0) {
        wait_vmcnt<0>();
    } else {
        if (j >= J)
            wait_vmcnt<J * PER>();
        else
            wait_slabs<PER, J - 1>(j);
    }
}

// One 256-byte LDS-DMA copy: lane l moves the dword at base + voff to LDS
// address lds + 4 l.  Written as inline assembly so that the compiler's
// wait-count pass, which cannot tell LDS-DMA targets apart, does not drain
// every copy in flight before each LDS read; the kernel orders the copies
// itself with explicit vmcnt waits and barriers.  m0 is restored afterwards.
GP_DEV void lds_dma_dword(const double *base, uint32_t voff, uint32_t lds_uniform) {
    uint32_t saved;
    asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %3\n\ts_nop 0\n\tglobal_load_lds_dword %1, %2\n\ts_mov_b32 m0, %0"
                 : "=&s"(saved)
                 : "v"(voff), "s"(base), "s"(lds_uniform)
                 : "memory");
}

// The same with 16 bytes per lane (gfx950): lane l moves base + voff .. + 15
// to LDS address lds + 16 l, so one instruction fills a 1 KB LDS span.
GP_DEV void lds_dma_dwordx4(const double *base, uint32_t voff, uint32_t lds_uniform) {
    uint32_t saved;
    asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %3\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %2\n\ts_mov_b32 m0, %0"
                 : "=&s"(saved)
                 : "v"(voff), "s"(base), "s"(lds_uniform)
                 : "memory");
}

// ---------------------------------------------------------------------------
// Launchers (all enqueue on `s`, return hipError_t of the launch).
// ---------------------------------------------------------------------------
// k_cov.hip
hipError_t launch_cov_lower(hipStream_t s, CovParams p, int64_t n, const double *X, double *C,
                            int64_t ldc, const int32_t *info);
hipError_t launch_cross_cov(hipStream_t s, CovParams p, int64_t n, int64_t m, const double *X,
                            const double *Xs, double *Cs, int64_t ld);
hipError_t launch_resid_matfree(hipStream_t s, CovParams p, int64_t n, const double *X,
                                const double *r0, const double *x, double *res,
                                double *partials, const int32_t *skip);
hipError_t launch_grad_contract(hipStream_t s, CovParams p, int64_t n, const double *X,
                                const double *Cinv, int64_t ldc, const double *alpha,
                                double *partials, int nparts, const int32_t *info);

// k_gemm.hip: C = beta C + alpha op(A) op(B) on 128x128 (or 128x64) tiles.
struct GemmDesc {
    const double *A;
    int64_t lda;
    const double *B;
    int64_t ldb;
    double *C;
    int64_t ldc;
    int64_t M, N, K;
    double alpha, beta;
    int ta, tb;    // op(A)[i,k] = ta ? A[k + i lda] : A[i + k lda]; op(B)[k,j] = tb ? B[j + k ldb] : B[k + j ldb]
    int lower;     // tiles and elements with i < j are skipped (C's (0,0) lies on the diagonal)
    int klo_i;     // skip k < tile row start (op(A) upper-zero structure)
    int klo_j;     // skip k < tile col start (op(B) lower-zero structure)
    int khi_i;     // 1: skip k >= tile row end (op(A) lower-triangular); 2: skip k >= tile row
                   // start (only the blocks of op(A) strictly left of the tile's diagonal block)
    int khi_j;     // skip k >= tile col end (op(B) upper-triangular)
    int64_t koff;   // absolute index of local k = 0 for the K-range flags (K split into chunks)
    int64_t batch;  // number of independent products
    int64_t sA, sB, sC; // element strides between batch members
    const int32_t *info; // skip everything if *info != 0 (may be null)
    int slab;            // FP64 direct-to-LDS kernel: K-slab of 16 columns in 2 stages (0, 16) or 8 in 4 (8)
    int odd_rows;        // 1: one element past the last row of every column of A and of B lies in the
                         // caller's storage (the factorisation's own panels), so that odd M and N can
                         // take the 16-byte copies of the direct-to-LDS kernel, whose last row pair
                         // then reads that element for the row past the matrix
};
hipError_t launch_gemm_f64(hipStream_t s, const GemmDesc &d);
// Trailing updates C -= P P^T restricted to the lower triangle, compute type
// chosen by prec (FP64, or FP32 / BF16 products with FP32 accumulation).
// band >= 0 with a low-precision prec: tiles with |bi - bj| < band use FP64.
// role: 1 trailing update, 2 update inside a panel (separate kernel names in traces).
hipError_t launch_syrk_lower(hipStream_t s, gp_prec_t prec, int band, const double *P,
                             int64_t ldp, double *C, int64_t ldc, int64_t M, int64_t N, int64_t K,
                             const int32_t *info, int role, int slab = 0);
// The FP64 trailing update of the lower triangle of order M in two launches
// (part 0: the first ncols columns' tiles, topped up to a multiple of
// `slots` with the first tiles of the rest; part 1: the rest).
// hipErrorInvalidValue, with nothing launched, where the split does not apply.
hipError_t launch_syrk_split(hipStream_t s, const double *P, int64_t ldp, double *C, int64_t ldc, int64_t M,
                             int64_t ncols, int64_t K, const int32_t *info, int part, int slots, int slab);
// Low-precision trailing updates from a packed copy of the panel: rows
// 0 .. Mpack - 1 of P (FP64, ld ldp, K columns) rounded once into Q
// (packed_panel_bytes(Mpack, K) bytes); a call then updates the M x N lower
// trapezoid whose panel rows start at packed row qrow0 (P points at that row).
// K must be a multiple of 32.  split (BF16 only): the panel is packed as hi
// and lo = bf16(x - hi) parts (packed_panel_bytes covers both) and every
// product is formed as hi hi^T + hi lo^T + lo hi^T.
int64_t packed_rows(int64_t M);
size_t packed_panel_bytes(int64_t M, int64_t K);
hipError_t launch_pack_panel(hipStream_t s, gp_prec_t prec, const double *P, int64_t ldp, int64_t M, int64_t K,
                             void *Q, int split = 0);
hipError_t launch_syrk_packed(hipStream_t s, gp_prec_t prec, int band, const double *P, int64_t ldp, const void *Q,
                              int64_t Mpack, int64_t qrow0, double *C, int64_t ldc, int64_t M, int64_t N, int64_t K,
                              const int32_t *info, int split = 0);
// The two halves of launch_syrk_packed, for callers that overlap them: the FP64
// tiles on the first `band` tile diagonals, and the low-precision rest.
hipError_t launch_band_f64(hipStream_t s, int band, const double *P, int64_t ldp, double *C, int64_t ldc, int64_t M,
                           int64_t N, int64_t K, const int32_t *info);
hipError_t launch_lowp_packed(hipStream_t s, gp_prec_t prec, int band, const double *P, int64_t ldp, const void *Q,
                              int64_t Mpack, int64_t qrow0, double *C, int64_t ldc, int64_t M, int64_t N, int64_t K,
                              const int32_t *info, int split = 0);
// C = beta C + alpha P P^T on the lower triangle of the M x M matrix C, P
// M x K (ld ldp), on the direct-to-LDS MFMA kernel; klo_i: P is zero left of
// its diagonal (P[i, k] = 0 for k < i), so tile rows i0.. start at k = i0.
hipError_t launch_syrk_dma(hipStream_t s, const double *P, int64_t ldp, double *C, int64_t ldc, int64_t M, int64_t K,
                           double alpha, double beta, int klo_i, const int32_t *info);
// Entries of a lower trapezoid of M rows x N columns (N <= M): N M - N (N - 1) / 2;
// an update of them with inner dimension K takes 2 K of flops per entry.
inline double syrk_entries(int64_t M, int64_t N) {
    return (double)N * (double)M - 0.5 * (double)N * (double)(N - 1);
}
inline double syrk_flops(int64_t M, int64_t N, int64_t K) { return 2.0 * (double)K * syrk_entries(M, N); }
// Panel solve in place: A[0:M, 0:jb] <- A[0:M, 0:jb] * Winv^T (Winv jb x jb lower, ld DB).
hipError_t launch_panel_solve(hipStream_t s, double *A, int64_t lda, const double *Winv,
                              int64_t M, int jb, const int32_t *info);

// k_chol.hip
hipError_t launch_diag_potrf(hipStream_t s, double *A, int64_t lda, int jb, double *Winv,
                             int32_t *info, int64_t col0);
hipError_t launch_diag_inv(hipStream_t s, const double *L, int64_t ldl, int64_t n, double *dinv);
// The diagonal K x K block of a panel (K <= 64 PF_MAXB) in one launch of
// ceil(K / 64) concurrent workgroups: L in place (A, lda), the 64 x 64 block
// inverses into dinv and, if W is non-null (K % 64 == 0), W = L^{-1} (ld ldw,
// zeros above the diagonal).  flags: panel_flags_bytes() of workspace.
// A non-positive pivot sets *info = col0 + its 1-based column in the block.
constexpr int PF_MAXB = 16;
constexpr size_t panel_flags_bytes() { return sizeof(int) * (PF_MAXB * PF_MAXB + 64); }
// raise_abort (test hook): the abort flag is raised before the launch, so
// every wait gives up at once and the launch reports info = -1.
hipError_t launch_panel_chol(hipStream_t s, double *A, int64_t lda, int K, double *dinv, double *W, int64_t ldw,
                             int *flags, int32_t *info, int64_t col0, int raise_abort = 0);
// W_b = L_bb^{-1} (K x K, ld K, zeros above the diagonal, at W + b K^2) for the
// nblocks consecutive K x K diagonal blocks b of a factored L (K % 64 == 0,
// K <= 64 PF_MAXB), from their 64 x 64 block inverses (dinv, consecutive).  One
// launch; flags: any valid pointer (nothing is waited for).
hipError_t launch_block_trtri(hipStream_t s, const double *L, int64_t ldl, int K, int64_t nblocks, const double *dinv,
                              double *W, int *flags, const int32_t *info);
// Work area of a triangular solve: trsv_work_bytes(n) bytes (counters and a
// mailbox of n doubles); the abort flag is its int [1].
size_t trsv_work_bytes(int64_t n);
// A wait of the solve that gives up leaves NaN sentinels in x and raises the
// abort flag in work; launch_solve_status then turns info 0 into -1.
// raise_abort (test hook) raises that flag before the launch.
hipError_t launch_trsv(hipStream_t s, int trans, const double *L, int64_t ldl, double *x, int64_t n,
                       const double *dinv, void *work, const int32_t *info, int raise_abort = 0);
hipError_t launch_solve_status(hipStream_t s, const void *work, int32_t *info);
// With *info != 0: out3 (3), grad (ngrad) and alpha (n) set to NaN (null pointers skipped).
hipError_t launch_fail_outputs(hipStream_t s, int64_t n, const int32_t *info, double *out3, double *alpha,
                               double *grad, int ngrad = 3);
hipError_t launch_sub_mu(hipStream_t s, int64_t n, const double *y, const double *mu, double *z);
hipError_t launch_copy_vec(hipStream_t s, int64_t n, const double *a, double *b);
hipError_t launch_loglik_reduce(hipStream_t s, int64_t n, const double *L, int64_t ldl,
                                const double *z, double *out3, const int32_t *info,
                                const int *sync);
hipError_t launch_fill(hipStream_t s, void *p, size_t bytes);

// k_aux.hip
// mode 0: out[j] = base + sum_i M_ij v_i; mode 1: out[j] = base - sum_i M_ij^2.
hipError_t launch_copy2d(hipStream_t s, int64_t rows, int64_t cols, const double *src, int64_t lds, double *dst,
                         int64_t ldd);
hipError_t launch_place_dinv(hipStream_t s, int64_t n, const double *dinv, double *W, int64_t ldw, int trans = 0);
// dst = src^T for a rows x cols block (batch blocks at element strides sstr / dstr).
hipError_t launch_transpose_copy(hipStream_t s, int64_t rows, int64_t cols, const double *src, int64_t lds,
                                 int64_t sstr, double *dst, int64_t ldd, int64_t dstr, int64_t batch);
// The FP64 direct-to-LDS MFMA kernel on a general product
//   C = beta C + alpha A B^T  (A: M x K, B: N x K, both column-major),
// with GemmDesc's lower / K-range / batch fields (ta = 0, tb = 1 form).
hipError_t launch_gemm_nt_dma(hipStream_t s, const GemmDesc &d);
hipError_t launch_grad_finish(hipStream_t s, int nparts, const double *partials, double *grad, int ngrad,
                              const int32_t *info);
// iterative refinement control (state: 8 doubles; done: int32 skip flag)
hipError_t launch_ir_init(hipStream_t s, int64_t n, const double *b, double *state, int32_t *done,
                          const int32_t *info);
hipError_t launch_ir_check(hipStream_t s, int64_t n, const double *res, double *state, int32_t *done, int last,
                           double tol);
hipError_t launch_copy_skip(hipStream_t s, int64_t n, const double *a, double *b, const int32_t *done);
hipError_t launch_axpy_skip(hipStream_t s, int64_t n, const double *dv, double *x, const int32_t *done);
hipError_t launch_ir_finish(hipStream_t s, int64_t n, const double *b, const double *x, const double *state,
                            double *out3, double *ir, const int32_t *info);
// Morton order: keys needs next_pow2(n) uint64, box 4 doubles.
hipError_t launch_morton(hipStream_t s, int64_t n, int dim, const double *X, int64_t *perm, uint64_t *keys,
                         double *box);
hipError_t launch_gather_points(hipStream_t s, int64_t n, int dim, const int64_t *perm, const double *X,
                                const double *y, const double *mu, double *Xp, double *yp, double *mup);
hipError_t launch_scatter_vec(hipStream_t s, int64_t n, const int64_t *perm, const double *src, double *dst);
hipError_t launch_set_info(hipStream_t s, int32_t *info);
hipError_t launch_tune_fill(hipStream_t s, double *A, int64_t lda, int64_t n);
// Row reductions of an m x n column-major matrix (compensated, two passes;
// partials holds 2 m rowreduce_chunks(n) doubles):
//   mode 0: out_j = base + sum_i Y(j, i) v_i      mode 1: out_j = base - sum_i Y(j, i)^2
int64_t rowreduce_chunks(int64_t n);
hipError_t launch_rowreduce(hipStream_t s, int mode, int64_t m, int64_t n, const double *Y, int64_t ldy,
                            const double *v, double base, double *partials, double *out);
// out[i + c ldo] += sum_{b <= a} L(i0 + a, i0 + b) E(i0 + b, c) over the
// 128-row diagonal blocks (i = i0 + a): the part of L E that the products on
// strictly lower blocks leave out.  Only the lower triangle of L is read.
constexpr int TRMM_DB = 128;
hipError_t launch_trmm_diag(hipStream_t s, int64_t m, int64_t r, const double *L, int64_t ldl, const double *E,
                            int64_t lde, double *out, int64_t ldo, const int32_t *info);
// out[i + c ldo] = mean ? mean[i] : mu  (m x r)
hipError_t launch_bcast_rows(hipStream_t s, int64_t m, int64_t r, const double *mean, double mu, double *out,
                             int64_t ldo);
// With *info != 0: out (m x r) set to NaN.
hipError_t launch_fail_fill(hipStream_t s, int64_t m, int64_t r, double *out, int64_t ldo, const int32_t *info);
// Strict upper triangle of the m x m matrix A set to zero.
hipError_t launch_zero_upper(hipStream_t s, int64_t m, double *A, int64_t lda);

// k_batch.hip
size_t batch_ws_bytes(int64_t nmax, int64_t nbatch, bool persistent, int tile);
int batch_run(hipStream_t s, int num_cu, int grid, int tile, void *&staging, int32_t nb, const gp_theta_t *th, const int64_t *nh,
              const int64_t *xoff, const int64_t *coff, int32_t dim, const double *X, const double *y,
              double *C_pool, double *out3, int32_t *info, void *ws, size_t ws_bytes);
void batch_staging_free(void *p);
