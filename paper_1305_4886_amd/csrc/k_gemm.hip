// k_gemm.hip -- matrix-core (MFMA) products for the blocked Cholesky and its
// relatives.  Section 2.1 of the paper: in the block Cholesky "most of the total
// work is in the matrix multiplications" that update the trailing blocks; here
// those updates, the panel solves (multiplication by an inverted diagonal
// block), the blocked triangular inverse and the product L^{-T} L^{-1} all run
// through one LDS-tiled FP64 MFMA kernel:
//
//   C[i, j] = beta C[i, j] + alpha sum_k op(A)[i, k] op(B)[k, j]
//
// Tiles are 128 x 128 (4 waves in a 2 x 2 grid, 64 x 64 per wave = 4 x 4
// v_mfma_f64_16x16x4 accumulators) or 128 x 64 for panel solves, K staged in
// steps of 16 through double-buffered LDS.  Global loads are mapped so that
// each wave reads 512 contiguous bytes per instruction when the operand is
// contiguous along the tile's M/N index.  Workgroup ids are remapped so that
// each of the eight XCDs (which receive workgroups round-robin) works on a
// contiguous range of tiles and shares panel rows through its own L2.
#include "internal.h"

#include <type_traits>

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

namespace {

constexpr int BK = 16;

struct TileMap {
    int64_t ntm, ntn, ntiles;
    int lower;
    int sgm, sgn;   // super-tile shape in tiles
    int bandmode;   // 0 all tiles, 1 only 0 <= bi - bj < band (own enumeration), 2 only bi - bj >= band,
                    // 3 the lower triangle with its first `band` tile columns first (split launches)
    int64_t band;
    int interleave; // 1: tile t = workgroup id (round-robin over the XCDs), 0: XCD-contiguous ranges
    int64_t t0;     // first logical tile of this launch (tiles t0 .. ntiles - 1)
    int64_t nfirst; // bandmode 3: tiles in the first `band` tile columns
};

GP_DEV void tri_decode(int64_t t, int64_t &bi, int64_t &bj) {
    double f = (sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5;
    int64_t r = (int64_t)f;
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    bi = r;
    bj = t - r * (r + 1) / 2;
}

// Tiles are enumerated in super-tiles of SG x SG tiles so that the ~64 tiles
// an XCD holds at once share SG row blocks of op(A) and SG of op(B) (about
// 4 MB of panel at K = 256, the size of one XCD's L2) instead of one row
// block and 64 column blocks.  Super-tiles: rectangular = row-major;
// lower = rows 0..SN-1 hold I + 1 super-tiles (triangle), rows >= SN hold
// SN.  Slots that fall above the diagonal or outside the matrix are idle.
constexpr int SG = 8;

GP_DEV bool decode_tile(const TileMap &tm, int64_t t, int64_t &bi, int64_t &bj) {
    if (tm.bandmode == 3) {
        // the first P = band tile columns (rows 0 .. P - 1 a triangle, then P
        // tiles a row), then the triangle right of them, row by row
        const int64_t P = tm.band;
        if (t < tm.nfirst) {
            const int64_t tri = P * (P + 1) / 2;
            if (t < tri) {
                tri_decode(t, bi, bj);
            } else {
                const int64_t u = t - tri;
                bi = P + u / P;
                bj = u - (bi - P) * P;
            }
        } else {
            tri_decode(t - tm.nfirst, bi, bj);
            bi += P;
            bj += P;
        }
        return bi < tm.ntm;
    }
    if (tm.bandmode == 1) {  // tiles on the first `band` tile diagonals: t = bj * band + offset
        bj = t / tm.band;
        bi = bj + (t - bj * tm.band);
        return bi < tm.ntm && bj < tm.ntn;
    }
    const int64_t SN = (tm.ntn + tm.sgn - 1) / tm.sgn;
    const int64_t per = (int64_t)tm.sgm * tm.sgn;
    const int64_t st = t / per, w = t - st * per;
    int64_t I, J;
    if (!tm.lower) {
        I = st / SN;
        J = st - I * SN;
    } else {
        const int64_t tri = SN * (SN + 1) / 2;
        if (st < tri) {
            tri_decode(st, I, J);
        } else {
            const int64_t u = st - tri;
            I = SN + u / SN;
            J = u - (I - SN) * SN;
        }
    }
    bi = I * tm.sgm + w / tm.sgn;
    bj = J * tm.sgn + w % tm.sgn;
    return bi < tm.ntm && bj < tm.ntn && (!tm.lower || bi >= bj) && (tm.bandmode != 2 || bi - bj >= tm.band);
}

// Eight XCDs receive workgroups round-robin; give each XCD a contiguous range
// of logical tiles (neighbouring tiles share panel rows in that XCD's L2).
// gridDim.x is a multiple of 8.  Products whose tiles have K ranges cut by a
// triangular operand keep the round-robin order instead: their busy tiles
// cluster in a few rows, which contiguous ranges would hand to one or two
// XCDs.
GP_DEV int64_t xcd_remap(const TileMap &tm) {
    if (tm.interleave) return tm.t0 + blockIdx.x;
    const int64_t g8 = gridDim.x >> 3;
    return tm.t0 + (int64_t)(blockIdx.x & 7) * g8 + (blockIdx.x >> 3);
}

// ---------------------------------------------------------------------------
// FP64 MFMA GEMM.  BM x BN tile, WM x WN waves.
// ---------------------------------------------------------------------------
// TAG only separates instantiations by role in kernel traces:
// 0 generic product, 1 FP64 trailing update, 2 update inside a panel,
// 3 panel solve, 4 FP64 band tiles of a mixed-precision trailing update.
template <int BM, int BN, int WM, int WN, int TA, int TB, int TAG>
__global__ __launch_bounds__(256, 2) void k_gemm_f64(GemmDesc d, TileMap tm) {
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int FM = WTM / 16, FN = WTN / 16;
    constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
    static_assert(WM * WN == 4, "4 waves");
    __shared__ double As[2][BK][BM + 1];
    __shared__ double Bs[2][BK][BN + 1];

    if (d.info && *d.info) return;
    const int64_t t = xcd_remap(tm);
    if (t >= tm.ntiles) return;
    int64_t bi, bj;
    if (!decode_tile(tm, t, bi, bj)) return;
    // tile indices are workgroup-uniform: keep them (and the slab base
    // pointers derived from them) in scalar registers
    bi = __builtin_amdgcn_readfirstlane((int)bi);
    bj = __builtin_amdgcn_readfirstlane((int)bj);
    const int64_t i0 = bi * BM, j0 = bj * BN;
    const int64_t bz = blockIdx.y;
    const double *A = d.A + bz * d.sA;
    const double *B = d.B + bz * d.sB;
    double *C = d.C + bz * d.sC;

    int64_t klo = 0, khi = d.K;
    if (d.klo_i && i0 > klo) klo = i0;
    if (d.klo_j && j0 > klo) klo = j0;
    if (d.khi_i && i0 + (d.khi_i == 2 ? 0 : BM) < khi) khi = i0 + (d.khi_i == 2 ? 0 : BM);
    if (d.khi_j && j0 + BN < khi) khi = j0 + BN;
    klo = (klo / BK) * BK;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;

    v4d acc[FM][FN];
#pragma unroll
    for (int m = 0; m < FM; ++m)
#pragma unroll
        for (int n = 0; n < FN; ++n) acc[m][n] = v4d{0.0, 0.0, 0.0, 0.0};

    // Loop-invariant load descriptors: element (ii, kk) of a K-slab sits at a
    // 32-bit offset from the slab's uniform base pointer, so a K-step issues
    // its 16 loads with no address arithmetic.  Rows/columns outside the
    // matrix read the slab base (a valid element) and are zeroed.
    uint32_t offA[LA], offB[LB];
    bool okA[LA], okB[LB];
#pragma unroll
    for (int r = 0; r < LA; ++r) {
        const int e = r * 256 + tid;
        const int ii = TA ? e / BK : e % BM;
        const int kk = TA ? e % BK : e / BM;
        okA[r] = i0 + ii < d.M;
        offA[r] = okA[r] ? (uint32_t)(8 * (TA ? kk + (int64_t)ii * d.lda : ii + (int64_t)kk * d.lda)) : 0u;
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
        const int e = r * 256 + tid;
        const int jj = TB ? e % BN : e / BK;
        const int kk = TB ? e / BN : e % BK;
        okB[r] = j0 + jj < d.N;
        offB[r] = okB[r] ? (uint32_t)(8 * (TB ? jj + (int64_t)kk * d.ldb : kk + (int64_t)jj * d.ldb)) : 0u;
    }
    const bool edge = (i0 + BM > d.M) || (j0 + BN > d.N);
    double ra[LA], rb[LB];

    auto gload = [&](int64_t k0) {
        const char *Ak = reinterpret_cast<const char *>(TA ? A + k0 + i0 * d.lda : A + i0 + k0 * d.lda);
        const char *Bk = reinterpret_cast<const char *>(TB ? B + j0 + k0 * d.ldb : B + k0 + j0 * d.ldb);
        auto ldA = [&](uint32_t o) { return *reinterpret_cast<const double *>(Ak + o); };
        auto ldB = [&](uint32_t o) { return *reinterpret_cast<const double *>(Bk + o); };
        if (k0 + BK <= khi) {
            if (!edge) {
#pragma unroll
                for (int r = 0; r < LA; ++r) ra[r] = ldA(offA[r]);
#pragma unroll
                for (int r = 0; r < LB; ++r) rb[r] = ldB(offB[r]);
            } else {
#pragma unroll
                for (int r = 0; r < LA; ++r) {
                    const double v = ldA(offA[r]);
                    ra[r] = okA[r] ? v : 0.0;
                }
#pragma unroll
                for (int r = 0; r < LB; ++r) {
                    const double v = ldB(offB[r]);
                    rb[r] = okB[r] ? v : 0.0;
                }
            }
        } else {  // K tail: columns k >= khi are zero
            const int kr = (int)(khi - k0);
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int e = r * 256 + tid;
                const int kk = TA ? e % BK : e / BM;
                const bool ok = okA[r] && kk < kr;
                const double v = ldA(ok ? offA[r] : 0u);
                ra[r] = ok ? v : 0.0;
            }
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                const int e = r * 256 + tid;
                const int kk = TB ? e / BN : e % BK;
                const bool ok = okB[r] && kk < kr;
                const double v = ldB(ok ? offB[r] : 0u);
                rb[r] = ok ? v : 0.0;
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
            const int e = r * 256 + tid;
            const int ii = TA ? e / BK : e % BM;
            const int kk = TA ? e % BK : e / BM;
            As[buf][kk][ii] = ra[r];
        }
#pragma unroll
        for (int r = 0; r < LB; ++r) {
            const int e = r * 256 + tid;
            const int jj = TB ? e % BN : e / BK;
            const int kk = TB ? e / BN : e % BK;
            Bs[buf][kk][jj] = rb[r];
        }
    };

    if (klo < khi) {
        gload(klo);
        sstore(0);
        __syncthreads();
        int buf = 0;
        for (int64_t k0 = klo; k0 < khi; k0 += BK) {
            const bool more = k0 + BK < khi;
            if (more) gload(k0 + BK);
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                double a[FM], b[FN];
#pragma unroll
                for (int m = 0; m < FM; ++m) a[m] = As[buf][kk + (lane >> 4)][wm * WTM + m * 16 + (lane & 15)];
#pragma unroll
                for (int n = 0; n < FN; ++n) b[n] = Bs[buf][kk + (lane >> 4)][wn * WTN + n * 16 + (lane & 15)];
#pragma unroll
                for (int m = 0; m < FM; ++m)
#pragma unroll
                    for (int n = 0; n < FN; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[n], acc[m][n], 0, 0, 0);
            }
            if (more) sstore(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }

    // D layout of v_mfma_f64_16x16x4 on gfx950 (checked with a probe of the
    // builtin): lane l, register r holds row l / 16 + 4 r, column l % 16.
    // All C loads of the tile are issued before any store so their latencies
    // overlap; interior tiles strictly below the diagonal skip every mask.
    const int64_t rb0 = i0 + wm * WTM + (lane >> 4);
    const int64_t cb0 = j0 + wn * WTN + (lane & 15);
    const bool interior = (i0 + BM <= d.M) && (j0 + BN <= d.N) && (!d.lower || i0 >= j0 + BN);
    const bool use_c = d.beta != 0.0;
    // Chunked per row group m: 4 FN loads in flight, then the stores, which
    // keeps the C staging within the register budget left by the accumulators.
    if (interior) {
#pragma unroll
        for (int m = 0; m < FM; ++m) {
            double cv[FN][4];
            if (use_c) {
#pragma unroll
                for (int n = 0; n < FN; ++n)
#pragma unroll
                    for (int r = 0; r < 4; ++r) cv[n][r] = C[(rb0 + m * 16 + 4 * r) + (cb0 + n * 16) * d.ldc];
            }
#pragma unroll
            for (int n = 0; n < FN; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double v = d.alpha * acc[m][n][r];
                    if (use_c) v = fma(d.beta, cv[n][r], v);
                    C[(rb0 + m * 16 + 4 * r) + (cb0 + n * 16) * d.ldc] = v;
                }
        }
    } else {
#pragma unroll
        for (int m = 0; m < FM; ++m) {
            double cv[FN][4];
#pragma unroll
            for (int n = 0; n < FN; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t gi = rb0 + m * 16 + 4 * r, gj = cb0 + n * 16;
                    const bool ok = use_c && gi < d.M && gj < d.N && (!d.lower || gi >= gj);
                    const double v = C[ok ? gi + gj * d.ldc : 0];
                    cv[n][r] = ok ? v : 0.0;
                }
#pragma unroll
            for (int n = 0; n < FN; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t gi = rb0 + m * 16 + 4 * r, gj = cb0 + n * 16;
                    const bool ok = gi < d.M && gj < d.N && (!d.lower || gi >= gj);
                    if (ok) C[gi + gj * d.ldc] = fma(d.beta, cv[n][r], d.alpha * acc[m][n][r]);
                }
        }
    }
}

// ---------------------------------------------------------------------------
// Trailing update C = beta C + alpha P P^T (lower tiles) with direct-to-LDS
// loads and a STAGES-deep LDS ring.  Each K-slab (BKD panel columns, 128 rows
// per operand) is copied by global_load_lds_dword (256 bytes per instruction)
// or global_load_lds_dwordx4 (a whole 1 KB column) straight into LDS, so
// STAGES - 1 slabs are in flight while the matrix cores consume the current
// one and no registers hold staged data.  A copy address is a scalar column
// base plus a 32-bit per-lane offset.  The copies of the next slab are spread
// between the matrix instructions and the LDS reads of step kk + 1 are issued
// before the MFMAs of step kk, so a wave keeps its matrix pipe busy while it
// feeds the ring.  Rows past the
// matrix are clamped to its last row: they feed only output rows / columns
// that are never stored; columns past K are zeroed in LDS.  With d.klo_i the
// K loop of a tile starts at its first row (an operand that is zero left of
// its diagonal, such as the transpose of a lower-triangular matrix).
// ---------------------------------------------------------------------------
// X4: one 16-byte-per-lane copy moves a whole 128-row column of a slab (four
// copies per wave and slab instead of sixteen 4-byte ones); needs 16-byte
// aligned column starts (even leading dimensions, aligned bases) and an even
// row count so that a lane's two rows never straddle the last row.
// NW waves per workgroup, 2 x (NW / 2) of 64 x (256 / NW): with NW = 8 (16-byte
// copies only) each wave holds 64 x 32 (eight accumulators, 108 VGPRs), so two
// workgroups give four waves per SIMD instead of two, which hides the
// per-slab barrier and LDS latencies better (measured 61.4 against 60.5
// TFLOP/s on the trailing update at n = 32768).
template <int STAGES, int BKD, int TAG, bool X4 = false, int NW = 4>
__global__ __launch_bounds__(64 * NW, 2) void k_syrk_dma(GemmDesc d, TileMap tm) {
    static_assert(NW == 4 || (NW == 8 && X4), "eight waves only with 16-byte copies");
    constexpr int BM = 128, WTM = 64, WTN = 256 / NW, FM = 4, FN = WTN / 16, NT = 64 * NW;
    constexpr int NKK = BKD / 4;           // MFMA K-steps per slab
    constexpr int PER = X4 ? NKK * 8 / NW : NKK * 2 * 4;  // copies per wave per slab
    constexpr int CPK = PER / NKK;         // copies per K-step
    constexpr int NPAIR = FM * FN / 2;     // MFMA pairs per K-step; a copy follows every NPAIR / CPK of them
    constexpr int CPOS = NW == 8 ? 0 : NPAIR / CPK - 1;  // which pair of such a group the copy follows (measured)
    static_assert(BKD % 4 == 0 && STAGES >= 2 && NPAIR % CPK == 0, "slab shape");
    static_assert((STAGES - 2) * PER < 64, "outstanding copies exceed vmcnt");
    static_assert(STAGES * 2 * BKD * BM >= NW * 32 * WTN, "the ring holds the epilogue's wave regions");
    __shared__ double Ls[STAGES][2][BKD][BM];  // [stage][operand][k][row]

    if (d.info && *d.info) return;
    const int64_t t = xcd_remap(tm);
    if (t >= tm.ntiles) return;
    int64_t bi, bj;
    if (!decode_tile(tm, t, bi, bj)) return;
    bi = __builtin_amdgcn_readfirstlane((int)bi);
    bj = __builtin_amdgcn_readfirstlane((int)bj);
    const int64_t i0 = bi * BM, j0 = bj * BM;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave & 1, wn = wave >> 1;
    const int64_t bz = blockIdx.y;
    const double *A = d.A + bz * d.sA;
    const double *B = d.B + bz * d.sB;
    double *C = d.C + bz * d.sC;
    // K range of this tile (operands are zero outside it by structure):
    // slabs kf .. kf + nk - 1; the last one holds ktail <= BKD columns below K
    int64_t klo = 0, khi = d.K;
    if (d.klo_i && i0 - d.koff > klo) klo = i0 - d.koff;
    if (d.klo_j && j0 - d.koff > klo) klo = j0 - d.koff;
    if (d.khi_i && i0 + (d.khi_i == 2 ? 0 : BM) - d.koff < khi) khi = i0 + (d.khi_i == 2 ? 0 : BM) - d.koff;
    if (d.khi_j && j0 + BM - d.koff < khi) khi = j0 + BM - d.koff;
    if (khi <= klo && d.beta == 1.0) return;  // nothing to add to this tile
    const int kf = (int)(klo / BKD);
    const int kl = khi > klo ? (int)((khi + BKD - 1) / BKD) : kf;
    const int nk = kl - kf;
    const int ktail = (int)(d.K - (int64_t)(kl - 1) * BKD);

    uint32_t offA[4], offB[4];
    if (X4) {  // lane l: rows 2 l, 2 l + 1; pairs past the matrix read its last pair, which for an
               // odd row count holds the element past the last row (odd_rows): it lands in the LDS
               // row of the first row past the matrix, whose results are never stored
        const int64_t ra = i0 + 2 * lane < d.M ? i0 + 2 * lane : ((d.M - 1) & ~(int64_t)1);
        const int64_t rb = j0 + 2 * lane < d.N ? j0 + 2 * lane : ((d.N - 1) & ~(int64_t)1);
        offA[0] = (uint32_t)(8 * ra);
        offB[0] = (uint32_t)(8 * rb);
    } else {   // copy q: rows 32 q + lane / 2, dword lane % 2
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t r = 32 * q + (lane >> 1);
            const int64_t ra = i0 + r < d.M ? i0 + r : d.M - 1;
            const int64_t rb = j0 + r < d.N ? j0 + r : d.N - 1;
            offA[q] = (uint32_t)(8 * ra + 4 * (lane & 1));
            offB[q] = (uint32_t)(8 * rb + 4 * (lane & 1));
        }
    }
    // copy c (0 .. PER - 1) of this wave for slab `slab` into stage st:
    //   X4: column wave + NW (c / 2) of operand c % 2, all 128 rows;
    //   else: column wave + 4 (c / 8), q = c % 8: operand A rows 32 q.. (q < 4), else B
    auto copy1 = [&](int slab, int st, int c) {
        const int kk = wave + (X4 ? NW * (c >> 1) : 4 * (c >> 3));
        int64_t kc = (int64_t)(kf + slab) * BKD + kk;
        if (kc >= d.K) kc = d.K - 1;  // tail columns: any valid address, zeroed in LDS below
        if (X4) {
            if ((c & 1) == 0)
                lds_dma_dwordx4(A + kc * d.lda, offA[0], (uint32_t)(uintptr_t)&Ls[st][0][kk][0]);
            else
                lds_dma_dwordx4(B + kc * d.ldb, offB[0], (uint32_t)(uintptr_t)&Ls[st][1][kk][0]);
        } else {
            const int q = c & 7;
            if (q < 4)
                lds_dma_dword(A + kc * d.lda, offA[q], (uint32_t)(uintptr_t)&Ls[st][0][kk][32 * q]);
            else
                lds_dma_dword(B + kc * d.ldb, offB[q - 4], (uint32_t)(uintptr_t)&Ls[st][1][kk][32 * (q - 4)]);
        }
    };

#pragma unroll
    for (int s = 0; s < STAGES - 1; ++s)
        if (s < nk) {
#pragma unroll
            for (int c = 0; c < PER; ++c) copy1(s, s, c);
        }

    v4d acc[FM][FN];
#pragma unroll
    for (int m = 0; m < FM; ++m)
#pragma unroll
        for (int n = 0; n < FN; ++n) acc[m][n] = v4d{0.0, 0.0, 0.0, 0.0};

    int st = 0;
    for (int k = 0; k < nk; ++k) {
        const int later = nk - 1 - k;
        wait_slabs<PER, STAGES - 2>(later < STAGES - 2 ? later : STAGES - 2);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        const bool more = k + STAGES - 1 < nk;
        const int ns = k + STAGES - 1, nst = st == 0 ? STAGES - 1 : st - 1;
        if (k == nk - 1 && ktail < BKD) {  // columns past K contribute zero (uniform branch)
            const int nz = (BKD - ktail) * BM;
            for (int e = tid; e < 2 * nz; e += NT) {
                const int op = e >= nz, r = e - op * nz;
                Ls[st][op][ktail + r / BM][r % BM] = 0.0;
            }
            __syncthreads();
        }
        double a[FM], b[FN];
#pragma unroll
        for (int m = 0; m < FM; ++m) a[m] = Ls[st][0][(lane >> 4)][wm * WTM + m * 16 + (lane & 15)];
#pragma unroll
        for (int n = 0; n < FN; ++n) b[n] = Ls[st][1][(lane >> 4)][wn * WTN + n * 16 + (lane & 15)];
#pragma unroll
        for (int kk = 0; kk < NKK; ++kk) {
            double an[FM], bn[FN];
            if (kk + 1 < NKK) {
#pragma unroll
                for (int m = 0; m < FM; ++m)
                    an[m] = Ls[st][0][4 * (kk + 1) + (lane >> 4)][wm * WTM + m * 16 + (lane & 15)];
#pragma unroll
                for (int n = 0; n < FN; ++n)
                    bn[n] = Ls[st][1][4 * (kk + 1) + (lane >> 4)][wn * WTN + n * 16 + (lane & 15)];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < NPAIR; ++q) {
                const int m = q / (FN / 2), n0 = (q % (FN / 2)) * 2;
                acc[m][n0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[n0], acc[m][n0], 0, 0, 0);
                acc[m][n0 + 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[n0 + 1], acc[m][n0 + 1], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                if (more && q % (NPAIR / CPK) == CPOS) copy1(ns, nst, kk * CPK + q / (NPAIR / CPK));
                __builtin_amdgcn_sched_barrier(0);
            }
            if (kk + 1 < NKK) {
#pragma unroll
                for (int m = 0; m < FM; ++m) a[m] = an[m];
#pragma unroll
                for (int n = 0; n < FN; ++n) b[n] = bn[n];
            }
        }
        st = st + 1 == STAGES ? 0 : st + 1;
    }

    // Epilogue through the (now idle) LDS ring: each wave writes its 64 x WTN
    // accumulator block in two halves of 32 rows into a private region
    // (32 WTN doubles) and reads it back with lane = row, so the C tile is
    // read and written as 256-byte column segments (the MFMA D layout -- lane
    // l, register r: row l / 16 + 4 r, column l % 16 -- would give 32-byte
    // pieces of 16 columns per instruction).  The C loads of a half are issued before the
    // LDS exchange.  Region: element (row p, column g) at g 32 + (p ^ 2 (g % 16)),
    // a swizzle that keeps both the writes and the reads free of bank conflicts.
    // Tiles on the diagonal or the matrix edge keep the direct, guarded
    // stores (a guarded LDS path would spill).
    const bool interior = (i0 + BM <= d.M) && (j0 + BM <= d.N) && (!d.lower || i0 >= j0 + BM);
    const bool use_c = d.beta != 0.0;
    if (interior) {
        double *R = &Ls[0][0][0][0] + wave * (32 * WTN);
        const int p = lane & 31, hc = lane >> 5;
        __syncthreads();  // every wave is past its last ring read
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t gi = i0 + wm * WTM + 32 * h + p;
            double *Cc = C + gi + (j0 + wn * WTN + hc) * d.ldc;
            double cv[WTN / 2];
            if (use_c) {
#pragma unroll
                for (int q = 0; q < WTN / 2; ++q) cv[q] = Cc[(int64_t)(2 * q) * d.ldc];
            }
#pragma unroll
            for (int mm = 0; mm < 2; ++mm)
#pragma unroll
                for (int n = 0; n < FN; ++n)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int rr = (lane >> 4) + 4 * r + 16 * mm, g = n * 16 + (lane & 15);
                        R[g * 32 + (rr ^ (2 * (g & 15)))] = acc[2 * h + mm][n][r];
                    }
            // the wave reads back only its own region: its LDS operations complete in order
#pragma unroll
            for (int q = 0; q < WTN / 2; ++q) {
                const int g = 2 * q + hc;
                const double v = R[g * 32 + (p ^ (2 * (g & 15)))];
                Cc[(int64_t)(2 * q) * d.ldc] = use_c ? fma(d.beta, cv[q], d.alpha * v) : d.alpha * v;
            }
        }
        return;
    }
    const int64_t rb0 = i0 + wm * WTM + (lane >> 4);
    const int64_t cb0 = j0 + wn * WTN + (lane & 15);
#pragma unroll
    for (int m = 0; m < FM; ++m) {
        double cv[FN][4];
#pragma unroll
        for (int n = 0; n < FN; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = rb0 + m * 16 + 4 * r, gj = cb0 + n * 16;
                const bool ok = use_c && gi < d.M && gj < d.N && (!d.lower || gi >= gj);
                const double v = C[ok ? gi + gj * d.ldc : 0];
                cv[n][r] = ok ? v : 0.0;
            }
#pragma unroll
        for (int n = 0; n < FN; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = rb0 + m * 16 + 4 * r, gj = cb0 + n * 16;
                const bool ok = gi < d.M && gj < d.N && (!d.lower || gi >= gj);
                if (ok) C[gi + gj * d.ldc] = fma(d.beta, cv[n][r], d.alpha * acc[m][n][r]);
            }
    }
}

// ---------------------------------------------------------------------------
// Low-precision trailing update from a packed copy of the panel.
// k_pack_panel rounds the FP64 panel P (M x K, ld lda) once per panel into Q:
//   FP32 (PREC 1): Q[k Mp + r]            (column-major, ld Mp)
//   BF16 (PREC 2): Q[(k / 32) Mp 32 + 32 r + k % 32]  (32-column slabs, 64 B per row)
// with rows M .. Mp - 1 zero (Mp a multiple of 128).  k_syrk_pk then runs the
// same four-stage direct-to-LDS pipeline as the FP64 kernel on Q, with FP32
// accumulation (v_mfma_f32_16x16x4_f32: one element per lane and operand, or
// v_mfma_f32_16x16x32_bf16: 8 consecutive k per lane), and subtracts the
// products from the FP64 tile.  D layout of both (checked with a probe):
// lane l, register r holds row 4 (l / 16) + r, column l % 16.
// ---------------------------------------------------------------------------
//   BF16 split (SPLIT 2): a second copy of the same layout follows the first
//   (at element Mp Kp, Kp = K rounded up to 32) holding the remainders
//   lo = bf16(x - hi), hi = bf16(x): x = hi + lo to about 16 significant bits.
template <int PREC, int SPLIT = 1>
__global__ void k_pack_panel(const double *__restrict__ P, int64_t lda, int64_t M, int64_t Mp, int64_t K,
                             void *__restrict__ Q) {
    const int64_t Kp = PREC == 1 ? K : ((K + 31) / 32) * 32;
    const int64_t total = Mp * Kp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        if (PREC == 1) {  // e = k Mp + r: coalesced in r on both sides
            const int64_t k = e / Mp, r = e - k * Mp;
            static_cast<float *>(Q)[e] = r < M ? (float)P[r + k * lda] : 0.f;
        } else {          // e = (s Mp + r) 32 + kk
            const int64_t kk = e & 31, sr = e >> 5;
            const int64_t sl = sr / Mp, r = sr - sl * Mp, k = 32 * sl + kk;
            const double x = (r < M && k < K) ? P[r + k * lda] : 0.0;
            const __bf16 hi = (__bf16)x;
            static_cast<__bf16 *>(Q)[e] = hi;
            if (SPLIT == 2) static_cast<__bf16 *>(Q)[total + e] = (__bf16)(x - (double)(float)hi);
        }
    }
}

// SPLIT 2 (BF16 only): the panel comes as hi and lo parts (k_pack_panel<2, 2>)
// and each product is hi hi^T + hi lo^T + lo hi^T, three MFMAs per block
// (the lo lo^T term, about 2^-16 of the product, is dropped).
template <int PREC, int TAG, int STAGES = 4, int BKD = (PREC == 1 ? 16 : 32), int SPLIT = 1>
__global__ __launch_bounds__(256, 2) void k_syrk_pk(GemmDesc d, TileMap tm, const void *__restrict__ Qv, int64_t Mp,
                                                    int64_t qrow0) {
    constexpr int BM = 128, WTM = 64, FM = 4, FN = 4;
    constexpr int EB = PREC == 1 ? 4 : 2;                       // bytes per element
    constexpr int PART = BM * BKD * EB;                         // bytes of one operand part per slab
    constexpr int CHUNKS = 2 * BM * BKD * EB / 1024;            // 1 KB copies per slab and part (both operands)
    constexpr int CPO = CHUNKS / 2;                             // per operand
    constexpr int PER = SPLIT * CHUNKS / 4;                     // per wave
    constexpr int NKK = PREC == 1 ? BKD / 4 : BKD / 32;         // MFMA K-steps per slab
    static_assert(SPLIT == 1 || (PREC == 2 && SPLIT == 2 && BKD == 32), "split: BF16, one 32-column slab");
    static_assert((STAGES - 2) * PER < 64, "outstanding copies exceed vmcnt");
    static_assert(PER % NKK == 0 && (PREC == 1 ? BKD % 16 == 0 : BKD % 32 == 0), "slab shape");
    static_assert(STAGES * 2 * SPLIT * PART >= 4 * 2048 * 8, "the ring holds the epilogue's four wave regions");
    __shared__ __attribute__((aligned(16))) char Ls[STAGES][2][SPLIT * PART];

    if (d.info && *d.info) return;
    const int64_t t = xcd_remap(tm);
    if (t >= tm.ntiles) return;
    int64_t bi, bj;
    if (!decode_tile(tm, t, bi, bj)) return;
    bi = __builtin_amdgcn_readfirstlane((int)bi);
    bj = __builtin_amdgcn_readfirstlane((int)bj);
    const int64_t i0 = bi * BM, j0 = bj * BM;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave & 1, wn = wave >> 1;
    double *C = d.C;
    const int nk = (int)((d.K + BKD - 1) / BKD);
    const char *Q = static_cast<const char *>(Qv);
    // 16-byte copies (global_load_lds_dwordx4), lane l -> LDS bytes 16 l .. of
    // a 1 KB chunk.  FP32 chunk cc: columns 2 cc (lanes 0-31) and 2 cc + 1
    // (lanes 32-63), 4 rows per lane; BF16 chunk cc: rows 16 cc .. 16 cc + 15,
    // contiguous in both layouts.
    const uint32_t voff = PREC == 1 ? (uint32_t)(4 * ((lane >> 5) * Mp + 4 * (lane & 31))) : 16u * (uint32_t)lane;

    // copy q of this wave for slab `slab` into stage st: chunk c = wave + 4 q;
    // BF16 chunk cc is rows 16 (cc % 8) .. of the (cc / 8)-th 32-column slab
    // (split: copies CHUNKS .. 2 CHUNKS - 1 take the lo part, one packed panel further on)
    const int64_t part_bytes = SPLIT == 2 ? 2 * Mp * (((d.K + 31) / 32) * 32) : 0;
    auto copy1 = [&](int slab, int st, int q) {
        const int c0 = wave + 4 * q;
        const int part = c0 / CHUNKS, c = c0 % CHUNKS;
        const int op = c / CPO, cc = c % CPO;
        const int64_t row0 = qrow0 + (op ? j0 : i0);
        const char *src;
        if (PREC == 1)
            src = Q + 4 * ((int64_t)(slab * BKD + 2 * cc) * Mp + row0);
        else
            src = Q + part * part_bytes +
                  2 * (((int64_t)(slab * (BKD / 32) + cc / 8) * Mp + row0) * 32 + 512 * (int64_t)(cc % 8));
        lds_dma_dwordx4(reinterpret_cast<const double *>(src), voff,
                        (uint32_t)(uintptr_t)&Ls[st][op][part * PART + 1024 * cc]);
    };

#pragma unroll
    for (int s = 0; s < STAGES - 1; ++s)
        if (s < nk) {
#pragma unroll
            for (int q = 0; q < PER; ++q) copy1(s, s, q);
        }

    v4f acc[FM][FN];
#pragma unroll
    for (int m = 0; m < FM; ++m)
#pragma unroll
        for (int n = 0; n < FN; ++n) acc[m][n] = v4f{0.f, 0.f, 0.f, 0.f};

    int st = 0;
    for (int k = 0; k < nk; ++k) {
        const int later = nk - 1 - k;
        wait_slabs<PER, STAGES - 2>(later < STAGES - 2 ? later : STAGES - 2);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        const bool more = k + STAGES - 1 < nk;
        const int ns = k + STAGES - 1, nst = st == 0 ? STAGES - 1 : st - 1;
#pragma unroll
        for (int kk = 0; kk < NKK; ++kk) {
            if (PREC == 1) {
                const float *A = reinterpret_cast<const float *>(&Ls[st][0][0]);
                const float *B = reinterpret_cast<const float *>(&Ls[st][1][0]);
                float a[FM], b[FN];
#pragma unroll
                for (int m = 0; m < FM; ++m) a[m] = A[(4 * kk + (lane >> 4)) * BM + wm * WTM + m * 16 + (lane & 15)];
#pragma unroll
                for (int n = 0; n < FN; ++n) b[n] = B[(4 * kk + (lane >> 4)) * BM + wn * WTM + n * 16 + (lane & 15)];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
#pragma unroll
                    for (int n = 0; n < FN; ++n)
                        acc[q][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], b[n], acc[q][n], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    if (more && q == 3) copy1(ns, nst, kk);  // PER == NKK: one copy per K-step
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else if (SPLIT == 2) {
                const __bf16 *A = reinterpret_cast<const __bf16 *>(&Ls[st][0][0]);
                const __bf16 *B = reinterpret_cast<const __bf16 *>(&Ls[st][1][0]);
                const __bf16 *Al = reinterpret_cast<const __bf16 *>(&Ls[st][0][PART]);
                const __bf16 *Bl = reinterpret_cast<const __bf16 *>(&Ls[st][1][PART]);
                v8bf a[FM], b[FN], al[FM], bl[FN];
#pragma unroll
                for (int m = 0; m < FM; ++m) {
                    const int o = (wm * WTM + m * 16 + (lane & 15)) * 32 + 8 * (lane >> 4);
                    a[m] = *reinterpret_cast<const v8bf *>(&A[o]);
                    al[m] = *reinterpret_cast<const v8bf *>(&Al[o]);
                }
#pragma unroll
                for (int n = 0; n < FN; ++n) {
                    const int o = (wn * WTM + n * 16 + (lane & 15)) * 32 + 8 * (lane >> 4);
                    b[n] = *reinterpret_cast<const v8bf *>(&B[o]);
                    bl[n] = *reinterpret_cast<const v8bf *>(&Bl[o]);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < FM * FN; ++q) {
                    const int m = q >> 2, n = q & 3;
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[m], b[n], acc[m][n], 0, 0, 0);
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bl[n], acc[m][n], 0, 0, 0);
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[n], acc[m][n], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    if (more && (q & 1) == 1) copy1(ns, nst, q >> 1);  // PER == 8 copies per slab
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                const __bf16 *A = reinterpret_cast<const __bf16 *>(&Ls[st][0][8192 * kk]);
                const __bf16 *B = reinterpret_cast<const __bf16 *>(&Ls[st][1][8192 * kk]);
                v8bf a[FM], b[FN];
#pragma unroll
                for (int m = 0; m < FM; ++m)
                    a[m] = *reinterpret_cast<const v8bf *>(&A[(wm * WTM + m * 16 + (lane & 15)) * 32 + 8 * (lane >> 4)]);
#pragma unroll
                for (int n = 0; n < FN; ++n)
                    b[n] = *reinterpret_cast<const v8bf *>(&B[(wn * WTM + n * 16 + (lane & 15)) * 32 + 8 * (lane >> 4)]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < FM * FN; ++q) {
                    const int m = q >> 2, n = q & 3;
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[n], acc[m][n], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    if (more && (q & 3) == 3) copy1(ns, nst, kk * 4 + (q >> 2));
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        st = st + 1 == STAGES ? 0 : st + 1;
    }

    // Interior tiles: the same LDS-transposed write-back as the FP64 kernel
    // (D layout here: lane l, register r holds row 4 (l / 16) + r, column
    // l % 16), with the region swizzle p ^ s(g), s(g) = (g % 4) + 16 ((g / 4) % 2),
    // which spreads these writes over 32 distinct slots per instruction.
    const bool interior = (i0 + BM <= d.M) && (j0 + BM <= d.N) && (i0 >= j0 + BM);
    if (interior) {
        double *R = reinterpret_cast<double *>(&Ls[0][0][0]) + wave * 2048;
        const int p = lane & 31, hc = lane >> 5;
        __syncthreads();  // every wave is past its last ring read
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t gi = i0 + wm * WTM + 32 * h + p;
            double *Cc = C + gi + (j0 + wn * WTM + hc) * d.ldc;
            double cv[32];
#pragma unroll
            for (int q = 0; q < 32; ++q) cv[q] = Cc[(int64_t)(2 * q) * d.ldc];
#pragma unroll
            for (int mm = 0; mm < 2; ++mm)
#pragma unroll
                for (int n = 0; n < FN; ++n)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int rr = 4 * (lane >> 4) + r + 16 * mm, g = n * 16 + (lane & 15);
                        R[g * 32 + (rr ^ ((g & 3) | ((g & 4) << 2)))] = (double)acc[2 * h + mm][n][r];
                    }
            // the wave reads back only its own region: its LDS operations complete in order
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                const int g = 2 * q + hc;
                Cc[(int64_t)(2 * q) * d.ldc] = cv[q] - R[g * 32 + (p ^ ((g & 3) | ((g & 4) << 2)))];
            }
        }
        return;
    }
    const int64_t rb0 = i0 + wm * WTM + 4 * (lane >> 4);
    const int64_t cb0 = j0 + wn * WTM + (lane & 15);
#pragma unroll
    for (int m = 0; m < FM; ++m) {
        double cv[FN][4];
#pragma unroll
        for (int n = 0; n < FN; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = rb0 + m * 16 + r, gj = cb0 + n * 16;
                const bool ok = gi < d.M && gj < d.N && gi >= gj;
                cv[n][r] = C[ok ? gi + gj * d.ldc : 0];
            }
#pragma unroll
        for (int n = 0; n < FN; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = rb0 + m * 16 + r, gj = cb0 + n * 16;
                const bool ok = gi < d.M && gj < d.N && gi >= gj;
                if (ok) C[gi + gj * d.ldc] = cv[n][r] - (double)acc[m][n][r];
            }
    }
}

// Super-tiles are SG x SG tiles, narrowed to the grid when it has fewer than
// SG tile columns.  A lower map needs square super-tiles unless a single
// super-tile column covers every tile column.
TileMap make_map(int64_t M, int64_t N, int BM, int BN, int lower) {
    TileMap tm;
    tm.lower = lower;
    tm.bandmode = 0;
    tm.band = 0;
    tm.interleave = 0;
    tm.t0 = 0;
    tm.nfirst = 0;
    tm.ntm = (M + BM - 1) / BM;
    tm.ntn = (N + BN - 1) / BN;
    if (lower && tm.ntn > tm.ntm) tm.ntn = tm.ntm;
    tm.sgn = (int)(tm.ntn < SG ? tm.ntn : SG);
    tm.sgm = SG;
    const int64_t SM = (tm.ntm + tm.sgm - 1) / tm.sgm, SN = (tm.ntn + tm.sgn - 1) / tm.sgn;
    const int64_t nsuper = lower ? SN * (SN + 1) / 2 + (SM - SN) * SN : SM * SN;
    tm.ntiles = nsuper * tm.sgm * tm.sgn;  // slots, including idle ones
    return tm;
}

template <int BM, int BN, int WM, int WN, int TA, int TB, int TAG = 0>
hipError_t run_f64(hipStream_t s, const GemmDesc &d) {
    if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
    TileMap tm = make_map(d.M, d.N, BM, BN, d.lower);
    tm.interleave = (d.klo_i || d.klo_j || d.khi_i || d.khi_j) ? 1 : 0;
    const int64_t g = ((tm.ntiles + 7) / 8) * 8;
    hipLaunchKernelGGL((k_gemm_f64<BM, BN, WM, WN, TA, TB, TAG>), dim3((unsigned)g, (unsigned)d.batch), dim3(256),
                       0, s, d, tm);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_f64(hipStream_t s, const GemmDesc &d) {
    if (d.ta && d.tb) return run_f64<128, 128, 2, 2, 1, 1>(s, d);
    if (d.ta) return run_f64<128, 128, 2, 2, 1, 0>(s, d);
    if (d.tb) return run_f64<128, 128, 2, 2, 0, 1>(s, d);
    return run_f64<128, 128, 2, 2, 0, 0>(s, d);
}

namespace {

// ---------------------------------------------------------------------------
// Low-precision trailing update C -= P P^T (lower tiles only): the FP64 panel
// is rounded to FP32 (PREC 1, v_mfma_f32_16x16x4_f32, K step 16) or BF16
// (PREC 2, v_mfma_f32_16x16x32_bf16, K step 32) while it is staged into LDS;
// products accumulate in FP32 and are subtracted from the FP64 tile.  D layout
// of both instructions (checked with a probe): lane l, register r holds row
// 4 (l / 16) + r, column l % 16.
// ---------------------------------------------------------------------------
template <int PREC>
__global__ __launch_bounds__(256, 2) void k_syrk_lowp(GemmDesc d, TileMap tm) {
    constexpr int BM = 128, BN = 128, WM = 2, WN = 2;
    constexpr int WTM = BM / WM, WTN = BN / WN, FM = WTM / 16, FN = WTN / 16;
    constexpr int KS = PREC == 1 ? 16 : 32;       // K per stage
    constexpr int LA = BM * KS / 256;             // loads per operand per thread
    constexpr int PADK = 8;                       // bf16 rows: 80-byte stride keeps 16-byte alignment
    typedef typename std::conditional<PREC == 1, float, __bf16>::type ET;
    // FP32: [k][i] layout (one element per lane per MFMA); BF16: [i][k] layout (8 k per lane)
    constexpr int ROWS = PREC == 1 ? KS : BM;
    constexpr int COLS = PREC == 1 ? BM + 1 : KS + PADK;
    __shared__ ET As[2][ROWS][COLS];
    __shared__ ET Bs[2][ROWS][COLS];

    if (d.info && *d.info) return;
    const int64_t t = xcd_remap(tm);
    if (t >= tm.ntiles) return;
    int64_t bi, bj;
    if (!decode_tile(tm, t, bi, bj)) return;
    const int64_t i0 = bi * BM, j0 = bj * BN;
    const double *P = d.A;
    double *C = d.C;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;

    v4f acc[FM][FN];
#pragma unroll
    for (int m = 0; m < FM; ++m)
#pragma unroll
        for (int n = 0; n < FN; ++n) acc[m][n] = v4f{0.f, 0.f, 0.f, 0.f};

    double ra[LA], rb[LA];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
            const int e = r * 256 + tid;
            const int ii = e % BM, kk = e / BM;
            const int64_t gk = k0 + kk;
            const int64_t gi = i0 + ii, gj = j0 + ii;
            const bool oka = gi < d.M && gk < d.K, okb = gj < d.N && gk < d.K;
            const double va = P[oka ? gi + gk * d.lda : 0];
            const double vb = P[okb ? gj + gk * d.lda : 0];
            ra[r] = oka ? va : 0.0;
            rb[r] = okb ? vb : 0.0;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
            const int e = r * 256 + tid;
            const int ii = e % BM, kk = e / BM;
            if (PREC == 1) {
                As[buf][kk][ii] = (ET)(float)ra[r];
                Bs[buf][kk][ii] = (ET)(float)rb[r];
            } else {
                As[buf][ii][kk] = (ET)(float)ra[r];
                Bs[buf][ii][kk] = (ET)(float)rb[r];
            }
        }
    };

    if (d.K > 0) {
        gload(0);
        sstore(0);
        __syncthreads();
        int buf = 0;
        for (int64_t k0 = 0; k0 < d.K; k0 += KS) {
            const bool more = k0 + KS < d.K;
            if (more) gload(k0 + KS);
            if (PREC == 1) {
#pragma unroll
                for (int kk = 0; kk < KS; kk += 4) {
                    float a[FM], b[FN];
#pragma unroll
                    for (int m = 0; m < FM; ++m)
                        a[m] = (float)As[buf][kk + (lane >> 4)][wm * WTM + m * 16 + (lane & 15)];
#pragma unroll
                    for (int n = 0; n < FN; ++n)
                        b[n] = (float)Bs[buf][kk + (lane >> 4)][wn * WTN + n * 16 + (lane & 15)];
#pragma unroll
                    for (int m = 0; m < FM; ++m)
#pragma unroll
                        for (int n = 0; n < FN; ++n)
                            acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], b[n], acc[m][n], 0, 0, 0);
                }
            } else {
                v8bf a[FM], b[FN];
#pragma unroll
                for (int m = 0; m < FM; ++m)
                    a[m] = *reinterpret_cast<const v8bf *>(&As[buf][wm * WTM + m * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
                for (int n = 0; n < FN; ++n)
                    b[n] = *reinterpret_cast<const v8bf *>(&Bs[buf][wn * WTN + n * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
                for (int m = 0; m < FM; ++m)
#pragma unroll
                    for (int n = 0; n < FN; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[n], acc[m][n], 0, 0, 0);
            }
            if (more) sstore(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }

    const int64_t rb0 = i0 + wm * WTM + 4 * (lane >> 4);
    const int64_t cb0 = j0 + wn * WTN + (lane & 15);
#pragma unroll
    for (int m = 0; m < FM; ++m) {
        double cv[FN][4];
#pragma unroll
        for (int n = 0; n < FN; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = rb0 + m * 16 + r, gj = cb0 + n * 16;
                const bool ok = gi < d.M && gj < d.N && gi >= gj;
                const double v = C[ok ? gi + gj * d.ldc : 0];
                cv[n][r] = ok ? v : 0.0;
            }
#pragma unroll
        for (int n = 0; n < FN; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = rb0 + m * 16 + r, gj = cb0 + n * 16;
                const bool ok = gi < d.M && gj < d.N && gi >= gj;
                if (ok) C[gi + gj * d.ldc] = cv[n][r] - (double)acc[m][n][r];
            }
    }
}

template <int PREC>
hipError_t run_lowp(hipStream_t s, const GemmDesc &d, int64_t band) {
    if (d.M <= 0 || d.N <= 0) return hipSuccess;
    TileMap tm = make_map(d.M, d.N, 128, 128, 1);
    tm.bandmode = band > 0 ? 2 : 0;
    tm.band = band;
    const int64_t g = ((tm.ntiles + 7) / 8) * 8;
    hipLaunchKernelGGL((k_syrk_lowp<PREC>), dim3((unsigned)g), dim3(256), 0, s, d, tm);
    return hipGetLastError();
}

// FP64 update of the tiles on the first `band` tile diagonals only.
hipError_t run_band_f64(hipStream_t s, const GemmDesc &d, int64_t band) {
    if (d.M <= 0 || d.N <= 0) return hipSuccess;
    TileMap tm = make_map(d.M, d.N, 128, 128, 1);
    tm.bandmode = 1;
    tm.band = band;
    tm.ntiles = tm.ntn * band;
    const int64_t g = ((tm.ntiles + 7) / 8) * 8;
    hipLaunchKernelGGL((k_gemm_f64<128, 128, 2, 2, 0, 1, 1>), dim3((unsigned)g), dim3(256), 0, s, d, tm);
    return hipGetLastError();
}

}  // namespace

namespace {

// Lower trapezoid of 128 x 128 tiles in row-major order (no super-tiles).
// Operands whose columns start on 16-byte boundaries, with even row counts
// (or odd ones with GemmDesc::odd_rows), take 16-byte copies and two LDS stages of 16 panel columns; others four
// stages of 8 columns with 4-byte copies.  Both rings are 64 KB (two
// workgroups per CU; the 16-byte form runs eight waves per workgroup).  Measured at K = 512, M = 32256 / 16310 / 8210:
// 65.0 / 60.7 / 53.0 TFLOP/s against 62.8 / 58.5 / 50.1.
template <int TAG>
hipError_t run_dma(hipStream_t s, const GemmDesc &d) {
    if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
    TileMap tm = make_map(d.M, d.N, 128, 128, d.lower);
    tm.sgm = tm.sgn = 1;
    tm.ntiles = d.lower ? tm.ntn * (tm.ntn + 1) / 2 + (tm.ntm - tm.ntn) * tm.ntn : tm.ntm * tm.ntn;
    tm.interleave = (d.klo_i || d.klo_j || d.khi_i || d.khi_j) ? 1 : 0;
    const int64_t g = ((tm.ntiles + 7) / 8) * 8;
    const bool x4 = d.M >= 2 && d.N >= 2 && (d.odd_rows || (d.M % 2 == 0 && d.N % 2 == 0)) && d.lda % 2 == 0 &&
                    d.ldb % 2 == 0 &&
                    ((uintptr_t)d.A & 15) == 0 && ((uintptr_t)d.B & 15) == 0 &&
                    (d.batch == 1 || (d.sA % 2 == 0 && d.sB % 2 == 0));
    if (x4 && d.slab == 8)  // 8-column slabs in four stages
        hipLaunchKernelGGL((k_syrk_dma<4, 8, TAG, true>), dim3((unsigned)g, (unsigned)d.batch), dim3(256), 0, s, d, tm);
    else if (x4)            // 16-column slabs in two stages, eight waves
        hipLaunchKernelGGL((k_syrk_dma<2, 16, TAG, true, 8>), dim3((unsigned)g, (unsigned)d.batch), dim3(512), 0, s, d,
                           tm);
    else
        hipLaunchKernelGGL((k_syrk_dma<4, 8, TAG, false>), dim3((unsigned)g, (unsigned)d.batch), dim3(256), 0, s, d,
                           tm);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_syrk_lower(hipStream_t s, gp_prec_t prec, int band, const double *P, int64_t ldp,
                             double *C, int64_t ldc, int64_t M, int64_t N, int64_t K,
                             const int32_t *info, int role, int slab) {
    GemmDesc d{};
    d.A = P; d.lda = ldp; d.B = P; d.ldb = ldp; d.C = C; d.ldc = ldc;
    d.M = M; d.N = N; d.K = K; d.alpha = -1.0; d.beta = 1.0;
    d.ta = 0; d.tb = 1; d.lower = 1; d.batch = 1; d.info = info; d.slab = slab;
    d.odd_rows = 1;  // P is a panel of the matrix being factored: row M of each of its columns exists
    if (prec == GP_FP64) {
        if (K % 8 == 0) return role == 1 ? run_dma<1>(s, d) : run_dma<2>(s, d);
        if (role == 1) return run_f64<128, 128, 2, 2, 0, 1, 1>(s, d);
        return run_f64<128, 128, 2, 2, 0, 1, 2>(s, d);
    }
    const int64_t b = band > 0 ? band : 0;
    if (b > 0) {
        hipError_t e = run_band_f64(s, d, b);
        if (e != hipSuccess) return e;
    }
    return prec == GP_FP32_TRAIL ? run_lowp<1>(s, d, b) : run_lowp<2>(s, d, b);
}

// FP64 trailing update of the lower triangle of order M (C -= P P^T, P: M x K)
// in two launches over one tile order in which the first ncols columns come
// first: part 0 covers those tiles and, to fill the last round of its
// `slots` concurrent workgroups when it has at least one full round, the
// first tiles of the rest; part 1 the remaining tiles.  A caller that waits
// for the first ncols columns only (the lookahead panel) waits for part 0,
// whose last round no longer runs mostly empty.  Returns
// hipErrorInvalidValue (nothing launched) when the split does not apply:
// FP64 only with 16-byte copies, ncols a positive multiple of 128 below M,
// K a multiple of 8.  part = -1 only asks.  P is a panel of the matrix being
// factored (an odd M reads row M of its columns, see GemmDesc::odd_rows).
hipError_t launch_syrk_split(hipStream_t s, const double *P, int64_t ldp, double *C, int64_t ldc, int64_t M,
                             int64_t ncols, int64_t K, const int32_t *info, int part, int slots, int slab) {
    GemmDesc d{};
    d.A = P; d.lda = ldp; d.B = P; d.ldb = ldp; d.C = C; d.ldc = ldc;
    d.M = M; d.N = M; d.K = K; d.alpha = -1.0; d.beta = 1.0;
    d.ta = 0; d.tb = 1; d.lower = 1; d.batch = 1; d.info = info; d.slab = slab; d.odd_rows = 1;
    const bool x4 = M >= 2 && ldp % 2 == 0 && ((uintptr_t)P & 15) == 0;
    if (!x4 || slab == 8 || K % 8 != 0 || ncols <= 0 || ncols % 128 != 0 || ncols >= M || slots <= 0)
        return hipErrorInvalidValue;
    if (part < 0) return hipSuccess;
    TileMap tm = make_map(M, M, 128, 128, 1);
    const int64_t T = tm.ntm, Pc = ncols / 128;
    tm.sgm = tm.sgn = 1;
    tm.bandmode = 3;
    tm.band = Pc;
    tm.nfirst = Pc * T - Pc * (Pc - 1) / 2;
    const int64_t total = tm.nfirst + (T - Pc) * (T - Pc + 1) / 2;
    // top up only a launch that has full rounds already: a last round of
    // fewer tiles than compute units runs each tile alone on its unit, faster
    // than a full round would
    int64_t split = tm.nfirst;
    if (tm.nfirst >= slots) split = (tm.nfirst + slots - 1) / slots * (int64_t)slots;
    if (split > total) split = total;
    tm.t0 = part == 0 ? 0 : split;
    tm.ntiles = part == 0 ? split : total;
    if (tm.ntiles <= tm.t0) return hipSuccess;
    const int64_t g = ((tm.ntiles - tm.t0 + 7) / 8) * 8;
    hipLaunchKernelGGL((k_syrk_dma<2, 16, 1, true, 8>), dim3((unsigned)g), dim3(512), 0, s, d, tm);
    return hipGetLastError();
}

int64_t packed_rows(int64_t M) { return ((M + 127) / 128 + 1) * 128; }

size_t packed_panel_bytes(int64_t M, int64_t K) {
    // FP32: one float per element; BF16 split: two bf16 parts -- the same size
    return (size_t)packed_rows(M) * (size_t)(((K + 31) / 32) * 32) * sizeof(float);
}

hipError_t launch_pack_panel(hipStream_t s, gp_prec_t prec, const double *P, int64_t ldp, int64_t M, int64_t K,
                             void *Q, int split) {
    if (M <= 0 || K <= 0) return hipSuccess;
    const int64_t Mp = packed_rows(M);
    const int64_t total = prec == GP_FP32_TRAIL ? Mp * K : Mp * ((K + 31) / 32) * 32;
    const int64_t g = (total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096;
    if (prec == GP_FP32_TRAIL)
        hipLaunchKernelGGL((k_pack_panel<1>), dim3((unsigned)g), dim3(256), 0, s, P, ldp, M, Mp, K, Q);
    else if (split)
        hipLaunchKernelGGL((k_pack_panel<2, 2>), dim3((unsigned)g), dim3(256), 0, s, P, ldp, M, Mp, K, Q);
    else
        hipLaunchKernelGGL((k_pack_panel<2>), dim3((unsigned)g), dim3(256), 0, s, P, ldp, M, Mp, K, Q);
    return hipGetLastError();
}

hipError_t launch_band_f64(hipStream_t s, int band, const double *P, int64_t ldp, double *C, int64_t ldc, int64_t M,
                           int64_t N, int64_t K, const int32_t *info) {
    if (M <= 0 || N <= 0 || K <= 0 || band <= 0) return hipSuccess;
    GemmDesc d{};
    d.A = P; d.lda = ldp; d.B = P; d.ldb = ldp; d.C = C; d.ldc = ldc;
    d.M = M; d.N = N; d.K = K; d.alpha = -1.0; d.beta = 1.0;
    d.ta = 0; d.tb = 1; d.lower = 1; d.batch = 1; d.info = info;
    d.odd_rows = 1;  // P is a panel of the matrix being factored
    TileMap tb = make_map(M, N, 128, 128, 1);
    tb.bandmode = 1;
    tb.band = band;
    tb.ntiles = tb.ntn * band;
    const int64_t g = ((tb.ntiles + 7) / 8) * 8;
    const bool x4 = M >= 2 && N >= 2 && ldp % 2 == 0 && ((uintptr_t)P & 15) == 0;
    if (K % 8 != 0)
        hipLaunchKernelGGL((k_gemm_f64<128, 128, 2, 2, 0, 1, 4>), dim3((unsigned)g), dim3(256), 0, s, d, tb);
    else if (x4)
        hipLaunchKernelGGL((k_syrk_dma<2, 16, 4, true, 8>), dim3((unsigned)g), dim3(512), 0, s, d, tb);
    else
        hipLaunchKernelGGL((k_syrk_dma<4, 8, 4, false>), dim3((unsigned)g), dim3(256), 0, s, d, tb);
    return hipGetLastError();
}

hipError_t launch_lowp_packed(hipStream_t s, gp_prec_t prec, int band, const double *P, int64_t ldp, const void *Q,
                              int64_t Mpack, int64_t qrow0, double *C, int64_t ldc, int64_t M, int64_t N, int64_t K,
                              const int32_t *info, int split) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    GemmDesc d{};
    d.A = P; d.lda = ldp; d.B = P; d.ldb = ldp; d.C = C; d.ldc = ldc;
    d.M = M; d.N = N; d.K = K; d.alpha = -1.0; d.beta = 1.0;
    d.ta = 0; d.tb = 1; d.lower = 1; d.batch = 1; d.info = info;
    const int64_t b = band > 0 ? band : 0;
    TileMap tm = make_map(M, N, 128, 128, 1);
    tm.sgm = tm.sgn = 1;
    tm.ntiles = tm.ntn * (tm.ntn + 1) / 2 + (tm.ntm - tm.ntn) * tm.ntn;
    tm.bandmode = b > 0 ? 2 : 0;
    tm.band = b;
    const int64_t g = ((tm.ntiles + 7) / 8) * 8;
    const int64_t Mp = packed_rows(Mpack);
    if (((uintptr_t)Q & 15) != 0 || qrow0 % 64 != 0) return hipErrorInvalidValue;  // 16-byte copies
    if (prec == GP_FP32_TRAIL)
        hipLaunchKernelGGL((k_syrk_pk<1, 1, 2, 32>), dim3((unsigned)g), dim3(256), 0, s, d, tm, Q, Mp, qrow0);
    else if (split)  // hi / lo parts, one 32-column slab of each per LDS stage
        hipLaunchKernelGGL((k_syrk_pk<2, 1, 2, 32, 2>), dim3((unsigned)g), dim3(256), 0, s, d, tm, Q, Mp, qrow0);
    else
        if (K % 64 == 0)  // two 32-column packed slabs per LDS stage
            hipLaunchKernelGGL((k_syrk_pk<2, 1, 2, 64>), dim3((unsigned)g), dim3(256), 0, s, d, tm, Q, Mp, qrow0);
        else
            hipLaunchKernelGGL((k_syrk_pk<2, 1>), dim3((unsigned)g), dim3(256), 0, s, d, tm, Q, Mp, qrow0);
    return hipGetLastError();
}

hipError_t launch_syrk_packed(hipStream_t s, gp_prec_t prec, int band, const double *P, int64_t ldp, const void *Q,
                              int64_t Mpack, int64_t qrow0, double *C, int64_t ldc, int64_t M, int64_t N, int64_t K,
                              const int32_t *info, int split) {
    hipError_t e = launch_band_f64(s, band, P, ldp, C, ldc, M, N, K, info);
    if (e != hipSuccess) return e;
    return launch_lowp_packed(s, prec, band, P, ldp, Q, Mpack, qrow0, C, ldc, M, N, K, info, split);
}

hipError_t launch_gemm_nt_dma(hipStream_t s, const GemmDesc &d) {
    // K in chunks of KC columns: every tile then streams a bounded slab of the
    // operands (the working set of the concurrent tiles stays cache- and
    // TLB-resident), at the cost of re-reading C once per chunk.
    constexpr int64_t KC = 1024;
    if (d.K <= KC) return run_dma<0>(s, d);
    for (int64_t k0 = 0; k0 < d.K; k0 += KC) {
        GemmDesc c = d;
        c.A = d.A + k0 * d.lda;
        c.B = d.B + k0 * d.ldb;
        c.K = d.K - k0 < KC ? d.K - k0 : KC;
        c.koff = d.koff + k0;
        c.beta = k0 == 0 ? d.beta : 1.0;
        hipError_t e = run_dma<0>(s, c);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_syrk_dma(hipStream_t s, const double *P, int64_t ldp, double *C, int64_t ldc, int64_t M, int64_t K,
                           double alpha, double beta, int klo_i, const int32_t *info) {
    GemmDesc d{};
    d.A = P; d.lda = ldp; d.B = P; d.ldb = ldp; d.C = C; d.ldc = ldc;
    d.M = M; d.N = M; d.K = K; d.alpha = alpha; d.beta = beta;
    d.ta = 0; d.tb = 1; d.lower = 1; d.klo_i = klo_i; d.batch = 1; d.info = info;
    constexpr int64_t KC = 1024;
    if (K <= KC) return run_dma<0>(s, d);
    // K in chunks; with klo_i, rows at or below a chunk's end get nothing from it
    for (int64_t k0 = 0; k0 < K; k0 += KC) {
        GemmDesc c = d;
        c.A = d.A + k0 * ldp;
        c.B = c.A;
        c.K = K - k0 < KC ? K - k0 : KC;
        c.koff = k0;
        c.beta = k0 == 0 ? beta : 1.0;
        if (klo_i && k0 > 0 && k0 + c.K < M) c.M = c.N = k0 + c.K;
        hipError_t e = run_dma<0>(s, c);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_panel_solve(hipStream_t s, double *A, int64_t lda, const double *Winv, int64_t M,
                              int jb, const int32_t *info) {
    // A[0:M, 0:jb] <- A * Winv^T : op(B)[k, j] = Winv[j, k] = Winv[j + k DB] (tb = 1).
    // Each workgroup covers all jb <= 64 output columns of its 128 rows, so the
    // in-place update reads every input element of its rows before writing.
    GemmDesc d{};
    d.A = A; d.lda = lda; d.B = Winv; d.ldb = DB; d.C = A; d.ldc = lda;
    d.M = M; d.N = jb; d.K = jb; d.alpha = 1.0; d.beta = 0.0;
    d.ta = 0; d.tb = 1; d.lower = 0; d.batch = 1; d.info = info;
    return run_f64<128, 64, 4, 1, 0, 1, 3>(s, d);
}
