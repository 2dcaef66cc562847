// api.hip -- the C ABI declared in include/gpmi.h: argument checks,
// workspace layout and the host-side orchestration of the kernels.
//
// Blocked Cholesky (Section 2.1, Fig. 1; the h = 1 schedule of Section 2.2 is
// the same dependency graph on one device): for each panel of nb columns,
//   for each 64-column sub-panel d:   factor + invert the diagonal block (LDS),
//                                     solve the rows below on the matrix cores,
//                                     update the rest of the panel;
//   then the trailing SYRK/GEMM update of everything to the right (matrix cores).
// With lookahead the columns of panel k+1 are updated first and panel k+1 is
// factored on a second stream while the rest of panel k's trailing update
// runs, which keeps the diagonal-block chain (the critical path of Section 2.1)
// off the critical path of the device.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>

#include "internal.h"

// from k_cov.hip
int resid_chunks(int64_t n);

namespace {

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int64_t nblocks(int64_t n) { return (n + DB - 1) / DB; }

bool ok_handle(gp_handle_t h) { return h && h->magic == 0x67706d69; }

// theta check: log sigma^2 and log tau^2 may be -inf (an exact zero), never
// +inf or NaN; log rho must be finite.
int check_theta(const gp_theta_t &th) {
    if (th.kind < GP_EXP || th.kind > GP_SEP_MATERN2) return 1;
    if (isnan(th.log_sigma2) || th.log_sigma2 == INFINITY) return 2;
    if (!isfinite(th.log_rho)) return 2;
    if (isnan(th.log_tau2) || th.log_tau2 == INFINITY) return 2;
    if (th.kind == GP_SEP_MATERN2 && !isfinite(th.log_rho2)) return 2;
    return 0;
}

// The separable family takes points (t, w, v): dimension 3.
bool bad_dim(const gp_theta_t &th, int dim) {
    return dim < 1 || dim > 16 || (th.kind == GP_SEP_MATERN2 && dim != 3);
}

CovParams cov_params(const gp_theta_t &th, int dim) {
    CovParams p;
    p.kind = th.kind;
    p.dim = dim;
    p.s2 = exp(th.log_sigma2);
    p.inv_rho = exp(-th.log_rho);
    p.t2 = exp(th.log_tau2);
    p.inv_rho2 = th.kind == GP_SEP_MATERN2 ? exp(-th.log_rho2) : 0.0;
    return p;
}

// ---- workspace layouts ------------------------------------------------------
struct Layout {
    size_t dinv = 0, sync = 0, z = 0, vec2 = 0, vec3 = 0, vec4 = 0, vec5 = 0, part = 0, big1 = 0, big2 = 0,
           big3 = 0, irst = 0, perm = 0, keys = 0, box = 0, xp = 0, yp = 0, mup = 0, pbuf = 0, vinv = 0,
           vtmp = 0, qbuf = 0, big4 = 0, pflags = 0, kw = 0, total = 0;
    // second factorisation (gp_simulate: the covariance of the new points)
    size_t dinv2 = 0, pflags2 = 0, pbuf2 = 0, vinv2 = 0, vtmp2 = 0, et = 0, meanv = 0;
};

// Buffers of the panel steps of the factorisation (null when n <= NB).
struct PanelBufs {
    double *pbuf = nullptr;  // copy of the rows below a diagonal block, (n - NB + 1) x NB
    double *vinv = nullptr;  // inverse of a diagonal block, NB x NB
    double *vtmp = nullptr;  // products of the blocked inverse, trtri_tmp_elems(NB)
    void *qbuf = nullptr;    // low-precision packed panel (mixed modes)
    int *pflags = nullptr;   // hand-over flags of the fused panel kernel
};

// Panel width: the option, or (0) 768 for FP64 and 512 for the mixed modes,
// whose FP32 / BF16 products accumulate over the panel width (768 measured
// 2 % faster than 512 in FP64; no difference in the mixed modes, where the
// shorter accumulation keeps the log-determinant error lower).
// Size bucket of the tuning table: floor(log2 n).
int size_bucket(int64_t n) {
    int b = 0;
    while (b < 62 && (int64_t(2) << b) <= n) ++b;
    return b;
}

const TuneEntry *tune_find(gp_handle_t h, int op, gp_prec_t prec, int64_t n) {
    const int b = size_bucket(n);
    for (const TuneEntry &e : h->tune)
        if (e.op == op && e.prec == (int32_t)prec && e.bucket == b) return &e;
    return nullptr;
}

void tune_store(gp_handle_t h, const TuneEntry &e) {
    for (TuneEntry &x : h->tune)
        if (x.op == e.op && x.prec == e.prec && x.bucket == e.bucket) {
            x = e;
            return;
        }
    h->tune.push_back(e);
}

// The tail width: panels that start where at most TAIL_SPAN x tail columns
// remain are that narrow (when it is below nb), because there a wide panel's
// chain of diagonal-block steps on the side stream outlasts the trailing
// update it overlaps.
constexpr int64_t TAIL_SPAN = 24;

// The factorisation's choices for (prec, n): explicit options (nb > 0) win;
// with nb = 0 (automatic) a tuned entry for n's size bucket, else the
// defaults; the tail width from the option (0: 512).
struct PotrfChoice {
    int64_t nb;
    int panel_cus, slab;
    int64_t tail;
};
PotrfChoice potrf_choice(gp_handle_t h, gp_prec_t prec, int64_t n) {
    PotrfChoice c;
    if (h->opt.nb > 0 || h->tuning)
        c = {h->opt.nb > 0 ? h->opt.nb : 768, h->opt.panel_cus, h->opt.syrk_slab, 0};
    else if (const TuneEntry *e = tune_find(h, 0, prec, n))
        c = {e->nb, e->panel_cus, e->syrk_slab, 0};
    else
        c = {prec == GP_FP64 ? 768 : (prec == GP_FP32_TRAIL ? 512 : 640), h->opt.panel_cus, h->opt.syrk_slab, 0};
    const int64_t tw = h->opt.tail_nb == 0 ? 512 : h->opt.tail_nb;
    c.tail = (tw > 0 && tw < c.nb) ? tw : c.nb;
    return c;
}

// Width of the panel that starts at column c of an n-column factorisation (the
// last one clipped to n).  Widths never grow along the factorisation.
int64_t panel_at(const PotrfChoice &ch, int64_t n, int64_t c) {
    const int64_t w = (ch.tail < ch.nb && n - c <= TAIL_SPAN * ch.tail) ? ch.tail : ch.nb;
    return c + w < n ? w : n - c;
}

// The widest panel (the first): what the panel buffers of the workspace hold.
int64_t panel_width(gp_handle_t h, gp_prec_t prec, int64_t n) {
    const PotrfChoice ch = potrf_choice(h, prec, n);
    const int64_t w = (ch.tail < ch.nb && n <= TAIL_SPAN * ch.tail) ? ch.tail : ch.nb;
    return w;
}

// The batched call's schedule: the option unless it is the automatic 0 and a
// tuned entry exists for the largest problem's size bucket.
int batch_grid_choice(gp_handle_t h, int64_t nmax) {
    if (h->opt.batch_grid != 0 || h->tuning) return h->opt.batch_grid;
    if (const TuneEntry *e = tune_find(h, 1, GP_FP64, nmax)) return e->batch_grid;
    return 0;
}

// Tile edge of the persistent batched launch, resolved the same way (128 by default).
int batch_tile_choice(gp_handle_t h, int64_t nmax) {
    if (h->opt.batch_tile != 0 || h->tuning) return h->opt.batch_tile != 0 ? h->opt.batch_tile : 128;
    if (const TuneEntry *e = tune_find(h, 1, GP_FP64, nmax))
        if (e->batch_tile != 0) return e->batch_tile;
    return 128;
}

// Workspace of the batched call: the largest over the tile edges a later call
// could pick (the table can change between the query and the call).
size_t batch_ws_any(gp_handle_t h, int64_t nmax, int64_t nbatch) {
    if (batch_grid_choice(h, nmax) < 0 && h->opt.batch_grid != 0) return batch_ws_bytes(nmax, nbatch, false, 64);
    const size_t a = batch_ws_bytes(nmax, nbatch, true, 64), b = batch_ws_bytes(nmax, nbatch, true, 128);
    const size_t c = batch_ws_bytes(nmax, nbatch, false, 64);
    return std::max(std::max(a, b), c);
}

// Reserved compute unit r of `reserve`: spaced ncu / reserve apart and offset
// by r mod 8, which gives every XCD the same share whether mask bits are
// numbered XCD by XCD or round-robin over the eight XCDs.
int reserved_cu(int r, int reserve, int ncu) {
    const int c = r * (ncu / reserve) + (r % 8);
    return c < ncu ? c : ncu - 1;
}

inline int64_t next_pow2(int64_t n) {
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Blocked triangular inverse by recursive doubling: at level S (S = 128, 256,
// ...) node a covers rows/cols [a S, min((a + 1) S, n)); its top half [aS,
// aS + S/2) and bottom half (h2 rows) are already inverted.  The product
// T = L21 W11 (h2 x S/2) of every node of the level lives in one buffer.
size_t trtri_tmp_elems(int64_t n) {
    size_t mx = 1;
    for (int64_t S = 2 * DB; S / 2 < n; S *= 2) {
        const int64_t h = S / 2;
        size_t tot = 0;
        for (int64_t o = 0; o + h < n; o += S) {
            const int64_t h2 = (o + S <= n) ? h : n - o - h;
            tot += (size_t)h2 * (size_t)h;
        }
        if (tot > mx) mx = tot;
    }
    return mx;
}

constexpr int GRAD_PARTS = 2048;

// Realizations per product of the simulation (the transposed normals of one
// chunk, SIM_CHUNK x m doubles, live in the workspace).
constexpr int64_t SIM_CHUNK = 512;

// Column band of the kriging solve C*^T L^{-T}: each band is solved by one
// product with the inverse of its diagonal block, then the columns right of
// it are updated with K = KRIGE_BAND.
constexpr int64_t KRIGE_BAND = 512;

Layout layout(gp_handle_t h, gp_op_t op, int64_t n, int64_t m, gp_prec_t prec) {
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += al256(bytes);
        return o;
    };
    const int64_t nb = nblocks(n);
    const size_t vec = sizeof(double) * (size_t)(n > 0 ? n : 1);
    const int64_t NB = panel_width(h, prec, n);
    auto take_panel = [&]() {
        if (n <= NB) return;
        L.pbuf = take(sizeof(double) * (size_t)(n - NB + 1) * (size_t)NB);
        L.vinv = take(sizeof(double) * (size_t)NB * (size_t)NB);
        L.vtmp = take(sizeof(double) * trtri_tmp_elems(NB));
        if (prec != GP_FP64) L.qbuf = take(packed_panel_bytes(n - NB, NB));
    };
    switch (op) {
    case GP_OP_POTRF:
        L.dinv = take(sizeof(double) * DB * DB * (size_t)nb);
        L.pflags = take(panel_flags_bytes());
        take_panel();
        break;
    case GP_OP_TRSV:
        L.dinv = take(sizeof(double) * DB * DB * (size_t)nb);
        L.sync = take(trsv_work_bytes(n));
        break;
    case GP_OP_TRSM:
        L.dinv = take(sizeof(double) * DB * DB * (size_t)nb);
        L.part = take(sizeof(double) * DB * (size_t)(m > 0 ? m : 1));
        break;
    case GP_OP_LOGLIK:
    case GP_OP_LOGLIK_GRAD:
        L.dinv = take(sizeof(double) * DB * DB * (size_t)nb);
        L.pflags = take(panel_flags_bytes());
        take_panel();
        L.sync = take(trsv_work_bytes(n));
        L.z = take(vec);     // L^{-1} b
        L.vec2 = take(vec);  // x = C^{-1} b (evaluation order)
        L.vec3 = take(vec);  // b = y - mu (evaluation order)
        L.part = take(sizeof(double) *
                      (size_t)(2 * GRAD_NQ * GRAD_PARTS > 4 * (n + 8) ? 2 * GRAD_NQ * GRAD_PARTS : 4 * (n + 8)));
        if (prec != GP_FP64) {
            L.vec4 = take(vec);  // residual
            L.vec5 = take(vec);  // correction
            L.irst = take(sizeof(double) * 8 + sizeof(int32_t) * 4);
            L.big2 = take(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)resid_chunks(n > 0 ? n : 1));
            L.perm = take(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
            L.keys = take(sizeof(uint64_t) * (size_t)next_pow2(n > 0 ? n : 1));
            L.box = take(sizeof(double) * 4);
            L.xp = take(sizeof(double) * 16 * (size_t)(n > 0 ? n : 1));
            L.yp = take(vec);
            L.mup = take(vec);
        }
        if (op == GP_OP_LOGLIK_GRAD) {
            // W = L^{-1} and V = W^T (n x n, ld n) and the product buffer of the blocked inverse
            L.big1 = take(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1));
            L.big4 = take(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1));
            L.big3 = take(sizeof(double) * trtri_tmp_elems(n));
        }
        break;
    case GP_OP_BATCHED:
        L.total = batch_ws_any(h, n > 0 ? n : 1, m > 0 ? m : 1);
        return L;
    case GP_OP_MORTON:
        L.keys = take(sizeof(uint64_t) * (size_t)next_pow2(n > 0 ? n : 1));
        L.box = take(sizeof(double) * 4);
        break;
    case GP_OP_TRMM:  // m = right-hand sides: their transpose
        L.et = take(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)(m > 0 ? m : 1));
        break;
    case GP_OP_SIMULATE: {
        // n data points (0: unconditional), m new points
        const size_t mm = (size_t)(m > 0 ? m : 1);
        if (n > 0) {
            L.dinv = take(sizeof(double) * DB * DB * (size_t)nb);
            L.big1 = take(sizeof(double) * (size_t)n * mm);
            L.part = take(sizeof(double) * KRIGE_BAND * mm);
            L.pflags = take(panel_flags_bytes());
            if (n >= KRIGE_BAND) L.kw = take(sizeof(double) * (size_t)(n / KRIGE_BAND) * KRIGE_BAND * KRIGE_BAND);
            L.big2 = take(sizeof(double) * 2 * mm * (size_t)rowreduce_chunks(n));
        }
        L.dinv2 = take(sizeof(double) * DB * DB * (size_t)nblocks(m));
        L.pflags2 = take(panel_flags_bytes());
        const int64_t NB2 = panel_width(h, GP_FP64, m);
        if (m > NB2) {
            L.pbuf2 = take(sizeof(double) * (size_t)(m - NB2 + 1) * (size_t)NB2);
            L.vinv2 = take(sizeof(double) * (size_t)NB2 * (size_t)NB2);
            L.vtmp2 = take(sizeof(double) * trtri_tmp_elems(NB2));
        }
        L.et = take(sizeof(double) * SIM_CHUNK * mm);
        L.meanv = take(sizeof(double) * mm);
        break;
    }
    case GP_OP_KRIGE_COV:
    case GP_OP_KRIGE:
        L.dinv = take(sizeof(double) * DB * DB * (size_t)nb);
        L.big1 = take(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)(m > 0 ? m : 1));  // C*^T, m x n
        L.part = take(sizeof(double) * KRIGE_BAND * (size_t)(m > 0 ? m : 1));                // m x band copy
        L.pflags = take(panel_flags_bytes());
        if (n >= KRIGE_BAND)  // inverses of the full KRIGE_BAND diagonal blocks
            L.kw = take(sizeof(double) * (size_t)(n / KRIGE_BAND) * KRIGE_BAND * KRIGE_BAND);
        L.big2 = take(sizeof(double) * 2 * (size_t)(m > 0 ? m : 1) * (size_t)(n > 0 ? rowreduce_chunks(n) : 1));
        break;
    default:
        break;
    }
    L.total = off < 256 ? 256 : off;
    return L;
}

template <typename T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

PanelBufs panel_bufs(void *ws, const Layout &L) {
    PanelBufs p;
    if (L.vinv) {  // never the first buffer of a layout
        p.pbuf = at<double>(ws, L.pbuf);
        p.vinv = at<double>(ws, L.vinv);
        p.vtmp = at<double>(ws, L.vtmp);
        if (L.qbuf) p.qbuf = at<char>(ws, L.qbuf);
    }
    if (L.pflags) p.pflags = at<int>(ws, L.pflags);
    return p;
}

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) return GP_ERR_HIP;                                                   \
    } while (0)

// Trailing update, bracketed by events when the handle profiles.
hipError_t trailing(gp_handle_t h, hipStream_t s, gp_prec_t prec, const double *P, int64_t ldp, double *C,
                    int64_t ldc, int64_t M, int64_t N, int64_t K, const int32_t *info, int slab) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->prof) {
        while (h->prof_ev.size() < h->prof_used + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
            h->prof_ev.push_back(e);
        }
        e0 = h->prof_ev[h->prof_used];
        e1 = h->prof_ev[h->prof_used + 1];
        h->prof_used += 2;
        hipEventRecord(e0, s);
    }
    hipError_t e = launch_syrk_lower(s, prec, h->opt.band, P, ldp, C, ldc, M, N, K, info, 1, slab);
    if (h->prof) {
        hipEventRecord(e1, s);
        h->prof_flops += syrk_flops(M, N, K);
        h->prof_bytes += 16.0 * syrk_entries(M, N);
        h->prof_launches += 1;
    }
    return e;
}

// One part of a split FP64 trailing update (launch_syrk_split), bracketed
// like trailing(); part 0 counts the work of the first ncols columns, part 1
// that of the rest, so that the two sum to the unsplit pair.
hipError_t trailing_part(gp_handle_t h, hipStream_t s, const double *P, int64_t ldp, double *C, int64_t ldc,
                         int64_t M, int64_t ncols, int64_t K, const int32_t *info, int slab, int slots, int part) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->prof) {
        while (h->prof_ev.size() < h->prof_used + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
            h->prof_ev.push_back(e);
        }
        e0 = h->prof_ev[h->prof_used];
        e1 = h->prof_ev[h->prof_used + 1];
        h->prof_used += 2;
        hipEventRecord(e0, s);
    }
    hipError_t e = launch_syrk_split(s, P, ldp, C, ldc, M, ncols, K, info, part, slots, slab);
    if (h->prof) {
        hipEventRecord(e1, s);
        const int64_t Mp = part == 0 ? M : M - ncols, Np = part == 0 ? ncols : M - ncols;
        h->prof_flops += syrk_flops(Mp, Np, K);
        h->prof_bytes += 16.0 * syrk_entries(Mp, Np);
        h->prof_launches += 1;
    }
    return e;
}

// Low-precision trailing update from the packed panel, bracketed like trailing().
hipError_t trailing_packed(gp_handle_t h, hipStream_t s, gp_prec_t prec, const double *P, int64_t ldp,
                           const void *Q, int64_t Mpack, int64_t qrow0, double *C, int64_t ldc, int64_t M,
                           int64_t N, int64_t K, const int32_t *info) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->prof) {
        while (h->prof_ev.size() < h->prof_used + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
            h->prof_ev.push_back(e);
        }
        e0 = h->prof_ev[h->prof_used];
        e1 = h->prof_ev[h->prof_used + 1];
        h->prof_used += 2;
        hipEventRecord(e0, s);
    }
    // FP64 band tiles on their own stream, concurrent with the low-precision
    // tiles (disjoint C tiles, same read-only panel)
    hipError_t e = hipSuccess;
    if (h->opt.band > 0) {
        e = hipEventRecord(h->ev_band_in, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(h->band, h->ev_band_in, 0);
        if (e == hipSuccess) e = launch_band_f64(h->band, h->opt.band, P, ldp, C, ldc, M, N, K, info);
        if (e == hipSuccess) e = hipEventRecord(h->ev_band_out, h->band);
    }
    if (e == hipSuccess)
        e = launch_lowp_packed(s, prec, h->opt.band, P, ldp, Q, Mpack, qrow0, C, ldc, M, N, K, info, h->opt.bf16_split);
    if (e == hipSuccess && h->opt.band > 0) e = hipStreamWaitEvent(s, h->ev_band_out, 0);
    if (h->prof) {
        hipEventRecord(e1, s);
        h->prof_flops += syrk_flops(M, N, K);
        h->prof_bytes += 16.0 * syrk_entries(M, N);
        h->prof_launches += 1;
    }
    return e;
}

// ---- blocked Cholesky -------------------------------------------------------
// Blocked triangular inverse W = L^{-1} of an n x n lower factor whose 64 x 64
// diagonal blocks are already inverted (dinv, consecutive blocks), by
// recursive doubling (see trtri_tmp_elems).  W is dense n x n with ldw == n;
// T holds trtri_tmp_elems(n) doubles.
int trtri_lower(hipStream_t s, int64_t n, const double *L, int64_t ldl, const double *dinv, double *W,
                double *T, const int32_t *info) {
    const int64_t ldw = n;
    HIPCHK(launch_fill(s, W, sizeof(double) * (size_t)n * (size_t)n));
    HIPCHK(launch_place_dinv(s, n, dinv, W, ldw));
    for (int64_t S = 2 * DB; S / 2 < n; S *= 2) {
        const int64_t hh = S / 2;
        const int64_t nfull = n / S;
        if (nfull > 0) {
            GemmDesc d{};
            d.A = L + hh; d.lda = ldl; d.sA = S * (1 + ldl);           // L21 of node 0
            d.B = W; d.ldb = ldw; d.sB = S * (1 + ldw);                 // W11
            d.C = T; d.ldc = hh; d.sC = hh * hh;
            d.M = hh; d.N = hh; d.K = hh; d.alpha = 1.0; d.beta = 0.0;
            d.klo_j = 1; d.batch = nfull; d.info = info;
            HIPCHK(launch_gemm_f64(s, d));
            GemmDesc e{};
            e.A = W + hh * (1 + ldw); e.lda = ldw; e.sA = S * (1 + ldw);  // W22
            e.B = T; e.ldb = hh; e.sB = hh * hh;
            e.C = W + hh; e.ldc = ldw; e.sC = S * (1 + ldw);              // W21
            e.M = hh; e.N = hh; e.K = hh; e.alpha = -1.0; e.beta = 0.0;
            e.khi_i = 1; e.batch = nfull; e.info = info;
            HIPCHK(launch_gemm_f64(s, e));
        }
        const int64_t o = nfull * S;
        const int64_t h2 = n - o - hh;
        if (h2 > 0) {
            GemmDesc d{};
            d.A = L + (o + hh) + o * ldl; d.lda = ldl;
            d.B = W + o * (1 + ldw); d.ldb = ldw;
            d.C = T; d.ldc = h2;
            d.M = h2; d.N = hh; d.K = hh; d.alpha = 1.0; d.beta = 0.0;
            d.klo_j = 1; d.batch = 1; d.info = info;
            HIPCHK(launch_gemm_f64(s, d));
            GemmDesc e{};
            e.A = W + (o + hh) * (1 + ldw); e.lda = ldw;
            e.B = T; e.ldb = h2;
            e.C = W + (o + hh) + o * ldw; e.ldc = ldw;
            e.M = h2; e.N = hh; e.K = h2; e.alpha = -1.0; e.beta = 0.0;
            e.khi_i = 1; e.batch = 1; e.info = info;
            HIPCHK(launch_gemm_f64(s, e));
        }
    }
    return GP_OK;
}

// W = L^{-1} (lower) and V = W^T (upper), both n x n with ld n, by recursive
// doubling on the NT MFMA kernel (products of the form A B^T with both
// operands column-major).  Per level and node, whose two halves are already
// inverted (W11, W22 and their transposes V11, V22):
//   Tt  = V11 L21^T      (= (L21 W11)^T, h x h2; V11 is zero left of its diagonal)
//   W21 = -W22 Tt^T      (W22 is zero right of its diagonal)
//   V12 = W21^T
// T holds trtri_tmp_elems(n) doubles.
int trtri_nt(hipStream_t s, int64_t n, const double *L, int64_t ldl, const double *dinv, double *W, double *V,
             double *T, const int32_t *info) {
    const int64_t ld = n;
    HIPCHK(launch_fill(s, W, sizeof(double) * (size_t)n * (size_t)n));
    HIPCHK(launch_fill(s, V, sizeof(double) * (size_t)n * (size_t)n));
    HIPCHK(launch_place_dinv(s, n, dinv, W, ld, 0));
    HIPCHK(launch_place_dinv(s, n, dinv, V, ld, 1));
    for (int64_t S = 2 * DB; S / 2 < n; S *= 2) {
        const int64_t h = S / 2;
        auto level = [&](int64_t o, int64_t h2, int64_t batch) -> hipError_t {
            GemmDesc a{};
            a.A = V + o * (1 + ld); a.lda = ld; a.sA = S * (1 + ld);
            a.B = L + (o + h) + o * ldl; a.ldb = ldl; a.sB = S * (1 + ldl);
            a.C = T; a.ldc = h; a.sC = h * h2;
            a.M = h; a.N = h2; a.K = h; a.alpha = 1.0; a.beta = 0.0;
            a.klo_i = 1; a.batch = batch; a.info = info;
            hipError_t e = launch_gemm_nt_dma(s, a);
            if (e != hipSuccess) return e;
            GemmDesc b{};
            b.A = W + (o + h) * (1 + ld); b.lda = ld; b.sA = S * (1 + ld);
            b.B = T; b.ldb = h; b.sB = h * h2;
            b.C = W + (o + h) + o * ld; b.ldc = ld; b.sC = S * (1 + ld);
            b.M = h2; b.N = h; b.K = h2; b.alpha = -1.0; b.beta = 0.0;
            b.khi_i = 1; b.batch = batch; b.info = info;
            e = launch_gemm_nt_dma(s, b);
            if (e != hipSuccess) return e;
            return launch_transpose_copy(s, h2, h, W + (o + h) + o * ld, ld, S * (1 + ld), V + o + (o + h) * ld, ld,
                                         S * (1 + ld), batch);
        };
        const int64_t nfull = n / S;
        if (nfull > 0) HIPCHK(level(0, h, nfull));
        const int64_t o = nfull * S, h2 = n - o - h;
        if (h2 > 0) HIPCHK(level(o, h2, 1));
    }
    return GP_OK;
}

// CU masks: bit c of word c / 32 enables compute unit c.  The reserved units
// are spread evenly over the index range so that each XCD keeps the same
// number of units for the trailing update.
static int make_masked_streams(gp_handle_t h, int reserve) {
    if (h->masked_for == reserve && h->main_cu) return GP_OK;
    if (h->main_cu) {
        hipStreamSynchronize(h->main_cu);
        hipStreamSynchronize(h->side_cu);
        hipStreamDestroy(h->main_cu);
        hipStreamDestroy(h->side_cu);
        h->main_cu = h->side_cu = nullptr;
        h->masked_for = 0;
    }
    const int ncu = h->num_cu;
    if (reserve <= 0 || reserve >= ncu / 2) return GP_OK;
    std::vector<uint32_t> all((size_t)(ncu + 31) / 32, 0u), rest;
    for (int c = 0; c < ncu; ++c) all[(size_t)c / 32] |= 1u << (c % 32);
    rest = all;
    for (int r = 0; r < reserve; ++r) {
        const int c = reserved_cu(r, reserve, ncu);
        rest[(size_t)c / 32] &= ~(1u << (c % 32));
    }
    if (hipExtStreamCreateWithCUMask(&h->main_cu, (uint32_t)rest.size(), rest.data()) != hipSuccess)
        return GP_ERR_HIP;
    if (hipExtStreamCreateWithCUMask(&h->side_cu, (uint32_t)all.size(), all.data()) != hipSuccess) {
        hipStreamDestroy(h->main_cu);
        h->main_cu = nullptr;
        return GP_ERR_HIP;
    }
    h->masked_for = reserve;
    return GP_OK;
}

// Right-looking blocked Cholesky (Section 2.1): per panel of NB columns,
// (1) the diagonal block A11 is factored in 64-column steps restricted to the
// block (one-wave factor + inverse of each 64 x 64 block, the block's rows
// below it multiplied by that inverse, update of the rest of the block), then
// inverted, V = L11^{-1}; (2) the rows below get L21 = A21 V^T as one product
// (A21 copied to pbuf first); (3) the trailing matrix gets A22 -= L21 L21^T.
// With lookahead, step (3) is split: the columns of the next panel first,
// then the next panel's step (1) on the side stream while the rest of (3)
// runs on the main one.
int potrf_impl(gp_handle_t h, gp_prec_t prec, int64_t n, double *A, int64_t lda, int32_t *info,
               double *dinv, const PanelBufs &pb) {
    hipStream_t user = h->stream;
    const PotrfChoice ch = potrf_choice(h, prec, n);
    HIPCHK(launch_set_info(user, info));
    if (n <= 0) return GP_OK;
    auto width = [&](int64_t c) { return panel_at(ch, n, c); };

    hipStream_t s = user, side = h->side;
    const bool la = h->opt.lookahead && n > width(0);
    // workgroups of the trailing update that run at once: two per compute
    // unit of the main stream
    const int main_cus = h->num_cu - (la ? ch.panel_cus : 0);
    const int slots = 2 * (main_cus > 0 ? main_cus : 1);
    if (la && ch.panel_cus > 0) {
        int rc = make_masked_streams(h, ch.panel_cus);
        if (rc) return rc;
        if (h->main_cu) {
            s = h->main_cu;
            side = h->side_cu;
            HIPCHK(hipEventRecord(h->ev_in, user));
            HIPCHK(hipStreamWaitEvent(s, h->ev_in, 0));
        }
    }

    // (1) for the panel [c0, c1)
    auto diag_block = [&](hipStream_t st, int64_t c0, int64_t c1) -> int {
        if (h->opt.fused_panel && pb.pflags && c1 - c0 <= DB * PF_MAXB && (c1 == n || pb.vinv)) {
            HIPCHK(launch_panel_chol(st, A + c0 + c0 * lda, lda, (int)(c1 - c0), dinv + (c0 / DB) * DB * DB,
                                     c1 < n ? pb.vinv : nullptr, c1 - c0, pb.pflags, info, c0,
                                     h->opt.fail_inject & 1));
            return GP_OK;
        }
        for (int64_t d = c0; d < c1; d += DB) {
            const int jb = (int)((n - d) < DB ? (n - d) : DB);
            double *W = dinv + (d / DB) * DB * DB;
            HIPCHK(launch_diag_potrf(st, A + d + d * lda, lda, jb, W, info, d));
            const int64_t Mi = c1 - d - jb;
            if (Mi > 0) {
                HIPCHK(launch_panel_solve(st, A + (d + jb) + d * lda, lda, W, Mi, jb, info));
                HIPCHK(launch_syrk_lower(st, GP_FP64, -1, A + (d + jb) + d * lda, lda,
                                         A + (d + jb) + (d + jb) * lda, lda, Mi, Mi, jb, info, 2));
            }
        }
        if (c1 < n) {
            int rc = trtri_lower(st, c1 - c0, A + c0 + c0 * lda, lda, dinv + (c0 / DB) * DB * DB, pb.vinv,
                                 pb.vtmp, info);
            if (rc) return rc;
        }
        return GP_OK;
    };
    // (2) for the panel [c0, c1), c1 < n
    auto below = [&](hipStream_t st, int64_t c0, int64_t c1) -> int {
        // pbuf's leading dimension is even, with a spare row for an odd M, so
        // that the product takes the 16-byte copies
        const int64_t M = n - c1, K = c1 - c0, ldq = M + (M & 1);
        HIPCHK(launch_copy2d(st, M, K, A + c1 + c0 * lda, lda, pb.pbuf, ldq));
        GemmDesc g{};
        g.A = pb.pbuf; g.lda = ldq; g.odd_rows = 1;
        g.B = pb.vinv; g.ldb = K; g.tb = 1;  // op(B)[k, j] = V[j, k], zero for k > j
        g.khi_j = 1;
        g.C = A + c1 + c0 * lda; g.ldc = lda;
        g.M = M; g.N = K; g.K = K; g.alpha = 1.0; g.beta = 0.0;
        g.batch = 1; g.info = info;
        HIPCHK(launch_gemm_nt_dma(st, g));
        return GP_OK;
    };

    int rc = 0;
    {
        const int64_t c1 = width(0);
        if ((rc = diag_block(s, 0, c1))) return rc;
        if (c1 < n && (rc = below(s, 0, c1))) return rc;
    }
    // panel [c0, c1) is factored; its trailing update runs while the next
    // panel [c1, c2) is factored on the side stream
    for (int64_t c0 = 0, c1 = width(0); c1 < n; c0 = c1, c1 += width(c1)) {
        const int64_t K = c1 - c0;
        const int64_t c2 = c1 + width(c1);
        const bool packed = prec != GP_FP64 && pb.qbuf && K % 32 == 0;
        if (packed) HIPCHK(launch_pack_panel(s, prec, A + c1 + c0 * lda, lda, n - c1, K, pb.qbuf, h->opt.bf16_split));
        // trailing update of rows / columns [r0, r1) x [r0, ...) from panel rows r0 ..
        auto update = [&](int64_t r0, int64_t ncols) -> hipError_t {
            const int64_t M = n - r0;
            if (packed)
                return trailing_packed(h, s, prec, A + r0 + c0 * lda, lda, pb.qbuf, n - c1, r0 - c1,
                                       A + r0 + r0 * lda, lda, M, ncols, K, info);
            return trailing(h, s, prec, A + r0 + c0 * lda, lda, A + r0 + r0 * lda, lda, M, ncols, K, info, ch.slab);
        };
        if (la) {
            // columns of the next panel first; then, on the side stream, its
            // diagonal block and the rows below it (columns c1 .. c2, which
            // the rest of this trailing update does not touch).  In FP64 the
            // two updates are the parts of one split tile order, the first
            // topped up with tiles of the rest to fill its last round.
            const double *Pn = A + c1 + c0 * lda;
            double *Ct = A + c1 + c1 * lda;
            const bool split = !packed && prec == GP_FP64 && c2 < n &&
                               launch_syrk_split(s, Pn, lda, Ct, lda, n - c1, c2 - c1, K, info, -1, slots,
                                                 ch.slab) == hipSuccess;
            HIPCHK(split ? trailing_part(h, s, Pn, lda, Ct, lda, n - c1, c2 - c1, K, info, ch.slab, slots, 0)
                         : update(c1, c2 - c1));
            HIPCHK(hipEventRecord(h->ev_cols, s));
            HIPCHK(hipStreamWaitEvent(side, h->ev_cols, 0));
            if ((rc = diag_block(side, c1, c2))) return rc;
            if (c2 < n && (rc = below(side, c1, c2))) return rc;
            HIPCHK(hipEventRecord(h->ev_panel, side));
            if (c2 < n)
                HIPCHK(split ? trailing_part(h, s, Pn, lda, Ct, lda, n - c1, c2 - c1, K, info, ch.slab, slots, 1)
                             : update(c2, n - c2));
            HIPCHK(hipStreamWaitEvent(s, h->ev_panel, 0));
        } else {
            HIPCHK(update(c1, n - c1));
            if ((rc = diag_block(s, c1, c2))) return rc;
            if (c2 < n && (rc = below(s, c1, c2))) return rc;
        }
    }
    if (s != user) {
        HIPCHK(hipEventRecord(h->ev_out, s));
        HIPCHK(hipStreamWaitEvent(user, h->ev_out, 0));
    }
    return GP_OK;
}


// ---- triangular solve with many right-hand sides ----------------------------
// Right-looking by 64-row blocks with the stored diagonal inverses: each block
// row is multiplied by its inverse (out of place through tmp), then the rows
// below (NOTRANS) or above (TRANS) are updated; the updates are gathered per
// 256-row band so the large product runs with K = 256 on the matrix cores.
int trsm_impl(gp_handle_t h, int trans, int64_t n, int64_t nrhs, const double *L, int64_t ldl, double *B,
              int64_t ldb, const double *dinv, double *tmp, const int32_t *info) {
    hipStream_t s = h->stream;
    const int64_t NBT = 256;
    auto gemm = [&](int ta, const double *A, int64_t lda, const double *Bm, int64_t ldbm, double *C, int64_t ldc,
                    int64_t M, int64_t N, int64_t K, double alpha, double beta) -> hipError_t {
        GemmDesc d{};
        d.A = A; d.lda = lda; d.B = Bm; d.ldb = ldbm; d.C = C; d.ldc = ldc;
        d.M = M; d.N = N; d.K = K; d.alpha = alpha; d.beta = beta;
        d.ta = ta; d.tb = 0; d.lower = 0; d.batch = 1; d.info = info;
        return launch_gemm_f64(s, d);
    };
    if (n <= 0 || nrhs <= 0) return GP_OK;
    if (!trans) {
        for (int64_t kb0 = 0; kb0 < n; kb0 += NBT) {
            const int64_t kb1 = (kb0 + NBT < n) ? kb0 + NBT : n;
            for (int64_t d = kb0; d < kb1; d += DB) {
                const int64_t jb = (n - d) < DB ? (n - d) : DB;
                HIPCHK(launch_copy2d(s, jb, nrhs, B + d, ldb, tmp, DB));
                HIPCHK(gemm(0, dinv + (d / DB) * DB * DB, DB, tmp, DB, B + d, ldb, jb, nrhs, jb, 1.0, 0.0));
                if (d + jb < kb1)
                    HIPCHK(gemm(0, L + (d + jb) + d * ldl, ldl, B + d, ldb, B + d + jb, ldb, kb1 - d - jb, nrhs, jb,
                                -1.0, 1.0));
            }
            if (kb1 < n)
                HIPCHK(gemm(0, L + kb1 + kb0 * ldl, ldl, B + kb0, ldb, B + kb1, ldb, n - kb1, nrhs, kb1 - kb0, -1.0,
                            1.0));
        }
    } else {
        const int64_t nblk = nblocks(n);
        int64_t kb1 = n;
        while (kb1 > 0) {
            const int64_t kb0 = ((kb1 - 1) / NBT) * NBT;
            for (int64_t b = (kb1 - 1) / DB; b >= kb0 / DB; --b) {
                const int64_t d = b * DB;
                const int64_t jb = (n - d) < DB ? (n - d) : DB;
                HIPCHK(launch_copy2d(s, jb, nrhs, B + d, ldb, tmp, DB));
                HIPCHK(gemm(1, dinv + b * DB * DB, DB, tmp, DB, B + d, ldb, jb, nrhs, jb, 1.0, 0.0));
                if (d > kb0)
                    HIPCHK(gemm(1, L + d + kb0 * ldl, ldl, B + d, ldb, B + kb0, ldb, d - kb0, nrhs, jb, -1.0, 1.0));
            }
            if (kb0 > 0)
                HIPCHK(gemm(1, L + kb0, ldl, B + kb0, ldb, B, ldb, kb0, nrhs, kb1 - kb0, -1.0, 1.0));
            kb1 = kb0;
            (void)nblk;
        }
    }
    return GP_OK;
}

// ---- right-side solve Y <- Y L^{-T} (Y: m x n, column-major, ld m) --------
// Right-looking by KRIGE_BAND-column bands on the NT matrix-core kernel (both
// operands column-major with contiguous rows, as its direct-to-LDS copies
// need).  The inverses W_B of all full diagonal bands come from one batched
// launch (Wb, (n / KRIGE_BAND) * KRIGE_BAND^2 doubles; flags as for the
// panel kernel); band B then becomes Y_B W_B^T in one product (triangular
// K-range skipped) and every band to its right takes Y_R -= Y_B L_RB^T.  A
// partial last band (or Wb == nullptr) is solved by 64-column blocks with
// the diagonal-block inverses in dinv.  tmp holds m x KRIGE_BAND doubles.
int trsm_right_lt(hipStream_t s, int64_t n, int64_t m, const double *L, int64_t ldl, double *Y, const double *dinv,
                  double *tmp, double *Wb, int *flags, const int32_t *info) {
    const int64_t NBT = KRIGE_BAND;
    auto nt = [&](const double *A, int64_t lda, const double *B, int64_t ldb, double *C, int64_t M, int64_t N,
                  int64_t K, double alpha, double beta, int khi_j) -> hipError_t {
        GemmDesc d{};
        d.A = A; d.lda = lda; d.B = B; d.ldb = ldb; d.C = C; d.ldc = m;
        d.M = M; d.N = N; d.K = K; d.alpha = alpha; d.beta = beta;
        d.ta = 0; d.tb = 1; d.khi_j = khi_j; d.batch = 1; d.info = info;
        return launch_gemm_nt_dma(s, d);
    };
    if (n <= 0 || m <= 0) return GP_OK;
    // inverses of all full diagonal bands in one launch
    if (Wb && n >= NBT) HIPCHK(launch_block_trtri(s, L, ldl, (int)NBT, n / NBT, dinv, Wb, flags, info));
    for (int64_t kb0 = 0; kb0 < n; kb0 += NBT) {
        const int64_t kb1 = (kb0 + NBT < n) ? kb0 + NBT : n;
        if (Wb && kb1 - kb0 == NBT) {
            // Y_B = Y_B W_B^T (W_B lower: op(B)[k, j] = W_B[j, k], zero for k > j)
            HIPCHK(launch_copy2d(s, m, NBT, Y + kb0 * m, m, tmp, m));
            HIPCHK(nt(tmp, m, Wb + (kb0 / NBT) * NBT * NBT, NBT, Y + kb0 * m, m, NBT, NBT, 1.0, 0.0, 1));
        } else {
            for (int64_t d = kb0; d < kb1; d += DB) {
                const int64_t jb = (n - d) < DB ? (n - d) : DB;
                HIPCHK(launch_copy2d(s, m, jb, Y + d * m, m, tmp, m));
                // X_d = tmp Winv_d^T
                HIPCHK(nt(tmp, m, dinv + (d / DB) * DB * DB, DB, Y + d * m, m, jb, jb, 1.0, 0.0, 0));
                if (d + jb < kb1)
                    HIPCHK(nt(Y + d * m, m, L + (d + jb) + d * ldl, ldl, Y + (d + jb) * m, m, kb1 - d - jb, jb, -1.0,
                              1.0, 0));
            }
        }
        if (kb1 < n)
            HIPCHK(nt(Y + kb0 * m, m, L + kb1 + kb0 * ldl, ldl, Y + kb1 * m, m, n - kb1, kb1 - kb0, -1.0, 1.0, 0));
    }
    return GP_OK;
}

// ---- C^{-1} = L^{-T} L^{-1} (lower) from the factor ------------------------
// W = L^{-1} by recursive doubling on 64-blocks (Winv of each diagonal block
// from the factorisation, then per level W21 = -W22 (L21 W11)), followed by
// C^{-1} = W^T W restricted to the lower triangle (K runs from the tile row,
// as rows of W above it are zero).  Both steps run on the matrix cores.
int cinv_impl(gp_handle_t h, int64_t n, double *C, int64_t ldc, const double *dinv, double *W, double *V,
              double *T, const int32_t *info) {
    hipStream_t s = h->stream;
    int rc = trtri_nt(s, n, C, ldc, dinv, W, V, T, info);
    if (rc) return rc;
    // C^{-1} = W^T W = V V^T (lower triangle), V zero left of its diagonal:
    // a SYRK whose tile rows i0.. start at k = i0
    HIPCHK(launch_syrk_dma(s, V, n, C, ldc, n, n, 1.0, 0.0, 1, info));
    return GP_OK;
}


// ---- one likelihood evaluation (optionally with gradient) -------------------
// FP64: C(theta) -> L -> z = L^{-1} b -> (logdet, q) -> alpha = L^{-T} z.
// Mixed: the points are optionally taken in Morton order, the trailing
// updates run in low precision, then x = C^{-1} b is refined against the FP64
// covariance regenerated from the points (matrix-free residual) and
// q = b^T x; the log-determinant comes from the mixed factor.
int loglik_core(gp_handle_t h, gp_op_t op, gp_theta_t th, gp_prec_t prec, int64_t n, int32_t dim,
                const double *X, const double *y, const double *mu, double *C, int64_t ldc, double *out3,
                double *grad3, double *alpha_dev, int32_t *info, double *ir, void *ws) {
    const Layout lay = layout(h, op, n, 0, prec);
    hipStream_t s = h->stream;
    const CovParams cp = cov_params(th, dim);
    const int ngrad = th.kind == GP_SEP_MATERN2 ? 4 : 3;
    double *dinv = at<double>(ws, lay.dinv);
    int *sync = at<int>(ws, lay.sync);
    double *z = at<double>(ws, lay.z);
    double *x = at<double>(ws, lay.vec2);
    double *b = at<double>(ws, lay.vec3);
    const bool mixed = prec != GP_FP64;
    const double *Xe = X, *ye = y, *mue = mu;
    int64_t *perm = nullptr;
    if (mixed && h->opt.reorder && n > 1) {
        perm = at<int64_t>(ws, lay.perm);
        double *Xp = at<double>(ws, lay.xp), *yp = at<double>(ws, lay.yp), *mp = at<double>(ws, lay.mup);
        HIPCHK(launch_morton(s, n, dim, X, perm, at<uint64_t>(ws, lay.keys), at<double>(ws, lay.box)));
        HIPCHK(launch_gather_points(s, n, dim, perm, X, y, mu, Xp, yp, mp));
        Xe = Xp;
        ye = yp;
        mue = mu ? mp : nullptr;
    }
    HIPCHK(launch_cov_lower(s, cp, n, Xe, C, ldc, nullptr));
    int rc = potrf_impl(h, prec, n, C, ldc, info, dinv, panel_bufs(ws, lay));
    if (rc) return rc;
    const int inj = (h->opt.fail_inject >> 1) & 1;
    // every solve is followed by its status check: a wait that gave up turns info into -1
    auto solve = [&](int trans, double *v, const int32_t *skip) -> hipError_t {
        hipError_t e = launch_trsv(s, trans, C, ldc, v, n, dinv, sync, skip, inj);
        if (e == hipSuccess && n > 0) e = launch_solve_status(s, sync, info);
        return e;
    };
    HIPCHK(launch_sub_mu(s, n, ye, mue, b));
    HIPCHK(launch_copy_vec(s, n, b, z));
    HIPCHK(solve(0, z, info));
    HIPCHK(launch_loglik_reduce(s, n, C, ldc, z, out3, info, nullptr));  // solve failures are in info
    const bool need_x = alpha_dev || grad3 || mixed;
    if (need_x) {
        HIPCHK(launch_copy_vec(s, n, z, x));
        HIPCHK(solve(1, x, info));
    }
    if (mixed) {
        double *res = at<double>(ws, lay.vec4), *dv = at<double>(ws, lay.vec5);
        double *state = at<double>(ws, lay.irst);
        int32_t *done = reinterpret_cast<int32_t *>(state + 8);
        HIPCHK(launch_ir_init(s, n, b, state, done, info));
        const int maxit = h->opt.ir_max_iter;
        for (int it = 0; it <= maxit; ++it) {
            HIPCHK(launch_resid_matfree(s, cp, n, Xe, b, x, res, at<double>(ws, lay.big2), done));
            HIPCHK(launch_ir_check(s, n, res, state, done, it == maxit, h->opt.ir_tol));
            if (it == maxit) break;
            HIPCHK(launch_copy_skip(s, n, res, dv, done));
            HIPCHK(solve(0, dv, done));
            HIPCHK(solve(1, dv, done));
            HIPCHK(launch_axpy_skip(s, n, dv, x, done));
        }
        HIPCHK(launch_ir_finish(s, n, b, x, state, out3, ir, info));
    }
    if (alpha_dev) {
        if (perm) HIPCHK(launch_scatter_vec(s, n, perm, x, alpha_dev));
        else HIPCHK(launch_copy_vec(s, n, x, alpha_dev));
    }
    if (grad3) {
        if (n > 0) {
            rc = cinv_impl(h, n, C, ldc, dinv, at<double>(ws, lay.big1), at<double>(ws, lay.big4),
                           at<double>(ws, lay.big3), info);
            if (rc) return rc;
        }
        double *part = at<double>(ws, lay.part);
        HIPCHK(launch_grad_contract(s, cp, n, Xe, C, ldc, x, part, GRAD_PARTS, info));
        HIPCHK(launch_grad_finish(s, GRAD_PARTS, part, grad3, ngrad, info));
    }
    // a failure anywhere above (info != 0): NaN scalars, alpha and gradient
    HIPCHK(launch_fail_outputs(s, n, info, out3, alpha_dev, grad3, ngrad));
    return GP_OK;
}

// ---- products with the lower factor and the prediction covariance -----------
// out = beta out + L E (L m x m lower, only its lower triangle read; E m x r,
// ld lde): the blocks strictly below the 128-row diagonal blocks on the
// matrix cores (E transposed into Et, r x m, so both operands stream rows),
// then the diagonal blocks by a small kernel that reads only their lower part.
int trmm_lower(hipStream_t s, int64_t m, int64_t r, const double *L, int64_t ldl, const double *E, int64_t lde,
               double *Et, double *out, int64_t ldo, double beta, const int32_t *info) {
    if (m <= 0 || r <= 0) return GP_OK;
    HIPCHK(launch_transpose_copy(s, m, r, E, lde, 0, Et, r, 0, 1));
    GemmDesc d{};
    d.A = L; d.lda = ldl; d.B = Et; d.ldb = r; d.C = out; d.ldc = ldo;
    d.M = m; d.N = r; d.K = m; d.alpha = 1.0; d.beta = beta;
    d.ta = 0; d.tb = 1; d.khi_i = 2; d.batch = 1; d.info = info;
    HIPCHK(launch_gemm_nt_dma(s, d));
    HIPCHK(launch_trmm_diag(s, m, r, L, ldl, E, lde, out, ldo, info));
    return GP_OK;
}

// The m new points against the n data points: Y = (L^{-1} C*)^T (m x n, ld m)
// and, if mean is non-null, mean_j = mu + c_j^T alpha (before the solve).
int cross_solve(hipStream_t s, const CovParams &cp, int64_t n, int64_t m, const double *X, const double *Xs,
                const double *L, int64_t ldl, const double *alpha, double mu, double *mean, void *ws,
                const Layout &lay) {
    double *Y = at<double>(ws, lay.big1);
    double *dinv = at<double>(ws, lay.dinv);
    HIPCHK(launch_diag_inv(s, L, ldl, n, dinv));
    HIPCHK(launch_cross_cov(s, cp, m, n, Xs, X, Y, m));  // Y(j, i) = sigma^2 k(|s_j - x_i| / rho)
    if (mean) HIPCHK(launch_rowreduce(s, 0, m, n, Y, m, alpha, mu, at<double>(ws, lay.big2), mean));
    return trsm_right_lt(s, n, m, L, ldl, Y, dinv, at<double>(ws, lay.part), lay.kw ? at<double>(ws, lay.kw) : nullptr,
                         at<int>(ws, lay.pflags), nullptr);
}

// S (lower, m x m) = C** (+ tau^2 I) - Y Y^T: the prior covariance of the new
// points less the part the data explain (nothing subtracted when n = 0).
int pred_cov(hipStream_t s, const CovParams &cp, int include_nugget, int64_t n, int64_t m, const double *Xs,
             const double *Y, double *S, int64_t lds) {
    CovParams pp = cp;
    if (!include_nugget) pp.t2 = 0.0;
    HIPCHK(launch_cov_lower(s, pp, m, Xs, S, lds, nullptr));
    if (n > 0) HIPCHK(launch_syrk_dma(s, Y, m, S, lds, m, n, -1.0, 1.0, 0, nullptr));
    return GP_OK;
}

}  // namespace

// ============================================================================
extern "C" {

const char *gp_strerror(int code) {
    if (code == GP_OK) return "success";
    if (code == GP_ERR_NONFINITE) return "non-finite scalar argument";
    if (code == GP_ERR_WS_TOO_SMALL) return "workspace smaller than gp_workspace_size()";
    if (code == GP_ERR_HIP) return "HIP runtime error";
    if (code == GP_ERR_NOT_SUPPORTED) return "option combination not supported";
    if (code == GP_ERR_BAD_HANDLE) return "invalid handle";
    if (code == GP_ERR_SCRATCH_LIMIT) return "problem needs more than the GP_SCRATCH_BYTES static workspace";
    if (code == GP_ERR_NO_CANDIDATE) return "no tuning candidate could be timed (each needs more workspace)";
    if (code == GP_ERR_IO) return "tuning table file could not be read or written";
    if (code < 0 && code > -100) return "invalid argument (index = -code)";
    return "unknown status";
}

static void default_options(gp_options_t *o) {
    memset(o, 0, sizeof(*o));
    o->nb = 0;  // automatic: see panel_width
    o->lookahead = 1;
    o->panel_cus = 0;
    o->band = 8;
    o->ir_max_iter = 20;
    o->ir_tol = 1e-10;
    o->reorder = 1;
    o->fused_panel = 1;
    o->batch_grid = 0;
    o->bf16_split = 1;
    o->batch_tile = 0;
    o->tail_nb = 0;
}

}  // extern "C"

// ---- static workspace of gp_loglik_noalloc ------------------------------------
// One array per device, part of this code object: it is allocated when the
// code object is loaded on a device and held until the process ends.  In host
// code `scratch` names a host-side shadow, never the device memory: kernels
// get the address hipGetSymbolAddress returns for the current device, looked
// up once per device at gp_create and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[GP_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Address of `scratch` on `dev` (the current device), looked up on the first
// call for that device; null if the lookup failed.
void *device_scratch(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[dev] = p;
        else (void)hipGetLastError();
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

int gp_create(gp_handle_t *h, void *stream) {
    if (!h) return -1;
    *h = nullptr;
    gp_handle_s *p = new (std::nothrow) gp_handle_s();
    if (!p) return GP_ERR_HIP;
    default_options(&p->opt);
    p->stream = (hipStream_t)stream;
    if (hipGetDevice(&p->device) != hipSuccess ||
        hipDeviceGetAttribute(&p->num_cu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess ||
        hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&p->band, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_band_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_band_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_cols, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_panel, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming) != hipSuccess) {
        if (p->side) hipStreamDestroy(p->side);
        if (p->band) hipStreamDestroy(p->band);
        if (p->ev_band_in) hipEventDestroy(p->ev_band_in);
        if (p->ev_band_out) hipEventDestroy(p->ev_band_out);
        if (p->ev_cols) hipEventDestroy(p->ev_cols);
        if (p->ev_panel) hipEventDestroy(p->ev_panel);
        if (p->ev_in) hipEventDestroy(p->ev_in);
        if (p->ev_out) hipEventDestroy(p->ev_out);
        delete p;
        return GP_ERR_HIP;
    }
    // the static workspace's address on this device (null if the lookup
    // failed: gp_loglik_noalloc then returns GP_ERR_HIP)
    p->scratch = device_scratch(p->device);
    {  // architecture name without its feature suffixes (gfx950:sramecc+:xnack- -> gfx950)
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
            size_t k = 0;
            while (k + 1 < sizeof p->arch && prop.gcnArchName[k] && prop.gcnArchName[k] != ':') {
                p->arch[k] = prop.gcnArchName[k];
                ++k;
            }
            p->arch[k] = 0;
        }
    }
    *h = p;
    return GP_OK;
}

int gp_profile(gp_handle_t h, int enable) {
    if (!ok_handle(h)) return -1;
    h->prof = enable ? 1 : 0;
    return GP_OK;
}

int gp_profile_read(gp_handle_t h, double *out4) {
    if (!ok_handle(h)) return -1;
    if (!out4) return -2;
    double ms = 0.0;
    for (size_t i = 0; i + 1 < h->prof_used; i += 2) {
        if (hipEventSynchronize(h->prof_ev[i + 1]) != hipSuccess) return GP_ERR_HIP;
        float t = 0.f;
        if (hipEventElapsedTime(&t, h->prof_ev[i], h->prof_ev[i + 1]) != hipSuccess) return GP_ERR_HIP;
        ms += t;
    }
    out4[0] = (double)h->prof_launches;
    out4[1] = ms;
    out4[2] = h->prof_flops;
    out4[3] = h->prof_bytes;
    h->prof_used = 0;
    h->prof_launches = 0;
    h->prof_flops = 0.0;
    h->prof_bytes = 0.0;
    return GP_OK;
}

int gp_destroy(gp_handle_t h) {
    if (!ok_handle(h)) return -1;
    for (hipEvent_t e : h->prof_ev) (void)hipEventDestroy(e);
    batch_staging_free(h->batch_staging);
    hipStreamSynchronize(h->side);
    hipStreamDestroy(h->side);
    hipStreamSynchronize(h->band);
    hipStreamDestroy(h->band);
    hipEventDestroy(h->ev_band_in);
    hipEventDestroy(h->ev_band_out);
    if (h->main_cu) {
        hipStreamSynchronize(h->main_cu);
        hipStreamSynchronize(h->side_cu);
        hipStreamDestroy(h->main_cu);
        hipStreamDestroy(h->side_cu);
    }
    hipEventDestroy(h->ev_cols);
    hipEventDestroy(h->ev_panel);
    hipEventDestroy(h->ev_in);
    hipEventDestroy(h->ev_out);
    h->magic = 0;
    delete h;
    return GP_OK;
}

int gp_set_stream(gp_handle_t h, void *stream) {
    if (!ok_handle(h)) return -1;
    h->stream = (hipStream_t)stream;
    return GP_OK;
}

int gp_set_options(gp_handle_t h, const gp_options_t *opt) {
    if (!ok_handle(h)) return -1;
    if (!opt) {
        default_options(&h->opt);
        return GP_OK;
    }
    if (opt->nb < 0 || opt->nb % DB != 0) return -2;
    if (opt->ir_max_iter < 0 || opt->band < -1 || opt->panel_cus < 0) return -2;
    if (opt->fused_panel != 0 && opt->fused_panel != 1) return -2;
    if (opt->batch_grid < -1) return -2;
    if (opt->fail_inject < 0 || opt->fail_inject > 3) return -2;
    if (opt->bf16_split != 0 && opt->bf16_split != 1) return -2;
    if (opt->syrk_slab != 0 && opt->syrk_slab != 8 && opt->syrk_slab != 16) return -2;
    if (opt->batch_tile != 0 && opt->batch_tile != 64 && opt->batch_tile != 128) return -2;
    if (opt->tail_nb < -1 || (opt->tail_nb > 0 && opt->tail_nb % DB != 0)) return -2;
    if (!(opt->ir_tol >= 0.0) || isinf(opt->ir_tol)) return GP_ERR_NONFINITE;
    h->opt = *opt;
    return GP_OK;
}

int gp_get_options(gp_handle_t h, gp_options_t *opt) {
    if (!ok_handle(h)) return -1;
    if (!opt) return -2;
    *opt = h->opt;
    return GP_OK;
}

int gp_workspace_size(gp_handle_t h, gp_op_t op, int64_t n, int64_t m, gp_prec_t prec, size_t *bytes) {
    if (!ok_handle(h)) return -1;
    if ((int)op < GP_OP_POTRF || (int)op > GP_OP_SIMULATE) return -2;
    if (n < 0) return -3;
    if (m < 0) return -4;
    if ((int)prec < GP_FP64 || (int)prec > GP_BF16_TRAIL) return -5;
    if (!bytes) return -6;
    *bytes = layout(h, op, n, m, prec).total;
    return GP_OK;
}

int gp_cov_build(gp_handle_t h, gp_theta_t th, int64_t n, int32_t dim, const double *X, double *C,
                 int64_t ldc) {
    if (!ok_handle(h)) return -1;
    if (int e = check_theta(th)) return e == 1 ? -2 : GP_ERR_NONFINITE;
    if (n < 0) return -3;
    if (bad_dim(th, dim)) return -4;
    if (n > 0 && !X) return -5;
    if (n > 0 && !C) return -6;
    if (ldc < (n > 1 ? n : 1)) return -7;
    HIPCHK(launch_cov_lower(h->stream, cov_params(th, dim), n, X, C, ldc, nullptr));
    return GP_OK;
}

int gp_cross_cov_build(gp_handle_t h, gp_theta_t th, int64_t n, int64_t m, int32_t dim, const double *X,
                       const double *Xs, double *Cs, int64_t ldcs) {
    if (!ok_handle(h)) return -1;
    if (int e = check_theta(th)) return e == 1 ? -2 : GP_ERR_NONFINITE;
    if (n < 0) return -3;
    if (m < 0) return -4;
    if (bad_dim(th, dim)) return -5;
    if (n > 0 && !X) return -6;
    if (m > 0 && !Xs) return -7;
    if (n > 0 && m > 0 && !Cs) return -8;
    if (ldcs < (n > 1 ? n : 1)) return -9;
    HIPCHK(launch_cross_cov(h->stream, cov_params(th, dim), n, m, X, Xs, Cs, ldcs));
    return GP_OK;
}

int gp_potrf(gp_handle_t h, gp_prec_t prec, int64_t n, double *A, int64_t lda, int32_t *info_dev,
             void *ws, size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if ((int)prec < GP_FP64 || (int)prec > GP_BF16_TRAIL) return -2;
    if (n < 0) return -3;
    if (n > 0 && !A) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (!info_dev) return -6;
    Layout L = layout(h, GP_OP_POTRF, n, 0, prec);
    if (!ws) return -7;
    if (ws_bytes < L.total) return GP_ERR_WS_TOO_SMALL;
    return potrf_impl(h, prec, n, A, lda, info_dev, at<double>(ws, L.dinv), panel_bufs(ws, L));
}

int gp_potrf_plan(gp_handle_t h, gp_prec_t prec, int64_t n, int32_t *nb, int32_t *panel_cus, int32_t *syrk_slab,
                  int32_t *tail_nb) {
    if (!ok_handle(h)) return -1;
    if (prec < GP_FP64 || prec > GP_BF16_TRAIL) return -2;
    if (n < 0) return -3;
    const PotrfChoice c = potrf_choice(h, prec, n);
    if (nb) *nb = (int32_t)c.nb;
    if (panel_cus) *panel_cus = c.panel_cus;
    if (syrk_slab) *syrk_slab = c.slab == 0 ? 16 : c.slab;
    if (tail_nb) *tail_nb = (int32_t)c.tail;
    return GP_OK;
}

int gp_tune_potrf(gp_handle_t h, gp_prec_t prec, int64_t n, double *A, int64_t lda, const int32_t *nb_cand,
                  int32_t n_nb, const int32_t *cu_cand, int32_t n_cu, int32_t *info_dev, double *ms_out, void *ws,
                  size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if ((int)prec < GP_FP64 || (int)prec > GP_BF16_TRAIL) return -2;
    if (n < 1) return -3;
    if (!A) return -4;
    if (lda < n) return -5;
    if (!nb_cand && n_nb > 0) return -6;
    if (n_nb < 1) return -7;
    for (int32_t i = 0; i < n_nb; ++i)
        if (nb_cand[i] <= 0 || nb_cand[i] % DB != 0) return -6;
    if (!cu_cand && n_cu > 0) return -8;
    if (n_cu < 1) return -9;
    for (int32_t i = 0; i < n_cu; ++i)
        if (cu_cand[i] < 0) return -8;
    if (!info_dev) return -10;
    if (!ws) return -12;
    hipStream_t s = h->stream;
    const gp_options_t saved = h->opt;
    double best = -1.0;
    gp_options_t best_opt = saved;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return GP_ERR_HIP;
    }
    int rc = GP_OK;
    h->tuning = 1;
    const int slabs[2] = {16, 8};
    for (int32_t a = 0; a < n_nb && rc == GP_OK; ++a) {
        for (int32_t b = 0; b < n_cu && rc == GP_OK; ++b) {
          double pair_best = -1.0;
          for (int sl = 0; sl < (prec == GP_FP64 ? 2 : 1) && rc == GP_OK; ++sl) {
            double ms = -1.0;
            h->opt = saved;
            h->opt.nb = nb_cand[a];
            h->opt.lookahead = 1;
            h->opt.panel_cus = cu_cand[b];
            h->opt.syrk_slab = slabs[sl];
            const Layout L = layout(h, GP_OP_POTRF, n, 0, prec);
            if (L.total <= ws_bytes) {
                for (int rep = 0; rep < 2 && rc == GP_OK; ++rep) {  // the first run also creates streams
                    if (launch_tune_fill(s, A, lda, n) != hipSuccess || hipEventRecord(e0, s) != hipSuccess) {
                        rc = GP_ERR_HIP;
                        break;
                    }
                    rc = potrf_impl(h, prec, n, A, lda, info_dev, at<double>(ws, L.dinv), panel_bufs(ws, L));
                    if (rc) break;
                    float t = 0.f;
                    int32_t info = 0;
                    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&t, e0, e1) != hipSuccess ||
                        hipMemcpy(&info, info_dev, sizeof info, hipMemcpyDeviceToHost) != hipSuccess) {
                        rc = GP_ERR_HIP;
                        break;
                    }
                    if (info != 0) {  // the test matrix is positive definite
                        rc = GP_ERR_HIP;
                        break;
                    }
                    ms = t;
                }
            }
            if (ms >= 0.0 && (pair_best < 0.0 || ms < pair_best)) pair_best = ms;
            if (ms >= 0.0 && (best < 0.0 || ms < best)) {
                best = ms;
                best_opt = h->opt;
            }
          }
          if (ms_out) ms_out[a * n_cu + b] = pair_best;
        }
    }
    h->tuning = 0;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) {
        h->opt = saved;
        return rc;
    }
    if (best < 0.0) {
        h->opt = saved;
        return GP_ERR_NO_CANDIDATE;
    }
    h->opt = best_opt;
    tune_store(h, TuneEntry{0, (int32_t)prec, size_bucket(n), (int32_t)best_opt.nb, best_opt.panel_cus,
                            best_opt.syrk_slab, 0});
    return GP_OK;
}

int gp_trsv(gp_handle_t h, gp_trans_t trans, int64_t n, const double *L, int64_t ldl, double *x, void *ws,
            size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (trans != GP_NOTRANS && trans != GP_TRANS) return -2;
    if (n < 0) return -3;
    if (n > 0 && !L) return -4;
    if (ldl < (n > 1 ? n : 1)) return -5;
    if (n > 0 && !x) return -6;
    Layout lay = layout(h, GP_OP_TRSV, n, 0, GP_FP64);
    if (!ws) return -7;
    if (ws_bytes < lay.total) return GP_ERR_WS_TOO_SMALL;
    if (n == 0) return GP_OK;
    double *dinv = at<double>(ws, lay.dinv);
    HIPCHK(launch_diag_inv(h->stream, L, ldl, n, dinv));
    HIPCHK(launch_trsv(h->stream, trans == GP_TRANS, L, ldl, x, n, dinv, at<int>(ws, lay.sync), nullptr));
    return GP_OK;
}

int gp_trsm(gp_handle_t h, gp_trans_t trans, int64_t n, int64_t nrhs, const double *L, int64_t ldl,
            double *B, int64_t ldb, void *ws, size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (trans != GP_NOTRANS && trans != GP_TRANS) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (n > 0 && !L) return -5;
    if (ldl < (n > 1 ? n : 1)) return -6;
    if (n > 0 && nrhs > 0 && !B) return -7;
    if (ldb < (n > 1 ? n : 1)) return -8;
    Layout lay = layout(h, GP_OP_TRSM, n, nrhs, GP_FP64);
    if (!ws) return -9;
    if (ws_bytes < lay.total) return GP_ERR_WS_TOO_SMALL;
    if (n == 0 || nrhs == 0) return GP_OK;
    double *dinv = at<double>(ws, lay.dinv);
    HIPCHK(launch_diag_inv(h->stream, L, ldl, n, dinv));
    return trsm_impl(h, trans == GP_TRANS, n, nrhs, L, ldl, B, ldb, dinv, at<double>(ws, lay.part), nullptr);
}

int gp_loglik(gp_handle_t h, gp_theta_t th, gp_prec_t prec, int64_t n, int32_t dim, const double *X,
              const double *y, const double *mu, double *C, int64_t ldc, double *out3_dev,
              double *alpha_dev, int32_t *info_dev, double *ir_dev, void *ws, size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (int e = check_theta(th)) return e == 1 ? -2 : GP_ERR_NONFINITE;
    if ((int)prec < GP_FP64 || (int)prec > GP_BF16_TRAIL) return -3;
    if (n < 0) return -4;
    if (bad_dim(th, dim)) return -5;
    if (n > 0 && !X) return -6;
    if (n > 0 && !y) return -7;
    if (n > 0 && !C) return -9;
    if (ldc < (n > 1 ? n : 1)) return -10;
    if (!out3_dev) return -11;
    if (!info_dev) return -13;
    Layout lay = layout(h, GP_OP_LOGLIK, n, 0, prec);
    if (!ws) return -15;
    if (ws_bytes < lay.total) return GP_ERR_WS_TOO_SMALL;
    return loglik_core(h, GP_OP_LOGLIK, th, prec, n, dim, X, y, mu, C, ldc, out3_dev, nullptr, alpha_dev,
                       info_dev, ir_dev, ws);
}

int gp_loglik_noalloc(gp_handle_t h, gp_theta_t th, gp_prec_t prec, int64_t n, int32_t dim, const double *X,
                      const double *y, const double *mu, double *C, int64_t ldc, double *out3_dev,
                      double *alpha_dev, int32_t *info_dev, double *ir_dev) {
    if (!ok_handle(h)) return -1;
    if (int e = check_theta(th)) return e == 1 ? -2 : GP_ERR_NONFINITE;
    if ((int)prec < GP_FP64 || (int)prec > GP_BF16_TRAIL) return -3;
    if (n < 0) return -4;
    if (bad_dim(th, dim)) return -5;
    if (n > 0 && !X) return -6;
    if (n > 0 && !y) return -7;
    if (n > 0 && !C) return -9;
    if (ldc < (n > 1 ? n : 1)) return -10;
    if (!out3_dev) return -11;
    if (!info_dev) return -13;
    // panel_cus > 0 would create CU-masked streams on first use
    if (potrf_choice(h, prec, n).panel_cus > 0) return GP_ERR_NOT_SUPPORTED;
    const Layout lay = layout(h, GP_OP_LOGLIK, n, 0, prec);
    if (lay.total > (size_t)GP_SCRATCH_BYTES) return GP_ERR_SCRATCH_LIMIT;
    if (!h->scratch) return GP_ERR_HIP;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device) return GP_ERR_HIP;
    return loglik_core(h, GP_OP_LOGLIK, th, prec, n, dim, X, y, mu, C, ldc, out3_dev, nullptr, alpha_dev,
                       info_dev, ir_dev, h->scratch);
}

int gp_loglik_grad(gp_handle_t h, gp_theta_t th, gp_prec_t prec, int64_t n, int32_t dim, const double *X,
                   const double *y, const double *mu, double *C, int64_t ldc, double *out3_dev,
                   double *grad3_dev, double *alpha_dev, int32_t *info_dev, double *ir_dev, void *ws,
                   size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (int e = check_theta(th)) return e == 1 ? -2 : GP_ERR_NONFINITE;
    if ((int)prec < GP_FP64 || (int)prec > GP_BF16_TRAIL) return -3;
    if (n < 0) return -4;
    if (bad_dim(th, dim)) return -5;
    if (n > 0 && !X) return -6;
    if (n > 0 && !y) return -7;
    if (n > 0 && !C) return -9;
    if (ldc < (n > 1 ? n : 1)) return -10;
    if (!out3_dev) return -11;
    if (!grad3_dev) return -12;
    if (!info_dev) return -14;
    Layout lay = layout(h, GP_OP_LOGLIK_GRAD, n, 0, prec);
    if (!ws) return -16;
    if (ws_bytes < lay.total) return GP_ERR_WS_TOO_SMALL;
    return loglik_core(h, GP_OP_LOGLIK_GRAD, th, prec, n, dim, X, y, mu, C, ldc, out3_dev, grad3_dev, alpha_dev,
                       info_dev, ir_dev, ws);
}

int gp_krige(gp_handle_t h, gp_theta_t th, int64_t n, int64_t m, int32_t dim, const double *X,
             const double *Xs, const double *L, int64_t ldl, const double *alpha, double mu,
             double *mean_dev, double *var_dev, int32_t include_nugget, void *ws, size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (int e = check_theta(th)) return e == 1 ? -2 : GP_ERR_NONFINITE;
    if (n < 0) return -3;
    if (m < 0) return -4;
    if (bad_dim(th, dim)) return -5;
    if (n > 0 && !X) return -6;
    if (m > 0 && !Xs) return -7;
    if (n > 0 && !L) return -8;
    if (ldl < (n > 1 ? n : 1)) return -9;
    if (n > 0 && !alpha) return -10;
    if (!isfinite(mu)) return GP_ERR_NONFINITE;
    if (m > 0 && !mean_dev) return -12;
    if (m > 0 && !var_dev) return -13;
    Layout lay = layout(h, GP_OP_KRIGE, n, m, GP_FP64);
    if (!ws) return -15;
    if (ws_bytes < lay.total) return GP_ERR_WS_TOO_SMALL;
    if (m == 0) return GP_OK;
    hipStream_t s = h->stream;
    const CovParams cp = cov_params(th, dim);
    const double base_var = cp.s2 + (include_nugget ? cp.t2 : 0.0);
    double *Y = at<double>(ws, lay.big1);  // Y = C*^T: m x n, ld m
    double *partials = at<double>(ws, lay.big2);
    if (n == 0) {
        HIPCHK(launch_rowreduce(s, 0, m, 0, Y, m, nullptr, mu, partials, mean_dev));
        HIPCHK(launch_rowreduce(s, 1, m, 0, Y, m, nullptr, base_var, partials, var_dev));
        return GP_OK;
    }
    double *dinv = at<double>(ws, lay.dinv);
    HIPCHK(launch_diag_inv(s, L, ldl, n, dinv));
    HIPCHK(launch_cross_cov(s, cp, m, n, Xs, X, Y, m));  // Y(j, i) = sigma^2 k(|s_j - x_i| / rho)
    HIPCHK(launch_rowreduce(s, 0, m, n, Y, m, alpha, mu, partials, mean_dev));
    int rc = trsm_right_lt(s, n, m, L, ldl, Y, dinv, at<double>(ws, lay.part), lay.kw ? at<double>(ws, lay.kw) : nullptr,
                           at<int>(ws, lay.pflags), nullptr);  // rows of L^{-1} C*, transposed
    if (rc) return rc;
    HIPCHK(launch_rowreduce(s, 1, m, n, Y, m, nullptr, base_var, partials, var_dev));
    return GP_OK;
}

int gp_krige_cov(gp_handle_t h, gp_theta_t th, int64_t n, int64_t m, int32_t dim, const double *X,
                 const double *Xs, const double *L, int64_t ldl, int32_t include_nugget, double *S, int64_t lds,
                 void *ws, size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (int e = check_theta(th)) return e == 1 ? -2 : GP_ERR_NONFINITE;
    if (n < 0) return -3;
    if (m < 0) return -4;
    if (bad_dim(th, dim)) return -5;
    if (n > 0 && !X) return -6;
    if (m > 0 && !Xs) return -7;
    if (n > 0 && !L) return -8;
    if (ldl < (n > 1 ? n : 1)) return -9;
    if (include_nugget != 0 && include_nugget != 1) return -10;
    if (m > 0 && !S) return -11;
    if (lds < (m > 1 ? m : 1)) return -12;
    Layout lay = layout(h, GP_OP_KRIGE_COV, n, m, GP_FP64);
    if (!ws) return -13;
    if (ws_bytes < lay.total) return GP_ERR_WS_TOO_SMALL;
    if (m == 0) return GP_OK;
    hipStream_t s = h->stream;
    const CovParams cp = cov_params(th, dim);
    if (n > 0) {
        int rc = cross_solve(s, cp, n, m, X, Xs, L, ldl, nullptr, 0.0, nullptr, ws, lay);
        if (rc) return rc;
    }
    return pred_cov(s, cp, include_nugget, n, m, Xs, n > 0 ? at<double>(ws, lay.big1) : nullptr, S, lds);
}

int gp_trmm(gp_handle_t h, int64_t n, int64_t nrhs, const double *L, int64_t ldl, const double *B, int64_t ldb,
            double *out, int64_t ldo, void *ws, size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    if (n > 0 && !L) return -4;
    if (ldl < (n > 1 ? n : 1)) return -5;
    if (n > 0 && nrhs > 0 && !B) return -6;
    if (ldb < (n > 1 ? n : 1)) return -7;
    if (n > 0 && nrhs > 0 && !out) return -8;
    if (ldo < (n > 1 ? n : 1)) return -9;
    Layout lay = layout(h, GP_OP_TRMM, n, nrhs, GP_FP64);
    if (!ws) return -10;
    if (ws_bytes < lay.total) return GP_ERR_WS_TOO_SMALL;
    return trmm_lower(h->stream, n, nrhs, L, ldl, B, ldb, at<double>(ws, lay.et), out, ldo, 0.0, nullptr);
}

int gp_simulate(gp_handle_t h, gp_theta_t th, int64_t n, int64_t m, int32_t dim, const double *X, const double *Xs,
                const double *L, int64_t ldl, const double *alpha, double mu, int32_t include_nugget, int64_t nreal,
                const double *eps, int64_t ldeps, double *out, int64_t ldo, double *S, int64_t lds, int32_t *info_dev,
                void *ws, size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (int e = check_theta(th)) return e == 1 ? -2 : GP_ERR_NONFINITE;
    if (n < 0) return -3;
    if (m < 0) return -4;
    if (bad_dim(th, dim)) return -5;
    if (n > 0 && !X) return -6;
    if (m > 0 && !Xs) return -7;
    if (n > 0 && !L) return -8;
    if (ldl < (n > 1 ? n : 1)) return -9;
    if (n > 0 && !alpha) return -10;
    if (!isfinite(mu)) return GP_ERR_NONFINITE;
    if (include_nugget != 0 && include_nugget != 1) return -12;
    if (nreal < 0) return -13;
    if (m > 0 && nreal > 0 && !eps) return -14;
    if (ldeps < (m > 1 ? m : 1)) return -15;
    if (m > 0 && nreal > 0 && !out) return -16;
    if (ldo < (m > 1 ? m : 1)) return -17;
    if (m > 0 && !S) return -18;
    if (lds < (m > 1 ? m : 1)) return -19;
    if (!info_dev) return -20;
    Layout lay = layout(h, GP_OP_SIMULATE, n, m, GP_FP64);
    if (!ws) return -21;
    if (ws_bytes < lay.total) return GP_ERR_WS_TOO_SMALL;
    hipStream_t s = h->stream;
    if (m == 0) return launch_set_info(s, info_dev) == hipSuccess ? GP_OK : GP_ERR_HIP;
    const CovParams cp = cov_params(th, dim);
    double *mean = n > 0 ? at<double>(ws, lay.meanv) : nullptr;
    if (n > 0) {
        int rc = cross_solve(s, cp, n, m, X, Xs, L, ldl, alpha, mu, mean, ws, lay);
        if (rc) return rc;
    }
    int rc = pred_cov(s, cp, include_nugget, n, m, Xs, n > 0 ? at<double>(ws, lay.big1) : nullptr, S, lds);
    if (rc) return rc;
    PanelBufs pb;
    if (lay.vinv2) {
        pb.pbuf = at<double>(ws, lay.pbuf2);
        pb.vinv = at<double>(ws, lay.vinv2);
        pb.vtmp = at<double>(ws, lay.vtmp2);
    }
    pb.pflags = at<int>(ws, lay.pflags2);
    rc = potrf_impl(h, GP_FP64, m, S, lds, info_dev, at<double>(ws, lay.dinv2), pb);
    if (rc) return rc;
    HIPCHK(launch_zero_upper(s, m, S, lds));
    double *Et = at<double>(ws, lay.et);
    for (int64_t r0 = 0; r0 < nreal; r0 += SIM_CHUNK) {
        const int64_t rc2 = nreal - r0 < SIM_CHUNK ? nreal - r0 : SIM_CHUNK;
        HIPCHK(launch_bcast_rows(s, m, rc2, mean, mu, out + r0 * ldo, ldo));
        rc = trmm_lower(s, m, rc2, S, lds, eps + r0 * ldeps, ldeps, Et, out + r0 * ldo, ldo, 1.0, info_dev);
        if (rc) return rc;
    }
    HIPCHK(launch_fail_fill(s, m, nreal, out, ldo, info_dev));
    return GP_OK;
}

int gp_loglik_batched(gp_handle_t h, int32_t nbatch, const gp_theta_t *th_host, const int64_t *n_host,
                      const int64_t *x_off_host, const int64_t *c_off_host, int32_t dim, const double *X,
                      const double *y, double *C_pool, double *out3_dev, int32_t *info_dev, void *ws,
                      size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (nbatch < 0) return -2;
    if (nbatch > 0 && !th_host) return -3;
    if (nbatch > 0 && !n_host) return -4;
    if (nbatch > 0 && !x_off_host) return -5;
    if (nbatch > 0 && !c_off_host) return -6;
    if (dim < 1 || dim > 16) return -7;
    int64_t tot = 0, nmax = 1;
    for (int b = 0; b < nbatch; ++b) {
        if (int e = check_theta(th_host[b])) return e == 1 ? -3 : GP_ERR_NONFINITE;
        if (th_host[b].kind == GP_SEP_MATERN2) return GP_ERR_NOT_SUPPORTED;
        if (n_host[b] < 0) return -4;
        if (x_off_host[b] < 0) return -5;
        if (c_off_host[b] < 0) return -6;
        tot += n_host[b];
        nmax = n_host[b] > nmax ? n_host[b] : nmax;
    }
    if (tot > 0 && (!X || !y || !C_pool)) return !X ? -8 : (!y ? -9 : -10);
    if (nbatch > 0 && !out3_dev) return -11;
    if (nbatch > 0 && !info_dev) return -12;
    if (!ws) return -13;
    if (nbatch == 0) return GP_OK;
    return batch_run(h->stream, h->num_cu, batch_grid_choice(h, nmax), batch_tile_choice(h, nmax), h->batch_staging,
                     nbatch, th_host, n_host,
                     x_off_host, c_off_host, dim,
                     X, y, C_pool, out3_dev, info_dev, ws, ws_bytes);
}

int gp_tune_batched(gp_handle_t h, int32_t nbatch, const gp_theta_t *th_host, const int64_t *n_host,
                    const int64_t *x_off_host, const int64_t *c_off_host, int32_t dim, const double *X,
                    const double *y, double *C_pool, double *out3_dev, int32_t *info_dev, const int32_t *grid_cand,
                    const int32_t *tile_cand, int32_t n_cand, double *ms_out, void *ws, size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (nbatch < 1) return -2;
    if (!grid_cand) return -13;
    if (n_cand < 1) return -15;
    for (int32_t c = 0; c < n_cand; ++c) {
        if (grid_cand[c] < -1) return -13;
        if (tile_cand && tile_cand[c] != 0 && tile_cand[c] != 64 && tile_cand[c] != 128) return -14;
    }
    if (!ws) return -17;
    int64_t nmax = 1;
    if (n_host)
        for (int32_t b = 0; b < nbatch; ++b) nmax = n_host[b] > nmax ? n_host[b] : nmax;
    hipStream_t s = h->stream;
    const gp_options_t saved = h->opt;
    double best = -1.0;
    int32_t best_grid = saved.batch_grid, best_tile = saved.batch_tile;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return GP_ERR_HIP;
    }
    int rc = GP_OK;
    h->tuning = 1;
    for (int32_t c = 0; c < n_cand && rc == GP_OK; ++c) {
        double ms = -1.0;
        h->opt = saved;
        h->opt.batch_grid = grid_cand[c];
        h->opt.batch_tile = tile_cand ? tile_cand[c] : saved.batch_tile;
        const bool pers = grid_cand[c] >= 0;
        if (batch_ws_bytes(nmax, nbatch, pers, pers ? batch_tile_choice(h, nmax) : 64) <= ws_bytes) {
            for (int rep = 0; rep < 2 && rc == GP_OK; ++rep) {  // the first run warms the staging
                if (hipEventRecord(e0, s) != hipSuccess) {
                    rc = GP_ERR_HIP;
                    break;
                }
                rc = gp_loglik_batched(h, nbatch, th_host, n_host, x_off_host, c_off_host, dim, X, y, C_pool, out3_dev,
                                       info_dev, ws, ws_bytes);
                if (rc) break;
                float t = 0.f;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
                    rc = GP_ERR_HIP;
                    break;
                }
                ms = t;
            }
        }
        if (ms_out) ms_out[c] = ms;
        if (ms >= 0.0 && (best < 0.0 || ms < best)) {
            best = ms;
            best_grid = grid_cand[c];
            best_tile = pers ? batch_tile_choice(h, nmax) : 0;
        }
    }
    h->tuning = 0;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    h->opt = saved;
    if (rc) return rc;
    if (best < 0.0) return GP_ERR_NO_CANDIDATE;
    h->opt.batch_grid = best_grid;
    h->opt.batch_tile = best_tile;
    tune_store(h, TuneEntry{1, (int32_t)GP_FP64, size_bucket(nmax), 0, 0, 0, best_grid, best_tile});
    return GP_OK;
}

int gp_tune_save(gp_handle_t h, const char *path) {
    if (!ok_handle(h)) return -1;
    if (!path) return -2;
    FILE *f = fopen(path, "w");
    if (!f) return GP_ERR_IO;
    fprintf(f, "# gpmi tuning table: arch op prec bucket nb panel_cus syrk_slab batch_grid batch_tile\n");
    fprintf(f, "# op 0 = factorisation, 1 = batched call; bucket = floor(log2 n)\n");
    for (const TuneEntry &e : h->tune)
        fprintf(f, "%s %d %d %d %d %d %d %d %d\n", h->arch, e.op, e.prec, e.bucket, e.nb, e.panel_cus, e.syrk_slab,
                e.batch_grid, e.batch_tile);
    const bool ok = fclose(f) == 0;
    return ok ? GP_OK : GP_ERR_IO;
}

int gp_tune_load(gp_handle_t h, const char *path, int32_t *loaded) {
    if (!ok_handle(h)) return -1;
    if (!path) return -2;
    FILE *f = fopen(path, "r");
    if (!f) return GP_ERR_IO;
    char line[256];
    int32_t cnt = 0;
    std::vector<TuneEntry> got;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        char arch[64];
        TuneEntry e{};
        const int got_n = sscanf(line, "%63s %d %d %d %d %d %d %d %d", arch, &e.op, &e.prec, &e.bucket, &e.nb,
                                 &e.panel_cus, &e.syrk_slab, &e.batch_grid, &e.batch_tile);
        if (got_n != 8 && got_n != 9) {  // 8 fields: a table written before the tile column (tile automatic)
            fclose(f);
            return GP_ERR_IO;
        }
        if (strcmp(arch, h->arch) != 0) continue;  // another device's measurements
        const bool valid = (e.op == 0 || e.op == 1) && e.prec >= GP_FP64 && e.prec <= GP_BF16_TRAIL && e.bucket >= 0 &&
                           e.bucket < 63 && (e.op == 1 || (e.nb > 0 && e.nb % DB == 0)) && e.panel_cus >= 0 &&
                           (e.syrk_slab == 0 || e.syrk_slab == 8 || e.syrk_slab == 16) && e.batch_grid >= -1 &&
                           (e.batch_tile == 0 || e.batch_tile == 64 || e.batch_tile == 128);
        if (!valid) {
            fclose(f);
            return GP_ERR_IO;
        }
        got.push_back(e);
        ++cnt;
    }
    fclose(f);
    for (const TuneEntry &e : got) tune_store(h, e);
    if (loaded) *loaded = cnt;
    return GP_OK;
}

int gp_tune_clear(gp_handle_t h) {
    if (!ok_handle(h)) return -1;
    h->tune.clear();
    return GP_OK;
}

int gp_morton_order(gp_handle_t h, int64_t n, int32_t dim, const double *X, int64_t *perm_dev, void *ws,
                    size_t ws_bytes) {
    if (!ok_handle(h)) return -1;
    if (n < 0 || n >= (int64_t(1) << 22)) return -2;
    if (dim < 1 || dim > 16) return -3;
    if (n > 0 && !X) return -4;
    if (n > 0 && !perm_dev) return -5;
    Layout lay = layout(h, GP_OP_MORTON, n, 0, GP_FP64);
    if (!ws) return -6;
    if (ws_bytes < lay.total) return GP_ERR_WS_TOO_SMALL;
    HIPCHK(launch_morton(h->stream, n, dim, X, perm_dev, at<uint64_t>(ws, lay.keys), at<double>(ws, lay.box)));
    return GP_OK;
}

}  // extern "C"
