// k_batch.hip -- many independent Gaussian-process likelihoods in one
// persistent launch (the same model and quantities as the single-problem
// path: C(theta), L L^T = C, L^{-1} y, log|C|, loglik; Section 1).
//
// Work is a host-built table of tasks on 64 x 64 tiles.  For problem b:
//   tile (i, j), i >= j:  build C_ij from the points, subtract
//       sum_{k < j} L_ik L_jk^T (left-looking, matrix cores), then factor +
//       invert it (i == j, one wave in registers) or multiply by the diagonal
//       block's inverse (i > j) -- the block Cholesky of Section 2.1 / Fig. 1;
//   solve i:  z_i = Winv_ii (y_i - sum_{k < i} L_ik z_k);
//   reduce:   log|C| = 2 sum log L_ii, q = z^T z, loglik.
// Tasks are ordered by dependency level (tile (j,j): 4j, tile (i>j, j): 4j + 2,
// solve i: 4i + 3, reduce: 4 nt + 1), then by problem size, so every task
// waits only on tasks with smaller tickets.  Workgroups take tickets from an
// atomic counter, hence every waited-on task belongs to a running workgroup
// and the launch cannot deadlock; each wait is bounded (abort flag).
#include "internal.h"

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

struct BProb {
    int64_t n, x_off, c_off, tflag_off, zflag_off, z_off, w_off;
    double s2, inv_rho, t2;
    int32_t kind, nt;
};
struct BTask {
    int32_t prob, i, j, type;  // type 0 tile, 1 solve, 2 reduce
};

constexpr int T = 64;

GP_DEV int64_t tri_index(int64_t i, int64_t j) { return i * (i + 1) / 2 + j; }

// Workgroup-uniform wait: returns the flag value (1 ready, 2 failed) or 0 on
// timeout / abort.
GP_DEV int wg_wait(const int *f, int *abortf, int *s_flag) {
    if (threadIdx.x == 0) {
        int spins = 0, v;
        while ((v = ld_acquire_agent(f)) == 0) {
            if (ld_acquire_agent(abortf)) break;
            __builtin_amdgcn_s_sleep(2);
            if (++spins > SPIN_LIMIT) {
                __hip_atomic_store(abortf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        *s_flag = v;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int v = *s_flag;
    __syncthreads();
    return v;
}

GP_DEV void wg_release(int *f, int v) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) st_release_agent(f, v);
}

__global__ __launch_bounds__(256, 1) void k_batch(const BProb *__restrict__ probs, const BTask *__restrict__ tasks,
                                                  int64_t ntasks, int dim, const double *__restrict__ X,
                                                  const double *__restrict__ y, double *C_pool, double *zbuf,
                                                  double *wbuf, int *flags, int *ctl, double *out3, int32_t *info) {
    __shared__ double As[T][T + 1];
    __shared__ double Bs[T][T + 1];
    __shared__ double red[4][T];
    __shared__ int s_task, s_flag, s_fail;
    int *abortf = &ctl[1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;  // 2 x 2 waves, 32 x 32 each

    for (;;) {
        if (tid == 0) s_task = atomicAdd(&ctl[0], 1);
        __syncthreads();
        const int64_t t = s_task;
        __syncthreads();
        if (t >= ntasks) break;
        const BTask tk = tasks[t];
        const BProb P = probs[tk.prob];
        const int64_t n = P.n, ld = P.n;
        double *L = C_pool + P.c_off;
        int *tflag = flags + P.tflag_off;
        int *zflag = flags + P.zflag_off;
        const double *Xb = X + P.x_off * dim;

        if (tk.type == 0) {
            const int i = tk.i, j = tk.j;
            const int64_t i0 = (int64_t)i * T, j0 = (int64_t)j * T;
            bool ok = true;
            v4d acc[2][2];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int q = 0; q < 2; ++q) acc[m][q] = v4d{0.0, 0.0, 0.0, 0.0};
            for (int k = 0; k < j && ok; ++k) {
                const int v1 = wg_wait(&tflag[tri_index(i, k)], abortf, &s_flag);
                const int v2 = wg_wait(&tflag[tri_index(j, k)], abortf, &s_flag);
                if (v1 != 1 || v2 != 1) {
                    ok = false;
                    break;
                }
                const int64_t k0 = (int64_t)k * T;  // block k < j is a full block
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
                __syncthreads();
            }
            if (!ok) {
                wg_release(&tflag[tri_index(i, j)], 2);
                continue;
            }
            // S = C_ij - acc, in the f64 MFMA layout (row lane/16 + 4r, column lane%16)
            double sv[2][2][4];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wm * 32 + m * 16 + (lane >> 4) + 4 * r;
                        const int col = wn * 32 + q * 16 + (lane & 15);
                        const int64_t gi = i0 + row, gj = j0 + col;
                        double c;
                        if (gi < n && gj < n) {
                            const double d = point_dist(Xb + gi * dim, Xb + gj * dim, dim);
                            c = P.s2 * cov_corr(P.kind, d * P.inv_rho) + (gi == gj ? P.t2 : 0.0);
                        } else {
                            c = (gi == gj) ? 1.0 : 0.0;  // identity padding of the last diagonal tile
                        }
                        sv[m][q][r] = c - acc[m][q][r];
                    }
            if (i == j) {
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int q = 0; q < 2; ++q)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            As[wm * 32 + m * 16 + (lane >> 4) + 4 * r][wn * 32 + q * 16 + (lane & 15)] = sv[m][q][r];
                if (tid == 0) s_fail = 0;
                __syncthreads();
                const int tj = (int)((n - j0) < T ? (n - j0) : T);
                if (w == 0) {
                    double a[T];
#pragma unroll
                    for (int c = 0; c < T; ++c) a[c] = (c <= lane) ? As[lane][c] : 0.0;
                    const int fail = wave_chol64(a, lane);
                    if (fail) {
                        if (lane == 0) s_fail = fail;
                    } else {
#pragma unroll
                        for (int c = 0; c < T; ++c) {
                            As[lane][c] = a[c];
                            if (lane < tj && c <= lane) L[(j0 + lane) + (j0 + c) * ld] = a[c];
                        }
                    }
                }
                __syncthreads();
                const int fail = s_fail;
                if (fail) {
                    if (tid == 0) info[tk.prob] = (int32_t)(j0 + fail);
                    wg_release(&tflag[tri_index(i, j)], 2);
                    continue;
                }
                if (w == 0) {
                    double wv[T];
                    wave_inv64(As, wv, lane);
                    double *W = wbuf + P.w_off + (int64_t)j * T * T;
#pragma unroll
                    for (int r = 0; r < T; ++r) W[r + lane * T] = wv[r];
                }
                wg_release(&tflag[tri_index(i, j)], 1);
            } else {
                const int vd = wg_wait(&tflag[tri_index(j, j)], abortf, &s_flag);
                if (vd != 1) {
                    wg_release(&tflag[tri_index(i, j)], 2);
                    continue;
                }
                // L_ij = S W_jj^T: A operand S staged k-major (As[kk][ii] = S[ii][kk]),
                // B operand op(B)[kk][jj] = W_jj[jj][kk] = W[jj + kk T].
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
                    double a[2], b[2];
#pragma unroll
                    for (int m = 0; m < 2; ++m) a[m] = As[kk + (lane >> 4)][wm * 32 + m * 16 + (lane & 15)];
#pragma unroll
                    for (int q = 0; q < 2; ++q) b[q] = Bs[kk + (lane >> 4)][wn * 32 + q * 16 + (lane & 15)];
#pragma unroll
                    for (int m = 0; m < 2; ++m)
#pragma unroll
                        for (int q = 0; q < 2; ++q)
                            o[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[q], o[m][q], 0, 0, 0);
                }
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int q = 0; q < 2; ++q)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int64_t gi = i0 + wm * 32 + m * 16 + (lane >> 4) + 4 * r;
                            const int64_t gj = j0 + wn * 32 + q * 16 + (lane & 15);
                            if (gi < n && gj < n) L[gi + gj * ld] = o[m][q][r];
                        }
                wg_release(&tflag[tri_index(i, j)], 1);
            }
        } else if (tk.type == 1) {
            const int i = tk.i;
            const int64_t i0 = (int64_t)i * T;
            const int vd = wg_wait(&tflag[tri_index(i, i)], abortf, &s_flag);
            const int vz = i > 0 ? wg_wait(&zflag[i - 1], abortf, &s_flag) : 1;
            if (vd != 1 || vz != 1) {
                wg_release(&zflag[i], 2);
                continue;
            }
            double *z = zbuf + P.z_off;
            const int64_t gi = i0 + lane;
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
            if (w == 0) {
                const double yb = rv ? y[P.x_off + gi] : 0.0;
                As[0][lane] = rv ? yb - (((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]) : 0.0;
            }
            __syncthreads();
            const double *W = wbuf + P.w_off + (int64_t)i * T * T;
            double sacc = 0.0;
            for (int c = w * 16; c < w * 16 + 16; ++c) sacc = fma(W[lane + c * T], As[0][c], sacc);
            red[w][lane] = sacc;
            __syncthreads();
            if (w == 0 && rv) z[gi] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
            wg_release(&zflag[i], 1);
        } else {
            const int nt = P.nt;
            const int vz = nt > 0 ? wg_wait(&zflag[nt - 1], abortf, &s_flag) : 1;
            const bool bad = vz != 1 || info[tk.prob] != 0 || ld_acquire_agent(abortf);
            CSum sl, sq;
            if (!bad) {
                const double *z = zbuf + P.z_off;
                for (int64_t q = tid; q < n; q += 256) {
                    sl.add(log(L[q + q * ld]));
                    sq.add(z[q] * z[q]);
                }
            }
            __shared__ double r2[4 * 256];
            r2[tid * 4 + 0] = sl.s; r2[tid * 4 + 1] = sl.c; r2[tid * 4 + 2] = sq.s; r2[tid * 4 + 3] = sq.c;
            __syncthreads();
            for (int st = 128; st > 0; st >>= 1) {
                if (tid < st) {
                    for (int h = 0; h < 2; ++h) {
                        CSum a, b;
                        a.s = r2[tid * 4 + 2 * h]; a.c = r2[tid * 4 + 2 * h + 1];
                        b.s = r2[(tid + st) * 4 + 2 * h]; b.c = r2[(tid + st) * 4 + 2 * h + 1];
                        a.merge(b);
                        r2[tid * 4 + 2 * h] = a.s; r2[tid * 4 + 2 * h + 1] = a.c;
                    }
                }
                __syncthreads();
            }
            if (tid == 0) {
                double *o = out3 + 3 * (int64_t)tk.prob;
                if (bad) {
                    o[0] = o[1] = o[2] = __builtin_nan("");
                    if (info[tk.prob] == 0 && vz != 2) info[tk.prob] = -1;  // watchdog expired
                } else {
                    const double logdet = 2.0 * (r2[0] + r2[1]);
                    const double q = r2[2] + r2[3];
                    o[1] = logdet;
                    o[2] = q;
                    o[0] = -0.5 * (((double)n * 1.8378770664093453 + logdet) + q);
                }
            }
            __syncthreads();
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side: task table, workspace layout, launch.
// ---------------------------------------------------------------------------
#include <algorithm>
#include <cmath>
#include <vector>

namespace {
inline size_t al256b(size_t x) { return (x + 255) & ~(size_t)255; }
}

size_t batch_ws_bytes(int64_t nmax, int64_t nbatch) {
    const int64_t nt = (nmax + T - 1) / T;
    const size_t per_tasks = (size_t)(nt * (nt + 1) / 2 + nt + 1);
    size_t b = 0;
    b += al256b(sizeof(BProb) * (size_t)nbatch);
    b += al256b(sizeof(BTask) * per_tasks * (size_t)nbatch);
    b += al256b(sizeof(int) * (per_tasks * (size_t)nbatch + 2));
    b += al256b(sizeof(double) * (size_t)nmax * (size_t)nbatch);
    b += al256b(sizeof(double) * (size_t)nt * T * T * (size_t)nbatch);
    return b + 256;
}

struct BatchStaging {
    std::vector<BProb> probs;
    std::vector<BTask> tasks;
    hipEvent_t done = nullptr;
};

int batch_run(hipStream_t s, int num_cu, void *&staging_ptr, int32_t nb, const gp_theta_t *th, const int64_t *nh,
              const int64_t *xoff, const int64_t *coff, int32_t dim, const double *X, const double *y,
              double *C_pool, double *out3, int32_t *info, void *ws, size_t ws_bytes) {
    BatchStaging *st = static_cast<BatchStaging *>(staging_ptr);
    if (!st) {
        st = new BatchStaging();
        staging_ptr = st;
    }
    if (st->done) {
        if (hipEventSynchronize(st->done) != hipSuccess) return GP_ERR_HIP;  // host copy of the last call is consumed
    } else if (hipEventCreateWithFlags(&st->done, hipEventDisableTiming) != hipSuccess) {
        return GP_ERR_HIP;
    }
    int64_t nmax = 1;
    for (int b = 0; b < nb; ++b) nmax = std::max(nmax, nh[b]);
    if (ws_bytes < batch_ws_bytes(nmax, nb)) return GP_ERR_WS_TOO_SMALL;
    st->probs.assign(nb, BProb{});
    int64_t toff = 0, zoff = 0, woff = 0;
    for (int b = 0; b < nb; ++b) {
        BProb &p = st->probs[b];
        p.n = nh[b];
        p.x_off = xoff[b];
        p.c_off = coff[b];
        p.nt = (int32_t)((p.n + T - 1) / T);
        p.tflag_off = toff;
        toff += (int64_t)p.nt * (p.nt + 1) / 2;
        p.zflag_off = toff;
        toff += p.nt;
        p.z_off = zoff;
        zoff += p.n;
        p.w_off = woff;
        woff += (int64_t)p.nt * T * T;
        p.kind = th[b].kind;
        p.s2 = std::exp(th[b].log_sigma2);
        p.inv_rho = std::exp(-th[b].log_rho);
        p.t2 = std::exp(th[b].log_tau2);
    }
    // order: level, then larger problems first, then row
    std::vector<int> rank(nb);
    for (int b = 0; b < nb; ++b) rank[b] = b;
    std::stable_sort(rank.begin(), rank.end(), [&](int a, int c) { return nh[a] > nh[c]; });
    std::vector<int> pos(nb);
    for (int r = 0; r < nb; ++r) pos[rank[r]] = r;
    struct Key {
        int64_t level;
        int32_t prank, i;
        BTask t;
    };
    std::vector<Key> keys;
    for (int b = 0; b < nb; ++b) {
        const int nt = st->probs[b].nt;
        if (nt == 0) {  // empty problem: only the reduce task (loglik 0)
            keys.push_back({1, pos[b], 0, BTask{b, 0, 0, 2}});
            continue;
        }
        for (int j = 0; j < nt; ++j)
            for (int i = j; i < nt; ++i) keys.push_back({4LL * j + (i > j ? 2 : 0), pos[b], i, BTask{b, i, j, 0}});
        for (int i = 0; i < nt; ++i) keys.push_back({4LL * i + 3, pos[b], i, BTask{b, i, i, 1}});
        keys.push_back({4LL * nt + 1, pos[b], 0, BTask{b, 0, 0, 2}});
    }
    std::stable_sort(keys.begin(), keys.end(), [](const Key &a, const Key &c) {
        if (a.level != c.level) return a.level < c.level;
        if (a.prank != c.prank) return a.prank < c.prank;
        return a.i < c.i;
    });
    st->tasks.resize(keys.size());
    for (size_t q = 0; q < keys.size(); ++q) st->tasks[q] = keys[q].t;
    const int64_t ntasks = (int64_t)st->tasks.size();

    char *base = static_cast<char *>(ws);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off += al256b(bytes);
        return p;
    };
    const int64_t ntmax = (nmax + T - 1) / T;
    const size_t per_tasks = (size_t)(ntmax * (ntmax + 1) / 2 + ntmax + 1);
    BProb *d_probs = reinterpret_cast<BProb *>(take(sizeof(BProb) * (size_t)nb));
    BTask *d_tasks = reinterpret_cast<BTask *>(take(sizeof(BTask) * per_tasks * (size_t)nb));
    int *d_flags = reinterpret_cast<int *>(take(sizeof(int) * (per_tasks * (size_t)nb + 2)));
    double *d_z = reinterpret_cast<double *>(take(sizeof(double) * (size_t)nmax * (size_t)nb));
    double *d_w = reinterpret_cast<double *>(take(sizeof(double) * (size_t)ntmax * T * T * (size_t)nb));
    int *ctl = d_flags + toff;  // [ticket, abort] after the flags

    if (hipMemcpyAsync(d_probs, st->probs.data(), sizeof(BProb) * (size_t)nb, hipMemcpyHostToDevice, s) != hipSuccess)
        return GP_ERR_HIP;
    if (ntasks > 0 && hipMemcpyAsync(d_tasks, st->tasks.data(), sizeof(BTask) * (size_t)ntasks, hipMemcpyHostToDevice,
                                     s) != hipSuccess)
        return GP_ERR_HIP;
    if (hipEventRecord(st->done, s) != hipSuccess) return GP_ERR_HIP;
    if (launch_fill(s, d_flags, sizeof(int) * (size_t)(toff + 2)) != hipSuccess) return GP_ERR_HIP;
    if (launch_fill(s, info, sizeof(int32_t) * (size_t)nb) != hipSuccess) return GP_ERR_HIP;
    if (ntasks == 0) return GP_OK;
    const int64_t grid = std::min<int64_t>(ntasks, (int64_t)num_cu);
    hipLaunchKernelGGL(k_batch, dim3((unsigned)grid), dim3(256), 0, s, d_probs, d_tasks, ntasks, dim, X, y, C_pool,
                       d_z, d_w, d_flags, ctl, out3, info);
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
