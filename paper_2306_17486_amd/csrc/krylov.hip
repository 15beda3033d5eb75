// Flexible GMRES(m) on gfx950 (Saad 1993; the outer Krylov method of the paper).
//
// Mixed precision: the basis V and the preconditioned vectors Z are complex
// single precision; every inner product and norm is accumulated in FP64; the
// Hessenberg matrix, the Givens rotations and the small triangular solve are
// FP64; x is complex double and the residual b - A x is recomputed in FP64 at
// every restart, which is what the stopping test uses.
//
// Every right-hand side of a batch advances in lock step; per-RHS flags in
// device memory switch finished ones off, so a whole restart cycle is enqueued
// without host round trips.  The host reads one flag per RHS per cycle.
//
// Lazy normalisation: v_{j+1} is stored as the orthogonalised w and its scale
// sigma_{j+1} = 1/||w|| is applied by every reader, which saves one full pass
// over the vector per iteration.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <mutex>

#include "hh_internal.h"
#include "krylov.h"

namespace hh {

constexpr int KT_X = 64, KT_Y = 16, KT_ROWS = 4;  // 64 x 16 tile, 256 threads
constexpr int MAXV = HH_MAX_RESTART + 1;

static inline int kblocks(int n) { return ((n + KT_X - 1) / KT_X) * ((n + KT_Y - 1) / KT_Y); }

// Block-wide sum of NV double2 values per thread; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum2(double2 (&v)[NV], int nact, double2* s_red /* [4][NV] */) {
    const int lane = threadIdx.x + threadIdx.y * blockDim.x;
    const int wid = lane >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < nact) {
            v[i].x = wave_sum(v[i].x);
            v[i].y = wave_sum(v[i].y);
        }
    }
    if ((lane & 63) == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nact) s_red[wid * NV + i] = v[i];
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            if (i < nact) {
                double2 a = s_red[i];
                for (int w = 1; w < 4; ++w) a = zadd(a, s_red[w * NV + i]);
                v[i] = a;
            }
        }
    }
}

// ||b||^2 partials (FP64) of a complex-single vector
__global__ void __launch_bounds__(256) k_norm2(const float2* __restrict__ b, int n, double2* __restrict__ parts) {
    __shared__ double2 s_red[4];
    const int r = blockIdx.z;
    const size_t nn = (size_t)n * n;
    const int j = blockIdx.x * KT_X + threadIdx.x;
    const int i0 = blockIdx.y * KT_Y + threadIdx.y * KT_ROWS;
    double2 acc[1] = {make_double2(0.0, 0.0)};
    if (j < n)
        for (int t = 0; t < KT_ROWS; ++t) {
            int i = i0 + t;
            if (i < n) {
                float2 v = b[r * nn + (size_t)i * n + j];
                acc[0].x += (double)v.x * v.x + (double)v.y * v.y;
            }
        }
    block_sum2<1>(acc, 1, s_red);
    if (threadIdx.x == 0 && threadIdx.y == 0)
        parts[(size_t)r * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = acc[0];
}

// r = b - A x in FP64 (x complex double); r stored single into V[r][0]; ||r||^2 partials.
// The zeroth-order term omega^2 kappa^2 (1 - i gamma) is formed in FP64 from
// the FP32 slowness as given, so this residual is that of eqs. 1-3 itself,
// not of the FP32-rounded coefficients the single-precision kernels use.
__global__ void __launch_bounds__(256) k_residual64(const double2* __restrict__ x, const float2* __restrict__ b,
                                                    float2* __restrict__ Vbase, size_t vstride, Coef64 cf64,
                                                    const int* __restrict__ inst, int n, double inv_h2,
                                                    double2* __restrict__ parts, const int* __restrict__ done) {
    __shared__ double2 s_red[4];
    const int r = blockIdx.z;
    const bool skip = done && done[r];
    const size_t nn = (size_t)n * n;
    const int j = blockIdx.x * KT_X + threadIdx.x;
    const int i0 = blockIdx.y * KT_Y + threadIdx.y * KT_ROWS;
    const double2* xr = x + r * nn;
    const float* kap = cf64.kappa + (size_t)(inst ? inst[r] : 0) * nn;
    double2 acc[1] = {make_double2(0.0, 0.0)};
    if (!skip && j < n) {
        const double2 z = make_double2(0.0, 0.0);
        for (int t = 0; t < KT_ROWS; ++t) {
            int i = i0 + t;
            if (i >= n) break;
            size_t o = (size_t)i * n + j;
            double2 c = xr[o];
            double2 up = i > 0 ? xr[o - n] : z, dn = i + 1 < n ? xr[o + n] : z;
            double2 lf = j > 0 ? xr[o - 1] : z, rt = j + 1 < n ? xr[o + 1] : z;
            const double k = kap[o];
            const double w2k2 = cf64.omega2 * k * k;
            const double g = abl_gamma(i, j, n, cf64.abl_w, cf64.gmax, cf64.gamma0);
            // A x = (4c - nb)/h^2 - w2k2 (1 - i g) c
            double2 m = make_double2(w2k2, -w2k2 * g);
            double2 Ax = make_double2((4.0 * c.x - up.x - dn.x - lf.x - rt.x) * inv_h2,
                                      (4.0 * c.y - up.y - dn.y - lf.y - rt.y) * inv_h2);
            Ax = zsub(Ax, zmul(m, c));
            float2 bv = b[r * nn + o];
            double2 rv = make_double2((double)bv.x - Ax.x, (double)bv.y - Ax.y);
            if (Vbase) Vbase[r * vstride + o] = make_float2((float)rv.x, (float)rv.y);
            acc[0].x += zabs2(rv);
        }
    }
    block_sum2<1>(acc, 1, s_red);
    if (threadIdx.x == 0 && threadIdx.y == 0)
        parts[(size_t)r * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = acc[0];
}

static Coef64 coef64(const hh_model* md) {
    Coef64 c;
    c.kappa = md->kappa0.as<float>();
    c.omega2 = md->d.omega * md->d.omega;
    c.abl_w = md->d.abl_width;
    c.gmax = md->d.abl_gamma_max;
    c.gamma0 = md->d.gamma0;
    return c;
}

// w = A z (FP32) written to V[j+1]; partial dots <v~_i, w>, i = 0..j: each
// thread sums its 4 points in FP32, the block and grid sums are FP64.  The
// read set (z, v_0..v_j) and the write set (v_{j+1}) do not overlap.
// Launched with NJ = j + 1: every per-thread array is indexed by compile-time
// constants only, so it stays in registers.
template <int NJ>
__global__ void __launch_bounds__(256) k_op_dots(const float2* __restrict__ Z, size_t zstride,
                                                 const float2* __restrict__ Vin, float2* __restrict__ Vout,
                                                 size_t vstride, int j, const float2* __restrict__ coef,
                                                 const int* __restrict__ inst, int n, float inv_h2,
                                                 double2* __restrict__ parts, int npart,
                                                 const int* __restrict__ active) {
    __shared__ double2 s_red[4 * NJ];
    const int r = blockIdx.z;
    if (!active[r]) return;
    const size_t nn = (size_t)n * n;
    const int jj = blockIdx.x * KT_X + threadIdx.x;
    const int i0 = blockIdx.y * KT_Y + threadIdx.y * KT_ROWS;
    const float2* zr = Z + r * zstride;
    const float2* Vr = Vin + r * vstride;
    const float2* cf = coef + (size_t)(inst ? inst[r] : 0) * nn;
    float2 pacc[NJ];
#pragma unroll
    for (int q = 0; q < NJ; ++q) pacc[q] = make_float2(0.f, 0.f);
    const float2 zero = make_float2(0.f, 0.f);
    float2* wout = Vout + r * vstride + (size_t)(j + 1) * nn;
    if (jj < n) {
        float2 up = (i0 > 0 && i0 - 1 < n) ? zr[(size_t)(i0 - 1) * n + jj] : zero;
        float2 cur = (i0 < n) ? zr[(size_t)i0 * n + jj] : zero;
#pragma unroll
        for (int t = 0; t < KT_ROWS; ++t) {
            const int i = i0 + t;
            if (i >= n) break;
            const size_t o = (size_t)i * n + jj;
            const float2 dn = (i + 1 < n) ? zr[o + n] : zero;
            const float2 lf = (jj > 0) ? zr[o - 1] : zero;
            const float2 rt = (jj + 1 < n) ? zr[o + 1] : zero;
            const float2 m = mass_of(cf[o], 0.f);
            // sum of neighbour differences: far less cancellation in FP32 than 4c - sum
            const float2 lap = make_float2(((cur.x - up.x) + (cur.x - dn.x)) + ((cur.x - lf.x) + (cur.x - rt.x)),
                                           ((cur.y - up.y) + (cur.y - dn.y)) + ((cur.y - lf.y) + (cur.y - rt.y)));
            const float2 w = csub(cscale(lap, inv_h2), cmul(m, cur));
            wout[o] = w;
#pragma unroll
            for (int q = 0; q < NJ; ++q) {
                const float2 v = Vr[(size_t)q * nn + o];
                // conj(v) * w
                pacc[q].x += v.x * w.x + v.y * w.y;
                pacc[q].y += v.x * w.y - v.y * w.x;
            }
            up = cur;
            cur = dn;
        }
    }
    double2 acc[NJ];
#pragma unroll
    for (int q = 0; q < NJ; ++q) acc[q] = make_double2((double)pacc[q].x, (double)pacc[q].y);
    block_sum2<NJ>(acc, NJ, s_red);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double2* p = parts + ((size_t)r * npart + blockIdx.y * gridDim.x + blockIdx.x) * MAXV;
#pragma unroll
        for (int q = 0; q < NJ; ++q) p[q] = acc[q];
    }
}

// w <- w - sum_i oc_i v~_i  (w = V[j+1]); partial ||w||^2
template <int NJ>
__global__ void __launch_bounds__(256) k_ortho(float2* __restrict__ V, size_t vstride, int j, const KState* __restrict__ st,
                                               int n, double2* __restrict__ parts, int npart,
                                               const int* __restrict__ active) {
    __shared__ double2 s_red[4];
    __shared__ float2 s_oc[NJ];
    const int r = blockIdx.z;
    if (!active[r]) return;
    const size_t nn = (size_t)n * n;
    const int lane = threadIdx.x + threadIdx.y * blockDim.x;
    const int nact = j + 1;
    if (lane < nact) s_oc[lane] = st[r].oc[lane];
    __syncthreads();
    const int jj = blockIdx.x * KT_X + threadIdx.x;
    const int i0 = blockIdx.y * KT_Y + threadIdx.y * KT_ROWS;
    double2 acc[1] = {make_double2(0.0, 0.0)};
    float2* Vr = V + r * vstride;
    if (jj < n) {
        for (int t = 0; t < KT_ROWS; ++t) {
            const int i = i0 + t;
            if (i >= n) break;
            size_t o = (size_t)i * n + jj;
            float2 w = Vr[(size_t)(j + 1) * nn + o];
#pragma unroll
            for (int q = 0; q < NJ; ++q)
                if (q < nact) w = csub(w, cmul(s_oc[q], Vr[(size_t)q * nn + o]));
            Vr[(size_t)(j + 1) * nn + o] = w;
            acc[0].x += (double)w.x * w.x + (double)w.y * w.y;
        }
    }
    block_sum2<1>(acc, 1, s_red);
    if (lane == 0) parts[(size_t)r * npart + blockIdx.y * gridDim.x + blockIdx.x] = acc[0];
}

// Sum the dot partials into column j of H (h_ij = sigma_i <v~_i, w>) and set the
// single-precision orthogonalisation coefficients oc_i = h_ij sigma_i.
__global__ void __launch_bounds__(256) k_arnoldi_col(const double2* __restrict__ parts, int npart, int j,
                                                     KState* __restrict__ st, const int* __restrict__ active) {
    __shared__ double2 s_red[4 * MAXV];
    const int r = blockIdx.x;
    if (!active[r]) return;
    const int nact = j + 1;
    double2 acc[MAXV];
#pragma unroll
    for (int q = 0; q < MAXV; ++q) acc[q] = make_double2(0.0, 0.0);
    for (int p = threadIdx.x; p < npart; p += 256) {
        const double2* pp = parts + ((size_t)r * npart + p) * MAXV;
#pragma unroll
        for (int q = 0; q < MAXV; ++q)
            if (q < nact) acc[q] = zadd(acc[q], pp[q]);
    }
    block_sum2<MAXV>(acc, nact, s_red);
    if (threadIdx.x == 0) {
        KState& S = st[r];
        for (int q = 0; q < nact; ++q) {
            double sg = S.sig[q];
            double2 h = make_double2(acc[q].x * sg, acc[q].y * sg);
            S.H[q][j] = h;
            S.oc[q] = make_float2((float)(h.x * sg), (float)(h.y * sg));
        }
    }
}

// Norm of the orthogonalised w, Givens update of column j, residual estimate,
// small triangular solve, per-RHS flags.
__global__ void __launch_bounds__(256) k_givens(const double2* __restrict__ parts, int npart, int j,
                                                KState* __restrict__ st, int* __restrict__ active,
                                                int* __restrict__ actc, int* __restrict__ actm,
                                                double* __restrict__ hist, int hist_len, double rtol, int max_iters,
                                                const int* __restrict__ caps) {
    __shared__ double2 s_red[4];
    const int r = blockIdx.x;
    if (!active[r]) return;
    double2 acc[1] = {make_double2(0.0, 0.0)};
    for (int p = threadIdx.x; p < npart; p += 256) acc[0] = zadd(acc[0], parts[(size_t)r * npart + p]);
    block_sum2<1>(acc, 1, s_red);
    if (threadIdx.x != 0) return;
    KState& S = st[r];
    const double hn = sqrt(acc[0].x);
    S.H[j + 1][j] = make_double2(hn, 0.0);
    S.sig[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
    // apply the previous rotations to column j
    double2 col[MAXV];
    for (int i = 0; i <= j + 1; ++i) col[i] = S.H[i][j];
    for (int i = 0; i < j; ++i) {
        double c = S.cs[i];
        double2 s = S.sn[i];
        double2 a = col[i], b = col[i + 1];
        col[i] = zadd(make_double2(c * a.x, c * a.y), zmul(s, b));
        col[i + 1] = zsub(make_double2(c * b.x, c * b.y), zmul(zconj(s), a));
    }
    // new rotation zeroing col[j+1]
    double2 a = col[j], b = col[j + 1];
    double na = sqrt(zabs2(a)), nb = sqrt(zabs2(b));
    double c;
    double2 s;
    if (nb == 0.0) {
        c = 1.0;
        s = make_double2(0.0, 0.0);
    } else if (na == 0.0) {
        c = 0.0;
        s = make_double2(1.0, 0.0);
    } else {
        double t = sqrt(na * na + nb * nb);
        c = na / t;
        double2 ph = make_double2(a.x / na, a.y / na);
        s = zmul(ph, make_double2(b.x / t, -b.y / t));
    }
    col[j] = zadd(make_double2(c * a.x, c * a.y), zmul(s, b));
    col[j + 1] = make_double2(0.0, 0.0);
    S.cs[j] = c;
    S.sn[j] = s;
    for (int i = 0; i <= j + 1; ++i) S.H[i][j] = col[i];
    double2 gj = S.g[j];
    S.g[j + 1] = zmul(make_double2(-s.x, s.y), gj);  // -conj(s) g_j
    S.g[j] = make_double2(c * gj.x, c * gj.y);
    // y = R^{-1} g (upper triangular, size j+1)
    for (int i = j; i >= 0; --i) {
        double2 t = S.g[i];
        for (int q = i + 1; q <= j; ++q) t = zsub(t, zmul(S.H[i][q], S.y[q]));
        S.y[i] = zdiv(t, S.H[i][i]);
    }
    S.k = j + 1;
    S.iters += 1;
    if (S.mode == PM_CNN) S.cnn_iters += 1;
    const double est = sqrt(zabs2(S.g[j + 1])) / S.bnorm;
    S.res_est = est;
    const bool bad = !isfinite(est) || !isfinite(hn);
    if (bad && S.mode == PM_CNN) {
        // a non-finite network output: this cycle's directions are dropped (x keeps
        // its last finite value) and the right-hand side continues with MG-only
        S.cnn_off = 1;
        S.k = 0;
    } else if (bad) {
        S.breakdown = 1;
    }
    if (hist && S.iters < hist_len) hist[(size_t)r * hist_len + S.iters] = bad ? S.res_cycle0 : est;
    const bool by_est = est <= rtol * S.tol_scale;
    if (by_est) S.ended_by_est = 1;
    const int cap = caps ? min(caps[r], max_iters) : max_iters;
    if (bad || by_est || S.iters >= cap || hn == 0.0) active[r] = actc[r] = actm[r] = 0;
}

// x += sum_{q<k} y_q z_q  (x complex double)
__global__ void __launch_bounds__(256) k_xupdate(double2* __restrict__ x, const float2* __restrict__ Z, size_t zstride,
                                                 const KState* __restrict__ st, int n) {
    __shared__ double2 s_y[HH_MAX_RESTART];
    __shared__ int s_k;
    const int r = blockIdx.z;
    const int lane = threadIdx.x + threadIdx.y * blockDim.x;
    if (lane == 0) s_k = st[r].breakdown ? 0 : st[r].k;
    if (lane < HH_MAX_RESTART) s_y[lane] = st[r].y[lane];
    __syncthreads();
    const int k = s_k;
    if (k == 0) return;
    const size_t nn = (size_t)n * n;
    const int jj = blockIdx.x * KT_X + threadIdx.x;
    const int i0 = blockIdx.y * KT_Y + threadIdx.y * KT_ROWS;
    if (jj >= n) return;
    for (int t = 0; t < KT_ROWS; ++t) {
        const int i = i0 + t;
        if (i >= n) break;
        size_t o = (size_t)i * n + jj;
        double2 acc = x[r * nn + o];
        for (int q = 0; q < k; ++q) {
            float2 z = Z[r * zstride + (size_t)q * nn + o];
            acc = zadd(acc, zmul(s_y[q], make_double2(z.x, z.y)));
        }
        x[r * nn + o] = acc;
    }
}

// ||b|| from partials; zero right-hand sides are finished at once (x = 0).
__global__ void k_init_state(const double2* __restrict__ parts, int npart, KState* __restrict__ st, int* done,
                             int* active, double* hist, int hist_len) {
    __shared__ double2 s_red[4];
    const int r = blockIdx.x;
    double2 acc[1] = {make_double2(0.0, 0.0)};
    for (int p = threadIdx.x; p < npart; p += 256) acc[0] = zadd(acc[0], parts[(size_t)r * npart + p]);
    block_sum2<1>(acc, 1, s_red);
    if (threadIdx.x != 0) return;
    KState& S = st[r];
    {
        uint64_t* w = reinterpret_cast<uint64_t*>(&S);
        for (size_t q = 0; q < sizeof(KState) / 8; ++q) w[q] = 0;
    }
    S.bnorm = sqrt(acc[0].x);
    S.tol_scale = 1.0;
    done[r] = S.bnorm == 0.0 ? 1 : 0;
    if (S.bnorm == 0.0) S.converged = 1;
    active[r] = 0;
    if (hist)
        for (int q = 0; q < hist_len; ++q) hist[(size_t)r * hist_len + q] = -1.0;
}

// Preconditioner of the next restart cycle of a CNN+MG solve: MG-only FGMRES
// judges the network, and the network judges MG-only.  A cycle that reduces
// the FP64 residual by less than probe_ratio (end / start above it) is
// followed by one probe cycle of the other preconditioner; the probe's
// preconditioner takes over if its cycle reduced the residual more, otherwise
// the previous one resumes and the wait before the next probe doubles
// (2, 4, 8, ... cycles; a switch resets it).  A right-hand side on which the
// network gave a non-finite result stays on MG-only.
__device__ static int next_mode(KState& S, int warm, int judge, double probe_ratio) {
    if (warm) return PM_WARM;
    if (S.cnn_off) {  // the network failed on this right-hand side
        S.probing = 0;
        return PM_MG;
    }
    if (S.mode == PM_WARM) return PM_CNN;
    const double q = S.res_cycle0 > 0.0 ? S.res_true / S.res_cycle0 : 0.0;
    const int cur = S.mode, other = cur == PM_CNN ? PM_MG : PM_CNN;
    if (S.probing) {
        S.probing = 0;
        if (q < S.q_base) {
            S.probe_gap = 0;
            S.probe_wait = 0;
            return cur;
        }
        S.probe_gap = S.probe_gap > 0 ? 2 * S.probe_gap : 2;
        S.probe_wait = S.probe_gap;
        return other;
    }
    S.q_base = q;
    if (judge && q > probe_ratio && S.probe_wait <= 0) {
        S.probing = 1;
        return other;
    }
    if (S.probe_wait > 0) S.probe_wait--;
    return cur;
}

// Start of a restart cycle: beta = ||r||, true relative residual, stopping test,
// and the masks of the RHS that use CNN+MG (actc) and MG-only (actm) in it.
__global__ void k_cycle_begin(const double2* __restrict__ parts, int npart, KState* __restrict__ st, int* done,
                              int* active, int* actc, int* actm, double* hist, int hist_len, double rtol,
                              int max_iters, int fixed, const int* __restrict__ caps, int cnn, int warm, int fallback,
                              double probe_ratio) {
    __shared__ double2 s_red[4];
    const int r = blockIdx.x;
    if (done[r]) {
        if (threadIdx.x == 0) {
            active[r] = actc[r] = actm[r] = 0;
            st[r].k = 0;  // a finished RHS takes no further x update
        }
        return;
    }
    double2 acc[1] = {make_double2(0.0, 0.0)};
    for (int p = threadIdx.x; p < npart; p += 256) acc[0] = zadd(acc[0], parts[(size_t)r * npart + p]);
    block_sum2<1>(acc, 1, s_red);
    if (threadIdx.x != 0) return;
    KState& S = st[r];
    const double beta = sqrt(acc[0].x);
    S.res_true = beta / S.bnorm;
    if (hist && S.iters < hist_len) hist[(size_t)r * hist_len + S.iters] = S.res_true;
    const bool bad = !(beta == beta);
    if (bad) S.breakdown = 1;
    if (!fixed && S.res_true <= rtol) S.converged = 1;
    // the previous cycle stopped on its residual estimate but the FP64 residual
    // says otherwise: ask the next cycles for a 10x deeper reduction
    if (S.ended_by_est && !S.converged) S.tol_scale = fmax(S.tol_scale * 0.1, 1e-4);
    S.ended_by_est = 0;
    const int cap = caps ? min(caps[r], max_iters) : max_iters;
    if (bad || S.converged || S.iters >= cap || beta == 0.0) {
        done[r] = 1;
        active[r] = actc[r] = actm[r] = 0;
        S.k = 0;  // the last cycle's correction is already in x
        return;
    }
    S.sig[0] = 1.0 / beta;
    for (int q = 0; q < MAXV; ++q) S.g[q] = make_double2(0.0, 0.0);
    S.g[0] = make_double2(beta, 0.0);
    S.k = 0;
    if (cnn) {
        S.mode = next_mode(S, warm, fallback, probe_ratio);
        if (S.mode == PM_MG) S.mg_cycles++;
    }
    S.res_cycle0 = S.res_true;
    const int c = cnn && S.mode == PM_CNN;
    active[r] = 1;
    actc[r] = c;
    actm[r] = !c;
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
template <int NJ>
static void launch_op_dots_t(dim3 g, dim3 b, hipStream_t s, const float2* Z, size_t zs, float2* V, size_t vs, int j,
                             const float2* cf, const int* inst, int n, float ih2, double2* parts, int np,
                             const int* act) {
    hipLaunchKernelGGL(k_op_dots<NJ>, g, b, 0, s, Z, zs, (const float2*)V, V, vs, j, cf, inst, n, ih2, parts, np,
                       act);
}
template <int NJ>
static void launch_ortho_t(dim3 g, dim3 b, hipStream_t s, float2* V, size_t vs, int j, const KState* st, int n,
                           double2* parts, int np, const int* act) {
    hipLaunchKernelGGL(k_ortho<NJ>, g, b, 0, s, V, vs, j, st, n, parts, np, act);
}

hh_status SolveWork::prepare(hh_ctx* c, hh_model* md, int nrhs_, int restart_, int hist_len_, bool cnn) {
    nrhs = nrhs_;
    restart = restart_;
    hist_len = hist_len_;
    n = md->lev[0].n;
    npart = kblocks(n);
    const size_t nn = (size_t)n * n;
    HH_TRY(V.ensure(c, (size_t)nrhs * (restart + 1) * nn * sizeof(float2)));
    HH_TRY(Z.ensure(c, (size_t)nrhs * restart * nn * sizeof(float2)));
    HH_TRY(state.ensure(c, (size_t)nrhs * sizeof(KState)));
    HH_TRY(flags.ensure(c, (size_t)4 * nrhs * sizeof(int)));
    HH_TRY(parts.ensure(c, (size_t)nrhs * npart * MAXV * sizeof(double2)));
    HH_TRY(inst.ensure(c, (size_t)nrhs * sizeof(int)));
    HH_TRY(hist.ensure(c, (size_t)nrhs * hist_len * sizeof(double) + 8));
    HH_TRY(vwork.ensure(c, vcycle_workspace_bytes(md, nrhs, cnn) + 256));
    return HH_OK;
}

hh_status capture_stream(hh_ctx* c, hipStream_t* out) {
    if (!c->cap_stream) HH_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    *out = c->cap_stream;
    return HH_OK;
}

// Graphs of restart cycles, keyed by the cycle's launch configuration; owned
// by one solve call.
struct CycleGraphs {
    struct Entry {
        int len, warm, cnt_c, cnt_m, seen;
        hipGraphExec_t exec;
    };
    static constexpr size_t MAX_ENTRIES = 512;
    std::vector<Entry> v;
    ~CycleGraphs() {
        for (auto& e : v)
            if (e.exec) (void)hipGraphExecDestroy(e.exec);
    }
    // the entry of a configuration (created unseen); null once the cache is full
    Entry* find(int len, int warm, int cnt_c, int cnt_m) {
        for (auto& e : v)
            if (e.len == len && e.warm == warm && e.cnt_c == cnt_c && e.cnt_m == cnt_m) return &e;
        if (v.size() >= MAX_ENTRIES) return nullptr;
        v.reserve(MAX_ENTRIES);  // entries never move: callers keep pointers
        v.push_back({len, warm, cnt_c, cnt_m, 0, nullptr});
        return &v.back();
    }
    // record body's launches on the context's capture stream into e->exec
    template <class F>
    hh_status capture(hh_ctx* ctx, Entry* e, F&& body) {
        hipStream_t cs;
        HH_TRY(capture_stream(ctx, &cs));
        hipStream_t saved = ctx->stream;
        ctx->stream = cs;
        hipError_t be = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        hh_status s = be == hipSuccess ? body() : HH_ERR_HIP;
        hipGraph_t g = nullptr;
        const hipError_t ee = be == hipSuccess ? hipStreamEndCapture(cs, &g) : be;
        ctx->stream = saved;
        if (s == HH_OK && ee != hipSuccess) {
            set_error("graph capture of a restart cycle failed: %s", hipGetErrorString(ee));
            s = HH_ERR_HIP;
        }
        if (s == HH_OK) {
            const hipError_t ie = hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                e->exec = nullptr;
                set_error("graph instantiation of a restart cycle failed: %s", hipGetErrorString(ie));
                s = HH_ERR_HIP;
            }
        }
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
};

// One FGMRES(m) solve driven in phases, so that several solves (models of
// different sizes) can interleave their restart cycles on their own streams:
// start(); then per cycle begin_cycle() (restart residual, per-RHS decisions,
// flags to the host), wait_cycle() (reads them; tells whether every RHS is
// done) and run_cycle() (the cycle's launches, eager or from a graph).  Every
// phase launches on `stream` (the context's stream is switched to it meanwhile).
class FgmresRun {
  public:
    FgmresRun(hh_model* md, SolveWork& W, const BatchMap& bm, const float2* b, double2* x, const hh_solve_opts& o,
              PrecondFn precond_cnn, void* precond_user, hipStream_t stream)
        : md_(md), W_(W), bm_(bm), b_(b), x_(x), o_(o), pc_(precond_cnn), pu_(precond_user), stream_(stream) {}
    ~FgmresRun() {
        if (hflags_) (void)hipHostFree(hflags_);
    }
    hh_status start();
    hh_status begin_cycle();
    hh_status wait_cycle(bool* finished);
    hh_status run_cycle();
    bool fixed_done() const { return fixed_done_; }

  private:
    // switches the context's stream to this solve's stream for one phase
    struct StreamGuard {
        hh_ctx* c;
        hipStream_t saved;
        StreamGuard(hh_ctx* ctx, hipStream_t s) : c(ctx), saved(ctx->stream) { c->stream = s; }
        ~StreamGuard() { c->stream = saved; }
    };
    hh_model* md_;
    SolveWork& W_;
    BatchMap bm_;
    const float2* b_;
    double2* x_;
    hh_solve_opts o_;
    PrecondFn pc_;
    void* pu_;
    hipStream_t stream_;
    int* hflags_ = nullptr;  // pinned host copy of [done | actc | actm]
    CycleGraphs graphs_;
    int cycle_ = 0, cnt_c_ = 0, cnt_m_ = 0;
    bool warm_ = false, fixed_done_ = false;
};

hh_status FgmresRun::start() {
    StreamGuard g(md_->ctx, stream_);
    const int n = W_.n, nrhs = W_.nrhs, np = W_.npart;
    const dim3 blk(KT_X, KT_Y / KT_ROWS);
    const dim3 grd((n + KT_X - 1) / KT_X, (n + KT_Y - 1) / KT_Y, nrhs);
    KState* S = W_.state.as<KState>();
    int* done = W_.flags.as<int>();
    if (!hflags_) HH_HIP(hipHostMalloc((void**)&hflags_, (size_t)3 * nrhs * sizeof(int), hipHostMallocDefault));
    hipLaunchKernelGGL(k_norm2, grd, blk, 0, stream_, b_, n, W_.parts.as<double2>());
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_init_state, dim3(nrhs), dim3(256), 0, stream_, W_.parts.as<double2>(), np, S, done,
                       done + 3 * nrhs, W_.hist.as<double>(), W_.hist_len);
    HH_LAUNCH_CHECK();
    if (!o_.use_x0) HH_HIP(hipMemsetAsync(x_, 0, (size_t)nrhs * n * n * sizeof(double2), stream_));
    return HH_OK;
}

hh_status FgmresRun::begin_cycle() {
    StreamGuard g(md_->ctx, stream_);
    hh_ctx* ctx = md_->ctx;
    const int n = W_.n, nrhs = W_.nrhs, np = W_.npart;
    const size_t vstride = (size_t)(W_.restart + 1) * n * n;
    const dim3 blk(KT_X, KT_Y / KT_ROWS);
    const dim3 grd((n + KT_X - 1) / KT_X, (n + KT_Y - 1) / KT_Y, nrhs);
    const Level& L0 = md_->lev[0];
    int* done = W_.flags.as<int>();
    const bool fixed = o_.fixed_iters > 0;
    const bool cnn = pc_ != nullptr;
    warm_ = cnn && cycle_ == 0 && o_.warm_mg_iters > 0;
    {
        ProfScope ps(ctx, HH_K_RESTART);
        hipLaunchKernelGGL(k_residual64, grd, blk, 0, stream_, x_, b_, W_.V.as<float2>(), vstride,
                           coef64(md_), bm_.inst, n, 1.0 / (L0.h * L0.h), W_.parts.as<double2>(), done);
    }
    HH_LAUNCH_CHECK();
    {
        ProfScope ps(ctx, HH_K_SMALL);
        hipLaunchKernelGGL(k_cycle_begin, dim3(nrhs), dim3(256), 0, stream_, W_.parts.as<double2>(), np,
                           W_.state.as<KState>(), done, done + 3 * nrhs, done + nrhs, done + 2 * nrhs,
                           W_.hist.as<double>(), W_.hist_len, fixed ? 0.0 : o_.rtol,
                           fixed ? o_.fixed_iters : o_.max_iters, fixed ? 1 : 0, W_.caps_dev, cnn ? 1 : 0,
                           warm_ ? 1 : 0, o_.fallback, o_.probe_ratio);
    }
    HH_LAUNCH_CHECK();
    HH_HIP(hipMemcpyAsync(hflags_, done, (size_t)3 * nrhs * sizeof(int), hipMemcpyDeviceToHost, stream_));
    return HH_OK;
}

hh_status FgmresRun::wait_cycle(bool* finished) {
    HH_HIP(hipStreamSynchronize(stream_));
    const int nrhs = W_.nrhs;
    bool all = true;
    cnt_c_ = cnt_m_ = 0;
    for (int r = 0; r < nrhs; ++r) {
        all = all && hflags_[r];
        cnt_c_ += hflags_[nrhs + r];
        cnt_m_ += hflags_[2 * nrhs + r];
    }
    *finished = all || fixed_done_;
    return HH_OK;
}

hh_status FgmresRun::run_cycle() {
    StreamGuard guard(md_->ctx, stream_);
    hh_model* md = md_;
    SolveWork& W = W_;
    const hh_solve_opts& o = o_;
    const BatchMap& bm = bm_;
    PrecondFn precond_cnn = pc_;
    void* precond_user = pu_;
    double2* x = x_;
    const float2* b = b_;
    const int* inst_dev = bm.inst;
    hh_ctx* ctx = md->ctx;
    hipStream_t st = stream_;
    const int n = W.n, nrhs = W.nrhs;
    const size_t nn = (size_t)n * n;
    const size_t vstride = (size_t)(W.restart + 1) * nn, zstride = (size_t)W.restart * nn;
    const dim3 blk(KT_X, KT_Y / KT_ROWS);
    const dim3 grd((n + KT_X - 1) / KT_X, (n + KT_Y - 1) / KT_Y, nrhs);
    const int np = W.npart;
    const Level& L0 = md->lev[0];
    const float ih2 = (float)(1.0 / (L0.h * L0.h));
    float2* V = W.V.as<float2>();
    float2* Z = W.Z.as<float2>();
    KState* S = W.state.as<KState>();
    int* done = W.flags.as<int>();  // [done | actc | actm | active]
    int* actc = done + nrhs;
    int* actm = done + 2 * nrhs;
    int* act = done + 3 * nrhs;
    double2* parts = W.parts.as<double2>();
    double* hist = W.hist.as<double>();
    const int sig_stride = (int)(sizeof(KState) / sizeof(double));
    const bool fixed = o.fixed_iters > 0;
    const double rtol = fixed ? 0.0 : o.rtol;
    const int max_iters = fixed ? o.fixed_iters : o.max_iters;
    const int cnt_c = cnt_c_, cnt_m = cnt_m_;
    const bool warm = warm_;
    const bool any_c = cnt_c > 0, any_m = cnt_m > 0;
    // the active counts only fall during a cycle: upper bounds for the coarse solves
    BatchMap bmc = bm, bmm = bm;
    bmc.nact = cnt_c;
    bmm.nact = cnt_m;
    int len = W.restart;
    if (warm) len = std::min(len, o.warm_mg_iters);
    if (fixed) len = std::min(len, o.fixed_iters);
    // every launch of the cycle, on the context's current stream (a capture
    // stream while a graph is recorded)
    auto body = [&]() -> hh_status {
        hipStream_t s = ctx->stream;
            for (int j = 0; j < len; ++j) {
                const float2* vj = V + (size_t)j * nn;
                const double* sg =
                    reinterpret_cast<const double*>(reinterpret_cast<const char*>(S) + offsetof(KState, sig)) + j;
                float2* zj = Z + (size_t)j * nn;
                // z_j = M(v_j) on strided [rhs] views: CNN+MG for the RHS in actc,
                // MG-only for those in actm (warm start, probes, fallback)
                if (any_c)
                    HH_TRY(precond_cnn(precond_user, md, W, bmc, vj, vstride, sg, sig_stride, zj, zstride, actc));
                if (any_m) HH_TRY(precond_mg_strided(md, W, bmm, vj, vstride, sg, sig_stride, zj, zstride, actm));
                // w = A z_j, dots with v_0..v_j
                {
                    ProfScope ps(ctx, HH_K_OP_DOTS);
                    switch (j + 1) {
#define HH_OPD(NJ) case NJ: launch_op_dots_t<NJ>(grd, blk, s, zj, zstride, V, vstride, j, L0.coef.as<float2>(), inst_dev, n, ih2, parts, np, act); break;
                        HH_OPD(1) HH_OPD(2) HH_OPD(3) HH_OPD(4) HH_OPD(5) HH_OPD(6) HH_OPD(7) HH_OPD(8)
                        HH_OPD(9) HH_OPD(10) HH_OPD(11) HH_OPD(12) HH_OPD(13) HH_OPD(14) HH_OPD(15) HH_OPD(16)
#undef HH_OPD
                        default: set_error("restart too long"); return HH_ERR_ARG;
                    }
                }
                HH_LAUNCH_CHECK();
                {
                    ProfScope ps(ctx, HH_K_SMALL);
                    hipLaunchKernelGGL(k_arnoldi_col, dim3(nrhs), dim3(256), 0, s, parts, np, j, S, act);
                }
                HH_LAUNCH_CHECK();
                {
                    ProfScope ps(ctx, HH_K_ORTHO);
                    switch (j + 1) {
#define HH_ORT(NJ) case NJ: launch_ortho_t<NJ>(grd, blk, s, V, vstride, j, S, n, parts, np, act); break;
                        HH_ORT(1) HH_ORT(2) HH_ORT(3) HH_ORT(4) HH_ORT(5) HH_ORT(6) HH_ORT(7) HH_ORT(8)
                        HH_ORT(9) HH_ORT(10) HH_ORT(11) HH_ORT(12) HH_ORT(13) HH_ORT(14) HH_ORT(15) HH_ORT(16)
#undef HH_ORT
                        default: set_error("restart too long"); return HH_ERR_ARG;
                    }
                }
                HH_LAUNCH_CHECK();
                {
                    ProfScope ps(ctx, HH_K_SMALL);
                    hipLaunchKernelGGL(k_givens, dim3(nrhs), dim3(256), 0, s, parts, np, j, S, act, actc, actm, hist,
                                       W.hist_len, rtol, max_iters, W.caps_dev);
                }
                HH_LAUNCH_CHECK();
            }
            {
                ProfScope ps(ctx, HH_K_RESTART);
                hipLaunchKernelGGL(k_xupdate, grd, blk, 0, s, x, Z, zstride, S, n);
            }
            HH_LAUNCH_CHECK();
            return HH_OK;
    };
    // graph path: a configuration runs eagerly the first time (lazy set-up and
    // coarse-solve tuning happen there), is captured the second time and
    // replayed after that
    CycleGraphs::Entry* ge = nullptr;
    if (o.graph && !fixed && ctx->prof_class < 0) ge = graphs_.find(len, warm ? 1 : 0, cnt_c, cnt_m);
    if (ge && !ge->exec && ge->seen >= 1 && (!any_c || coarse_capturable(md, nrhs, cnt_c)) &&
        (!any_m || coarse_capturable(md, nrhs, cnt_m)))
        HH_TRY(graphs_.capture(ctx, ge, body));
    if (ge && ge->exec) {
        HH_HIP(hipGraphLaunch(ge->exec, st));
    } else {
        HH_TRY(body());
        if (ge) ge->seen++;
    }
    ++cycle_;
    if (fixed) {
        // one cycle only: mark everything done after the final residual
        hipLaunchKernelGGL(k_residual64, grd, blk, 0, st, x, b, V, vstride, coef64(md), inst_dev, n,
                           1.0 / (L0.h * L0.h), parts, nullptr);
        HH_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_cycle_begin, dim3(nrhs), dim3(256), 0, st, parts, np, S, done, act, actc, actm, hist,
                           W.hist_len, rtol, 0, 1, W.caps_dev, 0, 0, 0, 0.0);
        HH_LAUNCH_CHECK();
        fixed_done_ = true;
    }
    return HH_OK;
}

hh_status fgmres_solve(hh_model* md, SolveWork& W, const BatchMap& bm, const float2* b, double2* x,
                       const hh_solve_opts& o, PrecondFn precond_cnn, void* precond_user) {
    FgmresRun run(md, W, bm, b, x, o, precond_cnn, precond_user, md->ctx->stream);
    HH_TRY(run.start());
    for (;;) {
        HH_TRY(run.begin_cycle());
        bool fin = false;
        HH_TRY(run.wait_cycle(&fin));
        if (fin) break;
        HH_TRY(run.run_cycle());
        if (run.fixed_done()) break;
    }
    return HH_OK;
}

hh_status fgmres_solve_many(int nruns, hh_model* const* md, SolveWork* const* W, const BatchMap* bm,
                            const float2* const* b, double2* const* x, const hh_solve_opts& o, PrecondFn precond_cnn,
                            const hipStream_t* streams) {
    // several streams at once: no cooperative coarse-solve variants meanwhile
    struct Concurrent {
        hh_ctx* c;
        bool saved;
        Concurrent(hh_ctx* ctx, bool on) : c(ctx), saved(ctx->concurrent) { c->concurrent = on; }
        ~Concurrent() { c->concurrent = saved; }
    } conc(md[0]->ctx, nruns > 1);
    std::vector<std::unique_ptr<FgmresRun>> runs;
    for (int i = 0; i < nruns; ++i) {
        runs.emplace_back(new (std::nothrow) FgmresRun(md[i], *W[i], bm[i], b[i], x[i], o, precond_cnn,
                                                       precond_cnn ? (void*)md[i] : nullptr, streams[i]));
        if (!runs.back()) {
            set_error("out of host memory");
            return HH_ERR_NOMEM;
        }
        HH_TRY(runs.back()->start());
    }
    std::vector<int> live(nruns);
    for (int i = 0; i < nruns; ++i) live[i] = i;
    while (!live.empty()) {
        // all restart residuals and decisions first, then the waits, then the
        // cycles: the streams overlap each other's work
        for (int i : live) HH_TRY(runs[i]->begin_cycle());
        std::vector<int> next;
        for (int i : live) {
            bool fin = false;
            HH_TRY(runs[i]->wait_cycle(&fin));
            if (!fin) next.push_back(i);
        }
        live.swap(next);
        for (int i : live) HH_TRY(runs[i]->run_cycle());
    }
    return HH_OK;
}

// ||b - A x|| / ||b|| in FP64 for complex-double solutions x (the solve's own
// restart-residual kernel, without storing the residual)
hh_status residual_norms(hh_model* md, int nrhs, const BatchMap& bm, const float2* b, const double2* x,
                         double* rel_host) {
    hh_ctx* ctx = md->ctx;
    const Level& L0 = md->lev[0];
    const int n = L0.n, np = kblocks(n);
    const dim3 blk(KT_X, KT_Y / KT_ROWS);
    const dim3 grd((n + KT_X - 1) / KT_X, (n + KT_Y - 1) / KT_Y, nrhs);
    Buf parts;
    HH_TRY(parts.ensure(ctx, (size_t)2 * nrhs * np * sizeof(double2)));
    double2* pr = parts.as<double2>();
    double2* pb = pr + (size_t)nrhs * np;
    hipLaunchKernelGGL(k_residual64, grd, blk, 0, ctx->stream, x, b, nullptr, (size_t)0, coef64(md), bm.inst,
                       n, 1.0 / (L0.h * L0.h), pr, nullptr);
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_norm2, grd, blk, 0, ctx->stream, b, n, pb);
    HH_LAUNCH_CHECK();
    std::vector<double2> h((size_t)2 * nrhs * np);
    HH_HIP(hipMemcpyAsync(h.data(), pr, h.size() * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
    HH_HIP(hipStreamSynchronize(ctx->stream));
    for (int r = 0; r < nrhs; ++r) {
        double sr = 0.0, sb = 0.0;
        for (int q = 0; q < np; ++q) {
            sr += h[(size_t)r * np + q].x;
            sb += h[(size_t)(nrhs + r) * np + q].x;
        }
        rel_host[r] = sb > 0.0 ? sqrt(sr / sb) : sqrt(sr);
    }
    return HH_OK;
}

// MG-only preconditioner on strided [rhs] views of V and Z
hh_status precond_mg_strided(hh_model* md, SolveWork& W, const BatchMap& bm, const float2* v, size_t vstride,
                             const double* sig, int sig_stride, float2* z, size_t zstride, const int* act) {
    return launch_vcycle_strided(md, W.nrhs, bm, v, vstride, sig, sig_stride, nullptr, 0, z, zstride, W.vwork.ptr,
                                 act);
}

// ---------------------------------------------------------------------------
// FP64 residual norms without any allocation (hh_residual_norms_noalloc).
// The partial sums live in a fixed device array instead of a workspace, one
// copy per GPU; its device address is looked up once per device when a
// context is created there and kept per device.  Every call on a device shares
// that device's array (calls that overlap on one GPU race); each call writes
// every word it reads, so nothing has to start at zero.
// ---------------------------------------------------------------------------
constexpr int NOALLOC_MAX_RHS = 256;
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)1 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

hh_status noalloc_init(int device) {
    HH_ARG(device >= 0 && device < NOALLOC_MAX_DEVICES, "device index below 64");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return HH_OK;
    HH_HIP(hipSetDevice(device));
    void* p = nullptr;
    HH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
        set_error("hipGetSymbolAddress returned no address for the residual-norm scratch array");
        return HH_ERR_HIP;
    }
    g_scratch_dev[device] = p;
    return HH_OK;
}

// out[0] = sum of pr[q].x, out[1] = sum of pb[q].x over q < np (FP64; one workgroup)
__global__ void __launch_bounds__(256) k_sum_parts(const double2* __restrict__ pr, const double2* __restrict__ pb,
                                                   int np, double* __restrict__ out) {
    __shared__ double s_a[4], s_b[4];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int q = t; q < np; q += 256) {
        a += pr[q].x;
        b += pb[q].x;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if ((t & 63) == 0) {
        s_a[t >> 6] = a;
        s_b[t >> 6] = b;
    }
    __syncthreads();
    if (t == 0) {
        out[0] = (s_a[0] + s_a[1]) + (s_a[2] + s_a[3]);
        out[1] = (s_b[0] + s_b[1]) + (s_b[2] + s_b[3]);
    }
}

}  // namespace hh

using namespace hh;

extern "C" hh_status hh_residual_norms_noalloc(hh_ctx* ctx, hh_model* m, int nrhs, const int* inst_host,
                                               const void* b_dev, const void* x_dev, double* rel_host) {
    HH_ARG(ctx && m && b_dev && x_dev && rel_host, "null pointer");
    HH_ARG(m->ctx == ctx, "model belongs to another context");
    HH_ARG(nrhs >= 1 && nrhs <= NOALLOC_MAX_RHS, "nrhs in 1..256 (the fixed scratch holds 256 results)");
    if (inst_host)
        for (int r = 0; r < nrhs; ++r)
            HH_ARG(inst_host[r] >= 0 && inst_host[r] < m->ninst, "instance index out of range");
    const Level& L0 = m->lev[0];
    const int n = L0.n, np = kblocks(n);
    const size_t res_bytes = (size_t)2 * NOALLOC_MAX_RHS * sizeof(double);
    HH_ARG(res_bytes + (size_t)2 * np * sizeof(double2) <= NOALLOC_SCRATCH_BYTES,
           "grid too large for the fixed 1 MiB scratch (n <= 4096)");
    HH_ARG(ctx->device >= 0 && ctx->device < NOALLOC_MAX_DEVICES, "device index below 64");
    void* base = g_scratch_dev[ctx->device];
    if (!base) {
        set_error("the residual-norm scratch of device %d was not set up (hh_ctx_create does it)", ctx->device);
        return HH_ERR_STATE;
    }
    HH_HIP(hipSetDevice(ctx->device));
    double* res = reinterpret_cast<double*>(base);
    double2* pr = reinterpret_cast<double2*>(reinterpret_cast<unsigned char*>(base) + res_bytes);
    double2* pb = pr + np;
    const size_t nn = (size_t)n * n;
    const dim3 blk(KT_X, KT_Y / KT_ROWS);
    const dim3 grd((n + KT_X - 1) / KT_X, (n + KT_Y - 1) / KT_Y, 1);
    Coef64 cf = coef64(m);
    const float* kappa = cf.kappa;
    for (int r = 0; r < nrhs; ++r) {  // one right-hand side at a time: the partials are reused
        cf.kappa = kappa + (size_t)(inst_host ? inst_host[r] : 0) * nn;
        hipLaunchKernelGGL(k_residual64, grd, blk, 0, ctx->stream, (const double2*)x_dev + r * nn,
                           (const float2*)b_dev + r * nn, nullptr, (size_t)0, cf, nullptr, n, 1.0 / (L0.h * L0.h),
                           pr, nullptr);
        HH_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_norm2, grd, blk, 0, ctx->stream, (const float2*)b_dev + r * nn, n, pb);
        HH_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, ctx->stream, pr, pb, np, res + 2 * r);
        HH_LAUNCH_CHECK();
    }
    double h[2 * NOALLOC_MAX_RHS];
    HH_HIP(hipMemcpyAsync(h, res, (size_t)2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HH_HIP(hipStreamSynchronize(ctx->stream));
    for (int r = 0; r < nrhs; ++r) {
        const double sr = h[2 * r], sb = h[2 * r + 1];
        rel_host[r] = sb > 0.0 ? sqrt(sr / sb) : sqrt(sr);
    }
    return HH_OK;
}
