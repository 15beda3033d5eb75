// Iterative coarsest-grid solve (Sec. 3.4, after the approach the paper cites
// there): k steps of GMRES on the shifted-Laplacian operator A_SL of the
// coarsest level, right-preconditioned by its diagonal D (Jacobi), starting
// from zero, with no restart.  Every kernel is batched over the V-cycle's
// right-hand sides (blockIdx.z or blockIdx.x = RHS) and skips those that are
// not active.  The basis is stored unnormalised, V_j with v_j = sig_j V_j;
// Gram-Schmidt is classical (all dots of a step in one pass) with FP64 sums;
// the small least-squares problem is rotated by complex Givens rotations in
// FP64 and solved by back substitution; the solution is x = D^-1 sum_i y_i v_i.
#include "hh_internal.h"

namespace hh {

constexpr int CG_MAXK = 16;
constexpr int CG_TX = 64, CG_TY = 4;  // tile of 256 threads, one coarse point each

struct CGState {
    double sig[CG_MAXK + 1];             // v_j = sig_j V_j
    double2 g[CG_MAXK + 1];              // rotated right-hand side of min ||beta e1 - Hbar y||
    double2 R[CG_MAXK * (CG_MAXK + 1)];  // Hessenberg columns, rotated: column j at R[j (K+1) + i]
    double cs[CG_MAXK];                  // Givens rotations (c real, s complex)
    double2 sn[CG_MAXK];
    float2 coef[CG_MAXK];                // update coefficients y_i sig_i
    int len;                             // Hessenberg columns completed
    int stop;                            // breakdown (w = 0): the Krylov space holds the solution
};

// 256-thread block sum of a double (4 waves)
__device__ __forceinline__ double cg_block_sum(double v, double* s_w) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_w[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s_w[w];
    return t;  // valid in thread 0
}

__device__ __forceinline__ float2 cg_diag(float2 c, float beta, float dgv) {
    const float2 mv = mass_of(c, beta);
    return make_float2(dgv - mv.x, -mv.y);
}

// V_0 = b, partial sums of |b|^2
__global__ void __launch_bounds__(256) k_cg_start(const float2* __restrict__ b, float2* __restrict__ V, size_t vs,
                                                  int m, double2* __restrict__ parts, int nb,
                                                  const int* __restrict__ active) {
    __shared__ double s_w[4];
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const int x = blockIdx.x * CG_TX + (threadIdx.x % CG_TX), y = blockIdx.y * CG_TY + (threadIdx.x / CG_TX);
    const size_t mm = (size_t)m * m;
    double s = 0.0;
    if (x < m && y < m) {
        const size_t o = (size_t)y * m + x;
        const float2 v = b[(size_t)r * mm + o];
        V[(size_t)r * vs + o] = v;
        s = (double)v.x * v.x + (double)v.y * v.y;
    }
    s = cg_block_sum(s, s_w);
    if (threadIdx.x == 0)
        parts[((size_t)r * nb + blockIdx.y * gridDim.x + blockIdx.x) * (CG_MAXK + 1)] = make_double2(s, 0.0);
}

// beta = ||b||: the least-squares right-hand side and the first basis scale
__global__ void __launch_bounds__(256) k_cg_begin(const double2* __restrict__ parts, int nb, CGState* __restrict__ S,
                                                  const int* __restrict__ active) {
    __shared__ double s_w[4];
    const int r = blockIdx.x;
    if (active && !active[r]) return;
    double s = 0.0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) s += parts[((size_t)r * nb + q) * (CG_MAXK + 1)].x;
    s = cg_block_sum(s, s_w);
    if (threadIdx.x == 0) {
        CGState& st = S[r];
        const double beta = sqrt(s);
        for (int i = 0; i <= CG_MAXK; ++i) st.g[i] = make_double2(0.0, 0.0);
        st.g[0] = make_double2(beta, 0.0);
        st.sig[0] = beta > 0.0 ? 1.0 / beta : 0.0;
        st.len = 0;
        st.stop = beta > 0.0 ? 0 : 1;  // b = 0: x = 0
    }
}

// Arnoldi step j = NJ - 1: W = A_SL D^-1 v_j (written to V_{j+1}) and the partial
// sums of <V_i, W>, i = 0..j
template <int NJ>
__global__ void __launch_bounds__(256) k_cg_arnoldi(float2* __restrict__ V, size_t vs, const float2* __restrict__ coef,
                                                    const int* __restrict__ inst, int m, float ih2, float beta,
                                                    const CGState* __restrict__ S, double2* __restrict__ parts,
                                                    int nb, const int* __restrict__ active) {
    __shared__ double s_w[4];
    constexpr int j = NJ - 1;
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const CGState& st = S[r];
    if (st.stop || st.len != j) return;
    const int x = blockIdx.x * CG_TX + (threadIdx.x % CG_TX), y = blockIdx.y * CG_TY + (threadIdx.x / CG_TX);
    const size_t mm = (size_t)m * m;
    const float2* cf = coef + (size_t)(inst ? inst[r] : 0) * mm;
    float2* Vr = V + (size_t)r * vs;
    const float2* vj = Vr + (size_t)j * mm;
    const float sj = (float)st.sig[j];
    const float dgv = 4.f * ih2;
    double2 acc[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) acc[i] = make_double2(0.0, 0.0);
    if (x < m && y < m) {
        const size_t o = (size_t)y * m + x;
        // z = D^-1 v_j at the point and its four neighbours (zero outside)
        auto z_at = [&](int yy, int xx) -> float2 {
            if (yy < 0 || yy >= m || xx < 0 || xx >= m) return make_float2(0.f, 0.f);
            const size_t q = (size_t)yy * m + xx;
            return cdiv(cscale(vj[q], sj), cg_diag(cf[q], beta, dgv));
        };
        const float2 zc = z_at(y, x);
        const float2 nbs = cadd(cadd(z_at(y - 1, x), z_at(y + 1, x)), cadd(z_at(y, x - 1), z_at(y, x + 1)));
        const float2 mv = mass_of(cf[o], beta);
        const float2 w = csub(make_float2((4.f * zc.x - nbs.x) * ih2, (4.f * zc.y - nbs.y) * ih2), cmul(mv, zc));
        Vr[(size_t)(j + 1) * mm + o] = w;
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            const float2 vi = Vr[(size_t)i * mm + o];
            // conj(v_i) w
            acc[i].x += (double)vi.x * w.x + (double)vi.y * w.y;
            acc[i].y += (double)vi.x * w.y - (double)vi.y * w.x;
        }
    }
    const size_t pb = ((size_t)r * nb + blockIdx.y * gridDim.x + blockIdx.x) * (CG_MAXK + 1);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const double sx = cg_block_sum(acc[i].x, s_w);
        const double sy = cg_block_sum(acc[i].y, s_w);
        if (threadIdx.x == 0) parts[pb + i] = make_double2(sx, sy);
    }
}

// Hessenberg column j: h_ij = <v_i, W> = sig_i <V_i, W>
__global__ void __launch_bounds__(256) k_cg_col(const double2* __restrict__ parts, int nb, int j,
                                                CGState* __restrict__ S, const int* __restrict__ active) {
    __shared__ double s_w[4];
    const int r = blockIdx.x;
    if (active && !active[r]) return;
    CGState& st = S[r];
    if (st.stop || st.len != j) return;
    for (int i = 0; i <= j; ++i) {
        double sx = 0.0, sy = 0.0;
        for (int q = threadIdx.x; q < nb; q += blockDim.x) {
            const double2 p = parts[((size_t)r * nb + q) * (CG_MAXK + 1) + i];
            sx += p.x;
            sy += p.y;
        }
        sx = cg_block_sum(sx, s_w);
        sy = cg_block_sum(sy, s_w);
        if (threadIdx.x == 0) st.R[j * (CG_MAXK + 1) + i] = make_double2(st.sig[i] * sx, st.sig[i] * sy);
    }
}

// W -= sum_i h_ij v_i; partial sums of |W|^2
template <int NJ>
__global__ void __launch_bounds__(256) k_cg_ortho(float2* __restrict__ V, size_t vs, int m,
                                                  const CGState* __restrict__ S, double2* __restrict__ parts, int nb,
                                                  const int* __restrict__ active) {
    __shared__ double s_w[4];
    constexpr int j = NJ - 1;
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const CGState& st = S[r];
    if (st.stop || st.len != j) return;
    const int x = blockIdx.x * CG_TX + (threadIdx.x % CG_TX), y = blockIdx.y * CG_TY + (threadIdx.x / CG_TX);
    const size_t mm = (size_t)m * m;
    float2* Vr = V + (size_t)r * vs;
    double s = 0.0;
    if (x < m && y < m) {
        const size_t o = (size_t)y * m + x;
        float2 w = Vr[(size_t)(j + 1) * mm + o];
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            const double2 h = st.R[j * (CG_MAXK + 1) + i];
            const float2 c = make_float2((float)(h.x * st.sig[i]), (float)(h.y * st.sig[i]));
            w = csub(w, cmul(c, Vr[(size_t)i * mm + o]));
        }
        Vr[(size_t)(j + 1) * mm + o] = w;
        s = (double)w.x * w.x + (double)w.y * w.y;
    }
    s = cg_block_sum(s, s_w);
    if (threadIdx.x == 0)
        parts[((size_t)r * nb + blockIdx.y * gridDim.x + blockIdx.x) * (CG_MAXK + 1)] = make_double2(s, 0.0);
}

// h_{j+1,j} = ||W||; the earlier rotations applied to column j, a new one
// annihilating h_{j+1,j}, and the least-squares right-hand side rotated along
__global__ void __launch_bounds__(256) k_cg_givens(const double2* __restrict__ parts, int nb, int j,
                                                   CGState* __restrict__ S, const int* __restrict__ active) {
    __shared__ double s_w[4];
    const int r = blockIdx.x;
    if (active && !active[r]) return;
    CGState& st = S[r];
    if (st.stop || st.len != j) return;
    double s = 0.0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) s += parts[((size_t)r * nb + q) * (CG_MAXK + 1)].x;
    s = cg_block_sum(s, s_w);
    if (threadIdx.x != 0) return;
    const double hn = sqrt(s);
    double2* col = st.R + j * (CG_MAXK + 1);
    col[j + 1] = make_double2(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        const double2 a = col[i], b = col[i + 1];
        const double c = st.cs[i];
        const double2 sn = st.sn[i];
        col[i] = zadd(make_double2(c * a.x, c * a.y), zmul(sn, b));
        col[i + 1] = zsub(make_double2(c * b.x, c * b.y), zmul(zconj(sn), a));
    }
    const double2 a = col[j], b = col[j + 1];
    const double na = sqrt(a.x * a.x + a.y * a.y), nbv = sqrt(b.x * b.x + b.y * b.y);
    const double rho = sqrt(na * na + nbv * nbv);
    double c = 1.0;
    double2 sn = make_double2(0.0, 0.0), ph = make_double2(1.0, 0.0);
    if (rho > 0.0) {
        if (na > 0.0) ph = make_double2(a.x / na, a.y / na);
        c = na / rho;
        sn = zmul(ph, make_double2(b.x / rho, -b.y / rho));  // (a/|a|) conj(b) / rho
    }
    st.cs[j] = c;
    st.sn[j] = sn;
    col[j] = make_double2(ph.x * rho, ph.y * rho);
    col[j + 1] = make_double2(0.0, 0.0);
    const double2 gj = st.g[j];
    st.g[j + 1] = zmul(make_double2(-sn.x, sn.y), gj);  // -conj(s) g_j
    st.g[j] = make_double2(c * gj.x, c * gj.y);
    st.sig[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
    st.len = j + 1;
    if (!(hn > 0.0) || !(rho > 0.0)) st.stop = 1;
}

// y = R^-1 g by back substitution; update coefficients y_i sig_i
__global__ void k_cg_finish(CGState* __restrict__ S, int nrhs, const int* __restrict__ active) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs || (active && !active[r])) return;
    CGState& st = S[r];
    double2 y[CG_MAXK];
    const int L = st.len;
    for (int i = L - 1; i >= 0; --i) {
        double2 t = st.g[i];
        for (int k = i + 1; k < L; ++k) t = zsub(t, zmul(st.R[k * (CG_MAXK + 1) + i], y[k]));
        const double2 d = st.R[i * (CG_MAXK + 1) + i];
        y[i] = (d.x != 0.0 || d.y != 0.0) ? zdiv(t, d) : make_double2(0.0, 0.0);
    }
    for (int i = 0; i < CG_MAXK; ++i)
        st.coef[i] = i < L ? make_float2((float)(y[i].x * st.sig[i]), (float)(y[i].y * st.sig[i]))
                           : make_float2(0.f, 0.f);
}

// x = D^-1 sum_{i < len} y_i sig_i V_i
__global__ void __launch_bounds__(256) k_cg_update(const float2* __restrict__ V, size_t vs,
                                                   const float2* __restrict__ coef, const int* __restrict__ inst,
                                                   int m, float ih2, float beta, const CGState* __restrict__ S,
                                                   float2* __restrict__ x, const int* __restrict__ active) {
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const int xx = blockIdx.x * CG_TX + (threadIdx.x % CG_TX), yy = blockIdx.y * CG_TY + (threadIdx.x / CG_TX);
    if (xx >= m || yy >= m) return;
    const size_t mm = (size_t)m * m, o = (size_t)yy * m + xx;
    const CGState& st = S[r];
    const float2* Vr = V + (size_t)r * vs;
    float2 acc = make_float2(0.f, 0.f);
    for (int i = 0; i < st.len; ++i) acc = cadd(acc, cmul(st.coef[i], Vr[(size_t)i * mm + o]));
    const float2* cf = coef + (size_t)(inst ? inst[r] : 0) * mm;
    x[(size_t)r * mm + o] = cdiv(acc, cg_diag(cf[o], beta, 4.f * ih2));
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int cg_blocks(int m) { return ((m + CG_TX - 1) / CG_TX) * ((m + CG_TY - 1) / CG_TY); }

size_t coarse_gmres_bytes(const hh_model* md, int nrhs) {
    const int K = md->d.coarse_iters;
    if (K <= 0) return 0;
    const size_t m = md->lev[md->nlev - 1].n;
    return (size_t)nrhs * (K + 1) * m * m * sizeof(float2) + 256 +
           (size_t)nrhs * cg_blocks((int)m) * (CG_MAXK + 1) * sizeof(double2) + 256 +
           (size_t)nrhs * sizeof(CGState) + 256;
}

int coarse_gmres_max_iters() { return CG_MAXK; }

template <int NJ>
static void cg_step(hipStream_t st, dim3 grd, float2* V, size_t vs, const float2* coef, const int* inst, int m,
                    float ih2, float beta, CGState* S, double2* parts, int nb, int nrhs, const int* active) {
    hipLaunchKernelGGL(k_cg_arnoldi<NJ>, grd, dim3(256), 0, st, V, vs, coef, inst, m, ih2, beta, S, parts, nb,
                       active);
    hipLaunchKernelGGL(k_cg_col, dim3(nrhs), dim3(256), 0, st, parts, nb, NJ - 1, S, active);
    hipLaunchKernelGGL(k_cg_ortho<NJ>, grd, dim3(256), 0, st, V, vs, m, S, parts, nb, active);
    hipLaunchKernelGGL(k_cg_givens, dim3(nrhs), dim3(256), 0, st, parts, nb, NJ - 1, S, active);
}

hh_status launch_coarse_gmres(hh_model* md, int nrhs, const int* inst, const float2* bc, float2* xc,
                              const int* active, void* work) {
    const int K = md->d.coarse_iters;
    const Level& lc = md->lev[md->nlev - 1];
    const int m = lc.n, nb = cg_blocks(m);
    const size_t vs = (size_t)(K + 1) * m * m;
    char* q = (char*)work;
    float2* V = (float2*)q;
    q += (size_t)nrhs * vs * sizeof(float2);
    q = (char*)(((uintptr_t)q + 255) & ~(uintptr_t)255);
    double2* parts = (double2*)q;
    q += (size_t)nrhs * nb * (CG_MAXK + 1) * sizeof(double2);
    q = (char*)(((uintptr_t)q + 255) & ~(uintptr_t)255);
    CGState* S = (CGState*)q;
    const float ih2 = (float)(1.0 / (lc.h * lc.h)), beta = (float)md->d.sl_beta;
    const float2* coef = lc.coef.as<float2>();
    hipStream_t st = md->ctx->stream;
    const dim3 grd((m + CG_TX - 1) / CG_TX, (m + CG_TY - 1) / CG_TY, nrhs);
    hipLaunchKernelGGL(k_cg_start, grd, dim3(256), 0, st, bc, V, vs, m, parts, nb, active);
    hipLaunchKernelGGL(k_cg_begin, dim3(nrhs), dim3(256), 0, st, parts, nb, S, active);
    HH_LAUNCH_CHECK();
    for (int j = 0; j < K; ++j) {
        switch (j + 1) {
#define HH_CG(NJ) case NJ: cg_step<NJ>(st, grd, V, vs, coef, inst, m, ih2, beta, S, parts, nb, nrhs, active); break;
            HH_CG(1) HH_CG(2) HH_CG(3) HH_CG(4) HH_CG(5) HH_CG(6) HH_CG(7) HH_CG(8)
            HH_CG(9) HH_CG(10) HH_CG(11) HH_CG(12) HH_CG(13) HH_CG(14) HH_CG(15) HH_CG(16)
#undef HH_CG
            default: set_error("coarse GMRES: more than %d steps", CG_MAXK); return HH_ERR_ARG;
        }
        HH_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_cg_finish, dim3((nrhs + 63) / 64), dim3(64), 0, st, S, nrhs, active);
    hipLaunchKernelGGL(k_cg_update, grd, dim3(256), 0, st, V, vs, coef, inst, m, ih2, beta, S, xc, active);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

}  // namespace hh
