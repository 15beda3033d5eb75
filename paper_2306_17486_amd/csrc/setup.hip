// Per-slowness-model setup: coefficient fields on every multigrid level and the
// exact factorisation of the coarsest shifted-Laplacian operator.
#include "hh_internal.h"

namespace hh {

// Level-0 coefficients {omega^2 kappa^2, gamma}: gamma = gamma0 plus the
// quadratic absorbing ramp ((w - d)/w)^2 * gmax at distance d < w from the
// nearest edge (Sec. 3.1).
__global__ void k_coef0(const float* __restrict__ kappa, float2* __restrict__ coef, int n, double omega,
                        int abl_w, double gmax, double gamma0) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int inst = blockIdx.z;
    if (j >= n) return;
    const size_t off = ((size_t)inst * n + i) * n + j;
    const double k = kappa[off];
    int d = min(min(i, n - 1 - i), min(j, n - 1 - j));
    double g = gamma0;
    if (d < abl_w) {
        double t = (double)(abl_w - d) / abl_w;
        g += gmax * t * t;
    }
    coef[off] = make_float2((float)(omega * omega * k * k), (float)g);
}

// Full weighting of a coefficient field with edge-replicating padding (eq. 8
// kernel, coarse I on fine 2I).
__global__ void k_coef_restrict(const float2* __restrict__ fine, float2* __restrict__ coarse, int nf) {
    const int nc = nf >> 1;
    const int J = blockIdx.x * blockDim.x + threadIdx.x;
    const int I = blockIdx.y;
    const int inst = blockIdx.z;
    if (J >= nc) return;
    const float2* f = fine + (size_t)inst * nf * nf;
    const float w1[3] = {0.25f, 0.5f, 0.25f};
    float sx = 0.f, sy = 0.f;
    for (int a = 0; a < 3; ++a) {
        int y = min(max(2 * I + a - 1, 0), nf - 1);
        for (int b = 0; b < 3; ++b) {
            int x = min(max(2 * J + b - 1, 0), nf - 1);
            float w = w1[a] * w1[b];
            float2 v = f[(size_t)y * nf + x];
            sx += w * v.x;
            sy += w * v.y;
        }
    }
    coarse[((size_t)inst * nc + I) * nc + J] = make_float2(sx, sy);
}

// ---------------------------------------------------------------------------
// Coarsest-level direct solver.  The shifted operator on an m x m grid is block
// tridiagonal in grid rows: diagonal blocks T_k (tridiagonal, 4/H^2 - mass on
// the diagonal, -1/H^2 off it) and off-diagonal blocks -c I with c = 1/H^2.
// The rows are eliminated from both ends towards the middle row p = m/2
// ("burn at both ends"), which halves the sequential chain:
//   top:    S_0 = T_0,         S_k = T_k - c^2 S_{k-1}^{-1}   (k = 0 .. p-1)
//   bottom: S_{m-1} = T_{m-1}, S_k = T_k - c^2 S_{k+1}^{-1}   (k = m-1 .. p+1)
//   middle: S_p = T_p - c^2 S_{p-1}^{-1} - c^2 S_{p+1}^{-1}
// The inverses Q_k = S_k^{-1} are formed in FP64 (in-place Gauss-Jordan without
// pivoting) and stored transposed in complex single precision:
// QT[k][j][i] = Q_k[i][j].  -i A_SL has a positive definite Hermitian part
// (omega^2 kappa^2 (gamma + beta) > 0 on the diagonal), which keeps every Schur
// complement nonsingular without pivoting.
// ---------------------------------------------------------------------------

// A <- T_k - c^2 (P1 + P2)   (P1, P2 may be null)
__device__ void build_schur(double2* A, const double2* P1, const double2* P2, const float2* cf, int k, int m,
                            double c, double beta) {
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        int i = e / m, j = e - i * m;
        double2 v = make_double2(0.0, 0.0);
        if (P1) v = zadd(v, P1[e]);
        if (P2) v = zadd(v, P2[e]);
        v = make_double2(-c * c * v.x, -c * c * v.y);
        if (i == j) {
            float2 cc = cf[(size_t)k * m + i];
            double w2k2 = cc.x, g = cc.y;
            // diagonal: 4c - omega^2 kappa^2 (1 - i (gamma + beta))
            v.x += 4.0 * c - w2k2;
            v.y += w2k2 * (g + beta);
        } else if (j == i - 1 || j == i + 1) {
            v.x += -c;
        }
        A[e] = v;
    }
    __syncthreads();
}

// In-place Gauss-Jordan inversion without pivoting (one workgroup), then store
// the transpose in single precision.
__device__ void invert_store(double2* A, float2* Qk, int m) {
    __shared__ double2 piv_s;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int p = 0; p < m; ++p) {
        if (tid == 0) {
            double2 a = A[(size_t)p * m + p];
            double den = a.x * a.x + a.y * a.y;
            piv_s = make_double2(a.x / den, -a.y / den);
        }
        __syncthreads();
        const double2 piv = piv_s;
        for (int j = tid; j < m; j += nt)
            if (j != p) A[(size_t)p * m + j] = zmul(A[(size_t)p * m + j], piv);
        __syncthreads();
        for (int e = tid; e < m * m; e += nt) {
            int i = e / m, j = e - i * m;
            if (i == p || j == p) continue;
            A[e] = zsub(A[e], zmul(A[(size_t)i * m + p], A[(size_t)p * m + j]));
        }
        __syncthreads();
        for (int i = tid; i < m; i += nt) {
            if (i != p) {
                double2 a = A[(size_t)i * m + p];
                A[(size_t)i * m + p] = zmul(make_double2(-a.x, -a.y), piv);
            }
        }
        if (tid == 0) A[(size_t)p * m + p] = piv;
        __syncthreads();
    }
    for (int e = tid; e < m * m; e += nt) {
        int i = e / m, j = e - i * m;
        double2 v = A[e];
        Qk[(size_t)j * m + i] = make_float2((float)v.x, (float)v.y);
    }
    __syncthreads();
}

// blockIdx.x = instance, blockIdx.y = 0 (top chain) or 1 (bottom chain).
// Scratch S per instance: [3][m][m] FP64 (top, bottom, middle).
__global__ void __launch_bounds__(1024) k_coarse_factor_ends(const float2* __restrict__ coef, double2* __restrict__ S,
                                                             float2* __restrict__ QT, int m, int p, double H,
                                                             double beta) {
    const int inst = blockIdx.x;
    const bool top = blockIdx.y == 0;
    const double c = 1.0 / (H * H);
    const size_t mm = (size_t)m * m;
    const float2* cf = coef + (size_t)inst * mm;
    double2* A = S + (size_t)inst * 3 * mm + (top ? 0 : mm);
    float2* Q = QT + (size_t)inst * mm * m;
    if (top) {
        for (int k = 0; k < p; ++k) {
            build_schur(A, k > 0 ? A : nullptr, nullptr, cf, k, m, c, beta);
            invert_store(A, Q + (size_t)k * mm, m);
        }
    } else {
        for (int k = m - 1; k > p; --k) {
            build_schur(A, k < m - 1 ? A : nullptr, nullptr, cf, k, m, c, beta);
            invert_store(A, Q + (size_t)k * mm, m);
        }
    }
}

__global__ void __launch_bounds__(1024) k_coarse_factor_mid(const float2* __restrict__ coef, double2* __restrict__ S,
                                                            float2* __restrict__ QT, int m, int p, double H,
                                                            double beta) {
    const int inst = blockIdx.x;
    const double c = 1.0 / (H * H);
    const size_t mm = (size_t)m * m;
    double2* base = S + (size_t)inst * 3 * mm;
    double2* A = base + 2 * mm;
    build_schur(A, p > 0 ? base : nullptr, p < m - 1 ? base + mm : nullptr, coef + (size_t)inst * mm, p, m, c, beta);
    invert_store(A, QT + (size_t)inst * mm * m + (size_t)p * mm, m);
}

hh_status setup_coefficients(hh_model* md, const float* kappa_dev) {
    hipStream_t st = md->ctx->stream;
    const hh_model_desc& d = md->d;
    Level& L0 = md->lev[0];
    {
        dim3 blk(256), grd((L0.n + 255) / 256, L0.n, md->ninst);
        hipLaunchKernelGGL(k_coef0, grd, blk, 0, st, kappa_dev, L0.coef.as<float2>(), L0.n, d.omega,
                           d.abl_width, d.abl_gamma_max, d.gamma0);
        HH_LAUNCH_CHECK();
    }
    for (int l = 1; l < md->nlev; ++l) {
        int nc = md->lev[l].n;
        dim3 blk(256), grd((nc + 255) / 256, nc, md->ninst);
        hipLaunchKernelGGL(k_coef_restrict, grd, blk, 0, st, md->lev[l - 1].coef.as<float2>(),
                           md->lev[l].coef.as<float2>(), md->lev[l - 1].n);
        HH_LAUNCH_CHECK();
    }
    return HH_OK;
}

hh_status setup_coarse_factors(hh_model* md) {
    hh_ctx* ctx = md->ctx;
    const Level& C = md->lev[md->nlev - 1];
    const int m = C.n;
    const int p = m / 2;
    md->m = m;
    HH_TRY(md->coarseQT.ensure(ctx, (size_t)md->ninst * m * m * m * sizeof(float2)));
    Buf S;
    HH_TRY(S.ensure(ctx, (size_t)md->ninst * 3 * m * m * sizeof(double2)));
    hipLaunchKernelGGL(k_coarse_factor_ends, dim3(md->ninst, 2), dim3(1024), 0, ctx->stream, C.coef.as<float2>(),
                       S.as<double2>(), md->coarseQT.as<float2>(), m, p, C.h, md->d.sl_beta);
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_coarse_factor_mid, dim3(md->ninst), dim3(1024), 0, ctx->stream, C.coef.as<float2>(),
                       S.as<double2>(), md->coarseQT.as<float2>(), m, p, C.h, md->d.sl_beta);
    HH_LAUNCH_CHECK();
    // S is released when this function returns: order the free after the kernels.
    HH_HIP(hipStreamSynchronize(ctx->stream));
    return HH_OK;
}

}  // namespace hh
