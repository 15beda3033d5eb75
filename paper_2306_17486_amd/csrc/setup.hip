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
    const double g = abl_gamma(i, j, n, abl_w, gmax, gamma0);
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

// In-place Gauss-Jordan inversion without pivoting (one workgroup).
__device__ void invert_inplace(double2* A, int m) {
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
}

// ... then store the transpose in single precision
__device__ void invert_store(double2* A, float2* Qk, int m) {
    invert_inplace(A, m);
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
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

// ---------------------------------------------------------------------------
// One level of cyclic reduction before the two-ended elimination.  With V_j =
// T_{2j+1}^{-1} (odd grid rows, j < Mo = floor(m/2)), eliminating the odd rows
// leaves a block-tridiagonal system on the even rows 2j, j < M = ceil(m/2):
//   D_j = T_{2j} - c^2 ([j >= 1] V_{j-1} + [j < Mo] V_j),  L_j = -c^2 V_{j-1},  U_j = -c^2 V_j,
//   b'_j = b_{2j} + c ([j >= 1] V_{j-1} b_{2j-1} + [j < Mo] V_j b_{2j+1}),
// and the odd rows follow from x_{2j+1} = V_j (b_{2j+1} + c x_{2j} + c x_{2j+2}).
// The reduced system is eliminated from both ends towards p = M/2:
//   top (j < p):      S_j = D_j - c^4 V_{j-1} Q_{j-1} V_{j-1},  P_j = c^2 Q_j V_{j-1},  R_j = c^2 Q_j V_j
//   bottom (j > p):   S_j = D_j - c^4 V_j Q_{j+1} V_j,          P_j = c^2 Q_j V_j,      R_j = c^2 Q_j V_{j-1}
//   middle:           S_p = D_p - c^4 V_{p-1} Q_{p-1} V_{p-1} - c^4 V_p Q_{p+1} V_p,
//                     P_p = c^2 Q_p V_{p-1},  R_p = c^2 Q_p V_p
// with Q_j = S_j^{-1}, so that the solve is
//   g_j = Q_j b'_j;  y_j = g_j + P_j y_{j-/+1} (forward from each end);
//   x_p = g_p + P_p y_{p-1} + R_p y_{p+1};  x_j = y_j + R_j x_{j+/-1} (backward).
// Factors per instance, complex single, transposed (slot[c][r] = M[r][c]):
// slots j (Q_j), M + j (P_j), 2M + j (R_j), 3M + j (V_j).
// ---------------------------------------------------------------------------
static inline __device__ __host__ int cr_M(int m) { return (m + 1) / 2; }
static inline __device__ __host__ int cr_Mo(int m) { return m / 2; }

// A <- T_k (the shifted operator's grid-row block), dense FP64
__device__ void build_tblock(double2* A, const float2* cf, int k, int m, double c, double beta) {
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int i = e / m, j = e - i * m;
        double2 v = make_double2(0.0, 0.0);
        if (i == j) {
            const float2 cc = cf[(size_t)k * m + i];
            const double w2k2 = cc.x, g = cc.y;
            v.x = 4.0 * c - w2k2;
            v.y = w2k2 * (g + beta);
        } else if (j == i - 1 || j == i + 1) {
            v.x = -c;
        }
        A[e] = v;
    }
    __syncthreads();
}

// C (+)= alpha A B for m x m FP64 complex matrices (row-major), one workgroup,
// 32 x 32 output tiles through LDS.  C must not alias A or B.
__device__ void zgemm_wg(double2* C, const double2* A, const double2* B, int m, double alpha, bool accumulate) {
    constexpr int T = 32;
    __shared__ double2 sa[T][T + 1];
    __shared__ double2 sb[T][T + 1];
    const int tid = threadIdx.x;  // blockDim.x == 1024: one output entry of the tile per thread
    const int ty = tid / T, tx = tid % T;
    const int nt = (m + T - 1) / T;
    for (int bi = 0; bi < nt; ++bi)
        for (int bj = 0; bj < nt; ++bj) {
            double2 acc = make_double2(0.0, 0.0);
            for (int bk = 0; bk < nt; ++bk) {
                const int ar = bi * T + ty, ac = bk * T + tx;
                const int br = bk * T + ty, bc = bj * T + tx;
                sa[ty][tx] = (ar < m && ac < m) ? A[(size_t)ar * m + ac] : make_double2(0.0, 0.0);
                sb[ty][tx] = (br < m && bc < m) ? B[(size_t)br * m + bc] : make_double2(0.0, 0.0);
                __syncthreads();
#pragma unroll 8
                for (int k = 0; k < T; ++k) acc = zadd(acc, zmul(sa[ty][k], sb[k][tx]));
                __syncthreads();
            }
            const int r = bi * T + ty, cc = bj * T + tx;
            if (r < m && cc < m) {
                const double2 v = make_double2(alpha * acc.x, alpha * acc.y);
                C[(size_t)r * m + cc] = accumulate ? zadd(C[(size_t)r * m + cc], v) : v;
            }
        }
    __syncthreads();
}

// store alpha * A (FP64, row-major) transposed in single precision
__device__ void store_slot(const double2* A, float2* slot, int m, double alpha) {
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int i = e / m, j = e - i * m;
        const double2 v = A[e];
        slot[(size_t)j * m + i] = make_float2((float)(alpha * v.x), (float)(alpha * v.y));
    }
    __syncthreads();
}


// V_j = T_{2j+1}^{-1}: blockIdx.x = j (< Mo), blockIdx.y = instance.
// Vd: FP64 copies [inst][Mo][m][m] (kept for the chain factorisation).
__global__ void __launch_bounds__(1024) k_cr_vinv(const float2* __restrict__ coef, double2* __restrict__ Vd,
                                                  float2* __restrict__ F, int m, double H, double beta) {
    const int j = blockIdx.x, inst = blockIdx.y;
    const int M = cr_M(m), Mo = cr_Mo(m);
    const size_t mm = (size_t)m * m;
    const double c = 1.0 / (H * H);
    double2* V = Vd + ((size_t)inst * Mo + j) * mm;
    build_tblock(V, coef + (size_t)inst * mm, 2 * j + 1, m, c, beta);
    invert_inplace(V, m);
    store_slot(V, F + ((size_t)inst * 4 * M + 3 * M + j) * mm, m, 1.0);
}

// A <- D_j = T_{2j} - c^2 ([j >= 1] V_{j-1} + [j < Mo] V_j)
__device__ void build_dblock(double2* A, const float2* cf, const double2* Vinst, int j, int m, double c,
                             double beta) {
    const int Mo = cr_Mo(m);
    const size_t mm = (size_t)m * m;
    build_tblock(A, cf, 2 * j, m, c, beta);
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        double2 v = A[e];
        if (j >= 1) {
            const double2 a = Vinst[(size_t)(j - 1) * mm + e];
            v.x -= c * c * a.x;
            v.y -= c * c * a.y;
        }
        if (j < Mo) {
            const double2 a = Vinst[(size_t)j * mm + e];
            v.x -= c * c * a.x;
            v.y -= c * c * a.y;
        }
        A[e] = v;
    }
    __syncthreads();
}

// The two chains of the reduced system: blockIdx.x = instance, blockIdx.y = 0 (top) / 1 (bottom).
// Scratch W per instance: [6][m][m] FP64: A, Qprev (top), A, Qprev (bottom), T1, T2 (temporaries
// of the top chain; the bottom chain uses the next two) -- laid out as [chain][3][m][m].
__global__ void __launch_bounds__(1024) k_cr_chain(const float2* __restrict__ coef, const double2* __restrict__ Vd,
                                                   double2* __restrict__ W, float2* __restrict__ F, int m,
                                                   double H, double beta) {
    const int inst = blockIdx.x;
    const bool top = blockIdx.y == 0;
    const int M = cr_M(m), Mo = cr_Mo(m), p = M / 2;
    const size_t mm = (size_t)m * m;
    const double c = 1.0 / (H * H), c2 = c * c;
    const float2* cf = coef + (size_t)inst * mm;
    const double2* Vi = Vd + (size_t)inst * Mo * mm;
    double2* base = W + ((size_t)inst * 2 + (top ? 0 : 1)) * 4 * mm;
    double2* A = base;            // S_j, then Q_j
    double2* Qp = base + mm;      // Q of the previous step
    double2* T1 = base + 2 * mm;  // temporaries
    double2* T2 = base + 3 * mm;
    float2* Fi = F + (size_t)inst * 4 * M * mm;
    const int first = top ? 0 : M - 1, last = top ? p - 1 : p + 1, dir = top ? 1 : -1;
    if (top ? (p < 1) : (M - 1 <= p)) return;  // empty chain
    for (int j = first;; j += dir) {
        build_dblock(A, cf, Vi, j, m, c, beta);
        if (j != first) {
            // the coupling block between j and the previous row: V_{j-1} (top) or V_j (bottom)
            const double2* Vc = Vi + (size_t)(top ? j - 1 : j) * mm;
            zgemm_wg(T1, Qp, Vc, m, 1.0, false);      // Q_prev V
            zgemm_wg(A, Vc, T1, m, -c2 * c2, true);    // S_j -= c^4 V Q_prev V
        }
        invert_inplace(A, m);                          // A = Q_j
        store_slot(A, Fi + (size_t)j * mm, m, 1.0);
        // P_j: couples to the previous row (exists unless j is the first of the chain)
        if (j != first) {
            const double2* Vc = Vi + (size_t)(top ? j - 1 : j) * mm;
            zgemm_wg(T2, A, Vc, m, c2, false);
            store_slot(T2, Fi + (size_t)(M + j) * mm, m, 1.0);
        }
        // R_j: couples to the next row towards the middle: V_j (top) or V_{j-1} (bottom)
        {
            const double2* Vn = Vi + (size_t)(top ? j : j - 1) * mm;
            zgemm_wg(T2, A, Vn, m, c2, false);
            store_slot(T2, Fi + (size_t)(2 * M + j) * mm, m, 1.0);
        }
        // keep Q_j for the next step (and for the middle row)
        for (int e = threadIdx.x; e < m * m; e += blockDim.x) Qp[e] = A[e];
        __syncthreads();
        if (j == last) break;
    }
}

// middle row: blockIdx.x = instance; uses the chains' last Q (W[.][0|1][1]).
__global__ void __launch_bounds__(1024) k_cr_mid(const float2* __restrict__ coef, const double2* __restrict__ Vd,
                                                 double2* __restrict__ W, double2* __restrict__ Wm,
                                                 float2* __restrict__ F, int m, double H, double beta) {
    const int inst = blockIdx.x;
    const int M = cr_M(m), Mo = cr_Mo(m), p = M / 2;
    const size_t mm = (size_t)m * m;
    const double c = 1.0 / (H * H), c2 = c * c;
    const double2* Vi = Vd + (size_t)inst * Mo * mm;
    const double2* Qtop = W + ((size_t)inst * 2 + 0) * 4 * mm + mm;
    const double2* Qbot = W + ((size_t)inst * 2 + 1) * 4 * mm + mm;
    double2* A = Wm + (size_t)inst * 2 * mm;
    double2* T1 = A + mm;
    float2* Fi = F + (size_t)inst * 4 * M * mm;
    build_dblock(A, coef + (size_t)inst * mm, Vi, p, m, c, beta);
    if (p >= 1) {
        const double2* Vc = Vi + (size_t)(p - 1) * mm;
        zgemm_wg(T1, Qtop, Vc, m, 1.0, false);
        zgemm_wg(A, Vc, T1, m, -c2 * c2, true);
    }
    if (p + 1 <= M - 1) {
        const double2* Vc = Vi + (size_t)p * mm;
        zgemm_wg(T1, Qbot, Vc, m, 1.0, false);
        zgemm_wg(A, Vc, T1, m, -c2 * c2, true);
    }
    invert_inplace(A, m);
    store_slot(A, Fi + (size_t)p * mm, m, 1.0);
    if (p >= 1) {
        zgemm_wg(T1, A, Vi + (size_t)(p - 1) * mm, m, c2, false);
        store_slot(T1, Fi + (size_t)(M + p) * mm, m, 1.0);
    }
    if (p + 1 <= M - 1) {
        zgemm_wg(T1, A, Vi + (size_t)p * mm, m, c2, false);
        store_slot(T1, Fi + (size_t)(2 * M + p) * mm, m, 1.0);
    }
}

// ---------------------------------------------------------------------------
// Multi-step chains.  Both recurrences of the reduced solve, y(s) = g(s) + P(s)
// y(s-1) forward and x(t) = y(t) + R(t) x(t-1) backward (chain index s, t from an
// end; x(-1) = x_p), keep their form when only every other index is kept:
//   y(s) = [g(s) + P(s) g(s-1)] + P(s) P(s-1) y(s-2),   y(1) = g(1) + P(1) g(0),
//   x(t) = [y(t) + R(t) y(t-1)] + R(t) R(t-1) x(t-2),   x(-1) = x_p,
// while the dropped indices follow in parallel, y(s) = g(s) + P(s) y(s-1) and
// x(t) = y(t) + R(t) x(t-1).  Applied l times, the sequential chain is 2^l times
// shorter for 4 l row-parallel phases.  This kernel forms one level's step
// factors from the previous level's (FP64 accumulation of the stored singles).
// Rows: index s at reduced row s (top) or M-1-s (bottom) forward, p-1-t or p+1+t
// backward.  With slot(X) = X^T row-major, slot(A B) = slot(B) slot(A).
// blockIdx.x: 32 x 32 output tile, blockIdx.y: (dir, end, i), z: instance.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_cr_level_prod(const float2* __restrict__ F, float2* __restrict__ FL,
                                                       int m, int lev, int depth) {
    const int M = cr_M(m), p = M / 2;
    const int Q = cr_qlev(M, p, lev);
    const int y = blockIdx.y;
    const int dir = y / (2 * Q), e = (y / Q) % 2, i = y % Q;
    const int nsteps = e == 0 ? p : M - 1 - p;
    if (i >= (nsteps >> lev) || (dir == 0 && i < 1)) return;
    const size_t mm = (size_t)m * m;
    const float2* Fi = F + (size_t)blockIdx.z * 4 * M * mm;
    float2* FLi = FL + (size_t)blockIdx.z * cr_fl_off(M, p, depth + 1) * mm;
    // the two factors of the previous level: index 2i+1 (A) and 2i (B)
    auto prev = [&](int k) -> const float2* {
        if (lev == 1) {
            const int row = dir == 0 ? (e == 0 ? k : M - 1 - k) : (e == 0 ? p - 1 - k : p + 1 + k);
            return Fi + (size_t)((dir == 0 ? M : 2 * M) + row) * mm;
        }
        return FLi + cr_fl_block(M, p, lev - 1, dir, e, k) * mm;
    };
    const float2* SA = prev(2 * i + 1);
    const float2* SB = prev(2 * i);
    float2* SC = FLi + cr_fl_block(M, p, lev, dir, e, i) * mm;
    const int nt = (m + 31) / 32;
    const int ti = blockIdx.x / nt, tj = blockIdx.x - ti * nt;
    __shared__ double2 sb[32][33];
    __shared__ double2 sa[32][33];
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    double2 acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < m; k0 += 32) {
        for (int e2 = threadIdx.x; e2 < 32 * 32; e2 += 256) {
            const int r = e2 / 32, c = e2 % 32;
            const int br = ti * 32 + r, bc = k0 + c, ar = k0 + r, ac = tj * 32 + c;
            const float2 vb = (br < m && bc < m) ? SB[(size_t)br * m + bc] : make_float2(0.f, 0.f);
            const float2 va = (ar < m && ac < m) ? SA[(size_t)ar * m + ac] : make_float2(0.f, 0.f);
            sb[r][c] = make_double2(vb.x, vb.y);
            sa[r][c] = make_double2(va.x, va.y);
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 32; ++kk) {
            const double2 av = sa[kk][tx];
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = zadd(acc[r], zmul(sb[ty + 8 * r][kk], av));
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = ti * 32 + ty + 8 * r, col = tj * 32 + tx;
        if (row < m && col < m) SC[(size_t)row * m + col] = make_float2((float)acc[r].x, (float)acc[r].y);
    }
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

static hh_status setup_coarse_reduced(hh_model* md) {
    hh_ctx* ctx = md->ctx;
    const Level& C = md->lev[md->nlev - 1];
    const int m = C.n;
    const int M = cr_M(m), Mo = cr_Mo(m);
    const size_t mm = (size_t)m * m;
    md->m = m;
    md->cr1 = true;
    HH_TRY(md->coarseQT.ensure(ctx, (size_t)md->ninst * 4 * M * mm * sizeof(float2)));
    Buf Vd, W, Wm;
    HH_TRY(Vd.ensure(ctx, (size_t)md->ninst * std::max(Mo, 1) * mm * sizeof(double2)));
    HH_TRY(W.ensure(ctx, (size_t)md->ninst * 8 * mm * sizeof(double2)));
    HH_TRY(Wm.ensure(ctx, (size_t)md->ninst * 2 * mm * sizeof(double2)));
    if (Mo > 0) {
        hipLaunchKernelGGL(k_cr_vinv, dim3(Mo, md->ninst), dim3(1024), 0, ctx->stream, C.coef.as<float2>(),
                           Vd.as<double2>(), md->coarseQT.as<float2>(), m, C.h, md->d.sl_beta);
        HH_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_cr_chain, dim3(md->ninst, 2), dim3(1024), 0, ctx->stream, C.coef.as<float2>(),
                       Vd.as<double2>(), W.as<double2>(), md->coarseQT.as<float2>(), m, C.h, md->d.sl_beta);
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cr_mid, dim3(md->ninst), dim3(1024), 0, ctx->stream, C.coef.as<float2>(), Vd.as<double2>(),
                       W.as<double2>(), Wm.as<double2>(), md->coarseQT.as<float2>(), m, C.h, md->d.sl_beta);
    HH_LAUNCH_CHECK();
    md->cr_depth = md->d.coarse_reduce - 1;
    if (md->cr_depth > 0) {
        const int p = M / 2, D = md->cr_depth;
        HH_TRY(md->coarseFL.ensure(ctx, (size_t)md->ninst * cr_fl_off(M, p, D + 1) * mm * sizeof(float2)));
        const int nt = (m + 31) / 32;
        for (int l = 1; l <= D; ++l) {  // each level from the previous one
            hipLaunchKernelGGL(k_cr_level_prod, dim3(nt * nt, 4 * cr_qlev(M, p, l), md->ninst), dim3(256), 0,
                               ctx->stream, md->coarseQT.as<float2>(), md->coarseFL.as<float2>(), m, l, D);
            HH_LAUNCH_CHECK();
        }
    }
    HH_HIP(hipStreamSynchronize(ctx->stream));  // scratch released on return
    return HH_OK;
}

hh_status setup_coarse_factors(hh_model* md) {
    if (md->d.coarse_iters > 0) {  // iterative coarsest-grid solve: nothing to factorise
        md->m = md->lev[md->nlev - 1].n;
        md->cr1 = false;
        md->cr_depth = 0;
        return HH_OK;
    }
    if (md->d.coarse_reduce) return setup_coarse_reduced(md);
    hh_ctx* ctx = md->ctx;
    const Level& C = md->lev[md->nlev - 1];
    const int m = C.n;
    const int p = m / 2;
    md->m = m;
    md->cr1 = false;
    md->cr_depth = 0;
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
