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
// Building blocks of the coarsest-level factorisations: 32 x 32 tile products
// and a blocked in-place inversion in FP64, one workgroup per output tile (and
// per matrix and medium), so that every sequential step of an elimination is
// spread over the whole chip.
// ---------------------------------------------------------------------------

// acc[r] += X[r0 + ty + 8 r][k] Y[k][c0 + tx] over k < kn (X rows < xr, Y columns < yc; the rest reads
// as zero).  256 threads, tx = tid % 32, ty = tid / 32.
__device__ void tile_mac(double2 (&acc)[4], const double2* __restrict__ X, int ldx, int xr,
                         const double2* __restrict__ Y, int ldy, int yc, int kn, int r0, int c0) {
    __shared__ double2 sx[32][33];
    __shared__ double2 sy[32][33];
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    const double2 z = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < kn; k0 += 32) {
        double2 vx[4], vy[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ty + 8 * q;
            vx[q] = (r0 + r < xr && k0 + tx < kn) ? X[(size_t)(r0 + r) * ldx + k0 + tx] : z;
            vy[q] = (k0 + r < kn && c0 + tx < yc) ? Y[(size_t)(k0 + r) * ldy + c0 + tx] : z;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            sx[ty + 8 * q][tx] = vx[q];
            sy[ty + 8 * q][tx] = vy[q];
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < 32; ++kk) {
            const double2 b = sy[kk][tx];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = zadd(acc[q], zmul(sx[ty + 8 * q][kk], b));
        }
        __syncthreads();
    }
}

// Blocked Gauss-Jordan inversion without pivoting of m x m FP64 matrices, one
// panel K (columns and rows [32 K, 32 K + 32)) per three launches; with the
// panel's pivot block P = A_KK:
//   1: A_KJ <- P^{-1} A_KJ  (J != K)                    one workgroup per column tile J
//   2: A_IJ <- A_IJ - A_IK A_KJ,  C_I = -A_IK P^{-1}    one workgroup per tile (I != K)
//   3: A_IK <- C_I,  A_KK <- P^{-1}                     one workgroup per row tile I
// which is the scalar in-place elimination applied to 32 x 32 blocks (every
// pivot block is a principal block of a Schur complement, nonsingular for the
// same reason as the scalar pivots).  P^{-1} is formed in LDS by the scalar
// elimination, the ragged last panel padded with the identity.  Matrices:
// X + inst * xi + z * xz for z = blockIdx.y (skipped where bit z of skip is set,
// z < 32), inst = blockIdx.z; scratch C (m x 32) and P^{-1} (32 x 32) at
// S + inst * si + z * sz.
struct BlkInv {
    double2* X;
    size_t xz, xi;
    double2* S;
    size_t sz, si;
    unsigned skip;
};

__global__ void __launch_bounds__(256) k_blkinv_row(BlkInv b, int m, int K) {
    const int z = blockIdx.y, inst = blockIdx.z;
    if (z < 32 && ((b.skip >> z) & 1u)) return;
    double2* A = b.X + inst * b.xi + z * b.xz;
    double2* Pv = b.S + inst * b.si + z * b.sz + 32 * (size_t)m;
    const int k0 = 32 * K, bk = min(32, m - k0), J = blockIdx.x, j0 = 32 * J, bj = min(32, m - j0);
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    __shared__ double2 P[2][32][33];  // the elimination alternates between two copies: one barrier per pivot
    __shared__ double2 Y[32][33];
    double2 vp[4], vy[4];  // all loads in flight before the first LDS store
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q;
        vp[q] = (r < bk && tx < bk) ? A[(size_t)(k0 + r) * m + k0 + tx] : make_double2(r == tx ? 1.0 : 0.0, 0.0);
        vy[q] = (J != K && r < bk && tx < bj) ? A[(size_t)(k0 + r) * m + j0 + tx] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        P[0][ty + 8 * q][tx] = vp[q];
        Y[ty + 8 * q][tx] = vy[q];
    }
    __syncthreads();
    for (int q0 = 0; q0 < 32; ++q0) {
        const double2(*Pc)[33] = P[q0 & 1];
        double2(*Pn)[33] = P[(q0 & 1) ^ 1];
        const double2 a = Pc[q0][q0];
        const double rden = 1.0 / (a.x * a.x + a.y * a.y);
        const double2 piv = make_double2(a.x * rden, -a.y * rden);
        const double2 rq = zmul(Pc[q0][tx], piv);  // the pivot row, scaled
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ty + 8 * q;
            const double2 f = Pc[r][q0];
            if (r == q0) Pn[r][tx] = tx == q0 ? piv : rq;
            else if (tx == q0) Pn[r][tx] = zmul(make_double2(-f.x, -f.y), piv);
            else Pn[r][tx] = zsub(Pc[r][tx], zmul(f, rq));
        }
        __syncthreads();
    }
    if (J == K) {
#pragma unroll
        for (int q = 0; q < 4; ++q) Pv[(ty + 8 * q) * 32 + tx] = P[0][ty + 8 * q][tx];
        return;
    }
    double2 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = make_double2(0.0, 0.0);
#pragma unroll 8
    for (int kk = 0; kk < 32; ++kk) {
        const double2 y = Y[kk][tx];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = zadd(acc[q], zmul(P[0][ty + 8 * q][kk], y));
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q;
        if (r < bk && tx < bj) A[(size_t)(k0 + r) * m + j0 + tx] = acc[q];
    }
}

__global__ void __launch_bounds__(256) k_blkinv_update(BlkInv b, int m, int K) {
    const int z = blockIdx.y, inst = blockIdx.z;
    if (z < 32 && ((b.skip >> z) & 1u)) return;
    const int nt = (m + 31) / 32, I = blockIdx.x / nt, J = blockIdx.x - I * nt;
    if (I == K) return;
    double2* A = b.X + inst * b.xi + z * b.xz;
    double2* C = b.S + inst * b.si + z * b.sz;
    const double2* Pv = C + 32 * (size_t)m;
    const int k0 = 32 * K, bk = min(32, m - k0), i0 = 32 * I, j0 = 32 * J;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    double2 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = make_double2(0.0, 0.0);
    if (J != K) {
        tile_mac(acc, A + k0, m, m, A + (size_t)k0 * m, m, m, bk, i0, j0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = i0 + ty + 8 * q, c = j0 + tx;
            if (r < m && c < m) A[(size_t)r * m + c] = zsub(A[(size_t)r * m + c], acc[q]);
        }
    } else {
        tile_mac(acc, A + k0, m, m, Pv, 32, bk, bk, i0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = i0 + ty + 8 * q;
            if (r < m) C[(size_t)r * 32 + tx] = make_double2(-acc[q].x, -acc[q].y);
        }
    }
}

__global__ void __launch_bounds__(256) k_blkinv_col(BlkInv b, int m, int K) {
    const int z = blockIdx.y, inst = blockIdx.z;
    if (z < 32 && ((b.skip >> z) & 1u)) return;
    double2* A = b.X + inst * b.xi + z * b.xz;
    const double2* C = b.S + inst * b.si + z * b.sz;
    const double2* Pv = C + 32 * (size_t)m;
    const int k0 = 32 * K, bk = min(32, m - k0), I = blockIdx.x, i0 = 32 * I;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    if (tx >= bk) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q;
        if (i0 + r >= m) break;
        A[(size_t)(i0 + r) * m + k0 + tx] = I == K ? Pv[r * 32 + tx] : C[(size_t)(i0 + r) * 32 + tx];
    }
}

static hh_status blk_invert(hipStream_t st, const BlkInv& b, int nz, int ninst, int m) {
    const int nt = (m + 31) / 32;
    for (int K = 0; K < nt; ++K) {
        hipLaunchKernelGGL(k_blkinv_row, dim3(nt, nz, ninst), dim3(256), 0, st, b, m, K);
        HH_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_blkinv_update, dim3(nt * nt, nz, ninst), dim3(256), 0, st, b, m, K);
        HH_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_blkinv_col, dim3(nt, nz, ninst), dim3(256), 0, st, b, m, K);
        HH_LAUNCH_CHECK();
    }
    return HH_OK;
}

// slot(z, inst)[c][r] = X(z, inst)[r][c] in complex single precision, through LDS:
// X(z, inst) = X + inst * xi + z * xz, slot(z, inst) = F + inst * fi + z * fz for
// z = blockIdx.y (skipped where bit z of skip is set, z < 32), inst = blockIdx.z.
// grid: (tiles, matrices, instances)
__global__ void __launch_bounds__(256) k_tstore(const double2* __restrict__ X, size_t xz, size_t xi,
                                                float2* __restrict__ F, long long fz, size_t fi, unsigned skip, int m) {
    const int z = blockIdx.y, inst = blockIdx.z;
    if (z < 32 && ((skip >> z) & 1u)) return;
    const double2* A = X + inst * xi + z * xz;
    float2* slot = F + inst * fi + (long long)z * fz;
    const int nt = (m + 31) / 32, ti = blockIdx.x / nt, tj = blockIdx.x - ti * nt;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    __shared__ float2 so[32][33];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 32 * ti + ty + 8 * q, c = 32 * tj + tx;
        const double2 v = (r < m && c < m) ? A[(size_t)r * m + c] : make_double2(0.0, 0.0);
        so[ty + 8 * q][tx] = make_float2((float)v.x, (float)v.y);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = 32 * tj + ty + 8 * q, r = 32 * ti + tx;
        if (r < m && c < m) slot[(size_t)c * m + r] = so[tx][ty + 8 * q];
    }
}

// Entry (r, col) of T_k, the shifted operator's block of grid row k (cf: that
// row's coefficients): 4c - omega^2 kappa^2 (1 - i (gamma + beta)) on the
// diagonal, -c beside it.
__device__ __forceinline__ double2 tblock_entry(const float2* __restrict__ cf, int r, int col, double c, double beta) {
    if (r == col) {
        const float2 cc = cf[r];
        const double w2k2 = cc.x, g = cc.y;
        return make_double2(4.0 * c - w2k2, w2k2 * (g + beta));
    }
    return make_double2(col == r - 1 || col == r + 1 ? -c : 0.0, 0.0);
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
// The inverses Q_k = S_k^{-1} are formed in FP64 (blocked Gauss-Jordan without
// pivoting, above) and stored transposed in complex single precision:
// QT[k][j][i] = Q_k[i][j].  -i A_SL has a positive definite Hermitian part
// (omega^2 kappa^2 (gamma + beta) > 0 on the diagonal), which keeps every Schur
// complement nonsingular without pivoting.
// ---------------------------------------------------------------------------

// Chains of the plain elimination: e = 0 takes rows k = s (s < p), e = 1 rows
// k = m - 1 - s (s < m - 1 - p).  Scratch per medium: three blocks (top, bottom,
// middle) of pf_chain_len(m) FP64 complex: A[2] (m x m, alternating with the
// step's parity), C (m x 32) and P (32 x 32) of the blocked inversion.
static inline __device__ __host__ int pf_nsteps(int m, int e) { return e == 0 ? m / 2 : m - 1 - m / 2; }
static inline __device__ __host__ size_t pf_chain_len(int m) { return 2 * (size_t)m * m + 32 * (size_t)m + 1024; }

// A = T_k - c^2 (the neighbouring rows' inverses): the previous step's (chains)
// or both chains' last (middle row).  grid: (tiles, 2 (chains) or 1 (mid), instances)
__global__ void __launch_bounds__(256) k_pf_schur(const float2* __restrict__ coef, double2* __restrict__ W, int m,
                                                  double H, double beta, int s, int mid) {
    const int inst = blockIdx.z;
    const size_t mm = (size_t)m * m, CH = pf_chain_len(m);
    double2* Wi = W + (size_t)inst * 3 * CH;
    int k;
    double2* A;
    const double2 *P1 = nullptr, *P2 = nullptr;
    if (mid) {
        const int n0 = pf_nsteps(m, 0), n1 = pf_nsteps(m, 1);
        k = m / 2;
        A = Wi + 2 * CH;
        if (n0 >= 1) P1 = Wi + ((n0 - 1) & 1) * mm;
        if (n1 >= 1) P2 = Wi + CH + ((n1 - 1) & 1) * mm;
    } else {
        const int e = blockIdx.y;
        if (s >= pf_nsteps(m, e)) return;
        k = e == 0 ? s : m - 1 - s;
        A = Wi + e * CH + (s & 1) * mm;
        if (s >= 1) P1 = Wi + e * CH + ((s - 1) & 1) * mm;
    }
    const double c = 1.0 / (H * H), c2 = c * c;
    const float2* cf = coef + (size_t)inst * mm + (size_t)k * m;
    const int nt = (m + 31) / 32, ti = blockIdx.x / nt, tj = blockIdx.x - ti * nt;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 32 * ti + ty + 8 * q, col = 32 * tj + tx;
        if (r >= m || col >= m) continue;
        const size_t o = (size_t)r * m + col;
        double2 v = make_double2(0.0, 0.0);
        if (P1) v = zadd(v, P1[o]);
        if (P2) v = zadd(v, P2[o]);
        v = make_double2(-c2 * v.x, -c2 * v.y);
        A[o] = zadd(v, tblock_entry(cf, r, col, c, beta));
    }
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

// V_j <- T_{2j+1} (dense FP64; inverted in place afterwards).  Vd: [inst][Mo][m][m],
// kept for the chain factorisation.  grid: (tiles, Mo, instances)
__global__ void __launch_bounds__(256) k_cr_tfill(const float2* __restrict__ coef, double2* __restrict__ Vd, int m,
                                                  double H, double beta) {
    const int j = blockIdx.y, inst = blockIdx.z, Mo = cr_Mo(m);
    const size_t mm = (size_t)m * m;
    double2* V = Vd + ((size_t)inst * Mo + j) * mm;
    const float2* cf = coef + (size_t)inst * mm + (size_t)(2 * j + 1) * m;
    const double c = 1.0 / (H * H);
    const int nt = (m + 31) / 32, ti = blockIdx.x / nt, tj = blockIdx.x - ti * nt;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 32 * ti + ty + 8 * q, col = 32 * tj + tx;
        if (r < m && col < m) V[(size_t)r * m + col] = tblock_entry(cf, r, col, c, beta);
    }
}


// ---------------------------------------------------------------------------
// Tile-parallel factorisation of the reduced chains.  A chain step (one row j)
// is a handful of m x m FP64 products and one inversion; each of these is
// spread over 32 x 32 output tiles, one workgroup per tile, chain and medium,
// and the step's phases are separate launches:
//   couple: T = Q_prev V_c                       (V_c: the block coupling j to the previous row)
//   schur:  A = D_j - c^4 V_c T                  (middle row: both ends' terms)
//   invert: A <- A^{-1}, blocked Gauss-Jordan over 32-wide panels (above)
//   store:  slots Q_j, P_j = c^2 Q_j V_c, R_j = c^2 Q_j V_n (complex single, transposed)
// Q_j stays in one of two FP64 buffers per chain (alternating with the step's
// parity) for the next step's coupling.
// Scratch per medium: three chain blocks (top, bottom, middle) of
// cf_chain_len(m) FP64 complex: A[2] (m x m), T (m x m), C (m x 32), P (32 x 32).
// ---------------------------------------------------------------------------
static inline __device__ __host__ size_t cf_chain_len(int m) { return 3 * (size_t)m * m + 32 * (size_t)m + 1024; }

// Chain bookkeeping: chain e = 0 (top) takes rows j = s for steps s < p, chain
// e = 1 (bottom) rows j = M - 1 - s for s < M - 1 - p; the middle row p is
// their common next row.  Coupling block to the previous row: V_{j-1} (top),
// V_j (bottom); to the next row: V_j (top), V_{j-1} (bottom).
static inline __device__ __host__ int cf_nsteps(int m, int e) {
    const int M = cr_M(m), p = M / 2;
    return e == 0 ? p : M - 1 - p;
}

// couple: T_e = Q_prev V_c for step s of chain e (mid: the step onto row p).
// grid: (tiles, 2, instances)
__global__ void __launch_bounds__(256) k_cf_couple(const double2* __restrict__ Vd, double2* __restrict__ W, int m,
                                                   int s, int mid) {
    const int e = blockIdx.y, inst = blockIdx.z;
    const int n = cf_nsteps(m, e);
    const int se = mid ? n : s;
    if (se < 1 || (!mid && se >= n)) return;
    const int M = cr_M(m), Mo = cr_Mo(m), j = e == 0 ? se : M - 1 - se;
    const size_t mm = (size_t)m * m, CH = cf_chain_len(m);
    const double2* Vc = Vd + ((size_t)inst * Mo + (e == 0 ? j - 1 : j)) * mm;
    double2* Wc = W + ((size_t)inst * 3 + e) * CH;
    const int nt = (m + 31) / 32, ti = blockIdx.x / nt, tj = blockIdx.x - ti * nt;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    double2 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = make_double2(0.0, 0.0);
    tile_mac(acc, Wc + ((se - 1) & 1) * mm, m, m, Vc, m, m, m, 32 * ti, 32 * tj);
    double2* T = Wc + 2 * mm;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 32 * ti + ty + 8 * q, c = 32 * tj + tx;
        if (r < m && c < m) T[(size_t)r * m + c] = acc[q];
    }
}

// schur: A = D_j - c^4 sum V_c T with D_j = T_{2j} - c^2 ([j >= 1] V_{j-1} + [j < Mo] V_j).
// grid: (tiles, 2 (chains) or 1 (mid), instances)
__global__ void __launch_bounds__(256) k_cf_schur(const float2* __restrict__ coef, const double2* __restrict__ Vd,
                                                  double2* __restrict__ W, int m, double H, double beta, int s,
                                                  int mid) {
    const int inst = blockIdx.z;
    const int M = cr_M(m), Mo = cr_Mo(m), p = M / 2;
    const size_t mm = (size_t)m * m, CH = cf_chain_len(m);
    const double2* Vi = Vd + (size_t)inst * Mo * mm;
    double2* Wi = W + (size_t)inst * 3 * CH;
    const int nt = (m + 31) / 32, ti = blockIdx.x / nt, tj = blockIdx.x - ti * nt;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    double2 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = make_double2(0.0, 0.0);
    int j;
    double2* A;
    if (mid) {
        j = p;
        A = Wi + 2 * CH;
        if (cf_nsteps(m, 0) >= 1) tile_mac(acc, Vi + (size_t)(p - 1) * mm, m, m, Wi + 2 * mm, m, m, m, 32 * ti, 32 * tj);
        if (cf_nsteps(m, 1) >= 1)
            tile_mac(acc, Vi + (size_t)p * mm, m, m, Wi + CH + 2 * mm, m, m, m, 32 * ti, 32 * tj);
    } else {
        const int e = blockIdx.y;
        if (s >= cf_nsteps(m, e)) return;
        j = e == 0 ? s : M - 1 - s;
        double2* Wc = Wi + e * CH;
        A = Wc + (s & 1) * mm;
        if (s >= 1) tile_mac(acc, Vi + (size_t)(e == 0 ? j - 1 : j) * mm, m, m, Wc + 2 * mm, m, m, m, 32 * ti, 32 * tj);
    }
    const double c = 1.0 / (H * H), c2 = c * c, c4 = c2 * c2;
    const float2* cf = coef + (size_t)inst * mm + (size_t)(2 * j) * m;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 32 * ti + ty + 8 * q, col = 32 * tj + tx;
        if (r >= m || col >= m) continue;
        const size_t o = (size_t)r * m + col;
        double2 v = zadd(make_double2(-c4 * acc[q].x, -c4 * acc[q].y), tblock_entry(cf, r, col, c, beta));
        if (j >= 1) {
            const double2 a = Vi[(size_t)(j - 1) * mm + o];
            v.x -= c2 * a.x;
            v.y -= c2 * a.y;
        }
        if (j < Mo) {
            const double2 a = Vi[(size_t)j * mm + o];
            v.x -= c2 * a.x;
            v.y -= c2 * a.y;
        }
        A[o] = v;
    }
}

// store: slots Q_j (role 0), P_j = c^2 Q_j V_c (role 1), R_j = c^2 Q_j V_n (role 2), transposed through LDS.
// grid: (3 * tiles, 2 (chains) or 1 (mid), instances)
__global__ void __launch_bounds__(256) k_cf_store(const double2* __restrict__ Vd, const double2* __restrict__ W,
                                                  float2* __restrict__ F, int m, double H, int s, int mid) {
    const int inst = blockIdx.z;
    const int M = cr_M(m), Mo = cr_Mo(m), p = M / 2;
    const size_t mm = (size_t)m * m, CH = cf_chain_len(m);
    const double2* Vi = Vd + (size_t)inst * Mo * mm;
    const double2* Wi = W + (size_t)inst * 3 * CH;
    const int nt = (m + 31) / 32, role = blockIdx.x / (nt * nt), t = blockIdx.x - role * nt * nt;
    const int ti = t / nt, tj = t - ti * nt;
    int j;
    const double2 *Q, *Vc, *Vn;
    if (mid) {
        j = p;
        Q = Wi + 2 * CH;
        Vc = p >= 1 ? Vi + (size_t)(p - 1) * mm : nullptr;
        Vn = p + 1 <= M - 1 ? Vi + (size_t)p * mm : nullptr;
    } else {
        const int e = blockIdx.y;
        if (s >= cf_nsteps(m, e)) return;
        j = e == 0 ? s : M - 1 - s;
        Q = Wi + e * CH + (s & 1) * mm;
        Vc = s >= 1 ? Vi + (size_t)(e == 0 ? j - 1 : j) * mm : nullptr;
        Vn = Vi + (size_t)(e == 0 ? j : j - 1) * mm;
    }
    const double2* Vr = role == 1 ? Vc : Vn;
    if (role > 0 && !Vr) return;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    double2 acc[4];
    double alpha = 1.0;
    if (role == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 32 * ti + ty + 8 * q, c = 32 * tj + tx;
            acc[q] = (r < m && c < m) ? Q[(size_t)r * m + c] : make_double2(0.0, 0.0);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = make_double2(0.0, 0.0);
        tile_mac(acc, Q, m, m, Vr, m, m, m, 32 * ti, 32 * tj);
        const double c = 1.0 / (H * H);
        alpha = c * c;
    }
    __shared__ float2 so[32][33];
#pragma unroll
    for (int q = 0; q < 4; ++q) so[ty + 8 * q][tx] = make_float2((float)(alpha * acc[q].x), (float)(alpha * acc[q].y));
    __syncthreads();
    float2* slot = F + ((size_t)inst * 4 * M + (size_t)role * M + j) * mm;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = 32 * tj + ty + 8 * q, r = 32 * ti + tx;  // slot[c][r] = M[r][c]
        if (r < m && c < m) slot[(size_t)c * m + r] = so[tx][ty + 8 * q];
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
    Buf Vd, W, Sv;
    const size_t CH = cf_chain_len(m), SL = 32 * (size_t)m + 1024;
    HH_TRY(Vd.ensure(ctx, (size_t)md->ninst * std::max(Mo, 1) * mm * sizeof(double2)));
    HH_TRY(W.ensure(ctx, (size_t)md->ninst * 3 * CH * sizeof(double2)));
    hipStream_t st = ctx->stream;
    if (Mo > 0) {  // V_j = T_{2j+1}^{-1}, all j at once
        const int nt = (m + 31) / 32, ni = md->ninst;
        HH_TRY(Sv.ensure(ctx, (size_t)ni * Mo * SL * sizeof(double2)));
        hipLaunchKernelGGL(k_cr_tfill, dim3(nt * nt, Mo, ni), dim3(256), 0, st, C.coef.as<float2>(),
                           Vd.as<double2>(), m, C.h, md->d.sl_beta);
        HH_LAUNCH_CHECK();
        const BlkInv bv{Vd.as<double2>(), mm, Mo * mm, Sv.as<double2>(), SL, Mo * SL, 0u};
        HH_TRY(blk_invert(st, bv, Mo, ni, m));
        hipLaunchKernelGGL(k_tstore, dim3(nt * nt, Mo, ni), dim3(256), 0, st, Vd.as<double2>(), mm, Mo * mm,
                           md->coarseQT.as<float2>() + 3 * M * mm, (long long)mm, 4 * M * mm, 0u, m);
        HH_LAUNCH_CHECK();
    }
    {
        const int nt = (m + 31) / 32, ntop = cf_nsteps(m, 0), nbot = cf_nsteps(m, 1), ni = md->ninst;
        const double beta = md->d.sl_beta;
        double2* Wd = W.as<double2>();
        const double2* Vp = Vd.as<double2>();
        float2* F = md->coarseQT.as<float2>();
        for (int s = 0; s < std::max(ntop, nbot); ++s) {  // both chains, one row each per step
            if (s >= 1) {
                hipLaunchKernelGGL(k_cf_couple, dim3(nt * nt, 2, ni), dim3(256), 0, st, Vp, Wd, m, s, 0);
                HH_LAUNCH_CHECK();
            }
            hipLaunchKernelGGL(k_cf_schur, dim3(nt * nt, 2, ni), dim3(256), 0, st, C.coef.as<float2>(), Vp, Wd, m,
                               C.h, beta, s, 0);
            HH_LAUNCH_CHECK();
            const BlkInv b{Wd + (s & 1) * mm, CH, 3 * CH, Wd + 3 * mm, CH, 3 * CH,
                           (s >= ntop ? 1u : 0u) | (s >= nbot ? 2u : 0u)};
            HH_TRY(blk_invert(st, b, 2, ni, m));
            hipLaunchKernelGGL(k_cf_store, dim3(3 * nt * nt, 2, ni), dim3(256), 0, st, Vp, Wd, F, m, C.h, s, 0);
            HH_LAUNCH_CHECK();
        }
        // the middle row, coupled to both chains' last rows
        if (ntop >= 1 || nbot >= 1) {
            hipLaunchKernelGGL(k_cf_couple, dim3(nt * nt, 2, ni), dim3(256), 0, st, Vp, Wd, m, 0, 1);
            HH_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_cf_schur, dim3(nt * nt, 1, ni), dim3(256), 0, st, C.coef.as<float2>(), Vp, Wd, m, C.h,
                           beta, 0, 1);
        HH_LAUNCH_CHECK();
        const BlkInv bm{Wd + 2 * CH, 0, 3 * CH, Wd + 2 * CH + 3 * mm, 0, 3 * CH, 0u};
        HH_TRY(blk_invert(st, bm, 1, ni, m));
        hipLaunchKernelGGL(k_cf_store, dim3(3 * nt * nt, 1, ni), dim3(256), 0, st, Vp, Wd, F, m, C.h, 0, 1);
        HH_LAUNCH_CHECK();
    }
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
    const size_t mm = (size_t)m * m, CP = pf_chain_len(m);
    Buf S;
    HH_TRY(S.ensure(ctx, (size_t)md->ninst * 3 * CP * sizeof(double2)));
    hipStream_t st = ctx->stream;
    const int nt = (m + 31) / 32, ntop = pf_nsteps(m, 0), nbot = pf_nsteps(m, 1), ni = md->ninst;
    const double beta = md->d.sl_beta;
    double2* Wd = S.as<double2>();
    float2* QT = md->coarseQT.as<float2>();
    for (int s = 0; s < std::max(ntop, nbot); ++s) {  // both chains, one row each per step
        const unsigned skip = (s >= ntop ? 1u : 0u) | (s >= nbot ? 2u : 0u);
        hipLaunchKernelGGL(k_pf_schur, dim3(nt * nt, 2, ni), dim3(256), 0, st, C.coef.as<float2>(), Wd, m, C.h, beta,
                           s, 0);
        HH_LAUNCH_CHECK();
        const BlkInv b{Wd + (s & 1) * mm, CP, 3 * CP, Wd + 2 * mm, CP, 3 * CP, skip};
        HH_TRY(blk_invert(st, b, 2, ni, m));
        // slots s (top) and m - 1 - s (bottom)
        hipLaunchKernelGGL(k_tstore, dim3(nt * nt, 2, ni), dim3(256), 0, st, Wd + (s & 1) * mm, CP, 3 * CP,
                           QT + (size_t)s * mm, (long long)(m - 1 - 2 * s) * (long long)mm, (size_t)m * mm, skip, m);
        HH_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_pf_schur, dim3(nt * nt, 1, ni), dim3(256), 0, st, C.coef.as<float2>(), Wd, m, C.h, beta, 0, 1);
    HH_LAUNCH_CHECK();
    const BlkInv bm{Wd + 2 * CP, 0, 3 * CP, Wd + 2 * CP + 2 * mm, 0, 3 * CP, 0u};
    HH_TRY(blk_invert(st, bm, 1, ni, m));
    hipLaunchKernelGGL(k_tstore, dim3(nt * nt, 1, ni), dim3(256), 0, st, Wd + 2 * CP, (size_t)0, 3 * CP,
                       QT + (size_t)p * mm, 0LL, (size_t)m * mm, 0u, m);
    HH_LAUNCH_CHECK();
    // S is released when this function returns: order the free after the kernels.
    HH_HIP(hipStreamSynchronize(ctx->stream));
    return HH_OK;
}

}  // namespace hh
