// Shifted-Laplacian multigrid on gfx950: operator application and one V-cycle
// (Sec. 3.2, Alg. 1 applied recursively; transfers of eq. 8).
//
// Data: complex single precision, [rhs][n][n]; coefficients {omega^2 kappa^2,
// gamma} per point and level, shared by all right-hand sides of one slowness
// model.  Each V-cycle level is two fused kernels:
//   down: x1 = relax(x0) (x0 = 0: x1 = w b / diag); r = b - A_SL x1; b_c = R r
//   up:   x = x1 + P e_c; z = x + w (b - A_SL x) / diag
// so the level reads b once in each direction and writes only the coarse
// right-hand side and the level's result.  The tiles are staged in LDS with the
// halo the stencil chain needs (2 fine cells for down, 1 for up).
#include <map>
#include <mutex>

#include "hh_internal.h"

namespace hh {

// ---------------------------------------------------------------------------
// y = A x   (A = -Delta_h - omega^2 kappa^2 (1 - i (gamma + shift)))
// 64 x 16 tile per 256-thread block; each thread walks 4 rows of one column.
// ---------------------------------------------------------------------------
constexpr int OP_TX = 64, OP_TY = 16, OP_ROWS = 4;

__global__ void __launch_bounds__(256) k_apply_op(const float2* __restrict__ x, float2* __restrict__ y,
                                                  const float2* __restrict__ coef, const int* __restrict__ inst,
                                                  int n, float inv_h2, float shift, const int* __restrict__ active) {
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const int j = blockIdx.x * OP_TX + threadIdx.x;
    const int i0 = blockIdx.y * OP_TY + threadIdx.y * OP_ROWS;
    if (j >= n) return;
    const size_t nn = (size_t)n * n;
    const float2* xr = x + r * nn;
    float2* yr = y + r * nn;
    const float2* cf = coef + (size_t)(inst ? inst[r] : 0) * nn;
    const float2 zero = make_float2(0.f, 0.f);
    float2 up = (i0 > 0 && i0 - 1 < n) ? xr[(size_t)(i0 - 1) * n + j] : zero;
    float2 cur = (i0 < n) ? xr[(size_t)i0 * n + j] : zero;
#pragma unroll
    for (int t = 0; t < OP_ROWS; ++t) {
        const int i = i0 + t;
        if (i >= n) break;
        float2 dn = (i + 1 < n) ? xr[(size_t)(i + 1) * n + j] : zero;
        float2 lf = (j > 0) ? xr[(size_t)i * n + j - 1] : zero;
        float2 rt = (j + 1 < n) ? xr[(size_t)i * n + j + 1] : zero;
        float2 m = mass_of(cf[(size_t)i * n + j], shift);
        float2 lap = make_float2((4.f * cur.x - up.x - dn.x - lf.x - rt.x) * inv_h2,
                                 (4.f * cur.y - up.y - dn.y - lf.y - rt.y) * inv_h2);
        yr[(size_t)i * n + j] = csub(lap, cmul(m, cur));
        up = cur;
        cur = dn;
    }
}

// ---------------------------------------------------------------------------
// Initial guess of the CNN+MG V-cycle straight from the network's
// half-resolution output o ([n/2][n/2] (re, im)): x0 = s P(o) at fine (i, j),
// with P the multigrid prolongation of eq. 8 (coarse I on fine 2I; odd fine
// indices average their two coarse neighbours) and s the network's output
// scale.  Reading o instead of a stored fine x0 saves the full-resolution
// vector's write and reads.
// ---------------------------------------------------------------------------
// The blocks stage the coarse tile they need, s_o[I - cy0][J - cx0] (zero
// outside the grid), and interpolate from LDS; i, j >= 0 are fine indices
// inside the grid.
// (256 threads; every load of a thread is issued before its first store, so that
// they are in flight together)
template <int CPW, int ROWS>
__device__ __forceinline__ void stage_half(float2* s_o, const float2* __restrict__ ob, int m, int cy0, int cx0) {
    constexpr int NE = ROWS * CPW, NJ = (NE + 255) / 256;
    float2 v[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int e = threadIdx.x + 256 * j;
        const int py = e / CPW, px = e - py * CPW;
        const int I = cy0 + py, J = cx0 + px;
        v[j] = (e < NE && I >= 0 && I < m && J >= 0 && J < m) ? ob[(size_t)I * m + J] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int e = threadIdx.x + 256 * j;
        if (e < NE) s_o[e] = v[j];
    }
}

// Bilinear value at fine parity (ey, ex) from coarse (ly, lx) of an LDS tile
// with row pitch w, without branches: the second row / column is ly + ey /
// lx + ex, so with a zero parity the pair averages a value with itself, which
// is exact -- the result equals the case-by-case formula (P of eq. 8) bit for bit.
__device__ __forceinline__ float2 interp_half(const float2* t, int w, int ly, int lx, int ey, int ex) {
    const float2 a = t[ly * w + lx], b = t[ly * w + lx + ex];
    const float2 c = t[(ly + ey) * w + lx], d = t[(ly + ey) * w + lx + ex];
    const float2 h0 = cscale(cadd(a, b), 0.5f), h1 = cscale(cadd(c, d), 0.5f);
    return cscale(cadd(h0, h1), 0.5f);
}

template <int CPW>
__device__ __forceinline__ float2 x0_from_half(const float2* s_o, int cy0, int cx0, int i, int j, float s) {
    return cscale(interp_half(s_o, CPW, (i >> 1) - cy0, (j >> 1) - cx0, i & 1, j & 1), s);
}

// The guess x0 = s P(o) on a fine LDS patch dst[PH][PW] whose first row and
// column are the fine cells (fy0, fx0), from the coarse tile s_o (pitch CPW,
// origin (fy0 >> 1, fx0 >> 1)), zero outside the n x n grid.  Each thread forms
// the four fine cells of one coarse cell, (2I + a, 2J + c), from its four
// corners, with interp_half's operations for each parity: (0, 0) gives the
// corner itself, (0, 1) and (1, 0) the midpoints, (1, 1) the mean of the two
// row midpoints -- bit for bit what interp_half returns, with one quarter of
// its index work.  256 threads.
template <int CPW, int PH, int PW>
__device__ __forceinline__ void x0_patch_from_half(float2 (*dst)[PW], const float2* s_o, int fy0, int fx0, int n,
                                                   float s) {
    const int by0 = fy0 >> 1, bx0 = fx0 >> 1;  // floor: fy0, fx0 may be negative
    constexpr int BH = PH / 2 + 1, BW = PW / 2 + 1;  // coarse cells touching the patch (at most)
    for (int e = threadIdx.x; e < BH * BW; e += 256) {
        const int by = e / BW, bx = e - by * BW;
        const float2* t = s_o + by * CPW + bx;
        const float2 a = t[0], b = t[1], c = t[CPW], d = t[CPW + 1];
        const float2 ab = cscale(cadd(a, b), 0.5f), cd = cscale(cadd(c, d), 0.5f);
        const float2 v[2][2] = {{a, ab}, {cscale(cadd(a, c), 0.5f), cscale(cadd(ab, cd), 0.5f)}};
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int gi = 2 * (by0 + by) + dy, gj = 2 * (bx0 + bx) + dx;
                const int py = gi - fy0, px = gj - fx0;
                if (py < 0 || py >= PH || px < 0 || px >= PW) continue;
                dst[py][px] = (gi >= 0 && gi < n && gj >= 0 && gj < n) ? cscale(v[dy][dx], s) : make_float2(0.f, 0.f);
            }
    }
}

// ---------------------------------------------------------------------------
// V-cycle down kernel on one level.
// Block = 256 threads computes a TCY x TCX tile of the coarse right-hand side.
// X0M: the level's initial guess -- 0 none; 1 a fine x0 (the relaxed x1 is then
// also written out for the up kernel); 2 the network's half-resolution output
// (x0h, scale x0s per RHS), from which the up kernel recomputes x1 itself.
// ---------------------------------------------------------------------------
constexpr int DN_TCX = 32, DN_TCY = 8;
constexpr int DN_TCY2 = 4;  // with the network's guess: four arrays in LDS, half-height tiles

template <int X0M, int TCY>
__global__ void __launch_bounds__(256) k_vc_down(const float2* __restrict__ b, size_t bstride,
                                                 const double* __restrict__ sig, int sig_stride,
                                                 const float2* __restrict__ x0, size_t x0stride,
                                                 float2* __restrict__ x1out, float2* __restrict__ bc,
                                                 const float2* __restrict__ coef, const int* __restrict__ inst,
                                                 int n, float inv_h2, float beta, float wj,
                                                 const int* __restrict__ active, const float2* __restrict__ x0h,
                                                 const float* __restrict__ x0s) {
    constexpr bool HAS_X0 = X0M != 0;
    constexpr int HALO = HAS_X0 ? 3 : 2;
    constexpr int PH = 2 * TCY + 2 * HALO - 1;  // fine rows 2I0-HALO .. 2I0+2TCY+HALO-2 (TCY coarse rows per tile)
    constexpr int PW = 2 * DN_TCX + 2 * HALO - 1;
    __shared__ float2 s_b[PH][PW];   // b, later r
    __shared__ float2 s_x[PH][PW];   // x1 (relaxed)
    __shared__ float2 s_m[PH][PW];   // shifted mass
    __shared__ float2 s_x0[HAS_X0 ? PH : 1][HAS_X0 ? PW : 1];
    // mode 2: the coarse tile of the network output under the fine patch
    constexpr int OPH = X0M == 2 ? PH / 2 + 2 : 1, OPW = X0M == 2 ? PW / 2 + 2 : 1;
    __shared__ float2 s_o[OPH * OPW];

    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const int tid = threadIdx.x;
    const int nc = n >> 1;
    const int I0 = blockIdx.y * TCY, J0 = blockIdx.x * DN_TCX;
    const int fy0 = 2 * I0 - HALO, fx0 = 2 * J0 - HALO;
    const size_t nn = (size_t)n * n;
    const float2* br = b + r * bstride;
    const float2* cf = coef + (size_t)(inst ? inst[r] : 0) * nn;
    const float s = sig ? (float)sig[(size_t)r * sig_stride] : 1.0f;
    const float dgv = 4.f * inv_h2;
    const float2 zero = make_float2(0.f, 0.f);
    const int ocy0 = fy0 >> 1, ocx0 = fx0 >> 1;  // floor halves (fy0, fx0 may be negative)
    // this thread's b and coefficients of the patch, loaded first so that they
    // are in flight together with the network-output tile below
    constexpr int NPT = (PH * PW + 255) / 256;
    float2 rb[NPT], rc[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int e = tid + j * 256;
        const int py = e / PW, px = e - py * PW;
        const int gi = fy0 + py, gj = fx0 + px;
        const bool in = e < PH * PW && gi >= 0 && gi < n && gj >= 0 && gj < n;
        const size_t o = (size_t)gi * n + gj;
        rb[j] = in ? br[o] : zero;
        rc[j] = in ? cf[o] : zero;
    }
    if (X0M == 2) {
        stage_half<OPW, OPH>(s_o, x0h + (size_t)r * (n >> 1) * (n >> 1), n >> 1, ocy0, ocx0);
        __syncthreads();
    }

    // stage b (scaled), the shifted mass and x0
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int e = tid + j * 256;
        if (e >= PH * PW) break;
        int py = e / PW, px = e - py * PW;
        int gi = fy0 + py, gj = fx0 + px;
        bool in = gi >= 0 && gi < n && gj >= 0 && gj < n;
        size_t o = (size_t)gi * n + gj;
        float2 bv = in ? cscale(rb[j], s) : zero;
        float2 mv = in ? mass_of(rc[j], beta) : zero;
        s_b[py][px] = bv;
        s_m[py][px] = mv;
        if (X0M == 1) {
            s_x0[py][px] = in ? x0[r * x0stride + o] : zero;
        } else if (X0M == 2) {
            // staged below, four fine cells per thread
        } else {
            // x1 = w b / diag with diag = 4/h^2 - mass
            float2 d = make_float2(dgv - mv.x, -mv.y);
            s_x[py][px] = in ? cscale(cdiv_rcp(bv, d), wj) : zero;
        }
    }
    if constexpr (X0M == 2) x0_patch_from_half<OPW, PH, PW>(s_x0, s_o, fy0, fx0, n, x0s[r]);
    __syncthreads();
    if (HAS_X0) {
        // x1 = x0 + w (b - A_SL x0)/diag on rows/cols 1..P-2 (the staging's
        // thread-to-cell map, so its index work is reused)
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int e = tid + j * 256;
            if (e >= PH * PW) break;
            int py = e / PW, px = e - py * PW;
            int gi = fy0 + py, gj = fx0 + px;
            bool in = gi >= 0 && gi < n && gj >= 0 && gj < n;
            float2 v = zero;
            if (in && py > 0 && py < PH - 1 && px > 0 && px < PW - 1) {
                float2 c = s_x0[py][px];
                float2 nb = cadd(cadd(s_x0[py - 1][px], s_x0[py + 1][px]), cadd(s_x0[py][px - 1], s_x0[py][px + 1]));
                float2 mv = s_m[py][px];
                float2 Ax = csub(make_float2((4.f * c.x - nb.x) * inv_h2, (4.f * c.y - nb.y) * inv_h2), cmul(mv, c));
                float2 d = make_float2(dgv - mv.x, -mv.y);
                v = cadd(c, cscale(cdiv_rcp(csub(s_b[py][px], Ax), d), wj));
            }
            s_x[py][px] = v;
        }
        __syncthreads();
        // write x1 on the fine cells this tile owns: rows 2I0 .. 2I0+2TCY-1
        for (int e = tid; X0M == 1 && e < 4 * TCY * DN_TCX; e += 256) {
            int ly = e / (2 * DN_TCX), lx = e - ly * (2 * DN_TCX);
            int gi = 2 * I0 + ly, gj = 2 * J0 + lx;
            if (gi < n && gj < n) x1out[r * nn + (size_t)gi * n + gj] = s_x[ly + HALO][lx + HALO];
        }
    }
    // residual r = b - A_SL x1 on rows/cols R0 .. P-1-R0 (the FW support)
    constexpr int R0 = HALO - 1;
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int e = tid + j * 256;
        if (e >= PH * PW) break;
        int py = e / PW, px = e - py * PW;
        if (py < R0 || py > PH - 1 - R0 || px < R0 || px > PW - 1 - R0) continue;
        int gi = fy0 + py, gj = fx0 + px;
        bool in = gi >= 0 && gi < n && gj >= 0 && gj < n;
        float2 rv = zero;
        if (in) {
            float2 c = s_x[py][px];
            float2 nb = cadd(cadd(s_x[py - 1][px], s_x[py + 1][px]), cadd(s_x[py][px - 1], s_x[py][px + 1]));
            float2 Ax = csub(make_float2((4.f * c.x - nb.x) * inv_h2, (4.f * c.y - nb.y) * inv_h2), cmul(s_m[py][px], c));
            rv = csub(s_b[py][px], Ax);
        }
        s_b[py][px] = rv;  // only this thread reads s_b at (py, px) in this phase
    }
    __syncthreads();
    // full-weighting restriction: coarse (I, J) <- fine 2I + a - 1, 2J + c - 1
    {
        int cy = tid / DN_TCX, cx = tid - cy * DN_TCX;
        int I = I0 + cy, J = J0 + cx;
        if (cy < TCY && I < nc && J < nc) {
            int py = 2 * cy + HALO - 1, px = 2 * cx + HALO - 1;
            const float w1[3] = {0.25f, 0.5f, 0.25f};
            float2 acc = zero;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc = cadd(acc, cscale(s_b[py + a][px + c], w1[a] * w1[c]));
            bc[(size_t)r * nc * nc + (size_t)I * nc + J] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// V-cycle up kernel on one level: prolong + correct + post-relaxation.
// Block = 256 threads computes a TY x TX fine tile.  X1M: where the relaxed x1
// comes from -- 0 recomputed as w b / diag (zero initial guess); 1 stored by
// the down kernel; 2 recomputed from the network's half-resolution output,
// x1 = x0 + w (b - A_SL x0) / diag with x0 = s P(o), the down kernel's formula.
// ---------------------------------------------------------------------------
constexpr int UP_TX = 64, UP_TY = 16;
constexpr int UP_TY2 = 8;  // with the network's guess: the x0 patch in LDS too, half-height tiles

template <int X1M, int TY>
__global__ void __launch_bounds__(256) k_vc_up(const float2* __restrict__ b, size_t bstride,
                                               const double* __restrict__ sig, int sig_stride,
                                               const float2* __restrict__ x1, const float2* __restrict__ ec,
                                               float2* __restrict__ z, size_t zstride,
                                               const float2* __restrict__ coef, const int* __restrict__ inst,
                                               int n, float inv_h2, float beta, float wj,
                                               const int* __restrict__ active, const float2* __restrict__ x0h,
                                               const float* __restrict__ x0s) {
    constexpr int PH = TY + 2, PW = UP_TX + 2;  // TY fine rows per tile
    constexpr int CH = TY / 2 + 2, CW = UP_TX / 2 + 2;
    constexpr int XH = X1M == 2 ? PH + 2 : 1, XW = X1M == 2 ? PW + 2 : 1;
    __shared__ float2 s_b[PH][PW];
    __shared__ float2 s_x[PH][PW];
    __shared__ float2 s_m[PH][PW];
    __shared__ float2 s_e[CH][CW];
    __shared__ float2 s_x0[XH][XW];  // x0 on fine rows y0-2 .. y0+TY+1 (mode 2)
    constexpr int OPH = X1M == 2 ? XH / 2 + 2 : 1, OPW = X1M == 2 ? XW / 2 + 2 : 1;
    __shared__ float2 s_o[OPH * OPW];  // the network output's coarse tile under s_x0

    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const int tid = threadIdx.x;
    const int nc = n >> 1;
    const int y0 = blockIdx.y * TY, x0 = blockIdx.x * UP_TX;
    const int cy0 = y0 / 2 - 1, cx0 = x0 / 2 - 1;
    const size_t nn = (size_t)n * n;
    const float2* br = b + r * bstride;
    const float2* cf = coef + (size_t)(inst ? inst[r] : 0) * nn;
    const float2* er = ec + (size_t)r * nc * nc;
    const float s = sig ? (float)sig[(size_t)r * sig_stride] : 1.0f;
    const float dg = 4.f * inv_h2;
    const float2 zero = make_float2(0.f, 0.f);

    // this thread's b and coefficients of the patch, loaded first so that they
    // are in flight together with the coarse tiles below
    constexpr int NPT = (PH * PW + 255) / 256;
    float2 rb[NPT], rc[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int e = tid + j * 256;
        const int py = e / PW, px = e - py * PW;
        const int gi = y0 - 1 + py, gj = x0 - 1 + px;
        const bool in = e < PH * PW && gi >= 0 && gi < n && gj >= 0 && gj < n;
        const size_t o = (size_t)gi * n + gj;
        rb[j] = in ? br[o] : zero;
        rc[j] = in ? cf[o] : zero;
    }
    stage_half<CW, CH>(&s_e[0][0], er, nc, cy0, cx0);  // the coarse correction's tile
    const int ocy0 = (y0 - 2) >> 1, ocx0 = (x0 - 2) >> 1;
    if constexpr (X1M == 2) {
        stage_half<OPW, OPH>(s_o, x0h + (size_t)r * nc * nc, nc, ocy0, ocx0);
        __syncthreads();
        x0_patch_from_half<OPW, XH, XW>(s_x0, s_o, y0 - 2, x0 - 2, n, x0s[r]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int e = tid + j * 256;
        if (e >= PH * PW) break;
        int py = e / PW, px = e - py * PW;
        int gi = y0 - 1 + py, gj = x0 - 1 + px;
        bool in = gi >= 0 && gi < n && gj >= 0 && gj < n;
        float2 bv = zero, mv = zero, xv = zero;
        if (in) {
            size_t o = (size_t)gi * n + gj;
            bv = cscale(rb[j], s);
            mv = mass_of(rc[j], beta);
            if (X1M == 1) {
                xv = x1[r * nn + o];
            } else if (X1M == 2) {
                const int qy = py + 1, qx = px + 1;  // s_x0 starts one row / column further out
                float2 c = s_x0[qy][qx];
                float2 nb = cadd(cadd(s_x0[qy - 1][qx], s_x0[qy + 1][qx]), cadd(s_x0[qy][qx - 1], s_x0[qy][qx + 1]));
                float2 Ax = csub(make_float2((4.f * c.x - nb.x) * inv_h2, (4.f * c.y - nb.y) * inv_h2), cmul(mv, c));
                float2 d = make_float2(dg - mv.x, -mv.y);
                xv = cadd(c, cscale(cdiv_rcp(csub(bv, Ax), d), wj));
            } else {
                xv = cscale(cdiv_rcp(bv, make_float2(dg - mv.x, -mv.y)), wj);
            }
            // bilinear prolongation: even index -> coarse i/2; odd -> mean of (i-1)/2, (i+1)/2
            const int ly = (gi >> 1) - cy0, lx = (gj >> 1) - cx0;
            xv = cadd(xv, interp_half(&s_e[0][0], CW, ly, lx, gi & 1, gj & 1));
        }
        s_b[py][px] = bv;
        s_m[py][px] = mv;
        s_x[py][px] = xv;
    }
    __syncthreads();
    for (int e = tid; e < TY * UP_TX; e += 256) {
        int ly = e / UP_TX, lx = e - ly * UP_TX;
        int gi = y0 + ly, gj = x0 + lx;
        if (gi >= n || gj >= n) continue;
        int py = ly + 1, px = lx + 1;
        float2 c = s_x[py][px];
        float2 nb = cadd(cadd(s_x[py - 1][px], s_x[py + 1][px]), cadd(s_x[py][px - 1], s_x[py][px + 1]));
        float2 mv = s_m[py][px];
        float2 Ax = csub(make_float2((4.f * c.x - nb.x) * inv_h2, (4.f * c.y - nb.y) * inv_h2), cmul(mv, c));
        float2 d = make_float2(dg - mv.x, -mv.y);
        z[r * zstride + (size_t)gi * n + gj] = cadd(c, cscale(cdiv_rcp(csub(s_b[py][px], Ax), d), wj));
    }
}

// ---------------------------------------------------------------------------
// Coarsest-level exact solve with the stored Schur inverses (see setup.hip),
// eliminating from both ends towards the middle row p:
//   forward (top)     w_k = b_k + c y_{k-1},  y_k = Q_k w_k       k = 0 .. p-1
//   forward (bottom)  w_k = b_k + c y_{k+1},  y_k = Q_k w_k       k = m-1 .. p+1
//   middle            x_p = Q_p (b_p + c y_{p-1} + c y_{p+1})
//   backward (top)    x_k = y_k + c Q_k x_{k+1}                   k = p-1 .. 0
//   backward (bottom) x_k = y_k + c Q_k x_{k-1}                   k = p+1 .. m-1
// Two launches (forward, then middle + backward); each launch has two
// workgroups per right-hand side (blockIdx.y = 0 top, 1 bottom), so the kernel
// boundary is the only synchronisation.  A step is a dense m x m complex
// matrix-vector product; QT is stored transposed so that the threads of a
// wave read consecutive rows of one column.  For m < 256 the column range is
// split over JP thread groups whose partial sums meet in LDS.
// ---------------------------------------------------------------------------
constexpr int CS_MAXM = 1024;
constexpr int CS_NT = 1024;  // threads per workgroup: every row, columns split JP = 1024/m ways
constexpr int CS_RMAX = 8;   // right-hand sides per workgroup: 1, 2, 4 or 8 (each Q_k read serves all of them)

template <int R>
struct CoarseMV {
    static constexpr int CH = R >= 4 ? 8 : 16;  // loads per chunk; the next chunk loads while one is used
    int m, JP, jlen, row, jp;
    __device__ CoarseMV(int m_) : m(m_) {
        JP = CS_NT / m;  // >= 1 since m <= 1024
        jlen = (m + JP - 1) / JP;
        row = threadIdx.x % m;
        jp = threadIdx.x / m;
    }
    // out[q] = sum_j Qk[j][row] v[q][j] for the R vectors s_v[q * m + j]; the JP
    // partial sums meet in s_part[q * CS_NT + t].  Valid in the owner threads (jp == 0).
    __device__ void apply(const float2* __restrict__ Qk, const float2* s_v, float2* s_part, float2 (&out)[R]) const {
        float2 qa[CH], qb[CH];
        apply(Qk, qa, qb, s_v, s_part, out);
    }
    // the same with the caller's chunk buffers (contents undefined on return)
    __device__ void apply(const float2* __restrict__ Qk, float2 (&qa)[CH], float2 (&qb)[CH], const float2* s_v,
                          float2* s_part, float2 (&out)[R]) const {
        float2 acc[R];
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = make_float2(0.f, 0.f);
        if (jp < JP) {
            const int j0 = jp * jlen, j1 = min(m, j0 + jlen);
            const float2* qp = Qk + row;
            int j = j0;
            if (j + CH <= j1) {
#pragma unroll
                for (int u = 0; u < CH; ++u) qa[u] = qp[(size_t)(j + u) * m];
                for (;;) {
                    const int jb = j + CH;
                    const bool hb = jb + CH <= j1;
                    if (hb) {
#pragma unroll
                        for (int u = 0; u < CH; ++u) qb[u] = qp[(size_t)(jb + u) * m];
                    }
#pragma unroll
                    for (int u = 0; u < CH; ++u)
#pragma unroll
                        for (int q = 0; q < R; ++q) acc[q] = cadd(acc[q], cmul(qa[u], s_v[q * m + j + u]));
                    j = jb;
                    if (!hb) break;
                    const int ja = j + CH;
                    const bool ha = ja + CH <= j1;
                    if (ha) {
#pragma unroll
                        for (int u = 0; u < CH; ++u) qa[u] = qp[(size_t)(ja + u) * m];
                    }
#pragma unroll
                    for (int u = 0; u < CH; ++u)
#pragma unroll
                        for (int q = 0; q < R; ++q) acc[q] = cadd(acc[q], cmul(qb[u], s_v[q * m + j + u]));
                    j = ja;
                    if (!ha) break;
                }
            }
            for (; j < j1; ++j) {
                const float2 qv = qp[(size_t)j * m];
#pragma unroll
                for (int q = 0; q < R; ++q) acc[q] = cadd(acc[q], cmul(qv, s_v[q * m + j]));
            }
        }
        if (JP > 1) {
            if (jp < JP)
#pragma unroll
                for (int q = 0; q < R; ++q) s_part[q * CS_NT + threadIdx.x] = acc[q];
            __syncthreads();
            if (jp == 0)
                for (int t = 1; t < JP; ++t)
#pragma unroll
                    for (int q = 0; q < R; ++q) acc[q] = cadd(acc[q], s_part[q * CS_NT + t * m + row]);
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < R; ++q) out[q] = acc[q];
    }
    __device__ bool owner() const { return jp == 0; }

    // Cross-step prefetch for the chains: the next step's matrix does not depend
    // on this step's result, so its first two chunks load while this step ends.
    // Smaller chunks than apply() (the two buffers stay live across the step);
    // needs every thread's column range to be whole chunk pairs (m = 128 .. 1024).
    static constexpr int PCH = R == 1 ? 8 : 4;
    __device__ bool pf_ok() const { return CS_NT % m == 0 && jlen % (2 * PCH) == 0; }
    // buffer resource over one m x m block (the block pointer is uniform in the
    // workgroup); loads then take the column offset from a scalar register
    __device__ __amdgpu_buffer_rsrc_t block_rsrc(const float2* Qk) const {
        const unsigned long long a = (unsigned long long)Qk;
        const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
        const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
        void* base = (void*)(((unsigned long long)hi << 32) | lo);
        return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, m * m * (int)sizeof(float2), 0x00020000);
    }
    __device__ float2 bload(__amdgpu_buffer_rsrc_t rs, int vo, int col) const {
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, col * m * 8, 0));
    }
    __device__ void preload(const float2* __restrict__ Qk, float2 (&qa)[PCH], float2 (&qb)[PCH]) const {
        const __amdgpu_buffer_rsrc_t rs = block_rsrc(Qk);
        const int vo = (row + jp * jlen * m) * 8;
#pragma unroll
        for (int u = 0; u < PCH; ++u) qa[u] = bload(rs, vo, u);
#pragma unroll
        for (int u = 0; u < PCH; ++u) qb[u] = bload(rs, vo, PCH + u);
    }
    // apply() with qa / qb holding Qk's first two chunks of this thread's columns
    // (preload() or the previous call); on return they hold Qnext's (if not null).
    __device__ void apply_pf(const float2* __restrict__ Qk, const float2* __restrict__ Qnext, float2 (&qa)[PCH],
                             float2 (&qb)[PCH], const float2* s_v, float2* s_part, float2 (&out)[R]) const {
        float2 acc[R];
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = make_float2(0.f, 0.f);
        const int j0 = jp * jlen, nch = jlen / PCH;
        const int vo = (row + j0 * m) * 8;
        const __amdgpu_buffer_rsrc_t rp = block_rsrc(Qk);
        const __amdgpu_buffer_rsrc_t rn = block_rsrc(Qnext ? Qnext : Qk);
        const float2* sv = s_v + j0;
        for (int k = 0; k < nch; k += 2) {
#pragma unroll
            for (int u = 0; u < PCH; ++u)
#pragma unroll
                for (int q = 0; q < R; ++q) acc[q] = cadd(acc[q], cmul(qa[u], sv[q * m + k * PCH + u]));
            if (k + 2 < nch) {
#pragma unroll
                for (int u = 0; u < PCH; ++u) qa[u] = bload(rp, vo, (k + 2) * PCH + u);
            } else if (Qnext) {
#pragma unroll
                for (int u = 0; u < PCH; ++u) qa[u] = bload(rn, vo, u);
            }
#pragma unroll
            for (int u = 0; u < PCH; ++u)
#pragma unroll
                for (int q = 0; q < R; ++q) acc[q] = cadd(acc[q], cmul(qb[u], sv[q * m + (k + 1) * PCH + u]));
            if (k + 3 < nch) {
#pragma unroll
                for (int u = 0; u < PCH; ++u) qb[u] = bload(rp, vo, (k + 3) * PCH + u);
            } else if (Qnext) {
#pragma unroll
                for (int u = 0; u < PCH; ++u) qb[u] = bload(rn, vo, PCH + u);
            }
        }
        if (JP > 1) {
#pragma unroll
            for (int q = 0; q < R; ++q) s_part[q * CS_NT + threadIdx.x] = acc[q];
            __syncthreads();
            if (jp == 0)
                for (int t = 1; t < JP; ++t)
#pragma unroll
                    for (int q = 0; q < R; ++q) acc[q] = cadd(acc[q], s_part[q * CS_NT + t * m + row]);
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < R; ++q) out[q] = acc[q];
    }
};

// dynamic LDS of a chain kernel: s_v [R][m], then s_part [R][CS_NT] when JP > 1
static inline size_t coarse_lds_bytes(int R, int m) {
    return (size_t)R * m * sizeof(float2) + (CS_NT / m > 1 ? (size_t)R * CS_NT * sizeof(float2) : 0);
}

// The R right-hand sides of this workgroup: slot blockIdx.x * R + q of the
// slot list (slots = NULL: slot s is RHS s); *nslots_dev (if given) bounds it.
// Entries < 0 are padding; all entries of one workgroup share a slowness model.
template <int R>
struct CoarseSlots {
    int rr[R];
    bool on[R];
    bool any;
    int r0;
    __device__ CoarseSlots(const int* slots, int nslots, const int* nslots_dev, const int* active, int grp) {
        const int ns = nslots_dev ? *nslots_dev : nslots;
        any = false;
        r0 = 0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int slot = grp * R + q;
            rr[q] = (slot < ns) ? (slots ? slots[slot] : slot) : -1;
            on[q] = rr[q] >= 0 && (!active || active[rr[q]]);
            any = any || on[q];
        }
#pragma unroll
        for (int q = R - 1; q >= 0; --q)
            if (on[q]) r0 = rr[q];
    }
};

// Active right-hand sides of a single-model solve packed to the front of
// `slots` (ascending), their count in *count.  One workgroup.
__global__ void __launch_bounds__(1024) k_coarse_compact(const int* __restrict__ active, int nrhs,
                                                         int* __restrict__ slots, int* __restrict__ count) {
    __shared__ int s_wsum[16];
    __shared__ int s_base;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int r0 = 0; r0 < nrhs; r0 += 1024) {
        const int r = r0 + threadIdx.x;
        const int f = (r < nrhs && active[r]) ? 1 : 0;
        const unsigned long long bal = __ballot(f);
        const int below = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) s_wsum[wid] = __popcll(bal);
        __syncthreads();
        int off = s_base;
        for (int w = 0; w < wid; ++w) off += s_wsum[w];
        if (f) slots[off + below] = r;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int w = 0; w < 16; ++w) t += s_wsum[w];
            s_base += t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = s_base;
}

// ends: [rhs][2][m], the last forward results y_{p-1} (slot 0) and y_{p+1}
// (slot 1), kept apart from x because the backward sweep overwrites x rows.
template <int R>
__global__ void __launch_bounds__(CS_NT) k_coarse_fwd(const float2* __restrict__ bcs, float2* __restrict__ x,
                                                      float2* __restrict__ ends, const float2* __restrict__ QT,
                                                      const int* __restrict__ inst, const int* __restrict__ slots,
                                                      int nslots, const int* __restrict__ nslots_dev, int m, int p,
                                                      float c, const int* __restrict__ active) {
    extern __shared__ float2 s_lds[];
    float2* s_v = s_lds;
    float2* s_part = s_lds + R * m;
    const bool top = blockIdx.y == 0;
    const CoarseSlots<R> g(slots, nslots, nslots_dev, active, blockIdx.x);
    if (!g.any) return;
    const size_t mm = (size_t)m * m;
    const float2* Q = QT + (size_t)(inst ? inst[g.r0] : 0) * mm * m;
    const CoarseMV<R> mv(m);
    const int nsteps = top ? p : (m - 1 - p);
    for (int s = 0; s < nsteps; ++s) {
        const int k = top ? s : (m - 1 - s);
        // w_k = b_k + c y_prev  (y_prev is in s_v from the previous step)
        if (mv.owner()) {
            const int i = mv.row;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                float2 w = g.on[q] ? bcs[(size_t)g.rr[q] * mm + (size_t)k * m + i] : make_float2(0.f, 0.f);
                if (s > 0) w = cadd(w, cscale(s_v[q * m + i], c));
                s_v[q * m + i] = w;
            }
        }
        __syncthreads();
        float2 out[R];
        mv.apply(Q + (size_t)k * mm, s_v, s_part, out);
        __syncthreads();
        if (mv.owner()) {
            const int i = mv.row;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                s_v[q * m + i] = out[q];
                if (g.on[q]) {
                    x[(size_t)g.rr[q] * mm + (size_t)k * m + i] = out[q];
                    if (s == nsteps - 1) ends[((size_t)g.rr[q] * 2 + (top ? 0 : 1)) * m + i] = out[q];
                }
            }
        }
        __syncthreads();
    }
}

template <int R>
__global__ void __launch_bounds__(CS_NT) k_coarse_bwd(const float2* __restrict__ bcs, float2* __restrict__ x,
                                                      const float2* __restrict__ ends, const float2* __restrict__ QT,
                                                      const int* __restrict__ inst, const int* __restrict__ slots,
                                                      int nslots, const int* __restrict__ nslots_dev, int m, int p,
                                                      float c, const int* __restrict__ active) {
    extern __shared__ float2 s_lds[];
    float2* s_v = s_lds;
    float2* s_part = s_lds + R * m;
    const bool top = blockIdx.y == 0;
    const CoarseSlots<R> g(slots, nslots, nslots_dev, active, blockIdx.x);
    if (!g.any) return;
    const size_t mm = (size_t)m * m;
    const float2* Q = QT + (size_t)(inst ? inst[g.r0] : 0) * mm * m;
    const CoarseMV<R> mv(m);
    // middle row: x_p = Q_p (b_p + c y_{p-1} + c y_{p+1}); both workgroups compute it
    if (mv.owner()) {
        const int i = mv.row;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float2 w = make_float2(0.f, 0.f);
            if (g.on[q]) {
                w = bcs[(size_t)g.rr[q] * mm + (size_t)p * m + i];
                if (p > 0) w = cadd(w, cscale(ends[((size_t)g.rr[q] * 2 + 0) * m + i], c));
                if (p < m - 1) w = cadd(w, cscale(ends[((size_t)g.rr[q] * 2 + 1) * m + i], c));
            }
            s_v[q * m + i] = w;
        }
    }
    __syncthreads();
    {
        float2 out[R];
        mv.apply(Q + (size_t)p * mm, s_v, s_part, out);
        __syncthreads();
        if (mv.owner()) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                s_v[q * m + mv.row] = out[q];
                if (top && g.on[q]) x[(size_t)g.rr[q] * mm + (size_t)p * m + mv.row] = out[q];
            }
        }
        __syncthreads();
    }
    const int nsteps = top ? p : (m - 1 - p);
    for (int s = 0; s < nsteps; ++s) {
        const int k = top ? (p - 1 - s) : (p + 1 + s);
        float2 out[R];
        mv.apply(Q + (size_t)k * mm, s_v, s_part, out);
        __syncthreads();
        if (mv.owner()) {
            const int i = mv.row;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                float2 v = make_float2(0.f, 0.f);
                if (g.on[q]) {
                    v = cadd(x[(size_t)g.rr[q] * mm + (size_t)k * m + i], cscale(out[q], c));
                    x[(size_t)g.rr[q] * mm + (size_t)k * m + i] = v;
                }
                s_v[q * m + i] = v;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Coarse solve after one level of cyclic reduction (factors described in
// setup.hip): odd grid rows by their tridiagonal inverses V_j, even rows by the
// two-ended elimination of the reduced system, whose chain is half as long.
// Per instance the factors are slots of m x m transposed complex singles:
// j (Q_j), M + j (P_j), 2M + j (R_j), 3M + j (V_j).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int crM(int m) { return (m + 1) / 2; }
__device__ __forceinline__ int crMo(int m) { return m / 2; }

// PH 1: t_j = V_j b_{2j+1}                         (j < Mo)
// PH 2: g_j = Q_j (b_{2j} + c (t_{j-1} + t_j))     (j < M; terms beyond the rows vanish)
// PH 3: x_{2j+1} = V_j (b_{2j+1} + c (x_{2j} + x_{2j+2}))   (j < Mo)
// blockIdx.x = right-hand-side group, blockIdx.y = reduced row j.
template <int R, int PH>
__global__ void __launch_bounds__(CS_NT) k_cr_par(const float2* __restrict__ bcs, float2* __restrict__ x,
                                                  float2* __restrict__ tw, float2* __restrict__ gw,
                                                  const float2* __restrict__ F, const int* __restrict__ inst,
                                                  const int* __restrict__ slots, int nslots,
                                                  const int* __restrict__ nslots_dev, int m, float c,
                                                  const int* __restrict__ active) {
    extern __shared__ float2 s_lds[];
    float2* s_v = s_lds;
    float2* s_part = s_lds + R * m;
    const int M = crM(m), Mo = crMo(m);
    const int j = blockIdx.y;
    if (j >= (PH == 2 ? M : Mo)) return;
    const CoarseSlots<R> g(slots, nslots, nslots_dev, active, blockIdx.x);
    if (!g.any) return;
    const size_t mm = (size_t)m * m;
    const float2* Fi = F + (size_t)(inst ? inst[g.r0] : 0) * 4 * M * mm;
    const float2* Mat = Fi + (size_t)(PH == 2 ? j : 3 * M + j) * mm;
    const CoarseMV<R> mv(m);
    if (mv.owner()) {
        const int i = mv.row;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float2 w = make_float2(0.f, 0.f);
            if (g.on[q]) {
                const size_t rb = (size_t)g.rr[q] * mm;
                if (PH == 1) {
                    w = bcs[rb + (size_t)(2 * j + 1) * m + i];
                } else if (PH == 2) {
                    const float2* t = tw + (size_t)g.rr[q] * Mo * m;
                    w = bcs[rb + (size_t)(2 * j) * m + i];
                    float2 a = make_float2(0.f, 0.f);
                    if (j >= 1) a = t[(size_t)(j - 1) * m + i];
                    if (j < Mo) a = cadd(a, t[(size_t)j * m + i]);
                    w = cadd(w, cscale(a, c));
                } else {
                    float2 a = x[rb + (size_t)(2 * j) * m + i];
                    if (2 * j + 2 <= m - 1) a = cadd(a, x[rb + (size_t)(2 * j + 2) * m + i]);
                    w = cadd(bcs[rb + (size_t)(2 * j + 1) * m + i], cscale(a, c));
                }
            }
            s_v[q * m + i] = w;
        }
    }
    __syncthreads();
    float2 out[R];
    mv.apply(Mat, s_v, s_part, out);
    if (mv.owner()) {
        const int i = mv.row;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (!g.on[q]) continue;
            if (PH == 1) tw[((size_t)g.rr[q] * Mo + j) * m + i] = out[q];
            else if (PH == 2) gw[((size_t)g.rr[q] * M + j) * m + i] = out[q];
            else x[(size_t)g.rr[q] * mm + (size_t)(2 * j + 1) * m + i] = out[q];
        }
    }
}

// The steps of one end's chains at level lev (0: every chain index, factors P_j
// at slot M + j and R_j at slot 2M + j; lev >= 1: the indices 2^lev (i+1) - 1
// with the multi-step factors of FL, built in setup.hip).  Forward index s sits
// at reduced row s (top) or M-1-s (bottom), backward index t at p-1-t or p+1+t.
struct CrSteps {
    const float2* Fi;
    const float2* FLi;
    size_t mm;
    int M, p, nsteps, n, lev, e;
    bool top;
    __device__ CrSteps(const float2* F, const float2* FL, int depth, int ii, int m, bool top_) {
        M = crM(m);
        p = M / 2;
        mm = (size_t)m * m;
        top = top_;
        e = top ? 0 : 1;
        lev = FL ? depth : 0;
        Fi = F + (size_t)ii * 4 * M * mm;
        FLi = FL ? FL + (size_t)ii * cr_fl_off(M, p, depth + 1) * mm : nullptr;
        nsteps = top ? p : (M - 1 - p);
        n = nsteps >> lev;
    }
    __device__ int index(int i) const { return ((i + 1) << lev) - 1; }
    __device__ int fwd_row(int i) const { return top ? index(i) : M - 1 - index(i); }
    __device__ int bwd_row(int i) const { return top ? p - 1 - index(i) : p + 1 + index(i); }
    __device__ const float2* fwd_mat(int i) const {
        return lev ? FLi + cr_fl_block(M, p, lev, 0, e, i) * mm : Fi + (size_t)(M + fwd_row(i)) * mm;
    }
    __device__ const float2* bwd_mat(int i) const {
        return lev ? FLi + cr_fl_block(M, p, lev, 1, e, i) * mm : Fi + (size_t)(2 * M + bwd_row(i)) * mm;
    }
};

// One work item of a multi-step phase at level lev >= 1 (kind 4: forward
// combine, 5: forward fill, 6: backward combine, 7: backward fill), on chain
// index i of level lev-1 (odd for the combines, even for the fills):
//   combine: hw[row] = src(row) + A(i) src(prow)        (the next level's vectors)
//   fill:    x[row]  = src(row) + A(i) x[prow]          (no product for the forward i = 0)
// with src = g (forward) or y in x (backward) at level 0, hw above; A the level
// lev-1 factor of index i; prow the row of i-1 (x_p's row p for the backward i = 0).
// Item yidx = end * H + k, H = ((max(p, M-1-p) >> (lev-1)) + 1) / 2.
struct CrItem {
    bool valid, prod, fwd, last;
    int e, row, prow;
    const float2* mat;
    __device__ CrItem(int kind, int lev, int depth, int yidx, int H, const float2* F, const float2* FL, int ii,
                      int m) {
        const int M = crM(m), p = M / 2;
        const size_t mm = (size_t)m * m;
        e = yidx / H;
        const int k = yidx - e * H;
        const int nsteps = e == 0 ? p : M - 1 - p;
        const int i = (kind == 4 || kind == 6) ? 2 * k + 1 : 2 * k;
        valid = e < 2 && i < (nsteps >> (lev - 1));
        fwd = kind <= 5;
        const int si = ((i + 1) << (lev - 1)) - 1, sp = (i << (lev - 1)) - 1;
        auto rowf = [&](int s) { return fwd ? (e == 0 ? s : M - 1 - s) : (e == 0 ? p - 1 - s : p + 1 + s); };
        row = rowf(si);
        prow = i >= 1 ? rowf(sp) : (fwd ? 0 : p);
        prod = !(kind == 5 && i == 0);
        last = fwd && si == nsteps - 1;
        if (lev == 1) mat = F + ((size_t)ii * 4 * M + (fwd ? M : 2 * M) + row) * mm;
        else mat = FL + ((size_t)ii * cr_fl_off(M, p, depth + 1) + cr_fl_block(M, p, lev - 1, fwd ? 0 : 1, e, i)) * mm;
    }
};

// forward chains of the reduced system: y_j = g_j + P_j y_{j -/+ 1}; y_j -> x row 2j.
// Multi-step (level l): y(s) = h(s) + A_l y(s - 2^l) over the kept indices, h from the
// forward combines (k_cr_pp / k_cr_mm, PH 4).
// PF: the next step's factor is prefetched (needs CoarseMV::pf_ok(); chosen by the host).
template <int R, bool PF>
__global__ void __launch_bounds__(CS_NT) k_cr_fwd(const float2* __restrict__ gw, const float2* __restrict__ hw,
                                                  float2* __restrict__ x, float2* __restrict__ ends,
                                                  const float2* __restrict__ F, const float2* __restrict__ FL,
                                                  int depth, const int* __restrict__ inst, const int* __restrict__ slots,
                                                  int nslots, const int* __restrict__ nslots_dev, int m,
                                                  const int* __restrict__ active) {
    extern __shared__ float2 s_lds[];
    float2* s_v = s_lds;
    float2* s_part = s_lds + R * m;
    const bool top = blockIdx.y == 0;
    const CoarseSlots<R> g(slots, nslots, nslots_dev, active, blockIdx.x);
    if (!g.any) return;
    const CrSteps cs(F, FL, depth, inst ? inst[g.r0] : 0, m, top);
    const int M = cs.M;
    const size_t mm = cs.mm;
    const float2* src = cs.lev ? hw : gw;
    const CoarseMV<R> mv(m);
    constexpr bool pf = PF;
    float2 qa[CoarseMV<R>::PCH], qb[CoarseMV<R>::PCH];
    if (pf && cs.n > 1) mv.preload(cs.fwd_mat(1), qa, qb);
    for (int s = 0; s < cs.n; ++s) {
        const int j = cs.fwd_row(s);
        // g_j (h_j) does not depend on this step's product: read it first
        float2 gv[R];
#pragma unroll
        for (int q = 0; q < R; ++q)
            gv[q] = (mv.owner() && g.on[q]) ? src[((size_t)g.rr[q] * M + j) * m + mv.row] : make_float2(0.f, 0.f);
        float2 out[R];
        if (s > 0) {
            if (pf) mv.apply_pf(cs.fwd_mat(s), s + 1 < cs.n ? cs.fwd_mat(s + 1) : nullptr, qa, qb, s_v, s_part, out);
            else mv.apply(cs.fwd_mat(s), s_v, s_part, out);
        }
        __syncthreads();
        if (mv.owner()) {
            const int i = mv.row;
            const bool last = cs.index(s) == cs.nsteps - 1;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                float2 y = make_float2(0.f, 0.f);
                if (g.on[q]) {
                    y = gv[q];
                    if (s > 0) y = cadd(y, out[q]);
                    x[(size_t)g.rr[q] * mm + (size_t)(2 * j) * m + i] = y;
                    if (last) ends[((size_t)g.rr[q] * 2 + (top ? 0 : 1)) * m + i] = y;
                }
                s_v[q * m + i] = y;
            }
        }
        __syncthreads();
    }
}

// middle row and backward chains: x_p = g_p + P_p y_{p-1} + R_p y_{p+1};
// x_j = y_j + R_j x_{j +/- 1} (y_j read from, x_j written to, x row 2j).
// Multi-step (level l): x(t) = k(t) + B_l x(t - 2^l) over the kept indices (x(-1) = x_p),
// k from the backward combines (PH 6).
template <int R, bool PF>
__global__ void __launch_bounds__(CS_NT) k_cr_bwd(const float2* __restrict__ gw, const float2* __restrict__ hw,
                                                  float2* __restrict__ x, const float2* __restrict__ ends,
                                                  const float2* __restrict__ F, const float2* __restrict__ FL,
                                                  int depth, const int* __restrict__ inst, const int* __restrict__ slots,
                                                  int nslots, const int* __restrict__ nslots_dev, int m,
                                                  const int* __restrict__ active) {
    extern __shared__ float2 s_lds[];
    float2* s_v = s_lds;
    float2* s_part = s_lds + R * m;
    const bool top = blockIdx.y == 0;
    const CoarseSlots<R> g(slots, nslots, nslots_dev, active, blockIdx.x);
    if (!g.any) return;
    const CrSteps cs(F, FL, depth, inst ? inst[g.r0] : 0, m, top);
    const int M = cs.M, p = cs.p;
    const size_t mm = cs.mm;
    const float2* Fi = cs.Fi;
    const CoarseMV<R> mv(m);
    float2 acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = make_float2(0.f, 0.f);
    // middle row, computed by both workgroups
    for (int side = 0; side < 2; ++side) {
        const bool has = side == 0 ? (p >= 1) : (p + 1 <= M - 1);
        if (!has) continue;
        if (mv.owner())
#pragma unroll
            for (int q = 0; q < R; ++q)
                s_v[q * m + mv.row] =
                    g.on[q] ? ends[((size_t)g.rr[q] * 2 + side) * m + mv.row] : make_float2(0.f, 0.f);
        __syncthreads();
        float2 out[R];
        mv.apply(Fi + (size_t)((side == 0 ? M : 2 * M) + p) * mm, s_v, s_part, out);
        __syncthreads();
        if (mv.owner())
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = cadd(acc[q], out[q]);
    }
    if (mv.owner()) {
        const int i = mv.row;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float2 v = make_float2(0.f, 0.f);
            if (g.on[q]) {
                v = cadd(gw[((size_t)g.rr[q] * M + p) * m + i], acc[q]);
                if (top) x[(size_t)g.rr[q] * mm + (size_t)(2 * p) * m + i] = v;
            }
            s_v[q * m + i] = v;
        }
    }
    constexpr bool pf = PF;
    float2 qa[CoarseMV<R>::PCH], qb[CoarseMV<R>::PCH];
    if (pf && cs.n > 0) mv.preload(cs.bwd_mat(0), qa, qb);
    __syncthreads();
    for (int s = 0; s < cs.n; ++s) {
        const int j = cs.bwd_row(s);
        // y_j (k_j) does not depend on this step's product: read it first
        float2 yv[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            yv[q] = make_float2(0.f, 0.f);
            if (mv.owner() && g.on[q])
                yv[q] = cs.lev ? hw[((size_t)g.rr[q] * M + j) * m + mv.row]
                                : x[(size_t)g.rr[q] * mm + (size_t)(2 * j) * m + mv.row];
        }
        float2 out[R];
        if (pf) mv.apply_pf(cs.bwd_mat(s), s + 1 < cs.n ? cs.bwd_mat(s + 1) : nullptr, qa, qb, s_v, s_part, out);
        else mv.apply(cs.bwd_mat(s), s_v, s_part, out);
        __syncthreads();
        if (mv.owner()) {
            const int i = mv.row;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                float2 v = make_float2(0.f, 0.f);
                if (g.on[q]) {
                    v = cadd(yv[q], out[q]);
                    x[(size_t)g.rr[q] * mm + (size_t)(2 * j) * m + i] = v;
                }
                s_v[q * m + i] = v;
            }
        }
        __syncthreads();
    }
}

// The multi-step phases on the vector ALUs (kind PH 4..7 at level lev, as in
// CrItem); blockIdx.x = right-hand-side group, blockIdx.y = item.
template <int R, int PH>
__global__ void __launch_bounds__(CS_NT) k_cr_pp(const float2* __restrict__ gw, float2* __restrict__ hw,
                                                 float2* __restrict__ x, float2* __restrict__ ends,
                                                 const float2* __restrict__ F, const float2* __restrict__ FL,
                                                 int lev, int depth, int H, const int* __restrict__ inst,
                                                 const int* __restrict__ slots, int nslots,
                                                 const int* __restrict__ nslots_dev, int m,
                                                 const int* __restrict__ active) {
    extern __shared__ float2 s_lds[];
    float2* s_v = s_lds;
    float2* s_part = s_lds + R * m;
    const int M = crM(m);
    const CoarseSlots<R> g(slots, nslots, nslots_dev, active, blockIdx.x);
    if (!g.any) return;
    const CrItem it(PH, lev, depth, blockIdx.y, H, F, FL, inst ? inst[g.r0] : 0, m);
    if (!it.valid) return;
    const size_t mm = (size_t)m * m;
    constexpr bool combine = PH == 4 || PH == 6;
    // the level's source vectors: g (forward) or y in x (backward) at level 0, hw above
    auto src = [&](int rr, int row, int r) -> float2 {
        if (lev > 1) return hw[((size_t)rr * M + row) * m + r];
        return it.fwd ? gw[((size_t)rr * M + row) * m + r] : x[(size_t)rr * mm + (size_t)(2 * row) * m + r];
    };
    const CoarseMV<R> mv(m);
    float2 base[R];
    if (mv.owner()) {
        const int r = mv.row;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float2 w = make_float2(0.f, 0.f);
            base[q] = make_float2(0.f, 0.f);
            if (g.on[q]) {
                base[q] = src(g.rr[q], it.row, r);
                if (it.prod)
                    w = combine ? src(g.rr[q], it.prow, r) : x[(size_t)g.rr[q] * mm + (size_t)(2 * it.prow) * m + r];
            }
            s_v[q * m + r] = w;
        }
    }
    float2 out[R];
#pragma unroll
    for (int q = 0; q < R; ++q) out[q] = make_float2(0.f, 0.f);
    if (it.prod) {
        __syncthreads();
        mv.apply(it.mat, s_v, s_part, out);
    }
    if (mv.owner()) {
        const int r = mv.row;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (!g.on[q]) continue;
            const float2 v = cadd(base[q], out[q]);
            if (combine) {
                hw[((size_t)g.rr[q] * M + it.row) * m + r] = v;
            } else {
                x[(size_t)g.rr[q] * mm + (size_t)(2 * it.row) * m + r] = v;
                if (it.last) ends[((size_t)g.rr[q] * 2 + it.e) * m + r] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Split coarse solve.  One chain step streams a whole m x m Schur inverse; a
// single workgroup cannot pull that faster than one CU's share of the memory
// system, so here the rows of every Q_k are shared by S workgroups ("slices")
// that advance through the chain together.  The slices of one (end, RHS
// group) unit exchange each step's result vector through a double-buffered
// global buffer and meet at a counter after every step.  All slices of a unit
// run on one XCD (blockIdx mod 8), the launch is cooperative (every workgroup
// resident), and every wait is bounded: on a timeout the kernel sets *err and
// carries on without waiting, so every wave reaches its end.
// ---------------------------------------------------------------------------
constexpr int CSP_NT = 256;
constexpr int CSP_SPIN_LIMIT = 1 << 22;  // ~0.1 s of polling

struct SplitGeom {
    int G;      // right-hand-side groups of R
    int S;      // slices per unit (RS rows each)
    int units;  // 2 G: unit u = group u / 2, end u % 2 (0 = top)
    int upx;    // units per XCD lane: ceil(units / 8)
};

__device__ __forceinline__ bool split_decode(const SplitGeom& geo, int& unit, int& slice) {
    const int b = blockIdx.x;
    const int xcd = b & 7, rest = b >> 3;
    const int lu = rest / geo.S;
    slice = rest - lu * geo.S;
    unit = lu * 8 + xcd;
    return unit < geo.units;
}

// all threads: wait until *cnt >= target (thread 0 polls with acquire loads)
__device__ __forceinline__ void split_wait(int* cnt, int target, int* err) {
    if (threadIdx.x == 0) {
        int spins = 0;
        while (!__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &&
               __hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > CSP_SPIN_LIMIT) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __syncthreads();
}

// all threads: the step's results (stored by wave 0) are released, then counted
__device__ __forceinline__ void split_arrive(int* cnt) {
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float2 load_agent(const float2* p) {
    const unsigned long long v =
        __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    float2 r;
    __builtin_memcpy(&r, &v, sizeof(r));
    return r;
}

// This thread's share of rows row0 .. row0 + RS - 1 of Q_k: row row0 + t % RS,
// columns j0 .. j0 + jlen - 1 with jlen = ceil(m / (CSP_NT / RS)) <= CSP_CMAX.
// Loaded one step ahead (Q_{k+1} does not depend on the chain), so the loads
// are in flight while the workgroup waits for its partners.
constexpr int CSP_CMAX = 32;

template <int RS>
__device__ __forceinline__ void split_load_q(const float2* __restrict__ Qk, int m, int row0,
                                             float2 (&qr)[CSP_CMAX]) {
    constexpr int JP = CSP_NT / RS;
    const int t = threadIdx.x, lr = t % RS, jp = t / RS;
    const int jlen = (m + JP - 1) / JP, j0 = jp * jlen;
    const bool row_ok = row0 + lr < m;
    const float2* qp = Qk + row0 + lr;
#pragma unroll
    for (int u = 0; u < CSP_CMAX; ++u)
        qr[u] = (row_ok && u < jlen && j0 + u < m) ? qp[(size_t)(j0 + u) * m] : make_float2(0.f, 0.f);
}

// rows row0 .. row0 + RS - 1 of Q_k v for the R vectors s_w[q * m + j], Q_k's
// share in registers; the CSP_NT / RS column parts meet in s_part.  Results
// in threads t < RS (wave 0).
template <int R, int RS>
__device__ __forceinline__ void split_compute(const float2 (&qr)[CSP_CMAX], const float2* s_w, float2* s_part, int m,
                                              float2 (&out)[R]) {
    constexpr int JP = CSP_NT / RS;
    const int t = threadIdx.x, lr = t % RS, jp = t / RS;
    const int jlen = (m + JP - 1) / JP, j0 = jp * jlen;
    float2 acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = make_float2(0.f, 0.f);
#pragma unroll
    for (int u = 0; u < CSP_CMAX; ++u) {
        if (u < jlen && j0 + u < m) {
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = cadd(acc[q], cmul(qr[u], s_w[q * m + j0 + u]));
        }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) s_part[(jp * RS + lr) * R + q] = acc[q];
    __syncthreads();
    if (t < RS) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float2 a = make_float2(0.f, 0.f);
            for (int u = 0; u < JP; ++u) a = cadd(a, s_part[(u * RS + t) * R + q]);
            out[q] = a;
        }
    }
}

// xch layout: [unit][parity][R][m]
template <int R>
__device__ __forceinline__ float2* xch_at(float2* xch, int unit, int par, int q, int m) {
    return xch + ((size_t)(unit * 2 + par) * R + q) * m;
}

template <int R, int RS>
__global__ void __launch_bounds__(CSP_NT) k_coarse_split_fwd(const float2* __restrict__ bcs, float2* __restrict__ x,
                                                             float2* __restrict__ ends, const float2* __restrict__ QT,
                                                             const int* __restrict__ inst, const int* __restrict__ slots,
                                                             int nslots, const int* __restrict__ nslots_dev, int m,
                                                             int p, float c, const int* __restrict__ active,
                                                             SplitGeom geo, float2* __restrict__ xch,
                                                             int* __restrict__ cnt, int* __restrict__ err) {
    extern __shared__ float2 s_lds[];
    float2* s_w = s_lds;
    float2* s_part = s_lds + R * m;
    int unit, slice;
    if (!split_decode(geo, unit, slice)) return;
    const bool top = (unit & 1) == 0;
    const CoarseSlots<R> g(slots, nslots, nslots_dev, active, unit >> 1);
    if (!g.any) return;  // the same for every slice of the unit
    const size_t mm = (size_t)m * m;
    const float2* Q = QT + (size_t)(inst ? inst[g.r0] : 0) * mm * m;
    const int row0 = slice * RS;
    const int nsteps = top ? p : (m - 1 - p);
    float2 qr[CSP_CMAX];
    if (nsteps > 0) split_load_q<RS>(Q + (size_t)(top ? 0 : m - 1) * mm, m, row0, qr);
    for (int s = 0; s < nsteps; ++s) {
        const int k = top ? s : (m - 1 - s);
        if (s > 0) split_wait(cnt + unit, geo.S * s, err);
        // w_k = b_k + c y_prev for every row
        for (int e = threadIdx.x; e < R * m; e += CSP_NT) {
            const int q = e / m, j = e - q * m;
            float2 w = make_float2(0.f, 0.f);
            if (g.on[q]) {
                w = bcs[(size_t)g.rr[q] * mm + (size_t)k * m + j];
                if (s > 0) w = cadd(w, cscale(load_agent(xch_at<R>(xch, unit, (s - 1) & 1, q, m) + j), c));
            }
            s_w[e] = w;
        }
        __syncthreads();
        float2 out[R];
        split_compute<R, RS>(qr, s_w, s_part, m, out);
        const int row = row0 + threadIdx.x;
        if (threadIdx.x < RS && row < m) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                xch_at<R>(xch, unit, s & 1, q, m)[row] = out[q];
                if (g.on[q]) {
                    x[(size_t)g.rr[q] * mm + (size_t)k * m + row] = out[q];
                    if (s == nsteps - 1) ends[((size_t)g.rr[q] * 2 + (top ? 0 : 1)) * m + row] = out[q];
                }
            }
        }
        split_arrive(cnt + unit);
        if (s + 1 < nsteps) split_load_q<RS>(Q + (size_t)(top ? k + 1 : k - 1) * mm, m, row0, qr);
    }
}

template <int R, int RS>
__global__ void __launch_bounds__(CSP_NT) k_coarse_split_bwd(const float2* __restrict__ bcs, float2* __restrict__ x,
                                                             const float2* __restrict__ ends,
                                                             const float2* __restrict__ QT,
                                                             const int* __restrict__ inst, const int* __restrict__ slots,
                                                             int nslots, const int* __restrict__ nslots_dev, int m,
                                                             int p, float c, const int* __restrict__ active,
                                                             SplitGeom geo, float2* __restrict__ xch,
                                                             int* __restrict__ cnt, int* __restrict__ err) {
    extern __shared__ float2 s_lds[];
    float2* s_w = s_lds;
    float2* s_part = s_lds + R * m;
    int unit, slice;
    if (!split_decode(geo, unit, slice)) return;
    const bool top = (unit & 1) == 0;
    const CoarseSlots<R> g(slots, nslots, nslots_dev, active, unit >> 1);
    if (!g.any) return;
    const size_t mm = (size_t)m * m;
    const float2* Q = QT + (size_t)(inst ? inst[g.r0] : 0) * mm * m;
    const int row0 = slice * RS;
    const int row = row0 + threadIdx.x;
    const int nsteps = top ? p : (m - 1 - p);
    float2 qr[CSP_CMAX];
    split_load_q<RS>(Q + (size_t)p * mm, m, row0, qr);
    // middle row (round 0): x_p = Q_p (b_p + c y_{p-1} + c y_{p+1}); both ends compute it
    for (int e = threadIdx.x; e < R * m; e += CSP_NT) {
        const int q = e / m, j = e - q * m;
        float2 w = make_float2(0.f, 0.f);
        if (g.on[q]) {
            w = bcs[(size_t)g.rr[q] * mm + (size_t)p * m + j];
            if (p > 0) w = cadd(w, cscale(ends[((size_t)g.rr[q] * 2 + 0) * m + j], c));
            if (p < m - 1) w = cadd(w, cscale(ends[((size_t)g.rr[q] * 2 + 1) * m + j], c));
        }
        s_w[e] = w;
    }
    __syncthreads();
    {
        float2 out[R];
        split_compute<R, RS>(qr, s_w, s_part, m, out);
        if (threadIdx.x < RS && row < m) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                xch_at<R>(xch, unit, 0, q, m)[row] = out[q];
                if (top && g.on[q]) x[(size_t)g.rr[q] * mm + (size_t)p * m + row] = out[q];
            }
        }
        split_arrive(cnt + unit);
        if (nsteps > 0) split_load_q<RS>(Q + (size_t)(top ? p - 1 : p + 1) * mm, m, row0, qr);
    }
    for (int s = 0; s < nsteps; ++s) {
        const int k = top ? (p - 1 - s) : (p + 1 + s);
        split_wait(cnt + unit, geo.S * (s + 1), err);
        for (int e = threadIdx.x; e < R * m; e += CSP_NT) {
            const int q = e / m, j = e - q * m;
            s_w[e] = g.on[q] ? load_agent(xch_at<R>(xch, unit, s & 1, q, m) + j) : make_float2(0.f, 0.f);
        }
        __syncthreads();
        float2 out[R];
        split_compute<R, RS>(qr, s_w, s_part, m, out);
        if (threadIdx.x < RS && row < m) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                float2 v = make_float2(0.f, 0.f);
                if (g.on[q]) {
                    v = cadd(x[(size_t)g.rr[q] * mm + (size_t)k * m + row], cscale(out[q], c));
                    x[(size_t)g.rr[q] * mm + (size_t)k * m + row] = v;
                }
                xch_at<R>(xch, unit, (s + 1) & 1, q, m)[row] = v;
            }
        }
        split_arrive(cnt + unit);
        if (s + 1 < nsteps) split_load_q<RS>(Q + (size_t)(top ? k - 1 : k + 1) * mm, m, row0, qr);
    }
}

// ---- split form of the reduced solve's chains ------------------------------
// The same slices, counters and exchange as the split solve above, on the
// reduced chains: forward y_j = g_j + P_j y_{j -/+ 1} (no product at an end's
// first row); middle row x_p = g_p + P_p y_{p-1} + R_p y_{p+1}; backward
// x_j = y_j + R_j x_{j +/- 1}.  Factor slots as in k_cr_fwd / k_cr_bwd.
template <int R, int RS>
__global__ void __launch_bounds__(CSP_NT) k_cr_split_fwd(const float2* __restrict__ gw, const float2* __restrict__ hw,
                                                         float2* __restrict__ x, float2* __restrict__ ends,
                                                         const float2* __restrict__ F, const float2* __restrict__ FL,
                                                         int depth, const int* __restrict__ inst,
                                                         const int* __restrict__ slots,
                                                         int nslots, const int* __restrict__ nslots_dev, int m,
                                                         const int* __restrict__ active, SplitGeom geo,
                                                         float2* __restrict__ xch, int* __restrict__ cnt,
                                                         int* __restrict__ err) {
    extern __shared__ float2 s_lds[];
    float2* s_w = s_lds;
    float2* s_part = s_lds + R * m;
    int unit, slice;
    if (!split_decode(geo, unit, slice)) return;
    const bool top = (unit & 1) == 0;
    const CoarseSlots<R> g(slots, nslots, nslots_dev, active, unit >> 1);
    if (!g.any) return;  // the same for every slice of the unit
    const CrSteps cs(F, FL, depth, inst ? inst[g.r0] : 0, m, top);
    const int M = cs.M;
    const size_t mm = cs.mm;
    const float2* src = cs.lev ? hw : gw;
    const int row0 = slice * RS;
    const int row = row0 + threadIdx.x;
    float2 qr[CSP_CMAX];
    if (cs.n > 1) split_load_q<RS>(cs.fwd_mat(1), m, row0, qr);
    for (int s = 0; s < cs.n; ++s) {
        const int j = cs.fwd_row(s);
        float2 out[R];
        if (s > 0) {
            split_wait(cnt + unit, geo.S * s, err);
            for (int e = threadIdx.x; e < R * m; e += CSP_NT) {
                const int q = e / m, i = e - q * m;
                s_w[e] = g.on[q] ? load_agent(xch_at<R>(xch, unit, (s - 1) & 1, q, m) + i) : make_float2(0.f, 0.f);
            }
            __syncthreads();
            split_compute<R, RS>(qr, s_w, s_part, m, out);
        }
        if (threadIdx.x < RS && row < m) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                float2 y = make_float2(0.f, 0.f);
                if (g.on[q]) {
                    y = src[((size_t)g.rr[q] * M + j) * m + row];
                    if (s > 0) y = cadd(y, out[q]);
                    x[(size_t)g.rr[q] * mm + (size_t)(2 * j) * m + row] = y;
                    if (cs.index(s) == cs.nsteps - 1) ends[((size_t)g.rr[q] * 2 + (top ? 0 : 1)) * m + row] = y;
                }
                xch_at<R>(xch, unit, s & 1, q, m)[row] = y;
            }
        }
        split_arrive(cnt + unit);
        if (s > 0 && s + 1 < cs.n) split_load_q<RS>(cs.fwd_mat(s + 1), m, row0, qr);
    }
}

template <int R, int RS>
__global__ void __launch_bounds__(CSP_NT) k_cr_split_bwd(const float2* __restrict__ gw, const float2* __restrict__ hw,
                                                         float2* __restrict__ x, const float2* __restrict__ ends,
                                                         const float2* __restrict__ F, const float2* __restrict__ FL,
                                                         int depth, const int* __restrict__ inst,
                                                         const int* __restrict__ slots,
                                                         int nslots, const int* __restrict__ nslots_dev, int m,
                                                         const int* __restrict__ active, SplitGeom geo,
                                                         float2* __restrict__ xch, int* __restrict__ cnt,
                                                         int* __restrict__ err) {
    extern __shared__ float2 s_lds[];
    float2* s_w = s_lds;
    float2* s_part = s_lds + R * m;
    int unit, slice;
    if (!split_decode(geo, unit, slice)) return;
    const bool top = (unit & 1) == 0;
    const CoarseSlots<R> g(slots, nslots, nslots_dev, active, unit >> 1);
    if (!g.any) return;
    const CrSteps cs(F, FL, depth, inst ? inst[g.r0] : 0, m, top);
    const int M = cs.M, p = cs.p;
    const size_t mm = cs.mm;
    const float2* Fi = cs.Fi;
    const int row0 = slice * RS;
    const int row = row0 + threadIdx.x;
    float2 qr[CSP_CMAX];
    // middle row (round 0), computed by both ends
    float2 acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = make_float2(0.f, 0.f);
    for (int side = 0; side < 2; ++side) {
        const bool has = side == 0 ? (p >= 1) : (p + 1 <= M - 1);
        if (!has) continue;
        split_load_q<RS>(Fi + (size_t)((side == 0 ? M : 2 * M) + p) * mm, m, row0, qr);
        for (int e = threadIdx.x; e < R * m; e += CSP_NT) {
            const int q = e / m, i = e - q * m;
            s_w[e] = g.on[q] ? ends[((size_t)g.rr[q] * 2 + side) * m + i] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        float2 out[R];
        split_compute<R, RS>(qr, s_w, s_part, m, out);
        if (threadIdx.x < RS)
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = cadd(acc[q], out[q]);
    }
    if (threadIdx.x < RS && row < m) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float2 v = make_float2(0.f, 0.f);
            if (g.on[q]) {
                v = cadd(gw[((size_t)g.rr[q] * M + p) * m + row], acc[q]);
                if (top) x[(size_t)g.rr[q] * mm + (size_t)(2 * p) * m + row] = v;
            }
            xch_at<R>(xch, unit, 0, q, m)[row] = v;
        }
    }
    split_arrive(cnt + unit);
    if (cs.n > 0) split_load_q<RS>(cs.bwd_mat(0), m, row0, qr);
    for (int s = 0; s < cs.n; ++s) {
        const int j = cs.bwd_row(s);
        split_wait(cnt + unit, geo.S * (s + 1), err);
        for (int e = threadIdx.x; e < R * m; e += CSP_NT) {
            const int q = e / m, i = e - q * m;
            s_w[e] = g.on[q] ? load_agent(xch_at<R>(xch, unit, s & 1, q, m) + i) : make_float2(0.f, 0.f);
        }
        __syncthreads();
        float2 out[R];
        split_compute<R, RS>(qr, s_w, s_part, m, out);
        if (threadIdx.x < RS && row < m) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                float2 v = make_float2(0.f, 0.f);
                if (g.on[q]) {
                    const size_t o = (size_t)g.rr[q] * mm + (size_t)(2 * j) * m + row;
                    v = cadd(cs.lev ? hw[((size_t)g.rr[q] * M + j) * m + row] : x[o], out[q]);
                    x[o] = v;
                }
                xch_at<R>(xch, unit, (s + 1) & 1, q, m)[row] = v;
            }
        }
        split_arrive(cnt + unit);
        if (s + 1 < cs.n) split_load_q<RS>(cs.bwd_mat(s + 1), m, row0, qr);
    }
}

__global__ void k_zero_ints(int* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hh_status launch_apply_op(hh_model* md, int level, float shift, int nrhs, const int* inst_dev,
                          const float2* x, float2* y, const int* active) {
    const Level& L = md->lev[level];
    ProfScope ps(md->ctx, HH_K_OPERATOR);
    dim3 blk(OP_TX, OP_TY / OP_ROWS), grd((L.n + OP_TX - 1) / OP_TX, (L.n + OP_TY - 1) / OP_TY, nrhs);
    hipLaunchKernelGGL(k_apply_op, grd, blk, 0, md->ctx->stream, x, y, L.coef.as<float2>(), inst_dev, L.n,
                       (float)(1.0 / (L.h * L.h)), shift, active);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// workspace: per level l >= 1: b_l and e_l [nrhs][n_l][n_l]; the coarse solve's
// [nrhs][2][m] exchange rows; x1 [nrhs][n][n] if with_x0; then the coarse
// solve's compacted slot list (nrhs ints) and its length
static size_t vcycle_float_bytes(const hh_model* md, int nrhs, bool with_x0) {
    size_t bytes = 0;
    for (int l = 1; l < md->nlev; ++l) bytes += 2 * (size_t)nrhs * md->lev[l].n * md->lev[l].n * sizeof(float2);
    bytes += 2 * (size_t)nrhs * md->lev[md->nlev - 1].n * sizeof(float2);
    if (with_x0) bytes += (size_t)nrhs * md->lev[0].n * md->lev[0].n * sizeof(float2);
    return bytes;
}

// slots of the coarse solve: the RHS list, or the grouping order padded per model
static int coarse_slot_bound(const hh_model* md, int nrhs) { return nrhs + CS_RMAX * md->ninst; }

// after the float part: slot list, its count, the split solve's step counters
// (2 sweeps x units) and exchange vectors ([unit][2][R][m], units * R <= 2 (slots + CS_RMAX))
struct CoarseWork {
    int* slots;
    int* count;
    int* cnt;
    float2* xch;
    float2* tw;  // reduced solve: V_j b_{2j+1}, [rhs][Mo][m]
    float2* gw;  // reduced solve: g_j, [rhs][M][m]
    float2* hw;  // multi-step chains: the combined vectors h, then k, at their reduced rows, [rhs][M][m]
};
static size_t coarse_work_bytes(const hh_model* md, int nrhs) {
    const size_t ns = (size_t)coarse_slot_bound(md, nrhs);
    const int m = md->lev[md->nlev - 1].n;
    return (ns + 64) * sizeof(int) + 4 * (ns + CS_RMAX) * sizeof(int) + 256 +
           4 * (ns + CS_RMAX) * (size_t)m * sizeof(float2) + 256 +
           (size_t)nrhs * (m / 2 + 2 * ((m + 1) / 2)) * m * sizeof(float2);
}
static CoarseWork coarse_work(const hh_model* md, void* base, int nrhs) {
    const size_t ns = (size_t)coarse_slot_bound(md, nrhs);
    const int m = md->lev[md->nlev - 1].n;
    CoarseWork w;
    char* q = (char*)base;
    w.slots = (int*)q;
    w.count = w.slots + ns;
    q += (ns + 64) * sizeof(int);
    w.cnt = (int*)q;
    q += 4 * (ns + CS_RMAX) * sizeof(int);
    q = (char*)(((uintptr_t)q + 255) & ~(uintptr_t)255);
    w.xch = (float2*)q;
    q += 4 * (ns + CS_RMAX) * (size_t)m * sizeof(float2);
    q = (char*)(((uintptr_t)q + 255) & ~(uintptr_t)255);
    w.tw = (float2*)q;
    w.gw = w.tw + (size_t)nrhs * (m / 2) * m;
    w.hw = w.gw + (size_t)nrhs * ((m + 1) / 2) * m;
    return w;
}

size_t vcycle_workspace_bytes(const hh_model* md, int nrhs, bool with_x0) {
    return vcycle_float_bytes(md, nrhs, with_x0) + coarse_work_bytes(md, nrhs) + 256 + coarse_gmres_bytes(md, nrhs) +
           256;
}

int coarse_group() { return CS_RMAX; }

// ---- coarse block solve: launch with R right-hand sides per workgroup -------
template <int R>
static hh_status launch_coarse_t(hh_ctx* ctx, const float2* bcs, float2* x, float2* ends, const float2* QT,
                                 const int* inst, const int* slots, int nslots, const int* nslots_dev, int m, int p,
                                 float c, const int* active) {
    static unsigned attr_devices = 0;  // devices on which the LDS limit was raised
    const size_t lds = coarse_lds_bytes(R, m);
    if (lds > 65536 && !(attr_devices & (1u << ctx->device))) {
        size_t most = 0;  // the largest need over every supported m
        for (int mm = 4; mm <= CS_MAXM; ++mm) most = std::max(most, coarse_lds_bytes(R, mm));
        const int want = (int)most;
        HH_HIP(hipFuncSetAttribute((const void*)k_coarse_fwd<R>, hipFuncAttributeMaxDynamicSharedMemorySize, want));
        HH_HIP(hipFuncSetAttribute((const void*)k_coarse_bwd<R>, hipFuncAttributeMaxDynamicSharedMemorySize, want));
        attr_devices |= 1u << ctx->device;
    }
    const dim3 grd((nslots + R - 1) / R, 2);
    hipLaunchKernelGGL(k_coarse_fwd<R>, grd, dim3(CS_NT), lds, ctx->stream, bcs, x, ends, QT, inst, slots, nslots,
                       nslots_dev, m, p, c, active);
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_coarse_bwd<R>, grd, dim3(CS_NT), lds, ctx->stream, bcs, x, ends, QT, inst, slots, nslots,
                       nslots_dev, m, p, c, active);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

static hh_status launch_coarse(int R, hh_ctx* ctx, const float2* bcs, float2* x, float2* ends, const float2* QT,
                               const int* inst, const int* slots, int nslots, const int* nslots_dev, int m, int p,
                               float c, const int* active) {
    switch (R) {
        case 1: return launch_coarse_t<1>(ctx, bcs, x, ends, QT, inst, slots, nslots, nslots_dev, m, p, c, active);
        case 2: return launch_coarse_t<2>(ctx, bcs, x, ends, QT, inst, slots, nslots, nslots_dev, m, p, c, active);
        case 4: return launch_coarse_t<4>(ctx, bcs, x, ends, QT, inst, slots, nslots, nslots_dev, m, p, c, active);
        case 8: return launch_coarse_t<8>(ctx, bcs, x, ends, QT, inst, slots, nslots, nslots_dev, m, p, c, active);
        default: set_error("coarse group size %d (1, 2, 4 or 8)", R); return HH_ERR_ARG;
    }
}

// ---- split solve: S workgroups per (end, group), cooperative launch ---------
static size_t split_lds_bytes(int R, int m) { return (size_t)R * m * sizeof(float2) + (size_t)CSP_NT * R * sizeof(float2); }

template <int R, int RS>
static hh_status launch_split_t(hh_model* md, const float2* bcs, float2* x, float2* ends, const int* inst,
                                const int* slots, int nslots, const int* nslots_dev, int m, int p, float c,
                                const int* active, const CoarseWork& cw, bool* fits) {
    hh_ctx* ctx = md->ctx;
    static unsigned attr_devices = 0;
    const size_t lds = split_lds_bytes(R, m);
    if (split_lds_bytes(R, CS_MAXM) > 65536 && !(attr_devices & (1u << ctx->device))) {
        const int want = (int)split_lds_bytes(R, CS_MAXM);
        HH_HIP(hipFuncSetAttribute((const void*)k_coarse_split_fwd<R, RS>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, want));
        HH_HIP(hipFuncSetAttribute((const void*)k_coarse_split_bwd<R, RS>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, want));
        attr_devices |= 1u << ctx->device;
    }
    if (ctx->concurrent || (m + CSP_NT / RS - 1) / (CSP_NT / RS) > CSP_CMAX) {
        *fits = false;  // other streams may hold CUs, or the column share exceeds the registers
        return HH_OK;
    }
    SplitGeom geo;
    geo.G = (nslots + R - 1) / R;
    geo.S = (m + RS - 1) / RS;
    geo.units = 2 * geo.G;
    geo.upx = (geo.units + 7) / 8;
    const int grid = 8 * geo.upx * geo.S;
    int per_cu_f = 0, per_cu_b = 0;
    HH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_f, (const void*)k_coarse_split_fwd<R, RS>, CSP_NT,
                                                        lds));
    HH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_b, (const void*)k_coarse_split_bwd<R, RS>, CSP_NT,
                                                        lds));
    if ((long long)std::min(per_cu_f, per_cu_b) * ctx->num_cus < grid) {
        *fits = false;  // not every workgroup could be resident: not offered
        return HH_OK;
    }
    *fits = true;
    hipLaunchKernelGGL(k_zero_ints, dim3((2 * geo.units + 255) / 256), dim3(256), 0, ctx->stream, cw.cnt,
                       2 * geo.units);
    HH_LAUNCH_CHECK();
    const float2* a_bcs = bcs;
    float2* a_x = x;
    float2* a_ends = ends;
    const float2* a_QT = md->coarseQT.as<float2>();
    const int* a_inst = inst;
    const int* a_slots = slots;
    int a_nslots = nslots;
    const int* a_nsd = nslots_dev;
    int a_m = m, a_p = p;
    float a_c = c;
    const int* a_act = active;
    float2* a_xch = cw.xch;
    int* a_cnt = cw.cnt;
    int* a_err = md->coarse_err.as<int>();
    void* args[] = {&a_bcs, &a_x, &a_ends, &a_QT, &a_inst, &a_slots, &a_nslots, &a_nsd, &a_m,   &a_p,
                    &a_c,   &a_act, &geo, &a_xch, &a_cnt, &a_err};
    const hipError_t le = hipLaunchCooperativeKernel((const void*)k_coarse_split_fwd<R, RS>, dim3(grid),
                                                     dim3(CSP_NT), args, (unsigned)lds, ctx->stream);
    if (le == hipErrorCooperativeLaunchTooLarge) {  // the runtime's residency bound is tighter: not offered
        (void)hipGetLastError();
        *fits = false;
        return HH_OK;
    }
    if (le != hipSuccess) {
        set_error("cooperative launch failed: %s", hipGetErrorString(le));
        return HH_ERR_HIP;
    }
    const float2* b_ends = ends;
    int* b_cnt = cw.cnt + geo.units;
    void* args_b[] = {&a_bcs, &a_x, &b_ends, &a_QT, &a_inst, &a_slots, &a_nslots, &a_nsd, &a_m,   &a_p,
                      &a_c,   &a_act, &geo, &a_xch, &b_cnt, &a_err};
    HH_HIP(hipLaunchCooperativeKernel((const void*)k_coarse_split_bwd<R, RS>, dim3(grid), dim3(CSP_NT), args_b,
                                      (unsigned)lds, ctx->stream));
    return HH_OK;
}

// ---- reduced solve (one level of cyclic reduction, then the two-ended chains) ----
// The row-parallel phases serve CS_RMAX right-hand sides per workgroup whatever
// the chains use: their blocks are then read CS_RMAX times fewer (slot groups of
// CS_RMAX never mix models: the grouping order is padded per model to CS_RMAX).
static hh_status launch_cr_mm(hh_model* md, int PH, int lev, const float2* bcs, float2* x, float2* ends,
                              const int* inst, const int* slots, int nslots, const int* nslots_dev, int m, float c,
                              const int* active, const CoarseWork& cw);

static hh_status launch_cr_par(hh_model* md, int PH, const float2* bcs, float2* x, const int* inst, const int* slots,
                               int nslots, const int* nslots_dev, int m, float c, const int* active,
                               const CoarseWork& cw) {
    if (md->coarse_mm && nslots > CS_RMAX)
        return launch_cr_mm(md, PH, 0, bcs, x, nullptr, inst, slots, nslots, nslots_dev, m, c, active, cw);
    constexpr int RP = CS_RMAX;
    hh_ctx* ctx = md->ctx;
    static unsigned attr_devices = 0;
    if (!(attr_devices & (1u << ctx->device))) {
        size_t mostp = 0;
        for (int mm_ = 4; mm_ <= CS_MAXM; ++mm_) mostp = std::max(mostp, coarse_lds_bytes(RP, mm_));
        if (mostp > 65536) {
            const int want = (int)mostp;
            HH_HIP(hipFuncSetAttribute((const void*)k_cr_par<RP, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, want));
            HH_HIP(hipFuncSetAttribute((const void*)k_cr_par<RP, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, want));
            HH_HIP(hipFuncSetAttribute((const void*)k_cr_par<RP, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, want));
        }
        attr_devices |= 1u << ctx->device;
    }
    const size_t ldsp = coarse_lds_bytes(RP, m);
    const int GP = (nslots + RP - 1) / RP;
    const int M = (m + 1) / 2, Mo = m / 2;
    const float2* F = md->coarseQT.as<float2>();
    hipStream_t st = ctx->stream;
    const int rows = PH == 2 ? M : Mo;
    if (rows == 0) return HH_OK;
    if (PH == 1)
        hipLaunchKernelGGL((k_cr_par<RP, 1>), dim3(GP, rows), dim3(CS_NT), ldsp, st, bcs, x, cw.tw, cw.gw, F, inst,
                           slots, nslots, nslots_dev, m, c, active);
    else if (PH == 2)
        hipLaunchKernelGGL((k_cr_par<RP, 2>), dim3(GP, rows), dim3(CS_NT), ldsp, st, bcs, x, cw.tw, cw.gw, F, inst,
                           slots, nslots, nslots_dev, m, c, active);
    else
        hipLaunchKernelGGL((k_cr_par<RP, 3>), dim3(GP, rows), dim3(CS_NT), ldsp, st, bcs, x, cw.tw, cw.gw, F, inst,
                           slots, nslots, nslots_dev, m, c, active);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// ---------------------------------------------------------------------------
// The row-parallel phases (PH 1..3 of k_cr_par, PH 4..7 of k_cr_pp) on the
// matrix cores.  One workgroup takes one factor block, a tile of 16 right-hand
// sides and a group of output columns; Y^T (16 x m) = W^T (16 x m) S (m x m), where S is the stored
// slot ([c][r] = the factor transposed) and W the phase's gathered input
// vectors (in LDS), as three real products on v_mfma_f32_16x16x4f32 (FP32
// inputs and accumulation, the precision of the vector-ALU form).  Wave w
// covers output columns CW cg + 16 w .. + 15 of column group cg.  A tile whose right-hand sides
// belong to several slowness models runs once per model, each pass with that
// model's factors and its own rows.
// ---------------------------------------------------------------------------
typedef float cmm_f4 __attribute__((ext_vector_type(4)));

// W^T rows padded to whole groups of 16 k-steps (any prefetch depth up to 16; zeros beyond m), plus one
static inline __host__ __device__ int cmm_kpad(int m) { return (m + 4 * 16 - 1) / (4 * 16) * (4 * 16); }
static inline size_t cmm_lds_bytes(int m) { return (size_t)16 * (cmm_kpad(m) + 1) * sizeof(float2); }

// NW waves per workgroup (16 columns each): sixteen for the phases over every
// factor block (PH 1..3), four for the multi-step phases, whose few blocks are
// then spread over more compute units
template <int PH>
constexpr int cmm_waves() { return PH <= 3 ? 16 : 4; }
// k-steps of factor fragments in flight per wave: deeper for the four-wave
// workgroups, whose few waves per compute unit hide less latency
template <int PH>
constexpr int cmm_depth() { return PH <= 3 ? 8 : 16; }

template <int PH>
__global__ void __launch_bounds__(64 * cmm_waves<PH>()) k_cr_mm(const float2* __restrict__ bcs, float2* __restrict__ x,
                                                  float2* __restrict__ tw, float2* __restrict__ gw,
                                                  float2* __restrict__ hw, float2* __restrict__ ends,
                                                  const float2* __restrict__ F, const float2* __restrict__ FL,
                                                  int lev, int depth, const int* __restrict__ inst,
                                                  const int* __restrict__ slots, int nslots,
                                                  const int* __restrict__ nslots_dev, int m, float cf,
                                                  const int* __restrict__ active, int rows, int ntiles) {
    extern __shared__ float2 s_w[];  // [16][ldw]: W^T, zero beyond m
    __shared__ int s_rr[16], s_in[16];
    const int M = crM(m), Mo = crMo(m), p = M / 2;
    const size_t mm = (size_t)m * m;
    constexpr int DPF = cmm_depth<PH>();
    const int m4 = cmm_kpad(m), ldw = m4 + 1, nks = m4 / 4;  // nks: a multiple of 16, so of DPF
    // workgroup -> (row, tile, column group): all workgroups of a row on one XCD
    // (workgroup id mod 8), so that its factor block is fetched into that XCD's L2 once
    constexpr int CMM_NT = 64 * cmm_waves<PH>(), CW = 16 * cmm_waves<PH>();  // threads, columns per workgroup
    const int ncg = (m + CW - 1) / CW, ntc = ntiles * ncg;
    const int xcd = blockIdx.x & 7, kk = blockIdx.x >> 3;
    const int row = (kk / ntc) * 8 + xcd, rem = kk % ntc;
    const int tile = rem / ncg, cg = rem - tile * ncg;
    if (row >= rows) return;
    // the block row (the reduced row for PH 1..3, the multi-step item for PH 4..7)
    int j, jm = 0;
    bool prod = true;
    const CrItem it0(PH >= 4 ? PH : 4, lev > 0 ? lev : 1, depth, row, rows / 2, F, FL, 0, m);
    if (PH <= 3) {
        j = row;
    } else {
        if (!it0.valid) return;
        j = it0.row;
        jm = it0.prow;
        prod = it0.prod;
    }
    const int slot_of = PH == 2 ? j : 3 * M + j;  // PH 1..3
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t < 16) {
        const int ns = nslots_dev ? *nslots_dev : nslots;
        const int slot = tile * 16 + t;
        const int rr = slot < ns ? (slots ? slots[slot] : slot) : -1;
        const bool on = rr >= 0 && (!active || active[rr]);
        s_rr[t] = on ? rr : -1;
        s_in[t] = on ? (inst ? inst[rr] : 0) : -1;
    }
    __syncthreads();
    int done = 0;
    for (;;) {
        // the next model of the tile (the same decision in every thread)
        int pm = -1;
        for (int q = 0; q < 16; ++q)
            if (s_rr[q] >= 0 && !((done >> q) & 1)) {
                pm = s_in[q];
                break;
            }
        if (pm < 0) break;
        int mask = 0;
        for (int q = 0; q < 16; ++q)
            if (s_rr[q] >= 0 && s_in[q] == pm) mask |= 1 << q;
        done |= mask;
        // gather W^T into LDS (four elements per thread in flight at a time)
        if (prod) {
            auto gather = [&](int e2) -> float2 {
                const int n = e2 / m4, c = e2 - n * m4;
                float2 w = make_float2(0.f, 0.f);
                const int rr = s_rr[n];
                if (((mask >> n) & 1) && c < m) {
                    const size_t rb = (size_t)rr * mm;
                    if (PH == 1) {
                        w = bcs[rb + (size_t)(2 * j + 1) * m + c];
                    } else if (PH == 2) {
                        w = bcs[rb + (size_t)(2 * j) * m + c];
                        float2 a = make_float2(0.f, 0.f);
                        if (j >= 1) a = tw[((size_t)rr * Mo + j - 1) * m + c];
                        if (j < Mo) a = cadd(a, tw[((size_t)rr * Mo + j) * m + c]);
                        w = cadd(w, cscale(a, cf));
                    } else if (PH == 3) {
                        float2 a = x[rb + (size_t)(2 * j) * m + c];
                        if (2 * j + 2 <= m - 1) a = cadd(a, x[rb + (size_t)(2 * j + 2) * m + c]);
                        w = cadd(bcs[rb + (size_t)(2 * j + 1) * m + c], cscale(a, cf));
                    } else if (PH == 4 || PH == 6) {  // the previous index's source vector
                        w = lev > 1 ? hw[((size_t)rr * M + jm) * m + c]
                                    : (PH == 4 ? gw[((size_t)rr * M + jm) * m + c] : x[rb + (size_t)(2 * jm) * m + c]);
                    } else {  // fills: the previous index's result
                        w = x[rb + (size_t)(2 * jm) * m + c];
                    }
                }
                return w;
            };
            const int total = 16 * m4;
            for (int e0 = t; e0 < total; e0 += 4 * CMM_NT) {
                float2 w[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int e2 = e0 + k * CMM_NT;
                    w[k] = e2 < total ? gather(e2) : make_float2(0.f, 0.f);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int e2 = e0 + k * CMM_NT;
                    if (e2 < total) {
                        const int n = e2 / m4, c = e2 - n * m4;
                        s_w[n * ldw + c] = w[k];
                    }
                }
            }
            __syncthreads();
        }
        const float2* S = PH <= 3 ? F + ((size_t)pm * 4 * M + slot_of) * mm
                                  : CrItem(PH, lev, depth, row, rows / 2, F, FL, pm, m).mat;
        const __amdgpu_buffer_rsrc_t rs = [&] {
            const unsigned long long a = (unsigned long long)S;
            const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
            const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
            return __builtin_amdgcn_make_buffer_rsrc((void*)(((unsigned long long)hi << 32) | lo), (short)0,
                                                     (int)(mm * sizeof(float2)), 0x00020000);
        }();
        const int kl = lane >> 4, cl = lane & 15;
        for (int cb = cg * CW + wave * 16; cb < m && cb < (cg + 1) * CW; cb += CW) {
            cmm_f4 accr = (cmm_f4){0.f, 0.f, 0.f, 0.f}, acci = (cmm_f4){0.f, 0.f, 0.f, 0.f};
            cmm_f4 accq = (cmm_f4){0.f, 0.f, 0.f, 0.f};
            if (prod) {
                // S fragment at k-step k: S[4 k + kl][cb + cl], row and column clamped into
                // the block (rows >= m meet zeros of W; columns >= m are not stored)
                const int col = min(cb + cl, m - 1);
                auto sfrag = [&](int k) {
                    const int off = (min(4 * k + kl, m - 1) * m + col) * (int)sizeof(float2);
                    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
                };
                // branch-free pipeline: every k-step refills its buffer DPF steps ahead
                // (past the end the clamped row is read and not used)
                float2 bq[DPF];
#pragma unroll
                for (int d = 0; d < DPF; ++d) {
                    bq[d] = sfrag(d);
                    __builtin_amdgcn_sched_barrier(0);  // issued in order of use
                }
                for (int ks = 0; ks < nks; ks += DPF) {
#pragma unroll
                    for (int d = 0; d < DPF; ++d) {
                        const int k = ks + d;
                        const float2 a = s_w[cl * ldw + 4 * k + kl];
                        const float2 b = bq[d];
                        bq[d] = sfrag(k + DPF);
                        // three real products (Gauss): ar br, ai bi, (ar + ai)(br + bi)
                        accr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, accr, 0, 0, 0);
                        accq = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, accq, 0, 0, 0);
                        acci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x + a.y, b.x + b.y, acci, 0, 0, 0);
                        // keep each refill in its k-step: the wait before a use is then
                        // for the load issued DPF steps earlier only
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                // Re = ar br - ai bi, Im = (ar + ai)(br + bi) - ar br - ai bi
                acci = acci - accr - accq;
                accr = accr - accq;
            }
            // lane holds rows (right-hand sides) 4 kl + v of column cb + cl
            const int r = cb + cl;
            if (r < m) {
                if (PH <= 3) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int n = 4 * kl + v;
                        if (!((mask >> n) & 1)) continue;
                        const int rr = s_rr[n];
                        const float2 y = make_float2(accr[v], acci[v]);
                        if (PH == 1) tw[((size_t)rr * Mo + j) * m + r] = y;
                        else if (PH == 2) gw[((size_t)rr * M + j) * m + r] = y;
                        else x[(size_t)rr * mm + (size_t)(2 * j + 1) * m + r] = y;
                    }
                } else {
                    // this index's source vectors (g / y at level 0, hw above), all loaded first
                    float2 b[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int n = 4 * kl + v;
                        b[v] = make_float2(0.f, 0.f);
                        if ((mask >> n) & 1) {
                            const int rr = s_rr[n];
                            const size_t oh = ((size_t)rr * M + j) * m + r;
                            const size_t ox = (size_t)rr * mm + (size_t)(2 * j) * m + r;
                            b[v] = lev > 1 ? hw[oh] : (PH <= 5 ? gw[oh] : x[ox]);
                        }
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int n = 4 * kl + v;
                        if (!((mask >> n) & 1)) continue;
                        const int rr = s_rr[n];
                        const size_t oh = ((size_t)rr * M + j) * m + r;
                        const size_t ox = (size_t)rr * mm + (size_t)(2 * j) * m + r;
                        const float2 val = cadd(b[v], make_float2(accr[v], acci[v]));
                        if (PH == 4 || PH == 6) {
                            hw[oh] = val;
                        } else {
                            x[ox] = val;
                            if (it0.last) ends[((size_t)rr * 2 + it0.e) * m + r] = val;
                        }
                    }
                }
            }
        }
        __syncthreads();  // s_w is rewritten by the next pass
    }
}

// items of a multi-step phase at level lev (per end)
static inline int cr_phase_half(int m, int lev) {
    const int M = (m + 1) / 2, p = M / 2;
    return ((std::max(p, M - 1 - p) >> (lev - 1)) + 1) / 2;
}

template <int PH>
static hh_status launch_cr_mm_t(hh_model* md, int lev, const float2* bcs, float2* x, float2* ends, const int* inst,
                                const int* slots, int nslots, const int* nslots_dev, int m, float c,
                                const int* active, const CoarseWork& cw) {
    hh_ctx* ctx = md->ctx;
    static unsigned attr_devices = 0;
    if (!(attr_devices & (1u << ctx->device))) {
        const size_t most = cmm_lds_bytes(CS_MAXM);
        if (most > 65536)
            HH_HIP(hipFuncSetAttribute((const void*)k_cr_mm<PH>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)most));
        attr_devices |= 1u << ctx->device;
    }
    const int M = (m + 1) / 2, Mo = m / 2;
    const int rows = PH <= 3 ? (PH == 2 ? M : Mo) : 2 * cr_phase_half(m, lev);
    if (rows == 0 || nslots == 0) return HH_OK;
    const int ntiles = (nslots + 15) / 16, cw_cols = 16 * cmm_waves<PH>(), ncg = (m + cw_cols - 1) / cw_cols;
    hipLaunchKernelGGL(k_cr_mm<PH>, dim3(ntiles * ncg * ((rows + 7) / 8) * 8), dim3(64 * cmm_waves<PH>()),
                       cmm_lds_bytes(m), ctx->stream,
                       bcs, x, cw.tw, cw.gw, cw.hw, ends, md->coarseQT.as<float2>(), md->coarseFL.as<float2>(), lev,
                       md->cr_depth, inst, slots, nslots, nslots_dev, m, c, active, rows, ntiles);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

static hh_status launch_cr_mm(hh_model* md, int PH, int lev, const float2* bcs, float2* x, float2* ends,
                              const int* inst, const int* slots, int nslots, const int* nslots_dev, int m, float c,
                              const int* active, const CoarseWork& cw) {
    switch (PH) {
        case 1: return launch_cr_mm_t<1>(md, lev, bcs, x, ends, inst, slots, nslots, nslots_dev, m, c, active, cw);
        case 2: return launch_cr_mm_t<2>(md, lev, bcs, x, ends, inst, slots, nslots, nslots_dev, m, c, active, cw);
        case 3: return launch_cr_mm_t<3>(md, lev, bcs, x, ends, inst, slots, nslots, nslots_dev, m, c, active, cw);
        case 4: return launch_cr_mm_t<4>(md, lev, bcs, x, ends, inst, slots, nslots, nslots_dev, m, c, active, cw);
        case 5: return launch_cr_mm_t<5>(md, lev, bcs, x, ends, inst, slots, nslots, nslots_dev, m, c, active, cw);
        case 6: return launch_cr_mm_t<6>(md, lev, bcs, x, ends, inst, slots, nslots, nslots_dev, m, c, active, cw);
        default: return launch_cr_mm_t<7>(md, lev, bcs, x, ends, inst, slots, nslots, nslots_dev, m, c, active, cw);
    }
}

// a multi-step phase (PH 4..7 at level lev; k_cr_pp, or k_cr_mm above one vector group)
static hh_status launch_cr_pp(hh_model* md, int PH, int lev, float2* x, float2* ends, const int* inst,
                              const int* slots, int nslots, const int* nslots_dev, int m, const int* active,
                              const CoarseWork& cw) {
    if (md->coarse_mm && nslots > CS_RMAX)
        return launch_cr_mm(md, PH, lev, nullptr, x, ends, inst, slots, nslots, nslots_dev, m, 0.f, active, cw);
    constexpr int RP = CS_RMAX;
    hh_ctx* ctx = md->ctx;
    static unsigned attr_devices = 0;
    if (!(attr_devices & (1u << ctx->device))) {
        size_t mostp = 0;
        for (int mm_ = 4; mm_ <= CS_MAXM; ++mm_) mostp = std::max(mostp, coarse_lds_bytes(RP, mm_));
        if (mostp > 65536) {
            const int want = (int)mostp;
            HH_HIP(hipFuncSetAttribute((const void*)k_cr_pp<RP, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, want));
            HH_HIP(hipFuncSetAttribute((const void*)k_cr_pp<RP, 5>, hipFuncAttributeMaxDynamicSharedMemorySize, want));
            HH_HIP(hipFuncSetAttribute((const void*)k_cr_pp<RP, 6>, hipFuncAttributeMaxDynamicSharedMemorySize, want));
            HH_HIP(hipFuncSetAttribute((const void*)k_cr_pp<RP, 7>, hipFuncAttributeMaxDynamicSharedMemorySize, want));
        }
        attr_devices |= 1u << ctx->device;
    }
    const int H = cr_phase_half(m, lev);
    if (H == 0 || nslots == 0) return HH_OK;
    const size_t ldsp = coarse_lds_bytes(RP, m);
    const dim3 grd((nslots + RP - 1) / RP, 2 * H);
    const float2* F = md->coarseQT.as<float2>();
    const float2* FL = md->coarseFL.as<float2>();
    const int D = md->cr_depth;
    hipStream_t st = ctx->stream;
    switch (PH) {
        case 4:
            hipLaunchKernelGGL((k_cr_pp<RP, 4>), grd, dim3(CS_NT), ldsp, st, cw.gw, cw.hw, x, ends, F, FL, lev, D, H,
                               inst, slots, nslots, nslots_dev, m, active);
            break;
        case 5:
            hipLaunchKernelGGL((k_cr_pp<RP, 5>), grd, dim3(CS_NT), ldsp, st, cw.gw, cw.hw, x, ends, F, FL, lev, D, H,
                               inst, slots, nslots, nslots_dev, m, active);
            break;
        case 6:
            hipLaunchKernelGGL((k_cr_pp<RP, 6>), grd, dim3(CS_NT), ldsp, st, cw.gw, cw.hw, x, ends, F, FL, lev, D, H,
                               inst, slots, nslots, nslots_dev, m, active);
            break;
        default:
            hipLaunchKernelGGL((k_cr_pp<RP, 7>), grd, dim3(CS_NT), ldsp, st, cw.gw, cw.hw, x, ends, F, FL, lev, D, H,
                               inst, slots, nslots, nslots_dev, m, active);
            break;
    }
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// the forward combines before the forward chains (levels 1 .. depth), the
// forward fills after them (depth .. 1); likewise backward around k_cr_bwd
static hh_status launch_cr_levels(hh_model* md, int PH, float2* x, float2* ends, const int* inst, const int* slots,
                                  int nslots, const int* nslots_dev, int m, const int* active, const CoarseWork& cw) {
    const int D = md->cr_depth;
    const bool up = PH == 4 || PH == 6;
    for (int k = 0; k < D; ++k)
        HH_TRY(launch_cr_pp(md, PH, up ? k + 1 : D - k, x, ends, inst, slots, nslots, nslots_dev, m, active, cw));
    return HH_OK;
}

template <int R>
static hh_status launch_cr_t(hh_model* md, const float2* bcs, float2* x, float2* ends, const int* inst,
                             const int* slots, int nslots, const int* nslots_dev, int m, float c, const int* active,
                             const CoarseWork& cw) {
    hh_ctx* ctx = md->ctx;
    static unsigned attr_devices = 0;
    const size_t lds = coarse_lds_bytes(R, m);
    if (!(attr_devices & (1u << ctx->device))) {
        size_t most = 0;
        for (int mm_ = 4; mm_ <= CS_MAXM; ++mm_) most = std::max(most, coarse_lds_bytes(R, mm_));
        if (most > 65536) {
            const int want = (int)most;
            HH_HIP(hipFuncSetAttribute((const void*)k_cr_fwd<R, false>, hipFuncAttributeMaxDynamicSharedMemorySize, want));
            HH_HIP(hipFuncSetAttribute((const void*)k_cr_bwd<R, false>, hipFuncAttributeMaxDynamicSharedMemorySize, want));
            if (R <= 4) {
                HH_HIP(hipFuncSetAttribute((const void*)k_cr_fwd<R, R <= 4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           want));
                HH_HIP(hipFuncSetAttribute((const void*)k_cr_bwd<R, R <= 4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           want));
            }
        }
        attr_devices |= 1u << ctx->device;
    }
    const int G = (nslots + R - 1) / R;
    const float2* F = md->coarseQT.as<float2>();
    hipStream_t st = ctx->stream;
    HH_TRY(launch_cr_par(md, 1, bcs, x, inst, slots, nslots, nslots_dev, m, c, active, cw));
    HH_TRY(launch_cr_par(md, 2, bcs, x, inst, slots, nslots, nslots_dev, m, c, active, cw));
    // prefetching chains where every thread's columns are whole chunk pairs
    // (the same test as CoarseMV::pf_ok()); not for R = 8, whose registers it would spill
    const int JP = CS_NT / m, jlen = (m + JP - 1) / JP, pch = R == 1 ? 8 : 4;
    const bool pf = R <= 4 && CS_NT % m == 0 && jlen % (2 * pch) == 0;
    const float2* FL = md->cr_depth > 0 ? md->coarseFL.as<float2>() : nullptr;
    const int D = md->cr_depth;
    HH_TRY(launch_cr_levels(md, 4, x, ends, inst, slots, nslots, nslots_dev, m, active, cw));
    if (pf)
        hipLaunchKernelGGL((k_cr_fwd<R, R <= 4>), dim3(G, 2), dim3(CS_NT), lds, st, cw.gw, cw.hw, x, ends, F, FL, D,
                           inst, slots, nslots, nslots_dev, m, active);
    else
        hipLaunchKernelGGL((k_cr_fwd<R, false>), dim3(G, 2), dim3(CS_NT), lds, st, cw.gw, cw.hw, x, ends, F, FL, D,
                           inst, slots, nslots, nslots_dev, m, active);
    HH_LAUNCH_CHECK();
    HH_TRY(launch_cr_levels(md, 5, x, ends, inst, slots, nslots, nslots_dev, m, active, cw));
    HH_TRY(launch_cr_levels(md, 6, x, ends, inst, slots, nslots, nslots_dev, m, active, cw));
    if (pf)
        hipLaunchKernelGGL((k_cr_bwd<R, R <= 4>), dim3(G, 2), dim3(CS_NT), lds, st, cw.gw, cw.hw, x, ends, F, FL, D,
                           inst, slots, nslots, nslots_dev, m, active);
    else
        hipLaunchKernelGGL((k_cr_bwd<R, false>), dim3(G, 2), dim3(CS_NT), lds, st, cw.gw, cw.hw, x, ends, F, FL, D,
                           inst, slots, nslots, nslots_dev, m, active);
    HH_LAUNCH_CHECK();
    HH_TRY(launch_cr_levels(md, 7, x, ends, inst, slots, nslots, nslots_dev, m, active, cw));
    return launch_cr_par(md, 3, bcs, x, inst, slots, nslots, nslots_dev, m, c, active, cw);
}

// the reduced solve with split chains (cooperative; offered when every
// workgroup can be resident and no other stream of the process may hold CUs)
template <int R, int RS>
static hh_status launch_cr_split_t(hh_model* md, const float2* bcs, float2* x, float2* ends, const int* inst,
                                   const int* slots, int nslots, const int* nslots_dev, int m, float c,
                                   const int* active, const CoarseWork& cw, bool* fits) {
    hh_ctx* ctx = md->ctx;
    *fits = false;
    if (ctx->concurrent) return HH_OK;
    static unsigned attr_devices = 0;
    const size_t lds = split_lds_bytes(R, m);
    if (split_lds_bytes(R, CS_MAXM) > 65536 && !(attr_devices & (1u << ctx->device))) {
        const int want = (int)split_lds_bytes(R, CS_MAXM);
        HH_HIP(hipFuncSetAttribute((const void*)k_cr_split_fwd<R, RS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   want));
        HH_HIP(hipFuncSetAttribute((const void*)k_cr_split_bwd<R, RS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   want));
        attr_devices |= 1u << ctx->device;
    }
    if ((m + CSP_NT / RS - 1) / (CSP_NT / RS) > CSP_CMAX) return HH_OK;  // column share exceeds the registers
    SplitGeom geo;
    geo.G = (nslots + R - 1) / R;
    geo.S = (m + RS - 1) / RS;
    geo.units = 2 * geo.G;
    geo.upx = (geo.units + 7) / 8;
    const int grid = 8 * geo.upx * geo.S;
    int per_cu_f = 0, per_cu_b = 0;
    HH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_f, (const void*)k_cr_split_fwd<R, RS>, CSP_NT, lds));
    HH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_b, (const void*)k_cr_split_bwd<R, RS>, CSP_NT, lds));
    if ((long long)std::min(per_cu_f, per_cu_b) * ctx->num_cus < grid) return HH_OK;  // not offered
    HH_TRY(launch_cr_par(md, 1, bcs, x, inst, slots, nslots, nslots_dev, m, c, active, cw));
    HH_TRY(launch_cr_par(md, 2, bcs, x, inst, slots, nslots, nslots_dev, m, c, active, cw));
    const float2* FL = md->cr_depth > 0 ? md->coarseFL.as<float2>() : nullptr;
    HH_TRY(launch_cr_levels(md, 4, x, ends, inst, slots, nslots, nslots_dev, m, active, cw));
    hipLaunchKernelGGL(k_zero_ints, dim3((2 * geo.units + 255) / 256), dim3(256), 0, ctx->stream, cw.cnt,
                       2 * geo.units);
    HH_LAUNCH_CHECK();
    const float2* a_gw = cw.gw;
    const float2* a_hw = cw.hw;
    float2* a_x = x;
    float2* a_ends = ends;
    const float2* a_F = md->coarseQT.as<float2>();
    const float2* a_FL = FL;
    int a_depth = md->cr_depth;
    const int* a_inst = inst;
    const int* a_slots = slots;
    int a_nslots = nslots;
    const int* a_nsd = nslots_dev;
    int a_m = m;
    const int* a_act = active;
    float2* a_xch = cw.xch;
    int* a_cnt = cw.cnt;
    int* a_err = md->coarse_err.as<int>();
    void* args[] = {&a_gw,    &a_hw,    &a_x,      &a_ends, &a_F, &a_FL, &a_depth, &a_inst, &a_slots,
                    &a_nslots, &a_nsd, &a_m, &a_act, &geo, &a_xch, &a_cnt, &a_err};
    const hipError_t le = hipLaunchCooperativeKernel((const void*)k_cr_split_fwd<R, RS>, dim3(grid), dim3(CSP_NT),
                                                     args, (unsigned)lds, ctx->stream);
    if (le == hipErrorCooperativeLaunchTooLarge) {  // the runtime's residency bound is tighter: not offered
        (void)hipGetLastError();
        return HH_OK;  // the phases launched so far are redone by the fallback
    }
    if (le != hipSuccess) {
        set_error("cooperative launch failed: %s", hipGetErrorString(le));
        return HH_ERR_HIP;
    }
    HH_TRY(launch_cr_levels(md, 5, x, ends, inst, slots, nslots, nslots_dev, m, active, cw));
    HH_TRY(launch_cr_levels(md, 6, x, ends, inst, slots, nslots, nslots_dev, m, active, cw));
    const float2* b_ends = ends;
    int* b_cnt = cw.cnt + geo.units;
    void* args_b[] = {&a_gw,    &a_hw,    &a_x,      &b_ends, &a_F, &a_FL, &a_depth, &a_inst, &a_slots,
                      &a_nslots, &a_nsd, &a_m, &a_act, &geo, &a_xch, &b_cnt, &a_err};
    HH_HIP(hipLaunchCooperativeKernel((const void*)k_cr_split_bwd<R, RS>, dim3(grid), dim3(CSP_NT), args_b,
                                      (unsigned)lds, ctx->stream));
    *fits = true;
    HH_TRY(launch_cr_levels(md, 7, x, ends, inst, slots, nslots, nslots_dev, m, active, cw));
    return launch_cr_par(md, 3, bcs, x, inst, slots, nslots, nslots_dev, m, c, active, cw);
}

// choice: R (1, 2, 4, 8) = chain with R right-hand sides per workgroup;
// 100 RS + R = split with RS rows per workgroup (RS = 8, 16, 32);
// 1000 + R = the reduced solve (models factorised with one level of cyclic reduction);
// 10000 + 100 RS + R = the reduced solve with split chains.
// The reduced chain codes (1001..1008) lie between the split codes with RS = 8
// (801..808) and those with RS = 16 (1601..1608).
static inline bool reduced_code(int c) { return (c > 1000 && c < 1100) || c > 10000; }
static inline bool cooperative_code(int c) { return (c >= 100 && c < 1000) || (c > 1100 && c < 10000) || c > 10000; }

static hh_status launch_coarse_choice(int choice, hh_model* md, const float2* bcs, float2* x, float2* ends,
                                      const int* inst, const int* slots, int nslots, const int* nslots_dev, int m,
                                      int p, float c, const int* active, const CoarseWork& cw, bool* fits) {
    *fits = true;
    if (choice > 10000) {
#define HH_CRSPLIT(RS_, R_)                                                                                \
    if (choice == 10000 + 100 * RS_ + R_)                                                                  \
        return launch_cr_split_t<R_, RS_>(md, bcs, x, ends, inst, slots, nslots, nslots_dev, m, c, active, cw, \
                                          fits);
        HH_CRSPLIT(8, 1) HH_CRSPLIT(8, 2) HH_CRSPLIT(8, 4) HH_CRSPLIT(8, 8)
        HH_CRSPLIT(16, 1) HH_CRSPLIT(16, 2) HH_CRSPLIT(16, 4) HH_CRSPLIT(16, 8)
        HH_CRSPLIT(32, 1) HH_CRSPLIT(32, 2) HH_CRSPLIT(32, 4) HH_CRSPLIT(32, 8)
#undef HH_CRSPLIT
        set_error("coarse-solve variant %d", choice);
        return HH_ERR_ARG;
    }
    if (reduced_code(choice)) {
        const float cc = c;
        switch (choice - 1000) {
            case 1: return launch_cr_t<1>(md, bcs, x, ends, inst, slots, nslots, nslots_dev, m, cc, active, cw);
            case 2: return launch_cr_t<2>(md, bcs, x, ends, inst, slots, nslots, nslots_dev, m, cc, active, cw);
            case 4: return launch_cr_t<4>(md, bcs, x, ends, inst, slots, nslots, nslots_dev, m, cc, active, cw);
            case 8: return launch_cr_t<8>(md, bcs, x, ends, inst, slots, nslots, nslots_dev, m, cc, active, cw);
            default: break;
        }
        set_error("coarse-solve variant %d", choice);
        return HH_ERR_ARG;
    }
    if (choice < 100)
        return launch_coarse(choice, md->ctx, bcs, x, ends, md->coarseQT.as<float2>(), inst, slots, nslots,
                             nslots_dev, m, p, c, active);
#define HH_SPLIT(RS_, R_)                                                                                  \
    if (choice == 100 * RS_ + R_)                                                                          \
        return launch_split_t<R_, RS_>(md, bcs, x, ends, inst, slots, nslots, nslots_dev, m, p, c, active, \
                                       cw, fits);
    HH_SPLIT(8, 1) HH_SPLIT(8, 2) HH_SPLIT(8, 4) HH_SPLIT(8, 8)
    HH_SPLIT(16, 1) HH_SPLIT(16, 2) HH_SPLIT(16, 4) HH_SPLIT(16, 8)
    HH_SPLIT(32, 1) HH_SPLIT(32, 2) HH_SPLIT(32, 4) HH_SPLIT(32, 8)
#undef HH_SPLIT
    set_error("coarse-solve variant %d", choice);
    return HH_ERR_ARG;
}

static bool valid_choice(int c) {
    if (c == 1 || c == 2 || c == 4 || c == 8) return true;
    if (c > 10000) c -= 10000;  // reduced split: the same RS / R pairs as the split
    else if (reduced_code(c)) return c == 1001 || c == 1002 || c == 1004 || c == 1008;
    const int rs = c / 100, r = c % 100;
    return (rs == 8 || rs == 16 || rs == 32) && (r == 1 || r == 2 || r == 4 || r == 8);
}

// the reduced solve's codes need the reduced factorisation, the others the plain one
bool coarse_choice_valid(const hh_model* md, int c) {
    return md->d.coarse_iters == 0 && valid_choice(c) && (reduced_code(c) == md->cr1);
}

// the split solve's timeout flag: reported (and cleared) after a solve
hh_status coarse_check_err(hh_model* md) {
    int e = 0;
    HH_HIP(hipMemcpyAsync(&e, md->coarse_err.ptr, sizeof(int), hipMemcpyDeviceToHost, md->ctx->stream));
    HH_HIP(hipStreamSynchronize(md->ctx->stream));
    if (e) {
        HH_HIP(hipMemsetAsync(md->coarse_err.ptr, 0, sizeof(int), md->ctx->stream));
        HH_HIP(hipStreamSynchronize(md->ctx->stream));
        set_error("coarse solve: a step wait of the split solve timed out (results invalid)");
        return HH_ERR_HIP;
    }
    return HH_OK;
}

// bucket of an active right-hand-side count: ceil(log2(n)), n >= 1
static int coarse_bucket(int n) {
    int b = 0;
    while ((1 << b) < n && b < HH_COARSE_BUCKETS - 1) ++b;
    return b;
}

// whether a V-cycle's coarse solve for nact active right-hand sides (of nrhs)
// is already decided (forced or tuned) and launches no cooperative kernel: then
// its launch sequence can be captured into a graph
bool coarse_capturable(const hh_model* md, int nrhs, int nact) {
    if (md->d.coarse_iters > 0) return true;
    const int na = nact > 0 ? std::min(nact, nrhs) : nrhs;
    const int c = md->coarse_R_forced > 0 ? md->coarse_R_forced : md->coarse_R[coarse_bucket(std::max(na, 1))];
    return c > 0 && !cooperative_code(c);
}

// Autotuner of the coarse solve: for each bucket of active right-hand sides,
// time every variant (chain with R right-hand sides per workgroup, split with
// RS rows per workgroup; fwd + bwd, second of two runs, HIP events on the
// context's stream) on the call's own data and keep the fastest.  The timed
// launches only write the solve's outputs, which the real launch then rewrites.
static hh_status coarse_pick(hh_model* md, int nact, const float2* bcs, float2* x, float2* ends, const int* slots,
                             int nslots, const int* nslots_dev, int m, int p, float c, const int* inst,
                             const int* active, const CoarseWork& cw, int* choice_out) {
    if (md->coarse_R_forced > 0) {
        *choice_out = md->coarse_R_forced;
        return HH_OK;
    }
    const int b = coarse_bucket(std::max(nact, 1));
    if (md->coarse_R[b] > 0) {
        *choice_out = md->coarse_R[b];
        return HH_OK;
    }
    std::vector<int> cand;
    for (int R = 1; R <= CS_RMAX; R *= 2) {
        if (R > 1 && R / 2 >= nact) break;  // groups larger than the work
        if (md->cr1) {
            cand.push_back(1000 + R);
            if (!md->ctx->concurrent)
                for (int rs = 8; rs <= 32; rs *= 2) cand.push_back(10000 + 100 * rs + R);
        } else {
            cand.push_back(R);
            if (!md->ctx->concurrent)
                for (int rs = 8; rs <= 32; rs *= 2) cand.push_back(100 * rs + R);
        }
    }
    hh_ctx* ctx = md->ctx;
    hipEvent_t e0, e1;
    HH_HIP(hipEventCreate(&e0));
    HH_HIP(hipEventCreate(&e1));
    int best = 1;
    float best_ms = 1e30f;
    hh_status st = HH_OK;
    for (int cidx = 0; cidx < (int)cand.size() && st == HH_OK; ++cidx) {
        float ms = 0.f;
        bool fits = true;
        for (int rep = 0; rep < 2 && st == HH_OK && fits; ++rep) {
            if (hipEventRecord(e0, ctx->stream) != hipSuccess) st = HH_ERR_HIP;
            if (st == HH_OK)
                st = launch_coarse_choice(cand[cidx], md, bcs, x, ends, inst, slots, nslots, nslots_dev, m, p, c,
                                          active, cw, &fits);
            if (st == HH_OK && (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = HH_ERR_HIP;
        }
        if (st == HH_OK && fits && ms < best_ms) {
            best_ms = ms;
            best = cand[cidx];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != HH_OK) {
        if (!hh_last_error()[0]) set_error("coarse-solve autotuning failed");
        return st;
    }
    md->coarse_R[b] = best;
    *choice_out = best;
    return HH_OK;
}

// ---------------------------------------------------------------------------
// Tile heights of the V-cycle's fused kernels, autotuned like the convolution
// tiles: for each (kernel, initial-guess mode, level size, batch) key, on its
// first launch outside graph capture, every height runs three times on the
// call's own data (HIP events, the faster of the last two counts; each run
// rewrites the same outputs)
// and the fastest is kept per device for the process.  Defaults: 8 coarse rows
// (4 with the network's guess, whose fourth LDS array halves them) for the down
// kernel, 16 fine rows (8 with the guess) for the up kernel.
// ---------------------------------------------------------------------------
struct VcDownArgs {
    const float2* b;
    size_t bstride;
    const double* sig;
    int sig_stride;
    const float2* x0;
    size_t x0stride;
    float2* x1out;
    float2* bc;
    const float2* coef;
    const int* inst;
    int n;
    float inv_h2, beta, wj;
    const int* active;
    const float2* x0h;
    const float* x0s;
    int nrhs;
};
struct VcUpArgs {
    const float2* b;
    size_t bstride;
    const double* sig;
    int sig_stride;
    const float2* x1;
    const float2* ec;
    float2* z;
    size_t zstride;
    const float2* coef;
    const int* inst;
    int n;
    float inv_h2, beta, wj;
    const int* active;
    const float2* x0h;
    const float* x0s;
    int nrhs;
};

// tile heights per kernel (0 down, 1 up) and mode; the first is the default
static int vc_heights(int kernel, int mode, int* h) {
    if (kernel == 0) {
        if (mode == 2) { h[0] = 4; h[1] = 2; h[2] = 8; return 3; }
        if (mode == 1) { h[0] = 8; h[1] = 4; return 2; }
        h[0] = 8; h[1] = 4; h[2] = 16; return 3;
    }
    if (mode == 2) { h[0] = 8; h[1] = 4; h[2] = 16; return 3; }
    h[0] = 16; h[1] = 8; h[2] = 32; return 3;
}

template <int X0M, int TCY>
static hh_status vc_down_t(hipStream_t st, const VcDownArgs& a) {
    const int nc = a.n / 2;
    dim3 grd((nc + DN_TCX - 1) / DN_TCX, (nc + TCY - 1) / TCY, a.nrhs);
    hipLaunchKernelGGL((k_vc_down<X0M, TCY>), grd, dim3(256), 0, st, a.b, a.bstride, a.sig, a.sig_stride, a.x0,
                       a.x0stride, a.x1out, a.bc, a.coef, a.inst, a.n, a.inv_h2, a.beta, a.wj, a.active, a.x0h,
                       a.x0s);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

static hh_status launch_vc_down(hipStream_t st, int mode, int tcy, const VcDownArgs& a) {
    if (mode == 2 && tcy == 4) return vc_down_t<2, 4>(st, a);
    if (mode == 2 && tcy == 2) return vc_down_t<2, 2>(st, a);
    if (mode == 2 && tcy == 8) return vc_down_t<2, 8>(st, a);
    if (mode == 1 && tcy == 8) return vc_down_t<1, 8>(st, a);
    if (mode == 1 && tcy == 4) return vc_down_t<1, 4>(st, a);
    if (mode == 0 && tcy == 8) return vc_down_t<0, 8>(st, a);
    if (mode == 0 && tcy == 4) return vc_down_t<0, 4>(st, a);
    if (mode == 0 && tcy == 16) return vc_down_t<0, 16>(st, a);
    set_error("no V-cycle down kernel for mode %d, %d rows", mode, tcy);
    return HH_ERR_ARG;
}

template <int X1M, int TY>
static hh_status vc_up_t(hipStream_t st, const VcUpArgs& a) {
    dim3 grd((a.n + UP_TX - 1) / UP_TX, (a.n + TY - 1) / TY, a.nrhs);
    hipLaunchKernelGGL((k_vc_up<X1M, TY>), grd, dim3(256), 0, st, a.b, a.bstride, a.sig, a.sig_stride, a.x1, a.ec,
                       a.z, a.zstride, a.coef, a.inst, a.n, a.inv_h2, a.beta, a.wj, a.active, a.x0h, a.x0s);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

static hh_status launch_vc_up(hipStream_t st, int mode, int ty, const VcUpArgs& a) {
    if (mode == 2 && ty == 8) return vc_up_t<2, 8>(st, a);
    if (mode == 2 && ty == 4) return vc_up_t<2, 4>(st, a);
    if (mode == 2 && ty == 16) return vc_up_t<2, 16>(st, a);
    if (mode == 1 && ty == 16) return vc_up_t<1, 16>(st, a);
    if (mode == 1 && ty == 8) return vc_up_t<1, 8>(st, a);
    if (mode == 1 && ty == 32) return vc_up_t<1, 32>(st, a);
    if (mode == 0 && ty == 16) return vc_up_t<0, 16>(st, a);
    if (mode == 0 && ty == 8) return vc_up_t<0, 8>(st, a);
    if (mode == 0 && ty == 32) return vc_up_t<0, 32>(st, a);
    set_error("no V-cycle up kernel for mode %d, %d rows", mode, ty);
    return HH_ERR_ARG;
}

namespace {
std::mutex g_vc_mu;
std::map<std::pair<int, uint64_t>, int> g_vc_tune;  // (device, key) -> height
int g_vc_forced[2][3] = {{0, 0, 0}, {0, 0, 0}};     // forced height per kernel and mode (0: autotune)
uint64_t vc_key(int kernel, int mode, int n, int nrhs) {
    return ((uint64_t)kernel << 60) | ((uint64_t)mode << 56) | ((uint64_t)n << 24) | (uint64_t)nrhs;
}
}  // namespace

template <class F>
static hh_status vc_tuned_launch(hipStream_t st, int kernel, int mode, int n, int nrhs, F launch) {
    int h[4];
    const int nh = vc_heights(kernel, mode, h);
    int dev = 0;
    HH_HIP(hipGetDevice(&dev));
    const uint64_t key = vc_key(kernel, mode, n, nrhs);
    {
        std::lock_guard<std::mutex> lk(g_vc_mu);
        if (g_vc_forced[kernel][mode] > 0) return launch(g_vc_forced[kernel][mode]);
        auto it = g_vc_tune.find({dev, key});
        if (it != g_vc_tune.end()) return launch(it->second);
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HH_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) return launch(h[0]);
    hipEvent_t e0, e1;
    HH_HIP(hipEventCreate(&e0));
    HH_HIP(hipEventCreate(&e1));
    int best = h[0];
    float best_ms = 1e30f;
    hh_status s = HH_OK;
    for (int v = 0; v < nh && s == HH_OK; ++v) {
        float ms = 0.f, ms_min = 1e30f;  // the faster of two timed runs after a warm-up run
        for (int rep = 0; rep < 3 && s == HH_OK; ++rep) {
            if (hipEventRecord(e0, st) != hipSuccess) s = HH_ERR_HIP;
            if (s == HH_OK) s = launch(h[v]);
            if (s == HH_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                               hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                s = HH_ERR_HIP;
            if (s == HH_OK && rep > 0) ms_min = std::min(ms_min, ms);
        }
        ms = ms_min;
        if (s == HH_OK && ms < best_ms) {
            best_ms = ms;
            best = h[v];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != HH_OK) {
        if (!hh_last_error()[0]) set_error("V-cycle tile autotuning failed");
        return s;
    }
    {
        std::lock_guard<std::mutex> lk(g_vc_mu);
        g_vc_tune[{dev, key}] = best;
    }
    return launch(best);
}

int vc_tuned_height(int device, int kernel, int mode, int n, int nrhs) {
    std::lock_guard<std::mutex> lk(g_vc_mu);
    auto it = g_vc_tune.find({device, vc_key(kernel, mode, n, nrhs)});
    return it == g_vc_tune.end() ? 0 : it->second;
}

hh_status vc_force_height(int kernel, int mode, int height) {
    if (kernel < 0 || kernel > 1 || mode < 0 || mode > 2) {
        set_error("kernel is 0 (down) or 1 (up), mode 0..2");
        return HH_ERR_ARG;
    }
    int h[4];
    const int nh = vc_heights(kernel, mode, h);
    bool ok = height == 0;
    for (int i = 0; i < nh; ++i) ok = ok || h[i] == height;
    if (!ok) {
        set_error("%d rows is not a tile height of this kernel and mode", height);
        return HH_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_vc_mu);
    g_vc_forced[kernel][mode] = height;
    return HH_OK;
}

hh_status launch_vcycle_strided(hh_model* md, int nrhs, const BatchMap& bm, const float2* b, size_t bstride,
                                const double* sig, int sig_stride, const float2* x0, size_t x0stride, float2* z,
                                size_t zstride, void* work, const int* active, const float2* x0h,
                                const float* x0s) {
    const int* inst_dev = bm.inst;
    hipStream_t st = md->ctx->stream;
    const float beta = (float)md->d.sl_beta, wj = (float)md->d.jacobi_w;
    const int L = md->nlev;
    float2* bl[HH_MAX_LEVELS] = {nullptr};
    float2* el[HH_MAX_LEVELS] = {nullptr};
    char* wp = (char*)work;
    for (int l = 1; l < L; ++l) {
        size_t sz = (size_t)nrhs * md->lev[l].n * md->lev[l].n * sizeof(float2);
        bl[l] = (float2*)wp;
        wp += sz;
        el[l] = (float2*)wp;
        wp += sz;
    }
    float2* ends = (float2*)wp;
    wp += 2 * (size_t)nrhs * md->lev[L - 1].n * sizeof(float2);
    float2* x1 = x0 ? (float2*)wp : nullptr;
    const CoarseWork cw = coarse_work(md, (char*)work + vcycle_float_bytes(md, nrhs, x0 != nullptr), nrhs);
    // down sweep
    for (int l = 0; l < L - 1; ++l) {
        const Level& lv = md->lev[l];
        const int nc = lv.n / 2;
        const size_t nl = (size_t)lv.n * lv.n;
        const float2* bin = (l == 0) ? b : bl[l];
        const size_t bs = (l == 0) ? bstride : nl;
        const double* sg = (l == 0) ? sig : nullptr;
        const float ih2 = (float)(1.0 / (lv.h * lv.h));
        ProfScope ps(md->ctx, l == 0 ? HH_K_VC_DOWN : HH_K_VC_MID);
        const int mode = (l == 0 && x0h) ? 2 : ((l == 0 && x0) ? 1 : 0);
        VcDownArgs da{bin, bs, sg, sig_stride, mode == 1 ? x0 : nullptr, mode == 1 ? x0stride : (size_t)0,
                      mode == 1 ? x1 : nullptr, bl[l + 1], lv.coef.as<float2>(), inst_dev, lv.n, ih2, beta, wj,
                      active, mode == 2 ? x0h : nullptr, mode == 2 ? x0s : nullptr, nrhs};
        HH_TRY(vc_tuned_launch(st, 0, mode, lv.n, nrhs, [&](int t) { return launch_vc_down(st, mode, t, da); }));
        (void)nc;
    }
    // coarsest exact solve
    {
        const Level& lc = md->lev[L - 1];
        ProfScope ps(md->ctx, HH_K_VC_COARSE);
        const int m = lc.n, p = m / 2;
        const float c = (float)(1.0 / (lc.h * lc.h));
        if (md->d.coarse_iters > 0) {
            char* gw = (char*)work + vcycle_float_bytes(md, nrhs, x0 != nullptr) + coarse_work_bytes(md, nrhs) + 256;
            gw = (char*)(((uintptr_t)gw + 255) & ~(uintptr_t)255);
            HH_TRY(launch_coarse_gmres(md, nrhs, inst_dev, bl[L - 1], el[L - 1], active, gw));
        } else {
            // every workgroup serves R right-hand sides of one slowness model: with
            // several models the host's grouping order (padded per model to
            // CS_RMAX); with one model the active right-hand sides, packed
            const int* slots = bm.order;
            int nslots = bm.order ? bm.nslots : nrhs;
            const int* nslots_dev = nullptr;
            if (!bm.order && active) {
                hipLaunchKernelGGL(k_coarse_compact, dim3(1), dim3(1024), 0, st, active, nrhs, cw.slots, cw.count);
                HH_LAUNCH_CHECK();
                slots = cw.slots;
                nslots_dev = cw.count;
                if (bm.nact > 0) nslots = std::min(nslots, bm.nact);
            }
            const int nact = bm.nact > 0 ? std::min(bm.nact, nrhs) : nrhs;
            int choice = 1;
            HH_TRY(coarse_pick(md, nact, bl[L - 1], el[L - 1], ends, slots, nslots, nslots_dev, m, p, c, inst_dev,
                               active, cw, &choice));
            bool fits = true;
            HH_TRY(launch_coarse_choice(choice, md, bl[L - 1], el[L - 1], ends, inst_dev, slots, nslots, nslots_dev, m,
                                        p, c, active, cw, &fits));
            if (!fits)  // a forced split variant that cannot be resident here: the chain
                HH_TRY(launch_coarse_choice(md->cr1 ? 1001 : 1, md, bl[L - 1], el[L - 1], ends, inst_dev, slots, nslots,
                                            nslots_dev, m, p, c, active, cw, &fits));
        }
    }
    // up sweep
    for (int l = L - 2; l >= 0; --l) {
        const Level& lv = md->lev[l];
        const size_t nl = (size_t)lv.n * lv.n;
        const float2* bin = (l == 0) ? b : bl[l];
        const size_t bs = (l == 0) ? bstride : nl;
        const double* sg = (l == 0) ? sig : nullptr;
        float2* out = (l == 0) ? z : el[l];
        const size_t os = (l == 0) ? zstride : nl;
        const float ih2 = (float)(1.0 / (lv.h * lv.h));
        ProfScope ps(md->ctx, l == 0 ? HH_K_VC_UP : HH_K_VC_MID);
        const int mode = (l == 0 && x0h) ? 2 : ((l == 0 && x0) ? 1 : 0);
        VcUpArgs ua{bin, bs, sg, sig_stride, mode == 1 ? x1 : nullptr, el[l + 1], out, os, lv.coef.as<float2>(),
                    inst_dev, lv.n, ih2, beta, wj, active, mode == 2 ? x0h : nullptr, mode == 2 ? x0s : nullptr,
                    nrhs};
        HH_TRY(vc_tuned_launch(st, 1, mode, lv.n, nrhs, [&](int t) { return launch_vc_up(st, mode, t, ua); }));
    }
    return HH_OK;
}

hh_status launch_vcycle(hh_model* md, int nrhs, const BatchMap& bm, const float2* b, const double* sig,
                        int sig_stride, const float2* x0, float2* z, void* work, const int* active) {
    const size_t nn = (size_t)md->lev[0].n * md->lev[0].n;
    return launch_vcycle_strided(md, nrhs, bm, b, nn, sig, sig_stride, x0, nn, z, nn, work, active);
}

}  // namespace hh
