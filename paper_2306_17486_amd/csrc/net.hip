// Encoder-solver network with the implicit coarsest layer (Sec. 4.1-4.4, Sec. 5.3):
// parameters, the encoder (once per slowness model), the Green's-function
// transforms of the implicit layer (eqs. 16-17), the forward pass and the
// CNN+MG preconditioner z = V(v; s Net(v / rms(v))).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include <atomic>

#include "net.h"

namespace hh {

// layer indices (same order as the flat parameter vector)
enum {
    L_ENC1_D = 0, L_ENC1_C1, L_ENC1_C2, L_ENC2_D, L_ENC2_C1, L_ENC2_C2, L_ENC3_D, L_ENC3_C1, L_ENC3_C2,
    L_S1_D, L_S1_C1, L_S1_C2, L_S2_D, L_S2_C1, L_S2_C2, L_S3_D, L_S3_C1, L_S3_C2, L_S4_D, L_S4_C1, L_S4_C2,
    L_U3_T, L_U3_C1, L_U3_C2, L_U2_T, L_U2_C1, L_U2_C2, L_U1_T, L_U1_C1, L_U1_C2, L_OUT
};

static void build_table(hh_net* net) {
    const int c1 = net->ch[0], c2 = net->ch[1], c3 = net->ch[2], c4 = net->ch[3];
    const int t[NET_LAYERS][3] = {
        {LK_DOWN, 2, c1},   {LK_CONV, c1, c1}, {LK_CONV, c1, c1},   // encoder level 1
        {LK_DOWN, c1, c2},  {LK_CONV, c2, c2}, {LK_CONV, c2, c2},   // encoder level 2
        {LK_DOWN, c2, c3},  {LK_CONV, c3, c3}, {LK_CONV, c3, c3},   // encoder level 3
        {LK_DOWN, 2, c1},   {LK_CONV, c1, c1}, {LK_CONV, c1, c1},   // solver level 1
        {LK_DOWN, c1, c2},  {LK_CONV, c2, c2}, {LK_CONV, c2, c2},   // solver level 2
        {LK_DOWN, c2, c3},  {LK_CONV, c3, c3}, {LK_CONV, c3, c3},   // solver level 3
        {LK_DOWN4, c3, c4}, {LK_CONV, c4, c4}, {LK_CONV, c4, c4},   // solver level 4
        {LK_UP4, c4, c3},   {LK_CONV, c3, c3}, {LK_CONV, c3, c3},   // up to level 3
        {LK_UP, c3, c2},    {LK_CONV, c2, c2}, {LK_CONV, c2, c2},   // up to level 2
        {LK_UP, c2, c1},    {LK_CONV, c1, c1}, {LK_CONV, c1, c1},   // up to level 1
        {LK_CONV, c1, 2}};                                          // projection to (re, im)
    size_t off = 0;
    for (int l = 0; l < NET_LAYERS; ++l) {
        LayerInfo& L = net->L[l];
        L.kind = t[l][0];
        L.cin = t[l][1];
        L.cout = t[l][2];
        L.woff = off;
        L.boff = off + (size_t)L.cin * L.cout * 9;
        off = L.boff + L.cout;
    }
    net->nk = c4 / 2;
    net->koff = off;
    net->nparams = off + (size_t)net->nk * 9 * 2;
}

// The lightweight network (Sec. 4.4, Sec. 5.3): the same encoder, down and up
// paths, with batch normalisation + softplus after every 3x3 convolution of a
// level (no bias there), and on the first three solver levels one inverted
// bottleneck in place of the two convolutions: 1x1 expansion by 6, depthwise
// 3x3, 1x1 shrink, each batch-normalised (softplus after the first two), the
// shrink's output added to the bottleneck's input.  Parameters per layer: the
// weights, then (batch-norm layers) scale, shift, running mean and running
// variance, or (the others) the biases.
enum {
    LL_ENC1_D = 0, LL_ENC1_C1, LL_ENC1_C2, LL_ENC2_D, LL_ENC2_C1, LL_ENC2_C2, LL_ENC3_D, LL_ENC3_C1, LL_ENC3_C2,
    LL_S1_D, LL_S1_E, LL_S1_W, LL_S1_S, LL_S2_D, LL_S2_E, LL_S2_W, LL_S2_S, LL_S3_D, LL_S3_E, LL_S3_W, LL_S3_S,
    LL_S4_D, LL_S4_C1, LL_S4_C2, LL_U3_T, LL_U3_C1, LL_U3_C2, LL_U2_T, LL_U2_C1, LL_U2_C2, LL_U1_T, LL_U1_C1,
    LL_U1_C2, LL_OUT
};
constexpr int LIGHT_EXPAND = 6;

static void build_light_table(hh_net* net) {
    const int c1 = net->ch[0], c2 = net->ch[1], c3 = net->ch[2], c4 = net->ch[3], t = LIGHT_EXPAND;
    const int tab[LIGHT_LAYERS][4] = {
        {LK_DOWN, 2, c1, 0},    {LK_CONV, c1, c1, 1},      {LK_CONV, c1, c1, 1},        // encoder level 1
        {LK_DOWN, c1, c2, 0},   {LK_CONV, c2, c2, 1},      {LK_CONV, c2, c2, 1},        // encoder level 2
        {LK_DOWN, c2, c3, 0},   {LK_CONV, c3, c3, 1},      {LK_CONV, c3, c3, 1},        // encoder level 3
        {LK_DOWN, 2, c1, 0},    {LK_PW, c1, t * c1, 1},    {LK_DW, t * c1, t * c1, 1},  // solver level 1
        {LK_PW, t * c1, c1, 1},
        {LK_DOWN, c1, c2, 0},   {LK_PW, c2, t * c2, 1},    {LK_DW, t * c2, t * c2, 1},  // solver level 2
        {LK_PW, t * c2, c2, 1},
        {LK_DOWN, c2, c3, 0},   {LK_PW, c3, t * c3, 1},    {LK_DW, t * c3, t * c3, 1},  // solver level 3
        {LK_PW, t * c3, c3, 1},
        {LK_DOWN4, c3, c4, 0},  {LK_CONV, c4, c4, 1},      {LK_CONV, c4, c4, 1},        // solver level 4
        {LK_UP4, c4, c3, 0},    {LK_CONV, c3, c3, 1},      {LK_CONV, c3, c3, 1},        // up to level 3
        {LK_UP, c3, c2, 0},     {LK_CONV, c2, c2, 1},      {LK_CONV, c2, c2, 1},        // up to level 2
        {LK_UP, c2, c1, 0},     {LK_CONV, c1, c1, 1},      {LK_CONV, c1, c1, 1},        // up to level 1
        {LK_CONV, c1, 2, 0}};                                                           // projection
    size_t off = 0;
    for (int l = 0; l < LIGHT_LAYERS; ++l) {
        LayerInfo& L = net->L[l];
        L.kind = tab[l][0];
        L.cin = tab[l][1];
        L.cout = tab[l][2];
        L.bn = tab[l][3];
        L.woff = off;
        off += L.kind == LK_PW ? (size_t)L.cin * L.cout
                               : (L.kind == LK_DW ? (size_t)L.cout * 9 : (size_t)L.cin * L.cout * 9);
        if (L.bn) {
            L.boff = (size_t)-1;
            L.goff = off;
            L.beoff = off + L.cout;
            L.rmoff = off + 2 * (size_t)L.cout;
            L.rvoff = off + 3 * (size_t)L.cout;
            off += 4 * (size_t)L.cout;
        } else {
            L.boff = off;
            off += L.cout;
        }
    }
    net->nlayers = LIGHT_LAYERS;
    net->nk = c4 / 2;
    net->koff = off;
    net->nparams = off + (size_t)net->nk * 9 * 2;
}

static inline int coarse_stride_of(int n) { return n >= 512 ? 2 : 1; }
static inline int coarsest_of(int n) { return n >= 512 ? n / 16 : n / 8; }

// map size of light layer l for fine size n
static int light_res(int l, int n) {
    if (l <= LL_ENC3_C2) return n >> (l / 3 + 1);
    if (l <= LL_S1_S || l >= LL_U1_T) return n / 2;
    if (l <= LL_S2_S || (l >= LL_U2_T && l <= LL_U2_C2)) return n / 4;
    if (l <= LL_S3_S || (l >= LL_U3_T && l <= LL_U3_C2)) return n / 8;
    return coarsest_of(n);
}
static inline int nextpow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

// sum |v|^2 partials (FP64) per right-hand side; grid (blocks, B)
__global__ void __launch_bounds__(256) k_sumsq(const float2* __restrict__ v, size_t vstride, size_t N,
                                               double* __restrict__ parts, const int* __restrict__ active) {
    __shared__ double s_red[4];
    const int b = blockIdx.y;
    double acc = 0.0;
    if (!active || active[b]) {
        const float2* vb = v + (size_t)b * vstride;
        for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256) {
            float2 z = vb[i];
            acc += (double)z.x * z.x + (double)z.y * z.y;
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) parts[(size_t)b * gridDim.x + blockIdx.x] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

// rms(v) -> input scale 1/rms, output scale h^2 sigma rms  (zero vector: both 0)
__global__ void k_scales(const double* __restrict__ parts, int nblk, size_t N, const double* __restrict__ sig,
                         int sig_stride, double h2, float* __restrict__ in_scale, float* __restrict__ out_scale,
                         int B) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double s = 0.0;
    for (int i = 0; i < nblk; ++i) s += parts[(size_t)b * nblk + i];
    const double rms = sqrt(s / (double)N);
    const double sg = sig ? sig[(size_t)b * sig_stride] : 1.0;
    in_scale[b] = rms > 0.0 ? (float)(1.0 / rms) : 0.f;
    out_scale[b] = rms > 0.0 ? (float)(h2 * sg * rms) : 0.f;
}

// the same scales from a known norm: the vectors are FGMRES's lazily normalised
// basis vectors, whose norm is 1/sig as the orthogonalisation measured it, so
// rms = 1/(sqrt(N) sig), in_scale = sqrt(N) sig and out_scale = h^2 / sqrt(N)
__global__ void k_scales_known(const double* __restrict__ sig, int sig_stride, size_t N, double h2,
                               float* __restrict__ in_scale, float* __restrict__ out_scale, int B) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double sg = sig[(size_t)b * sig_stride];
    const double rn = sqrt((double)N);
    in_scale[b] = sg > 0.0 ? (float)(rn * sg) : 0.f;
    out_scale[b] = sg > 0.0 ? (float)(h2 / rn) : 0.f;
}

// The network's input and output scales per sample (C9 reading of Sec. 4.3: the
// network works on a unit-rms residual): in_scale = 1/rms(v), out_scale =
// h^2 sig rms(v); with known_norm (sig given) from sig alone, without a pass over v.
static hh_status launch_scales(hipStream_t st, const float2* v, size_t vstride, size_t N, double* parts,
                               const int* active, const double* sig, int sig_stride, double h2, float* in_scale,
                               float* out_scale, int B, bool known_norm) {
    if (known_norm && sig) {
        hipLaunchKernelGGL(k_scales_known, dim3((B + 63) / 64), dim3(64), 0, st, sig, sig_stride, N, h2, in_scale,
                           out_scale, B);
        HH_LAUNCH_CHECK();
        return HH_OK;
    }
    const int nblk = 64;
    hipLaunchKernelGGL(k_sumsq, dim3(nblk, B), dim3(256), 0, st, v, vstride, N, parts, active);
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scales, dim3((B + 63) / 64), dim3(64), 0, st, parts, nblk, N, sig, sig_stride, h2, in_scale,
                       out_scale, B);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// First layer of the encoder / solver: 3x3 stride-2 convolution from 2 input
// channels (BF16-rounded) to 16 channels, + bias, + optional skip.  The input
// is either a complex vector scaled per RHS (solver: v / rms(v)) or the
// coefficient field (encoder: (omega h)^2 kappa^2 and (omega h)^2 kappa^2 gamma).
// A block computes CI_TY x CI_TX outputs from the (2 CI_TY + 1) x (2 CI_TX + 1)
// input patch staged once in LDS, on the matrix cores (v_mfma_f32_16x16x4f32,
// FP32 products and sums): out (16 channels x 16 pixels) = W (16 x 18, k = c * 9 + tap, padded
// to 20) x patch (18 x 16 pixels).  Lane l holds the weight W[l % 16][k] and the
// input value of k for pixel l % 16, with k = 4 q + l / 16 in k-step q, and
// receives channels 4 (l / 16) .. +3 of pixel l % 16.  Wave w computes output
// rows 2w and 2w + 1 of the 8 x 64 tile, 16 pixels per MFMA group.
constexpr int CI_TY = 8, CI_TX = 64;
typedef float cin_f4 __attribute__((ext_vector_type(4)));
template <int SRC>
__global__ void __launch_bounds__(256) k_conv_in_mfma(const float2* __restrict__ src, size_t src_bstride,
                                                      const float* __restrict__ in_scale,
                                                      const int* __restrict__ src_map, float h2,
                                                      const float* __restrict__ W, const float* __restrict__ bias,
                                                      const uint16_t* __restrict__ skip,
                                                      const int* __restrict__ skip_map, uint16_t* __restrict__ y,
                                                      int n, const int* __restrict__ active) {
    constexpr int COUT = 16;
    constexpr int PH = 2 * CI_TY + 1, PW = 2 * CI_TX + 1;
    static_assert(CI_TY == 8 && CI_TX == 64, "two output rows per wave, four 16-pixel groups per row");
    __shared__ float s_a[2][PH][PW + 1];
    const int b = blockIdx.z;
    if (active && !active[b]) return;
    const int m = n / 2;
    const int oy0 = blockIdx.y * CI_TY, ox0 = blockIdx.x * CI_TX;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int cl = lane & 15, kl = lane >> 4;
    // this lane's weights for the five k-steps (zero past k = 17) and biases
    float wa[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int k = 4 * q + kl;
        wa[q] = k < 18 ? W[(cl * 2 + k / 9) * 9 + k % 9] : 0.f;
    }
    float bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bv[i] = bias[4 * kl + i];
    const float2* sb = src + (size_t)(src_map ? src_map[b] : b) * src_bstride;
    const float sc = (SRC == 0) ? in_scale[b] : 1.f;
    // the patch: every load of this thread issued before the first store, so
    // that they are in flight together
    constexpr int NST = (PH * PW + 255) / 256;
    float2 pv[NST];
#pragma unroll
    for (int j = 0; j < NST; ++j) {
        const int e = tid + j * 256;
        const int py = e / PW, px = e - py * PW;
        const int iy = 2 * oy0 - 1 + py, ix = 2 * ox0 - 1 + px;
        pv[j] = (e < PH * PW && iy >= 0 && iy < n && ix >= 0 && ix < n) ? sb[iy * n + ix] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int j = 0; j < NST; ++j) {
        const int e = tid + j * 256;
        if (e >= PH * PW) break;
        const int py = e / PW, px = e - py * PW;
        const int iy = 2 * oy0 - 1 + py, ix = 2 * ox0 - 1 + px;
        float a0 = 0.f, a1 = 0.f;
        if (iy >= 0 && iy < n && ix >= 0 && ix < n) {  // zero padding stays zero whatever the scale
            if (SRC == 0) {
                a0 = pv[j].x * sc;
                a1 = pv[j].y * sc;
            } else {
                a0 = pv[j].x * h2;
                a1 = a0 * pv[j].y;
            }
        }
        s_a[0][py][px] = bf2f(f2bf(a0));
        s_a[1][py][px] = bf2f(f2bf(a1));
    }
    __syncthreads();
    const uint16_t* skb = skip ? skip + (size_t)(skip_map ? skip_map[b] : b) * m * m * COUT : nullptr;
#pragma unroll
    for (int g = 0; g < 8; ++g) {
        const int ly = 2 * wave + (g >> 2), lx = (g & 3) * 16 + cl;
        cin_f4 acc = (cin_f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const int k = 4 * q + kl;
            float bval = 0.f;
            if (k < 18) {
                const int c = k / 9, t = k % 9;
                bval = s_a[c][2 * ly + t / 3][2 * lx + t % 3];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[q], bval, acc, 0, 0, 0);
        }
        const int oy = oy0 + ly, ox = ox0 + lx;
        if (oy >= m || ox >= m) continue;
        const size_t pix = (size_t)oy * m + ox;
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = acc[i] + bv[i];
        if (skb) {
            const uint2 s2 = *reinterpret_cast<const uint2*>(skb + pix * COUT + 4 * kl);
            v[0] += bf2f((uint16_t)(s2.x & 0xffff));
            v[1] += bf2f((uint16_t)(s2.x >> 16));
            v[2] += bf2f((uint16_t)(s2.y & 0xffff));
            v[3] += bf2f((uint16_t)(s2.y >> 16));
        }
        uint2 o2;
        o2.x = f2bf2(v[0], v[1]);
        o2.y = f2bf2(v[2], v[3]);
        *reinterpret_cast<uint2*>(y + ((size_t)b * m * m + pix) * COUT + 4 * kl) = o2;
    }
}

static inline dim3 conv_in_grid(int n, int B) {
    const int m = n / 2;
    return dim3((m + CI_TX - 1) / CI_TX, (m + CI_TY - 1) / CI_TY, B);
}

// x0 = out_scale * P(o): bilinear prolongation (the multigrid's, eq. 8) of the
// half-resolution (re, im) output to the fine grid, as a complex vector.
__global__ void __launch_bounds__(256) k_prolong_x0(const float2* __restrict__ o, const float* __restrict__ out_scale,
                                                    float2* __restrict__ x0, int n, const int* __restrict__ active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n * n) return;
    const int i = p / n, j = p - i * n;
    const int m = n / 2;
    const float2* ob = o + (size_t)b * m * m;
    auto at = [&](int I, int J) -> float2 {
        return (I < m && J < m) ? ob[(size_t)I * m + J] : make_float2(0.f, 0.f);
    };
    const int I = i >> 1, J = j >> 1;
    float2 v;
    if (!(i & 1) && !(j & 1)) {
        v = at(I, J);
    } else if (!(i & 1)) {
        v = cscale(cadd(at(I, J), at(I, J + 1)), 0.5f);
    } else if (!(j & 1)) {
        v = cscale(cadd(at(I, J), at(I + 1, J)), 0.5f);
    } else {
        v = cscale(cadd(cadd(at(I, J), at(I, J + 1)), cadd(at(I + 1, J), at(I + 1, J + 1))), 0.25f);
    }
    x0[(size_t)b * n * n + p] = cscale(v, out_scale[b]);
}

// ---------------------------------------------------------------------------
// Implicit layer (eq. 16): per (RHS, complex channel c = channels 2c, 2c+1),
// y = crop(IFFT(Ghat_c * FFT(zero-pad(x)))) on an M x M grid, M = 2 nc.  The
// whole transform stays in LDS: radix-2 decimation in frequency forward (rows
// holding data, then all columns) leaves the spectrum in bit-reversed order,
// where it is multiplied by Ghat (stored bit-reversed, scaled by 1/M^2);
// decimation in time inverse (all columns, then the kept rows) returns natural
// order.  No permutation pass is needed.
// ---------------------------------------------------------------------------
// Radix-2 butterfly sweeps over nvec vectors of length M in LDS (vector v at
// s[v * vstride + k * estride]), two consecutive stages fused per pass where
// two remain (radix 2^2: the same butterflies in the same order, held in
// registers between the stages, so one barrier instead of two).  Threads run
// along the elements (rows) or across the vectors (vfast: columns, so that
// neighbouring threads touch neighbouring LDS words).
template <int M, int NT>
__device__ __forceinline__ void impl_dif_sweep(float2* s, int nvec, int vstride, int estride, bool vfast,
                                               const float2* tw) {
    int len = M;
    while (len >= 4) {  // stages len and len / 2 together
        const int half = len >> 1, q = len >> 2, twa = M / len, twb = 2 * twa;
        for (int t = threadIdx.x; t < nvec * (M / 4); t += NT) {
            const int v = vfast ? t % nvec : t / (M / 4), g = vfast ? t / nvec : t % (M / 4);
            const int blk = g / q, j = g - blk * q;
            const int e0 = v * vstride + (blk * len + j) * estride, e1 = e0 + q * estride;
            const int e2 = e0 + half * estride, e3 = e2 + q * estride;
            const float2 a0 = s[e0], a1 = s[e1], a2 = s[e2], a3 = s[e3];
            const float2 b0 = cadd(a0, a2), b2 = cmul(csub(a0, a2), tw[j * twa]);
            const float2 b1 = cadd(a1, a3), b3 = cmul(csub(a1, a3), tw[(j + q) * twa]);
            s[e0] = cadd(b0, b1);
            s[e1] = cmul(csub(b0, b1), tw[j * twb]);
            s[e2] = cadd(b2, b3);
            s[e3] = cmul(csub(b2, b3), tw[j * twb]);
        }
        __syncthreads();
        len >>= 2;
    }
    if (len == 2) {  // one stage left
        for (int t = threadIdx.x; t < nvec * (M / 2); t += NT) {
            const int v = vfast ? t % nvec : t / (M / 2), g = vfast ? t / nvec : t % (M / 2);
            const int e0 = v * vstride + (2 * g) * estride, e1 = e0 + estride;
            const float2 a = s[e0], bb = s[e1];
            s[e0] = cadd(a, bb);
            s[e1] = cmul(csub(a, bb), tw[0]);
        }
        __syncthreads();
    }
}

template <int M, int NT>
__device__ __forceinline__ void impl_dit_sweep(float2* s, int nvec, int vstride, int estride, bool vfast,
                                               const float2* tw) {
    int len = 2;
    while (2 * len <= M) {  // stages len and 2 len together
        const int hl = len >> 1, twa = M / len, twb = M / (2 * len);
        for (int t = threadIdx.x; t < nvec * (M / 4); t += NT) {
            const int v = vfast ? t % nvec : t / (M / 4), g = vfast ? t / nvec : t % (M / 4);
            const int blk = g / hl, j = g - blk * hl;
            const int e0 = v * vstride + (blk * 2 * len + j) * estride, e1 = e0 + hl * estride;
            const int e2 = e0 + len * estride, e3 = e2 + hl * estride;
            float2 wa = tw[j * twa];
            wa.y = -wa.y;
            const float2 a0 = s[e0], a1 = cmul(s[e1], wa), a2 = s[e2], a3 = cmul(s[e3], wa);
            const float2 c0 = cadd(a0, a1), c1 = csub(a0, a1), c2 = cadd(a2, a3), c3 = csub(a2, a3);
            float2 w0 = tw[j * twb], w1 = tw[(j + hl) * twb];
            w0.y = -w0.y;
            w1.y = -w1.y;
            const float2 d2 = cmul(c2, w0), d3 = cmul(c3, w1);
            s[e0] = cadd(c0, d2);
            s[e2] = csub(c0, d2);
            s[e1] = cadd(c1, d3);
            s[e3] = csub(c1, d3);
        }
        __syncthreads();
        len <<= 2;
    }
    if (len == M) {  // one stage left
        const int hl = M >> 1;
        for (int t = threadIdx.x; t < nvec * (M / 2); t += NT) {
            const int v = vfast ? t % nvec : t / (M / 2), j = vfast ? t / nvec : t % (M / 2);
            const int e0 = v * vstride + j * estride, e1 = e0 + hl * estride;
            float2 w = tw[j];
            w.y = -w.y;
            const float2 a = s[e0], bb = cmul(s[e1], w);
            s[e0] = cadd(a, bb);
            s[e1] = csub(a, bb);
        }
        __syncthreads();
    }
}

template <int M, int NT>
__global__ void __launch_bounds__(NT) k_implicit(const uint16_t* __restrict__ xin, uint16_t* __restrict__ yout,
                                                 const float2* __restrict__ Gbr, int nc, int nk, int conjG,
                                                 const uint16_t* __restrict__ mask, const int* __restrict__ active) {
    extern __shared__ float2 s_dyn[];
    constexpr int P = M + 1;
    float2* s = s_dyn;
    float2* tw = s_dyn + M * P;
    const int c = blockIdx.x, b = blockIdx.y;
    if (active && !active[b]) return;
    const int tid = threadIdx.x;
    const int CH = 2 * nk;
    for (int t = tid; t < M / 2; t += NT) {
        float sn, cs;
        sincospif(-2.0f * (float)t / (float)M, &sn, &cs);
        tw[t] = make_float2(cs, sn);
    }
    // the input map (nc <= M / 2) and this thread's share of Ghat_c: every load
    // issued before the first is used, Ghat's in flight during the forward sweeps
    constexpr int NI = (M / 2 * (M / 2) + NT - 1) / NT, NG = (M * M + NT - 1) / NT;
    uint32_t raw[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = tid + i * NT;
        const int y = e / nc, x = e - y * nc;
        raw[i] = e < nc * nc ? *reinterpret_cast<const uint32_t*>(xin + (((size_t)b * nc + y) * nc + x) * CH + 2 * c)
                             : 0u;
    }
    float2 g[NG];
    {
        const float2* G = Gbr + (size_t)c * M * M;
#pragma unroll
        for (int i = 0; i < NG; ++i) {
            const int e = tid + i * NT;
            g[i] = e < M * M ? G[e] : make_float2(0.f, 0.f);
        }
    }
    for (int e = tid; e < M * P; e += NT) s[e] = make_float2(0.f, 0.f);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = tid + i * NT;
        const int y = e / nc, x = e - y * nc;
        if (e < nc * nc) s[y * P + x] = make_float2(bf2f((uint16_t)(raw[i] & 0xffff)), bf2f((uint16_t)(raw[i] >> 16)));
    }
    __syncthreads();
    // forward DIF along the nc data rows, then all columns (bit-reversed spectrum)
    impl_dif_sweep<M, NT>(s, nc, P, 1, false, tw);
    impl_dif_sweep<M, NT>(s, M, 1, P, true, tw);
    // spectrum (bit-reversed both ways) times Ghat_c
#pragma unroll
    for (int i = 0; i < NG; ++i) {
        const int e = tid + i * NT;
        if (e >= M * M) break;
        float2 gv = g[i];
        if (conjG) gv.y = -gv.y;
        const int r = e / M, col = e - r * M;
        s[r * P + col] = cmul(s[r * P + col], gv);
    }
    __syncthreads();
    // inverse DIT along all columns, then the nc kept rows (natural order)
    impl_dit_sweep<M, NT>(s, M, 1, P, true, tw);
    impl_dit_sweep<M, NT>(s, nc, P, 1, false, tw);
    for (int e = tid; e < nc * nc; e += NT) {
        const int y = e / nc, x = e - y * nc;
        float2 v = s[y * P + x];
        const size_t o = (((size_t)b * nc + y) * nc + x) * CH + 2 * c;
        if (mask) {
            const uint32_t mr = *reinterpret_cast<const uint32_t*>(mask + o);
            if (!(bf2f((uint16_t)(mr & 0xffff)) > 0.f)) v.x = 0.f;
            if (!(bf2f((uint16_t)(mr >> 16)) > 0.f)) v.y = 0.f;
        }
        *reinterpret_cast<uint32_t*>(yout + o) = f2bf2(v.x, v.y);
    }
}

static size_t implicit_lds_bytes(int M) { return ((size_t)M * (M + 1) + M / 2) * sizeof(float2); }

// ---------------------------------------------------------------------------
// Implicit layer for transforms too large for LDS (M = 256, 512: coarsest maps
// of 128^2 and 256^2).  The same transform in three passes through a scratch
// array W [B][nk][nc][M] in HBM: (1) forward DIF along the nc data rows,
// (2) per column: forward DIF along the column, the product with Ghat_c,
// inverse DIT along the column, keeping the nc rows the output needs,
// (3) inverse DIT along those rows, keeping nc columns.  Forward only.
// ---------------------------------------------------------------------------
constexpr int IMPL_RPB = 4;  // rows per workgroup in passes 1 and 3
constexpr int IMPL_CPB = 8;  // columns per workgroup in pass 2

template <int M>
__device__ __forceinline__ void impl_twiddles(float2* tw) {
    for (int t = threadIdx.x; t < M / 2; t += blockDim.x) {
        float sn, cs;
        sincospif(-2.0f * (float)t / (float)M, &sn, &cs);
        tw[t] = make_float2(cs, sn);
    }
}

// forward DIF on `cnt` vectors of length M, vector v at s[v * vstride + k * estride]
template <int M>
__device__ __forceinline__ void impl_dif(float2* s, int cnt, int vstride, int estride, const float2* tw) {
    for (int len = M; len >= 2; len >>= 1) {
        const int half = len >> 1, tws = M / len;
        for (int t = threadIdx.x; t < cnt * (M / 2); t += blockDim.x) {
            const int v = t / (M / 2), bf = t - v * (M / 2);
            const int blk = bf / half, j = bf - blk * half;
            const int i0 = v * vstride + (blk * len + j) * estride, i1 = i0 + half * estride;
            const float2 a = s[i0], bb = s[i1];
            s[i0] = cadd(a, bb);
            s[i1] = cmul(csub(a, bb), tw[j * tws]);
        }
        __syncthreads();
    }
}

// inverse DIT (conjugate twiddles, no scaling) on `cnt` vectors of length M
template <int M>
__device__ __forceinline__ void impl_dit_inv(float2* s, int cnt, int vstride, int estride, const float2* tw) {
    for (int len = 2; len <= M; len <<= 1) {
        const int half = len >> 1, tws = M / len;
        for (int t = threadIdx.x; t < cnt * (M / 2); t += blockDim.x) {
            const int v = t / (M / 2), bf = t - v * (M / 2);
            const int blk = bf / half, j = bf - blk * half;
            const int i0 = v * vstride + (blk * len + j) * estride, i1 = i0 + half * estride;
            float2 w = tw[j * tws];
            w.y = -w.y;
            const float2 a = s[i0], bb = cmul(s[i1], w);
            s[i0] = cadd(a, bb);
            s[i1] = csub(a, bb);
        }
        __syncthreads();
    }
}

template <int M>
__global__ void __launch_bounds__(256) k_implicit_rows_fwd(const uint16_t* __restrict__ xin, float2* __restrict__ W,
                                                           int nc, int nk, const int* __restrict__ active) {
    __shared__ float2 s[IMPL_RPB * M];
    __shared__ float2 tw[M / 2];
    const int c = blockIdx.y, b = blockIdx.z, r0 = blockIdx.x * IMPL_RPB;
    if (active && !active[b]) return;
    const int CH = 2 * nk;
    const int rows = min(IMPL_RPB, nc - r0);
    impl_twiddles<M>(tw);
    for (int e = threadIdx.x; e < IMPL_RPB * M; e += blockDim.x) {
        const int v = e / M, x = e - v * M;
        float2 val = make_float2(0.f, 0.f);
        if (v < rows && x < nc) {
            const uint32_t raw =
                *reinterpret_cast<const uint32_t*>(xin + (((size_t)b * nc + r0 + v) * nc + x) * CH + 2 * c);
            val = make_float2(bf2f((uint16_t)(raw & 0xffff)), bf2f((uint16_t)(raw >> 16)));
        }
        s[e] = val;
    }
    __syncthreads();
    impl_dif<M>(s, rows, M, 1, tw);
    float2* Wr = W + (((size_t)b * nk + c) * nc + r0) * M;
    for (int e = threadIdx.x; e < rows * M; e += blockDim.x) Wr[e] = s[e];
}

template <int M>
__global__ void __launch_bounds__(256) k_implicit_cols(float2* __restrict__ W, const float2* __restrict__ Gbr, int nc,
                                                       int nk, const int* __restrict__ active) {
    constexpr int P = M + 1;
    __shared__ float2 s[IMPL_CPB * P];
    __shared__ float2 tw[M / 2];
    const int c = blockIdx.y, b = blockIdx.z, k0 = blockIdx.x * IMPL_CPB;
    if (active && !active[b]) return;
    impl_twiddles<M>(tw);
    float2* Wc = W + ((size_t)b * nk + c) * nc * M;
    // column cl of the tile at s[cl * P + row]; rows >= nc are zero
    for (int e = threadIdx.x; e < IMPL_CPB * M; e += blockDim.x) {
        const int row = e / IMPL_CPB, cl = e - row * IMPL_CPB;
        s[cl * P + row] = row < nc ? Wc[(size_t)row * M + k0 + cl] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    impl_dif<M>(s, IMPL_CPB, P, 1, tw);
    const float2* G = Gbr + (size_t)c * M * M;
    for (int e = threadIdx.x; e < IMPL_CPB * M; e += blockDim.x) {
        const int r = e / IMPL_CPB, cl = e - r * IMPL_CPB;
        s[cl * P + r] = cmul(s[cl * P + r], G[(size_t)r * M + k0 + cl]);
    }
    __syncthreads();
    impl_dit_inv<M>(s, IMPL_CPB, P, 1, tw);
    for (int e = threadIdx.x; e < IMPL_CPB * nc; e += blockDim.x) {
        const int row = e / IMPL_CPB, cl = e - row * IMPL_CPB;
        Wc[(size_t)row * M + k0 + cl] = s[cl * P + row];
    }
}

template <int M>
__global__ void __launch_bounds__(256) k_implicit_rows_inv(const float2* __restrict__ W, uint16_t* __restrict__ yout,
                                                           int nc, int nk, const int* __restrict__ active) {
    __shared__ float2 s[IMPL_RPB * M];
    __shared__ float2 tw[M / 2];
    const int c = blockIdx.y, b = blockIdx.z, r0 = blockIdx.x * IMPL_RPB;
    if (active && !active[b]) return;
    const int CH = 2 * nk;
    const int rows = min(IMPL_RPB, nc - r0);
    impl_twiddles<M>(tw);
    const float2* Wr = W + (((size_t)b * nk + c) * nc + r0) * M;
    for (int e = threadIdx.x; e < IMPL_RPB * M; e += blockDim.x) s[e] = e < rows * M ? Wr[e] : make_float2(0.f, 0.f);
    __syncthreads();
    impl_dit_inv<M>(s, rows, M, 1, tw);
    for (int e = threadIdx.x; e < rows * nc; e += blockDim.x) {
        const int v = e / nc, x = e - v * nc;
        const float2 val = s[v * M + x];
        *reinterpret_cast<uint32_t*>(yout + (((size_t)b * nc + r0 + v) * nc + x) * CH + 2 * c) =
            f2bf2(val.x, val.y);
    }
}

template <int M>
static hh_status launch_implicit_large_t(hipStream_t st, const uint16_t* x, uint16_t* y, const float2* Gbr, int nc,
                                         int nk, int B, float2* work, const int* active) {
    const dim3 gr((nc + IMPL_RPB - 1) / IMPL_RPB, nk, B), gc(M / IMPL_CPB, nk, B);
    hipLaunchKernelGGL(k_implicit_rows_fwd<M>, gr, dim3(256), 0, st, x, work, nc, nk, active);
    hipLaunchKernelGGL(k_implicit_cols<M>, gc, dim3(256), 0, st, work, Gbr, nc, nk, active);
    hipLaunchKernelGGL(k_implicit_rows_inv<M>, gr, dim3(256), 0, st, work, y, nc, nk, active);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// scratch of the large-transform path (0 when the transform fits LDS)
size_t implicit_work_bytes(int M, int nc, int nk, int B) {
    return M > 128 ? (size_t)B * nk * nc * M * sizeof(float2) : 0;
}

hh_status launch_implicit(hipStream_t st, int M, const uint16_t* x, uint16_t* y, const float2* Gbr, int nc, int nk,
                          int B, bool conjG, const int* active, const uint16_t* mask = nullptr,
                          float2* work = nullptr) {
    if (M == 256 || M == 512) {
        if (conjG || mask || !work) {
            set_error("implicit layer: transforms of %d points run forward only (no adjoint, needs scratch)", M);
            return HH_ERR_ARG;
        }
        return M == 256 ? launch_implicit_large_t<256>(st, x, y, Gbr, nc, nk, B, work, active)
                        : launch_implicit_large_t<512>(st, x, y, Gbr, nc, nk, B, work, active);
    }
    const size_t lds = implicit_lds_bytes(M);
    if (2 * nc > M) {  // the in-LDS kernel stages at most (M/2)^2 input points per map
        set_error("implicit layer: map %d x %d does not fit a transform of %d points", nc, nc, M);
        return HH_ERR_ARG;
    }
    dim3 grd(nk, B);
#define HH_IMP(MM, NTT)                                                                                  \
    if (M == MM) {                                                                                       \
        static bool attr_set = false;                                                                    \
        if (!attr_set) {                                                                                 \
            HH_HIP(hipFuncSetAttribute((const void*)k_implicit<MM, NTT>,                                 \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));           \
            attr_set = true;                                                                             \
        }                                                                                                \
        hipLaunchKernelGGL((k_implicit<MM, NTT>), grd, dim3(NTT), lds, st, x, y, Gbr, nc, nk, conjG ? 1 : 0, \
                           mask, active);                                                                \
        HH_LAUNCH_CHECK();                                                                               \
        return HH_OK;                                                                                    \
    }
    HH_IMP(16, 256)
    HH_IMP(32, 256)
    HH_IMP(64, 512)
    HH_IMP(128, 1024)
#undef HH_IMP
    set_error("implicit layer: transform size %d not supported (coarsest map must be at most 256 x 256)", M);
    return HH_ERR_ARG;
}

// ---------------------------------------------------------------------------
// Explicit coarsest layer (the explicit U-Net of Sec. 5.2): each complex channel
// c (real channels 2c, 2c+1) is convolved with its 3x3 kernel K_c instead of
// being mapped through K_c's Green's function:
//   y[i][j] = sum_{a,e} K_c[a][e] z[i - a + 1][j - e + 1]   (zero outside the map)
// ADJ: the adjoint, gz[i][j] = sum_{a,e} conj(K_c[a][e]) gy[i + a - 1][j + e - 1],
// zeroed where mask <= 0 (the ReLU derivative of the layer below).  One thread
// per pixel and complex channel; BF16 NHWC in and out, FP32 arithmetic.
// ---------------------------------------------------------------------------
template <bool ADJ>
__global__ void __launch_bounds__(256) k_explicit(const uint16_t* __restrict__ x, uint16_t* __restrict__ y,
                                                  const float* __restrict__ K, int m, int nk,
                                                  const uint16_t* __restrict__ mask, const int* __restrict__ active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= m * m * nk) return;
    const int c = t % nk, pix = t / nk;
    const int i = pix / m, j = pix - i * m;
    const int C2 = 2 * nk;
    const uint16_t* xb = x + (size_t)b * m * m * C2;
    float yr = 0.f, yi = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const int si = ADJ ? i + a - 1 : i - a + 1, sj = ADJ ? j + e - 1 : j - e + 1;
            if (si < 0 || si >= m || sj < 0 || sj >= m) continue;
            const uint32_t v = *reinterpret_cast<const uint32_t*>(xb + ((size_t)si * m + sj) * C2 + 2 * c);
            const float zr = bf2f((uint16_t)(v & 0xffff)), zi = bf2f((uint16_t)(v >> 16));
            const float kr = K[(c * 9 + a * 3 + e) * 2], ki = ADJ ? -K[(c * 9 + a * 3 + e) * 2 + 1]
                                                                  : K[(c * 9 + a * 3 + e) * 2 + 1];
            yr += kr * zr - ki * zi;
            yi += kr * zi + ki * zr;
        }
    const size_t po = ((size_t)b * m * m + pix) * C2 + 2 * c;
    if (mask) {
        const uint32_t mv = *reinterpret_cast<const uint32_t*>(mask + po);
        if (!(bf2f((uint16_t)(mv & 0xffff)) > 0.f)) yr = 0.f;
        if (!(bf2f((uint16_t)(mv >> 16)) > 0.f)) yi = 0.f;
    }
    *reinterpret_cast<uint32_t*>(y + po) = f2bf2(yr, yi);
}

// Kernel gradient of the explicit layer, per block of EK_PIX pixels of one
// sample: part[b][blk][c * 9 + tap] = sum over the block's pixels p of
// conj(z[p - d_tap]) gy[p] (FP64), d_tap = (a - 1, e - 1).  One thread per
// (channel, tap) pair.
constexpr int EK_PIX = 256;
__global__ void __launch_bounds__(320) k_explicit_kgrad(const uint16_t* __restrict__ z, const uint16_t* __restrict__ gy,
                                                        int m, int nk, double2* __restrict__ part) {
    const int b = blockIdx.y, blk = blockIdx.x;
    const int t = threadIdx.x;
    const int nblk = gridDim.x;
    if (t >= nk * 9) return;
    const int c = t / 9, tap = t - 9 * c, a = tap / 3, e = tap - 3 * a;
    const int C2 = 2 * nk;
    const uint16_t* zb = z + (size_t)b * m * m * C2;
    const uint16_t* gb = gy + (size_t)b * m * m * C2;
    double sr = 0.0, si = 0.0;
    const int p0 = blk * EK_PIX, p1 = min(p0 + EK_PIX, m * m);
    for (int p = p0; p < p1; ++p) {
        const int i = p / m, j = p - i * m;
        const int zi_ = i - a + 1, zj_ = j - e + 1;
        if (zi_ < 0 || zi_ >= m || zj_ < 0 || zj_ >= m) continue;
        const uint32_t zv = *reinterpret_cast<const uint32_t*>(zb + ((size_t)zi_ * m + zj_) * C2 + 2 * c);
        const uint32_t gv = *reinterpret_cast<const uint32_t*>(gb + (size_t)p * C2 + 2 * c);
        const double zr = bf2f((uint16_t)(zv & 0xffff)), zim = bf2f((uint16_t)(zv >> 16));
        const double gr = bf2f((uint16_t)(gv & 0xffff)), gim = bf2f((uint16_t)(gv >> 16));
        // conj(z) * gy
        sr += zr * gr + zim * gim;
        si += zr * gim - zim * gr;
    }
    part[((size_t)b * nblk + blk) * (nk * 9) + t] = make_double2(sr, si);
}

// gK[c][tap] = sum of the partials (fixed order), stored as (d/dRe, d/dIm) floats
__global__ void k_explicit_kgrad_reduce(const double2* __restrict__ part, int nrows, int count,
                                        float* __restrict__ gK) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    double sr = 0.0, si = 0.0;
    for (int r = 0; r < nrows; ++r) {
        const double2 v = part[(size_t)r * count + t];
        sr += v.x;
        si += v.y;
    }
    gK[2 * t] = (float)sr;
    gK[2 * t + 1] = (float)si;
}

hh_status launch_explicit(hipStream_t st, const uint16_t* x, uint16_t* y, const float* K, int m, int nk, int B,
                          bool adjoint, const int* active, const uint16_t* mask) {
    const dim3 grd((m * m * nk + 255) / 256, B);
    if (adjoint)
        hipLaunchKernelGGL(k_explicit<true>, grd, dim3(256), 0, st, x, y, K, m, nk, mask, active);
    else
        hipLaunchKernelGGL(k_explicit<false>, grd, dim3(256), 0, st, x, y, K, m, nk, mask, active);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// ---------------------------------------------------------------------------
// Green's function of the implicit kernels (eq. 17), FP64.
//   S[c][p][q] = conj(K^)/(|K^|^2 + eps) * F(delta)[p][q],  F(delta) = (-1)^(p+q)
//   G = IFFT_N(S) on the crop [N/2 - nc, N/2 + nc)^2 only, Ghat = FFT_M(ifftshift(G))
// evaluated as separable DFTs restricted to the needed rows/columns.
// ---------------------------------------------------------------------------
__global__ void k_green_S(const float* __restrict__ K, double2* __restrict__ S, int N, double eps) {
    const int c = blockIdx.y;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= N * N) return;
    const int p = idx / N, q = idx - p * N;
    double re = 0.0, im = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int bb = 0; bb < 3; ++bb) {
            const double kr = K[((size_t)c * 9 + a * 3 + bb) * 2], ki = K[((size_t)c * 9 + a * 3 + bb) * 2 + 1];
            long t = ((long)p * (a - 1) + (long)q * (bb - 1)) % N;
            if (t < 0) t += N;
            double sn, cs;
            sincospi(-2.0 * (double)t / (double)N, &sn, &cs);
            re += kr * cs - ki * sn;
            im += kr * sn + ki * cs;
        }
    const double den = re * re + im * im + eps;
    const double sign = ((p + q) & 1) ? -1.0 : 1.0;
    S[(size_t)c * N * N + idx] = make_double2(sign * re / den, -sign * im / den);
}

// out[b][r][k] = scale * sum_i in[b][r][i] exp(sign 2 pi i (i + oin)(k + oout) / N)   (axis = 1)
// out[b][k][r] = scale * sum_i in[b][i][r] exp(...)                                   (axis = 0)
__global__ void __launch_bounds__(256) k_dft_pass(const double2* __restrict__ in, double2* __restrict__ out, int R,
                                                  int Lin, int Lout, int N, int oin, int oout, int sign,
                                                  double scale, int axis) {
    __shared__ double2 s_tw[2048];
    for (int t = threadIdx.x; t < N; t += 256) {
        double sn, cs;
        sincospi(2.0 * sign * (double)t / (double)N, &sn, &cs);
        s_tw[t] = make_double2(cs, sn);
    }
    __syncthreads();
    const int b = blockIdx.y;
    const int o = blockIdx.x * 256 + threadIdx.x;
    if (o >= R * Lout) return;
    int r, k;
    if (axis == 1) {
        r = o / Lout;
        k = o - r * Lout;
    } else {
        k = o / R;
        r = o - k * R;
    }
    // N is a power of two: indices mod N by masking; the twiddle index
    // (i + oin)(k + oout) mod N advances by kk per step
    const int msk = N - 1;
    const int kk = (k + oout) & msk;
    int tix = (int)(((long)(oin & msk) * kk) & msk);
    double re = 0.0, im = 0.0;
    for (int i = 0; i < Lin; ++i, tix = (tix + kk) & msk) {
        const double2 w = s_tw[tix];
        const double2 v = (axis == 1) ? in[((size_t)b * R + r) * Lin + i] : in[((size_t)b * Lin + i) * R + r];
        re += v.x * w.x - v.y * w.y;
        im += v.x * w.y + v.y * w.x;
    }
    const double2 res = make_double2(re * scale, im * scale);
    if (axis == 1)
        out[((size_t)b * R + r) * Lout + k] = res;
    else
        out[((size_t)b * Lout + k) * R + r] = res;
}

__device__ __forceinline__ int bitrev(int x, int bits) { return (int)(__brev((unsigned)x) >> (32 - bits)); }

// Gbr[c][r][col] = Ghat[c][br(r)][br(col)] / M^2 (single precision)
__global__ void k_green_store(const double2* __restrict__ Gh, float2* __restrict__ Gbr, int M, int bits) {
    const int c = blockIdx.y;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= M * M) return;
    const int r = e / M, col = e - r * M;
    const double2 v = Gh[(size_t)c * M * M + (size_t)bitrev(r, bits) * M + bitrev(col, bits)];
    const double sc = 1.0 / ((double)M * M);
    Gbr[(size_t)c * M * M + e] = make_float2((float)(v.x * sc), (float)(v.y * sc));
}

static hh_status dft_pass(hipStream_t st, const double2* in, double2* out, int nb, int R, int Lin, int Lout, int N,
                          int oin, int oout, int sign, double scale, int axis) {
    if (N > 2048 || (N & (N - 1))) {
        set_error("Green's function grid %d: a power of two up to 2048", N);
        return HH_ERR_ARG;
    }
    dim3 grd((R * Lout + 255) / 256, nb);
    hipLaunchKernelGGL(k_dft_pass, grd, dim3(256), 0, st, in, out, R, Lin, Lout, N, oin, oout, sign, scale, axis);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// Ghat of every implicit kernel for the coarsest size nc into Gbr [nk][M][M]
hh_status green_forward(hh_net* net, int nc, float2* Gbr, double eps) {
    hipStream_t st = net->ctx->stream;
    const int M = 2 * nc, N = nextpow2(3 * M), nk = net->nk;
    Buf S, T, G, H;
    HH_TRY(S.ensure(net->ctx, (size_t)nk * N * N * sizeof(double2)));
    HH_TRY(T.ensure(net->ctx, (size_t)nk * N * M * sizeof(double2)));
    HH_TRY(G.ensure(net->ctx, (size_t)nk * M * M * sizeof(double2)));
    HH_TRY(H.ensure(net->ctx, (size_t)nk * M * M * sizeof(double2)));
    const float* K = net->params.as<float>() + net->koff;
    hipLaunchKernelGGL(k_green_S, dim3((N * N + 255) / 256, nk), dim3(256), 0, st, K, S.as<double2>(), N, eps);
    HH_LAUNCH_CHECK();
    // G[g1][g2] = (1/N^2) sum_{p,q} S[p][q] exp(+2 pi i (p y + q x)/N), y = N/2 - nc + g1, x = N/2 - nc + g2
    HH_TRY(dft_pass(st, S.as<double2>(), T.as<double2>(), nk, N, N, M, N, 0, N / 2 - nc, +1, 1.0, 1));
    HH_TRY(dft_pass(st, T.as<double2>(), G.as<double2>(), nk, M, N, M, N, 0, N / 2 - nc, +1,
                    1.0 / ((double)N * N), 0));
    // Ghat[k1][k2] = sum_{g1,g2} G[g1][g2] exp(-2 pi i (k1 (g1 - nc) + k2 (g2 - nc))/M)
    HH_TRY(dft_pass(st, G.as<double2>(), H.as<double2>(), nk, M, M, M, M, -nc, 0, -1, 1.0, 1));
    HH_TRY(dft_pass(st, H.as<double2>(), G.as<double2>(), nk, M, M, M, M, -nc, 0, -1, 1.0, 0));
    int bits = 0;
    while ((1 << bits) < M) ++bits;
    hipLaunchKernelGGL(k_green_store, dim3((M * M + 255) / 256, nk), dim3(256), 0, st, G.as<double2>(), Gbr, M, bits);
    HH_LAUNCH_CHECK();
    HH_HIP(hipStreamSynchronize(st));  // scratch buffers are released on return
    return HH_OK;
}

// ---------------------------------------------------------------------------
// parameters / packing
// ---------------------------------------------------------------------------
// the lightweight network: BN folded into `folded` (inference); BF16 packs of
// every 3x3 and pointwise layer in training (unfolded), input-gradient and
// (batch-norm layers) folded inference forms
static hh_status light_pack(hh_net* net) {
    hipStream_t st = net->ctx->stream;
    const float* P = net->params.as<float>();
    HH_TRY(net->folded.ensure(net->ctx, net->nparams * sizeof(float)));
    float* F = net->folded.as<float>();
    HH_HIP(hipMemcpyAsync(F, P, net->nparams * sizeof(float), hipMemcpyDeviceToDevice, st));
    size_t off = 0;
    for (int l = 0; l < LIGHT_LAYERS; ++l) {
        const LayerInfo& L = net->L[l];
        net->pk_fwd[l] = net->pk_bwd[l] = net->pk_inf[l] = (size_t)-1;
        if (L.bn) {
            const int per = L.kind == LK_PW ? L.cin : (L.kind == LK_DW ? 9 : L.cin * 9);
            HH_TRY(bn_fold(st, P + L.woff, P + L.goff, P + L.beoff, P + L.rmoff, P + L.rvoff, L.cout, per,
                           F + L.woff, F + L.beoff));
        }
        if (L.kind == LK_PW) {
            const size_t e = (size_t)L.cin * L.cout;
            net->pk_fwd[l] = off;
            net->pk_bwd[l] = off + e;
            net->pk_inf[l] = off + 2 * e;
            off += 3 * e;
        } else if (L.kind != LK_DW && L.cin >= 16 && L.cout >= 16) {
            net->pk_fwd[l] = off;
            off += packed_weight_elems(L.cin, L.cout);
            net->pk_bwd[l] = off;
            off += packed_weight_elems(L.cout, L.cin);
            if (L.bn) {
                net->pk_inf[l] = off;
                off += packed_weight_elems(L.cin, L.cout);
            }
        }
        off = (off + 7) & ~(size_t)7;  // 16-byte aligned blocks
    }
    net->pk_proj_hi = off;
    off += packed_weight_elems(16, 16);
    net->pk_proj_lo = off;
    off += packed_weight_elems(16, 16);
    HH_TRY(net->packed.ensure(net->ctx, off * sizeof(uint16_t) + 256));
    uint16_t* pk = net->packed.as<uint16_t>();
    for (int l = 0; l < LIGHT_LAYERS; ++l) {
        const LayerInfo& L = net->L[l];
        if (L.kind == LK_PW) {
            HH_TRY(pack_pointwise(st, P + L.woff, pk + net->pk_fwd[l], L.cout, L.cin, false));
            HH_TRY(pack_pointwise(st, P + L.woff, pk + net->pk_bwd[l], L.cout, L.cin, true));
            HH_TRY(pack_pointwise(st, F + L.woff, pk + net->pk_inf[l], L.cout, L.cin, false));
        } else if (net->pk_fwd[l] != (size_t)-1) {
            const bool up = L.kind == LK_UP || L.kind == LK_UP4;
            HH_TRY(pack_weights(st, P + L.woff, pk + net->pk_fwd[l], L.cin, L.cout, up));
            HH_TRY(pack_weights(st, P + L.woff, pk + net->pk_bwd[l], L.cout, L.cin, !up));
            if (L.bn) HH_TRY(pack_weights(st, F + L.woff, pk + net->pk_inf[l], L.cin, L.cout, up));
        }
    }
    HH_TRY(pack_weights_split(st, P + net->L[LL_OUT].woff, pk + net->pk_proj_hi, pk + net->pk_proj_lo, 16, 2, 16));
    net->packed_valid = true;
    return HH_OK;
}

hh_status net_pack(hh_net* net) {
    if (net->packed_valid) return HH_OK;
    if (net->light) return light_pack(net);
    hipStream_t st = net->ctx->stream;
    size_t off = 0;
    for (int l = 0; l < NET_LAYERS; ++l) {
        const LayerInfo& L = net->L[l];
        net->pk_fwd[l] = net->pk_bwd[l] = (size_t)-1;
        if (L.cin >= 16 && L.cout >= 16) {
            net->pk_fwd[l] = off;
            off += packed_weight_elems(L.cin, L.cout);
            net->pk_bwd[l] = off;
            off += packed_weight_elems(L.cout, L.cin);
        }
    }
    // the projection layer: 16 -> 2 padded to 16 output channels, high and low BF16 parts
    net->pk_proj_hi = off;
    off += packed_weight_elems(16, 16);
    net->pk_proj_lo = off;
    off += packed_weight_elems(16, 16);
    HH_TRY(net->packed.ensure(net->ctx, off * sizeof(uint16_t) + 256));
    const float* P = net->params.as<float>();
    uint16_t* pk = net->packed.as<uint16_t>();
    for (int l = 0; l < NET_LAYERS; ++l) {
        const LayerInfo& L = net->L[l];
        if (net->pk_fwd[l] == (size_t)-1) continue;
        const bool up = L.kind == LK_UP || L.kind == LK_UP4;
        // forward: convolutions direct; transposed convolutions flipped (T2 / S1 over zero-interleaved input)
        HH_TRY(pack_weights(st, P + L.woff, pk + net->pk_fwd[l], L.cin, L.cout, up));
        // input gradient: convolutions -> flipped (cin' = cout); transposed -> direct as a convolution
        HH_TRY(pack_weights(st, P + L.woff, pk + net->pk_bwd[l], L.cout, L.cin, !up));
    }
    HH_TRY(pack_weights_split(st, P + net->L[L_OUT].woff, pk + net->pk_proj_hi, pk + net->pk_proj_lo, 16, 2, 16));
    net->packed_valid = true;
    return HH_OK;
}

// activations of one forward pass on a batch
struct NetActs {
    int B = 0, n = 0;
    Buf a[NET_LAYERS];  // output of every layer (BF16 NHWC); a[L_OUT] holds the FP32 (re, im) projection
    Buf imp;            // implicit-layer output
    Buf impw;           // implicit-layer scratch for transforms larger than LDS
    Buf parts, scales;  // rms partials, in/out scales
    Buf zeros;          // skip map of one slowness model shared by the batch
    hh_status ensure(hh_net* net, int B_, int n_) {
        if (B_ <= B && n_ == n) return HH_OK;
        B = std::max(B_, B);
        n = n_;
        const int s4 = coarse_stride_of(n), ncs = coarsest_of(n);
        for (int l = L_S1_D; l <= L_OUT; ++l) {
            const LayerInfo& L = net->L[l];
            int m;
            if (l <= L_S1_C2 || (l >= L_U1_T && l <= L_U1_C2) || l == L_OUT) m = n / 2;
            else if (l <= L_S2_C2 || (l >= L_U2_T && l <= L_U2_C2)) m = n / 4;
            else if (l <= L_S3_C2 || (l >= L_U3_T && l <= L_U3_C2)) m = n / 8;
            else m = ncs;
            (void)s4;
            const size_t esz = (l == L_OUT) ? sizeof(float) : sizeof(uint16_t);
            HH_TRY(a[l].ensure(net->ctx, (size_t)B * m * m * L.cout * esz));
        }
        HH_TRY(imp.ensure(net->ctx, (size_t)B * ncs * ncs * net->ch[3] * sizeof(uint16_t)));
        if (implicit_work_bytes(2 * ncs, ncs, net->nk, B) > 0)
            HH_TRY(impw.ensure(net->ctx, implicit_work_bytes(2 * ncs, ncs, net->nk, B)));
        HH_TRY(parts.ensure(net->ctx, (size_t)B * 64 * sizeof(double)));
        HH_TRY(scales.ensure(net->ctx, (size_t)2 * B * sizeof(float)));
        HH_TRY(zeros.ensure(net->ctx, (size_t)B * sizeof(int)));
        HH_HIP(hipMemsetAsync(zeros.ptr, 0, (size_t)B * sizeof(int), net->ctx->stream));
        return HH_OK;
    }
    // elements of one sample in a[l] (BF16 maps; floats for the projection)
    size_t sample_elems(const hh_net* net, int l) const {
        int m;
        if (l <= L_S1_C2 || (l >= L_U1_T && l <= L_U1_C2) || l == L_OUT) m = n / 2;
        else if (l <= L_S2_C2 || (l >= L_U2_T && l <= L_U2_C2)) m = n / 4;
        else if (l <= L_S3_C2 || (l >= L_U3_T && l <= L_U3_C2)) m = n / 8;
        else m = coarsest_of(n);
        return (size_t)m * m * net->L[l].cout;
    }
};

// activations of the lightweight network: encoder layers (EB batch entries,
// one per slowness model) and solver layers (B right-hand sides); in training
// also the pre-normalisation outputs and batch statistics of the batch-norm layers
struct LightActs {
    int B = 0, n = 0, EB = 0, En = 0;
    bool train = false, etrain = false;
    Buf a[LIGHT_LAYERS];     // layer outputs (BF16 NHWC); a[LL_OUT]: FP32 (re, im) at n/2
    Buf z[LIGHT_LAYERS];     // training: pre-normalisation outputs
    Buf stat;                // training: float4 (mean, sd, scale, shift) per channel of every batch-norm layer
    size_t stat_off[LIGHT_LAYERS] = {0};
    Buf imp, impw, parts, scales, zeros, bnpart;
    hh_status ensure_stat(hh_net* net) {
        size_t off = 0;
        for (int l = 0; l < LIGHT_LAYERS; ++l) {
            stat_off[l] = off;
            if (net->L[l].bn) off += net->L[l].cout;
        }
        return stat.ensure(net->ctx, off * sizeof(float4));
    }
    hh_status ensure_layers(hh_net* net, int l0, int l1, int Bn, int nn, bool tr) {
        for (int l = l0; l <= l1; ++l) {
            // the expanded tensors of the bottlenecks exist in HBM only in training
            const LayerInfo& L = net->L[l];
            if (!tr && (L.kind == LK_DW || (L.kind == LK_PW && L.cout > L.cin))) continue;
            const int m = light_res(l, nn);
            const size_t px = (size_t)Bn * m * m;
            const size_t esz = (l == LL_OUT) ? sizeof(float) : sizeof(uint16_t);
            HH_TRY(a[l].ensure(net->ctx, px * net->L[l].cout * esz));
            if (tr && net->L[l].bn) HH_TRY(z[l].ensure(net->ctx, px * net->L[l].cout * sizeof(uint16_t)));
        }
        return HH_OK;
    }
    hh_status ensure_enc(hh_net* net, int EB_, int n_, bool tr) {
        if (EB_ <= EB && n_ == En && (!tr || etrain)) return HH_OK;
        EB = std::max(EB_, EB);
        En = n_;
        etrain = etrain || tr;
        HH_TRY(ensure_stat(net));
        return ensure_layers(net, LL_ENC1_D, LL_ENC3_C2, EB, En, etrain);
    }
    hh_status ensure(hh_net* net, int B_, int n_, bool tr) {
        if (B_ <= B && n_ == n && (!tr || train)) return HH_OK;
        B = std::max(B_, B);
        n = n_;
        train = train || tr;
        HH_TRY(ensure_stat(net));
        HH_TRY(ensure_layers(net, LL_S1_D, LL_OUT, B, n, train));
        const int ncs = coarsest_of(n);
        HH_TRY(imp.ensure(net->ctx, (size_t)B * ncs * ncs * net->ch[3] * sizeof(uint16_t)));
        if (implicit_work_bytes(2 * ncs, ncs, net->nk, B) > 0)
            HH_TRY(impw.ensure(net->ctx, implicit_work_bytes(2 * ncs, ncs, net->nk, B)));
        HH_TRY(parts.ensure(net->ctx, (size_t)B * 64 * sizeof(double)));
        HH_TRY(scales.ensure(net->ctx, (size_t)2 * B * sizeof(float)));
        HH_TRY(zeros.ensure(net->ctx, (size_t)B * sizeof(int)));
        HH_HIP(hipMemsetAsync(zeros.ptr, 0, (size_t)B * sizeof(int), net->ctx->stream));
        return HH_OK;
    }
    uint16_t* out(int l) const { return a[l].as<uint16_t>(); }
    float4* st(int l) const { return stat.as<float4>() + stat_off[l]; }
};

// ---------------------------------------------------------------------------
// per-model network state: encodings and Ghat
// ---------------------------------------------------------------------------
struct NetCache {
    hh_net* net = nullptr;
    unsigned long long uid = 0;      // the network the cache was built for (0: none)
    unsigned long long version = 0;
    int n = 0, nc = 0, M = 0;
    Buf enc[9];    // BF16 outputs of the 9 encoder layers per instance (E1, E2, E3 = enc[2], enc[5], enc[8])
    Buf Gbr;       // bit-reversed, scaled Ghat [nk][M][M]
    NetActs acts;  // forward activations of the solves on this model
    LightActs lacts;  // the same for the lightweight network (encoder outputs in lacts.a[0..8])
};

void net_model_release(hh_model* m) {
    delete reinterpret_cast<NetCache*>(m->netcache);
    m->netcache = nullptr;
}

static hh_status conv_layer(hh_net* net, int l, int mode, const uint16_t* x, int B, int Hin, int Win, uint16_t* y,
                            int Hout, int Wout, const uint16_t* skip, const int* skip_map, bool relu,
                            const int* active, float* yf = nullptr) {
    const LayerInfo& L = net->L[l];
    ConvArgs a{};
    a.x = x;
    a.y = y;
    a.yf = yf;
    a.wp = net->packed.as<uint16_t>() + net->pk_fwd[l];
    a.bias = net->params.as<float>() + L.boff;
    a.skip = skip;
    a.skip_map = skip_map;
    a.mask = nullptr;
    a.act = relu ? ACT_RELU : ACT_NONE;
    a.B = B;
    a.Hin = Hin;
    a.Win = Win;
    a.Hout = Hout;
    a.Wout = Wout;
    a.active = active;
    return launch_conv(net->ctx->stream, net->ctx->num_cus, L.cin, L.cout, mode, a);
}

// Encoder (Sec. 5.3): three levels of (strided conv, conv+ReLU, conv+ReLU) on
// the dimensionless mass term of every slowness model of the model; every layer
// output is kept (the training pass needs them).
hh_status encoder_forward(hh_net* net, hh_model* md, Buf* enc) {
    hipStream_t st = net->ctx->stream;
    const int n = md->lev[0].n, B = md->ninst;
    const double h = md->lev[0].h;
    for (int l = 0; l < 9; ++l) {
        const int lev = l / 3 + 1;
        HH_TRY(enc[l].ensure(net->ctx, (size_t)B * (n >> lev) * (n >> lev) * net->L[l].cout * sizeof(uint16_t)));
    }
    auto E = [&](int l) { return enc[l].as<uint16_t>(); };
    const float* P = net->params.as<float>();
    const int m1 = n / 2;
    hipLaunchKernelGGL((k_conv_in_mfma<1>), conv_in_grid(n, B), dim3(256), 0, st,
                       md->lev[0].coef.as<float2>(), (size_t)n * n, nullptr, nullptr, (float)(h * h),
                       P + net->L[L_ENC1_D].woff, P + net->L[L_ENC1_D].boff, nullptr, nullptr, E(L_ENC1_D), n,
                       nullptr);
    HH_LAUNCH_CHECK();
    HH_TRY(conv_layer(net, L_ENC1_C1, CM_S1, E(L_ENC1_D), B, m1, m1, E(L_ENC1_C1), m1, m1, nullptr, nullptr, true, nullptr));
    HH_TRY(conv_layer(net, L_ENC1_C2, CM_S1, E(L_ENC1_C1), B, m1, m1, E(L_ENC1_C2), m1, m1, nullptr, nullptr, true, nullptr));
    for (int k = 0; k < 2; ++k) {
        const int mi = n >> (k + 1), mo = mi / 2;
        const int l = (k == 0) ? L_ENC2_D : L_ENC3_D;
        HH_TRY(conv_layer(net, l, CM_S2, E(l - 1), B, mi, mi, E(l), mo, mo, nullptr, nullptr, false, nullptr));
        HH_TRY(conv_layer(net, l + 1, CM_S1, E(l), B, mo, mo, E(l + 1), mo, mo, nullptr, nullptr, true, nullptr));
        HH_TRY(conv_layer(net, l + 2, CM_S1, E(l + 1), B, mo, mo, E(l + 2), mo, mo, nullptr, nullptr, true, nullptr));
    }
    return HH_OK;
}

// ---------------------------------------------------------------------------
// lightweight network, forward (inference: batch norm folded into the weights;
// training: batch statistics over the batch, running averages updated when
// `update`)
// ---------------------------------------------------------------------------
// batch-norm + activation of layer l from its pre-normalisation output A.z[l]
static hh_status light_bn(hh_net* net, LightActs& A, int l, size_t npix, int act, const uint16_t* res, bool update) {
    const LayerInfo& L = net->L[l];
    float* P = net->params.as<float>();
    const BnParams bp{P + L.goff, P + L.beoff, P + L.rmoff, P + L.rvoff};
    return bn_train_forward(net->ctx->stream, net->ctx, A.bnpart, L.cout, A.z[l].as<uint16_t>(), npix, bp, update,
                            A.st(l), act, res, A.out(l));
}

// 3x3 layer l (convolution, stride-2 or transposed) into A.a[l]: with batch
// norm either the folded form with softplus fused, or (training) the raw
// convolution into A.z[l] and the normalisation; otherwise bias and skip
static hh_status light_conv(hh_net* net, LightActs& A, int l, int mode, const uint16_t* x, int B, int Hin, int Win,
                            int Hout, int Wout, const uint16_t* skip, const int* smap, const int* active, bool train,
                            bool update) {
    const LayerInfo& L = net->L[l];
    const uint16_t* pk = net->packed.as<uint16_t>();
    ConvArgs a{};
    a.x = x;
    a.B = B;
    a.Hin = Hin;
    a.Win = Win;
    a.Hout = Hout;
    a.Wout = Wout;
    a.active = active;
    a.skip = skip;
    a.skip_map = skip ? smap : nullptr;
    if (!L.bn) {
        a.y = A.out(l);
        a.wp = pk + net->pk_fwd[l];
        a.bias = net->params.as<float>() + L.boff;
        a.act = ACT_NONE;
        return launch_conv(net->ctx->stream, net->ctx->num_cus, L.cin, L.cout, mode, a);
    }
    if (!train) {
        a.y = A.out(l);
        a.wp = pk + net->pk_inf[l];
        a.bias = net->folded.as<float>() + L.beoff;
        a.act = ACT_SOFTPLUS;
        return launch_conv(net->ctx->stream, net->ctx->num_cus, L.cin, L.cout, mode, a);
    }
    a.y = A.z[l].as<uint16_t>();
    a.wp = pk + net->pk_fwd[l];
    a.bias = nullptr;
    a.act = ACT_NONE;
    a.active = nullptr;
    HH_TRY(launch_conv(net->ctx->stream, net->ctx->num_cus, L.cin, L.cout, mode, a));
    return light_bn(net, A, l, (size_t)B * Hout * Wout, ACT_SOFTPLUS, nullptr, update);
}

// inverted bottleneck of the layers le (expansion), le + 1 (depthwise), le + 2
// (shrink) on x [B][m][m][c]: A.a[le + 2] = x + BN(shrink(...))
static hh_status light_ib(hh_net* net, LightActs& A, int le, const uint16_t* x, int B, int m, const int* active,
                          bool train, bool update) {
    const int lw = le + 1, ls = le + 2;
    const LayerInfo &E = net->L[le], &Dw = net->L[lw], &S = net->L[ls];
    hipStream_t st = net->ctx->stream;
    const int cus = net->ctx->num_cus;
    const size_t npix = (size_t)B * m * m;
    const float* P = net->params.as<float>();
    const float* F = net->folded.as<float>();
    const uint16_t* pk = net->packed.as<uint16_t>();
    PwArgs pa{};
    pa.npix = npix;
    pa.pix_per_b = m * m;
    DwArgs da{};
    da.B = B;
    da.H = da.W = m;
    if (!train) {  // one fused kernel: the expanded channels stay in LDS
        IbArgs ia{};
        ia.x = x;
        ia.y = A.out(ls);
        ia.we = pk + net->pk_inf[le];
        ia.be = F + E.beoff;
        ia.wd = F + Dw.woff;
        ia.bd = F + Dw.beoff;
        ia.ws = pk + net->pk_inf[ls];
        ia.bs = F + S.beoff;
        ia.B = B;
        ia.m = m;
        ia.active = active;
        return launch_ib_fused(st, cus, E.cin, ia);
    }
    pa.x = x;
    pa.y = A.z[le].as<uint16_t>();
    pa.w = pk + net->pk_fwd[le];
    HH_TRY(launch_pointwise(st, cus, E.cin, E.cout, pa));
    HH_TRY(light_bn(net, A, le, npix, ACT_SOFTPLUS, nullptr, update));
    da.x = A.out(le);
    da.y = A.z[lw].as<uint16_t>();
    da.w = P + Dw.woff;
    HH_TRY(launch_depthwise(st, cus, Dw.cout, da));
    HH_TRY(light_bn(net, A, lw, npix, ACT_SOFTPLUS, nullptr, update));
    pa.x = A.out(lw);
    pa.y = A.z[ls].as<uint16_t>();
    pa.w = pk + net->pk_fwd[ls];
    HH_TRY(launch_pointwise(st, cus, S.cin, S.cout, pa));
    return light_bn(net, A, ls, npix, ACT_NONE, x, update);
}

// encoder of the lightweight network on every slowness model of md (A.a[0..8])
static hh_status light_encoder_forward(hh_net* net, hh_model* md, LightActs& A, bool train, bool update) {
    hipStream_t st = net->ctx->stream;
    const int n = md->lev[0].n, B = md->ninst;
    const double h = md->lev[0].h;
    HH_TRY(A.ensure_enc(net, B, n, train));
    const float* P = net->params.as<float>();
    hipLaunchKernelGGL((k_conv_in_mfma<1>), conv_in_grid(n, B), dim3(256), 0, st, md->lev[0].coef.as<float2>(),
                       (size_t)n * n, nullptr, nullptr, (float)(h * h), P + net->L[LL_ENC1_D].woff,
                       P + net->L[LL_ENC1_D].boff, nullptr, nullptr, A.out(LL_ENC1_D), n, nullptr);
    HH_LAUNCH_CHECK();
    for (int k = 0; k < 3; ++k) {
        const int l = 3 * k, m = n >> (k + 1);
        if (k > 0)
            HH_TRY(light_conv(net, A, l, CM_S2, A.out(l - 1), B, 2 * m, 2 * m, m, m, nullptr, nullptr, nullptr, train,
                              update));
        HH_TRY(light_conv(net, A, l + 1, CM_S1, A.out(l), B, m, m, m, m, nullptr, nullptr, nullptr, train, update));
        HH_TRY(light_conv(net, A, l + 2, CM_S1, A.out(l + 1), B, m, m, m, m, nullptr, nullptr, nullptr, train,
                          update));
    }
    return HH_OK;
}

// solver part of the lightweight network on B vectors v (see net_forward_core)
static hh_status light_forward(hh_net* net, int n, double h, LightActs& A, int B, const int* smap, const uint16_t* E1,
                               const uint16_t* E2, const uint16_t* E3, const float2* Gbr, const float2* v,
                               size_t vstride, const double* sig, int sig_stride, float2* x0, const int* active,
                               bool train, bool update, bool known_norm = false) {
    hipStream_t st = net->ctx->stream;
    HH_TRY(A.ensure(net, B, n, train));
    if (train) active = nullptr;
    float* in_scale = A.scales.as<float>();
    float* out_scale = in_scale + B;
    HH_TRY(launch_scales(st, v, vstride, (size_t)n * n, A.parts.as<double>(), active, sig, sig_stride, h * h, in_scale,
                         out_scale, B, known_norm));
    const float* P = net->params.as<float>();
    const int m1 = n / 2, m2 = n / 4, m3 = n / 8, m4 = coarsest_of(n), s4 = coarse_stride_of(n);
    auto o = [&](int l) { return A.out(l); };
    uint16_t* imp = A.imp.as<uint16_t>();
    {
        ProfScope ps(net->ctx, HH_K_CONV);
        hipLaunchKernelGGL((k_conv_in_mfma<0>), conv_in_grid(n, B), dim3(256), 0, st, v, vstride, in_scale, nullptr,
                           0.f, P + net->L[LL_S1_D].woff, P + net->L[LL_S1_D].boff, E1, smap, o(LL_S1_D), n, active);
        HH_LAUNCH_CHECK();
        HH_TRY(light_ib(net, A, LL_S1_E, o(LL_S1_D), B, m1, active, train, update));
        HH_TRY(light_conv(net, A, LL_S2_D, CM_S2, o(LL_S1_S), B, m1, m1, m2, m2, E2, smap, active, train, update));
        HH_TRY(light_ib(net, A, LL_S2_E, o(LL_S2_D), B, m2, active, train, update));
        HH_TRY(light_conv(net, A, LL_S3_D, CM_S2, o(LL_S2_S), B, m2, m2, m3, m3, E3, smap, active, train, update));
        HH_TRY(light_ib(net, A, LL_S3_E, o(LL_S3_D), B, m3, active, train, update));
        HH_TRY(light_conv(net, A, LL_S4_D, s4 == 2 ? CM_S2 : CM_S1, o(LL_S3_S), B, m3, m3, m4, m4, nullptr, nullptr,
                          active, train, update));
        HH_TRY(light_conv(net, A, LL_S4_C1, CM_S1, o(LL_S4_D), B, m4, m4, m4, m4, nullptr, nullptr, active, train,
                          update));
        HH_TRY(light_conv(net, A, LL_S4_C2, CM_S1, o(LL_S4_C1), B, m4, m4, m4, m4, nullptr, nullptr, active, train,
                          update));
    }
    {
        ProfScope ps(net->ctx, HH_K_NET_OTHER);
        if (net->explicit_coarse)
            HH_TRY(launch_explicit(st, o(LL_S4_C2), imp, P + net->koff, m4, net->nk, B, false, active, nullptr));
        else
            HH_TRY(launch_implicit(st, 2 * m4, o(LL_S4_C2), imp, Gbr, m4, net->nk, B, false, active, nullptr,
                                   A.impw.ptr ? A.impw.as<float2>() : nullptr));
    }
    {
        ProfScope ps(net->ctx, HH_K_CONV);
        HH_TRY(light_conv(net, A, LL_U3_T, s4 == 2 ? CM_T2 : CM_S1, imp, B, m4, m4, m3, m3, o(LL_S3_S), nullptr,
                          active, train, update));
        HH_TRY(light_conv(net, A, LL_U3_C1, CM_S1, o(LL_U3_T), B, m3, m3, m3, m3, nullptr, nullptr, active, train,
                          update));
        HH_TRY(light_conv(net, A, LL_U3_C2, CM_S1, o(LL_U3_C1), B, m3, m3, m3, m3, nullptr, nullptr, active, train,
                          update));
        HH_TRY(light_conv(net, A, LL_U2_T, CM_T2, o(LL_U3_C2), B, m3, m3, m2, m2, o(LL_S2_S), nullptr, active, train,
                          update));
        HH_TRY(light_conv(net, A, LL_U2_C1, CM_S1, o(LL_U2_T), B, m2, m2, m2, m2, nullptr, nullptr, active, train,
                          update));
        HH_TRY(light_conv(net, A, LL_U2_C2, CM_S1, o(LL_U2_C1), B, m2, m2, m2, m2, nullptr, nullptr, active, train,
                          update));
        HH_TRY(light_conv(net, A, LL_U1_T, CM_T2, o(LL_U2_C2), B, m2, m2, m1, m1, o(LL_S1_S), nullptr, active, train,
                          update));
        HH_TRY(light_conv(net, A, LL_U1_C1, CM_S1, o(LL_U1_T), B, m1, m1, m1, m1, nullptr, nullptr, active, train,
                          update));
        HH_TRY(light_conv(net, A, LL_U1_C2, CM_S1, o(LL_U1_C1), B, m1, m1, m1, m1, nullptr, nullptr, active, train,
                          update));
    }
    {
        ProfScope ps(net->ctx, HH_K_NET_OTHER);
        float2* out = A.a[LL_OUT].as<float2>();
        ConvArgs pa{};
        pa.x = o(LL_U1_C2);
        pa.wp = net->packed.as<uint16_t>() + net->pk_proj_hi;
        pa.wp_lo = net->packed.as<uint16_t>() + net->pk_proj_lo;
        pa.bias = P + net->L[LL_OUT].boff;
        pa.yproj = out;
        pa.B = B;
        pa.Hin = pa.Win = pa.Hout = pa.Wout = m1;
        pa.active = active;
        HH_TRY(launch_conv_proj(st, net->ctx->num_cus, pa));
        if (x0) {
            hipLaunchKernelGGL(k_prolong_x0, dim3((n * n + 255) / 256, B), dim3(256), 0, st, out, out_scale, x0, n,
                               active);
            HH_LAUNCH_CHECK();
        }
    }
    return HH_OK;
}

hh_status net_prepare_model(hh_model* md) {
    hh_net* net = md->net;
    if (!net) return HH_ERR_STATE;
    NetCache* nc = reinterpret_cast<NetCache*>(md->netcache);
    if (!nc) {
        nc = new (std::nothrow) NetCache();
        if (!nc) {
            set_error("out of host memory");
            return HH_ERR_NOMEM;
        }
        md->netcache = nc;
    }
    HH_TRY(net_pack(net));
    if (nc->uid == net->uid && nc->version == net->version && nc->n == md->lev[0].n) {
        nc->net = net;
        return HH_OK;
    }
    nc->uid = 0;  // invalid until rebuilt below
    const int n = md->lev[0].n;
    if (n % 16 != 0) {
        set_error("the network needs n divisible by 16 (n = %d)", n);
        return HH_ERR_ARG;
    }
    HH_TRY(net_pack(net));
    nc->n = n;
    nc->nc = coarsest_of(n);
    nc->M = 2 * nc->nc;
    HH_TRY(nc->Gbr.ensure(net->ctx, (size_t)net->nk * nc->M * nc->M * sizeof(float2)));
    if (!net->explicit_coarse) HH_TRY(green_forward(net, nc->nc, nc->Gbr.as<float2>(), 1e-5));
    if (net->ch[0] != 16) {
        set_error("first-level channel count must be 16");
        return HH_ERR_ARG;
    }
    if (net->light)
        HH_TRY(light_encoder_forward(net, md, nc->lacts, false, false));
    else
        HH_TRY(encoder_forward(net, md, nc->enc));
    nc->net = net;
    nc->uid = net->uid;
    nc->version = net->version;
    return HH_OK;
}

// e = out_scale * P(Net(v * in_scale)) for the B vectors v (stride vstride);
// writes x0 (complex single, [B][n][n]).  Encodings come from the model cache.
// Forward pass on B vectors v.  E1..E3: encodings ([.][m][m][c] BF16) indexed
// through smap (null: identity); Gbr: transformed Green's functions.  Keeps
// every activation in A; writes x0 = out_scale * P(o) when x0 is not null.
static hh_status net_forward_chunk(hh_net* net, int n, NetActs& A, int b0, int Bc, const float* in_scale0,
                                   const float* out_scale0, const int* smap0, const uint16_t* E1, const uint16_t* E2,
                                   const uint16_t* E3, const float2* Gbr, const float2* v0, size_t vstride,
                                   float2* x00, const int* active0, bool keep);

hh_status net_forward_core(hh_net* net, int n, double h, NetActs& A, int B, const int* smap, const uint16_t* E1,
                           const uint16_t* E2, const uint16_t* E3, const float2* Gbr, const float2* v, size_t vstride,
                           const double* sig, int sig_stride, float2* x0, const int* active, bool keep,
                           bool known_norm = false) {
    hipStream_t st = net->ctx->stream;
    HH_TRY(A.ensure(net, B, n));
    float* in_scale = A.scales.as<float>();
    float* out_scale = in_scale + B;
    HH_TRY(launch_scales(st, v, vstride, (size_t)n * n, A.parts.as<double>(), active, sig, sig_stride, h * h, in_scale,
                         out_scale, B, known_norm));
    // The whole batch in every launch.  (Running it through the network in
    // chunks of 8 or 16 samples, so that a layer's output could still sit in
    // the last-level cache for the next layer, measured 16% and 7% slower.)
    return net_forward_chunk(net, n, A, 0, B, in_scale, out_scale, smap, E1, E2, E3, Gbr, v, vstride, x0, active,
                             keep);
}

// samples b0 .. b0 + Bc - 1 of net_forward_core (scales already computed)
static hh_status net_forward_chunk(hh_net* net, int n, NetActs& A, int b0, int Bc, const float* in_scale0,
                                   const float* out_scale0, const int* smap0, const uint16_t* E1, const uint16_t* E2,
                                   const uint16_t* E3, const float2* Gbr, const float2* v0, size_t vstride,
                                   float2* x00, const int* active0, bool keep) {
    hipStream_t st = net->ctx->stream;
    const float* P = net->params.as<float>();
    const int m1 = n / 2, m2 = n / 4, m3 = n / 8, m4 = coarsest_of(n), s4 = coarse_stride_of(n);
    const int B = Bc;
    const int* active = active0 ? active0 + b0 : nullptr;
    const int* smap = smap0 ? smap0 + b0 : nullptr;
    if (!smap0) {  // sample b uses encoding b: the chunk's encodings start at b0
        E1 += (size_t)b0 * m1 * m1 * 16;
        E2 += (size_t)b0 * m2 * m2 * 32;
        E3 += (size_t)b0 * m3 * m3 * 64;
    }
    const float2* v = v0 + (size_t)b0 * vstride;
    float2* x0 = x00 ? x00 + (size_t)b0 * n * n : nullptr;
    const float* in_scale = in_scale0 + b0;
    const float* out_scale = out_scale0 + b0;
    auto act = [&](int l) { return A.a[l].as<uint16_t>() + (size_t)b0 * A.sample_elems(net, l); };
    uint16_t* imp = A.imp.as<uint16_t>() + (size_t)b0 * m4 * m4 * net->ch[3];
    float2* impw = A.impw.ptr ? A.impw.as<float2>() + (size_t)b0 * net->nk * m4 * (2 * m4) : nullptr;
    // layers l and l + 1 (stride 1, ReLU): fused for inference when both have 16
    // channels; the training pass keeps the intermediate output for its backward
    auto conv_pair = [&](int l, const uint16_t* x, uint16_t* mid, uint16_t* y, int m) -> hh_status {
        const LayerInfo &L1 = net->L[l], &L2 = net->L[l + 1];
        if (keep || L1.cin != 16 || L1.cout != 16 || L2.cout != 16) {
            HH_TRY(conv_layer(net, l, CM_S1, x, B, m, m, mid, m, m, nullptr, nullptr, true, active));
            return conv_layer(net, l + 1, CM_S1, mid, B, m, m, y, m, m, nullptr, nullptr, true, active);
        }
        ConvArgs a{};
        a.x = x;
        a.y = y;
        a.ymid = mid;
        a.wp = net->packed.as<uint16_t>() + net->pk_fwd[l];
        a.bias = P + L1.boff;
        a.wp2 = net->packed.as<uint16_t>() + net->pk_fwd[l + 1];
        a.bias2 = P + L2.boff;
        a.act = ACT_RELU;
        a.B = B;
        a.Hin = a.Win = a.Hout = a.Wout = m;
        a.active = active;
        return launch_conv(st, net->ctx->num_cus, 16, 16, CM_PAIR, a);
    };
    {
        ProfScope ps(net->ctx, HH_K_CONV);
        hipLaunchKernelGGL((k_conv_in_mfma<0>), conv_in_grid(n, B), dim3(256), 0, st, v, vstride, in_scale,
                           nullptr, 0.f, P + net->L[L_S1_D].woff, P + net->L[L_S1_D].boff, E1,
                           smap, act(L_S1_D), n, active);
        HH_LAUNCH_CHECK();
    }
    {
        ProfScope ps(net->ctx, HH_K_CONV);
        // level 1
        HH_TRY(conv_pair(L_S1_C1, act(L_S1_D), act(L_S1_C1), act(L_S1_C2), m1));
        // level 2
        HH_TRY(conv_layer(net, L_S2_D, CM_S2, act(L_S1_C2), B, m1, m1, act(L_S2_D), m2, m2, E2, smap, false, active));
        HH_TRY(conv_layer(net, L_S2_C1, CM_S1, act(L_S2_D), B, m2, m2, act(L_S2_C1), m2, m2, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_S2_C2, CM_S1, act(L_S2_C1), B, m2, m2, act(L_S2_C2), m2, m2, nullptr, nullptr, true, active));
        // level 3
        HH_TRY(conv_layer(net, L_S3_D, CM_S2, act(L_S2_C2), B, m2, m2, act(L_S3_D), m3, m3, E3, smap, false, active));
        HH_TRY(conv_layer(net, L_S3_C1, CM_S1, act(L_S3_D), B, m3, m3, act(L_S3_C1), m3, m3, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_S3_C2, CM_S1, act(L_S3_C1), B, m3, m3, act(L_S3_C2), m3, m3, nullptr, nullptr, true, active));
        // level 4 (stride 1 below n = 512)
        HH_TRY(conv_layer(net, L_S4_D, s4 == 2 ? CM_S2 : CM_S1, act(L_S3_C2), B, m3, m3, act(L_S4_D), m4, m4, nullptr, nullptr, false, active));
        HH_TRY(conv_layer(net, L_S4_C1, CM_S1, act(L_S4_D), B, m4, m4, act(L_S4_C1), m4, m4, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_S4_C2, CM_S1, act(L_S4_C1), B, m4, m4, act(L_S4_C2), m4, m4, nullptr, nullptr, true, active));
    }
    {
        ProfScope ps(net->ctx, HH_K_NET_OTHER);
        if (net->explicit_coarse)
            HH_TRY(launch_explicit(st, act(L_S4_C2), imp, P + net->koff, m4, net->nk, B, false, active, nullptr));
        else
            HH_TRY(launch_implicit(st, 2 * m4, act(L_S4_C2), imp, Gbr, m4, net->nk, B, false, active, nullptr,
                                   impw));
    }
    {
        ProfScope ps(net->ctx, HH_K_CONV);
        // up to level 3: transposed stride-2 (stride-1 below n = 512), + level-3 features
        HH_TRY(conv_layer(net, L_U3_T, s4 == 2 ? CM_T2 : CM_S1, imp, B, m4, m4, act(L_U3_T), m3, m3, act(L_S3_C2), nullptr, false, active));
        HH_TRY(conv_layer(net, L_U3_C1, CM_S1, act(L_U3_T), B, m3, m3, act(L_U3_C1), m3, m3, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_U3_C2, CM_S1, act(L_U3_C1), B, m3, m3, act(L_U3_C2), m3, m3, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_U2_T, CM_T2, act(L_U3_C2), B, m3, m3, act(L_U2_T), m2, m2, act(L_S2_C2), nullptr, false, active));
        HH_TRY(conv_layer(net, L_U2_C1, CM_S1, act(L_U2_T), B, m2, m2, act(L_U2_C1), m2, m2, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_U2_C2, CM_S1, act(L_U2_C1), B, m2, m2, act(L_U2_C2), m2, m2, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_U1_T, CM_T2, act(L_U2_C2), B, m2, m2, act(L_U1_T), m1, m1, act(L_S1_C2), nullptr, false, active));
        HH_TRY(conv_pair(L_U1_C1, act(L_U1_T), act(L_U1_C1), act(L_U1_C2), m1));
    }
    {
        ProfScope ps(net->ctx, HH_K_NET_OTHER);
        float2* o = A.a[L_OUT].as<float2>() + (size_t)b0 * m1 * m1;
        ConvArgs pa{};
        pa.x = act(L_U1_C2);
        pa.wp = net->packed.as<uint16_t>() + net->pk_proj_hi;
        pa.wp_lo = net->packed.as<uint16_t>() + net->pk_proj_lo;
        pa.bias = P + net->L[L_OUT].boff;
        pa.yproj = o;
        pa.B = B;
        pa.Hin = pa.Win = pa.Hout = pa.Wout = m1;
        pa.active = active;
        HH_TRY(launch_conv_proj(st, net->ctx->num_cus, pa));
        if (x0) {
            hipLaunchKernelGGL(k_prolong_x0, dim3((n * n + 255) / 256, B), dim3(256), 0, st, o, out_scale, x0, n,
                               active);
            HH_LAUNCH_CHECK();
        }
    }
    return HH_OK;
}

hh_status net_forward_batch(hh_net* net, hh_model* md, NetActs& A, int B, const BatchMap& bm, const float2* v,
                            size_t vstride, const double* sig, int sig_stride, float2* x0, const int* active,
                            bool known_norm) {
    NetCache* nc = reinterpret_cast<NetCache*>(md->netcache);
    HH_TRY(A.ensure(net, B, md->lev[0].n));
    const int* smap = md->ninst > 1 ? bm.inst : A.zeros.as<int>();
    return net_forward_core(net, md->lev[0].n, md->lev[0].h, A, B, smap, nc->enc[L_ENC1_C2].as<uint16_t>(),
                            nc->enc[L_ENC2_C2].as<uint16_t>(), nc->enc[L_ENC3_C2].as<uint16_t>(),
                            nc->Gbr.as<float2>(), v, vstride, sig, sig_stride, x0, active, false, known_norm);
}

// either network's forward pass on B vectors of model md (encodings and Ghat from
// the model cache), and where its half-resolution output and scales are kept
// (known_norm: v are FGMRES basis vectors of norm 1/sig, see launch_scales)
static hh_status net_forward_model(hh_net* net, hh_model* md, int B, const BatchMap& bm, const float2* v,
                                   size_t vstride, const double* sig, int sig_stride, float2* x0, const int* active,
                                   bool known_norm = false) {
    NetCache* nc = reinterpret_cast<NetCache*>(md->netcache);
    if (!net->light)
        return net_forward_batch(net, md, nc->acts, B, bm, v, vstride, sig, sig_stride, x0, active, known_norm);
    LightActs& A = nc->lacts;
    HH_TRY(A.ensure(net, B, md->lev[0].n, false));
    const int* smap = md->ninst > 1 ? bm.inst : A.zeros.as<int>();
    return light_forward(net, md->lev[0].n, md->lev[0].h, A, B, smap, A.out(LL_ENC1_C2), A.out(LL_ENC2_C2),
                         A.out(LL_ENC3_C2), nc->Gbr.as<float2>(), v, vstride, sig, sig_stride, x0, active, false,
                         false, known_norm);
}
static const float2* net_out_of(const NetCache* nc, const hh_net* net) {
    return net->light ? nc->lacts.a[LL_OUT].as<float2>() : nc->acts.a[L_OUT].as<float2>();
}
static const float* net_out_scale_of(const NetCache* nc, const hh_net* net, int B) {
    return (net->light ? nc->lacts.scales.as<float>() : nc->acts.scales.as<float>()) + B;
}

// ---------------------------------------------------------------------------
// CNN+MG preconditioner used by the solve
// ---------------------------------------------------------------------------
hh_status net_precond(void* user, hh_model* md, SolveWork& W, const BatchMap& bm, const float2* v, size_t vstride,
                      const double* sig, int sig_stride, float2* z, size_t zstride, const int* act) {
    (void)user;
    hh_net* net = md->net;
    if (!net) {
        set_error("no network attached to the model");
        return HH_ERR_STATE;
    }
    HH_TRY(net_prepare_model(md));
    NetCache* nc = reinterpret_cast<NetCache*>(md->netcache);
    // the V-cycle reads the network's half-resolution output and interpolates
    // the initial guess itself: no fine x0 is stored
    // v are the solve's lazily normalised basis vectors: their norms are 1/sig
    HH_TRY(net_forward_model(net, md, W.nrhs, bm, v, vstride, sig, sig_stride, nullptr, act, true));
    return launch_vcycle_strided(md, W.nrhs, bm, v, vstride, sig, sig_stride, nullptr, 0, z, zstride, W.vwork.ptr, act,
                                 net_out_of(nc, net), net_out_scale_of(nc, net, W.nrhs));
}

// ===========================================================================
// Training (Sec. 4.3, Sec. 5.3): MSE loss (eq. 19) on method-generated pairs
// (eq. 20), backward pass through every layer, Adam on the FP32 masters.
// ===========================================================================

// ---- weight gradients of the 16/32/64-channel layers -----------------------
// part[blk][oo][ii][t] = sum over the block's output pixels p of
//   A[b][p][oo] * X[b][src(p, t)][ii],   src = p + (ky-1, kx-1) (S1) or 2p + (ky-1, kx-1) (S2).
// Convolutions: A = output gradient, X = layer input -> dW (cout, cin, 3, 3).
// Transposed convolutions: A = layer input, X = output gradient -> dW (cin, cout, 3, 3).
template <int CA, int CX, int MODE>
struct WgCfg {
    static constexpr int TC = 32;
    static constexpr int TR = (MODE == CM_S2) ? (CX >= 64 ? 2 : 4) : 4;
    static constexpr int PH = (MODE == CM_S2) ? 2 * TR + 1 : TR + 2;
    static constexpr int PW = (MODE == CM_S2) ? 2 * TC + 1 : TC + 2;
};

template <int CA, int CX, int MODE>
__global__ void __launch_bounds__(256) k_wgrad(const uint16_t* __restrict__ A, const uint16_t* __restrict__ X,
                                               float* __restrict__ part, int Ho, int Wo, int Hi, int Wi, int tiles_x,
                                               int tiles_y) {
    using Cf = WgCfg<CA, CX, MODE>;
    __shared__ __attribute__((aligned(16))) uint16_t sA[Cf::TR * Cf::TC * CA];
    __shared__ __attribute__((aligned(16))) uint16_t sX[Cf::PH * Cf::PW * CX];
    const int blk = blockIdx.x;
    const int b = blk / (tiles_x * tiles_y);
    const int rem = blk - b * tiles_x * tiles_y;
    const int ty = rem / tiles_x, tx = rem - ty * tiles_x;
    const int y0 = ty * Cf::TR, x0 = tx * Cf::TC;
    const int tid = threadIdx.x;
    const uint16_t* Ab = A + (size_t)b * Ho * Wo * CA;
    const uint16_t* Xb = X + (size_t)b * Hi * Wi * CX;
    for (int e = tid; e < Cf::TR * Cf::TC * (CA / 8); e += 256) {
        const int v = e % (CA / 8), pix = e / (CA / 8);
        const int r = pix / Cf::TC, c = pix - r * Cf::TC;
        const int oy = y0 + r, ox = x0 + c;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (oy < Ho && ox < Wo) val = *reinterpret_cast<const uint4*>(Ab + ((size_t)oy * Wo + ox) * CA + 8 * v);
        *reinterpret_cast<uint4*>(&sA[pix * CA + 8 * v]) = val;
    }
    for (int e = tid; e < Cf::PH * Cf::PW * (CX / 8); e += 256) {
        const int v = e % (CX / 8), pix = e / (CX / 8);
        const int py = pix / Cf::PW, px = pix - py * Cf::PW;
        const int iy = (MODE == CM_S2 ? 2 * y0 : y0) - 1 + py, ix = (MODE == CM_S2 ? 2 * x0 : x0) - 1 + px;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (iy >= 0 && iy < Hi && ix >= 0 && ix < Wi)
            val = *reinterpret_cast<const uint4*>(Xb + ((size_t)iy * Wi + ix) * CX + 8 * v);
        *reinterpret_cast<uint4*>(&sX[pix * CX + 8 * v]) = val;
    }
    __syncthreads();
    constexpr int NOB = CA / 4, NIB = CX / 4;
    for (int it = tid; it < 9 * NOB * NIB; it += 256) {
        const int t = it / (NOB * NIB);
        const int r2 = it - t * NOB * NIB;
        const int ob = r2 / NIB, ib = r2 - ob * NIB;
        const int ky = t / 3, kx = t - 3 * ky;
        float acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
        for (int p = 0; p < Cf::TR * Cf::TC; ++p) {
            const int r = p / Cf::TC, c = p - r * Cf::TC;
            const uint2 ar = *reinterpret_cast<const uint2*>(&sA[p * CA + 4 * ob]);
            const int sy = (MODE == CM_S2 ? 2 * r : r) + ky, sx = (MODE == CM_S2 ? 2 * c : c) + kx;
            const uint2 xr = *reinterpret_cast<const uint2*>(&sX[(sy * Cf::PW + sx) * CX + 4 * ib]);
            const float a[4] = {bf2f((uint16_t)(ar.x & 0xffff)), bf2f((uint16_t)(ar.x >> 16)),
                                bf2f((uint16_t)(ar.y & 0xffff)), bf2f((uint16_t)(ar.y >> 16))};
            const float x[4] = {bf2f((uint16_t)(xr.x & 0xffff)), bf2f((uint16_t)(xr.x >> 16)),
                                bf2f((uint16_t)(xr.y & 0xffff)), bf2f((uint16_t)(xr.y >> 16))};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * x[j];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) part[(((size_t)blk * CA + 4 * ob + i) * CX + 4 * ib + j) * 9 + t] = acc[i][j];
    }
}

// Deterministic reduction of per-block partial sums, out[e] = scale * sum_b part[b][e], in two
// stages so that thousands of partial rows are read by many workgroups: stage one sums the rows
// of each slice of `chunk` consecutive blocks into the slice's first row (in place: the thread
// for column e of a slice is the only one that reads or writes that column of the slice), stage
// two sums those first rows in slice order.
__global__ void k_reduce_slices(float* __restrict__ part, int nblk, int count, int chunk) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const int b0 = blockIdx.y * chunk, b1 = min(b0 + chunk, nblk);
    float acc = 0.f;
    for (int b = b0; b < b1; ++b) acc += part[(size_t)b * count + e];
    part[(size_t)b0 * count + e] = acc;
}

__global__ void k_reduce_part(const float* __restrict__ part, int nrow, int rstride, int count,
                              float* __restrict__ out, float scale) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    float acc = 0.f;
    for (int b = 0; b < nrow; ++b) acc += part[(size_t)b * rstride * count + e];
    out[e] = acc * scale;
}

static hh_status reduce_partials(hipStream_t st, float* part, int nblk, int count, float* out, float scale) {
    const int gx = (count + 255) / 256;
    int chunk = nblk, nslice = 1;
    if (nblk >= 64) {  // aim at about 2048 workgroups for the first stage
        const int want = std::max(1, std::min(nblk / 8, (2048 + gx - 1) / gx));
        chunk = (nblk + want - 1) / want;
        nslice = (nblk + chunk - 1) / chunk;
    }
    if (nslice > 1) {
        hipLaunchKernelGGL(k_reduce_slices, dim3(gx, nslice), dim3(256), 0, st, part, nblk, count, chunk);
        HH_LAUNCH_CHECK();
    }
    // without the first stage every block's row is summed directly
    hipLaunchKernelGGL(k_reduce_part, dim3(gx), dim3(256), 0, st, part, nslice > 1 ? nslice : nblk,
                       nslice > 1 ? chunk : 1, count, out, scale);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

template <int CA, int CX, int MODE>
static hh_status launch_wgrad_t(hipStream_t st, const uint16_t* A, const uint16_t* X, int B, int Ho, int Wo, int Hi,
                                int Wi, Buf& part, hh_ctx* ctx, float* out) {
    using Cf = WgCfg<CA, CX, MODE>;
    const int tx = (Wo + Cf::TC - 1) / Cf::TC, ty = (Ho + Cf::TR - 1) / Cf::TR;
    const int nblk = B * tx * ty;
    const int count = CA * CX * 9;
    HH_TRY(part.ensure(ctx, (size_t)nblk * count * sizeof(float)));
    hipLaunchKernelGGL((k_wgrad<CA, CX, MODE>), dim3(nblk), dim3(256), 0, st, A, X, part.as<float>(), Ho, Wo, Hi, Wi,
                       tx, ty);
    HH_LAUNCH_CHECK();
    HH_TRY(reduce_partials(st, part.as<float>(), nblk, count, out, 1.f));
    return HH_OK;
}

static hh_status launch_wgrad(hipStream_t st, int ca, int cx, int mode, const uint16_t* A, const uint16_t* X, int B,
                              int Ho, int Wo, int Hi, int Wi, Buf& part, hh_ctx* ctx, float* out) {
#define HH_WG(CA_, CX_, MD)                      \
    if (ca == CA_ && cx == CX_ && mode == MD) \
        return launch_wgrad_t<CA_, CX_, MD>(st, A, X, B, Ho, Wo, Hi, Wi, part, ctx, out);
    HH_WG(16, 16, CM_S1)
    HH_WG(32, 32, CM_S1)
    HH_WG(64, 64, CM_S1)
    HH_WG(32, 16, CM_S2)
    HH_WG(64, 32, CM_S2)
    HH_WG(64, 64, CM_S2)
#undef HH_WG
    set_error("no weight-gradient kernel for %d x %d mode %d", ca, cx, mode);
    return HH_ERR_ARG;
}

// channel sums of a BF16 NHWC tensor over all pixels: part[blk][c]
template <int C>
__global__ void __launch_bounds__(256) k_chsum(const uint16_t* __restrict__ A, size_t npix, float* __restrict__ part) {
    __shared__ float s[256];
    constexpr int PPB = 256 / C;  // pixels handled concurrently
    const int c = threadIdx.x % C, lane_p = threadIdx.x / C;
    float acc = 0.f;
    for (size_t p = (size_t)blockIdx.x * PPB + lane_p; p < npix; p += (size_t)gridDim.x * PPB)
        acc += bf2f(A[p * C + c]);
    s[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < C) {
        float t = 0.f;
        for (int q = 0; q < PPB; ++q) t += s[q * C + threadIdx.x];
        part[(size_t)blockIdx.x * C + threadIdx.x] = t;
    }
}

static hh_status launch_bgrad(hipStream_t st, int C, const uint16_t* A, size_t npix, Buf& part, hh_ctx* ctx,
                              float* out) {
    const int nblk = 512;
    HH_TRY(part.ensure(ctx, (size_t)nblk * C * sizeof(float)));
    if (C == 16)
        hipLaunchKernelGGL(k_chsum<16>, dim3(nblk), dim3(256), 0, st, A, npix, part.as<float>());
    else if (C == 32)
        hipLaunchKernelGGL(k_chsum<32>, dim3(nblk), dim3(256), 0, st, A, npix, part.as<float>());
    else if (C == 64)
        hipLaunchKernelGGL(k_chsum<64>, dim3(nblk), dim3(256), 0, st, A, npix, part.as<float>());
    else {
        set_error("channel sum for %d channels", C);
        return HH_ERR_ARG;
    }
    HH_LAUNCH_CHECK();
    HH_TRY(reduce_partials(st, part.as<float>(), nblk, C, out, 1.f));
    return HH_OK;
}

// ---- projection layer (CIN -> 2) backward --------------------------------
// input gradient: g[q][c] = sum_{o,t} W[o][c][t] go[q - off(t)][o], masked by (x > 0) unless mask is null
template <int CIN>
__global__ void __launch_bounds__(256) k_out_dgrad(const float2* __restrict__ go, const float* __restrict__ W,
                                                   const uint16_t* __restrict__ mask, uint16_t* __restrict__ g, int m) {
    __shared__ float s_w[2 * CIN * 9];
    for (int e = threadIdx.x; e < 2 * CIN * 9; e += 256) s_w[e] = W[e];
    __syncthreads();
    const int b = blockIdx.y;
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= m * m) return;
    const int qy = q / m, qx = q - qy * m;
    float acc[CIN];
#pragma unroll
    for (int c = 0; c < CIN; ++c) acc[c] = 0.f;
    for (int t = 0; t < 9; ++t) {
        const int py = qy - (t / 3 - 1), px = qx - (t % 3 - 1);
        if (py < 0 || py >= m || px < 0 || px >= m) continue;
        const float2 gv = go[(size_t)b * m * m + (size_t)py * m + px];
#pragma unroll
        for (int c = 0; c < CIN; ++c) acc[c] += s_w[(0 * CIN + c) * 9 + t] * gv.x + s_w[(1 * CIN + c) * 9 + t] * gv.y;
    }
    const size_t o = ((size_t)b * m * m + q) * CIN;
#pragma unroll
    for (int c0 = 0; c0 < CIN; c0 += 8) {
        uint4 mr = mask ? *reinterpret_cast<const uint4*>(mask + o + c0) : make_uint4(0, 0, 0, 0);
        const uint16_t* mh = reinterpret_cast<const uint16_t*>(&mr);
        uint16_t out[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) out[u] = f2bf((!mask || bf2f(mh[u]) > 0.f) ? acc[c0 + u] : 0.f);
        *reinterpret_cast<uint4*>(g + o + c0) = *reinterpret_cast<uint4*>(out);
    }
}

// weight gradient: part[blk][o][c][t] = sum_p go[p][o] x[p + off(t)][c];  bias: part[blk][2*CIN*9 + o]
template <int CIN>
__global__ void __launch_bounds__(256) k_out_wgrad(const float2* __restrict__ go, const uint16_t* __restrict__ x,
                                                   float* __restrict__ part, int m, int chunk) {
    const int blk = blockIdx.x;
    const int b = blockIdx.y;
    const int nb = gridDim.x;
    const int count = 2 * CIN * 9 + 2;
    for (int it = threadIdx.x; it < count; it += 256) {
        float acc = 0.f;
        const int p0 = blk * chunk, p1 = min(m * m, p0 + chunk);
        if (it < 2 * CIN * 9) {
            const int o = it / (CIN * 9), c = (it / 9) % CIN, t = it % 9;
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            for (int p = p0; p < p1; ++p) {
                const int py = p / m, px = p - py * m;
                const int sy = py + dy, sx = px + dx;
                if (sy < 0 || sy >= m || sx < 0 || sx >= m) continue;
                const float2 gv = go[(size_t)b * m * m + p];
                acc += (o == 0 ? gv.x : gv.y) * bf2f(x[(((size_t)b * m + sy) * m + sx) * CIN + c]);
            }
        } else {
            const int o = it - 2 * CIN * 9;
            for (int p = p0; p < p1; ++p) {
                const float2 gv = go[(size_t)b * m * m + p];
                acc += (o == 0 ? gv.x : gv.y);
            }
        }
        part[((size_t)b * nb + blk) * count + it] = acc;
    }
}

// ---- first layer (2 -> COUT, stride 2) weight + bias gradient --------------
template <int SRC, int COUT>
__global__ void __launch_bounds__(256) k_in_wgrad(const uint16_t* __restrict__ g, const float2* __restrict__ src,
                                                  size_t src_bstride, const float* __restrict__ in_scale, float h2,
                                                  float* __restrict__ part, int n, int chunk) {
    const int blk = blockIdx.x, b = blockIdx.y, nb = gridDim.x;
    const int m = n / 2;
    const int count = COUT * 18 + COUT;
    const float sc = (SRC == 0) ? in_scale[b] : 1.f;
    const float2* sb = src + (size_t)b * src_bstride;
    const int p0 = blk * chunk, p1 = min(m * m, p0 + chunk);
    for (int it = threadIdx.x; it < count; it += 256) {
        float acc = 0.f;
        if (it < COUT * 18) {
            const int co = it / 18, ci = (it / 9) % 2, t = it % 9;
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            for (int p = p0; p < p1; ++p) {
                const int oy = p / m, ox = p - oy * m;
                const int iy = 2 * oy + dy, ix = 2 * ox + dx;
                if (iy < 0 || iy >= n || ix < 0 || ix >= n) continue;
                const float2 v = sb[(size_t)iy * n + ix];
                float a;
                if (SRC == 0) {
                    a = (ci == 0 ? v.x : v.y) * sc;
                } else {
                    const float m0 = v.x * h2;
                    a = ci == 0 ? m0 : m0 * v.y;
                }
                a = bf2f(f2bf(a));
                acc += bf2f(g[((size_t)b * m * m + p) * COUT + co]) * a;
            }
        } else {
            const int co = it - COUT * 18;
            for (int p = p0; p < p1; ++p) acc += bf2f(g[((size_t)b * m * m + p) * COUT + co]);
        }
        part[((size_t)b * nb + blk) * count + it] = acc;
    }
}

// ---- implicit layer: gradient of the transformed Green's functions --------
// part[b][c][k1][k2] = conj(FFT(pad z))[k] * FFT(pad gy)[k] / M^2 (natural order)
template <int M, int NT>
__global__ void __launch_bounds__(NT) k_implicit_ggrad(const uint16_t* __restrict__ z, const uint16_t* __restrict__ gy,
                                                       float2* __restrict__ part, int nc, int nk) {
    extern __shared__ float2 s_dyn[];
    constexpr int P = M + 1;
    float2* s0 = s_dyn;
    float2* s1 = s_dyn + M * P;
    float2* tw = s_dyn + 2 * M * P;
    const int c = blockIdx.x, b = blockIdx.y;
    const int tid = threadIdx.x;
    const int CH = 2 * nk;
    for (int t = tid; t < M / 2; t += NT) {
        float sn, cs;
        sincospif(-2.0f * (float)t / (float)M, &sn, &cs);
        tw[t] = make_float2(cs, sn);
    }
    for (int e = tid; e < 2 * M * P; e += NT) s_dyn[e] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int e = tid; e < nc * nc; e += NT) {
        const int y = e / nc, x = e - y * nc;
        const size_t o = (((size_t)b * nc + y) * nc + x) * CH + 2 * c;
        const uint32_t r0 = *reinterpret_cast<const uint32_t*>(z + o);
        const uint32_t r1 = *reinterpret_cast<const uint32_t*>(gy + o);
        s0[y * P + x] = make_float2(bf2f((uint16_t)(r0 & 0xffff)), bf2f((uint16_t)(r0 >> 16)));
        s1[y * P + x] = make_float2(bf2f((uint16_t)(r1 & 0xffff)), bf2f((uint16_t)(r1 >> 16)));
    }
    __syncthreads();
    for (int len = M; len >= 2; len >>= 1) {
        const int half = len >> 1, tws = M / len;
        for (int t = tid; t < 2 * nc * (M / 2); t += NT) {
            float2* s = (t < nc * (M / 2)) ? s0 : s1;
            const int tt = t % (nc * (M / 2));
            const int row = tt / (M / 2), bf = tt - row * (M / 2);
            const int blk = bf / half, j = bf - blk * half;
            const int i0 = row * P + blk * len + j, i1 = i0 + half;
            const float2 a = s[i0], bb = s[i1];
            s[i0] = cadd(a, bb);
            s[i1] = cmul(csub(a, bb), tw[j * tws]);
        }
        __syncthreads();
    }
    for (int len = M; len >= 2; len >>= 1) {
        const int half = len >> 1, tws = M / len;
        for (int t = tid; t < 2 * M * (M / 2); t += NT) {
            float2* s = (t < M * (M / 2)) ? s0 : s1;
            const int tt = t % (M * (M / 2));
            const int col = tt % M, bf = tt / M;
            const int blk = bf / half, j = bf - blk * half;
            const int i0 = (blk * len + j) * P + col, i1 = i0 + half * P;
            const float2 a = s[i0], bb = s[i1];
            s[i0] = cadd(a, bb);
            s[i1] = cmul(csub(a, bb), tw[j * tws]);
        }
        __syncthreads();
    }
    int bits = 0;
    while ((1 << bits) < M) ++bits;
    const float sc = 1.f / ((float)M * M);
    for (int e = tid; e < M * M; e += NT) {
        const int r = e / M, col = e - r * M;
        const float2 a = s0[r * P + col], g = s1[r * P + col];
        // conj(a) * g
        const float2 pr = make_float2((a.x * g.x + a.y * g.y) * sc, (a.x * g.y - a.y * g.x) * sc);
        const int k1 = (int)(__brev((unsigned)r) >> (32 - bits)), k2 = (int)(__brev((unsigned)col) >> (32 - bits));
        part[(((size_t)b * nk + c) * M + k1) * M + k2] = pr;
    }
}

// the same for transforms too large for two maps in LDS (M = 128, the 1024^2
// network): FFT(pad z) goes through a scratch map in global memory (written
// and read back by the same threads), FFT(pad gy) stays in LDS
template <int M, int NT>
__global__ void __launch_bounds__(NT) k_implicit_ggrad_big(const uint16_t* __restrict__ z,
                                                           const uint16_t* __restrict__ gy, float2* __restrict__ scratch,
                                                           float2* __restrict__ part, int nc, int nk) {
    extern __shared__ float2 s_dyn[];
    constexpr int P = M + 1;
    float2* s = s_dyn;
    float2* tw = s_dyn + M * P;
    const int c = blockIdx.x, b = blockIdx.y;
    const int tid = threadIdx.x;
    const int CH = 2 * nk;
    float2* zs = scratch + ((size_t)b * nk + c) * M * M;
    for (int t = tid; t < M / 2; t += NT) {
        float sn, cs;
        sincospif(-2.0f * (float)t / (float)M, &sn, &cs);
        tw[t] = make_float2(cs, sn);
    }
    int bits = 0;
    while ((1 << bits) < M) ++bits;
    const float sc = 1.f / ((float)M * M);
    for (int pass = 0; pass < 2; ++pass) {
        const uint16_t* src = pass == 0 ? z : gy;
        __syncthreads();  // the previous pass is done with s
        for (int e = tid; e < M * P; e += NT) s[e] = make_float2(0.f, 0.f);
        __syncthreads();
        for (int e = tid; e < nc * nc; e += NT) {
            const int y = e / nc, x = e - y * nc;
            const uint32_t r0 = *reinterpret_cast<const uint32_t*>(src + (((size_t)b * nc + y) * nc + x) * CH + 2 * c);
            s[y * P + x] = make_float2(bf2f((uint16_t)(r0 & 0xffff)), bf2f((uint16_t)(r0 >> 16)));
        }
        __syncthreads();
        for (int len = M; len >= 2; len >>= 1) {  // rows holding data
            const int half = len >> 1, tws = M / len;
            for (int t = tid; t < nc * (M / 2); t += NT) {
                const int row = t / (M / 2), bf = t - row * (M / 2);
                const int blk = bf / half, j = bf - blk * half;
                const int i0 = row * P + blk * len + j, i1 = i0 + half;
                const float2 a = s[i0], bb = s[i1];
                s[i0] = cadd(a, bb);
                s[i1] = cmul(csub(a, bb), tw[j * tws]);
            }
            __syncthreads();
        }
        for (int len = M; len >= 2; len >>= 1) {  // all columns
            const int half = len >> 1, tws = M / len;
            for (int t = tid; t < M * (M / 2); t += NT) {
                const int col = t % M, bf = t / M;
                const int blk = bf / half, j = bf - blk * half;
                const int i0 = (blk * len + j) * P + col, i1 = i0 + half * P;
                const float2 a = s[i0], bb = s[i1];
                s[i0] = cadd(a, bb);
                s[i1] = cmul(csub(a, bb), tw[j * tws]);
            }
            __syncthreads();
        }
        for (int e = tid; e < M * M; e += NT) {
            const int r = e / M, col = e - r * M;
            if (pass == 0) {
                zs[e] = s[r * P + col];
            } else {
                const float2 a = zs[e], g = s[r * P + col];  // written by this thread in pass 0
                const float2 pr = make_float2((a.x * g.x + a.y * g.y) * sc, (a.x * g.y - a.y * g.x) * sc);
                const int k1 = (int)(__brev((unsigned)r) >> (32 - bits));
                const int k2 = (int)(__brev((unsigned)col) >> (32 - bits));
                part[(((size_t)b * nk + c) * M + k1) * M + k2] = pr;
            }
        }
    }
}

// gG[c][e] = sum_b part[b][c][e]  (FP64)
__global__ void k_reduce_ggrad(const float2* __restrict__ part, int B, int count, double2* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < B; ++b) {
        const float2 v = part[(size_t)b * count + e];
        re += v.x;
        im += v.y;
    }
    out[e] = make_double2(re, im);
}

// ---- Green's function backward -------------------------------------------
// gS -> gKhat: gf = conj(F(delta)) gS, then the real Jacobian of
// f(z) = conj(z)/(|z|^2 + eps) at z = Khat.
__global__ void k_green_gkhat(const double2* __restrict__ gS, const float* __restrict__ K, double2* __restrict__ gKh,
                              int N, double eps) {
    const int c = blockIdx.y;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= N * N) return;
    const int p = idx / N, q = idx - p * N;
    double re = 0.0, im = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int bb = 0; bb < 3; ++bb) {
            const double kr = K[((size_t)c * 9 + a * 3 + bb) * 2], ki = K[((size_t)c * 9 + a * 3 + bb) * 2 + 1];
            long t = ((long)p * (a - 1) + (long)q * (bb - 1)) % N;
            if (t < 0) t += N;
            double sn, cs;
            sincospi(-2.0 * (double)t / (double)N, &sn, &cs);
            re += kr * cs - ki * sn;
            im += kr * sn + ki * cs;
        }
    const double sign = ((p + q) & 1) ? -1.0 : 1.0;
    const double2 g = gS[(size_t)c * N * N + idx];
    const double gfr = sign * g.x, gfi = sign * g.y;
    const double d = re * re + im * im + eps;
    const double dfr_da = 1.0 / d - 2 * re * re / (d * d), dfr_db = -2 * re * im / (d * d);
    const double dfi_da = 2 * re * im / (d * d), dfi_db = -1.0 / d + 2 * im * im / (d * d);
    gKh[(size_t)c * N * N + idx] = make_double2(gfr * dfr_da + gfi * dfi_da, gfr * dfr_db + gfi * dfi_db);
}

// gK[c][a][b] = sum_{p,q} gKhat[p][q] exp(+2 pi i (p (a-1) + q (b-1)) / N), written as (re, im) floats
__global__ void __launch_bounds__(256) k_green_gK(const double2* __restrict__ gKh, float* __restrict__ gK, int N) {
    __shared__ double s_re[256], s_im[256];
    const int c = blockIdx.y, tap = blockIdx.x;
    const int a = tap / 3, bb = tap % 3;
    double re = 0.0, im = 0.0;
    for (int idx = threadIdx.x; idx < N * N; idx += 256) {
        const int p = idx / N, q = idx - p * N;
        long t = ((long)p * (a - 1) + (long)q * (bb - 1)) % N;
        if (t < 0) t += N;
        double sn, cs;
        sincospi(2.0 * (double)t / (double)N, &sn, &cs);
        const double2 g = gKh[(size_t)c * N * N + idx];
        re += g.x * cs - g.y * sn;
        im += g.x * sn + g.y * cs;
    }
    s_re[threadIdx.x] = re;
    s_im[threadIdx.x] = im;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_re[threadIdx.x] += s_re[threadIdx.x + w];
            s_im[threadIdx.x] += s_im[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        gK[((size_t)c * 9 + tap) * 2] = (float)s_re[0];
        gK[((size_t)c * 9 + tap) * 2 + 1] = (float)s_im[0];
    }
}

// dL/dK from dL/dGhat (natural order, FP64), eq. 17 backward
static hh_status green_backward(hh_net* net, int nc, const double2* gGh, float* gK, double eps) {
    hipStream_t st = net->ctx->stream;
    const int M = 2 * nc, N = nextpow2(3 * M), nk = net->nk;
    Buf A, Bt, S, Kh;
    HH_TRY(A.ensure(net->ctx, (size_t)nk * M * M * sizeof(double2)));
    HH_TRY(Bt.ensure(net->ctx, (size_t)nk * M * N * sizeof(double2)));
    HH_TRY(S.ensure(net->ctx, (size_t)nk * N * N * sizeof(double2)));
    HH_TRY(Kh.ensure(net->ctx, (size_t)nk * N * N * sizeof(double2)));
    // gG[g1][g2] = sum_k gGhat[k1][k2] exp(+2 pi i (k1 (g1 - nc) + k2 (g2 - nc)) / M)
    HH_TRY(dft_pass(st, gGh, A.as<double2>(), nk, M, M, M, M, 0, -nc, +1, 1.0, 1));
    HH_TRY(dft_pass(st, A.as<double2>(), S.as<double2>(), nk, M, M, M, M, 0, -nc, +1, 1.0, 0));
    // gS[p][q] = (1/N^2) sum_g gG[g1][g2] exp(-2 pi i (p y(g1) + q x(g2)) / N), y = N/2 - nc + g
    HH_TRY(dft_pass(st, S.as<double2>(), Bt.as<double2>(), nk, M, M, N, N, N / 2 - nc, 0, -1, 1.0, 1));
    HH_TRY(dft_pass(st, Bt.as<double2>(), S.as<double2>(), nk, N, M, N, N, N / 2 - nc, 0, -1, 1.0 / ((double)N * N), 0));
    const float* K = net->params.as<float>() + net->koff;
    hipLaunchKernelGGL(k_green_gkhat, dim3((N * N + 255) / 256, nk), dim3(256), 0, st, S.as<double2>(), K,
                       Kh.as<double2>(), N, eps);
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_green_gK, dim3(9, nk), dim3(256), 0, st, Kh.as<double2>(), gK, N);
    HH_LAUNCH_CHECK();
    HH_HIP(hipStreamSynchronize(st));  // scratch released on return
    return HH_OK;
}

// ---- loss (eq. 19) and its gradient at the projection layer --------------
// d = P(o) - e / s per fine point (s = h^2 rms(r)); loss partials sum |d|^2;
// gfull = (2 / B) d
__global__ void __launch_bounds__(256) k_loss(const float2* __restrict__ o, const float2* __restrict__ e,
                                              const float* __restrict__ s, float2* __restrict__ gfull,
                                              double* __restrict__ parts, int n, float inv_b) {
    __shared__ double s_red[4];
    const int b = blockIdx.y;
    const int m = n / 2;
    const float sc = s[b] > 0.f ? 1.f / s[b] : 0.f;
    double acc = 0.0;
    for (int p = blockIdx.x * 256 + threadIdx.x; p < n * n; p += gridDim.x * 256) {
        const int i = p / n, j = p - i * n;
        const float2* ob = o + (size_t)b * m * m;
        auto at = [&](int I, int J) -> float2 {
            return (I < m && J < m) ? ob[(size_t)I * m + J] : make_float2(0.f, 0.f);
        };
        const int I = i >> 1, J = j >> 1;
        float2 v;
        if (!(i & 1) && !(j & 1)) v = at(I, J);
        else if (!(i & 1)) v = cscale(cadd(at(I, J), at(I, J + 1)), 0.5f);
        else if (!(j & 1)) v = cscale(cadd(at(I, J), at(I + 1, J)), 0.5f);
        else v = cscale(cadd(cadd(at(I, J), at(I, J + 1)), cadd(at(I + 1, J), at(I + 1, J + 1))), 0.25f);
        const float2 t = cscale(e[(size_t)b * n * n + p], sc);
        const float2 d = csub(v, t);
        acc += (double)d.x * d.x + (double)d.y * d.y;
        gfull[(size_t)b * n * n + p] = cscale(d, 2.f * inv_b);
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) parts[(size_t)b * gridDim.x + blockIdx.x] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

// go = P^T gfull = 4 R gfull  (full weighting, zero ghosts)
__global__ void __launch_bounds__(256) k_restrict4(const float2* __restrict__ gfull, float2* __restrict__ go, int n) {
    const int b = blockIdx.y;
    const int m = n / 2;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= m * m) return;
    const int I = p / m, J = p - I * m;
    const float w1[3] = {0.25f, 0.5f, 0.25f};
    float2 acc = make_float2(0.f, 0.f);
    for (int a = 0; a < 3; ++a) {
        const int y = 2 * I + a - 1;
        if (y < 0 || y >= n) continue;
        for (int c = 0; c < 3; ++c) {
            const int x = 2 * J + c - 1;
            if (x < 0 || x >= n) continue;
            acc = cadd(acc, cscale(gfull[(size_t)b * n * n + (size_t)y * n + x], 4.f * w1[a] * w1[c]));
        }
    }
    go[(size_t)b * m * m + p] = acc;
}

// ---- elementwise: g = (g_in + add) masked by (mask > 0), BF16 -------------
__global__ void k_mask_add(const uint16_t* __restrict__ gin, const uint16_t* __restrict__ add,
                           const uint16_t* __restrict__ mask, uint16_t* __restrict__ g, size_t count) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= count) return;
    float v = bf2f(gin[e]) + (add ? bf2f(add[e]) : 0.f);
    if (!(bf2f(mask[e]) > 0.f)) v = 0.f;
    g[e] = f2bf(v);
}

// ---- Adam (Kingma & Ba), FP32 masters ------------------------------------
// global gradient norm: per-block FP64 partial sums of g^2 ...
constexpr int GN_BLOCKS = 256;  // one partial per thread of the single-block final reduction
__global__ void __launch_bounds__(256) k_grad_norm_parts(const float* __restrict__ g, size_t N,
                                                         double* __restrict__ parts) {
    __shared__ double s_red[4];
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (size_t)GN_BLOCKS * 256)
        acc += (double)g[i] * g[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) parts[blockIdx.x] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

// ... and out[0] = ||g||, out[1] = clip factor min(1, max_norm / ||g||) (1 when max_norm = 0);
// the partials sit at out + 2
__global__ void __launch_bounds__(256) k_grad_norm(double* __restrict__ out, double max_norm) {
    __shared__ double s_red[4];
    double acc = threadIdx.x < GN_BLOCKS ? out[2 + threadIdx.x] : 0.0;
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double nrm = sqrt(s_red[0] + s_red[1] + s_red[2] + s_red[3]);
        out[0] = nrm;
        out[1] = (max_norm > 0.0 && nrm > max_norm) ? max_norm / nrm : 1.0;
    }
}

// Adam on the FP32 masters with the gradient scaled by the clip factor gn[1]
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, const double* __restrict__ gn,
                       float* __restrict__ m, float* __restrict__ v, size_t N, float lr, float b1, float b2, float eps,
                       float bc1, float bc2) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const float gi = g[i] * (float)gn[1];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ---------------------------------------------------------------------------
// training step
// ---------------------------------------------------------------------------
struct TrainWork {
    NetActs acts;         // solver activations
    Buf gn;               // gradient norm, clip factor, partial sums
    Buf enc[9];           // encoder activations
    Buf G[NET_LAYERS];    // gradients w.r.t. each layer's output (pre-activation for ReLU layers)
    Buf gimp;             // gradient w.r.t. the implicit layer's output
    Buf gfull, go;        // loss gradient at full / half resolution
    Buf lparts;           // loss partials
    Buf part, part2;      // reduction scratch
    Buf gGh_part, gGh;    // implicit-layer kernel gradients
    Buf ggscratch;        // implicit-layer gradient scratch maps (transform size 128)
    Buf Gbr;              // transformed Green's functions of this step
    // the lightweight network
    LightActs lacts;
    Buf LG[LIGHT_LAYERS];   // gradients w.r.t. each layer's output
    Buf LGZ[LIGHT_LAYERS];  // ... and w.r.t. the pre-normalisation output of batch-norm layers
    Buf coef;               // batch-norm backward coefficients
};

static hh_status ensure_grads(hh_net* net, TrainWork& T, int B, int n) {
    const int ncs = coarsest_of(n);
    for (int l = 0; l < NET_LAYERS; ++l) {
        int m;
        if (l < L_S1_D) m = n >> (l / 3 + 1);
        else if (l <= L_S1_C2 || (l >= L_U1_T && l <= L_U1_C2) || l == L_OUT) m = n / 2;
        else if (l <= L_S2_C2 || (l >= L_U2_T && l <= L_U2_C2)) m = n / 4;
        else if (l <= L_S3_C2 || (l >= L_U3_T && l <= L_U3_C2)) m = n / 8;
        else m = ncs;
        if (l == L_OUT) continue;
        HH_TRY(T.G[l].ensure(net->ctx, (size_t)B * m * m * net->L[l].cout * sizeof(uint16_t)));
    }
    HH_TRY(T.gimp.ensure(net->ctx, (size_t)B * ncs * ncs * net->ch[3] * sizeof(uint16_t)));
    HH_TRY(T.gfull.ensure(net->ctx, (size_t)B * n * n * sizeof(float2)));
    HH_TRY(T.go.ensure(net->ctx, (size_t)B * (n / 2) * (n / 2) * sizeof(float2)));
    HH_TRY(T.lparts.ensure(net->ctx, (size_t)B * 64 * sizeof(double)));
    return HH_OK;
}

// dgrad of layer l: g_in = conv_l^T (gout), + add, masked by `mask`
static hh_status dgrad_layer(hh_net* net, int l, int mode, const uint16_t* gout, int B, int Hout, int Wout,
                             uint16_t* gin, int Hin, int Win, const uint16_t* add, const uint16_t* mask) {
    const LayerInfo& L = net->L[l];
    ConvArgs a{};
    a.x = gout;
    a.y = gin;
    a.wp = net->packed.as<uint16_t>() + net->pk_bwd[l];
    a.bias = nullptr;
    a.skip = add;
    a.mask = mask;
    a.act = ACT_NONE;
    a.B = B;
    a.Hin = Hout;
    a.Win = Wout;
    a.Hout = Hin;
    a.Wout = Win;
    return launch_conv(net->ctx->stream, net->ctx->num_cus, L.cout, L.cin, mode, a);
}

}  // namespace hh

using namespace hh;

// loss = sum of the per-block partials written by k_loss / (B n^2); optionally
// the gradient norm written by k_grad_norm
static hh_status read_loss(hh_ctx* ctx, const Buf& lparts, int B, int n, const Buf* gn, double* loss_out,
                           double* grad_norm_out) {
    std::vector<double> lp((size_t)B * 64);
    double g[2] = {0.0, 1.0};
    HH_HIP(hipMemcpyAsync(lp.data(), lparts.ptr, lp.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (gn) HH_HIP(hipMemcpyAsync(g, gn->ptr, sizeof(g), hipMemcpyDeviceToHost, ctx->stream));
    HH_HIP(hipStreamSynchronize(ctx->stream));
    double L = 0.0;
    for (double v : lp) L += v;
    if (loss_out) *loss_out = L / ((double)B * n * n);
    if (grad_norm_out) *grad_norm_out = g[0];
    return HH_OK;
}

// gradient of the transformed Green's functions (natural order, FP64):
// gGh[c][k] = sum_b conj(FFT(pad z_b))[k] FFT(pad gy_b)[k] / M^2, M = 2 nc,
// through per-sample partials (and, for M = 128, a scratch map per sample and channel)
static hh_status implicit_ggrad(hh_ctx* ctx, int nk, int nc, int B, const uint16_t* z, const uint16_t* gy, Buf& part,
                                Buf& scratch, double2* gGh) {
    hipStream_t st = ctx->stream;
    const int M = 2 * nc;
    HH_TRY(part.ensure(ctx, (size_t)B * nk * M * M * sizeof(float2)));
    dim3 grd(nk, B);
    if (M == 128) {
        const size_t lds = ((size_t)M * (M + 1) + M / 2) * sizeof(float2);
        HH_TRY(scratch.ensure(ctx, (size_t)B * nk * M * M * sizeof(float2)));
        static bool attr = false;
        if (!attr) {
            HH_HIP(hipFuncSetAttribute((const void*)k_implicit_ggrad_big<128, 1024>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            attr = true;
        }
        hipLaunchKernelGGL((k_implicit_ggrad_big<128, 1024>), grd, dim3(1024), lds, st, z, gy,
                           scratch.as<float2>(), part.as<float2>(), nc, nk);
    } else {
        const size_t lds = ((size_t)2 * M * (M + 1) + M / 2) * sizeof(float2);
        if (M == 32) {
            hipLaunchKernelGGL((k_implicit_ggrad<32, 256>), grd, dim3(256), lds, st, z, gy, part.as<float2>(), nc, nk);
        } else if (M == 64) {
            static bool attr = false;
            if (!attr) {
                HH_HIP(hipFuncSetAttribute((const void*)k_implicit_ggrad<64, 512>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
                attr = true;
            }
            hipLaunchKernelGGL((k_implicit_ggrad<64, 512>), grd, dim3(512), lds, st, z, gy, part.as<float2>(), nc, nk);
        } else if (M == 16) {
            hipLaunchKernelGGL((k_implicit_ggrad<16, 256>), grd, dim3(256), lds, st, z, gy, part.as<float2>(), nc, nk);
        } else {
            set_error("implicit-layer gradient: transform size %d not supported (16 .. 128)", M);
            return HH_ERR_ARG;
        }
    }
    HH_LAUNCH_CHECK();
    const int count = nk * M * M;
    hipLaunchKernelGGL(k_reduce_ggrad, dim3((count + 255) / 256), dim3(256), 0, st, part.as<float2>(), B, count, gGh);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// coarsest layer backward: gin = adjoint(T.gimp) masked by `mask` (null: none),
// and the gradient of its kernels from its input z (B maps of m4 x m4) into GR
static hh_status coarse_backward(hh_ctx* ctx, hh_net* net, TrainWork& T, int B, int m4, const uint16_t* z,
                                 const uint16_t* mask, uint16_t* gin, float* GR) {
    hipStream_t st = ctx->stream;
    const float* P = net->params.as<float>();
    const int nc = m4, M = 2 * m4;
    if (net->explicit_coarse) {
        HH_TRY(launch_explicit(st, T.gimp.as<uint16_t>(), gin, P + net->koff, m4, net->nk, B, true, nullptr,
                               mask));
        const int nblk = (m4 * m4 + EK_PIX - 1) / EK_PIX, count = net->nk * 9;
        HH_TRY(T.gGh_part.ensure(ctx, (size_t)B * nblk * count * sizeof(double2)));
        hipLaunchKernelGGL(k_explicit_kgrad, dim3(nblk, B), dim3(320), 0, st, z, T.gimp.as<uint16_t>(), m4,
                           net->nk, T.gGh_part.as<double2>());
        HH_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_explicit_kgrad_reduce, dim3((count + 255) / 256), dim3(256), 0, st,
                           T.gGh_part.as<double2>(), B * nblk, count, GR + net->koff);
        HH_LAUNCH_CHECK();
    } else {
        HH_TRY(launch_implicit(st, M, T.gimp.as<uint16_t>(), gin, T.Gbr.as<float2>(), m4, net->nk, B, true,
                               nullptr, mask));
        HH_TRY(T.gGh.ensure(ctx, (size_t)net->nk * M * M * sizeof(double2)));
        HH_TRY(implicit_ggrad(ctx, net->nk, nc, B, z, T.gimp.as<uint16_t>(), T.gGh_part, T.ggscratch,
                              T.gGh.as<double2>()));
        HH_TRY(green_backward(net, nc, T.gGh.as<double2>(), GR + net->koff, 1e-5));
    }
    return HH_OK;
}

// gradient norm and clip factor (on the device), Adam when lr > 0, and the loss
static hh_status finish_train_step(hh_ctx* ctx, hh_net* net, TrainWork& T, int B, int n, double lr,
                                   double max_grad_norm, double* loss_out, double* grad_norm_out) {
    hipStream_t st = ctx->stream;
    float* GR = net->grads.as<float>();
    HH_TRY(T.gn.ensure(ctx, (GN_BLOCKS + 2) * sizeof(double)));
    hipLaunchKernelGGL(k_grad_norm_parts, dim3(GN_BLOCKS), dim3(256), 0, st, GR, net->nparams,
                       T.gn.as<double>() + 2);
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_grad_norm, dim3(1), dim3(256), 0, st, T.gn.as<double>(), max_grad_norm);
    HH_LAUNCH_CHECK();
    // ---- Adam
    if (lr > 0.0) {
        if (!net->adam_m.ptr) {
            HH_TRY(net->adam_m.ensure(ctx, net->nparams * sizeof(float)));
            HH_TRY(net->adam_v.ensure(ctx, net->nparams * sizeof(float)));
            HH_HIP(hipMemsetAsync(net->adam_m.ptr, 0, net->nparams * sizeof(float), st));
            HH_HIP(hipMemsetAsync(net->adam_v.ptr, 0, net->nparams * sizeof(float), st));
        }
        net->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float bc1 = (float)(1.0 - pow(0.9, (double)net->step)), bc2 = (float)(1.0 - pow(0.999, (double)net->step));
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((net->nparams + 255) / 256)), dim3(256), 0, st,
                           net->params.as<float>(), GR, T.gn.as<double>(), net->adam_m.as<float>(),
                           net->adam_v.as<float>(), net->nparams, (float)lr, b1, b2, 1e-8f, bc1, bc2);
        HH_LAUNCH_CHECK();
        net->packed_valid = false;
        net->version++;
    }
    return read_loss(ctx, T.lparts, B, n, &T.gn, loss_out, grad_norm_out);
}

// The lightweight network's training step (see train_core): forward with batch
// statistics (running averages updated when lr > 0), loss, backward through
// batch norm, softplus, the inverted bottlenecks and every convolution.
static hh_status light_train_core(hh_ctx* ctx, hh_net* net, hh_model* md, TrainWork& T, int B, const void* r_dev,
                                  const void* e_dev, double lr, double max_grad_norm, double* loss_out,
                                  double* grad_norm_out, bool backward) {
    hipStream_t st = ctx->stream;
    const int n = md->lev[0].n;
    const double h = md->lev[0].h;
    const int m1 = n / 2, m2 = n / 4, m3 = n / 8, m4 = coarsest_of(n), s4 = coarse_stride_of(n);
    LightActs& A = T.lacts;
    const bool train = backward;  // the validation loss (no backward) applies the running statistics
    const bool update = backward && lr > 0.0;
    HH_TRY(light_encoder_forward(net, md, A, train, update));
    HH_TRY(A.ensure(net, B, n, train));
    const int* smap = md->ninst == 1 ? A.zeros.as<int>() : nullptr;  // sample b uses slowness model b
    HH_TRY(light_forward(net, n, h, A, B, smap, A.out(LL_ENC1_C2), A.out(LL_ENC2_C2), A.out(LL_ENC3_C2),
                         T.Gbr.as<float2>(), (const float2*)r_dev, (size_t)n * n, nullptr, 0, nullptr, nullptr,
                         train, update));
    HH_TRY(T.gfull.ensure(ctx, (size_t)B * n * n * sizeof(float2)));
    HH_TRY(T.go.ensure(ctx, (size_t)B * m1 * m1 * sizeof(float2)));
    HH_TRY(T.lparts.ensure(ctx, (size_t)B * 64 * sizeof(double)));
    const float* out_scale = A.scales.as<float>() + B;
    hipLaunchKernelGGL(k_loss, dim3(64, B), dim3(256), 0, st, A.a[LL_OUT].as<float2>(), (const float2*)e_dev,
                       out_scale, T.gfull.as<float2>(), T.lparts.as<double>(), n, (float)(1.0 / ((double)B * n * n)));
    HH_LAUNCH_CHECK();
    if (!backward) return read_loss(ctx, T.lparts, B, n, nullptr, loss_out, nullptr);
    if (md->ninst != B) {
        set_error("training with one slowness model shared by the batch is not supported");
        return HH_ERR_ARG;
    }
    if (update) {  // the running statistics changed: the folded weights are stale
        net->packed_valid = false;
        net->version++;
    }
    hipLaunchKernelGGL(k_restrict4, dim3((m1 * m1 + 255) / 256, B), dim3(256), 0, st, T.gfull.as<float2>(),
                       T.go.as<float2>(), n);
    HH_LAUNCH_CHECK();
    // gradient buffers
    for (int l = 0; l < LL_OUT; ++l) {
        const int m = light_res(l, n);
        const size_t bytes = (size_t)B * m * m * net->L[l].cout * sizeof(uint16_t);
        HH_TRY(T.LG[l].ensure(ctx, bytes));
        if (net->L[l].bn) HH_TRY(T.LGZ[l].ensure(ctx, bytes));
    }
    HH_TRY(T.gimp.ensure(ctx, (size_t)B * m4 * m4 * net->ch[3] * sizeof(uint16_t)));
    HH_TRY(net->grads.ensure(ctx, net->nparams * sizeof(float)));
    float* GR = net->grads.as<float>();
    const float* P = net->params.as<float>();
    auto o = [&](int l) { return A.out(l); };
    auto G = [&](int l) { return T.LG[l].as<uint16_t>(); };
    auto GZ = [&](int l) { return T.LGZ[l].as<uint16_t>(); };
    // ---- projection layer (its weights and 2 biases are contiguous)
    {
        const int chunk = 1024;
        const int nb = (m1 * m1 + chunk - 1) / chunk;
        const int count = 2 * 16 * 9 + 2;
        HH_TRY(T.part.ensure(ctx, (size_t)B * nb * count * sizeof(float)));
        hipLaunchKernelGGL(k_out_wgrad<16>, dim3(nb, B), dim3(256), 0, st, T.go.as<float2>(), o(LL_U1_C2),
                           T.part.as<float>(), m1, chunk);
        HH_LAUNCH_CHECK();
        HH_TRY(reduce_partials(st, T.part.as<float>(), B * nb, count, GR + net->L[LL_OUT].woff, 1.f));
        hipLaunchKernelGGL(k_out_dgrad<16>, dim3((m1 * m1 + 255) / 256, B), dim3(256), 0, st, T.go.as<float2>(),
                           P + net->L[LL_OUT].woff, nullptr, G(LL_U1_C2), m1);
        HH_LAUNCH_CHECK();
    }
    // batch norm (+ activation) backward of layer l from the gradient gout of its output, into GZ(l)
    auto bn_back = [&](int l, const uint16_t* gout, size_t npix, int act) -> hh_status {
        const LayerInfo& L = net->L[l];
        const BnGrads gr{GR + L.goff, GR + L.beoff, GR + L.rmoff, GR + L.rvoff};
        return bn_train_backward(st, ctx, T.part2, T.coef, L.cout, gout, A.z[l].as<uint16_t>(), npix, P + L.goff,
                                 A.st(l), act, gr, GZ(l));
    };
    // 3x3 conv + batch norm + softplus layer l (stride 1, size m) from the gradient gout
    // of its output: weight gradient from its input x, input gradient into gin
    auto cb_back = [&](int l, const uint16_t* gout, const uint16_t* x, int m, uint16_t* gin) -> hh_status {
        const LayerInfo& L = net->L[l];
        HH_TRY(bn_back(l, gout, (size_t)B * m * m, ACT_SOFTPLUS));
        HH_TRY(launch_wgrad(st, L.cout, L.cin, CM_S1, GZ(l), x, B, m, m, m, m, T.part, ctx, GR + L.woff));
        return dgrad_layer(net, l, CM_S1, GZ(l), B, m, m, gin, m, m, nullptr, nullptr);
    };
    // strided convolution l (bias, no normalisation; input x at mi, output at mo, gradient G(l))
    auto down_back = [&](int l, int wmode, int dmode, const uint16_t* x, int mi, int mo, uint16_t* gin,
                         const uint16_t* add) -> hh_status {
        const LayerInfo& L = net->L[l];
        HH_TRY(launch_wgrad(st, L.cout, L.cin, wmode, G(l), x, B, mo, mo, mi, mi, T.part, ctx, GR + L.woff));
        HH_TRY(launch_bgrad(st, L.cout, G(l), (size_t)B * mo * mo, T.part2, ctx, GR + L.boff));
        return dgrad_layer(net, l, dmode, G(l), B, mo, mo, gin, mi, mi, add, nullptr);
    };
    // transposed convolution l (input x at mi, output at mo)
    auto up_back = [&](int l, int mode, const uint16_t* x, int mi, int mo, uint16_t* gin) -> hh_status {
        const LayerInfo& L = net->L[l];
        HH_TRY(launch_wgrad(st, L.cin, L.cout, mode, x, G(l), B, mi, mi, mo, mo, T.part, ctx, GR + L.woff));
        HH_TRY(launch_bgrad(st, L.cout, G(l), (size_t)B * mo * mo, T.part2, ctx, GR + L.boff));
        return dgrad_layer(net, l, mode, G(l), B, mo, mo, gin, mi, mi, nullptr, nullptr);
    };
    // inverted bottleneck le .. le + 2 on input x (size m): gradient gout of its output,
    // input gradient into gin (the skip path's gout included)
    auto ib_back = [&](int le, const uint16_t* x, int m, const uint16_t* gout, uint16_t* gin) -> hh_status {
        const int lw = le + 1, ls = le + 2;
        const LayerInfo &E = net->L[le], &Dw = net->L[lw], &S = net->L[ls];
        const size_t npix = (size_t)B * m * m;
        const uint16_t* pk = net->packed.as<uint16_t>();
        HH_TRY(bn_back(ls, gout, npix, ACT_NONE));
        HH_TRY(launch_pw_wgrad(st, ctx, T.part, S.cin, S.cout, GZ(ls), o(lw), npix, GR + S.woff));
        PwArgs pa{};
        pa.npix = npix;
        pa.pix_per_b = m * m;
        pa.x = GZ(ls);
        pa.y = G(lw);
        pa.w = pk + net->pk_bwd[ls];
        HH_TRY(launch_pointwise(st, ctx->num_cus, S.cout, S.cin, pa));
        HH_TRY(bn_back(lw, G(lw), npix, ACT_SOFTPLUS));
        HH_TRY(launch_dw_wgrad(st, ctx, T.part, Dw.cout, GZ(lw), o(le), B, m, m, GR + Dw.woff));
        DwArgs da{};
        da.x = GZ(lw);
        da.y = G(le);
        da.w = P + Dw.woff;
        da.flip = 1;
        da.B = B;
        da.H = da.W = m;
        HH_TRY(launch_depthwise(st, ctx->num_cus, Dw.cout, da));
        HH_TRY(bn_back(le, G(le), npix, ACT_SOFTPLUS));
        HH_TRY(launch_pw_wgrad(st, ctx, T.part, E.cin, E.cout, GZ(le), x, npix, GR + E.woff));
        pa.x = GZ(le);
        pa.y = gin;
        pa.w = pk + net->pk_bwd[le];
        pa.res = gout;
        return launch_pointwise(st, ctx->num_cus, E.cout, E.cin, pa);
    };
    // ---- up path
    HH_TRY(cb_back(LL_U1_C2, G(LL_U1_C2), o(LL_U1_C1), m1, G(LL_U1_C1)));
    HH_TRY(cb_back(LL_U1_C1, G(LL_U1_C1), o(LL_U1_T), m1, G(LL_U1_T)));
    HH_TRY(up_back(LL_U1_T, CM_S2, o(LL_U2_C2), m2, m1, G(LL_U2_C2)));
    HH_TRY(cb_back(LL_U2_C2, G(LL_U2_C2), o(LL_U2_C1), m2, G(LL_U2_C1)));
    HH_TRY(cb_back(LL_U2_C1, G(LL_U2_C1), o(LL_U2_T), m2, G(LL_U2_T)));
    HH_TRY(up_back(LL_U2_T, CM_S2, o(LL_U3_C2), m3, m2, G(LL_U3_C2)));
    HH_TRY(cb_back(LL_U3_C2, G(LL_U3_C2), o(LL_U3_C1), m3, G(LL_U3_C1)));
    HH_TRY(cb_back(LL_U3_C1, G(LL_U3_C1), o(LL_U3_T), m3, G(LL_U3_T)));
    HH_TRY(up_back(LL_U3_T, s4 == 2 ? CM_S2 : CM_S1, A.imp.as<uint16_t>(), m4, m3, T.gimp.as<uint16_t>()));
    // ---- coarsest layer (no mask: softplus derivatives sit in the batch-norm backward)
    HH_TRY(coarse_backward(ctx, net, T, B, m4, o(LL_S4_C2), nullptr, G(LL_S4_C2), GR));
    // ---- level 4 and the down path (G of each strided layer's output is also its encoding's gradient)
    HH_TRY(cb_back(LL_S4_C2, G(LL_S4_C2), o(LL_S4_C1), m4, G(LL_S4_C1)));
    HH_TRY(cb_back(LL_S4_C1, G(LL_S4_C1), o(LL_S4_D), m4, G(LL_S4_D)));
    HH_TRY(down_back(LL_S4_D, s4 == 2 ? CM_S2 : CM_S1, s4 == 2 ? CM_T2 : CM_S1, o(LL_S3_S), m3, m4, G(LL_S3_S),
                     G(LL_U3_T)));
    HH_TRY(ib_back(LL_S3_E, o(LL_S3_D), m3, G(LL_S3_S), G(LL_S3_D)));
    HH_TRY(down_back(LL_S3_D, CM_S2, CM_T2, o(LL_S2_S), m2, m3, G(LL_S2_S), G(LL_U2_T)));
    HH_TRY(ib_back(LL_S2_E, o(LL_S2_D), m2, G(LL_S2_S), G(LL_S2_D)));
    HH_TRY(down_back(LL_S2_D, CM_S2, CM_T2, o(LL_S1_S), m1, m2, G(LL_S1_S), G(LL_U1_T)));
    HH_TRY(ib_back(LL_S1_E, o(LL_S1_D), m1, G(LL_S1_S), G(LL_S1_D)));
    const int chunk = 1024;
    const int nb = (m1 * m1 + chunk - 1) / chunk;
    const int count = 16 * 18 + 16;  // weights and biases of the 2 -> 16 layer
    HH_TRY(T.part.ensure(ctx, (size_t)B * nb * count * sizeof(float)));
    hipLaunchKernelGGL((k_in_wgrad<0, 16>), dim3(nb, B), dim3(256), 0, st, G(LL_S1_D), (const float2*)r_dev,
                       (size_t)n * n, A.scales.as<float>(), 0.f, T.part.as<float>(), n, chunk);
    HH_LAUNCH_CHECK();
    HH_TRY(reduce_partials(st, T.part.as<float>(), B * nb, count, GR + net->L[LL_S1_D].woff, 1.f));
    // ---- encoder: the encodings' gradients are G(LL_S3_D), G(LL_S2_D), G(LL_S1_D)
    HH_TRY(cb_back(LL_ENC3_C2, G(LL_S3_D), o(LL_ENC3_C1), m3, G(LL_ENC3_C1)));
    HH_TRY(cb_back(LL_ENC3_C1, G(LL_ENC3_C1), o(LL_ENC3_D), m3, G(LL_ENC3_D)));
    HH_TRY(down_back(LL_ENC3_D, CM_S2, CM_T2, o(LL_ENC2_C2), m2, m3, G(LL_ENC2_C2), G(LL_S2_D)));
    HH_TRY(cb_back(LL_ENC2_C2, G(LL_ENC2_C2), o(LL_ENC2_C1), m2, G(LL_ENC2_C1)));
    HH_TRY(cb_back(LL_ENC2_C1, G(LL_ENC2_C1), o(LL_ENC2_D), m2, G(LL_ENC2_D)));
    HH_TRY(down_back(LL_ENC2_D, CM_S2, CM_T2, o(LL_ENC1_C2), m1, m2, G(LL_ENC1_C2), G(LL_S1_D)));
    HH_TRY(cb_back(LL_ENC1_C2, G(LL_ENC1_C2), o(LL_ENC1_C1), m1, G(LL_ENC1_C1)));
    HH_TRY(cb_back(LL_ENC1_C1, G(LL_ENC1_C1), o(LL_ENC1_D), m1, G(LL_ENC1_D)));
    hipLaunchKernelGGL((k_in_wgrad<1, 16>), dim3(nb, B), dim3(256), 0, st, G(LL_ENC1_D), md->lev[0].coef.as<float2>(),
                       (size_t)n * n, nullptr, (float)(h * h), T.part.as<float>(), n, chunk);
    HH_LAUNCH_CHECK();
    HH_TRY(reduce_partials(st, T.part.as<float>(), B * nb, count, GR + net->L[LL_ENC1_D].woff, 1.f));
    return finish_train_step(ctx, net, T, B, n, lr, max_grad_norm, loss_out, grad_norm_out);
}

// forward pass and loss on B pairs; with backward set, also every gradient and
// (lr > 0) one Adam step on the gradient clipped to max_grad_norm (0 = no clip)
static hh_status train_core(hh_ctx* ctx, hh_net* net, hh_model* md, int B, const void* r_dev, const void* e_dev,
                            double lr, double max_grad_norm, double* loss_out, double* grad_norm_out,
                            bool backward) {
    HH_ARG(ctx && net && md && r_dev && e_dev, "null pointer");
    HH_ARG(net->ctx == ctx && md->ctx == ctx, "objects of another context");
    HH_ARG(B >= 1 && (md->ninst == B || md->ninst == 1), "model must hold one slowness model per sample (or one)");
    const int n = md->lev[0].n;
    HH_ARG(n % 16 == 0 && n >= 64 && n <= 1024 && (n & (n - 1)) == 0,
           "training sizes: n a power of two from 64 to 1024 (implicit-layer gradient transforms up to 128)");
    HH_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    if (!net->train_work) {
        net->train_work = new (std::nothrow) TrainWork();
        if (!net->train_work) {
            set_error("out of host memory");
            return HH_ERR_NOMEM;
        }
    }
    TrainWork& T = *reinterpret_cast<TrainWork*>(net->train_work);
    HH_TRY(net_pack(net));
    const double h = md->lev[0].h;
    const int nc = coarsest_of(n), M = 2 * nc;
    HH_TRY(T.Gbr.ensure(ctx, (size_t)net->nk * M * M * sizeof(float2)));
    if (!net->explicit_coarse) HH_TRY(green_forward(net, nc, T.Gbr.as<float2>(), 1e-5));
    if (net->light)
        return light_train_core(ctx, net, md, T, B, r_dev, e_dev, lr, max_grad_norm, loss_out, grad_norm_out,
                                backward);
    HH_TRY(encoder_forward(net, md, T.enc));
    NetActs& A = T.acts;
    HH_TRY(A.ensure(net, B, n));
    const int* smap = md->ninst == 1 ? A.zeros.as<int>() : nullptr;  // sample b uses slowness model b
    HH_TRY(net_forward_core(net, n, h, A, B, smap, T.enc[L_ENC1_C2].as<uint16_t>(), T.enc[L_ENC2_C2].as<uint16_t>(),
                            T.enc[L_ENC3_C2].as<uint16_t>(), T.Gbr.as<float2>(), (const float2*)r_dev, (size_t)n * n,
                            nullptr, 0, nullptr, nullptr, true));
    HH_TRY(ensure_grads(net, T, B, n));
    float* out_scale = A.scales.as<float>() + B;
    // ---- loss and gradient at the projection layer
    const int m1 = n / 2, m2 = n / 4, m3 = n / 8, m4 = nc;
    hipLaunchKernelGGL(k_loss, dim3(64, B), dim3(256), 0, st, A.a[L_OUT].as<float2>(), (const float2*)e_dev, out_scale,
                       T.gfull.as<float2>(), T.lparts.as<double>(), n, (float)(1.0 / ((double)B * n * n)));
    HH_LAUNCH_CHECK();
    if (!backward) return read_loss(ctx, T.lparts, B, n, nullptr, loss_out, nullptr);
    hipLaunchKernelGGL(k_restrict4, dim3((m1 * m1 + 255) / 256, B), dim3(256), 0, st, T.gfull.as<float2>(),
                       T.go.as<float2>(), n);
    HH_LAUNCH_CHECK();
    HH_TRY(net->grads.ensure(ctx, net->nparams * sizeof(float)));
    float* GR = net->grads.as<float>();
    const float* P = net->params.as<float>();
    auto act = [&](int l) { return A.a[l].as<uint16_t>(); };
    auto G = [&](int l) { return T.G[l].as<uint16_t>(); };
    auto enc = [&](int l) { return T.enc[l].as<uint16_t>(); };
    // ---- projection layer
    {
        const int chunk = 1024;
        const int nb = (m1 * m1 + chunk - 1) / chunk;
        const int count = 2 * 16 * 9 + 2;
        HH_TRY(T.part.ensure(ctx, (size_t)B * nb * count * sizeof(float)));
        hipLaunchKernelGGL(k_out_wgrad<16>, dim3(nb, B), dim3(256), 0, st, T.go.as<float2>(), act(L_U1_C2),
                           T.part.as<float>(), m1, chunk);
        HH_LAUNCH_CHECK();
        // the weights and the 2 biases are contiguous
        HH_TRY(reduce_partials(st, T.part.as<float>(), B * nb, count, GR + net->L[L_OUT].woff, 1.f));
        hipLaunchKernelGGL(k_out_dgrad<16>, dim3((m1 * m1 + 255) / 256, B), dim3(256), 0, st, T.go.as<float2>(),
                           P + net->L[L_OUT].woff, act(L_U1_C2), G(L_U1_C2), m1);
        HH_LAUNCH_CHECK();
    }
    // generic helpers for a 16/32/64-channel layer l whose pre-activation gradient is G(l)
    auto wgrad_conv = [&](int l, int mode, const uint16_t* x, int Hin, int Win, int Hout, int Wout) -> hh_status {
        const LayerInfo& L = net->L[l];
        HH_TRY(launch_wgrad(st, L.cout, L.cin, mode, G(l), x, B, Hout, Wout, Hin, Win, T.part, ctx, GR + L.woff));
        return launch_bgrad(st, L.cout, G(l), (size_t)B * Hout * Wout, T.part2, ctx, GR + L.boff);
    };
    // transposed convolution l (input x at Hin, output gradient G(l) at Hout): dW (cin, cout)
    auto wgrad_convT = [&](int l, int mode, const uint16_t* x, int Hin, int Hout) -> hh_status {
        const LayerInfo& L = net->L[l];
        HH_TRY(launch_wgrad(st, L.cin, L.cout, mode, x, G(l), B, Hin, Hin, Hout, Hout, T.part, ctx, GR + L.woff));
        return launch_bgrad(st, L.cout, G(l), (size_t)B * Hout * Hout, T.part2, ctx, GR + L.boff);
    };
    const int s4 = coarse_stride_of(n);
    // ---- up path, level 1
    HH_TRY(wgrad_conv(L_U1_C2, CM_S1, act(L_U1_C1), m1, m1, m1, m1));
    HH_TRY(dgrad_layer(net, L_U1_C2, CM_S1, G(L_U1_C2), B, m1, m1, G(L_U1_C1), m1, m1, nullptr, act(L_U1_C1)));
    HH_TRY(wgrad_conv(L_U1_C1, CM_S1, act(L_U1_T), m1, m1, m1, m1));
    HH_TRY(dgrad_layer(net, L_U1_C1, CM_S1, G(L_U1_C1), B, m1, m1, G(L_U1_T), m1, m1, nullptr, nullptr));
    HH_TRY(wgrad_convT(L_U1_T, CM_S2, act(L_U2_C2), m2, m1));
    HH_TRY(dgrad_layer(net, L_U1_T, CM_S2, G(L_U1_T), B, m1, m1, G(L_U2_C2), m2, m2, nullptr, act(L_U2_C2)));
    // ---- up path, level 2
    HH_TRY(wgrad_conv(L_U2_C2, CM_S1, act(L_U2_C1), m2, m2, m2, m2));
    HH_TRY(dgrad_layer(net, L_U2_C2, CM_S1, G(L_U2_C2), B, m2, m2, G(L_U2_C1), m2, m2, nullptr, act(L_U2_C1)));
    HH_TRY(wgrad_conv(L_U2_C1, CM_S1, act(L_U2_T), m2, m2, m2, m2));
    HH_TRY(dgrad_layer(net, L_U2_C1, CM_S1, G(L_U2_C1), B, m2, m2, G(L_U2_T), m2, m2, nullptr, nullptr));
    HH_TRY(wgrad_convT(L_U2_T, CM_S2, act(L_U3_C2), m3, m2));
    HH_TRY(dgrad_layer(net, L_U2_T, CM_S2, G(L_U2_T), B, m2, m2, G(L_U3_C2), m3, m3, nullptr, act(L_U3_C2)));
    // ---- up path, level 3
    HH_TRY(wgrad_conv(L_U3_C2, CM_S1, act(L_U3_C1), m3, m3, m3, m3));
    HH_TRY(dgrad_layer(net, L_U3_C2, CM_S1, G(L_U3_C2), B, m3, m3, G(L_U3_C1), m3, m3, nullptr, act(L_U3_C1)));
    HH_TRY(wgrad_conv(L_U3_C1, CM_S1, act(L_U3_T), m3, m3, m3, m3));
    HH_TRY(dgrad_layer(net, L_U3_C1, CM_S1, G(L_U3_C1), B, m3, m3, G(L_U3_T), m3, m3, nullptr, nullptr));
    HH_TRY(wgrad_convT(L_U3_T, s4 == 2 ? CM_S2 : CM_S1, A.imp.as<uint16_t>(), m4, m3));
    HH_TRY(dgrad_layer(net, L_U3_T, s4 == 2 ? CM_S2 : CM_S1, G(L_U3_T), B, m3, m3, T.gimp.as<uint16_t>(), m4, m4,
                       nullptr, nullptr));
    HH_TRY(coarse_backward(ctx, net, T, B, m4, act(L_S4_C2), act(L_S4_C2), G(L_S4_C2), GR));
    // ---- down path, level 4
    HH_TRY(wgrad_conv(L_S4_C2, CM_S1, act(L_S4_C1), m4, m4, m4, m4));
    HH_TRY(dgrad_layer(net, L_S4_C2, CM_S1, G(L_S4_C2), B, m4, m4, G(L_S4_C1), m4, m4, nullptr, act(L_S4_C1)));
    HH_TRY(wgrad_conv(L_S4_C1, CM_S1, act(L_S4_D), m4, m4, m4, m4));
    HH_TRY(dgrad_layer(net, L_S4_C1, CM_S1, G(L_S4_C1), B, m4, m4, G(L_S4_D), m4, m4, nullptr, nullptr));
    HH_TRY(wgrad_conv(L_S4_D, s4 == 2 ? CM_S2 : CM_S1, act(L_S3_C2), m3, m3, m4, m4));
    HH_TRY(dgrad_layer(net, L_S4_D, s4 == 2 ? CM_T2 : CM_S1, G(L_S4_D), B, m4, m4, G(L_S3_C2), m3, m3, G(L_U3_T),
                       act(L_S3_C2)));
    // ---- down path, levels 3 .. 1 (G(L_Sk_D) is also the gradient of the encodings Ek)
    const int lvl_d[3] = {L_S3_D, L_S2_D, L_S1_D};
    const int lvl_m[3] = {m3, m2, m1};
    const int up_t[3] = {L_U2_T, L_U1_T, -1};
    for (int k = 0; k < 3; ++k) {
        const int ld = lvl_d[k], mm = lvl_m[k];
        HH_TRY(wgrad_conv(ld + 2, CM_S1, act(ld + 1), mm, mm, mm, mm));
        HH_TRY(dgrad_layer(net, ld + 2, CM_S1, G(ld + 2), B, mm, mm, G(ld + 1), mm, mm, nullptr, act(ld + 1)));
        HH_TRY(wgrad_conv(ld + 1, CM_S1, act(ld), mm, mm, mm, mm));
        HH_TRY(dgrad_layer(net, ld + 1, CM_S1, G(ld + 1), B, mm, mm, G(ld), mm, mm, nullptr, nullptr));
        if (k < 2) {
            HH_TRY(wgrad_conv(ld, CM_S2, act(ld - 1), 2 * mm, 2 * mm, mm, mm));
            HH_TRY(dgrad_layer(net, ld, CM_T2, G(ld), B, mm, mm, G(ld - 1), 2 * mm, 2 * mm, G(up_t[k]),
                               act(ld - 1)));
        }
    }
    {   // first solver layer (2 -> 16, stride 2) from the scaled residual
        const int chunk = 1024;
        const int nb = (m1 * m1 + chunk - 1) / chunk;
        const int count = 16 * 18 + 16;
        HH_TRY(T.part.ensure(ctx, (size_t)B * nb * count * sizeof(float)));
        hipLaunchKernelGGL((k_in_wgrad<0, 16>), dim3(nb, B), dim3(256), 0, st, G(L_S1_D), (const float2*)r_dev,
                           (size_t)n * n, A.scales.as<float>(), 0.f, T.part.as<float>(), n, chunk);
        HH_LAUNCH_CHECK();
        HH_TRY(reduce_partials(st, T.part.as<float>(), B * nb, count, GR + net->L[L_S1_D].woff, 1.f));
    }
    // ---- encoder (the encodings' gradients are G(L_S1_D), G(L_S2_D), G(L_S3_D))
    {
        const int EB = md->ninst;
        if (EB != B) {
            set_error("training with one slowness model shared by the batch is not supported");
            return HH_ERR_ARG;
        }
        const int lvl_c2[3] = {L_ENC3_C2, L_ENC2_C2, L_ENC1_C2};
        const int lvl_gs[3] = {L_S3_D, L_S2_D, L_S1_D};
        for (int k = 0; k < 3; ++k) {
            const int l2 = lvl_c2[k], mm = lvl_m[k];
            const size_t cnt = (size_t)B * mm * mm * net->L[l2].cout;
            if (k == 0) {
                hipLaunchKernelGGL(k_mask_add, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, G(lvl_gs[k]),
                                   nullptr, enc(l2), G(l2), cnt);
                HH_LAUNCH_CHECK();
            }
            HH_TRY(wgrad_conv(l2, CM_S1, enc(l2 - 1), mm, mm, mm, mm));
            HH_TRY(dgrad_layer(net, l2, CM_S1, G(l2), B, mm, mm, G(l2 - 1), mm, mm, nullptr, enc(l2 - 1)));
            HH_TRY(wgrad_conv(l2 - 1, CM_S1, enc(l2 - 2), mm, mm, mm, mm));
            HH_TRY(dgrad_layer(net, l2 - 1, CM_S1, G(l2 - 1), B, mm, mm, G(l2 - 2), mm, mm, nullptr, nullptr));
            if (k < 2) {
                // strided conv of this level: input E_{k-1} (at 2 mm); its gradient adds the solver's
                HH_TRY(wgrad_conv(l2 - 2, CM_S2, enc(l2 - 3), 2 * mm, 2 * mm, mm, mm));
                HH_TRY(dgrad_layer(net, l2 - 2, CM_T2, G(l2 - 2), B, mm, mm, G(l2 - 3), 2 * mm, 2 * mm,
                                   G(lvl_gs[k + 1]), enc(l2 - 3)));
            }
        }
        const int chunk = 1024;
        const int nb = (m1 * m1 + chunk - 1) / chunk;
        const int count = 16 * 18 + 16;
        HH_TRY(T.part.ensure(ctx, (size_t)B * nb * count * sizeof(float)));
        hipLaunchKernelGGL((k_in_wgrad<1, 16>), dim3(nb, B), dim3(256), 0, st, G(L_ENC1_D),
                           md->lev[0].coef.as<float2>(), (size_t)n * n, nullptr, (float)(h * h), T.part.as<float>(), n,
                           chunk);
        HH_LAUNCH_CHECK();
        HH_TRY(reduce_partials(st, T.part.as<float>(), B * nb, count, GR + net->L[L_ENC1_D].woff, 1.f));
    }
    return finish_train_step(ctx, net, T, B, n, lr, max_grad_norm, loss_out, grad_norm_out);
}

extern "C" hh_status hh_train_step(hh_ctx* ctx, hh_net* net, hh_model* md, int B, const void* r_dev,
                                   const void* e_dev, double lr, double max_grad_norm, double* loss_out,
                                   double* grad_norm_out) {
    HH_ARG(max_grad_norm >= 0.0, "max_grad_norm >= 0");
    return train_core(ctx, net, md, B, r_dev, e_dev, lr, max_grad_norm, loss_out, grad_norm_out, true);
}

extern "C" hh_status hh_eval_loss(hh_ctx* ctx, hh_net* net, hh_model* md, int B, const void* r_dev,
                                  const void* e_dev, double* loss_out) {
    return train_core(ctx, net, md, B, r_dev, e_dev, 0.0, 0.0, loss_out, nullptr, false);
}

// e = x - xt (xt complex double), single precision
__global__ void k_err_pair(const float2* __restrict__ x, const double2* __restrict__ xt, float2* __restrict__ e,
                           size_t count) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const float2 a = x[i];
    const double2 b = xt[i];
    e[i] = make_float2((float)((double)a.x - b.x), (float)((double)a.y - b.y));
}

extern "C" hh_status hh_gen_training_pairs(hh_ctx* ctx, hh_model* m, int nb, const void* x_dev, const int* kiters_host,
                                           void* e_dev, void* r_dev) {
    HH_ARG(ctx && m && x_dev && kiters_host && e_dev && r_dev, "null pointer");
    HH_ARG(m->ctx == ctx, "model of another context");
    HH_ARG(nb >= 1 && (m->ninst == nb || m->ninst == 1), "one slowness model per sample (or one)");
    int kmax = 0;
    for (int b = 0; b < nb; ++b) {
        HH_ARG(kiters_host[b] >= 1 && kiters_host[b] <= HH_MAX_RESTART, "iterations per sample in 1..HH_MAX_RESTART");
        kmax = std::max(kmax, kiters_host[b]);
    }
    HH_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int n = m->lev[0].n;
    const size_t nn = (size_t)n * n;
    Buf ib, bb, xt, caps;
    BatchMap bm;
    std::vector<int> ident(nb);
    for (int b = 0; b < nb; ++b) ident[b] = m->ninst == 1 ? 0 : b;
    HH_TRY(upload_inst_map(m, ib, nb, ident.data(), &bm));
    HH_TRY(bb.ensure(ctx, (size_t)nb * nn * sizeof(float2)));
    HH_TRY(xt.ensure(ctx, (size_t)nb * nn * sizeof(double2)));
    HH_TRY(caps.ensure(ctx, (size_t)nb * sizeof(int)));
    HH_HIP(hipMemcpyAsync(caps.ptr, kiters_host, (size_t)nb * sizeof(int), hipMemcpyHostToDevice, st));
    // b = A x (training operator of the model), x~ = k FGMRES-MG iterations from 0 (eq. 20)
    HH_TRY(launch_apply_op(m, 0, 0.f, nb, bm.inst, (const float2*)x_dev, bb.as<float2>(), nullptr));
    if (!ctx->work) {
        ctx->work = new (std::nothrow) SolveWork();
        if (!ctx->work) {
            set_error("out of host memory");
            return HH_ERR_NOMEM;
        }
    }
    SolveWork& W = *ctx->work;
    hh_solve_opts o;
    hh_solve_opts_default(&o);
    o.fixed_iters = kmax;
    o.restart = std::max(kmax, 1);
    HH_TRY(W.prepare(ctx, m, nb, o.restart, kmax + 1, false));
    W.caps_dev = caps.as<int>();
    hh_status s = fgmres_solve(m, W, bm, bb.as<float2>(), xt.as<double2>(), o, nullptr, nullptr);
    W.caps_dev = nullptr;
    if (s < 0) return s;
    HH_TRY(coarse_check_err(m));
    // e = x - x~, r = A e
    hipLaunchKernelGGL(k_err_pair, dim3((unsigned)(((size_t)nb * nn + 255) / 256)), dim3(256), 0, st,
                       (const float2*)x_dev, xt.as<double2>(), (float2*)e_dev, (size_t)nb * nn);
    HH_LAUNCH_CHECK();
    HH_TRY(launch_apply_op(m, 0, 0.f, nb, bm.inst, (const float2*)e_dev, (float2*)r_dev, nullptr));
    HH_HIP(hipStreamSynchronize(st));
    return HH_OK;
}

hh_net::~hh_net() { delete reinterpret_cast<hh::TrainWork*>(train_work); }

extern "C" hh_status hh_net_get_grads(hh_net* net, float* host) {
    HH_ARG(net && host, "null pointer");
    HH_ARG(net->grads.ptr, "no gradients computed yet");
    HH_HIP(hipStreamSynchronize(net->ctx->stream));
    HH_HIP(hipMemcpy(host, net->grads.ptr, net->nparams * sizeof(float), hipMemcpyDeviceToHost));
    return HH_OK;
}

namespace hh {

}  // namespace hh

using namespace hh;

extern "C" {

static bool valid_channels(const int* ch) { return ch[0] == 16 && ch[1] == 32 && ch[2] == 64 && ch[3] == 64; }

hh_status hh_net_create(hh_ctx* ctx, const hh_net_desc* d, const float* params_host, hh_net** out) {
    HH_ARG(ctx && d && out, "null pointer");
    *out = nullptr;
    HH_ARG(valid_channels(d->ch), "channels must be (16, 32, 64, 64)");
    HH_ARG(d->explicit_coarse == 0 || d->explicit_coarse == 1, "explicit_coarse is 0 or 1");
    HH_ARG(d->arch == HH_ARCH_UNET || d->arch == HH_ARCH_LIGHT, "arch is HH_ARCH_UNET or HH_ARCH_LIGHT");
    HH_HIP(hipSetDevice(ctx->device));
    hh_net* net = new (std::nothrow) hh_net();
    if (!net) {
        set_error("out of host memory");
        return HH_ERR_NOMEM;
    }
    net->ctx = ctx;
    {
        static std::atomic<unsigned long long> next_uid{1};
        net->uid = next_uid.fetch_add(1);
    }
    for (int i = 0; i < 4; ++i) net->ch[i] = d->ch[i];
    net->explicit_coarse = d->explicit_coarse ? 1 : 0;
    net->light = d->arch == HH_ARCH_LIGHT ? 1 : 0;
    if (net->light)
        build_light_table(net);
    else
        build_table(net);
    hh_status s = net->params.ensure(ctx, net->nparams * sizeof(float));
    if (s >= 0 && params_host) {
        if (hipMemcpy(net->params.ptr, params_host, net->nparams * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
            set_error("copying the parameters failed");
            s = HH_ERR_HIP;
        }
    } else if (s >= 0) {
        if (hipMemset(net->params.ptr, 0, net->nparams * sizeof(float)) != hipSuccess) s = HH_ERR_HIP;
    }
    if (s < 0) {
        delete net;
        return s;
    }
    *out = net;
    return HH_OK;
}

size_t hh_net_num_params(const hh_net* net) { return net ? net->nparams : 0; }

hh_status hh_net_get_params(hh_net* net, float* host) {
    HH_ARG(net && host, "null pointer");
    HH_HIP(hipStreamSynchronize(net->ctx->stream));
    HH_HIP(hipMemcpy(host, net->params.ptr, net->nparams * sizeof(float), hipMemcpyDeviceToHost));
    return HH_OK;
}

hh_status hh_net_set_params(hh_net* net, const float* host) {
    HH_ARG(net && host, "null pointer");
    HH_HIP(hipStreamSynchronize(net->ctx->stream));
    HH_HIP(hipMemcpy(net->params.ptr, host, net->nparams * sizeof(float), hipMemcpyHostToDevice));
    net->packed_valid = false;
    net->version++;
    return HH_OK;
}

hh_status hh_net_destroy(hh_net* net) {
    if (!net) return HH_OK;
    (void)hipStreamSynchronize(net->ctx->stream);
    delete net;
    return HH_OK;
}

// file format 1: no coarsest-layer kind (implicit); 2: an int of flags after the
// channels, bit 0 the explicit coarsest layer, bit 1 the lightweight network
static const char kMagic[8] = {'H', 'H', 'N', 'E', 'T', '0', '0', '2'};
static const char kMagic1[8] = {'H', 'H', 'N', 'E', 'T', '0', '0', '1'};

hh_status hh_net_save(hh_net* net, const char* path) {
    HH_ARG(net && path, "null pointer");
    std::vector<float> p(net->nparams), m, v;
    HH_TRY(hh_net_get_params(net, p.data()));
    const int have_adam = net->adam_m.ptr && net->adam_v.ptr ? 1 : 0;
    if (have_adam) {
        m.resize(net->nparams);
        v.resize(net->nparams);
        HH_HIP(hipMemcpy(m.data(), net->adam_m.ptr, net->nparams * sizeof(float), hipMemcpyDeviceToHost));
        HH_HIP(hipMemcpy(v.data(), net->adam_v.ptr, net->nparams * sizeof(float), hipMemcpyDeviceToHost));
    }
    FILE* f = fopen(path, "wb");
    if (!f) {
        set_error("cannot open %s for writing", path);
        return HH_ERR_ARG;
    }
    const long long np = (long long)net->nparams, step = net->step;
    const int flags = net->explicit_coarse | (net->light << 1);
    bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(net->ch, sizeof(int), 4, f) == 4 &&
              fwrite(&flags, sizeof(int), 1, f) == 1 && fwrite(&np, sizeof(np), 1, f) == 1 && fwrite(&step, sizeof(step), 1, f) == 1 &&
              fwrite(&have_adam, sizeof(int), 1, f) == 1 && fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
    if (ok && have_adam)
        ok = fwrite(m.data(), sizeof(float), m.size(), f) == m.size() &&
             fwrite(v.data(), sizeof(float), v.size(), f) == v.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok) {
        set_error("writing %s failed", path);
        return HH_ERR_ARG;
    }
    return HH_OK;
}

hh_status hh_net_load(hh_ctx* ctx, const char* path, hh_net** out) {
    HH_ARG(ctx && path && out, "null pointer");
    *out = nullptr;
    FILE* f = fopen(path, "rb");
    if (!f) {
        set_error("cannot open %s", path);
        return HH_ERR_ARG;
    }
    char magic[8];
    hh_net_desc d;
    long long np = 0, step = 0;
    int have_adam = 0;
    int flags = 0;
    bool ok = fread(magic, 1, 8, f) == 8 && (memcmp(magic, kMagic, 8) == 0 || memcmp(magic, kMagic1, 8) == 0) &&
              fread(d.ch, sizeof(int), 4, f) == 4;
    if (ok && memcmp(magic, kMagic, 8) == 0) ok = fread(&flags, sizeof(int), 1, f) == 1 && flags >= 0 && flags <= 3;
    d.explicit_coarse = flags & 1;
    d.arch = (flags >> 1) & 1 ? HH_ARCH_LIGHT : HH_ARCH_UNET;
    ok = ok && fread(&np, sizeof(np), 1, f) == 1 && fread(&step, sizeof(step), 1, f) == 1 &&
         fread(&have_adam, sizeof(int), 1, f) == 1;
    std::vector<float> p, m, v;
    if (ok && np > 0 && np < (1LL << 30)) {
        p.resize((size_t)np);
        ok = fread(p.data(), sizeof(float), p.size(), f) == p.size();
        if (ok && have_adam) {
            m.resize((size_t)np);
            v.resize((size_t)np);
            ok = fread(m.data(), sizeof(float), m.size(), f) == m.size() &&
                 fread(v.data(), sizeof(float), v.size(), f) == v.size();
        }
    } else {
        ok = false;
    }
    fclose(f);
    if (!ok) {
        set_error("%s is not a valid network file", path);
        return HH_ERR_ARG;
    }
    hh_net* net = nullptr;
    HH_TRY(hh_net_create(ctx, &d, p.data(), &net));
    if ((long long)net->nparams != np) {
        hh_net_destroy(net);
        set_error("%s: parameter count mismatch", path);
        return HH_ERR_ARG;
    }
    net->step = step;
    if (have_adam) {
        hh_status s = net->adam_m.ensure(ctx, (size_t)np * sizeof(float));
        if (s >= 0) s = net->adam_v.ensure(ctx, (size_t)np * sizeof(float));
        if (s < 0 || hipMemcpy(net->adam_m.ptr, m.data(), (size_t)np * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(net->adam_v.ptr, v.data(), (size_t)np * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
            hh_net_destroy(net);
            set_error("restoring the optimizer state failed");
            return HH_ERR_HIP;
        }
    }
    *out = net;
    return HH_OK;
}

hh_status hh_model_attach_net(hh_model* m, hh_net* net) {
    HH_ARG(m, "null pointer");
    HH_ARG(!net || net->ctx == m->ctx, "network belongs to another context");
    m->net = net;
    if (!net) return HH_OK;
    HH_HIP(hipSetDevice(m->ctx->device));
    HH_TRY(net_prepare_model(m));
    HH_HIP(hipStreamSynchronize(m->ctx->stream));
    return HH_OK;
}

hh_status hh_net_forward(hh_model* m, int nrhs, const int* inst_host, const void* r_dev, void* e_dev) {
    HH_ARG(m && r_dev && e_dev, "null pointer");
    HH_ARG(m->net, "no network attached to the model");
    HH_ARG(nrhs >= 1, "nrhs >= 1");
    HH_HIP(hipSetDevice(m->ctx->device));
    HH_TRY(net_prepare_model(m));
    Buf ib;
    BatchMap bm;
    HH_TRY(upload_inst_map(m, ib, nrhs, inst_host, &bm));
    const size_t nn = (size_t)m->lev[0].n * m->lev[0].n;
    HH_TRY(net_forward_model(m->net, m, nrhs, bm, (const float2*)r_dev, nn, nullptr, 0, (float2*)e_dev, nullptr));
    HH_HIP(hipStreamSynchronize(m->ctx->stream));
    return HH_OK;
}

hh_status hh_apply_cnn_precond(hh_model* m, int nrhs, const int* inst_host, const void* v_dev, void* z_dev) {
    HH_ARG(m && v_dev && z_dev, "null pointer");
    HH_ARG(m->net, "no network attached to the model");
    HH_ARG(nrhs >= 1, "nrhs >= 1");
    HH_HIP(hipSetDevice(m->ctx->device));
    HH_TRY(net_prepare_model(m));
    Buf ib, work;
    BatchMap bm;
    HH_TRY(upload_inst_map(m, ib, nrhs, inst_host, &bm));
    HH_TRY(work.ensure(m->ctx, vcycle_workspace_bytes(m, nrhs, false) + 256));
    NetCache* nc = reinterpret_cast<NetCache*>(m->netcache);
    const size_t nn = (size_t)m->lev[0].n * m->lev[0].n;
    const float2* v = (const float2*)v_dev;
    HH_TRY(net_forward_model(m->net, m, nrhs, bm, v, nn, nullptr, 0, nullptr, nullptr));
    HH_TRY(launch_vcycle_strided(m, nrhs, bm, v, nn, nullptr, 0, nullptr, 0, (float2*)z_dev, nn, work.ptr, nullptr,
                                 net_out_of(nc, m->net), net_out_scale_of(nc, m->net, nrhs)));
    HH_HIP(hipStreamSynchronize(m->ctx->stream));
    return coarse_check_err(m);
}

hh_status hh_conv_test(hh_ctx* ctx, int cin, int cout, int mode, int B, int Hin, int Win, const void* x_dev,
                       const float* w_dev, int flipped, const float* bias_dev, const void* skip_dev, int act,
                       void* y_dev, float* yf_dev, const int* active_host, int variant) {
    HH_ARG(ctx && x_dev && w_dev && y_dev, "null pointer");
    HH_ARG(mode >= 0 && mode <= 2, "mode");
    HH_ARG(B >= 1 && Hin >= 1 && Win >= 1, "sizes");
    HH_HIP(hipSetDevice(ctx->device));
    Buf wp, actb;
    HH_TRY(wp.ensure(ctx, packed_weight_elems(cin, cout) * sizeof(uint16_t) + 256));
    HH_TRY(pack_weights(ctx->stream, w_dev, wp.as<uint16_t>(), cin, cout, flipped != 0));
    if (active_host) {
        HH_TRY(actb.ensure(ctx, (size_t)B * sizeof(int)));
        HH_HIP(hipMemcpyAsync(actb.ptr, active_host, (size_t)B * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    }
    ConvArgs a{};
    a.x = (const uint16_t*)x_dev;
    a.y = (uint16_t*)y_dev;
    a.yf = yf_dev;
    a.wp = wp.as<uint16_t>();
    a.bias = bias_dev;
    a.skip = (const uint16_t*)skip_dev;
    a.act = act;
    a.B = B;
    a.Hin = Hin;
    a.Win = Win;
    a.Hout = mode == CM_S2 ? Hin / 2 : (mode == CM_T2 ? 2 * Hin : Hin);
    a.Wout = mode == CM_S2 ? Win / 2 : (mode == CM_T2 ? 2 * Win : Win);
    a.active = actb.as<int>();
    HH_TRY(launch_conv(ctx->stream, ctx->num_cus, cin, cout, mode, a, variant));
    HH_HIP(hipStreamSynchronize(ctx->stream));
    return HH_OK;
}

hh_status hh_conv_pair_test(hh_ctx* ctx, int B, int H, int W, const void* x_dev, const float* w1_dev,
                            const float* b1_dev, const float* w2_dev, const float* b2_dev, void* mid_dev, void* y_dev,
                            const int* active_host, int variant) {
    HH_ARG(ctx && x_dev && w1_dev && w2_dev && mid_dev && y_dev, "null pointer");
    HH_ARG(B >= 1 && H >= 1 && W >= 1, "sizes");
    HH_HIP(hipSetDevice(ctx->device));
    const size_t pe = packed_weight_elems(16, 16);
    Buf wp, actb;
    HH_TRY(wp.ensure(ctx, 2 * pe * sizeof(uint16_t) + 256));
    HH_TRY(pack_weights(ctx->stream, w1_dev, wp.as<uint16_t>(), 16, 16, false));
    HH_TRY(pack_weights(ctx->stream, w2_dev, wp.as<uint16_t>() + pe, 16, 16, false));
    if (active_host) {
        HH_TRY(actb.ensure(ctx, (size_t)B * sizeof(int)));
        HH_HIP(hipMemcpyAsync(actb.ptr, active_host, (size_t)B * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    }
    ConvArgs a{};
    a.x = (const uint16_t*)x_dev;
    a.y = (uint16_t*)y_dev;
    a.ymid = (uint16_t*)mid_dev;
    a.wp = wp.as<uint16_t>();
    a.bias = b1_dev;
    a.wp2 = wp.as<uint16_t>() + pe;
    a.bias2 = b2_dev;
    a.act = ACT_RELU;
    a.B = B;
    a.Hin = a.Hout = H;
    a.Win = a.Wout = W;
    a.active = actb.as<int>();
    HH_TRY(launch_conv(ctx->stream, ctx->num_cus, 16, 16, CM_PAIR, a, variant));
    HH_HIP(hipStreamSynchronize(ctx->stream));
    return HH_OK;
}

hh_status hh_wgrad_test(hh_ctx* ctx, int ca, int cx, int mode, int B, int Ho, int Wo, int Hi, int Wi,
                        const void* a_dev, const void* x_dev, float* out_dev) {
    HH_ARG(ctx && a_dev && x_dev && out_dev, "null pointer");
    HH_ARG(mode == CM_S1 || mode == CM_S2, "mode");
    HH_ARG(B > 0 && Ho > 0 && Wo > 0 && Hi > 0 && Wi > 0, "sizes");
    HH_ARG(mode == CM_S1 ? (Hi == Ho && Wi == Wo) : (Hi == 2 * Ho && Wi == 2 * Wo), "input/output sizes");
    HH_HIP(hipSetDevice(ctx->device));
    Buf part;
    HH_TRY(launch_wgrad(ctx->stream, ca, cx, mode, (const uint16_t*)a_dev, (const uint16_t*)x_dev, B, Ho, Wo, Hi, Wi,
                        part, ctx, out_dev));
    HH_HIP(hipStreamSynchronize(ctx->stream));
    return HH_OK;
}

int hh_conv_variants(int cin, int cout, int mode, int* codes, int max) {
    return codes ? conv_variant_list(cin, cout, mode, codes, max) : conv_variant_list(cin, cout, mode, nullptr, 0);
}

int hh_conv_tuned_variant(int device, int cin, int cout, int mode, int Hout, int Wout, int B) {
    return conv_tuned_variant(device, cin, cout, mode, Hout, Wout, B);
}

hh_status hh_conv_force_variant(int cin, int cout, int mode, int code) {
    return conv_force_variant(cin, cout, mode, code);
}

hh_status hh_pointwise_test(hh_ctx* ctx, int cin, int cout, size_t npix, const void* x_dev, const float* w_dev,
                            const float* bias_dev, const void* res_dev, int act, void* y_dev, float* yf_dev) {
    HH_ARG(ctx && x_dev && w_dev && y_dev, "null pointer");
    HH_ARG(act == ACT_NONE || act == ACT_SOFTPLUS, "act is 0 or 2");
    HH_HIP(hipSetDevice(ctx->device));
    Buf wp;
    HH_TRY(wp.ensure(ctx, (size_t)cin * cout * sizeof(uint16_t)));
    HH_TRY(pack_pointwise(ctx->stream, w_dev, wp.as<uint16_t>(), cout, cin, false));
    PwArgs a{};
    a.x = (const uint16_t*)x_dev;
    a.y = (uint16_t*)y_dev;
    a.yf = yf_dev;
    a.w = wp.as<uint16_t>();
    a.bias = bias_dev;
    a.res = (const uint16_t*)res_dev;
    a.act = act;
    a.npix = npix;
    HH_TRY(launch_pointwise(ctx->stream, ctx->num_cus, cin, cout, a));
    HH_HIP(hipStreamSynchronize(ctx->stream));
    return HH_OK;
}

hh_status hh_depthwise_test(hh_ctx* ctx, int C, int B, int H, int W, const void* x_dev, const float* w_dev,
                            const float* bias_dev, int act, int flip, void* y_dev, float* yf_dev) {
    HH_ARG(ctx && x_dev && w_dev && y_dev, "null pointer");
    HH_ARG(act == ACT_NONE || act == ACT_SOFTPLUS, "act is 0 or 2");
    HH_ARG(B >= 1 && H >= 1 && W >= 1, "sizes");
    HH_HIP(hipSetDevice(ctx->device));
    DwArgs a{};
    a.x = (const uint16_t*)x_dev;
    a.y = (uint16_t*)y_dev;
    a.yf = yf_dev;
    a.w = w_dev;
    a.bias = bias_dev;
    a.act = act;
    a.flip = flip ? 1 : 0;
    a.B = B;
    a.H = H;
    a.W = W;
    HH_TRY(launch_depthwise(ctx->stream, ctx->num_cus, C, a));
    HH_HIP(hipStreamSynchronize(ctx->stream));
    return HH_OK;
}

hh_status hh_implicit_ggrad_test(hh_ctx* ctx, int nk, int nc, int B, const void* z_dev, const void* gy_dev,
                                 void* out_dev) {
    HH_ARG(ctx && z_dev && gy_dev && out_dev, "null pointer");
    HH_ARG(nk >= 1 && B >= 1, "sizes");
    HH_HIP(hipSetDevice(ctx->device));
    Buf part, scratch;
    HH_TRY(implicit_ggrad(ctx, nk, nc, B, (const uint16_t*)z_dev, (const uint16_t*)gy_dev, part, scratch,
                          (double2*)out_dev));
    HH_HIP(hipStreamSynchronize(ctx->stream));
    return HH_OK;
}

hh_status hh_implicit_test(hh_net* net, int nc, int B, const void* x_dev, void* y_dev, int adjoint) {
    HH_ARG(net && x_dev && y_dev, "null pointer");
    HH_HIP(hipSetDevice(net->ctx->device));
    if (net->explicit_coarse) {
        HH_TRY(launch_explicit(net->ctx->stream, (const uint16_t*)x_dev, (uint16_t*)y_dev,
                               net->params.as<float>() + net->koff, nc, net->nk, B, adjoint != 0, nullptr, nullptr));
        HH_HIP(hipStreamSynchronize(net->ctx->stream));
        return HH_OK;
    }
    Buf G, Wk;
    const int M = 2 * nc;
    HH_TRY(G.ensure(net->ctx, (size_t)net->nk * M * M * sizeof(float2)));
    HH_TRY(green_forward(net, nc, G.as<float2>(), 1e-5));
    if (implicit_work_bytes(M, nc, net->nk, B) > 0) HH_TRY(Wk.ensure(net->ctx, implicit_work_bytes(M, nc, net->nk, B)));
    HH_TRY(launch_implicit(net->ctx->stream, M, (const uint16_t*)x_dev, (uint16_t*)y_dev, G.as<float2>(), nc, net->nk,
                           B, adjoint != 0, nullptr, nullptr, Wk.as<float2>()));
    HH_HIP(hipStreamSynchronize(net->ctx->stream));
    return HH_OK;
}

}  // extern "C"
