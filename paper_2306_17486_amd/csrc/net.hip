// Encoder-solver network with the implicit coarsest layer (Sec. 4.1-4.4, Sec. 5.3):
// parameters, the encoder (once per slowness model), the Green's-function
// transforms of the implicit layer (eqs. 16-17), the forward pass and the
// CNN+MG preconditioner z = V(v; s Net(v / rms(v))).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>

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

static inline int coarse_stride_of(int n) { return n >= 512 ? 2 : 1; }
static inline int coarsest_of(int n) { return n >= 512 ? n / 16 : n / 8; }
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

// First layer of the encoder / solver: 3x3 stride-2 convolution from 2 input
// channels (BF16-rounded) to COUT channels, + bias, + optional skip.  The input
// is either a complex vector scaled per RHS (solver: v / rms(v)) or the
// coefficient field (encoder: (omega h)^2 kappa^2 and (omega h)^2 kappa^2 gamma).
template <int SRC, int COUT>
__global__ void __launch_bounds__(256) k_conv_in(const float2* __restrict__ src, size_t src_bstride,
                                                 const float* __restrict__ in_scale, const int* __restrict__ src_map,
                                                 float h2, const float* __restrict__ W, const float* __restrict__ bias,
                                                 const uint16_t* __restrict__ skip, const int* __restrict__ skip_map,
                                                 uint16_t* __restrict__ y, int n, const int* __restrict__ active) {
    __shared__ float s_w[COUT * 18];
    __shared__ float s_b[COUT];
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    for (int e = threadIdx.x; e < COUT * 18; e += 256) s_w[e] = W[e];
    for (int e = threadIdx.x; e < COUT; e += 256) s_b[e] = bias[e];
    __syncthreads();
    const int m = n / 2;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= m * m) return;
    const int oy = p / m, ox = p - oy * m;
    const float2* sb = src + (size_t)(src_map ? src_map[b] : b) * src_bstride;
    const float sc = (SRC == 0) ? in_scale[b] : 1.f;
    float in[2][9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int iy = 2 * oy + t / 3 - 1, ix = 2 * ox + t % 3 - 1;
        float a0 = 0.f, a1 = 0.f;
        if (iy >= 0 && iy < n && ix >= 0 && ix < n) {
            const float2 v = sb[(size_t)iy * n + ix];
            if (SRC == 0) {
                a0 = v.x * sc;
                a1 = v.y * sc;
            } else {
                a0 = v.x * h2;
                a1 = a0 * v.y;
            }
        }
        in[0][t] = bf2f(f2bf(a0));
        in[1][t] = bf2f(f2bf(a1));
    }
    const size_t po = ((size_t)b * m * m + p) * COUT;
    const uint16_t* sk = skip ? skip + ((size_t)(skip_map ? skip_map[b] : b) * m * m + p) * COUT : nullptr;
#pragma unroll
    for (int c0 = 0; c0 < COUT; c0 += 8) {
        uint16_t o[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int co = c0 + u;
            float acc = s_b[co];
#pragma unroll
            for (int t = 0; t < 9; ++t) acc += s_w[(co * 2 + 0) * 9 + t] * in[0][t] + s_w[(co * 2 + 1) * 9 + t] * in[1][t];
            if (sk) acc += bf2f(sk[co]);
            o[u] = f2bf(acc);
        }
        *reinterpret_cast<uint4*>(y + po + c0) = *reinterpret_cast<uint4*>(o);
    }
}

// Projection layer: 3x3 stride-1 convolution CIN -> 2 channels + bias, FP32 output
template <int CIN>
__global__ void __launch_bounds__(256) k_conv_out(const uint16_t* __restrict__ x, const float* __restrict__ W,
                                                  const float* __restrict__ bias, float2* __restrict__ o, int m,
                                                  const int* __restrict__ active) {
    __shared__ float s_w[2 * CIN * 9];
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    for (int e = threadIdx.x; e < 2 * CIN * 9; e += 256) s_w[e] = W[e];
    __syncthreads();
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= m * m) return;
    const int oy = p / m, ox = p - oy * m;
    float a0 = bias[0], a1 = bias[1];
    const uint16_t* xb = x + (size_t)b * m * m * CIN;
    for (int t = 0; t < 9; ++t) {
        const int iy = oy + t / 3 - 1, ix = ox + t % 3 - 1;
        if (iy < 0 || iy >= m || ix < 0 || ix >= m) continue;
        const uint16_t* px = xb + ((size_t)iy * m + ix) * CIN;
#pragma unroll
        for (int c0 = 0; c0 < CIN; c0 += 8) {
            uint4 raw = *reinterpret_cast<const uint4*>(px + c0);
            const uint16_t* h = reinterpret_cast<const uint16_t*>(&raw);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float v = bf2f(h[u]);
                a0 += s_w[(0 * CIN + c0 + u) * 9 + t] * v;
                a1 += s_w[(1 * CIN + c0 + u) * 9 + t] * v;
            }
        }
    }
    o[(size_t)b * m * m + p] = make_float2(a0, a1);
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
template <int M, int NT>
__global__ void __launch_bounds__(NT) k_implicit(const uint16_t* __restrict__ xin, uint16_t* __restrict__ yout,
                                                 const float2* __restrict__ Gbr, int nc, int nk, int conjG,
                                                 const int* __restrict__ active) {
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
    for (int e = tid; e < M * P; e += NT) s[e] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int e = tid; e < nc * nc; e += NT) {
        const int y = e / nc, x = e - y * nc;
        const uint16_t* px = xin + (((size_t)b * nc + y) * nc + x) * CH + 2 * c;
        const uint32_t raw = *reinterpret_cast<const uint32_t*>(px);
        s[y * P + x] = make_float2(bf2f((uint16_t)(raw & 0xffff)), bf2f((uint16_t)(raw >> 16)));
    }
    __syncthreads();
    // forward DIF along the nc data rows
    for (int len = M; len >= 2; len >>= 1) {
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
    // forward DIF along all columns
    for (int len = M; len >= 2; len >>= 1) {
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
    // spectrum (bit-reversed both ways) times Ghat_c
    {
        const float2* G = Gbr + (size_t)c * M * M;
        for (int e = tid; e < M * M; e += NT) {
            float2 g = G[e];
            if (conjG) g.y = -g.y;
            const int r = e / M, col = e - r * M;
            s[r * P + col] = cmul(s[r * P + col], g);
        }
    }
    __syncthreads();
    // inverse DIT along all columns
    for (int len = 2; len <= M; len <<= 1) {
        const int half = len >> 1, tws = M / len;
        for (int t = tid; t < M * (M / 2); t += NT) {
            const int col = t % M, bf = t / M;
            const int blk = bf / half, j = bf - blk * half;
            const int i0 = (blk * len + j) * P + col, i1 = i0 + half * P;
            float2 w = tw[j * tws];
            w.y = -w.y;
            const float2 a = s[i0], bb = cmul(s[i1], w);
            s[i0] = cadd(a, bb);
            s[i1] = csub(a, bb);
        }
        __syncthreads();
    }
    // inverse DIT along the nc kept rows
    for (int len = 2; len <= M; len <<= 1) {
        const int half = len >> 1, tws = M / len;
        for (int t = tid; t < nc * (M / 2); t += NT) {
            const int row = t / (M / 2), bf = t - row * (M / 2);
            const int blk = bf / half, j = bf - blk * half;
            const int i0 = row * P + blk * len + j, i1 = i0 + half;
            float2 w = tw[j * tws];
            w.y = -w.y;
            const float2 a = s[i0], bb = cmul(s[i1], w);
            s[i0] = cadd(a, bb);
            s[i1] = csub(a, bb);
        }
        __syncthreads();
    }
    for (int e = tid; e < nc * nc; e += NT) {
        const int y = e / nc, x = e - y * nc;
        const float2 v = s[y * P + x];
        uint16_t* py = yout + (((size_t)b * nc + y) * nc + x) * CH + 2 * c;
        *reinterpret_cast<uint32_t*>(py) = (uint32_t)f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16);
    }
}

static size_t implicit_lds_bytes(int M) { return ((size_t)M * (M + 1) + M / 2) * sizeof(float2); }

hh_status launch_implicit(hipStream_t st, int M, const uint16_t* x, uint16_t* y, const float2* Gbr, int nc, int nk,
                          int B, bool conjG, const int* active) {
    const size_t lds = implicit_lds_bytes(M);
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
                           active);                                                                      \
        HH_LAUNCH_CHECK();                                                                               \
        return HH_OK;                                                                                    \
    }
    HH_IMP(16, 256)
    HH_IMP(32, 256)
    HH_IMP(64, 512)
    HH_IMP(128, 1024)
#undef HH_IMP
    set_error("implicit layer: transform size %d not supported (coarsest map must be at most 64 x 64)", M);
    return HH_ERR_ARG;
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
    __shared__ double2 s_tw[1024];
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
    long kk = ((long)(k + oout)) % N;
    if (kk < 0) kk += N;
    double re = 0.0, im = 0.0;
    for (int i = 0; i < Lin; ++i) {
        long ii = ((long)(i + oin)) % N;
        if (ii < 0) ii += N;
        const double2 w = s_tw[(ii * kk) % N];
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
    if (N > 1024) {
        set_error("Green's function grid %d too large", N);
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
hh_status net_pack(hh_net* net) {
    if (net->packed_valid) return HH_OK;
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
    net->packed_valid = true;
    return HH_OK;
}

// activations of one forward pass on a batch
struct NetActs {
    int B = 0, n = 0;
    Buf a[NET_LAYERS];  // output of every layer (BF16 NHWC); a[L_OUT] holds the FP32 (re, im) projection
    Buf imp;            // implicit-layer output
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
        HH_TRY(parts.ensure(net->ctx, (size_t)B * 64 * sizeof(double)));
        HH_TRY(scales.ensure(net->ctx, (size_t)2 * B * sizeof(float)));
        HH_TRY(zeros.ensure(net->ctx, (size_t)B * sizeof(int)));
        HH_HIP(hipMemsetAsync(zeros.ptr, 0, (size_t)B * sizeof(int), net->ctx->stream));
        return HH_OK;
    }
};

// ---------------------------------------------------------------------------
// per-model network state: encodings and Ghat
// ---------------------------------------------------------------------------
struct NetCache {
    hh_net* net = nullptr;
    unsigned long long version = 0;
    int n = 0, nc = 0, M = 0;
    Buf E[3];      // BF16 encodings per instance
    Buf tmp[2];    // encoder temporaries
    Buf Gbr;       // bit-reversed, scaled Ghat [nk][M][M]
    NetActs acts;  // forward activations of the solves on this model
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
    a.relu = relu ? 1 : 0;
    a.B = B;
    a.Hin = Hin;
    a.Win = Win;
    a.Hout = Hout;
    a.Wout = Wout;
    a.active = active;
    return launch_conv(net->ctx->stream, net->ctx->num_cus, L.cin, L.cout, mode, a);
}

// Encoder (Sec. 5.3): three levels of (strided conv, conv+ReLU, conv+ReLU) on
// the dimensionless mass term of every slowness model of the model.
static hh_status run_encoder(hh_net* net, hh_model* md, NetCache* nc) {
    hipStream_t st = net->ctx->stream;
    const int n = md->lev[0].n, B = md->ninst;
    const double h = md->lev[0].h;
    const int c[3] = {net->ch[0], net->ch[1], net->ch[2]};
    size_t tmax = 0;
    for (int l = 0; l < 3; ++l) {
        const size_t sz = (size_t)B * (n >> (l + 1)) * (n >> (l + 1)) * c[l] * sizeof(uint16_t);
        HH_TRY(nc->E[l].ensure(net->ctx, sz));
        tmax = std::max(tmax, sz);
    }
    HH_TRY(nc->tmp[0].ensure(net->ctx, tmax));
    HH_TRY(nc->tmp[1].ensure(net->ctx, tmax));
    uint16_t* t0 = nc->tmp[0].as<uint16_t>();
    uint16_t* t1 = nc->tmp[1].as<uint16_t>();
    const float* P = net->params.as<float>();
    {
        const int m = n / 2;
        dim3 grd((m * m + 255) / 256, B);
        if (c[0] != 16) {
            set_error("first-level channel count must be 16");
            return HH_ERR_ARG;
        }
        hipLaunchKernelGGL((k_conv_in<1, 16>), grd, dim3(256), 0, st, md->lev[0].coef.as<float2>(), (size_t)n * n,
                           nullptr, nullptr, (float)(h * h), P + net->L[L_ENC1_D].woff, P + net->L[L_ENC1_D].boff,
                           nullptr, nullptr, t0, n, nullptr);
        HH_LAUNCH_CHECK();
        HH_TRY(conv_layer(net, L_ENC1_C1, CM_S1, t0, B, m, m, t1, m, m, nullptr, nullptr, true, nullptr));
        HH_TRY(conv_layer(net, L_ENC1_C2, CM_S1, t1, B, m, m, nc->E[0].as<uint16_t>(), m, m, nullptr, nullptr, true,
                          nullptr));
    }
    const int ld[2] = {L_ENC2_D, L_ENC3_D};
    for (int k = 0; k < 2; ++k) {
        const int mi = n >> (k + 1), mo = mi / 2;
        const int l = ld[k];
        HH_TRY(conv_layer(net, l, CM_S2, nc->E[k].as<uint16_t>(), B, mi, mi, t0, mo, mo, nullptr, nullptr, false,
                          nullptr));
        HH_TRY(conv_layer(net, l + 1, CM_S1, t0, B, mo, mo, t1, mo, mo, nullptr, nullptr, true, nullptr));
        HH_TRY(conv_layer(net, l + 2, CM_S1, t1, B, mo, mo, nc->E[k + 1].as<uint16_t>(), mo, mo, nullptr, nullptr,
                          true, nullptr));
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
    if (nc->net == net && nc->version == net->version && nc->n == md->lev[0].n) return HH_OK;
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
    HH_TRY(green_forward(net, nc->nc, nc->Gbr.as<float2>(), 1e-5));
    HH_TRY(run_encoder(net, md, nc));
    nc->net = net;
    nc->version = net->version;
    return HH_OK;
}

// e = out_scale * P(Net(v * in_scale)) for the B vectors v (stride vstride);
// writes x0 (complex single, [B][n][n]).  Encodings come from the model cache.
hh_status net_forward_batch(hh_net* net, hh_model* md, NetActs& A, int B, const BatchMap& bm, const float2* v,
                            size_t vstride, const double* sig, int sig_stride, float2* x0, const int* active) {
    hipStream_t st = net->ctx->stream;
    NetCache* nc = reinterpret_cast<NetCache*>(md->netcache);
    const int n = md->lev[0].n;
    const double h = md->lev[0].h;
    HH_TRY(A.ensure(net, B, n));
    const int* smap = md->ninst > 1 ? bm.inst : A.zeros.as<int>();
    float* in_scale = A.scales.as<float>();
    float* out_scale = in_scale + B;
    // rms scaling (C9 reading of Sec. 4.3: the network works on a unit-rms residual)
    {
        const int nblk = 64;
        hipLaunchKernelGGL(k_sumsq, dim3(nblk, B), dim3(256), 0, st, v, vstride, (size_t)n * n, A.parts.as<double>(),
                           active);
        HH_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_scales, dim3((B + 63) / 64), dim3(64), 0, st, A.parts.as<double>(), nblk, (size_t)n * n,
                           sig, sig_stride, h * h, in_scale, out_scale, B);
        HH_LAUNCH_CHECK();
    }
    const float* P = net->params.as<float>();
    auto act = [&](int l) { return A.a[l].as<uint16_t>(); };
    const int m1 = n / 2, m2 = n / 4, m3 = n / 8, m4 = coarsest_of(n), s4 = coarse_stride_of(n);
    {
        ProfScope ps(net->ctx, HH_K_CONV);
        hipLaunchKernelGGL((k_conv_in<0, 16>), dim3((m1 * m1 + 255) / 256, B), dim3(256), 0, st, v, vstride, in_scale,
                           nullptr, 0.f, P + net->L[L_S1_D].woff, P + net->L[L_S1_D].boff, nc->E[0].as<uint16_t>(),
                           smap, act(L_S1_D), n, active);
        HH_LAUNCH_CHECK();
    }
    {
        ProfScope ps(net->ctx, HH_K_CONV);
        // level 1
        HH_TRY(conv_layer(net, L_S1_C1, CM_S1, act(L_S1_D), B, m1, m1, act(L_S1_C1), m1, m1, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_S1_C2, CM_S1, act(L_S1_C1), B, m1, m1, act(L_S1_C2), m1, m1, nullptr, nullptr, true, active));
        // level 2
        HH_TRY(conv_layer(net, L_S2_D, CM_S2, act(L_S1_C2), B, m1, m1, act(L_S2_D), m2, m2, nc->E[1].as<uint16_t>(), smap, false, active));
        HH_TRY(conv_layer(net, L_S2_C1, CM_S1, act(L_S2_D), B, m2, m2, act(L_S2_C1), m2, m2, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_S2_C2, CM_S1, act(L_S2_C1), B, m2, m2, act(L_S2_C2), m2, m2, nullptr, nullptr, true, active));
        // level 3
        HH_TRY(conv_layer(net, L_S3_D, CM_S2, act(L_S2_C2), B, m2, m2, act(L_S3_D), m3, m3, nc->E[2].as<uint16_t>(), smap, false, active));
        HH_TRY(conv_layer(net, L_S3_C1, CM_S1, act(L_S3_D), B, m3, m3, act(L_S3_C1), m3, m3, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_S3_C2, CM_S1, act(L_S3_C1), B, m3, m3, act(L_S3_C2), m3, m3, nullptr, nullptr, true, active));
        // level 4 (stride 1 below n = 512)
        HH_TRY(conv_layer(net, L_S4_D, s4 == 2 ? CM_S2 : CM_S1, act(L_S3_C2), B, m3, m3, act(L_S4_D), m4, m4, nullptr, nullptr, false, active));
        HH_TRY(conv_layer(net, L_S4_C1, CM_S1, act(L_S4_D), B, m4, m4, act(L_S4_C1), m4, m4, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_S4_C2, CM_S1, act(L_S4_C1), B, m4, m4, act(L_S4_C2), m4, m4, nullptr, nullptr, true, active));
    }
    {
        ProfScope ps(net->ctx, HH_K_NET_OTHER);
        HH_TRY(launch_implicit(st, 2 * m4, act(L_S4_C2), A.imp.as<uint16_t>(), nc->Gbr.as<float2>(), m4, net->nk, B,
                               false, active));
    }
    {
        ProfScope ps(net->ctx, HH_K_CONV);
        // up to level 3: transposed stride-2 (stride-1 below n = 512), + level-3 features
        HH_TRY(conv_layer(net, L_U3_T, s4 == 2 ? CM_T2 : CM_S1, A.imp.as<uint16_t>(), B, m4, m4, act(L_U3_T), m3, m3, act(L_S3_C2), nullptr, false, active));
        HH_TRY(conv_layer(net, L_U3_C1, CM_S1, act(L_U3_T), B, m3, m3, act(L_U3_C1), m3, m3, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_U3_C2, CM_S1, act(L_U3_C1), B, m3, m3, act(L_U3_C2), m3, m3, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_U2_T, CM_T2, act(L_U3_C2), B, m3, m3, act(L_U2_T), m2, m2, act(L_S2_C2), nullptr, false, active));
        HH_TRY(conv_layer(net, L_U2_C1, CM_S1, act(L_U2_T), B, m2, m2, act(L_U2_C1), m2, m2, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_U2_C2, CM_S1, act(L_U2_C1), B, m2, m2, act(L_U2_C2), m2, m2, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_U1_T, CM_T2, act(L_U2_C2), B, m2, m2, act(L_U1_T), m1, m1, act(L_S1_C2), nullptr, false, active));
        HH_TRY(conv_layer(net, L_U1_C1, CM_S1, act(L_U1_T), B, m1, m1, act(L_U1_C1), m1, m1, nullptr, nullptr, true, active));
        HH_TRY(conv_layer(net, L_U1_C2, CM_S1, act(L_U1_C1), B, m1, m1, act(L_U1_C2), m1, m1, nullptr, nullptr, true, active));
    }
    {
        ProfScope ps(net->ctx, HH_K_NET_OTHER);
        float2* o = A.a[L_OUT].as<float2>();
        hipLaunchKernelGGL((k_conv_out<16>), dim3((m1 * m1 + 255) / 256, B), dim3(256), 0, st, act(L_U1_C2),
                           P + net->L[L_OUT].woff, P + net->L[L_OUT].boff, o, m1, active);
        HH_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_prolong_x0, dim3((n * n + 255) / 256, B), dim3(256), 0, st, o, out_scale, x0, n, active);
        HH_LAUNCH_CHECK();
    }
    return HH_OK;
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
    float2* x0 = W.x0net.as<float2>();
    HH_TRY(net_forward_batch(net, md, nc->acts, W.nrhs, bm, v, vstride, sig, sig_stride, x0, act));
    const size_t nn = (size_t)md->lev[0].n * md->lev[0].n;
    return launch_vcycle_strided(md, W.nrhs, bm, v, vstride, sig, sig_stride, x0, nn, z, zstride, W.vwork.ptr, act);
}

}  // namespace hh

using namespace hh;

extern "C" {

static bool valid_channels(const int* ch) { return ch[0] == 16 && ch[1] == 32 && ch[2] == 64 && ch[3] == 64; }

hh_status hh_net_create(hh_ctx* ctx, const hh_net_desc* d, const float* params_host, hh_net** out) {
    HH_ARG(ctx && d && out, "null pointer");
    *out = nullptr;
    HH_ARG(valid_channels(d->ch), "channels must be (16, 32, 64, 64)");
    HH_HIP(hipSetDevice(ctx->device));
    hh_net* net = new (std::nothrow) hh_net();
    if (!net) {
        set_error("out of host memory");
        return HH_ERR_NOMEM;
    }
    net->ctx = ctx;
    for (int i = 0; i < 4; ++i) net->ch[i] = d->ch[i];
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

static const char kMagic[8] = {'H', 'H', 'N', 'E', 'T', '0', '0', '1'};

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
    bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(net->ch, sizeof(int), 4, f) == 4 &&
              fwrite(&np, sizeof(np), 1, f) == 1 && fwrite(&step, sizeof(step), 1, f) == 1 &&
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
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMagic, 8) == 0 && fread(d.ch, sizeof(int), 4, f) == 4 &&
              fread(&np, sizeof(np), 1, f) == 1 && fread(&step, sizeof(step), 1, f) == 1 &&
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
    NetCache* nc = reinterpret_cast<NetCache*>(m->netcache);
    const size_t nn = (size_t)m->lev[0].n * m->lev[0].n;
    HH_TRY(net_forward_batch(m->net, m, nc->acts, nrhs, bm, (const float2*)r_dev, nn, nullptr, 0, (float2*)e_dev,
                             nullptr));
    HH_HIP(hipStreamSynchronize(m->ctx->stream));
    return HH_OK;
}

hh_status hh_conv_test(hh_ctx* ctx, int cin, int cout, int mode, int B, int Hin, int Win, const void* x_dev,
                       const float* w_dev, int flipped, const float* bias_dev, const void* skip_dev, int relu,
                       void* y_dev, float* yf_dev) {
    HH_ARG(ctx && x_dev && w_dev && y_dev, "null pointer");
    HH_ARG(mode >= 0 && mode <= 2, "mode");
    HH_HIP(hipSetDevice(ctx->device));
    Buf wp;
    HH_TRY(wp.ensure(ctx, packed_weight_elems(cin, cout) * sizeof(uint16_t) + 256));
    HH_TRY(pack_weights(ctx->stream, w_dev, wp.as<uint16_t>(), cin, cout, flipped != 0));
    ConvArgs a{};
    a.x = (const uint16_t*)x_dev;
    a.y = (uint16_t*)y_dev;
    a.yf = yf_dev;
    a.wp = wp.as<uint16_t>();
    a.bias = bias_dev;
    a.skip = (const uint16_t*)skip_dev;
    a.relu = relu;
    a.B = B;
    a.Hin = Hin;
    a.Win = Win;
    a.Hout = mode == CM_S2 ? Hin / 2 : (mode == CM_T2 ? 2 * Hin : Hin);
    a.Wout = mode == CM_S2 ? Win / 2 : (mode == CM_T2 ? 2 * Win : Win);
    HH_TRY(launch_conv(ctx->stream, ctx->num_cus, cin, cout, mode, a));
    HH_HIP(hipStreamSynchronize(ctx->stream));
    return HH_OK;
}

hh_status hh_implicit_test(hh_net* net, int nc, int B, const void* x_dev, void* y_dev, int adjoint) {
    HH_ARG(net && x_dev && y_dev, "null pointer");
    HH_HIP(hipSetDevice(net->ctx->device));
    Buf G;
    const int M = 2 * nc;
    HH_TRY(G.ensure(net->ctx, (size_t)net->nk * M * M * sizeof(float2)));
    HH_TRY(green_forward(net, nc, G.as<float2>(), 1e-5));
    HH_TRY(launch_implicit(net->ctx->stream, M, (const uint16_t*)x_dev, (uint16_t*)y_dev, G.as<float2>(), nc, net->nk,
                           B, adjoint != 0, nullptr));
    HH_HIP(hipStreamSynchronize(net->ctx->stream));
    return HH_OK;
}

}  // extern "C"
