// Kernels of the lightweight encoder-solver network (Sec. 4.4, Sec. 5.3):
// pointwise (1x1) convolutions on the matrix cores, depthwise 3x3
// convolutions, batch normalisation in its training form (batch statistics,
// running averages, backward) and its folding into the weights at inference.
// Activations are BF16 NHWC [pixel][channel]; accumulation is FP32 (sums over
// pixels for statistics in FP64).
#include "net.h"

namespace hh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr double BN_EPS = 1e-5;
constexpr double BN_MOMENTUM = 0.1;

// out[e] = sum_b part[b][e]  (deterministic second stage of the reductions)
__global__ void k_sum_blocks(const float* __restrict__ part, int nblk, int count, float* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    float acc = 0.f;
    for (int b = 0; b < nblk; ++b) acc += part[(size_t)b * count + e];
    out[e] = acc;
}

__device__ __forceinline__ void unpack8(uint4 r, float (&f)[8]) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = bf2f((uint16_t)(w[i] & 0xffff));
        f[2 * i + 1] = bf2f((uint16_t)(w[i] >> 16));
    }
}
__device__ __forceinline__ uint4 pack8(const float (&f)[8]) {
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = f2bf2(f[2 * i], f[2 * i + 1]);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// ---------------------------------------------------------------------------
// Batch-normalisation folding (inference): per output channel o,
//   W'[o][...] = W[o][...] g[o] / sqrt(rv[o] + eps),   b'[o] = be[o] - rm[o] g[o] / sqrt(rv[o] + eps)
// (W's first index is the output channel: 3x3, 1x1 and depthwise layers).
// ---------------------------------------------------------------------------
__global__ void k_bn_fold(const float* __restrict__ W, const float* __restrict__ g, const float* __restrict__ be,
                          const float* __restrict__ rm, const float* __restrict__ rv, int cout, int per,
                          float* __restrict__ Wf, float* __restrict__ bf) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < cout * per) {
        const int o = e / per;
        Wf[e] = (float)((double)W[e] * (double)g[o] / sqrt((double)rv[o] + BN_EPS));
    }
    if (e < cout) bf[e] = (float)((double)be[e] - (double)rm[e] * (double)g[e] / sqrt((double)rv[e] + BN_EPS));
}

hh_status bn_fold(hipStream_t st, const float* W, const float* g, const float* be, const float* rm, const float* rv,
                  int cout, int per, float* Wf, float* bf) {
    const int total = cout * per;
    hipLaunchKernelGGL(k_bn_fold, dim3((total + 255) / 256), dim3(256), 0, st, W, g, be, rm, rv, cout, per, Wf, bf);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// ---------------------------------------------------------------------------
// Pointwise convolution y[p][o] = act(sum_c W[o][c] x[p][c] + bias[o]) + res[p][o]
// as a GEMM on the matrix cores: A = 16 output channels x k (weights, from
// LDS), B = k x 16 pixels (straight from the NHWC input), D = 16 channels x
// 16 pixels.  k steps of 32 (v_mfma_f32_16x16x32_bf16) or, for 16 input
// channels, one step of 16 (v_mfma_f32_16x16x16_bf16).
// Weights: BF16 [cout][cin] (pack_pointwise).
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
struct PwCfg {
    static constexpr int KC = (CIN % 32 == 0) ? 32 : 16;               // k per MFMA
    static constexpr int NK = CIN / KC;                                 // k steps
    static constexpr int NO = COUT / 16;                                // output-channel tiles
    static constexpr int PB = CIN <= 64 ? 4 : (CIN <= 192 ? 2 : 1);     // 16-pixel blocks per wave step
    static constexpr int WP = CIN + 8;                                  // LDS pitch of a weight row (BF16)
    static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channel counts are multiples of 16");
};

template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_pointwise(PwArgs a) {
    using C = PwCfg<CIN, COUT>;
    __shared__ __attribute__((aligned(16))) uint16_t s_w[COUT * C::WP];
    for (int e = threadIdx.x; e < COUT * CIN / 8; e += 256) {
        const int o = e / (CIN / 8), k8 = e - o * (CIN / 8);
        *reinterpret_cast<uint4*>(&s_w[o * C::WP + 8 * k8]) = reinterpret_cast<const uint4*>(a.w)[e];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lp = lane & 15, lg = lane >> 4;
    const size_t nb16 = (a.npix + 15) / 16;
    const size_t ngroups = (nb16 + C::PB - 1) / C::PB;
    for (size_t grp = (size_t)blockIdx.x * 4 + wave; grp < ngroups; grp += (size_t)gridDim.x * 4) {
        const size_t p0 = grp * C::PB * 16;
        // a group lies within one batch entry (pix_per_b is a multiple of the group size)
        if (a.active && !a.active[p0 / a.pix_per_b]) continue;
        // B operand: the group's pixels, all k steps
        uint4 bfr[C::PB][C::NK];
#pragma unroll
        for (int q = 0; q < C::PB; ++q) {
            const size_t p = p0 + q * 16 + lp;
#pragma unroll
            for (int kc = 0; kc < C::NK; ++kc) {
                uint4 v = make_uint4(0, 0, 0, 0);
                if (p < a.npix) {
                    if constexpr (C::KC == 32) {
                        v = *reinterpret_cast<const uint4*>(a.x + p * CIN + kc * 32 + 8 * lg);
                    } else {
                        const uint2 h = *reinterpret_cast<const uint2*>(a.x + p * CIN + kc * 16 + 4 * lg);
                        v.x = h.x;
                        v.y = h.y;
                    }
                }
                bfr[q][kc] = v;
            }
        }
#pragma unroll 1
        for (int ot = 0; ot < C::NO; ++ot) {
            f32x4 acc[C::PB];
#pragma unroll
            for (int q = 0; q < C::PB; ++q) acc[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < C::NK; ++kc) {
                const uint16_t* wr = &s_w[(ot * 16 + lp) * C::WP];
                if constexpr (C::KC == 32) {
                    const uint4 wv = *reinterpret_cast<const uint4*>(wr + kc * 32 + 8 * lg);
                    const bf16x8 A = *reinterpret_cast<const bf16x8*>(&wv);
#pragma unroll
                    for (int q = 0; q < C::PB; ++q)
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            A, *reinterpret_cast<const bf16x8*>(&bfr[q][kc]), acc[q], 0, 0, 0);
                } else {
                    const uint2 wv = *reinterpret_cast<const uint2*>(wr + kc * 16 + 4 * lg);
                    const s16x4 A = *reinterpret_cast<const s16x4*>(&wv);
#pragma unroll
                    for (int q = 0; q < C::PB; ++q) {
                        const uint2 bv = make_uint2(bfr[q][kc].x, bfr[q][kc].y);
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                            A, *reinterpret_cast<const s16x4*>(&bv), acc[q], 0, 0, 0);
                    }
                }
            }
            // epilogue: lane holds channels ot*16 + 4 lg .. +3 of pixel p0 + q*16 + lp
            const int co = ot * 16 + 4 * lg;
            float bias4[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) bias4[i] = a.bias ? a.bias[co + i] : 0.f;
#pragma unroll
            for (int q = 0; q < C::PB; ++q) {
                const size_t p = p0 + q * 16 + lp;
                if (p >= a.npix) continue;
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    v[i] = acc[q][i] + bias4[i];
                    if (a.act == ACT_SOFTPLUS) v[i] = softplus_f(v[i]);
                }
                const size_t po = p * COUT + co;
                if (a.res) {
                    const uint2 r2 = *reinterpret_cast<const uint2*>(a.res + po);
                    v[0] += bf2f((uint16_t)(r2.x & 0xffff));
                    v[1] += bf2f((uint16_t)(r2.x >> 16));
                    v[2] += bf2f((uint16_t)(r2.y & 0xffff));
                    v[3] += bf2f((uint16_t)(r2.y >> 16));
                }
                uint2 o2;
                o2.x = f2bf2(v[0], v[1]);
                o2.y = f2bf2(v[2], v[3]);
                *reinterpret_cast<uint2*>(a.y + po) = o2;
                if (a.yf) *reinterpret_cast<float4*>(a.yf + po) = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
    }
}

template <int CIN, int COUT>
static hh_status launch_pw_t(hipStream_t st, int num_cus, const PwArgs& a) {
    using C = PwCfg<CIN, COUT>;
    const size_t groups = ((a.npix + 15) / 16 + C::PB - 1) / C::PB;
    if (a.active && (a.pix_per_b <= 0 || a.pix_per_b % (C::PB * 16) != 0)) {
        set_error("pointwise convolution: %d pixels per batch entry is not a multiple of %d", a.pix_per_b,
                  C::PB * 16);
        return HH_ERR_ARG;
    }
    const size_t want = (groups + 3) / 4;
    const int grid = (int)std::max<size_t>(1, std::min<size_t>(want, (size_t)num_cus * 8));
    hipLaunchKernelGGL((k_pointwise<CIN, COUT>), dim3(grid), dim3(256), 0, st, a);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

hh_status launch_pointwise(hipStream_t st, int num_cus, int cin, int cout, const PwArgs& a) {
    if (a.npix == 0) return HH_OK;
#define HH_PW(CI, CO) \
    if (cin == CI && cout == CO) return launch_pw_t<CI, CO>(st, num_cus, a);
    HH_PW(16, 96)
    HH_PW(96, 16)
    HH_PW(32, 192)
    HH_PW(192, 32)
    HH_PW(64, 384)
    HH_PW(384, 64)
#undef HH_PW
    set_error("no pointwise kernel for %d -> %d channels", cin, cout);
    return HH_ERR_ARG;
}

// BF16 weights of a pointwise layer: out[o][c] = W[o][c] (transpose = 0) or
// out[c][o] = W[o][c] (transpose = 1: the weights of its input gradient)
__global__ void k_pack_pw(const float* __restrict__ W, uint16_t* __restrict__ out, int cout, int cin, int transpose) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cout * cin) return;
    const int o = e / cin, c = e - o * cin;
    out[transpose ? (size_t)c * cout + o : (size_t)e] = f2bf(W[e]);
}

hh_status pack_pointwise(hipStream_t st, const float* W, uint16_t* out, int cout, int cin, bool transpose) {
    hipLaunchKernelGGL(k_pack_pw, dim3((cout * cin + 255) / 256), dim3(256), 0, st, W, out, cout, cin,
                       transpose ? 1 : 0);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// ---------------------------------------------------------------------------
// Depthwise 3x3 convolution (stride 1, zero padding):
//   y[b][i][j][c] = act(sum_{a,e} w[c][a][e] x[b][i+a-1][j+e-1][c] + bias[c])
// flip = 1 uses w[c][2-a][2-e] (the input gradient of the layer).  One thread
// per pixel and 8 channels; weights FP32 in LDS as [tap][c].
// ---------------------------------------------------------------------------
template <int C>
__global__ void __launch_bounds__(256) k_depthwise(DwArgs a) {
    __shared__ __attribute__((aligned(16))) float s_w[9 * C];
    __shared__ __attribute__((aligned(16))) float s_b[C];
    for (int e = threadIdx.x; e < 9 * C; e += 256) {
        const int t = e / C, c = e - t * C;
        s_w[e] = a.w[c * 9 + (a.flip ? 8 - t : t)];
    }
    for (int c = threadIdx.x; c < C; c += 256) s_b[c] = a.bias ? a.bias[c] : 0.f;
    __syncthreads();
    constexpr int V = C / 8;
    const size_t hw = (size_t)a.H * a.W;
    const size_t total = (size_t)a.B * hw * V;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const int v = (int)(e % V);
        const size_t pix = e / V;
        const int b = (int)(pix / hw);
        if (a.active && !a.active[b]) continue;
        const int rem = (int)(pix - (size_t)b * hw);
        const int i = rem / a.W, j = rem - i * a.W;
        float acc[8];
        {
            const float4 b0 = *reinterpret_cast<const float4*>(&s_b[8 * v]);
            const float4 b1 = *reinterpret_cast<const float4*>(&s_b[8 * v + 4]);
            acc[0] = b0.x; acc[1] = b0.y; acc[2] = b0.z; acc[3] = b0.w;
            acc[4] = b1.x; acc[5] = b1.y; acc[6] = b1.z; acc[7] = b1.w;
        }
        const uint16_t* xb = a.x + (size_t)b * hw * C;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ii = i + t / 3 - 1, jj = j + t % 3 - 1;
            if (ii < 0 || ii >= a.H || jj < 0 || jj >= a.W) continue;
            float xv[8];
            unpack8(*reinterpret_cast<const uint4*>(xb + ((size_t)ii * a.W + jj) * C + 8 * v), xv);
            const float4 w0 = *reinterpret_cast<const float4*>(&s_w[t * C + 8 * v]);
            const float4 w1 = *reinterpret_cast<const float4*>(&s_w[t * C + 8 * v + 4]);
            acc[0] += w0.x * xv[0]; acc[1] += w0.y * xv[1]; acc[2] += w0.z * xv[2]; acc[3] += w0.w * xv[3];
            acc[4] += w1.x * xv[4]; acc[5] += w1.y * xv[5]; acc[6] += w1.z * xv[6]; acc[7] += w1.w * xv[7];
        }
        if (a.act == ACT_SOFTPLUS)
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] = softplus_f(acc[u]);
        const size_t po = pix * C + 8 * v;
        *reinterpret_cast<uint4*>(a.y + po) = pack8(acc);
        if (a.yf) {
            *reinterpret_cast<float4*>(a.yf + po) = make_float4(acc[0], acc[1], acc[2], acc[3]);
            *reinterpret_cast<float4*>(a.yf + po + 4) = make_float4(acc[4], acc[5], acc[6], acc[7]);
        }
    }
}

static int elementwise_grid(size_t work, int num_cus) {
    return (int)std::max<size_t>(1, std::min<size_t>((work + 255) / 256, (size_t)num_cus * 16));
}

hh_status launch_depthwise(hipStream_t st, int num_cus, int C, const DwArgs& a) {
    const size_t work = (size_t)a.B * a.H * a.W * (C / 8);
    if (work == 0) return HH_OK;
    const int grid = elementwise_grid(work, num_cus);
    if (C == 96)
        hipLaunchKernelGGL(k_depthwise<96>, dim3(grid), dim3(256), 0, st, a);
    else if (C == 192)
        hipLaunchKernelGGL(k_depthwise<192>, dim3(grid), dim3(256), 0, st, a);
    else if (C == 384)
        hipLaunchKernelGGL(k_depthwise<384>, dim3(grid), dim3(256), 0, st, a);
    else {
        set_error("no depthwise kernel for %d channels", C);
        return HH_ERR_ARG;
    }
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// ---------------------------------------------------------------------------
// Batch normalisation, training form, over the npix pixels of a BF16 tensor
// z [npix][C] (all batch entries, rows and columns).
// ---------------------------------------------------------------------------
constexpr int BN_BLOCKS = 256;

// per-block FP64 partial sums: part[blk][c][0] = sum z, [1] = sum z^2 (MODE 0);
// backward (MODE 1): [0] = sum gy, [1] = sum gy xhat, gy = gout * act'(yhat)
template <int C, int MODE>
__global__ void __launch_bounds__(256) k_bn_sums(const uint16_t* __restrict__ z, const uint16_t* __restrict__ gout,
                                                 const float4* __restrict__ stat, int act, size_t npix,
                                                 double* __restrict__ part) {
    constexpr int V = C / 8, R = 256 / V;  // threads per pixel, pixels per block step
    __shared__ double s[256 * 16];
    const int t = threadIdx.x;
    const int v = t % V, r = t / V;
    double s0[8], s1[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) s0[u] = s1[u] = 0.0;
    float4 st[8];
    if (MODE == 1) {
#pragma unroll
        for (int u = 0; u < 8; ++u) st[u] = stat[8 * v + u];
    }
    if (r < R) {
        for (size_t p = (size_t)blockIdx.x * R + r; p < npix; p += (size_t)gridDim.x * R) {
            float zv[8];
            unpack8(*reinterpret_cast<const uint4*>(z + p * C + 8 * v), zv);
            if (MODE == 0) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    s0[u] += zv[u];
                    s1[u] += (double)zv[u] * zv[u];
                }
            } else {
                float gv[8];
                unpack8(*reinterpret_cast<const uint4*>(gout + p * C + 8 * v), gv);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    // stat: (mean, sd, scale, shift)
                    const float yh = zv[u] * st[u].z + st[u].w;
                    const float gy = act == ACT_SOFTPLUS ? gv[u] * logistic_f(yh) : gv[u];
                    const float xh = (zv[u] - st[u].x) / st[u].y;
                    s0[u] += gy;
                    s1[u] += (double)gy * xh;
                }
            }
        }
    }
    if (r < R) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            s[(r * V + v) * 16 + 2 * u] = s0[u];
            s[(r * V + v) * 16 + 2 * u + 1] = s1[u];
        }
    }
    __syncthreads();
    for (int j = t; j < 2 * C; j += 256) {
        const int c = j >> 1, k = j & 1;
        const int vv = c >> 3, u = c & 7;
        double acc = 0.0;
        for (int rr = 0; rr < R; ++rr) acc += s[(rr * V + vv) * 16 + 2 * u + k];
        part[(size_t)blockIdx.x * 2 * C + j] = acc;
    }
}

// per channel: mean, biased variance -> stat = (mean, sd, g/sd, be - mean g/sd);
// running averages updated in place (unbiased variance) when update != 0
__global__ void k_bn_finalize(const double* __restrict__ part, int nblk, int C, double m, const float* __restrict__ g,
                              const float* __restrict__ be, float* __restrict__ rm, float* __restrict__ rv, int update,
                              float4* __restrict__ stat) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    double S = 0.0, SS = 0.0;
    for (int b = 0; b < nblk; ++b) {
        S += part[(size_t)b * 2 * C + 2 * c];
        SS += part[(size_t)b * 2 * C + 2 * c + 1];
    }
    const double mean = S / m;
    const double var = fmax(SS / m - mean * mean, 0.0);
    const double sd = sqrt(var + BN_EPS);
    const double scale = (double)g[c] / sd;
    stat[c] = make_float4((float)mean, (float)sd, (float)scale, (float)((double)be[c] - mean * scale));
    if (update) {
        rm[c] = (float)((1.0 - BN_MOMENTUM) * rm[c] + BN_MOMENTUM * mean);
        rv[c] = (float)((1.0 - BN_MOMENTUM) * rv[c] + BN_MOMENTUM * var * m / (m - 1.0));
    }
}

// y = act(scale z + shift) (+ res)
template <int C>
__global__ void __launch_bounds__(256) k_bn_apply(const uint16_t* __restrict__ z, const float4* __restrict__ stat,
                                                  int act, const uint16_t* __restrict__ res, uint16_t* __restrict__ y,
                                                  size_t npix) {
    constexpr int V = C / 8;
    const size_t total = npix * V;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const int v = (int)(e % V);
        float zv[8], rv8[8];
        unpack8(*reinterpret_cast<const uint4*>(z + e * 8), zv);
        if (res) unpack8(*reinterpret_cast<const uint4*>(res + e * 8), rv8);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float4 st = stat[8 * v + u];
            float o = zv[u] * st.z + st.w;
            if (act == ACT_SOFTPLUS) o = softplus_f(o);
            if (res) o += rv8[u];
            zv[u] = o;
        }
        *reinterpret_cast<uint4*>(y + e * 8) = pack8(zv);
    }
}

// backward coefficients per channel: grads of g and be (running statistics get
// zero), and coef = (g/sd, mean of gy, mean of gy xhat)
__global__ void k_bn_bwd_finalize(const double* __restrict__ part, int nblk, int C, double m,
                                  const float* __restrict__ g, const float4* __restrict__ stat, float* __restrict__ gr_g,
                                  float* __restrict__ gr_be, float* __restrict__ gr_rm, float* __restrict__ gr_rv,
                                  float4* __restrict__ coef) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    double sg = 0.0, sgx = 0.0;
    for (int b = 0; b < nblk; ++b) {
        sg += part[(size_t)b * 2 * C + 2 * c];
        sgx += part[(size_t)b * 2 * C + 2 * c + 1];
    }
    gr_g[c] = (float)sgx;
    gr_be[c] = (float)sg;
    gr_rm[c] = 0.f;
    gr_rv[c] = 0.f;
    coef[c] = make_float4((float)((double)g[c] / (double)stat[c].y), (float)(sg / m), (float)(sgx / m), 0.f);
}

// gz = (g/sd) (gy - mean(gy) - xhat mean(gy xhat))
template <int C>
__global__ void __launch_bounds__(256) k_bn_bwd_apply(const uint16_t* __restrict__ gout, const uint16_t* __restrict__ z,
                                                      const float4* __restrict__ stat, const float4* __restrict__ coef,
                                                      int act, uint16_t* __restrict__ gz, size_t npix) {
    constexpr int V = C / 8;
    const size_t total = npix * V;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const int v = (int)(e % V);
        float zv[8], gv[8];
        unpack8(*reinterpret_cast<const uint4*>(z + e * 8), zv);
        unpack8(*reinterpret_cast<const uint4*>(gout + e * 8), gv);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float4 st = stat[8 * v + u];
            const float4 cf = coef[8 * v + u];
            const float gy = act == ACT_SOFTPLUS ? gv[u] * logistic_f(zv[u] * st.z + st.w) : gv[u];
            const float xh = (zv[u] - st.x) / st.y;
            gv[u] = cf.x * (gy - cf.y - xh * cf.z);
        }
        *reinterpret_cast<uint4*>(gz + e * 8) = pack8(gv);
    }
}

template <int C>
static hh_status bn_fwd_t(hipStream_t st, hh_ctx* ctx, Buf& part, const uint16_t* z, size_t npix, const BnParams& p,
                          bool update, float4* stat, int act, const uint16_t* res, uint16_t* y) {
    HH_TRY(part.ensure(ctx, (size_t)BN_BLOCKS * 2 * C * sizeof(double)));
    hipLaunchKernelGGL((k_bn_sums<C, 0>), dim3(BN_BLOCKS), dim3(256), 0, st, z, nullptr, nullptr, 0, npix,
                       part.as<double>());
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bn_finalize, dim3((C + 63) / 64), dim3(64), 0, st, part.as<double>(), BN_BLOCKS, C,
                       (double)npix, p.g, p.be, p.rm, p.rv, update ? 1 : 0, stat);
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bn_apply<C>, dim3(elementwise_grid(npix * (C / 8), ctx->num_cus)), dim3(256), 0, st, z,
                       stat, act, res, y, npix);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

template <int C>
static hh_status bn_bwd_t(hipStream_t st, hh_ctx* ctx, Buf& part, Buf& coef, const uint16_t* gout,
                          const uint16_t* z, size_t npix, const float* g, const float4* stat, int act,
                          const BnGrads& gr, uint16_t* gz) {
    HH_TRY(part.ensure(ctx, (size_t)BN_BLOCKS * 2 * C * sizeof(double)));
    HH_TRY(coef.ensure(ctx, (size_t)C * sizeof(float4)));
    hipLaunchKernelGGL((k_bn_sums<C, 1>), dim3(BN_BLOCKS), dim3(256), 0, st, z, gout, stat, act, npix,
                       part.as<double>());
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bn_bwd_finalize, dim3((C + 63) / 64), dim3(64), 0, st, part.as<double>(), BN_BLOCKS, C,
                       (double)npix, g, stat, gr.g, gr.be, gr.rm, gr.rv, coef.as<float4>());
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bn_bwd_apply<C>, dim3(elementwise_grid(npix * (C / 8), ctx->num_cus)), dim3(256), 0, st,
                       gout, z, stat, coef.as<float4>(), act, gz, npix);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

#define HH_BN_CHANNELS(F) F(16) F(32) F(64) F(96) F(192) F(384)

hh_status bn_train_forward(hipStream_t st, hh_ctx* ctx, Buf& part, int C, const uint16_t* z, size_t npix,
                           const BnParams& p, bool update, float4* stat, int act, const uint16_t* res, uint16_t* y) {
    if (npix < 2) {
        set_error("batch normalisation needs at least 2 values per channel");
        return HH_ERR_ARG;
    }
#define HH_BNF(CC) \
    if (C == CC) return bn_fwd_t<CC>(st, ctx, part, z, npix, p, update, stat, act, res, y);
    HH_BN_CHANNELS(HH_BNF)
#undef HH_BNF
    set_error("batch normalisation of %d channels", C);
    return HH_ERR_ARG;
}

hh_status bn_train_backward(hipStream_t st, hh_ctx* ctx, Buf& part, Buf& coef, int C, const uint16_t* gout,
                            const uint16_t* z, size_t npix, const float* g, const float4* stat, int act,
                            const BnGrads& gr, uint16_t* gz) {
#define HH_BNB(CC) \
    if (C == CC) return bn_bwd_t<CC>(st, ctx, part, coef, gout, z, npix, g, stat, act, gr, gz);
    HH_BN_CHANNELS(HH_BNB)
#undef HH_BNB
    set_error("batch normalisation of %d channels", C);
    return HH_ERR_ARG;
}

// ---------------------------------------------------------------------------
// Weight gradient of a pointwise layer: gW[o][c] = sum_p g[p][o] x[p][c]
// (g: gradient of the layer's output [npix][COUT], x: its input [npix][CIN]).
// Each block takes a contiguous pixel range, staged through LDS 32 pixels at a
// time in FP32; thread (io, ic) owns an RO x RC tile of gW.  Partials per
// block, summed by k_sum_blocks.
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
struct PwgCfg {
    static constexpr int R = CIN * COUT / 256;  // outputs per thread
    static constexpr int RO = (COUT >= 6 * CIN) ? (R >= 96 ? 12 : 6) : (CIN >= 6 * COUT ? (R >= 96 ? 8 : (R >= 24 ? 4 : 1)) : 1);
    static constexpr int RC = R / RO;
    static constexpr int TO = COUT / RO, TC = CIN / RC;
    static constexpr int PCH = 32;  // pixels per LDS stage
    static_assert(TO * TC == 256 && RO * RC == R, "thread tiling");
};

template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_pw_wgrad(const uint16_t* __restrict__ g, const uint16_t* __restrict__ x,
                                                  size_t npix, size_t chunk, float* __restrict__ part) {
    using C = PwgCfg<CIN, COUT>;
    __shared__ float s_g[C::PCH][COUT + 1];
    __shared__ float s_x[C::PCH][CIN + 1];
    const int t = threadIdx.x;
    const int io = t / C::TC, ic = t - io * C::TC;
    float acc[C::RO][C::RC];
#pragma unroll
    for (int i = 0; i < C::RO; ++i)
#pragma unroll
        for (int j = 0; j < C::RC; ++j) acc[i][j] = 0.f;
    const size_t pb = (size_t)blockIdx.x * chunk, pe = std::min(npix, pb + chunk);
    for (size_t p0 = pb; p0 < pe; p0 += C::PCH) {
        __syncthreads();
        for (int e = t; e < C::PCH * COUT / 8; e += 256) {
            const int pp = e / (COUT / 8), v = e - pp * (COUT / 8);
            float f[8];
            if (p0 + pp < pe) unpack8(*reinterpret_cast<const uint4*>(g + (p0 + pp) * COUT + 8 * v), f);
            else
#pragma unroll
                for (int u = 0; u < 8; ++u) f[u] = 0.f;
#pragma unroll
            for (int u = 0; u < 8; ++u) s_g[pp][8 * v + u] = f[u];
        }
        for (int e = t; e < C::PCH * CIN / 8; e += 256) {
            const int pp = e / (CIN / 8), v = e - pp * (CIN / 8);
            float f[8];
            if (p0 + pp < pe) unpack8(*reinterpret_cast<const uint4*>(x + (p0 + pp) * CIN + 8 * v), f);
            else
#pragma unroll
                for (int u = 0; u < 8; ++u) f[u] = 0.f;
#pragma unroll
            for (int u = 0; u < 8; ++u) s_x[pp][8 * v + u] = f[u];
        }
        __syncthreads();
#pragma unroll 4
        for (int pp = 0; pp < C::PCH; ++pp) {
            float gv[C::RO], xv[C::RC];
#pragma unroll
            for (int i = 0; i < C::RO; ++i) gv[i] = s_g[pp][io * C::RO + i];
#pragma unroll
            for (int j = 0; j < C::RC; ++j) xv[j] = s_x[pp][ic * C::RC + j];
#pragma unroll
            for (int i = 0; i < C::RO; ++i)
#pragma unroll
                for (int j = 0; j < C::RC; ++j) acc[i][j] += gv[i] * xv[j];
        }
    }
    float* out = part + (size_t)blockIdx.x * COUT * CIN;
#pragma unroll
    for (int i = 0; i < C::RO; ++i)
#pragma unroll
        for (int j = 0; j < C::RC; ++j) out[(size_t)(io * C::RO + i) * CIN + ic * C::RC + j] = acc[i][j];
}

template <int CIN, int COUT>
static hh_status pw_wgrad_t(hipStream_t st, hh_ctx* ctx, Buf& part, const uint16_t* g, const uint16_t* x,
                            size_t npix, float* out) {
    const int nblk = (int)std::max<size_t>(1, std::min<size_t>(512, (npix + 255) / 256));
    const size_t chunk = (npix + nblk - 1) / nblk;
    const int count = CIN * COUT;
    HH_TRY(part.ensure(ctx, (size_t)nblk * count * sizeof(float)));
    hipLaunchKernelGGL((k_pw_wgrad<CIN, COUT>), dim3(nblk), dim3(256), 0, st, g, x, npix, chunk, part.as<float>());
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_blocks, dim3((count + 255) / 256), dim3(256), 0, st, part.as<float>(), nblk, count, out);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

hh_status launch_pw_wgrad(hipStream_t st, hh_ctx* ctx, Buf& part, int cin, int cout, const uint16_t* g,
                          const uint16_t* x, size_t npix, float* out) {
#define HH_PWG(CI, CO) \
    if (cin == CI && cout == CO) return pw_wgrad_t<CI, CO>(st, ctx, part, g, x, npix, out);
    HH_PWG(16, 96)
    HH_PWG(96, 16)
    HH_PWG(32, 192)
    HH_PWG(192, 32)
    HH_PWG(64, 384)
    HH_PWG(384, 64)
#undef HH_PWG
    set_error("no pointwise weight-gradient kernel for %d -> %d channels", cin, cout);
    return HH_ERR_ARG;
}

// ---------------------------------------------------------------------------
// Weight gradient of a depthwise layer: gw[c][a][e] = sum_p g[p][c] x[p + (a-1, e-1)][c]
// (zero outside the image).  Thread = 8 channels of a pixel stream; the 9 x 8
// sums are reduced over the block tap by tap through LDS.
// ---------------------------------------------------------------------------
template <int C>
__global__ void __launch_bounds__(256) k_dw_wgrad(const uint16_t* __restrict__ g, const uint16_t* __restrict__ x,
                                                  int B, int H, int W, float* __restrict__ part) {
    constexpr int V = C / 8, R = 256 / V;
    __shared__ float s[256 * 8];
    const int t = threadIdx.x;
    const int v = t % V, r = t / V;
    float acc[9][8];
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[k][u] = 0.f;
    const size_t hw = (size_t)H * W, npix = (size_t)B * hw;
    if (r < R) {
        for (size_t p = (size_t)blockIdx.x * R + r; p < npix; p += (size_t)gridDim.x * R) {
            const int b = (int)(p / hw);
            const int rem = (int)(p - (size_t)b * hw);
            const int i = rem / W, j = rem - i * W;
            float gv[8];
            unpack8(*reinterpret_cast<const uint4*>(g + p * C + 8 * v), gv);
            const uint16_t* xb = x + (size_t)b * hw * C;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int ii = i + k / 3 - 1, jj = j + k % 3 - 1;
                if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
                float xv[8];
                unpack8(*reinterpret_cast<const uint4*>(xb + ((size_t)ii * W + jj) * C + 8 * v), xv);
#pragma unroll
                for (int u = 0; u < 8; ++u) acc[k][u] += gv[u] * xv[u];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 8; ++u) s[t * 8 + u] = (r < R) ? acc[k][u] : 0.f;
        __syncthreads();
        for (int c = t; c < C; c += 256) {
            float sum = 0.f;
            for (int rr = 0; rr < R; ++rr) sum += s[(rr * V + (c >> 3)) * 8 + (c & 7)];
            part[((size_t)blockIdx.x * C + c) * 9 + k] = sum;
        }
    }
}

hh_status launch_dw_wgrad(hipStream_t st, hh_ctx* ctx, Buf& part, int C, const uint16_t* g, const uint16_t* x,
                          int B, int H, int W, float* out) {
    const size_t npix = (size_t)B * H * W;
    const int nblk = (int)std::max<size_t>(1, std::min<size_t>(512, (npix + 255) / 256));
    const int count = C * 9;
    HH_TRY(part.ensure(ctx, (size_t)nblk * count * sizeof(float)));
    if (C == 96)
        hipLaunchKernelGGL(k_dw_wgrad<96>, dim3(nblk), dim3(256), 0, st, g, x, B, H, W, part.as<float>());
    else if (C == 192)
        hipLaunchKernelGGL(k_dw_wgrad<192>, dim3(nblk), dim3(256), 0, st, g, x, B, H, W, part.as<float>());
    else if (C == 384)
        hipLaunchKernelGGL(k_dw_wgrad<384>, dim3(nblk), dim3(256), 0, st, g, x, B, H, W, part.as<float>());
    else {
        set_error("no depthwise weight-gradient kernel for %d channels", C);
        return HH_ERR_ARG;
    }
    HH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_blocks, dim3((count + 255) / 256), dim3(256), 0, st, part.as<float>(), nblk, count, out);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

}  // namespace hh

namespace hh {

// ---------------------------------------------------------------------------
// The inverted bottleneck fused into one kernel (inference): the 6c expanded
// channels never leave LDS.  Per output tile of TH x TW pixels the input
// patch with a one-pixel halo is staged in LDS once; then for every chunk of
// EC = 32 expanded channels:
//   expansion  he = softplus(We x + be) on the halo patch   (MFMA: A = 16 expanded
//              channels x c, B = c x 16 halo pixels), zero outside the image
//              (the depthwise layer's zero padding), BF16 in LDS;
//   depthwise  hw = softplus(dw(he) + bd) on the matrix cores as well: per 16
//              channels, K = 9 taps x 16 channels (5 steps of 32, the last half
//              empty) with a block-diagonal A (the weight w[r][t] where the
//              k index's channel equals the row) and B = the tap-shifted he
//              rows, one 16-byte LDS read per lane and step;
//   shrink     acc += Ws[:, chunk] hw   (MFMA, K = 32): the depthwise result
//              is already in the lane layout of a B operand, with the chunk's
//              channels in the order (4 lg .. 4 lg + 3, 16 + 4 lg .. 16 + 4 lg + 3),
//              which the shrink weights' A fragment follows;
// and finally y = acc + bs + x.  HBM traffic: x once (plus the halo) and y.
// ---------------------------------------------------------------------------
template <int C>
struct IbCfg {
    static constexpr int E = 6 * C;                         // expanded channels
    static constexpr int EC = 32;                           // expanded channels per chunk
    static constexpr int NCH = E / EC;                      // chunks
    static constexpr int TW = C >= 64 ? 16 : 32;            // output tile columns
    static constexpr int TH = 8;                            // output tile rows
    static constexpr int HW_ = TW + 2, HH_ = TH + 2;        // halo patch
    static constexpr int HPX = HW_ * HH_;                   // halo pixels
    static constexpr int HPB = (HPX + 15) / 16;             // 16-pixel blocks of the halo patch
    static constexpr int OPB = TH * TW / 16;                // 16-pixel blocks of the output tile
    static constexpr int PBW = OPB / 4;                     // output blocks per wave
    static constexpr int CT = C / 16;                       // output channel tiles
    static constexpr int XP = C + 8;                        // LDS pitch of a halo pixel (BF16)
    static constexpr int EP = EC + 8;                       // LDS pitch of an expanded pixel / shrink row
    static constexpr int KE = C % 32 == 0 ? 32 : 16;        // k per expansion MFMA
    static constexpr int DS = 5;                            // depthwise k steps (9 taps x 16 channels, padded)
    static_assert(OPB % 4 == 0, "output blocks shared by 4 waves");
};

template <int C>
__global__ void __launch_bounds__(256, 2) k_ib_fused(IbArgs a) {
    using G = IbCfg<C>;
    __shared__ __attribute__((aligned(16))) uint16_t s_x[G::HPB * 16 * G::XP];
    __shared__ __attribute__((aligned(16))) uint16_t s_he[G::HPB * 16 * G::EP];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int lp = lane & 15, lg = lane >> 4;
    const int per_b = a.tiles_x * a.tiles_y;
    auto next_active = [&](int t) {
        while (t < a.ntiles && a.active && !a.active[t / per_b]) t += gridDim.x;
        return t;
    };
    float bsv[G::CT][4];
#pragma unroll
    for (int ct = 0; ct < G::CT; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) bsv[ct][i] = a.bs[ct * 16 + 4 * lg + i];
    // this lane's slot in the depthwise A fragments: the k index 8 lg + j of step s
    // is tap 2 s + (lg >> 1), channel 8 (lg & 1) + j; only j = lp - 8 (lg & 1) can
    // meet the row lp
    const int dj = lp - 8 * (lg & 1);
    // the halo patch of a tile, gathered into registers (zero outside the image):
    // element e = pixel * (C / 8) + vector; the next tile's is in flight while
    // this one is computed
    constexpr int NV = C / 8;
    constexpr int NPF = (G::HPB * 16 * NV + 255) / 256;
    auto gather = [&](int tile, uint4 (&g)[NPF <= 3 ? NPF : 1]) {
        constexpr int NG = NPF <= 3 ? NPF : 1;
        const int b = tile / per_b;
        const int rem = tile - b * per_b;
        const int ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
        const uint16_t* xb = a.x + (size_t)b * a.m * a.m * C;
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            const int e = tid + j * 256;
            const int px = e / NV, v = e - px * NV;
            const int py = px / G::HW_, pxx = px - py * G::HW_;
            const int iy = ty * G::TH - 1 + py, ix = tx * G::TW - 1 + pxx;
            uint4 val = make_uint4(0, 0, 0, 0);
            if (px < G::HPX && iy >= 0 && iy < a.m && ix >= 0 && ix < a.m)
                val = *reinterpret_cast<const uint4*>(xb + ((size_t)iy * a.m + ix) * C + 8 * v);
            g[j] = val;
        }
    };
    constexpr bool PF = NPF <= 3;         // small patches: prefetch the next tile's in registers
    constexpr int NPR = PF ? NPF : 1;
    uint4 pf[NPR];
    int tile = next_active(blockIdx.x);
    if (PF && tile < a.ntiles) gather(tile, pf);
    while (tile < a.ntiles) {
        const int b = tile / per_b;
        const int rem = tile - b * per_b;
        const int ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
        const int y0 = ty * G::TH, x0 = tx * G::TW;
        const int nxt = next_active(tile + gridDim.x);
        __syncthreads();  // the previous tile's readers are done with s_x and s_he
        if constexpr (PF) {
#pragma unroll
            for (int j = 0; j < NPF; ++j) {
                const int e = tid + j * 256;
                if (e < G::HPB * 16 * NV) *reinterpret_cast<uint4*>(&s_x[(e / NV) * G::XP + 8 * (e % NV)]) = pf[j];
            }
            if (nxt < a.ntiles) gather(nxt, pf);
        } else {
            const uint16_t* xb = a.x + (size_t)b * a.m * a.m * C;
            for (int e = tid; e < G::HPB * 16 * NV; e += 256) {
                const int px = e / NV, v = e - px * NV;
                const int py = px / G::HW_, pxx = px - py * G::HW_;
                const int iy = y0 - 1 + py, ix = x0 - 1 + pxx;
                uint4 val = make_uint4(0, 0, 0, 0);
                if (px < G::HPX && iy >= 0 && iy < a.m && ix >= 0 && ix < a.m)
                    val = *reinterpret_cast<const uint4*>(xb + ((size_t)iy * a.m + ix) * C + 8 * v);
                *reinterpret_cast<uint4*>(&s_x[px * G::XP + 8 * v]) = val;
            }
        }
        // halo pixels pb * 16 + lp of this lane inside the image (the expanded map is zero elsewhere)
        uint32_t imask = 0;
#pragma unroll
        for (int pb = 0; pb < G::HPB; ++pb) {
            const int px = pb * 16 + lp;
            const int py = px / G::HW_, pxx = px - py * G::HW_;
            const int iy = y0 - 1 + py, ix = x0 - 1 + pxx;
            if (px < G::HPX && iy >= 0 && iy < a.m && ix >= 0 && ix < a.m) imask |= 1u << pb;
        }
        f32x4 acc[G::CT][G::PBW];
#pragma unroll
        for (int ct = 0; ct < G::CT; ++ct)
#pragma unroll
            for (int q = 0; q < G::PBW; ++q) acc[ct][q] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
        for (int ch = 0; ch < G::NCH; ++ch) {
            const int e0 = ch * G::EC;
            // this chunk's weight fragments and biases, straight from global memory (cached)
            uint4 weA[2][C / G::KE];
            float be8[8];
#pragma unroll
            for (int et = 0; et < 2; ++et) {
#pragma unroll
                for (int kk = 0; kk < C / G::KE; ++kk) {
                    const uint16_t* wr = a.we + (size_t)(e0 + et * 16 + lp) * C + kk * G::KE;
                    if constexpr (G::KE == 32) {
                        weA[et][kk] = *reinterpret_cast<const uint4*>(wr + 8 * lg);
                    } else {
                        const uint2 h = *reinterpret_cast<const uint2*>(wr + 4 * lg);
                        weA[et][kk] = make_uint4(h.x, h.y, 0, 0);
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) be8[4 * et + i] = a.be[e0 + et * 16 + 4 * lg + i];
            }
            float wdv[2][G::DS];
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int st = 0; st < G::DS; ++st) {
                    const int t = 2 * st + (lg >> 1);
                    wdv[g][st] = (t < 9 && dj >= 0 && dj < 8) ? a.wd[(size_t)(e0 + g * 16 + lp) * 9 + t] : 0.f;
                }
            bf16x8 wsA[G::CT];
#pragma unroll
            for (int ct = 0; ct < G::CT; ++ct) {
                const uint16_t* wr = a.ws + (size_t)(ct * 16 + lp) * G::E + e0;
                const uint2 lo = *reinterpret_cast<const uint2*>(wr + 4 * lg);
                const uint2 hi = *reinterpret_cast<const uint2*>(wr + 16 + 4 * lg);
                const uint4 u4 = make_uint4(lo.x, lo.y, hi.x, hi.y);
                wsA[ct] = *reinterpret_cast<const bf16x8*>(&u4);
            }
            float bd8[8];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bd8[i] = a.bd[e0 + 4 * lg + i];
                bd8[4 + i] = a.bd[e0 + 16 + 4 * lg + i];
            }
            if (ch > 0) __syncthreads();  // the previous chunk's depthwise is done with s_he
            // ---- expansion on the halo patch: (EC / 16) x HPB MFMA tiles over the 4 waves
#pragma unroll 2
            for (int pr = wave; pr < 2 * G::HPB; pr += 4) {
                const int et = pr >= G::HPB ? 1 : 0;
                const int pb = pr - et * G::HPB;
                f32x4 d = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kk = 0; kk < C / G::KE; ++kk) {
                    const uint4 A = et ? weA[1][kk] : weA[0][kk];
                    if constexpr (G::KE == 32) {
                        const uint4 bv = *reinterpret_cast<const uint4*>(&s_x[(pb * 16 + lp) * G::XP + kk * 32 + 8 * lg]);
                        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(&A),
                                                                    *reinterpret_cast<const bf16x8*>(&bv), d, 0, 0, 0);
                    } else {
                        const uint2 av = make_uint2(A.x, A.y);
                        const uint2 bv = *reinterpret_cast<const uint2*>(&s_x[(pb * 16 + lp) * G::XP + 4 * lg]);
                        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(*reinterpret_cast<const s16x4*>(&av),
                                                                      *reinterpret_cast<const s16x4*>(&bv), d, 0, 0, 0);
                    }
                }
                // lane: expanded channels et*16 + 4 lg .. +3 of halo pixel pb*16 + lp
                const bool inside = (imask >> pb) & 1u;
                float o[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) o[i] = inside ? softplus_f(d[i] + (et ? be8[4 + i] : be8[i])) : 0.f;
                *reinterpret_cast<uint2*>(&s_he[(pb * 16 + lp) * G::EP + et * 16 + 4 * lg]) =
                    make_uint2(f2bf2(o[0], o[1]), f2bf2(o[2], o[3]));
            }
            // depthwise A fragments of this chunk (block-diagonal, BF16 weights)
            bf16x8 dA[2][G::DS];
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int st = 0; st < G::DS; ++st) {
                    const float w = wdv[g][st];
                    uint32_t wv[4];
#pragma unroll
                    for (int h = 0; h < 4; ++h)
                        wv[h] = f2bf2(2 * h == dj ? w : 0.f, 2 * h + 1 == dj ? w : 0.f);
                    const uint4 u4 = make_uint4(wv[0], wv[1], wv[2], wv[3]);
                    dA[g][st] = *reinterpret_cast<const bf16x8*>(&u4);
                }
            __syncthreads();  // s_he complete
            // all of this wave's pixel blocks advance together through the 5 steps:
            // 2 PBW independent accumulation chains keep the matrix cores fed
            f32x4 dd[G::PBW][2];
#pragma unroll
            for (int q = 0; q < G::PBW; ++q) dd[q][0] = dd[q][1] = (f32x4){0.f, 0.f, 0.f, 0.f};
            // tap offset of this lane's k slots in each step (tap 2 st + (lg >> 1))
#pragma unroll
            for (int st = 0; st < G::DS; ++st) {
                const int t = 2 * st + (lg >> 1);
                const int toff = (t / 3) * G::HW_ + t % 3;
                uint4 r[G::PBW][2];
#pragma unroll
                for (int q = 0; q < G::PBW; ++q) {
                    const int p = (wave * G::PBW + q) * 16 + lp;  // output pixel of the tile
                    const int oy = p / G::TW, ox = p - oy * G::TW;
                    const int hp = oy * G::HW_ + ox + toff;
                    r[q][0] = r[q][1] = make_uint4(0, 0, 0, 0);
                    if (t < 9) {
                        r[q][0] = *reinterpret_cast<const uint4*>(&s_he[hp * G::EP + 8 * (lg & 1)]);
                        r[q][1] = *reinterpret_cast<const uint4*>(&s_he[hp * G::EP + 16 + 8 * (lg & 1)]);
                    }
                }
#pragma unroll
                for (int q = 0; q < G::PBW; ++q)
#pragma unroll
                    for (int g = 0; g < 2; ++g)
                        dd[q][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            dA[g][st], *reinterpret_cast<const bf16x8*>(&r[q][g]), dd[q][g], 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < G::PBW; ++q) {
                float hv[8];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    hv[i] = softplus_f(dd[q][0][i] + bd8[i]);
                    hv[4 + i] = softplus_f(dd[q][1][i] + bd8[4 + i]);
                }
                const uint4 hb = pack8(hv);
#pragma unroll
                for (int ct = 0; ct < G::CT; ++ct)
                    acc[ct][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        wsA[ct], *reinterpret_cast<const bf16x8*>(&hb), acc[ct][q], 0, 0, 0);
            }
        }
        // ---- y = acc + bs + x: lane holds channels ct*16 + 4 lg .. +3 of pixel p
#pragma unroll
        for (int q = 0; q < G::PBW; ++q) {
            const int p = (wave * G::PBW + q) * 16 + lp;
            const int oy = p / G::TW, ox = p - oy * G::TW;
            const int iy = y0 + oy, ix = x0 + ox;
            if (iy >= a.m || ix >= a.m) continue;
            const int hp = (oy + 1) * G::HW_ + ox + 1;
#pragma unroll
            for (int ct = 0; ct < G::CT; ++ct) {
                const int co = ct * 16 + 4 * lg;
                const uint2 r2 = *reinterpret_cast<const uint2*>(&s_x[hp * G::XP + co]);
                const float v0 = acc[ct][q][0] + bsv[ct][0] + bf2f((uint16_t)(r2.x & 0xffff));
                const float v1 = acc[ct][q][1] + bsv[ct][1] + bf2f((uint16_t)(r2.x >> 16));
                const float v2 = acc[ct][q][2] + bsv[ct][2] + bf2f((uint16_t)(r2.y & 0xffff));
                const float v3 = acc[ct][q][3] + bsv[ct][3] + bf2f((uint16_t)(r2.y >> 16));
                *reinterpret_cast<uint2*>(a.y + (((size_t)b * a.m + iy) * a.m + ix) * C + co) =
                    make_uint2(f2bf2(v0, v1), f2bf2(v2, v3));
            }
        }
        tile = nxt;
    }
}

template <int C>
static hh_status launch_ib_t(hipStream_t st, int num_cus, IbArgs a) {
    using G = IbCfg<C>;
    a.tiles_x = (a.m + G::TW - 1) / G::TW;
    a.tiles_y = (a.m + G::TH - 1) / G::TH;
    a.ntiles = a.B * a.tiles_x * a.tiles_y;
    if (a.ntiles == 0) return HH_OK;
    const int grid = std::min(a.ntiles, num_cus * 2);
    hipLaunchKernelGGL(k_ib_fused<C>, dim3(grid), dim3(256), 0, st, a);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

hh_status launch_ib_fused(hipStream_t st, int num_cus, int c, IbArgs a) {
    if (c == 16) return launch_ib_t<16>(st, num_cus, a);
    if (c == 32) return launch_ib_t<32>(st, num_cus, a);
    if (c == 64) return launch_ib_t<64>(st, num_cus, a);
    set_error("no fused bottleneck kernel for %d channels", c);
    return HH_ERR_ARG;
}

}  // namespace hh
