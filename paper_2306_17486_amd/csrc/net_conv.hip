// Convolutions of the encoder-solver network on gfx950 (Sec. 3.3, eq. 9; the
// 3x3 layers of Sec. 4.1 / 5.3).  Activations are BF16 NHWC [b][y][x][c].
//
// Every 16/32/64-channel 3x3 convolution -- forward and input gradient -- is
// one implicit GEMM on the matrix cores: out[p][o] = sum_k Wg[k][o] * in[src(p,k)],
// k = tap * CIN + ci, with v_mfma_f32_16x16x32_bf16 (FP32 accumulation):
//   A operand = 16 output channels x 32 k   (the packed weights, held in VGPRs)
//   B operand = 32 k x 16 output pixels      (8 consecutive channels per lane from LDS)
//   D         = 16 channels x 16 pixels      (each lane owns 4 consecutive channels of one pixel)
// Modes: S1 (stride 1), S2 (stride 2, the downsampling layers), T2 (stride-2
// transposed convolution, evaluated as a stride-1 convolution over the
// zero-interleaved input with flipped weights).  The input gradients of the
// three layer kinds are again S1/S2/T2 convolutions with repacked weights.
// The epilogue fuses bias, a sum skip connection, the activation (ReLU, or
// softplus for the lightweight network), and (backward) the ReLU mask of the
// tensor whose gradient is produced.
#include <map>
#include <mutex>

#include "net.h"

namespace hh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Weight packing: FP32 layer weights -> BF16 chunks Wp[ch][o][32] of the
// gather form Wg[tap][o][i] (k = tap * CIN + i, zero beyond tap 8).
//   direct:   Wg[t][o][i] = W[o][i][t]       (W's first index is the output channel)
//   flipped:  Wg[t][o][i] = W[i][o][8 - t]   (W's first index is the input channel)
// ---------------------------------------------------------------------------
__global__ void k_pack_weights(const float* __restrict__ W, uint16_t* __restrict__ Wp, int cin, int cout, int flipped,
                               int nch) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = nch * cout * 32;
    if (e >= total) return;
    const int kk = e % 32, o = (e / 32) % cout, ch = e / (32 * cout);
    const int k = ch * 32 + kk;
    const int t = k / cin, i = k % cin;
    float v = 0.f;
    if (t < 9) v = flipped ? W[((size_t)i * cout + o) * 9 + (8 - t)] : W[((size_t)o * cin + i) * 9 + t];
    Wp[e] = f2bf(v);
}

// Split packing for a layer with cout_real < cout output channels kept in FP32
// precision: Wp_hi = BF16(W), Wp_lo = BF16(W - Wp_hi) (together 16 significant
// bits), output channels cout_real .. cout-1 zero.
__global__ void k_pack_weights_split(const float* __restrict__ W, uint16_t* __restrict__ Wp_hi,
                                     uint16_t* __restrict__ Wp_lo, int cin, int cout_real, int cout, int nch) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = nch * cout * 32;
    if (e >= total) return;
    const int kk = e % 32, o = (e / 32) % cout, ch = e / (32 * cout);
    const int k = ch * 32 + kk;
    const int t = k / cin, i = k % cin;
    const float v = (t < 9 && o < cout_real) ? W[((size_t)o * cin + i) * 9 + t] : 0.f;
    const uint16_t hi = f2bf(v);
    Wp_hi[e] = hi;
    Wp_lo[e] = f2bf(v - bf2f(hi));
}

// ---------------------------------------------------------------------------
// The MFMA convolution.  PROJ: the projection layer (16 -> 2 channels): the
// weights as a BF16 high and low part (two MFMAs per k chunk, products of the
// BF16 activations exact, so the layer keeps its FP32 weights to 2^-17), and
// the output as FP32 (re, im) pairs.
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int MODE, int TR_ = 0>
struct ConvCfg {
    static constexpr int TC = 32;                                               // output tile columns
    // output tile rows (TR_ = 0: the default of the shape)
    static constexpr int TR = TR_ > 0 ? TR_
                                      : (MODE == CM_S2) ? (CIN >= 32 ? 2 : 4) : (CIN >= 64 ? 2 : (CIN >= 32 ? 4 : 16));
    static constexpr int NT = COUT / 16;                                        // channel tiles
    // channel tiles per wave: a pixel fragment read from LDS feeds CT MFMAs;
    // the weights' VGPRs (CT * NCH * 4) stay within 72 so that two or more
    // waves per SIMD remain resident
    static constexpr int NCH = (9 * CIN + 31) / 32;                             // k chunks
    static constexpr int CT = (NT >= 2 && 2 * NCH <= 18) ? 2 : 1;
    static constexpr int NG = NT / CT;                                          // channel groups
    static constexpr int WPT = 4 / NG;                                          // waves per channel group
    static constexpr int PB = TR * (TC / 16);                                   // 16-pixel blocks per tile
    static constexpr int PBW = PB / WPT;                                        // pixel blocks per wave
    static constexpr int PH = (MODE == CM_S2) ? 2 * TR + 1 : TR + 2;            // staged input rows
    static constexpr int PW = (MODE == CM_S2) ? 2 * TC + 1 : TC + 2;            // staged input cols
    static constexpr int CP = CIN + 8;                                          // LDS channel pitch (bf16)
    static constexpr int LDS_BYTES = PH * PW * CP * 2;
};

// One lane's epilogue: four consecutive output channels of one pixel at element
// offset off of its batch entry (one entry holds fewer than 2^31 elements):
// bias, sum skip, activation, ReLU-derivative mask, BF16 store and the optional
// FP32 copy.  yb / yfb / kb / mb: the entry's output, FP32 copy, skip and mask
// tensors (uniform per tile; the last three may be null).
__device__ __forceinline__ void conv_epilogue4(const f32x4& acc, const float (&bias)[4], int act, uint16_t* yb,
                                               float* yfb, const uint16_t* kb, const uint16_t* mb, int off) {
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = acc[i] + bias[i];
    if (kb) {
        const uint2 s2 = *reinterpret_cast<const uint2*>(kb + off);
        v[0] += bf2f((uint16_t)(s2.x & 0xffff));
        v[1] += bf2f((uint16_t)(s2.x >> 16));
        v[2] += bf2f((uint16_t)(s2.y & 0xffff));
        v[3] += bf2f((uint16_t)(s2.y >> 16));
    }
    if (act == ACT_RELU) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = fmaxf(v[i], 0.f);
    } else if (act == ACT_SOFTPLUS) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = softplus_f(v[i]);
    }
    if (mb) {
        const uint2 m2 = *reinterpret_cast<const uint2*>(mb + off);
        if (!(bf2f((uint16_t)(m2.x & 0xffff)) > 0.f)) v[0] = 0.f;
        if (!(bf2f((uint16_t)(m2.x >> 16)) > 0.f)) v[1] = 0.f;
        if (!(bf2f((uint16_t)(m2.y & 0xffff)) > 0.f)) v[2] = 0.f;
        if (!(bf2f((uint16_t)(m2.y >> 16)) > 0.f)) v[3] = 0.f;
    }
    uint2 o2;
    o2.x = f2bf2(v[0], v[1]);
    o2.y = f2bf2(v[2], v[3]);
    *reinterpret_cast<uint2*>(yb + off) = o2;
    if (yfb) *reinterpret_cast<float4*>(yfb + off) = make_float4(v[0], v[1], v[2], v[3]);
}

// a tile's per-entry tensor bases for conv_epilogue4
struct EpiBases {
    uint16_t* yb;
    float* yfb;
    const uint16_t* kb;
    const uint16_t* mb;
};
template <int COUT>
__device__ __forceinline__ EpiBases epi_bases(const ConvArgs& a, int b) {
    const size_t per = (size_t)a.Hout * a.Wout * COUT;
    const int sb = a.skip ? (a.skip_map ? a.skip_map[b] : b) : 0;
    return EpiBases{a.y + b * per, a.yf ? a.yf + b * per : nullptr, a.skip ? a.skip + sb * per : nullptr,
                    a.mask ? a.mask + b * per : nullptr};
}

template <int CIN, int COUT, int MODE, bool PROJ = false, int TR_ = 0>
__global__ void __launch_bounds__(256, 2) k_conv_mfma(ConvArgs a) {  // >= 2 waves per SIMD resident
    using C = ConvCfg<CIN, COUT, MODE, TR_>;
    static_assert(!PROJ || (CIN == 16 && COUT == 16 && MODE == CM_S1 && C::CT == 1 && C::NG == 1),
                  "projection: one 16-channel tile, stride 1");
    __shared__ __attribute__((aligned(16))) uint16_t s_in[C::PH * C::PW * C::CP];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int cg = wave % C::NG;           // channel group of this wave: tiles cg*CT .. cg*CT+CT-1
    const int wsub = wave / C::NG;         // which share of the pixel blocks
    const int lp = lane & 15, lg = lane >> 4;

    // this wave's weights stay in VGPRs for all tiles
    bf16x8 wreg[C::CT][C::NCH];
    bf16x8 wlo[PROJ ? C::NCH : 1];
    {
        const uint4* wp4 = reinterpret_cast<const uint4*>(a.wp);
#pragma unroll
        for (int c = 0; c < C::CT; ++c)
#pragma unroll
            for (int ch = 0; ch < C::NCH; ++ch) {
                uint4 v = wp4[((size_t)ch * COUT + (cg * C::CT + c) * 16 + lp) * 4 + lg];
                wreg[c][ch] = *reinterpret_cast<bf16x8*>(&v);
            }
        if (PROJ) {
            const uint4* wl4 = reinterpret_cast<const uint4*>(a.wp_lo);
#pragma unroll
            for (int ch = 0; ch < C::NCH; ++ch) {
                uint4 v = wl4[((size_t)ch * COUT + lp) * 4 + lg];
                wlo[ch] = *reinterpret_cast<bf16x8*>(&v);
            }
        }
    }
    float bias4[C::CT][4];
#pragma unroll
    for (int c = 0; c < C::CT; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = (cg * C::CT + c) * 16 + 4 * lg + i;
            bias4[c][i] = (a.bias && (!PROJ || co < 2)) ? a.bias[co] : 0.f;
        }
    wait_all_memory();

    // ---- the input patch of a tile (zero padding / zero interleaving), gathered
    // into registers: element e = pixel * VEC + v of the PH x PW patch ----
    constexpr int VEC = CIN / 8;
    constexpr int NE = C::PH * C::PW * VEC;
    constexpr int NPF = (NE + 255) / 256;  // gathers per thread
    constexpr bool PF = NPF <= 6;           // small patches: the next tile's gather overlaps this tile's MFMAs
    const int per_b = a.tiles_x * a.tiles_y;
    // element e of a tile's patch (zero outside the input)
    auto elem = [&](int tile, int e) -> uint4 {
        const int b = tile / per_b;
        const int rem = tile - b * per_b;
        const int ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
        const int y0 = ty * C::TR, x0 = tx * C::TC;
        const uint16_t* xb = a.x + (size_t)b * a.Hin * a.Win * CIN;
        {
            const int v = e % VEC, pix = e / VEC;
            const int py = pix / C::PW, px = pix - py * C::PW;
            int iy, ix;
            bool in;
            if (MODE == CM_S1) {
                iy = y0 - 1 + py;
                ix = x0 - 1 + px;
                in = iy >= 0 && iy < a.Hin && ix >= 0 && ix < a.Win;
            } else if (MODE == CM_S2) {
                iy = 2 * y0 - 1 + py;
                ix = 2 * x0 - 1 + px;
                in = iy >= 0 && iy < a.Hin && ix >= 0 && ix < a.Win;
            } else {  // T2: u[2i][2j] = x[i][j]
                const int uy = y0 - 1 + py, ux = x0 - 1 + px;
                in = uy >= 0 && ux >= 0 && !(uy & 1) && !(ux & 1) && (uy >> 1) < a.Hin && (ux >> 1) < a.Win;
                iy = uy >> 1;
                ix = ux >> 1;
            }
            uint4 val = make_uint4(0, 0, 0, 0);
            if (e < NE && in) val = *reinterpret_cast<const uint4*>(xb + (iy * a.Win + ix) * CIN + 8 * v);
            return val;
        }
    };
    auto to_lds = [&](int e, uint4 val) {
        const int v = e % VEC, pix = e / VEC;
        *reinterpret_cast<uint4*>(&s_in[pix * C::CP + 8 * v]) = val;
    };
    constexpr int NPR = PF ? NPF : 1;  // registers held between tiles
    auto gather = [&](int tile, uint4 (&g)[NPR]) {
#pragma unroll
        for (int j = 0; j < NPR; ++j) g[j] = elem(tile, tid + j * 256);
    };
    auto put = [&](const uint4 (&g)[NPR]) {
#pragma unroll
        for (int j = 0; j < NPR; ++j)
            if (tid + j * 256 < NE) to_lds(tid + j * 256, g[j]);
    };
    // the next tile of this workgroup whose batch entry is active (uniform)
    auto next_active = [&](int t) {
        while (t < a.ntiles && a.active && !a.active[t / per_b]) t += gridDim.x;
        return t;
    };
    uint4 pf[NPR];
    int tile = next_active(blockIdx.x);
    if (PF && tile < a.ntiles) gather(tile, pf);
    while (tile < a.ntiles) {
        const int b = tile / per_b;
        const int rem = tile - b * per_b;
        const int ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
        const int y0 = ty * C::TR, x0 = tx * C::TC;
        const int nxt = next_active(tile + gridDim.x);
        __syncthreads();  // previous tile's readers are done with s_in
        if (PF) {
            put(pf);
        } else {
            // four loads of this thread in flight at a time
            for (int e0 = tid; e0 < NE; e0 += 4 * 256) {
                uint4 v4[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) v4[k] = elem(tile, e0 + k * 256);
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (e0 + k * 256 < NE) to_lds(e0 + k * 256, v4[k]);
            }
        }
        __syncthreads();
        if (PF && nxt < a.ntiles) gather(nxt, pf);  // in flight during the MFMAs below
        // ---- MFMA over the k chunks ----
        f32x4 acc[C::PBW][C::CT];
#pragma unroll
        for (int q = 0; q < C::PBW; ++q)
#pragma unroll
            for (int c = 0; c < C::CT; ++c) acc[q][c] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < C::NCH; ++ch) {
            const int k0 = ch * 32 + 8 * lg;
            const int tap = k0 / CIN, ci = k0 % CIN;
            const int ky = tap / 3, kx = tap - 3 * ky;
#pragma unroll
            for (int q = 0; q < C::PBW; ++q) {
                const int pbk = wsub * C::PBW + q;          // pixel block in the tile
                const int ry = pbk / (C::TC / 16), rx = (pbk % (C::TC / 16)) * 16 + lp;
                bf16x8 bv;
                if (tap < 9) {
                    int sy, sx;
                    if (MODE == CM_S2) {
                        sy = 2 * ry + ky;
                        sx = 2 * rx + kx;
                    } else {
                        sy = ry + ky;
                        sx = rx + kx;
                    }
                    uint4 raw = *reinterpret_cast<const uint4*>(&s_in[(sy * C::PW + sx) * C::CP + ci]);
                    bv = *reinterpret_cast<bf16x8*>(&raw);
                } else {
                    uint4 z = make_uint4(0, 0, 0, 0);
                    bv = *reinterpret_cast<bf16x8*>(&z);
                }
#pragma unroll
                for (int c = 0; c < C::CT; ++c)
                    acc[q][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wreg[c][ch], bv, acc[q][c], 0, 0, 0);
                if (PROJ) acc[q][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wlo[ch], bv, acc[q][0], 0, 0, 0);
            }
        }
        if constexpr (PROJ) {
            // lanes with lg == 0 hold output channels 0 (re) and 1 (im)
#pragma unroll
            for (int q = 0; q < C::PBW; ++q) {
                const int pbk = wsub * C::PBW + q;
                const int ry = pbk / (C::TC / 16), rx = (pbk % (C::TC / 16)) * 16 + lp;
                const int oy = y0 + ry, ox = x0 + rx;
                if (lg != 0 || oy >= a.Hout || ox >= a.Wout) continue;
                a.yproj[((size_t)b * a.Hout + oy) * a.Wout + ox] =
                    make_float2(acc[q][0][0] + bias4[0][0], acc[q][0][1] + bias4[0][1]);
            }
            tile = nxt;
            continue;
        }
        // ---- epilogue: lane owns channels (cg*CT + c)*16 + 4 lg .. +3 of one pixel per block ----
        const EpiBases eb = epi_bases<COUT>(a, b);
#pragma unroll
        for (int q = 0; q < C::PBW; ++q)
#pragma unroll
        for (int c = 0; c < C::CT; ++c) {
            const int co = (cg * C::CT + c) * 16 + 4 * lg;
            const int pbk = wsub * C::PBW + q;
            const int ry = pbk / (C::TC / 16), rx = (pbk % (C::TC / 16)) * 16 + lp;
            const int oy = y0 + ry, ox = x0 + rx;
            if (oy >= a.Hout || ox >= a.Wout) continue;
            conv_epilogue4(acc[q][c], bias4[c], a.act, eb.yb, eb.yfb, eb.kb, eb.mb, (oy * a.Wout + ox) * COUT + co);
        }
        tile = nxt;
    }
}

// ---------------------------------------------------------------------------
// The same convolution (S1 / S2) with the input patch copied from HBM straight
// into LDS by buffer loads (buffer_load_dwordx4 ... lds: 16 bytes per lane,
// no VGPR staging), so that tiles can be taller without the registers the
// prefetch above needs.  Out-of-range offsets read as zero (the buffer's
// range check), which gives the zero padding.
//
// LDS layout: slot q = 16 bytes; pixel P of the patch owns slots P*S .. P*S+S-1
// (S = CIN/8 vectors of 8 channels), vector j stored in slot P*S + (j ^ f(P)),
// f(P) = (P / (16/S)) mod S.  A B-operand read takes vector j of 16
// consecutive pixels; P mod 16 decides both the 256-byte bank row offset and
// the swizzle, so those 16 reads hit 16 distinct 16-byte bank groups.
// Each wave's buffer load fills 64 consecutive slots (lane l -> slot base + l);
// the lane loads whatever vector that slot holds under the swizzle.
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int MODE, int TR_>
struct DmaCfg {
    static constexpr int TC = 32;                                   // output tile columns
    static constexpr int TR = TR_;                                  // output tile rows
    static constexpr int NT = COUT / 16;                            // channel tiles
    static constexpr int NCH = (9 * CIN + 31) / 32;                 // k chunks
    static constexpr int CT = (NT >= 2 && 2 * NCH <= 18) ? 2 : 1;   // channel tiles per wave
    static constexpr int NG = NT / CT;                              // channel groups
    static constexpr int WPT = 4 / NG;                              // waves per channel group
    static constexpr int PB = TR * (TC / 16);                       // 16-pixel blocks per tile
    static constexpr int PBW = PB / WPT;                            // pixel blocks per wave
    static constexpr int PH = (MODE == CM_S2) ? 2 * TR + 1 : TR + 2;
    static constexpr int PW = (MODE == CM_S2) ? 2 * TC + 1 : TC + 2;
    static constexpr int S = CIN / 8;                               // 16-byte vectors per pixel
    static constexpr int SH = S == 2 ? 3 : (S == 4 ? 2 : 1);        // log2(16 / S)
    static constexpr int NSLOT = PH * PW * S;
    static constexpr int NROUND = (NSLOT + 255) / 256;
    static_assert(S == 2 || S == 4 || S == 8, "16, 32 or 64 input channels");
    static_assert(PB % WPT == 0, "pixel blocks shared evenly");
    static_assert(NROUND <= 15, "buffer loads per thread fit the vmcnt wait immediate");
};

__device__ __forceinline__ int dma_slot(int P, int j, int S, int SH) { return P * S + (j ^ ((P >> SH) & (S - 1))); }

template <int CIN, int COUT, int MODE, int TR>
__global__ void __launch_bounds__(256) k_conv_dma(ConvArgs a) {
    using C = DmaCfg<CIN, COUT, MODE, TR>;
    __shared__ __attribute__((aligned(16))) uint4 s_in[C::NROUND * 256];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int cg = wave % C::NG;
    const int wsub = wave / C::NG;
    const int lp = lane & 15, lg = lane >> 4;

    bf16x8 wreg[C::CT][C::NCH];
    {
        const uint4* wp4 = reinterpret_cast<const uint4*>(a.wp);
#pragma unroll
        for (int c = 0; c < C::CT; ++c)
#pragma unroll
            for (int ch = 0; ch < C::NCH; ++ch) {
                uint4 v = wp4[((size_t)ch * COUT + (cg * C::CT + c) * 16 + lp) * 4 + lg];
                wreg[c][ch] = *reinterpret_cast<bf16x8*>(&v);
            }
    }
    float bias4[C::CT][4];
#pragma unroll
    for (int c = 0; c < C::CT; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i) bias4[c][i] = a.bias ? a.bias[(cg * C::CT + c) * 16 + 4 * lg + i] : 0.f;
    wait_all_memory();

    const int per_b = a.tiles_x * a.tiles_y;
    const uint32_t bytes_b = (uint32_t)a.Hin * a.Win * CIN * 2;
    auto next_active = [&](int t) {
        while (t < a.ntiles && a.active && !a.active[t / per_b]) t += gridDim.x;
        return t;
    };
    int tile = next_active(blockIdx.x);
    while (tile < a.ntiles) {
        const int b = tile / per_b;
        const int rem = tile - b * per_b;
        const int ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
        const int y0 = ty * C::TR, x0 = tx * C::TC;
        const int nxt = next_active(tile + gridDim.x);
        __syncthreads();  // the previous tile's readers are done with s_in
        {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(a.x + (size_t)b * a.Hin * a.Win * CIN), (short)0, (int)bytes_b, 0x00020000);
#pragma unroll
            for (int r = 0; r < C::NROUND; ++r) {
                const int q = r * 256 + tid;
                const int P = q / C::S, jp = q - P * C::S;
                const int j = jp ^ ((P >> C::SH) & (C::S - 1));
                const int py = P / C::PW, px = P - py * C::PW;
                const int iy = (MODE == CM_S2 ? 2 * y0 : y0) - 1 + py;
                const int ix = (MODE == CM_S2 ? 2 * x0 : x0) - 1 + px;
                const bool in = q < C::NSLOT && iy >= 0 && iy < a.Hin && ix >= 0 && ix < a.Win;
                const int off = in ? ((iy * a.Win + ix) * CIN + 8 * j) * 2 : 0x7ffffff0;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rs, (__attribute__((address_space(3))) void*)(s_in + r * 256 + wave * 64), 16, off, 0, 0, 0);
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        }
        __syncthreads();
        f32x4 acc[C::PBW][C::CT];
#pragma unroll
        for (int q = 0; q < C::PBW; ++q)
#pragma unroll
            for (int c = 0; c < C::CT; ++c) acc[q][c] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < C::NCH; ++ch) {
            const int k0 = ch * 32 + 8 * lg;
            const int tap = k0 / CIN, ci = k0 % CIN;
            const int ky = tap / 3, kx = tap - 3 * ky;
#pragma unroll
            for (int q = 0; q < C::PBW; ++q) {
                const int pbk = wsub * C::PBW + q;
                const int ry = pbk / (C::TC / 16), rx = (pbk % (C::TC / 16)) * 16 + lp;
                bf16x8 bv;
                if (tap < 9) {
                    const int sy = (MODE == CM_S2 ? 2 * ry : ry) + ky;
                    const int sx = (MODE == CM_S2 ? 2 * rx : rx) + kx;
                    const uint4 raw = s_in[dma_slot(sy * C::PW + sx, ci >> 3, C::S, C::SH)];
                    bv = *reinterpret_cast<const bf16x8*>(&raw);
                } else {
                    const uint4 z = make_uint4(0, 0, 0, 0);
                    bv = *reinterpret_cast<const bf16x8*>(&z);
                }
#pragma unroll
                for (int c = 0; c < C::CT; ++c)
                    acc[q][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wreg[c][ch], bv, acc[q][c], 0, 0, 0);
            }
        }
        const EpiBases eb = epi_bases<COUT>(a, b);
#pragma unroll
        for (int q = 0; q < C::PBW; ++q)
#pragma unroll
            for (int c = 0; c < C::CT; ++c) {
                const int co = (cg * C::CT + c) * 16 + 4 * lg;
                const int pbk = wsub * C::PBW + q;
                const int ry = pbk / (C::TC / 16), rx = (pbk % (C::TC / 16)) * 16 + lp;
                const int oy = y0 + ry, ox = x0 + rx;
                if (oy >= a.Hout || ox >= a.Wout) continue;
                conv_epilogue4(acc[q][c], bias4[c], a.act, eb.yb, eb.yfb, eb.kb, eb.mb,
                               (oy * a.Wout + ox) * COUT + co);
            }
        tile = nxt;
    }
}

// ---------------------------------------------------------------------------
// Stride-2 transposed convolution by output parity.  With u the zero-interleaved
// input (u[2i][2j] = x[i][j]), out[oy][ox] = sum_t Wg[t] u[oy + ky - 1][ox + kx - 1]
// only meets nonzero u where oy + ky - 1 and ox + kx - 1 are even: an even output
// row uses tap row ky = 1 only, an odd one ky = 0 and 2 (the same for columns).
// So each 16-pixel block takes 16 outputs of one row with one column parity
// (ox = x0 + px + 2 l); the four parity classes use 1, 2, 2 and 4 taps, 9 per
// four outputs instead of 36.  Every chunk is one tap x 32 input channels, so
// the weights are the same packed chunks as the interleaved form's.
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int TR_ = 0>
struct T2Cfg {
    static constexpr int TC = 32;                        // output tile columns
    static constexpr int TR = TR_ > 0 ? TR_ : (CIN >= 64 ? 4 : 8);  // output tile rows (even; TR_ = 0: default)
    static constexpr int NT = COUT / 16;                 // channel tiles
    static constexpr int WPT = 4 / NT;                   // waves per channel tile
    static constexpr int PB = TR * 2;                    // (row, column parity) blocks
    static constexpr int PBW = PB / WPT;                 // blocks per wave
    static constexpr int CB = CIN / 32;                  // 32-channel blocks per tap
    static constexpr int NCH = 9 * CB;                   // weight chunks
    static constexpr int PH = TR / 2 + 1;                // staged input rows y0/2 .. y0/2 + TR/2
    static constexpr int PW = TC / 2 + 1;                // staged input cols x0/2 .. x0/2 + TC/2
    static constexpr int CP = CIN + 8;                   // LDS channel pitch (bf16)
    static_assert(CIN % 32 == 0, "one tap per weight chunk");
    static_assert(PBW % 4 == 0, "row and column parity of a block fixed at compile time");
};

template <int CIN, int COUT, int TR_ = 0>
__global__ void __launch_bounds__(256) k_conv_t2(ConvArgs a) {
    using C = T2Cfg<CIN, COUT, TR_>;
    __shared__ __attribute__((aligned(16))) uint16_t s_in[C::PH * C::PW * C::CP];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int ct = wave % C::NT;
    const int wsub = wave / C::NT;
    const int lp = lane & 15, lg = lane >> 4;

    bf16x8 wreg[C::NCH];
    {
        const uint4* wp4 = reinterpret_cast<const uint4*>(a.wp);
#pragma unroll
        for (int ch = 0; ch < C::NCH; ++ch) {
            uint4 v = wp4[((size_t)ch * COUT + ct * 16 + lp) * 4 + lg];
            wreg[ch] = *reinterpret_cast<bf16x8*>(&v);
        }
    }
    float bias4[4] = {0.f, 0.f, 0.f, 0.f};
    if (a.bias)
#pragma unroll
        for (int i = 0; i < 4; ++i) bias4[i] = a.bias[ct * 16 + 4 * lg + i];
    wait_all_memory();

    // the input patch, gathered into registers one active tile ahead while
    // the current tile's MFMAs run; not for 64 -> 64, whose extra registers
    // would cost a resident wave per SIMD
    constexpr int VEC = CIN / 8;
    constexpr int NE = C::PH * C::PW * VEC;
    constexpr bool PF = !(CIN == 64 && COUT == 64);
    constexpr int NPF = PF ? (NE + 255) / 256 : 1;
    static_assert(!PF || NPF <= 5, "patch gathered into registers");
    const int per_b = a.tiles_x * a.tiles_y;
    auto gather = [&](int tile, uint4 (&g)[NPF]) {
        const int b = tile / per_b;
        const int rem = tile - b * per_b;
        const int ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
        const int y0 = ty * C::TR, x0 = tx * C::TC;
        const uint16_t* xb = a.x + (size_t)b * a.Hin * a.Win * CIN;
#pragma unroll
        for (int j = 0; j < NPF; ++j) {
            const int e = tid + j * 256;
            const int v = e % VEC, pix = e / VEC;
            const int py = pix / C::PW, px = pix - py * C::PW;
            const int iy = (y0 >> 1) + py, ix = (x0 >> 1) + px;
            g[j] = make_uint4(0, 0, 0, 0);
            if (e < NE && iy < a.Hin && ix < a.Win)
                g[j] = *reinterpret_cast<const uint4*>(xb + (iy * a.Win + ix) * CIN + 8 * v);
        }
    };
    // without prefetch: gather and store element by element
    auto stage_now = [&](int tile) {
        const int b = tile / per_b;
        const int rem = tile - b * per_b;
        const int ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
        const int y0 = ty * C::TR, x0 = tx * C::TC;
        const uint16_t* xb = a.x + (size_t)b * a.Hin * a.Win * CIN;
        // all of this thread's loads issued before its first store
        constexpr int NJ = (NE + 255) / 256;
        uint4 val[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int e = tid + j * 256;
            const int v = e % VEC, pix = e / VEC;
            const int py = pix / C::PW, px = pix - py * C::PW;
            const int iy = (y0 >> 1) + py, ix = (x0 >> 1) + px;
            val[j] = make_uint4(0, 0, 0, 0);
            if (e < NE && iy < a.Hin && ix < a.Win)
                val[j] = *reinterpret_cast<const uint4*>(xb + (iy * a.Win + ix) * CIN + 8 * v);
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int e = tid + j * 256;
            if (e < NE) *reinterpret_cast<uint4*>(&s_in[(e / VEC) * C::CP + 8 * (e % VEC)]) = val[j];
        }
    };
    auto next_active = [&](int t) {
        while (t < a.ntiles && a.active && !a.active[t / per_b]) t += gridDim.x;
        return t;
    };
    uint4 pf[NPF];
    int tile = next_active(blockIdx.x);
    if (PF && tile < a.ntiles) gather(tile, pf);
    while (tile < a.ntiles) {
        const int b = tile / per_b;
        const int rem = tile - b * per_b;
        const int ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
        const int y0 = ty * C::TR, x0 = tx * C::TC;
        const int nxt = next_active(tile + gridDim.x);
        __syncthreads();  // previous tile's readers are done with s_in
        if (PF) {
#pragma unroll
            for (int j = 0; j < NPF; ++j) {
                const int e = tid + j * 256;
                if (e < NE) {
                    const int v = e % VEC, pix = e / VEC;
                    *reinterpret_cast<uint4*>(&s_in[pix * C::CP + 8 * v]) = pf[j];
                }
            }
        } else {
            stage_now(tile);
        }
        __syncthreads();
        if (PF && nxt < a.ntiles) gather(nxt, pf);
        f32x4 acc[C::PBW];
#pragma unroll
        for (int q = 0; q < C::PBW; ++q) {
            acc[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
            const int ry = (wsub * C::PBW + q) >> 1;  // parity (q >> 1) & 1, since 4 | PBW
            const bool odd_row = (q >> 1) & 1, odd_col = q & 1;
#pragma unroll
            for (int ty_ = 0; ty_ < 2; ++ty_) {
                if (!odd_row && ty_ > 0) break;
                const int ky = odd_row ? 2 * ty_ : 1;
#pragma unroll
                for (int tx_ = 0; tx_ < 2; ++tx_) {
                    if (!odd_col && tx_ > 0) break;
                    const int kx = odd_col ? 2 * tx_ : 1;
                    const int tap = ky * 3 + kx;
                    const int sy = (ry + ky - 1) >> 1;
                    const int sx = lp + ((odd_col ? kx : kx - 1) >> 1);
#pragma unroll
                    for (int cb = 0; cb < C::CB; ++cb) {
                        const uint4 raw =
                            *reinterpret_cast<const uint4*>(&s_in[(sy * C::PW + sx) * C::CP + cb * 32 + 8 * lg]);
                        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&raw);
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wreg[tap * C::CB + cb], bv, acc[q], 0, 0, 0);
                    }
                }
            }
        }
        const int co = ct * 16 + 4 * lg;
        const EpiBases eb = epi_bases<COUT>(a, b);
#pragma unroll
        for (int q = 0; q < C::PBW; ++q) {
            const int ry = (wsub * C::PBW + q) >> 1;
            const int oy = y0 + ry, ox = x0 + (q & 1) + 2 * lp;
            if (oy >= a.Hout || ox >= a.Wout) continue;
            conv_epilogue4(acc[q], bias4, a.act, eb.yb, eb.yfb, eb.kb, eb.mb, (oy * a.Wout + ox) * COUT + co);
        }
        tile = nxt;
    }
}

template <int CIN, int COUT, int TR = 0>
static hh_status launch_t2_t(hipStream_t st, ConvArgs a, int num_cus) {
    using C = T2Cfg<CIN, COUT, TR>;
    a.tiles_x = (a.Wout + C::TC - 1) / C::TC;
    a.tiles_y = (a.Hout + C::TR - 1) / C::TR;
    a.ntiles = a.B * a.tiles_x * a.tiles_y;
    if (a.ntiles == 0) return HH_OK;
    const int grid = std::min(a.ntiles, 8 * num_cus);
    hipLaunchKernelGGL((k_conv_t2<CIN, COUT, TR>), dim3(grid), dim3(256), 0, st, a);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// ---------------------------------------------------------------------------
// Two stride-1 16-channel layers with ReLU, fused (inference):
//   y = relu(conv(W2, relu(conv(W1, x) + b1)) + b2).
// Per TR x 32 output tile the (TR + 4) x 36 input patch is staged in LDS; the
// first layer is evaluated over the tile and a one-pixel ring around it,
// (TR + 2) x 34 pixels, into LDS as BF16 (zero outside the image, which is the
// second layer's zero padding); the second layer reads it from there, so the
// intermediate tensor never goes through HBM.  The first layer's 16-pixel
// blocks run over the flattened ring region (a block may wrap a row end).
// Every output takes the same k chunks in the same order as k_conv_mfma and
// the intermediate is rounded to BF16 as that kernel stores it, so the result
// is bit-identical to the two layers launched separately.
// ---------------------------------------------------------------------------
template <int TR>
struct PairCfg {
    static constexpr int C = 16, TC = 32, CP = C + 8;          // channels, tile columns, LDS pitch (bf16)
    static constexpr int MH = TR + 2, MW = TC + 2;             // ring region (first layer's outputs)
    static constexpr int IH = TR + 4, IW = TC + 4;             // input patch
    static constexpr int P1 = MH * MW, NB1 = (P1 + 15) / 16;   // ring pixels, their 16-pixel blocks
    static constexpr int NB2 = TR * TC / 16;                   // output blocks
    static constexpr int NCH = (9 * C + 31) / 32;              // k chunks per layer
    static constexpr int J1 = (NB1 + 3) / 4;                   // first-layer blocks per wave (at most)
    static constexpr int G1 = 2;                               // of which accumulated together
    static constexpr int J2 = NB2 / 4;                         // output blocks per wave
    static constexpr int G2 = 2;                               // of which accumulated together
    static constexpr int NE = IH * IW * (C / 8);               // 16-byte vectors of the patch
    static constexpr int NPF = (NE + 255) / 256;               // gathers per thread
    static_assert(NB2 % 4 == 0 && J2 % G2 == 0, "output blocks split evenly over the four waves");
};

template <int TR>
__global__ void __launch_bounds__(256, TR >= 16 ? 2 : 4) k_conv_pair16(ConvArgs a) {
    using C = PairCfg<TR>;
    __shared__ __attribute__((aligned(16))) uint16_t s_in[C::IH * C::IW * C::CP];
    __shared__ __attribute__((aligned(16))) uint16_t s_mid[C::P1 * C::CP];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int lp = lane & 15, lg = lane >> 4;

    // both layers' weights stay in VGPRs for all tiles
    bf16x8 w1[C::NCH], w2[C::NCH];
    {
        const uint4* p1 = reinterpret_cast<const uint4*>(a.wp);
        const uint4* p2 = reinterpret_cast<const uint4*>(a.wp2);
#pragma unroll
        for (int ch = 0; ch < C::NCH; ++ch) {
            uint4 v1 = p1[((size_t)ch * 16 + lp) * 4 + lg];
            uint4 v2 = p2[((size_t)ch * 16 + lp) * 4 + lg];
            w1[ch] = *reinterpret_cast<bf16x8*>(&v1);
            w2[ch] = *reinterpret_cast<bf16x8*>(&v2);
        }
    }
    float b1[4], b2[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        b1[i] = a.bias ? a.bias[4 * lg + i] : 0.f;
        b2[i] = a.bias2 ? a.bias2[4 * lg + i] : 0.f;
    }
    wait_all_memory();

    const int per_b = a.tiles_x * a.tiles_y;
    // input vector e of a tile's patch (zero outside the image)
    auto elem = [&](int tile, int e) -> uint4 {
        const int b = tile / per_b;
        const int rem = tile - b * per_b;
        const int ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
        const int v = e & 1, pix = e >> 1;
        const int py = pix / C::IW, px = pix - py * C::IW;
        const int iy = ty * TR - 2 + py, ix = tx * C::TC - 2 + px;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (e < C::NE && iy >= 0 && iy < a.Hin && ix >= 0 && ix < a.Win)
            val = *reinterpret_cast<const uint4*>(a.x + (size_t)b * a.Hin * a.Win * 16 + ((iy * a.Win + ix) * 16 + 8 * v));
        return val;
    };
    auto next_active = [&](int t) {
        while (t < a.ntiles && a.active && !a.active[t / per_b]) t += gridDim.x;
        return t;
    };
    // B operand of chunk ch for a pixel whose 3x3 window starts at (sy, sx) of a
    // region of width W held in buf (tap 9 of the last chunk is zero)
    auto bfrag = [&](const uint16_t* buf, int W, int sy, int sx, int ch) -> bf16x8 {
        const int k0 = ch * 32 + 8 * lg;
        const int tap = k0 >> 4, ci = k0 & 15;
        uint4 raw = make_uint4(0, 0, 0, 0);
        if (tap < 9) {
            const int ky = tap / 3, kx = tap - 3 * ky;
            raw = *reinterpret_cast<const uint4*>(&buf[((sy + ky) * W + sx + kx) * C::CP + ci]);
        }
        return *reinterpret_cast<bf16x8*>(&raw);
    };

    uint4 pf[C::NPF];
    int tile = next_active(blockIdx.x);
    if (tile < a.ntiles) {
#pragma unroll
        for (int j = 0; j < C::NPF; ++j) pf[j] = elem(tile, tid + j * 256);
    }
    while (tile < a.ntiles) {
        const int b = tile / per_b;
        const int rem = tile - b * per_b;
        const int ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
        const int y0 = ty * TR, x0 = tx * C::TC;
        const int nxt = next_active(tile + gridDim.x);
        __syncthreads();  // the previous tile's readers of s_in and s_mid are done
#pragma unroll
        for (int j = 0; j < C::NPF; ++j) {
            const int e = tid + j * 256;
            if (e < C::NE) *reinterpret_cast<uint4*>(&s_in[(e >> 1) * C::CP + 8 * (e & 1)]) = pf[j];
        }
        __syncthreads();
        if (nxt < a.ntiles) {  // the next tile's patch is in flight during both layers
#pragma unroll
            for (int j = 0; j < C::NPF; ++j) pf[j] = elem(nxt, tid + j * 256);
        }
        // ---- first layer over the ring region: blocks wave, wave + 4, ... ----
#pragma unroll 1
        for (int g0 = 0; g0 < C::J1; g0 += C::G1) {
            f32x4 acc[C::G1];
#pragma unroll
            for (int q = 0; q < C::G1; ++q) acc[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ch = 0; ch < C::NCH; ++ch)
#pragma unroll
                for (int q = 0; q < C::G1; ++q) {
                    const int blk = wave + 4 * (g0 + q);
                    if (g0 + q >= C::J1 || blk >= C::NB1) continue;  // uniform per wave
                    const int p = min(blk * 16 + lp, C::P1 - 1);     // lanes past the region: discarded
                    const int my = p / C::MW, mx = p - my * C::MW;
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[ch], bfrag(s_in, C::IW, my, mx, ch), acc[q],
                                                                     0, 0, 0);
                }
#pragma unroll
            for (int q = 0; q < C::G1; ++q) {
                const int blk = wave + 4 * (g0 + q);
                if (g0 + q >= C::J1 || blk >= C::NB1) continue;
                const int p = blk * 16 + lp;
                if (p >= C::P1) continue;
                const int my = p / C::MW, mx = p - my * C::MW;
                const int gy = y0 - 1 + my, gx = x0 - 1 + mx;
                const bool in = gy >= 0 && gy < a.Hin && gx >= 0 && gx < a.Win;
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = in ? fmaxf(acc[q][i] + b1[i], 0.f) : 0.f;
                uint2 o2;
                o2.x = f2bf2(v[0], v[1]);
                o2.y = f2bf2(v[2], v[3]);
                *reinterpret_cast<uint2*>(&s_mid[p * C::CP + 4 * lg]) = o2;
            }
        }
        __syncthreads();  // s_mid complete
        // ---- second layer over the tile: blocks wave * J2 .. + J2 - 1, G2 at a time ----
        uint16_t* yb = a.y + (size_t)b * a.Hout * a.Wout * 16;
#pragma unroll 1
        for (int g0 = 0; g0 < C::J2; g0 += C::G2) {
            f32x4 acc2[C::G2];
#pragma unroll
            for (int q = 0; q < C::G2; ++q) acc2[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ch = 0; ch < C::NCH; ++ch)
#pragma unroll
                for (int q = 0; q < C::G2; ++q) {
                    const int pbk = wave * C::J2 + g0 + q;
                    const int ry = pbk >> 1, rx = (pbk & 1) * 16 + lp;
                    acc2[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2[ch], bfrag(s_mid, C::MW, ry, rx, ch),
                                                                      acc2[q], 0, 0, 0);
                }
#pragma unroll
            for (int q = 0; q < C::G2; ++q) {
                const int pbk = wave * C::J2 + g0 + q;
                const int oy = y0 + (pbk >> 1), ox = x0 + (pbk & 1) * 16 + lp;
                if (oy >= a.Hout || ox >= a.Wout) continue;
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = fmaxf(acc2[q][i] + b2[i], 0.f);
                uint2 o2;
                o2.x = f2bf2(v[0], v[1]);
                o2.y = f2bf2(v[2], v[3]);
                *reinterpret_cast<uint2*>(yb + ((oy * a.Wout + ox) * 16 + 4 * lg)) = o2;
            }
        }
        tile = nxt;
    }
}

template <int TR>
static hh_status launch_pair_t(hipStream_t st, ConvArgs a, int num_cus) {
    using C = PairCfg<TR>;
    a.tiles_x = (a.Wout + C::TC - 1) / C::TC;
    a.tiles_y = (a.Hout + TR - 1) / TR;
    a.ntiles = a.B * a.tiles_x * a.tiles_y;
    if (a.ntiles == 0) return HH_OK;
    const int grid = std::min(a.ntiles, 8 * num_cus);
    hipLaunchKernelGGL((k_conv_pair16<TR>), dim3(grid), dim3(256), 0, st, a);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// ---------------------------------------------------------------------------
// Tile autotuner.  Every stride-1 and stride-2 layer shape has several
// variants: the register-prefetch kernel (k_conv_mfma) and the direct-to-LDS
// kernel (k_conv_dma) at several tile heights; the transposed layers their one
// kernel (k_conv_t2) at several heights.  Variant code: TR for the register and
// transposed kernels, 100 + TR for the direct-to-LDS one.  On the first launch of
// a (shape, output size, batch) key on a device, outside graph capture, every
// variant runs three times on the call's own data (HIP events on the launch
// stream, the faster of the last two counts) and the fastest is kept for the
// process; then the chosen variant runs once more (each run rewrites the same
// output, so the result does not depend on which ran last).  All variants take the same k
// chunks in the same order for every output pixel: their results are
// bit-identical.  Defaults (before tuning, or while a stream captures): the
// direct-to-LDS kernel for the strided layers (measured at the 1024^2
// network's shapes, 42 right-hand sides: 16 -> 32 121 -> 112 us, 32 -> 64
// 74 -> 68, 64 -> 64 48 -> 34), the register kernel for stride 1 (16 -> 16
// 181 against 185-224 us, 32 -> 32 113 against 122-131 us).
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int MODE, int TR>
static hh_status launch_reg(hipStream_t st, ConvArgs a, int num_cus) {
    using C = ConvCfg<CIN, COUT, MODE, TR>;
    a.tiles_x = (a.Wout + C::TC - 1) / C::TC;
    a.tiles_y = (a.Hout + C::TR - 1) / C::TR;
    a.ntiles = a.B * a.tiles_x * a.tiles_y;
    if (a.ntiles == 0) return HH_OK;
    const int grid = std::min(a.ntiles, 8 * num_cus);
    hipLaunchKernelGGL((k_conv_mfma<CIN, COUT, MODE, false, TR>), dim3(grid), dim3(256), 0, st, a);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

template <int CIN, int COUT, int MODE, int TR>
static hh_status launch_dma(hipStream_t st, ConvArgs a, int num_cus) {
    using C = DmaCfg<CIN, COUT, MODE, TR>;
    a.tiles_x = (a.Wout + C::TC - 1) / C::TC;
    a.tiles_y = (a.Hout + C::TR - 1) / C::TR;
    a.ntiles = a.B * a.tiles_x * a.tiles_y;
    if (a.ntiles == 0) return HH_OK;
    const int grid = std::min(a.ntiles, 8 * num_cus);
    hipLaunchKernelGGL((k_conv_dma<CIN, COUT, MODE, TR>), dim3(grid), dim3(256), 0, st, a);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

// the variants of a shape (first: the default)
static int conv_variants(int cin, int cout, int mode, int* codes) {
    static const int v16[] = {16, 8, 4, 108, 116};
    static const int v32[] = {4, 2, 8, 104, 108};
    static const int v64[] = {2, 1, 4, 102, 104};
    static const int s16[] = {104, 102, 108, 4};
    static const int s32[] = {102, 104, 2, 4};
    static const int s64[] = {102, 101, 2};
    static const int t16[] = {8, 16};
    static const int t32[] = {4, 8, 16};
    static const int t64[] = {4, 2, 8};
    static const int p16[] = {8, 16, 4, 1};  // fused at 8, 16 or 4 rows; 1: the two layers launched separately
    const int* v = nullptr;
    int nv = 0;
    if (mode == CM_T2 && cin == 32 && cout == 16) { v = t16; nv = 2; }
    if (mode == CM_T2 && cin == 64 && cout == 32) { v = t32; nv = 3; }
    if (mode == CM_T2 && cin == 64 && cout == 64) { v = t64; nv = 3; }
    if (mode == CM_S1 && cin == 16 && cout == 16) { v = v16; nv = 5; }
    if (mode == CM_S1 && cin == 32 && cout == 32) { v = v32; nv = 5; }
    if (mode == CM_S1 && cin == 64 && cout == 64) { v = v64; nv = 5; }
    if (mode == CM_S2 && cin == 16 && cout == 32) { v = s16; nv = 4; }
    if (mode == CM_S2 && cin == 32 && cout == 64) { v = s32; nv = 4; }
    if (mode == CM_S2 && cin == 64 && cout == 64) { v = s64; nv = 3; }
    if (mode == CM_PAIR && cin == 16 && cout == 16) { v = p16; nv = 4; }
    for (int i = 0; i < nv; ++i) codes[i] = v[i];
    return nv;
}

static hh_status launch_variant(hipStream_t st, int num_cus, int cin, int cout, int mode, int code,
                                const ConvArgs& a) {
#define HH_V(CI, CO, MD, CODE, CALL) \
    if (cin == CI && cout == CO && mode == MD && code == CODE) return CALL(st, a, num_cus);
    HH_V(16, 16, CM_S1, 16, (launch_reg<16, 16, CM_S1, 16>))
    HH_V(16, 16, CM_S1, 8, (launch_reg<16, 16, CM_S1, 8>))
    HH_V(16, 16, CM_S1, 4, (launch_reg<16, 16, CM_S1, 4>))
    HH_V(16, 16, CM_S1, 108, (launch_dma<16, 16, CM_S1, 8>))
    HH_V(16, 16, CM_S1, 116, (launch_dma<16, 16, CM_S1, 16>))
    HH_V(32, 32, CM_S1, 4, (launch_reg<32, 32, CM_S1, 4>))
    HH_V(32, 32, CM_S1, 2, (launch_reg<32, 32, CM_S1, 2>))
    HH_V(32, 32, CM_S1, 8, (launch_reg<32, 32, CM_S1, 8>))
    HH_V(32, 32, CM_S1, 104, (launch_dma<32, 32, CM_S1, 4>))
    HH_V(32, 32, CM_S1, 108, (launch_dma<32, 32, CM_S1, 8>))
    HH_V(64, 64, CM_S1, 2, (launch_reg<64, 64, CM_S1, 2>))
    HH_V(64, 64, CM_S1, 1, (launch_reg<64, 64, CM_S1, 1>))
    HH_V(64, 64, CM_S1, 4, (launch_reg<64, 64, CM_S1, 4>))
    HH_V(64, 64, CM_S1, 102, (launch_dma<64, 64, CM_S1, 2>))
    HH_V(64, 64, CM_S1, 104, (launch_dma<64, 64, CM_S1, 4>))
    HH_V(16, 32, CM_S2, 104, (launch_dma<16, 32, CM_S2, 4>))
    HH_V(16, 32, CM_S2, 102, (launch_dma<16, 32, CM_S2, 2>))
    HH_V(16, 32, CM_S2, 108, (launch_dma<16, 32, CM_S2, 8>))
    HH_V(16, 32, CM_S2, 4, (launch_reg<16, 32, CM_S2, 4>))
    HH_V(32, 64, CM_S2, 102, (launch_dma<32, 64, CM_S2, 2>))
    HH_V(32, 64, CM_S2, 104, (launch_dma<32, 64, CM_S2, 4>))
    HH_V(32, 64, CM_S2, 2, (launch_reg<32, 64, CM_S2, 2>))
    HH_V(32, 64, CM_S2, 4, (launch_reg<32, 64, CM_S2, 4>))
    HH_V(64, 64, CM_S2, 102, (launch_dma<64, 64, CM_S2, 2>))
    HH_V(64, 64, CM_S2, 101, (launch_dma<64, 64, CM_S2, 1>))
    HH_V(64, 64, CM_S2, 2, (launch_reg<64, 64, CM_S2, 2>))
    HH_V(32, 16, CM_T2, 8, (launch_t2_t<32, 16, 8>))
    HH_V(32, 16, CM_T2, 16, (launch_t2_t<32, 16, 16>))
    HH_V(64, 32, CM_T2, 8, (launch_t2_t<64, 32, 8>))
    HH_V(64, 32, CM_T2, 4, (launch_t2_t<64, 32, 4>))
    HH_V(64, 32, CM_T2, 16, (launch_t2_t<64, 32, 16>))
    HH_V(64, 64, CM_T2, 4, (launch_t2_t<64, 64, 4>))
    HH_V(64, 64, CM_T2, 2, (launch_t2_t<64, 64, 2>))
    HH_V(64, 64, CM_T2, 8, (launch_t2_t<64, 64, 8>))
    HH_V(16, 16, CM_PAIR, 16, (launch_pair_t<16>))
    HH_V(16, 16, CM_PAIR, 8, (launch_pair_t<8>))
    HH_V(16, 16, CM_PAIR, 4, (launch_pair_t<4>))
#undef HH_V
    if (cin == 16 && cout == 16 && mode == CM_PAIR && code == 1) {  // unfused: through the intermediate tensor
        ConvArgs a1 = a;
        a1.y = a.ymid;
        HH_TRY(launch_conv(st, num_cus, 16, 16, CM_S1, a1));
        ConvArgs a2 = a;
        a2.x = a.ymid;
        a2.wp = a.wp2;
        a2.bias = a.bias2;
        return launch_conv(st, num_cus, 16, 16, CM_S1, a2);
    }
    set_error("no convolution variant %d for cin=%d cout=%d mode=%d", code, cin, cout, mode);
    return HH_ERR_ARG;
}

namespace {
std::mutex g_tune_mu;
std::map<std::pair<int, uint64_t>, int> g_tune;  // (device, key) -> chosen variant
std::map<uint64_t, int> g_forced;                // (cin, cout, mode) -> forced variant
uint64_t tune_key(int cin, int cout, int mode, const ConvArgs& a) {
    return ((uint64_t)cin << 56) | ((uint64_t)cout << 48) | ((uint64_t)mode << 44) | ((uint64_t)a.Hout << 30) |
           ((uint64_t)a.Wout << 16) | (uint64_t)a.B;
}
uint64_t shape_key(int cin, int cout, int mode) { return ((uint64_t)cin << 16) | ((uint64_t)cout << 4) | mode; }
}  // namespace

// times the variants of a key on the call's data; returns the fastest
static hh_status conv_tune(hipStream_t st, int num_cus, int cin, int cout, int mode, const ConvArgs& a,
                           const int* codes, int nv, int* best) {
    hipEvent_t e0, e1;
    HH_HIP(hipEventCreate(&e0));
    HH_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    *best = codes[0];
    hh_status s = HH_OK;
    for (int v = 0; v < nv && s == HH_OK; ++v) {
        float ms = 0.f, ms_min = 1e30f;  // the faster of two timed runs after a warm-up run
        for (int rep = 0; rep < 3 && s == HH_OK; ++rep) {
            if (hipEventRecord(e0, st) != hipSuccess) s = HH_ERR_HIP;
            if (s == HH_OK) s = launch_variant(st, num_cus, cin, cout, mode, codes[v], a);
            if (s == HH_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                               hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                s = HH_ERR_HIP;
            if (s == HH_OK && rep > 0) ms_min = std::min(ms_min, ms);
        }
        ms = ms_min;
        if (s == HH_OK && ms < best_ms) {
            best_ms = ms;
            *best = codes[v];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != HH_OK && !hh_last_error()[0]) set_error("convolution autotuning failed");
    return s;
}

hh_status launch_conv(hipStream_t st, int num_cus, int cin, int cout, int mode, const ConvArgs& a, int variant) {
    int codes[8];
    const int nv = conv_variants(cin, cout, mode, codes);
    if (nv == 0) {
        set_error("no convolution kernel for cin=%d cout=%d mode=%d", cin, cout, mode);
        return HH_ERR_ARG;
    }
    if (mode == CM_PAIR && (a.act != ACT_RELU || a.skip || a.mask || a.yf || !a.ymid || !a.wp2 ||
                            a.Hin != a.Hout || a.Win != a.Wout)) {
        set_error("fused layer pair: two stride-1 ReLU layers without skip, mask or FP32 copy, with an "
                  "intermediate buffer");
        return HH_ERR_ARG;
    }
    if (variant != 0) return launch_variant(st, num_cus, cin, cout, mode, variant, a);
    int dev = 0;
    HH_HIP(hipGetDevice(&dev));
    const uint64_t key = tune_key(cin, cout, mode, a);
    int chosen = 0;
    {  // looked up under the lock, launched after it (the unfused pair launches its layers through here)
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto f = g_forced.find(shape_key(cin, cout, mode));
        if (f != g_forced.end()) {
            chosen = f->second;
        } else {
            auto it = g_tune.find({dev, key});
            if (it != g_tune.end()) chosen = it->second;
        }
    }
    if (chosen != 0) return launch_variant(st, num_cus, cin, cout, mode, chosen, a);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HH_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone || a.B * a.Hout * a.Wout == 0)
        return launch_variant(st, num_cus, cin, cout, mode, codes[0], a);
    int best = codes[0];
    HH_TRY(conv_tune(st, num_cus, cin, cout, mode, a, codes, nv, &best));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[{dev, key}] = best;
    }
    return launch_variant(st, num_cus, cin, cout, mode, best, a);
}

int conv_tuned_variant(int device, int cin, int cout, int mode, int Hout, int Wout, int B) {
    ConvArgs a{};
    a.Hout = Hout;
    a.Wout = Wout;
    a.B = B;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find({device, tune_key(cin, cout, mode, a)});
    return it == g_tune.end() ? 0 : it->second;
}

hh_status conv_force_variant(int cin, int cout, int mode, int code) {
    int codes[8];
    const int nv = conv_variants(cin, cout, mode, codes);
    bool ok = code == 0;
    for (int i = 0; i < nv; ++i) ok = ok || codes[i] == code;
    if (!ok) {
        set_error("variant %d is not one of the layer shape's", code);
        return HH_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (code == 0)
        g_forced.erase(shape_key(cin, cout, mode));
    else
        g_forced[shape_key(cin, cout, mode)] = code;
    return HH_OK;
}

int conv_variant_list(int cin, int cout, int mode, int* codes, int max) {
    int tmp[8];
    const int nv = conv_variants(cin, cout, mode, tmp);
    for (int i = 0; codes && i < nv && i < max; ++i) codes[i] = tmp[i];
    return nv;
}

hh_status launch_conv_proj(hipStream_t st, int num_cus, const ConvArgs& a0) {
    using C = ConvCfg<16, 16, CM_S1>;
    ConvArgs a = a0;
    a.tiles_x = (a.Wout + C::TC - 1) / C::TC;
    a.tiles_y = (a.Hout + C::TR - 1) / C::TR;
    a.ntiles = a.B * a.tiles_x * a.tiles_y;
    if (a.ntiles == 0) return HH_OK;
    const int grid = std::min(a.ntiles, 8 * num_cus);
    hipLaunchKernelGGL((k_conv_mfma<16, 16, CM_S1, true>), dim3(grid), dim3(256), 0, st, a);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

hh_status pack_weights_split(hipStream_t st, const float* W, uint16_t* Wp_hi, uint16_t* Wp_lo, int cin, int cout_real,
                             int cout) {
    const int nch = (9 * cin + 31) / 32;
    const int total = nch * cout * 32;
    hipLaunchKernelGGL(k_pack_weights_split, dim3((total + 255) / 256), dim3(256), 0, st, W, Wp_hi, Wp_lo, cin,
                       cout_real, cout, nch);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

hh_status pack_weights(hipStream_t st, const float* W, uint16_t* Wp, int cin, int cout, bool flipped) {
    const int nch = (9 * cin + 31) / 32;
    const int total = nch * cout * 32;
    hipLaunchKernelGGL(k_pack_weights, dim3((total + 255) / 256), dim3(256), 0, st, W, Wp, cin, cout,
                       flipped ? 1 : 0, nch);
    HH_LAUNCH_CHECK();
    return HH_OK;
}

size_t packed_weight_elems(int cin, int cout) { return (size_t)((9 * cin + 31) / 32) * cout * 32; }

}  // namespace hh
