// Internal interface of the encoder-solver network (net*.hip).
#pragma once
#include <algorithm>

#include "hh_internal.h"
#include "krylov.h"

namespace hh {

// stride 1, stride 2, transposed stride 2; two stride-1 layers with ReLU fused (16 channels, inference)
enum { CM_S1 = 0, CM_S2 = 1, CM_T2 = 2, CM_PAIR = 3 };
enum { ACT_NONE = 0, ACT_RELU = 1, ACT_SOFTPLUS = 2 };

// Waits until every outstanding memory operation of the wave has completed.
// Called after a persistent kernel has loaded its weights and biases into
// registers, before its tile loop: otherwise the compiler's wait insertion,
// merging the loop's entry with its back edge, keeps those loads pending
// inside the loop and waits for them with counts that also cover the next
// tile's prefetch, so the prefetch no longer overlaps the MFMAs.
__device__ __forceinline__ void wait_all_memory() { __builtin_amdgcn_s_waitcnt(0); }

// softplus log(1 + e^v) without overflow, and its derivative (the logistic function)
__device__ __forceinline__ float softplus_f(float v) { return fmaxf(v, 0.f) + __logf(1.f + __expf(-fabsf(v))); }
__device__ __forceinline__ float logistic_f(float v) { return 1.f / (1.f + __expf(-v)); }

// ---- convolution kernels (net_conv.hip) ----
struct ConvArgs {
    const uint16_t* x;     // input [B][Hin][Win][cin] BF16
    uint16_t* y;           // output [B][Hout][Wout][cout] BF16
    float* yf;             // optional FP32 copy of the output (parity tests), may be null
    const uint16_t* wp;    // packed weights
    const float* bias;     // [cout] or null
    const uint16_t* skip;  // added before the activation, [.][Hout][Wout][cout] or null
    const int* skip_map;   // batch index of the skip tensor per output batch entry (null: identity)
    const uint16_t* mask;  // output zeroed where mask <= 0 (ReLU derivative), or null
    int act;               // ACT_NONE, ACT_RELU or ACT_SOFTPLUS, after bias and skip
    int B, Hin, Win, Hout, Wout;
    int tiles_x, tiles_y, ntiles;  // filled by the launcher
    const int* active;     // per batch entry: skipped when 0 (null: all active)
    // projection layer (16 -> 2, FP32 weights as a BF16 high part wp plus a BF16
    // low part wp_lo, output channels 2..15 zero): FP32 (re, im) output [B][H][W]
    const uint16_t* wp_lo;
    float2* yproj;
    // fused pair (CM_PAIR): the second layer's packed weights and bias (wp, bias are
    // the first layer's), and the intermediate tensor that the unfused variant writes
    const uint16_t* wp2;
    const float* bias2;
    uint16_t* ymid;
};
// variant 0: the autotuned choice for this (shape, output size, batch) key (tuned
// on the first launch outside graph capture); otherwise a variant code of the shape
hh_status launch_conv(hipStream_t st, int num_cus, int cin, int cout, int mode, const ConvArgs& a, int variant = 0);
int conv_tuned_variant(int device, int cin, int cout, int mode, int Hout, int Wout, int B);  // 0: not tuned
hh_status conv_force_variant(int cin, int cout, int mode, int code);                         // 0: autotune
int conv_variant_list(int cin, int cout, int mode, int* codes, int max);
// the 16 -> 2 projection (stride 1) on the convolution kernel, weights split into BF16 high + low parts
hh_status launch_conv_proj(hipStream_t st, int num_cus, const ConvArgs& a);
hh_status pack_weights_split(hipStream_t st, const float* W, uint16_t* Wp_hi, uint16_t* Wp_lo, int cin, int cout_real,
                             int cout);
hh_status pack_weights(hipStream_t st, const float* W, uint16_t* Wp, int cin, int cout, bool flipped);
size_t packed_weight_elems(int cin, int cout);

// ---- lightweight network kernels (net_light.hip) ----
struct PwArgs {            // pointwise (1x1) convolution, BF16 NHWC
    const uint16_t* x;     // input [npix][cin]
    uint16_t* y;           // output [npix][cout]
    float* yf;             // optional FP32 copy of the output, may be null
    const uint16_t* w;     // BF16 weights [cout][cin] (pack_pointwise)
    const float* bias;     // [cout] or null
    const uint16_t* res;   // added after the activation, [npix][cout], or null
    int act;               // ACT_NONE or ACT_SOFTPLUS
    size_t npix;
    int pix_per_b;         // pixels per batch entry (for `active`)
    const int* active;     // per batch entry: skipped when 0 (null: all active)
};
struct DwArgs {            // depthwise 3x3 convolution (stride 1, zero padding), BF16 NHWC
    const uint16_t* x;     // input [B][H][W][C]
    uint16_t* y;           // output, same shape
    float* yf;             // optional FP32 copy, may be null
    const float* w;        // FP32 weights [C][3][3]
    const float* bias;     // [C] or null
    int act;               // ACT_NONE or ACT_SOFTPLUS
    int flip;              // 1: taps reversed (the input gradient)
    int B, H, W;
    const int* active;
};
struct BnParams {          // batch normalisation of one layer (running statistics updated in place)
    const float* g;
    const float* be;
    float* rm;
    float* rv;
};
struct BnGrads {
    float* g;
    float* be;
    float* rm;             // written with zeros (running statistics are not trained)
    float* rv;
};
hh_status launch_pointwise(hipStream_t st, int num_cus, int cin, int cout, const PwArgs& a);
hh_status pack_pointwise(hipStream_t st, const float* W, uint16_t* out, int cout, int cin, bool transpose);
hh_status launch_depthwise(hipStream_t st, int num_cus, int C, const DwArgs& a);
hh_status bn_fold(hipStream_t st, const float* W, const float* g, const float* be, const float* rm, const float* rv,
                  int cout, int per, float* Wf, float* bf);
// training form: stat[c] = (mean, sd, g/sd, be - mean g/sd) over the npix pixels of z;
// y = act(stat.z z + stat.w) (+ res); running statistics updated when `update`
hh_status bn_train_forward(hipStream_t st, hh_ctx* ctx, Buf& part, int C, const uint16_t* z, size_t npix,
                           const BnParams& p, bool update, float4* stat, int act, const uint16_t* res, uint16_t* y);
// its backward: gz from the gradient gout of y (act's derivative included); grads of g and be
hh_status bn_train_backward(hipStream_t st, hh_ctx* ctx, Buf& part, Buf& coef, int C, const uint16_t* gout,
                            const uint16_t* z, size_t npix, const float* g, const float4* stat, int act,
                            const BnGrads& gr, uint16_t* gz);
// the inverted bottleneck in one kernel (inference, batch norm folded):
// y = x + Ws (softplus(dw(softplus(We x + be)) + bw)) + bs on x [B][m][m][c]
struct IbArgs {
    const uint16_t* x;     // input [B][m][m][c] BF16 (also the residual)
    uint16_t* y;           // output, same shape
    const uint16_t* we;    // expansion weights BF16 [6c][c]
    const float* be;       // its bias [6c]
    const float* wd;       // depthwise weights FP32 [6c][3][3]
    const float* bd;       // its bias [6c]
    const uint16_t* ws;    // shrink weights BF16 [c][6c]
    const float* bs;       // its bias [c]
    int B, m;
    const int* active;     // per batch entry: skipped when 0 (null: all active)
    int tiles_x, tiles_y, ntiles;  // filled by the launcher
};
hh_status launch_ib_fused(hipStream_t st, int num_cus, int c, IbArgs a);
hh_status launch_pw_wgrad(hipStream_t st, hh_ctx* ctx, Buf& part, int cin, int cout, const uint16_t* g,
                          const uint16_t* x, size_t npix, float* out);
hh_status launch_dw_wgrad(hipStream_t st, hh_ctx* ctx, Buf& part, int C, const uint16_t* g, const uint16_t* x,
                          int B, int H, int W, float* out);

// ---- layer table ----
// LK_PW: pointwise 1x1, LK_DW: depthwise 3x3 (lightweight network)
enum LayerKind { LK_CONV = 0, LK_DOWN = 1, LK_UP = 2, LK_DOWN4 = 3, LK_UP4 = 4, LK_PW = 5, LK_DW = 6 };
constexpr int NET_LAYERS = 31;    // the U-Net
constexpr int LIGHT_LAYERS = 34;  // the lightweight network
constexpr int NET_MAX_LAYERS = 34;
struct LayerInfo {
    int kind, cin, cout;
    size_t woff, boff;  // offsets (floats) into the flat parameter vector (boff: bias, or -1 with batch norm)
    int bn = 0;         // followed by batch normalisation (lightweight network)
    size_t goff = 0, beoff = 0, rmoff = 0, rvoff = 0;  // its scale, shift, running mean and variance
};
// the CNN preconditioner of the solve
hh_status net_precond(void* user, hh_model* md, SolveWork& W, const BatchMap& bm, const float2* v, size_t vstride,
                      const double* sig, int sig_stride, float2* z, size_t zstride, const int* act);
void net_model_release(hh_model* m);

}  // namespace hh

struct hh_net {
    hh_ctx* ctx = nullptr;
    int ch[4] = {16, 32, 64, 64};
    int nk = 32;                            // complex channels of the implicit layer (= ch[3] / 2)
    int explicit_coarse = 0;                // 1: the coarsest layer multiplies by K instead of inverting it
    int light = 0;                          // 1: the lightweight network (inverted bottlenecks, batch norm, softplus)
    int nlayers = hh::NET_LAYERS;
    hh::LayerInfo L[hh::NET_MAX_LAYERS];
    size_t koff = 0;                        // offset of the implicit kernels (nk x 3 x 3 complex)
    size_t nparams = 0;                     // floats
    hh::Buf params;                         // FP32 master parameters
    hh::Buf grads;                          // FP32 gradients
    hh::Buf adam_m, adam_v;                 // Adam moments
    hh::Buf packed;                         // BF16 packed weights (forward + input-gradient forms)
    size_t pk_fwd[hh::NET_MAX_LAYERS] = {0}, pk_bwd[hh::NET_MAX_LAYERS] = {0};
    size_t pk_inf[hh::NET_MAX_LAYERS] = {0};  // lightweight network: batch norm folded (inference)
    hh::Buf folded;                         // lightweight network: parameters with batch norm folded
    size_t pk_proj_hi = 0, pk_proj_lo = 0;  // the projection layer's split weights in `packed`
    bool packed_valid = false;
    long long step = 0;
    unsigned long long version = 1;         // bumped whenever the parameters change
    unsigned long long uid = 0;             // unique per network of the process (caches key on it, not on
                                            // the address, which a later network may reuse)
    void* train_work = nullptr;             // training workspace (net.hip)
    ~hh_net();
};
