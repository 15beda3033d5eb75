// Internal interface of the encoder-solver network (net*.hip).
#pragma once
#include <algorithm>

#include "hh_internal.h"
#include "krylov.h"

namespace hh {

enum { CM_S1 = 0, CM_S2 = 1, CM_T2 = 2 };  // stride 1, stride 2, transposed stride 2

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
    int relu;
    int B, Hin, Win, Hout, Wout;
    int tiles_x, tiles_y, ntiles;  // filled by the launcher
    const int* active;     // per batch entry: skipped when 0 (null: all active)
    // projection layer (16 -> 2, FP32 weights as a BF16 high part wp plus a BF16
    // low part wp_lo, output channels 2..15 zero): FP32 (re, im) output [B][H][W]
    const uint16_t* wp_lo;
    float2* yproj;
};
hh_status launch_conv(hipStream_t st, int num_cus, int cin, int cout, int mode, const ConvArgs& a);
// the 16 -> 2 projection (stride 1) on the convolution kernel, weights split into BF16 high + low parts
hh_status launch_conv_proj(hipStream_t st, int num_cus, const ConvArgs& a);
hh_status pack_weights_split(hipStream_t st, const float* W, uint16_t* Wp_hi, uint16_t* Wp_lo, int cin, int cout_real,
                             int cout);
hh_status pack_weights(hipStream_t st, const float* W, uint16_t* Wp, int cin, int cout, bool flipped);
size_t packed_weight_elems(int cin, int cout);

// ---- layer table ----
enum LayerKind { LK_CONV = 0, LK_DOWN = 1, LK_UP = 2, LK_DOWN4 = 3, LK_UP4 = 4 };
constexpr int NET_LAYERS = 31;
struct LayerInfo {
    int kind, cin, cout;
    size_t woff, boff;  // offsets (floats) into the flat parameter vector
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
    hh::LayerInfo L[hh::NET_LAYERS];
    size_t koff = 0;                        // offset of the implicit kernels (nk x 3 x 3 complex)
    size_t nparams = 0;                     // floats
    hh::Buf params;                         // FP32 master parameters
    hh::Buf grads;                          // FP32 gradients
    hh::Buf adam_m, adam_v;                 // Adam moments
    hh::Buf packed;                         // BF16 packed weights (forward + input-gradient forms)
    size_t pk_fwd[hh::NET_LAYERS] = {0}, pk_bwd[hh::NET_LAYERS] = {0};
    size_t pk_proj_hi = 0, pk_proj_lo = 0;  // the projection layer's split weights in `packed`
    bool packed_valid = false;
    long long step = 0;
    unsigned long long version = 1;         // bumped whenever the parameters change
    unsigned long long uid = 0;             // unique per network of the process (caches key on it, not on
                                            // the address, which a later network may reuse)
    void* train_work = nullptr;             // training workspace (net.hip)
    ~hh_net();
};
