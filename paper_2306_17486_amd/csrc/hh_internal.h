// Internal declarations shared by the HIP translation units of libhh.
// Not part of the public C ABI (see include/hh.h).
#pragma once

#include <hip/hip_runtime.h>
#include <algorithm>
#include <stdint.h>
#include <stddef.h>

#include <string>
#include <vector>

#include "../../include/hh.h"

// ---------------------------------------------------------------------------
// error plumbing: no exception crosses the ABI; every failing call records a
// thread-local message and returns a negative status.
// ---------------------------------------------------------------------------
namespace hh {

void set_error(const char* fmt, ...);

#define HH_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::hh::set_error("%s failed at %s:%d: %s", #call, __FILE__, __LINE__,     \
                            hipGetErrorString(e_));                                    \
            return HH_ERR_HIP;                                                         \
        }                                                                              \
    } while (0)

#define HH_TRY(call)                       \
    do {                                   \
        hh_status s_ = (call);             \
        if (s_ < 0) return s_;             \
    } while (0)

#define HH_ARG(cond, msg)                                               \
    do {                                                                \
        if (!(cond)) {                                                  \
            ::hh::set_error("invalid argument: %s (%s)", msg, #cond);   \
            return HH_ERR_ARG;                                          \
        }                                                               \
    } while (0)

#define HH_LAUNCH_CHECK()                                                               \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess) {                                                        \
            ::hh::set_error("kernel launch failed at %s:%d: %s", __FILE__, __LINE__,  \
                            hipGetErrorString(e_));                                    \
            return HH_ERR_HIP;                                                         \
        }                                                                              \
    } while (0)

}  // namespace hh

// ---------------------------------------------------------------------------
// opaque handle contents
// ---------------------------------------------------------------------------
namespace hh { struct SolveWork; }

struct hh_ctx {
    hh::SolveWork* work = nullptr;  // solve workspace, reused across calls
    // event timing of kernel classes (hh_profile_begin / hh_profile_end):
    // prof_class = -1 off, HH_K_NUM_CLASSES = every class, else one class
    int prof_class = -1;
    struct ProfRec { int cls; hipEvent_t a, b; };
    std::vector<ProfRec> prof_events;
    int device = 0;
    hipStream_t stream = nullptr;
    hh_alloc_fn alloc = nullptr;
    hh_free_fn dealloc = nullptr;
    void* user = nullptr;
    int num_cus = 256;
    hipStream_t cap_stream = nullptr;  // graph capture (the caller's stream may be the null stream)
    bool concurrent = false;           // several streams of this context run at once (batched solve):
                                       // no cooperative launches, whose workgroups must all be resident
};

namespace hh {

// Device allocation through the caller's allocator (or hipMalloc).
hh_status dalloc(hh_ctx* c, void** p, size_t bytes);
void dfree(hh_ctx* c, void* p);

// A device buffer that frees itself through the context's allocator.
struct Buf {
    hh_ctx* ctx = nullptr;
    void* ptr = nullptr;
    size_t bytes = 0;
    Buf() = default;
    Buf(const Buf&) = delete;
    Buf& operator=(const Buf&) = delete;
    ~Buf() { release(); }
    void release() {
        if (ptr && ctx) dfree(ctx, ptr);
        ptr = nullptr;
        bytes = 0;
    }
    hh_status ensure(hh_ctx* c, size_t want) {
        if (ptr && bytes >= want) return HH_OK;
        release();
        ctx = c;
        if (want == 0) return HH_OK;
        hh_status s = dalloc(c, &ptr, want);
        if (s == HH_OK) bytes = want;
        return s;
    }
    template <class T> T* as() const { return reinterpret_cast<T*>(ptr); }
};

// Right-hand-side -> slowness-model map of one batch on the device.  `order`
// lists RHS indices grouped by model and padded with -1 so that consecutive
// groups of `group` entries never mix models (NULL when there is one model).
struct BatchMap {
    const int* inst = nullptr;
    const int* order = nullptr;
    int nslots = 0;
    int nact = 0;  // upper bound of the right-hand sides active in this call (0 = all)
};

// One multigrid level of a model (all instances share n).
struct Level {
    int n = 0;       // points per dimension
    double h = 0;    // spacing
    Buf coef;        // float2 [ninst][n][n] = {omega^2 kappa^2, gamma}
};

}  // namespace hh

// buckets of the coarse-solve autotuner: active right-hand-side counts
// 1, 2, 3-4, 5-8, ..., with the last bucket open-ended
#define HH_COARSE_BUCKETS 12

struct hh_model {
    hh_ctx* ctx = nullptr;
    hh_model_desc d{};
    int ninst = 0;
    int nlev = 0;
    hh::Level lev[HH_MAX_LEVELS];
    hh::Buf kappa0;        // float [ninst][n][n]: the slowness as given, for the FP64 residual
    hh::Buf coarseQT;      // coarse factors, transposed complex singles: [ninst][m][m][m] Schur inverses of the
                           // two-ended elimination, or (cr1) [ninst][4 ceil(m/2)][m][m] reduced-solve slots
    int m = 0;             // coarsest points per dimension
    hh::Buf kfeat;         // encoder input features (bf16 NHWC, 2 channels) when a net is attached
    hh_net* net = nullptr; // attached network (not owned)
    void* netcache = nullptr;  // per-model network state (encodings, Green's transforms)
    int coarse_R[HH_COARSE_BUCKETS] = {0};  // coarse-solve variant per active-count bucket (0 = not tuned)
    int coarse_R_forced = 0;                // fixed variant (R, or 100 RS + R for the split solve); 0: autotuned
    hh::Buf coarse_err;                     // device int: a split-solve wait timed out
    bool cr1 = false;                       // coarseQT holds the reduced factorisation (one level of cyclic reduction)
    int cr_depth = 0;                       // cr1 chains run 2^depth steps at a time (coarse_reduce - 1)
    bool coarse_mm = true;                  // row-parallel phases of the reduced solve on the matrix cores
    hh::Buf coarseFL;                       // the multi-step chain factors of levels 1..depth (hh::cr_fl_block)
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
namespace hh {

__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a / b
__host__ __device__ __forceinline__ float2 cdiv(float2 a, float2 b) {
    float den = b.x * b.x + b.y * b.y;
    return make_float2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}
// a / b with one hardware reciprocal of |b|^2 (about 1 ulp; the relaxation
// sweeps divide by the shifted diagonal at every point and sweep)
// ---- multi-step chains of the reduced coarse solve ----
// The two chains of each end run over chain indices s = 0 .. nsteps-1 (top:
// p of them, bottom: M-1-p, M = ceil(m/2), p = M/2).  Level l >= 1 keeps the
// indices 2^l (i + 1) - 1, i < nsteps >> l, whose step factors are the products
// A_l(i) = A_{l-1}(2i+1) A_{l-1}(2i) (forward, i >= 1) and B_l(i) = B_{l-1}(2i+1)
// B_{l-1}(2i) (backward), stored per instance as blocks
// [level][dir (0 fwd, 1 bwd)][end][i] with Q_l = (max(p, M-1-p) >> l) + 1 slots per end.
__host__ __device__ __forceinline__ int cr_qlev(int M, int p, int l) {
    return ((p > M - 1 - p ? p : M - 1 - p) >> l) + 1;
}
__host__ __device__ __forceinline__ size_t cr_fl_off(int M, int p, int l) {  // first block of level l
    size_t o = 0;
    for (int k = 1; k < l; ++k) o += 4 * (size_t)cr_qlev(M, p, k);
    return o;
}
__host__ __device__ __forceinline__ size_t cr_fl_block(int M, int p, int l, int dir, int e, int i) {
    return cr_fl_off(M, p, l) + (size_t)(dir * 2 + e) * cr_qlev(M, p, l) + i;
}

__device__ __forceinline__ float2 cdiv_rcp(float2 a, float2 b) {
    const float inv = __builtin_amdgcn_rcpf(b.x * b.x + b.y * b.y);
    return make_float2((a.x * b.x + a.y * b.y) * inv, (a.y * b.x - a.x * b.y) * inv);
}
__host__ __device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
    double den = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}
__host__ __device__ __forceinline__ double zabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// Attenuation gamma(i, j) of eq. 1: gamma0 plus the absorbing layer's
// quadratic ramp, gmax ((w - d) / w)^2 at distance d < w from the nearest edge.
__host__ __device__ __forceinline__ double abl_gamma(int i, int j, int n, int abl_w, double gmax, double gamma0) {
    const int di = i < n - 1 - i ? i : n - 1 - i, dj = j < n - 1 - j ? j : n - 1 - j;
    const int d = di < dj ? di : dj;
    double g = gamma0;
    if (d < abl_w) {
        const double t = (double)(abl_w - d) / abl_w;
        g += gmax * t * t;
    }
    return g;
}

// What the FP64 residual needs to form the operator's zeroth-order term in
// FP64 from the FP32 slowness: omega^2 kappa^2 (1 - i gamma).
struct Coef64 {
    const float* kappa;  // [ninst][n][n]
    double omega2;
    int abl_w;
    double gmax, gamma0;
};

// Zeroth-order term omega^2 kappa^2 (1 - i (gamma + shift)) from the stored
// coefficient pair {omega^2 kappa^2, gamma}.
__device__ __forceinline__ float2 mass_of(float2 c, float shift) {
    return make_float2(c.x, -c.x * (c.y + shift));
}

// FP32 <-> BF16 (round to nearest even; NaN stays NaN): the conversion is
// gfx950's v_cvt_pk_bf16_f32, which the compiler pairs for two values
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
typedef __bf16 hh_bf16x2 __attribute__((ext_vector_type(2)));
// two values packed (a in the low half): one conversion instruction
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
    const hh_bf16x2 v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// Wavefront (64 lanes) sum of a double.
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace hh

// ---------------------------------------------------------------------------
// Per-kernel-class timing: brackets the launches of the selected class with
// HIP events recorded on the context's stream.
// ---------------------------------------------------------------------------
namespace hh {
struct ProfScope {
    hh_ctx* c;
    int cls;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(hh_ctx* ctx, int k) : c(ctx), cls(k) {
        if (c->prof_class != cls && c->prof_class != HH_K_NUM_CLASSES) return;
        if (hipEventCreate(&a) != hipSuccess) return;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            a = nullptr;
            return;
        }
        (void)hipEventRecord(a, c->stream);
    }
    ~ProfScope() {
        if (!b) return;
        (void)hipEventRecord(b, c->stream);
        c->prof_events.push_back({cls, a, b});
    }
};
}  // namespace hh

// ---------------------------------------------------------------------------
// internal launchers (host functions, defined in the .hip files)
// ---------------------------------------------------------------------------
namespace hh {

// setup.hip
hh_status setup_coefficients(hh_model* m, const float* kappa_dev);
hh_status setup_coarse_factors(hh_model* m);

// mg.hip
hh_status launch_apply_op(hh_model* m, int level, float shift, int nrhs, const int* inst_dev,
                          const float2* x, float2* y, const int* active);
// V-cycle on level 0: b (optionally scaled per RHS by sig[r*sig_stride]), optional
// initial guess x0, result z.  work: scratch laid out by vcycle_workspace_bytes.
size_t vcycle_workspace_bytes(const hh_model* m, int nrhs, bool with_x0);
hh_status launch_vcycle(hh_model* m, int nrhs, const BatchMap& bm, const float2* b, const double* sig,
                        int sig_stride, const float2* x0, float2* z, void* work, const int* active);
// Same with explicit element strides between consecutive right-hand sides.
// x0h (with x0s): the initial guess given as the network's half-resolution
// output [nrhs][n/2][n/2] and its per-RHS scale, x0 = x0s P(x0h) (x0 unused).
hh_status launch_vcycle_strided(hh_model* m, int nrhs, const BatchMap& bm, const float2* b, size_t bstride,
                                const double* sig, int sig_stride, const float2* x0, size_t x0stride, float2* z,
                                size_t zstride, void* work, const int* active, const float2* x0h = nullptr,
                                const float* x0s = nullptr);
// RHS per workgroup of the coarsest solve (the grouping unit of BatchMap::order)
int coarse_group();
bool coarse_choice_valid(const hh_model* md, int c);
bool coarse_capturable(const hh_model* md, int nrhs, int nact);
// iterative coarsest-grid solve (coarse_gmres.hip): workspace bytes for nrhs
// right-hand sides (0 with the exact solve), the launcher, the step limit
size_t coarse_gmres_bytes(const hh_model* md, int nrhs);
hh_status launch_coarse_gmres(hh_model* md, int nrhs, const int* inst, const float2* bc, float2* xc,
                              const int* active, void* work);
int coarse_gmres_max_iters();
// a non-blocking stream of the context for graph capture (created on first use)
hh_status capture_stream(hh_ctx* c, hipStream_t* out);
hh_status coarse_check_err(hh_model* md);
// the fixed scratch of hh_residual_norms_noalloc: look up its address on
// `device` (once per device; krylov.hip)
hh_status noalloc_init(int device);
// V-cycle tile autotuner (mg.hip): the height chosen for a key (0: not tuned), forcing one
int vc_tuned_height(int device, int kernel, int mode, int n, int nrhs);
hh_status vc_force_height(int kernel, int mode, int height);
// copy a host RHS -> slowness-model map to the device (api.hip)
hh_status upload_inst_map(hh_model* m, Buf& buf, int nrhs, const int* inst_host, BatchMap* out);

}  // namespace hh
