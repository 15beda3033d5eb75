// C ABI of libhh: contexts, models, solves and the parity-test entry points.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <memory>
#include <new>
#include <vector>

#include "hh_internal.h"
#include "krylov.h"
#include "net.h"

namespace hh {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

hh_status dalloc(hh_ctx* c, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return HH_OK;
    if (c->alloc) {
        *p = c->alloc(bytes, c->user);
        if (!*p) {
            set_error("allocator callback returned NULL for %zu bytes", bytes);
            return HH_ERR_NOMEM;
        }
        return HH_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        return HH_ERR_NOMEM;
    }
    return HH_OK;
}

void dfree(hh_ctx* c, void* p) {
    if (!p) return;
    if (c->dealloc)
        c->dealloc(p, c->user);
    else
        (void)hipFree(p);
}

// Copy a host int[nrhs] RHS -> instance map to the device (NULL = all zeros)
// together with the grouping order of the coarse solve (see BatchMap).
hh_status upload_inst_map(hh_model* m, Buf& buf, int nrhs, const int* inst_host, BatchMap* out) {
    *out = BatchMap();
    if (inst_host)
        for (int r = 0; r < nrhs; ++r)
            HH_ARG(inst_host[r] >= 0 && inst_host[r] < m->ninst, "instance index out of range");
    if (m->ninst == 1) return HH_OK;  // one model: no map needed
    const int G = coarse_group();
    std::vector<int> inst(nrhs, 0);
    if (inst_host)
        for (int r = 0; r < nrhs; ++r) inst[r] = inst_host[r];
    std::vector<int> order;
    for (int k = 0; k < m->ninst; ++k) {
        int cnt = 0;
        for (int r = 0; r < nrhs; ++r)
            if (inst[r] == k) {
                order.push_back(r);
                ++cnt;
            }
        while (cnt % G) {
            order.push_back(-1);
            ++cnt;
        }
    }
    std::vector<int> packed(inst);
    packed.insert(packed.end(), order.begin(), order.end());
    HH_TRY(buf.ensure(m->ctx, packed.size() * sizeof(int)));
    HH_HIP(hipMemcpyAsync(buf.ptr, packed.data(), packed.size() * sizeof(int), hipMemcpyHostToDevice, m->ctx->stream));
    HH_HIP(hipStreamSynchronize(m->ctx->stream));  // the host vectors go out of scope
    out->inst = buf.as<int>();
    out->order = buf.as<int>() + nrhs;
    out->nslots = (int)order.size();
    return HH_OK;
}

}  // namespace hh

using namespace hh;

extern "C" {

const char* hh_version(void) { return "libhh 0.1 (gfx950)"; }

const char* hh_last_error(void) { return g_err; }

hh_status hh_ctx_create(int device, void* stream, hh_alloc_fn alloc, hh_free_fn free_fn, void* user, hh_ctx** out) {
    HH_ARG(out != nullptr, "out is NULL");
    *out = nullptr;
    HH_ARG((alloc == nullptr) == (free_fn == nullptr), "alloc and free must be given together");
    int count = 0;
    HH_HIP(hipGetDeviceCount(&count));
    HH_ARG(device >= 0 && device < count, "device index out of range");
    HH_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    HH_HIP(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_error("libhh is built for gfx950 only; device %d is %s", device, prop.gcnArchName);
        return HH_ERR_ARG;
    }
    hh_ctx* c = new (std::nothrow) hh_ctx();
    if (!c) {
        set_error("out of host memory");
        return HH_ERR_NOMEM;
    }
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->alloc = alloc;
    c->dealloc = free_fn;
    c->user = user;
    c->num_cus = prop.multiProcessorCount;
    hh_status s = noalloc_init(device);
    if (s != HH_OK) {
        delete c;
        return s;
    }
    *out = c;
    return HH_OK;
}

hh_status hh_ctx_destroy(hh_ctx* ctx) {
    if (!ctx) return HH_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    delete ctx->work;
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return HH_OK;
}

void hh_model_desc_default(hh_model_desc* d) {
    if (!d) return;
    memset(d, 0, sizeof(*d));
    d->abl_width = 16;
    d->abl_gamma_max = 1.0;
    d->gamma0 = 0.0;
    d->sl_beta = 0.5;
    d->levels = 3;
    d->nu_pre = 1;
    d->nu_post = 1;
    d->jacobi_w = 0.8;
    d->coarse_reduce = 4;
    d->coarse_iters = 0;
}

hh_status hh_model_create(hh_ctx* ctx, const hh_model_desc* d, int ninst, const float* kappa_dev, hh_model** out) {
    HH_ARG(ctx && d && kappa_dev && out, "null pointer");
    *out = nullptr;
    HH_ARG(ninst >= 1, "ninst >= 1");
    HH_ARG(d->levels >= 2 && d->levels <= HH_MAX_LEVELS, "levels in 2..HH_MAX_LEVELS");
    HH_ARG(d->n >= 16 && d->n % (1 << (d->levels - 1)) == 0, "n >= 16 and divisible by 2^(levels-1)");
    HH_ARG(d->nu_pre == 1 && d->nu_post == 1, "one pre- and one post-relaxation sweep");
    HH_ARG((d->n >> (d->levels - 1)) <= 1024, "coarsest grid at most 1024 x 1024");
    HH_ARG(d->omega >= 0.0 && d->abl_width >= 0 && d->sl_beta > 0.0, "omega >= 0, abl_width >= 0, sl_beta > 0");
    HH_ARG(d->coarse_iters >= 0 && d->coarse_iters <= coarse_gmres_max_iters(), "coarse_iters in 0..16");
    HH_ARG(d->coarse_reduce >= 0 && d->coarse_reduce <= 5, "coarse_reduce in 0..5");
    HH_HIP(hipSetDevice(ctx->device));
    hh_model* m = new (std::nothrow) hh_model();
    if (!m) {
        set_error("out of host memory");
        return HH_ERR_NOMEM;
    }
    m->ctx = ctx;
    m->d = *d;
    m->ninst = ninst;
    m->nlev = d->levels;
    for (int l = 0; l < m->nlev; ++l) {
        m->lev[l].n = d->n >> l;
        m->lev[l].h = (double)(1 << l) / d->n;
        hh_status s = m->lev[l].coef.ensure(ctx, (size_t)ninst * m->lev[l].n * m->lev[l].n * sizeof(float2));
        if (s < 0) {
            delete m;
            return s;
        }
    }
    hh_status s = m->kappa0.ensure(ctx, (size_t)ninst * d->n * d->n * sizeof(float));
    if (s >= 0 && hipMemcpyAsync(m->kappa0.ptr, kappa_dev, (size_t)ninst * d->n * d->n * sizeof(float),
                                 hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess) {
        set_error("hipMemcpyAsync failed");
        s = HH_ERR_HIP;
    }
    if (s >= 0) s = setup_coefficients(m, kappa_dev);
    if (s >= 0) s = setup_coarse_factors(m);
    if (s >= 0) s = m->coarse_err.ensure(ctx, 256);
    if (s >= 0 && hipMemsetAsync(m->coarse_err.ptr, 0, sizeof(int), ctx->stream) != hipSuccess) {
        set_error("hipMemsetAsync failed");
        s = HH_ERR_HIP;
    }
    if (s >= 0 && hipStreamSynchronize(ctx->stream) != hipSuccess) {
        set_error("hipStreamSynchronize failed");
        s = HH_ERR_HIP;
    }
    if (s < 0) {
        delete m;
        return s;
    }
    *out = m;
    return HH_OK;
}

hh_status hh_model_destroy(hh_model* m) {
    if (!m) return HH_OK;
    (void)hipStreamSynchronize(m->ctx->stream);
    net_model_release(m);
    delete m;
    return HH_OK;
}

void hh_solve_opts_default(hh_solve_opts* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->restart = 10;
    o->max_iters = 2000;
    o->rtol = 1e-6;
    o->precond = HH_PRECOND_MG;
    o->warm_mg_iters = 3;
    o->use_x0 = 0;
    o->fixed_iters = 0;
    o->fallback = 1;
    o->probe_ratio = 0.5;
    o->graph = 1;
}

static hh_status check_solve_args(hh_ctx* ctx, hh_model* m, int nrhs, const void* b_dev, void* x_dev,
                                  const hh_solve_opts* o) {
    HH_ARG(ctx && m && b_dev && x_dev && o, "null pointer");
    HH_ARG(m->ctx == ctx, "model belongs to another context");
    HH_ARG(nrhs >= 1, "nrhs >= 1");
    HH_ARG(o->restart >= 1 && o->restart <= HH_MAX_RESTART, "restart in 1..HH_MAX_RESTART");
    HH_ARG(o->max_iters >= 1 && o->rtol >= 0.0, "max_iters >= 1, rtol >= 0");
    HH_ARG(o->precond == HH_PRECOND_MG || o->precond == HH_PRECOND_CNN_MG, "precond");
    HH_ARG(o->fixed_iters >= 0 && o->fixed_iters <= o->restart, "0 <= fixed_iters <= restart");
    HH_ARG(o->probe_ratio >= 0.0 && o->probe_ratio <= 1.0, "0 <= probe_ratio <= 1");
    HH_ARG(o->precond == HH_PRECOND_MG || m->net != nullptr, "CNN_MG needs a network attached to the model");
    return HH_OK;
}

// per-RHS results of a finished solve (stream synchronised here)
static hh_status read_results(hh_ctx* ctx, hipStream_t st, SolveWork& W, int nrhs, int hist_len, bool fixed,
                              double* res_hist_host, int* iters_host, int* converged_host, double* final_res_host,
                              int* mg_cycles_host, int* cnn_iters_host) {
    (void)ctx;
    std::vector<KState> hs(nrhs);
    HH_HIP(hipMemcpyAsync(hs.data(), W.state.ptr, (size_t)nrhs * sizeof(KState), hipMemcpyDeviceToHost, st));
    if (res_hist_host)
        HH_HIP(hipMemcpyAsync(res_hist_host, W.hist.ptr, (size_t)nrhs * hist_len * sizeof(double),
                              hipMemcpyDeviceToHost, st));
    HH_HIP(hipStreamSynchronize(st));
    bool all_conv = true, broke = false;
    for (int r = 0; r < nrhs; ++r) {
        if (iters_host) iters_host[r] = hs[r].iters;
        if (converged_host) converged_host[r] = hs[r].converged;
        if (final_res_host) final_res_host[r] = hs[r].res_true;
        if (mg_cycles_host) mg_cycles_host[r] = hs[r].mg_cycles;
        if (cnn_iters_host) cnn_iters_host[r] = hs[r].cnn_iters;
        all_conv = all_conv && hs[r].converged;
        broke = broke || hs[r].breakdown;
    }
    if (broke) {
        set_error("NaN or Inf met in the solve");
        return HH_ERR_BREAKDOWN;
    }
    if (fixed) return HH_OK;
    return all_conv ? HH_OK : HH_NOT_CONVERGED;
}

hh_status hh_solve(hh_ctx* ctx, hh_model* m, int nrhs, const int* inst_host, const void* b_dev, void* x_dev,
                   const hh_solve_opts* o, double* res_hist_host, int* iters_host, int* converged_host,
                   double* final_res_host, int* mg_cycles_host, int* cnn_iters_host) {
    HH_TRY(check_solve_args(ctx, m, nrhs, b_dev, x_dev, o));
    HH_HIP(hipSetDevice(ctx->device));
    if (!ctx->work) {
        ctx->work = new (std::nothrow) SolveWork();
        if (!ctx->work) {
            set_error("out of host memory");
            return HH_ERR_NOMEM;
        }
    }
    SolveWork& W = *ctx->work;
    const bool cnn = o->precond == HH_PRECOND_CNN_MG;
    const int max_it = o->fixed_iters > 0 ? o->fixed_iters : o->max_iters;
    const int hist_len = max_it + 1;
    HH_TRY(W.prepare(ctx, m, nrhs, o->restart, hist_len, cnn));
    BatchMap bm;
    HH_TRY(upload_inst_map(m, W.inst, nrhs, inst_host, &bm));
    hh_status s = fgmres_solve(m, W, bm, (const float2*)b_dev, (double2*)x_dev, *o,
                               cnn ? net_precond : nullptr, cnn ? (void*)m : nullptr);
    if (s < 0) return s;
    HH_TRY(coarse_check_err(m));
    return read_results(ctx, ctx->stream, W, nrhs, hist_len, o->fixed_iters > 0, res_hist_host, iters_host,
                        converged_host, final_res_host, mg_cycles_host, cnn_iters_host);
}

hh_status hh_solve_batch(hh_ctx* ctx, int nmodels, hh_model* const* models, const int* nrhs,
                         const int* const* inst_host, const void* const* b_dev, void* const* x_dev,
                         const hh_solve_opts* o, int* const* iters_host, int* const* converged_host,
                         double* const* final_res_host, int* const* mg_cycles_host, int* const* cnn_iters_host) {
    HH_ARG(ctx && models && nrhs && b_dev && x_dev && o, "null pointer");
    HH_ARG(nmodels >= 1, "nmodels >= 1");
    HH_ARG(o->fixed_iters == 0, "fixed_iters must be 0 in a batch");
    for (int i = 0; i < nmodels; ++i) {
        HH_TRY(check_solve_args(ctx, models[i], nrhs[i], b_dev[i], x_dev[i], o));
        for (int k = 0; k < i; ++k) HH_ARG(models[k] != models[i], "a model appears twice in the batch");
    }
    HH_HIP(hipSetDevice(ctx->device));
    const bool cnn = o->precond == HH_PRECOND_CNN_MG;
    const int hist_len = o->max_iters + 1;
    std::vector<std::unique_ptr<SolveWork>> work(nmodels);
    std::vector<SolveWork*> wp(nmodels);
    std::vector<BatchMap> bm(nmodels);
    std::vector<hh_model*> mp(models, models + nmodels);
    std::vector<const float2*> bp(nmodels);
    std::vector<double2*> xp(nmodels);
    for (int i = 0; i < nmodels; ++i) {
        work[i].reset(new (std::nothrow) SolveWork());
        if (!work[i]) {
            set_error("out of host memory");
            return HH_ERR_NOMEM;
        }
        wp[i] = work[i].get();
        HH_TRY(wp[i]->prepare(ctx, models[i], nrhs[i], o->restart, hist_len, cnn));
        HH_TRY(upload_inst_map(models[i], wp[i]->inst, nrhs[i], inst_host ? inst_host[i] : nullptr, &bm[i]));
        bp[i] = (const float2*)b_dev[i];
        xp[i] = (double2*)x_dev[i];
    }
    // one stream per model (default priority); inputs are ordered by the
    // context's stream, which is idle here
    HH_HIP(hipStreamSynchronize(ctx->stream));
    struct Streams {
        std::vector<hipStream_t> s;
        ~Streams() {
            for (hipStream_t x : s) {
                (void)hipStreamSynchronize(x);
                (void)hipStreamDestroy(x);
            }
        }
    } streams;
    for (int i = 0; i < nmodels; ++i) {
        hipStream_t x;
        HH_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        streams.s.push_back(x);
    }
    hh_status s = fgmres_solve_many(nmodels, mp.data(), wp.data(), bm.data(), bp.data(), xp.data(), *o,
                                    cnn ? net_precond : nullptr, streams.s.data());
    for (hipStream_t x : streams.s) HH_HIP(hipStreamSynchronize(x));
    if (s < 0) return s;
    hh_status worst = HH_OK;
    for (int i = 0; i < nmodels; ++i) {
        HH_TRY(coarse_check_err(models[i]));
        const hh_status r = read_results(ctx, ctx->stream, *wp[i], nrhs[i], hist_len, false, nullptr,
                                         iters_host ? iters_host[i] : nullptr,
                                         converged_host ? converged_host[i] : nullptr,
                                         final_res_host ? final_res_host[i] : nullptr,
                                         mg_cycles_host ? mg_cycles_host[i] : nullptr,
                                         cnn_iters_host ? cnn_iters_host[i] : nullptr);
        if (r < 0) return r;
        if (r == HH_NOT_CONVERGED) worst = HH_NOT_CONVERGED;
    }
    return worst;
}

hh_status hh_apply_operator(hh_model* m, int level, double shift, int nrhs, const int* inst_host, const void* x_dev,
                            void* y_dev) {
    HH_ARG(m && x_dev && y_dev, "null pointer");
    HH_ARG(level >= 0 && level < m->nlev, "level");
    HH_ARG(nrhs >= 1, "nrhs >= 1");
    HH_HIP(hipSetDevice(m->ctx->device));
    Buf ib;
    BatchMap bm;
    HH_TRY(upload_inst_map(m, ib, nrhs, inst_host, &bm));
    HH_TRY(launch_apply_op(m, level, (float)shift, nrhs, bm.inst, (const float2*)x_dev, (float2*)y_dev, nullptr));
    HH_HIP(hipStreamSynchronize(m->ctx->stream));
    return HH_OK;
}

hh_status hh_apply_vcycle(hh_model* m, int nrhs, const int* inst_host, const void* b_dev, const void* x0_dev,
                          void* x_dev) {
    HH_ARG(m && b_dev && x_dev, "null pointer");
    HH_ARG(nrhs >= 1, "nrhs >= 1");
    HH_HIP(hipSetDevice(m->ctx->device));
    Buf ib, work;
    BatchMap bm;
    HH_TRY(upload_inst_map(m, ib, nrhs, inst_host, &bm));
    HH_TRY(work.ensure(m->ctx, vcycle_workspace_bytes(m, nrhs, x0_dev != nullptr) + 256));
    HH_TRY(launch_vcycle(m, nrhs, bm, (const float2*)b_dev, nullptr, 0, (const float2*)x0_dev, (float2*)x_dev,
                         work.ptr, nullptr));
    HH_HIP(hipStreamSynchronize(m->ctx->stream));
    return coarse_check_err(m);
}

hh_status hh_residual_norms(hh_ctx* ctx, hh_model* m, int nrhs, const int* inst_host, const void* b_dev,
                            const void* x_dev, double* rel_host) {
    HH_ARG(ctx && m && b_dev && x_dev && rel_host, "null pointer");
    HH_ARG(m->ctx == ctx, "model belongs to another context");
    HH_ARG(nrhs >= 1, "nrhs >= 1");
    HH_HIP(hipSetDevice(ctx->device));
    Buf ib;
    BatchMap bm;
    HH_TRY(upload_inst_map(m, ib, nrhs, inst_host, &bm));
    return residual_norms(m, nrhs, bm, (const float2*)b_dev, (const double2*)x_dev, rel_host);
}

hh_status hh_model_set_coarse_group(hh_model* m, int R) {
    HH_ARG(m, "null pointer");
    HH_ARG(R == 0 || coarse_choice_valid(m, R),
           "variant 0 (autotune); R = 1, 2, 4, 8 or 100 RS + R (RS = 8, 16, 32) for the plain factorisation; "
           "1000 + R for the reduced one");
    m->coarse_R_forced = R;
    if (R == 0)
        for (int b = 0; b < HH_COARSE_BUCKETS; ++b) m->coarse_R[b] = 0;
    return HH_OK;
}

int hh_model_coarse_group(const hh_model* m, int nact) {
    if (!m || nact < 1) return -1;
    if (m->coarse_R_forced > 0) return m->coarse_R_forced;
    int b = 0;
    while ((1 << b) < nact && b < HH_COARSE_BUCKETS - 1) ++b;
    return m->coarse_R[b];
}

int hh_vcycle_tuned_height(int device, int kernel, int mode, int n, int nrhs) {
    return vc_tuned_height(device, kernel, mode, n, nrhs);
}

hh_status hh_vcycle_force_height(int kernel, int mode, int height) { return vc_force_height(kernel, mode, height); }

hh_status hh_profile_begin(hh_ctx* ctx, int cls) {
    HH_ARG(ctx, "null pointer");
    HH_ARG(cls >= 0 && cls <= HH_K_NUM_CLASSES, "kernel class");
    HH_HIP(hipStreamSynchronize(ctx->stream));
    for (auto& e : ctx->prof_events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    ctx->prof_events.clear();
    ctx->prof_class = cls;
    return HH_OK;
}

hh_status hh_profile_end(hh_ctx* ctx, double* total_ms, long long* launches) {
    HH_ARG(ctx && total_ms && launches, "null pointer");
    HH_HIP(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < HH_K_NUM_CLASSES; ++k) {
        total_ms[k] = 0.0;
        launches[k] = 0;
    }
    hipError_t err = hipSuccess;
    for (auto& e : ctx->prof_events) {
        float ms = 0.f;
        hipError_t q = hipEventElapsedTime(&ms, e.a, e.b);
        if (q != hipSuccess && err == hipSuccess) err = q;
        total_ms[e.cls] += ms;
        launches[e.cls] += 1;
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    ctx->prof_events.clear();
    ctx->prof_class = -1;
    if (err != hipSuccess) {
        set_error("hipEventElapsedTime failed: %s", hipGetErrorString(err));
        return HH_ERR_HIP;
    }
    return HH_OK;
}

}  // extern "C"
