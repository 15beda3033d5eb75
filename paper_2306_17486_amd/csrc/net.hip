// Encoder-solver network (filled in with the CNN kernels).
#include "net.h"

namespace hh {

void net_model_release(hh_model* m) { (void)m; }

hh_status net_precond(void* user, hh_model* md, SolveWork& W, const BatchMap& bm, const float2* v, size_t vstride,
                      const double* sig, int sig_stride, float2* z, size_t zstride, const int* act) {
    (void)user; (void)md; (void)W; (void)bm; (void)v; (void)vstride; (void)sig; (void)sig_stride; (void)z;
    (void)zstride; (void)act;
    set_error("network preconditioner not available");
    return HH_ERR_STATE;
}

}  // namespace hh
