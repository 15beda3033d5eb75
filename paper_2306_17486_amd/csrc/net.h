// Internal interface of the encoder-solver network (net.hip).
#pragma once
#include "hh_internal.h"
#include "krylov.h"

namespace hh {

// Release the per-model network state (encodings, Green's transforms).
void net_model_release(hh_model* m);

// CNN+MG preconditioner: z = V-cycle(v; x0 = s Net(h^2 v / s)), s = rms(h^2 v).
hh_status net_precond(void* user, hh_model* md, SolveWork& W, const BatchMap& bm, const float2* v, size_t vstride,
                      const double* sig, int sig_stride, float2* z, size_t zstride, const int* act);

}  // namespace hh
