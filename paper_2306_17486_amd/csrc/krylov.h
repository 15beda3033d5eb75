// Internal FGMRES state shared by the solver translation units.
#pragma once
#include "hh_internal.h"

namespace hh {

// Per right-hand-side Arnoldi / least-squares state (device memory, FP64).
struct KState {
    double2 H[HH_MAX_RESTART + 1][HH_MAX_RESTART];  // Hessenberg, rotated in place
    double cs[HH_MAX_RESTART];                      // Givens cosines (real)
    double2 sn[HH_MAX_RESTART];                     // Givens sines
    double2 g[HH_MAX_RESTART + 1];                  // rotated beta e1
    double2 y[HH_MAX_RESTART];                      // current least-squares solution
    double sig[HH_MAX_RESTART + 1];                 // 1/||v_i|| of the stored basis vectors
    float2 oc[HH_MAX_RESTART + 1];                  // single-precision projection coefficients
    double bnorm, res_est, res_true;
    double tol_scale;  // inner-cycle target = rtol * tol_scale (tightened when the FP64 residual refutes it)
    int k, iters, converged, breakdown;
    int ended_by_est;
    int mode;                   // preconditioner of the current cycle (PM_*)
    int probing;                // 1: the current cycle probes the other preconditioner
    int probe_wait, probe_gap;  // cycles before the next probe may run, and the next wait
    int mg_cycles;              // MG-only cycles after the warm start (probes included)
    int cnn_iters;              // iterations preconditioned by CNN+MG
    int cnn_off;                // the network gave a non-finite result: MG-only from then on
    double res_cycle0;          // true relative residual at the start of the current cycle
    double q_base;              // residual reduction of the last cycle of the preconditioner in use
};
// Preconditioner of a restart cycle of a CNN+MG solve (per RHS).
enum { PM_WARM = 0, PM_CNN = 1, PM_MG = 2 };
static_assert(sizeof(KState) % 8 == 0, "KState must be a whole number of doubles");

// Device workspace of one solve (grown on demand, reused across calls).
struct SolveWork {
    int nrhs = 0, restart = 0, hist_len = 0, n = 0, npart = 0;
    Buf V, Z, state, flags, parts, inst, hist, vwork;
    const int* caps_dev = nullptr;  // optional per-RHS iteration caps (training-data generation)
    hh_status prepare(hh_ctx* c, hh_model* md, int nrhs, int restart, int hist_len, bool cnn);
};

// Network part of the CNN+MG preconditioner: z_j = V(v_j; Net(v_j)).
typedef hh_status (*PrecondFn)(void* user, hh_model* md, SolveWork& W, const BatchMap& bm, const float2* v,
                               size_t vstride, const double* sig, int sig_stride, float2* z, size_t zstride,
                               const int* act);

hh_status fgmres_solve(hh_model* md, SolveWork& W, const BatchMap& bm, const float2* b, double2* x,
                       const hh_solve_opts& o, PrecondFn precond_cnn, void* precond_user);
// Several solves (one per model, any sizes) with interleaved restart cycles,
// solve i on streams[i]; fixed_iters must be 0.
hh_status fgmres_solve_many(int nruns, hh_model* const* md, SolveWork* const* W, const BatchMap* bm,
                            const float2* const* b, double2* const* x, const hh_solve_opts& o, PrecondFn precond_cnn,
                            const hipStream_t* streams);
hh_status precond_mg_strided(hh_model* md, SolveWork& W, const BatchMap& bm, const float2* v, size_t vstride,
                             const double* sig, int sig_stride, float2* z, size_t zstride, const int* act);

hh_status residual_norms(hh_model* md, int nrhs, const BatchMap& bm, const float2* b, const double2* x,
                         double* rel_host);

}  // namespace hh
