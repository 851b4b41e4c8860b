// Host-side launchers of the STML kernels (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "stml_dev.h"

namespace stml {

// Scratch the reductions use: partial slots and the last-block counter.
struct RedBuf {
  double* part;         // capacity: kRedSlots doubles
  unsigned* counter;    // one zero-initialised counter per kernel in flight
};
constexpr size_t kRedSlots = (size_t)16 * 65536;

// Temporal-predictor tables of one subset K_q (device pointers).
struct LinTab {            // per frame k: z_k = wl y_left + wr y_right
  int* left;
  int* right;
  double* wl;
  double* wr;
};
struct ThomasTab {         // factorisation of M + beta D^T D for one K_q
  double* invp;            // 1 / pivot_k
  double* cp;              // c'_k (super-diagonal after elimination)
  int* mask;               // 1 if k in K_q
};

Geom make_geom(int dim, const int* ext, double h);
Model make_model(int dim, double h, int nK, double alpha, double lambda,
                 int reg);

int tile_blocks(const Geom& g);
int tile_threads(int nK);

hipError_t launch_fill(float* p, size_t count, float v, hipStream_t s);
hipError_t launch_check_finite(const float* p, size_t count, Scal* sc,
                               hipStream_t s);
hipError_t launch_restrict(int dim, const float* fine, float* coarse, int n,
                           const Geom& gf, const Geom& gc, hipStream_t s);
hipError_t launch_prolong(int dim, const float* coarse, float* fine,
                          int fields, const Geom& gc, const Geom& gf,
                          hipStream_t s);

hipError_t launch_eval(int dim, const float* T, const float* u, const int* K,
                       const Geom& g, const Model& md, float* grad,
                       float* dW, RedBuf rb, Scal* sc, hipStream_t s);
hipError_t launch_hessvec(int dim, const float* v, const float* dW,
                          const Geom& g, const Model& md, float* hv,
                          RedBuf rb, Scal* sc, hipStream_t s);

// PCG on H delta = -g (device-resident scalars in sc).
hipError_t launch_pcg_init(int dim, const float* grad, const float* dW,
                           const Geom& g, const Model& md, float* x, float* r,
                           float* z, float* p, RedBuf rb, Scal* sc,
                           hipStream_t s);
hipError_t launch_pcg_hv(int dim, const float* p, const float* dW,
                         const Geom& g, const Model& md, float* q, RedBuf rb,
                         Scal* sc, hipStream_t s);
hipError_t launch_pcg_update(int dim, const float* p, const float* q,
                             const float* dW, const Geom& g, const Model& md,
                             float* x, float* r, float* z, int fixed,
                             double rtol, RedBuf rb, Scal* sc, hipStream_t s);
hipError_t launch_pcg_pupdate(const float* z, float* p, size_t count,
                              Scal* sc, hipStream_t s);

// Objective at u + t_i delta for kTrialSteps values of t (t = 0 allowed);
// also g.delta and max |delta|.  Results in sc->Jt, sc->slope, sc->maxd.
hipError_t launch_trial(int dim, const float* T, const float* u,
                        const float* delta, const float* grad, const int* K,
                        const Geom& g, const Model& md, const double* t,
                        RedBuf rb, Scal* sc, hipStream_t s);
// u[K[j]] += t delta_j
hipError_t launch_accept(float* u, const float* delta, const int* K, int nK,
                         int dim, long long N, double t, hipStream_t s);

hipError_t launch_linear_predict(const float* Y, float* Z, float* Yout,
                                 LinTab tab, int n, int dim, long long N,
                                 hipStream_t s);
hipError_t launch_ls_predict(float* Y, float* Z, ThomasTab tab, int n,
                             int dim, long long N, double beta,
                             hipStream_t s);

}  // namespace stml
