// Learned Davidson preconditioner: network state and kernel launchers.
#pragma once
#include <cstdint>
#include "../../include/dmrg.h"

namespace dmrg {

constexpr int MLP_IN = DMRG_MLP_IN;
constexpr double MLP_A_MAX = DMRG_MLP_A_MAX;

// arguments of the fused forward kernel (see kernels_mlp.hip)
struct FwdArgs {
  const float *params;
  int64_t n;
  // mode 0
  const float *x;
  float *g;
  float *z1, *z2;          // optional pre-activations [n][W]
  // mode 1 (Davidson): per-segment theta, sigma, f1 and absolute floor
  const double *d, *r;
  const double *theta, *sigma, *f1, *floor_;
  const int64_t *seg_off;  // [nseg + 1]
  int nseg;
  double *t;
};

bool mlp_width_ok(int W);
void launch_mlp_forward(int W, int mode, const FwdArgs &A, void *stream);
void launch_mlp_backward(int W, const float *params, const float *x, const float *a, const float *b, int64_t n,
                         const float *g, const float *z1, const float *z2, float *dg, float *dz2, float *dz1,
                         double *lpart, float *grad, void *stream);
void launch_adam(float *p, float *m, float *v, const float *gr, int64_t n, float lr, float b1, float b2, float eps,
                 float c1, float c2, void *stream);
void launch_gather(const float *x, const float *a, const float *b, int64_t n, uint64_t seed, uint64_t step, int batch,
                   float *xb, float *ab, float *bb, void *stream);
void launch_exact_corr(const double *psi, const double *u, int64_t n, double c, double *ts, void *stream);
void launch_collect(const double *d, const double *r, const double *ts, int64_t n, double theta, double sigma,
                    double f1, double s, double floor_, float *x, float *a, float *b, void *stream);

}  // namespace dmrg

// device-side network state (opaque in the C ABI)
struct dmrg_mlp {
  int width = 0;
  int64_t nparams = 0;
  float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  int64_t adam_t = 0;
  // training scratch, sized for `cap` rows
  int64_t cap = 0;
  float *xb = nullptr, *ab = nullptr, *bb = nullptr, *g = nullptr, *dg = nullptr;
  float *z1 = nullptr, *z2 = nullptr, *dz2 = nullptr, *dz1 = nullptr;
  double *lpart = nullptr;
  // completion of the last launch sequence of the entry points that return
  // before their work is done (forward, step, adam_step): reading or freeing
  // the parameters waits for it instead of for the whole device
  mutable hipEvent_t done = nullptr;
  mutable bool pending = false;
};
