// Learned Davidson preconditioner: network state, parameter I/O and the
// minibatch Adam training loop (kernels in kernels_mlp.hip).
#include <hip/hip_runtime_api.h>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>
#include "common.hpp"
#include "mlp.hpp"

using namespace dmrg;

namespace {

#define HIPCHK(x)                                                                 \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #x); \
      return DMRG_EHIP;                                                           \
    }                                                                             \
  } while (0)

int64_t count_params(int W) { return (int64_t)MLP_IN * W + W + (int64_t)W * W + W + W + 1; }

template <class T>
int dev_alloc(T **p, int64_t n) {
  *p = nullptr;
  if (hipMalloc((void **)p, sizeof(T) * (size_t)std::max<int64_t>(n, 1)) != hipSuccess) {
    *p = nullptr;
    set_error("hipMalloc failed for the preconditioner network");
    return DMRG_ENOMEM;
  }
  return DMRG_OK;
}

void release_scratch(dmrg_mlp *m) {
  for (void *q : {(void *)m->xb, (void *)m->ab, (void *)m->bb, (void *)m->g, (void *)m->dg, (void *)m->z1,
                  (void *)m->z2, (void *)m->dz2, (void *)m->dz1, (void *)m->lpart})
    if (q) (void)hipFree(q);
  m->xb = m->ab = m->bb = m->g = m->dg = m->z1 = m->z2 = m->dz2 = m->dz1 = nullptr;
  m->lpart = nullptr;
  m->cap = 0;
}

int ensure_scratch(dmrg_mlp *m, int64_t rows) {
  if (rows <= m->cap) return DMRG_OK;
  release_scratch(m);
  const int64_t W = m->width;
  int rc;
  if ((rc = dev_alloc(&m->xb, rows * MLP_IN)) || (rc = dev_alloc(&m->ab, rows)) || (rc = dev_alloc(&m->bb, rows)) ||
      (rc = dev_alloc(&m->g, rows)) || (rc = dev_alloc(&m->dg, rows)) || (rc = dev_alloc(&m->z1, rows * W)) ||
      (rc = dev_alloc(&m->z2, rows * W)) || (rc = dev_alloc(&m->dz2, rows * W)) || (rc = dev_alloc(&m->dz1, rows * W)) ||
      (rc = dev_alloc(&m->lpart, (rows + 255) / 256))) {
    release_scratch(m);
    return rc;
  }
  m->cap = rows;
  return DMRG_OK;
}

// forward with stored activations, then the backward pass: loss partials in
// m->lpart, gradient in m->grad
int loss_grad_rows(dmrg_mlp *m, const float *x, const float *a, const float *b, int64_t n, void *stream) {
  FwdArgs A{};
  A.params = m->p;
  A.n = n;
  A.x = x;
  A.g = m->g;
  A.z1 = m->z1;
  A.z2 = m->z2;
  launch_mlp_forward(m->width, 0, A, stream);
  launch_mlp_backward(m->width, m->p, x, a, b, n, m->g, m->z1, m->z2, m->dg, m->dz2, m->dz1, m->lpart, m->grad,
                      stream);
  HIPCHK(hipGetLastError());
  return DMRG_OK;
}

int read_loss(dmrg_mlp *m, int64_t n, double *loss, void *stream) {
  const int64_t nb = (n + 255) / 256;
  std::vector<double> h((size_t)nb);
  HIPCHK(hipMemcpyAsync(h.data(), m->lpart, sizeof(double) * nb, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  double s = 0.0;
  for (double v : h) s += v;
  *loss = s / (double)n;
  return DMRG_OK;
}

int adam(dmrg_mlp *m, const float *grad, float lr, float b1, float b2, float eps, void *stream) {
  m->adam_t++;
  const double c1 = 1.0 / (1.0 - std::pow((double)b1, (double)m->adam_t));
  const double c2 = 1.0 / (1.0 - std::pow((double)b2, (double)m->adam_t));
  launch_adam(m->p, m->m, m->v, grad, m->nparams, lr, b1, b2, eps, (float)c1, (float)c2, stream);
  HIPCHK(hipGetLastError());
  return DMRG_OK;
}

}  // namespace

namespace {
int mark_done(const dmrg_mlp *m, void *stream) {
  if (!m->done) HIPCHK(hipEventCreateWithFlags(&m->done, hipEventDisableTiming));
  HIPCHK(hipEventRecord(m->done, (hipStream_t)stream));
  m->pending = true;
  return DMRG_OK;
}
void wait_done(const dmrg_mlp *m) {
  if (m->done && m->pending) (void)hipEventSynchronize(m->done);
  m->pending = false;
}
}  // namespace

extern "C" int dmrg_mlp_create(int32_t width, uint64_t seed, dmrg_mlp_t **out) {
  if (!out) { set_error("null output handle"); return DMRG_EINVAL; }
  *out = nullptr;
  if (!mlp_width_ok(width)) { set_error("network width must be 32, 64, 128 or 256"); return DMRG_EINVAL; }
  dmrg_mlp *m = new dmrg_mlp();
  m->width = width;
  m->nparams = count_params(width);
  int rc;
  if ((rc = dev_alloc(&m->p, m->nparams)) || (rc = dev_alloc(&m->m, m->nparams)) ||
      (rc = dev_alloc(&m->v, m->nparams)) || (rc = dev_alloc(&m->grad, m->nparams))) {
    dmrg_mlp_free(m);
    return rc;
  }
  // He-scaled normal weights, small biases, a small output layer
  std::mt19937_64 gen(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<float> h((size_t)m->nparams);
  size_t k = 0;
  for (int i = 0; i < MLP_IN * width; i++) h[k++] = (float)(nd(gen) * std::sqrt(2.0 / MLP_IN));
  for (int i = 0; i < width; i++) h[k++] = (float)(0.1 * nd(gen));
  for (int64_t i = 0; i < (int64_t)width * width; i++) h[k++] = (float)(nd(gen) * std::sqrt(2.0 / width));
  for (int i = 0; i < width; i++) h[k++] = (float)(0.1 * nd(gen));
  for (int i = 0; i < width; i++) h[k++] = (float)(0.1 * nd(gen) / std::sqrt((double)width));
  h[k++] = 0.0f;
  if ((rc = dmrg_mlp_set_params(m, h.data(), m->nparams))) {
    dmrg_mlp_free(m);
    return rc;
  }
  *out = m;
  return DMRG_OK;
}

extern "C" int64_t dmrg_mlp_num_params(const dmrg_mlp_t *m) { return m ? m->nparams : -1; }

extern "C" int dmrg_mlp_set_params(dmrg_mlp_t *m, const float *host, int64_t n) {
  if (!m || !host || n != m->nparams) { set_error("parameter count mismatch"); return DMRG_EINVAL; }
  for (int64_t i = 0; i < n; i++)
    if (!std::isfinite(host[i])) { set_error("non-finite network parameter"); return DMRG_ENONFINITE; }
  wait_done(m);
  HIPCHK(hipMemcpy(m->p, host, sizeof(float) * n, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(m->m, 0, sizeof(float) * n));
  HIPCHK(hipMemset(m->v, 0, sizeof(float) * n));
  m->adam_t = 0;
  return DMRG_OK;
}

extern "C" int dmrg_mlp_get_params(const dmrg_mlp_t *m, float *host, int64_t n) {
  if (!m || !host || n != m->nparams) { set_error("parameter count mismatch"); return DMRG_EINVAL; }
  wait_done(m);
  HIPCHK(hipMemcpy(host, m->p, sizeof(float) * n, hipMemcpyDeviceToHost));
  return DMRG_OK;
}

extern "C" int dmrg_mlp_forward(dmrg_mlp_t *m, const float *x, int64_t n, float *g, void *stream) {
  if (!m || (n > 0 && (!x || !g)) || n < 0) { set_error("bad forward arguments"); return DMRG_EINVAL; }
  if (n == 0) return DMRG_OK;
  FwdArgs A{};
  A.params = m->p;
  A.n = n;
  A.x = x;
  A.g = g;
  launch_mlp_forward(m->width, 0, A, stream);
  HIPCHK(hipGetLastError());
  return mark_done(m, stream);
}

extern "C" int dmrg_mlp_step(const dmrg_mlp_t *m, const double *diag, const double *r, int32_t nseg,
                             const int64_t *seg_off, const double *theta, const double *sigma, const double *rnorm,
                             double floor, double *t, void *stream) {
  if (!m || !diag || !r || !t || nseg < 1 || !seg_off || !theta || !sigma || !rnorm || !(floor > 0.0)) {
    set_error("bad learned-step arguments");
    return DMRG_EINVAL;
  }
  if (seg_off[0] != 0) { set_error("seg_off[0] must be 0"); return DMRG_EINVAL; }
  for (int k = 0; k < nseg; k++)
    if (seg_off[k + 1] < seg_off[k] || !(sigma[k] > 0.0) || !(rnorm[k] > 0.0)) {
      set_error("segments must be ordered, sigma and rnorm positive");
      return DMRG_EINVAL;
    }
  const int64_t n = seg_off[nseg];
  if (n == 0) return DMRG_OK;
  // per-segment inputs of the fused kernel: theta, sigma, feature f1, absolute floor, offsets
  std::vector<double> h((size_t)4 * nseg);
  for (int k = 0; k < nseg; k++) {
    h[k] = theta[k];
    h[nseg + k] = sigma[k];
    h[2 * nseg + k] = std::log10(rnorm[k]) / 8.0;
    h[3 * nseg + k] = floor * sigma[k];
  }
  void *d = nullptr;
  if (hipMalloc(&d, sizeof(double) * h.size() + sizeof(int64_t) * (nseg + 1)) != hipSuccess) {
    set_error("hipMalloc failed in dmrg_mlp_step");
    return DMRG_ENOMEM;
  }
  double *dh = (double *)d;
  int64_t *doff = (int64_t *)(dh + h.size());
  hipStream_t s = (hipStream_t)stream;
  int rc = DMRG_OK;
  if (hipMemcpyAsync(dh, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(doff, seg_off, sizeof(int64_t) * (nseg + 1), hipMemcpyHostToDevice, s) != hipSuccess) {
    set_error("copy failed in dmrg_mlp_step");
    rc = DMRG_EHIP;
  } else {
    FwdArgs A{};
    A.params = m->p;
    A.n = n;
    A.d = diag;
    A.r = r;
    A.theta = dh;
    A.sigma = dh + nseg;
    A.f1 = dh + 2 * nseg;
    A.floor_ = dh + 3 * nseg;
    A.seg_off = doff;
    A.nseg = nseg;
    A.t = t;
    launch_mlp_forward(m->width, 1, A, stream);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      set_error("learned-step kernel failed");
      rc = DMRG_EHIP;
    }
  }
  (void)hipFree(d);
  return rc;
}

extern "C" int dmrg_mlp_loss_grad(dmrg_mlp_t *m, const float *x, const float *a, const float *b, int64_t n,
                                  double *loss, float *grad, void *stream) {
  if (!m || !x || !a || !b || !loss || !grad || n < 1) { set_error("bad gradient arguments"); return DMRG_EINVAL; }
  int rc;
  if ((rc = ensure_scratch(m, n))) return rc;
  if ((rc = loss_grad_rows(m, x, a, b, n, stream))) return rc;
  HIPCHK(hipMemcpyAsync(grad, m->grad, sizeof(float) * m->nparams, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return read_loss(m, n, loss, stream);
}

extern "C" int dmrg_mlp_adam_step(dmrg_mlp_t *m, const float *grad, float lr, float beta1, float beta2, float eps,
                                  void *stream) {
  if (!m || !grad || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps > 0.0f)) {
    set_error("bad Adam arguments");
    return DMRG_EINVAL;
  }
  int rc = adam(m, grad, lr, beta1, beta2, eps, stream);
  return rc ? rc : mark_done(m, stream);
}

extern "C" int dmrg_mlp_train(dmrg_mlp_t *m, const float *x, const float *a, const float *b, int64_t n,
                              const dmrg_mlp_train_opts_t *o, float *loss_trace, void *stream) {
  if (!m || !x || !a || !b || !o || n < 1 || o->batch < 1 || o->steps < 0 || !(o->lr > 0.0f)) {
    set_error("bad training arguments");
    return DMRG_EINVAL;
  }
  int rc;
  if ((rc = ensure_scratch(m, o->batch))) return rc;
  for (int step = 0; step < o->steps; step++) {
    launch_gather(x, a, b, n, o->seed, (uint64_t)step, o->batch, m->xb, m->ab, m->bb, stream);
    if ((rc = loss_grad_rows(m, m->xb, m->ab, m->bb, o->batch, stream))) return rc;
    if (loss_trace) {
      double l;
      if ((rc = read_loss(m, o->batch, &l, stream))) return rc;
      loss_trace[step] = (float)l;
    }
    if ((rc = adam(m, m->grad, o->lr, o->beta1, o->beta2, o->eps, stream))) return rc;
  }
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  return DMRG_OK;
}

extern "C" void dmrg_mlp_free(dmrg_mlp_t *m) {
  if (!m) return;
  wait_done(m);
  if (m->done) (void)hipEventDestroy(m->done);
  release_scratch(m);
  for (void *q : {(void *)m->p, (void *)m->m, (void *)m->v, (void *)m->grad})
    if (q) (void)hipFree(q);
  delete m;
}
