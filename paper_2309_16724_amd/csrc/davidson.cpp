// Davidson eigensolver for the lowest eigenpair of H_eff (paper, Sec. II:
// the effective Hamiltonian is diagonalised by Lanczos or Davidson, 85-90% of
// the run time).  Built only on the public H.psi entry points; all vector
// work runs in the FP64 kernels of kernels_vec.hip, the m x m projected
// problem (m <= 64) is solved by a cyclic Jacobi sweep on the host.
//
// Details the paper leaves open (same reading as the oracle): block size 1;
// thick restart to the current and previous Ritz vectors when the subspace
// reaches m_max; two-pass classical Gram-Schmidt; correction
// t = -r / (diag - theta) with |diag - theta| floored; convergence when
// ||H u - theta u||_2 <= tol for the normalised Ritz vector u.
#include <hip/hip_runtime_api.h>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>
#include "common.hpp"
#include "davidson.hpp"

using namespace dmrg;

namespace dmrg {

void jacobi_eigh(int m, const double *A, double *w, double *Z) {
  std::vector<double> a(A, A + (size_t)m * m);
  for (int i = 0; i < m; i++)
    for (int j = 0; j < m; j++) Z[i * m + j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < m; i++)
      for (int j = 0; j < m; j++) {
        tot += a[i * m + j] * a[i * m + j];
        if (i != j) off += a[i * m + j] * a[i * m + j];
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < m; p++)
      for (int q = p + 1; q < m; q++) {
        double apq = a[p * m + q];
        if (apq == 0.0) continue;
        double theta = (a[q * m + q] - a[p * m + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < m; k++) {   // columns p, q
          double akp = a[k * m + p], akq = a[k * m + q];
          a[k * m + p] = c * akp - s * akq;
          a[k * m + q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; k++) {   // rows p, q
          double apk = a[p * m + k], aqk = a[q * m + k];
          a[p * m + k] = c * apk - s * aqk;
          a[q * m + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < m; k++) {
          double zkp = Z[k * m + p], zkq = Z[k * m + q];
          Z[k * m + p] = c * zkp - s * zkq;
          Z[k * m + q] = s * zkp + c * zkq;
        }
      }
  }
  // sort ascending
  std::vector<int> idx(m);
  for (int i = 0; i < m; i++) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a[x * m + x] < a[y * m + y]; });
  std::vector<double> Zs((size_t)m * m);
  for (int j = 0; j < m; j++) {
    w[j] = a[idx[j] * m + idx[j]];
    for (int i = 0; i < m; i++) Zs[i * m + j] = Z[i * m + idx[j]];
  }
  std::memcpy(Z, Zs.data(), sizeof(double) * m * m);
}

}  // namespace dmrg

namespace {

struct DevBuf {
  std::vector<void *> ptrs;
  ~DevBuf() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  double *get(int64_t n) {
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(double) * std::max<int64_t>(n, 1)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return (double *)p;
  }
};

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #x);    \
      return DMRG_EHIP;                                                              \
    }                                                                                \
  } while (0)

}  // namespace

extern "C" int dmrg_davidson(dmrg_plan_t *p, double *psi, double *evals, const dmrg_dav_opts_t *o,
                             dmrg_dav_stats_t *st, void *stream) {
  if (!p || !psi || !evals) { set_error("null argument"); return DMRG_EINVAL; }
  dmrg_dav_opts_t opt = {1e-8, 1000, 24, 0, 1e-8, 0};
  if (o) opt = *o;
  if (opt.m_max < 3 || opt.m_max > 64 || opt.max_iter < 1 || !(opt.tol > 0.0) || !(opt.floor > 0.0)) {
    set_error("bad Davidson options (m_max in [3,64], max_iter >= 1, tol > 0, floor > 0)");
    return DMRG_EINVAL;
  }
  if (opt.precond != 0) { set_error("only the diagonal preconditioner is available"); return DMRG_EINVAL; }
  int64_t off1, len1;
  if (dmrg_psi_layout(p, 1, &off1, &len1) == DMRG_OK) {
    set_error("dmrg_davidson needs a single-problem plan");
    return DMRG_EINVAL;
  }
  dmrg_plan_stats_t ps;
  dmrg_plan_stats(p, &ps);
  const int64_t n = ps.psi_len;
  const int M = opt.m_max;
  hipStream_t s = (hipStream_t)stream;
  auto t_start = std::chrono::steady_clock::now();
  DevBuf buf;
  double *V = buf.get((int64_t)M * n), *W = buf.get((int64_t)M * n);
  double *u = buf.get(n), *hu = buf.get(n), *r = buf.get(n), *t = buf.get(n), *uprev = buf.get(n);
  double *diag = buf.get(n), *tmp = buf.get(2 * n);
  double *part = buf.get(vec_dots_part_len(n, M + 2));
  double *dout = buf.get(2 * M + 4), *dcoef = buf.get(2 * M + 4);
  if (!V || !W || !u || !hu || !r || !t || !uprev || !diag || !tmp || !part || !dout || !dcoef) {
    set_error("hipMalloc failed in Davidson");
    return DMRG_ENOMEM;
  }
  int rc;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double t_hpsi = 0.0;
  int n_hpsi = 0;
  auto apply = [&](const double *x, double *y) -> int {
    HIPCHK(hipEventRecord(e0, s));
    int c = dmrg_apply_H(p, x, y, stream);
    if (c) return c;
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    t_hpsi += ms * 1e-3;
    n_hpsi++;
    return DMRG_OK;
  };
  auto dots_host = [&](const double *Vs, int m, const double *x, double *out) -> int {
    vec_dots(Vs, n, m, x, n, part, dout, stream);
    HIPCHK(hipMemcpyAsync(out, dout, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return DMRG_OK;
  };
  if ((rc = dmrg_diag_H(p, diag, stream))) return rc;
  // starting vector
  HIPCHK(hipMemcpyAsync(V, psi, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  double nn;
  if ((rc = dots_host(V, 1, V, &nn))) return rc;
  if (!(nn > 0.0) || !std::isfinite(nn)) { set_error("starting vector is zero or not finite"); return DMRG_ENONFINITE; }
  vec_scale(V, 1.0 / std::sqrt(nn), n, stream);
  if ((rc = apply(V, W))) return rc;
  std::vector<double> G((size_t)M * M, 0.0), w(M), Z((size_t)M * M), col(M + 2), c(M);
  if ((rc = dots_host(V, 1, W, &G[0]))) return rc;
  int m = 1;
  bool have_prev = false, converged = false;
  double theta = 0.0, rnorm = 0.0;
  int it = 0;
  for (it = 1; it <= opt.max_iter; it++) {
    std::vector<double> Gm((size_t)m * m);
    for (int i = 0; i < m; i++)
      for (int j = 0; j < m; j++) Gm[i * m + j] = 0.5 * (G[i * M + j] + G[j * M + i]);
    jacobi_eigh(m, Gm.data(), w.data(), Z.data());
    theta = w[0];
    for (int i = 0; i < m; i++) c[i] = Z[i * m + 0];
    if (!std::isfinite(theta)) { set_error("non-finite Ritz value"); return DMRG_ENONFINITE; }
    HIPCHK(hipMemcpyAsync(dcoef, c.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
    vec_combo(V, n, m, dcoef, 1.0, 0.0, u, n, stream);
    vec_combo(W, n, m, dcoef, 1.0, 0.0, hu, n, stream);
    vec_resid(hu, u, diag, theta, opt.floor, r, t, n, stream);
    double rr;
    if ((rc = dots_host(r, 1, r, &rr))) return rc;
    rnorm = std::sqrt(rr);
    if (!std::isfinite(rnorm)) { set_error("non-finite residual"); return DMRG_ENONFINITE; }
    if (rnorm <= opt.tol) { converged = true; break; }
    if (m >= M) {
      // thick restart in coefficient space: span{u, u_prev}
      std::vector<double> c1(c.begin(), c.begin() + m), c2(m, 0.0);
      double n1 = 0.0;
      for (double x : c1) n1 += x * x;
      for (double &x : c1) x /= std::sqrt(n1);
      int k = 1;
      if (have_prev) {
        if ((rc = dots_host(V, m, uprev, c2.data()))) return rc;
        for (int pass = 0; pass < 2; pass++) {
          double d = 0.0;
          for (int i = 0; i < m; i++) d += c1[i] * c2[i];
          for (int i = 0; i < m; i++) c2[i] -= d * c1[i];
        }
        double n2 = 0.0;
        for (double x : c2) n2 += x * x;
        if (std::sqrt(n2) > 1e-8) {
          for (double &x : c2) x /= std::sqrt(n2);
          k = 2;
        }
      }
      // new basis vectors and their images, then the projected matrix Cm^T G Cm
      std::vector<double> Cm((size_t)m * k);
      for (int i = 0; i < m; i++) {
        Cm[i * k + 0] = c1[i];
        if (k == 2) Cm[i * k + 1] = c2[i];
      }
      for (int j = 0; j < k; j++) {
        std::vector<double> cj(m);
        for (int i = 0; i < m; i++) cj[i] = Cm[i * k + j];
        HIPCHK(hipMemcpyAsync(dcoef, cj.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
        vec_combo(V, n, m, dcoef, 1.0, 0.0, tmp + (int64_t)j * n, n, stream);
        HIPCHK(hipStreamSynchronize(s));
      }
      for (int j = 0; j < k; j++)
        HIPCHK(hipMemcpyAsync(V + (int64_t)j * n, tmp + (int64_t)j * n, sizeof(double) * n,
                              hipMemcpyDeviceToDevice, s));
      for (int j = 0; j < k; j++) {
        std::vector<double> cj(m);
        for (int i = 0; i < m; i++) cj[i] = Cm[i * k + j];
        HIPCHK(hipMemcpyAsync(dcoef, cj.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
        vec_combo(W, n, m, dcoef, 1.0, 0.0, tmp + (int64_t)j * n, n, stream);
        HIPCHK(hipStreamSynchronize(s));
      }
      for (int j = 0; j < k; j++)
        HIPCHK(hipMemcpyAsync(W + (int64_t)j * n, tmp + (int64_t)j * n, sizeof(double) * n,
                              hipMemcpyDeviceToDevice, s));
      std::vector<double> Gn((size_t)M * M, 0.0);
      for (int a = 0; a < k; a++)
        for (int b = 0; b < k; b++) {
          double x = 0.0;
          for (int i = 0; i < m; i++)
            for (int j = 0; j < m; j++) x += Cm[i * k + a] * Gm[i * m + j] * Cm[j * k + b];
          Gn[a * M + b] = x;
        }
      G.swap(Gn);
      m = k;
    }
    // two-pass classical Gram-Schmidt of t against V[0:m), written into V[m]
    double *vt = V + (int64_t)m * n;
    HIPCHK(hipMemcpyAsync(vt, t, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    for (int pass = 0; pass < 2; pass++) {
      vec_dots(V, n, m, vt, n, part, dout, stream);
      vec_combo(V, n, m, dout, -1.0, 1.0, vt, n, stream);
    }
    double tt;
    if ((rc = dots_host(vt, 1, vt, &tt))) return rc;
    if (!(std::sqrt(tt) >= 1e-12)) {
      HIPCHK(hipMemcpyAsync(vt, r, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      for (int pass = 0; pass < 2; pass++) {
        vec_dots(V, n, m, vt, n, part, dout, stream);
        vec_combo(V, n, m, dout, -1.0, 1.0, vt, n, stream);
      }
      if ((rc = dots_host(vt, 1, vt, &tt))) return rc;
      if (!(tt > 0.0)) { set_error("Davidson subspace collapsed"); return DMRG_ENOCONV; }
    }
    vec_scale(vt, 1.0 / std::sqrt(tt), n, stream);
    if ((rc = apply(vt, W + (int64_t)m * n))) return rc;
    if ((rc = dots_host(V, m + 1, W + (int64_t)m * n, col.data()))) return rc;
    for (int i = 0; i <= m; i++) {
      G[i * M + m] = col[i];
      G[m * M + i] = col[i];
    }
    m++;
    HIPCHK(hipMemcpyAsync(uprev, u, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    have_prev = true;
  }
  // return the Ritz vector (normalised) and value
  HIPCHK(hipMemcpyAsync(psi, u, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  evals[0] = theta;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->iters = converged ? it : opt.max_iter;
    st->n_hpsi = n_hpsi;
    st->converged = converged ? 1 : 0;
    st->residual = rnorm;
    st->energy = theta;
    st->t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    st->t_hpsi_s = t_hpsi;
  }
  if (!converged) { set_error("Davidson did not converge; best Ritz pair returned"); return DMRG_ENOCONV; }
  return DMRG_OK;
}
