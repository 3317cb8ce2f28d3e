// Davidson eigensolver for the lowest eigenpair of H_eff (paper, Sec. II:
// the effective Hamiltonian is diagonalised by Lanczos or Davidson, 85-90% of
// the run time), for every problem of a plan at once.  Built on the public
// H.psi entry points; all vector work runs in the FP64 kernels of
// kernels_vec.hip (segmented per problem), the small projected problems
// (m <= 64) are solved by cyclic Jacobi sweeps on the host.
//
// Details the paper leaves open (same reading as the oracle): block size 1;
// thick restart to the current and previous Ritz vectors when the subspace
// reaches m_max; two-pass classical Gram-Schmidt; correction
// t = -r / (diag - theta) with |diag - theta| floored at floor * sigma, sigma
// the root mean square of diag - theta over the problem (a relative floor:
// the cap on the few elements with diag ~ theta follows the spread of the
// diagonal, so one default serves problems of any size), optionally corrected
// per element by the learned network (mlp.cpp), with a guard that falls back
// to the diagonal step and a patience rule that turns the learned steps of a
// problem off once its residual stops reaching new minima (a network can be
// finite and well aligned yet stall the solve); convergence when
// ||H u - theta u||_2 <= tol for the
// normalised Ritz vector u.  Problems of a batch share the basis-column
// index: a converged problem stops adding vectors (its segments of later
// columns are zero), restarts are global.
#include <hip/hip_runtime_api.h>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>
#include "common.hpp"
#include "davidson.hpp"
#include "mlp.hpp"

using namespace dmrg;

namespace dmrg {

int jacobi_eigh(int m, const double *A, double *w, double *Z) {
  std::vector<double> a(A, A + (size_t)m * m);
  for (int i = 0; i < m; i++)
    for (int j = 0; j < m; j++) Z[i * m + j] = i == j ? 1.0 : 0.0;
  int sweep = 0;
  for (; sweep < JACOBI_MAX_SWEEPS; sweep++) {
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
        // after a few sweeps an element below the rounding of both diagonal
        // entries is set to zero (else rounding keeps the off-diagonal mass
        // above any relative threshold and every solve runs all sweeps)
        const double g = 100.0 * std::fabs(apq);
        if (sweep > 3 && std::fabs(a[p * m + p]) + g == std::fabs(a[p * m + p]) &&
            std::fabs(a[q * m + q]) + g == std::fabs(a[q * m + q])) {
          a[p * m + q] = a[q * m + p] = 0.0;
          continue;
        }
        double theta = (a[q * m + q] - a[p * m + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < m; k++) {
          double akp = a[k * m + p], akq = a[k * m + q];
          a[k * m + p] = c * akp - s * akq;
          a[k * m + q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; k++) {
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
  std::vector<int> idx(m);
  for (int i = 0; i < m; i++) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a[x * m + x] < a[y * m + y]; });
  std::vector<double> Zs((size_t)m * m);
  for (int j = 0; j < m; j++) {
    w[j] = a[idx[j] * m + idx[j]];
    for (int i = 0; i < m; i++) Zs[i * m + j] = Z[i * m + idx[j]];
  }
  std::memcpy(Z, Zs.data(), sizeof(double) * m * m);
  return sweep;
}

}  // namespace dmrg

namespace {

// device buffers of one solve, from the plan's allocator, returned at the end
struct DevBuf {
  dmrg_plan_t *plan;
  std::vector<void *> ptrs;
  explicit DevBuf(dmrg_plan_t *p) : plan(p) {}
  ~DevBuf() {
    for (void *p : ptrs) plan_dfree(plan, p);
  }
  void *raw(int64_t bytes) {
    void *p = plan_dalloc(plan, (size_t)std::max<int64_t>(bytes, 8));
    if (!p) return nullptr;
    ptrs.push_back(p);
    return p;
  }
  double *get(int64_t n) { return (double *)raw(sizeof(double) * n); }
};

// Page-locked host staging for the solver's small transfers (dot products
// down, coefficients and per-problem scalars up): copies from pageable
// memory are staged by the runtime and cost about 0.1 ms each.  Uploads are
// copied into the arena first, so the caller's vectors may change at once;
// the fill pointer returns to zero only after the stream has been
// synchronised (no copy from the arena is pending then).
struct HostStage {
  double *p = nullptr;
  size_t cap = 0, used = 0;
  hipStream_t s = nullptr;
  ~HostStage() {
    if (!p) return;
    (void)hipStreamSynchronize(s);   // an early return may leave a copy pending
    (void)hipHostFree(p);
  }
  bool init(size_t n, hipStream_t stream) {
    cap = n;
    s = stream;
    return hipHostMalloc((void **)&p, sizeof(double) * n, hipHostMallocDefault) == hipSuccess;
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

struct ProbState {
  int64_t off = 0, len = 0;
  std::vector<int> cols;          // global basis columns that belong to this problem
  std::vector<double> G;          // projected matrix over `cols` (row-major, size cols^2)
  std::vector<double> c;          // Ritz coefficients over `cols`
  double theta = 0.0, rnorm = 0.0;
  bool active = true, have_prev = false;
  int iters = 0;
  // learned steps stay on while the residual keeps reaching new minima
  double best_r = INFINITY;
  int best_it = 0;
  bool mlp_on = true;
  double sum_d = 0.0, sum_d2 = 0.0;   // sums of diag and diag^2 over the segment
};

// training-row capture of dmrg_mlp_collect (single-problem plans)
struct Collect {
  const double *psi_star = nullptr;   // converged vector, device
  double *ts = nullptr;               // device scratch, psi_len
  float *x = nullptr, *a = nullptr, *b = nullptr;
  int64_t cap = 0, rows = 0;
  int32_t nrec = 0;
};

}  // namespace

static int check_opts(const dmrg_dav_opts_t *o, dmrg_dav_opts_t *opt) {
  *opt = {1e-8, 1000, 24, DMRG_PRECOND_DIAG, 0, 1e-2, nullptr, 0, 0};
  if (o) *opt = *o;
  if (opt->m_max < 3 || opt->m_max > 64 || opt->max_iter < 1 || !(opt->tol > 0.0) || !(opt->floor > 0.0) ||
      opt->mlp_patience < 0) {
    set_error("bad Davidson options (m_max in [3,64], max_iter >= 1, tol > 0, floor > 0, mlp_patience >= 0)");
    return DMRG_EINVAL;
  }
  if (opt->mlp_patience == 0) opt->mlp_patience = 30;
  if (opt->precond != DMRG_PRECOND_DIAG && opt->precond != DMRG_PRECOND_MLP) {
    set_error("unknown preconditioner");
    return DMRG_EINVAL;
  }
  if (opt->precond == DMRG_PRECOND_MLP && !opt->mlp) {
    set_error("learned preconditioner requested without a network");
    return DMRG_EINVAL;
  }
  return DMRG_OK;
}

static int solve(dmrg_plan_t *p, double *psi, double *evals, const dmrg_dav_opts_t &opt, dmrg_dav_stats_t *st,
                 void *stream, Collect *col) {
  std::vector<ProbState> P;
  for (int k = 0;; k++) {
    int64_t off, len;
    if (dmrg_psi_layout(p, k, &off, &len) != DMRG_OK) break;
    ProbState s;
    s.off = off;
    s.len = len;
    P.push_back(s);
  }
  set_error("");
  const int np = (int)P.size();
  if (np == 0) { set_error("empty plan"); return DMRG_EINVAL; }
  dmrg_plan_stats_t ps;
  dmrg_plan_stats(p, &ps);
  const int64_t n = ps.psi_len;
  const int M = opt.m_max;
  hipStream_t s = (hipStream_t)stream;
  auto t_start = std::chrono::steady_clock::now();
  // chunk table
  std::vector<VChunk> chunks;
  std::vector<int32_t> seg0;
  for (int k = 0; k < np; k++) {
    seg0.push_back((int32_t)chunks.size());
    for (int64_t i0 = P[k].off; i0 < P[k].off + P[k].len; i0 += VCHUNK)
      chunks.push_back({i0, std::min(P[k].off + P[k].len, i0 + VCHUNK), k, 0});
  }
  seg0.push_back((int32_t)chunks.size());
  DevBuf buf(p);
  VChunk *d_chunks = (VChunk *)buf.raw(sizeof(VChunk) * chunks.size());
  int32_t *d_seg0 = (int32_t *)buf.raw(sizeof(int32_t) * seg0.size());
  double *V = buf.get((int64_t)M * n), *W = buf.get((int64_t)M * n);
  double *u = buf.get(n), *hu = buf.get(n), *r = buf.get(n), *t = buf.get(n), *uprev = buf.get(n);
  double *diag = buf.get(n), *tmp = buf.get(2 * n);
  const bool use_mlp = opt.precond == DMRG_PRECOND_MLP;
  double *tm = use_mlp ? buf.get(n) : nullptr, *ones = buf.get(n);
  double *dth = buf.get(np), *dsig = buf.get(np), *df1 = buf.get(np), *dflag = buf.get(np);
  double *dfloor = buf.get(np);
  int64_t *dsegoff = (int64_t *)buf.raw(sizeof(int64_t) * (np + 1));
  double *part = buf.get((int64_t)std::max<size_t>(chunks.size(), 1) * (M + 2));
  double *dout = buf.get((int64_t)np * (M + 2)), *dcoef = buf.get((int64_t)np * M);
  double *dvec = buf.get(np);
  if (!d_chunks || !d_seg0 || !V || !W || !u || !hu || !r || !t || !uprev || !diag || !tmp || !part || !dout ||
      !dcoef || !dvec || (use_mlp && !tm) || !ones || !dth || !dsig || !df1 || !dflag || !dsegoff || !dfloor) {
    set_error("hipMalloc failed in Davidson");
    return DMRG_ENOMEM;
  }
  HIPCHK(hipMemcpy(d_chunks, chunks.data(), sizeof(VChunk) * chunks.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d_seg0, seg0.data(), sizeof(int32_t) * seg0.size(), hipMemcpyHostToDevice));
  VecCtx X{d_chunks, (int)chunks.size(), d_seg0, np, part};
  int rc;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double t_hpsi = 0.0;
  int n_hpsi = 0;
  HostStage hs, up;
  if (!hs.init((size_t)np * (M + 2), s) || !up.init((size_t)np * (4 * M + 16), s)) {
    set_error("hipHostMalloc failed in Davidson");
    return DMRG_ENOMEM;
  }
  auto apply = [&](const double *x, double *y) -> int {
    HIPCHK(hipEventRecord(e0, s));
    int c = dmrg_apply_H(p, x, y, stream);
    if (c) return c;
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    up.used = 0;   // every earlier copy on the stream has completed
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    t_hpsi += ms * 1e-3;
    n_hpsi++;
    return DMRG_OK;
  };
  // per-problem dot products of m columns of Vs with x: host out[k * m + j]
  double *const hout = hs.p;
  // upload of cnt doubles through the page-locked arena
  auto put = [&](double *dst, const double *src, size_t cnt) -> int {
    if (up.used + cnt > up.cap) {
      HIPCHK(hipStreamSynchronize(s));
      up.used = 0;
    }
    double *h = up.p + up.used;
    std::memcpy(h, src, sizeof(double) * cnt);
    up.used += cnt;
    HIPCHK(hipMemcpyAsync(dst, h, sizeof(double) * cnt, hipMemcpyHostToDevice, s));
    return DMRG_OK;
  };
  auto dots_host = [&](const double *Vs, int m, const double *x) -> int {
    vec_dots(X, Vs, n, m, x, dout, stream);
    HIPCHK(hipMemcpyAsync(hout, dout, sizeof(double) * np * m, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    up.used = 0;
    return DMRG_OK;
  };
  auto put_vec = [&](const std::vector<double> &v) -> int { return put(dvec, v.data(), (size_t)np); };
  auto put_coef = [&](const std::vector<double> &cf) -> int {   // np x M row-major
    return put(dcoef, cf.data(), (size_t)np * M);
  };
  if ((rc = dmrg_diag_H(p, diag, stream))) return rc;
  {
    std::vector<int64_t> so(np + 1);
    for (int k = 0; k < np; k++) so[k] = P[k].off;
    so[np] = n;
    HIPCHK(hipMemcpy(dsegoff, so.data(), sizeof(int64_t) * (np + 1), hipMemcpyHostToDevice));
  }
  vec_fill(X, 1.0, ones, stream);
  if ((rc = dots_host(diag, 1, ones))) return rc;
  for (int k = 0; k < np; k++) P[k].sum_d = hout[k];
  if ((rc = dots_host(diag, 1, diag))) return rc;
  for (int k = 0; k < np; k++) P[k].sum_d2 = hout[k];
  // root mean square of diag - theta over problem k's segment
  auto sigma_of = [&](int k, double th) {
    const ProbState &S = P[k];
    double v = (S.sum_d2 - 2.0 * th * S.sum_d + (double)S.len * th * th) / (double)std::max<int64_t>(S.len, 1);
    return std::sqrt(std::max(v, 1e-300));
  };
  int fallbacks = 0;
  HIPCHK(hipMemcpyAsync(V, psi, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  if ((rc = dots_host(V, 1, V))) return rc;
  std::vector<double> sc(np);
  for (int k = 0; k < np; k++) {
    double nn = hout[k];
    if (!(nn > 0.0) || !std::isfinite(nn)) { set_error("starting vector is zero or not finite"); return DMRG_ENONFINITE; }
    sc[k] = 1.0 / std::sqrt(nn);
  }
  if ((rc = put_vec(sc))) return rc;
  vec_scale(X, dvec, V, stream);
  if ((rc = apply(V, W))) return rc;
  if ((rc = dots_host(V, 1, W))) return rc;
  for (int k = 0; k < np; k++) {
    P[k].cols = {0};
    P[k].G = {hout[k]};
  }
  int m = 1;
  int it = 0;
  int n_active = np;
  std::vector<double> coef((size_t)np * M, 0.0), thetas(np, 0.0), floors(np, 1.0);
  for (it = 1; it <= opt.max_iter && n_active > 0; it++) {
    // Ritz pairs
    std::fill(coef.begin(), coef.end(), 0.0);
    for (int k = 0; k < np; k++) {
      ProbState &S = P[k];
      if (!S.active) continue;
      int mk = (int)S.cols.size();
      std::vector<double> Gm((size_t)mk * mk), w(mk), Z((size_t)mk * mk);
      for (int i = 0; i < mk; i++)
        for (int j = 0; j < mk; j++) Gm[i * mk + j] = 0.5 * (S.G[i * mk + j] + S.G[j * mk + i]);
      jacobi_eigh(mk, Gm.data(), w.data(), Z.data());
      S.theta = w[0];
      if (!std::isfinite(S.theta)) { set_error("non-finite Ritz value"); return DMRG_ENONFINITE; }
      S.c.assign(mk, 0.0);
      for (int i = 0; i < mk; i++) {
        S.c[i] = Z[i * mk + 0];
        coef[(size_t)k * M + S.cols[i]] = S.c[i];
      }
      thetas[k] = S.theta;
      // relative floor: the denominator cap scales with the spread of d - theta
      floors[k] = opt.floor * sigma_of(k, S.theta);
    }
    if ((rc = put_coef(coef)) || (rc = put_vec(thetas)) || (rc = put(dfloor, floors.data(), (size_t)np))) return rc;
    vec_combo(X, V, n, m, dcoef, M, 1.0, 0.0, u, stream);
    vec_combo(X, W, n, m, dcoef, M, 1.0, 0.0, hu, stream);
    vec_resid(X, hu, u, diag, dvec, dfloor, r, t, stream);
    if ((rc = dots_host(r, 1, r))) return rc;
    for (int k = 0; k < np; k++) {
      ProbState &S = P[k];
      if (!S.active) continue;
      S.iters = it;
      S.rnorm = std::sqrt(hout[k]);
      if (!std::isfinite(S.rnorm)) { set_error("non-finite residual"); return DMRG_ENONFINITE; }
      if (S.rnorm < S.best_r) {
        S.best_r = S.rnorm;
        S.best_it = it;
      } else if (use_mlp && S.mlp_on && it - S.best_it >= opt.mlp_patience) {
        S.mlp_on = false;   // stagnating with learned steps: diagonal steps from here on
      }
      if (S.rnorm <= opt.tol) {
        S.active = false;
        n_active--;
        HIPCHK(hipMemcpyAsync(psi + S.off, u + S.off, sizeof(double) * S.len, hipMemcpyDeviceToDevice, s));
      }
    }
    if (n_active == 0) break;
    if (opt.verbose > 0 && it % 25 == 0) {
      double rmax = 0.0;
      for (const ProbState &S : P)
        if (S.active) rmax = std::max(rmax, S.rnorm);
      std::fprintf(stderr, "# davidson iteration %d: %d of %d problems active, largest residual %.3e\n", it,
                   n_active, np, rmax);
      std::fflush(stderr);
    }
    if (col && P[0].active) {
      // exact correction of this iteration from the converged vector
      if ((rc = dots_host(u, 1, col->psi_star))) return rc;
      const double c = hout[0];
      if (std::fabs(c) >= 1e-3) {
        launch_exact_corr(col->psi_star, u, n, 1.0 / c, col->ts, stream);
        if ((rc = dots_host(col->ts, 1, col->ts))) return rc;
        const double tn = std::sqrt(hout[0]);
        if (tn > 0.0 && std::isfinite(tn) && col->rows + n <= col->cap) {
          launch_collect(diag, r, col->ts, n, P[0].theta, sigma_of(0, P[0].theta),
                         std::log10(std::max(P[0].rnorm, 1e-300)) / 8.0, std::sqrt((double)n) / tn, floors[0],
                         col->x + col->rows * MLP_IN, col->a + col->rows, col->b + col->rows, stream);
          HIPCHK(hipGetLastError());
          col->rows += n;
          col->nrec++;
        }
      }
    }
    bool mlp_live = false;
    for (const ProbState &S : P) mlp_live = mlp_live || (S.active && S.mlp_on);
    if (use_mlp && mlp_live) {
      // learned correction t_mlp = td (1 + g(x)) into tm, then the guard
      std::vector<double> sig(np, 1.0), f1(np, 0.0), th(np, 0.0);
      for (int k = 0; k < np; k++) {
        th[k] = P[k].theta;
        if (!P[k].active) continue;
        sig[k] = sigma_of(k, P[k].theta);
        f1[k] = std::log10(std::max(P[k].rnorm, 1e-300)) / 8.0;
      }
      if ((rc = put(dth, th.data(), (size_t)np)) || (rc = put(dsig, sig.data(), (size_t)np)) ||
          (rc = put(df1, f1.data(), (size_t)np)))
        return rc;
      FwdArgs A{};
      A.params = opt.mlp->p;
      A.n = n;
      A.d = diag;
      A.r = r;
      A.theta = dth;
      A.sigma = dsig;
      A.f1 = df1;
      A.seg_off = dsegoff;
      A.nseg = np;
      A.floor_ = dfloor;
      A.t = tm;
      launch_mlp_forward(opt.mlp->width, 1, A, stream);
      HIPCHK(hipGetLastError());
      if ((rc = dots_host(tm, 1, tm))) return rc;
      std::vector<double> mm(hout, hout + np);
      if ((rc = dots_host(tm, 1, t))) return rc;
      std::vector<double> mt(hout, hout + np);
      if ((rc = dots_host(t, 1, t))) return rc;
      std::vector<double> flag(np, 0.0);
      for (int k = 0; k < np; k++) {
        if (!P[k].active || !P[k].mlp_on) continue;
        const double tt = hout[k];
        const bool ok = std::isfinite(mm[k]) && std::isfinite(mt[k]) && mm[k] > 0.0 &&
                        std::fabs(mt[k]) >= DMRG_MLP_GUARD * std::sqrt(mm[k] * tt);
        flag[k] = ok ? 1.0 : 0.0;
        fallbacks += !ok;
      }
      if ((rc = put(dflag, flag.data(), (size_t)np))) return rc;
      vec_select(X, dflag, tm, t, stream);
      HIPCHK(hipStreamSynchronize(s));
    }
    if (m >= M) {
      // global thick restart: per problem span{u, u_prev} in coefficient space
      if ((rc = dots_host(V, m, uprev))) return rc;
      std::vector<double> c0((size_t)np * M, 0.0), c1((size_t)np * M, 0.0);
      std::vector<std::vector<double>> Cm(np);
      std::vector<int> kk(np, 0);
      for (int k = 0; k < np; k++) {
        ProbState &S = P[k];
        if (!S.active) continue;
        int mk = (int)S.cols.size();
        std::vector<double> a(S.c), b(mk, 0.0);
        double na = 0.0;
        for (double x : a) na += x * x;
        for (double &x : a) x /= std::sqrt(na);
        kk[k] = 1;
        if (S.have_prev) {
          for (int i = 0; i < mk; i++) b[i] = hout[(size_t)k * m + S.cols[i]];
          for (int pass = 0; pass < 2; pass++) {
            double d = 0.0;
            for (int i = 0; i < mk; i++) d += a[i] * b[i];
            for (int i = 0; i < mk; i++) b[i] -= d * a[i];
          }
          double nb = 0.0;
          for (double x : b) nb += x * x;
          if (std::sqrt(nb) > 1e-8) {
            for (double &x : b) x /= std::sqrt(nb);
            kk[k] = 2;
          }
        }
        Cm[k].assign((size_t)mk * 2, 0.0);
        for (int i = 0; i < mk; i++) {
          Cm[k][i * 2] = a[i];
          Cm[k][i * 2 + 1] = kk[k] == 2 ? b[i] : 0.0;
          c0[(size_t)k * M + S.cols[i]] = a[i];
          c1[(size_t)k * M + S.cols[i]] = kk[k] == 2 ? b[i] : 0.0;
        }
      }
      for (int j = 0; j < 2; j++) {
        if ((rc = put_coef(j == 0 ? c0 : c1))) return rc;
        vec_combo(X, V, n, m, dcoef, M, 1.0, 0.0, tmp + (int64_t)j * n, stream);
        HIPCHK(hipStreamSynchronize(s));
      }
      HIPCHK(hipMemcpyAsync(V, tmp, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, s));
      for (int j = 0; j < 2; j++) {
        if ((rc = put_coef(j == 0 ? c0 : c1))) return rc;
        vec_combo(X, W, n, m, dcoef, M, 1.0, 0.0, tmp + (int64_t)j * n, stream);
        HIPCHK(hipStreamSynchronize(s));
      }
      HIPCHK(hipMemcpyAsync(W, tmp, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, s));
      for (int k = 0; k < np; k++) {
        ProbState &S = P[k];
        if (!S.active) { S.cols.clear(); continue; }
        int mk = (int)S.cols.size(), q = kk[k];
        std::vector<double> Gn((size_t)q * q, 0.0);
        for (int a = 0; a < q; a++)
          for (int b = 0; b < q; b++) {
            double x = 0.0;
            for (int i = 0; i < mk; i++)
              for (int j = 0; j < mk; j++)
                x += Cm[k][i * 2 + a] * 0.5 * (S.G[i * mk + j] + S.G[j * mk + i]) * Cm[k][j * 2 + b];
            Gn[a * q + b] = x;
          }
        S.G = Gn;
        S.cols.clear();
        for (int a = 0; a < q; a++) S.cols.push_back(a);
      }
      m = 2;
    }
    // two-pass classical Gram-Schmidt of t against V[0:m), written into V[m]
    double *vt = V + (int64_t)m * n;
    HIPCHK(hipMemcpyAsync(vt, t, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    for (int pass = 0; pass < 2; pass++) {
      vec_dots(X, V, n, m, vt, dout, stream);
      vec_combo(X, V, n, m, dout, m, -1.0, 1.0, vt, stream);
    }
    if ((rc = dots_host(vt, 1, vt))) return rc;
    bool refill = false;
    for (int k = 0; k < np; k++)
      if (P[k].active && !(std::sqrt(hout[k]) >= 1e-12)) {
        HIPCHK(hipMemcpyAsync(vt + P[k].off, r + P[k].off, sizeof(double) * P[k].len, hipMemcpyDeviceToDevice, s));
        refill = true;
      }
    if (refill) {
      for (int pass = 0; pass < 2; pass++) {
        vec_dots(X, V, n, m, vt, dout, stream);
        vec_combo(X, V, n, m, dout, m, -1.0, 1.0, vt, stream);
      }
      if ((rc = dots_host(vt, 1, vt))) return rc;
    }
    for (int k = 0; k < np; k++) {
      if (!P[k].active) { sc[k] = 0.0; continue; }
      if (!(hout[k] > 0.0)) { set_error("Davidson subspace collapsed"); return DMRG_ENOCONV; }
      sc[k] = 1.0 / std::sqrt(hout[k]);
    }
    if ((rc = put_vec(sc))) return rc;
    vec_scale(X, dvec, vt, stream);
    if ((rc = apply(vt, W + (int64_t)m * n))) return rc;
    if ((rc = dots_host(V, m + 1, W + (int64_t)m * n))) return rc;
    for (int k = 0; k < np; k++) {
      ProbState &S = P[k];
      if (!S.active) continue;
      int mk = (int)S.cols.size();
      std::vector<double> Gn((size_t)(mk + 1) * (mk + 1), 0.0);
      for (int i = 0; i < mk; i++)
        for (int j = 0; j < mk; j++) Gn[i * (mk + 1) + j] = S.G[i * mk + j];
      for (int i = 0; i < mk; i++) {
        double x = hout[(size_t)k * (m + 1) + S.cols[i]];
        Gn[i * (mk + 1) + mk] = x;
        Gn[mk * (mk + 1) + i] = x;
      }
      Gn[mk * (mk + 1) + mk] = hout[(size_t)k * (m + 1) + m];
      S.G = Gn;
      S.cols.push_back(m);
      S.have_prev = true;
    }
    m++;
    HIPCHK(hipMemcpyAsync(uprev, u, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  }
  // problems still active: return their best pair
  for (int k = 0; k < np; k++)
    if (P[k].active)
      HIPCHK(hipMemcpyAsync(psi + P[k].off, u + P[k].off, sizeof(double) * P[k].len, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  int conv = 0, maxit = 0;
  double maxres = 0.0;
  for (int k = 0; k < np; k++) {
    evals[k] = P[k].theta;
    conv += !P[k].active;
    maxit = std::max(maxit, P[k].iters);
    maxres = std::max(maxres, P[k].rnorm);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->iters = maxit;
    st->n_hpsi = n_hpsi;
    st->fallbacks = fallbacks;
    st->switched = 0;
    for (const ProbState &S : P) st->switched += use_mlp && !S.mlp_on;
    st->converged = conv;
    st->residual = maxres;
    st->energy = P[0].theta;
    st->sigma = sigma_of(0, P[0].theta);
    st->t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    st->t_hpsi_s = t_hpsi;
  }
  if (conv < np) { set_error("Davidson did not converge for every problem; best Ritz pairs returned"); return DMRG_ENOCONV; }
  return DMRG_OK;
}

extern "C" int dmrg_debug_jacobi(int32_t m, const double *A, double *w, double *Z) {
  if (m < 1 || m > 64 || !A || !w || !Z) {
    set_error("dmrg_debug_jacobi: 1 <= m <= 64 and non-NULL arrays");
    return DMRG_EINVAL;
  }
  return dmrg::jacobi_eigh(m, A, w, Z);
}

extern "C" int dmrg_davidson(dmrg_plan_t *p, double *psi, double *evals, const dmrg_dav_opts_t *o,
                             dmrg_dav_stats_t *st, void *stream) {
  if (!p || !psi || !evals) { set_error("null argument"); return DMRG_EINVAL; }
  dmrg_dav_opts_t opt;
  int rc = check_opts(o, &opt);
  if (rc) return rc;
  return solve(p, psi, evals, opt, st, stream, nullptr);
}

extern "C" int dmrg_mlp_collect(dmrg_plan_t *p, const double *psi0, const dmrg_dav_opts_t *o, int64_t capacity,
                                float *x, float *a, float *b, int64_t *n_rows, int32_t *n_records, void *stream) {
  if (!p || !psi0 || !x || !a || !b || !n_rows || !n_records || capacity < 0) {
    set_error("null argument");
    return DMRG_EINVAL;
  }
  dmrg_dav_opts_t opt;
  int rc = check_opts(o, &opt);
  if (rc) return rc;
  opt.precond = DMRG_PRECOND_DIAG;
  opt.mlp = nullptr;
  int64_t off, len;
  if (dmrg_psi_layout(p, 1, &off, &len) == DMRG_OK) {
    set_error("training rows are collected from single-problem plans");
    return DMRG_EINVAL;
  }
  set_error("");
  if ((rc = dmrg_psi_layout(p, 0, &off, &len))) return rc;
  hipStream_t s = (hipStream_t)stream;
  DevBuf buf(p);
  double *star = buf.get(len), *ts = buf.get(len);
  if (!star || !ts) { set_error("hipMalloc failed in training-row capture"); return DMRG_ENOMEM; }
  double ev;
  HIPCHK(hipMemcpyAsync(star, psi0, sizeof(double) * len, hipMemcpyDeviceToDevice, s));
  if ((rc = solve(p, star, &ev, opt, nullptr, stream, nullptr))) return rc;
  double *work = buf.get(len);
  if (!work) { set_error("hipMalloc failed in training-row capture"); return DMRG_ENOMEM; }
  HIPCHK(hipMemcpyAsync(work, psi0, sizeof(double) * len, hipMemcpyDeviceToDevice, s));
  Collect col;
  col.psi_star = star;
  col.ts = ts;
  col.x = x;
  col.a = a;
  col.b = b;
  col.cap = capacity;
  if ((rc = solve(p, work, &ev, opt, nullptr, stream, &col))) return rc;
  *n_rows = col.rows;
  *n_records = col.nrec;
  return DMRG_OK;
}
