// Host-only entry points: error reporting, Wigner inspection and the
// test-only host evaluation of the task list.
#include "common.hpp"
#include <cmath>
#include <cstring>

namespace dmrg {
static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
}  // namespace dmrg

using namespace dmrg;

extern "C" const char *dmrg_last_error(void) { return g_last_error.c_str(); }

extern "C" double dmrg_wigner_6j(int a, int b, int c, int d, int e, int f) { return w6j(a, b, c, d, e, f); }
extern "C" double dmrg_wigner_9j(int j1, int j2, int j, int k1, int k2, int k, int j1p, int j2p, int jp) {
  return w9j(j1, j2, j, k1, k2, k, j1p, j2p, jp);
}
extern "C" double dmrg_ctilde(int j1, int j2, int j, int k1, int k2, int k, int j1p, int j2p, int jp) {
  return ctilde(j1, j2, j, k1, k2, k, j1p, j2p, jp);
}

// C (m x n) = op(A) * op(B) accumulated with scale; column-major; plain loops.
static void gemm_ref(int m, int n, int k, double s, const double *A, int lda, bool ta, const double *B,
                     int ldb, bool tb, double *C, int ldc) {
  for (int j = 0; j < n; j++)
    for (int i = 0; i < m; i++) {
      double acc = 0.0;
      for (int l = 0; l < k; l++) {
        double a = ta ? A[l + (int64_t)i * lda] : A[i + (int64_t)l * lda];
        double b = tb ? B[j + (int64_t)l * ldb] : B[l + (int64_t)j * ldb];
        acc += a * b;
      }
      C[i + (int64_t)j * ldc] += s * acc;
    }
}

extern "C" int dmrg_debug_host_apply(const dmrg_problem_t *prob, const double *psi, double *y,
                                     dmrg_plan_stats_t *st) {
  try {
    if (!prob || !psi || !y) { set_error("null argument"); return DMRG_EINVAL; }
    Tasks T;
    BlockModel L, R;
    Error err{0, ""};
    if (build_tasks_for_problem(*prob, L, R, T, err)) { set_error(err.msg); return err.code; }
    std::memset(y, 0, sizeof(double) * T.size);
    std::vector<double> dressed;
    dress_on_host(T, R, dressed);
    std::vector<double> T1;
    int64_t ntask = 0;
    for (const Task &tk : T.tasks) {
      const PsiBlock &E = T.blocks[tk.E], &F = T.blocks[tk.F];
      const Row &row = T.rows[tk.row];
      const double *X = psi + E.off;
      double *Y = y + F.off;
      for (const PosAlpha &pa : row.pos) {
        ntask++;
        double s = tk.v * pa.alpha;
        // first stage: T1 = X op(D)^T  (d_L x d_R')
        const double *Tm = X;
        int ldt = E.dL;
        if (tk.recD >= 0) {
          const dmrg_oprec_t &r = R.rec[tk.recD];
          int rows = R.sec[r.row_sec].dim, cols = R.sec[r.col_sec].dim;
          const double *D = tk.dress >= 0
                                ? dressed.data() + T.dress[tk.dress].off + (int64_t)pa.pD * rows * cols
                                : R.data + r.off + (int64_t)pa.pD * rows * cols;
          T1.assign((size_t)E.dL * F.dR, 0.0);
          if (!tk.adjD) gemm_ref(E.dL, F.dR, E.dR, 1.0, X, E.dL, false, D, rows, true, T1.data(), E.dL);
          else gemm_ref(E.dL, F.dR, E.dR, 1.0, X, E.dL, false, D, rows, false, T1.data(), E.dL);
          Tm = T1.data();
        }
        // second stage: Y += s op(A) T1
        if (tk.recA >= 0) {
          const dmrg_oprec_t &r = L.rec[tk.recA];
          int rows = L.sec[r.row_sec].dim, cols = L.sec[r.col_sec].dim;
          const double *A = L.data + r.off + (int64_t)pa.pA * rows * cols;
          if (!tk.adjA) gemm_ref(F.dL, F.dR, E.dL, s, A, rows, false, Tm, ldt, false, Y, F.dL);
          else gemm_ref(F.dL, F.dR, E.dL, s, A, rows, true, Tm, ldt, false, Y, F.dL);
        } else {
          for (int j = 0; j < F.dR; j++)
            for (int i = 0; i < F.dL; i++) Y[i + (int64_t)j * F.dL] += s * Tm[i + (int64_t)j * ldt];
        }
      }
    }
    if (st) {
      std::memset(st, 0, sizeof(*st));
      st->psi_len = T.size;
      st->n_blocks = (int64_t)T.blocks.size();
      st->n_rows = (int64_t)T.rows.size();
      st->n_tasks = ntask;
      st->flops = T.flops;
    }
    return DMRG_OK;
  } catch (const std::exception &e) {
    set_error(e.what());
    return DMRG_EINVAL;
  }
}
