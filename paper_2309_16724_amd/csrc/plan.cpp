// Plan construction (host) and the C ABI entry points that drive the GPU.
#include "plan.hpp"
#include <hip/hip_runtime_api.h>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <set>

using namespace dmrg;

namespace {

struct ProbPlan {
  BlockModel L, R;
  Tasks T;
  int64_t psi_off = 0;
  int base_l = 0, base_r = 0;
};

}  // namespace

struct dmrg_plan {
  std::vector<std::unique_ptr<ProbPlan>> probs;
  int64_t psi_len = 0;
  std::vector<const double *> bases_h;
  const double **d_bases = nullptr;
  double *d_work = nullptr;
  int64_t work_elems = 0;
  std::vector<Chunk> chunks;
  std::vector<DiagBlock> dblocks;
  std::vector<DiagTerm> dterms;
  DiagBlock *d_dblocks = nullptr;
  DiagTerm *d_dterms = nullptr;
  dmrg_plan_stats_t stats;
  int precision = 0, n_slices = 0;
  std::vector<void *> allocs;
  // profiling: events around every first- and second-stage launch
  int profiling = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<int, int>>> ev_marks;   // (stage, (start ev, stop ev))
  std::vector<double> ev_flops;                                  // algorithmic flops per mark
  ~dmrg_plan() {
    for (auto e : ev_pool) (void)hipEventDestroy(e);
  }
};

namespace {

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) {                                                            \
      set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #x);      \
      return DMRG_EHIP;                                                                \
    }                                                                                  \
  } while (0)

template <class T>
int upload(dmrg_plan *p, const std::vector<T> &v, T **out) {
  *out = nullptr;
  if (v.empty()) return DMRG_OK;
  void *d = nullptr;
  hipError_t e = hipMalloc(&d, sizeof(T) * v.size());
  if (e != hipSuccess) { set_error("hipMalloc failed for plan tables"); return DMRG_ENOMEM; }
  p->allocs.push_back(d);
  HIPCHK(hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  *out = (T *)d;
  return DMRG_OK;
}

struct StripeKey {
  int prob, E, rec, adj;
  bool operator<(const StripeKey &o) const {
    return std::tie(prob, E, rec, adj) < std::tie(o.prob, o.E, o.rec, o.adj);
  }
};

struct Stripe {
  std::vector<int> slots;   // sorted pD
  int64_t off = 0;
  int dL = 0, dRin = 0, dRout = 0;
};

struct TaskRef { int prob; int task; };

int build_plan(dmrg_plan *P, int64_t budget_bytes, bool device) {
  // ---- split tasks into chunks whose stripes fit the workspace budget
  std::vector<std::vector<TaskRef>> chunk_tasks(1);
  std::map<StripeKey, std::set<int>> cur;
  int64_t cur_bytes = 0;
  for (int k = 0; k < (int)P->probs.size(); k++) {
    const Tasks &T = P->probs[k]->T;
    for (int ti = 0; ti < (int)T.tasks.size(); ti++) {
      const Task &tk = T.tasks[ti];
      int64_t add = 0;
      StripeKey key{k, tk.E, tk.recD, tk.adjD};
      if (tk.recD >= 0) {
        const PsiBlock &E = T.blocks[tk.E], &F = T.blocks[tk.F];
        auto it = cur.find(key);
        for (const auto &pa : T.rows[tk.row].pos)
          if (it == cur.end() || !it->second.count(pa.pD)) add += (int64_t)E.dL * F.dR * 8;
      }
      if (cur_bytes + add > budget_bytes && !chunk_tasks.back().empty()) {
        chunk_tasks.emplace_back();
        cur.clear();
        cur_bytes = 0;
        add = 0;
        if (tk.recD >= 0) {
          const PsiBlock &E = T.blocks[tk.E], &F = T.blocks[tk.F];
          add = (int64_t)T.rows[tk.row].pos.size() * E.dL * F.dR * 8;
        }
      }
      if (tk.recD >= 0)
        for (const auto &pa : T.rows[tk.row].pos) cur[key].insert(pa.pD);
      cur_bytes += add;
      chunk_tasks.back().push_back({k, ti});
    }
  }
  P->stats.flops = P->stats.stage1_flops = P->stats.stage2_flops = 0.0;
  int64_t max_work = 0;
  for (auto &ct : chunk_tasks) {
    Chunk ch;
    std::map<StripeKey, Stripe> stripes;
    for (auto &r : ct) {
      const Tasks &T = P->probs[r.prob]->T;
      const Task &tk = T.tasks[r.task];
      if (tk.recD < 0) continue;
      StripeKey key{r.prob, tk.E, tk.recD, tk.adjD};
      Stripe &s = stripes[key];
      s.dL = T.blocks[tk.E].dL;
      s.dRin = T.blocks[tk.E].dR;
      s.dRout = T.blocks[tk.F].dR;
      for (const auto &pa : T.rows[tk.row].pos) s.slots.push_back(pa.pD);
    }
    int64_t woff = 0;
    for (auto &kv : stripes) {
      Stripe &s = kv.second;
      std::sort(s.slots.begin(), s.slots.end());
      s.slots.erase(std::unique(s.slots.begin(), s.slots.end()), s.slots.end());
      s.off = woff;
      woff += (int64_t)s.dL * s.dRout * s.slots.size();
      woff = (woff + 31) / 32 * 32;
      // first-stage tiles: T_slot = X_E op(D_pD)
      const ProbPlan &pp = *P->probs[kv.first.prob];
      const PsiBlock &E = pp.T.blocks[kv.first.E];
      const dmrg_oprec_t &rec = pp.R.rec[kv.first.rec];
      int rows = pp.R.sec[rec.row_sec].dim, cols = pp.R.sec[rec.col_sec].dim;
      int64_t ldt = (int64_t)s.dL * s.slots.size();
      for (size_t si = 0; si < s.slots.size(); si++) {
        Seg g{};
        g.a_base = BASE_PSI;
        g.a_off = pp.psi_off + E.off;
        g.a_p = 0; g.a_i = 1; g.a_k = s.dL;
        g.K = s.dRin; g.kb = s.dRin;
        g.b_base = pp.base_r;
        g.b_off = rec.off + (int64_t)s.slots[si] * rows * cols;
        if (!kv.first.adj) { g.b_k = rows; g.b_j = 1; }     // stored D is dR' x dR
        else { g.b_k = 1; g.b_j = rows; }                   // stored D is dR x dR'
        g.s = 1.0;
        int sidx = (int)ch.seg1.size();
        ch.seg1.push_back(g);
        P->stats.stage1_flops += 2.0 * s.dL * s.dRin * s.dRout;
        ch.flops1 += 2.0 * s.dL * s.dRin * s.dRout;
        for (int i0 = 0; i0 < s.dL; i0 += TILE)
          for (int j0 = 0; j0 < s.dRout; j0 += TILE) {
            Tile t{};
            t.c_base = BASE_WORK;
            t.c_off = s.off + (int64_t)si * s.dL;
            t.ldc = ldt;
            t.m = s.dL; t.n = s.dRout; t.i0 = i0; t.j0 = j0;
            t.seg0 = sidx; t.nseg = 1; t.accumulate = 0;
            ch.tile1.push_back(t);
          }
      }
    }
    max_work = std::max(max_work, woff);
    // second stage: segments grouped by output block
    std::map<std::pair<int, int>, std::vector<Seg>> byF;
    for (auto &r : ct) {
      const ProbPlan &pp = *P->probs[r.prob];
      const Tasks &T = pp.T;
      const Task &tk = T.tasks[r.task];
      const PsiBlock &E = T.blocks[tk.E], &F = T.blocks[tk.F];
      const Row &row = T.rows[tk.row];
      const Stripe *st = nullptr;
      if (tk.recD >= 0) st = &stripes.at(StripeKey{r.prob, tk.E, tk.recD, tk.adjD});
      auto slot_of = [&](int pD) {
        return (int)(std::lower_bound(st->slots.begin(), st->slots.end(), pD) - st->slots.begin());
      };
      int rowsA = 0, colsA = 0;
      int64_t recoffA = 0;
      if (tk.recA >= 0) {
        const dmrg_oprec_t &ra = pp.L.rec[tk.recA];
        rowsA = pp.L.sec[ra.row_sec].dim; colsA = pp.L.sec[ra.col_sec].dim;
        recoffA = ra.off;
      }
      auto &segs = byF[{r.prob, tk.F}];
      size_t q = 0;
      while (q < row.pos.size()) {
        size_t q1 = q + 1;
        if (tk.recA >= 0 && st)
          while (q1 < row.pos.size() && row.pos[q1].pA == row.pos[q1 - 1].pA + 1 &&
                 slot_of(row.pos[q1].pD) == slot_of(row.pos[q1 - 1].pD) + 1 &&
                 row.pos[q1].alpha == row.pos[q].alpha)
            q1++;
        int run = (int)(q1 - q);
        Seg g{};
        g.s = tk.v * row.pos[q].alpha;
        if (st) {
          g.b_base = BASE_WORK;
          g.b_off = st->off + (int64_t)slot_of(row.pos[q].pD) * E.dL;
          g.b_k = 1;
          g.b_j = (int64_t)E.dL * st->slots.size();
        } else {
          g.b_base = BASE_PSI;
          g.b_off = pp.psi_off + E.off;
          g.b_k = 1;
          g.b_j = E.dL;
        }
        if (tk.recA >= 0) {
          g.a_base = pp.base_l;
          g.a_off = recoffA + (int64_t)row.pos[q].pA * rowsA * colsA;
          g.a_p = (int64_t)rowsA * colsA;
          if (!tk.adjA) { g.a_i = 1; g.a_k = rowsA; }    // stored A is dL' x dL
          else { g.a_i = rowsA; g.a_k = 1; }             // stored A is dL x dL'
          g.kb = E.dL;
          g.K = run * E.dL;
          P->stats.stage2_flops += 2.0 * F.dL * g.K * F.dR;
          ch.flops2 += 2.0 * F.dL * g.K * F.dR;
        } else {
          g.a_base = -1;
          g.K = E.dL;
          g.kb = E.dL;
        }
        segs.push_back(g);
        q = q1;
      }
    }
    std::vector<std::pair<double, Tile>> tiles2;
    for (auto &kv : byF) {
      const ProbPlan &pp = *P->probs[kv.first.first];
      const PsiBlock &F = pp.T.blocks[kv.first.second];
      int seg0 = (int)ch.seg2.size();
      double kcost = 0.0;
      for (auto &g : kv.second) {
        ch.seg2.push_back(g);
        kcost += g.a_base < 0 ? 1.0 : (double)g.K;
      }
      for (int i0 = 0; i0 < F.dL; i0 += TILE)
        for (int j0 = 0; j0 < F.dR; j0 += TILE) {
          Tile t{};
          t.c_base = BASE_Y;
          t.c_off = pp.psi_off + F.off;
          t.ldc = F.dL;
          t.m = F.dL; t.n = F.dR; t.i0 = i0; t.j0 = j0;
          t.seg0 = seg0; t.nseg = (int)kv.second.size(); t.accumulate = 1;
          tiles2.push_back({kcost, t});
        }
    }
    std::stable_sort(tiles2.begin(), tiles2.end(),
                     [](const std::pair<double, Tile> &a, const std::pair<double, Tile> &b) {
                       return a.first > b.first;
                     });
    for (auto &x : tiles2) ch.tile2.push_back(x.second);
    P->chunks.push_back(std::move(ch));
  }
  P->stats.flops = P->stats.stage1_flops + P->stats.stage2_flops;
  P->stats.n_chunks = (int)P->chunks.size();
  P->stats.workspace_bytes = max_work * 8;
  P->work_elems = max_work;
  // diagonal terms (tasks whose input and output blocks coincide)
  for (int k = 0; k < (int)P->probs.size(); k++) {
    const ProbPlan &pp = *P->probs[k];
    const Tasks &T = pp.T;
    std::vector<std::vector<DiagTerm>> per(T.blocks.size());
    for (const Task &tk : T.tasks) {
      if (tk.E != tk.F) continue;
      const PsiBlock &E = T.blocks[tk.E];
      for (const auto &pa : T.rows[tk.row].pos) {
        DiagTerm d{};
        d.s = tk.v * pa.alpha;
        if (tk.recA >= 0) {
          const dmrg_oprec_t &ra = pp.L.rec[tk.recA];
          d.a_base = pp.base_l;
          d.a_off = ra.off + (int64_t)pa.pA * E.dL * E.dL;
          d.a_step = E.dL + 1;
        } else d.a_base = -1;
        if (tk.recD >= 0) {
          const dmrg_oprec_t &rd = pp.R.rec[tk.recD];
          d.d_base = pp.base_r;
          d.d_off = rd.off + (int64_t)pa.pD * E.dR * E.dR;
          d.d_step = E.dR + 1;
        } else d.d_base = -1;
        per[tk.E].push_back(d);
      }
    }
    for (size_t b = 0; b < T.blocks.size(); b++) {
      DiagBlock db{};
      db.off = pp.psi_off + T.blocks[b].off;
      db.m = T.blocks[b].dL;
      db.n = T.blocks[b].dR;
      db.t0 = (int)P->dterms.size();
      db.nt = (int)per[b].size();
      for (auto &d : per[b]) P->dterms.push_back(d);
      P->dblocks.push_back(db);
    }
  }
  if (!device) return DMRG_OK;
  // ---- upload
  int rc;
  for (auto &ch : P->chunks) {
    if ((rc = upload(P, ch.seg1, &ch.d_seg1)) || (rc = upload(P, ch.seg2, &ch.d_seg2)) ||
        (rc = upload(P, ch.tile1, &ch.d_tile1)) || (rc = upload(P, ch.tile2, &ch.d_tile2)))
      return rc;
    P->stats.n_stage1 += (int64_t)ch.seg1.size();
    P->stats.n_segments += (int64_t)ch.seg2.size();
  }
  if ((rc = upload(P, P->dblocks, &P->d_dblocks)) || (rc = upload(P, P->dterms, &P->d_dterms))) return rc;
  if ((rc = upload(P, P->bases_h, (const double ***)&P->d_bases))) return rc;
  if (P->work_elems > 0) {
    void *d = nullptr;
    if (hipMalloc(&d, sizeof(double) * P->work_elems) != hipSuccess) {
      set_error("hipMalloc failed for the stripe workspace");
      return DMRG_ENOMEM;
    }
    P->allocs.push_back(d);
    P->d_work = (double *)d;
  }
  return DMRG_OK;
}

}  // namespace

extern "C" void dmrg_plan_free(dmrg_plan_t *p) {
  if (!p) return;
  for (void *a : p->allocs) (void)hipFree(a);
  delete p;
}

extern "C" int dmrg_build_tasks(const dmrg_problem_t *probs, int32_t n_probs, const dmrg_plan_opts_t *opts,
                                void *stream, dmrg_plan_t **out) {
  (void)stream;
  if (!out) { set_error("null output pointer"); return DMRG_EINVAL; }
  *out = nullptr;
  if (!probs || n_probs <= 0) { set_error("no problems"); return DMRG_EINVAL; }
  dmrg_plan *P = new dmrg_plan();
  std::memset(&P->stats, 0, sizeof(P->stats));
  try {
    P->precision = opts ? opts->precision : DMRG_FP64;
    P->n_slices = opts ? opts->n_slices : 0;
    if (P->precision != DMRG_FP64) {
      set_error("only DMRG_FP64 is available in this build");
      dmrg_plan_free(P);
      return DMRG_EINVAL;
    }
    int64_t budget = (opts && opts->workspace_bytes > 0) ? opts->workspace_bytes : ((int64_t)16 << 30);
    int64_t off = 0;
    for (int k = 0; k < n_probs; k++) {
      auto pp = std::make_unique<ProbPlan>();
      Error err{0, ""};
      if (!probs[k].ldata && probs[k].site_l > 0) { set_error("left operator data missing"); dmrg_plan_free(P); return DMRG_EINVAL; }
      if (build_tasks_for_problem(probs[k], pp->L, pp->R, pp->T, err)) {
        set_error("problem " + std::to_string(k) + ": " + err.msg);
        dmrg_plan_free(P);
        return err.code;
      }
      pp->psi_off = off;
      off += pp->T.size;
      pp->base_l = BASE_OPS + (int)P->bases_h.size();
      P->bases_h.push_back(probs[k].ldata);
      pp->base_r = BASE_OPS + (int)P->bases_h.size();
      P->bases_h.push_back(probs[k].rdata);
      P->stats.n_blocks += (int64_t)pp->T.blocks.size();
      P->stats.n_rows += (int64_t)pp->T.rows.size();
      for (auto &tk : pp->T.tasks) P->stats.n_tasks += (int64_t)pp->T.rows[tk.row].pos.size();
      P->probs.push_back(std::move(pp));
    }
    P->psi_len = off;
    P->stats.psi_len = off;
    int rc = build_plan(P, budget, true);
    if (rc) { dmrg_plan_free(P); return rc; }
    *out = P;
    return DMRG_OK;
  } catch (const std::exception &e) {
    set_error(std::string("exception: ") + e.what());
    dmrg_plan_free(P);
    return DMRG_ENOMEM;
  }
}

extern "C" int dmrg_psi_layout(const dmrg_plan_t *p, int32_t prob, int64_t *off, int64_t *len) {
  if (!p || prob < 0 || prob >= (int)p->probs.size()) { set_error("bad plan or problem index"); return DMRG_EINVAL; }
  if (off) *off = p->probs[prob]->psi_off;
  if (len) *len = p->probs[prob]->T.size;
  return DMRG_OK;
}

static int next_event(dmrg_plan *p, size_t &idx) {
  if (idx >= p->ev_pool.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    p->ev_pool.push_back(e);
  }
  return DMRG_OK;
}

extern "C" int dmrg_apply_H(dmrg_plan_t *p, const double *psi, double *hpsi, void *stream) {
  if (!p || !psi || !hpsi) { set_error("null argument"); return DMRG_EINVAL; }
  if (psi == hpsi) { set_error("psi and hpsi must not alias"); return DMRG_EINVAL; }
  launch_zero(hpsi, p->psi_len, stream);
  size_t ev = p->ev_marks.empty() ? 0 : (size_t)p->ev_marks.back().second.second + 1;
  for (auto &ch : p->chunks) {
    for (int stage = 1; stage <= 2; stage++) {
      int e0 = -1;
      if (p->profiling) {
        int rc = next_event(p, ev);
        if (rc) return rc;
        e0 = (int)ev;
        HIPCHK(hipEventRecord(p->ev_pool[ev++], (hipStream_t)stream));
      }
      if (stage == 1)
        launch_tiles_f64(1, ch.d_tile1, ch.d_seg1, (int)ch.tile1.size(), p->d_bases, psi, hpsi, p->d_work, stream);
      else
        launch_tiles_f64(2, ch.d_tile2, ch.d_seg2, (int)ch.tile2.size(), p->d_bases, psi, hpsi, p->d_work, stream);
      if (p->profiling) {
        int rc = next_event(p, ev);
        if (rc) return rc;
        HIPCHK(hipEventRecord(p->ev_pool[ev], (hipStream_t)stream));
        p->ev_marks.push_back({stage, {e0, (int)ev}});
        p->ev_flops.push_back(stage == 1 ? ch.flops1 : ch.flops2);
        ev++;
      }
    }
  }
  HIPCHK(hipGetLastError());
  return DMRG_OK;
}

extern "C" int dmrg_set_profiling(dmrg_plan_t *p, int32_t on) {
  if (!p) { set_error("null plan"); return DMRG_EINVAL; }
  p->profiling = on ? 1 : 0;
  p->ev_marks.clear();
  p->ev_flops.clear();
  return DMRG_OK;
}

extern "C" int dmrg_get_profile(dmrg_plan_t *p, int32_t stage, int64_t *n_launches, double *total_ms,
                                double *total_flops) {
  if (!p || stage < 1 || stage > 2) { set_error("bad plan or stage"); return DMRG_EINVAL; }
  int64_t n = 0;
  double ms = 0.0, fl = 0.0;
  for (size_t i = 0; i < p->ev_marks.size(); i++) {
    if (p->ev_marks[i].first != stage) continue;
    float t = 0.0f;
    HIPCHK(hipEventSynchronize(p->ev_pool[p->ev_marks[i].second.second]));
    HIPCHK(hipEventElapsedTime(&t, p->ev_pool[p->ev_marks[i].second.first],
                               p->ev_pool[p->ev_marks[i].second.second]));
    n++;
    ms += t;
    fl += p->ev_flops[i];
  }
  if (n_launches) *n_launches = n;
  if (total_ms) *total_ms = ms;
  if (total_flops) *total_flops = fl;
  return DMRG_OK;
}

extern "C" int dmrg_diag_H(dmrg_plan_t *p, double *diag, void *stream) {
  if (!p || !diag) { set_error("null argument"); return DMRG_EINVAL; }
  launch_diag(p->d_dblocks, p->d_dterms, (int)p->dblocks.size(), p->d_bases, diag, stream);
  HIPCHK(hipGetLastError());
  return DMRG_OK;
}

extern "C" int dmrg_plan_stats(const dmrg_plan_t *p, dmrg_plan_stats_t *st) {
  if (!p || !st) { set_error("null argument"); return DMRG_EINVAL; }
  *st = p->stats;
  return DMRG_OK;
}

// ---------------------------------------------------------------------------
// Test-only: build the plan for one problem whose operator data are HOST
// arrays and execute its tile and segment lists on the CPU with the kernels'
// addressing (no GPU use).  Checks the plan layout without a device.
static void host_tiles(const std::vector<Tile> &tiles, const std::vector<Seg> &segs,
                       const std::vector<const double *> &bases, const double *psi, double *y,
                       double *work) {
  auto base = [&](int id) -> const double * {
    return id == BASE_PSI ? psi : id == BASE_Y ? y : id == BASE_WORK ? work : bases[id - BASE_OPS];
  };
  for (const Tile &T : tiles) {
    int mt = std::min(TILE, T.m - T.i0), nt = std::min(TILE, T.n - T.j0);
    std::vector<double> acc((size_t)mt * nt, 0.0);
    for (int si = 0; si < T.nseg; si++) {
      const Seg &S = segs[T.seg0 + si];
      const double *B = base(S.b_base) + S.b_off;
      if (S.a_base < 0) {
        for (int j = 0; j < nt; j++)
          for (int i = 0; i < mt; i++)
            acc[i + (size_t)j * mt] += S.s * B[(int64_t)(T.i0 + i) * S.b_k + (int64_t)(T.j0 + j) * S.b_j];
        continue;
      }
      const double *A = base(S.a_base) + S.a_off;
      for (int j = 0; j < nt; j++)
        for (int i = 0; i < mt; i++) {
          double a = 0.0;
          for (int k = 0; k < S.K; k++) {
            int p = k / S.kb, kr = k - p * S.kb;
            a += S.s * A[(int64_t)p * S.a_p + (int64_t)(T.i0 + i) * S.a_i + (int64_t)kr * S.a_k] *
                 B[(int64_t)k * S.b_k + (int64_t)(T.j0 + j) * S.b_j];
          }
          acc[i + (size_t)j * mt] += a;
        }
    }
    double *C = const_cast<double *>(base(T.c_base)) + T.c_off;
    for (int j = 0; j < nt; j++)
      for (int i = 0; i < mt; i++) {
        double &c = C[(int64_t)(T.i0 + i) + (int64_t)(T.j0 + j) * T.ldc];
        c = T.accumulate ? c + acc[i + (size_t)j * mt] : acc[i + (size_t)j * mt];
      }
  }
}

extern "C" int dmrg_debug_plan_host_apply(const dmrg_problem_t *prob, const double *psi, double *y,
                                          int64_t workspace_bytes) {
  dmrg_plan *P = new dmrg_plan();
  std::memset(&P->stats, 0, sizeof(P->stats));
  auto pp = std::make_unique<ProbPlan>();
  Error err{0, ""};
  if (build_tasks_for_problem(*prob, pp->L, pp->R, pp->T, err)) {
    set_error(err.msg);
    delete P;
    return err.code;
  }
  pp->base_l = BASE_OPS;
  pp->base_r = BASE_OPS + 1;
  P->bases_h = {prob->ldata, prob->rdata};
  int64_t n = pp->T.size;
  P->probs.push_back(std::move(pp));
  P->psi_len = n;
  int rc = build_plan(P, workspace_bytes > 0 ? workspace_bytes : ((int64_t)16 << 30), false);
  if (rc) { delete P; return rc; }
  std::vector<double> work((size_t)std::max<int64_t>(P->work_elems, 1), 0.0);
  std::memset(y, 0, sizeof(double) * n);
  for (auto &ch : P->chunks) {
    host_tiles(ch.tile1, ch.seg1, P->bases_h, psi, y, work.data());
    host_tiles(ch.tile2, ch.seg2, P->bases_h, psi, y, work.data());
  }
  delete P;
  return DMRG_OK;
}
