// Plan construction (host) and the C ABI entry points that drive the GPU.
#include "plan.hpp"
#include <hip/hip_runtime_api.h>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <chrono>
#include <climits>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <stdexcept>

using namespace dmrg;

namespace {

struct ProbPlan {
  BlockModel L, R;
  Tasks T;
  int64_t psi_off = 0;
  int base_l = 0, base_r = 0, base_dress = 0;
  // transposed copies of every operator block (operators applied as adjoints
  // are read from these, so that all operand loads run along contiguous rows)
  int base_lT = 0, base_rT = 0, base_dressT = 0;
  double *d_dress = nullptr;          // dressed right-block data (device)
  double *d_lT = nullptr, *d_rT = nullptr, *d_dressT = nullptr;
  std::vector<double> h_dress;        // host copies (test paths only)
  std::vector<double> h_lT, h_rT, h_dressT;
};

std::vector<TransJob> trans_jobs(const BlockModel &M) {
  std::vector<TransJob> v;
  for (const dmrg_oprec_t &r : M.rec)
    v.push_back({r.off, M.sec[r.row_sec].dim, M.sec[r.col_sec].dim, r.npos, 0});
  return v;
}

std::vector<TransJob> trans_jobs(const Tasks &T) {
  std::vector<TransJob> v;
  for (const Dress &d : T.dress) v.push_back({d.off, d.rows, d.cols, d.npos, 0});
  return v;
}

void transpose_on_host(const std::vector<TransJob> &jobs, const double *src, int64_t len, std::vector<double> &dst) {
  dst.assign((size_t)std::max<int64_t>(len, 1), 0.0);
  for (const TransJob &J : jobs) {
    const int64_t bs = (int64_t)J.rows * J.cols;
    for (int p = 0; p < J.npos; p++)
      for (int c = 0; c < J.cols; c++)
        for (int r = 0; r < J.rows; r++)
          dst[J.off + p * bs + c + (int64_t)r * J.cols] = src[J.off + p * bs + r + (int64_t)c * J.rows];
  }
}

}  // namespace

struct dmrg_plan {
  std::vector<std::unique_ptr<ProbPlan>> probs;
  int64_t psi_len = 0;
  std::vector<const double *> bases_h;
  const double **d_bases = nullptr;
  double *d_work = nullptr;
  int64_t work_elems = 0;
  double *d_part = nullptr;
  int64_t part_elems = 0;
  int32_t *d_counters = nullptr;      // per-XCD queue counters of the work-group launches
  std::vector<Chunk> chunks;
  std::vector<DiagBlock> dblocks;
  std::vector<DiagTerm> dterms;
  DiagBlock *d_dblocks = nullptr;
  DiagTerm *d_dterms = nullptr;
  dmrg_plan_stats_t stats;
  int precision = 0, n_slices = 0;
  // split precision
  std::vector<SliceJob> jobs_ops, jobs_psi;
  SliceJob *d_jobs_ops = nullptr, *d_jobs_psi = nullptr;
  int64_t sb_elems[N_SBUF] = {0, 0, 0, 0}, sb_exps[N_SBUF] = {0, 0, 0, 0};
  SliceBufs sb{};
  std::vector<uint16_t> h_sb[N_SBUF];      // host copies (test emulation only)
  std::vector<int32_t> h_se[N_SBUF];
  std::vector<void *> allocs;          // problem-level device memory (kept across re-planning)
  std::vector<void *> plan_allocs;     // tile lists, workspace, slices (freed by re-planning)
  // device memory source (caller's callbacks or hipMalloc)
  void *(*alloc_fn)(size_t, void *) = nullptr;
  void (*free_fn)(void *, void *) = nullptr;
  void *alloc_ctx = nullptr;
  std::string tune_cache;
  std::map<void *, size_t> sizes;      // live allocations and their sizes
  int64_t held = 0;                    // bytes held
  void *dalloc(size_t bytes) {
    bytes = std::max<size_t>(bytes, 8);
    void *p = nullptr;
    if (alloc_fn) p = alloc_fn(bytes, alloc_ctx);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (p) {
      sizes[p] = bytes;
      held += (int64_t)bytes;
    }
    return p;
  }
  void dfree(void *p) {
    if (!p) return;
    auto it = sizes.find(p);
    if (it != sizes.end()) {
      held -= (int64_t)it->second;
      sizes.erase(it);
    }
    if (free_fn) free_fn(p, alloc_ctx);
    else (void)hipFree(p);
  }
  // settings of the tile lists
  int kpart = KPART, tile_policy = 0, xcd = 0, flags = 0;
  int macro_min = MACRO_MIN;          // split plans: work-group tiles for outputs >= this (0: none)
  int wide_min = WIDE_MIN;            // split plans, s <= 5: wide tiles for outputs >= this (0: none)
  int64_t budget = DEFAULT_WORKSPACE;
  int tuned = 0;
  double tune_ms = 0.0;
  // profiling: events around every first- and second-stage launch
  int profiling = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<int, int>>> ev_marks;   // (stage, (start ev, stop ev))
  std::vector<double> ev_flops;                                  // algorithmic flops per mark
  // recorded launch sequences, one per (psi, hpsi) pair
  struct GraphEntry {
    const double *psi;
    double *y;
    hipGraph_t g;
    hipGraphExec_t x;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t cap_stream = nullptr;
  hipStream_t build_stream = nullptr;   // caller's stream of dmrg_build_tasks
  // recorded after the last launch sequence on the caller's stream: freeing
  // or re-planning waits for it instead of for the whole device
  hipEvent_t done_ev = nullptr;
  bool done_pending = false;
  void wait_done() {
    if (done_ev && done_pending) (void)hipEventSynchronize(done_ev);
    if (cap_stream) (void)hipStreamSynchronize(cap_stream);
    (void)hipStreamSynchronize(build_stream);
    done_pending = false;
  }
  int mark_done(void *stream) {
    if (!done_ev && hipEventCreateWithFlags(&done_ev, hipEventDisableTiming) != hipSuccess) return DMRG_EHIP;
    if (hipEventRecord(done_ev, (hipStream_t)stream) != hipSuccess) return DMRG_EHIP;
    done_pending = true;
    return DMRG_OK;
  }
  void drop_graphs() {
    for (auto &e : graphs) {
      (void)hipGraphExecDestroy(e.x);
      (void)hipGraphDestroy(e.g);
    }
    graphs.clear();
  }
  ~dmrg_plan() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (done_ev) (void)hipEventDestroy(done_ev);
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
int upload(dmrg_plan *p, const std::vector<T> &v, T **out, bool plan_level = true) {
  *out = nullptr;
  if (v.empty()) return DMRG_OK;
  void *d = p->dalloc(sizeof(T) * v.size());
  if (!d) { set_error("device allocation failed for plan tables"); return DMRG_ENOMEM; }
  (plan_level ? p->plan_allocs : p->allocs).push_back(d);
  HIPCHK(hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  *out = (T *)d;
  return DMRG_OK;
}

struct StripeKey {
  int prob, E, rec, adj, dress;
  bool operator<(const StripeKey &o) const {
    return std::tie(prob, E, rec, adj, dress) < std::tie(o.prob, o.E, o.rec, o.adj, o.dress);
  }
};

struct Stripe {
  std::vector<int> slots;   // sorted pD
  int64_t off = 0;
  int dL = 0, dRin = 0, dRout = 0;
  int index = 0;
};

struct TaskRef { int prob; int task; };

// MFMA row blocks of the tiles of an m x n output: skinny outputs get 16x64 or
// 64x16 tiles, the rest 32x32
int tile_mb(int m, int n, int policy) {
  if (m <= 16) return 1;
  if (policy == 0 && n <= 16) return 4;
  return 2;
}

// Grid cells (row tile, column tile) of an nr x nc tile grid in patches of
// PATCH x PATCH, patch-major, row-major inside a patch.  Work groups take
// consecutive list entries (on one XCD with DMRG_PLAN_XCD), so the tiles that
// run side by side share PATCH operand row bands and PATCH column bands in
// that XCD's L2 instead of each fetching its own.
constexpr int PATCH = 8;
std::vector<std::pair<int, int>> patch_order(int nr, int nc) {
  std::vector<std::pair<int, int>> v;
  for (int pr = 0; pr < nr; pr += PATCH)
    for (int pc = 0; pc < nc; pc += PATCH)
      for (int r = pr; r < std::min(nr, pr + PATCH); r++)
        for (int c = pc; c < std::min(nc, pc + PATCH); c++) v.push_back({r, c});
  return v;
}

// algorithmic flops of a tile list: 2 (tile rows) (tile columns) K over its
// segments with a left operator (identity segments are additions)
double list_flops(const std::vector<Tile> &tiles, const std::vector<Seg> &segs) {
  double f = 0.0;
  for (const Tile &t : tiles) {
    const double mt = std::min(tile_rows(t.mb), t.m - t.i0), nt = std::min(tile_cols(t.mb), t.n - t.j0);
    for (int i = 0; i < t.nseg; i++)
      if (segs[t.seg0 + i].a_base >= 0) f += 2.0 * mt * nt * segs[t.seg0 + i].K;
  }
  return f;
}

// NXCD contiguous ranges of a tile list with about equal summed cost
XcdQueues xcd_queues(const std::vector<double> &cost) {
  XcdQueues q{};
  double tot = 0.0;
  for (double c : cost) tot += c;
  const int n = (int)cost.size();
  double acc = 0.0;
  int i = 0;
  q.start[0] = 0;
  for (int x = 1; x < NXCD; x++) {
    while (i < n && acc + 0.5 * cost[i] < tot * x / NXCD) acc += cost[i++];
    q.start[x] = i;
  }
  q.start[NXCD] = n;
  return q;
}

// work-group tiles for split plans whose output is at least macro_min on both sides
bool use_macro(const dmrg_plan *P, int m, int n) {
  return P->precision == DMRG_SPLIT_BF16 && P->macro_min > 0 && m >= P->macro_min && n >= P->macro_min;
}

bool use_wide(const dmrg_plan *P, int m, int n) {
  return P->precision == DMRG_SPLIT_BF16 && P->n_slices <= WIDE_MAX_SLICES && P->wide_min > 0 &&
         m >= P->wide_min && n >= P->wide_min;
}

// Tiles of an m x n output (top-left corner and kind mb).  Outputs that take
// wide tiles are cut into 128-wide row and column bands (a last band of at
// least wide_min lines is wide too): the wide x wide cells in patch order,
// then the rest of the output -- the columns beyond the wide bands next to
// them, then the rows below -- in tiles chosen for those strips.  Other
// outputs get one kind of tile in patch order.
struct Cell { int i0, j0, mb; };
std::vector<Cell> output_cells(const dmrg_plan *P, int m, int n) {
  std::vector<Cell> v;
  auto grid = [&](int r0, int c0, int rows, int cols) {
    if (rows <= 0 || cols <= 0) return;
    const int mb = use_macro(P, rows, cols) ? MACRO_MB : tile_mb(rows, cols, P->tile_policy);
    const int tr = tile_rows(mb), tc = tile_cols(mb);
    for (const auto &c : patch_order((rows + tr - 1) / tr, (cols + tc - 1) / tc))
      v.push_back({r0 + c.first * tr, c0 + c.second * tc, mb});
  };
  if (!use_wide(P, m, n)) {
    grid(0, 0, m, n);
    return v;
  }
  const int tail = std::min(P->wide_min, WIDE_EDGE);
  auto bands = [&](int len) { return len / WIDE_EDGE + (len % WIDE_EDGE >= tail ? 1 : 0); };
  const int nr = bands(m), nc = bands(n);
  const int mw = std::min(m, nr * WIDE_EDGE), nw = std::min(n, nc * WIDE_EDGE);
  for (const auto &c : patch_order(nr, nc)) v.push_back({c.first * WIDE_EDGE, c.second * WIDE_EDGE, WIDE_MB});
  grid(0, nw, mw, n - nw);
  grid(mw, 0, m - mw, n);
  return v;
}

int prepare_device(dmrg_plan *P);
int autotune(dmrg_plan *P, void *stream);
int replan(dmrg_plan *P);

int build_plan(dmrg_plan *P, int64_t budget_bytes, bool device) {
  const bool trow = P->precision != DMRG_SPLIT_BF16;   // stripe layout, see the first stage
  // ---- split tasks into chunks whose stripes fit the workspace budget
  std::vector<std::vector<TaskRef>> chunk_tasks(1);
  std::map<StripeKey, std::set<int>> cur;
  int64_t cur_bytes = 0;
  for (int k = 0; k < (int)P->probs.size(); k++) {
    const Tasks &T = P->probs[k]->T;
    for (int ti = 0; ti < (int)T.tasks.size(); ti++) {
      const Task &tk = T.tasks[ti];
      int64_t add = 0;
      StripeKey key{k, tk.E, tk.recD, tk.adjD, tk.dress};
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
      StripeKey key{r.prob, tk.E, tk.recD, tk.adjD, tk.dress};
      Stripe &s = stripes[key];
      s.dL = T.blocks[tk.E].dL;
      s.dRin = T.blocks[tk.E].dR;
      s.dRout = T.blocks[tk.F].dR;
      for (const auto &pa : T.rows[tk.row].pos) s.slots.push_back(pa.pD);
    }
    int64_t woff = 0;
    std::vector<double> cost1, cost1m, cost1x;   // K of every stage-1 tile
    for (auto &kv : stripes) {
      Stripe &s = kv.second;
      std::sort(s.slots.begin(), s.slots.end());
      s.slots.erase(std::unique(s.slots.begin(), s.slots.end()), s.slots.end());
      s.off = woff;
      s.index = (int)ch.stripes.size();
      ch.stripes.push_back({kv.first.prob, kv.first.E, kv.first.rec, kv.first.adj, kv.first.dress, woff, s.dL,
                            s.dRin, s.dRout, (int)s.slots.size(), 0});
      woff += (int64_t)s.dL * s.dRout * s.slots.size();
      woff = (woff + 31) / 32 * 32;
      // first stage: T_h = X [op(D_s0) ... op(D_s1-1)] for each run of consecutive positions.
      // FP64 plans store the stripe as a row-major d_L x (nslots d_R') matrix
      // (slot s in columns [s d_R', (s+1) d_R')), so that both stages access
      // it along rows; split plans slice it per column and store it
      // column-major (slot s is the d_L x d_R' block at off + s d_L d_R').
      const ProbPlan &pp = *P->probs[kv.first.prob];
      const PsiBlock &E = pp.T.blocks[kv.first.E];
      const dmrg_oprec_t &rec = pp.R.rec[kv.first.rec];
      int rows = pp.R.sec[rec.row_sec].dim, cols = pp.R.sec[rec.col_sec].dim;
      size_t s0 = 0;
      while (s0 < s.slots.size()) {
        size_t s1 = s0 + 1;
        while (s1 < s.slots.size() && s.slots[s1] == s.slots[s1 - 1] + 1) s1++;
        Seg g{};
        g.a_base = BASE_PSI;
        g.a_off = pp.psi_off + E.off;
        g.a_p = 0; g.a_i = 1; g.a_k = s.dL;
        g.K = s.dRin; g.a_kb = s.dRin;
        const bool dressed = kv.first.dress >= 0, adj = kv.first.adj != 0;
        if (dressed) {
          g.b_base = adj ? pp.base_dressT : pp.base_dress;
          g.b_off = pp.T.dress[kv.first.dress].off + (int64_t)s.slots[s0] * rows * cols;
        } else {
          g.b_base = adj ? pp.base_rT : pp.base_r;
          g.b_off = rec.off + (int64_t)s.slots[s0] * rows * cols;
        }
        g.b_kb = s.dRin; g.b_pk = 0;
        g.b_nb = s.dRout; g.b_pn = (int64_t)rows * cols;
        if (!adj) { g.b_k = rows; g.b_n = 1; }    // op(D) = D^T, D stored d_R' x d_R
        else { g.b_k = cols; g.b_n = 1; }         // op(D) = D from the transposed copy (d_R' x d_R)
        g.s = 1.0;
        int sidx = (int)ch.seg1.size();
        ch.seg1.push_back(g);
        ch.s1info.push_back({s.index, (int)s0, s.slots[s0]});
        int N = (int)(s1 - s0) * s.dRout;
        double fl = 2.0 * s.dL * s.dRin * N;
        P->stats.stage1_flops += fl;
        ch.flops1 += fl;
        for (const Cell &cell : output_cells(P, s.dL, N)) {
            const int i0 = cell.i0, j0 = cell.j0, mb = cell.mb;
            Tile t{};
            t.c_base = BASE_WORK;
            if (trow) {
              t.c_off = s.off + (int64_t)s0 * s.dRout;
              t.ldc = (int64_t)s.slots.size() * s.dRout;
              t.rowmajor = 1;
            } else {
              t.c_off = s.off + (int64_t)s0 * s.dL * s.dRout;
              t.ldc = s.dL;
            }
            t.m = s.dL; t.n = N; t.i0 = i0; t.j0 = j0; t.ci0 = i0; t.cj0 = j0;
            t.mb = mb;
            t.seg0 = sidx; t.nseg = 1; t.accumulate = 0;
            if (mb == WIDE_MB) {
              ch.tile1x.push_back(t);
              cost1x.push_back(s.dRin);
            } else if (mb == MACRO_MB) {
              ch.tile1m.push_back(t);
              cost1m.push_back(s.dRin);
            } else {
              ch.tile1.push_back(t);
              cost1.push_back(s.dRin);
            }
          }
        s0 = s1;
      }
    }
    max_work = std::max(max_work, woff);
    // second stage: segments grouped by output block
    std::map<std::pair<int, int>, std::vector<std::pair<Seg, Seg2Info>>> byF;
    for (auto &r : ct) {
      const ProbPlan &pp = *P->probs[r.prob];
      const Tasks &T = pp.T;
      const Task &tk = T.tasks[r.task];
      const PsiBlock &E = T.blocks[tk.E], &F = T.blocks[tk.F];
      const Row &row = T.rows[tk.row];
      const Stripe *st = nullptr;
      if (tk.recD >= 0) st = &stripes.at(StripeKey{r.prob, tk.E, tk.recD, tk.adjD, tk.dress});
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
        if (st && trow) {
          // B = [T_s; T_s+1; ...]: slot s of the row-major stripe in columns s d_R'..
          g.b_base = BASE_WORK;
          g.b_off = st->off + (int64_t)slot_of(row.pos[q].pD) * F.dR;
          g.b_kb = E.dL;
          g.b_pk = F.dR;
          g.b_k = (int64_t)st->slots.size() * F.dR;
          g.b_n = 1;
        } else if (st) {
          // column-major stripe: slot s is the d_L x d_R' block at s d_L d_R'
          g.b_base = BASE_WORK;
          g.b_off = st->off + (int64_t)slot_of(row.pos[q].pD) * E.dL * F.dR;
          g.b_kb = E.dL;
          g.b_pk = (int64_t)E.dL * F.dR;
          g.b_k = 1;
          g.b_n = E.dL;
        } else {
          g.b_base = BASE_PSI;
          g.b_off = pp.psi_off + E.off;
          g.b_kb = E.dL;
          g.b_pk = 0;
          g.b_k = 1;
          g.b_n = E.dL;
        }
        g.b_nb = F.dR; g.b_pn = 0;
        Seg2Info inf{r.prob, tk.E, st ? st->index : -1, st ? slot_of(row.pos[q].pD) : 0,
                     tk.recA, tk.adjA, row.pos[q].pA, run};
        if (tk.recA >= 0) {
          g.a_base = tk.adjA ? pp.base_lT : pp.base_l;
          g.a_off = recoffA + (int64_t)row.pos[q].pA * rowsA * colsA;
          g.a_p = (int64_t)rowsA * colsA;
          if (!tk.adjA) { g.a_i = 1; g.a_k = rowsA; }    // stored A is d_L' x d_L
          else { g.a_i = 1; g.a_k = colsA; }             // A stored d_L x d_L', read from its transpose
          g.a_kb = E.dL;
          g.K = run * E.dL;
          P->stats.stage2_flops += 2.0 * F.dL * g.K * F.dR;
          ch.flops2 += 2.0 * F.dL * g.K * F.dR;
        } else {
          g.a_base = -1;
          g.K = E.dL;
          g.a_kb = E.dL;
        }
        segs.push_back({g, inf});
        q = q1;
      }
    }
    std::vector<std::pair<double, Tile>> tiles2, tiles2m, tiles2x;
    int64_t npart = 0;   // partial-tile elements
    for (auto &kv : byF) {
      const ProbPlan &pp = *P->probs[kv.first.first];
      const PsiBlock &F = pp.T.blocks[kv.first.second];
      // pieces of at most KPART along K, cut at position boundaries
      std::vector<Seg> pieces;
      std::vector<Seg2Info> pinfo;
      for (auto &gi : kv.second) {
        const Seg &g = gi.first;
        if (g.a_base < 0 || g.K <= P->kpart) { pieces.push_back(g); pinfo.push_back(gi.second); continue; }
        int npos = g.K / g.a_kb;
        int per = std::max(1, P->kpart / g.a_kb);
        for (int p0 = 0; p0 < npos; p0 += per) {
          int p1 = std::min(npos, p0 + per);
          Seg h = g;
          h.a_off += (int64_t)p0 * g.a_p;
          h.b_off += (int64_t)p0 * g.b_pk;
          h.K = (p1 - p0) * g.a_kb;
          pieces.push_back(h);
          Seg2Info hi = gi.second;
          hi.pA0 += p0;
          hi.slot0 += p0;
          hi.run = p1 - p0;
          pinfo.push_back(hi);
        }
      }
      // parts: consecutive pieces with summed K up to KPART (identity pieces count as d_L)
      std::vector<std::pair<int, int>> parts;   // [begin, end) into pieces
      std::vector<double> pcost;
      int b0 = 0;
      double cost = 0.0;
      for (int i = 0; i < (int)pieces.size(); i++) {
        double c = pieces[i].a_base < 0 ? 0.25 * pieces[i].K : (double)pieces[i].K;
        if (i > b0 && cost + c > P->kpart) {
          parts.push_back({b0, i});
          pcost.push_back(cost);
          b0 = i;
          cost = 0.0;
        }
        cost += c;
      }
      parts.push_back({b0, (int)pieces.size()});
      pcost.push_back(cost);
      int seg0 = (int)ch.seg2.size();
      for (auto &g : pieces) ch.seg2.push_back(g);
      for (auto &gi : pinfo) ch.s2info.push_back(gi);
      const auto cells = output_cells(P, F.dL, F.dR);
      const int np = (int)parts.size();
      // partial tiles of cell c, part p at npart + coff[c] + p tm tn (tm x tn
      // the cell's tile shape); the list runs over parts (outer) and cells in
      // patch order (inner), so the tiles that run together share their K range
      std::vector<int64_t> coff(cells.size() + 1, 0);
      for (size_t c = 0; c < cells.size(); c++)
        coff[c + 1] = coff[c] + (int64_t)np * tile_rows(cells[c].mb) * tile_cols(cells[c].mb);
      for (int pi = 0; pi < np; pi++)
        for (size_t c = 0; c < cells.size(); c++) {
          const int i0 = cells[c].i0, j0 = cells[c].j0, mb = cells[c].mb;
          const int tm = tile_rows(mb), tn = tile_cols(mb);
          auto &dst = mb == WIDE_MB ? tiles2x : mb == MACRO_MB ? tiles2m : tiles2;
          Tile t{};
          t.m = F.dL; t.n = F.dR; t.i0 = i0; t.j0 = j0; t.mb = mb;
          t.seg0 = seg0 + parts[pi].first;
          t.nseg = parts[pi].second - parts[pi].first;
          if (np == 1) {
            t.c_base = BASE_Y;
            t.c_off = pp.psi_off + F.off;
            t.ldc = F.dL;
            t.ci0 = i0; t.cj0 = j0;
            t.accumulate = 1;
          } else {
            if (pi == 0) {
              Reduce r{};
              r.y_off = pp.psi_off + F.off;
              r.ldc = F.dL;
              r.part_off = npart + coff[c];
              r.m = F.dL; r.n = F.dR; r.i0 = i0; r.j0 = j0; r.tm = tm; r.tn = tn;
              r.nparts = np;
              ch.red2.push_back(r);
            }
            t.c_base = BASE_PART;
            t.c_off = npart + coff[c] + (int64_t)pi * tm * tn;
            t.ldc = tm;
            t.ci0 = 0; t.cj0 = 0;
            t.accumulate = 0;
          }
          dst.push_back({pcost[pi], t});
        }
      if (np > 1) npart += coff[cells.size()];
    }
    ch.part_elems = npart;
    P->part_elems = std::max(P->part_elems, ch.part_elems);
    auto by_cost = [](const std::pair<double, Tile> &a, const std::pair<double, Tile> &b) {
      return a.first > b.first;
    };
    std::stable_sort(tiles2.begin(), tiles2.end(), by_cost);
    std::stable_sort(tiles2m.begin(), tiles2m.end(), by_cost);
    std::stable_sort(tiles2x.begin(), tiles2x.end(), by_cost);
    std::vector<double> cost2, cost2m, cost2x;
    for (auto &x : tiles2) {
      ch.tile2.push_back(x.second);
      cost2.push_back(x.first);
    }
    for (auto &x : tiles2m) {
      ch.tile2m.push_back(x.second);
      cost2m.push_back(x.first);
    }
    for (auto &x : tiles2x) {
      ch.tile2x.push_back(x.second);
      cost2x.push_back(x.first);
    }
    ch.q1 = xcd_queues(cost1);
    ch.q2 = xcd_queues(cost2);
    ch.flops1m = list_flops(ch.tile1m, ch.seg1);
    ch.flops1w = list_flops(ch.tile1, ch.seg1);
    ch.flops2m = list_flops(ch.tile2m, ch.seg2);
    ch.flops2w = list_flops(ch.tile2, ch.seg2);
    ch.q1m = xcd_queues(cost1m);
    ch.q2m = xcd_queues(cost2m);
    ch.flops1x = list_flops(ch.tile1x, ch.seg1);
    ch.flops2x = list_flops(ch.tile2x, ch.seg2);
    ch.q1x = xcd_queues(cost1x);
    ch.q2x = xcd_queues(cost2x);
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
          if (tk.dress >= 0) {
            d.d_base = pp.base_dress;
            d.d_off = T.dress[tk.dress].off + (int64_t)pa.pD * E.dR * E.dR;
          } else {
            d.d_base = pp.base_r;
            d.d_off = rd.off + (int64_t)pa.pD * E.dR * E.dR;
          }
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
        (rc = upload(P, ch.tile1, &ch.d_tile1)) || (rc = upload(P, ch.tile2, &ch.d_tile2)) ||
        (rc = upload(P, ch.tile1m, &ch.d_tile1m)) || (rc = upload(P, ch.tile2m, &ch.d_tile2m)) ||
        (rc = upload(P, ch.tile1x, &ch.d_tile1x)) || (rc = upload(P, ch.tile2x, &ch.d_tile2x)) ||
        (rc = upload(P, ch.red2, &ch.d_red2)))
      return rc;
    P->stats.n_stage1 += (int64_t)ch.seg1.size();
    P->stats.n_segments += (int64_t)ch.seg2.size();
  }
  if ((rc = upload(P, P->dblocks, &P->d_dblocks)) || (rc = upload(P, P->dterms, &P->d_dterms))) return rc;
  if (P->work_elems > 0) {
    void *d = P->dalloc(sizeof(double) * P->work_elems);
    if (!d) {
      set_error("device allocation failed for the stripe workspace");
      return DMRG_ENOMEM;
    }
    P->plan_allocs.push_back(d);
    P->d_work = (double *)d;
  }
  {
    void *d = P->dalloc(sizeof(int32_t) * QUEUE_INTS);
    if (!d) {
      set_error("device allocation failed for the work queue counters");
      return DMRG_ENOMEM;
    }
    P->plan_allocs.push_back(d);
    P->d_counters = (int32_t *)d;
  }
  if (P->part_elems > 0) {
    void *d = P->dalloc(sizeof(double) * P->part_elems);
    if (!d) {
      set_error("device allocation failed for the partial-tile buffer");
      return DMRG_ENOMEM;
    }
    P->plan_allocs.push_back(d);
    P->d_part = (double *)d;
  }
  return DMRG_OK;
}

// Device data that depend on the problems only: operand base table, dressed
// right-block operators and transposed operator copies (kept across
// re-planning).
int prepare_device(dmrg_plan *P) {
  int rc;
  if ((rc = upload(P, P->bases_h, (const double ***)&P->d_bases, false))) return rc;
  // dressed right-block operators: computed on the device once
  for (auto &ppu : P->probs) {
    ProbPlan &pp = *ppu;
    if (pp.T.dress.empty()) continue;
    std::vector<DressItem> items;
    std::vector<int64_t> soff;
    std::vector<double> alpha;
    for (const Dress &d : pp.T.dress) {
      const dmrg_oprec_t &r = pp.R.rec[d.rec];
      int64_t bs = (int64_t)d.rows * d.cols;
      for (int j = 0; j < d.npos; j++) {
        DressItem it{};
        it.dst_off = d.off + (int64_t)j * bs;
        it.n = bs;
        it.t0 = (int)soff.size();
        for (int t = d.start[j]; t < d.start[j + 1]; t++) {
          soff.push_back(r.off + (int64_t)d.src_pos[t] * bs);
          alpha.push_back(d.src_alpha[t]);
        }
        it.t1 = (int)soff.size();
        it.src_base = pp.base_r;
        it.dst_base = pp.base_dress;
        items.push_back(it);
      }
    }
    DressItem *d_items = nullptr;
    int64_t *d_soff = nullptr;
    double *d_alpha = nullptr;
    if ((rc = upload(P, items, &d_items, false)) || (rc = upload(P, soff, &d_soff, false)) ||
        (rc = upload(P, alpha, &d_alpha, false)))
      return rc;
    launch_dress(d_items, (int)items.size(), d_soff, d_alpha, P->d_bases, pp.d_dress, P->build_stream);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(P->build_stream));
  // transposed operator copies
  for (auto &ppu : P->probs) {
    ProbPlan &pp = *ppu;
    const double *src[3] = {P->bases_h[pp.base_l - BASE_OPS], P->bases_h[pp.base_r - BASE_OPS], pp.d_dress};
    double *dst[3] = {pp.d_lT, pp.d_rT, pp.d_dressT};
    std::vector<TransJob> jobs[3] = {trans_jobs(pp.L), trans_jobs(pp.R), trans_jobs(pp.T)};
    for (int q = 0; q < 3; q++) {
      if (!src[q] || !dst[q] || jobs[q].empty()) continue;
      TransJob *d_jobs = nullptr;
      if ((rc = upload(P, jobs[q], &d_jobs, false))) return rc;
      launch_transpose(d_jobs, (int)jobs[q].size(), src[q], dst[q], P->build_stream);
      HIPCHK(hipGetLastError());
    }
  }
  HIPCHK(hipStreamSynchronize(P->build_stream));
  return DMRG_OK;
}

}  // namespace


// ---------------------------------------------------------------------------
// Split-precision plan: slice layouts of every operand and split segments
// parallel to the FP64 segments (same tiles, parts and reduction).
namespace {

struct VarInfo { int64_t off, exp; int kbp; int64_t line_len; int lines_per_pos; };

static int rup8(int x) { return (x + 7) / 8 * 8; }

// every slicing job's line must have fewer than 2^31 values (32-bit indexing)
static void check_jobs(const std::vector<SliceJob> &jobs) {
  for (const SliceJob &j : jobs)
    if ((int64_t)j.npos * j.kbp >= ((int64_t)1 << 31)) throw std::length_error("slice line longer than 2^31");
}

void build_split(dmrg_plan *P) {
  for (int b = 0; b < N_SBUF; b++) P->sb_elems[b] = P->sb_exps[b] = 0;
  P->jobs_ops.clear();
  P->jobs_psi.clear();
  // operator-record variants: 0 A rows (adjA=0), 1 A columns (adjA=1),
  // 2 D for adjD=0 (lines = stored rows per position), 3 D for adjD=1 (stored columns)
  std::map<std::array<int, 4>, VarInfo> vars;   // (prob, source (0 L rec, 1 R rec, 2 dressed), index, variant)
  auto variant = [&](int prob, int srcsel, int idx, int var) -> VarInfo {
    std::array<int, 4> key{prob, srcsel, idx, var};
    auto it = vars.find(key);
    if (it != vars.end()) return it->second;
    const ProbPlan &pp = *P->probs[prob];
    int R0, C0, npos, base;
    int64_t src_off;
    if (srcsel == 0) {
      const dmrg_oprec_t &r = pp.L.rec[idx];
      R0 = pp.L.sec[r.row_sec].dim; C0 = pp.L.sec[r.col_sec].dim; npos = r.npos; base = pp.base_l; src_off = r.off;
    } else if (srcsel == 1) {
      const dmrg_oprec_t &r = pp.R.rec[idx];
      R0 = pp.R.sec[r.row_sec].dim; C0 = pp.R.sec[r.col_sec].dim; npos = r.npos; base = pp.base_r; src_off = r.off;
    } else {
      const Dress &d = pp.T.dress[idx];
      R0 = d.rows; C0 = d.cols; npos = d.npos; base = pp.base_dress; src_off = d.off;
    }
    VarInfo v{};
    v.off = P->sb_elems[SBUF_OPS];
    v.exp = P->sb_exps[SBUF_OPS];
    int64_t bs = (int64_t)R0 * C0;
    if (var == 0 || var == 1) {
      int nrho = var == 0 ? R0 : C0, kb = var == 0 ? C0 : R0;
      v.kbp = rup8(kb);
      v.line_len = (int64_t)npos * v.kbp;
      v.lines_per_pos = 0;
      SliceJob j{};
      j.src_base = base; j.src_off = src_off;
      j.s_rho = var == 0 ? 1 : R0; j.s_pos = bs; j.s_k = var == 0 ? R0 : 1;
      j.dst_buf = SBUF_OPS; j.dst_off = v.off; j.exp_off = v.exp;
      j.nrho = nrho; j.npos = npos; j.kb = kb; j.kbp = v.kbp;
      P->jobs_ops.push_back(j);
      P->sb_elems[SBUF_OPS] += (int64_t)nrho * v.line_len;
      P->sb_exps[SBUF_OPS] += nrho;
    } else {
      int nrho = var == 2 ? R0 : C0, kb = var == 2 ? C0 : R0;
      v.kbp = rup8(kb);
      v.line_len = v.kbp;
      v.lines_per_pos = nrho;
      for (int p = 0; p < npos; p++) {
        SliceJob j{};
        j.src_base = base; j.src_off = src_off + (int64_t)p * bs;
        j.s_rho = var == 2 ? 1 : R0; j.s_pos = 0; j.s_k = var == 2 ? R0 : 1;
        j.dst_buf = SBUF_OPS; j.dst_off = v.off + (int64_t)p * nrho * v.kbp; j.exp_off = v.exp + (int64_t)p * nrho;
        j.nrho = nrho; j.npos = 1; j.kb = kb; j.kbp = v.kbp;
        P->jobs_ops.push_back(j);
      }
      P->sb_elems[SBUF_OPS] += (int64_t)npos * nrho * v.kbp;
      P->sb_exps[SBUF_OPS] += (int64_t)npos * nrho;
    }
    vars[key] = v;
    return v;
  };
  // psi slices: every block as a first-stage A operand (rows over columns) and
  // as a second-stage B operand (columns over rows)
  std::vector<std::vector<std::array<int64_t, 4>>> psi_off(P->probs.size());   // rows off/exp, cols off/exp
  for (int k = 0; k < (int)P->probs.size(); k++) {
    const ProbPlan &pp = *P->probs[k];
    for (const PsiBlock &E : pp.T.blocks) {
      std::array<int64_t, 4> o{};
      SliceJob j{};
      j.src_base = BASE_PSI; j.src_off = pp.psi_off + E.off;
      j.s_rho = 1; j.s_pos = 0; j.s_k = E.dL;
      j.nrho = E.dL; j.npos = 1; j.kb = E.dR; j.kbp = rup8(E.dR);
      j.dst_buf = SBUF_PSIR; j.dst_off = P->sb_elems[SBUF_PSIR]; j.exp_off = P->sb_exps[SBUF_PSIR];
      o[0] = j.dst_off; o[1] = j.exp_off;
      P->sb_elems[SBUF_PSIR] += (int64_t)E.dL * j.kbp;
      P->sb_exps[SBUF_PSIR] += E.dL;
      P->jobs_psi.push_back(j);
      SliceJob c{};
      c.src_base = BASE_PSI; c.src_off = pp.psi_off + E.off;
      c.s_rho = E.dL; c.s_pos = 0; c.s_k = 1;
      c.nrho = E.dR; c.npos = 1; c.kb = E.dL; c.kbp = rup8(E.dL);
      c.dst_buf = SBUF_PSIC; c.dst_off = P->sb_elems[SBUF_PSIC]; c.exp_off = P->sb_exps[SBUF_PSIC];
      o[2] = c.dst_off; o[3] = c.exp_off;
      P->sb_elems[SBUF_PSIC] += (int64_t)E.dR * c.kbp;
      P->sb_exps[SBUF_PSIC] += E.dR;
      P->jobs_psi.push_back(c);
      psi_off[k].push_back(o);
    }
  }
  int64_t t_elems_max = 0, t_exps_max = 0;
  for (auto &ch : P->chunks) {
    ch.sseg1.clear();
    ch.sseg2.clear();
    ch.tjobs.clear();
    ch.titems.clear();
    // stripe slices (second-stage B operands), per chunk
    std::vector<std::array<int64_t, 3>> toff;   // off, exp, kbp
    int64_t te = 0, tx = 0;
    for (const StripeInfo &si : ch.stripes) {
      SliceJob j{};
      j.src_base = BASE_WORK; j.src_off = si.off;
      j.s_rho = si.dL; j.s_pos = (int64_t)si.dL * si.dRout; j.s_k = 1;   // column-major stripes
      j.nrho = si.dRout; j.npos = si.nslots; j.kb = si.dL; j.kbp = rup8(si.dL);
      j.dst_buf = SBUF_T; j.dst_off = te; j.exp_off = tx;
      toff.push_back({te, tx, j.kbp});
      const int64_t tot = (int64_t)si.dRout * si.nslots * j.kbp;
      if (tot >= ((int64_t)1 << 31)) throw std::length_error("stripe slice job longer than 2^31");
      for (int64_t e0 = 0; e0 < tot; e0 += TSLICE_CHUNK) ch.titems.push_back({(int32_t)ch.tjobs.size(), (int32_t)e0});
      te += tot;
      tx += si.dRout;
      ch.tjobs.push_back(j);
    }
    ch.t_elems = te;
    ch.t_exps = tx;
    t_elems_max = std::max(t_elems_max, te);
    t_exps_max = std::max(t_exps_max, tx);
    // first stage: X (psi rows) times op(D) (record or dressed variant)
    for (size_t i = 0; i < ch.seg1.size(); i++) {
      const Seg1Info &inf = ch.s1info[i];
      const StripeInfo &si = ch.stripes[inf.stripe];
      int var = si.adj ? 3 : 2;
      VarInfo v = si.dress >= 0 ? variant(si.prob, 2, si.dress, var) : variant(si.prob, 1, si.rec, var);
      SegS q{};
      q.a_buf = SBUF_PSIR;
      q.a_off = psi_off[si.prob][si.E][0];
      q.a_ld = rup8(si.dRin);
      q.a_exp = psi_off[si.prob][si.E][1];
      q.b_buf = SBUF_OPS;
      q.b_off = v.off + (int64_t)inf.pD0 * v.lines_per_pos * v.kbp;
      q.b_ld = v.kbp;
      q.b_exp = v.exp + (int64_t)inf.pD0 * v.lines_per_pos;
      q.K = rup8(si.dRin);
      q.t_nb = si.dRout;
      q.t_exp = toff[inf.stripe][1];
      ch.sseg1.push_back(q);
    }
    // second stage
    for (size_t i = 0; i < ch.seg2.size(); i++) {
      const Seg2Info &inf = ch.s2info[i];
      const PsiBlock &E = P->probs[inf.prob]->T.blocks[inf.E];
      SegS q{};
      q.t_exp = -1;
      if (inf.recA < 0) {
        q.K = 0;
        ch.sseg2.push_back(q);
        continue;
      }
      VarInfo v = variant(inf.prob, 0, inf.recA, inf.adjA ? 1 : 0);
      q.a_buf = SBUF_OPS;
      q.a_off = v.off + (int64_t)inf.pA0 * v.kbp;
      q.a_ld = v.line_len;
      q.a_exp = v.exp;
      if (inf.stripe >= 0) {
        const StripeInfo &si = ch.stripes[inf.stripe];
        q.b_buf = SBUF_T;
        q.b_off = toff[inf.stripe][0] + (int64_t)inf.slot0 * toff[inf.stripe][2];
        q.b_ld = (int64_t)si.nslots * toff[inf.stripe][2];
        q.b_exp = toff[inf.stripe][1];
      } else {
        q.b_buf = SBUF_PSIC;
        q.b_off = psi_off[inf.prob][inf.E][2];
        q.b_ld = rup8(E.dL);
        q.b_exp = psi_off[inf.prob][inf.E][3];
      }
      q.K = inf.run * v.kbp;
      ch.sseg2.push_back(q);
    }
  }
  P->sb_elems[SBUF_T] = t_elems_max;
  P->sb_exps[SBUF_T] = t_exps_max;
  check_jobs(P->jobs_ops);
  check_jobs(P->jobs_psi);
  for (auto &ch : P->chunks) check_jobs(ch.tjobs);
  // the split kernels address a segment's slice lines with 32-bit byte
  // offsets from the slice base: rows * ld * 2 s bytes must stay below 2^32
  for (auto &ch : P->chunks)
    for (int st = 0; st < 6; st++) {
      const auto &tiles = st == 0 ? ch.tile1 : st == 1 ? ch.tile1m : st == 2 ? ch.tile1x
                        : st == 3 ? ch.tile2 : st == 4 ? ch.tile2m : ch.tile2x;
      const auto &ss = st < 3 ? ch.sseg1 : ch.sseg2;
      for (const Tile &t : tiles)
        for (int i = 0; i < t.nseg; i++) {
          const SegS &q = ss[t.seg0 + i];
          if (q.K > 0 && ((int64_t)t.m * q.a_ld * 2 * P->n_slices >= ((int64_t)1 << 32) ||
                          (int64_t)t.n * q.b_ld * 2 * P->n_slices >= ((int64_t)1 << 32)))
            throw std::length_error("split operand lines span 4 GiB or more");
        }
    }
}

}  // namespace

namespace {
int upload_split(dmrg_plan *P) {
  build_split(P);
  int rc;
  if ((rc = upload(P, P->jobs_ops, &P->d_jobs_ops)) || (rc = upload(P, P->jobs_psi, &P->d_jobs_psi))) return rc;
  for (auto &ch : P->chunks)
    if ((rc = upload(P, ch.sseg1, &ch.d_sseg1)) || (rc = upload(P, ch.sseg2, &ch.d_sseg2)) ||
        (rc = upload(P, ch.tjobs, &ch.d_tjobs)) || (rc = upload(P, ch.titems, &ch.d_titems)))
      return rc;
  for (int b = 0; b < N_SBUF; b++) {
    void *d = P->dalloc(sizeof(uint16_t) * std::max<int64_t>(1, P->sb_elems[b] * P->n_slices));
    if (d) P->plan_allocs.push_back(d);
    // exponent arrays carry WIDE_EDGE spare entries: the wide tiles read the
    // exponents of up to 128 lines past an output's last line (never stored)
    void *e = d ? P->dalloc(sizeof(int32_t) * (P->sb_exps[b] + WIDE_EDGE)) : nullptr;
    if (!d || !e) {
      set_error("device allocation failed for slice buffers");
      return DMRG_ENOMEM;
    }
    P->plan_allocs.push_back(e);
    P->sb.data[b] = (uint16_t *)d;
    P->sb.exps[b] = (int32_t *)e;
  }
  // operator slices: once per plan (the operators are constant during Davidson)
  launch_slices(P->d_jobs_ops, (int)P->jobs_ops.size(), P->n_slices, P->d_bases, nullptr, nullptr, P->sb,
                P->build_stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(P->build_stream));
  return DMRG_OK;
}
}  // namespace

namespace {

// Frees the tile lists, workspace and slices (not the problem-level data).
void release_plan(dmrg_plan *P) {
  P->wait_done();
  P->drop_graphs();
  for (void *a : P->plan_allocs) P->dfree(a);
  P->plan_allocs.clear();
  P->chunks.clear();
  P->dblocks.clear();
  P->dterms.clear();
  P->d_dblocks = nullptr;
  P->d_dterms = nullptr;
  P->d_work = nullptr;
  P->d_part = nullptr;
  P->d_counters = nullptr;
  P->work_elems = P->part_elems = 0;
  P->jobs_ops.clear();
  P->jobs_psi.clear();
  P->d_jobs_ops = P->d_jobs_psi = nullptr;
  P->sb = SliceBufs{};
  for (int b = 0; b < N_SBUF; b++) P->sb_elems[b] = P->sb_exps[b] = 0;
  P->stats.n_stage1 = P->stats.n_segments = 0;
}

// Kernel launches of one H.psi issued by enqueue (launchers skip empty lists).
int count_launches(const dmrg_plan *P) {
  const bool split = P->precision == DMRG_SPLIT_BF16;
  int n = P->psi_len > 0;
  if (split) n += !P->jobs_psi.empty();
  for (const Chunk &ch : P->chunks) {
    // every tile launch clears its queue counters first
    n += 2 * (!ch.tile1.empty() + !ch.tile2.empty() + !ch.tile1m.empty() + !ch.tile2m.empty() +
              !ch.tile1x.empty() + !ch.tile2x.empty()) +
         !ch.red2.empty();
    if (split) n += (ch.t_exps > 0) + !ch.titems.empty();
  }
  return n;
}

// Tile lists for the plan's current settings.
int replan(dmrg_plan *P) {
  release_plan(P);
  int rc = build_plan(P, P->budget, true);
  if (!rc && P->precision == DMRG_SPLIT_BF16) rc = upload_split(P);
  P->stats.launches = rc ? 0 : count_launches(P);
  return rc;
}

// The launch sequence of one H.psi.
int enqueue(dmrg_plan *p, const double *psi, double *hpsi, void *stream, bool prof);

int time_apply(dmrg_plan *P, const double *x, double *y, void *stream, double *ms) {
  hipStream_t s = (hipStream_t)stream;
  int rc = enqueue(P, x, y, stream, false);
  if (rc) return rc;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  for (int i = 0; i < 3 && !rc; i++) rc = enqueue(P, x, y, stream, false);
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float f = 0.0f;
  HIPCHK(hipEventElapsedTime(&f, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = f / 3.0;
  return rc;
}

// FNV-1a hash of what the tile lists depend on
uint64_t plan_hash(const dmrg_plan *P) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int i = 0; i < 8; i++) {
      h ^= (uint64_t)((v >> (8 * i)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  mix(P->precision);
  mix(P->n_slices);
  mix(P->xcd);
  mix(P->macro_min);
  mix(P->wide_min);
  mix(P->budget);
  for (const auto &pp : P->probs) {
    mix((int64_t)pp->T.blocks.size());
    for (const PsiBlock &b : pp->T.blocks) mix(((int64_t)b.dL << 32) | b.dR);
    mix((int64_t)pp->T.tasks.size());
    mix((int64_t)pp->T.rows.size());
  }
  return h;
}

std::mutex g_tune_mu;
// kpart, tile policy, workspace cap, work-group tile threshold, wide tile threshold
using TuneChoice = std::array<int64_t, 5>;
std::map<uint64_t, TuneChoice> g_tune_cache;

// one line per plan-shape hash: "<hash> <kpart> <tile_policy> <cap> <macro_min> <wide_min>"
bool read_tune_file(const std::string &path, uint64_t key, TuneChoice &out) {
  if (path.empty()) return false;
  FILE *f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  unsigned long long h;
  long long a, b, c, d, e;
  bool found = false;
  while (std::fscanf(f, "%llx %lld %lld %lld %lld %lld", &h, &a, &b, &c, &d, &e) == 6)
    if ((uint64_t)h == key) {   // the last line of a key wins
      out = {a, b, c, d, e};
      found = true;
    }
  std::fclose(f);
  return found;
}

void append_tune_file(const std::string &path, uint64_t key, const TuneChoice &c) {
  if (path.empty()) return;
  FILE *f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%016llx %lld %lld %lld %lld %lld\n", (unsigned long long)key, (long long)c[0], (long long)c[1],
               (long long)c[2], (long long)c[3], (long long)c[4]);
  std::fclose(f);
}

void apply_choice(dmrg_plan *P, const TuneChoice &c) {
  P->kpart = (int)c[0];
  P->tile_policy = (int)c[1];
  P->budget = c[2];
  P->macro_min = (int)c[3];
  P->wide_min = (int)c[4];
}

// Times candidate settings on the live plan and keeps the fastest (see
// DMRG_PLAN_AUTOTUNE): kpart x tile policy at the requested workspace cap,
// then (split plans) the work-group tile threshold, then smaller caps (more,
// smaller launches whose stripes stay in the last-level cache).  Choices are
// cached for the process and, with a tune_cache path, in that file.
int autotune(dmrg_plan *P, void *stream) {
  auto t0 = std::chrono::steady_clock::now();
  const uint64_t key = plan_hash(P);
  TuneChoice hit{};
  bool have = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      hit = it->second;
      have = true;
      P->tuned = 0;
    } else if (read_tune_file(P->tune_cache, key, hit)) {
      g_tune_cache[key] = hit;
      have = true;
      P->tuned = -1;
    }
  }
  if (have) {
    apply_choice(P, hit);
    int rc = replan(P);
    P->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
  }
  double *x = (double *)P->dalloc(sizeof(double) * std::max<int64_t>(P->psi_len, 1));
  double *y = x ? (double *)P->dalloc(sizeof(double) * std::max<int64_t>(P->psi_len, 1)) : nullptr;
  if (!x || !y) {
    P->dfree(x);
    set_error("device allocation failed in the autotuner");
    return DMRG_ENOMEM;
  }
  int rc = hipMemsetAsync(x, 0, sizeof(double) * std::max<int64_t>(P->psi_len, 1), (hipStream_t)stream) == hipSuccess
               ? DMRG_OK : DMRG_EHIP;
  const int64_t base = P->budget;
  double best = 1e300;
  TuneChoice bc{P->kpart, P->tile_policy, base, P->macro_min, P->wide_min};
  auto trial = [&](const TuneChoice &c) {
    if (rc) return;
    apply_choice(P, c);
    double ms = 0.0;
    rc = replan(P);
    if (!rc) rc = time_apply(P, x, y, stream, &ms);
    P->tuned++;
    if (!rc && ms < best) {
      best = ms;
      bc = c;
    }
  };
  const int64_t mm0 = P->macro_min, wm0 = P->wide_min;
  for (int kp : {1024, 2048, 4096})
    for (int pol : {0, 1}) trial({kp, pol, base, mm0, wm0});
  if (P->precision == DMRG_SPLIT_BF16) {
    const TuneChoice b0 = bc;
    for (int mm : {0, 32, 48, 96})
      if (mm != mm0) trial({b0[0], b0[1], base, mm, b0[4]});
    if (P->n_slices <= WIDE_MAX_SLICES) {
      const TuneChoice b2 = bc;
      for (int wm : {0, 48, 96, 192})
        if (wm != wm0) trial({b2[0], b2[1], base, b2[3], wm});
    }
  }
  {
    const TuneChoice b1 = bc;
    for (int64_t b : {(int64_t)512 << 20, (int64_t)192 << 20})
      if (b < base) trial({b1[0], b1[1], b, b1[3], b1[4]});
  }
  P->dfree(x);
  P->dfree(y);
  if (rc) return rc;
  apply_choice(P, bc);
  rc = replan(P);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = bc;
    append_tune_file(P->tune_cache, key, bc);
  }
  P->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

}  // namespace

extern "C" void dmrg_plan_free(dmrg_plan_t *p) {
  if (!p) return;
  p->wait_done();
  p->drop_graphs();
  for (void *a : p->plan_allocs) p->dfree(a);
  for (void *a : p->allocs) p->dfree(a);
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
  P->build_stream = (hipStream_t)stream;
  if (opts && (!opts->alloc_fn) != (!opts->free_fn)) {
    set_error("alloc_fn and free_fn must be given together");
    delete P;
    return DMRG_EINVAL;
  }
  if (opts) {
    P->alloc_fn = opts->alloc_fn;
    P->free_fn = opts->free_fn;
    P->alloc_ctx = opts->alloc_ctx;
    if (opts->tune_cache) P->tune_cache = opts->tune_cache;
  }
  try {
    P->precision = opts ? opts->precision : DMRG_FP64;
    P->n_slices = opts ? opts->n_slices : 0;
    if (P->precision != DMRG_FP64 && P->precision != DMRG_SPLIT_BF16) {
      set_error("unknown precision");
      dmrg_plan_free(P);
      return DMRG_EINVAL;
    }
    if (P->precision == DMRG_SPLIT_BF16 && (P->n_slices < 3 || P->n_slices > 7)) {
      set_error("split precision needs 3 <= n_slices <= 7");
      dmrg_plan_free(P);
      return DMRG_EINVAL;
    }
    int64_t budget = (opts && opts->workspace_bytes > 0) ? opts->workspace_bytes : DEFAULT_WORKSPACE;
    int64_t off = 0;
    for (int k = 0; k < n_probs; k++) {
      auto pp = std::make_unique<ProbPlan>();
      Error err{0, ""};
      if (!probs[k].ldata && probs[k].site_l > 0) { set_error("left operator data missing"); dmrg_plan_free(P); return DMRG_EINVAL; }
      auto tt0 = std::chrono::steady_clock::now();
      if (build_tasks_for_problem(probs[k], pp->L, pp->R, pp->T, err)) {
        set_error("problem " + std::to_string(k) + ": " + err.msg);
        dmrg_plan_free(P);
        return err.code;
      }
      P->stats.tasks_ms +=
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tt0).count();
      pp->psi_off = off;
      off += pp->T.size;
      pp->base_l = BASE_OPS + (int)P->bases_h.size();
      P->bases_h.push_back(probs[k].ldata);
      pp->base_r = BASE_OPS + (int)P->bases_h.size();
      P->bases_h.push_back(probs[k].rdata);
      pp->base_dress = BASE_OPS + (int)P->bases_h.size();
      if (pp->T.dress_len > 0) {
        void *d = P->dalloc(sizeof(double) * pp->T.dress_len);
        if (!d) {
          set_error("device allocation failed for dressed operators");
          dmrg_plan_free(P);
          return DMRG_ENOMEM;
        }
        P->allocs.push_back(d);
        pp->d_dress = (double *)d;
      }
      P->bases_h.push_back(pp->d_dress);
      // transposed copies (filled on the device by build_plan)
      double **tdst[3] = {&pp->d_lT, &pp->d_rT, &pp->d_dressT};
      const int64_t tlen[3] = {probs[k].ldata ? probs[k].ldata_len : 0, probs[k].rdata ? probs[k].rdata_len : 0,
                               pp->T.dress_len};
      int *tbase[3] = {&pp->base_lT, &pp->base_rT, &pp->base_dressT};
      for (int q = 0; q < 3; q++) {
        *tbase[q] = BASE_OPS + (int)P->bases_h.size();
        if (tlen[q] > 0) {
          void *d = P->dalloc(sizeof(double) * tlen[q]);
          if (!d) {
            set_error("device allocation failed for transposed operators");
            dmrg_plan_free(P);
            return DMRG_ENOMEM;
          }
          P->allocs.push_back(d);
          *tdst[q] = (double *)d;
        }
        P->bases_h.push_back(*tdst[q]);
      }
      P->stats.n_blocks += (int64_t)pp->T.blocks.size();
      P->stats.n_rows += (int64_t)pp->T.rows.size();
      for (auto &tk : pp->T.tasks) P->stats.n_tasks += (int64_t)pp->T.rows[tk.row].pos.size();
      P->probs.push_back(std::move(pp));
    }
    P->psi_len = off;
    P->stats.psi_len = off;
    P->flags = opts ? opts->flags : 0;
    P->xcd = (P->flags & DMRG_PLAN_XCD) ? 1 : 0;
    P->kpart = (opts && opts->kpart > 0) ? opts->kpart : KPART;
    P->tile_policy = opts ? opts->tile_policy : 0;
    P->macro_min = !opts || opts->macro_min == 0 ? MACRO_MIN : std::max(0, opts->macro_min);
    P->wide_min = !opts || opts->wide_min == 0 ? WIDE_MIN : std::max(0, opts->wide_min);
    P->budget = budget;
    if (P->kpart < 64 || P->kpart > (1 << 20) || P->tile_policy < 0 || P->tile_policy > 1) {
      set_error("kpart must be in [64, 2^20] and tile_policy 0 or 1");
      dmrg_plan_free(P);
      return DMRG_EINVAL;
    }
    auto tp0 = std::chrono::steady_clock::now();
    int rc = prepare_device(P);
    if (!rc) rc = (P->flags & DMRG_PLAN_AUTOTUNE) ? autotune(P, stream) : replan(P);
    P->stats.plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp0).count();
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

namespace {
// Scratch memory of one launch sequence: stripe workspace, partial tiles and
// (split plans) the stripe slices with their line exponents.
struct RunBufs {
  double *work, *part;
  SliceBufs sb;
  int32_t *counters;
};

int enqueue_with(dmrg_plan *p, const double *psi, double *hpsi, void *stream, bool prof, const RunBufs &B) {
  launch_zero(hpsi, p->psi_len, stream);
  const bool split = p->precision == DMRG_SPLIT_BF16;
  if (split)
    launch_slices(p->d_jobs_psi, (int)p->jobs_psi.size(), p->n_slices, p->d_bases, psi, B.work, B.sb, stream);
  size_t ev = p->ev_marks.empty() ? 0 : (size_t)p->ev_marks.back().second.second + 1;
  for (auto &ch : p->chunks) {
    for (int stage = 1; stage <= 2; stage++) {
      // stripe line exponents are maxima taken by the first stage's tiles;
      // the stripe slices follow it (both outside the stages' event windows)
      if (split && stage == 1) launch_fill_int(B.sb.exps[SBUF_T], ch.t_exps, INT_MIN, stream);
      if (split && stage == 2)
        launch_tslices(ch.d_tjobs, ch.d_titems, (int)ch.titems.size(), p->n_slices, B.work, B.sb, stream);
      // profiling: an event pair around each tile launch, marked 10 + stage
      // (work-group tiles), 20 + stage (wavefront tiles) or 30 + stage (wide
      // tiles) with its flops
      auto timed = [&](int code, double flops, auto &&launch) -> int {
        if (!prof) {
          launch();
          return DMRG_OK;
        }
        int rc = next_event(p, ev);
        if (rc) return rc;
        const int e0 = (int)ev;
        HIPCHK(hipEventRecord(p->ev_pool[ev++], (hipStream_t)stream));
        launch();
        if ((rc = next_event(p, ev))) return rc;
        HIPCHK(hipEventRecord(p->ev_pool[ev], (hipStream_t)stream));
        p->ev_marks.push_back({code, {e0, (int)ev}});
        p->ev_flops.push_back(flops);
        ev++;
        return DMRG_OK;
      };
      int rc = DMRG_OK;
      if (split) {
        // wide tiles, work-group tiles (the larger outputs), then the wavefront tiles
        const bool s1 = stage == 1;
        if (!(s1 ? ch.tile1x : ch.tile2x).empty())
          rc = timed(30 + stage, s1 ? ch.flops1x : ch.flops2x, [&] {
            launch_wide_split(stage, s1 ? ch.d_tile1x : ch.d_tile2x, s1 ? ch.d_seg1 : ch.d_seg2,
                              s1 ? ch.d_sseg1 : ch.d_sseg2, (int)(s1 ? ch.tile1x : ch.tile2x).size(),
                              s1 ? ch.q1x : ch.q2x, B.counters, p->n_slices, p->d_bases, psi, hpsi, B.work,
                              B.part, B.sb, stream);
          });
        if (!rc && !(s1 ? ch.tile1m : ch.tile2m).empty())
          rc = timed(10 + stage, s1 ? ch.flops1m : ch.flops2m, [&] {
            launch_macro_split(stage, s1 ? ch.d_tile1m : ch.d_tile2m, s1 ? ch.d_seg1 : ch.d_seg2,
                               s1 ? ch.d_sseg1 : ch.d_sseg2, (int)(s1 ? ch.tile1m : ch.tile2m).size(),
                               s1 ? ch.q1m : ch.q2m, B.counters, p->n_slices, p->d_bases, psi, hpsi, B.work,
                               B.part, B.sb, stream);
          });
        if (!rc && !(s1 ? ch.tile1 : ch.tile2).empty())
          rc = timed(20 + stage, s1 ? ch.flops1w : ch.flops2w, [&] {
            launch_tiles_split(stage, s1 ? ch.d_tile1 : ch.d_tile2, s1 ? ch.d_seg1 : ch.d_seg2,
                               s1 ? ch.d_sseg1 : ch.d_sseg2, (int)(s1 ? ch.tile1 : ch.tile2).size(),
                               s1 ? ch.q1 : ch.q2, B.counters, p->n_slices, p->d_bases, psi, hpsi, B.work,
                               B.part, B.sb, stream);
          });
      } else {
        const bool s1 = stage == 1;
        if (!(s1 ? ch.tile1 : ch.tile2).empty())
          rc = timed(20 + stage, s1 ? ch.flops1w : ch.flops2w, [&] {
            launch_tiles_f64(stage, s1 ? ch.d_tile1 : ch.d_tile2, s1 ? ch.d_seg1 : ch.d_seg2,
                             (int)(s1 ? ch.tile1 : ch.tile2).size(), s1 ? ch.q1 : ch.q2, B.counters, p->d_bases,
                             psi, hpsi, B.work, B.part, stream);
          });
      }
      if (rc) return rc;
    }
    launch_reduce(ch.d_red2, (int)ch.red2.size(), B.part, hpsi, stream);
  }
  HIPCHK(hipGetLastError());
  return DMRG_OK;
}

int enqueue(dmrg_plan *p, const double *psi, double *hpsi, void *stream, bool prof) {
  return enqueue_with(p, psi, hpsi, stream, prof, RunBufs{p->d_work, p->d_part, p->sb, p->d_counters});
}
}  // namespace

namespace dmrg {
void *plan_dalloc(dmrg_plan_t *p, size_t bytes) { return p->dalloc(bytes); }
void plan_dfree(dmrg_plan_t *p, void *ptr) { p->dfree(ptr); }

// Byte layout of the scratch memory of one H.psi (see dmrg_apply_H_static):
// stripe workspace, partial tiles, stripe slices, stripe exponents, each
// 256-byte aligned.  Returns the total.
int64_t plan_scratch_layout(const dmrg_plan_t *p, int64_t off[SCRATCH_REGIONS]) {
  auto up = [](int64_t x) { return (x + 255) / 256 * 256; };
  const bool split = p->precision == DMRG_SPLIT_BF16;
  int64_t o = 0;
  off[0] = o; o = up(o + 8 * std::max<int64_t>(p->work_elems, 1));
  off[1] = o; o = up(o + 8 * std::max<int64_t>(p->part_elems, 1));
  off[2] = o; if (split) o = up(o + 2 * std::max<int64_t>(p->sb_elems[SBUF_T], 1) * p->n_slices);
  off[3] = o; if (split) o = up(o + 4 * (p->sb_exps[SBUF_T] + WIDE_EDGE));   // spare entries: see upload_split
  off[4] = o; o = up(o + 4 * QUEUE_INTS);
  return o;
}

// One H.psi with the scratch memory at `base` (laid out by
// plan_scratch_layout); no allocation, no graph, no profiling events.
int enqueue_scratch(dmrg_plan_t *p, const double *psi, double *hpsi, void *stream, char *base) {
  int64_t off[SCRATCH_REGIONS];
  plan_scratch_layout(p, off);
  RunBufs B{(double *)(base + off[0]), (double *)(base + off[1]), p->sb, (int32_t *)(base + off[4])};
  if (p->precision == DMRG_SPLIT_BF16) {
    B.sb.data[SBUF_T] = (uint16_t *)(base + off[2]);
    B.sb.exps[SBUF_T] = (int32_t *)(base + off[3]);
  }
  int rc = enqueue_with(p, psi, hpsi, stream, false, B);
  return rc ? rc : p->mark_done(stream);
}
}  // namespace dmrg

extern "C" int dmrg_apply_H(dmrg_plan_t *p, const double *psi, double *hpsi, void *stream) {
  if (!p || !psi || !hpsi) { set_error("null argument"); return DMRG_EINVAL; }
  if (psi == hpsi) { set_error("psi and hpsi must not alias"); return DMRG_EINVAL; }
  if (!(p->flags & DMRG_PLAN_GRAPH) || p->profiling) {
    int rc = enqueue(p, psi, hpsi, stream, p->profiling != 0);
    return rc ? rc : p->mark_done(stream);
  }
  dmrg_plan::GraphEntry *ge = nullptr;
  for (auto &e : p->graphs)
    if (e.psi == psi && e.y == hpsi) ge = &e;
  if (!ge) {
    if (!p->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    if (p->graphs.size() >= 64) {
      (void)hipGraphExecDestroy(p->graphs.front().x);
      (void)hipGraphDestroy(p->graphs.front().g);
      p->graphs.erase(p->graphs.begin());
    }
    HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue(p, psi, hpsi, p->cap_stream, false);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) {
      set_error(std::string("HIP error: ") + hipGetErrorString(e) + " at graph capture");
      return DMRG_EHIP;
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      set_error(std::string("HIP error: ") + hipGetErrorString(e) + " at graph instantiation");
      return DMRG_EHIP;
    }
    p->graphs.push_back({psi, hpsi, g, x});
    ge = &p->graphs.back();
  }
  HIPCHK(hipGraphLaunch(ge->x, (hipStream_t)stream));
  return p->mark_done(stream);
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
  if (!p || !(stage == 1 || stage == 2 || ((stage / 10 >= 1 && stage / 10 <= 3) && (stage % 10 == 1 || stage % 10 == 2)))) {
    set_error("bad plan or stage");
    return DMRG_EINVAL;
  }
  int64_t n = 0;
  double ms = 0.0, fl = 0.0;
  for (size_t i = 0; i < p->ev_marks.size(); i++) {
    const int code = p->ev_marks[i].first;
    if (!(code == stage || (stage <= 2 && code % 10 == stage))) continue;
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
  return p->mark_done(stream);
}

extern "C" int dmrg_plan_stats(const dmrg_plan_t *p, dmrg_plan_stats_t *st) {
  if (!p || !st) { set_error("null argument"); return DMRG_EINVAL; }
  *st = p->stats;
  st->kpart = p->kpart;
  st->tile_policy = p->tile_policy;
  st->xcd = p->xcd;
  st->tuned = p->tuned;
  st->workspace_cap = p->budget;
  st->tune_ms = p->tune_ms;
  st->macro_min = p->precision == DMRG_SPLIT_BF16 ? p->macro_min : 0;
  st->wide_min = p->precision == DMRG_SPLIT_BF16 && p->n_slices <= WIDE_MAX_SLICES ? p->wide_min : 0;
  st->device_bytes = p->held;
  return DMRG_OK;
}

// ---------------------------------------------------------------------------
// Test-only: build the plan for one problem whose operator data are HOST
// arrays and execute its tile and segment lists on the CPU with the kernels'
// addressing (no GPU use).  Checks the plan layout without a device.
static void host_tiles(const std::vector<Tile> &tiles, const std::vector<Seg> &segs,
                       const std::vector<const double *> &bases, const double *psi, double *y,
                       double *work, double *part) {
  auto base = [&](int id) -> const double * {
    return id == BASE_PSI ? psi : id == BASE_Y ? y : id == BASE_WORK ? work : id == BASE_PART ? part
                                                                                               : bases[id - BASE_OPS];
  };
  auto Bel = [](const Seg &S, const double *B, int64_t k, int64_t n) {
    int64_t pk = k / S.b_kb, pn = n / S.b_nb;
    return B[pk * S.b_pk + (k - pk * S.b_kb) * S.b_k + pn * S.b_pn + (n - pn * S.b_nb) * S.b_n];
  };
  for (const Tile &T : tiles) {
    int tm = tile_rows(T.mb), tn = tile_cols(T.mb);
    int mt = std::min(tm, T.m - T.i0), nt = std::min(tn, T.n - T.j0);
    std::vector<double> acc((size_t)mt * nt, 0.0);
    for (int si = 0; si < T.nseg; si++) {
      const Seg &S = segs[T.seg0 + si];
      const double *B = base(S.b_base) + S.b_off;
      if (S.a_base < 0) {
        for (int j = 0; j < nt; j++)
          for (int i = 0; i < mt; i++) acc[i + (size_t)j * mt] += S.s * Bel(S, B, T.i0 + i, T.j0 + j);
        continue;
      }
      const double *A = base(S.a_base) + S.a_off;
      for (int j = 0; j < nt; j++)
        for (int i = 0; i < mt; i++) {
          double a = 0.0;
          for (int k = 0; k < S.K; k++) {
            int p = k / S.a_kb, kr = k - p * S.a_kb;
            a += S.s * A[(int64_t)p * S.a_p + (int64_t)(T.i0 + i) * S.a_i + (int64_t)kr * S.a_k] *
                 Bel(S, B, k, T.j0 + j);
          }
          acc[i + (size_t)j * mt] += a;
        }
    }
    double *C = const_cast<double *>(base(T.c_base)) + T.c_off;
    for (int j = 0; j < nt; j++)
      for (int i = 0; i < mt; i++) {
        double &c = T.rowmajor ? C[(int64_t)(T.ci0 + i) * T.ldc + (T.cj0 + j)]
                               : C[(int64_t)(T.ci0 + i) + (int64_t)(T.cj0 + j) * T.ldc];
        c = T.accumulate ? c + acc[i + (size_t)j * mt] : acc[i + (size_t)j * mt];
      }
  }
}

// host emulation of slice_kernel
static void host_slices(const std::vector<SliceJob> &jobs, int ns, const std::vector<const double *> &bases,
                        const double *psi, const double *work, std::vector<uint16_t> *sbd,
                        std::vector<int32_t> *sbe) {
  auto base = [&](int id) -> const double * {
    return id == BASE_PSI ? psi : id == BASE_WORK ? work : bases[id - BASE_OPS];
  };
  for (const SliceJob &J : jobs) {
    const double *src = base(J.src_base) + J.src_off;
    int64_t len = (int64_t)J.npos * J.kbp;
    for (int rho = 0; rho < J.nrho; rho++) {
      const double *line = src + (int64_t)rho * J.s_rho;
      double m = 0.0;
      for (int p = 0; p < J.npos; p++)
        for (int kk = 0; kk < J.kb; kk++) m = std::max(m, std::fabs(line[(int64_t)p * J.s_pos + (int64_t)kk * J.s_k]));
      int e = 0;
      if (m > 0.0) {
        int ex;
        double mant = std::frexp(m, &ex);
        e = (mant == 0.5) ? ex - 1 : ex;
      }
      sbe[J.dst_buf][J.exp_off + rho] = e;
      for (int64_t idx = 0; idx < len; idx++) {
        int p = (int)(idx / J.kbp), kk = (int)(idx - (int64_t)p * J.kbp);
        double x = kk < J.kb ? line[(int64_t)p * J.s_pos + (int64_t)kk * J.s_k] : 0.0;
        double yv = std::ldexp(x, -e);
        for (int t = 0; t < ns; t++) {
          double a = std::nearbyint(yv * 256.0);
          yv = yv * 256.0 - a;
          float af = (float)std::ldexp(a, -SLICE_BITS * t);   // digit t at its weight 2^(-8t)
          uint32_t bits;
          std::memcpy(&bits, &af, 4);
          sbd[J.dst_buf][slice_index(J.dst_off + (int64_t)rho * len + idx, t, ns)] = (uint16_t)(bits >> 16);
        }
      }
    }
  }
}

static double bf16v(uint16_t b) {
  uint32_t bits = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &bits, 4);
  return (double)f;
}

// host emulation of the split work items (same fold points as the kernels)
static void host_tiles_split(const std::vector<Tile> &tiles, const std::vector<Seg> &segs,
                             const std::vector<SegS> &ssegs, int ns, const std::vector<const double *> &bases,
                             const double *psi, double *y, double *work, double *part,
                             std::vector<uint16_t> *sbd, std::vector<int32_t> *sbe) {
  auto base = [&](int id) -> const double * {
    return id == BASE_PSI ? psi : id == BASE_Y ? y : id == BASE_WORK ? work : id == BASE_PART ? part
                                                                                               : bases[id - BASE_OPS];
  };
  for (const Tile &T : tiles) {
    int tm = tile_rows(T.mb), tn = tile_cols(T.mb);
    int mt = std::min(tm, T.m - T.i0), nt = std::min(tn, T.n - T.j0);
    std::vector<double> acc((size_t)mt * nt, 0.0);
    for (int si = 0; si < T.nseg; si++) {
      const Seg &S = segs[T.seg0 + si];
      const SegS &Q = ssegs[T.seg0 + si];
      if (Q.K == 0) {
        const double *B = base(S.b_base) + S.b_off;
        for (int j = 0; j < nt; j++)
          for (int i = 0; i < mt; i++) {
            int64_t k = T.i0 + i, n = T.j0 + j;
            int64_t pk = k / S.b_kb, pn = n / S.b_nb;
            acc[i + (size_t)j * mt] +=
                S.s * B[pk * S.b_pk + (k - pk * S.b_kb) * S.b_k + pn * S.b_pn + (n - pn * S.b_nb) * S.b_n];
          }
        continue;
      }
      const uint16_t *A = sbd[Q.a_buf].data(), *B = sbd[Q.b_buf].data();   // slices interleaved
      const int32_t *ea = sbe[Q.a_buf].data() + Q.a_exp;
      const int32_t *eb = sbe[Q.b_buf].data() + Q.b_exp;
      for (int j = 0; j < nt; j++)
        for (int i = 0; i < mt; i++) {
          const int64_t ar = Q.a_off + (int64_t)(T.i0 + i) * Q.a_ld;   // line starts (unsliced layout)
          const int64_t bc = Q.b_off + (int64_t)(T.j0 + j) * Q.b_ld;
          double tot = 0.0;
          for (int k0 = 0; k0 < Q.K; k0 += split_fold_k(ns)) {
            double x = 0.0;
            for (int d = 0; d < ns; d++) {
              double qd = 0.0;
              for (int t = 0; t <= d; t++)
                for (int k = k0; k < std::min(Q.K, k0 + split_fold_k(ns)); k++)
                  qd += bf16v(A[slice_index(ar + k, t, ns)]) * bf16v(B[slice_index(bc + k, d - t, ns)]);
              x += std::ldexp(qd, -2 * SLICE_BITS);   // slices carry their digit weights
            }
            tot += S.s * std::ldexp(x, ea[T.i0 + i] + eb[T.j0 + j]);
          }
          acc[i + (size_t)j * mt] += tot;
        }
    }
    double *C = const_cast<double *>(base(T.c_base)) + T.c_off;
    for (int j = 0; j < nt; j++)
      for (int i = 0; i < mt; i++) {
        double &c = T.rowmajor ? C[(int64_t)(T.ci0 + i) * T.ldc + (T.cj0 + j)]
                               : C[(int64_t)(T.ci0 + i) + (int64_t)(T.cj0 + j) * T.ldc];
        c = T.accumulate ? c + acc[i + (size_t)j * mt] : acc[i + (size_t)j * mt];
      }
  }
}

static void host_reduce(const std::vector<Reduce> &red, const double *part, double *y) {
  for (const Reduce &R : red) {
    int mt = std::min(R.tm, R.m - R.i0), nt = std::min(R.tn, R.n - R.j0);
    for (int j = 0; j < nt; j++)
      for (int i = 0; i < mt; i++) {
        double v = 0.0;
        for (int p = 0; p < R.nparts; p++)
          v += part[R.part_off + (int64_t)p * R.tm * R.tn + i + (int64_t)j * R.tm];
        y[R.y_off + (int64_t)(R.i0 + i) + (int64_t)(R.j0 + j) * R.ldc] += v;
      }
  }
}

extern "C" int dmrg_debug_plan_host_apply(const dmrg_problem_t *prob, const double *psi, double *y,
                                          const dmrg_plan_opts_t *opts, dmrg_plan_stats_t *st) {
  int64_t workspace_bytes = opts ? opts->workspace_bytes : 0;
  dmrg_plan *P = new dmrg_plan();
  std::memset(&P->stats, 0, sizeof(P->stats));
  P->precision = opts ? opts->precision : DMRG_FP64;
  P->n_slices = opts ? opts->n_slices : 0;
  P->kpart = (opts && opts->kpart > 0) ? opts->kpart : KPART;
  P->tile_policy = opts ? opts->tile_policy : 0;
  P->macro_min = !opts || opts->macro_min == 0 ? MACRO_MIN : std::max(0, opts->macro_min);
  P->wide_min = !opts || opts->wide_min == 0 ? WIDE_MIN : std::max(0, opts->wide_min);
  auto pp = std::make_unique<ProbPlan>();
  Error err{0, ""};
  auto tt0 = std::chrono::steady_clock::now();
  if (build_tasks_for_problem(*prob, pp->L, pp->R, pp->T, err)) {
    set_error(err.msg);
    delete P;
    return err.code;
  }
  P->stats.tasks_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tt0).count();
  pp->base_l = BASE_OPS;
  pp->base_r = BASE_OPS + 1;
  pp->base_dress = BASE_OPS + 2;
  pp->base_lT = BASE_OPS + 3;
  pp->base_rT = BASE_OPS + 4;
  pp->base_dressT = BASE_OPS + 5;
  dress_on_host(pp->T, pp->R, pp->h_dress);
  if (prob->ldata) transpose_on_host(trans_jobs(pp->L), prob->ldata, prob->ldata_len, pp->h_lT);
  if (prob->rdata) transpose_on_host(trans_jobs(pp->R), prob->rdata, prob->rdata_len, pp->h_rT);
  if (!pp->h_dress.empty())
    transpose_on_host(trans_jobs(pp->T), pp->h_dress.data(), (int64_t)pp->h_dress.size(), pp->h_dressT);
  P->bases_h = {prob->ldata, prob->rdata, pp->h_dress.data(), pp->h_lT.data(), pp->h_rT.data(),
                pp->h_dressT.data()};
  int64_t n = pp->T.size;
  P->stats.psi_len = n;
  P->stats.n_blocks = (int64_t)pp->T.blocks.size();
  P->stats.n_rows = (int64_t)pp->T.rows.size();
  for (auto &tk : pp->T.tasks) P->stats.n_tasks += (int64_t)pp->T.rows[tk.row].pos.size();
  P->probs.push_back(std::move(pp));
  P->psi_len = n;
  auto tp0 = std::chrono::steady_clock::now();
  int rc = build_plan(P, workspace_bytes > 0 ? workspace_bytes : DEFAULT_WORKSPACE, false);
  if (rc) { delete P; return rc; }
  P->stats.plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp0).count();
  for (auto &ch : P->chunks) {
    P->stats.n_stage1 += (int64_t)ch.seg1.size();
    P->stats.n_segments += (int64_t)ch.seg2.size();
  }
  if (st) *st = P->stats;
  if (!psi || !y) { delete P; return DMRG_OK; }
  std::vector<double> work((size_t)std::max<int64_t>(P->work_elems, 1), 0.0);
  std::vector<double> part((size_t)std::max<int64_t>(P->part_elems, 1), 0.0);
  std::memset(y, 0, sizeof(double) * n);
  if (P->precision == DMRG_SPLIT_BF16) {
    try {
      build_split(P);
    } catch (const std::exception &e) {
      set_error(std::string("exception: ") + e.what());
      delete P;
      return DMRG_EINVAL;
    }
    int ns = P->n_slices;
    for (int b = 0; b < N_SBUF; b++) {
      P->h_sb[b].assign((size_t)std::max<int64_t>(1, P->sb_elems[b] * ns), 0);
      P->h_se[b].assign((size_t)std::max<int64_t>(1, P->sb_exps[b]), 0);
    }
    host_slices(P->jobs_ops, ns, P->bases_h, psi, work.data(), P->h_sb, P->h_se);
    host_slices(P->jobs_psi, ns, P->bases_h, psi, work.data(), P->h_sb, P->h_se);
    for (auto &ch : P->chunks) {
      host_tiles_split(ch.tile1m, ch.seg1, ch.sseg1, ns, P->bases_h, psi, y, work.data(), part.data(), P->h_sb,
                       P->h_se);
      host_tiles_split(ch.tile1x, ch.seg1, ch.sseg1, ns, P->bases_h, psi, y, work.data(), part.data(), P->h_sb,
                       P->h_se);
      host_tiles_split(ch.tile1, ch.seg1, ch.sseg1, ns, P->bases_h, psi, y, work.data(), part.data(), P->h_sb,
                       P->h_se);
      host_slices(ch.tjobs, ns, P->bases_h, psi, work.data(), P->h_sb, P->h_se);
      host_tiles_split(ch.tile2m, ch.seg2, ch.sseg2, ns, P->bases_h, psi, y, work.data(), part.data(), P->h_sb,
                       P->h_se);
      host_tiles_split(ch.tile2x, ch.seg2, ch.sseg2, ns, P->bases_h, psi, y, work.data(), part.data(), P->h_sb,
                       P->h_se);
      host_tiles_split(ch.tile2, ch.seg2, ch.sseg2, ns, P->bases_h, psi, y, work.data(), part.data(), P->h_sb,
                       P->h_se);
      host_reduce(ch.red2, part.data(), y);
    }
    delete P;
    return DMRG_OK;
  }
  for (auto &ch : P->chunks) {
    host_tiles(ch.tile1, ch.seg1, P->bases_h, psi, y, work.data(), part.data());
    host_tiles(ch.tile2, ch.seg2, P->bases_h, psi, y, work.data(), part.data());
    host_reduce(ch.red2, part.data(), y);
  }
  delete P;
  return DMRG_OK;
}

// Test-only: per-tile work of one stage of the plan built for `prob` (host
// operator data): rows of (m, n, number of segments, summed K).
extern "C" int64_t dmrg_debug_plan_tiles(const dmrg_problem_t *prob, const dmrg_plan_opts_t *opts, int32_t stage,
                                         int64_t *out, int64_t cap) {
  dmrg_plan *P = new dmrg_plan();
  std::memset(&P->stats, 0, sizeof(P->stats));
  P->precision = opts ? opts->precision : DMRG_FP64;
  P->n_slices = opts ? opts->n_slices : 0;
  P->kpart = (opts && opts->kpart > 0) ? opts->kpart : KPART;
  P->tile_policy = opts ? opts->tile_policy : 0;
  P->macro_min = !opts || opts->macro_min == 0 ? MACRO_MIN : std::max(0, opts->macro_min);
  P->wide_min = !opts || opts->wide_min == 0 ? WIDE_MIN : std::max(0, opts->wide_min);
  auto pp = std::make_unique<ProbPlan>();
  Error err{0, ""};
  if (build_tasks_for_problem(*prob, pp->L, pp->R, pp->T, err)) { set_error(err.msg); delete P; return err.code; }
  pp->base_l = BASE_OPS; pp->base_r = BASE_OPS + 1; pp->base_dress = BASE_OPS + 2;
  P->bases_h = {prob->ldata, prob->rdata, nullptr};
  P->psi_len = pp->T.size;
  P->probs.push_back(std::move(pp));
  int rc = build_plan(P, DEFAULT_WORKSPACE, false);
  if (rc) { delete P; return rc; }
  int64_t n = 0;
  for (auto &ch : P->chunks) {
    std::vector<Tile> tiles = stage == 1 ? ch.tile1x : ch.tile2x;
    for (const Tile &t : stage == 1 ? ch.tile1m : ch.tile2m) tiles.push_back(t);
    for (const Tile &t : stage == 1 ? ch.tile1 : ch.tile2) tiles.push_back(t);
    const auto &segs = stage == 1 ? ch.seg1 : ch.seg2;
    for (const Tile &t : tiles) {
      int64_t sk = 0;
      for (int i = 0; i < t.nseg; i++) sk += segs[t.seg0 + i].a_base < 0 ? 0 : segs[t.seg0 + i].K;
      if (out && n < cap) {
        int64_t *o = out + 7 * n;
        o[0] = std::min(tile_rows(t.mb), t.m - t.i0);
        o[1] = std::min(tile_cols(t.mb), t.n - t.j0);
        o[2] = t.nseg;
        o[3] = sk;
        o[4] = t.m;
        o[5] = t.n;
        o[6] = t.mb;
      }
      n++;
    }
  }
  delete P;
  return n;
}
