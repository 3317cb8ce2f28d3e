// Two-site sweeps on the device (Sec. II: two-site DMRG; Sec. I: the
// Davidson solve and the renormalization of the block operators are the two
// parts of every step).  At every bond the two-site problem of the current
// blocks is planned (dmrg_build_tasks) and solved (dmrg_davidson); the
// wavefunction is cut to at most D multiplets of the growing block and its
// site (dmrg_truncate) and that block is renormalized in the kept basis
// (dmrg_renorm_*) into the block of the next bond.  Grown blocks stay in
// device memory from step to step; only their sector and record tables live
// on the host.
//  - left to right: the left block grows; it is kept in the all-pairs form
//    (P and Q over every outside pair) that its renormalization needs, and
//    its H.psi form (the pairs that touch the two sites) is cut from the
//    all-pairs records by device copies of the selected positions;
//  - right to left: the right block grows; the caller's left blocks are in
//    the H.psi form or in the all-pairs form (cut the same way), so that the
//    left blocks a left-to-right sweep returns can be passed straight in.
// With an output table, every grown block is handed to the caller (host
// tables from malloc, device data from hipMalloc; dmrg_block_release).
#include <hip/hip_runtime.h>
#include "common.hpp"
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace dmrg;

namespace {

// a grown block: host tables, device data (owned unless it is the caller's)
struct OwnedBlock {
  std::vector<dmrg_sector_t> sec;
  std::vector<dmrg_oprec_t> rec;
  double *data = nullptr;
  int64_t len = 0;
  bool owned = false;
  void borrow(const dmrg_block_t &b) {
    sec.assign(b.sec, b.sec + b.n_sec);
    rec.assign(b.rec, b.rec + b.n_rec);
    data = const_cast<double *>(b.data);
    len = b.data_len;
    owned = false;
  }
  void release() {
    if (owned && data) (void)hipFree(data);
    data = nullptr;
    owned = false;
  }
};

// label lists of the left block's P and Q at bond p: every outside pair
// (all-pairs form) or the pairs with an index at p or p + 1 (H.psi form);
// x <= y lexicographic, x < y for P1
std::vector<std::array<int, 2>> pq_labels(int fam, int p, int n, bool all) {
  std::vector<std::array<int, 2>> res;
  for (int x = p; x < n; x++)
    for (int y = x + (fam == F_P1 ? 1 : 0); y < n; y++) {
      if (!all && x >= p + 2 && y >= p + 2) continue;
      res.push_back({x, y});
    }
  return res;
}

bool is_pq(int f) { return f == F_P0 || f == F_P1 || f == F_Q0 || f == F_Q1; }

// SplitMix64 (Steele, Lea & Flood 2014) and Box-Muller normals for the seeded
// Davidson start vectors
uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double uniform01(uint64_t &s) { return ((splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

bool valid_block(const dmrg_block_t *b) {
  return b && b->n_sec >= 0 && b->n_rec >= 0 && (b->n_sec == 0 || b->sec) && (b->n_rec == 0 || b->rec);
}

// The H.psi form of a left block at bond p: records and the positions to
// copy.  P and Q records in the all-pairs form are cut to the pairs that
// touch the sites; records already in the H.psi form pass (unless
// require_all); the other records pass whole.
struct Copy { int64_t dst, src, n; };
int hpsi_form(const std::vector<dmrg_sector_t> &sec, const dmrg_oprec_t *rec, int64_t n_rec, int64_t len, int p,
              int n_orb, bool require_all, std::vector<dmrg_oprec_t> &crec, std::vector<Copy> &copies,
              int64_t &clen) {
  crec.clear();
  copies.clear();
  clen = 0;
  for (int64_t k = 0; k < n_rec; k++) {
    const dmrg_oprec_t &r = rec[k];
    if (r.row_sec < 0 || r.row_sec >= (int)sec.size() || r.col_sec < 0 || r.col_sec >= (int)sec.size()) {
      set_error("left block record with a bad sector");
      return DMRG_EINVAL;
    }
    const int64_t bs = (int64_t)sec[r.row_sec].dim * sec[r.col_sec].dim;
    if (r.npos < 0 || r.off < 0 || r.off + (int64_t)r.npos * bs > len) {
      set_error("left block record outside its data");
      return DMRG_EINVAL;
    }
    dmrg_oprec_t c = r;
    c.off = clen;
    if (is_pq(r.fam)) {
      auto all = pq_labels(r.fam, p, n_orb, true), want = pq_labels(r.fam, p, n_orb, false);
      if ((int)all.size() == r.npos) {
        c.npos = (int32_t)want.size();
        size_t j = 0;
        for (size_t i = 0; i < all.size() && j < want.size(); i++)
          if (all[i] == want[j]) {
            copies.push_back({clen + (int64_t)j * bs, r.off + (int64_t)i * bs, bs});
            j++;
          }
      } else if (!require_all && (int)want.size() == r.npos) {
        copies.push_back({clen, r.off, (int64_t)r.npos * bs});
      } else {
        set_error(require_all ? "left block P/Q records are not in the all-pairs form"
                              : "left block P/Q records are in neither the all-pairs nor the H.psi form");
        return DMRG_EINVAL;
      }
    } else {
      copies.push_back({clen, r.off, (int64_t)r.npos * bs});
    }
    if (c.npos == 0) continue;
    clen += (int64_t)c.npos * bs;
    crec.push_back(c);
  }
  return DMRG_OK;
}

// the per-bond resources of a sweep and its two steps
struct Sweep {
  hipStream_t hs;
  void *stream;
  dmrg_plan_t *plan = nullptr;
  dmrg_renorm_t *ren = nullptr;
  double *psi = nullptr, *u = nullptr, *cat = nullptr, *out = nullptr;
  OwnedBlock grown;   // the block that the sweep grows
  dmrg_block_t *outs = nullptr;   // caller's table of grown blocks, or NULL
  int n_out = 0;                  // entries filled so far

  explicit Sweep(void *s, dmrg_block_t *o) : hs((hipStream_t)s), stream(s), outs(o) {}
  void free_bond() {
    (void)hipStreamSynchronize(hs);
    if (plan) dmrg_plan_free(plan);
    if (ren) dmrg_renorm_free(ren);
    void *ptrs[] = {psi, u, cat, out};
    for (void *q : ptrs)
      if (q) (void)hipFree(q);
    plan = nullptr;
    ren = nullptr;
    psi = u = cat = out = nullptr;
  }
  int fail(int rc) {
    std::string msg = dmrg_last_error();
    free_bond();
    grown.release();
    for (int i = 0; i < n_out; i++) dmrg_block_release(&outs[i]);
    set_error(msg);
    return rc;
  }

  // the grown block goes to the caller's table (entry i); the sweep keeps
  // reading it until the next cut but no longer frees it
  int hand_out(int i) {
    if (!outs) return DMRG_OK;
    dmrg_block_t &b = outs[i];
    auto *sec = (dmrg_sector_t *)std::malloc(sizeof(dmrg_sector_t) * std::max<size_t>(grown.sec.size(), 1));
    auto *rec = (dmrg_oprec_t *)std::malloc(sizeof(dmrg_oprec_t) * std::max<size_t>(grown.rec.size(), 1));
    if (!sec || !rec) {
      std::free(sec);
      std::free(rec);
      set_error("out of host memory");
      return DMRG_ENOMEM;
    }
    std::copy(grown.sec.begin(), grown.sec.end(), sec);
    std::copy(grown.rec.begin(), grown.rec.end(), rec);
    b = dmrg_block_t{(int32_t)grown.sec.size(), 0, sec, (int64_t)grown.rec.size(), rec, grown.data, grown.len};
    grown.owned = false;
    n_out = i + 1;
    return DMRG_OK;
  }

  // Davidson on the problem `pr` from a seeded start vector
  int solve(const dmrg_problem_t &pr, const dmrg_plan_opts_t *popts, const dmrg_dav_opts_t *dav, uint64_t seed,
            int p, dmrg_sweep_step_t &S) {
    if (int rc = dmrg_build_tasks(&pr, 1, popts, stream, &plan)) return rc;
    int64_t off = 0, n = 0;
    dmrg_plan_stats_t pst{};
    if (int rc = dmrg_psi_layout(plan, 0, &off, &n)) return rc;
    if (int rc = dmrg_plan_stats(plan, &pst)) return rc;
    if (off < 0 || n < 1 || off + n > pst.psi_len) {
      set_error("unexpected wavefunction layout");
      return DMRG_EINVAL;
    }
    std::vector<double> x((size_t)pst.psi_len, 0.0);
    uint64_t st = seed + (uint64_t)p * 0x100000001ull;
    for (int64_t i = 0; i < n; i += 2) {
      const double r1 = std::sqrt(-2.0 * std::log(uniform01(st))), t = 6.283185307179586 * uniform01(st);
      x[off + i] = r1 * std::cos(t);
      if (i + 1 < n) x[off + i + 1] = r1 * std::sin(t);
    }
    double nrm = 0.0;
    for (double v : x) nrm += v * v;
    for (double &v : x) v /= std::sqrt(nrm);
    if (hipMalloc(&psi, sizeof(double) * pst.psi_len) != hipSuccess ||
        hipMemcpyAsync(psi, x.data(), sizeof(double) * pst.psi_len, hipMemcpyHostToDevice, hs) != hipSuccess ||
        hipStreamSynchronize(hs) != hipSuccess) {
      set_error("uploading the start vector failed");
      return DMRG_EHIP;
    }
    double e = 0.0;
    dmrg_dav_stats_t ds{};
    if (int rc = dmrg_davidson(plan, psi, &e, dav, &ds, stream)) return rc;
    S.energy = e;
    S.iters = ds.iters;
    S.kept = 0;
    S.kept_weight = 1.0;
    S.pad = 0;
    return DMRG_OK;
  }

  // truncation of psi (problem pt) and renormalization of the grown block
  // (problem pr, the same bond) into the grown block of the next bond
  int cut(const dmrg_problem_t &pt, const dmrg_problem_t &pr, int32_t flags, int32_t max_kept,
          dmrg_sweep_step_t &S) {
    const int32_t tflags = flags & DMRG_RENORM_RIGHT;
    int32_t nk = 0;
    int64_t ul = 0;
    double w[2] = {0.0, 0.0};
    if (int rc = dmrg_truncate(&pt, tflags, psi, max_kept, 1e-14, nullptr, 0, &nk, nullptr, 0, &ul, w, stream))
      return rc;
    std::vector<dmrg_rkeep_t> keep((size_t)std::max(nk, 1));
    if (hipMalloc(&u, sizeof(double) * std::max<int64_t>(ul, 1)) != hipSuccess) {
      set_error("hipMalloc failed");
      return DMRG_ENOMEM;
    }
    if (int rc = dmrg_truncate(&pt, tflags, psi, max_kept, 1e-14, keep.data(), nk, &nk, u, ul, &ul, w, stream))
      return rc;
    S.kept = 0;
    for (int i = 0; i < nk; i++) S.kept += keep[i].kept;
    S.kept_weight = w[1] > 0.0 ? w[0] / w[1] : 0.0;
    if (int rc = dmrg_renorm_create(&pr, keep.data(), nk, 0, flags, ul, &ren)) return rc;
    int64_t nrec = 0, olen = 0;
    if (int rc = dmrg_renorm_records(ren, nullptr, 0, &nrec, &olen)) return rc;
    std::vector<dmrg_oprec_t> orec((size_t)std::max<int64_t>(nrec, 1));
    if (int rc = dmrg_renorm_records(ren, orec.data(), nrec, &nrec, &olen)) return rc;
    if (hipMalloc(&out, sizeof(double) * std::max<int64_t>(olen, 1)) != hipSuccess) {
      set_error("hipMalloc failed");
      return DMRG_ENOMEM;
    }
    if (int rc = dmrg_renorm_apply(ren, u, out, stream)) return rc;
    if (hipStreamSynchronize(hs) != hipSuccess) {
      set_error("renormalization failed");
      return DMRG_EHIP;
    }
    grown.release();
    grown.sec.clear();
    for (int i = 0; i < nk; i++) grown.sec.push_back(dmrg_sector_t{keep[i].n, keep[i].two_s, keep[i].kept});
    grown.rec.assign(orec.begin(), orec.begin() + nrec);
    grown.data = out;
    grown.len = olen;
    grown.owned = true;
    out = nullptr;
    return DMRG_OK;
  }
};

dmrg_problem_t make_problem(int32_t n_orb, int32_t n_elec, int32_t two_s, const double *h1, const double *eri,
                            int p, const std::vector<dmrg_sector_t> &lsec, const dmrg_oprec_t *lrec, int64_t n_lrec,
                            const double *ldata, int64_t ldata_len, const dmrg_block_t &R) {
  dmrg_problem_t pr{};
  pr.n_orb = n_orb;
  pr.n_elec = n_elec;
  pr.two_s = two_s;
  pr.site_l = p;
  pr.h1 = h1;
  pr.eri = eri;
  pr.n_lsec = (int32_t)lsec.size();
  pr.lsec = lsec.data();
  pr.n_rsec = R.n_sec;
  pr.rsec = R.sec;
  pr.n_lrec = n_lrec;
  pr.lrec = lrec;
  pr.n_rrec = R.n_rec;
  pr.rrec = R.rec;
  pr.ldata = ldata;
  pr.ldata_len = ldata_len;
  pr.rdata = R.data;
  pr.rdata_len = R.data_len;
  return pr;
}

dmrg_block_t view(const OwnedBlock &b) {
  return dmrg_block_t{(int32_t)b.sec.size(), 0, b.sec.data(), (int64_t)b.rec.size(), b.rec.data(), b.data, b.len};
}

}  // namespace

extern "C" int dmrg_sweep_left_to_right(int32_t n_orb, int32_t n_elec, int32_t two_s, const double *h1,
                                        const double *eri, int32_t bond0, const dmrg_block_t *left,
                                        const dmrg_block_t *rights, int32_t max_kept, const dmrg_plan_opts_t *plan_opts,
                                        const dmrg_dav_opts_t *dav, uint64_t seed, dmrg_sweep_step_t *steps,
                                        dmrg_block_t *grown_out,
                                        void *stream) {
  if (!h1 || !eri || !valid_block(left) || !rights || !steps || bond0 < 1 || bond0 > n_orb - 2 || max_kept < 1) {
    set_error("bad sweep arguments (1 <= bond0 <= n_orb - 2, max_kept >= 1)");
    return DMRG_EINVAL;
  }
  for (int p = bond0; p <= n_orb - 2; p++)
    if (!valid_block(&rights[p - bond0])) {
      set_error("bad right block table");
      return DMRG_EINVAL;
    }
  if (grown_out)
    for (int i = 0; i <= n_orb - 2 - bond0; i++) grown_out[i] = dmrg_block_t{0, 0, nullptr, 0, nullptr, nullptr, 0};
  Sweep W(stream, grown_out);
  OwnedBlock &L = W.grown;
  L.borrow(*left);
  for (int p = bond0; p <= n_orb - 2; p++) {
    const dmrg_block_t &Rb = rights[p - bond0];
    // H.psi form of the left block: P and Q positions of the pairs at the sites
    std::vector<dmrg_oprec_t> crec;
    std::vector<Copy> copies;
    int64_t clen = 0;
    if (int rc = hpsi_form(L.sec, L.rec.data(), (int64_t)L.rec.size(), L.len, p, n_orb, true, crec, copies, clen))
      return W.fail(rc);
    if (hipMalloc(&W.cat, sizeof(double) * std::max<int64_t>(clen, 1)) != hipSuccess) {
      set_error("hipMalloc failed");
      return W.fail(DMRG_ENOMEM);
    }
    for (const Copy &c : copies)
      if (c.n > 0 &&
          hipMemcpyAsync(W.cat + c.dst, L.data + c.src, sizeof(double) * c.n, hipMemcpyDeviceToDevice, W.hs) !=
              hipSuccess) {
        set_error("copying the left block failed");
        return W.fail(DMRG_EHIP);
      }
    const dmrg_problem_t pr =
        make_problem(n_orb, n_elec, two_s, h1, eri, p, L.sec, crec.data(), (int64_t)crec.size(), W.cat, clen, Rb);
    dmrg_sweep_step_t &S = steps[p - bond0];
    S.bond = p;
    if (int rc = W.solve(pr, plan_opts, dav, seed, p, S)) return W.fail(rc);
    if (p == n_orb - 2) break;
    // truncation (H.psi form) and renormalization of the all-pairs block
    const dmrg_problem_t pa = make_problem(n_orb, n_elec, two_s, h1, eri, p, L.sec, L.rec.data(),
                                           (int64_t)L.rec.size(), L.data, L.len, Rb);
    if (int rc = W.cut(pr, pa, DMRG_RENORM_ALL_PAIRS, max_kept, S)) return W.fail(rc);
    if (int rc = W.hand_out(p - bond0)) return W.fail(rc);
    W.free_bond();
  }
  W.free_bond();
  L.release();
  return DMRG_OK;
}

extern "C" int dmrg_sweep_right_to_left(int32_t n_orb, int32_t n_elec, int32_t two_s, const double *h1,
                                        const double *eri, int32_t bond0, const dmrg_block_t *lefts,
                                        const dmrg_block_t *right, int32_t max_kept, const dmrg_plan_opts_t *plan_opts,
                                        const dmrg_dav_opts_t *dav, uint64_t seed, dmrg_sweep_step_t *steps,
                                        dmrg_block_t *grown_out,
                                        void *stream) {
  if (!h1 || !eri || !lefts || !valid_block(right) || !steps || bond0 < 0 || bond0 > n_orb - 3 || max_kept < 1) {
    set_error("bad sweep arguments (0 <= bond0 <= n_orb - 3, max_kept >= 1)");
    return DMRG_EINVAL;
  }
  for (int p = 0; p <= bond0; p++)
    if (!valid_block(&lefts[p])) {
      set_error("bad left block table");
      return DMRG_EINVAL;
    }
  if (grown_out)
    for (int i = 0; i <= bond0; i++) grown_out[i] = dmrg_block_t{0, 0, nullptr, 0, nullptr, nullptr, 0};
  Sweep W(stream, grown_out);
  OwnedBlock &R = W.grown;
  R.borrow(*right);
  for (int p = bond0; p >= 0; p--) {
    const dmrg_block_t &Lb = lefts[p];
    const std::vector<dmrg_sector_t> lsec(Lb.sec, Lb.sec + Lb.n_sec);
    std::vector<dmrg_oprec_t> crec;
    std::vector<Copy> copies;
    int64_t clen = 0;
    if (int rc = hpsi_form(lsec, Lb.rec, Lb.n_rec, Lb.data_len, p, n_orb, false, crec, copies, clen))
      return W.fail(rc);
    if (hipMalloc(&W.cat, sizeof(double) * std::max<int64_t>(clen, 1)) != hipSuccess) {
      set_error("hipMalloc failed");
      return W.fail(DMRG_ENOMEM);
    }
    for (const Copy &c : copies)
      if (c.n > 0 &&
          hipMemcpyAsync(W.cat + c.dst, Lb.data + c.src, sizeof(double) * c.n, hipMemcpyDeviceToDevice, W.hs) !=
              hipSuccess) {
        set_error("copying the left block failed");
        return W.fail(DMRG_EHIP);
      }
    const dmrg_block_t Rb = view(R);
    const dmrg_problem_t pr =
        make_problem(n_orb, n_elec, two_s, h1, eri, p, lsec, crec.data(), (int64_t)crec.size(), W.cat, clen, Rb);
    dmrg_sweep_step_t &S = steps[bond0 - p];
    S.bond = p;
    if (int rc = W.solve(pr, plan_opts, dav, seed, p, S)) return W.fail(rc);
    if (p == 0) break;
    if (int rc = W.cut(pr, pr, DMRG_RENORM_RIGHT, max_kept, S)) return W.fail(rc);
    if (int rc = W.hand_out(bond0 - p)) return W.fail(rc);
    W.free_bond();
  }
  W.free_bond();
  R.release();
  return DMRG_OK;
}

extern "C" void dmrg_block_release(dmrg_block_t *b) {
  if (!b) return;
  std::free(const_cast<dmrg_sector_t *>(b->sec));
  std::free(const_cast<dmrg_oprec_t *>(b->rec));
  if (b->data) (void)hipFree(const_cast<double *>(b->data));
  *b = dmrg_block_t{0, 0, nullptr, 0, nullptr, nullptr, 0};
}
