// A left-to-right two-site sweep on the device (Sec. II: two-site DMRG;
// Sec. I: the Davidson solve and the renormalization of the block operators
// are the two parts of every step).  At every bond the two-site problem of
// the current left block and the caller's right block of that bond is
// planned (dmrg_build_tasks, FP64) and solved (dmrg_davidson); the
// wavefunction is cut to at most D multiplets of (left block x site)
// (dmrg_truncate) and the left block is renormalized in that basis
// (dmrg_renorm_*, all-pairs form) into the left block of the next bond.
// Blocks stay in device memory from step to step; only their sector and
// record tables live on the host.  The H.psi form of the left block (P and Q
// over the pairs that touch the two sites) is cut from its all-pairs records
// by device copies of the selected positions.
#include <hip/hip_runtime.h>
#include "common.hpp"
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

using namespace dmrg;

namespace {

// a block owned by the sweep: host tables, device data
struct OwnedBlock {
  std::vector<dmrg_sector_t> sec;
  std::vector<dmrg_oprec_t> rec;
  double *data = nullptr;
  int64_t len = 0;
  bool owned = false;
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

}  // namespace

extern "C" int dmrg_sweep_left_to_right(int32_t n_orb, int32_t n_elec, int32_t two_s, const double *h1,
                                        const double *eri, int32_t bond0, const dmrg_block_t *left,
                                        const dmrg_block_t *rights, int32_t max_kept, const dmrg_dav_opts_t *dav,
                                        uint64_t seed, dmrg_sweep_step_t *steps, void *stream) {
  if (!h1 || !eri || !left || !rights || !steps || bond0 < 1 || bond0 > n_orb - 2 || max_kept < 1) {
    set_error("bad sweep arguments (1 <= bond0 <= n_orb - 2, max_kept >= 1)");
    return DMRG_EINVAL;
  }
  hipStream_t hs = (hipStream_t)stream;
  OwnedBlock L;
  L.sec.assign(left->sec, left->sec + left->n_sec);
  L.rec.assign(left->rec, left->rec + left->n_rec);
  L.data = const_cast<double *>(left->data);
  L.len = left->data_len;
  dmrg_plan_t *plan = nullptr;
  dmrg_renorm_t *ren = nullptr;
  double *psi = nullptr, *u = nullptr, *cat = nullptr, *out = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(hs);
    if (plan) dmrg_plan_free(plan);
    if (ren) dmrg_renorm_free(ren);
    void *ptrs[] = {psi, u, cat, out};
    for (void *q : ptrs)
      if (q) (void)hipFree(q);
    plan = nullptr; ren = nullptr; psi = u = cat = out = nullptr;
  };
  auto fail = [&](int rc) {
    std::string msg = dmrg_last_error();
    cleanup();
    L.release();
    set_error(msg);
    return rc;
  };
  for (int p = bond0; p <= n_orb - 2; p++) {
    const dmrg_block_t &Rb = rights[p - bond0];
    // H.psi form of the left block: P and Q positions of the pairs at the sites
    std::vector<dmrg_oprec_t> crec;
    int64_t clen = 0;
    struct Copy { int64_t dst, src, n; };
    std::vector<Copy> copies;
    for (const dmrg_oprec_t &r : L.rec) {
      if (r.row_sec < 0 || r.row_sec >= (int)L.sec.size() || r.col_sec < 0 || r.col_sec >= (int)L.sec.size()) {
        set_error("left block record with a bad sector");
        return fail(DMRG_EINVAL);
      }
      const int64_t bs = (int64_t)L.sec[r.row_sec].dim * L.sec[r.col_sec].dim;
      if (r.npos < 0 || r.off < 0 || r.off + (int64_t)r.npos * bs > L.len) {
        set_error("left block record outside its data");
        return fail(DMRG_EINVAL);
      }
      dmrg_oprec_t c = r;
      c.off = clen;
      if (is_pq(r.fam)) {
        auto all = pq_labels(r.fam, p, n_orb, true), want = pq_labels(r.fam, p, n_orb, false);
        if ((int)all.size() != r.npos) { set_error("left block P/Q records are not in the all-pairs form"); return fail(DMRG_EINVAL); }
        c.npos = (int32_t)want.size();
        size_t j = 0;
        for (size_t i = 0; i < all.size() && j < want.size(); i++)
          if (all[i] == want[j]) { copies.push_back({clen + (int64_t)j * bs, r.off + (int64_t)i * bs, bs}); j++; }
      } else {
        copies.push_back({clen, r.off, (int64_t)r.npos * bs});
      }
      if (c.npos == 0) continue;
      clen += (int64_t)c.npos * bs;
      crec.push_back(c);
    }
    if (hipMalloc(&cat, sizeof(double) * std::max<int64_t>(clen, 1)) != hipSuccess) { set_error("hipMalloc failed"); return fail(DMRG_ENOMEM); }
    for (const Copy &c : copies)
      if (c.n > 0 && hipMemcpyAsync(cat + c.dst, L.data + c.src, sizeof(double) * c.n, hipMemcpyDeviceToDevice, hs) != hipSuccess) {
        set_error("copying the left block failed");
        return fail(DMRG_EHIP);
      }
    dmrg_problem_t pr{};
    pr.n_orb = n_orb; pr.n_elec = n_elec; pr.two_s = two_s; pr.site_l = p;
    pr.h1 = h1; pr.eri = eri;
    pr.n_lsec = (int32_t)L.sec.size(); pr.lsec = L.sec.data();
    pr.n_rsec = Rb.n_sec; pr.rsec = Rb.sec;
    pr.n_lrec = (int64_t)crec.size(); pr.lrec = crec.data();
    pr.n_rrec = Rb.n_rec; pr.rrec = Rb.rec;
    pr.ldata = cat; pr.ldata_len = clen;
    pr.rdata = Rb.data; pr.rdata_len = Rb.data_len;
    if (int rc = dmrg_build_tasks(&pr, 1, nullptr, stream, &plan)) return fail(rc);
    int64_t off = 0, n = 0;
    dmrg_plan_stats_t pst{};
    if (int rc = dmrg_psi_layout(plan, 0, &off, &n)) return fail(rc);
    if (int rc = dmrg_plan_stats(plan, &pst)) return fail(rc);
    if (off < 0 || n < 1 || off + n > pst.psi_len) { set_error("unexpected wavefunction layout"); return fail(DMRG_EINVAL); }
    std::vector<double> x((size_t)pst.psi_len, 0.0);
    uint64_t st = seed + (uint64_t)p * 0x100000001ull;
    double nrm = 0.0;
    for (int64_t i = 0; i < n; i += 2) {
      const double r1 = std::sqrt(-2.0 * std::log(uniform01(st))), t = 6.283185307179586 * uniform01(st);
      x[off + i] = r1 * std::cos(t);
      if (i + 1 < n) x[off + i + 1] = r1 * std::sin(t);
    }
    for (double v : x) nrm += v * v;
    for (double &v : x) v /= std::sqrt(nrm);
    if (hipMalloc(&psi, sizeof(double) * pst.psi_len) != hipSuccess ||
        hipMemcpyAsync(psi, x.data(), sizeof(double) * pst.psi_len, hipMemcpyHostToDevice, hs) != hipSuccess ||
        hipStreamSynchronize(hs) != hipSuccess) {
      set_error("uploading the start vector failed");
      return fail(DMRG_EHIP);
    }
    double e = 0.0;
    dmrg_dav_stats_t ds{};
    if (int rc = dmrg_davidson(plan, psi, &e, dav, &ds, stream)) return fail(rc);
    dmrg_sweep_step_t &S = steps[p - bond0];
    S.bond = p; S.energy = e; S.iters = ds.iters; S.kept = 0; S.kept_weight = 1.0; S.pad = 0;
    if (p == n_orb - 2) break;
    // truncation and renormalization into the left block of bond p + 1
    int32_t nk = 0;
    int64_t ul = 0;
    double w[2] = {0.0, 0.0};
    if (int rc = dmrg_truncate(&pr, 0, psi, max_kept, 1e-14, nullptr, 0, &nk, nullptr, 0, &ul, w, stream)) return fail(rc);
    std::vector<dmrg_rkeep_t> keep((size_t)std::max(nk, 1));
    if (hipMalloc(&u, sizeof(double) * std::max<int64_t>(ul, 1)) != hipSuccess) { set_error("hipMalloc failed"); return fail(DMRG_ENOMEM); }
    if (int rc = dmrg_truncate(&pr, 0, psi, max_kept, 1e-14, keep.data(), nk, &nk, u, ul, &ul, w, stream)) return fail(rc);
    S.kept = 0;
    for (int i = 0; i < nk; i++) S.kept += keep[i].kept;
    S.kept_weight = w[1] > 0.0 ? w[0] / w[1] : 0.0;
    dmrg_problem_t pa = pr;   // the all-pairs left block
    pa.n_lrec = (int64_t)L.rec.size(); pa.lrec = L.rec.data();
    pa.ldata = L.data; pa.ldata_len = L.len;
    if (int rc = dmrg_renorm_create(&pa, keep.data(), nk, 0, DMRG_RENORM_ALL_PAIRS, ul, &ren)) return fail(rc);
    int64_t nrec = 0, olen = 0;
    if (int rc = dmrg_renorm_records(ren, nullptr, 0, &nrec, &olen)) return fail(rc);
    std::vector<dmrg_oprec_t> orec((size_t)std::max<int64_t>(nrec, 1));
    if (int rc = dmrg_renorm_records(ren, orec.data(), nrec, &nrec, &olen)) return fail(rc);
    if (hipMalloc(&out, sizeof(double) * std::max<int64_t>(olen, 1)) != hipSuccess) { set_error("hipMalloc failed"); return fail(DMRG_ENOMEM); }
    if (int rc = dmrg_renorm_apply(ren, u, out, stream)) return fail(rc);
    if (hipStreamSynchronize(hs) != hipSuccess) { set_error("renormalization failed"); return fail(DMRG_EHIP); }
    // the new left block replaces the old one
    L.release();
    L.sec.clear();
    for (int i = 0; i < nk; i++) L.sec.push_back(dmrg_sector_t{keep[i].n, keep[i].two_s, keep[i].kept});
    L.rec.assign(orec.begin(), orec.begin() + nrec);
    L.data = out; L.len = olen; L.owned = true;
    out = nullptr;
    cleanup();
  }
  cleanup();
  L.release();
  return DMRG_OK;
}
