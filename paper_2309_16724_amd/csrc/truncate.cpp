// Truncation of a two-site step for the renormalization of the left block.
//
// After the Davidson solve the wavefunction is cut to at most D multiplets
// of (left block x left site) (Sec. II: the two-site DMRG step; the paper
// leaves the rule to the reviews it cites).  For every product sector
// (N, 2S) of the left block and the site -- rows ordered as in the
// renormalization's product basis: components (left sector a, site
// multiplet m), a ascending then m -- the reduced density matrix is
//     rho(a, a') = sum over right parts c of X_{a,c} X_{a',c}^T,
// X_{a,c} the d_a x d_R block of psi with (L l) part (a; N, 2S) and right
// part c = (r, R sector, 2S_rR).  The products run on the FP64 tile engine
// (one output tile per rho block, every right part a segment along K); the
// eigenvectors come from rocSOLVER's dsyevd, sector by sector on the
// caller's stream; the largest eigenvalues over all sectors are kept.  The
// mirror cuts (right site) x (right block) for the renormalization of the
// right block: rho(b, b') = sum over left parts c of X_{c,b}^T X_{c,b'}.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>
#include "common.hpp"
#include "plan.hpp"
#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>

using namespace dmrg;

namespace {

const int TSITE_N[3] = {0, 1, 2};
const int TSITE_S[3] = {0, 1, 0};

struct TComp { int lsec, site, row0, dim; };
struct TSec {
  int n = 0, two_s = 0, rows = 0;
  std::vector<TComp> comps;
};

// product sectors of (site) x (right block), (N, 2S) ascending: components
// site multiplet outer, right sector inner
std::vector<TSec> right_product(const std::vector<dmrg_sector_t> &rsec) {
  std::map<std::pair<int, int>, TSec> m;
  for (int s = 0; s < 3; s++)
    for (int a = 0; a < (int)rsec.size(); a++)
      for (int S = std::abs(rsec[a].two_s - TSITE_S[s]); S <= rsec[a].two_s + TSITE_S[s]; S += 2) {
        TSec &r = m[{rsec[a].n + TSITE_N[s], S}];
        r.n = rsec[a].n + TSITE_N[s];
        r.two_s = S;
        r.comps.push_back({a, s, r.rows, rsec[a].dim});
        r.rows += rsec[a].dim;
      }
  std::vector<TSec> out;
  for (auto &kv : m) out.push_back(kv.second);
  return out;
}

// product sectors of (left block) x (site), (N, 2S) ascending; components
// in the order left sector, then site multiplet
std::vector<TSec> left_product(const std::vector<dmrg_sector_t> &lsec) {
  std::map<std::pair<int, int>, TSec> m;
  for (int a = 0; a < (int)lsec.size(); a++)
    for (int s = 0; s < 3; s++)
      for (int S = std::abs(lsec[a].two_s - TSITE_S[s]); S <= lsec[a].two_s + TSITE_S[s]; S += 2) {
        TSec &r = m[{lsec[a].n + TSITE_N[s], S}];
        r.n = lsec[a].n + TSITE_N[s];
        r.two_s = S;
        r.comps.push_back({a, s, r.rows, lsec[a].dim});
        r.rows += lsec[a].dim;
      }
  std::vector<TSec> out;
  for (auto &kv : m) out.push_back(kv.second);
  return out;
}

int tile_shape(int m, int n) { return m <= 16 ? 1 : n <= 16 ? 4 : 2; }

// The density-matrix products of one truncation: rho of every product
// sector (offsets roff, column-major rows x rows) as tiles over psi.
struct RhoLists {
  std::vector<TSec> prod;
  std::vector<int64_t> roff;
  std::vector<Tile> tiles;
  std::vector<Seg> segs;
  std::vector<double> cost;
};

int build_rho(const dmrg_problem_t *prob, int32_t flags, RhoLists &RL) {
  const bool right = flags & 2;   // DMRG_RENORM_RIGHT: (right site) x (right block)
  std::vector<TSec> &prod = RL.prod;
  std::vector<int64_t> &roff = RL.roff;
  std::vector<Tile> &tiles = RL.tiles;
  std::vector<Seg> &segs = RL.segs;
  std::vector<double> &cost = RL.cost;
  Error err{0, ""};
  BlockModel L, R;
  if (build_block(L, 0, *prob, err) || build_block(R, 1, *prob, err)) { set_error(err.msg); return err.code; }
  std::vector<PsiBlock> blocks;
  int64_t size = 0;
  psi_blocks(L, R, prob->n_elec, prob->two_s, blocks, size);
  if (blocks.empty()) { set_error("no wavefunction block has the target N and S"); return DMRG_ESYM; }
  prod = right ? right_product(R.sec) : left_product(L.sec);
  std::map<std::pair<int, int>, int> sidx;
  for (int i = 0; i < (int)prod.size(); i++) sidx[{prod[i].n, prod[i].two_s}] = i;
  // per sector: component -> (right part -> block)
  std::vector<std::map<int, std::map<std::tuple<int, int, int>, int>>> parts(prod.size());
  for (int bi = 0; bi < (int)blocks.size(); bi++) {
    const PsiBlock &b = blocks[bi];
    const int si = right ? sidx.at({R.sec[b.iR].n + TSITE_N[b.r], b.SrR}) : sidx.at({L.sec[b.iL].n + TSITE_N[b.l], b.SLl});
    int ci = -1;
    for (int c = 0; c < (int)prod[si].comps.size(); c++)
      if (right ? (prod[si].comps[c].lsec == b.iR && prod[si].comps[c].site == b.r)
                : (prod[si].comps[c].lsec == b.iL && prod[si].comps[c].site == b.l))
        ci = c;
    parts[si][ci][right ? std::make_tuple(b.iL, b.l, b.SLl) : std::make_tuple(b.r, b.iR, b.SrR)] = bi;
  }
  // rho blocks as tiles: rho(a, a') += X_{a,c} X_{a',c}^T over common right parts c
  roff.assign(prod.size() + 1, 0);
  for (size_t i = 0; i < prod.size(); i++) roff[i + 1] = roff[i] + (int64_t)prod[i].rows * prod[i].rows;
  for (size_t si = 0; si < prod.size(); si++) {
    const TSec &P = prod[si];
    for (auto &ka : parts[si])
      for (auto &kb : parts[si]) {
        const TComp &ca = P.comps[ka.first], &cb = P.comps[kb.first];
        const int seg0 = (int)segs.size();
        double ksum = 0.0;
        for (auto &pc : ka.second) {
          auto it = kb.second.find(pc.first);
          if (it == kb.second.end()) continue;
          const PsiBlock &A = blocks[pc.second], &Bb = blocks[it->second];
          Seg S{};
          S.a_base = BASE_PSI; S.a_off = A.off; S.a_p = 0;
          S.b_base = BASE_PSI; S.b_off = Bb.off; S.b_pk = 0; S.b_pn = 0;
          if (!right) {   // X_a X_a'^T: K over the right part's columns
            S.a_i = 1; S.a_k = A.dL; S.b_k = Bb.dL; S.b_n = 1;
            S.K = A.dR; S.b_nb = Bb.dL;
          } else {        // X_b^T X_b': K over the left part's rows
            S.a_i = A.dL; S.a_k = 1; S.b_k = 1; S.b_n = Bb.dL;
            S.K = A.dL; S.b_nb = Bb.dR;
          }
          S.a_kb = S.K; S.b_kb = S.K;
          S.s = 1.0;
          segs.push_back(S);
          ksum += S.K;
        }
        const int nseg = (int)segs.size() - seg0;
        if (nseg == 0) continue;
        const int m = ca.dim, n = cb.dim, mb = tile_shape(m, n), tr = tile_rows(mb), tc = tile_cols(mb);
        for (int i0 = 0; i0 < m; i0 += tr)
          for (int j0 = 0; j0 < n; j0 += tc) {
            Tile T{};
            T.c_off = roff[si] + ca.row0 + (int64_t)cb.row0 * P.rows;
            T.ldc = P.rows; T.c_base = BASE_Y;
            T.m = m; T.n = n; T.i0 = i0; T.j0 = j0; T.ci0 = i0; T.cj0 = j0;
            T.mb = mb; T.seg0 = seg0; T.nseg = nseg; T.accumulate = 0; T.rowmajor = 0;
            tiles.push_back(T);
            cost.push_back((double)std::min(tr, m - i0) * std::min(tc, n - j0) * ksum);
          }
      }
  }
  // every lane's reads stay inside psi (lanes past the tile or K read row 0,
  // column 0 or element K - 1 of their operand)
  for (const Tile &T : tiles)
    for (int i = 0; i < T.nseg; i++) {
      const Seg &S = segs[T.seg0 + i];
      if (S.a_off + (int64_t)(T.m - 1) * S.a_i + (int64_t)(S.K - 1) * S.a_k >= size ||
          S.b_off + (int64_t)(S.K - 1) * S.b_k + (int64_t)(T.n - 1) * S.b_n >= size) {
        set_error("internal: a density-matrix product reaches beyond psi");
        return DMRG_ERANGE;
      }
    }
  return DMRG_OK;
}

}  // namespace

extern "C" int dmrg_truncate(const dmrg_problem_t *prob, int32_t flags, const double *psi, int32_t max_kept, double cutoff,
                             dmrg_rkeep_t *keep, int32_t keep_cap, int32_t *n_keep, double *u, int64_t u_cap,
                             int64_t *u_len, double *weights, void *stream) {
  if (!prob || !psi || !n_keep || !u_len || max_kept < 0 || (flags & ~2)) {
    set_error("null argument, negative max_kept or unknown flag");
    return DMRG_EINVAL;
  }
  RhoLists RL;
  if (int rc = build_rho(prob, flags, RL)) return rc;
  std::vector<TSec> &prod = RL.prod;
  std::vector<int64_t> &roff = RL.roff;
  std::vector<Tile> &tiles = RL.tiles;
  std::vector<Seg> &segs = RL.segs;
  std::vector<double> &cost = RL.cost;
  std::vector<int> ord(tiles.size());
  for (size_t i = 0; i < ord.size(); i++) ord[i] = (int)i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<Tile> st(tiles.size());
  std::vector<double> sc(tiles.size());
  for (size_t i = 0; i < ord.size(); i++) { st[i] = tiles[ord[i]]; sc[i] = cost[ord[i]]; }
  XcdQueues q{};
  {
    double tot = 0.0, acc = 0.0;
    for (double c : sc) tot += c;
    int i = 0;
    const int n = (int)sc.size();
    for (int x = 1; x < NXCD; x++) {
      while (i < n && acc + 0.5 * sc[i] < tot * x / NXCD) acc += sc[i++];
      q.start[x] = i;
    }
    q.start[0] = 0;
    q.start[NXCD] = n;
  }
  int maxn = 1;
  for (const TSec &P : prod) maxn = std::max(maxn, P.rows);
  hipStream_t hs = (hipStream_t)stream;
  Tile *d_t = nullptr;
  Seg *d_s = nullptr;
  int32_t *d_cnt = nullptr, *d_info = nullptr;
  double *d_rho = nullptr, *d_w = nullptr, *d_e = nullptr;
  const double **d_bases = nullptr;
  rocblas_handle h = nullptr;
  auto cleanup = [&]() {
    if (h) rocblas_destroy_handle(h);
    void *ptrs[] = {d_t, d_s, d_cnt, d_info, d_rho, d_w, d_e, (void *)d_bases};
    for (void *p : ptrs)
      if (p) (void)hipFree(p);
  };
  auto fail = [&](int code, const char *msg) {
    (void)hipStreamSynchronize(hs);
    cleanup();
    set_error(msg);
    return code;
  };
  bool ok = hipMalloc((void **)&d_t, std::max<size_t>(16, st.size() * sizeof(Tile))) == hipSuccess &&
            hipMalloc((void **)&d_s, std::max<size_t>(16, segs.size() * sizeof(Seg))) == hipSuccess &&
            hipMalloc((void **)&d_cnt, QUEUE_INTS * sizeof(int32_t)) == hipSuccess &&
            hipMalloc((void **)&d_info, prod.size() * sizeof(int32_t)) == hipSuccess &&
            hipMalloc((void **)&d_rho, std::max<int64_t>(1, roff.back()) * sizeof(double)) == hipSuccess &&
            hipMalloc((void **)&d_w, std::max<int64_t>(1, prod.empty() ? 1 : (int64_t)prod.size() * maxn) * sizeof(double)) == hipSuccess &&
            hipMalloc((void **)&d_e, (size_t)maxn * sizeof(double)) == hipSuccess &&
            hipMalloc((void **)&d_bases, 16) == hipSuccess;
  if (!ok) return fail(DMRG_ENOMEM, "device allocation failed");
  if (hipMemcpyAsync(d_t, st.data(), st.size() * sizeof(Tile), hipMemcpyHostToDevice, hs) != hipSuccess ||
      hipMemcpyAsync(d_s, segs.data(), segs.size() * sizeof(Seg), hipMemcpyHostToDevice, hs) != hipSuccess)
    return fail(DMRG_EHIP, "copying the density-matrix lists failed");
  launch_zero(d_rho, roff.back(), stream);
  launch_tiles_f64(1, d_t, d_s, (int)st.size(), q, d_cnt, d_bases, psi, d_rho, nullptr, nullptr, stream);
  if (rocblas_create_handle(&h) != rocblas_status_success || rocblas_set_stream(h, hs) != rocblas_status_success)
    return fail(DMRG_EHIP, "rocBLAS handle");
  for (size_t si = 0; si < prod.size(); si++) {
    const int n = prod[si].rows;
    if (rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_lower, n, d_rho + roff[si], n, d_w + si * maxn, d_e,
                         d_info + si) != rocblas_status_success)
      return fail(DMRG_EHIP, "rocsolver_dsyevd failed");
  }
  std::vector<double> w((size_t)prod.size() * maxn);
  std::vector<int32_t> info(prod.size());
  if (hipMemcpyAsync(w.data(), d_w, w.size() * sizeof(double), hipMemcpyDeviceToHost, hs) != hipSuccess ||
      hipMemcpyAsync(info.data(), d_info, info.size() * sizeof(int32_t), hipMemcpyDeviceToHost, hs) != hipSuccess ||
      hipStreamSynchronize(hs) != hipSuccess)
    return fail(DMRG_EHIP, "reading the eigenvalues failed");
  for (int32_t v : info)
    if (v != 0) return fail(DMRG_EHIP, "the eigensolver did not converge");
  // the largest eigenvalues over all sectors (ties: sector order, then rank)
  std::vector<std::tuple<double, int, int>> cand;
  double total = 0.0;
  for (size_t si = 0; si < prod.size(); si++) {
    const int n = prod[si].rows;
    for (int i = n - 1; i >= 0; i--) {
      const double v = w[si * maxn + i];
      total += v;
      if (v > cutoff) cand.push_back(std::make_tuple(-v, (int)si, n - 1 - i));
    }
  }
  std::sort(cand.begin(), cand.end());
  std::vector<int> take(prod.size(), 0);
  double kept_w = 0.0;
  for (size_t i = 0; i < cand.size() && (int64_t)i < max_kept; i++) {
    take[std::get<1>(cand[i])]++;
    kept_w -= std::get<0>(cand[i]);
  }
  int nk = 0;
  int64_t ul = 0;
  for (size_t si = 0; si < prod.size(); si++)
    if (take[si]) { nk++; ul += (int64_t)prod[si].rows * take[si]; }
  *n_keep = nk;
  *u_len = ul;
  if (weights) { weights[0] = kept_w; weights[1] = total; }
  if (!keep || !u) { cleanup(); return DMRG_OK; }
  if (keep_cap < nk || u_cap < ul) return fail(DMRG_ERANGE, "keep or U array too small");
  int k = 0;
  int64_t off = 0;
  for (size_t si = 0; si < prod.size(); si++) {
    if (!take[si]) continue;
    const int n = prod[si].rows;
    keep[k++] = dmrg_rkeep_t{prod[si].n, prod[si].two_s, take[si], 0, off};
    // eigenvectors in descending eigenvalue order (dsyevd returns them ascending)
    for (int j = 0; j < take[si]; j++)
      if (hipMemcpyAsync(u + off + (int64_t)j * n, d_rho + roff[si] + (int64_t)(n - 1 - j) * n, (size_t)n * sizeof(double),
                         hipMemcpyDeviceToDevice, hs) != hipSuccess)
        return fail(DMRG_EHIP, "copying the kept eigenvectors failed");
    off += (int64_t)n * take[si];
  }
  if (hipStreamSynchronize(hs) != hipSuccess) return fail(DMRG_EHIP, "truncation failed");
  cleanup();
  return DMRG_OK;
}

// Test-only: the density matrices of dmrg_truncate computed on the host with
// the kernels' addressing from a HOST psi: rho of every product sector in
// product order, column-major rows x rows, concatenated (rho NULL: only the
// length in *len).
extern "C" int dmrg_debug_truncate_rho_host(const dmrg_problem_t *prob, int32_t flags, const double *psi,
                                            double *rho, int64_t cap, int64_t *len) {
  if (!prob || !len || (flags & ~2)) { set_error("null argument or unknown flag"); return DMRG_EINVAL; }
  RhoLists RL;
  if (int rc = build_rho(prob, flags, RL)) return rc;
  *len = RL.roff.back();
  if (!rho) return DMRG_OK;
  if (!psi || cap < *len) { set_error("missing psi or rho too small"); return DMRG_ERANGE; }
  std::fill(rho, rho + *len, 0.0);
  for (const Tile &T : RL.tiles) {
    const int mt = std::min(tile_rows(T.mb), T.m - T.i0), nt = std::min(tile_cols(T.mb), T.n - T.j0);
    for (int j = 0; j < nt; j++)
      for (int i = 0; i < mt; i++) {
        double acc = 0.0;
        for (int si = 0; si < T.nseg; si++) {
          const Seg &S = RL.segs[T.seg0 + si];
          for (int k = 0; k < S.K; k++)
            acc += S.s * psi[S.a_off + (int64_t)(T.i0 + i) * S.a_i + (int64_t)k * S.a_k] *
                   psi[S.b_off + (int64_t)k * S.b_k + (int64_t)(T.j0 + j) * S.b_n];
        }
        rho[T.c_off + (T.ci0 + i) + (int64_t)(T.cj0 + j) * T.ldc] = acc;
      }
  }
  return DMRG_OK;
}
