// Renormalization of the left block through the left site.
//
// After a two-site step the left block L = [0, l) and the site l merge into
// the block L' = [0, l] of the next bond (Sec. I: block operators are
// renormalized during the contraction, 5-10 % of the run time; Sec. II C:
// the block x site tensor product A (x) B is processed sector by sector like
// the U(1) one, every result scaled by the factor C~ of Eq. (4) that the
// paper keeps in its W9j(l) table).  The basis of L' is given per (N, 2S)
// sector by U, whose rows are the coupled product states ((L S_L) x (l s)) S
// and whose columns are the kept states, so every operator of L' is
//     O'(b', a') = sum_terms coef  U_b'[rows of (b, s_b)]^T  op(A)(b, a)  U_a'[rows of (a, s_a)].
// Each term is alpha [A^kA (x) B^kB]^K with A a stored member of L (or the
// identity) and B a site operator (or the identity); coef = alpha C~
// <s_b||B||s_a> (-1)^(parity(B) N_a) (and the adjoint phase when A is
// applied as an adjoint).  The products run on the FP64 stripe engine of
// H.psi in two launches: T = op(A) U_a'[rows] for every distinct
// (member, ket component) and O' = sum coef U_b'[rows]^T T, every output
// tile summing its terms in a fixed order (no atomics, reproducible).
//
// Terms: members of L' whose labels lie in L are [A (x) 1]; members with the
// label l are products of single creation and annihilation operators; the
// block Hamiltonian of L' is H restricted to the orbitals [0, l] with the
// parts of two or more indices in L taken from the complementary operators
// S_l, P_ll, Q_ll of L; S_x of L' (x > l) is S_x of L plus the parts with
// one index at l, which are P_xl and Q_xl of L times a single site operator,
// plus explicit products.  Spin-orbital products are projected onto the
// coupled form by their Q = K component (the same Clebsch-Gordan projection
// the operator table of H.psi uses).  P and Q of L' are not produced: they
// need P and Q of L for every outside pair, while the H.psi input keeps only
// the pairs that touch the two sites.
#include <hip/hip_runtime.h>
#include "common.hpp"
#include "plan.hpp"
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>

using namespace dmrg;

namespace {

// wavefront tile shape for an m x n output: 16 x 64 for short outputs,
// 64 x 16 for narrow ones, else 32 x 32
int tile_mb(int m, int n) { return m <= 16 ? 1 : n <= 16 ? 4 : 2; }

// NXCD contiguous ranges of a cost-sorted tile list with about equal cost
XcdQueues equal_cost_ranges(const std::vector<double> &cost) {
  XcdQueues q{};
  double tot = 0.0;
  for (double c : cost) tot += c;
  const int n = (int)cost.size();
  double acc = 0.0;
  int i = 0;
  for (int x = 1; x < NXCD; x++) {
    while (i < n && acc + 0.5 * cost[i] < tot * x / NXCD) acc += cost[i++];
    q.start[x] = i;
  }
  q.start[0] = 0;
  q.start[NXCD] = n;
  return q;
}

const int RSITE_N[3] = {0, 1, 2};
const int RSITE_S[3] = {0, 1, 0};
constexpr int RENORM_DEFAULT_MASK =
    (1 << F_H) | (1 << F_C) | (1 << F_A0) | (1 << F_A1) | (1 << F_B0) | (1 << F_B1) | (1 << F_S);
constexpr int RENORM_PAIR_MASK = (1 << F_P0) | (1 << F_P1) | (1 << F_Q0) | (1 << F_Q1);
constexpr int RENORM_ALL_PAIRS = 1;   // dmrg_renorm_create flags
constexpr int RENORM_RIGHT = 2;
constexpr int RENORM_RIGHT_MASK =
    (1 << F_H) | (1 << F_C) | (1 << F_S) | (1 << F_P0) | (1 << F_P1) | (1 << F_Q0) | (1 << F_Q1);

// factor of a spin-orbital product: part 0 the block (a family component),
// part 1 the site (an elementary a+ (adj 0) or a~ (adj 1) component)
struct RF {
  int part, fam, adj, k2, q2;
};
struct RProd {
  double coef;
  std::vector<RF> f;
};

double sgn2(int x2) { return ((x2 / 2) % 2) ? -1.0 : 1.0; }   // (-1)^(x2/2), x2 even
int rf_parity(const RF &c) { return c.part == 1 ? 1 : FAM_PAR[c.fam]; }

// a+_{x s} = C_s; a_{x s} = (-1)^(1/2 + s) C~_{-s}
RF elem(int x, int p, int s2, bool dagger, double &coef) {
  RF f{x < p ? 0 : 1, F_C, dagger ? 0 : 1, 1, dagger ? s2 : -s2};
  if (!dagger && ((1 + s2) / 2) % 2) coef = -coef;
  return f;
}
RF famc(int fam, int adj, int q2) { return RF{0, fam, adj, FAM_TWO_K[fam], q2}; }

// (T_q)^+ = (-1)^(k+q) T~_{-q};  (T~_q)^+ = (-1)^(k+q) (-1)^(2k) T_{-q}
RProd adjoint(const RProd &p) {
  RProd r;
  r.coef = p.coef;
  for (auto it = p.f.rbegin(); it != p.f.rend(); ++it) {
    RF c = *it;
    if (((c.k2 + c.q2) / 2) % 2) r.coef = -r.coef;
    if (c.adj && (c.k2 % 2)) r.coef = -r.coef;
    c.adj ^= 1;
    c.q2 = -c.q2;
    r.f.push_back(c);
  }
  return r;
}

struct TermKey {
  PT a, b;
  bool operator<(const TermKey &o) const {
    if (a < o.a) return true;
    if (o.a < a) return false;
    return b < o.b;
  }
};

// Coupled terms alpha [A (x) B]^K (side 0: block A then site B) or
// alpha [B (x) A]^K (side 1: site then block) of products that make up the
// Q = K component of a rank-K operator.  Factors are reordered into
// Jordan-Wigner order: the block first on side 0, the site first on side 1.
int project_rank(const std::vector<RProd> &prods, SiteAlgebra &site, int K2,
                 std::vector<std::pair<TermKey, double>> &out, Error &err, int side = 0) {
  auto jw = [side](const RF &c) { return side == 0 ? c.part : 1 - c.part; };
  std::map<TermKey, std::map<std::pair<int, int>, double>> F;
  for (const RProd &pr : prods) {
    if (pr.coef == 0.0) continue;
    std::vector<RF> f = pr.f;
    double sign = 1.0;
    for (size_t i = 0; i < f.size(); i++)
      for (size_t j = i + 1; j < f.size(); j++)
        if (jw(f[i]) > jw(f[j]) && rf_parity(f[i]) && rf_parity(f[j])) sign = -sign;
    std::stable_sort(f.begin(), f.end(), [&](const RF &a, const RF &b) { return jw(a) < jw(b); });
    PT ta;
    int qa = 0;
    std::vector<int> adj;
    std::vector<RF> mine;
    for (const RF &c : f) {
      if (c.part == 0) {
        if (ta.kind) { err = {DMRG_EINVAL, "internal: two block factors in one product"}; return err.code; }
        ta.kind = 1; ta.id = c.fam; ta.adj = c.adj; ta.k2 = c.k2; ta.par = FAM_PAR[c.fam];
        qa = c.q2;
      } else {
        mine.push_back(c);
        adj.push_back(c.adj);
      }
    }
    if (mine.empty()) {
      F[{ta, PT()}][{qa, 0}] += pr.coef * sign;
      continue;
    }
    // site string: expand over the intermediate couplings, left to right
    std::function<void(size_t, int, int, double, std::vector<int> &)> rec =
        [&](size_t i, int kacc, int qacc, double w, std::vector<int> &inter) {
          if (i == mine.size()) {
            PT tb;
            tb.kind = 2; tb.id = site.get(adj, inter); tb.k2 = kacc; tb.par = (int)(mine.size() % 2);
            F[{ta, tb}][{qa, qacc}] += pr.coef * sign * w;
            return;
          }
          const int qn = mine[i].q2;
          for (int knew = std::abs(kacc - 1); knew <= kacc + 1; knew += 2) {
            if (std::abs(qacc + qn) > knew) continue;
            double c = cg(kacc, qacc, 1, qn, knew, qacc + qn);
            if (c == 0.0) continue;
            inter.push_back(knew);
            rec(i + 1, knew, qacc + qn, w * c, inter);
            inter.pop_back();
          }
        };
    std::vector<int> inter;
    rec(1, 1, mine[0].q2, 1.0, inter);
  }
  for (auto &kv : F) {
    const TermKey &k = kv.first;
    if (k.b.kind == 2) {
      const auto &sf = site.fams[k.b.id];
      bool nz = false;
      for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) nz = nz || sf.red[i][j] != 0.0;
      if (!nz) continue;
    }
    double fmax = 0.0;
    for (auto &qv : kv.second) fmax = std::max(fmax, std::fabs(qv.second));
    if (fmax < 1e-15) continue;
    const int ka = k.a.k2, kb = k.b.k2;
    // least-squares alpha over the components, then every component checked
    double num = 0.0, den = 0.0;
    for (int q1 = -ka; q1 <= ka; q1 += 2) {
      int q2 = K2 - q1;
      if (std::abs(q2) > kb) continue;
      double c = side == 0 ? cg(ka, q1, kb, q2, K2, K2) : cg(kb, q2, ka, q1, K2, K2);
      auto it = kv.second.find({q1, q2});
      double fv = it == kv.second.end() ? 0.0 : it->second;
      num += c * fv;
      den += c * c;
    }
    double alpha = den > 0.0 ? num / den : 0.0;
    double resid = 0.0;
    for (auto &qv : kv.second) {
      double c = side == 0 ? cg(ka, qv.first.first, kb, qv.first.second, K2, K2)
                           : cg(kb, qv.first.second, ka, qv.first.first, K2, K2);
      resid = std::max(resid, std::fabs(qv.second - alpha * c));
    }
    if (resid > 1e-10 * fmax) {
      err = {DMRG_EINVAL, "internal: operator is not a coupled tensor of the target rank"};
      return err.code;
    }
    if (std::fabs(alpha) > 1e-13 * fmax) out.push_back({k, alpha});
  }
  return DMRG_OK;
}

// label lists of the left block's families at bond p (orbitals [0, p); S:
// outside orbitals [p, n); P, Q: every outside pair, lexicographic -- the
// all-pairs form)
std::vector<std::array<int, 2>> left_labels(int fam, int p, int n) {
  std::vector<std::array<int, 2>> res;
  auto grouped = [&](bool strict) {
    for (int x = 0; x < p; x++) for (int y = x + 1; y < p; y++) res.push_back({x, y});
    if (!strict) for (int x = 0; x < p; x++) res.push_back({x, x});
  };
  switch (fam) {
    case F_H: res.push_back({-1, -1}); break;
    case F_C: for (int i = 0; i < p; i++) res.push_back({i, -1}); break;
    case F_A0: case F_B0: case F_B1: grouped(false); break;
    case F_A1: grouped(true); break;
    case F_S: for (int x = p; x < n; x++) res.push_back({x, -1}); break;
    default:
      for (int x = p; x < n; x++)
        for (int y = x + (fam == F_P1 ? 1 : 0); y < n; y++) res.push_back({x, y});
      break;
  }
  return res;
}

// one term of an operator of L'
struct RTerm {
  int fam, pos;      // target member of L'
  PT ta;             // L factor (kind 0 identity, 1 family)
  int posA;
  PT tb;             // site factor (kind 0 identity, 2 site family)
  double alpha;
  int dress = -1;    // >= 0: the L factor is dressed operator `dress` (posA unused)
};

// A dressed operator: sum_j alpha_j C_j (or the sum of their adjoints) over
// positions j of the C family, one block per C record.
struct DressG {
  int adj;
  std::vector<std::pair<int, double>> src;   // (position, alpha)
};

int add_projected(const std::vector<RProd> &prods, SiteAlgebra &site, const BlockModel &L, int fam, int pos,
                  int x, int y, std::vector<RTerm> &terms, Error &err, int side = 0) {
  std::vector<std::pair<TermKey, double>> outs;
  if (project_rank(prods, site, FAM_TWO_K[fam], outs, err, side)) return err.code;
  for (auto &o : outs) {
    RTerm t{fam, pos, o.first.a, 0, o.first.b, o.second, -1};
    if (t.ta.kind == 1) {
      t.posA = L.pos(t.ta.id, x, y);
      if (t.posA < 0) { err = {DMRG_EINVAL, "internal: left label not in family"}; return err.code; }
    }
    terms.push_back(t);
  }
  return DMRG_OK;
}

int build_terms(const dmrg_problem_t &pr, const BlockModel &L, SiteAlgebra &site, int mask,
                std::vector<RTerm> &terms, Error &err) {
  const int p = pr.site_l, n = pr.n_orb;
  const int sp[2] = {1, -1};
  auto h = [&](int i, int j) { return pr.h1[(int64_t)i * n + j]; };
  auto v = [&](int i, int j, int k, int l) { return pr.eri[(((int64_t)i * n + j) * n + k) * n + l]; };
  for (int fam = 0; fam < N_FAM; fam++) {
    if (!(mask & (1 << fam))) continue;
    auto labs = left_labels(fam, p + 1, n);
    for (int pos = 0; pos < (int)labs.size(); pos++) {
      const int x = labs[pos][0], y = labs[pos][1];
      if (fam == F_H) {
        // block Hamiltonian of L
        {
          std::vector<RProd> pp{{1.0, {famc(F_H, 0, 0)}}};
          if (add_projected(pp, site, L, fam, pos, -1, -1, terms, err)) return err.code;
        }
        // three indices in L: sum_s a+_ls (S_l)_s + h.c., (S_x)_s = -sqrt2 (-1)^(1/2+s) S~_{-s}
        {
          std::vector<RProd> pp;
          for (int s : sp) {
            RProd q;
            q.coef = -std::sqrt(2.0) * sgn2(1 + s);
            q.f.push_back(elem(p, p, s, true, q.coef));
            q.f.push_back(famc(F_S, 0, -s));
            pp.push_back(q);
          }
          for (size_t i = 0, m = pp.size(); i < m; i++) pp.push_back(adjoint(pp[i]));
          if (add_projected(pp, site, L, fam, pos, p, -1, terms, err)) return err.code;
        }
        // two indices in L: 1/2 sum a+_ls a+_lt (P_ll)_ts + h.c.;  sum (Q_ll)_ts a+_lt a_ls
        {
          std::vector<RProd> pp;
          for (int s : sp)
            for (int t : sp) {
              double cP = sgn2(2 + t + s) * cg(1, -t, 1, -s, 0, -t - s);
              if (cP == 0.0) continue;
              RProd q;
              q.coef = 0.5 * cP;
              q.f.push_back(elem(p, p, s, true, q.coef));
              q.f.push_back(elem(p, p, t, true, q.coef));
              q.f.push_back(famc(F_P0, 0, -t - s));
              pp.push_back(q);
            }
          for (size_t i = 0, m = pp.size(); i < m; i++) pp.push_back(adjoint(pp[i]));
          if (add_projected(pp, site, L, fam, pos, p, p, terms, err)) return err.code;
        }
        {
          std::vector<RProd> pp;
          for (int s : sp)
            for (int t : sp) {
              std::vector<std::pair<double, RF>> parts;
              if (s == t) parts.push_back({-1.0 / std::sqrt(2.0), famc(F_Q0, 0, 0)});
              double c1 = cg(1, s, 1, -t, 2, s - t);
              if (c1 != 0.0) parts.push_back({-sgn2(1 + t) * c1 / std::sqrt(3.0), famc(F_Q1, 0, s - t)});
              for (auto &qp : parts) {
                RProd q;
                q.coef = qp.first;
                q.f.push_back(qp.second);
                q.f.push_back(elem(p, p, t, true, q.coef));
                q.f.push_back(elem(p, p, s, false, q.coef));
                pp.push_back(q);
              }
            }
          if (add_projected(pp, site, L, fam, pos, p, p, terms, err)) return err.code;
        }
        // at most one index in L, the others on the site: one instance per L orbital
        for (int li = -1; li < p; li++) {
          auto in_inst = [&](std::initializer_list<int> idx) {
            int nl = 0, which = -1;
            for (int i : idx) if (i < p) { nl++; which = i; }
            return nl == (li < 0 ? 0 : 1) && (li < 0 || which == li) && nl <= 1;
          };
          std::vector<RProd> pp;
          for (int i = 0; i <= p; i++)
            for (int j = 0; j <= p; j++) {
              if (!in_inst({i, j}) || h(i, j) == 0.0) continue;
              for (int s : sp) {
                RProd q;
                q.coef = h(i, j);
                q.f.push_back(elem(i, p, s, true, q.coef));
                q.f.push_back(elem(j, p, s, false, q.coef));
                pp.push_back(q);
              }
            }
          for (int i = 0; i <= p; i++)
            for (int j = 0; j <= p; j++)
              for (int k = 0; k <= p; k++)
                for (int l = 0; l <= p; l++) {
                  if (!in_inst({i, j, k, l}) || v(i, j, k, l) == 0.0) continue;
                  for (int s : sp)
                    for (int t : sp) {
                      if ((i == k || j == l) && s == t) continue;
                      RProd q;
                      q.coef = 0.5 * v(i, j, k, l);
                      q.f.push_back(elem(i, p, s, true, q.coef));
                      q.f.push_back(elem(k, p, t, true, q.coef));
                      q.f.push_back(elem(l, p, t, false, q.coef));
                      q.f.push_back(elem(j, p, s, false, q.coef));
                      pp.push_back(q);
                    }
                }
          if (pp.empty()) continue;
          if (add_projected(pp, site, L, fam, pos, li, -1, terms, err)) return err.code;
        }
        continue;
      }
      if (fam == F_P0 || fam == F_P1 || fam == F_Q0 || fam == F_Q1) {
        // P^K / Q^K of L' for the pair (x, y) (x, y > l): the member of L for
        // the same pair plus the terms with an index at l, explicit, from
        //   (P_xy)_ts = sum (xj|yl) a_lt a_js,
        //   (Q_xy)_ts = delta_ts sum (xy|kl) E_kl - sum (xl|ky) a+_ks a_lt,
        // and the tensor components they carry:
        //   P^K_K = sum_{-t-s=K} <1/2 -t, 1/2 -s|K K> (-1)^(1+t+s) (P_xy)_ts,
        //   Q0 = -sum_s (Q_xy)_ss / sqrt2,  Q1_{+1} = -sqrt3 (Q_xy)_{dn up}
        {
          RTerm t;
          t.fam = fam; t.pos = pos;
          t.ta.kind = 1; t.ta.id = fam; t.ta.adj = 0; t.ta.k2 = FAM_TWO_K[fam]; t.ta.par = FAM_PAR[fam];
          t.posA = L.pos(fam, x, y);
          if (t.posA < 0) { err = {DMRG_EINVAL, "left block lacks P or Q for an outside pair"}; return err.code; }
          t.alpha = 1.0;
          terms.push_back(t);
        }
        const int K2 = FAM_TWO_K[fam];
        std::vector<std::array<double, 3>> ts;    // (t, s, weight)
        for (int t : sp)
          for (int s2 : sp) {
            if (fam == F_P0 || fam == F_P1) {
              if (-t - s2 == K2) ts.push_back({(double)t, (double)s2, cg(1, -t, 1, -s2, K2, K2) * sgn2(2 + t + s2)});
            } else if (fam == F_Q0) {
              if (t == s2) ts.push_back({(double)t, (double)s2, -1.0 / std::sqrt(2.0)});
            } else if (t == -1 && s2 == 1) {
              ts.push_back({(double)t, (double)s2, -std::sqrt(3.0)});
            }
          }
        for (int li = -1; li < p; li++) {
          auto inst = [&](int i1, int i2) {
            if (i1 < p && i2 < p) return false;
            int which = i1 < p ? i1 : i2 < p ? i2 : -1;
            return which == li;
          };
          std::vector<RProd> pp;
          for (auto &w : ts) {
            const int t = (int)w[0], s2 = (int)w[1];
            if (w[2] == 0.0) continue;
            for (int a = 0; a <= p; a++)
              for (int b = 0; b <= p; b++) {
                if (!inst(a, b)) continue;
                if (fam == F_P0 || fam == F_P1) {         // j = a, l = b: (xj|yl) a_lt a_js
                  double vv = v(x, a, y, b);
                  if (vv == 0.0) continue;
                  RProd q;
                  q.coef = w[2] * vv;
                  q.f.push_back(elem(b, p, t, false, q.coef));
                  q.f.push_back(elem(a, p, s2, false, q.coef));
                  pp.push_back(q);
                } else {                                   // k = a, l = b
                  if (t == s2 && v(x, y, a, b) != 0.0)
                    for (int sg : sp) {
                      RProd q;
                      q.coef = w[2] * v(x, y, a, b);
                      q.f.push_back(elem(a, p, sg, true, q.coef));
                      q.f.push_back(elem(b, p, sg, false, q.coef));
                      pp.push_back(q);
                    }
                  if (v(x, b, a, y) != 0.0) {
                    RProd q;
                    q.coef = -w[2] * v(x, b, a, y);
                    q.f.push_back(elem(a, p, s2, true, q.coef));
                    q.f.push_back(elem(b, p, t, false, q.coef));
                    pp.push_back(q);
                  }
                }
              }
          }
          if (pp.empty()) continue;
          if (add_projected(pp, site, L, fam, pos, li, -1, terms, err)) return err.code;
        }
        continue;
      }
      if (fam == F_S) {
        // S_x of L' (x > l): component +1/2 = -(S_x)_dn / sqrt2 with
        // (S_x)_s = sum_{j,k,l in [0, l]} (xj|kl) E_kl a_js; the part inside L
        // is the stored S_x, the parts with one index at l are
        // sum_t (P_xl)_ts a+_lt and sum_t (Q_xl)_st a_lt of L, the rest explicit
        const double scale = -1.0 / std::sqrt(2.0);
        const int s = -1;
        {
          RTerm t;
          t.fam = fam; t.pos = pos;
          t.ta.kind = 1; t.ta.id = F_S; t.ta.adj = 0; t.ta.k2 = 1; t.ta.par = FAM_PAR[F_S];
          t.posA = L.pos(F_S, x);
          if (t.posA < 0) { err = {DMRG_EINVAL, "left block lacks S for an outside orbital"}; return err.code; }
          t.alpha = 1.0;
          terms.push_back(t);
        }
        // (P_xl)_ts = -(P_lx)_st; (P_lx)_st = (-1)^(1+s+t) sum_K <1/2 -s, 1/2 -t|K -s-t> P^K_{-s-t}
        {
          std::vector<RProd> pp;
          for (int t : sp)
            for (int K = 0; K <= 2; K += 2) {
              double cP = sgn2(2 + s + t) * cg(1, -s, 1, -t, K, -s - t);
              if (cP == 0.0) continue;
              RProd q;
              q.coef = -scale * cP;
              q.f.push_back(famc(K == 0 ? F_P0 : F_P1, 0, -s - t));
              q.f.push_back(elem(p, p, t, true, q.coef));
              pp.push_back(q);
            }
          if (add_projected(pp, site, L, fam, pos, p, x, terms, err)) return err.code;
        }
        // sum_t (Q_xl)_st a_lt = [sum_t a+_lt (Q_lx)_ts]^+
        {
          std::vector<RProd> pp;
          for (int t : sp) {
            std::vector<std::pair<double, RF>> parts;
            if (s == t) parts.push_back({-1.0 / std::sqrt(2.0), famc(F_Q0, 0, 0)});
            double c1 = cg(1, s, 1, -t, 2, s - t);
            if (c1 != 0.0) parts.push_back({-sgn2(1 + t) * c1 / std::sqrt(3.0), famc(F_Q1, 0, s - t)});
            for (auto &qp : parts) {
              RProd q;
              q.coef = scale * qp.first;
              q.f.push_back(elem(p, p, t, true, q.coef));
              q.f.push_back(qp.second);
              pp.push_back(adjoint(q));
            }
          }
          if (add_projected(pp, site, L, fam, pos, p, x, terms, err)) return err.code;
        }
        // two or three of j, k, l at l: explicit, one instance per L orbital
        for (int li = -1; li < p; li++) {
          std::vector<RProd> pp;
          for (int j = 0; j <= p; j++)
            for (int k = 0; k <= p; k++)
              for (int l = 0; l <= p; l++) {
                int atp = (j == p) + (k == p) + (l == p);
                if (atp < 2 || v(x, j, k, l) == 0.0) continue;
                int which = j < p ? j : k < p ? k : l < p ? l : -1;
                if (which != li) continue;
                for (int t : sp) {
                  RProd q;
                  q.coef = scale * v(x, j, k, l);
                  q.f.push_back(elem(k, p, t, true, q.coef));
                  q.f.push_back(elem(l, p, t, false, q.coef));
                  q.f.push_back(elem(j, p, s, false, q.coef));
                  pp.push_back(q);
                }
              }
          if (pp.empty()) continue;
          if (add_projected(pp, site, L, fam, pos, li, -1, terms, err)) return err.code;
        }
        continue;
      }
      if (x < p && (y < 0 || y < p)) {
        // a member of L: [A (x) 1]
        RTerm t;
        t.fam = fam; t.pos = pos;
        t.ta.kind = 1; t.ta.id = fam; t.ta.adj = 0; t.ta.k2 = FAM_TWO_K[fam]; t.ta.par = FAM_PAR[fam];
        t.posA = L.pos(fam, x, y);
        if (t.posA < 0) { err = {DMRG_EINVAL, "left block lacks a member of its own family"}; return err.code; }
        t.alpha = 1.0;
        terms.push_back(t);
        continue;
      }
      const int K2 = FAM_TWO_K[fam];
      std::vector<RProd> pp;
      if (fam == F_C) {
        RProd q;
        q.coef = 1.0;
        q.f.push_back(elem(x, p, 1, true, q.coef));
        pp.push_back(q);
      } else {
        for (int s : sp) {
          int t = K2 - s;
          if (std::abs(t) != 1) continue;
          double c = cg(1, s, 1, t, K2, K2);
          if (c == 0.0) continue;
          RProd q;
          q.coef = c;
          q.f.push_back(elem(x, p, s, true, q.coef));
          if (fam == F_A0 || fam == F_A1) q.f.push_back(elem(y, p, t, true, q.coef));
          else q.f.push_back(RF{y < p ? 0 : 1, F_C, 1, 1, t});     // a~_{y t}
          pp.push_back(q);
        }
      }
      if (add_projected(pp, site, L, fam, pos, x < p ? x : -1, -1, terms, err)) return err.code;
    }
  }
  return DMRG_OK;
}

// label lists of a right block's families at bond p (block [p + 2, n); the
// H.psi catalogue: S over [0, p + 2), P and Q over the grouped pairs)
std::vector<std::array<int, 2>> right_labels(int fam, int p, int n) {
  std::vector<std::array<int, 2>> res;
  const bool strict = fam == F_P1;
  switch (fam) {
    case F_H: res.push_back({-1, -1}); break;
    case F_C: for (int i = p + 2; i < n; i++) res.push_back({i, -1}); break;
    case F_S: for (int x = 0; x < p + 2; x++) res.push_back({x, -1}); break;
    case F_P0: case F_P1: case F_Q0: case F_Q1:
      for (int x = 0; x < p; x++) for (int y = x + 1; y < p; y++) res.push_back({x, y});
      if (!strict) for (int x = 0; x < p; x++) res.push_back({x, x});
      for (int x = 0; x < p; x++) res.push_back({x, p});
      for (int x = 0; x < p; x++) res.push_back({x, p + 1});
      if (!strict) res.push_back({p, p});
      res.push_back({p, p + 1});
      if (!strict) res.push_back({p + 1, p + 1});
      break;
    default: break;
  }
  return res;
}

// a+_{x s} / a_{x s} on the right side: block orbitals x > r, the site r
RF elem_r(int x, int r, int s2, bool dagger, double &coef) {
  RF f{x > r ? 0 : 1, F_C, dagger ? 0 : 1, 1, dagger ? s2 : -s2};
  if (!dagger && ((1 + s2) / 2) % 2) coef = -coef;
  return f;
}

// Terms of the enlarged right block R' = [r, n) (r = site_l + 1), a right
// block at bond site_l - 1: H restricted to [r, n) (S_r, P_rr, Q_rr of R for
// the parts with two or more indices in R), C, S_x, P_xy, Q_xy (x, y < r) --
// the mirror of build_terms with the site before the block.
int build_terms_right(const dmrg_problem_t &pr, const BlockModel &R, SiteAlgebra &site, int mask,
                      std::vector<RTerm> &terms, Error &err) {
  const int p = pr.site_l, n = pr.n_orb, r = p + 1;
  const int sp[2] = {1, -1};
  auto h = [&](int i, int j) { return pr.h1[(int64_t)i * n + j]; };
  auto v = [&](int i, int j, int k, int l) { return pr.eri[(((int64_t)i * n + j) * n + k) * n + l]; };
  auto direct = [&](int fam, int pos, int x, int y) -> bool {
    RTerm t;
    t.fam = fam; t.pos = pos;
    t.ta.kind = 1; t.ta.id = fam; t.ta.adj = 0; t.ta.k2 = FAM_TWO_K[fam]; t.ta.par = FAM_PAR[fam];
    t.posA = R.pos(fam, x, y);
    t.alpha = 1.0;
    if (t.posA < 0) { err = {DMRG_EINVAL, "right block lacks a member the enlarged block needs"}; return false; }
    terms.push_back(t);
    return true;
  };
  auto proj = [&](const std::vector<RProd> &pp, int fam, int pos, int x, int y) {
    return add_projected(pp, site, R, fam, pos, x, y, terms, err, 1);
  };
  for (int fam = 0; fam < N_FAM; fam++) {
    if (!(mask & (1 << fam))) continue;
    auto labs = right_labels(fam, p - 1, n);
    for (int pos = 0; pos < (int)labs.size(); pos++) {
      const int x = labs[pos][0], y = labs[pos][1];
      if (fam == F_H) {
        { std::vector<RProd> pp{{1.0, {famc(F_H, 0, 0)}}}; if (proj(pp, fam, pos, -1, -1)) return err.code; }
        {
          std::vector<RProd> pp;
          for (int s : sp) {
            RProd q;
            q.coef = -std::sqrt(2.0) * sgn2(1 + s);
            q.f.push_back(elem_r(r, r, s, true, q.coef));
            q.f.push_back(famc(F_S, 0, -s));
            pp.push_back(q);
          }
          for (size_t i = 0, m = pp.size(); i < m; i++) pp.push_back(adjoint(pp[i]));
          if (proj(pp, fam, pos, r, -1)) return err.code;
        }
        {
          std::vector<RProd> pp;
          for (int s : sp)
            for (int t : sp) {
              double cP = sgn2(2 + t + s) * cg(1, -t, 1, -s, 0, -t - s);
              if (cP == 0.0) continue;
              RProd q;
              q.coef = 0.5 * cP;
              q.f.push_back(elem_r(r, r, s, true, q.coef));
              q.f.push_back(elem_r(r, r, t, true, q.coef));
              q.f.push_back(famc(F_P0, 0, -t - s));
              pp.push_back(q);
            }
          for (size_t i = 0, m = pp.size(); i < m; i++) pp.push_back(adjoint(pp[i]));
          if (proj(pp, fam, pos, r, r)) return err.code;
        }
        {
          std::vector<RProd> pp;
          for (int s : sp)
            for (int t : sp) {
              std::vector<std::pair<double, RF>> parts;
              if (s == t) parts.push_back({-1.0 / std::sqrt(2.0), famc(F_Q0, 0, 0)});
              double c1 = cg(1, s, 1, -t, 2, s - t);
              if (c1 != 0.0) parts.push_back({-sgn2(1 + t) * c1 / std::sqrt(3.0), famc(F_Q1, 0, s - t)});
              for (auto &qp : parts) {
                RProd q;
                q.coef = qp.first;
                q.f.push_back(qp.second);
                q.f.push_back(elem_r(r, r, t, true, q.coef));
                q.f.push_back(elem_r(r, r, s, false, q.coef));
                pp.push_back(q);
              }
            }
          if (proj(pp, fam, pos, r, r)) return err.code;
        }
        for (int bi = -1; bi < n; bi++) {
          if (bi >= 0 && bi <= r) continue;
          auto in_inst = [&](std::initializer_list<int> idx) {
            int nb = 0, which = -1;
            for (int i : idx) if (i > r) { nb++; which = i; }
            return nb == (bi < 0 ? 0 : 1) && (bi < 0 || which == bi);
          };
          std::vector<RProd> pp;
          for (int i = r; i < n; i++)
            for (int j = r; j < n; j++) {
              if (!in_inst({i, j}) || h(i, j) == 0.0) continue;
              for (int s : sp) {
                RProd q;
                q.coef = h(i, j);
                q.f.push_back(elem_r(i, r, s, true, q.coef));
                q.f.push_back(elem_r(j, r, s, false, q.coef));
                pp.push_back(q);
              }
            }
          for (int i = r; i < n; i++)
            for (int j = r; j < n; j++)
              for (int k = r; k < n; k++)
                for (int l = r; l < n; l++) {
                  if (!in_inst({i, j, k, l}) || v(i, j, k, l) == 0.0) continue;
                  for (int s : sp)
                    for (int t : sp) {
                      if ((i == k || j == l) && s == t) continue;
                      RProd q;
                      q.coef = 0.5 * v(i, j, k, l);
                      q.f.push_back(elem_r(i, r, s, true, q.coef));
                      q.f.push_back(elem_r(k, r, t, true, q.coef));
                      q.f.push_back(elem_r(l, r, t, false, q.coef));
                      q.f.push_back(elem_r(j, r, s, false, q.coef));
                      pp.push_back(q);
                    }
                }
          if (pp.empty()) continue;
          if (proj(pp, fam, pos, bi, -1)) return err.code;
        }
        continue;
      }
      if (fam == F_C) {
        if (x > r) { if (!direct(fam, pos, x, -1)) return err.code; continue; }
        RProd q;
        q.coef = 1.0;
        q.f.push_back(elem_r(r, r, 1, true, q.coef));
        if (proj({q}, fam, pos, -1, -1)) return err.code;
        continue;
      }
      if (fam == F_S) {
        // (S_x)_s of R' (x < r): S_x of R + sum_t (P_xr)_ts a+_rt + sum_t (Q_xr)_st a_rt + explicit
        const double scale = -1.0 / std::sqrt(2.0);
        const int s = -1;
        if (!direct(fam, pos, x, -1)) return err.code;
        {
          std::vector<RProd> pp;
          for (int t : sp)
            for (int K = 0; K <= 2; K += 2) {
              double cP = sgn2(2 + t + s) * cg(1, -t, 1, -s, K, -t - s);
              if (cP == 0.0) continue;
              RProd q;
              q.coef = scale * cP;
              q.f.push_back(famc(K == 0 ? F_P0 : F_P1, 0, -t - s));
              q.f.push_back(elem_r(r, r, t, true, q.coef));
              pp.push_back(q);
            }
          if (proj(pp, fam, pos, x, r)) return err.code;
        }
        {
          std::vector<RProd> pp;
          for (int t : sp) {
            std::vector<std::pair<double, RF>> parts;   // (Q_xr)_st: t2 = s, s2 = t
            if (t == s) parts.push_back({-1.0 / std::sqrt(2.0), famc(F_Q0, 0, 0)});
            double c1 = cg(1, t, 1, -s, 2, t - s);
            if (c1 != 0.0) parts.push_back({-sgn2(1 + s) * c1 / std::sqrt(3.0), famc(F_Q1, 0, t - s)});
            for (auto &qp : parts) {
              RProd q;
              q.coef = scale * qp.first;
              q.f.push_back(qp.second);
              q.f.push_back(elem_r(r, r, t, false, q.coef));
              pp.push_back(q);
            }
          }
          if (proj(pp, fam, pos, x, r)) return err.code;
        }
        for (int bi = -1; bi < n; bi++) {
          if (bi >= 0 && bi <= r) continue;
          std::vector<RProd> pp;
          for (int j = r; j < n; j++)
            for (int k = r; k < n; k++)
              for (int l = r; l < n; l++) {
                int atr = (j == r) + (k == r) + (l == r);
                if (atr < 2 || v(x, j, k, l) == 0.0) continue;
                int which = j > r ? j : k > r ? k : l > r ? l : -1;
                if (which != bi) continue;
                for (int t : sp) {
                  RProd q;
                  q.coef = scale * v(x, j, k, l);
                  q.f.push_back(elem_r(k, r, t, true, q.coef));
                  q.f.push_back(elem_r(l, r, t, false, q.coef));
                  q.f.push_back(elem_r(j, r, s, false, q.coef));
                  pp.push_back(q);
                }
              }
          if (pp.empty()) continue;
          if (proj(pp, fam, pos, bi, -1)) return err.code;
        }
        continue;
      }
      // P^K / Q^K of R' for the pair (x, y), x, y < r
      if (!direct(fam, pos, x, y)) return err.code;
      const int K2 = FAM_TWO_K[fam];
      std::vector<std::array<double, 3>> ts;
      for (int t : sp)
        for (int s2 : sp) {
          if (fam == F_P0 || fam == F_P1) {
            if (-t - s2 == K2) ts.push_back({(double)t, (double)s2, cg(1, -t, 1, -s2, K2, K2) * sgn2(2 + t + s2)});
          } else if (fam == F_Q0) {
            if (t == s2) ts.push_back({(double)t, (double)s2, -1.0 / std::sqrt(2.0)});
          } else if (t == -1 && s2 == 1) {
            ts.push_back({(double)t, (double)s2, -std::sqrt(3.0)});
          }
        }
      for (int bi = -1; bi < n; bi++) {
        if (bi >= 0 && bi <= r) continue;
        auto inst = [&](int i1, int i2) {
          if (i1 > r && i2 > r) return false;
          int which = i1 > r ? i1 : i2 > r ? i2 : -1;
          return which == bi;
        };
        std::vector<RProd> pp;
        for (auto &w : ts) {
          const int t = (int)w[0], s2 = (int)w[1];
          for (int a = r; a < n; a++)
            for (int b = r; b < n; b++) {
              if (!inst(a, b)) continue;
              if (fam == F_P0 || fam == F_P1) {
                double vv = v(x, a, y, b);
                if (vv == 0.0) continue;
                RProd q;
                q.coef = w[2] * vv;
                q.f.push_back(elem_r(b, r, t, false, q.coef));
                q.f.push_back(elem_r(a, r, s2, false, q.coef));
                pp.push_back(q);
              } else {
                if (t == s2 && v(x, y, a, b) != 0.0)
                  for (int sg : sp) {
                    RProd q;
                    q.coef = w[2] * v(x, y, a, b);
                    q.f.push_back(elem_r(a, r, sg, true, q.coef));
                    q.f.push_back(elem_r(b, r, sg, false, q.coef));
                    pp.push_back(q);
                  }
                if (v(x, b, a, y) != 0.0) {
                  RProd q;
                  q.coef = -w[2] * v(x, b, a, y);
                  q.f.push_back(elem_r(a, r, s2, true, q.coef));
                  q.f.push_back(elem_r(b, r, t, false, q.coef));
                  pp.push_back(q);
                }
              }
            }
        }
        if (pp.empty()) continue;
        if (proj(pp, fam, pos, bi, -1)) return err.code;
      }
    }
  }
  return DMRG_OK;
}

struct RComp { int lsec, site, row0, dim; };
struct RSec {
  int n, two_s, rows;
  std::vector<RComp> comps;
};

// right side: components (site multiplet, block sector) with the site outer
std::vector<RSec> product_sectors_right(const std::vector<dmrg_sector_t> &bsec) {
  std::map<std::pair<int, int>, RSec> m;
  for (int s = 0; s < 3; s++)
    for (int a = 0; a < (int)bsec.size(); a++)
      for (int S = std::abs(bsec[a].two_s - RSITE_S[s]); S <= bsec[a].two_s + RSITE_S[s]; S += 2) {
        auto &r = m[{bsec[a].n + RSITE_N[s], S}];
        r.n = bsec[a].n + RSITE_N[s];
        r.two_s = S;
        r.comps.push_back({a, s, r.rows, bsec[a].dim});
        r.rows += bsec[a].dim;
      }
  std::vector<RSec> out;
  for (auto &kv : m) out.push_back(kv.second);
  return out;
}

std::vector<RSec> product_sectors(const std::vector<dmrg_sector_t> &lsec) {
  std::map<std::pair<int, int>, RSec> m;
  for (int a = 0; a < (int)lsec.size(); a++)
    for (int s = 0; s < 3; s++)
      for (int S = std::abs(lsec[a].two_s - RSITE_S[s]); S <= lsec[a].two_s + RSITE_S[s]; S += 2) {
        auto &r = m[{lsec[a].n + RSITE_N[s], S}];
        r.n = lsec[a].n + RSITE_N[s];
        r.two_s = S;
        r.comps.push_back({a, s, r.rows, lsec[a].dim});
        r.rows += lsec[a].dim;
      }
  std::vector<RSec> out;
  for (auto &kv : m) out.push_back(kv.second);
  return out;
}

struct Built {
  std::vector<dmrg_oprec_t> recs;
  int64_t out_len = 0;
  std::vector<Tile> t1, t2;
  std::vector<Seg> s1, s2;
  XcdQueues q1{}, q2{};
  int64_t work_len = 0;
  std::vector<TransJob> ujobs;   // U -> U^T per kept sector (every apply)
  std::vector<TransJob> ljobs;   // left records used as adjoints -> transposed copy (once)
  std::vector<DressItem> ditems; // dressed operators (once, after the transposed copy)
  std::vector<int64_t> dsrc;     // their source offsets ...
  std::vector<double> dalpha;    // ... and weights
  int64_t dress_len = 0;
  int64_t n_terms = 0;
  double flops1 = 0.0, flops2 = 0.0;
  double build_ms = 0.0;
};

// The left block in the catalogue form (build_block) or, with all_pairs,
// with P and Q over every outside pair: the other families are read as
// usual and P, Q are checked and indexed here.
int build_left(BlockModel &L, const dmrg_problem_t &pr, bool all_pairs, Error &err) {
  if (!all_pairs) return build_block(L, 0, pr, err);
  auto is_pq = [](int f) { return f == F_P0 || f == F_P1 || f == F_Q0 || f == F_Q1; };
  std::vector<dmrg_oprec_t> other, pq;
  for (int64_t i = 0; i < pr.n_lrec; i++) (is_pq(pr.lrec[i].fam) ? pq : other).push_back(pr.lrec[i]);
  dmrg_problem_t p2 = pr;
  p2.lrec = other.data();
  p2.n_lrec = (int64_t)other.size();
  if (build_block(L, 0, p2, err)) return err.code;
  for (int f : {F_P0, F_P1, F_Q0, F_Q1}) {
    L.labels[f] = left_labels(f, pr.site_l, pr.n_orb);
    L.label_pos[f].clear();
    for (size_t i = 0; i < L.labels[f].size(); i++) L.label_pos[f][L.labels[f][i]] = (int)i;
  }
  for (const dmrg_oprec_t &r : pq) {
    const int ns = (int)L.sec.size();
    if (r.row_sec < 0 || r.row_sec >= ns || r.col_sec < 0 || r.col_sec >= ns) {
      err = {DMRG_EINVAL, "operator record with bad family or sector"};
      return err.code;
    }
    if (r.npos != (int)L.labels[r.fam].size()) {
      err = {DMRG_EINVAL, "record npos differs from the all-pairs label count"};
      return err.code;
    }
    const auto &sr = L.sec[r.row_sec], &sc = L.sec[r.col_sec];
    const int k2 = FAM_TWO_K[r.fam];
    if (sr.n != sc.n + FAM_DN[r.fam] || sr.two_s < std::abs(sc.two_s - k2) || sr.two_s > sc.two_s + k2) {
      err = {DMRG_ESYM, "operator record violates N or spin selection rules"};
      return err.code;
    }
    if (r.off < 0 || r.off + (int64_t)r.npos * sr.dim * sc.dim > L.data_len) {
      err = {DMRG_ERANGE, "operator record beyond its data array"};
      return err.code;
    }
    const int64_t key = ((int64_t)r.fam * 1000003 + r.row_sec) * 1000003 + r.col_sec;
    if (L.rec_index.count(key)) { err = {DMRG_EINVAL, "duplicate operator record"}; return err.code; }
    L.rec_index[key] = (int)L.rec.size();
    L.rec.push_back(r);
  }
  return DMRG_OK;
}

int build_renorm(const dmrg_problem_t *prob, const dmrg_rkeep_t *keep, int n_keep, int mask, int flags,
                 int64_t u_len, Built &B, Error &err) {
  auto t0 = std::chrono::steady_clock::now();
  if (!prob || !keep || n_keep <= 0) { err = {DMRG_EINVAL, "null problem or empty keep list"}; return err.code; }
  const dmrg_problem_t &pr = *prob;
  if (pr.site_l < 1 || pr.site_l + 1 > pr.n_orb || !pr.h1 || !pr.eri) {
    err = {DMRG_EINVAL, "renormalization needs a non-empty left block, the site and the integrals"};
    return err.code;
  }
  const bool all_pairs = flags & RENORM_ALL_PAIRS;
  const bool right = flags & RENORM_RIGHT;
  if (flags & ~(RENORM_ALL_PAIRS | RENORM_RIGHT) || (right && all_pairs)) {
    err = {DMRG_EINVAL, "unknown renormalization flag or combination"};
    return err.code;
  }
  if (right && pr.site_l + 2 >= pr.n_orb) {
    err = {DMRG_EINVAL, "renormalization of the right block needs a non-empty right block"};
    return err.code;
  }
  const int allowed = right ? RENORM_RIGHT_MASK : RENORM_DEFAULT_MASK | (all_pairs ? RENORM_PAIR_MASK : 0);
  if (mask == 0) mask = allowed;
  if (mask & ~allowed) {
    err = {DMRG_EINVAL, all_pairs ? "unknown family in the mask"
                                  : "P and Q of the enlarged block need a left block with all outside pairs"};
    return err.code;
  }
  const int n4 = pr.n_orb;
  for (int64_t i = 0; i < (int64_t)n4 * n4; i++)
    if (!std::isfinite(pr.h1[i])) { err = {DMRG_ENONFINITE, "non-finite one-electron integral"}; return err.code; }
  for (int64_t i = 0; i < (int64_t)n4 * n4 * n4 * n4; i++)
    if (!std::isfinite(pr.eri[i])) { err = {DMRG_ENONFINITE, "non-finite two-electron integral"}; return err.code; }
  // L: the block being enlarged (the right block with RENORM_RIGHT)
  BlockModel L;
  if (right ? build_block(L, 1, pr, err) : build_left(L, pr, all_pairs, err)) return err.code;
  const int64_t blen = right ? pr.rdata_len : pr.ldata_len;
  SiteAlgebra site;
  std::vector<RTerm> terms;
  if (right ? build_terms_right(pr, L, site, mask, terms, err) : build_terms(pr, L, site, mask, terms, err))
    return err.code;
  // Dressing: terms that differ only in the position of their C factor (a
  // sum over an orbital j with integral weights, e.g. sum_j (xj|yl) C~_j (x)
  // a~_l in P_xy) are merged into one term on sum_j alpha_j C_j, formed once
  // when the lists are created (the dressing H.psi applies to its right-block
  // rows); the products then run once per merged term instead of once per j.
  std::vector<DressG> dress;
  {
    struct DK {
      int fam, pos, adj;
      PT tb;
      bool operator<(const DK &o) const {
        if (std::tie(fam, pos, adj) != std::tie(o.fam, o.pos, o.adj)) return std::tie(fam, pos, adj) < std::tie(o.fam, o.pos, o.adj);
        return tb < o.tb;
      }
    };
    std::map<DK, std::vector<int>> groups;
    for (int i = 0; i < (int)terms.size(); i++) {
      const RTerm &t = terms[i];
      if (t.ta.kind == 1 && t.ta.id == F_C) groups[{t.fam, t.pos, t.ta.adj, t.tb}].push_back(i);
    }
    std::vector<char> drop(terms.size(), 0);
    std::vector<RTerm> merged;
    for (auto &kv : groups) {
      if (kv.second.size() < 2) continue;
      DressG g;
      g.adj = kv.first.adj;
      for (int i : kv.second) {
        g.src.push_back({terms[i].posA, terms[i].alpha});
        drop[i] = 1;
      }
      RTerm t = terms[kv.second[0]];
      t.alpha = 1.0;
      t.posA = 0;
      t.dress = (int)dress.size();
      dress.push_back(g);
      merged.push_back(t);
    }
    std::vector<RTerm> kept_terms;
    for (size_t i = 0; i < terms.size(); i++)
      if (!drop[i]) kept_terms.push_back(terms[i]);
    for (auto &t : merged) kept_terms.push_back(t);
    terms.swap(kept_terms);
  }
  B.n_terms = (int64_t)terms.size();
  std::vector<RSec> prod = right ? product_sectors_right(L.sec) : product_sectors(L.sec);
  std::map<std::pair<int, int>, int> pidx;
  for (int i = 0; i < (int)prod.size(); i++) pidx[{prod[i].n, prod[i].two_s}] = i;
  std::vector<int> kp(n_keep);
  std::vector<int> used(prod.size(), 0);
  for (int k = 0; k < n_keep; k++) {
    auto it = pidx.find({keep[k].n, keep[k].two_s});
    if (it == pidx.end()) { err = {DMRG_ESYM, "kept sector is not a product sector of the block and the site"}; return err.code; }
    if (used[it->second]++) { err = {DMRG_EINVAL, "kept sector listed twice"}; return err.code; }
    const RSec &ps = prod[it->second];
    if (keep[k].kept <= 0 || keep[k].kept > ps.rows) { err = {DMRG_EINVAL, "kept dimension outside [1, product rows]"}; return err.code; }
    if (keep[k].u_off < 0 || keep[k].u_off + (int64_t)ps.rows * keep[k].kept > u_len) {
      err = {DMRG_ERANGE, "truncation matrix beyond its array"};
      return err.code;
    }
    kp[k] = it->second;
  }
  // contributions: output (fam, pos, bra kept, ket kept) <- sum coef Ub^T T
  struct OKey {
    int fam, bk, ak, pos;
    bool operator<(const OKey &o) const { return std::tie(fam, bk, ak, pos) < std::tie(o.fam, o.bk, o.ak, o.pos); }
  };
  struct TKey {
    int rec, posA, adj, ak, ac;
    bool operator<(const TKey &o) const {
      return std::tie(rec, posA, adj, ak, ac) < std::tie(o.rec, o.posA, o.adj, o.ak, o.ac);
    }
  };
  struct CKey {
    int tix, ak, ac, bk, bc;   // tix >= 0: stage-1 product; < 0: U rows of (ak, ac) directly
    bool operator<(const CKey &o) const { return std::tie(tix, ak, ac, bk, bc) < std::tie(o.tix, o.ak, o.ac, o.bk, o.bc); }
  };
  std::map<TKey, int> tindex;
  std::vector<TKey> tkeys;
  std::map<OKey, std::map<CKey, double>> contrib;
  CtildeTable wl;
  for (const RTerm &t : terms) {
    const int K = FAM_TWO_K[t.fam], dN = FAM_DN[t.fam];
    const int kA = t.ta.kind ? t.ta.k2 : 0, kB = t.tb.kind ? t.tb.k2 : 0;
    for (int ak = 0; ak < n_keep; ak++)
      for (int bk = 0; bk < n_keep; bk++) {
        const RSec &pa = prod[kp[ak]], &pb = prod[kp[bk]];
        if (pb.n != pa.n + dN || pb.two_s < std::abs(pa.two_s - K) || pb.two_s > pa.two_s + K) continue;
        for (int ac = 0; ac < (int)pa.comps.size(); ac++)
          for (int bc = 0; bc < (int)pb.comps.size(); bc++) {
            const RComp &ca = pa.comps[ac], &cb = pb.comps[bc];
            double sv = 1.0;
            if (t.tb.kind == 0) {
              if (ca.site != cb.site) continue;
            } else {
              sv = site.fams[t.tb.id].red[cb.site][ca.site];
              if (sv == 0.0) continue;
            }
            int rec = -1;
            double ph = 1.0;
            const int Sa = L.sec[ca.lsec].two_s, Sb = L.sec[cb.lsec].two_s;
            if (t.ta.kind == 0) {
              if (ca.lsec != cb.lsec) continue;
            } else if (!t.ta.adj) {
              rec = L.find_rec(t.ta.id, cb.lsec, ca.lsec);
            } else {
              rec = L.find_rec(t.ta.id, ca.lsec, cb.lsec);
              ph = sgn2(Sa + t.ta.k2 - Sb) * std::sqrt((Sa + 1.0) / (Sb + 1.0));
            }
            if (t.ta.kind && rec < 0) continue;
            // Eq. (4) factor in the W9j(l) role (block x site) or the W9j(r)
            // role (site x block); Jordan-Wigner sign of the later factor
            // passing the earlier part of the ket
            double c, sgn;
            if (!right) {
              c = wl.get(Sa, RSITE_S[ca.site], pa.two_s, kA, kB, K, Sb, RSITE_S[cb.site], pb.two_s);
              sgn = (t.tb.kind && t.tb.par && (L.sec[ca.lsec].n % 2)) ? -1.0 : 1.0;
            } else {
              c = wl.get(RSITE_S[ca.site], Sa, pa.two_s, kB, kA, K, RSITE_S[cb.site], Sb, pb.two_s);
              sgn = (t.ta.kind && t.ta.par && (RSITE_N[ca.site] % 2)) ? -1.0 : 1.0;
            }
            if (c == 0.0) continue;
            double coef = t.alpha * sv * c * sgn * ph;
            if (std::fabs(coef) < 1e-300) continue;
            int tix = -1;
            if (rec >= 0) {
              TKey tk{rec, t.dress >= 0 ? -1 - t.dress : t.posA, t.ta.adj, ak, ac};
              auto it = tindex.find(tk);
              if (it == tindex.end()) {
                it = tindex.emplace(tk, (int)tkeys.size()).first;
                tkeys.push_back(tk);
              }
              tix = it->second;
            }
            contrib[{t.fam, bk, ak, t.pos}][{tix, tix >= 0 ? -1 : ak, tix >= 0 ? -1 : ac, bk, bc}] += coef;
          }
      }
  }
  // output records: every (family, bra, ket) with a contribution, all positions
  std::map<std::array<int, 3>, int64_t> rec_off;
  for (auto &kv : contrib) rec_off[{kv.first.fam, kv.first.bk, kv.first.ak}] = 0;
  B.recs.clear();
  B.out_len = 0;
  for (auto &kv : rec_off) {
    dmrg_oprec_t r;
    r.fam = kv.first[0];
    r.row_sec = kv.first[1];
    r.col_sec = kv.first[2];
    r.npos = (int32_t)(right ? right_labels(r.fam, pr.site_l - 1, pr.n_orb) : left_labels(r.fam, pr.site_l + 1, pr.n_orb)).size();
    r.off = B.out_len;
    kv.second = B.out_len;
    B.out_len += (int64_t)r.npos * keep[r.row_sec].kept * keep[r.col_sec].kept;
    B.recs.push_back(r);
  }
  auto kept = [&](int k) { return keep[k].kept; };
  auto prows = [&](int k) { return prod[kp[k]].rows; };
  auto comp = [&](int k, int c) -> const RComp & { return prod[kp[k]].comps[c]; };
  // stage 1: T = op(A) U_a'[rows of the ket component]
  std::vector<int64_t> toff(tkeys.size());
  B.t1.clear(); B.s1.clear(); B.t2.clear(); B.s2.clear();
  std::vector<double> cost1, cost2;
  B.work_len = 0;
  B.flops1 = B.flops2 = 0.0;
  auto add_tiles = [&](std::vector<Tile> &tiles, std::vector<double> &cost, int m, int n, int c_base,
                       int64_t c_off, int64_t ldc, int seg0, int nseg, double ksum, int rowmajor) {
    const int mb = tile_mb(m, n), tr = tile_rows(mb), tc = tile_cols(mb);
    for (int i0 = 0; i0 < m; i0 += tr)
      for (int j0 = 0; j0 < n; j0 += tc) {
        Tile T{};
        T.c_off = c_off; T.ldc = ldc; T.c_base = c_base;
        T.m = m; T.n = n; T.i0 = i0; T.j0 = j0; T.ci0 = i0; T.cj0 = j0;
        T.mb = mb; T.seg0 = seg0; T.nseg = nseg; T.accumulate = 0; T.rowmajor = rowmajor;
        tiles.push_back(T);
        cost.push_back((double)std::min(tr, m - i0) * std::min(tc, n - j0) * ksum);
      }
  };
  // Operand layouts that let every wavefront load whole lines (lanes run
  // along output rows of A and along output columns of B): U is read from
  // its per-sector transpose U^T (kept x rows, column-major), adjoint left
  // members from a transposed copy of their records, and T is stored
  // row-major (ket kept states fastest).
  std::vector<char> ladj(L.rec.size(), 0);
  for (const TKey &k : tkeys)
    if (k.adj) ladj[k.rec] = 1;
  // dressed operators: one block per C record per group, from the records
  // (or their transposed copies for adjoint groups)
  std::vector<int> crec;
  for (size_t i = 0; i < L.rec.size(); i++)
    if (L.rec[i].fam == F_C) crec.push_back((int)i);
  std::vector<int64_t> crec_off(L.rec.size(), -1);
  int64_t csize = 0;
  for (int i : crec) {
    crec_off[i] = csize;
    csize += (int64_t)L.sec[L.rec[i].row_sec].dim * L.sec[L.rec[i].col_sec].dim;
  }
  B.ditems.clear(); B.dsrc.clear(); B.dalpha.clear();
  B.dress_len = csize * (int64_t)dress.size();
  for (size_t g = 0; g < dress.size(); g++) {
    for (int i : crec) {
      const dmrg_oprec_t &r = L.rec[i];
      const int64_t bs = (int64_t)L.sec[r.row_sec].dim * L.sec[r.col_sec].dim;
      if (dress[g].adj) ladj[i] = 1;
      DressItem d{};
      d.dst_off = (int64_t)g * csize + crec_off[i];
      d.n = bs;
      d.t0 = (int32_t)B.dsrc.size();
      for (auto &sa : dress[g].src) {
        B.dsrc.push_back(r.off + (int64_t)sa.first * bs);
        B.dalpha.push_back(sa.second);
      }
      d.t1 = (int32_t)B.dsrc.size();
      d.src_base = dress[g].adj ? BASE_OPS + 1 : BASE_OPS;
      d.dst_base = BASE_OPS + 2;
      B.ditems.push_back(d);
    }
  }
  B.ljobs.clear();
  for (size_t i = 0; i < L.rec.size(); i++)
    if (ladj[i]) {
      const dmrg_oprec_t &r = L.rec[i];
      B.ljobs.push_back(TransJob{r.off, L.sec[r.row_sec].dim, L.sec[r.col_sec].dim, r.npos, 0});
    }
  B.ujobs.clear();
  for (int k = 0; k < n_keep; k++) B.ujobs.push_back(TransJob{keep[k].u_off, prows(k), kept(k), 1, 0});
  for (size_t i = 0; i < tkeys.size(); i++) {
    const TKey &k = tkeys[i];
    const dmrg_oprec_t &r = L.rec[k.rec];
    const int rr = L.sec[r.row_sec].dim, rc = L.sec[r.col_sec].dim;
    const int m = k.adj ? rc : rr, K = k.adj ? rr : rc, n = kept(k.ak);
    const RComp &ca = comp(k.ak, k.ac);
    Seg S{};
    if (k.posA >= 0) {
      S.a_base = k.adj ? BASE_OPS + 1 : BASE_OPS;
      S.a_off = r.off + (int64_t)k.posA * rr * rc;
    } else {                        // dressed operator -1 - posA, same orientation
      S.a_base = BASE_OPS + 2;
      S.a_off = (int64_t)(-1 - k.posA) * csize + crec_off[k.rec];
    }
    S.a_i = 1;
    S.a_k = k.adj ? rc : rr;       // the transposed record is rc x rr
    S.a_p = 0;
    S.a_kb = K;
    S.b_base = BASE_PSI;            // U^T: element (c, r) at u_off + c + r * kept
    S.b_off = keep[k.ak].u_off + (int64_t)ca.row0 * n;
    S.b_k = n; S.b_n = 1; S.b_kb = K; S.b_nb = n; S.b_pk = 0; S.b_pn = 0;
    S.K = K;
    S.s = 1.0;
    toff[i] = B.work_len;
    int seg0 = (int)B.s1.size();
    B.s1.push_back(S);
    add_tiles(B.t1, cost1, m, n, BASE_WORK, toff[i], n, seg0, 1, K, 1);
    B.work_len += (int64_t)m * n;
    B.flops1 += 2.0 * m * n * K;
  }
  // stage 2: O'(b', a')[pos] = sum coef U_b'[rows]^T T
  for (auto &kv : contrib) {
    const OKey &o = kv.first;
    const int m = kept(o.bk), n = kept(o.ak);
    int seg0 = (int)B.s2.size();
    double ksum = 0.0;
    for (auto &cv : kv.second) {
      const CKey &c = cv.first;
      const RComp &cb = comp(c.bk, c.bc);
      Seg S{};
      S.a_base = BASE_PSI;          // U_b'^T rows block: A(i, k) = U^T[i + (row0 + k) kept_b']
      S.a_off = keep[c.bk].u_off + (int64_t)cb.row0 * m;
      S.a_i = 1;
      S.a_k = m;
      S.a_p = 0;
      S.K = cb.dim;
      S.a_kb = S.K;
      if (c.tix >= 0) {             // T row-major, d_b x kept_a'
        S.b_base = BASE_WORK;
        S.b_off = toff[c.tix];
      } else {                      // identity left factor: U_a'^T rows block
        S.b_base = BASE_PSI;
        S.b_off = keep[c.ak].u_off + (int64_t)comp(c.ak, c.ac).row0 * n;
      }
      S.b_k = n;
      S.b_n = 1;
      S.b_kb = S.K; S.b_nb = n; S.b_pk = 0; S.b_pn = 0;
      S.s = cv.second;
      B.s2.push_back(S);
      ksum += S.K;
      B.flops2 += 2.0 * m * n * S.K;
    }
    const int64_t off = rec_off[{o.fam, o.bk, o.ak}] + (int64_t)o.pos * m * n;
    add_tiles(B.t2, cost2, m, n, BASE_Y, off, m, seg0, (int)B.s2.size() - seg0, ksum, 0);
  }
  // every element a kernel lane may touch lies inside its array (lanes past
  // the tile or K read inside the operand: row 0, column 0, element K - 1)
  auto inside = [&](const std::vector<Tile> &tiles, const std::vector<Seg> &segs) {
    auto len = [&](int base) { return base == BASE_PSI ? u_len : base == BASE_Y ? B.out_len
                                    : base == BASE_WORK ? B.work_len : base == BASE_OPS + 2 ? B.dress_len
                                    : blen; };
    for (const Tile &T : tiles) {
      const int64_t last = T.rowmajor ? (int64_t)(T.m - 1) * T.ldc + (T.n - 1) : (T.m - 1) + (int64_t)(T.n - 1) * T.ldc;
      if (T.c_off < 0 || T.c_off + last >= len(T.c_base)) return false;
      for (int i = 0; i < T.nseg; i++) {
        const Seg &S = segs[T.seg0 + i];
        if (S.K <= 0 || S.a_off < 0 || S.b_off < 0) return false;
        if (S.a_off + (int64_t)(T.m - 1) * S.a_i + (int64_t)(S.K - 1) * S.a_k >= len(S.a_base)) return false;
        if (S.b_off + (int64_t)(S.K - 1) * S.b_k + (int64_t)(T.n - 1) * S.b_n >= len(S.b_base)) return false;
      }
    }
    return true;
  };
  if (!inside(B.t1, B.s1) || !inside(B.t2, B.s2)) {
    err = {DMRG_ERANGE, "internal: a product reaches beyond its array"};
    return err.code;
  }
  // cost-sorted lists, cut into per-XCD ranges
  auto sort_list = [](std::vector<Tile> &tiles, std::vector<double> &cost) {
    std::vector<int> ord(tiles.size());
    for (size_t i = 0; i < ord.size(); i++) ord[i] = (int)i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<Tile> t2(tiles.size());
    std::vector<double> c2(tiles.size());
    for (size_t i = 0; i < ord.size(); i++) { t2[i] = tiles[ord[i]]; c2[i] = cost[ord[i]]; }
    tiles.swap(t2);
    cost.swap(c2);
  };
  sort_list(B.t1, cost1);
  sort_list(B.t2, cost2);
  B.q1 = equal_cost_ranges(cost1);
  B.q2 = equal_cost_ranges(cost2);
  B.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return DMRG_OK;
}

// host execution of a tile list with the kernels' addressing (test path)
void host_run(const std::vector<Tile> &tiles, const std::vector<Seg> &segs, const double *ops, const double *opsT,
              const double *dressed, const double *u, double *out, double *work) {
  auto base = [&](int id) -> const double * {
    return id == BASE_PSI ? u : id == BASE_Y ? out : id == BASE_WORK ? work : id == BASE_OPS ? ops
         : id == BASE_OPS + 1 ? opsT : dressed;
  };
  for (const Tile &T : tiles) {
    const int mt = std::min(tile_rows(T.mb), T.m - T.i0), nt = std::min(tile_cols(T.mb), T.n - T.j0);
    std::vector<double> acc((size_t)mt * nt, 0.0);
    for (int si = 0; si < T.nseg; si++) {
      const Seg &S = segs[T.seg0 + si];
      const double *A = base(S.a_base) + S.a_off, *Bp = base(S.b_base) + S.b_off;
      for (int j = 0; j < nt; j++)
        for (int i = 0; i < mt; i++) {
          double a = 0.0;
          for (int k = 0; k < S.K; k++)
            a += A[(int64_t)(T.i0 + i) * S.a_i + (int64_t)k * S.a_k] * Bp[(int64_t)k * S.b_k + (int64_t)(T.j0 + j) * S.b_n];
          acc[i + (size_t)j * mt] += S.s * a;
        }
    }
    double *C = const_cast<double *>(base(T.c_base)) + T.c_off;
    for (int j = 0; j < nt; j++)
      for (int i = 0; i < mt; i++)
        C[T.rowmajor ? (int64_t)(T.ci0 + i) * T.ldc + (T.cj0 + j) : (int64_t)(T.ci0 + i) + (int64_t)(T.cj0 + j) * T.ldc] =
            acc[i + (size_t)j * mt];
  }
}

// dst block (c, r) = src block (r, c) for every job (the transpose kernel's rule)
void host_transpose(const std::vector<TransJob> &jobs, const double *src, double *dst) {
  for (const TransJob &J : jobs) {
    const int64_t bs = (int64_t)J.rows * J.cols;
    for (int p = 0; p < J.npos; p++)
      for (int c = 0; c < J.cols; c++)
        for (int r = 0; r < J.rows; r++) dst[J.off + p * bs + c + (int64_t)r * J.cols] = src[J.off + p * bs + r + (int64_t)c * J.rows];
  }
}

}  // namespace

struct dmrg_renorm {
  Built b;
  const double *ldata = nullptr;
  Tile *d_t1 = nullptr, *d_t2 = nullptr;
  Seg *d_s1 = nullptr, *d_s2 = nullptr;
  TransJob *d_uj = nullptr, *d_lj = nullptr;
  const double **d_bases = nullptr;
  int32_t *d_cnt = nullptr;
  double *d_work = nullptr, *d_ut = nullptr, *d_lt = nullptr, *d_dress = nullptr;
  DressItem *d_di = nullptr;
  int64_t *d_dsrc = nullptr;
  double *d_dalpha = nullptr;
  int64_t u_len = 0;
  // profiling: an event pair around each stage launch of every apply
  bool prof = false;
  std::vector<hipEvent_t> ev;      // 4 per recorded apply
};

extern "C" void dmrg_renorm_free(dmrg_renorm_t *r) {
  if (!r) return;
  for (hipEvent_t e : r->ev) (void)hipEventDestroy(e);
  void *ptrs[] = {r->d_t1, r->d_t2, r->d_s1, r->d_s2, r->d_uj, r->d_lj, (void *)r->d_bases, r->d_cnt,
                  r->d_work, r->d_ut, r->d_lt, r->d_dress, r->d_di, r->d_dsrc, r->d_dalpha};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete r;
}

extern "C" int dmrg_renorm_product(const dmrg_problem_t *prob, int32_t flags, dmrg_sector_t *sec, int32_t sec_cap,
                                   int32_t *n_sec, dmrg_rcomp_t *comp, int32_t comp_cap, int32_t *n_comp) {
  const bool right = flags & RENORM_RIGHT;
  const int ns = prob ? (right ? prob->n_rsec : prob->n_lsec) : 0;
  const dmrg_sector_t *bs = prob ? (right ? prob->rsec : prob->lsec) : nullptr;
  if (!prob || !n_sec || !n_comp || ns <= 0 || !bs) {
    set_error("null argument or empty sector table");
    return DMRG_EINVAL;
  }
  std::vector<dmrg_sector_t> ls(bs, bs + ns);
  std::vector<RSec> prod = right ? product_sectors_right(ls) : product_sectors(ls);
  *n_sec = (int32_t)prod.size();
  int32_t nc = 0;
  for (int i = 0; i < (int)prod.size(); i++) {
    if (sec && i < sec_cap) sec[i] = dmrg_sector_t{prod[i].n, prod[i].two_s, prod[i].rows};
    for (const RComp &c : prod[i].comps) {
      if (comp && nc < comp_cap) comp[nc] = dmrg_rcomp_t{i, c.lsec, c.site, c.row0, c.dim, 0};
      nc++;
    }
  }
  *n_comp = nc;
  if ((sec && *n_sec > sec_cap) || (comp && nc > comp_cap)) {
    set_error("output arrays too small");
    return DMRG_ERANGE;
  }
  return DMRG_OK;
}

extern "C" int dmrg_renorm_create(const dmrg_problem_t *prob, const dmrg_rkeep_t *keep, int32_t n_keep,
                                  int32_t fam_mask, int32_t flags, int64_t u_len, dmrg_renorm_t **out) {
  if (!out) { set_error("null output"); return DMRG_EINVAL; }
  *out = nullptr;
  try {
    auto r = std::make_unique<dmrg_renorm>();
    Error err{0, ""};
    if (build_renorm(prob, keep, n_keep, fam_mask, flags, u_len, r->b, err)) { set_error(err.msg); return err.code; }
    const bool right = flags & RENORM_RIGHT;
    const double *bdata = right ? prob->rdata : prob->ldata;
    const int64_t blen = right ? prob->rdata_len : prob->ldata_len;
    if (!bdata) { set_error("operator data of the block missing"); return DMRG_EINVAL; }
    r->ldata = bdata;
    auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
      if (bytes == 0) bytes = 16;
      if (hipMalloc(dst, bytes) != hipSuccess) return false;
      return !src || hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    r->u_len = u_len;
    bool ok = up((void **)&r->d_ut, nullptr, (size_t)u_len * sizeof(double)) &&
              up((void **)&r->d_lt, nullptr, r->b.ljobs.empty() ? 0 : (size_t)blen * sizeof(double)) &&
              up((void **)&r->d_uj, r->b.ujobs.data(), r->b.ujobs.size() * sizeof(TransJob)) &&
              up((void **)&r->d_lj, r->b.ljobs.data(), r->b.ljobs.size() * sizeof(TransJob));
    ok = ok && up((void **)&r->d_dress, nullptr, (size_t)r->b.dress_len * sizeof(double)) &&
         up((void **)&r->d_di, r->b.ditems.data(), r->b.ditems.size() * sizeof(DressItem)) &&
         up((void **)&r->d_dsrc, r->b.dsrc.data(), r->b.dsrc.size() * sizeof(int64_t)) &&
         up((void **)&r->d_dalpha, r->b.dalpha.data(), r->b.dalpha.size() * sizeof(double));
    const double *bases[3] = {bdata, r->d_lt, r->d_dress};
    ok = ok && up((void **)&r->d_t1, r->b.t1.data(), r->b.t1.size() * sizeof(Tile)) &&
              up((void **)&r->d_t2, r->b.t2.data(), r->b.t2.size() * sizeof(Tile)) &&
              up((void **)&r->d_s1, r->b.s1.data(), r->b.s1.size() * sizeof(Seg)) &&
              up((void **)&r->d_s2, r->b.s2.data(), r->b.s2.size() * sizeof(Seg)) &&
              up((void **)&r->d_bases, bases, sizeof(bases)) &&
              up((void **)&r->d_cnt, nullptr, QUEUE_INTS * sizeof(int32_t)) &&
              up((void **)&r->d_work, nullptr, (size_t)r->b.work_len * sizeof(double));
    if (!ok) {
      dmrg_renorm_free(r.release());
      set_error("device allocation or copy failed");
      return DMRG_ENOMEM;
    }
    // transposed copies of the left records applied as adjoints, then the
    // dressed operators (once)
    if (!r->b.ljobs.empty() || !r->b.ditems.empty()) {
      launch_transpose(r->d_lj, (int)r->b.ljobs.size(), bdata, r->d_lt, nullptr);
      launch_dress(r->d_di, (int)r->b.ditems.size(), r->d_dsrc, r->d_dalpha, r->d_bases, r->d_dress, nullptr);
      if (hipStreamSynchronize(nullptr) != hipSuccess) {
        dmrg_renorm_free(r.release());
        set_error("transposing or dressing the left records failed");
        return DMRG_EHIP;
      }
    }
    *out = r.release();
    return DMRG_OK;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return DMRG_ENOMEM;
  } catch (...) {
    set_error("internal error");
    return DMRG_EINVAL;
  }
}

extern "C" int dmrg_renorm_records(const dmrg_renorm_t *r, dmrg_oprec_t *rec, int64_t cap, int64_t *n_rec,
                                   int64_t *data_len) {
  if (!r || !n_rec || !data_len) { set_error("null argument"); return DMRG_EINVAL; }
  *n_rec = (int64_t)r->b.recs.size();
  *data_len = r->b.out_len;
  if (rec) {
    if (cap < *n_rec) { set_error("record array too small"); return DMRG_ERANGE; }
    std::memcpy(rec, r->b.recs.data(), r->b.recs.size() * sizeof(dmrg_oprec_t));
  }
  return DMRG_OK;
}

extern "C" int dmrg_renorm_apply(dmrg_renorm_t *r, const double *u, double *out, void *stream) {
  if (!r || !u || !out) { set_error("null argument"); return DMRG_EINVAL; }
  hipEvent_t ev[4] = {};
  if (r->prof) {
    for (auto &x : ev)
      if (hipEventCreate(&x) != hipSuccess) { set_error("hipEventCreate failed"); return DMRG_EHIP; }
  }
  hipStream_t hs = (hipStream_t)stream;
  launch_transpose(r->d_uj, (int)r->b.ujobs.size(), u, r->d_ut, stream);
  launch_zero(out, r->b.out_len, stream);
  if (r->prof) (void)hipEventRecord(ev[0], hs);
  launch_tiles_f64(1, r->d_t1, r->d_s1, (int)r->b.t1.size(), r->b.q1, r->d_cnt, r->d_bases, r->d_ut, out,
                   r->d_work, nullptr, stream);
  if (r->prof) { (void)hipEventRecord(ev[1], hs); (void)hipEventRecord(ev[2], hs); }
  launch_tiles_f64(2, r->d_t2, r->d_s2, (int)r->b.t2.size(), r->b.q2, r->d_cnt, r->d_bases, r->d_ut, out,
                   r->d_work, nullptr, stream);
  if (r->prof) {
    (void)hipEventRecord(ev[3], hs);
    for (auto &x : ev) r->ev.push_back(x);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { set_error(std::string("HIP: ") + hipGetErrorString(e)); return DMRG_EHIP; }
  return DMRG_OK;
}

extern "C" int dmrg_renorm_set_profiling(dmrg_renorm_t *r, int32_t on) {
  if (!r) { set_error("null argument"); return DMRG_EINVAL; }
  for (hipEvent_t e : r->ev) (void)hipEventDestroy(e);
  r->ev.clear();
  r->prof = on != 0;
  return DMRG_OK;
}

extern "C" int dmrg_renorm_get_profile(dmrg_renorm_t *r, int32_t stage, int64_t *n_launches, double *total_ms,
                                       double *total_flops) {
  if (!r || (stage != 1 && stage != 2) || !n_launches || !total_ms || !total_flops) {
    set_error("bad renormalization profile query");
    return DMRG_EINVAL;
  }
  int64_t n = 0;
  double ms = 0.0;
  for (size_t i = 0; i + 3 < r->ev.size(); i += 4) {
    hipEvent_t a = r->ev[i + (stage == 1 ? 0 : 2)], b = r->ev[i + (stage == 1 ? 1 : 3)];
    if (hipEventSynchronize(b) != hipSuccess) { set_error("hipEventSynchronize failed"); return DMRG_EHIP; }
    float t = 0.0f;
    if (hipEventElapsedTime(&t, a, b) != hipSuccess) { set_error("hipEventElapsedTime failed"); return DMRG_EHIP; }
    ms += t;
    n++;
  }
  *n_launches = n;
  *total_ms = ms;
  *total_flops = n * (stage == 1 ? r->b.flops1 : r->b.flops2);
  return DMRG_OK;
}

extern "C" int dmrg_renorm_stats(const dmrg_renorm_t *r, dmrg_renorm_stats_t *st) {
  if (!r || !st) { set_error("null argument"); return DMRG_EINVAL; }
  std::memset(st, 0, sizeof(*st));
  st->n_terms = r->b.n_terms;
  st->n_products1 = (int64_t)r->b.s1.size();
  st->n_products2 = (int64_t)r->b.s2.size();
  st->n_tiles1 = (int64_t)r->b.t1.size();
  st->n_tiles2 = (int64_t)r->b.t2.size();
  st->work_elems = r->b.work_len;
  st->out_elems = r->b.out_len;
  st->flops1 = r->b.flops1;
  st->flops2 = r->b.flops2;
  st->build_ms = r->b.build_ms;
  st->n_records = (int64_t)r->b.recs.size();
  return DMRG_OK;
}

extern "C" int dmrg_debug_renorm_host(const dmrg_problem_t *prob, const dmrg_rkeep_t *keep, int32_t n_keep,
                                      int32_t fam_mask, int32_t flags, const double *u, int64_t u_len, double *out,
                                      int64_t out_len, dmrg_oprec_t *rec, int64_t rec_cap,
                                      dmrg_renorm_stats_t *st) {
  try {
    Built b;
    Error err{0, ""};
    if (build_renorm(prob, keep, n_keep, fam_mask, flags, u_len, b, err)) { set_error(err.msg); return err.code; }
    if (st) {
      std::memset(st, 0, sizeof(*st));
      st->n_terms = b.n_terms;
      st->n_products1 = (int64_t)b.s1.size();
      st->n_products2 = (int64_t)b.s2.size();
      st->n_tiles1 = (int64_t)b.t1.size();
      st->n_tiles2 = (int64_t)b.t2.size();
      st->work_elems = b.work_len;
      st->out_elems = b.out_len;
      st->flops1 = b.flops1;
      st->flops2 = b.flops2;
      st->build_ms = b.build_ms;
      st->n_records = (int64_t)b.recs.size();
    }
    if (rec) std::memcpy(rec, b.recs.data(), std::min<int64_t>(rec_cap, (int64_t)b.recs.size()) * sizeof(dmrg_oprec_t));
    if (!out) return DMRG_OK;
    const bool right = flags & RENORM_RIGHT;
    const double *bdata = right ? prob->rdata : prob->ldata;
    const int64_t blen = right ? prob->rdata_len : prob->ldata_len;
    if (!u || !bdata || out_len < b.out_len) { set_error("missing input or output too small"); return DMRG_EINVAL; }
    std::vector<double> work((size_t)std::max<int64_t>(b.work_len, 1));
    std::vector<double> ut((size_t)std::max<int64_t>(u_len, 1)), lt;
    host_transpose(b.ujobs, u, ut.data());
    if (!b.ljobs.empty()) {
      lt.assign((size_t)blen, 0.0);
      host_transpose(b.ljobs, bdata, lt.data());
    }
    std::vector<double> dr((size_t)std::max<int64_t>(b.dress_len, 1), 0.0);
    for (const DressItem &d : b.ditems) {
      const double *src = d.src_base == BASE_OPS ? bdata : lt.data();
      for (int64_t e = 0; e < d.n; e++) {
        double acc = 0.0;
        for (int t = d.t0; t < d.t1; t++) acc += b.dalpha[t] * src[b.dsrc[t] + e];
        dr[d.dst_off + e] = acc;
      }
    }
    std::fill(out, out + b.out_len, 0.0);
    host_run(b.t1, b.s1, bdata, lt.data(), dr.data(), ut.data(), out, work.data());
    host_run(b.t2, b.s2, bdata, lt.data(), dr.data(), ut.data(), out, work.data());
    return DMRG_OK;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return DMRG_ENOMEM;
  }
}
