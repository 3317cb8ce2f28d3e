// Host side of the H.psi library: block models, site algebra, the operator
// table (Eq. 2 combinations with their SU(2)-rescaled coupling constants),
// wavefunction blocks and the sector-task / sector-value tables (Eq. 3-4).
#include "common.hpp"
#include <cmath>
#include <algorithm>
#include <functional>
#include <sstream>

namespace dmrg {

const int FAM_TWO_K[N_FAM] = {0, 1, 0, 2, 0, 2, 1, 0, 2, 0, 2};
const int FAM_DN[N_FAM] = {0, 1, 2, 2, 0, 0, -1, -2, -2, 0, 0};
const int FAM_PAR[N_FAM] = {0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0};

static const int SITE_N[3] = {0, 1, 2};
static const int SITE_S[3] = {0, 1, 0};

// ------------------------------------------------------------------ blocks
static std::vector<std::array<int, 2>> family_labels(int fam, int role, int L, int p) {
  int lo = role == 0 ? 0 : p + 2, hi = role == 0 ? p : L;
  std::vector<int> out;
  if (role == 0) for (int x = p; x < L; x++) out.push_back(x);
  else for (int x = 0; x < p + 2; x++) out.push_back(x);
  std::vector<std::array<int, 2>> res;
  // grouped pair order: x<y inside, (x,x) inside, then (x,p), (x,p+1) and site pairs
  auto grouped = [&](int a, int b, bool strict, bool sites) {
    for (int x = a; x < b; x++) for (int y = x + 1; y < b; y++) res.push_back({x, y});
    if (!strict) for (int x = a; x < b; x++) res.push_back({x, x});
    if (sites) {
      for (int x = a; x < b; x++) res.push_back({x, p});
      for (int x = a; x < b; x++) res.push_back({x, p + 1});
      if (!strict) res.push_back({p, p});
      res.push_back({p, p + 1});
      if (!strict) res.push_back({p + 1, p + 1});
    }
  };
  switch (fam) {
    case F_H: res.push_back({-1, -1}); break;
    case F_C: for (int i = lo; i < hi; i++) res.push_back({i, -1}); break;
    case F_A0: case F_B0: case F_B1: grouped(lo, hi, false, false); break;
    case F_A1: grouped(lo, hi, true, false); break;
    case F_S: for (int x : out) res.push_back({x, -1}); break;
    default: {
      bool strict = fam == F_P1;
      if (role == 1) { grouped(0, p, strict, true); break; }
      for (int x : out)
        for (int y : out) {
          if (strict ? !(x < y) : !(x <= y)) continue;
          if (x >= p + 2 && y >= p + 2) continue;
          res.push_back({x, y});
        }
    }
  }
  return res;
}

int build_block(BlockModel &b, int role, const dmrg_problem_t &pr, Error &err) {
  b.role = role;
  b.n_orb = pr.n_orb;
  b.p = pr.site_l;
  b.lo = role == 0 ? 0 : pr.site_l + 2;
  b.hi = role == 0 ? pr.site_l : pr.n_orb;
  int ns = role == 0 ? pr.n_lsec : pr.n_rsec;
  const dmrg_sector_t *sec = role == 0 ? pr.lsec : pr.rsec;
  int64_t nr = role == 0 ? pr.n_lrec : pr.n_rrec;
  const dmrg_oprec_t *rec = role == 0 ? pr.lrec : pr.rrec;
  b.data = role == 0 ? pr.ldata : pr.rdata;
  b.data_len = role == 0 ? pr.ldata_len : pr.rdata_len;
  if (ns <= 0 || !sec) { err = {DMRG_EINVAL, "empty sector table"}; return err.code; }
  b.sec.assign(sec, sec + ns);
  int n = b.hi - b.lo;
  for (auto &s : b.sec) {
    if (s.dim <= 0 || s.n < 0 || s.n > 2 * n || s.two_s < 0 || s.two_s > std::min(s.n, 2 * n - s.n) ||
        (s.n + s.two_s) % 2) {
      err = {DMRG_ESYM, "sector with impossible (N, 2S, dim)"};
      return err.code;
    }
  }
  b.labels.assign(N_FAM, {});
  b.label_pos.assign(N_FAM, {});
  for (int f = 0; f < N_FAM; f++) {
    b.labels[f] = family_labels(f, role, pr.n_orb, pr.site_l);
    for (size_t i = 0; i < b.labels[f].size(); i++) b.label_pos[f][b.labels[f][i]] = (int)i;
  }
  b.rec.assign(rec, rec + (nr > 0 ? nr : 0));
  for (size_t i = 0; i < b.rec.size(); i++) {
    auto &r = b.rec[i];
    if (r.fam < 0 || r.fam >= N_FAM || r.row_sec < 0 || r.row_sec >= ns || r.col_sec < 0 ||
        r.col_sec >= ns) {
      err = {DMRG_EINVAL, "operator record with bad family or sector"};
      return err.code;
    }
    if (role == 1 && (r.fam >= F_A0 && r.fam <= F_B1)) {
      err = {DMRG_EINVAL, "pair families A/B are left-block only"};
      return err.code;
    }
    if (r.npos != (int)b.labels[r.fam].size()) {
      err = {DMRG_EINVAL, "record npos differs from the family label count"};
      return err.code;
    }
    const auto &sr = b.sec[r.row_sec], &sc = b.sec[r.col_sec];
    int k2 = FAM_TWO_K[r.fam];
    if (sr.n != sc.n + FAM_DN[r.fam] || sr.two_s < std::abs(sc.two_s - k2) || sr.two_s > sc.two_s + k2) {
      err = {DMRG_ESYM, "operator record violates N or spin selection rules"};
      return err.code;
    }
    int64_t len = (int64_t)r.npos * sr.dim * sc.dim;
    if (r.off < 0 || r.off + len > b.data_len) {
      err = {DMRG_ERANGE, "operator record beyond its data array"};
      return err.code;
    }
    int64_t key = ((int64_t)r.fam * 1000003 + r.row_sec) * 1000003 + r.col_sec;
    if (b.rec_index.count(key)) { err = {DMRG_EINVAL, "duplicate operator record"}; return err.code; }
    b.rec_index[key] = (int)i;
  }
  return DMRG_OK;
}

// ------------------------------------------------------------------ site algebra
typedef std::array<double, 16> M4;   // row-major 4x4; states |0>,|up>,|dn>,|updn>

static M4 m4zero() { M4 m; m.fill(0.0); return m; }
static M4 m4mul(const M4 &a, const M4 &b) {
  M4 c = m4zero();
  for (int i = 0; i < 4; i++)
    for (int k = 0; k < 4; k++)
      if (a[i * 4 + k] != 0.0)
        for (int j = 0; j < 4; j++) c[i * 4 + j] += a[i * 4 + k] * b[k * 4 + j];
  return c;
}
static M4 m4T(const M4 &a) {
  M4 c;
  for (int i = 0; i < 4; i++) for (int j = 0; j < 4; j++) c[i * 4 + j] = a[j * 4 + i];
  return c;
}

// elementary site tensor component: adj 0 -> a+_q, adj 1 -> a~_q
static M4 site_elem(int adj, int q2) {
  M4 cu = m4zero(), cd = m4zero();
  cu[1 * 4 + 0] = 1.0;  cu[3 * 4 + 2] = 1.0;     // a+_up
  cd[2 * 4 + 0] = 1.0;  cd[3 * 4 + 1] = -1.0;    // a+_dn (passes the up electron)
  if (adj == 0) return q2 > 0 ? cu : cd;
  if (q2 > 0) return m4T(cd);                    // a~_{+1/2} = a_dn
  M4 r = m4T(cu);
  for (auto &x : r) x = -x;                      // a~_{-1/2} = -a_up
  return r;
}

// M-resolved site state of multiplet m with doubled projection M2
static int site_state(int m, int M2) {
  if (m == 0) return 0;
  if (m == 2) return 3;
  return M2 > 0 ? 1 : 2;
}

int SiteAlgebra::get(const std::vector<int> &adj, const std::vector<int> &inter) {
  auto key = std::make_pair(adj, inter);
  auto it = index.find(key);
  if (it != index.end()) return it->second;
  // components of the left-to-right coupled string
  std::map<int, M4> acc;
  acc[1] = site_elem(adj[0], 1);
  acc[-1] = site_elem(adj[0], -1);
  int kacc = 1;
  for (size_t i = 1; i < adj.size(); i++) {
    int knew = inter[i - 1];
    std::map<int, M4> nxt;
    for (int Q = -knew; Q <= knew; Q += 2) {
      M4 s = m4zero();
      bool any = false;
      for (auto &kv : acc) {
        int qb = Q - kv.first;
        if (std::abs(qb) != 1) continue;
        double c = cg(kacc, kv.first, 1, qb, knew, Q);
        if (c == 0.0) continue;
        M4 prod = m4mul(kv.second, site_elem(adj[i], qb));
        for (int t = 0; t < 16; t++) s[t] += c * prod[t];
        any = true;
      }
      if (any) nxt[Q] = s;
    }
    acc.swap(nxt);
    kacc = knew;
  }
  SiteFamily f;
  f.adj = adj;
  f.inter = inter;
  f.k2 = kacc;
  f.parity = (int)(adj.size() % 2);
  for (int b = 0; b < 3; b++)
    for (int a = 0; a < 3; a++) {
      f.red[b][a] = 0.0;
      int Sa = SITE_S[a], Sb = SITE_S[b];
      if (Sb < std::abs(Sa - kacc) || Sb > Sa + kacc) continue;
      double best = 0.0;
      int bq = 0, bMa = 0;
      for (int q = -kacc; q <= kacc; q += 2) {
        int Ma = Sb - q;
        if (std::abs(Ma) > Sa) continue;
        double c = cg(Sa, Ma, kacc, q, Sb, Sb);
        if (std::fabs(c) > std::fabs(best)) { best = c; bq = q; bMa = Ma; }
      }
      if (best == 0.0 || !acc.count(bq)) continue;
      const M4 &m = acc[bq];
      double el = m[site_state(b, Sb) * 4 + site_state(a, bMa)];
      f.red[b][a] = el / best;
      if (std::fabs(f.red[b][a]) < 1e-14) f.red[b][a] = 0.0;
    }
  int idx = (int)fams.size();
  fams.push_back(f);
  index[key] = idx;
  return idx;
}

// ------------------------------------------------------------------ CG projection
// A factor component: one tensor component on one partition, in operator order.
struct FComp {
  int part;    // 0 L, 1 l, 2 r, 3 R
  int kind;    // 0 block family, 1 site elementary (a+ or a~)
  int fam;
  int adj;
  int k2, q2;
};
struct Product {
  double coef;
  std::vector<FComp> f;
};

static int fcomp_parity(const FComp &c) { return c.kind == 1 ? 1 : FAM_PAR[c.fam]; }

// (T_q)^+ = (-1)^{k+q} Tbar_{-q};  (Tbar_q)^+ = (-1)^{k+q} (-1)^{2k} T_{-q}
static Product adjoint(const Product &p) {
  Product r;
  r.coef = p.coef;
  for (auto it = p.f.rbegin(); it != p.f.rend(); ++it) {
    FComp c = *it;
    int e = (c.k2 + c.q2) / 2;
    if (e % 2) r.coef = -r.coef;
    if (c.adj && (c.k2 % 2)) r.coef = -r.coef;
    c.adj ^= 1;
    c.q2 = -c.q2;
    r.f.push_back(c);
  }
  return r;
}

struct EngOut {
  PT t[4];
  int K2;
  double alpha;
};

struct PTKey {
  PT t[4];
  bool operator<(const PTKey &o) const {
    for (int i = 0; i < 4; i++) {
      if (t[i] < o.t[i]) return true;
      if (o.t[i] < t[i]) return false;
    }
    return false;
  }
};

struct Opt { PT t; int q2; double w; };

static int project(const std::vector<Product> &prods, SiteAlgebra &site, std::vector<EngOut> &out,
                   Error &err) {
  std::map<PTKey, std::map<std::array<int, 4>, double>> F;
  for (const auto &pr : prods) {
    if (pr.coef == 0.0) continue;
    std::vector<FComp> f = pr.f;
    double sign = 1.0;
    for (size_t i = 0; i < f.size(); i++)
      for (size_t j = i + 1; j < f.size(); j++)
        if (f[i].part > f[j].part && fcomp_parity(f[i]) && fcomp_parity(f[j])) sign = -sign;
    std::stable_sort(f.begin(), f.end(), [](const FComp &a, const FComp &b) { return a.part < b.part; });
    std::vector<Opt> opts[4];
    for (int pt = 0; pt < 4; pt++) {
      std::vector<FComp> mine;
      for (auto &c : f) if (c.part == pt) mine.push_back(c);
      if (mine.empty()) { opts[pt].push_back({PT(), 0, 1.0}); continue; }
      if (pt == 0 || pt == 3) {
        if (mine.size() > 1) { err = {DMRG_EINVAL, "two block factors on one block"}; return err.code; }
        PT t;
        t.kind = 1; t.id = mine[0].fam; t.adj = mine[0].adj; t.k2 = mine[0].k2; t.par = FAM_PAR[mine[0].fam];
        opts[pt].push_back({t, mine[0].q2, 1.0});
        continue;
      }
      // site string: expand over intermediate couplings
      std::vector<int> adj;
      for (auto &c : mine) adj.push_back(c.adj);
      std::function<void(size_t, int, int, double, std::vector<int> &)> rec =
          [&](size_t i, int kacc, int qacc, double w, std::vector<int> &inter) {
            if (i == mine.size()) {
              PT t;
              t.kind = 2; t.id = site.get(adj, inter); t.adj = 0; t.k2 = kacc; t.par = (int)(mine.size() % 2);
              opts[pt].push_back({t, qacc, w});
              return;
            }
            int qn = mine[i].q2;
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
    for (auto &a : opts[0])
      for (auto &b : opts[1])
        for (auto &c : opts[2])
          for (auto &d : opts[3]) {
            PTKey k;
            k.t[0] = a.t; k.t[1] = b.t; k.t[2] = c.t; k.t[3] = d.t;
            std::array<int, 4> q = {a.q2, b.q2, c.q2, d.q2};
            F[k][q] += pr.coef * sign * a.w * b.w * c.w * d.w;
          }
  }
  for (auto &kv : F) {
    const PTKey &k = kv.first;
    // drop keys whose site family vanishes identically
    bool zero = false;
    for (int pt = 1; pt <= 2; pt++)
      if (k.t[pt].kind == 2) {
        const auto &sf = site.fams[k.t[pt].id];
        bool nz = false;
        for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) nz = nz || sf.red[i][j] != 0.0;
        if (!nz) zero = true;
      }
    if (zero) continue;
    int kA = k.t[0].k2, kB = k.t[1].k2, kC = k.t[2].k2, kD = k.t[3].k2;
    double fmax = 0.0;
    for (auto &qv : kv.second) fmax = std::max(fmax, std::fabs(qv.second));
    if (fmax < 1e-15) continue;
    std::vector<std::pair<int, double>> alphas;
    for (int K = std::max(std::abs(kA - kB), std::abs(kC - kD)); K <= std::min(kA + kB, kC + kD); K += 2) {
      if ((kA + kB + K) % 2 || (kC + kD + K) % 2) continue;
      double a = 0.0;
      for (auto &qv : kv.second) {
        const auto &q = qv.first;
        int Q1 = q[0] + q[1], Q2 = q[2] + q[3];
        if (Q1 + Q2 != 0) continue;
        a += qv.second * cg(kA, q[0], kB, q[1], K, Q1) * cg(kC, q[2], kD, q[3], K, Q2) * cg(K, Q1, K, Q2, 0, 0);
      }
      if (std::fabs(a) > 1e-13 * fmax) alphas.push_back({K, a});
    }
    // the term must be a spin scalar: reconstruct every component
    double resid = 0.0;
    for (int qA = -kA; qA <= kA; qA += 2)
      for (int qB = -kB; qB <= kB; qB += 2)
        for (int qC = -kC; qC <= kC; qC += 2)
          for (int qD = -kD; qD <= kD; qD += 2) {
            double rec = 0.0;
            for (auto &ka : alphas) {
              int K = ka.first;
              rec += ka.second * cg(kA, qA, kB, qB, K, qA + qB) * cg(kC, qC, kD, qD, K, qC + qD) *
                     cg(K, qA + qB, K, qC + qD, 0, 0);
            }
            auto it = kv.second.find({qA, qB, qC, qD});
            double f = it == kv.second.end() ? 0.0 : it->second;
            resid = std::max(resid, std::fabs(f - rec));
          }
    if (resid > 1e-10 * fmax) {
      err = {DMRG_EINVAL, "internal: operator combination is not a spin scalar"};
      return err.code;
    }
    for (auto &ka : alphas) {
      EngOut o;
      for (int i = 0; i < 4; i++) o.t[i] = k.t[i];
      o.K2 = ka.first;
      o.alpha = ka.second;
      out.push_back(o);
    }
  }
  return DMRG_OK;
}

// ------------------------------------------------------------------ operator table
namespace {

struct Ctx {
  const dmrg_problem_t &pr;
  const BlockModel &L, &R;
  SiteAlgebra &site;
  std::map<RowKey, std::map<std::pair<int, int>, double>> acc;
  Error &err;
  int p, Lorb;
  int part(int x) const { return x < p ? 0 : x == p ? 1 : x == p + 1 ? 2 : 3; }
  double h(int i, int j) const { return pr.h1[(int64_t)i * Lorb + j]; }
  double v(int i, int j, int k, int l) const {
    return pr.eri[(((int64_t)i * Lorb + j) * Lorb + k) * Lorb + l];
  }
};

// creation (dagger) or annihilation of orbital x with spin s2 as a tensor component:
// a+_s = C_s ; a_s = (-1)^{1/2+s} C~_{-s}
static FComp elem(const Ctx &c, int x, int s2, bool dagger, double &coef) {
  FComp f;
  f.part = c.part(x);
  f.kind = (f.part == 1 || f.part == 2) ? 1 : 0;
  f.fam = F_C;
  f.adj = dagger ? 0 : 1;
  f.k2 = 1;
  f.q2 = dagger ? s2 : -s2;
  if (!dagger && ((1 + s2) / 2) % 2) coef = -coef;
  return f;
}

static FComp famc(int part, int fam, int adj, int q2) {
  FComp f;
  f.part = part; f.kind = 0; f.fam = fam; f.adj = adj; f.k2 = FAM_TWO_K[fam]; f.q2 = q2;
  return f;
}

static double ph(int x2) {  // (-1)^(x2/2), x2 even
  return ((x2 / 2) % 2 != 0) ? -1.0 : 1.0;
}

struct Label { int x = -1, y = -1; };

static int add_instance(Ctx &c, const std::vector<Product> &prods, Label labL, Label labR,
                        double scale) {
  std::vector<EngOut> outs;
  if (project(prods, c.site, outs, c.err)) return c.err.code;
  for (auto &o : outs) {
    int pA = 0, pD = 0;
    if (o.t[0].kind == 1) {
      pA = c.L.pos(o.t[0].id, labL.x, labL.y);
      if (pA < 0) { c.err = {DMRG_EINVAL, "internal: left label not in family"}; return c.err.code; }
    }
    if (o.t[3].kind == 1) {
      pD = c.R.pos(o.t[3].id, labR.x, labR.y);
      if (pD < 0) { c.err = {DMRG_EINVAL, "internal: right label not in family"}; return c.err.code; }
    }
    RowKey k;
    for (int i = 0; i < 4; i++) k.t[i] = o.t[i];
    k.K2 = o.K2;
    c.acc[k][{pA, pD}] += scale * o.alpha;
  }
  return DMRG_OK;
}

static void with_adjoints(std::vector<Product> &p) {
  size_t n = p.size();
  for (size_t i = 0; i < n; i++) p.push_back(adjoint(p[i]));
}

}  // namespace

int build_rows(const dmrg_problem_t &pr, const BlockModel &L, const BlockModel &R, SiteAlgebra &site,
               std::vector<Row> &rows, Error &err) {
  Ctx c{pr, L, R, site, {}, err, pr.site_l, pr.n_orb};
  const int p = c.p, Lo = c.Lorb;
  const int sp[2] = {1, -1};
  const bool hasL = p > 0, hasR = p + 2 < Lo;
  auto lab1 = [&](int x) { Label l; l.x = x; return l; };
  // block Hamiltonians (all indices inside one block)
  if (hasL) {
    std::vector<Product> pp{{1.0, {famc(0, F_H, 0, 0)}}};
    if (add_instance(c, pp, Label(), Label(), 1.0)) return err.code;
  }
  if (hasR) {
    std::vector<Product> pp{{1.0, {famc(3, F_H, 0, 0)}}};
    if (add_instance(c, pp, Label(), Label(), 1.0)) return err.code;
  }
  // three indices in one block: sum_s a+_xs (S_x)_s + h.c., (S_x)_s = -sqrt2 (-1)^{1/2+s} S~_{-s}
  for (int X = 0; X < 2; X++) {
    if (X == 0 ? !hasL : !hasR) continue;
    int xpart = X == 0 ? 0 : 3;
    const BlockModel &B = X == 0 ? L : R;
    for (auto &lab : B.labels[F_S]) {
      int x = lab[0];
      std::vector<Product> pp;
      for (int s : sp) {
        Product q;
        q.coef = -std::sqrt(2.0) * ph(1 + s);
        q.f.push_back(elem(c, x, s, true, q.coef));
        q.f.push_back(famc(xpart, F_S, 0, -s));
        pp.push_back(q);
      }
      with_adjoints(pp);
      Label lx = lab1(x), none;
      int xp = c.part(x);
      Label labL = X == 0 ? lx : (xp == 0 ? lx : none);
      Label labR = X == 1 ? lx : (xp == 3 ? lx : none);
      if (add_instance(c, pp, labL, labR, 1.0)) return err.code;
    }
  }
  // two indices in one block: P and Q complementary operators, x <= y folded
  for (int X = 0; X < 2; X++) {
    if (X == 0 ? !hasL : !hasR) continue;
    int xpart = X == 0 ? 0 : 3;
    const BlockModel &B = X == 0 ? L : R;
    for (auto &lab : B.labels[F_Q0]) {
      int x = lab[0], y = lab[1];
      bool same = X == 1 && x < p && y < p;
      Label lxy; lxy.x = x; lxy.y = y;
      Label labL, labR;
      if (X == 0) labL = lxy; else labR = lxy;
      if (same) labL = lxy;
      else {
        int px = c.part(x), py = c.part(y);
        int other = X == 0 ? 3 : 0;
        Label &lo = X == 0 ? labR : labL;
        if (px == other) lo = lab1(x);
        if (py == other) lo = lab1(y);
      }
      double mult = x < y ? 2.0 : 1.0;
      // --- P: 1/2 sum_st a+_xs a+_yt (P_xy)_{ts} + h.c.
      {
        std::vector<Product> pp;
        for (int s : sp)
          for (int t : sp)
            for (int K = 0; K <= 2; K += 2) {
              if (K == 2 && x == y) continue;
              double cP = ph(2 + t + s) * cg(1, -t, 1, -s, K, -t - s);
              if (cP == 0.0) continue;
              FComp Pc = famc(xpart, K == 0 ? F_P0 : F_P1, 0, -t - s);
              if (same) {
                for (int K2 = 0; K2 <= 2; K2 += 2) {
                  if (K2 == 2 && x == y) continue;
                  double cA = cg(1, s, 1, t, K2, s + t);
                  if (cA == 0.0) continue;
                  Product q;
                  q.coef = 0.5 * mult * cP * cA;
                  q.f.push_back(famc(0, K2 == 0 ? F_A0 : F_A1, 0, s + t));
                  q.f.push_back(Pc);
                  pp.push_back(q);
                }
              } else {
                Product q;
                q.coef = 0.5 * mult * cP;
                q.f.push_back(elem(c, x, s, true, q.coef));
                q.f.push_back(elem(c, y, t, true, q.coef));
                q.f.push_back(Pc);
                pp.push_back(q);
              }
            }
        with_adjoints(pp);
        if (add_instance(c, pp, labL, labR, 1.0)) return err.code;
      }
      // --- Q: sum_st (Q_xy)_{ts} a+_xt a_ys (+ h.c. for x < y)
      {
        std::vector<Product> pp;
        for (int s : sp)
          for (int t : sp) {
            std::vector<std::pair<double, FComp>> qparts;
            if (s == t) qparts.push_back({-1.0 / std::sqrt(2.0), famc(xpart, F_Q0, 0, 0)});
            double c1 = cg(1, s, 1, -t, 2, s - t);
            if (c1 != 0.0)
              qparts.push_back({-ph(1 + t) * c1 / std::sqrt(3.0), famc(xpart, F_Q1, 0, s - t)});
            for (auto &qpart : qparts) {
              if (same) {
                for (int K2 = 0; K2 <= 2; K2 += 2) {
                  double cB = ph(1 + s) * cg(1, t, 1, -s, K2, t - s);
                  if (cB == 0.0) continue;
                  Product q;
                  q.coef = qpart.first * cB;
                  q.f.push_back(qpart.second);
                  q.f.push_back(famc(0, K2 == 0 ? F_B0 : F_B1, 0, t - s));
                  pp.push_back(q);
                }
              } else {
                Product q;
                q.coef = qpart.first;
                q.f.push_back(qpart.second);
                q.f.push_back(elem(c, x, t, true, q.coef));
                q.f.push_back(elem(c, y, s, false, q.coef));
                pp.push_back(q);
              }
            }
          }
        if (x < y) with_adjoints(pp);
        if (add_instance(c, pp, labL, labR, 1.0)) return err.code;
      }
    }
  }
  // explicit products: at most one index in each block
  auto nblk = [&](std::initializer_list<int> idx, int &nl, int &nr) {
    nl = nr = 0;
    for (int i : idx) { nl += i < p; nr += i >= p + 2; }
  };
  auto block_labels = [&](std::initializer_list<int> idx, Label &lL, Label &lR) {
    for (int i : idx) {
      if (i < p) lL.x = i;
      if (i >= p + 2) lR.x = i;
    }
  };
  for (int i = 0; i < Lo; i++)
    for (int j = 0; j < Lo; j++) {
      int nl, nr;
      nblk({i, j}, nl, nr);
      if (nl > 1 || nr > 1) continue;
      double hv = c.h(i, j);
      if (hv == 0.0) continue;
      std::vector<Product> pp;
      for (int s : sp) {
        Product q;
        q.coef = 1.0;
        q.f.push_back(elem(c, i, s, true, q.coef));
        q.f.push_back(elem(c, j, s, false, q.coef));
        pp.push_back(q);
      }
      Label lL, lR;
      block_labels({i, j}, lL, lR);
      if (add_instance(c, pp, lL, lR, hv)) return err.code;
    }
  for (int i = 0; i < Lo; i++)
    for (int j = 0; j < Lo; j++)
      for (int k = 0; k < Lo; k++)
        for (int l = 0; l < Lo; l++) {
          int nl, nr;
          nblk({i, j, k, l}, nl, nr);
          if (nl > 1 || nr > 1) continue;
          double vv = c.v(i, j, k, l);
          if (vv == 0.0) continue;
          std::vector<Product> pp;
          for (int s : sp)
            for (int t : sp) {
              if (i == k && s == t) continue;
              if (j == l && s == t) continue;
              Product q;
              q.coef = 1.0;
              q.f.push_back(elem(c, i, s, true, q.coef));
              q.f.push_back(elem(c, k, t, true, q.coef));
              q.f.push_back(elem(c, l, t, false, q.coef));
              q.f.push_back(elem(c, j, s, false, q.coef));
              pp.push_back(q);
            }
          Label lL, lR;
          block_labels({i, j, k, l}, lL, lR);
          if (add_instance(c, pp, lL, lR, 0.5 * vv)) return err.code;
        }
  rows.clear();
  for (auto &kv : c.acc) {
    Row r;
    r.key = kv.first;
    for (auto &pa : kv.second)
      if (pa.second != 0.0) r.pos.push_back({pa.first.first, pa.first.second, pa.second});
    if (!r.pos.empty()) rows.push_back(r);
  }
  return DMRG_OK;
}

// ------------------------------------------------------------------ wavefunction blocks
void psi_blocks(const BlockModel &L, const BlockModel &R, int n_elec, int two_s,
                std::vector<PsiBlock> &out, int64_t &size) {
  out.clear();
  size = 0;
  for (int iL = 0; iL < (int)L.sec.size(); iL++) {
    const auto &sl = L.sec[iL];
    for (int l = 0; l < 3; l++)
      for (int SLl = std::abs(sl.two_s - SITE_S[l]); SLl <= sl.two_s + SITE_S[l]; SLl += 2)
        for (int r = 0; r < 3; r++)
          for (int iR = 0; iR < (int)R.sec.size(); iR++) {
            const auto &sr = R.sec[iR];
            if (sl.n + SITE_N[l] + SITE_N[r] + sr.n != n_elec) continue;
            for (int SrR = std::abs(SITE_S[r] - sr.two_s); SrR <= SITE_S[r] + sr.two_s; SrR += 2) {
              if (!(std::abs(SLl - SrR) <= two_s && two_s <= SLl + SrR)) continue;
              PsiBlock b{iL, l, SLl, r, iR, SrR, sl.dim, sr.dim, size};
              out.push_back(b);
              size += (int64_t)sl.dim * sr.dim;
            }
          }
  }
}

// ------------------------------------------------------------------ sector tasks
int build_tasks_for_problem(const dmrg_problem_t &pr, BlockModel &L, BlockModel &R, Tasks &T,
                            Error &err) {
  if (pr.n_orb < 2 || pr.site_l < 0 || pr.site_l + 2 > pr.n_orb || pr.n_elec < 0 ||
      pr.n_elec > 2 * pr.n_orb || pr.two_s < 0 || (pr.n_elec + pr.two_s) % 2) {
    err = {DMRG_EINVAL, "bad orbital count, bond, electron count or spin"};
    return err.code;
  }
  if (!pr.h1 || !pr.eri) { err = {DMRG_EINVAL, "integrals missing"}; return err.code; }
  for (int64_t i = 0; i < (int64_t)pr.n_orb * pr.n_orb; i++)
    if (!std::isfinite(pr.h1[i])) { err = {DMRG_ENONFINITE, "non-finite one-electron integral"}; return err.code; }
  int64_t n4 = (int64_t)pr.n_orb * pr.n_orb * pr.n_orb * pr.n_orb;
  for (int64_t i = 0; i < n4; i++)
    if (!std::isfinite(pr.eri[i])) { err = {DMRG_ENONFINITE, "non-finite two-electron integral"}; return err.code; }
  if (build_block(L, 0, pr, err) || build_block(R, 1, pr, err)) return err.code;
  psi_blocks(L, R, pr.n_elec, pr.two_s, T.blocks, T.size);
  if (T.blocks.empty()) { err = {DMRG_ESYM, "no wavefunction block has the target N and S"}; return err.code; }
  if (build_rows(pr, L, R, T.site, T.rows, err)) return err.code;
  // block lookup
  std::map<std::array<int, 6>, int> bidx;
  for (size_t i = 0; i < T.blocks.size(); i++) {
    const auto &b = T.blocks[i];
    bidx[{b.iL, b.l, b.SLl, b.r, b.iR, b.SrR}] = (int)i;
  }
  // rows with two position indices: keep, per left position, its list of
  // (right position, alpha); the row then runs over left positions only
  std::vector<std::vector<std::pair<int, std::vector<std::pair<int, double>>>>> dress_src(T.rows.size());
  for (size_t ri = 0; ri < T.rows.size(); ri++) {
    Row &row = T.rows[ri];
    std::map<int, std::vector<std::pair<int, double>>> byA;
    for (auto &pa : row.pos) byA[pa.pA].push_back({pa.pD, pa.alpha});
    if (byA.size() == row.pos.size()) continue;      // one right position per left one
    if (row.key.t[3].kind != 1) continue;             // identity on the right: nothing to sum
    std::vector<PosAlpha> np;
    int j = 0;
    for (auto &kv : byA) {
      np.push_back({kv.first, j++, 1.0});
      dress_src[ri].push_back({kv.first, kv.second});
    }
    row.pos = np;
  }
  std::map<std::pair<int, int>, int> dress_of;   // (row, source record) -> dressed record
  T.dress.clear();
  T.dress_len = 0;
  CtildeTable wl, wr, wh;
  T.tasks.clear();
  T.flops = 0.0;
  for (size_t ri = 0; ri < T.rows.size(); ri++) {
    const Row &row = T.rows[ri];
    const PT &tA = row.key.t[0], &tB = row.key.t[1], &tC = row.key.t[2], &tD = row.key.t[3];
    const int K = row.key.K2;
    for (size_t ei = 0; ei < T.blocks.size(); ei++) {
      const PsiBlock &E = T.blocks[ei];
      const auto &sL = L.sec[E.iL];
      const auto &sR = R.sec[E.iR];
      // left operator options: (iL', record, phase)
      struct Side { int sec, rec; double ph; };
      std::vector<Side> As, Ds;
      auto side_opts = [&](const PT &t, const BlockModel &B, int ket, std::vector<Side> &o) {
        if (t.kind == 0) { o.push_back({ket, -1, 1.0}); return; }
        for (int s2 = 0; s2 < (int)B.sec.size(); s2++) {
          if (!t.adj) {
            int rr = B.find_rec(t.id, s2, ket);
            if (rr >= 0) o.push_back({s2, rr, 1.0});
          } else {
            int rr = B.find_rec(t.id, ket, s2);
            if (rr >= 0) {
              int Sk = B.sec[ket].two_s, Sb = B.sec[s2].two_s;
              double ph = (((Sk + t.k2 - Sb) / 2) % 2 ? -1.0 : 1.0) * std::sqrt((Sk + 1.0) / (Sb + 1.0));
              o.push_back({s2, rr, ph});
            }
          }
        }
      };
      side_opts(tA, L, E.iL, As);
      side_opts(tD, R, E.iR, Ds);
      if (As.empty() || Ds.empty()) continue;
      std::vector<std::pair<int, double>> Bs, Cs;
      if (tB.kind == 0) Bs.push_back({E.l, 1.0});
      else for (int l2 = 0; l2 < 3; l2++) { double x = T.site.fams[tB.id].red[l2][E.l]; if (x != 0.0) Bs.push_back({l2, x}); }
      if (tC.kind == 0) Cs.push_back({E.r, 1.0});
      else for (int r2 = 0; r2 < 3; r2++) { double x = T.site.fams[tC.id].red[r2][E.r]; if (x != 0.0) Cs.push_back({r2, x}); }
      int pB = tB.par, pC = tC.par, pD = tD.par;
      int NL = sL.n;
      double jw = ((pB * NL + pC * (NL + SITE_N[E.l]) + pD * (NL + SITE_N[E.l] + SITE_N[E.r])) % 2) ? -1.0 : 1.0;
      for (auto &a : As)
        for (auto &bb : Bs)
          for (auto &cc : Cs)
            for (auto &d : Ds) {
              int SL2 = L.sec[a.sec].two_s, SR2 = R.sec[d.sec].two_s;
              int sl2 = SITE_S[bb.first], sr2 = SITE_S[cc.first];
              for (int SLl2 = std::abs(SL2 - sl2); SLl2 <= SL2 + sl2; SLl2 += 2) {
                if (SLl2 < std::abs(E.SLl - K) || SLl2 > E.SLl + K) continue;
                double cl = wl.get(sL.two_s, SITE_S[E.l], E.SLl, tA.k2, tB.k2, K, SL2, sl2, SLl2);
                if (cl == 0.0) continue;
                for (int SrR2 = std::abs(sr2 - SR2); SrR2 <= sr2 + SR2; SrR2 += 2) {
                  if (SrR2 < std::abs(E.SrR - K) || SrR2 > E.SrR + K) continue;
                  auto it = bidx.find({a.sec, bb.first, SLl2, cc.first, d.sec, SrR2});
                  if (it == bidx.end()) continue;
                  double cr = wr.get(SITE_S[E.r], sR.two_s, E.SrR, tC.k2, tD.k2, K, sr2, SR2, SrR2);
                  if (cr == 0.0) continue;
                  double ch = wh.get(E.SLl, E.SrR, pr.two_s, K, K, 0, SLl2, SrR2, pr.two_s);
                  if (ch == 0.0) continue;
                  double v = jw * a.ph * d.ph * bb.second * cc.second * cl * cr * ch;
                  if (std::fabs(v) < 1e-300) continue;
                  Task tk;
                  tk.row = (int)ri;
                  tk.E = (int)ei;
                  tk.F = it->second;
                  tk.recA = a.rec;
                  tk.recD = d.rec;
                  tk.adjA = tA.adj;
                  tk.adjD = tD.adj;
                  tk.v = v;
                  if (!dress_src[ri].empty() && tk.recD >= 0) {
                    auto key = std::make_pair((int)ri, tk.recD);
                    auto dit = dress_of.find(key);
                    if (dit == dress_of.end()) {
                      Dress d;
                      d.rec = tk.recD;
                      const dmrg_oprec_t &rr = R.rec[tk.recD];
                      d.rows = R.sec[rr.row_sec].dim;
                      d.cols = R.sec[rr.col_sec].dim;
                      d.npos = (int)dress_src[ri].size();
                      d.start.push_back(0);
                      for (auto &e : dress_src[ri]) {
                        for (auto &pa : e.second) {
                          d.src_pos.push_back(pa.first);
                          d.src_alpha.push_back(pa.second);
                        }
                        d.start.push_back((int)d.src_pos.size());
                      }
                      d.off = T.dress_len;
                      T.dress_len += (int64_t)d.npos * d.rows * d.cols;
                      dit = dress_of.emplace(key, (int)T.dress.size()).first;
                      T.dress.push_back(std::move(d));
                    }
                    tk.dress = dit->second;
                  }
                  T.tasks.push_back(tk);
                  const PsiBlock &Fb = T.blocks[tk.F];
                  double npos = (double)row.pos.size();
                  if (tk.recD >= 0) T.flops += npos * 2.0 * E.dL * E.dR * Fb.dR;
                  if (tk.recA >= 0) T.flops += npos * 2.0 * Fb.dL * E.dL * Fb.dR;
                }
              }
            }
    }
  }
  return DMRG_OK;
}

void dress_on_host(const Tasks &T, const BlockModel &R, std::vector<double> &out) {
  out.assign((size_t)std::max<int64_t>(T.dress_len, 1), 0.0);
  for (const Dress &d : T.dress) {
    const dmrg_oprec_t &r = R.rec[d.rec];
    int64_t bs = (int64_t)d.rows * d.cols;
    for (int j = 0; j < d.npos; j++)
      for (int t = d.start[j]; t < d.start[j + 1]; t++) {
        const double *src = R.data + r.off + (int64_t)d.src_pos[t] * bs;
        double *dst = out.data() + d.off + (int64_t)j * bs;
        for (int64_t e = 0; e < bs; e++) dst[e] += d.src_alpha[t] * src[e];
      }
  }
}

}  // namespace dmrg
