// Wigner coupling coefficients (paper: Appendix A, Eqs. (A2)-(A4), and Eq. (4)).
// Racah sums are evaluated in binary128 so that cancellation between terms
// leaves far more than FP64 accuracy for the spins used here; the result is
// rounded once to FP64.
#include "common.hpp"
#include <cmath>

namespace dmrg {

typedef __float128 q128;

static q128 qfact(int n) {
  static std::vector<q128> tab;
  if (tab.empty()) {
    tab.resize(171);
    tab[0] = 1;
    for (int i = 1; i < 171; i++) tab[i] = tab[i - 1] * (q128)i;
  }
  return tab[n];
}

static bool tri(int a, int b, int c) {
  return a >= 0 && b >= 0 && c >= 0 && std::abs(a - b) <= c && c <= a + b && ((a + b + c) % 2 == 0);
}

// squared triangle coefficient g~(a,b,c)^2 of Eq. (A4)
static q128 g2(int a, int b, int c) {
  return qfact((a + b - c) / 2) * qfact((a - b + c) / 2) * qfact((-a + b + c) / 2) /
         qfact((a + b + c) / 2 + 1);
}

static double qsqrt_to_double(q128 x) {
  long double lx = (long double)x;
  return (double)std::sqrt(lx);
}

double w6j(int a, int b, int c, int d, int e, int f) {
  if (!(tri(a, b, c) && tri(c, d, e) && tri(a, e, f) && tri(b, d, f))) return 0.0;
  int n2 = (a + b + c) / 2, n3 = (c + d + e) / 2, n4 = (a + e + f) / 2, n5 = (b + d + f) / 2;
  int n6 = (a + b + d + e) / 2, n7 = (a + c + d + f) / 2, n8 = (b + c + e + f) / 2;
  int nmin = std::max(std::max(0, n2), std::max(std::max(n3, n4), n5));
  int nmax = std::min(n6, std::min(n7, n8));
  q128 s = 0;
  for (int n = nmin; n <= nmax; n++) {
    q128 t = qfact(n + 1) / (qfact(n - n2) * qfact(n - n3) * qfact(n - n4) * qfact(n - n5) *
                             qfact(n6 - n) * qfact(n7 - n) * qfact(n8 - n));
    s += (n % 2) ? -t : t;
  }
  q128 pre2 = g2(a, b, c) * g2(c, d, e) * g2(a, e, f) * g2(b, d, f);
  return (double)((long double)s * (long double)qsqrt_to_double(pre2));
}

double w9j(int j1, int j2, int j, int k1, int k2, int k, int j1p, int j2p, int jp) {
  int xmin = std::max(j1 - jp, std::max(j2 - k, k1 - j2p));
  int xmax = std::min(j1 + jp, std::min(j2 + k, k1 + j2p));
  double tot = 0.0;
  for (int x = xmin; x <= xmax; x += 2) {
    if (x < 0) continue;
    double t = w6j(j1, j2, j, k, jp, x) * w6j(k1, k2, k, j2, x, j2p) * w6j(j1p, j2p, jp, x, j1, k1);
    tot += ((x % 2) ? -1.0 : 1.0) * (x + 1) * t;   // (-1)^(2x) with x doubled
  }
  return tot;
}

double ctilde(int j1, int j2, int j, int k1, int k2, int k, int j1p, int j2p, int jp) {
  double w = w9j(j1, j2, j, k1, k2, k, j1p, j2p, jp);
  if (w == 0.0) return 0.0;
  return std::sqrt((double)(j1p + 1) * (j2p + 1) * (j + 1) * (k + 1)) * w;
}

double cg(int j1, int m1, int j2, int m2, int J, int M) {
  if (m1 + m2 != M || std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(M) > J) return 0.0;
  if (!tri(j1, j2, J) || (j1 + m1) % 2 || (j2 + m2) % 2 || (J + M) % 2) return 0.0;
  q128 pre = (q128)(J + 1) * qfact((j1 + j2 - J) / 2) * qfact((j1 - j2 + J) / 2) *
             qfact((-j1 + j2 + J) / 2) / qfact((j1 + j2 + J) / 2 + 1);
  pre *= qfact((j1 + m1) / 2) * qfact((j1 - m1) / 2) * qfact((j2 + m2) / 2) * qfact((j2 - m2) / 2) *
         qfact((J + M) / 2) * qfact((J - M) / 2);
  q128 s = 0;
  for (int kk = 0; kk <= (j1 + j2 - J) / 2; kk++) {
    int d[6] = {kk, (j1 + j2 - J) / 2 - kk, (j1 - m1) / 2 - kk, (j2 + m2) / 2 - kk,
                (J - j2 + m1) / 2 + kk, (J - j1 - m2) / 2 + kk};
    bool ok = true;
    for (int i = 0; i < 6; i++) ok = ok && d[i] >= 0;
    if (!ok) continue;
    q128 den = 1;
    for (int i = 0; i < 6; i++) den *= qfact(d[i]);
    s += (kk % 2 ? -1 : 1) / den;
  }
  return (double)((long double)s * (long double)qsqrt_to_double(pre));
}

double CtildeTable::get(int j1, int j2, int j, int k1, int k2, int k, int j1p, int j2p, int jp) {
  uint64_t key = 0;
  int v[9] = {j1, j2, j, k1, k2, k, j1p, j2p, jp};
  for (int i = 0; i < 9; i++) key = key * 128 + (uint64_t)(v[i] & 127);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  double c = ctilde(j1, j2, j, k1, k2, k, j1p, j2p, jp);
  cache.emplace(key, c);
  return c;
}

}  // namespace dmrg
