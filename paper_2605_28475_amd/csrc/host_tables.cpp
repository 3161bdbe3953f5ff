// Angular tables (Sections 4.1-4.2) and quadrature rules, host FP64.
#include <algorithm>
#include <cmath>
#include <complex>
#include <stdexcept>
#include <thread>

#include "wefq_host.h"

namespace wefq {

std::vector<Channel> enumerate_channels(int L) {
  std::vector<Channel> out;
  for (int l1 = 0; l1 <= L; ++l1)
    for (int l2 = 0; l2 <= L; ++l2)
      for (int l3 = std::abs(l1 - l2); l3 <= std::min(l1 + l2, L); ++l3)
        if ((l1 + l2 + l3) % 2 == 0) out.push_back({l1, l2, l3});
  return out;
}

static long double lfact(int n) {
  static const std::vector<long double> tab = [] {   // thread-safe one-time initialization
    std::vector<long double> t(200);
    t[0] = 1.0L;
    for (int i = 1; i < 200; ++i) t[i] = t[i - 1] * (long double)i;
    return t;
  }();
  if (n < 0 || n >= 200) throw std::runtime_error("factorial argument out of range");
  return tab[n];
}

long double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
  if (m1 + m2 + m3 != 0) return 0.0L;
  if (j3 < std::abs(j1 - j2) || j3 > j1 + j2) return 0.0L;
  if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3) return 0.0L;
  long double tri = std::sqrt(lfact(j1 + j2 - j3) * lfact(j1 - j2 + j3) * lfact(-j1 + j2 + j3) /
                              lfact(j1 + j2 + j3 + 1));
  long double pre = std::sqrt(lfact(j1 + m1) * lfact(j1 - m1) * lfact(j2 + m2) * lfact(j2 - m2) *
                              lfact(j3 + m3) * lfact(j3 - m3));
  int kmin = std::max({0, j2 - j3 - m1, j1 - j3 + m2});
  int kmax = std::min({j1 + j2 - j3, j1 - m1, j2 + m2});
  long double sum = 0.0L;
  for (int k = kmin; k <= kmax; ++k) {
    long double den = lfact(k) * lfact(j3 - j2 + k + m1) * lfact(j3 - j1 + k - m2) *
                      lfact(j1 + j2 - j3 - k) * lfact(j1 - k - m1) * lfact(j2 - k + m2);
    sum += ((k & 1) ? -1.0L : 1.0L) / den;
  }
  int ph = j1 - j2 - m3;
  return ((ph & 1) ? -1.0L : 1.0L) * tri * pre * sum;
}

// Coefficients of Y^R_{l,m} in terms of complex Y_l^mu: pairs (mu, coefficient).
static int real_to_complex(int m, std::pair<int, std::complex<long double>> out[2]) {
  const long double s = 1.0L / std::sqrt(2.0L);
  if (m == 0) { out[0] = {0, {1.0L, 0.0L}}; return 1; }
  int a = std::abs(m);
  long double sgn = (a & 1) ? -1.0L : 1.0L;
  if (m > 0) {          // ((-1)^m Y^m + Y^-m)/sqrt2
    out[0] = {a, {sgn * s, 0.0L}};
    out[1] = {-a, {s, 0.0L}};
  } else {              // ((-1)^a Y^a - Y^-a)/(i sqrt2)
    out[0] = {a, {0.0L, -sgn * s}};
    out[1] = {-a, {0.0L, s}};
  }
  return 2;
}

// The real Gaunt weight given the m-independent factor
// base = sqrt((2l1+1)(2l2+1)(2l3+1)/(4 pi)) (l1 l2 l3; 0 0 0).
static double real_gaunt_base(long double base, int l1, int m1, int l2, int m2, int l3, int m3) {
  std::pair<int, std::complex<long double>> a[2], b[2], c[2];
  int na = real_to_complex(m1, a), nb = real_to_complex(m2, b), nc = real_to_complex(m3, c);
  std::complex<long double> acc = 0.0L;
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nb; ++j)
      for (int k = 0; k < nc; ++k) {
        int mu1 = a[i].first, mu2 = b[j].first, mu3 = c[k].first;
        if (mu1 + mu2 + mu3 != 0) continue;
        acc += a[i].second * b[j].second * c[k].second * wigner3j(l1, l2, l3, mu1, mu2, mu3);
      }
  return (double)(acc.real() * base);
}

static long double gaunt_base(int l1, int l2, int l3) {
  const long double pi = 3.141592653589793238462643383279502884L;
  return std::sqrt((long double)(2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1) / (4.0L * pi)) *
         wigner3j(l1, l2, l3, 0, 0, 0);
}

double real_gaunt(int l1, int m1, int l2, int m2, int l3, int m3) {
  if ((l1 + l2 + l3) & 1) return 0.0;
  if (l3 < std::abs(l1 - l2) || l3 > l1 + l2) return 0.0;
  return real_gaunt_base(gaunt_base(l1, l2, l3), l1, m1, l2, m2, l3, m3);
}

// Rows for q3 in [q3a, q3b), in table order.  For given (q2, q3) only the channels'
// l1 (triangle rule, even sum) and |m1| in {|m2| + |m3|, ||m2| - |m3||} can carry a
// nonzero weight (the complex components need mu1 + mu2 + mu3 = 0), so only those q1 are
// visited, in increasing order.
static void coo_rows(int L, double tol, const std::vector<int>& cid, const std::vector<long double>& base, int q3a,
                     int q3b, std::vector<CooRow>& rows) {
  const int NQ = (L + 1) * (L + 1);
  for (int q3 = q3a; q3 < q3b; ++q3) {
    const int l3 = l_of_q(q3), m3 = q3 - l3 * l3 - l3;
    for (int q2 = 0; q2 < NQ; ++q2) {
      const int l2 = l_of_q(q2), m2 = q2 - l2 * l2 - l2;
      const int a2 = std::abs(m2), a3 = std::abs(m3);
      for (int l1 = std::abs(l2 - l3); l1 <= std::min(L, l2 + l3); l1 += 2) {
        const int ci = (l1 * (L + 1) + l2) * (L + 1) + l3;
        const int c = cid[ci];
        if (c < 0) continue;
        int cand[4] = {-(a2 + a3), -std::abs(a2 - a3), std::abs(a2 - a3), a2 + a3};
        for (int i = 0; i < 4; ++i) {
          const int m1 = cand[i];
          if (i > 0 && m1 == cand[i - 1]) continue;
          if (std::abs(m1) > l1) continue;
          double g = real_gaunt_base(base[ci], l1, m1, l2, m2, l3, m3);
          if (std::fabs(g) > tol) rows.push_back({l1 * l1 + l1 + m1, q2, q3, c, g});
        }
      }
    }
  }
}

std::vector<CooRow> build_coo(int L, double tol) {
  std::vector<Channel> ch = enumerate_channels(L);
  const int NQ = (L + 1) * (L + 1);
  std::vector<int> cid((L + 1) * (L + 1) * (L + 1), -1);
  std::vector<long double> base(cid.size(), 0.0L);
  for (size_t i = 0; i < ch.size(); ++i) {
    const int ci = (ch[i].l1 * (L + 1) + ch[i].l2) * (L + 1) + ch[i].l3;
    cid[ci] = (int)i;
    base[ci] = gaunt_base(ch[i].l1, ch[i].l2, ch[i].l3);
  }
  // q3 ranges on host threads; the pieces are concatenated in q3 order
  const int nth = std::max(1, std::min({16, NQ, (int)std::thread::hardware_concurrency()}));
  std::vector<std::vector<CooRow>> part(nth);
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t)
    pool.emplace_back([&, t] { coo_rows(L, tol, cid, base, NQ * t / nth, NQ * (t + 1) / nth, part[t]); });
  for (auto& th : pool) th.join();
  std::vector<CooRow> rows;
  for (auto& p : part) rows.insert(rows.end(), p.begin(), p.end());
  return rows;
}

// ---------------------------------------------------------------- quadrature
// Symmetric tridiagonal eigenvalues by the implicit QL method with shifts.
static void tridiag_eigenvalues(std::vector<long double>& d, std::vector<long double> e) {
  int n = (int)d.size();
  e.push_back(0.0L);
  for (int l = 0; l < n; ++l) {
    int iter = 0, m;
    do {
      for (m = l; m < n - 1; ++m) {
        long double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-19L * dd) break;
      }
      if (m != l) {
        if (++iter > 200) throw std::runtime_error("QL iteration did not converge");
        long double g = (d[l + 1] - d[l]) / (2.0L * e[l]);
        long double r = std::hypot(g, 1.0L);
        g = d[m] - d[l] + e[l] / (g + (g >= 0 ? std::fabs(r) : -std::fabs(r)));
        long double s = 1.0L, c = 1.0L, p = 0.0L;
        int i;
        for (i = m - 1; i >= l; --i) {
          long double f = s * e[i], b = c * e[i];
          r = std::hypot(f, g);
          e[i + 1] = r;
          if (r == 0.0L) { d[i + 1] -= p; e[m] = 0.0L; break; }
          s = f / r; c = g / r;
          g = d[i + 1] - p;
          r = (d[i] - g) * s + 2.0L * c * b;
          p = s * r;
          d[i + 1] = g + p;
          g = c * r - b;
        }
        if (r == 0.0L && i >= l) continue;
        d[l] -= p; e[l] = g; e[m] = 0.0L;
      }
    } while (m != l);
  }
}

void gauss_rule(int kind, int n, double alpha, std::vector<double>& x, std::vector<double>& w) {
  if (n < 1) throw std::runtime_error("quadrature size must be >= 1");
  std::vector<long double> d(n), e(std::max(0, n - 1));
  long double a = alpha;
  for (int i = 0; i < n; ++i) {
    if (kind == 0) d[i] = 0.0L;
    else d[i] = 2.0L * i + a + 1.0L;
  }
  for (int i = 1; i < n; ++i) {
    if (kind == 0) e[i - 1] = (long double)i / std::sqrt(4.0L * i * i - 1.0L);
    else e[i - 1] = std::sqrt((long double)i * (i + a));
  }
  tridiag_eigenvalues(d, e);
  std::sort(d.begin(), d.end());
  x.assign(n, 0.0); w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    long double t = d[i], pn = 0, pm1 = 0;
    for (int it = 0; it < 6; ++it) {          // Newton polish on the three-term recurrence
      long double p0 = 1.0L, p1;
      if (kind == 0) {
        p1 = t;
        for (int k = 1; k < n; ++k) { long double p2 = ((2 * k + 1) * t * p1 - k * p0) / (k + 1); p0 = p1; p1 = p2; }
        if (n == 1) { p1 = t; p0 = 1.0L; }
        pn = p1; pm1 = p0;
        long double dp = n * (t * pn - pm1) / (t * t - 1.0L);
        t -= pn / dp;
      } else {
        p1 = 1.0L + a - t;
        if (n == 1) { pn = p1; pm1 = 1.0L; }
        else {
          for (int k = 1; k < n; ++k) { long double p2 = ((2 * k + 1 + a - t) * p1 - (k + a) * p0) / (k + 1); p0 = p1; p1 = p2; }
          pn = p1; pm1 = p0;
        }
        long double dp = (n * pn - (n + a) * pm1) / t;
        t -= pn / dp;
      }
    }
    // weights from the polished node
    long double p0 = 1.0L, p1;
    if (kind == 0) {
      p1 = t;
      for (int k = 1; k < n; ++k) { long double p2 = ((2 * k + 1) * t * p1 - k * p0) / (k + 1); p0 = p1; p1 = p2; }
      if (n == 1) { p1 = t; p0 = 1.0L; }
      long double dp = n * (t * p1 - p0) / (t * t - 1.0L);
      w[i] = (double)(2.0L / ((1.0L - t * t) * dp * dp));
    } else {
      p1 = 1.0L + a - t;
      if (n == 1) p0 = 1.0L;
      else for (int k = 1; k < n; ++k) { long double p2 = ((2 * k + 1 + a - t) * p1 - (k + a) * p0) / (k + 1); p0 = p1; p1 = p2; }
      // w = Gamma(n+a+1) t / (n! (n+a)^2 L_{n-1}(t)^2)
      long double lg = std::lgamma(n + a + 1.0L) - std::lgamma((long double)n + 1.0L);
      w[i] = (double)(std::exp(lg) * t / ((n + a) * (n + a) * p0 * p0));
    }
    x[i] = (double)t;
  }
}

}  // namespace wefq
