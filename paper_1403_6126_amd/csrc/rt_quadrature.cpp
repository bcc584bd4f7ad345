// Angle sets of Section 3 (host code): the discrete directions n_m and
// weights W_m with which J = sum W I, H = sum W n I, K = sum W n n I, the
// weights normalised to sum 1.  Sets that are symmetric under reflections
// and permutations of the axes give K_ii / J = 1/3 for isotropic I, which
// the method requires for any number of angles.
#include <algorithm>
#include <cmath>
#include <vector>

#include "rt.h"

namespace {

// n-point Gauss-Legendre nodes (ascending) and weights on [-1, 1].
bool gauss_legendre(int n, std::vector<double> &x, std::vector<double> &wt) {
  x.assign(n, 0.0);
  wt.assign(n, 0.0);
  const int half = n / 2;
  for (int i = 0; i < half; ++i) {
    // largest roots first: asymptotic guess cos(pi (i + 3/4)/(n + 1/2))
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int iter = 0; iter < 200; ++iter) {
      double pm1 = 1.0, p = z;
      for (int k = 2; k <= n; ++k) {
        const double pn = ((2.0 * k - 1.0) * z * p - (k - 1.0) * pm1) / k;
        pm1 = p;
        p = pn;
      }
      dp = n * (pm1 - z * p) / (1.0 - z * z);
      const double step = p / dp;
      z -= step;
      if (std::fabs(step) <= 1e-17) break;
    }
    double pm1 = 1.0, p = z;
    for (int k = 2; k <= n; ++k) {
      const double pn = ((2.0 * k - 1.0) * z * p - (k - 1.0) * pm1) / k;
      pm1 = p;
      p = pn;
    }
    dp = n * (pm1 - z * p) / (1.0 - z * z);
    const double wgt = 2.0 / ((1.0 - z * z) * dp * dp);
    x[n - 1 - i] = z;
    x[i] = -z;
    wt[n - 1 - i] = wgt;
    wt[i] = wgt;
  }
  return true;
}

double odd_double_factorial(int k) {
  double r = 1.0;
  for (int j = k; j > 1; j -= 2) r *= j;
  return r;
}

// Average over the unit sphere of x^(2a) y^(2b) z^(2c).
double sphere_mean(int a, int b, int c) {
  return odd_double_factorial(2 * a - 1) * odd_double_factorial(2 * b - 1) *
         odd_double_factorial(2 * c - 1) / odd_double_factorial(2 * (a + b + c) + 1);
}

// Solves the square system M x = r (row-major, k x k) by Gaussian
// elimination with partial pivoting.
bool solve_dense(std::vector<double> M, std::vector<double> r, int k, std::vector<double> &x) {
  for (int col = 0; col < k; ++col) {
    int piv = col;
    for (int i = col + 1; i < k; ++i)
      if (std::fabs(M[i * k + col]) > std::fabs(M[piv * k + col])) piv = i;
    if (M[piv * k + col] == 0.0) return false;
    if (piv != col) {
      for (int j = 0; j < k; ++j) std::swap(M[col * k + j], M[piv * k + j]);
      std::swap(r[col], r[piv]);
    }
    for (int i = col + 1; i < k; ++i) {
      const double f = M[i * k + col] / M[col * k + col];
      for (int j = col; j < k; ++j) M[i * k + j] -= f * M[col * k + j];
      r[i] -= f * r[col];
    }
  }
  x.assign(k, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    double s = r[i];
    for (int j = i + 1; j < k; ++j) s -= M[i * k + j] * x[j];
    x[i] = s / M[i * k + i];
  }
  return true;
}

// Level-symmetric set of even order N in [2, 16].
int level_symmetric(int order, std::vector<double> &mu, std::vector<double> &w) {
  const int half = order / 2;
  std::vector<double> lev2(half);
  for (int i = 1; i <= half; ++i) lev2[i - 1] = (6.0 * i - 5.0) / (3.0 * (order - 1));
  const int s = half + 2;
  struct Pt {
    int i, j, k;
  };
  std::vector<Pt> pts;
  for (int i = 1; i <= half; ++i)
    for (int j = 1; j <= half; ++j) {
      const int k = s - i - j;
      if (k >= 1 && k <= half) pts.push_back({i, j, k});
    }
  // permutation classes, identified by the sorted index triple
  auto key = [](const Pt &p) {
    int a[3] = {p.i, p.j, p.k};
    std::sort(a, a + 3);
    return a[0] * 10000 + a[1] * 100 + a[2];
  };
  std::vector<int> classes;
  for (const Pt &p : pts) classes.push_back(key(p));
  std::sort(classes.begin(), classes.end());
  classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
  const int nc = (int)classes.size();
  auto class_of = [&](const Pt &p) {
    return (int)(std::lower_bound(classes.begin(), classes.end(), key(p)) - classes.begin());
  };
  // candidate conditions in graded order; keep the first independent ones
  std::vector<double> sel_rows, sel_rhs, basis;  // basis: orthonormalised kept rows
  int kept = 0;
  for (int deg = 0; deg <= 2 * order && kept < nc; ++deg)
    for (int a = deg; a >= 0 && kept < nc; --a)
      for (int b = std::min(a, deg - a); b >= 0 && kept < nc; --b) {
        const int c = deg - a - b;
        if (c > b) continue;
        std::vector<double> row(nc, 0.0);
        for (const Pt &p : pts)
          row[class_of(p)] += std::pow(lev2[p.i - 1], a) * std::pow(lev2[p.j - 1], b) *
                              std::pow(lev2[p.k - 1], c);
        std::vector<double> res = row;
        for (int q = 0; q < kept; ++q) {
          double dot = 0.0;
          for (int t = 0; t < nc; ++t) dot += res[t] * basis[q * nc + t];
          for (int t = 0; t < nc; ++t) res[t] -= dot * basis[q * nc + t];
        }
        double rn = 0.0, n0 = 0.0;
        for (int t = 0; t < nc; ++t) {
          rn += res[t] * res[t];
          n0 += row[t] * row[t];
        }
        if (std::sqrt(rn) <= 1e-9 * std::sqrt(n0)) continue;
        for (int t = 0; t < nc; ++t) basis.push_back(res[t] / std::sqrt(rn));
        sel_rows.insert(sel_rows.end(), row.begin(), row.end());
        sel_rhs.push_back(sphere_mean(a, b, c));
        ++kept;
      }
  if (kept != nc) return RT_EUNSUPPORTED;
  std::vector<double> wc;
  if (!solve_dense(sel_rows, sel_rhs, nc, wc)) return RT_EUNSUPPORTED;
  for (double x : wc)
    if (!(x > 0.0)) return RT_EUNSUPPORTED;
  mu.clear();
  w.clear();
  for (int o = 0; o < 8; ++o) {
    const double sx = (o & 1) ? -1.0 : 1.0, sy = (o & 2) ? -1.0 : 1.0, sz = (o & 4) ? -1.0 : 1.0;
    for (const Pt &p : pts) {
      mu.push_back(sx * std::sqrt(lev2[p.i - 1]));
      mu.push_back(sy * std::sqrt(lev2[p.j - 1]));
      mu.push_back(sz * std::sqrt(lev2[p.k - 1]));
      w.push_back(wc[class_of(p)] / 8.0);
    }
  }
  return (int)w.size();
}

}  // namespace

extern "C" int rt_quadrature(int kind, int order, double *mu, double *w, int cap) {
  std::vector<double> m, wt;
  if (kind == RT_QUAD_GAUSS_LEGENDRE) {
    if (order < 2 || order % 2 || order > RT_MAX_ANGLES) return RT_EINVAL;
    std::vector<double> x, ww;
    gauss_legendre(order, x, ww);
    for (int i = 0; i < order; ++i) {
      m.push_back(x[i]);
      m.push_back(0.0);
      m.push_back(0.0);
      wt.push_back(0.5 * ww[i]);
    }
  } else if (kind == RT_QUAD_LEVEL_SYMMETRIC) {
    if (order < 2 || order % 2 || order > 16) return RT_EINVAL;
    const int st = level_symmetric(order, m, wt);
    if (st < 0) return st;
  } else {
    return RT_EINVAL;
  }
  const int n = (int)wt.size();
  if (mu && w) {
    if (cap < n) return RT_EINVAL;
    for (int i = 0; i < n; ++i) {
      w[i] = wt[i];
      for (int k = 0; k < 3; ++k) mu[3 * i + k] = m[3 * i + k];
    }
  }
  return n;
}
