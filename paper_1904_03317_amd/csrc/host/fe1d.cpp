#include "fe1d.hpp"

#include <cmath>

#include "common.hpp"

namespace gmg {

namespace {

// P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int m = 2; m <= n; ++m) {
    double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = n * (x * p1 - p0) / (x * x - 1.0);
}

// roots of P_n on (-1,1) by Newton from Chebyshev-like guesses
void gauss_legendre(int n, double* xs, double* ws) {
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(n, x, p, dp);
      double dx = p / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    double p, dp;
    legendre(n, x, p, dp);
    xs[n - 1 - i] = x;
    ws[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

// interior Gauss-Lobatto points: roots of P_k', Newton with
// P_k'' = (2x P_k' - k(k+1) P_k) / (1 - x^2).
void lobatto_interior(int k, double* xs) {
  for (int j = 1; j < k; ++j) {
    double x = -std::cos(M_PI * j / k);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(k, x, p, dp);
      double d2p = (2.0 * x * dp - k * (k + 1.0) * p) / (1.0 - x * x);
      double dx = dp / d2p;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    xs[j - 1] = x;
  }
}

}  // namespace

void lagrange_values(const FE1D& fe, double xi, double* out) {
  for (int j = 0; j < fe.n; ++j) {
    double v = 1.0;
    for (int m = 0; m < fe.n; ++m)
      if (m != j) v *= (xi - fe.x[m]) / (fe.x[j] - fe.x[m]);
    out[j] = v;
  }
}

void lagrange_derivs(const FE1D& fe, double xi, double* out) {
  for (int j = 0; j < fe.n; ++j) {
    double s = 0.0;
    for (int i = 0; i < fe.n; ++i) {
      if (i == j) continue;
      double t = 1.0 / (fe.x[j] - fe.x[i]);
      for (int m = 0; m < fe.n; ++m)
        if (m != j && m != i) t *= (xi - fe.x[m]) / (fe.x[j] - fe.x[m]);
      s += t;
    }
    out[j] = s;
  }
}

void lagrange_second_derivs(const FE1D& fe, double xi, double* out) {
  for (int j = 0; j < fe.n; ++j) {
    double s = 0.0;
    for (int a = 0; a < fe.n; ++a) {
      if (a == j) continue;
      for (int b = 0; b < fe.n; ++b) {
        if (b == j || b == a) continue;
        double t = 1.0 / ((fe.x[j] - fe.x[a]) * (fe.x[j] - fe.x[b]));
        for (int m = 0; m < fe.n; ++m)
          if (m != j && m != a && m != b) t *= (xi - fe.x[m]) / (fe.x[j] - fe.x[m]);
        s += t;
      }
    }
    out[j] = s;
  }
}

void gauss_01(int n, double* x, double* w) {
  gauss_legendre(n, x, w);
  for (int q = 0; q < n; ++q) {
    x[q] = 0.5 * (x[q] + 1.0);
    w[q] *= 0.5;
  }
}

FE1D make_fe1d(int k) {
  if (k < 1 || k > 4) fail(-1, "degree must be in 1..4");
  FE1D fe;
  fe.k = k;
  fe.n = k + 1;
  double t[5];
  t[0] = -1.0;
  t[k] = 1.0;
  if (k > 1) lobatto_interior(k, t + 1);
  for (int j = 0; j <= k; ++j) fe.x[j] = 0.5 * (t[j] + 1.0);
  double y[5];
  for (int j = 0; j <= k; ++j) y[j] = 0.5 * (fe.x[j] + (1.0 - fe.x[k - j]));
  for (int j = 0; j <= k; ++j) fe.x[j] = y[j];
  fe.x[0] = 0.0;
  fe.x[k] = 1.0;
  if (k % 2 == 0) fe.x[k / 2] = 0.5;

  const int nq = k + 1;
  double qx[5], qw[5];
  gauss_legendre(nq, qx, qw);
  for (int q = 0; q < nq; ++q) {
    qx[q] = 0.5 * (qx[q] + 1.0);
    qw[q] *= 0.5;
  }
  const int n = fe.n;
  for (int q = 0; q < nq; ++q) {
    double v[5], d[5];
    lagrange_values(fe, qx[q], v);
    lagrange_derivs(fe, qx[q], d);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        fe.M[i * n + j] += qw[q] * v[i] * v[j];
        fe.K[i * n + j] += qw[q] * d[i] * d[j];
      }
  }
  for (int i = 0; i <= k; ++i) fe.fam[i] = 0.5 * fe.x[i];
  for (int i = 1; i <= k; ++i) fe.fam[k + i] = 0.5 * (1.0 + fe.x[i]);
  for (int i = 0; i < 2 * k + 1; ++i) {
    double v[5];
    lagrange_values(fe, fe.fam[i], v);
    for (int J = 0; J < n; ++J) fe.E[i * n + J] = v[J];
  }
  return fe;
}

}  // namespace gmg
