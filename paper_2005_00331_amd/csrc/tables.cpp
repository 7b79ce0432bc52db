// 1D finite-element tables on the unit interval (host, FP64).
// Gauss-Legendre points by Newton iteration on the Legendre polynomial
// (three-term recurrence), equispaced Lagrange values and derivatives by the
// product rule, and the collocation derivative on the Gauss points in
// barycentric form: C[q][r] = (a_q/a_r)/(x_q - x_r) for q != r,
// C[q][q] = sum_{j != q} 1/(x_q - x_j), a_i = prod_{j != i} (x_i - x_j).
#include <cmath>

#include "internal.h"

namespace mfpff {

static void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int j = 2; j <= n; ++j) {
    const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = n * (x * p1 - p0) / (x * x - 1.0);
}

static void gauss01(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(n, z, p, dp);
      const double dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    double p, dp;
    legendre(n, z, p, dp);
    // ascending order on [0, 1]
    x[n - 1 - i] = 0.5 * (z + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 0.5 * 2/((1-z^2) P'^2)
  }
}

void make_tables(int k, Tables<double>& t) {
  const int n = k + 1;
  double xq[kMaxDeg + 1], wq[kMaxDeg + 1], xi[kMaxDeg + 1];
  gauss01(n, xq, wq);
  for (int i = 0; i < n; ++i) xi[i] = (double)i / k;
  for (int q = 0; q < kMaxDeg + 1; ++q)
    for (int i = 0; i < kMaxDeg + 1; ++i) t.B[q][i] = t.D[q][i] = t.C[q][i] = 0.0;
  for (int q = 0; q < n; ++q) {
    t.w[q] = wq[q];
    for (int i = 0; i < n; ++i) {
      double v = 1.0;
      for (int m = 0; m < n; ++m)
        if (m != i) v *= (xq[q] - xi[m]) / (xi[i] - xi[m]);
      t.B[q][i] = v;
      double d = 0.0;
      for (int m = 0; m < n; ++m) {
        if (m == i) continue;
        double term = 1.0 / (xi[i] - xi[m]);
        for (int j = 0; j < n; ++j)
          if (j != i && j != m) term *= (xq[q] - xi[j]) / (xi[i] - xi[j]);
        d += term;
      }
      t.D[q][i] = d;
    }
  }
  double a[kMaxDeg + 1];
  for (int i = 0; i < n; ++i) {
    a[i] = 1.0;
    for (int j = 0; j < n; ++j)
      if (j != i) a[i] *= (xq[i] - xq[j]);
  }
  for (int q = 0; q < n; ++q)
    for (int r = 0; r < n; ++r) {
      if (q != r) {
        t.C[q][r] = (a[q] / a[r]) / (xq[q] - xq[r]);
      } else {
        double s = 0.0;
        for (int j = 0; j < n; ++j)
          if (j != q) s += 1.0 / (xq[q] - xq[j]);
        t.C[q][q] = s;
      }
    }
}

}  // namespace mfpff
