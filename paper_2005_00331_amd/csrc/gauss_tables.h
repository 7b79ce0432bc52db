// The 1D finite-element tables of Q1-Q4 on the unit interval as compile-time constants, for the
// kernels that keep them in registers (the 2D row kernel and the 3D line kernel).
//
// Gauss-Legendre points of the k+1 point rule mapped to [0, 1] (closed forms: 1/2 -+ sqrt(3)/6;
// 1/2 and 1/2 -+ sqrt(15)/10; 1/2 -+ sqrt(3/7 -+ 2/7 sqrt(6/5))/2; 1/2, 1/2 -+ sqrt(5 -+
// 2 sqrt(10/7))/6), written out to 21 digits, with their weights; equispaced Lagrange nodes i/k.
// B[q][i] = l_i(x_q) and D[q][i] = l_i'(x_q) follow from the Lagrange product formula.  As
// constants they occupy no scalar registers (a table passed as a kernel argument takes
// 2 (k+1)^2 + k+1 doubles of them, which the compiler spills into vector lanes at Q3/Q4), and
// after unrolling the compiler folds the entries that are 0 or +-1 (at even k the middle Gauss
// point is a node).
#pragma once

namespace mfpff {

template <int K>
struct GaussRule;
template <>
struct GaussRule<1> {
  static __host__ __device__ constexpr double x(int q) { return q == 0 ? 0.21132486540518711775 : 0.78867513459481288225; }
  static __host__ __device__ constexpr double w(int) { return 0.5; }
};
template <>
struct GaussRule<2> {
  static __host__ __device__ constexpr double x(int q) {
    return q == 0 ? 0.11270166537925831148 : (q == 1 ? 0.5 : 0.88729833462074168852);
  }
  static __host__ __device__ constexpr double w(int q) { return q == 1 ? 4.0 / 9.0 : 5.0 / 18.0; }
};
template <>
struct GaussRule<3> {
  static __host__ __device__ constexpr double x(int q) {
    return q == 0 ? 0.069431844202973712388
                  : (q == 1 ? 0.33000947820757186760 : (q == 2 ? 0.66999052179242813240 : 0.93056815579702628761));
  }
  static __host__ __device__ constexpr double w(int q) {
    return (q == 0 || q == 3) ? 0.17392742256872692869 : 0.32607257743127307131;
  }
};
template <>
struct GaussRule<4> {
  static __host__ __device__ constexpr double x(int q) {
    return q == 0 ? 0.046910077030668003601
                  : (q == 1 ? 0.23076534494715845448
                            : (q == 2 ? 0.5 : (q == 3 ? 0.76923465505284154552 : 0.95308992296933199640)));
  }
  static __host__ __device__ constexpr double w(int q) {
    return (q == 0 || q == 4) ? 0.11846344252809454376 : ((q == 1 || q == 3) ? 0.23931433524968323402 : 128.0 / 450.0);
  }
};

template <int K>
struct ConstTab {
  static constexpr int NP = K + 1;
  static __host__ __device__ constexpr double node(int i) { return (double)i / K; }
  static __host__ __device__ constexpr double x(int q) { return GaussRule<K>::x(q); }
  static __host__ __device__ constexpr double w(int q) { return GaussRule<K>::w(q); }
  // l_i(x_q)
  static __host__ __device__ constexpr double B(int q, int i) {
    double v = 1.0;
    for (int m = 0; m <= K; ++m)
      if (m != i) v *= (x(q) - node(m)) / (node(i) - node(m));
    return v;
  }
  // l_i'(x_q) by the product rule
  static __host__ __device__ constexpr double D(int q, int i) {
    double d = 0.0;
    for (int m = 0; m <= K; ++m) {
      if (m == i) continue;
      double t = 1.0 / (node(i) - node(m));
      for (int j = 0; j <= K; ++j)
        if (j != i && j != m) t *= (x(q) - node(j)) / (node(i) - node(j));
      d += t;
    }
    return d;
  }
};

}  // namespace mfpff
