// Spectral (Miehe) split at one quadrature point, device side (gfx950).
//
// Section 2.1: with (lambda_i, v_i) the eigensystem of the strain e,
//   e^+ = sum_i <lambda_i>_+ v_i v_i^T,  e^- = e - e^+,
//   E^+ = lambda/2 <tr e>_+^2 + mu e^+ : e^+,  sigma^+ = lambda <tr e>_+ I + 2 mu e^+,
//   E^- = lambda/2 <tr e>_-^2 + mu e^- : e^-,  sigma^- = lambda <tr e>_- I + 2 mu e^-.
// Section 3.5 (derivative of the eigensystem): the derivative of e^+ in a
// direction de is taken in the eigenbasis with divided differences,
//   V^T de^+ V = F o (V^T de V),  F_ij = (<l_i>_+ - <l_j>_+) / (l_i - l_j),
// F_ij = [l_i >= 0] where l_i = l_j, which equals Algorithm 2 on distinct
// eigenvalues and does not depend on the eigenvectors on repeated ones.
// The tangent of g(phi~) sigma^+ + sigma^- is then
//   T(de) = lambda (g H + 1 - H) tr(de) I + 2 mu (de + (g - 1) de^+),  H = [tr e >= 0].
//
// Eigensystem: closed form in 2D (rotation angle from atan2); cyclic Jacobi
// rotations in 3D (a fixed number of sweeps, enough for FP64 on 3x3).
#pragma once
#include "internal.h"

namespace mfpff {

// SPLIT_NONE: the isotropic model without a split (the whole energy degraded); it runs the
// volumetric/deviatoric code with the tension branch taken at every point
enum SplitKind : int { SPLIT_AMOR = 0, SPLIT_MIEHE = 1, SPLIT_NONE = 2 };

// Voigt order of symmetric tensors: 2D (xx, yy, xy); 3D (xx, yy, zz, xy, xz, yz); strains in
// engineering form (shear entries doubled) so that the tangent matrix is symmetric
template <int DIM>
__host__ __device__ constexpr int n_voigt() { return DIM * (DIM + 1) / 2; }

template <int DIM>
struct VoigtPairs;
template <>
struct VoigtPairs<2> {
  static __device__ __forceinline__ int i(int k) { return k == 2 ? 0 : k; }
  static __device__ __forceinline__ int j(int k) { return k == 2 ? 1 : k; }
};
template <>
struct VoigtPairs<3> {
  static __device__ __forceinline__ int i(int k) { return k < 3 ? k : (k == 5 ? 1 : 0); }
  static __device__ __forceinline__ int j(int k) { return k < 3 ? k : (k == 3 ? 1 : 2); }
};

// coefficients of the cached spectral tangent per Gauss point: the upper triangle of the
// Voigt tangent, g'(phi) sigma^+ (Voigt), g''(phi) E^+ + Gc/eps
template <int DIM>
__host__ __device__ constexpr int n_qcoef_miehe() {
  return n_voigt<DIM>() * (n_voigt<DIM>() + 1) / 2 + n_voigt<DIM>() + 1;
}

template <int DIM, typename T>
struct Eig {
  T ev[DIM];
  T V[DIM][DIM];  // columns are eigenvectors
};

template <typename T>
__device__ __forceinline__ T pos(T x) {
  return x > T(0) ? x : T(0);
}

template <int DIM, typename T>
__device__ __forceinline__ Eig<DIM, T> eig_sym(const T (&e)[DIM][DIM]) {
  Eig<DIM, T> r;
  if constexpr (DIM == 2) {
    const T a = e[0][0], b = e[0][1], c = e[1][1];
    const T m = T(0.5) * (a + c), h = T(0.5) * (a - c);
    const T rad = sqrt(h * h + b * b);
    const T th = T(0.5) * atan2(b, h);
    const T cs = cos(th), sn = sin(th);
    r.ev[0] = m + rad;  // along (cs, sn)
    r.ev[1] = m - rad;  // along (-sn, cs)
    r.V[0][0] = cs;
    r.V[1][0] = sn;
    r.V[0][1] = -sn;
    r.V[1][1] = cs;
  } else {
    T A[3][3], V[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        A[i][j] = e[i][j];
        V[i][j] = i == j ? T(1) : T(0);
      }
    // cyclic Jacobi: each rotation zeroes A[p][q] (Jacobi's method; the rotation is chosen with
    // the smaller angle, t = sign(tau) / (|tau| + sqrt(1 + tau^2)))
#pragma unroll
    for (int sweep = 0; sweep < 6; ++sweep) {
#pragma unroll
      for (int pq = 0; pq < 3; ++pq) {
        const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
        // a rotation is taken unconditionally: where A[p][q] is already zero, t = 0 makes it the
        // identity, so every lane follows the same instruction stream (selects, no branch)
        const T apq = A[p][q];
        const bool live = apq != T(0);
        const T tau = live ? (A[q][q] - A[p][p]) / (T(2) * apq) : T(0);
        const T t = live ? (tau >= T(0) ? T(1) : T(-1)) / (fabs(tau) + sqrt(T(1) + tau * tau)) : T(0);
        const T cs = T(1) / sqrt(T(1) + t * t), sn = t * cs;
        // A <- J^T A J with J the rotation in the (p, q) plane
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T akp = A[k][p], akq = A[k][q];
          A[k][p] = cs * akp - sn * akq;
          A[k][q] = sn * akp + cs * akq;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T apk = A[p][k], aqk = A[q][k];
          A[p][k] = cs * apk - sn * aqk;
          A[q][k] = sn * apk + cs * aqk;
        }
        A[p][q] = A[q][p] = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T vkp = V[k][p], vkq = V[k][q];
          V[k][p] = cs * vkp - sn * vkq;
          V[k][q] = sn * vkp + cs * vkq;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      r.ev[i] = A[i][i];
#pragma unroll
      for (int j = 0; j < 3; ++j) r.V[i][j] = V[i][j];
    }
  }
  return r;
}

// divided differences of the positive part
template <int DIM, typename T>
__device__ __forceinline__ void divided_differences(const Eig<DIM, T>& g, T (&F)[DIM][DIM]) {
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      const T li = g.ev[i], lj = g.ev[j];
      F[i][j] = li == lj ? (li >= T(0) ? T(1) : T(0)) : (pos(li) - pos(lj)) / (li - lj);
    }
}

// out = V (F o (V^T de V)) V^T
template <int DIM, typename T>
__device__ __forceinline__ void dpositive(const Eig<DIM, T>& g, const T (&F)[DIM][DIM], const T (&de)[DIM][DIM],
                                          T (&out)[DIM][DIM]) {
  T W[DIM][DIM], M[DIM][DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      T s = 0;
#pragma unroll
      for (int l = 0; l < DIM; ++l) s += de[i][l] * g.V[l][b];
      W[i][b] = s;  // de V
    }
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      T s = 0;
#pragma unroll
      for (int i = 0; i < DIM; ++i) s += g.V[i][a] * W[i][b];
      M[a][b] = F[a][b] * s;  // F o (V^T de V)
    }
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      T s = 0;
#pragma unroll
      for (int a = 0; a < DIM; ++a) s += g.V[i][a] * M[a][b];
      W[i][b] = s;  // V M
    }
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      T s = 0;
#pragma unroll
      for (int b = 0; b < DIM; ++b) s += W[i][b] * g.V[j][b];
      out[i][j] = s;  // V M V^T
    }
}

// stresses and energies of the split at strain e
template <int DIM, typename T>
struct MiehePoint {
  Eig<DIM, T> eig;
  T t;                         // tr e
  bool H;                      // tr e >= 0
  T sp[DIM][DIM], sm[DIM][DIM];  // sigma^+, sigma^-
  T Ep, Em;
};

template <int DIM, typename T>
__device__ __forceinline__ MiehePoint<DIM, T> miehe_point(const T (&e)[DIM][DIM], T lam, T mu) {
  MiehePoint<DIM, T> r;
  r.eig = eig_sym<DIM, T>(e);
  T t = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) t += e[i][i];
  r.t = t;
  r.H = t >= T(0);
  const T tp = pos(t), tm = t - tp;
  T epp = 0, emm = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      T s = 0;
#pragma unroll
      for (int a = 0; a < DIM; ++a) s += r.eig.V[i][a] * pos(r.eig.ev[a]) * r.eig.V[j][a];
      const T em = e[i][j] - s;
      r.sp[i][j] = T(2) * mu * s + (i == j ? lam * tp : T(0));
      r.sm[i][j] = T(2) * mu * em + (i == j ? lam * tm : T(0));
      epp += s * s;
      emm += em * em;
    }
  r.Ep = T(0.5) * lam * tp * tp + mu * epp;
  r.Em = T(0.5) * lam * tm * tm + mu * emm;
  return r;
}

// T(de) = lambda (g H + 1 - H) tr(de) I + 2 mu (de + (g - 1) de^+)
template <int DIM, typename T>
__device__ __forceinline__ void miehe_tangent_apply(const Eig<DIM, T>& g, const T (&F)[DIM][DIM], bool H, T gt, T lam,
                                                    T mu, const T (&de)[DIM][DIM], T (&out)[DIM][DIM]) {
  T dp[DIM][DIM];
  dpositive<DIM, T>(g, F, de, dp);
  T tde = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) tde += de[i][i];
  const T vol = lam * (H ? gt : T(1)) * tde;
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) out[i][j] = T(2) * mu * (de[i][j] + (gt - T(1)) * dp[i][j]) + (i == j ? vol : T(0));
}

// Voigt tangent (upper triangle, row-major) of T at the point: column k is T applied to the
// unit engineering strain k
template <int DIM, typename T>
__device__ __forceinline__ void miehe_voigt_tangent(const Eig<DIM, T>& g, bool H, T gt, T lam, T mu,
                                                    T (&Dv)[n_voigt<DIM>()][n_voigt<DIM>()]) {
  constexpr int NV = n_voigt<DIM>();
  T F[DIM][DIM];
  divided_differences<DIM, T>(g, F);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    T de[DIM][DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) de[i][j] = T(0);
    const int a = VoigtPairs<DIM>::i(k), b = VoigtPairs<DIM>::j(k);
    if (a == b) {
      de[a][a] = T(1);
    } else {
      de[a][b] = T(0.5);
      de[b][a] = T(0.5);
    }
    T s[DIM][DIM];
    miehe_tangent_apply<DIM, T>(g, F, H, gt, lam, mu, de, s);
#pragma unroll
    for (int r = 0; r < NV; ++r) Dv[r][k] = s[VoigtPairs<DIM>::i(r)][VoigtPairs<DIM>::j(r)];
  }
}

}  // namespace mfpff
