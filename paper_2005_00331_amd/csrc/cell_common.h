// Device building blocks of the matrix-free cell kernels (gfx950).
//
// A workgroup holds CPB cells of (k+1)^d points each, one thread per (cell,
// point); nodes and Gauss points share that tensor shape.  Per-field tensors
// live in LDS as [field][cell][point].  Values at quadrature points come from
// d sum-factorised 1D sweeps with the basis table B; gradients from the
// collocation derivative C at the Gauss points; test integration runs the
// transposed collocation and basis sweeps (Section 3.4: the element operator
// is evaluated through the tensor-product structure of the unit cell).
#pragma once
#include "bounds.h"
#include "internal.h"
#include "miehe.h"

namespace mfpff {

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <int DIM, int K, int NT = kThreads>
struct Shape {
  static constexpr int NP = K + 1;
  static constexpr int P = ipow(NP, DIM);
  static constexpr int CPB = NT / P;
  static constexpr int NPTS = CPB * P;
  static constexpr int NBUF = DIM * DIM + DIM + 1;
};

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

// out[f][c][p] = sum_r mat[digit_dir(p)][r] * in[f][c][p with digit_dir = r]
template <int NP, int P, int NPTS, typename T>
__device__ __forceinline__ void sweep(const T* __restrict__ in, T* __restrict__ out, int nf,
                                      const T* __restrict__ mat, int dir, int tid) {
  if (tid >= NPTS) return;
  const int c = tid / P, p = tid - (tid / P) * P;
  const int st = dir == 0 ? 1 : (dir == 1 ? NP : NP * NP);
  const int dg = (p / st) % NP;
  const int base = c * P + p - dg * st;
  const T* m = mat + dg * NP;
  for (int f = 0; f < nf; ++f) {
    const T* src = in + f * NPTS + base;
    T acc = 0;
#pragma unroll
    for (int r = 0; r < NP; ++r) acc += m[r] * src[r * st];
    out[f * NPTS + c * P + p] = acc;
  }
}

// Derivative along dir at the own point from a value tensor (matrix C).
template <int NP, int P, int NPTS, typename T>
__device__ __forceinline__ T coll_deriv(const T* __restrict__ V, const T* __restrict__ C, int dir, int c, int p) {
  const int st = dir == 0 ? 1 : (dir == 1 ? NP : NP * NP);
  const int dg = (p / st) % NP;
  const T* src = V + c * P + p - dg * st;
  const T* m = C + dg * NP;
  T acc = 0;
#pragma unroll
  for (int r = 0; r < NP; ++r) acc += m[r] * src[r * st];
  return acc;
}

template <int DIM, int K>
__device__ __forceinline__ long long node_of(const Geom& g, long long cell, int p) {
  constexpr int NP = K + 1;
  const long long N = g.N, M = g.M;
  const unsigned uc = (unsigned)cell, un = (unsigned)N, q1 = uc / un;
  const long long cx = uc - q1 * un;
  const long long cy = q1 % un;
  const int i0 = p % NP, i1 = (p / NP) % NP;
  long long node = (K * cx + i0) + M * (K * cy + i1);
  long long clast = cy, ilast = i1;
  if (DIM == 3) {
    const long long cz = q1 / un;
    const int i2 = p / (NP * NP);
    node += M * M * (K * cz + i2);
    clast = cz;
    ilast = i2;
  }
  // slit mesh: a cell just above the slit plane takes the duplicates of its slit-plane nodes
  // that lie below x = 1/2 (the tip at x = 1/2 is shared)
  if (g.slit && clast == N / 2 && ilast == 0 && K * cx + i0 < K * N / 2)
    node = g.n_grid + (K * cx + i0) + (DIM == 3 ? (K * N / 2) * (K * cy + i1) : 0);
  return MFPFF_IN(node, g.n_nodes);
}

template <int NP, typename T>
struct SharedTables {
  T B[NP * NP], Bt[NP * NP], C[NP * NP], Ct[NP * NP], W[NP];
  __device__ void load(const Tables<T>* tab, int tid) {
    if (tid < NP * NP) {
      const int q = tid / NP, i = tid % NP;
      B[tid] = tab->B[q][i];
      Bt[i * NP + q] = tab->B[q][i];
      C[tid] = tab->C[q][i];
      Ct[i * NP + q] = tab->C[q][i];
    }
    if (tid < NP) W[tid] = tab->w[tid];
  }
};

// Field layout in buf0 before cell_compute:
//   operator modes: x_0..x_d, u_0..u_{d-1}, phi, phi~   (2d+3 fields)
//   residual:       u_0..u_{d-1}, phi, phi~              (d+2 fields)
// Runs the interpolation sweeps, the quadrature-point physics of eq. (G)
// (or eq. (residual)), and the test integration; returns the LDS tensor of
// the d+1 cell-local results [comp][cell][node].  All threads of the block
// must call it (it contains barriers); the caller has synchronised buf0.
// Tangent coefficients per Gauss point (MODE_QDATA writes them, QD products read them):
// [0] g(phi~) with its sign bit set where tr e < 0 (the split coefficients g K or K and 2 mu g are
// rebuilt from it with the same operations), [1 ..] g'(phi) sigma^+ (00, 11, (22), 01, (02, 12)),
// [last] g''(phi) E^+ + Gc/eps; qcf points at this block's [coefficient][point][cell]
template <int DIM>
__host__ __device__ constexpr int n_qcoef() { return 2 + DIM * (DIM + 1) / 2; }

template <int DIM, int K, typename T, int MODE, int NT = kThreads, bool QD = false>
__device__ const T* cell_compute(T* buf0, T* buf1, const SharedTables<K + 1, T>& st, const MatParams& mp, T h,
                                 int tid, const T* qcf = nullptr, T* qcf_out = nullptr) {
  using S = Shape<DIM, K, NT>;
  constexpr int NP = S::NP, P = S::P, NPTS = S::NPTS, CPB = S::CPB;
  constexpr bool XMODE = (MODE == MODE_APPLY || MODE == MODE_APPLY_T || MODE == MODE_BLOCK || MODE == MODE_ELEM);
  const bool miehe = mp.split == SPLIT_MIEHE;
  const int NQ = miehe ? n_qcoef_miehe<DIM>() : n_qcoef<DIM>();
  constexpr int NVG = n_voigt<DIM>();              // Voigt components
  constexpr int NTAN = NVG * (NVG + 1) / 2;        // stored entries of the spectral Voigt tangent
  // symmetric index pairs of the stored g'(phi) sigma^+ components
  constexpr int SI[6] = {0, 1, DIM == 3 ? 2 : 0, 0, 0, 1};
  constexpr int SJ[6] = {0, 1, DIM == 3 ? 2 : 1, 1, 2, 2};
  constexpr int NS = DIM * (DIM + 1) / 2;
  const int nf = (XMODE && QD) ? DIM + 1 : (XMODE ? (2 * DIM + 3) : DIM + 2);
  const bool inb = tid < NPTS;
  const int c = inb ? tid / P : 0;
  const int p = inb ? tid % P : 0;

  sweep<NP, P, NPTS, T>(buf0, buf1, nf, st.B, 0, tid);
  __syncthreads();
  sweep<NP, P, NPTS, T>(buf1, buf0, nf, st.B, 1, tid);
  __syncthreads();
  if (DIM == 3) {
    sweep<NP, P, NPTS, T>(buf0, buf1, nf, st.B, 2, tid);
    __syncthreads();
  }
  T* V = DIM == 2 ? buf0 : buf1;
  T* W = DIM == 2 ? buf1 : buf0;

  const T ih = T(1) / h;
  const T lam = (T)mp.lam, mu = (T)mp.mu, Gc = (T)mp.Gc, eps = (T)mp.eps, kap = (T)mp.kappa;
  const T Kb = lam + T(2) * mu / T(DIM);

  // ---- quadrature-point physics -> flux tensors in W:
  // [cc*DIM + m] u-test component cc along m; [DIM*DIM + m] phi gradient; [DIM*DIM + DIM] phi value
  if constexpr (MODE == MODE_QDATA) {
    // fields u_0..u_{d-1}, phi, phi~ interpolated in V: store the tangent coefficients
    if (inb) {
      const int o = c * P + p;
      T gu[DIM][DIM];
#pragma unroll
      for (int cc = 0; cc < DIM; ++cc)
#pragma unroll
        for (int m = 0; m < DIM; ++m) gu[cc][m] = coll_deriv<NP, P, NPTS, T>(V + cc * NPTS, st.C, m, c, p) * ih;
      const T ph = V[DIM * NPTS + o];
      const T pt = V[(DIM + 1) * NPTS + o];
      T e[DIM][DIM];
      T t = 0;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
#pragma unroll
        for (int j = 0; j < DIM; ++j) e[i][j] = T(0.5) * (gu[i][j] + gu[j][i]);
        t += e[i][i];
      }
      const bool H = t >= T(0) || mp.split == SPLIT_NONE;
      const T tp = H ? t : T(0);
      T devdev = 0;
#pragma unroll
      for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          const T dv = e[i][j] - (i == j ? t / T(DIM) : T(0));
          devdev += dv * dv;
        }
      const T Ep = T(0.5) * Kb * tp * tp + mu * devdev;
      const T gt = (T(1) - kap) * pt * pt + kap;
      const T dg = T(2) * (T(1) - kap) * ph;
      const T ddg = T(2) * (T(1) - kap);
      T* q = qcf_out + (long long)p * CPB + c;
      constexpr int QS = P * CPB;  // coefficient stride
      if (miehe) {
        // spectral split: upper triangle of the Voigt tangent, g'(phi) sigma^+, g'' E^+ + Gc/eps
        const MiehePoint<DIM, T> mpt = miehe_point<DIM, T>(e, lam, mu);
        T Dv[NVG][NVG];
        miehe_voigt_tangent<DIM, T>(mpt.eig, mpt.H, gt, lam, mu, Dv);
#pragma unroll
        for (int r = 0, kk = 0; r < NVG; ++r)
#pragma unroll
          for (int c2 = r; c2 < NVG; ++c2, ++kk) q[kk * QS] = Dv[r][c2];
#pragma unroll
        for (int k = 0; k < NVG; ++k) q[(NTAN + k) * QS] = dg * mpt.sp[SI[k]][SJ[k]];
        q[(NQ - 1) * QS] = ddg * mpt.Ep + Gc / eps;
        return V;
      }
      q[0] = H ? gt : -gt;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int i = SI[k], j = SJ[k];
        const T spij = T(2) * mu * (e[i][j] - (i == j ? t / T(DIM) : T(0))) + (i == j ? Kb * tp : T(0));
        q[(1 + k) * QS] = dg * spij;
      }
      q[(NQ - 1) * QS] = ddg * Ep + Gc / eps;
    }
    return V;
  }

  if constexpr (XMODE && QD) {
    // products from the cached tangent coefficients: only x is interpolated (fields x_0..x_d);
    // the fluxes stay in registers and pass through LDS one test component at a time, so the
    // block needs d+1 field slots per buffer instead of d^2+d+1
    T flux[DIM + 1][DIM + 1] = {};  // [test component][direction]; [d][d] = phi value flux
    const int o = c * P + p;
    if (inb) {
    T jxw = st.W[p % NP] * st.W[(p / NP) % NP] * h * h;
    if (DIM == 3) jxw *= st.W[p / (NP * NP)] * h;
    const T* q = qcf + (long long)p * CPB + c;
    constexpr int QS = P * CPB;
    const T gsv = q[0], cpp = q[(NQ - 1) * QS];
    const T gta = abs_bits(gsv);
    const T cvol = sign_bit(gsv) ? Kb : gta * Kb, cdev = gta * T(2) * mu;
    T gsp[DIM][DIM];
    if (MODE != MODE_BLOCK) {
      const int co = miehe ? NTAN : 1;  // first coupling coefficient
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const T v = q[(co + k) * QS];
        gsp[SI[k]][SJ[k]] = v;
        gsp[SJ[k]][SI[k]] = v;
      }
    }
    T gx[DIM][DIM];
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc)
#pragma unroll
      for (int m = 0; m < DIM; ++m) gx[cc][m] = coll_deriv<NP, P, NPTS, T>(V + cc * NPTS, st.C, m, c, p) * ih;
    const T dph = V[DIM * NPTS + o];
    T de[DIM][DIM];
    T dt = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
#pragma unroll
      for (int j = 0; j < DIM; ++j) de[i][j] = T(0.5) * (gx[i][j] + gx[j][i]);
      dt += de[i][i];
    }
    const T vol = cvol * dt;
    T Su[DIM][DIM];
    T spde = 0;
    if (miehe) {
      // Voigt tangent times the engineering strain of the trial function
      T dv[NVG], sv[NVG];
#pragma unroll
      for (int k = 0; k < NVG; ++k) dv[k] = (SI[k] == SJ[k] ? T(1) : T(2)) * de[SI[k]][SJ[k]];
#pragma unroll
      for (int r = 0; r < NVG; ++r) sv[r] = T(0);
#pragma unroll
      for (int r = 0, kk = 0; r < NVG; ++r)
#pragma unroll
        for (int c2 = r; c2 < NVG; ++c2, ++kk) {
          const T dvk = q[kk * QS];
          sv[r] += dvk * dv[c2];
          if (c2 != r) sv[c2] += dvk * dv[r];
        }
#pragma unroll
      for (int k = 0; k < NVG; ++k) {
        Su[SI[k]][SJ[k]] = sv[k];
        Su[SJ[k]][SI[k]] = sv[k];
      }
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        if (!miehe) Su[i][j] = cdev * (de[i][j] - (i == j ? dt / T(DIM) : T(0))) + (i == j ? vol : T(0));
        if (MODE == MODE_APPLY || MODE == MODE_ELEM) spde += gsp[i][j] * de[i][j];
        if (MODE == MODE_APPLY_T) Su[i][j] += dph * gsp[i][j];
      }
    const T fval = cpp * dph + spde;
    T fgrad[DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m) fgrad[m] = Gc * eps * coll_deriv<NP, P, NPTS, T>(V + DIM * NPTS, st.C, m, c, p) * ih;
    const T jg = jxw * ih;
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc)
#pragma unroll
      for (int m = 0; m < DIM; ++m) flux[cc][m] = jg * Su[cc][m];
#pragma unroll
    for (int m = 0; m < DIM; ++m) flux[DIM][m] = jg * fgrad[m];
    flux[DIM][DIM] = jxw * fval;
    }
    __syncthreads();  // every read of V is done
#pragma unroll
    for (int tc = 0; tc <= DIM; ++tc) {
      if (inb) {
#pragma unroll
        for (int m = 0; m < DIM; ++m) W[m * NPTS + o] = flux[tc][m];
      }
      __syncthreads();
      if (inb) {
        T sv = (tc == DIM) ? flux[DIM][DIM] : T(0);
#pragma unroll
        for (int m = 0; m < DIM; ++m) sv += coll_deriv<NP, P, NPTS, T>(W + m * NPTS, st.Ct, m, c, p);
        V[tc * NPTS + o] = sv;
      }
      __syncthreads();
    }
  }
  if (inb && !(XMODE && QD)) {
    const int o = c * P + p;
    T jxw = st.W[p % NP] * st.W[(p / NP) % NP] * h * h;
    if (DIM == 3) jxw *= st.W[p / (NP * NP)] * h;
    const int fu = XMODE ? DIM + 1 : 0;
    const int fph = fu + DIM, fpt = fu + DIM + 1;
    T gu[DIM][DIM];
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc)
#pragma unroll
      for (int m = 0; m < DIM; ++m) gu[cc][m] = coll_deriv<NP, P, NPTS, T>(V + (fu + cc) * NPTS, st.C, m, c, p) * ih;
    const T ph = V[fph * NPTS + o];
    const T pt = V[fpt * NPTS + o];
    T e[DIM][DIM];
    T t = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
#pragma unroll
      for (int j = 0; j < DIM; ++j) e[i][j] = T(0.5) * (gu[i][j] + gu[j][i]);
      t += e[i][i];
    }
    // tension/compression split of the trace: branch-free selects
    const bool H = t >= T(0) || mp.split == SPLIT_NONE;
    const T tp = H ? t : T(0);
    const T tm = H ? T(0) : t;
    T devdev = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        const T dv = e[i][j] - (i == j ? t / T(DIM) : T(0));
        devdev += dv * dv;
      }
    const T Ep = T(0.5) * Kb * tp * tp + mu * devdev;
    const T gt = (T(1) - kap) * pt * pt + kap;
    const T dg = T(2) * (T(1) - kap) * ph;
    const T ddg = T(2) * (T(1) - kap);
    T sp[DIM][DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j)
        sp[i][j] = T(2) * mu * (e[i][j] - (i == j ? t / T(DIM) : T(0))) + (i == j ? Kb * tp : T(0));
    // spectral split: sigma^+, sigma^-, E^+ from the eigensystem of e
    MiehePoint<DIM, T> mpt{};
    T Fdd[DIM][DIM] = {};
    if (miehe) {
      mpt = miehe_point<DIM, T>(e, lam, mu);
      divided_differences<DIM, T>(mpt.eig, Fdd);
    }
    const T EpS = miehe ? mpt.Ep : Ep;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j)
        if (miehe) sp[i][j] = mpt.sp[i][j];

    T Su[DIM][DIM];
    T fval = 0, fgrad[DIM];
    if (XMODE) {
      T gx[DIM][DIM];
#pragma unroll
      for (int cc = 0; cc < DIM; ++cc)
#pragma unroll
        for (int m = 0; m < DIM; ++m) gx[cc][m] = coll_deriv<NP, P, NPTS, T>(V + cc * NPTS, st.C, m, c, p) * ih;
      const T dph = V[DIM * NPTS + o];
      T de[DIM][DIM];
      T dt = 0;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
#pragma unroll
        for (int j = 0; j < DIM; ++j) de[i][j] = T(0.5) * (gx[i][j] + gx[j][i]);
        dt += de[i][i];
      }
      // delta sigma = g~ [K H dt I + 2 mu dev de] + K (1-H) dt I  (spectral split: miehe.h)
      const T vol = (H ? gt * Kb * dt : Kb * dt);
      T spde = 0;
      if (miehe) miehe_tangent_apply<DIM, T>(mpt.eig, Fdd, H, gt, lam, mu, de, Su);
#pragma unroll
      for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          if (!miehe) Su[i][j] = gt * T(2) * mu * (de[i][j] - (i == j ? dt / T(DIM) : T(0))) + (i == j ? vol : T(0));
          spde += sp[i][j] * de[i][j];
        }
      if (MODE == MODE_APPLY_T) {
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
          for (int j = 0; j < DIM; ++j) Su[i][j] += dg * dph * sp[i][j];
      }
      fval = (ddg * EpS + Gc / eps) * dph;
      if (MODE == MODE_APPLY || MODE == MODE_ELEM) fval += dg * spde;
#pragma unroll
      for (int m = 0; m < DIM; ++m) fgrad[m] = Gc * eps * coll_deriv<NP, P, NPTS, T>(V + DIM * NPTS, st.C, m, c, p) * ih;
    } else {  // residual
#pragma unroll
      for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) Su[i][j] = miehe ? gt * mpt.sp[i][j] + mpt.sm[i][j] : gt * sp[i][j] + (i == j ? Kb * tm : T(0));
      fval = dg * EpS - Gc * (T(1) - ph) / eps;
#pragma unroll
      for (int m = 0; m < DIM; ++m) fgrad[m] = Gc * eps * coll_deriv<NP, P, NPTS, T>(V + fph * NPTS, st.C, m, c, p) * ih;
    }
    const T jg = jxw * ih;
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc)
#pragma unroll
      for (int m = 0; m < DIM; ++m) W[(cc * DIM + m) * NPTS + o] = jg * Su[cc][m];
#pragma unroll
    for (int m = 0; m < DIM; ++m) W[(DIM * DIM + m) * NPTS + o] = jg * fgrad[m];
    W[(DIM * DIM + DIM) * NPTS + o] = jxw * fval;
  }
  if constexpr (!(XMODE && QD)) {
  __syncthreads();

  // ---- transposed collocation: s_t(q') = value flux + sum_m C^T along m of the grad flux
  if (inb) {
    const int o = c * P + p;
#pragma unroll
    for (int tc = 0; tc <= DIM; ++tc) {
      T s = (tc == DIM) ? W[(DIM * DIM + DIM) * NPTS + o] : T(0);
#pragma unroll
      for (int m = 0; m < DIM; ++m) s += coll_deriv<NP, P, NPTS, T>(W + (tc * DIM + m) * NPTS, st.Ct, m, c, p);
      V[tc * NPTS + o] = s;
    }
  }
  __syncthreads();
  }

  // ---- integrate: d sweeps with B^T
  sweep<NP, P, NPTS, T>(V, W, DIM + 1, st.Bt, 0, tid);
  __syncthreads();
  sweep<NP, P, NPTS, T>(W, V, DIM + 1, st.Bt, 1, tid);
  __syncthreads();
  if (DIM == 3) {
    sweep<NP, P, NPTS, T>(V, W, DIM + 1, st.Bt, 2, tid);
    __syncthreads();
    return W;
  }
  return V;
}

}  // namespace mfpff
