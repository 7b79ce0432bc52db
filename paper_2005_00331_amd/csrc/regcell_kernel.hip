// Register-resident cell kernel for 2D Q1/Q2 levels with fused epilogues (gfx950).
//
// One thread computes one whole cell: its (k+1)^2 nodal values of every field
// are loaded into registers, values and gradients at the Gauss points come
// from sum-factorised 1D contractions done in registers (the 1D tables are a
// by-value kernel argument, uniform across the wave, so they sit in scalar
// registers), the quadrature-point physics of eq. (G) runs on them and the
// transposed contractions give the cell's (k+1)^2 x 3 results.  There are no
// LDS sweeps and no barriers in the cell computation, so the latency chain of
// a workgroup is one gather, the arithmetic and one scatter.
//
// A workgroup of 16 x 16 threads computes 16 x 16 cells and owns the nodes of
// the upper-right 15 x 15 of them (the first row and column are the halo whose
// contributions complete the low-face nodes).  Results are added to an LDS node
// accumulator in four colour phases (cells of one colour share no node), so the
// sum order is fixed; the owning thread then applies the epilogue of the
// operation (product, residual with Chebyshev start, Chebyshev step).
#include "internal.h"

namespace mfpff {

namespace {

template <int NP, typename T>
struct Tab2 {
  T B[NP][NP];  // [q][i]
  T D[NP][NP];
  T w[NP];
};

// f[i1][i0] nodal values -> v, g0 (d/dxi_0), g1 (d/dxi_1) at Gauss points [q1][q0] (unit cell)
template <int NP, typename T>
__device__ __forceinline__ void interp(const T (&f)[NP][NP], const Tab2<NP, T>& tb, T (&v)[NP][NP], T (&g0)[NP][NP],
                                       T (&g1)[NP][NP], bool need_v) {
  T t[NP][NP], td[NP][NP];  // [q0][i1]
#pragma unroll
  for (int q0 = 0; q0 < NP; ++q0)
#pragma unroll
    for (int i1 = 0; i1 < NP; ++i1) {
      T s = 0, sd = 0;
#pragma unroll
      for (int i0 = 0; i0 < NP; ++i0) {
        s += tb.B[q0][i0] * f[i1][i0];
        sd += tb.D[q0][i0] * f[i1][i0];
      }
      t[q0][i1] = s;
      td[q0][i1] = sd;
    }
#pragma unroll
  for (int q1 = 0; q1 < NP; ++q1)
#pragma unroll
    for (int q0 = 0; q0 < NP; ++q0) {
      T sv = 0, s0 = 0, s1 = 0;
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1) {
        if (need_v) sv += tb.B[q1][i1] * t[q0][i1];
        s0 += tb.B[q1][i1] * td[q0][i1];
        s1 += tb.D[q1][i1] * t[q0][i1];
      }
      if (need_v) v[q1][q0] = sv;
      g0[q1][q0] = s0;
      g1[q1][q0] = s1;
    }
}

// values only
template <int NP, typename T>
__device__ __forceinline__ void interp_v(const T (&f)[NP][NP], const Tab2<NP, T>& tb, T (&v)[NP][NP]) {
  T t[NP][NP];
#pragma unroll
  for (int q0 = 0; q0 < NP; ++q0)
#pragma unroll
    for (int i1 = 0; i1 < NP; ++i1) {
      T s = 0;
#pragma unroll
      for (int i0 = 0; i0 < NP; ++i0) s += tb.B[q0][i0] * f[i1][i0];
      t[q0][i1] = s;
    }
#pragma unroll
  for (int q1 = 0; q1 < NP; ++q1)
#pragma unroll
    for (int q0 = 0; q0 < NP; ++q0) {
      T s = 0;
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1) s += tb.B[q1][i1] * t[q0][i1];
      v[q1][q0] = s;
    }
}

// y[i1][i0] = sum_q Fv N_i + F0 dN_i/dxi_0 + F1 dN_i/dxi_1 (fluxes [q1][q0], any of them may be absent)
template <int NP, typename T>
__device__ __forceinline__ void integrate(const T (&Fv)[NP][NP], const T (&F0)[NP][NP], const T (&F1)[NP][NP], bool has_v,
                                          const Tab2<NP, T>& tb, T (&y)[NP][NP]) {
  T sb[NP][NP], s0[NP][NP];  // [q0][i1]
#pragma unroll
  for (int q0 = 0; q0 < NP; ++q0)
#pragma unroll
    for (int i1 = 0; i1 < NP; ++i1) {
      T a = 0, b = 0;
#pragma unroll
      for (int q1 = 0; q1 < NP; ++q1) {
        a += (has_v ? tb.B[q1][i1] * Fv[q1][q0] : T(0)) + tb.D[q1][i1] * F1[q1][q0];
        b += tb.B[q1][i1] * F0[q1][q0];
      }
      sb[q0][i1] = a;
      s0[q0][i1] = b;
    }
#pragma unroll
  for (int i1 = 0; i1 < NP; ++i1)
#pragma unroll
    for (int i0 = 0; i0 < NP; ++i0) {
      T s = 0;
#pragma unroll
      for (int q0 = 0; q0 < NP; ++q0) s += tb.B[q0][i0] * sb[q0][i1] + tb.D[q0][i0] * s0[q0][i1];
      y[i1][i0] = s;
    }
}

}  // namespace

constexpr int kRegTile = 16;  // computed cells per direction per workgroup
constexpr int kRegOwn = kRegTile - 1;

long long regcell_blocks_2d(const Geom& g) {
  const long long nt = (g.N + kRegOwn - 1) / kRegOwn;
  return nt * nt;
}

template <int K, typename T, int MODE, int EPI>
__global__ __launch_bounds__(kRegTile* kRegTile) void regcell_kernel_2d(CellArgs<T> a, Epilogue<T> e, Tab2<K + 1, T> tb) {
  constexpr int NP = K + 1;
  constexpr int AN = K * kRegTile + 1;
  __shared__ T acc[3 * AN * AN];
  const Geom g = a.g;
  const int N = g.N;
  const long long M = g.M, nn = g.n_nodes;
  const int ntx = (N + kRegOwn - 1) / kRegOwn;
  const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
  const int cx0 = tx * kRegOwn, cy0 = ty * kRegOwn;
  const int cx1 = min(cx0 + kRegOwn, N), cy1 = min(cy0 + kRegOwn, N);
  const int li = threadIdx.x % kRegTile, lj = threadIdx.x / kRegTile;
  const int cx = cx0 - 1 + li, cy = cy0 - 1 + lj;
  const bool valid = cx >= 0 && cy >= 0 && cx < cx1 && cy < cy1;
  for (int i = threadIdx.x; i < 3 * AN * AN; i += blockDim.x) acc[i] = T(0);

  // ---- issue every global load of the cell up front (one memory round trip)
  T fin[7][NP][NP];  // u_0, u_1, phi, phi~, x_0, x_1, x_phi (x zeroed at fixed dofs)
  if (valid) {
#pragma unroll
    for (int i1 = 0; i1 < NP; ++i1)
#pragma unroll
      for (int i0 = 0; i0 < NP; ++i0) {
        const long long nd = (long long)(K * cx + i0) + M * (K * cy + i1);
        const uint8_t mk = a.mask ? a.mask[nd] : (uint8_t)0;
        fin[0][i1][i0] = a.u[nd];
        fin[1][i1][i0] = a.u[nn + nd];
        fin[2][i1][i0] = a.phi[nd];
        fin[3][i1][i0] = a.phit[nd];
        const T x0 = a.x[nd], x1 = a.x[nn + nd], x2 = a.x[2 * nn + nd];
        fin[4][i1][i0] = (mk & kMaskU) ? T(0) : x0;
        fin[5][i1][i0] = (mk & kMaskU) ? T(0) : x1;
        fin[6][i1][i0] = (mk & kMaskPhi) ? T(0) : x2;
      }
  }
  // ---- epilogue operands of the owned nodes, also loaded before the arithmetic
  const int nox = K * (cx1 - cx0) + (cx1 == N ? 1 : 0);
  const int noy = K * (cy1 - cy0) + (cy1 == N ? 1 : 0);
  const int nown = nox * noy;
  constexpr int MAXO = ((K * kRegOwn + 1) * (K * kRegOwn + 1) + kRegTile * kRegTile - 1) / (kRegTile * kRegTile);
  long long enode[MAXO];
  int ebo[MAXO];
  uint8_t em[MAXO];
  T ea[MAXO][3], eb[MAXO][3], ec[MAXO][3], ex[MAXO][3];  // resid: b, dinv; cheb: r, d, dinv, z
#pragma unroll
  for (int j = 0; j < MAXO; ++j) {
    const int o = threadIdx.x + j * kRegTile * kRegTile;
    const bool ok = o < nown;
    const int ox = ok ? o % nox : 0, oy = ok ? o / nox : 0;
    enode[j] = ok ? (long long)(K * cx0 + ox) + M * (K * cy0 + oy) : -1;
    ebo[j] = (K + oy) * AN + K + ox;
    em[j] = (ok && a.mask) ? a.mask[enode[j]] : (uint8_t)0;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const long long idx = cc * nn + enode[j];
      ea[j][cc] = eb[j][cc] = ec[j][cc] = ex[j][cc] = T(0);
      if (ok && EPI == EPI_RESID) {
        ea[j][cc] = e.b[idx];
        if (e.z0) eb[j][cc] = e.dinv[idx];
      } else if (ok && EPI == EPI_CHEB) {
        ea[j][cc] = e.r[idx];
        eb[j][cc] = e.d[idx];
        ec[j][cc] = e.dinv[idx];
        ex[j][cc] = a.x[idx];
      }
    }
  }

  T y[3][NP][NP];
  if (valid) {
    const T h = (T)g.h, ih = T(1) / h;
    const T lam = (T)a.m.lam, mu = (T)a.m.mu, Gc = (T)a.m.Gc, eps = (T)a.m.eps, kap = (T)a.m.kappa;
    const T Kb = lam + T(2) * mu / T(2);
    T gu00[NP][NP], gu01[NP][NP], gu10[NP][NP], gu11[NP][NP], dummy[NP][NP];
    interp<NP, T>(fin[0], tb, dummy, gu00, gu01, false);
    interp<NP, T>(fin[1], tb, dummy, gu10, gu11, false);
    T phq[NP][NP], ptq[NP][NP];
    interp_v<NP, T>(fin[2], tb, phq);
    interp_v<NP, T>(fin[3], tb, ptq);
    // per point: volumetric and deviatoric tangent factors, g'(phi) sigma^+, phi-phi coefficient
    T cvol[NP][NP], cdev[NP][NP], sxx[NP][NP], syy[NP][NP], sxy[NP][NP], cpp[NP][NP];
#pragma unroll
    for (int q1 = 0; q1 < NP; ++q1)
#pragma unroll
      for (int q0 = 0; q0 < NP; ++q0) {
        const T exx = gu00[q1][q0] * ih, eyy = gu11[q1][q0] * ih;
        const T exy = T(0.5) * (gu01[q1][q0] + gu10[q1][q0]) * ih;
        const T t = exx + eyy;
        const bool H = t >= T(0);
        const T tp = H ? t : T(0);
        const T dxx = exx - T(0.5) * t, dyy = eyy - T(0.5) * t;
        const T Ep = T(0.5) * Kb * tp * tp + mu * (dxx * dxx + dyy * dyy + T(2) * exy * exy);
        const T pt = ptq[q1][q0];
        const T gt = (T(1) - kap) * pt * pt + kap;
        const T dg = T(2) * (T(1) - kap) * phq[q1][q0];
        cvol[q1][q0] = H ? gt * Kb : Kb;
        cdev[q1][q0] = T(2) * mu * gt;
        sxx[q1][q0] = dg * (T(2) * mu * dxx + Kb * tp);
        syy[q1][q0] = dg * (T(2) * mu * dyy + Kb * tp);
        sxy[q1][q0] = dg * (T(2) * mu * exy);
        cpp[q1][q0] = T(2) * (T(1) - kap) * Ep + Gc / eps;
      }
    // ---- trial functions
    T gx00[NP][NP], gx01[NP][NP], gx10[NP][NP], gx11[NP][NP], pv[NP][NP], pg0[NP][NP], pg1[NP][NP];
    interp<NP, T>(fin[4], tb, dummy, gx00, gx01, false);
    interp<NP, T>(fin[5], tb, dummy, gx10, gx11, false);
    interp<NP, T>(fin[6], tb, pv, pg0, pg1, true);
    // ---- fluxes (scaled by the quadrature weight and the Jacobian factors)
    T F0x[NP][NP], F1x[NP][NP], F0y[NP][NP], F1y[NP][NP], Fv[NP][NP], F0p[NP][NP], F1p[NP][NP];
#pragma unroll
    for (int q1 = 0; q1 < NP; ++q1)
#pragma unroll
      for (int q0 = 0; q0 < NP; ++q0) {
        const T wq = tb.w[q0] * tb.w[q1];  // JxW / h^2
        const T dxx = gx00[q1][q0] * ih, dyy = gx11[q1][q0] * ih;
        const T dxy = T(0.5) * (gx01[q1][q0] + gx10[q1][q0]) * ih;
        const T dt = dxx + dyy;
        const T vol = cvol[q1][q0] * dt - cdev[q1][q0] * T(0.5) * dt;
        T Sxx = cdev[q1][q0] * dxx + vol;
        T Syy = cdev[q1][q0] * dyy + vol;
        T Sxy = cdev[q1][q0] * dxy;
        const T dph = pv[q1][q0];
        T fv = cpp[q1][q0] * dph;
        if (MODE == MODE_APPLY) fv += sxx[q1][q0] * dxx + syy[q1][q0] * dyy + T(2) * sxy[q1][q0] * dxy;
        if (MODE == MODE_APPLY_T) {
          Sxx += dph * sxx[q1][q0];
          Syy += dph * syy[q1][q0];
          Sxy += dph * sxy[q1][q0];
        }
        // gradient fluxes carry JxW / h = w h; value flux JxW = w h^2
        const T wg = wq * h;
        F0x[q1][q0] = wg * Sxx;
        F1x[q1][q0] = wg * Sxy;
        F0y[q1][q0] = wg * Sxy;
        F1y[q1][q0] = wg * Syy;
        Fv[q1][q0] = wq * h * h * fv;
        F0p[q1][q0] = wg * Gc * eps * pg0[q1][q0] * ih;
        F1p[q1][q0] = wg * Gc * eps * pg1[q1][q0] * ih;
      }
    integrate<NP, T>(dummy, F0x, F1x, false, tb, y[0]);
    integrate<NP, T>(dummy, F0y, F1y, false, tb, y[1]);
    integrate<NP, T>(Fv, F0p, F1p, true, tb, y[2]);
  }
  __syncthreads();
  // ---- colour-phased accumulation into the node box (fixed order)
  const int colour = (cx & 1) + 2 * (cy & 1);
  for (int ph = 0; ph < 4; ++ph) {
    if (valid && colour == ph) {
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1)
#pragma unroll
        for (int i0 = 0; i0 < NP; ++i0) {
          const int o = (K * lj + i1) * AN + K * li + i0;
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) acc[cc * AN * AN + o] += y[cc][i1][i0];
        }
    }
    __syncthreads();
  }
  // ---- fused epilogue on the owned nodes (operands already in registers)
#pragma unroll
  for (int j = 0; j < MAXO; ++j) {
    if (enode[j] < 0) continue;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const long long idx = cc * nn + enode[j];
      const bool fixed = (cc < 2) ? (em[j] & kMaskU) : (em[j] & kMaskPhi);
      const T xo = (EPI == EPI_CHEB) ? ex[j][cc] : (fixed ? a.x[idx] : T(0));
      const T gx = fixed ? xo : acc[cc * AN * AN + ebo[j]];
      if (EPI == EPI_APPLY) {
        e.y[idx] = gx;
      } else if (EPI == EPI_RESID) {
        const T rv = ea[j][cc] - gx;
        e.y[idx] = rv;
        if (e.z0) {
          const T zv = eb[j][cc] * rv * (cc < 2 ? e.ith_u : e.ith_p);
          e.z0[idx] = zv;
          e.d0[idx] = zv;
        }
      } else {
        const bool isu = cc < 2;
        const T dn = (isu ? e.c1u : e.c1p) * eb[j][cc] + (isu ? e.c2u : e.c2p) * ec[j][cc] * (ea[j][cc] - gx);
        e.d[idx] = dn;
        const T zn = xo + dn;
        e.y[idx] = zn;
        if (e.xout) e.xout[idx] = e.xacc[idx] + zn;
      }
    }
  }
}

template <int K, typename T>
static hipError_t launch_reg_k(int mode, int epi, const CellArgs<T>& a, const Epilogue<T>& e, const Tables<double>& t64,
                               hipStream_t s) {
  Tab2<K + 1, T> tb;
  for (int q = 0; q <= K; ++q) {
    tb.w[q] = (T)t64.w[q];
    for (int i = 0; i <= K; ++i) {
      tb.B[q][i] = (T)t64.B[q][i];
      tb.D[q][i] = (T)t64.D[q][i];
    }
  }
  const long long nb = regcell_blocks_2d(a.g);
  dim3 grid((unsigned)nb), block(kRegTile * kRegTile);
#define MFPFF_R(MD, EP)                                                                                 \
  if (mode == MD && epi == EP) {                                                                        \
    hipLaunchKernelGGL((regcell_kernel_2d<K, T, MD, EP>), grid, block, 0, s, a, e, tb);                 \
    return hipGetLastError();                                                                           \
  }
  MFPFF_R(MODE_APPLY, EPI_APPLY)
  MFPFF_R(MODE_APPLY_T, EPI_APPLY)
  MFPFF_R(MODE_BLOCK, EPI_APPLY)
  MFPFF_R(MODE_APPLY, EPI_RESID)
  MFPFF_R(MODE_BLOCK, EPI_CHEB)
#undef MFPFF_R
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_regcell_2d(int mode, int epi, const CellArgs<T>& a, const Epilogue<T>& e, const Tables<double>& t64,
                             hipStream_t s) {
  if (a.g.dim != 2) return hipErrorInvalidValue;
  if (a.g.k == 1) return launch_reg_k<1, T>(mode, epi, a, e, t64, s);
  if (a.g.k == 2) return launch_reg_k<2, T>(mode, epi, a, e, t64, s);
  return hipErrorInvalidValue;
}

template hipError_t launch_regcell_2d<double>(int, int, const CellArgs<double>&, const Epilogue<double>&, const Tables<double>&,
                                              hipStream_t);
template hipError_t launch_regcell_2d<float>(int, int, const CellArgs<float>&, const Epilogue<float>&, const Tables<double>&,
                                             hipStream_t);

}  // namespace mfpff
