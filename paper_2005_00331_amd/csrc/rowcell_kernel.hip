// Cell kernel for 2D Q1/Q2 levels with fused epilogues (gfx950).
//
// Each cell is shared by k+1 threads, thread (cell, r) for r = 0..k.  The
// threads are laid out r-major, so one wavefront holds one r for the 64 cells
// of an 8 x 8 tile and nothing diverges:
//  - thread r loads node row r of its cell and contracts it along x with the
//    1D basis B and its derivative D at the Gauss points (Section 3.4: the
//    element operator is applied through its tensor-product structure);
//  - the x-contractions go through LDS, and thread r contracts along y for the
//    Gauss-point row r, which gives values and gradients at its k+1 points;
//  - it evaluates eq. (G) at those points (tangent of the split stress, the
//    coupling g'(phi) sigma^+ and the phase-field terms);
//  - the transposed contractions run the same way back: along x for its point
//    row, through LDS, along y for its node row.
// LDS exchanges are double-buffered (two field kinds per buffer), so each
// exchange costs one barrier.  A workgroup computes 8 x 8 cells and owns the
// nodes of the upper-right 7 x 7 (the first row and column are the halo that
// completes the low-face nodes).  Results are added to an LDS node box in four
// colour phases (cells of one colour share no node, and the k+1 threads of a
// cell write different node rows), so the sum order is fixed; the owning
// threads then apply the epilogue of the operation (product, residual with the
// Chebyshev start, Chebyshev step).
#include "internal.h"
#include "bounds.h"
#include "gauss_tables.h"
#include "miehe.h"

namespace mfpff {

// element at a 32-bit byte offset from a uniform base: the address is the scalar base plus one
// vector offset (no 64-bit address arithmetic per access); the set-up keeps 2D Q1/Q2 levels
// below 2^28 nodes, so node * 8 fits in 32 bits
template <typename T>
__device__ __forceinline__ T& at_off(T* base, uint32_t boff) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff);
}
template <typename T>
__device__ __forceinline__ const T& at_off(const T* base, uint32_t boff) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
}

constexpr int kRowTile = 8;              // computed cells per direction per workgroup
constexpr int kRowOwn = kRowTile - 1;    // owned cells per direction
constexpr int kRowCells = kRowTile * kRowTile;  // one wavefront per r

long long rowcell_blocks_2d(const Geom& g) {
  const long long nt = (g.N + kRowOwn - 1) / kRowOwn;
  return nt * nt;
}
long long rowcell_qdata_len(const Geom& g, int split) {
  return rowcell_blocks_2d(g) * (split == SPLIT_MIEHE ? n_qcoef_miehe<2>() : kQCoef) * (g.k + 1) * (g.k + 1) * kRowCells;
}

// at most 128 VGPRs: four wavefronts per SIMD (the FP64 products issue well below peak with one or two);
// three for the spectral split (its Voigt tangent holds twice the coefficients), none for MODE_QDATA
// QD: the tangent coefficients come from a.qd instead of being computed from u, phi, phi~
// EARLY (grids of at most two workgroups per CU, where occupancy does not matter): the epilogue
// operands are loaded with the cell inputs, so the kernel waits for memory once, not twice
// SPLIT (products from the cache): the cached coefficients are those of the volumetric/
// deviatoric split (kQCoef per point) or of the spectral split (the Voigt tangent, the coupling
// and the phase coefficient, n_qcoef_miehe<2>() per point); MODE_QDATA writes either by a.m.split
template <int K, typename T, int MODE, int EPI, bool QD, bool EARLY, int SPLIT = SPLIT_AMOR>
__global__ __launch_bounds__(kRowCells*(K + 1)) __attribute__((amdgpu_waves_per_eu(EARLY || MODE == MODE_QDATA ? 1 : (SPLIT == SPLIT_MIEHE ? 3 : 4)))) void rowcell_kernel_2d(
    CellArgs<T> a, Epilogue<T> e) {
  constexpr int NP = K + 1;
  constexpr int NT = kRowCells * NP;
  constexpr int AN = K * kRowTile + 1;      // node box per direction
  constexpr int KS = NP * NP * kRowCells;   // one field kind: [q or i][row][cell]
  __shared__ T acc[3 * AN * AN];
  __shared__ T xch[2][2 * KS];
  const int tid = threadIdx.x;
  const int r = __builtin_amdgcn_readfirstlane(tid / kRowCells);  // uniform per wavefront
  const int cl = tid - r * kRowCells;
  const int li = cl % kRowTile, lj = cl / kRowTile;
  const Geom g = a.g;
  const int N = g.N;
  const long long M = g.M, nn = g.n_nodes;
  const int ntx = (N + kRowOwn - 1) / kRowOwn;
  // XCD-aware tile order: hardware block b runs on XCD b % 8, and each XCD takes a contiguous
  // range of tiles, so tiles that share halo nodes share that XCD's L2 (the cached coefficients
  // stay indexed by the hardware block, the same in the writing and the reading launch)
  const unsigned G = gridDim.x, bb = blockIdx.x, xcd = bb % 8, per = G / 8, rem = G % 8;
  const int lt = (int)MFPFF_IN(xcd * per + min(xcd, rem) + bb / 8, (long long)ntx * ntx);
  const int tx = lt % ntx, ty = lt / ntx;
  const int cx0 = tx * kRowOwn, cy0 = ty * kRowOwn;
  const int cx1 = min(cx0 + kRowOwn, N), cy1 = min(cy0 + kRowOwn, N);
  const int cx = cx0 - 1 + li, cy = cy0 - 1 + lj;
  const bool valid = cx >= 0 && cy >= 0 && cx < cx1 && cy < cy1;
  for (int i = tid; i < 3 * AN * AN; i += NT) acc[i] = T(0);

  using TB = ConstTab<K>;  // compile-time 1D tables (no scalar registers, zero entries folded)
  // table entries of row / column r (r is uniform per wavefront: scalar selects of constants)
  T Br[NP], Dr[NP], Bc[NP], Dc[NP];  // B[r][i], D[r][i], B[q][r], D[q][r]
  T wr = T(0);
#pragma unroll
  for (int rr = 0; rr < NP; ++rr) {
    if (r != rr) continue;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      Br[i] = (T)TB::B(rr, i);
      Dr[i] = (T)TB::D(rr, i);
      Bc[i] = (T)TB::B(i, rr);
      Dc[i] = (T)TB::D(i, rr);
    }
    wr = (T)TB::w(rr);
  }

  // ---- node row r of the cell: u_0, u_1, phi, phi~, x_0, x_1, x_phi (x zeroed at fixed dofs).
  // Every load is unconditional (invalid lanes read node 0 / their own tile slot) and the
  // masking is a bitwise select afterwards, so all loads of a thread are in flight together
  // (a select on the mask before the load made the compiler wait for the mask first).
  constexpr bool LIN = !QD;                // linearisation computed here
  constexpr bool XIN = MODE != MODE_QDATA;  // a trial vector is applied
  const long long nd0 = valid ? (long long)(K * cx) + M * (K * cy + r) : 0;
  T f[7][NP];
  uint8_t mk[NP];
#pragma unroll
  for (int i0 = 0; i0 < NP; ++i0) {
    const uint32_t nd = (uint32_t)MFPFF_IN(nd0 + i0, nn), bo = nd * (uint32_t)sizeof(T);
    if (LIN) {
      f[0][i0] = at_off(a.u, bo);
      f[1][i0] = at_off(a.u + nn, bo);
      f[2][i0] = at_off(a.phi, bo);
      f[3][i0] = at_off(a.phit, bo);
    }
    if (XIN) {
      mk[i0] = a.mask ? a.mask[nd] : (uint8_t)0;
      f[4][i0] = at_off(a.x, bo);
      f[5][i0] = at_off(a.x + nn, bo);
      f[6][i0] = at_off(a.x + 2 * nn, bo);
    }
  }
  // cached tangent coefficients of the Gauss row r, stored per tile (halo cells included) so
  // that every load of a wavefront reads 64 consecutive values
  constexpr int NQR = SPLIT == SPLIT_MIEHE ? n_qcoef_miehe<2>() : kQCoef;
  const T* qtile = a.qd + (long long)blockIdx.x * NQR * NP * NP * kRowCells + (r * NP) * kRowCells + cl;
  T qc[NQR][NP];
  if (QD) {
#pragma unroll
    for (int c = 0; c < NQR; ++c)
#pragma unroll
      for (int q0 = 0; q0 < NP; ++q0) qc[c][q0] = qtile[(c * NP * NP + q0) * kRowCells];
  }
#pragma unroll
  for (int i0 = 0; i0 < NP; ++i0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) f[q][i0] = LIN ? keep_if(f[q][i0], valid) : T(0);
    const bool ku = XIN && valid && !(mk[i0] & kMaskU), kp = XIN && valid && !(mk[i0] & kMaskPhi);
    f[4][i0] = keep_if(f[4][i0], ku);
    f[5][i0] = keep_if(f[5][i0], ku);
    f[6][i0] = keep_if(f[6][i0], kp);
  }
  if (QD) {
#pragma unroll
    for (int c = 0; c < NQR; ++c)
#pragma unroll
      for (int q0 = 0; q0 < NP; ++q0) qc[c][q0] = keep_if(qc[c][q0], valid);
  }

  // ---- owned nodes and their epilogue operands (resid: b, dinv; cheb: r, d, dinv, x), loaded
  // after the cell work so that they do not hold registers through it
  const int nox = K * (cx1 - cx0) + (cx1 == N ? 1 : 0);
  const int noy = K * (cy1 - cy0) + (cy1 == N ? 1 : 0);
  // owned nodes enumerated in a box of power-of-two width OW >= K * kRowOwn + 1 (mask and shift,
  // no division); slots past the tile's nox x noy nodes do nothing
  constexpr int OW = K == 1 ? 8 : 16;
  constexpr int OWL = K == 1 ? 3 : 4;
  static_assert(OW >= K * kRowOwn + 1 && (1 << OWL) == OW, "owned-node box");
  constexpr int MAXO = (OW * OW + NT - 1) / NT;
  struct Owned {
    uint32_t boff;  // byte offset of the node in a component block
    bool ok;
    int bo;
    uint8_t m;
    T ea[3], eb[3], ec[3], ex[3];
  };
  auto eload = [&](int j, Owned& o) {
    const int id = tid + j * NT;
    const int ox = id & (OW - 1), oy = id >> OWL;
    const bool ok = ox < nox && oy < noy;
    o.ok = ok;
    const uint32_t node = ok ? (uint32_t)MFPFF_IN((long long)(K * cx0 + ox) + M * (K * cy0 + oy), nn) : 0u;
    o.boff = node * (uint32_t)sizeof(T);
    o.bo = (K + oy) * AN + K + ox;
    o.m = (ok && a.mask) ? a.mask[node] : (uint8_t)0;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const long long cb = cc * nn;
      o.ea[cc] = o.eb[cc] = o.ec[cc] = o.ex[cc] = T(0);
      if (ok && EPI == EPI_RESID) {
        o.ea[cc] = at_off(e.b + cb, o.boff);
        if (e.z0) o.eb[cc] = at_off(e.dinv + cb, o.boff);
        o.ex[cc] = at_off(a.x + cb, o.boff);
      } else if (ok && EPI == EPI_CHEB) {
        o.ea[cc] = at_off(e.r + cb, o.boff);
        o.eb[cc] = at_off(e.d + cb, o.boff);
        o.ec[cc] = at_off(e.dinv + cb, o.boff);
        o.ex[cc] = at_off(a.x + cb, o.boff);
      } else if (ok) {
        o.ex[cc] = at_off(a.x + cb, o.boff);
      }
    }
  };
  auto efinish = [&](const Owned& o) {
    if (!o.ok) return;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const long long cb = cc * nn;
      const bool fixed = (cc < 2) ? (o.m & kMaskU) : (o.m & kMaskPhi);
      const T xo = o.ex[cc];
      const T gx = fixed ? xo : acc[cc * AN * AN + o.bo];
      if (EPI == EPI_APPLY) {
        at_off(e.y + cb, o.boff) = gx;
        if (e.xcopy) at_off(e.xcopy + cb, o.boff) = xo;
      } else if (EPI == EPI_RESID) {
        const T rv = o.ea[cc] - gx;
        at_off(e.y + cb, o.boff) = rv;
        if (e.z0) {
          const T zv = o.eb[cc] * rv * (cc < 2 ? e.ith_u : e.ith_p);
          at_off(e.z0 + cb, o.boff) = zv;
          at_off(e.d0 + cb, o.boff) = zv;
        }
      } else {
        const bool isu = cc < 2;
        const T dn = (isu ? e.c1u : e.c1p) * o.eb[cc] + (isu ? e.c2u : e.c2p) * o.ec[cc] * (o.ea[cc] - gx);
        at_off(e.d + cb, o.boff) = dn;
        const T zn = xo + dn;
        at_off(e.y + cb, o.boff) = zn;
        if (e.xout) at_off(e.xout + cb, o.boff) = at_off(e.xacc + cb, o.boff) + zn;
      }
    }
  };

  Owned pre[EARLY ? MAXO : 1];
  if (EARLY) {
#pragma unroll
    for (int j = 0; j < MAXO; ++j) eload(j, pre[j]);
  }

  int slot = 0;
  // publish two kinds of this thread's row (indexed [q][r]); after the barrier every
  // thread reads the NP rows of its own cell
  auto put = [&](const T (&k0)[NP], const T (&k1)[NP]) {
    T* s = xch[slot];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      s[(q * NP + r) * kRowCells + cl] = k0[q];
      s[KS + (q * NP + r) * kRowCells + cl] = k1[q];
    }
    __syncthreads();
  };
  auto get = [&](int kind, int q, int row) -> T { return xch[slot][kind * KS + (q * NP + row) * kRowCells + cl]; };
  // x-contraction of node row r: t = B f, td = D f at the Gauss abscissae
  auto xcon = [&](const T (&v)[NP], T (&t)[NP], T (&td)[NP]) {
#pragma unroll
    for (int q0 = 0; q0 < NP; ++q0) {
      T s = 0, sd = 0;
#pragma unroll
      for (int i0 = 0; i0 < NP; ++i0) {
        // terms whose table entry is zero are dropped (constant after unrolling): x + 0 v = x
        if (TB::B(q0, i0) != 0.0) s += (T)TB::B(q0, i0) * v[i0];
        if (TB::D(q0, i0) != 0.0) sd += (T)TB::D(q0, i0) * v[i0];
      }
      t[q0] = s;
      td[q0] = sd;
    }
  };
  // gradient (d/dxi_0, d/dxi_1) at Gauss row r from the exchanged t (kind 0) and td (kind 1)
  auto ygrad = [&](T (&g0)[NP], T (&g1)[NP]) {
#pragma unroll
    for (int q0 = 0; q0 < NP; ++q0) {
      T s0 = 0, s1 = 0;
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1) {
        s0 += Br[i1] * get(1, q0, i1);
        s1 += Dr[i1] * get(0, q0, i1);
      }
      g0[q0] = s0;
      g1[q0] = s1;
    }
  };

  const T h = (T)g.h, ih = T(1) / h;
  const T lam = (T)a.m.lam, mu = (T)a.m.mu, Gc = (T)a.m.Gc, eps = (T)a.m.eps, kap = (T)a.m.kappa;
  const T Kb = lam + T(2) * mu / T(2);

  // ---- linearisation at the Gauss points of row r
  T gu00[NP], gu01[NP], gu10[NP], gu11[NP], phq[NP], ptq[NP];
  if (LIN) {
    T t[NP], td[NP];
    xcon(f[0], t, td);
    put(t, td);
    ygrad(gu00, gu01);
    slot ^= 1;
    xcon(f[1], t, td);
    put(t, td);
    ygrad(gu10, gu11);
    slot ^= 1;
    T tp[NP], tt[NP];
    xcon(f[2], tp, td);
    xcon(f[3], tt, td);
    put(tp, tt);
#pragma unroll
    for (int q0 = 0; q0 < NP; ++q0) {
      T s0 = 0, s1 = 0;
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1) {
        s0 += Br[i1] * get(0, q0, i1);
        s1 += Br[i1] * get(1, q0, i1);
      }
      phq[q0] = s0;
      ptq[q0] = s1;
    }
    slot ^= 1;
  }
  // gs = g(phi~) with its sign bit set where tr e < 0 (compression), so the two split
  // coefficients g K or K and 2 mu g come from one stored value, bit for bit
  T gs[NP], sxx[NP], syy[NP], sxy[NP], cpp[NP];
  constexpr int NQM = n_qcoef_miehe<2>();
  const bool miehe_rt = a.m.split == SPLIT_MIEHE;  // MODE_QDATA: which coefficients to write
  T mq[MODE == MODE_QDATA ? NQM : 1][NP];
#pragma unroll
  for (int q0 = 0; q0 < NP; ++q0) {
    if (QD) {
      if (SPLIT == SPLIT_MIEHE) {
        // Voigt tangent (upper triangle) stays in qc[0..5]; coupling and phase coefficient
        gs[q0] = T(0);
        sxx[q0] = qc[6][q0];
        syy[q0] = qc[7][q0];
        sxy[q0] = qc[8][q0];
        cpp[q0] = qc[9][q0];
      } else {
        gs[q0] = qc[0][q0];
        sxx[q0] = qc[1][q0];
        syy[q0] = qc[2][q0];
        sxy[q0] = qc[3][q0];
        cpp[q0] = qc[4][q0];
      }
      continue;
    }
    const T exx = gu00[q0] * ih, eyy = gu11[q0] * ih;
    const T exy = T(0.5) * (gu01[q0] + gu10[q0]) * ih;
    const T t = exx + eyy;
    const bool H = t >= T(0) || a.m.split == SPLIT_NONE;
    const T tp = H ? t : T(0);
    const T dxx = exx - T(0.5) * t, dyy = eyy - T(0.5) * t;
    const T Ep = T(0.5) * Kb * tp * tp + mu * (dxx * dxx + dyy * dyy + T(2) * exy * exy);
    const T pt = ptq[q0];
    const T gt = (T(1) - kap) * pt * pt + kap;
    const T dg = T(2) * (T(1) - kap) * phq[q0];
    gs[q0] = H ? gt : -gt;
    sxx[q0] = dg * (T(2) * mu * dxx + Kb * tp);
    syy[q0] = dg * (T(2) * mu * dyy + Kb * tp);
    sxy[q0] = dg * (T(2) * mu * exy);
    cpp[q0] = T(2) * (T(1) - kap) * Ep + Gc / eps;
    if (MODE == MODE_QDATA && miehe_rt) {
      const T e2[2][2] = {{exx, exy}, {exy, eyy}};
      const MiehePoint<2, T> mpt = miehe_point<2, T>(e2, lam, mu);
      T Dv[3][3];
      miehe_voigt_tangent<2, T>(mpt.eig, mpt.H, gt, lam, mu, Dv);
      mq[0][q0] = Dv[0][0];
      mq[1][q0] = Dv[0][1];
      mq[2][q0] = Dv[0][2];
      mq[3][q0] = Dv[1][1];
      mq[4][q0] = Dv[1][2];
      mq[5][q0] = Dv[2][2];
      mq[6][q0] = dg * mpt.sp[0][0];
      mq[7][q0] = dg * mpt.sp[1][1];
      mq[8][q0] = dg * mpt.sp[0][1];
      mq[NQM - 1][q0] = T(2) * (T(1) - kap) * mpt.Ep + Gc / eps;
    }
  }

  if (MODE == MODE_QDATA) {
    if (valid && miehe_rt) {
      T* o = a.qd_out + (long long)blockIdx.x * NQM * NP * NP * kRowCells + (r * NP) * kRowCells + cl;
      constexpr int cs = NP * NP * kRowCells;
#pragma unroll
      for (int c = 0; c < NQM; ++c)
#pragma unroll
        for (int q0 = 0; q0 < NP; ++q0) o[c * cs + q0 * kRowCells] = mq[MODE == MODE_QDATA ? c : 0][q0];
    } else if (valid) {
      T* o = a.qd_out + (long long)blockIdx.x * kQCoef * NP * NP * kRowCells + (r * NP) * kRowCells + cl;
      constexpr int cs = NP * NP * kRowCells;  // coefficient stride
#pragma unroll
      for (int q0 = 0; q0 < NP; ++q0) {
        o[q0 * kRowCells] = gs[q0];
        o[cs + q0 * kRowCells] = sxx[q0];
        o[2 * cs + q0 * kRowCells] = syy[q0];
        o[3 * cs + q0 * kRowCells] = sxy[q0];
        o[4 * cs + q0 * kRowCells] = cpp[q0];
      }
    }
    return;
  }
  T cvol[NP], cdev[NP];
#pragma unroll
  for (int q0 = 0; q0 < NP; ++q0) {
    const T gt = abs_bits(gs[q0]);
    cvol[q0] = sign_bit(gs[q0]) ? Kb : gt * Kb;
    cdev[q0] = T(2) * mu * gt;
  }

  // ---- trial functions at the Gauss points of row r
  T gx00[NP], gx01[NP], gx10[NP], gx11[NP], pv[NP], pg0[NP], pg1[NP];
  {
    T t[NP], td[NP];
    xcon(f[4], t, td);
    put(t, td);
    ygrad(gx00, gx01);
    slot ^= 1;
    xcon(f[5], t, td);
    put(t, td);
    ygrad(gx10, gx11);
    slot ^= 1;
    xcon(f[6], t, td);
    put(t, td);
    ygrad(pg0, pg1);
#pragma unroll
    for (int q0 = 0; q0 < NP; ++q0) {
      T s = 0;
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1) s += Br[i1] * get(0, q0, i1);
      pv[q0] = s;
    }
    slot ^= 1;
  }

  // ---- fluxes (quadrature weight and Jacobian factors included)
  T F0x[NP], F1x[NP], F0y[NP], F1y[NP], Fv[NP], F0p[NP], F1p[NP];
#pragma unroll
  for (int q0 = 0; q0 < NP; ++q0) {
    const T wq = (T)TB::w(q0) * wr;  // JxW / h^2
    const T dxx = gx00[q0] * ih, dyy = gx11[q0] * ih;
    const T dxy = T(0.5) * (gx01[q0] + gx10[q0]) * ih;
    const T dt = dxx + dyy;
    const T vol = cvol[q0] * dt - cdev[q0] * T(0.5) * dt;
    T Sxx = cdev[q0] * dxx + vol;
    T Syy = cdev[q0] * dyy + vol;
    T Sxy = cdev[q0] * dxy;
    if (QD && SPLIT == SPLIT_MIEHE) {
      // Voigt tangent times the engineering strain (dxx, dyy, 2 dxy)
      const T d2 = T(2) * dxy;
      Sxx = qc[0][q0] * dxx + qc[1][q0] * dyy + qc[2][q0] * d2;
      Syy = qc[1][q0] * dxx + qc[3][q0] * dyy + qc[4][q0] * d2;
      Sxy = qc[2][q0] * dxx + qc[4][q0] * dyy + qc[5][q0] * d2;
    }
    const T dph = pv[q0];
    T fv = cpp[q0] * dph;
    if (MODE == MODE_APPLY) fv += sxx[q0] * dxx + syy[q0] * dyy + T(2) * sxy[q0] * dxy;
    if (MODE == MODE_APPLY_T) {
      Sxx += dph * sxx[q0];
      Syy += dph * syy[q0];
      Sxy += dph * sxy[q0];
    }
    // gradient fluxes carry JxW / h = w h; the value flux JxW = w h^2
    const T wg = wq * h;
    F0x[q0] = wg * Sxx;
    F1x[q0] = wg * Sxy;
    F0y[q0] = wg * Sxy;
    F1y[q0] = wg * Syy;
    Fv[q0] = wq * h * h * fv;
    F0p[q0] = wg * Gc * eps * pg0[q0] * ih;
    F1p[q0] = wg * Gc * eps * pg1[q0] * ih;
  }

  // ---- test functions: along x for Gauss row r, then along y for node row r
  // y[i1][i0] = sum_q1 B[q1][i1] (sum_q0 B[q0][i0] Fv + D[q0][i0] F0) + D[q1][i1] (sum_q0 B[q0][i0] F1)
  T y[3][NP];
  auto integ = [&](const T (&Fvv)[NP], const T (&F0)[NP], const T (&F1)[NP], bool has_v, T (&out)[NP]) {
    T ka[NP], kb[NP];
#pragma unroll
    for (int i0 = 0; i0 < NP; ++i0) {
      T sa = 0, sb = 0;
#pragma unroll
      for (int q0 = 0; q0 < NP; ++q0) {
        if (has_v && TB::B(q0, i0) != 0.0) sa += (T)TB::B(q0, i0) * Fvv[q0];
        if (TB::D(q0, i0) != 0.0) sa += (T)TB::D(q0, i0) * F0[q0];
        if (TB::B(q0, i0) != 0.0) sb += (T)TB::B(q0, i0) * F1[q0];
      }
      ka[i0] = sa;
      kb[i0] = sb;
    }
    put(ka, kb);
#pragma unroll
    for (int i0 = 0; i0 < NP; ++i0) {
      T s = 0;
#pragma unroll
      for (int q1 = 0; q1 < NP; ++q1) s += Bc[q1] * get(0, i0, q1) + Dc[q1] * get(1, i0, q1);
      out[i0] = s;
    }
    slot ^= 1;
  };
  integ(Fv, F0x, F1x, false, y[0]);
  integ(Fv, F0y, F1y, false, y[1]);
  integ(Fv, F0p, F1p, true, y[2]);

  // ---- colour-phased accumulation into the node box (fixed order)
  const int colour = (cx & 1) + 2 * (cy & 1);
  for (int ph = 0; ph < 4; ++ph) {
    if (valid && colour == ph) {
#pragma unroll
      for (int i0 = 0; i0 < NP; ++i0) {
        const int o = (K * lj + r) * AN + K * li + i0;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) acc[cc * AN * AN + o] += y[cc][i0];
      }
    }
    __syncthreads();
  }
  // ---- fused epilogue on the owned nodes
#pragma unroll
  for (int j = 0; j < MAXO; ++j) {
    if (EARLY) {
      efinish(pre[j]);
    } else {
      Owned on;
      eload(j, on);
      efinish(on);
    }
  }
}

template <int K, typename T>
static hipError_t launch_row_k(int mode, int epi, const CellArgs<T>& a, const Epilogue<T>& e, hipStream_t s) {
  const long long nb = rowcell_blocks_2d(a.g);
  const bool early = nb <= 512;
  dim3 grid((unsigned)nb), block(kRowCells * (K + 1));
  const bool miehe = a.m.split == SPLIT_MIEHE;
  if (miehe && !a.qd && mode != MODE_QDATA) return hipErrorInvalidValue;  // spectral products read the cache
#define MFPFF_R(MD, EP)                                                                                              \
  if (mode == MD && epi == EP) {                                                                                     \
    if (miehe && early)                                                                                              \
      hipLaunchKernelGGL((rowcell_kernel_2d<K, T, MD, EP, true, true, SPLIT_MIEHE>), grid, block, 0, s, a, e); \
    else if (miehe)                                                                                                  \
      hipLaunchKernelGGL((rowcell_kernel_2d<K, T, MD, EP, true, false, SPLIT_MIEHE>), grid, block, 0, s, a, e); \
    else if (a.qd && early)                                                                                          \
      hipLaunchKernelGGL((rowcell_kernel_2d<K, T, MD, EP, true, true>), grid, block, 0, s, a, e);          \
    else if (a.qd)                                                                                                   \
      hipLaunchKernelGGL((rowcell_kernel_2d<K, T, MD, EP, true, false>), grid, block, 0, s, a, e);         \
    else                                                                                                             \
      hipLaunchKernelGGL((rowcell_kernel_2d<K, T, MD, EP, false, false>), grid, block, 0, s, a, e);        \
    return hipGetLastError();                                                                                        \
  }
  if (mode == MODE_QDATA) {
    hipLaunchKernelGGL((rowcell_kernel_2d<K, T, MODE_QDATA, EPI_APPLY, false, false>), grid, block, 0, s, a, e);
    return hipGetLastError();
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
hipError_t launch_rowcell_2d(int mode, int epi, const CellArgs<T>& a, const Epilogue<T>& e, hipStream_t s) {
  if (a.g.dim != 2) return hipErrorInvalidValue;
  if (a.g.k == 1) return launch_row_k<1, T>(mode, epi, a, e, s);
  if (a.g.k == 2) return launch_row_k<2, T>(mode, epi, a, e, s);
  return hipErrorInvalidValue;
}

template hipError_t launch_rowcell_2d<double>(int, int, const CellArgs<double>&, const Epilogue<double>&, hipStream_t);
template hipError_t launch_rowcell_2d<float>(int, int, const CellArgs<float>&, const Epilogue<float>&, hipStream_t);

}  // namespace mfpff

MFPFF_BOUNDS_READER(bounds_hits_rowcell)
