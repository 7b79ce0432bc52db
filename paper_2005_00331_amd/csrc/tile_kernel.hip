// Owner-computes cell kernel for 2D levels with fused vector epilogues (gfx950).
//
// A workgroup owns the nodes of a TT x TT tile of cells and computes every
// cell that touches them: its own cells plus one halo layer on the low side
// (the neighbour tile owns the shared low-face nodes, so the halo cells are
// the only redundant work).  Cell results are summed into an LDS node
// accumulator in a fixed order (batch, then candidate cell), so the product
// is deterministic and needs no atomics and no pre-initialised output.
// Because each owned node's value is complete inside the workgroup, the
// vector update that consumes it runs in the same kernel:
//   EPI_APPLY : y = G^ x
//   EPI_RESID : r = b - G^ x   (optionally z = D^-1 r / theta, d = z: the
//               start of the Chebyshev smoother)
//   EPI_CHEB  : t = diag(G^_uu, G^_phiphi) z; d = c1 d + c2 D^-1 (r - t);
//               z' = z + d (one Chebyshev-Jacobi step of the smoother,
//               Section 3.3), optionally x' = x + z'.
#include "bounds.h"
#include "cell_common.h"

namespace mfpff {

template <int K>
struct Tile2 {
  static constexpr int TT = K == 1 ? 16 : (K == 2 ? 8 : (K == 3 ? 6 : 4));
};

long long tile_blocks_2d(const Geom& g) {
  const int TT = g.k == 1 ? 16 : (g.k == 2 ? 8 : (g.k == 3 ? 6 : 4));
  const long long nt = (g.N + TT - 1) / TT;
  return nt * nt;
}

template <int K, typename T, int MODE, int EPI>
__global__ __launch_bounds__(kThreads) void tile_kernel_2d(CellArgs<T> a, Epilogue<T> e, const Tables<T>* __restrict__ tab) {
  constexpr int DIM = 2;
  using S = Shape<DIM, K>;
  constexpr int NP = S::NP, P = S::P, CPB = S::CPB, NPTS = S::NPTS, NBUF = S::NBUF;
  constexpr int TT = Tile2<K>::TT;
  constexpr int AN = (K * TT + 1) * (K * TT + 1);
  __shared__ SharedTables<NP, T> st;
  __shared__ T buf0[NBUF * NPTS];
  __shared__ T buf1[NBUF * NPTS];
  __shared__ T acc[(DIM + 1) * AN];

  const int tid = threadIdx.x;
  st.load(tab, tid);
  const Geom g = a.g;
  const int N = g.N;
  const long long M = g.M, nn = g.n_nodes;
  const int ntx = (N + TT - 1) / TT;
  // XCD-aware tile order: hardware block b runs on XCD b % 8, and each XCD takes a contiguous range
  // of tiles, so tiles that share halo nodes share that XCD's L2
  const unsigned G = gridDim.x, bb = blockIdx.x, xcd = bb % 8, per = G / 8, rem = G % 8;
  const int lt = (int)(xcd * per + min(xcd, rem) + bb / 8);
  const int tx = lt % ntx, ty = lt / ntx;
  const int cx0 = tx * TT, cy0 = ty * TT;
  const int cx1 = min(cx0 + TT, N), cy1 = min(cy0 + TT, N);
  const int ccx0 = max(cx0 - 1, 0), ccy0 = max(cy0 - 1, 0);
  const int ncx = cx1 - ccx0, ncy = cy1 - ccy0;
  const int ncomp = ncx * ncy;
  const int nox = K * (cx1 - cx0) + (cx1 == N ? 1 : 0);
  const int noy = K * (cy1 - cy0) + (cy1 == N ? 1 : 0);
  const int nown = nox * noy;
  for (int i = tid; i < (DIM + 1) * AN; i += kThreads) acc[i] = T(0);

  const bool inb = tid < NPTS;
  const int c = inb ? tid / P : 0;
  const int p = inb ? tid % P : 0;
  const int nbatch = (ncomp + CPB - 1) / CPB;
  for (int b = 0; b < nbatch; ++b) {
    // ---- gather the batch's cells
    const int ci = b * CPB + c;
    const bool valid = inb && ci < ncomp;
    if (inb) {
      const int o = c * P + p;
      long long node = 0;
      uint8_t mk = 0;
      if (valid) {
        const int cx = ccx0 + ci % ncx, cy = ccy0 + ci / ncx;
        node = MFPFF_IN((long long)(K * cx + p % NP) + M * (K * cy + p / NP), nn);
        mk = a.mask ? a.mask[node] : (uint8_t)0;
      }
#pragma unroll
      for (int cc = 0; cc <= DIM; ++cc) {
        const bool fixed = (cc < DIM) ? (mk & kMaskU) : (mk & kMaskPhi);
        buf0[cc * NPTS + o] = (valid && !fixed) ? a.x[cc * nn + node] : T(0);
      }
#pragma unroll
      for (int cc = 0; cc < DIM; ++cc) buf0[(DIM + 1 + cc) * NPTS + o] = valid ? a.u[cc * nn + node] : T(0);
      buf0[(2 * DIM + 1) * NPTS + o] = valid ? a.phi[node] : T(0);
      buf0[(2 * DIM + 2) * NPTS + o] = valid ? a.phit[node] : T(0);
    }
    __syncthreads();
    const T* R = cell_compute<DIM, K, T, MODE>(buf0, buf1, st, a.m, (T)g.h, tid);
    // ---- sum this batch's cell results into the owned nodes (fixed order)
    const int lo = b * CPB, hi = b * CPB + CPB;
    for (int o = tid; o < nown; o += kThreads) {
      const int gi = K * cx0 + o % nox, gj = K * cy0 + o / nox;
      int cxs[2], lxs[2], nxs = 0, cys[2], lys[2], nys = 0;
      if (gi % K == 0) {
        if (gi / K - 1 >= ccx0) { cxs[nxs] = gi / K - 1; lxs[nxs++] = K; }
        if (gi / K < cx1) { cxs[nxs] = gi / K; lxs[nxs++] = 0; }
      } else {
        cxs[nxs] = gi / K; lxs[nxs++] = gi % K;
      }
      if (gj % K == 0) {
        if (gj / K - 1 >= ccy0) { cys[nys] = gj / K - 1; lys[nys++] = K; }
        if (gj / K < cy1) { cys[nys] = gj / K; lys[nys++] = 0; }
      } else {
        cys[nys] = gj / K; lys[nys++] = gj % K;
      }
      T s[DIM + 1] = {};
      for (int jy = 0; jy < nys; ++jy)
        for (int jx = 0; jx < nxs; ++jx) {
          const int cidx = (cys[jy] - ccy0) * ncx + (cxs[jx] - ccx0);
          if (cidx >= lo && cidx < hi) {
            const int off = (cidx - lo) * P + lxs[jx] + NP * lys[jy];
#pragma unroll
            for (int cc = 0; cc <= DIM; ++cc) s[cc] += R[cc * NPTS + off];
          }
        }
#pragma unroll
      for (int cc = 0; cc <= DIM; ++cc) acc[cc * AN + o] += s[cc];
    }
    __syncthreads();
  }

  // ---- fused epilogue on the owned nodes
  for (int o = tid; o < nown; o += kThreads) {
    const long long node = MFPFF_IN((long long)(K * cx0 + o % nox) + M * (K * cy0 + o / nox), nn);
    const uint8_t mk = a.mask ? a.mask[node] : (uint8_t)0;
#pragma unroll
    for (int cc = 0; cc <= DIM; ++cc) {
      const long long idx = cc * nn + node;
      const bool fixed = (cc < DIM) ? (mk & kMaskU) : (mk & kMaskPhi);
      const T gx = fixed ? a.x[idx] : acc[cc * AN + o];
      if (EPI == EPI_APPLY) {
        e.y[idx] = gx;
        if (e.xcopy) e.xcopy[idx] = a.x[idx];
      } else if (EPI == EPI_RESID) {
        const T rv = e.b[idx] - gx;
        e.y[idx] = rv;
        if (e.z0) {
          const T zv = e.dinv[idx] * rv * (cc < DIM ? e.ith_u : e.ith_p);
          e.z0[idx] = zv;
          e.d0[idx] = zv;
        }
      } else {  // EPI_CHEB
        const bool isu = cc < DIM;
        const T dn = (isu ? e.c1u : e.c1p) * e.d[idx] + (isu ? e.c2u : e.c2p) * e.dinv[idx] * (e.r[idx] - gx);
        e.d[idx] = dn;
        const T zn = a.x[idx] + dn;
        e.y[idx] = zn;
        if (e.xout) e.xout[idx] = e.xacc[idx] + zn;
      }
    }
  }
}

template <int K, typename T>
static hipError_t launch_tile_k(int mode, int epi, const CellArgs<T>& a, const Epilogue<T>& e, const Tables<T>* tab,
                                hipStream_t s) {
  const long long nb = tile_blocks_2d(a.g);
  dim3 grid((unsigned)nb), block(kThreads);
#define MFPFF_T(MD, EP) \
  if (mode == MD && epi == EP) { hipLaunchKernelGGL((tile_kernel_2d<K, T, MD, EP>), grid, block, 0, s, a, e, tab); return hipGetLastError(); }
  MFPFF_T(MODE_APPLY, EPI_APPLY)
  MFPFF_T(MODE_APPLY_T, EPI_APPLY)
  MFPFF_T(MODE_BLOCK, EPI_APPLY)
  MFPFF_T(MODE_APPLY, EPI_RESID)
  MFPFF_T(MODE_BLOCK, EPI_CHEB)
#undef MFPFF_T
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_tile_2d(int mode, int epi, const CellArgs<T>& a, const Epilogue<T>& e, const Tables<T>* tab, hipStream_t s) {
  if (a.g.dim != 2) return hipErrorInvalidValue;
  switch (a.g.k) {
    case 1: return launch_tile_k<1, T>(mode, epi, a, e, tab, s);
    case 2: return launch_tile_k<2, T>(mode, epi, a, e, tab, s);
    case 3: return launch_tile_k<3, T>(mode, epi, a, e, tab, s);
    case 4: return launch_tile_k<4, T>(mode, epi, a, e, tab, s);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_tile_2d<double>(int, int, const CellArgs<double>&, const Epilogue<double>&, const Tables<double>*,
                                           hipStream_t);
template hipError_t launch_tile_2d<float>(int, int, const CellArgs<float>&, const Epilogue<float>&, const Tables<float>*,
                                          hipStream_t);

}  // namespace mfpff

MFPFF_BOUNDS_READER(bounds_hits_tile)
