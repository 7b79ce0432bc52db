// Matrix-free cell kernels for the phase-field fracture Jacobian (gfx950).
//
// One workgroup of 256 threads processes a batch of CPB = 256 / (k+1)^d cells,
// one thread per (cell, local point): nodes and Gauss points have the same
// tensor shape (k+1)^d.  Values at quadrature points come from d sum-factorised
// 1D sweeps with the basis table B (Section 3.4: the element operator is
// evaluated through its tensor-product structure on the unit cell instead of
// forming G_k); gradients from the collocation derivative at the Gauss points;
// test-function integration runs the transposed sweeps.  The quadrature-point
// physics is eq. (G) (or eq. (residual)) with the volumetric/deviatoric split
// written branch-free: the tension/compression choice is a select on tr e
// (the masking idea of Algorithm 3, mapped to per-lane v_cndmask).
// Cell contributions are scattered with hardware FP64/FP32 atomics.
#include <type_traits>

#include "cell_common.h"

namespace mfpff {

// QD: products from the cached tangent coefficients (a.qd), so only x is gathered;
// MODE_QDATA writes those coefficients (a.qd_out) from u, phi, phi~
template <int DIM, int K, typename T, int MODE, bool QD = false>
__global__ __launch_bounds__(kThreads) void cell_kernel(CellArgs<T> a, const Tables<T>* __restrict__ tab) {
  using S = Shape<DIM, K>;
  constexpr int NP = S::NP, P = S::P, CPB = S::CPB, NPTS = S::NPTS;
  constexpr bool XMODE = (MODE == MODE_APPLY || MODE == MODE_APPLY_T || MODE == MODE_BLOCK || MODE == MODE_ELEM);
  constexpr int NBUF = (XMODE && QD) ? DIM + 1 : S::NBUF;  // field slots per LDS buffer
  __shared__ SharedTables<NP, T> st;
  __shared__ T buf0[NBUF * NPTS];
  __shared__ T buf1[NBUF * NPTS];

  const int tid = threadIdx.x;
  st.load(tab, tid);

  const Geom g = a.g;
  const long long nn = g.n_nodes;
  const long long ncells = DIM == 2 ? (long long)g.N * g.N : (long long)g.N * g.N * g.N;
  const bool inb = tid < NPTS;
  const int c = inb ? tid / P : 0;
  const int p = inb ? tid % P : 0;
  constexpr int NCOL = (DIM + 1) * P;
  const long long vcell = (long long)blockIdx.x * CPB + c;
  long long cell = vcell;
  int jcomp = 0, jp = 0;
  if (MODE == MODE_ELEM) {
    cell = vcell / NCOL;
    const int j = (int)(vcell % NCOL);
    jcomp = j / P;
    jp = j % P;
  }
  const bool valid = inb && cell < ncells;
  const long long node = valid ? node_of<DIM, K>(g, cell, p) : 0;  // invalid lanes read node 0
  const uint8_t mk = a.mask ? a.mask[node] : (uint8_t)0;

  // ---------------- gather nodal values into buf0
  // field order: XMODE: x_0..x_d, u_0..u_{d-1}, phi, phit
  //              RESIDUAL: u_0..u_{d-1}, phi, phit
  //              PVJP: phi, v_phi
  if (inb) {
    const int o = c * P + p;
    if (XMODE) {
      bool colfixed = false;
      long long jnode = 0;
      if (MODE == MODE_ELEM && valid) {
        jnode = node_of<DIM, K>(g, cell, jp);
        const uint8_t jm = a.mask ? a.mask[jnode] : (uint8_t)0;
        colfixed = (jcomp < DIM) ? (jm & kMaskU) : (jm & kMaskPhi);
      }
      // loads are unconditional and masked by bitwise selects afterwards (all in flight at once)
      T xv[DIM + 1];
      if (MODE != MODE_ELEM) {
#pragma unroll
        for (int cc = 0; cc <= DIM; ++cc) xv[cc] = a.x[cc * nn + node];
      }
      T lin[DIM + 2];
      if (!QD) {
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc) lin[cc] = a.u[cc * nn + node];
        lin[DIM] = a.phi[node];
        lin[DIM + 1] = a.phit[node];
      }
#pragma unroll
      for (int cc = 0; cc <= DIM; ++cc) {
        T v;
        if (MODE == MODE_ELEM) {
          v = (valid && cc == jcomp && p == jp && !colfixed) ? T(1) : T(0);
        } else {
          const bool fixed = (cc < DIM) ? (mk & kMaskU) : (mk & kMaskPhi);
          v = keep_if(xv[cc], valid && !fixed);
        }
        buf0[cc * NPTS + o] = v;
      }
      if (!QD) {
#pragma unroll
        for (int cc = 0; cc < DIM + 2; ++cc) buf0[(DIM + 1 + cc) * NPTS + o] = keep_if(lin[cc], valid);
      }
    } else if (MODE == MODE_RESIDUAL || MODE == MODE_QDATA) {
      T lin[DIM + 2];
#pragma unroll
      for (int cc = 0; cc < DIM; ++cc) lin[cc] = a.u[cc * nn + node];
      lin[DIM] = a.phi[node];
      lin[DIM + 1] = a.phit[node];
#pragma unroll
      for (int cc = 0; cc < DIM + 2; ++cc) buf0[cc * NPTS + o] = keep_if(lin[cc], valid);
    } else {  // PVJP
      buf0[o] = valid ? a.phi[node] : T(0);
      buf0[NPTS + o] = valid ? a.x[DIM * nn + node] : T(0);
    }
  }
  __syncthreads();

  if constexpr (MODE == MODE_PVJP) {
    // values and gradients of phi and v_phi; per-block sums of
    // (1-phi, v) and (grad phi, grad v) weighted for dGc and deps
    __shared__ double sred[2 * kThreads];
    sweep<NP, P, NPTS, T>(buf0, buf1, 2, st.B, 0, tid);
    __syncthreads();
    sweep<NP, P, NPTS, T>(buf1, buf0, 2, st.B, 1, tid);
    __syncthreads();
    if (DIM == 3) {
      sweep<NP, P, NPTS, T>(buf0, buf1, 2, st.B, 2, tid);
      __syncthreads();
    }
    const T* V = DIM == 2 ? buf0 : buf1;
    const T h = (T)g.h, ih = T(1) / h, Gc = (T)a.m.Gc, eps = (T)a.m.eps;
    double s0 = 0, s1 = 0;
    if (valid) {
      T jxw = st.W[p % NP] * st.W[(p / NP) % NP] * h * h;
      if (DIM == 3) jxw *= st.W[p / (NP * NP)] * h;
      const T ph = V[c * P + p];
      const T vq = V[NPTS + c * P + p];
      T gpgv = 0;
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        const T gp = coll_deriv<NP, P, NPTS, T>(V, st.C, m, c, p) * ih;
        const T gv = coll_deriv<NP, P, NPTS, T>(V + NPTS, st.C, m, c, p) * ih;
        gpgv += gp * gv;
      }
      const T om = (T(1) - ph) * vq;
      s0 = (double)(jxw * (-om / eps + eps * gpgv));
      s1 = (double)(jxw * Gc * (om / (eps * eps) + gpgv));
    }
    sred[tid] = s0;
    sred[kThreads + tid] = s1;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if (tid < w) {
        sred[tid] += sred[tid + w];
        sred[kThreads + tid] += sred[kThreads + tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      a.partials[2 * blockIdx.x] = sred[0];
      a.partials[2 * blockIdx.x + 1] = sred[kThreads];
    }
  } else {
    const int NQ = a.m.split == SPLIT_MIEHE ? n_qcoef_miehe<DIM>() : n_qcoef<DIM>();
    const long long qoff = (long long)blockIdx.x * NQ * P * CPB;
    const T* R = cell_compute<DIM, K, T, MODE, kThreads, QD>(buf0, buf1, st, a.m, (T)g.h, tid, QD ? a.qd + qoff : nullptr,
                                                             MODE == MODE_QDATA ? a.qd_out + qoff : nullptr);
    if constexpr (MODE == MODE_QDATA) return;

    if constexpr (MODE == MODE_APPLY || MODE == MODE_APPLY_T || MODE == MODE_BLOCK || MODE == MODE_RESIDUAL) {
      if (a.elem) {
        // one coalesced copy of the block's results, laid out [block][component][point][cell of
        // the block] so that the node gather reads runs of consecutive cells
        constexpr int NC = DIM + 1;
        const long long cell0 = (long long)blockIdx.x * CPB;
        T* eb = a.elem + cell0 * NC * P;
        for (int idx = tid; idx < CPB * NC * P; idx += blockDim.x) {
          const int rem = idx / CPB, c2 = idx - rem * CPB;
          const int cc = rem / P;
          if (cell0 + c2 < ncells) eb[idx] = R[cc * NPTS + c2 * P + (rem - cc * P)];
        }
        return;
      }
    }

    // ---------------- scatter
    if (valid) {
      const int o = c * P + p;
      if (MODE == MODE_ELEM && a.elem_mat) {
        // column jcomp*P + jp of the cell's element matrix, rows (component, local node)
        double* em = a.elem_mat + ((long long)cell * NCOL + p) * NCOL + jcomp * P + jp;
#pragma unroll
        for (int cc = 0; cc <= DIM; ++cc) em[(long long)cc * P * NCOL] = (double)R[cc * NPTS + o];
      } else if (MODE == MODE_ELEM) {
        const long long jnode = node_of<DIM, K>(g, cell, jp);
        const uint8_t jm = a.mask ? a.mask[jnode] : (uint8_t)0;
        const bool colfixed = (jcomp < DIM) ? (jm & kMaskU) : (jm & kMaskPhi);
        if (!colfixed) {
          const long long col = jcomp * nn + jnode;
#pragma unroll
          for (int cc = 0; cc <= DIM; ++cc) {
            const bool fixed = (cc < DIM) ? (mk & kMaskU) : (mk & kMaskPhi);
            if (!fixed) atomic_add(a.dense + (cc * nn + node) * a.ld + col, (double)R[cc * NPTS + o]);
          }
        }
      } else {
        const bool resmode = (MODE == MODE_RESIDUAL);
#pragma unroll
        for (int cc = 0; cc <= DIM; ++cc) {
          const bool fixed = resmode ? false : ((cc < DIM) ? (mk & kMaskU) : (mk & kMaskPhi));
          if (!fixed) atomic_add(a.y + cc * nn + node, a.scale * R[cc * NPTS + o]);
        }
      }
    }
  }
}

// Diagonal of G (unconstrained rows; fixed rows are set to 1 afterwards).
// diag_u[c](p)  = sum_m sum_q alpha_{c,m}(q) prod_{m'} F_{m,m'}[q_{m'}][p_{m'}]
// with F = D^2 along m and B^2 elsewhere, alpha from the tangent
// delta sigma = a tr(de) I + b de: alpha_{c,m} = JxW (b/2 + [m=c](a + b/2)) / h^2;
// diag_phi(p)   = sum_q JxW (g'' E^+ + Gc/eps) B^2... + sum_m JxW Gc eps / h^2 (...).
// Spectral split (SPLIT): the tangent is a full Voigt matrix Dv at each point, so with
// v(c, m) the Voigt index of the strain pair (c, m), alpha_{c,m} = JxW Dv[v(c,m)][v(c,m)] / h^2
// and the cross terms m < m' add beta = 2 JxW Dv[v(c,m)][v(c,m')] / h^2 times the product of
// B D along m and m' and B^2 elsewhere.
template <int DIM>
__device__ __forceinline__ int voigt_of(int c, int m) {
  if (c == m) return c;
  if (DIM == 2) return 2;
  const int lo = c < m ? c : m, hi = c < m ? m : c;
  return lo == 0 ? (hi == 1 ? 3 : 4) : 5;
}

template <int DIM, int K, typename T, int SPLIT = SPLIT_AMOR>
__global__ __launch_bounds__(kThreads) void diag_kernel(CellArgs<T> a, const Tables<T>* __restrict__ tab) {
  using S = Shape<DIM, K>;
  constexpr int NP = S::NP, P = S::P, CPB = S::CPB, NPTS = S::NPTS;
  constexpr int NT = DIM * (DIM + 1) + 1;                    // isotropic fields
  constexpr int NPAIR = DIM * (DIM - 1) / 2;                 // pairs m < m'
  constexpr int NX = SPLIT == SPLIT_MIEHE ? NT + DIM * NPAIR : NT;
  constexpr int NBUF = NX > S::NBUF ? NX : S::NBUF;
  __shared__ T sB[NP * NP], sC[NP * NP], sB2t[NP * NP], sD2t[NP * NP], sBDt[NP * NP], sW[NP];
  __shared__ T buf0[NBUF * NPTS];
  __shared__ T buf1[NBUF * NPTS];
  const int tid = threadIdx.x;
  if (tid < NP * NP) {
    const int q = tid / NP, i = tid % NP;
    sB[tid] = tab->B[q][i];
    sC[tid] = tab->C[q][i];
    sB2t[i * NP + q] = tab->B[q][i] * tab->B[q][i];
    sD2t[i * NP + q] = tab->D[q][i] * tab->D[q][i];
    sBDt[i * NP + q] = tab->B[q][i] * tab->D[q][i];
  }
  if (tid < NP) sW[tid] = tab->w[tid];
  const Geom g = a.g;
  const long long nn = g.n_nodes;
  const long long ncells = DIM == 2 ? (long long)g.N * g.N : (long long)g.N * g.N * g.N;
  const bool inb = tid < NPTS;
  const int c = inb ? tid / P : 0;
  const int p = inb ? tid % P : 0;
  const long long cell = (long long)blockIdx.x * CPB + c;
  const bool valid = inb && cell < ncells;
  const long long node = valid ? node_of<DIM, K>(g, cell, p) : 0;
  if (inb) {
    const int o = c * P + p;
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc) buf0[cc * NPTS + o] = valid ? a.u[cc * nn + node] : T(0);
    buf0[DIM * NPTS + o] = valid ? a.phit[node] : T(0);
  }
  __syncthreads();
  sweep<NP, P, NPTS, T>(buf0, buf1, DIM + 1, sB, 0, tid);
  __syncthreads();
  sweep<NP, P, NPTS, T>(buf1, buf0, DIM + 1, sB, 1, tid);
  __syncthreads();
  if (DIM == 3) {
    sweep<NP, P, NPTS, T>(buf0, buf1, DIM + 1, sB, 2, tid);
    __syncthreads();
  }
  T* V = DIM == 2 ? buf0 : buf1;
  T* W = DIM == 2 ? buf1 : buf0;
  const T h = (T)g.h;
  const T ih = T(1) / h;
  const T lam = (T)a.m.lam, mu = (T)a.m.mu, Gc = (T)a.m.Gc, eps = (T)a.m.eps, kap = (T)a.m.kappa;
  const T Kb = lam + T(2) * mu / T(DIM);
  // the phase-field terms (phi rows) use E^+ of the split; g'' E^+ is read where the split is spectral
  T gu[DIM][DIM];
  T jxw = 0;
  if (inb) {
    const int o = c * P + p;
    jxw = sW[p % NP] * sW[(p / NP) % NP] * h * h;
    if (DIM == 3) jxw *= sW[p / (NP * NP)] * h;
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc)
#pragma unroll
      for (int m = 0; m < DIM; ++m) gu[cc][m] = coll_deriv<NP, P, NPTS, T>(V + cc * NPTS, sC, m, c, p) * ih;
    const T pt = V[DIM * NPTS + o];
    T t = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) t += gu[i][i];
    const bool H = t >= T(0) || a.m.split == SPLIT_NONE;
    const T tp = H ? t : T(0);
    T devdev = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        const T eij = T(0.5) * (gu[i][j] + gu[j][i]);
        const T dv = eij - (i == j ? t / T(DIM) : T(0));
        devdev += dv * dv;
      }
    T Ep = T(0.5) * Kb * tp * tp + mu * devdev;
    const T gt = (T(1) - kap) * pt * pt + kap;
    const T ddg = T(2) * (T(1) - kap);
    const T ih2 = ih * ih;
    if (SPLIT == SPLIT_MIEHE) {
      T e[DIM][DIM];
#pragma unroll
      for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) e[i][j] = T(0.5) * (gu[i][j] + gu[j][i]);
      const MiehePoint<DIM, T> mpt = miehe_point<DIM, T>(e, lam, mu);
      Ep = mpt.Ep;
      T Dv[n_voigt<DIM>()][n_voigt<DIM>()];
      miehe_voigt_tangent<DIM, T>(mpt.eig, mpt.H, gt, lam, mu, Dv);
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc) {
          const int vm = voigt_of<DIM>(cc, m);
          W[(m * (DIM + 1) + cc) * NPTS + o] = jxw * ih2 * Dv[vm][vm];
        }
        W[(m * (DIM + 1) + DIM) * NPTS + o] = jxw * ih2 * Gc * eps;
      }
#pragma unroll
      for (int cc = 0; cc < DIM; ++cc)
#pragma unroll
        for (int pi = 0, m = 0; m < DIM; ++m)
#pragma unroll
          for (int m2 = m + 1; m2 < DIM; ++m2, ++pi)
            W[(NT + cc * NPAIR + pi) * NPTS + o] = jxw * ih2 * T(2) * Dv[voigt_of<DIM>(cc, m)][voigt_of<DIM>(cc, m2)];
    } else {
      const T av = (H ? gt * Kb : Kb) - T(2) * mu * gt / T(DIM);
      const T bv = T(2) * mu * gt;
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc)
          W[(m * (DIM + 1) + cc) * NPTS + o] = jxw * ih2 * (T(0.5) * bv + (m == cc ? av + T(0.5) * bv : T(0)));
        W[(m * (DIM + 1) + DIM) * NPTS + o] = jxw * ih2 * Gc * eps;
      }
    }
    W[(NT - 1) * NPTS + o] = jxw * (ddg * Ep + Gc / eps);
  }
  __syncthreads();
  // three transposed sweeps with per-tensor matrices (D^2 along its own direction; B D along
  // both directions of a cross term)
  T* in = W;
  T* out = V;
#pragma unroll
  for (int dir = 0; dir < DIM; ++dir) {
    if (inb) {
      const int st = dir == 0 ? 1 : (dir == 1 ? NP : NP * NP);
      const int dg = (p / st) % NP;
      const int base = c * P + p - dg * st;
      for (int f = 0; f < NX; ++f) {
        const T* tabr;
        if (f < NT) {
          const int grp = f / (DIM + 1);
          tabr = ((f < NT - 1) && grp == dir ? sD2t : sB2t);
        } else {
          // pair index -> (m, m')
          const int pi = (f - NT) % (NPAIR > 0 ? NPAIR : 1);
          const int m = (DIM == 2 || pi < 2) ? 0 : 1;
          const int m2 = DIM == 2 ? 1 : (pi == 0 ? 1 : 2);
          tabr = (dir == m || dir == m2) ? sBDt : sB2t;
        }
        const T* mrow = tabr + dg * NP;
        const T* src = in + f * NPTS + base;
        T acc = 0;
#pragma unroll
        for (int r = 0; r < NP; ++r) acc += mrow[r] * src[r * st];
        out[f * NPTS + c * P + p] = acc;
      }
    }
    __syncthreads();
    T* tmp = in;
    in = out;
    out = tmp;
  }
  if (valid) {
    const int o = c * P + p;
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc) {
      T s = 0;
#pragma unroll
      for (int m = 0; m < DIM; ++m) s += in[(m * (DIM + 1) + cc) * NPTS + o];
      if (SPLIT == SPLIT_MIEHE) {
#pragma unroll
        for (int pi = 0; pi < NPAIR; ++pi) s += in[(NT + cc * NPAIR + pi) * NPTS + o];
      }
      atomic_add(a.y + cc * nn + node, s);
    }
    T s = in[(NT - 1) * NPTS + o];
#pragma unroll
    for (int m = 0; m < DIM; ++m) s += in[(m * (DIM + 1) + DIM) * NPTS + o];
    atomic_add(a.y + DIM * nn + node, s);
  }
}

static int cpb_of(int dim, int k) {
  int P = 1;
  for (int i = 0; i < dim; ++i) P *= (k + 1);
  return kThreads / P;
}

long long cell_blocks(const Geom& g, int mode) {
  long long nc = (long long)g.N * g.N * (g.dim == 3 ? g.N : 1);
  int P = 1;
  for (int i = 0; i < g.dim; ++i) P *= (g.k + 1);
  if (mode == MODE_ELEM) nc *= (long long)(g.dim + 1) * P;
  const int cpb = cpb_of(g.dim, g.k);
  return (nc + cpb - 1) / cpb;
}

template <int DIM, int K, typename T>
static hipError_t launch_dk(int mode, const CellArgs<T>& a, const Tables<T>* tab, hipStream_t s) {
  const long long nb = cell_blocks(a.g, mode);
  if (nb <= 0) return hipSuccess;
  if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 grid((unsigned)nb), block(kThreads);
  const bool qd = DIM == 3 && a.qd != nullptr;
  if (qd && a.elem && (mode == MODE_APPLY || mode == MODE_APPLY_T || mode == MODE_BLOCK)) {
    if (a.mfma && K >= 3 && a.m.split == SPLIT_AMOR) return launch_mfmacell<T>(mode, a, tab, s);
    return launch_linecell<T>(mode, a, tab, s);
  }
  switch (mode) {
    case MODE_APPLY:
      if (qd) hipLaunchKernelGGL((cell_kernel<DIM, K, T, MODE_APPLY, true>), grid, block, 0, s, a, tab);
      else hipLaunchKernelGGL((cell_kernel<DIM, K, T, MODE_APPLY>), grid, block, 0, s, a, tab);
      break;
    case MODE_APPLY_T:
      if (qd) hipLaunchKernelGGL((cell_kernel<DIM, K, T, MODE_APPLY_T, true>), grid, block, 0, s, a, tab);
      else hipLaunchKernelGGL((cell_kernel<DIM, K, T, MODE_APPLY_T>), grid, block, 0, s, a, tab);
      break;
    case MODE_BLOCK:
      if (qd) hipLaunchKernelGGL((cell_kernel<DIM, K, T, MODE_BLOCK, true>), grid, block, 0, s, a, tab);
      else hipLaunchKernelGGL((cell_kernel<DIM, K, T, MODE_BLOCK>), grid, block, 0, s, a, tab);
      break;
    case MODE_QDATA:
      if (DIM != 3 || !a.qd_out) return hipErrorInvalidValue;
      hipLaunchKernelGGL((cell_kernel<DIM, K, T, MODE_QDATA>), grid, block, 0, s, a, tab);
      break;
    default:
      if constexpr (std::is_same<T, double>::value) {
        if (mode == MODE_RESIDUAL) hipLaunchKernelGGL((cell_kernel<DIM, K, T, MODE_RESIDUAL>), grid, block, 0, s, a, tab);
        else if (mode == MODE_PVJP) hipLaunchKernelGGL((cell_kernel<DIM, K, T, MODE_PVJP>), grid, block, 0, s, a, tab);
        else if (mode == MODE_ELEM) hipLaunchKernelGGL((cell_kernel<DIM, K, T, MODE_ELEM>), grid, block, 0, s, a, tab);
        else return hipErrorInvalidValue;
      } else {
        return hipErrorInvalidValue;
      }
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cell(int mode, const CellArgs<T>& a, const Tables<T>* tab, hipStream_t s) {
  const int d = a.g.dim, k = a.g.k;
#define MFPFF_CASE(D, KK) \
  if (d == D && k == KK) return launch_dk<D, KK, T>(mode, a, tab, s);
  MFPFF_CASE(2, 1) MFPFF_CASE(2, 2) MFPFF_CASE(2, 3) MFPFF_CASE(2, 4)
  MFPFF_CASE(3, 1) MFPFF_CASE(3, 2) MFPFF_CASE(3, 3) MFPFF_CASE(3, 4)
#undef MFPFF_CASE
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_diag(const CellArgs<T>& a, const Tables<T>* tab, hipStream_t s) {
  const long long nb = cell_blocks(a.g, MODE_APPLY);
  if (nb <= 0) return hipSuccess;
  dim3 grid((unsigned)nb), block(kThreads);
  const int d = a.g.dim, k = a.g.k;
#define MFPFF_CASE(D, KK)                                                                             \
  if (d == D && k == KK) {                                                                            \
    if (a.m.split == SPLIT_MIEHE) hipLaunchKernelGGL((diag_kernel<D, KK, T, SPLIT_MIEHE>), grid, block, 0, s, a, tab); \
    else hipLaunchKernelGGL((diag_kernel<D, KK, T>), grid, block, 0, s, a, tab);                      \
    return hipGetLastError();                                                                         \
  }
  MFPFF_CASE(2, 1) MFPFF_CASE(2, 2) MFPFF_CASE(2, 3) MFPFF_CASE(2, 4)
  MFPFF_CASE(3, 1) MFPFF_CASE(3, 2) MFPFF_CASE(3, 3) MFPFF_CASE(3, 4)
#undef MFPFF_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- node gather (3D)
// Every node adds the results of the (at most 8) cells that contain it, in a fixed order
// (z, then y, then x neighbour), and applies the epilogue of the operation:
//   EPI_APPLY: y = G^ x;  EPI_RESID: r = b - G^ x (optional Chebyshev start);
//   EPI_CHEB:  d = c1 d + c2 D^-1 (r - G^_blk z), z' = z + d (optional xout = xacc + z').
// Fixed rows take the identity.  Workgroups are mapped so that each XCD works on one
// contiguous range of nodes (its L2 then holds the element lines its nodes share).
long long cell_qdata_len(const Geom& g, int split) {
  const long long P = (long long)(g.k + 1) * (g.k + 1) * (g.k + 1);
  return cell_blocks(g, MODE_APPLY) * cpb_of(g.dim, g.k) * P * (split == SPLIT_MIEHE ? n_qcoef_miehe<3>() : n_qcoef<3>());
}

long long elem_len(const Geom& g) {
  const long long P = (long long)(g.k + 1) * (g.k + 1) * (g.k + 1);
  return cell_blocks(g, MODE_APPLY) * cpb_of(g.dim, g.k) * (g.dim + 1) * P;
}

template <int K, typename T, int EPI>
__global__ __launch_bounds__(kThreads) void gather3d_kernel(const T* __restrict__ E, CellArgs<T> a, Epilogue<T> e) {
  constexpr int NP = K + 1, P = NP * NP * NP, NC = 4, CPB = kThreads / P;
  const Geom g = a.g;
  const int N = g.N;
  const long long M = g.M, nn = g.n_nodes;
  // XCD-aware block order: hardware block b runs on XCD b % 8
  const unsigned G = gridDim.x, b = blockIdx.x, x = b % 8, q = G / 8, rem = G % 8;
  const unsigned lb = x * q + min(x, rem) + b / 8;
  const long long node = (long long)lb * blockDim.x + threadIdx.x;
  if (node >= nn) return;
  const unsigned um = (unsigned)M, q1 = (unsigned)node / um, q2 = q1 / um;
  const int ix = (int)((unsigned)node - q1 * um), iy = (int)(q1 - q2 * um), iz = (int)q2;
  int cx[2], lx[2], cy[2], ly[2], cz[2], lz[2];
  auto axis = [&](int i, int (&cc)[2], int (&li)[2]) -> int {
    const int c = i / K, r = i - c * K;
    if (r != 0) {
      cc[0] = c;
      li[0] = r;
      return 1;
    }
    int n = 0;
    if (c - 1 >= 0) {
      cc[n] = c - 1;
      li[n] = K;
      ++n;
    }
    if (c < N) {
      cc[n] = c;
      li[n] = 0;
      ++n;
    }
    return n;
  };
  const int nx = axis(ix, cx, lx), ny = axis(iy, cy, ly), nz = axis(iz, cz, lz);
  T sum[NC] = {T(0), T(0), T(0), T(0)};
  for (int kz = 0; kz < nz; ++kz)
    for (int ky = 0; ky < ny; ++ky)
      for (int kx = 0; kx < nx; ++kx) {
        const long long cell = MFPFF_IN(cx[kx] + (long long)N * (cy[ky] + (long long)N * cz[kz]), (long long)N * N * N);
        const int p = lx[kx] + NP * (ly[ky] + NP * lz[kz]);
        const long long blk = cell / CPB;
        const T* src = E + (blk * NC * P + p) * CPB + (cell - blk * CPB);
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) sum[cc] += src[cc * P * CPB];
      }
  const uint8_t m = a.mask ? a.mask[node] : (uint8_t)0;
#pragma unroll
  for (int cc = 0; cc < NC; ++cc) {
    const long long idx = cc * nn + node;
    const bool fixed = (cc < 3) ? (m & kMaskU) : (m & kMaskPhi);
    const T xo = a.x[idx];  // unconditional: a load behind the mask test would wait for the mask
    const T gx = fixed ? xo : sum[cc];
    if (EPI == EPI_APPLY) {
      e.y[idx] = gx;
      if (e.xcopy) e.xcopy[idx] = xo;
    } else if (EPI == EPI_RESID) {
      const T rv = e.b[idx] - gx;
      e.y[idx] = rv;
      if (e.z0) {
        const T zv = e.dinv[idx] * rv * (cc < 3 ? e.ith_u : e.ith_p);
        e.z0[idx] = zv;
        e.d0[idx] = zv;
      }
    } else {
      const bool isu = cc < 3;
      const T dn = (isu ? e.c1u : e.c1p) * e.d[idx] + (isu ? e.c2u : e.c2p) * e.dinv[idx] * (e.r[idx] - gx);
      e.d[idx] = dn;
      const T zn = xo + dn;
      e.y[idx] = zn;
      if (e.xout) e.xout[idx] = e.xacc[idx] + zn;
    }
  }
}

template <int K, typename T>
static hipError_t launch_gk(int epi, const T* elem, const CellArgs<T>& a, const Epilogue<T>& e, hipStream_t s) {
  const long long nb = (a.g.n_nodes + kThreads - 1) / kThreads;
  if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 grid((unsigned)nb), block(kThreads);
  if (epi == EPI_APPLY) hipLaunchKernelGGL((gather3d_kernel<K, T, EPI_APPLY>), grid, block, 0, s, elem, a, e);
  else if (epi == EPI_RESID) hipLaunchKernelGGL((gather3d_kernel<K, T, EPI_RESID>), grid, block, 0, s, elem, a, e);
  else if (epi == EPI_CHEB) hipLaunchKernelGGL((gather3d_kernel<K, T, EPI_CHEB>), grid, block, 0, s, elem, a, e);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_3d(int epi, const T* elem, const CellArgs<T>& a, const Epilogue<T>& e, hipStream_t s) {
  if (a.g.dim != 3) return hipErrorInvalidValue;
  switch (a.g.k) {
    case 1: return launch_gk<1, T>(epi, elem, a, e, s);
    case 2: return launch_gk<2, T>(epi, elem, a, e, s);
    case 3: return launch_gk<3, T>(epi, elem, a, e, s);
    case 4: return launch_gk<4, T>(epi, elem, a, e, s);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_gather_3d<double>(int, const double*, const CellArgs<double>&, const Epilogue<double>&, hipStream_t);
template hipError_t launch_gather_3d<float>(int, const float*, const CellArgs<float>&, const Epilogue<float>&, hipStream_t);

template hipError_t launch_cell<double>(int, const CellArgs<double>&, const Tables<double>*, hipStream_t);
template hipError_t launch_cell<float>(int, const CellArgs<float>&, const Tables<float>*, hipStream_t);
template hipError_t launch_diag<double>(const CellArgs<double>&, const Tables<double>*, hipStream_t);

}  // namespace mfpff

MFPFF_BOUNDS_READER(bounds_hits_cell)
