// 3D products from the cached tangent coefficients, one thread per node line (gfx950).
//
// Each cell is shared by (k+1)^2 threads.  The contractions of the sum factorisation
// (Section 3.4: the element operator is applied through its tensor-product structure)
// are done line by line in registers: a thread holds k+1 values along one direction
// and contracts them with the 1D basis B and its derivative D.  Between directions
// the partial results go through LDS, so every LDS value written is read once per
// contraction that needs it (one-thread-per-point sweeps read each value k+1 times).
//
// Forward, per trial field: x-step (B, D), y-step (B, D), z-step (B, D) give the three
// reference derivatives at the Gauss points (and the value for phi) on the z-line of
// Gauss points owned by the thread.  The point physics of eq. (G) uses the cached
// coefficients; the test integration runs the transposed steps z, y, x.  Cell results
// go to the element buffer in the layout of the point-per-thread kernel, so the node
// gather and its fused epilogues are shared.
//
// A workgroup takes NOB consecutive blocks of that layout (CPB cells each), so the
// coefficient cache and the element buffer are read and written in its order.
#include "cell_common.h"
#include "gauss_tables.h"
#include "miehe.h"

namespace mfpff {

namespace {

template <int K>
struct LineShape {
  static constexpr int NP = K + 1;
  static constexpr int P = NP * NP * NP;  // points (and nodes) per cell
  static constexpr int L = NP * NP;       // lines per cell
  static constexpr int CPB = kThreads / P;            // cells per block of the shared layouts
  static constexpr int NOB = kThreads / (CPB * L);    // layout blocks per workgroup
  static constexpr int CW = NOB * CPB;                // cells per workgroup
  static constexpr int NT = CW * L;                   // threads
  static constexpr int TS = CW * P;                   // one LDS tensor
};

// waves per SIMD the register allocation must allow: four (at most 128 VGPRs) wherever the
// 13 (k+1) values a thread holds at its Gauss points fit without spilling; three for FP64 Q3,
// two for FP64 Q4
template <int K, typename T, int SPLIT>
struct LineWaves {
  static constexpr int amor = (K <= 2 || sizeof(T) == 4) ? 4 : (K == 3 ? 3 : 2);
  // the spectral split reads the 21 entries of the Voigt tangent per point: one wave fewer
  static constexpr int value = SPLIT == 1 ? (amor > 2 ? amor - 1 : 2) : amor;
};

}  // namespace

long long linecell_blocks(const Geom& g) {
  const long long nc = (long long)g.N * g.N * g.N;
  int cw = 0;
  switch (g.k) {
    case 1: cw = LineShape<1>::CW; break;
    case 2: cw = LineShape<2>::CW; break;
    case 3: cw = LineShape<3>::CW; break;
    case 4: cw = LineShape<4>::CW; break;
    default: return -1;
  }
  return (nc + cw - 1) / cw;
}

// SPLIT: the cached coefficients are those of the volumetric/deviatoric split or of the
// spectral split (upper triangle of the Voigt tangent, coupling, phase coefficient)
template <int K, typename T, int MODE, int SPLIT = SPLIT_AMOR>
__global__ __launch_bounds__(LineShape<K>::NT) __attribute__((amdgpu_waves_per_eu(LineWaves<K, T, SPLIT>::value))) void linecell_kernel(
    CellArgs<T> a, const Tables<T>* __restrict__ tabd) {
  using S = LineShape<K>;
  constexpr int NP = S::NP, P = S::P, L = S::L, CPB = S::CPB, CW = S::CW, TS = S::TS;
  constexpr int NQ = SPLIT == SPLIT_MIEHE ? n_qcoef_miehe<3>() : n_qcoef<3>();
  constexpr int CO = SPLIT == SPLIT_MIEHE ? 21 : 1;  // first coupling coefficient
  constexpr int NC = 4;
  __shared__ T lds[5 * TS];
  T* bufA = lds;           // two tensors
  T* bufB = lds + 2 * TS;  // three tensors

  const int tid = threadIdx.x;
  const int c = tid / L, l = tid - c * L;
  const int la = l % NP, lb = l / NP;  // x-step: (i1, i2); y-step: (q0, i2); z-step: (q0, q1)
  const Geom g = a.g;
  const unsigned N = (unsigned)g.N;
  const long long nn = g.n_nodes, M = g.M;
  const long long ncells = (long long)N * N * N;
  const long long cell0 = (long long)blockIdx.x * CW;
  const long long cell = cell0 + c;
  const bool valid = cell < ncells;
  const long long vc = valid ? cell : 0;  // invalid lanes read cell 0 and store nothing

  // 1D tables: compile-time constants up to Q3 (no scalar registers; the zero and unit entries
  // fold).  At Q4 the constants would be kept in vector registers and spill to scratch, so the
  // entries come from the device copy as uniform values, and only the rows q <= k/2: the points
  // and nodes are symmetric about 1/2, so B[q][i] = B[k-q][k-i] and D[q][i] = -D[k-q][k-i]
  // (31 values in scalar registers instead of 55, which spilled into vector lanes)
  constexpr int NH = K / 2 + 1;
  T Bh[NH][NP], Dh[NH][NP], wv[NH];
  if (K == 4) {
#pragma unroll
    for (int q = 0; q < NH; ++q) {
      wv[q] = tabd->w[q];
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        Bh[q][i] = tabd->B[q][i];
        Dh[q][i] = tabd->D[q][i];
      }
    }
  }
  auto TBB = [&](int q, int i) -> T {
    return K == 4 ? (q < NH ? Bh[q][i] : Bh[K - q][K - i]) : (T)ConstTab<K>::B(q, i);
  };
  auto TBD = [&](int q, int i) -> T {
    return K == 4 ? (q < NH ? Dh[q][i] : -Dh[K - q][K - i]) : (T)ConstTab<K>::D(q, i);
  };
  auto TBW = [&](int q) -> T { return K == 4 ? (q < NH ? wv[q] : wv[K - q]) : (T)ConstTab<K>::w(q); };

  // ---- x-lines of the trial vector (node row (la, lb) of the cell), masked at fixed dofs
  const unsigned uc = (unsigned)vc, q1c = uc / N, cz = q1c / N;
  const unsigned cx = uc - q1c * N, cy = q1c - cz * N;
  const long long n0 = (long long)(K * cx) + M * (long long)(K * cy + la) + M * M * (long long)(K * cz + lb);
  T xl[NC][NP];
  uint8_t mk[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const long long nd = MFPFF_IN(n0 + i, nn);
    mk[i] = a.mask ? a.mask[nd] : (uint8_t)0;
#pragma unroll
    for (int f = 0; f < NC; ++f) xl[f][i] = a.x[f * nn + nd];
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const bool ku = valid && !(mk[i] & kMaskU), kp = valid && !(mk[i] & kMaskPhi);
#pragma unroll
    for (int f = 0; f < NC; ++f) xl[f][i] = keep_if(xl[f][i], f < 3 ? ku : kp);
  }

  const int lo = c * P + l;  // this thread's line base in the [cell][point] layouts (for z-lines)
  // x-step layout offset: node row (la, lb) -> c*P + NP*la + NP^2*lb; y-step: (q0=la, i2=lb)
  const int xo = c * P + NP * la + NP * NP * lb;
  const int yo = c * P + la + NP * NP * lb;

  // ---- forward: reference derivatives (and phi value) on the thread's z-line of points
  T gr[NC][3][NP];  // [field][d/dxi_m][q2]
  T pv[NP];         // phi value
#pragma unroll
  for (int f = 0; f < NC; ++f) {
    // x-step: Bx X, Dx X
    {
      T* s = bufA;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        T sb = 0, sd = 0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          sb += TBB(q, i) * xl[f][i];
          sd += TBD(q, i) * xl[f][i];
        }
        s[xo + q] = sb;
        s[TS + xo + q] = sd;
      }
    }
    __syncthreads();
    // y-step on (q0, i2): By K0, Dy K0, By K1
    {
      T k0[NP], k1[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        k0[i] = bufA[yo + NP * i];
        k1[i] = bufA[TS + yo + NP * i];
      }
      T* s = bufB;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          s0 += TBB(q, i) * k0[i];
          s1 += TBD(q, i) * k0[i];
          s2 += TBB(q, i) * k1[i];
        }
        s[yo + NP * q] = s0;
        s[TS + yo + NP * q] = s1;
        s[2 * TS + yo + NP * q] = s2;
      }
    }
    __syncthreads();
    // z-step on (q0, q1): d/dz = Dz BxBy, d/dy = Bz BxDy, d/dx = Bz DxBy (phi: value Bz BxBy)
    {
      T y0[NP], y1[NP], y2[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        y0[i] = bufB[lo + L * i];
        y1[i] = bufB[TS + lo + L * i];
        y2[i] = bufB[2 * TS + lo + L * i];
      }
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        T dz = 0, dy = 0, dx = 0, v = 0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          dz += TBD(q, i) * y0[i];
          dy += TBB(q, i) * y1[i];
          dx += TBB(q, i) * y2[i];
          if (f == 3) v += TBB(q, i) * y0[i];
        }
        gr[f][0][q] = dx;
        gr[f][1][q] = dy;
        gr[f][2][q] = dz;
        if (f == 3) pv[q] = v;
      }
    }
  }

  // ---- point physics of eq. (G) from the cached coefficients, on the points (la, lb, q2)
  const T h = (T)g.h, ih = T(1) / h;
  const T Gc = (T)a.m.Gc, eps = (T)a.m.eps, lam = (T)a.m.lam, mu = (T)a.m.mu;
  const T Kb = lam + T(2) * mu / T(3);
  const long long blk = vc / CPB;
  const int cw = (int)(vc - blk * CPB);
  const T* qb = a.qd + blk * NQ * P * CPB + cw;
  constexpr int SI[6] = {0, 1, 2, 0, 0, 1};
  constexpr int SJ[6] = {0, 1, 2, 1, 2, 2};
  // fluxes overwrite the derivatives: gr[cc][m] <- JxW/h Su[cc][m] (cc < 3), gr[3][m] <- JxW/h Gc eps d phi/dx_m,
  // pv <- JxW (g'' E^+ + Gc/eps) dphi + coupling
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int p = l + L * q;
    const T* qq = qb + (long long)p * CPB;
    constexpr int QS = P * CPB;
    const T gsv = keep_if(qq[0], valid), cpp = keep_if(qq[(NQ - 1) * QS], valid);
    const T gta = abs_bits(gsv);
    const T cvol = sign_bit(gsv) ? Kb : gta * Kb, cdev = gta * T(2) * mu;
    T gsp[3][3];
    if (MODE != MODE_BLOCK) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const T v = keep_if(qq[(CO + k) * QS], valid);
        gsp[SI[k]][SJ[k]] = v;
        gsp[SJ[k]][SI[k]] = v;
      }
    }
    T de[3][3];
    T dt = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int j = 0; j < 3; ++j) de[i][j] = T(0.5) * (gr[i][j][q] + gr[j][i][q]) * ih;
      dt += de[i][i];
    }
    const T vol = cvol * dt;
    const T dph = pv[q];
    T Su[3][3];
    T spde = 0;
    if (SPLIT == SPLIT_MIEHE) {
      // Voigt tangent times the engineering strain
      T dv[6], sv[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        dv[k] = (k < 3 ? T(1) : T(2)) * de[SI[k]][SJ[k]];
        sv[k] = T(0);
      }
#pragma unroll
      for (int r = 0, kk = 0; r < 6; ++r)
#pragma unroll
        for (int c2 = r; c2 < 6; ++c2, ++kk) {
          const T dk = keep_if(qq[kk * QS], valid);
          sv[r] += dk * dv[c2];
          if (c2 != r) sv[c2] += dk * dv[r];
        }
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        Su[SI[k]][SJ[k]] = sv[k];
        Su[SJ[k]][SI[k]] = sv[k];
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (SPLIT != SPLIT_MIEHE) Su[i][j] = cdev * (de[i][j] - (i == j ? dt / T(3) : T(0))) + (i == j ? vol : T(0));
        if (MODE == MODE_APPLY) spde += gsp[i][j] * de[i][j];
        if (MODE == MODE_APPLY_T) Su[i][j] += dph * gsp[i][j];
      }
    const T fval = cpp * dph + spde;
    const T jxw = TBW(la) * TBW(lb) * TBW(q) * h * h * h;
    const T jg = jxw * ih;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
      for (int m = 0; m < 3; ++m) gr[cc][m][q] = jg * Su[cc][m];
#pragma unroll
    for (int m = 0; m < 3; ++m) gr[3][m][q] = jg * Gc * eps * gr[3][m][q] * ih;
    pv[q] = jxw * fval;
  }
  __syncthreads();  // every forward read of bufB is done

  // ---- test integration per component: z-step (transposed), y-step, x-step
  T yl[NC][NP];
#pragma unroll
  for (int tc = 0; tc < NC; ++tc) {
    {
      T* s = bufB;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        T a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          a1 += TBD(q, i) * gr[tc][2][q];
          if (tc == 3) a1 += TBB(q, i) * pv[q];
          a2 += TBB(q, i) * gr[tc][0][q];
          a3 += TBB(q, i) * gr[tc][1][q];
        }
        s[lo + L * i] = a1;
        s[TS + lo + L * i] = a2;
        s[2 * TS + lo + L * i] = a3;
      }
    }
    __syncthreads();
    {
      T a1[NP], a2[NP], a3[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        a1[q] = bufB[yo + NP * q];
        a2[q] = bufB[TS + yo + NP * q];
        a3[q] = bufB[2 * TS + yo + NP * q];
      }
      T* s = bufA;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        T b1 = 0, b2 = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          b1 += TBB(q, i) * a1[q] + TBD(q, i) * a3[q];
          b2 += TBB(q, i) * a2[q];
        }
        s[yo + NP * i] = b1;
        s[TS + yo + NP * i] = b2;
      }
    }
    __syncthreads();
    {
      T b1[NP], b2[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        b1[q] = bufA[xo + q];
        b2[q] = bufA[TS + xo + q];
      }
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        T s = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) s += TBB(q, i) * b1[q] + TBD(q, i) * b2[q];
        yl[tc][i] = s;
      }
    }
  }

  // ---- element buffer: stage [component][cell][point] in LDS, then one coalesced copy in
  // the shared layout [block][component][point][cell of the block]
  __syncthreads();  // every read of bufA is done
#pragma unroll
  for (int tc = 0; tc < NC; ++tc)
#pragma unroll
    for (int i = 0; i < NP; ++i) lds[tc * TS + xo + i] = yl[tc][i];
  __syncthreads();
  T* eb = a.elem + cell0 * NC * P;
  for (int idx = tid; idx < CW * NC * P; idx += blockDim.x) {
    const int ob = idx / (CPB * NC * P);
    const int r = idx - ob * (CPB * NC * P);
    const int rem = r / CPB, c2 = r - rem * CPB;
    const int cc = rem / P, p = rem - cc * P;
    const int cl = ob * CPB + c2;
    if (cell0 + cl < ncells) eb[idx] = lds[cc * TS + cl * P + p];
  }
}

template <int K, typename T>
static hipError_t launch_lk(int mode, const CellArgs<T>& a, const Tables<T>* tab, hipStream_t s) {
  const long long nb = linecell_blocks(a.g);
  if (nb <= 0) return hipSuccess;
  if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 grid((unsigned)nb), block(LineShape<K>::NT);
  const bool miehe = a.m.split == SPLIT_MIEHE;
  switch (mode) {
#define MFPFF_L(MD)                                                                                       \
  case MD:                                                                                                \
    if (miehe) hipLaunchKernelGGL((linecell_kernel<K, T, MD, SPLIT_MIEHE>), grid, block, 0, s, a, tab);   \
    else hipLaunchKernelGGL((linecell_kernel<K, T, MD>), grid, block, 0, s, a, tab);                     \
    break;
    MFPFF_L(MODE_APPLY)
    MFPFF_L(MODE_APPLY_T)
    MFPFF_L(MODE_BLOCK)
#undef MFPFF_L
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_linecell(int mode, const CellArgs<T>& a, const Tables<T>* tab, hipStream_t s) {
  if (a.g.dim != 3 || !a.qd || !a.elem) return hipErrorInvalidValue;
  switch (a.g.k) {
    case 1: return launch_lk<1, T>(mode, a, tab, s);
    case 2: return launch_lk<2, T>(mode, a, tab, s);
    case 3: return launch_lk<3, T>(mode, a, tab, s);
    case 4: return launch_lk<4, T>(mode, a, tab, s);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_linecell<double>(int, const CellArgs<double>&, const Tables<double>*, hipStream_t);
template hipError_t launch_linecell<float>(int, const CellArgs<float>&, const Tables<float>*, hipStream_t);

}  // namespace mfpff

MFPFF_BOUNDS_READER(bounds_hits_linecell)
