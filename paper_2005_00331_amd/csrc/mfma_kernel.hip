// 3D products at degree 3 and 4 with the 1D contractions on the matrix cores (gfx950).
//
// Sum factorisation (Section 3.4) applies the element operator as a sequence of 1D
// contractions along x, y and z.  Each contraction is a small dense product
//   out[row][line] = sum_k A[row][k] in[k][line]
// with A one of the 1D tables B (basis at the Gauss points), D (its derivative) or their
// transposes, possibly stacked ([B; D]: two outputs from one input) or concatenated
// ([B^T | D^T]: the sum of two contractions), and one column per node line of the cells of
// the workgroup.  These products run as MFMA instructions made of independent 4 x 4 blocks:
//   FP64: v_mfma_f64_4x4x4f64, four blocks of 4 rows x 4 lines with k = 4 per instruction;
//   FP32: v_mfma_f32_4x4x1f32, sixteen blocks of 4 rows x 4 lines with k = 1 per instruction.
// Blocks are small, so the padding of the k+1 = 4 or 5 rows and the contraction length is
// small too (no padding at degree 3; at degree 4, 10 stacked rows fill 12 and, in FP64, the
// 5 (10) long contraction fills 8 (12)).
//
// Data flow per workgroup of CW cells: the trial values go into LDS by node line; the forward
// contractions (x: [B; D]; y: [B; D] and B; z: D, B, B and, for phi, B) leave the reference
// derivatives (and the phi value) of all four fields at the Gauss points in LDS; one thread
// per point evaluates eq. (G) from the cached tangent coefficients (the same per-point code as
// the vector-unit line kernel) and overwrites them with the fluxes; the transposed
// contractions (z: [D^T | B^T], B^T, B^T; y: [B^T | D^T], B^T; x: [B^T | D^T]) integrate
// against the test functions.  Cell results leave through the element buffer in the layout of
// the other 3D kernels, so the node gather and its fused epilogues are shared.
#include "cell_common.h"

namespace mfpff {

namespace {

typedef float mx_v4f __attribute__((ext_vector_type(4)));

// lane layouts of the two instructions (lane l of the 64-wide wavefront):
//  f64 4x4x4, block b = (l & 15) >> 2: A_b[row l & 3][k l >> 4], B_b[k l >> 4][col l & 3],
//           D_b[row l >> 4][col l & 3]; so the 16 columns of one instruction are the lines
//           l & 15, lane l feeds contraction index (l >> 4) + 4 s in step s and receives
//           row 4 m + (l >> 4) of row block m
//  f32 4x4x1, block b = l >> 2: A_b[row l & 3][0], B_b[0][col l & 3], D_b[row r][col l & 3]
//           in register r; so the 64 columns are the lines l, every lane feeds contraction
//           index s in step s and receives rows 4 m .. 4 m + 3
template <typename T>
struct Mx;
template <>
struct Mx<double> {
  static constexpr int LPI = 16;  // lines per instruction
  static constexpr int KK = 4;    // contraction indices per instruction
  using Acc = double;
  __device__ static int line(int l) { return l & 15; }
  __device__ static int kb(int l) { return l >> 4; }  // contraction index fed by this lane (B operand)
  __device__ static int ar(int l) { return l & 3; }   // A operand row
  __device__ static int ak(int l) { return l >> 4; }  // A operand contraction index
  __device__ static Acc zero() { return 0.0; }
  __device__ static Acc mma(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0); }
  static constexpr int ROWS_OUT = 1;  // rows of a row block held per lane
  __device__ static int out_row(int l, int r) { return (l >> 4) + 0 * r; }
  __device__ static double get(const Acc& c, int) { return c; }
};
template <>
struct Mx<float> {
  static constexpr int LPI = 64;
  static constexpr int KK = 1;
  using Acc = mx_v4f;
  __device__ static int line(int l) { return l; }
  __device__ static int kb(int) { return 0; }
  __device__ static int ar(int l) { return l & 3; }
  __device__ static int ak(int) { return 0; }
  __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static Acc mma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0); }
  static constexpr int ROWS_OUT = 4;
  __device__ static int out_row(int, int r) { return r; }
  __device__ static float get(const Acc& c, int r) { return c[r]; }
};

// 1D table selectors of a contraction: A[r][k] = B[r][k], D[r][k], B[k][r] or D[k][r]
enum { TB = 0, TD = 1, TBT = 2, TDT = 3, TNONE = 4 };

template <int K, typename T>
struct MShape {
  static constexpr int NP = K + 1;
  static constexpr int P = NP * NP * NP;
  static constexpr int L = NP * NP;
  static constexpr int CPB = kThreads / P;  // cells per block of the shared cache / element layouts
  // cells per workgroup: whole layout blocks, about 125 (FP64) or 250 (FP32) lines per step
  static constexpr int CW = sizeof(T) == 8 ? (K == 4 ? 4 : 8) : (K == 4 ? 8 : 16);
  static constexpr int TS = CW * P;          // one LDS tensor
  static constexpr int NL = CW * L;          // lines of one contraction step
  static constexpr int NTEN = 19;            // LDS tensors of the schedule in mfmacell_kernel
};

// One contraction step along AXIS over all lines of the workgroup, shared by the waves:
// NR stacked row sets (outputs out0, out1) times NS concatenated contraction segments
// (inputs in0, in1); table Trs of row set r and segment s.
template <typename T, int NP, int CW, int AXIS, int NR, int NS, int T00, int T01, int T10, int T11>
__device__ __forceinline__ void contract(const T* in0, const T* in1, T* out0, T* out1, const T* Bs, const T* Ds,
                                         int lane, int wave, int nwaves) {
  using X = Mx<T>;
  constexpr int P = NP * NP * NP, L = NP * NP, NL = CW * L;
  constexpr int R = NR * NP, NRB = (R + 3) / 4;
  constexpr int KT = NS * NP, NKS = (KT + X::KK - 1) / X::KK;
  constexpr int ST = AXIS == 0 ? 1 : (AXIS == 1 ? NP : NP * NP);
  // operator values of this lane, per row block and contraction step (loop invariant)
  T av[NRB][NKS];
#pragma unroll
  for (int m = 0; m < NRB; ++m)
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
      const int r = 4 * m + X::ar(lane), k = X::ak(lane) + X::KK * s;
      T v = T(0);
      if (r < R && k < KT) {
        const int rs = r / NP, rr = r - rs * NP, ks = k / NP, kk = k - ks * NP;
        const int t = rs == 0 ? (ks == 0 ? T00 : T01) : (ks == 0 ? T10 : T11);
        v = t == TB ? Bs[rr * NP + kk] : t == TD ? Ds[rr * NP + kk] : t == TBT ? Bs[kk * NP + rr]
                                                                   : t == TDT ? Ds[kk * NP + rr] : T(0);
      }
      av[m][s] = v;
    }
  constexpr int NIT = (NL + X::LPI - 1) / X::LPI;
  for (int it = wave; it < NIT; it += nwaves) {
    const int ln = it * X::LPI + X::line(lane);
    const bool lv = ln < NL;
    const int c = lv ? ln / L : 0, rl = lv ? ln - c * L : 0;
    const int j = rl % NP, kq = rl / NP;
    // base of the line: the two other axes in increasing order take (j, kq)
    const int base = c * P + (AXIS == 0 ? NP * j + L * kq : (AXIS == 1 ? j + L * kq : j + NP * kq));
    T bv[NKS];
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
      // every load stays inside the tensors (padding lanes read index 0 of segment 0) and is
      // zeroed afterwards
      const int k = X::kb(lane) + X::KK * s;
      const bool kv = lv && k < KT;
      const int kc = kv ? k : 0;
      const int ks = kc / NP, kk = kc - ks * NP;
      bv[s] = keep_if((ks == 0 ? in0 : in1)[base + ST * kk], kv);
    }
#pragma unroll
    for (int m = 0; m < NRB; ++m) {
      typename X::Acc acc = X::zero();
#pragma unroll
      for (int s = 0; s < NKS; ++s) acc = X::mma(av[m][s], bv[s], acc);
#pragma unroll
      for (int q = 0; q < X::ROWS_OUT; ++q) {
        const int r = 4 * m + X::out_row(lane, q);
        if (lv && r < R) {
          const int rs = r / NP, rr = r - rs * NP;
          (rs == 0 ? out0 : out1)[base + ST * rr] = X::get(acc, q);
        }
      }
    }
  }
}

}  // namespace

long long mfmacell_blocks(const Geom& g, bool f32) {
  const long long nc = (long long)g.N * g.N * g.N;
  int cw = 0;
  if (g.k == 3) cw = f32 ? MShape<3, float>::CW : MShape<3, double>::CW;
  else if (g.k == 4) cw = f32 ? MShape<4, float>::CW : MShape<4, double>::CW;
  else return -1;
  return (nc + cw - 1) / cw;
}

template <int K, typename T, int MODE>
__global__ __launch_bounds__(kThreads) void mfmacell_kernel(CellArgs<T> a, const Tables<T>* __restrict__ tabd) {
  using S = MShape<K, T>;
  constexpr int NP = S::NP, P = S::P, L = S::L, CPB = S::CPB, CW = S::CW, TS = S::TS, NL = S::NL;
  constexpr int NQ = n_qcoef<3>();
  constexpr int NC = 4;
  __shared__ T lds[S::NTEN * TS];
  __shared__ T Bs[NP * NP], Ds[NP * NP], Ws[NP];
  // 19 LDS tensors [cell][z][y][x] used by a fixed schedule:
  //   slots 0..3       trial values of fields 0..3 (consumed by their x-steps, then work space)
  //   slots 4+3f+m     reference derivative m of displacement field f at the Gauss points, then
  //                    its flux, then (slot 4+3f) the test integral of component f
  //   slots 13,14,15   phi derivatives (then fluxes, then slot 13 the phi test integral)
  //   slot 16          phi value (then the phase-field point term)
  //   slots 17,18      work space
  auto SL = [&](int t) { return lds + t * TS; };
  auto GD = [&](int f, int m) { return lds + (4 + 3 * f + m) * TS; };  // field f (3: phi), derivative m

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int nwaves = kThreads / 64;
  const Geom g = a.g;
  const unsigned N = (unsigned)g.N;
  const long long nn = g.n_nodes, M = g.M;
  const long long ncells = (long long)N * N * N;
  const long long cell0 = (long long)blockIdx.x * CW;
  if (tid < NP * NP) {
    const int q = tid / NP, i = tid - (tid / NP) * NP;
    Bs[tid] = tabd->B[q][i];
    Ds[tid] = tabd->D[q][i];
  }
  if (tid < NP) Ws[tid] = tabd->w[tid];

  // ---- trial values by x-line (one thread per line of a cell), zero at fixed dofs
  for (int ln = tid; ln < NL; ln += kThreads) {
    const int c = ln / L, rl = ln - c * L, la = rl % NP, lb = rl / NP;
    const long long cell = cell0 + c;
    const bool valid = cell < ncells;
    const unsigned uc = (unsigned)(valid ? cell : 0), q1c = uc / N, cz = q1c / N;
    const unsigned cx = uc - q1c * N, cy = q1c - cz * N;
    const long long n0 = (long long)(K * cx) + M * (long long)(K * cy + la) + M * M * (long long)(K * cz + lb);
    T xl[NC][NP];
    uint8_t mk[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      mk[i] = a.mask ? a.mask[n0 + i] : (uint8_t)0;
#pragma unroll
      for (int f = 0; f < NC; ++f) xl[f][i] = a.x[f * nn + n0 + i];
    }
    const int o = c * P + NP * la + L * lb;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const bool ku = valid && !(mk[i] & kMaskU), kp = valid && !(mk[i] & kMaskPhi);
#pragma unroll
      for (int f = 0; f < NC; ++f) SL(f)[o + i] = keep_if(xl[f][i], f < 3 ? ku : kp);
    }
  }
  __syncthreads();

  // ---- forward contractions of field f:
  //   x: [B; D] X_f -> (A, Dx)           A = slot 17, Dx = slot 18
  //   y: [B; D] A -> (U00, U01), B Dx -> U10, in the derivative slots of field f+1 (f = 3: slots 0..2)
  //   z: B U10 -> d/dx, B U01 -> d/dy, D U00 -> d/dz (phi also B U00 -> value) into the slots of field f
#pragma unroll 1
  for (int f = 0; f < NC; ++f) {
    T* A = SL(17);
    T* Dx = SL(18);
    T* U00 = f < 3 ? GD(f + 1, 0) : SL(0);
    T* U01 = f < 3 ? GD(f + 1, 1) : SL(1);
    T* U10 = f < 3 ? GD(f + 1, 2) : SL(2);
    {
      contract<T, NP, CW, 0, 2, 1, TB, TNONE, TD, TNONE>(SL(f), nullptr, A, Dx, Bs, Ds, lane, wave, nwaves);
    }
    __syncthreads();
    {
      contract<T, NP, CW, 1, 2, 1, TB, TNONE, TD, TNONE>(A, nullptr, U00, U01, Bs, Ds, lane, wave, nwaves);
      contract<T, NP, CW, 1, 1, 1, TB, TNONE, TNONE, TNONE>(Dx, nullptr, U10, nullptr, Bs, Ds, lane, wave, nwaves);
    }
    __syncthreads();
    {
      contract<T, NP, CW, 2, 1, 1, TB, TNONE, TNONE, TNONE>(U10, nullptr, GD(f, 0), nullptr, Bs, Ds, lane, wave, nwaves);
      contract<T, NP, CW, 2, 1, 1, TB, TNONE, TNONE, TNONE>(U01, nullptr, GD(f, 1), nullptr, Bs, Ds, lane, wave, nwaves);
      if (f == 3) {
        contract<T, NP, CW, 2, 2, 1, TB, TNONE, TD, TNONE>(U00, nullptr, SL(16), GD(f, 2), Bs, Ds, lane, wave, nwaves);
      } else {
        contract<T, NP, CW, 2, 1, 1, TD, TNONE, TNONE, TNONE>(U00, nullptr, GD(f, 2), nullptr, Bs, Ds, lane, wave, nwaves);
      }
    }
    __syncthreads();
  }

  // ---- point physics of eq. (G) from the cached tangent coefficients (as in the line kernel):
  // the derivatives are overwritten by the fluxes, the phi value by the phase-field point term
  {
    const T h = (T)g.h, ih = T(1) / h;
    const T Gc = (T)a.m.Gc, eps = (T)a.m.eps, lam = (T)a.m.lam, mu = (T)a.m.mu;
    const T Kb = lam + T(2) * mu / T(3);
    constexpr int SI[6] = {0, 1, 2, 0, 0, 1};
    constexpr int SJ[6] = {0, 1, 2, 1, 2, 2};
    constexpr int QS = P * CPB;
    for (int f = tid; f < CW * P; f += kThreads) {
      const int c = f % CW, p = f / CW;
      const long long cell = cell0 + c;
      const bool valid = cell < ncells;
      const long long vc = valid ? cell : 0;
      const long long blk = vc / CPB;
      const int cw = (int)(vc - blk * CPB);
      const T* qq = a.qd + blk * NQ * P * CPB + cw + (long long)p * CPB;
      const int o = c * P + p;
      const T gsv = keep_if(qq[0], valid), cpp = keep_if(qq[(NQ - 1) * QS], valid);
      const T gta = abs_bits(gsv);
      const T cvol = sign_bit(gsv) ? Kb : gta * Kb, cdev = gta * T(2) * mu;
      T gsp[3][3];
      if (MODE != MODE_BLOCK) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const T v = keep_if(qq[(1 + k) * QS], valid);
          gsp[SI[k]][SJ[k]] = v;
          gsp[SJ[k]][SI[k]] = v;
        }
      }
      T gr[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int m = 0; m < 3; ++m) gr[i][m] = GD(i, m)[o];
      T de[3][3];
      T dt = 0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) de[i][j] = T(0.5) * (gr[i][j] + gr[j][i]) * ih;
        dt += de[i][i];
      }
      const T vol = cvol * dt;
      const T dph = SL(16)[o];
      T Su[3][3];
      T spde = 0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          Su[i][j] = cdev * (de[i][j] - (i == j ? dt / T(3) : T(0))) + (i == j ? vol : T(0));
          if (MODE == MODE_APPLY) spde += gsp[i][j] * de[i][j];
          if (MODE == MODE_APPLY_T) Su[i][j] += dph * gsp[i][j];
        }
      const T fval = cpp * dph + spde;
      const int q0 = p % NP, q1 = (p / NP) % NP, q2 = p / L;
      const T jxw = Ws[q0] * Ws[q1] * Ws[q2] * h * h * h;
      const T jg = jxw * ih;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int m = 0; m < 3; ++m) GD(cc, m)[o] = jg * Su[cc][m];
#pragma unroll
      for (int m = 0; m < 3; ++m) GD(3, m)[o] = jg * Gc * eps * GD(3, m)[o] * ih;
      SL(16)[o] = jxw * fval;
    }
  }
  __syncthreads();

  // ---- test integration of component tc from its fluxes F0, F1, F2 (phi also Fv, slot 16):
  //   z: a1 = D^T F2 (+ B^T Fv) -> slot 17, a2 = B^T F0 -> slot 18, a3 = B^T F1 -> slot 0
  //   y: b1 = B^T a1 + D^T a3 -> slot 1, b2 = B^T a2 -> slot 2
  //   x: B^T b1 + D^T b2 -> slot of F0
#pragma unroll 1
  for (int tc = 0; tc < NC; ++tc) {
    T* F0 = GD(tc, 0);
    T* F1 = GD(tc, 1);
    T* F2 = GD(tc, 2);
    if (tc == 3) {
      contract<T, NP, CW, 2, 1, 2, TDT, TBT, TNONE, TNONE>(F2, SL(16), SL(17), nullptr, Bs, Ds, lane, wave, nwaves);
    } else {
      contract<T, NP, CW, 2, 1, 1, TDT, TNONE, TNONE, TNONE>(F2, nullptr, SL(17), nullptr, Bs, Ds, lane, wave, nwaves);
    }
    {
      contract<T, NP, CW, 2, 1, 1, TBT, TNONE, TNONE, TNONE>(F0, nullptr, SL(18), nullptr, Bs, Ds, lane, wave, nwaves);
      contract<T, NP, CW, 2, 1, 1, TBT, TNONE, TNONE, TNONE>(F1, nullptr, SL(0), nullptr, Bs, Ds, lane, wave, nwaves);
    }
    __syncthreads();
    {
      contract<T, NP, CW, 1, 1, 2, TBT, TDT, TNONE, TNONE>(SL(17), SL(0), SL(1), nullptr, Bs, Ds, lane, wave, nwaves);
      contract<T, NP, CW, 1, 1, 1, TBT, TNONE, TNONE, TNONE>(SL(18), nullptr, SL(2), nullptr, Bs, Ds, lane, wave, nwaves);
    }
    __syncthreads();
    {
      // the fluxes of this component are no longer needed: its test integral takes the slot of F0
      contract<T, NP, CW, 0, 1, 2, TBT, TDT, TNONE, TNONE>(SL(1), SL(2), F0, nullptr, Bs, Ds, lane, wave, nwaves);
    }
    __syncthreads();
  }

  // ---- element buffer: one coalesced copy in the shared layout
  // [block][component][point][cell of the block] from the slots 4, 7, 10, 13 ([cell][point])
  T* eb = a.elem + cell0 * NC * P;
  for (int idx = tid; idx < CW * NC * P; idx += kThreads) {
    const int ob = idx / (CPB * NC * P);
    const int r = idx - ob * (CPB * NC * P);
    const int rem = r / CPB, c2 = r - rem * CPB;
    const int cc = rem / P, p = rem - cc * P;
    const int cl = ob * CPB + c2;
    if (cell0 + cl < ncells) eb[idx] = GD(cc, 0)[cl * P + p];
  }
}

template <int K, typename T>
static hipError_t launch_mk(int mode, const CellArgs<T>& a, const Tables<T>* tab, hipStream_t s) {
  using S = MShape<K, T>;
  const long long nb = mfmacell_blocks(a.g, sizeof(T) == 4);
  if (nb <= 0) return hipSuccess;
  if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 grid((unsigned)nb), block(kThreads);
  switch (mode) {
    case MODE_APPLY: hipLaunchKernelGGL((mfmacell_kernel<K, T, MODE_APPLY>), grid, block, 0, s, a, tab); break;
    case MODE_APPLY_T: hipLaunchKernelGGL((mfmacell_kernel<K, T, MODE_APPLY_T>), grid, block, 0, s, a, tab); break;
    case MODE_BLOCK: hipLaunchKernelGGL((mfmacell_kernel<K, T, MODE_BLOCK>), grid, block, 0, s, a, tab); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mfmacell(int mode, const CellArgs<T>& a, const Tables<T>* tab, hipStream_t s) {
  if (a.g.dim != 3 || !a.qd || !a.elem || a.m.split != SPLIT_AMOR) return hipErrorInvalidValue;
  switch (a.g.k) {
    case 3: return launch_mk<3, T>(mode, a, tab, s);
    case 4: return launch_mk<4, T>(mode, a, tab, s);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_mfmacell<double>(int, const CellArgs<double>&, const Tables<double>*, hipStream_t);
template hipError_t launch_mfmacell<float>(int, const CellArgs<float>&, const Tables<float>*, hipStream_t);

}  // namespace mfpff
