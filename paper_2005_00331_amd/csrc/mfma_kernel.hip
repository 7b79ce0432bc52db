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
// Blocks are small, so little of each instruction is padding (none at degree 3; at degree 4
// the 5 or 10 rows fill 8 or 12 and, in FP64, the contraction of length 5 fills 8).
//
// Data flow per workgroup of CW cells, 12 LDS tensors [cell][z][y][x], three per field:
//   1. trial values by node line into LDS;
//   2. x-step of all four fields: [B; D] X -> (Bx X, Dx X), in place;
//   3. y-step: [B; D] (Bx X) -> (By Bx X, Dy Bx X), By (Dx X), in place;
//   4. per group of z-lines, in registers: the z-step (d/dx = Bz By Dx X, d/dy = Bz Dy Bx X,
//      d/dz = Dz By Bx X, phi value = Bz By Bx X) for all four fields, eq. (G) at each Gauss
//      point from the cached tangent coefficients (one lane and register per point), and the
//      transposed z-step of every test component, whose inputs are the fluxes exactly where the
//      forward outputs left them (the output rows of one instruction are the contraction indices
//      of the next); results go back to LDS in place;
//   5. transposed y-step and 6. transposed x-step of all four components, in place;
//   7. the cell results leave through the element buffer in the layout of the other 3D
//      kernels, so the node gather and its fused epilogues are shared.
// Six barriers per workgroup; every contraction of steps 2, 3, 5 and 6 covers the lines of all
// four fields or components at once.
#include "cell_common.h"

namespace mfpff {

namespace {

typedef float mx_v4f __attribute__((ext_vector_type(4)));

// lane layouts of the two instructions (lane l of the 64-wide wavefront):
//  f64 4x4x4, block b = (l & 15) >> 2: A_b[row l & 3][k l >> 4], B_b[k l >> 4][col l & 3],
//           D_b[row l >> 4][col l & 3]; so the 16 columns of one instruction are the lines
//           l & 15, lane l feeds contraction index (l >> 4) + 4 s in step s and receives
//           row (l >> 4) + 4 m of row block m
//  f32 4x4x1, block b = l >> 2: A_b[row l & 3][0], B_b[0][col l & 3], D_b[row r][col l & 3]
//           in register r; so the 64 columns are the lines l, every lane feeds contraction
//           index s in step s and receives rows 4 m .. 4 m + 3
template <typename T>
struct Mx;
template <>
struct Mx<double> {
  static constexpr int LPI = 16;  // lines per instruction
  static constexpr int KK = 4;    // contraction indices per instruction
  static constexpr int RPL = 1;   // rows of a row block held per lane
  using Acc = double;
  __device__ static int line(int l) { return l & 15; }
  __device__ static int kb(int l) { return l >> 4; }  // contraction index fed by this lane (B operand)
  __device__ static int ar(int l) { return l & 3; }   // A operand row
  __device__ static int ak(int l) { return l >> 4; }  // A operand contraction index
  __device__ static Acc zero() { return 0.0; }
  __device__ static Acc mma(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int l, int m, int) { return (l >> 4) + 4 * m; }  // output row of (m, register)
  __device__ static double get(const Acc& c, int) { return c; }
  __device__ static void put(Acc& c, int, double v) { c = v; }
};
template <>
struct Mx<float> {
  static constexpr int LPI = 64;
  static constexpr int KK = 1;
  static constexpr int RPL = 4;
  using Acc = mx_v4f;
  __device__ static int line(int l) { return l; }
  __device__ static int kb(int) { return 0; }
  __device__ static int ar(int l) { return l & 3; }
  __device__ static int ak(int) { return 0; }
  __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static Acc mma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int, int m, int r) { return 4 * m + r; }
  __device__ static float get(const Acc& c, int r) { return c[r]; }
  __device__ static void put(Acc& c, int r, float v) { c[r] = v; }
};

// 1D table selectors of a contraction: A[r][k] = B[r][k], D[r][k], B[k][r] or D[k][r]
enum { TB = 0, TD = 1, TBT = 2, TDT = 3, TNONE = 4 };

template <typename T>
__device__ __forceinline__ T table_at(int t, int r, int k, const T* Bs, const T* Ds, int NP) {
  return t == TB ? Bs[r * NP + k] : t == TD ? Ds[r * NP + k] : t == TBT ? Bs[k * NP + r] : t == TDT ? Ds[k * NP + r] : T(0);
}

template <int K, typename T>
struct MShape {
  static constexpr int NP = K + 1;
  static constexpr int P = NP * NP * NP;
  static constexpr int L = NP * NP;
  static constexpr int CPB = kThreads / P;  // cells per block of the shared cache / element layouts
  // cells per workgroup: whole layout blocks; the 12 tensors and the coefficients of CW cells take
  // 80 KB (two workgroups per CU)
  static constexpr int CW = sizeof(T) == 8 ? (K == 4 ? 4 : 8) : (K == 4 ? 8 : 16);
  static constexpr int TS = CW * P;          // one LDS tensor
  static constexpr int NL = CW * L;          // lines of one field in one direction
  static constexpr int NTEN = 12;
};

// line number ln (cell c, the other two axes (j, kq) in increasing order) -> its first position
template <int NP, int AXIS>
__device__ __forceinline__ int line_base(int ln) {
  constexpr int P = NP * NP * NP, L = NP * NP;
  const int c = ln / L, rl = ln - c * L;
  const int j = rl % NP, kq = rl / NP;
  return c * P + (AXIS == 0 ? NP * j + L * kq : (AXIS == 1 ? j + L * kq : j + NP * kq));
}

// One contraction step along AXIS for the lines of NF tensor groups (fields) at once, shared by
// the waves: NR stacked row sets (outputs o0, o1) times NS concatenated segments (inputs i0, i1)
// with table Trs for row set r and segment s; the tensors of group f are the given pointers plus
// f * GS.  Outputs may overwrite the inputs (in place): every lane loads all contraction indices
// of its lines before any output of those lines is stored, and no other lane or wave reads them.
template <typename T, int NP, int CW, int AXIS, int NF, int NR, int NS, int T00, int T01, int T10, int T11>
__device__ __forceinline__ void contract(const T* i0, const T* i1, T* o0, T* o1, int GS, const T* Bs, const T* Ds,
                                         int lane, int wave, int nwaves) {
  using X = Mx<T>;
  constexpr int L = NP * NP, NL = CW * L;
  constexpr int R = NR * NP, NRB = (R + 3) / 4;
  constexpr int KT = NS * NP, NKS = (KT + X::KK - 1) / X::KK;
  constexpr int ST = AXIS == 0 ? 1 : (AXIS == 1 ? NP : NP * NP);
  // operator values of this lane per row block and contraction step (loop invariant)
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
        v = table_at<T>(t, rr, kk, Bs, Ds, NP);
      }
      av[m][s] = v;
    }
  constexpr int NIT1 = (NL + X::LPI - 1) / X::LPI;  // instruction groups per field
  for (int it = wave; it < NF * NIT1; it += nwaves) {
    const int f = it / NIT1, itl = it - f * NIT1;
    const int ln = itl * X::LPI + X::line(lane);
    const bool lv = ln < NL;
    const int base = line_base<NP, AXIS>(lv ? ln : 0) + f * GS;
    T bv[NKS];
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
      // padding lanes read index 0 of segment 0 (inside the tensor) and are zeroed
      const int k = X::kb(lane) + X::KK * s;
      const bool kv = lv && k < KT;
      const int kc = kv ? k : 0;
      const int ks = kc / NP, kk = kc - ks * NP;
      bv[s] = keep_if((ks == 0 ? i0 : i1)[base + ST * kk], kv);
    }
#pragma unroll
    for (int m = 0; m < NRB; ++m) {
      typename X::Acc acc = X::zero();
#pragma unroll
      for (int s = 0; s < NKS; ++s) acc = X::mma(av[m][s], bv[s], acc);
#pragma unroll
      for (int q = 0; q < X::RPL; ++q) {
        const int r = X::row(lane, m, q);
        if (lv && r < R) {
          const int rs = r / NP, rr = r - rs * NP;
          (rs == 0 ? o0 : o1)[base + ST * rr] = X::get(acc, q);
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
// two waves per SIMD: the LDS of two workgroups fills the CU, so more would not run anyway
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void mfmacell_kernel(
    CellArgs<T> a, const Tables<T>* __restrict__ tabd) {
  using S = MShape<K, T>;
  using X = Mx<T>;
  using Acc = typename X::Acc;
  constexpr int NP = S::NP, P = S::P, L = S::L, CPB = S::CPB, CW = S::CW, TS = S::TS, NL = S::NL;
  constexpr int NQ = n_qcoef<3>();
  constexpr int NC = 4;
  constexpr int NRB = (NP + 3) / 4;                  // row blocks of NP rows (z-step outputs)
  constexpr int NKS = (NP + X::KK - 1) / X::KK;      // steps of a contraction of length NP
  __shared__ T lds[S::NTEN * TS];
  // the workgroup's cached tangent coefficients, copied in their layout [block][coefficient][point]
  // [cell of the block] at the start, so that the point physics of step 4 reads LDS
  __shared__ T ldq[CW * NQ * P];
  __shared__ T Bs[NP * NP], Ds[NP * NP], Ws[NP];
  // tensor slots of field f: 3f, 3f+1, 3f+2
  auto SL = [&](int t) { return lds + t * TS; };

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
  {
    // whole layout blocks of this workgroup that exist (the last workgroup may have fewer)
    const long long blk0 = cell0 / CPB, nblk = (ncells + CPB - 1) / CPB;
    const long long have = (nblk - blk0) * NQ * P * CPB;
    const int len = (int)(have < (long long)CW * NQ * P ? have : (long long)CW * NQ * P);
    const T* src = a.qd + blk0 * NQ * P * CPB;
#pragma unroll 4
    for (int i = tid; i < len; i += kThreads) ldq[i] = src[i];
  }

  // ---- 1. trial values by x-line (one thread per line of a cell), zero at fixed dofs, into slot 3f
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
      const long long nd = MFPFF_IN(n0 + i, nn);
      mk[i] = a.mask ? a.mask[nd] : (uint8_t)0;
#pragma unroll
      for (int f = 0; f < NC; ++f) xl[f][i] = a.x[f * nn + nd];
    }
    const int o = c * P + NP * la + L * lb;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const bool ku = valid && !(mk[i] & kMaskU), kp = valid && !(mk[i] & kMaskPhi);
#pragma unroll
      for (int f = 0; f < NC; ++f) SL(3 * f)[o + i] = keep_if(xl[f][i], f < 3 ? ku : kp);
    }
  }
  __syncthreads();
  // ---- 2. x-step: [B; D] X -> (Bx X in slot 3f, Dx X in slot 3f+1)
  contract<T, NP, CW, 0, NC, 2, 1, TB, TNONE, TD, TNONE>(SL(0), nullptr, SL(0), SL(1), 3 * TS, Bs, Ds, lane, wave,
                                                         nwaves);
  __syncthreads();
  // ---- 3. y-step: [B; D] (Bx X) -> (U00 in slot 3f, U01 in slot 3f+2); By (Dx X) -> U10 in slot 3f+1
  contract<T, NP, CW, 1, NC, 2, 1, TB, TNONE, TD, TNONE>(SL(0), nullptr, SL(0), SL(2), 3 * TS, Bs, Ds, lane, wave,
                                                         nwaves);
  contract<T, NP, CW, 1, NC, 1, 1, TB, TNONE, TNONE, TNONE>(SL(1), nullptr, SL(1), nullptr, 3 * TS, Bs, Ds, lane, wave,
                                                            nwaves);
  __syncthreads();

  // ---- 4. z-lines in registers: forward z-step, point physics, transposed z-step
  {
    // operator values of this lane: forward B and D (rows q, index i), transposed B^T and D^T
    // (rows i, index q), per row block m and step s
    T aB[NRB][NKS], aD[NRB][NKS], aBt[NRB][NKS], aDt[NRB][NKS];
#pragma unroll
    for (int m = 0; m < NRB; ++m)
#pragma unroll
      for (int s = 0; s < NKS; ++s) {
        const int r = 4 * m + X::ar(lane), k = X::ak(lane) + X::KK * s;
        const bool ok = r < NP && k < NP;
        const int rc = ok ? r : 0, kc = ok ? k : 0;
        aB[m][s] = keep_if(Bs[rc * NP + kc], ok);
        aD[m][s] = keep_if(Ds[rc * NP + kc], ok);
        aBt[m][s] = keep_if(Bs[kc * NP + rc], ok);
        aDt[m][s] = keep_if(Ds[kc * NP + rc], ok);
      }
    const T h = (T)g.h, ih = T(1) / h;
    const T Gc = (T)a.m.Gc, eps = (T)a.m.eps, lam = (T)a.m.lam, mu = (T)a.m.mu;
    const T Kb = lam + T(2) * mu / T(3);
    constexpr int SI[6] = {0, 1, 2, 0, 0, 1};
    constexpr int SJ[6] = {0, 1, 2, 1, 2, 2};
    constexpr int QS = P * CPB;
    constexpr int NIT = (NL + X::LPI - 1) / X::LPI;
    for (int it = wave; it < NIT; it += nwaves) {
      const int ln = it * X::LPI + X::line(lane);
      const bool lv = ln < NL;
      const int base = line_base<NP, 2>(lv ? ln : 0);
      const int c = (lv ? ln : 0) / L;
      // forward: G[f][0..2] = d/dx, d/dy, d/dz of field f, pv = phi value, per row block
      Acc G[NC][3][NRB], pv[NRB];
#pragma unroll
      for (int f = 0; f < NC; ++f) {
        T b00[NKS], b01[NKS], b10[NKS];
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
          const int k = X::kb(lane) + X::KK * s;
          const bool kv = lv && k < NP;
          const int o = base + L * (kv ? k : 0);
          b00[s] = keep_if(SL(3 * f)[o], kv);
          b10[s] = keep_if(SL(3 * f + 1)[o], kv);
          b01[s] = keep_if(SL(3 * f + 2)[o], kv);
        }
#pragma unroll
        for (int m = 0; m < NRB; ++m) {
          Acc gx = X::zero(), gy = X::zero(), gz = X::zero(), gv = X::zero();
#pragma unroll
          for (int s = 0; s < NKS; ++s) {
            gx = X::mma(aB[m][s], b10[s], gx);
            gy = X::mma(aB[m][s], b01[s], gy);
            gz = X::mma(aD[m][s], b00[s], gz);
            if (f == 3) gv = X::mma(aB[m][s], b00[s], gv);
          }
          G[f][0][m] = gx;
          G[f][1][m] = gy;
          G[f][2][m] = gz;
          if (f == 3) pv[m] = gv;
        }
      }
      // eq. (G) at the Gauss point of every (row block, register): the line kernel's per-point
      // code from the cached coefficients; derivatives become fluxes, the phi value the point term
      const long long cell = cell0 + c;
      const bool cvalid = lv && cell < ncells;
      const int cb = cvalid ? c / CPB : 0, cw = cvalid ? c - (c / CPB) * CPB : 0;  // block and cell in it
      const int pxy = base - c * P;  // q0 + NP q1
      const int q0 = pxy % NP, q1 = pxy / NP;
#pragma unroll
      for (int m = 0; m < NRB; ++m)
#pragma unroll
        for (int q = 0; q < X::RPL; ++q) {
          const int q2 = X::row(lane, m, q);
          const bool valid = cvalid && q2 < NP;
          const int q2c = q2 < NP ? q2 : 0;
          const int p = pxy + L * q2c;
          const T* qq = ldq + cb * NQ * P * CPB + cw + p * CPB;
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
          T de[3][3];
          T dt = 0;
#pragma unroll
          for (int i = 0; i < 3; ++i) {
#pragma unroll
            for (int j = 0; j < 3; ++j)
              de[i][j] = T(0.5) * (X::get(G[i][j][m], q) + X::get(G[j][i][m], q)) * ih;
            dt += de[i][i];
          }
          const T vol = cvol * dt;
          const T dph = X::get(pv[m], q);
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
          // padding rows and lines get zero fluxes, so that they add nothing in the transposed step
          const T jxw = keep_if(Ws[q0] * Ws[q1] * Ws[q2c] * h * h * h, valid);
          const T jg = jxw * ih;
#pragma unroll
          for (int cc = 0; cc < 3; ++cc)
#pragma unroll
            for (int mm = 0; mm < 3; ++mm) X::put(G[cc][mm][m], q, jg * Su[cc][mm]);
#pragma unroll
          for (int mm = 0; mm < 3; ++mm) X::put(G[3][mm][m], q, jg * Gc * eps * X::get(G[3][mm][m], q) * ih);
          X::put(pv[m], q, jxw * fval);
        }
      // transposed z-step of component tc: a1 = D^T F2 (+ B^T Fv) -> slot 3tc, a2 = B^T F0 -> slot
      // 3tc+1, a3 = B^T F1 -> slot 3tc+2; the B operand of step s is the flux at row s of the lane's
      // line, held by this lane (FP64: row block s; FP32: row block s/4, register s%4)
#pragma unroll
      for (int tc = 0; tc < NC; ++tc) {
        T f0[NKS], f1[NKS], f2[NKS], fv[NKS];
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
          const int mb = (s * X::KK) / 4, rb = (s * X::KK) % 4;
          f0[s] = X::get(G[tc][0][mb], rb);
          f1[s] = X::get(G[tc][1][mb], rb);
          f2[s] = X::get(G[tc][2][mb], rb);
          fv[s] = X::get(pv[mb], rb);
        }
#pragma unroll
        for (int m = 0; m < NRB; ++m) {
          Acc a1 = X::zero(), a2 = X::zero(), a3 = X::zero();
#pragma unroll
          for (int s = 0; s < NKS; ++s) {
            a1 = X::mma(aDt[m][s], f2[s], a1);
            a2 = X::mma(aBt[m][s], f0[s], a2);
            a3 = X::mma(aBt[m][s], f1[s], a3);
          }
          if (tc == 3) {
#pragma unroll
            for (int s = 0; s < NKS; ++s) a1 = X::mma(aBt[m][s], fv[s], a1);
          }
#pragma unroll
          for (int q = 0; q < X::RPL; ++q) {
            const int r = X::row(lane, m, q);
            if (lv && r < NP) {
              const int o = base + L * r;
              SL(3 * tc)[o] = X::get(a1, q);
              SL(3 * tc + 1)[o] = X::get(a2, q);
              SL(3 * tc + 2)[o] = X::get(a3, q);
            }
          }
        }
      }
    }
  }
  __syncthreads();
  // ---- 5. transposed y-step: b1 = By^T a1 + Dy^T a3 -> slot 3tc, b2 = By^T a2 -> slot 3tc+1
  contract<T, NP, CW, 1, NC, 1, 2, TBT, TDT, TNONE, TNONE>(SL(0), SL(2), SL(0), nullptr, 3 * TS, Bs, Ds, lane, wave,
                                                           nwaves);
  contract<T, NP, CW, 1, NC, 1, 1, TBT, TNONE, TNONE, TNONE>(SL(1), nullptr, SL(1), nullptr, 3 * TS, Bs, Ds, lane, wave,
                                                             nwaves);
  __syncthreads();
  // ---- 6. transposed x-step: Bx^T b1 + Dx^T b2 -> slot 3tc
  contract<T, NP, CW, 0, NC, 1, 2, TBT, TDT, TNONE, TNONE>(SL(0), SL(1), SL(0), nullptr, 3 * TS, Bs, Ds, lane, wave,
                                                           nwaves);
  __syncthreads();

  // ---- 7. element buffer: one coalesced copy in the shared layout
  // [block][component][point][cell of the block] from the slots 0, 3, 6, 9 ([cell][point])
  T* eb = a.elem + cell0 * NC * P;
  for (int idx = tid; idx < CW * NC * P; idx += kThreads) {
    const int ob = idx / (CPB * NC * P);
    const int r = idx - ob * (CPB * NC * P);
    const int rem = r / CPB, c2 = r - rem * CPB;
    const int cc = rem / P, p = rem - cc * P;
    const int cl = ob * CPB + c2;
    if (cell0 + cl < ncells) eb[idx] = SL(3 * cc)[cl * P + p];
  }
}

template <int K, typename T>
static hipError_t launch_mk(int mode, const CellArgs<T>& a, const Tables<T>* tab, hipStream_t s) {
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

MFPFF_BOUNDS_READER(bounds_hits_mfma)
