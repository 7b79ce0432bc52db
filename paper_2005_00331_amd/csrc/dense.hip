// Dense FP64 kernels of the coarse-grid solve (gfx950).
//
// The coarsest level is solved exactly with the block lower-triangular
// structure of the Jacobian (Section 3.3): x_u = G_uu^-1 r_u,
// x_phi = G_phiphi^-1 (r_phi - G_phiu x_u).  Each diagonal block is factorised
// once per linearisation by a blocked right-looking Cholesky (panels of 32
// factored in LDS, trailing updates as tiled products), and the inverse
// factor W = L^-1 is formed by a blocked triangular solve, so that a V-cycle
// applies the coarse inverse as four dense matrix-vector products
// (A^-1 = W^T W) instead of sequential substitutions.  A block that is not
// positive definite is inverted explicitly by Gauss-Jordan elimination with
// partial pivoting instead (one product per solve).
#include <cmath>

#include "internal.h"

namespace mfpff {

constexpr int TB = 32;

__global__ void set_fixed_diag_kernel(double* A, long long ld, const uint8_t* mask, long long nn, int dim) {
  const long long n = (long long)(dim + 1) * nn;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const long long comp = udiv(i, nn);
    const uint8_t m = mask[i - comp * nn];
    const bool f = comp < dim ? (m & kMaskU) : (m & kMaskPhi);
    if (f) A[i * ld + i] = 1.0;
  }
}
void k_dense_set_fixed_diag(double* A, long long ld, const uint8_t* mask, long long nn, int dim, hipStream_t s) {
  long long nb = ((dim + 1) * nn + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(set_fixed_diag_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, A, ld, mask, nn, dim);
}

__global__ void extract_block_kernel(double* dst, long long ldd, const double* src, long long lds, long long r0, long long c0,
                                     long long nr, long long nc) {
  const long long total = nr * nc;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
    const long long r = i / nc, c = i - (i / nc) * nc;
    dst[r * ldd + c] = src[(r0 + r) * lds + c0 + c];
  }
}
void k_extract_block(double* dst, long long ldd, const double* src, long long lds, long long r0, long long c0, long long nr,
                     long long nc, hipStream_t s) {
  long long nb = (nr * nc + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(extract_block_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, dst, ldd, src, lds, r0, c0, nr, nc);
}

// v from lane `lane` (uniform), as two 32-bit reads into scalar registers
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Factor the diagonal block at k0 (identity padding past n) with one wavefront: lane i < TB
// holds row i in registers, each column of L goes through LDS once.  Block 0 writes L11 to
// `diag` (copied into A by the next launch, so that no block reads a half-written diagonal
// block); block b >= 1 solves X L11^T = A[rows of b][k0:k0+TB] in place.
constexpr int kPanelLanes = 64;
__global__ __launch_bounds__(kPanelLanes) void potrf_panel_kernel(double* A, int n, int k0, int* info, double* diag) {
  __shared__ double L[TB][TB + 1];
  __shared__ double X[TB][TB + 1];
  __shared__ double col[TB];
  __shared__ double rinv[TB];  // 1 / L[j][j]
  const int tid = threadIdx.x;
  // every load of the block (the diagonal block and, for b >= 1, its panel rows) is issued before
  // the first LDS store, so the block waits for memory once; lane t takes column t % TB of the
  // rows t / TB + 2 q
  constexpr int PER = TB * TB / kPanelLanes;
  const int lj = tid % TB, li = tid / TB;
  const int r0 = k0 + blockIdx.x * TB;
  double lv[PER], xv[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = li + q * (kPanelLanes / TB);
    const int gi = k0 + i, gj = k0 + lj, gx = r0 + i;
    lv[q] = (gi < n && gj < n) ? A[(long long)gi * n + gj] : (i == lj ? 1.0 : 0.0);
    xv[q] = (blockIdx.x > 0 && gx < n && gj < n) ? A[(long long)gx * n + gj] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = li + q * (kPanelLanes / TB);
    L[i][lj] = lv[q];
    X[i][lj] = xv[q];
  }
  __syncthreads();
  {
    const int i = tid < TB ? tid : TB - 1;  // lanes past TB shadow the last row and store nothing
    double row[TB];
#pragma clang loop unroll(full)
    for (int l = 0; l < TB; ++l) row[l] = L[i][l];
#pragma clang loop unroll(full)
    for (int j = 0; j < TB; ++j) {
      // every lane reads the pivot from lane j and takes r = 1 / sqrt(pivot) itself (one
      // reciprocal square root, no LDS round trip): L[j][j] = pivot * r, L[i][j] = A[i][j] * r
      double d = readlane_f64(row[j], j);
      if (!(d > 0.0)) {
        if (tid == j && blockIdx.x == 0) atomicMax(info, k0 + j + 1);
        d = 1.0;
      }
      const double r = rsqrt(d);
      if (tid == j) {
        row[j] = d * r;
        rinv[j] = r;
      } else if (tid > j && tid < TB) {
        row[j] *= r;
        col[tid] = row[j];
      }
      __syncthreads();
      if (tid > j && tid < TB) {
        const double lij = row[j];
#pragma clang loop unroll(full)
        for (int l = 0; l < TB; ++l)
          if (l > j) row[l] -= lij * col[l];  // entries past the diagonal are never read
      }
      __syncthreads();
    }
    if (tid < TB) {
#pragma clang loop unroll(full)
      for (int l = 0; l < TB; ++l) L[i][l] = row[l];
    }
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int e = tid; e < TB * TB; e += blockDim.x) diag[e] = L[e / TB][e % TB];
    return;
  }
  if (tid < TB) {
    // row tid of X L11^T = A_panel, unrolled so the row stays in registers
    const int i = tid;
    double xr[TB];
#pragma clang loop unroll(full)
    for (int j = 0; j < TB; ++j) xr[j] = X[i][j];
#pragma clang loop unroll(full)
    for (int j = 0; j < TB; ++j) {
      const double xj = xr[j] * rinv[j];
      xr[j] = xj;
#pragma clang loop unroll(full)
      for (int l = 0; l < TB; ++l)
        if (l > j) xr[l] -= xj * L[l][j];
    }
#pragma clang loop unroll(full)
    for (int j = 0; j < TB; ++j) X[i][j] = xr[j];
  }
  __syncthreads();
  for (int e = tid; e < TB * TB; e += blockDim.x) {
    const int i = e / TB, j = e % TB;
    const int gi = r0 + i, gj = k0 + j;
    if (gi < n && gj < n) A[(long long)gi * n + gj] = X[i][j];
  }
}

// Lower triangle of the factored diagonal block back into A (workgroup 0 of the launch that
// follows the panel kernel)
__device__ void copy_diag(double* A, int n, int k0, const double* diag) {
  for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) {
    const int i = e / TB, j = e % TB;
    const int gi = k0 + i, gj = k0 + j;
    if (gi < n && gj < n && j <= i) A[(long long)gi * n + gj] = diag[e];
  }
}
__global__ void copy_diag_kernel(double* A, int n, int k0, const double* diag) { copy_diag(A, n, k0, diag); }

// Trailing update A[i][j] -= sum_l L[i][l] L[j][l], l in the panel, for tiles bi >= bj
// (rows and columns past the panel, so the diagonal block is not touched: workgroup 0 also
// copies it back from `diag`).
__global__ __launch_bounds__(kThreads) void syrk_update_kernel(double* A, int n, int k0, const double* diag) {
  __shared__ double Li[TB][TB + 1];
  __shared__ double Lj[TB][TB + 1];
  if (blockIdx.x == 0) copy_diag(A, n, k0, diag);
  const int k1 = k0 + TB;
  // blockIdx.x -> (bi, bj), bi >= bj
  int t = blockIdx.x, bi = 0;
  while (t > bi) {
    t -= bi + 1;
    ++bi;
  }
  const int bj = t;
  const int ri = k1 + bi * TB, rj = k1 + bj * TB;
  const int tid = threadIdx.x;
  constexpr int PER = TB * TB / kThreads;
  const int ll = tid % TB, l0 = tid / TB;
  double a[PER], b[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = l0 + q * (kThreads / TB);
    const int gl = k0 + ll;
    a[q] = (ri + i < n && gl < n) ? A[(long long)(ri + i) * n + gl] : 0.0;
    b[q] = (rj + i < n && gl < n) ? A[(long long)(rj + i) * n + gl] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    Li[l0 + q * (kThreads / TB)][ll] = a[q];
    Lj[l0 + q * (kThreads / TB)][ll] = b[q];
  }
  __syncthreads();
  for (int e = tid; e < TB * TB; e += blockDim.x) {
    const int i = e / TB, j = e % TB;
    const int gi = ri + i, gj = rj + j;
    if (gi < n && gj < n && gj <= gi) {
      double acc = 0;
#pragma unroll 8
      for (int l = 0; l < TB; ++l) acc += Li[i][l] * Lj[j][l];
      A[(long long)gi * n + gj] -= acc;
    }
  }
}

hipError_t cholesky_lower(double* A, int n, int* info_dev, double* scratch, hipStream_t s) {
  for (int k0 = 0; k0 < n; k0 += TB) {
    const int nrb = (n - k0 + TB - 1) / TB;
    hipLaunchKernelGGL(potrf_panel_kernel, dim3(nrb), dim3(kPanelLanes), 0, s, A, n, k0, info_dev, scratch);
    const int k1 = k0 + TB;
    if (k1 < n) {
      const int nt = (n - k1 + TB - 1) / TB;
      hipLaunchKernelGGL(syrk_update_kernel, dim3(nt * (nt + 1) / 2), dim3(kThreads), 0, s, A, n, k0,
                         (const double*)scratch);
    } else {
      hipLaunchKernelGGL(copy_diag_kernel, dim3(1), dim3(kThreads), 0, s, A, n, k0, (const double*)scratch);
    }
  }
  return hipGetLastError();
}

__global__ void eye_kernel(double* W, int n) {
  const long long total = (long long)n * n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x)
    W[e] = (e / n == e % n) ? 1.0 : 0.0;
}
// W[k0:k0+TB, 0:ncols] = L11^-1 W[k0:k0+TB, 0:ncols]: one wave per block, one column per
// lane, staged through LDS and solved in registers; L11 is read from LDS at addresses common
// to the wave (broadcast)
constexpr int kTrsmLanes = 64;
__global__ __launch_bounds__(kTrsmLanes) void trsm_diag_kernel(double* W, const double* L, int n, int k0, int ncols) {
  __shared__ double L11[TB][TB + 1];
  __shared__ double xs[TB][kTrsmLanes];
  __shared__ double rinv[TB];  // 1 / L11[j][j]
  const int tid = threadIdx.x;
  const int col = blockIdx.x * kTrsmLanes + tid;
  const bool ok = col < ncols;
  // all loads (L11 and this lane's column of the TB rows of W) before the first LDS store
  constexpr int PER = TB * TB / kTrsmLanes;
  const int lj = tid % TB, li = tid / TB;
  double lv[PER], wv[TB];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = li + q * (kTrsmLanes / TB);
    const int gi = k0 + i, gj = k0 + lj;
    lv[q] = (gi < n && gj < n) ? L[(long long)gi * n + gj] : (i == lj ? 1.0 : 0.0);
  }
#pragma unroll
  for (int i = 0; i < TB; ++i) wv[i] = (ok && k0 + i < n) ? W[(long long)(k0 + i) * n + col] : 0.0;
#pragma unroll
  for (int q = 0; q < PER; ++q) L11[li + q * (kTrsmLanes / TB)][lj] = lv[q];
#pragma unroll
  for (int i = 0; i < TB; ++i) xs[i][tid] = wv[i];
  __syncthreads();
  if (tid < TB) rinv[tid] = 1.0 / L11[tid][tid];
  __syncthreads();
  double xr[TB];
#pragma clang loop unroll(full)
  for (int i = 0; i < TB; ++i) xr[i] = xs[i][tid];
#pragma clang loop unroll(full)
  for (int j = 0; j < TB; ++j) {
    const double xj = xr[j] * rinv[j];
    xr[j] = xj;
#pragma clang loop unroll(full)
    for (int i = 0; i < TB; ++i)
      if (i > j) xr[i] -= L11[i][j] * xj;
  }
#pragma clang loop unroll(full)
  for (int i = 0; i < TB; ++i) xs[i][tid] = xr[i];
  if (!ok) return;
  for (int i = 0; i < TB; ++i)
    if (k0 + i < n) W[(long long)(k0 + i) * n + col] = xs[i][tid];
}
// W[r][c] -= sum_l L[r][k0+l] W[k0+l][c] for r >= k0+TB, c < ncols
__global__ __launch_bounds__(kThreads) void trsm_update_kernel(double* W, const double* L, int n, int k0, int ncols) {
  __shared__ double Ls[TB][TB + 1];
  __shared__ double Ws[TB][TB + 1];
  const int r0 = k0 + TB + blockIdx.y * TB;
  const int c0 = blockIdx.x * TB;
  const int tid = threadIdx.x;
  constexpr int PER = TB * TB / kThreads;
  const int ll = tid % TB, l0 = tid / TB;
  double a[PER], b[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = l0 + q * (kThreads / TB);
    a[q] = (r0 + i < n && k0 + ll < n) ? L[(long long)(r0 + i) * n + k0 + ll] : 0.0;
    b[q] = (k0 + i < n && c0 + ll < ncols) ? W[(long long)(k0 + i) * n + c0 + ll] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    Ls[l0 + q * (kThreads / TB)][ll] = a[q];
    Ws[l0 + q * (kThreads / TB)][ll] = b[q];
  }
  __syncthreads();
  for (int e = tid; e < TB * TB; e += blockDim.x) {
    const int i = e / TB, j = e % TB;
    if (r0 + i < n && c0 + j < ncols) {
      double acc = 0;
#pragma unroll 8
      for (int l = 0; l < TB; ++l) acc += Ls[i][l] * Ws[l][j];
      W[(long long)(r0 + i) * n + c0 + j] -= acc;
    }
  }
}

hipError_t tri_inverse_lower(double* W, const double* L, int n, hipStream_t s) {
  const long long total = (long long)n * n;
  long long nb = (total + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(eye_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, W, n);
  for (int k0 = 0; k0 < n; k0 += TB) {
    const int ncols = k0 + TB < n ? k0 + TB : n;
    hipLaunchKernelGGL(trsm_diag_kernel, dim3((ncols + kTrsmLanes - 1) / kTrsmLanes), dim3(kTrsmLanes), 0, s, W, L, n, k0,
                       ncols);
    const int rows = n - (k0 + TB);
    if (rows > 0) {
      dim3 grid((ncols + TB - 1) / TB, (rows + TB - 1) / TB);
      hipLaunchKernelGGL(trsm_update_kernel, grid, dim3(kThreads), 0, s, W, L, n, k0, ncols);
    }
  }
  return hipGetLastError();
}

// Gauss-Jordan inversion with partial pivoting, the fallback for a coarse block whose Cholesky met
// a non-positive pivot (an indefinite block, which a negative degradation floor produces).  Step k
// takes the row of largest |M[i][k]|, i >= k (the first one on ties), swaps it into row k, scales
// row k by the pivot and clears column k from every other row; the same row operations turn the
// identity into M^-1.  work[0..n) holds the multipliers of a step, work[n..n+3) the pivot value,
// its row and the old M[k][k].  Columns left of k in M are not kept up to date: no later step
// reads them.
constexpr int kPivLanes = 1024;
__global__ __launch_bounds__(kPivLanes) void gj_pivot_kernel(const double* M, int n, int k, double* work, int* info) {
  __shared__ double sv[kPivLanes];
  __shared__ int si[kPivLanes];
  double best = -1.0;
  int bi = k;
  for (int i = k + (int)threadIdx.x; i < n; i += kPivLanes) {
    const double v = fabs(M[(long long)i * n + k]);
    if (v > best) {
      best = v;
      bi = i;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int w = kPivLanes / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double ov = sv[threadIdx.x + w];
      const int oi = si[threadIdx.x + w];
      if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int p = si[0];
    double pv = M[(long long)p * n + k];
    if (!(sv[0] > 0.0)) {  // a zero (or NaN) column: the block is singular
      if (*info == 0) *info = k + 1;
      pv = 1.0;
    }
    work[n] = pv;
    work[n + 1] = (double)p;
    work[n + 2] = M[(long long)k * n + k];
  }
}

__global__ void gj_swap_scale_kernel(double* M, double* Inv, int n, int k, double* work) {
  const double pv = work[n];
  const int p = (int)work[n + 1];
  const double mkk = work[n + 2];
  const double rp = 1.0 / pv;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    // multiplier of row j: column k after the swap (rows k and p are the only ones written here)
    work[j] = j == k ? 0.0 : (j == p ? mkk : M[(long long)j * n + k]);
    const double mk = M[(long long)k * n + j], mp = M[(long long)p * n + j];
    const double ik = Inv[(long long)k * n + j], ip = Inv[(long long)p * n + j];
    M[(long long)p * n + j] = mk;
    Inv[(long long)p * n + j] = ik;
    M[(long long)k * n + j] = mp * rp;
    Inv[(long long)k * n + j] = ip * rp;
  }
}

__global__ void gj_eliminate_kernel(double* M, double* Inv, int n, int k, const double* f) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double mk = M[(long long)k * n + j], ik = Inv[(long long)k * n + j];
  for (int i = blockIdx.y; i < n; i += gridDim.y) {
    const double fi = f[i];
    if (i == k || fi == 0.0) continue;
    if (j > k) M[(long long)i * n + j] -= fi * mk;
    Inv[(long long)i * n + j] -= fi * ik;
  }
}

hipError_t gauss_jordan_inverse(double* Inv, double* M, int n, int* info_dev, double* work, hipStream_t s) {
  const long long total = (long long)n * n;
  long long nb = (total + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(eye_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, Inv, n);
  const unsigned gx = (unsigned)((n + kThreads - 1) / kThreads);
  const unsigned gy = (unsigned)(n < 256 ? n : 256);
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(gj_pivot_kernel, dim3(1), dim3(kPivLanes), 0, s, (const double*)M, n, k, work, info_dev);
    hipLaunchKernelGGL(gj_swap_scale_kernel, dim3(gx), dim3(kThreads), 0, s, M, Inv, n, k, work);
    hipLaunchKernelGGL(gj_eliminate_kernel, dim3(gx, gy), dim3(kThreads), 0, s, M, Inv, n, k, (const double*)work);
  }
  return hipGetLastError();
}

__global__ void transpose_kernel(double* At, const double* A, int n) {
  __shared__ double t[TB][TB + 1];
  const int bx = blockIdx.x * TB, by = blockIdx.y * TB;
  for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) {
    const int i = e / TB, j = e % TB;
    if (by + i < n && bx + j < n) t[i][j] = A[(long long)(by + i) * n + bx + j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) {
    const int i = e / TB, j = e % TB;
    if (bx + i < n && by + j < n) At[(long long)(bx + i) * n + by + j] = t[j][i];
  }
}
void k_transpose(double* At, const double* A, int n, hipStream_t s) {
  dim3 grid((n + TB - 1) / TB, (n + TB - 1) / TB);
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(kThreads), 0, s, At, A, n);
}

// y = alpha * A x + yin.  One workgroup per row: thread t takes the columns t, t + 256, ...
// in chunks of kGemvChunk per thread whose loads are all issued before the first product
// (the tail of a chunk reads a clamped in-range column with weight 0), so a row of a few
// thousand columns costs one or two memory round trips; then a fixed-order block reduction.
constexpr int kGemvChunk = 8;
// Vec: x and yin as FP64 or FP32 (the FP32 V-cycle's coarse right-hand side is read as it is);
// y32, if given, receives y rounded to FP32 as well (the FP32 V-cycle's coarse solution); y may
// be null then
__device__ __forceinline__ double vec_at(const void* v, int f32, int j) {
  return f32 ? (double)static_cast<const float*>(v)[j] : static_cast<const double*>(v)[j];
}
__global__ __launch_bounds__(kThreads) void gemv_kernel(double* y, float* y32, const double* A, long long lda,
                                                        const void* x, int x32, int cols, double alpha, const void* yin,
                                                        int yin32, int shape) {
  __shared__ double part[kThreads / 64];
  const int row = blockIdx.x;
  const int t = threadIdx.x;
  const int j0 = shape == GEMV_UPPER ? row : 0;
  const int j1 = shape == GEMV_LOWER ? row + 1 : cols;
  const double* a = A + (long long)row * lda;
  double acc = 0;
  for (int base = j0 + t; base < j1; base += kGemvChunk * kThreads) {
    double av[kGemvChunk], xv[kGemvChunk];
#pragma unroll
    for (int i = 0; i < kGemvChunk; ++i) {
      const int j = min(base + i * kThreads, j1 - 1);
      av[i] = a[j];
      xv[i] = vec_at(x, x32, j);
    }
#pragma unroll
    for (int i = 0; i < kGemvChunk; ++i) acc += base + i * kThreads < j1 ? av[i] * xv[i] : 0.0;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((t & 63) == 0) part[t >> 6] = acc;
  __syncthreads();
  if (t == 0) {
    double s = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) s += part[w];
    const double v = alpha * s + (yin ? vec_at(yin, yin32, row) : 0.0);
    if (y) y[row] = v;
    if (y32) y32[row] = (float)v;
  }
}
void k_gemv(double* y, const double* A, long long lda, const double* x, int rows, int cols, double alpha, const double* yin,
            int shape, hipStream_t s) {
  k_gemv_mixed(y, nullptr, A, lda, x, false, rows, cols, alpha, yin, false, shape, s);
}
void k_gemv_mixed(double* y, float* y32, const double* A, long long lda, const void* x, bool x32, int rows, int cols,
                  double alpha, const void* yin, bool yin32, int shape, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(gemv_kernel, dim3((unsigned)rows), dim3(kThreads), 0, s, y, y32, A, lda, x, x32 ? 1 : 0, cols, alpha,
                     yin, yin32 ? 1 : 0, shape);
}

}  // namespace mfpff
