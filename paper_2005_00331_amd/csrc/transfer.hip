// Level transfers (gfx950).  The prolongation between nested structured
// levels is the Kronecker product over axes of one 1D interpolation matrix
// (coarse basis functions evaluated at fine nodes), applied per component;
// restriction is its transpose.  Both can be applied axis by axis: each pass
// maps one axis through a padded row-sparse 1D matrix (thread per output
// entry, gather, no atomics), so a 3D transfer reads each input a few times
// instead of (k+1)^3 times; the masks are fused into the first and last pass.
// In 2D the prolongation is one gather pass (prolong_kernel), which saves a
// launch on the small levels.
#include "bounds.h"
#include "internal.h"

namespace mfpff {

struct Dims3 {
  long long n[3];
};

__device__ __forceinline__ bool comp_fixed(const uint8_t* mask, long long node, long long comp, int dim) {
  const uint8_t m = mask[node];
  return comp < dim ? (m & kMaskU) : (m & kMaskPhi);
}

template <typename T>
__global__ void axis_apply_kernel(T* out, const T* in, const int* col, const double* val, const float* valf, int width,
                                  int axis, int dim, Dims3 din, int nout_axis, int ncomp, const uint8_t* in_mask,
                                  const uint8_t* out_mask, int add, ChebStart<T> cs) {
  long long nin[3] = {din.n[0], din.n[1], din.n[2]};
  long long no[3] = {nin[0], nin[1], nin[2]};
  no[axis] = nout_axis;
  long long per_in = 1, per_out = 1;
  for (int a = 0; a < dim; ++a) {
    per_in *= nin[a];
    per_out *= no[a];
  }
  const long long total = per_out * ncomp;
  long long sin[3] = {1, nin[0], nin[0] * nin[1]};
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long long)gridDim.x * blockDim.x) {
    const unsigned comp = udiv(idx, per_out);
    unsigned rem = (unsigned)(idx - (long long)comp * per_out);
    long long o[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
      const unsigned q = rem / (unsigned)no[a];
      o[a] = rem - q * (unsigned)no[a];
      rem = q;
    }
    long long base = comp * per_in;
    for (int a = 0; a < dim; ++a)
      if (a != axis) base += o[a] * sin[a];
    const int row = (int)o[axis];
    T acc = 0;
    const bool ofix = out_mask && comp_fixed(out_mask, (idx - comp * per_out), comp, dim);
    if (!ofix) {
      for (int j = 0; j < width; ++j) {
        const int ci = col[row * width + j];
        if (ci < 0) break;
        const T w = sizeof(T) == 8 ? (T)val[row * width + j] : (T)valf[row * width + j];
        const long long ii = MFPFF_IN(base + (long long)ci * sin[axis], per_in * ncomp);
        if (in_mask && comp_fixed(in_mask, ii - comp * per_in, comp, dim)) continue;
        acc += w * in[ii];
      }
    }
    if (!add) out[idx] = acc;
    else if (!ofix) out[idx] += acc;
    if (cs.z0) {
      const T zv = cs.dinv[idx] * acc * (comp < (unsigned)dim ? cs.ith_u : cs.ith_p);
      cs.z0[idx] = zv;
      cs.d0[idx] = zv;
    }
  }
}

template <typename T>
void k_axis_apply(T* out, const T* in, const Sparse1D& A, int axis, int dim, const long long* dims_in, int ncomp,
                  const uint8_t* in_mask, const uint8_t* out_mask, hipStream_t s, bool add, ChebStart<T> cs) {
  Dims3 d{{dims_in[0], dims_in[1], dim == 3 ? dims_in[2] : 1}};
  long long total = ncomp;
  for (int a = 0; a < dim; ++a) total *= (a == axis ? A.n_out : d.n[a]);
  long long nb = (total + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(axis_apply_kernel<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, out, in, A.col, A.val, A.valf, A.width,
                     axis, dim, d, A.n_out, ncomp, in_mask, out_mask, add ? 1 : 0, cs);
}

// out = / += P~ xc on the fine level (2D): gather of the coarse values of a fine node's row
// pair; W is the padded row width and every load is issued unconditionally (padding reads
// node 0 with weight 0)
template <typename T, int W>
__global__ void prolong_kernel(T* out, const T* xc, const int* col, const double* val, const float* valf,
                               const uint8_t* mask_c, const uint8_t* mask_f, Geom gf, Geom gc, int add) {
  const long long nnf = gf.n_nodes, nnc = gc.n_nodes;
  const unsigned Mf = (unsigned)gf.M;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nnf; i += (long long)gridDim.x * blockDim.x) {
    const unsigned q = (unsigned)i / Mf;
    const int f0 = (int)((unsigned)i - q * Mf), f1 = (int)q;
    int c0[W], c1[W];
    T w0[W], w1[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int a = col[f0 * W + j], b = col[f1 * W + j];
      c0[j] = a < 0 ? 0 : a;
      c1[j] = b < 0 ? 0 : b;
      w0[j] = a < 0 ? T(0) : (sizeof(T) == 8 ? (T)val[f0 * W + j] : (T)valf[f0 * W + j]);
      w1[j] = b < 0 ? T(0) : (sizeof(T) == 8 ? (T)val[f1 * W + j] : (T)valf[f1 * W + j]);
    }
    T v[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int j1 = 0; j1 < W; ++j1) {
#pragma unroll
      for (int j0 = 0; j0 < W; ++j0) {
        const T w = w1[j1] * w0[j0];
        const long long nc = MFPFF_IN(c0[j0] + (long long)gc.M * c1[j1], nnc);
        const uint8_t mc = mask_c[nc];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          const T xv = xc[cc * nnc + nc];
          v[cc] += w * keep_if(xv, !(cc < 2 ? (mc & kMaskU) : (mc & kMaskPhi)));
        }
      }
    }
    const uint8_t mf = mask_f[i];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const bool fx = cc < 2 ? (mf & kMaskU) : (mf & kMaskPhi);
      const long long idx = cc * nnf + i;
      if (add) {
        if (!fx) out[idx] += v[cc];
      } else {
        out[idx] = fx ? T(0) : v[cc];
      }
    }
  }
}

template <typename T>
void k_prolong(T* out, const T* xc, const Sparse1D& P, const uint8_t* mask_c, const uint8_t* mask_f, const Geom& gf,
               const Geom& gc, bool add, hipStream_t s) {
  long long nb = (gf.n_nodes + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  const dim3 g((unsigned)nb), b(kThreads);
#define MFPFF_PW(WW)                                                                                                 \
  case WW:                                                                                                           \
    hipLaunchKernelGGL((prolong_kernel<T, WW>), g, b, 0, s, out, xc, P.col, P.val, P.valf, mask_c, mask_f, gf, gc, \
                       add ? 1 : 0);                                                                                 \
    break;
  switch (P.width) {
    MFPFF_PW(1) MFPFF_PW(2) MFPFF_PW(3) MFPFF_PW(4) MFPFF_PW(5)
    default: break;  // the host uses the axis passes for wider rows
  }
#undef MFPFF_PW
}



// zero the fixed dofs of a level vector
template <typename T>
__global__ void mask_comp_kernel(T* y, const uint8_t* mask, long long nn, int dim) {
  const long long n = (long long)(dim + 1) * nn;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const long long comp = udiv(i, nn);
    const uint8_t m = mask[i - comp * nn];
    const bool f = comp < dim ? (m & kMaskU) : (m & kMaskPhi);
    if (f) y[i] = T(0);
  }
}
template <typename T>
void k_mask_comp(T* y, const uint8_t* mask, long long nn, int dim, hipStream_t s) {
  long long nb = ((dim + 1) * nn + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(mask_comp_kernel<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, y, mask, nn, dim);
}
// y += P x on free dofs (x already interpolated)
template <typename T>
__global__ void add_masked_kernel(T* y, const T* x, const uint8_t* mask, long long nn, int dim) {
  const long long n = (long long)(dim + 1) * nn;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const long long comp = udiv(i, nn);
    const uint8_t m = mask[i - comp * nn];
    const bool f = comp < dim ? (m & kMaskU) : (m & kMaskPhi);
    if (!f) y[i] += x[i];
  }
}
template <typename T>
void k_add_masked(T* y, const T* x, const uint8_t* mask, long long nn, int dim, hipStream_t s) {
  long long nb = ((dim + 1) * nn + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(add_masked_kernel<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, y, x, mask, nn, dim);
}

template void k_axis_apply<double>(double*, const double*, const Sparse1D&, int, int, const long long*, int, const uint8_t*,
                                   const uint8_t*, hipStream_t, bool, ChebStart<double>);
template void k_axis_apply<float>(float*, const float*, const Sparse1D&, int, int, const long long*, int, const uint8_t*,
                                  const uint8_t*, hipStream_t, bool, ChebStart<float>);
template void k_prolong<double>(double*, const double*, const Sparse1D&, const uint8_t*, const uint8_t*, const Geom&,
                                const Geom&, bool, hipStream_t);
template void k_prolong<float>(float*, const float*, const Sparse1D&, const uint8_t*, const uint8_t*, const Geom&, const Geom&,
                               bool, hipStream_t);
template void k_mask_comp<double>(double*, const uint8_t*, long long, int, hipStream_t);
template void k_mask_comp<float>(float*, const uint8_t*, long long, int, hipStream_t);
template void k_add_masked<double>(double*, const double*, const uint8_t*, long long, int, hipStream_t);
template void k_add_masked<float>(float*, const float*, const uint8_t*, long long, int, hipStream_t);

}  // namespace mfpff

MFPFF_BOUNDS_READER(bounds_hits_transfer)
