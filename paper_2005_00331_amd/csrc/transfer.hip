// Level transfers (gfx950).  The prolongation between nested structured
// levels is the Kronecker product over axes of one 1D interpolation matrix
// (coarse basis functions evaluated at fine nodes), applied per component;
// restriction is its transpose.  Both can be applied axis by axis: each pass
// maps one axis through a padded row-sparse 1D matrix (thread per output
// entry, gather, no atomics), so a 3D transfer reads each input a few times
// instead of (k+1)^3 times; the masks are fused into the first and last pass.
// In 2D the prolongation is one gather pass (prolong_kernel), which saves a
// launch on the small levels.
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
                                  const uint8_t* out_mask, int add) {
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
        const long long ii = base + (long long)ci * sin[axis];
        if (in_mask && comp_fixed(in_mask, ii - comp * per_in, comp, dim)) continue;
        acc += w * in[ii];
      }
    }
    if (!add) out[idx] = acc;
    else if (!ofix) out[idx] += acc;
  }
}

template <typename T>
void k_axis_apply(T* out, const T* in, const Sparse1D& A, int axis, int dim, const long long* dims_in, int ncomp,
                  const uint8_t* in_mask, const uint8_t* out_mask, hipStream_t s, bool add) {
  Dims3 d{{dims_in[0], dims_in[1], dim == 3 ? dims_in[2] : 1}};
  long long total = ncomp;
  for (int a = 0; a < dim; ++a) total *= (a == axis ? A.n_out : d.n[a]);
  long long nb = (total + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(axis_apply_kernel<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, out, in, A.col, A.val, A.valf, A.width,
                     axis, dim, d, A.n_out, ncomp, in_mask, out_mask, add ? 1 : 0);
}

// out = / += P~ xc on the fine level: gather of (kc+1)^d coarse values per fine node
template <typename T>
__global__ void prolong_kernel(T* out, const T* xc, const int* col, const double* val, const float* valf, int width,
                               const uint8_t* mask_c, const uint8_t* mask_f, Geom gf, Geom gc, int add) {
  const long long nnf = gf.n_nodes, nnc = gc.n_nodes;
  const int dim = gf.dim;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nnf; i += (long long)gridDim.x * blockDim.x) {
    int f[3] = {0, 0, 0};
    unsigned rem = (unsigned)i;
    for (int a = 0; a < dim; ++a) {
      const unsigned q = rem / (unsigned)gf.M;
      f[a] = (int)(rem - q * (unsigned)gf.M);
      rem = q;
    }
    T v[4] = {T(0), T(0), T(0), T(0)};
    const int w2 = dim == 3 ? width : 1;
    for (int j2 = 0; j2 < w2; ++j2) {
      int c2 = 0;
      T wz = T(1);
      if (dim == 3) {
        c2 = col[f[2] * width + j2];
        if (c2 < 0) break;
        wz = sizeof(T) == 8 ? (T)val[f[2] * width + j2] : (T)valf[f[2] * width + j2];
      }
      for (int j1 = 0; j1 < width; ++j1) {
        const int c1 = col[f[1] * width + j1];
        if (c1 < 0) break;
        const T wy = wz * (sizeof(T) == 8 ? (T)val[f[1] * width + j1] : (T)valf[f[1] * width + j1]);
        for (int j0 = 0; j0 < width; ++j0) {
          const int c0 = col[f[0] * width + j0];
          if (c0 < 0) break;
          const T w = wy * (sizeof(T) == 8 ? (T)val[f[0] * width + j0] : (T)valf[f[0] * width + j0]);
          const long long nc = c0 + (long long)gc.M * (c1 + (long long)gc.M * c2);
          const uint8_t mc = mask_c[nc];
          for (int cc = 0; cc <= dim; ++cc) {
            const bool fx = cc < dim ? (mc & kMaskU) : (mc & kMaskPhi);
            if (!fx) v[cc] += w * xc[cc * nnc + nc];
          }
        }
      }
    }
    const uint8_t mf = mask_f[i];
    for (int cc = 0; cc <= dim; ++cc) {
      const bool fx = cc < dim ? (mf & kMaskU) : (mf & kMaskPhi);
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
  hipLaunchKernelGGL(prolong_kernel<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, out, xc, P.col, P.val, P.valf, P.width,
                     mask_c, mask_f, gf, gc, add ? 1 : 0);
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
                                   const uint8_t*, hipStream_t, bool);
template void k_axis_apply<float>(float*, const float*, const Sparse1D&, int, int, const long long*, int, const uint8_t*,
                                  const uint8_t*, hipStream_t, bool);
template void k_prolong<double>(double*, const double*, const Sparse1D&, const uint8_t*, const uint8_t*, const Geom&,
                                const Geom&, bool, hipStream_t);
template void k_prolong<float>(float*, const float*, const Sparse1D&, const uint8_t*, const uint8_t*, const Geom&, const Geom&,
                               bool, hipStream_t);
template void k_mask_comp<double>(double*, const uint8_t*, long long, int, hipStream_t);
template void k_mask_comp<float>(float*, const uint8_t*, long long, int, hipStream_t);
template void k_add_masked<double>(double*, const double*, const uint8_t*, long long, int, hipStream_t);
template void k_add_masked<float>(float*, const float*, const uint8_t*, long long, int, hipStream_t);

}  // namespace mfpff
