// Vector, reduction and small bookkeeping kernels (gfx950).
// Element-wise kernels are grid-stride loops over contiguous vectors; reductions
// write one partial per workgroup and a single workgroup finishes them in a
// fixed order, so repeated runs are bitwise identical.
#include <type_traits>

#include "bounds.h"
#include "internal.h"

namespace mfpff {

static inline unsigned grid_for(long long n, int per = kThreads) {
  long long b = (n + per - 1) / per;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

#define GSTRIDE(i, n) for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

__device__ __forceinline__ bool fixed_at(const uint8_t* mask, long long i, long long nn, int dim) {
  if (!mask) return false;
  const long long comp = udiv(i, nn);
  const uint8_t m = mask[i - comp * nn];
  return comp < dim ? (m & kMaskU) : (m & kMaskPhi);
}

// y = b + scale * (I - P) x   (b may be null)
template <typename T>
__global__ void mask_init_kernel(T* y, const T* b, const T* x, const uint8_t* mask, long long nn, int dim, T scale) {
  const long long n = (long long)(dim + 1) * nn;
  GSTRIDE(i, n) {
    T v = b ? b[i] : T(0);
    if (fixed_at(mask, i, nn, dim)) v += scale * x[i];
    y[i] = v;
  }
}
template <typename T>
void k_mask_init(T* y, const T* b, const T* x, const uint8_t* mask, long long nn, int dim, T scale, hipStream_t s) {
  hipLaunchKernelGGL(mask_init_kernel<T>, dim3(grid_for((dim + 1) * nn)), dim3(kThreads), 0, s, y, b, x, mask, nn, dim, scale);
}

template <typename T>
__global__ void copy_kernel(T* y, const T* x, long long n) { GSTRIDE(i, n) y[i] = x[i]; }
template <typename T>
void k_copy(T* y, const T* x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, y, x, n);
}
template <typename T>
__global__ void fill_kernel(T* y, T v, long long n) { GSTRIDE(i, n) y[i] = v; }
template <typename T>
void k_fill(T* y, T v, long long n, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, y, v, n);
}
template <typename T>
__global__ void axpy_kernel(T* y, T a, const T* x, long long n) { GSTRIDE(i, n) y[i] += a * x[i]; }
template <typename T>
void k_axpy(T* y, T a, const T* x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, y, a, x, n);
}

// dinv = 1/diag on free dofs, 1 on fixed dofs; optional FP64 copy of the diagonal itself
template <typename T>
__global__ void diag_finish_kernel(T* dinv, double* dout, const T* diag, const uint8_t* mask, long long nn, int dim) {
  const long long n = (long long)(dim + 1) * nn;
  GSTRIDE(i, n) {
    const bool f = fixed_at(mask, i, nn, dim);
    const T dv = f ? T(1) : diag[i];
    if (dinv) dinv[i] = T(1) / dv;
    if (dout) dout[i] = (double)dv;
  }
}
template <typename T>
void k_diag_finish(T* dinv, double* dout, const T* diag, const uint8_t* mask, long long nn, int dim, hipStream_t s) {
  hipLaunchKernelGGL(diag_finish_kernel<T>, dim3(grid_for((dim + 1) * nn)), dim3(kThreads), 0, s, dinv, dout, diag, mask, nn, dim);
}

// Chebyshev start: z = D^-1 r / theta_b, d = z
template <typename T>
__global__ void cheb_init_kernel(T* z, T* d, const T* r, const T* dinv, long long nn, int dim, T itu, T itp) {
  const long long n = (long long)(dim + 1) * nn;
  const long long nu = (long long)dim * nn;
  GSTRIDE(i, n) {
    const T v = dinv[i] * r[i] * (i < nu ? itu : itp);
    z[i] = v;
    d[i] = v;
  }
}
template <typename T>
void k_cheb_init(T* z, T* d, const T* r, const T* dinv, long long nn, int dim, T itu, T itp, hipStream_t s) {
  hipLaunchKernelGGL(cheb_init_kernel<T>, dim3(grid_for((dim + 1) * nn)), dim3(kThreads), 0, s, z, d, r, dinv, nn, dim, itu, itp);
}
// Chebyshev step: d = c1 d + c2 D^-1 (r - t); z += d
template <typename T>
__global__ void cheb_step_kernel(T* z, T* d, const T* r, const T* t, const T* dinv, long long nn, int dim,
                                 T c1u, T c2u, T c1p, T c2p) {
  const long long n = (long long)(dim + 1) * nn;
  const long long nu = (long long)dim * nn;
  GSTRIDE(i, n) {
    const bool isu = i < nu;
    const T dn = (isu ? c1u : c1p) * d[i] + (isu ? c2u : c2p) * dinv[i] * (r[i] - t[i]);
    d[i] = dn;
    z[i] += dn;
  }
}
template <typename T>
void k_cheb_step(T* z, T* d, const T* r, const T* t, const T* dinv, long long nn, int dim, T c1u, T c2u, T c1p, T c2p,
                 hipStream_t s) {
  hipLaunchKernelGGL(cheb_step_kernel<T>, dim3(grid_for((dim + 1) * nn)), dim3(kThreads), 0, s, z, d, r, t, dinv, nn, dim,
                     c1u, c2u, c1p, c2p);
}

// one Chebyshev step after t = A_blk z: d = c1 d + c2 D^-1 (r - t); z' = z + d; optional x' = x + z'
template <typename T>
__global__ void cheb_update_kernel(T* zout, T* d, const T* zin, const T* r, const T* t, const T* dinv, long long nn, int dim,
                                   T c1u, T c2u, T c1p, T c2p, const T* xacc, T* xout) {
  const long long n = (long long)(dim + 1) * nn;
  const long long nu = (long long)dim * nn;
  GSTRIDE(i, n) {
    const bool isu = i < nu;
    const T dn = (isu ? c1u : c1p) * d[i] + (isu ? c2u : c2p) * dinv[i] * (r[i] - t[i]);
    d[i] = dn;
    const T zn = zin[i] + dn;
    zout[i] = zn;
    if (xout) xout[i] = xacc[i] + zn;
  }
}
template <typename T>
void k_cheb_update(T* zout, T* d, const T* zin, const T* r, const T* t, const T* dinv, long long nn, int dim, T c1u, T c2u,
                   T c1p, T c2p, const T* xacc, T* xout, hipStream_t s) {
  hipLaunchKernelGGL(cheb_update_kernel<T>, dim3(grid_for((dim + 1) * nn)), dim3(kThreads), 0, s, zout, d, zin, r, t, dinv, nn,
                     dim, c1u, c2u, c1p, c2p, xacc, xout);
}

__global__ void d2f_kernel(float* y, const double* x, long long n) { GSTRIDE(i, n) y[i] = (float)x[i]; }
__global__ void f2d_kernel(double* y, const float* x, long long n) { GSTRIDE(i, n) y[i] = (double)x[i]; }
void k_cast_d2f(float* y, const double* x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(d2f_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, y, x, n);
}
void k_cast_f2d(double* y, const float* x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(f2d_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, y, x, n);
}

// y = scale * P y (zero fixed dofs, scale the rest)
__global__ void mask_vec_kernel(double* y, const uint8_t* mask, long long nn, int dim, double scale) {
  const long long n = (long long)(dim + 1) * nn;
  GSTRIDE(i, n) y[i] = fixed_at(mask, i, nn, dim) ? 0.0 : scale * y[i];
}
void k_mask_vec(double* y, const uint8_t* mask, long long nn, int dim, double scale, hipStream_t s) {
  hipLaunchKernelGGL(mask_vec_kernel, dim3(grid_for((dim + 1) * nn)), dim3(kThreads), 0, s, y, mask, nn, dim, scale);
}

__device__ __forceinline__ uint8_t dirichlet_bit(long long node, const Geom& g, int dirichlet) {
  if (!dirichlet || node >= g.n_grid) return 0;  // slit duplicates lie on the mid-plane
  long long stride = 1;
  for (int a = 0; a < g.dim - 1; ++a) stride *= g.M;
  const long long i = (node / stride) % g.M;
  return (i == 0 || i == g.M - 1) ? kMaskU : (uint8_t)0;
}

// Finest level: pack u, phi, phi~ into the level field array and build the mask.
__global__ void fine_fields_kernel(double* lin, uint8_t* mask, const double* u, const double* phi, const double* phit,
                                   const uint8_t* active, Geom g, int dirichlet) {
  const long long nn = g.n_nodes;
  GSTRIDE(i, nn) {
    for (int c = 0; c < g.dim; ++c) lin[c * nn + i] = u[c * nn + i];
    lin[g.dim * nn + i] = phi[i];
    lin[(g.dim + 1) * nn + i] = phit[i];
    mask[i] = (uint8_t)((active && active[i]) ? kMaskPhi : 0) | dirichlet_bit(i, g, dirichlet);
  }
}
void k_fine_fields(double* lin, uint8_t* mask, const double* u, const double* phi, const double* phit, const uint8_t* active,
                   const Geom& g, int dirichlet, hipStream_t s) {
  hipLaunchKernelGGL(fine_fields_kernel, dim3(grid_for(g.n_nodes)), dim3(kThreads), 0, s, lin, mask, u, phi, phit, active, g,
                     dirichlet);
}

// Coarse level: inject fields and the active bit from the coincident fine node.
__global__ void inject_kernel(double* lin_c, uint8_t* mask_c, const double* lin_f, const uint8_t* mask_f, Geom gc, Geom gf,
                              int dirichlet) {
  const long long nnc = gc.n_nodes, nnf = gf.n_nodes;
  const long long ratio = ((long long)gf.k * gf.N) / ((long long)gc.k * gc.N);
  GSTRIDE(i, nnc) {
    long long rem = i, fi = 0, fs = 1;
    for (int a = 0; a < gc.dim; ++a) {
      const long long ia = rem % gc.M;
      rem /= gc.M;
      fi += ia * ratio * fs;
      fs *= gf.M;
    }
    if (gc.slit && i >= gc.n_grid) {
      // a coarse duplicate (slit node, side above the slit) takes the fine duplicate at its
      // position: duplicates are numbered along the first axis, then the second (3D)
      const long long sx_c = (long long)gc.k * gc.N / 2, sx_f = (long long)gf.k * gf.N / 2;
      const long long j = i - gc.n_grid, i0 = j % sx_c, i1 = j / sx_c;
      fi = gf.n_grid + i0 * ratio + (gc.dim == 3 ? sx_f * (i1 * ratio) : 0);
    }
    fi = MFPFF_IN(fi, nnf);
    for (int c = 0; c < gc.dim + 2; ++c) lin_c[c * nnc + i] = lin_f[c * nnf + fi];
    mask_c[i] = (uint8_t)(mask_f[fi] & kMaskPhi) | dirichlet_bit(i, gc, dirichlet);
  }
}
void k_inject(double* lin_c, uint8_t* mask_c, const double* lin_f, const uint8_t* mask_f, const Geom& gc, const Geom& gf,
              int dirichlet, hipStream_t s) {
  hipLaunchKernelGGL(inject_kernel, dim3(grid_for(gc.n_nodes)), dim3(kThreads), 0, s, lin_c, mask_c, lin_f, mask_f, gc, gf,
                     dirichlet);
}

// Row-sum-lumped phi mass: product over axes of h * (sum of the 1D basis
// integrals of the cells that share the node).
// On a slit mesh a slit-plane node below x = 1/2 has only the cells below it (local index k along
// the last axis), its duplicate only those above it (local index 0).
__global__ void lumped_mass_kernel(double* ml, Geom g, const double* w1d) {
  const long long ns = (long long)g.k * g.N / 2;  // slit nodes per line along the first axis
  GSTRIDE(i, g.n_nodes) {
    long long gi = i;
    int side = 0;  // 1: grid node on the slit (lower side), 2: duplicate (upper side)
    if (g.slit) {
      if (i >= g.n_grid) {
        const long long j = i - g.n_grid;
        gi = (j % ns) + (g.dim == 3 ? (long long)g.M * (j / ns) : 0) + (g.n_grid / g.M) * (g.M / 2);
        side = 2;
      } else if ((i / (g.n_grid / g.M)) == g.M / 2 && (i % g.M) < ns) {
        side = 1;
      }
    }
    long long rem = gi;
    double v = 1.0;
    for (int a = 0; a < g.dim; ++a) {
      const long long ia = rem % g.M;
      rem /= g.M;
      const int loc = (int)(ia % g.k);
      double wa;
      if (a == g.dim - 1 && side != 0) wa = side == 1 ? w1d[g.k] : w1d[0];
      else if (loc == 0) wa = (ia > 0 ? w1d[g.k] : 0.0) + (ia < g.M - 1 ? w1d[0] : 0.0);
      else wa = w1d[loc];
      v *= g.h * wa;
    }
    ml[i] = v;
  }
}

// Slit levels: the epilogue of a product accumulated by the cell kernel's scatter into y
// (y = P G P x, or -P G P x for a residual): identity at fixed rows, y = b + y for a residual.
template <typename T>
__global__ void slit_epilogue_kernel(T* y, const T* x, const T* b, const uint8_t* mask, long long nn, int dim) {
  const long long n = (long long)(dim + 1) * nn;
  GSTRIDE(i, n) {
    const long long node = i % nn;
    const int cc = (int)(i / nn);
    const uint8_t m = mask ? mask[node] : (uint8_t)0;
    const bool fixed = cc < dim ? (m & kMaskU) : (m & kMaskPhi);
    const T gx = fixed ? (b ? -x[i] : x[i]) : y[i];
    y[i] = b ? b[i] + gx : gx;
  }
}
template <typename T>
void k_slit_epilogue(T* y, const T* x, const T* b, const uint8_t* mask, long long nn, int dim, hipStream_t s) {
  hipLaunchKernelGGL(slit_epilogue_kernel<T>, dim3(grid_for((long long)(dim + 1) * nn)), dim3(kThreads), 0, s, y, x, b, mask,
                     nn, dim);
}
template void k_slit_epilogue<double>(double*, const double*, const double*, const uint8_t*, long long, int, hipStream_t);
template void k_slit_epilogue<float>(float*, const float*, const float*, const uint8_t*, long long, int, hipStream_t);
void k_lumped_mass(double* ml, const Geom& g, const double* w1d, hipStream_t s) {
  hipLaunchKernelGGL(lumped_mass_kernel, dim3(grid_for(g.n_nodes)), dim3(kThreads), 0, s, ml, g, w1d);
}

// Transfer between a slit level and the next coarser one by a CSR matrix per component (rows:
// output nodes): out = M_out A M_in in, i.e. fixed outputs are 0 (left unchanged with add) and
// fixed inputs are skipped; the prolongation and its transpose, the restriction, both use it
template <typename T>
__global__ void csr_transfer_kernel(T* out, const T* in, CsrDev A, const uint8_t* mask_in, const uint8_t* mask_out,
                                    long long n_out, long long n_in, int dim, int add) {
  const long long n = (long long)(dim + 1) * n_out;
  GSTRIDE(i, n) {
    const int cc = (int)(i / n_out);
    const long long node = i - (long long)cc * n_out;
    const bool ofix = mask_out && fixed_at(mask_out, i, n_out, dim);
    T acc = 0;
    if (!ofix) {
      for (int e = A.rowptr[node]; e < A.rowptr[node + 1]; ++e) {
        const long long j = (long long)cc * n_in + MFPFF_IN(A.col[e], n_in);
        if (mask_in && fixed_at(mask_in, j, n_in, dim)) continue;
        acc += (sizeof(T) == 8 ? (T)A.val[e] : (T)A.valf[e]) * in[j];
      }
    }
    if (add) {
      if (!ofix) out[i] += acc;
    } else {
      out[i] = ofix ? T(0) : acc;
    }
  }
}
template <typename T>
void k_csr_transfer(T* out, const T* in, const CsrDev& A, const uint8_t* mask_in, const uint8_t* mask_out, long long n_out,
                    long long n_in, int dim, bool add, hipStream_t s) {
  hipLaunchKernelGGL(csr_transfer_kernel<T>, dim3(grid_for((long long)(dim + 1) * n_out)), dim3(kThreads), 0, s, out, in, A,
                     mask_in, mask_out, n_out, n_in, dim, add ? 1 : 0);
}
template void k_csr_transfer<double>(double*, const double*, const CsrDev&, const uint8_t*, const uint8_t*, long long,
                                     long long, int, bool, hipStream_t);
template void k_csr_transfer<float>(float*, const float*, const CsrDev&, const uint8_t*, const uint8_t*, long long,
                                    long long, int, bool, hipStream_t);

// Algorithm 1 active set: -(M_L^-1 R_phi)_i + c (phi - phi_old)_i > 0
__global__ void active_set_kernel(uint8_t* act, const double* R, const double* phi, const double* phi_old, const double* ml,
                                  long long nn, int dim, double c) {
  GSTRIDE(i, nn) {
    const double ind = -R[(long long)dim * nn + i] / ml[i] + c * (phi[i] - phi_old[i]);
    act[i] = ind > 0.0 ? 1 : 0;
  }
}
void k_active_set(uint8_t* act, const double* R, const double* phi, const double* phi_old, const double* ml, long long nn,
                  int dim, double c, hipStream_t s) {
  hipLaunchKernelGGL(active_set_kernel, dim3(grid_for(nn)), dim3(kThreads), 0, s, act, R, phi, phi_old, ml, nn, dim, c);
}

// Stopping test of Algorithm 1, one pass: per workgroup, the sum of R_i^2 over the free dofs
// (u-dofs off the Dirichlet faces, phi-dofs outside the active set act) and the number of
// nodes where act differs from prev.  part: 2 doubles per workgroup (sum, count).
__global__ void pdas_check_kernel(double* part, const double* R, const uint8_t* act, const uint8_t* prev, Geom g,
                                  int dirichlet) {
  __shared__ double sh[2][kThreads / 64];
  const long long nn = g.n_nodes;
  const int dim = g.dim;
  const unsigned M = (unsigned)g.M;
  double ss = 0, nd = 0;
  GSTRIDE(i, nn) {
    // index of the node along the last axis (the Dirichlet faces are normal to it)
    const unsigned q = (unsigned)i / M;
    const unsigned last = dim == 2 ? q : q / M;
    const bool dir = dirichlet && i < g.n_grid && (last == 0 || last == M - 1);
    const bool a = act[i] != 0;
    if (!dir) {
      for (int cc = 0; cc < dim; ++cc) {
        const double r = R[cc * nn + i];
        ss += r * r;
      }
    }
    if (!a) {
      const double r = R[dim * nn + i];
      ss += r * r;
    }
    nd += (prev[i] != 0) != a ? 1.0 : 0.0;
  }
  for (int off = 32; off > 0; off >>= 1) {
    ss += __shfl_down(ss, off, 64);
    nd += __shfl_down(nd, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wid] = ss;
    sh[1][wid] = nd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
      a += sh[0][w];
      b += sh[1][w];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}
int pdas_check_blocks(long long nn) {
  const long long b = (nn + kThreads - 1) / kThreads;
  return (int)(b < 256 ? (b < 1 ? 1 : b) : 256);
}
void k_pdas_check(double* part, const double* R, const uint8_t* act, const uint8_t* prev, const Geom& g, int dirichlet,
                  hipStream_t s) {
  hipLaunchKernelGGL(pdas_check_kernel, dim3((unsigned)pdas_check_blocks(g.n_nodes)), dim3(kThreads), 0, s, part, R, act,
                     prev, g, dirichlet);
}

// primal-dual active-set update: the iterate is put on the obstacle on the active set,
// phi_i := phi_old_i where act_i != 0
__global__ void project_active_kernel(double* phi, const double* phi_old, const uint8_t* act, long long n) {
  GSTRIDE(i, n) if (act[i]) phi[i] = phi_old[i];
}
void k_project_active(double* phi, const double* phi_old, const uint8_t* act, long long n, hipStream_t s) {
  hipLaunchKernelGGL(project_active_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, phi, phi_old, act, n);
}

// Load stepping (Section 5): every displacement component is 0 on the bottom face and
// t du on the top face (the two faces normal to the last axis); thread i < n_face covers
// bottom node i, thread n_face + i top node i.
__global__ void impose_faces_kernel(double* u, Geom g, double t0, double t1, double t2) {
  const long long nf = g.dim == 2 ? (long long)g.M : (long long)g.M * g.M;
  const long long top_off = (long long)(g.M - 1) * nf;
  GSTRIDE(i, 2 * nf) {
    const bool top = i >= nf;
    const long long node = MFPFF_IN(top ? i - nf + top_off : i, g.n_nodes);
    u[node] = top ? t0 : 0.0;
    u[g.n_nodes + node] = top ? t1 : 0.0;
    if (g.dim == 3) u[2 * g.n_nodes + node] = top ? t2 : 0.0;
  }
}
void k_impose_faces(double* u, const Geom& g, const double* top, hipStream_t s) {
  const long long nf = g.dim == 2 ? (long long)g.M : (long long)g.M * g.M;
  hipLaunchKernelGGL(impose_faces_kernel, dim3(grid_for(2 * nf)), dim3(kThreads), 0, s, u, g, top[0], top[1],
                     g.dim == 3 ? top[2] : 0.0);
}

// phi~ = 2 phi_{n-1} - phi_{n-2}: linear extrapolation over two equal steps (Section 3)
__global__ void extrapolate_kernel(double* pt, const double* p1, const double* p2, long long n) {
  GSTRIDE(i, n) pt[i] = 2.0 * p1[i] - p2[i];
}
void k_extrapolate(double* pt, const double* p1, const double* p2, long long n, hipStream_t s) {
  hipLaunchKernelGGL(extrapolate_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, pt, p1, p2, n);
}

// reaction on a face: out[f * dim + c] = sum over the nodes of face f (0 bottom, 1 top) of the
// displacement residual row of component c; one workgroup per (face, component), fixed order
__global__ void face_reaction_kernel(double* out, const double* R, Geom g) {
  __shared__ double sh[kThreads / 64];
  const int f = blockIdx.x / g.dim, c = blockIdx.x % g.dim;
  const long long nf = g.dim == 2 ? (long long)g.M : (long long)g.M * g.M;
  const double* r = R + c * g.n_nodes + (f ? (long long)(g.M - 1) * nf : 0);
  double s = 0;
  (void)MFPFF_IN((f ? (long long)(g.M - 1) * nf : 0) + nf - 1, g.n_nodes);  // the face's last node
  for (long long i = threadIdx.x; i < nf; i += blockDim.x) s += r[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0;
    for (int w = 0; w < kThreads / 64; ++w) a += sh[w];
    out[blockIdx.x] = a;
  }
}
void k_face_reaction(double* out, const double* R, const Geom& g, hipStream_t s) {
  hipLaunchKernelGGL(face_reaction_kernel, dim3(2 * g.dim), dim3(kThreads), 0, s, out, R, g);
}

// SplitMix64 (Steele, Lea, Flood 2014): output n of stream st with seed s is
// mix(s + (n + 1 + st * 2^40) * 0x9E3779B97F4A7C15), mapped to [-1, 1).
__device__ __forceinline__ double splitmix_pm1(unsigned long long seed, unsigned long long st, unsigned long long n) {
  unsigned long long z = seed + (n + 1ULL + (st << 40)) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}
__global__ void splitmix_start_kernel(double* v, const uint8_t* mask, long long nn, int dim, unsigned long long seed, int su,
                                      int sp) {
  const long long n = (long long)(dim + 1) * nn;
  const long long nu = (long long)dim * nn;
  GSTRIDE(i, n) {
    const double r = i < nu ? splitmix_pm1(seed, (unsigned long long)su, (unsigned long long)i)
                            : splitmix_pm1(seed, (unsigned long long)sp, (unsigned long long)(i - nu));
    v[i] = fixed_at(mask, i, nn, dim) ? 0.0 : r;
  }
}
void k_splitmix_start(double* v, const uint8_t* mask, long long nn, int dim, unsigned long long seed, int su, int sp,
                      hipStream_t s) {
  hipLaunchKernelGGL(splitmix_start_kernel, dim3(grid_for((dim + 1) * nn)), dim3(kThreads), 0, s, v, mask, nn, dim, seed, su,
                     sp);
}

// ---------------------------------------------------------------- reductions
constexpr int kRedBlocks = 512;
int dot_blocks(long long n) {
  long long b = (n + kThreads - 1) / kThreads;
  return (int)(b < kRedBlocks ? (b < 1 ? 1 : b) : kRedBlocks);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  // wave64 shuffle reduction then across the 4 waves
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();
  return r;
}

// part[b * nvec + j] = sum over this block's range of V_j . w
__global__ void multidot_partials_kernel(double* part, const double* V, long long ldv, int nvec, const double* w, long long n) {
  __shared__ double sh[8];
  const int nb = gridDim.x;
  const long long chunk = (n + nb - 1) / nb;
  const long long lo = (long long)blockIdx.x * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  for (int j = 0; j < nvec; ++j) {
    double acc = 0;
    const double* v = V + (long long)j * ldv;
    for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) acc += v[i] * w[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * nvec + j] = s;
  }
}
void k_multidot_partials(double* part, const double* V, long long ldv, int nvec, const double* w, long long n, hipStream_t s) {
  hipLaunchKernelGGL(multidot_partials_kernel, dim3(dot_blocks(n)), dim3(kThreads), 0, s, part, V, ldv, nvec, w, n);
}
__global__ void multidot_finish_kernel(double* out, const double* part, int nblocks, int nvec) {
  __shared__ double sh[8];
  for (int j = 0; j < nvec; ++j) {
    double acc = 0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) acc += part[(long long)b * nvec + j];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[j] = s;
  }
}
void k_multidot_finish(double* out, const double* part, int nblocks, int nvec, hipStream_t s) {
  hipLaunchKernelGGL(multidot_finish_kernel, dim3(1), dim3(kThreads), 0, s, out, part, nblocks, nvec);
}

// two segment sums of a.b: [0, nu) and [nu, n)
__global__ void seg_dot_partials_kernel(double* part, const double* a, const double* b, long long nu, long long n) {
  __shared__ double sh[8];
  const int nb = gridDim.x;
  for (int sgm = 0; sgm < 2; ++sgm) {
    const long long s0 = sgm == 0 ? 0 : nu, s1 = sgm == 0 ? nu : n;
    const long long len = s1 - s0;
    const long long chunk = (len + nb - 1) / nb;
    const long long lo = s0 + (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < s1 ? lo + chunk : s1;
    double acc = 0;
    for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) acc += a[i] * b[i];
    const double sum = block_sum(acc, sh);
    if (threadIdx.x == 0) part[2 * blockIdx.x + sgm] = sum;
  }
}
void k_seg_dot_partials(double* part, const double* a, const double* b, long long nu, long long n, hipStream_t s) {
  hipLaunchKernelGGL(seg_dot_partials_kernel, dim3(dot_blocks(n)), dim3(kThreads), 0, s, part, a, b, nu, n);
}

// w += sign * sum_j coef[j] V_j  (coefficients read from device memory)
__global__ void maxpy_dev_kernel(double* w, const double* V, long long ldv, int nvec, const double* coef, double sign, long long n) {
  GSTRIDE(i, n) {
    double acc = 0;
    for (int j = 0; j < nvec; ++j) acc += coef[j] * V[(long long)j * ldv + i];
    w[i] += sign * acc;
  }
}
void k_maxpy_dev(double* w, const double* V, long long ldv, int nvec, const double* coef, double sign, long long n, hipStream_t s) {
  hipLaunchKernelGGL(maxpy_dev_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, w, V, ldv, nvec, coef, sign, n);
}
// ---------------------------------------------------------------- Arnoldi passes
// One pass over the Krylov basis V (nvec <= kOrthMax vectors) and the new
// vector w; every workgroup writes its partial sums, and orth_finish_kernel
// adds them in block order (a device-wide fence inside the pass would write
// back the whole L2 of every XCD once per workgroup).
//   ORTH_DOTS:        part -> V_j . w
//   ORTH_UPDATE_DOTS: w <- w - V c;  part -> V_j . w        (c on the device)
//   ORTH_UPDATE_NORM: w <- w - V c;  part -> w . w
//   ORTH_UPDATE_DOTS_NORM: w <- w - V c;  part -> V_j . w, then w . w (nvec + 1 sums)
enum OrthMode : int { ORTH_DOTS = 0, ORTH_UPDATE_DOTS = 1, ORTH_UPDATE_NORM = 2, ORTH_UPDATE_DOTS_NORM = 3 };

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int MODE, int NV>
__global__ __launch_bounds__(kThreads) void orth_pass_kernel(double* __restrict__ w, const double* __restrict__ V,
                                                             long long ldv, const double* __restrict__ coef,
                                                             double* __restrict__ part, long long n) {
  constexpr int NA = MODE == ORTH_UPDATE_NORM ? 1 : (MODE == ORTH_UPDATE_DOTS_NORM ? NV + 1 : NV);  // sums per thread
  constexpr int NW = kThreads / 64;
  __shared__ double sh[NW][NA];
  double c[NV];
  if (MODE != ORTH_DOTS) {
#pragma unroll
    for (int j = 0; j < NV; ++j) c[j] = coef[j];
  }
  double acc[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) acc[j] = 0.0;
  // one element (the scalar tail of an odd n) or two consecutive ones per step; the basis stride
  // ldv is even and every vector 16-byte aligned, so a pair is one 16-byte load per vector
  auto step = [&](long long i, auto tag) {
    constexpr int W = decltype(tag)::value;
    using V2 = typename std::conditional<W == 2, double2, double>::type;
    V2 v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = *reinterpret_cast<const V2*>(V + (long long)j * ldv + i);
    V2 wi = *reinterpret_cast<const V2*>(w + i);
    // keep every load of the step in flight before the arithmetic (the register allocator
    // would otherwise interleave them to save registers)
    __builtin_amdgcn_sched_barrier(0);
    double* wl = reinterpret_cast<double*>(&wi);
#pragma unroll
    for (int e = 0; e < W; ++e) {
      if (MODE != ORTH_DOTS) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < NV; ++j) t += c[j] * reinterpret_cast<const double*>(&v[j])[e];
        wl[e] -= t;
      }
      if (MODE == ORTH_UPDATE_NORM) {
        acc[0] += wl[e] * wl[e];
      } else {
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] += reinterpret_cast<const double*>(&v[j])[e] * wl[e];
        if (MODE == ORTH_UPDATE_DOTS_NORM) acc[NV] += wl[e] * wl[e];
      }
    }
    if (MODE != ORTH_DOTS) *reinterpret_cast<V2*>(w + i) = wi;
  };
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long long p = gid; 2 * p + 1 < n; p += stride) step(2 * p, std::integral_constant<int, 2>());
  if ((n & 1) && gid == 0) step(n - 1, std::integral_constant<int, 1>());
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const double r = wave_sum(acc[j]);
    if (lane == 0) sh[wid][j] = r;
  }
  __syncthreads();
  if (threadIdx.x < NA) {
    double r = 0.0;
    for (int q = 0; q < NW; ++q) r += sh[q][threadIdx.x];
    part[(long long)blockIdx.x * NA + threadIdx.x] = r;
  }
}

// out[j] = sum over blocks b (in order per lane, then a fixed tree) of part[b * nout + j]; one wave per j
constexpr int kFinishThreads = 1024;
__global__ __launch_bounds__(kFinishThreads) void orth_finish_kernel(double* __restrict__ out, const double* __restrict__ part,
                                                                     int nb, int nout) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j = wid; j < nout; j += kFinishThreads / 64) {
    double r = 0.0;
    for (int b = lane; b < nb; b += 64) r += part[(long long)b * nout + j];
    r = wave_sum(r);
    if (lane == 0) out[j] = r;
  }
}

int orth_blocks(long long n) { return dot_blocks(n); }

// one instantiation per basis size, so that every load and accumulator is unconditional
template <int MODE, int NV>
static void launch_orth(int nvec, double* w, const double* V, long long ldv, const double* coef, double* part,
                        long long n, hipStream_t s) {
  if constexpr (NV <= kOrthMax) {
    if (nvec == NV) {
      hipLaunchKernelGGL((orth_pass_kernel<MODE, NV>), dim3(orth_blocks(n)), dim3(kThreads), 0, s, w, V, ldv, coef, part, n);
      return;
    }
    launch_orth<MODE, NV + 1>(nvec, w, V, ldv, coef, part, n, s);
  }
}

void k_orth_pass(int mode, double* w, const double* V, long long ldv, int nvec, const double* coef, double* part,
                 double* out, long long n, hipStream_t s) {
  if (mode == ORTH_DOTS)
    launch_orth<ORTH_DOTS, 1>(nvec, w, V, ldv, coef, part, n, s);
  else if (mode == ORTH_UPDATE_DOTS)
    launch_orth<ORTH_UPDATE_DOTS, 1>(nvec, w, V, ldv, coef, part, n, s);
  else if (mode == ORTH_UPDATE_NORM)
    launch_orth<ORTH_UPDATE_NORM, 1>(nvec, w, V, ldv, coef, part, n, s);
  else
    launch_orth<ORTH_UPDATE_DOTS_NORM, 1>(nvec, w, V, ldv, coef, part, n, s);
  const int nout = mode == ORTH_UPDATE_NORM ? 1 : (mode == ORTH_UPDATE_DOTS_NORM ? nvec + 1 : nvec);
  hipLaunchKernelGGL(orth_finish_kernel, dim3(1), dim3(kFinishThreads), 0, s, out, part, orth_blocks(n), nout);
}

// y = x / d with d = denom[0], or d = sqrt(denom[0]) when SQ; optionally also y2 = y in the
// precision of the V-cycle (the preconditioner's input) and the finest level's Chebyshev start
// from y2 (the same expression as cheb_init_kernel)
template <typename T2>
struct StartT {
  T2* z0;
  T2* d0;
  const T2* dinv;
  T2 itu, itp;
  long long nu;
};
template <typename T2>
StartT<T2> start_t(const VStart& v) {
  return StartT<T2>{(T2*)v.z0, (T2*)v.d0, (const T2*)v.dinv, (T2)v.ith_u, (T2)v.ith_p, v.nu};
}
template <typename T2>
__device__ __forceinline__ void write_start(const StartT<T2>& cs, long long i, T2 b) {
  if (cs.z0) {
    const T2 z = cs.dinv[i] * b * (i < cs.nu ? cs.itu : cs.itp);
    cs.z0[i] = z;
    cs.d0[i] = z;
  }
}
template <bool SQ, typename T2>
__global__ void scale_dev_kernel(double* y, T2* y2, const double* x, const double* denom, long long n, StartT<T2> cs) {
  const double d = SQ ? sqrt(denom[0]) : denom[0];
  GSTRIDE(i, n) {
    const double v = x[i] / d;
    y[i] = v;
    if (y2) {
      const T2 b = (T2)v;
      y2[i] = b;
      write_start(cs, i, b);
    }
  }
}
template <bool SQ>
void launch_scale(double* y, const double* x, const double* denom, long long n, hipStream_t s, void* y2, bool y2_f32,
                  const VStart& vs) {
  if (y2_f32)
    hipLaunchKernelGGL((scale_dev_kernel<SQ, float>), dim3(grid_for(n)), dim3(kThreads), 0, s, y, (float*)y2, x, denom, n,
                       start_t<float>(vs));
  else
    hipLaunchKernelGGL((scale_dev_kernel<SQ, double>), dim3(grid_for(n)), dim3(kThreads), 0, s, y, (double*)y2, x, denom, n,
                       start_t<double>(vs));
}
void k_scale_dev(double* y, const double* x, const double* denom, long long n, hipStream_t s, void* y2, bool y2_f32,
                 const VStart& vs) {
  launch_scale<false>(y, x, denom, n, s, y2, y2_f32, vs);
}
void k_scale_rsqrt_dev(double* y, const double* x, const double* sq, long long n, hipStream_t s, void* y2, bool y2_f32,
                       const VStart& vs) {
  launch_scale<true>(y, x, sq, n, s, y2, y2_f32, vs);
}
// The second Gram-Schmidt projection fused with the normalisation (CGS2 with the norm taken by
// Pythagoras): c = (h2_0 .. h2_{NV-1}, |w|^2) from ORTH_UPDATE_DOTS_NORM, |w - V h2|^2 =
// |w|^2 - |h2|^2 since the basis is orthonormal; v = (w - V h2) / |w - V h2| goes to vout and,
// in the V-cycle's precision, to y2 with the finest level's Chebyshev start.  A non-positive
// |w - V h2|^2 (w in the span of the basis: the Krylov space is invariant) writes v = 0.
template <int NV, typename T2>
__global__ __launch_bounds__(kThreads) void orth_normalize_kernel(double* __restrict__ vout, T2* __restrict__ y2,
                                                                  const double* __restrict__ w, const double* __restrict__ V,
                                                                  long long ldv, const double* __restrict__ coef, long long n,
                                                                  StartT<T2> cs) {
  double c[NV];
  double hn2 = coef[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    c[j] = coef[j];
    hn2 -= c[j] * c[j];
  }
  const double hn = hn2 > 0.0 ? sqrt(hn2) : 0.0;
  auto one = [&](long long i, double wi, const double* vj) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) t += c[j] * vj[j];
    const double v = hn > 0.0 ? (wi - t) / hn : 0.0;
    vout[i] = v;
    const T2 b = (T2)v;
    y2[i] = b;
    write_start(cs, i, b);
  };
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long long p = gid; 2 * p + 1 < n; p += stride) {
    const long long i = 2 * p;
    double2 v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = *reinterpret_cast<const double2*>(V + (long long)j * ldv + i);
    const double2 wi = *reinterpret_cast<const double2*>(w + i);
    __builtin_amdgcn_sched_barrier(0);
    double a[NV], b[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      a[j] = v[j].x;
      b[j] = v[j].y;
    }
    one(i, wi.x, a);
    one(i + 1, wi.y, b);
  }
  if ((n & 1) && gid == 0) {
    double a[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) a[j] = V[(long long)j * ldv + n - 1];
    one(n - 1, w[n - 1], a);
  }
}
template <int NV, typename T2>
static void launch_normalize(int nvec, double* vout, T2* y2, const double* w, const double* V, long long ldv,
                             const double* coef, long long n, const StartT<T2>& cs, hipStream_t s) {
  if constexpr (NV <= kOrthMax) {
    if (nvec == NV) {
      hipLaunchKernelGGL((orth_normalize_kernel<NV, T2>), dim3(grid_for(n / 2 + 1)), dim3(kThreads), 0, s, vout, y2, w, V, ldv,
                         coef, n, cs);
      return;
    }
    launch_normalize<NV + 1, T2>(nvec, vout, y2, w, V, ldv, coef, n, cs, s);
  }
}
void k_orth_normalize(double* vout, void* y2, bool y2_f32, const double* w, const double* V, long long ldv, int nvec,
                      const double* coef, long long n, const VStart& vs, hipStream_t s) {
  if (y2_f32) launch_normalize<1, float>(nvec, vout, (float*)y2, w, V, ldv, coef, n, start_t<float>(vs), s);
  else launch_normalize<1, double>(nvec, vout, (double*)y2, w, V, ldv, coef, n, start_t<double>(vs), s);
}

template <typename T2>
__global__ void vcycle_input_kernel(T2* b, const double* r, long long n, StartT<T2> cs) {
  GSTRIDE(i, n) {
    const T2 v = (T2)r[i];
    b[i] = v;
    write_start(cs, i, v);
  }
}
void k_vcycle_input(void* b, bool b_f32, const double* r, long long n, const VStart& vs, hipStream_t s) {
  if (b_f32)
    hipLaunchKernelGGL(vcycle_input_kernel<float>, dim3(grid_for(n)), dim3(kThreads), 0, s, (float*)b, r, n,
                       start_t<float>(vs));
  else
    hipLaunchKernelGGL(vcycle_input_kernel<double>, dim3(grid_for(n)), dim3(kThreads), 0, s, (double*)b, r, n,
                       start_t<double>(vs));
}
__global__ void sum_pvjp_kernel(double* out, const double* part, int nb) {
  __shared__ double sh[8];
  // both sums in one pass over the partials, loads of several iterations in flight
  double a0 = 0, a1 = 0;
#pragma unroll 8
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const double2 v = reinterpret_cast<const double2*>(part)[b];
    a0 += v.x;
    a1 += v.y;
  }
  const double s0 = block_sum(a0, sh);
  const double s1 = block_sum(a1, sh);
  if (threadIdx.x == 0) {
    out[0] = s0;
    out[1] = s1;
  }
}
void k_sum_pvjp(double* out2, const double* part, int nb, hipStream_t s) {
  hipLaunchKernelGGL(sum_pvjp_kernel, dim3(1), dim3(kThreads), 0, s, out2, part, nb);
}

// ---------------------------------------------------------------- CG-Lanczos
// Block-wise Jacobi-preconditioned CG (u block and phi block at once), all
// scalars kept on the device.  Breakdown rules: stop a block when r.z == 0
// or p.Ap <= 0.
__global__ void lanczos_init_kernel(LanczosState* st, const double* part, int nb) {
  __shared__ double sh[8];
  for (int b = 0; b < 2; ++b) {
    double acc = 0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[2 * i + b];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) {
      st->rz[b] = s;
      st->active[b] = 1;
      st->count[b] = 0;
      st->alpha[b] = 0;
      st->beta[b] = 0;
    }
  }
}
void k_lanczos_init(LanczosState* st, const double* part, int nb, hipStream_t s) {
  hipLaunchKernelGGL(lanczos_init_kernel, dim3(1), dim3(kThreads), 0, s, st, part, nb);
}
__global__ void lanczos_alpha_kernel(LanczosState* st, const double* part, int nb, int step) {
  __shared__ double sh[8];
  for (int b = 0; b < 2; ++b) {
    double acc = 0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[2 * i + b];
    const double pAp = block_sum(acc, sh);
    if (threadIdx.x == 0) {
      if (st->active[b]) {
        if (st->rz[b] == 0.0 || !(pAp > 0.0)) {
          st->active[b] = 0;
          st->alpha[b] = 0;
        } else {
          const double al = st->rz[b] / pAp;
          st->alpha[b] = al;
          st->alphas[b][step] = al;
          st->count[b] = step + 1;
        }
      } else {
        st->alpha[b] = 0;
      }
    }
  }
}
void k_lanczos_alpha(LanczosState* st, const double* part, int nb, int step, hipStream_t s) {
  hipLaunchKernelGGL(lanczos_alpha_kernel, dim3(1), dim3(kThreads), 0, s, st, part, nb, step);
}
// r -= alpha_b t ; z = dinv r ; partials of r.z per block
__global__ void lanczos_update_r_kernel(double* r, double* z, double* part, const double* t, const double* dinv,
                                        const LanczosState* st, long long nu, long long n) {
  __shared__ double sh[8];
  const double au = st->active[0] ? st->alpha[0] : 0.0;
  const double ap = st->active[1] ? st->alpha[1] : 0.0;
  const int nb = gridDim.x;
  for (int sgm = 0; sgm < 2; ++sgm) {
    const long long s0 = sgm == 0 ? 0 : nu, s1 = sgm == 0 ? nu : n;
    const long long len = s1 - s0;
    const long long chunk = (len + nb - 1) / nb;
    const long long lo = s0 + (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < s1 ? lo + chunk : s1;
    const double a = sgm == 0 ? au : ap;
    double acc = 0;
    for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const double rv = r[i] - a * t[i];
      const double zv = dinv[i] * rv;
      r[i] = rv;
      z[i] = zv;
      acc += rv * zv;
    }
    const double sum = block_sum(acc, sh);
    if (threadIdx.x == 0) part[2 * blockIdx.x + sgm] = sum;
  }
}
void k_lanczos_update_r(double* r, double* z, double* part, const double* t, const double* dinv, const LanczosState* st,
                        long long nu, long long n, hipStream_t s) {
  hipLaunchKernelGGL(lanczos_update_r_kernel, dim3(dot_blocks(n)), dim3(kThreads), 0, s, r, z, part, t, dinv, st, nu, n);
}
// z = dinv r and partials of r.z (start of the iteration)
__global__ void lanczos_rz_kernel(double* part, const double* r, const double* dinv, double* z, long long nu, long long n) {
  __shared__ double sh[8];
  const int nb = gridDim.x;
  for (int sgm = 0; sgm < 2; ++sgm) {
    const long long s0 = sgm == 0 ? 0 : nu, s1 = sgm == 0 ? nu : n;
    const long long len = s1 - s0;
    const long long chunk = (len + nb - 1) / nb;
    const long long lo = s0 + (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < s1 ? lo + chunk : s1;
    double acc = 0;
    for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const double zv = dinv[i] * r[i];
      z[i] = zv;
      acc += r[i] * zv;
    }
    const double sum = block_sum(acc, sh);
    if (threadIdx.x == 0) part[2 * blockIdx.x + sgm] = sum;
  }
}
void k_lanczos_rz_partials(double* part, const double* r, const double* dinv, double* z, long long nu, long long n,
                           hipStream_t s) {
  hipLaunchKernelGGL(lanczos_rz_kernel, dim3(dot_blocks(n)), dim3(kThreads), 0, s, part, r, dinv, z, nu, n);
}
__global__ void lanczos_beta_kernel(LanczosState* st, const double* part, int nb, int step) {
  __shared__ double sh[8];
  for (int b = 0; b < 2; ++b) {
    double acc = 0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[2 * i + b];
    const double rzn = block_sum(acc, sh);
    if (threadIdx.x == 0) {
      if (st->active[b]) {
        const double be = rzn / st->rz[b];
        st->beta[b] = be;
        st->betas[b][step] = be;
        st->rz[b] = rzn;
      } else {
        st->beta[b] = 0;
      }
    }
  }
}
void k_lanczos_beta(LanczosState* st, const double* part, int nb, int step, hipStream_t s) {
  hipLaunchKernelGGL(lanczos_beta_kernel, dim3(1), dim3(kThreads), 0, s, st, part, nb, step);
}
// p = z + beta_b p (active blocks only)
__global__ void lanczos_update_p_kernel(double* p, const double* z, const LanczosState* st, long long nu, long long n) {
  const int au = st->active[0], ap = st->active[1];
  const double bu = st->beta[0], bp = st->beta[1];
  GSTRIDE(i, n) {
    const bool isu = i < nu;
    if (isu ? au : ap) p[i] = z[i] + (isu ? bu : bp) * p[i];
  }
}
void k_lanczos_update_p(double* p, const double* z, const LanczosState* st, long long nu, long long n, hipStream_t s) {
  hipLaunchKernelGGL(lanczos_update_p_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, p, z, st, nu, n);
}

#define INST(T)                                                                                                    \
  template void k_mask_init<T>(T*, const T*, const T*, const uint8_t*, long long, int, T, hipStream_t);            \
  template void k_copy<T>(T*, const T*, long long, hipStream_t);                                                   \
  template void k_fill<T>(T*, T, long long, hipStream_t);                                                          \
  template void k_axpy<T>(T*, T, const T*, long long, hipStream_t);                                                \
  template void k_diag_finish<T>(T*, double*, const T*, const uint8_t*, long long, int, hipStream_t);              \
  template void k_cheb_init<T>(T*, T*, const T*, const T*, long long, int, T, T, hipStream_t);                     \
  template void k_cheb_step<T>(T*, T*, const T*, const T*, const T*, long long, int, T, T, T, T, hipStream_t);     \
  template void k_cheb_update<T>(T*, T*, const T*, const T*, const T*, const T*, long long, int, T, T, T, T,      \
                                 const T*, T*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace mfpff

MFPFF_BOUNDS_READER(bounds_hits_vector)
