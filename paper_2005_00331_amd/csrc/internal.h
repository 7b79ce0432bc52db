// Internal declarations shared by the host solver core and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace mfpff {

constexpr int kMaxDeg = 4;
constexpr int kThreads = 256;
// Index arithmetic in the kernels divides in 32 bits (a 64-bit division by a runtime value costs
// ~100 instructions on gfx950); mfpff_setup_mesh_levels rejects levels with 2^31 or more dofs.
__host__ __device__ __forceinline__ unsigned udiv(unsigned long long a, unsigned long long b) {
  return (unsigned)a / (unsigned)b;
}
// v where keep, else +0: a bitwise select, so that the compiler does not turn it into a branch
// around the load that produced v (which would wait for the condition before issuing the load)
// sign bit of v (true for -0.0 too) and |v|, both by bits
template <typename T>
__device__ __forceinline__ bool sign_bit(T v) {
  if constexpr (sizeof(T) == 8) return __double_as_longlong(v) < 0;
  else return __float_as_int(v) < 0;
}
template <typename T>
__device__ __forceinline__ T abs_bits(T v) {
  if constexpr (sizeof(T) == 8) return __longlong_as_double(__double_as_longlong(v) & 0x7fffffffffffffffll);
  else return __int_as_float(__float_as_int(v) & 0x7fffffff);
}

template <typename T>
__device__ __forceinline__ T keep_if(T v, bool keep) {
  if constexpr (sizeof(T) == 8) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v) & (keep ? ~0ull : 0ull);
    return __longlong_as_double((long long)b);
  } else {
    const unsigned b = __float_as_uint(v) & (keep ? ~0u : 0u);
    return __uint_as_float(b);
  }
}

// Geometry of one structured level: unit square/cube, N cells per direction,
// Q_k with equispaced nodes, M = k*N + 1 nodes per direction.
struct Geom {
  int dim, k, N, M;
  long long n_nodes;  // grid nodes plus, on a slit mesh, the duplicated slit nodes after them
  double h;
  long long n_grid;   // M^dim
  int slit;           // the slit of the notched tests (Section 5.1) on the mid-plane of the last axis,
                      // x < 1/2: its k N / 2 (3D: times M) grid nodes belong to the cells below it and
                      // duplicates, numbered n_grid + i0 (+ (k N / 2) i1), to the cells above it
};

struct MatParams {
  double lam, mu, Gc, eps, kappa;
  int split;  // SplitKind: 0 volumetric/deviatoric (Amor), 1 spectral (Miehe)
};

// 1D tables of one degree k on the unit interval (q = k+1 Gauss points):
//   B[q][i]  = l_i(x_q)           Lagrange basis on equispaced nodes
//   D[q][i]  = l_i'(x_q)
//   C[q][r]  = derivative at x_q of the Lagrange polynomial through the Gauss
//              points that is 1 at x_r (collocation derivative)
//   w[q]     = Gauss weight
template <typename T>
struct Tables {
  T B[kMaxDeg + 1][kMaxDeg + 1];
  T D[kMaxDeg + 1][kMaxDeg + 1];
  T C[kMaxDeg + 1][kMaxDeg + 1];
  T w[kMaxDeg + 1];
};

void make_tables(int k, Tables<double>& t);

// Node mask bits
constexpr uint8_t kMaskPhi = 1;   // phi dof fixed (active set)
constexpr uint8_t kMaskU = 2;     // all displacement dofs fixed (Dirichlet)

enum CellMode : int {
  MODE_APPLY = 0,     // full operator G
  MODE_APPLY_T = 1,   // transpose G^T
  MODE_BLOCK = 2,     // diag(G_uu, G_phiphi)
  MODE_RESIDUAL = 3,  // residual (no x)
  MODE_PVJP = 4,      // parameter cotangents (x = v)
  MODE_ELEM = 5,      // element columns of G scattered into a dense matrix
  MODE_QDATA = 6      // tangent coefficients at the Gauss points (written to qd_out): 2D Q1/Q2, 3D
};

// Tangent coefficients of eq. (G) cached per Gauss point for the 2D row kernel:
// g(phi~) with the sign bit set where tr e < 0, g'(phi) sigma^+ (xx, yy, xy), g''(phi) E^+ + Gc/eps;
// layout [tile][coefficient][Gauss row][Gauss column][cell of the tile],
// rowcell_qdata_len values per level
constexpr int kQCoef = 5;
long long rowcell_qdata_len(const Geom& g, int split);

template <typename T>
struct CellArgs {
  Geom g;
  MatParams m;
  const T* x;          // input vector (APPLY*, BLOCK, PVJP), (d+1)*n_nodes
  T* y;                // output accumulated with atomics
  const T* u;          // displacement, d*n_nodes
  const T* phi;        // n_nodes
  const T* phit;       // n_nodes
  const uint8_t* mask; // per node, may be null (nothing fixed)
  T scale;             // contributions multiply by this (+1 apply, -1 residual form)
  double* partials;    // PVJP: 2 doubles per block
  double* dense;       // ELEM: row-major (d+1)*n_nodes square matrix
  double* elem_mat;    // ELEM: element matrices [cell][row][column] instead of the dense scatter
  long long ld;        // ELEM: leading dimension
  const T* qd;         // 2D Q1/Q2: cached tangent coefficients (null: computed from u, phi, phi~)
  T* qd_out;           // MODE_QDATA: where the coefficients go
  T* elem;             // 3D operator modes: cell results [cell][component][point] instead of atomics
  int mfma;            // 3D products at degree >= 3 (volumetric/deviatoric split): contractions on the
                       // matrix cores (mfma_kernel.hip) instead of the vector unit (linecell_kernel.hip)
};

// Fused vector epilogues of the owner-computes kernels (tile_kernel.hip)
enum EpiKind : int { EPI_APPLY = 0, EPI_RESID = 1, EPI_CHEB = 2 };
template <typename T>
struct Epilogue {
  T* y;                 // apply: y; resid: r; cheb: new iterate z'
  const T* b;           // resid: right-hand side
  T* z0;                // resid: optional Chebyshev start z = D^-1 r / theta
  T* d0;                //        and d = z
  const T* dinv;        // inverse diagonal
  T ith_u, ith_p;       // 1/theta per block
  const T* r;           // cheb: smoother right-hand side
  T* d;                 // cheb: direction, updated in place
  T c1u, c2u, c1p, c2p; // cheb: d = c1 d + c2 D^-1 (r - t)
  const T* xacc;        // cheb: optional xout = xacc + z'
  T* xout;
  T* xcopy;             // apply: optional copy of x (every node written)
};
// node gather of the 3D element results (cell_kernel with a.elem) with a fused epilogue
template <typename T>
hipError_t launch_gather_3d(int epi, const T* elem, const CellArgs<T>& a, const Epilogue<T>& e, hipStream_t s);
long long elem_len(const Geom& g);  // values in the element buffer of one level
// 3D products (APPLY, APPLY_T, BLOCK) from the cached coefficients into the element buffer,
// one thread per node line (linecell_kernel.hip); a.qd and a.elem required
template <typename T>
hipError_t launch_linecell(int mode, const CellArgs<T>& a, const Tables<T>* tab_dev, hipStream_t s);
long long cell_qdata_len(const Geom& g, int split);  // 3D: values of the cached tangent coefficients of one level
// the same 3D products at degree 3 and 4 with the 1D contractions on the matrix cores (MFMA),
// volumetric/deviatoric split only (mfma_kernel.hip); a.qd and a.elem required
template <typename T>
hipError_t launch_mfmacell(int mode, const CellArgs<T>& a, const Tables<T>* tab_dev, hipStream_t s);
template <typename T>
hipError_t launch_tile_2d(int mode, int epi, const CellArgs<T>& a, const Epilogue<T>& e, const Tables<T>* tab, hipStream_t s);
long long tile_blocks_2d(const Geom& g);
template <typename T>
hipError_t launch_rowcell_2d(int mode, int epi, const CellArgs<T>& a, const Epilogue<T>& e, hipStream_t s);
long long rowcell_blocks_2d(const Geom& g);

// ---- launchers (cell_kernel.hip)
template <typename T>
hipError_t launch_cell(int mode, const CellArgs<T>& a, const Tables<T>* tab_dev, hipStream_t s);
template <typename T>
hipError_t launch_diag(const CellArgs<T>& a, const Tables<T>* tab_dev, hipStream_t s);
long long cell_blocks(const Geom& g, int mode);

// ---- vector kernels (vector_ops.hip); n = element count
template <typename T>
void k_mask_init(T* y, const T* b, const T* x, const uint8_t* mask, long long nn, int dim, T scale, hipStream_t s);
template <typename T>
void k_copy(T* y, const T* x, long long n, hipStream_t s);
template <typename T>
void k_fill(T* y, T v, long long n, hipStream_t s);
template <typename T>
void k_axpy(T* y, T a, const T* x, long long n, hipStream_t s);
template <typename T>
void k_diag_finish(T* dinv, double* diag_out, const T* diag, const uint8_t* mask, long long nn, int dim, hipStream_t s);
template <typename T>
void k_cheb_init(T* z, T* d, const T* r, const T* dinv, long long nn, int dim, T inv_th_u, T inv_th_p, hipStream_t s);
template <typename T>
void k_cheb_step(T* z, T* d, const T* r, const T* t, const T* dinv, long long nn, int dim,
                 T c1u, T c2u, T c1p, T c2p, hipStream_t s);
template <typename T>
void k_cheb_update(T* zout, T* d, const T* zin, const T* r, const T* t, const T* dinv, long long nn, int dim,
                   T c1u, T c2u, T c1p, T c2p, const T* xacc, T* xout, hipStream_t s);
void k_cast_d2f(float* y, const double* x, long long n, hipStream_t s);
void k_cast_f2d(double* y, const float* x, long long n, hipStream_t s);
void k_mask_vec(double* y, const uint8_t* mask, long long nn, int dim, double scale, hipStream_t s);
template <typename T>
void k_slit_epilogue(T* y, const T* x, const T* b, const uint8_t* mask, long long nn, int dim, hipStream_t s);
void k_inject(double* lin_c, uint8_t* mask_c, const double* lin_f, const uint8_t* mask_f,
              const Geom& gc, const Geom& gf, int dirichlet, hipStream_t s);
void k_fine_fields(double* lin, uint8_t* mask, const double* u, const double* phi, const double* phit,
                   const uint8_t* active, const Geom& g, int dirichlet, hipStream_t s);
void k_lumped_mass(double* ml, const Geom& g, const double* w1d, hipStream_t s);
void k_active_set(uint8_t* act, const double* R, const double* phi, const double* phi_old, const double* ml,
                  long long nn, int dim, double c, hipStream_t s);
void k_splitmix_start(double* v, const uint8_t* mask, long long nn, int dim, unsigned long long seed,
                      int stream_u, int stream_p, hipStream_t s);

// Reductions: partial sums per block, then a one-block finish.
int dot_blocks(long long n);
// phi_i := phi_old_i on the active set (the projected active-set update)
void k_project_active(double* phi, const double* phi_old, const uint8_t* act, long long n, hipStream_t s);
// load stepping: boundary values on the two faces normal to the last axis (bottom 0, top
// top[0..dim)), phi~ = 2 p1 - p2, and per-(face, component) reaction sums (2 * dim values)
void k_impose_faces(double* u, const Geom& g, const double* top, hipStream_t s);
void k_extrapolate(double* pt, const double* p1, const double* p2, long long n, hipStream_t s);
void k_face_reaction(double* out, const double* R, const Geom& g, hipStream_t s);
// stopping test of Algorithm 1: per-workgroup (sum of R^2 on the free dofs, changed nodes of act vs prev)
int pdas_check_blocks(long long nn);
void k_pdas_check(double* part, const double* R, const uint8_t* act, const uint8_t* prev, const Geom& g, int dirichlet,
                  hipStream_t s);
void k_multidot_partials(double* part, const double* V, long long ldv, int nvec, const double* w, long long n, hipStream_t s);
void k_multidot_finish(double* out, const double* part, int nblocks, int nvec, hipStream_t s);
void k_seg_dot_partials(double* part, const double* a, const double* b, long long nu, long long n, hipStream_t s);
void k_maxpy_dev(double* w, const double* V, long long ldv, int nvec, const double* coef, double sign, long long n, hipStream_t s);
// The finest level's Chebyshev start written with the V-cycle's right-hand side b (in the
// V-cycle's precision): z0 = d0 = D^-1 b / theta per block (z0 null: none, a one-level V-cycle)
struct VStart {
  void* z0 = nullptr;
  void* d0 = nullptr;
  const void* dinv = nullptr;
  double ith_u = 1.0, ith_p = 1.0;
  long long nu = 0;  // displacement dofs (the u block ends there)
};
// y = x / denom[0] (rsqrt: x / sqrt(denom[0])); y2, if given, receives a copy (FP32 when y2_f32)
// and then vs the Chebyshev start from that copy
void k_scale_dev(double* y, const double* x, const double* denom, long long n, hipStream_t s, void* y2 = nullptr,
                 bool y2_f32 = false, const VStart& vs = VStart{});
void k_scale_rsqrt_dev(double* y, const double* x, const double* sq, long long n, hipStream_t s, void* y2 = nullptr,
                       bool y2_f32 = false, const VStart& vs = VStart{});
// b = r in the V-cycle's precision and the Chebyshev start from it
void k_vcycle_input(void* b, bool b_f32, const double* r, long long n, const VStart& vs, hipStream_t s);
// Arnoldi passes (modes: 0 dots, 1 update + dots, 2 update + squared norm, 3 update + dots +
// squared norm), each followed by a one-workgroup launch that finishes the reduction into out;
// nvec <= kOrthMax; part holds orth_blocks(n) * (nvec + 1) doubles
constexpr int kOrthMax = 32;
int orth_blocks(long long n);
void k_orth_pass(int mode, double* w, const double* V, long long ldv, int nvec, const double* coef, double* part,
                 double* out, long long n, hipStream_t s);
// vout = (w - V c) / sqrt(c[nvec] - |c|^2) with c from mode 3 (0 when that is not positive), and
// y2 = vout in the V-cycle's precision with the Chebyshev start vs
void k_orth_normalize(double* vout, void* y2, bool y2_f32, const double* w, const double* V, long long ldv, int nvec,
                      const double* coef, long long n, const VStart& vs, hipStream_t s);
void k_sum_pvjp(double* out2, const double* part, int nblocks, hipStream_t s);

// CG-Lanczos device scalars
struct LanczosState {
  double rz[2], alpha[2], beta[2];
  int active[2], count[2];
  double alphas[2][64], betas[2][64];
};
void k_lanczos_alpha(LanczosState* st, const double* part, int nblocks, int step, hipStream_t s);
void k_lanczos_update_r(double* r, double* z, double* part, const double* t, const double* dinv,
                        const LanczosState* st, long long nu, long long n, hipStream_t s);
void k_lanczos_beta(LanczosState* st, const double* part, int nblocks, int step, hipStream_t s);
void k_lanczos_update_p(double* p, const double* z, const LanczosState* st, long long nu, long long n, hipStream_t s);
void k_lanczos_init(LanczosState* st, const double* part, int nblocks, hipStream_t s);
void k_lanczos_rz_partials(double* part, const double* r, const double* dinv, double* z, long long nu, long long n, hipStream_t s);

// ---- transfers (transfer.hip): apply a 1D sparse matrix along one axis
struct Sparse1D {
  int n_out, n_in, width;   // rows (outputs), columns (inputs), entries per row (padded)
  const int* col;           // n_out*width, -1 = padding
  const double* val;        // n_out*width
  const float* valf;
};
// a CSR matrix on the device (the transfers of slit levels)
struct CsrDev {
  const int* rowptr;  // n_rows + 1
  const int* col;
  const double* val;
  const float* valf;
};
template <typename T>
void k_csr_transfer(T* out, const T* in, const CsrDev& A, const uint8_t* mask_in, const uint8_t* mask_out, long long n_out,
                    long long n_in, int dim, bool add, hipStream_t s);
// Chebyshev start written by a restriction's last pass: z0 = d0 = D^-1 out / theta_b (z0 null: none)
template <typename T>
struct ChebStart {
  T* z0 = nullptr;
  T* d0 = nullptr;
  const T* dinv = nullptr;
  T ith_u = T(1), ith_p = T(1);
};
// in_mask: zero inputs at fixed dofs (input must be a whole level vector);
// out_mask: zero outputs at fixed dofs (output must be a whole level vector);
// add: out += result instead (fixed outputs left unchanged); cs: see ChebStart (last pass only)
template <typename T>
void k_axis_apply(T* out, const T* in, const Sparse1D& A, int axis, int dim, const long long* dims_in,
                  int ncomp, const uint8_t* in_mask, const uint8_t* out_mask, hipStream_t s, bool add = false,
                  ChebStart<T> cs = ChebStart<T>{});
// out (fine level) = / += P~ xc: single pass, (kc+1)^d coarse terms per fine node
template <typename T>
void k_prolong(T* out, const T* xc, const Sparse1D& P, const uint8_t* mask_c, const uint8_t* mask_f, const Geom& gf,
               const Geom& gc, bool add, hipStream_t s);
template <typename T>
void k_mask_comp(T* y, const uint8_t* mask, long long nn, int dim, hipStream_t s);
template <typename T>
void k_add_masked(T* y, const T* x, const uint8_t* mask, long long nn, int dim, hipStream_t s);

// ---- dense coarse solver (dense.hip), row-major FP64
void k_dense_set_fixed_diag(double* A, long long ld, const uint8_t* mask, long long nn, int dim, hipStream_t s);
void k_extract_block(double* dst, long long ldd, const double* src, long long lds, long long r0, long long c0,
                     long long nr, long long nc, hipStream_t s);
hipError_t cholesky_lower(double* A, int n, int* info_dev, double* scratch, hipStream_t s);  // info_dev zeroed by the caller
hipError_t tri_inverse_lower(double* W, const double* L, int n, hipStream_t s);
// Inv = M^-1 by Gauss-Jordan with partial pivoting (M overwritten; *info_dev = first zero-pivot
// step + 1, zeroed by the caller; work holds n + 3 doubles)
hipError_t gauss_jordan_inverse(double* Inv, double* M, int n, int* info_dev, double* work, hipStream_t s);
void k_transpose(double* At, const double* A, int n, hipStream_t s);
// y = alpha A x (+ yin); GEMV_LOWER / GEMV_UPPER read only row i's entries j <= i / j >= i
enum GemvShape : int { GEMV_FULL = 0, GEMV_LOWER = 1, GEMV_UPPER = 2 };
void k_gemv(double* y, const double* A, long long lda, const double* x, int rows, int cols, double alpha,
            const double* yin, int shape, hipStream_t s);
// the same with x and yin in FP64 or FP32 (x32, yin32) and an optional FP32 copy of y (y32; y may
// then be null)
void k_gemv_mixed(double* y, float* y32, const double* A, long long lda, const void* x, bool x32, int rows, int cols,
                  double alpha, const void* yin, bool yin32, int shape, hipStream_t s);

}  // namespace mfpff
