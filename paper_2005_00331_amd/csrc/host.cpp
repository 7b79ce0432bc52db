// Host solver core and C ABI of libmfpff (see include/mfpff.h).
//
// Orchestrates the GPU kernels: level hierarchy set-up, linearisation
// (field injection, diagonals, CG-Lanczos estimates, coarse factorisation),
// the monolithic V-cycle of Section 3.3, flexible GMRES with classical
// Gram-Schmidt twice (Givens rotations on the host), and the active-set
// Newton step of Algorithm 1.  All device work is enqueued on one stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mfpff.h"
#include "internal.h"

using namespace mfpff;

namespace {

struct HipError {
  hipError_t e;
  const char* what;
};
struct StatusError {
  mfpff_status st;
  std::string msg;
};

#define HIPCHK(call)                                  \
  do {                                                \
    hipError_t _e = (call);                           \
    if (_e != hipSuccess) throw HipError{_e, #call};  \
  } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

template <typename T>
T* dalloc(size_t n) {
  void* p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw StatusError{MFPFF_ERR_OOM, "device allocation failed"};
  return (T*)p;
}

struct HostSparse {
  int n_out = 0, n_in = 0, width = 0;
  std::vector<int> col;
  std::vector<double> val;
};

struct DevSparse {
  Sparse1D s{};
  int* col = nullptr;
  double* val = nullptr;
  float* valf = nullptr;
};

// a CSR matrix on the host and its device copy (the per-component transfers of slit levels)
struct HostCsr {
  int n_rows = 0, n_cols = 0;
  std::vector<int> rowptr, col;
  std::vector<double> val;
};
struct DevCsrBuf {
  int* rowptr = nullptr;
  int* col = nullptr;
  double* val = nullptr;
  float* valf = nullptr;
  CsrDev view() const { return CsrDev{rowptr, col, val, valf}; }
};

struct Level {
  Geom g{};
  long long nn = 0, n = 0;
  double* lin = nullptr;   // (d+2)*nn
  float* lin32 = nullptr;
  uint8_t* mask = nullptr;
  double* dinv = nullptr;
  float* dinv32 = nullptr;
  double* diag = nullptr;  // FP64 diagonal of G^ (1 at fixed dofs)
  double* qd = nullptr;    // 2D Q1/Q2: tangent coefficients at the Gauss points (set with the point)
  float* qd32 = nullptr;
  bool qd_ok = false;
  double lam[2] = {1.0, 1.0};
  int lsteps[2] = {0, 0};
  std::vector<double> c1u, c2u, c1p, c2p;  // Chebyshev step coefficients, index i = 1..s-1
  double ith_u = 1.0, ith_p = 1.0;
  void* w[7] = {};  // V-cycle vectors b, x, r, t, d, z, z2
  DevSparse P1, R1;  // transfer from level-1 to this level
  DevCsrBuf SP, SR;  // slit levels: the same transfer as CSR matrices (prolongation, restriction)
};
enum { WB = 0, WX = 1, WR = 2, WT = 3, WD = 4, WZ = 5, WZ2 = 6, NW = 7 };

}  // namespace

struct mfpff_ctx {
  mfpff_problem prob{};
  hipStream_t s = nullptr;
  int device = -1;  // HIP device current at set-up (the stream's device)
  int dim = 2, L = 0;  // L = index of the finest level
  bool f32 = false;
  std::vector<Level> lv;
  Tables<double>* tab64[kMaxDeg + 1] = {};
  Tables<float>* tab32[kMaxDeg + 1] = {};
  double* w1d = nullptr;  // integrals of the finest-degree 1D basis functions
  double* ml = nullptr;   // lumped phi mass on the finest level
  // transfer temporaries (finest-level size)
  double* t64a = nullptr;
  double* t64b = nullptr;
  float* t32a = nullptr;
  float* t32b = nullptr;
  // 3D: cell results of one product, gathered per node (element buffer, sized for the largest level)
  void* elem = nullptr;
  // coarse solve
  int nu0 = 0, np0 = 0;
  double* dense = nullptr;
  double* Auu = nullptr;
  double* App = nullptr;
  double* Wu = nullptr;
  double* WuT = nullptr;
  double* Wp = nullptr;
  double* WpT = nullptr;
  double* Gpu = nullptr;
  double* cs_out = nullptr;
  double* cs_t = nullptr;
  int* info_dev = nullptr;
  double* chol_scratch = nullptr;
  // a block whose Cholesky failed holds its explicit inverse in W (WT unused): one product
  bool coarse_lu[2] = {false, false};
  double* lu_work = nullptr;  // multipliers and pivot of the Gauss-Jordan fallback (allocated on first use)
  // Lanczos / scratch (finest size, FP64)
  LanczosState* lst = nullptr;
  double* s64[5] = {};
  double* part = nullptr;
  int part_len = 0;
  // GMRES
  int m = 30;
  double* V = nullptr;
  long long ldv = 0;  // stride of the basis vectors in V
  double* Z = nullptr;
  double* gw = nullptr;
  double* gr = nullptr;
  double* hdev = nullptr;   // two Arnoldi result buffers (h1, h2, |w|^2), kHBuf doubles each
  double* hhost = nullptr;  // pinned: mirrors of both buffers, then staging for y and beta
  hipEvent_t hev[2] = {nullptr, nullptr};
  double* ycoef = nullptr;
  // Newton
  double* R = nullptr;
  double* b = nullptr;
  double* dU = nullptr;
  double* pvjp_part = nullptr;
  uint8_t* act_prev = nullptr;   // active-set loop: the previous step's active set
  double* pdas_part = nullptr;   // active-set loop: stopping-test partial sums
  double* phit_ext = nullptr;    // load stepping: the extrapolated phi~
  double* react = nullptr;       // load stepping: face reaction sums
  double* pvjp_out = nullptr;
  bool linearized = false;  // full linearisation (smoothers, coarse solve)
  bool has_point = false;   // fields and masks injected (products allowed)
  double* finite_flag = nullptr;
  double hhost_scalar = 0.0;
  // V-cycle captured as a graph after each linearisation (replayed per GMRES iteration)
  hipStream_t cap_s = nullptr;
  // the two coarse factorisations run on side streams while the Lanczos estimates run on s
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
  hipGraphExec_t vgraph = nullptr;
  bool graph_ok = true;
  std::string err;
};

namespace {

Geom make_geom(int dim, int N, int k, int slit = 0) {
  Geom g{};
  g.dim = dim;
  g.k = k;
  g.N = N;
  g.M = k * N + 1;
  g.n_grid = 1;
  for (int a = 0; a < dim; ++a) g.n_grid *= g.M;
  g.slit = slit;
  g.n_nodes = g.n_grid + (slit ? (long long)(k * N / 2) * (dim == 3 ? g.M : 1) : 0);
  g.h = 1.0 / N;
  return g;
}

double lagr(int k, int j, double x) {
  double v = 1.0;
  for (int m = 0; m <= k; ++m)
    if (m != j) v *= (x - (double)m / k) / ((double)j / k - (double)m / k);
  return v;
}

// 1D prolongation: fine node i gets the coarse basis values at its position.
void build_transfer(const Geom& gf, const Geom& gc, HostSparse& P, HostSparse& R) {
  const long long den = (long long)gf.k * gf.N;
  std::vector<std::vector<std::pair<int, double>>> rows(gf.M), cols(gc.M);
  for (int i = 0; i < gf.M; ++i) {
    long long cell = (long long)i * gc.N / den;
    if (cell > gc.N - 1) cell = gc.N - 1;
    const double xi = (double)((long long)i * gc.N - cell * den) / (double)den;
    for (int j = 0; j <= gc.k; ++j) {
      const double w = lagr(gc.k, j, xi);
      if (w != 0.0) {
        const int jc = (int)(gc.k * cell + j);
        rows[i].push_back({jc, w});
        cols[jc].push_back({i, w});
      }
    }
  }
  auto pack = [](std::vector<std::vector<std::pair<int, double>>>& lst, int nin, HostSparse& S) {
    S.n_out = (int)lst.size();
    S.n_in = nin;
    S.width = 0;
    for (auto& r : lst) S.width = std::max(S.width, (int)r.size());
    S.col.assign((size_t)S.n_out * S.width, -1);
    S.val.assign((size_t)S.n_out * S.width, 0.0);
    for (int o = 0; o < S.n_out; ++o)
      for (size_t j = 0; j < lst[o].size(); ++j) {
        S.col[(size_t)o * S.width + j] = lst[o][j].first;
        S.val[(size_t)o * S.width + j] = lst[o][j].second;
      }
  };
  pack(rows, gc.M, P);
  pack(cols, gf.M, R);
}

// Prolongation between two slit levels (rows: fine nodes, columns: coarse nodes), per component.
// Between grid nodes it is the tensor product of the 1D interpolation P1; each fine node takes
// the coarse values of its own side of the slit: a fine grid node strictly above the slit plane,
// and every fine duplicate (which interpolates like its grid node, along the plane), reads the
// duplicate of a coarse slit node (plane index kN/2, first index below kN/2) in place of that
// node.  Grid nodes below the plane or on it (the lower side) and the tip are unchanged.
HostCsr build_slit_prolongation(const Geom& gf, const Geom& gc, const HostSparse& P1) {
  const int d = gf.dim;
  const long long Mf = gf.M, Mc = gc.M, nsf = (long long)gf.k * gf.N / 2, nsc = (long long)gc.k * gc.N / 2;
  const long long plane_f = Mf / 2, plane_c = Mc / 2;
  HostCsr A;
  A.n_rows = (int)gf.n_nodes;
  A.n_cols = (int)gc.n_nodes;
  A.rowptr.assign((size_t)gf.n_nodes + 1, 0);
  size_t per_row = 1;
  for (int a = 0; a < d; ++a) per_row *= (size_t)P1.width;
  A.col.reserve((size_t)gf.n_nodes * per_row);
  A.val.reserve((size_t)gf.n_nodes * per_row);
  auto emit_row = [&](const long long* fm, bool other_side) {
    // the tensor product of the 1D rows of fm's indices
    int cnt[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a) {
      cnt[a] = 0;
      while (cnt[a] < P1.width && P1.col[(size_t)fm[a] * P1.width + cnt[a]] >= 0) ++cnt[a];
    }
    for (int e2 = 0; e2 < (d == 3 ? cnt[2] : 1); ++e2)
      for (int e1 = 0; e1 < cnt[1]; ++e1)
        for (int e0 = 0; e0 < cnt[0]; ++e0) {
          const int es[3] = {e0, e1, e2};
          long long cm[3] = {0, 0, 0}, col = 0, stride = 1;
          double w = 1.0;
          for (int a = 0; a < d; ++a) {
            const size_t o = (size_t)fm[a] * P1.width + es[a];
            cm[a] = P1.col[o];
            w *= P1.val[o];
            col += cm[a] * stride;
            stride *= Mc;
          }
          if (other_side && cm[d - 1] == plane_c && cm[0] < nsc) col = gc.n_grid + cm[0] + (d == 3 ? nsc * cm[1] : 0);
          A.col.push_back((int)col);
          A.val.push_back(w);
        }
  };
  long long row = 0;
  for (long long f = 0; f < gf.n_grid; ++f, ++row) {
    long long fm[3] = {0, 0, 0}, rem = f;
    for (int a = 0; a < d; ++a) {
      fm[a] = rem % Mf;
      rem /= Mf;
    }
    emit_row(fm, fm[d - 1] > plane_f);
    A.rowptr[(size_t)row + 1] = (int)A.col.size();
  }
  for (long long j = 0; j < gf.n_nodes - gf.n_grid; ++j, ++row) {
    const long long fm[3] = {j % nsf, d == 3 ? j / nsf : plane_f, plane_f};
    emit_row(fm, true);
    A.rowptr[(size_t)row + 1] = (int)A.col.size();
  }
  return A;
}

HostCsr csr_transpose(const HostCsr& A) {
  HostCsr T;
  T.n_rows = A.n_cols;
  T.n_cols = A.n_rows;
  T.rowptr.assign((size_t)A.n_cols + 1, 0);
  for (int c : A.col) ++T.rowptr[(size_t)c + 1];
  for (int i = 0; i < A.n_cols; ++i) T.rowptr[(size_t)i + 1] += T.rowptr[i];
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  std::vector<int> next(T.rowptr.begin(), T.rowptr.end() - 1);
  for (int r = 0; r < A.n_rows; ++r)  // rows in order: each transposed row lists its entries by fine node
    for (int e = A.rowptr[r]; e < A.rowptr[(size_t)r + 1]; ++e) {
      const int o = next[A.col[e]]++;
      T.col[o] = r;
      T.val[o] = A.val[e];
    }
  return T;
}

DevCsrBuf upload_csr(const HostCsr& h) {
  DevCsrBuf d;
  const size_t nnz = h.col.size();
  d.rowptr = dalloc<int>(h.rowptr.size());
  d.col = dalloc<int>(nnz);
  d.val = dalloc<double>(nnz);
  d.valf = dalloc<float>(nnz);
  std::vector<float> vf(h.val.begin(), h.val.end());
  HIPCHK(hipMemcpy(d.rowptr, h.rowptr.data(), h.rowptr.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d.col, h.col.data(), nnz * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d.val, h.val.data(), nnz * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d.valf, vf.data(), nnz * sizeof(float), hipMemcpyHostToDevice));
  return d;
}

DevSparse upload(const HostSparse& h, hipStream_t s) {
  DevSparse d;
  const size_t n = (size_t)h.n_out * h.width;
  d.col = dalloc<int>(n);
  d.val = dalloc<double>(n);
  d.valf = dalloc<float>(n);
  std::vector<float> vf(h.val.begin(), h.val.end());
  HIPCHK(hipMemcpy(d.col, h.col.data(), n * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d.val, h.val.data(), n * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d.valf, vf.data(), n * sizeof(float), hipMemcpyHostToDevice));
  d.s.n_out = h.n_out;
  d.s.n_in = h.n_in;
  d.s.width = h.width;
  d.s.col = d.col;
  d.s.val = d.val;
  d.s.valf = d.valf;
  return d;
}

// Largest eigenvalue of the symmetric tridiagonal (diag a, off b) by Sturm bisection.
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int n = (int)a.size();
  if (n == 0) return 1.0;
  double lo = a[0], hi = a[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < n - 1 ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  // count of eigenvalues < x
  auto count = [&](double x) {
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < n; ++i) {
      const double qq = (q == 0.0) ? 1e-300 : q;
      q = a[i] - x - b[i - 1] * b[i - 1] / qq;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count(mid) >= n) hi = mid;  // all eigenvalues below mid
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

template <typename T>
const T* level_qd(const Level& L);
template <>
const double* level_qd<double>(const Level& L) { return L.qd_ok ? L.qd : nullptr; }
template <>
const float* level_qd<float>(const Level& L) { return L.qd_ok ? L.qd32 : nullptr; }

template <typename T>
CellArgs<T> cell_args(mfpff_ctx* c, const Level& L, const T* lin, const T* x, T* y, T scale) {
  CellArgs<T> a{};
  a.g = L.g;
  a.m = MatParams{c->prob.lambda, c->prob.mu, c->prob.Gc, c->prob.eps, c->prob.kappa, c->prob.split};
  a.x = x;
  a.y = y;
  a.u = lin;
  a.phi = lin + (size_t)c->dim * L.nn;
  a.phit = lin + (size_t)(c->dim + 1) * L.nn;
  a.mask = L.mask;
  a.scale = scale;
  a.qd = level_qd<T>(L);
  a.mfma = c->prob.contraction == MFPFF_CONTRACT_MFMA;
  return a;
}

template <typename T>
const T* level_lin(mfpff_ctx* c, const Level& L);
template <>
const double* level_lin<double>(mfpff_ctx*, const Level& L) { return L.lin; }
template <>
const float* level_lin<float>(mfpff_ctx*, const Level& L) { return L.lin32; }
template <typename T>
const T* level_dinv(const Level& L);
template <>
const double* level_dinv<double>(const Level& L) { return L.dinv; }
template <>
const float* level_dinv<float>(const Level& L) { return L.dinv32; }
template <typename T>
const Tables<T>* tab(mfpff_ctx* c, int k);
template <>
const Tables<double>* tab<double>(mfpff_ctx* c, int k) { return c->tab64[k]; }
template <>
const Tables<float>* tab<float>(mfpff_ctx* c, int k) { return c->tab32[k]; }

// 2D owner-computes launch: row-shared cell kernel for Q1/Q2, LDS tile kernel otherwise
template <typename T>
void launch_2d(mfpff_ctx* c, const Level& L, int mode, int epi, const CellArgs<T>& a, const Epilogue<T>& e) {
  if (L.g.k <= 2) HIPCHK(launch_rowcell_2d<T>(mode, epi, a, e, c->s));
  else HIPCHK(launch_tile_2d<T>(mode, epi, a, e, tab<T>(c, L.g.k), c->s));
}

// one product with its epilogue: 2D owner-computes kernels; 3D cell kernel into the element
// buffer, then the node gather
template <typename T>
void launch_fused(mfpff_ctx* c, const Level& L, int mode, int epi, CellArgs<T> a, const Epilogue<T>& e) {
  if (L.g.slit) {
    // slit levels: the cell kernel computes at the Gauss points and scatters through the slit-aware
    // node map with atomics; the identity rows (and, for a residual, b) follow elementwise, then
    // the Chebyshev start or step (a step's product t = A_blk z is formed in z')
    k_fill<T>(e.y, T(0), L.n, c->s);
    a.y = e.y;
    a.qd = nullptr;
    a.elem = nullptr;
    HIPCHK(launch_cell<T>(mode, a, tab<T>(c, L.g.k), c->s));
    k_slit_epilogue<T>(e.y, a.x, epi == EPI_RESID ? e.b : nullptr, a.mask, L.nn, c->dim, c->s);
    if (epi == EPI_APPLY && e.xcopy) k_copy<T>(e.xcopy, a.x, L.n, c->s);
    if (epi == EPI_RESID && e.z0) k_cheb_init<T>(e.z0, e.d0, e.y, e.dinv, L.nn, c->dim, e.ith_u, e.ith_p, c->s);
    if (epi == EPI_CHEB)
      k_cheb_update<T>(e.y, e.d, a.x, e.r, e.y, e.dinv, L.nn, c->dim, e.c1u, e.c2u, e.c1p, e.c2p, e.xacc, e.xout, c->s);
    LAUNCHCHK();
    return;
  }
  if (c->dim == 2) {
    launch_2d<T>(c, L, mode, epi, a, e);
    return;
  }
  a.elem = (T*)c->elem;
  HIPCHK(launch_cell<T>(mode, a, tab<T>(c, L.g.k), c->s));
  HIPCHK(launch_gather_3d<T>(epi, (const T*)c->elem, a, e, c->s));
}

// residual R(u, phi; phi~) on the finest level into R (F.n values): in 3D the cell kernel writes
// the element buffer and the node gather adds the cell contributions of every node in a fixed
// order; in 2D the cell kernel adds them into R
void residual_launch(mfpff_ctx* c, const double* u, const double* phi, const double* pt, double* R) {
  Level& F = c->lv[c->L];
  CellArgs<double> a = cell_args<double>(c, F, F.lin, nullptr, R, 1.0);
  a.u = u;
  a.phi = phi;
  a.phit = pt;
  a.mask = nullptr;
  if (c->dim == 3 && !F.g.slit) {
    a.elem = (double*)c->elem;
    HIPCHK(launch_cell<double>(MODE_RESIDUAL, a, c->tab64[F.g.k], c->s));
    // the gather reads x at every node before it writes y there (same thread); with no mask
    // the value is not used, so R itself serves
    a.x = R;
    Epilogue<double> e{};
    e.y = R;
    HIPCHK(launch_gather_3d<double>(EPI_APPLY, (const double*)c->elem, a, e, c->s));
    return;
  }
  k_fill<double>(R, 0.0, F.n, c->s);
  HIPCHK(launch_cell<double>(MODE_RESIDUAL, a, c->tab64[F.g.k], c->s));
}

// y = op(G^) x on level l, or y = b - G^ x when b != null (op = G); xcopy (b null): also a copy
// of x, written by the product's epilogue;
// accumulate: y += P op(G) P x without initialising y (atomic cell kernel)
template <typename T>
void apply_op(mfpff_ctx* c, int l, int mode, const T* x, T* y, const T* b, bool accumulate = false, T* xcopy = nullptr) {
  Level& L = c->lv[l];
  const T scale = b ? T(-1) : T(1);
  CellArgs<T> a = cell_args<T>(c, L, level_lin<T>(c, L), x, y, scale);
  if (!accumulate) {
    Epilogue<T> e{};
    e.y = y;
    e.b = b;
    e.xcopy = b ? nullptr : xcopy;
    launch_fused<T>(c, L, mode, b ? EPI_RESID : EPI_APPLY, a, e);
    return;
  }
  HIPCHK(launch_cell<T>(mode, a, tab<T>(c, L.g.k), c->s));
}

// r = b - G^ x; with z0 != null also the Chebyshev start z0 = D^-1 r / theta, d0 = z0
template <typename T>
void op_resid(mfpff_ctx* c, int l, const T* b, const T* x, T* r, T* z0, T* d0) {
  Level& L = c->lv[l];
  CellArgs<T> a = cell_args<T>(c, L, level_lin<T>(c, L), x, r, T(-1));
  Epilogue<T> e{};
  e.y = r;
  e.b = b;
  e.z0 = z0;
  e.d0 = d0;
  e.dinv = level_dinv<T>(L);
  e.ith_u = (T)L.ith_u;
  e.ith_p = (T)L.ith_p;
  launch_fused<T>(c, L, MODE_APPLY, EPI_RESID, a, e);
}

// Chebyshev step i (1-based): zout = zin + d', d' = c1 d + c2 D^-1 (r - A_blk zin); optional xout = xacc + zout
template <typename T>
void op_cheb_step(mfpff_ctx* c, int l, int i, const T* zin, T* zout, const T* r, T* d, T* t, const T* xacc, T* xout) {
  Level& L = c->lv[l];
  const T c1u = (T)L.c1u[i - 1], c2u = (T)L.c2u[i - 1], c1p = (T)L.c1p[i - 1], c2p = (T)L.c2p[i - 1];
  CellArgs<T> a = cell_args<T>(c, L, level_lin<T>(c, L), zin, zout, T(1));
  Epilogue<T> e{};
  e.y = zout;
  e.dinv = level_dinv<T>(L);
  e.r = r;
  e.d = d;
  e.c1u = c1u;
  e.c2u = c2u;
  e.c1p = c1p;
  e.c2p = c2p;
  e.xacc = xacc;
  e.xout = xout;
  launch_fused<T>(c, L, MODE_BLOCK, EPI_CHEB, a, e);
}

// x = diag(C_u, C_phi) r (Chebyshev from zero); work vectors zA, zB, d, t (x distinct from them);
// started: the Chebyshev start z = d = D^-1 r / theta is already in (s == 1 ? x : zA) and d
template <typename T>
void chebyshev(mfpff_ctx* c, int l, const T* r, T* x, T* zA, T* zB, T* d, T* t, bool started = false) {
  Level& L = c->lv[l];
  const int s = c->prob.cheb_degree;
  T* zc = (s == 1) ? x : zA;
  if (!started) {
    k_cheb_init<T>(zc, d, r, level_dinv<T>(L), L.nn, c->dim, (T)L.ith_u, (T)L.ith_p, c->s);
    LAUNCHCHK();
  }
  for (int i = 1; i < s; ++i) {
    T* zn = (i == s - 1) ? x : (zc == zA ? zB : zA);
    op_cheb_step<T>(c, l, i, zc, zn, r, d, t, nullptr, nullptr);
    zc = zn;
  }
}

// x += diag(C_u, C_phi)(b - G^ x): residual with the fused Chebyshev start, then s-1 steps
template <typename T>
void post_smooth(mfpff_ctx* c, int l, const T* b, T* x, T* r, T* zA, T* zB, T* d, T* t) {
  Level& L = c->lv[l];
  const int s = c->prob.cheb_degree;
  op_resid<T>(c, l, b, x, r, zA, d);
  if (s == 1) {
    k_axpy<T>(x, T(1), zA, L.n, c->s);
    LAUNCHCHK();
    return;
  }
  T* zc = zA;
  for (int i = 1; i < s; ++i) {
    T* zn = zc == zA ? zB : zA;
    const bool last = i == s - 1;
    op_cheb_step<T>(c, l, i, zc, zn, r, d, t, last ? x : nullptr, last ? x : nullptr);
    zc = zn;
  }
}

// masked transfer between level l-1 and l; dir 0: out(level l) = P~ in (or += when add);
// dir 1: out(level l-1) = R~ in (axis passes, masks fused into the first and last pass)
template <typename T>
void transfer(mfpff_ctx* c, int l, int dir, const T* in, T* out, bool add, T* ta, T* tb,
              ChebStart<T> cs = ChebStart<T>{}) {
  Level& F = c->lv[l];
  Level& C = c->lv[l - 1];
  const int d = c->dim, nc = d + 1;
  if (F.g.slit) {
    // slit levels: the CSR prolongation or its transpose, masked on both sides
    if (dir == 0) {
      k_csr_transfer<T>(out, in, F.SP.view(), C.mask, F.mask, F.nn, C.nn, d, add, c->s);
    } else {
      k_csr_transfer<T>(out, in, F.SR.view(), F.mask, C.mask, C.nn, F.nn, d, false, c->s);
      if (cs.z0) k_cheb_init<T>(cs.z0, cs.d0, out, cs.dinv, C.nn, d, cs.ith_u, cs.ith_p, c->s);
    }
    LAUNCHCHK();
    return;
  }
  if (dir == 0 && d == 2 && F.P1.s.width <= 5) {
    k_prolong<T>(out, in, F.P1.s, C.mask, F.mask, F.g, C.g, add, c->s);
  } else if (dir == 0) {
    // 3D (and wide 2D rows): axis passes (coarse mask on the first, fine mask and accumulation
    // on the last)
    long long dims[3] = {C.g.M, C.g.M, C.g.M};
    const T* src = in;
    T* bufs[2] = {ta, tb};
    for (int ax = 0; ax < d; ++ax) {
      const bool first = ax == 0, last = ax == d - 1;
      T* o = last ? out : bufs[ax & 1];
      k_axis_apply<T>(o, src, F.P1.s, ax, d, dims, nc, first ? C.mask : nullptr, last ? F.mask : nullptr, c->s,
                      last && add);
      dims[ax] = F.g.M;
      src = o;
    }
  } else {
    long long dims[3] = {F.g.M, F.g.M, F.g.M};
    const T* src = in;
    T* bufs[2] = {ta, tb};
    for (int ax = 0; ax < d; ++ax) {
      const bool first = ax == 0, last = ax == d - 1;
      T* o = last ? out : bufs[ax & 1];
      k_axis_apply<T>(o, src, F.R1.s, ax, d, dims, nc, first ? F.mask : nullptr, last ? C.mask : nullptr, c->s, false,
                      last ? cs : ChebStart<T>{});
      dims[ax] = C.g.M;
      src = o;
    }
  }
  LAUNCHCHK();
}

// x = G^_0^-1 r by the block lower-triangular structure.  r in FP64 or FP32 (r32); the solution
// goes to x64 (FP64) and/or x32 (FP32, the FP32 V-cycle); without x64 the u part is kept in FP64
// in cs_out for the coupling product
void coarse_solve_any(mfpff_ctx* c, const void* r, bool r32, double* x64, float* x32) {
  const int nu = c->nu0, np = c->np0;
  double* xu = x64 ? x64 : c->cs_out;
  float* xu32 = x32;
  float* xp32 = x32 ? x32 + nu : nullptr;
  double* xp = x64 ? x64 + nu : nullptr;
  const void* rp = r32 ? (const void*)((const float*)r + nu) : (const void*)((const double*)r + nu);
  // W = L^-1 is lower triangular and W^T upper: each product reads only the stored triangle;
  // after the LU fallback W is the block's full inverse
  if (c->coarse_lu[0]) {
    k_gemv_mixed(xu, xu32, c->Wu, nu, r, r32, nu, nu, 1.0, nullptr, false, GEMV_FULL, c->s);
  } else {
    k_gemv_mixed(c->cs_t, nullptr, c->Wu, nu, r, r32, nu, nu, 1.0, nullptr, false, GEMV_LOWER, c->s);
    k_gemv_mixed(xu, xu32, c->WuT, nu, c->cs_t, false, nu, nu, 1.0, nullptr, false, GEMV_UPPER, c->s);
  }
  k_gemv_mixed(c->cs_t + nu, nullptr, c->Gpu, nu, xu, false, np, nu, -1.0, rp, r32, GEMV_FULL, c->s);
  if (c->coarse_lu[1]) {
    k_gemv_mixed(xp, xp32, c->Wp, np, c->cs_t + nu, false, np, np, 1.0, nullptr, false, GEMV_FULL, c->s);
  } else {
    k_gemv(c->cs_t, c->Wp, np, c->cs_t + nu, np, np, 1.0, nullptr, GEMV_LOWER, c->s);
    k_gemv_mixed(xp, xp32, c->WpT, np, c->cs_t, false, np, np, 1.0, nullptr, false, GEMV_UPPER, c->s);
  }
  LAUNCHCHK();
}

void coarse_solve64(mfpff_ctx* c, const double* r, double* x) { coarse_solve_any(c, r, false, x, nullptr); }

template <typename T>
void coarse_solve_T(mfpff_ctx* c, const T* r, T* x);
template <>
void coarse_solve_T<double>(mfpff_ctx* c, const double* r, double* x) {
  coarse_solve64(c, r, x);
}
// the FP32 V-cycle: FP32 right-hand side read and FP32 solution written by the FP64 products
template <>
void coarse_solve_T<float>(mfpff_ctx* c, const float* r, float* x) {
  coarse_solve_any(c, r, true, nullptr, x);
}

template <typename T>
void vcycle_rec(mfpff_ctx* c, int l, bool started = false) {
  Level& L = c->lv[l];
  T* b = (T*)L.w[WB];
  T* x = (T*)L.w[WX];
  if (l == 0) {
    coarse_solve_T<T>(c, b, x);
    return;
  }
  T* r = (T*)L.w[WR];
  T* t = (T*)L.w[WT];
  T* d = (T*)L.w[WD];
  T* zA = (T*)L.w[WZ];
  T* zB = (T*)L.w[WZ2];
  T* ta = std::is_same<T, double>::value ? (T*)c->t64a : (T*)c->t32a;
  T* tb = std::is_same<T, double>::value ? (T*)c->t64b : (T*)c->t32b;
  chebyshev<T>(c, l, b, x, zA, zB, d, t, started);
  op_resid<T>(c, l, b, x, r, (T*)nullptr, (T*)nullptr);
  // restriction; its last pass also writes the coarser level's Chebyshev start
  Level& C = c->lv[l - 1];
  const bool cstart = l - 1 > 0;
  ChebStart<T> cs;
  if (cstart) {
    cs.z0 = (T*)C.w[c->prob.cheb_degree == 1 ? WX : WZ];
    cs.d0 = (T*)C.w[WD];
    cs.dinv = level_dinv<T>(C);
    cs.ith_u = (T)C.ith_u;
    cs.ith_p = (T)C.ith_p;
  }
  transfer<T>(c, l, 1, r, (T*)C.w[WB], false, ta, tb, cs);
  vcycle_rec<T>(c, l - 1, cstart);
  transfer<T>(c, l, 0, (const T*)c->lv[l - 1].w[WX], x, true, ta, tb);
  post_smooth<T>(c, l, b, x, r, zA, zB, d, t);
}

// the finest level's Chebyshev start is written with its right-hand side (vstart)
void vcycle_body(mfpff_ctx* c) {
  if (c->f32) vcycle_rec<float>(c, c->L, c->L > 0);
  else vcycle_rec<double>(c, c->L, c->L > 0);
}

// where the V-cycle's input writes the finest level's Chebyshev start (none on one level)
VStart vstart(mfpff_ctx* c) {
  VStart v{};
  if (c->L == 0) return v;
  Level& F = c->lv[c->L];
  v.z0 = F.w[c->prob.cheb_degree == 1 ? WX : WZ];
  v.d0 = F.w[WD];
  v.dinv = c->f32 ? (const void*)F.dinv32 : (const void*)F.dinv;
  v.ith_u = F.ith_u;
  v.ith_p = F.ith_p;
  v.nu = (long long)c->dim * F.nn;
  return v;
}

// Record the V-cycle (finest WB and its Chebyshev start -> WX) into a graph on a private stream.  The
// launches only read level buffers, tables and coefficients that stay fixed
// until the next linearisation.  Any failure leaves the direct launch path.
void capture_vcycle(mfpff_ctx* c) {
  if (c->vgraph) {
    (void)hipGraphExecDestroy(c->vgraph);
    c->vgraph = nullptr;
  }
  if (!c->graph_ok) return;
  if (!c->cap_s && hipStreamCreateWithFlags(&c->cap_s, hipStreamNonBlocking) != hipSuccess) {
    c->graph_ok = false;
    return;
  }
  hipStream_t user = c->s;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(c->cap_s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    c->graph_ok = false;
    return;
  }
  c->s = c->cap_s;
  bool ok = true;
  try {
    vcycle_body(c);
  } catch (...) {
    ok = false;
  }
  c->s = user;
  if (hipStreamEndCapture(c->cap_s, &g) != hipSuccess || !g) ok = false;
  if (ok && hipGraphInstantiate(&c->vgraph, g, nullptr, nullptr, 0) != hipSuccess) {
    c->vgraph = nullptr;
    ok = false;
  }
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
  if (!ok) {
    c->graph_ok = false;
    c->vgraph = nullptr;
  }
}

// z = V(r) on the finest level, FP64 in/out; b_ready: the caller has already written r into the
// finest level's right-hand side and its Chebyshev start; z null (FP64 V-cycle only): the result
// stays in the finest level's x
void precondition(mfpff_ctx* c, const double* r, double* z, bool b_ready = false) {
  Level& F = c->lv[c->L];
  if (!b_ready) {
    k_vcycle_input(F.w[WB], c->f32, r, F.n, vstart(c), c->s);
    LAUNCHCHK();
  }
  if (c->vgraph) HIPCHK(hipGraphLaunch(c->vgraph, c->s));
  else vcycle_body(c);
  if (c->f32) k_cast_f2d(z, (const float*)F.w[WX], F.n, c->s);
  else if (z) k_copy<double>(z, (const double*)F.w[WX], F.n, c->s);
  LAUNCHCHK();
}

void cheb_coefficients(mfpff_ctx* c, Level& L) {
  const int s = c->prob.cheb_degree;
  L.c1u.clear();
  L.c2u.clear();
  L.c1p.clear();
  L.c2p.clear();
  double th[2], de[2], rho[2];
  for (int b = 0; b < 2; ++b) {
    const double lo = c->prob.cheb_lo * L.lam[b], hi = c->prob.cheb_hi * L.lam[b];
    th[b] = 0.5 * (hi + lo);
    de[b] = 0.5 * (hi - lo);
    rho[b] = de[b] / th[b];  // 1/sigma
  }
  L.ith_u = 1.0 / th[0];
  L.ith_p = 1.0 / th[1];
  for (int i = 1; i < s; ++i) {
    double c1[2], c2[2];
    for (int b = 0; b < 2; ++b) {
      const double sigma = th[b] / de[b];
      const double rn = 1.0 / (2.0 * sigma - rho[b]);
      c1[b] = rn * rho[b];
      c2[b] = 2.0 * rn / de[b];
      rho[b] = rn;
    }
    L.c1u.push_back(c1[0]);
    L.c2u.push_back(c2[0]);
    L.c1p.push_back(c1[1]);
    L.c2p.push_back(c2[1]);
  }
}

void lanczos_level(mfpff_ctx* c, int l) {
  Level& L = c->lv[l];
  const long long n = L.n, nu = (long long)c->dim * L.nn;
  double *v = c->s64[0], *r = c->s64[1], *z = c->s64[2], *p = c->s64[3], *t = c->s64[4];
  LanczosState* st = c->lst + l;
  const int nb = dot_blocks(n);
  k_splitmix_start(v, L.mask, L.nn, c->dim, c->prob.lanczos_seed, 2 * l, 2 * l + 1, c->s);
  k_copy<double>(r, v, n, c->s);
  k_lanczos_rz_partials(c->part, r, L.dinv, z, nu, n, c->s);
  k_lanczos_init(st, c->part, nb, c->s);
  k_copy<double>(p, z, n, c->s);
  for (int j = 0; j < c->prob.lanczos_steps; ++j) {
    apply_op<double>(c, l, MODE_BLOCK, p, t, nullptr);
    k_seg_dot_partials(c->part, p, t, nu, n, c->s);
    k_lanczos_alpha(st, c->part, nb, j, c->s);
    k_lanczos_update_r(r, z, c->part, t, L.dinv, st, nu, n, c->s);
    k_lanczos_beta(st, c->part, nb, j, c->s);
    k_lanczos_update_p(p, z, st, nu, n, c->s);
  }
  LAUNCHCHK();
}

constexpr long long kMaxCoarseDofs = 16384;

void coarse_alloc(mfpff_ctx* c) {
  if (c->dense) return;
  Level& C = c->lv[0];
  if (C.n > kMaxCoarseDofs)
    throw StatusError{MFPFF_ERR_ARG, "coarsest level too large for the dense coarse solve (more than 16384 dofs)"};
  const size_t n0 = (size_t)C.n;
  c->dense = dalloc<double>(n0 * n0);
  c->Auu = dalloc<double>((size_t)c->nu0 * c->nu0);
  c->App = dalloc<double>((size_t)c->np0 * c->np0);
  c->Wu = dalloc<double>((size_t)c->nu0 * c->nu0);
  c->WuT = dalloc<double>((size_t)c->nu0 * c->nu0);
  c->Wp = dalloc<double>((size_t)c->np0 * c->np0);
  c->WpT = dalloc<double>((size_t)c->np0 * c->np0);
  c->Gpu = dalloc<double>((size_t)c->np0 * c->nu0);
  c->cs_out = dalloc<double>(n0);
  c->cs_t = dalloc<double>(n0);
}

void coarse_setup(mfpff_ctx* c) {
  coarse_alloc(c);
  Level& C = c->lv[0];
  const long long n = C.n;
  HIPCHK(hipMemsetAsync(c->dense, 0, (size_t)n * n * sizeof(double), c->s));
  CellArgs<double> a = cell_args<double>(c, C, C.lin, nullptr, nullptr, 1.0);
  a.dense = c->dense;
  a.ld = n;
  HIPCHK(launch_cell<double>(MODE_ELEM, a, c->tab64[C.g.k], c->s));
  k_dense_set_fixed_diag(c->dense, n, C.mask, C.nn, c->dim, c->s);
  const int nu = c->nu0, np = c->np0;
  k_extract_block(c->Auu, nu, c->dense, n, 0, 0, nu, nu, c->s);
  k_extract_block(c->App, np, c->dense, n, nu, nu, np, np, c->s);
  k_extract_block(c->Gpu, nu, c->dense, n, nu, 0, np, nu, c->s);
  HIPCHK(hipMemsetAsync(c->info_dev, 0, 2 * sizeof(int), c->s));
  // fork: u and phi blocks factorised and inverted concurrently; coarse_join waits for both
  HIPCHK(hipEventRecord(c->ev_fork, c->s));
  double* A[2] = {c->Auu, c->App};
  double* W[2] = {c->Wu, c->Wp};
  double* WT[2] = {c->WuT, c->WpT};
  const int nb[2] = {nu, np};
  for (int b = 0; b < 2; ++b) {
    hipStream_t ss = c->side[b];
    HIPCHK(hipStreamWaitEvent(ss, c->ev_fork, 0));
    HIPCHK(cholesky_lower(A[b], nb[b], c->info_dev + b, c->chol_scratch + b * 32 * 32, ss));
    HIPCHK(tri_inverse_lower(W[b], A[b], nb[b], ss));
    k_transpose(WT[b], W[b], nb[b], ss);
    LAUNCHCHK();
    HIPCHK(hipEventRecord(c->ev_join[b], ss));
  }
}

void coarse_join(mfpff_ctx* c) {
  for (int b = 0; b < 2; ++b) HIPCHK(hipStreamWaitEvent(c->s, c->ev_join[b], 0));
}

// Blocks whose Cholesky met a non-positive pivot (failed[b] != 0): extracted again from the dense
// coarse operator and inverted by Gauss-Jordan with partial pivoting.  Only a zero pivot there
// (a singular block) is an error.
void coarse_lu_fallback(mfpff_ctx* c, const int* failed) {
  const int nu = c->nu0, np = c->np0;
  const long long n = c->lv[0].n;
  if (!c->lu_work) c->lu_work = dalloc<double>((size_t)std::max(nu, np) + 3);
  HIPCHK(hipMemsetAsync(c->info_dev, 0, 2 * sizeof(int), c->s));
  if (failed[0]) {
    k_extract_block(c->Auu, nu, c->dense, n, 0, 0, nu, nu, c->s);
    HIPCHK(gauss_jordan_inverse(c->Wu, c->Auu, nu, c->info_dev, c->lu_work, c->s));
  }
  if (failed[1]) {
    k_extract_block(c->App, np, c->dense, n, nu, nu, np, np, c->s);
    HIPCHK(gauss_jordan_inverse(c->Wp, c->App, np, c->info_dev + 1, c->lu_work, c->s));
  }
  int sing[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(sing, c->info_dev, 2 * sizeof(int), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  if (sing[0] || sing[1]) throw StatusError{MFPFF_ERR_NUMERIC, "coarse block is singular (zero pivot in the LU after the Cholesky failed)"};
  for (int b = 0; b < 2; ++b) c->coarse_lu[b] = failed[b] != 0;
}

// timing event owned for one scope (destroyed on every exit path, exceptions included)
struct ScopedEvent {
  hipEvent_t e = nullptr;
  ScopedEvent() { HIPCHK(hipEventCreate(&e)); }
  ~ScopedEvent() {
    if (e) (void)hipEventDestroy(e);
  }
  ScopedEvent(const ScopedEvent&) = delete;
  ScopedEvent& operator=(const ScopedEvent&) = delete;
};

void require_state(mfpff_ctx* c) {
  if (!c->linearized) throw StatusError{MFPFF_ERR_STATE, "set_linearization has not been called"};
}
void require_point(mfpff_ctx* c) {
  if (!c->has_point) throw StatusError{MFPFF_ERR_STATE, "neither set_point nor set_linearization has been called"};
}
void require_level(mfpff_ctx* c, int l) {
  if (l < 0 || l > c->L) throw StatusError{MFPFF_ERR_ARG, "level index out of range"};
}
void require_ptr(const void* p, const char* name) {
  if (!p) throw StatusError{MFPFF_ERR_ARG, std::string("null pointer: ") + name};
}

// Arnoldi result buffers: h1 at +0, h2 at +80, |w|^2 at +160 (restart <= 64)
constexpr int kHBuf = 240;
constexpr int kHostY = 2 * kHBuf;      // pinned staging of the least-squares solution
constexpr int kHostBeta = kHostY + 80;  // pinned staging of the residual norm
constexpr int kHostLen = kHostBeta + 8;

void ensure_gmres(mfpff_ctx* c) {
  if (c->V) return;
  const long long n = c->lv[c->L].n;
  c->m = c->prob.restart;
  // basis vectors 512-byte aligned (stride a multiple of 64 elements): the orthogonalisation
  // passes read them two elements per lane
  c->ldv = (n + 63) / 64 * 64;
  c->V = dalloc<double>((size_t)(c->m + 1) * c->ldv);
  c->Z = dalloc<double>((size_t)c->m * n);
  c->gw = dalloc<double>(n);
  c->gr = dalloc<double>(n);
  c->hdev = dalloc<double>(2 * kHBuf);
  c->ycoef = dalloc<double>(80);
  HIPCHK(hipHostMalloc((void**)&c->hhost, kHostLen * sizeof(double), hipHostMallocDefault));
  for (int b = 0; b < 2; ++b) HIPCHK(hipEventCreateWithFlags(&c->hev[b], hipEventDisableTiming));
}

double dev_norm(mfpff_ctx* c, const double* x, long long n, double* out_dev) {
  const int nb = dot_blocks(n);
  k_multidot_partials(c->part, x, n, 1, x, n, c->s);
  k_multidot_finish(out_dev, c->part, nb, 1, c->s);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(c->hhost, out_dev, sizeof(double), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  return std::sqrt(c->hhost[0]);
}

// Right-preconditioned FGMRES(m), CGS2, x0 = 0.
// The device work of Arnoldi step j+1 (normalisation, V-cycle, product,
// orthogonalisation) is queued before the host waits for the results of step j,
// so the GPU does not idle while the host applies the Givens rotations; when
// step j ends the cycle, the queued step only overwrites basis columns that are
// not used.
mfpff_status gmres(mfpff_ctx* c, const double* b, double* x, mfpff_solve_info* info) {
  ensure_gmres(c);
  const int m = c->m;
  const long long n = c->lv[c->L].n;
  const int nb = dot_blocks(n);
  k_fill<double>(x, 0.0, n, c->s);
  const double bnorm = dev_norm(c, b, n, c->hdev + 160);
  int it = 0;
  const double tol = c->prob.rtol * bnorm;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  double relres = 0.0;
  bool conv = false;
  if (bnorm == 0.0) {
    conv = true;
  }
  // v_j is written together with the V-cycle's right-hand side (FP32 for the mixed V-cycle) and
  // the finest level's Chebyshev start
  void* vb = c->lv[c->L].w[WB];
  const VStart vs = vstart(c);
  // step j: z_j = V(v_j), w = G^ z_j, the CGS2 sums against v_0..v_j into buffer j % 2 (the
  // second projection itself is applied when v_{j+1} is normalised), copied to the host
  auto arnoldi = [&](int j) {
    double* vj = c->V + (size_t)j * c->ldv;
    double* zj = c->Z + (size_t)j * n;
    double* hb = c->hdev + (j & 1) * kHBuf;
    double *h1 = hb, *h2 = hb + 80, *hn = hb + 160;
    if (c->f32) {
      precondition(c, vj, zj, true);
      apply_op<double>(c, c->L, MODE_APPLY, zj, c->gw, nullptr);
    } else {
      // the product reads z_j where the V-cycle left it and its epilogue stores the copy in Z
      precondition(c, vj, nullptr, true);
      apply_op<double>(c, c->L, MODE_APPLY, (const double*)c->lv[c->L].w[WX], c->gw, nullptr, false, zj);
    }
    if (j + 1 <= kOrthMax) {
      // two passes over V (each with all basis vectors at once): h1 = V^T w; w -= V h1 with
      // h2 = V^T w and |w|^2.  The second projection w -= V h2 is applied with the
      // normalisation of v_{j+1} (k_orth_normalize), |w - V h2|^2 = |w|^2 - |h2|^2
      k_orth_pass(0, c->gw, c->V, c->ldv, j + 1, nullptr, c->part, h1, n, c->s);
      k_orth_pass(3, c->gw, c->V, c->ldv, j + 1, h1, c->part, h2, n, c->s);
    } else {
      k_multidot_partials(c->part, c->V, c->ldv, j + 1, c->gw, n, c->s);
      k_multidot_finish(h1, c->part, nb, j + 1, c->s);
      k_maxpy_dev(c->gw, c->V, c->ldv, j + 1, h1, -1.0, n, c->s);
      k_multidot_partials(c->part, c->V, c->ldv, j + 1, c->gw, n, c->s);
      k_multidot_finish(h2, c->part, nb, j + 1, c->s);
      k_maxpy_dev(c->gw, c->V, c->ldv, j + 1, h2, -1.0, n, c->s);
      k_multidot_partials(c->part, c->gw, n, 1, c->gw, n, c->s);
      k_multidot_finish(hn, c->part, nb, 1, c->s);
    }
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(c->hhost + (j & 1) * kHBuf, hb, kHBuf * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipEventRecord(c->hev[j & 1], c->s));
  };
  while (!conv) {
    // r = b - G^ x
    apply_op<double>(c, c->L, MODE_APPLY, x, c->gr, b);
    const double beta = dev_norm(c, c->gr, n, c->hdev + 160);
    relres = beta / bnorm;
    if (beta <= tol) {
      conv = true;
      break;
    }
    if (it >= c->prob.max_iter) break;
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    c->hhost[kHostBeta] = beta;  // pinned staging, not a target of any device-to-host copy
    HIPCHK(hipMemcpyAsync(c->ycoef, &c->hhost[kHostBeta], sizeof(double), hipMemcpyHostToDevice, c->s));
    k_scale_dev(c->V, c->gr, c->ycoef, n, c->s, vb, c->f32, vs);
    arnoldi(0);
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      if (j + 1 < m) {
        // queue step j+1: v_{j+1} from w and the sums of step j in buffer j % 2
        double* hb = c->hdev + (j & 1) * kHBuf;
        if (j + 1 <= kOrthMax)
          k_orth_normalize(c->V + (size_t)(j + 1) * c->ldv, vb, c->f32, c->gw, c->V, c->ldv, j + 1, hb + 80, n, vs, c->s);
        else
          k_scale_rsqrt_dev(c->V + (size_t)(j + 1) * c->ldv, c->gw, hb + 160, n, c->s, vb, c->f32, vs);
        arnoldi(j + 1);
      }
      HIPCHK(hipEventSynchronize(c->hev[j & 1]));
      const double* hh = c->hhost + (j & 1) * kHBuf;
      double hnorm;
      if (j + 1 <= kOrthMax) {
        // |w - V h2| by Pythagoras, in the order the normalisation kernel takes
        double hn2 = hh[80 + j + 1];
        for (int i = 0; i <= j; ++i) hn2 -= hh[80 + i] * hh[80 + i];
        hnorm = hn2 > 0.0 ? std::sqrt(hn2) : 0.0;
      } else {
        hnorm = std::sqrt(hh[160]);
      }
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh[i] + hh[80 + i];
      H[(size_t)(j + 1) * m + j] = hnorm;
      for (int i = 0; i < j; ++i) {
        const double tmp = cs[i] * H[(size_t)i * m + j] + sn[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)(i + 1) * m + j] = -sn[i] * H[(size_t)i * m + j] + cs[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = tmp;
      }
      const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
      if (bb == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        const double rr = std::hypot(a, bb);
        cs[j] = a / rr;
        sn[j] = bb / rr;
      }
      H[(size_t)j * m + j] = cs[j] * a + sn[j] * bb;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      jend = j + 1;
      if (std::fabs(g[j + 1]) <= tol || it >= c->prob.max_iter || hnorm == 0.0) break;
    }
    for (int i = jend - 1; i >= 0; --i) {
      double sacc = g[i];
      for (int k = i + 1; k < jend; ++k) sacc -= H[(size_t)i * m + k] * y[k];
      y[i] = sacc / H[(size_t)i * m + i];
    }
    for (int i = 0; i < jend; ++i) c->hhost[kHostY + i] = y[i];
    HIPCHK(hipMemcpyAsync(c->ycoef, &c->hhost[kHostY], jend * sizeof(double), hipMemcpyHostToDevice, c->s));
    k_maxpy_dev(x, c->Z, n, jend, c->ycoef, 1.0, n, c->s);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(c->s));  // staging buffers are reused next cycle
  }
  if (info) {
    info->iterations = it;
    info->converged = conv ? 1 : 0;
    info->rel_residual = relres;
  }
  return conv ? MFPFF_OK : MFPFF_ERR_NOCONV;
}

// fields and masks on every level (FP32 copies too); checks the inputs are finite
void set_point(mfpff_ctx* c, const double* u, const double* phi, const double* phi_old, const uint8_t* active,
               const double* phit) {
  const int d = c->dim;
  Level& F = c->lv[c->L];
  c->has_point = false;
  c->linearized = false;
  k_fine_fields(F.lin, F.mask, u, phi, phit ? phit : phi_old, active, F.g, c->prob.dirichlet, c->s);
  LAUNCHCHK();
  for (int l = c->L - 1; l >= 0; --l) {
    k_inject(c->lv[l].lin, c->lv[l].mask, c->lv[l + 1].lin, c->lv[l + 1].mask, c->lv[l].g, c->lv[l + 1].g,
             c->prob.dirichlet, c->s);
    LAUNCHCHK();
  }
  if (c->f32)
    for (int l = 0; l <= c->L; ++l) k_cast_d2f(c->lv[l].lin32, c->lv[l].lin, (long long)(d + 2) * c->lv[l].nn, c->s);
  // tangent coefficients at the Gauss points of the 2D Q1/Q2 levels
  for (int l = 0; l <= c->L; ++l) {
    Level& L = c->lv[l];
    L.qd_ok = false;
    if (!L.qd) continue;
    CellArgs<double> a = cell_args<double>(c, L, L.lin, nullptr, nullptr, 1.0);
    a.qd_out = L.qd;
    if (d == 2) launch_2d<double>(c, L, MODE_QDATA, EPI_APPLY, a, Epilogue<double>{});
    else HIPCHK(launch_cell<double>(MODE_QDATA, a, c->tab64[L.g.k], c->s));
    if (L.qd32) {
      CellArgs<float> a32 = cell_args<float>(c, L, L.lin32, nullptr, nullptr, 1.0f);
      a32.qd_out = L.qd32;
      if (d == 2) launch_2d<float>(c, L, MODE_QDATA, EPI_APPLY, a32, Epilogue<float>{});
      else HIPCHK(launch_cell<float>(MODE_QDATA, a32, c->tab32[L.g.k], c->s));
    }
    L.qd_ok = true;
  }
  // finite check of the finest fields: sum of squares is finite unless some entry is inf or nan
  const long long nf = (long long)(d + 2) * F.nn;
  const int nb = dot_blocks(nf);
  k_multidot_partials(c->part, F.lin, nf, 1, F.lin, nf, c->s);
  k_multidot_finish(c->finite_flag, c->part, nb, 1, c->s);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(&c->hhost_scalar, c->finite_flag, sizeof(double), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  const double fl = c->hhost_scalar;
  if (!std::isfinite(fl)) throw StatusError{MFPFF_ERR_NUMERIC, "non-finite value in u, phi or phi_tilde"};
  c->has_point = true;
}

void set_linearization(mfpff_ctx* c, const double* u, const double* phi, const double* phi_old, const uint8_t* active,
                       const double* phit) {
  const int d = c->dim;
  set_point(c, u, phi, phi_old, active, phit);
  for (int l = 0; l <= c->L; ++l) {
    Level& L = c->lv[l];
    // diagonal
    double* tmp = c->s64[0];
    k_fill<double>(tmp, 0.0, L.n, c->s);
    CellArgs<double> a = cell_args<double>(c, L, L.lin, nullptr, tmp, 1.0);
    HIPCHK(launch_diag<double>(a, c->tab64[L.g.k], c->s));
    k_diag_finish<double>(L.dinv, L.diag, tmp, L.mask, L.nn, d, c->s);
    if (c->f32) k_cast_d2f(L.dinv32, L.dinv, L.n, c->s);
    LAUNCHCHK();
  }
  coarse_setup(c);  // forks the dense factorisations onto the side streams
  for (int l = 1; l <= c->L; ++l) lanczos_level(c, l);
  coarse_join(c);
  // read back Lanczos scalars and the factorisation status
  std::vector<LanczosState> hs(c->L + 1);
  HIPCHK(hipMemcpyAsync(hs.data(), c->lst, (c->L + 1) * sizeof(LanczosState), hipMemcpyDeviceToHost, c->s));
  int info[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(info, c->info_dev, 2 * sizeof(int), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  c->coarse_lu[0] = c->coarse_lu[1] = false;
  if (info[0] || info[1]) coarse_lu_fallback(c, info);
  for (int l = 1; l <= c->L; ++l) {
    Level& L = c->lv[l];
    for (int b = 0; b < 2; ++b) {
      const int cnt = hs[l].count[b];
      std::vector<double> dg(cnt), off(cnt > 0 ? cnt - 1 : 0);
      for (int j = 0; j < cnt; ++j) {
        const double al = hs[l].alphas[b][j];
        dg[j] = 1.0 / al + (j > 0 ? hs[l].betas[b][j - 1] / hs[l].alphas[b][j - 1] : 0.0);
        if (j < cnt - 1) off[j] = std::sqrt(hs[l].betas[b][j]) / al;
      }
      L.lam[b] = cnt == 0 ? 1.0 : (cnt == 1 ? dg[0] : tridiag_max_eig(dg, off));
      L.lsteps[b] = cnt;
    }
    cheb_coefficients(c, L);
  }
  capture_vcycle(c);
  c->linearized = true;
}

}  // namespace

// Static scratch of mfpff_residual_param_vjp_noalloc: the per-block partial sums of the
// parameter-cotangent kernel (two doubles per block, at most kNoAllocMaxBlocks blocks) followed by
// the two totals.  Every device the library runs on holds one copy (2 MiB) until the process
// ends.  Host code never passes the name `scratch` to a kernel or a copy (on the host it is a
// stand-in, not a device address): mfpff_setup_mesh_levels resolves its device address once per
// device with hipGetSymbolAddress, and the entry point uses that address.
namespace {
constexpr long long kNoAllocMaxBlocks = 1LL << 17;
constexpr int kNoAllocMaxDevices = 64;
}  // namespace
static __device__ __align__(256) double scratch[2 * kNoAllocMaxBlocks + 2];
namespace {
std::mutex g_scratch_mu;
double* g_scratch_dev[kNoAllocMaxDevices] = {};

// Resolve the device address of `scratch` on device `dev` (the current device) once.
hipError_t noalloc_scratch_init(int dev) {
  if (dev < 0 || dev >= kNoAllocMaxDevices) return hipSuccess;  // the no-alloc entry point then refuses
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_dev[dev] = static_cast<double*>(ptr);
  return hipSuccess;
}

double* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_dev[dev];
}
}  // namespace

namespace {
mfpff_status run(mfpff_ctx* c, const std::function<mfpff_status()>& fn) {
  if (!c) return MFPFF_ERR_ARG;
  try {
    c->err.clear();
    return fn();
  } catch (const StatusError& e) {
    c->err = e.msg;
    return e.st;
  } catch (const HipError& e) {
    c->err = std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.what;
    return MFPFF_ERR_HIP;
  } catch (const std::exception& e) {
    c->err = e.what();
    return MFPFF_ERR_ARG;
  }
}
}  // namespace

namespace {
// Parameter cotangents <v, dR/dGc>, <v, dR/deps> of eq. (residual) on the finest level: the cell
// kernel writes two partial sums per block into `partials`, one workgroup adds them in a fixed
// order into out2[0..1], and the pair is copied to the host (synchronises the stream).
void param_vjp(mfpff_ctx* c, const double* u, const double* phi, const double* phi_tilde, const double* v,
               double* partials, double* out2d, double* dGc_host, double* deps_host) {
  require_ptr(phi, "phi");
  require_ptr(v, "v");
  require_ptr(dGc_host, "dGc_host");
  require_ptr(deps_host, "deps_host");
  Level& F = c->lv[c->L];
  CellArgs<double> a = cell_args<double>(c, F, F.lin, v, nullptr, 1.0);
  a.u = u;
  a.phi = phi;
  a.phit = phi_tilde;
  a.mask = nullptr;
  a.partials = partials;
  HIPCHK(launch_cell<double>(MODE_PVJP, a, c->tab64[F.g.k], c->s));
  const long long nb = cell_blocks(F.g, MODE_PVJP);
  k_sum_pvjp(out2d, partials, (int)nb, c->s);
  LAUNCHCHK();
  double out2[2];
  HIPCHK(hipMemcpyAsync(out2, out2d, 2 * sizeof(double), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  *dGc_host = out2[0];
  *deps_host = out2[1];
}
}  // namespace

// per-file counters of the bounds-checking build (bounds.h)
#ifdef MFPFF_BOUNDS
namespace mfpff {
unsigned int bounds_hits_cell();
unsigned int bounds_hits_linecell();
unsigned int bounds_hits_mfma();
unsigned int bounds_hits_rowcell();
unsigned int bounds_hits_tile();
unsigned int bounds_hits_transfer();
unsigned int bounds_hits_vector();
}  // namespace mfpff
#endif

extern "C" {

mfpff_status mfpff_setup_mesh_levels(const mfpff_problem* prob, void* hip_stream, mfpff_ctx** out) {
  if (!prob || !out) return MFPFF_ERR_ARG;
  *out = nullptr;
  const mfpff_problem& p = *prob;
  if (p.dim != 2 && p.dim != 3) return MFPFF_ERR_ARG;
  if (p.n_levels < 1 || p.n_levels > MFPFF_MAX_LEVELS) return MFPFF_ERR_ARG;
  if (p.cheb_degree < 1 || p.cheb_degree > 32 || p.lanczos_steps < 0 || p.lanczos_steps > 64) return MFPFF_ERR_ARG;
  if (p.restart < 1 || p.restart > 64 || p.max_iter < 0 || !(p.rtol >= 0.0)) return MFPFF_ERR_ARG;
  if (p.vcycle_prec != MFPFF_F64 && p.vcycle_prec != MFPFF_F32) return MFPFF_ERR_ARG;
  if (p.split != MFPFF_SPLIT_AMOR && p.split != MFPFF_SPLIT_MIEHE && p.split != MFPFF_SPLIT_NONE) return MFPFF_ERR_ARG;
  if (p.pdas_project != 0 && p.pdas_project != 1) return MFPFF_ERR_ARG;
  if (p.contraction != MFPFF_CONTRACT_VALU && p.contraction != MFPFF_CONTRACT_MFMA) return MFPFF_ERR_ARG;
  // the slit geometry: an even cell count on every level (the slit ends at a node)
  if (p.slit != 0 && p.slit != 1) return MFPFF_ERR_ARG;
  for (int l = 0; p.slit && l < p.n_levels; ++l)
    if (p.level_N[l] % 2 != 0) return MFPFF_ERR_ARG;
  if (!(p.eps > 0.0) || !(p.kappa > -1.0 && p.kappa < 1.0) || !(p.cheb_hi > p.cheb_lo) || !(p.cheb_lo > 0.0)) return MFPFF_ERR_ARG;
  for (int l = 0; l < p.n_levels; ++l) {
    if (p.level_N[l] < 1 || p.level_k[l] < 1 || p.level_k[l] > kMaxDeg) return MFPFF_ERR_ARG;
    if (l > 0) {
      const int Nc = p.level_N[l - 1], kc = p.level_k[l - 1], Nf = p.level_N[l], kf = p.level_k[l];
      const bool hstep = (Nf == 2 * Nc && kf == kc);
      const bool pstep = (Nf == Nc && kf > kc && kf % kc == 0);
      if (!hstep && !pstep) return MFPFF_ERR_ARG;
    }
  }
  mfpff_ctx* c = new mfpff_ctx();
  c->prob = p;
  c->s = (hipStream_t)hip_stream;
  c->dim = p.dim;
  c->L = p.n_levels - 1;
  c->f32 = p.vcycle_prec == MFPFF_F32;
  if (const char* ev = getenv("MFPFF_NO_GRAPH")) c->graph_ok = !(ev[0] == '1');
  mfpff_status st = run(c, [&]() -> mfpff_status {
    const int d = c->dim;
    HIPCHK(hipGetDevice(&c->device));
    HIPCHK(noalloc_scratch_init(c->device));
    c->lv.resize(p.n_levels);
    size_t elem_bytes = 0;
    for (int l = 0; l < p.n_levels; ++l) {
      Level& L = c->lv[l];
      L.g = make_geom(d, p.level_N[l], p.level_k[l], p.slit);
      L.nn = L.g.n_nodes;
      L.n = (long long)(d + 1) * L.nn;
      if (L.n >= (1LL << 31)) throw StatusError{MFPFF_ERR_ARG, "a level with 2^31 or more dofs is not supported"};
      // the 2D Q1/Q2 kernel addresses nodes by 32-bit byte offsets
      if (d == 2 && L.g.k <= 2 && L.nn >= (1LL << 28))
        throw StatusError{MFPFF_ERR_ARG, "a 2D Q1/Q2 level with 2^28 or more nodes is not supported"};
      L.lin = dalloc<double>((size_t)(d + 2) * L.nn);
      L.mask = dalloc<uint8_t>(L.nn);
      L.dinv = dalloc<double>(L.n);
      L.diag = dalloc<double>(L.n);
      if (c->f32) {
        L.lin32 = dalloc<float>((size_t)(d + 2) * L.nn);
        L.dinv32 = dalloc<float>(L.n);
      }
      if (d == 3) {
        const size_t eb = (size_t)elem_len(L.g) * sizeof(double);
        if (eb > elem_bytes) elem_bytes = eb;
      }
      if (((d == 2 && L.g.k <= 2) || d == 3) && !p.slit) {
        const size_t nq = (size_t)(d == 2 ? rowcell_qdata_len(L.g, p.split) : cell_qdata_len(L.g, p.split));
        L.qd = dalloc<double>(nq);
        if (c->f32) L.qd32 = dalloc<float>(nq);
      }
      const size_t es = c->f32 ? sizeof(float) : sizeof(double);
      for (int w = 0; w < NW; ++w) {
        void* ptr = nullptr;
        if (hipMalloc(&ptr, (size_t)L.n * es) != hipSuccess) throw StatusError{MFPFF_ERR_OOM, "device allocation failed"};
        L.w[w] = ptr;
      }
      if (l > 0) {
        HostSparse P, R;
        build_transfer(L.g, c->lv[l - 1].g, P, R);
        L.P1 = upload(P, c->s);
        L.R1 = upload(R, c->s);
        if (p.slit) {
          const long long nnz = (long long)L.nn * (long long)std::pow((double)P.width, d);
          if (nnz >= (1LL << 31)) throw StatusError{MFPFF_ERR_ARG, "slit level too large for its CSR transfer"};
          const HostCsr SP = build_slit_prolongation(L.g, c->lv[l - 1].g, P);
          L.SP = upload_csr(SP);
          L.SR = upload_csr(csr_transpose(SP));
        }
      }
      const int k = L.g.k;
      if (!c->tab64[k]) {
        Tables<double> t{};
        make_tables(k, t);
        Tables<float> tf{};
        for (int i = 0; i <= kMaxDeg; ++i) {
          tf.w[i] = (float)t.w[i];
          for (int j = 0; j <= kMaxDeg; ++j) {
            tf.B[i][j] = (float)t.B[i][j];
            tf.D[i][j] = (float)t.D[i][j];
            tf.C[i][j] = (float)t.C[i][j];
          }
        }
        c->tab64[k] = dalloc<Tables<double>>(1);
        c->tab32[k] = dalloc<Tables<float>>(1);
        HIPCHK(hipMemcpy(c->tab64[k], &t, sizeof(t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->tab32[k], &tf, sizeof(tf), hipMemcpyHostToDevice));
      }
    }
    if (elem_bytes) c->elem = dalloc<char>(elem_bytes);
    Level& F = c->lv[c->L];
    const long long nF = F.n;
    c->t64a = dalloc<double>(nF);
    c->t64b = dalloc<double>(nF);
    if (c->f32) {
      c->t32a = dalloc<float>(nF);
      c->t32b = dalloc<float>(nF);
    }
    for (int i = 0; i < 5; ++i) c->s64[i] = dalloc<double>(nF);
    c->part_len = 512 * 80;
    c->part = dalloc<double>(c->part_len);
    c->lst = dalloc<LanczosState>(c->L + 1);
    HIPCHK(hipMemset(c->lst, 0, (c->L + 1) * sizeof(LanczosState)));
    // coarse sizes (storage is allocated by the first full linearisation)
    Level& C = c->lv[0];
    c->nu0 = (int)(d * C.nn);
    c->np0 = (int)C.nn;
    c->info_dev = dalloc<int>(2);
    c->chol_scratch = dalloc<double>(2 * 32 * 32);
    for (int b = 0; b < 2; ++b) {
      if (hipStreamCreateWithFlags(&c->side[b], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&c->ev_join[b], hipEventDisableTiming) != hipSuccess)
        throw StatusError{MFPFF_ERR_HIP, "stream or event creation failed"};
    }
    if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess)
      throw StatusError{MFPFF_ERR_HIP, "event creation failed"};
    c->finite_flag = dalloc<double>(1);
    // lumped mass on the finest level: integrals of the 1D basis functions
    Tables<double> t{};
    make_tables(F.g.k, t);
    double w1[kMaxDeg + 1] = {};
    for (int i = 0; i <= F.g.k; ++i)
      for (int q = 0; q <= F.g.k; ++q) w1[i] += t.w[q] * t.B[q][i];
    c->w1d = dalloc<double>(kMaxDeg + 1);
    HIPCHK(hipMemcpy(c->w1d, w1, sizeof(w1), hipMemcpyHostToDevice));
    c->ml = dalloc<double>(F.nn);
    k_lumped_mass(c->ml, F.g, c->w1d, c->s);
    c->R = dalloc<double>(nF);
    c->b = dalloc<double>(nF);
    c->dU = dalloc<double>(nF);
    const long long pb = cell_blocks(F.g, MODE_PVJP);
    c->pvjp_part = dalloc<double>((size_t)2 * pb);
    c->pvjp_out = dalloc<double>(2);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(c->s));
    return MFPFF_OK;
  });
  if (st != MFPFF_OK) {
    fprintf(stderr, "mfpff_setup_mesh_levels: %s\n", c->err.c_str());
    mfpff_destroy(c);
    return st;
  }
  *out = c;
  return MFPFF_OK;
}

void mfpff_destroy(mfpff_ctx* c) {
  if (!c) return;
  if (c->s) (void)hipStreamSynchronize(c->s);
  else (void)hipDeviceSynchronize();
  for (auto ss : c->side)
    if (ss) (void)hipStreamSynchronize(ss);
  auto F = [](void* p) {
    if (p) (void)hipFree(p);
  };
  for (auto& L : c->lv) {
    F(L.lin);
    F(L.lin32);
    F(L.qd);
    F(L.qd32);
    F(L.mask);
    F(L.dinv);
    F(L.dinv32);
    F(L.diag);
    for (auto w : L.w) F(w);
    F(L.P1.col);
    F(L.P1.val);
    F(L.P1.valf);
    F(L.R1.col);
    F(L.R1.val);
    F(L.R1.valf);
    for (DevCsrBuf* b : {&L.SP, &L.SR}) {
      F(b->rowptr);
      F(b->col);
      F(b->val);
      F(b->valf);
    }
  }
  for (int k = 0; k <= kMaxDeg; ++k) {
    F(c->tab64[k]);
    F(c->tab32[k]);
  }
  void* ps[] = {c->elem, c->finite_flag, c->w1d, c->ml, c->t64a, c->t64b, c->t32a, c->t32b, c->dense, c->Auu, c->App, c->Wu, c->WuT, c->Wp,
                c->WpT, c->Gpu, c->cs_out, c->cs_t, c->info_dev, c->chol_scratch, c->lu_work, c->lst, c->part, c->V,
                c->Z, c->gw, c->gr, c->hdev, c->ycoef, c->R, c->b, c->dU, c->pvjp_part, c->pvjp_out, c->act_prev, c->pdas_part,
                c->phit_ext, c->react};
  for (void* p : ps) F(p);
  for (int i = 0; i < 5; ++i) F(c->s64[i]);
  if (c->hhost) (void)hipHostFree(c->hhost);
  for (auto e : c->hev)
    if (e) (void)hipEventDestroy(e);
  if (c->vgraph) (void)hipGraphExecDestroy(c->vgraph);
  if (c->cap_s) (void)hipStreamDestroy(c->cap_s);
  for (int b = 0; b < 2; ++b) {
    if (c->side[b]) (void)hipStreamDestroy(c->side[b]);
    if (c->ev_join[b]) (void)hipEventDestroy(c->ev_join[b]);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  delete c;
}

const char* mfpff_last_error(const mfpff_ctx* c) { return c ? c->err.c_str() : "null context"; }

long long mfpff_debug_bounds_hits(void) {
#ifdef MFPFF_BOUNDS
  using namespace mfpff;
  if (hipDeviceSynchronize() != hipSuccess) return -2;
  const unsigned int h[] = {bounds_hits_cell(), bounds_hits_linecell(), bounds_hits_mfma(), bounds_hits_rowcell(),
                            bounds_hits_tile(), bounds_hits_transfer(), bounds_hits_vector()};
  long long sum = 0;
  for (unsigned int v : h) {
    if (v == ~0u) return -2;
    sum += v;
  }
  return sum;
#else
  return -1;
#endif
}

mfpff_status mfpff_sizes(const mfpff_ctx* c, int level, size_t* n_nodes, size_t* n_dofs) {
  if (!c || !n_nodes || !n_dofs || level < 0 || level > c->L) return MFPFF_ERR_ARG;
  *n_nodes = (size_t)c->lv[level].nn;
  *n_dofs = (size_t)c->lv[level].n;
  return MFPFF_OK;
}

mfpff_status mfpff_level_info(mfpff_ctx* c, int level, mfpff_level_desc* out) {
  return run(c, [&]() {
    require_level(c, level);
    require_ptr(out, "out");
    const Level& L = c->lv[level];
    out->N = L.g.N;
    out->k = L.g.k;
    out->n_nodes = L.nn;
    out->n_dofs = L.n;
    out->lambda_u = L.lam[0];
    out->lambda_phi = L.lam[1];
    out->lanczos_steps_u = L.lsteps[0];
    out->lanczos_steps_phi = L.lsteps[1];
    return MFPFF_OK;
  });
}

mfpff_status mfpff_set_linearization(mfpff_ctx* c, const double* u, const double* phi, const double* phi_old,
                                     const uint8_t* active, const double* phi_tilde) {
  return run(c, [&]() {
    require_ptr(u, "u");
    require_ptr(phi, "phi");
    require_ptr(phi_old, "phi_old");
    require_ptr(active, "active");
    set_linearization(c, u, phi, phi_old, active, phi_tilde);
    return MFPFF_OK;
  });
}

mfpff_status mfpff_set_point(mfpff_ctx* c, const double* u, const double* phi, const double* phi_old,
                             const uint8_t* active, const double* phi_tilde) {
  return run(c, [&]() {
    require_ptr(u, "u");
    require_ptr(phi, "phi");
    require_ptr(phi_old, "phi_old");
    require_ptr(active, "active");
    set_point(c, u, phi, phi_old, active, phi_tilde);
    return MFPFF_OK;
  });
}

mfpff_status mfpff_apply_jacobian(mfpff_ctx* c, int level, const void* x, void* y, int prec, int op) {
  return run(c, [&]() {
    require_point(c);
    require_level(c, level);
    require_ptr(x, "x");
    require_ptr(y, "y");
    if (x == y) throw StatusError{MFPFF_ERR_ARG, "x and y alias"};
    int mode;
    const bool acc = (op & MFPFF_OP_ACCUMULATE) != 0;
    const int base = op & ~MFPFF_OP_ACCUMULATE;
    if (base == MFPFF_OP_G) mode = MODE_APPLY;
    else if (base == MFPFF_OP_GT) mode = MODE_APPLY_T;
    else if (base == MFPFF_OP_BLOCKDIAG) mode = MODE_BLOCK;
    else throw StatusError{MFPFF_ERR_ARG, "unknown operator"};
    if (prec == MFPFF_F64) {
      apply_op<double>(c, level, mode, (const double*)x, (double*)y, nullptr, acc);
    } else if (prec == MFPFF_F32) {
      if (!c->f32) throw StatusError{MFPFF_ERR_ARG, "FP32 level data exist only with an FP32 V-cycle"};
      apply_op<float>(c, level, mode, (const float*)x, (float*)y, nullptr, acc);
    } else {
      throw StatusError{MFPFF_ERR_ARG, "unknown precision"};
    }
    return MFPFF_OK;
  });
}

mfpff_status mfpff_diagonal(mfpff_ctx* c, int level, double* diag) {
  return run(c, [&]() {
    require_state(c);
    require_level(c, level);
    require_ptr(diag, "diag");
    k_copy<double>(diag, c->lv[level].diag, c->lv[level].n, c->s);
    LAUNCHCHK();
    return MFPFF_OK;
  });
}

mfpff_status mfpff_element_matrices(mfpff_ctx* c, int level, double* em) {
  return run(c, [&]() {
    require_point(c);
    require_level(c, level);
    require_ptr(em, "em");
    Level& L = c->lv[level];
    CellArgs<double> a = cell_args<double>(c, L, L.lin, nullptr, nullptr, 1.0);
    a.mask = nullptr;  // unconstrained
    a.qd = nullptr;
    a.elem_mat = em;
    HIPCHK(launch_cell<double>(MODE_ELEM, a, c->tab64[L.g.k], c->s));
    return MFPFF_OK;
  });
}

mfpff_status mfpff_smooth(mfpff_ctx* c, int level, const double* r, double* z) {
  return run(c, [&]() {
    require_state(c);
    require_level(c, level);
    if (level < 1) throw StatusError{MFPFF_ERR_ARG, "the coarsest level has no smoother"};
    require_ptr(r, "r");
    require_ptr(z, "z");
    if (r == z) throw StatusError{MFPFF_ERR_ARG, "r and z alias"};
    chebyshev<double>(c, level, r, z, c->s64[0], c->s64[1], c->s64[2], c->s64[3]);
    return MFPFF_OK;
  });
}

mfpff_status mfpff_transfer(mfpff_ctx* c, int level, int direction, const double* in, double* out) {
  return run(c, [&]() {
    require_level(c, level);
    if (level < 1) throw StatusError{MFPFF_ERR_ARG, "transfer needs level >= 1"};
    if (direction != 0 && direction != 1) throw StatusError{MFPFF_ERR_ARG, "direction must be 0 or 1"};
    require_state(c);
    require_ptr(in, "in");
    require_ptr(out, "out");
    transfer<double>(c, level, direction, in, out, false, c->t64a, c->t64b);
    return MFPFF_OK;
  });
}

mfpff_status mfpff_coarse_solve(mfpff_ctx* c, const double* r, double* x) {
  return run(c, [&]() {
    require_state(c);
    require_ptr(r, "r");
    require_ptr(x, "x");
    coarse_solve64(c, r, x);
    return MFPFF_OK;
  });
}

mfpff_status mfpff_vcycle(mfpff_ctx* c, const double* r, double* z) {
  return run(c, [&]() {
    require_state(c);
    require_ptr(r, "r");
    require_ptr(z, "z");
    precondition(c, r, z);
    return MFPFF_OK;
  });
}

mfpff_status mfpff_gmres_solve(mfpff_ctx* c, const double* b, double* x, mfpff_solve_info* info) {
  return run(c, [&]() {
    require_state(c);
    require_ptr(b, "b");
    require_ptr(x, "x");
    ScopedEvent e0, e1;
    HIPCHK(hipEventRecord(e0.e, c->s));
    mfpff_solve_info loc{};
    mfpff_status st = gmres(c, b, x, &loc);
    HIPCHK(hipEventRecord(e1.e, c->s));
    HIPCHK(hipEventSynchronize(e1.e));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0.e, e1.e));
    loc.ms_solve = ms;
    if (info) *info = loc;
    if (st == MFPFF_ERR_NOCONV) c->err = "GMRES reached max_iter";
    return st;
  });
}

mfpff_status mfpff_residual(mfpff_ctx* c, const double* u, const double* phi, const double* phi_tilde, double* R) {
  return run(c, [&]() {
    require_ptr(u, "u");
    require_ptr(phi, "phi");
    require_ptr(phi_tilde, "phi_tilde");
    require_ptr(R, "R");
    residual_launch(c, u, phi, phi_tilde, R);
    return MFPFF_OK;
  });
}

mfpff_status mfpff_residual_param_vjp(mfpff_ctx* c, const double* u, const double* phi, const double* phi_tilde,
                                      const double* v, double* dGc_host, double* deps_host) {
  return run(c, [&]() {
    param_vjp(c, u, phi, phi_tilde, v, c->pvjp_part, c->pvjp_out, dGc_host, deps_host);
    return MFPFF_OK;
  });
}

mfpff_status mfpff_residual_param_vjp_noalloc(mfpff_ctx* c, const double* u, const double* phi,
                                              const double* phi_tilde, const double* v, double* dGc_host,
                                              double* deps_host) {
  return run(c, [&]() {
    const long long nb = cell_blocks(c->lv[c->L].g, MODE_PVJP);
    if (nb > kNoAllocMaxBlocks)
      throw StatusError{MFPFF_ERR_ARG, "mfpff_residual_param_vjp_noalloc: the finest level needs " +
                                           std::to_string(nb) + " partial-sum blocks, the static scratch holds " +
                                           std::to_string(kNoAllocMaxBlocks)};
    double* sp = noalloc_scratch(c->device);
    if (!sp) throw StatusError{MFPFF_ERR_STATE, "mfpff_residual_param_vjp_noalloc: no static scratch on this device"};
    param_vjp(c, u, phi, phi_tilde, v, sp, sp + 2 * kNoAllocMaxBlocks, dGc_host, deps_host);
    return MFPFF_OK;
  });
}

mfpff_status mfpff_active_set(mfpff_ctx* c, const double* R, const double* phi, const double* phi_old, uint8_t* active) {
  return run(c, [&]() {
    require_ptr(R, "R");
    require_ptr(phi, "phi");
    require_ptr(phi_old, "phi_old");
    require_ptr(active, "active");
    Level& F = c->lv[c->L];
    k_active_set(active, R, phi, phi_old, c->ml, F.nn, c->dim, c->prob.as_c, c->s);
    LAUNCHCHK();
    return MFPFF_OK;
  });
}

}  // extern "C"

namespace {
// residual at (u, phi; phi~) into c->R
static void residual_into_R(mfpff_ctx* c, const double* u, const double* phi, const double* pt) {
  residual_launch(c, u, phi, pt, c->R);
}

// residual at (u, phi; phi~) into c->R and the active set of Algorithm 1 from it
static void residual_and_active(mfpff_ctx* c, const double* u, const double* phi, const double* phi_old, const double* pt,
                                uint8_t* active) {
  Level& F = c->lv[c->L];
  residual_into_R(c, u, phi, pt);
  k_active_set(active, c->R, phi, phi_old, c->ml, F.nn, c->dim, c->prob.as_c, c->s);
  LAUNCHCHK();
}

// linearise at (u, phi, active), solve G^ dU = -P R (R in c->R), update u and phi; fills
// iterations, residual and times of *loc.  With pdas_project, phi := phi_old on the active set
// first and R is evaluated again there, so that delta phi = 0 on A keeps the iterate on the
// obstacle.
static mfpff_status linearise_solve_update(mfpff_ctx* c, double* u, double* phi, const double* phi_old, const double* pt,
                                           const uint8_t* active, hipEvent_t e0, mfpff_solve_info* loc) {
  Level& F = c->lv[c->L];
  const int d = c->dim;
  ScopedEvent e1, e2;
  c->linearized = false;
  if (c->prob.pdas_project) {
    k_project_active(phi, phi_old, active, F.nn, c->s);
    LAUNCHCHK();
    residual_into_R(c, u, phi, pt);
  }
  set_linearization(c, u, phi, phi_old, active, pt);
  HIPCHK(hipEventRecord(e1.e, c->s));
  // b = -P R
  k_copy<double>(c->b, c->R, F.n, c->s);
  k_mask_vec(c->b, F.mask, F.nn, d, -1.0, c->s);
  LAUNCHCHK();
  mfpff_status st = gmres(c, c->b, c->dU, loc);
  k_axpy<double>(u, 1.0, c->dU, (long long)d * F.nn, c->s);
  k_axpy<double>(phi, 1.0, c->dU + (size_t)d * F.nn, F.nn, c->s);
  LAUNCHCHK();
  HIPCHK(hipEventRecord(e2.e, c->s));
  HIPCHK(hipEventSynchronize(e2.e));
  float ms1 = 0, ms2 = 0;
  HIPCHK(hipEventElapsedTime(&ms1, e0, e1.e));
  HIPCHK(hipEventElapsedTime(&ms2, e1.e, e2.e));
  loc->ms_setup = ms1;
  loc->ms_solve = ms2;
  return st;
}

// Algorithm 1 to its stopping test from (u, phi) with U^old = phi_old and phi~ = pt; fills
// everything of *out but ms_total.  On return c->R holds the residual at the final iterate,
// except after a failed linear solve (then it is the residual before that step's update).
static mfpff_status pdas_loop(mfpff_ctx* c, double* u, double* phi, const double* phi_old, const double* pt,
                              uint8_t* active, int max_newton, double tol, mfpff_pdas_info* out) {
  Level& F = c->lv[c->L];
  if (!c->act_prev) c->act_prev = dalloc<uint8_t>(F.nn);
  if (!c->pdas_part) c->pdas_part = dalloc<double>((size_t)2 * pdas_check_blocks(F.nn));
  const int nb = pdas_check_blocks(F.nn);
  std::vector<double> ph((size_t)2 * nb);
  mfpff_status st = MFPFF_ERR_NOCONV;
  double r0 = -1.0;
  for (int k = 0; k <= max_newton; ++k) {
    ScopedEvent e0;
    HIPCHK(hipEventRecord(e0.e, c->s));
    residual_and_active(c, u, phi, phi_old, pt, active);
    // stopping test: the active set repeats and ||P_k R_k|| <= tol ||P_0 R_0||
    k_pdas_check(c->pdas_part, c->R, active, c->act_prev, F.g, c->prob.dirichlet, c->s);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(ph.data(), c->pdas_part, ph.size() * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    double ss = 0, nd = 0;
    for (int b = 0; b < nb; ++b) {
      ss += ph[2 * b];
      nd += ph[2 * b + 1];
    }
    const double rn = std::sqrt(ss);
    if (r0 < 0) r0 = rn;
    out->rel_residual = r0 > 0 ? rn / r0 : 0.0;
    if (k > 0 && nd == 0.0 && rn <= tol * r0) {
      st = MFPFF_OK;
      out->converged = 1;
      break;
    }
    if (k == max_newton) break;
    mfpff_solve_info loc{};
    const mfpff_status sst = linearise_solve_update(c, u, phi, phi_old, pt, active, e0.e, &loc);
    out->newton_steps = k + 1;
    out->gmres_iterations += loc.iterations;
    HIPCHK(hipMemcpyAsync(c->act_prev, active, F.nn, hipMemcpyDeviceToDevice, c->s));
    if (sst != MFPFF_OK) {
      st = sst;
      c->err = "GMRES reached max_iter inside the active-set loop";
      break;
    }
  }
  HIPCHK(hipStreamSynchronize(c->s));
  std::vector<uint8_t> ah(F.nn);
  HIPCHK(hipMemcpy(ah.data(), active, F.nn, hipMemcpyDeviceToHost));
  for (auto v : ah) out->n_active += v ? 1 : 0;
  if (st == MFPFF_ERR_NOCONV && !out->converged && c->err.empty()) c->err = "active-set loop reached max_newton";
  return st;
}

static int count_active(mfpff_ctx* c) {
  Level& F = c->lv[c->L];
  std::vector<uint8_t> mh(F.nn);
  HIPCHK(hipMemcpy(mh.data(), F.mask, F.nn, hipMemcpyDeviceToHost));
  int na = 0;
  for (auto v : mh) na += (v & kMaskPhi) ? 1 : 0;
  return na;
}
}  // namespace

extern "C" {

mfpff_status mfpff_newton_step(mfpff_ctx* c, double* u, double* phi, const double* phi_old, const double* phi_tilde,
                               uint8_t* active, mfpff_solve_info* info) {
  return run(c, [&]() {
    require_ptr(u, "u");
    require_ptr(phi, "phi");
    require_ptr(phi_old, "phi_old");
    require_ptr(active, "active");
    const double* pt = phi_tilde ? phi_tilde : phi_old;
    ScopedEvent e0;
    HIPCHK(hipEventRecord(e0.e, c->s));
    residual_and_active(c, u, phi, phi_old, pt, active);
    mfpff_solve_info loc{};
    const mfpff_status st = linearise_solve_update(c, u, phi, phi_old, pt, active, e0.e, &loc);
    loc.n_active = count_active(c);
    if (info) *info = loc;
    if (st == MFPFF_ERR_NOCONV) c->err = "GMRES reached max_iter";
    return st;
  });
}

mfpff_status mfpff_pdas_solve(mfpff_ctx* c, double* u, double* phi, const double* phi_old, const double* phi_tilde,
                              uint8_t* active, int max_newton, double tol, mfpff_pdas_info* info) {
  return run(c, [&]() {
    require_ptr(u, "u");
    require_ptr(phi, "phi");
    require_ptr(phi_old, "phi_old");
    require_ptr(active, "active");
    if (max_newton < 0 || !(tol >= 0.0)) throw StatusError{MFPFF_ERR_ARG, "max_newton must be >= 0 and tol >= 0"};
    const auto t0 = std::chrono::steady_clock::now();
    mfpff_pdas_info out{};
    const mfpff_status st = pdas_loop(c, u, phi, phi_old, phi_tilde ? phi_tilde : phi_old, active, max_newton, tol, &out);
    out.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = out;
    return st;
  });
}

mfpff_status mfpff_load_step(mfpff_ctx* c, double* u, double* phi, const double* phi_prev, const double* phi_prev2,
                             const double* u_top, uint8_t* active, int max_newton, double tol, mfpff_load_info* info) {
  return run(c, [&]() {
    require_ptr(u, "u");
    require_ptr(phi, "phi");
    require_ptr(phi_prev, "phi_prev");
    require_ptr(u_top, "u_top");
    require_ptr(active, "active");
    if (max_newton < 0 || !(tol >= 0.0)) throw StatusError{MFPFF_ERR_ARG, "max_newton must be >= 0 and tol >= 0"};
    if (!c->prob.dirichlet) throw StatusError{MFPFF_ERR_ARG, "load stepping needs the Dirichlet faces (dirichlet = 1)"};
    if (phi_prev == phi || phi_prev2 == phi)
      throw StatusError{MFPFF_ERR_ARG, "phi_prev and phi_prev2 must not alias phi (phi is updated in place)"};
    for (int a = 0; a < c->dim; ++a)
      if (!std::isfinite(u_top[a])) throw StatusError{MFPFF_ERR_ARG, "u_top must be finite"};
    const auto t0 = std::chrono::steady_clock::now();
    Level& F = c->lv[c->L];
    if (!c->phit_ext) c->phit_ext = dalloc<double>(F.nn);
    if (!c->react) c->react = dalloc<double>(6);
    k_impose_faces(u, F.g, u_top, c->s);
    const double* pt = phi_prev;
    if (phi_prev2) {
      k_extrapolate(c->phit_ext, phi_prev, phi_prev2, F.nn, c->s);
      pt = c->phit_ext;
    }
    LAUNCHCHK();
    mfpff_load_info out{};
    const mfpff_status st = pdas_loop(c, u, phi, phi_prev, pt, active, max_newton, tol, &out.pdas);
    // reactions from the residual at the returned state (after a failed linear solve the loop's
    // last residual belongs to the state before that step's update)
    residual_into_R(c, u, phi, pt);
    k_face_reaction(c->react, c->R, F.g, c->s);
    LAUNCHCHK();
    double rh[6] = {0, 0, 0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(rh, c->react, 2 * c->dim * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    for (int a = 0; a < c->dim; ++a) {
      out.reaction_bottom[a] = rh[a];
      out.reaction_top[a] = rh[c->dim + a];
    }
    out.pdas.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = out;
    return st;
  });
}

}  // extern "C"
