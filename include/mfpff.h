/*
 * mfpff: matrix-free linear solves for the semi-smooth Newton step of the
 * coupled displacement / phase-field fracture problem, on AMD MI355X (gfx950).
 *
 * Method: Jodlbauer, Langer, Wick, "Parallel matrix-free higher-order finite
 * element solvers for phase-field fracture problems".  Each Newton step of
 * the primal-dual active-set method (Algorithm 1) solves G dU = -R on the
 * inactive set, with R the residual of eq. (residual) and G its derivative
 * eq. (G) (phi~ frozen, so G is block lower triangular, Section 3.3).  The
 * product with G is evaluated cell by cell without a stored matrix
 * (Section 3.4); GMRES is preconditioned by a monolithic geometric multigrid
 * V-cycle with a block-diagonal Chebyshev-Jacobi smoother (Section 3.3).
 *
 * Conventions (all entry points):
 *   - Domain [0,1]^dim, N cells per direction, Q_k with equispaced nodes,
 *     Gauss quadrature with k+1 points per direction.
 *   - Nodes are numbered lexicographically, node = i0 + M*i1 (+ M*M*i2),
 *     M = k*N + 1; n_nodes = M^dim.
 *   - Vectors are component-blocked: [u_0 | ... | u_{dim-1} | phi], each
 *     block n_nodes long; n_dofs = (dim+1)*n_nodes.  The displacement u
 *     argument is the first dim blocks of that layout (dim*n_nodes values).
 *   - Vector and field arguments are DEVICE pointers owned by the caller,
 *     contiguous, 8-byte doubles unless stated (4-byte floats when a
 *     precision argument says FP32).  The library keeps no caller pointer
 *     past the call.
 *   - The active set is one byte per node (non-zero = the phi-dof of that
 *     node is fixed, delta phi = 0).  Homogeneous Dirichlet conditions fix
 *     every displacement dof on the two faces normal to the last axis when
 *     `dirichlet` is set.  Fixed dofs get identity rows and columns:
 *     G^ = P G P + (I - P), P the diagonal 0/1 matrix of free dofs.
 *   - Work is enqueued on the HIP stream given at creation.  Entry points
 *     that return host values (gmres_solve, residual_param_vjp, newton_step,
 *     level_info) synchronise that stream; the others are asynchronous.
 *   - Errors are reported by status codes; no exception crosses this ABI.
 *     mfpff_last_error() returns a message for the last failure of a context.
 *   - A context is not thread-safe; use one per host thread.
 */
#ifndef MFPFF_H
#define MFPFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MFPFF_MAX_LEVELS 16

typedef struct mfpff_ctx mfpff_ctx;

typedef enum {
  MFPFF_OK = 0,
  MFPFF_ERR_ARG = 1,      /* invalid argument (sizes, degree, level index, null pointer) */
  MFPFF_ERR_STATE = 2,    /* called before mfpff_set_linearization */
  MFPFF_ERR_OOM = 3,      /* device allocation failed */
  MFPFF_ERR_HIP = 4,      /* a HIP runtime call failed */
  MFPFF_ERR_NOCONV = 5,   /* GMRES reached max_iter; the last iterate is returned */
  MFPFF_ERR_NUMERIC = 6   /* non-finite value or failed factorisation */
} mfpff_status;

typedef enum { MFPFF_F64 = 0, MFPFF_F32 = 1 } mfpff_prec;

/* Tension/compression split of the elastic energy (Section 2.1).  AMOR: volumetric/deviatoric,
 * E^+ = K/2 <tr e>_+^2 + mu dev e : dev e with K = lambda + 2 mu / dim.  MIEHE: spectral,
 * E^+ = lambda/2 <tr e>_+^2 + mu e^+ : e^+ with e^+ the positive part of the strain from its
 * eigensystem; the tangent differentiates e^+ in the eigenbasis (Section 3.5) with divided
 * differences, which equal Algorithm 2 on distinct eigenvalues.  NONE: the isotropic model of
 * Section 5 (no split): E^+ = lambda/2 tr(e)^2 + mu e : e, E^- = 0. */
typedef enum { MFPFF_SPLIT_AMOR = 0, MFPFF_SPLIT_MIEHE = 1, MFPFF_SPLIT_NONE = 2 } mfpff_split;

/* Engine of the sum-factorised 1D contractions (Section 3.4) of the 3D products at degree 3
 * and 4 with the volumetric/deviatoric split: the vector unit (one thread per node line), or
 * the matrix cores (MFMA blocks of 4 x 4; both give the same operator up to rounding).  Other
 * degrees and splits always use the vector unit. */
typedef enum { MFPFF_CONTRACT_VALU = 0, MFPFF_CONTRACT_MFMA = 1 } mfpff_contraction;

typedef enum {
  MFPFF_OP_G = 0,         /* y = G^ x */
  MFPFF_OP_GT = 1,        /* y = G^T-hat x (transpose: coupling moves to the u rows) */
  MFPFF_OP_BLOCKDIAG = 2, /* y = diag(G^_uu, G^_phiphi) x (smoother operator) */
  MFPFF_OP_ACCUMULATE = 16 /* flag: y += P op(G) P x on the free rows, y not initialised
                              (one cell-kernel launch, no identity part) */
} mfpff_op;

/* Problem description.  Levels run from the coarsest (index 0) to the
 * finest (index n_levels-1).  Consecutive levels are either an h-step
 * (N halves, same degree) or a p-step (same N, lower degree dividing the
 * finer one); coarse nodes are then a subset of fine nodes. */
typedef struct {
  int dim;                          /* 2 or 3 */
  int n_levels;                     /* 1 .. MFPFF_MAX_LEVELS */
  int level_N[MFPFF_MAX_LEVELS];    /* cells per direction */
  int level_k[MFPFF_MAX_LEVELS];    /* degree, 1 .. 4 */
  int dirichlet;                    /* 1: delta u = 0 on the faces normal to the last axis */
  double lambda, mu;                /* Lame parameters */
  double Gc, eps, kappa;            /* toughness, length scale, degradation floor (Section 2.1):
                                       g(phi) = (1 - kappa) phi^2 + kappa.  The model takes
                                       0 <= kappa << 1; any kappa in (-1, 1) is accepted, and a
                                       negative one (g < 0 where phi is small) makes G^_uu
                                       indefinite, which the coarse solve meets with LU */
  double as_c;                      /* constant c of the active-set rule of Algorithm 1 */
  int cheb_degree;                  /* Chebyshev polynomial degree s (s-1 operator products) */
  double cheb_lo, cheb_hi;          /* interval factors (Section 3.3: 0.24, 1.2) */
  int lanczos_steps;                /* CG steps of the lambda_max estimate */
  unsigned long long lanczos_seed;  /* SplitMix64 seed of the start vectors */
  int vcycle_prec;                  /* mfpff_prec of levels and smoothers inside the V-cycle */
  int restart;                      /* GMRES restart length m (<= 64) */
  int max_iter;                     /* total GMRES iteration cap */
  double rtol;                      /* relative true-residual tolerance */
  int split;                        /* mfpff_split */
  int pdas_project;                 /* active-set update of Algorithm 1: 0 keeps phi on A_k (delta
                                       phi = 0, as the paper writes it); 1 first sets phi := phi_old
                                       on A_k (the iterate on the obstacle, the primal-dual active
                                       set update) and linearises there */
  int contraction;                  /* mfpff_contraction: engine of the 1D contractions of the 3D
                                       products at degree 3 and 4 (volumetric/deviatoric split) */
  int slit;                         /* 1: the slit geometry of the notched tests (Section 5.1): the
                                       cells on the two sides of the mid-plane of the last axis are
                                       not connected for x < 1/2.  Those slit-plane nodes exist
                                       twice: the grid node belongs to the cells below the slit, a
                                       duplicate, numbered after the M^dim grid nodes (first axis
                                       fastest, then the second axis in 3D), to the cells above, so
                                       n_nodes = M^dim + (kN/2) M^(dim-2).  Requires even N on
                                       every level (each level is a slit mesh); products use the
                                       cell kernel with the slit-aware node map.  A coarse
                                       duplicate is injected from the fine duplicate at its
                                       position; the prolongation gives every fine node the coarse
                                       values of its own side of the slit (a fine node above the
                                       plane, or a fine duplicate, reads a coarse slit node's
                                       duplicate), and the restriction is its transpose */
} mfpff_problem;

typedef struct {
  int iterations;                   /* GMRES iterations (preconditioner applications) */
  int converged;                    /* 1 if ||b - G^ x|| <= rtol ||b|| */
  double rel_residual;              /* ||b - G^ x|| / ||b|| computed at the end */
  double ms_setup;                  /* time of set_linearization inside newton_step, ms */
  double ms_solve;                  /* time of the GMRES solve, ms */
  int n_active;                     /* newton_step: size of the active set */
} mfpff_solve_info;

typedef struct {
  int N, k;
  long long n_nodes, n_dofs;
  double lambda_u, lambda_phi;      /* Ritz estimates of lambda_max(D^-1 G^_bb), after linearisation */
  int lanczos_steps_u, lanczos_steps_phi;
} mfpff_level_desc;

/* Build the level hierarchy (the Q_k meshes of Section 3.1 and the multigrid levels of
 * Section 3.3), 1D tables and all device storage for a problem (the mesh set-up of the solver).
 * `prob` is read during the call only; `hip_stream` is a hipStream_t (NULL: the default stream)
 * on the current device, which every later call of the context uses.  On success *out owns every
 * device allocation.  MFPFF_ERR_ARG for an invalid description, including a level with 2^31 or
 * more dofs or a 2D Q1/Q2 level with 2^28 or more nodes; MFPFF_ERR_OOM when device memory runs
 * out. */
mfpff_status mfpff_setup_mesh_levels(const mfpff_problem* prob, void* hip_stream, mfpff_ctx** out);

/* Release a context and everything it owns.  NULL is ignored.  (Library housekeeping; no passage
 * of the paper.) */
void mfpff_destroy(mfpff_ctx* ctx);

/* Message describing the last failure on this context ("" if none).  (Library housekeeping.) */
const char* mfpff_last_error(const mfpff_ctx* ctx);

/* Debug kernel build (sources compiled with -DMFPFF_BOUNDS, libmfpff_bounds.so): the kernels check
 * every node, cell and transfer index they compute against its range, count an index outside it
 * and use 0 in its place (reported, never a memory fault).  Returns the number counted since the
 * library was loaded, after synchronising the device; -1 from the regular build, which has no
 * checks; -2 if the counters cannot be read.  For the library's own tests, not for production
 * callers. */
long long mfpff_debug_bounds_hits(void);

/* Number of nodes and of dofs ((dim+1) * n_nodes, component-blocked) of level `level`
 * (0 = coarsest .. n_levels-1 = finest): the Q_k nodal dofs of Section 3.1 on that level.  Host only: no device work, no synchronisation.
 * MFPFF_ERR_ARG for a NULL argument or a level out of range (no message is stored, the
 * context being read-only here). */
mfpff_status mfpff_sizes(const mfpff_ctx* ctx, int level, size_t* n_nodes, size_t* n_dofs);

/* Sizes and smoother data of one level (synchronises): the largest-eigenvalue estimates that set
 * the Chebyshev interval of Section 3.3.  Before any linearisation lambda_u = lambda_phi = 1 and
 * the step counts are 0.  MFPFF_ERR_ARG for a NULL argument or a level out of range. */
mfpff_status mfpff_level_info(mfpff_ctx* ctx, int level, mfpff_level_desc* out);

/* Freeze the linearisation point of eq. (G) and set up the multigrid preconditioner of
 * Section 3.3 (Algorithm 1 calls this once per Newton step): u (dim*n_nodes), phi, phi_old
 * and phi_tilde (n_nodes each; phi_tilde NULL means phi_old) and the active
 * set (n_nodes bytes) on the finest level.  Injects fields and masks to every
 * coarser level, builds the diagonals, the Chebyshev intervals (CG-Lanczos
 * estimates) and the factorised coarse blocks (Cholesky; a block that is not
 * positive definite is inverted by Gauss-Jordan elimination with partial
 * pivoting instead).  Fails with MFPFF_ERR_NUMERIC when an input field holds a
 * non-finite value or a coarse block is singular (a zero pivot), and with
 * MFPFF_ERR_ARG when the coarsest level has more than 16384 dofs (its dense
 * factorisation is allocated on first use). */
mfpff_status mfpff_set_linearization(mfpff_ctx* ctx, const double* u, const double* phi,
                                     const double* phi_old, const uint8_t* active,
                                     const double* phi_tilde);

/* Product-only linearisation of eq. (G): the same fields, active set and Dirichlet rows
 * as mfpff_set_linearization, injected to every level, but no diagonals,
 * smoother intervals or coarse factorisation.  Enough for
 * mfpff_apply_jacobian (any op) on every level; mfpff_vcycle, mfpff_smooth,
 * mfpff_diagonal, mfpff_coarse_solve and mfpff_gmres_solve still need
 * mfpff_set_linearization (MFPFF_ERR_STATE otherwise).  Used by the backward
 * of the residual, where only the transposed product is needed. */
mfpff_status mfpff_set_point(mfpff_ctx* ctx, const double* u, const double* phi, const double* phi_old,
                             const uint8_t* active, const double* phi_tilde);

/* y = op(G^_level) x on one level: the product with the Jacobian of eq. (G), constrained as in
 * Algorithm 1 (fixed dofs get identity rows and columns), evaluated cell by cell by sum
 * factorisation without a stored matrix (Section 3.4).  x, y: n_dofs of that level (device),
 * FP64 or FP32 per `prec` (FP32 uses the FP32 copy of the level data).  x and y must not alias.
 * `op` is an mfpff_op value (G^, its transpose, or the block-diagonal operator of the smoother),
 * optionally or-ed with MFPFF_OP_ACCUMULATE.  MFPFF_ERR_STATE before a point is set,
 * MFPFF_ERR_ARG for a level out of range, a NULL pointer, or an unknown op or precision. */
mfpff_status mfpff_apply_jacobian(mfpff_ctx* ctx, int level, const void* x, void* y, int prec, int op);

/* Diagonal of G^_level (1 at fixed dofs), FP64, n_dofs of the level (device): the Jacobi scaling
 * of the Chebyshev-Jacobi smoother of Section 3.3, which needs only the diagonal and the product.
 * MFPFF_ERR_STATE before mfpff_set_linearization. */
mfpff_status mfpff_diagonal(mfpff_ctx* ctx, int level, double* diag);

/* z = diag(C_u, C_phi) r on level >= 1: the block-diagonal Chebyshev-Jacobi smoother of
 * Section 3.3 (one polynomial per block on [0.24, 1.2] lambda_max), applied to r from a zero start
 * (FP64, device vectors of the level's n_dofs).  MFPFF_ERR_STATE before mfpff_set_linearization,
 * MFPFF_ERR_ARG for level 0 or out of range. */
mfpff_status mfpff_smooth(mfpff_ctx* ctx, int level, const double* r, double* z);

/* Masked transfer between level-1 and level (level >= 1) of the geometric multigrid of
 * Section 3.3: direction 0 is prolongation (in: level-1 vector, out: level vector), 1 is
 * restriction (the transpose).  The interpolation is the Kronecker product of the 1D Lagrange
 * interpolation matrices, per component, with fixed dofs zeroed on both sides.  FP64, device
 * vectors.  MFPFF_ERR_STATE before a point is set, MFPFF_ERR_ARG for a bad level or direction. */
mfpff_status mfpff_transfer(mfpff_ctx* ctx, int level, int direction, const double* in, double* out);

/* Exact FP64 solve with the coarsest level operator, using the block lower-triangular structure
 * of eq. (G) that Section 3.3 points out: x_u = G^_uu^-1 r_u, x_phi = G^_phiphi^-1 (r_phi -
 * G^_phiu x_u) (the paper runs Chebyshev over the whole spectrum there instead), each block
 * inverse from its Cholesky factor or, where that failed, from Gauss-Jordan.  r, x: device,
 * n_dofs of level 0.  MFPFF_ERR_STATE before mfpff_set_linearization. */
mfpff_status mfpff_coarse_solve(mfpff_ctx* ctx, const double* r, double* x);

/* One V-cycle of the monolithic geometric multigrid of Section 3.3 on the finest level:
 * z = V(r), pre- and post-smoothing on every level, exact coarse solve.  r, z: device, finest
 * n_dofs, FP64 (the levels run in the problem's V-cycle precision, with casts at the ends).
 * MFPFF_ERR_STATE before mfpff_set_linearization. */
mfpff_status mfpff_vcycle(mfpff_ctx* ctx, const double* r, double* z);

/* The linear solve of each Newton step of Algorithm 1 (Section 3.3: GMRES preconditioned by the
 * multigrid V-cycle): right-preconditioned flexible GMRES(m), classical Gram-Schmidt twice (the
 * norm after the second projection taken as sqrt(|w|^2 - |h2|^2), the basis being orthonormal),
 * x0 = 0, until ||b - G^ x|| <= rtol ||b|| (FP64 outer iteration; V-cycle precision per the
 * problem).  b, x: device, finest n_dofs.  MFPFF_ERR_NOCONV leaves the last iterate in x (info
 * filled); MFPFF_ERR_STATE before mfpff_set_linearization.  Synchronises. */
mfpff_status mfpff_gmres_solve(mfpff_ctx* ctx, const double* b, double* x, mfpff_solve_info* info);

/* Residual of eq. (residual) on the finest level at (u, phi) with phi~ in
 * the degradation of the displacement equation; unconstrained (no masks).  u (dim*n_nodes), phi,
 * phi_tilde (n_nodes) and R (n_dofs): device.  Needs no linearisation. */
mfpff_status mfpff_residual(mfpff_ctx* ctx, const double* u, const double* phi,
                            const double* phi_tilde, double* R);

/* Parameter cotangents of the residual of eq. (residual) at (u, phi; phi~):
 * dGc = <v, dR/dGc>, deps = <v, dR/deps> (only the phase-field rows depend on Gc and eps).  u, phi,
 * phi_tilde, v: device (v: n_dofs); dGc_host, deps_host: host doubles.  The point is passed
 * explicitly, so the result does not depend on an earlier call.  Synchronises. */
mfpff_status mfpff_residual_param_vjp(mfpff_ctx* ctx, const double* u, const double* phi,
                                      const double* phi_tilde, const double* v,
                                      double* dGc_host, double* deps_host);

/* The same parameter cotangents as mfpff_residual_param_vjp, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the per-block partial sums live in a static device array of the library (2 MiB per
 * device, held until the process ends) instead of the context's buffer.  This call performs no
 * hipMalloc, hipFree or other allocation.  Limit: the finest level may need at most 131072
 * partial-sum blocks of the cotangent kernel (about 1.2 M cells in 3D Q2, 3.7 M in 2D Q2); larger
 * contexts get MFPFF_ERR_ARG with a message.  Every call on one device shares that array, so calls
 * that overlap on one device (several host threads, or contexts on different streams whose work
 * overlaps) race; calls queued on one stream do not.  Results are bit-identical to
 * mfpff_residual_param_vjp.  Synchronises. */
mfpff_status mfpff_residual_param_vjp_noalloc(mfpff_ctx* ctx, const double* u, const double* phi,
                                              const double* phi_tilde, const double* v,
                                              double* dGc_host, double* deps_host);

/* Active set of Algorithm 1 from the residual R (as returned by
 * mfpff_residual): active_i = [ -(M_L^-1 R_phi)_i + c (phi - phi_old)_i > 0 ],
 * M_L the row-sum-lumped phi mass matrix. */
mfpff_status mfpff_active_set(mfpff_ctx* ctx, const double* R, const double* phi,
                              const double* phi_old, uint8_t* active);

/* Unconstrained element matrices of eq. (G) on one level at the current point (after
 * mfpff_set_point or mfpff_set_linearization), FP64, for assembling the sparse Jacobian (the
 * matrix-based product that Section 6 compares the matrix-free one against).  em (device,
 * caller-owned) receives n_cells * nl * nl values, nl = (dim + 1) (k + 1)^dim, laid out
 * [cell][row][column]; cells in lexicographic order (x fastest), local rows and columns
 * (component, local node) with the local node lexicographic in the cell (x fastest), so that
 * local node (i0, i1, i2) of cell (cx, cy, cz) is global node
 * (k cx + i0) + M (k cy + i1) + M^2 (k cz + i2), M = k N + 1, and dof = component * n_nodes + node.
 * MFPFF_ERR_STATE before a point is set. */
mfpff_status mfpff_element_matrices(mfpff_ctx* ctx, int level, double* em);

/* One semi-smooth Newton step of Algorithm 1 on the finest level: residual,
 * active set (written to `active`), linearisation, b = -P R, GMRES solve,
 * u += du, phi += dphi (u, phi updated in place).  Synchronises. */
mfpff_status mfpff_newton_step(mfpff_ctx* ctx, double* u, double* phi, const double* phi_old,
                               const double* phi_tilde, uint8_t* active, mfpff_solve_info* info);

/* Result of mfpff_pdas_solve. */
typedef struct {
  int newton_steps;                 /* Newton steps taken (linear solves) */
  int converged;                    /* 1: the active set repeated and ||P R|| <= tol ||P_0 R_0|| */
  int gmres_iterations;             /* FGMRES iterations summed over the steps */
  int n_active;                     /* size of the final active set */
  double rel_residual;              /* ||P_k R_k|| / ||P_0 R_0|| at the last test */
  double ms_total;                  /* wall time of the call, ms */
} mfpff_pdas_info;

/* Algorithm 1 (primal-dual active set) to its stopping test: repeat
 *   R_k = R(u, phi; phi~), A_k from the active-set rule (as in mfpff_active_set),
 *   stop if k > 0, A_k = A_{k-1} and ||P_k R_k||_2 <= tol ||P_0 R_0||_2
 *   (P_k: free dofs, i.e. u-dofs off the Dirichlet faces and phi-dofs outside A_k;
 *    the paper's eps_as is read relative to the first iterate),
 *   otherwise one Newton step as mfpff_newton_step with A_k,
 * for at most max_newton steps.  u (dim*n_nodes), phi (n_nodes) are device arrays updated in
 * place; phi_old, phi_tilde (NULL: phi_old) are read; active (n_nodes bytes, device) receives the
 * final active set.  Returns MFPFF_OK when the test is met, MFPFF_ERR_NOCONV after max_newton
 * steps or when a linear solve reaches max_iter (the state is the last iterate; *info is filled
 * either way), MFPFF_ERR_ARG for max_newton < 0, tol < 0 or a null pointer.  Synchronises. */
mfpff_status mfpff_pdas_solve(mfpff_ctx* ctx, double* u, double* phi, const double* phi_old,
                              const double* phi_tilde, uint8_t* active, int max_newton, double tol,
                              mfpff_pdas_info* info);

/* Result of mfpff_load_step. */
typedef struct {
  mfpff_pdas_info pdas;             /* the active-set loop of the step (ms_total: the whole call) */
  double reaction_top[3];           /* per component, the sum of the displacement residual rows
                                       over the top face's nodes at the final iterate */
  double reaction_bottom[3];        /* the same over the bottom face (unused entries: 0) */
} mfpff_load_info;

/* One load step of the single-edge-notched tests (Section 5: a displacement prescribed on the
 * top boundary that grows with the step, the bottom held fixed), with the extrapolated phase
 * field of Section 3 in the degradation g:
 *   u := 0 on the bottom face and u := u_top on the top face, every component (the two faces
 *        normal to the last axis, the faces the Dirichlet mask fixes);
 *   phi~ := 2 phi_prev - phi_prev2 (linear extrapolation over two equal steps; phi_prev2 NULL,
 *        the first step: phi~ := phi_prev);
 *   Algorithm 1 as mfpff_pdas_solve from (u, phi) with phi_old = phi_prev and this phi~;
 *   reactions from the residual at the final iterate.
 * u (dim*n_nodes) and phi (n_nodes) are device arrays updated in place (on entry normally the
 * previous step's solution, phi a copy of phi_prev); phi_prev, phi_prev2 (n_nodes, device) are read
 * and must not be the array phi; u_top is a host array of dim values; active (n_nodes bytes,
 * device) receives the final active set.  Status as mfpff_pdas_solve; MFPFF_ERR_ARG also when the
 * problem has dirichlet = 0, u_top is not finite, or phi_prev or phi_prev2 is phi.  *info is filled
 * whenever the loop ran.  Synchronises. */
mfpff_status mfpff_load_step(mfpff_ctx* ctx, double* u, double* phi, const double* phi_prev,
                             const double* phi_prev2, const double* u_top, uint8_t* active,
                             int max_newton, double tol, mfpff_load_info* info);

#ifdef __cplusplus
}
#endif
#endif /* MFPFF_H */
