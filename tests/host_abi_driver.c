/* Host-side driver of the C boundary, built with AddressSanitizer and UndefinedBehaviorSanitizer
 * against a library whose host code carries the same instrumentation.  It takes every path
 * that needs no device: argument validation of the problem, null contexts and pointers on every
 * entry point, and a set-up that either succeeds (a device is present: the context is queried
 * and destroyed) or fails on the first runtime call and frees its partial context.  Prints "ok"
 * and exits 0 when every status is the documented one; a sanitizer report ends it earlier. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "mfpff.h"

static int failures = 0;

#define EXPECT(cond)                                           \
  do {                                                         \
    if (!(cond)) {                                             \
      fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                              \
    }                                                          \
  } while (0)

static mfpff_problem good(void) {
  mfpff_problem p;
  memset(&p, 0, sizeof p);
  p.dim = 2;
  p.n_levels = 2;
  p.level_N[0] = 4;
  p.level_N[1] = 8;
  p.level_k[0] = p.level_k[1] = 1;
  p.dirichlet = 1;
  p.lambda = 121.15e3;
  p.mu = 80.77e3;
  p.Gc = 2.7;
  p.eps = 0.25;
  p.kappa = 1e-10;
  p.as_c = 1.0;
  p.cheb_degree = 5;
  p.cheb_lo = 0.24;
  p.cheb_hi = 1.2;
  p.lanczos_steps = 15;
  p.lanczos_seed = 7;
  p.vcycle_prec = MFPFF_F64;
  p.restart = 30;
  p.max_iter = 100;
  p.rtol = 1e-6;
  p.split = MFPFF_SPLIT_AMOR;
  return p;
}

static void expect_rejected(mfpff_problem p) {
  mfpff_ctx* c = (mfpff_ctx*)&p; /* must be reset to NULL by the call */
  EXPECT(mfpff_setup_mesh_levels(&p, NULL, &c) == MFPFF_ERR_ARG);
  EXPECT(c == NULL);
}

int main(void) {
  mfpff_problem p;
  /* one invalid field at a time */
  p = good(); p.dim = 5; expect_rejected(p);
  p = good(); p.dim = 1; expect_rejected(p);
  p = good(); p.n_levels = 0; expect_rejected(p);
  p = good(); p.n_levels = MFPFF_MAX_LEVELS + 1; expect_rejected(p);
  p = good(); p.cheb_degree = 0; expect_rejected(p);
  p = good(); p.cheb_degree = 33; expect_rejected(p);
  p = good(); p.lanczos_steps = 65; expect_rejected(p);
  p = good(); p.restart = 0; expect_rejected(p);
  p = good(); p.restart = 65; expect_rejected(p);
  p = good(); p.max_iter = -1; expect_rejected(p);
  p = good(); p.rtol = NAN; expect_rejected(p);
  p = good(); p.vcycle_prec = 7; expect_rejected(p);
  p = good(); p.split = 3; expect_rejected(p);
  p = good(); p.pdas_project = 2; expect_rejected(p);
  p = good(); p.contraction = 2; expect_rejected(p);
  p = good(); p.slit = 2; expect_rejected(p);
  p = good(); p.slit = 1; p.level_N[0] = 3; p.level_N[1] = 6; expect_rejected(p);  /* odd coarse N */
  p = good(); p.n_levels = 1; p.level_N[0] = 7; p.slit = 1; expect_rejected(p);  /* odd N */
  p = good(); p.eps = 0.0; expect_rejected(p);
  p = good(); p.kappa = -1.0; expect_rejected(p);
  p = good(); p.kappa = 1.0; expect_rejected(p);
  p = good(); p.kappa = NAN; expect_rejected(p);
  p = good(); p.cheb_lo = 1.2; p.cheb_hi = 0.24; expect_rejected(p);
  p = good(); p.cheb_lo = 0.0; expect_rejected(p);
  p = good(); p.level_k[1] = 5; p.level_k[0] = 5; expect_rejected(p);   /* degree above 4 */
  p = good(); p.level_N[1] = 0; expect_rejected(p);
  p = good(); p.level_k[1] = 2; expect_rejected(p);                     /* neither h- nor p-step */
  p = good(); p.level_N[1] = 12; expect_rejected(p);
  {
    mfpff_ctx* c = NULL;
    EXPECT(mfpff_setup_mesh_levels(NULL, NULL, &c) == MFPFF_ERR_ARG);
    p = good();
    EXPECT(mfpff_setup_mesh_levels(&p, NULL, NULL) == MFPFF_ERR_ARG);
  }

  /* null contexts: every entry point refuses them without touching its other arguments */
  double d = 0.0, e = 0.0;
  size_t nn = 0, nd = 0;
  mfpff_level_desc desc;
  mfpff_solve_info si;
  mfpff_pdas_info pi;
  mfpff_load_info li;
  EXPECT(strcmp(mfpff_last_error(NULL), "null context") == 0);
  EXPECT(mfpff_debug_bounds_hits() == -1); /* the regular library has no index checks */
  mfpff_destroy(NULL);
  EXPECT(mfpff_sizes(NULL, 0, &nn, &nd) == MFPFF_ERR_ARG);
  EXPECT(mfpff_level_info(NULL, 0, &desc) == MFPFF_ERR_ARG);
  EXPECT(mfpff_set_linearization(NULL, NULL, NULL, NULL, NULL, NULL) == MFPFF_ERR_ARG);
  EXPECT(mfpff_set_point(NULL, NULL, NULL, NULL, NULL, NULL) == MFPFF_ERR_ARG);
  EXPECT(mfpff_apply_jacobian(NULL, 0, NULL, NULL, MFPFF_F64, MFPFF_OP_G) == MFPFF_ERR_ARG);
  EXPECT(mfpff_diagonal(NULL, 0, NULL) == MFPFF_ERR_ARG);
  EXPECT(mfpff_smooth(NULL, 0, NULL, NULL) == MFPFF_ERR_ARG);
  EXPECT(mfpff_transfer(NULL, 0, 0, NULL, NULL) == MFPFF_ERR_ARG);
  EXPECT(mfpff_coarse_solve(NULL, NULL, NULL) == MFPFF_ERR_ARG);
  EXPECT(mfpff_vcycle(NULL, NULL, NULL) == MFPFF_ERR_ARG);
  EXPECT(mfpff_gmres_solve(NULL, NULL, NULL, &si) == MFPFF_ERR_ARG);
  EXPECT(mfpff_residual(NULL, NULL, NULL, NULL, NULL) == MFPFF_ERR_ARG);
  EXPECT(mfpff_residual_param_vjp(NULL, NULL, NULL, NULL, NULL, &d, &e) == MFPFF_ERR_ARG);
  EXPECT(mfpff_residual_param_vjp_noalloc(NULL, NULL, NULL, NULL, NULL, &d, &e) == MFPFF_ERR_ARG);
  EXPECT(mfpff_active_set(NULL, NULL, NULL, NULL, NULL) == MFPFF_ERR_ARG);
  EXPECT(mfpff_element_matrices(NULL, 0, NULL) == MFPFF_ERR_ARG);
  EXPECT(mfpff_newton_step(NULL, NULL, NULL, NULL, NULL, NULL, &si) == MFPFF_ERR_ARG);
  EXPECT(mfpff_pdas_solve(NULL, NULL, NULL, NULL, NULL, NULL, 5, 1e-8, &pi) == MFPFF_ERR_ARG);
  EXPECT(mfpff_load_step(NULL, NULL, NULL, NULL, NULL, NULL, NULL, 5, 1e-8, &li) == MFPFF_ERR_ARG);

  /* a valid problem: without a device the set-up fails on its first runtime call and frees the
   * partial context (the leak checker sees it); with one it succeeds and is destroyed */
  {
    mfpff_ctx* c = NULL;
    p = good();
    mfpff_status st = mfpff_setup_mesh_levels(&p, NULL, &c);
    if (st == MFPFF_OK) {
      EXPECT(c != NULL);
      EXPECT(mfpff_sizes(c, 1, &nn, &nd) == MFPFF_OK && nn == 81 && nd == 243);
      EXPECT(mfpff_sizes(c, 2, &nn, &nd) == MFPFF_ERR_ARG);
      mfpff_destroy(c);
    } else {
      EXPECT(st == MFPFF_ERR_HIP || st == MFPFF_ERR_OOM);
      EXPECT(c == NULL);
    }
  }
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("ok\n");
  return 0;
}
