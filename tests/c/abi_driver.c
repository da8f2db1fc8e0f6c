/* A plain C (C99) client of libmlcc: the header compiles as C, and the calls
 * behave as include/mlcc.h states.
 *
 *   abi_driver            calls that need no device: argument errors and the
 *                         footprint estimate
 *   abi_driver gpu FILE   a small MLCC2 problem end to end on device 0 from
 *                         FILE (int32 O V J o v, then L [J][n][n] and eps [n]
 *                         as doubles): prints the ground-state energy and the
 *                         three lowest excitation energies
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mlcc.h"

static int fails = 0;
#define EXPECT(c)                                                     \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "abi_driver.c:%d: expected %s\n", __LINE__, #c); \
      ++fails;                                                        \
    }                                                                 \
  } while (0)

static int cpu_checks(void) {
  mlcc_problem_desc d;
  int64_t dims[8];
  double e = 0.0;
  mlcc_solver_opts o;
  uint64_t t = 0;
  uint64_t f1, f2, f3;
  memset(&d, 0, sizeof d);
  memset(&o, 0, sizeof o);
  d.n_occ = 8;
  d.n_vir = 40;
  d.n_chol = 100;
  d.n_occ_act = 5;
  d.n_vir_act = 25;
  d.model = MLCC_MLCC2;
  d.precision = MLCC_FP64;
  f1 = mlcc_request_footprint(&d, 3, NULL);
  d.n_chol = 200;
  f2 = mlcc_request_footprint(&d, 3, NULL);
  d.precision = MLCC_FP32;
  f3 = mlcc_request_footprint(&d, 3, NULL);
  EXPECT(f1 > 0 && f2 > f1 && f3 < f2);
  EXPECT(mlcc_request_footprint(NULL, 3, NULL) == 0);
  EXPECT(mlcc_problem_dims(NULL, dims) == MLCC_E_ARG);
  EXPECT(mlcc_set_amplitudes(NULL, NULL, NULL) == MLCC_E_ARG);
  EXPECT(mlcc_residual(NULL, NULL, NULL, NULL, &e) == MLCC_E_ARG);
  EXPECT(mlcc_ground_state(NULL, &o, NULL, &e, NULL) == MLCC_E_ARG);
  EXPECT(mlcc_jacobian_transform(NULL, 1, NULL, NULL) == MLCC_E_ARG);
  EXPECT(mlcc_davidson_solve(NULL, 1, &o, NULL, NULL, NULL) == MLCC_E_ARG);
  EXPECT(mlcc_submit(NULL, &d, 1, &o, &o, &t) == MLCC_E_ARG);
  EXPECT(mlcc_server_destroy(NULL) == MLCC_E_ARG);
  EXPECT(mlcc_problem_destroy(NULL) == MLCC_E_ARG);
  return fails;
}

static int gpu_run(const char *path) {
  FILE *f = fopen(path, "rb");
  int32_t hdr[5];
  int64_t n, nl;
  double *L, *eps, t1e = 0.0, w[3];
  mlcc_context *ctx = NULL;
  mlcc_problem *P = NULL;
  mlcc_problem_desc d;
  mlcc_solver_opts o;
  mlcc_info info;
  mlcc_status st;
  if (!f || fread(hdr, sizeof(int32_t), 5, f) != 5) return 2;
  n = (int64_t)hdr[0] + hdr[1];
  nl = (int64_t)hdr[2] * n * n;
  L = malloc(sizeof(double) * nl);
  eps = malloc(sizeof(double) * n);
  if (!L || !eps || fread(L, sizeof(double), nl, f) != (size_t)nl ||
      fread(eps, sizeof(double), n, f) != (size_t)n)
    return 2;
  fclose(f);
  memset(&d, 0, sizeof d);
  d.n_occ = hdr[0];
  d.n_vir = hdr[1];
  d.n_chol = hdr[2];
  d.n_occ_act = hdr[3];
  d.n_vir_act = hdr[4];
  d.model = MLCC_MLCC2;
  d.precision = MLCC_FP64;
  d.L = L;
  d.eps = eps;
  st = mlcc_context_create(0, NULL, 0, &ctx);
  if (st != MLCC_OK) {
    fprintf(stderr, "context: %s\n", mlcc_last_error(NULL));
    return 3;
  }
  st = mlcc_problem_create(ctx, &d, &P);
  free(L); /* the library copied the inputs */
  free(eps);
  if (st != MLCC_OK) {
    fprintf(stderr, "problem: %s\n", mlcc_last_error(ctx));
    return 3;
  }
  memset(&o, 0, sizeof o);
  o.tol = 1e-10;
  o.max_iter = 100;
  {
    double *t1 = malloc(sizeof(double) * hdr[0] * hdr[1]);
    st = mlcc_ground_state(P, &o, t1, &t1e, &info);
    free(t1);
  }
  EXPECT(st == MLCC_OK && info.converged == 1);
  o.tol = 1e-8;
  o.effective = 1;
  st = mlcc_davidson_solve(P, 3, &o, w, NULL, &info);
  EXPECT(st == MLCC_OK && info.converged == 1);
  printf("%.15e %.15e %.15e %.15e\n", t1e, w[0], w[1], w[2]);
  EXPECT(mlcc_problem_destroy(P) == MLCC_OK);
  EXPECT(mlcc_context_destroy(ctx) == MLCC_OK);
  return fails;
}

int main(int argc, char **argv) {
  if (argc > 2 && strcmp(argv[1], "gpu") == 0) return gpu_run(argv[2]);
  return cpu_checks();
}
