/* Exercises the oracle (assembly, ILUT, V-cycle, solver, CG, BiCGSTAB,
 * operator injection) under AddressSanitizer and UndefinedBehaviorSanitizer.
 * Built together with oracle/oracle.c; exit status 0 when every solve
 * converges or fails with the expected status. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  double tau, fill;
  int limit_mode, coarse_cycles, gs_variant, coarse_min, nu1, nu2;
  int ordering, nd_leaf;
  int mass_transfer;
  int projection;
  double diverge;
} orc_opts;
void *orc_create(int dim, int p, int nel, int geom, int rhs, int pde, const int *freq, const orc_opts *o,
                 int stage_mask, int *status);
void orc_default_opts(orc_opts *o);
void orc_free(void *s);
int orc_info(const void *s, int64_t *out);
int orc_get_vec(const void *s, int which, double *out);
int orc_get_csr(const void *s, int which, int lev, int64_t *dims, int64_t *rp, int *ci, double *v);
int orc_set_operator(void *s, int n, const int64_t *rp, const int *ci, const double *v);
int orc_solve(void *s, const double *b, double *x, double tol, int maxit, double *hist, int *iters);
int orc_bicgstab(void *s, const double *b, double *x, double tol, int maxit, int precond, double *hist, int *iters);
int orc_cg(void *s, const double *b, double *x, double tol, int maxit, int jacobi, int *iters);
double orc_l2_error(void *s, const double *uh);

static int run(int dim, int p, int nel, int geom, int pde, int mass, int proj, int mode) {
  orc_opts o;
  orc_default_opts(&o);
  o.mass_transfer = mass;
  o.projection = proj;
  o.limit_mode = mode;
  int freq[3] = {1, 1, 1}, st = 0;
  void *s = orc_create(dim, p, nel, geom, geom, pde, freq, &o, 0, &st);
  if (!s || st) return 1;
  int64_t info[32];
  orc_info(s, info);
  int n = (int)info[0];
  double *f = malloc(sizeof(double) * n), *x = calloc(n, sizeof(double)), *hist = malloc(sizeof(double) * 101);
  orc_get_vec(s, 0, f);
  int it = 0;
  int rc = orc_solve(s, f, x, 1e-8, 100, hist, &it);
  double e = orc_l2_error(s, x);
  for (int i = 0; i < n; ++i) x[i] = 0.0;
  int rc2 = orc_bicgstab(s, f, x, 1e-8, 100, 1, hist, &it);
  for (int i = 0; i < n; ++i) x[i] = 0.0;
  int rc3 = pde ? 0 : orc_cg(s, f, x, 1e-10, 10000, 1, &it);
  /* the injected negative identity has no positive pivots issue; an empty row fails */
  int64_t dims[3];
  orc_get_csr(s, 0, 0, dims, NULL, NULL, NULL);
  int64_t *rp = malloc(sizeof(int64_t) * (dims[0] + 1));
  int *ci = malloc(sizeof(int) * dims[2]);
  double *v = malloc(sizeof(double) * dims[2]);
  orc_get_csr(s, 0, 0, dims, rp, ci, v);
  for (int64_t k = rp[1]; k < rp[2]; ++k) v[k] = 0.0; /* row 1: all zero */
  int rc4 = orc_set_operator(s, n, rp, ci, v);
  printf("dim %d p %d nel %d geom %d pde %d mass %d proj %d mode %d: solve %d bicgstab %d cg %d zero-row %d L2 %.2e\n",
         dim, p, nel, geom, pde, mass, proj, mode, rc, rc2, rc3, rc4, e);
  free(f); free(x); free(hist); free(rp); free(ci); free(v);
  orc_free(s);
  return (rc == 0 && rc2 == 0 && rc3 == 0 && rc4 == 4) ? 0 : 1;
}

int main(void) {
  int bad = 0;
  bad |= run(2, 2, 16, 0, 0, 0, 0, 2);
  bad |= run(2, 3, 16, 1, 0, 0, 0, 0);
  bad |= run(2, 2, 16, 0, 1, 0, 0, 2);
  bad |= run(2, 3, 16, 0, 0, 1, 0, 1);
  bad |= run(2, 4, 16, 1, 0, 0, 1, 2);
  bad |= run(3, 2, 8, 0, 0, 0, 0, 2);
  printf(bad ? "FAILED\n" : "OK\n");
  return bad;
}
