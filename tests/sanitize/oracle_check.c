/* Every entry point of the C oracle on small lattices (2^4, 4^4, 2x4x2x4) under
 * AddressSanitizer / UndefinedBehaviorSanitizer: each call must return success and
 * finite results.  Prints "oracle_check ok" and exits 0 when every check holds. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ov_oracle.h"

typedef double complex cplx;
static int fails = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);      \
      ++fails;                                                            \
    }                                                                     \
  } while (0)

static unsigned long long rng = 88172645463325252ULL;
static double urand(void) { /* xorshift64: test data only */
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (double)(rng >> 11) / 9007199254740992.0 - 0.5;
}
static void fill(cplx *v, long n, double s) {
  for (long i = 0; i < n; ++i) v[i] = s * (urand() + I * urand());
}
static int finite_all(const cplx *v, long n) {
  for (long i = 0; i < n; ++i)
    if (!isfinite(creal(v[i])) || !isfinite(cimag(v[i]))) return 0;
  return 1;
}

static void run(int X, int Y, int Z, int T, int bc, int dirac) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.dims[0] = X; p.dims[1] = Y; p.dims[2] = Z; p.dims[3] = T;
  p.bc_t = bc;
  p.M0 = 1.0;
  p.m_re = 0.05;
  p.g_re = 0.3;
  p.n_poles = 12;
  p.lambda_min = 1e-2;
  p.lambda_max = 8.0;
  p.inner_tol = 1e-12;
  p.max_inner = 2000;
  p.dirac = dirac;
  CHECK(orc_init(&p) == 0);
  const long V = (long)X * Y * Z * T, N = 4 * V;
  cplx *phi = malloc(sizeof(cplx) * V), *in = malloc(sizeof(cplx) * N);
  cplx *out = malloc(sizeof(cplx) * N), *x = malloc(sizeof(cplx) * N);
  cplx *G = malloc(sizeof(cplx) * V), *F = malloc(sizeof(cplx) * V);
  fill(phi, V, 0.5);
  fill(in, N, 1.0);
  long long inner = 0;
  for (int op = ORC_OP_HW; op <= ORC_OP_MDAGM; ++op) {
    CHECK(orc_apply(&p, op, phi, in, out, &inner) == 0);
    CHECK(finite_all(out, N));
  }
  if (dirac == ORC_DIRAC_OVERLAP_MS) {
    orc_dw(&p, in, out);
    CHECK(finite_all(out, N));
    orc_hw(&p, in, out);
    CHECK(finite_all(out, N));
    orc_ms_stats ms;
    CHECK(orc_sign(&p, in, out, &ms) == 0 && ms.converged);
    double sig[3] = {0.1, 1.0, 10.0}, coef[3] = {1.0, 0.5, 0.25};
    cplx *ys = malloc(sizeof(cplx) * 3 * N);
    CHECK(orc_multishift(&p, 3, sig, coef, 1e-12, 2000, in, out, ys, &ms) == 0);
    CHECK(finite_all(ys, 3 * N));
    free(ys);
  }
  orc_cg_stats st;
  memset(x, 0, sizeof(cplx) * N);
  CHECK(orc_solve(&p, phi, in, x, 1e-10, 2000, &st) == 0);
  CHECK(orc_residual(&p, phi, in, x) <= 1e-10);
  double S = 0;
  CHECK(orc_force(&p, phi, in, 1e-10, 2000, &S, G, &st) == 0);
  CHECK(isfinite(S) && finite_all(G, V));
  double al[3] = {0.3, 0.2, 0.1}, be[3] = {0.05, 1.0, 20.0};
  CHECK(orc_rational(&p, phi, 0.5, 3, al, be, in, out, 1e-10, 2000) == 0);
  CHECK(finite_all(out, N));
  CHECK(orc_rational_force(&p, phi, 0.5, 3, al, be, in, 1e-10, 2000, &S, G) == 0);
  CHECK(isfinite(S) && finite_all(G, V));
  if (bc < 0 && T % 2 == 0) {
    CHECK(orc_m0inv(&p, 0, in, out, 1e-12, 2000) == 0);
    CHECK(orc_m0inv(&p, 1, in, out, 1e-12, 2000) == 0);
    CHECK(finite_all(out, N));
  }
  int nr = X / 2 + Y / 2 + Z / 2 + T / 2 + 1;
  double *f = malloc(sizeof(double) * nr);
  CHECK(orc_locality(&p, 0, f, nr) == 0);
  free(f);
  CHECK(orc_boson(&p, phi, &S, G, F) == 0);
  CHECK(isfinite(S) && finite_all(G, V) && finite_all(F, V));
  if (V <= 64) {
    cplx *pi = malloc(sizeof(cplx) * V), *eta = malloc(sizeof(cplx) * N);
    fill(pi, V, 1.0);
    double dH = 0, parts[8];
    int acc = 0;
    CHECK(orc_rhmc_trajectory_ex(&p, phi, pi, in, 2, 0.1, 0.5, 3, al, be, 0.5, 3, al, be, 0.5,
                                 1e-10, 2000, &dH, &acc, eta, parts) == 0);
    CHECK(isfinite(dH) && finite_all(eta, N));
    free(pi);
    free(eta);
  }
  free(phi); free(in); free(out); free(x); free(G); free(F);
}

int main(void) {
  cplx g[16];
  for (int mu = 0; mu < 5; ++mu) CHECK(orc_gamma(mu, g) == 0);
  double a[32], b[32], delta, d0;
  for (int n = 1; n <= 32; ++n) CHECK(orc_zolotarev(n, 1e-4, 8.0, a, b, &delta, &d0) == 0);
  double sn, cn, dn, K;
  orc_sncndn(0.3, 1e-10, &sn, &cn, &dn, &K);
  CHECK(isfinite(sn) && isfinite(K));
  run(2, 2, 2, 2, -1, ORC_DIRAC_OVERLAP_MS);
  run(2, 2, 2, 2, 1, ORC_DIRAC_OVERLAP_MS);
  run(2, 4, 2, 4, -1, ORC_DIRAC_OVERLAP_MS);
  run(4, 4, 4, 4, -1, ORC_DIRAC_OVERLAP_MS);
  run(2, 2, 2, 4, -1, ORC_DIRAC_OVERLAP_RAT);
  run(2, 2, 2, 4, -1, ORC_DIRAC_OVERLAP_EXACT);
  run(2, 2, 2, 4, -1, ORC_DIRAC_DSLASH);
  if (fails) {
    fprintf(stderr, "oracle_check: %d failures\n", fails);
    return 1;
  }
  printf("oracle_check ok\n");
  return 0;
}
