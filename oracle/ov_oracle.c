/*
 * ov_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Slow on purpose: full 4x4 gamma matrices, one vector operation per loop,
 * every shifted search direction kept explicitly.  OpenMP only splits the
 * site loops.  Nothing here is shared with the GPU library.
 *
 * Paper: Chen, Dzienkowski, Giedt, "Lattice Wess-Zumino model with
 * Ginsparg-Wilson fermions: one-loop results and GPU benchmarks" (arXiv:1005.3276).
 *   - lattice operators A = 1 - a D_W, D = (1 - A (A^dag A)^-1/2)/a: Sec. 2.2
 *   - gamma conventions: Sec. 2.1
 *   - fermion matrix with Yukawa coupling g: Sec. 7.1 (Pfaffian phase)
 *   - antiperiodic time for the fermion: Sec. 3.1 (mode analysis), Sec. 3.2
 *   - CG on MdagM for each system: Sec. 7.2 (pseudofermions), Sec. 7.3 (preconditioning)
 * The sign function is evaluated by Zolotarev's optimal rational approximation
 * (Akhiezer; Chiu et al. 2002; van den Eshof et al. 2002) with a multi-shift CG
 * (Jegerlehner 1996); the paper itself applies D exactly in momentum space.
 */
#include "ov_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ gamma */

/* Sec. 2.1: gamma_0 = [[0,1],[1,0]], gamma_i = [[0, i sigma_i], [-i sigma_i, 0]],
 * gamma_5 = diag(-1, 1) in 2x2 blocks.  Directions x,y,z use gamma_1,2,3 and
 * t uses gamma_0. */
static void build_gamma(int mu, cplx g[4][4]) {
  const cplx Im = _Complex_I;
  cplx s[3][2][2] = {
      {{0, 1}, {1, 0}},
      {{0, -Im}, {Im, 0}},
      {{1, 0}, {0, -1}},
  };
  memset(g, 0, sizeof(cplx) * 16);
  if (mu == 4) {
    g[0][0] = -1; g[1][1] = -1; g[2][2] = 1; g[3][3] = 1;
    return;
  }
  if (mu == 3) {
    for (int i = 0; i < 2; ++i) { g[i][i + 2] = 1; g[i + 2][i] = 1; }
    return;
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      g[i][j + 2] = Im * s[mu][i][j];
      g[i + 2][j] = -Im * s[mu][i][j];
    }
}

int orc_gamma(int mu, cplx *out16) {
  if (mu < 0 || mu > 4) return 1;
  cplx g[4][4];
  build_gamma(mu, g);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out16[4 * i + j] = g[i][j];
  return 0;
}

/* ------------------------------------------------------------- Zolotarev */

/* Jacobi elliptic functions by the arithmetic-geometric mean (Abramowitz &
 * Stegun 16.4), parameter m = 1 - m1 given through its complement so that
 * m1 ~ 1e-10 keeps full precision.  Long double throughout. */
static void sncndn_ld(long double u, long double m1, long double *sn, long double *cn,
                      long double *dn, long double *K) {
  long double a[80], c[80];
  long double A = 1.0L, B = sqrtl(m1);
  int N = 0;
  a[0] = 1.0L;
  c[0] = sqrtl(1.0L - m1);
  while (N < 70) {
    long double An = 0.5L * (A + B);
    long double Bn = sqrtl(A * B);
    long double Cn = 0.5L * (A - B);
    ++N;
    a[N] = An; c[N] = Cn;
    A = An; B = Bn;
    if (fabsl(Cn) <= LDBL_EPSILON * An) break;
  }
  *K = 3.14159265358979323846264338327950288L / (2.0L * a[N]);
  long double phi = ldexpl(a[N] * u, N);
  long double phi1 = phi;
  for (int n = N; n >= 1; --n) {
    phi1 = phi;
    phi = 0.5L * (phi + asinl(c[n] / a[n] * sinl(phi)));
  }
  *sn = sinl(phi);
  *cn = cosl(phi);
  *dn = cosl(phi) / cosl(phi1 - phi);
}

void orc_sncndn(double u, double m1, double *sn, double *cn, double *dn, double *K) {
  long double s, c, d, k;
  sncndn_ld(u, m1, &s, &c, &d, &k);
  *sn = (double)s; *cn = (double)c; *dn = (double)d; *K = (double)k;
}

/* product form f(x) = (x/lmin) prod_{l=1}^{n-1} (Y + c_{2l}) / prod_{l=1}^{n} (Y + c_{2l-1}),
 * Y = (x/lmin)^2; c[1..2n-1]. */
static long double zolo_f(long double x, long double lmin, int n, const long double *c) {
  long double y = (x / lmin) * (x / lmin);
  long double v = x / lmin;
  for (int l = 1; l <= n - 1; ++l) v *= (y + c[2 * l]);
  for (int l = 1; l <= n; ++l) v /= (y + c[2 * l - 1]);
  return v;
}

/* golden-section search for an extremum of zolo_f on [lo, hi] (log x). */
static long double zolo_refine(long double lo, long double hi, long double lmin, int n,
                               const long double *c, int want_max) {
  const long double gr = 0.61803398874989484820458683436563811L;
  long double a = logl(lo), b = logl(hi);
  long double x1 = b - gr * (b - a), x2 = a + gr * (b - a);
  long double f1 = zolo_f(expl(x1), lmin, n, c), f2 = zolo_f(expl(x2), lmin, n, c);
  for (int it = 0; it < 200 && (b - a) > 1e-15L; ++it) {
    int left = want_max ? (f1 > f2) : (f1 < f2);
    if (left) {
      b = x2; x2 = x1; f2 = f1;
      x1 = b - gr * (b - a); f1 = zolo_f(expl(x1), lmin, n, c);
    } else {
      a = x1; x1 = x2; f1 = f2;
      x2 = a + gr * (b - a); f2 = zolo_f(expl(x2), lmin, n, c);
    }
  }
  return zolo_f(expl(0.5L * (a + b)), lmin, n, c);
}

int orc_zolotarev(int n, double lmin_d, double lmax_d, double *a_out, double *b_out,
                  double *delta_out, double *d0_out) {
  if (n < 1 || n > ORC_MAX_POLES || !(lmin_d > 0) || !(lmax_d > lmin_d)) return 1;
  long double lmin = lmin_d, lmax = lmax_d;
  long double bb = (lmax / lmin) * (lmax / lmin); /* b = (lmax/lmin)^2 */
  long double m1 = 1.0L / bb;                     /* complementary parameter */
  long double c[2 * ORC_MAX_POLES + 1];
  long double sn, cn, dn, K;
  sncndn_ld(0.0L, m1, &sn, &cn, &dn, &K);
  /* c_l = sn^2/cn^2 at u = l K / (2n); for l > n use c_l c_{2n-l} = b. */
  for (int l = 1; l <= n; ++l) {
    long double u = (long double)l * K / (2.0L * n);
    sncndn_ld(u, m1, &sn, &cn, &dn, &K);
    c[l] = (sn * sn) / (cn * cn);
  }
  for (int l = n + 1; l <= 2 * n - 1; ++l) c[l] = bb / c[2 * n - l];

  /* extremes of f on [lmin, lmax]: dense log sampling, then refinement */
  enum { NS = 8000 };
  static long double xs[NS + 1], fs[NS + 1];
  long double fmax = -1.0L, fmin = 1e300L;
  for (int i = 0; i <= NS; ++i) {
    xs[i] = expl(logl(lmin) + (logl(lmax) - logl(lmin)) * i / NS);
    fs[i] = zolo_f(xs[i], lmin, n, c);
    if (fs[i] > fmax) fmax = fs[i];
    if (fs[i] < fmin) fmin = fs[i];
  }
  for (int i = 1; i < NS; ++i) {
    if (fs[i] >= fs[i - 1] && fs[i] >= fs[i + 1]) {
      long double v = zolo_refine(xs[i - 1], xs[i + 1], lmin, n, c, 1);
      if (v > fmax) fmax = v;
    }
    if (fs[i] <= fs[i - 1] && fs[i] <= fs[i + 1]) {
      long double v = zolo_refine(xs[i - 1], xs[i + 1], lmin, n, c, 0);
      if (v < fmin) fmin = v;
    }
  }
  long double d0 = 2.0L / (fmax + fmin);
  long double delta = (fmax - fmin) / (fmax + fmin);

  /* partial fractions R0(Y) = sum_k r_k / (Y + c_{2k-1}) */
  for (int k = 1; k <= n; ++k) {
    long double ck = c[2 * k - 1];
    long double num = 1.0L, den = 1.0L;
    for (int l = 1; l <= n - 1; ++l) num *= (c[2 * l] - ck);
    for (int l = 1; l <= n; ++l)
      if (l != k) den *= (c[2 * l - 1] - ck);
    long double rk = num / den;
    a_out[k - 1] = (double)(d0 * rk * lmin);
    b_out[k - 1] = (double)(ck * lmin * lmin);
  }
  if (delta_out) *delta_out = (double)delta;
  if (d0_out) *d0_out = (double)d0;
  return 0;
}

/* --------------------------------------------------------------- geometry */

static long long volume(const orc_params *p) {
  return (long long)p->dims[0] * p->dims[1] * p->dims[2] * p->dims[3];
}

/* neighbour of site i in direction mu, forward (dir = +1) or backward (-1);
 * *ph receives the boundary phase of the hop. */
static long long neighbour(const orc_params *p, long long i, int mu, int dir, double *ph) {
  int co[4];
  long long r = i;
  for (int d = 0; d < 4; ++d) { co[d] = (int)(r % p->dims[d]); r /= p->dims[d]; }
  *ph = 1.0;
  int L = p->dims[mu];
  int nc = co[mu] + dir;
  if (nc == L) { nc = 0; if (mu == 3) *ph = (double)p->bc_t; }
  if (nc == -1) { nc = L - 1; if (mu == 3) *ph = (double)p->bc_t; }
  co[mu] = nc;
  return co[0] + (long long)p->dims[0] * (co[1] + (long long)p->dims[1] *
                                          (co[2] + (long long)p->dims[2] * co[3]));
}

/* ------------------------------------------------------------ vector ops */

static cplx *vec_new(long long n) { return (cplx *)calloc((size_t)n, sizeof(cplx)); }

static double vec_norm2(long long n, const cplx *x) {
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (long long i = 0; i < n; ++i) s += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
  return s;
}

static cplx vec_dot(long long n, const cplx *x, const cplx *y) { /* x^dag y */
  double sr = 0.0, si = 0.0;
#pragma omp parallel for reduction(+ : sr, si) schedule(static)
  for (long long i = 0; i < n; ++i) {
    cplx v = conj(x[i]) * y[i];
    sr += creal(v);
    si += cimag(v);
  }
  return sr + _Complex_I * si;
}

static void vec_copy(long long n, cplx *y, const cplx *x) { memcpy(y, x, (size_t)n * sizeof(cplx)); }

static void vec_axpy(long long n, cplx a, const cplx *x, cplx *y) { /* y += a x */
#pragma omp parallel for schedule(static)
  for (long long i = 0; i < n; ++i) y[i] += a * x[i];
}

static void vec_xpay(long long n, const cplx *x, cplx a, cplx *y) { /* y = x + a y */
#pragma omp parallel for schedule(static)
  for (long long i = 0; i < n; ++i) y[i] = x[i] + a * y[i];
}

static void apply_g5(long long V, const cplx *in, cplx *out) {
  cplx g5[4][4];
  build_gamma(4, g5);
#pragma omp parallel for schedule(static)
  for (long long x = 0; x < V; ++x) {
    cplx v[4];
    for (int s = 0; s < 4; ++s) {
      v[s] = 0;
      for (int t = 0; t < 4; ++t) v[s] += g5[s][t] * in[4 * x + t];
    }
    for (int s = 0; s < 4; ++s) out[4 * x + s] = v[s];
  }
}

/* ------------------------------------------------------------- operators */

void orc_dw(const orc_params *p, const cplx *in, cplx *out) {
  long long V = volume(p);
  cplx gm[4][4][4], one[4][4];
  for (int mu = 0; mu < 4; ++mu) build_gamma(mu, gm[mu]);
  memset(one, 0, sizeof(one));
  for (int s = 0; s < 4; ++s) one[s][s] = 1;
  double diag = 4.0 - p->M0;
#pragma omp parallel for schedule(static)
  for (long long x = 0; x < V; ++x) {
    cplx acc[4];
    for (int s = 0; s < 4; ++s) acc[s] = diag * in[4 * x + s];
    for (int mu = 0; mu < 4; ++mu) {
      double phf, phb;
      long long xf = neighbour(p, x, mu, +1, &phf);
      long long xb = neighbour(p, x, mu, -1, &phb);
      for (int s = 0; s < 4; ++s) {
        cplx v = 0;
        for (int t = 0; t < 4; ++t) {
          v += (one[s][t] - gm[mu][s][t]) * phf * in[4 * xf + t];
          v += (one[s][t] + gm[mu][s][t]) * phb * in[4 * xb + t];
        }
        acc[s] -= 0.5 * v;
      }
    }
    for (int s = 0; s < 4; ++s) out[4 * x + s] = acc[s];
  }
}

void orc_hw(const orc_params *p, const cplx *in, cplx *out) {
  long long V = volume(p);
  cplx *tmp = vec_new(4 * V);
  orc_dw(p, in, tmp);
  apply_g5(V, tmp, out);
  free(tmp);
}

/* -------------------------------------------------------- multi-shift CG */

/* Jegerlehner's multi-shift CG: one Krylov space of H_W^2 serves every
 * shifted system (H_W^2 + sig_k) y_k = src.  Base shift 0 (H_W^2 >= 1 for the
 * free Wilson operator at M0 = 1). */
int orc_multishift(const orc_params *p, int n, const double *sig, const double *coef,
                   double tol, int maxit, const cplx *src, cplx *acc, cplx *ys,
                   orc_ms_stats *st) {
  long long V = volume(p), N = 4 * V;
  if (acc) memset(acc, 0, (size_t)N * sizeof(cplx));
  if (ys) memset(ys, 0, (size_t)n * N * sizeof(cplx));
  double srcn = sqrt(vec_norm2(N, src));
  if (st) { st->iters = 0; st->converged = 1; st->max_shift_res = 0.0; }
  if (srcn == 0.0) return 0;

  cplx *r = vec_new(N), *P = vec_new(N), *t = vec_new(N), *w = vec_new(N);
  cplx **pk = (cplx **)malloc(sizeof(cplx *) * n);
  double *zeta = malloc(sizeof(double) * n), *zeta_old = malloc(sizeof(double) * n);
  double *zeta_new = malloc(sizeof(double) * n);
  int *active = malloc(sizeof(int) * n);
  vec_copy(N, r, src);
  vec_copy(N, P, src);
  for (int k = 0; k < n; ++k) {
    pk[k] = vec_new(N);
    vec_copy(N, pk[k], src);
    zeta[k] = zeta_old[k] = 1.0;
    active[k] = 1;
  }
  double alpha_old = 1.0, beta_old = 0.0;
  double rr = vec_norm2(N, r);
  int it = 0, nactive = n;
  while (nactive > 0 && it < maxit) {
    orc_hw(p, P, t);
    orc_hw(p, t, w);
    double pw = creal(vec_dot(N, P, w));
    double alpha = rr / pw;
    for (int k = 0; k < n; ++k) {
      if (!active[k]) continue;
      zeta_new[k] = zeta[k] * zeta_old[k] * alpha_old /
                    (alpha_old * zeta_old[k] * (1.0 + alpha * sig[k]) +
                     alpha * beta_old * (zeta_old[k] - zeta[k]));
      double ak = alpha * zeta_new[k] / zeta[k];
      if (ys) vec_axpy(N, ak, pk[k], ys + (long long)k * N);
      if (acc) vec_axpy(N, coef[k] * ak, pk[k], acc);
    }
    vec_axpy(N, -alpha, w, r);
    double rr_new = vec_norm2(N, r);
    double beta = rr_new / rr;
    for (int k = 0; k < n; ++k) {
      if (!active[k]) continue;
      double bk = beta * (zeta_new[k] / zeta[k]) * (zeta_new[k] / zeta[k]);
      /* p_k = zeta_new r + bk p_k */
      cplx *q = pk[k];
#pragma omp parallel for schedule(static)
      for (long long i = 0; i < N; ++i) q[i] = zeta_new[k] * r[i] + bk * q[i];
    }
    vec_xpay(N, r, beta, P);
    for (int k = 0; k < n; ++k) {
      if (!active[k]) continue;
      zeta_old[k] = zeta[k];
      zeta[k] = zeta_new[k];
    }
    alpha_old = alpha;
    beta_old = beta;
    rr = rr_new;
    ++it;
    for (int k = 0; k < n; ++k) {
      if (active[k] && fabs(zeta[k]) * sqrt(rr) <= tol * srcn) {
        active[k] = 0;
        --nactive;
      }
    }
  }
  if (st) {
    double mx = 0.0;
    for (int k = 0; k < n; ++k) {
      double v = fabs(zeta[k]) * sqrt(rr) / srcn;
      if (v > mx) mx = v;
    }
    st->iters = it;
    st->converged = nactive == 0;
    st->max_shift_res = mx;
  }
  for (int k = 0; k < n; ++k) free(pk[k]);
  free(pk); free(zeta); free(zeta_old); free(zeta_new); free(active);
  free(r); free(P); free(t); free(w);
  return nactive == 0 ? 0 : 2;
}

int orc_init(orc_params *p) {
  for (int d = 0; d < 4; ++d)
    if (p->dims[d] < 2) return 1;
  if (p->bc_t != 1 && p->bc_t != -1) return 1;
  if (p->dirac < ORC_DIRAC_OVERLAP_MS || p->dirac > ORC_DIRAC_DSLASH) return 1;
  /* Dslash needs 1 - D/2 invertible at every lattice momentum: no momentum with
   * every p_mu in {0, pi}, which antiperiodic time with T even guarantees */
  if (p->dirac == ORC_DIRAC_DSLASH && (p->bc_t != -1 || (p->dims[3] & 1))) return 1;
  if (p->n_poles < 1 || p->n_poles > ORC_MAX_POLES) return 1;
  if (p->inner_tol <= 0 || p->max_inner < 1) return 1;
  return orc_zolotarev(p->n_poles, p->lambda_min, p->lambda_max, p->a, p->b, &p->delta,
                       &p->d0);
}

int orc_sign(const orc_params *p, const cplx *in, cplx *out, orc_ms_stats *st) {
  long long N = 4 * volume(p);
  cplx *acc = vec_new(N);
  int rc = orc_multishift(p, p->n_poles, p->b, p->a, p->inner_tol, p->max_inner, in, acc,
                          NULL, st);
  orc_hw(p, acc, out);
  free(acc);
  return rc;
}

/* ------------------------------------------------ momentum-space operators
 * Sec. 7.2: without a gauge field the Dirac operator is diagonal in momentum
 * space.  For a field ~ exp(+i p.x) the Wilson operator of orc_dw is the 4x4
 * matrix D_W(p) = (4 - M0 - sum_mu cos p_mu) + i sum_mu gamma_mu sin p_mu, and
 * H_W(p) = g5 D_W(p) with H_W(p)^2 = s2(p) 1.  Momenta: p_mu = 2 pi k / L_mu,
 * and (2 k + 1) pi / T in time for antiperiodic fermions (Sec. 3.1). */
static double momentum(const orc_params *p, int mu, int k) {
  const double shift = (mu == 3 && p->bc_t < 0) ? 1.0 : 0.0;
  return M_PI * (2.0 * k + shift) / p->dims[mu];
}

static void mat4_mul(cplx a[4][4], cplx b[4][4], cplx out[4][4]) {
  cplx t[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx v = 0;
      for (int k = 0; k < 4; ++k) v += a[i][k] * b[k][j];
      t[i][j] = v;
    }
  memcpy(out, t, sizeof(t));
}

/* inverse by Gauss-Jordan elimination with partial pivoting; 1 if singular */
static int mat4_inv(cplx a[4][4], cplx out[4][4]) {
  cplx m[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 8; ++j) m[i][j] = j < 4 ? a[i][j] : (j - 4 == i ? 1.0 : 0.0);
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (cabs(m[r][c]) > cabs(m[piv][c])) piv = r;
    if (cabs(m[piv][c]) < 1e-300) return 1;
    if (piv != c)
      for (int j = 0; j < 8; ++j) { cplx t = m[c][j]; m[c][j] = m[piv][j]; m[piv][j] = t; }
    cplx d = m[c][c];
    for (int j = 0; j < 8; ++j) m[c][j] /= d;
    for (int r = 0; r < 4; ++r)
      if (r != c) {
        cplx f = m[r][c];
        for (int j = 0; j < 8; ++j) m[r][j] -= f * m[c][j];
      }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out[i][j] = m[i][j + 4];
  return 0;
}

/* D(p) of form p->dirac (or its adjoint): D_ov = 1 + g5 eps(p), eps = H_W(p) R
 * with R = sum_k a_k / (s2 + b_k) (rational) or 1 / sqrt(s2) (exact), and
 * Dslash = (1 - D_ov / 2)^-1 D_ov (Sec. 2.2). */
static int dirac_symbol(const orc_params *p, const double pm[4], int dag, cplx D[4][4]) {
  cplx gm[5][4][4];
  for (int mu = 0; mu < 5; ++mu) build_gamma(mu, gm[mu]);
  double w = 4.0 - p->M0, s2 = 0.0;
  for (int mu = 0; mu < 4; ++mu) w -= cos(pm[mu]);
  cplx DW[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      DW[i][j] = (i == j) ? w : 0.0;
      for (int mu = 0; mu < 4; ++mu) DW[i][j] += _Complex_I * sin(pm[mu]) * gm[mu][i][j];
    }
  s2 = w * w;
  for (int mu = 0; mu < 4; ++mu) s2 += sin(pm[mu]) * sin(pm[mu]);
  double R = 0.0;
  if (p->dirac == ORC_DIRAC_OVERLAP_RAT)
    for (int k = 0; k < p->n_poles; ++k) R += p->a[k] / (s2 + p->b[k]);
  else
    R = 1.0 / sqrt(s2);
  cplx H[4][4], eps[4][4], g5eps[4][4];
  mat4_mul(gm[4], DW, H);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) eps[i][j] = H[i][j] * R;
  mat4_mul(gm[4], eps, g5eps);
  cplx Dov[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) Dov[i][j] = (i == j ? 1.0 : 0.0) + g5eps[i][j];
  cplx out[4][4];
  if (p->dirac == ORC_DIRAC_DSLASH) {
    cplx A[4][4], Ai[4][4];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) A[i][j] = (i == j ? 1.0 : 0.0) - 0.5 * Dov[i][j];
    if (mat4_inv(A, Ai)) return 1;
    mat4_mul(Ai, Dov, out);
  } else {
    memcpy(out, Dov, sizeof(out));
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) D[i][j] = dag ? conj(out[j][i]) : out[i][j];
  return 0;
}

/* out = D in (dag: D^dag in) through the plain 4-D discrete Fourier transform
 *   in~(p) = sum_x exp(-i p.x) in(x),   out(x) = 1/V sum_p exp(+i p.x) D(p) in~(p). */
static int momentum_apply(const orc_params *p, int dag, const cplx *in, cplx *out) {
  const int L[4] = {p->dims[0], p->dims[1], p->dims[2], p->dims[3]};
  const long long V = volume(p);
  cplx *ph[4];  /* ph[mu][k * L + x] = exp(-i p_mu(k) x) */
  for (int mu = 0; mu < 4; ++mu) {
    ph[mu] = vec_new((long long)L[mu] * L[mu]);
    for (int k = 0; k < L[mu]; ++k)
      for (int x = 0; x < L[mu]; ++x) ph[mu][k * L[mu] + x] = cexp(-_Complex_I * momentum(p, mu, k) * x);
  }
  cplx *hat = vec_new(4 * V);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(|| : bad)
  for (long long kk = 0; kk < V; ++kk) {
    long long r = kk;
    const int kx = r % L[0]; r /= L[0];
    const int ky = r % L[1]; r /= L[1];
    const int kz = r % L[2];
    const int kt = (int)(r / L[2]);
    cplx acc[4] = {0, 0, 0, 0};
    for (long long i = 0; i < V; ++i) {
      long long q = i;
      const int x = q % L[0]; q /= L[0];
      const int y = q % L[1]; q /= L[1];
      const int z = q % L[2];
      const int t = (int)(q / L[2]);
      const cplx e = ph[0][kx * L[0] + x] * ph[1][ky * L[1] + y] * ph[2][kz * L[2] + z] *
                     ph[3][kt * L[3] + t];
      for (int s = 0; s < 4; ++s) acc[s] += e * in[4 * i + s];
    }
    const double pm[4] = {momentum(p, 0, kx), momentum(p, 1, ky), momentum(p, 2, kz),
                          momentum(p, 3, kt)};
    cplx D[4][4] = {{0}};
    if (dirac_symbol(p, pm, dag, D)) bad = 1;
    for (int s = 0; s < 4; ++s) {
      cplx v = 0;
      for (int t = 0; t < 4; ++t) v += D[s][t] * acc[t];
      hat[4 * kk + s] = v;
    }
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (long long i = 0; i < V; ++i) {
    long long q = i;
    const int x = q % L[0]; q /= L[0];
    const int y = q % L[1]; q /= L[1];
    const int z = q % L[2];
    const int t = (int)(q / L[2]);
    cplx acc[4] = {0, 0, 0, 0};
    for (long long kk = 0; kk < V; ++kk) {
      long long r = kk;
      const int kx = r % L[0]; r /= L[0];
      const int ky = r % L[1]; r /= L[1];
      const int kz = r % L[2];
      const int kt = (int)(r / L[2]);
      const cplx e = conj(ph[0][kx * L[0] + x] * ph[1][ky * L[1] + y] * ph[2][kz * L[2] + z] *
                          ph[3][kt * L[3] + t]);
      for (int s = 0; s < 4; ++s) acc[s] += e * hat[4 * kk + s];
    }
    for (int s = 0; s < 4; ++s) out[4 * i + s] = acc[s] / (double)V;
  }
  for (int mu = 0; mu < 4; ++mu) free(ph[mu]);
  free(hat);
  return bad;
}

/* Yukawa term added to out: c+ P+ in + c- P- in (dag = 0) or its adjoint (dag = 1). */
static void add_yukawa(const orc_params *p, const cplx *phi, const cplx *in, cplx *out,
                       int dag) {
  long long V = volume(p);
  cplx g5[4][4];
  build_gamma(4, g5);
  cplx m = p->m_re + _Complex_I * p->m_im;
  cplx g = p->g_re + _Complex_I * p->g_im;
#pragma omp parallel for schedule(static)
  for (long long x = 0; x < V; ++x) {
    cplx cp = m + g * phi[x];
    cplx cm = conj(m) + conj(g) * conj(phi[x]);
    if (dag) { cp = conj(cp); cm = conj(cm); }
    for (int s = 0; s < 4; ++s) {
      cplx v = 0;
      for (int t = 0; t < 4; ++t) {
        double id = (s == t) ? 1.0 : 0.0;
        cplx pp = 0.5 * (id + g5[s][t]); /* P+ */
        cplx pm = 0.5 * (id - g5[s][t]); /* P- */
        v += (cp * pp + cm * pm) * in[4 * x + t];
      }
      out[4 * x + s] += v;
    }
  }
}

static int apply_one(const orc_params *p, int op, const cplx *phi, const cplx *in, cplx *out,
                     long long *inner) {
  long long V = volume(p), N = 4 * V;
  orc_ms_stats st = {0, 1, 0.0};
  int rc = 0;
  cplx *tmp = vec_new(N), *eps = vec_new(N);
  if (p->dirac != ORC_DIRAC_OVERLAP_MS && op != ORC_OP_HW) {
    if (op != ORC_OP_DOV && op != ORC_OP_M && op != ORC_OP_DOV_DAG && op != ORC_OP_M_DAG) {
      rc = 1;
    } else {
      const int dag = (op == ORC_OP_DOV_DAG || op == ORC_OP_M_DAG);
      rc = momentum_apply(p, dag, in, out);
      if (op == ORC_OP_M || op == ORC_OP_M_DAG) add_yukawa(p, phi, in, out, dag);
    }
    free(tmp);
    free(eps);
    return rc;
  }
  switch (op) {
    case ORC_OP_HW:
      orc_hw(p, in, out);
      break;
    case ORC_OP_DOV:
    case ORC_OP_M:
      rc = orc_sign(p, in, eps, &st);
      apply_g5(V, eps, tmp);
      for (long long i = 0; i < N; ++i) out[i] = in[i] + tmp[i];
      if (op == ORC_OP_M) add_yukawa(p, phi, in, out, 0);
      break;
    case ORC_OP_DOV_DAG:
    case ORC_OP_M_DAG:
      apply_g5(V, in, tmp);
      rc = orc_sign(p, tmp, eps, &st);
      for (long long i = 0; i < N; ++i) out[i] = in[i] + eps[i];
      if (op == ORC_OP_M_DAG) add_yukawa(p, phi, in, out, 1);
      break;
    default:
      rc = 1;
  }
  if (inner) *inner += st.iters;
  free(tmp);
  free(eps);
  return rc;
}

int orc_apply(const orc_params *p, int op, const cplx *phi, const cplx *in, cplx *out,
              long long *inner) {
  if (op == ORC_OP_MDAGM) {
    long long N = 4 * volume(p);
    cplx *u = vec_new(N);
    int rc = apply_one(p, ORC_OP_M, phi, in, u, inner);
    int rc2 = apply_one(p, ORC_OP_M_DAG, phi, u, out, inner);
    free(u);
    return rc ? rc : rc2;
  }
  return apply_one(p, op, phi, in, out, inner);
}

double orc_residual(const orc_params *p, const cplx *phi, const cplx *b, const cplx *x) {
  long long N = 4 * volume(p);
  cplx *q = vec_new(N);
  orc_apply(p, ORC_OP_MDAGM, phi, x, q, NULL);
  for (long long i = 0; i < N; ++i) q[i] = b[i] - q[i];
  double res = sqrt(vec_norm2(N, q) / vec_norm2(N, b));
  free(q);
  return res;
}

/* CG on MdagM x = b (Sec. 7.3 states the problem), x0 = 0.  The true residual is
 * recomputed every 25 iterations and whenever the recursive one meets tol; the
 * iteration ends only on the true residual, restarting from it if needed. */
/* CG on (MdagM + shift) x = b from x = 0, stopping on the true relative residual. */
static int cg_mdagm(const orc_params *p, const cplx *phi, double shift, const cplx *b, cplx *x,
                    double tol, int maxit, orc_cg_stats *st) {
  long long N = 4 * volume(p);
  long long inner = 0;
  memset(x, 0, (size_t)N * sizeof(cplx));
  double bn = sqrt(vec_norm2(N, b));
  if (st) { st->iters = 0; st->converged = 1; st->inner_iters = 0; st->true_rel_res = 0; }
  if (bn == 0.0) return 0;
  cplx *r = vec_new(N), *pv = vec_new(N), *q = vec_new(N), *rt = vec_new(N);
  vec_copy(N, r, b);
  vec_copy(N, pv, r);
  double rr = vec_norm2(N, r);
  int it = 0, conv = 0;
  double true_res = 1.0;
  while (it < maxit) {
    orc_apply(p, ORC_OP_MDAGM, phi, pv, q, &inner);
    vec_axpy(N, shift, pv, q);
    double pq = creal(vec_dot(N, pv, q));
    double alpha = rr / pq;
    vec_axpy(N, alpha, pv, x);
    vec_axpy(N, -alpha, q, r);
    double rr_new = vec_norm2(N, r);
    ++it;
    if (sqrt(rr_new) <= tol * bn || it % 25 == 0) {
      orc_apply(p, ORC_OP_MDAGM, phi, x, rt, &inner);
      vec_axpy(N, shift, x, rt);
      for (long long i = 0; i < N; ++i) rt[i] = b[i] - rt[i];
      double rtn = vec_norm2(N, rt);
      true_res = sqrt(rtn) / bn;
      if (true_res <= tol) { conv = 1; break; }
      if (sqrt(rr_new) <= tol * bn) { /* recursive residual drifted: restart */
        vec_copy(N, r, rt);
        vec_copy(N, pv, r);
        rr = rtn;
        continue;
      }
    }
    double beta = rr_new / rr;
    vec_xpay(N, r, beta, pv);
    rr = rr_new;
  }
  if (!conv) {
    orc_apply(p, ORC_OP_MDAGM, phi, x, rt, &inner);
    vec_axpy(N, shift, x, rt);
    for (long long i = 0; i < N; ++i) rt[i] = b[i] - rt[i];
    true_res = sqrt(vec_norm2(N, rt)) / bn;
  }
  if (st) {
    st->iters = it;
    st->converged = conv;
    st->inner_iters = inner;
    st->true_rel_res = true_res;
  }
  free(r); free(pv); free(q); free(rt);
  return conv ? 0 : 2;
}

int orc_solve(const orc_params *p, const cplx *phi, const cplx *b, cplx *x, double tol,
              int maxit, orc_cg_stats *st) {
  return cg_mdagm(p, phi, 0.0, b, x, tol, maxit, st);
}

/* HMC force of S = xi^dag (MdagM)^-1 xi.  With X = (MdagM)^-1 xi and Y = M X,
 * dS = -2 Re[ Y^dag dM X ] and dM = g P+ dphi + g* P- dphi*, so
 *   dS/dphi_x = -g [ Y_x^dag P+ X_x + X_x^dag P- Y_x ],
 *   G_x = dS/dRe phi_x + i dS/dIm phi_x = 2 conj(dS/dphi_x)   (S real). */
/* G_x += w * 2 conj(dS/dphi_x) for dS/dphi_x = -g [ Y_x^dag P+ X_x + X_x^dag P- Y_x ]. */
static void force_density(const orc_params *p, const cplx *X, const cplx *Y, double w, cplx *G) {
  long long V = volume(p);
  cplx g5[4][4];
  build_gamma(4, g5);
  cplx g = p->g_re + _Complex_I * p->g_im;
#pragma omp parallel for schedule(static)
  for (long long x = 0; x < V; ++x) {
    cplx t1 = 0, t2 = 0;
    for (int s = 0; s < 4; ++s)
      for (int t = 0; t < 4; ++t) {
        double id = (s == t) ? 1.0 : 0.0;
        cplx pp = 0.5 * (id + g5[s][t]);
        cplx pm = 0.5 * (id - g5[s][t]);
        t1 += conj(Y[4 * x + s]) * pp * X[4 * x + t];
        t2 += conj(X[4 * x + s]) * pm * Y[4 * x + t];
      }
    cplx dS = -g * (t1 + t2);
    G[x] += w * 2.0 * conj(dS);
  }
}

/* HMC force of S = xi^dag (MdagM)^-1 xi.  With X = (MdagM)^-1 xi and Y = M X,
 * dS = -2 Re[ Y^dag dM X ] and dM = g P+ dphi + g* P- dphi*, so
 *   dS/dphi_x = -g [ Y_x^dag P+ X_x + X_x^dag P- Y_x ],
 *   G_x = dS/dRe phi_x + i dS/dIm phi_x = 2 conj(dS/dphi_x)   (S real). */
int orc_force(const orc_params *p, const cplx *phi, const cplx *xi, double tol, int maxit,
              double *S, cplx *G, orc_cg_stats *st) {
  long long V = volume(p), N = 4 * V;
  cplx *X = vec_new(N), *Y = vec_new(N);
  int rc = orc_solve(p, phi, xi, X, tol, maxit, st);
  long long inner = 0;
  orc_apply(p, ORC_OP_M, phi, X, Y, &inner);
  if (st) st->inner_iters += inner;
  memset(G, 0, (size_t)V * sizeof(cplx));
  force_density(p, X, Y, 1.0, G);
  *S = creal(vec_dot(N, xi, X));
  free(X);
  free(Y);
  return rc;
}

/* Rational functions of MdagM for RHMC (Sec. 7.3, pseudofermion heatbath and
 * action): out = a0 in + sum_i alpha_i (MdagM + beta_i)^-1 in, each shifted
 * system solved by its own CG as the paper does. */
int orc_rational(const orc_params *p, const cplx *phi, double a0, int n, const double *alpha,
                 const double *beta, const cplx *in, cplx *out, double tol, int maxit) {
  long long N = 4 * volume(p);
  cplx *X = vec_new(N);
  int rc = 0;
  for (long long i = 0; i < N; ++i) out[i] = a0 * in[i];
  for (int k = 0; k < n; ++k) {
    int r = cg_mdagm(p, phi, beta[k], in, X, tol, maxit, NULL);
    if (r) rc = r;
    vec_axpy(N, alpha[k], X, out);
  }
  free(X);
  return rc;
}

/* Force of S = Re xi^dag R(MdagM) xi, R(x) = a0 + sum_i alpha_i / (x + beta_i):
 * with X_i = (MdagM + beta_i)^-1 xi, Y_i = M X_i, dS = -sum_i alpha_i 2 Re[Y_i^dag dM X_i],
 * so G = sum_i alpha_i G(X_i, Y_i) with the density of orc_force. */
int orc_rational_force(const orc_params *p, const cplx *phi, double a0, int n,
                       const double *alpha, const double *beta, const cplx *xi, double tol,
                       int maxit, double *S, cplx *G) {
  long long V = volume(p), N = 4 * V;
  cplx *X = vec_new(N), *Y = vec_new(N);
  long long inner = 0;
  int rc = 0;
  memset(G, 0, (size_t)V * sizeof(cplx));
  double s = a0 * vec_norm2(N, xi);
  for (int k = 0; k < n; ++k) {
    int r = cg_mdagm(p, phi, beta[k], xi, X, tol, maxit, NULL);
    if (r) rc = r;
    orc_apply(p, ORC_OP_M, phi, X, Y, &inner);
    force_density(p, X, Y, alpha[k], G);
    s += alpha[k] * creal(vec_dot(N, xi, X));
  }
  *S = s;
  free(X);
  free(Y);
  return rc;
}

/* Free-field preconditioner of Sec. 7.3: M0 is the fermion matrix at phi = 0
 * (same operator, same rational sign), and the preconditioned problem uses
 * M0^-1 and M0^-dag.  Taken from their definitions:
 *   M0^-1 v   = (M0^dag M0)^-1 M0^dag v,
 *   M0^-dag v = M0 (M0^dag M0)^-1 v,
 * with the CG of orc_solve on MdagM at phi = 0 (true relative residual <= tol). */
int orc_m0inv(const orc_params *p, int dag, const cplx *in, cplx *out, double tol, int maxit) {
  long long V = volume(p), N = 4 * V;
  cplx *phi0 = vec_new(V), *t = vec_new(N);
  long long inner = 0;
  int rc;
  if (!dag) {
    orc_apply(p, ORC_OP_M_DAG, phi0, in, t, &inner);
    rc = orc_solve(p, phi0, t, out, tol, maxit, NULL);
  } else {
    rc = orc_solve(p, phi0, in, t, tol, maxit, NULL);
    orc_apply(p, ORC_OP_M, phi0, t, out, &inner);
  }
  free(phi0);
  free(t);
  return rc;
}

/* Locality probe of Sec. 3.2: psi = D eta for a unit point source eta at the
 * origin in spin component spin (D of form p->dirac; for the paper's probe,
 * Dslash), and f(r) = max { ||psi(x)|| : ||x||_1 = r } with the taxi-driver
 * distance ||x||_1 = sum_mu min(x_mu, L_mu - x_mu).  f[0 .. nr-1]; returns 1 if
 * nr is smaller than the largest distance + 1. */
int orc_locality(const orc_params *p, int spin, double *f, int nr) {
  long long V = volume(p), N = 4 * V;
  int rmax = 0;
  for (int mu = 0; mu < 4; ++mu) rmax += p->dims[mu] / 2;
  if (nr < rmax + 1 || spin < 0 || spin > 3) return 1;
  cplx *eta = vec_new(N), *psi = vec_new(N);
  eta[spin] = 1.0;
  long long inner = 0;
  int rc = orc_apply(p, ORC_OP_DOV, NULL, eta, psi, &inner);
  for (int r = 0; r < nr; ++r) f[r] = 0.0;
  for (long long i = 0; i < V; ++i) {
    long long q = i;
    int r = 0;
    for (int mu = 0; mu < 4; ++mu) {
      const int L = p->dims[mu];
      const int x = (int)(q % L);
      q /= L;
      r += x < L - x ? x : L - x;
    }
    double n2 = 0.0;
    for (int s = 0; s < 4; ++s) n2 += creal(psi[4 * i + s] * conj(psi[4 * i + s]));
    if (sqrt(n2) > f[r]) f[r] = sqrt(n2);
  }
  free(eta);
  free(psi);
  return rc;
}

/* ------------------------------------------------ RHMC (Sec. 7.3, eq. acws)
 * Bosonic part of the action (a = 1), for a periodic complex scalar phi:
 *   S_B = sum_x [ 2 conj(phi) (D_2 phi) + conj(W') ((1 - D_2/2) W') ],
 * D_2 the scalar part of the exact-sign overlap operator (D(p) = D_2(p) + gamma
 * part; D_2(p) = 1 + w(p)/s(p), so D^dag D = 2 D_2), W' = m phi + lam phi^2 with
 * lam = g/2: the Yukawa coefficient g of M is the paper's 2g (eq. fmat), so that
 * M's Yukawa term is W''(phi) = m + g phi.
 *   G = dS/dRe phi + i dS/dIm phi = 2 [ 2 D_2 phi + conj(W''(phi)) (1 - D_2/2) W' ],
 *   F = -(1 - D_2/2) conj(W')   (the auxiliary field at the stationary point of
 *                                eq. lata).                                      */
static void scalar_d2_apply(const orc_params *p, int which, const cplx *in, cplx *out) {
  /* which 0: D_2, 1: 1 - D_2/2 ; periodic momenta in every direction */
  const int L[4] = {p->dims[0], p->dims[1], p->dims[2], p->dims[3]};
  const long long V = volume(p);
  cplx *hat = vec_new(V);
#pragma omp parallel for schedule(dynamic, 16)
  for (long long kk = 0; kk < V; ++kk) {
    long long r = kk;
    int k[4];
    for (int mu = 0; mu < 4; ++mu) { k[mu] = (int)(r % L[mu]); r /= L[mu]; }
    cplx acc = 0;
    for (long long i = 0; i < V; ++i) {
      long long q = i;
      double ph = 0.0;
      for (int mu = 0; mu < 4; ++mu) {
        const int x = (int)(q % L[mu]);
        q /= L[mu];
        ph += 2.0 * M_PI * (double)k[mu] * x / L[mu];
      }
      acc += cexp(-_Complex_I * ph) * in[i];
    }
    double w = 4.0 - p->M0, s2 = 0.0;
    for (int mu = 0; mu < 4; ++mu) {
      const double pm = 2.0 * M_PI * k[mu] / L[mu];
      w -= cos(pm);
      s2 += sin(pm) * sin(pm);
    }
    s2 += w * w;
    const double d2 = 1.0 + w / sqrt(s2);
    hat[kk] = acc * (which == 0 ? d2 : 1.0 - 0.5 * d2);
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (long long i = 0; i < V; ++i) {
    long long q = i;
    int x[4];
    for (int mu = 0; mu < 4; ++mu) { x[mu] = (int)(q % L[mu]); q /= L[mu]; }
    cplx acc = 0;
    for (long long kk = 0; kk < V; ++kk) {
      long long r = kk;
      double ph = 0.0;
      for (int mu = 0; mu < 4; ++mu) {
        const int k = (int)(r % L[mu]);
        r /= L[mu];
        ph += 2.0 * M_PI * (double)k * x[mu] / L[mu];
      }
      acc += cexp(_Complex_I * ph) * hat[kk];
    }
    out[i] = acc / (double)V;
  }
  free(hat);
}

int orc_boson(const orc_params *p, const cplx *phi, double *S, cplx *G, cplx *F) {
  const long long V = volume(p);
  const cplx m = p->m_re + _Complex_I * p->m_im;
  const cplx g = p->g_re + _Complex_I * p->g_im;
  const cplx lam = 0.5 * g;
  cplx *W1 = vec_new(V), *D2phi = vec_new(V), *KW = vec_new(V), *cW = vec_new(V);
  for (long long x = 0; x < V; ++x) W1[x] = m * phi[x] + lam * phi[x] * phi[x];
  scalar_d2_apply(p, 0, phi, D2phi);
  scalar_d2_apply(p, 1, W1, KW);
  double s = 0.0;
  for (long long x = 0; x < V; ++x) {
    s += creal(2.0 * conj(phi[x]) * D2phi[x] + conj(W1[x]) * KW[x]);
    if (G) G[x] = 2.0 * (2.0 * D2phi[x] + conj(m + g * phi[x]) * KW[x]);
    cW[x] = conj(W1[x]);
  }
  if (S) *S = s;
  if (F) {
    scalar_d2_apply(p, 1, cW, F);
    for (long long x = 0; x < V; ++x) F[x] = -F[x];
  }
  free(W1); free(D2phi); free(KW); free(cW);
  return 0;
}

/* One RHMC trajectory (Sec. 7.3): pseudofermion heatbath eta = r18(MdagM) R, then
 * leapfrog molecular dynamics of length tau in nsteps steps for
 *   H = 1/2 sum |pi_x|^2 + S_B(phi) + S_PF(phi),  S_PF = Re eta^dag r14(MdagM) eta,
 * (r18 ~ x^{1/8}, r14 ~ x^{-1/4}: a0 + sum alpha_i/(x + beta_i)), with
 * dphi/dt = pi and dpi/dt = -G; accepted when u < exp(-dH).  phi is updated in
 * place when accepted.  Momenta pi, the Gaussian R and u are inputs. */
int orc_rhmc_trajectory_ex(const orc_params *p, cplx *phi, const cplx *pi0, const cplx *R,
                           int nsteps, double tau, double a18, int n18, const double *al18,
                           const double *be18, double a14, int n14, const double *al14,
                           const double *be14, double u, double tol, int maxit, double *dH,
                           int *accepted, cplx *eta_out, double *H_parts) {
  const long long V = volume(p), N = 4 * V;
  cplx *eta = vec_new(N), *ph = vec_new(V), *pi = vec_new(V), *G = vec_new(V), *Gf = vec_new(V);
  /* pseudofermion heatbath: eta = (MdagM)^{1/8} R through the x^{1/8} rational */
  int rc = orc_rational(p, phi, a18, n18, al18, be18, R, eta, tol, maxit);
  memcpy(ph, phi, (size_t)V * sizeof(cplx));
  memcpy(pi, pi0, (size_t)V * sizeof(cplx));
  const double eps = tau / nsteps;
  double Sb, Sf, H0, H1;
  /* force at the start, and H0 */
  orc_boson(p, ph, &Sb, G, NULL);
  rc |= orc_rational_force(p, ph, a14, n14, al14, be14, eta, tol, maxit, &Sf, Gf);
  H0 = 0.5 * vec_norm2(V, pi) + Sb + Sf;
  if (H_parts) {  /* kinetic, bosonic and pseudofermion parts of H at the start */
    H_parts[0] = 0.5 * vec_norm2(V, pi);
    H_parts[1] = Sb;
    H_parts[2] = Sf;
  }
  if (eta_out) memcpy(eta_out, eta, (size_t)N * sizeof(cplx));
  for (int k = 0; k < nsteps; ++k) {
    for (long long x = 0; x < V; ++x) pi[x] -= 0.5 * eps * (G[x] + Gf[x]);
    for (long long x = 0; x < V; ++x) ph[x] += eps * pi[x];
    orc_boson(p, ph, &Sb, G, NULL);
    rc |= orc_rational_force(p, ph, a14, n14, al14, be14, eta, tol, maxit, &Sf, Gf);
    for (long long x = 0; x < V; ++x) pi[x] -= 0.5 * eps * (G[x] + Gf[x]);
  }
  H1 = 0.5 * vec_norm2(V, pi) + Sb + Sf;
  *dH = H1 - H0;
  *accepted = (u < exp(-*dH)) ? 1 : 0;
  if (*accepted) memcpy(phi, ph, (size_t)V * sizeof(cplx));
  free(eta); free(ph); free(pi); free(G); free(Gf);
  return rc;
}

int orc_rhmc_trajectory(const orc_params *p, cplx *phi, const cplx *pi0, const cplx *R,
                        int nsteps, double tau, double a18, int n18, const double *al18,
                        const double *be18, double a14, int n14, const double *al14,
                        const double *be14, double u, double tol, int maxit, double *dH,
                        int *accepted) {
  return orc_rhmc_trajectory_ex(p, phi, pi0, R, nsteps, tau, a18, n18, al18, be18, a14, n14,
                                al14, be14, u, tol, maxit, dH, accepted, NULL, NULL);
}
