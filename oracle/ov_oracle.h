/*
 * ov_oracle.h -- plain FP64 CPU oracle for the overlap / Wess-Zumino hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * reference that the GPU path is judged against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or generator with the GPU library.
 *
 * Conventions (lattice spacing a = 1, Wilson parameter r = 1):
 *   site index   i = x + X*(y + Y*(z + Z*t))                       (dims = X,Y,Z,T)
 *   field        complex128 array [V][4] (spin innermost)
 *   gamma basis  the paper's chiral basis (Sec. 2.1 "Continuum"):
 *                g_t = [[0,1],[1,0]], g_i = [[0, i s_i], [-i s_i, 0]] (i = x,y,z),
 *                g5  = diag(-1,-1,+1,+1);  P+- = (1 +- g5)/2
 *   Wilson       D_W(-M0) psi_x = (4 - M0) psi_x
 *                   - 1/2 sum_mu [ (1 - g_mu) ph psi_{x+mu} + (1 + g_mu) ph psi_{x-mu} ]
 *                (Sec. 2.2, operators A and D_W, with the sign of the Wilson term
 *                 fixed by the momentum-space forms of Sec. 3.1); ph = bc_t on hops
 *                 that cross the time boundary, 1 otherwise.
 *   H_W          g5 D_W(-M0)
 *   sign         eps(psi) = H_W sum_k a_k (H_W^2 + b_k)^-1 psi   (Zolotarev pole sum)
 *   D_ov         psi + g5 eps(psi);   D_ov^dag psi = psi + eps(g5 psi)
 *   M            D_ov + c+ P+ + c- P-,  c+ = m + g phi_x,  c- = m* + g* phi*_x
 *                (fermion matrix, Sec. 7.1 form with coupling g)
 */
#ifndef OV_ORACLE_H
#define OV_ORACLE_H

#include <complex.h>

#define ORC_MAX_POLES 64

typedef struct {
  int dims[4];          /* X, Y, Z, T: each >= 2 */
  int bc_t;             /* +1 periodic, -1 antiperiodic time for the fermion */
  double M0;            /* Wilson mass in D_W(-M0); 1.0 in every workload */
  double m_re, m_im;    /* fermion mass m */
  double g_re, g_im;    /* Yukawa coupling g */
  int n_poles;          /* Zolotarev poles (shifts in H_W^2) */
  double lambda_min;    /* interval [lambda_min, lambda_max] bounding |eig(H_W)| */
  double lambda_max;
  double inner_tol;     /* multi-shift stop: |zeta_k| ||r|| <= inner_tol ||src|| */
  int max_inner;        /* multi-shift iteration cap */
  /* filled by orc_init */
  double a[ORC_MAX_POLES];
  double b[ORC_MAX_POLES];
  double delta;         /* max |x R(x^2) - 1| on the interval */
  double d0;            /* minimax normalisation */
  int dirac;            /* form of the Dirac operator D inside M (see ORC_DIRAC_*) */
} orc_params;

/* Forms of D (set before orc_init; 0 is the default):
 *   ORC_DIRAC_OVERLAP_MS     D_ov with the rational sign by multi-shift CG on H_W^2
 *   ORC_DIRAC_OVERLAP_RAT    D_ov with the same rational sign, per momentum
 *   ORC_DIRAC_OVERLAP_EXACT  D_ov with the exact sign H_W / |H_W|, per momentum
 *   ORC_DIRAC_DSLASH         Dslash = (1 - D_ov/2)^-1 D_ov with the exact sign
 *                            (the paper's kernel, Sec. 2.2 and eq. fmat of Sec. 7.1);
 *                            needs antiperiodic time with T even (Sec. 3.1)
 * The per-momentum forms follow Sec. 7.2: with no gauge field D is diagonal in
 * momentum space, so the field is Fourier transformed, multiplied by the 4x4
 * matrix D(p) and transformed back. */
enum { ORC_DIRAC_OVERLAP_MS = 0, ORC_DIRAC_OVERLAP_RAT = 1, ORC_DIRAC_OVERLAP_EXACT = 2,
       ORC_DIRAC_DSLASH = 3 };

typedef struct {
  int iters;            /* Krylov iterations */
  int converged;        /* 1 if every shift met the tolerance */
  double max_shift_res; /* max_k |zeta_k| ||r|| / ||src|| at exit */
} orc_ms_stats;

typedef struct {
  int iters;            /* outer CG iterations */
  int converged;
  long long inner_iters;/* multi-shift iterations summed over every application */
  double true_rel_res;  /* ||b - MdagM x|| / ||b|| with this oracle's operator */
} orc_cg_stats;

enum { ORC_OP_HW = 0, ORC_OP_DOV = 1, ORC_OP_DOV_DAG = 2, ORC_OP_M = 3,
       ORC_OP_M_DAG = 4, ORC_OP_MDAGM = 5 };

/* gamma matrix (mu = 0,1,2,3 for x,y,z,t; mu = 4 for gamma5), row-major 4x4. */
int orc_gamma(int mu, double complex *out16);

/* Zolotarev optimal approximation sign(x) ~ x sum_k a_k / (x^2 + b_k) for
 * lmin <= |x| <= lmax.  Returns 0 on success. */
int orc_zolotarev(int n, double lmin, double lmax, double *a, double *b,
                  double *delta, double *d0);

/* Jacobi sn, cn, dn for parameter m = 1 - m1 (exposed for pin tests). */
void orc_sncndn(double u, double m1, double *sn, double *cn, double *dn, double *K);

/* Validates params and fills a, b, delta, d0.  Returns 0 on success. */
int orc_init(orc_params *p);

void orc_dw(const orc_params *p, const double complex *in, double complex *out);
void orc_hw(const orc_params *p, const double complex *in, double complex *out);

/* Multi-shift CG on (H_W^2 + sig_k) y_k = src.  acc = sum_k coef_k y_k if acc != NULL;
 * ys (n_shift * V * 4) receives every y_k if ys != NULL. */
int orc_multishift(const orc_params *p, int n_shift, const double *sig, const double *coef,
                   double tol, int maxit, const double complex *src, double complex *acc,
                   double complex *ys, orc_ms_stats *st);

/* eps(in) with the Zolotarev coefficients in p. */
int orc_sign(const orc_params *p, const double complex *in, double complex *out,
             orc_ms_stats *st);

/* out = op(in); phi is complex128 [V] (may be NULL for HW/DOV/DOV_DAG).  DOV and
 * DOV_DAG apply the operator D of form p->dirac (and its adjoint); M and M_DAG
 * add the Yukawa term to it. */
int orc_apply(const orc_params *p, int op, const double complex *phi,
              const double complex *in, double complex *out, long long *inner_iters);

/* CG on MdagM x = b from x = 0; stops on the true relative residual. */
int orc_solve(const orc_params *p, const double complex *phi, const double complex *b,
              double complex *x, double tol, int maxit, orc_cg_stats *st);

/* S = Re xi^dag (MdagM)^-1 xi and G_x = dS/dRe phi_x + i dS/dIm phi_x. */
int orc_force(const orc_params *p, const double complex *phi, const double complex *xi,
              double tol, int maxit, double *S, double complex *G, orc_cg_stats *st);

/* RHMC rational layers (Sec. 7.3): out = a0 in + sum_i alpha_i (MdagM + beta_i)^-1 in,
 * one CG per shifted system (true relative residual <= tol each). */
int orc_rational(const orc_params *p, const double complex *phi, double a0, int n,
                 const double *alpha, const double *beta, const double complex *in,
                 double complex *out, double tol, int maxit);

/* S = Re xi^dag R(MdagM) xi and G_x = dS/dRe phi_x + i dS/dIm phi_x for
 * R(x) = a0 + sum_i alpha_i / (x + beta_i). */
int orc_rational_force(const orc_params *p, const double complex *phi, double a0, int n,
                       const double *alpha, const double *beta, const double complex *xi,
                       double tol, int maxit, double *S, double complex *G);

/* true relative residual ||b - MdagM x|| / ||b|| */
double orc_residual(const orc_params *p, const double complex *phi,
                    const double complex *b, const double complex *x);

/* out = M0^-1 in (dag = 0) or M0^-dag in (dag = 1), M0 = M at phi = 0 (the
 * free-field preconditioner of Sec. 7.3), by CG to relative residual tol. */
int orc_m0inv(const orc_params *p, int dag, const double complex *in, double complex *out,
              double tol, int maxit);

/* Locality probe (Sec. 3.2): f(r) = max ||(D eta)(x)|| over ||x||_1 = r for a unit
 * point source eta at the origin in spin component spin; f has nr >= sum L/2 + 1
 * entries. */
int orc_locality(const orc_params *p, int spin, double *f, int nr);

/* Bosonic action of eq. acws for a periodic complex scalar phi [V] (W' = m phi +
 * (g/2) phi^2, D_2 the scalar part of the exact overlap operator): S (may be NULL),
 * G = dS/dRe phi + i dS/dIm phi (may be NULL), F = -(1 - D_2/2) conj(W') (may be NULL). */
int orc_boson(const orc_params *p, const double complex *phi, double *S, double complex *G,
              double complex *F);

/* One RHMC trajectory (heatbath, leapfrog, Metropolis with the input u); phi [V] is
 * replaced by the end point when accepted.  dH = H_end - H_start. */
int orc_rhmc_trajectory(const orc_params *p, double complex *phi, const double complex *pi0,
                        const double complex *R, int nsteps, double tau, double a18, int n18,
                        const double *al18, const double *be18, double a14, int n14,
                        const double *al14, const double *be14, double u, double tol,
                        int maxit, double *dH, int *accepted);

/* The same trajectory with its start exposed: eta_out (4 V, may be NULL) receives the
 * heatbath field eta = r18(MdagM) R, H_parts (3 doubles, may be NULL) the kinetic,
 * bosonic and pseudofermion parts of H at the start of the trajectory. */
int orc_rhmc_trajectory_ex(const orc_params *p, double complex *phi, const double complex *pi0,
                           const double complex *R, int nsteps, double tau, double a18, int n18,
                           const double *al18, const double *be18, double a14, int n14,
                           const double *al14, const double *be14, double u, double tol,
                           int maxit, double *dH, int *accepted, double complex *eta_out,
                           double *H_parts);

int orc_threads(void);

#endif
