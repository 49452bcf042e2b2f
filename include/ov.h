/*
 * ov.h -- C ABI of the MI355X overlap-fermion library (libov.so).
 *
 * The library applies and inverts the fermion matrix of the lattice
 * Wess-Zumino model of arXiv:1005.3276 in its overlap form
 *
 *     M = D_ov + (m + g phi_x) P+ + (m* + g* phi*_x) P-
 *     D_ov = 1 + g5 sign(H_W),   H_W = g5 D_W(-M0)
 *
 * (lattice operators A = 1 - a D_W and D = (1 - A (A^dag A)^-1/2)/a of Sec. 2.2,
 * with a = 1; fermion matrix as in Sec. 7.1 with coupling g).  sign(H_W) is
 * Zolotarev's optimal rational approximation x sum_k a_k/(x^2 + b_k), evaluated
 * by a multi-shift conjugate gradient on H_W^2; M^dag M x = b is solved by CG
 * (Sec. 7.2 and 7.3 pose this problem), in FP64 or in mixed FP32/FP64 with
 * reliable updates and an FP64 true residual (Sec. 7.3 names mixed-precision
 * CG as the way to use single precision); ov_force returns the HMC force of
 * S = xi^dag (M^dag M)^-1 xi (molecular dynamics, Sec. 7.3).
 *
 * Conventions (shared with every entry point):
 *   - dims = {X, Y, Z, T}; site index i = x + X*(y + Y*(z + Z*t)).
 *   - Every field at the ABI is complex128 device memory, C-contiguous
 *     (nrhs, T, Z, Y, X, 4): spin innermost, then x, y, z, t, then rhs.
 *     phi is complex128 device memory (T, Z, Y, X).
 *   - gamma matrices in the paper's chiral basis (Sec. 2.1):
 *     g_t = [[0,1],[1,0]], g_{x,y,z} = [[0, i s_{1,2,3}], [-i s_{1,2,3}, 0]],
 *     g5 = diag(-1,-1,1,1); P+ = (1+g5)/2 acts on spins 2,3.
 *   - D_W(-M0) psi_x = (4 - M0) psi_x
 *        - 1/2 sum_mu [(1 - g_mu) ph psi_{x+mu} + (1 + g_mu) ph psi_{x-mu}],
 *     ph = bc_t for hops across the time boundary (fermions antiperiodic in
 *     time, Sec. 3.1), space periodic.
 *
 * Ownership: the caller owns every field, phi and the workspace (device
 * memory, e.g. from torch).  The library owns only the context.  All work is
 * enqueued on the context's HIP stream; entry points return after the result
 * is complete on that stream unless stated otherwise.  One context per
 * stream; contexts are not thread-safe.
 *
 * Errors: every function returns ov_status; no exception or abort crosses the
 * ABI.  On OV_ERR_NOT_CONVERGED outputs hold the best iterate and the stats
 * are filled; on any other error outputs are undefined.  ov_last_error()
 * gives a human-readable reason.
 */
#ifndef OV_H
#define OV_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OV_OK = 0,
  OV_ERR_INVALID_ARG = 1,   /* bad params, null pointer, odd or < 2 extent */
  OV_ERR_NOT_CONVERGED = 2, /* iteration cap reached; best iterate returned */
  OV_ERR_BREAKDOWN = 3,     /* non-finite or non-positive CG scalar (NaN input ...) */
  OV_ERR_SPECTRUM = 4,      /* free |H_W| range not inside [lambda_min, lambda_max] */
  OV_ERR_WORKSPACE = 5,     /* workspace missing or too small */
  OV_ERR_DEVICE = 6         /* HIP runtime error; destroy the context */
} ov_status;

typedef enum { OV_FP64 = 0, OV_MIXED = 1 } ov_precision;

/* Form of the Dirac operator D inside M = D + (m + g phi) P+ + (m* + g* phi*) P-. */
typedef enum {
  OV_DIRAC_OVERLAP_MS = 0,    /* D_ov = 1 + g5 eps(H_W), eps the Zolotarev rational by
                                 multi-shift CG on H_W^2 (default) */
  OV_DIRAC_OVERLAP_RAT = 1,   /* the same rational sign evaluated per momentum: with no
                                 gauge field D is diagonal in momentum space (Sec. 7.2) */
  OV_DIRAC_OVERLAP_EXACT = 2, /* D_ov with the exact sign H_W / |H_W|, per momentum */
  OV_DIRAC_DSLASH = 3         /* the paper's kernel Dslash = (1 - D_ov/2)^-1 D_ov with the
                                 exact sign (Sec. 2.2, fermion matrix of Sec. 7.1);
                                 needs bc_t = -1 */
} ov_dirac;

typedef enum {
  OV_OP_HW = 0,      /* H_W = g5 D_W(-M0) */
  OV_OP_DOV = 1,     /* D psi; D_ov psi = psi + g5 eps(psi) for OV_DIRAC_OVERLAP_MS */
  OV_OP_DOV_DAG = 2, /* D^dag psi; D_ov^dag psi = psi + eps(g5 psi) */
  OV_OP_M = 3,       /* D psi + c+ P+ psi + c- P- psi */
  OV_OP_M_DAG = 4,   /* D^dag psi + c+* P+ psi + c-* P- psi */
  OV_OP_MDAGM = 5,   /* M^dag M psi */
  OV_OP_M0INV = 6,   /* M0^-1 psi, M0 = D + m P+ + m* P- the free (phi = 0) fermion
                        matrix with the same D (the multi-shift form uses its rational
                        sign per momentum): the preconditioner of
                        Sec. 7.3, applied exactly in momentum space (per-axis DFTs;
                        needs every extent <= 64, X*Y <= 1024, X*Z <= 1024) */
  OV_OP_M0INV_DAG = 7 /* M0^-dag psi (same limits) */
} ov_op;

typedef struct {
  int dims[4];             /* X, Y, Z, T: each even and >= 2 */
  int bc_t;                /* -1 antiperiodic time (default), +1 periodic */
  double M0;               /* Wilson mass in D_W(-M0); 1.0 (r = 1) */
  double m_re, m_im;       /* fermion mass m */
  double g_re, g_im;       /* Yukawa coupling g */
  int n_poles;             /* Zolotarev poles, 1..32 */
  double lambda_min;       /* [lambda_min, lambda_max] bounds |eig(H_W)| (not H_W^2) */
  double lambda_max;
  double inner_tol;        /* multi-shift stop |zeta_k| ||r|| <= tol ||src|| for
                              ov_sign/ov_apply and the FP64 solver's inner sign */
  double outer_tol;        /* solve stop: true ||b - MdagM x|| / ||b|| */
  double truth_tol;        /* FP64 multi-shift tolerance of true residuals (1e-12) */
  double mixed_inner_tol;  /* FP32 multi-shift tolerance of the mixed solver */
  double reliable_delta;   /* reliable update when ||r|| drops below delta * ||r_true||
                              (default 3e-4, for the preconditioned solver; without the
                              preconditioner 0.01 with inner_relax 1e-3 converges in
                              about half the iterations); also, in preconditioned solves,
                              at a stagnating recursion (no new
                              minimum of ||r|| in 8 iterations, or under a quarter of the
                              decades its best 8-iteration window gained), and a relaxed
                              inner sign is tightened tenfold for a system whose true
                              residual comes back 10x above the recursive one */
  int max_inner;           /* multi-shift iteration cap (<= basis capacity) */
  int max_outer;           /* outer CG iteration cap */
  ov_precision precision;  /* OV_FP64 or OV_MIXED for ov_solve / ov_force */
  double inner_relax;      /* inexact-Krylov relaxation of the solver's inner sign
                              (default 3e-4):
                              tol_j = inner_relax * ||r_cycle|| / ||r_j||, clamped to
                              [inner tolerance, inner_tol_max]; 0 keeps it fixed */
  double inner_tol_max;    /* loosest inner multi-shift tolerance the relaxation uses */
  int precondition;        /* 1 (default): solve with the free-field preconditioner of
                              Sec. 7.3, CG on (M M0^-1)^dag (M M0^-1) x~ = M0^-dag b,
                              x = M0^-1 x~ (lattice limits of OV_OP_M0INV); 0: plain CG
                              on MdagM.  Convergence is always judged on the FP64 true
                              residual of the original system. */
  int dirac;               /* ov_dirac: form of D in M (default OV_DIRAC_OVERLAP_MS); the
                              momentum-space forms have the limits of OV_OP_M0INV and
                              need no inner solve (inner tolerances are unused) */
  double truth_relax;      /* intermediate true residuals (reliable updates before the
                              final check) use the multi-shift tolerance
                              max(truth_tol, min(1e-6, truth_relax * recursive residual));
                              default 0.01 */
  int inner_form;          /* MdagM in the solvers for OV_DIRAC_OVERLAP_MS:
                              1 (default): Ginsparg-Wilson form (Sec. 2.2).  The CG
                              iterations take eps^2 = 1 (D^dag D = D + D^dag) and apply
                              (1 + |1 + c|^2) v + (1 + c*) g5 eps(v) + eps(g5 (1 + Y) v)
                              with c the site's c- / c+ of Y: one multi-shift solve with
                              two independent sources instead of two dependent ones,
                              differing from MdagM only through 1 - eps^2 (the rational
                              approximation error).  The FP64 true residuals apply the
                              exact identity MdagM x = |1 + c|^2 x + (1 + c*) g5 eps(x)
                              + eps(g5 (1 + Y) x) + eps^2 x, eps^2 x taken from the
                              Krylov space of x of the same two-source multi-shift (the
                              final check at truth_tol / 10).  0: M, then M^dag, for
                              both. */
  int pc_mass;             /* mass of the preconditioner M0 of a preconditioned solve:
                              1 (default): the root mean square over the lattice of the
                              site-local coefficient c = m + g phi (in the direction of
                              m; real when m = 0), the free-field operator closest to M
                              on average; 0: the action's mass m, the phi = 0 operator
                              of Sec. 7.3.  OV_OP_M0INV(_DAG) of ov_apply always use m. */
  double shift_pc_cutoff;  /* ov_rational (heatbath / action, Sec. 7.3): shifts beta_i <=
                              this cutoff are solved one at a time, (MdagM + beta_i) X =
                              b by the preconditioned solver (context precision, reliable
                              updates, free shifted preconditioner (M0^dag M0 + beta_i)^-1)
                              and the rest by one multi-shift CG; 0 (default): every shift
                              by the multi-shift CG.  The paper's cutoff is 100.  Needs
                              precondition = 1 and inner_form = 1 or a momentum-space
                              dirac (else every shift takes the multi-shift CG). */
} ov_params;

typedef struct {
  int outer_iters;         /* CG iterations on MdagM */
  int reliable_updates;    /* FP64 true-residual recomputations */
  long long inner_iters;   /* multi-shift iterations summed over all sign applications */
  long long stencil_apps;  /* H_W applications (2 per multi-shift iteration + finals) */
  double true_rel_res;     /* last FP64 true relative residual (solves) */
  double max_shift_res;    /* max_k |zeta_k| ||r|| / ||src|| of the last multi-shift */
  double seconds;          /* wall time of the call (host clock, stream synchronised) */
  double model_bytes;      /* algorithmic HBM bytes moved (byte model) */
  int stagnations;         /* reliable updates forced by a recursion that made no progress
                              for 8 iterations (restarted with p = z) */
  int fp64_fallback;       /* 1: the mixed solve's true residual fell by less than half in
                              two reliable-update cycles in a row, and the FP64 solver (fixed
                              inner tolerance inner_tol, no relaxation) finished the system
                              from the mixed iterate (ov_force: solved again in FP64) */
} ov_stats;

typedef struct ov_ctx ov_ctx;

/* Fill p with the defaults (4^4 antiperiodic, M0 = 1, 20 poles on [1e-3, 8], ...). */
void ov_params_default(ov_params *p);

/* Create a context on HIP stream `hip_stream` (hipStream_t; NULL = default stream)
 * of the current device.  Computes the Zolotarev coefficients and checks the
 * analytic free spectrum of |H_W| against [lambda_min, lambda_max]
 * (OV_ERR_SPECTRUM).  *out receives the context (NULL on error). */
ov_status ov_ctx_create(const ov_params *p, void *hip_stream, ov_ctx **out);
ov_status ov_ctx_destroy(ov_ctx *ctx);

/* Device bytes of workspace that every call on nrhs right-hand sides needs (sign, apply,
 * solve, force, locality, boson, pack/unpack), whatever launch shape ov_set_launch or
 * the autotuner selects.  0 for a null context or nrhs < 1. */
size_t ov_workspace_bytes(const ov_ctx *ctx, int nrhs);

/* Device bytes of workspace ov_rational / ov_rational_force need for nrhs right-hand
 * sides and nshift (1..32) shifted systems (each shift keeps its own solution and search
 * direction).  0 for invalid arguments. */
size_t ov_workspace_bytes_rational(const ov_ctx *ctx, int nrhs, int nshift);

/* Hand the context a caller-owned device buffer (256-byte aligned; dev_ptr = NULL
 * returns to library-owned workspace).  While one is set, a call that needs more than
 * `bytes` returns OV_ERR_WORKSPACE and launches nothing: the library never adds a
 * hidden allocation to a caller's workspace.  Without one, calls allocate and keep their
 * own workspace (freed by ov_ctx_destroy). */
ov_status ov_set_workspace(ov_ctx *ctx, void *dev_ptr, size_t bytes);

/* Zolotarev coefficients (n_poles each) and the max error delta on the interval. */
ov_status ov_get_coeffs(const ov_ctx *ctx, double *a, double *b, double *delta);

/* Host-only Zolotarev generator: sign(x) ~ x sum_k a_k/(x^2+b_k) on
 * lmin <= |x| <= lmax with max error *delta.  No device work. */
ov_status ov_zolotarev(int n, double lmin, double lmax, double *a, double *b, double *delta);

/* out = eps(in) = H_W sum_k a_k (H_W^2 + b_k)^-1 in, FP64, for nrhs fields. */
ov_status ov_sign(ov_ctx *ctx, void *out, const void *in, int nrhs, ov_stats *st);

/* out = op(in) for nrhs fields (FP64).  phi is required for OV_OP_M, OV_OP_M_DAG and
 * OV_OP_MDAGM and ignored otherwise. */
ov_status ov_apply(ov_ctx *ctx, ov_op op, void *out, const void *in, const void *phi,
                   int nrhs, ov_stats *st);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): ov_apply with every scratch
 * buffer of the call (multi-shift basis, partial sums, counters, tables) carved from
 * one library-static device array of OV_NOALLOC_SCRATCH_BYTES per device instead of
 * a workspace.  Same arguments, kernels and results as ov_apply (bit for bit at the
 * same launch shape); the caller still owns in, out and phi.  The call allocates
 * nothing (no hipMalloc/hipFree, no host staging: that is set up by ov_ctx_create for
 * up to 16 right-hand sides) and ignores any workspace set with ov_set_workspace.
 * Limits and errors: a call whose buffers exceed the array (ov_workspace_bytes of the
 * same context and nrhs is an upper bound; e.g. at inner_tol 1e-12 the multi-shift
 * basis of one 8^4 field takes 30.7 MB, so 8^4 fits 2 right-hand sides), or nrhs > 16,
 * returns OV_ERR_WORKSPACE and launches nothing; other errors as ov_apply.  The array
 * keeps the last call's contents; every call clears what must start at zero.  All
 * contexts on one device share that device's array, so no-allocation calls that
 * overlap in time on one device (different streams or threads) race: serialise them.
 * Kernel-duration sampling (ov_kernel_sampling) is suspended during the call. */
#define OV_NOALLOC_SCRATCH_BYTES (64u << 20)
ov_status ov_apply_noalloc(ov_ctx *ctx, ov_op op, void *out, const void *in, const void *phi,
                           int nrhs, ov_stats *st);

/* Solve MdagM x = b for nrhs right-hand sides (all in one batched launch
 * sequence).  x is the initial guess on entry (zero it for a cold start) and
 * the solution on exit.  st may be NULL or an array of nrhs stats. */
ov_status ov_solve(ov_ctx *ctx, void *x, const void *b, const void *phi, int nrhs,
                   ov_stats *st);

/* Solve n systems of possibly different lattices in one batched sequence.
 * Every context must share precision, n_poles, interval and tolerances; the
 * first context's stream is used.  st: sum_i nrhs[i] stats (may be NULL). */
ov_status ov_solve_batch(int n, ov_ctx *const *ctx, void *const *x, const void *const *b,
                         const void *const *phi, const int *nrhs, ov_stats *st);

/* HMC force of S = sum_rhs Re xi^dag (MdagM)^-1 xi:
 *   grad_phi[x] = dS/dRe phi_x + i dS/dIm phi_x  (complex128 [V], device; summed over rhs)
 *   S_host[r]   = Re xi_r^dag X_r  (host array of nrhs doubles)
 * X = (MdagM)^-1 xi is solved with the context's precision; M X is recomputed
 * rather than storing shifted solutions. */
ov_status ov_force(ov_ctx *ctx, void *grad_phi, double *S_host, const void *xi,
                   const void *phi, int nrhs, ov_stats *st);

/* Rational functions of MdagM for the RHMC layers of Sec. 7.3 (pseudofermion heatbath
 * (MdagM)^{1/8} R and action (MdagM)^{-1/4}, each as a0 + sum_i alpha_i / (x + beta_i)):
 *   out_r = a0 in_r + sum_i alpha_i (MdagM + beta_i)^-1 in_r
 * for nrhs fields (complex128 layout above; phi as for ov_apply).  alpha, beta: host
 * arrays of n (1..32) doubles, beta_i >= 0.  One multi-shift CG on MdagM in FP64 serves
 * every shift (the paper solves one CG per shift); shift i stops when its recursive
 * residual |zeta_i| ||r|| <= outer_tol ||in||.  No preconditioning (M0 does not
 * commute with the shifts).  The D of the context's form is used; the multi-shift
 * form evaluates the sign at inner_tol.  st: nrhs stats (outer_iters = iterations). */
ov_status ov_rational(ov_ctx *ctx, double a0, int n, const double *alpha, const double *beta,
                      void *out, const void *in, const void *phi, int nrhs, ov_stats *st);

/* Force of S_r = Re xi_r^dag R(MdagM) xi_r with R as in ov_rational:
 *   grad_phi = sum_r dS_r/dRe phi + i dS_r/dIm phi  (complex128 [V], device)
 *   S_host[r] = S_r (host, nrhs doubles)
 * X_i = (MdagM + beta_i)^-1 xi from one multi-shift CG, Y_i = M X_i recomputed per
 * shift (sign at truth_tol for the multi-shift form), G = sum_i alpha_i G(X_i, Y_i)
 * with the density of ov_force. */
ov_status ov_rational_force(ov_ctx *ctx, double a0, int n, const double *alpha,
                            const double *beta, void *grad_phi, double *S_host, const void *xi,
                            const void *phi, int nrhs, ov_stats *st);

/* Bosonic part of the lattice action (eq. acws, a = 1) for a periodic complex scalar
 * phi (complex128 [V], device):
 *   S_B = sum_x [ 2 conj(phi) (D_2 phi) + conj(W') ((1 - D_2/2) W') ],
 *   W' = m phi + (g/2) phi^2,  D_2(p) = 1 + w(p)/|H_W(p)| the scalar part of the exact
 *   overlap operator (D^dag D = 2 D_2).  g is the Yukawa coefficient of M, i.e. the
 *   paper's 2g of eq. fmat, so that M's Yukawa term is W''(phi) = m + g phi.
 * S_host: host double.  G (device complex128 [V], may be NULL) = dS/dRe phi + i dS/dIm phi
 * = 2 [2 D_2 phi + conj(m + g phi) (1 - D_2/2) W'].  F (device complex128 [V], may be
 * NULL) = -(1 - D_2/2) conj(W'), the auxiliary field at the stationary point of eq. lata
 * (its lattice average is the Ward-identity observable of Sec. 7.4).  Lattice limits of
 * OV_OP_M0INV. */
ov_status ov_boson(ov_ctx *ctx, const void *phi, double *S_host, void *G, void *F);

/* One RHMC trajectory (Sec. 7.3): pseudofermion heatbath eta = r18(MdagM) R, leapfrog
 * molecular dynamics of length tau in nsteps steps for
 *   H = 1/2 sum_x |pi_x|^2 + S_B(phi) + Re eta^dag r14(MdagM) eta
 * (dphi/dt = pi, dpi/dt = -G), and the Metropolis decision u < exp(-dH).
 * r18 ~ x^{1/8} and r14 ~ x^{-1/4} are given as (a0, n, alpha, beta) of ov_rational.
 * phi: device complex128 [V], replaced by the end point when accepted.  pi0 (complex128
 * [V]) and R (one field) are the caller's Gaussian draws and u its uniform draw.
 * Writes dH = H_end - H_start and accepted (0/1).  Allocates its trajectory state
 * (8 V complex values) with hipMalloc for the duration of the call. */
ov_status ov_rhmc_trajectory(ov_ctx *ctx, void *phi, const void *pi0, const void *R,
                             int nsteps, double tau, double a18, int n18, const double *al18,
                             const double *be18, double a14, int n14, const double *al14,
                             const double *be14, double u, double *dH, int *accepted,
                             ov_stats *st);

/* Locality probe of Sec. 3.2: psi = D eta for a unit point source eta at the origin
 * in spin component `spin` (0..3), D the context's Dirac form (the paper probes
 * OV_DIRAC_DSLASH), and f[r] = max ||psi(x)|| (spinor norm) over the sites at
 * taxi-driver distance r = sum_mu min(x_mu, L_mu - x_mu), for r = 0 .. nr-1.
 * f is a host array of nr >= sum_mu L_mu/2 + 1 doubles (entries beyond the largest
 * distance are set to 0).  st: one stats record (may be NULL). */
ov_status ov_locality(ov_ctx *ctx, int spin, double *f, int nr, ov_stats *st);

/* Single Wilson-stencil pass out = H_W in on fields already in the library's
 * internal layout, for bandwidth measurement: prec 0 = FP64, 1 = FP32; in/out
 * hold nrhs * 4 * V complex values in spin-planar order (see DESIGN notes in
 * ov_pack).  reps launches back to back. */
ov_status ov_stencil_bench(ov_ctx *ctx, int prec, void *out, const void *in, int nrhs,
                           int reps, float *ms_per_launch);

/* Convert nrhs ABI fields (complex128 AoS) to / from the internal spin-planar
 * layout of precision prec (0 FP64, 1 FP32): plane s of rhs r holds V complex
 * values at offset (r*4 + s)*V. */
ov_status ov_pack(ov_ctx *ctx, int prec, void *dst, const void *src, int nrhs);
ov_status ov_unpack(ov_ctx *ctx, int prec, void *dst, const void *src, int nrhs);

/* Tuning knobs chosen by the autotuner: threads per block and sites per thread
 * for the stencil kernels (0 = keep). */
ov_status ov_set_launch(ov_ctx *ctx, int block, int sites_per_thread);
ov_status ov_get_launch(const ov_ctx *ctx, int *block, int *sites_per_thread);

/* Autotuner probe: time `iters` multi-shift iterations (t pass + r pass, the
 * solver's hot loop) in precision prec (0 FP64, 1 FP32) for nrhs systems of
 * this lattice with `block` threads per workgroup (64..256, multiple of 64) and
 * `sites_per_thread` (1..16), on a deterministic synthetic source.  Writes the
 * mean time per iteration in microseconds.  The context's launch setting is
 * left unchanged; apply the winner with ov_set_launch. */
ov_status ov_tune_ms(ov_ctx *ctx, int prec, int nrhs, int block, int sites_per_thread, int iters,
                     float *us_per_iter);

/* Kernel-duration sampling with HIP events recorded on the context's stream.
 * While max_per_call > 0, the first max_per_call launches of each multi-shift
 * kernel (0 = FP32 t pass  t_n = H r_n + beta t_{n-1},  1 = FP32 r pass
 * r_{n+1} = r_n - alpha H t_n, 2 = the persistent kernel running every iteration
 * of one multi-shift solve, 3 / 4 = the FP64 t / r passes) in every
 * sign/apply/solve/force call are bracketed by
 * events; the sampled per-pass launches (kernels 0 and 1) also record, in every
 * workgroup, device wall-clock stamps at its start and after its last wave.
 * ov_kernel_times returns, per kernel, the summed event duration (ms: from the
 * completion of the preceding work to the kernel's completion, so it includes
 * the dispatch gap), the number of sampled launches, their summed algorithmic
 * HBM bytes (3 spinor fields per site and pass: two read, one written; two
 * passes per iteration), and the summed kernel-only span max(end) - min(start)
 * over the workgroups (ms; what a kernel trace reports) with its launch count.
 * Any output pointer may be NULL.  reset != 0 clears the sums.  The stamp buffer
 * (2 x 8 bytes per workgroup and sampled launch) is allocated with hipMalloc
 * when sampling first needs it and freed by ov_ctx_destroy. */
ov_status ov_kernel_sampling(ov_ctx *ctx, int max_per_call);
ov_status ov_kernel_times(ov_ctx *ctx, int kernel, double *total_ms, long long *count,
                          double *bytes, double *kernel_ms, long long *kernel_count, int reset);

const char *ov_status_string(ov_status s);
const char *ov_last_error(const ov_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* OV_H */
