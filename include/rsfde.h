/*
 * rsfde.h -- C ABI of the MI355X (gfx950) solver for the quasi-compact
 * Crank-Nicolson discretisation of the variable-coefficient Riesz space
 * fractional diffusion equation, solved at every time step by GMRES(m) with the
 * sine-transform (tau) preconditioner.
 *
 * Problem (Section 1, eq. RSFDE): e(x,t) u_t = sum_i kappa_i d^{alpha_i} u / d|x_i|^{alpha_i} + f
 * on prod_i (lo_i, hi_i) x (0, T], u = 0 on the boundary, u(x,0) = psi(x),
 * 1 < alpha_i < 2, kappa_i >= 0 with sum_i kappa_i > 0, e bounded with positive minimum.
 *
 * Scheme (Section 2, eq. tls): with N_i interior points per axis,
 * h_i = (hi_i - lo_i)/(N_i + 1) and dt = T/M, every step solves
 *     A u^{(m+1)} = b^{(m)},  A = B_alpha E^{(m+1/2)} + S_alpha,
 *     b^{(m)} = (B_alpha E^{(m+1/2)} - S_alpha) u^{(m)} + dt F^{(m+1/2)},
 * where B_alpha = B_{alpha_d} x ... x B_{alpha_1} (eq. Ha, tridiagonal factors),
 * E = diag(e(grid, t_{m+1/2})), S_alpha the d-level symmetric Toeplitz matrix of
 * eq. Salpha with eta_i = kappa_i dt / (2 h_i^{alpha_i}) and the FCD weights of eq. eq0,
 * and F the compact operator applied to f (eq. eq2.2, Appendix A).
 *
 * Solver (Section 3): left-preconditioned GMRES(m) on the one-sided system
 * (eq. one-sided), which is GMRES on A u = b with preconditioner
 * B_alpha P_alpha = ebar B_alpha + tau(S_alpha) (eqs. Pa, tauSalpha, bard), applied
 * through the d-dimensional sine transform (eq. diag).  The stopping rule is
 * ||z_k||_2 <= rtol ||z_0||_2 on the preconditioned residual z (Section 4).
 *
 * Memory: every vector argument is DEVICE memory owned by the caller.  Grid
 * vectors are stored lexicographically with x_1 fastest (Section 2): interior
 * vectors hold prod_i N_i doubles, closure-grid vectors prod_i (N_i + 2) doubles.
 * The library never allocates device memory: all its device state lives in the
 * caller's workspace (sized by rsfde_workspace_size).  It allocates a small host
 * structure and a little pinned host memory for status read-back, released by
 * rsfde_destroy.
 *
 * Streams: all device work of a handle is enqueued on the hipStream_t given to
 * rsfde_setup (a void* here; NULL is the default stream).  A handle is not
 * re-entrant and must not be used from two threads at once.
 *
 * Errors: every function returns an int status.  0 is success, negative values
 * are errors, positive values are warnings.  Argument checks run on the host
 * before any HIP call, so they behave the same on a machine without a GPU.
 * No C++ exception crosses this boundary.
 */
#ifndef RSFDE_H
#define RSFDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define RSFDE_OK               0
#define RSFDE_W_NOT_CONVERGED  1   /* GMRES hit max_cycles (or max_outer); u holds the last iterate */
#define RSFDE_E_INVALID_ARG   -1   /* a parameter or pointer failed validation */
#define RSFDE_E_WORKSPACE     -2   /* workspace NULL, misaligned (256 B) or too small */
#define RSFDE_E_HIP           -3   /* a HIP runtime call failed; rsfde_strerror gives details */
#define RSFDE_E_NONFINITE     -4   /* a NaN/Inf appeared in a residual norm */
#define RSFDE_E_UNSUPPORTED   -5   /* N_i + 1 outside the transform sizes built into the library */
#define RSFDE_E_STATE         -6   /* call order violated, e.g. a step before ebar is known */

/* ---- precision forms ---------------------------------------------------- */
#define RSFDE_FP64   0  /* every operation in FP64 */
#define RSFDE_MIXED  1  /* FP32 operator/preconditioner inside GMRES, FP64 Arnoldi,
                           Givens and norms, FP64 true-residual iterative refinement */

/* ---- solver forms (Section 3) ---------------------------------------------
 * With Atilde = E + B_alpha^{-1} S_alpha and btilde = B_alpha^{-1} b (eq. equi) and
 * the tau preconditioner P_alpha (eq. Pa):
 *   RSFDE_OPGM  GMRES on P^{-1} Atilde u = P^{-1} btilde (eq. one-sided), run as
 *               (B P)^{-1} A u = (B P)^{-1} b, which is the same system;
 *   RSFDE_TPGM  GMRES on P^{-1/2} Atilde P^{-1/2} utilde = P^{-1/2} btilde (eq. Pls),
 *               started from utilde_0 = P^{1/2} u^{(m)} (or 0) and stopped on its own
 *               residual; u^{(m+1)} = P^{-1/2} utilde.  FP64 only; instances of this
 *               form are stepped one at a time (no batched launches). */
#define RSFDE_OPGM  0
#define RSFDE_TPGM  1
/*   RSFDE_SPGM  the paper's comparison solver (Section 4): GMRES on A u = b (eq. tls)
 *               left-preconditioned by ebar c(B_alpha) + c(S_alpha), the Strang
 *               circulants of every factor (c(B)^{1/2} P_c c(B)^{1/2} with P_c of the
 *               Strang preconditioner); FP64 only, stepped one instance at a time. */
#define RSFDE_SPGM  2

typedef struct rsfde_ctx* rsfde_handle;

/* One problem instance.  Fields beyond the paper's statement are solver settings. */
typedef struct {
  int     d;            /* spatial dimension, 1..3 */
  int64_t n[3];         /* N_i interior points on axis i (N_i + 1 must be 2^p or 3*2^p, 4 <= 2(N_i+1) <= 4096) */
  double  lo[3], hi[3]; /* the box prod_i (lo_i, hi_i), lo_i < hi_i */
  double  alpha[3];     /* fractional orders, 1 < alpha_i < 2 */
  double  kappa[3];     /* diffusion coefficients kappa_i >= 0, sum > 0 */
  double  dt;           /* time step (T/M), > 0 */
  double  e_min, e_max; /* e_check and e_hat of eq. dhat; both 0 means "not known yet":
                           then rsfde_set_ebar must be called, or rsfde_solve pre-scans e */
  int     restart;      /* GMRES restart length m, 1..64 */
  double  rtol;         /* relative tolerance on the preconditioned residual, > 0 */
  int     max_cycles;   /* GMRES cycles allowed per step, >= 1 (RSFDE_FP64; the mixed form
                           runs one FP32 cycle per refinement sweep and is bounded by
                           max_outer alone) */
  int     precision;    /* RSFDE_FP64 or RSFDE_MIXED */
  int     x0_mode;      /* 0: GMRES starts from u^{(m)}; 1: from zero */
  double  inner_rtol;   /* RSFDE_MIXED: tolerance of each FP32 inner solve relative to its
                           starting residual (0 -> sqrt(outer bound), clamped to
                           [1e-6, 1e-3], so that two sweeps reach the outer bound) */
  int     max_outer;    /* RSFDE_MIXED: refinement sweeps allowed per step (0 -> 30) */
  int     method;       /* RSFDE_OPGM (0), RSFDE_TPGM or RSFDE_SPGM; the last two with
                           RSFDE_MIXED are RSFDE_E_UNSUPPORTED */
  double  outer_rtol;   /* RSFDE_MIXED: refinement stops once the FP64 preconditioned true
                           residual satisfies ||z|| <= outer_rtol ||z_0|| (0 -> rtol / 10,
                           so that the refined solution stays within rounding of the FP64
                           solve's); must not exceed rtol.  Ignored by RSFDE_FP64 */
} rsfde_params;

/* Per-instance result of one step (summed over the steps of rsfde_solve). */
typedef struct {
  int    iters;         /* Arnoldi iterations (all cycles; all inner solves in the mixed form) */
  int    cycles;        /* GMRES cycles */
  int    outer_sweeps;  /* refinement sweeps (mixed form), else 0 */
  int    converged;     /* 1 when the stopping rule was met */
  double beta0;         /* ||z_0||_2 of the (last) step */
  double rel_pres;      /* final preconditioned residual / beta0 of the (last) step: the
                           GMRES estimate |g_{k+1}| (RSFDE_FP64) or the recomputed FP64
                           residual of the last refinement sweep (RSFDE_MIXED) */
  double rel_true_res;  /* ||M (b - A u^{(m+1)})||_2 / beta0 of the (last) step, recomputed
                           in FP64 from the returned u with the stopping rule's
                           preconditioner M; computed by the mixed form's last sweep, and
                           in the other forms only while rsfde_set_true_residual is on
                           (else -1) */
} rsfde_stats;

/* Analytic field families the library can evaluate on the device (synthetic
 * workloads).  Kinds and the meaning of c[] follow the workload descriptions:
 *   e: CONST c0 | SUMSQ_EXP (sum x_i^2 + exp(-t))/c0 | POLY_T c0 + c1 (1 + c2 t) prod x_i^c3
 *      | SINPROD_COS c0 + c1 prod sin(pi x_i) cos t | SINE_FIELD c0 + c1 (1 + g/sum|a|)/2
 *   f: ZERO | MANUFACTURED (u = c0 exp(-t) prod x_i^c1 (1 - x_i)^c1 on the unit box,
 *      f = e u_t - sum_i kappa_i d^{alpha_i} u, e the instance's e field) | SINE_MODES g
 *   psi: ZERO | MANUFACTURED u(x, 0)
 * with g = sum_K a_K prod_i sin(k_i pi x_i), amplitudes a (host array of
 * modes^d values, k_1 fastest, mode numbers from 1). */
#define RSFDE_FIELD_ZERO          0
#define RSFDE_FIELD_CONST         1
#define RSFDE_FIELD_SUMSQ_EXP     2
#define RSFDE_FIELD_POLY_T        3
#define RSFDE_FIELD_SINPROD_COS   4
#define RSFDE_FIELD_SINE_FIELD    5
#define RSFDE_FIELD_MANUFACTURED  6
#define RSFDE_FIELD_SINE_MODES    7

typedef struct {
  int           kind;
  double        c[4];
  int           modes;          /* K <= 8 for the mode families, else 0 */
  const double* amp;            /* host pointer to K^d amplitudes (copied), or NULL */
  int           time_dependent; /* 0 lets the library evaluate the field once */
} rsfde_field;

#define RSFDE_WHICH_E    0  /* e on the interior grid */
#define RSFDE_WHICH_F    1  /* f on the closure grid */
#define RSFDE_WHICH_PSI  2  /* psi on the interior grid */

/* Sample callback for rsfde_solve: fill e(interior, t) and f(closure, t) for
 * one instance at t = t_{m+1/2}, enqueueing work on `stream`; return 0 on success. */
typedef int (*rsfde_sample_fn)(void* ctx, int instance, double t,
                               double* e_interior, double* f_closure, void* stream);

/* ---- entry points ------------------------------------------------------- */

/* Bytes of device workspace needed for `count` instances p[0..count-1]
 * (count >= 1; count > 1 is the batched form, all instances stepping together).
 * Validates p (RSFDE_E_INVALID_ARG / RSFDE_E_UNSUPPORTED).  Host only. */
int rsfde_workspace_size(const rsfde_params* p, int count, size_t* bytes);

/* Validate, partition the caller's device workspace (256-byte aligned, at least
 * rsfde_workspace_size bytes; owned by the caller and kept alive until
 * rsfde_destroy) and build the per-axis coefficient tables on the device: FCD
 * weights s_k (eq. eq0 recurrence), the circulant spectrum of the Toeplitz
 * factors, the tau eigenvalues q (eq. q) and the B eigenvalues (Lemma Heig).
 * The preconditioner does not depend on the step (Section 3 remark), so this runs once. */
int rsfde_setup(const rsfde_params* p, int count, void* workspace, size_t bytes,
                void* stream, rsfde_handle* out);

/* Set e_check / e_hat (eq. dhat) of one instance; ebar = (e_min + e_max)/2 (eq. bard). */
int rsfde_set_ebar(rsfde_handle h, int instance, double e_min, double e_max);

/* One Crank-Nicolson step for every instance: given e at t_{m+1/2} on the interior
 * and f at t_{m+1/2} on the closure grid (device pointers per instance, t_m = m dt is
 * informational), overwrite u[i] = u^{(m)} with u^{(m+1)} (u[i] 16-byte aligned).  stats (host array of
 * `count`, may be NULL) receives per-instance counters.  Synchronises the stream
 * before returning.  Returns the worst status over the instances. */
int rsfde_step(rsfde_handle h, double t_m, const double* const* e_half,
               const double* const* f_half, double* const* u, rsfde_stats* stats);

/* M steps from t = 0.  sample == NULL uses the fields registered with
 * rsfde_set_fields.  When an instance's e_min = e_max = 0 the e field is first
 * sampled at all M midpoints to get ebar.  u[i] holds psi on entry, u^{(M)} on exit;
 * stats accumulate iterations over the steps. */
int rsfde_solve(rsfde_handle h, int M, rsfde_sample_fn sample, void* ctx,
                double* const* u, rsfde_stats* stats);

/* Steps m0 .. m0+M-1 (t_m = m dt, m0 >= 0) of the same time loop as rsfde_solve,
 * which is the case m0 = 0: u[i] holds u^{(m0)} on entry and u^{(m0+M)} on exit.
 * The loop runs in the library, so a long run split over several calls
 * continues the same time levels without a host round trip per step.  An
 * instance whose ebar is not known yet is pre-scanned over this call's M
 * midpoints only; a run split over several calls should set ebar for all of its
 * steps first (rsfde_prescan_ebar or rsfde_set_ebar).  Errors as rsfde_solve,
 * and RSFDE_E_INVALID_ARG for m0 < 0. */
int rsfde_solve_range(rsfde_handle h, int m0, int M, rsfde_sample_fn sample, void* ctx,
                      double* const* u, rsfde_stats* stats);

/* Release the host state of a handle (not the caller's workspace). */
int rsfde_destroy(rsfde_handle h);

/* Human-readable text for a status code (includes the last HIP error for RSFDE_E_HIP). */
const char* rsfde_strerror(int status);

/* ---- built-in synthetic fields ------------------------------------------ */

/* Register the analytic e, f and psi families of one instance (copies the specs). */
int rsfde_set_fields(rsfde_handle h, int instance, const rsfde_field* e,
                     const rsfde_field* f, const rsfde_field* psi);

/* Evaluate a registered field of one instance at time t into `out` (device):
 * which = RSFDE_WHICH_E (interior), RSFDE_WHICH_F (closure grid), RSFDE_WHICH_PSI. */
int rsfde_eval_field(rsfde_handle h, int instance, int which, double t, double* out);

/* The same for every instance of the handle in one launch: out[i] (device) receives
 * instance i's field, in the layout rsfde_eval_field uses.  Every instance needs
 * its fields registered.  Errors: RSFDE_E_INVALID_ARG (null handle/array/entry,
 * bad `which`), RSFDE_E_STATE (fields not registered), RSFDE_E_HIP. */
int rsfde_eval_field_batch(rsfde_handle h, int which, double t, double* const* out);

/* ---- operator entry points (single instance; device pointers; on the handle's stream) */

/* out = A v = B_alpha (e .* v) + S_alpha v (eq. tls). */
int rsfde_apply_A(rsfde_handle h, int instance, const double* e, const double* v, double* out);

/* out = (B_alpha P_alpha)^{-1} r = S diag(1/mu) S r, the sine-transform solve with the
 * tau preconditioner (eqs. Pa, tauSalpha, diag); needs ebar to be set. */
int rsfde_apply_prec(rsfde_handle h, int instance, const double* r, double* out);

/* The same (B_alpha P_alpha)^{-1} r as rsfde_apply_prec, bit for bit, for callers that
 * cannot allocate device memory or bring a workspace for temporaries (code under
 * HIP graph capture, tight serving loops).  The pass temporaries (none for d = 1,
 * two FP64 vectors for d = 2, four for d = 3) live in a static device array of
 * RSFDE_NOALLOC_SCRATCH_BYTES per GPU, held by the library until the process
 * ends; the call itself allocates nothing and creates no events (kernel timing is
 * suspended for it).  Every call on one GPU shares that array: calls that overlap
 * on one GPU (two streams, two threads) race and must be ordered by the caller.
 * Nothing in the array needs to start at zero (every pass writes its whole output).
 * Errors: RSFDE_E_INVALID_ARG, RSFDE_E_STATE (ebar not set), RSFDE_E_WORKSPACE (the
 * temporaries, each rounded up to 256 bytes, exceed RSFDE_NOALLOC_SCRATCH_BYTES:
 * more than 2^22 unknowns in 2-D or 2^21 in 3-D), RSFDE_E_HIP. */
#define RSFDE_NOALLOC_SCRATCH_BYTES (64u << 20)
int rsfde_apply_prec_noalloc(rsfde_handle h, int instance, const double* r, double* out);

/* out = S diag(g) S r for one of the sine-basis diagonals g of Section 3, with
 * Lambda_K the eigenvalues of B_alpha and mu_K those of B_alpha P_alpha:
 *   RSFDE_PREC_BP_INV     (B_alpha P_alpha)^{-1}       g = 1/mu      (as rsfde_apply_prec)
 *   RSFDE_PREC_PHALF_BINV P_alpha^{-1/2} B_alpha^{-1}  g = 1/sqrt(Lambda mu)   (eq. Pls)
 *   RSFDE_PREC_PHALF      P_alpha^{-1/2}               g = sqrt(Lambda / mu)   (eq. Pls)
 * and, for an instance of the RSFDE_SPGM form only, the Strang circulant solve
 *   RSFDE_PREC_STRANG     (ebar c(B) + c(S))^{-1} = (1/prod N_l) H diag(1/m) H, with H
 *                         the separable Hartley transform and m the eigenvalues of
 *                         ebar c(B) + c(S) (Section 4)
 * r and out: FP64 device vectors of the instance's size, not overlapping; needs ebar.
 * Errors: RSFDE_E_INVALID_ARG (bad form, null pointer), RSFDE_E_STATE (ebar not set,
 * or RSFDE_PREC_STRANG on another form), RSFDE_E_HIP. */
#define RSFDE_PREC_BP_INV      0
#define RSFDE_PREC_PHALF_BINV  1
#define RSFDE_PREC_PHALF       2
#define RSFDE_PREC_STRANG      3
int rsfde_apply_prec_form(rsfde_handle h, int instance, int form, const double* r, double* out);

/* out = F = (H_{alpha_d} ... H_{alpha_1}) f restricted to the interior, from f on the
 * closure grid (eq. eq2.2, Appendix A). */
int rsfde_compute_F(rsfde_handle h, int instance, const double* f_closure, double* out);

/* out = b = B_alpha (e .* u) - S_alpha u + dt F (eq. tls). */
int rsfde_rhs(rsfde_handle h, int instance, const double* e, const double* F,
              const double* u, double* out);

/* Copy the setup tables of one axis to host arrays of length N_axis (any may be
 * NULL): FCD weights s_0..s_{N-1}, tau eigenvalues q_0..q_{N-1} (eq. q, obtained on
 * the device from the circulant spectrum) and B eigenvalues lambda_1..lambda_N. */
int rsfde_get_tables(rsfde_handle h, int instance, int axis, double* s, double* q,
                     double* lambda);

/* Evaluate the registered e field of one instance at the M midpoints
 * t_{m+1/2} = (m + 1/2) dt and set ebar from its extremes (eq. dhat, eq. bard).
 * Time-independent fields are sampled once. */
int rsfde_prescan_ebar(rsfde_handle h, int instance, int M);

/* True-residual check (enable = 1; default 0): every step of the FP64 forms ends
 * with one more residual evaluation in FP64, z = M (b - A u^{(m+1)}) with the
 * stopping rule's preconditioner M (Section 4), and reports ||z|| / ||z_0|| as
 * rsfde_stats.rel_true_res.  It costs about one Arnoldi iteration per step and
 * changes no result.  The mixed form always reports it.  Errors: RSFDE_E_INVALID_ARG. */
int rsfde_set_true_residual(rsfde_handle h, int enable);

/* Graph replay (enable = 1) or direct launches (0, the default) for the Arnoldi
 * steps.  With replay on, each step's launch sequence (operator chain and the
 * three CGS2 sweeps) is captured once per (step index, pending resolve) on a
 * private stream and replayed as one graph on the handle's stream; results are
 * bit-identical to direct launches.  Steps are launched directly while a kernel
 * class is being timed (rsfde_set_timing), and in batched cycles that run on a
 * partial instance set.  Captured graphs follow the e buffer and the batched
 * plan; they are released by rsfde_set_graph(h, 0) and rsfde_destroy.
 * Errors: RSFDE_E_INVALID_ARG, RSFDE_E_HIP. */
int rsfde_set_graph(rsfde_handle h, int enable);

/* Workgroup shape the tile autotuner picked at setup for the pencil passes of one
 * instance along `axis`: operator passes (transform = 0) or transform passes
 * (transform = 1), in the FP64 chains (precision = RSFDE_FP64) or the FP32 inner
 * chains of the mixed form (RSFDE_MIXED).  *length = L = 2(N_axis + 1), the
 * transform length; *per_workgroup = complex transforms per workgroup (two real
 * pencils each).  The pass kernel is rsfde_pass_kernel<R, code, per_workgroup,
 * axis > 0> (rsfde_dst_kernel for transform passes) with the plan code of
 * rsfde_get_pass_plan.  Host only.  Errors: RSFDE_E_INVALID_ARG. */
int rsfde_get_pass_shape(rsfde_handle h, int instance, int axis, int precision, int transform,
                         int* length, int* per_workgroup);

/* Radix plan the autotuner picked for the same pencil pass as rsfde_get_pass_shape:
 * *code is the pass kernel's length template argument (L for the length's default
 * plan, L + 65536 for its alternative plan) and radices[0 .. *nstage) the radices
 * of its Stockham stages (radices: room for 8).  The autotuner times both plans
 * of a length where it has two (2(N+1) >= 256) with three tile widths each, and
 * keeps its choices per GPU architecture for the process (and, with
 * RSFDE_TUNE_CACHE=<file>, across processes).  Host only.
 * Errors: RSFDE_E_INVALID_ARG. */
int rsfde_get_pass_plan(rsfde_handle h, int instance, int axis, int precision, int transform,
                        int* code, int* radices, int* nstage);

/* Kernel classes for HIP-event timing (bit i of the mask enables class i). */
#define RSFDE_K_MV_FIRST    0  /* first-axis operator pass */
#define RSFDE_K_MV_MID      1  /* middle-axis operator pass (d = 3) */
#define RSFDE_K_MV_LAST     2  /* last-axis operator pass (+ fused sine transform) */
#define RSFDE_K_DST         3  /* sine-transform pass */
#define RSFDE_K_DSD         4  /* transform, 1/mu scaling, transform pass */
#define RSFDE_K_DOTS        5  /* Arnoldi sweep A: dot products of the basis with w */
#define RSFDE_K_ORTH_DOTS   6  /* Arnoldi sweep B: second projection of the newest basis
                                  vector, first projection of w, their dot products */
#define RSFDE_K_ORTH_NORM   7  /* (no longer launched: CGS2 runs in two sweeps) */
#define RSFDE_K_UPDATE      8  /* solution update */
#define RSFDE_K_NCLASS      9

/* Stamp HIP events at the start and end of one launch in every `every` (>= 1)
 * of each kernel class in `mask` (on the handle's stream) and reset the
 * counters; mask 0 switches timing off.  rsfde_get_timing returns, for one
 * class, the launches timed since then, their summed milliseconds and their
 * summed algorithmic HBM bytes (arrays read plus arrays written, each counted
 * once). */
int rsfde_set_timing(rsfde_handle h, unsigned mask, int every);
int rsfde_get_timing(rsfde_handle h, int kclass, long long* launches, double* ms, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* RSFDE_H */
