/*
 * rt.h -- C ABI of the MI355X implicit radiation / ionization / gas-energy
 * Newton step.
 *
 * The library advances the reaction-diffusion system that remains after the
 * hydrodynamic sub-step of an operator-split cosmological radiation-
 * hydrodynamics solver (D. R. Reynolds, J. C. Hayes, P. Paschos,
 * M. L. Norman: Sec. 3.1, Eqs. 19-21): the gas-energy correction e_c, the
 * species fractions x_i and the flux-limited-diffusion radiation energy E,
 * with one theta-scheme time step (Sec. 3.2, Eqs. 22-24) solved by a
 * globalised inexact Newton method (Sec. 3.2) whose linear systems are
 * reduced by a Schur complement to a scalar 7-point diffusion system
 * (Sec. 3.2.1, Eqs. 33-35) and solved by a multigrid-preconditioned Krylov
 * method.  The residual evaluates the flux limiter of Eq. 12 at the state it
 * acts on (Eq. 29 with D_E(U)); the Newton matrix is its exact derivative,
 * so the Schur matrix is not symmetric and the Krylov method is flexible
 * GMRES, preconditioned by a V-cycle of a symmetric M-matrix built beside it.
 *
 * Conventions common to every entry point
 *   Grid     nx*ny*nz cells, periodic in every direction, cell (i,j,k) at
 *            flat index (i*ny + j)*nz + k (z fastest).  Each n is even and
 *            divisible by 2^(mg_levels-1) with a coarsest size >= 4.
 *   Fields   device pointers to FP64 arrays.  A state U is structure-of-
 *            arrays [nv][nx][ny][nz] with nv = nspecies + 2 and row order
 *            (e_c, x_1..x_Ns, E) (Sec. 3.2, the unknown vector of Eq. 29):
 *            e_c gas-energy correction (erg/g), x_i = n_i/n_H for HI and
 *            n_i/n_He for HeI, HeII, E comoving radiation energy (erg/cm^3).
 *            n_H is comoving (cm^-3), e_h the specific gas energy left by the
 *            hydrodynamic sub-step (erg/g), dx a comoving length (cm).
 *   Memory   the caller allocates every device array, including the
 *            workspace sized by rt_workspace_bytes; the library never
 *            allocates or frees device memory.  It owns only the small host
 *            object behind rt_grid and a few pinned host bytes for scalar
 *            read-back.  Pointers passed to rt_set_medium must
 *            stay valid while the grid uses them.
 *   Streams  every call enqueues on the hipStream_t given to rt_create_grid.
 *            Calls that return host scalars synchronise that stream; others
 *            do not.
 *   Errors   every call returns an rt_status; no exception crosses the ABI.
 *            rt_last_error(grid) describes the last failure.  A grid is not
 *            thread-safe; distinct grids are independent.
 */
#ifndef RT_H
#define RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rt_status {
  RT_OK = 0,
  RT_EINVAL = -1,        /* invalid argument, size or call order */
  RT_EDEVICE = -2,       /* a HIP runtime call failed */
  RT_ENOCONV = -3,       /* Newton hit newton_maxit above tolerance; U holds the last iterate */
  RT_ELINESEARCH = -4,   /* line search fell below lambda_min; U holds the last iterate */
  RT_ENONFINITE = -5     /* a residual norm was NaN or Inf */
} rt_status;

/* Problem and solver parameters (plain old data; copied at rt_create_grid). */
typedef struct rt_params {
  int32_t nx, ny, nz;
  int32_t nspecies;         /* 1: HI; 3: HI, HeI, HeII (Sec. 2, Eq. 4); 0: LTE */
  double  dx;               /* comoving cell width (cm) */
  double  theta;            /* theta-scheme weight in (0, 1] (Sec. 3.2) */
  double  u_e, u_E;         /* unit scales of e_c and E (Sec. 3.2.2, Eq. 36) */
  int32_t grey;             /* m of Eq. 5: 0 monochromatic, 1 grey (Sec. 2.2) */
  int32_t isothermal;       /* 1: rates use T_iso and G, Lambda are dropped */
  double  T_iso;            /* K */
  double  y_he;             /* n_He / n_H */
  double  K_gamma[3];       /* photoionization constants per species (Eq. 45) */
  double  K_kappa[3];       /* opacity constants (cm^2) */
  double  K_heat[3];        /* photo-heating constants (cm^2) */
  double  hnu_mean;         /* energy per source photon (erg) */
  int32_t limiter_mode;     /* 0: flux limiter of Eq. 12; 1: constant D0 */
  double  D0;               /* cm^2/s, limiter_mode 1 only */
  double  newton_tol;       /* RMS-norm tolerance (Eq. 30) */
  int32_t newton_maxit;     /* <= RT_MAX_NEWTON */
  double  pcg_rtol;         /* ||r||_2 <= pcg_rtol ||b||_2 */
  int32_t pcg_maxit;
  int32_t mg_levels;        /* >= 1 */
  int32_t mg_pre, mg_post;  /* red-black Gauss-Seidel sweeps before/after */
  int32_t mg_coarse_sweeps; /* coarsest level: this many (red,black) then (black,red) */
  int32_t mg_fp32;          /* 1: V-cycle in FP32 (Newton, CG, local solves stay FP64) */
  int32_t max_sources;      /* capacity of the point-source list */
  double  pcg_forcing;      /* inexact-Newton forcing (Sec. 3.2.1); > 0: the CG solve */
                            /* of Newton iteration k also stops once ||r||_2 =       */
                            /* ||J S_k + f(U_k)||_2 <= pcg_forcing ||f(U_k)||_2 (the  */
                            /* paper's delta_k = 1e-6 ||f||); 0: relative test alone */
  int32_t box_size;         /* > 0: add to every V-cycle a subdomain correction: a */
                            /* box of box_size^3 cells centred on each source,    */
                            /* solved by box_inner PCG iterations with its own    */
                            /* box_levels-level V-cycle (0: V-cycle alone)        */
  int32_t box_levels;
  int32_t box_inner;
  int32_t box_coarse_sweeps; /* coarsest box level: this many (red,black) then     */
                             /* (black,red) (0: mg_coarse_sweeps)                 */
  int32_t lte;              /* 1: LTE coupling (Sec. 2.1, Eq. 9), nspecies = 0,  */
                            /* U = (e_c, E); 0: the non-LTE rates              */
  double  kappa_lte;        /* LTE absorption coefficient (proper, 1/cm)        */
  double  kappaP_lte;       /* LTE Planck-mean coefficient (proper, 1/cm)       */
  double  mu_lte;           /* LTE mean particle mass (units of m_H)            */
  int32_t boundary;         /* 0: periodic; 1: reflecting walls on all six      */
                            /* domain faces (zero diffusive flux through them); */
                            /* 2: the x-left face holds E at E_dirichlet (a     */
                            /* ghost cell one width outside), the other faces   */
                            /* reflect                                          */
  double  E_dirichlet;      /* boundary 2: comoving E of the x-left ghost cell  */
  int32_t krylov_restart;   /* Schur solve: 1..30 flexible GMRES restarted every */
                            /* this many iterations (the Newton matrix is not    */
                            /* symmetric); 0: flexible CG on the preconditioner's */
                            /* symmetric operator, which is the Schur matrix only */
                            /* for a constant diffusion coefficient (limiter_mode */
                            /* 1).  The workspace holds 2 krylov_restart + 1     */
                            /* extra FP64 fields                                  */
  int32_t limiter_lag;      /* 0: the limiter of Eq. 12 evaluated at the state the */
                            /* residual acts on (Eq. 29 as printed); 1: the face   */
                            /* coefficients held at their time-level-n values for  */
                            /* the whole step (the diffusion term is then linear   */
                            /* in E and the Schur matrix symmetric); needs         */
                            /* rt_time_level before rt_eval_residual and           */
                            /* rt_schur_form                                       */
  int32_t box_s_sweeps;     /* with box_size > 0: after the correction, this many  */
                            /* red-black Gauss-Seidel (red, black) pairs on the    */
                            /* Schur matrix S itself (not the symmetric operator)  */
                            /* over the cells of each box, box by box; 0..256, and */
                            /* > 0 only with krylov_restart > 0                    */
} rt_params;

/* Scale factor a and adot/a at t^n (old) and t^{n+1} (new). */
typedef struct rt_cosmo { double a_old, H_old, a_new, H_new; } rt_cosmo;

#define RT_MAX_NEWTON 32

typedef struct rt_newton_stats {
  int32_t status;           /* rt_status of the step */
  int32_t newton_its;
  int32_t cg_its_total;
  int32_t vcycles;
  int32_t ls_trials;        /* residual evaluations inside line searches */
  int32_t used_alt_guess;   /* 1 if the alternative initial guess was taken */
  double  fnorm_guess;      /* ||f(U_0)|| of the caller's guess */
  double  fnorm_alt;        /* ||f|| of the alternative guess (or -1) */
  double  fnorm_final;
  int32_t cg_its[RT_MAX_NEWTON];
  double  lambda[RT_MAX_NEWTON];
  double  fnorm[RT_MAX_NEWTON + 1];
} rt_newton_stats;

typedef struct rt_grid rt_grid;

/* Bytes of device workspace a grid with these parameters needs. */
int rt_workspace_bytes(const rt_params* p, uint64_t* bytes);

/* Create a grid over a caller-allocated device workspace (>= the size above,
 * 256-byte aligned).  hip_stream is a hipStream_t (NULL: default stream).
 * RT_EINVAL on inconsistent parameters or a short workspace. */
int rt_create_grid(const rt_params* p, void* d_ws, uint64_t ws_bytes,
                   void* hip_stream, rt_grid** out);
int rt_destroy_grid(rt_grid* g);
const char* rt_last_error(const rt_grid* g);

/* Fixed-per-step medium: d_nH [N] comoving n_H, d_eh [N] specific energy
 * e_h of the hydrodynamic state (Sec. 3.1; e^{n+1} = e_h + e_c). */
int rt_set_medium(rt_grid* g, const double* d_nH, const double* d_eh);

/* Point sources (host arrays): flat cell index and photon rate (1/s).  Their
 * emissivity 4 pi eta = Q <h nu> / dx^3 (Sec. 2, Eq. 5) enters the
 * time-level vector.  RT_EINVAL if n > max_sources or a cell is out of range. */
int rt_set_sources(rt_grid* g, int32_t n, const int64_t* h_cells, const double* h_Q);

/* Time-level setup (Sec. 3.2, Eqs. 22-24): writes d_gn [nv][N] =
 * U^n + dt (theta-1) [L_e; L_n; D_E + L_E](U^n) + dt [0; 0; 4 pi eta], the
 * explicit part (theta < 1) with the flux limiter of Eq. 12 at U^n.  With
 * limiter_lag it also stores those face coefficients for the step. */
int rt_time_level(rt_grid* g, const double* d_Un, double dt, const rt_cosmo* c,
                  double* d_gn);

/* Nonlinear residual (Sec. 3.2, Eq. 29) in scaled variables f_v / u_v,
 * written to d_f [nv][N], and its RMS norm (Eq. 30) to *h_rms (may be NULL,
 * then nothing synchronises).  D_E(U) of Eq. 25 takes the face coefficients
 * of Eq. 12 from E and the species fractions of d_U itself (limiter_lag:
 * the time-level coefficients). */
int rt_eval_residual(rt_grid* g, const double* d_U, const double* d_gn, double dt,
                     const rt_cosmo* c, double* d_f, double* h_rms);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * residual of rt_eval_residual without a grid or workspace, bit-identical to
 * it for the same parameters, medium and time-level data.  It calls no
 * hipMalloc, hipFree or allocating library routine: the reduction partials
 * and sums live in a static device array of 16 MiB + 256 B (NCOMP 4 x 2^19
 * block partials), which each GPU the library runs on holds until the
 * process ends; its device address is looked up once per device with
 * hipGetSymbolAddress on the first call (with that device current).
 *   p       grid parameters, as for rt_create_grid (limiter_lag must be 0:
 *           the lagged reading needs a grid's time-level coefficients)
 *   d_nH, d_eh [N], d_U, d_gn [nv][N]  device inputs as for rt_set_medium,
 *           rt_eval_residual (d_gn from rt_time_level of a grid, or the
 *           caller's own g^n of Eqs. 22-24)
 *   hip_stream  hipStream_t of the current device (NULL: default stream)
 *   d_f [nv][N]  device output, scaled residual
 *   h_rms   host output, RMS norm of Eq. 30 (NULL: none, and no host sync)
 *   err, err_len  optional host buffer for the message of a failure
 * Returns RT_EINVAL (message in err) for invalid parameters, the lagged
 * reading, null pointers or a grid whose partials exceed the array (more
 * than 2^19 stencil blocks: larger than 512^3); RT_EDEVICE for HIP errors.
 * All calls on one GPU share its array and keep the last call's contents:
 * calls that overlap on one GPU (other threads, other streams) race. */
int rt_eval_residual_noalloc(const rt_params* p, const double* d_nH, const double* d_eh,
                             const double* d_U, const double* d_gn, double dt,
                             const rt_cosmo* c, void* hip_stream, double* d_f, double* h_rms,
                             char* err, size_t err_len);

/* Cell-local Newton blocks (Sec. 3.2.1, Eqs. 31-34) in scaled variables:
 * d_M [nb][nb][N] = I + dt theta J_MM (row-major per cell),
 * d_Ucol [nb][N] = dt theta J_ME, d_Lrow [nb][N] = dt theta J_EM,
 * d_dloc [N] = 1 + dt theta dL_E/dE; nb = nspecies + 1. */
int rt_local_jacobian(rt_grid* g, const double* d_U, double dt, const rt_cosmo* c,
                      double* d_M, double* d_Ucol, double* d_Lrow, double* d_dloc);

/* Schur steps (i)-(ii) set-up (Sec. 3.2.1) for the exact Newton matrix of
 * the residual above: per cell GEPP on M gives f~_M = M^-1 f_M and
 * W = M^-1 U; the Schur matrix S = D - L W, with D the derivative of the
 * face fluxes of Eq. 25 with respect to E (through the gradient, R_f and
 * E_f of Eq. 12) and the species fractions of both cells of each face
 * (through the face opacity, folded in through W and f~_M, which keeps S
 * 7-point), and the right side d_b [N] = L f~_M - f_E (plus the fractions'
 * face terms).  S is not symmetric.  Beside it the preconditioner's
 * symmetric M-matrix: the cell-local part of S plus, on every face, the
 * derivative of the flux with respect to E_Q - E_P at fixed E_f and
 * opacity (>= 0), its diagonal raised to S's own where that is larger.
 * f~_M, W and both operators stay in the workspace for rt_mg_pcg_solve
 * and the line search. */
int rt_schur_form(rt_grid* g, const double* d_U, const double* d_f, double dt,
                  const rt_cosmo* c, double* d_b);

/* Copies of the workspace Schur data (any pointer may be NULL):
 * f~_M [nb][N], W [nb][N], the Schur diagonal [N], and the preconditioner
 * operator's +x/+y/+z face couplings c [N] each. */
int rt_schur_get(rt_grid* g, double* d_ftM, double* d_W, double* d_diag,
                 double* d_cx, double* d_cy, double* d_cz);

/* Copies of the rest (any pointer may be NULL): the Schur matrix's face
 * couplings fw = -S_{P,P+e_d} and bw = -S_{P+e_d,P} [3][N] (d = x, y, z
 * major), so that (S x)_P = diag_P x_P - sum_d (fw_d[P] x_{P+e_d} +
 * bw_d[P-e_d] x_{P-e_d}), and the preconditioner operator's diagonal [N]. */
int rt_schur_get_full(rt_grid* g, double* d_fw, double* d_bw, double* d_pdiag);

/* Replace the workspace Schur matrix by a caller's symmetric operator
 * (S x)_P = diag_P x_P - sum over faces c_f x_nbr, which is then also the
 * preconditioner's operator (for solver tests). */
int rt_set_operator(rt_grid* g, const double* d_diag, const double* d_cx,
                    const double* d_cy, const double* d_cz);

/* One application z = V r of the multigrid V-cycle preconditioner on the
 * preconditioner's operator (red-black Gauss-Seidel, trilinear transfers,
 * face-averaged coarse operators). */
int rt_mg_vcycle(rt_grid* g, const double* d_r, double* d_z);

/* Solve S s = b from s = 0 by the multigrid-preconditioned Krylov method of
 * krylov_restart (flexible GMRES, or CG for a symmetric operator) until
 * ||r||_2 <= rtol ||b||_2 (GMRES: its least-squares estimate) or maxit
 * iterations (rtol = 0: exactly maxit); *h_relres gets ||r||_2 / ||b||_2. */
int rt_mg_pcg_solve(rt_grid* g, const double* d_b, double* d_sE, double rtol,
                    int32_t maxit, int32_t* h_iters, double* h_relres);

/* Explicit predictor (Sec. 3.2.4, Eq. 44): writes d_Upred [nv][N] =
 * U^n - dt [L_e; L_n; D_E + L_E](U^n) + dt [0; 0; 4 pi eta], the forward
 * Euler step of the system (Eq. 44 printed with the tendency's sign such
 * that it steps backwards; this is the forward step), expansion factors
 * a_old, H_old and the limiter at U^n, then projected onto the physical
 * bounds (fractions into [0, 1], the helium pair to a sum <= 1, E >= 0) with
 * e_c kept at its t^n value where e_h + e_c would not be positive.  Meant as
 * the d_Ualt guess of rt_newton_step.  d_Upred must not be d_Un (RT_EINVAL). */
int rt_predict(rt_grid* g, const double* d_Un, double dt, const rt_cosmo* c, double* d_Upred);

/* Time-error estimate of Sec. 3.2.3 (Eqs. 41-42) between the new state and
 * the predictor, in the normalized unknowns U_v / u_v: with
 * w = sqrt(|a b|) + 1 and q = |a - b| / w per cell and unknown,
 * *h_eps = (sum q^p / (N nv))^(1/p) for p > 0, max q for p <= 0 (the max
 * norm).  Synchronises the stream.  RT_EINVAL for a non-finite p. */
int rt_time_error(rt_grid* g, const double* d_Unew, const double* d_Upred, double p,
                  double* h_eps);

/* One implicit time step (Sec. 3.2): time level from d_Un, Newton from the
 * guess in d_U (in: U_0, out: U^{n+1}).  If d_Ualt is not NULL it is a
 * second candidate guess: the one with the smaller initial residual norm is
 * used.  h_stats may be NULL.  Returns the step status (also in h_stats). */
int rt_newton_step(rt_grid* g, const double* d_Un, double* d_U, const double* d_Ualt,
                   double dt, const rt_cosmo* c, rt_newton_stats* h_stats);

/* End of an operator-split step (Sec. 3.1): e_h += e_c and e_c = 0 in place,
 * so that d_U can serve as U^n of the next step.  d_eh is the array given to
 * rt_set_medium (the caller owns it). */
int rt_fold_energy(rt_grid* g, double* d_U, double* d_eh);

/* Kernel classes timed by rt_timing. */
enum {
  RT_K_TIMELEVEL = 0,   /* face coefficients, explicit part, sources */
  RT_K_RESIDUAL,        /* residual + norm partials */
  RT_K_TRIAL,           /* line-search trial point */
  RT_K_SCHUR,           /* local blocks + GEPP + Schur assembly */
  RT_K_RBGS_FINE,       /* red-black Gauss-Seidel half sweep, finest level */
  RT_K_RBGS_COARSE,     /* same, coarser levels */
  RT_K_MG_TRANSFER,     /* multigrid residual, restriction, prolongation */
  RT_K_MG_SETUP,        /* coarse and box operators, precision conversion */
  RT_K_SPMV,            /* Schur matrix-vector product + dot */
  RT_K_CG_VECTOR,       /* CG updates and dots */
  RT_K_REDUCE,          /* final reductions and CG scalars */
  RT_K_BOX,             /* source-subdomain correction (one entry per graph replay) */
  RT_K_OTHER,
  RT_K_COUNT
};
typedef struct rt_kernel_timing {
  int32_t count[RT_K_COUNT];      /* launches */
  double  total_ms[RT_K_COUNT];   /* summed HIP-event durations */
  double  bytes[RT_K_COUNT];      /* algorithmic bytes (every field a launch    */
                                  /* must read or write, once) of ALL launches */
                                  /* made while collection was on, whatever    */
                                  /* classes are selected for events; final    */
                                  /* reductions and sources count 0, a box     */
                                  /* graph replay the sum over its launches    */
} rt_kernel_timing;

/* Per-launch HIP-event timing on the grid's stream.  enable = 1 clears and
 * starts collection; enable = 0 stops it, synchronises, and fills *out (may
 * be NULL).  Timing adds two event records per launch. */
int rt_timing(rt_grid* g, int32_t enable, rt_kernel_timing* out);

/* Restrict per-launch timing to the kernel classes whose bit (1 << class) is
 * set in `mask` (the default is every class), so that a measurement of one
 * class does not pay two event records on every other launch.  Takes effect
 * for launches after the call; RT_EINVAL for a null grid. */
int rt_timing_classes(rt_grid* g, uint32_t mask);

/* The source-subdomain correction (box_size > 0) issues a few hundred small
 * launches per V-cycle; by default the library captures them into a HIP
 * graph (on a private stream) per pair of input and output vectors in use
 * (FGMRES maps each basis vector to its own preconditioned vector: up to 31
 * pairs), replays the matching one, and drops them all when the number of
 * sources changes or graphs are switched off.  enable = 0 issues them one
 * by one instead:
 * the same kernels in the same order, so the results are identical.  A
 * timed correction counts as one RT_K_BOX entry per replay.  RT_EINVAL for
 * a null grid. */
int rt_use_graphs(rt_grid* g, int32_t enable);

/* Spectrum constants of Sec. 3.2.5 (Eq. 45) for a monochromatic 13.6 eV
 * (grey = 0) or a T_B blackbody (grey = 1) spectrum, by host quadrature. */
int rt_spectrum_constants(int32_t grey, double T_B, double* K_gamma3, double* K_kappa3,
                          double* K_heat3, double* hnu_mean);

/* ---- learned Newton initial guess (beside the paper's method) ------------
 * A 4-layer 3x3x3 periodic convolution network (channels nin -> 16 -> 16 ->
 * 16 -> nout, LeakyReLU 0.01 between layers) maps two time levels to a guess
 * of the next one; BF16 weights and activations, FP32 accumulation (MFMA).
 * Features per cell, for levels n and n-1: log10(E/u_E), e/u_e, logit(x_i)/10
 * (x clipped to [1e-12, 1 - 1e-12], E floored at 1e-10 u_E), plus
 * log10(n_H / nH_mean): nin = 2 (nspecies + 2) + 1.  Outputs (nout =
 * nspecies + 2): a correction to the linear extrapolation 2 t^n - t^(n-1) of
 * t = (log10 E/u_E, e/u_e, logit x_i / 10); the guess is the inverse
 * transform of their sum, with e_c = e - e_h.  Parameters (host FP32, flat): per
 * layer the weights in (offset, co, ci) order, offset o = (dx,dy,dz) =
 * (o/9 - 1, (o/3)%3 - 1, o%3 - 1), then the co biases.  Requires nz % 16 == 0
 * and nx, ny >= 3.  The caller owns the device workspace. */
typedef struct rt_net rt_net;
int rt_net_workspace_bytes(int32_t nspecies, int32_t nx, int32_t ny, int32_t nz, uint64_t* bytes);
int rt_net_create(int32_t nspecies, int32_t nx, int32_t ny, int32_t nz, void* d_ws,
                  uint64_t ws_bytes, void* hip_stream, rt_net** out);
int rt_net_destroy(rt_net* n);
const char* rt_net_last_error(const rt_net* n);
int rt_net_num_params(const rt_net* n);
/* Set (and reset the Adam state) / read the FP32 master parameters. */
int rt_net_set_params(rt_net* n, const float* h_theta, int32_t count);
int rt_net_get_params(rt_net* n, float* h_theta, int32_t count);
/* Guess d_Uguess [nv][N] from levels n (d_Un, total specific energy d_en) and
 * n-1 (d_Unm1, d_enm1); d_eh is the e_h of the coming step (for e_c). */
int rt_net_forward(rt_net* n, const double* d_Un, const double* d_Unm1, const double* d_en,
                   const double* d_enm1, const double* d_nH, double nH_mean, double u_e,
                   double u_E, const double* d_eh, double* d_Uguess);
/* Copies of the last network output [nout][N] (FP32) and of the BF16 input
 * features widened to FP32 [16][N] (either pointer may be NULL). */
int rt_net_get_output(rt_net* n, float* d_out, float* d_feat);
/* One training sample (levels n-1, n with converged level n+1 as target):
 * mean squared error (radiation channel weighted per cell by E^n/u_E over its
 * box mean, capped at 100; other channels by 1) to *h_loss, gradient to h_grad
 * (host, may be NULL); lr > 0 then applies one Adam step (beta 0.9/0.999,
 * eps 1e-8) on the gradient clipped to global norm 1. */
int rt_net_train_step(rt_net* n, const double* d_Un, const double* d_Unm1, const double* d_en,
                      const double* d_enm1, const double* d_nH, double nH_mean, double u_e,
                      double u_E, const double* d_Unp1, const double* d_enp1, float lr,
                      float* h_loss, float* h_grad);

#ifdef __cplusplus
}
#endif
#endif /* RT_H */
