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
 * (Sec. 3.2.1, Eqs. 33-35) and solved by multigrid-preconditioned conjugate
 * gradients.
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
 *            object behind rt_grid.  Pointers passed to rt_set_medium must
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
  int32_t nspecies;         /* 1: HI; 3: HI, HeI, HeII (Sec. 2, Eq. 4) */
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
 * U^n + dt (theta-1) [L_e; L_n; D_E + L_E](U^n) + dt [0; 0; 4 pi eta], and
 * stores in the workspace the flux-limiter face coefficients of Eq. 12
 * evaluated at U^n, which every later residual and Schur call of the step
 * uses (the limiter is lagged to time level n). */
int rt_time_level(rt_grid* g, const double* d_Un, double dt, const rt_cosmo* c,
                  double* d_gn);

/* Nonlinear residual (Sec. 3.2, Eq. 29) in scaled variables f_v / u_v,
 * written to d_f [nv][N], and its RMS norm (Eq. 30) to *h_rms (may be NULL,
 * then nothing synchronises).  Uses the time-level coefficients. */
int rt_eval_residual(rt_grid* g, const double* d_U, const double* d_gn, double dt,
                     const rt_cosmo* c, double* d_f, double* h_rms);

/* Cell-local Newton blocks (Sec. 3.2.1, Eqs. 31-34) in scaled variables:
 * d_M [nb][nb][N] = I + dt theta J_MM (row-major per cell),
 * d_Ucol [nb][N] = dt theta J_ME, d_Lrow [nb][N] = dt theta J_EM,
 * d_dloc [N] = 1 + dt theta dL_E/dE; nb = nspecies + 1. */
int rt_local_jacobian(rt_grid* g, const double* d_U, double dt, const rt_cosmo* c,
                      double* d_M, double* d_Ucol, double* d_Lrow, double* d_dloc);

/* Schur steps (i)-(ii) set-up (Sec. 3.2.1): per cell GEPP on M gives
 * f~_M = M^-1 f_M and W = M^-1 U; the Schur matrix S = D - L W (7-point,
 * symmetric) and right side d_b [N] = L f~_M - f_E.  f~_M, W and S stay in
 * the workspace for rt_mg_pcg_solve and the line search. */
int rt_schur_form(rt_grid* g, const double* d_U, const double* d_f, double dt,
                  const rt_cosmo* c, double* d_b);

/* Copies of the workspace Schur data (any pointer may be NULL):
 * f~_M [nb][N], W [nb][N], diag [N], and the +x/+y/+z face couplings [N]. */
int rt_schur_get(rt_grid* g, double* d_ftM, double* d_W, double* d_diag,
                 double* d_cx, double* d_cy, double* d_cz);

/* Replace the workspace Schur matrix by a caller operator
 * (S x)_P = diag_P x_P - sum over faces c_f x_nbr (for solver tests). */
int rt_set_operator(rt_grid* g, const double* d_diag, const double* d_cx,
                    const double* d_cy, const double* d_cz);

/* One application z = V r of the multigrid V-cycle preconditioner on the
 * current Schur matrix (red-black Gauss-Seidel, trilinear transfers, face-
 * averaged coarse operators). */
int rt_mg_vcycle(rt_grid* g, const double* d_r, double* d_z);

/* Solve S s = b by multigrid-preconditioned CG from s = 0 until
 * ||r||_2 <= rtol ||b||_2 or maxit iterations (rtol = 0: exactly maxit). */
int rt_mg_pcg_solve(rt_grid* g, const double* d_b, double* d_sE, double rtol,
                    int32_t maxit, int32_t* h_iters, double* h_relres);

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
  RT_K_MG_SETUP,        /* coarse operators and precision conversion */
  RT_K_SPMV,            /* Schur matrix-vector product + dot */
  RT_K_CG_VECTOR,       /* CG updates and dots */
  RT_K_REDUCE,          /* final reductions and CG scalars */
  RT_K_OTHER,
  RT_K_COUNT
};
typedef struct rt_kernel_timing {
  int32_t count[RT_K_COUNT];      /* launches */
  double  total_ms[RT_K_COUNT];   /* summed HIP-event durations */
} rt_kernel_timing;

/* Per-launch HIP-event timing on the grid's stream.  enable = 1 clears and
 * starts collection; enable = 0 stops it, synchronises, and fills *out (may
 * be NULL).  Timing adds two event records per launch. */
int rt_timing(rt_grid* g, int32_t enable, rt_kernel_timing* out);

/* Spectrum constants of Sec. 3.2.5 (Eq. 45) for a monochromatic 13.6 eV
 * (grey = 0) or a T_B blackbody (grey = 1) spectrum, by host quadrature. */
int rt_spectrum_constants(int32_t grey, double T_B, double* K_gamma3, double* K_kappa3,
                          double* K_heat3, double* hnu_mean);

#ifdef __cplusplus
}
#endif
#endif /* RT_H */
