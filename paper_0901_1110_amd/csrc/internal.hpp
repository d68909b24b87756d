// Launchers of the gfx950 kernels (defined in kernels.hip) used by the host
// solver control (api.hip).  All launches are asynchronous on `st`.
#pragma once

#include <hip/hip_runtime.h>

#include "physics.hpp"

namespace rtk {

constexpr int BLOCK = 256;          // threads per block (4 wave64)
constexpr int MAX_PARTS = 2048;     // partial sums per reduction
constexpr int NCOMP_MAX = 4;        // components per reduction
constexpr int KMAX = 32;            // components of the FGMRES reductions (restart <= KMAX - 2)

// Number of blocks a reduction kernel over n items uses (fixed per n, so the
// summation tree, and therefore the result, is deterministic).
inline int reduce_blocks(long n) {
  long b = (n + BLOCK - 1) / BLOCK;
  return (int)(b < MAX_PARTS ? (b < 1 ? 1 : b) : MAX_PARTS);
}

// Indices of the device scalar slots used by CG.
enum Scalar { S_RHO = 0, S_PQ, S_ALPHA, S_RR, S_ZR, S_ZQ, S_BETA, S_BB, S_FN, S_VIOL, S_TSUM, S_TMAX,
              S_RHO2, S_COUNT };
// the box correction's inner CG: partial sets longer than this are reduced by
// a launch of their own into these box scalar slots (one partial of
// NCOMP_MAX components each) instead of by every block of the next kernel
constexpr int BOX_INLINE_PARTS = 256;
constexpr int BOX_SLOT_ZPARTS = 16, BOX_SLOT_PQPARTS = 20;
static_assert(S_COUNT <= BOX_SLOT_ZPARTS && BOX_SLOT_PQPARTS + NCOMP_MAX <= 32, "box scalar slots");

struct Step {     // per-call time-step data
  double dt, a, H;
};

// ---- residual / time level ----
void launch_faces(const DevParams& P, const double* Un, const double* nH, double a,
                  double* D, hipStream_t st);
void launch_explicit(const DevParams& P, const double* Un, const double* nH, const double* eh,
                     const double* D, Step s, double* g, hipStream_t st);
void launch_sources(const long long* cells, const double* Q, int n, double scale, double* gE,
                    hipStream_t st);
// residual with the flux limiter evaluated at U, or (Dlag non-null) with the
// face coefficients stored at time level n
void launch_residual(const DevParams& P, const double* U, const double* g, const double* nH,
                     const double* eh, const double* Dlag, Step s, double* f, double* parts,
                     hipStream_t st);
// explicit predictor: projection of U^n - dt L(U^n) + sources (already in Up)
void launch_predict_project(const DevParams& P, const double* Un, const double* eh, double* Up,
                            hipStream_t st);
// time-error partials (sum of q^p for p > 0, max q); returns the partial count
int launch_time_error(const DevParams& P, const double* A, const double* B, double p,
                      double* parts, hipStream_t st);
void launch_final_summax(const double* parts, int nparts, double* out, hipStream_t st);
void launch_trial(const DevParams& P, const double* U, const double* ftM, const double* W,
                  const double* sE, double lambda, double* Ut, hipStream_t st);
void launch_local_jac(const DevParams& P, const double* U, const double* nH, const double* eh,
                      Step s, double* M, double* Ucol, double* Lrow, double* dloc,
                      hipStream_t st);
// Schur step (i) and the local part of (ii): ftM, W, loc (local diagonal), b
// (local right side), om, ph (species columns coupled through the opacity)
void launch_schur_local(const DevParams& P, const double* U, const double* f, const double* nH,
                        const double* eh, Step s, double* ftM, double* W, double* loc, double* b,
                        double* om, double* ph, hipStream_t st);
// the face terms: diag, the preconditioner's pdiag and couplings c (3N),
// the full operator's couplings fw, bw (3N each), b completed; pd32..cz32
// non-null: FP32 colour-split copies of pdiag and c
// (Dlag non-null: the lagged face coefficients, a symmetric S)
void launch_schur_faces(const DevParams& P, const double* U, const double* nH, const double* Dlag,
                        Step s, const double* loc, const double* om, const double* ph,
                        double* diag, double* pdiag, double* c, double* fw, double* bw, double* b,
                        float* pd32, float* cx32, float* cy32, float* cz32, hipStream_t st);

// ---- flexible GMRES kernels (FP64); the reductions return their block count ----
int launch_spmv_full(int nx, int ny, int nz, const double* diag, const double* fw,
                     const double* bw, const double* z, const double* bsub, double* w,
                     double* zcopy, const double* V, int nvec, double* parts, hipStream_t st);
int launch_gs_pass(long N, double* w, const double* V, int nvec, const double* coef, int dots,
                   double* parts, hipStream_t st);
void launch_scale(long N, double* v, double sf, double* copy, float* r32, int ny, int nz,
                  hipStream_t st);
void launch_combine(long N, double* x, const double* Z, int nvec, const double* y, hipStream_t st);
void launch_final_multi(const double* parts, int nblk, int ncomp, double* out, hipStream_t st);

// ---- reductions / scalars ----
void launch_final_reduce(const double* parts, int nparts, int ncomp, double* out,
                         hipStream_t st);
// the final reduction of p.q followed by alpha, and of (z.r, z.q) followed
// by beta and rho <- z.r, each in one launch
void launch_final_reduce_alpha(const double* parts, int nparts, double* sc, hipStream_t st);
void launch_final_reduce_beta(const double* parts, int nparts, double* sc, hipStream_t st);

// ---- CG vector kernels (FP64) ----
void launch_spmv_dot(int nx, int ny, int nz, const double* diag, const double* cx,
                     const double* cy, const double* cz, const double* p, double* q,
                     double* parts, hipStream_t st);
void launch_update_xr(long n, double* x, double* r, const double* p, const double* q,
                      const double* sc, double* parts, hipStream_t st,
                      float* r32 = nullptr, int ny = 0, int nz = 0);
void launch_dot2(long n, const double* z, const double* r, const double* q, double* parts,
                 hipStream_t st);
void launch_dot1(long n, const double* a, const double* b, double* parts, hipStream_t st,
                 double* copy_b = nullptr);
void launch_update_p(long n, double* p, const double* z, const double* sc, hipStream_t st);

// ---- multigrid (T = double or float) ----
template <class T>
struct Level {
  int nx, ny, nz;
  T *diag, *cx, *cy, *cz;   // operator
  T *x, *b, *r;             // solution, right side, residual scratch
  int split = 0;            // 1: colour-split rows (finest level of the FP32 cycle)
  int blocks = 1;           // independent x-blocks (zero coupling between them)
};
template <class T> void launch_fill(long n, T* x, T v, hipStream_t st);
template <class T> void launch_rbgs(const Level<T>& L, int colour, hipStream_t st);
// first (red, black) pair from x = 0
template <class T> void launch_rbgs_first_pair(const Level<T>& L, T* xo, hipStream_t st);
// half-sweep whose result (both colours) goes widened to out64 instead of x;
// parts non-null: also the block partials of out64.r64 and out64.q64
template <class T>
void launch_rbgs_out64(const Level<T>& L, int colour, double* out64, const double* r64,
                       const double* q64, double* parts, hipStream_t st);
// half-sweep in place that also leaves the block partials of x.r and x.q
// (all cells); returns their count
template <class T>
int launch_rbgs_dots(const Level<T>& L, int colour, const T* r, const T* q, double* parts,
                     hipStream_t st);
template <class T> void launch_coarse_solve(const Level<T>& L, int sweeps, hipStream_t st);
// coarsest solve with each x-block in registers and LDS, one workgroup per
// block (n / blocks <= COARSE_LDS_MAX, nx divisible by blocks)
template <class T> void launch_coarse_solve_lds(const Level<T>& L, int sweeps, hipStream_t st);
constexpr int COARSE_LDS_MAX = 4096;
int stencil_blocks(int nx, int ny, int nz);   // blocks (= partial sums) of a 3-D stencil launch
constexpr int COARSE_SOLVE_MAX = 8192;        // coarsest levels up to this size: one workgroup
// red_only: the level's black cells satisfy their equations (the smoothing
// ended with the black half-sweep), so their residual is taken as zero
template <class T> void launch_mg_residual(const Level<T>& L, int red_only, hipStream_t st);
template <class T> void launch_restrict(const Level<T>& F, const Level<T>& C, int red_only,
                                        hipStream_t st);
// colour >= 0: correct only the cells of that colour
template <class T> void launch_prolong_add(const Level<T>& C, const Level<T>& F, int colour, hipStream_t st);
template <class T> void launch_coarsen(const Level<T>& F, const Level<T>& C, hipStream_t st);
void launch_fold_energy(int N, double* U, double* eh, hipStream_t st);
void launch_cvt_d2f(long n, const double* a, float* b, hipStream_t st);
// source subdomains (boxes of B^3 cells around each source, stacked along x)
void launch_box_extract(int nx, int ny, int nz, int B, int nbox, const long long* cells,
                        const double* diag, const double* cx, const double* cy, const double* cz,
                        double* bd, double* bx, double* by, double* bz, hipStream_t st);
// r - S z on the box cells, into the stacked box vector bv
template <class T>
void launch_box_residual(int nx, int ny, int nz, int B, int nbox, const long long* cells,
                         const double* diag, const double* cx, const double* cy, const double* cz,
                         const double* r, const double* z, T* bv, hipStream_t st);
// z += box s's part of the stacked vector y; parts non-null: also the
// stencil_blocks(B, B, B) block partials of y.r and y.q over the box
template <class T>
void launch_box_scatter_add(int nx, int ny, int nz, int B, int nbox, const long long* cells, int s,
                            const T* y, double* z, const double* r, const double* q,
                            double* parts, hipStream_t st);
// red-black half-sweep of colour `colour` on S z = r (full Schur operator,
// FP64 main grid) over the cells of box s
void launch_box_smooth_s(int nx, int ny, int nz, int B, int nbox, const long long* cells, int s,
                         int colour, const double* diag, const double* fw, const double* bw,
                         const double* r, double* z, hipStream_t st);
// all `sweeps` (red, black) sweeps of launch_box_smooth_s over box s in one
// workgroup with the box in LDS; for B <= BOX_S_LDS_MAX and B smaller than
// nx, ny and nz
constexpr int BOX_S_LDS_MAX = 16;
void launch_box_smooth_s_lds(int nx, int ny, int nz, int B, int nbox, const long long* cells, int s,
                             int sweeps, const double* diag, const double* fw, const double* bw,
                             const double* r, double* z, hipStream_t st);
// inner PCG of the correction on the stacked boxes (level L: the box
// operator in T); the reduction launches return their partial count
template <class T>
int launch_box_dot1p(long n, const T* r, const T* z, T* p, double* parts, hipStream_t st);
// beta from the partials of z.r, z.q (rho <- z.r into slot rho_out),
// pout = z + beta pin (first: z), q = S pout, partials of pout.q
template <class T>
int launch_box_spmv_p(const Level<T>& L, const T* z, const T* pin, T* pout, T* q,
                      const double* zparts, int nz_parts, double* sc, int rho_in, int rho_out,
                      bool first, double* parts, hipStream_t st);
// alpha = sc[rho] / (p.q) from its partials (into sc[S_ALPHA]), x += alpha p, r -= alpha q
template <class T>
void launch_box_update_xr(long n, T* x, T* r, const T* p, const T* q, const double* pqparts,
                          int npq, double* sc, int rho, hipStream_t st);
// the update above fused with the first (red, black) pair of the box V-cycle
// (level L, right side rn = ro - alpha q, written to rn; L.x receives the pair)
template <class T>
void launch_box_update_first_pair(const Level<T>& L, T* x, const T* ro, T* rn, const T* p,
                                  const T* q, const double* pqparts, int npq, double* sc, int rho,
                                  hipStream_t st);
template <class T>
int launch_box_dot2(long n, const T* z, const T* r, const T* q, double* parts, hipStream_t st);
// FP64 natural field -> FP32 field in the layout of level L
void launch_cvt_d2f_level(const Level<float>& L, const double* a, float* b, hipStream_t st);
// FP64 natural field -> the colour-split FP64 finest level L (L.split set)
void launch_cvt_split_d(const Level<double>& L, const double* a, double* b, hipStream_t st);
void launch_cvt_f2d(long n, const float* a, double* b, hipStream_t st);

}  // namespace rtk
