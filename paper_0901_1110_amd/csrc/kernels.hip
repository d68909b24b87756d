// gfx950 kernels of the implicit radiation / ionization / energy Newton step.
//
// Layout: every field is structure-of-arrays FP64 (FP32 for the mixed-
// precision V-cycle), cell (i,j,k) at (i*ny + j)*nz + k, periodic.  One
// thread owns one cell; consecutive lanes of a 64-wide wavefront own
// consecutive z cells, so every field access of a wavefront is a coalesced
// 512-byte (FP64) line run and the +-z, +-y neighbours of a block are served
// from the L2 lines the block itself brings in.  All kernels are HBM-bound
// (a few hundred flops per cell against 50-150 bytes); reductions are
// deterministic: fixed grid, wave64 butterfly, fixed-order block and final
// combine.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace rtk {

// ---------------------------------------------------------------------------
// indexing: stencil kernels launch a 3-D grid, x along z (fastest), y along
// y, one grid slice per x-plane, so cell coordinates need no division.
struct Nb {
  int xm, xp, ym, yp, zm, zp;
};

__device__ inline Nb nbrs(int i, int j, int k, int nx, int ny, int nz) {
  const int sx = ny * nz;
  const int idx = (i * ny + j) * nz + k;
  Nb n;
  n.xp = idx + (i + 1 < nx ? sx : -(nx - 1) * sx);
  n.xm = idx + (i > 0 ? -sx : (nx - 1) * sx);
  n.yp = idx + (j + 1 < ny ? nz : -(ny - 1) * nz);
  n.ym = idx + (j > 0 ? -nz : (ny - 1) * nz);
  n.zp = idx + (k + 1 < nz ? 1 : -(nz - 1));
  n.zm = idx + (k > 0 ? -1 : (nz - 1));
  return n;
}

// coordinates of this thread in a 3-D launch over (nx, ny, ext); ok = in range
struct C3 {
  int i, j, k;
  bool ok;
};
__device__ inline C3 coord3(int ny, int ext) {
  C3 c;
  c.k = blockIdx.x * blockDim.x + threadIdx.x;
  c.j = blockIdx.y * blockDim.y + threadIdx.y;
  c.i = blockIdx.z;
  c.ok = c.k < ext && c.j < ny;
  return c;
}
__device__ inline int block_linear() {
  return (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
}

// ---------------------------------------------------------------------------
// deterministic block reduction of NC values (result valid in thread 0)
template <int NC>
__device__ inline void block_reduce(double (&v)[NC], double* out) {
  __shared__ double sh[BLOCK / 64][NC];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int nthr = blockDim.x * blockDim.y;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double x = v[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[c] = x;
  }
  const int lane = tid & 63;
  const int w = tid >> 6;
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NC; ++c) sh[w][c] = v[c];
  }
  __syncthreads();
  if (tid == 0) {
    const int nw = (nthr + 63) >> 6;
    const int b = block_linear();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double s = 0.0;
      for (int i = 0; i < nw; ++i) s += sh[i][c];
      out[(size_t)b * NCOMP_MAX + c] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// time level: face coefficients at U^n (lagged flux limiter)
template <int NS>
__global__ __launch_bounds__(BLOCK) void k_faces(DevParams P, const double* __restrict__ Un,
                                                  const double* __restrict__ nH, double a,
                                                  double* __restrict__ D) {
  const int N = P.N;
  const C3 c = coord3(P.ny, P.nz);
  if (!c.ok) return;
  const int idx = (c.i * P.ny + c.j) * P.nz + c.k;
  const Nb nb = nbrs(c.i, c.j, c.k, P.nx, P.ny, P.nz);
  const double* E = Un + (NS + 1) * N;
  double x[NS > 0 ? NS : 1];
  const int nbr[3] = {nb.xp, nb.yp, nb.zp};
#pragma unroll
  for (int s = 0; s < NS; ++s) x[s] = Un[(1 + s) * N + idx];
  const double kP = opacity<NS>(x, nH[idx], a, P);
  const double EP = E[idx];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int q = nbr[d];
    double xq[NS > 0 ? NS : 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) xq[s] = Un[(1 + s) * N + q];
    const double kQ = opacity<NS>(xq, nH[q], a, P);
    // non-periodic: no face joins the last cell of a row to the first; with
    // the x-left Dirichlet face that x slot holds the face between the ghost
    // cell (E_dirichlet, the first cell's opacity) and the first cell
    const bool wrap = d == 0 ? c.i == P.nx - 1 : (d == 1 ? c.j == P.ny - 1 : c.k == P.nz - 1);
    if (P.bc != 0 && wrap)
      D[d * N + idx] = (P.bc == 2 && d == 0) ? face_D(P.Eb, E[q], kQ, kQ, a, P) : 0.0;
    else
      D[d * N + idx] = face_D(EP, E[q], kP, kQ, a, P);
  }
}

// sum over the faces of D_f (E_nbr - E_P) with the +/- ordering of the text;
// with the x-left Dirichlet face (bc 2) the first cell's x neighbour is the
// ghost value and the last cell has no +x face
__device__ inline double diffusion_sum(const double* __restrict__ E, const double* __restrict__ D,
                                       int N, int idx, const Nb& nb, double EP, int i,
                                       const DevParams& P) {
  double acc = 0.0;
  double Dxp = D[idx], Exm = E[nb.xm];
  if (P.bc == 2) {
    if (i == P.nx - 1) Dxp = 0.0;
    if (i == 0) Exm = P.Eb;
  }
  acc += Dxp * (E[nb.xp] - EP) - D[nb.xm] * (EP - Exm);
  acc += D[N + idx] * (E[nb.yp] - EP) - D[N + nb.ym] * (EP - E[nb.ym]);
  acc += D[2 * N + idx] * (E[nb.zp] - EP) - D[2 * N + nb.zm] * (EP - E[nb.zm]);
  return acc;
}

// g = U^n + dt (theta - 1) [L; D_E + L_E](U^n)   (theta != 1)
template <int NS>
__global__ __launch_bounds__(BLOCK) void k_explicit(DevParams P, const double* __restrict__ Un,
                                                     const double* __restrict__ nH,
                                                     const double* __restrict__ eh,
                                                     const double* __restrict__ D, Step s,
                                                     double* __restrict__ g) {
  constexpr int NV = NS + 2;
  const int N = P.N;
  const C3 c = coord3(P.ny, P.nz);
  if (!c.ok) return;
  const int idx = (c.i * P.ny + c.j) * P.nz + c.k;
  double u[NV], L[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = Un[v * N + idx];
  local_ops<NS, double>(u, nH[idx], eh[idx], s.a, s.H, P, L);
  const Nb nb = nbrs(c.i, c.j, c.k, P.nx, P.ny, P.nz);
  const double dif = diffusion_sum(Un + (NS + 1) * N, D, N, idx, nb, u[NS + 1], c.i, P);
  L[NS + 1] += -dif / (s.a * s.a * P.dx * P.dx);
  const double w = s.dt * (P.theta - 1.0);
#pragma unroll
  for (int v = 0; v < NV; ++v) g[v * N + idx] = u[v] + w * L[v];
}

__global__ void k_sources(const long long* __restrict__ cells, const double* __restrict__ Q, int n,
                          double scale, double* __restrict__ gE) {
  // one thread, fixed order: several sources may share a cell
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int i = 0; i < n; ++i) gE[cells[i]] += scale * Q[i];
  }
}

// ---------------------------------------------------------------------------
// live face fluxes: the limiter of Eq. 12 evaluated at the state U itself

// proper opacity of cell q of the state U
template <int NS>
__device__ inline double opacity_of(const double* __restrict__ U, const double* __restrict__ nH,
                                    int N, int q, double a, const DevParams& P) {
  double x[NS > 0 ? NS : 1];
#pragma unroll
  for (int s = 0; s < NS; ++s) x[s] = U[(1 + s) * N + q];
  return opacity<NS>(x, nH[q], a, P);
}

// sum over the three directions of F_{P+} - F_{P-}, F = D_f (E_Q - E_P) with
// D_f from E and the opacities of the face's two cells.  Non-periodic grids
// carry no flux through the domain faces, except the x-left Dirichlet face
// (bc 2), whose ghost cell holds E_dirichlet with the first cell's opacity.
// A face is evaluated by both of its cells with the same arguments in the
// same order, so both see the same value.
template <int NS>
__device__ inline double live_flux_sum(const double* __restrict__ U, const double* __restrict__ nH,
                                       int N, int idx, const Nb& nb, int i, int j, int k,
                                       double a, const DevParams& P) {
  const double* E = U + (NS + 1) * N;
  const double EP = E[idx];
  const double kP = opacity_of<NS>(U, nH, N, idx, a, P);
  const int np_[3] = {nb.xp, nb.yp, nb.zp};
  const int nm_[3] = {nb.xm, nb.ym, nb.zm};
  const bool last[3] = {i == P.nx - 1, j == P.ny - 1, k == P.nz - 1};
  const bool first[3] = {i == 0, j == 0, k == 0};
  double acc = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double Fp = 0.0, Fm = 0.0;
    if (!(P.bc != 0 && last[d])) {
      const int q = np_[d];
      const double EQ = E[q];
      Fp = face_D(EP, EQ, kP, opacity_of<NS>(U, nH, N, q, a, P), a, P) * (EQ - EP);
    }
    if (!(P.bc != 0 && first[d])) {
      const int r = nm_[d];
      const double ER = E[r];
      Fm = face_D(ER, EP, opacity_of<NS>(U, nH, N, r, a, P), kP, a, P) * (EP - ER);
    } else if (P.bc == 2 && d == 0) {
      Fm = face_D(P.Eb, EP, kP, kP, a, P) * (EP - P.Eb);
    }
    acc += Fp - Fm;
  }
  return acc;
}

// ---------------------------------------------------------------------------
// residual f~ = (U + dt theta [L; D_E + L_E](U) - g) / u  and sum f~^2,
// count of cells with e_h + e_c <= 0; D_E(U) with the limiter at U
// Dlag non-null: the face coefficients held at time level n (the lagged
// limiter reading) instead of the limiter at U
template <int NS>
__global__ __launch_bounds__(BLOCK) void k_residual(DevParams P, const double* __restrict__ U,
                                                     const double* __restrict__ g,
                                                     const double* __restrict__ nH,
                                                     const double* __restrict__ eh,
                                                     const double* __restrict__ Dlag, Step s,
                                                     double* __restrict__ f,
                                                     double* __restrict__ parts) {
  constexpr int NV = NS + 2;
  const int N = P.N;
  const double dtt = s.dt * P.theta;
  const double inv_a2dx2 = 1.0 / (s.a * s.a * P.dx * P.dx);
  double acc[2] = {0.0, 0.0};
  const C3 c = coord3(P.ny, P.nz);
  if (c.ok) {
    const int idx = (c.i * P.ny + c.j) * P.nz + c.k;
    double u[NV], L[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[v * N + idx];
    const double ehv = eh[idx];
    local_ops<NS, double>(u, nH[idx], ehv, s.a, s.H, P, L);
    const Nb nb = nbrs(c.i, c.j, c.k, P.nx, P.ny, P.nz);
    const double dif =
        Dlag ? diffusion_sum(U + (NS + 1) * N, Dlag, N, idx, nb, u[NS + 1], c.i, P)
             : live_flux_sum<NS>(U, nH, N, idx, nb, c.i, c.j, c.k, s.a, P);
    L[NS + 1] += -dif * inv_a2dx2;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double sc = v == 0 ? P.u_e : (v == NS + 1 ? P.u_E : 1.0);
      const double fv = (u[v] + dtt * L[v] - g[v * N + idx]) / sc;
      f[v * N + idx] = fv;
      acc[0] += fv * fv;
    }
    if (!(ehv + u[0] > 0.0)) acc[1] += 1.0;
  }
  block_reduce<2>(acc, parts);
}

// trial point U_t = project(U + lambda u * [s_M; s_E]), s_M = -f~_M - W s_E
template <int NS>
__global__ __launch_bounds__(BLOCK) void k_trial(DevParams P, const double* __restrict__ U,
                                                  const double* __restrict__ ftM,
                                                  const double* __restrict__ W,
                                                  const double* __restrict__ sE, double lam,
                                                  double* __restrict__ Ut) {
  constexpr int NB = NS + 1;
  const int N = P.N;
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= N) return;
  const double se = sE[idx];
  double v[NS + 2];
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    const double sc = r == 0 ? P.u_e : 1.0;
    const double step = (-ftM[r * N + idx] - W[r * N + idx] * se) * sc;
    v[r] = U[r * N + idx] + lam * step;
  }
  v[NB] = U[NB * N + idx] + lam * (se * P.u_E);
  // projection onto the physical bounds
#pragma unroll
  for (int r = 1; r <= NS; ++r) v[r] = fmin(fmax(v[r], 0.0), 1.0);
  if constexpr (NS == 3) {
    const double tot = v[2] + v[3];
    if (tot > 1.0) {
      v[2] = v[2] / tot;
      v[3] = v[3] / tot;
    }
  }
  v[NB] = fmax(v[NB], 0.0);
#pragma unroll
  for (int r = 0; r < NS + 2; ++r) Ut[r * N + idx] = v[r];
}

// the explicit predictor's projection (Sec. 3.2.4): fractions into [0, 1]
// (the helium pair rescaled to a sum <= 1), E >= 0, and e_c kept at its
// value at t^n where e_h + e_c would not be positive
template <int NS>
__global__ __launch_bounds__(BLOCK) void k_predict_project(DevParams P, const double* __restrict__ Un,
                                                          const double* __restrict__ eh,
                                                          double* __restrict__ Up) {
  const int N = P.N;
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= N) return;
  double v[NS + 2];
#pragma unroll
  for (int r = 0; r < NS + 2; ++r) v[r] = Up[r * N + idx];
#pragma unroll
  for (int r = 1; r <= NS; ++r) v[r] = fmin(fmax(v[r], 0.0), 1.0);
  if constexpr (NS == 3) {
    const double tot = v[2] + v[3];
    if (tot > 1.0) {
      v[2] = v[2] / tot;
      v[3] = v[3] / tot;
    }
  }
  v[NS + 1] = fmax(v[NS + 1], 0.0);
  if (!(eh[idx] + v[0] > 0.0)) v[0] = Un[idx];
#pragma unroll
  for (int r = 0; r < NS + 2; ++r) Up[r * N + idx] = v[r];
}

// time-error estimate (Sec. 3.2.3, Eqs. 41-42) in the normalized unknowns:
// q = |a - b| / (sqrt(|a b|) + 1); block partials of sum q^p (p > 0) and of
// max q
template <int NS>
__global__ __launch_bounds__(BLOCK) void k_time_error(DevParams P, const double* __restrict__ A,
                                                     const double* __restrict__ B, double p,
                                                     double* __restrict__ parts) {
  constexpr int NV = NS + 2;
  const int N = P.N;
  double sum = 0.0, mx = 0.0;
  for (int idx = blockIdx.x * BLOCK + threadIdx.x; idx < N; idx += gridDim.x * BLOCK) {
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      const double sc = r == 0 ? P.u_e : (r == NV - 1 ? P.u_E : 1.0);
      const double a = A[(size_t)r * N + idx] / sc, b = B[(size_t)r * N + idx] / sc;
      const double q = fabs(a - b) / (sqrt(fabs(a * b)) + 1.0);
      mx = fmax(mx, q);
      if (p > 0.0) sum += p == 2.0 ? q * q : (p == 1.0 ? q : pow(q, p));
    }
  }
  __shared__ double sh[BLOCK / 64][2];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sum += __shfl_xor(sum, off, 64);
    mx = fmax(mx, __shfl_xor(mx, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6][0] = sum;
    sh[threadIdx.x >> 6][1] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, m = 0.0;
    for (int w = 0; w < BLOCK / 64; ++w) {
      s += sh[w][0];
      m = fmax(m, sh[w][1]);
    }
    parts[(size_t)blockIdx.x * NCOMP_MAX] = s;
    parts[(size_t)blockIdx.x * NCOMP_MAX + 1] = m;
  }
}
// out[0] = sum of the partials' first components (fixed order), out[1] = max
// of the second
__global__ __launch_bounds__(1024) void k_final_summax(const double* __restrict__ parts, int nparts,
                                                       double* __restrict__ out) {
  __shared__ double sh[1024 / 64][2];
  double s = 0.0, m = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 1024) {
    s += parts[(size_t)i * NCOMP_MAX];
    m = fmax(m, parts[(size_t)i * NCOMP_MAX + 1]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    m = fmax(m, __shfl_xor(m, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6][0] = s;
    sh[threadIdx.x >> 6][1] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0, u = 0.0;
    for (int w = 0; w < 1024 / 64; ++w) {
      t += sh[w][0];
      u = fmax(u, sh[w][1]);
    }
    out[0] = t;
    out[1] = u;
  }
}

// ---------------------------------------------------------------------------
// local Jacobian blocks by forward-mode differentiation of local_ops
template <int NS>
__device__ inline void local_blocks(const DevParams& P, const double* u, double nHv, double ehv,
                                    Step s, double (&M)[NS + 1][NS + 1], double (&Uc)[NS + 1],
                                    double (&Lr)[NS + 1], double& dloc) {
  constexpr int NV = NS + 2;
  constexpr int NB = NS + 1;
  double us[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) us[v] = v == 0 ? P.u_e : (v == NV - 1 ? P.u_E : 1.0);
  Dual<NV> ud[NV], Ld[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    ud[v] = Dual<NV>(u[v]);
    ud[v].d[v] = us[v];          // derivative with respect to the scaled unknown
  }
  local_ops<NS, Dual<NV>>(ud, nHv, ehv, s.a, s.H, P, Ld);
  const double dtt = s.dt * P.theta;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
#pragma unroll
    for (int j = 0; j < NB; ++j) M[i][j] = (i == j ? 1.0 : 0.0) + dtt * Ld[i].d[j] / us[i];
    Uc[i] = dtt * Ld[i].d[NB] / us[i];
    Lr[i] = dtt * Ld[NB].d[i] / us[NB];
  }
  dloc = 1.0 + dtt * Ld[NB].d[NB] / us[NB];
}

template <int NS>
__global__ __launch_bounds__(BLOCK) void k_local_jac(DevParams P, const double* __restrict__ U,
                                                      const double* __restrict__ nH,
                                                      const double* __restrict__ eh, Step s,
                                                      double* __restrict__ Mo,
                                                      double* __restrict__ Uo,
                                                      double* __restrict__ Lo,
                                                      double* __restrict__ Do) {
  constexpr int NB = NS + 1;
  const int N = P.N;
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= N) return;
  double u[NS + 2];
#pragma unroll
  for (int v = 0; v < NS + 2; ++v) u[v] = U[v * N + idx];
  double M[NB][NB], Uc[NB], Lr[NB], dloc;
  local_blocks<NS>(P, u, nH[idx], eh[idx], s, M, Uc, Lr, dloc);
#pragma unroll
  for (int i = 0; i < NB; ++i) {
#pragma unroll
    for (int j = 0; j < NB; ++j) Mo[(i * NB + j) * N + idx] = M[i][j];
    Uo[i * N + idx] = Uc[i];
    Lo[i * N + idx] = Lr[i];
  }
  Do[idx] = dloc;
}

// Gaussian elimination with partial pivoting on one small dense system with
// two right-hand sides, fully in registers.  Pivot: largest |a_ik|, first on
// ties (a row is moved up only if strictly larger).
template <int NB>
__device__ inline void gepp2(double (&A)[NB][NB], double (&B)[NB][2]) {
#pragma unroll
  for (int k = 0; k < NB; ++k) {
#pragma unroll
    for (int i = k + 1; i < NB; ++i) {
      if (fabs(A[i][k]) > fabs(A[k][k])) {
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const double t = A[k][j]; A[k][j] = A[i][j]; A[i][j] = t;
        }
        const double t0 = B[k][0]; B[k][0] = B[i][0]; B[i][0] = t0;
        const double t1 = B[k][1]; B[k][1] = B[i][1]; B[i][1] = t1;
      }
    }
    const double inv = 1.0 / A[k][k];
#pragma unroll
    for (int i = k + 1; i < NB; ++i) {
      const double l = A[i][k] * inv;
#pragma unroll
      for (int j = k + 1; j < NB; ++j) A[i][j] -= l * A[k][j];
      B[i][0] -= l * B[k][0];
      B[i][1] -= l * B[k][1];
    }
  }
#pragma unroll
  for (int i = NB - 1; i >= 0; --i) {
    double s0 = B[i][0], s1 = B[i][1];
#pragma unroll
    for (int j = i + 1; j < NB; ++j) {
      s0 -= A[i][j] * B[j][0];
      s1 -= A[i][j] * B[j][1];
    }
    B[i][0] = s0 / A[i][i];
    B[i][1] = s1 / A[i][i];
  }
}

// Schur step (i) per cell and the cell-local part of step (ii):
// f~_M, W = M^-1 [f_M, U] (GEPP); loc = 1 + dt theta dL_E/dE - L W;
// b = L f~_M - f_E; om = sum_s dkappa/dx_s W_s and ph = sum_s dkappa/dx_s f~_s
// (the species columns that the face opacities couple to the E rows)
template <int NS>
__global__ __launch_bounds__(BLOCK) void k_schur_local(DevParams P, const double* __restrict__ U,
                                                        const double* __restrict__ f,
                                                        const double* __restrict__ nH,
                                                        const double* __restrict__ eh, Step s,
                                                        double* __restrict__ ftM,
                                                        double* __restrict__ Wo,
                                                        double* __restrict__ loc,
                                                        double* __restrict__ b,
                                                        double* __restrict__ om,
                                                        double* __restrict__ ph) {
  constexpr int NB = NS + 1;
  const int N = P.N;
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= N) return;
  double u[NS + 2];
#pragma unroll
  for (int v = 0; v < NS + 2; ++v) u[v] = U[v * N + idx];
  const double nHv = nH[idx];
  double M[NB][NB], Uc[NB], Lr[NB], dloc;
  local_blocks<NS>(P, u, nHv, eh[idx], s, M, Uc, Lr, dloc);
  double B[NB][2];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    B[i][0] = f[i * N + idx];
    B[i][1] = Uc[i];
  }
  gepp2<NB>(M, B);
  double lw = 0.0, lf = 0.0;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    lw += Lr[i] * B[i][1];
    lf += Lr[i] * B[i][0];
    ftM[i * N + idx] = B[i][0];
    Wo[i * N + idx] = B[i][1];
  }
  loc[idx] = dloc - lw;
  b[idx] = lf - f[NB * N + idx];
  double dk[NS > 0 ? NS : 1];
  opacity_derivs<NS>(nHv, s.a, P, dk);
  double o = 0.0, p = 0.0;
#pragma unroll
  for (int sp = 0; sp < NS; ++sp) {
    o += dk[sp] * B[1 + sp][1];
    p += dk[sp] * B[1 + sp][0];
  }
  om[idx] = o;
  ph[idx] = p;
}

// Schur step (ii), the face terms: for every face (P, Q = P + e_d) with
// k = dt theta / (a^2 dx^2) and kk = k dF/dkappa_f / (2 u_E) (each cell's
// share of the face opacity),
//   fw = k dF/dE_Q - kk om_Q  (= -S_{P,Q}),  bw = -k dF/dE_P + kk om_P (= -S_{Q,P}),
//   diag_P += bw, diag_Q += fw, b_P -= kk (ph_P + ph_Q), b_Q += kk (ph_P + ph_Q),
// and for the preconditioner's operator c = k (D + T) >= 0 with
// pdiag = loc + the six c.  Each thread forms the + faces of its cell
// (stored) and the - faces (the same expressions as the neighbour's + face).
// The x-left Dirichlet face (bc 2) adds its Q terms to the first cell.
// loc and b arrive from k_schur_local; diag, pdiag, b leave complete.
// Dlag non-null (lagged limiter): the flux is D_f (E_Q - E_P) with the stored
// coefficients, so dF/dE_Q = -dF/dE_P = D + T = D_f and nothing depends on
// the opacity: S is symmetric and equals the preconditioner's operator.
__device__ inline FaceJac lagged_jac(double D) {
  FaceJac J;
  J.D = D; J.DT = D; J.dEP = -D; J.dEQ = D; J.dk = 0.0;
  return J;
}
template <int NS>
__global__ __launch_bounds__(BLOCK) void k_schur_faces(DevParams P, const double* __restrict__ U,
                                                        const double* __restrict__ nH,
                                                        const double* __restrict__ Dlag, Step s,
                                                        const double* __restrict__ loc,
                                                        const double* __restrict__ om,
                                                        const double* __restrict__ ph,
                                                        double* __restrict__ diag,
                                                        double* __restrict__ pdiag,
                                                        double* __restrict__ cf,
                                                        double* __restrict__ fw,
                                                        double* __restrict__ bw,
                                                        double* __restrict__ b,
                                                        float* __restrict__ pd32,
                                                        float* __restrict__ cx32,
                                                        float* __restrict__ cy32,
                                                        float* __restrict__ cz32) {
  const int N = P.N;
  const C3 c = coord3(P.ny, P.nz);
  if (!c.ok) return;
  const int idx = (c.i * P.ny + c.j) * P.nz + c.k;
  const Nb nb = nbrs(c.i, c.j, c.k, P.nx, P.ny, P.nz);
  const double a = s.a;
  const double kf = s.dt * P.theta / (a * a * P.dx * P.dx);
  const double kq = 0.5 * kf / P.u_E;
  const double* E = U + (NS + 1) * N;
  const double EP = E[idx];
  const double kP = opacity_of<NS>(U, nH, N, idx, a, P);
  const double omP = om[idx], phP = ph[idx];
  const int np_[3] = {nb.xp, nb.yp, nb.zp};
  const int nm_[3] = {nb.xm, nb.ym, nb.zm};
  const bool last[3] = {c.i == P.nx - 1, c.j == P.ny - 1, c.k == P.nz - 1};
  const bool first[3] = {c.i == 0, c.j == 0, c.k == 0};
  const double lc = loc[idx];
  double dg = lc, pd = lc, bb = b[idx];
  double cst[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (P.bc == 2 && d == 0 && first[0]) {
      // the ghost face: Q terms only, full opacity derivative
      const FaceJac J = Dlag ? lagged_jac(Dlag[nb.xm]) : face_jac(P.Eb, EP, kP, kP, a, P, false);
      dg += kf * J.dEQ - (2.0 * kq) * J.dk * omP;
      pd += kf * J.DT;
      bb += (2.0 * kq) * J.dk * phP;
    }
    double f_ = 0.0, b_ = 0.0, c_ = 0.0;
    if (!(P.bc != 0 && last[d])) {
      const int q = np_[d];
      const FaceJac J = Dlag ? lagged_jac(Dlag[d * N + idx])
                             : face_jac(EP, E[q], kP, opacity_of<NS>(U, nH, N, q, a, P), a, P);
      const double kk = kq * J.dk;
      f_ = kf * J.dEQ - kk * om[q];
      b_ = -kf * J.dEP + kk * omP;
      c_ = kf * J.DT;
      bb -= kk * (phP + ph[q]);
    }
    double fm = 0.0, cm = 0.0, flm = 0.0;
    if (!(P.bc != 0 && first[d])) {
      const int r = nm_[d];
      const FaceJac J = Dlag ? lagged_jac(Dlag[d * N + r])
                             : face_jac(E[r], EP, opacity_of<NS>(U, nH, N, r, a, P), kP, a, P);
      const double kk = kq * J.dk;
      fm = kf * J.dEQ - kk * omP;
      cm = kf * J.DT;
      flm = kk * (ph[r] + phP);
    }
    dg = (dg + b_) + fm;
    pd = (pd + c_) + cm;
    bb += flm;
    fw[d * N + idx] = f_;
    bw[d * N + idx] = b_;
    cf[d * N + idx] = c_;
    cst[d] = c_;
  }
  // the preconditioner's diagonal is raised to S's own where that is larger
  // (P stays diagonally dominant)
  if (dg > pd) pd = dg;
  diag[idx] = dg;
  pdiag[idx] = pd;
  b[idx] = bb;
  if (pd32) {
    // FP32 copy for the finest V-cycle level, colour-split: the cells of one
    // colour of a row first, k = 2m + ((k + i + j) & 1) at place
    // ((k + i + j) & 1) nz/2 + m
    const int sidx = (c.i * P.ny + c.j) * P.nz + ((c.k + c.i + c.j) & 1) * (P.nz >> 1) + (c.k >> 1);
    pd32[sidx] = (float)pd;
    cx32[sidx] = (float)cst[0];
    cy32[sidx] = (float)cst[1];
    cz32[sidx] = (float)cst[2];
  }
}

// ---------------------------------------------------------------------------
// reductions and CG scalars
// post = 1: then alpha = rho / (p.q) (out = sc + S_PQ); post = 2: then the
// flexible (Polak-Ribiere) beta = (z.r - z.r_old) / rho, with r - r_old =
// -alpha q, i.e. -alpha (z.q) / rho, and rho <- z.r (out = sc + S_ZR, two
// components)
__global__ __launch_bounds__(1024) void k_final_reduce(const double* __restrict__ parts,
                                                       int nparts, int ncomp,
                                                       double* out, double* sc, int post) {
  __shared__ double sh[1024 / 64][NCOMP_MAX];
  __shared__ double tot[NCOMP_MAX];
  for (int c = 0; c < ncomp; ++c) {
    // eight independent chains (fixed assignment and combine order), so the
    // loads of a thread are in flight together
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int i = threadIdx.x;
    for (; i + 7 * 1024 < nparts; i += 8 * 1024) {
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += parts[(i + u * 1024) * NCOMP_MAX + c];
    }
    for (int u = 0; i < nparts; i += 1024, ++u) a[u] += parts[i * NCOMP_MAX + c];
    double x = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][c] = x;
  }
  __syncthreads();
  if (threadIdx.x < ncomp) {
    double s = 0.0;
    for (int w = 0; w < 1024 / 64; ++w) s += sh[w][threadIdx.x];
    out[threadIdx.x] = s;
    tot[threadIdx.x] = s;
  }
  if (post != 0) {
    __syncthreads();
    if (threadIdx.x == 0) {
      if (post == 1) {
        sc[S_ALPHA] = sc[S_RHO] / tot[0];
      } else {
        sc[S_BETA] = (-sc[S_ALPHA] * tot[1]) / sc[S_RHO];
        sc[S_RHO] = tot[0];
      }
    }
  }
}


__global__ __launch_bounds__(BLOCK) void k_spmv_dot(int nx, int ny, int nz,
                                                     const double* __restrict__ diag,
                                                     const double* __restrict__ cx,
                                                     const double* __restrict__ cy,
                                                     const double* __restrict__ cz,
                                                     const double* __restrict__ p,
                                                     double* __restrict__ q,
                                                     double* __restrict__ parts) {
  double acc[1] = {0.0};
  const C3 c = coord3(ny, nz);
  if (c.ok) {
    const int idx = (c.i * ny + c.j) * nz + c.k;
    const Nb nb = nbrs(c.i, c.j, c.k, nx, ny, nz);
    const double pv = p[idx];
    double y = diag[idx] * pv;
    y = y - cx[idx] * p[nb.xp] - cx[nb.xm] * p[nb.xm];
    y = y - cy[idx] * p[nb.yp] - cy[nb.ym] * p[nb.ym];
    y = y - cz[idx] * p[nb.zp] - cz[nb.zm] * p[nb.zm];
    q[idx] = y;
    acc[0] += pv * y;
  }
  block_reduce<1>(acc, parts);
}

// r32 non-null: also the FP32 copy of the new r in the colour-split layout of
// the FP32 cycle's finest level (ny, nz its extents), so that the V-cycle
// that follows needs no conversion pass
__global__ __launch_bounds__(BLOCK) void k_update_xr(long n, double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ q,
                                                      const double* __restrict__ sc,
                                                      double* __restrict__ parts,
                                                      float* __restrict__ r32, int ny, int nz) {
  const double alpha = sc[S_ALPHA];
  double acc[1] = {0.0};
  for (long i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long)gridDim.x * BLOCK) {
    x[i] = x[i] + alpha * p[i];
    const double rv = r[i] - alpha * q[i];
    r[i] = rv;
    acc[0] += rv * rv;
    if (r32) {
      const long row = i / nz;
      const int k = (int)(i - row * nz);
      const int j = (int)(row % ny), ii = (int)(row / ny);
      r32[row * nz + ((k + ii + j) & 1) * (nz >> 1) + (k >> 1)] = (float)rv;
    }
  }
  block_reduce<1>(acc, parts);
}

__global__ __launch_bounds__(BLOCK) void k_dot2(long n, const double* __restrict__ z,
                                                 const double* __restrict__ r,
                                                 const double* __restrict__ q,
                                                 double* __restrict__ parts) {
  double acc[2] = {0.0, 0.0};
  for (long i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long)gridDim.x * BLOCK) {
    const double zv = z[i];
    acc[0] += zv * r[i];
    acc[1] += zv * q[i];
  }
  block_reduce<2>(acc, parts);
}

// partials of a.b; copy_b non-null: also copy_b = b (the copy rides on the read)
__global__ __launch_bounds__(BLOCK) void k_dot1(long n, const double* __restrict__ a,
                                                 const double* __restrict__ b,
                                                 double* __restrict__ parts,
                                                 double* __restrict__ copy_b) {
  double acc[1] = {0.0};
  for (long i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long)gridDim.x * BLOCK) {
    const double bv = b[i];
    acc[0] += a[i] * bv;
    if (copy_b) copy_b[i] = bv;
  }
  block_reduce<1>(acc, parts);
}

__global__ __launch_bounds__(BLOCK) void k_update_p(long n, double* __restrict__ p,
                                                     const double* __restrict__ z,
                                                     const double* __restrict__ sc) {
  const double beta = sc[S_BETA];
  const long i = blockIdx.x * (long)BLOCK + threadIdx.x;
  if (i < n) p[i] = z[i] + beta * p[i];
}

// ---------------------------------------------------------------------------
// flexible GMRES on the full (non-symmetric) Schur operator.  Reductions with
// up to KMAX components: grid-stride kernels with a fixed block count
// (reduce_blocks), partials laid out [component][block], one final-reduce
// workgroup per component (fixed order: deterministic).

// (i, j, k) of flat cell index n on an nx x ny x nz grid
__device__ inline void cell_ijk(long n, int ny, int nz, int& i, int& j, int& k) {
  const long row = n / nz;
  k = (int)(n - row * nz);
  i = (int)(row / ny);
  j = (int)(row - (long)i * ny);
}

// block partials of NC compile-time components (slot c of parts: c * nblk + block)
template <int NC>
__device__ inline void block_reduce_n(const double (&v)[NC], double* __restrict__ parts,
                                      int nblk) {
  __shared__ double sh[BLOCK / 64][NC];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double x = v[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) sh[w][c] = x;
  }
  __syncthreads();
  if (tid < NC) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < BLOCK / 64; ++i) t += sh[i][tid];
    parts[(size_t)tid * nblk + blockIdx.x] = t;
  }
}

// The vector kernels below take the number of basis vectors as a template
// argument: every load of a cell is then issued unconditionally, ahead of
// its use, instead of behind a run-time test per vector (which serialised
// the loads of a thread).  The grid-stride loops walk the cells of a fixed
// number of blocks (reduce_blocks), so the partial sums, and hence the
// results, do not depend on timing.

// Cells of this block in a grid-stride walk that keeps each XCD on one
// contiguous part of the grid.  The hardware places block b on XCD b mod 8;
// with a block count and N divisible by 8, XCD x walks cells
// [x N/8, (x+1) N/8) with its gridDim/8 blocks, so the neighbour rows and
// planes a stencil reads were fetched into the same XCD's L2 by its own
// blocks (with plain round-robin every row's y-neighbours sit on two other
// XCDs).  Otherwise the plain grid-stride walk.  Either way each block's cell
// set is fixed, so its partial sums do not depend on timing.
struct XcdRange {
  long first, end, stride;
};
__device__ inline XcdRange xcd_range(long N) {
  const int nb = gridDim.x;
  if ((nb & 7) == 0 && (N & 7) == 0) {
    const long chunk = N >> 3;
    const long base = (long)(blockIdx.x & 7) * chunk;
    return XcdRange{base + (long)(blockIdx.x >> 3) * BLOCK + threadIdx.x, base + chunk,
                    (long)(nb >> 3) * BLOCK};
  }
  return XcdRange{blockIdx.x * (long)BLOCK + threadIdx.x, N, (long)nb * BLOCK};
}

// a load of a value this launch reads once: marked non-temporal so that it
// does not push out of L2 the values that neighbouring cells read again
__device__ inline double ldnt(const double* p) { return __builtin_nontemporal_load(p); }

// w = S z (bsub null) or w = bsub - S z for the full 7-point operator
// (S x)_P = diag_P x_P - sum_d [fw_d[P] x_{P+d} + bw_d[P-d] x_{P-d}];
// zcopy non-null: also zcopy = z.  Partials of w.V_i (i < NV, V_i at
// V + i N) and of w.w (component NV).  The operator and the basis vectors
// are read once (non-temporal); z at seven points, and the XCD-contiguous
// walk keeps its neighbour rows and planes in the walking XCD's L2.
template <int NV>
__global__ __launch_bounds__(BLOCK) void k_spmv_full(int nx, int ny, int nz,
                                                      const double* __restrict__ diag,
                                                      const double* __restrict__ fw,
                                                      const double* __restrict__ bw,
                                                      const double* __restrict__ z,
                                                      const double* __restrict__ bsub,
                                                      double* __restrict__ w,
                                                      double* __restrict__ zcopy,
                                                      const double* __restrict__ V,
                                                      double* __restrict__ parts, int nblk) {
  const long N = (long)nx * ny * nz;
  double acc[NV + 1];
#pragma unroll
  for (int c = 0; c <= NV; ++c) acc[c] = 0.0;
  const XcdRange xr = xcd_range(N);
  for (long n = xr.first; n < xr.end; n += xr.stride) {
    int i, j, k;
    cell_ijk(n, ny, nz, i, j, k);
    const Nb nb = nbrs(i, j, k, nx, ny, nz);
    const int idx = (int)n;
    double vv[NV > 0 ? NV : 1];
#pragma unroll
    for (int c = 0; c < NV; ++c) vv[c] = ldnt(&V[(size_t)c * N + idx]);
    const double zv = z[idx];
    double y = ldnt(&diag[idx]) * zv;
    y = y - ldnt(&fw[idx]) * z[nb.xp] - ldnt(&bw[nb.xm]) * z[nb.xm];
    y = y - ldnt(&fw[N + idx]) * z[nb.yp] - ldnt(&bw[N + nb.ym]) * z[nb.ym];
    y = y - ldnt(&fw[2 * N + idx]) * z[nb.zp] - ldnt(&bw[2 * N + nb.zm]) * z[nb.zm];
    if (bsub) y = bsub[idx] - y;
    w[idx] = y;
    if (zcopy) zcopy[idx] = zv;
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[c] += y * vv[c];
    acc[NV] += y * y;
  }
  block_reduce_n<NV + 1>(acc, parts, nblk);
}

// Gram-Schmidt pass: w -= sum_{i < NV} coef[i] V_i (coef on the device);
// partials of w.V_i (DOTS) and of w.w (component NV, or 0 without DOTS)
template <int NV, bool DOTS>
__global__ __launch_bounds__(BLOCK) void k_gs_pass(long N, double* __restrict__ w,
                                                    const double* __restrict__ V,
                                                    const double* __restrict__ coef,
                                                    double* __restrict__ parts, int nblk) {
  __shared__ double cs[NV];
  if (threadIdx.x < NV) cs[threadIdx.x] = coef[threadIdx.x];
  __syncthreads();
  constexpr int NA = DOTS ? NV + 1 : 1;
  double acc[NA];
#pragma unroll
  for (int c = 0; c < NA; ++c) acc[c] = 0.0;
  for (long n = blockIdx.x * (long)BLOCK + threadIdx.x; n < N; n += (long)gridDim.x * BLOCK) {
    double vv[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) vv[c] = V[(size_t)c * N + n];
    double y = w[n];
#pragma unroll
    for (int c = 0; c < NV; ++c) y -= cs[c] * vv[c];
    w[n] = y;
    if constexpr (DOTS) {
#pragma unroll
      for (int c = 0; c < NV; ++c) acc[c] += y * vv[c];
    }
    acc[NA - 1] += y * y;
  }
  block_reduce_n<NA>(acc, parts, nblk);
}

// v *= s; copy non-null: copy = v (after scaling); r32 non-null: the FP32
// copy in the colour-split layout of the FP32 cycle's finest level
__global__ __launch_bounds__(BLOCK) void k_scale(long N, double* __restrict__ v, double sf,
                                                  double* __restrict__ copy,
                                                  float* __restrict__ r32, int ny, int nz) {
  for (long n = blockIdx.x * (long)BLOCK + threadIdx.x; n < N; n += (long)gridDim.x * BLOCK) {
    const double y = v[n] * sf;
    v[n] = y;
    if (copy) copy[n] = y;
    if (r32) {
      const long row = n / nz;
      const int k = (int)(n - row * nz);
      const int j = (int)(row % ny), ii = (int)(row / ny);
      r32[row * nz + ((k + ii + j) & 1) * (nz >> 1) + (k >> 1)] = (float)y;
    }
  }
}

// x += sum_{i < NV} y[i] Z_i (y on the device)
template <int NV>
__global__ __launch_bounds__(BLOCK) void k_combine(long N, double* __restrict__ x,
                                                    const double* __restrict__ Z,
                                                    const double* __restrict__ y) {
  __shared__ double ys[NV];
  if (threadIdx.x < NV) ys[threadIdx.x] = y[threadIdx.x];
  __syncthreads();
  for (long n = blockIdx.x * (long)BLOCK + threadIdx.x; n < N; n += (long)gridDim.x * BLOCK) {
    double zz[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) zz[c] = Z[(size_t)c * N + n];
    double t = x[n];
#pragma unroll
    for (int c = 0; c < NV; ++c) t += ys[c] * zz[c];
    x[n] = t;
  }
}

// out[c] = sum over the blocks of parts[c * nblk + block]; one workgroup per
// component, fixed order
__global__ __launch_bounds__(1024) void k_final_multi(const double* __restrict__ parts, int nblk,
                                                       double* __restrict__ out) {
  __shared__ double sh[1024 / 64];
  const int c = blockIdx.x;
  double a = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 1024) a += parts[(size_t)c * nblk + i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 1024 / 64; ++w) t += sh[w];
    out[c] = t;
  }
}

// ---------------------------------------------------------------------------
// multigrid
template <class T>
__global__ __launch_bounds__(BLOCK) void k_fill(long n, T* __restrict__ x, T v) {
  const long i = blockIdx.x * (long)BLOCK + threadIdx.x;
  if (i < n) x[i] = v;
}

__device__ inline int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Finest-level layout of the FP32 V-cycle.  Natural: cell (i,j,k) at
// (i*ny + j)*nz + k.  Colour-split (SF): each z-row holds its colour-0 cells,
// then its colour-1 cells, each half in k order, so cell (i,j,k) sits at
// (i*ny + j)*nz + ((i+j+k) & 1)*(nz/2) + k/2.  A half-sweep then touches dense
// half-rows only: the six neighbours of a cell have the other colour and sit
// at k/2 (the z neighbours at k/2 or the place next to it) of that colour's
// half of the same or an adjacent row.
template <bool SF>
__device__ inline int lidx(int i, int j, int k, int ny, int nz) {
  if constexpr (SF) return (i * ny + j) * nz + ((i + j + k) & 1) * (nz >> 1) + (k >> 1);
  else return (i * ny + j) * nz + k;
}
// k of the cell stored at place q of row (i, j): threads that walk a row in
// storage order touch consecutive addresses
template <bool SF>
__device__ inline int stored_k(int i, int j, int q, int nz) {
  if constexpr (SF) {
    const int hz = nz >> 1;
    const int c = q >= hz ? 1 : 0;
    return 2 * (q - c * hz) + ((c + i + j) & 1);
  } else {
    return q;
  }
}
struct Nb7 {
  int c, xm, xp, ym, yp, zm, zp;
};
template <bool SF>
__device__ inline Nb7 nbrs7(int i, int j, int k, int nx, int ny, int nz) {
  if constexpr (!SF) {
    const Nb n = nbrs(i, j, k, nx, ny, nz);
    return Nb7{(i * ny + j) * nz + k, n.xm, n.xp, n.ym, n.yp, n.zm, n.zp};
  } else {
    const int ip = i + 1 < nx ? i + 1 : 0, im = i > 0 ? i - 1 : nx - 1;
    const int jp = j + 1 < ny ? j + 1 : 0, jm = j > 0 ? j - 1 : ny - 1;
    const int kp = k + 1 < nz ? k + 1 : 0, km = k > 0 ? k - 1 : nz - 1;
    return Nb7{lidx<true>(i, j, k, ny, nz),  lidx<true>(im, j, k, ny, nz),
               lidx<true>(ip, j, k, ny, nz), lidx<true>(i, jm, k, ny, nz),
               lidx<true>(i, jp, k, ny, nz), lidx<true>(i, j, km, ny, nz),
               lidx<true>(i, j, kp, ny, nz)};
  }
}

// one colour of a red-black Gauss-Seidel sweep (colour = (i+j+k) mod 2);
// the launch's x extent is nz/2: thread kk owns the kk-th cell of the colour
// in its z-row (nz even)
template <class T, bool SF = false>
__device__ inline void rbgs_update(const Level<T>& L, int i, int j, int k) {
  const Nb7 nb = nbrs7<SF>(i, j, k, L.nx, L.ny, L.nz);
  const T* x = L.x;
  T s = L.b[nb.c];
  s = s + L.cx[nb.c] * x[nb.xp] + L.cx[nb.xm] * x[nb.xm];
  s = s + L.cy[nb.c] * x[nb.yp] + L.cy[nb.ym] * x[nb.ym];
  s = s + L.cz[nb.c] * x[nb.zp] + L.cz[nb.zm] * x[nb.zm];
  L.x[nb.c] = s / L.diag[nb.c];
}

template <class T, bool SF>
__global__ __launch_bounds__(BLOCK) void k_rbgs(Level<T> L, int colour) {
  const C3 c = coord3(L.ny, L.nz >> 1);
  if (!c.ok) return;
  const int k = 2 * c.k + ((c.i + c.j + colour) & 1);
  rbgs_update<T, SF>(L, c.i, c.j, k);
}

// the last half-sweep of a V-cycle with the result widened into a FP64
// vector (natural layout): the thread of cell k also copies its pair partner
// k ^ 1 (the other colour, final already), so out64 receives every cell and x
// is not stored.  With parts given, the block partials of out64.r64 and
// out64.q64 (the CG dots that follow the V-cycle) are formed on the way.
template <class T, bool SF>
__global__ __launch_bounds__(BLOCK) void k_rbgs_out64(Level<T> L, int colour,
                                                      double* __restrict__ out64,
                                                      const double* __restrict__ r64,
                                                      const double* __restrict__ q64,
                                                      double* __restrict__ parts) {
  double acc[2] = {0.0, 0.0};
  const C3 c = coord3(L.ny, L.nz >> 1);
  if (c.ok) {
    const int i = c.i, j = c.j;
    const int k = 2 * c.k + ((i + j + colour) & 1);
    const int row = (i * L.ny + j) * L.nz;
    const Nb7 nb = nbrs7<SF>(i, j, k, L.nx, L.ny, L.nz);
    const T* x = L.x;
    T s = L.b[nb.c];
    s = s + L.cx[nb.c] * x[nb.xp] + L.cx[nb.xm] * x[nb.xm];
    s = s + L.cy[nb.c] * x[nb.yp] + L.cy[nb.ym] * x[nb.ym];
    s = s + L.cz[nb.c] * x[nb.zp] + L.cz[nb.zm] * x[nb.zm];
    const double z0 = (double)(s / L.diag[nb.c]);
    const double z1 = (double)x[lidx<SF>(i, j, k ^ 1, L.ny, L.nz)];
    out64[row + k] = z0;
    out64[row + (k ^ 1)] = z1;
    if (parts) {
      acc[0] = z0 * r64[row + k] + z1 * r64[row + (k ^ 1)];
      acc[1] = z0 * q64[row + k] + z1 * q64[row + (k ^ 1)];
    }
  }
  if (parts) block_reduce<2>(acc, parts);
}

// the last half-sweep of a V-cycle with the two dots that follow it: x is
// updated in place, and the thread of cell k also reads its pair partner
// k ^ 1 (the other colour, final already) to form the block partials of x.r
// and x.q over both cells (r, q in the level's type, FP64 products and sums)
template <class T, bool SF>
__global__ __launch_bounds__(BLOCK) void k_rbgs_dots(Level<T> L, int colour,
                                                     const T* __restrict__ r,
                                                     const T* __restrict__ q,
                                                     double* __restrict__ parts) {
  double acc[2] = {0.0, 0.0};
  const C3 c = coord3(L.ny, L.nz >> 1);
  if (c.ok) {
    const int k = 2 * c.k + ((c.i + c.j + colour) & 1);
    const Nb7 nb = nbrs7<SF>(c.i, c.j, k, L.nx, L.ny, L.nz);
    const T* x = L.x;
    T s = L.b[nb.c];
    s = s + L.cx[nb.c] * x[nb.xp] + L.cx[nb.xm] * x[nb.xm];
    s = s + L.cy[nb.c] * x[nb.yp] + L.cy[nb.ym] * x[nb.ym];
    s = s + L.cz[nb.c] * x[nb.zp] + L.cz[nb.zm] * x[nb.zm];
    const T z0 = s / L.diag[nb.c];
    const int pc = lidx<SF>(c.i, c.j, k ^ 1, L.ny, L.nz);
    const T z1 = x[pc];
    L.x[nb.c] = z0;
    acc[0] = (double)z0 * (double)r[nb.c] + (double)z1 * (double)r[pc];
    acc[1] = (double)z0 * (double)q[nb.c] + (double)z1 * (double)q[pc];
  }
  block_reduce<2>(acc, parts);
}

// the first (red, black) pair from x = 0 in one pass: red cells take b/diag,
// black cells use their red neighbours' b/diag (the values the red half-sweep
// would have produced)
template <class T, bool SF>
__global__ __launch_bounds__(BLOCK) void k_rbgs_first_pair(Level<T> L, T* __restrict__ xo) {
  const C3 c = coord3(L.ny, L.nz);
  if (!c.ok) return;
  const int k = stored_k<SF>(c.i, c.j, c.k, L.nz);
  const T* b = L.b;
  const T* d = L.diag;
  if (((c.i + c.j + k) & 1) == 0) {
    const int idx = lidx<SF>(c.i, c.j, k, L.ny, L.nz);
    xo[idx] = b[idx] / d[idx];
    return;
  }
  const Nb7 nb = nbrs7<SF>(c.i, c.j, k, L.nx, L.ny, L.nz);
  T s = b[nb.c];
  s = s + L.cx[nb.c] * (b[nb.xp] / d[nb.xp]) + L.cx[nb.xm] * (b[nb.xm] / d[nb.xm]);
  s = s + L.cy[nb.c] * (b[nb.yp] / d[nb.yp]) + L.cy[nb.ym] * (b[nb.ym] / d[nb.ym]);
  s = s + L.cz[nb.c] * (b[nb.zp] / d[nb.zp]) + L.cz[nb.zm] * (b[nb.zm] / d[nb.zm]);
  xo[nb.c] = s / d[nb.c];
}

// coarsest-level solve in one workgroup: `sweeps` x (red, black) from x = 0,
// then `sweeps` x (black, red); the level is small enough to stay in L2
template <class T>
__global__ __launch_bounds__(1024) void k_coarse_solve(Level<T> L, int sweeps) {
  const int half = L.nz >> 1;
  const int n2 = L.nx * L.ny * half;
  const int N = 2 * n2;
  for (int idx = threadIdx.x; idx < N; idx += blockDim.x) L.x[idx] = T(0);
  __threadfence_block();
  __syncthreads();
  for (int s = 0; s < 2 * sweeps; ++s) {
    for (int h = 0; h < 2; ++h) {
      const int colour = (s < sweeps) ? h : 1 - h;
      for (int t = threadIdx.x; t < n2; t += blockDim.x) {
        const int row = t / half;
        const int j = row % L.ny;
        const int i = row / L.ny;
        const int k = 2 * (t - row * half) + ((i + j + colour) & 1);
        rbgs_update(L, i, j, k);
      }
      __threadfence_block();
      __syncthreads();
    }
  }
}

// coarsest-level solve in one workgroup with the level held on chip: each
// thread keeps the right side and the seven coefficients of its cells in
// registers and x lives in LDS, so the 4*sweeps half-sweeps touch no memory
constexpr int CS_THREADS = 1024, CS_CPT = 2;   // up to 2 * 1024 * 2 = 4096 cells
// One workgroup per independent x-block of the level (L.blocks of them; the
// couplings between blocks are zero, as between the boxes of the subdomain
// hierarchy): the block's coefficients sit in registers, its x in LDS.
template <class T>
__global__ __launch_bounds__(CS_THREADS) void k_coarse_solve_lds(Level<T> L, int sweeps) {
  __shared__ T xs[2 * CS_THREADS * CS_CPT];
  const int nx = L.nx / L.blocks, ny = L.ny, nz = L.nz;
  const int base = blockIdx.x * nx * ny * nz;   // first cell of this block
  const int half = nz >> 1;
  const int n2 = nx * ny * half;
  const int tid = threadIdx.x;
  T cb[2][CS_CPT], cd[2][CS_CPT], c6[2][CS_CPT][6];
  int nb6[2][CS_CPT][6], own[2][CS_CPT];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int m = 0; m < CS_CPT; ++m) {
      const int t = tid + m * CS_THREADS;
      own[c][m] = -1;
      if (t < n2) {
        const int row = t / half;
        const int j = row % ny;
        const int i = row / ny;
        const int k = 2 * (t - row * half) + ((i + j + c) & 1);
        const int idx = (i * ny + j) * nz + k;
        const Nb nb = nbrs(i, j, k, nx, ny, nz);
        own[c][m] = idx;
        cb[c][m] = L.b[base + idx];
        cd[c][m] = L.diag[base + idx];
        c6[c][m][0] = L.cx[base + idx];   nb6[c][m][0] = nb.xp;
        c6[c][m][1] = L.cx[base + nb.xm]; nb6[c][m][1] = nb.xm;
        c6[c][m][2] = L.cy[base + idx];   nb6[c][m][2] = nb.yp;
        c6[c][m][3] = L.cy[base + nb.ym]; nb6[c][m][3] = nb.ym;
        c6[c][m][4] = L.cz[base + idx];   nb6[c][m][4] = nb.zp;
        c6[c][m][5] = L.cz[base + nb.zm]; nb6[c][m][5] = nb.zm;
      }
    }
  }
  for (int t = tid; t < 2 * n2; t += CS_THREADS) xs[t] = T(0);
  __syncthreads();
  for (int s = 0; s < 2 * sweeps; ++s) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int colour = (s < sweeps) ? h : 1 - h;
#pragma unroll
      for (int m = 0; m < CS_CPT; ++m) {
        // both colours are unrolled so the arrays stay in registers
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          if (c == colour && own[c][m] >= 0) {
            T sum = cb[c][m];
            sum = sum + c6[c][m][0] * xs[nb6[c][m][0]] + c6[c][m][1] * xs[nb6[c][m][1]];
            sum = sum + c6[c][m][2] * xs[nb6[c][m][2]] + c6[c][m][3] * xs[nb6[c][m][3]];
            sum = sum + c6[c][m][4] * xs[nb6[c][m][4]] + c6[c][m][5] * xs[nb6[c][m][5]];
            xs[own[c][m]] = sum / cd[c][m];
          }
        }
      }
      __syncthreads();
    }
  }
  for (int t = tid; t < 2 * n2; t += CS_THREADS) L.x[base + t] = xs[t];
}

// r = b - A x.  red_only: after a smoothing that ended with the black
// half-sweep every black cell satisfies its equation (its residual is zero up
// to rounding), so only the red cells' residual is formed and stored; the
// black places of r are left as they are and k_restrict does not read them
template <class T, bool SF>
__global__ __launch_bounds__(BLOCK) void k_mg_residual(Level<T> L, int red_only) {
  const C3 c = coord3(L.ny, red_only ? L.nz >> 1 : L.nz);
  if (!c.ok) return;
  const int k = red_only ? 2 * c.k + ((c.i + c.j) & 1) : stored_k<SF>(c.i, c.j, c.k, L.nz);
  const Nb7 nb = nbrs7<SF>(c.i, c.j, k, L.nx, L.ny, L.nz);
  const int idx = nb.c;
  const T* x = L.x;
  T y = L.diag[idx] * x[idx];
  y = y - L.cx[idx] * x[nb.xp] - L.cx[nb.xm] * x[nb.xm];
  y = y - L.cy[idx] * x[nb.yp] - L.cy[nb.ym] * x[nb.ym];
  y = y - L.cz[idx] * x[nb.zp] - L.cz[nb.zm] * x[nb.zm];
  L.r[idx] = L.b[idx] - y;
}

// b_coarse = R r_fine with R = P^T / 8: weights (1,3,3,1)/8 per axis over
// fine cells 2I-1 .. 2I+2; red_only: the black cells' residual is zero (see
// k_mg_residual) and is not read: two of the four k per fine (i, j), picked
// without a branch so that all 32 loads issue together.
template <class T, bool SF>
__global__ __launch_bounds__(BLOCK) void k_restrict(Level<T> F, Level<T> C, int red_only) {
  const C3 c = coord3(C.ny, C.nz);
  if (!c.ok) return;
  const int I = c.i, J = c.j, K = c.k;
  const T w[4] = {T(0.125), T(0.375), T(0.375), T(0.125)};
  int kk[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) kk[q] = wrap(2 * K - 1 + q, F.nz);
  T acc = T(0);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = wrap(2 * I - 1 + a, F.nx);
    T acc_j = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = wrap(2 * J - 1 + b, F.ny);
      T acc_k = T(0);
      if (red_only) {
        // the red k of this (i, j) are kk[q0] and kk[q0 + 2]: kk[q] has the
        // parity of q + 1 (nz is even, so the wrap keeps it)
        const int q0 = (i + j + 1) & 1;
        const int ka = q0 ? kk[1] : kk[0], kb = q0 ? kk[3] : kk[2];
        const T wa = q0 ? w[1] : w[0], wb = q0 ? w[3] : w[2];
        acc_k = wa * F.r[lidx<SF>(i, j, ka, F.ny, F.nz)] + wb * F.r[lidx<SF>(i, j, kb, F.ny, F.nz)];
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc_k += w[q] * F.r[lidx<SF>(i, j, kk[q], F.ny, F.nz)];
      }
      acc_j += w[b] * acc_k;
    }
    acc += w[a] * acc_j;
  }
  C.b[(I * C.ny + J) * C.nz + K] = acc;
}

// x_fine += P x_coarse: cell-centred trilinear, weights 3/4 (parent) and 1/4
// (the parent's neighbour on the child's side) per axis.  With colour >= 0
// only the cells of that colour are corrected: a post-smoothing that begins
// with the other colour overwrites those cells without reading them.
template <class T, bool SF>
__global__ __launch_bounds__(BLOCK) void k_prolong_add(Level<T> C, Level<T> F, int colour) {
  const C3 c = coord3(F.ny, colour >= 0 ? F.nz >> 1 : F.nz);
  if (!c.ok) return;
  const int i = c.i, j = c.j;
  const int k = colour >= 0 ? 2 * c.k + ((i + j + colour) & 1) : stored_k<SF>(i, j, c.k, F.nz);
  const int idx = lidx<SF>(i, j, k, F.ny, F.nz);
  const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
  const int I1 = wrap(I0 + ((i & 1) ? 1 : -1), C.nx);
  const int J1 = wrap(J0 + ((j & 1) ? 1 : -1), C.ny);
  const int K1 = wrap(K0 + ((k & 1) ? 1 : -1), C.nz);
  const T* x = C.x;
  auto at = [&](int a, int b, int cc) { return x[(a * C.ny + b) * C.nz + cc]; };
  const T w0 = T(0.75), w1 = T(0.25);
  const T zI0 = w0 * (w0 * at(I0, J0, K0) + w1 * at(I0, J0, K1)) +
                w1 * (w0 * at(I0, J1, K0) + w1 * at(I0, J1, K1));
  const T zI1 = w0 * (w0 * at(I1, J0, K0) + w1 * at(I1, J0, K1)) +
                w1 * (w0 * at(I1, J1, K0) + w1 * at(I1, J1, K1));
  F.x[idx] = F.x[idx] + (w0 * zI0 + w1 * zI1);
}

// coarse operator: mean local part over the 8 children; face couplings from
// the series (harmonic) coupling along the normal, mean over the 2x2 fine
// columns, times 1/4; diag = local + sum
template <class T, bool SF>
__global__ __launch_bounds__(BLOCK) void k_coarsen(Level<T> F, Level<T> C) {
  const C3 c = coord3(C.ny, C.nz);
  if (!c.ok) return;
  const int I = c.i, J = c.j, K = c.k;
  const int idx = (I * C.ny + J) * C.nz + K;
  auto fi = [&](int i, int j, int k) {
    return lidx<SF>(wrap(i, F.nx), wrap(j, F.ny), wrap(k, F.nz), F.ny, F.nz);
  };
  T local = T(0);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int cc = 0; cc < 2; ++cc) {
        const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + cc;
        const int p = fi(i, j, k);
        const T cs = ((F.cx[p] + F.cx[fi(i - 1, j, k)]) + (F.cy[p] + F.cy[fi(i, j - 1, k)])) +
                     (F.cz[p] + F.cz[fi(i, j, k - 1)]);
        local += F.diag[p] - cs;
      }
  local *= T(0.125);
  // couplings on the + faces of coarse cell (I,J,K) and of its - neighbours:
  // per fine column crossing the coarse face, the series coupling of fine
  // faces 2I0, 2I0+1, 2I0+2 along d (weights 1/4, 1/2, 1/4), then the mean
  // over the 2x2 columns, times 1/4
  auto face = [&](const T* cf, int d, int i0, int j0, int k0) {
    T sum = T(0);
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) {
        T inv = T(0);
        bool zero = false;
        for (int m = 0; m < 3; ++m) {
          int i = 2 * i0, j = 2 * j0, k = 2 * k0;
          if (d == 0) { i += m; j += u; k += v; }
          if (d == 1) { j += m; i += u; k += v; }
          if (d == 2) { k += m; i += u; j += v; }
          const T cv = cf[fi(i, j, k)];
          if (!(cv > T(0))) zero = true;
          else inv += (m == 1 ? T(0.5) : T(0.25)) / cv;
        }
        sum += zero ? T(0) : T(1) / inv;
      }
    return T(0.0625) * sum;
  };
  const T cxp = face(F.cx, 0, I, J, K), cxm = face(F.cx, 0, I - 1, J, K);
  const T cyp = face(F.cy, 1, I, J, K), cym = face(F.cy, 1, I, J - 1, K);
  const T czp = face(F.cz, 2, I, J, K), czm = face(F.cz, 2, I, J, K - 1);
  C.cx[idx] = cxp;
  C.cy[idx] = cyp;
  C.cz[idx] = czp;
  C.diag[idx] = local + (((cxp + cxm) + (cyp + cym)) + (czp + czm));
}

// ---------------------------------------------------------------------------
// source subdomains: a box of B^3 cells centred on each source, the boxes
// stacked along x into one (nbox*B) x B x B periodic grid.  Box cell
// (X, j, k), X = s*B + bi, is global cell (c_s + (bi, j, k) - B/2) mod n.
struct BoxMap {
  int nx, ny, nz, B, nbox;
};
__device__ inline int box_global(const BoxMap& m, long long c, int bi, int bj, int bk) {
  const int ny = m.ny, nz = m.nz;
  const int ci = (int)(c / ((long long)ny * nz));
  const int cj = (int)((c / nz) % ny);
  const int ck = (int)(c % nz);
  const int h = m.B >> 1;
  int i = (ci - h + bi) % m.nx, j = (cj - h + bj) % ny, k = (ck - h + bk) % nz;
  if (i < 0) i += m.nx;
  if (j < 0) j += ny;
  if (k < 0) k += nz;
  return (i * ny + j) * nz + k;
}
// the operator restricted to the boxes: diagonal unchanged, couplings inside
// a box kept, couplings out of a box (its last layer in each direction, which
// the periodic storage would join to the next box) zero
__global__ __launch_bounds__(BLOCK) void k_box_extract(BoxMap m, const long long* __restrict__ cells,
                                                        const double* __restrict__ diag,
                                                        const double* __restrict__ cx,
                                                        const double* __restrict__ cy,
                                                        const double* __restrict__ cz,
                                                        double* __restrict__ bd, double* __restrict__ bx,
                                                        double* __restrict__ by, double* __restrict__ bz) {
  const C3 c = coord3(m.B, m.B);
  if (!c.ok) return;
  const int s = c.i / m.B, bi = c.i - s * m.B;
  const int g = box_global(m, cells[s], bi, c.j, c.k);
  const int o = (c.i * m.B + c.j) * m.B + c.k;
  bd[o] = diag[g];
  bx[o] = bi == m.B - 1 ? 0.0 : cx[g];
  by[o] = c.j == m.B - 1 ? 0.0 : cy[g];
  bz[o] = c.k == m.B - 1 ? 0.0 : cz[g];
}
// the residual r - S z left by the V-cycle, on the box cells (S the global
// operator, z the V-cycle's result), rounded to the box solve's type
template <class T>
__global__ __launch_bounds__(BLOCK) void k_box_residual(BoxMap m, const long long* __restrict__ cells,
                                                         const double* __restrict__ diag,
                                                         const double* __restrict__ cx,
                                                         const double* __restrict__ cy,
                                                         const double* __restrict__ cz,
                                                         const double* __restrict__ r,
                                                         const double* __restrict__ z,
                                                         T* __restrict__ bv) {
  const C3 c = coord3(m.B, m.B);
  if (!c.ok) return;
  const int s = c.i / m.B;
  const int g = box_global(m, cells[s], c.i - s * m.B, c.j, c.k);
  const int k = g % m.nz, j = (g / m.nz) % m.ny, i = g / (m.nz * m.ny);
  const Nb nb = nbrs(i, j, k, m.nx, m.ny, m.nz);
  double y = diag[g] * z[g];
  y = y - cx[g] * z[nb.xp] - cx[nb.xm] * z[nb.xm];
  y = y - cy[g] * z[nb.yp] - cy[nb.ym] * z[nb.ym];
  y = y - cz[g] * z[nb.zp] - cz[nb.zm] * z[nb.zm];
  bv[(c.i * m.B + c.j) * m.B + c.k] = (T)(r[g] - y);
}
// z += the box's part of y, one box per launch (overlapping boxes add in box
// order); with parts, also the block partials of y.r and y.q over the box,
// which complete the V-cycle's own partials of z.r and z.q
template <class T>
__global__ __launch_bounds__(BLOCK) void k_box_scatter_add(BoxMap m, const long long* __restrict__ cells,
                                                            int s, const T* __restrict__ y,
                                                            double* __restrict__ z,
                                                            const double* __restrict__ r,
                                                            const double* __restrict__ q,
                                                            double* __restrict__ parts) {
  const C3 c = coord3(m.B, m.B);
  double acc[2] = {0.0, 0.0};
  if (c.ok) {
    const int g = box_global(m, cells[s], c.i, c.j, c.k);
    const double yv = (double)y[((s * m.B + c.i) * m.B + c.j) * m.B + c.k];
    z[g] += yv;
    if (parts) {
      acc[0] = yv * r[g];
      acc[1] = yv * q[g];
    }
  }
  if (parts) block_reduce<2>(acc, parts);
}

// one red-black Gauss-Seidel half-sweep of colour `colour` on S z = r over
// the cells of box s, with the full Schur operator (diag, fw, bw; FP64, the
// main grid): z_P = (r_P + sum_d [fw_d[P] z_{P+d} + bw_d[P-d] z_{P-d}]) / diag_P
// for the box's cells of that colour (colour = (i + j + k) & 1 on the grid)
__global__ __launch_bounds__(BLOCK) void k_box_smooth_s(BoxMap m, const long long* __restrict__ cells,
                                                         int s, int colour,
                                                         const double* __restrict__ diag,
                                                         const double* __restrict__ fw,
                                                         const double* __restrict__ bw,
                                                         const double* __restrict__ r,
                                                         double* __restrict__ z) {
  const C3 c = coord3(m.B, m.B);
  if (!c.ok) return;
  const int g = box_global(m, cells[s], c.i, c.j, c.k);
  const int nyz = m.ny * m.nz;
  const int gi = g / nyz, gj = (g - gi * nyz) / m.nz, gk = g - gi * nyz - gj * m.nz;
  if (((gi + gj + gk) & 1) != colour) return;
  const Nb nb = nbrs(gi, gj, gk, m.nx, m.ny, m.nz);
  const long N = (long)m.nx * nyz;
  double t = r[g];
  t = t + fw[g] * z[nb.xp] + bw[nb.xm] * z[nb.xm];
  t = t + fw[N + g] * z[nb.yp] + bw[N + nb.ym] * z[nb.ym];
  t = t + fw[2 * N + g] * z[nb.zp] + bw[2 * N + nb.zm] * z[nb.zm];
  z[g] = t / diag[g];
}

// all `sweeps` (red, black) sweeps of k_box_smooth_s over box s in one
// workgroup, for B <= BOX_S_LDS_MAX and B below the grid size in every
// direction: the box's z and its one-cell halo sit in LDS, each owned cell's
// r, diagonal and six couplings in registers, so the 2 * sweeps half-sweeps
// touch no memory.  The halo is not updated, as in the per-half-sweep form:
// with B < n no halo cell is also a box cell.  Same arithmetic per cell.
// Threads own cells by colour: place p of a colour's list is the m-th cell of
// that colour in z-line (bi, bj) (p = line * B/2 + m; B is even, so every line
// holds B/2 cells of each colour), so a half-sweep keeps every lane busy.
constexpr int BS_THREADS = 1024;
constexpr int BS_CPC = (BOX_S_LDS_MAX * BOX_S_LDS_MAX * BOX_S_LDS_MAX / 2 + BS_THREADS - 1) /
                       BS_THREADS;   // cells per thread and colour
__global__ __launch_bounds__(BS_THREADS) void k_box_smooth_s_lds(BoxMap m,
                                                                  const long long* __restrict__ cells,
                                                                  int s, int sweeps,
                                                                  const double* __restrict__ diag,
                                                                  const double* __restrict__ fw,
                                                                  const double* __restrict__ bw,
                                                                  const double* __restrict__ r,
                                                                  double* __restrict__ z) {
  constexpr int E = BOX_S_LDS_MAX + 2;
  __shared__ double zs[E * E * E];
  const int B = m.B, H = B + 2, H2 = H * H, hb = B >> 1, nhalf = B * B * hb;
  const int nyz = m.ny * m.nz;
  const long N = (long)m.nx * nyz;
  const long long c0 = cells[s];
  const int tid = threadIdx.x;
  for (int t = tid; t < H2 * H; t += BS_THREADS) {
    const int hi = t / H2, hj = (t / H) % H, hk = t % H;
    zs[t] = z[box_global(m, c0, hi - 1, hj - 1, hk - 1)];
  }
  // colour of box cell (0, 0, 0); box cell (bi, bj, bk) has colour
  // (p0 + bi + bj + bk) & 1 (the grid sizes are even)
  const int g0 = box_global(m, c0, 0, 0, 0);
  const int p0 = (g0 / nyz + (g0 % nyz) / m.nz + g0 % m.nz) & 1;
  double cr[2][BS_CPC], cd[2][BS_CPC], c6[2][BS_CPC][6];
  int own[2][BS_CPC], gl[2][BS_CPC];
#pragma unroll
  for (int colour = 0; colour < 2; ++colour) {
#pragma unroll
    for (int q = 0; q < BS_CPC; ++q) {
      const int p = tid + q * BS_THREADS;
      own[colour][q] = -1;
      gl[colour][q] = 0;
      if (p < nhalf) {
        const int line = p / hb, mm = p - line * hb;
        const int bi = line / B, bj = line - bi * B;
        const int bk = 2 * mm + ((colour + p0 + bi + bj) & 1);
        const int g = box_global(m, c0, bi, bj, bk);
        const int gi = g / nyz, gj = (g - gi * nyz) / m.nz, gk = g - gi * nyz - gj * m.nz;
        const Nb nb = nbrs(gi, gj, gk, m.nx, m.ny, m.nz);
        own[colour][q] = ((bi + 1) * H + (bj + 1)) * H + (bk + 1);
        gl[colour][q] = g;
        cr[colour][q] = r[g];
        cd[colour][q] = diag[g];
        c6[colour][q][0] = fw[g];
        c6[colour][q][1] = bw[nb.xm];
        c6[colour][q][2] = fw[N + g];
        c6[colour][q][3] = bw[N + nb.ym];
        c6[colour][q][4] = fw[2 * N + g];
        c6[colour][q][5] = bw[2 * N + nb.zm];
      }
    }
  }
  __syncthreads();
  for (int k = 0; k < sweeps; ++k) {
#pragma unroll
    for (int colour = 0; colour < 2; ++colour) {
#pragma unroll
      for (int q = 0; q < BS_CPC; ++q) {
        const int o = own[colour][q];
        if (o >= 0) {
          double t = cr[colour][q];
          t = t + c6[colour][q][0] * zs[o + H2] + c6[colour][q][1] * zs[o - H2];
          t = t + c6[colour][q][2] * zs[o + H] + c6[colour][q][3] * zs[o - H];
          t = t + c6[colour][q][4] * zs[o + 1] + c6[colour][q][5] * zs[o - 1];
          zs[o] = t / cd[colour][q];
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int colour = 0; colour < 2; ++colour)
#pragma unroll
    for (int q = 0; q < BS_CPC; ++q)
      if (own[colour][q] >= 0) z[gl[colour][q]] = zs[own[colour][q]];
}

// ---- inner PCG of the subdomain correction, T the box V-cycle's type (the
// vectors are kept in it; dot products accumulate in FP64 and leave block
// partials, which the kernel that needs a CG scalar sums itself).
// rho = r.z, p = z
template <class T>
__global__ __launch_bounds__(BLOCK) void k_box_dot1p(long n, const T* __restrict__ r,
                                                      const T* __restrict__ z, T* __restrict__ p,
                                                      double* __restrict__ parts) {
  double acc[1] = {0.0};
  const long i = blockIdx.x * (long)BLOCK + threadIdx.x;
  if (i < n) {
    const T zv = z[i];
    p[i] = zv;
    acc[0] = (double)r[i] * (double)zv;
  }
  block_reduce<1>(acc, parts);
}
// sum over np block partials of component c in a fixed order, so that every
// block of a launch obtains the same value; returned to all threads (every
// thread of the block must call it)
__device__ inline double block_sum_parts(const double* __restrict__ parts, int np, int c) {
  __shared__ double sh[BLOCK / 64];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int nthr = blockDim.x * blockDim.y;
  double s = 0.0;
  for (int i = tid; i < np; i += nthr) s += parts[(size_t)i * NCOMP_MAX + c];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((tid & 63) == 0) sh[tid >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (nthr + 63) >> 6; ++w) t += sh[w];
  __syncthreads();
  return t;
}
// new direction and product in one pass (stacked boxes): beta = -alpha (z.q)
// / rho from the previous iteration's partials of z.r and z.q (rho <- z.r
// into the other slot, by one thread), p' = z + beta p formed at the cell and
// its six neighbours (p' goes to its own buffer: the old p is still read by
// other blocks), q = S p', and the partials of p'.q.  first: p' = z.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_box_spmv_p(int nx, int ny, int nz,
                                                       const T* __restrict__ diag,
                                                       const T* __restrict__ cx,
                                                       const T* __restrict__ cy,
                                                       const T* __restrict__ cz,
                                                       const T* __restrict__ z,
                                                       const T* __restrict__ pin,
                                                       T* __restrict__ pout, T* __restrict__ q,
                                                       const double* __restrict__ zparts, int nz_parts,
                                                       double* sc, int rho_in, int rho_out,
                                                       int first, double* __restrict__ parts) {
  double beta = 0.0;
  if (!first) {
    const double zr = block_sum_parts(zparts, nz_parts, 0);
    const double zq = block_sum_parts(zparts, nz_parts, 1);
    // a fixed number of iterations runs whatever the convergence: once the
    // box residual has vanished (rho = 0) the direction is z itself
    const double rho_prev = sc[rho_in];
    beta = rho_prev != 0.0 ? (-sc[S_ALPHA] * zq) / rho_prev : 0.0;
    if (block_linear() == 0 && threadIdx.x == 0 && threadIdx.y == 0) sc[rho_out] = zr;
  }
  auto pn = [&](int i) -> T { return first ? z[i] : (T)(z[i] + beta * pin[i]); };
  double acc[1] = {0.0};
  const C3 c = coord3(ny, nz);
  if (c.ok) {
    const int idx = (c.i * ny + c.j) * nz + c.k;
    const Nb nb = nbrs(c.i, c.j, c.k, nx, ny, nz);
    const T pv = pn(idx);
    T y = diag[idx] * pv;
    y = y - cx[idx] * pn(nb.xp) - cx[nb.xm] * pn(nb.xm);
    y = y - cy[idx] * pn(nb.yp) - cy[nb.ym] * pn(nb.ym);
    y = y - cz[idx] * pn(nb.zp) - cz[nb.zm] * pn(nb.zm);
    pout[idx] = pv;
    q[idx] = y;
    acc[0] = (double)pv * (double)y;
  }
  block_reduce<1>(acc, parts);
}
// alpha = rho / (p.q) from the product's partials (stored by one thread),
// x += alpha p, r -= alpha q
template <class T>
__global__ __launch_bounds__(BLOCK) void k_box_update_xr(long n, T* __restrict__ x, T* __restrict__ r,
                                                          const T* __restrict__ p,
                                                          const T* __restrict__ q,
                                                          const double* __restrict__ pqparts,
                                                          int npq, double* sc, int rho) {
  // p.q > 0 for any p != 0 (S is positive definite); p = 0 once the box
  // residual has vanished, and then x and r stay as they are
  const double pq = block_sum_parts(pqparts, npq, 0);
  const double alpha = pq > 0.0 ? sc[rho] / pq : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[S_ALPHA] = alpha;
  const long i = blockIdx.x * (long)BLOCK + threadIdx.x;
  if (i >= n) return;
  x[i] = (T)(x[i] + alpha * p[i]);
  r[i] = (T)(r[i] - alpha * q[i]);
}
// the box V-cycle's first (red, black) pair from z = 0 fused with the CG
// update before it: alpha as in k_box_update_xr, x += alpha p and
// rn = ro - alpha q at the thread's cell (rn in its own buffer: other blocks
// still read ro), then the pair with right side rn, whose values at the six
// neighbours the black cells form themselves from ro and q (natural layout)
template <class T>
__global__ __launch_bounds__(BLOCK) void k_box_update_first_pair(Level<T> L, T* __restrict__ x,
                                                                  const T* __restrict__ ro,
                                                                  T* __restrict__ rn,
                                                                  const T* __restrict__ p,
                                                                  const T* __restrict__ q,
                                                                  const double* __restrict__ pqparts,
                                                                  int npq, double* sc, int rho) {
  const double pq = block_sum_parts(pqparts, npq, 0);
  const double alpha = pq > 0.0 ? sc[rho] / pq : 0.0;
  if (block_linear() == 0 && threadIdx.x == 0 && threadIdx.y == 0) sc[S_ALPHA] = alpha;
  const C3 c = coord3(L.ny, L.nz);
  if (!c.ok) return;
  const int idx = (c.i * L.ny + c.j) * L.nz + c.k;
  auto rnew = [&](int i) -> T { return (T)(ro[i] - alpha * q[i]); };
  x[idx] = (T)(x[idx] + alpha * p[idx]);
  const T bc = rnew(idx);
  rn[idx] = bc;
  const T* d = L.diag;
  if (((c.i + c.j + c.k) & 1) == 0) {
    L.x[idx] = bc / d[idx];
    return;
  }
  const Nb nb = nbrs(c.i, c.j, c.k, L.nx, L.ny, L.nz);
  T s = bc;
  s = s + L.cx[idx] * (rnew(nb.xp) / d[nb.xp]) + L.cx[nb.xm] * (rnew(nb.xm) / d[nb.xm]);
  s = s + L.cy[idx] * (rnew(nb.yp) / d[nb.yp]) + L.cy[nb.ym] * (rnew(nb.ym) / d[nb.ym]);
  s = s + L.cz[idx] * (rnew(nb.zp) / d[nb.zp]) + L.cz[nb.zm] * (rnew(nb.zm) / d[nb.zm]);
  L.x[idx] = s / d[idx];
}
// the partials of z.r and z.q
template <class T>
__global__ __launch_bounds__(BLOCK) void k_box_dot2(long n, const T* __restrict__ z,
                                                     const T* __restrict__ r, const T* __restrict__ q,
                                                     double* __restrict__ parts) {
  double acc[2] = {0.0, 0.0};
  const long i = blockIdx.x * (long)BLOCK + threadIdx.x;
  if (i < n) {
    const double zv = z[i];
    acc[0] = zv * (double)r[i];
    acc[1] = zv * (double)q[i];
  }
  block_reduce<2>(acc, parts);
}

// FP64 natural -> colour-split finest level (FP32, or FP64 for the FP64 cycle)
template <class TO>
__global__ __launch_bounds__(BLOCK) void k_cvt_d2f_split(int nx, int ny, int nz,
                                                          const double* __restrict__ a,
                                                          TO* __restrict__ b) {
  const C3 c = coord3(ny, nz);
  if (!c.ok) return;
  const int k = stored_k<true>(c.i, c.j, c.k, nz);
  b[(c.i * ny + c.j) * nz + c.k] = (TO)a[(c.i * ny + c.j) * nz + k];
}

__global__ __launch_bounds__(BLOCK) void k_cvt_d2f(long n, const double* __restrict__ a,
                                                    float* __restrict__ b) {
  const long i = blockIdx.x * (long)BLOCK + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
__global__ __launch_bounds__(BLOCK) void k_cvt_f2d(long n, const float* __restrict__ a,
                                                    double* __restrict__ b) {
  const long i = blockIdx.x * (long)BLOCK + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

__global__ __launch_bounds__(BLOCK) void k_fold_energy(int N, double* __restrict__ U,
                                                        double* __restrict__ eh) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i < N) {
    eh[i] = eh[i] + U[i];
    U[i] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// launchers
static inline dim3 grid_for(long n) { return dim3((unsigned)((n + BLOCK - 1) / BLOCK)); }

// 3-D launch over (nx, ny, ext): x along z, y along y, z over x-planes
struct Geo {
  dim3 g, b;
};
static inline Geo geo3(int nx, int ny, int ext) {
  const int bx = ext < BLOCK ? ext : BLOCK;
  int by = BLOCK / bx;
  if (by > ny) by = ny;
  return Geo{dim3((unsigned)((ext + bx - 1) / bx), (unsigned)((ny + by - 1) / by), (unsigned)nx),
             dim3((unsigned)bx, (unsigned)by, 1)};
}
int stencil_blocks(int nx, int ny, int nz) {
  const Geo q = geo3(nx, ny, nz);
  return (int)(q.g.x * q.g.y * q.g.z);
}

// launches KERN<NS> for the grid's species count (0: LTE, 1: H, 3: H + He)
#define RT_NS(P, KERN, ...)                                            \
  do {                                                                  \
    if ((P).ns == 0) hipLaunchKernelGGL((KERN<0>), __VA_ARGS__);        \
    else if ((P).ns == 1) hipLaunchKernelGGL((KERN<1>), __VA_ARGS__);   \
    else hipLaunchKernelGGL((KERN<3>), __VA_ARGS__);                    \
  } while (0)
void launch_faces(const DevParams& P, const double* Un, const double* nH, double a, double* D,
                  hipStream_t st) {
  const Geo q = geo3(P.nx, P.ny, P.nz);
  RT_NS(P, k_faces, q.g, q.b, 0, st, P, Un, nH, a, D);
}

void launch_explicit(const DevParams& P, const double* Un, const double* nH, const double* eh,
                     const double* D, Step s, double* g, hipStream_t st) {
  const Geo q = geo3(P.nx, P.ny, P.nz);
  RT_NS(P, k_explicit, q.g, q.b, 0, st, P, Un, nH, eh, D, s, g);
}

void launch_sources(const long long* cells, const double* Q, int n, double scale, double* gE,
                    hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_sources, dim3(1), dim3(64), 0, st, cells, Q, n, scale, gE);
}

void launch_residual(const DevParams& P, const double* U, const double* g, const double* nH,
                     const double* eh, const double* Dlag, Step s, double* f, double* parts,
                     hipStream_t st) {
  const Geo q = geo3(P.nx, P.ny, P.nz);
  RT_NS(P, k_residual, q.g, q.b, 0, st, P, U, g, nH, eh, Dlag, s, f, parts);
}

void launch_predict_project(const DevParams& P, const double* Un, const double* eh, double* Up,
                            hipStream_t st) {
  RT_NS(P, k_predict_project, grid_for(P.N), dim3(BLOCK), 0, st, P, Un, eh, Up);
}
int launch_time_error(const DevParams& P, const double* A, const double* B, double p,
                      double* parts, hipStream_t st) {
  const int nb = reduce_blocks(P.N);
  RT_NS(P, k_time_error, dim3(nb), dim3(BLOCK), 0, st, P, A, B, p, parts);
  return nb;
}
void launch_final_summax(const double* parts, int nparts, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_final_summax, dim3(1), dim3(1024), 0, st, parts, nparts, out);
}
void launch_trial(const DevParams& P, const double* U, const double* ftM, const double* W,
                  const double* sE, double lambda, double* Ut, hipStream_t st) {
  RT_NS(P, k_trial, grid_for(P.N), dim3(BLOCK), 0, st, P, U, ftM, W, sE, lambda, Ut);
}

void launch_local_jac(const DevParams& P, const double* U, const double* nH, const double* eh,
                      Step s, double* M, double* Ucol, double* Lrow, double* dloc,
                      hipStream_t st) {
  RT_NS(P, k_local_jac, grid_for(P.N), dim3(BLOCK), 0, st, P, U, nH, eh, s, M, Ucol, Lrow, dloc);
}

void launch_final_reduce(const double* parts, int nparts, int ncomp, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_final_reduce, dim3(1), dim3(1024), 0, st, parts, nparts, ncomp, out,
                     (double*)nullptr, 0);
}
void launch_final_reduce_alpha(const double* parts, int nparts, double* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_final_reduce, dim3(1), dim3(1024), 0, st, parts, nparts, 1, sc + S_PQ,
                     sc, 1);
}
void launch_final_reduce_beta(const double* parts, int nparts, double* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_final_reduce, dim3(1), dim3(1024), 0, st, parts, nparts, 2, sc + S_ZR,
                     sc, 2);
}

void launch_spmv_dot(int nx, int ny, int nz, const double* diag, const double* cx,
                     const double* cy, const double* cz, const double* p, double* q,
                     double* parts, hipStream_t st) {
  const Geo g = geo3(nx, ny, nz);
  hipLaunchKernelGGL(k_spmv_dot, g.g, g.b, 0, st, nx, ny, nz, diag, cx, cy, cz, p, q, parts);
}
void launch_update_xr(long n, double* x, double* r, const double* p, const double* q,
                      const double* sc, double* parts, hipStream_t st, float* r32, int ny,
                      int nz) {
  hipLaunchKernelGGL(k_update_xr, dim3(reduce_blocks(n)), dim3(BLOCK), 0, st, n, x, r, p, q, sc,
                     parts, r32, ny, nz);
}
void launch_dot2(long n, const double* z, const double* r, const double* q, double* parts,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_dot2, dim3(reduce_blocks(n)), dim3(BLOCK), 0, st, n, z, r, q, parts);
}
void launch_dot1(long n, const double* a, const double* b, double* parts, hipStream_t st,
                 double* copy_b) {
  hipLaunchKernelGGL(k_dot1, dim3(reduce_blocks(n)), dim3(BLOCK), 0, st, n, a, b, parts, copy_b);
}
void launch_update_p(long n, double* p, const double* z, const double* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_update_p, grid_for(n), dim3(BLOCK), 0, st, n, p, z, sc);
}

void launch_schur_local(const DevParams& P, const double* U, const double* f, const double* nH,
                        const double* eh, Step s, double* ftM, double* W, double* loc, double* b,
                        double* om, double* ph, hipStream_t st) {
  RT_NS(P, k_schur_local, grid_for(P.N), dim3(BLOCK), 0, st, P, U, f, nH, eh, s, ftM, W, loc, b,
        om, ph);
}
void launch_schur_faces(const DevParams& P, const double* U, const double* nH, const double* Dlag,
                        Step s, const double* loc, const double* om, const double* ph,
                        double* diag, double* pdiag, double* c, double* fw, double* bw, double* b,
                        float* pd32, float* cx32, float* cy32, float* cz32, hipStream_t st) {
  const Geo q = geo3(P.nx, P.ny, P.nz);
  RT_NS(P, k_schur_faces, q.g, q.b, 0, st, P, U, nH, Dlag, s, loc, om, ph, diag, pdiag, c, fw, bw,
        b, pd32, cx32, cy32, cz32);
}
// one case per vector count 0..KMAX-1 (a run-time count selects a
// compile-time instantiation)
#define RT_VEC_CASES_1(X)                                                                  \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)       \
  X(16) X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29)    \
  X(30) X(31)
#define RT_VEC_CASES(X) X(0) RT_VEC_CASES_1(X)
static_assert(KMAX == 32, "RT_VEC_CASES lists the vector counts 0..KMAX-1");

int launch_spmv_full(int nx, int ny, int nz, const double* diag, const double* fw,
                     const double* bw, const double* z, const double* bsub, double* w,
                     double* zcopy, const double* V, int nvec, double* parts, hipStream_t st) {
  const long N = (long)nx * ny * nz;
  const int nb = reduce_blocks(N);
  switch (nvec) {
#define RT_SPMV_CASE(NV)                                                                      \
  case NV:                                                                                   \
    hipLaunchKernelGGL(k_spmv_full<NV>, dim3(nb), dim3(BLOCK), 0, st, nx, ny, nz, diag, fw,  \
                       bw, z, bsub, w, zcopy, V, parts, nb);                                  \
    break;
    RT_VEC_CASES(RT_SPMV_CASE)
#undef RT_SPMV_CASE
    default:
      return -1;   // beyond KMAX - 1: the host never asks for it (restart <= KMAX - 2)
  }
  return nb;
}
int launch_gs_pass(long N, double* w, const double* V, int nvec, const double* coef, int dots,
                   double* parts, hipStream_t st) {
  const int nb = reduce_blocks(N);
  switch (nvec) {
#define RT_GS_CASE(NV)                                                                    \
  case NV:                                                                               \
    if (dots)                                                                            \
      hipLaunchKernelGGL((k_gs_pass<NV, true>), dim3(nb), dim3(BLOCK), 0, st, N, w, V,   \
                         coef, parts, nb);                                               \
    else                                                                                 \
      hipLaunchKernelGGL((k_gs_pass<NV, false>), dim3(nb), dim3(BLOCK), 0, st, N, w, V,  \
                         coef, parts, nb);                                               \
    break;
    RT_VEC_CASES_1(RT_GS_CASE)
#undef RT_GS_CASE
    default:
      return -1;
  }
  return nb;
}
void launch_scale(long N, double* v, double sf, double* copy, float* r32, int ny, int nz,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(reduce_blocks(N)), dim3(BLOCK), 0, st, N, v, sf, copy, r32, ny,
                     nz);
}
void launch_combine(long N, double* x, const double* Z, int nvec, const double* y,
                    hipStream_t st) {
  switch (nvec) {
#define RT_COMBINE_CASE(NV)                                                                   \
  case NV:                                                                                   \
    hipLaunchKernelGGL(k_combine<NV>, dim3(reduce_blocks(N)), dim3(BLOCK), 0, st, N, x, Z,   \
                       y);                                                                   \
    break;
    RT_VEC_CASES_1(RT_COMBINE_CASE)
#undef RT_COMBINE_CASE
    default:
      break;
  }
}
void launch_final_multi(const double* parts, int nblk, int ncomp, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_final_multi, dim3(ncomp), dim3(1024), 0, st, parts, nblk, out);
}

template <class T>
void launch_fill(long n, T* x, T v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill<T>, grid_for(n), dim3(BLOCK), 0, st, n, x, v);
}
// a finest level of the FP32 cycle may be colour-split (Level::split); the
// launchers pick the matching instantiation
#define RT_LAYOUT(L, KERN, T, ...)                                                     \
  do {                                                                                 \
    if ((L).split) hipLaunchKernelGGL((KERN<T, true>), __VA_ARGS__);                   \
    else hipLaunchKernelGGL((KERN<T, false>), __VA_ARGS__);                            \
  } while (0)
template <class T>
void launch_rbgs(const Level<T>& L, int colour, hipStream_t st) {
  const Geo q = geo3(L.nx, L.ny, L.nz / 2);
  RT_LAYOUT(L, k_rbgs, T, q.g, q.b, 0, st, L, colour);
}
template <class T>
void launch_rbgs_first_pair(const Level<T>& L, T* xo, hipStream_t st) {
  const Geo q = geo3(L.nx, L.ny, L.nz);
  RT_LAYOUT(L, k_rbgs_first_pair, T, q.g, q.b, 0, st, L, xo);
}
template <class T>
void launch_rbgs_out64(const Level<T>& L, int colour, double* out64, const double* r64,
                       const double* q64, double* parts, hipStream_t st) {
  const Geo q = geo3(L.nx, L.ny, L.nz / 2);
  RT_LAYOUT(L, k_rbgs_out64, T, q.g, q.b, 0, st, L, colour, out64, r64, q64, parts);
}
template <class T>
int launch_rbgs_dots(const Level<T>& L, int colour, const T* r, const T* q, double* parts,
                     hipStream_t st) {
  const Geo g = geo3(L.nx, L.ny, L.nz / 2);
  RT_LAYOUT(L, k_rbgs_dots, T, g.g, g.b, 0, st, L, colour, r, q, parts);
  return (int)(g.g.x * g.g.y * g.g.z);
}
template <class T>
void launch_coarse_solve_lds(const Level<T>& L, int sweeps, hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_solve_lds<T>, dim3(L.blocks), dim3(CS_THREADS), 0, st, L, sweeps);
}
template <class T>
void launch_coarse_solve(const Level<T>& L, int sweeps, hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_solve<T>, dim3(1), dim3(1024), 0, st, L, sweeps);
}
template <class T>
void launch_mg_residual(const Level<T>& L, int red_only, hipStream_t st) {
  const Geo q = geo3(L.nx, L.ny, red_only ? L.nz / 2 : L.nz);
  RT_LAYOUT(L, k_mg_residual, T, q.g, q.b, 0, st, L, red_only);
}
template <class T>
void launch_restrict(const Level<T>& F, const Level<T>& C, int red_only, hipStream_t st) {
  const Geo q = geo3(C.nx, C.ny, C.nz);
  RT_LAYOUT(F, k_restrict, T, q.g, q.b, 0, st, F, C, red_only);
}
template <class T>
void launch_prolong_add(const Level<T>& C, const Level<T>& F, int colour, hipStream_t st) {
  const Geo q = geo3(F.nx, F.ny, colour >= 0 ? F.nz / 2 : F.nz);
  RT_LAYOUT(F, k_prolong_add, T, q.g, q.b, 0, st, C, F, colour);
}
template <class T>
void launch_coarsen(const Level<T>& F, const Level<T>& C, hipStream_t st) {
  const Geo q = geo3(C.nx, C.ny, C.nz);
  RT_LAYOUT(F, k_coarsen, T, q.g, q.b, 0, st, F, C);
}
void launch_box_extract(int nx, int ny, int nz, int B, int nbox, const long long* cells,
                        const double* diag, const double* cx, const double* cy, const double* cz,
                        double* bd, double* bx, double* by, double* bz, hipStream_t st) {
  const BoxMap m{nx, ny, nz, B, nbox};
  const Geo q = geo3(nbox * B, B, B);
  hipLaunchKernelGGL(k_box_extract, q.g, q.b, 0, st, m, cells, diag, cx, cy, cz, bd, bx, by, bz);
}
template <class T>
void launch_box_residual(int nx, int ny, int nz, int B, int nbox, const long long* cells,
                         const double* diag, const double* cx, const double* cy, const double* cz,
                         const double* r, const double* z, T* bv, hipStream_t st) {
  const BoxMap m{nx, ny, nz, B, nbox};
  const Geo q = geo3(nbox * B, B, B);
  hipLaunchKernelGGL(k_box_residual<T>, q.g, q.b, 0, st, m, cells, diag, cx, cy, cz, r, z, bv);
}
template <class T>
void launch_box_scatter_add(int nx, int ny, int nz, int B, int nbox, const long long* cells, int s,
                            const T* y, double* z, const double* r, const double* q,
                            double* parts, hipStream_t st) {
  const BoxMap m{nx, ny, nz, B, nbox};
  const Geo gq = geo3(B, B, B);
  hipLaunchKernelGGL(k_box_scatter_add<T>, gq.g, gq.b, 0, st, m, cells, s, y, z, r, q, parts);
}
void launch_box_smooth_s(int nx, int ny, int nz, int B, int nbox, const long long* cells, int s,
                         int colour, const double* diag, const double* fw, const double* bw,
                         const double* r, double* z, hipStream_t st) {
  const BoxMap m{nx, ny, nz, B, nbox};
  const Geo gq = geo3(B, B, B);
  hipLaunchKernelGGL(k_box_smooth_s, gq.g, gq.b, 0, st, m, cells, s, colour, diag, fw, bw, r, z);
}
void launch_box_smooth_s_lds(int nx, int ny, int nz, int B, int nbox, const long long* cells, int s,
                             int sweeps, const double* diag, const double* fw, const double* bw,
                             const double* r, double* z, hipStream_t st) {
  const BoxMap m{nx, ny, nz, B, nbox};
  hipLaunchKernelGGL(k_box_smooth_s_lds, dim3(1), dim3(BS_THREADS), 0, st, m, cells, s, sweeps, diag,
                     fw, bw, r, z);
}
template <class T>
int launch_box_dot1p(long n, const T* r, const T* z, T* p, double* parts, hipStream_t st) {
  hipLaunchKernelGGL(k_box_dot1p<T>, grid_for(n), dim3(BLOCK), 0, st, n, r, z, p, parts);
  return (int)grid_for(n).x;
}
template <class T>
int launch_box_spmv_p(const Level<T>& L, const T* z, const T* pin, T* pout, T* q,
                      const double* zparts, int nz_parts, double* sc, int rho_in, int rho_out,
                      bool first, double* parts, hipStream_t st) {
  const Geo g = geo3(L.nx, L.ny, L.nz);
  hipLaunchKernelGGL(k_box_spmv_p<T>, g.g, g.b, 0, st, L.nx, L.ny, L.nz, L.diag, L.cx, L.cy, L.cz,
                     z, pin, pout, q, zparts, nz_parts, sc, rho_in, rho_out, first ? 1 : 0, parts);
  return (int)(g.g.x * g.g.y * g.g.z);
}
template <class T>
void launch_box_update_xr(long n, T* x, T* r, const T* p, const T* q, const double* pqparts,
                          int npq, double* sc, int rho, hipStream_t st) {
  hipLaunchKernelGGL(k_box_update_xr<T>, grid_for(n), dim3(BLOCK), 0, st, n, x, r, p, q, pqparts,
                     npq, sc, rho);
}
template <class T>
void launch_box_update_first_pair(const Level<T>& L, T* x, const T* ro, T* rn, const T* p,
                                  const T* q, const double* pqparts, int npq, double* sc, int rho,
                                  hipStream_t st) {
  const Geo g = geo3(L.nx, L.ny, L.nz);
  hipLaunchKernelGGL(k_box_update_first_pair<T>, g.g, g.b, 0, st, L, x, ro, rn, p, q, pqparts, npq,
                     sc, rho);
}
template <class T>
int launch_box_dot2(long n, const T* z, const T* r, const T* q, double* parts, hipStream_t st) {
  hipLaunchKernelGGL(k_box_dot2<T>, grid_for(n), dim3(BLOCK), 0, st, n, z, r, q, parts);
  return (int)grid_for(n).x;
}
#define RT_BOX_INST(T)                                                                          \
  template void launch_box_residual<T>(int, int, int, int, int, const long long*, const double*, \
                                       const double*, const double*, const double*,            \
                                       const double*, const double*, T*, hipStream_t);          \
  template void launch_box_scatter_add<T>(int, int, int, int, int, const long long*, int,       \
                                          const T*, double*, const double*, const double*,     \
                                          double*, hipStream_t);                                \
  template int launch_box_dot1p<T>(long, const T*, const T*, T*, double*, hipStream_t);        \
  template int launch_box_spmv_p<T>(const Level<T>&, const T*, const T*, T*, T*, const double*,  \
                                    int, double*, int, int, bool, double*, hipStream_t);        \
  template void launch_box_update_xr<T>(long, T*, T*, const T*, const T*, const double*, int,   \
                                        double*, int, hipStream_t);                             \
  template void launch_box_update_first_pair<T>(const Level<T>&, T*, const T*, T*, const T*,      \
                                                const T*, const double*, int, double*, int,     \
                                                hipStream_t);                                   \
  template int launch_box_dot2<T>(long, const T*, const T*, const T*, double*, hipStream_t);
RT_BOX_INST(double)
RT_BOX_INST(float)
#undef RT_BOX_INST
void launch_cvt_split_d(const Level<double>& L, const double* a, double* b, hipStream_t st) {
  const Geo q = geo3(L.nx, L.ny, L.nz);
  hipLaunchKernelGGL(k_cvt_d2f_split<double>, q.g, q.b, 0, st, L.nx, L.ny, L.nz, a, b);
}
void launch_cvt_d2f_level(const Level<float>& L, const double* a, float* b, hipStream_t st) {
  if (L.split) {
    const Geo q = geo3(L.nx, L.ny, L.nz);
    hipLaunchKernelGGL(k_cvt_d2f_split<float>, q.g, q.b, 0, st, L.nx, L.ny, L.nz, a, b);
  } else {
    const long n = (long)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k_cvt_d2f, grid_for(n), dim3(BLOCK), 0, st, n, a, b);
  }
}
void launch_fold_energy(int N, double* U, double* eh, hipStream_t st) {
  hipLaunchKernelGGL(k_fold_energy, grid_for(N), dim3(BLOCK), 0, st, N, U, eh);
}
void launch_cvt_d2f(long n, const double* a, float* b, hipStream_t st) {
  hipLaunchKernelGGL(k_cvt_d2f, grid_for(n), dim3(BLOCK), 0, st, n, a, b);
}
void launch_cvt_f2d(long n, const float* a, double* b, hipStream_t st) {
  hipLaunchKernelGGL(k_cvt_f2d, grid_for(n), dim3(BLOCK), 0, st, n, a, b);
}

#define RT_INST(T)                                                                   \
  template void launch_fill<T>(long, T*, T, hipStream_t);                            \
  template void launch_rbgs<T>(const Level<T>&, int, hipStream_t);                   \
  template void launch_rbgs_first_pair<T>(const Level<T>&, T*, hipStream_t);         \
  template void launch_rbgs_out64<T>(const Level<T>&, int, double*, const double*, const double*, double*, hipStream_t); \
  template int launch_rbgs_dots<T>(const Level<T>&, int, const T*, const T*, double*, hipStream_t); \
  template void launch_coarse_solve<T>(const Level<T>&, int, hipStream_t);           \
  template void launch_coarse_solve_lds<T>(const Level<T>&, int, hipStream_t); \
  template void launch_mg_residual<T>(const Level<T>&, int, hipStream_t);            \
  template void launch_restrict<T>(const Level<T>&, const Level<T>&, int, hipStream_t); \
  template void launch_prolong_add<T>(const Level<T>&, const Level<T>&, int, hipStream_t); \
  template void launch_coarsen<T>(const Level<T>&, const Level<T>&, hipStream_t);
RT_INST(double)
RT_INST(float)
#undef RT_INST

}  // namespace rtk
