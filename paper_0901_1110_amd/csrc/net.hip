// Learned Newton initial guess: a 4-layer 3x3x3 periodic convolution network
// trained and run with BF16 MFMA (v_mfma_f32_16x16x16_bf16, FP32 accumulate).
//
// Not part of the paper's method: it only proposes U_0 for the Newton
// iteration, which the unchanged tolerance judges (the previous state is the
// fallback, chosen by initial residual inside rt_newton_step).
//
// Layout: activations channels-last BF16 [N][16] (32 B per cell, channels
// beyond the layer width are zero), cell (i*ny + j)*nz + k.  A convolution is
// an implicit GEMM per kernel offset o: out[co][cell] += W_o[co][ci] *
// in[ci][cell + off_o].  One wave computes a 16 (co) x 16 (cells along z)
// tile: MFMA A = weights (M = co, K = ci), B = shifted input (K = ci, N =
// cells).  Lane l holds A[l%16][4(l/16)..+3], B[4(l/16)..+3][l%16] and
// D[4(l/16)..+3][l%16], so every operand and result is one 8-byte access of
// four consecutive channels of one cell.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rt.h"

namespace rtn {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;

constexpr int CH = 16;          // padded channel width
constexpr int NOFF = 27;
constexpr int WG_BLOCKS = 512;  // split-K blocks of the weight gradient
constexpr float LEAK = 0.01f;
constexpr double X_CLIP = 1e-12;
constexpr double LOGIT_SCALE = 10.0;
constexpr double E_FLOOR_REL = 1e-10;
constexpr double W_CAP = 100.0;        // cap of the per-cell radiation loss weight
constexpr float CLIP = 1.0f;           // global gradient-norm clip of each Adam step   // radiation below 1e-10 u_E is invisible in the scaled residual

// float -> bf16, round to nearest even (finite inputs)
__device__ inline bf16 f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}
__device__ inline float bf2f(bf16 h) { return __uint_as_float(((unsigned)h) << 16); }

struct Geo {
  int nx, ny, nz, N;
};

__device__ inline int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ inline int off_cell(const Geo& g, int i, int j, int k, int o) {
  const int di = o / 9 - 1, dj = (o / 3) % 3 - 1, dk = o % 3 - 1;
  return (wrapi(i + di, g.nx) * g.ny + wrapi(j + dj, g.ny)) * g.nz + wrapi(k + dk, g.nz);
}

// --------------------------------------------------------------------------
// forward / data-gradient convolution, marching through x-planes.  A block
// owns a TJ x TK (y, z) tile and walks PI consecutive x-planes; the input of
// three planes over the tile plus a one-cell halo sits in LDS (slot = plane
// mod 3, 32 B per cell), so each input cell is fetched from memory about
// once per plane rather than once per kernel offset, and every lane keeps
// its 27 weight fragments (MFMA A operands) in registers.  A wave computes
// 16 (co) x 16 (cells along z) tiles with 27 MFMAs in offset order.
// In LDS the four 8-byte channel quads of a cell at position x of its row
// are stored in the order q ^ ((x >> 2) & 3): with 32 B per cell the 16
// lanes that read one quad of 16 consecutive cells would otherwise fall on
// four bank pairs.  The key depends on x only, so a lane's three z shifts
// have fixed quad offsets and, with the row length a compile-time constant,
// all 27 operand reads of a tile are immediate offsets from nine bases.
// mode 0: forward, out = act(bias + W * in); act = LeakyReLU if leaky.
// mode 1: data gradient, out = (sum_o Wt_o g[cell + off_o]) * leaky'(hprev),
//         Wt_o = W_{26-o}^T (both modes read the source at +off_o).
// last: write FP32 SoA [nout][N] instead of BF16 channels-last.
struct Tile {
  int TJ, TK, PI, ntj, ntk;
};
template <int TK>
__global__ __launch_bounds__(256) void k_conv(Geo g, Tile T, const bf16* __restrict__ in,
                                              const bf16* __restrict__ W,     // [27][16][16]
                                              const float* __restrict__ bias, int mode,
                                              int leaky, const bf16* __restrict__ hprev,
                                              bf16* __restrict__ out, float* __restrict__ out32,
                                              int nout) {
  extern __shared__ __align__(16) char lds[];
  constexpr int RK = TK + 2;                        // cells per LDS row (tile + halo)
  constexpr int CPR = TK / 16;                      // 16-cell chunks per tile row
  const int RJ = T.TJ + 2;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int q = lane >> 4;                          // channel quad
  const int col = lane & 15;
  int blk = blockIdx.x;
  const int tk = blk % T.ntk;
  blk /= T.ntk;
  const int tj = blk % T.ntj;
  const int i0 = (blk / T.ntj) * T.PI;
  const int j0 = tj * T.TJ, k0 = tk * TK;
  v4s a[NOFF];
#pragma unroll
  for (int o = 0; o < NOFF; ++o)
    a[o] = *reinterpret_cast<const v4s*>(W + (o * CH + col) * CH + 4 * q);
  float bq[4] = {0.f, 0.f, 0.f, 0.f};
  if (mode == 0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) bq[t] = bias[4 * q + t];
  }
  const int slot_bytes = RJ * RK * 32;
  auto slot = [&](int p) { return lds + ((p % 3 + 3) % 3) * slot_bytes; };
  // this thread's share of a plane load (16-byte halves t = tid + 256 u of
  // the (RJ, RK) tile with halo), the same in every plane but for the plane
  // offset: source offset within the plane, and LDS offset with bit 0 set
  // where the two quads are swapped (quads 2h, 2h + 1 land in the half
  // h ^ (sw >> 1), swapped if sw is odd; -1: no element)
  constexpr int NU = (6 * RK * 2 + 255) / 256;      // TJ <= 4
  int goff[NU], loff[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int t = threadIdx.x + 256 * u;
    loff[u] = -1;
    goff[u] = 0;
    if (t < RJ * RK * 2) {
      const int cr = t >> 1, h = t & 1;
      const int r = cr / RK, c = cr - r * RK;
      const int j = wrapi(j0 - 1 + r, g.ny), k = wrapi(k0 - 1 + c, g.nz);
      const int sw = (c >> 2) & 3;
      goff[u] = (j * g.nz + k) * CH + 8 * h;
      loff[u] = cr * 32 + 16 * (h ^ (sw >> 1)) + (sw & 1);
    }
  }
  const size_t pstride = (size_t)g.ny * g.nz * CH;
  uint4 pre[NU];
  auto fetch_plane = [&](int p) {
    const bf16* src = in + (size_t)wrapi(p, g.nx) * pstride;
#pragma unroll
    for (int u = 0; u < NU; ++u)
      if (loff[u] >= 0) pre[u] = *reinterpret_cast<const uint4*>(src + goff[u]);
  };
  auto store_plane = [&](int p) {
    char* s = slot(p);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      if (loff[u] < 0) continue;
      uint4 v = pre[u];
      if (loff[u] & 1) v = make_uint4(v.z, v.w, v.x, v.y);
      *reinterpret_cast<uint4*>(s + (loff[u] & ~1)) = v;
    }
  };
  // byte offset of this lane's quad in the cells at x = kc + col + e (kc is
  // a multiple of 16, so the key is that of col + e)
  int qo[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) qo[e] = 8 * (q ^ (((col + e) >> 2) & 3));
  const int nch = T.TJ * CPR;
  // plane i + 1 is fetched into registers while plane i - 1 ... i are in
  // use and stored into the slot of plane i - 2 after every wave is done
  // with that plane
  fetch_plane(i0 - 1);
  store_plane(i0 - 1);
  fetch_plane(i0);
  store_plane(i0);
  fetch_plane(i0 + 1);
  for (int i = i0; i < i0 + T.PI; ++i) {
    store_plane(i + 1);
    __syncthreads();
    if (i + 1 < i0 + T.PI) fetch_plane(i + 2);
    const char* sp[3] = {slot(i - 1), slot(i), slot(i + 1)};
    for (int ch = wv; ch < nch; ch += 4) {
      const int jj = ch / CPR;
      const int kc = (ch - jj * CPR) << 4;
      const int rc = (jj * RK + kc + col) * 32;
      v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int o = 0; o < NOFF; ++o) {
        const int di = o / 9, dj = (o / 3) % 3, dk = o % 3;   // shifts + 1
        const char* bp = sp[di] + rc + qo[dk];
        const v4s b = *reinterpret_cast<const v4s*>(bp + (dj * RK + dk) * 32);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[o], b, acc, 0, 0, 0);
      }
      const int cell = (i * g.ny + j0 + jj) * g.nz + k0 + kc + col;
      float v[4] = {acc[0], acc[1], acc[2], acc[3]};
      if (mode == 0) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          v[t] += bq[t];
          if (leaky) v[t] = v[t] > 0.f ? v[t] : LEAK * v[t];
        }
      } else if (hprev) {
        const v4s hp = *reinterpret_cast<const v4s*>(hprev + (size_t)cell * CH + 4 * q);
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] *= bf2f((bf16)hp[t]) > 0.f ? 1.f : LEAK;
      }
      if (out32) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (4 * q + t < nout) out32[(size_t)(4 * q + t) * g.N + cell] = v[t];
      } else {
        v4s r;
#pragma unroll
        for (int t = 0; t < 4; ++t) r[t] = (short)f2bf(v[t]);
        *reinterpret_cast<v4s*>(out + (size_t)cell * CH + 4 * q) = r;
      }
    }
    __syncthreads();     // plane i's slots are read: plane i + 2 may replace i - 1
  }
}

// weight gradient, split-K over cells: block b accumulates
//   dW[o][co][ci] = sum_cells gout[cell][co] * in[cell + off_o][ci]
// for its cell range; wave w owns offsets w, w+4, ...  MFMA A = gout^T
// (M = co, K = 16 cells), B = shifted input (K = cells, N = ci).
__global__ __launch_bounds__(256) void k_conv_wgrad(Geo g, const bf16* __restrict__ gout,
                                                    const bf16* __restrict__ in,
                                                    float* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int q = lane >> 4;
  const int col = lane & 15;
  const int nchunk = g.N / 16;
  const int per = (nchunk + gridDim.x - 1) / gridDim.x;
  const int c0 = blockIdx.x * per;
  const int c1 = min(nchunk, c0 + per);
  v4f acc[7];
#pragma unroll
  for (int s = 0; s < 7; ++s) acc[s] = v4f{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  const int cpr = g.nz >> 4;
  for (int ch = c0; ch < c1; ++ch) {
    const int row = ch / cpr;
    const int kb = ((ch - row * cpr) << 4) + 4 * q;   // this lane's first cell (k)
    const int j = row % g.ny;
    const int i = row / g.ny;
    const int cell = row * g.nz + kb;
    v4s a;
#pragma unroll
    for (int t = 0; t < 4; ++t) a[t] = (short)gout[(size_t)(cell + t) * CH + col];
    if (w == 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) bsum += bf2f((bf16)a[t]);
    }
#pragma unroll
    for (int s = 0; s < 7; ++s) {
      const int o = w + 4 * s;
      if (o < NOFF) {
        v4s b;
#pragma unroll
        for (int t = 0; t < 4; ++t) b[t] = (short)in[(size_t)off_cell(g, i, j, kb + t, o) * CH + col];
        acc[s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[s], 0, 0, 0);
      }
    }
  }
  float* P = part + (size_t)blockIdx.x * (NOFF * 256 + 16);
#pragma unroll
  for (int s = 0; s < 7; ++s) {
    const int o = w + 4 * s;
    if (o < NOFF) {
#pragma unroll
      for (int t = 0; t < 4; ++t) P[(o * 16 + 4 * q + t) * 16 + col] = acc[s][t];
    }
  }
  if (w == 0) {
    // sum the four cell quads of each channel (fixed butterfly order)
    bsum += __shfl_xor(bsum, 16, 64);
    bsum += __shfl_xor(bsum, 32, 64);
    if (lane < 16) P[NOFF * 256 + lane] = bsum;
  }
}

// deterministic reduction of the split-K partials into the flat gradient of
// one layer (order: W (27, co, ci) then bias)
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nblk, int CO, int CI,
                               float* __restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int nW = NOFF * CO * CI;
  if (e >= nW + CO) return;
  int src;
  if (e < nW) {
    const int o = e / (CO * CI), r = e % (CO * CI), co = r / CI, ci = r % CI;
    src = (o * 16 + co) * 16 + ci;
  } else {
    src = NOFF * 256 + (e - nW);
  }
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * (NOFF * 256 + 16) + src];
  grad[e] = (float)s;
}

// --------------------------------------------------------------------------
// features, targets, decode, loss
__device__ inline double logit_s(double x) {
  x = fmin(fmax(x, X_CLIP), 1.0 - X_CLIP);
  return log(x / (1.0 - x)) / LOGIT_SCALE;
}

struct Scales {
  double u_e, u_E, nH_mean;
  int ns;
};

// transformed coordinates of a state: (log10 E/u_E, e/u_e, logit x / 10 ...)
__device__ inline void transform(const double* U, const double* e, int c, int N, const Scales& S,
                                 double* t) {
  t[0] = log10(fmax(U[(size_t)(S.ns + 1) * N + c], E_FLOOR_REL * S.u_E) / S.u_E);
  t[1] = e[c] / S.u_e;
  for (int s = 0; s < S.ns; ++s) t[2 + s] = logit_s(U[(size_t)(1 + s) * N + c]);
}

// base non-null: also the FP64 extrapolation 2 t^n - t^(n-1) that the
// decode adds the network's correction to ([nt][N])
__global__ void k_features(int N, Scales S, const double* __restrict__ Un,
                           const double* __restrict__ Unm1, const double* __restrict__ en,
                           const double* __restrict__ enm1, const double* __restrict__ nH,
                           bf16* __restrict__ feat, double* __restrict__ base) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double t[5], tm[5];
  float f[CH];
#pragma unroll
  for (int q = 0; q < CH; ++q) f[q] = 0.f;
  const int nt = S.ns + 2;
  transform(Un, en, c, N, S, t);
  for (int q = 0; q < nt; ++q) f[q] = (float)t[q];
  transform(Unm1, enm1, c, N, S, tm);
  for (int q = 0; q < nt; ++q) f[nt + q] = (float)tm[q];
  if (base)
    for (int q = 0; q < nt; ++q) base[(size_t)q * N + c] = 2.0 * t[q] - tm[q];
  f[2 * nt] = (float)log10(nH[c] / S.nH_mean);
  v4s* out = reinterpret_cast<v4s*>(feat + (size_t)c * CH);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    v4s r;
#pragma unroll
    for (int t2 = 0; t2 < 4; ++t2) r[t2] = (short)f2bf(f[4 * v + t2]);
    out[v] = r;
  }
}

// training target: level n+1 minus the linear extrapolation 2 t^n - t^(n-1)
__global__ void k_target(int N, Scales S, const double* __restrict__ Un,
                         const double* __restrict__ en, const double* __restrict__ Unm1,
                         const double* __restrict__ enm1, const double* __restrict__ Unp1,
                         const double* __restrict__ enp1, float* __restrict__ tgt,
                         double* __restrict__ wE) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  wE[c] = fmax(Un[(size_t)(S.ns + 1) * N + c], E_FLOOR_REL * S.u_E) / S.u_E;
  double a[5], am[5], b[5];
  transform(Un, en, c, N, S, a);
  transform(Unm1, enm1, c, N, S, am);
  transform(Unp1, enp1, c, N, S, b);
  for (int q = 0; q < S.ns + 2; ++q)
    tgt[(size_t)q * N + c] = (float)(b[q] - (2.0 * a[q] - am[q]));
}

// guess = inverse transform of (linear extrapolation + network correction)
// base: the extrapolation the features pass stored
__global__ void k_decode(int N, Scales S, const double* __restrict__ base,
                         const double* __restrict__ eh, const float* __restrict__ d,
                         double* __restrict__ Ug) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double t[5];
  const int ns = S.ns;
  for (int q = 0; q < ns + 2; ++q) t[q] = base[(size_t)q * N + c] + (double)d[(size_t)q * N + c];
  Ug[(size_t)(ns + 1) * N + c] = S.u_E * pow(10.0, t[0]);
  Ug[c] = S.u_e * t[1] - eh[c];
  double x[3];
  for (int s = 0; s < ns; ++s) x[s] = 1.0 / (1.0 + exp(-t[2 + s] * LOGIT_SCALE));
  if (ns == 3) {
    const double tot = x[1] + x[2];
    if (tot > 1.0) {
      x[1] /= tot;
      x[2] /= tot;
    }
  }
  for (int s = 0; s < ns; ++s) Ug[(size_t)(1 + s) * N + c] = x[s];
}

// weighted MSE: gradient 2 w (out - target) / (N nout) as BF16 channels-last,
// loss partials; channel 0 weight = wE[cell] / mean(wE), others 1
__global__ __launch_bounds__(256) void k_loss(int N, int nout, const float* __restrict__ out,
                                              const float* __restrict__ tgt,
                                              const double* __restrict__ wE,
                                              const double* __restrict__ wsum,
                                              bf16* __restrict__ gout, double* __restrict__ part) {
  __shared__ double sh[4];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (c < N) {
    const float scale = 2.0f / ((float)N * (float)nout);
    const double w0 = fmin(wE[c] * ((double)N / wsum[0]), W_CAP);
    bf16 r[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) r[q] = 0;
    for (int q = 0; q < nout; ++q) {
      const float dq = out[(size_t)q * N + c] - tgt[(size_t)q * N + c];
      const double wq = q == 0 ? w0 : 1.0;
      acc += wq * dq * dq;
      r[q] = f2bf((float)(wq * scale * dq));
    }
    v4s* o = reinterpret_cast<v4s*>(gout + (size_t)c * CH);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      v4s t;
#pragma unroll
      for (int u = 0; u < 4; ++u) t[u] = (short)r[4 * v + u];
      o[v] = t;
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ void k_sum(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += part[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += sh[w];
    out[0] = t;
  }
}

// Adam on the FP32 master parameters (flat order), then nothing else: the
// BF16 GEMM layouts are rebuilt by k_pack
__global__ void k_gnorm(int P, const float* __restrict__ gr, double* __restrict__ out) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < P; i += 1024) s += (double)gr[i] * gr[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += sh[w];
    out[0] = sqrt(t);
  }
}

__global__ void k_adam(int P, float* __restrict__ th, float* __restrict__ m,
                       float* __restrict__ v, const float* __restrict__ gr,
                       const double* __restrict__ gnorm, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P) return;
  const float clip = gnorm[0] > CLIP ? (float)(CLIP / gnorm[0]) : 1.0f;
  const float gv = gr[e] * clip;
  const float mv = b1 * m[e] + (1.f - b1) * gv;
  const float vv = b2 * v[e] + (1.f - b2) * gv * gv;
  m[e] = mv;
  v[e] = vv;
  th[e] -= lr * (mv / c1) / (sqrtf(vv / c2) + eps);
}

// master parameters of one layer -> BF16 [27][16][16] (forward: [o][co][ci],
// transposed for the data gradient: [26-o][ci][co]) and FP32 bias [16]
__global__ void k_pack(const float* __restrict__ th, int CO, int CI, bf16* __restrict__ Wf,
                       bf16* __restrict__ Wt, float* __restrict__ bias) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < NOFF * 256) {
    const int o = e / 256, co = (e / 16) % 16, ci = e % 16;
    float w = 0.f;
    if (co < CO && ci < CI) w = th[(o * CO + co) * CI + ci];
    const bf16 h = f2bf(w);
    Wf[(o * 16 + co) * 16 + ci] = h;
    Wt[((NOFF - 1 - o) * 16 + ci) * 16 + co] = h;
  }
  if (e < 16) bias[e] = e < CO ? th[NOFF * CO * CI + e] : 0.f;
}

__global__ void k_unpack_feat(int N, const bf16* __restrict__ a, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  for (int q = 0; q < CH; ++q) out[(size_t)q * N + c] = bf2f(a[(size_t)c * CH + q]);
}

}  // namespace rtn

using namespace rtn;

// ===========================================================================
struct rt_net {
  int ns, nin, nout, P;
  Geo g;
  hipStream_t st;
  int CI[4], CO[4], off[4];
  bf16 *feat, *h[3], *gA, *gB;
  float *out, *tgt, *part, *grad, *th, *m, *v, *bias;
  bf16 *Wf, *Wt;
  double *lpart, *lsum, *wE, *wsum;
  double* base;   // FP64 extrapolation 2 t(U^n) - t(U^(n-1)) of the last features pass
  int nblk_loss;
  int step = 0;
  std::string err;
};

namespace {

size_t carve_net(int ns, int nx, int ny, int nz, char* base, rt_net* n) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) / 256 * 256;
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const size_t N = (size_t)nx * ny * nz;
  const int nin = 2 * (ns + 2) + 1, nout = ns + 2;
  const int CI[4] = {nin, 16, 16, 16}, CO[4] = {16, 16, 16, nout};
  int P = 0;
  for (int l = 0; l < 4; ++l) P += NOFF * CI[l] * CO[l] + CO[l];
  rt_net tmp;
  rt_net* t = n ? n : &tmp;
  t->feat = (bf16*)take(N * CH * 2);
  for (int l = 0; l < 3; ++l) t->h[l] = (bf16*)take(N * CH * 2);
  t->gA = (bf16*)take(N * CH * 2);
  t->gB = (bf16*)take(N * CH * 2);
  t->out = (float*)take(N * nout * 4);
  t->tgt = (float*)take(N * nout * 4);
  t->part = (float*)take((size_t)WG_BLOCKS * (NOFF * 256 + 16) * 4);
  t->grad = (float*)take((size_t)P * 4);
  t->th = (float*)take((size_t)P * 4);
  t->m = (float*)take((size_t)P * 4);
  t->v = (float*)take((size_t)P * 4);
  t->bias = (float*)take(4 * 16 * 4);
  t->Wf = (bf16*)take(4 * NOFF * 256 * 2);
  t->Wt = (bf16*)take(4 * NOFF * 256 * 2);
  t->nblk_loss = (int)((N + 255) / 256);
  t->lpart = (double*)take((size_t)t->nblk_loss * 8);
  t->lsum = (double*)take(64);
  t->wE = (double*)take(N * 8);
  t->wsum = (double*)take(64);
  t->base = (double*)take(N * nout * 8);
  if (n) {
    n->ns = ns; n->nin = nin; n->nout = nout; n->P = P;
    int o = 0;
    for (int l = 0; l < 4; ++l) {
      n->CI[l] = CI[l]; n->CO[l] = CO[l]; n->off[l] = o;
      o += NOFF * CI[l] * CO[l] + CO[l];
    }
  }
  return off + 256;
}

int nfail(rt_net* n, int code, const char* msg) {
  if (n) n->err = msg;
  return code;
}

#define NCHK(n, call)                                                   \
  do {                                                                  \
    hipError_t e_ = (call);                                             \
    if (e_ != hipSuccess) return nfail((n), RT_EDEVICE, hipGetErrorString(e_)); \
  } while (0)

bool geom_ok(int nx, int ny, int nz) {
  // cell indices are 32-bit; every channel or field offset is formed in size_t
  return nx >= 3 && ny >= 3 && nz >= 16 && nz % 16 == 0 &&
         (double)nx * ny * nz < 2147483647.0;
}

inline unsigned nb(long n, int b) { return (unsigned)((n + b - 1) / b); }

void pack_all(rt_net* n) {
  for (int l = 0; l < 4; ++l)
    hipLaunchKernelGGL(k_pack, dim3(nb(NOFF * 256, 256)), dim3(256), 0, n->st, n->th + n->off[l],
                       n->CO[l], n->CI[l], n->Wf + l * NOFF * 256, n->Wt + l * NOFF * 256,
                       n->bias + 16 * l);
}

// tile of the plane-marching convolution: TK in {64, 32, 16} dividing nz,
// TJ in {4, 2, 1} dividing ny, and the longest march in {16, 8, 4, 2}
// dividing nx that still leaves at least 512 blocks
Tile conv_tile(const Geo& g) {
  Tile t;
  t.TK = g.nz % 64 == 0 ? 64 : (g.nz % 32 == 0 ? 32 : 16);
  t.TJ = g.ny % 4 == 0 ? 4 : (g.ny % 2 == 0 ? 2 : 1);
  t.ntj = g.ny / t.TJ;
  t.ntk = g.nz / t.TK;
  t.PI = 1;
  for (int c : {16, 8, 4, 2}) {
    if (g.nx % c == 0 && (long)t.ntj * t.ntk * (g.nx / c) >= 512) {
      t.PI = c;
      break;
    }
  }
  return t;
}

void launch_conv(rt_net* n, const bf16* in, int layer, int mode, int leaky, const bf16* hprev,
                 bf16* out, float* out32) {
  const bf16* W = (mode == 0 ? n->Wf : n->Wt) + layer * NOFF * 256;
  const Tile t = conv_tile(n->g);
  const unsigned blocks = (unsigned)((long)t.ntj * t.ntk * (n->g.nx / t.PI));
  const size_t lds = (size_t)3 * (t.TJ + 2) * (t.TK + 2) * 32;
  auto kern = t.TK == 64 ? k_conv<64> : (t.TK == 32 ? k_conv<32> : k_conv<16>);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), lds, n->st, n->g, t, in, W,
                     n->bias + 16 * layer, mode, leaky, hprev, out, out32, n->nout);
}

Scales scales(rt_net* n, double u_e, double u_E, double nH_mean) {
  return Scales{u_e, u_E, nH_mean, n->ns};
}

void forward(rt_net* n) {
  launch_conv(n, n->feat, 0, 0, 1, nullptr, n->h[0], nullptr);
  launch_conv(n, n->h[0], 1, 0, 1, nullptr, n->h[1], nullptr);
  launch_conv(n, n->h[1], 2, 0, 1, nullptr, n->h[2], nullptr);
  launch_conv(n, n->h[2], 3, 0, 0, nullptr, nullptr, n->out);
}

}  // namespace

extern "C" {

int rt_net_workspace_bytes(int32_t nspecies, int32_t nx, int32_t ny, int32_t nz, uint64_t* bytes) {
  if (!bytes || (nspecies != 1 && nspecies != 3) || !geom_ok(nx, ny, nz)) return RT_EINVAL;
  *bytes = carve_net(nspecies, nx, ny, nz, nullptr, nullptr);
  return RT_OK;
}

int rt_net_create(int32_t nspecies, int32_t nx, int32_t ny, int32_t nz, void* d_ws,
                  uint64_t ws_bytes, void* hip_stream, rt_net** out) {
  if (!out) return RT_EINVAL;
  *out = nullptr;
  if ((nspecies != 1 && nspecies != 3) || !geom_ok(nx, ny, nz)) return RT_EINVAL;
  const size_t need = carve_net(nspecies, nx, ny, nz, nullptr, nullptr);
  if (!d_ws || ws_bytes < need) return RT_EINVAL;
  char* base = reinterpret_cast<char*>(d_ws);
  base += (256 - reinterpret_cast<uintptr_t>(base) % 256) % 256;
  rt_net* n = new rt_net();
  n->g = Geo{nx, ny, nz, nx * ny * nz};
  n->st = reinterpret_cast<hipStream_t>(hip_stream);
  carve_net(nspecies, nx, ny, nz, base, n);
  hipError_t e = hipMemsetAsync(n->m, 0, (size_t)n->P * 4, n->st);
  if (e == hipSuccess) e = hipMemsetAsync(n->v, 0, (size_t)n->P * 4, n->st);
  if (e == hipSuccess) e = hipMemsetAsync(n->th, 0, (size_t)n->P * 4, n->st);
  if (e == hipSuccess) e = hipStreamSynchronize(n->st);
  if (e != hipSuccess) {
    delete n;
    return RT_EDEVICE;
  }
  *out = n;
  return RT_OK;
}

int rt_net_destroy(rt_net* n) {
  delete n;
  return RT_OK;
}

const char* rt_net_last_error(const rt_net* n) { return n ? n->err.c_str() : "null net"; }

int rt_net_num_params(const rt_net* n) { return n ? n->P : -1; }

int rt_net_set_params(rt_net* n, const float* h_theta, int32_t count) {
  if (!n || !h_theta || count != n->P) return nfail(n, RT_EINVAL, "parameter count mismatch");
  NCHK(n, hipMemcpyAsync(n->th, h_theta, (size_t)n->P * 4, hipMemcpyHostToDevice, n->st));
  NCHK(n, hipMemsetAsync(n->m, 0, (size_t)n->P * 4, n->st));
  NCHK(n, hipMemsetAsync(n->v, 0, (size_t)n->P * 4, n->st));
  n->step = 0;
  pack_all(n);
  NCHK(n, hipStreamSynchronize(n->st));
  return RT_OK;
}

int rt_net_get_params(rt_net* n, float* h_theta, int32_t count) {
  if (!n || !h_theta || count != n->P) return nfail(n, RT_EINVAL, "parameter count mismatch");
  NCHK(n, hipMemcpyAsync(h_theta, n->th, (size_t)n->P * 4, hipMemcpyDeviceToHost, n->st));
  NCHK(n, hipStreamSynchronize(n->st));
  return RT_OK;
}

int rt_net_forward(rt_net* n, const double* d_Un, const double* d_Unm1, const double* d_en,
                   const double* d_enm1, const double* d_nH, double nH_mean, double u_e,
                   double u_E, const double* d_eh, double* d_Uguess) {
  if (!n || !d_Un || !d_Unm1 || !d_en || !d_enm1 || !d_nH || !d_eh || !d_Uguess ||
      !(nH_mean > 0) || !(u_e > 0) || !(u_E > 0))
    return nfail(n, RT_EINVAL, "bad argument");
  const Scales S = scales(n, u_e, u_E, nH_mean);
  const int N = n->g.N;
  hipLaunchKernelGGL(k_features, dim3(nb(N, 256)), dim3(256), 0, n->st, N, S, d_Un, d_Unm1, d_en,
                     d_enm1, d_nH, n->feat, n->base);
  forward(n);
  hipLaunchKernelGGL(k_decode, dim3(nb(N, 256)), dim3(256), 0, n->st, N, S, n->base, d_eh, n->out,
                     d_Uguess);
  NCHK(n, hipGetLastError());
  return RT_OK;
}

int rt_net_get_output(rt_net* n, float* d_out, float* d_feat) {
  if (!n) return RT_EINVAL;
  const int N = n->g.N;
  if (d_out)
    NCHK(n, hipMemcpyAsync(d_out, n->out, (size_t)n->nout * N * 4, hipMemcpyDeviceToDevice, n->st));
  if (d_feat)
    hipLaunchKernelGGL(k_unpack_feat, dim3(nb(N, 256)), dim3(256), 0, n->st, N, n->feat, d_feat);
  NCHK(n, hipGetLastError());
  return RT_OK;
}

// loss and gradient for one sample (levels n-1, n -> n+1); lr > 0 also
// applies one Adam step.  *h_loss receives the mean squared error.
int rt_net_train_step(rt_net* n, const double* d_Un, const double* d_Unm1, const double* d_en,
                      const double* d_enm1, const double* d_nH, double nH_mean, double u_e,
                      double u_E, const double* d_Unp1, const double* d_enp1, float lr,
                      float* h_loss, float* h_grad) {
  if (!n || !d_Un || !d_Unm1 || !d_en || !d_enm1 || !d_nH || !d_Unp1 || !d_enp1 ||
      !(nH_mean > 0) || !(lr >= 0))
    return nfail(n, RT_EINVAL, "bad argument");
  const Scales S = scales(n, u_e, u_E, nH_mean);
  const int N = n->g.N;
  hipLaunchKernelGGL(k_features, dim3(nb(N, 256)), dim3(256), 0, n->st, N, S, d_Un, d_Unm1, d_en,
                     d_enm1, d_nH, n->feat, nullptr);
  hipLaunchKernelGGL(k_target, dim3(nb(N, 256)), dim3(256), 0, n->st, N, S, d_Un, d_en, d_Unm1,
                     d_enm1, d_Unp1, d_enp1, n->tgt, n->wE);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, n->st, n->wE, N, n->wsum);
  forward(n);
  hipLaunchKernelGGL(k_loss, dim3(n->nblk_loss), dim3(256), 0, n->st, N, n->nout, n->out, n->tgt,
                     n->wE, n->wsum, n->gA, n->lpart);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, n->st, n->lpart, n->nblk_loss, n->lsum);
  // backward: layer 3 .. 0
  const bf16* layer_in[4] = {n->feat, n->h[0], n->h[1], n->h[2]};
  bf16* g = n->gA;
  bf16* gnext = n->gB;
  for (int l = 3; l >= 0; --l) {
    hipLaunchKernelGGL(k_conv_wgrad, dim3(WG_BLOCKS), dim3(256), 0, n->st, n->g, g, layer_in[l],
                       n->part);
    const int nW = NOFF * n->CO[l] * n->CI[l] + n->CO[l];
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb(nW, 256)), dim3(256), 0, n->st, n->part, WG_BLOCKS,
                       n->CO[l], n->CI[l], n->grad + n->off[l]);
    if (l > 0) {
      // gradient wrt this layer's input, times LeakyReLU' of the previous layer
      launch_conv(n, g, l, 1, 0, layer_in[l], gnext, nullptr);
      std::swap(g, gnext);
    }
  }
  if (lr > 0) {
    ++n->step;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)n->step), c2 = 1.f - std::pow(b2, (float)n->step);
    hipLaunchKernelGGL(k_gnorm, dim3(1), dim3(1024), 0, n->st, n->P, n->grad, n->wsum + 1);
    hipLaunchKernelGGL(k_adam, dim3(nb(n->P, 256)), dim3(256), 0, n->st, n->P, n->th, n->m, n->v,
                       n->grad, n->wsum + 1, lr, b1, b2, 1e-8f, c1, c2);
    pack_all(n);
  }
  double loss = 0.0;
  NCHK(n, hipMemcpyAsync(&loss, n->lsum, 8, hipMemcpyDeviceToHost, n->st));
  if (h_grad) NCHK(n, hipMemcpyAsync(h_grad, n->grad, (size_t)n->P * 4, hipMemcpyDeviceToHost, n->st));
  NCHK(n, hipStreamSynchronize(n->st));
  if (h_loss) *h_loss = (float)(loss / ((double)N * n->nout));
  return RT_OK;
}

}  // extern "C"
