// Host solver control and C ABI of the implicit Newton step (see rt.h).
//
// Only control scalars cross the host/device boundary: the residual norm and
// bound-violation count of each line-search trial and ||r||^2 of each CG
// iteration (8-16 byte copies).  CG's alpha and beta stay on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rt.h"
#include "internal.hpp"

using namespace rtk;

namespace {

constexpr double LAMBDA_MIN = 1.0 / 1024.0;   // line-search floor 2^-10
constexpr double ARMIJO = 1.0e-4;
constexpr size_t ALIGN = 256;

struct Carver {
  char* base;
  size_t off = 0;
  bool dry;
  template <class T>
  T* take(size_t count) {
    off = (off + ALIGN - 1) / ALIGN * ALIGN;
    T* p = dry ? nullptr : reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

struct Workspace {
  double *D, *g, *f, *ft, *Ut;
  double *ftM, *W;
  // Schur matrix: diagonal and the two couplings of every +x/+y/+z face
  // (fw = -S_{P,P+d}, bw = -S_{P+d,P}; 3N each, direction-major); the
  // preconditioner's symmetric operator: pdiag and the face couplings c
  // (cx, cy, cz point into one 3N block); right side b
  double *diag, *fw, *bw, *pdiag, *cx, *cy, *cz, *b;
  double *om, *ph;          // species columns coupled through the face opacity
  double *x, *r, *z, *p, *q;
  // flexible GMRES: basis V (restart + 1 vectors), preconditioned vectors Z
  // (restart), multi-component partials, device scalars
  double *V = nullptr, *Z = nullptr, *gparts = nullptr, *gh = nullptr, *gy = nullptr;
  double *parts, *sc;
  long long* src_cells;
  double* src_Q;
  std::vector<Level<double>> L64;
  std::vector<Level<float>> L32;
  float* r32;   // FP32 copy of the CG residual fed to the V-cycle
  // source subdomains: boxes of B^3 cells around the sources, stacked along x
  int box_cap = 0;                        // boxes the workspace holds (max_sources)
  double *bd, *bcx, *bcy, *bcz;           // box operator (FP64, level 0 of B64)
  double *bxv, *br, *br2, *bz, *bp, *bp2, *bq;  // inner PCG vectors (FP32 cycle: float inside)
  double *bparts, *bparts2, *bsc;
  std::vector<Level<double>> B64;
  std::vector<Level<float>> B32;
  size_t nparts_cap;
};

}  // namespace

struct Timer {
  bool on = false;
  uint32_t mask = 0xffffffffu;            // classes recorded while on
  std::vector<hipEvent_t> pool;           // events, reused across collections
  std::vector<int> cls;                   // class of each recorded launch
  size_t used = 0;
  double bytes[RT_K_COUNT] = {};          // algorithmic bytes of the recorded launches
};

struct rt_grid {
  Timer tm;
  rt_params prm;
  DevParams P;
  hipStream_t st;
  Workspace w;
  const double* nH = nullptr;
  const double* eh = nullptr;
  int nsrc = 0;
  bool have_tl = false;     // lagged limiter: time-level face coefficients present
  bool mg_stale = true;     // coarse operators need rebuilding
  bool have_op = false;     // a Schur matrix is present
  bool l0_fp32 = false;     // the finest level's operator copy (FP32, or colour-split FP64) is current
  const double* r32_of = nullptr;   // the CG residual whose FP32 copy is the finest right side
  double* hpin = nullptr;   // pinned host scalars for asynchronous read-back
  int nbox = 0;             // active source subdomains (0: V-cycle alone)
  int tk_override = -1;     // >= 0: time every launch under this class
  bool capturing = false;   // launches go into the box graph: bytes to cap_bytes
  double cap_bytes = 0.0;
  double cg_rate1 = 0.0;    // residual reduction of the last solve's first CG step (0: none yet)
  hipEvent_t ev_rd = nullptr;
  // the source-subdomain correction as a captured graph (a few hundred small
  // launches replayed by one), valid for the (r, z, nbox) it was captured for
  bool graphs = true;
  hipStream_t cap_st = nullptr;
  struct BoxGraph {
    hipGraphExec_t exec = nullptr;
    const double* r = nullptr;
    double* z = nullptr;
    int nbox = 0, dots = 0;
    double bytes = 0.0;     // algorithmic bytes of one replay
  };
  // one captured correction per (r, z, dots) in use: FGMRES applies the
  // preconditioner to each basis vector v_j into its own z_j
  std::vector<BoxGraph> box_graphs;
  std::string err;
};

namespace {

int fail(rt_grid* g, int code, const char* fmt, ...) {
  if (g) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g->err = buf;
  }
  return code;
}

// record a start event (returns the slot) / stop event around a launch
inline long tstart(rt_grid* g, int cls) {
  Timer& t = g->tm;
  if (g->tk_override >= 0) cls = g->tk_override;
  if (!t.on || !((t.mask >> cls) & 1u)) return -1;
  if (t.used + 2 > t.pool.size()) {
    const size_t grow = t.pool.size() < 1024 ? 1024 : t.pool.size();
    for (size_t i = 0; i < grow; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) { t.on = false; return -1; }
      t.pool.push_back(e);
    }
  }
  const long slot = (long)t.used;
  if (hipEventRecord(t.pool[t.used], g->st) != hipSuccess) {
    t.on = false;   // timing stops; the launch itself goes ahead
    return -1;
  }
  t.used += 2;
  t.cls.push_back(cls);
  return slot;
}
inline void tstop(rt_grid* g, long slot) {
  if (slot >= 0) (void)hipEventRecord(g->tm.pool[slot + 1], g->st);
}
#define TK(g, cls, expr)               \
  do {                                 \
    const long slot_ = tstart(g, cls); \
    expr;                              \
    tstop(g, slot_);                   \
  } while (0)
// the same, also counting the launch's algorithmic bytes (each field it
// must read or write, once) for its class: while timing is on, whatever
// classes are selected for events, and into the graph's figure while the
// box correction is being captured
inline void addb(rt_grid* g, int cls, double nbytes) {
  if (g->capturing) {
    g->cap_bytes += nbytes;
    return;
  }
  if (!g->tm.on) return;
  if (g->tk_override >= 0) cls = g->tk_override;
  g->tm.bytes[cls] += nbytes;
}
#define TKB(g, cls, nbytes, expr) \
  do {                            \
    TK(g, cls, expr);             \
    addb(g, cls, (nbytes));       \
  } while (0)

#define HIPCHK(g, call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail((g), RT_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));              \
  } while (0)

#define RTCHK(call)              \
  do {                           \
    int s_ = (call);             \
    if (s_ != RT_OK) return s_;  \
  } while (0)

bool is_pow2_div(int n, int levels) {
  const int f = 1 << (levels - 1);
  return n % f == 0 && (n / f) >= 4 && ((n / f) % 2 == 0);
}

int validate(const rt_params* p, std::string* why) {
  auto bad = [&](const char* m) { *why = m; return RT_EINVAL; };
  if (!p) return bad("null params");
  if (p->lte != 0 && p->lte != 1) return bad("lte must be 0 or 1");
  if (p->boundary < 0 || p->boundary > 2) return bad("boundary must be 0, 1 or 2");
  if (p->boundary == 2 && (!(p->E_dirichlet >= 0.0) || !std::isfinite(p->E_dirichlet)))
    return bad("E_dirichlet must be finite and >= 0");
  if (p->lte ? p->nspecies != 0 : (p->nspecies != 1 && p->nspecies != 3))
    return bad("nspecies must be 1 or 3 (0 exactly with lte)");
  if (p->lte && (!(p->kappa_lte >= 0.0) || !(p->kappaP_lte >= 0.0) || !(p->mu_lte > 0.0) ||
                 !std::isfinite(p->kappa_lte) || !std::isfinite(p->kappaP_lte) ||
                 !std::isfinite(p->mu_lte)))
    return bad("LTE coefficients must be finite, kappa >= 0 and mu > 0");
  if (p->mg_levels < 1 || p->mg_levels > 12) return bad("mg_levels out of range");
  if (!is_pow2_div(p->nx, p->mg_levels) || !is_pow2_div(p->ny, p->mg_levels) ||
      !is_pow2_div(p->nz, p->mg_levels))
    return bad("grid sizes must be divisible by 2^(mg_levels-1) with an even coarsest size >= 4");
  const double N = (double)p->nx * p->ny * p->nz;
  if (N * (p->nspecies + 2) >= 2147483647.0) return bad("grid too large for 32-bit indexing");
  if (!(p->dx > 0) || !(p->theta > 0 && p->theta <= 1)) return bad("dx or theta invalid");
  if (!(p->u_e > 0) || !(p->u_E > 0)) return bad("unit scales must be positive");
  if (p->newton_maxit < 0 || p->newton_maxit > RT_MAX_NEWTON) return bad("newton_maxit out of range");
  if (p->pcg_maxit < 0 || p->mg_pre < 0 || p->mg_post < 0 || p->mg_coarse_sweeps < 1)
    return bad("negative solver counts");
  if (p->max_sources < 0) return bad("max_sources < 0");
  if (!(p->pcg_forcing >= 0.0) || !std::isfinite(p->pcg_forcing)) return bad("pcg_forcing must be finite and >= 0");
  if (p->limiter_mode != 0 && p->limiter_mode != 1) return bad("limiter_mode must be 0 or 1");
  if (p->limiter_lag != 0 && p->limiter_lag != 1) return bad("limiter_lag must be 0 or 1");
  if (p->krylov_restart < 0 || p->krylov_restart > KMAX - 2)
    return bad("krylov_restart out of range (0: PCG, 1..30: FGMRES restart length)");
  if (p->box_size < 0) return bad("box_size < 0");
  if (p->box_s_sweeps < 0 || p->box_s_sweeps > 256) return bad("box_s_sweeps out of range (0..256)");
  if (p->box_s_sweeps > 0 && p->krylov_restart == 0)
    return bad("box_s_sweeps needs FGMRES (krylov_restart > 0): the sweeps make the "
               "preconditioner non-symmetric");
  if (p->box_size > 0) {
    if (p->box_levels < 1 || p->box_levels > 12 || p->box_inner < 1 || p->box_coarse_sweeps < 0)
      return bad("box_levels out of range, box_inner < 1 or box_coarse_sweeps < 0");
    if (!is_pow2_div(p->box_size, p->box_levels))
      return bad("box_size must be divisible by 2^(box_levels-1) with an even coarsest size >= 4");
    if (p->box_size > p->nx || p->box_size > p->ny || p->box_size > p->nz)
      return bad("box_size larger than the grid");
  }
  return RT_OK;
}

// device parameters of a grid (the kernels' copy of rt_params)
void fill_params(const rt_params* p, DevParams& P) {
  P.nx = p->nx; P.ny = p->ny; P.nz = p->nz;
  P.ns = p->nspecies; P.nv = p->nspecies + 2; P.nb = p->nspecies + 1;
  P.kap_lte = p->kappa_lte; P.kapP_lte = p->kappaP_lte; P.mu_lte = p->mu_lte;
  P.bc = p->boundary;
  P.Eb = p->E_dirichlet;
  P.N = p->nx * p->ny * p->nz;
  P.iso = p->isothermal; P.lim_mode = p->limiter_mode;
  P.dx = p->dx; P.theta = p->theta; P.u_e = p->u_e; P.u_E = p->u_E;
  P.m = p->grey ? 1.0 : 0.0; P.y = p->y_he; P.T_iso = p->T_iso; P.D0 = p->D0;
  for (int s = 0; s < 3; ++s) {
    P.Kg[s] = p->K_gamma[s]; P.Kk[s] = p->K_kappa[s]; P.Kh[s] = p->K_heat[s];
  }
  if (p->nspecies == 1) {
    for (int s = 1; s < 3; ++s) P.Kg[s] = P.Kk[s] = P.Kh[s] = 0.0;
  }
  P.hnu = p->hnu_mean;
  P.alpha0[0] = 2.59e-13;                            // case-B HII at 1e4 K
  P.alpha0[1] = 2.72e-13;                            // HeII (placeholder datum)
  P.alpha0[2] = 2.0 * 2.59e-13 * std::pow(4.0, 0.7); // HeIII, hydrogenic Z = 2
}

// The finest level of the FP32 cycle is smoothed with pre- and post-sweeps
// (not handled by the coarsest-level solve): it is stored colour-split, and
// its last half-sweep writes the FP64 result directly.
bool fp32_fused(const rt_params* p) {
  return p->mg_fp32 && p->mg_levels > 1 && p->mg_pre > 0 && p->mg_post > 0;
}
// The same layout for the finest level of the FP64 cycle: its operator, right
// side and iterate are colour-split copies (the operator converted once per
// Newton iteration, the right side per application) and its last half-sweep
// writes the result in natural order
bool fp64_split(const rt_params* p) {
  return !p->mg_fp32 && p->mg_levels > 1 && p->mg_pre > 0 && p->mg_post > 0;
}

size_t carve(const rt_params* p, char* base, Workspace* w) {
  Carver c{base, 0, base == nullptr};
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  const int nv = p->nspecies + 2, nb = p->nspecies + 1;
  w->D = c.take<double>(3 * N);
  w->g = c.take<double>(nv * N);
  w->f = c.take<double>(nv * N);
  w->ft = c.take<double>(nv * N);
  w->Ut = c.take<double>(nv * N);
  w->ftM = c.take<double>(nb * N);
  w->W = c.take<double>(nb * N);
  w->diag = c.take<double>(N);
  w->fw = c.take<double>(3 * N);
  w->bw = c.take<double>(3 * N);
  w->pdiag = c.take<double>(N);
  w->cx = c.take<double>(3 * N);
  w->cy = w->cx ? w->cx + N : nullptr;
  w->cz = w->cx ? w->cx + 2 * N : nullptr;
  w->b = c.take<double>(N);
  w->om = c.take<double>(N);
  w->ph = c.take<double>(N);
  w->x = c.take<double>(N);
  w->r = c.take<double>(N);
  w->z = c.take<double>(N);
  w->p = c.take<double>(N);
  w->q = c.take<double>(N);
  {
    size_t sb = (size_t)stencil_blocks(p->nx, p->ny, p->nz);
    if (p->box_size > 0)   // the corrections' own dot partials follow the V-cycle's
      sb += (size_t)p->max_sources * stencil_blocks(p->box_size, p->box_size, p->box_size);
    w->nparts_cap = sb > (size_t)MAX_PARTS ? sb : (size_t)MAX_PARTS;
    w->parts = c.take<double>(w->nparts_cap * NCOMP_MAX);
  }
  w->sc = c.take<double>(32);
  if (p->krylov_restart > 0) {
    w->V = c.take<double>((size_t)(p->krylov_restart + 1) * N);
    w->Z = c.take<double>((size_t)p->krylov_restart * N);
  }
  w->gparts = c.take<double>((size_t)KMAX * MAX_PARTS);
  w->gh = c.take<double>(3 * KMAX);
  w->gy = c.take<double>(KMAX);
  w->src_cells = c.take<long long>(p->max_sources > 0 ? p->max_sources : 1);
  w->src_Q = c.take<double>(p->max_sources > 0 ? p->max_sources : 1);
  w->L64.clear();
  w->L32.clear();
  w->r32 = nullptr;
  int nx = p->nx, ny = p->ny, nz = p->nz;
  for (int l = 0; l < p->mg_levels; ++l) {
    const size_t n = (size_t)nx * ny * nz;
    if (!p->mg_fp32) {
      Level<double> L{nx, ny, nz};
      if (l == 0 && fp64_split(p)) {
        // colour-split copies of the preconditioner's operator, right side
        // and iterate
        L.diag = c.take<double>(n); L.cx = c.take<double>(n); L.cy = c.take<double>(n);
        L.cz = c.take<double>(n); L.x = c.take<double>(n); L.b = c.take<double>(n);
        L.r = c.take<double>(n);
        L.split = 1;
      } else if (l == 0) {
        // the V-cycle is built on the preconditioner's operator
        L.diag = w->pdiag; L.cx = w->cx; L.cy = w->cy; L.cz = w->cz;
        L.x = nullptr; L.b = nullptr;          // bound per application
        L.r = c.take<double>(n);
      } else {
        L.diag = c.take<double>(n); L.cx = c.take<double>(n); L.cy = c.take<double>(n);
        L.cz = c.take<double>(n); L.x = c.take<double>(n); L.b = c.take<double>(n);
        L.r = c.take<double>(n);
      }
      w->L64.push_back(L);
    } else {
      Level<float> L{nx, ny, nz};
      L.diag = c.take<float>(n); L.cx = c.take<float>(n); L.cy = c.take<float>(n);
      L.cz = c.take<float>(n); L.x = c.take<float>(n); L.b = c.take<float>(n);
      L.r = c.take<float>(n);
      L.split = (l == 0 && fp32_fused(p)) ? 1 : 0;
      w->L32.push_back(L);
    }
    nx /= 2; ny /= 2; nz /= 2;
  }
  w->B64.clear();
  w->B32.clear();
  w->box_cap = 0;
  if (p->box_size > 0 && p->max_sources > 0) {
    const int B = p->box_size;
    w->box_cap = p->max_sources;
    const size_t nb3 = (size_t)w->box_cap * B * B * B;
    w->bd = c.take<double>(nb3); w->bcx = c.take<double>(nb3);
    w->bcy = c.take<double>(nb3); w->bcz = c.take<double>(nb3);
    w->bxv = c.take<double>(nb3); w->br = c.take<double>(nb3);
    w->bz = c.take<double>(nb3); w->bp = c.take<double>(nb3); w->bq = c.take<double>(nb3);
    w->bp2 = c.take<double>(nb3); w->br2 = c.take<double>(nb3);
    const size_t sb = (size_t)stencil_blocks(w->box_cap * B, B, B);
    w->bparts = c.take<double>((sb > (size_t)MAX_PARTS ? sb : (size_t)MAX_PARTS) * NCOMP_MAX);
    w->bparts2 = c.take<double>((sb > (size_t)MAX_PARTS ? sb : (size_t)MAX_PARTS) * NCOMP_MAX);
    w->bsc = c.take<double>(32);
    // levels sized for every box; rt_set_sources sets the extent in use
    int bx = w->box_cap * B, by = B, bz = B;
    for (int l = 0; l < p->box_levels; ++l) {
      const size_t n = (size_t)bx * by * bz;
      if (!p->mg_fp32) {
        Level<double> L{bx, by, bz};
        if (l == 0) {
          L.diag = w->bd; L.cx = w->bcx; L.cy = w->bcy; L.cz = w->bcz;
          L.x = nullptr; L.b = nullptr;          // bound per application
          L.r = c.take<double>(n);
        } else {
          L.diag = c.take<double>(n); L.cx = c.take<double>(n); L.cy = c.take<double>(n);
          L.cz = c.take<double>(n); L.x = c.take<double>(n); L.b = c.take<double>(n);
          L.r = c.take<double>(n);
        }
        w->B64.push_back(L);
      } else {
        Level<float> L{bx, by, bz};
        L.diag = c.take<float>(n); L.cx = c.take<float>(n); L.cy = c.take<float>(n);
        L.cz = c.take<float>(n); L.x = c.take<float>(n); L.b = c.take<float>(n);
        L.r = c.take<float>(n);
        w->B32.push_back(L);
      }
      bx /= 2; by /= 2; bz /= 2;
    }
  }
  return c.off + ALIGN;
}

// extent of the box levels in use for nbox boxes (0: no subdomain correction)
void drop_box_graph(rt_grid* g) {
  for (auto& b : g->box_graphs)
    if (b.exec) (void)hipGraphExecDestroy(b.exec);   // nothing to report on release
  g->box_graphs.clear();
}

void set_box_extent(rt_grid* g, int nbox) {
  Workspace& w = g->w;
  g->nbox = (g->prm.box_size > 0 && nbox > 0 && nbox <= w.box_cap) ? nbox : 0;
  drop_box_graph(g);
  const int B = g->prm.box_size;
  const int blocks = g->nbox > 0 ? g->nbox : 1;   // the boxes are uncoupled
  for (size_t l = 0; l < w.B64.size(); ++l) {
    w.B64[l].nx = (g->nbox * B) >> l; w.B64[l].ny = B >> l; w.B64[l].nz = B >> l;
    w.B64[l].blocks = blocks;
  }
  for (size_t l = 0; l < w.B32.size(); ++l) {
    w.B32[l].nx = (g->nbox * B) >> l; w.B32[l].ny = B >> l; w.B32[l].nz = B >> l;
    w.B32[l].blocks = blocks;
  }
}

Step step_new(double dt, const rt_cosmo* c) { return Step{dt, c->a_new, c->H_new}; }

// ---------------------------------------------------------------------------
// multigrid
// cs: sweeps of the coarsest solve.  out64 (the colour-split finest level of
// the FP32 or FP64 cycle): the last smoothing launch writes the result, in
// FP64 and natural order, to this vector itself
// rd, qd, pd (a level in natural layout): the last smoothing launch also
// leaves the block partials of x.rd and x.qd in pd
template <class T>
void vcycle(rt_grid* g, std::vector<Level<T>>& Ls, int l, int cs, double* out64 = nullptr,
            const double* r64 = nullptr, const double* q64 = nullptr, double* parts = nullptr,
            const T* rd = nullptr, const T* qd = nullptr, double* pd = nullptr,
            bool first_done = false) {
  const rt_params& p = g->prm;
  hipStream_t st = g->st;
  Level<T>& L = Ls[l];
  const bool coarsest = (l + 1 == (int)Ls.size());
  const int kc = l == 0 ? RT_K_RBGS_FINE : RT_K_RBGS_COARSE;
  const long n = (long)L.nx * L.ny * L.nz;
  // algorithmic bytes, per field of this level: a half-sweep reads the three
  // coupling arrays (the - faces of a cell are stored at the other colour's
  // cells), the diagonal and right side of its colour and the other colour's
  // x, and writes its colour's x: 5 fields.  The first pair from x = 0 and a
  // coarsest solve read the operator and right side once and write x: 6
  const double F = (double)sizeof(T) * n;
  if (coarsest && L.nx % L.blocks == 0 && n / L.blocks <= COARSE_LDS_MAX) {
    TKB(g, kc, 6.0 * F, launch_coarse_solve_lds<T>(L, cs, st));
    return;
  }
  if (coarsest && n <= COARSE_SOLVE_MAX) {
    TKB(g, kc, 6.0 * F, launch_coarse_solve<T>(L, cs, st));
    return;
  }
  const int pre = coarsest ? cs : p.mg_pre;
  const int post = coarsest ? cs : p.mg_post;
  if (pre > 0) {
    // (red, black) from x = 0, unless a fused launch has already done it
    if (!first_done) TKB(g, kc, 6.0 * F, launch_rbgs_first_pair<T>(L, L.x, st));
    for (int s = 1; s < pre; ++s) {
      TKB(g, kc, 5.0 * F, launch_rbgs<T>(L, 0, st));
      TKB(g, kc, 5.0 * F, launch_rbgs<T>(L, 1, st));
    }
  } else {
    TKB(g, RT_K_OTHER, F, launch_fill<T>(n, L.x, T(0), st));
  }
  if (!coarsest) {
    // residual: operator (4), x, b in, r out; restriction: r in, coarse b out;
    // prolongation: coarse x in, the corrected cells of x in and out.  After
    // a pre-smoothing (which ends with the black half-sweep) only the red
    // cells have a residual: the residual reads the red cells' diag, b, x and
    // own couplings, the black cells' couplings and x, and writes the red r
    // (5.5 fields); the restriction reads the red r (0.5 + 0.125)
    const int ro = pre > 0 ? 1 : 0;
    TKB(g, RT_K_MG_TRANSFER, (ro ? 5.5 : 7.0) * F, launch_mg_residual<T>(L, ro, st));
    TKB(g, RT_K_MG_TRANSFER, (ro ? 0.625 : 1.125) * F, launch_restrict<T>(L, Ls[l + 1], ro, st));
    vcycle<T>(g, Ls, l + 1, cs);
    // the post-smoothing starts with black: only red cells need the correction
    TKB(g, RT_K_MG_TRANSFER, (post > 0 ? 1.125 : 2.125) * F,
        launch_prolong_add<T>(Ls[l + 1], L, post > 0 ? 0 : -1, st));
  }
  for (int s = 0; s < post; ++s) {
    TKB(g, kc, 5.0 * F, launch_rbgs<T>(L, 1, st));
    if (out64 && s + 1 == post) {
      // no x write: both colours go widened to out64 (8 B), and with the dot
      // partials r64 and q64 are read (16 B)
      TKB(g, kc, 4.5 * F + (8.0 + (parts ? 16.0 : 0.0)) * n,
          launch_rbgs_out64<T>(L, 0, out64, r64, q64, parts, st));
    } else if (pd && s + 1 == post) {
      TKB(g, kc, 7.0 * F, launch_rbgs_dots<T>(L, 0, rd, qd, pd, st));
    } else {
      TKB(g, kc, 5.0 * F, launch_rbgs<T>(L, 0, st));
    }
  }
}

int build_hierarchy(rt_grid* g) {
  if (!g->mg_stale) return RT_OK;
  Workspace& w = g->w;
  const long N = g->P.N;
  if (!g->prm.mg_fp32) {
    Level<double>& L0 = w.L64[0];
    if (L0.split && !g->l0_fp32) {
      TK(g, RT_K_MG_SETUP, launch_cvt_split_d(L0, w.pdiag, L0.diag, g->st));
      TK(g, RT_K_MG_SETUP, launch_cvt_split_d(L0, w.cx, L0.cx, g->st));
      TK(g, RT_K_MG_SETUP, launch_cvt_split_d(L0, w.cy, L0.cy, g->st));
      TK(g, RT_K_MG_SETUP, launch_cvt_split_d(L0, w.cz, L0.cz, g->st));
      g->l0_fp32 = true;
    }
    for (size_t l = 1; l < w.L64.size(); ++l) TK(g, RT_K_MG_SETUP, launch_coarsen<double>(w.L64[l - 1], w.L64[l], g->st));
  } else {
    Level<float>& L0 = w.L32[0];
    if (!g->l0_fp32) {
      TK(g, RT_K_MG_SETUP, launch_cvt_d2f_level(L0, w.pdiag, L0.diag, g->st));
      TK(g, RT_K_MG_SETUP, launch_cvt_d2f_level(L0, w.cx, L0.cx, g->st));
      TK(g, RT_K_MG_SETUP, launch_cvt_d2f_level(L0, w.cy, L0.cy, g->st));
      TK(g, RT_K_MG_SETUP, launch_cvt_d2f_level(L0, w.cz, L0.cz, g->st));
      g->l0_fp32 = true;
    }
    for (size_t l = 1; l < w.L32.size(); ++l) TK(g, RT_K_MG_SETUP, launch_coarsen<float>(w.L32[l - 1], w.L32[l], g->st));
  }
  if (g->nbox > 0) {
    // the operator restricted to the source boxes, and its hierarchy
    const int B = g->prm.box_size;
    const long nb3 = (long)g->nbox * B * B * B;
    TK(g, RT_K_MG_SETUP, launch_box_extract(g->P.nx, g->P.ny, g->P.nz, B, g->nbox, w.src_cells,
                                            w.pdiag, w.cx, w.cy, w.cz, w.bd, w.bcx, w.bcy, w.bcz,
                                            g->st));
    if (!g->prm.mg_fp32) {
      for (size_t l = 1; l < w.B64.size(); ++l) TK(g, RT_K_MG_SETUP, launch_coarsen<double>(w.B64[l - 1], w.B64[l], g->st));
    } else {
      Level<float>& L0 = w.B32[0];
      TK(g, RT_K_MG_SETUP, launch_cvt_d2f(nb3, w.bd, L0.diag, g->st));
      TK(g, RT_K_MG_SETUP, launch_cvt_d2f(nb3, w.bcx, L0.cx, g->st));
      TK(g, RT_K_MG_SETUP, launch_cvt_d2f(nb3, w.bcy, L0.cy, g->st));
      TK(g, RT_K_MG_SETUP, launch_cvt_d2f(nb3, w.bcz, L0.cz, g->st));
      for (size_t l = 1; l < w.B32.size(); ++l) TK(g, RT_K_MG_SETUP, launch_coarsen<float>(w.B32[l - 1], w.B32[l], g->st));
    }
  }
  g->mg_stale = false;
  HIPCHK(g, hipGetLastError());
  return RT_OK;
}

// z = V r on the current hierarchy.  With dots set, the FP32 cycle's last
// half-sweep also leaves the block partials of z.r and z.q (q = w.q) in
// w.parts and the call returns their count; otherwise it returns 0.
int apply_vcycle(rt_grid* g, const double* r, double* z, bool dots = false) {
  Workspace& w = g->w;
  const long N = g->P.N;
  if (!g->prm.mg_fp32) {
    Level<double>& L0 = w.L64[0];
    if (L0.split) {
      // r into the colour-split right side; the last half-sweep writes z
      TKB(g, RT_K_MG_TRANSFER, 16.0 * N, launch_cvt_split_d(L0, r, L0.b, g->st));
      vcycle<double>(g, w.L64, 0, g->prm.mg_coarse_sweeps, z);
      return 0;
    }
    L0.b = const_cast<double*>(r);
    L0.x = z;
    vcycle<double>(g, w.L64, 0, g->prm.mg_coarse_sweeps);
    return 0;
  }
  Level<float>& L0 = w.L32[0];
  if (fp32_fused(&g->prm)) {
    // r is converted (into the colour-split layout) by a pass of its own:
    // read at seven points by the first pair, FP64 r costs more than it saves.
    // The CG's own residual arrives converted by its update.
    if (g->r32_of != r) TKB(g, RT_K_MG_TRANSFER, 12.0 * N, launch_cvt_d2f_level(L0, r, L0.b, g->st));
    g->r32_of = r == w.r ? r : nullptr;
    if (dots) {
      vcycle<float>(g, w.L32, 0, g->prm.mg_coarse_sweeps, z, r, w.q, w.parts);
      return stencil_blocks(L0.nx, L0.ny, L0.nz / 2);
    }
    vcycle<float>(g, w.L32, 0, g->prm.mg_coarse_sweeps, z);
    return 0;
  }
  TKB(g, RT_K_MG_TRANSFER, 12.0 * N, launch_cvt_d2f(N, r, L0.b, g->st));
  vcycle<float>(g, w.L32, 0, g->prm.mg_coarse_sweeps);
  TKB(g, RT_K_MG_TRANSFER, 12.0 * N, launch_cvt_f2d(N, L0.x, z, g->st));
  return 0;
}

int box_cs(const rt_grid* g) {
  return g->prm.box_coarse_sweeps > 0 ? g->prm.box_coarse_sweeps : g->prm.mg_coarse_sweeps;
}

template <class T> std::vector<Level<T>>& box_hier(Workspace& w);
template <> std::vector<Level<double>>& box_hier<double>(Workspace& w) { return w.B64; }
template <> std::vector<Level<float>>& box_hier<float>(Workspace& w) { return w.B32; }

// Source-subdomain correction after the V-cycle: z += the boxes' part of an
// approximate solution of the box operator with right side r - S z (the
// residual the V-cycle left) on the boxes, namely box_inner iterations of
// flexible PCG from zero with the box V-cycle, all in T (the V-cycle's
// type; FP64 dots).  The iterations run without host read-back, so the whole
// sequence is fixed and can be captured.
// dots > 0: the V-cycle left that many partials of z.r and z.q (q = w.q) in
// w.parts; the scatter appends those of the correction
template <class T>
void box_correct_t(rt_grid* g, const double* r, double* z, int dots) {
  Workspace& w = g->w;
  hipStream_t st = g->st;
  const int B = g->prm.box_size;
  std::vector<Level<T>>& Ls = box_hier<T>(w);
  Level<T>& L0 = Ls[0];
  const long n = (long)L0.nx * L0.ny * L0.nz;
  T* x = reinterpret_cast<T*>(w.bxv);
  T* br = reinterpret_cast<T*>(w.br);
  T* bz = reinterpret_cast<T*>(w.bz);
  T* bp = reinterpret_cast<T*>(w.bp);
  T* bq = reinterpret_cast<T*>(w.bq);
  g->tk_override = RT_K_BOX;
  const double F = (double)sizeof(T) * n;   // one field over the stacked boxes
  // r - S z on the box cells: the FP64 operator (4), r and z in, T out
  TKB(g, RT_K_BOX, 48.0 * n + F,
      launch_box_residual<T>(g->P.nx, g->P.ny, g->P.nz, B, g->nbox, w.src_cells, w.pdiag, w.cx,
                             w.cy, w.cz, r, z, br, st));
  TKB(g, RT_K_BOX, F, launch_fill<T>(n, x, T(0), st));
  L0.b = br;   // the box V-cycle maps r -> z in place
  L0.x = bz;
  vcycle<T>(g, Ls, 0, box_cs(g));
  int np = 0;
  TKB(g, RT_K_BOX, 3.0 * F, np = launch_box_dot1p<T>(n, br, bz, bp, w.bparts, st));
  TK(g, RT_K_BOX, launch_final_reduce(w.bparts, np, 1, w.bsc + S_RHO, st));
  // the CG scalars are formed by the kernels that use them (each block sums
  // the partials itself), rho alternates between two slots and p between two
  // buffers, so an iteration is the product, the update and the V-cycle,
  // whose last half-sweep forms the dots: no reduction launches
  T* pb[2] = {reinterpret_cast<T*>(w.bp2), bp};
  // the box V-cycle's last half-sweep forms z.r and z.q (it exists when the
  // box level is not the coarsest and post-smooths)
  const bool fuse_dots = Ls.size() > 1 && g->prm.mg_post > 0;
  int nzp = 0;
  // the update before each box V-cycle runs inside its first (red, black)
  // pair (when the cycle pre-smooths and is not a coarsest solve); r then
  // alternates between two buffers
  const bool fuse_first = Ls.size() > 1 && g->prm.mg_pre > 0;
  T* rb[2] = {br, reinterpret_cast<T*>(w.br2)};
  int ri = 0;
  // every block of the product and of the update sums all block partials of
  // the kernel before it (blocks x partials reads); with many boxes one
  // launch reduces them first, into box scalar slots laid out as a single
  // partial, and the kernels read that one
  auto once = [&](double* parts, int np_, int ncomp, int slot) -> std::pair<const double*, int> {
    if (np_ <= BOX_INLINE_PARTS) return {parts, np_};
    TK(g, RT_K_BOX, launch_final_reduce(parts, np_, ncomp, w.bsc + slot, st));
    return {w.bsc + slot, 1};
  };
  for (int it = 1; it <= g->prm.box_inner; ++it) {
    const int rho = (it & 1) ? S_RHO : S_RHO2, rho_prev = (it & 1) ? S_RHO2 : S_RHO;
    T* p = pb[it & 1];
    const T* p_prev = pb[(it + 1) & 1];
    // operator (4), z, p_prev in; p, q out
    const std::pair<const double*, int> zp =
        it == 1 ? std::pair<const double*, int>{w.bparts, 0} : once(w.bparts, nzp, 2, BOX_SLOT_ZPARTS);
    TKB(g, RT_K_BOX, (it == 1 ? 7.0 : 8.0) * F,
        np = launch_box_spmv_p<T>(L0, bz, p_prev, p, bq, zp.first, zp.second, w.bsc, rho_prev,
                                  rho, it == 1, w.bparts2, st));
    const std::pair<const double*, int> pq = once(w.bparts2, np, 1, BOX_SLOT_PQPARTS);
    const bool last = it == g->prm.box_inner;
    if (last || !fuse_first) {
      TKB(g, RT_K_BOX, 6.0 * F,
          launch_box_update_xr<T>(n, x, rb[ri], p, bq, pq.first, pq.second, w.bsc, rho, st));
      if (last) break;
    } else {
      // x, p, q, r in, x, the new r and the pair's z out, the operator (4)
      TKB(g, RT_K_BOX, 11.0 * F,
          launch_box_update_first_pair<T>(L0, x, rb[ri], rb[ri ^ 1], p, bq, pq.first, pq.second,
                                          w.bsc, rho, st));
      ri ^= 1;
    }
    T* r = rb[ri];
    L0.b = r;
    if (fuse_dots) {
      vcycle<T>(g, Ls, 0, box_cs(g), nullptr, nullptr, nullptr, nullptr, r, bq, w.bparts, fuse_first);
      nzp = stencil_blocks(L0.nx, L0.ny, L0.nz / 2);
    } else {
      vcycle<T>(g, Ls, 0, box_cs(g), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                fuse_first);
      TKB(g, RT_K_BOX, 3.0 * F, nzp = launch_box_dot2<T>(n, bz, r, bq, w.bparts, st));
    }
  }
  L0.b = br;
  // boxes may overlap: one launch per box, in source order
  const int nbb = stencil_blocks(B, B, B);
  // per box: its part of y in, z in and out, with the dots r and q in
  const double Fb = (double)B * B * B;
  for (int s = 0; s < g->nbox; ++s)
    TKB(g, RT_K_BOX, Fb * (sizeof(T) + 16.0 + (dots > 0 ? 16.0 : 0.0)),
        launch_box_scatter_add<T>(g->P.nx, g->P.ny, g->P.nz, B, g->nbox, w.src_cells, s, x, z, r,
                                  w.q,
                                  dots > 0 ? w.parts + (size_t)(dots + s * nbb) * NCOMP_MAX
                                           : nullptr,
                                  st));
  // red-black sweeps on S itself over each box, box by box in source order;
  // a box below BOX_S_LDS_MAX and the grid size takes all its sweeps in one
  // on-chip launch (diag, fw, bw, r in, z in and out once), a larger one a
  // launch per half-sweep (the box's diag, fw, bw, r and z cells each time)
  const bool s_lds = B <= BOX_S_LDS_MAX && B < g->P.nx && B < g->P.ny && B < g->P.nz;
  for (int s = 0; s < g->nbox && g->prm.box_s_sweeps > 0; ++s) {
    if (s_lds) {
      TKB(g, RT_K_BOX, Fb * 8.0 * 10.0,
          launch_box_smooth_s_lds(g->P.nx, g->P.ny, g->P.nz, B, g->nbox, w.src_cells, s,
                                  g->prm.box_s_sweeps, w.diag, w.fw, w.bw, r, z, st));
      continue;
    }
    for (int k = 0; k < g->prm.box_s_sweeps; ++k)
      for (int colour = 0; colour < 2; ++colour)
        TKB(g, RT_K_BOX, Fb * 8.0 * 5.0,
            launch_box_smooth_s(g->P.nx, g->P.ny, g->P.nz, B, g->nbox, w.src_cells, s, colour,
                                w.diag, w.fw, w.bw, r, z, st));
  }
  g->tk_override = -1;
}

void box_correct_launches(rt_grid* g, const double* r, double* z, int dots) {
  if (g->prm.mg_fp32) box_correct_t<float>(g, r, z, dots);
  else box_correct_t<double>(g, r, z, dots);
}

// capture the correction for (r, z, dots) on a private stream (the caller's
// stream may be the null stream, which cannot be captured); nothing runs
// meanwhile
int capture_box(rt_grid* g, rt_grid::BoxGraph& bg, const double* r, double* z, int dots) {
  if (bg.exec) (void)hipGraphExecDestroy(bg.exec);   // nothing to report on release
  bg.exec = nullptr;
  if (!g->cap_st) HIPCHK(g, hipStreamCreateWithFlags(&g->cap_st, hipStreamNonBlocking));
  hipStream_t caller = g->st;
  const bool timing = g->tm.on;
  g->tm.on = false;   // no event records inside the graph
  g->st = g->cap_st;
  g->capturing = true;
  g->cap_bytes = 0.0;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(g->st, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    box_correct_launches(g, r, z, dots);
    e = hipStreamEndCapture(g->st, &graph);
  }
  g->capturing = false;
  g->st = caller;
  g->tm.on = timing;
  if (e == hipSuccess) e = hipGraphInstantiate(&bg.exec, graph, nullptr, nullptr, 0);
  if (graph) {
    const hipError_t e2 = hipGraphDestroy(graph);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess) {
    if (bg.exec) (void)hipGraphExecDestroy(bg.exec);
    bg.exec = nullptr;
    return fail(g, RT_EDEVICE, "capturing the subdomain correction: %s", hipGetErrorString(e));
  }
  bg.r = r;
  bg.z = z;
  bg.nbox = g->nbox;
  bg.dots = dots;
  bg.bytes = g->cap_bytes;
  return RT_OK;
}

// one replay of the captured graph (timed as one launch), or with graphs
// off the launches one by one
int box_correct(rt_grid* g, const double* r, double* z, int dots) {
  if (!g->graphs) {
    box_correct_launches(g, r, z, dots);
    return RT_OK;
  }
  rt_grid::BoxGraph* hit = nullptr;
  for (auto& b : g->box_graphs)
    if (b.exec && b.r == r && b.z == z && b.nbox == g->nbox && b.dots == dots) hit = &b;
  if (!hit) {
    // at most one graph per FGMRES basis vector and dot variant
    if (g->box_graphs.size() >= (size_t)(2 * KMAX + 4)) drop_box_graph(g);
    g->box_graphs.emplace_back();
    const int rc = capture_box(g, g->box_graphs.back(), r, z, dots);
    if (rc != RT_OK) {
      g->box_graphs.pop_back();
      return rc;
    }
    hit = &g->box_graphs.back();
  }
  rt_grid::BoxGraph& bg = *hit;
  hipError_t e = hipSuccess;
  TKB(g, RT_K_BOX, bg.bytes, e = hipGraphLaunch(bg.exec, g->st));
  HIPCHK(g, e);
  return RT_OK;
}

// the CG preconditioner: the V-cycle, plus the source-subdomain correction
// when one is configured.  *nd: the number of partials of z.r and z.q the
// application left in w.parts (the FP32 cycle forms them when dots is set;
// the correction then adds its own), else 0
int apply_precond(rt_grid* g, const double* r, double* z, bool dots, int* nd) {
  const int nv = apply_vcycle(g, r, z, dots);
  if (g->nbox == 0) {
    *nd = nv;
    return RT_OK;
  }
  *nd = nv > 0 ? nv + g->nbox * stencil_blocks(g->prm.box_size, g->prm.box_size, g->prm.box_size)
               : 0;
  return box_correct(g, r, z, nv);
}

int read_scalars(rt_grid* g, const double* d, double* h, int n) {
  HIPCHK(g, hipMemcpyAsync(h, d, n * sizeof(double), hipMemcpyDeviceToHost, g->st));
  HIPCHK(g, hipStreamSynchronize(g->st));
  return RT_OK;
}

// reduce `ncomp` partials of the last reduction kernel into sc[slot...]
void finish_reduce(rt_grid* g, int n_items_blocks, int ncomp, int slot) {
  TK(g, RT_K_REDUCE, launch_final_reduce(g->w.parts, n_items_blocks, ncomp, g->w.sc + slot, g->st));
}

// PCG on the preconditioner's operator (pdiag, c): solves S x = b when S is
// that symmetric operator (constant limiter D0, no species opacity terms)
// stops at ||r||_2 <= max(rtol ||b||_2, atol)
int pcg(rt_grid* g, const double* b, double* x, double rtol, double atol, int maxit, int* iters,
        double* relres, int* vcycles) {
  Workspace& w = g->w;
  const long N = g->P.N;
  const int nparts = reduce_blocks(N);
  RTCHK(build_hierarchy(g));
  double h[2];
  const double F = 8.0 * N;
  TKB(g, RT_K_CG_VECTOR, 2.0 * F, launch_dot1(N, b, b, w.parts, g->st, w.r));   // and r = b
  g->r32_of = nullptr;
  finish_reduce(g, nparts, 1, S_BB);
  RTCHK(read_scalars(g, w.sc + S_BB, h, 1));
  const double bn = std::sqrt(h[0]);
  const double thr = std::max(rtol * bn, atol);
  TKB(g, RT_K_CG_VECTOR, F, launch_fill<double>(N, x, 0.0, g->st));
  *iters = 0;
  *relres = 0.0;
  if (!(bn > 0.0)) {
    if (!std::isfinite(bn)) return fail(g, RT_ENONFINITE, "non-finite Schur right side");
    HIPCHK(g, hipGetLastError());
    return RT_OK;
  }
  int nd = 0;
  RTCHK(apply_precond(g, w.r, w.z, false, &nd));
  ++*vcycles;
  TKB(g, RT_K_CG_VECTOR, 3.0 * F, launch_dot1(N, w.r, w.z, w.parts, g->st, w.p));   // and p = z
  finish_reduce(g, nparts, 1, S_RHO);
  // The tail of an iteration (V-cycle, dots, new direction) writes only z, p
  // and CG scalars, so it can be enqueued before this iteration's residual
  // norm has come back to the host: the device then never idles on the
  // read-back.  If that norm turns out converged, the enqueued tail (a whole
  // preconditioner application) is discarded work, while waiting for the norm
  // costs only the read-back latency.  So the tail runs ahead only when the
  // norm predicted from the last reduction factor (for the first step: the
  // first step of the previous solve) stays well above the tolerance.
  constexpr double LOOKAHEAD = 4.0;
  auto tail = [&]() -> int {
    RTCHK(apply_precond(g, w.r, w.z, true, &nd));
    ++*vcycles;
    if (nd == 0) TKB(g, RT_K_CG_VECTOR, 3.0 * F, launch_dot2(N, w.z, w.r, w.q, w.parts, g->st));
    TK(g, RT_K_REDUCE, launch_final_reduce_beta(w.parts, nd > 0 ? nd : nparts, w.sc, g->st));
    TKB(g, RT_K_CG_VECTOR, 3.0 * F, launch_update_p(N, w.p, w.z, w.sc, g->st));
    return RT_OK;
  };
  double rn = bn, rn_prev = 0.0;
  int k = 0;
  for (k = 1; k <= maxit; ++k) {
    const double pred = k > 1 ? rn * (rn / rn_prev) : (g->cg_rate1 > 0.0 ? bn * g->cg_rate1 : HUGE_VAL);
    TKB(g, RT_K_SPMV, 6.0 * F,
        launch_spmv_dot(g->P.nx, g->P.ny, g->P.nz, w.pdiag, w.cx, w.cy, w.cz, w.p, w.q, w.parts,
                        g->st));
    TK(g, RT_K_REDUCE, launch_final_reduce_alpha(w.parts, stencil_blocks(g->P.nx, g->P.ny, g->P.nz),
                                                 w.sc, g->st));
    if (fp32_fused(&g->prm)) {
      TKB(g, RT_K_CG_VECTOR, 6.5 * F,
          launch_update_xr(N, x, w.r, w.p, w.q, w.sc, w.parts, g->st, w.L32[0].b, g->P.ny,
                           g->P.nz));
      g->r32_of = w.r;
    } else {
      TKB(g, RT_K_CG_VECTOR, 6.0 * F, launch_update_xr(N, x, w.r, w.p, w.q, w.sc, w.parts, g->st));
    }
    finish_reduce(g, nparts, 1, S_RR);
    HIPCHK(g, hipMemcpyAsync(g->hpin, w.sc + S_RR, sizeof(double), hipMemcpyDeviceToHost, g->st));
    HIPCHK(g, hipEventRecord(g->ev_rd, g->st));
    const bool ahead = k < maxit && pred > LOOKAHEAD * thr;
    if (ahead) RTCHK(tail());
    HIPCHK(g, hipEventSynchronize(g->ev_rd));
    rn_prev = rn;
    rn = std::sqrt(g->hpin[0]);
    if (!std::isfinite(rn)) return fail(g, RT_ENONFINITE, "non-finite CG residual");
    if (k == 1) g->cg_rate1 = rn / bn;
    if (rn <= thr) break;
    if (k == maxit) break;
    if (!ahead) RTCHK(tail());
  }
  *iters = k > maxit ? maxit : k;
  *relres = rn / bn;
  HIPCHK(g, hipGetLastError());
  return RT_OK;
}

// second Gram-Schmidt pass when the projection leaves less than this
// fraction of the product's norm (a loss of two digits or more)
constexpr double REORTH = 0.01;

// Flexible GMRES(m) on the workspace Schur operator (diag, fw, bw), right-
// preconditioned by apply_precond (the V-cycle of the preconditioner's
// operator plus the subdomain correction), from x = 0.  Classical
// Gram-Schmidt in one fused pass (the product forms the dots), a second pass
// where the first cancelled two digits or more (||w'|| < REORTH ||w||), Givens
// rotations on the host; stops once the least-squares residual
// <= max(rtol ||b||_2, atol), after maxit iterations in all (rtol = atol = 0:
// exactly maxit), restarting every m.  The host reads j + 2 scalars per
// iteration (one more after a second pass).
int fgmres(rt_grid* g, const double* b, double* x, double rtol, double atol, int maxit,
           int* iters, double* relres, int* vcycles) {
  Workspace& w = g->w;
  const DevParams& P = g->P;
  const long N = P.N;
  const int m = g->prm.krylov_restart;
  const int nparts = reduce_blocks(N);
  RTCHK(build_hierarchy(g));
  double* hp = g->hpin;
  const double F = 8.0 * N;   // bytes of one FP64 field
  TKB(g, RT_K_CG_VECTOR, F, launch_dot1(N, b, b, w.parts, g->st));
  finish_reduce(g, nparts, 1, S_BB);
  RTCHK(read_scalars(g, w.sc + S_BB, hp, 1));
  const double bn = std::sqrt(hp[0]);
  const double thr = std::max(rtol * bn, atol);
  TKB(g, RT_K_CG_VECTOR, F, launch_fill<double>(N, x, 0.0, g->st));
  *iters = 0;
  *relres = 0.0;
  if (!(bn > 0.0)) {
    if (!std::isfinite(bn)) return fail(g, RT_ENONFINITE, "non-finite Schur right side");
    HIPCHK(g, hipGetLastError());
    return RT_OK;
  }
  // the preconditioner maps v_j to z_j directly (the subdomain correction
  // keeps one captured graph per pair); the normalisation also writes the
  // FP32 colour-split copy of v_j for the FP32 cycle
  float* r32 = fp32_fused(&g->prm) ? w.L32[0].b : nullptr;
  auto normalise = [&](double* v, double sf) {
    TKB(g, RT_K_CG_VECTOR, 2.0 * F + (r32 ? 0.5 * F : 0.0),
        launch_scale(N, v, sf, nullptr, r32, P.ny, P.nz, g->st));
    g->r32_of = r32 ? v : nullptr;
  };
  std::vector<double> H((size_t)m * (m + 1)), cs(m), sn(m), gv(m + 1), y(m);
  int its = 0;
  double est = bn;
  bool first = true;
  while (true) {
    double beta;
    if (first) {
      beta = bn;
      HIPCHK(g, hipMemcpyAsync(w.V, b, N * sizeof(double), hipMemcpyDeviceToDevice, g->st));
    } else {
      int nb = 0;
      TKB(g, RT_K_SPMV, 10.0 * F,
          nb = launch_spmv_full(P.nx, P.ny, P.nz, w.diag, w.fw, w.bw, x, b, w.V, nullptr, w.V, 0,
                                w.gparts, g->st));
      TK(g, RT_K_REDUCE, launch_final_multi(w.gparts, nb, 1, w.gh, g->st));
      RTCHK(read_scalars(g, w.gh, hp, 1));
      beta = std::sqrt(hp[0]);
      if (!std::isfinite(beta)) return fail(g, RT_ENONFINITE, "non-finite FGMRES residual");
      if (!(beta > 0.0)) { est = 0.0; break; }
    }
    normalise(w.V, 1.0 / beta);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    bool done = false;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = w.V + (size_t)j * N;
      double* vn = w.V + (size_t)(j + 1) * N;
      double* zj = w.Z + (size_t)j * N;
      int nd = 0;
      RTCHK(apply_precond(g, vj, zj, false, &nd));
      ++*vcycles;
      int nb = 0;
      TKB(g, RT_K_SPMV, (9.0 + (j + 1)) * F,
          nb = launch_spmv_full(P.nx, P.ny, P.nz, w.diag, w.fw, w.bw, zj, nullptr, vn, nullptr,
                                w.V, j + 1, w.gparts, g->st));
      TK(g, RT_K_REDUCE, launch_final_multi(w.gparts, nb, j + 2, w.gh, g->st));
      TKB(g, RT_K_CG_VECTOR, (j + 3.0) * F,
          nb = launch_gs_pass(N, vn, w.V, j + 1, w.gh, 1, w.gparts, g->st));
      TK(g, RT_K_REDUCE, launch_final_multi(w.gparts, nb, j + 2, w.gh + KMAX, g->st));
      HIPCHK(g, hipMemcpyAsync(hp, w.gh, 2 * KMAX * sizeof(double), hipMemcpyDeviceToHost, g->st));
      HIPCHK(g, hipStreamSynchronize(g->st));
      double* h = &H[(size_t)j * (m + 1)];
      for (int i = 0; i <= j; ++i) h[i] = hp[i];
      const double wn = std::sqrt(hp[j + 1]);
      double hn = std::sqrt(hp[KMAX + j + 1]);
      if (hn < REORTH * wn) {
        for (int i = 0; i <= j; ++i) h[i] += hp[KMAX + i];
        TKB(g, RT_K_CG_VECTOR, (j + 3.0) * F,
            nb = launch_gs_pass(N, vn, w.V, j + 1, w.gh + KMAX, 0, w.gparts, g->st));
        TK(g, RT_K_REDUCE, launch_final_multi(w.gparts, nb, 1, w.gh + 2 * KMAX, g->st));
        RTCHK(read_scalars(g, w.gh + 2 * KMAX, hp, 1));
        hn = std::sqrt(hp[0]);
      }
      if (!std::isfinite(hn)) return fail(g, RT_ENONFINITE, "non-finite FGMRES basis vector");
      h[j + 1] = hn;
      if (hn > 0.0) normalise(vn, 1.0 / hn);
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
      }
      const double den = std::sqrt(h[j] * h[j] + h[j + 1] * h[j + 1]);
      cs[j] = den > 0.0 ? h[j] / den : 1.0;
      sn[j] = den > 0.0 ? h[j + 1] / den : 0.0;
      h[j] = den;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      ++its;
      k = j + 1;
      est = std::fabs(gv[j + 1]);
      if (est <= thr || its >= maxit || hn == 0.0) {
        done = true;
        break;
      }
    }
    for (int i = k - 1; i >= 0; --i) {
      double t = gv[i];
      for (int l = i + 1; l < k; ++l) t -= H[(size_t)l * (m + 1) + i] * y[l];
      const double d = H[(size_t)i * (m + 1) + i];
      y[i] = d != 0.0 ? t / d : 0.0;
    }
    for (int i = 0; i < k; ++i) hp[i] = y[i];
    HIPCHK(g, hipMemcpyAsync(w.gy, hp, k * sizeof(double), hipMemcpyHostToDevice, g->st));
    TKB(g, RT_K_CG_VECTOR, (k + 2.0) * F, launch_combine(N, x, w.Z, k, w.gy, g->st));
    // the host buffer is reused by the next read-back: the copy must be done
    HIPCHK(g, hipStreamSynchronize(g->st));
    if (done) break;
    first = false;
  }
  *iters = its;
  *relres = est / bn;
  HIPCHK(g, hipGetLastError());
  return RT_OK;
}

// the Schur solve: FGMRES on the full operator, or (krylov_restart = 0) PCG
// on the symmetric preconditioner operator
int krylov(rt_grid* g, const double* b, double* x, double rtol, double atol, int maxit, int* iters,
           double* relres, int* vcycles) {
  if (g->prm.krylov_restart > 0) return fgmres(g, b, x, rtol, atol, maxit, iters, relres, vcycles);
  return pcg(g, b, x, rtol, atol, maxit, iters, relres, vcycles);
}

// face coefficients of the lagged-limiter reading (null: the limiter at the iterate)
const double* lagged_D(const rt_grid* g) { return g->prm.limiter_lag ? g->w.D : nullptr; }

int time_level(rt_grid* g, const double* Un, double dt, const rt_cosmo* c, double* gn) {
  const DevParams& P = g->P;
  // the limiter at U^n: for the explicit part, and for the whole step with
  // the lagged reading
  // faces: E and the fractions, n_H in, D (3) out; explicit part: U, n_H,
  // e_h, D in, g out
  if (P.theta != 1.0 || g->prm.limiter_lag)
    TKB(g, RT_K_TIMELEVEL, (P.nb + 4.0) * 8.0 * P.N,
        launch_faces(P, Un, g->nH, c->a_old, g->w.D, g->st));
  if (P.theta != 1.0) {
    TKB(g, RT_K_TIMELEVEL, (2.0 * P.nv + 5.0) * 8.0 * P.N,
        launch_explicit(P, Un, g->nH, g->eh, g->w.D, Step{dt, c->a_old, c->H_old}, gn, g->st));
  } else {
    HIPCHK(g, hipMemcpyAsync(gn, Un, (size_t)P.nv * P.N * sizeof(double),
                             hipMemcpyDeviceToDevice, g->st));
  }
  const double scale = dt * P.hnu / (P.dx * P.dx * P.dx);
  TK(g, RT_K_TIMELEVEL, launch_sources(g->w.src_cells, g->w.src_Q, g->nsrc, scale, gn + (size_t)(P.nv - 1) * P.N, g->st));
  g->have_tl = true;
  HIPCHK(g, hipGetLastError());
  return RT_OK;
}

// residual + norm; returns rms in *fn and violation count in *viol (sync)
int residual_norm(rt_grid* g, const double* U, const double* gn, Step s, double* f, double* fn,
                  double* viol) {
  const DevParams& P = g->P;
  TKB(g, RT_K_RESIDUAL, (3.0 * P.nv + 2.0 + (g->prm.limiter_lag ? 3.0 : 0.0)) * 8.0 * P.N,
      launch_residual(P, U, gn, g->nH, g->eh, lagged_D(g), s, f, g->w.parts, g->st));
  finish_reduce(g, stencil_blocks(P.nx, P.ny, P.nz), 2, S_FN);
  double h[2];
  RTCHK(read_scalars(g, g->w.sc + S_FN, h, 2));
  *fn = std::sqrt(h[0] / ((double)P.N * P.nv));
  *viol = h[1];
  return RT_OK;
}

int check_ready(rt_grid* g, bool need_tl = false) {
  if (!g) return RT_EINVAL;
  if (!g->nH || !g->eh) return fail(g, RT_EINVAL, "rt_set_medium has not been called");
  if (need_tl && g->prm.limiter_lag && !g->have_tl)
    return fail(g, RT_EINVAL, "limiter_lag: rt_time_level has not been called");
  return RT_OK;
}

// Schur assembly into the workspace operator (the local blocks, then the
// face terms); with the colour-split FP32 finest level the face kernel also
// writes that level's copy of the preconditioner's operator
void schur_into_workspace(rt_grid* g, const double* U, const double* f, Step s, double* b) {
  Workspace& w = g->w;
  const bool f32 = g->prm.mg_fp32 && !w.L32.empty() && w.L32[0].split;
  Level<float>* L0 = f32 ? &w.L32[0] : nullptr;
  launch_schur_local(g->P, U, f, g->nH, g->eh, s, w.ftM, w.W, w.diag, b, w.om, w.ph, g->st);
  launch_schur_faces(g->P, U, g->nH, lagged_D(g), s, w.diag, w.om, w.ph, w.diag, w.pdiag, w.cx,
                     w.fw, w.bw, b,
                     f32 ? L0->diag : nullptr, f32 ? L0->cx : nullptr, f32 ? L0->cy : nullptr,
                     f32 ? L0->cz : nullptr, g->st);
  g->l0_fp32 = f32;
  g->mg_stale = true;
  g->have_op = true;
}

}  // namespace

// ===========================================================================
// ---------------------------------------------------------------------------
// allocation-free residual: the block partials and the final sums of the
// residual norm live in a static device array instead of a grid's workspace.
// Every call on one GPU uses that GPU's copy; the reductions overwrite every
// slot they read (each block writes its partial, the final reduction its
// sums), so nothing has to start at zero.  Calls that overlap on one GPU race.

namespace {
constexpr long NOALLOC_MAX_BLOCKS = 1L << 19;   // the partials of a 512^3 grid
constexpr size_t NOALLOC_SUMS = (size_t)NOALLOC_MAX_BLOCKS * NCOMP_MAX;
constexpr size_t NOALLOC_DOUBLES = NOALLOC_SUMS + 32;
constexpr int NOALLOC_MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {

std::mutex scratch_mu;
double* scratch_ptr[NOALLOC_MAX_DEVICES] = {};

int noalloc_fail(char* err, size_t len, int code, const char* fmt, ...) {
  if (err && len > 0) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(err, len, fmt, ap);
    va_end(ap);
  }
  return code;
}

// the device address of the current device's copy of `scratch`, looked up
// once per device (the host-side name is not a device address)
int scratch_on_device(double** out, char* err, size_t len) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return noalloc_fail(err, len, RT_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return noalloc_fail(err, len, RT_EDEVICE, "device %d beyond the %d supported", dev,
                        NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return noalloc_fail(err, len, RT_EDEVICE, "hipGetSymbolAddress(scratch): %s",
                          hipGetErrorString(e));
    scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = scratch_ptr[dev];
  return RT_OK;
}

}  // namespace

extern "C" {

int rt_workspace_bytes(const rt_params* p, uint64_t* bytes) {
  std::string why;
  if (!bytes || validate(p, &why) != RT_OK) return RT_EINVAL;
  Workspace w;
  *bytes = carve(p, nullptr, &w);
  return RT_OK;
}

int rt_create_grid(const rt_params* p, void* d_ws, uint64_t ws_bytes, void* hip_stream,
                   rt_grid** out) {
  if (!out) return RT_EINVAL;
  *out = nullptr;
  std::string why;
  if (validate(p, &why) != RT_OK) return RT_EINVAL;
  Workspace tmp;
  const size_t need = carve(p, nullptr, &tmp);
  if (!d_ws || ws_bytes < need) return RT_EINVAL;
  char* base = reinterpret_cast<char*>(d_ws);
  base += (ALIGN - reinterpret_cast<uintptr_t>(base) % ALIGN) % ALIGN;
  rt_grid* g = new rt_grid();
  g->prm = *p;
  g->st = reinterpret_cast<hipStream_t>(hip_stream);
  carve(p, base, &g->w);
  fill_params(p, g->P);
  if (hipHostMalloc(reinterpret_cast<void**>(&g->hpin), 3 * KMAX * sizeof(double),
                    hipHostMallocDefault) !=
          hipSuccess ||
      hipEventCreateWithFlags(&g->ev_rd, hipEventDisableTiming) != hipSuccess) {
    if (g->hpin) (void)hipHostFree(g->hpin);
    delete g;
    return RT_EDEVICE;
  }
  *out = g;
  return RT_OK;
}

int rt_destroy_grid(rt_grid* g) {
  if (g) {
    for (hipEvent_t e : g->tm.pool) (void)hipEventDestroy(e);
    if (g->ev_rd) (void)hipEventDestroy(g->ev_rd);
    if (g->hpin) (void)hipHostFree(g->hpin);
    drop_box_graph(g);
    if (g->cap_st) (void)hipStreamDestroy(g->cap_st);
  }
  delete g;
  return RT_OK;
}

const char* rt_last_error(const rt_grid* g) { return g ? g->err.c_str() : "null grid"; }

int rt_set_medium(rt_grid* g, const double* d_nH, const double* d_eh) {
  if (!g) return RT_EINVAL;
  if (!d_nH || !d_eh) return fail(g, RT_EINVAL, "null medium pointer");
  g->nH = d_nH;
  g->eh = d_eh;
  g->have_tl = false;
  return RT_OK;
}

int rt_set_sources(rt_grid* g, int32_t n, const int64_t* h_cells, const double* h_Q) {
  if (!g) return RT_EINVAL;
  if (n < 0 || n > g->prm.max_sources) return fail(g, RT_EINVAL, "source count %d out of range", n);
  if (n > 0 && (!h_cells || !h_Q)) return fail(g, RT_EINVAL, "null source arrays");
  for (int i = 0; i < n; ++i) {
    if (h_cells[i] < 0 || h_cells[i] >= g->P.N)
      return fail(g, RT_EINVAL, "source cell %lld out of range", (long long)h_cells[i]);
    if (!std::isfinite(h_Q[i]) || h_Q[i] < 0) return fail(g, RT_EINVAL, "invalid source rate");
  }
  if (n > 0) {
    HIPCHK(g, hipMemcpyAsync(g->w.src_cells, h_cells, n * sizeof(long long),
                             hipMemcpyHostToDevice, g->st));
    HIPCHK(g, hipMemcpyAsync(g->w.src_Q, h_Q, n * sizeof(double), hipMemcpyHostToDevice, g->st));
    HIPCHK(g, hipStreamSynchronize(g->st));
  }
  g->nsrc = n;
  set_box_extent(g, n);
  g->mg_stale = true;
  g->have_tl = false;
  return RT_OK;
}

int rt_time_level(rt_grid* g, const double* d_Un, double dt, const rt_cosmo* c, double* d_gn) {
  RTCHK(check_ready(g));
  if (!d_Un || !d_gn || !c) return fail(g, RT_EINVAL, "null argument");
  return time_level(g, d_Un, dt, c, d_gn);
}

int rt_predict(rt_grid* g, const double* d_Un, double dt, const rt_cosmo* c, double* d_Upred) {
  RTCHK(check_ready(g));
  if (!d_Un || !d_Upred || !c) return fail(g, RT_EINVAL, "null argument");
  if (d_Upred == d_Un) return fail(g, RT_EINVAL, "d_Upred must not be d_Un");
  const DevParams& P = g->P;
  DevParams P0 = P;
  P0.theta = 0.0;   // the explicit part of a theta = 0 step is the forward Euler update
  TK(g, RT_K_TIMELEVEL, launch_faces(P, d_Un, g->nH, c->a_old, g->w.D, g->st));
  TK(g, RT_K_TIMELEVEL, launch_explicit(P0, d_Un, g->nH, g->eh, g->w.D, Step{dt, c->a_old, c->H_old},
                                        d_Upred, g->st));
  const double scale = dt * P.hnu / (P.dx * P.dx * P.dx);
  TK(g, RT_K_TIMELEVEL, launch_sources(g->w.src_cells, g->w.src_Q, g->nsrc, scale,
                                       d_Upred + (size_t)(P.nv - 1) * P.N, g->st));
  TK(g, RT_K_TIMELEVEL, launch_predict_project(P, d_Un, g->eh, d_Upred, g->st));
  HIPCHK(g, hipGetLastError());
  return RT_OK;
}

int rt_time_error(rt_grid* g, const double* d_Unew, const double* d_Upred, double p, double* h_eps) {
  if (!g) return RT_EINVAL;
  if (!d_Unew || !d_Upred || !h_eps) return fail(g, RT_EINVAL, "null argument");
  if (!std::isfinite(p)) return fail(g, RT_EINVAL, "p must be finite (p <= 0: max norm)");
  const DevParams& P = g->P;
  int nb = 0;
  TK(g, RT_K_REDUCE, nb = launch_time_error(P, d_Unew, d_Upred, p, g->w.parts, g->st));
  TK(g, RT_K_REDUCE, launch_final_summax(g->w.parts, nb, g->w.sc + S_TSUM, g->st));
  double h[2];
  RTCHK(read_scalars(g, g->w.sc + S_TSUM, h, 2));
  *h_eps = p > 0.0 ? std::pow(h[0] / ((double)P.N * P.nv), 1.0 / p) : h[1];
  if (!std::isfinite(*h_eps)) return fail(g, RT_ENONFINITE, "non-finite time-error estimate");
  return RT_OK;
}

int rt_eval_residual(rt_grid* g, const double* d_U, const double* d_gn, double dt,
                     const rt_cosmo* c, double* d_f, double* h_rms) {
  RTCHK(check_ready(g, true));
  if (!d_U || !d_gn || !d_f || !c) return fail(g, RT_EINVAL, "null argument");
  if (h_rms) {
    double viol;
    RTCHK(residual_norm(g, d_U, d_gn, step_new(dt, c), d_f, h_rms, &viol));
  } else {
    launch_residual(g->P, d_U, d_gn, g->nH, g->eh, lagged_D(g), step_new(dt, c), d_f, g->w.parts,
                    g->st);
  }
  HIPCHK(g, hipGetLastError());
  return RT_OK;
}

int rt_eval_residual_noalloc(const rt_params* p, const double* d_nH, const double* d_eh,
                             const double* d_U, const double* d_gn, double dt, const rt_cosmo* c,
                             void* hip_stream, double* d_f, double* h_rms, char* err,
                             size_t err_len) {
  std::string why;
  if (validate(p, &why) != RT_OK)
    return noalloc_fail(err, err_len, RT_EINVAL, "invalid parameters: %s", why.c_str());
  if (p->limiter_lag)
    return noalloc_fail(err, err_len, RT_EINVAL,
                        "limiter_lag = 1 needs a grid's time-level face coefficients "
                        "(rt_time_level, rt_eval_residual)");
  const long blocks = stencil_blocks(p->nx, p->ny, p->nz);
  if (blocks > NOALLOC_MAX_BLOCKS)
    return noalloc_fail(err, err_len, RT_EINVAL,
                        "grid %dx%dx%d needs %ld partial sums; the static scratch holds %ld "
                        "(grids up to 512^3 cells)",
                        p->nx, p->ny, p->nz, blocks, NOALLOC_MAX_BLOCKS);
  if (!d_nH || !d_eh || !d_U || !d_gn || !d_f || !c)
    return noalloc_fail(err, err_len, RT_EINVAL, "null argument");
  double* scr = nullptr;
  RTCHK(scratch_on_device(&scr, err, err_len));
  DevParams P;
  fill_params(p, P);
  const hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  launch_residual(P, d_U, d_gn, d_nH, d_eh, nullptr, Step{dt, c->a_new, c->H_new}, d_f, scr, st);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && h_rms) {
    launch_final_reduce(scr, (int)blocks, 2, scr + NOALLOC_SUMS, st);
    double h[2] = {0.0, 0.0};
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h, scr + NOALLOC_SUMS, 2 * sizeof(double),
                                            hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) *h_rms = std::sqrt(h[0] / ((double)P.N * P.nv));
  }
  if (e != hipSuccess) return noalloc_fail(err, err_len, RT_EDEVICE, "HIP: %s", hipGetErrorString(e));
  return RT_OK;
}

int rt_local_jacobian(rt_grid* g, const double* d_U, double dt, const rt_cosmo* c, double* d_M,
                      double* d_Ucol, double* d_Lrow, double* d_dloc) {
  RTCHK(check_ready(g));
  if (!d_U || !d_M || !d_Ucol || !d_Lrow || !d_dloc || !c)
    return fail(g, RT_EINVAL, "null argument");
  launch_local_jac(g->P, d_U, g->nH, g->eh, step_new(dt, c), d_M, d_Ucol, d_Lrow, d_dloc, g->st);
  HIPCHK(g, hipGetLastError());
  return RT_OK;
}

int rt_schur_form(rt_grid* g, const double* d_U, const double* d_f, double dt, const rt_cosmo* c,
                  double* d_b) {
  RTCHK(check_ready(g, true));
  if (!d_U || !d_f || !d_b || !c) return fail(g, RT_EINVAL, "null argument");
  schur_into_workspace(g, d_U, d_f, step_new(dt, c), d_b);
  HIPCHK(g, hipGetLastError());
  return RT_OK;
}

int rt_schur_get(rt_grid* g, double* d_ftM, double* d_W, double* d_diag, double* d_cx,
                 double* d_cy, double* d_cz) {
  if (!g) return RT_EINVAL;
  if (!g->have_op) return fail(g, RT_EINVAL, "no Schur matrix yet");
  const size_t N = g->P.N, nb = g->P.nb;
  Workspace& w = g->w;
  auto cp = [&](double* dst, const double* src, size_t n) -> int {
    if (dst) HIPCHK(g, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, g->st));
    return RT_OK;
  };
  RTCHK(cp(d_ftM, w.ftM, nb * N));
  RTCHK(cp(d_W, w.W, nb * N));
  RTCHK(cp(d_diag, w.diag, N));
  RTCHK(cp(d_cx, w.cx, N));
  RTCHK(cp(d_cy, w.cy, N));
  RTCHK(cp(d_cz, w.cz, N));
  return RT_OK;
}

int rt_schur_get_full(rt_grid* g, double* d_fw, double* d_bw, double* d_pdiag) {
  if (!g) return RT_EINVAL;
  if (!g->have_op) return fail(g, RT_EINVAL, "no Schur matrix yet");
  const size_t N = g->P.N;
  Workspace& w = g->w;
  if (d_fw) HIPCHK(g, hipMemcpyAsync(d_fw, w.fw, 3 * N * 8, hipMemcpyDeviceToDevice, g->st));
  if (d_bw) HIPCHK(g, hipMemcpyAsync(d_bw, w.bw, 3 * N * 8, hipMemcpyDeviceToDevice, g->st));
  if (d_pdiag) HIPCHK(g, hipMemcpyAsync(d_pdiag, w.pdiag, N * 8, hipMemcpyDeviceToDevice, g->st));
  return RT_OK;
}

int rt_set_operator(rt_grid* g, const double* d_diag, const double* d_cx, const double* d_cy,
                    const double* d_cz) {
  if (!g) return RT_EINVAL;
  if (!d_diag || !d_cx || !d_cy || !d_cz) return fail(g, RT_EINVAL, "null operator array");
  const size_t N = g->P.N;
  Workspace& w = g->w;
  // a symmetric operator: the Schur matrix and the preconditioner's are the same
  HIPCHK(g, hipMemcpyAsync(w.diag, d_diag, N * 8, hipMemcpyDeviceToDevice, g->st));
  HIPCHK(g, hipMemcpyAsync(w.pdiag, d_diag, N * 8, hipMemcpyDeviceToDevice, g->st));
  const double* cs[3] = {d_cx, d_cy, d_cz};
  for (int d = 0; d < 3; ++d) {
    HIPCHK(g, hipMemcpyAsync(w.cx + d * N, cs[d], N * 8, hipMemcpyDeviceToDevice, g->st));
    HIPCHK(g, hipMemcpyAsync(w.fw + d * N, cs[d], N * 8, hipMemcpyDeviceToDevice, g->st));
    HIPCHK(g, hipMemcpyAsync(w.bw + d * N, cs[d], N * 8, hipMemcpyDeviceToDevice, g->st));
  }
  g->mg_stale = true;
  g->l0_fp32 = false;
  g->have_op = true;
  return RT_OK;
}

int rt_mg_vcycle(rt_grid* g, const double* d_r, double* d_z) {
  if (!g) return RT_EINVAL;
  if (!g->have_op) return fail(g, RT_EINVAL, "no Schur matrix yet");
  if (!d_r || !d_z) return fail(g, RT_EINVAL, "null argument");
  RTCHK(build_hierarchy(g));
  apply_vcycle(g, d_r, d_z);
  HIPCHK(g, hipGetLastError());
  return RT_OK;
}

int rt_mg_pcg_solve(rt_grid* g, const double* d_b, double* d_sE, double rtol, int32_t maxit,
                    int32_t* h_iters, double* h_relres) {
  if (!g) return RT_EINVAL;
  if (!g->have_op) return fail(g, RT_EINVAL, "no Schur matrix yet");
  if (!d_b || !d_sE || maxit < 0 || !(rtol >= 0)) return fail(g, RT_EINVAL, "bad argument");
  int its = 0, vc = 0;
  double rr = 0;
  RTCHK(krylov(g, d_b, d_sE, rtol, 0.0, maxit, &its, &rr, &vc));
  if (h_iters) *h_iters = its;
  if (h_relres) *h_relres = rr;
  return RT_OK;
}

int rt_newton_step(rt_grid* g, const double* d_Un, double* d_U, const double* d_Ualt, double dt,
                   const rt_cosmo* c, rt_newton_stats* h_stats) {
  RTCHK(check_ready(g));
  if (!d_Un || !d_U || !c || !(dt > 0)) return fail(g, RT_EINVAL, "bad argument");
  rt_newton_stats st;
  std::memset(&st, 0, sizeof st);
  st.fnorm_alt = -1.0;
  Workspace& w = g->w;
  const DevParams& P = g->P;
  const size_t bytesU = (size_t)P.nv * P.N * sizeof(double);
  const Step s = step_new(dt, c);
  auto finish = [&](int status) {
    st.status = status;
    if (h_stats) *h_stats = st;
    return status;
  };
  RTCHK(time_level(g, d_Un, dt, c, w.g));
  double fn, viol;
  RTCHK(residual_norm(g, d_U, w.g, s, w.f, &fn, &viol));
  st.fnorm_guess = fn;
  bool use_alt = false;
  if (d_Ualt) {
    double fa, va;
    RTCHK(residual_norm(g, d_Ualt, w.g, s, w.ft, &fa, &va));
    st.fnorm_alt = fa;
    if (std::isfinite(fa) && va == 0.0 && fa < fn) {
      use_alt = true;
      std::swap(w.f, w.ft);
      fn = fa;
      st.used_alt_guess = 1;
    }
  }
  st.fnorm[0] = fn;
  if (!std::isfinite(fn)) return finish(fail(g, RT_ENONFINITE, "non-finite initial residual"));
  // current iterate: the caller's buffer, w.Ut or (read only, until the first
  // accepted trial) the alternative guess, which is therefore not copied
  const double* cur = use_alt ? d_Ualt : d_U;
  double* spare = w.Ut;
  int k = 0;
  int status = RT_OK;
  while (fn >= g->prm.newton_tol && k < g->prm.newton_maxit) {
    // local: U, f, n_H, e_h in; f~_M, W, loc, b, om, ph out.  faces: E and the
    // fractions, n_H, loc, om, ph, b in; diag, pdiag, c (3), fw (3), bw (3),
    // b out (+ the FP32 copies of pdiag and c)
    TKB(g, RT_K_SCHUR,
        ((2.0 * P.nv + 2.0 + 2.0 * P.nb + 4.0) + (P.ns + 1.0 + 5.0 + 12.0 +
         (g->prm.limiter_lag ? 3.0 : 0.0)) + (g->prm.mg_fp32 ? 2.0 : 0.0)) * 8.0 * P.N,
        schur_into_workspace(g, cur, w.f, s, w.b));
    int its = 0, vc = 0;
    double rr = 0;
    // ||J S + f||_2 equals the Schur residual norm (the local rows are solved
    // exactly), and ||f||_2 = sqrt(N nv) times the RMS norm
    const double atol = g->prm.pcg_forcing * fn * std::sqrt((double)P.N * P.nv);
    status = krylov(g, w.b, w.x, g->prm.pcg_rtol, atol, g->prm.pcg_maxit, &its, &rr, &vc);
    if (status != RT_OK) break;
    st.cg_its[k] = its;
    st.cg_its_total += its;
    st.vcycles += vc;
    double lam = 1.0, ftn = 0.0;
    bool ok = false;
    while (status == RT_OK) {
      TKB(g, RT_K_TRIAL, (2.0 * P.nv + 2.0 * P.nb + 1.0) * 8.0 * P.N,
          launch_trial(P, cur, w.ftM, w.W, w.x, lam, spare, g->st));
      status = residual_norm(g, spare, w.g, s, w.ft, &ftn, &viol);
      if (status != RT_OK) break;
      ++st.ls_trials;
      if (viol == 0.0 && ftn <= (1.0 - ARMIJO * lam) * fn) {
        ok = true;
        break;
      }
      lam *= 0.5;
      if (lam < LAMBDA_MIN) break;
    }
    if (status != RT_OK) break;
    if (!ok) {
      status = fail(g, RT_ELINESEARCH, "line search failed at Newton iteration %d", k);
      break;
    }
    {
      // the accepted trial becomes the iterate; the next trial goes to the
      // other writable buffer (never the alternative guess)
      double* accepted = spare;
      spare = cur == d_Ualt ? (accepted == w.Ut ? d_U : w.Ut) : const_cast<double*>(cur);
      cur = accepted;
    }
    std::swap(w.f, w.ft);
    fn = ftn;
    st.lambda[k] = lam;
    st.fnorm[k + 1] = fn;
    ++k;
  }
  st.newton_its = k;
  st.fnorm_final = fn;
  // the last accepted iterate ends in the caller's buffer
  if (cur != d_U) HIPCHK(g, hipMemcpyAsync(d_U, cur, bytesU, hipMemcpyDeviceToDevice, g->st));
  HIPCHK(g, hipStreamSynchronize(g->st));
  if (status == RT_OK) {
    if (!std::isfinite(fn)) status = fail(g, RT_ENONFINITE, "non-finite residual");
    else if (fn >= g->prm.newton_tol) status = fail(g, RT_ENOCONV, "no convergence in %d its", k);
  }
  return finish(status);
}

int rt_timing(rt_grid* g, int32_t enable, rt_kernel_timing* out) {
  if (!g) return RT_EINVAL;
  Timer& t = g->tm;
  if (enable) {
    t.on = true;
    t.used = 0;
    t.cls.clear();
    for (double& b : t.bytes) b = 0.0;
    return RT_OK;
  }
  t.on = false;
  HIPCHK(g, hipStreamSynchronize(g->st));
  if (out) {
    std::memset(out, 0, sizeof *out);
    for (size_t i = 0; i < t.cls.size(); ++i) {
      float ms = 0.f;
      HIPCHK(g, hipEventElapsedTime(&ms, t.pool[2 * i], t.pool[2 * i + 1]));
      out->count[t.cls[i]] += 1;
      out->total_ms[t.cls[i]] += ms;
    }
    for (int c = 0; c < RT_K_COUNT; ++c) out->bytes[c] = t.bytes[c];
  }
  t.used = 0;
  t.cls.clear();
  return RT_OK;
}

int rt_timing_classes(rt_grid* g, uint32_t mask) {
  if (!g) return RT_EINVAL;
  g->tm.mask = mask;
  return RT_OK;
}

int rt_use_graphs(rt_grid* g, int32_t enable) {
  if (!g) return RT_EINVAL;
  g->graphs = enable != 0;
  if (!g->graphs) drop_box_graph(g);
  return RT_OK;
}

int rt_fold_energy(rt_grid* g, double* d_U, double* d_eh) {
  if (!g) return RT_EINVAL;
  if (!d_U || !d_eh) return fail(g, RT_EINVAL, "null argument");
  launch_fold_energy(g->P.N, d_U, d_eh, g->st);
  HIPCHK(g, hipGetLastError());
  return RT_OK;
}

// ---------------------------------------------------------------------------
// spectrum constants by composite Gauss-Legendre quadrature on log(nu)
int rt_spectrum_constants(int32_t grey, double T_B, double* Kg, double* Kk, double* Kh,
                          double* hnu) {
  if (!Kg || !Kk || !Kh || !hnu) return RT_EINVAL;
  const double h = 6.62607015e-27, kB = 1.380649e-16, eV = 1.602176634e-12;
  const double thr[3] = {13.6 * eV, 24.6 * eV, 54.4 * eV};
  const double sig0[3] = {6.30e-18, 7.42e-18, 1.575e-18};
  if (!grey) {
    Kg[0] = sig0[0] / thr[0]; Kk[0] = sig0[0]; Kh[0] = 0.0;
    for (int s = 1; s < 3; ++s) Kg[s] = Kk[s] = Kh[s] = 0.0;
    *hnu = thr[0];
    return RT_OK;
  }
  if (!(T_B > 0)) return RT_EINVAL;
  // 20-point Gauss-Legendre nodes/weights on [-1, 1]
  static const double xg[10] = {0.0765265211334973, 0.2277858511416451, 0.3737060887154195,
                                0.5108670019508271, 0.6360536807265150, 0.7463319064601508,
                                0.8391169718222188, 0.9122344282513259, 0.9639719272779138,
                                0.9931285991850949};
  static const double wg[10] = {0.1527533871307258, 0.1491729864726037, 0.1420961093183820,
                                0.1316886384491766, 0.1181945319615184, 0.1019301198172404,
                                0.0832767415767048, 0.0626720483341091, 0.0406014298003869,
                                0.0176140071391521};
  const double kT = kB * T_B;
  auto chi = [&](double e) { return e * e * e / std::expm1(e / kT); };   // e = h nu
  auto sigma = [&](int s, double e) { return e < thr[s] ? 0.0 : sig0[s] * std::pow(e / thr[s], -3.0); };
  // integrate f(e) de over [lo, hi] on a log grid, panels split at thresholds
  auto integ = [&](auto f, double lo, double hi) {
    double edges[8];
    int ne = 0;
    edges[ne++] = lo;
    for (int s = 1; s < 3; ++s)
      if (thr[s] > lo && thr[s] < hi) edges[ne++] = thr[s];
    edges[ne++] = hi;
    double total = 0.0;
    for (int e = 0; e + 1 < ne; ++e) {
      const double a = std::log(edges[e]), b = std::log(edges[e + 1]);
      const int panels = 400;
      const double hpan = (b - a) / panels;
      for (int pnl = 0; pnl < panels; ++pnl) {
        const double mid = a + (pnl + 0.5) * hpan, half = 0.5 * hpan;
        for (int q = 0; q < 10; ++q) {
          for (int sgn = -1; sgn <= 1; sgn += 2) {
            const double t = mid + sgn * half * xg[q];
            const double en = std::exp(t);
            total += wg[q] * half * f(en) * en;   // de = e dt
          }
        }
      }
    }
    return total;
  };
  const double hi = 80.0 * kT + 100.0 * thr[0];
  const double norm = integ([&](double e) { return chi(e); }, thr[0], hi);
  for (int s = 0; s < 3; ++s) {
    Kg[s] = integ([&](double e) { return sigma(s, e) * chi(e) / e; }, thr[s], hi) / norm;
    Kk[s] = integ([&](double e) { return sigma(s, e) * chi(e); }, thr[s], hi) / norm;
    Kh[s] = integ([&](double e) { return sigma(s, e) * (1.0 - thr[s] / e) * chi(e); }, thr[s], hi) / norm;
  }
  const double photons = integ([&](double e) { return chi(e) / e; }, thr[0], hi);
  *hnu = norm / photons;
  (void)h;
  return RT_OK;
}

}  // extern "C"
