// Host side of the thermocapillary step library: workspace carve-up, step
// orchestration (S1..S8), the PCG / multigrid driver, FP64 iterative
// refinement of the FP32 pressure solve, and the C ABI declared in tcf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/tcf.h"
#include "tcf_internal.h"

using namespace tcf;

namespace {

thread_local std::string g_err;

tcf_status fail(tcf_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHECK(expr)                                                                        \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(TCF_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));           \
  } while (0)

constexpr size_t kAlign = 256;
// over-correction of the piecewise-constant coarse correction
#ifndef TCF_OMEGA_C
#define TCF_OMEGA_C 1.9
#endif
constexpr double kOmegaC = TCF_OMEGA_C;
// the Chebyshev interval [lo, hi] of D^-1 K whose nodes give the 3-D sweep weights
#ifndef TCF_CHEB_LO
#define TCF_CHEB_LO 0.4
#endif
#ifndef TCF_CHEB_HI
#define TCF_CHEB_HI 2.0
#endif
constexpr int kCoarseSweeps = 30;
// fraction of the FP64 target that an inner FP32 solve aims at (its
// recurrence residual overstates the true reduction by FP32 rounding)
#ifndef TCF_REFINE_SAFETY
#define TCF_REFINE_SAFETY 0.5
#endif
constexpr double kRefineSafety = TCF_REFINE_SAFETY;
// the two finest-level post-smoothing sweeps as one pass (FP32, 3-D)
#ifndef TCF_FUSE_POST
#define TCF_FUSE_POST 1
#endif
constexpr bool kFusePost = TCF_FUSE_POST != 0;
// levels of at most this many cells (and everything below them) run as one
// block (the coarse tail of the V-cycle)
#ifndef TCF_MG_TAIL_CELLS
#define TCF_MG_TAIL_CELLS kTailCells
#endif
constexpr long kMgTailCells = TCF_MG_TAIL_CELLS;
static_assert(kMgTailCells <= kTailCells, "the tail stages a level's residuals in LDS of kTailCells values");

// Bump allocator over the caller's workspace; with base == nullptr it only
// counts bytes, so sizing and carving share one code path.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <class T>
  T* take(long n) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? (T*)(base + off) : nullptr;
    off += sizeof(T) * (size_t)std::max(n, 1L);
    return p;
  }
};

template <class R>
struct Fields {
  R *a = nullptr, *T = nullptr;            // state alpha, T (precision R)
  R *u = nullptr, *v = nullptr, *w = nullptr;  // velocity read by the stencils (alias of u64.. in FP64)
  R *a1, *T1, *a2, *T2;                    // RK3 stage values
  R *c = nullptr, *c1 = nullptr, *c2 = nullptr;  // species field and its RK3 stages (species configs)
  // N-phase configs: fractions of phases 3, 4 and their RK3 stages; the
  // mixture (rho, mu, rho c_p, lambda, the density as a fraction of the
  // operator's range, the condensed fraction 1 - alpha_1); per-pair
  // sigma*kappa; the face CSF force
  R *p3 = nullptr, *p31 = nullptr, *p32 = nullptr, *p4 = nullptr, *p41 = nullptr, *p42 = nullptr;
  R *mrcp = nullptr, *mlam = nullptr, *mdq = nullptr;  // N-phase mixture: rho c_p, lambda, heat-source delta
  R *marho = nullptr, *mamu = nullptr;                 // density and viscosity as fractions of their ranges
  R *skp = nullptr, *nrm = nullptr, *dsp = nullptr;  // per pair: sigma*kappa; normals and delta (scratch)
  R *fx = nullptr, *fy = nullptr, *fz = nullptr;
  R *sk, *Mx, *My, *Mz;                    // sigma*kappa, Marangoni vector
  R *us, *vs, *ws;                         // predictor
  std::vector<Level<R>> lv;                // Poisson levels (level 0 = fine)
  R *r, *z, *z2, *d, *d2;                  // PCG vectors on the fine level (d ping-pong)
  R* x;                                    // FP32 mode: inner correction e
  R* cinv = nullptr;                       // dense inverse of the coarsest level (if small)
  double* cfac = nullptr;                  // FP64 scratch of its factorisation
};

struct Dims {
  int dim, nx, ny, nz;
  long N, Nu, Nv, Nw;
};

Dims dims_of(const tcf_config* c) {
  Dims d;
  d.dim = c->dim;
  d.nx = c->nx;
  d.ny = c->ny;
  d.nz = c->dim == 2 ? 1 : c->nz;
  d.N = (long)d.nx * d.ny * d.nz;
  d.Nu = (long)(d.nx + 1) * d.ny * d.nz;
  d.Nv = (long)d.nx * (d.ny + 1) * d.nz;
  d.Nw = d.dim == 3 ? (long)d.nx * d.ny * (d.nz + 1) : 0;
  return d;
}

std::vector<std::array<int, 3>> level_dims(const Dims& D, int max_levels) {
  std::vector<std::array<int, 3>> v;
  int nx = D.nx, ny = D.ny, nz = D.nz;
  v.push_back({nx, ny, nz});
  for (;;) {
    if (max_levels > 0 && (int)v.size() >= max_levels) break;
    long n = (long)nx * ny * nz;
    bool can = nx % 2 == 0 && ny % 2 == 0 && nx >= 4 && ny >= 4 && (D.dim == 2 || (nz % 2 == 0 && nz >= 4)) && n > 64;
    if (!can) break;
    nx /= 2;
    ny /= 2;
    if (D.dim == 3) nz /= 2;
    v.push_back({nx, ny, nz});
  }
  return v;
}

}  // namespace

struct tcf_grid {
  tcf_config cfg;
  Dims D;
  KParams P;
  hipStream_t stream;
  // a second stream (default priority) on which a step builds the pressure
  // operator and its initial guess while the geometry and the predictor run
  // on `stream`; forked and joined through the two events.  Grids from
  // tcf_init_grid_static have none and run everything on `stream`.
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  bool side_forked = false;  // the current step's side work is on `side`
  bool fp32;
  bool has_fields = false;
  bool has_species = false;  // species field set (configs with species = 1)
  double* phist[2] = {nullptr, nullptr};  // p^(n-1), p^(n-2) of the extrapolated guess
  int nhist = 0;                           // how many of them are held
  // integrator 1: per stage the stage pressures of the last steps (newest
  // first), and how many steps they hold
  double* shist[3][3] = {};
  int snhist = 0;
  bool has_phases = false;   // fractions of phases 3 (and 4) set (N-phase configs)
  int nph = 2;               // number of phases
  double op_rho1 = 0.0, op_rho2 = 0.0;  // density range of the pressure operator's linear mix
  double t = 0.0;
  // FP64 state and scratch (both modes)
  double *u64, *v64, *w64, *p64, *b64, *r64, *ax64, *ay64, *az64, *zero64;
  double *un64 = nullptr, *vn64 = nullptr, *wn64 = nullptr;  // base velocity u^n (integrator 1)
  const void* a_op = nullptr;  // volume fraction of the pressure operator in use
  Fields<double> f64;
  Fields<float> f32;
  float *ax32, *ay32, *az32;
  double* part[6];
  int nb;  // capacity of each partial array
  double* scal;
  int* iflag;
  double* hscal;  // pinned host mirror (pageable, inside the slot, on a fixed-workspace grid)
  int* hflag;
  hipEvent_t rb_ev = nullptr;  // completion of the last copy into hscal
  // On a grid with a host-coherent mirror the device writes the block into
  // it (publish) followed by a ticket the host polls; pub_dev is the
  // mirror's device address (null: the block is copied with hipMemcpyAsync).
  void* pub_dev = nullptr;
  unsigned* pub_dticket = nullptr;
  volatile unsigned* pub_ticket = nullptr;
  unsigned pub_seq = 0, pub_want = 0;
  int static_dev = -1;         // device whose fixed workspace this grid uses (-1: caller's workspace)
  // CG iterations the last solve of each kind took (0: none yet): the
  // state's pressure or another right-hand side, first or later refinement
  int pcg_expect[4] = {0, 0, 0, 0};
  size_t bytes;
  // adjoint scratch (configs with TCF_WITH_ADJOINT; FP64 only)
  struct Adj {
    double *ab, *Tb, *usb, *vsb, *wsb, *ub, *vb, *wb, *pbar, *y, *skb, *Mxb, *Myb, *Mzb;
    double* vsum;  // the predictor's forward viscous term per face (one component at a time)
    double *nbx, *nby, *nbz, *dsb, *wa, *wT, *sa, *sT;
    double* pnext;   // the pressure of the state given to the last backward step
    double* yh[2];   // the adjoint pressures of the two calls before the last (newest first)
    long Ne;
    // time and step of the last backward step: when the next call is the
    // step before it, its forward solve starts from pnext (the solution it
    // recomputes) and its adjoint solve from the last y
    double t_last = 0.0, dt_last = 0.0;
    bool chain = false;
    int nchain = 0;  // consecutive chained calls whose adjoint pressures are held (A.y, then yh)
  } adj{};
  bool has_adj = false;
  // optional event timing of one kernel family (measurement only)
  int prof_family = -1;
  std::vector<hipEvent_t> prof_ev;  // start/end pairs
  size_t prof_used = 0;
  double prof_ms = 0.0;
  long prof_count = 0;
};

namespace {

enum Family { FAM_TRANSPORT = 0, FAM_GEOMETRY, FAM_PREDICTOR, FAM_SMOOTH0, FAM_SPMV, FAM_RESID64, FAM_PROJECT,
              FAM_SPECIES, FAM_UPDATE, FAM_SMOOTH2, FAM_N };
const char* kFamilyNames[FAM_N] = {"transport", "geometry", "predictor", "smooth", "spmv",
                                   "resid64", "project", "species", "update", "smooth2"};
constexpr size_t kProfPairs = 512;

hipError_t prof_flush(tcf_grid* g) {
  if (g->prof_used == 0) return hipSuccess;
  hipError_t e = hipEventSynchronize(g->prof_ev[2 * g->prof_used - 1]);
  if (e != hipSuccess) return e;
  for (size_t k = 0; k < g->prof_used; ++k) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, g->prof_ev[2 * k], g->prof_ev[2 * k + 1]);
    if (e != hipSuccess) return e;
    g->prof_ms += ms;
    g->prof_count += 1;
  }
  g->prof_used = 0;
  return hipSuccess;
}

// Brackets the launches of one kernel family with events on the grid's stream.
struct Prof {
  tcf_grid* g;
  bool on;
  Prof(tcf_grid* gg, int fam) : g(gg), on(fam >= 0 && gg->prof_family == fam) {
    if (!on) return;
    if (g->prof_used == kProfPairs) prof_flush(g);
    hipEventRecord(g->prof_ev[2 * g->prof_used], g->stream);
  }
  ~Prof() {
    if (!on) return;
    hipEventRecord(g->prof_ev[2 * g->prof_used + 1], g->stream);
    g->prof_used += 1;
  }
};

template <class R>
void carve_fields(Carver& cv, const Dims& D, Fields<R>& F, int mg_levels, bool alias_state, bool species, int nph,
                  double* u64, double* v64, double* w64, double* ax64, double* ay64, double* az64) {
  const long N = D.N;
  F.a = cv.take<R>(N);
  F.T = cv.take<R>(N);
  if (species) {
    F.c = cv.take<R>(N);
    F.c1 = cv.take<R>(N);
    F.c2 = cv.take<R>(N);
  }
  if (nph > 2) {
    F.p3 = cv.take<R>(N);
    F.p31 = cv.take<R>(N);
    F.p32 = cv.take<R>(N);
    if (nph == 4) {
      F.p4 = cv.take<R>(N);
      F.p41 = cv.take<R>(N);
      F.p42 = cv.take<R>(N);
    }
    F.mrcp = cv.take<R>(N);
    F.mlam = cv.take<R>(N);
    F.mdq = cv.take<R>(N);
    F.marho = cv.take<R>(N);
    F.mamu = cv.take<R>(N);
    const int npair = nph == 4 ? 6 : 3;
    F.skp = cv.take<R>(npair * N);
    F.nrm = cv.take<R>(3L * npair * N);
    F.dsp = cv.take<R>(npair * N);
    F.fx = cv.take<R>(D.Nu);
    F.fy = cv.take<R>(D.Nv);
    F.fz = D.dim == 3 ? cv.take<R>(D.Nw) : nullptr;
  }
  if (alias_state) {
    F.u = (R*)u64;
    F.v = (R*)v64;
    F.w = (R*)w64;
  } else {
    F.u = cv.take<R>(D.Nu);
    F.v = cv.take<R>(D.Nv);
    F.w = D.dim == 3 ? cv.take<R>(D.Nw) : nullptr;
  }
  F.a1 = cv.take<R>(N);
  F.T1 = cv.take<R>(N);
  F.a2 = cv.take<R>(N);
  F.T2 = cv.take<R>(N);
  F.sk = cv.take<R>(N);
  F.Mx = cv.take<R>(N);
  F.My = cv.take<R>(N);
  F.Mz = D.dim == 3 ? cv.take<R>(N) : nullptr;
  F.us = cv.take<R>(D.Nu);
  F.vs = cv.take<R>(D.Nv);
  F.ws = D.dim == 3 ? cv.take<R>(D.Nw) : nullptr;
  F.r = cv.take<R>(N);
  F.z = cv.take<R>(N);
  F.z2 = cv.take<R>(N);
  F.d = cv.take<R>(N);
  F.d2 = cv.take<R>(N);
  F.x = alias_state ? nullptr : cv.take<R>(N);
  auto ld = level_dims(D, mg_levels);
  F.lv.clear();
  for (size_t l = 0; l < ld.size(); ++l) {
    Level<R> L;
    L.nx = ld[l][0];
    L.ny = ld[l][1];
    L.nz = ld[l][2];
    const long n = L.n();
    const long nu = (long)(L.nx + 1) * L.ny * L.nz, nv = (long)L.nx * (L.ny + 1) * L.nz,
               nw = D.dim == 3 ? (long)L.nx * L.ny * (L.nz + 1) : 0;
    // level 0 of a multi-level hierarchy is applied matrix-free from alpha:
    // only the FP64 path keeps its weights (aliased), and 1/diag is not kept
    const bool matfree = l == 0 && ld.size() > 1;
    if (l == 0 && alias_state) {
      L.ax = (R*)ax64;
      L.ay = (R*)ay64;
      L.az = (R*)az64;
    } else if (matfree) {
      L.ax = L.ay = L.az = nullptr;
    } else {
      L.ax = cv.take<R>(nu);
      L.ay = cv.take<R>(nv);
      L.az = D.dim == 3 ? cv.take<R>(nw) : nullptr;
    }
    L.wdiag = matfree ? nullptr : cv.take<R>(n);
    if (l > 0) {
      L.x = cv.take<R>(n);
      L.x2 = cv.take<R>(n);
      L.b = cv.take<R>(n);
    } else {
      L.x = L.x2 = L.b = nullptr;
    }
    F.lv.push_back(L);
  }
  // the coarsest level needs x2 for its ping-pong even when it is level 0
  if (F.lv.size() == 1) F.lv[0].x2 = cv.take<R>(N);
  const long nc = F.lv.back().n();
  if (nc <= kCoarseDenseMax && F.lv.size() > 1) {
    F.cinv = cv.take<R>(nc * nc);
    F.cfac = cv.take<double>(nc * nc);
  } else {
    F.cinv = nullptr;
    F.cfac = nullptr;
  }
}

// The extrapolated initial guess is used by the one-solve integrator.
bool extrapolates(const tcf_config* c) { return c->p_extrapolate > 0 && c->integrator == 0; }

size_t carve(const tcf_config* c, void* base, tcf_grid* g) {
  Dims D = dims_of(c);
  Carver cv(base);
  tcf_grid dummy;
  tcf_grid* G = g ? g : &dummy;
  G->u64 = cv.take<double>(D.Nu);
  G->v64 = cv.take<double>(D.Nv);
  G->w64 = D.dim == 3 ? cv.take<double>(D.Nw) : nullptr;
  G->p64 = cv.take<double>(D.N);
  G->b64 = cv.take<double>(D.N);
  G->r64 = cv.take<double>(D.N);
  G->zero64 = cv.take<double>(D.N);
  if (extrapolates(c))
    for (int q = 0; q < c->p_extrapolate; ++q) G->phist[q] = cv.take<double>(D.N);
  if (c->p_extrapolate > 0 && c->integrator == 1)
    for (int k = 0; k < 3; ++k)
      for (int q = 0; q <= c->p_extrapolate; ++q) G->shist[k][q] = cv.take<double>(D.N);
  if (c->integrator == 1) {
    G->un64 = cv.take<double>(D.Nu);
    G->vn64 = cv.take<double>(D.Nv);
    G->wn64 = D.dim == 3 ? cv.take<double>(D.Nw) : nullptr;
  }
  // FP64 fine face weights: read by the FP64 path and by single-level
  // hierarchies; the FP32 refinement recomputes them from alpha
  if (c->precision != TCF_FP32_REFINE || level_dims(D, c->mg_levels).size() == 1) {
    G->ax64 = cv.take<double>(D.Nu);
    G->ay64 = cv.take<double>(D.Nv);
    G->az64 = D.dim == 3 ? cv.take<double>(D.Nw) : nullptr;
  } else {
    G->ax64 = G->ay64 = G->az64 = nullptr;
  }
  if (c->precision == TCF_FP32_REFINE)
    carve_fields<float>(cv, D, G->f32, c->mg_levels, false, c->species != 0, c->nphases, nullptr, nullptr, nullptr,
                        nullptr, nullptr, nullptr);
  else
    carve_fields<double>(cv, D, G->f64, c->mg_levels, true, c->species != 0, c->nphases, G->u64, G->v64, G->w64,
                         G->ax64, G->ay64, G->az64);
  const int nb = (int)std::max<long>((D.N + 255) / 256, (long)nblocks_cells(D.nx, D.ny, D.nz));
  G->nb = nb;
  if (c->flags & TCF_WITH_ADJOINT) {
    auto& A = G->adj;
    const long N = D.N;
    A.Ne = (long)(D.nx + 2) * (D.ny + 2) * (D.dim == 3 ? D.nz + 2 : 1);
    A.ab = cv.take<double>(N);
    A.Tb = cv.take<double>(N);
    A.usb = cv.take<double>(D.Nu);
    A.vsb = cv.take<double>(D.Nv);
    A.wsb = D.dim == 3 ? cv.take<double>(D.Nw) : nullptr;
    A.ub = cv.take<double>(D.Nu);
    A.vb = cv.take<double>(D.Nv);
    A.wb = D.dim == 3 ? cv.take<double>(D.Nw) : nullptr;
    A.pbar = cv.take<double>(N);
    A.pnext = cv.take<double>(N);
    A.yh[0] = cv.take<double>(N);
    A.yh[1] = cv.take<double>(N);
    A.y = cv.take<double>(N);
    A.skb = cv.take<double>(N);
    A.Mxb = cv.take<double>(N);
    A.Myb = cv.take<double>(N);
    A.Mzb = D.dim == 3 ? cv.take<double>(N) : nullptr;
    A.nbx = cv.take<double>(A.Ne);
    A.nby = cv.take<double>(A.Ne);
    A.nbz = D.dim == 3 ? cv.take<double>(A.Ne) : nullptr;
    A.dsb = cv.take<double>(A.Ne);
    A.vsum = cv.take<double>(std::max(D.Nu, std::max(D.Nv, D.Nw)));
    A.wa = cv.take<double>(N);
    A.wT = cv.take<double>(N);
    A.sa = cv.take<double>(N);
    A.sT = cv.take<double>(N);
    G->has_adj = true;
  }
  double* pbase = cv.take<double>(6L * nb);  // contiguous: diagnostics write 6 strided arrays
  for (int k = 0; k < 6; ++k) G->part[k] = pbase ? pbase + (long)k * nb : nullptr;
  G->scal = cv.take<double>(S_NSLOT + (I_NFLAG * sizeof(int) + sizeof(double) - 1) / sizeof(double));
  G->iflag = G->scal ? (int*)(G->scal + S_NSLOT) : nullptr;  // flags follow the scalars (one read-back)
  return cv.off + kAlign;
}

std::string validate(const tcf_config* c) {
  if (!c) return "cfg is NULL";
  if (c->dim != 2 && c->dim != 3) return "dim must be 2 or 3";
  if (c->nx < 4 || c->ny < 4) return "nx and ny must be >= 4";
  if (c->dim == 2 && c->nz != 1) return "nz must be 1 in 2D";
  if (c->dim == 3 && c->nz < 4) return "nz must be >= 4 in 3D";
  if ((double)c->nx * c->ny * (c->dim == 3 ? c->nz : 1) > 2.0e9) return "grid too large (more than 2e9 cells)";
  if (!(c->h > 0.0) || !std::isfinite(c->h)) return "h must be positive";
  if (c->precision != TCF_FP64 && c->precision != TCF_FP32_REFINE) return "unknown precision";
  if (c->flags & ~(TCF_TRANSPORT_ONLY | TCF_WITH_ADJOINT)) return "unknown flags";
  if ((c->flags & TCF_WITH_ADJOINT) && c->precision != TCF_FP64) return "the adjoint needs precision TCF_FP64";
  if (c->species != 0 && c->species != 1) return "species must be 0 or 1";
  if (c->species && (c->flags & TCF_WITH_ADJOINT)) return "the adjoint does not cover the species field";
  if (c->species && (!std::isfinite(c->dsigma_dc) || !std::isfinite(c->c0))) return "dsigma_dc and c0 must be finite";
  if (c->integrator != 0 && c->integrator != 1) return "integrator must be 0 or 1";
  if (c->integrator == 1 && (c->flags & TCF_WITH_ADJOINT)) return "the adjoint covers integrator 0 only";
  if (c->nphases != 0 && (c->nphases < 2 || c->nphases > 4)) return "nphases must be 0, 2, 3 or 4";
  if (c->nphases > 2) {
    if (c->species) return "the N-phase model is not combined with a species";
    if (c->integrator == 1) return "the N-phase model uses integrator 0";
    if (c->flags & TCF_WITH_ADJOINT) return "the adjoint covers the two-phase model only";
    for (int q = 0; q < c->nphases - 2; ++q)
      if (!(c->rho34[q] > 0 && c->rhocp34[q] > 0 && c->mu34[q] >= 0 && c->lambda34[q] >= 0))
        return "phase 3/4 materials: densities and rho*c_p positive, mu and lambda non-negative";
    for (int q = 0; q < 6; ++q)
      if (!std::isfinite(c->pair_sigma0[q]) || !std::isfinite(c->pair_dsigma_dT[q]))
        return "pair surface tensions must be finite";
  }
  if (!(c->rho1 > 0 && c->rho2 > 0)) return "densities must be positive";
  if (!(c->mu1 >= 0 && c->mu2 >= 0)) return "viscosities must be non-negative";
  if (!(c->rhocp1 > 0 && c->rhocp2 > 0)) return "rho*c_p must be positive";
  if (!(c->lambda1 >= 0 && c->lambda2 >= 0)) return "conductivities must be non-negative";
  for (int k = 0; k < 6; ++k)
    if (c->T_bc[k] != 0 && c->T_bc[k] != 1) return "T_bc entries must be 0 or 1";
  if (c->q_power != 0.0 && !(c->q_radius > 0)) return "q_radius must be positive";
  if (!(c->weno_eps > 0)) return "weno_eps must be positive";
  if (!(c->normal_eps > 0)) return "normal_eps must be positive";
  if (!(c->p_rtol > 0)) return "p_rtol must be positive";
  if (c->p_maxit < 1) return "p_maxit must be >= 1";
  if (c->mg_nu < 1 || c->mg_nu > 8) return "mg_nu must be in 1..8";
  if (c->mg_levels < 0) return "mg_levels must be >= 0";
  if (c->p_extrapolate < 0 || c->p_extrapolate > 2) return "p_extrapolate must be 0, 1 or 2";
  if (c->precision == TCF_FP32_REFINE && (!(c->inner_rtol > 0 && c->inner_rtol < 1) || c->refine_maxit < 1))
    return "FP32 mode needs 0 < inner_rtol < 1 and refine_maxit >= 1";
  return "";
}

KParams make_params(const tcf_config* c) {
  KParams P{};
  Dims D = dims_of(c);
  P.nx = D.nx;
  P.ny = D.ny;
  P.nz = D.nz;
  P.dim = D.dim;
  P.h = c->h;
  P.ih = 1.0 / c->h;
  P.rho1 = c->rho1;
  P.rho2 = c->rho2;
  P.mu1 = c->mu1;
  P.mu2 = c->mu2;
  P.rhocp1 = c->rhocp1;
  P.rhocp2 = c->rhocp2;
  P.lam1 = c->lambda1;
  P.lam2 = c->lambda2;
  P.sigma0 = c->sigma0;
  P.s = c->dsigma_dT;
  P.T0 = c->T0;
  P.sc = c->species ? c->dsigma_dc : 0.0;
  P.c0 = c->species ? c->c0 : 0.0;
  P.nph = c->nphases > 2 ? c->nphases : 2;
  for (int q = 0; q < 2; ++q) {
    P.mat34[0][q] = c->rho34[q];
    P.mat34[1][q] = c->mu34[q];
    P.mat34[2][q] = c->rhocp34[q];
    P.mat34[3][q] = c->lambda34[q];
  }
  for (int q = 0; q < 6; ++q) {
    P.sig0p[q] = c->pair_sigma0[q];
    P.dsigp[q] = c->pair_dsigma_dT[q];
  }
  for (int k = 0; k < 6; ++k) {
    P.Tbc[k] = c->T_bc[k];
    P.Tw[k] = c->T_wall[k];
  }
  P.qP = c->q_power;
  P.qr = c->q_radius;
  P.qx0 = c->q_x0;
  P.qy0 = c->q_y0;
  P.qvx = c->q_vx;
  P.qvy = c->q_vy;
  P.weno_eps = c->weno_eps;
  P.neps = c->normal_eps;
  return P;
}

// The scalar block and the flags are one device block (flags after the
// S_NSLOT doubles) mirrored by one pinned host block: one copy per read.
constexpr size_t kScalBlockBytes = sizeof(double) * S_NSLOT + sizeof(int) * I_NFLAG;

static_assert(kScalBlockBytes % 8 == 0, "the scalar block is copied in 8-byte words");
// host-coherent mirror: the block, then the ticket at kPubTicketOffset
constexpr size_t kPubTicketOffset = 256, kPubBytes = 320;
static_assert(kScalBlockBytes <= kPubTicketOffset, "the ticket follows the block");

// Wait until the ticket of the publish queued last has arrived.  The stream
// is queried now and then, so that an error on it, or a stream that has
// drained without the ticket, ends the wait with an error instead of
// spinning for ever.
hipError_t wait_ticket(tcf_grid* g) {
  const unsigned want = g->pub_want;
  for (unsigned n = 1;; ++n) {
    if (*g->pub_ticket == want) break;
    if (n % 4096 == 0) {
      const hipError_t e = hipStreamQuery(g->stream);
      if (e == hipSuccess) {
        // the publish has run: its stores are visible once it is complete
        for (int r = 0; r < 1000000 && *g->pub_ticket != want; ++r) {
        }
        if (*g->pub_ticket != want) return hipErrorLaunchFailure;
        break;
      }
      if (e != hipErrorNotReady) return e;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return hipSuccess;
}

hipError_t publish_block(tcf_grid* g, bool reset_flags = false) {
  g->pub_want = ++g->pub_seq;
  publish(g->stream, g->scal, (int)(kScalBlockBytes / 8), g->pub_dev, g->pub_dticket, g->pub_want,
          reset_flags ? g->iflag : nullptr);
  return hipGetLastError();
}

// reset_flags: on a grid with a host-coherent mirror, the device clears the
// flags once they are copied (the caller needs no init_flags after it).
hipError_t read_back(tcf_grid* g, bool reset_flags = false) {
  if (g->pub_dev) {
    const hipError_t e = publish_block(g, reset_flags);
    return e != hipSuccess ? e : wait_ticket(g);
  }
  hipError_t e = hipMemcpyAsync(g->hscal, g->scal, kScalBlockBytes, hipMemcpyDeviceToHost, g->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(g->stream);
}

// The copy of read_back queued without waiting; wait_back blocks until it
// has landed, while the stream may already run the work queued after it.
// On a fixed-workspace grid the mirror is pageable host memory, which a
// queued copy may fill after the event completes: the copy is waited for
// on the stream there.
hipError_t read_back_async(tcf_grid* g) {
  if (g->pub_dev) return publish_block(g);
  hipError_t e = hipMemcpyAsync(g->hscal, g->scal, kScalBlockBytes, hipMemcpyDeviceToHost, g->stream);
  if (e != hipSuccess) return e;
  if (g->static_dev >= 0 && (e = hipStreamSynchronize(g->stream)) != hipSuccess) return e;
  return hipEventRecord(g->rb_ev, g->stream);
}
hipError_t wait_back(tcf_grid* g) { return g->pub_dev ? wait_ticket(g) : hipEventSynchronize(g->rb_ev); }

// Launch constants of the pressure operator: the grid's, with the density
// range of the operator's linear mix (no step size: for the solver only).
KParams op_params(const tcf_grid* g) {
  KParams P = g->P;
  P.rho1 = g->op_rho1;
  P.rho2 = g->op_rho2;
  return P;
}

// Operator hierarchy.  Level 0 is applied matrix-free from alpha; its
// stored weights exist only where something reads them: the FP64 path (its
// initial residual and the coarsening) and single-level hierarchies (the
// coarsest-level solve).  Otherwise level 1 is coarsened straight from alpha.
template <class R>
void build_levels(tcf_grid* g, Fields<R>& F, const R* a, bool level0_stored) {
  const int dim = g->D.dim;
  if (F.lv.size() == 1) make_wdiag<R>(g->stream, dim, F.lv[0], 1.0);
  for (size_t l = 1; l < F.lv.size(); ++l) {
    // the level's weights and 1/diag in one pass
    if (l == 1 && !level0_stored) coarsen_from_alpha<R>(op_params(g), g->stream, a, F.lv[1]);
    else coarsen_weights<R>(g->stream, dim, F.lv[l - 1], F.lv[l]);
  }
  if (F.cinv) coarse_factor<R>(g->stream, dim, F.lv.back(), F.cfac, F.cinv);
}

template <class R>
Fields<R>& fields(tcf_grid* g);
template <>
Fields<double>& fields<double>(tcf_grid* g) { return g->f64; }
template <>
Fields<float>& fields<float>(tcf_grid* g) { return g->f32; }

template <class R>
Fine<R> fine_desc(tcf_grid* g) {
  Fine<R> F;
  F.a = g->a_op ? (const R*)g->a_op : fields<R>(g).a;
  F.nx = g->D.nx;
  F.ny = g->D.ny;
  F.nz = g->D.nz;
  F.rho1 = g->op_rho1;
  F.drho = g->op_rho2 - g->op_rho1;
  F.c2 = 2.0 / (g->cfg.h * g->cfg.h);
  return F;
}

// Constant damped-Jacobi weight (the many-sweep coarsest-level smoother).
inline double jacobi_omega(int dim) { return dim == 2 ? 0.8 : 6.0 / 7.0; }

// Weight of pre-smoothing sweep k of nu.  3D: the reciprocals of the
// Chebyshev nodes of degree nu on [lmax/5, lmax] of D^-1 K, lmax = 2 (a
// bound on its spectrum), so the nu sweeps together damp that upper part of
// the spectrum; with nu = 2 this takes the CG iteration count at 128^3 from
// 13-14 to 9-10.  2D: the constant weight (the schedule gains nothing
// there).  Post-smoothing takes the weights in reverse order, which keeps
// the V-cycle, and so the preconditioner, symmetric.
inline double sweep_omega(int dim, int nu, int k) {
  if (dim == 2) return 0.8;
  const double lo = TCF_CHEB_LO, hi = TCF_CHEB_HI;
  const double lam = 0.5 * (lo + hi) + 0.5 * (hi - lo) * std::cos((2.0 * k + 1.0) * M_PI / (2.0 * nu));
  return 1.0 / lam;
}

// Symmetric V-cycle: out = M b on level l (zero initial guess).  part (level
// 0 only) receives the partials of b.out and *np their count.  Buffers
// alternate so that the last write lands in out.  With first_done the first
// Jacobi sweep (omega_0 b / diag) is already in tmp.
// The inner FP32 solve's right-hand side taken straight from the FP64
// refinement residual: the first sweep of the first V-cycle scales r64 into
// the solve's r (see fine_smooth_first64); part receives the partials of
// |r|^2 (np of them), reduced with tolerance factor tau2 once that cycle is
// queued.
struct FromR64 {
  const double* r64;
  double* part;
  double tau2;
  int np;
};

// The rest of the V-cycle from level l runs in one block (k_mg_tail).
template <class R>
bool tail_at(const Fields<R>& F, size_t l, int nu) {
  long tail_lds = 0;
  for (size_t q = l; q < F.lv.size(); ++q) tail_lds += 3 * F.lv[q].n();
  return F.lv[l].n() <= kMgTailCells && F.lv.size() - l <= (size_t)kTailLevels && nu <= kTailNu &&
         tail_lds <= kTailLds;
}

// Coarse level l runs its cycle as the fused pair of launches
// (mg_sweep_restrict, mg_prolong_sweep2): two sweeps on each side, a
// launch-bound size, a coarser level below it and no one-block tail from it.
// Its first pre-sweep (written by the parent's restriction) is kept in the
// level's x instead of x2.
template <class R>
bool fused_level(const tcf_grid* g, const Fields<R>& F, size_t l) {
  return l >= 1 && l + 1 < F.lv.size() && g->cfg.mg_nu == 2 && mg_fused_level(F.lv[l].n()) &&
         !tail_at(F, l, g->cfg.mg_nu);
}

// Where the restriction into level c writes c's first pre-sweep: none if c is
// the coarsest (solved, not smoothed), x for a fused level, else x2.
template <class R>
R* first_sweep_target(const tcf_grid* g, Fields<R>& F, size_t c) {
  if (c + 1 >= F.lv.size()) return nullptr;
  return fused_level(g, F, c) ? F.lv[c].x : F.lv[c].x2;
}

template <class R>
R* vcycle(tcf_grid* g, Fields<R>& F, size_t l, const R* b, R* out, R* tmp, double* part, bool first_done, int* np,
          FromR64* f64 = nullptr) {
  hipStream_t s = g->stream;
  const int dim = g->D.dim;
  const int nu = g->cfg.mg_nu;
  auto wpre = [&](int k) { return sweep_omega(dim, nu, k); };
  auto wpost = [&](int k) { return sweep_omega(dim, nu, nu - 1 - k); };
  const Level<R>& L = F.lv[l];
  if (l + 1 == F.lv.size()) {
    Level<R> Lc = L;
    Lc.x2 = tmp;
    if (F.cinv) coarse_apply<R>(s, (int)L.n(), F.cinv, b, out, g->iflag);
    else mg_coarse_solve<R>(s, dim, Lc, b, out, kCoarseSweeps, jacobi_omega(dim), g->iflag);
    if (part) *np = dot_partials<R>(s, L.n(), b, out, part);
    return out;
  }
  R* bufs[2] = {tmp, out};
  Level<R>& C = F.lv[l + 1];
  if (l == 0) {
    const Fine<R> Fd = fine_desc<R>(g);
    int w = 1;
    if (!first_done) {
      if constexpr (std::is_same<R, float>::value) {
        if (f64)  // b is the solve's r, written here
          f64->np = fine_smooth_first64(s, dim, Fd, wpre(0), f64->r64, g->scal, const_cast<float*>(b), bufs[0],
                                        f64->part);
        else
          fine_smooth_first<R>(s, dim, Fd, wpre(0), b, bufs[0], g->iflag);
      } else {
        fine_smooth_first<R>(s, dim, Fd, wpre(0), b, bufs[0], g->iflag);
      }
    }
    for (int k = 1; k < nu; ++k, ++w) {
      Prof pr(g, FAM_SMOOTH0);
      fine_smooth<R>(s, dim, Fd, wpre(k), b, bufs[(w - 1) & 1], bufs[w & 1], nullptr, 0, 0, 0.0, nullptr, g->iflag);
    }
    const R* cur = bufs[(w - 1) & 1];
    // a coarse level that smooths gets its first sweep from the restriction
    const bool cfirst = l + 2 < F.lv.size();
    fine_resid_restrict<R>(s, dim, Fd, b, cur, C.b, C.wdiag, first_sweep_target(g, F, 1), wpre(0), g->iflag);
    vcycle<R>(g, F, 1, C.b, C.x, C.x2, nullptr, cfirst, nullptr);
    if constexpr (std::is_same<R, float>::value) {
      if (kFusePost && dim == 3 && nu == 2) {
        // both post-sweeps in one pass; it cannot write over its input, so
        // the result lands in the other buffer
        Prof pr(g, FAM_SMOOTH2);
        R* dst = bufs[w & 1];
        const int n = fine_smooth2(s, Fd, wpost(0), wpost(1), b, cur, dst, C.x, C.nx, C.ny, kOmegaC, part,
                                   g->iflag);
        if (np) *np = n;
        return dst;
      }
    }
    int n = fine_smooth<R>(s, dim, Fd, wpost(0), b, cur, bufs[w & 1], C.x, C.nx, C.ny, kOmegaC,
                           nu == 1 ? part : nullptr, g->iflag);
    ++w;
    for (int k = 1; k < nu; ++k, ++w) {
      Prof pr(g, FAM_SMOOTH0);
      n = fine_smooth<R>(s, dim, Fd, wpost(k), b, bufs[(w - 1) & 1], bufs[w & 1], nullptr, 0, 0, 0.0,
                         k == nu - 1 ? part : nullptr, g->iflag);
    }
    if (np) *np = n;
    return out;
  }
  if (tail_at(F, l, nu)) {
    // the rest of the cycle in one block (b, out, tmp are this level's b, x, x2)
    MgTail<R> T{};
    T.nl = (int)(F.lv.size() - l);
    for (int q = 0; q < T.nl; ++q) T.lv[q] = F.lv[l + q];
    T.nu = nu;
    T.first_done = first_done ? 1 : 0;
    T.cinv = F.cinv;
    T.csweeps = kCoarseSweeps;
    T.cj = jacobi_omega(dim);
    T.omc = kOmegaC;
    for (int k = 0; k < nu; ++k) {
      T.wpre[k] = wpre(k);
      T.wpost[k] = wpost(k);
    }
    mg_tail<R>(s, dim, T, g->iflag);
    return out;
  }
  const bool cfirst = l + 2 < F.lv.size();
  if (first_done && fused_level(g, F, l)) {
    // x1 (the first pre-sweep) is in out; x2 goes to tmp and the result to out
    mg_sweep_restrict<R>(s, dim, L, b, out, tmp, C.b, C.wdiag, first_sweep_target(g, F, l + 1), wpre(1), wpre(0),
                         g->iflag);
    vcycle<R>(g, F, l + 1, C.b, C.x, C.x2, nullptr, cfirst, nullptr);
    mg_prolong_sweep2<R>(s, dim, L, C, b, tmp, out, kOmegaC, wpost(0), wpost(1), g->iflag);
    return out;
  }
  int w = 0;  // next write goes to bufs[w & 1]
  if (!first_done) mg_smooth_first<R>(s, L, b, bufs[w & 1], wpre(0), g->iflag);
  ++w;
  for (int k = 1; k < nu; ++k, ++w)
    mg_smooth<R>(s, dim, L, b, bufs[(w - 1) & 1], bufs[w & 1], wpre(k), nullptr, g->iflag);
  const R* cur = bufs[(w - 1) & 1];
  mg_resid_restrict<R>(s, dim, L, b, cur, C.b, C.wdiag, first_sweep_target(g, F, l + 1), wpre(0), g->iflag);
  vcycle<R>(g, F, l + 1, C.b, C.x, C.x2, nullptr, cfirst, nullptr);
  mg_prolong_smooth<R>(s, dim, L, C, b, cur, bufs[w & 1], kOmegaC, wpost(0), nullptr, g->iflag);
  ++w;
  for (int k = 1; k < nu; ++k, ++w)
    mg_smooth<R>(s, dim, L, b, bufs[(w - 1) & 1], bufs[w & 1], wpost(k), nullptr, g->iflag);
  return out;
}

// PCG iterations on K x = rhs with r holding the initial residual and the
// done flag / tolerance already set.  The search direction ping-pongs
// between d and d2; the first Jacobi sweep of each preconditioner
// application is fused into the x/r update.  The convergence flag of an
// iteration is set with its residual norm, before its preconditioner: it is
// copied to the host there, and the host waits for that copy (not for the
// stream) while the preconditioner runs, then queues the next iteration.
// Every kernel of the solve returns at once when the flag is set, so an
// initial residual already below the tolerance ends after the first
// iteration with no work done.  From the iteration count at which the last
// solve of the same kind converged on, the host waits for the flag before
// queuing the preconditioner instead: a solve that has converged then ends
// without queuing a preconditioner whose kernels would all return at once.
// With x_zero, x starts from zero without being cleared: the first update
// writes x = alpha d (the first update always runs, the flag being set only
// by the residual norm after it).
// With f64, r is filled from the FP64 residual by the first preconditioner
// application (multigrid hierarchies of two or more levels only).
// One reduction launch per iteration: r.z and d.K d are summed from their
// block partials by every block of the pass that needs them (the SpMV pass
// forms beta, the update pass alpha); r.r, which the host reads, goes
// through a finalize.
template <class R>
tcf_status pcg_iterate(tcf_grid* g, Fields<R>& F, R* x, R* r, int maxit, int kind, bool x_zero, int* iters,
                       bool* converged, FromR64* f64 = nullptr) {
  hipStream_t s = g->stream;
  const int dim = g->D.dim;
  const Fine<R> Fd = fine_desc<R>(g);
  const double wj = sweep_omega(dim, g->cfg.mg_nu, 0);  // first pre-smoothing sweep, fused into the update
  *converged = false;
  // partials: r.z of each preconditioner application -> part[0], folded by
  // the next SpMV pass; d.K d of the SpMV -> part[1], folded by the update
  // pass; r.r of the update -> part[0], reduced by the convergence test
  int nrz = 0, ndq = 0, nrr = 0;
  R* z = vcycle<R>(g, F, 0, r, F.z, F.z2, g->part[0], false, &nrz, f64);
  if (f64) finalize(s, f64->part, f64->np, g->scal, g->iflag, F_BB, 0, f64->tau2);
  R* dcur = F.d;
  R* dnext = F.d2;
  const int expect = g->pcg_expect[kind];
  int last = 0;
  for (int it = 1; it <= maxit; ++it) {
    last = it;
    {
      Prof pr(g, FAM_SPMV);
      ndq = fine_spmv_upd<R>(s, dim, Fd, z, dcur, dnext, g->scal, it, g->part[0], nrz, g->part[1], g->iflag);
    }
    std::swap(dcur, dnext);
    {
      Prof pr(g, FAM_UPDATE);
      nrr = fine_update_smooth<R>(s, dim, Fd, wj, g->scal, it, x_zero && it == 1 ? 1 : 0, x, r, dcur, F.z2,
                                  g->part[1], ndq, g->part[0], g->iflag);
    }
    finalize(s, g->part[0], nrr, g->scal, g->iflag, F_RR, 0, 1.0);
    HIPCHECK(read_back_async(g));
    if (expect > 0 && it >= expect) {
      HIPCHECK(wait_back(g));
      if (g->hflag[I_DONE]) break;
    }
    z = vcycle<R>(g, F, 0, r, F.z, F.z2, g->part[0], true, &nrz);
    HIPCHECK(wait_back(g));
    if (g->hflag[I_DONE]) break;
  }
  *iters = g->hflag[I_ITERS];
  *converged = g->hflag[I_DONE] != 0 && std::isfinite(g->hscal[S_RR]);
  g->pcg_expect[kind] = *converged ? last : 0;
  return TCF_OK;
}

// FP64 solve of A p = b (b in b64, its mean in scal[S_MEAN]); p warm start.
tcf_status solve_fp64(tcf_grid* g, double* p, int kind, int* iters, double* relres, bool* converged) {
  hipStream_t s = g->stream;
  Fields<double>& F = g->f64;
  const Level<double>& L0 = F.lv[0];
  const int nbc = nblocks_cells(g->D.nx, g->D.ny, g->D.nz);
  init_flags(s, g->iflag);
  rhs_resid<double>(s, g->D.dim, L0, g->b64, g->scal, p, F.r, g->part[0], g->part[1]);
  const double rt = g->cfg.p_rtol;
  finalize(s, g->part[0], nbc, g->scal, g->iflag, F_BB, 0, rt * rt);
  finalize(s, g->part[1], nbc, g->scal, g->iflag, F_RR, 0, 0.0);
  HIPCHECK(read_back(g));
  const double bb = g->hscal[S_BB];
  if (!std::isfinite(bb) || !std::isfinite(g->hscal[S_RR])) {
    *iters = 0;
    *relres = NAN;
    *converged = false;
    return TCF_E_NONFINITE;
  }
  if (bb == 0.0) {
    fill_f64(s, g->D.N, p, 0.0);
    *iters = 0;
    *relres = 0.0;
    *converged = true;
    return TCF_OK;
  }
  tcf_status st = pcg_iterate<double>(g, F, p, F.r, g->cfg.p_maxit, kind, false, iters, converged);
  if (st != TCF_OK) return st;
  *relres = std::sqrt(g->hscal[S_RR] / bb);
  if (!std::isfinite(g->hscal[S_RR])) return TCF_E_NONFINITE;
  return TCF_OK;
}

// FP32 inner MG-PCG inside FP64 iterative refinement.
// psum: the number of partials of sum(p) left in part[2] by the last
// correction (0: none, the caller sums p itself).
tcf_status solve_refined(tcf_grid* g, double* p, int kind, int* iters, int* nref, double* relres, bool* converged,
                         int* psum) {
  hipStream_t s = g->stream;
  Fields<float>& F = g->f32;
  const long N = g->D.N;
  const int dim = g->D.dim;
  const int nb1 = (int)((N + 255) / 256);
  const double rt = g->cfg.p_rtol, irt = g->cfg.inner_rtol;
  *iters = 0;
  *nref = 0;
  *converged = false;
  *psum = 0;
  double bb = 0.0;
  int nrp = 0;
  for (int ref = 0;; ++ref) {
    {
      Prof pr(g, FAM_RESID64);
      nrp = resid64a<float>(op_params(g), s, fine_desc<float>(g).a, g->b64, g->scal, p, g->r64, g->part[0],
                            g->part[1]);
    }
    finalize2(s, g->part[0], g->part[1], nrp, g->scal, g->iflag, F_STORE, S_BB64, 0.0, F_SCALE, 0, (double)N);
    // the read-back clears the flags for the inner solve where it can (no
    // kernel after the solve reads them)
    const bool cleared = g->pub_dev != nullptr;
    HIPCHECK(read_back(g, cleared));
    bb = g->hscal[S_BB64];
    const double rr = g->hscal[S_RR64];
    if (!std::isfinite(bb) || !std::isfinite(rr)) {
      *relres = NAN;
      return TCF_E_NONFINITE;
    }
    if (bb == 0.0) {
      fill_f64(s, N, p, 0.0);
      *relres = 0.0;
      *converged = true;
      return TCF_OK;
    }
    *relres = std::sqrt(rr / bb);
    if (rr <= rt * rt * bb) {
      *converged = true;
      break;
    }
    if (ref >= g->cfg.refine_maxit) break;
    // inner solve of K e = r64 / scale in FP32 from e = 0
    // reduce the scaled residual only as far as this sweep needs to reach
    // the FP64 target (never below inner_rtol)
    const double tau = std::min(0.5, std::max(irt, kRefineSafety * rt * std::sqrt(bb / rr)));
    // the scaled residual r32 = r64 / scale with the partials of |r32|^2:
    // from the first sweep of a multigrid hierarchy, else in a pass of its own
    FromR64 f64{g->r64, g->part[1], tau * tau, 0};
    const bool fused = F.lv.size() > 1;
    if (!cleared) init_flags(s, g->iflag);
    if (!fused) {
      scale_to32(s, N, g->r64, g->scal, F.r, g->part[0]);
      finalize(s, g->part[0], nb1, g->scal, g->iflag, F_BB, 0, tau * tau);
    }
    int it = 0;
    bool conv = false;
    tcf_status st = pcg_iterate<float>(g, F, F.x, F.r, g->cfg.p_maxit, kind + (ref > 0 ? 1 : 0), true, &it, &conv,
                                       fused ? &f64 : nullptr);
    if (st != TCF_OK) return st;
    *iters += it;
    *psum = add_scaled(s, N, F.x, g->scal, p, g->part[2]);
    *nref = ref + 1;
  }
  return TCF_OK;
}

// Fine face weights from a volume fraction (the state's alpha unless one is
// given) and the whole hierarchy; the finest-level kernels and the FP64
// refinement residual recompute their weights from the same alpha.
// The density of the operator is rho_op1 + clamp(a) (rho_op2 - rho_op1):
// the two-phase mix of alpha (the state's unless a stage's is given) by
// default; the N-phase step passes its mixture density as a fraction of a
// range that holds every mixture.
template <class R>
void prepare_operator(tcf_grid* g, const R* a = nullptr, double rho_op1 = NAN, double rho_op2 = NAN) {
  Fields<R>& F = fields<R>(g);
  if (!a) a = F.a;
  if (std::isnan(rho_op1) || std::isnan(rho_op2)) {
    rho_op1 = g->cfg.rho1;
    rho_op2 = g->cfg.rho2;
  }
  g->a_op = a;
  g->op_rho1 = rho_op1;
  g->op_rho2 = rho_op2;
  const KParams P = op_params(g);
  bool stored = true;
  if (!g->fp32)
    face_weights<R>(P, g->stream, a, g->ax64, g->ay64, g->az64, nullptr, nullptr, nullptr);
  else if (F.lv.size() == 1)
    face_weights<R>(P, g->stream, a, g->ax64, g->ay64, g->az64, g->f32.lv[0].ax, g->f32.lv[0].ay,
                    g->f32.lv[0].az);
  else
    stored = false;  // the FP64 refinement residual recomputes its weights from alpha
  build_levels<R>(g, F, a, stored);
}

tcf_status solve(tcf_grid* g, double* p, tcf_step_info* inf) {
  int iters = 0, nref = 0;
  double relres = 0.0;
  bool conv = false;
  tcf_status st;
  const int kind = p == g->p64 ? 0 : 2;
  int nbp = 0;  // partials of sum(p) in part[2], if the solve left them
  if (g->fp32) st = solve_refined(g, p, kind, &iters, &nref, &relres, &conv, &nbp);
  else st = solve_fp64(g, p, kind, &iters, &relres, &conv);
  if (st != TCF_OK) return st;
  // gauge: mean(p) = 0
  if (nbp == 0) nbp = sum64_partials(g->stream, g->D.N, p, g->part[2]);
  finalize(g->stream, g->part[2], nbp, g->scal, g->iflag, F_MEAN, S_PMEAN, (double)g->D.N);
  subtract_mean(g->stream, g->D.N, g->scal, S_PMEAN, p);
  if (inf) {
    inf->cg_iters = iters;
    inf->refine_iters = nref;
    inf->p_relres = relres;
  }
  if (!conv) return fail(TCF_E_NOT_CONVERGED, "pressure solve did not reach p_rtol (relres " + std::to_string(relres) + ")");
  return TCF_OK;
}

template <class R>
tcf_status step_diag(tcf_grid* g, double dt, double dt_proj, tcf_step_info* inf, bool launched = false);

// N-phase model: a range of material `which` (0 density, 1 viscosity) that
// holds every mixture P_1 + sum_j clamp(alpha_j)(P_j - P_1), so that the
// linear mix of its fraction in the pressure kernels and the predictor
// never clamps.
void np_range(const tcf_grid* g, int which, double* lo, double* hi) {
  const KParams& P = g->P;
  const double p1 = which == 0 ? P.rho1 : P.mu1, p2 = which == 0 ? P.rho2 : P.mu2;
  double l = p1 + std::min(0.0, p2 - p1), h = p1 + std::max(0.0, p2 - p1);
  for (int q = 0; q < g->nph - 2; ++q) {
    l += std::min(0.0, P.mat34[which][q] - p1);
    h += std::max(0.0, P.mat34[which][q] - p1);
  }
  *lo = l;
  *hi = h > l ? h : l + 1.0;  // equal values: every fraction is 0
}
void np_rho_range(const tcf_grid* g, double* lo, double* hi) { np_range(g, 0, lo, hi); }

// Density and viscosity of the mixture of the given fractions, as fractions
// of their ranges (N-phase fields of F).
template <class R>
void np_mix(tcf_grid* g, const R* a2, const R* a3, const R* a4) {
  Fields<R>& F = fields<R>(g);
  double lo, hi, mlo, mhi;
  np_range(g, 0, &lo, &hi);
  np_range(g, 1, &mlo, &mhi);
  np_mixture<R>(g->P, g->stream, a2, a3, a4, F.marho, F.mamu, lo, hi, mlo, mhi);
}

// S2-S5 of the N-phase model at the state fractions: mixture, per-pair
// geometry, face CSF force, predictor into F.us, F.vs, F.ws.
template <class R>
void np_momentum_rhs(tcf_grid* g, const KParams& P) {
  Fields<R>& F = fields<R>(g);
  hipStream_t s = g->stream;
  np_mix<R>(g, F.a, F.p3, F.p4);
  {
    Prof pr(g, FAM_GEOMETRY);
    np_geometry<R>(P, s, F.a, F.p3, F.p4, F.T, F.nrm, F.dsp, F.skp, F.Mx, F.My, F.Mz);
    np_face_force<R>(P, s, F.a, F.p3, F.p4, F.skp, F.Mx, F.My, F.Mz, F.fx, F.fy, F.fz);
  }
  // the predictor in its material form: viscosity and density fractions
  // of their ranges, and the face force
  KParams Pm = P;
  np_range(g, 0, &Pm.rho1, &Pm.rho2);
  np_range(g, 1, &Pm.mu1, &Pm.mu2);
  Prof pr(g, FAM_PREDICTOR);
  predictor_mat<R>(Pm, s, F.mamu, F.marho, F.fx, F.fy, F.fz, F.u, F.v, F.w, F.us, F.vs, F.ws);
}

// The pressure operator of the current state: the two-phase mix of alpha,
// or the N-phase mixture density as a fraction of its range.
template <class R>
void prepare_state_operator(tcf_grid* g) {
  if (g->nph > 2) {
    Fields<R>& F = fields<R>(g);
    np_mix<R>(g, F.a, F.p3, F.p4);
    double lo, hi;
    np_rho_range(g, &lo, &hi);
    prepare_operator<R>(g, F.marho, lo, hi);
  } else {
    prepare_operator<R>(g);
  }
}

// Initial guess of the step's pressure solve (p_extrapolate > 0): the
// extrapolation through p and the previous pressures held, of the order
// configured or as far as they go, while the history shifts by one.  The
// guess is written into the buffer of the oldest pressure, and the three
// buffers change roles (no copies).
void pressure_guess(tcf_grid* g) {
  const int K = g->cfg.p_extrapolate;
  if (!g->phist[0]) return;
  const int m = std::min(g->nhist, K);
  double* p = g->p64;
  double* h1 = g->phist[0];
  double* h2 = g->phist[1];
  if (m == 0) {  // no guess: p stays, the history shifts
    if (K == 2) std::swap(g->phist[0], g->phist[1]);
    copy_f64(g->stream, g->D.N, p, g->phist[0]);
  } else {
    double* out = K == 2 ? h2 : h1;  // the oldest pressure's buffer
    extrapolate_f64(g->stream, g->D.N, m, p, h1, h2, out);
    g->p64 = out;
    if (K == 2) g->phist[1] = h1;
    g->phist[0] = p;
  }
  g->nhist = std::min(g->nhist + 1, K);
}

// One step of the N-phase model (integrator 0): SSP-RK3 transport of alpha,
// T and the fractions of phases 3 (and 4) with u^n frozen, each stage's T
// right-hand side with the mixture of that stage's fractions; then the
// mixture, geometry, face force and predictor at the new fractions, the
// pressure solve with the mixture density, and the projection.
template <class R>
tcf_status step_np(tcf_grid* g, double dt, tcf_step_info* inf, bool want_diag) {
  hipStream_t s = g->stream;
  Fields<R>& F = fields<R>(g);
  const Dims& D = g->D;
  KParams P = g->P;
  P.dt = dt;
  P.t = g->t;
  R* as[3] = {F.a, F.a1, F.a2};
  R* ao[3] = {F.a1, F.a2, F.a};
  R* Ts[3] = {F.T, F.T1, F.T2};
  R* To[3] = {F.T1, F.T2, F.T};
  R* p3s[3] = {F.p3, F.p31, F.p32};
  R* p3o[3] = {F.p31, F.p32, F.p3};
  R* p4s[3] = {F.p4, F.p41, F.p42};
  R* p4o[3] = {F.p41, F.p42, F.p4};
  const double cb[3] = {0.0, 0.75, 1.0 / 3.0}, ci[3] = {1.0, 0.25, 2.0 / 3.0};
  for (int k = 0; k < 3; ++k) {
    Prof pr(g, FAM_TRANSPORT);
    np_mixture_thermal<R>(P, s, as[k], p3s[k], g->nph == 4 ? p4s[k] : nullptr, F.mrcp, F.mlam, F.mdq);
    transport_temperature<R>(P, s, F.mlam, F.mrcp, F.mdq, Ts[k], F.T, F.u, F.v, F.w, To[k], cb[k], ci[k]);
    transport_scalar<R>(P, s, as[k], F.a, F.u, F.v, F.w, ao[k], cb[k], ci[k]);
    transport_scalar<R>(P, s, p3s[k], F.p3, F.u, F.v, F.w, p3o[k], cb[k], ci[k]);
    if (g->nph == 4) transport_scalar<R>(P, s, p4s[k], F.p4, F.u, F.v, F.w, p4o[k], cb[k], ci[k]);
  }
  tcf_status st = TCF_OK;
  if (!(g->cfg.flags & TCF_TRANSPORT_ONLY)) {
    np_momentum_rhs<R>(g, P);
    const int nbc = nblocks_cells(D.nx, D.ny, D.nz);
    divergence_rhs<R>(P, s, F.us, F.vs, F.ws, g->b64, g->part[0]);
    finalize(s, g->part[0], nbc, g->scal, g->iflag, F_MEAN, S_MEAN, (double)D.N);
    double lo, hi;
    np_rho_range(g, &lo, &hi);
    prepare_operator<R>(g, F.marho, lo, hi);  // F.marho: the mixture of the new fractions
    pressure_guess(g);
    st = solve(g, g->p64, inf);
    if (st != TCF_OK && st != TCF_E_NOT_CONVERGED) return st;
    KParams Pp = P;  // this step's constants with the operator's density range
    Pp.rho1 = lo;
    Pp.rho2 = hi;
    Prof pr(g, FAM_PROJECT);
    if (want_diag)  // with the end-of-step diagnostics in the same pass
      project_diag<R>(Pp, s, F.marho, F.a, g->p64, F.us, F.vs, F.ws, g->u64, g->v64, g->w64, g->fp32 ? F.u : nullptr,
                      g->fp32 ? F.v : nullptr, g->fp32 ? F.w : nullptr, g->part[0], g->nb, g->scal);
    else
      project<R>(Pp, s, F.marho, g->p64, F.us, F.vs, F.ws, g->u64, g->v64, g->w64, g->fp32 ? F.u : nullptr,
                 g->fp32 ? F.v : nullptr, g->fp32 ? F.w : nullptr);
  }
  g->t += dt;
  const bool fused = want_diag && !(g->cfg.flags & TCF_TRANSPORT_ONLY);
  const tcf_status sd = want_diag ? step_diag<R>(g, dt, dt, inf, fused) : TCF_OK;
  return sd != TCF_OK ? sd : st;
}

void release_side(tcf_grid* g) {
  if (g->join_ev) hipEventDestroy(g->join_ev);
  if (g->fork_ev) hipEventDestroy(g->fork_ev);
  if (g->side) hipStreamDestroy(g->side);
  g->join_ev = g->fork_ev = nullptr;
  g->side = nullptr;
}

// Run `work` (launches on g->stream) on the side stream after everything
// queued on the main stream so far; join_side() makes the main stream wait
// for it.  While a kernel family is being timed (tcf_profile) the work stays
// on the main stream, so that the family's events time its kernels alone.
template <class F>
void on_side(tcf_grid* g, F&& work) {
  g->side_forked = g->side && g->prof_family < 0;
  if (!g->side_forked) {
    work();
    return;
  }
  hipEventRecord(g->fork_ev, g->stream);
  hipStreamWaitEvent(g->side, g->fork_ev, 0);
  hipStream_t main = g->stream;
  g->stream = g->side;
  work();
  g->stream = main;
  hipEventRecord(g->join_ev, g->side);
}
void join_side(tcf_grid* g) {
  if (g->side_forked) hipStreamWaitEvent(g->stream, g->join_ev, 0);
  g->side_forked = false;
}

// One step S1..S8 in precision R.
template <class R>
tcf_status step_once(tcf_grid* g, double dt, tcf_step_info* inf, bool want_diag) {
  hipStream_t s = g->stream;
  Fields<R>& F = fields<R>(g);
  KParams P = g->P;
  P.dt = dt;
  P.t = g->t;
  const Dims& D = g->D;
  // S1: SSP-RK3 with frozen u^n (stage 3 writes the state in place)
  {
    Prof pr(g, FAM_TRANSPORT);
    transport_stage<R>(P, s, F.a, F.T, F.a, F.T, F.u, F.v, F.w, F.a1, F.T1, 0.0, 1.0);
  }
  {
    Prof pr(g, FAM_TRANSPORT);
    transport_stage<R>(P, s, F.a1, F.T1, F.a, F.T, F.u, F.v, F.w, F.a2, F.T2, 0.75, 0.25);
  }
  {
    Prof pr(g, FAM_TRANSPORT);
    transport_stage<R>(P, s, F.a2, F.T2, F.a, F.T, F.u, F.v, F.w, F.a, F.T, 1.0 / 3.0, 2.0 / 3.0);
  }
  if (F.c) {  // the species: the same three stages
    {
      Prof pr(g, FAM_SPECIES);
      transport_scalar<R>(P, s, F.c, F.c, F.u, F.v, F.w, F.c1, 0.0, 1.0);
    }
    {
      Prof pr(g, FAM_SPECIES);
      transport_scalar<R>(P, s, F.c1, F.c, F.u, F.v, F.w, F.c2, 0.75, 0.25);
    }
    {
      Prof pr(g, FAM_SPECIES);
      transport_scalar<R>(P, s, F.c2, F.c, F.u, F.v, F.w, F.c, 1.0 / 3.0, 2.0 / 3.0);
    }
  }
  tcf_status st = TCF_OK;
  if (!(g->cfg.flags & TCF_TRANSPORT_ONLY)) {
    // the operator of alpha^{n+1} and the pressure's initial guess depend on
    // neither the geometry nor the predictor: built beside them
    on_side(g, [&] {
      prepare_operator<R>(g);
      pressure_guess(g);
    });
    // S2-S5
    {
      Prof pr(g, FAM_GEOMETRY);
      geometry<R>(P, s, F.a, F.T, F.c, F.sk, F.Mx, F.My, F.Mz);
    }
    {
      Prof pr(g, FAM_PREDICTOR);
      predictor<R>(P, s, F.a, F.sk, F.Mx, F.My, F.Mz, F.u, F.v, F.w, F.us, F.vs, F.ws);
    }
    // S6
    const int nbc = nblocks_cells(D.nx, D.ny, D.nz);
    divergence_rhs<R>(P, s, F.us, F.vs, F.ws, g->b64, g->part[0]);
    finalize(s, g->part[0], nbc, g->scal, g->iflag, F_MEAN, S_MEAN, (double)D.N);
    // S7
    join_side(g);
    st = solve(g, g->p64, inf);
    if (st != TCF_OK && st != TCF_E_NOT_CONVERGED) return st;
    // S8
    Prof pr(g, FAM_PROJECT);
    if (want_diag)  // with the end-of-step diagnostics in the same pass
      project_diag<R>(P, s, F.a, F.a, g->p64, F.us, F.vs, F.ws, g->u64, g->v64, g->w64, g->fp32 ? F.u : nullptr,
                      g->fp32 ? F.v : nullptr, g->fp32 ? F.w : nullptr, g->part[0], g->nb, g->scal);
    else
      project<R>(P, s, F.a, g->p64, F.us, F.vs, F.ws, g->u64, g->v64, g->w64, g->fp32 ? F.u : nullptr,
                 g->fp32 ? F.v : nullptr, g->fp32 ? F.w : nullptr);
  }
  g->t += dt;
  const bool fused = want_diag && !(g->cfg.flags & TCF_TRANSPORT_ONLY);
  const tcf_status sd = want_diag ? step_diag<R>(g, dt, dt, inf, fused) : TCF_OK;
  return sd != TCF_OK ? sd : st;
}

// End-of-step diagnostics into inf (FP64 reductions).  dt_proj is the step
// of the last projection: the divergence ratio is |D u| / |D u~| with
// D u~ = dt_proj b.
template <class R>
tcf_status step_diag(tcf_grid* g, double dt, double dt_proj, tcf_step_info* inf, bool launched) {
  hipStream_t s = g->stream;
  Fields<R>& F = fields<R>(g);
  const KParams& P = g->P;
  {
    if (!launched) diagnostics<R>(P, s, F.a, g->u64, g->v64, g->w64, g->part[0], g->nb, g->scal);
    HIPCHECK(read_back(g));
    const double* h = g->hscal;
    if (inf) {
      inf->sum_alpha = h[S_SUMA];
      inf->alpha_min = h[S_AMIN];
      inf->alpha_max = h[S_AMAX];
      inf->cfl_max = dt * h[S_UMAX] / g->cfg.h;
      const double bb = g->fp32 ? h[S_BB64] : h[S_BB];
      inf->div_rel = (g->cfg.flags & TCF_TRANSPORT_ONLY) || bb == 0.0 ? 0.0 : std::sqrt(h[S_DIV2] / bb) / dt_proj;
      inf->nonfinite = (h[S_NONFIN] > 0.0 || !std::isfinite(h[S_SUMA])) ? 1 : 0;
    }
    if (h[S_NONFIN] > 0.0 || !std::isfinite(h[S_SUMA])) return fail(TCF_E_NONFINITE, "non-finite fields after step");
  }
  return TCF_OK;
}

// One step of the time-accurate integrator: SSP-RK3 (Shu-Osher) over the
// whole state with a projection in every stage.  Stage k (0, 1, 2) takes all
// right-hand sides at the stage state q_k = (alpha_k, T_k, c_k, u_k) and the
// heat source at t + (0, 1, 1/2) dt:
//   alpha_{k+1} = cb_k alpha^n + ci_k (alpha_k + dt L(q_k))   (T and c alike)
//   u~          = cb_k u^n + ci_k (u_k + dt F(q_k))           (predictor, combine)
//   u_{k+1}     = u~ - ci_k dt beta(alpha_k) G p,  D beta(alpha_k) G p = D u~ / (ci_k dt)
// with (cb, ci) = (0, 1), (3/4, 1/4), (1/3, 2/3).  The projection takes the
// density of the state the stage's momentum right-hand side was taken at.
// Stage arrays: alpha_0 = F.a (also the base), alpha_1 = F.a1, alpha_2 =
// F.a2; the last stage writes the base in place.  u^n is kept in FP64.
template <class R>
tcf_status step_rk3p(tcf_grid* g, double dt, tcf_step_info* inf, bool want_diag) {
  hipStream_t s = g->stream;
  Fields<R>& F = fields<R>(g);
  const Dims& D = g->D;
  const bool mom = !(g->cfg.flags & TCF_TRANSPORT_ONLY);
  R* as[3] = {F.a, F.a1, F.a2};
  R* ao[3] = {F.a1, F.a2, F.a};
  R* Ts[3] = {F.T, F.T1, F.T2};
  R* To[3] = {F.T1, F.T2, F.T};
  R* cs[3] = {F.c, F.c1, F.c2};
  R* co[3] = {F.c1, F.c2, F.c};
  const double cb[3] = {0.0, 0.75, 1.0 / 3.0}, ci[3] = {1.0, 0.25, 2.0 / 3.0}, tc[3] = {0.0, 1.0, 0.5};
  if (mom) {
    copy_f64(s, D.Nu, g->u64, g->un64);
    copy_f64(s, D.Nv, g->v64, g->vn64);
    if (D.dim == 3) copy_f64(s, D.Nw, g->w64, g->wn64);
  }
  tcf_status worst = TCF_OK;
  tcf_step_info acc{};
  double dt_proj = dt;
  for (int k = 0; k < 3; ++k) {
    KParams P = g->P;
    P.dt = dt;
    P.t = g->t + tc[k] * dt;
    if (mom) {
      {
        Prof pr(g, FAM_GEOMETRY);
        geometry<R>(P, s, as[k], Ts[k], F.c ? cs[k] : nullptr, F.sk, F.Mx, F.My, F.Mz);
      }
      Prof pr(g, FAM_PREDICTOR);
      predictor<R>(P, s, as[k], F.sk, F.Mx, F.My, F.Mz, F.u, F.v, F.w, F.us, F.vs, F.ws);
    }
    {
      Prof pr(g, FAM_TRANSPORT);
      transport_stage<R>(P, s, as[k], Ts[k], F.a, F.T, F.u, F.v, F.w, ao[k], To[k], cb[k], ci[k]);
    }
    if (F.c) {
      Prof pr(g, FAM_SPECIES);
      transport_scalar<R>(P, s, cs[k], F.c, F.u, F.v, F.w, co[k], cb[k], ci[k]);
    }
    if (!mom) continue;
    if (k > 0) {
      rk_combine<R>(s, D.Nu, k, g->un64, F.us);
      rk_combine<R>(s, D.Nv, k, g->vn64, F.vs);
      if (D.dim == 3) rk_combine<R>(s, D.Nw, k, g->wn64, F.ws);
    }
    KParams Pp = P;
    Pp.dt = ci[k] * dt;  // the projection's step
    const int nbc = nblocks_cells(D.nx, D.ny, D.nz);
    divergence_rhs<R>(Pp, s, F.us, F.vs, F.ws, g->b64, g->part[0]);
    finalize(s, g->part[0], nbc, g->scal, g->iflag, F_MEAN, S_MEAN, (double)D.N);
    prepare_operator<R>(g, as[k]);
    // initial guess: this stage's pressures of the last steps extrapolated
    // in time (else the previous stage's pressure)
    double** H = g->shist[k];
    const int K = g->cfg.p_extrapolate;
    if (H[0] && g->snhist > 0) {
      const int m = std::min(g->snhist - 1, K);
      if (m == 0) copy_f64(s, D.N, H[0], g->p64);
      else extrapolate_f64(s, D.N, m, H[0], H[1], H[2], g->p64);
    }
    tcf_step_info si{};
    const tcf_status st = solve(g, g->p64, &si);
    if (H[0]) {  // the stage's history shifts: the oldest buffer takes this pressure
      double* old = H[K];
      for (int q = K; q > 0; --q) H[q] = H[q - 1];
      H[0] = old;
      copy_f64(s, D.N, g->p64, H[0]);
    }
    if (st != TCF_OK && st != TCF_E_NOT_CONVERGED) return st;
    if (st != TCF_OK) worst = st;
    acc.cg_iters += si.cg_iters;
    acc.refine_iters += si.refine_iters;
    acc.p_relres = std::max(acc.p_relres, si.p_relres);
    Prof pr(g, FAM_PROJECT);
    if (want_diag && k == 2)  // the last projection with the end-of-step diagnostics
      project_diag<R>(Pp, s, as[k], F.a, g->p64, F.us, F.vs, F.ws, g->u64, g->v64, g->w64,
                      g->fp32 ? F.u : nullptr, g->fp32 ? F.v : nullptr, g->fp32 ? F.w : nullptr, g->part[0], g->nb,
                      g->scal);
    else
      project<R>(Pp, s, as[k], g->p64, F.us, F.vs, F.ws, g->u64, g->v64, g->w64, g->fp32 ? F.u : nullptr,
                 g->fp32 ? F.v : nullptr, g->fp32 ? F.w : nullptr);
    dt_proj = Pp.dt;
  }
  if (mom) g->snhist = std::min(g->snhist + 1, g->cfg.p_extrapolate + 1);
  g->t += dt;
  if (inf) {
    inf->cg_iters = acc.cg_iters;
    inf->refine_iters = acc.refine_iters;
    inf->p_relres = acc.p_relres;
  }
  const tcf_status sd = want_diag ? step_diag<R>(g, dt, dt_proj, inf, mom) : TCF_OK;
  return sd != TCF_OK ? sd : worst;
}

template <class R>
tcf_status predictor_only(tcf_grid* g, double dt, double* us, double* vs, double* ws) {
  hipStream_t s = g->stream;
  Fields<R>& F = fields<R>(g);
  KParams P = g->P;
  P.dt = dt;
  P.t = g->t;
  if (g->nph > 2) {
    np_momentum_rhs<R>(g, P);
  } else {
    geometry<R>(P, s, F.a, F.T, F.c, F.sk, F.Mx, F.My, F.Mz);
    predictor<R>(P, s, F.a, F.sk, F.Mx, F.My, F.Mz, F.u, F.v, F.w, F.us, F.vs, F.ws);
  }
  const Dims& D = g->D;
  if (g->fp32) {
    to_f64(s, D.Nu, (const float*)F.us, us);
    to_f64(s, D.Nv, (const float*)F.vs, vs);
    if (D.dim == 3) to_f64(s, D.Nw, (const float*)F.ws, ws);
  } else {
    copy_f64(s, D.Nu, (const double*)F.us, us);
    copy_f64(s, D.Nv, (const double*)F.vs, vs);
    if (D.dim == 3) copy_f64(s, D.Nw, (const double*)F.ws, ws);
  }
  HIPCHECK(hipGetLastError());
  return TCF_OK;
}

// ---------------------------------------------------------------------------
// Adjoint driver (FP64).

// S1 forward, keeping the stage states in f64.a1/T1, a2/T2; state arrays end
// at (alpha^{n+1}, T^{n+1}).
void forward_transport_keep(tcf_grid* g, const KParams& P) {
  Fields<double>& F = g->f64;
  hipStream_t s = g->stream;
  transport_stage<double>(P, s, F.a, F.T, F.a, F.T, F.u, F.v, F.w, F.a1, F.T1, 0.0, 1.0);
  transport_stage<double>(P, s, F.a1, F.T1, F.a, F.T, F.u, F.v, F.w, F.a2, F.T2, 0.75, 0.25);
  transport_stage<double>(P, s, F.a2, F.T2, F.a, F.T, F.u, F.v, F.w, F.a, F.T, 1.0 / 3.0, 2.0 / 3.0);
}

// Transposed SSP-RK3 (stages recomputed by the caller): given the adjoint
// (va, vT) of (alpha^{n+1}, T^{n+1}), write (ab, Tb) = adjoint of (alpha^n,
// T^n) and accumulate the face-velocity adjoints.
void rk3_reverse(tcf_grid* g, const KParams& P, const double* a0, const double* T0, const double* va,
                 const double* vT, double* ab, double* Tb, const double* const stages[4] = nullptr) {
  Fields<double>& F = g->f64;
  // the stage values: the grid's own (recomputed forward), or the caller's
  const double* a1 = stages ? stages[0] : F.a1;
  const double* T1 = stages ? stages[1] : F.T1;
  const double* a2 = stages ? stages[2] : F.a2;
  const double* T2 = stages ? stages[3] : F.T2;
  auto& A = g->adj;
  hipStream_t s = g->stream;
  const long N = g->D.N;
  // stage 3: out = 1/3 base + 2/3 G(a2, T2)
  adj_scale(s, N, 2.0 / 3.0, va, A.wa);
  adj_scale(s, N, 2.0 / 3.0, vT, A.wT);
  fill_f64(s, N, A.sa, 0.0);
  fill_f64(s, N, A.sT, 0.0);
  adj_transport_stage(P, s, a2, T2, F.u, F.v, F.w, A.wa, A.wT, A.sa, A.sT, A.ub, A.vb, A.wb);
  adj_scale(s, N, 1.0 / 3.0, va, ab);
  adj_scale(s, N, 1.0 / 3.0, vT, Tb);
  // stage 2: a2 = 3/4 base + 1/4 G(a1, T1)
  adj_axpy(s, N, 0.75, A.sa, ab);
  adj_axpy(s, N, 0.75, A.sT, Tb);
  adj_scale(s, N, 0.25, A.sa, A.wa);
  adj_scale(s, N, 0.25, A.sT, A.wT);
  fill_f64(s, N, A.sa, 0.0);
  fill_f64(s, N, A.sT, 0.0);
  adj_transport_stage(P, s, a1, T1, F.u, F.v, F.w, A.wa, A.wT, A.sa, A.sT, A.ub, A.vb, A.wb);
  // stage 1: a1 = G(a0, T0)
  adj_transport_stage(P, s, a0, T0, F.u, F.v, F.w, A.sa, A.sT, ab, Tb, A.ub, A.vb, A.wb);
}

void zero_adj_faces(tcf_grid* g) {
  auto& A = g->adj;
  const Dims& D = g->D;
  fill_f64(g->stream, D.Nu, A.ub, 0.0);
  fill_f64(g->stream, D.Nv, A.vb, 0.0);
  if (D.dim == 3) fill_f64(g->stream, D.Nw, A.wb, 0.0);
}

// (S2..S5)^T at the current fields (alpha', T', u^n) for a given ubar*;
// accumulates into A.ab, A.Tb, A.ub.. and stores sbar in scal[S_SBAR].
void predictor_reverse(tcf_grid* g, const KParams& P, const double* usb, const double* vsb, const double* wsb) {
  Fields<double>& F = g->f64;
  auto& A = g->adj;
  hipStream_t s = g->stream;
  const long N = g->D.N;
  fill_f64(s, N, A.skb, 0.0);
  fill_f64(s, N, A.Mxb, 0.0);
  fill_f64(s, N, A.Myb, 0.0);
  if (g->D.dim == 3) fill_f64(s, N, A.Mzb, 0.0);
  fill_f64(s, A.Ne, A.nbx, 0.0);
  fill_f64(s, A.Ne, A.nby, 0.0);
  if (g->D.dim == 3) fill_f64(s, A.Ne, A.nbz, 0.0);
  fill_f64(s, A.Ne, A.dsb, 0.0);
  adj_predictor(P, s, F.a, F.sk, F.Mx, F.My, F.Mz, F.u, F.v, F.w, usb, vsb, wsb, A.ub, A.vb, A.wb, A.ab, A.skb,
                A.Mxb, A.Myb, A.Mzb, A.vsum);
  const int np = adj_geometry(P, s, F.a, F.T, A.skb, A.Mxb, A.Myb, A.Mzb, A.Tb, A.nbx, A.nby, A.nbz, A.dsb, A.ab,
                              g->part[0]);
  finalize(s, g->part[0], np, g->scal, g->iflag, F_STORE, S_SBAR, 0.0);
}

tcf_status adj_checks(tcf_grid* g) {
  if (!g) return fail(TCF_E_INVALID, "grid is NULL");
  if (!g->has_adj) return fail(TCF_E_INVALID, "grid was not initialised with TCF_WITH_ADJOINT");
  return TCF_OK;
}

// Carve the workspace and clear what must start at zero (scalars, flags,
// the zero vector, the pressure); the rest of the workspace is written
// before it is read, so a reused workspace needs no clearing.
void init_handle(tcf_grid* g, const tcf_config* cfg, void* workspace, size_t bytes, void* hip_stream) {
  g->cfg = *cfg;
  if (g->cfg.dim == 2) g->cfg.nz = 1;
  g->D = dims_of(&g->cfg);
  g->P = make_params(&g->cfg);
  g->nph = g->P.nph;
  g->op_rho1 = g->cfg.rho1;
  g->op_rho2 = g->cfg.rho2;
  g->stream = (hipStream_t)hip_stream;
  g->fp32 = cfg->precision == TCF_FP32_REFINE;
  g->bytes = bytes;
  carve(&g->cfg, workspace, g);
}

void clear_start(tcf_grid* g) {
  g->hflag = (int*)(g->hscal + S_NSLOT);
  fill_f64(g->stream, S_NSLOT, g->scal, 0.0);
  init_flags(g->stream, g->iflag);
  fill_f64(g->stream, g->D.N, g->zero64, 0.0);
  fill_f64(g->stream, g->D.N, g->p64, 0.0);
}

}  // namespace

// -----------------------------------------------------------------------------
// Fixed workspace of tcf_init_grid_static: one array per GPU, held until the
// process ends.  In host code its name is only a stand-in: its device
// address on each GPU comes from hipGetSymbolAddress (once per device, with
// that device current) and only that address is passed on.
static __device__ __align__(256) unsigned char scratch[TCF_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxStaticDevices = 64;
struct StaticSlot {
  void* ptr = nullptr;      // device address of scratch on this GPU (nullptr: not looked up yet)
  hipEvent_t ev = nullptr;  // read-back event of the slot's grids, kept for the process
  bool in_use = false;      // a grid on this GPU's fixed workspace is open
  tcf_grid grid;            // the handle, reset by each tcf_init_grid_static
  alignas(64) unsigned char mirror[kScalBlockBytes];  // host mirror of the scalar block
};
StaticSlot g_static[kMaxStaticDevices];
std::mutex g_static_mu;

}  // namespace

// =============================================================================
// C ABI
extern "C" {

size_t tcf_workspace_bytes(const tcf_config* cfg) {
  if (!validate(cfg).empty()) return 0;
  return carve(cfg, nullptr, nullptr);
}

tcf_status tcf_init_grid(const tcf_config* cfg, void* workspace, size_t bytes, void* hip_stream, tcf_grid** out) {
  g_err.clear();
  if (!out) return fail(TCF_E_INVALID, "out is NULL");
  *out = nullptr;
  std::string why = validate(cfg);
  if (!why.empty()) return fail(TCF_E_INVALID, why);
  const size_t need = carve(cfg, nullptr, nullptr);
  if (!workspace) return fail(TCF_E_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)workspace % kAlign) return fail(TCF_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < need) return fail(TCF_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  tcf_grid* g = new (std::nothrow) tcf_grid();
  if (!g) return fail(TCF_E_INVALID, "host allocation failed");
  init_handle(g, cfg, workspace, bytes, hip_stream);
  if (hipHostMalloc((void**)&g->hscal, kPubBytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    delete g;
    return fail(TCF_E_DEVICE, "pinned host buffer allocation failed");
  }
  std::memset(g->hscal, 0, kPubBytes);
  if (hipHostGetDevicePointer(&g->pub_dev, g->hscal, 0) != hipSuccess || !g->pub_dev) {
    hipHostFree(g->hscal);
    delete g;
    return fail(TCF_E_DEVICE, "device address of the pinned host buffer not available");
  }
  g->pub_ticket = (volatile unsigned*)((char*)g->hscal + kPubTicketOffset);
  g->pub_dticket = (unsigned*)((char*)g->pub_dev + kPubTicketOffset);
  if (hipEventCreateWithFlags(&g->rb_ev, hipEventDisableTiming) != hipSuccess) {
    hipHostFree(g->hscal);
    delete g;
    return fail(TCF_E_DEVICE, "event creation failed");
  }
  if (hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&g->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&g->join_ev, hipEventDisableTiming) != hipSuccess) {
    release_side(g);
    hipEventDestroy(g->rb_ev);
    hipHostFree(g->hscal);
    delete g;
    return fail(TCF_E_DEVICE, "side stream creation failed");
  }
  clear_start(g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    release_side(g);
    hipEventDestroy(g->rb_ev);
    hipHostFree(g->hscal);
    delete g;
    return fail(TCF_E_DEVICE, std::string("init kernels: ") + hipGetErrorString(e));
  }
  *out = g;
  return TCF_OK;
}

tcf_status tcf_init_grid_static(const tcf_config* cfg, void* hip_stream, tcf_grid** out) {
  g_err.clear();
  if (!out) return fail(TCF_E_INVALID, "out is NULL");
  *out = nullptr;
  std::string why = validate(cfg);
  if (!why.empty()) return fail(TCF_E_INVALID, why);
  const size_t need = carve(cfg, nullptr, nullptr);
  if (need > TCF_STATIC_WORKSPACE_BYTES)
    return fail(TCF_E_WORKSPACE, "configuration needs " + std::to_string(need) +
                                     " bytes of workspace; the fixed workspace holds " +
                                     std::to_string((size_t)TCF_STATIC_WORKSPACE_BYTES));
  int dev = -1;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxStaticDevices) return fail(TCF_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticSlot& sl = g_static[dev];
  if (sl.in_use)
    return fail(TCF_E_STATE, "the fixed workspace of this GPU is in use by an open grid (tcf_destroy it first)");
  if (!sl.ptr) {
    // once per device, with that device current
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail(TCF_E_DEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    if (!p || (uintptr_t)p % kAlign) return fail(TCF_E_DEVICE, "fixed workspace address is not 256-byte aligned");
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return fail(TCF_E_DEVICE, std::string("event creation: ") + hipGetErrorString(e));
    sl.ptr = p;
    sl.ev = ev;
  }
  tcf_grid* g = &sl.grid;
  g->prof_ev.clear();
  *g = tcf_grid();
  init_handle(g, cfg, sl.ptr, TCF_STATIC_WORKSPACE_BYTES, hip_stream);
  g->hscal = (double*)sl.mirror;
  g->rb_ev = sl.ev;
  g->static_dev = dev;
  clear_start(g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TCF_E_DEVICE, std::string("init kernels: ") + hipGetErrorString(e));
  sl.in_use = true;
  *out = g;
  return TCF_OK;
}

tcf_status tcf_set_fields(tcf_grid* g, double t, const double* alpha, const double* T, const double* u,
                          const double* v, const double* w, const double* p) {
  g_err.clear();
  if (!g) return fail(TCF_E_INVALID, "grid is NULL");
  if (!alpha || !T || !u || !v) return fail(TCF_E_INVALID, "alpha, T, u, v must be non-NULL");
  if (g->D.dim == 3 && !w) return fail(TCF_E_INVALID, "w must be non-NULL in 3D");
  if (g->D.dim == 2 && w) return fail(TCF_E_INVALID, "w must be NULL in 2D");
  if (!std::isfinite(t)) return fail(TCF_E_INVALID, "t must be finite");
  hipStream_t s = g->stream;
  const Dims& D = g->D;
  copy_f64(s, D.Nu, u, g->u64);
  copy_f64(s, D.Nv, v, g->v64);
  if (D.dim == 3) copy_f64(s, D.Nw, w, g->w64);
  zero_walls<double>(g->P, s, g->u64, g->v64, g->w64);
  if (p) copy_f64(s, D.N, p, g->p64);
  else fill_f64(s, D.N, g->p64, 0.0);
  if (g->fp32) {
    to_f32(s, D.N, alpha, g->f32.a);
    to_f32(s, D.N, T, g->f32.T);
    to_f32(s, D.Nu, g->u64, g->f32.u);
    to_f32(s, D.Nv, g->v64, g->f32.v);
    if (D.dim == 3) to_f32(s, D.Nw, g->w64, g->f32.w);
  } else {
    copy_f64(s, D.N, alpha, g->f64.a);
    copy_f64(s, D.N, T, g->f64.T);
  }
  HIPCHECK(hipGetLastError());
  g->t = t;
  g->has_fields = true;
  g->nhist = 0;
  g->snhist = 0;
  return TCF_OK;
}

tcf_status tcf_get_fields(const tcf_grid* gc, double* t, double* alpha, double* T, double* u, double* v, double* w,
                          double* p) {
  g_err.clear();
  if (!gc) return fail(TCF_E_INVALID, "grid is NULL");
  tcf_grid* g = const_cast<tcf_grid*>(gc);
  if (!g->has_fields) return fail(TCF_E_STATE, "fields not set");
  hipStream_t s = g->stream;
  const Dims& D = g->D;
  if (t) *t = g->t;
  if (g->fp32) {
    if (alpha) to_f64(s, D.N, g->f32.a, alpha);
    if (T) to_f64(s, D.N, g->f32.T, T);
  } else {
    if (alpha) copy_f64(s, D.N, g->f64.a, alpha);
    if (T) copy_f64(s, D.N, g->f64.T, T);
  }
  if (u) copy_f64(s, D.Nu, g->u64, u);
  if (v) copy_f64(s, D.Nv, g->v64, v);
  if (w && D.dim == 3) copy_f64(s, D.Nw, g->w64, w);
  if (p) copy_f64(s, D.N, g->p64, p);
  HIPCHECK(hipGetLastError());
  return TCF_OK;
}

tcf_status tcf_get_pressure_history(const tcf_grid* gc, double* p1, double* p2, int* held) {
  g_err.clear();
  if (!gc || !held) return fail(TCF_E_INVALID, "grid and held must be non-NULL");
  tcf_grid* g = const_cast<tcf_grid*>(gc);
  if (!g->phist[0]) return fail(TCF_E_STATE, "the grid does not extrapolate the pressure");
  if ((g->nhist >= 1 && !p1) || (g->nhist >= 2 && !p2))
    return fail(TCF_E_INVALID, "p1 (and p2 with two pressures held) must be non-NULL");
  *held = g->nhist;
  if (g->nhist >= 1) copy_f64(g->stream, g->D.N, g->phist[0], p1);
  if (g->nhist >= 2) copy_f64(g->stream, g->D.N, g->phist[1], p2);
  HIPCHECK(hipGetLastError());
  return TCF_OK;
}

tcf_status tcf_set_pressure_history(tcf_grid* g, const double* p1, const double* p2, int held) {
  g_err.clear();
  if (!g) return fail(TCF_E_INVALID, "grid is NULL");
  if (!g->phist[0]) return fail(TCF_E_STATE, "the grid does not extrapolate the pressure");
  if (held < 0 || held > g->cfg.p_extrapolate) return fail(TCF_E_INVALID, "held must be in 0..p_extrapolate");
  if ((held >= 1 && !p1) || (held >= 2 && !p2))
    return fail(TCF_E_INVALID, "p1 (and p2 with held = 2) must be non-NULL");
  if (held >= 1) copy_f64(g->stream, g->D.N, p1, g->phist[0]);
  if (held >= 2) copy_f64(g->stream, g->D.N, p2, g->phist[1]);
  HIPCHECK(hipGetLastError());
  g->nhist = held;
  return TCF_OK;
}

tcf_status tcf_set_species(tcf_grid* g, const double* c) {
  g_err.clear();
  if (!g) return fail(TCF_E_INVALID, "grid is NULL");
  if (!g->cfg.species) return fail(TCF_E_STATE, "the grid was created without a species (species = 0)");
  if (!c) return fail(TCF_E_INVALID, "c must be non-NULL");
  if (g->fp32) to_f32(g->stream, g->D.N, c, g->f32.c);
  else copy_f64(g->stream, g->D.N, c, g->f64.c);
  HIPCHECK(hipGetLastError());
  g->has_species = true;
  return TCF_OK;
}

tcf_status tcf_set_phases(tcf_grid* g, const double* a3, const double* a4) {
  g_err.clear();
  if (!g) return fail(TCF_E_INVALID, "grid is NULL");
  if (g->nph <= 2) return fail(TCF_E_STATE, "the grid has two phases (nphases < 3)");
  if (!a3 || (g->nph == 4 && !a4)) return fail(TCF_E_INVALID, "a3 (and a4 with four phases) must be non-NULL");
  const long N = g->D.N;
  if (g->fp32) {
    to_f32(g->stream, N, a3, g->f32.p3);
    if (g->nph == 4) to_f32(g->stream, N, a4, g->f32.p4);
  } else {
    copy_f64(g->stream, N, a3, g->f64.p3);
    if (g->nph == 4) copy_f64(g->stream, N, a4, g->f64.p4);
  }
  HIPCHECK(hipGetLastError());
  g->has_phases = true;
  return TCF_OK;
}

tcf_status tcf_get_phases(const tcf_grid* gc, double* a3, double* a4) {
  g_err.clear();
  if (!gc) return fail(TCF_E_INVALID, "grid is NULL");
  tcf_grid* g = const_cast<tcf_grid*>(gc);
  if (g->nph <= 2) return fail(TCF_E_STATE, "the grid has two phases (nphases < 3)");
  if (!g->has_phases) return fail(TCF_E_STATE, "phase fractions not set");
  if (!a3 || (g->nph == 4 && !a4)) return fail(TCF_E_INVALID, "a3 (and a4 with four phases) must be non-NULL");
  const long N = g->D.N;
  if (g->fp32) {
    to_f64(g->stream, N, g->f32.p3, a3);
    if (g->nph == 4) to_f64(g->stream, N, g->f32.p4, a4);
  } else {
    copy_f64(g->stream, N, g->f64.p3, a3);
    if (g->nph == 4) copy_f64(g->stream, N, g->f64.p4, a4);
  }
  HIPCHECK(hipGetLastError());
  return TCF_OK;
}

tcf_status tcf_get_species(const tcf_grid* gc, double* c) {
  g_err.clear();
  if (!gc) return fail(TCF_E_INVALID, "grid is NULL");
  tcf_grid* g = const_cast<tcf_grid*>(gc);
  if (!g->cfg.species) return fail(TCF_E_STATE, "the grid was created without a species (species = 0)");
  if (!g->has_species) return fail(TCF_E_STATE, "species field not set");
  if (!c) return fail(TCF_E_INVALID, "c must be non-NULL");
  if (g->fp32) to_f64(g->stream, g->D.N, g->f32.c, c);
  else copy_f64(g->stream, g->D.N, g->f64.c, c);
  HIPCHECK(hipGetLastError());
  return TCF_OK;
}

tcf_status tcf_step(tcf_grid* g, double dt, int nsteps, tcf_step_info* info) {
  g_err.clear();
  if (!g) return fail(TCF_E_INVALID, "grid is NULL");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(TCF_E_INVALID, "dt must be positive and finite");
  if (nsteps < 0) return fail(TCF_E_INVALID, "nsteps must be >= 0");
  if (!g->has_fields) return fail(TCF_E_STATE, "fields not set");
  if (g->cfg.species && !g->has_species) return fail(TCF_E_STATE, "species field not set");
  if (g->nph > 2 && !g->has_phases) return fail(TCF_E_STATE, "phase fractions not set");
  if (info) std::memset(info, 0, sizeof(*info));
  tcf_status worst = TCF_OK;
  for (int k = 0; k < nsteps; ++k) {
    const bool last = k == nsteps - 1;
    tcf_step_info* inf = last ? info : nullptr;
    const bool diag = last && info != nullptr;
    tcf_status st = g->nph > 2 ? (g->fp32 ? step_np<float>(g, dt, inf, diag) : step_np<double>(g, dt, inf, diag))
                    : g->cfg.integrator == 1
                        ? (g->fp32 ? step_rk3p<float>(g, dt, inf, diag) : step_rk3p<double>(g, dt, inf, diag))
                        : (g->fp32 ? step_once<float>(g, dt, inf, diag) : step_once<double>(g, dt, inf, diag));
    if (st == TCF_E_NOT_CONVERGED) {
      worst = st;
      continue;
    }
    if (st != TCF_OK) {
      if (st == TCF_E_NONFINITE && info) info->nonfinite = 1;
      if (st == TCF_E_NONFINITE && g_err.empty()) g_err = "non-finite residual in step " + std::to_string(k);
      return st;
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TCF_E_DEVICE, std::string("step kernels: ") + hipGetErrorString(e));
  if (worst != TCF_OK && g_err.empty()) g_err = "pressure solve did not converge";
  return worst;
}

tcf_status tcf_solve_pressure(tcf_grid* g, const double* rhs, double* p, tcf_step_info* info) {
  g_err.clear();
  if (!g) return fail(TCF_E_INVALID, "grid is NULL");
  if (!rhs || !p) return fail(TCF_E_INVALID, "rhs and p must be non-NULL");
  if (!g->has_fields) return fail(TCF_E_STATE, "fields not set");
  if (info) std::memset(info, 0, sizeof(*info));
  hipStream_t s = g->stream;
  const long N = g->D.N;
  copy_f64(s, N, rhs, g->b64);
  const int nbp = sum64_partials(s, N, g->b64, g->part[0]);
  finalize(s, g->part[0], nbp, g->scal, g->iflag, F_MEAN, S_MEAN, (double)N);
  if (g->fp32) prepare_state_operator<float>(g);
  else prepare_state_operator<double>(g);
  tcf_status st = solve(g, p, info);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(TCF_E_DEVICE, std::string("solve: ") + hipGetErrorString(e));
  return st;
}

tcf_status tcf_predictor(tcf_grid* g, double dt, double* us, double* vs, double* ws) {
  g_err.clear();
  if (!g) return fail(TCF_E_INVALID, "grid is NULL");
  if (!us || !vs || (g->D.dim == 3 && !ws)) return fail(TCF_E_INVALID, "output pointers must be non-NULL");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(TCF_E_INVALID, "dt must be positive and finite");
  if (!g->has_fields) return fail(TCF_E_STATE, "fields not set");
  if (g->cfg.species && !g->has_species) return fail(TCF_E_STATE, "species field not set");
  if (g->nph > 2 && !g->has_phases) return fail(TCF_E_STATE, "phase fractions not set");
  return g->fp32 ? predictor_only<float>(g, dt, us, vs, ws) : predictor_only<double>(g, dt, us, vs, ws);
}

tcf_status tcf_apply_A(tcf_grid* g, const double* x, double* y) {
  g_err.clear();
  if (!g) return fail(TCF_E_INVALID, "grid is NULL");
  if (!x || !y) return fail(TCF_E_INVALID, "x and y must be non-NULL");
  if (!g->has_fields) return fail(TCF_E_STATE, "fields not set");
  if (g->nph > 2 && !g->has_phases) return fail(TCF_E_STATE, "phase fractions not set");
  hipStream_t s = g->stream;
  if (g->fp32) prepare_state_operator<float>(g);
  else prepare_state_operator<double>(g);
  // y = -(0 - 0) - K x = A x, with scal[S_MEAN] = 0 and a zero rhs
  fill_f64(s, 1, g->scal + S_MEAN, 0.0);
  const KParams Pop = op_params(g);
  if (g->fp32) resid64a<float>(Pop, s, fine_desc<float>(g).a, g->zero64, g->scal, x, y, g->part[0], g->part[1]);
  else resid64a<double>(Pop, s, fine_desc<double>(g).a, g->zero64, g->scal, x, y, g->part[0], g->part[1]);
  HIPCHECK(hipGetLastError());
  return TCF_OK;
}

void tcf_destroy(tcf_grid* g) {
  if (!g) return;
  hipStreamSynchronize(g->stream);
  for (hipEvent_t e : g->prof_ev) hipEventDestroy(e);
  if (g->static_dev >= 0) {  // the handle, its event and mirror belong to the device's slot
    g->prof_ev.clear();
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static[g->static_dev].in_use = false;
    return;
  }
  if (g->side) hipStreamSynchronize(g->side);
  release_side(g);
  if (g->rb_ev) hipEventDestroy(g->rb_ev);
  hipHostFree(g->hscal);
  delete g;
}

tcf_status tcf_profile(tcf_grid* g, const char* family) {
  g_err.clear();
  if (!g) return fail(TCF_E_INVALID, "grid is NULL");
  HIPCHECK(prof_flush(g));
  g->prof_ms = 0.0;
  g->prof_count = 0;
  g->prof_family = -1;
  if (!family || !*family) return TCF_OK;
  int fam = -1;
  for (int k = 0; k < FAM_N; ++k)
    if (std::strcmp(family, kFamilyNames[k]) == 0) fam = k;
  if (fam < 0) return fail(TCF_E_INVALID, std::string("unknown kernel family ") + family);
  if (g->prof_ev.empty()) {
    g->prof_ev.resize(2 * kProfPairs);
    for (auto& e : g->prof_ev) HIPCHECK(hipEventCreate(&e));
  }
  g->prof_family = fam;
  return TCF_OK;
}

tcf_status tcf_profile_read(tcf_grid* g, double* total_ms, long* launches) {
  g_err.clear();
  if (!g || !total_ms || !launches) return fail(TCF_E_INVALID, "NULL argument");
  HIPCHECK(prof_flush(g));
  *total_ms = g->prof_ms;
  *launches = g->prof_count;
  return TCF_OK;
}

// The reverse sweep of one adjoint step (S8^T .. S1^T) once the grid holds
// the forward step's intermediates: alpha, T, p of step n+1 in F.a, F.T,
// p64, u^n in F.u.., the geometry of step n+1 and the pressure operator of
// alpha^{n+1}; the transport's stage values in F.a1.. or in stages.
static tcf_status backward_sweep(tcf_grid* g, KParams& P, double t_n, double dt, const double* const state_n[6],
                          const double* const adj_np1[5], double* const adj_n[5], double* dL_dsigmaT,
                          const double* const stages[4]) {
  hipStream_t s = g->stream;
  Fields<double>& F = g->f64;
  auto& A = g->adj;
  const Dims& D = g->D;
  const long N = D.N;
  const bool chain = A.chain && A.dt_last == dt && std::fabs(A.t_last - (t_n + dt)) <= 1e-6 * dt;
  // ---- S8^T
  copy_f64(s, N, adj_np1[0], A.ab);
  copy_f64(s, N, adj_np1[1], A.Tb);
  adj_project(P, s, F.a, g->p64, adj_np1[2], adj_np1[3], D.dim == 3 ? adj_np1[4] : nullptr, A.pbar, A.ab);
  // ---- S7^T: y = A^+ pbar with the same symmetric operator, then dA/dalpha
  copy_f64(s, N, A.pbar, g->b64);
  const int nbp = sum64_partials(s, N, g->b64, g->part[0]);
  finalize(s, g->part[0], nbp, g->scal, g->iflag, F_MEAN, S_MEAN, (double)N);
  // the adjoint pressure: zero, or the last one extrapolated through the
  // earlier ones held (quadratic in the step index once three are held)
  if (!chain) {
    fill_f64(s, N, A.y, 0.0);
    A.nchain = 0;
  } else if (A.nchain >= 2) {
    const int m = std::min(A.nchain - 1, 2);
    // the guess goes into the buffer of the oldest (yh[1]: read in place
    // when m = 2, free when m = 1); then the roles shift by one
    double* out = A.yh[1];
    extrapolate_f64(s, N, m, A.y, A.yh[0], A.yh[1], out);
    A.yh[1] = A.yh[0];
    A.yh[0] = A.y;
    A.y = out;
  } else {
    copy_f64(s, N, A.y, A.yh[0]);  // keep the last one as history
  }
  tcf_status st = solve(g, A.y, nullptr);
  if (st != TCF_OK && st != TCF_E_NOT_CONVERGED) return st;
  adj_poisson_alpha(P, s, F.a, g->p64, A.y, A.ab);
  // ---- S6^T
  adj_rhs(P, s, adj_np1[2], adj_np1[3], D.dim == 3 ? adj_np1[4] : nullptr, A.y, A.usb, A.vsb, A.wsb);
  // ---- (S2..S5)^T
  zero_adj_faces(g);
  predictor_reverse(g, P, A.usb, A.vsb, A.wsb);
  adj_add_scalar(s, dL_dsigmaT, g->scal + S_SBAR);
  // ---- S1^T
  rk3_reverse(g, P, state_n[0], state_n[1], A.ab, A.Tb, adj_n[0], adj_n[1], stages);
  zero_walls<double>(P, s, A.ub, A.vb, A.wb);
  copy_f64(s, D.Nu, A.ub, adj_n[2]);
  copy_f64(s, D.Nv, A.vb, adj_n[3]);
  if (D.dim == 3) copy_f64(s, D.Nw, A.wb, adj_n[4]);
  if (state_n[5]) copy_f64(s, N, state_n[5], A.pnext);
  else fill_f64(s, N, A.pnext, 0.0);
  A.t_last = t_n;
  A.dt_last = dt;
  A.chain = true;
  A.nchain = std::min(A.nchain + 1, 3);
  HIPCHECK(hipGetLastError());
  return st;
}

static tcf_status backward_args(tcf_grid* g, double t_n, double dt, const double* const state_n[6],
                         const double* const adj_np1[5], double* const adj_n[5], double* dL_dsigmaT) {
  tcf_status st = adj_checks(g);
  if (st != TCF_OK) return st;
  if (g->cfg.flags & TCF_TRANSPORT_ONLY)
    return fail(TCF_E_INVALID, "the step adjoint covers S1..S8; this grid steps with TCF_TRANSPORT_ONLY");
  const Dims& D = g->D;
  if (!state_n || !adj_np1 || !adj_n || !dL_dsigmaT) return fail(TCF_E_INVALID, "NULL argument");
  for (int k = 0; k < 5; ++k) {
    const bool need = k < 4 || D.dim == 3;
    if (need && (!state_n[k] || !adj_np1[k] || !adj_n[k])) return fail(TCF_E_INVALID, "NULL field pointer");
  }
  if (!(dt > 0) || !std::isfinite(dt) || !std::isfinite(t_n)) return fail(TCF_E_INVALID, "bad dt or t_n");
  return TCF_OK;
}

tcf_status tcf_step_backward(tcf_grid* g, double t_n, double dt, const double* const state_n[6],
                             const double* const adj_np1[5], double* const adj_n[5], double* dL_dsigmaT) {
  g_err.clear();
  tcf_status st = backward_args(g, t_n, dt, state_n, adj_np1, adj_n, dL_dsigmaT);
  if (st != TCF_OK) return st;
  const Dims& D = g->D;
  st = tcf_set_fields(g, t_n, state_n[0], state_n[1], state_n[2], state_n[3], D.dim == 3 ? state_n[4] : nullptr,
                      state_n[5]);
  if (st != TCF_OK) return st;
  hipStream_t s = g->stream;
  Fields<double>& F = g->f64;
  auto& A = g->adj;
  KParams P = g->P;
  P.dt = dt;
  P.t = t_n;
  const long N = D.N;
  // ---- forward S1..S7, keeping what the reverse sweep reads
  forward_transport_keep(g, P);
  geometry<double>(P, s, F.a, F.T, nullptr, F.sk, F.Mx, F.My, F.Mz);
  predictor<double>(P, s, F.a, F.sk, F.Mx, F.My, F.Mz, F.u, F.v, F.w, F.us, F.vs, F.ws);
  const int nbc = nblocks_cells(D.nx, D.ny, D.nz);
  divergence_rhs<double>(P, s, F.us, F.vs, F.ws, g->b64, g->part[0]);
  finalize(s, g->part[0], nbc, g->scal, g->iflag, F_MEAN, S_MEAN, (double)N);
  prepare_operator<double>(g);
  // the previous call was the step after this one: its state's pressure is
  // what this forward solve recomputes, and its adjoint solution is close
  // to this one (initial guesses only: both solves still run to p_rtol)
  const bool chain = A.chain && A.dt_last == dt && std::fabs(A.t_last - (t_n + dt)) <= 1e-6 * dt;
  if (chain) copy_f64(s, N, A.pnext, g->p64);
  st = solve(g, g->p64, nullptr);
  if (st != TCF_OK && st != TCF_E_NOT_CONVERGED) return st;
  return backward_sweep(g, P, t_n, dt, state_n, adj_np1, adj_n, dL_dsigmaT, nullptr);
}

// One step of integrator 0 (FP64, two phases, no species) whose pressure
// p^{n+1} is given instead of solved for: S1-S5 and S8 exactly as step_once
// runs them, so with the pressure an earlier run of this step produced the
// state is bitwise that run's.  The pressure history is not advanced (it is
// marked empty, so a later solve starts from p^{n+1}).
tcf_status step_given_p(tcf_grid* g, double dt, const double* p_np1) {
  hipStream_t s = g->stream;
  Fields<double>& F = g->f64;
  KParams P = g->P;
  P.dt = dt;
  P.t = g->t;
  transport_stage<double>(P, s, F.a, F.T, F.a, F.T, F.u, F.v, F.w, F.a1, F.T1, 0.0, 1.0);
  transport_stage<double>(P, s, F.a1, F.T1, F.a, F.T, F.u, F.v, F.w, F.a2, F.T2, 0.75, 0.25);
  transport_stage<double>(P, s, F.a2, F.T2, F.a, F.T, F.u, F.v, F.w, F.a, F.T, 1.0 / 3.0, 2.0 / 3.0);
  if (!(g->cfg.flags & TCF_TRANSPORT_ONLY)) {
    geometry<double>(P, s, F.a, F.T, nullptr, F.sk, F.Mx, F.My, F.Mz);
    predictor<double>(P, s, F.a, F.sk, F.Mx, F.My, F.Mz, F.u, F.v, F.w, F.us, F.vs, F.ws);
    copy_f64(s, g->D.N, p_np1, g->p64);
    project<double>(P, s, F.a, g->p64, F.us, F.vs, F.ws, g->u64, g->v64, g->w64, nullptr, nullptr, nullptr);
    g->nhist = 0;
  }
  g->t += dt;
  HIPCHECK(hipGetLastError());
  return TCF_OK;
}

tcf_status tcf_step_keep(tcf_grid* g, double dt, double* const stages[4], const double* p_np1) {
  g_err.clear();
  tcf_status st = adj_checks(g);
  if (st != TCF_OK) return st;
  if (!stages || !stages[0] || !stages[1] || !stages[2] || !stages[3]) return fail(TCF_E_INVALID, "NULL stage pointer");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(TCF_E_INVALID, "dt must be positive and finite");
  if (!g->has_fields) return fail(TCF_E_STATE, "fields not set");
  // the step's transport writes its stage values into the caller's arrays
  // (nothing else in the step uses the grid's own stage arrays)
  Fields<double>& F = g->f64;
  double* const own[4] = {F.a1, F.T1, F.a2, F.T2};
  F.a1 = stages[0];
  F.T1 = stages[1];
  F.a2 = stages[2];
  F.T2 = stages[3];
  st = p_np1 ? step_given_p(g, dt, p_np1) : tcf_step(g, dt, 1, nullptr);
  F.a1 = own[0];
  F.T1 = own[1];
  F.a2 = own[2];
  F.T2 = own[3];
  return st;
}

tcf_status tcf_step_backward_kept(tcf_grid* g, double t_n, double dt, const double* const state_n[6],
                                  const double* const stages[4], const double* const state_np1[3],
                                  const double* const adj_np1[5], double* const adj_n[5], double* dL_dsigmaT) {
  g_err.clear();
  tcf_status st = backward_args(g, t_n, dt, state_n, adj_np1, adj_n, dL_dsigmaT);
  if (st != TCF_OK) return st;
  if (!stages || !stages[0] || !stages[1] || !stages[2] || !stages[3]) return fail(TCF_E_INVALID, "NULL stage pointer");
  if (!state_np1 || !state_np1[0] || !state_np1[1] || !state_np1[2])
    return fail(TCF_E_INVALID, "NULL pointer in state_np1");
  hipStream_t s = g->stream;
  Fields<double>& F = g->f64;
  const Dims& D = g->D;
  KParams P = g->P;
  P.dt = dt;
  P.t = t_n;
  const long N = D.N;
  // u^n (walls zeroed, as tcf_set_fields does) and alpha, T, p of step n+1
  copy_f64(s, D.Nu, state_n[2], g->u64);
  copy_f64(s, D.Nv, state_n[3], g->v64);
  if (D.dim == 3) copy_f64(s, D.Nw, state_n[4], g->w64);
  zero_walls<double>(P, s, g->u64, g->v64, g->w64);
  copy_f64(s, N, state_np1[0], F.a);
  copy_f64(s, N, state_np1[1], F.T);
  copy_f64(s, N, state_np1[2], g->p64);
  g->t = t_n;
  g->has_fields = true;
  g->nhist = 0;
  g->snhist = 0;
  // the geometry of step n+1 and the operator of alpha^{n+1}; the predictor,
  // the divergence and the forward solve are not needed
  geometry<double>(P, s, F.a, F.T, nullptr, F.sk, F.Mx, F.My, F.Mz);
  prepare_operator<double>(g);
  return backward_sweep(g, P, t_n, dt, state_n, adj_np1, adj_n, dL_dsigmaT, stages);
}

tcf_status tcf_adjoint_transport(tcf_grid* g, double dt, const double* ab_in, const double* Tb_in, double* ab_out,
                                 double* Tb_out, double* ub, double* vb, double* wb) {
  g_err.clear();
  tcf_status st = adj_checks(g);
  if (st != TCF_OK) return st;
  const Dims& D = g->D;
  if (!ab_in || !Tb_in || !ab_out || !Tb_out || !ub || !vb || (D.dim == 3 && !wb))
    return fail(TCF_E_INVALID, "NULL argument");
  if (ab_in == ab_out || Tb_in == Tb_out) return fail(TCF_E_INVALID, "input and output adjoints must not alias");
  if (!g->has_fields) return fail(TCF_E_STATE, "fields not set");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(TCF_E_INVALID, "bad dt");
  hipStream_t s = g->stream;
  Fields<double>& F = g->f64;
  auto& A = g->adj;
  KParams P = g->P;
  P.dt = dt;
  P.t = g->t;
  const long N = D.N;
  // stages from the current state, without touching it: stage 3 is not needed
  transport_stage<double>(P, s, F.a, F.T, F.a, F.T, F.u, F.v, F.w, F.a1, F.T1, 0.0, 1.0);
  transport_stage<double>(P, s, F.a1, F.T1, F.a, F.T, F.u, F.v, F.w, F.a2, F.T2, 0.75, 0.25);
  // the base state is read from copies (rk3_reverse reads a0/T0 after using sa/sT)
  copy_f64(s, N, F.a, A.pbar);
  copy_f64(s, N, F.T, A.y);
  A.chain = false;  // A.y no longer holds an adjoint pressure
  zero_adj_faces(g);
  rk3_reverse(g, P, A.pbar, A.y, ab_in, Tb_in, ab_out, Tb_out);
  zero_walls<double>(P, s, A.ub, A.vb, A.wb);
  copy_f64(s, D.Nu, A.ub, ub);
  copy_f64(s, D.Nv, A.vb, vb);
  if (D.dim == 3) copy_f64(s, D.Nw, A.wb, wb);
  HIPCHECK(hipGetLastError());
  return TCF_OK;
}

tcf_status tcf_adjoint_predictor(tcf_grid* g, double dt, const double* usb, const double* vsb, const double* wsb,
                                 double* ab, double* Tb, double* ub, double* vb, double* wb, double* sbar) {
  g_err.clear();
  tcf_status st = adj_checks(g);
  if (st != TCF_OK) return st;
  const Dims& D = g->D;
  if (!usb || !vsb || !ab || !Tb || !ub || !vb || !sbar || (D.dim == 3 && (!wsb || !wb)))
    return fail(TCF_E_INVALID, "NULL argument");
  if (!g->has_fields) return fail(TCF_E_STATE, "fields not set");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(TCF_E_INVALID, "bad dt");
  hipStream_t s = g->stream;
  Fields<double>& F = g->f64;
  auto& A = g->adj;
  KParams P = g->P;
  P.dt = dt;
  P.t = g->t;
  geometry<double>(P, s, F.a, F.T, nullptr, F.sk, F.Mx, F.My, F.Mz);
  fill_f64(s, D.N, A.ab, 0.0);
  fill_f64(s, D.N, A.Tb, 0.0);
  zero_adj_faces(g);
  predictor_reverse(g, P, usb, vsb, wsb);
  zero_walls<double>(P, s, A.ub, A.vb, A.wb);
  copy_f64(s, D.N, A.ab, ab);
  copy_f64(s, D.N, A.Tb, Tb);
  copy_f64(s, D.Nu, A.ub, ub);
  copy_f64(s, D.Nv, A.vb, vb);
  if (D.dim == 3) copy_f64(s, D.Nw, A.wb, wb);
  copy_f64(s, 1, g->scal + S_SBAR, sbar);
  HIPCHECK(hipGetLastError());
  return TCF_OK;
}

const char* tcf_last_error(void) { return g_err.c_str(); }

}  // extern "C"
