// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tcf {

// Constants of one launch, passed by value.  Material laws mix linearly in
// clamp(alpha, 0, 1); sigma(T) = sigma0 + s (T - T0).
struct KParams {
  int nx, ny, nz, dim;
  double h, ih, dt, t;
  double rho1, rho2, mu1, mu2, rhocp1, rhocp2, lam1, lam2;
  double sigma0, s, T0;
  double sc, c0;  // species: sigma += sc (c - c0) (sc = 0 without a species)
  // N-phase model (nph 3 or 4; 2 otherwise): material values of phases 3
  // and 4 (rho, mu, rho c_p, lambda) and per-pair sigma0 / dsigma/dT in the
  // order (1,2), (1,3), (1,4), (2,3), (2,4), (3,4)
  int nph;
  double mat34[4][2];
  double sig0p[6], dsigp[6];
  int Tbc[6];
  double Tw[6];
  double qP, qr, qx0, qy0, qvx, qvy;
  double weno_eps, neps;
};

// One multigrid level: face weights of K (the positive semi-definite
// negative of A), omega/diag, and work vectors.
template <class R>
struct Level {
  int nx, ny, nz;
  R *ax, *ay, *az, *wdiag;
  R *x, *x2, *b;
  __host__ __device__ long n() const { return (long)nx * ny * nz; }
};

// The coarse end of a V-cycle run by one block (levels of at most
// kTailCells cells): lv[0] the tail's first level, lv[nl - 1] the coarsest,
// solved by cinv (dense inverse) or csweeps damped-Jacobi sweeps of weight
// cj; pre- and post-smoothing weights, the coarse-correction weight omc;
// first_done: lv[0].x2 already holds the first pre-smoothing sweep.
constexpr int kTailLevels = 8, kTailCells = 1024, kTailNu = 8;
// LDS values of the tail: three vectors per level; a level holds at most a
// quarter of its parent's cells, so all levels below the first at most a third
constexpr int kTailLds = 3 * (kTailCells + kTailCells / 3 + 1);
template <class R>
struct MgTail {
  Level<R> lv[kTailLevels];
  int nl, nu, csweeps, first_done;
  const R* cinv;
  double wpre[kTailNu], wpost[kTailNu];
  double omc, cj;
};

// Finest level of the pressure operator: face weights recomputed from alpha,
// a_f = c2 / (rho_L + rho_R) with rho = rho1 + clamp(alpha, 0, 1) drho.
template <class R>
struct Fine {
  const R* a;
  int nx, ny, nz;
  double rho1, drho, c2;
};

// Slots of the device scalar block (FP64).
enum Slot { S_MEAN = 0, S_BB, S_RR, S_RZ, S_DQ, S_ALPHA, S_BETA, S_TOL2, S_SCALE,
            S_SUMA, S_AMIN, S_AMAX, S_UMAX, S_DIV2, S_NONFIN, S_RR64, S_BB64, S_PMEAN, S_SBAR, S_RZ2, S_NSLOT = 24 };
// Integer flags: done, iteration count.
enum IFlag { I_DONE = 0, I_ITERS = 1, I_NFLAG = 4 };
// r.z of the k-th preconditioned residual of a PCG solve (k = 0 after the
// first preconditioner application): the slots alternate, so that a kernel
// can write rz_k while every block still reads rz_(k-1)
__host__ __device__ inline int rz_slot(int k) { return (k & 1) ? S_RZ2 : S_RZ; }
enum FinOp { F_STORE = 0, F_MEAN, F_BB, F_RR, F_MIN, F_MAX, F_SCALE };

constexpr int kBlock = 256;
constexpr int kCoarseDenseMax = 512;  // coarsest levels up to this size are solved exactly
inline int nblocks_cells(int nx, int ny, int nz) { return ((nx + 63) / 64) * ((ny + 3) / 4) * nz; }

// ---- launchers (defined in tcf_kernels.hip) --------------------------------
template <class R>
void transport_stage(const KParams& P, hipStream_t s, const R* a, const R* T, const R* ab, const R* Tb,
                     const R* u, const R* v, const R* w, R* ao, R* To, double cb, double ci);
// One SSP-RK3 stage of a passive cell field (the species) with alpha's
// transport: qo = cb qb + ci (q + dt L(q)).
template <class R>
void transport_scalar(const KParams& P, hipStream_t s, const R* q, const R* qb, const R* u, const R* v, const R* w,
                      R* qo, double cb, double ci);
// One SSP-RK3 stage of T alone with cell materials (the N-phase mixture):
// lam the conductivity, rcp the heat capacity rho c_p, dq the interface
// delta of the heat source (read only with P.qP != 0).
template <class R>
void transport_temperature(const KParams& P, hipStream_t s, const R* lam, const R* rcp, const R* dq, const R* T,
                           const R* Tb, const R* u, const R* v, const R* w, R* To, double cb, double ci);
template <class R>
// c: species field or NULL (no solutal term)
void geometry(const KParams& P, hipStream_t s, const R* a, const R* T, const R* c, R* sk, R* Mx, R* My, R* Mz);
template <class R>
void predictor(const KParams& P, hipStream_t s, const R* a, const R* sk, const R* Mx, const R* My,
               const R* Mz, const R* u, const R* v, const R* w, R* us, R* vs, R* ws);
// b = D u* / dt in FP64, per-block partial sums of b -> part
template <class R>
void divergence_rhs(const KParams& P, hipStream_t s, const R* us, const R* vs, const R* ws, double* b,
                    double* part);
// fine-level face weights (FP64) from alpha; optional FP32 copies
template <class R>
void face_weights(const KParams& P, hipStream_t s, const R* a, double* ax, double* ay, double* az,
                  float* fx, float* fy, float* fz);
template <class R>
void make_wdiag(hipStream_t s, int dim, const Level<R>& L, double omega);
// Galerkin weights of the coarse level C from the level F below it, and
// C's 1/diag, in one pass
template <class R>
void coarsen_weights(hipStream_t s, int dim, const Level<R>& F, const Level<R>& C);
// the same for level 1 straight from alpha (the fine weights are not stored)
template <class R>
void coarsen_from_alpha(const KParams& P, hipStream_t s, const R* a, const Level<R>& C);

// PCG / multigrid building blocks on a level; all partial sums in FP64
template <class R>
void rhs_resid(hipStream_t s, int dim, const Level<R>& L, const double* b, const double* scal, R* x, R* r,
               double* part_bb, double* part_rr);
template <class R>
void spmv_dot(hipStream_t s, int dim, const Level<R>& L, const R* d, R* q, double* part,
              const int* iflag);
template <class R>
void update_xr(hipStream_t s, long n, const double* scal, R* x, R* r, const R* d, const R* q, double* part, const int* iflag);
template <class R>
void update_d(hipStream_t s, long n, const double* scal, const R* z, R* d, int first, const int* iflag);
template <class R>
void mg_smooth_first(hipStream_t s, const Level<R>& L, const R* b, R* x, double om, const int* iflag);
template <class R>
void mg_smooth(hipStream_t s, int dim, const Level<R>& L, const R* b, const R* x, R* xo, double om, double* part_rz,
               const int* iflag);
template <class R>
void mg_resid_restrict(hipStream_t s, int dim, const Level<R>& F, const R* b, const R* x, R* bc, const R* wdc,
                       R* x1c, double om0, const int* iflag);
template <class R>
void mg_prolong_smooth(hipStream_t s, int dim, const Level<R>& F, const Level<R>& C, const R* b, const R* x,
                       R* xo, double omega_c, double om, double* part_rz, const int* iflag);
// Levels whose two pre-sweeps' second sweep, residual and restriction, and
// whose prolongation and two post-sweeps, run as one launch each (levels
// of at most this many cells, where a kernel costs its launch)
bool mg_fused_level(long n);
template <class R>
void mg_sweep_restrict(hipStream_t s, int dim, const Level<R>& F, const R* b, const R* x, R* xo, R* bc,
                       const R* wdc, R* x1c, double om, double om0, const int* iflag);
template <class R>
void mg_prolong_sweep2(hipStream_t s, int dim, const Level<R>& F, const Level<R>& C, const R* b, const R* x, R* xo,
                       double omega_c, double om1, double om2, const int* iflag);
template <class R>
void mg_coarse_solve(hipStream_t s, int dim, const Level<R>& L, const R* b, R* x, int sweeps, double om,
                     const int* iflag);

// finest-level fused kernels (tcf_fine.hip); return the number of partials
int fine_blocks(int nx, int ny, int nz);
// the inner solve's first sweep from the FP64 residual: r32 = r64 / scale
// (scal[S_SCALE]) written, z1 = omega r32 / diag, partials of |r32|^2
int fine_smooth_first64(hipStream_t s, int dim, const Fine<float>& F, double omega, const double* r64,
                        const double* scal, float* r32, float* z1, double* part);
// r = -(b - mean) - K p in FP64 with the fine weights recomputed from alpha
// (densities rho1 + clamp(alpha)(rho2 - rho1) of P); block partials of
// ||rhs||^2 and ||r||^2
template <class R>
int resid64a(const KParams& P, hipStream_t s, const R* a, const double* b, const double* scal, const double* p,
             double* r, double* pbb, double* prr);
template <class R>
int fine_spmv_upd(hipStream_t s, int dim, const Fine<R>& F, const R* z, const R* dold, R* dnew, double* scal,
                  int it, const double* rzpart, int nrz, double* part, const int* iflag);
template <class R>
int fine_update_smooth(hipStream_t s, int dim, const Fine<R>& F, double omega, double* scal, int it, int xzero, R* x,
                       R* r, const R* d, R* z1, const double* dqpart, int ndq, double* part, const int* iflag);
template <class R>
void fine_smooth_first(hipStream_t s, int dim, const Fine<R>& F, double omega, const R* b, R* z1, const int* iflag);
template <class R>
int fine_smooth(hipStream_t s, int dim, const Fine<R>& F, double omega, const R* b, const R* x, R* xo, const R* e,
                int cnx, int cny, double omc, double* part, const int* iflag);
// two sweeps (om1 then om2; the first on x + omc P e when e is given) in one
// pass, FP32 3-D; xo must not alias x
int fine_smooth2(hipStream_t s, const Fine<float>& F, double om1, double om2, const float* b, const float* x,
                 float* xo, const float* e, int cnx, int cny, double omc, double* part, const int* iflag);
template <class R>
// bc = R (b - K0 x); with x1c also x1c = om0 wdc bc (the coarse level's first sweep)
void fine_resid_restrict(hipStream_t s, int dim, const Fine<R>& F, const R* b, const R* x, R* bc, const R* wdc, R* x1c,
                         double om0, const int* iflag);

// exact coarsest-level solve (levels with at most kCoarseDenseMax cells)
template <class R>
void coarse_factor(hipStream_t s, int dim, const Level<R>& L, double* A, R* Minv);
template <class R>
void coarse_apply(hipStream_t s, int n, const R* Minv, const R* b, R* out, const int* iflag);
template <class R>
void mg_tail(hipStream_t s, int dim, const MgTail<R>& T, const int* iflag);

void finalize(hipStream_t s, const double* part, int nparts, double* scal, int* iflag, int op, int slot,
              double arg);
// Two finalizes of nparts partials each in one launch (one block each); the
// two must write different slots.
void finalize2(hipStream_t s, const double* part0, const double* part1, int nparts, double* scal, int* iflag,
               int op0, int slot0, double arg0, int op1, int slot1, double arg1);
void init_flags(hipStream_t s, int* iflag);
// Copies nwords 8-byte words from device memory src to host-coherent memory
// dst (device-visible), then stores value into *ticket (host memory), in
// that order as seen by the host; then clears the flags at reset_flags
// (I_NFLAG ints, the copy holds their values before) unless it is null.
void publish(hipStream_t s, const void* src, int nwords, void* dst, unsigned* ticket, unsigned value,
             int* reset_flags = nullptr);

// FP64 refinement helpers (FP32 mode)
// r32 = r / scal[S_SCALE]; part: nblocks(256) partials of |r32|^2
void scale_to32(hipStream_t s, long n, const double* r, const double* scal, float* r32, double* part);
// p += scal[S_SCALE] e; part: nblocks(256) partials of the new p, as
// sum64_partials(p) gives them; returns their number
int add_scaled(hipStream_t s, long n, const float* e, const double* scal, double* p, double* part);
void subtract_mean(hipStream_t s, long n, const double* scal, int slot, double* p);
int sum64_partials(hipStream_t s, long n, const double* x, double* part);
template <class R>
int dot_partials(hipStream_t s, long n, const R* x, const R* y, double* part);
template <class R>
void fill(hipStream_t s, long n, R* y, double v);

template <class R>
void project(const KParams& P, hipStream_t s, const R* a, const double* p, const R* us, const R* vs,
             const R* ws, double* u, double* v, double* w, R* ur, R* vr, R* wr);
// S8 and the diagnostics in one pass: the projection on the density fraction
// arho (mixed over [P.rho1, P.rho2]), the diagnostics of the volume fraction
// a on the projected velocity, as diagnostics() computes them
template <class R>
void project_diag(const KParams& P, hipStream_t s, const R* arho, const R* a, const double* p, const R* us,
                  const R* vs, const R* ws, double* u, double* v, double* w, R* ur, R* vr, R* wr, double* part,
                  int stride, double* scal);
// per-block partials of the six diagnostics (stride apart, at most stride
// blocks) reduced into scal[S_SUMA .. S_NONFIN]
template <class R>
void diagnostics(const KParams& P, hipStream_t s, const R* a, const double* u, const double* v,
                 const double* w, double* part, int stride, double* scal);

// adjoint (tcf_adjoint.hip), FP64
void adj_project(const KParams& P, hipStream_t s, const double* a, const double* p, const double* ub,
                 const double* vb, const double* wb, double* pbar, double* abar);
void adj_poisson_alpha(const KParams& P, hipStream_t s, const double* a, const double* p, const double* y,
                       double* abar);
void adj_rhs(const KParams& P, hipStream_t s, const double* ubp, const double* vbp, const double* wbp,
             const double* y, double* usb, double* vsb, double* wsb);
void adj_predictor(const KParams& P, hipStream_t s, const double* a, const double* sk, const double* Mx,
                   const double* My, const double* Mz, const double* u, const double* v, const double* w,
                   const double* usb, const double* vsb, const double* wsb, double* ubar, double* vbar,
                   double* wbar, double* abar, double* skbar, double* Mxb, double* Myb, double* Mzb,
                   double* vsum);
int adj_geometry(const KParams& P, hipStream_t s, const double* a, const double* T, const double* skb,
                 const double* Mxb, const double* Myb, const double* Mzb, double* Tbar, double* nbx, double* nby,
                 double* nbz, double* dsb, double* abar, double* spart);
void adj_transport_stage(const KParams& P, hipStream_t s, const double* a, const double* T, const double* u,
                         const double* v, const double* w, const double* wa, const double* wT, double* ab,
                         double* Tb, double* ub, double* vb, double* wb);
void adj_scale(hipStream_t s, long n, double f, const double* x, double* y);
void adj_axpy(hipStream_t s, long n, double f, const double* x, double* y);
void adj_add_scalar(hipStream_t s, double* dst, const double* src);

// N-phase model (tcf_nphase.hip).  Mixture per cell from the fractions of
// phases 2..N: the density and the viscosity as fractions of [rlo, rhi]
// and [mlo, mhi]; or (thermal) rho c_p, lambda and, with a heat source, the
// interface delta of the condensed fraction 1 - alpha_1.  Per-pair
// sigma*kappa (pair-major) and the summed Marangoni vector; the face CSF
// force.  a4 = NULL with three phases.
template <class R>
void np_mixture(const KParams& P, hipStream_t s, const R* a2, const R* a3, const R* a4, R* arho, R* amu, double rlo,
                double rhi, double mlo, double mhi);
template <class R>
void np_mixture_thermal(const KParams& P, hipStream_t s, const R* a2, const R* a3, const R* a4, R* rcp, R* lam,
                        R* dq);
// (nrm: 3 N per pair, dsp: N per pair; scratch of the two geometry passes)
template <class R>
void np_geometry(const KParams& P, hipStream_t s, const R* a2, const R* a3, const R* a4, const R* T, R* nrm, R* dsp,
                 R* skp, R* Mx, R* My, R* Mz);
template <class R>
void np_face_force(const KParams& P, hipStream_t s, const R* a2, const R* a3, const R* a4, const R* skp, const R* Mx,
                   const R* My, const R* Mz, R* fx, R* fy, R* fz);
// the predictor in its material form: amu the viscosity as a fraction of
// [P.mu1, P.mu2], arho the density as a fraction of [P.rho1, P.rho2], and
// the face CSF force fx, fy, fz on the faces
template <class R>
void predictor_mat(const KParams& P, hipStream_t s, const R* amu, const R* arho, const R* fx, const R* fy,
                   const R* fz, const R* u, const R* v, const R* w, R* us, R* vs, R* ws);

// SSP-RK3 stage combination of a face velocity with the FP64 base velocity
// (stage 1: 3/4 base + 1/4 x; stage 2: base/3 + 2/3 x), in place
template <class R>
void rk_combine(hipStream_t s, long n, int stage, const double* base, R* x);

// conversions
void to_f32(hipStream_t s, long n, const double* x, float* y);
void to_f64(hipStream_t s, long n, const float* x, double* y);
void copy_f64(hipStream_t s, long n, const double* x, double* y);
// out = the extrapolation in time of order m (1 or 2) through p and the
// previous pressures h1 = p^(n-1), h2 = p^(n-2): 2 p - h1, or 3 p - 3 h1 +
// h2 (out may be h1 or h2; h2 is not read for m = 1)
void extrapolate_f64(hipStream_t s, long n, int m, const double* p, const double* h1, const double* h2, double* out);
void fill_f64(hipStream_t s, long n, double* y, double v);
template <class R>
void zero_walls(const KParams& P, hipStream_t s, R* u, R* v, R* w);

}  // namespace tcf
