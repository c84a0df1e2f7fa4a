// Discrete adjoint of one projection step (FP64).
//
// Each kernel recomputes the forward local quantities it needs (WENO5 weights
// and smoothness indicators included; nothing of the forward stencils is
// stored) and applies the transposed local Jacobian.  Contributions that
// several outputs make to one input are accumulated with FP64 vector atomics,
// so adjoint sums are not bitwise reproducible run to run (rounding order).
// Non-smooth points take a fixed branch: the upwind choice follows the sign
// of the advecting velocity (zero takes the left-biased stencil, as in the
// forward step) and the derivative of clamp(alpha, 0, 1) is 1 inside (0, 1)
// and 0 elsewhere.
#include "tcf_device.h"
#include "tcf_internal.h"

namespace tcf {
namespace {

using namespace dev;

__device__ __forceinline__ double dclamp(double a) { return (a > 0.0 && a < 1.0) ? 1.0 : 0.0; }
__device__ __forceinline__ void aadd(double* p, double v) {
  if (v != 0.0) atomicAdd(p, v);
}

// ---- ghost-aware index maps: value = sign * array[index] (+ a constant) ----
template <int DIM>
__device__ __forceinline__ long a_idx(int i, int j, int k, int nx, int ny, int nz) {
  return cidx(refl(i, nx), refl(j, ny), DIM == 3 ? refl(k, nz) : 0, nx, ny);
}
template <int DIM>
__device__ __forceinline__ long t_idx(int i, int j, int k, const KParams& P, double& sg) {
  sg = 1.0;
  if (i < 0 && P.Tbc[0]) sg = -sg;
  if (i >= P.nx && P.Tbc[1]) sg = -sg;
  if (j < 0 && P.Tbc[2]) sg = -sg;
  if (j >= P.ny && P.Tbc[3]) sg = -sg;
  if (DIM == 3) {
    if (k < 0 && P.Tbc[4]) sg = -sg;
    if (k >= P.nz && P.Tbc[5]) sg = -sg;
  }
  return a_idx<DIM>(i, j, k, P.nx, P.ny, P.nz);
}
template <int C, int DIM>
__device__ __forceinline__ long v_idx(int i, int j, int k, int nx, int ny, int nz, double& sg) {
  sg = 1.0;
  int id[3] = {i, j, k};
  const int n[3] = {nx, ny, nz};
#pragma unroll
  for (int e = 0; e < DIM; ++e) {
    if (e == C) {
      if (id[e] < 0) { id[e] = -id[e]; sg = -sg; }
      else if (id[e] > n[e]) { id[e] = 2 * n[e] - id[e]; sg = -sg; }
    } else {
      if (id[e] < 0) { id[e] = -1 - id[e]; sg = -sg; }
      else if (id[e] >= n[e]) { id[e] = 2 * n[e] - 1 - id[e]; sg = -sg; }
    }
  }
  if (DIM == 2) id[2] = 0;
  return fidx<C>(id[0], id[1], id[2], nx, ny);
}

// WENO5-JS value at the right edge of c and its gradient w.r.t. (a,b,c,d,e):
// dW/dx = sum_k w_k dq_k/dx - (2/S) sum_k (q_k - W) a_k/(eps+beta_k) dbeta_k/dx
__device__ double weno5_g(double a, double b, double c, double d, double e, double eps, double g[5]) {
  const double q0 = (2.0 * a - 7.0 * b + 11.0 * c) * (1.0 / 6.0);
  const double q1 = (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
  const double q2 = (2.0 * c + 5.0 * d - e) * (1.0 / 6.0);
  const double t0 = a - 2.0 * b + c, u0 = a - 4.0 * b + 3.0 * c;
  const double t1 = b - 2.0 * c + d, u1 = b - d;
  const double t2 = c - 2.0 * d + e, u2 = 3.0 * c - 4.0 * d + e;
  const double e0 = eps + ((13.0 / 12.0) * t0 * t0 + 0.25 * u0 * u0);
  const double e1 = eps + ((13.0 / 12.0) * t1 * t1 + 0.25 * u1 * u1);
  const double e2 = eps + ((13.0 / 12.0) * t2 * t2 + 0.25 * u2 * u2);
  // four reciprocals (1/e_k, 1/S), the rest by multiplication
  const double ie0 = 1.0 / e0, ie1 = 1.0 / e1, ie2 = 1.0 / e2;
  const double a0 = 0.1 * ie0 * ie0, a1 = 0.6 * ie1 * ie1, a2 = 0.3 * ie2 * ie2;
  const double S = a0 + a1 + a2, iS = 1.0 / S;
  const double W = (a0 * q0 + a1 * q1 + a2 * q2) * iS;
  const double w0 = a0 * iS, w1 = a1 * iS, w2 = a2 * iS;
  // coefficients c_k = -(2/S)(q_k - W) a_k / e_k multiply dbeta_k/dx
  const double c0 = -2.0 * iS * (q0 - W) * a0 * ie0;
  const double c1 = -2.0 * iS * (q1 - W) * a1 * ie1;
  const double c2 = -2.0 * iS * (q2 - W) * a2 * ie2;
  // dbeta0/d(a,b,c) = 13/6 t0 (1,-2,1) + 1/2 u0 (1,-4,3)
  const double b0a = (13.0 / 6.0) * t0 + 0.5 * u0, b0b = -(13.0 / 3.0) * t0 - 2.0 * u0,
               b0c = (13.0 / 6.0) * t0 + 1.5 * u0;
  // dbeta1/d(b,c,d) = 13/6 t1 (1,-2,1) + 1/2 u1 (1,0,-1)
  const double b1b = (13.0 / 6.0) * t1 + 0.5 * u1, b1c = -(13.0 / 3.0) * t1, b1d = (13.0 / 6.0) * t1 - 0.5 * u1;
  // dbeta2/d(c,d,e) = 13/6 t2 (1,-2,1) + 1/2 u2 (3,-4,1)
  const double b2c = (13.0 / 6.0) * t2 + 1.5 * u2, b2d = -(13.0 / 3.0) * t2 - 2.0 * u2,
               b2e = (13.0 / 6.0) * t2 + 0.5 * u2;
  g[0] = w0 * (2.0 / 6.0) + c0 * b0a;
  g[1] = w0 * (-7.0 / 6.0) + w1 * (-1.0 / 6.0) + c0 * b0b + c1 * b1b;
  g[2] = w0 * (11.0 / 6.0) + w1 * (5.0 / 6.0) + w2 * (2.0 / 6.0) + c0 * b0c + c1 * b1c + c2 * b2c;
  g[3] = w1 * (2.0 / 6.0) + w2 * (5.0 / 6.0) + c1 * b1d + c2 * b2d;
  g[4] = w2 * (-1.0 / 6.0) + c2 * b2e;
  return W;
}

// q[k] = Q(f-3+k), k = 0..5; upwind value at face f and its gradient gq[0..5].
// The stencil is picked by the sign before the one evaluation (and the
// gradient mapped back), so the lanes of a wavefront with both signs share it.
__device__ __forceinline__ double upwind_g(const double* q, double vel, double eps, double gq[6]) {
  double g[5];
  const bool pos = vel >= 0.0;
  const double W = weno5_g(pos ? q[0] : q[5], pos ? q[1] : q[4], pos ? q[2] : q[3], pos ? q[3] : q[2],
                           pos ? q[4] : q[1], eps, g);
  gq[0] = pos ? g[0] : 0.0;
  gq[1] = pos ? g[1] : g[4];
  gq[2] = pos ? g[2] : g[3];
  gq[3] = pos ? g[3] : g[2];
  gq[4] = pos ? g[4] : g[1];
  gq[5] = pos ? 0.0 : g[0];
  return W;
}

__device__ __forceinline__ double mix1(double a, double p1, double p2) {
  const double ac = a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
  return p1 + ac * (p2 - p1);
}

// ===========================================================================
// S8^T: projection.  Per cell (gather over its faces): pbar = dU'/dp^T ubar',
// abar += d(beta_f)/d(alpha) terms.  u'_f = u*_f - dt beta_f (p_R - p_L)/h.
template <int DIM>
__global__ __launch_bounds__(256) void ka_project(KParams P, const double* __restrict__ a, const double* __restrict__ p,
                                                  const double* __restrict__ ub, const double* __restrict__ vb,
                                                  const double* __restrict__ wb, double* __restrict__ pbar,
                                                  double* __restrict__ abar) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  if (i >= nx || j >= ny) return;
  const long c = cidx(i, j, k, nx, ny);
  const double ac = a[c], rc = mix1(ac, P.rho1, P.rho2), drc = (P.rho2 - P.rho1) * dclamp(ac);
  double pb = 0.0, ab = 0.0;
  const int id[3] = {i, j, k};
  const int nn[3] = {nx, ny, nz};
  const double* ubs[3] = {ub, vb, wb};
  for (int d = 0; d < DIM; ++d) {
    for (int side = 0; side < 2; ++side) {
      // side 0: low face (c is R), side 1: high face (c is L)
      const int fpos = id[d] + side;
      if (fpos == 0 || fpos == nn[d]) continue;
      int o[3] = {0, 0, 0};
      o[d] = side ? 1 : -1;
      const long cn = cidx(i + o[0], j + o[1], k + o[2], nx, ny);
      int fi[3] = {i, j, k};
      fi[d] = fpos;
      long f;
      if (d == 0) f = fidx<0>(fi[0], fi[1], fi[2], nx, ny);
      else if (d == 1) f = fidx<1>(fi[0], fi[1], fi[2], nx, ny);
      else f = fidx<2>(fi[0], fi[1], fi[2], nx, ny);
      const double ubar = ubs[d][f];
      const double rn = mix1(a[cn], P.rho1, P.rho2);
      const double beta = 1.0 / (0.5 * (rc + rn));
      // c is R on its low face, L on its high face
      const double pR = side ? p[cn] : p[c], pL = side ? p[c] : p[cn];
      pb += (side ? 1.0 : -1.0) * P.dt * beta * ubar * P.ih;
      const double dbeta = -beta * beta * 0.5 * drc;
      ab += ubar * (-P.dt * (pR - pL) * P.ih) * dbeta;
    }
  }
  pbar[c] = pb;
  abar[c] += ab;
}

// Poisson operator term: abar += sum_f dbeta_f/dalpha (p_R - p_L)(y_R - y_L)/h^2
template <int DIM>
__global__ __launch_bounds__(256) void ka_poisson_alpha(KParams P, const double* __restrict__ a,
                                                        const double* __restrict__ p, const double* __restrict__ y,
                                                        double* __restrict__ abar) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  if (i >= nx || j >= ny) return;
  const long c = cidx(i, j, k, nx, ny);
  const double ac = a[c], rc = mix1(ac, P.rho1, P.rho2), drc = (P.rho2 - P.rho1) * dclamp(ac);
  const int id[3] = {i, j, k};
  const int nn[3] = {nx, ny, nz};
  double ab = 0.0;
  for (int d = 0; d < DIM; ++d)
    for (int side = 0; side < 2; ++side) {
      const int fpos = id[d] + side;
      if (fpos == 0 || fpos == nn[d]) continue;
      int o[3] = {0, 0, 0};
      o[d] = side ? 1 : -1;
      const long cn = cidx(i + o[0], j + o[1], k + o[2], nx, ny);
      const double rn = mix1(a[cn], P.rho1, P.rho2);
      const double beta = 1.0 / (0.5 * (rc + rn));
      const double dbeta = -beta * beta * 0.5 * drc;
      // (p_R - p_L)(y_R - y_L) is the same product from either side
      ab += dbeta * (p[cn] - p[c]) * (y[cn] - y[c]) * P.ih * P.ih;
    }
  abar[c] += ab;
}

// ubar* on interior faces: ubar' + (y_L - y_R)/(h dt); zero on walls
template <int DIM, int D>
__global__ __launch_bounds__(256) void ka_rhs_face(KParams P, const double* __restrict__ ubp,
                                                   const double* __restrict__ y, double* __restrict__ usb) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int fnx = nx + (D == 0), fny = ny + (D == 1);
  if (i >= fnx || j >= fny) return;
  const int id[3] = {i, j, k};
  const int nD = D == 0 ? nx : (D == 1 ? ny : nz);
  const long f = fidx<D>(i, j, k, nx, ny);
  if (id[D] == 0 || id[D] == nD) {
    usb[f] = 0.0;
    return;
  }
  int L[3] = {i, j, k};
  L[D] -= 1;
  const long cL = cidx(L[0], L[1], L[2], nx, ny), cR = cidx(i, j, k, nx, ny);
  usb[f] = ubp[f] + (y[cL] - y[cR]) * P.ih / P.dt;
}

// ===========================================================================
// (S4-S5)^T: the predictor on interior faces.
// ---------------------------------------------------------------------------
// The predictor's adjoint in two parts, with the scattered sums of the flux
// terms gathered in LDS first (one kernel doing all of it per face issued
// ~50 FP64 atomics per face at 176 VGPRs, two waves per SIMD).
//
// ka_pred_face<DIM, D>: the terms that do not depend on a flux direction:
// the direct term u*_f = u_f + ..., the CSF force (sigma kappa, M and the
// alpha difference), and the face density 1/rho_f (whose derivative needs
// the forward viscous term: the direction kernels below leave it, summed
// over the directions in their order, in vsum).  One thread per cell
// gathers the terms of its two D-faces into its own sigma kappa, M and
// alpha adjoints (each face's terms recomputed by both of its cells), and
// the cell after a face adds that face's direct term: no atomics.

// Box over a block's faces (one LDS array of doubles): origin and extent in
// the virtual index space of the target array (ghost positions included).
struct Box {
  int o[3], e[3];
  __device__ int n() const { return e[0] * e[1] * e[2]; }
  __device__ int at(int x, int y, int z) const { return ((z - o[2]) * e[1] + (y - o[1])) * e[0] + (x - o[0]); }
  __device__ void pos(int q, int& x, int& y, int& z) const {
    x = o[0] + q % e[0];
    y = o[1] + (q / e[0]) % e[1];
    z = o[2] + q / (e[0] * e[1]);
  }
};

template <int DIM, int D>
__global__ __launch_bounds__(256) void ka_pred_face(KParams P, const double* __restrict__ a,
                                                    const double* __restrict__ sk, const double* __restrict__ M,
                                                    const double* __restrict__ vsum, const double* __restrict__ usb,
                                                    double* __restrict__ udb, double* __restrict__ abar,
                                                    double* __restrict__ skbar, double* __restrict__ Mbar) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  if (i >= nx || j >= ny) return;
  const int id[3] = {i, j, k};
  const int nD = D == 0 ? nx : (D == 1 ? ny : nz);
  const double ih = P.ih, dt = P.dt;
  const long c = cidx(i, j, k, nx, ny);
  double skb = 0.0, Mb = 0.0, ab = 0.0;
  // side 0: the face below the cell (the cell is its R), side 1: the face above (L)
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int fD = id[D] + side;
    if (fD == 0 || fD == nD) continue;  // wall faces carry no terms
    int F[3] = {i, j, k};
    F[D] = fD;
    const long fo = fidx<D>(F[0], F[1], F[2], nx, ny);
    const double ob = usb[fo];
    if (ob == 0.0) continue;
    int L[3] = {F[0], F[1], F[2]};
    L[D] -= 1;
    const long cL = cidx(L[0], L[1], L[2], nx, ny), cR = cidx(F[0], F[1], F[2], nx, ny);
    const double aL = a[cL], aR = a[cR];
    const double fst = 0.5 * (sk[cL] + sk[cR]) * (aR - aL) * ih + 0.5 * (M[cL] + M[cR]);
    const double rhof = 0.5 * (mix1(aL, P.rho1, P.rho2) + mix1(aR, P.rho1, P.rho2));
    const double visc = vsum[fo];  // the forward viscous term, summed over the directions by ka_pred_dir
    if (side == 0) udb[fo] += ob;  // direct term, added once by the cell after the face
    const double fstb = dt * ob / rhof;
    const double rhofb = -dt * ob * (visc + fst) / (rhof * rhof);
    skb += fstb * 0.5 * (aR - aL) * ih;
    Mb += 0.5 * fstb;
    if (side == 0) ab += rhofb * 0.5 * (P.rho2 - P.rho1) * dclamp(aR) + fstb * 0.5 * (sk[cL] + sk[cR]) * ih;
    else ab += rhofb * 0.5 * (P.rho2 - P.rho1) * dclamp(aL) - fstb * 0.5 * (sk[cL] + sk[cR]) * ih;
  }
  skbar[c] += skb;
  Mbar[c] += Mb;
  abar[c] += ab;
}

// ka_pred_dir<DIM, D, E>: per face of component D, the reverse of its
// convective and viscous fluxes along axis E: the WENO5 gradients of the
// advected values (the seven D-faces along E), the advecting velocity of
// component E (E != D) and the viscosities.  A block is 64 faces along x
// times 4 along y (E = x) or 8 along E (E = y, z); the contributions to the
// D-faces, the E-faces and the cells are gathered in LDS boxes over the
// block's stencil (virtual positions, ghosts included) and sent to memory
// with one global atomic per box entry through the ghost rules.
template <int DIM, int D, int E>
__global__ __launch_bounds__(256) void ka_pred_dir(KParams P, const double* __restrict__ a,
                                                   const double* __restrict__ ud, const double* __restrict__ ue,
                                                   const double* __restrict__ usb, double* __restrict__ udb,
                                                   double* __restrict__ ueb, double* __restrict__ abar,
                                                   double* __restrict__ vsum) {
  constexpr int BYE = E == 0 ? 4 : 4;  // threads across the x rows
  constexpr int NB = 64 * BYE;
  // the block's faces: x in [x0, x0+64), and 4 along y (E = 0, 1) or z (E = 2)
  const int x0 = blockIdx.x * 64;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + 64 * ty;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  int f0[3], fe[3];  // block's face range (component D index space): origin, extent
  f0[0] = x0;
  fe[0] = 64;
  if (E == 2) {
    f0[1] = blockIdx.y; fe[1] = 1;
    f0[2] = blockIdx.z * BYE; fe[2] = BYE;
  } else {
    f0[1] = blockIdx.y * BYE; fe[1] = BYE;
    f0[2] = blockIdx.z; fe[2] = 1;
  }
  // boxes: D-faces extended by 3 along E; E-faces extended by -1 along D and
  // +1 along E; cells extended by -1 along D and -1..+1 along E
  Box bu, bv, bc;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    bu.o[d] = f0[d] - (d == E ? 3 : 0);
    bu.e[d] = fe[d] + (d == E ? 6 : 0);
    bv.o[d] = f0[d] - (d == D ? 1 : 0);
    bv.e[d] = fe[d] + (d == D ? 1 : 0) + (d == E ? 1 : 0);
    bc.o[d] = f0[d] - (d == D ? 1 : 0) - (d == E && E != D ? 1 : 0);
    bc.e[d] = fe[d] + (d == D ? 1 : 0) + (d == E && E != D ? 2 : 0);
  }
  // sizes: bu <= 70 x 4 or 64 x 10; bv, bc <= 66 x 6 x 2
  __shared__ double su[70 * 10], sv[66 * 6 * 2], sc[66 * 6 * 2];
  const int nu = bu.n(), nvv = E != D ? bv.n() : 0, ncc = bc.n();
  for (int q = tid; q < nu; q += NB) su[q] = 0.0;
  for (int q = tid; q < nvv; q += NB) sv[q] = 0.0;
  for (int q = tid; q < ncc; q += NB) sc[q] = 0.0;
  __syncthreads();
  const int i = x0 + tx, j = E == 2 ? f0[1] : f0[1] + ty, k = E == 2 ? f0[2] + ty : f0[2];
  const int id[3] = {i, j, k};
  const int fnx = nx + (D == 0), fny = ny + (D == 1), fnz = (DIM == 3 ? nz : 1) + (D == 2);
  const int nD = D == 0 ? nx : (D == 1 ? ny : nz);
  const bool act = i < fnx && j < fny && k < fnz && id[D] > 0 && id[D] < nD;
  const double ob = act ? usb[fidx<D>(i, j, k, nx, ny)] : 0.0;
  if (act && ob != 0.0) {
    const double eps = P.weno_eps, ih = P.ih, dt = P.dt;
    int L[3] = {i, j, k};
    L[D] -= 1;
    const long cL = cidx(L[0], L[1], L[2], nx, ny), cR = cidx(i, j, k, nx, ny);
    const double aL = a[cL], aR = a[cR];
    const double rhof = 0.5 * (mix1(aL, P.rho1, P.rho2) + mix1(aR, P.rho1, P.rho2));
    const double convb = -dt * ob, viscb = dt * ob / rhof;
    const double Fhib = convb * ih, Flob = -convb * ih;
    const double thib = viscb * ih, tlob = -viscb * ih;
    const double dmu = P.mu2 - P.mu1;
    double vpart = 0.0;  // this direction's part of the forward viscous term
    // the seven D-faces along E (virtual offsets -3..3) and their values
    double q[7], qb[7];
    for (int m = 0; m < 7; ++m) {
      int o[3] = {i, j, k};
      o[E] += m - 3;
      double sg;
      const long qi = v_idx<D, DIM>(o[0], o[1], o[2], nx, ny, nz, sg);
      q[m] = sg * ud[qi];
      qb[m] = 0.0;
    }
    if (E == D) {
      const double Ulo = 0.5 * (q[2] + q[3]), Uhi = 0.5 * (q[3] + q[4]);
      double g[6];
      double W = upwind_g(q, Ulo, eps, g);
      double Ub = Flob * W;
      for (int m = 0; m < 6; ++m) qb[m] += Flob * Ulo * g[m];
      qb[2] += 0.5 * Ub;
      qb[3] += 0.5 * Ub;
      W = upwind_g(q + 1, Uhi, eps, g);
      Ub = Fhib * W;
      for (int m = 0; m < 6; ++m) qb[m + 1] += Fhib * Uhi * g[m];
      qb[3] += 0.5 * Ub;
      qb[4] += 0.5 * Ub;
      const double mL = mix1(aL, P.mu1, P.mu2), mR = mix1(aR, P.mu1, P.mu2);
      vpart = (2.0 * mR * (q[4] - q[3]) * ih - 2.0 * mL * (q[3] - q[2]) * ih) * ih;
      atomicAdd(&sc[bc.at(L[0], L[1], L[2])], tlob * 2.0 * (q[3] - q[2]) * ih * dmu * dclamp(aL));
      atomicAdd(&sc[bc.at(i, j, k)], thib * 2.0 * (q[4] - q[3]) * ih * dmu * dclamp(aR));
      qb[3] += tlob * 2.0 * mL * ih;
      qb[2] -= tlob * 2.0 * mL * ih;
      qb[4] += thib * 2.0 * mR * ih;
      qb[3] -= thib * 2.0 * mR * ih;
    } else {
      double tau[2];
      for (int side = 0; side < 2; ++side) {
        const double Fb = side ? Fhib : Flob, tb = side ? thib : tlob;
        const int ef = id[E] + side;
        int pL[3] = {L[0], L[1], L[2]}, pR[3] = {i, j, k};
        pL[E] = ef;
        pR[E] = ef;
        double sL, sR;
        const long iL = v_idx<E, DIM>(pL[0], pL[1], pL[2], nx, ny, nz, sL);
        const long iR = v_idx<E, DIM>(pR[0], pR[1], pR[2], nx, ny, nz, sR);
        const double veL = sL * ue[iL], veR = sR * ue[iR];
        const double Vb = 0.5 * (veL + veR);
        double g[6];
        const double W = upwind_g(q + side, Vb, eps, g);
        const double Vbb = Fb * W;
        for (int m = 0; m < 6; ++m) qb[m + side] += Fb * Vb * g[m];
        double veLb = 0.5 * Vbb, veRb = 0.5 * Vbb;
        int cc[4][3] = {{L[0], L[1], L[2]}, {i, j, k}, {L[0], L[1], L[2]}, {i, j, k}};
        cc[0][E] = ef - 1; cc[1][E] = ef - 1; cc[2][E] = ef; cc[3][E] = ef;
        double me = 0.0, da[4];
        for (int q4 = 0; q4 < 4; ++q4) {
          const double av = a[a_idx<DIM>(cc[q4][0], cc[q4][1], cc[q4][2], nx, ny, nz)];
          me += 0.25 * mix1(av, P.mu1, P.mu2);
          da[q4] = dclamp(av);
        }
        const double dud = (q[3 + side] - q[2 + side]) * ih, dve = (veR - veL) * ih;
        tau[side] = me * (dud + dve);
        const double meb = tb * (dud + dve);
        const double dudb = tb * me, dveb = tb * me;
        qb[3 + side] += dudb * ih;
        qb[2 + side] -= dudb * ih;
        veRb += dveb * ih;
        veLb -= dveb * ih;
        for (int q4 = 0; q4 < 4; ++q4)
          atomicAdd(&sc[bc.at(cc[q4][0], cc[q4][1], cc[q4][2])], 0.25 * meb * dmu * da[q4]);
        atomicAdd(&sv[bv.at(pL[0], pL[1], pL[2])], veLb);
        atomicAdd(&sv[bv.at(pR[0], pR[1], pR[2])], veRb);
      }
      vpart = (tau[1] - tau[0]) * ih;
    }
    // the forward viscous term of the face, summed over the directions in order
    const long fo = fidx<D>(i, j, k, nx, ny);
    vsum[fo] = E == 0 ? 0.0 + vpart : vsum[fo] + vpart;
    for (int m = 0; m < 7; ++m) {
      int o[3] = {i, j, k};
      o[E] += m - 3;
      atomicAdd(&su[bu.at(o[0], o[1], o[2])], qb[m]);
    }
  }
  __syncthreads();
  // flush through the ghost rules: D-faces and E-faces odd, cells even
  for (int q = tid; q < nu; q += NB) {
    const double vq = su[q];
    if (vq == 0.0) continue;
    int x, y, z;
    bu.pos(q, x, y, z);
    double sg;
    const long g = v_idx<D, DIM>(x, y, z, nx, ny, nz, sg);
    atomicAdd(&udb[g], sg * vq);
  }
  for (int q = tid; q < nvv; q += NB) {
    const double vq = sv[q];
    if (vq == 0.0) continue;
    int x, y, z;
    bv.pos(q, x, y, z);
    double sg;
    const long g = v_idx<E, DIM>(x, y, z, nx, ny, nz, sg);
    atomicAdd(&ueb[g], sg * vq);
  }
  for (int q = tid; q < ncc; q += NB) {
    const double vq = sc[q];
    if (vq == 0.0) continue;
    int x, y, z;
    bc.pos(q, x, y, z);
    atomicAdd(&abar[a_idx<DIM>(x, y, z, nx, ny, nz)], vq);
  }
}

// ===========================================================================
// S3^T, part 1 (interior cells): from skbar, Mbar -> Tbar, sbar partials, and
// nbar / dsbar on the ghost-extended grid.
template <int DIM>
__device__ __forceinline__ void normal_of(const double* __restrict__ a, int i, int j, int k, int nx, int ny, int nz,
                                          double ih2, double ne, double n[3]) {
  const double gx = (A_at<DIM>(a, i + 1, j, k, nx, ny, nz) - A_at<DIM>(a, i - 1, j, k, nx, ny, nz)) * ih2;
  const double gy = (A_at<DIM>(a, i, j + 1, k, nx, ny, nz) - A_at<DIM>(a, i, j - 1, k, nx, ny, nz)) * ih2;
  const double gz = DIM == 3 ? (A_at<DIM>(a, i, j, k + 1, nx, ny, nz) - A_at<DIM>(a, i, j, k - 1, nx, ny, nz)) * ih2 : 0.0;
  const double inv = 1.0 / sqrt(gx * gx + gy * gy + gz * gz + ne * ne);
  n[0] = gx * inv;
  n[1] = gy * inv;
  n[2] = gz * inv;
}

__device__ __forceinline__ long eidx(int i, int j, int k, int nx, int ny, int oz) {
  return (long)(i + 1) + (long)(nx + 2) * ((long)(j + 1) + (long)(ny + 2) * (k + oz));
}

template <int DIM>
__global__ __launch_bounds__(256) void ka_geom_cell(KParams P, const double* __restrict__ a,
                                                    const double* __restrict__ T, const double* __restrict__ skb,
                                                    const double* __restrict__ Mxb, const double* __restrict__ Myb,
                                                    const double* __restrict__ Mzb, double* __restrict__ Tbar,
                                                    double* __restrict__ nbx, double* __restrict__ nby,
                                                    double* __restrict__ nbz, double* __restrict__ dsb,
                                                    double* __restrict__ spart) {
  __shared__ double sh[8];
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int oz = DIM == 3 ? 1 : 0;
  double sacc = 0.0;
  if (i < nx && j < ny) {
    const double ih2 = 0.5 * P.ih, ne = P.neps, s = P.s;
    const long c = cidx(i, j, k, nx, ny);
    // forward recompute
    double nn[3], np[3];
    normal_of<DIM>(a, i + 1, j, k, nx, ny, nz, ih2, ne, np);
    normal_of<DIM>(a, i - 1, j, k, nx, ny, nz, ih2, ne, nn);
    double divn = (np[0] - nn[0]) * ih2;
    normal_of<DIM>(a, i, j + 1, k, nx, ny, nz, ih2, ne, np);
    normal_of<DIM>(a, i, j - 1, k, nx, ny, nz, ih2, ne, nn);
    divn += (np[1] - nn[1]) * ih2;
    if (DIM == 3) {
      normal_of<DIM>(a, i, j, k + 1, nx, ny, nz, ih2, ne, np);
      normal_of<DIM>(a, i, j, k - 1, nx, ny, nz, ih2, ne, nn);
      divn += (np[2] - nn[2]) * ih2;
    }
    const double kappa = -divn;
    const double gx = (A_at<DIM>(a, i + 1, j, k, nx, ny, nz) - A_at<DIM>(a, i - 1, j, k, nx, ny, nz)) * ih2;
    const double gy = (A_at<DIM>(a, i, j + 1, k, nx, ny, nz) - A_at<DIM>(a, i, j - 1, k, nx, ny, nz)) * ih2;
    const double gz = DIM == 3 ? (A_at<DIM>(a, i, j, k + 1, nx, ny, nz) - A_at<DIM>(a, i, j, k - 1, nx, ny, nz)) * ih2 : 0.0;
    const double g2 = gx * gx + gy * gy + gz * gz;
    const double ge = sqrt(g2 + ne * ne);
    const double ds = g2 / (ge + ne);
    const double n[3] = {gx / ge, gy / ge, gz / ge};
    const double sigma = P.sigma0 + s * (T[c] - P.T0);
    double dT[3];  // T(c+e) - T(c-e)
    dT[0] = T_at<DIM>(T, i + 1, j, k, P) - T_at<DIM>(T, i - 1, j, k, P);
    dT[1] = T_at<DIM>(T, i, j + 1, k, P) - T_at<DIM>(T, i, j - 1, k, P);
    dT[2] = DIM == 3 ? T_at<DIM>(T, i, j, k + 1, P) - T_at<DIM>(T, i, j, k - 1, P) : 0.0;
    const double gs[3] = {s * dT[0] * ih2, s * dT[1] * ih2, s * dT[2] * ih2};
    const double ndg = n[0] * gs[0] + n[1] * gs[1] + n[2] * gs[2];
    // reverse of sk = sigma kappa
    const double skbar = skb[c];
    const double sigb = skbar * kappa, kapb = skbar * sigma;
    aadd(&Tbar[c], s * sigb);
    sacc += sigb * (T[c] - P.T0);
    // reverse of M = ds (gs - n (n.gs))
    const double Mb[3] = {Mxb[c], Myb[c], DIM == 3 ? Mzb[c] : 0.0};
    const double nMb = n[0] * Mb[0] + n[1] * Mb[1] + n[2] * Mb[2];
    const double dsbar = Mb[0] * (gs[0] - n[0] * ndg) + Mb[1] * (gs[1] - n[1] * ndg) + Mb[2] * (gs[2] - n[2] * ndg);
    double gsb[3], nb[3];
    for (int d = 0; d < 3; ++d) {
      gsb[d] = ds * (Mb[d] - n[d] * nMb);
      nb[d] = -ds * (Mb[d] * ndg + nMb * gs[d]);
    }
    // gs_d = s (T(c+e_d) - T(c-e_d))/(2h)
    for (int d = 0; d < DIM; ++d) {
      sacc += gsb[d] * dT[d] * ih2;
      int o[3] = {0, 0, 0};
      o[d] = 1;
      double sgp, sgm;
      const long ip = t_idx<DIM>(i + o[0], j + o[1], k + o[2], P, sgp);
      const long im = t_idx<DIM>(i - o[0], j - o[1], k - o[2], P, sgm);
      aadd(&Tbar[ip], sgp * s * gsb[d] * ih2);
      aadd(&Tbar[im], -sgm * s * gsb[d] * ih2);
    }
    // kappa = -sum_d (n_d(c+e_d) - n_d(c-e_d))/(2h)
    double* nbs[3] = {nbx, nby, nbz};
    for (int d = 0; d < DIM; ++d) {
      int o[3] = {0, 0, 0};
      o[d] = 1;
      aadd(&nbs[d][eidx(i + o[0], j + o[1], k + o[2], nx, ny, oz)], -kapb * ih2);
      aadd(&nbs[d][eidx(i - o[0], j - o[1], k - o[2], nx, ny, oz)], kapb * ih2);
    }
    const long ec = eidx(i, j, k, nx, ny, oz);
    for (int d = 0; d < DIM; ++d) aadd(&nbs[d][ec], nb[d]);
    dsb[ec] += dsbar;  // written by its own cell only in this kernel
  }
  const double r = block_reduce<0>(sacc, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) spart[block_linear()] = r;
}

// S3^T, part 2 (ghost-extended cells): nbar, dsbar -> gbar -> abar.
template <int DIM>
__global__ __launch_bounds__(256) void ka_geom_ext(KParams P, const double* __restrict__ a,
                                                   const double* __restrict__ nbx, const double* __restrict__ nby,
                                                   const double* __restrict__ nbz, const double* __restrict__ dsb,
                                                   double* __restrict__ abar) {
  const int oz = DIM == 3 ? 1 : 0;
  const int i = blockIdx.x * BX + threadIdx.x - 1, j = blockIdx.y * BY + threadIdx.y - 1, k = blockIdx.z - oz;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  if (i > nx || j > ny) return;
  const long ec = eidx(i, j, k, nx, ny, oz);
  const double nb[3] = {nbx[ec], nby[ec], DIM == 3 ? nbz[ec] : 0.0};
  const double db = dsb[ec];
  if (nb[0] == 0.0 && nb[1] == 0.0 && nb[2] == 0.0 && db == 0.0) return;
  const double ih2 = 0.5 * P.ih, ne = P.neps;
  const double gx = (A_at<DIM>(a, i + 1, j, k, nx, ny, nz) - A_at<DIM>(a, i - 1, j, k, nx, ny, nz)) * ih2;
  const double gy = (A_at<DIM>(a, i, j + 1, k, nx, ny, nz) - A_at<DIM>(a, i, j - 1, k, nx, ny, nz)) * ih2;
  const double gz = DIM == 3 ? (A_at<DIM>(a, i, j, k + 1, nx, ny, nz) - A_at<DIM>(a, i, j, k - 1, nx, ny, nz)) * ih2 : 0.0;
  const double ge = sqrt(gx * gx + gy * gy + gz * gz + ne * ne);
  const double n[3] = {gx / ge, gy / ge, gz / ge};
  const double nnb = n[0] * nb[0] + n[1] * nb[1] + n[2] * nb[2];
  for (int d = 0; d < DIM; ++d) {
    // n = g/ge: gbar = (nbar - n (n.nbar))/ge ; delta_s = ge - eps_n: gbar += dsbar n
    const double gb = (nb[d] - n[d] * nnb) / ge + db * n[d];
    int o[3] = {0, 0, 0};
    o[d] = 1;
    aadd(&abar[a_idx<DIM>(i + o[0], j + o[1], k + o[2], nx, ny, nz)], gb * ih2);
    aadd(&abar[a_idx<DIM>(i - o[0], j - o[1], k - o[2], nx, ny, nz)], -gb * ih2);
  }
}

// ===========================================================================
// S1^T: one RK stage G(a, T) = (a + dt La(a), T + dt LT(a, T)) transposed,
// applied to w = (wa, wT) and accumulated into (ab, Tb) and the face-velocity
// adjoints.  Face part: advective fluxes and conduction across interior
// faces.  The scattered sums are gathered per block first: a block is
// 64 x BE faces, 64 along x and BE (4 for D = x, else 8) along the next
// axis (y for D = x and y; z for D = z, one y-row per block), and
// every contribution of its faces to a cell of alpha or T (stencil cells
// f-3..f+2 along D, ghosts included, and the two cells of the conduction
// term) is added into an LDS box over those cells (LDS FP64 atomics); then
// each box entry goes to memory with one global atomic, through the ghost
// rule of its cell (even reflection; the sign of a Dirichlet T ghost).  This
// replaces 16 global atomics per face by (BE + 5) / BE or 69 / 64 per cell.
template <int DIM, int D, int BE>
__global__ __launch_bounds__(64 * BE) void ka_transport_face_g(KParams P, const double* __restrict__ a,
                                                               const double* __restrict__ T,
                                                               const double* __restrict__ uD,
                                                               const double* __restrict__ wa,
                                                               const double* __restrict__ wT,
                                                               double* __restrict__ ab, double* __restrict__ Tb,
                                                               double* __restrict__ uDb) {
  // box: along D the cells f0-3 .. f0+NF+1 of the block's faces f0 .. f0+NF-1
  constexpr int NF = D == 0 ? 64 : BE;          // faces of the block along D
  constexpr int NV = NF + 5;                    // box cells along D
  constexpr int NW = D == 0 ? BE : 64;          // box width across D
  __shared__ double bxa[NV * NW], bxt[NV * NW];
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + 64 * ty;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  for (int q = tid; q < NV * NW; q += 64 * BE) {
    bxa[q] = 0.0;
    bxt[q] = 0.0;
  }
  int i, j, k, f0, w;  // this thread's face; first face of the block along D; its column across D
  if (D == 0) { i = blockIdx.x * 64 + tx; j = blockIdx.y * BE + ty; k = blockIdx.z; f0 = blockIdx.x * 64; w = ty; }
  else if (D == 1) { i = blockIdx.x * 64 + tx; j = blockIdx.y * BE + ty; k = blockIdx.z; f0 = blockIdx.y * BE; w = tx; }
  else { i = blockIdx.x * 64 + tx; j = blockIdx.y; k = blockIdx.z * BE + ty; f0 = blockIdx.z * BE; w = tx; }
  const int id[3] = {i, j, k};
  const int nD = D == 0 ? nx : (D == 1 ? ny : nz);
  const int fD = id[D];
  // box index of the cell at position c along D (this thread's column across D)
  auto bidx = [&](int c) { return D == 0 ? w * NV + (c - (f0 - 3)) : (c - (f0 - 3)) * NW + w; };
  const bool inr = (D == 0 ? (i <= nx && j < ny) : (D == 1 ? (i < nx && j <= ny) : (i < nx && k <= nz))) &&
                   (DIM == 3 || k == 0);
  const bool act = inr && fD > 0 && fD < nD;
  __syncthreads();
  if (act) {
    const long f = fidx<D>(i, j, k, nx, ny);
    int L[3] = {i, j, k};
    L[D] -= 1;
    const long cL = cidx(L[0], L[1], L[2], nx, ny), cR = cidx(i, j, k, nx, ny);
    const double ih = P.ih, dt = P.dt, eps = P.weno_eps;
    const double Fab = dt * (wa[cR] - wa[cL]) * ih;
    const double FTb = dt * (wT[cR] - wT[cL]) * ih;
    const double uf = uD[f];
    double qa[6], qt[6];
    for (int m = 0; m < 6; ++m) {
      int o[3] = {i, j, k};
      o[D] = fD - 3 + m;
      qa[m] = a[a_idx<DIM>(o[0], o[1], o[2], nx, ny, nz)];
      qt[m] = T_at<DIM>(T, o[0], o[1], o[2], P);
    }
    double ga[6], gt[6];
    const double Wa = upwind_g(qa, uf, eps, ga);
    const double Wt = upwind_g(qt, uf, eps, gt);
    uDb[f] += Fab * Wa + FTb * Wt;
    for (int m = 0; m < 6; ++m) {
      const int q = bidx(fD - 3 + m);
      const double va = Fab * uf * ga[m], vt = FTb * uf * gt[m];
      if (va != 0.0) atomicAdd(&bxa[q], va);
      if (vt != 0.0) atomicAdd(&bxt[q], vt);
    }
    const double aL = a[cL], aR = a[cR];
    const double rcL = mix1(aL, P.rhocp1, P.rhocp2), rcR = mix1(aR, P.rhocp1, P.rhocp2);
    const double Phib = dt * (wT[cL] / rcL - wT[cR] / rcR);
    const double lf = 0.5 * (mix1(aL, P.lam1, P.lam2) + mix1(aR, P.lam1, P.lam2));
    const double ih2 = ih * ih;
    const double dTf = (T[cR] - T[cL]) * ih2;
    const double dl = P.lam2 - P.lam1;
    atomicAdd(&bxt[bidx(fD)], Phib * lf * ih2);
    atomicAdd(&bxt[bidx(fD - 1)], -Phib * lf * ih2);
    atomicAdd(&bxa[bidx(fD - 1)], Phib * dTf * 0.5 * dl * dclamp(aL));
    atomicAdd(&bxa[bidx(fD)], Phib * dTf * 0.5 * dl * dclamp(aR));
  }
  __syncthreads();
  // flush: one global atomic per box cell, through its ghost rule
  for (int q = tid; q < NV * NW; q += 64 * BE) {
    const double va = bxa[q], vt = bxt[q];
    if (va == 0.0 && vt == 0.0) continue;
    int c[3];
    if (D == 0) { c[0] = f0 - 3 + q % NV; c[1] = blockIdx.y * BE + q / NV; c[2] = blockIdx.z; }
    else if (D == 1) { c[0] = blockIdx.x * 64 + q % NW; c[1] = f0 - 3 + q / NW; c[2] = blockIdx.z; }
    else { c[0] = blockIdx.x * 64 + q % NW; c[1] = blockIdx.y; c[2] = f0 - 3 + q / NW; }
    if (va != 0.0) atomicAdd(&ab[a_idx<DIM>(c[0], c[1], c[2], nx, ny, nz)], va);
    if (vt != 0.0) {
      double sg;
      const long it = t_idx<DIM>(c[0], c[1], c[2], P, sg);
      atomicAdd(&Tb[it], vt * sg);
    }
  }
}

// Cell part: identity, wall conduction faces, rho c_p, heat source.
template <int DIM>
__global__ __launch_bounds__(256) void ka_transport_cell(KParams P, const double* __restrict__ a,
                                                         const double* __restrict__ T, const double* __restrict__ wa,
                                                         const double* __restrict__ wT, double* __restrict__ ab,
                                                         double* __restrict__ Tb) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  if (i >= nx || j >= ny) return;
  const long c = cidx(i, j, k, nx, ny);
  const double dt = P.dt, ih = P.ih, ih2 = ih * ih;
  const double wac = wa[c], wTc = wT[c];
  const double ac = a[c], Tc = T[c];
  const double rcp = mix1(ac, P.rhocp1, P.rhocp2);
  const double lc = mix1(ac, P.lam1, P.lam2);
  const double dl = (P.lam2 - P.lam1) * dclamp(ac);
  const double wc = dt * wTc / rcp;  // adjoint weight of cond_c and src_c
  double cond = 0.0, abc = 0.0, Tbc = 0.0;
  const int di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
  for (int f = 0; f < 2 * DIM; ++f) {
    const int ii = i + di[f], jj = j + dj[f], kk = k + dk[f];
    const double an = A_at<DIM>(a, ii, jj, kk, nx, ny, nz);
    const double Tn = T_at<DIM>(T, ii, jj, kk, P);
    const double lf = 0.5 * (lc + mix1(an, P.lam1, P.lam2));
    cond += lf * (Tn - Tc);
    const bool wall = ii < 0 || ii >= nx || jj < 0 || jj >= ny || (DIM == 3 && (kk < 0 || kk >= nz));
    if (wall) {
      // ghost neighbour mirrors this cell: a_g = a_c, T_g = sg T_c (+ const)
      double sg;
      (void)t_idx<DIM>(ii, jj, kk, P, sg);
      Tbc += wc * lf * (sg - 1.0) * ih2;
      abc += wc * (Tn - Tc) * ih2 * dl;  // lambda_f = lambda(a_c): d/da_c = lambda'
    }
  }
  cond *= ih2;
  double src = 0.0;
  if (P.qP != 0.0) {
    const double h2 = 0.5 * ih;
    const double gx = (A_at<DIM>(a, i + 1, j, k, nx, ny, nz) - A_at<DIM>(a, i - 1, j, k, nx, ny, nz)) * h2;
    const double gy = (A_at<DIM>(a, i, j + 1, k, nx, ny, nz) - A_at<DIM>(a, i, j - 1, k, nx, ny, nz)) * h2;
    const double gz = DIM == 3 ? (A_at<DIM>(a, i, j, k + 1, nx, ny, nz) - A_at<DIM>(a, i, j, k - 1, nx, ny, nz)) * h2 : 0.0;
    const double g2 = gx * gx + gy * gy + gz * gz;
    if (g2 != 0.0) {  // away from the interface delta_s and its derivative vanish
      const double ne = P.neps;
      const double ge = sqrt(g2 + ne * ne);
      const double xl = P.qx0 + P.qvx * P.t, yl = P.qy0 + P.qvy * P.t;
      const double x = (i + 0.5) * P.h, y = (j + 0.5) * P.h;
      const double r2 = (x - xl) * (x - xl) + (y - yl) * (y - yl);
      const double R2 = P.qr * P.qr;
      const double Q = 2.0 * P.qP / (M_PI * R2) * exp(-2.0 * r2 / R2);
      src = Q * g2 / (ge + ne);
      // d delta_s / d g = g / ge
      const double gb[3] = {wc * Q * gx / ge, wc * Q * gy / ge, wc * Q * gz / ge};
      for (int d = 0; d < DIM; ++d) {
        int o[3] = {0, 0, 0};
        o[d] = 1;
        aadd(&ab[a_idx<DIM>(i + o[0], j + o[1], k + o[2], nx, ny, nz)], gb[d] * h2);
        aadd(&ab[a_idx<DIM>(i - o[0], j - o[1], k - o[2], nx, ny, nz)], -gb[d] * h2);
      }
    }
  }
  // rho c_p in the denominator
  abc += -wc * (cond + src) * (P.rhocp2 - P.rhocp1) * dclamp(ac) / rcp;
  // the identity part and this cell's terms in one update each: in this
  // kernel Tb[c] is written by its own thread only (a plain update), ab[c]
  // also by the heat-source terms of the neighbours (an atomic)
  aadd(&ab[c], wac + abc);
  Tb[c] += wTc + Tbc;
}

// y = s * x ; y += s * x
__global__ __launch_bounds__(256) void ka_scale(long n, double s, const double* __restrict__ x, double* __restrict__ y) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) y[c] = s * x[c];
}
__global__ __launch_bounds__(256) void ka_axpy(long n, double s, const double* __restrict__ x, double* __restrict__ y) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) y[c] += s * x[c];
}
// accumulate a device scalar (one thread)
__global__ void ka_add_scalar(double* dst, const double* src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] += src[0];
}

inline dim3 grid_of(int fnx, int fny, int fnz) { return dim3((fnx + BX - 1) / BX, (fny + BY - 1) / BY, fnz); }
inline int nb1(long n) { return (int)((n + 255) / 256); }

}  // namespace

// ---- launchers -------------------------------------------------------------
void adj_project(const KParams& P, hipStream_t s, const double* a, const double* p, const double* ub,
                 const double* vb, const double* wb, double* pbar, double* abar) {
  dim3 g = grid_of(P.nx, P.ny, P.nz), b(BX, BY);
  if (P.dim == 3) hipLaunchKernelGGL((ka_project<3>), g, b, 0, s, P, a, p, ub, vb, wb, pbar, abar);
  else hipLaunchKernelGGL((ka_project<2>), g, b, 0, s, P, a, p, ub, vb, wb, pbar, abar);
}

void adj_poisson_alpha(const KParams& P, hipStream_t s, const double* a, const double* p, const double* y,
                       double* abar) {
  dim3 g = grid_of(P.nx, P.ny, P.nz), b(BX, BY);
  if (P.dim == 3) hipLaunchKernelGGL((ka_poisson_alpha<3>), g, b, 0, s, P, a, p, y, abar);
  else hipLaunchKernelGGL((ka_poisson_alpha<2>), g, b, 0, s, P, a, p, y, abar);
}

void adj_rhs(const KParams& P, hipStream_t s, const double* ubp, const double* vbp, const double* wbp,
             const double* y, double* usb, double* vsb, double* wsb) {
  dim3 b(BX, BY);
  if (P.dim == 3) {
    hipLaunchKernelGGL((ka_rhs_face<3, 0>), grid_of(P.nx + 1, P.ny, P.nz), b, 0, s, P, ubp, y, usb);
    hipLaunchKernelGGL((ka_rhs_face<3, 1>), grid_of(P.nx, P.ny + 1, P.nz), b, 0, s, P, vbp, y, vsb);
    hipLaunchKernelGGL((ka_rhs_face<3, 2>), grid_of(P.nx, P.ny, P.nz + 1), b, 0, s, P, wbp, y, wsb);
  } else {
    hipLaunchKernelGGL((ka_rhs_face<2, 0>), grid_of(P.nx + 1, P.ny, 1), b, 0, s, P, ubp, y, usb);
    hipLaunchKernelGGL((ka_rhs_face<2, 1>), grid_of(P.nx, P.ny + 1, 1), b, 0, s, P, vbp, y, vsb);
  }
}

// the direction kernels of component D (its x, y and z fluxes)
template <int DIM, int D, int E>
void pred_dir(const KParams& P, hipStream_t s, const double* a, const double* const vel[3], double* const velb[3],
              const double* usb, double* abar, double* vsum) {
  const int fnx = P.nx + (D == 0), fny = P.ny + (D == 1), fnz = (DIM == 3 ? P.nz : 1) + (D == 2);
  const dim3 g = E == 2 ? dim3((fnx + 63) / 64, fny, (fnz + 3) / 4) : dim3((fnx + 63) / 64, (fny + 3) / 4, fnz);
  hipLaunchKernelGGL((ka_pred_dir<DIM, D, E>), g, dim3(64, 4), 0, s, P, a, vel[D], vel[E], usb, velb[D], velb[E],
                     abar, vsum);
}
// component D: its x, y (and z) flux kernels, then the face kernel that
// reads the viscous term they summed
template <int DIM, int D>
void pred_component(const KParams& P, hipStream_t s, const double* a, const double* sk, const double* M,
                    const double* const vel[3], double* const velb[3], const double* usb, double* abar,
                    double* skbar, double* Mbar, double* vsum) {
  pred_dir<DIM, D, 0>(P, s, a, vel, velb, usb, abar, vsum);
  pred_dir<DIM, D, 1>(P, s, a, vel, velb, usb, abar, vsum);
  if constexpr (DIM == 3) pred_dir<DIM, D, 2>(P, s, a, vel, velb, usb, abar, vsum);
  const dim3 g = grid_of(P.nx, P.ny, DIM == 3 ? P.nz : 1);  // one thread per cell
  hipLaunchKernelGGL((ka_pred_face<DIM, D>), g, dim3(BX, BY), 0, s, P, a, sk, M, vsum, usb, velb[D], abar, skbar,
                     Mbar);
}

void adj_predictor(const KParams& P, hipStream_t s, const double* a, const double* sk, const double* Mx,
                   const double* My, const double* Mz, const double* u, const double* v, const double* w,
                   const double* usb, const double* vsb, const double* wsb, double* ubar, double* vbar,
                   double* wbar, double* abar, double* skbar, double* Mxb, double* Myb, double* Mzb, double* vsum) {
  const double* const vel[3] = {u, v, w};
  double* const velb[3] = {ubar, vbar, wbar};
  if (P.dim == 3) {
    pred_component<3, 0>(P, s, a, sk, Mx, vel, velb, usb, abar, skbar, Mxb, vsum);
    pred_component<3, 1>(P, s, a, sk, My, vel, velb, vsb, abar, skbar, Myb, vsum);
    pred_component<3, 2>(P, s, a, sk, Mz, vel, velb, wsb, abar, skbar, Mzb, vsum);
  } else {
    pred_component<2, 0>(P, s, a, sk, Mx, vel, velb, usb, abar, skbar, Mxb, vsum);
    pred_component<2, 1>(P, s, a, sk, My, vel, velb, vsb, abar, skbar, Myb, vsum);
  }
}

int adj_geometry(const KParams& P, hipStream_t s, const double* a, const double* T, const double* skb,
                 const double* Mxb, const double* Myb, const double* Mzb, double* Tbar, double* nbx, double* nby,
                 double* nbz, double* dsb, double* abar, double* spart) {
  dim3 b(BX, BY);
  dim3 g = grid_of(P.nx, P.ny, P.nz);
  const int oz = P.dim == 3 ? 1 : 0;
  dim3 ge = grid_of(P.nx + 2, P.ny + 2, P.nz + 2 * oz);
  if (P.dim == 3) {
    hipLaunchKernelGGL((ka_geom_cell<3>), g, b, 0, s, P, a, T, skb, Mxb, Myb, Mzb, Tbar, nbx, nby, nbz, dsb, spart);
    hipLaunchKernelGGL((ka_geom_ext<3>), ge, b, 0, s, P, a, nbx, nby, nbz, dsb, abar);
  } else {
    hipLaunchKernelGGL((ka_geom_cell<2>), g, b, 0, s, P, a, T, skb, Mxb, Myb, Mzb, Tbar, nbx, nby, nbz, dsb, spart);
    hipLaunchKernelGGL((ka_geom_ext<2>), ge, b, 0, s, P, a, nbx, nby, nbz, dsb, abar);
  }
  return (int)(g.x * g.y * g.z);
}

void adj_transport_stage(const KParams& P, hipStream_t s, const double* a, const double* T, const double* u,
                         const double* v, const double* w, const double* wa, const double* wT, double* ab,
                         double* Tb, double* ub, double* vb, double* wb) {
  dim3 b(BX, BY);
  const int gx0 = (P.nx + 1 + 63) / 64, gx = (P.nx + 63) / 64;
  if (P.dim == 3) {
    hipLaunchKernelGGL((ka_transport_face_g<3, 0, 4>), dim3(gx0, (P.ny + 3) / 4, P.nz), dim3(64, 4), 0, s, P, a, T, u,
                       wa, wT, ab, Tb, ub);
    hipLaunchKernelGGL((ka_transport_face_g<3, 1, 8>), dim3(gx, (P.ny + 1 + 7) / 8, P.nz), dim3(64, 8), 0, s, P, a, T,
                       v, wa, wT, ab, Tb, vb);
    hipLaunchKernelGGL((ka_transport_face_g<3, 2, 8>), dim3(gx, P.ny, (P.nz + 1 + 7) / 8), dim3(64, 8), 0, s, P, a, T,
                       w, wa, wT, ab, Tb, wb);
    hipLaunchKernelGGL((ka_transport_cell<3>), grid_of(P.nx, P.ny, P.nz), b, 0, s, P, a, T, wa, wT, ab, Tb);
  } else {
    hipLaunchKernelGGL((ka_transport_face_g<2, 0, 4>), dim3(gx0, (P.ny + 3) / 4, 1), dim3(64, 4), 0, s, P, a, T, u, wa,
                       wT, ab, Tb, ub);
    hipLaunchKernelGGL((ka_transport_face_g<2, 1, 8>), dim3(gx, (P.ny + 1 + 7) / 8, 1), dim3(64, 8), 0, s, P, a, T, v,
                       wa, wT, ab, Tb, vb);
    hipLaunchKernelGGL((ka_transport_cell<2>), grid_of(P.nx, P.ny, 1), b, 0, s, P, a, T, wa, wT, ab, Tb);
  }
}

void adj_scale(hipStream_t s, long n, double f, const double* x, double* y) {
  hipLaunchKernelGGL(ka_scale, dim3(nb1(n)), dim3(256), 0, s, n, f, x, y);
}
void adj_axpy(hipStream_t s, long n, double f, const double* x, double* y) {
  hipLaunchKernelGGL(ka_axpy, dim3(nb1(n)), dim3(256), 0, s, n, f, x, y);
}
void adj_add_scalar(hipStream_t s, double* dst, const double* src) {
  hipLaunchKernelGGL(ka_add_scalar, dim3(1), dim3(64), 0, s, dst, src);
}

}  // namespace tcf
