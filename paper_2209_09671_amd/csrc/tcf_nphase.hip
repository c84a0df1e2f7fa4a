// N-phase VOF kernels (eq. 1 for every phase of several in one domain).
//
// Phase 1 is the background with alpha_1 = 1 - (alpha_2 + alpha_3 [+
// alpha_4]); phases 2..N are carried by the scalar WENO5 / SSP-RK3 transport
// of the two-phase path.  These kernels produce what the two-phase kernels
// take from alpha alone: the mixture (material laws linear in each clamped
// fraction relative to phase 1) and the per-pair interface geometry and CSF
// force.  The temperature stage and the momentum predictor are the
// two-phase kernels in their material forms, fed the mixture's
// conductivity, heat capacity and heat-source delta, and its viscosity,
// density and this face force.  Each surface-tension pair i < j acts
// through its pair gradient g_ij = alpha_i grad alpha_j - alpha_j grad
// alpha_i (grad alpha for two phases) with the curvature and Marangoni
// terms of eqs. 4-7.  One thread per cell or face on 64 x 4
// blocks; ghost values by reflected indexing as in the two-phase kernels.
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "tcf_device.h"
#include "tcf_internal.h"

namespace tcf {
namespace {

using namespace dev;

inline dim3 grid_np(int fnx, int fny, int fnz) { return dim3((fnx + BX - 1) / BX, (fny + BY - 1) / BY, fnz); }
inline dim3 blk_np() { return dim3(BX, BY, 1); }

// Pairs (i, j) of an N-phase grid in the order of the pair tables; slot =
// position in the six-pair table (1,2), (1,3), (1,4), (2,3), (2,4), (3,4).
template <int NPH>
struct PairList;
template <>
struct PairList<3> {
  static constexpr int n = 3;
  __device__ static int I(int p) { return p == 2 ? 2 : 1; }
  __device__ static int J(int p) { return p == 0 ? 2 : 3; }
  __device__ static int slot(int p) { return p == 2 ? 3 : p; }
};
template <>
struct PairList<4> {
  static constexpr int n = 6;
  __device__ static int I(int p) { return p < 3 ? 1 : (p < 5 ? 2 : 3); }
  __device__ static int J(int p) { return p < 3 ? p + 2 : (p < 5 ? p - 0 : 4); }
  __device__ static int slot(int p) { return p; }
};

template <class R>
struct Phases {
  const R* a2;
  const R* a3;
  const R* a4;
};

// fraction of phase q (1..4) at a cell, ghosts by even reflection
template <int DIM, int NPH, class R>
__device__ __forceinline__ R ph_at(const Phases<R>& F, int q, int i, int j, int k, int nx, int ny, int nz) {
  if (q == 2) return A_at<DIM>(F.a2, i, j, k, nx, ny, nz);
  if (q == 3) return A_at<DIM>(F.a3, i, j, k, nx, ny, nz);
  if (NPH == 4 && q == 4) return A_at<DIM>(F.a4, i, j, k, nx, ny, nz);
  R s = A_at<DIM>(F.a2, i, j, k, nx, ny, nz) + A_at<DIM>(F.a3, i, j, k, nx, ny, nz);
  if (NPH == 4) s += A_at<DIM>(F.a4, i, j, k, nx, ny, nz);
  return R(1) - s;
}

// ---------------------------------------------------------------------------
// Mixture per cell of rho, mu, rho c_p, lambda = P_1 + sum_j clamp(alpha_j)
// (P_j - P_1) (FP64, then stored in R).  THERMAL: o0 = rho c_p, o1 =
// lambda, and with a heat source o2 = the delta |grad a_c|^2 / (|grad
// a_c|_eps + eps) of the condensed fraction a_c = 1 - alpha_1 (central
// differences, even ghosts).  Otherwise o0, o1 = the density and the
// viscosity as fractions (P - lo) / (hi - lo) of ranges that hold every
// mixture, which the linear mixes of the pressure kernels and the predictor
// turn back into rho and mu.
template <class R, int DIM, int NPH, bool THERMAL>
__global__ __launch_bounds__(256) void k_np_mixture(KParams P, Phases<R> F, R* __restrict__ o0, R* __restrict__ o1,
                                                    R* __restrict__ o2, double lo0, double hi0, double lo1,
                                                    double hi1) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  if (i >= nx || j >= ny) return;
  const long c = cidx(i, j, k, nx, ny);
  auto cl = [](double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); };
  const double a2 = (double)F.a2[c], a3 = (double)F.a3[c], a4 = NPH == 4 ? (double)F.a4[c] : 0.0;
  const double p1[4] = {P.rho1, P.mu1, P.rhocp1, P.lam1}, p2[4] = {P.rho2, P.mu2, P.rhocp2, P.lam2};
  double m[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int q = THERMAL ? 2 + r : r;
    double v = p1[q] + cl(a2) * (p2[q] - p1[q]);
    v += cl(a3) * (P.mat34[q][0] - p1[q]);
    if (NPH == 4) v += cl(a4) * (P.mat34[q][1] - p1[q]);
    m[r] = v;
  }
  if (THERMAL) {
    o0[c] = R(m[0]);
    o1[c] = R(m[1]);
    if (P.qP != 0.0) {
      auto acond = [&](int ii, int jj, int kk) {
        double sm = (double)A_at<DIM>(F.a2, ii, jj, kk, nx, ny, nz) + (double)A_at<DIM>(F.a3, ii, jj, kk, nx, ny, nz);
        if (NPH == 4) sm += (double)A_at<DIM>(F.a4, ii, jj, kk, nx, ny, nz);
        return R(1.0 - (1.0 - sm));
      };
      const R ih2 = R(0.5 * P.ih), ne = R(P.neps);
      const R g0 = (acond(i + 1, j, k) - acond(i - 1, j, k)) * ih2;
      const R g1 = (acond(i, j + 1, k) - acond(i, j - 1, k)) * ih2;
      const R g2 = DIM == 3 ? (acond(i, j, k + 1) - acond(i, j, k - 1)) * ih2 : R(0);
      const R gg = g0 * g0 + g1 * g1 + g2 * g2;
      o2[c] = gg / (sqrt(gg + ne * ne) + ne);
    }
  } else {
    o0[c] = R((m[0] - lo0) / (hi0 - lo0));
    o1[c] = R((m[1] - lo1) / (hi1 - lo1));
  }
}

// ---------------------------------------------------------------------------
// Geometry per interior cell in two passes: for each pair, the pair
// gradient g = alpha_i grad alpha_j - alpha_j grad alpha_i (central
// differences of the phases, even ghosts) and from it the normal and delta;
// then sigma_ij kappa_ij (pair-major) and the Marangoni vector summed over
// the pairs.
template <class R, int DIM, int NPH>
__device__ __forceinline__ void pair_grad(const Phases<R>& F, int I, int J, int i, int j, int k, int nx, int ny,
                                          int nz, R ih2, R g[3]) {
  const R ai = ph_at<DIM, NPH>(F, I, i, j, k, nx, ny, nz), aj = ph_at<DIM, NPH>(F, J, i, j, k, nx, ny, nz);
  auto d = [&](int q, int di, int dj, int dk) {
    return (ph_at<DIM, NPH>(F, q, i + di, j + dj, k + dk, nx, ny, nz) -
            ph_at<DIM, NPH>(F, q, i - di, j - dj, k - dk, nx, ny, nz)) * ih2;
  };
  g[0] = ai * d(J, 1, 0, 0) - aj * d(I, 1, 0, 0);
  g[1] = ai * d(J, 0, 1, 0) - aj * d(I, 0, 1, 0);
  g[2] = DIM == 3 ? ai * d(J, 0, 0, 1) - aj * d(I, 0, 0, 1) : R(0);
}

// Pass A: per interior cell and pair, the unit normal n = g / |g|_eps
// (pair-major, three components) and delta = |g|^2 / (|g|_eps + eps).
template <class R, int DIM, int NPH>
__global__ __launch_bounds__(256) void k_np_normals(KParams P, Phases<R> F, R* __restrict__ nrm,
                                                    R* __restrict__ dsp) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  if (i >= nx || j >= ny) return;
  const R ih2 = R(0.5 * P.ih), ne = R(P.neps);
  const long c = cidx(i, j, k, nx, ny);
  const long N = (long)nx * ny * nz;
  for (int p = 0; p < PairList<NPH>::n; ++p) {
    R g[3];
    pair_grad<R, DIM, NPH>(F, PairList<NPH>::I(p), PairList<NPH>::J(p), i, j, k, nx, ny, nz, ih2, g);
    const R g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    const R ge = sqrt(g2 + ne * ne);
    nrm[(3 * p + 0) * N + c] = g[0] / ge;
    nrm[(3 * p + 1) * N + c] = g[1] / ge;
    nrm[(3 * p + 2) * N + c] = g[2] / ge;
    dsp[p * N + c] = g2 / (ge + ne);
  }
}

// Pass B: per interior cell and pair, kappa = -div n by central differences
// of the stored normals.  Across a wall the neighbour's normal is the
// cell's own with the wall-normal component negated: the even reflection of
// the phases makes the pair gradient of a ghost cell exactly that.  Then
// sigma_ij kappa_ij into skp and the Marangoni vector summed over the pairs.
template <class R, int DIM, int NPH>
__global__ __launch_bounds__(256) void k_np_geometry(KParams P, const R* __restrict__ nrm, const R* __restrict__ dsp,
                                                     const R* __restrict__ T, R* __restrict__ skp,
                                                     R* __restrict__ Mx, R* __restrict__ My, R* __restrict__ Mz) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  if (i >= nx || j >= ny) return;
  const R ih2 = R(0.5 * P.ih);
  const long c = cidx(i, j, k, nx, ny);
  const long N = (long)nx * ny * nz, pl = (long)nx * ny;
  const R Tc = T[c];
  const R dT0 = (T_at<DIM>(T, i + 1, j, k, P) - T_at<DIM>(T, i - 1, j, k, P)) * ih2;
  const R dT1 = (T_at<DIM>(T, i, j + 1, k, P) - T_at<DIM>(T, i, j - 1, k, P)) * ih2;
  const R dT2 = DIM == 3 ? (T_at<DIM>(T, i, j, k + 1, P) - T_at<DIM>(T, i, j, k - 1, P)) * ih2 : R(0);
  R M0 = R(0), M1 = R(0), M2 = R(0);
  for (int p = 0; p < PairList<NPH>::n; ++p) {
    const int sl = PairList<NPH>::slot(p);
    const R* nxp = nrm + (3 * p + 0) * N;
    const R* nyp = nrm + (3 * p + 1) * N;
    const R* nzp = nrm + (3 * p + 2) * N;
    const R n0 = nxp[c], n1 = nyp[c], n2 = DIM == 3 ? nzp[c] : R(0);
    R divn = ((i + 1 < nx ? nxp[c + 1] : -n0) - (i > 0 ? nxp[c - 1] : -n0)) * ih2;
    divn += ((j + 1 < ny ? nyp[c + nx] : -n1) - (j > 0 ? nyp[c - nx] : -n1)) * ih2;
    if (DIM == 3) divn += ((k + 1 < nz ? nzp[c + pl] : -n2) - (k > 0 ? nzp[c - pl] : -n2)) * ih2;
    const R ds = dsp[p * N + c];
    const R sT = R(P.dsigp[sl]);
    const R sigma = R(P.sig0p[sl]) + sT * (Tc - R(P.T0));
    const R gs0 = sT * dT0, gs1 = sT * dT1, gs2 = sT * dT2;
    const R ndg = n0 * gs0 + n1 * gs1 + n2 * gs2;
    M0 += ds * (gs0 - n0 * ndg);
    M1 += ds * (gs1 - n1 * ndg);
    M2 += ds * (gs2 - n2 * ndg);
    skp[p * N + c] = sigma * -divn;
  }
  Mx[c] = M0;
  My[c] = M1;
  if (DIM == 3) Mz[c] = M2;
}

// 3-D pair geometry marching along z (one kernel): a 64 x 4 tile per block
// over a chunk of planes.  The fractions of phases 2..N of planes k-1 ..
// k+2 with a two-cell ring (ghosts by even reflection on load) sit in a
// five-slot LDS ring per phase; for each pair the in-plane normals of plane
// k (tile and one-cell ring) are computed once into LDS and the own
// column's z normal of plane k+1 is carried.  The pair gradients, normals,
// deltas and the rest are the expressions of the two-pass kernels above,
// whose stored normals at ghost cells are the same values.
constexpr int NGX = BX + 4, NGY = BY + 4, NGR = 5;
constexpr int NGN = (NGX * NGY + BX * BY - 1) / (BX * BY);

template <class R, int NPH>
__global__ __launch_bounds__(256) void k_np_geometry_z(KParams P, int kz, int ntx, int nty, Phases<R> F,
                                                       const R* __restrict__ T, R* __restrict__ skp,
                                                       R* __restrict__ Mx, R* __restrict__ My, R* __restrict__ Mz) {
  constexpr int NF = NPH - 1, NP = PairList<NPH>::n;
  __shared__ R sa[NF][NGR][NGY][NGX];
  __shared__ R snx[NP][BY + 2][BX + 2], sny[NP][BY + 2][BX + 2];
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int t = xcd_tile();
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + BX * ty;
  const int i0 = (t % ntx) * BX, j0 = ((t / ntx) % nty) * BY, tz = t / (ntx * nty);
  const int k0 = tz * kz, k1 = min(k0 + kz, nz);
  const int i = i0 + tx, j = j0 + ty;
  const bool act = i < nx && j < ny;
  const R ih2 = R(0.5 * P.ih), ne = R(P.neps);
  const size_t pl = (size_t)nx * ny;
  const long N = (long)nx * ny * nz;
  const R* src[3] = {F.a2, F.a3, F.a4};
  unsigned off[NGN];
  for (int q = 0; q < NGN; ++q) {
    const int e = tid + q * BX * BY;
    const int ex = e % NGX, ey = e / NGX;
    const int ri = min(max(refl(i0 - 2 + ex, nx), 0), nx - 1), rj = min(max(refl(j0 - 2 + ey, ny), 0), ny - 1);
    off[q] = e < NGX * NGY ? (unsigned)(ri + nx * rj) : 0u;
  }
  auto plane = [&](int kk) { return (size_t)min(max(refl(kk, nz), 0), nz - 1) * pl; };
  auto slot = [](int kk) { return ((kk % NGR) + NGR) % NGR; };
  R v[NF][NGN];
  auto load = [&](int kk) {
    const size_t po = plane(kk);
    for (int f = 0; f < NF; ++f)
      for (int q = 0; q < NGN; ++q) v[f][q] = src[f][po + off[q]];
  };
  auto store = [&](int kk) {
    const int sl = slot(kk);
    for (int q = 0; q < NGN; ++q) {
      const int e = tid + q * BX * BY;
      if (e < NGX * NGY)
        for (int f = 0; f < NF; ++f) sa[f][sl][e / NGX][e % NGX] = v[f][q];
    }
  };
  // fraction of phase q (1..NPH) at tile position (x, y) of a slot
  auto ph = [&](int q, int sl, int y, int x) {
    if (q >= 2) return sa[q - 2][sl][y][x];
    R sm = sa[0][sl][y][x] + sa[1][sl][y][x];
    if (NPH == 4) sm += sa[NF - 1][sl][y][x];
    return R(1) - sm;
  };
  // pair gradient of pair p at tile position (x, y) of plane slot sc (z
  // neighbours in slots sm, sp)
  auto grad = [&](int p, int sm, int sc, int sp, int y, int x, R g[3]) {
    const int I = PairList<NPH>::I(p), J = PairList<NPH>::J(p);
    const R ai = ph(I, sc, y, x), aj = ph(J, sc, y, x);
    auto dx = [&](int q) { return (ph(q, sc, y, x + 1) - ph(q, sc, y, x - 1)) * ih2; };
    auto dy = [&](int q) { return (ph(q, sc, y + 1, x) - ph(q, sc, y - 1, x)) * ih2; };
    auto dz = [&](int q) { return (ph(q, sp, y, x) - ph(q, sm, y, x)) * ih2; };
    g[0] = ai * dx(J) - aj * dx(I);
    g[1] = ai * dy(J) - aj * dy(I);
    g[2] = ai * dz(J) - aj * dz(I);
  };
  for (int kk = k0 - 1; kk <= k0 + 2; ++kk) {
    load(kk);
    store(kk);
  }
  load(k0 + 3);
  const int ic = min(i, nx - 1), jc = min(j, ny - 1);
  R nzm[NP], nzc[NP];
  for (int p = 0; p < NP; ++p) {
    R g[3];
    pair_grad<R, 3, NPH>(F, PairList<NPH>::I(p), PairList<NPH>::J(p), ic, jc, k0 - 1, nx, ny, nz, ih2, g);
    R g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    nzm[p] = g[2] / sqrt(g2 + ne * ne);
    pair_grad<R, 3, NPH>(F, PairList<NPH>::I(p), PairList<NPH>::J(p), ic, jc, k0, nx, ny, nz, ih2, g);
    g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    nzc[p] = g[2] / sqrt(g2 + ne * ne);
  }
  const int X = tx + 2, Y = ty + 2;
  for (int k = k0; k < k1; ++k) {
    __syncthreads();
    const int sm = slot(k - 1), sc = slot(k), sp = slot(k + 1), sq = slot(k + 2);
    for (int e = tid; e < (BX + 2) * (BY + 2); e += BX * BY) {
      const int px = e % (BX + 2) + 1, py = e / (BX + 2) + 1;
      for (int p = 0; p < NP; ++p) {
        R g[3];
        grad(p, sm, sc, sp, py, px, g);
        const R g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        const R ge = sqrt(g2 + ne * ne);
        snx[p][py - 1][px - 1] = g[0] / ge;
        sny[p][py - 1][px - 1] = g[1] / ge;
      }
    }
    R nzp[NP];
    for (int p = 0; p < NP; ++p) {
      R g[3];
      grad(p, sc, sp, sq, Y, X, g);
      const R g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
      nzp[p] = g[2] / sqrt(g2 + ne * ne);
    }
    store(k + 3);
    load(min(k + 4, nz + 2));
    __syncthreads();
    if (act) {
      const long c = cidx(i, j, k, nx, ny);
      const R Tc = T[c];
      const R dT0 = (T_at<3>(T, i + 1, j, k, P) - T_at<3>(T, i - 1, j, k, P)) * ih2;
      const R dT1 = (T_at<3>(T, i, j + 1, k, P) - T_at<3>(T, i, j - 1, k, P)) * ih2;
      const R dT2 = (T_at<3>(T, i, j, k + 1, P) - T_at<3>(T, i, j, k - 1, P)) * ih2;
      R M0 = R(0), M1 = R(0), M2 = R(0);
      for (int p = 0; p < NP; ++p) {
        const int sl = PairList<NPH>::slot(p);
        R g[3];
        grad(p, sm, sc, sp, Y, X, g);
        const R g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        const R ge = sqrt(g2 + ne * ne);
        const R n0 = g[0] / ge, n1 = g[1] / ge, n2 = g[2] / ge;
        const R ds = g2 / (ge + ne);
        R divn = (snx[p][ty + 1][tx + 2] - snx[p][ty + 1][tx]) * ih2;
        divn += (sny[p][ty + 2][tx + 1] - sny[p][ty][tx + 1]) * ih2;
        divn += (nzp[p] - nzm[p]) * ih2;
        const R sT = R(P.dsigp[sl]);
        const R sigma = R(P.sig0p[sl]) + sT * (Tc - R(P.T0));
        const R gs0 = sT * dT0, gs1 = sT * dT1, gs2 = sT * dT2;
        const R ndg = n0 * gs0 + n1 * gs1 + n2 * gs2;
        M0 += ds * (gs0 - n0 * ndg);
        M1 += ds * (gs1 - n1 * ndg);
        M2 += ds * (gs2 - n2 * ndg);
        skp[p * N + c] = sigma * -divn;
      }
      Mx[c] = M0;
      My[c] = M1;
      Mz[c] = M2;
    }
    for (int p = 0; p < NP; ++p) {
      nzm[p] = nzc[p];
      nzc[p] = nzp[p];
    }
  }
}

// ---------------------------------------------------------------------------
// Face CSF force of direction D: 1/2 (M_L + M_R)_D plus, per pair,
// 1/2 (skp_L + skp_R) times the face pair gradient avg(alpha_i)(alpha_j,R -
// alpha_j,L)/h - avg(alpha_j)(alpha_i,R - alpha_i,L)/h; wall faces 0.
template <class R, int DIM, int D, int NPH>
__global__ __launch_bounds__(256) void k_np_face_force(KParams P, Phases<R> F, const R* __restrict__ skp,
                                                       const R* __restrict__ Md, R* __restrict__ f) {
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int fnx = nx + (D == 0), fny = ny + (D == 1);
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i >= fnx || j >= fny) return;
  const long fi = (long)i + (long)fnx * ((long)j + (long)fny * k);
  const int m = D == 0 ? i : (D == 1 ? j : k), nd = D == 0 ? nx : (D == 1 ? ny : nz);
  if (m == 0 || m == nd) {
    f[fi] = R(0);
    return;
  }
  const int iL = i - (D == 0), jL = j - (D == 1), kL = k - (D == 2);
  const long cL = cidx(iL, jL, kL, nx, ny), cR = cidx(i, j, k, nx, ny);
  const long N = (long)nx * ny * nz;
  const R ih = R(P.ih);
  R fo = R(0.5) * (Md[cL] + Md[cR]);
  for (int p = 0; p < PairList<NPH>::n; ++p) {
    const int I = PairList<NPH>::I(p), J = PairList<NPH>::J(p);
    const R aiL = ph_at<DIM, NPH>(F, I, iL, jL, kL, nx, ny, nz), aiR = ph_at<DIM, NPH>(F, I, i, j, k, nx, ny, nz);
    const R ajL = ph_at<DIM, NPH>(F, J, iL, jL, kL, nx, ny, nz), ajR = ph_at<DIM, NPH>(F, J, i, j, k, nx, ny, nz);
    const R G = (R(0.5) * (aiL + aiR) * (ajR - ajL) - R(0.5) * (ajL + ajR) * (aiR - aiL)) * ih;
    fo += R(0.5) * (skp[p * N + cL] + skp[p * N + cR]) * G;
  }
  f[fi] = fo;
}

}  // namespace

// ---- launchers ---------------------------------------------------------------
template <class R, bool THERMAL>
static void mixture(const KParams& P, hipStream_t s, const Phases<R>& F, R* o0, R* o1, R* o2, double lo0,
                    double hi0, double lo1, double hi1) {
  const dim3 g = grid_np(P.nx, P.ny, P.dim == 3 ? P.nz : 1);
  if (P.dim == 3) {
    if (P.nph == 4)
      hipLaunchKernelGGL((k_np_mixture<R, 3, 4, THERMAL>), g, blk_np(), 0, s, P, F, o0, o1, o2, lo0, hi0, lo1, hi1);
    else
      hipLaunchKernelGGL((k_np_mixture<R, 3, 3, THERMAL>), g, blk_np(), 0, s, P, F, o0, o1, o2, lo0, hi0, lo1, hi1);
  } else {
    if (P.nph == 4)
      hipLaunchKernelGGL((k_np_mixture<R, 2, 4, THERMAL>), g, blk_np(), 0, s, P, F, o0, o1, o2, lo0, hi0, lo1, hi1);
    else
      hipLaunchKernelGGL((k_np_mixture<R, 2, 3, THERMAL>), g, blk_np(), 0, s, P, F, o0, o1, o2, lo0, hi0, lo1, hi1);
  }
}

template <class R>
void np_mixture_thermal(const KParams& P, hipStream_t s, const R* a2, const R* a3, const R* a4, R* rcp, R* lam,
                        R* dq) {
  mixture<R, true>(P, s, Phases<R>{a2, a3, a4}, rcp, lam, dq, 0.0, 1.0, 0.0, 1.0);
}

template <class R>
void np_mixture(const KParams& P, hipStream_t s, const R* a2, const R* a3, const R* a4, R* arho, R* amu, double rlo,
                double rhi, double mlo, double mhi) {
  mixture<R, false>(P, s, Phases<R>{a2, a3, a4}, arho, amu, nullptr, rlo, rhi, mlo, mhi);
}

template <class R, int DIM, int NPH>
static void geometry_dim(const KParams& P, hipStream_t s, const Phases<R>& F, const R* T, R* nrm, R* dsp, R* skp,
                         R* Mx, R* My, R* Mz) {
  if (DIM == 3) {
    // chunks of planes so that the grid has >= 2048 blocks of 256
    const int ntx = (P.nx + BX - 1) / BX, nty = (P.ny + BY - 1) / BY;
    int nch = std::max(1, std::min(P.nz, (2048 + ntx * nty - 1) / (ntx * nty)));
    const int kz = (P.nz + nch - 1) / nch;
    nch = (P.nz + kz - 1) / kz;
    hipLaunchKernelGGL((k_np_geometry_z<R, NPH>), dim3(ntx * nty * nch), blk_np(), 0, s, P, kz, ntx, nty, F, T, skp,
                       Mx, My, Mz);
    return;
  }
  const dim3 g = grid_np(P.nx, P.ny, 1);
  hipLaunchKernelGGL((k_np_normals<R, DIM, NPH>), g, blk_np(), 0, s, P, F, nrm, dsp);
  hipLaunchKernelGGL((k_np_geometry<R, DIM, NPH>), g, blk_np(), 0, s, P, nrm, dsp, T, skp, Mx, My, Mz);
}

template <class R>
void np_geometry(const KParams& P, hipStream_t s, const R* a2, const R* a3, const R* a4, const R* T, R* nrm, R* dsp,
                 R* skp, R* Mx, R* My, R* Mz) {
  const Phases<R> F{a2, a3, a4};
  if (P.dim == 3) {
    if (P.nph == 4) geometry_dim<R, 3, 4>(P, s, F, T, nrm, dsp, skp, Mx, My, Mz);
    else geometry_dim<R, 3, 3>(P, s, F, T, nrm, dsp, skp, Mx, My, Mz);
  } else {
    if (P.nph == 4) geometry_dim<R, 2, 4>(P, s, F, T, nrm, dsp, skp, Mx, My, Mz);
    else geometry_dim<R, 2, 3>(P, s, F, T, nrm, dsp, skp, Mx, My, Mz);
  }
}

template <class R, int DIM, int NPH>
static void face_force_dim(const KParams& P, hipStream_t s, const Phases<R>& F, const R* skp, const R* Mx, const R* My,
                           const R* Mz, R* fx, R* fy, R* fz) {
  hipLaunchKernelGGL((k_np_face_force<R, DIM, 0, NPH>), grid_np(P.nx + 1, P.ny, P.nz), blk_np(), 0, s, P, F, skp, Mx, fx);
  hipLaunchKernelGGL((k_np_face_force<R, DIM, 1, NPH>), grid_np(P.nx, P.ny + 1, P.nz), blk_np(), 0, s, P, F, skp, My, fy);
  if (DIM == 3)
    hipLaunchKernelGGL((k_np_face_force<R, DIM, 2, NPH>), grid_np(P.nx, P.ny, P.nz + 1), blk_np(), 0, s, P, F, skp, Mz, fz);
}

template <class R>
void np_face_force(const KParams& P, hipStream_t s, const R* a2, const R* a3, const R* a4, const R* skp, const R* Mx,
                   const R* My, const R* Mz, R* fx, R* fy, R* fz) {
  const Phases<R> F{a2, a3, a4};
  if (P.dim == 3) {
    if (P.nph == 4) face_force_dim<R, 3, 4>(P, s, F, skp, Mx, My, Mz, fx, fy, fz);
    else face_force_dim<R, 3, 3>(P, s, F, skp, Mx, My, Mz, fx, fy, fz);
  } else {
    if (P.nph == 4) face_force_dim<R, 2, 4>(P, s, F, skp, Mx, My, Mz, fx, fy, fz);
    else face_force_dim<R, 2, 3>(P, s, F, skp, Mx, My, Mz, fx, fy, fz);
  }
}

#define TCF_NP_INST(R)                                                                                              \
  template void np_mixture<R>(const KParams&, hipStream_t, const R*, const R*, const R*, R*, R*, double, double,   \
                              double, double);                                                                     \
  template void np_mixture_thermal<R>(const KParams&, hipStream_t, const R*, const R*, const R*, R*, R*, R*);      \
  template void np_geometry<R>(const KParams&, hipStream_t, const R*, const R*, const R*, const R*, R*, R*, R*,   \
                               R*, R*, R*);                                                                        \
  template void np_face_force<R>(const KParams&, hipStream_t, const R*, const R*, const R*, const R*, const R*,    \
                                 const R*, const R*, R*, R*, R*);

TCF_NP_INST(double)
TCF_NP_INST(float)

}  // namespace tcf
