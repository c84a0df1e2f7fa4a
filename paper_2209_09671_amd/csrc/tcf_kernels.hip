// HIP kernels of the thermocapillary projection step for gfx950.
//
// Launch shape: blocks of 64 x 4 threads (one wavefront per x-row segment,
// so every global access along x is a coalesced 64-lane transaction), grid
// over (x tiles, y tiles, z planes).  Ghost values outside the walls are
// produced on the fly by reflected indexing (see the ghost rules below), so
// the arrays have exactly the ABI layout and need no padding or ghost-fill
// pass.  Reductions are deterministic: wavefront shuffles, then LDS, then one
// FP64 partial per block, summed in a fixed order by a one-block finalize (or
// by every block of the consuming kernel, in the same fixed order).
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "tcf_device.h"
#include "tcf_internal.h"

namespace tcf {
namespace {

using namespace dev;

// ---------------------------------------------------------------------------
// S3: interface geometry per interior cell -> sigma*kappa, M.
template <class R, int DIM>
__device__ __forceinline__ void normal_at(const R* __restrict__ a, int i, int j, int k, int nx, int ny, int nz,
                                          R ih2, R ne, R n[3]) {
  const R gx = (A_at<DIM>(a, i + 1, j, k, nx, ny, nz) - A_at<DIM>(a, i - 1, j, k, nx, ny, nz)) * ih2;
  const R gy = (A_at<DIM>(a, i, j + 1, k, nx, ny, nz) - A_at<DIM>(a, i, j - 1, k, nx, ny, nz)) * ih2;
  const R gz = DIM == 3 ? (A_at<DIM>(a, i, j, k + 1, nx, ny, nz) - A_at<DIM>(a, i, j, k - 1, nx, ny, nz)) * ih2 : R(0);
  const R inv = frsq(gx * gx + gy * gy + gz * gz + ne * ne);
  n[0] = gx * inv;
  n[1] = gy * inv;
  n[2] = gz * inv;
}

template <class R, int DIM>
__global__ __launch_bounds__(256) void k_geometry(KParams P, const R* __restrict__ a, const R* __restrict__ T,
                                                  const R* __restrict__ cf, R* __restrict__ sk, R* __restrict__ Mx,
                                                  R* __restrict__ My, R* __restrict__ Mz) {
  // the in-plane normals of the block's tile and its one-cell ring (ghost
  // cells included) are computed once into LDS; the two z neighbours' by
  // each thread
  __shared__ R sn[2][BY + 2][BX + 2];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i = blockIdx.x * BX + tx, j = blockIdx.y * BY + ty, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const R ih2 = R(0.5 * P.ih), ne = R(P.neps);
  for (int q = tx + BX * ty; q < (BX + 2) * (BY + 2); q += BX * BY) {
    const int qx = q % (BX + 2), qy = q / (BX + 2);
    const int ii = blockIdx.x * BX - 1 + qx, jj = blockIdx.y * BY - 1 + qy;
    if (ii <= nx && jj <= ny) {
      R nq[3];
      normal_at<R, DIM>(a, ii, jj, k, nx, ny, nz, ih2, ne, nq);
      sn[0][qy][qx] = nq[0];
      sn[1][qy][qx] = nq[1];
    }
  }
  __syncthreads();
  if (i >= nx || j >= ny) return;
  R nn[3], np[3];
  R divn = (sn[0][ty + 1][tx + 2] - sn[0][ty + 1][tx]) * ih2;
  divn += (sn[1][ty + 2][tx + 1] - sn[1][ty][tx + 1]) * ih2;
  if (DIM == 3) {
    normal_at<R, DIM>(a, i, j, k + 1, nx, ny, nz, ih2, ne, np);
    normal_at<R, DIM>(a, i, j, k - 1, nx, ny, nz, ih2, ne, nn);
    divn += (np[2] - nn[2]) * ih2;
  }
  const R kappa = -divn;
  const R gx = (A_at<DIM>(a, i + 1, j, k, nx, ny, nz) - A_at<DIM>(a, i - 1, j, k, nx, ny, nz)) * ih2;
  const R gy = (A_at<DIM>(a, i, j + 1, k, nx, ny, nz) - A_at<DIM>(a, i, j - 1, k, nx, ny, nz)) * ih2;
  const R gz = DIM == 3 ? (A_at<DIM>(a, i, j, k + 1, nx, ny, nz) - A_at<DIM>(a, i, j, k - 1, nx, ny, nz)) * ih2 : R(0);
  const R g2 = gx * gx + gy * gy + gz * gz;
  const R q2 = g2 + ne * ne, ig = frsq(q2);  // 1 / |grad alpha|_eps
  const R ds = g2 * frcp(q2 * ig + ne);
  const R n0 = gx * ig, n1 = gy * ig, n2 = gz * ig;
  const long c = cidx(i, j, k, nx, ny);
  const R s = R(P.s);
  R sigma = R(P.sigma0) + s * (T[c] - R(P.T0));
  R gs0 = s * (T_at<DIM>(T, i + 1, j, k, P) - T_at<DIM>(T, i - 1, j, k, P)) * ih2;
  R gs1 = s * (T_at<DIM>(T, i, j + 1, k, P) - T_at<DIM>(T, i, j - 1, k, P)) * ih2;
  R gs2 = DIM == 3 ? s * (T_at<DIM>(T, i, j, k + 1, P) - T_at<DIM>(T, i, j, k - 1, P)) * ih2 : R(0);
  if (cf) {  // solutal part: sigma += s_c (c - c0), grad sigma += s_c grad c (even ghosts)
    const R sc = R(P.sc);
    sigma += sc * (cf[c] - R(P.c0));
    gs0 += sc * (A_at<DIM>(cf, i + 1, j, k, nx, ny, nz) - A_at<DIM>(cf, i - 1, j, k, nx, ny, nz)) * ih2;
    gs1 += sc * (A_at<DIM>(cf, i, j + 1, k, nx, ny, nz) - A_at<DIM>(cf, i, j - 1, k, nx, ny, nz)) * ih2;
    if (DIM == 3) gs2 += sc * (A_at<DIM>(cf, i, j, k + 1, nx, ny, nz) - A_at<DIM>(cf, i, j, k - 1, nx, ny, nz)) * ih2;
  }
  const R ndg = n0 * gs0 + n1 * gs1 + n2 * gs2;
  sk[c] = sigma * kappa;
  Mx[c] = ds * (gs0 - n0 * ndg);
  My[c] = ds * (gs1 - n1 * ndg);
  if (DIM == 3) Mz[c] = ds * (gs2 - n2 * ndg);
}

// The 3-D geometry marching along z: a 64 x 4 tile per block over a chunk
// of planes.  alpha of planes k-1 .. k+2 with a two-cell ring (ghosts by
// even reflection on load) sits in a five-slot LDS ring, so every plane of
// alpha is read from memory once per tile; the in-plane normals of plane k
// (tile and one-cell ring) are computed once into LDS and the own column's
// z normal of plane k+1 is carried to the next two planes.  Every normal
// and gradient is the same expression as in k_geometry, on the same values.
constexpr int GX = BX + 4, GY = BY + 4, GR = 5;  // alpha tile with its ring, ring slots
constexpr int GN = ((GX * GY) + BX * BY - 1) / (BX * BY);  // alpha loads per thread and plane

template <class R>
__global__ __launch_bounds__(256) void k_geometry_z(KParams P, int kz, int ntx, int nty, const R* __restrict__ a,
                                                    const R* __restrict__ T, const R* __restrict__ cf,
                                                    R* __restrict__ sk, R* __restrict__ Mx, R* __restrict__ My,
                                                    R* __restrict__ Mz) {
  __shared__ R sa[GR][GY][GX];
  __shared__ R snx[BY + 2][BX + 2], sny[BY + 2][BX + 2];
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int t = xcd_tile();
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + BX * ty;
  const int i0 = (t % ntx) * BX, j0 = ((t / ntx) % nty) * BY, tz = t / (ntx * nty);
  const int k0 = tz * kz, k1 = min(k0 + kz, nz);
  const int i = i0 + tx, j = j0 + ty;
  const bool act = i < nx && j < ny;
  const R ih2 = R(0.5 * P.ih), ne = R(P.neps);
  const size_t pl = (size_t)nx * ny;
  // in-plane source offsets of this thread's ring-tile positions (positions
  // past the ring map to a valid cell and are never read)
  unsigned off[GN];
  for (int q = 0; q < GN; ++q) {
    const int e = tid + q * BX * BY;
    const int ex = e % GX, ey = e / GX;
    const int ri = min(max(refl(i0 - 2 + ex, nx), 0), nx - 1), rj = min(max(refl(j0 - 2 + ey, ny), 0), ny - 1);
    off[q] = e < GX * GY ? (unsigned)(ri + nx * rj) : 0u;
  }
  auto plane = [&](int kk) { return (size_t)min(max(refl(kk, nz), 0), nz - 1) * pl; };
  R v[GN];
  auto load = [&](int kk) {
    const size_t po = plane(kk);
    for (int q = 0; q < GN; ++q) v[q] = a[po + off[q]];
  };
  auto store = [&](int kk) {
    const int sl = ((kk % GR) + GR) % GR;
    for (int q = 0; q < GN; ++q) {
      const int e = tid + q * BX * BY;
      if (e < GX * GY) sa[sl][e / GX][e % GX] = v[q];
    }
  };
  auto slot = [&](int kk) { return ((kk % GR) + GR) % GR; };
  for (int kk = k0 - 1; kk <= k0 + 2; ++kk) {
    load(kk);
    store(kk);
  }
  load(k0 + 3);
  // z normals of the own column at planes k0 - 1 and k0
  const int ic = min(i, nx - 1), jc = min(j, ny - 1);
  R nq[3];
  normal_at<R, 3>(a, ic, jc, k0 - 1, nx, ny, nz, ih2, ne, nq);
  R nzm = nq[2];
  normal_at<R, 3>(a, ic, jc, k0, nx, ny, nz, ih2, ne, nq);
  R nzc = nq[2];
  const int X = tx + 2, Y = ty + 2;  // own cell in the alpha tile
  for (int k = k0; k < k1; ++k) {
    __syncthreads();  // planes k-1 .. k+2 are in LDS; the previous plane's reads are done
    const int sm = slot(k - 1), sc = slot(k), sp = slot(k + 1), sq = slot(k + 2);
    // in-plane normals of plane k on the tile and its ring
    for (int e = tid; e < (BX + 2) * (BY + 2); e += BX * BY) {
      const int px = e % (BX + 2) + 1, py = e / (BX + 2) + 1;  // position in the alpha tile
      const R gx = (sa[sc][py][px + 1] - sa[sc][py][px - 1]) * ih2;
      const R gy = (sa[sc][py + 1][px] - sa[sc][py - 1][px]) * ih2;
      const R gz = (sa[sp][py][px] - sa[sm][py][px]) * ih2;
      const R inv = frsq(gx * gx + gy * gy + gz * gz + ne * ne);
      snx[py - 1][px - 1] = gx * inv;
      sny[py - 1][px - 1] = gy * inv;
    }
    // the own column's z normal of plane k + 1
    R nzp;
    {
      const R gx = (sa[sp][Y][X + 1] - sa[sp][Y][X - 1]) * ih2;
      const R gy = (sa[sp][Y + 1][X] - sa[sp][Y - 1][X]) * ih2;
      const R gz = (sa[sq][Y][X] - sa[sc][Y][X]) * ih2;
      const R inv = frsq(gx * gx + gy * gy + gz * gz + ne * ne);
      nzp = gz * inv;
    }
    // plane k + 3 into the slot of plane k - 2 (no longer read), then prefetch k + 4
    store(k + 3);
    load(min(k + 4, nz + 2));
    __syncthreads();
    if (act) {
      R divn = (snx[ty + 1][tx + 2] - snx[ty + 1][tx]) * ih2;
      divn += (sny[ty + 2][tx + 1] - sny[ty][tx + 1]) * ih2;
      divn += (nzp - nzm) * ih2;
      const R kappa = -divn;
      const R gx = (sa[sc][Y][X + 1] - sa[sc][Y][X - 1]) * ih2;
      const R gy = (sa[sc][Y + 1][X] - sa[sc][Y - 1][X]) * ih2;
      const R gz = (sa[sp][Y][X] - sa[sm][Y][X]) * ih2;
      const R g2 = gx * gx + gy * gy + gz * gz;
      const R q2 = g2 + ne * ne, ig = frsq(q2);  // 1 / |grad alpha|_eps
      const R ds = g2 * frcp(q2 * ig + ne);
      const R n0 = gx * ig, n1 = gy * ig, n2 = gz * ig;
      const long c = cidx(i, j, k, nx, ny);
      const R s = R(P.s);
      R sigma = R(P.sigma0) + s * (T[c] - R(P.T0));
      R gs0 = s * (T_at<3>(T, i + 1, j, k, P) - T_at<3>(T, i - 1, j, k, P)) * ih2;
      R gs1 = s * (T_at<3>(T, i, j + 1, k, P) - T_at<3>(T, i, j - 1, k, P)) * ih2;
      R gs2 = s * (T_at<3>(T, i, j, k + 1, P) - T_at<3>(T, i, j, k - 1, P)) * ih2;
      if (cf) {
        const R sc_ = R(P.sc);
        sigma += sc_ * (cf[c] - R(P.c0));
        gs0 += sc_ * (A_at<3>(cf, i + 1, j, k, nx, ny, nz) - A_at<3>(cf, i - 1, j, k, nx, ny, nz)) * ih2;
        gs1 += sc_ * (A_at<3>(cf, i, j + 1, k, nx, ny, nz) - A_at<3>(cf, i, j - 1, k, nx, ny, nz)) * ih2;
        gs2 += sc_ * (A_at<3>(cf, i, j, k + 1, nx, ny, nz) - A_at<3>(cf, i, j, k - 1, nx, ny, nz)) * ih2;
      }
      const R ndg = n0 * gs0 + n1 * gs1 + n2 * gs2;
      sk[c] = sigma * kappa;
      Mx[c] = ds * (gs0 - n0 * ndg);
      My[c] = ds * (gs1 - n1 * ndg);
      Mz[c] = ds * (gs2 - n2 * ndg);
    }
    nzm = nzc;
    nzc = nzp;
  }
}

// ---------------------------------------------------------------------------
// S6: b = D u* / dt (FP64), block partial sums of b.
template <class R, int DIM>
__global__ __launch_bounds__(256) void k_divergence(KParams P, const R* __restrict__ us, const R* __restrict__ vs,
                                                    const R* __restrict__ ws, double* __restrict__ b,
                                                    double* __restrict__ part) {
  __shared__ double sh[8];
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny;
  double val = 0.0;
  if (i < nx && j < ny) {
    double s = ((double)us[fidx<0>(i + 1, j, k, nx, ny)] - (double)us[fidx<0>(i, j, k, nx, ny)]) +
               ((double)vs[fidx<1>(i, j + 1, k, nx, ny)] - (double)vs[fidx<1>(i, j, k, nx, ny)]);
    if (DIM == 3) s += (double)ws[fidx<2>(i, j, k + 1, nx, ny)] - (double)ws[fidx<2>(i, j, k, nx, ny)];
    val = s * P.ih / P.dt;
    b[cidx(i, j, k, nx, ny)] = val;
  }
  const double r = block_reduce<0>(val, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[block_linear()] = r;
}

// Fine-level face weights a_f = 1/(h^2 rho_f) on interior faces, 0 on walls.
template <class R, int DIM, int D>
__global__ __launch_bounds__(256) void k_face_weights(KParams P, const R* __restrict__ a, double* __restrict__ af,
                                                      float* __restrict__ f32) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int fnx = nx + (D == 0), fny = ny + (D == 1);
  if (i >= fnx || j >= fny) return;
  const int id[3] = {i, j, k};
  const int nD = D == 0 ? nx : (D == 1 ? ny : nz);
  const long fo = fidx<D>(i, j, k, nx, ny);
  double val = 0.0;
  if (id[D] > 0 && id[D] < nD) {
    int L[3] = {i, j, k};
    L[D] -= 1;
    const double rL = mixp((double)a[cidx(L[0], L[1], L[2], nx, ny)], P.rho1, P.rho2);
    const double rR = mixp((double)a[cidx(i, j, k, nx, ny)], P.rho1, P.rho2);
    val = (P.ih * P.ih) / (0.5 * (rL + rR));
  }
  af[fo] = val;
  if (f32) f32[fo] = (float)val;
}

// Sum of the face weights of a cell -> omega / diag.
template <class R, int DIM>
__global__ __launch_bounds__(256) void k_wdiag(int nx, int ny, int nz, const R* __restrict__ ax,
                                               const R* __restrict__ ay, const R* __restrict__ az,
                                               R* __restrict__ wd, R omega) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i >= nx || j >= ny) return;
  R d = ax[fidx<0>(i, j, k, nx, ny)] + ax[fidx<0>(i + 1, j, k, nx, ny)] + ay[fidx<1>(i, j, k, nx, ny)] +
        ay[fidx<1>(i, j + 1, k, nx, ny)];
  if (DIM == 3) d += az[fidx<2>(i, j, k, nx, ny)] + az[fidx<2>(i, j, k + 1, nx, ny)];
  wd[cidx(i, j, k, nx, ny)] = d > R(0) ? omega / d : R(0);
}

// One coarse level of the Galerkin hierarchy in one pass.  A fine face
// weight along D: stored (ff), or with FROMA computed from alpha as the
// finest weights are defined, (R)((1/h^2) / (0.5 (rho_L + rho_R))), 0 on the
// walls (the first coarse level when the finest weights are not stored).
template <class R, int D, bool FROMA>
__device__ __forceinline__ R fine_w(const KParams& P, const R* __restrict__ a, const R* __restrict__ ff, int fnx,
                                    int fny, int fnz, int i, int j, int k) {
  if (!FROMA) return ff[fidx<D>(i, j, k, fnx, fny)];
  const int id[3] = {i, j, k};
  const int nD = D == 0 ? fnx : (D == 1 ? fny : fnz);
  if (id[D] <= 0 || id[D] >= nD) return R(0);
  int L[3] = {i, j, k};
  L[D] -= 1;
  const double ih2 = P.ih * P.ih;
  const double rL = mixp((double)a[cidx(L[0], L[1], L[2], fnx, fny)], P.rho1, P.rho2);
  const double rR = mixp((double)a[cidx(i, j, k, fnx, fny)], P.rho1, P.rho2);
  return R(ih2 / (0.5 * (rL + rR)));
}

// Coarse face (I, J, K) along D: the sum of the 2x2 fine faces it covers
// (piecewise-constant P, R = P^T), in a fixed order.
template <class R, int DIM, int D, bool FROMA>
__device__ __forceinline__ R coarse_face(const KParams& P, const R* __restrict__ a, const R* __restrict__ ff,
                                         int fnx, int fny, int fnz, int I, int J, int K) {
  const int kz = DIM == 3 ? 2 : 1;
  R s = R(0);
  if (D == 0) {
    for (int dk = 0; dk < kz; ++dk)
      for (int dj = 0; dj < 2; ++dj) s += fine_w<R, 0, FROMA>(P, a, ff, fnx, fny, fnz, 2 * I, 2 * J + dj, kz * K + dk);
  } else if (D == 1) {
    for (int dk = 0; dk < kz; ++dk)
      for (int di = 0; di < 2; ++di) s += fine_w<R, 1, FROMA>(P, a, ff, fnx, fny, fnz, 2 * I + di, 2 * J, kz * K + dk);
  } else {
    for (int dj = 0; dj < 2; ++dj)
      for (int di = 0; di < 2; ++di) s += fine_w<R, 2, FROMA>(P, a, ff, fnx, fny, fnz, 2 * I + di, 2 * J + dj, 2 * K);
  }
  return s;
}

// One thread per coarse cell: its low face weights along x, y, z (and the
// wall faces at the high ends) and, with WD, omega / diag of the cell, whose
// high faces (written by the neighbours) are recomputed with the same sums.
template <class R, int DIM, bool FROMA, bool WD>
__global__ __launch_bounds__(256) void k_coarsen_level(KParams P, const R* __restrict__ a, const R* __restrict__ fx,
                                                       const R* __restrict__ fy, const R* __restrict__ fz, int fnx,
                                                       int fny, int fnz, int cnx, int cny, int cnz,
                                                       R* __restrict__ cx, R* __restrict__ cy, R* __restrict__ cz,
                                                       R* __restrict__ wd, R omega) {
  const int I = blockIdx.x * BX + threadIdx.x, J = blockIdx.y * BY + threadIdx.y, K = blockIdx.z;
  if (I >= cnx || J >= cny) return;
  const R x0 = coarse_face<R, DIM, 0, FROMA>(P, a, fx, fnx, fny, fnz, I, J, K);
  const R x1 = WD || I == cnx - 1 ? coarse_face<R, DIM, 0, FROMA>(P, a, fx, fnx, fny, fnz, I + 1, J, K) : R(0);
  const R y0 = coarse_face<R, DIM, 1, FROMA>(P, a, fy, fnx, fny, fnz, I, J, K);
  const R y1 = WD || J == cny - 1 ? coarse_face<R, DIM, 1, FROMA>(P, a, fy, fnx, fny, fnz, I, J + 1, K) : R(0);
  cx[fidx<0>(I, J, K, cnx, cny)] = x0;
  if (I == cnx - 1) cx[fidx<0>(cnx, J, K, cnx, cny)] = x1;
  cy[fidx<1>(I, J, K, cnx, cny)] = y0;
  if (J == cny - 1) cy[fidx<1>(I, cny, K, cnx, cny)] = y1;
  R d = x0 + x1 + y0 + y1;
  if (DIM == 3) {
    const R z0 = coarse_face<R, DIM, 2, FROMA>(P, a, fz, fnx, fny, fnz, I, J, K);
    const R z1 = WD || K == cnz - 1 ? coarse_face<R, DIM, 2, FROMA>(P, a, fz, fnx, fny, fnz, I, J, K + 1) : R(0);
    cz[fidx<2>(I, J, K, cnx, cny)] = z0;
    if (K == cnz - 1) cz[fidx<2>(I, J, cnz, cnx, cny)] = z1;
    d += z0 + z1;
  }
  if (WD) wd[cidx(I, J, K, cnx, cny)] = d > R(0) ? omega / d : R(0);
}

// (K x)_c = sum_f a_f (x_c - x_nb) over the faces inside the domain (walls
// carry a_f = 0 and add nothing).  Every load is issued unconditionally (a
// neighbour beyond a wall reads the cell itself, the wall's face weight is
// in bounds) and the wall terms are dropped by selects, so the loads go out
// together instead of one branch, and one memory round trip, per face.
template <class R, int DIM>
__device__ __forceinline__ R applyK(const R* __restrict__ x, const R* __restrict__ ax, const R* __restrict__ ay,
                                    const R* __restrict__ az, int i, int j, int k, int nx, int ny, int nz) {
  const long c = cidx(i, j, k, nx, ny);
  const long pl = (long)nx * ny;
  const bool w = i > 0, e = i < nx - 1, so = j > 0, no = j < ny - 1;
  const bool lo = DIM == 3 && k > 0, hi = DIM == 3 && k < nz - 1;
  const R xc = x[c];
  const R xw = x[w ? c - 1 : c], xe = x[e ? c + 1 : c], xs = x[so ? c - nx : c], xn = x[no ? c + nx : c];
  const R aw = ax[fidx<0>(i, j, k, nx, ny)], ae = ax[fidx<0>(i + 1, j, k, nx, ny)];
  const R as = ay[fidx<1>(i, j, k, nx, ny)], an = ay[fidx<1>(i, j + 1, k, nx, ny)];
  R xl = R(0), xh = R(0), al = R(0), ah = R(0);
  if (DIM == 3) {
    xl = x[lo ? c - pl : c];
    xh = x[hi ? c + pl : c];
    al = az[fidx<2>(i, j, k, nx, ny)];
    ah = az[fidx<2>(i, j, k + 1, nx, ny)];
  }
  R s = R(0);
  s = w ? s + aw * (xc - xw) : s;
  s = e ? s + ae * (xc - xe) : s;
  s = so ? s + as * (xc - xs) : s;
  s = no ? s + an * (xc - xn) : s;
  if (DIM == 3) {
    s = lo ? s + al * (xc - xl) : s;
    s = hi ? s + ah * (xc - xh) : s;
  }
  return s;
}

// applyK with the neighbours taken from X(i, j, k) (an LDS tile) instead of
// an array: the same loads and the same order of the face terms, so the
// result is applyK's bit for bit
template <class R, int DIM, class XAT>
__device__ __forceinline__ R applyK_at(const XAT& X, const R* __restrict__ ax, const R* __restrict__ ay,
                                       const R* __restrict__ az, int i, int j, int k, int nx, int ny, int nz) {
  const bool w = i > 0, e = i < nx - 1, so = j > 0, no = j < ny - 1;
  const bool lo = DIM == 3 && k > 0, hi = DIM == 3 && k < nz - 1;
  const R xc = X(i, j, k);
  const R xw = X(w ? i - 1 : i, j, k), xe = X(e ? i + 1 : i, j, k);
  const R xs = X(i, so ? j - 1 : j, k), xn = X(i, no ? j + 1 : j, k);
  const R aw = ax[fidx<0>(i, j, k, nx, ny)], ae = ax[fidx<0>(i + 1, j, k, nx, ny)];
  const R as = ay[fidx<1>(i, j, k, nx, ny)], an = ay[fidx<1>(i, j + 1, k, nx, ny)];
  R xl = R(0), xh = R(0), al = R(0), ah = R(0);
  if (DIM == 3) {
    xl = X(i, j, lo ? k - 1 : k);
    xh = X(i, j, hi ? k + 1 : k);
    al = az[fidx<2>(i, j, k, nx, ny)];
    ah = az[fidx<2>(i, j, k + 1, nx, ny)];
  }
  R s = R(0);
  s = w ? s + aw * (xc - xw) : s;
  s = e ? s + ae * (xc - xe) : s;
  s = so ? s + as * (xc - xs) : s;
  s = no ? s + an * (xc - xn) : s;
  if (DIM == 3) {
    s = lo ? s + al * (xc - xl) : s;
    s = hi ? s + ah * (xc - xh) : s;
  }
  return s;
}

// rhs = -(b - mean); r = rhs - K x (FP64 b, level precision vectors)
template <class R, int DIM>
__global__ __launch_bounds__(256) void k_rhs_resid(Level<R> L, const double* __restrict__ b,
                                                   const double* __restrict__ scal, R* __restrict__ x,
                                                   R* __restrict__ r, double* __restrict__ pbb,
                                                   double* __restrict__ prr) {
  __shared__ double sh[8];
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  double vb = 0.0, vr = 0.0;
  if (i < L.nx && j < L.ny) {
    const long c = cidx(i, j, k, L.nx, L.ny);
    const double rhs = -(b[c] - scal[S_MEAN]);
    const R rr = R(rhs) - applyK<R, DIM>(x, L.ax, L.ay, L.az, i, j, k, L.nx, L.ny, L.nz);
    r[c] = rr;
    vb = rhs * rhs;
    vr = (double)rr * (double)rr;
  }
  const double sb = block_reduce<0>(vb, sh);
  const double sr = block_reduce<0>(vr, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    pbb[block_linear()] = sb;
    prr[block_linear()] = sr;
  }
}

template <class R, int DIM>
__global__ __launch_bounds__(256) void k_spmv_dot(Level<R> L, const R* __restrict__ d, R* __restrict__ q,
                                                  double* __restrict__ part, const int* __restrict__ iflag) {
  if (iflag[I_DONE]) return;
  __shared__ double sh[8];
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  double val = 0.0;
  if (i < L.nx && j < L.ny) {
    const long c = cidx(i, j, k, L.nx, L.ny);
    const R qq = applyK<R, DIM>(d, L.ax, L.ay, L.az, i, j, k, L.nx, L.ny, L.nz);
    q[c] = qq;
    val = (double)d[c] * (double)qq;
  }
  const double s = block_reduce<0>(val, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[block_linear()] = s;
}

template <class R>
__global__ __launch_bounds__(256) void k_update_xr(long n, const double* __restrict__ scal, R* __restrict__ x,
                                                   R* __restrict__ r, const R* __restrict__ d,
                                                   const R* __restrict__ q, double* __restrict__ part,
                                                   const int* __restrict__ iflag) {
  if (iflag[I_DONE]) return;
  __shared__ double sh[8];
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double val = 0.0;
  if (c < n) {
    const R al = R(scal[S_ALPHA]);
    x[c] += al * d[c];
    const R rr = r[c] - al * q[c];
    r[c] = rr;
    val = (double)rr * (double)rr;
  }
  const double s = block_reduce<0>(val, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <class R>
__global__ __launch_bounds__(256) void k_update_d(long n, const double* __restrict__ scal, const R* __restrict__ z,
                                                  R* __restrict__ d, int first, const int* __restrict__ iflag) {
  if (iflag[I_DONE]) return;
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  d[c] = first ? z[c] : z[c] + R(scal[S_BETA]) * d[c];
}

template <class R>
__global__ __launch_bounds__(256) void k_smooth_first(long n, const R* __restrict__ wd, const R* __restrict__ b,
                                                      R* __restrict__ x, R om, const int* __restrict__ iflag) {
  if (iflag[I_DONE]) return;
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) x[c] = om * wd[c] * b[c];
}

// Per-cell bodies of the multigrid level kernels, shared by the one-kernel
// coarse tail below so that both produce the same values.
// damped Jacobi sweep of cell c = (i, j, k): x + om wdiag (b - K x)
template <class R, int DIM>
__device__ __forceinline__ R smooth_cell(const Level<R>& L, const R* __restrict__ b, const R* __restrict__ x, R om,
                                         int i, int j, int k, long c) {
  const R wd = L.wdiag[c], bc = b[c];
  const R Kx = applyK<R, DIM>(x, L.ax, L.ay, L.az, i, j, k, L.nx, L.ny, L.nz);
  return x[c] + om * wd * (bc - Kx);
}

// residual b - K x of cell (i, j, k)
template <class R, int DIM>
__device__ __forceinline__ R resid_cell(const Level<R>& F, const R* __restrict__ b, const R* __restrict__ x, int i,
                                        int j, int k) {
  return b[cidx(i, j, k, F.nx, F.ny)] - applyK<R, DIM>(x, F.ax, F.ay, F.az, i, j, k, F.nx, F.ny, F.nz);
}

// x' = x + omc P e (piecewise-constant prolongation on the fly), then one
// sweep: x' + om wdiag (b - K x') at cell (i, j, k)
template <class R, int DIM>
__device__ __forceinline__ R prolong_smooth_cell(const Level<R>& L, int cnx, int cny, const R* __restrict__ e,
                                                 const R* __restrict__ b, const R* __restrict__ x, R omc, R om, int i,
                                                 int j, int k) {
  const int kz = DIM == 3 ? 2 : 1;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  auto xp = [&](int ii, int jj, int kk) {
    return x[cidx(ii, jj, kk, nx, ny)] + omc * e[cidx(ii >> 1, jj >> 1, kk / kz, cnx, cny)];
  };
  // (the loads of all faces go out together, as in applyK)
  const long c = cidx(i, j, k, nx, ny);
  const R wd = L.wdiag[c], bc = b[c];
  const bool w = i > 0, ea = i < nx - 1, so = j > 0, no = j < ny - 1;
  const bool lo = DIM == 3 && k > 0, hi = DIM == 3 && k < nz - 1;
  const R xc = xp(i, j, k);
  const R xw = xp(w ? i - 1 : i, j, k), xe = xp(ea ? i + 1 : i, j, k);
  const R xs = xp(i, so ? j - 1 : j, k), xn = xp(i, no ? j + 1 : j, k);
  const R aw = L.ax[fidx<0>(i, j, k, nx, ny)], ae = L.ax[fidx<0>(i + 1, j, k, nx, ny)];
  const R as = L.ay[fidx<1>(i, j, k, nx, ny)], an = L.ay[fidx<1>(i, j + 1, k, nx, ny)];
  R s = R(0);
  s = w ? s + aw * (xc - xw) : s;
  s = ea ? s + ae * (xc - xe) : s;
  s = so ? s + as * (xc - xs) : s;
  s = no ? s + an * (xc - xn) : s;
  if (DIM == 3) {
    const R xl = xp(i, j, lo ? k - 1 : k), xh = xp(i, j, hi ? k + 1 : k);
    const R al = L.az[fidx<2>(i, j, k, nx, ny)], ah = L.az[fidx<2>(i, j, k + 1, nx, ny)];
    s = lo ? s + al * (xc - xl) : s;
    s = hi ? s + ah * (xc - xh) : s;
  }
  return xc + om * wd * (bc - s);
}

// damped Jacobi: xo = x + om wdiag (b - K x) (wdiag = 1 / diag); optional
// partial of b.xo (= r.z on the finest level)
template <class R, int DIM, bool LATE>
__global__ __launch_bounds__(256) void k_smooth(Level<R> L, const R* __restrict__ b, const R* __restrict__ x,
                                                R* __restrict__ xo, R om, double* __restrict__ part,
                                                const int* __restrict__ iflag) {
  const int done = iflag[I_DONE];
  if (!LATE && done) return;
  __shared__ double sh[8];
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const bool in = i < L.nx && j < L.ny;
  const long c = in ? cidx(i, j, k, L.nx, L.ny) : 0;
  R xn = R(0), bc = R(0);
  if (in) {
    xn = smooth_cell<R, DIM>(L, b, x, om, i, j, k, c);
    bc = b[c];
  }
  if (done) return;
  double val = 0.0;
  if (in) {
    xo[c] = xn;
    val = (double)bc * (double)xn;
  }
  if (part) {
    const double s = block_reduce<0>(val, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[block_linear()] = s;
  }
}

// bc = R (b - K x): each coarse cell sums the residuals of its children.
// A 64 x 4 block owns a 64 x 4 x kz tile of fine cells (kz = 2 planes in
// 3D): each thread computes the residuals of its column's kz cells into
// LDS, then one thread per coarse cell of the tile (32 x 2) sums its
// children in (dk, dj, di) order.
template <class R, int DIM, bool LATE>
__global__ __launch_bounds__(256) void k_resid_restrict(Level<R> F, int cnx, int cny, int cnz,
                                                        const R* __restrict__ b, const R* __restrict__ x,
                                                        R* __restrict__ bc, const R* __restrict__ wdc,
                                                        R* __restrict__ x1c, R om0, const int* __restrict__ iflag) {
  const int done = iflag[I_DONE];
  if (!LATE && done) return;
  constexpr int kz = DIM == 3 ? 2 : 1;
  __shared__ R rs[kz][BY][BX];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i = blockIdx.x * BX + tx, j = blockIdx.y * BY + ty, K = blockIdx.z;
  if (i < F.nx && j < F.ny) {
    R rv[kz];
    for (int dk = 0; dk < kz; ++dk) rv[dk] = resid_cell<R, DIM>(F, b, x, i, j, kz * K + dk);
    for (int dk = 0; dk < kz; ++dk) rs[dk][ty][tx] = rv[dk];
  }
  if (done) return;
  __syncthreads();
  const int t = tx + BX * ty;
  if (t >= (BX / 2) * (BY / 2)) return;
  const int ti = t % (BX / 2), tj = t / (BX / 2);
  const int I = blockIdx.x * (BX / 2) + ti, J = blockIdx.y * (BY / 2) + tj;
  if (I >= cnx || J >= cny) return;
  R s = R(0);
  for (int dk = 0; dk < kz; ++dk)
    for (int dj = 0; dj < 2; ++dj)
      for (int di = 0; di < 2; ++di) s += rs[dk][2 * tj + dj][2 * ti + di];
  const long ci = cidx(I, J, K, cnx, cny);
  bc[ci] = s;
  if (x1c) x1c[ci] = om0 * wdc[ci] * s;  // the coarse level's first sweep from zero
}

// x' = x + omega_c P e (on the fly), xo = x' + om wdiag (b - K x')
template <class R, int DIM, bool LATE>
__global__ __launch_bounds__(256) void k_prolong_smooth(Level<R> L, int cnx, int cny, const R* __restrict__ e,
                                                        const R* __restrict__ b, const R* __restrict__ x,
                                                        R* __restrict__ xo, R omc, R om, double* __restrict__ part,
                                                        const int* __restrict__ iflag) {
  const int done = iflag[I_DONE];
  if (!LATE && done) return;
  __shared__ double sh[8];
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const bool in = i < L.nx && j < L.ny;
  const long c = in ? cidx(i, j, k, L.nx, L.ny) : 0;
  R xn = R(0), bv = R(0);
  if (in) {
    xn = prolong_smooth_cell<R, DIM>(L, cnx, cny, e, b, x, omc, om, i, j, k);
    bv = b[c];
  }
  if (done) return;
  double val = 0.0;
  if (in) {
    xo[c] = xn;
    val = (double)bv * (double)xn;
  }
  if (part) {
    const double s = block_reduce<0>(val, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[block_linear()] = s;
  }
}

// Levels of at most 64^3 cells (their kernels take about the same time
// whatever their size: the launch, not the work) with two sweeps before
// and after the coarse correction run two launches per V-cycle instead of
// four.  A block owns a CTX x CTY x CTZ tile (CTZ = 1 in 2-D); its first
// stage sweeps the tile and a one-cell ring (in the domain) into LDS, each
// ring cell being swept again by every block that borders it, and the second
// stage takes the tile's neighbours from there:
//   k_sweep_restrict: x2 = sweep(x1) (written), r = b - K x2, b_c = R r, and
//     the coarse level's first sweep x1_c = om0 b_c / diag_c;
//   k_prolong_sweep2: x' = x + omc P e swept twice, the result written.
// Every value is the one the per-level kernels compute (same cell bodies,
// same order of the face terms and of the children's sum).
constexpr int CTX = 16, CTY = 8;
template <int DIM>
constexpr int ctile_z() {
  return DIM == 3 ? 4 : 1;
}
template <int DIM>
constexpr int ctile_threads() {
  return CTX * CTY * ctile_z<DIM>();
}

template <class R, int DIM>
__global__ __launch_bounds__(ctile_threads<DIM>()) void k_sweep_restrict(Level<R> L, int cnx, int cny,
                                                                      const R* __restrict__ b,
                                                                      const R* __restrict__ x, R* __restrict__ xo,
                                                                      R* __restrict__ bc, const R* __restrict__ wdc,
                                                                      R* __restrict__ x1c, R om, R om0,
                                                                      const int* __restrict__ iflag) {
  constexpr int TZ = ctile_z<DIM>(), NT = ctile_threads<DIM>();
  constexpr int RX = CTX + 2, RY = CTY + 2, RZ = DIM == 3 ? TZ + 2 : 1, NR = RX * RY * RZ;
  constexpr int KZ = DIM == 3 ? 2 : 1;  // fine planes per coarse plane
  __shared__ R s1[NR];
  __shared__ R sr[NT];
  const int done = iflag[I_DONE];
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const int i0 = blockIdx.x * CTX, j0 = blockIdx.y * CTY, k0 = blockIdx.z * TZ;
  const int tid = threadIdx.x;
  for (int q = tid; q < NR; q += NT) {
    const int rx = q % RX, ry = (q / RX) % RY, rz = q / (RX * RY);
    const int ii = i0 - 1 + rx, jj = j0 - 1 + ry, kk = DIM == 3 ? k0 - 1 + rz : 0;
    if (ii >= 0 && ii < nx && jj >= 0 && jj < ny && kk >= 0 && kk < nz)
      s1[q] = smooth_cell<R, DIM>(L, b, x, om, ii, jj, kk, cidx(ii, jj, kk, nx, ny));
  }
  if (done) return;  // the same for the whole block
  __syncthreads();
  const int tx = tid % CTX, ty = (tid / CTX) % CTY, tz = tid / (CTX * CTY);
  const int i = i0 + tx, j = j0 + ty, k = k0 + tz;
  // (every position X is asked for lies in the tile or its ring, in the domain)
  auto X = [&](int ii, int jj, int kk) {
    return s1[(ii - i0 + 1) + RX * ((jj - j0 + 1) + RY * (DIM == 3 ? kk - k0 + 1 : 0))];
  };
  if (i < nx && j < ny && k < nz) {
    const long c = cidx(i, j, k, nx, ny);
    xo[c] = X(i, j, k);
    sr[tid] = b[c] - applyK_at<R, DIM>(X, L.ax, L.ay, L.az, i, j, k, nx, ny, nz);
  }
  __syncthreads();
  // one thread per coarse cell of the tile sums its children in (dk, dj, di)
  // order; the level's sizes are even, so a cell's children are all inside
  // the domain or none is
  constexpr int CX = CTX / 2, CY = CTY / 2, CZ = TZ / KZ;
  if (tid < CX * CY * CZ) {
    const int ti = tid % CX, tj = (tid / CX) % CY, tk = tid / (CX * CY);
    const int I = i0 / 2 + ti, J = j0 / 2 + tj, K = k0 / KZ + tk;
    if (2 * I < nx && 2 * J < ny && KZ * K < nz) {
      R sum = R(0);
      for (int dk = 0; dk < KZ; ++dk)
        for (int dj = 0; dj < 2; ++dj)
          for (int di = 0; di < 2; ++di) sum += sr[(2 * ti + di) + CTX * ((2 * tj + dj) + CTY * (KZ * tk + dk))];
      const long ci = cidx(I, J, K, cnx, cny);
      bc[ci] = sum;
      if (x1c) x1c[ci] = om0 * wdc[ci] * sum;
    }
  }
}

template <class R, int DIM>
__global__ __launch_bounds__(ctile_threads<DIM>()) void k_prolong_sweep2(Level<R> L, int cnx, int cny,
                                                                      const R* __restrict__ e,
                                                                      const R* __restrict__ b,
                                                                      const R* __restrict__ x, R* __restrict__ xo,
                                                                      R omc, R om1, R om2,
                                                                      const int* __restrict__ iflag) {
  constexpr int TZ = ctile_z<DIM>(), NT = ctile_threads<DIM>();
  constexpr int RX = CTX + 2, RY = CTY + 2, RZ = DIM == 3 ? TZ + 2 : 1, NR = RX * RY * RZ;
  __shared__ R s1[NR];
  const int done = iflag[I_DONE];
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const int i0 = blockIdx.x * CTX, j0 = blockIdx.y * CTY, k0 = blockIdx.z * TZ;
  const int tid = threadIdx.x;
  for (int q = tid; q < NR; q += NT) {
    const int rx = q % RX, ry = (q / RX) % RY, rz = q / (RX * RY);
    const int ii = i0 - 1 + rx, jj = j0 - 1 + ry, kk = DIM == 3 ? k0 - 1 + rz : 0;
    if (ii >= 0 && ii < nx && jj >= 0 && jj < ny && kk >= 0 && kk < nz)
      s1[q] = prolong_smooth_cell<R, DIM>(L, cnx, cny, e, b, x, omc, om1, ii, jj, kk);
  }
  if (done) return;  // the same for the whole block
  __syncthreads();
  const int tx = tid % CTX, ty = (tid / CTX) % CTY, tz = tid / (CTX * CTY);
  const int i = i0 + tx, j = j0 + ty, k = k0 + tz;
  auto X = [&](int ii, int jj, int kk) {
    return s1[(ii - i0 + 1) + RX * ((jj - j0 + 1) + RY * (DIM == 3 ? kk - k0 + 1 : 0))];
  };
  if (i < nx && j < ny && k < nz) {
    const long c = cidx(i, j, k, nx, ny);
    const R wd = L.wdiag[c], bv = b[c];
    const R Kx = applyK_at<R, DIM>(X, L.ax, L.ay, L.az, i, j, k, nx, ny, nz);
    xo[c] = X(i, j, k) + om2 * wd * (bv - Kx);
  }
}

// Coarsest level: fixed number of damped-Jacobi sweeps from zero in one block
// (x and x2 are ping-pong buffers; the result ends in x).
template <class R, int DIM>
__global__ __launch_bounds__(1024) void k_coarse(Level<R> L, const R* __restrict__ b, R* __restrict__ x,
                                                 R* __restrict__ x2, int sweeps, R om, const int* __restrict__ iflag) {
  if (iflag[I_DONE]) return;
  const long n = L.n();
  for (long c = threadIdx.x; c < n; c += blockDim.x) x[c] = R(0);
  __syncthreads();
  R* src = x;
  R* dst = x2;
  for (int s = 0; s < sweeps; ++s) {
    for (long c = threadIdx.x; c < n; c += blockDim.x) {
      const int i = (int)(c % L.nx), j = (int)((c / L.nx) % L.ny), k = (int)(c / ((long)L.nx * L.ny));
      const R Kx = applyK<R, DIM>(src, L.ax, L.ay, L.az, i, j, k, L.nx, L.ny, L.nz);
      dst[c] = src[c] + om * L.wdiag[c] * (b[c] - Kx);
    }
    __syncthreads();
    R* t = src;
    src = dst;
    dst = t;
  }
  if (src != x)
    for (long c = threadIdx.x; c < n; c += blockDim.x) x[c] = src[c];
}

// Coarsest level, exact solve: assemble K_c + (gamma/n) 1 1^T (gamma = mean
// diagonal; K_c is singular with the constants as null space, the rank-one
// term makes the matrix SPD and acts as the pseudo-inverse on mean-free
// data), invert it in FP64 by Gauss-Jordan without pivoting (valid for SPD),
// and store the symmetrised inverse in level precision.  One block.
template <class R, int DIM>
__global__ __launch_bounds__(1024) void k_coarse_factor(Level<R> L, double* __restrict__ A, R* __restrict__ Minv) {
  __shared__ double col[kCoarseDenseMax];
  __shared__ double sh[16];
  const int n = (int)L.n();
  const int t = threadIdx.x, nt = blockDim.x;
  const long nn = (long)n * n;
  for (long e = t; e < nn; e += nt) A[e] = 0.0;
  __syncthreads();
  double dsum = 0.0;
  for (int c = t; c < n; c += nt) {
    const int i = c % L.nx, j = (c / L.nx) % L.ny, k = c / (L.nx * L.ny);
    double d = 0.0;
    auto off = [&](int nb, double w) {
      A[(long)c * n + nb] = -w;
      d += w;
    };
    if (i > 0) off(c - 1, (double)L.ax[fidx<0>(i, j, k, L.nx, L.ny)]);
    if (i < L.nx - 1) off(c + 1, (double)L.ax[fidx<0>(i + 1, j, k, L.nx, L.ny)]);
    if (j > 0) off(c - L.nx, (double)L.ay[fidx<1>(i, j, k, L.nx, L.ny)]);
    if (j < L.ny - 1) off(c + L.nx, (double)L.ay[fidx<1>(i, j + 1, k, L.nx, L.ny)]);
    if (DIM == 3) {
      const int pl = L.nx * L.ny;
      if (k > 0) off(c - pl, (double)L.az[fidx<2>(i, j, k, L.nx, L.ny)]);
      if (k < L.nz - 1) off(c + pl, (double)L.az[fidx<2>(i, j, k + 1, L.nx, L.ny)]);
    }
    A[(long)c * n + c] = d;
    dsum += d;
  }
  const double gamma = block_reduce<0>(dsum, sh) / n;
  __syncthreads();
  for (long e = t; e < nn; e += nt) A[e] += gamma / n;
  __syncthreads();
  // in-place Gauss-Jordan inversion
  for (int p = 0; p < n; ++p) {
    for (int i = t; i < n; i += nt) col[i] = A[(long)i * n + p];
    __syncthreads();
    const double piv = 1.0 / col[p];
    for (int j = t; j < n; j += nt) A[(long)p * n + j] = (j == p ? 1.0 : A[(long)p * n + j]) * piv;
    __syncthreads();
    for (long e = t; e < nn; e += nt) {
      const int i = (int)(e / n), j = (int)(e % n);
      if (i == p) continue;
      const double prow = A[(long)p * n + j];
      A[e] = (j == p ? 0.0 : A[e]) - col[i] * prow;
    }
    __syncthreads();
  }
  for (long e = t; e < nn; e += nt) {
    const int i = (int)(e / n), j = (int)(e % n);
    Minv[e] = R(0.5 * (A[e] + A[(long)j * n + i]));
  }
}

// The same inverse for a coarsest level of at most kCoarseLdsMax cells: the
// matrix is assembled in LDS (rows padded by one double against bank
// conflicts) and eliminated in registers, four entries per thread; per pivot
// one barrier after the pivot row and column are published through LDS and
// one after the elimination.
constexpr int kCoarseLdsMax = 64;
template <class R, int DIM>
__global__ __launch_bounds__(1024) void k_coarse_factor_lds(Level<R> L, R* __restrict__ Minv) {
  constexpr int LD = kCoarseLdsMax + 1;
  __shared__ double A[kCoarseLdsMax * LD];
  __shared__ double col[kCoarseLdsMax], prow[kCoarseLdsMax], spj[kCoarseLdsMax];
  __shared__ double sh[16];
  const int n = (int)L.n();
  const int t = threadIdx.x, nt = blockDim.x;
  for (int e = t; e < n * n; e += nt) A[(e / n) * LD + e % n] = 0.0;
  __syncthreads();
  double dsum = 0.0;
  for (int c = t; c < n; c += nt) {
    const int i = c % L.nx, j = (c / L.nx) % L.ny, k = c / (L.nx * L.ny);
    // all six face weights are loaded before any is used (every index is in
    // bounds; walls are dropped below)
    const double w0 = (double)L.ax[fidx<0>(i, j, k, L.nx, L.ny)], w1 = (double)L.ax[fidx<0>(i + 1, j, k, L.nx, L.ny)];
    const double w2 = (double)L.ay[fidx<1>(i, j, k, L.nx, L.ny)], w3 = (double)L.ay[fidx<1>(i, j + 1, k, L.nx, L.ny)];
    double w4 = 0.0, w5 = 0.0;
    if (DIM == 3) {
      w4 = (double)L.az[fidx<2>(i, j, k, L.nx, L.ny)];
      w5 = (double)L.az[fidx<2>(i, j, k + 1, L.nx, L.ny)];
    }
    double d = 0.0;
    auto off = [&](int nb, double w) {
      A[c * LD + nb] = -w;
      d += w;
    };
    if (i > 0) off(c - 1, w0);
    if (i < L.nx - 1) off(c + 1, w1);
    if (j > 0) off(c - L.nx, w2);
    if (j < L.ny - 1) off(c + L.nx, w3);
    if (DIM == 3) {
      const int pl = L.nx * L.ny;
      if (k > 0) off(c - pl, w4);
      if (k < L.nz - 1) off(c + pl, w5);
    }
    A[c * LD + c] = d;
    dsum += d;
  }
  const double gamma = block_reduce<0>(dsum, sh) / n;
  __syncthreads();
  for (int e = t; e < n * n; e += nt) A[(e / n) * LD + e % n] += gamma / n;
  __syncthreads();
  // Thread t owns column j = t % 64 of rows t / 64 + 16 r, r = 0..3
  // (blockDim = 1024), held in registers during the elimination; only the
  // pivot column and row of each step pass through LDS.
  const int jj = t & (kCoarseLdsMax - 1), i0 = t >> 6;
  double m[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + 16 * r;
    m[r] = i < n && jj < n ? A[i * LD + jj] : 0.0;
  }
  // The scaled pivot row is formed once per column (by the pivot row's
  // owners) and read by all: one division per column and step instead of
  // one per element.
  for (int p = 0; p < n; ++p) {
    const int rp = p >> 4;
    if (jj == p) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (i0 + 16 * r < n) col[i0 + 16 * r] = m[r];
    }
    if ((p & 15) == i0 && jj < n) prow[jj] = rp == 0 ? m[0] : (rp == 1 ? m[1] : (rp == 2 ? m[2] : m[3]));
    __syncthreads();
    if ((p & 15) == i0 && jj < n) spj[jj] = (jj == p ? 1.0 : prow[jj]) / col[p];
    __syncthreads();
    if (jj < n) {
      const double pj = spj[jj];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 16 * r;
        if (i < n) m[r] = i == p ? pj : (jj == p ? 0.0 : m[r]) - col[i] * pj;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + 16 * r;
    if (i < n && jj < n) A[i * LD + jj] = m[r];
  }
  __syncthreads();
  for (int e = t; e < n * n; e += nt) {
    const int i = e / n, j = e % n;
    Minv[e] = R(0.5 * (A[i * LD + j] + A[j * LD + i]));
  }
}

// out = Minv b on the coarsest level (one block, one row per thread).
template <class R>
__global__ __launch_bounds__(1024) void k_coarse_apply(int n, const R* __restrict__ Minv, const R* __restrict__ b,
                                                       R* __restrict__ out, const int* __restrict__ iflag) {
  if (iflag[I_DONE]) return;
  __shared__ R sb[kCoarseDenseMax];
  for (int j = threadIdx.x; j < n; j += blockDim.x) sb[j] = b[j];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const R* row = Minv + (long)i * n;
    R s0 = R(0), s1 = R(0);
    int j = 0;
    for (; j + 1 < n; j += 2) {
      s0 += row[j] * sb[j];
      s1 += row[j + 1] * sb[j + 1];
    }
    if (j < n) s0 += row[j] * sb[j];
    out[i] = s0 + s1;
  }
}

// The coarse end of the symmetric V-cycle in one block: from the tail's
// first level (its right-hand side, and unless first_done is clear its
// first pre-smoothing sweep, in b and x2) down to the coarsest level and
// back up, with the same sweeps, restrictions, coarsest solve and
// prolongations, and the same per-cell arithmetic, as the per-level kernels.
// Every level's iterates and right-hand side live in LDS for the whole
// tail (three vectors per level), the face weights are read from memory,
// a block barrier separates the phases, and only the result reaches memory
// (the first level's x).  A thread owns up to kTailPer cells of a level and
// issues all their loads before its first store.  A restriction stages the
// fine residuals in the level's free iterate buffer, then sums each coarse
// cell's children in the per-level kernel's order.
constexpr int kTailThreads = 1024, kTailPer = kTailCells / kTailThreads;
static_assert(kTailPer * kTailThreads == kTailCells, "tail cells per thread");

template <class R, int DIM>
__global__ __launch_bounds__(kTailThreads) void k_mg_tail(MgTail<R> T, const int* __restrict__ iflag) {
  const int done = iflag[I_DONE];  // tested after the first loads (one round trip for both)
  __shared__ R sm[kTailLds];
  const int t = threadIdx.x;
  const int kz = DIM == 3 ? 2 : 1;
  // (32-bit index arithmetic: a tail level holds at most kTailCells cells)
  auto ijk = [](int c, int nx, int ny, int& i, int& j, int& k) {
    const int q = c / nx;
    i = c - q * nx;
    j = q % ny;
    k = q / ny;
  };
  // out[c] = fn(c) for the level's n cells, then a block barrier
  auto phase = [&](int n, R* out, auto fn) {
    R v[kTailPer];
#pragma unroll
    for (int u = 0; u < kTailPer; ++u) {
      const int c = t + u * kTailThreads;
      if (c < n) v[u] = fn(c);
    }
#pragma unroll
    for (int u = 0; u < kTailPer; ++u) {
      const int c = t + u * kTailThreads;
      if (c < n) out[c] = v[u];
    }
    __syncthreads();
  };
  // LDS vectors of level l: X0 (the role of x2), X1 (of x), B (of b)
  auto base = [&](int l) {
    int off = 0;
    for (int q = 0; q < l; ++q) off += 3 * (int)T.lv[q].n();
    return sm + off;
  };
  auto X0 = [&](int l) { return base(l); };
  auto X1 = [&](int l) { return base(l) + (int)T.lv[l].n(); };
  auto Bv = [&](int l) { return base(l) + 2 * (int)T.lv[l].n(); };
  {
    const Level<R>& L = T.lv[0];
    const int n = (int)L.n();
    R* b0 = Bv(0);
    R* x0 = X0(0);
    phase(n, b0, [&](int c) { return L.b[c]; });
    if (done) return;
    if (T.first_done) phase(n, x0, [&](int c) { return L.x2[c]; });
    else phase(n, x0, [&](int c) { return R(T.wpre[0]) * L.wdiag[c] * b0[c]; });
  }
  // after the pre-smoothing of a level its iterate is in buffer (nu - 1) & 1
  // of {X0, X1}, and buffer nu & 1 is free until the post-smoothing
  for (int l = 0; l + 1 < T.nl; ++l) {
    const Level<R>& L = T.lv[l];
    const int n = (int)L.n();
    auto buf = [&](int w) { return (w & 1) ? X1(l) : X0(l); };
    const R* b = Bv(l);
    int w = 1;
    for (int q = 1; q < T.nu; ++q, ++w) {
      const R* xi = buf(w - 1);
      phase(n, buf(w), [&](int c) {
        int i, j, k;
        ijk(c, L.nx, L.ny, i, j, k);
        return smooth_cell<R, DIM>(L, b, xi, R(T.wpre[q]), i, j, k, c);
      });
    }
    const R* cur = buf(w - 1);
    R* rs = buf(w);
    // restriction into level l + 1 (and its first sweep unless it is the coarsest)
    phase(n, rs, [&](int c) {
      int i, j, k;
      ijk(c, L.nx, L.ny, i, j, k);
      return resid_cell<R, DIM>(L, b, cur, i, j, k);
    });
    const Level<R>& C = T.lv[l + 1];
    const int nc = (int)C.n();
    R* bc = Bv(l + 1);
    phase(nc, bc, [&](int ci) {
      int I, J, K;
      ijk(ci, C.nx, C.ny, I, J, K);
      R s = R(0);
      for (int dk = 0; dk < kz; ++dk)
        for (int dj = 0; dj < 2; ++dj)
          for (int di = 0; di < 2; ++di) s += rs[cidx(2 * I + di, 2 * J + dj, kz * K + dk, L.nx, L.ny)];
      return s;
    });
    if (l + 2 < T.nl) phase(nc, X0(l + 1), [&](int ci) { return R(T.wpre[0]) * C.wdiag[ci] * bc[ci]; });
  }
  // coarsest level: x = Minv b (dense inverse), else damped-Jacobi sweeps from zero
  {
    const int lc = T.nl - 1;
    const Level<R>& L = T.lv[lc];
    const int n = (int)L.n();
    const R* b = Bv(lc);
    R* x = X1(lc);
    if (T.cinv) {
      phase(n, x, [&](int i) {
        const R* row = T.cinv + (long)i * n;
        R s0 = R(0), s1 = R(0);
        int j = 0;
        for (; j + 1 < n; j += 2) {
          s0 += row[j] * b[j];
          s1 += row[j + 1] * b[j + 1];
        }
        if (j < n) s0 += row[j] * b[j];
        return s0 + s1;
      });
    } else {
      phase(n, x, [&](int) { return R(0); });
      R* src = x;
      R* dst = X0(lc);
      for (int q = 0; q < T.csweeps; ++q) {
        const R* xi = src;
        phase(n, dst, [&](int c) {
          int i, j, k;
          ijk(c, L.nx, L.ny, i, j, k);
          const R Kx = applyK<R, DIM>(xi, L.ax, L.ay, L.az, i, j, k, L.nx, L.ny, L.nz);
          return xi[c] + R(T.cj) * L.wdiag[c] * (b[c] - Kx);
        });
        R* tmp = src;
        src = dst;
        dst = tmp;
      }
      if (src != x) {
        const R* xi = src;
        phase(n, x, [&](int c) { return xi[c]; });
      }
    }
  }
  for (int l = T.nl - 2; l >= 0; --l) {
    const Level<R>& L = T.lv[l];
    const Level<R>& C = T.lv[l + 1];
    const int n = (int)L.n();
    auto buf = [&](int w) { return (w & 1) ? X1(l) : X0(l); };
    const R* b = Bv(l);
    const R* e = X1(l + 1);
    const R* cur = buf(T.nu - 1);
    // the level's last write (buffer 1, the role of x) of level 0 goes to memory
    auto dest = [&](int w) { return (l == 0 && w == 2 * T.nu - 1) ? L.x : buf(w); };
    int w = T.nu;
    phase(n, dest(w), [&](int c) {
      int i, j, k;
      ijk(c, L.nx, L.ny, i, j, k);
      return prolong_smooth_cell<R, DIM>(L, C.nx, C.ny, e, b, cur, R(T.omc), R(T.wpost[0]), i, j, k);
    });
    ++w;
    for (int q = 1; q < T.nu; ++q, ++w) {
      const R* xi = buf(w - 1);
      phase(n, dest(w), [&](int c) {
        int i, j, k;
        ijk(c, L.nx, L.ny, i, j, k);
        return smooth_cell<R, DIM>(L, b, xi, R(T.wpost[q]), i, j, k, c);
      });
    }
  }
}

// Deterministic finalize of per-block partials, one block per reduction
// (block b takes job b): each of the 1024 threads folds a fixed strided
// subset with four independent accumulators, then the block reduces in a
// fixed order.  The jobs of one launch write different slots.
struct FinJob {
  const double* part;
  int n, op, slot;
  double arg;
};
__global__ __launch_bounds__(1024) void k_finalize(FinJob j0, FinJob j1, double* __restrict__ scal,
                                                   int* __restrict__ iflag) {
  __shared__ double sh[16];
  const FinJob& J = blockIdx.x == 0 ? j0 : j1;
  const double* __restrict__ part = J.part;
  const int n = J.n, op = J.op, slot = J.slot;
  const double arg = J.arg;
  // the done flag is loaded with the partials and tested before the reduction
  const bool gated = op == F_RR;
  const int done = gated ? iflag[I_DONE] : 0;
  const int t = threadIdx.x, nt = blockDim.x;
  double v;
  if (op == F_MIN || op == F_MAX) {
    const double init = op == F_MIN ? DBL_MAX : -DBL_MAX;
    double a0 = init, a1 = init;
    int q = t;
    for (; q + nt < n; q += 2 * nt) {
      const double p0 = part[q], p1 = part[q + nt];
      a0 = op == F_MIN ? fmin(a0, p0) : fmax(a0, p0);
      a1 = op == F_MIN ? fmin(a1, p1) : fmax(a1, p1);
    }
    if (q < n) a0 = op == F_MIN ? fmin(a0, part[q]) : fmax(a0, part[q]);
    if (done) return;
    v = op == F_MIN ? fmin(a0, a1) : fmax(a0, a1);
    v = op == F_MIN ? block_reduce<2>(v, sh) : block_reduce<1>(v, sh);
  } else {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int q = t;
    for (; q + 3 * nt < n; q += 4 * nt) {
      a0 += part[q];
      a1 += part[q + nt];
      a2 += part[q + 2 * nt];
      a3 += part[q + 3 * nt];
    }
    for (; q < n; q += nt) a0 += part[q];
    if (done) return;
    v = block_reduce<0>((a0 + a1) + (a2 + a3), sh);
  }
  if (t != 0) return;
  switch (op) {
    case F_STORE: case F_MIN: case F_MAX: scal[slot] = v; break;
    case F_MEAN: scal[slot] = v / arg; break;
    case F_BB: scal[S_BB] = v; scal[S_TOL2] = arg * v; break;
    case F_RR:
      scal[S_RR] = v;
      iflag[I_ITERS] += (int)arg;
      if (!(v > scal[S_TOL2])) iflag[I_DONE] = 1;   // also stops on NaN
      break;
    case F_SCALE: scal[S_RR64] = v; scal[S_SCALE] = sqrt(v / arg); break;
  }
}

// Copy of the scalar block (scalars and flags, nwords 8-byte words) into
// host memory that the host polls, then the ticket it waits for.  One
// wavefront: its fence covers every store of the copy, so the host that
// sees the ticket sees the block.
// With reset set, the flags (reset[0 .. I_NFLAG)) are cleared after they
// have been copied.
__global__ __launch_bounds__(64) void k_publish(const unsigned long long* src, int nwords,
                                                unsigned long long* dst, unsigned* ticket, unsigned value,
                                                int* reset) {
  for (int q = threadIdx.x; q < nwords; q += 64) dst[q] = src[q];
  __threadfence_system();
  if (threadIdx.x == 0) __hip_atomic_store(ticket, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  if (reset && threadIdx.x < I_NFLAG) reset[threadIdx.x] = 0;
}

__global__ void k_init_flags(int* iflag) {
  if (threadIdx.x < I_NFLAG) iflag[threadIdx.x] = 0;
}

// r32 = r / scale in FP32, and per-block partials of |r32|^2 (FP64)
__global__ __launch_bounds__(256) void k_scale_to32(long n, const double* __restrict__ r,
                                                    const double* __restrict__ scal, float* __restrict__ r32,
                                                    double* __restrict__ part) {
  __shared__ double sh[8];
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (c < n) {
    const float q = (float)(r[c] / scal[S_SCALE]);
    r32[c] = q;
    v = (double)q * (double)q;
  }
  const double sm = block_reduce<0>(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = sm;
}
// p += scale e, with per-block partial sums of the new p (the blocks and the
// order of k_sum64, so the mean is the one k_sum64 would give)
__global__ __launch_bounds__(256) void k_add_scaled(long n, const float* __restrict__ e,
                                                    const double* __restrict__ scal, double* __restrict__ p,
                                                    double* __restrict__ part) {
  __shared__ double sh[8];
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (c < n) {
    v = p[c] + scal[S_SCALE] * (double)e[c];
    p[c] = v;
  }
  const double s = block_reduce<0>(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ __launch_bounds__(256) void k_sub_mean(long n, const double* __restrict__ scal, int slot,
                                                  double* __restrict__ p) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) p[c] -= scal[slot];
}

// per-block partial sums of x (FP64) and of x.y (level precision)
__global__ __launch_bounds__(256) void k_sum64(long n, const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double sh[8];
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const double v = c < n ? x[c] : 0.0;
  const double s = block_reduce<0>(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
template <class R>
__global__ __launch_bounds__(256) void k_dot(long n, const R* __restrict__ x, const R* __restrict__ y,
                                             double* __restrict__ part) {
  __shared__ double sh[8];
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const double v = c < n ? (double)x[c] * (double)y[c] : 0.0;
  const double s = block_reduce<0>(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
template <class R>
__global__ __launch_bounds__(256) void k_fill(long n, R* __restrict__ y, R v) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) y[c] = v;
}

// ---------------------------------------------------------------------------
// S8: projection; in FP32 mode also refresh the FP32 mirror of the velocity.
// One interior face between the cells L and R.
template <class R>
__device__ __forceinline__ double proj_face(const KParams& P, R usv, R aL, R aR, double pL, double pR) {
  const double rhof = 0.5 * (mixp((double)aL, P.rho1, P.rho2) + mixp((double)aR, P.rho1, P.rho2));
  return (double)usv - P.dt * (1.0 / rhof) * (pR - pL) * P.ih;
}

template <class R, int DIM, int D>
__global__ __launch_bounds__(256) void k_project(KParams P, const R* __restrict__ a, const double* __restrict__ p,
                                                 const R* __restrict__ us, double* __restrict__ u,
                                                 R* __restrict__ ur) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int fnx = nx + (D == 0), fny = ny + (D == 1);
  if (i >= fnx || j >= fny) return;
  const int id[3] = {i, j, k};
  const int nD = D == 0 ? nx : (D == 1 ? ny : nz);
  const long fo = fidx<D>(i, j, k, nx, ny);
  double val = 0.0;
  if (id[D] > 0 && id[D] < nD) {
    int L[3] = {i, j, k};
    L[D] -= 1;
    const long cL = cidx(L[0], L[1], L[2], nx, ny), cR = cidx(i, j, k, nx, ny);
    val = proj_face(P, us[fo], a[cL], a[cR], p[cL], p[cR]);
  }
  u[fo] = val;
  if (ur) ur[fo] = (R)val;
}

// Block partials of the six diagnostics, stride apart: sum alpha, min alpha,
// max alpha, |Du|^2, max |u_f|, non-finite flag.
__device__ __forceinline__ void diag_partials(double s, double mn, double mx, double d2, double um, double fin,
                                              double* part, int stride, double* sh) {
  const int bl = blockIdx.x;
  double r;
  r = block_reduce<0>(s, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[bl] = r;
  r = block_reduce<2>(mn, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[stride + bl] = r;
  r = block_reduce<1>(mx, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[2 * stride + bl] = r;
  r = block_reduce<0>(d2, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[3 * stride + bl] = r;
  r = block_reduce<1>(um, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[4 * stride + bl] = r;
  r = block_reduce<1>(fin, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[5 * stride + bl] = r;
}

// Diagnostics per cell: alpha (sum/min/max), |D u|^2 and max |u_f| over the
// cell's low faces (every interior face is some cell's low face), and a
// non-finite flag.  Each thread marches its column over a chunk of kz planes
// (the z face between two planes is loaded once and carried); the block then
// reduces once.  Loads use indexes clamped into the grid, so every thread
// issues the same loads; only active columns contribute.
template <class R, int DIM>
__global__ __launch_bounds__(256) void k_diag(KParams P, int kz, int ntx, int nty, const R* __restrict__ a,
                                              const double* __restrict__ u, const double* __restrict__ v,
                                              const double* __restrict__ w, double* __restrict__ part, int stride) {
  __shared__ double sh[8];
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int t = xcd_tile();
  const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
  const int i = tx * BX + threadIdx.x, j = ty * BY + threadIdx.y;
  const int k0 = tz * kz, k1 = min(k0 + kz, nz);
  const bool act = i < nx && j < ny;
  const int ic = min(i, nx - 1), jc = min(j, ny - 1);
  double s = 0.0, mn = DBL_MAX, mx = -DBL_MAX, d2 = 0.0, um = 0.0, fin = 0.0;
  double w0 = DIM == 3 ? w[fidx<2>(ic, jc, k0, nx, ny)] : 0.0;
  for (int k = k0; k < k1; ++k) {
    const double av = (double)a[cidx(ic, jc, k, nx, ny)];
    const double u0 = u[fidx<0>(ic, jc, k, nx, ny)], u1 = u[fidx<0>(ic + 1, jc, k, nx, ny)];
    const double v0 = v[fidx<1>(ic, jc, k, nx, ny)], v1 = v[fidx<1>(ic, jc + 1, k, nx, ny)];
    const double w1 = DIM == 3 ? w[fidx<2>(ic, jc, k + 1, nx, ny)] : 0.0;
    double dv = (u1 - u0) + (v1 - v0);
    double m = fmax(fabs(u0), fabs(v0));
    double chk = av + u0 + v0;
    if (DIM == 3) {
      dv += w1 - w0;
      m = fmax(m, fabs(w0));
      chk += w0;
    }
    dv *= P.ih;
    if (act) {
      s += av;
      mn = fmin(mn, av);
      mx = fmax(mx, av);
      d2 += dv * dv;
      um = fmax(um, m);
      fin = isfinite(chk) ? fin : 1.0;
    }
    w0 = w1;
  }
  diag_partials(s, mn, mx, d2, um, fin, part, stride, sh);
}

// S8 fused with the diagnostics of k_diag: one pass instead of one per
// velocity component plus k_diag.  Each thread marches the column of
// k_diag's plan and writes the projected low faces of its cells (and the wall
// faces at the high ends).  It recomputes its in-plane high faces from the
// same operands with the same arithmetic (bitwise the values their own cells
// write) and carries the z face between planes, so the diagnostics see
// exactly the stored velocities and follow k_diag's order.  arho is the
// density fraction of the projection (mixed over [P.rho1, P.rho2]), a the
// volume fraction the diagnostics sum.  The column's centre values of p and
// arho roll through registers; every operand of a plane is loaded one plane
// ahead (the last prefetch of a chunk re-reads its last plane and is not
// used); in-plane neighbours are clamped into the grid (a wall face reads
// none of them).
template <class R, int DIM>
__global__ __launch_bounds__(256) void k_project_diag(KParams P, int kz, int ntx, int nty, const R* __restrict__ arho,
                                                      const R* __restrict__ a, const double* __restrict__ p,
                                                      const R* __restrict__ us, const R* __restrict__ vs,
                                                      const R* __restrict__ ws, double* __restrict__ u,
                                                      double* __restrict__ v, double* __restrict__ w,
                                                      R* __restrict__ ur, R* __restrict__ vr, R* __restrict__ wr,
                                                      double* __restrict__ part, int stride) {
  __shared__ double sh[8];
  const int nx = P.nx, ny = P.ny, nz = DIM == 3 ? P.nz : 1;
  const int t = xcd_tile();
  const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
  const int i = tx * BX + threadIdx.x, j = ty * BY + threadIdx.y;
  const int k0 = tz * kz, k1 = min(k0 + kz, nz);
  const bool act = i < nx && j < ny;
  const int ic = min(i, nx - 1), jc = min(j, ny - 1);
  const long pl = (long)nx * ny, col = (long)ic + (long)nx * jc;
  const bool xlo = ic > 0, xhi = ic < nx - 1, ylo = jc > 0, yhi = jc < ny - 1;
  const long oxm = xlo ? -1 : 0, oxp = xhi ? 1 : 0, oym = ylo ? -(long)nx : 0, oyp = yhi ? (long)nx : 0;
  auto plane = [&](int kk) { return (long)min(max(kk, 0), nz - 1) * pl; };
  double s = 0.0, mn = DBL_MAX, mx = -DBL_MAX, d2 = 0.0, um = 0.0, fin = 0.0;
  double pm = p[col + plane(k0 - 1)], pc = p[col + plane(k0)], pp = p[col + plane(k0 + 1)];
  R am = arho[col + plane(k0 - 1)], ac = arho[col + plane(k0)], ap = arho[col + plane(k0 + 1)];
  double wlo = 0.0;  // projected z face below the plane
  if (DIM == 3 && k0 > 0) wlo = proj_face(P, ws[col + (long)k0 * pl], am, ac, pm, pc);
  // the operands of plane k: p and arho of the column two planes up, the
  // in-plane neighbours, the predicted faces and alpha of the cell
  struct Ops {
    double pn, px0, px1, py0, py1;
    R an, ax0, ax1, ay0, ay1, usl, ush, vsl, vsh, wsh, av;
  };
  auto load = [&](int kk, Ops& o) {
    const long c = col + (long)kk * pl, cn = col + plane(kk + 2);
    const long fx = fidx<0>(ic, jc, kk, nx, ny), fy = fidx<1>(ic, jc, kk, nx, ny);
    o.pn = p[cn];
    o.an = arho[cn];
    o.px0 = p[c + oxm];
    o.px1 = p[c + oxp];
    o.py0 = p[c + oym];
    o.py1 = p[c + oyp];
    o.ax0 = arho[c + oxm];
    o.ax1 = arho[c + oxp];
    o.ay0 = arho[c + oym];
    o.ay1 = arho[c + oyp];
    o.usl = us[fx];
    o.ush = us[fx + 1];
    o.vsl = vs[fy];
    o.vsh = vs[fy + nx];
    o.wsh = DIM == 3 ? ws[c + pl] : R(0);
    o.av = a[c];
  };
  // plane k from `cur`, while the next plane's operands load into `nxt`; two
  // operand sets take turns (two planes per pass), so none is copied
  auto step = [&](int k, const Ops& cur, Ops& nxt) {
    load(min(k + 1, k1 - 1), nxt);
    const long c = col + (long)k * pl;
    const long fx = fidx<0>(ic, jc, k, nx, ny), fy = fidx<1>(ic, jc, k, nx, ny);
    const double pn = cur.pn, px0 = cur.px0, px1 = cur.px1, py0 = cur.py0, py1 = cur.py1;
    const R an = cur.an, ax0 = cur.ax0, ax1 = cur.ax1, ay0 = cur.ay0, ay1 = cur.ay1;
    const R usl = cur.usl, ush = cur.ush, vsl = cur.vsl, vsh = cur.vsh, wsh = cur.wsh;
    const double av = (double)cur.av;
    const double u0 = xlo ? proj_face(P, usl, ax0, ac, px0, pc) : 0.0;
    const double u1 = xhi ? proj_face(P, ush, ac, ax1, pc, px1) : 0.0;
    const double v0 = ylo ? proj_face(P, vsl, ay0, ac, py0, pc) : 0.0;
    const double v1 = yhi ? proj_face(P, vsh, ac, ay1, pc, py1) : 0.0;
    const double w0 = wlo;
    const double w1 = DIM == 3 && k + 1 < nz ? proj_face(P, wsh, ac, ap, pc, pp) : 0.0;
    if (act) {
      u[fx] = u0;
      v[fy] = v0;
      if (ur) ur[fx] = (R)u0;
      if (vr) vr[fy] = (R)v0;
      if (i == nx - 1) {
        u[fx + 1] = 0.0;
        if (ur) ur[fx + 1] = R(0);
      }
      if (j == ny - 1) {
        v[fy + nx] = 0.0;
        if (vr) vr[fy + nx] = R(0);
      }
      if (DIM == 3) {
        w[c] = w0;
        if (wr) wr[c] = (R)w0;
        if (k == nz - 1) {
          w[c + pl] = 0.0;
          if (wr) wr[c + pl] = R(0);
        }
      }
    }
    // the diagnostics of k_diag on the projected faces
    double dv = (u1 - u0) + (v1 - v0);
    double m = fmax(fabs(u0), fabs(v0));
    double chk = av + u0 + v0;
    if (DIM == 3) {
      dv += w1 - w0;
      m = fmax(m, fabs(w0));
      chk += w0;
    }
    dv *= P.ih;
    if (act) {
      s += av;
      mn = fmin(mn, av);
      mx = fmax(mx, av);
      d2 += dv * dv;
      um = fmax(um, m);
      fin = isfinite(chk) ? fin : 1.0;
    }
    wlo = w1;
    pm = pc;
    pc = pp;
    pp = pn;
    am = ac;
    ac = ap;
    ap = an;
  };
  Ops oa, ob;
  load(k0, oa);
  int k = k0;
  for (; k + 1 < k1; k += 2) {
    step(k, oa, ob);
    step(k + 1, ob, oa);
  }
  if (k < k1) step(k, oa, ob);
  diag_partials(s, mn, mx, d2, um, fin, part, stride, sh);
}

// The six diagnostics reductions of k_diag's partials in one launch, each in
// the fixed order of k_finalize: sum alpha, min alpha, max alpha, |Du|^2,
// max |u_f|, non-finite flag.
__global__ __launch_bounds__(1024) void k_finalize_diag(const double* __restrict__ part, int n, int stride,
                                                        double* __restrict__ scal) {
  __shared__ double sh[16];
  const int t = threadIdx.x, nt = blockDim.x;
  const int slots[6] = {S_SUMA, S_AMIN, S_AMAX, S_DIV2, S_UMAX, S_NONFIN};
  for (int q6 = 0; q6 < 6; ++q6) {
    const double* pp = part + (long)q6 * stride;
    const int kind = (q6 == 0 || q6 == 3) ? 0 : (q6 == 1 ? 2 : 1);  // 0 sum, 1 max, 2 min
    double v;
    if (kind == 0) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int q = t;
      for (; q + 3 * nt < n; q += 4 * nt) {
        a0 += pp[q];
        a1 += pp[q + nt];
        a2 += pp[q + 2 * nt];
        a3 += pp[q + 3 * nt];
      }
      for (; q < n; q += nt) a0 += pp[q];
      v = block_reduce<0>((a0 + a1) + (a2 + a3), sh);
    } else {
      const double init = kind == 2 ? DBL_MAX : -DBL_MAX;
      double a0 = init;
      for (int q = t; q < n; q += nt) a0 = kind == 2 ? fmin(a0, pp[q]) : fmax(a0, pp[q]);
      v = kind == 2 ? block_reduce<2>(a0, sh) : block_reduce<1>(a0, sh);
    }
    if (t == 0) scal[slots[q6]] = v;
    __syncthreads();
  }
}

// Shu-Osher SSP-RK3 combination of a face velocity with the step's base
// velocity (FP64): stage 1 x <- 3/4 base + 1/4 x, stage 2 x <- base/3 + 2/3 x.
template <class R>
__global__ __launch_bounds__(256) void k_rk_combine(long n, int stage, const double* __restrict__ base,
                                                    R* __restrict__ x) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double b = base[c], v = (double)x[c];
  x[c] = R(stage == 1 ? 0.75 * b + 0.25 * v : b / 3.0 + 2.0 / 3.0 * v);
}

__global__ __launch_bounds__(256) void k_to_f32(long n, const double* __restrict__ x, float* __restrict__ y) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) y[c] = (float)x[c];
}
__global__ __launch_bounds__(256) void k_to_f64(long n, const float* __restrict__ x, double* __restrict__ y) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) y[c] = (double)x[c];
}
template <int M>
__global__ __launch_bounds__(256) void k_extrapolate64(long n, const double* __restrict__ p, const double* h1,
                                                       const double* h2, double* out) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  out[c] = M == 1 ? 2.0 * p[c] - h1[c] : 3.0 * p[c] - 3.0 * h1[c] + h2[c];
}

__global__ __launch_bounds__(256) void k_copy64(long n, const double* __restrict__ x, double* __restrict__ y) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) y[c] = x[c];
}
__global__ __launch_bounds__(256) void k_fill64(long n, double* __restrict__ y, double v) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) y[c] = v;
}

template <class R, int D>
__global__ __launch_bounds__(256) void k_zero_walls(int nx, int ny, int nz, R* __restrict__ f) {
  // threads cover the two wall planes of component D
  const int nD = D == 0 ? nx : (D == 1 ? ny : nz);
  const int a0 = D == 0 ? ny : nx, a1 = D == 2 ? ny : nz;  // extents of the plane
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long plane = (long)a0 * a1;
  if (t >= 2 * plane) return;
  const int side = (int)(t / plane);
  const long q = t % plane;
  const int p0 = (int)(q % a0), p1 = (int)(q / a0);
  const int m = side ? nD : 0;
  long idx;
  if (D == 0) idx = fidx<0>(m, p0, p1, nx, ny);
  else if (D == 1) idx = fidx<1>(p0, m, p1, nx, ny);
  else idx = fidx<2>(p0, p1, m, nx, ny);
  f[idx] = R(0);
}

inline dim3 grid_for(int fnx, int fny, int fnz) { return dim3((fnx + BX - 1) / BX, (fny + BY - 1) / BY, fnz); }
inline dim3 blk() { return dim3(BX, BY, 1); }
inline int nblk1(long n) { return (int)((n + 255) / 256); }

}  // namespace

// =============================================================================
// Launchers
template <class R>
void geometry(const KParams& P, hipStream_t s, const R* a, const R* T, const R* c, R* sk, R* Mx, R* My, R* Mz) {
  if (P.dim == 3) {
    // chunks of planes so that the grid has >= 2048 blocks of 256
    const int ntx = (P.nx + BX - 1) / BX, nty = (P.ny + BY - 1) / BY;
    int nch = std::max(1, std::min(P.nz, (2048 + ntx * nty - 1) / (ntx * nty)));
    const int kz = (P.nz + nch - 1) / nch;
    nch = (P.nz + kz - 1) / kz;
    hipLaunchKernelGGL((k_geometry_z<R>), dim3(ntx * nty * nch), blk(), 0, s, P, kz, ntx, nty, a, T, c, sk, Mx, My,
                       Mz);
  } else {
    hipLaunchKernelGGL((k_geometry<R, 2>), grid_for(P.nx, P.ny, 1), blk(), 0, s, P, a, T, c, sk, Mx, My, Mz);
  }
}

template <class R>
void divergence_rhs(const KParams& P, hipStream_t s, const R* us, const R* vs, const R* ws, double* b,
                    double* part) {
  dim3 g = grid_for(P.nx, P.ny, P.nz);
  if (P.dim == 3) hipLaunchKernelGGL((k_divergence<R, 3>), g, blk(), 0, s, P, us, vs, ws, b, part);
  else hipLaunchKernelGGL((k_divergence<R, 2>), g, blk(), 0, s, P, us, vs, ws, b, part);
}

template <class R>
void face_weights(const KParams& P, hipStream_t s, const R* a, double* ax, double* ay, double* az, float* fx,
                  float* fy, float* fz) {
  if (P.dim == 3) {
    hipLaunchKernelGGL((k_face_weights<R, 3, 0>), grid_for(P.nx + 1, P.ny, P.nz), blk(), 0, s, P, a, ax, fx);
    hipLaunchKernelGGL((k_face_weights<R, 3, 1>), grid_for(P.nx, P.ny + 1, P.nz), blk(), 0, s, P, a, ay, fy);
    hipLaunchKernelGGL((k_face_weights<R, 3, 2>), grid_for(P.nx, P.ny, P.nz + 1), blk(), 0, s, P, a, az, fz);
  } else {
    hipLaunchKernelGGL((k_face_weights<R, 2, 0>), grid_for(P.nx + 1, P.ny, 1), blk(), 0, s, P, a, ax, fx);
    hipLaunchKernelGGL((k_face_weights<R, 2, 1>), grid_for(P.nx, P.ny + 1, 1), blk(), 0, s, P, a, ay, fy);
  }
}

template <class R>
void make_wdiag(hipStream_t s, int dim, const Level<R>& L, double omega) {
  dim3 g = grid_for(L.nx, L.ny, L.nz);
  if (dim == 3) hipLaunchKernelGGL((k_wdiag<R, 3>), g, blk(), 0, s, L.nx, L.ny, L.nz, L.ax, L.ay, L.az, L.wdiag, R(omega));
  else hipLaunchKernelGGL((k_wdiag<R, 2>), g, blk(), 0, s, L.nx, L.ny, L.nz, L.ax, L.ay, L.az, L.wdiag, R(omega));
}

template <class R>
void coarsen_weights(hipStream_t s, int dim, const Level<R>& F, const Level<R>& C) {
  const KParams P{};
  if (dim == 3)
    hipLaunchKernelGGL((k_coarsen_level<R, 3, false, true>), grid_for(C.nx, C.ny, C.nz), blk(), 0, s, P, nullptr, F.ax, F.ay,
                       F.az, F.nx, F.ny, F.nz, C.nx, C.ny, C.nz, C.ax, C.ay, C.az, C.wdiag, R(1.0));
  else
    hipLaunchKernelGGL((k_coarsen_level<R, 2, false, true>), grid_for(C.nx, C.ny, 1), blk(), 0, s, P, nullptr, F.ax, F.ay,
                       nullptr, F.nx, F.ny, F.nz, C.nx, C.ny, C.nz, C.ax, C.ay, nullptr, C.wdiag, R(1.0));
}

template <class R>
void rhs_resid(hipStream_t s, int dim, const Level<R>& L, const double* b, const double* scal, R* x, R* r,
               double* pbb, double* prr) {
  dim3 g = grid_for(L.nx, L.ny, L.nz);
  if (dim == 3) hipLaunchKernelGGL((k_rhs_resid<R, 3>), g, blk(), 0, s, L, b, scal, x, r, pbb, prr);
  else hipLaunchKernelGGL((k_rhs_resid<R, 2>), g, blk(), 0, s, L, b, scal, x, r, pbb, prr);
}

template <class R>
void spmv_dot(hipStream_t s, int dim, const Level<R>& L, const R* d, R* q, double* part,
              const int* iflag) {
  dim3 g = grid_for(L.nx, L.ny, L.nz);
  if (dim == 3) hipLaunchKernelGGL((k_spmv_dot<R, 3>), g, blk(), 0, s, L, d, q, part, iflag);
  else hipLaunchKernelGGL((k_spmv_dot<R, 2>), g, blk(), 0, s, L, d, q, part, iflag);
}

template <class R>
void update_xr(hipStream_t s, long n, const double* scal, R* x, R* r, const R* d, const R* q, double* part, const int* iflag) {
  hipLaunchKernelGGL((k_update_xr<R>), dim3(nblk1(n)), dim3(256), 0, s, n, scal, x, r, d, q, part, iflag);
}

template <class R>
void update_d(hipStream_t s, long n, const double* scal, const R* z, R* d, int first, const int* iflag) {
  hipLaunchKernelGGL((k_update_d<R>), dim3(nblk1(n)), dim3(256), 0, s, n, scal, z, d, first, iflag);
}

// Kernels of levels up to this many cells load the done flag together with
// their data and test it before their first store (one memory round trip
// before the stores instead of two); larger levels test it before loading,
// so that a cycle queued after convergence reads nothing.
constexpr long kLateFlagCells = 64L * 64 * 64;
inline bool late_flag(long n) { return n <= kLateFlagCells; }

template <class R>
void mg_smooth_first(hipStream_t s, const Level<R>& L, const R* b, R* x, double om, const int* iflag) {
  hipLaunchKernelGGL((k_smooth_first<R>), dim3(nblk1(L.n())), dim3(256), 0, s, L.n(), L.wdiag, b, x, R(om), iflag);
}

template <class R>
void mg_smooth(hipStream_t s, int dim, const Level<R>& L, const R* b, const R* x, R* xo, double om, double* part,
               const int* iflag) {
  dim3 g = grid_for(L.nx, L.ny, L.nz);
  auto go = [&](auto kern) { hipLaunchKernelGGL(kern, g, blk(), 0, s, L, b, x, xo, R(om), part, iflag); };
  const bool late = late_flag(L.n());
  if (dim == 3) late ? go(k_smooth<R, 3, true>) : go(k_smooth<R, 3, false>);
  else late ? go(k_smooth<R, 2, true>) : go(k_smooth<R, 2, false>);
}

template <class R>
void mg_resid_restrict(hipStream_t s, int dim, const Level<R>& F, const R* b, const R* x, R* bc, const R* wdc,
                       R* x1c, double om0, const int* iflag) {
  const int cnx = F.nx / 2, cny = F.ny / 2, cnz = dim == 3 ? F.nz / 2 : 1;
  dim3 g = grid_for(F.nx, F.ny, cnz);  // blocks of fine tiles, one coarse plane each
  auto go = [&](auto kern) { hipLaunchKernelGGL(kern, g, blk(), 0, s, F, cnx, cny, cnz, b, x, bc, wdc, x1c, R(om0), iflag); };
  const bool late = late_flag(F.n());
  if (dim == 3) late ? go(k_resid_restrict<R, 3, true>) : go(k_resid_restrict<R, 3, false>);
  else late ? go(k_resid_restrict<R, 2, true>) : go(k_resid_restrict<R, 2, false>);
}

template <class R>
void mg_prolong_smooth(hipStream_t s, int dim, const Level<R>& F, const Level<R>& C, const R* b, const R* x, R* xo,
                       double omega_c, double om, double* part, const int* iflag) {
  dim3 g = grid_for(F.nx, F.ny, F.nz);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, g, blk(), 0, s, F, C.nx, C.ny, C.x, b, x, xo, R(omega_c), R(om), part, iflag);
  };
  const bool late = late_flag(F.n());
  if (dim == 3) late ? go(k_prolong_smooth<R, 3, true>) : go(k_prolong_smooth<R, 3, false>);
  else late ? go(k_prolong_smooth<R, 2, true>) : go(k_prolong_smooth<R, 2, false>);
}

bool mg_fused_level(long n) { return late_flag(n); }

template <class R>
void mg_sweep_restrict(hipStream_t s, int dim, const Level<R>& F, const R* b, const R* x, R* xo, R* bc,
                       const R* wdc, R* x1c, double om, double om0, const int* iflag) {
  const int cnx = F.nx / 2, cny = F.ny / 2;
  if (dim == 3) {
    const dim3 g((F.nx + CTX - 1) / CTX, (F.ny + CTY - 1) / CTY, (F.nz + ctile_z<3>() - 1) / ctile_z<3>());
    hipLaunchKernelGGL((k_sweep_restrict<R, 3>), g, dim3(ctile_threads<3>()), 0, s, F, cnx, cny, b, x, xo, bc, wdc, x1c,
                       R(om), R(om0), iflag);
  } else {
    const dim3 g((F.nx + CTX - 1) / CTX, (F.ny + CTY - 1) / CTY, 1);
    hipLaunchKernelGGL((k_sweep_restrict<R, 2>), g, dim3(ctile_threads<2>()), 0, s, F, cnx, cny, b, x, xo, bc, wdc, x1c,
                       R(om), R(om0), iflag);
  }
}

template <class R>
void mg_prolong_sweep2(hipStream_t s, int dim, const Level<R>& F, const Level<R>& C, const R* b, const R* x, R* xo,
                       double omega_c, double om1, double om2, const int* iflag) {
  if (dim == 3) {
    const dim3 g((F.nx + CTX - 1) / CTX, (F.ny + CTY - 1) / CTY, (F.nz + ctile_z<3>() - 1) / ctile_z<3>());
    hipLaunchKernelGGL((k_prolong_sweep2<R, 3>), g, dim3(ctile_threads<3>()), 0, s, F, C.nx, C.ny, C.x, b, x, xo,
                       R(omega_c), R(om1), R(om2), iflag);
  } else {
    const dim3 g((F.nx + CTX - 1) / CTX, (F.ny + CTY - 1) / CTY, 1);
    hipLaunchKernelGGL((k_prolong_sweep2<R, 2>), g, dim3(ctile_threads<2>()), 0, s, F, C.nx, C.ny, C.x, b, x, xo,
                       R(omega_c), R(om1), R(om2), iflag);
  }
}

template <class R>
void mg_coarse_solve(hipStream_t s, int dim, const Level<R>& L, const R* b, R* x, int sweeps, double om,
                     const int* iflag) {
  if (dim == 3) hipLaunchKernelGGL((k_coarse<R, 3>), dim3(1), dim3(1024), 0, s, L, b, x, L.x2, sweeps, R(om), iflag);
  else hipLaunchKernelGGL((k_coarse<R, 2>), dim3(1), dim3(1024), 0, s, L, b, x, L.x2, sweeps, R(om), iflag);
}

template <class R>
void coarse_factor(hipStream_t s, int dim, const Level<R>& L, double* A, R* Minv) {
  if (L.n() <= kCoarseLdsMax) {
    if (dim == 3) hipLaunchKernelGGL((k_coarse_factor_lds<R, 3>), dim3(1), dim3(1024), 0, s, L, Minv);
    else hipLaunchKernelGGL((k_coarse_factor_lds<R, 2>), dim3(1), dim3(1024), 0, s, L, Minv);
  } else if (dim == 3) {
    hipLaunchKernelGGL((k_coarse_factor<R, 3>), dim3(1), dim3(1024), 0, s, L, A, Minv);
  } else {
    hipLaunchKernelGGL((k_coarse_factor<R, 2>), dim3(1), dim3(1024), 0, s, L, A, Minv);
  }
}

template <class R>
void coarse_apply(hipStream_t s, int n, const R* Minv, const R* b, R* out, const int* iflag) {
  hipLaunchKernelGGL((k_coarse_apply<R>), dim3(1), dim3(1024), 0, s, n, Minv, b, out, iflag);
}

template <class R>
void mg_tail(hipStream_t s, int dim, const MgTail<R>& T, const int* iflag) {
  if (dim == 3) hipLaunchKernelGGL((k_mg_tail<R, 3>), dim3(1), dim3(kTailThreads), 0, s, T, iflag);
  else hipLaunchKernelGGL((k_mg_tail<R, 2>), dim3(1), dim3(kTailThreads), 0, s, T, iflag);
}
template void mg_tail<double>(hipStream_t, int, const MgTail<double>&, const int*);
template void mg_tail<float>(hipStream_t, int, const MgTail<float>&, const int*);
template void coarse_factor<double>(hipStream_t, int, const Level<double>&, double*, double*);
template void coarse_factor<float>(hipStream_t, int, const Level<float>&, double*, float*);
template void coarse_apply<double>(hipStream_t, int, const double*, const double*, double*, const int*);
template void coarse_apply<float>(hipStream_t, int, const float*, const float*, float*, const int*);

void finalize(hipStream_t s, const double* part, int nparts, double* scal, int* iflag, int op, int slot,
              double arg) {
  const FinJob j{part, nparts, op, slot, arg};
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, j, j, scal, iflag);
}

void finalize2(hipStream_t s, const double* part0, const double* part1, int nparts, double* scal, int* iflag,
               int op0, int slot0, double arg0, int op1, int slot1, double arg1) {
  const FinJob j0{part0, nparts, op0, slot0, arg0}, j1{part1, nparts, op1, slot1, arg1};
  hipLaunchKernelGGL(k_finalize, dim3(2), dim3(1024), 0, s, j0, j1, scal, iflag);
}

void init_flags(hipStream_t s, int* iflag) { hipLaunchKernelGGL(k_init_flags, dim3(1), dim3(64), 0, s, iflag); }

void publish(hipStream_t s, const void* src, int nwords, void* dst, unsigned* ticket, unsigned value,
             int* reset_flags) {
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, (const unsigned long long*)src, nwords,
                     (unsigned long long*)dst, ticket, value, reset_flags);
}

template <class R>
void coarsen_from_alpha(const KParams& P, hipStream_t s, const R* a, const Level<R>& C) {
  // each fine weight takes an FP64 division here: the faces are computed once
  // and 1/diag in a pass of its own instead of recomputing the high faces
  if (P.dim == 3)
    hipLaunchKernelGGL((k_coarsen_level<R, 3, true, false>), grid_for(C.nx, C.ny, C.nz), blk(), 0, s, P, a, nullptr,
                       nullptr, nullptr, P.nx, P.ny, P.nz, C.nx, C.ny, C.nz, C.ax, C.ay, C.az, C.wdiag, R(1.0));
  else
    hipLaunchKernelGGL((k_coarsen_level<R, 2, true, false>), grid_for(C.nx, C.ny, 1), blk(), 0, s, P, a, nullptr,
                       nullptr, nullptr, P.nx, P.ny, 1, C.nx, C.ny, C.nz, C.ax, C.ay, nullptr, C.wdiag, R(1.0));
  make_wdiag<R>(s, P.dim, C, 1.0);
}

void scale_to32(hipStream_t s, long n, const double* r, const double* scal, float* r32, double* part) {
  hipLaunchKernelGGL(k_scale_to32, dim3(nblk1(n)), dim3(256), 0, s, n, r, scal, r32, part);
}
int add_scaled(hipStream_t s, long n, const float* e, const double* scal, double* p, double* part) {
  hipLaunchKernelGGL(k_add_scaled, dim3(nblk1(n)), dim3(256), 0, s, n, e, scal, p, part);
  return nblk1(n);
}
void subtract_mean(hipStream_t s, long n, const double* scal, int slot, double* p) {
  hipLaunchKernelGGL(k_sub_mean, dim3(nblk1(n)), dim3(256), 0, s, n, scal, slot, p);
}
int sum64_partials(hipStream_t s, long n, const double* x, double* part) {
  hipLaunchKernelGGL(k_sum64, dim3(nblk1(n)), dim3(256), 0, s, n, x, part);
  return nblk1(n);
}
template <class R>
int dot_partials(hipStream_t s, long n, const R* x, const R* y, double* part) {
  hipLaunchKernelGGL((k_dot<R>), dim3(nblk1(n)), dim3(256), 0, s, n, x, y, part);
  return nblk1(n);
}
template <class R>
void fill(hipStream_t s, long n, R* y, double v) {
  hipLaunchKernelGGL((k_fill<R>), dim3(nblk1(n)), dim3(256), 0, s, n, y, R(v));
}
template int dot_partials<double>(hipStream_t, long, const double*, const double*, double*);
template int dot_partials<float>(hipStream_t, long, const float*, const float*, double*);
template void fill<double>(hipStream_t, long, double*, double);
template void fill<float>(hipStream_t, long, float*, double);

template <class R>
void project(const KParams& P, hipStream_t s, const R* a, const double* p, const R* us, const R* vs, const R* ws,
             double* u, double* v, double* w, R* ur, R* vr, R* wr) {
  if (P.dim == 3) {
    hipLaunchKernelGGL((k_project<R, 3, 0>), grid_for(P.nx + 1, P.ny, P.nz), blk(), 0, s, P, a, p, us, u, ur);
    hipLaunchKernelGGL((k_project<R, 3, 1>), grid_for(P.nx, P.ny + 1, P.nz), blk(), 0, s, P, a, p, vs, v, vr);
    hipLaunchKernelGGL((k_project<R, 3, 2>), grid_for(P.nx, P.ny, P.nz + 1), blk(), 0, s, P, a, p, ws, w, wr);
  } else {
    hipLaunchKernelGGL((k_project<R, 2, 0>), grid_for(P.nx + 1, P.ny, 1), blk(), 0, s, P, a, p, us, u, ur);
    hipLaunchKernelGGL((k_project<R, 2, 1>), grid_for(P.nx, P.ny + 1, 1), blk(), 0, s, P, a, p, vs, v, vr);
  }
}

// Column plan of the diagnostics: chunks of planes so that the grid has
// >= 2048 blocks of 256; returns the number of blocks.
static int diag_plan(const KParams& P, int* kz, int* ntx, int* nty) {
  *ntx = (P.nx + BX - 1) / BX;
  *nty = (P.ny + BY - 1) / BY;
  const int nz = P.dim == 3 ? P.nz : 1;
  const int cols = *ntx * *nty;
  int nch = std::max(1, std::min(nz, (2048 + cols - 1) / cols));
  *kz = (nz + nch - 1) / nch;
  nch = (nz + *kz - 1) / *kz;
  return cols * nch;
}

template <class R>
void project_diag(const KParams& P, hipStream_t s, const R* arho, const R* a, const double* p, const R* us,
                  const R* vs, const R* ws, double* u, double* v, double* w, R* ur, R* vr, R* wr, double* part,
                  int stride, double* scal) {
  int kz, ntx, nty;
  const int nb = diag_plan(P, &kz, &ntx, &nty);
  if (P.dim == 3)
    hipLaunchKernelGGL((k_project_diag<R, 3>), dim3(nb), blk(), 0, s, P, kz, ntx, nty, arho, a, p, us, vs, ws, u, v, w,
                       ur, vr, wr, part, stride);
  else
    hipLaunchKernelGGL((k_project_diag<R, 2>), dim3(nb), blk(), 0, s, P, kz, ntx, nty, arho, a, p, us, vs, ws, u, v, w,
                       ur, vr, wr, part, stride);
  hipLaunchKernelGGL(k_finalize_diag, dim3(1), dim3(1024), 0, s, part, nb, stride, scal);
}

template <class R>
void diagnostics(const KParams& P, hipStream_t s, const R* a, const double* u, const double* v, const double* w,
                 double* part, int stride, double* scal) {
  int kz, ntx, nty;
  const int nb = diag_plan(P, &kz, &ntx, &nty);
  if (P.dim == 3) hipLaunchKernelGGL((k_diag<R, 3>), dim3(nb), blk(), 0, s, P, kz, ntx, nty, a, u, v, w, part, stride);
  else hipLaunchKernelGGL((k_diag<R, 2>), dim3(nb), blk(), 0, s, P, kz, ntx, nty, a, u, v, w, part, stride);
  hipLaunchKernelGGL(k_finalize_diag, dim3(1), dim3(1024), 0, s, part, nb, stride, scal);
}

template <class R>
void rk_combine(hipStream_t s, long n, int stage, const double* base, R* x) {
  hipLaunchKernelGGL((k_rk_combine<R>), dim3(nblk1(n)), dim3(256), 0, s, n, stage, base, x);
}
template void rk_combine<double>(hipStream_t, long, int, const double*, double*);
template void rk_combine<float>(hipStream_t, long, int, const double*, float*);

void to_f32(hipStream_t s, long n, const double* x, float* y) {
  hipLaunchKernelGGL(k_to_f32, dim3(nblk1(n)), dim3(256), 0, s, n, x, y);
}
void to_f64(hipStream_t s, long n, const float* x, double* y) {
  hipLaunchKernelGGL(k_to_f64, dim3(nblk1(n)), dim3(256), 0, s, n, x, y);
}
void extrapolate_f64(hipStream_t s, long n, int m, const double* p, const double* h1, const double* h2,
                     double* out) {
  const dim3 g(nblk1(n)), b(256);
  if (m == 1) hipLaunchKernelGGL((k_extrapolate64<1>), g, b, 0, s, n, p, h1, h2, out);
  else hipLaunchKernelGGL((k_extrapolate64<2>), g, b, 0, s, n, p, h1, h2, out);
}

void copy_f64(hipStream_t s, long n, const double* x, double* y) {
  hipLaunchKernelGGL(k_copy64, dim3(nblk1(n)), dim3(256), 0, s, n, x, y);
}
void fill_f64(hipStream_t s, long n, double* y, double v) {
  hipLaunchKernelGGL(k_fill64, dim3(nblk1(n)), dim3(256), 0, s, n, y, v);
}

template <class R>
void zero_walls(const KParams& P, hipStream_t s, R* u, R* v, R* w) {
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  hipLaunchKernelGGL((k_zero_walls<R, 0>), dim3(nblk1(2L * ny * nz)), dim3(256), 0, s, nx, ny, nz, u);
  hipLaunchKernelGGL((k_zero_walls<R, 1>), dim3(nblk1(2L * nx * nz)), dim3(256), 0, s, nx, ny, nz, v);
  if (P.dim == 3) hipLaunchKernelGGL((k_zero_walls<R, 2>), dim3(nblk1(2L * nx * ny)), dim3(256), 0, s, nx, ny, nz, w);
}

// explicit instantiations
#define TCF_INST(R)                                                                                               \
  template void geometry<R>(const KParams&, hipStream_t, const R*, const R*, const R*, R*, R*, R*, R*);          \
  template void divergence_rhs<R>(const KParams&, hipStream_t, const R*, const R*, const R*, double*, double*);                                                                          \
  template void face_weights<R>(const KParams&, hipStream_t, const R*, double*, double*, double*, float*, float*, \
                                float*);                                                                          \
  template void make_wdiag<R>(hipStream_t, int, const Level<R>&, double);                                         \
  template void coarsen_weights<R>(hipStream_t, int, const Level<R>&, const Level<R>&);                           \
  template void coarsen_from_alpha<R>(const KParams&, hipStream_t, const R*, const Level<R>&);                    \
  template void rhs_resid<R>(hipStream_t, int, const Level<R>&, const double*, const double*, R*, R*, double*,    \
                             double*);                                                                      \
  template void spmv_dot<R>(hipStream_t, int, const Level<R>&, const R*, R*, double*, const int*);          \
  template void update_xr<R>(hipStream_t, long, const double*, R*, R*, const R*, const R*, double*, const int*);                                                                         \
  template void update_d<R>(hipStream_t, long, const double*, const R*, R*, int, const int*);                     \
  template void mg_smooth_first<R>(hipStream_t, const Level<R>&, const R*, R*, double, const int*);                       \
  template void mg_smooth<R>(hipStream_t, int, const Level<R>&, const R*, const R*, R*, double, double*, const int*);                                                                         \
  template void mg_resid_restrict<R>(hipStream_t, int, const Level<R>&, const R*, const R*, R*, const R*, R*,     \
                                     double, const int*);                                                   \
  template void mg_prolong_smooth<R>(hipStream_t, int, const Level<R>&, const Level<R>&, const R*, const R*, R*,  \
                                     double, double, double*, const int*);                                  \
  template void mg_sweep_restrict<R>(hipStream_t, int, const Level<R>&, const R*, const R*, R*, R*, const R*, R*, \
                                     double, double, const int*);                                               \
  template void mg_prolong_sweep2<R>(hipStream_t, int, const Level<R>&, const Level<R>&, const R*, const R*, R*,  \
                                     double, double, double, const int*);                                       \
  template void mg_coarse_solve<R>(hipStream_t, int, const Level<R>&, const R*, R*, int, double, const int*);             \
  template void project<R>(const KParams&, hipStream_t, const R*, const double*, const R*, const R*, const R*,    \
                           double*, double*, double*, R*, R*, R*);                                                \
  template void diagnostics<R>(const KParams&, hipStream_t, const R*, const double*, const double*,               \
                               const double*, double*, int, double*);                                       \
  template void project_diag<R>(const KParams&, hipStream_t, const R*, const R*, const double*, const R*,        \
                                const R*, const R*, double*, double*, double*, R*, R*, R*, double*, int,       \
                                double*);                                                                   \
  template void zero_walls<R>(const KParams&, hipStream_t, R*, R*, R*);

TCF_INST(double)
TCF_INST(float)

}  // namespace tcf
