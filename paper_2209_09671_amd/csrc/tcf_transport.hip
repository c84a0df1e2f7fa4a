// S1 transport stage (WENO5 fluxes of alpha and T, conduction, heat source,
// SSP-RK3 combination), computing every face flux once.
//
// A block owns a 64 x 8 column tile and marches along z over a chunk of
// planes.  alpha and T of the tile's column are carried in 7-plane register
// queues (k-3..k+3), so the z-face fluxes come from registers and the flux
// of the high z-face is reused as the next plane's low face.  The current
// plane, with a 3-cell halo in x and y (ghost rules applied on load), sits
// in a double-buffered LDS tile; the halo of the next plane is prefetched.
// x-face fluxes: each lane computes its low face, the high face arrives from
// the next lane by a wavefront shuffle (a wavefront is one 64-wide row).
// y-face fluxes: each row computes its low face; the high face is read from
// the next row through LDS.  WENO5 weights use one reciprocal per face.
#include <algorithm>

#include "tcf_device.h"
#include "tcf_internal.h"

namespace tcf {
namespace {

using namespace dev;

constexpr int TX = 64, TY = 8, H = 3;
constexpr int SX = TX + 2 * H, SY = TY + 2 * H;
constexpr int NHALO = 2 * H * TY + 2 * H * TX;  // x strips + y strips (corners unused)

// WENO5-JS with the normalisation folded into one reciprocal.
__device__ __forceinline__ float rcpx(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcpx(double x) { return 1.0 / x; }

template <class R>
__device__ __forceinline__ R weno5x(R a, R b, R c, R d, R e, R eps) {
  const R q0 = (R(2) * a - R(7) * b + R(11) * c);
  const R q1 = (-b + R(5) * c + R(2) * d);
  const R q2 = (R(2) * c + R(5) * d - e);
  const R t0 = a - R(2) * b + c, u0 = a - R(4) * b + R(3) * c;
  const R t1 = b - R(2) * c + d, u1 = b - d;
  const R t2 = c - R(2) * d + e, u2 = R(3) * c - R(4) * d + e;
  const R i0 = rcpx(eps + (R(13.0 / 12.0) * t0 * t0 + R(0.25) * u0 * u0));
  const R i1 = rcpx(eps + (R(13.0 / 12.0) * t1 * t1 + R(0.25) * u1 * u1));
  const R i2 = rcpx(eps + (R(13.0 / 12.0) * t2 * t2 + R(0.25) * u2 * u2));
  const R a0 = R(0.1) * i0 * i0, a1 = R(0.6) * i1 * i1, a2 = R(0.3) * i2 * i2;
  return (a0 * q0 + a1 * q1 + a2 * q2) * rcpx(R(6) * (a0 + a1 + a2));
}

// q[m] = Q(f-3+m); value at face f, upwind by the sign of vel
template <class R>
__device__ __forceinline__ R upw(R q0, R q1, R q2, R q3, R q4, R q5, R vel, R eps) {
  return vel >= R(0) ? weno5x(q0, q1, q2, q3, q4, eps) : weno5x(q5, q4, q3, q2, q1, eps);
}

// halo slot -> (ox, oy) offset in the LDS tile (0..SX-1, 0..SY-1)
__device__ __forceinline__ void halo_pos(int h, int& ox, int& oy) {
  if (h < 2 * H * TY) {  // x strips: 3 columns left, 3 right, rows 0..TY-1
    const int side = h / (H * TY), r = h % (H * TY);
    ox = side ? TX + H + (r % H) : (r % H);
    oy = H + r / H;
  } else {  // y strips: 3 rows below, 3 above, columns 0..TX-1
    const int q = h - 2 * H * TY;
    const int side = q / (H * TX), r = q % (H * TX);
    ox = H + r % TX;
    oy = side ? TY + H + r / TX : r / TX;
  }
}

template <class R, int DIM>
__global__ __launch_bounds__(512) void k_transport2(KParams P, int kz, int ntx, int nty, const R* __restrict__ a,
                                                    const R* __restrict__ T, const R* ab, const R* Tb,
                                                    const R* __restrict__ u, const R* __restrict__ v,
                                                    const R* __restrict__ w, R* ao, R* To, R cb, R ci) {
  __shared__ R sa[2][SY][SX];
  __shared__ R sT[2][SY][SX];
  __shared__ R fya[TY][TX];  // low y-face fluxes of the tile rows
  __shared__ R fyt[TY][TX];
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
  // XCD-grouped tile numbering (see the pressure kernels)
  const int nb = gridDim.x, bl = blockIdx.x;
  const int t = (nb % 8 == 0) ? (bl % 8) * (nb / 8) + bl / 8 : bl;
  const int tile_x = t % ntx, rr = t / ntx, tile_y = rr % nty, tile_z = rr / nty;
  const int i0 = tile_x * TX, j0 = tile_y * TY;
  const int i = i0 + tx, j = j0 + ty;
  const int k0 = tile_z * kz, k1 = min(k0 + kz, nz);
  const bool act = i < nx && j < ny;
  // in-tile positions up to 3 cells past the domain hold ghost values that the
  // stencils of the last active cells read (corners are never read)
  const bool cval = i < nx + H && j < ny + H && !(i >= nx && j >= ny);
  const R eps = R(P.weno_eps), ih = R(P.ih), dt = R(P.dt);
  const long pl = (long)nx * ny;
  // halo role of this thread
  int hox = 0, hoy = 0;
  const bool hrole = tid < NHALO;
  if (hrole) halo_pos(tid, hox, hoy);
  const int hi = i0 + hox - H, hj = j0 + hoy - H;
  const bool hvalid = hrole && hi >= -H && hi < nx + H && hj >= -H && hj < ny + H &&
                      (hi >= 0 && hi < nx ? true : (hj >= 0 && hj < ny)) && (hj >= 0 && hj < ny ? true : (hi >= 0 && hi < nx));
  auto ld_a = [&](int ii, int jj, int kk) { return A_at<DIM>(a, ii, jj, kk, nx, ny, nz); };
  auto ld_T = [&](int ii, int jj, int kk) { return T_at<DIM>(T, ii, jj, kk, P); };
  // column queues (k-3 .. k+3); in 2D only the centre is used
  R qa[7], qt[7];
  for (int m = 0; m < 7; ++m) {
    qa[m] = R(0);
    qt[m] = R(0);
  }
  if (cval) {
    if (DIM == 3) {
      for (int m = 0; m < 6; ++m) {
        qa[m + 1] = ld_a(i, j, k0 - 3 + m);
        qt[m + 1] = ld_T(i, j, k0 - 3 + m);
      }
    } else {
      qa[3] = ld_a(i, j, 0);
      qt[3] = ld_T(i, j, 0);
    }
  }
  R ha = R(0), hT = R(0);
  if (hvalid) {
    ha = ld_a(hi, hj, k0);
    hT = ld_T(hi, hj, k0);
  }
  // Gaussian surface heat flux of the column (x, y, t), FP64, once per column
  R qcol = R(0);
  if (P.qP != 0.0 && act) {
    const double xl = P.qx0 + P.qvx * P.t, yl = P.qy0 + P.qvy * P.t;
    const double x = (i + 0.5) * P.h, y = (j + 0.5) * P.h;
    const double r2 = (x - xl) * (x - xl) + (y - yl) * (y - yl);
    const double R2 = P.qr * P.qr;
    qcol = R(2.0 * P.qP / (M_PI * R2) * exp(-2.0 * r2 / R2));
  }
  R fza_lo = R(0), fzt_lo = R(0);  // low z-face flux carried between planes
  bool have_lo = false;
  int buf = 0;
  for (int k = k0; k < k1; ++k) {
    // shift the queues and prefetch plane k+3 and the next plane's halo
    if (DIM == 3) {
      for (int m = 0; m < 6; ++m) {
        qa[m] = qa[m + 1];
        qt[m] = qt[m + 1];
      }
      qa[6] = cval ? ld_a(i, j, k + 3) : R(0);
      qt[6] = cval ? ld_T(i, j, k + 3) : R(0);
    }
    R nha = R(0), nhT = R(0);
    if (hvalid && k + 1 < k1) {
      nha = ld_a(hi, hj, k + 1);
      nhT = ld_T(hi, hj, k + 1);
    }
    // publish the plane
    if (cval) {
      sa[buf][ty + H][tx + H] = qa[3];
      sT[buf][ty + H][tx + H] = qt[3];
    }
    if (hvalid) {
      sa[buf][hoy][hox] = ha;
      sT[buf][hoy][hox] = hT;
    }
    __syncthreads();
    R Fxa_lo = R(0), Fxt_lo = R(0), Fya_lo = R(0), Fyt_lo = R(0);
    const long c = (long)i + (long)nx * ((long)j + (long)ny * k);
    R ulo = R(0), uhi = R(0), vlo = R(0), vhi = R(0);
    if (act) {
      const int X = tx + H, Y = ty + H;
      ulo = u[fidx<0>(i, j, k, nx, ny)];
      vlo = v[fidx<1>(i, j, k, nx, ny)];
      if (i > 0) {
        Fxa_lo = ulo * upw(sa[buf][Y][X - 3], sa[buf][Y][X - 2], sa[buf][Y][X - 1], sa[buf][Y][X], sa[buf][Y][X + 1],
                           sa[buf][Y][X + 2], ulo, eps);
        Fxt_lo = ulo * upw(sT[buf][Y][X - 3], sT[buf][Y][X - 2], sT[buf][Y][X - 1], sT[buf][Y][X], sT[buf][Y][X + 1],
                           sT[buf][Y][X + 2], ulo, eps);
      }
      if (j > 0) {
        Fya_lo = vlo * upw(sa[buf][Y - 3][X], sa[buf][Y - 2][X], sa[buf][Y - 1][X], sa[buf][Y][X], sa[buf][Y + 1][X],
                           sa[buf][Y + 2][X], vlo, eps);
        Fyt_lo = vlo * upw(sT[buf][Y - 3][X], sT[buf][Y - 2][X], sT[buf][Y - 1][X], sT[buf][Y][X], sT[buf][Y + 1][X],
                           sT[buf][Y + 2][X], vlo, eps);
      }
      fya[ty][tx] = Fya_lo;
      fyt[ty][tx] = Fyt_lo;
    }
    // high x-face: next lane's low face, computed here at the tile edge
    R Fxa_hi = __shfl_down(Fxa_lo, 1, 64), Fxt_hi = __shfl_down(Fxt_lo, 1, 64);
    if (act) {
      const int X = tx + H, Y = ty + H;
      if (i + 1 >= nx) {
        Fxa_hi = R(0);
        Fxt_hi = R(0);
      } else if (tx == TX - 1) {
        uhi = u[fidx<0>(i + 1, j, k, nx, ny)];
        Fxa_hi = uhi * upw(sa[buf][Y][X - 2], sa[buf][Y][X - 1], sa[buf][Y][X], sa[buf][Y][X + 1], sa[buf][Y][X + 2],
                           sa[buf][Y][X + 3], uhi, eps);
        Fxt_hi = uhi * upw(sT[buf][Y][X - 2], sT[buf][Y][X - 1], sT[buf][Y][X], sT[buf][Y][X + 1], sT[buf][Y][X + 2],
                           sT[buf][Y][X + 3], uhi, eps);
      }
    }
    __syncthreads();
    if (act) {
      const int X = tx + H, Y = ty + H;
      R Fya_hi = R(0), Fyt_hi = R(0);
      if (j + 1 < ny) {
        if (ty < TY - 1) {
          Fya_hi = fya[ty + 1][tx];
          Fyt_hi = fyt[ty + 1][tx];
        } else {
          vhi = v[fidx<1>(i, j + 1, k, nx, ny)];
          Fya_hi = vhi * upw(sa[buf][Y - 2][X], sa[buf][Y - 1][X], sa[buf][Y][X], sa[buf][Y + 1][X],
                             sa[buf][Y + 2][X], sa[buf][Y + 3][X], vhi, eps);
          Fyt_hi = vhi * upw(sT[buf][Y - 2][X], sT[buf][Y - 1][X], sT[buf][Y][X], sT[buf][Y + 1][X],
                             sT[buf][Y + 2][X], sT[buf][Y + 3][X], vhi, eps);
        }
      }
      R diva = (Fxa_hi - Fxa_lo) + (Fya_hi - Fya_lo);
      R divt = (Fxt_hi - Fxt_lo) + (Fyt_hi - Fyt_lo);
      if (DIM == 3) {
        if (!have_lo) {
          fza_lo = R(0);
          fzt_lo = R(0);
          if (k > 0) {
            const R wl = w[fidx<2>(i, j, k, nx, ny)];
            fza_lo = wl * upw(qa[0], qa[1], qa[2], qa[3], qa[4], qa[5], wl, eps);
            fzt_lo = wl * upw(qt[0], qt[1], qt[2], qt[3], qt[4], qt[5], wl, eps);
          }
        }
        R fza_hi = R(0), fzt_hi = R(0);
        if (k + 1 < nz) {
          const R wh = w[fidx<2>(i, j, k + 1, nx, ny)];
          fza_hi = wh * upw(qa[1], qa[2], qa[3], qa[4], qa[5], qa[6], wh, eps);
          fzt_hi = wh * upw(qt[1], qt[2], qt[3], qt[4], qt[5], qt[6], wh, eps);
        }
        diva += fza_hi - fza_lo;
        divt += fzt_hi - fzt_lo;
        fza_lo = fza_hi;
        fzt_lo = fzt_hi;
        have_lo = true;
      }
      const R ac = qa[3], Tc = qt[3];
      const R La = -diva * ih;
      // conduction: arithmetic-mean face conductivity, ghosts from the tile
      const R lc = mixp(ac, P.lam1, P.lam2);
      R cond = R(0);
      {
        const R an[4] = {sa[buf][Y][X - 1], sa[buf][Y][X + 1], sa[buf][Y - 1][X], sa[buf][Y + 1][X]};
        const R tn[4] = {sT[buf][Y][X - 1], sT[buf][Y][X + 1], sT[buf][Y - 1][X], sT[buf][Y + 1][X]};
        for (int f = 0; f < 4; ++f) cond += R(0.5) * (lc + mixp(an[f], P.lam1, P.lam2)) * (tn[f] - Tc);
        if (DIM == 3) {
          cond += R(0.5) * (lc + mixp(qa[2], P.lam1, P.lam2)) * (qt[2] - Tc);
          cond += R(0.5) * (lc + mixp(qa[4], P.lam1, P.lam2)) * (qt[4] - Tc);
        }
      }
      cond *= ih * ih;
      R src = R(0);
      if (P.qP != 0.0) {
        const R h2 = R(0.5) * ih;
        const R gx = (sa[buf][Y][X + 1] - sa[buf][Y][X - 1]) * h2;
        const R gy = (sa[buf][Y + 1][X] - sa[buf][Y - 1][X]) * h2;
        const R gz = DIM == 3 ? (qa[4] - qa[2]) * h2 : R(0);
        const R g2 = gx * gx + gy * gy + gz * gz;
        const R ne = R(P.neps);
        const R ds = g2 / (sqrt(g2 + ne * ne) + ne);
        src = qcol * ds;
      }
      const R LT = -divt * ih + (cond + src) / mixp(ac, P.rhocp1, P.rhocp2);
      ao[c] = cb * ab[c] + ci * (ac + dt * La);
      To[c] = cb * Tb[c] + ci * (Tc + dt * LT);
    }
    ha = nha;
    hT = nhT;
    buf ^= 1;
  }
}

}  // namespace

int transport_plan(int nx, int ny, int nz, int* kz, int* ntx, int* nty) {
  *ntx = (nx + TX - 1) / TX;
  *nty = (ny + TY - 1) / TY;
  const int cols = *ntx * *nty;
  int ntz = std::max(1, std::min(nz, (1024 + cols - 1) / cols));
  int k = (nz + ntz - 1) / ntz;
  if (k < 8 && nz >= 8) k = 8;
  *kz = std::max(1, k);
  ntz = (nz + *kz - 1) / *kz;
  return cols * ntz;
}

template <class R>
void transport_stage(const KParams& P, hipStream_t s, const R* a, const R* T, const R* ab, const R* Tb, const R* u,
                     const R* v, const R* w, R* ao, R* To, double cb, double ci) {
  int kz, ntx, nty;
  const int nb = transport_plan(P.nx, P.ny, P.nz, &kz, &ntx, &nty);
  if (P.dim == 3)
    hipLaunchKernelGGL((k_transport2<R, 3>), dim3(nb), dim3(TX, TY), 0, s, P, kz, ntx, nty, a, T, ab, Tb, u, v, w, ao,
                       To, R(cb), R(ci));
  else
    hipLaunchKernelGGL((k_transport2<R, 2>), dim3(nb), dim3(TX, TY), 0, s, P, kz, ntx, nty, a, T, ab, Tb, u, v, w, ao,
                       To, R(cb), R(ci));
}

template void transport_stage<double>(const KParams&, hipStream_t, const double*, const double*, const double*,
                                      const double*, const double*, const double*, const double*, double*, double*,
                                      double, double);
template void transport_stage<float>(const KParams&, hipStream_t, const float*, const float*, const float*,
                                     const float*, const float*, const float*, const float*, float*, float*, double,
                                     double);

}  // namespace tcf
