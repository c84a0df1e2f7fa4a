// S4-S5 momentum predictor (WENO5 convection of each velocity component,
// viscous stress divergence, CSF surface tension + Marangoni force),
// computing every flux once.
//
// One launch per component D.  A block owns a 64 x 8 tile of D-faces and
// marches along z.  u_D of the tile's column sits in a 7-plane register
// queue; the current plane, with a 3-face halo in x and y (ghost rules
// applied on load), sits in a double-buffered LDS tile.  For every
// direction E the face needs the flux pair (convective flux, viscous
// stress) on its low and high side; a thread computes the low pair and
// takes the high pair from its neighbour: the next lane (E = x, wavefront
// shuffle), the next row (E = y, LDS) or its own previous plane (E = z,
// registers).  Threads at the tile edge compute the missing high pair.
//
// Flux positions: for E = D the pair sits at the cell centre between two
// D-faces (advecting velocity = mean of the two u_D, stress = 2 mu du_D/dx_D
// with the cell's viscosity); for E != D it sits on the edge between two
// D-faces (advecting velocity = mean of u_E over the two cells on either side
// along D, stress = mu_edge (du_D/dx_E + du_E/dx_D) with mu_edge the mean of
// the four adjacent cell viscosities).
#include <algorithm>

#include "tcf_device.h"
#include "tcf_internal.h"

namespace tcf {
namespace {

using namespace dev;

constexpr int TX = 64, TY = 8, H = 3;
constexpr int SX = TX + 2 * H, SY = TY + 2 * H;
constexpr int NHALO = 2 * H * TY + 2 * H * TX;

__device__ __forceinline__ float rcpx(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcpx(double x) { return 1.0 / x; }

// WENO5-JS reconstruction at the right edge of c, with one reciprocal for
// the normalisation of each smoothness weight and one for the blend.
template <class R>
__device__ __forceinline__ R weno5r(R a, R b, R c, R d, R e, R eps) {
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

// Upwind value at the face between q2 and q3 (q0..q5 = Q(f-3..f+2)); the
// stencil is mirrored by selecting operands, so only one WENO is evaluated.
template <class R>
__device__ __forceinline__ R upw1(R q0, R q1, R q2, R q3, R q4, R q5, R vel, R eps) {
  const bool p = vel >= R(0);
  return weno5r(p ? q0 : q5, p ? q1 : q4, p ? q2 : q3, p ? q3 : q2, p ? q4 : q1, eps);
}

__device__ __forceinline__ int clampi(int x, int n) { return min(max(x, 0), n - 1); }

__device__ __forceinline__ void halo_pos(int h, int& ox, int& oy) {
  if (h < 2 * H * TY) {
    const int side = h / (H * TY), r = h % (H * TY);
    ox = side ? TX + H + (r % H) : (r % H);
    oy = H + r / H;
  } else {
    const int q = h - 2 * H * TY;
    const int side = q / (H * TX), r = q % (H * TX);
    ox = H + r % TX;
    oy = side ? TY + H + r / TX : r / TX;
  }
}

template <class R, int DIM, int D>
struct PredArgs {
  KParams P;
  const R* a;
  const R* sk;
  const R* M;
  const R* u;
  const R* v;
  const R* w;
  R* out;
};

// Cell value with 1-deep even ghosts (a clamp).
template <class R>
__device__ __forceinline__ R cellv(const R* __restrict__ f, int i, int j, int k, int nx, int ny, int nz) {
  return f[cidx(clampi(i, nx), clampi(j, ny), clampi(k, nz), nx, ny)];
}

// Low-side flux pair of direction E for the D-face p (face index along D,
// cell indices along the other axes; along E the face p sits between the
// flux position and p + e_E).  q0..q5 = u_D(p - 3 e_E .. p + 2 e_E).
template <class R, int DIM, int D, int E>
__device__ __forceinline__ void flux_lo(const KParams& P, const R* __restrict__ a, const R* __restrict__ ue, int pi,
                                        int pj, int pk, R q0, R q1, R q2, R q3, R q4, R q5, R eps, R ih, R& F,
                                        R& tau) {
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  int cl[3] = {pi, pj, pk};
  cl[D] -= 1;
  if (E == D) {
    const R U = R(0.5) * (q2 + q3);
    F = U * upw1(q0, q1, q2, q3, q4, q5, U, eps);
    const R mu = mixp(cellv(a, cl[0], cl[1], cl[2], nx, ny, nz), P.mu1, P.mu2);
    tau = R(2) * mu * (q3 - q2) * ih;
  } else {
    const int cr[3] = {pi, pj, pk};
    // u_E on its face p[E], in the cells on either side along D
    int eL[3] = {cl[0], cl[1], cl[2]}, eR[3] = {cr[0], cr[1], cr[2]};
    const int nn[3] = {nx, ny, nz};
    eL[D] = clampi(eL[D], nn[D]);
    eR[D] = clampi(eR[D], nn[D]);
    const R vL = ue[fidx<E>(eL[0], eL[1], DIM == 3 ? eL[2] : 0, nx, ny)];
    const R vR = ue[fidx<E>(eR[0], eR[1], DIM == 3 ? eR[2] : 0, nx, ny)];
    const R Vb = R(0.5) * (vL + vR);
    F = Vb * upw1(q0, q1, q2, q3, q4, q5, Vb, eps);
    // the four cells around the edge: (L, R along D) x (p_E - 1, p_E)
    int lm[3] = {cl[0], cl[1], cl[2]}, rm[3] = {cr[0], cr[1], cr[2]};
    lm[E] -= 1;
    rm[E] -= 1;
    const R me = R(0.25) * (mixp(cellv(a, lm[0], lm[1], lm[2], nx, ny, nz), P.mu1, P.mu2) +
                            mixp(cellv(a, rm[0], rm[1], rm[2], nx, ny, nz), P.mu1, P.mu2) +
                            mixp(cellv(a, cl[0], cl[1], cl[2], nx, ny, nz), P.mu1, P.mu2) +
                            mixp(cellv(a, cr[0], cr[1], cr[2], nx, ny, nz), P.mu1, P.mu2));
    tau = me * ((q3 - q2) + (vR - vL)) * ih;
  }
}

template <class R, int DIM, int D>
__global__ __launch_bounds__(512) void k_pred2(PredArgs<R, DIM, D> A, int kz, int ntx, int nty) {
  __shared__ R sU[2][SY][SX];
  __shared__ R fyF[TY][TX];
  __shared__ R fyT[TY][TX];
  const KParams& P = A.P;
  const R* __restrict__ a = A.a;
  const R* __restrict__ ud = D == 0 ? A.u : (D == 1 ? A.v : A.w);
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  // face-index extents of component D
  const int fn0 = nx + (D == 0), fn1 = ny + (D == 1), fn2 = DIM == 3 ? nz + (D == 2) : 1;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
  const int nb = gridDim.x, bl = blockIdx.x;
  const int t = (nb % 8 == 0) ? (bl % 8) * (nb / 8) + bl / 8 : bl;
  const int tile_x = t % ntx, rr = t / ntx, tile_y = rr % nty, tile_z = rr / nty;
  const int i0 = tile_x * TX, j0 = tile_y * TY;
  const int i = i0 + tx, j = j0 + ty;
  const int k0 = tile_z * kz, k1 = min(k0 + kz, fn2);
  const bool act = i < fn0 && j < fn1;
  const bool cval = i < fn0 + H && j < fn1 + H && !(i >= fn0 && j >= fn1);
  // low-side flux producers: E = x for columns up to the last flux position
  // (x = nx), E = y likewise; the face's own row/column must be a valid one
  const bool xlo = j < fn1 && i <= nx && (D != 0 || i >= 1);
  const bool ylo = i < fn0 && j <= ny && (D != 1 || j >= 1);
  const R eps = R(P.weno_eps), ih = R(P.ih), dt = R(P.dt);
  int hox = 0, hoy = 0;
  const bool hrole = tid < NHALO;
  if (hrole) halo_pos(tid, hox, hoy);
  const int hi = i0 + hox - H, hj = j0 + hoy - H;
  const bool hvalid = hrole && hi >= -H && hi < fn0 + H && hj >= -H && hj < fn1 + H &&
                      (hi >= 0 && hi < fn0 ? true : (hj >= 0 && hj < fn1)) &&
                      (hj >= 0 && hj < fn1 ? true : (hi >= 0 && hi < fn0));
  auto ldU = [&](int ii, int jj, int kk) { return V_at<D, DIM>(ud, ii, jj, kk, nx, ny, nz); };
  R q[7];
#pragma unroll
  for (int m = 0; m < 7; ++m) q[m] = R(0);
  if (cval) {
    if (DIM == 3) {
#pragma unroll
      for (int m = 0; m < 6; ++m) q[m + 1] = ldU(i, j, k0 - 3 + m);
    } else {
      q[3] = ldU(i, j, 0);
    }
  }
  R hu = hvalid ? ldU(hi, hj, k0) : R(0);
  R fz_lo = R(0), tz_lo = R(0);
  bool have_lo = false;
  int buf = 0;
  const R* ue_z = A.w;
  for (int k = k0; k < k1; ++k) {
    if (DIM == 3) {
#pragma unroll
      for (int m = 0; m < 6; ++m) q[m] = q[m + 1];
      q[6] = cval ? ldU(i, j, k + 3) : R(0);
    }
    const R nhu = (hvalid && k + 1 < k1) ? ldU(hi, hj, k + 1) : R(0);
    if (cval) sU[buf][ty + H][tx + H] = q[3];
    if (hvalid) sU[buf][hoy][hox] = hu;
    __syncthreads();
    const int X = tx + H, Y = ty + H;
    // x: low pair by every producer, high pair from the next lane
    R fx = R(0), tx_ = R(0);
    if (xlo)
      flux_lo<R, DIM, D, 0>(P, a, A.u, i, j, k, sU[buf][Y][X - 3], sU[buf][Y][X - 2], sU[buf][Y][X - 1],
                            sU[buf][Y][X], sU[buf][Y][X + 1], sU[buf][Y][X + 2], eps, ih, fx, tx_);
    R fy = R(0), ty_ = R(0);
    if (ylo)
      flux_lo<R, DIM, D, 1>(P, a, A.v, i, j, k, sU[buf][Y - 3][X], sU[buf][Y - 2][X], sU[buf][Y - 1][X],
                            sU[buf][Y][X], sU[buf][Y + 1][X], sU[buf][Y + 2][X], eps, ih, fy, ty_);
    fyF[ty][tx] = fy;
    fyT[ty][tx] = ty_;
    R fxh = __shfl_down(fx, 1, 64), txh = __shfl_down(tx_, 1, 64);
    const bool interior = act && (D == 0 ? (i >= 1 && i < nx) : (D == 1 ? (j >= 1 && j < ny) : (k >= 1 && k < nz)));
    if (interior && tx == TX - 1)
      flux_lo<R, DIM, D, 0>(P, a, A.u, i + 1, j, k, sU[buf][Y][X - 2], sU[buf][Y][X - 1], sU[buf][Y][X],
                            sU[buf][Y][X + 1], sU[buf][Y][X + 2], sU[buf][Y][X + 3], eps, ih, fxh, txh);
    __syncthreads();
    R fyh = R(0), tyh = R(0);
    if (interior) {
      if (ty < TY - 1) {
        fyh = fyF[ty + 1][tx];
        tyh = fyT[ty + 1][tx];
      } else {
        flux_lo<R, DIM, D, 1>(P, a, A.v, i, j + 1, k, sU[buf][Y - 2][X], sU[buf][Y - 1][X], sU[buf][Y][X],
                              sU[buf][Y + 1][X], sU[buf][Y + 2][X], sU[buf][Y + 3][X], eps, ih, fyh, tyh);
      }
    }
    R conv = (fxh - fx) + (fyh - fy);
    R visc = (txh - tx_) + (tyh - ty_);
    if (DIM == 3) {
      // z: the high pair of this plane is the low pair of the next one
      const bool zprod = act && (D != 2 || k < nz);
      if (!have_lo && act && (D != 2 || k >= 1))
        flux_lo<R, DIM, D, 2>(P, a, ue_z, i, j, k, q[0], q[1], q[2], q[3], q[4], q[5], eps, ih, fz_lo, tz_lo);
      R fzh = R(0), tzh = R(0);
      if (zprod)
        flux_lo<R, DIM, D, 2>(P, a, ue_z, i, j, k + 1, q[1], q[2], q[3], q[4], q[5], q[6], eps, ih, fzh, tzh);
      conv += fzh - fz_lo;
      visc += tzh - tz_lo;
      fz_lo = fzh;
      tz_lo = tzh;
      have_lo = true;
    }
    if (act) {
      const long fo = fidx<D>(i, j, k, nx, ny);
      R val = R(0);
      if (interior) {
        int cl[3] = {i, j, k};
        cl[D] -= 1;
        const long cL = cidx(cl[0], cl[1], cl[2], nx, ny), cR = cidx(i, j, k, nx, ny);
        const R aL = a[cL], aR = a[cR];
        const R fst = R(0.5) * (A.sk[cL] + A.sk[cR]) * (aR - aL) * ih + R(0.5) * (A.M[cL] + A.M[cR]);
        const R rhof = R(0.5) * (mixp(aL, P.rho1, P.rho2) + mixp(aR, P.rho1, P.rho2));
        val = q[3] + dt * (-conv * ih + (visc * ih + fst) / rhof);
      }
      A.out[fo] = val;
    }
    hu = nhu;
    buf ^= 1;
  }
}

int pred_plan(int fn0, int fn1, int fn2, int* kz, int* ntx, int* nty) {
  *ntx = (fn0 + TX - 1) / TX;
  *nty = (fn1 + TY - 1) / TY;
  const int cols = *ntx * *nty;
  int ntz = std::max(1, std::min(fn2, (1024 + cols - 1) / cols));
  int k = (fn2 + ntz - 1) / ntz;
  if (k < 8 && fn2 >= 8) k = 8;
  *kz = std::max(1, k);
  ntz = (fn2 + *kz - 1) / *kz;
  return cols * ntz;
}

template <class R, int DIM, int D>
void launch_pred(const KParams& P, hipStream_t s, const R* a, const R* sk, const R* M, const R* u, const R* v,
                 const R* w, R* out) {
  const int fn0 = P.nx + (D == 0), fn1 = P.ny + (D == 1), fn2 = DIM == 3 ? P.nz + (D == 2) : 1;
  int kz, ntx, nty;
  const int nb = pred_plan(fn0, fn1, fn2, &kz, &ntx, &nty);
  PredArgs<R, DIM, D> A{P, a, sk, M, u, v, w, out};
  hipLaunchKernelGGL((k_pred2<R, DIM, D>), dim3(nb), dim3(TX, TY), 0, s, A, kz, ntx, nty);
}

}  // namespace

template <class R>
void predictor(const KParams& P, hipStream_t s, const R* a, const R* sk, const R* Mx, const R* My, const R* Mz,
               const R* u, const R* v, const R* w, R* us, R* vs, R* ws) {
  if (P.dim == 3) {
    launch_pred<R, 3, 0>(P, s, a, sk, Mx, u, v, w, us);
    launch_pred<R, 3, 1>(P, s, a, sk, My, u, v, w, vs);
    launch_pred<R, 3, 2>(P, s, a, sk, Mz, u, v, w, ws);
  } else {
    launch_pred<R, 2, 0>(P, s, a, sk, Mx, u, v, w, us);
    launch_pred<R, 2, 1>(P, s, a, sk, My, u, v, w, vs);
  }
}

template void predictor<double>(const KParams&, hipStream_t, const double*, const double*, const double*,
                                const double*, const double*, const double*, const double*, const double*, double*,
                                double*, double*);
template void predictor<float>(const KParams&, hipStream_t, const float*, const float*, const float*, const float*,
                               const float*, const float*, const float*, const float*, float*, float*, float*);

}  // namespace tcf
