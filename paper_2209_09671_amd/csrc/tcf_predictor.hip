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
#include <type_traits>

#include "tcf_device.h"
#include "tcf_internal.h"

namespace tcf {
namespace {

using namespace dev;

#ifndef TCF_PRED_PF
#define TCF_PRED_PF 1
#endif

constexpr int TX = 64, TY = 8, H = 3;
constexpr int SX = TX + 2 * H, SY = TY + 2 * H;
constexpr int NHALO = 2 * H * TY + 2 * H * TX;

__device__ __forceinline__ float rcpx(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcpx(double x) { return 1.0 / x; }

// WENO5-JS reconstruction at the right edge of c, with one reciprocal: the
// nonlinear weights d_k / x_k^2 (x_k = eps + beta_k) are put over the common
// denominator (x_0 x_1 x_2)^2 and scaled by 10 (d = 1, 6, 3); in FP32 the
// x_k are first scaled by a power of two (wscale) that keeps the products in
// range.  With
// t_k the second differences and u_k the one-sided differences of the three
// candidate stencils, the candidates' values are c + (t_0 + 3 u_0)/12,
// c + (t_1 - 3 u_1)/12 and c + (t_2 - 3 u_2)/12: the blend is c plus the
// weighted mean of those corrections.  The smoothness indicators
// beta_k = (13/12) t_k^2 + (1/4) u_k^2 and epsilon are both taken times
// 12/13 (eps_w = (12/13) eps), which leaves the normalised weights
// d_k / (eps + beta_k)^2 unchanged: one multiply and two FMAs per indicator.
// FP32: the three smoothness terms are scaled by one power of two that
// brings the largest into [1/2, 1) (exact, so the normalised weights are
// unchanged), which keeps the products of the common denominator in range;
// a term below 1e-19 of the largest then has a weight that underflows to
// zero, against weights of order 1.  FP64 needs no scaling.
__device__ __forceinline__ void wscale(float& x0, float& x1, float& x2) {
  const int e = __builtin_amdgcn_frexp_expf(fmaxf(x0, fmaxf(x1, x2)));
  x0 = __builtin_amdgcn_ldexpf(x0, -e);
  x1 = __builtin_amdgcn_ldexpf(x1, -e);
  x2 = __builtin_amdgcn_ldexpf(x2, -e);
}
__device__ __forceinline__ void wscale(double&, double&, double&) {}

template <class R>
__device__ __forceinline__ R weno5r(R a, R b, R c, R d, R e, R epsw) {
  const R t0 = a - R(2) * b + c, u0 = a - R(4) * b + R(3) * c;
  const R t1 = b - R(2) * c + d, u1 = b - d;
  const R t2 = c - R(2) * d + e, u2 = R(3) * c - R(4) * d + e;
  const R cu = R(3.0 / 13.0);
  const R x0 = fma(cu * u0, u0, fma(t0, t0, epsw));
  const R x1 = fma(cu * u1, u1, fma(t1, t1, epsw));
  const R x2 = fma(cu * u2, u2, fma(t2, t2, epsw));
  R y0 = x0, y1 = x1, y2 = x2;
  wscale(y0, y1, y2);
  const R p12 = y1 * y2, p02 = y0 * y2, p01 = y0 * y1;
  const R a0 = p12 * p12, a1 = R(6) * p02 * p02, a2 = R(3) * p01 * p01;
  const R sc = fma(a2, fma(R(-3), u2, t2), fma(a1, fma(R(-3), u1, t1), a0 * fma(R(3), u0, t0)));
  return fma(sc, rcpx(R(12) * (a0 + a1 + a2)), c);
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
  const R* ff;  // the material form: the face CSF force on the D-faces
};

// In-plane offsets of one in-plane flux position (direction E = x or y) of
// the D-face (px, py): cells L and R on either side along D (for D = z the
// same column, in planes k-1 and k), the same cells shifted by -1 along E,
// and u_E on face p_E in the columns of L and R.  Cell indices outside the
// domain take the 1-deep even ghost (a clamp); face indices along E are in
// range for every producer.
struct SiteXY {
  unsigned cL, cR, sL, sR, eL, eR;
};

template <int D, int E>
__device__ __forceinline__ SiteXY site_xy(int px, int py, int nx, int ny) {
  const int cxL = px - (D == 0), cyL = py - (D == 1), cxR = px, cyR = py;
  auto coff = [&](int x, int y) { return (unsigned)(clampi(x, nx) + nx * clampi(y, ny)); };
  SiteXY s;
  s.cL = coff(cxL, cyL);
  s.cR = coff(cxR, cyR);
  s.sL = coff(cxL - (E == 0), cyL - (E == 1));
  s.sR = coff(cxR - (E == 0), cyR - (E == 1));
  if (E == 0) {  // u on x-face px, cell rows of L and R
    s.eL = (unsigned)(px + (nx + 1) * clampi(cyL, ny));
    s.eR = (unsigned)(px + (nx + 1) * clampi(cyR, ny));
  } else {  // v on y-face py, cell columns of L and R
    s.eL = (unsigned)(clampi(cxL, nx) + nx * py);
    s.eR = (unsigned)(clampi(cxR, nx) + nx * py);
  }
  return s;
}

// Per-plane operands of one in-plane flux item: the cells L and R (c, cR),
// the same shifted by -1 along E (s, sR) and u_E in the columns of L and R.
// For E = D only c (the cell between the two D-faces) is used.
template <class R>
struct FluxOps {
  R c, cR, s, sR, vL, vR;
};

template <class R, int D, int E>
__device__ __forceinline__ void load_ops(FluxOps<R>& o, const SiteXY& s, const R* __restrict__ aL,
                                         const R* __restrict__ aR, const R* __restrict__ eLp,
                                         const R* __restrict__ eRp) {
  o.c = aL[s.cL];
  if (E != D) {
    o.cR = aR[s.cR];
    o.s = aL[s.sL];
    o.sR = aR[s.sR];
    o.vL = eLp[s.eL];
    o.vR = eRp[s.eR];
  }
}

// Low-side flux pair (convective flux, viscous stress times h) of the
// in-plane direction E; q0..q5 = u_D(p - 3 e_E .. p + 2 e_E).
template <class R, int D, int E>
__device__ __forceinline__ void flux_pair(const KParams& P, const FluxOps<R>& o, R q0, R q1, R q2, R q3, R q4, R q5,
                                          R eps, R& F, R& tau) {
  if (E == D) {  // cell-centred: advecting velocity from u_D, stress 2 mu du_D/dx_D
    const R U = R(0.5) * (q2 + q3);
    F = U * upw1(q0, q1, q2, q3, q4, q5, U, eps);
    tau = R(2) * mixp(o.c, P.mu1, P.mu2) * (q3 - q2);
  } else {  // edge: u_E averaged over L and R, mu over the four cells
    const R Vb = R(0.5) * (o.vL + o.vR);
    F = Vb * upw1(q0, q1, q2, q3, q4, q5, Vb, eps);
    const R me = R(0.25) * (mixp(o.s, P.mu1, P.mu2) + mixp(o.sR, P.mu1, P.mu2) + mixp(o.c, P.mu1, P.mu2) +
                            mixp(o.cR, P.mu1, P.mu2));
    tau = me * ((q3 - q2) + (o.vR - o.vL));
  }
}

// Per-plane operands of the face itself: z-edge (D != z: u_z on the high
// z-face in the columns of L and R, alpha of plane k+1) or cell-centre
// (D = z: alpha of the cell above the face), and the force operands.
template <class R>
struct FaceOps {
  R wL, wR, apL, apR;  // D != z: w(k+1) at L, R and alpha(k+1) at L, R; D = z: apR = alpha(k)
  R skL, skR, mL, mR;  // sigma*kappa and M_D in the cells L and R
};

// PF: the per-plane operands of the first flux items and of the face are
// loaded one plane ahead (FP32); otherwise at the top of their own plane.
// MAT: the material form of the N-phase model.  a is then the viscosity
// as a fraction of [mu1, mu2], sk the density as a fraction of [rho1, rho2],
// and the face force comes precomputed (ff) instead of from sigma*kappa, M
// and the jump of alpha; every other operand and step is the same.
template <class R, int DIM, int D, bool PF, bool MAT>
__device__ __forceinline__ void pred_body(const PredArgs<R, DIM, D>& A, int kz, int ntx, int nty) {
  __shared__ R sU[2][SY][SX];
  __shared__ R fxF[TY][TX + 1];
  __shared__ R fxT[TY][TX + 1];
  __shared__ R fyF[TY + 1][TX];
  __shared__ R fyT[TY + 1][TX];
  const KParams& P = A.P;
  const R* __restrict__ a = A.a;
  const R* __restrict__ ud = D == 0 ? A.u : (D == 1 ? A.v : A.w);
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  // face-index extents of u_D; the tiles and the march cover faces 0..n-1
  // along D, the last wall face is written by its neighbour
  const int fn0 = nx + (D == 0), fn1 = ny + (D == 1);
  const int mz = DIM == 3 ? nz : 1;
  const size_t plc = (size_t)nx * ny, plu = (size_t)(nx + 1) * ny, plv = (size_t)nx * (ny + 1);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
  const int nb = gridDim.x, bl = blockIdx.x;
  const int t = (nb % 8 == 0) ? (bl % 8) * (nb / 8) + bl / 8 : bl;
  const int tile_x = t % ntx, rr = t / ntx, tile_y = rr % nty, tile_z = rr / nty;
  const int i0 = tile_x * TX, j0 = tile_y * TY;
  const int i = i0 + tx, j = j0 + ty;
  const int k0 = tile_z * kz, k1 = min(k0 + kz, mz);
  const bool act = i < fn0 && j < fn1;
  const bool cval = i < fn0 + H && j < fn1 + H && !(i >= fn0 && j >= fn1);
  const R eps = R(P.weno_eps * (12.0 / 13.0)), ih = R(P.ih), dt = R(P.dt);  // eps_w of weno5r
  // x-direction flux items: per row the 64 faces' low sides and the last
  // face's high side (65 positions, 520 per tile); every thread takes one,
  // threads 64..71 one more
  const int nxi = (tid >= 64 && tid < 72) ? 2 : 1;
  int xr[2], xm[2];
  bool xon[2];
#pragma unroll
  for (int qq = 0; qq < 2; ++qq) {
    const int wi = qq == 0 ? tid : 512 + (tid - 64);
    xr[qq] = wi / (TX + 1);
    xm[qq] = wi % (TX + 1);
    const int px = i0 + xm[qq], py = j0 + xr[qq];
    xon[qq] = qq < nxi && xr[qq] < TY && py < fn1 && px <= nx && (D != 0 || px >= 1);
  }
  // offsets of the first items are kept; those of the second items (72
  // threads) are recomputed where they are used
  const SiteXY xs0 = site_xy<D, 0>(i0 + xm[0], j0 + xr[0], nx, ny);
  // y-direction flux items: 9 rows of 64; threads 0..63 also take row 8
  const int nyi = tid < 64 ? 2 : 1;
  int yr[2];
  bool yon[2];
#pragma unroll
  for (int qq = 0; qq < 2; ++qq) {
    yr[qq] = qq == 0 ? ty : TY;
    const int px = i, py = j0 + yr[qq];
    yon[qq] = qq < nyi && px < fn0 && py <= ny && (D != 1 || py >= 1);
  }
  const SiteXY ys0 = site_xy<D, 1>(i, j0 + yr[0], nx, ny);
  // own face: in-plane offsets of its cells L and R (also the columns of w
  // on the z-edges)
  const unsigned oL = (unsigned)(clampi(i - (D == 0), nx) + nx * clampi(j - (D == 1), ny));
  const unsigned oR = (unsigned)(clampi(i, nx) + nx * clampi(j, ny));
  // MAT: in-plane offset and plane stride of this thread's D-face (clamped)
  const size_t ffo = (size_t)clampi(i, fn0) + (size_t)fn0 * clampi(j, fn1), ffp = (size_t)fn0 * fn1;
  int hox = 0, hoy = 0;
  const bool hrole = tid < NHALO;
  if (hrole) halo_pos(tid, hox, hoy);
  const int hi = i0 + hox - H, hj = j0 + hoy - H;
  const bool hvalid = hrole && hi >= -H && hi < fn0 + H && hj >= -H && hj < fn1 + H &&
                      (hi >= 0 && hi < fn0 ? true : (hj >= 0 && hj < fn1)) &&
                      (hj >= 0 && hj < fn1 ? true : (hi >= 0 && hi < fn0));
  // u_D with its ghost rules: odd reflection about the walls (normal: about
  // the wall face, tangential: about the wall); the in-plane part is fixed
  // per thread, the plane part is uniform
  const size_t plD = (size_t)fn0 * fn1;
  auto refl = [](int id, int n, bool normal, R& sg) {
    if (id < 0) {
      id = normal ? -id : -1 - id;
      sg = -sg;
    } else if (id > n - (normal ? 0 : 1)) {
      id = normal ? 2 * n - id : 2 * n - 1 - id;
      sg = -sg;
    }
    return id;
  };
  auto inplane = [&](int ii, int jj, R& sg) {
    sg = R(1);
    const int ri = refl(ii, nx, D == 0, sg), rj = refl(jj, ny, D == 1, sg);
    return (unsigned)(ri + fn0 * rj);
  };
  R qsg, hsg;
  const unsigned qoff = inplane(i, j, qsg);
  const unsigned hoff = inplane(hi, hj, hsg);
  // raw load of plane kk and the sign of its z ghost rule (applied at use)
  auto ldU = [&](unsigned off, int kk) {
    R sz = R(1);
    const R* pl = DIM == 2 ? ud : ud + (size_t)refl(kk, nz, D == 2, sz) * plD;
    return pl[off];
  };
  auto zsg = [&](int kk) {
    R sz = R(1);
    if (DIM == 3) refl(kk, nz, D == 2, sz);
    return sz;
  };
  // cell plane kk with the 1-deep even ghost along z
  auto cpl = [&](const R* f, int kk) { return f + (size_t)min(max(kk, 0), nz - 1) * plc; };
  // Operand loads of plane kk: flux item qq (first or second) and the face.
  // The first items (one plane ahead) and the face are loaded
  // unconditionally (every offset is a valid cell), so the count of loads in
  // flight is path independent and the waits for one plane's operands do
  // not drain the next plane's; the second items (72 threads) are issued
  // first.
  auto load_items = [&](int kk, int qq, FluxOps<R>& xn, FluxOps<R>& yn) {
    const int kL = kk - (D == 2);
    const R* aL = cpl(a, kL);
    const R* aR = cpl(a, kk);
    const R* uL = A.u + (size_t)min(max(kL, 0), nz - 1) * plu;
    const R* uR = A.u + (size_t)min(kk, nz - 1) * plu;
    const R* vL = A.v + (size_t)min(max(kL, 0), nz - 1) * plv;
    const R* vR = A.v + (size_t)min(kk, nz - 1) * plv;
    if (qq == 0) {
      load_ops<R, D, 0>(xn, xs0, aL, aR, uL, uR);
      load_ops<R, D, 1>(yn, ys0, aL, aR, vL, vR);
    } else {
      if (xon[1]) load_ops<R, D, 0>(xn, site_xy<D, 0>(i0 + xm[1], j0 + xr[1], nx, ny), aL, aR, uL, uR);
      if (yon[1]) load_ops<R, D, 1>(yn, site_xy<D, 1>(i, j0 + TY, nx, ny), aL, aR, vL, vR);
    }
  };
  auto load_face = [&](int kk, FaceOps<R>& fn) {
    const int kL = kk - (D == 2);
    const R* aR = cpl(a, kk);
    if (DIM == 3 && D != 2) {
      const R* wk = A.w + (size_t)min(kk + 1, nz) * plc;
      const R* ap = cpl(a, kk + 1);
      fn.wL = wk[oL];
      fn.wR = wk[oR];
      fn.apL = ap[oL];
      fn.apR = ap[oR];
    } else {
      fn.apR = aR[oR];
    }
    fn.skL = cpl(A.sk, kL)[oL];
    fn.skR = cpl(A.sk, kk)[oR];
    if (MAT) {
      fn.mL = A.ff[ffo + (size_t)kk * ffp];
    } else {
      fn.mL = cpl(A.M, kL)[oL];
      fn.mR = cpl(A.M, kk)[oR];
    }
  };
  FluxOps<R> xo{}, yo{};
  if (PF) load_items(k0, 0, xo, yo);
  // alpha of the cells L and R in plane k (D != z), or of the cell below
  // the face (D = z): carried from plane to plane
  R acL = R(0), acR = R(0);
  if (act) {
    if (D != 2) {
      acL = a[(size_t)k0 * plc + oL];
      acR = a[(size_t)k0 * plc + oR];
    } else {
      acL = cpl(a, k0 - 1)[oR];
    }
  }
  // u_D column queue (k-3 .. k+3); plane k+3 enters from qin, loaded one
  // plane earlier.  Threads outside the ghost band load a valid cell and do
  // not use it.
  const unsigned qo = cval ? qoff : 0u, ho = hvalid ? hoff : 0u;
  const int kq = k1 + 2;  // last plane the queue needs
  R q[7];
#pragma unroll
  for (int m = 0; m < 7; ++m) q[m] = R(0);
  R qin = R(0);
  if (DIM == 3) {
#pragma unroll
    for (int m = 0; m < 6; ++m) q[m + 1] = (qsg * zsg(k0 - 3 + m)) * ldU(qo, k0 - 3 + m);
    qin = ldU(qo, min(k0 + 3, kq));
  } else {
    q[3] = qsg * ldU(qo, 0);
  }
  R hu = ldU(ho, k0);  // halo of plane k (raw)
  R fz_lo = R(0), tz_lo = R(0);
  bool have_lo = false;
  int buf = 0;
  for (int k = k0; k < k1; ++k) {
    // second items of this plane first, then the next plane's operands
    // (PF) or this plane's
    // (the face operands are used after the second barrier: loaded for this
    // plane, after the second items and before the prefetches)
    FluxOps<R> xn{}, yn{}, x2{}, y2{};
    FaceOps<R> fo{};
    if (nxi > 1 || nyi > 1) load_items(k, 1, x2, y2);
    load_face(k, fo);
    if (PF)
      load_items(min(k + 1, k1 - 1), 0, xn, yn);
    else
      load_items(k, 0, xo, yo);
    if (DIM == 3) {
#pragma unroll
      for (int m = 0; m < 6; ++m) q[m] = q[m + 1];
      q[6] = (qsg * zsg(k + 3)) * qin;
      qin = ldU(qo, min(k + 4, kq));
    }
    // publish the plane, then load the next plane's halo
    if (cval) sU[buf][ty + H][tx + H] = q[3];
    if (hvalid) sU[buf][hoy][hox] = hsg * hu;
    hu = ldU(ho, min(k + 1, k1 - 1));
    __syncthreads();
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) {
      if (qq < nxi) {
        R F = R(0), T_ = R(0);
        if (qq == 0) {
          // every thread's first item is evaluated (its operands and LDS
          // row are always valid) and kept by a select: no exec-mask
          // updates around the evaluation
          const R* rw = &sU[buf][xr[0] + H][xm[0]];
          R Fv, Tv;
          flux_pair<R, D, 0>(P, xo, rw[0], rw[1], rw[2], rw[3], rw[4], rw[5], eps, Fv, Tv);
          F = xon[0] ? Fv : R(0);
          T_ = xon[0] ? Tv : R(0);
        } else if (xon[qq]) {
          const R* rw = &sU[buf][xr[qq] + H][xm[qq]];
          flux_pair<R, D, 0>(P, x2, rw[0], rw[1], rw[2], rw[3], rw[4], rw[5], eps, F, T_);
        }
        if (xr[qq] < TY) {
          fxF[xr[qq]][xm[qq]] = F;
          fxT[xr[qq]][xm[qq]] = T_;
        }
      }
    }
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) {
      if (qq < nyi) {
        R F = R(0), T_ = R(0);
        const int Y = yr[qq] + H, X = tx + H;
        if (qq == 0) {  // as for the x items
          R Fv, Tv;
          flux_pair<R, D, 1>(P, yo, sU[buf][Y - 3][X], sU[buf][Y - 2][X], sU[buf][Y - 1][X], sU[buf][Y][X],
                             sU[buf][Y + 1][X], sU[buf][Y + 2][X], eps, Fv, Tv);
          F = yon[0] ? Fv : R(0);
          T_ = yon[0] ? Tv : R(0);
        } else if (yon[qq]) {
          flux_pair<R, D, 1>(P, y2, sU[buf][Y - 3][X], sU[buf][Y - 2][X], sU[buf][Y - 1][X], sU[buf][Y][X],
                             sU[buf][Y + 1][X], sU[buf][Y + 2][X], eps, F, T_);
        }
        fyF[yr[qq]][tx] = F;
        fyT[yr[qq]][tx] = T_;
      }
    }
    __syncthreads();
    const bool interior = act && (D == 0 ? (i >= 1 && i < nx) : (D == 1 ? (j >= 1 && j < ny) : (k >= 1)));
    R conv = R(0), visc = R(0);
    // alpha of the cells L and R of this face
    const R alL = acL, alR = D == 2 ? fo.apR : acR;
    if (DIM == 3 && act) {
      // z: the high pair of this plane is the low pair of the next one
      if (D == 2) {
        if (!have_lo && k >= 1) {
          const R U = R(0.5) * (q[2] + q[3]);
          fz_lo = U * upw1(q[0], q[1], q[2], q[3], q[4], q[5], U, eps);
          tz_lo = R(2) * mixp(acL, P.mu1, P.mu2) * (q[3] - q[2]);
        }
        const R U = R(0.5) * (q[3] + q[4]);
        const R fzh = U * upw1(q[1], q[2], q[3], q[4], q[5], q[6], U, eps);
        const R tzh = R(2) * mixp(fo.apR, P.mu1, P.mu2) * (q[4] - q[3]);
        conv = fzh - fz_lo;
        visc = tzh - tz_lo;
        fz_lo = fzh;
        tz_lo = tzh;
      } else {
        if (!have_lo) {
          const R* wk = A.w + (size_t)k * plc;
          const R* am = cpl(a, k - 1);
          const R wL = wk[oL], wR = wk[oR];
          const R Vb = R(0.5) * (wL + wR);
          fz_lo = Vb * upw1(q[0], q[1], q[2], q[3], q[4], q[5], Vb, eps);
          const R me = R(0.25) * (mixp(am[oL], P.mu1, P.mu2) + mixp(am[oR], P.mu1, P.mu2) +
                                  mixp(acL, P.mu1, P.mu2) + mixp(acR, P.mu1, P.mu2));
          tz_lo = me * ((q[3] - q[2]) + (wR - wL));
        }
        const R Vb = R(0.5) * (fo.wL + fo.wR);
        const R fzh = Vb * upw1(q[1], q[2], q[3], q[4], q[5], q[6], Vb, eps);
        const R me = R(0.25) * (mixp(acL, P.mu1, P.mu2) + mixp(acR, P.mu1, P.mu2) + mixp(fo.apL, P.mu1, P.mu2) +
                                mixp(fo.apR, P.mu1, P.mu2));
        const R tzh = me * ((q[4] - q[3]) + (fo.wR - fo.wL));
        conv = fzh - fz_lo;
        visc = tzh - tz_lo;
        fz_lo = fzh;
        tz_lo = tzh;
      }
      have_lo = true;
    }
    if (interior) {
      conv += (fxF[ty][tx + 1] - fxF[ty][tx]) + (fyF[ty + 1][tx] - fyF[ty][tx]);
      visc += (fxT[ty][tx + 1] - fxT[ty][tx]) + (fyT[ty + 1][tx] - fyT[ty][tx]);
      const R fst = MAT ? fo.mL : R(0.5) * (fo.skL + fo.skR) * (alR - alL) * ih + R(0.5) * (fo.mL + fo.mR);
      const R rhof = MAT ? R(0.5) * (mixp(fo.skL, P.rho1, P.rho2) + mixp(fo.skR, P.rho1, P.rho2))
                         : R(0.5) * (mixp(alL, P.rho1, P.rho2) + mixp(alR, P.rho1, P.rho2));
      A.out[fidx<D>(i, j, k, nx, ny)] = q[3] + dt * (-conv * ih + (visc * ih * ih + fst) * rcpx(rhof));
    } else if (act) {
      A.out[fidx<D>(i, j, k, nx, ny)] = R(0);
    }
    // the wall face at the far end along D
    if (act) {
      if (D == 0 && i == nx - 1) A.out[fidx<0>(nx, j, k, nx, ny)] = R(0);
      if (D == 1 && j == ny - 1) A.out[fidx<1>(i, ny, k, nx, ny)] = R(0);
      if (D == 2 && k == nz - 1) A.out[fidx<2>(i, j, nz, nx, ny)] = R(0);
    }
    // carry alpha to the next plane and rotate the prefetched operands
    if (D != 2) {
      acL = fo.apL;
      acR = fo.apR;
    } else {
      acL = fo.apR;
    }
    if (PF) {
      xo = xn;
      yo = yn;
    }
    buf ^= 1;
  }
}

// FP32 runs two 512-thread blocks per CU (at most 128 VGPRs); FP64 one.
template <class R, int DIM, int D, bool MAT>
__global__ __launch_bounds__(512, 4) void k_pred2_f(PredArgs<R, DIM, D> A, int kz, int ntx, int nty) {
  pred_body<R, DIM, D, true, MAT>(A, kz, ntx, nty);
}
template <class R, int DIM, int D, bool MAT>
__global__ __launch_bounds__(512) void k_pred2_d(PredArgs<R, DIM, D> A, int kz, int ntx, int nty) {
  pred_body<R, DIM, D, false, MAT>(A, kz, ntx, nty);
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

template <class R, int DIM, int D, bool MAT>
void launch_pred(const KParams& P, hipStream_t s, const R* a, const R* sk, const R* M, const R* u, const R* v,
                 const R* w, R* out, const R* ff) {
  int kz, ntx, nty;
  const int nb = pred_plan(P.nx, P.ny, DIM == 3 ? P.nz : 1, &kz, &ntx, &nty);
  PredArgs<R, DIM, D> A{P, a, sk, M, u, v, w, out, ff};
  if (std::is_same<R, float>::value && TCF_PRED_PF)
    hipLaunchKernelGGL((k_pred2_f<R, DIM, D, MAT>), dim3(nb), dim3(TX, TY), 0, s, A, kz, ntx, nty);
  else
    hipLaunchKernelGGL((k_pred2_d<R, DIM, D, MAT>), dim3(nb), dim3(TX, TY), 0, s, A, kz, ntx, nty);
}

}  // namespace

template <class R>
void predictor(const KParams& P, hipStream_t s, const R* a, const R* sk, const R* Mx, const R* My, const R* Mz,
               const R* u, const R* v, const R* w, R* us, R* vs, R* ws) {
  if (P.dim == 3) {
    launch_pred<R, 3, 0, false>(P, s, a, sk, Mx, u, v, w, us, nullptr);
    launch_pred<R, 3, 1, false>(P, s, a, sk, My, u, v, w, vs, nullptr);
    launch_pred<R, 3, 2, false>(P, s, a, sk, Mz, u, v, w, ws, nullptr);
  } else {
    launch_pred<R, 2, 0, false>(P, s, a, sk, Mx, u, v, w, us, nullptr);
    launch_pred<R, 2, 1, false>(P, s, a, sk, My, u, v, w, vs, nullptr);
  }
}

template <class R>
void predictor_mat(const KParams& P, hipStream_t s, const R* amu, const R* arho, const R* fx, const R* fy,
                   const R* fz, const R* u, const R* v, const R* w, R* us, R* vs, R* ws) {
  if (P.dim == 3) {
    launch_pred<R, 3, 0, true>(P, s, amu, arho, nullptr, u, v, w, us, fx);
    launch_pred<R, 3, 1, true>(P, s, amu, arho, nullptr, u, v, w, vs, fy);
    launch_pred<R, 3, 2, true>(P, s, amu, arho, nullptr, u, v, w, ws, fz);
  } else {
    launch_pred<R, 2, 0, true>(P, s, amu, arho, nullptr, u, v, w, us, fx);
    launch_pred<R, 2, 1, true>(P, s, amu, arho, nullptr, u, v, w, vs, fy);
  }
}
template void predictor_mat<double>(const KParams&, hipStream_t, const double*, const double*, const double*,
                                    const double*, const double*, const double*, const double*, const double*,
                                    double*, double*, double*);
template void predictor_mat<float>(const KParams&, hipStream_t, const float*, const float*, const float*,
                                   const float*, const float*, const float*, const float*, const float*, float*,
                                   float*, float*);

template void predictor<double>(const KParams&, hipStream_t, const double*, const double*, const double*,
                                const double*, const double*, const double*, const double*, const double*, double*,
                                double*, double*);
template void predictor<float>(const KParams&, hipStream_t, const float*, const float*, const float*, const float*,
                               const float*, const float*, const float*, const float*, float*, float*, float*);

}  // namespace tcf
