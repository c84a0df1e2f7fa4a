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
// the next row through LDS.  The faces past the tile's high edges (the high
// x-face of each row, the high y-face of each column: 72 per plane and field)
// are computed one per lane by the first wavefronts and passed through LDS, so
// no wavefront issues a WENO5 evaluation for a single lane.  A WENO5
// evaluation takes one reciprocal (the weights over a common denominator),
// on the stencil picked by the velocity's sign.  The kernel also runs in two other modes (below):
// one passive cell field, or T alone with cell materials.
#include <algorithm>

#include <type_traits>

#include "tcf_device.h"
#include "tcf_internal.h"

namespace tcf {
namespace {

using namespace dev;

constexpr int TX = 64, TY = 8, H = 3;
constexpr int SX = TX + 2 * H, SY = TY + 2 * H;
constexpr int NHALO = 2 * H * TY + 2 * H * TX;  // x strips + y strips (corners unused)
constexpr int NE = TY + TX;                     // tile-edge faces of a plane: x (one per row), y (one per column)

// WENO5-JS.  With t_k the second differences and u_k the one-sided
// differences of the three candidate stencils (a..e = Q(f-2..f+2), upwind
// side first), the candidates' face values are c + (t_0 + 3 u_0)/12,
// c + (t_1 - 3 u_1)/12 and c + (t_2 - 3 u_2)/12, so the blend is c plus the
// weighted mean of those corrections and reuses the indicators' t_k and u_k.
// The smoothness indicators beta_k = (13/12) t_k^2 + (1/4) u_k^2 and epsilon
// are both taken times 12/13, which leaves the nonlinear weights
// d_k / (eps + beta_k)^2 unchanged after normalisation: x_k = eps' + t_k^2 +
// (3/13) u_k^2 with eps' = (12/13) eps (eps_w below), one multiply and two
// FMAs per indicator.  The weights are put over the common denominator
// (x_0 x_1 x_2)^2 and scaled by 10 (d = 1, 6, 3), so the evaluation takes one
// reciprocal, that of the normalisation (in FP32 after the power-of-two
// scaling of wscale, which keeps the products in range).
__device__ __forceinline__ float rcpx(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcpx(double x) { return 1.0 / x; }
// square root: the hardware instruction in FP32 (within an ulp), correctly
// rounded in FP64
__device__ __forceinline__ float sqrtx(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrtx(double x) { return sqrt(x); }

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

// SC: scale the smoothness terms (wscale); a field of order one (the
// two-phase volume fraction, whose terms stay below about 30) needs no
// scaling.
template <bool SC, class R>
__device__ __forceinline__ R weno5x(R a, R b, R c, R d, R e, R epsw) {
  const R t0 = a - R(2) * b + c, u0 = a - R(4) * b + R(3) * c;
  const R t1 = b - R(2) * c + d, u1 = b - d;
  const R t2 = c - R(2) * d + e, u2 = R(3) * c - R(4) * d + e;
  const R cu = R(3.0 / 13.0);
  const R x0 = fma(cu * u0, u0, fma(t0, t0, epsw));
  const R x1 = fma(cu * u1, u1, fma(t1, t1, epsw));
  const R x2 = fma(cu * u2, u2, fma(t2, t2, epsw));
  R y0 = x0, y1 = x1, y2 = x2;
  if (SC) wscale(y0, y1, y2);
  const R p12 = y1 * y2, p02 = y0 * y2, p01 = y0 * y1;
  const R a0 = p12 * p12, a1 = R(6) * p02 * p02, a2 = R(3) * p01 * p01;
  const R sc = fma(a2, fma(R(-3), u2, t2), fma(a1, fma(R(-3), u1, t1), a0 * fma(R(3), u0, t0)));
  return fma(sc, rcpx(R(12) * (a0 + a1 + a2)), c);
}

// q[m] = Q(f-3+m); value at face f, upwind by the sign of vel.  The stencil
// is picked before the one WENO5 evaluation, so lanes of both signs share it.
template <bool SC = true, class R>
__device__ __forceinline__ R upw(R q0, R q1, R q2, R q3, R q4, R q5, R vel, R eps) {
  const bool pos = vel >= R(0);
  return weno5x<SC>(pos ? q0 : q5, pos ? q1 : q4, pos ? q2 : q3, pos ? q3 : q2, pos ? q4 : q1, eps);
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

// Ghost map of a column (ii, jj): in-plane offset of its mirror cell (even
// reflection) and the affine map T = s raw + t of the Dirichlet walls it
// lies beyond (each such wall maps v to 2 T_w - v).
template <class R>
struct ColMap {
  unsigned off;
  R s, t;
};

template <class R>
__device__ __forceinline__ ColMap<R> col_map(const KParams& P, int ii, int jj, bool valid) {
  ColMap<R> m{0u, R(1), R(0)};
  if (!valid) return m;
  auto flip = [&](int side) {
    if (P.Tbc[side]) {
      m.s = -m.s;
      m.t = R(2) * R(P.Tw[side]) - m.t;
    }
  };
  int ri = ii, rj = jj;
  if (ii < 0) {
    ri = -1 - ii;
    flip(0);
  } else if (ii >= P.nx) {
    ri = 2 * P.nx - 1 - ii;
    flip(1);
  }
  if (jj < 0) {
    rj = -1 - jj;
    flip(2);
  } else if (jj >= P.ny) {
    rj = 2 * P.ny - 1 - jj;
    flip(3);
  }
  m.off = (unsigned)(ri + P.nx * rj);
  return m;
}

// MODE 1: alpha and T (the stage of S1).
// MODE 0: the "alpha" slot carries any passive cell field (the species, the
// fraction of a further phase) with exactly alpha's arithmetic; nothing of T
// is touched.
// MODE 2: T alone with cell materials: the "alpha" slot carries the
// conductivity lambda (read with its halo for the face means, not
// transported, ab and ao unused), rc the heat capacity rho c_p and dq the
// interface delta that the heat flux is spread over.
template <class R, int DIM, int MODE>
__global__ __launch_bounds__(512, sizeof(R) == 4 ? 4 : 1) void k_transport2(KParams P, int kz, int ntx, int nty, const R* __restrict__ a,
                                                    const R* __restrict__ T, const R* ab, const R* Tb,
                                                    const R* __restrict__ u, const R* __restrict__ v,
                                                    const R* __restrict__ w, R* ao, R* To, R cb, R ci,
                                                    const R* __restrict__ rc, const R* __restrict__ dq) {
  constexpr bool WT = MODE != 0, WA = MODE != 2;
  constexpr bool SCA = MODE != 1;  // the two-phase alpha's WENO5 terms need no scaling
  constexpr int NF = WT ? 2 : 1;                   // LDS fields: the alpha slot, T
  constexpr int NEF = (WA ? 1 : 0) + (WT ? 1 : 0);  // transported fields
  __shared__ R sq[NF][2][SY][SX];                  // [field][buffer][row][column]
  R(*sa)[SY][SX] = sq[0];
  R(*sT)[SY][SX] = sq[NF - 1];
  __shared__ R fya[TY][TX];  // low y-face fluxes of the tile rows
  __shared__ R fyt[WT ? TY : 1][WT ? TX : 1];
  __shared__ R sedge[2][NE];  // tile-edge face fluxes [alpha slot, T][x edges, then y edges]
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
  const R eps = R(P.weno_eps * (12.0 / 13.0)), ih = R(P.ih), dt = R(P.dt);  // eps_w of weno5x
  const size_t pl = (size_t)nx * ny, plu = (size_t)(nx + 1) * ny, plv = (size_t)nx * (ny + 1);
  // halo role of this thread
  int hox = 0, hoy = 0;
  const bool hrole = tid < NHALO;
  if (hrole) halo_pos(tid, hox, hoy);
  const int hi = i0 + hox - H, hj = j0 + hoy - H;
  const bool hvalid = hrole && hi >= -H && hi < nx + H && hj >= -H && hj < ny + H &&
                      (hi >= 0 && hi < nx ? true : (hj >= 0 && hj < ny)) && (hj >= 0 && hj < ny ? true : (hi >= 0 && hi < nx));
  // Every load below is issued unconditionally (positions a thread does not
  // need map to a valid cell, planes are clamped or reflected), so the count
  // of loads in flight is path independent and waiting for one plane's data
  // does not drain the prefetches of the next.  Loaded values are consumed
  // one plane after their load.
  const ColMap<R> cm = col_map<R>(P, i, j, cval);
  const ColMap<R> hm = col_map<R>(P, hi, hj, hvalid);
  auto zrefl = [&](int kk) { return DIM == 3 ? (kk < 0 ? -1 - kk : (kk >= nz ? 2 * nz - 1 - kk : kk)) : 0; };
  auto tval = [&](const ColMap<R>& m, R raw, int kk) {
    R v0 = m.s * raw + m.t;
    if (DIM == 3) {
      if (kk < 0 && P.Tbc[4]) v0 = R(2) * R(P.Tw[4]) - v0;
      if (kk >= nz && P.Tbc[5]) v0 = R(2) * R(P.Tw[5]) - v0;
    }
    return v0;
  };
  auto ldA = [&](unsigned off, int kk) { return a[off + (size_t)zrefl(kk) * pl]; };
  auto ldT = [&](unsigned off, int kk) { return T[off + (size_t)zrefl(kk) * pl]; };
  // in-plane offsets of the face velocities (low and high faces) and cells
  const int ic = min(i, nx - 1), jc = min(j, ny - 1);
  const unsigned uoL = (unsigned)(min(i, nx) + (nx + 1) * jc);
  const unsigned voL = (unsigned)(ic + nx * min(j, ny));
  const unsigned co = (unsigned)(ic + nx * jc);
  // column queues: planes k-3 .. k+4 of the pair of planes (k, k+1) the
  // loop computes per pass (plane k reads entries 0..6, plane k+1 entries
  // 1..7); in 2D only the centre (entry 3) is used
  R qa[8], qt[8];
  for (int m = 0; m < 8; ++m) {
    qa[m] = R(0);
    qt[m] = R(0);
  }
  const int kq = min(k1 + 2, nz + 2);  // last plane the queues need
  R ia0 = R(0), iT0 = R(0), ia1 = R(0), iT1 = R(0);  // planes k+5 and k+6 of the column, in flight
  if (DIM == 3) {
    for (int m = 0; m < 8; ++m) {
      const int kk = k0 - 3 + m, kl = min(kk, kq);
      qa[m] = ldA(cm.off, kl);
      if (WT) qt[m] = tval(cm, ldT(cm.off, kl), kk);
    }
  } else {
    qa[3] = ldA(cm.off, 0);
    if (WT) qt[3] = tval(cm, ldT(cm.off, 0), 0);
  }
  const bool wq = MODE == 2 && P.qP != 0.0;
  const R wL0 = DIM == 3 ? w[(size_t)k0 * pl + co] : R(0);
  // Tile-edge role: lane tid < NEF * NE computes field ef at edge face ee,
  // the high x-face of row ee (ee < TY) or the high y-face of column ee - TY.
  // Its 6-cell stencil starts at LDS offset est with stride 1 (x) or SX (y);
  // the face velocity offset is clamped so that every lane's load is valid.
  const bool erole = tid < NEF * NE;
  const int ee = tid % NE, ef = (WA && WT) ? min(tid / NE, 1) : (WA ? 0 : 1);
  const bool ex = ee < TY;
  const int est = ex ? (ee + H) * SX + TX : TY * SX + (ee - TY) + H, es = ex ? 1 : SX;
  const R* __restrict__ ev = ex ? u : v;
  const size_t epl = ex ? plu : plv;
  const unsigned eoff = ex ? (unsigned)(min(i0 + TX, nx) + (nx + 1) * min(j0 + ee, ny - 1))
                           : (unsigned)(min(i0 + ee - TY, nx - 1) + nx * min(j0 + TY, ny));
  R eV = ev[(size_t)k0 * epl + eoff];
  // Gaussian surface heat flux of the column (x, y, t), FP64, once per column
  R qcol = R(0);
  if (WT && P.qP != 0.0 && act) {
    const double xl = P.qx0 + P.qvx * P.t, yl = P.qy0 + P.qvy * P.t;
    const double x = (i + 0.5) * P.h, y = (j + 0.5) * P.h;
    const double r2 = (x - xl) * (x - xl) + (y - yl) * (y - yl);
    const double R2 = P.qr * P.qr;
    qcol = R(2.0 * P.qP / (M_PI * R2) * exp(-2.0 * r2 / R2));
  }
  // One plane's operands, loaded one plane ahead: the velocities of its
  // faces, the tile-edge face velocity, the base state, the halo (raw T).
  // Two sets take turns (the loop computes two planes per pass), so no
  // register is copied from plane to plane.
  struct Pre {
    R u, v, w, ev, ba, bT, rc, dq, ha, hT;
  };
  auto load_pre = [&](Pre& p, int kk) {
    p.u = u[(size_t)kk * plu + uoL];
    p.v = v[(size_t)kk * plv + voL];
    p.ev = ev[(size_t)kk * epl + eoff];
    p.w = DIM == 3 ? w[(size_t)min(kk + 1, nz) * pl + co] : R(0);
    p.ba = WA ? ab[(size_t)kk * pl + co] : R(0);
    p.bT = WT ? Tb[(size_t)kk * pl + co] : R(0);
    p.rc = MODE == 2 ? rc[(size_t)kk * pl + co] : R(0);
    p.dq = wq ? dq[(size_t)kk * pl + co] : R(0);
    p.ha = ldA(hm.off, kk);
    p.hT = WT ? ldT(hm.off, kk) : R(0);
  };
  R fza_lo = R(0), fzt_lo = R(0);  // low z-face flux carried between planes
  bool have_lo = false;
  // plane k from the queue entries o .. o + 6 and the LDS buffer o
  auto plane = [&](int k, auto oc, const Pre& cur, Pre& nxt) {
    constexpr int o = decltype(oc)::value, buf = o;
    // load plane k+5 of the column (it enters the queue after the pass)
    if (DIM == 3) {
      (o == 0 ? ia0 : ia1) = ldA(cm.off, min(k + 5, kq));
      if (WT) (o == 0 ? iT0 : iT1) = ldT(cm.off, min(k + 5, kq));
    }
    // publish the plane, then load the next plane's operands
    if (cval) {
      sa[buf][ty + H][tx + H] = qa[o + 3];
      if (WT) sT[buf][ty + H][tx + H] = qt[o + 3];
    }
    if (hvalid) {
      sa[buf][hoy][hox] = cur.ha;
      if (WT) sT[buf][hoy][hox] = tval(hm, cur.hT, k);
    }
    load_pre(nxt, min(k + 1, k1 - 1));
    __syncthreads();
    R Fxa_lo = R(0), Fxt_lo = R(0), Fya_lo = R(0), Fyt_lo = R(0);
    const size_t c = (size_t)k * pl + co;
    if (act) {
      const int X = tx + H, Y = ty + H;
      // the low x- and y-face fluxes are evaluated on every active cell (the
      // tile holds the ghost values there) and the wall faces are dropped by
      // selects, without exec-mask updates around the evaluations
      if (WA) {
        const R fx = cur.u * upw<SCA>(sa[buf][Y][X - 3], sa[buf][Y][X - 2], sa[buf][Y][X - 1], sa[buf][Y][X],
                                 sa[buf][Y][X + 1], sa[buf][Y][X + 2], cur.u, eps);
        const R fy = cur.v * upw<SCA>(sa[buf][Y - 3][X], sa[buf][Y - 2][X], sa[buf][Y - 1][X], sa[buf][Y][X],
                                 sa[buf][Y + 1][X], sa[buf][Y + 2][X], cur.v, eps);
        Fxa_lo = i > 0 ? fx : R(0);
        Fya_lo = j > 0 ? fy : R(0);
      }
      if (WT) {
        const R fx = cur.u * upw(sT[buf][Y][X - 3], sT[buf][Y][X - 2], sT[buf][Y][X - 1], sT[buf][Y][X],
                                 sT[buf][Y][X + 1], sT[buf][Y][X + 2], cur.u, eps);
        const R fy = cur.v * upw(sT[buf][Y - 3][X], sT[buf][Y - 2][X], sT[buf][Y - 1][X], sT[buf][Y][X],
                                 sT[buf][Y + 1][X], sT[buf][Y + 2][X], cur.v, eps);
        Fxt_lo = i > 0 ? fx : R(0);
        Fyt_lo = j > 0 ? fy : R(0);
      }
      if (WA) fya[ty][tx] = Fya_lo;
      if (WT) fyt[ty][tx] = Fyt_lo;
    }
    // tile-edge faces (their values are read only where the face is inside
    // the domain; elsewhere the stencil holds stale LDS and is unused)
    if (erole) {
      const R* sb = &sq[ef][buf][0][0] + est;
      sedge[ef][ee] = cur.ev * upw(sb[0], sb[es], sb[2 * es], sb[3 * es], sb[4 * es], sb[5 * es], cur.ev, eps);
    }
    // high x-face: next lane's low face
    R Fxa_hi = __shfl_down(Fxa_lo, 1, 64), Fxt_hi = WT ? __shfl_down(Fxt_lo, 1, 64) : R(0);
    __syncthreads();
    if (act) {
      const int X = tx + H, Y = ty + H;
      if (i + 1 >= nx) {
        Fxa_hi = R(0);
        Fxt_hi = R(0);
      } else if (tx == TX - 1) {
        if (WA) Fxa_hi = sedge[0][ty];
        if (WT) Fxt_hi = sedge[1][ty];
      }
      R Fya_hi = R(0), Fyt_hi = R(0);
      if (j + 1 < ny) {
        if (ty < TY - 1) {
          if (WA) Fya_hi = fya[ty + 1][tx];
          if (WT) Fyt_hi = fyt[ty + 1][tx];
        } else {
          if (WA) Fya_hi = sedge[0][TY + tx];
          if (WT) Fyt_hi = sedge[1][TY + tx];
        }
      }
      R diva = (Fxa_hi - Fxa_lo) + (Fya_hi - Fya_lo);
      R divt = (Fxt_hi - Fxt_lo) + (Fyt_hi - Fyt_lo);
      if (DIM == 3) {
        if (!have_lo) {
          fza_lo = R(0);
          fzt_lo = R(0);
          if (k > 0) {
            if (WA)
              fza_lo = wL0 * upw<SCA>(qa[o + 0], qa[o + 1], qa[o + 2], qa[o + 3], qa[o + 4], qa[o + 5], wL0, eps);
            if (WT)
              fzt_lo = wL0 * upw(qt[o + 0], qt[o + 1], qt[o + 2], qt[o + 3], qt[o + 4], qt[o + 5], wL0, eps);
          }
        }
        R fza_hi = R(0), fzt_hi = R(0);
        if (k + 1 < nz) {
          if (WA)
            fza_hi = cur.w * upw<SCA>(qa[o + 1], qa[o + 2], qa[o + 3], qa[o + 4], qa[o + 5], qa[o + 6], cur.w, eps);
          if (WT)
            fzt_hi = cur.w * upw(qt[o + 1], qt[o + 2], qt[o + 3], qt[o + 4], qt[o + 5], qt[o + 6], cur.w, eps);
        }
        diva += fza_hi - fza_lo;
        divt += fzt_hi - fzt_lo;
        fza_lo = fza_hi;
        fzt_lo = fzt_hi;
        have_lo = true;
      }
      const R ac = qa[o + 3], Tc = qt[o + 3];
      const R La = -diva * ih;
      if (WA) ao[c] = cb * cur.ba + ci * (ac + dt * La);
      if (WT) {
        // conduction: arithmetic-mean face conductivity, ghosts from the tile
        auto lam = [&](R x) { return MODE == 2 ? x : mixp(x, P.lam1, P.lam2); };
        const R lc = lam(ac);
        R cond = R(0);
        {
          const R an[4] = {sa[buf][Y][X - 1], sa[buf][Y][X + 1], sa[buf][Y - 1][X], sa[buf][Y + 1][X]};
          const R tn[4] = {sT[buf][Y][X - 1], sT[buf][Y][X + 1], sT[buf][Y - 1][X], sT[buf][Y + 1][X]};
          for (int f = 0; f < 4; ++f) cond += R(0.5) * (lc + lam(an[f])) * (tn[f] - Tc);
          if (DIM == 3) {
            cond += R(0.5) * (lc + lam(qa[o + 2])) * (qt[o + 2] - Tc);
            cond += R(0.5) * (lc + lam(qa[o + 4])) * (qt[o + 4] - Tc);
          }
        }
        cond *= ih * ih;
        R src = R(0);
        if (MODE == 2) {
          src = qcol * cur.dq;
        } else if (P.qP != 0.0) {
          const R h2 = R(0.5) * ih;
          const R gx = (sa[buf][Y][X + 1] - sa[buf][Y][X - 1]) * h2;
          const R gy = (sa[buf][Y + 1][X] - sa[buf][Y - 1][X]) * h2;
          const R gz = DIM == 3 ? (qa[o + 4] - qa[o + 2]) * h2 : R(0);
          const R g2 = gx * gx + gy * gy + gz * gz;
          if (g2 != R(0)) {  // delta_s vanishes off the interface (skipped by whole wavefronts there)
            const R ne = R(P.neps);
            src = qcol * (g2 * rcpx(sqrtx(g2 + ne * ne) + ne));
          }
        }
        const R LT = -divt * ih + (cond + src) * rcpx(MODE == 2 ? cur.rc : mixp(ac, P.rhocp1, P.rhocp2));
        To[c] = cb * cur.bT + ci * (Tc + dt * LT);
      }
    }
  };
  Pre pa, pb;
  load_pre(pa, k0);
  int k = k0;
  for (; k + 1 < k1; k += 2) {
    plane(k, std::integral_constant<int, 0>(), pa, pb);
    plane(k + 1, std::integral_constant<int, 1>(), pb, pa);
    // the queues move on by two planes
    if (DIM == 3) {
      for (int m = 0; m < 6; ++m) {
        qa[m] = qa[m + 2];
        qt[m] = qt[m + 2];
      }
      qa[6] = ia0;
      qa[7] = ia1;
      if (WT) {
        qt[6] = tval(cm, iT0, k + 5);
        qt[7] = tval(cm, iT1, k + 6);
      }
    }
  }
  if (k < k1) plane(k, std::integral_constant<int, 0>(), pa, pb);
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
    hipLaunchKernelGGL((k_transport2<R, 3, 1>), dim3(nb), dim3(TX, TY), 0, s, P, kz, ntx, nty, a, T, ab, Tb, u, v, w,
                       ao, To, R(cb), R(ci), nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_transport2<R, 2, 1>), dim3(nb), dim3(TX, TY), 0, s, P, kz, ntx, nty, a, T, ab, Tb, u, v, w,
                       ao, To, R(cb), R(ci), nullptr, nullptr);
}

template <class R>
void transport_temperature(const KParams& P, hipStream_t s, const R* lam, const R* rcp, const R* dq, const R* T,
                           const R* Tb, const R* u, const R* v, const R* w, R* To, double cb, double ci) {
  int kz, ntx, nty;
  const int nb = transport_plan(P.nx, P.ny, P.nz, &kz, &ntx, &nty);
  if (P.dim == 3)
    hipLaunchKernelGGL((k_transport2<R, 3, 2>), dim3(nb), dim3(TX, TY), 0, s, P, kz, ntx, nty, lam, T, nullptr, Tb, u,
                       v, w, nullptr, To, R(cb), R(ci), rcp, dq);
  else
    hipLaunchKernelGGL((k_transport2<R, 2, 2>), dim3(nb), dim3(TX, TY), 0, s, P, kz, ntx, nty, lam, T, nullptr, Tb, u,
                       v, w, nullptr, To, R(cb), R(ci), rcp, dq);
}

template <class R>
void transport_scalar(const KParams& P, hipStream_t s, const R* q, const R* qb, const R* u, const R* v, const R* w,
                      R* qo, double cb, double ci) {
  int kz, ntx, nty;
  const int nb = transport_plan(P.nx, P.ny, P.nz, &kz, &ntx, &nty);
  if (P.dim == 3)
    hipLaunchKernelGGL((k_transport2<R, 3, 0>), dim3(nb), dim3(TX, TY), 0, s, P, kz, ntx, nty, q, nullptr, qb, nullptr,
                       u, v, w, qo, nullptr, R(cb), R(ci), nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_transport2<R, 2, 0>), dim3(nb), dim3(TX, TY), 0, s, P, kz, ntx, nty, q, nullptr, qb, nullptr,
                       u, v, w, qo, nullptr, R(cb), R(ci), nullptr, nullptr);
}

template void transport_stage<double>(const KParams&, hipStream_t, const double*, const double*, const double*,
                                      const double*, const double*, const double*, const double*, double*, double*,
                                      double, double);
template void transport_stage<float>(const KParams&, hipStream_t, const float*, const float*, const float*,
                                     const float*, const float*, const float*, const float*, float*, float*, double,
                                     double);
template void transport_scalar<double>(const KParams&, hipStream_t, const double*, const double*, const double*,
                                       const double*, const double*, double*, double, double);
template void transport_scalar<float>(const KParams&, hipStream_t, const float*, const float*, const float*,
                                      const float*, const float*, float*, double, double);
template void transport_temperature<double>(const KParams&, hipStream_t, const double*, const double*, const double*,
                                            const double*, const double*, const double*, const double*, const double*,
                                            double*, double, double);
template void transport_temperature<float>(const KParams&, hipStream_t, const float*, const float*, const float*,
                                           const float*, const float*, const float*, const float*, const float*,
                                           float*, double, double);

}  // namespace tcf
