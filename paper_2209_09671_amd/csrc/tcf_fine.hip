// Finest-level kernels of the pressure solver (PCG + multigrid on level 0).
//
// On the finest grid the face weights of K = -A are not stored: each kernel
// recomputes a_f = 2 / (h^2 (rho_L + rho_R)) from the volume fraction it
// already streams (one value per cell instead of one per face and axis).
// Each block owns a 64 x 8 column tile and marches along z over a chunk of
// planes, carrying the z-neighbours of the streamed arrays in registers; the
// in-plane neighbours come from the same block's loads (L1) or the adjacent
// tile's (L2).  Tiles are numbered so that the blocks one XCD receives (the
// dispatcher deals blocks round-robin over the 8 XCDs) form a contiguous
// slab, which keeps the y-halo rows in that XCD's L2.  The CG vector updates
// are fused into the stencil passes: d <- z + beta d into the SpMV, and
// x += alpha d, r -= alpha q plus the first Jacobi sweep into one pass.
// The FP64 residual of the refinement marches the same way with FP64
// densities, weights and pressure.
#include <algorithm>
#include <type_traits>

#include "tcf_device.h"
#include "tcf_internal.h"

namespace tcf {
namespace {

using namespace dev;

#ifndef TCF_FINE_FY
#define TCF_FINE_FY 8
#endif
#ifndef TCF_FINE_BLOCKS
#define TCF_FINE_BLOCKS 1024
#endif
constexpr int FX = 64, FY = TCF_FINE_FY;

template <class R>
struct Op0 {
  const R* a;    // volume fraction
  int nx, ny, nz;
  double rho1, drho, c2;  // rho = rho1 + clamp(alpha) drho; a_f = c2 / (rho_L + rho_R), c2 = 2/h^2
};

template <class R>
__device__ __forceinline__ R rho0(const Op0<R>& op, R a) {
  a = a < R(0) ? R(0) : (a > R(1) ? R(1) : a);
  return R(op.rho1) + a * R(op.drho);
}
template <>
__device__ __forceinline__ float rho0<float>(const Op0<float>& op, float a) {
  return float(op.rho1) + __builtin_amdgcn_fmed3f(a, 0.0f, 1.0f) * float(op.drho);
}
__device__ __forceinline__ double coef(double c2, double s) { return c2 / s; }
__device__ __forceinline__ float coef(float c2, float s) { return c2 * __builtin_amdgcn_rcpf(s); }
__device__ __forceinline__ double recip(double s) { return 1.0 / s; }
__device__ __forceinline__ float recip(float s) { return __builtin_amdgcn_rcpf(s); }

// The FP64 operator on a volume fraction of type A (the refinement
// residual): densities and face weights a_f = c2 / (rho_L + rho_R) in FP64,
// with c2 = 2/h^2 formed as 2 (1/h)^2.
template <class A>
struct Op64 {
  const A* a;
  int nx, ny, nz;
  double rho1, drho, c2;
};

template <class A>
__device__ __forceinline__ double rho0(const Op64<A>& op, A a) {
  double x = (double)a;
  x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
  return op.rho1 + x * op.drho;
}

// FP64 reciprocal: hardware estimate refined by three Newton steps (each
// doubles the correct bits; the result is within an ulp or two of 1/x, all
// that the FP64 residual needs: the projection's own 1/rho_f agrees with it
// to rounding).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

struct Tile {
  int i, j, k0, k1;
  bool act;
};

// XCD-grouped tile numbering: block b runs on XCD b % 8; give that XCD the
// contiguous tile range [x * nb/8, (x+1) * nb/8).
__device__ __forceinline__ Tile tile_of(int nx, int ny, int nz, int ntx, int nty, int kz) {
  const int nb = gridDim.x, b = blockIdx.x;
  const int t = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int tx = t % ntx, rr = t / ntx;
  const int ty = rr % nty, tz = rr / nty;
  Tile T;
  T.i = tx * FX + threadIdx.x;
  T.j = ty * FY + threadIdx.y;
  T.k0 = tz * kz;
  T.k1 = min(T.k0 + kz, nz);
  T.act = T.i < nx && T.j < ny && T.k0 < nz;
  return T;
}

constexpr int LX = FX + 2, LY = FY + 2;

// face weight between cells with densities rc and rn
template <class R>
__device__ __forceinline__ R wface(const Op0<R>& op, R rc, R rn) {
  return coef(R(op.c2), rc + rn);
}
template <class A>
__device__ __forceinline__ double wface(const Op64<A>& op, double rc, double rn) {
  return op.c2 * rcp64(rc + rn);
}

// Plane march over a z-chunk with one streamed field x and the volume
// fraction.  Per plane: the tile and its one-cell halo go to a
// double-buffered LDS plane (one barrier per plane), the z-neighbours stay
// in registers.  Loads run three planes ahead (per-cell operands pre(c) two
// planes ahead) and are issued unconditionally, with the plane index clamped
// to the chunk (a clamped load re-reads a cached plane and is not used), so
// the number of loads in flight is the same on every path and the waits for
// a plane's data do not drain the later prefetches.  The planes rotate
// through five register slots by renaming (the loop is unrolled by five), so
// no value is copied while its load is in flight; raw loads (xld) are
// combined (xval) and alpha becomes a density only when the plane is used.
// The weight of the face to the next plane is carried to it.  For each
// active cell body(c, k, xc, Kx, dg, pv) receives K0 x, the diagonal and
// pv = pre(c).  With POST, all threads then pass a second barrier and
// post(k) runs (the restriction).
template <class R, class AR, class XR, class PV>
struct Slot {
  XR xr, hyr, hxr;   // raw loads of x: centre and halo
  AR a, gy, gx;      // alpha (as stored): centre and halo
  PV pv;             // per-cell operands
  R xv, rho;         // x and density of the centre, once the plane is next
};

template <class R, int DIM, bool HASX, bool POST, class OP, class XLD, class XVAL, class PRE, class BODY, class PST>
__device__ __forceinline__ void march(const OP& op, const Tile& T, const XLD& xld, const XVAL& xval,
                                      const PRE& pre, const BODY& body, const PST& post) {
  __shared__ R sx[2][LY][LX];
  __shared__ R sa[2][LY][LX];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int nx = op.nx, ny = op.ny, nz = op.nz;
  const long pl = (long)nx * ny;
  const int yr = (ty == 0) ? -1 : (ty == FY - 1 ? 1 : 0);
  const int xr = (tx == 0) ? -1 : (tx == FX - 1 ? 1 : 0);
  const bool hasy = T.act && yr != 0 && T.j + yr >= 0 && T.j + yr < ny;
  const bool hasx = T.act && xr != 0 && T.i + xr >= 0 && T.i + xr < nx;
  const long col = T.act ? (long)T.i + (long)nx * T.j : 0;
  const long oyc = hasy ? (long)yr * nx : 0, oxc = hasx ? xr : 0;  // halo offset, own cell if none
  const int hyj = hasy ? T.j + yr : T.j, hxi = hasx ? T.i + xr : T.i;
  using XR = decltype(xld(0L, 0, 0, 0));
  using PV = decltype(pre(0L));
  using AR = std::remove_cv_t<std::remove_reference_t<decltype(op.a[0])>>;
  using S = Slot<R, AR, XR, PV>;
  // last plane whose centre is read (the z-neighbour of the chunk's last
  // plane), last plane of the chunk
  const int kc = DIM == 3 ? min(T.k1, nz - 1) : 0;
  const int kh = max(T.k1 - 1, T.k0);
  auto load_centre = [&](int k, S& s) {
    const int kk = min(max(k, 0), kc);
    const long c = col + pl * kk;
    if (HASX) s.xr = xld(c, T.i, T.j, kk);
    s.a = op.a[c];
  };
  auto load_halo = [&](int k, S& s) {
    const int kk = min(k, kh);
    const long c = col + pl * kk;
    if (HASX) {
      s.hyr = xld(c + oyc, T.i, hyj, kk);
      s.hxr = xld(c + oxc, hxi, T.j, kk);
    }
    s.gy = op.a[c + oyc];
    s.gx = op.a[c + oxc];
  };
  auto load_pv = [&](int k, S& s) { s.pv = pre(col + pl * min(k, kh)); };
  auto finish = [&](S& s) {  // the plane is about to be used
    if (HASX) s.xv = xval(s.xr);
    s.rho = rho0(op, s.a);
  };
  S A{}, B{}, C{}, D{}, E{};  // planes k0-1, k0, k0+1, k0+2; E receives k0+3
  if (DIM == 3) load_centre(T.k0 - 1, A);
  load_centre(T.k0, B);
  load_halo(T.k0, B);
  load_pv(T.k0, B);
  if (DIM == 3) {
    load_centre(T.k0 + 1, C);
    load_halo(T.k0 + 1, C);
    load_pv(T.k0 + 1, C);
    load_centre(T.k0 + 2, D);
    load_halo(T.k0 + 2, D);
  }
  if (DIM == 3) finish(A);
  finish(B);
  R wz = R(0);  // weight of the face between planes k-1 and k
  if (DIM == 3 && T.act && T.k0 > 0) wz = wface(op, B.rho, A.rho);
  // one plane; M = k-1, Cc = k, P1 = k+1, P2 = k+2, P3 receives k+3
  auto step = [&](int k, S& M, S& Cc, S& P1, S& P2, S& P3) {
    if (DIM == 3) {
      load_centre(k + 3, P3);
      load_halo(k + 3, P3);
      load_pv(k + 2, P2);
      finish(P1);
    }
    const int buf = k & 1;
    const R rc = Cc.rho;
    if (T.act) {
      if (HASX) sx[buf][ty + 1][tx + 1] = Cc.xv;
      sa[buf][ty + 1][tx + 1] = rc;
      if (hasy) {
        if (HASX) sx[buf][ty + 1 + yr][tx + 1] = xval(Cc.hyr);
        sa[buf][ty + 1 + yr][tx + 1] = rho0(op, Cc.gy);
      }
      if (hasx) {
        if (HASX) sx[buf][ty + 1][tx + 1 + xr] = xval(Cc.hxr);
        sa[buf][ty + 1][tx + 1 + xr] = rho0(op, Cc.gx);
      }
    }
    __syncthreads();
    if (T.act) {
      const long c = col + pl * k;
      R s = R(0), d = R(0);
      if (T.i > 0) {
        const R w = wface(op, rc, sa[buf][ty + 1][tx]);
        if (HASX) s += w * (Cc.xv - sx[buf][ty + 1][tx]);
        d += w;
      }
      if (T.i < nx - 1) {
        const R w = wface(op, rc, sa[buf][ty + 1][tx + 2]);
        if (HASX) s += w * (Cc.xv - sx[buf][ty + 1][tx + 2]);
        d += w;
      }
      if (T.j > 0) {
        const R w = wface(op, rc, sa[buf][ty][tx + 1]);
        if (HASX) s += w * (Cc.xv - sx[buf][ty][tx + 1]);
        d += w;
      }
      if (T.j < ny - 1) {
        const R w = wface(op, rc, sa[buf][ty + 2][tx + 1]);
        if (HASX) s += w * (Cc.xv - sx[buf][ty + 2][tx + 1]);
        d += w;
      }
      if (DIM == 3) {
        if (k > 0) {
          if (HASX) s += wz * (Cc.xv - M.xv);
          d += wz;
        }
        wz = R(0);
        if (k < nz - 1) {
          wz = wface(op, rc, P1.rho);
          if (HASX) s += wz * (Cc.xv - P1.xv);
          d += wz;
        }
      }
      body(c, k, Cc.xv, s, d, Cc.pv);
    }
    if (POST) {
      __syncthreads();
      post(k);
    }
  };
  int k = T.k0;
  for (; k + 5 <= T.k1; k += 5) {
    step(k, A, B, C, D, E);
    step(k + 1, B, C, D, E, A);
    step(k + 2, C, D, E, A, B);
    step(k + 3, D, E, A, B, C);
    step(k + 4, E, A, B, C, D);
  }
  const int rem = T.k1 - k;
  if (rem > 0) step(k, A, B, C, D, E);
  if (rem > 1) step(k + 1, B, C, D, E, A);
  if (rem > 2) step(k + 2, C, D, E, A, B);
  if (rem > 3) step(k + 3, D, E, A, B, C);
}

struct Empty {};
template <class R>
struct Vec2 {
  R a, b;
};
template <class R>
struct Vec4 {
  R a, b, c, d;
};
template <class R>
struct Ident {
  __device__ R operator()(R v) const { return v; }
};

struct NoPost {
  __device__ void operator()(int) const {}
};

__device__ __forceinline__ void write_partial(double acc, double* part) {
  __shared__ double sh[16];
  const double s = block_reduce<0>(acc, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = s;
}

// Sum of the n per-block partials of the previous pass, computed by every
// block of a consumer kernel instead of by a reduction launch of its own:
// 256 fixed lanes (the block's first 256 threads) each add a strided subset
// with four accumulators, and block_reduce sums the lanes in a fixed order
// (the other threads add exact zeros), so every block of any size >= 256
// gets the same value, bit for bit.
__device__ __forceinline__ double fold_partials(const double* __restrict__ part, int n) {
  __shared__ double sh[16];
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (tid < 256) {
    int q = tid;
    for (; q + 768 < n; q += 1024) {
      a0 += part[q];
      a1 += part[q + 256];
      a2 += part[q + 512];
      a3 += part[q + 768];
    }
    for (; q < n; q += 256) a0 += part[q];
  }
  return block_reduce<0>((a0 + a1) + (a2 + a3), sh);
}

// PCG iteration it (1-based), first pass.  rz_(it-1) = r.z of the last
// preconditioner application is folded from its partials (rzp, nrz) and
// stored in rz_slot(it - 1) by block 0; beta = rz_(it-1) / rz_(it-2).
// d' = z + beta d (d' = z on the first iteration); partial d'.K0 d' (K0 d'
// itself is not stored: the update pass recomputes it from d')
template <class R, int DIM>
__global__ __launch_bounds__(FX * FY) void k0_spmv_upd(Op0<R> op, int kz, int ntx, int nty, const R* __restrict__ z,
                                                   const R* __restrict__ dold, R* __restrict__ dnew,
                                                   double* __restrict__ scal, int it,
                                                   const double* __restrict__ rzp, int nrz,
                                                   double* __restrict__ part, const int* __restrict__ iflag) {
  if (iflag[I_DONE]) return;
  const Tile T = tile_of(op.nx, op.ny, op.nz, ntx, nty, kz);
  const bool first = it == 1;
  const double rz = fold_partials(rzp, nrz);
  const double bd = first ? 0.0 : rz / scal[rz_slot(it - 2)];
  if (blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
    scal[rz_slot(it - 1)] = rz;
    scal[S_BETA] = bd;
  }
  // on the first iteration d' = z + 0 z (the old direction is not read)
  const R beta = R(bd);
  const R* __restrict__ dsrc = first ? z : dold;
  auto X = [&](long c, int, int, int) { return Vec2<R>{z[c], dsrc[c]}; };
  auto XV = [&](const Vec2<R>& v) { return v.a + beta * v.b; };
  double acc = 0.0;
  auto pre = [&](long) { return Empty{}; };
  auto body = [&](long c, int, R xc, R Kx, R, const Empty&) {
    dnew[c] = xc;
    acc += (double)xc * (double)Kx;
  };
  march<R, DIM, true, false>(op, T, X, XV, pre, body, NoPost());
  write_partial(acc, part);
}

// x += alpha d; r -= alpha K0 d (K0 d recomputed from the streamed d, the
// same arithmetic as the SpMV pass; partial r.r); z1 = omega r / diag (first
// sweep of the next V-cycle from a zero guess).  With xzero, x starts from
// zero and is not read (x = alpha d).
// alpha = rz_(it-1) / d'.K0 d', the latter folded from the SpMV pass's
// partials (dqp, ndq); block 0 stores d'.K0 d' and alpha.
template <class R, int DIM>
__global__ __launch_bounds__(FX * FY) void k0_update_smooth(Op0<R> op, int kz, int ntx, int nty, R omega,
                                                        double* __restrict__ scal, int it, int xzero,
                                                        R* __restrict__ x, R* __restrict__ r,
                                                        const R* __restrict__ d, R* __restrict__ z1,
                                                        const double* __restrict__ dqp, int ndq,
                                                        double* __restrict__ part, const int* __restrict__ iflag) {
  if (iflag[I_DONE]) return;
  const Tile T = tile_of(op.nx, op.ny, op.nz, ntx, nty, kz);
  const double dq = fold_partials(dqp, ndq);
  const double ad = scal[rz_slot(it - 1)] / dq;
  if (blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
    scal[S_DQ] = dq;
    scal[S_ALPHA] = ad;
  }
  const R al = R(ad);
  double acc = 0.0;
  auto X = [&](long c, int, int, int) { return d[c]; };
  const R* __restrict__ xs = xzero ? r : x;  // from zero: a load of r, which is read anyway
  auto pre = [&](long c) { return Vec2<R>{xs[c], r[c]}; };
  const Ident<R> XV;
  auto body = [&](long c, int, R dc, R Kd, R dg, const Vec2<R>& v) {
    x[c] = (xzero ? R(0) : v.a) + al * dc;
    const R rn = v.b - al * Kd;
    r[c] = rn;
    acc += (double)rn * (double)rn;
    z1[c] = omega * recip(dg) * rn;
  };
  march<R, DIM, true, false>(op, T, X, XV, pre, body, NoPost());
  write_partial(acc, part);
}

// z1 = omega b / diag
template <class R, int DIM>
__global__ __launch_bounds__(FX * FY) void k0_smooth_first(Op0<R> op, int kz, int ntx, int nty, R omega,
                                                       const R* __restrict__ b, R* __restrict__ z1,
                                                       const int* __restrict__ iflag) {
  if (iflag[I_DONE]) return;
  const Tile T = tile_of(op.nx, op.ny, op.nz, ntx, nty, kz);
  auto X = [&](long, int, int, int) { return R(0); };
  const Ident<R> XV;
  auto pre = [&](long c) { return b[c]; };
  auto body = [&](long c, int, R, R, R dg, R bc) { z1[c] = omega * recip(dg) * bc; };
  march<R, DIM, false, false>(op, T, X, XV, pre, body, NoPost());
}

// The inner FP32 solve's first sweep straight from the FP64 refinement
// residual: r32 = (float)(r64 / scale) is written as the inner right-hand
// side, z1 = omega r32 / diag, and block partials of |r32|^2 (one pass
// instead of a scaling pass and a sweep).
template <int DIM>
__global__ __launch_bounds__(FX * FY) void k0_smooth_first64(Op0<float> op, int kz, int ntx, int nty, float omega,
                                                         const double* __restrict__ r64,
                                                         const double* __restrict__ scal, float* __restrict__ r32,
                                                         float* __restrict__ z1, double* __restrict__ part) {
  const Tile T = tile_of(op.nx, op.ny, op.nz, ntx, nty, kz);
  const double scale = scal[S_SCALE];
  double acc = 0.0;
  auto X = [&](long, int, int, int) { return 0.0f; };
  const Ident<float> XV;
  auto pre = [&](long c) { return r64[c]; };
  auto body = [&](long c, int, float, float, float dg, double rv) {
    const float q = (float)(rv / scale);
    r32[c] = q;
    z1[c] = omega * recip(dg) * q;
    acc += (double)q * (double)q;
  };
  march<float, DIM, false, false>(op, T, X, XV, pre, body, NoPost());
  write_partial(acc, part);
}

// damped Jacobi xo = x + omega (b - K0 x) / diag; optional partial b.xo.
// PRO: the sweep acts on x' = x + omc * P e, the coarse correction applied on
// the fly (e is the next-coarser level's solution).
template <class R, int DIM, bool PRO>
__global__ __launch_bounds__(FX * FY) void k0_smooth(Op0<R> op, int kz, int ntx, int nty, R omega,
                                                 const R* __restrict__ b, const R* __restrict__ x,
                                                 R* __restrict__ xo, const R* __restrict__ e, int cnx, int cny,
                                                 R omc, double* __restrict__ part, const int* __restrict__ iflag) {
  if (iflag[I_DONE]) return;
  const Tile T = tile_of(op.nx, op.ny, op.nz, ntx, nty, kz);
  double acc = 0.0;
  auto pre = [&](long c) { return b[c]; };
  auto body = [&](long c, int, R xc, R Kx, R dg, R bc) {
    const R xn = xc + omega * recip(dg) * (bc - Kx);
    xo[c] = xn;
    acc += (double)bc * (double)xn;
  };
  auto X = [&](long c, int ii, int jj, int kk) {
    if (!PRO) return Vec2<R>{x[c], R(0)};
    return Vec2<R>{x[c],
                   e[(long)(ii >> 1) + (long)cnx * ((long)(jj >> 1) + (long)cny * (DIM == 3 ? (kk >> 1) : 0))]};
  };
  auto XV = [&](const Vec2<R>& v) { return PRO ? v.a + omc * v.b : v.a; };
  march<R, DIM, true, false>(op, T, X, XV, pre, body, NoPost());
  if (part) write_partial(acc, part);
}

// Two damped-Jacobi sweeps in one z-march (temporal blocking):
//   x1 = x0' + w1 (b - K0 x0') / diag,   x2 = x1 + w2 (b - K0 x1) / diag,
// with x0' = x0 + omc P e under PRO (the coarse correction applied on the
// fly).  The first sweep runs on the tile and a one-cell ring (the second
// sweep's in-plane neighbours), one plane ahead of the second.  x0', the
// density and b of the tile with a two-cell ring go through a four-plane
// LDS ring (planes k-1..k+1 in use, k+2 being written), the first sweep's
// plane through a two-plane one; a thread's own cell keeps its first-sweep
// value, face weights and diagonal in registers for the second sweep.  The
// face terms are summed in the order of the single sweep (k0_smooth).  One
// barrier per plane: plane k+2 is written after it, when every thread is
// done with plane k-2, whose slot it takes.  Tiles are 64 x TYK.  The loop
// computes two planes per pass, the own cell's kept values alternating
// between two register sets instead of being copied from plane to plane
// (99 -> 93 us at 256^3, against 61 + 66 us for the two single sweeps).
// The pass is bound by its instruction stream (the ring, LDS traffic, six
// reciprocals per first-sweep cell), not by HBM: loading two planes ahead
// (more registers, fewer blocks per CU) measured 108 us against 105 us of
// the one-plane loop, and 64 x 16 tiles 111 us.
template <int TYK>
__device__ __forceinline__ Tile tile_of_ty(int nx, int ny, int nz, int ntx, int nty, int kz) {
  const int nb = gridDim.x, b = blockIdx.x;
  const int t = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int tx = t % ntx, rr = t / ntx;
  const int ty = rr % nty, tz = rr / nty;
  Tile T;
  T.i = tx * FX + threadIdx.x;
  T.j = ty * TYK + threadIdx.y;
  T.k0 = tz * kz;
  T.k1 = min(T.k0 + kz, nz);
  T.act = T.i < nx && T.j < ny && T.k0 < nz;
  return T;
}

constexpr int S2Y = 8;  // rows of the fused sweep's tile (16 measured slower: 111 against 105 us at 256^3)

template <class R, bool PRO, int TYK>
__global__ __launch_bounds__(FX * TYK) void k0_smooth2(Op0<R> op, int kz, int ntx, int nty, R om1, R om2,
                                                   const R* __restrict__ b, const R* __restrict__ x,
                                                   R* __restrict__ xo, const R* __restrict__ e, int cnx, int cny,
                                                   R omc, double* __restrict__ part,
                                                   const int* __restrict__ iflag) {
  constexpr int RX2 = FX + 4, RY2 = TYK + 4, NR2 = RX2 * RY2;  // two-cell ring region
  constexpr int NRING = 2 * (FX + 2) + 2 * TYK;                // one-cell ring of the tile
  constexpr int NT = FX * TYK;
  static_assert(NR2 <= 2 * NT && NRING <= NT, "two load items and one ring cell per thread");
  if (iflag[I_DONE]) return;
  __shared__ R sx[4][NR2];
  __shared__ R sr[4][NR2];
  __shared__ R sb[4][NR2];
  __shared__ R s1[2][NR2];
  const Tile T = tile_of_ty<TYK>(op.nx, op.ny, op.nz, ntx, nty, kz);
  if (T.k0 >= op.nz) return;  // the same for the whole block
  const int nx = op.nx, ny = op.ny, nz = op.nz;
  const long pl = (long)nx * ny;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + FX * ty;
  const int i0 = T.i - tx, j0 = T.j - ty;  // tile origin
  // load items: region cells tid and tid + NT
  long lc[2], lec[2];
  int lslot[2];
  bool lon[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int q = tid + NT * m;
    lon[m] = q < NR2;
    const int rx = q % RX2, ry = q / RX2;
    const int gi = min(max(i0 - 2 + rx, 0), nx - 1), gj = min(max(j0 - 2 + ry, 0), ny - 1);
    lc[m] = (long)gi + (long)nx * gj;
    lslot[m] = lon[m] ? q : 0;
    lec[m] = PRO ? (long)(gi >> 1) + (long)cnx * (long)(gj >> 1) : 0;
  }
  const long cplane = (long)cnx * cny;
  // first-sweep items: the own cell, and for tid < NRING one ring cell
  int qx[2], qy[2];
  qx[0] = tx + 1;
  qy[0] = ty + 1;
  if (tid < FX + 2) { qx[1] = tid; qy[1] = 0; }
  else if (tid < 2 * (FX + 2)) { qx[1] = tid - (FX + 2); qy[1] = TYK + 1; }
  else if (tid < 2 * (FX + 2) + TYK) { qx[1] = 0; qy[1] = tid - 2 * (FX + 2) + 1; }
  else if (tid < NRING) { qx[1] = FX + 1; qy[1] = tid - 2 * (FX + 2) - TYK + 1; }
  else { qx[1] = 0; qy[1] = 0; }
  int gi1[2], gj1[2], li[2];
  bool in1[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    gi1[m] = i0 - 1 + qx[m];
    gj1[m] = j0 - 1 + qy[m];
    in1[m] = (m == 0 || tid < NRING) && gi1[m] >= 0 && gi1[m] < nx && gj1[m] >= 0 && gj1[m] < ny;
    li[m] = (qy[m] + 1) * RX2 + (qx[m] + 1);  // position in the two-cell-ring region
  }
  const bool own = T.act;
  // planes: first sweep on [ks, ke], second on [k0, k1)
  const int k0 = T.k0, k1 = T.k1;
  const int ks = max(k0 - 1, 0), ke = min(k1, nz - 1);
  const int kend = min(k1, nz);  // last plane step: the second sweep of k1 - 1 needs x1 of k1 (if k1 < nz)
  R ldx[2], lda[2], ldb[2], lde[2];
  auto issue = [&](int k) {  // loads of plane k (clamped), into the staging registers
    const int kk = min(max(k, 0), nz - 1);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const long c = lc[m] + pl * kk;
      ldx[m] = x[c];
      lda[m] = op.a[c];
      ldb[m] = b[c];
      if (PRO) lde[m] = e[lec[m] + cplane * (kk >> 1)];
    }
  };
  auto store = [&](int k) {  // the staged plane k into its LDS slot
    const int sl = k & 3;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (lon[m]) {
        sx[sl][lslot[m]] = PRO ? ldx[m] + omc * lde[m] : ldx[m];
        sr[sl][lslot[m]] = rho0(op, lda[m]);
        sb[sl][lslot[m]] = ldb[m];
      }
    }
  };
  // the own cell's first-sweep value, face weights, diagonal and b of one
  // plane, kept for its second sweep one plane later; two of them take
  // turns (the loop runs two planes per pass), so nothing is copied between
  // planes
  struct Own {
    R w[6], x1, dg, b;
    bool in;
  };
  Own oa{{R(0), R(0), R(0), R(0), R(0), R(0)}, R(0), R(1), R(0), false}, ob = oa;
  R px1m = R(0);  // first-sweep value of the own cell two planes back
  double acc = 0.0;
  if (ks > 0) {
    issue(ks - 1);
    store(ks - 1);
  }
  issue(ks);
  store(ks);
  if (ks + 1 <= nz - 1) {
    issue(ks + 1);
    store(ks + 1);
  }
  issue(ks + 2);
  // plane k: the first sweep of plane k into `now`, then the second sweep of
  // plane k - 1 from `prev`
  auto plane = [&](int k, Own& now, const Own& prev) {
    __syncthreads();
    const int sc = k & 3, sm = (k + 3) & 3, sp = (k + 1) & 3;
    now.in = false;
    if (k <= ke) {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        if (!in1[m]) continue;
        const int l = li[m];
        const R rc = sr[sc][l], xc = sx[sc][l];
        // every face is evaluated (the region holds clamped values beyond a
        // wall) and a wall face is dropped by a select, not a branch: no
        // exec-mask updates per face
        const bool on[6] = {gi1[m] > 0, gi1[m] < nx - 1, gj1[m] > 0, gj1[m] < ny - 1, k > 0, k < nz - 1};
        const int off[6] = {-1, 1, -RX2, RX2, 0, 0};
        R s = R(0), d = R(0), wv[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const R rn = f < 4 ? sr[sc][l + off[f]] : (f == 4 ? sr[sm][l] : sr[sp][l]);
          const R xn = f < 4 ? sx[sc][l + off[f]] : (f == 4 ? sx[sm][l] : sx[sp][l]);
          const R wf = coef(R(op.c2), f == 4 ? rn + rc : rc + rn);
          wv[f] = on[f] ? wf : R(0);
          s = on[f] ? s + wf * (xc - xn) : s;
          d = on[f] ? d + wf : d;
        }
        const R bc = sb[sc][l];
        const R x1 = xc + om1 * recip(d) * (bc - s);
        s1[k & 1][l] = x1;
        if (m == 0) {
          now.x1 = x1;
          now.dg = d;
          now.b = bc;
          now.in = true;
#pragma unroll
          for (int f = 0; f < 6; ++f) now.w[f] = wv[f];
        }
      }
    }
    if (k + 2 <= nz - 1 && k + 2 <= kend + 1) {
      store(k + 2);
      issue(k + 3);
    }
    // second sweep of plane k - 1 (own cell)
    const int k2 = k - 1;
    if (own && k2 >= k0 && k2 < k1 && prev.in) {
      const int l = li[0], sl = k2 & 1;
      // selects, as in the first sweep (a first-sweep value beyond a wall
      // is never computed, so it must not reach the sum even times zero);
      // the four in-plane neighbours are read before any is used (inside the
      // tile's ring, so in bounds), so that no face becomes a branch around
      // its own LDS read
      const R nw = s1[sl][l - 1], ne = s1[sl][l + 1], ns = s1[sl][l - RX2], nn = s1[sl][l + RX2];
      const R px1 = prev.x1;
      R s = R(0);
      s = T.i > 0 ? s + prev.w[0] * (px1 - nw) : s;
      s = T.i < nx - 1 ? s + prev.w[1] * (px1 - ne) : s;
      s = T.j > 0 ? s + prev.w[2] * (px1 - ns) : s;
      s = T.j < ny - 1 ? s + prev.w[3] * (px1 - nn) : s;
      s = k2 > 0 ? s + prev.w[4] * (px1 - px1m) : s;
      s = k2 < nz - 1 ? s + prev.w[5] * (px1 - now.x1) : s;
      const R x2 = px1 + om2 * recip(prev.dg) * (prev.b - s);
      xo[(long)T.i + (long)nx * T.j + pl * k2] = x2;
      acc += (double)prev.b * (double)x2;
    }
    px1m = prev.x1;
  };
  int k = ks;
  for (; k + 1 <= kend; k += 2) {
    plane(k, oa, ob);
    plane(k + 1, ob, oa);
  }
  if (k <= kend) plane(k, oa, ob);
  if (part) {
    __shared__ double sh[16];
    const double sacc = block_reduce<0>(acc, sh);
    if (tid == 0) part[blockIdx.x] = sacc;
  }
}

// bc = R (b - K0 x): fine cells marched like the sweeps; the 2x2 in-plane
// sum goes through LDS, the pair of planes is summed in a register, and the
// thread at the even corner of each 2x2(x2) group writes the coarse value.
// With x1c it also writes the coarse level's first sweep from zero,
// x1c = om0 bc / diag_c (wdc = 1 / diag_c).
template <class R, int DIM>
__global__ __launch_bounds__(FX * FY) void k0_resid_restrict(Op0<R> op, int kz, int ntx, int nty, int cnx, int cny,
                                                         const R* __restrict__ b, const R* __restrict__ x,
                                                         R* __restrict__ bc, const R* __restrict__ wdc,
                                                         R* __restrict__ x1c, R om0, const int* __restrict__ iflag) {
  if (iflag[I_DONE]) return;
  __shared__ R sres[FY][FX];
  const Tile T = tile_of(op.nx, op.ny, op.nz, ntx, nty, kz);
  const int tx = threadIdx.x, ty = threadIdx.y;
  R zsum = R(0), wdv = R(0);
  auto X = [&](long c, int, int, int) { return x[c]; };
  const Ident<R> XV;
  auto pre = [&](long c) { return b[c]; };
  auto body = [&](long, int, R, R Kx, R, R bc) { sres[ty][tx] = bc - Kx; };
  // The four threads of a 2x2 group sum the same four residuals and store the
  // same coarse value (no thread-dependent store); 1/diag of the coarse cell
  // is loaded by every thread at the even plane and used at the odd one.
  const long cbase = T.act ? (long)(T.i >> 1) + (long)cnx * (long)(T.j >> 1) : 0;
  const long cplane = (long)cnx * cny;
  const int bx = tx & ~1, by = ty & ~1;
  auto post = [&](int k) {
    const long ci = cbase + cplane * (DIM == 3 ? (k >> 1) : 0);
    if (x1c && (DIM == 2 || !(k & 1))) wdv = wdc[ci];
    if (T.act) {
      // the partner cells lie inside the tile (nx, ny even)
      zsum += (sres[by][bx] + sres[by][bx + 1]) + (sres[by + 1][bx] + sres[by + 1][bx + 1]);
      if (DIM == 2 || (k & 1)) {
        bc[ci] = zsum;
        if (x1c) x1c[ci] = om0 * wdv * zsum;
        zsum = R(0);
      }
    }
  };
  march<R, DIM, true, true>(op, T, X, XV, pre, body, post);
}

// FP64 residual of the refinement, r = -(b - mean b) - K p, with block
// partials of ||b - mean b||^2 and ||r||^2.  28 bytes per cell (alpha as
// stored, b and p read, r written) instead of the 48 of stored FP64 weights.
template <class A, int DIM>
__global__ __launch_bounds__(FX * FY) void k0_resid64(Op64<A> op, int kz, int ntx, int nty,
                                                  const double* __restrict__ b, const double* __restrict__ scal,
                                                  const double* __restrict__ p, double* __restrict__ r,
                                                  double* __restrict__ pbb, double* __restrict__ prr) {
  const Tile T = tile_of(op.nx, op.ny, op.nz, ntx, nty, kz);
  const double mean = scal[S_MEAN];
  double vb = 0.0, vr = 0.0;
  auto X = [&](long c, int, int, int) { return p[c]; };
  const Ident<double> XV;
  auto pre = [&](long c) { return b[c]; };
  auto body = [&](long c, int, double, double Kp, double, double bc) {
    const double rhs = -(bc - mean);
    const double rr = rhs - Kp;
    r[c] = rr;
    vb += rhs * rhs;
    vr += rr * rr;
  };
  march<double, DIM, true, false>(op, T, X, XV, pre, body, NoPost());
  write_partial(vb, pbb);
  write_partial(vr, prr);
}

struct Launch {
  int ntx, nty, kz, nblocks;
};

Launch plan(int nx, int ny, int nz, int target = TCF_FINE_BLOCKS, int ty = FY) {
  Launch L;
  L.ntx = (nx + FX - 1) / FX;
  L.nty = (ny + ty - 1) / ty;
  const int cols = L.ntx * L.nty;
  // aim for >= target blocks (TCF_FINE_BLOCKS: two full rounds of the two
  // blocks per CU that most of these kernels' register counts allow) with
  // chunks of at least 8 planes
  int ntz = std::max(1, std::min(nz, (target + cols - 1) / cols));
  int kz = (nz + ntz - 1) / ntz;
  if (kz < 8 && nz >= 8) kz = 8;
  if (nz > 1 && (kz & 1)) kz += 1;  // plane pairs of the restriction stay in one chunk
  L.kz = std::max(1, kz);
  ntz = (nz + L.kz - 1) / L.kz;
  L.nblocks = cols * ntz;
  return L;
}

template <class R>
Op0<R> op_of(const Fine<R>& F) {
  Op0<R> o;
  o.a = F.a;
  o.nx = F.nx;
  o.ny = F.ny;
  o.nz = F.nz;
  o.rho1 = F.rho1;
  o.drho = F.drho;
  o.c2 = F.c2;
  return o;
}

}  // namespace

int fine_blocks(int nx, int ny, int nz) { return plan(nx, ny, nz).nblocks; }

template <class R>
int fine_spmv_upd(hipStream_t s, int dim, const Fine<R>& F, const R* z, const R* dold, R* dnew, double* scal,
                  int it, const double* rzpart, int nrz, double* part, const int* iflag) {
  const Launch L = plan(F.nx, F.ny, F.nz);
  const Op0<R> op = op_of(F);
  if (dim == 3)
    hipLaunchKernelGGL((k0_spmv_upd<R, 3>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty, z, dold, dnew,
                       scal, it, rzpart, nrz, part, iflag);
  else
    hipLaunchKernelGGL((k0_spmv_upd<R, 2>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty, z, dold, dnew,
                       scal, it, rzpart, nrz, part, iflag);
  return L.nblocks;
}

template <class R>
int fine_update_smooth(hipStream_t s, int dim, const Fine<R>& F, double omega, double* scal, int it, int xzero, R* x,
                       R* r, const R* d, R* z1, const double* dqpart, int ndq, double* part, const int* iflag) {
  const Launch L = plan(F.nx, F.ny, F.nz);
  const Op0<R> op = op_of(F);
  if (dim == 3)
    hipLaunchKernelGGL((k0_update_smooth<R, 3>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty, R(omega),
                       scal, it, xzero, x, r, d, z1, dqpart, ndq, part, iflag);
  else
    hipLaunchKernelGGL((k0_update_smooth<R, 2>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty, R(omega),
                       scal, it, xzero, x, r, d, z1, dqpart, ndq, part, iflag);
  return L.nblocks;
}

template <class R>
void fine_smooth_first(hipStream_t s, int dim, const Fine<R>& F, double omega, const R* b, R* z1, const int* iflag) {
  const Launch L = plan(F.nx, F.ny, F.nz);
  const Op0<R> op = op_of(F);
  if (dim == 3)
    hipLaunchKernelGGL((k0_smooth_first<R, 3>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty, R(omega),
                       b, z1, iflag);
  else
    hipLaunchKernelGGL((k0_smooth_first<R, 2>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty, R(omega),
                       b, z1, iflag);
}

// Blocks the GPU holds at once for kernel k (512 threads), over all CUs; 0
// if the runtime cannot tell.
int resident_blocks(const void* k) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, FX * FY, 0) != hipSuccess)
    return 0;
  return per * ncu;
}

// The plain sweep holds more blocks per CU than the other finest-level
// kernels (fewer registers): it is launched as one full round of them, so
// that no partial round trails.
template <class R, int DIM>
int sweep_blocks() {
  static const int n = [] {
    const int r = resident_blocks((const void*)k0_smooth<R, DIM, false>);
    return r >= 256 ? r : TCF_FINE_BLOCKS;
  }();
  return n;
}

int fine_smooth_first64(hipStream_t s, int dim, const Fine<float>& F, double omega, const double* r64,
                        const double* scal, float* r32, float* z1, double* part) {
  const Launch L = plan(F.nx, F.ny, F.nz);
  const Op0<float> op = op_of(F);
  if (dim == 3)
    hipLaunchKernelGGL((k0_smooth_first64<3>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty,
                       float(omega), r64, scal, r32, z1, part);
  else
    hipLaunchKernelGGL((k0_smooth_first64<2>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty,
                       float(omega), r64, scal, r32, z1, part);
  return L.nblocks;
}

template <class R>
int fine_smooth(hipStream_t s, int dim, const Fine<R>& F, double omega, const R* b, const R* x, R* xo, const R* e,
                int cnx, int cny, double omc, double* part, const int* iflag) {
  const int target = e ? TCF_FINE_BLOCKS : (dim == 3 ? sweep_blocks<R, 3>() : sweep_blocks<R, 2>());
  const Launch L = plan(F.nx, F.ny, F.nz, target);
  const Op0<R> op = op_of(F);
  if (dim == 3) {
    if (e)
      hipLaunchKernelGGL((k0_smooth<R, 3, true>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty,
                         R(omega), b, x, xo, e, cnx, cny, R(omc), part, iflag);
    else
      hipLaunchKernelGGL((k0_smooth<R, 3, false>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty,
                         R(omega), b, x, xo, e, cnx, cny, R(omc), part, iflag);
  } else {
    if (e)
      hipLaunchKernelGGL((k0_smooth<R, 2, true>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty,
                         R(omega), b, x, xo, e, cnx, cny, R(omc), part, iflag);
    else
      hipLaunchKernelGGL((k0_smooth<R, 2, false>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty,
                         R(omega), b, x, xo, e, cnx, cny, R(omc), part, iflag);
  }
  return L.nblocks;
}

// Both post-smoothing sweeps (the first with the coarse correction) in one
// pass: FP32, 3-D.
int fine_smooth2(hipStream_t s, const Fine<float>& F, double om1, double om2, const float* b, const float* x,
                 float* xo, const float* e, int cnx, int cny, double omc, double* part, const int* iflag) {
  const Launch L = plan(F.nx, F.ny, F.nz, TCF_FINE_BLOCKS * FY / S2Y, S2Y);
  const Op0<float> op = op_of(F);
  if (e)
    hipLaunchKernelGGL((k0_smooth2<float, true, S2Y>), dim3(L.nblocks), dim3(FX, S2Y), 0, s, op, L.kz, L.ntx, L.nty,
                       float(om1), float(om2), b, x, xo, e, cnx, cny, float(omc), part, iflag);
  else
    hipLaunchKernelGGL((k0_smooth2<float, false, S2Y>), dim3(L.nblocks), dim3(FX, S2Y), 0, s, op, L.kz, L.ntx, L.nty,
                       float(om1), float(om2), b, x, xo, e, cnx, cny, float(omc), part, iflag);
  return L.nblocks;
}

template <class R>
void fine_resid_restrict(hipStream_t s, int dim, const Fine<R>& F, const R* b, const R* x, R* bc, const R* wdc, R* x1c,
                         double om0, const int* iflag) {
  const int cnx = F.nx / 2, cny = F.ny / 2;
  const Launch L = plan(F.nx, F.ny, F.nz);
  const Op0<R> op = op_of(F);
  if (dim == 3)
    hipLaunchKernelGGL((k0_resid_restrict<R, 3>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty, cnx, cny,
                       b, x, bc, wdc, x1c, R(om0), iflag);
  else
    hipLaunchKernelGGL((k0_resid_restrict<R, 2>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty, cnx, cny,
                       b, x, bc, wdc, x1c, R(om0), iflag);
}

template <class R>
int resid64a(const KParams& P, hipStream_t s, const R* a, const double* b, const double* scal, const double* p,
             double* r, double* pbb, double* prr) {
  const int nz = P.dim == 3 ? P.nz : 1;
  const Launch L = plan(P.nx, P.ny, nz);
  const Op64<R> op{a, P.nx, P.ny, nz, P.rho1, P.rho2 - P.rho1, 2.0 * P.ih * P.ih};
  if (P.dim == 3)
    hipLaunchKernelGGL((k0_resid64<R, 3>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty, b, scal, p, r,
                       pbb, prr);
  else
    hipLaunchKernelGGL((k0_resid64<R, 2>), dim3(L.nblocks), dim3(FX, FY), 0, s, op, L.kz, L.ntx, L.nty, b, scal, p, r,
                       pbb, prr);
  return L.nblocks;
}

#define TCF_FINE_INST(R)                                                                                          \
  template int fine_spmv_upd<R>(hipStream_t, int, const Fine<R>&, const R*, const R*, R*, double*, int,           \
                                const double*, int, double*, const int*);                                         \
  template int fine_update_smooth<R>(hipStream_t, int, const Fine<R>&, double, double*, int, int, R*, R*, const R*, \
                                     R*, const double*, int, double*, const int*);                               \
  template void fine_smooth_first<R>(hipStream_t, int, const Fine<R>&, double, const R*, R*, const int*);         \
  template int fine_smooth<R>(hipStream_t, int, const Fine<R>&, double, const R*, const R*, R*, const R*, int,    \
                              int, double, double*, const int*);                                                  \
  template void fine_resid_restrict<R>(hipStream_t, int, const Fine<R>&, const R*, const R*, R*, const R*, R*, double,  \
                                        const int*);                                                              \
  template int resid64a<R>(const KParams&, hipStream_t, const R*, const double*, const double*, const double*,    \
                           double*, double*, double*);

TCF_FINE_INST(double)
TCF_FINE_INST(float)

}  // namespace tcf
