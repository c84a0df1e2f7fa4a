// Device helpers shared by the HIP kernel files: index maps, ghost rules,
// material mixing, WENO5, and deterministic block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "tcf_internal.h"

namespace tcf {
namespace dev {

constexpr int BX = 64, BY = 4;

// ---------------------------------------------------------------------------
// Ghost rules.  alpha: even reflection.  T: even (Neumann) or 2 T_w - mirror
// (Dirichlet).  Velocity component C: odd reflection about its wall faces
// along C (normal), odd reflection about the wall along the other axes
// (tangential, no slip).
// Reciprocal and reciprocal square root: the hardware instructions in FP32
// (within about an ulp, far inside the FP32 path's error budget), correctly
// rounded in FP64.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsq(double x) { return 1.0 / sqrt(x); }

__device__ __forceinline__ int refl(int i, int n) { return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i); }

__device__ __forceinline__ long cidx(int i, int j, int k, int nx, int ny) {
  return (long)i + (long)nx * ((long)j + (long)ny * k);
}

template <int DIM, class R>
__device__ __forceinline__ R A_at(const R* __restrict__ a, int i, int j, int k, int nx, int ny, int nz) {
  return a[cidx(refl(i, nx), refl(j, ny), DIM == 3 ? refl(k, nz) : 0, nx, ny)];
}

template <int DIM, class R>
__device__ __forceinline__ R T_at(const R* __restrict__ T, int i, int j, int k, const KParams& P) {
  R v = T[cidx(refl(i, P.nx), refl(j, P.ny), DIM == 3 ? refl(k, P.nz) : 0, P.nx, P.ny)];
  if (i < 0 && P.Tbc[0]) v = R(2) * R(P.Tw[0]) - v;
  if (i >= P.nx && P.Tbc[1]) v = R(2) * R(P.Tw[1]) - v;
  if (j < 0 && P.Tbc[2]) v = R(2) * R(P.Tw[2]) - v;
  if (j >= P.ny && P.Tbc[3]) v = R(2) * R(P.Tw[3]) - v;
  if (DIM == 3) {
    if (k < 0 && P.Tbc[4]) v = R(2) * R(P.Tw[4]) - v;
    if (k >= P.nz && P.Tbc[5]) v = R(2) * R(P.Tw[5]) - v;
  }
  return v;
}

template <int C>
__device__ __forceinline__ long fidx(int i, int j, int k, int nx, int ny) {
  if (C == 0) return (long)i + (long)(nx + 1) * ((long)j + (long)ny * k);
  if (C == 1) return (long)i + (long)nx * ((long)j + (long)(ny + 1) * k);
  return (long)i + (long)nx * ((long)j + (long)ny * k);
}

template <int C, int DIM, class R>
__device__ __forceinline__ R V_at(const R* __restrict__ uc, int i, int j, int k, int nx, int ny, int nz) {
  R sg = R(1);
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
  return sg * uc[fidx<C>(id[0], id[1], id[2], nx, ny)];
}

// Linear material mix p1 + clamp(a, 0, 1) (p2 - p1).
template <class R>
__device__ __forceinline__ R mixp(R a, double p1, double p2) {
  a = a < R(0) ? R(0) : (a > R(1) ? R(1) : a);
  return R(p1) + a * R(p2 - p1);
}
// FP32: the clamp is one median-of-three (identical for every finite a).
template <>
__device__ __forceinline__ float mixp<float>(float a, double p1, double p2) {
  return float(p1) + __builtin_amdgcn_fmed3f(a, 0.0f, 1.0f) * float(p2 - p1);
}

// ---------------------------------------------------------------------------
// Deterministic block reduction (256 threads = 4 wavefronts of 64).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
  return v;
}

template <int OP>  // 0 sum, 1 max, 2 min
__device__ __forceinline__ double block_reduce(double v, double* sh) {
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  const int lane = tid & 63, wid = tid >> 6;
  v = OP == 0 ? wave_sum(v) : (OP == 1 ? wave_max(v) : wave_min(v));
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = sh[0];
  const int nw = (blockDim.x * blockDim.y + 63) >> 6;
  for (int w = 1; w < nw; ++w) r = OP == 0 ? r + sh[w] : (OP == 1 ? fmax(r, sh[w]) : fmin(r, sh[w]));
  return r;
}

__device__ __forceinline__ int block_linear() { return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z); }
// Tile number of a block of a 1-D grid, grouped by XCD: the dispatcher deals
// blocks round-robin over the 8 XCDs (block b runs on XCD b % 8), so XCD x
// receives the contiguous tile range [x nb/8, (x+1) nb/8) and neighbouring
// tiles share that XCD's L2.
__device__ __forceinline__ int xcd_tile() {
  const int nb = gridDim.x, b = blockIdx.x;
  return (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
}


}  // namespace dev
}  // namespace tcf
