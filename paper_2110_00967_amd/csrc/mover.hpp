// mover.hpp -- moving rigid disks (Eqs. dep1, theta2), advanced inside the
// step kernel.
//
// The launch that computes step N uses, for each moving disk, the state S
// that the forces of step N - 1 produce.  Step N - 1 left, for every tile of
// the disk's window (a square of cells around its reference point), the sums
// over the tile of its momentum-exchange terms (Sec. 2.3.1) and of its
// points' stress-integration terms at the tile's sample nodes (Sec. 2.3.2).
// Every workgroup whose tile meets a window adds those partial sums itself,
// in one fixed order, so all of them obtain the same S bit for bit without
// waiting for one another; the workgroup of the tile holding the disk's
// centre cell records the forces and the new state.  Then the disk's solid
// cells, interface cells and sample nodes follow from S by exact integer
// tests, with no mask to rebuild.
#pragma once

#include "sample.hpp"

namespace vp {

// Width of the force sums' order: FIN_W virtual lanes, lane v summing terms
// v, v + FIN_W, ...; each virtual wave of 64 lanes reduced by wave_sum_f64,
// the FIN_W / 64 wave sums added in order.  Every workgroup size runs the
// same order (a block of NT threads takes the virtual waves w, w + NT/64,
// ... with its waves w).
constexpr int FIN_W = 256;
constexpr int FIN_WAVES = FIN_W / 64;

// Several disks, one state each: a node is solid when inside one of them;
// id() gives the disk (1..n) or 0.
struct MultiDiskSolid {
  int n;
  long long X[MAX_MOVERS], Y[MAX_MOVERS], R[MAX_MOVERS];
  __device__ __forceinline__ int id(int i, int j) const {
    int r = 0;
#pragma unroll
    for (int k = MAX_MOVERS - 1; k >= 0; --k)
      if (k < n && disk_inside(X[k], Y[k], R[k], i, j)) r = k + 1;
    return r;
  }
  __device__ __forceinline__ bool operator()(int i, int j) const { return id(i, j) != 0; }
};

// The same, with the disks' centres and radii read from memory (LDS) at
// each test instead of held in registers.
struct DiskSetRef {
  int n;
  const long long *X, *Y, *R;
  __device__ __forceinline__ int id(int i, int j) const {
    for (int k = 0; k < n; ++k)
      if (disk_inside(X[k], Y[k], R[k], i, j)) return k + 1;
    return 0;
  }
  __device__ __forceinline__ bool operator()(int i, int j) const { return id(i, j) != 0; }
};

__device__ __forceinline__ long long fixq_of(double v) { return llround(v * FIXQ); }

// x of the lane that DPP control `ctrl` selects (both halves of the double)
template <int CTRL> __device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ double readlane_f64(double x, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), lane),
                          __builtin_amdgcn_readlane(__double2loint(x), lane));
}

// Sum of x over the 64 lanes of a wave, in one fixed order, the same in
// every lane: within each row of 16 lanes, lanes paired by swapping
// neighbours, then pairs, then the two halves of each group of 8 (mirrored),
// then the two halves of the row (mirrored) -- every step adds two equal-sized
// partial sums, so all lanes of a row hold the same bits; then the four row
// sums (r0 + r1) + (r2 + r3).  Data-parallel-primitive moves instead of LDS
// permutes keep the chain short.
__device__ __forceinline__ double wave_sum_f64(double x) {
  x += dpp_f64<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp_f64<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  x += dpp_f64<0x141>(x);  // row_half_mirror
  x += dpp_f64<0x140>(x);  // row_mirror
  return (readlane_f64(x, 0) + readlane_f64(x, 16)) + (readlane_f64(x, 32) + readlane_f64(x, 48));
}

// lower corner of the (2 h + 1)^2-cell window of a disk at state B
__device__ __forceinline__ void mover_origin(const BodyDev &B, int h, int &ox, int &oy) {
  ox = (int)floor(B.x) - h;
  oy = (int)floor(B.y) - h;
}

__device__ __forceinline__ int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// The tiles (MOV_BX x MOV_BY) of the window of a disk at state B: the first
// tile (tx0, ty0) and the box's size ntx x nty (at most M.ptx x M.pty).
__device__ __forceinline__ void mover_tile_box(const BodyDev &B, int h, int &tx0, int &ty0, int &ntx, int &nty) {
  int ox, oy;
  mover_origin(B, h, ox, oy);
  tx0 = floordiv(ox, MOV_BX);
  ty0 = floordiv(oy, MOV_BY);
  ntx = floordiv(ox + 2 * h, MOV_BX) - tx0 + 1;
  nty = floordiv(oy + 2 * h, MOV_BY) - ty0 + 1;
}

// Forces of the step that used state B of disk M: F[0..2] momentum exchange
// (Fx, Fy, torque), F[3..5] stress integration, from the tile partials of
// that step's window (part, slot (ty - ty0) * M.ptx + (tx - tx0)), tiles
// outside the lattice skipped.  One fixed order whatever the workgroup size:
// FIN_W virtual lanes, lane v taking slots v, v + FIN_W, ...; a fixed-order
// sum per virtual wave of 64 (wave_sum_f64), the wave sums added in order.
// Every thread returns the same six sums.  lds: FIN_WAVES * 6 doubles.
template <int NT>
__device__ __forceinline__ void mover_forces(const MoverDev &M, const BodyDev &B, const double *__restrict__ part,
                                             int tiles_x, int tiles_y, double *lds, double (&F)[6]) {
  // force and geometry arithmetic: no multiply-add fusion, so that every kernel
  // that inlines this (alone, batched, any tile) rounds it the same way
  #pragma clang fp contract(off)
  static_assert(NT % 64 == 0, "whole waves");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int tx0, ty0, ntx, nty;
  mover_tile_box(B, M.half, tx0, ty0, ntx, nty);
  const int nbox = ntx * nty;
  for (int k = wave; k < FIN_WAVES; k += NT / 64) {
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int q = k * 64 + lane; q < nbox; q += FIN_W) {
      const int tx = tx0 + q % ntx, ty = ty0 + q / ntx;
      if (tx < 0 || tx >= tiles_x || ty < 0 || ty >= tiles_y) continue;
      const double *w = part + (long long)(M.part0 + (ty - ty0) * M.ptx + (tx - tx0)) * PART_ENTRY;
#pragma unroll
      for (int i = 0; i < 6; ++i) v[i] += w[i];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const double x = wave_sum_f64(v[i]);
      if (lane == 0) lds[k * 6 + i] = x;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double x = 0.0;
    for (int k = 0; k < FIN_WAVES; ++k) x += lds[k * 6 + i];
    F[i] = x;
  }
  __syncthreads();  // lds is reused by the caller
}

// Eqs. dep1, theta2 with dt = 1, semi-implicit Euler: velocities from the
// force of the step (free disk: F/m + (1 - rho0/rho_s) g, T/I), then
// positions and angle from the new velocities; a prescribed motion keeps its
// velocities.  Each operation rounded on its own (no contraction), in the
// order of the plain formulas.
__device__ __forceinline__ BodyDev mover_update(const MoverDev &M, const BodyDev &B, const double (&F)[6]) {
  // force and geometry arithmetic: no multiply-add fusion, so that every kernel
  // that inlines this (alone, batched, any tile) rounds it the same way
  #pragma clang fp contract(off)
  BodyDev S = B;
  if (M.mode == MODE_FREE) {
    const bool si = M.source != 0;
    const double fx = si ? F[3] : F[0], fy = si ? F[4] : F[1], tq = si ? F[5] : F[2];
    S.u = __dadd_rn(S.u, __dadd_rn(fx / M.mass, __dmul_rn(M.buoy, M.gx)));
    S.v = __dadd_rn(S.v, __dadd_rn(fy / M.mass, __dmul_rn(M.buoy, M.gy)));
    S.omega = __dadd_rn(S.omega, tq / M.inertia);
  }
  S.x = __dadd_rn(S.x, S.u);
  S.y = __dadd_rn(S.y, S.v);
  S.theta = __dadd_rn(S.theta, S.omega);
  return S;
}

}  // namespace vp
