// sample.hpp -- geometry shared by the step kernel and the set-up kernels:
// the exact disk test on the 1/4096 grid (Eq. fcar for a disk), the
// stress-integration sample nodes of a point (Sec. 2.3.2) and the placement
// of a rigid body's points (Eqs. dep1, theta2).
#pragma once

#include "d2q9.hpp"

namespace vp {

// chi of a disk: cell (i, j) is inside when its centre is within the radius,
// exact integer arithmetic on the 1/FIXQ grid
__device__ __forceinline__ bool disk_inside(long long X, long long Y, long long R, int i, int j) {
  const long long dx = (long long)i * FIXQ - X, dy = (long long)j * FIXQ - Y;
  return dx * dx + dy * dy <= R * R;
}

// Solid test of a lattice node for the sample-node search: the mask (any
// geometry), or, for a moving disk alone in its lattice, the disk rule that
// has just built its mask (the same answer without a memory round trip).
struct MaskSolid {
  const uint8_t *mask;
  int pitch;
  __device__ __forceinline__ bool operator()(int X, int Y) const {
    return (mask[(long long)Y * pitch + X] & M_BODY) != 0;
  }
};
struct DiskSolid {
  long long X, Y, R;  // centre and radius on the 1/FIXQ grid
  __device__ __forceinline__ bool operator()(int i, int j) const { return disk_inside(X, Y, R, i, j); }
};

// Sample node of a point: the lattice direction beta maximizing
// (c_beta . n)/|c_beta| (first on ties), then the first fluid node inside the
// lattice among r_0 + k c_beta, k = 0..4, r_0 the node nearest to the point.
template <typename Solid>
__device__ __forceinline__ int si_node(const Solid &solid, int nx, int ny, double px, double py, double n0,
                                       double n1) {
  const double S = 0.70710678118654752440;
  // scores of c_1..c_8 in order, the first maximum kept
  double bs = n0;
  int bx = 1, by = 0;
  const auto take = [&](double sc, int X, int Y) {
    if (sc > bs) {
      bs = sc;
      bx = X;
      by = Y;
    }
  };
  take(n1, 0, 1);
  take(-n0, -1, 0);
  take(-n1, 0, -1);
  take((n0 + n1) * S, 1, 1);
  take((-n0 + n1) * S, -1, 1);
  take((-n0 - n1) * S, -1, -1);
  take((n0 - n1) * S, 1, -1);
  const int ix = (int)floor(px + 0.5), iy = (int)floor(py + 0.5);
  for (int k = 0; k <= 4; ++k) {
    const int X = ix + k * bx, Y = iy + k * by;
    if (X < 0 || X >= nx || Y < 0 || Y >= ny) continue;
    if (!solid(X, Y)) return Y * nx + X;
  }
  return -1;
}

// Stencil of an integration point: rule 0, the sample node above with weight
// 1; rule 1, the bilinear interpolation at p = x + 1.5 n over the 4 nodes
// around p when all are fluid and inside the lattice (rule 0 otherwise).
// Returns the number of (node, weight) pairs, 0 when there is no sample node.
// The interpolation point is formed without FMA contraction so the floor()
// decisions match a plain evaluation.
template <typename Solid>
__device__ __forceinline__ int si_stencil(const Solid &solid, int nx, int ny, int rule, double px, double py,
                                          double n0, double n1, int (&node)[4], double (&w)[4]) {
  // force and geometry arithmetic: no multiply-add fusion, so that every kernel
  // that inlines this (alone, batched, any tile) rounds it the same way
  #pragma clang fp contract(off)
  if (rule == 1) {
    const double qx = __dadd_rn(px, __dmul_rn(1.5, n0)), qy = __dadd_rn(py, __dmul_rn(1.5, n1));
    const int i0 = (int)floor(qx), j0 = (int)floor(qy);
    if (i0 >= 0 && j0 >= 0 && i0 + 1 < nx && j0 + 1 < ny) {
      const double fx = __dsub_rn(qx, (double)i0), fy = __dsub_rn(qy, (double)j0);
      bool ok = true;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int X = i0 + (k & 1), Y = j0 + (k >> 1);
        node[k] = Y * nx + X;
        if (solid(X, Y)) ok = false;
        w[k] = __dmul_rn((k & 1) ? fx : __dsub_rn(1.0, fx), (k >> 1) ? fy : __dsub_rn(1.0, fy));
      }
      if (ok) return 4;
    }
  }
  node[0] = si_node(solid, nx, ny, px, py, n0, n1);
  w[0] = 1.0;
  return node[0] >= 0 ? 1 : 0;
}

// world position and normal of a point stored as (a, b) and normal (c, d)
// (points of a moving body are kept in the body frame and placed with the
// current state; co, sn = cos, sin of its angle)
__device__ __forceinline__ void si_place(double a, double b, double c, double d, int moving, const BodyDev &B,
                                         double co, double sn, double &px, double &py, double &n0, double &n1) {
  // force and geometry arithmetic: no multiply-add fusion, so that every kernel
  // that inlines this (alone, batched, any tile) rounds it the same way
  #pragma clang fp contract(off)
  if (!moving) {
    px = a; py = b; n0 = c; n1 = d;
    return;
  }
  px = B.x + (co * a - sn * b);
  py = B.y + (sn * a + co * b);
  n0 = co * c - sn * d;
  n1 = sn * c + co * d;
}

// the same for registered point i
__device__ __forceinline__ void si_world(const double *__restrict__ pts, int maxp, int i, int moving,
                                         const BodyDev &B, double co, double sn, double &px, double &py,
                                         double &n0, double &n1) {
  si_place(pts[i], pts[maxp + i], pts[2 * maxp + i], pts[3 * maxp + i], moving, B, co, sn, px, py, n0, n1);
}

}  // namespace vp
