// d2q9.hpp -- D2Q9 constants, storage traits and device-side state shared by
// the HIP kernels of the VP-LBM library (gfx950).
//
// Velocity set and weights: Sec. 2.2 (c_0 = 0, c_1..4 along the axes,
// c_5..8 along the diagonals; w = 4/9, 1/9, 1/36; c_s^2 = 1/3).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vp {

constexpr int Q = 9;

__host__ __device__ constexpr int cx(int a) {
  return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0);
}
__host__ __device__ constexpr int cy(int a) {
  return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp(int a) {
  return a == 0 ? 0 : (a <= 4 ? ((a + 1) % 4) + 1 : ((a - 5 + 2) % 4) + 5);
}
// population with the x (resp. y) velocity component reversed
__host__ __device__ constexpr int flipx(int a) {
  return a == 1 ? 3 : a == 3 ? 1 : a == 5 ? 6 : a == 6 ? 5 : a == 7 ? 8 : a == 8 ? 7 : a;
}
__host__ __device__ constexpr int flipy(int a) {
  return a == 2 ? 4 : a == 4 ? 2 : a == 5 ? 8 : a == 8 ? 5 : a == 6 ? 7 : a == 7 ? 6 : a;
}
__host__ __device__ constexpr double wgt(int a) {
  return a == 0 ? 4.0 / 9.0 : (a <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}

static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opp axis");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opp diag");

// mask byte layout
constexpr uint8_t M_BODY = 0x3F;    // body id 1..63 of a solid cell, 0 = fluid (chi = id != 0, Eq. fcar)
constexpr int MAX_BODIES = 63;
constexpr uint8_t M_SAMPLE = 0x40;  // stress-integration sample node
constexpr uint8_t M_IFACE = 0x80;   // a lattice neighbour has the other phase

enum { EDGE_PERIODIC = 0, EDGE_VELOCITY = 1, EDGE_FREESLIP = 2, EDGE_OUTFLOW = 3, EDGE_CONVECTIVE = 4 };

// Convective-edge state: the previous streamed value of each incoming
// population at each edge cell, [edge][slot][cell along the edge] with the
// west and east blocks ny long and the south and north blocks nx long.  The
// slot of a population is its velocity component along the edge (0, +1, -1).
// Population layout (array of structures of arrays): the 9 deviations of
// each run of 64 cells along a row are stored together, plane by plane, so
// one cell update touches 9 neighbouring 64-element blocks instead of 9
// planes a lattice apart.  Element (a, x, y), with pitch a multiple of 64:
//   ((y * (pitch / 64) + x / 64) * 9 + a) * 64 + x % 64,
// in 64 bits (a lattice may hold more than 2^31 elements; cells ny pitch <
// 2^31, so cell indices fit an int).
__host__ __device__ inline long long pop_index(int a, int x, int y, int pitch) {
  return (((long long)y * (pitch >> 6) + (x >> 6)) * Q + a) * 64 + (x & 63);
}
constexpr int CHUNK_ELEMS = 64 * 9;  // one run of 64 cells, all populations

// Index of a perimeter cell (x == 0, x == nx - 1, y == 0 or y == ny - 1):
// the west column, the east column, then the south and the north row
// without their corners; 2 ny + 2 (nx - 2) cells in all.
__host__ __device__ inline int perim_index(int x, int y, int nx, int ny) {
  if (x == 0) return y;
  if (x == nx - 1) return ny + y;
  if (y == 0) return 2 * ny + (x - 1);
  return 2 * ny + (nx - 2) + (x - 1);
}
__host__ __device__ inline int perim_count(int nx, int ny) { return 2 * ny + 2 * (nx - 2); }

__host__ __device__ constexpr int cbc_slot(int along) { return along == 0 ? 0 : (along > 0 ? 1 : 2); }
__host__ __device__ inline long long cbc_offset(int edge, int nx, int ny) {
  return edge < 2 ? (long long)edge * 3 * ny : 6LL * ny + (long long)(edge - 2) * 3 * nx;
}
enum { WEST = 0, EAST = 1, SOUTH = 2, NORTH = 3 };
enum { MODE_STATIC = 0, MODE_PRESCRIBED = 1, MODE_FREE = 2 };
enum { SHAPE_NONE = 0, SHAPE_DISK = 1, SHAPE_POLYGON = 2, SHAPE_MASK = 3 };

// storage of the deviations d_a = f_a - w_a rho0
// Store of v at the global-memory address base + bytes, base uniform.  The
// empty asm makes the optimizer take the base as it is, so each plane's
// store stays "scalar base + 32-bit lane offset" instead of being re-derived
// from the previous plane's address with 64-bit vector arithmetic.
#define VP_GLOBAL __attribute__((address_space(1)))
template <typename U> __device__ __forceinline__ void st_global(const void *base, uint32_t bytes, U v) {
  asm volatile("" : "+s"(base));
  *(VP_GLOBAL U *)((VP_GLOBAL const char *)base + bytes) = v;
}

template <typename S> struct Store;
template <> struct Store<double> {
  using T = double;
  static __device__ __forceinline__ double ld(const double *p) { return *p; }
  static __device__ __forceinline__ void st(double *p, double v) { *p = v; }
  static __device__ __forceinline__ void st_at(double *base, uint32_t bytes, double v) {
    st_global<double>(base, bytes, v);
  }
};
template <> struct Store<float> {
  using T = float;
  static __device__ __forceinline__ float ld(const float *p) { return *p; }
  static __device__ __forceinline__ void st(float *p, float v) { *p = v; }
  static __device__ __forceinline__ void st_at(float *base, uint32_t bytes, float v) {
    st_global<float>(base, bytes, v);
  }
};
template <> struct Store<__half> {
  using T = float;
  static __device__ __forceinline__ float ld(const __half *p) { return __half2float(*p); }
  static __device__ __forceinline__ void st(__half *p, float v) { *p = __float2half_rn(v); }
  static __device__ __forceinline__ void st_at(__half *base, uint32_t bytes, float v) {
    st_global<unsigned short>(base, bytes, __half_as_ushort(__float2half_rn(v)));
  }
};

// p advanced by a 32-bit byte offset (scalar base + per-lane offset addressing)
template <typename S> __device__ __forceinline__ S *at(S *p, uint32_t bytes) {
  return (S *)((char *)p + bytes);
}
template <typename S> __device__ __forceinline__ const S *at(const S *p, uint32_t bytes) {
  return (const S *)((const char *)p + bytes);
}


// c_a . (vx, vy) with the zero and unit components of c_a folded away
// (exactly the same value as the full dot product for finite inputs)
template <typename T> __device__ __forceinline__ T dotc(int a, T vx, T vy) {
  const int X = cx(a), Y = cy(a);
  if (X == 0 && Y == 0) return T(0);
  if (X == 0) return Y > 0 ? vy : -vy;
  if (Y == 0) return X > 0 ? vx : -vx;
  return (X > 0 ? vx : -vx) + (Y > 0 ? vy : -vy);
}

// 1/x.  FP32: the hardware reciprocal (1 ulp, not unbiased) refined by one
// Newton step r' = r + r (1 - x r), which removes the bias that would
// otherwise drift momentum over thousands of steps.  FP64: division.
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

struct BodyDev {
  double x, y, theta, u, v, omega;
};

// Device-resident control block (one per lattice).
// Per-body ranges of the force terms the finalize sums: interface slots
// [me0, me1) and stress-integration records [rec0, rec1).
struct BodyTab {
  int me0, me1, rec0, rec1;
};

struct Ctl {
  BodyDev body;        // body 1: state used by the next step (bodies 2.. are static, in a table)
  int win[4];          // cell window x0, y0, x1, y1 (exclusive) holding every
                       // interface and sample cell
  int region[4];       // last mask region rebuilt for a moving body
  int nrec;            // stress-integration records
  int nslot;           // interface cells (momentum-exchange slots)
  int nbody;           // bodies, ids 1..nbody
  int npts;            // registered stress-integration points
  int si_moving;       // points stored in the body frame
  int err;             // bit 0: a point without sample node; bit 1: a fluid cell
                       // linked to two bodies; bit 2: a sample node shared by two bodies;
                       // bit 3: interface slots exhausted; bit 4: a non-finite density
  long long step;      // steps completed since initialization
  double last[6];      // forces of body 1 in the last step: ME (Fx, Fy, T), SI (Fx, Fy, T)
  int mode, shape, source;
  int si_rule;         // 0: nearest fluid node along n; 1: interpolated at x + 1.5 n
  double r;            // disk radius
  double mass, inertia, gx, gy, buoy;
  long long fq[3];     // disk centre / radius on the 1/4096 grid (mask of the current state)
};

// Aggregated stress-integration weights of one sample node:
// F_x += s_xx ax + s_xy ay, F_y += s_xy ax + s_yy ay,
// T   += s_xx txx + s_xy txy + s_yy tyy.
struct SiRec {
  int cell;  // y * nx + x
  int pad;
  double ax, ay, txx, txy, tyy;
};

// A moving rigid disk (Eqs. dep1, theta2), stepped inside the step kernel:
// the step that uses state S computes the disk's solid cells, interface
// cells and sample nodes from S on the fly, inside a square window around
// it, and every tile of the window stores the sums of its cells' force
// terms (momentum exchange and stress integration); the next launch adds
// those partial sums into the step's forces and advances the state.  States
// alternate between two slots by the number of updates applied (see the step
// kernel).
constexpr int MAX_MOVERS = 4;
constexpr int WIN_MARGIN = 8;   // window half size = ceil(largest radius of disk and points) + WIN_MARGIN
constexpr int PART_ENTRY = 8;   // doubles per tile partial: ME Fx, Fy, T, SI Fx, Fy, T, -, -
constexpr int MOV_BX = 64, MOV_BY = 4;  // the tile of the moving-disk step kernels
struct MoverDev {
  BodyDev B[2];        // state after k updates in slot k & 1
  double r, mass, inertia, gx, gy, buoy;
  long long R;         // radius on the 1/FIXQ grid
  long long nfin;      // steps of this disk whose forces are in the history
  int mode, source;    // MODE_PRESCRIBED or MODE_FREE; force driving a free disk (0 ME, 1 SI)
  int half;            // window: (2 half + 1)^2 cells, lower corner at floor(x_G) - half
  int pt0, pt1;        // its stress-integration points [pt0, pt1) (body frame)
  int part0;           // its first tile partial in the partial buffers
  int ptx, pty;        // its partials: a grid of ptx x pty tiles (room for any window position)
  int mwin[4];         // mask bytes written by the last flush: x0, y0, x1, y1 (exclusive)
};

constexpr int ME_STRIDE = 4;    // doubles per interface slot (ME Fx, Fy, T of one cell)
constexpr int SIG_STRIDE = 4;   // doubles per stress slot of a sample node (xx, xy, yy)
constexpr int FIXQ = 4096;      // fixed-point grid of geometry coordinates

}  // namespace vp
