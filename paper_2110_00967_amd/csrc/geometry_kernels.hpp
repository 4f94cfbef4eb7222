// geometry_kernels.hpp -- device kernels around the step: initialization,
// solid indicator chi (Eq. fcar) for disks and polygons, interface flags,
// rigid-body update (Eqs. dep1, theta2), stress-integration sample nodes and
// weights (Sec. 2.3.2), one-shot stress integration, and readback staging.
#pragma once

#include "d2q9.hpp"
#include "step_kernel.hpp"

namespace vp {

// ----------------------------------------------------------------------------
// Post-collision deviation a of cell (x, y) in the layout `lay` the
// population buffer holds: 0, two buffers (slot a of the cell); 1, AA after
// an even launch or the initialization (slot opp(a) of the cell); 2, AA after
// an odd launch (slot a of x + c_a, or the perimeter copy ec when that
// leaves the lattice).  For readers that run between steps.
// ----------------------------------------------------------------------------
template <typename S>
__device__ __forceinline__ typename Store<S>::T load_post(const S *F, const S *ec, int lay, int nx, int ny,
                                                          int pitch, int nper, int x, int y, int a) {
  if (lay == 0) return Store<S>::ld(F + pop_index(a, x, y, pitch));
  if (lay == 1) return Store<S>::ld(F + pop_index(opp(a), x, y, pitch));
  const int tx = x + cx(a), ty = y + cy(a);
  if (tx >= 0 && tx < nx && ty >= 0 && ty < ny) return Store<S>::ld(F + pop_index(a, tx, ty, pitch));
  return Store<S>::ld(ec + (long long)a * nper + perim_index(x, y, nx, ny));
}

// The 9 deviations streaming into (x, y) from a post-collision state in any
// layout, with the edge rules and the convective blend (state not updated)
template <typename S, typename T>
__device__ __forceinline__ void pull_post(const S *F, const S *ec, int lay, const StepArgs<T> &P, int x, int y,
                                          T (&d)[Q]) {
  unsigned conv = 0;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    int pop, sx, sy;
    T add;
    bool cv;
    edge_source(P, x, y, a, pop, sx, sy, add, cv);
    d[a] = load_post(F, ec, lay, P.nx, P.ny, P.pitch, P.nper, sx, sy, pop) + add;
    conv |= cv ? 1u << a : 0u;
  }
#pragma unroll
  for (int a = 1; a < Q; ++a)
    if (conv >> a & 1u) d[a] = (*cbc_slot_ptr(P, x, y, a) + cbc_speed(P, x, a, false) * d[a]) * cbc_speed(P, x, a, true);
}

// ----------------------------------------------------------------------------
// initialization: d_a = f^eq_a(rho, u) - w_a rho0 (second-order equilibrium),
// stored in slot a (two buffers) or, for the AA pattern (swapped), in slot
// opp(a) with the perimeter copy in ec
// ----------------------------------------------------------------------------
template <typename S>
__global__ void k_init(S *__restrict__ f, const uint8_t *__restrict__ mask, int nx, int ny, int pitch,
                       int row0, int nrows, const double *__restrict__ rho_in,
                       const double *__restrict__ ux_in, const double *__restrict__ uy_in,
                       double rho_u, double ux_u, double uy_u, const Ctl *__restrict__ ctl, double rho0,
                       int swapped, S *__restrict__ ec, int nper) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int yl = blockIdx.y;
  if (x >= nx || yl >= nrows) return;
  const int y = row0 + yl;
  const long long c = (long long)y * pitch + x;
  double rho, ux, uy;
  if (rho_in) {
    const long long k = (long long)yl * nx + x;
    rho = rho_in[k];
    ux = ux_in[k];
    uy = uy_in[k];
  } else {
    rho = rho_u;
    ux = ux_u;
    uy = uy_u;
    if ((mask[c] & M_BODY) == 1) {  // body 1's cells start at its velocity (the others are static)
      const BodyDev B = ctl->body;
      ux = B.u - B.omega * (double(y) - B.y);
      uy = B.v + B.omega * (double(x) - B.x);
    }
  }
  const double uu = 1.5 * (ux * ux + uy * uy);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const double cu = cx(a) * ux + cy(a) * uy;
    const double d = wgt(a) * (rho - rho0) + wgt(a) * rho * (3.0 * cu + 4.5 * cu * cu - uu);
    Store<S>::st(f + pop_index(swapped ? opp(a) : a, x, y, pitch), (typename Store<S>::T)d);
    if (swapped && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1))
      Store<S>::st(ec + (long long)a * nper + perim_index(x, y, nx, ny), (typename Store<S>::T)d);
  }
}

// interface slots from (cell, slot) pairs numbered on the host
__global__ void k_scatter_slots(const int *__restrict__ pairs, int n, int *__restrict__ imap) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) imap[pairs[2 * k]] = pairs[2 * k + 1];
}

// convective-edge state <- the current populations entering through each
// convective edge (one thread per cell along an edge, all 4 edges)
template <typename S>
__global__ void k_cbc_init(const S *__restrict__ f, const StepArgs<typename Store<S>::T> P, int swapped) {
  using T = typename Store<S>::T;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, e = blockIdx.y;
  if (P.kind[e] != EDGE_CONVECTIVE) return;
  const int len = e < 2 ? P.ny : P.nx;
  if (i >= len) return;
  const int x = e == WEST ? 0 : (e == EAST ? P.nx - 1 : i);
  const int y = e == SOUTH ? 0 : (e == NORTH ? P.ny - 1 : i);
  const int in = (e == WEST || e == SOUTH) ? 1 : -1;  // inward component along the normal
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    const int cn = e < 2 ? cx(a) : cy(a), ca = e < 2 ? cy(a) : cx(a);
    if (cn != in) continue;
    P.cbc[cbc_offset(e, P.nx, P.ny) + (long long)cbc_slot(ca) * len + i] =
        T(Store<S>::ld(f + pop_index(swapped ? opp(a) : a, x, y, P.pitch)));
  }
}

// post-collision populations f_a = w_a rho0 + d_a of the window columns
// [x0, x0 + w), rows [row0, row0 + nrows) -> out[9][nrows][w] (layouts as in
// load_post)
template <typename S>
__global__ void k_read_pop(const S *__restrict__ f, const S *__restrict__ ec, int lay, int nx, int ny, int nper,
                           int x0, int w, int pitch, int row0, int nrows, double rho0,
                           double *__restrict__ out) {
  const int xl = blockIdx.x * blockDim.x + threadIdx.x;
  const int yl = blockIdx.y;
  if (xl >= w || yl >= nrows) return;
#pragma unroll
  for (int a = 0; a < Q; ++a)
    out[((long long)a * nrows + yl) * w + xl] =
        wgt(a) * rho0 + double(load_post(f, ec, lay, nx, ny, pitch, nper, x0 + xl, row0 + yl, a));
}

template <typename T>
__global__ void k_read_macro(const T *__restrict__ r, const T *__restrict__ u, const T *__restrict__ v,
                             int x0, int w, int pitch, int row0, int nrows, double *__restrict__ out) {
  const int xl = blockIdx.x * blockDim.x + threadIdx.x;
  const int yl = blockIdx.y;
  if (xl >= w || yl >= nrows) return;
  const long long c = (long long)(row0 + yl) * pitch + x0 + xl;
  const long long o = (long long)yl * w + xl;
  const long long n = (long long)nrows * w;
  out[o] = double(r[c]);
  out[n + o] = double(u[c]);
  out[2 * n + o] = double(v[c]);
}

// ----------------------------------------------------------------------------
// chi: exact inside tests on the 1/4096 grid (integer arithmetic)
// ----------------------------------------------------------------------------
__device__ __forceinline__ bool disk_inside(long long X, long long Y, long long R, int i, int j) {
  const long long dx = (long long)i * FIXQ - X, dy = (long long)j * FIXQ - Y;
  return dx * dx + dy * dy <= R * R;
}

// even-odd rule; a centre exactly on an edge counts as inside
__device__ __forceinline__ bool polygon_inside(const long long *__restrict__ vx,
                                               const long long *__restrict__ vy, int nv, int i, int j) {
  const long long px = (long long)i * FIXQ, py = (long long)j * FIXQ;
  bool in = false;
  long long ax = vx[nv - 1], ay = vy[nv - 1];
  for (int e = 0; e < nv; ++e) {
    const long long bx = vx[e], by = vy[e];
    const long long orient = (ax - bx) * (py - by) - (ay - by) * (px - bx);
    // orient is the cross product of (a - b) and (p - b): zero when p is on the line
    if (orient == 0 && px >= min(ax, bx) && px <= max(ax, bx) && py >= min(ay, by) &&
        py <= max(ay, by))
      return true;
    if ((by > py) != (ay > py)) {
      // the edge b -> a crosses the horizontal through p right of p when the
      // orientation has the sign of (ay - by)
      if ((orient > 0) == (ay > by)) in = !in;
    }
    ax = bx;
    ay = by;
  }
  return in;
}

// rewrite mask bytes of a region from a disk: bit 0 = inside; flags cleared
__global__ void k_mask_disk(uint8_t *__restrict__ mask, int pitch, int x0, int y0, int x1, int y1,
                            long long X, long long Y, long long R) {
  const int i = x0 + blockIdx.x * blockDim.x + threadIdx.x;
  const int j = y0 + blockIdx.y;
  if (i >= x1 || j >= y1) return;
  mask[(long long)j * pitch + i] = disk_inside(X, Y, R, i, j) ? 1 : 0;  // body 1
}

__global__ void k_mask_polygon(uint8_t *__restrict__ mask, int pitch, int x0, int y0, int x1, int y1,
                               const long long *__restrict__ vx, const long long *__restrict__ vy,
                               int nv) {
  const int i = x0 + blockIdx.x * blockDim.x + threadIdx.x;
  const int j = y0 + blockIdx.y;
  if (i >= x1 || j >= y1) return;
  mask[(long long)j * pitch + i] = polygon_inside(vx, vy, nv, i, j) ? 1 : 0;  // body 1
}

// interface bit over a region: some lattice neighbour (periodic edges wrap,
// none beyond other edges) has the other phase; keeps the body id, clears
// the sample bit.  A fluid cell linked to two different bodies sets bit 1
// of *err (its links could not be attributed to one body).
__global__ void k_mask_flags(uint8_t *__restrict__ mask, int nx, int ny, int pitch, int x0, int y0,
                             int x1, int y1, int perx, int pery, int *__restrict__ err) {
  const int i = x0 + blockIdx.x * blockDim.x + threadIdx.x;
  const int j = y0 + blockIdx.y;
  if (i >= x1 || j >= y1) return;
  const long long c = (long long)j * pitch + i;
  const int own = mask[c] & M_BODY;
  bool iface = false;
  int other = 0;
  bool two = false;
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    int X = i + cx(a), Y = j + cy(a);
    if (X < 0 || X >= nx) {
      if (!perx) continue;
      X = X < 0 ? X + nx : X - nx;
    }
    if (Y < 0 || Y >= ny) {
      if (!pery) continue;
      Y = Y < 0 ? Y + ny : Y - ny;
    }
    const int nid = mask[(long long)Y * pitch + X] & M_BODY;
    if ((nid != 0) != (own != 0)) iface = true;
    if (!own && nid) {
      two = two || (other && other != nid);
      other = nid;
    }
  }
  if (two) atomicOr(err, 2);
  mask[c] = (uint8_t)(own | (iface ? M_IFACE : 0));
}

// ----------------------------------------------------------------------------
// stress-integration sample nodes and aggregated weights (one workgroup)
// ----------------------------------------------------------------------------
constexpr int SI_NT = 1024;
constexpr int SI_MAX = 4096;

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
  double sc[Q];
  sc[1] = n0;
  sc[2] = n1;
  sc[3] = -n0;
  sc[4] = -n1;
  sc[5] = (n0 + n1) * S;
  sc[6] = (-n0 + n1) * S;
  sc[7] = (-n0 - n1) * S;
  sc[8] = (n0 - n1) * S;
  int best = 1;
#pragma unroll
  for (int a = 2; a < Q; ++a)
    if (sc[a] > sc[best]) best = a;
  int bx = 0, by = 0;
#pragma unroll
  for (int a = 1; a < Q; ++a)
    if (a == best) { bx = cx(a); by = cy(a); }
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

// Point threadIdx.x (position, normal, body), loaded ahead by a caller that
// has other work to overlap with the loads; ok = false when not loaded.
struct PtPre {
  double a, b, c, d, ds, body;
  bool ok;
};

__device__ __forceinline__ PtPre si_prefetch(const double *__restrict__ pts, int maxp, int npts) {
  PtPre p{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, false};
  const int i = threadIdx.x;
  if (i < npts) {
    p.a = pts[i];
    p.b = pts[maxp + i];
    p.c = pts[2 * maxp + i];
    p.d = pts[3 * maxp + i];
    p.ds = pts[4 * maxp + i];
    p.body = pts[5 * maxp + i];
    p.ok = true;
  }
  return p;
}

// exclusive prefix sum over the SI_NT threads of the block; *total gets the sum
__device__ __forceinline__ int block_exclusive_scan(int v, int *wsum /*[SI_NT/64]*/, int *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(incl, off, 64);
    if (lane >= off) incl += u;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < SI_NT / 64; ++w) {
      const int t = wsum[w];
      wsum[w] = run;
      run += t;
    }
    *total = run;
  }
  __syncthreads();
  return wsum[wave] + incl - v;
}

// Bitonic sort of key[0, N), N a power of two <= SI_MAX, by the SI_NT threads
// of the block; on return key[] holds the sorted keys.  Element e lives in a
// register of thread e % SI_NT (register e / SI_NT), so the compare-exchange
// partner e ^ stride is: for stride < 64, a lane of the same wave (a
// shuffle, no barrier); for stride >= SI_NT, another register of the same
// thread; in between, another wave (through LDS, two barriers).
__device__ __forceinline__ void block_bitonic_sort(unsigned long long *key, int N) {
  constexpr int NJ = SI_MAX / SI_NT;
  unsigned long long v[NJ];
  const int tid = threadIdx.x, lane = tid & 63;
  const int nj = N > SI_NT ? N / SI_NT : 1;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int e = tid + j * SI_NT;
    v[j] = (j < nj && e < N) ? key[e] : ~0ull;  // lanes beyond N only meet each other
  }
  for (int size = 2; size <= N; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= SI_NT) {
        // register pairs (j, j ^ js); both indices compile-time after unrolling
        const int js = stride / SI_NT;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
#pragma unroll
          for (int jp = j + 1; jp < NJ; ++jp) {
            if ((j ^ jp) == js && jp < nj) {
              const bool up = ((tid + j * SI_NT) & size) == 0;
              const unsigned long long a = v[j], b = v[jp];
              if ((a > b) == up) {
                v[j] = b;
                v[jp] = a;
              }
            }
          }
        }
      } else if (stride >= 64) {
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          if (j < nj) key[tid + j * SI_NT] = v[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int e = tid + j * SI_NT;
          if (j < nj && e < N) {
            const unsigned long long p = key[e ^ stride];
            const bool keep_min = ((e & stride) == 0) == ((e & size) == 0);
            v[j] = keep_min ? (v[j] < p ? v[j] : p) : (v[j] < p ? p : v[j]);
          }
        }
        __syncthreads();
      } else {
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          // N >= 64 here (N <= RANK_SORT_MAX goes to block_rank_sort), so a
          // wave holds N's elements entirely or not at all
          if (j >= nj || (tid & ~63) + j * SI_NT >= N) continue;
          const unsigned long long p = __shfl_xor(v[j], stride, 64);
          const int e = tid + j * SI_NT;
          const bool keep_min = ((lane & stride) == 0) == ((e & size) == 0);
          v[j] = keep_min ? (v[j] < p ? v[j] : p) : (v[j] < p ? p : v[j]);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int e = tid + j * SI_NT;
    if (j < nj && e < N) key[e] = v[j];
  }
  __syncthreads();
}

// Sort of key[0, N), N <= RANK_SORT_MAX <= SI_NT, by ranks: element t goes to
// the number of keys below it (ties by index).  One pass of broadcast LDS
// reads instead of the log^2 N stages of the bitonic network.
constexpr int RANK_SORT_MAX = 256;
__device__ __forceinline__ void block_rank_sort(unsigned long long *key, int N) {
  const int t = threadIdx.x;
  unsigned long long k = 0;
  int r = 0;
  if (t < N) {
    k = key[t];
    for (int j = 0; j < N; ++j) {
      const unsigned long long q = key[j];
      r += (q < k) | ((q == k) & (j < t));
    }
  }
  __syncthreads();
  if (t < N) key[r] = k;
  __syncthreads();
}

__device__ __forceinline__ void block_sort_keys(unsigned long long *key, int N) {
  if (N <= RANK_SORT_MAX)
    block_rank_sort(key, N);
  else
    block_bitonic_sort(key, N);
}

// Sample nodes and per-node weights of all registered points (one workgroup
// of SI_NT threads; called by k_si_select and, for a moving disk, at the end
// of k_body_step after the mask was rebuilt).  solid: the solid test the
// sample-node search uses (see MaskSolid, DiskSolid).  npts, moving, rule
// and B are the control block's point count, point frame flag, stencil rule
// and body-1 state, passed in by the caller with co, sn = cos, sin of
// B.theta (1, 0 for points stored in the world frame).  stage (LDS, 5 x stage_pts
// doubles, or null) keeps the world position, normal and length of points
// below stage_pts from the key pass for the record pass.  check_shared:
// flag a sample node claimed by two bodies (error bit 2); a lattice with a
// single body cannot have one.
template <typename Solid>
__device__ __forceinline__ void si_select_block(const Solid &solid, const PtPre &pre, uint8_t *__restrict__ mask,
                                                Ctl *__restrict__ ctl,
                                const double *__restrict__ pts, int maxp, SiRec *__restrict__ recs,
                                int *__restrict__ si_map, BodyTab *__restrict__ bt,
                                const BodyDev *__restrict__ bodies, int nx, int ny, int pitch, const int npts,
                                const int moving, const int rule, const BodyDev &B, const double co,
                                const double sn, double *stage, int stage_pts, bool check_shared,
                                const int *win_now = nullptr) {
  // key = (body, node, entry): records come out grouped by body, then by node
  constexpr int NODE_SHIFT = 14, BODY_SHIFT = 45;  // entry < 2^14, node < 2^31
  __shared__ unsigned long long key[SI_MAX];
  __shared__ unsigned char recbody[SI_MAX];
  __shared__ int wsum[SI_NT / 64];
  __shared__ int nrec_total;
  __shared__ int bb[4];
  __shared__ int missing, shared_node;
  const int per_pt = rule == 1 ? 4 : 1;  // stencil entries per point
  const int nent = npts * per_pt;
  int N = 4;  // >= per_pt, so every key slot below is written
  while (N < nent) N <<= 1;
  if (threadIdx.x == 0) {
    bb[0] = nx; bb[1] = ny; bb[2] = -1; bb[3] = -1;
    missing = 0;
    shared_node = 0;
  }
  if (threadIdx.x < MAX_BODIES) {
    bt[threadIdx.x].rec0 = 0;
    bt[threadIdx.x].rec1 = 0;
  }
  __syncthreads();
  // one key per stencil entry; entry = point * per_pt + k.  The sample
  // nodes' bounding box is reduced per wave, then merged in LDS.
  int bx0 = nx, by0 = ny, bx1 = -1, by1 = -1;
  for (int i = threadIdx.x; i < N / per_pt; i += SI_NT) {
    unsigned long long kk[4] = {~0ull, ~0ull, ~0ull, ~0ull};
    if (i < npts) {
      double px, py, n0, n1;
      unsigned long long body;
      double ds;
      if (pre.ok && i == (int)threadIdx.x) {
        si_place(pre.a, pre.b, pre.c, pre.d, moving, B, co, sn, px, py, n0, n1);
        body = (unsigned long long)pre.body;
        ds = pre.ds;
      } else {
        si_world(pts, maxp, i, moving, B, co, sn, px, py, n0, n1);
        body = (unsigned long long)pts[5 * maxp + i];
        ds = stage ? pts[4 * maxp + i] : 0.0;
      }
      if (stage && i < stage_pts) {
        stage[i] = px;
        stage[stage_pts + i] = py;
        stage[2 * stage_pts + i] = n0;
        stage[3 * stage_pts + i] = n1;
        stage[4 * stage_pts + i] = ds;
      }
      int node[4];
      double w[4];
      const int c = si_stencil(solid, nx, ny, rule, px, py, n0, n1, node, w);
      if (c == 0) atomicAdd(&missing, 1);
      for (int k = 0; k < c; ++k) {
        kk[k] = (body << BODY_SHIFT) | ((unsigned long long)(unsigned)node[k] << NODE_SHIFT) |
                (unsigned)(i * per_pt + k);
        const int X = node[k] % nx, Y = node[k] / nx;
        bx0 = min(bx0, X);
        by0 = min(by0, Y);
        bx1 = max(bx1, X);
        by1 = max(by1, Y);
      }
    }
    for (int k = 0; k < per_pt; ++k) key[i * per_pt + k] = kk[k];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    bx0 = min(bx0, __shfl_xor(bx0, off, 64));
    by0 = min(by0, __shfl_xor(by0, off, 64));
    bx1 = max(bx1, __shfl_xor(bx1, off, 64));
    by1 = max(by1, __shfl_xor(by1, off, 64));
  }
  if ((threadIdx.x & 63) == 0 && bx1 >= 0) {
    atomicMin(&bb[0], bx0);
    atomicMin(&bb[1], by0);
    atomicMax(&bb[2], bx1);
    atomicMax(&bb[3], by1);
  }
  __syncthreads();
  block_sort_keys(key, N);
  // segment heads (one record per body and node) -> record indices (each
  // thread owns a contiguous chunk)
  const unsigned long long INVALID = ~0ull;
  auto group = [&](int j) { return key[j] >> NODE_SHIFT; };  // (body, node)
  const int per = (N + SI_NT - 1) / SI_NT;
  const int j0 = threadIdx.x * per, j1 = min(j0 + per, N);
  int cnt = 0;
  for (int j = j0; j < j1; ++j)
    if (key[j] != INVALID && (j == 0 || group(j - 1) != group(j))) ++cnt;
  int r = block_exclusive_scan(cnt, wsum, &nrec_total);
  for (int j = j0; j < j1; ++j) {
    if (key[j] == INVALID || (j > 0 && group(j - 1) == group(j))) continue;
    const int body = (int)(key[j] >> BODY_SHIFT);
    const unsigned node = (unsigned)((key[j] >> NODE_SHIFT) & 0x7FFFFFFFu);
    const BodyDev Bb = body <= 1 ? B : bodies[body];  // torque reference of the record's body
    double ax = 0.0, ay = 0.0, txx = 0.0, txy = 0.0, tyy = 0.0;
    for (int k = j; k < N && key[k] != INVALID && group(k) == group(j); ++k) {
      const int e = (int)(key[k] & ((1u << NODE_SHIFT) - 1));
      const int i = e / per_pt;
      double px, py, n0, n1, ds;
      if (stage && i < stage_pts) {
        px = stage[i];
        py = stage[stage_pts + i];
        n0 = stage[2 * stage_pts + i];
        n1 = stage[3 * stage_pts + i];
        ds = stage[4 * stage_pts + i];
      } else {
        si_world(pts, maxp, i, moving, B, co, sn, px, py, n0, n1);
        ds = pts[4 * maxp + i];
      }
      int nd[4];
      double w[4];
      si_stencil(solid, nx, ny, rule, px, py, n0, n1, nd, w);
      const int ke = e % per_pt;
      double we = w[0];
#pragma unroll
      for (int k = 1; k < 4; ++k)
        if (k == ke) we = w[k];  // register select (no indexed private array)
      const double s = ds * we;
      const double rx = px - Bb.x, ry = py - Bb.y;
      ax += s * n0;
      ay += s * n1;
      txx += s * (-ry * n0);
      txy += s * (rx * n0 - ry * n1);
      tyy += s * (rx * n1);
    }
    SiRec R;
    R.cell = (int)node;
    R.pad = 0;
    R.ax = ax; R.ay = ay; R.txx = txx; R.txy = txy; R.tyy = tyy;
    recs[r] = R;
    recbody[r] = (unsigned char)body;
    const int X = (int)node % nx, Y = (int)node / nx;
    const long long cc = (long long)Y * pitch + X;
    si_map[cc] = r;
    // sample bit (a node sampled for two bodies would need two slots)
    unsigned *wd = (unsigned *)(mask + (cc & ~3LL));
    const unsigned bit = (unsigned)M_SAMPLE << (8 * (cc & 3));
    if (check_shared) {
      if (atomicOr(wd, bit) & bit) atomicOr(&shared_node, 1);
    } else {
      atomicOr(wd, bit);
    }
    ++r;
  }
  __syncthreads();
  // each body's record range (records are grouped by body)
  for (int k = threadIdx.x; k < nrec_total; k += SI_NT) {
    const int b = recbody[k] - 1;
    if (k == 0 || recbody[k - 1] != recbody[k]) bt[b].rec0 = k;
    if (k == nrec_total - 1 || recbody[k + 1] != recbody[k]) bt[b].rec1 = k + 1;
  }
  if (threadIdx.x == 0) {
    ctl->nrec = nrec_total;
    if (missing) ctl->err |= 1;
    if (shared_node) ctl->err |= 4;
    if (bb[2] >= 0) {
      // the force window so far (win_now: the caller's copy of what it wrote)
      int wn[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) wn[k] = win_now ? win_now[k] : ctl->win[k];
      if (wn[2] <= wn[0] || wn[3] <= wn[1]) {
        ctl->win[0] = bb[0]; ctl->win[1] = bb[1]; ctl->win[2] = bb[2] + 1; ctl->win[3] = bb[3] + 1;
      } else {
        ctl->win[0] = min(wn[0], bb[0]);
        ctl->win[1] = min(wn[1], bb[1]);
        ctl->win[2] = max(wn[2], bb[2] + 1);
        ctl->win[3] = max(wn[3], bb[3] + 1);
      }
    }
  }
}

__global__ void __launch_bounds__(SI_NT)
    k_si_select(uint8_t *__restrict__ mask, Ctl *__restrict__ ctl, const double *__restrict__ pts,
                int maxp, SiRec *__restrict__ recs, int *__restrict__ si_map, BodyTab *__restrict__ bt,
                const BodyDev *__restrict__ bodies, int nx, int ny, int pitch) {
  const BodyDev B = ctl->body;
  const int moving = ctl->si_moving;
  const double co = moving ? cos(B.theta) : 1.0, sn = moving ? sin(B.theta) : 0.0;
  si_select_block(MaskSolid{mask, pitch}, PtPre{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, false}, mask, ctl, pts, maxp, recs,
                  si_map, bt, bodies, nx, ny, pitch, ctl->npts, moving, ctl->si_rule, B, co, sn, nullptr, 0, true);
}

// ----------------------------------------------------------------------------
// moving disk: rigid-body update, then rebuild chi and flags over the union of
// the old and new regions (one workgroup)
// ----------------------------------------------------------------------------
constexpr int BODY_NT = 1024;
constexpr int INSIDE_LDS = 32768;  // bytes of disk tests the body kernel stages in LDS
constexpr int REGION_MARGIN = 6;  // covers links (1) and sample walks (5)

__device__ __forceinline__ void body_step_block(uint8_t *__restrict__ mask, Ctl *__restrict__ ctl,
                                const double *__restrict__ me, const double *__restrict__ sig,
                                double *__restrict__ hist, int cap, int maxb, int nx, int ny, int pitch,
                                int perx, int pery, const double *__restrict__ pts, int maxp,
                                SiRec *__restrict__ recs, int *__restrict__ si_map, int *__restrict__ imap,
                                int maxslot, BodyTab *__restrict__ bt, const BodyDev *__restrict__ bodies) {
  static_assert(BODY_NT == SI_NT, "the block scan assumes SI_NT threads");
  __shared__ int reg[4];   // union region to rewrite
  __shared__ long long q[3];
  __shared__ double lds[FIN_WAVES * 6];
  __shared__ int wsum[BODY_NT / 64];
  __shared__ int nslot;
  __shared__ double flast[6];  // forces of the step just taken (ME, SI)
  __shared__ BodyDev Bnew;     // body state after the update
  __shared__ double cs[2];     // cos, sin of its angle (for points in the body frame)
  __shared__ int winsh[4];     // force window written by the update
  // disk tests of the rebuild, then the points staged by the sample selection
  __shared__ double lds_stage[INSIDE_LDS / sizeof(double)];
  uint8_t *inside = (uint8_t *)lds_stage;
  // Loads that do not depend on the finalize, issued first so their latency
  // overlaps it: the control-block fields of the update (the finalize does
  // not write them) and this thread's stress-integration point.
  const BodyDev B0 = ctl->body;
  const int mode = ctl->mode, source = ctl->source;
  const double mass = ctl->mass, inertia = ctl->inertia, buoy = ctl->buoy, cgx = ctl->gx, cgy = ctl->gy;
  const double crad = ctl->r;
  const int oreg0 = ctl->region[0], oreg1 = ctl->region[1], oreg2 = ctl->region[2], oreg3 = ctl->region[3];
  const int npts0 = ctl->npts, si_moving = ctl->si_moving, si_rule = ctl->si_rule;
  const PtPre pre = si_prefetch(pts, maxp, npts0);
  // the finalize's first slot and record per virtual lane, loaded with the
  // control block instead of after the slot ranges (the disk is body 1 and
  // the only body: its ranges start at 0; records fit maxp at least)
  FinPre fp;
  fp.me_ok = false;
  fp.rec_ok = false;
  if (threadIdx.x < FIN_W) {
    const int t = threadIdx.x;
    if (t < maxslot) {
#pragma unroll
      for (int i = 0; i < 3; ++i) fp.me[i] = me[(long long)t * ME_STRIDE + i];
      fp.me_ok = true;
    }
    if (t < maxp) {
#pragma unroll
      for (int i = 0; i < 3; ++i) fp.g[i] = sig[(long long)t * SIG_STRIDE + i];
      fp.R = recs[t];
      fp.rec_ok = true;
    }
  }
  // forces of the step just taken, needed by the update below (the only
  // body: a moving disk is alone in its lattice)
  finalize_block<BODY_NT>(me, sig, recs, bt, ctl, hist, cap, maxb, lds, flast, &fp);
  __syncthreads();
  if (threadIdx.x == 0) {
    BodyDev B = B0;
    if (mode == MODE_FREE) {
      // Eqs. dep1/theta2, semi-implicit Euler, dt = 1
      const double *F = flast + 3 * source;
      B.u += F[0] / mass + buoy * cgx;
      B.v += F[1] / mass + buoy * cgy;
      B.omega += F[2] / inertia;
    }
    B.x += B.u;
    B.y += B.v;
    B.theta += B.omega;
    ctl->body = B;
    Bnew = B;
    const long long X = llround(B.x * FIXQ), Y = llround(B.y * FIXQ), R = llround(crad * FIXQ);
    ctl->fq[0] = X;
    ctl->fq[1] = Y;
    ctl->fq[2] = R;
    q[0] = X;
    q[1] = Y;
    q[2] = R;
    // bounding box of the disk (cells whose centre can be inside)
    const int bx0 = (int)((X - R) / FIXQ) - 1, bx1 = (int)((X + R) / FIXQ) + 2;
    const int by0 = (int)((Y - R) / FIXQ) - 1, by1 = (int)((Y + R) / FIXQ) + 2;
    int nr[4] = {max(bx0 - REGION_MARGIN, 0), max(by0 - REGION_MARGIN, 0),
                 min(bx1 + REGION_MARGIN, nx), min(by1 + REGION_MARGIN, ny)};
    reg[0] = min(nr[0], oreg0);
    reg[1] = min(nr[1], oreg1);
    reg[2] = max(nr[2], oreg2);
    reg[3] = max(nr[3], oreg3);
#pragma unroll
    for (int k = 0; k < 4; ++k) ctl->region[k] = nr[k];
    // force window: interface cells lie within one cell of the disk's box;
    // the sample-node selection extends it afterwards
    int wn[4] = {max(bx0 - 1, 0), max(by0 - 1, 0), min(bx1 + 1, nx), min(by1 + 1, ny)};
    if (wn[2] <= wn[0] || wn[3] <= wn[1]) {
      // body outside the lattice: keep a one-cell window so forces are still published
      wn[0] = wn[1] = 0;
      wn[2] = wn[3] = 1;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      ctl->win[k] = wn[k];
      winsh[k] = wn[k];
    }
  } else if (threadIdx.x == 64) {
    // the new angle as thread 0 forms it, and its cos and sin (in another
    // wave, in parallel with the update)
    double om = B0.omega;
    if (mode == MODE_FREE) om += flast[3 * source + 2] / inertia;
    const double th = B0.theta + om;
    cs[0] = si_moving ? cos(th) : 1.0;
    cs[1] = si_moving ? sin(th) : 0.0;
  }
  __syncthreads();
  const int x0 = reg[0], y0 = reg[1], w = reg[2] - reg[0], h = reg[3] - reg[1];
  const long long X = q[0], Y = q[1], R = q[2];
  // this thread's cells are t = threadIdx.x + k BODY_NT; bit k of ifbits
  // records an interface cell (rounds past 64 read the mask back)
  unsigned long long ifbits = 0;
  int cnt = 0;
  // the disk test of every cell of the region and a one-cell ring around it
  // (neighbours wrapped across periodic edges; 2 = no such neighbour), once
  // per cell in LDS when it fits, instead of once per link
  const int W2 = w + 2, H2 = h + 2;
  const bool staged = W2 * H2 <= INSIDE_LDS;
  if (staged) {
    for (int t = threadIdx.x; t < W2 * H2; t += BODY_NT) {
      int I = x0 - 1 + t % W2, J = y0 - 1 + t / W2;
      bool there = true;
      if (I < 0 || I >= nx) {
        there = perx != 0;
        I = I < 0 ? I + nx : I - nx;
      }
      if (J < 0 || J >= ny) {
        there = there && pery != 0;
        J = J < 0 ? J + ny : J - ny;
      }
      inside[t] = there ? (disk_inside(X, Y, R, I, J) ? 1 : 0) : 2;
    }
    __syncthreads();
  }
  for (int t = threadIdx.x, k = 0; t < w * h; t += BODY_NT, ++k) {
    const int i = x0 + t % w, j = y0 + t / w;
    bool own, iface = false;
    if (staged) {
      const int c = (t / w + 1) * W2 + t % w + 1;
      own = inside[c] == 1;
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        const uint8_t nb = inside[c + cy(a) * W2 + cx(a)];
        if (nb != 2 && (nb == 1) != own) iface = true;
      }
    } else {
      own = disk_inside(X, Y, R, i, j);
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        int I = i + cx(a), J = j + cy(a);
        if (I < 0 || I >= nx) {
          if (!perx) continue;
          I = I < 0 ? I + nx : I - nx;
        }
        if (J < 0 || J >= ny) {
          if (!pery) continue;
          J = J < 0 ? J + ny : J - ny;
        }
        if (disk_inside(X, Y, R, I, J) != own) iface = true;
      }
    }
    mask[(long long)j * pitch + i] = (own ? 1 : 0) | (iface ? M_IFACE : 0);
    if (iface) {
      ++cnt;
      if (k < 64) ifbits |= 1ull << k;
    }
  }
  // the rebuilt mask must be visible to every thread of the block
  __threadfence_block();
  __syncthreads();
  {
    // interface slots, thread by thread and each thread's cells in order (all
    // of the disk's interface cells lie in its region).  A slot beyond the
    // capacity drops its interface bit and flags the error (bit 3) instead of
    // writing out of bounds.
    int slot = block_exclusive_scan(cnt, wsum, &nslot);
    for (int t = threadIdx.x, k = 0; t < w * h; t += BODY_NT, ++k) {
      const long long c = (long long)(y0 + t / w) * pitch + x0 + t % w;
      if (!(k < 64 ? (ifbits >> k) & 1 : (mask[c] & M_IFACE))) continue;
      if (slot < maxslot) {
        imap[c] = slot;
      } else {
        mask[c] &= (uint8_t)~M_IFACE;
        atomicOr(&ctl->err, 8);
      }
      ++slot;
    }
    if (threadIdx.x == 0) {
      ctl->nslot = min(nslot, maxslot);
      bt[0].me0 = 0;
      bt[0].me1 = min(nslot, maxslot);
    }
  }
  if (npts0 > 0) {
    __threadfence_block();
    __syncthreads();
    // the disk is the lattice's only body: its rule is the mask just built
    si_select_block(DiskSolid{q[0], q[1], q[2]}, pre, mask, ctl, pts, maxp, recs, si_map, bt, bodies, nx, ny, pitch,
                    npts0, si_moving, si_rule, Bnew, cs[0], cs[1], lds_stage,
                    (int)(INSIDE_LDS / sizeof(double) / 5), false, winsh);
  }
}

__global__ void __launch_bounds__(BODY_NT)
    k_body_step(uint8_t *__restrict__ mask, Ctl *__restrict__ ctl, const double *__restrict__ me,
                const double *__restrict__ sig, double *__restrict__ hist, int cap, int maxb, int nx, int ny,
                int pitch, int perx, int pery, const double *__restrict__ pts, int maxp, SiRec *__restrict__ recs,
                int *__restrict__ si_map, int *__restrict__ imap, int maxslot, BodyTab *__restrict__ bt,
                const BodyDev *__restrict__ bodies) {
  body_step_block(mask, ctl, me, sig, hist, cap, maxb, nx, ny, pitch, perx, pery, pts, maxp, recs, si_map, imap,
                  maxslot, bt, bodies);
}

// body kernel of a batched launch: one workgroup per moving lattice
template <typename T>
__global__ void __launch_bounds__(BODY_NT)
    k_body_step_batch(const CaseDesc<T> *__restrict__ cases, const int *__restrict__ moving, int flip) {
  const CaseDesc<T> &C = cases[moving[blockIdx.x]];
  body_step_block(C.mask, C.ctl, C.me[C.pbit0 ^ flip], C.sig[C.pbit0 ^ flip], C.hist, C.cap, C.maxb, C.P.nx,
                  C.P.ny, C.P.pitch, C.perx, C.pery, C.pts, C.maxp, const_cast<SiRec *>(C.recs),
                  const_cast<int *>(C.si_map), const_cast<int *>(C.imap), C.maxslot, C.bt, C.P.bodies);
}

// ----------------------------------------------------------------------------
// one-shot stress integration over given world points on the populations
// streamed from the current post-collision state (one workgroup)
// ----------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(SI_NT)
    k_si_at(const S *__restrict__ fin, const S *__restrict__ ec, int lay, const uint8_t *__restrict__ mask,
            const StepArgs<typename Store<S>::T> P, const Ctl *__restrict__ ctl,
            const double *__restrict__ pts, int maxp, int npts, double *__restrict__ out) {
  using T = typename Store<S>::T;
  const BodyDev B = ctl->body;
  const int rule = ctl->si_rule;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < npts; i += SI_NT) {
    const double px = pts[i], py = pts[maxp + i], n0 = pts[2 * maxp + i], n1 = pts[3 * maxp + i];
    const double s = pts[4 * maxp + i];
    int nodes[4];
    double wts[4];
    const int cnt = si_stencil(MaskSolid{mask, P.pitch}, P.nx, P.ny, rule, px, py, n0, n1, nodes, wts);
    if (cnt == 0) {
      v[5] += 1.0;  // counts points without a sample node
      continue;
    }
    double sxx = 0.0, sxy = 0.0, syy = 0.0;
    for (int q = 0; q < cnt; ++q) {
      const int x = nodes[q] % P.nx, y = nodes[q] / P.nx;
      double d[Q];
      {
        T dt[Q];
        if (lay == 0)
          pull_edge_all<S, T, false>(fin, P, x, y, dt);
        else
          pull_post<S, T>(fin, ec, lay, P, x, y, dt);
#pragma unroll
        for (int a = 0; a < Q; ++a) d[a] = double(dt[a]);
      }
      double drho = 0.0, mx = 0.0, my = 0.0;
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        drho += d[a];
        mx += cx(a) * d[a];
        my += cy(a) * d[a];
      }
      const double rho = P.rho0d + drho;
      const double ux = (mx + 0.5 * double(P.gx)) / rho, uy = (my + 0.5 * double(P.gy)) / rho;
      const double uu = 1.5 * (ux * ux + uy * uy);
      double pxx = 0.0, pxy = 0.0, pyy = 0.0;
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        const double cu = cx(a) * ux + cy(a) * uy;
        const double deq = wgt(a) * drho + wgt(a) * rho * (3.0 * cu + 4.5 * cu * cu - uu);
        const double ne = d[a] - deq;
        pxx += cx(a) * cx(a) * ne;
        pxy += cx(a) * cy(a) * ne;
        pyy += cy(a) * cy(a) * ne;
      }
      const double pr = drho / 3.0;
      sxx += wts[q] * (-pr - P.facd * pxx);
      sxy += wts[q] * (-P.facd * pxy);
      syy += wts[q] * (-pr - P.facd * pyy);
    }
    const double tx = s * (sxx * n0 + sxy * n1), ty = s * (sxy * n0 + syy * n1);
    v[0] += tx;
    v[1] += ty;
    v[2] += (px - B.x) * ty - (py - B.y) * tx;
  }
  __shared__ double lds[(SI_NT / 64) * 6];
  block_reduce<SI_NT, 6>(v, lds);
  if (threadIdx.x == 0) {
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
    out[3] = v[5];
  }
}

}  // namespace vp
