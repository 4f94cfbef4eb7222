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
                       int row0, int nrows, int col0, int ncols, const double *__restrict__ rho_in,
                       const double *__restrict__ ux_in, const double *__restrict__ uy_in,
                       double rho_u, double ux_u, double uy_u, const Ctl *__restrict__ ctl, double rho0,
                       int swapped, S *__restrict__ ec, int nper, const MoverDev *__restrict__ mov, int nmov,
                       int slot) {
  const int xl = blockIdx.x * blockDim.x + threadIdx.x;
  const int yl = blockIdx.y;
  if (xl >= ncols || yl >= nrows) return;
  const int x = col0 + xl, y = row0 + yl;
  const long long c = (long long)y * pitch + x;
  double rho, ux, uy;
  if (rho_in) {  // [nrows][ncols] staged values
    const long long k = (long long)yl * ncols + xl;
    rho = rho_in[k];
    ux = ux_in[k];
    uy = uy_in[k];
  } else {
    rho = rho_u;
    ux = ux_u;
    uy = uy_u;
    const int id = mask[c] & M_BODY;
    if (id != 0 && id <= nmov) {  // a moving disk's cells start at its rigid velocity
      const BodyDev B = mov[id - 1].B[slot];
      ux = B.u - B.omega * (double(y) - B.y);
      uy = B.v + B.omega * (double(x) - B.x);
    } else if (id == 1) {  // body 1's cells start at its velocity (static bodies 2.. at rest)
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
// chi: exact inside tests on the 1/4096 grid (integer arithmetic; disk_inside
// is in sample.hpp)
// ----------------------------------------------------------------------------
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
// moving disks between steps (one workgroup)
// ----------------------------------------------------------------------------
constexpr int REGION_MARGIN = 6;  // set-up: a disk's mask region around its box (links 1, sample walks 5)
constexpr int FLUSH_NT = 256;

// The mask bytes of the disks' windows from their states st (fx, fy: the
// centres on the 1/FIXQ grid; cs: two doubles of LDS): the bytes the last
// rewrite (or the set-up) wrote are cleared, then solid ids and interface
// bits over every window, then the sample bits of every point; each disk's
// rectangle is kept in mwin.  The step launches never read these bytes for
// a lattice with moving disks: they serve reads of the mask between steps.
// One workgroup of FLUSH_NT threads.
__device__ __forceinline__ void mover_mask(MoverDev *__restrict__ mov, int nmov, const BodyDev *st,
                                           const long long *fx, const long long *fy, const double *__restrict__ pts,
                                           int maxp, int rule, int nx, int ny, int pitch, int perx, int pery,
                                           uint8_t *__restrict__ mask, Ctl *__restrict__ ctl, double *cs) {
  MultiDiskSolid cur;
  cur.n = nmov;
#pragma unroll
  for (int k = 0; k < MAX_MOVERS; ++k) {
    cur.X[k] = fx[k < nmov ? k : 0];
    cur.Y[k] = fy[k < nmov ? k : 0];
    cur.R[k] = mov[k < nmov ? k : 0].R;
  }
  // clear what the last flush wrote
  for (int k = 0; k < nmov; ++k) {
    const int x0 = mov[k].mwin[0], y0 = mov[k].mwin[1], w = mov[k].mwin[2] - x0, h = mov[k].mwin[3] - y0;
    for (int t = threadIdx.x; t < w * h; t += FLUSH_NT) mask[(long long)(y0 + t / w) * pitch + x0 + t % w] = 0;
  }
  __threadfence_block();
  __syncthreads();
  // solid ids and interface bits over every window at the new states
  int wr[MAX_MOVERS][4];
#pragma unroll
  for (int k = 0; k < MAX_MOVERS; ++k) {
    const int kk = k < nmov ? k : 0;
    const int h = mov[kk].half;
    int ox, oy;
    mover_origin(st[kk], h, ox, oy);
    wr[k][0] = max(ox, 0);
    wr[k][1] = max(oy, 0);
    wr[k][2] = min(ox + 2 * h + 1, nx);
    wr[k][3] = min(oy + 2 * h + 1, ny);
  }
  for (int k = 0; k < nmov; ++k) {
    int x0 = 0, y0 = 0, x1 = 0, y1 = 0;
#pragma unroll
    for (int q = 0; q < MAX_MOVERS; ++q)
      if (q == k) { x0 = wr[q][0]; y0 = wr[q][1]; x1 = wr[q][2]; y1 = wr[q][3]; }
    const int w = x1 - x0, h = y1 - y0;
    for (int t = threadIdx.x; t < w * h; t += FLUSH_NT) {
      const int i = x0 + t % w, j = y0 + t / w;
      const int own = cur.id(i, j);
      bool iface = false, two = false;
      int other = 0;
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
        const int nid = cur.id(I, J);
        iface = iface || ((nid != 0) != (own != 0));
        if (!own && nid) {
          two = two || (other && other != nid);
          other = nid;
        }
      }
      if (two) atomicOr(&ctl->err, 2);
      mask[(long long)j * pitch + i] = (uint8_t)(own | (iface ? M_IFACE : 0));
    }
    if (threadIdx.x == 0) {
      mov[k].mwin[0] = x0;
      mov[k].mwin[1] = y0;
      mov[k].mwin[2] = x1;
      mov[k].mwin[3] = y1;
    }
  }
  __threadfence_block();
  __syncthreads();
  // sample bits of every point at the new states
  for (int k = 0; k < nmov; ++k) {
    const BodyDev S = st[k];
    if (threadIdx.x == 0) sincos(S.theta, &cs[1], &cs[0]);
    __syncthreads();
    const double co = cs[0], sn = cs[1];
    for (int i = mov[k].pt0 + (int)threadIdx.x; i < mov[k].pt1; i += FLUSH_NT) {
      double px, py, n0, n1;
      si_world(pts, maxp, i, 1, S, co, sn, px, py, n0, n1);
      int node[4];
      double wt[4];
      const int c = si_stencil(cur, nx, ny, rule, px, py, n0, n1, node, wt);
      if (c == 0) atomicOr(&ctl->err, 1);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < c) {
          const long long cc = (long long)(node[q] / nx) * pitch + node[q] % nx;
          atomicOr((unsigned *)(mask + (cc & ~3LL)), (unsigned)M_SAMPLE << (8 * (cc & 3)));
        }
      }
    }
    __syncthreads();
  }
}

// After the launch of step N (pb = N & 1): the disks' forces of step N are
// summed and their states advanced exactly as the next step launch would do
// it (mover_prologue: the same sums in the same order, the same update), so
// that forces, states and the mask can be read between steps; the next
// launch then starts from these states.  Then the mask of the disks'
// windows is rewritten from the new states (mover_mask).
__global__ void __launch_bounds__(FLUSH_NT)
    k_mover_flush(MoverDev *__restrict__ mov, int nmov, const double *__restrict__ win, int pb,
                  const double *__restrict__ pts, int maxp, int rule, int nx, int ny, int pitch, int perx, int pery,
                  uint8_t *__restrict__ mask, Ctl *__restrict__ ctl, double *__restrict__ hist, int cap, int maxb) {
  __shared__ double red[FIN_WAVES * 6];
  __shared__ double cs[2];
  __shared__ BodyDev st[MAX_MOVERS];
  __shared__ long long fx[MAX_MOVERS], fy[MAX_MOVERS];
  const int sread = pb ^ 1;
  const int tiles_x = (nx + MOV_BX - 1) / MOV_BX, tiles_y = (ny + MOV_BY - 1) / MOV_BY;
  for (int k = 0; k < nmov; ++k) {
    MoverDev &M = mov[k];
    const BodyDev B = M.B[sread];
    double F[6];
    mover_forces<FLUSH_NT>(M, B, win, tiles_x, tiles_y, red, F);
    const BodyDev S = mover_update(M, B, F);
    if (threadIdx.x == 0) {
      st[k] = S;
      fx[k] = fixq_of(S.x);
      fy[k] = fixq_of(S.y);
      M.B[pb] = S;
      const long long n = M.nfin + 1;
      double *hh = hist + ((n % cap) * maxb + k) * 6;
#pragma unroll
      for (int i = 0; i < 6; ++i) hh[i] = F[i];
      M.nfin = n;
      if (k == 0) {
#pragma unroll
        for (int i = 0; i < 6; ++i) ctl->last[i] = F[i];
        ctl->step = n;
        ctl->body = S;
      }
      if (fabs(S.x - B.x) >= 1.0 || fabs(S.y - B.y) >= 1.0) atomicOr(&ctl->err, 32);
    }
  }
  __syncthreads();
  mover_mask(mov, nmov, st, fx, fy, pts, maxp, rule, nx, ny, pitch, perx, pery, mask, ctl, cs);
}

// The mask of the disks' windows from the states in slot `slot` (set-up and
// changes of the points between steps).
__global__ void __launch_bounds__(FLUSH_NT)
    k_mover_mask(MoverDev *__restrict__ mov, int nmov, int slot, const double *__restrict__ pts, int maxp, int rule,
                 int nx, int ny, int pitch, int perx, int pery, uint8_t *__restrict__ mask, Ctl *__restrict__ ctl) {
  __shared__ double cs[2];
  __shared__ BodyDev st[MAX_MOVERS];
  __shared__ long long fx[MAX_MOVERS], fy[MAX_MOVERS];
  if ((int)threadIdx.x < nmov) {
    const BodyDev S = mov[threadIdx.x].B[slot];
    st[threadIdx.x] = S;
    fx[threadIdx.x] = fixq_of(S.x);
    fy[threadIdx.x] = fixq_of(S.y);
  }
  __syncthreads();
  mover_mask(mov, nmov, st, fx, fy, pts, maxp, rule, nx, ny, pitch, perx, pery, mask, ctl, cs);
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
