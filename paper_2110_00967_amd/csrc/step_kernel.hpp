// step_kernel.hpp -- the fused VP-LBM time step for gfx950.
//
// One thread updates one cell x of step n (state between steps: the
// post-collision deviations d~^{n-1} in buffer A, the 9 populations of each
// run of 64 cells along a row stored together, see pop_index):
//   1. pull streaming  f^n_a(x) = f~^{n-1}_a(x - c_a)   (Eq. eqBd) with the
//      edge rules (periodic, half-way bounce-back, specular, zero-gradient,
//      convective);
//   2. rho = sum f, m = sum c f; penalized velocity
//      u = (m + G/2 + k/2 rho u_s) / (rho (1 + k/2)), k = chi/eta
//      (Eqs. updatestep, updatestep3, updatestepm) and force density
//      F = G - rho k (u - u_s)  (penalization term of Eq. 1);
//   3. f^eq (Sec. 2.2), forcing term in the form of Guo et al. (cited for
//      F_alpha in Eq. eqBd) with the (1 - 1/(2 tau)) prefactor of Eq. TRT,
//      BGK or TRT relaxation, store into buffer B;
//   4. interface cells: momentum exchange (Eq. MMEL) of every pulled
//      population that crossed the solid/fluid boundary -- the same link sum
//      as Sec. 2.3.1 evaluated on f~^{n-1}, gathered per destination -- into
//      the cell's own slot (numbered body by body);
//   5. sample cells: stress (Sec. 2.3.2 sigma) of the streamed populations
//      into the node's record slot;
//   6. block 0 of the next step -- after the kernel boundary made them
//      visible -- sums each body's slots, and contracts its records with the
//      aggregated integration weights (Eq. defFf), in fixed order
//      (deterministic), into the force-history ring.  Slots alternate
//      between two buffers by step parity.
// HBM traffic per cell: 9 loads + 9 stores of the storage type + 1 mask byte.
#pragma once

#include "mover.hpp"

namespace vp {

template <typename T> struct StepArgs {
  int nx, ny, pitch;
  long long plane;      // ny * pitch
  int tiles_x, ntiles, per_xcd;
  unsigned tx_magic;    // floor((2^32 - 1) / tiles_x) (0 when tiles_x = 1), see tile_cell
  int rot[8];           // per XCD: the band's tiles start this far in (see k_step)
  int kind[4];          // edge kinds W, E, S, N
  T wu[4][2];           // 6 rho0 u_w of each edge: bounce-back increment w_a c_a . wu
  T omega, fac, kpen, rho0, gx, gy;
  T khalf, a1, kk;      // penalization in solid cells: k/2, 1/(1 + k/2), k/(1 + k/2)
  int trt;              // 0: BGK; 1: TRT (the kernel is chosen accordingly)
  T omega_m, fac_m;     // TRT: 1/tau- and 1 - 1/(2 tau-) (BGK: the same as omega, fac)
  T fo, fo9, fo3;       // tau+ - 1/2, 9 (tau+ - 1/2), 3 (tau- - 1/2)
  double facd, rho0d;
  const BodyDev *bodies;  // static bodies 2..: bodies[id] (body 1 lives in the control block)
  T *cbc;               // convective-edge state (see cbc_offset)
  T cbu[4];             // convection speed U of each convective edge
  T cbi[4];             // 1 / (1 + U)
  // AA pattern: the perimeter cells' post-collision populations kept by the
  // previous launch (read) and by this one (written), [9][nper] of the
  // storage type (see aa_pull_edge)
  const void *ec_in;
  void *ec_out;
  int nper;
  // moving disks (mover.hpp): nmov of them in mov, their points in pts
  // ([6][maxp], body frame), the lattice's stencil rule
  MoverDev *mov;
  int nmov;
  const double *pts;
  int maxp, si_rule;
  int wblocks;          // single-lattice launch: workgroups of the disks' hit boxes (see k_step)
};

// Source of deviation a arriving at (x, y) (any cell, edge or not): axis by
// axis, x first, when x - c_a leaves the lattice: periodic wraps, outflow
// clamps, free-slip takes the mirrored population of the edge cell itself,
// velocity bounces back the cell's own opposite population with the
// moving-wall increment `add` (and ends the resolution).  A convective edge
// resolves its source like outflow; `conv` tells that its blend applies (the
// first edge crossed, x first, unless a bounce-back ended the resolution).
// With c_a fixed only one x edge and one y edge can be crossed; the edge
// kinds are uniform, so the branches are uniform and the per-lane part is
// selects.
template <typename T>
__device__ __forceinline__ void edge_source(const StepArgs<T> &P, int x, int y, int a, int &pop, int &sx,
                                            int &sy, T &add, bool &conv) {
  const int cxa = cx(a), cya = cy(a);
  sx = x - cxa;
  sy = y - cya;
  pop = a;
  bool bb = false, cvx = false, cvy = false;
  add = T(0);
  // edge parameters are selected with constant indices only (no dynamic
  // indexing of the by-value argument block, which would spill it)
  if (cxa != 0) {
    const bool w = cxa > 0;  // c_x > 0 can only cross the west edge
    const bool out = w ? sx < 0 : sx >= P.nx;
    const int k = w ? P.kind[WEST] : P.kind[EAST];
    if (k == EDGE_VELOCITY) {
      bb = out;
      add = out ? T(wgt(a)) * (w ? T(cxa) * P.wu[WEST][0] + T(cya) * P.wu[WEST][1]
                                 : T(cxa) * P.wu[EAST][0] + T(cya) * P.wu[EAST][1])
                : T(0);
    } else if (k == EDGE_PERIODIC) {
      sx = out ? (w ? sx + P.nx : sx - P.nx) : sx;
    } else if (k == EDGE_OUTFLOW || k == EDGE_CONVECTIVE) {
      sx = out ? (w ? 0 : P.nx - 1) : sx;
      cvx = out && k == EDGE_CONVECTIVE;
    } else {
      pop = out ? flipx(pop) : pop;
      sx = out ? x : sx;
    }
  }
  if (cya != 0) {
    const bool s_ = cya > 0;  // c_y > 0 can only cross the south edge
    const bool out = s_ ? sy < 0 : sy >= P.ny;
    const int k = s_ ? P.kind[SOUTH] : P.kind[NORTH];
    if (k == EDGE_VELOCITY) {
      const bool hit = out && !bb;
      add = hit ? T(wgt(a)) * (s_ ? T(cxa) * P.wu[SOUTH][0] + T(cya) * P.wu[SOUTH][1]
                                  : T(cxa) * P.wu[NORTH][0] + T(cya) * P.wu[NORTH][1])
                : add;
      bb = bb || out;
    } else if (k == EDGE_PERIODIC) {
      sy = out ? (s_ ? sy + P.ny : sy - P.ny) : sy;
    } else if (k == EDGE_OUTFLOW || k == EDGE_CONVECTIVE) {
      sy = out ? (s_ ? 0 : P.ny - 1) : sy;
      cvy = out && k == EDGE_CONVECTIVE;
    } else {
      pop = out ? flipy(pop) : pop;
      sy = out ? y : sy;
    }
  }
  if (bb) {  // bounce-back: the cell's own opposite population
    pop = opp(a);
    sx = x;
    sy = y;
  }
  conv = (cvx || cvy) && !bb;
}

// Convective-edge state slot of population a at (x, y), given that its blend
// applies: the x edge when a crosses it and it is convective, else the y edge.
template <typename T>
__device__ __forceinline__ T *cbc_slot_ptr(const StepArgs<T> &P, int x, int y, int a) {
  const int cxa = cx(a), cya = cy(a);
  bool xe = false;
  if (cxa != 0) {
    const bool out = cxa > 0 ? x == 0 : x == P.nx - 1;
    xe = out && (cxa > 0 ? P.kind[WEST] : P.kind[EAST]) == EDGE_CONVECTIVE;
  }
  if (xe) return P.cbc + cbc_offset(cxa > 0 ? WEST : EAST, P.nx, P.ny) + (long long)cbc_slot(cya) * P.ny + y;
  return P.cbc + cbc_offset(cya > 0 ? SOUTH : NORTH, P.nx, P.ny) + (long long)cbc_slot(cxa) * P.nx + x;
}

template <typename T>
__device__ __forceinline__ T cbc_speed(const StepArgs<T> &P, int x, int a, bool inv) {
  const int cxa = cx(a), cya = cy(a);
  bool xe = false;
  if (cxa != 0) {
    const bool out = cxa > 0 ? x == 0 : x == P.nx - 1;
    xe = out && (cxa > 0 ? P.kind[WEST] : P.kind[EAST]) == EDGE_CONVECTIVE;
  }
  const int e = xe ? (cxa > 0 ? WEST : EAST) : (cya > 0 ? SOUTH : NORTH);
  // constant-index selection (see edge_source)
  const T u = e == WEST ? P.cbu[WEST] : e == EAST ? P.cbu[EAST] : e == SOUTH ? P.cbu[SOUTH] : P.cbu[NORTH];
  const T i = e == WEST ? P.cbi[WEST] : e == EAST ? P.cbi[EAST] : e == SOUTH ? P.cbi[SOUTH] : P.cbi[NORTH];
  return inv ? i : u;
}

// All 9 deviations arriving at (x, y).  The population loads go out first,
// together; then convective edges blend f(t+1) = (f(t) + U f_clamped) / (1 + U)
// with the state f(t) they left at the previous step (and store the new one
// when UPDATE).  Keeping the state traffic out of the first loop keeps the
// 9 loads in one memory round trip.
template <typename S, typename T, bool UPDATE>
__device__ __forceinline__ void pull_edge_all(const S *__restrict__ fin, const StepArgs<T> &P, int x, int y,
                                              T (&d)[Q]) {
  unsigned conv = 0;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    int pop, sx, sy;
    T add;
    bool cv;
    edge_source(P, x, y, a, pop, sx, sy, add, cv);
    d[a] = Store<S>::ld(fin + pop_index(pop, sx, sy, P.pitch)) + add;
    conv |= cv ? 1u << a : 0u;
  }
  if (conv) {  // only convective edge cells
    T st[Q];
#pragma unroll
    for (int a = 1; a < Q; ++a)
      if (conv >> a & 1u) st[a] = *cbc_slot_ptr(P, x, y, a);
#pragma unroll
    for (int a = 1; a < Q; ++a)
      if (conv >> a & 1u) {
        d[a] = (st[a] + cbc_speed(P, x, a, false) * d[a]) * cbc_speed(P, x, a, true);
        if (UPDATE) *cbc_slot_ptr(P, x, y, a) = d[a];
      }
  }
}

// AA pattern (one population buffer F, updated in place; Bailey et al.'s
// alternating scheme).  The odd launch of a pair pulls d~_a from slot
// opp(a) of x - c_a, where the even launch left it, and pushes its result to
// slot a of x + c_a; the even launch reads slot a of x and writes slot
// opp(a) of x.  Every slot is read and written by one thread only, which
// reads all of its slots before it writes any.  A source outside the lattice
// goes through the edge rules above; their sources are perimeter cells, so
// every launch also keeps the post-collision populations of its perimeter
// cells (ec_out) and the next launch reads the edge sources there (ec_in):
// the same stored values the two-buffer path reads from its source buffer.
template <typename S, typename T, int AA>
__device__ __forceinline__ void aa_pull_edge(const S *F, const StepArgs<T> &P, int x, int y, T (&d)[Q]) {
  const S *ec = (const S *)P.ec_in;
  unsigned conv = 0;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const int rx = x - cx(a), ry = y - cy(a);
    const bool in = rx >= 0 && rx < P.nx && ry >= 0 && ry < P.ny;
    int pop, sx, sy;
    T add;
    bool cv;
    edge_source(P, x, y, a, pop, sx, sy, add, cv);
    const long long k = in ? (AA == 1 ? pop_index(opp(a), rx, ry, P.pitch) : pop_index(a, x, y, P.pitch))
                           : (long long)(pop * P.nper + perim_index(sx, sy, P.nx, P.ny));
    d[a] = Store<S>::ld((in ? F : ec) + k) + (in ? T(0) : add);
    conv |= (!in && cv) ? 1u << a : 0u;
  }
  if (conv) {  // only convective edge cells (as in pull_edge_all)
    T st[Q];
#pragma unroll
    for (int a = 1; a < Q; ++a)
      if (conv >> a & 1u) st[a] = *cbc_slot_ptr(P, x, y, a);
#pragma unroll
    for (int a = 1; a < Q; ++a)
      if (conv >> a & 1u) {
        d[a] = (st[a] + cbc_speed(P, x, a, false) * d[a]) * cbc_speed(P, x, a, true);
        *cbc_slot_ptr(P, x, y, a) = d[a];
      }
  }
}

// Fast path addressing (interior waves: a wave is one aligned run of 64
// cells of one row, all with their neighbours inside the lattice):
// population a of row `row` at chunk `cw` (both wave-uniform), as a scalar
// base shifted back one chunk, so that the lane
// offsets lo[s + 1] of the elements at x + s (s = -1, 0, +1, crossing into
// the neighbouring chunk at the run's ends) are all non-negative.
template <typename S, typename T>
__device__ __forceinline__ S *fast_base(S *F, const StepArgs<T> &P, int row, int cw, int a) {
  return F + ((long long)row * (P.pitch >> 6) + cw) * CHUNK_ELEMS + a * 64 - CHUNK_ELEMS;
}

// Population a of the wave's own run of 64 cells (row `row`, chunk `cw`,
// both wave-uniform in every tile): scalar base + lane * sizeof(S)
template <typename S, typename T>
__device__ __forceinline__ S *own_base(S *F, const StepArgs<T> &P, int row, int cw, int a) {
  return F + ((long long)row * (P.pitch >> 6) + cw) * CHUNK_ELEMS + a * 64;
}

// Store the post-collision deviation v of population a of cell (x, y):
// two-buffer (AA = 0) in place; even AA launch (AA = 2) into slot opp(a) of
// the cell.  A perimeter cell (eidx >= 0) of an AA launch also keeps v in
// ec_out.  interior: the wave-uniform fast-path flag, with the wave's row
// yw, chunk cw and lane byte offset lb (own cell).
template <typename S, int AA, typename T>
__device__ __forceinline__ void put_pop(S *F, const StepArgs<T> &P, bool interior, uint32_t lb, int yw, int cw,
                                        int a, T v, int eidx) {
  static_assert(AA != 1, "odd AA launches store through put_pops_odd");
  Store<S>::st_at(own_base(F, P, yw, cw, AA == 0 ? a : opp(a)), lb, v);
  if constexpr (AA != 0) {
    if (!interior && eidx >= 0) Store<S>::st((S *)P.ec_out + (a * P.nper + eidx), v);
  }
}

// The nine post-collision deviations v of an odd AA launch, each into slot a
// of x + c_a (dropped when that leaves the lattice: its consumers read the
// perimeter copy, which a perimeter cell, eidx >= 0, keeps in ec_out).  They
// are stored together after the collision, in one wave-uniform branch: an
// interior wave from the bases of rows yw - 1, yw, yw + 1 computed once, plus
// the lane offsets lo (see fast_base).  Stores interleaved with the
// collision, each behind its own branch, recomputed a row base per store.
template <typename S, typename T>
__device__ __forceinline__ void put_pops_odd(S *F, const StepArgs<T> &P, bool interior, const uint32_t (&lo)[3],
                                             int yw, int cw, int x, int y, const T (&v)[Q], int eidx) {
  if (interior) {
    S *rb[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) rb[r] = fast_base(F, P, yw - 1 + r, cw, 0);
#pragma unroll
    for (int a = 0; a < Q; ++a) Store<S>::st_at(rb[1 + cy(a)] + a * 64, lo[1 + cx(a)], v[a]);
  } else {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const int tx = x + cx(a), ty = y + cy(a);
      if (tx >= 0 && tx < P.nx && ty >= 0 && ty < P.ny) Store<S>::st(F + pop_index(a, tx, ty, P.pitch), v[a]);
      if (eidx >= 0) Store<S>::st((S *)P.ec_out + (a * P.nper + eidx), v[a]);
    }
  }
}

template <int NT, int N>
__device__ __forceinline__ void block_reduce(double (&v)[N], double *lds /*[NT/64][N]*/) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = v[i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    v[i] = s;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) lds[wave * N + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += lds[w * N + i];
      v[i] = s;
    }
  }
}

// The force finalize sums in the order of FIN_W virtual lanes (mover.hpp),
// so forces do not depend on the tile shape or on which kernel finalizes.

// The first ME slot and SI record of a thread's virtual lane v0 (slot and
// record v0 of body 1's ranges, which start at 0 in a lattice with a single
// body), loaded before the ranges are known so that the two loads do not
// wait for one another.
struct FinPre {
  double me[3], g[3];
  SiRec R;
  bool me_ok, rec_ok;  // v0 within the slot / record capacity, values loaded
};

// Forces of one step -> its force-history slots, body by body
// (deterministic: fixed assignment and order).  ME: the contributions the
// interface cells stored in their slots.  SI: the stress each sample node
// stored (sig), contracted with the node's aggregated weights, record by
// record.  hist[(n mod cap) * maxb + b][6]; the control block keeps body 1's.
// lds holds FIN_WAVES * 6 doubles; out0, when given (LDS, 6 doubles), gets
// body 1's forces from thread 0.  pre, when given, holds this thread's first
// slot and record of body 1 (NT >= FIN_W: one virtual lane per thread); they
// enter the sums exactly where the loads would have.
template <int NT>
__device__ __forceinline__ void finalize_block(const double *__restrict__ me, const double *__restrict__ sig,
                                               const SiRec *__restrict__ recs, const BodyTab *__restrict__ bt,
                                               Ctl *__restrict__ ctl, double *__restrict__ hist, int cap, int maxb,
                                               double *lds, double *out0 = nullptr,
                                               const FinPre *pre = nullptr) {
  // force and geometry arithmetic: no multiply-add fusion, so that every kernel
  // that inlines this (alone, batched, any tile) rounds it the same way
  #pragma clang fp contract(off)
  static_assert(NT % 64 == 0, "whole waves");
  const long long n = ctl->step + 1;
  const int nb = ctl->nbody;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const BodyTab T0 = bt[0];  // issued with the control-block loads
  for (int b = 0; b < nb; ++b) {
    const BodyTab T = b == 0 ? T0 : bt[b];
    for (int k = wave; k < FIN_WAVES; k += NT / 64) {
      const int v0 = k * 64 + lane;  // this thread's virtual lane
      double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      const bool first = pre != nullptr && NT >= FIN_W && b == 0;
      int r0 = T.me0 + v0;
      if (first && T.me0 == 0 && r0 < T.me1 && pre->me_ok) {
#pragma unroll
        for (int i = 0; i < 3; ++i) v[i] += pre->me[i];
        r0 += FIN_W;
      }
      for (int r = r0; r < T.me1; r += FIN_W) {
#pragma unroll
        for (int i = 0; i < 3; ++i) v[i] += me[(long long)r * ME_STRIDE + i];
      }
      int q0 = T.rec0 + v0;
      if (first && T.rec0 == 0 && q0 < T.rec1 && pre->rec_ok) {
        const double *g = pre->g;
        const SiRec &R = pre->R;
        v[3] += g[0] * R.ax + g[1] * R.ay;
        v[4] += g[1] * R.ax + g[2] * R.ay;
        v[5] += g[0] * R.txx + g[1] * R.txy + g[2] * R.tyy;
        q0 += FIN_W;
      }
      for (int r = q0; r < T.rec1; r += FIN_W) {
        const double *g = sig + (long long)r * SIG_STRIDE;
        const SiRec R = recs[r];
        v[3] += g[0] * R.ax + g[1] * R.ay;
        v[4] += g[1] * R.ax + g[2] * R.ay;
        v[5] += g[0] * R.txx + g[1] * R.txy + g[2] * R.tyy;
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        double x = v[i];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) lds[k * 6 + i] = x;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double *h = hist + ((n % cap) * maxb + b) * 6;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        double x = 0.0;
        for (int k = 0; k < FIN_WAVES; ++k) x += lds[k * 6 + i];
        h[i] = x;
        if (b == 0) {
          ctl->last[i] = x;
          if (out0) out0[i] = x;
        }
      }
    }
    __syncthreads();  // lds is reused by the next body
  }
  if (threadIdx.x == 0) ctl->step = n;
}

// Torque reference point of body id (1..63): body 1's from the control block
// (it may move), the others' from the static table.  Only body 1 has a
// velocity; bodies 2.. are static.
template <typename T>
__device__ __forceinline__ void body_ref(const Ctl *__restrict__ ctl, const StepArgs<T> &P, int id, double &bx,
                                         double &by) {
  if (id <= 1) {
    bx = ctl->body.x;
    by = ctl->body.y;
  } else {
    bx = P.bodies[id].x;
    by = P.bodies[id].y;
  }
}

// Masks of the 8 lattice neighbours x - c_a of (x, y): wrapped across
// periodic edges; a neighbour beyond another edge does not exist and reads
// as fluid (0), so that it can neither link to the cell nor lend it a body.
template <typename T>
__device__ __forceinline__ void nbr_masks(const uint8_t *__restrict__ mask, const StepArgs<T> &P, int x, int y,
                                          uint8_t (&nm)[Q]) {
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    int sx = x - cx(a), sy = y - cy(a);
    bool there = true;
    if (cx(a) != 0) {
      const bool out = cx(a) > 0 ? sx < 0 : sx >= P.nx;
      there = !out || (cx(a) > 0 ? P.kind[WEST] : P.kind[EAST]) == EDGE_PERIODIC;
    }
    if (cy(a) != 0) {
      const bool out = cy(a) > 0 ? sy < 0 : sy >= P.ny;
      there = there && (!out || (cy(a) > 0 ? P.kind[SOUTH] : P.kind[NORTH]) == EDGE_PERIODIC);
    }
    sx = sx < 0 ? sx + P.nx : (sx >= P.nx ? sx - P.nx : sx);
    sy = sy < 0 ? sy + P.ny : (sy >= P.ny ? sy - P.ny : sy);
    nm[a] = there ? mask[(uint32_t)(sy * P.pitch + sx)] : (uint8_t)0;
  }
}

// One stress-integration point placed at its disk's state of this step, as
// the tile sees it: its stencil nodes inside the tile and their weights.
struct PtPlace {
  int in;          // bit q: stencil node q lies in the tile
  unsigned cell;   // tile cell of node q in bits 8q..8q+7
  double n0, n1;   // normal
  double rx, ry;   // lever arm from the disk's centre
  double s[4];     // ds times the stencil weight of node q
};

// A workgroup's view of the moving disks for one step (LDS).
template <int BX, int BY> struct MovLds {
  BodyDev st[MAX_MOVERS];  // state each disk uses in this step
  double cs[MAX_MOVERS][2];  // cos, sin of its angle
  long long fx[MAX_MOVERS], fy[MAX_MOVERS], fr[MAX_MOVERS];  // its centre and radius on the 1/FIXQ grid
  double red[FIN_WAVES * 6];  // force sums
  double sg[BX * BY][3];      // stress of the tile's sample nodes
  int anyme, anys;            // bit k: the tile has interface cells / sample nodes of disk k
  int smp[BX * BY];           // per tile cell: bit k = sample node of disk k
  uint8_t sid[(BX + 2) * (BY + 2)];  // tile and a one-cell ring: disk id (1..), 0 fluid, 0xFF no cell
  PtPlace pl[BX * BY];               // point t of the disks as placed by thread t
};

// The kernel's one MovLds of its tile shape.  A kernel that inlines the tile
// code twice (the batched AA kernel: odd and even launches) shares it
// between the copies instead of holding two, which would halve the
// workgroups an LDS of 160 KB holds (26.7 KB each at 64x4).
template <int BX, int BY> __device__ __forceinline__ MovLds<BX, BY> &mov_lds() {
  __shared__ MovLds<BX, BY> ml;
  return ml;
}

// The points of all moving disks are numbered disk by disk: disk k holds
// [pt1 of disk k - 1, pt1 of disk k).  The disk of point i:
__device__ __forceinline__ int point_disk(const int (&pt1)[MAX_MOVERS], int nmov, int i) {
  int k = 0;
#pragma unroll
  for (int q = 0; q < MAX_MOVERS - 1; ++q) k += (q + 1 < nmov && i >= pt1[q]) ? 1 : 0;
  return k;
}

// Point (a, b), normal (c, d), length ds of disk k placed at the disk's
// state of this step (ml.st, ml.cs), with its sample stencil among the disks
// cur; returns the stencil size (0: no sample node).
template <typename T, int BX, int BY>
__device__ __forceinline__ int place_point(const StepArgs<T> &P, const MovLds<BX, BY> &ml, const DiskSetRef &cur,
                                           int k, double a, double b, double c, double d, double ds, int x0, int y0,
                                           PtPlace &pp) {
  // force and geometry arithmetic: no multiply-add fusion, so that every kernel
  // that inlines this (alone, batched, any tile) rounds it the same way
  #pragma clang fp contract(off)
  const BodyDev S = ml.st[k];
  double px, py, n0, n1;
  si_place(a, b, c, d, 1, S, ml.cs[k][0], ml.cs[k][1], px, py, n0, n1);
  int node[4];
  double wt[4];
  const int cnt = si_stencil(cur, P.nx, P.ny, P.si_rule, px, py, n0, n1, node, wt);
  pp.in = 0;
  pp.cell = 0;
  pp.n0 = n0;
  pp.n1 = n1;
  pp.rx = px - S.x;
  pp.ry = py - S.y;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    pp.s[q] = ds * wt[q];
    if (q < cnt) {
      const int X = node[q] % P.nx - x0, Y = node[q] / P.nx - y0;
      if (X >= 0 && X < BX && Y >= 0 && Y < BY) {
        pp.in |= 1 << q;
        pp.cell |= (unsigned)(Y * BX + X) << (8 * q);
      }
    }
  }
  return cnt;
}

// The stress-integration terms of a placed point over its nodes in the
// tile (stress ml.sg): force s (sigma . n), torque r x that force.
template <int BX, int BY>
__device__ __forceinline__ void point_terms(const PtPlace &pp, const MovLds<BX, BY> &ml, double (&v)[6]) {
  // force and geometry arithmetic: no multiply-add fusion, so that every kernel
  // that inlines this (alone, batched, any tile) rounds it the same way
  #pragma clang fp contract(off)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (pp.in & (1 << q)) {
      const double *g = ml.sg[(pp.cell >> (8 * q)) & 0xFF];
      const double s = pp.s[q];
      const double fx = s * (g[0] * pp.n0 + g[1] * pp.n1), fy = s * (g[1] * pp.n0 + g[2] * pp.n1);
      v[3] += fx;
      v[4] += fy;
      v[5] += pp.rx * fy - pp.ry * fx;
    }
  }
}

// The tiles whose workgroups take part in a disk's step: those whose tile
// and one-cell ring meet the disk's window grown by two cells (a disk moves
// less than a cell per step), at the state (bx, by) the launch starts from --
// the box of tile indices [hx0, hx1] x [hy0, hy1].  It spans at most
// hit_tiles(h, BX) x hit_tiles(h, BY) tiles.
template <int BX, int BY>
__device__ __forceinline__ void hit_box(double bx, double by, int h, int &hx0, int &hy0, int &hx1, int &hy1) {
  const int ox = (int)floor(bx) - h, oy = (int)floor(by) - h, side = 2 * h + 1;
  hx0 = floordiv(ox - 3, BX);
  hx1 = floordiv(ox + side + 2, BX);
  hy0 = floordiv(oy - 3, BY);
  hy1 = floordiv(oy + side + 2, BY);
}
__host__ __device__ constexpr int hit_tiles(int h, int B) { return (2 * h + 6 + B - 1) / B + 1; }
template <int BX, int BY>
__device__ __forceinline__ bool in_hit_box(double bx, double by, int h, int tx, int ty) {
  int hx0, hy0, hx1, hy1;
  hit_box<BX, BY>(bx, by, h, hx0, hy0, hx1, hy1);
  return tx >= hx0 && tx <= hx1 && ty >= hy0 && ty <= hy1;
}

// Where a batched launch starts the XCD bands of the next one (see
// batch_place).  A band's key holds an epoch (40 bits) over the inverted
// rotation (24 bits), so that the largest key is the newest epoch's
// smallest rotation, and zero (the initial state) the oldest.
constexpr int ROT_BITS = 24;
constexpr unsigned long long ROT_MASK = (1ull << ROT_BITS) - 1, EPOCH_MASK = (1ull << 40) - 1;
__host__ __device__ constexpr unsigned long long band_key(unsigned long long epoch, long long rot) {
  return (epoch & EPOCH_MASK) << ROT_BITS | (ROT_MASK - (unsigned long long)rot);
}
// A batched launch's part in the rotation (mover_prologue records the keys
// of the launch after it): flip, the launch's flip (-1 outside batched
// launches); tile0, the lattice's first global tile; per_xcd, the tiles of
// a band.  Plain integers, so that nothing wide stays live through the tile
// code for it.
struct BandRot {
  int flip = -1;
  int tile0 = 0, per_xcd = 1;
};

// Band rotation state of the batched launches with moving disks on a
// device: the keys recorded for the launches of flip 0 and 1, then their
// epochs.  The launch of flip f reads keys[f] and epoch[f]; for the launch
// after it, it sets epoch[f ^ 1] = epoch[f] + 1 and records keys[f ^ 1]
// (atomic maximum: several disks in a band keep the earliest).  A slot is
// never written by the launch that reads it.  One per device, at a fixed
// address, so that its reads need nothing read first (a pointer argument
// would add a dependent read before the tile is known); zero at load.  Batches that run at the same time on
// one device share it: their rotations then mix, which orders their work
// less well and changes no result.
struct BandState {
  unsigned long long keys[2][8];
  unsigned long long epoch[2];
};
__device__ BandState g_band;

// The moving disks' part of one workgroup of the launch that computes step N
// (parity pb = N & 1; pending: the forces of step N - 1 are still to be
// summed and the states advanced by them).  States: slot k & 1 of
// MoverDev::B holds the state after k updates, so the state this launch
// starts from is in slot pb when pending, else in slot pb ^ 1.  Returns false
// (and touches no LDS) when the tile is outside every disk's hit box (known:
// the caller has found it inside one); then no cell of the tile is solid,
// interface or sample node of a moving disk, and the tile is outside every
// window of this step.  Otherwise, with every thread of the workgroup:
//   1. pending: the forces of step N - 1 of every disk (mover_forces on the
//      tile partials of step N - 1, part_prev), its new state (mover_update);
//      the workgroup of the tile holding the disk's centre cell writes the
//      state to the other slot, the forces to the history ring, flags a
//      disk that moved a cell or more (error bit 5) and, in a batched
//      launch, records where the next launch starts the disk's band (xr);
//   2. the solid ids of the tile and its ring, and the sample nodes of every
//      point that fall in the tile, at the states of this step (error bit 0
//      for a point without sample node).  Thread t places points t, t + NT,
//      ... and keeps the first in ml.pl[t] for mover_epilogue.
// The loads that do not depend on one another are issued together: the
// disks' positions first, then the partial sums with the points.
template <typename T, int BX, int BY>
__device__ __forceinline__ bool mover_prologue(int tx, int ty, const StepArgs<T> &P, Ctl *__restrict__ ctl,
                                               const double *__restrict__ part_prev, double *__restrict__ hist,
                                               int cap, int maxb, int pb, int pending, bool known,
                                               MovLds<BX, BY> &ml, const BandRot &xr = BandRot()) {
  // force and geometry arithmetic: no multiply-add fusion, so that every kernel
  // that inlines this (alone, batched, any tile) rounds it the same way
  #pragma clang fp contract(off)
  constexpr int NT = BX * BY;
  static_assert(BX == MOV_BX && BY == MOV_BY, "moving disks run the tile of their partials");
  const int x0 = tx * BX, y0 = ty * BY;
  const int sread = pending ? pb : pb ^ 1;
  const int nmov = P.nmov;
  bool hit = known;
  int pt1[MAX_MOVERS];
  int ptot = 0;
#pragma unroll
  for (int k = 0; k < MAX_MOVERS; ++k) {
    pt1[k] = 0;
    if (k < nmov) {
      const MoverDev &M = P.mov[k];
      pt1[k] = M.pt1;
      ptot = pt1[k];
      if (!known) hit = hit || in_hit_box<BX, BY>(M.B[sread].x, M.B[sread].y, M.half, tx, ty);
    }
  }
  if (!hit) return false;
  // the epoch of the launch after this one, for the band keys the recording
  // workgroups write (read here, well before they need it)
  const unsigned long long epoch_next = xr.flip >= 0 ? g_band.epoch[xr.flip] + 1 : 0;
  // this thread's first point and its disk's radius, in flight with the sums
  const int i0 = threadIdx.x;
  double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0, q4 = 0.0;
  if (i0 < ptot) {
    q0 = P.pts[i0];
    q1 = P.pts[P.maxp + i0];
    q2 = P.pts[2 * P.maxp + i0];
    q3 = P.pts[3 * P.maxp + i0];
    q4 = P.pts[4 * P.maxp + i0];
  }
  const long long rk = (int)threadIdx.x < nmov ? P.mov[threadIdx.x].R : 0;
  if (pending) {
    const int tiles_x = (P.nx + BX - 1) / BX, tiles_y = (P.ny + BY - 1) / BY;
    for (int k = 0; k < nmov; ++k) {
      MoverDev &M = P.mov[k];
      const BodyDev B = M.B[sread];
      double F[6];
      mover_forces<NT>(M, B, part_prev, tiles_x, tiles_y, ml.red, F);
      const BodyDev S = mover_update(M, B, F);
      if (threadIdx.x == 0) ml.st[k] = S;
      const int ci = min(max((int)floor(B.x), 0), P.nx - 1), cj = min(max((int)floor(B.y), 0), P.ny - 1);
      if (threadIdx.x == 0 && ci >= x0 && ci < x0 + BX && cj >= y0 && cj < y0 + BY) {
        // the recording workgroup of this disk (exactly one per launch)
        M.B[sread ^ 1] = S;
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
        if (xr.flip >= 0) {
          // the next launch starts the band holding this disk's hit box a
          // tile row before the box (the disk moves less than a cell per
          // step), so that the box's workgroups are among its first; of
          // several disks in one band the earliest, so that the others
          // follow it in order
          int hx0, hy0, hx1, hy1;
          hit_box<BX, BY>(S.x, S.y, M.half, hx0, hy0, hx1, hy1);
          const long long g = xr.tile0 + (long long)max(hy0 - 1, 0) * tiles_x;
          const long long band = g / xr.per_xcd;
          const long long rot = g - band * xr.per_xcd;
          if (band < 8 && rot <= (long long)ROT_MASK)
            atomicMax(&g_band.keys[xr.flip ^ 1][band], band_key(epoch_next, rot));
        }
      }
    }
  } else if ((int)threadIdx.x < nmov) {
    ml.st[threadIdx.x] = P.mov[threadIdx.x].B[sread];
  }
  if (threadIdx.x == 0) {
    ml.anyme = 0;
    ml.anys = 0;
  }
  __syncthreads();
  if ((int)threadIdx.x < nmov) {
    const int k = threadIdx.x;
    const BodyDev S = ml.st[k];
    double sn, co;
    sincos(S.theta, &sn, &co);
    ml.cs[k][0] = co;
    ml.cs[k][1] = sn;
    ml.fx[k] = fixq_of(S.x);
    ml.fy[k] = fixq_of(S.y);
    ml.fr[k] = rk;
  }
  for (int t = threadIdx.x; t < BX * BY; t += NT) ml.smp[t] = 0;
  __syncthreads();
  const DiskSetRef cur{nmov, ml.fx, ml.fy, ml.fr};
  const bool perx = P.kind[WEST] == EDGE_PERIODIC, pery = P.kind[SOUTH] == EDGE_PERIODIC;
  for (int t = threadIdx.x; t < (BX + 2) * (BY + 2); t += NT) {
    int X = x0 - 1 + t % (BX + 2), Y = y0 - 1 + t / (BX + 2);
    bool there = true;
    if (X < 0 || X >= P.nx) {
      there = perx;
      X = X < 0 ? X + P.nx : X - P.nx;
    }
    if (Y < 0 || Y >= P.ny) {
      there = there && pery;
      Y = Y < 0 ? Y + P.ny : Y - P.ny;
    }
    ml.sid[t] = there ? (uint8_t)cur.id(X, Y) : (uint8_t)0xFF;
  }
  // point i0 of the disks (thread i0), kept in ml.pl for mover_epilogue;
  // more than NT points in all: the others after it, placed again there
  for (int i = i0; i < ptot; i += NT) {
    const bool first = i == i0;
    double a = q0, b = q1, cn = q2, dn = q3, ds = q4;
    if (!first) {
      a = P.pts[i];
      b = P.pts[P.maxp + i];
      cn = P.pts[2 * P.maxp + i];
      dn = P.pts[3 * P.maxp + i];
      ds = P.pts[4 * P.maxp + i];
    }
    const int k = point_disk(pt1, nmov, i);
    PtPlace t;
    if (place_point(P, ml, cur, k, a, b, cn, dn, ds, x0, y0, t) == 0) atomicOr(&ctl->err, 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (t.in & (1 << q)) {
        atomicOr(&ml.smp[(t.cell >> (8 * q)) & 0xFF], 1 << k);
        atomicOr(&ml.anys, 1 << k);
      }
    }
    if (first) ml.pl[threadIdx.x] = t;
  }
  if (i0 >= ptot) ml.pl[threadIdx.x].in = 0;
  __syncthreads();
  return true;
}

// The tile's partial sums of the step for every disk whose window (at the
// disk's state of this step) covers the tile: the momentum exchange of the
// cells linked to the disk (acc, bid), and the stress integration of the
// disk's points over the sample nodes in the tile (each node's stress sg,
// weighted by the point's stencil weight and ds, contracted with its normal;
// torque about the disk's centre).  Thread t adds the terms of points t (as
// mover_prologue placed it, ml.pl[t]), t + NT, ..., then each sum is
// reduced in one fixed order (wave_sum_f64 per wave, the waves in order) and
// written by thread 0 to the disk's slot of the tile in part.  Uniform over
// the workgroup (mover_prologue returned true).
template <typename T, int BX, int BY>
__device__ __forceinline__ void mover_epilogue(int tx, int ty, const StepArgs<T> &P, const double (&acc)[3], int bid,
                                               const double (&sg)[3], double *__restrict__ part,
                                               MovLds<BX, BY> &ml) {
  // force and geometry arithmetic: no multiply-add fusion, so that every kernel
  // that inlines this (alone, batched, any tile) rounds it the same way
  #pragma clang fp contract(off)
  constexpr int NT = BX * BY, NW = NT / 64;
  static_assert(NW <= FIN_WAVES, "one partial per wave in ml.red");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  ml.sg[threadIdx.x][0] = sg[0];
  ml.sg[threadIdx.x][1] = sg[1];
  ml.sg[threadIdx.x][2] = sg[2];
  if (bid) atomicOr(&ml.anyme, 1 << (bid - 1));
  __syncthreads();
  const int anyme = ml.anyme, anys = ml.anys;
  const int nmov = P.nmov;
  int pt1[MAX_MOVERS];
  int ptot = 0;
#pragma unroll
  for (int k = 0; k < MAX_MOVERS; ++k) {
    pt1[k] = k < nmov ? P.mov[k].pt1 : 0;
    if (k < nmov) ptot = pt1[k];
  }
  for (int k = 0; k < nmov; ++k) {
    const MoverDev &M = P.mov[k];
    int tx0, ty0, ntx, nty;
    mover_tile_box(ml.st[k], M.half, tx0, ty0, ntx, nty);
    if (tx < tx0 || tx >= tx0 + ntx || ty < ty0 || ty >= ty0 + nty) continue;
    double *w = part + (long long)(M.part0 + (ty - ty0) * M.ptx + (tx - tx0)) * PART_ENTRY;
    if (!((anyme | anys) & (1 << k))) {
      if (threadIdx.x < 6) w[threadIdx.x] = 0.0;
      continue;
    }
    const bool mine = bid == k + 1;
    double v[6] = {mine ? acc[0] : 0.0, mine ? acc[1] : 0.0, mine ? acc[2] : 0.0, 0.0, 0.0, 0.0};
    if (anys & (1 << k)) {
      if ((int)threadIdx.x < ptot && point_disk(pt1, nmov, threadIdx.x) == k) point_terms(ml.pl[threadIdx.x], ml, v);
      if (ptot > NT) {
        // points t + NT, ...: placed again
        const DiskSetRef cur{P.nmov, ml.fx, ml.fy, ml.fr};
        for (int i = (int)threadIdx.x + NT; i < ptot; i += NT) {
          if (point_disk(pt1, nmov, i) != k) continue;
          PtPlace t;
          place_point(P, ml, cur, k, P.pts[i], P.pts[P.maxp + i], P.pts[2 * P.maxp + i], P.pts[3 * P.maxp + i],
                      P.pts[4 * P.maxp + i], tx * BX, ty * BY, t);
          point_terms(t, ml, v);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const double x = wave_sum_f64(v[i]);
      if (lane == 0) ml.red[wave * 6 + i] = x;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
      double x = 0.0;
      for (int q = 0; q < NW; ++q) x += ml.red[q * 6 + threadIdx.x];
      w[threadIdx.x] = x;
    }
    __syncthreads();
  }
}

// One thread's cell of a tile: its place and how its populations are
// addressed.  A wave is one aligned run of 64 cells of one row (tiles are 64,
// 128 or 256 cells wide), so its row and chunk are scalars; when the run's
// cells all have their 8 neighbours inside the lattice (interior, decided
// per wave), each population loads from a scalar base (fast_base) + one of
// three small lane offsets, and stores the same way.
struct TileCell {
  int tx, ty, lx, ly, x, y, c, yw, cw;
  bool interior, live;
  uint32_t lb, lo[3];
};

template <typename S, int BX, int BY, typename T>
__device__ __forceinline__ TileCell tile_cell(int tile, const StepArgs<T> &P) {
  TileCell t;
  // tile / tiles_x by multiply-high with m = floor((2^32 - 1) / tiles_x):
  // the estimate is the quotient or one less (tile < 2^31), fixed by one
  // comparison; m = 0 stands for tiles_x = 1
  t.ty = P.tx_magic ? (int)__umulhi((unsigned)tile, P.tx_magic) : tile;
  t.tx = tile - t.ty * P.tiles_x;
  if (t.tx >= P.tiles_x) {
    t.tx -= P.tiles_x;
    t.ty += 1;
  }
  t.lx = threadIdx.x % BX;
  t.ly = threadIdx.x / BX;
  t.x = t.tx * BX + t.lx;
  t.y = t.ty * BY + t.ly;
  t.live = t.x < P.nx && t.y < P.ny;
  t.c = t.y * P.pitch + t.x;
  const int lane = t.x & 63;
  t.lb = (uint32_t)(lane * sizeof(S));
  t.lo[0] = (uint32_t)((lane > 0 ? lane + CHUNK_ELEMS - 1 : 63) * sizeof(S));
  t.lo[1] = (uint32_t)((lane + CHUNK_ELEMS) * sizeof(S));
  t.lo[2] = (uint32_t)((lane < 63 ? lane + CHUNK_ELEMS + 1 : 2 * CHUNK_ELEMS) * sizeof(S));
  t.yw = __builtin_amdgcn_readfirstlane(t.y);
  t.cw = __builtin_amdgcn_readfirstlane(t.x >> 6);
  // fast path per wave (one aligned run of 64 cells of one row): every cell
  // of the run and all its neighbours inside the lattice; the waves of an
  // edge tile whose own run is clear of the edges take it too
  const int xw = t.cw * 64;
  t.interior = (xw >= 1) & (xw + 64 <= P.nx - 1) & (t.yw >= 1) & (t.yw <= P.ny - 2);
  return t;
}

// The streamed populations of a live cell.  AA launches read through fout,
// the pointer they write through: the thread's own stores overwrite the
// slots it read (a read-only view of the buffer would let the compiler
// re-load a value after such a store).
template <typename S, int AA, typename T>
__device__ __forceinline__ void load_cell(const TileCell &t, const S *__restrict__ fin, S *__restrict__ fout,
                                          const StepArgs<T> &P, T (&d)[Q]) {
  const S *src = AA == 0 ? fin : (const S *)fout;
  if (t.interior) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      if constexpr (AA == 0)
        d[a] = Store<S>::ld(at(fast_base(src, P, t.yw - cy(a), t.cw, a), t.lo[1 - cx(a)]));
      else if constexpr (AA == 1)
        d[a] = Store<S>::ld(at(fast_base(src, P, t.yw - cy(a), t.cw, opp(a)), t.lo[1 - cx(a)]));
      else
        d[a] = Store<S>::ld(at(fast_base(src, P, t.yw, t.cw, a), t.lo[1]));
    }
  } else if constexpr (AA == 0) {
    pull_edge_all<S, T, true>(src, P, t.x, t.y, d);
  } else {
    aa_pull_edge<S, T, AA>(src, P, t.x, t.y, d);
  }
}

// The force terms' buffers and body tables of a lattice, as the tile code
// reaches them (FB in step_tile and cell_update): ctl (counters, error bits,
// body 1's state), recs (SI records), si_map / imap (slot of each sample /
// interface cell), bt (body table), me_out / me_prev and sig_out / sig_prev
// (interface and sample-node terms of this step and the step before), hist
// (force history ring of cap entries of maxb bodies).  ArgBufs holds them as
// values: the single-lattice kernel's arguments, or what a batched launch
// with moving disks reads from the lattice's description at the start; a
// batched launch without them reads each only where a cell needs it
// (DescBufs; batch_bufs chooses).
struct ArgBufs {
  Ctl *ctl_;
  const SiRec *recs_;
  const int *si_map_, *imap_;
  const BodyTab *bt_;
  double *me_out_;
  const double *me_prev_;
  double *sig_out_;
  const double *sig_prev_;
  double *hist_;
  int cap_, maxb_;
  __device__ Ctl *ctl() const { return ctl_; }
  __device__ const SiRec *recs() const { return recs_; }
  __device__ const int *si_map() const { return si_map_; }
  __device__ const int *imap() const { return imap_; }
  __device__ const BodyTab *bt() const { return bt_; }
  __device__ double *me_out() const { return me_out_; }
  __device__ const double *me_prev() const { return me_prev_; }
  __device__ double *sig_out() const { return sig_out_; }
  __device__ const double *sig_prev() const { return sig_prev_; }
  __device__ double *hist() const { return hist_; }
  __device__ int cap() const { return cap_; }
  __device__ int maxb() const { return maxb_; }
};

// The update of a live cell with flags m (body id, interface, sample node)
// from its streamed populations d: moments, penalization, collision and the
// stores of the post-collision populations (and the macroscopic fields when
// MACRO); at an interface cell its momentum-exchange terms (acc, and the
// body bid its links belong to), at a sample node its stress (sg).  Static
// bodies store them in their slots for the finalize; moving disks (MOV with
// P.nmov > 0) keep them for mover_epilogue and take their states and the
// neighbours' ids from ml.
template <typename S, int BX, int BY, bool MACRO, bool TRT, int AA, bool MOV, typename T, typename ML, typename FB>
__device__ __forceinline__ void cell_update(const TileCell &t, const T (&d)[Q], uint8_t m, S *__restrict__ fout,
                                            const uint8_t *__restrict__ mask, const StepArgs<T> &P, const FB &fb,
                                            T *__restrict__ mrho, T *__restrict__ mux, T *__restrict__ muy,
                                            const ML &ml, double (&acc)[3], int &bid, double (&sg)[3]) {
  const int x = t.x, y = t.y, c = t.c, yw = t.yw, cw = t.cw;
  const bool tile_interior = t.interior;
  const uint32_t lb = t.lb;
  const uint32_t(&lo)[3] = t.lo;
  const int sc = (t.ly + 1) * (BX + 2) + t.lx + 1;  // the cell in the ring array ml.sid
  const int eidx = (AA != 0 && !tile_interior && (x == 0 || x == P.nx - 1 || y == 0 || y == P.ny - 1))
                       ? perim_index(x, y, P.nx, P.ny)
                       : -1;

  // moments (of the deviations: sum w = 1, sum w c = 0)
  const T drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
  const T mx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
  const T my = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
  const T rho = P.rho0 + drho;
  // a non-finite density means the run diverged: one lane per such wave
  // flags it (error bit 4) for the host's next check
  {
    const unsigned long long bad = __ballot(!(fabs(drho) <= T(1e30)));
    if (bad && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)bad) - 1)) atomicOr(&fb.ctl()->err, 16);
  }

  // penalized velocity (Eq. updatestepm) and force; k = 0 in fluid cells
  T khalf = T(0), a1 = T(1), kk = T(0), usx = T(0), usy = T(0);
  const int id = m & M_BODY;
  const bool chi = id != 0;
  if (chi) {
    khalf = P.khalf;
    a1 = P.a1;
    kk = P.kk;
    if (MOV && P.nmov > 0) {  // a moving disk: its state of this step
      const BodyDev B = ml.st[id - 1];
      usx = T(B.u - B.omega * (double(y) - B.y));
      usy = T(B.v + B.omega * (double(x) - B.x));
    } else if (id == 1) {  // the only static-lattice body that can move (u_s = 0 in the static ones)
      const BodyDev B = fb.ctl()->body;
      usx = T(B.u - B.omega * (double(y) - B.y));
      usy = T(B.v + B.omega * (double(x) - B.x));
    }
  }
  const T hx = mx + T(0.5) * P.gx, hy = my + T(0.5) * P.gy;
  const T den = a1 * recip(rho);  // 1 / (rho (1 + k/2))
  const T ux = (hx + khalf * rho * usx) * den;
  const T uy = (hy + khalf * rho * usy) * den;
  const T Fx = P.gx - kk * (hx - rho * usx);
  const T Fy = P.gy - kk * (hy - rho * usy);

  const T uu15 = T(1.5) * (ux * ux + uy * uy);
  const T uF3 = T(3) * (ux * Fx + uy * Fy);
  T ov[Q];  // odd AA launch: the results, stored together after the collision
  {
    // Collision with the forcing term (Eqs. TRT and eqBd; BGK is tau- =
    // tau+), per pair (a, a') with c_a' = -c_a.  Since 1 - 1/(2 tau) =
    // (tau - 1/2) / tau, the forcing term enters as a shift of the
    // equilibrium, even part by (tau+ - 1/2) F_even and odd part by
    // (tau- - 1/2) F_odd:
    //   q_a = wgt_a (De + Do),  q_a' = wgt_a (De - Do),
    //   De = drho - 1.5 rho u.u - 3 (tau+ - 1/2) u.F
    //        + (c.u) (4.5 rho (c.u) + 9 (tau+ - 1/2) (c.F)),
    //   Do = 3 rho (c.u) + 3 (tau- - 1/2) (c.F),
    // and out = d - (d - q)_even / tau+ - (d - q)_odd / tau-.  The
    // non-equilibrium part d - q is formed before it is scaled, which
    // keeps the FP32 rounding of mass and momentum unbiased.
    const T C1 = drho - rho * uu15 - P.fo * uF3;
    const T R45 = T(4.5) * rho, R3 = T(3) * rho;
    const T o0 = d[0] - P.omega * (d[0] - T(wgt(0)) * C1);
    if constexpr (AA == 1)
      ov[0] = o0;
    else
      put_pop<S, AA>(fout, P, tile_interior, lb, yw, cw, 0, o0, eidx);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int a = k < 2 ? k + 1 : k + 3;  // 1, 2, 5, 6; a' = 3, 4, 7, 8
      const int o = opp(a);
      const T w = T(wgt(a));
      const T cu = dotc(a, ux, uy);
      const T cF = dotc(a, Fx, Fy);
      const T De = cu * (R45 * cu + P.fo9 * cF) + C1;
      const T Do = R3 * cu + P.fo3 * cF;
      T oa, oo;
      if constexpr (!TRT) {
        oa = d[a] - P.omega * (d[a] - w * (De + Do));
        oo = d[o] - P.omega * (d[o] - w * (De - Do));
      } else {
        const T se = T(0.5) * (d[a] + d[o]) - w * De;
        const T so = T(0.5) * (d[a] - d[o]) - w * Do;
        oa = d[a] - P.omega * se - P.omega_m * so;
        oo = d[o] - P.omega * se + P.omega_m * so;
      }
      if constexpr (AA == 1) {
        ov[a] = oa;
        ov[o] = oo;
      } else {
        put_pop<S, AA>(fout, P, tile_interior, lb, yw, cw, a, oa, eidx);
        put_pop<S, AA>(fout, P, tile_interior, lb, yw, cw, o, oo, eidx);
      }
    }
  }
  if constexpr (AA == 1) put_pops_odd<S>(fout, P, tile_interior, lo, yw, cw, x, y, ov, eidx);
  if (MACRO) {
    mrho[(uint32_t)c] = rho;
    mux[(uint32_t)c] = ux;
    muy[(uint32_t)c] = uy;
  }

  if (m & M_IFACE) {
#pragma clang fp contract(off)  // (see finalize_block)
    // momentum exchange: every population pulled across the interface;
    // the link's interface point is its midpoint seen from its fluid node.
    // The 8 neighbour masks are loaded all at once (a load inside the
    // divergent loop below would cost one memory round trip per link).
    // The cell's links all belong to one body: its own if solid, else that
    // of its solid neighbours (a fluid cell is linked to one body at most).
    bool movl = false;  // a lattice with moving disks: every body moves
    if constexpr (MOV) movl = P.nmov > 0;
    uint8_t nm[Q];
    if constexpr (MOV) {
      if (movl) {
#pragma unroll
        for (int a = 1; a < Q; ++a) {
          const uint8_t nb = ml.sid[sc - cy(a) * (BX + 2) - cx(a)];
          nm[a] = nb == 0xFF ? 0 : nb;
        }
      } else {
        nbr_masks(mask, P, x, y, nm);
      }
    } else {
      nbr_masks(mask, P, x, y, nm);
    }
    bid = id;
#pragma unroll
    for (int a = 1; a < Q; ++a) bid = bid ? bid : (nm[a] & M_BODY);
    double bx, by;
    if constexpr (MOV) {
      if (movl) {
        bx = ml.st[bid - 1].x;
        by = ml.st[bid - 1].y;
      } else {
        body_ref(fb.ctl(), P, bid, bx, by);
      }
    } else {
      body_ref(fb.ctl(), P, bid, bx, by);
    }
    const bool moving = movl || bid == 1;  // u_s = 0 on the links of static bodies 2..
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      int sx = x - cx(a), sy = y - cy(a);
      bool link = true;
      if (sx < 0 || sx >= P.nx) {
        if ((sx < 0 ? P.kind[WEST] : P.kind[EAST]) != EDGE_PERIODIC) link = false;
        sx = sx < 0 ? sx + P.nx : sx - P.nx;
      }
      if (sy < 0 || sy >= P.ny) {
        if ((sy < 0 ? P.kind[SOUTH] : P.kind[NORTH]) != EDGE_PERIODIC) link = false;
        sy = sy < 0 ? sy + P.ny : sy - P.ny;
      }
      const bool schi = (nm[a] & M_BODY) != 0;
      if (!link || schi == chi) continue;
      double gx, gy, s;
      if (chi) { gx = sx + 0.5 * cx(a); gy = sy + 0.5 * cy(a); s = 1.0; }
      else { gx = x - 0.5 * cx(a); gy = y - 0.5 * cy(a); s = -1.0; }
      double ugx = 0.0, ugy = 0.0;
      if (moving) {
        if constexpr (MOV) {
          if (movl) {
            const BodyDev &B = ml.st[bid - 1];
            ugx = B.u - B.omega * (gy - B.y);
            ugy = B.v + B.omega * (gx - B.x);
          } else {
            const BodyDev &B = fb.ctl()->body;
            ugx = B.u - B.omega * (gy - B.y);
            ugy = B.v + B.omega * (gx - B.x);
          }
        } else {
          const BodyDev &B = fb.ctl()->body;
          ugx = B.u - B.omega * (gy - B.y);
          ugy = B.v + B.omega * (gx - B.x);
        }
      }
      const double fa = wgt(a) * P.rho0d + double(d[a]);
      const double lx_ = s * (cx(a) - ugx) * fa, ly_ = s * (cy(a) - ugy) * fa;
      acc[0] += lx_;
      acc[1] += ly_;
      acc[2] += (gx - bx) * ly_ - (gy - by) * lx_;
    }
    if (!movl) {
      // this cell's contribution goes to its slot; the finalize sums them
      double *o = fb.me_out() + (long long)fb.imap()[(uint32_t)c] * ME_STRIDE;
      o[0] = acc[0];
      o[1] = acc[1];
      o[2] = acc[2];
    }
  }
  if (m & M_SAMPLE) {
#pragma clang fp contract(off)  // (see finalize_block)
    // stress of the streamed populations at a (fluid) sample node
    T pxx = T(0), pxy = T(0), pyy = T(0);
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      const T w = T(wgt(a));
      const T cu = dotc(a, ux, uy);
      const T ne = d[a] - (w * drho + w * rho * (T(3) * cu + T(4.5) * cu * cu - uu15));
      pxx += T(cx(a) * cx(a)) * ne;
      pxy += T(cx(a) * cy(a)) * ne;
      pyy += T(cy(a) * cy(a)) * ne;
    }
    const double pr = double(drho) / 3.0;
    sg[0] = -pr - P.facd * double(pxx);
    sg[1] = -P.facd * double(pxy);
    sg[2] = -pr - P.facd * double(pyy);
    if (!(MOV && P.nmov > 0)) {
      // the node's stress goes to its record's slot; the finalize
      // contracts it with the aggregated weights
      double *g = fb.sig_out() + (long long)fb.si_map()[(uint32_t)c] * SIG_STRIDE;
      g[0] = sg[0];
      g[1] = sg[1];
      g[2] = sg[2];
    }
  }
}

// One workgroup's tile of the step (tile < P.ntiles): the body of the step
// kernel, shared by the single-lattice and the batched launch.  The
// workgroup of tile 0 also finalizes the previous step's forces (fin_prev).
// MOV: the lattice may hold moving disks (P.nmov > 0; no static bodies
// then): their cells take solid, interface and sample flags from the disks'
// states (mover_prologue) instead of the mask, and their force terms go to
// per-tile partial sums in me_out (mover_epilogue); pb is the parity of the
// step, mov_pending tells that the previous step's disk forces are still to
// be summed.  SPLIT (the single-lattice launch): win tells that the tile is
// one of a disk's hit box (taken by the workgroups that come first); a
// plain workgroup leaves the hit boxes' tiles alone.  Otherwise every
// workgroup tests its tile itself.
template <typename S, int BX, int BY, bool MACRO, bool TRT, int AA, bool MOV = false, bool SPLIT = false,
          typename FB>
__device__ __forceinline__ void step_tile(int tile, const S *__restrict__ fin, S *__restrict__ fout,
                                          const uint8_t *__restrict__ mask, const StepArgs<typename Store<S>::T> P,
                                          const FB &fb, int fin_prev, typename Store<S>::T *__restrict__ mrho,
                                          typename Store<S>::T *__restrict__ mux,
                                          typename Store<S>::T *__restrict__ muy, int pb = 0, int mov_pending = 0,
                                          bool win = false, const BandRot &xr = BandRot()) {
  using T = typename Store<S>::T;
  constexpr int NT = BX * BY;
  const TileCell t = tile_cell<S, BX, BY>(tile, P);

  // the cell's mask byte, then its streamed populations, loaded first: with
  // moving disks they are in flight while the disks' states are read.  The
  // mask goes out before the populations, since 2-byte populations are
  // converted as they arrive and a load issued after them would wait for
  // all nine.
  uint8_t mk = 0;
  if (!MOV || P.nmov == 0) mk = t.live ? mask[(uint32_t)t.c] : 0;
  T d[Q];
  if (t.live) load_cell<S, AA>(t, fin, fout, P, d);

  // moving disks: the states of this step and the tile's flags (LDS)
  bool mwg = false;  // the tile meets a disk's window
  MovLds<(MOV ? BX : 1), (MOV ? BY : 1)> &ml = mov_lds<(MOV ? BX : 1), (MOV ? BY : 1)>();
  if constexpr (MOV) {
    if (P.nmov > 0) {
      if (SPLIT && !win) {
        // a plain workgroup of the split launch: a tile of a hit box is the
        // hit boxes' workgroups' (nothing stored here), any other tile holds
        // plain fluid cells
        const int sread = mov_pending ? pb : pb ^ 1;
        bool hit = false;
        for (int k = 0; k < P.nmov; ++k)
          hit = hit || in_hit_box<BX, BY>(P.mov[k].B[sread].x, P.mov[k].B[sread].y, P.mov[k].half, t.tx, t.ty);
        if (hit) return;
      } else {
        mwg = mover_prologue<T, BX, BY>(t.tx, t.ty, P, fb.ctl(), fb.me_prev(), fb.hist(), fb.cap(), fb.maxb(), pb,
                                        mov_pending, SPLIT, ml, xr);
      }
    }
  }

  double acc[3] = {0.0, 0.0, 0.0};  // the cell's momentum exchange
  int bid = 0;                      // the body its links belong to
  double sg[3] = {0.0, 0.0, 0.0};   // its stress, at a sample node
  if (t.live) {
    // the cell's flags: the mask, or for a lattice with moving disks the
    // disks' ids around the cell (its tile ring index sc)
    uint8_t m = mk;
    if (MOV && P.nmov > 0 && mwg) {
      const int sc = (t.ly + 1) * (BX + 2) + t.lx + 1;
      const uint8_t own = ml.sid[sc];
      bool iface = false;
      int other = 0;
      bool two = false;
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        const uint8_t nb = ml.sid[sc - cy(a) * (BX + 2) - cx(a)];
        if (nb == 0xFF) continue;
        iface = iface || ((nb != 0) != (own != 0));
        if (!own && nb) {
          two = two || (other && other != nb);
          other = nb;
        }
      }
      if (two) atomicOr(&fb.ctl()->err, 2);
      const int sb = ml.smp[t.ly * BX + t.lx];
      if (sb & (sb - 1)) atomicOr(&fb.ctl()->err, 4);  // a node sampled for two disks
      m = (uint8_t)(own | (iface ? M_IFACE : 0) | (sb ? M_SAMPLE : 0));
    }
    cell_update<S, BX, BY, MACRO, TRT, AA, MOV>(t, d, m, fout, mask, P, fb, mrho, mux, muy, ml, acc, bid, sg);
  }
  if constexpr (MOV) {
    if (mwg) mover_epilogue<T, BX, BY>(t.tx, t.ty, P, acc, bid, sg, fb.me_out(), ml);
  }

  if (fin_prev && tile == 0) {
    // forces of the previous step (same slots and records: only static
    // bodies defer)
    __shared__ double lds[FIN_WAVES * 6];
    finalize_block<NT>(fb.me_prev(), fb.sig_prev(), fb.recs(), fb.bt(), fb.ctl(), fb.hist(), fb.cap(), fb.maxb(),
                       lds);
  }
}

// Launch with moving disks (P.nmov > 0): workgroup b < P.wblocks takes tile
// b of the disks' hit boxes laid end to end, disk by disk, each box as
// hit_tiles(h, BX) x hit_tiles(h, BY) tiles from its lower corner; -1 for a
// place outside the box or the lattice, or a tile an earlier disk's box
// already holds.
template <int BX, int BY, typename T>
__device__ __forceinline__ int window_block_tile(int b, const StepArgs<T> &P, int sread) {
  const int tiles_y = (P.ny + BY - 1) / BY;
  // every disk's reference point and window, read at once (one round trip)
  int h[MAX_MOVERS];
  double bx[MAX_MOVERS], by[MAX_MOVERS];
#pragma unroll
  for (int k = 0; k < MAX_MOVERS; ++k) {
    const int kk = k < P.nmov ? k : 0;
    h[k] = P.mov[kk].half;
    bx[k] = P.mov[kk].B[sread].x;
    by[k] = P.mov[kk].B[sread].y;
  }
  int tile = -1, j = b;
  bool found = false;
#pragma unroll
  for (int k = 0; k < MAX_MOVERS; ++k) {
    if (k >= P.nmov || found) continue;
    const int n = hit_tiles(h[k], BX) * hit_tiles(h[k], BY);
    if (j >= n) {
      j -= n;
      continue;
    }
    found = true;
    int hx0, hy0, hx1, hy1;
    hit_box<BX, BY>(bx[k], by[k], h[k], hx0, hy0, hx1, hy1);
    const int w = hit_tiles(h[k], BX);
    const int tx = hx0 + j % w, ty = hy0 + j / w;
    if (tx > hx1 || ty > hy1 || tx < 0 || ty < 0 || tx >= P.tiles_x || ty >= tiles_y) continue;
    bool earlier = false;
#pragma unroll
    for (int q = 0; q < k; ++q) earlier = earlier || in_hit_box<BX, BY>(bx[q], by[q], h[q], tx, ty);
    if (!earlier) tile = ty * P.tiles_x + tx;
  }
  return tile;
}

// Resident waves per SIMD the step kernels are compiled for: 8 for 4- and
// 2-byte storage (register budget 64 VGPRs and the SGPRs that allow 8 waves);
// FP64 needs more VGPRs and is left to the compiler.
template <typename S> constexpr int step_waves() { return sizeof(typename Store<S>::T) == 8 ? 1 : 8; }
// With moving disks the workgroups of the disks' windows run a long serial
// prologue and epilogue (force sums, state update, point stencils); the
// register budget of 4 waves per SIMD keeps them free of spills.
template <typename S, bool MOV> constexpr int step_waves_mov() { return MOV && step_waves<S>() > 4 ? 4 : step_waves<S>(); }

template <typename S, int BX, int BY, bool MACRO, bool TRT, int AA, bool MOV = false>
__global__ void __launch_bounds__(BX *BY, (step_waves_mov<S, MOV>()))
    k_step(const S *__restrict__ fin, S *__restrict__ fout, const uint8_t *__restrict__ mask,
           const StepArgs<typename Store<S>::T> P, Ctl *__restrict__ ctl,
           const SiRec *__restrict__ recs, const int *__restrict__ si_map,
           const int *__restrict__ imap, const BodyTab *__restrict__ bt, double *__restrict__ me_out,
           const double *__restrict__ me_prev, double *__restrict__ sig_out, const double *__restrict__ sig_prev,
           int fin_prev, double *__restrict__ hist, int cap, int maxb, typename Store<S>::T *__restrict__ mrho,
           typename Store<S>::T *__restrict__ mux, typename Store<S>::T *__restrict__ muy, int pb, int mov_pending) {
  if constexpr (MOV) {
    // moving disks (P.nmov > 0): the first P.wblocks workgroups (a multiple
    // of 8) take the tiles of the disks' hit boxes, so that their long serial
    // work starts first; the others take the tiles XCD by XCD as below and
    // leave those of the hit boxes alone
    const int b = blockIdx.x;
    int tile;
    const bool win = b < P.wblocks;
    if (win) {
      // these workgroups share their compute units with plain tiles; their
      // waves go first in instruction issue
      __builtin_amdgcn_s_setprio(3);
      tile = window_block_tile<BX, BY>(b, P, mov_pending ? pb : pb ^ 1);
      if (tile < 0) return;
    } else {
      const int bb = b - P.wblocks, xcd = bb & 7, i = bb >> 3;
      const int start = xcd * P.per_xcd, len = min(P.per_xcd, P.ntiles - start);
      if (i >= len) return;
      tile = start + i;
    }
    const ArgBufs fb{ctl, recs, si_map, imap, bt, me_out, me_prev, sig_out, sig_prev, hist, cap, maxb};
    step_tile<S, BX, BY, MACRO, TRT, AA, true, true>(tile, fin, fout, mask, P, fb, 0, mrho, mux, muy, pb, mov_pending,
                                                     win);
    return;
  }
  // XCD-aware tile order: consecutive workgroups go round-robin over the 8
  // XCDs, so give each XCD a contiguous band of tiles (shared halo lines stay
  // in that XCD's L2).  A band only a few rounds of workgroups deep is
  // rotated to start at the first row of the force window it holds: the
  // slower tiles there are dispatched first and overlap the rest of the band
  // instead of extending its end.
  const int b = blockIdx.x, xcd = b & 7, i = b >> 3;
  const int start = xcd * P.per_xcd, len = min(P.per_xcd, P.ntiles - start);
  if (i >= len) return;
  int t = i + P.rot[xcd];
  t -= t >= len ? len : 0;
  const int tile = start + t;
  const ArgBufs fb{ctl, recs, si_map, imap, bt, me_out, me_prev, sig_out, sig_prev, hist, cap, maxb};
  step_tile<S, BX, BY, MACRO, TRT, AA, MOV>(tile, fin, fout, mask, P, fb, fin_prev, mrho, mux, muy, pb, mov_pending);
}

// Per-lattice description for the batched step: one launch covers the tiles
// of every active lattice, laid end to end in tile order.
template <typename T> struct CaseDesc {
  StepArgs<T> P;
  const void *buf[2];     // populations of parity 0 and 1
  uint8_t *mask;
  Ctl *ctl;
  const SiRec *recs;
  const int *si_map;
  const int *imap;        // interface slot of each interface cell
  BodyTab *bt;
  double *me[2];          // interface contributions of steps with parity 0 and 1
  double *sig[2];         // sample-node stresses of steps with parity 0 and 1
  double *hist;
  int cap, maxb;
  int tile0;              // first global tile of this lattice
  int ntiles;             // its tiles
  int cur0;               // parity of the buffer holding the state at launch 0
  int pbit0;              // parity of the step computed by launch 0
  int pending0;           // launch 0 finalizes the static bodies' forces of the step before it
  int mov_pending0;       // launch 0 sums the moving disks' forces of the step before it
  // AA pattern: the perimeter copies kept by the steps of parity 0 and 1
  void *ec[2];
};

// The lattice table of a batched launch has one entry per block of
// TILE_BLOCK consecutive global tiles: the lattice of the block's first tile
// and the block's tiles that start a lattice.  Some kilobytes for millions
// of tiles, it stays in the caches while the populations stream past (an
// entry per tile would be evicted from L2 by every launch, and each
// workgroup would wait for HBM before its first population load), and the
// lattice of any tile follows from its block's entry alone, with no further
// dependent read.
constexpr int TILE_BLOCK = 64;
struct BlockCase {
  int first;                 // lattice of the block's first tile
  int pad;
  unsigned long long starts; // bit j (j >= 1): tile j of the block is a lattice's first
};

// The table from the descriptors (tiles of lattice i are [tile0, tile0 +
// ntiles), in order, ntiles >= 1): one thread per block, binary search on
// tile0 for the first tile's lattice, then the lattices starting inside.
template <typename T>
__global__ void k_fill_tile_case(const CaseDesc<T> *__restrict__ cases, int ncases, int nblocks,
                                 BlockCase *__restrict__ table) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nblocks) return;
  const int t = k * TILE_BLOCK;
  int lo = 0, hi = ncases - 1;  // last lattice with tile0 <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cases[mid].tile0 <= t) lo = mid; else hi = mid - 1;
  }
  unsigned long long starts = 0;
  for (int c = lo + 1; c < ncases && cases[c].tile0 < t + TILE_BLOCK; ++c) starts |= 1ull << (cases[c].tile0 - t);
  BlockCase e;
  e.first = lo;
  e.pad = 0;
  e.starts = starts;
  table[k] = e;
}

// The lattice of global tile g: its block's first lattice plus the lattices
// that start at tiles 1..j of the block (j = g's place in it).
__device__ __forceinline__ int lattice_in(const BlockCase &e, int g) {
  const int j = g % TILE_BLOCK;
  return e.first + __popcll(e.starts & ((2ull << j) - 2ull));
}
__device__ __forceinline__ int tile_lattice(const BlockCase *__restrict__ table, int g) {
  return lattice_in(table[g / TILE_BLOCK], g);
}

// p as a global-memory pointer: pointers read from a descriptor in memory
// would otherwise be generic, and every access through them a flat access
// (slower to issue, and counted against both the vector-memory and the
// scalar wait counters)
template <typename U> __device__ __forceinline__ U *gp(U *p) {
  // rebuilt from its (uniform) bits, so that the compiler cannot fold the
  // global view away again
  const uintptr_t x = (uintptr_t)p;
  const uintptr_t lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)x);
  const uintptr_t hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(x >> 32));
  return (U *)(VP_GLOBAL char *)((hi << 32) | lo);
}

// The description's pointers as global pointers.
template <typename T> __device__ __forceinline__ void global_ptrs(StepArgs<T> &P) {
  P.bodies = gp(P.bodies);
  P.cbc = gp(P.cbc);
  P.ec_in = gp(P.ec_in);
  P.ec_out = gp(P.ec_out);
  P.mov = gp(P.mov);
  P.pts = gp(P.pts);
}

// The force terms' buffers and body tables of a batched launch's lattice
// (see ArgBufs), read from its description where a cell needs them: held
// from the workgroup's start they would take some twenty scalar registers,
// which the compiler spills one read at a time before the first population
// load.  pb: the parity of the step the launch computes.
template <typename T> struct DescBufs {
  const CaseDesc<T> *C;
  int pb;
  __device__ Ctl *ctl() const { return gp(C->ctl); }
  __device__ const SiRec *recs() const { return gp(C->recs); }
  __device__ const int *si_map() const { return gp(C->si_map); }
  __device__ const int *imap() const { return gp(C->imap); }
  __device__ const BodyTab *bt() const { return gp((const BodyTab *)C->bt); }
  __device__ double *me_out() const { return gp(C->me[pb]); }
  __device__ const double *me_prev() const { return gp((const double *)C->me[pb ^ 1]); }
  __device__ double *sig_out() const { return gp(C->sig[pb]); }
  __device__ const double *sig_prev() const { return gp((const double *)C->sig[pb ^ 1]); }
  __device__ double *hist() const { return gp(C->hist); }
  __device__ int cap() const { return C->cap; }
  __device__ int maxb() const { return C->maxb; }
};

// The buffers a batched launch's tile code reaches: read where used
// (DescBufs) without moving disks; with moving disks every workgroup of a
// lattice with disks reaches some of them in its hit test, and reads made
// there, one after another, cost more than reading all of them at the start
// (ArgBufs).
template <bool MOV, typename T>
__device__ __forceinline__ auto batch_bufs(const CaseDesc<T> *__restrict__ C, int pb) {
  if constexpr (MOV)
    return ArgBufs{C->ctl, C->recs, C->si_map, C->imap, C->bt, C->me[pb], C->me[pb ^ 1], C->sig[pb], C->sig[pb ^ 1],
                   C->hist, C->cap, C->maxb};
  else
    return DescBufs<T>{C, pb};
}

// The place of workgroup b of a batched launch: its global tile (gtile) and
// the description of that tile's lattice, or null for none.  The workgroups go round-robin
// over the 8 XCDs, and XCD x takes the band of per_xcd consecutive tiles
// from x * per_xcd (shared halo lines stay in its L2).  With moving disks
// (ROT) band x starts r tiles in and wraps round, so that the long serial
// work of a disk's hit-box workgroups starts among the band's first
// workgroups instead of wherever the disk sits: r from the band's key
// (band_key) the launch before recorded (mover_prologue); a key of another
// epoch (stale, or none yet) or a rotation outside the band counts as r = 0.
// The band state lives at a fixed address, so its reads need nothing read
// before them.  Any r gives the same results: it only orders the work.
template <bool ROT, typename CD>
__device__ __forceinline__ const CD *batch_place(int b, int total_tiles, int per_xcd, const BlockCase *__restrict__ table,
                                                 const CD *cases, int flip, int &gtile, unsigned long long &epoch) {
  const int x = b & 7, i = b >> 3, start = x * per_xcd;
  if constexpr (!ROT) {
    gtile = start + i;
    if (gtile >= total_tiles) return nullptr;
    return cases + tile_lattice(table, gtile);
  } else {
    // (both flips' keys and epochs, chosen by flip afterwards; a workgroup
    // without tile reads the table at the last tile and leaves after it)
    const unsigned long long k0 = g_band.keys[0][x], k1 = g_band.keys[1][x];
    const unsigned long long e0 = g_band.epoch[0], e1 = g_band.epoch[1];
    const unsigned long long key = flip ? k1 : k0;
    epoch = flip ? e1 : e0;
    const int len = min(per_xcd, total_tiles - start);
    long long r = (key >> ROT_BITS) == (epoch & EPOCH_MASK) ? (long long)(ROT_MASK - (key & ROT_MASK)) : 0;
    r = r < len ? r : 0;
    const int t = i + (int)r;
    gtile = min(start + (t >= len ? t - len : t), total_tiles - 1);
    const CD *c = cases + tile_lattice(table, gtile);
    return i < len ? c : nullptr;
  }
}

// Batched step: launch number `flip` (0 or 1, alternating) of a run over
// ncases lattices; the lattice of each tile comes from the lattice table.
// MOV: some lattice of the batch has moving disks.  ROT (with MOV): the
// bands start at the disks' hit boxes (batch_place), for launches short
// enough that a disk's serial work decides when they end; the form without
// it keeps the plain tiles' code as it is for long launches (the rotation's
// reads and records cost them some registers).
template <typename S, int BX, int BY, bool TRT, bool MOV = false, bool ROT = false>
__global__ void __launch_bounds__(BX *BY, (step_waves_mov<S, MOV>()))
    k_step_batch(const CaseDesc<typename Store<S>::T> *__restrict__ cases,
                 const BlockCase *__restrict__ table, int total_tiles, int per_xcd, int flip, int first) {
  using T = typename Store<S>::T;
  // the tile and the description of its lattice, then the description's
  // fields, read once (unconditionally, so that the reads go out together)
  int gtile;
  unsigned long long epoch = 0;
  const CaseDesc<T> *__restrict__ C =
      batch_place<MOV && ROT>(blockIdx.x, total_tiles, per_xcd, table, cases, flip, gtile, epoch);
  if (!C) return;
  if (MOV && ROT && blockIdx.x == 0 && threadIdx.x == 0) g_band.epoch[flip ^ 1] = epoch + 1;
  StepArgs<T> P = C->P;
  global_ptrs(P);
  const int par = C->cur0 ^ flip, pb = C->pbit0 ^ flip;
  const int pend0 = C->pending0, mpend0 = C->mov_pending0;
  const int fin_prev = P.nmov ? 0 : (first ? pend0 : 1);
  const int mov_pending = first ? mpend0 : 1;
  const S *fin = gp((const S *)C->buf[par]);
  S *fout = gp((S *)C->buf[par ^ 1]);
  // (the force terms' buffers serve interface and sample cells, the finalize
  // and the disks' work only: read where used unless MOV, see batch_bufs)
  step_tile<S, BX, BY, false, TRT, 0, MOV>(gtile - C->tile0, fin, fout, gp(C->mask), P, batch_bufs<MOV>(C, pb),
                                           fin_prev, nullptr, nullptr, nullptr, pb, mov_pending, false,
                                           (ROT ? BandRot{flip, C->tile0, per_xcd} : BandRot()));
}

// Batched step of lattices in the AA pattern (one population buffer each):
// the launch computing an odd step pulls and pushes (AA = 1), an even step
// stays in the cell (AA = 2), per lattice by its own step parity; the
// perimeter copies alternate with it (read: the previous step's, written:
// this step's).  PAR = 1 or 2: every lattice of the launch computes an odd
// (1) or an even (2) step, and the kernel holds that tile code only; PAR = 0
// (lattices of mixed parity) holds both, chosen per lattice, whose combined
// register pressure makes the 2-byte kernel spill its scalars far more.
template <typename S, bool TRT, bool MOV = false, bool ROT = false, int PAR = 0>
__global__ void __launch_bounds__(256, (step_waves_mov<S, MOV>()))
    k_step_batch_aa(const CaseDesc<typename Store<S>::T> *__restrict__ cases,
                    const BlockCase *__restrict__ table, int total_tiles, int per_xcd, int flip, int first) {
  using T = typename Store<S>::T;
  int gtile;
  unsigned long long epoch = 0;
  const CaseDesc<T> *__restrict__ C =
      batch_place<MOV && ROT>(blockIdx.x, total_tiles, per_xcd, table, cases, flip, gtile, epoch);
  if (!C) return;
  if (MOV && ROT && blockIdx.x == 0 && threadIdx.x == 0) g_band.epoch[flip ^ 1] = epoch + 1;
  StepArgs<T> P = C->P;
  global_ptrs(P);
  const int pb = PAR ? (PAR == 1 ? 1 : 0) : C->pbit0 ^ flip;
  P.ec_in = gp(C->ec[pb ^ 1]);
  P.ec_out = gp(C->ec[pb]);
  const int pend0 = C->pending0, mpend0 = C->mov_pending0;
  const int fin_prev = P.nmov ? 0 : (first ? pend0 : 1);
  const int mov_pending = first ? mpend0 : 1;
  S *F = gp((S *)C->buf[0]);
  if (PAR == 1 || (PAR == 0 && pb))
    step_tile<S, 64, 4, false, TRT, 1, MOV>(gtile - C->tile0, nullptr, F, gp(C->mask), P, batch_bufs<MOV>(C, pb),
                                            fin_prev, nullptr, nullptr, nullptr, pb, mov_pending, false,
                                            (ROT ? BandRot{flip, C->tile0, per_xcd} : BandRot()));
  else
    step_tile<S, 64, 4, false, TRT, 2, MOV>(gtile - C->tile0, nullptr, F, gp(C->mask), P, batch_bufs<MOV>(C, pb),
                                            fin_prev, nullptr, nullptr, nullptr, pb, mov_pending, false,
                                            (ROT ? BandRot{flip, C->tile0, per_xcd} : BandRot()));
}

template <int NT>
__global__ void __launch_bounds__(NT)
    k_finalize(const double *__restrict__ me, const double *__restrict__ sig, const SiRec *__restrict__ recs,
               const BodyTab *__restrict__ bt, Ctl *__restrict__ ctl, double *__restrict__ hist, int cap, int maxb) {
  __shared__ double lds[FIN_WAVES * 6];
  finalize_block<NT>(me, sig, recs, bt, ctl, hist, cap, maxb, lds);
}

}  // namespace vp
