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

#include "d2q9.hpp"

namespace vp {

template <typename T> struct StepArgs {
  int nx, ny, pitch;
  long long plane;      // ny * pitch
  int tiles_x, ntiles, per_xcd;
  unsigned tx_magic;    // floor(2^32 / tiles_x) + 1 (0 when tiles_x = 1)
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
    // element index in 32 bits: 9 ny pitch < 2^31 for every accepted lattice
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
    const int k = in ? (AA == 1 ? pop_index(opp(a), rx, ry, P.pitch) : pop_index(a, x, y, P.pitch))
                     : pop * P.nper + perim_index(sx, sy, P.nx, P.ny);
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

// Fast path addressing (interior tiles, where a wave is one aligned run of
// 64 cells of one row): population a of row `row` at chunk `cw` (both
// wave-uniform), as a scalar base shifted back one chunk, so that the lane
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
// the cell; odd AA launch (AA = 1) into slot a of x + c_a, dropped when that
// leaves the lattice (its consumers read the perimeter copy).  A perimeter
// cell (eidx >= 0) of an AA launch also keeps v in ec_out.  interior: the
// workgroup-uniform fast-path flag, with the wave's row yw, chunk cw, lane
// byte offset lb (own cell) and lane offsets lo (see fast_base).
template <typename S, int AA, typename T>
__device__ __forceinline__ void put_pop(S *F, const StepArgs<T> &P, bool interior, uint32_t lb,
                                        const uint32_t (&lo)[3], int yw, int cw, int x, int y, int a, T v,
                                        int eidx) {
  if constexpr (AA == 0 || AA == 2) {
    Store<S>::st_at(own_base(F, P, yw, cw, AA == 0 ? a : opp(a)), lb, v);
  } else {
    if (interior) {
      Store<S>::st_at(fast_base(F, P, yw + cy(a), cw, a), lo[1 + cx(a)], v);
    } else {
      const int tx = x + cx(a), ty = y + cy(a);
      if (tx >= 0 && tx < P.nx && ty >= 0 && ty < P.ny) Store<S>::st(F + pop_index(a, tx, ty, P.pitch), v);
    }
  }
  if constexpr (AA != 0) {
    if (!interior && eidx >= 0) Store<S>::st((S *)P.ec_out + (a * P.nper + eidx), v);
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

// Width of the force finalize's summation order: FIN_W virtual lanes, lane v
// summing slots v, v + FIN_W, ...; each virtual wave of 64 lanes reduced by a
// butterfly, the FIN_W / 64 wave sums added in order.  Every workgroup size
// runs the same order (a block of NT threads takes the virtual waves
// w, w + NT/64, ... with its waves w), so forces do not depend on the tile
// shape or on which kernel finalizes.
constexpr int FIN_W = 256;
constexpr int FIN_WAVES = FIN_W / 64;

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

// Masks of the 8 lattice neighbours of (x, y), wrapped into the lattice (the
// momentum exchange decides separately which links are real)
template <typename T>
__device__ __forceinline__ void nbr_masks(const uint8_t *__restrict__ mask, const StepArgs<T> &P, int x, int y,
                                          uint8_t (&nm)[Q]) {
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    int sx = x - cx(a), sy = y - cy(a);
    sx = sx < 0 ? sx + P.nx : (sx >= P.nx ? sx - P.nx : sx);
    sy = sy < 0 ? sy + P.ny : (sy >= P.ny ? sy - P.ny : sy);
    nm[a] = mask[(uint32_t)(sy * P.pitch + sx)];
  }
}

// One workgroup's tile of the step (tile < P.ntiles): the body of the step
// kernel, shared by the single-lattice and the batched launch.  The
// workgroup of tile 0 also finalizes the previous step's forces (fin_prev).
template <typename S, int BX, int BY, bool MACRO, bool TRT, int AA>
__device__ __forceinline__ void step_tile(
    int tile, const S *__restrict__ fin, S *__restrict__ fout, const uint8_t *__restrict__ mask,
    const StepArgs<typename Store<S>::T> P, Ctl *__restrict__ ctl, const SiRec *__restrict__ recs,
    const int *__restrict__ si_map, const int *__restrict__ imap, const BodyTab *__restrict__ bt,
    double *__restrict__ me_out, const double *__restrict__ me_prev, double *__restrict__ sig_out,
    const double *__restrict__ sig_prev, int fin_prev, double *__restrict__ hist, int cap, int maxb,
    typename Store<S>::T *__restrict__ mrho, typename Store<S>::T *__restrict__ mux,
    typename Store<S>::T *__restrict__ muy) {
  using T = typename Store<S>::T;
  constexpr int NT = BX * BY;
  // tile / tiles_x by multiply-high (exact while tile * tiles_x < 2^32, which
  // every accepted lattice satisfies: tiles_x^2 * ny <= 58,255 * pitch < 2^30)
  const int ty = P.tx_magic ? (int)__umulhi((unsigned)tile, P.tx_magic) : tile;
  const int tx = tile - ty * P.tiles_x;
  const int lx = threadIdx.x % BX, ly = threadIdx.x / BX;
  const int x = tx * BX + lx, y = ty * BY + ly;


  // Every cell of the tile has all 8 neighbours inside the lattice: the
  // workgroup-uniform fast path.  A wave is then one run of 64 cells of one
  // row (tiles are 64, 128 or 256 cells wide), so its row and chunk are
  // scalars; each population loads from a scalar base (fast_base) + one of
  // three small lane offsets, and stores the same way.
  const bool tile_interior = (tx * BX >= 1) & (tx * BX + BX <= P.nx - 1) & (ty * BY >= 1) &
                             (ty * BY + BY <= P.ny - 1);

  if (x < P.nx && y < P.ny) {
    const int c = y * P.pitch + x;
    const int lane = x & 63;
    const uint32_t lb = (uint32_t)(lane * sizeof(S));
    const uint32_t lo[3] = {(uint32_t)((lane > 0 ? lane + CHUNK_ELEMS - 1 : 63) * sizeof(S)),
                            (uint32_t)((lane + CHUNK_ELEMS) * sizeof(S)),
                            (uint32_t)((lane < 63 ? lane + CHUNK_ELEMS + 1 : 2 * CHUNK_ELEMS) * sizeof(S))};
    const int yw = __builtin_amdgcn_readfirstlane(y), cw = __builtin_amdgcn_readfirstlane(x >> 6);
    const uint8_t m = mask[(uint32_t)c];
    T d[Q];
    // AA launches read through fout, the pointer they write through: the
    // thread's own stores overwrite the slots it read (a read-only view of
    // the buffer would let the compiler re-load a value after such a store)
    const S *src = AA == 0 ? fin : (const S *)fout;
    if (tile_interior) {
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        if constexpr (AA == 0)
          d[a] = Store<S>::ld(at(fast_base(src, P, yw - cy(a), cw, a), lo[1 - cx(a)]));
        else if constexpr (AA == 1)
          d[a] = Store<S>::ld(at(fast_base(src, P, yw - cy(a), cw, opp(a)), lo[1 - cx(a)]));
        else
          d[a] = Store<S>::ld(at(fast_base(src, P, yw, cw, a), lo[1]));
      }
    } else if constexpr (AA == 0) {
      pull_edge_all<S, T, true>(src, P, x, y, d);
    } else {
      aa_pull_edge<S, T, AA>(src, P, x, y, d);
    }
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
      if (bad && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)bad) - 1)) atomicOr(&ctl->err, 16);
    }

    // penalized velocity (Eq. updatestepm) and force; k = 0 in fluid cells
    T khalf = T(0), a1 = T(1), kk = T(0), usx = T(0), usy = T(0);
    const int id = m & M_BODY;
    const bool chi = id != 0;
    if (chi) {
      khalf = P.khalf;
      a1 = P.a1;
      kk = P.kk;
      if (id == 1) {  // the only body that can move (u_s = 0 in the static ones)
        const BodyDev B = ctl->body;
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
      put_pop<S, AA>(fout, P, tile_interior, lb, lo, yw, cw, x, y, 0, d[0] - P.omega * (d[0] - T(wgt(0)) * C1),
                     eidx);
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
        put_pop<S, AA>(fout, P, tile_interior, lb, lo, yw, cw, x, y, a, oa, eidx);
        put_pop<S, AA>(fout, P, tile_interior, lb, lo, yw, cw, x, y, o, oo, eidx);
      }
    }
    if (MACRO) {
      mrho[(uint32_t)c] = rho;
      mux[(uint32_t)c] = ux;
      muy[(uint32_t)c] = uy;
    }

    if (m & M_IFACE) {
      // momentum exchange: every population pulled across the interface;
      // the link's interface point is its midpoint seen from its fluid node.
      // The 8 neighbour masks are loaded all at once (a load inside the
      // divergent loop below would cost one memory round trip per link).
      // The cell's links all belong to one body: its own if solid, else that
      // of its solid neighbours (a fluid cell is linked to one body at most).
      uint8_t nm[Q];
      nbr_masks(mask, P, x, y, nm);
      int bid = id;
#pragma unroll
      for (int a = 1; a < Q; ++a) bid = bid ? bid : (nm[a] & M_BODY);
      double bx, by;
      body_ref(ctl, P, bid, bx, by);
      const bool moving = bid == 1;  // u_s = 0 on the links of the static bodies
      double acc[3] = {0.0, 0.0, 0.0};
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
          const BodyDev &B = ctl->body;
          ugx = B.u - B.omega * (gy - B.y);
          ugy = B.v + B.omega * (gx - B.x);
        }
        const double fa = wgt(a) * P.rho0d + double(d[a]);
        const double lx = s * (cx(a) - ugx) * fa, ly = s * (cy(a) - ugy) * fa;
        acc[0] += lx;
        acc[1] += ly;
        acc[2] += (gx - bx) * ly - (gy - by) * lx;
      }
      // this cell's contribution goes to its slot; the finalize sums them
      double *o = me_out + (long long)imap[(uint32_t)c] * ME_STRIDE;
      o[0] = acc[0];
      o[1] = acc[1];
      o[2] = acc[2];
    }
    if (m & M_SAMPLE) {
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
      const double sxx = -pr - P.facd * double(pxx);
      const double sxy = -P.facd * double(pxy);
      const double syy = -pr - P.facd * double(pyy);
      // the node's stress goes to its record's slot; the finalize contracts
      // it with the aggregated weights
      double *g = sig_out + (long long)si_map[(uint32_t)c] * SIG_STRIDE;
      g[0] = sxx;
      g[1] = sxy;
      g[2] = syy;
    }
  }

  if (fin_prev && tile == 0) {
    // forces of the previous step (same slots and records: only static
    // bodies defer)
    __shared__ double lds[FIN_WAVES * 6];
    finalize_block<NT>(me_prev, sig_prev, recs, bt, ctl, hist, cap, maxb, lds);
  }
}

// Resident waves per SIMD the step kernels are compiled for: 8 for 4- and
// 2-byte storage (register budget 64 VGPRs and the SGPRs that allow 8 waves);
// FP64 needs more VGPRs and is left to the compiler.
template <typename S> constexpr int step_waves() { return sizeof(typename Store<S>::T) == 8 ? 1 : 8; }

template <typename S, int BX, int BY, bool MACRO, bool TRT, int AA>
__global__ void __launch_bounds__(BX *BY, step_waves<S>())
    k_step(const S *__restrict__ fin, S *__restrict__ fout, const uint8_t *__restrict__ mask,
           const StepArgs<typename Store<S>::T> P, Ctl *__restrict__ ctl,
           const SiRec *__restrict__ recs, const int *__restrict__ si_map,
           const int *__restrict__ imap, const BodyTab *__restrict__ bt, double *__restrict__ me_out,
           const double *__restrict__ me_prev, double *__restrict__ sig_out, const double *__restrict__ sig_prev,
           int fin_prev, double *__restrict__ hist, int cap, int maxb, typename Store<S>::T *__restrict__ mrho,
           typename Store<S>::T *__restrict__ mux, typename Store<S>::T *__restrict__ muy) {
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
  step_tile<S, BX, BY, MACRO, TRT, AA>(tile, fin, fout, mask, P, ctl, recs, si_map, imap, bt, me_out, me_prev, sig_out,
                                   sig_prev, fin_prev, hist, cap, maxb, mrho, mux, muy);
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
  int pending0;           // launch 0 finalizes the forces of the step before it
  int moving;             // forces are finalized by the body kernel instead
  // body-kernel arguments
  int perx, pery, maxp, maxslot;
  const double *pts;
  // AA pattern: the perimeter copies kept by the steps of parity 0 and 1
  void *ec[2];
};

// Lattice of every global tile of a batched launch, from the descriptors
// (tiles of lattice i are [tile0, tile0 + ntiles), in order): one thread per
// tile, binary search on tile0.
template <typename T>
__global__ void k_fill_tile_case(const CaseDesc<T> *__restrict__ cases, int ncases, int total,
                                 int *__restrict__ tile_case) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  int lo = 0, hi = ncases - 1;  // last lattice with tile0 <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cases[mid].tile0 <= t) lo = mid; else hi = mid - 1;
  }
  tile_case[t] = lo;
}

// Batched step: launch number `flip` (0 or 1, alternating) of a run over
// ncases lattices; the lattice of each tile comes from the tile table.
template <typename S, int BX, int BY, bool TRT>
__global__ void __launch_bounds__(BX *BY, step_waves<S>())
    k_step_batch(const CaseDesc<typename Store<S>::T> *__restrict__ cases,
                 const int *__restrict__ tile_case, int total_tiles, int per_xcd, int flip, int first) {
  using T = typename Store<S>::T;
  const int b = blockIdx.x;
  const int gtile = (b & 7) * per_xcd + (b >> 3);
  if (gtile >= total_tiles) return;
  // the lattice of this tile, then its description, read once
  const CaseDesc<T> *__restrict__ C = cases + tile_case[gtile];
  const StepArgs<T> P = C->P;
  const int par = C->cur0 ^ flip, pb = C->pbit0 ^ flip;
  const int fin_prev = C->moving ? 0 : (first ? C->pending0 : 1);
  const S *fin = (const S *)C->buf[par];
  S *fout = (S *)C->buf[par ^ 1];
  step_tile<S, BX, BY, false, TRT, 0>(gtile - C->tile0, fin, fout, C->mask, P, C->ctl, C->recs, C->si_map, C->imap,
                                   C->bt, C->me[pb], C->me[pb ^ 1], C->sig[pb], C->sig[pb ^ 1], fin_prev, C->hist,
                                   C->cap, C->maxb, nullptr, nullptr, nullptr);
}

// Batched step of lattices in the AA pattern (one population buffer each):
// the launch computing an odd step pulls and pushes (AA = 1), an even step
// stays in the cell (AA = 2), per lattice by its own step parity; the
// perimeter copies alternate with it (read: the previous step's, written:
// this step's).
template <typename S, bool TRT>
__global__ void __launch_bounds__(256, step_waves<S>())
    k_step_batch_aa(const CaseDesc<typename Store<S>::T> *__restrict__ cases,
                    const int *__restrict__ tile_case, int total_tiles, int per_xcd, int flip, int first) {
  using T = typename Store<S>::T;
  const int b = blockIdx.x;
  const int gtile = (b & 7) * per_xcd + (b >> 3);
  if (gtile >= total_tiles) return;
  const CaseDesc<T> *__restrict__ C = cases + tile_case[gtile];
  StepArgs<T> P = C->P;
  const int pb = C->pbit0 ^ flip;
  P.ec_in = C->ec[pb ^ 1];
  P.ec_out = C->ec[pb];
  const int fin_prev = C->moving ? 0 : (first ? C->pending0 : 1);
  S *F = (S *)C->buf[0];
  if (pb)
    step_tile<S, 64, 4, false, TRT, 1>(gtile - C->tile0, nullptr, F, C->mask, P, C->ctl, C->recs, C->si_map,
                                       C->imap, C->bt, C->me[pb], C->me[pb ^ 1], C->sig[pb], C->sig[pb ^ 1],
                                       fin_prev, C->hist, C->cap, C->maxb, nullptr, nullptr, nullptr);
  else
    step_tile<S, 64, 4, false, TRT, 2>(gtile - C->tile0, nullptr, F, C->mask, P, C->ctl, C->recs, C->si_map,
                                       C->imap, C->bt, C->me[pb], C->me[pb ^ 1], C->sig[pb], C->sig[pb ^ 1],
                                       fin_prev, C->hist, C->cap, C->maxb, nullptr, nullptr, nullptr);
}

template <int NT>
__global__ void __launch_bounds__(NT)
    k_finalize(const double *__restrict__ me, const double *__restrict__ sig, const SiRec *__restrict__ recs,
               const BodyTab *__restrict__ bt, Ctl *__restrict__ ctl, double *__restrict__ hist, int cap, int maxb) {
  __shared__ double lds[FIN_WAVES * 6];
  finalize_block<NT>(me, sig, recs, bt, ctl, hist, cap, maxb, lds);
}

}  // namespace vp
