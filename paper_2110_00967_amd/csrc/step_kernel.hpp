// step_kernel.hpp -- the fused VP-LBM time step for gfx950.
//
// One thread updates one cell x of step n (state between steps: the
// post-collision deviations d~^{n-1} in buffer A, structure of arrays
// [9][ny][pitch]):
//   1. pull streaming  f^n_a(x) = f~^{n-1}_a(x - c_a)   (Eq. eqBd) with the
//      edge rules (periodic, half-way bounce-back, specular, zero-gradient);
//   2. rho = sum f, m = sum c f; penalized velocity
//      u = (m + G/2 + k/2 rho u_s) / (rho (1 + k/2)), k = chi/eta
//      (Eqs. updatestep, updatestep3, updatestepm) and force density
//      F = G - rho k (u - u_s)  (penalization term of Eq. 1);
//   3. f^eq (Sec. 2.2), forcing term in the form of Guo et al. (cited for
//      F_alpha in Eq. eqBd) with the (1 - 1/(2 tau)) prefactor of Eq. TRT,
//      BGK relaxation, store into buffer B;
//   4. interface cells: momentum exchange (Eq. MMEL) of every pulled
//      population that crossed the solid/fluid boundary -- the same link sum
//      as Sec. 2.3.1 evaluated on f~^{n-1}, gathered per destination;
//   5. sample cells: stress (Sec. 2.3.2 sigma) of the streamed populations,
//      contracted with the node's aggregated integration weights (Eq. defFf);
//   6. blocks inside the force window reduce (ME, SI) in FP64 with wave
//      shuffles and LDS and write one partial per block (two partial buffers,
//      alternating by step); block 0 of the next step -- after the kernel
//      boundary made them visible -- sums the previous step's partials in
//      window order (deterministic) into the force-history ring.
// HBM traffic per cell: 9 loads + 9 stores of the storage type + 1 mask byte.
#pragma once

#include "d2q9.hpp"

namespace vp {

template <typename T> struct StepArgs {
  int nx, ny, pitch;
  long long plane;      // ny * pitch
  int tiles_x, ntiles, per_xcd;
  int kind[4];          // edge kinds W, E, S, N
  T wu[4][2];           // 6 rho0 u_w of each edge: bounce-back increment w_a c_a . wu
  T omega, fac, kpen, rho0, gx, gy;
  int trt;              // 0: BGK; 1: TRT (the kernel is chosen accordingly)
  T omega_m, fac_m;     // TRT: 1/tau- and 1 - 1/(2 tau-)
  double facd, rho0d;
};

// Value of deviation a arriving at (x, y) when x - c_a leaves the lattice:
// axis by axis, x first; periodic wraps, outflow clamps, free-slip takes the
// mirrored population of the edge cell itself, velocity bounces back the
// cell's own opposite population with the moving-wall increment.
template <typename S, typename T>
__device__ __forceinline__ T pull_edge(const S *__restrict__ fin, const StepArgs<T> &P, int x,
                                       int y, int a, int cxa, int cya) {
  int sx = x - cxa, sy = y - cya, pop = a;
  // edge parameters are selected with constant indices only (no dynamic
  // indexing of the by-value argument block, which would spill it)
  if (sx < 0 || sx >= P.nx) {
    const bool w = sx < 0;
    const int k = w ? P.kind[WEST] : P.kind[EAST];
    if (k == EDGE_VELOCITY)
      return Store<S>::ld(fin + (long long)opp(a) * P.plane + (long long)y * P.pitch + x) +
             T(wgt(a)) * (w ? T(cxa) * P.wu[WEST][0] + T(cya) * P.wu[WEST][1]
                            : T(cxa) * P.wu[EAST][0] + T(cya) * P.wu[EAST][1]);
    if (k == EDGE_PERIODIC) sx = sx < 0 ? sx + P.nx : sx - P.nx;
    else if (k == EDGE_OUTFLOW) sx = sx < 0 ? 0 : P.nx - 1;
    else { sx = x; pop = flipx(pop); }
  }
  if (sy < 0 || sy >= P.ny) {
    const bool s_ = sy < 0;
    const int k = s_ ? P.kind[SOUTH] : P.kind[NORTH];
    if (k == EDGE_VELOCITY)
      return Store<S>::ld(fin + (long long)opp(a) * P.plane + (long long)y * P.pitch + x) +
             T(wgt(a)) * (s_ ? T(cxa) * P.wu[SOUTH][0] + T(cya) * P.wu[SOUTH][1]
                             : T(cxa) * P.wu[NORTH][0] + T(cya) * P.wu[NORTH][1]);
    if (k == EDGE_PERIODIC) sy = sy < 0 ? sy + P.ny : sy - P.ny;
    else if (k == EDGE_OUTFLOW) sy = sy < 0 ? 0 : P.ny - 1;
    else { sy = y; pop = flipy(pop); }
  }
  return Store<S>::ld(fin + (long long)pop * P.plane + (long long)sy * P.pitch + sx);
}

template <int NT>
__device__ __forceinline__ void block_reduce6(double (&v)[6], double *lds /*[NT/64][6]*/) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double s = v[i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    v[i] = s;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) lds[wave * 6 + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += lds[w * 6 + i];
      v[i] = s;
    }
  }
}

// Fixed-order sum of one step's window partials -> force-history slot of the
// next unfinished step (deterministic: same window, same order, same sum).
template <int NT>
__device__ __forceinline__ void finalize_block(const double *__restrict__ part, int nwx, int nwy,
                                               Ctl *__restrict__ ctl, double *__restrict__ hist, int cap,
                                               double *lds) {
  const int nwin = (nwx > 0 && nwy > 0) ? nwx * nwy : 0;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < nwin; t += NT) {
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] += part[(long long)t * PART_STRIDE + i];
  }
  block_reduce6<NT>(v, lds);
  if (threadIdx.x == 0) {
    const long long n = ctl->step + 1;
    double *h = hist + (n % cap) * 6;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      h[i] = v[i];
      ctl->last[i] = v[i];
    }
    ctl->step = n;
  }
}

// One workgroup's tile of the step (tile < P.ntiles): the body of the step
// kernel, shared by the single-lattice and the batched launch.  The
// workgroup of tile 0 also finalizes the previous step's forces (fin_prev).
template <typename S, int BX, int BY, bool MACRO, bool TRT>
__device__ __forceinline__ void step_tile(
    int tile, const S *__restrict__ fin, S *__restrict__ fout, const uint8_t *__restrict__ mask,
    const StepArgs<typename Store<S>::T> P, Ctl *__restrict__ ctl, const SiRec *__restrict__ recs,
    const int *__restrict__ si_map, double *__restrict__ part_out, const double *__restrict__ part_prev,
    int fin_prev, double *__restrict__ hist, int cap, typename Store<S>::T *__restrict__ mrho,
    typename Store<S>::T *__restrict__ mux, typename Store<S>::T *__restrict__ muy) {
  using T = typename Store<S>::T;
  constexpr int NT = BX * BY;
  const int tx = tile % P.tiles_x, ty = tile / P.tiles_x;
  const int lx = threadIdx.x % BX, ly = threadIdx.x / BX;
  const int x = tx * BX + lx, y = ty * BY + ly;

  const int wx0 = ctl->win[0] / BX, wy0 = ctl->win[1] / BY;
  const int wx1 = (ctl->win[2] + BX - 1) / BX, wy1 = (ctl->win[3] + BY - 1) / BY;
  const bool inwin = tx >= wx0 && tx < wx1 && ty >= wy0 && ty < wy1;

  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};

  if (x < P.nx && y < P.ny) {
    const long long c = (long long)y * P.pitch + x;
    const uint8_t m = mask[c];
    T d[Q];
    const bool interior = (x > 0) & (x < P.nx - 1) & (y > 0) & (y < P.ny - 1);
    if (interior) {
#pragma unroll
      for (int a = 0; a < Q; ++a)
        d[a] = Store<S>::ld(fin + a * P.plane + c - (long long)cy(a) * P.pitch - cx(a));
    } else {
#pragma unroll
      for (int a = 0; a < Q; ++a) d[a] = pull_edge<S, T>(fin, P, x, y, a, cx(a), cy(a));
    }

    // moments (of the deviations: sum w = 1, sum w c = 0)
    const T drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    const T mx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    const T my = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
    const T rho = P.rho0 + drho;

    T k = T(0), usx = T(0), usy = T(0);
    const bool chi = (m & M_SOLID) != 0;
    if (chi) {
      k = P.kpen;
      const BodyDev B = ctl->body;
      usx = T(B.u - B.omega * (double(y) - B.y));
      usy = T(B.v + B.omega * (double(x) - B.x));
    }
    const T hx = mx + T(0.5) * P.gx, hy = my + T(0.5) * P.gy;
    const T den = T(1) / (rho * (T(1) + T(0.5) * k));
    const T ux = (hx + T(0.5) * k * rho * usx) * den;
    const T uy = (hy + T(0.5) * k * rho * usy) * den;
    const T kk = k / (T(1) + T(0.5) * k);
    const T Fx = P.gx - kk * (hx - rho * usx);
    const T Fy = P.gy - kk * (hy - rho * usy);

    const T uu15 = T(1.5) * (ux * ux + uy * uy);
    const T uF3 = T(3) * (ux * Fx + uy * Fy);
    T deq[Q];
    if constexpr (!TRT) {
      // BGK
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const T w = T(wgt(a));
        const T cu = T(cx(a)) * ux + T(cy(a)) * uy;
        const T cF = T(cx(a)) * Fx + T(cy(a)) * Fy;
        deq[a] = w * drho + w * rho * (T(3) * cu + T(4.5) * cu * cu - uu15);
        const T Fa = w * (T(3) * cF - uF3 + T(9) * cu * cF);
        const T out = d[a] - P.omega * (d[a] - deq[a]) + P.fac * Fa;
        Store<S>::st(fout + a * P.plane + c, out);
      }
    } else {
      // TRT (Eq. TRT): even / odd parts of the non-equilibrium and of the
      // forcing term relax with tau+ / tau-
      T Fa[Q];
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const T w = T(wgt(a));
        const T cu = T(cx(a)) * ux + T(cy(a)) * uy;
        const T cF = T(cx(a)) * Fx + T(cy(a)) * Fy;
        deq[a] = w * drho + w * rho * (T(3) * cu + T(4.5) * cu * cu - uu15);
        Fa[a] = w * (T(3) * cF - uF3 + T(9) * cu * cF);
      }
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const int o = opp(a);
        const T nep = T(0.5) * ((d[a] - deq[a]) + (d[o] - deq[o]));
        const T nem = T(0.5) * ((d[a] - deq[a]) - (d[o] - deq[o]));
        const T out = d[a] - P.omega * nep - P.omega_m * nem + P.fac * (T(0.5) * (Fa[a] + Fa[o])) +
                      P.fac_m * (T(0.5) * (Fa[a] - Fa[o]));
        Store<S>::st(fout + a * P.plane + c, out);
      }
    }
    if (MACRO) {
      mrho[c] = rho;
      mux[c] = ux;
      muy[c] = uy;
    }

    if (m & M_IFACE) {
      // momentum exchange: every population pulled across the interface;
      // the link's interface point is its midpoint seen from its fluid node
      const BodyDev B = ctl->body;
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
        if (!link) continue;
        const bool schi = (mask[(long long)sy * P.pitch + sx] & M_SOLID) != 0;
        if (schi == chi) continue;
        double gx, gy, s;
        if (chi) { gx = sx + 0.5 * cx(a); gy = sy + 0.5 * cy(a); s = 1.0; }
        else { gx = x - 0.5 * cx(a); gy = y - 0.5 * cy(a); s = -1.0; }
        const double ugx = B.u - B.omega * (gy - B.y), ugy = B.v + B.omega * (gx - B.x);
        const double fa = wgt(a) * P.rho0d + double(d[a]);
        const double lx = s * (cx(a) - ugx) * fa, ly = s * (cy(a) - ugy) * fa;
        acc[0] += lx;
        acc[1] += ly;
        acc[2] += (gx - B.x) * ly - (gy - B.y) * lx;
      }
    }
    if (m & M_SAMPLE) {
      // stress of the streamed populations at a (fluid) sample node
      T pxx = T(0), pxy = T(0), pyy = T(0);
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        const T ne = d[a] - deq[a];
        pxx += T(cx(a) * cx(a)) * ne;
        pxy += T(cx(a) * cy(a)) * ne;
        pyy += T(cy(a) * cy(a)) * ne;
      }
      const double pr = double(drho) / 3.0;
      const double sxx = -pr - P.facd * double(pxx);
      const double sxy = -P.facd * double(pxy);
      const double syy = -pr - P.facd * double(pyy);
      const SiRec R = recs[si_map[c]];
      acc[3] += sxx * R.ax + sxy * R.ay;
      acc[4] += sxy * R.ax + syy * R.ay;
      acc[5] += sxx * R.txx + sxy * R.txy + syy * R.tyy;
    }
  }

  __shared__ double lds[(NT / 64) * 6];
  if (inwin) {
    block_reduce6<NT>(acc, lds);
    if (threadIdx.x == 0) {
      double *o = part_out + (long long)((ty - wy0) * (wx1 - wx0) + (tx - wx0)) * PART_STRIDE;
#pragma unroll
      for (int i = 0; i < 6; ++i) o[i] = acc[i];
    }
  }
  if (fin_prev && tile == 0) {
    // forces of the previous step (same window: only static bodies defer)
    __syncthreads();
    finalize_block<NT>(part_prev, wx1 - wx0, wy1 - wy0, ctl, hist, cap, lds);
  }
}

template <typename S, int BX, int BY, bool MACRO, bool TRT>
__global__ void __launch_bounds__(BX *BY)
    k_step(const S *__restrict__ fin, S *__restrict__ fout, const uint8_t *__restrict__ mask,
           const StepArgs<typename Store<S>::T> P, Ctl *__restrict__ ctl,
           const SiRec *__restrict__ recs, const int *__restrict__ si_map,
           double *__restrict__ part_out, const double *__restrict__ part_prev, int fin_prev,
           double *__restrict__ hist, int cap, typename Store<S>::T *__restrict__ mrho,
           typename Store<S>::T *__restrict__ mux, typename Store<S>::T *__restrict__ muy) {
  // XCD-aware tile order: consecutive workgroups go round-robin over the 8
  // XCDs, so give each XCD a contiguous band of tiles (shared halo lines stay
  // in that XCD's L2).
  const int b = blockIdx.x;
  const int tile = (b & 7) * P.per_xcd + (b >> 3);
  if (tile >= P.ntiles) return;
  step_tile<S, BX, BY, MACRO, TRT>(tile, fin, fout, mask, P, ctl, recs, si_map, part_out, part_prev, fin_prev,
                                   hist, cap, mrho, mux, muy);
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
  double *part[2];        // partial sums of steps with parity 0 and 1
  double *hist;
  int cap;
  int tile0;              // first global tile of this lattice
  int cur0;               // parity of the buffer holding the state at launch 0
  int pbit0;              // parity of the step computed by launch 0
  int pending0;           // launch 0 finalizes the forces of the step before it
  int moving;             // forces are finalized by the body kernel instead
  // body-kernel arguments
  int tw, by, perx, pery, maxp;
  const double *pts;
};

// Batched step: launch number `flip` (0 or 1, alternating) of a run over
// ncases lattices; the lattice of a tile is found by binary search on tile0.
template <typename S, int BX, int BY, bool TRT>
__global__ void __launch_bounds__(BX *BY)
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
  double *pout = C->part[pb];
  const double *pprev = C->part[pb ^ 1];
  step_tile<S, BX, BY, false, TRT>(gtile - C->tile0, fin, fout, C->mask, P, C->ctl, C->recs, C->si_map, pout, pprev,
                              fin_prev, C->hist, C->cap, nullptr, nullptr, nullptr);
}

template <int NT>
__global__ void __launch_bounds__(NT)
    k_finalize(const double *__restrict__ part, Ctl *__restrict__ ctl, double *__restrict__ hist, int cap,
               int BX, int BY) {
  __shared__ double lds[(NT / 64) * 6];
  const int wx0 = ctl->win[0] / BX, wy0 = ctl->win[1] / BY;
  const int wx1 = (ctl->win[2] + BX - 1) / BX, wy1 = (ctl->win[3] + BY - 1) / BY;
  finalize_block<NT>(part, wx1 - wx0, wy1 - wy0, ctl, hist, cap, lds);
}

}  // namespace vp
