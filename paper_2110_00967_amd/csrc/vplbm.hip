// vplbm.hip -- host side of the VP-LBM library: the C ABI of include/vplbm.h.
//
// Device memory of one lattice (carved from one buffer, 256-byte aligned):
//   A, B     : populations, 9 ny pitch elements of the storage type, runs of
//              64 cells x 9 populations (pop_index; ping-pong;
//              one buffer only with the AA pattern, plus its perimeter copies)
//   mask     : [ny][pitch] bytes (bits 0-5 body id, 6 SI sample, 7 interface)
//   macro    : rho, ux, uy [ny][pitch] of the compute type (written on request)
//   si_map   : [ny][pitch] int, record index of a sample node
//   imap     : [ny][pitch] int, momentum-exchange slot of an interface cell
//   me, sig  : per-interface-cell ME sums and per-record stresses, by parity
//   hist     : force-history ring [cap][max_bodies][6] doubles
//   ctl, bt  : control block (body 1 state, window, counters), per-body ranges
//   recs     : stress-integration records, pts: SI points [6][maxp]
//   verts    : polygon vertices on the 1/4096 grid [2][maxv] int64
//   staging  : bounded host<->device staging for setup and readback
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vplbm.h"
#include "d2q9.hpp"
#include "geometry_kernels.hpp"
#include "step_kernel.hpp"

using namespace vp;

// launch a kernel after dropping any error an unrelated HIP call left pending,
// so that the check right after the launch reports this launch only
#define VP_LAUNCH(...)           \
  do {                           \
    (void)hipGetLastError();     \
    hipLaunchKernelGGL(__VA_ARGS__); \
  } while (0)

namespace {

constexpr size_t ALIGN = 256;
constexpr size_t STAGE_DOUBLES = 1 << 18;  // 2 MiB staging
constexpr int DEFAULT_HIST = 4096;
constexpr int DEFAULT_PTS = 4096;
constexpr int DEFAULT_VERTS = 4096;
constexpr int WG_SLOTS_PER_XCD = 256;  // 32 CUs x 8 resident workgroups of the step kernel
constexpr int ROT_MAX_ROUNDS = 16;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_size(int prec) { return prec == VPLBM_F64 ? 8 : (prec == VPLBM_F32 ? 4 : 2); }
size_t compute_size(int prec) { return prec == VPLBM_F64 ? 8 : 4; }

int pitch_of(const vplbm_params &p) {
  // rows start on 256-byte boundaries for every storage type
  const int q = (int)(ALIGN / elem_size(p.precision));
  return (int)align_up((size_t)p.nx, (size_t)std::max(q, 64));
}

struct Layout {
  size_t A, B, ec, ec_stride, mask, mrho, mux, muy, si_map, imap, me, me_stride, sig, sig_stride, cbc, hist, ctl, bt, bodies,
      movers, recs, pts, verts, staging, siout, total;
};

int max_bodies_of(const vplbm_params &p) { return p.max_bodies > 0 ? p.max_bodies : 1; }
// interface cells (momentum-exchange slots): the given capacity, or room for
// a boundary 16 cells thick along the whole lattice perimeter
long long max_slots_of(const vplbm_params &p) {
  if (p.max_interface_cells > 0) return p.max_interface_cells;
  return std::min<long long>((long long)p.nx * p.ny, 32LL * ((long long)p.nx + p.ny));
}

Layout layout_of(const vplbm_params &p) {
  Layout L{};
  const int pitch = pitch_of(p);
  const size_t cells = (size_t)p.ny * pitch;
  const int cap = p.hist_capacity > 0 ? p.hist_capacity : DEFAULT_HIST;
  const int maxp = p.max_si_points > 0 ? p.max_si_points : DEFAULT_PTS;
  const int maxv = p.max_vertices > 0 ? p.max_vertices : DEFAULT_VERTS;
  const size_t maxb = (size_t)max_bodies_of(p);
  const size_t maxslot = (size_t)max_slots_of(p);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, ALIGN);
    return at;
  };
  L.A = take(9 * cells * elem_size(p.precision));
  // the AA pattern keeps one population buffer, plus its perimeter cells'
  // post-collision populations from the last two launches
  const bool aa = p.streaming == VPLBM_STREAM_AA;
  L.B = aa ? L.A : take(9 * cells * elem_size(p.precision));
  L.ec_stride = aa ? align_up((size_t)9 * perim_count(p.nx, p.ny) * elem_size(p.precision), ALIGN) : 0;
  L.ec = take(2 * L.ec_stride);
  L.mask = take(cells);
  L.mrho = take(cells * compute_size(p.precision));
  L.mux = take(cells * compute_size(p.precision));
  L.muy = take(cells * compute_size(p.precision));
  L.si_map = take(cells * sizeof(int));
  L.imap = take(cells * sizeof(int));
  // momentum exchange of each interface cell, by step parity
  L.me_stride = maxslot * ME_STRIDE * sizeof(double);
  L.me = take(2 * L.me_stride);
  L.hist = take((size_t)cap * maxb * 6 * sizeof(double));
  L.ctl = take(sizeof(Ctl));
  L.bt = take((size_t)MAX_BODIES * sizeof(BodyTab));
  L.bodies = take((size_t)(MAX_BODIES + 1) * sizeof(BodyDev));
  L.movers = take((size_t)MAX_MOVERS * sizeof(MoverDev));
  // one record per distinct sample node: up to 4 per point with the interpolated rule
  const size_t maxrec = (size_t)maxp * (p.si_rule == 1 ? 4 : 1);
  L.recs = take(maxrec * sizeof(SiRec));
  // stress of each sample node, by step parity (read back by the finalize)
  L.sig_stride = maxrec * SIG_STRIDE * sizeof(double);
  L.sig = take(2 * L.sig_stride);
  // convective-edge state: 3 incoming populations along each of the 4 edges
  L.cbc = take((size_t)3 * (2 * (size_t)p.ny + 2 * (size_t)p.nx) * compute_size(p.precision));
  L.pts = take((size_t)6 * maxp * sizeof(double));  // x, y, nx, ny, ds, body
  L.verts = take((size_t)2 * maxv * sizeof(long long));
  L.staging = take(STAGE_DOUBLES * sizeof(double));
  L.siout = take(8 * sizeof(double));
  L.total = o;
  return L;
}

bool valid_edge(const vplbm_edge &e) {
  return e.kind >= VPLBM_BC_PERIODIC && e.kind <= VPLBM_BC_CONVECTIVE && std::isfinite(e.ux) &&
         std::isfinite(e.uy) && (e.kind != VPLBM_BC_CONVECTIVE || e.ux >= 0.0);
}

const char *check_params(const vplbm_params *p) {
  if (!p) return "params is NULL";
  if (p->nx < 4 || p->ny < 4) return "nx and ny must be >= 4";
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return "tau must be finite and > 1/2";
  if (!(p->eta > 0.0)) return "eta must be > 0 (or +inf)";
  if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return "rho0 must be finite and > 0";
  if (p->precision < VPLBM_F64 || p->precision > VPLBM_F16DEV) return "unknown precision";
  if (!valid_edge(p->west) || !valid_edge(p->east) || !valid_edge(p->south) || !valid_edge(p->north))
    return "invalid edge condition";
  if ((p->west.kind == VPLBM_BC_PERIODIC) != (p->east.kind == VPLBM_BC_PERIODIC))
    return "west and east must both be periodic or both not";
  if ((p->south.kind == VPLBM_BC_PERIODIC) != (p->north.kind == VPLBM_BC_PERIODIC))
    return "south and north must both be periodic or both not";
  if (!(p->trt_lambda >= 0.0) || !std::isfinite(p->trt_lambda)) return "trt_lambda must be finite and >= 0";
  if (p->hist_capacity < 0 || p->max_si_points < 0 || p->max_vertices < 0 || p->max_bodies < 0 ||
      p->max_interface_cells < 0)
    return "capacities must be >= 0";
  if (p->max_bodies > MAX_BODIES) return "max_bodies exceeds 63";
  if (p->streaming != VPLBM_STREAM_AB && p->streaming != VPLBM_STREAM_AA)
    return "streaming must be VPLBM_STREAM_AB or VPLBM_STREAM_AA";
  if (p->max_si_points > SI_MAX) return "max_si_points exceeds 4096";
  if (p->si_rule != 0 && p->si_rule != 1) return "si_rule must be 0 or 1";
  if (p->si_rule == 1 && (p->max_si_points == 0 || p->max_si_points > SI_MAX / 4))
    return "si_rule 1 needs max_si_points in 1..1024";
  const long long pitch = pitch_of(*p);
  if ((long long)p->ny * pitch >= (1LL << 31)) return "lattice too large (ny * pitch cells must be < 2^31)";
  return nullptr;
}

}  // namespace

struct vplbm_lattice {
  vplbm_params p{};
  Layout L{};
  int pitch = 0;
  long long plane = 0;
  hipStream_t stream = nullptr;
  char *base = nullptr;
  bool owns = false;
  int cur = 0;  // 0: A holds the state, 1: B
  long long nstep = 0;
  bool pending = false;  // forces of the last step not yet summed into the history
  // force window (cells) of a static body, cached for the step kernel's tile
  // order; refreshed from the device after geometry changes
  int pwin[4] = {0, 0, 0, 0};
  bool pwin_ok = false;
  bool initialized = false;
  bool macro_valid = false;
  int cap = 0, maxp = 0, maxv = 0, maxb = 1;
  long long maxslot = 0;
  int nbody = 1;                          // bodies in the mask (ids 1..nbody)
  std::vector<double> refs;               // static multi-body: reference point of each body [2][nbody]
  // points registered per body, [5][n] each (index = body id); only body 1
  // when the lattice holds one body
  std::vector<std::vector<double>> si_sets = std::vector<std::vector<double>>(MAX_BODIES + 1);
  int bx = 64, by = 4;  // step tile shape
  double gx = 0.0, gy = 0.0;
  int shape = SHAPE_NONE, mode = MODE_STATIC;
  double disk_r = 0.0;
  // moving disks (mover.hpp): their number, host copies of their set-up, and
  // whether the forces of the last step are still to be summed into their
  // states (vplbm_sync and every read do it)
  int nmov = 0;
  std::vector<MoverDev> movers;
  bool mov_pending = false;
  int npts = 0;
  std::vector<double> si_world;  // host copy of the registered world points [5][npts]
  std::vector<int> si_body;      // body of each registered point (1..nbody)
  std::string err;

  char *at(size_t off) const { return base + off; }
  bool aa() const { return p.streaming == VPLBM_STREAM_AA; }
  // AA: perimeter copy written by the launch of step n (the initialization
  // counts as step 0)
  void *ec(long long n) const { return at(L.ec + (size_t)(n & 1) * L.ec_stride); }
  // layout of the post-collision state between steps (see load_post)
  int layout() const { return aa() ? ((nstep & 1) ? 2 : 1) : 0; }
  void *A() const { return at(cur == 0 ? L.A : L.B); }
  void *Bbuf() const { return at(cur == 0 ? L.B : L.A); }
  uint8_t *mask() const { return (uint8_t *)at(L.mask); }
  Ctl *ctl() const { return (Ctl *)at(L.ctl); }
  // interface contributions and sample stresses written by step n live in buffer n % 2
  double *me(long long n) const { return (double *)at(L.me + (size_t)(n & 1) * L.me_stride); }
  int *imap() const { return (int *)at(L.imap); }
  BodyTab *bt() const { return (BodyTab *)at(L.bt); }
  BodyDev *bodies() const { return (BodyDev *)at(L.bodies); }
  int *err_dev() const { return (int *)((char *)ctl() + offsetof(Ctl, err)); }
  double *sig(long long n) const { return (double *)at(L.sig + (size_t)(n & 1) * L.sig_stride); }
  const SiRec *recs() const { return (const SiRec *)at(L.recs); }
  MoverDev *movers_dev() const { return (MoverDev *)at(L.movers); }

  int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }
  int hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return VPLBM_OK;
    return fail(VPLBM_EHIP, "%s: %s", what, hipGetErrorString(e));
  }
  int launched(const char *what) { return hip(hipGetLastError(), what); }
  // drop an error left pending by an unrelated HIP call before our own work
  void clear_stale() { (void)hipGetLastError(); }
  int sync() { return hip(hipStreamSynchronize(stream), "hipStreamSynchronize"); }

  int ctl_pull(Ctl &c) {
    int rc = hip(hipMemcpyAsync(&c, ctl(), sizeof(Ctl), hipMemcpyDeviceToHost, stream), "ctl read");
    if (rc) return rc;
    return sync();
  }
  int ctl_push(const Ctl &c) {
    int rc = hip(hipMemcpyAsync(ctl(), &c, sizeof(Ctl), hipMemcpyHostToDevice, stream), "ctl write");
    if (rc) return rc;
    return sync();
  }

  bool periodic_x() const { return p.west.kind == VPLBM_BC_PERIODIC; }
  bool periodic_y() const { return p.south.kind == VPLBM_BC_PERIODIC; }

  // arguments of a step launch with tiles of tbx x tby cells (by default the
  // lattice's own tile; batched launches pass 64x4)
  template <typename T> StepArgs<T> step_args(int tbx = 0, int tby = 0) const {
    const int bx = tbx > 0 ? tbx : this->bx, by = tby > 0 ? tby : this->by;
    StepArgs<T> a{};
    a.nx = p.nx;
    a.ny = p.ny;
    a.pitch = pitch;
    a.plane = plane;
    a.tiles_x = (p.nx + bx - 1) / bx;
    // tile / tiles_x by multiply-high and one correction (see tile_cell)
    a.tx_magic = a.tiles_x == 1 ? 0u : (unsigned)(0xFFFFFFFFull / (unsigned)a.tiles_x);
    const int tiles_y = (p.ny + by - 1) / by;
    a.ntiles = a.tiles_x * tiles_y;
    a.per_xcd = (a.ntiles + 7) / 8;
    // rotate each XCD band that holds rows of a static body's force window to
    // start at the first of them, when the band is at most ROT_MAX_ROUNDS
    // rounds of workgroups deep (deeper bands absorb the slower tiles)
    if (pwin_ok && mode == MODE_STATIC && pwin[3] > pwin[1] &&
        a.per_xcd <= ROT_MAX_ROUNDS * WG_SLOTS_PER_XCD) {
      const int w0 = (pwin[1] / by) * a.tiles_x, w1 = ((pwin[3] + by - 1) / by) * a.tiles_x;
      for (int k = 0; k < 8; ++k) {
        const int s0 = k * a.per_xcd, len = std::min(a.per_xcd, a.ntiles - s0);
        if (len > 0 && w0 < s0 + len && w1 > s0) a.rot[k] = std::max(w0, s0) - s0;
      }
    }
    const vplbm_edge *E[4] = {&p.west, &p.east, &p.south, &p.north};
    for (int e = 0; e < 4; ++e) {
      a.kind[e] = E[e]->kind;
      a.wu[e][0] = T(6.0 * p.rho0 * E[e]->ux);
      a.wu[e][1] = T(6.0 * p.rho0 * E[e]->uy);
    }
    a.omega = T(1.0 / p.tau);
    a.fac = T(1.0 - 0.5 / p.tau);
    a.facd = 1.0 - 0.5 / p.tau;
    const double kpen = std::isinf(p.eta) ? 0.0 : 1.0 / p.eta;
    a.kpen = T(kpen);
    a.khalf = T(0.5 * kpen);
    a.a1 = T(1.0 / (1.0 + 0.5 * kpen));
    a.kk = T(kpen / (1.0 + 0.5 * kpen));
    a.trt = p.trt_lambda > 0.0 ? 1 : 0;
    const double tau_m = p.trt_lambda > 0.0 ? p.trt_lambda / (p.tau - 0.5) + 0.5 : p.tau;
    a.omega_m = T(1.0 / tau_m);
    a.fac_m = T(1.0 - 0.5 / tau_m);
    a.fo = T(p.tau - 0.5);
    a.fo9 = T(9.0 * (p.tau - 0.5));
    a.fo3 = T(3.0 * (tau_m - 0.5));
    a.rho0 = T(p.rho0);
    a.rho0d = p.rho0;
    a.gx = T(gx);
    a.gy = T(gy);
    a.cbc = (T *)at(L.cbc);
    a.bodies = bodies();
    a.nper = perim_count(p.nx, p.ny);
    a.ec_in = ec(nstep);
    a.ec_out = ec(nstep + 1);
    for (int e = 0; e < 4; ++e) {
      const double U = E[e]->kind == VPLBM_BC_CONVECTIVE ? E[e]->ux : 0.0;
      a.cbu[e] = T(U);
      a.cbi[e] = T(1.0 / (1.0 + U));
    }
    a.mov = movers_dev();
    a.nmov = nmov;
    a.pts = (const double *)at(L.pts);
    a.maxp = maxp;
    a.si_rule = p.si_rule;
    a.wblocks = 0;
    for (int k = 0; k < nmov; ++k) a.wblocks += hit_tiles(movers[k].half, MOV_BX) * hit_tiles(movers[k].half, MOV_BY);
    a.wblocks = (a.wblocks + 7) / 8 * 8;
    return a;
  }
};

// ----------------------------------------------------------------------------
// kernel dispatch
// ----------------------------------------------------------------------------
namespace {

// cache the force window of a static body for the tile order of the step
// kernel (one device read after a geometry change; a moving body's window
// lives on the device only)
int resolve_pwin(vplbm_lattice *L) {
  if (L->pwin_ok) return VPLBM_OK;
  L->pwin[0] = L->pwin[1] = L->pwin[2] = L->pwin[3] = 0;
  if (L->mode == MODE_STATIC) {
    Ctl c;
    const int rc = L->ctl_pull(c);
    if (rc) return rc;
    for (int k = 0; k < 4; ++k) L->pwin[k] = c.win[k];
  }
  L->pwin_ok = true;
  return VPLBM_OK;
}

template <typename S, int BX, int BY, int AA, bool MOV>
int launch_step_t(vplbm_lattice *L, bool macro) {
  using T = typename Store<S>::T;
  const StepArgs<T> a = L->step_args<T>();
  // with moving disks: the hit boxes' workgroups first (see k_step)
  const int grid = (MOV ? a.wblocks : 0) + 8 * a.per_xcd;
  // AA launches read and write the one buffer through fout
  const S *fin = AA == 0 ? (const S *)L->A() : nullptr;
  S *fout = (S *)L->Bbuf();
  T *r = (T *)L->at(L->L.mrho), *u = (T *)L->at(L->L.mux), *v = (T *)L->at(L->L.muy);
  const SiRec *recs = (const SiRec *)L->at(L->L.recs);
  const int *smap = (const int *)L->at(L->L.si_map);
  const long long n = L->nstep + 1;  // the step this launch computes
  double *mout = L->me(n);
  const double *mprev = L->me(n - 1);
  double *gout = L->sig(n);
  const double *gprev = L->sig(n - 1);
  const int fin_prev = L->pending ? 1 : 0;
  const int pb = (int)(n & 1), mpend = L->mov_pending ? 1 : 0;
  double *hist = (double *)L->at(L->L.hist);
  const int *imap = L->imap();
  const BodyTab *bt = L->bt();
#define VP_STEP_ARGS                                                                                              \
  dim3(grid), dim3(BX * BY), 0, L->stream, fin, fout, L->mask(), a, L->ctl(), recs, smap, imap, bt, mout, mprev, gout, \
      gprev, fin_prev, hist, L->cap, L->maxb, r, u, v, pb, mpend
  if (macro) {
    if (a.trt)
      VP_LAUNCH((k_step<S, BX, BY, true, true, AA, MOV>), VP_STEP_ARGS);
    else
      VP_LAUNCH((k_step<S, BX, BY, true, false, AA, MOV>), VP_STEP_ARGS);
  } else {
    if (a.trt)
      VP_LAUNCH((k_step<S, BX, BY, false, true, AA, MOV>), VP_STEP_ARGS);
    else
      VP_LAUNCH((k_step<S, BX, BY, false, false, AA, MOV>), VP_STEP_ARGS);
  }
#undef VP_STEP_ARGS
  return L->launched("k_step");
}

template <typename S> int launch_step_s(vplbm_lattice *L, bool macro) {
  if (L->nmov) {  // moving disks: 64x4 tiles (see vplbm_set_tile)
    if (L->bx != 64 || L->by != 4) return L->fail(VPLBM_EINVAL, "a lattice with moving disks runs the 64x4 tile only");
    if (!L->aa()) return launch_step_t<S, 64, 4, 0, true>(L, macro);
    return ((L->nstep + 1) & 1) ? launch_step_t<S, 64, 4, 1, true>(L, macro) : launch_step_t<S, 64, 4, 2, true>(L, macro);
  }
  if (L->aa()) {  // odd steps pull and push, even steps stay in the cell (64x4 tiles)
    if (L->bx != 64 || L->by != 4) return L->fail(VPLBM_EINVAL, "the AA pattern runs with the 64x4 tile only");
    return ((L->nstep + 1) & 1) ? launch_step_t<S, 64, 4, 1, false>(L, macro)
                                : launch_step_t<S, 64, 4, 2, false>(L, macro);
  }
  if (L->bx == 64 && L->by == 4) return launch_step_t<S, 64, 4, 0, false>(L, macro);
  if (L->bx == 128 && L->by == 2) return launch_step_t<S, 128, 2, 0, false>(L, macro);
  if (L->bx == 256 && L->by == 1) return launch_step_t<S, 256, 1, 0, false>(L, macro);
  if (L->bx == 64 && L->by == 1) return launch_step_t<S, 64, 1, 0, false>(L, macro);
  if (L->bx == 64 && L->by == 2) return launch_step_t<S, 64, 2, 0, false>(L, macro);
  if (L->bx == 128 && L->by == 1) return launch_step_t<S, 128, 1, 0, false>(L, macro);
  return L->fail(VPLBM_EINVAL, "unsupported tile shape %dx%d", L->bx, L->by);
}

int launch_step(vplbm_lattice *L, bool macro) {
  const int rc = resolve_pwin(L);
  if (rc) return rc;
  switch (L->p.precision) {
    case VPLBM_F64: return launch_step_s<double>(L, macro);
    case VPLBM_F32: return launch_step_s<float>(L, macro);
    default: return launch_step_s<__half>(L, macro);
  }
}

template <typename S>
int launch_init_s(vplbm_lattice *L, int row0, int nrows, int col0, int ncols, const double *r, const double *u,
                  const double *v, double ru, double uu, double vu) {
  dim3 blk(256), grd((ncols + 255) / 256, nrows);
  VP_LAUNCH((k_init<S>), grd, blk, 0, L->stream, (S *)L->A(), L->mask(), L->p.nx, L->p.ny,
                     L->pitch, row0, nrows, col0, ncols, r, u, v, ru, uu, vu, L->ctl(), L->p.rho0, (int)L->aa(),
                     (S *)L->ec(0), perim_count(L->p.nx, L->p.ny), (const MoverDev *)L->movers_dev(), L->nmov,
                     (int)(L->nstep & 1));
  return L->launched("k_init");
}

// rows [row0, row0 + nrows) x columns [col0, col0 + ncols); ncols < 0: all
int launch_init(vplbm_lattice *L, int row0, int nrows, const double *r, const double *u,
                const double *v, double ru, double uu, double vu, int col0 = 0, int ncols = -1) {
  if (ncols < 0) ncols = L->p.nx;
  switch (L->p.precision) {
    case VPLBM_F64: return launch_init_s<double>(L, row0, nrows, col0, ncols, r, u, v, ru, uu, vu);
    case VPLBM_F32: return launch_init_s<float>(L, row0, nrows, col0, ncols, r, u, v, ru, uu, vu);
    default: return launch_init_s<__half>(L, row0, nrows, col0, ncols, r, u, v, ru, uu, vu);
  }
}

// convective edges: their state starts from the populations just initialized
template <typename S> int launch_cbc_init_s(vplbm_lattice *L) {
  const StepArgs<typename Store<S>::T> a = L->step_args<typename Store<S>::T>();
  const int len = std::max(L->p.nx, L->p.ny);
  VP_LAUNCH((k_cbc_init<S>), dim3((len + 255) / 256, 4), dim3(256), 0, L->stream, (const S *)L->A(), a,
            (int)L->aa());
  return L->launched("k_cbc_init");
}

int init_cbc(vplbm_lattice *L) {
  const vplbm_edge *E[4] = {&L->p.west, &L->p.east, &L->p.south, &L->p.north};
  bool any = false;
  for (int e = 0; e < 4; ++e) any = any || E[e]->kind == VPLBM_BC_CONVECTIVE;
  if (!any) return VPLBM_OK;
  switch (L->p.precision) {
    case VPLBM_F64: return launch_cbc_init_s<double>(L);
    case VPLBM_F32: return launch_cbc_init_s<float>(L);
    default: return launch_cbc_init_s<__half>(L);
  }
}

template <typename S>
int launch_read_pop_s(vplbm_lattice *L, int x0, int w, int row0, int nrows, double *out) {
  dim3 blk(256), grd((w + 255) / 256, nrows);
  VP_LAUNCH((k_read_pop<S>), grd, blk, 0, L->stream, (const S *)L->A(), (const S *)L->ec(L->nstep),
            L->layout(), L->p.nx, L->p.ny, perim_count(L->p.nx, L->p.ny), x0, w, L->pitch, row0, nrows,
            L->p.rho0, out);
  return L->launched("k_read_pop");
}

int launch_read_pop(vplbm_lattice *L, int x0, int w, int row0, int nrows, double *out) {
  switch (L->p.precision) {
    case VPLBM_F64: return launch_read_pop_s<double>(L, x0, w, row0, nrows, out);
    case VPLBM_F32: return launch_read_pop_s<float>(L, x0, w, row0, nrows, out);
    default: return launch_read_pop_s<__half>(L, x0, w, row0, nrows, out);
  }
}

template <typename S> int launch_si_at_s(vplbm_lattice *L, int npts, double *out) {
  using T = typename Store<S>::T;
  const StepArgs<T> a = L->step_args<T>();
  VP_LAUNCH((k_si_at<S>), dim3(1), dim3(SI_NT), 0, L->stream, (const S *)L->A(), (const S *)L->ec(L->nstep),
            L->layout(), L->mask(),
                     a, L->ctl(), (const double *)L->at(L->L.staging), L->maxp, npts, out);
  return L->launched("k_si_at");
}

int launch_flags(vplbm_lattice *L, int x0, int y0, int x1, int y1) {
  if (x1 <= x0 || y1 <= y0) return VPLBM_OK;
  dim3 blk(256), grd((x1 - x0 + 255) / 256, y1 - y0);
  VP_LAUNCH(k_mask_flags, grd, blk, 0, L->stream, L->mask(), L->p.nx, L->p.ny, L->pitch, x0,
                     y0, x1, y1, (int)L->periodic_x(), (int)L->periodic_y(), L->err_dev());
  return L->launched("k_mask_flags");
}

int launch_si_select(vplbm_lattice *L) {
  VP_LAUNCH(k_si_select, dim3(1), dim3(SI_NT), 0, L->stream, L->mask(), L->ctl(),
                     (const double *)L->at(L->L.pts), L->maxp, (SiRec *)L->at(L->L.recs),
                     (int *)L->at(L->L.si_map), L->bt(), (const BodyDev *)L->bodies(), L->p.nx, L->p.ny,
                     L->pitch);
  return L->launched("k_si_select");
}

// The moving disks' forces of the last step summed and their states advanced
// (between steps, as the next step launch would do it), the mask bytes of
// their windows rewritten from the new states.
int flush_movers(vplbm_lattice *L) {
  if (!L->nmov || !L->mov_pending) return VPLBM_OK;
  const long long n = L->nstep;
  VP_LAUNCH(k_mover_flush, dim3(1), dim3(FLUSH_NT), 0, L->stream, L->movers_dev(), L->nmov,
            (const double *)L->me(n), (int)(n & 1), (const double *)L->at(L->L.pts), L->maxp, L->p.si_rule, L->p.nx,
            L->p.ny, L->pitch, (int)L->periodic_x(), (int)L->periodic_y(), L->mask(), L->ctl(),
            (double *)L->at(L->L.hist), L->cap, L->maxb);
  const int rc = L->launched("k_mover_flush");
  if (!rc) L->mov_pending = false;
  return rc;
}

// The mask of the moving disks' windows rewritten from their current
// states (no step pending: the state after nstep updates, slot nstep & 1).
int launch_mover_mask(vplbm_lattice *L) {
  VP_LAUNCH(k_mover_mask, dim3(1), dim3(FLUSH_NT), 0, L->stream, L->movers_dev(), L->nmov, (int)(L->nstep & 1),
            (const double *)L->at(L->L.pts), L->maxp, L->p.si_rule, L->p.nx, L->p.ny, L->pitch,
            (int)L->periodic_x(), (int)L->periodic_y(), L->mask(), L->ctl());
  return L->launched("k_mover_mask");
}

// sum the last step's force terms into the history (forces readable)
int flush(vplbm_lattice *L) {
  int rc = flush_movers(L);
  if (rc || !L->pending) return rc;
  VP_LAUNCH((k_finalize<256>), dim3(1), dim3(256), 0, L->stream, (const double *)L->me(L->nstep),
                     (const double *)L->sig(L->nstep), L->recs(), (const BodyTab *)L->bt(), L->ctl(),
                     (double *)L->at(L->L.hist), L->cap, L->maxb);
  rc = L->launched("k_finalize");
  if (!rc) L->pending = false;
  return rc;
}

// one time step: the step kernel.  Its force terms are summed by the next
// step launch (or by flush()): static bodies' by its first workgroup, moving
// disks' by every workgroup near them, which also advance the disks.
int one_step(vplbm_lattice *L, bool macro) {
  const int rc = launch_step(L, macro);
  if (rc) return rc;
  if (L->nmov)
    L->mov_pending = true;
  else
    L->pending = true;
  L->cur ^= 1;
  L->nstep += 1;
  return VPLBM_OK;
}

long long fixq(double v) { return llround(v * FIXQ); }

int pull_movers(vplbm_lattice *L) {
  L->movers.resize(MAX_MOVERS);
  if (!L->nmov) return VPLBM_OK;
  int rc = L->hip(hipMemcpyAsync(L->movers.data(), L->movers_dev(), sizeof(MoverDev) * L->nmov,
                                 hipMemcpyDeviceToHost, L->stream),
                  "movers read");
  if (!rc) rc = L->sync();
  return rc;
}

int push_movers(vplbm_lattice *L) {
  if (!L->nmov) return VPLBM_OK;
  int rc = L->hip(hipMemcpyAsync(L->movers_dev(), L->movers.data(), sizeof(MoverDev) * L->nmov,
                                 hipMemcpyHostToDevice, L->stream),
                  "movers write");
  if (!rc) rc = L->sync();
  return rc;
}

// Window half size of a moving disk: its radius or its farthest point from
// the reference point, whichever is larger, plus WIN_MARGIN (interface
// links, sample walks of up to four nodes along a diagonal, a cell of motion).
// (xr, yr): the reference point at which the points were registered.
int mover_half(const vplbm_lattice *L, double r, double xr, double yr, int pt0, int pt1) {
  double rmax = r;
  const int n = L->npts;
  for (int i = pt0; i < pt1; ++i) {
    const double dx = L->si_world[i] - xr, dy = L->si_world[n + i] - yr;
    rmax = std::max(rmax, std::sqrt(dx * dx + dy * dy));
  }
  return (int)std::ceil(rmax) + WIN_MARGIN;
}

// The tiles (MOV_BX x MOV_BY) a window of 2 h + 1 cells a side can meet,
// wherever it lies: its partial-sum grid, gx x gy.
void mover_grid(int h, int &gx, int &gy) {
  const int side = 2 * h + 1;
  gx = (side - 1 + MOV_BX - 1) / MOV_BX + 1;
  gy = (side - 1 + MOV_BY - 1) / MOV_BY + 1;
}

// The disks' tile partials live in the interface-slot buffers (one set per
// step parity): PART_ENTRY doubles per tile of each disk's grid, in slots of
// ME_STRIDE doubles.
int check_moving_capacity(vplbm_lattice *L, int nmov, const int *half) {
  long long need = 0;
  for (int k = 0; k < nmov; ++k) {
    int gx, gy;
    mover_grid(half[k], gx, gy);
    need += (long long)gx * gy;
  }
  need = need * PART_ENTRY / ME_STRIDE;
  if (need > L->maxslot)
    return L->fail(VPLBM_EINVAL, "max_interface_cells = %lld is below the moving disks' tile partials (%lld slots)",
                   L->maxslot, need);
  return VPLBM_OK;
}

// the window rectangle (clipped to the lattice) of a disk at (x, y)
void mover_rect(const vplbm_lattice *L, double x, double y, int h, int (&r)[4]) {
  const int ox = (int)std::floor(x) - h, oy = (int)std::floor(y) - h;
  r[0] = std::max(ox, 0);
  r[1] = std::max(oy, 0);
  r[2] = std::min(ox + 2 * h + 1, L->p.nx);
  r[3] = std::min(oy + 2 * h + 1, L->p.ny);
}

// Body 1, a disk with the motion c.mode (prescribed or free) and the state
// c.body, becomes a moving disk of the step kernel (mover.hpp): its states,
// dynamics, window and points go to the device.  The caller has checked the
// window capacity.
int become_mover(vplbm_lattice *L, const Ctl &c) {
  MoverDev m{};
  m.B[0] = m.B[1] = c.body;
  m.r = L->disk_r;
  m.mass = c.mass;
  m.inertia = c.inertia;
  m.gx = c.gx;
  m.gy = c.gy;
  m.buoy = c.buoy;
  m.R = fixq(L->disk_r);
  m.nfin = c.step;
  m.mode = c.mode;
  m.source = c.source;
  m.half = mover_half(L, L->disk_r, c.body.x, c.body.y, 0, L->npts);
  m.pt0 = 0;
  m.pt1 = L->npts;
  m.part0 = 0;
  mover_grid(m.half, m.ptx, m.pty);
  // the mask bytes the set-up wrote (the disk's region, the sample nodes):
  // within the window, which the first flush clears
  int r[4];
  mover_rect(L, c.body.x, c.body.y, m.half, r);
  for (int k = 0; k < 4; ++k) m.mwin[k] = r[k];
  m.mwin[0] = std::min(m.mwin[0], c.region[0]);
  m.mwin[1] = std::min(m.mwin[1], c.region[1]);
  m.mwin[2] = std::max(m.mwin[2], c.region[2]);
  m.mwin[3] = std::max(m.mwin[3], c.region[3]);
  L->movers.assign(MAX_MOVERS, MoverDev{});
  L->movers[0] = m;
  L->nmov = 1;
  L->mov_pending = false;
  L->bx = 64;  // the moving-disk step kernels run 64x4 tiles
  L->by = 4;
  return push_movers(L);
}


// the registered points of bodies 1..nbody, concatenated body by body
void rebuild_points(vplbm_lattice *L) {
  int n = 0;
  for (int b = 1; b <= L->nbody; ++b) n += (int)(L->si_sets[b].size() / 5);
  L->si_world.assign((size_t)5 * n, 0.0);
  L->si_body.assign(n, 1);
  int o = 0;
  for (int b = 1; b <= L->nbody; ++b) {
    const std::vector<double> &v = L->si_sets[b];
    const int m = (int)(v.size() / 5);
    for (int i = 0; i < m; ++i) {
      for (int k = 0; k < 5; ++k) L->si_world[(size_t)k * n + o + i] = v[(size_t)k * m + i];
      L->si_body[o + i] = b;
    }
    o += m;
  }
  L->npts = n;
}

// clear the mask and SI tables, reset the force window
int reset_geometry(vplbm_lattice *L, Ctl &c) {
  int rc = L->hip(hipMemsetAsync(L->mask(), 0, (size_t)L->p.ny * L->pitch, L->stream), "mask clear");
  if (rc) return rc;
  // the force window is never empty: with no body it is the first cell, so
  // the step kernel still publishes (zero) forces for every step
  c.win[0] = c.win[1] = 0;
  c.win[2] = c.win[3] = 1;
  c.region[0] = c.region[1] = c.region[2] = c.region[3] = 0;
  c.nrec = 0;
  c.nslot = 0;
  c.nbody = 1;
  L->nbody = 1;
  L->refs.clear();
  L->nmov = 0;  // a new geometry is static until a motion is set
  L->mov_pending = false;
  bool others = false;  // points of bodies 2.. go with their bodies
  for (int b = 2; b <= MAX_BODIES; ++b) {
    others = others || !L->si_sets[b].empty();
    L->si_sets[b].clear();
  }
  if (others) {
    rebuild_points(L);
    c.npts = L->npts;
  }
  rc = L->hip(hipMemsetAsync(L->bt(), 0, (size_t)MAX_BODIES * sizeof(BodyTab), L->stream), "body table clear");
  if (!rc) rc = L->hip(hipMemsetAsync(L->bodies(), 0, (size_t)(MAX_BODIES + 1) * sizeof(BodyDev), L->stream),
                       "bodies clear");
  return rc;
}

// reselect sample nodes after the mask or the points changed
int refresh_si(vplbm_lattice *L) {
  if (L->npts == 0) return VPLBM_OK;
  return launch_si_select(L);
}

int check_sample_error(vplbm_lattice *L) {
  Ctl c;
  int rc = L->ctl_pull(c);
  if (rc) return rc;
  const int e = c.err;
  if (e & 16) return L->fail(VPLBM_EUNSTABLE, "the solution diverged (a non-finite density at some step)");
  if (e & 32)
    return L->fail(VPLBM_EUNSTABLE, "a moving disk moved a cell or more in one step (or left the lattice)");
  if (e & 15) {
    c.err = 0;
    rc = L->ctl_push(c);
    if (rc) return rc;
  }
  if (e & 8)
    return L->fail(VPLBM_ESTATE, "more interface cells than max_interface_cells = %lld: the momentum exchange "
                                 "dropped some",
                   L->maxslot);
  if (e & 2) return L->fail(VPLBM_EINVAL, "a fluid cell is linked to two different bodies");
  if (e & 4) return L->fail(VPLBM_EINVAL, "a sample node serves two different bodies");
  if (e & 1)
    return L->fail(VPLBM_ENOSAMPLE, "a stress-integration point has no fluid sample node within 4 "
                                    "nodes along its normal");
  return VPLBM_OK;
}

// Number the interface cells (one momentum-exchange slot each), body by
// body and row-major inside a body, from the current mask: a solid cell
// belongs to its own body, a fluid one to the body of its solid lattice
// neighbours.  Writes imap, each body's slot range and nslot.
int number_interfaces(vplbm_lattice *L) {
  const int nx = L->p.nx, ny = L->p.ny, pitch = L->pitch;
  std::vector<uint8_t> m((size_t)ny * pitch);
  int rc = L->hip(hipMemcpyAsync(m.data(), L->mask(), m.size(), hipMemcpyDeviceToHost, L->stream), "mask read");
  if (!rc) rc = L->sync();
  if (rc) return rc;
  const bool px = L->periodic_x(), py = L->periodic_y();
  std::vector<std::vector<int>> cells(MAX_BODIES + 1);
  static const int CXH[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, CYH[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const uint8_t v = m[(size_t)j * pitch + i];
      if (!(v & M_IFACE)) continue;
      int b = v & M_BODY;
      for (int a = 1; a < 9 && !b; ++a) {
        int X = i + CXH[a], Y = j + CYH[a];
        if (X < 0 || X >= nx) {
          if (!px) continue;
          X = (X + nx) % nx;
        }
        if (Y < 0 || Y >= ny) {
          if (!py) continue;
          Y = (Y + ny) % ny;
        }
        b = m[(size_t)Y * pitch + X] & M_BODY;
      }
      if (b) cells[b].push_back(j * pitch + i);
    }
  std::vector<BodyTab> bt(MAX_BODIES);
  rc = L->hip(hipMemcpyAsync(bt.data(), L->bt(), bt.size() * sizeof(BodyTab), hipMemcpyDeviceToHost, L->stream),
              "body table read");
  if (!rc) rc = L->sync();
  if (rc) return rc;
  std::vector<int> pairs;
  int slot = 0;
  for (int b = 1; b <= MAX_BODIES; ++b) {
    bt[b - 1].me0 = slot;
    for (int c : cells[b]) {
      pairs.push_back(c);
      pairs.push_back(slot++);
    }
    bt[b - 1].me1 = slot;
  }
  if (slot > L->maxslot)
    return L->fail(VPLBM_EINVAL, "%d interface cells exceed max_interface_cells = %lld", slot, L->maxslot);
  // scatter the slot numbers through the staging buffer, in chunks
  int *stage = (int *)L->at(L->L.staging);
  const size_t chunk = STAGE_DOUBLES;  // pairs of ints per chunk (8 bytes each)
  for (size_t k = 0; k < pairs.size() / 2; k += chunk) {
    const size_t nk = std::min(chunk, pairs.size() / 2 - k);
    rc = L->hip(hipMemcpyAsync(stage, pairs.data() + 2 * k, nk * 2 * sizeof(int), hipMemcpyHostToDevice, L->stream),
                "slot upload");
    if (rc) return rc;
    VP_LAUNCH(k_scatter_slots, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, L->stream, (const int *)stage,
              (int)nk, L->imap());
    rc = L->launched("k_scatter_slots");
    if (!rc) rc = L->sync();
    if (rc) return rc;
  }
  rc = L->hip(hipMemcpyAsync(L->bt(), bt.data(), bt.size() * sizeof(BodyTab), hipMemcpyHostToDevice, L->stream),
              "body table write");
  if (rc) return rc;
  Ctl c;
  rc = L->ctl_pull(c);
  if (rc) return rc;
  c.nslot = slot;
  return L->ctl_push(c);
}

// store SI points (world frame or, for a moving body, body frame) in device memory
int upload_points(vplbm_lattice *L, const Ctl &c, const BodyDev *refs = nullptr) {
  const int n = L->npts, mp = L->maxp;
  std::vector<double> buf((size_t)6 * mp, 0.0);
  const bool moving = L->mode != MODE_STATIC;
  for (int i = 0; i < n; ++i) {
    const double x = L->si_world[i], y = L->si_world[n + i];
    const double nx = L->si_world[2 * n + i], ny = L->si_world[3 * n + i];
    const int b = L->si_body.empty() ? 1 : L->si_body[i];
    const BodyDev &R = refs ? refs[b - 1] : c.body;  // the body's state the points are given at
    const double co = std::cos(-R.theta), sn = std::sin(-R.theta);
    if (moving) {
      const double dx = x - R.x, dy = y - R.y;
      buf[i] = co * dx - sn * dy;
      buf[mp + i] = sn * dx + co * dy;
      buf[2 * mp + i] = co * nx - sn * ny;
      buf[3 * mp + i] = sn * nx + co * ny;
    } else {
      buf[i] = x;
      buf[mp + i] = y;
      buf[2 * mp + i] = nx;
      buf[3 * mp + i] = ny;
    }
    buf[4 * mp + i] = L->si_world[4 * n + i];
    buf[5 * mp + i] = L->si_body.empty() ? 1.0 : (double)L->si_body[i];
  }
  int rc = L->hip(hipMemcpyAsync(L->at(L->L.pts), buf.data(), buf.size() * sizeof(double),
                                 hipMemcpyHostToDevice, L->stream),
                  "SI points upload");
  if (rc) return rc;
  return L->sync();
}

}  // namespace

// ----------------------------------------------------------------------------
// C ABI
// ----------------------------------------------------------------------------
extern "C" {

size_t vplbm_required_bytes(const vplbm_params *p) {
  if (check_params(p)) return 0;
  return layout_of(*p).total;
}

// message of the last failed vplbm_create on this thread (no handle exists)
static thread_local std::string g_create_err;

int vplbm_create(const vplbm_params *p, void *dev_mem, size_t dev_bytes, void *hip_stream,
                 vplbm_lattice **out) {
  g_create_err.clear();
  if (!out) return VPLBM_EINVAL;
  *out = nullptr;
  if (const char *why = check_params(p)) {
    g_create_err = why;
    return VPLBM_EINVAL;
  }
  // an error left pending by an earlier, unrelated HIP call must not be
  // reported as ours
  (void)hipGetLastError();
  auto *L = new (std::nothrow) vplbm_lattice();
  if (!L) return VPLBM_ENOMEM;
  L->p = *p;
  L->L = layout_of(*p);
  L->pitch = pitch_of(*p);
  L->plane = (long long)p->ny * L->pitch;
  L->stream = (hipStream_t)hip_stream;
  L->cap = p->hist_capacity > 0 ? p->hist_capacity : DEFAULT_HIST;
  L->maxp = p->max_si_points > 0 ? p->max_si_points : DEFAULT_PTS;
  L->maxv = p->max_vertices > 0 ? p->max_vertices : DEFAULT_VERTS;
  L->maxb = max_bodies_of(*p);
  L->maxslot = max_slots_of(*p);
  // default step tile, the faster shape as measured on MI355X: 64x4, or
  // 128x2 for population buffers far beyond the 256 MB Infinity Cache (over
  // 1 GiB; FP64, at 6 waves per SIMD, from 256 MB).  The AA pattern runs
  // with 64x4.
  const double pop_bytes = 2.0 * 9.0 * (double)elem_size(p->precision) * (double)L->plane;
  const double wide_from = (p->precision == VPLBM_F64 ? 256.0 : 1024.0) * (1 << 20);
  if (!L->aa() && pop_bytes > wide_from) {
    L->bx = 128;
    L->by = 2;
  }
  if (dev_mem) {
    if (dev_bytes < L->L.total || ((uintptr_t)dev_mem % ALIGN) != 0) {
      g_create_err = "device buffer smaller than vplbm_required_bytes or not 256-byte aligned";
      delete L;
      return VPLBM_ENOMEM;
    }
    L->base = (char *)dev_mem;
  } else {
    if (hipMalloc((void **)&L->base, L->L.total) != hipSuccess) {
      (void)hipGetLastError();
      g_create_err = "hipMalloc failed";
      delete L;
      return VPLBM_ENOMEM;
    }
    L->owns = true;
  }
  Ctl c{};
  c.mode = MODE_STATIC;
  c.shape = SHAPE_NONE;
  c.si_rule = p->si_rule;
  int rc = reset_geometry(L, c);
  if (!rc) rc = L->ctl_push(c);
  if (!rc) rc = launch_init(L, 0, L->p.ny, nullptr, nullptr, nullptr, p->rho0, 0.0, 0.0);
  if (!rc) rc = L->sync();
  if (rc) {
    g_create_err = L->err;
    if (L->owns) (void)hipFree(L->base);
    delete L;
    return rc;
  }
  L->initialized = true;
  *out = L;
  return VPLBM_OK;
}

int vplbm_destroy(vplbm_lattice *L) {
  if (!L) return VPLBM_EINVAL;
  (void)hipStreamSynchronize(L->stream);
  if (L->owns) (void)hipFree(L->base);
  delete L;
  return VPLBM_OK;
}

const char *vplbm_last_error(const vplbm_lattice *L) { return L ? L->err.c_str() : g_create_err.c_str(); }

static int reset_counters(vplbm_lattice *L) {
  int rc = init_cbc(L);
  if (rc) return rc;
  Ctl c;
  rc = L->ctl_pull(c);
  if (rc) return rc;
  c.step = 0;
  for (int i = 0; i < 6; ++i) c.last[i] = 0.0;
  c.err = 0;
  rc = L->ctl_push(c);
  if (rc) return rc;
  if (L->nmov) {
    // moving disks restart from their current state (both slots), no step taken
    rc = pull_movers(L);
    if (rc) return rc;
    for (int k = 0; k < L->nmov; ++k) {
      MoverDev &m = L->movers[k];
      const BodyDev now = m.B[L->nstep & 1];
      m.B[0] = m.B[1] = now;
      m.nfin = 0;
    }
    rc = push_movers(L);
    if (rc) return rc;
  }
  L->nstep = 0;
  L->pending = false;
  L->mov_pending = false;
  L->macro_valid = false;
  return VPLBM_OK;
}

int vplbm_init_uniform(vplbm_lattice *L, double rho, double ux, double uy) {
  if (!L) return VPLBM_EINVAL;
  if (!(rho > 0.0) || !std::isfinite(rho) || !std::isfinite(ux) || !std::isfinite(uy))
    return L->fail(VPLBM_EINVAL, "rho must be > 0 and velocities finite");
  int rc = flush(L);  // a moving disk's state and mask as of the last step
  if (!rc) rc = launch_init(L, 0, L->p.ny, nullptr, nullptr, nullptr, rho, ux, uy);
  if (!rc) rc = reset_counters(L);
  return rc;
}

int vplbm_set_fields(vplbm_lattice *L, const double *rho, const double *ux, const double *uy) {
  if (!L || !rho || !ux || !uy) return L ? L->fail(VPLBM_EINVAL, "NULL field") : VPLBM_EINVAL;
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  const int nx = L->p.nx, ny = L->p.ny;
  for (long long k = 0; k < (long long)nx * ny; ++k)
    if (!(rho[k] > 0.0) || !std::isfinite(rho[k]) || !std::isfinite(ux[k]) || !std::isfinite(uy[k]))
      return L->fail(VPLBM_EINVAL, "field value at %lld is invalid", k);
  // staged in blocks of rows of a strip of columns (the whole width when it fits)
  const int wmax = (int)(STAGE_DOUBLES / 3);
  double *st = (double *)L->at(L->L.staging);
  for (int c0 = 0; c0 < nx; c0 += wmax) {
    const int wc = std::min(wmax, nx - c0);
    const int rows = std::max(1, (int)(STAGE_DOUBLES / (3 * (size_t)wc)));
    for (int y0 = 0; y0 < ny; y0 += rows) {
      const int nr = std::min(rows, ny - y0);
      const size_t n = (size_t)nr * wc;
      const double *src[3] = {rho, ux, uy};
      int rc = VPLBM_OK;
      for (int k = 0; k < 3 && !rc; ++k)
        rc = L->hip(hipMemcpy2DAsync(st + k * n, (size_t)wc * 8, src[k] + (size_t)y0 * nx + c0, (size_t)nx * 8,
                                     (size_t)wc * 8, (size_t)nr, hipMemcpyHostToDevice, L->stream),
                    "field upload");
      if (!rc) rc = launch_init(L, y0, nr, st, st + n, st + 2 * n, 0, 0, 0, c0, wc);
      if (!rc) rc = L->sync();
      if (rc) return rc;
    }
  }
  return reset_counters(L);
}

int vplbm_set_body_force(vplbm_lattice *L, double gx, double gy) {
  if (!L) return VPLBM_EINVAL;
  if (!std::isfinite(gx) || !std::isfinite(gy)) return L->fail(VPLBM_EINVAL, "force must be finite");
  L->gx = gx;
  L->gy = gy;
  return VPLBM_OK;
}

static int finish_geometry(vplbm_lattice *L, Ctl &c, int fx0, int fy0, int fx1, int fy1) {
  // interface flags over the region, then the window, then sample nodes
  int rc = launch_flags(L, fx0, fy0, fx1, fy1);
  if (!rc) rc = L->sync();
  if (rc) return rc;
  Ctl d;
  rc = L->ctl_pull(d);
  if (rc) return rc;
  d.win[0] = c.win[0]; d.win[1] = c.win[1]; d.win[2] = c.win[2]; d.win[3] = c.win[3];
  for (int k = 0; k < 4; ++k) d.region[k] = c.region[k];
  d.body = c.body;
  d.shape = c.shape;
  d.mode = c.mode;
  d.r = c.r;
  d.nrec = 0;
  d.si_moving = L->mode != MODE_STATIC;
  for (int k = 0; k < 3; ++k) d.fq[k] = c.fq[k];
  d.nbody = L->nbody;
  rc = L->ctl_push(d);
  if (!rc) rc = check_sample_error(L);  // a fluid cell linked to two bodies
  if (!rc) rc = number_interfaces(L);
  if (rc) return rc;
  if (L->npts) {
    rc = upload_points(L, d);
    if (!rc) rc = refresh_si(L);
    if (!rc) rc = check_sample_error(L);
  }
  return rc;
}

int vplbm_set_body_disk(vplbm_lattice *L, double xc, double yc, double r) {
  if (!L) return VPLBM_EINVAL;
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  L->pwin_ok = false;
  if (!std::isfinite(xc) || !std::isfinite(yc) || !(r > 0.0) || !std::isfinite(r))
    return L->fail(VPLBM_EINVAL, "disk needs finite centre and r > 0");
  const int nx = L->p.nx, ny = L->p.ny;
  if (xc - r < 1.0 || xc + r > nx - 2.0 || yc - r < 1.0 || yc + r > ny - 2.0)
    return L->fail(VPLBM_EINVAL, "disk must stay one cell inside the lattice");
  Ctl c;
  int rc = L->ctl_pull(c);
  if (rc) return rc;
  rc = reset_geometry(L, c);
  if (rc) return rc;
  const long long X = fixq(xc), Y = fixq(yc), R = fixq(r);
  const int bx0 = (int)((X - R) / FIXQ) - 1, bx1 = (int)((X + R) / FIXQ) + 2;
  const int by0 = (int)((Y - R) / FIXQ) - 1, by1 = (int)((Y + R) / FIXQ) + 2;
  const int x0 = std::max(bx0, 0), x1 = std::min(bx1, nx), y0 = std::max(by0, 0), y1 = std::min(by1, ny);
  if (x1 <= x0 || y1 <= y0) return L->fail(VPLBM_EINVAL, "empty disk region");
  dim3 blk(256), grd((x1 - x0 + 255) / 256, y1 - y0);
  VP_LAUNCH(k_mask_disk, grd, blk, 0, L->stream, L->mask(), L->pitch, x0, y0, x1, y1, X, Y, R);
  rc = L->launched("k_mask_disk");
  if (rc) return rc;
  c.body = BodyDev{xc, yc, 0.0, 0.0, 0.0, 0.0};
  c.shape = SHAPE_DISK;
  c.mode = MODE_STATIC;
  c.r = r;
  c.fq[0] = X; c.fq[1] = Y; c.fq[2] = R;
  c.win[0] = std::max(bx0 - 1, 0); c.win[1] = std::max(by0 - 1, 0);
  c.win[2] = std::min(bx1 + 1, nx); c.win[3] = std::min(by1 + 1, ny);
  c.region[0] = std::max(bx0 - REGION_MARGIN, 0); c.region[1] = std::max(by0 - REGION_MARGIN, 0);
  c.region[2] = std::min(bx1 + REGION_MARGIN, nx); c.region[3] = std::min(by1 + REGION_MARGIN, ny);
  L->shape = SHAPE_DISK;
  L->mode = MODE_STATIC;
  L->disk_r = r;
  return finish_geometry(L, c, c.win[0], c.win[1], c.win[2], c.win[3]);
}

int vplbm_set_body_polygon(vplbm_lattice *L, const double *xy, int nvert, double xref, double yref) {
  if (!L) return VPLBM_EINVAL;
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  L->pwin_ok = false;
  if (!xy || nvert < 3 || nvert > L->maxv)
    return L->fail(VPLBM_EINVAL, "polygon needs 3..%d vertices", L->maxv);
  if (!std::isfinite(xref) || !std::isfinite(yref)) return L->fail(VPLBM_EINVAL, "reference point");
  const int nx = L->p.nx, ny = L->p.ny;
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  std::vector<long long> v(2 * (size_t)L->maxv, 0);
  for (int k = 0; k < nvert; ++k) {
    const double x = xy[2 * k], y = xy[2 * k + 1];
    if (!std::isfinite(x) || !std::isfinite(y)) return L->fail(VPLBM_EINVAL, "vertex %d not finite", k);
    xmin = std::min(xmin, x); xmax = std::max(xmax, x);
    ymin = std::min(ymin, y); ymax = std::max(ymax, y);
    v[k] = fixq(x);
    v[L->maxv + k] = fixq(y);
  }
  if (xmin < 1.0 || xmax > nx - 2.0 || ymin < 1.0 || ymax > ny - 2.0)
    return L->fail(VPLBM_EINVAL, "polygon must stay one cell inside the lattice");
  Ctl c;
  int rc = L->ctl_pull(c);
  if (rc) return rc;
  rc = reset_geometry(L, c);
  if (rc) return rc;
  long long *dv = (long long *)L->at(L->L.verts);
  rc = L->hip(hipMemcpyAsync(dv, v.data(), v.size() * sizeof(long long), hipMemcpyHostToDevice, L->stream),
              "vertices");
  if (rc) return rc;
  const int x0 = std::max((int)std::floor(xmin) - 1, 0), x1 = std::min((int)std::ceil(xmax) + 2, nx);
  const int y0 = std::max((int)std::floor(ymin) - 1, 0), y1 = std::min((int)std::ceil(ymax) + 2, ny);
  if (x1 <= x0 || y1 <= y0) return L->fail(VPLBM_EINVAL, "empty polygon region");
  dim3 blk(256), grd((x1 - x0 + 255) / 256, y1 - y0);
  VP_LAUNCH(k_mask_polygon, grd, blk, 0, L->stream, L->mask(), L->pitch, x0, y0, x1, y1, dv,
                     dv + L->maxv, nvert);
  rc = L->launched("k_mask_polygon");
  if (!rc) rc = L->sync();
  if (rc) return rc;
  c.body = BodyDev{xref, yref, 0.0, 0.0, 0.0, 0.0};
  c.shape = SHAPE_POLYGON;
  c.mode = MODE_STATIC;
  c.r = 0.0;
  c.win[0] = std::max(x0 - 1, 0); c.win[1] = std::max(y0 - 1, 0);
  c.win[2] = std::min(x1 + 1, nx); c.win[3] = std::min(y1 + 1, ny);
  for (int k = 0; k < 4; ++k) c.region[k] = c.win[k];
  L->shape = SHAPE_POLYGON;
  L->mode = MODE_STATIC;
  return finish_geometry(L, c, c.win[0], c.win[1], c.win[2], c.win[3]);
}

int vplbm_set_mask(vplbm_lattice *L, const uint8_t *solid) {
  if (!L || !solid) return L ? L->fail(VPLBM_EINVAL, "NULL mask") : VPLBM_EINVAL;
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  L->pwin_ok = false;
  const int nx = L->p.nx, ny = L->p.ny;
  std::vector<uint8_t> rows((size_t)ny * L->pitch, 0);
  int x0 = nx, y0 = ny, x1 = -1, y1 = -1;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      if (solid[(size_t)j * nx + i]) {
        rows[(size_t)j * L->pitch + i] = 1;  // body 1
        x0 = std::min(x0, i); x1 = std::max(x1, i);
        y0 = std::min(y0, j); y1 = std::max(y1, j);
      }
  Ctl c;
  int rc = L->ctl_pull(c);
  if (rc) return rc;
  rc = reset_geometry(L, c);
  if (rc) return rc;
  rc = L->hip(hipMemcpyAsync(L->mask(), rows.data(), rows.size(), hipMemcpyHostToDevice, L->stream),
              "mask upload");
  if (!rc) rc = L->sync();
  if (rc) return rc;
  c.body = BodyDev{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  c.shape = SHAPE_MASK;
  c.mode = MODE_STATIC;
  if (x1 >= 0) {
    // interface cells lie within one cell of the solid's box; a box reaching
    // a periodic edge wraps, so the window then spans that axis
    int w0 = x0 - 1, w1 = x1 + 2, h0 = y0 - 1, h1 = y1 + 2;
    if (w0 < 0 || w1 > nx) { if (L->periodic_x()) { w0 = 0; w1 = nx; } else { w0 = std::max(w0, 0); w1 = std::min(w1, nx); } }
    if (h0 < 0 || h1 > ny) { if (L->periodic_y()) { h0 = 0; h1 = ny; } else { h0 = std::max(h0, 0); h1 = std::min(h1, ny); } }
    c.win[0] = w0; c.win[1] = h0; c.win[2] = w1; c.win[3] = h1;
  }
  for (int k = 0; k < 4; ++k) c.region[k] = c.win[k];
  L->shape = SHAPE_MASK;
  L->mode = MODE_STATIC;
  return finish_geometry(L, c, 0, 0, nx, ny);
}

int vplbm_set_body_motion(vplbm_lattice *L, const vplbm_body_state *s) {
  if (!L || !s) return L ? L->fail(VPLBM_EINVAL, "NULL state") : VPLBM_EINVAL;
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  L->pwin_ok = false;
  const double v[6] = {s->x, s->y, s->theta, s->u, s->v, s->omega};
  for (double e : v)
    if (!std::isfinite(e)) return L->fail(VPLBM_EINVAL, "state not finite");
  const bool moves = s->u != 0.0 || s->v != 0.0 || s->omega != 0.0;
  if (L->shape == SHAPE_NONE) return L->fail(VPLBM_ESTATE, "no body");
  if (L->shape != SHAPE_DISK && moves)
    return L->fail(VPLBM_EINVAL, "only disks can move; polygons and masks are static");
  if (moves) {
    const int h = mover_half(L, L->disk_r, s->x, s->y, 0, L->npts);
    const int rc = check_moving_capacity(L, 1, &h);
    if (rc) return rc;
  }
  Ctl c;
  int rc = L->ctl_pull(c);
  if (rc) return rc;
  if (L->shape == SHAPE_DISK) {
    const double r = L->disk_r;
    const int nx = L->p.nx, ny = L->p.ny;
    if (s->x - r < 1.0 || s->x + r > nx - 2.0 || s->y - r < 1.0 || s->y + r > ny - 2.0)
      return L->fail(VPLBM_EINVAL, "disk must stay one cell inside the lattice");
    // rebuild the mask at the new position (same as a fresh disk)
    const int npts = L->npts;
    L->npts = 0;
    rc = vplbm_set_body_disk(L, s->x, s->y, r);
    L->npts = npts;
    if (rc) return rc;
    rc = L->ctl_pull(c);
    if (rc) return rc;
  }
  c.body = BodyDev{s->x, s->y, s->theta, s->u, s->v, s->omega};
  c.mode = moves ? MODE_PRESCRIBED : MODE_STATIC;
  L->mode = c.mode;
  rc = L->ctl_push(c);
  if (rc) return rc;
  if (L->npts) {
    rc = upload_points(L, c);
    if (rc) return rc;
    c.si_moving = L->mode != MODE_STATIC;
    Ctl d;
    rc = L->ctl_pull(d);
    if (rc) return rc;
    d.si_moving = c.si_moving;
    rc = L->ctl_push(d);
    if (!rc) rc = launch_flags(L, d.region[0], d.region[1], d.region[2], d.region[3]);
    if (!rc) rc = refresh_si(L);
    if (!rc) rc = check_sample_error(L);
  }
  if (!rc && moves) {
    rc = L->ctl_pull(c);
    if (!rc) rc = become_mover(L, c);
  }
  return rc;
}

int vplbm_set_body_dynamics(vplbm_lattice *L, double rho_s, double gx, double gy, int source) {
  if (!L) return VPLBM_EINVAL;
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  L->pwin_ok = false;
  if (L->shape != SHAPE_DISK) return L->fail(VPLBM_ESTATE, "free bodies must be disks");
  {
    Ctl c0;
    int rc = L->ctl_pull(c0);
    if (rc) return rc;
    const int h = mover_half(L, L->disk_r, c0.body.x, c0.body.y, 0, L->npts);
    rc = check_moving_capacity(L, 1, &h);
    if (rc) return rc;
  }
  if (!(rho_s > 0.0) || !std::isfinite(rho_s) || !std::isfinite(gx) || !std::isfinite(gy))
    return L->fail(VPLBM_EINVAL, "rho_s > 0 and finite gravity required");
  if (source != VPLBM_FORCE_ME && source != VPLBM_FORCE_SI)
    return L->fail(VPLBM_EINVAL, "force_source must be ME (0) or SI (1)");
  Ctl c;
  int rc = L->ctl_pull(c);
  if (rc) return rc;
  const double r = L->disk_r;
  c.mass = rho_s * M_PI * r * r;
  c.inertia = 0.5 * c.mass * r * r;
  c.gx = gx;
  c.gy = gy;
  c.buoy = 1.0 - L->p.rho0 / rho_s;
  c.source = source;
  c.mode = MODE_FREE;
  c.si_moving = 1;
  L->mode = MODE_FREE;
  rc = L->ctl_push(c);
  if (!rc && L->npts) rc = upload_points(L, c);
  if (!rc) rc = become_mover(L, c);
  return rc;
}

int vplbm_set_moving_disks(vplbm_lattice *L, const vplbm_disk *d, int n, double gx, double gy, int source) {
  if (!L) return VPLBM_EINVAL;
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  L->pwin_ok = false;
  if (!d) return L->fail(VPLBM_EINVAL, "NULL disks");
  if (n < 1 || n > MAX_MOVERS) return L->fail(VPLBM_EINVAL, "n must be in 1..%d", MAX_MOVERS);
  if (n > L->maxb) return L->fail(VPLBM_EINVAL, "n = %d exceeds max_bodies = %d", n, L->maxb);
  if (source != VPLBM_FORCE_ME && source != VPLBM_FORCE_SI)
    return L->fail(VPLBM_EINVAL, "force_source must be ME (0) or SI (1)");
  if (!std::isfinite(gx) || !std::isfinite(gy)) return L->fail(VPLBM_EINVAL, "gravity must be finite");
  const int nx = L->p.nx, ny = L->p.ny;
  int half[MAX_MOVERS];
  for (int k = 0; k < n; ++k) {
    const vplbm_disk &e = d[k];
    const double v[8] = {e.x, e.y, e.r, e.theta, e.u, e.v, e.omega, e.rho_s};
    for (double q : v)
      if (!std::isfinite(q)) return L->fail(VPLBM_EINVAL, "disk %d: values must be finite", k);
    if (!(e.r > 0.0) || e.rho_s < 0.0) return L->fail(VPLBM_EINVAL, "disk %d: r > 0 and rho_s >= 0 required", k);
    if (e.x - e.r < 1.0 || e.x + e.r > nx - 2.0 || e.y - e.r < 1.0 || e.y + e.r > ny - 2.0)
      return L->fail(VPLBM_EINVAL, "disk %d must stay one cell inside the lattice", k);
    for (int q = 0; q < k; ++q)
      if (std::hypot(e.x - d[q].x, e.y - d[q].y) <= e.r + d[q].r + 2.0)
        return L->fail(VPLBM_EINVAL, "disks %d and %d are less than two cells apart", q, k);
    half[k] = (int)std::ceil(e.r) + WIN_MARGIN;
  }
  int rc = check_moving_capacity(L, n, half);
  if (rc) return rc;
  Ctl c;
  rc = L->ctl_pull(c);
  if (!rc) rc = reset_geometry(L, c);
  if (rc) return rc;
  for (int b = 1; b <= MAX_BODIES; ++b) L->si_sets[b].clear();
  L->nbody = n;
  rebuild_points(L);
  const double rho0 = L->p.rho0;
  std::vector<MoverDev> mv(MAX_MOVERS, MoverDev{});
  int part = 0;
  for (int k = 0; k < n; ++k) {
    const vplbm_disk &e = d[k];
    MoverDev &m = mv[k];
    m.B[0] = m.B[1] = BodyDev{e.x, e.y, e.theta, e.u, e.v, e.omega};
    m.r = e.r;
    m.R = fixq(e.r);
    m.mode = e.rho_s > 0.0 ? MODE_FREE : MODE_PRESCRIBED;
    m.mass = e.rho_s > 0.0 ? e.rho_s * M_PI * e.r * e.r : 0.0;
    m.inertia = 0.5 * m.mass * e.r * e.r;
    m.gx = gx;
    m.gy = gy;
    m.buoy = e.rho_s > 0.0 ? 1.0 - rho0 / e.rho_s : 0.0;
    m.source = source;
    m.nfin = c.step;
    m.half = half[k];
    m.pt0 = m.pt1 = 0;
    m.part0 = part;
    mover_grid(half[k], m.ptx, m.pty);
    part += m.ptx * m.pty;
  }
  // body 1 in the control block, as the single-body calls see it
  c.nbody = n;
  c.body = mv[0].B[0];
  c.shape = SHAPE_DISK;
  c.mode = mv[0].mode;
  c.r = d[0].r;
  c.mass = mv[0].mass;
  c.inertia = mv[0].inertia;
  c.gx = gx;
  c.gy = gy;
  c.buoy = mv[0].buoy;
  c.source = source;
  c.si_moving = 1;
  c.npts = 0;
  c.nrec = 0;
  c.err = 0;
  rc = L->ctl_push(c);
  if (rc) return rc;
  L->shape = SHAPE_DISK;
  L->mode = c.mode;
  L->disk_r = d[0].r;
  L->movers = mv;
  L->nmov = n;
  L->mov_pending = false;
  L->pending = false;
  L->bx = 64;  // the moving-disk step kernels run 64x4 tiles
  L->by = 4;
  rc = push_movers(L);
  if (!rc) rc = launch_mover_mask(L);
  if (!rc) rc = L->sync();
  if (!rc) rc = check_sample_error(L);
  return rc;
}

// Points of moving disk `body` (the caller has checked them and flushed):
// stored in the disk's frame at its current state; every disk's point
// range, window and partial grid follow, and the mask of the windows is
// rewritten.
int set_points_moving(vplbm_lattice *L, int body, const double *xy, const double *nrm, const double *ds, int npts) {
  if (body > L->nmov) return L->fail(VPLBM_EINVAL, "body %d is not a moving disk", body);
  int rc = pull_movers(L);
  if (rc) return rc;
  const int slot = (int)(L->nstep & 1);  // the current states
  int half[MAX_MOVERS];
  for (int k = 0; k < L->nmov; ++k) half[k] = L->movers[k].half;
  {
    const BodyDev &B = L->movers[body - 1].B[slot];
    double rmax = L->movers[body - 1].r;
    for (int i = 0; i < npts; ++i) rmax = std::max(rmax, std::hypot(xy[2 * i] - B.x, xy[2 * i + 1] - B.y));
    half[body - 1] = (int)std::ceil(rmax) + WIN_MARGIN;
  }
  rc = check_moving_capacity(L, L->nmov, half);
  if (rc) return rc;
  std::vector<double> &v = L->si_sets[body];
  v.assign((size_t)5 * npts, 0.0);
  for (int i = 0; i < npts; ++i) {
    v[i] = xy[2 * i];
    v[npts + i] = xy[2 * i + 1];
    v[2 * npts + i] = nrm[2 * i];
    v[3 * npts + i] = nrm[2 * i + 1];
    v[4 * npts + i] = ds[i];
  }
  rebuild_points(L);  // body by body: disk k's points follow disk k - 1's
  int o = 0, part = 0;
  BodyDev refs[MAX_MOVERS];
  for (int k = 0; k < L->nmov; ++k) {
    MoverDev &m = L->movers[k];
    const int nk = (int)(L->si_sets[k + 1].size() / 5);
    m.pt0 = o;
    m.pt1 = o + nk;
    o += nk;
    m.half = half[k];
    mover_grid(half[k], m.ptx, m.pty);
    m.part0 = part;
    part += m.ptx * m.pty;
    refs[k] = m.B[slot];
  }
  Ctl c;
  rc = L->ctl_pull(c);
  if (rc) return rc;
  c.npts = L->npts;
  c.si_moving = 1;
  c.nrec = 0;
  rc = L->ctl_push(c);
  if (!rc) rc = upload_points(L, c, refs);
  if (!rc) rc = push_movers(L);
  if (!rc) rc = launch_mover_mask(L);
  if (!rc) rc = L->sync();
  if (!rc) rc = check_sample_error(L);
  return rc;
}

int vplbm_set_si_points_body(vplbm_lattice *L, int body, const double *xy, const double *nrm, const double *ds,
                             int npts) {
  if (!L) return VPLBM_EINVAL;
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  L->pwin_ok = false;
  if (body < 1 || body > L->nbody) return L->fail(VPLBM_EINVAL, "body must be in 1..%d", L->nbody);
  if (npts < 0 || npts > L->maxp) return L->fail(VPLBM_EINVAL, "npts must be in 0..%d", L->maxp);
  if (npts > 0 && (!xy || !nrm || !ds)) return L->fail(VPLBM_EINVAL, "NULL point arrays");
  for (int i = 0; i < npts; ++i)
    if (!std::isfinite(xy[2 * i]) || !std::isfinite(xy[2 * i + 1]) || !std::isfinite(nrm[2 * i]) ||
        !std::isfinite(nrm[2 * i + 1]) || !std::isfinite(ds[i]))
      return L->fail(VPLBM_EINVAL, "point %d not finite", i);
  int total = npts;
  for (int b = 1; b <= L->nbody; ++b)
    if (b != body) total += (int)(L->si_sets[b].size() / 5);
  if (total > L->maxp) return L->fail(VPLBM_EINVAL, "%d points in all exceed max_si_points = %d", total, L->maxp);
  if (L->nmov) return set_points_moving(L, body, xy, nrm, ds, npts);
  std::vector<double> &v = L->si_sets[body];
  v.assign((size_t)5 * npts, 0.0);
  for (int i = 0; i < npts; ++i) {
    v[i] = xy[2 * i];
    v[npts + i] = xy[2 * i + 1];
    v[2 * npts + i] = nrm[2 * i];
    v[3 * npts + i] = nrm[2 * i + 1];
    v[4 * npts + i] = ds[i];
  }
  rebuild_points(L);
  Ctl c;
  int rc = L->ctl_pull(c);
  if (rc) return rc;
  c.npts = L->npts;
  c.si_moving = L->mode != MODE_STATIC;
  c.nrec = 0;
  rc = L->ctl_push(c);
  if (rc) return rc;
  // clear old sample bits: recompute flags over the window and region (for
  // a moving disk, the window its last flush wrote)
  const int x0 = std::min(c.win[0], c.region[0]), y0 = std::min(c.win[1], c.region[1]);
  const int x1 = std::max(c.win[2], c.region[2]), y1 = std::max(c.win[3], c.region[3]);
  rc = launch_flags(L, x0, y0, x1, y1);
  if (!rc) rc = L->sync();
  if (rc) return rc;
  if (L->npts == 0) {
    // no records: every body's record range empty
    std::vector<BodyTab> bt(MAX_BODIES);
    rc = L->hip(hipMemcpyAsync(bt.data(), L->bt(), bt.size() * sizeof(BodyTab), hipMemcpyDeviceToHost, L->stream),
                "body table read");
    if (!rc) rc = L->sync();
    if (rc) return rc;
    for (BodyTab &t : bt) t.rec0 = t.rec1 = 0;
    rc = L->hip(hipMemcpyAsync(L->bt(), bt.data(), bt.size() * sizeof(BodyTab), hipMemcpyHostToDevice, L->stream),
                "body table write");
    if (!rc) rc = L->sync();
    return rc;
  }
  rc = upload_points(L, c);
  if (!rc) rc = refresh_si(L);
  if (!rc) rc = check_sample_error(L);
  return rc;
}

int vplbm_set_si_points(vplbm_lattice *L, const double *xy, const double *nrm, const double *ds, int npts) {
  return vplbm_set_si_points_body(L, 1, xy, nrm, ds, npts);
}

int vplbm_set_body_ids(vplbm_lattice *L, const uint8_t *ids, int nbody, const double *ref_xy) {
  if (!L || !ids || !ref_xy) return L ? L->fail(VPLBM_EINVAL, "NULL argument") : VPLBM_EINVAL;
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  L->pwin_ok = false;
  if (nbody < 1 || nbody > L->maxb) return L->fail(VPLBM_EINVAL, "nbody must be in 1..max_bodies = %d", L->maxb);
  for (int k = 0; k < 2 * nbody; ++k)
    if (!std::isfinite(ref_xy[k])) return L->fail(VPLBM_EINVAL, "reference point %d not finite", k / 2);
  const int nx = L->p.nx, ny = L->p.ny;
  std::vector<uint8_t> rows((size_t)ny * L->pitch, 0);
  int x0 = nx, y0 = ny, x1 = -1, y1 = -1;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int id = ids[(size_t)j * nx + i];
      if (!id) continue;
      if (id > nbody) return L->fail(VPLBM_EINVAL, "cell (%d, %d) has body id %d > nbody = %d", i, j, id, nbody);
      rows[(size_t)j * L->pitch + i] = (uint8_t)id;
      x0 = std::min(x0, i); x1 = std::max(x1, i);
      y0 = std::min(y0, j); y1 = std::max(y1, j);
    }
  Ctl c;
  int rc = L->ctl_pull(c);
  if (rc) return rc;
  // the points of the previous geometry go with it
  for (auto &v : L->si_sets) v.clear();
  L->si_world.clear();
  L->si_body.clear();
  L->npts = 0;
  c.npts = 0;
  rc = reset_geometry(L, c);
  if (rc) return rc;
  std::vector<BodyDev> tab(MAX_BODIES + 1, BodyDev{0.0, 0.0, 0.0, 0.0, 0.0, 0.0});
  for (int b = 1; b <= nbody; ++b) tab[b] = BodyDev{ref_xy[2 * (b - 1)], ref_xy[2 * (b - 1) + 1], 0.0, 0.0, 0.0, 0.0};
  rc = L->hip(hipMemcpyAsync(L->mask(), rows.data(), rows.size(), hipMemcpyHostToDevice, L->stream), "mask upload");
  if (!rc)
    rc = L->hip(hipMemcpyAsync(L->bodies(), tab.data(), tab.size() * sizeof(BodyDev), hipMemcpyHostToDevice,
                               L->stream),
                "bodies upload");
  if (!rc) rc = L->sync();
  if (rc) return rc;
  c.body = tab[1];
  c.shape = SHAPE_MASK;
  c.mode = MODE_STATIC;
  if (x1 >= 0) {
    int w0 = x0 - 1, w1 = x1 + 2, h0 = y0 - 1, h1 = y1 + 2;
    if (w0 < 0 || w1 > nx) { if (L->periodic_x()) { w0 = 0; w1 = nx; } else { w0 = std::max(w0, 0); w1 = std::min(w1, nx); } }
    if (h0 < 0 || h1 > ny) { if (L->periodic_y()) { h0 = 0; h1 = ny; } else { h0 = std::max(h0, 0); h1 = std::min(h1, ny); } }
    c.win[0] = w0; c.win[1] = h0; c.win[2] = w1; c.win[3] = h1;
  }
  for (int k = 0; k < 4; ++k) c.region[k] = c.win[k];
  L->shape = SHAPE_MASK;
  L->mode = MODE_STATIC;
  L->nbody = nbody;
  L->refs.assign(ref_xy, ref_xy + 2 * nbody);
  return finish_geometry(L, c, 0, 0, nx, ny);
}

int vplbm_step(vplbm_lattice *L, int nsteps, int flags) {
  if (!L) return VPLBM_EINVAL;
  if (nsteps < 0) return L->fail(VPLBM_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return VPLBM_OK;
  for (int i = 0; i < nsteps; ++i) {
    const bool macro = (flags & VPLBM_STEP_MACRO) && i == nsteps - 1;
    L->macro_valid = false;
    int rc = one_step(L, macro);
    if (rc) return rc;
  }
  L->macro_valid = (flags & VPLBM_STEP_MACRO) != 0;
  return VPLBM_OK;
}

int vplbm_step_timed(vplbm_lattice *L, int nsteps, int flags, double *kernel_ms) {
  if (!L || !kernel_ms) return VPLBM_EINVAL;
  if (nsteps < 0) return L->fail(VPLBM_EINVAL, "nsteps must be >= 0");
  *kernel_ms = 0.0;
  if (nsteps == 0) return VPLBM_OK;
  std::vector<hipEvent_t> ev(2 * (size_t)nsteps, nullptr);
  int rc = VPLBM_OK;
  for (auto &e : ev)
    if (!rc) rc = L->hip(hipEventCreate(&e), "hipEventCreate");
  int done = 0;
  L->macro_valid = false;
  for (int i = 0; i < nsteps && !rc; ++i) {
    const bool macro = (flags & VPLBM_STEP_MACRO) && i == nsteps - 1;
    rc = L->hip(hipEventRecord(ev[2 * i], L->stream), "hipEventRecord");
    if (!rc) rc = launch_step(L, macro);
    if (!rc) rc = L->hip(hipEventRecord(ev[2 * i + 1], L->stream), "hipEventRecord");
    if (!rc) {
      if (L->nmov)
        L->mov_pending = true;
      else
        L->pending = true;
      L->cur ^= 1;
      L->nstep += 1;
      ++done;
    }
  }
  L->macro_valid = (flags & VPLBM_STEP_MACRO) != 0 && done == nsteps;
  if (!rc) rc = L->sync();
  double total = 0.0;
  for (int i = 0; i < done && !rc; ++i) {
    float ms = 0.f;
    rc = L->hip(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]), "hipEventElapsedTime");
    total += ms;
  }
  for (auto &e : ev)
    if (e) (void)hipEventDestroy(e);
  *kernel_ms = total;
  return rc;
}

int vplbm_sync(vplbm_lattice *L) {
  if (!L) return VPLBM_EINVAL;
  int rc = flush(L);
  if (!rc) rc = L->sync();
  if (rc) return rc;
  return check_sample_error(L);  // divergence flag; lost sample nodes of a moving body
}

long long vplbm_step_count(const vplbm_lattice *L) { return L ? L->nstep : -1; }

int vplbm_set_tile(vplbm_lattice *L, int bx, int by) {
  if (!L) return VPLBM_EINVAL;
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  const bool ok = (bx == 64 && (by == 1 || by == 2 || by == 4)) || (bx == 128 && (by == 1 || by == 2)) ||
                  (bx == 256 && by == 1);
  if (!ok) return L->fail(VPLBM_EINVAL, "unsupported tile %dx%d", bx, by);
  if (L->aa() && (bx != 64 || by != 4)) return L->fail(VPLBM_EINVAL, "the AA pattern runs with the 64x4 tile only");
  if (L->nmov && (bx != 64 || by != 4))
    return L->fail(VPLBM_EINVAL, "a lattice with moving disks runs the 64x4 tile only");
  L->bx = bx;
  L->by = by;
  return VPLBM_OK;
}

int vplbm_get_tile(const vplbm_lattice *L, int *bx, int *by) {
  if (!L || !bx || !by) return VPLBM_EINVAL;
  *bx = L->bx;
  *by = L->by;
  return VPLBM_OK;
}

static int read_last(vplbm_lattice *L, int which, double out[3]) {
  if (!L || !out) return VPLBM_EINVAL;
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  if (L->nstep == 0) return L->fail(VPLBM_ESTATE, "no step taken yet");
  Ctl c;
  int rc = L->ctl_pull(c);
  if (rc) return rc;
  for (int i = 0; i < 3; ++i) out[i] = c.last[3 * which + i];
  if (c.err & 16) return L->fail(VPLBM_EUNSTABLE, "the solution diverged (a non-finite density at some step)");
  if (c.err & 32)
    return L->fail(VPLBM_EUNSTABLE, "a moving disk moved a cell or more in one step (or left the lattice)");
  if (c.err & 8)
    return L->fail(VPLBM_ESTATE, "more interface cells than max_interface_cells = %lld: the momentum exchange "
                                 "dropped some",
                   L->maxslot);
  if (c.err & 1) return L->fail(VPLBM_ENOSAMPLE, "a stress-integration point lost its sample node");
  return VPLBM_OK;
}

int vplbm_forces_me(vplbm_lattice *L, double out[3]) { return read_last(L, 0, out); }
int vplbm_forces_si(vplbm_lattice *L, double out[3]) { return read_last(L, 1, out); }

int vplbm_forces_si_at(vplbm_lattice *L, const double *xy, const double *nrm, const double *ds, int npts,
                       double out[3]) {
  if (!L || !out) return VPLBM_EINVAL;
  if (npts < 0 || npts > L->maxp || (npts > 0 && (!xy || !nrm || !ds)))
    return L->fail(VPLBM_EINVAL, "bad points");
  {
    const int frc = flush_movers(L);  // moving disks' mask and state after the last step
    if (frc) return frc;
  }
  const int mp = L->maxp;
  std::vector<double> buf((size_t)5 * mp, 0.0);
  for (int i = 0; i < npts; ++i) {
    buf[i] = xy[2 * i];
    buf[mp + i] = xy[2 * i + 1];
    buf[2 * mp + i] = nrm[2 * i];
    buf[3 * mp + i] = nrm[2 * i + 1];
    buf[4 * mp + i] = ds[i];
  }
  if ((size_t)5 * mp > STAGE_DOUBLES) return L->fail(VPLBM_EINVAL, "too many points");
  double *st = (double *)L->at(L->L.staging);
  double *o = (double *)L->at(L->L.siout);
  int rc = L->hip(hipMemcpyAsync(st, buf.data(), buf.size() * 8, hipMemcpyHostToDevice, L->stream), "pts");
  if (rc) return rc;
  switch (L->p.precision) {
    case VPLBM_F64: rc = launch_si_at_s<double>(L, npts, o); break;
    case VPLBM_F32: rc = launch_si_at_s<float>(L, npts, o); break;
    default: rc = launch_si_at_s<__half>(L, npts, o); break;
  }
  if (rc) return rc;
  double h[4];
  rc = L->hip(hipMemcpyAsync(h, o, sizeof h, hipMemcpyDeviceToHost, L->stream), "si_at read");
  if (!rc) rc = L->sync();
  if (rc) return rc;
  out[0] = h[0]; out[1] = h[1]; out[2] = h[2];
  if (h[3] != 0.0) return L->fail(VPLBM_ENOSAMPLE, "%d points without a sample node", (int)h[3]);
  return VPLBM_OK;
}

int vplbm_force_history_body(vplbm_lattice *L, int body, int which, long long first, int n, double *out) {
  if (!L || !out || n < 0) return VPLBM_EINVAL;
  if (body < 1 || body > L->nbody) return L->fail(VPLBM_EINVAL, "body must be in 1..%d", L->nbody);
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  if (which != VPLBM_FORCE_ME && which != VPLBM_FORCE_SI) return L->fail(VPLBM_EINVAL, "which");
  if (first < 1 || first + n - 1 > L->nstep || first <= L->nstep - L->cap)
    return L->fail(VPLBM_EINVAL, "steps %lld..%lld outside the kept history", first, first + n - 1);
  std::vector<double> h((size_t)L->cap * L->maxb * 6);
  int rc = L->hip(hipMemcpyAsync(h.data(), L->at(L->L.hist), h.size() * 8, hipMemcpyDeviceToHost, L->stream),
                  "history read");
  if (!rc) rc = L->sync();
  if (rc) return rc;
  for (int k = 0; k < n; ++k) {
    const long long s = (first + k) % L->cap;
    for (int i = 0; i < 3; ++i) out[3 * k + i] = h[(s * L->maxb + (body - 1)) * 6 + 3 * which + i];
  }
  return VPLBM_OK;
}

int vplbm_force_history(vplbm_lattice *L, int which, long long first, int n, double *out) {
  return vplbm_force_history_body(L, 1, which, first, n, out);
}

int vplbm_forces_body(vplbm_lattice *L, int body, int which, double out[3]) {
  if (!L || !out) return VPLBM_EINVAL;
  if (body < 1 || body > L->nbody) return L->fail(VPLBM_EINVAL, "body must be in 1..%d", L->nbody);
  if (which != VPLBM_FORCE_ME && which != VPLBM_FORCE_SI) return L->fail(VPLBM_EINVAL, "which");
  if (body == 1) return read_last(L, which, out);
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  if (L->nstep == 0) return L->fail(VPLBM_ESTATE, "no step taken yet");
  return vplbm_force_history_body(L, body, which, L->nstep, 1, out);
}

int vplbm_get_body_state(vplbm_lattice *L, vplbm_body_state *out) {
  if (!L || !out) return VPLBM_EINVAL;
  {
    const int frc = flush_movers(L);  // a moving disk's state after the last step
    if (frc) return frc;
  }
  Ctl c;
  int rc = L->ctl_pull(c);
  if (rc) return rc;
  *out = vplbm_body_state{c.body.x, c.body.y, c.body.theta, c.body.u, c.body.v, c.body.omega};
  return VPLBM_OK;
}

int vplbm_get_body_state_of(vplbm_lattice *L, int body, vplbm_body_state *out) {
  if (!L || !out) return VPLBM_EINVAL;
  if (body < 1 || body > L->nbody) return L->fail(VPLBM_EINVAL, "body must be in 1..%d", L->nbody);
  if (body == 1) return vplbm_get_body_state(L, out);
  {
    const int frc = flush_movers(L);  // the disks' states after the last step
    if (frc) return frc;
  }
  BodyDev B;
  if (body <= L->nmov) {
    const int rc = pull_movers(L);
    if (rc) return rc;
    B = L->movers[body - 1].B[L->nstep & 1];
  } else {
    const int rc = L->hip(hipMemcpyAsync(&B, L->bodies() + body, sizeof(BodyDev), hipMemcpyDeviceToHost, L->stream),
                          "body read");
    if (rc) return rc;
    const int src = L->sync();
    if (src) return src;
  }
  *out = vplbm_body_state{B.x, B.y, B.theta, B.u, B.v, B.omega};
  return VPLBM_OK;
}

static bool bad_window(const vplbm_lattice *L, int x0, int y0, int w, int h) {
  return x0 < 0 || y0 < 0 || w < 1 || h < 1 || x0 > L->p.nx - w || y0 > L->p.ny - h;
}

int vplbm_read_macro_window(vplbm_lattice *L, int x0, int y0, int w, int h, double *rho, double *ux,
                            double *uy) {
  if (!L || !rho || !ux || !uy) return VPLBM_EINVAL;
  if (bad_window(L, x0, y0, w, h)) return L->fail(VPLBM_EINVAL, "window outside the lattice");
  if (!L->macro_valid) return L->fail(VPLBM_ESTATE, "last step did not store rho and u (VPLBM_STEP_MACRO)");
  const int wmax = (int)(STAGE_DOUBLES / 3);
  if (w > wmax) {  // wider than one staged row: strips of columns
    std::vector<double> part;
    for (int c0 = 0; c0 < w; c0 += wmax) {
      const int wc = std::min(wmax, w - c0);
      part.resize((size_t)3 * wc * h);
      double *pr = part.data(), *pu = pr + (size_t)wc * h, *pv = pu + (size_t)wc * h;
      const int rc = vplbm_read_macro_window(L, x0 + c0, y0, wc, h, pr, pu, pv);
      if (rc) return rc;
      for (int r = 0; r < h; ++r) {
        std::memcpy(rho + (size_t)r * w + c0, pr + (size_t)r * wc, (size_t)wc * 8);
        std::memcpy(ux + (size_t)r * w + c0, pu + (size_t)r * wc, (size_t)wc * 8);
        std::memcpy(uy + (size_t)r * w + c0, pv + (size_t)r * wc, (size_t)wc * 8);
      }
    }
    return VPLBM_OK;
  }
  const int rows = std::max(1, (int)(STAGE_DOUBLES / (3 * (size_t)w)));
  double *st = (double *)L->at(L->L.staging);
  std::vector<double> hb;
  for (int r0 = 0; r0 < h; r0 += rows) {
    const int nr = std::min(rows, h - r0);
    const size_t n = (size_t)nr * w;
    dim3 blk(256), grd((w + 255) / 256, nr);
    if (L->p.precision == VPLBM_F64)
      VP_LAUNCH((k_read_macro<double>), grd, blk, 0, L->stream, (const double *)L->at(L->L.mrho),
                         (const double *)L->at(L->L.mux), (const double *)L->at(L->L.muy), x0, w, L->pitch,
                         y0 + r0, nr, st);
    else
      VP_LAUNCH((k_read_macro<float>), grd, blk, 0, L->stream, (const float *)L->at(L->L.mrho),
                         (const float *)L->at(L->L.mux), (const float *)L->at(L->L.muy), x0, w, L->pitch,
                         y0 + r0, nr, st);
    int rc = L->launched("k_read_macro");
    hb.resize(3 * n);
    if (!rc) rc = L->hip(hipMemcpyAsync(hb.data(), st, 3 * n * 8, hipMemcpyDeviceToHost, L->stream), "macro");
    if (!rc) rc = L->sync();
    if (rc) return rc;
    std::memcpy(rho + (size_t)r0 * w, hb.data(), n * 8);
    std::memcpy(ux + (size_t)r0 * w, hb.data() + n, n * 8);
    std::memcpy(uy + (size_t)r0 * w, hb.data() + 2 * n, n * 8);
  }
  return VPLBM_OK;
}

int vplbm_read_macro_device(vplbm_lattice *L, void *rho, void *ux, void *uy) {
  if (!L || !rho || !ux || !uy) return L ? L->fail(VPLBM_EINVAL, "NULL output") : VPLBM_EINVAL;
  if (!L->macro_valid) return L->fail(VPLBM_ESTATE, "last step did not store rho and u (VPLBM_STEP_MACRO)");
  const size_t es = compute_size(L->p.precision);
  const size_t off[3] = {L->L.mrho, L->L.mux, L->L.muy};
  void *dst[3] = {rho, ux, uy};
  for (int k = 0; k < 3; ++k) {
    const int rc = L->hip(hipMemcpy2DAsync(dst[k], (size_t)L->p.nx * es, L->at(off[k]), (size_t)L->pitch * es,
                                           (size_t)L->p.nx * es, (size_t)L->p.ny, hipMemcpyDeviceToDevice,
                                           L->stream),
                          "macro device copy");
    if (rc) return rc;
  }
  return VPLBM_OK;
}

int vplbm_read_macro(vplbm_lattice *L, double *rho, double *ux, double *uy) {
  if (!L) return VPLBM_EINVAL;
  return vplbm_read_macro_window(L, 0, 0, L->p.nx, L->p.ny, rho, ux, uy);
}

int vplbm_read_populations_window(vplbm_lattice *L, int x0, int y0, int w, int h, double *f) {
  if (!L || !f) return VPLBM_EINVAL;
  if (bad_window(L, x0, y0, w, h)) return L->fail(VPLBM_EINVAL, "window outside the lattice");
  {
    const int frc = flush(L);
    if (frc) return frc;
  }
  const int wmax = (int)(STAGE_DOUBLES / Q);
  if (w > wmax) {  // wider than one staged row: strips of columns
    std::vector<double> part;
    for (int c0 = 0; c0 < w; c0 += wmax) {
      const int wc = std::min(wmax, w - c0);
      part.resize((size_t)Q * wc * h);
      const int rc = vplbm_read_populations_window(L, x0 + c0, y0, wc, h, part.data());
      if (rc) return rc;
      for (int a = 0; a < Q; ++a)
        for (int r = 0; r < h; ++r)
          std::memcpy(f + ((size_t)a * h + r) * w + c0, part.data() + ((size_t)a * h + r) * wc, (size_t)wc * 8);
    }
    return VPLBM_OK;
  }
  const int rows = std::max(1, (int)(STAGE_DOUBLES / (9 * (size_t)w)));
  double *st = (double *)L->at(L->L.staging);
  std::vector<double> hb;
  for (int r0 = 0; r0 < h; r0 += rows) {
    const int nr = std::min(rows, h - r0);
    const size_t n = (size_t)nr * w;
    int rc = launch_read_pop(L, x0, w, y0 + r0, nr, st);
    hb.resize(9 * n);
    if (!rc) rc = L->hip(hipMemcpyAsync(hb.data(), st, 9 * n * 8, hipMemcpyDeviceToHost, L->stream), "pop");
    if (!rc) rc = L->sync();
    if (rc) return rc;
    for (int a = 0; a < Q; ++a)
      std::memcpy(f + (size_t)a * w * h + (size_t)r0 * w, hb.data() + a * n, n * 8);
  }
  return VPLBM_OK;
}

int vplbm_read_populations(vplbm_lattice *L, double *f) {
  if (!L) return VPLBM_EINVAL;
  return vplbm_read_populations_window(L, 0, 0, L->p.nx, L->p.ny, f);
}

int vplbm_read_mask(vplbm_lattice *L, uint8_t *out) {
  if (!L || !out) return VPLBM_EINVAL;
  {
    const int frc = flush_movers(L);  // moving disks' mask bytes after the last step
    if (frc) return frc;
  }
  int rc = L->hip(hipMemcpy2DAsync(out, L->p.nx, L->mask(), L->pitch, L->p.nx, L->p.ny,
                                   hipMemcpyDeviceToHost, L->stream),
                  "mask read");
  if (!rc) rc = L->sync();
  return rc;
}

// ----------------------------------------------------------------------------
// batches: several lattices stepped by one launch per step
// ----------------------------------------------------------------------------
}  // extern "C"

// What a captured graph of batched launch pairs bakes in besides the device
// tables' contents: the launch shape and arguments.
struct GraphKey {
  int nact = -1, bx = 0, mov = 0;
  int aapar = -1;  // AA batches: the parity of the flip-0 launches' steps when every lattice shares it
  long long total = 0;
  bool operator==(const GraphKey &o) const {
    return nact == o.nact && bx == o.bx && mov == o.mov && aapar == o.aapar && total == o.total;
  }
  bool operator!=(const GraphKey &o) const { return !(*this == o); }
};

struct vplbm_batch {
  std::vector<vplbm_lattice *> cases;
  hipStream_t stream = nullptr;      // the lattices' stream
  hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
  int prec = 0;
  bool trt = false;  // collision of every lattice of the batch
  bool aa = false;   // storage scheme of every lattice of the batch
  int bx = 64, by = 4;  // tile of the batched launches
  char *desc_dev = nullptr;
  int ncap = 0;                  // descriptors the device table holds
  BlockCase *tile_case_dev = nullptr;  // lattice table: one entry per block of TILE_BLOCK global tiles
  long long tile_case_cap = 0;
  std::vector<char> desc_host;
  hipGraphExec_t graph = nullptr;  // groups of launch pairs (parities 1, 0) of the current active set
  GraphKey graph_key;
  std::string err;
  int fail(int code, const std::string &m) {
    err = m;
    return code;
  }
  int hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return VPLBM_OK;
    return fail(VPLBM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  }
};

namespace {

template <typename S> constexpr size_t desc_size() { return sizeof(CaseDesc<typename Store<S>::T>); }

size_t desc_size_of(int prec) {
  return prec == VPLBM_F64 ? desc_size<double>() : (prec == VPLBM_F32 ? desc_size<float>() : desc_size<__half>());
}

// tiles k_step_batch is instantiated for (AA batches: 64x4 only)
bool batch_tile_ok(int bx, int by) { return (bx == 64 && by == 4) || (bx == 128 && by == 2) || (bx == 256 && by == 1); }

// What one run of batched launches needs: the lattices' common settings,
// the device tables with their capacity, host staging for the descriptors,
// and, when allowed, graph replay.
struct BatchExec {
  int prec = 0;
  bool trt = false, aa = false;
  bool mov = false;  // some active lattice has moving disks (the chunk's kernels handle them; 64x4 tiles)
  int aapar0 = -1;   // AA: parity of the step every lattice computes in flip-0 launches (-1: mixed)
  int bx = 64, by = 4;
  hipStream_t stream = nullptr;
  char *desc_dev = nullptr;   // descriptors, one per active lattice
  BlockCase *tile_dev = nullptr;  // lattice table (one entry per TILE_BLOCK global tiles)
  long long tile_cap = 0;     // global tiles it has room for
  char *desc_host = nullptr;  // host staging, room for every lattice
  hipStream_t cap_stream = nullptr;  // graph capture (null: direct launches only)
  hipGraphExec_t *graph = nullptr;
  GraphKey *graph_key = nullptr;
};

template <typename S>
void fill_desc(vplbm_lattice *L, int tile0, int bx, int by, void *out) {
  using T = typename Store<S>::T;
  CaseDesc<T> d{};
  d.P = L->step_args<T>(bx, by);
  d.buf[0] = L->at(L->L.A);
  d.buf[1] = L->at(L->L.B);
  d.mask = L->mask();
  d.ctl = L->ctl();
  d.recs = (const SiRec *)L->at(L->L.recs);
  d.si_map = (const int *)L->at(L->L.si_map);
  d.imap = L->imap();
  d.bt = L->bt();
  d.me[0] = L->me(0);
  d.me[1] = L->me(1);
  d.sig[0] = L->sig(0);
  d.sig[1] = L->sig(1);
  d.hist = (double *)L->at(L->L.hist);
  d.cap = L->cap;
  d.maxb = L->maxb;
  d.tile0 = tile0;
  d.ntiles = d.P.ntiles;
  d.cur0 = L->cur;
  d.pbit0 = (int)((L->nstep + 1) & 1);
  d.pending0 = L->pending ? 1 : 0;
  d.mov_pending0 = L->mov_pending ? 1 : 0;
  d.ec[0] = L->aa() ? L->ec(0) : nullptr;
  d.ec[1] = L->aa() ? L->ec(1) : nullptr;
  std::memcpy(out, &d, sizeof d);
}

int batch_tiles(vplbm_lattice *L, int bx, int by) { return L->step_args<float>(bx, by).ntiles; }

// lattices that can share one batched launch: one precision, collision,
// stream and storage scheme, each once
const char *batch_check(vplbm_lattice *const *lats, int n) {
  if (!lats || n < 1) return "no lattices";
  for (int k = 0; k < n; ++k) {
    if (!lats[k]) return "NULL lattice";
    if (lats[k]->p.precision != lats[0]->p.precision) return "lattices of different precisions";
    if (lats[k]->stream != lats[0]->stream) return "lattices on different streams";
    if ((lats[k]->p.trt_lambda > 0.0) != (lats[0]->p.trt_lambda > 0.0)) return "BGK and TRT lattices mixed";
    if (lats[k]->aa() != lats[0]->aa()) return "a batch takes lattices of one storage scheme (all AB or all AA)";
    for (int j = 0; j < k; ++j)
      if (lats[j] == lats[k]) return "a lattice appears twice";
  }
  return nullptr;
}

template <typename S, int BX, int BY, bool MOV, bool ROT = false>
void launch_batch_ab(const BatchExec &X, hipStream_t st, dim3 grid, int total, int per, int flip, int first) {
  const auto *descs = (const CaseDesc<typename Store<S>::T> *)X.desc_dev;
  if (X.trt)
    hipLaunchKernelGGL((k_step_batch<S, BX, BY, true, MOV, ROT>), grid, dim3(BX * BY), 0, st, descs, X.tile_dev,
                       total, per, flip, first);
  else
    hipLaunchKernelGGL((k_step_batch<S, BX, BY, false, MOV, ROT>), grid, dim3(BX * BY), 0, st, descs, X.tile_dev,
                       total, per, flip, first);
}

template <typename S, bool TRT, bool MOV, bool ROT>
void launch_aa_par(int par, const BatchExec &X, hipStream_t st, dim3 grid, int total, int per, int flip,
                   int first) {
  const auto *descs = (const CaseDesc<typename Store<S>::T> *)X.desc_dev;
  if (par == 1)
    hipLaunchKernelGGL((k_step_batch_aa<S, TRT, MOV, ROT, 1>), grid, dim3(256), 0, st, descs, X.tile_dev, total, per,
                       flip, first);
  else if (par == 2)
    hipLaunchKernelGGL((k_step_batch_aa<S, TRT, MOV, ROT, 2>), grid, dim3(256), 0, st, descs, X.tile_dev, total, per,
                       flip, first);
  else
    hipLaunchKernelGGL((k_step_batch_aa<S, TRT, MOV, ROT, 0>), grid, dim3(256), 0, st, descs, X.tile_dev, total, per,
                       flip, first);
}

// AA batches: the kernel holding only the odd (1) or the even (2) tile code
// when every lattice of the launch computes a step of that parity, else the
// one that chooses per lattice (0)
template <typename S, bool MOV, bool ROT = false>
void launch_batch_aa(const BatchExec &X, hipStream_t st, dim3 grid, int total, int per, int flip, int first) {
  const int par = X.aapar0 < 0 ? 0 : ((X.aapar0 ^ flip) ? 1 : 2);
  if (X.trt)
    launch_aa_par<S, true, MOV, ROT>(par, X, st, grid, total, per, flip, first);
  else
    launch_aa_par<S, false, MOV, ROT>(par, X, st, grid, total, per, flip, first);
}

// Batched launches with moving disks of at most this many (64x4) tiles
// start their XCD bands at the disks' hit boxes (k_step_batch's ROT).  About
// 2 M cells: the plain tiles then take a few times the hit-box workgroups'
// serial work (10-12 us), so that where that work starts decides when the
// launch ends; the sedimenting disk (400 x 2000) batched alone 20.6 -> 17.0
// us per step.  Longer launches keep the form without rotation, whose plain
// tiles run 3-7% faster (a mix of 12 airfoil and sedimentation lattices,
// 8.5 M cells).
constexpr int ROT_MAX_TILES = 8192;

// the tile a chunk's launches run: the batch's, or 64x4 when a lattice has
// moving disks or the lattices are in the AA pattern
int chunk_bx(const BatchExec &X) { return (X.mov || X.aa) ? 64 : X.bx; }
int chunk_by(const BatchExec &X) { return (X.mov || X.aa) ? 4 : X.by; }

template <typename S>
void launch_batch_s(const BatchExec &X, hipStream_t st, int total, int flip, int first) {
  const int per = (total + 7) / 8;
  const dim3 grid(8 * per);
  const bool rot = total <= ROT_MAX_TILES;
  if (X.aa) {  // 64x4 tiles
    if (X.mov && rot)
      launch_batch_aa<S, true, true>(X, st, grid, total, per, flip, first);
    else if (X.mov)
      launch_batch_aa<S, true>(X, st, grid, total, per, flip, first);
    else
      launch_batch_aa<S, false>(X, st, grid, total, per, flip, first);
  } else if (X.mov && rot) {
    launch_batch_ab<S, 64, 4, true, true>(X, st, grid, total, per, flip, first);
  } else if (X.mov) {
    launch_batch_ab<S, 64, 4, true>(X, st, grid, total, per, flip, first);
  } else if (X.bx == 128 && X.by == 2) {
    launch_batch_ab<S, 128, 2, false>(X, st, grid, total, per, flip, first);
  } else if (X.bx == 256) {
    launch_batch_ab<S, 256, 1, false>(X, st, grid, total, per, flip, first);
  } else {
    launch_batch_ab<S, 64, 4, false>(X, st, grid, total, per, flip, first);
  }
}

void launch_batch(const BatchExec &X, hipStream_t st, int total, int flip, int first) {
  switch (X.prec) {
    case VPLBM_F64: launch_batch_s<double>(X, st, total, flip, first); break;
    case VPLBM_F32: launch_batch_s<float>(X, st, total, flip, first); break;
    default: launch_batch_s<__half>(X, st, total, flip, first); break;
  }
}

// entries of the lattice table for `tiles` global tiles
long long table_entries(long long tiles) { return (tiles + TILE_BLOCK - 1) / TILE_BLOCK; }

// the lattice table from the descriptors just uploaded, on the device
void launch_fill_tiles(const BatchExec &X, int nact, int total) {
  const int nblocks = (int)table_entries(total);
  const dim3 grid((nblocks + 255) / 256), block(256);
  switch (X.prec) {
    case VPLBM_F64:
      hipLaunchKernelGGL((k_fill_tile_case<double>), grid, block, 0, X.stream, (const CaseDesc<double> *)X.desc_dev,
                         nact, nblocks, X.tile_dev);
      break;
    case VPLBM_F32:
      hipLaunchKernelGGL((k_fill_tile_case<float>), grid, block, 0, X.stream, (const CaseDesc<float> *)X.desc_dev,
                         nact, nblocks, X.tile_dev);
      break;
    default:
      hipLaunchKernelGGL((k_fill_tile_case<float>), grid, block, 0, X.stream, (const CaseDesc<float> *)X.desc_dev,
                         nact, nblocks, X.tile_dev);
      break;
  }
}

// step pairs per captured graph: one launch call per group keeps the host
// ahead of short kernels
constexpr int GRAPH_PAIRS = 16;

// Advance lattice k by nsteps[k] steps with batched launches (see
// vplbm_batch_step).  Chunks run while some lattice has steps left; a chunk
// advances every active lattice by the smallest remaining count.
int batch_run(BatchExec &X, vplbm_lattice *const *lats, int n, const int *nsteps, std::string &err) {
  auto fail = [&](int code, const std::string &m) {
    err = m;
    return code;
  };
  auto hipck = [&](hipError_t e, const char *what) {
    return e == hipSuccess ? VPLBM_OK : fail(VPLBM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  std::vector<long long> rem(n);
  for (int k = 0; k < n; ++k) {
    if (nsteps[k] < 0) return fail(VPLBM_EINVAL, "negative step count");
    rem[k] = nsteps[k];
  }
  const size_t dsz = desc_size_of(X.prec);
  std::vector<int> act;
  act.reserve(n);
  for (;;) {
    act.clear();
    long long chunk = 0;
    for (int k = 0; k < n; ++k)
      if (rem[k] > 0) {
        act.push_back(k);
        chunk = chunk == 0 ? rem[k] : std::min(chunk, rem[k]);
      }
    if (act.empty()) break;
    // the host staging is rewritten below: the last chunk's copies must be done
    int rc = hipck(hipStreamSynchronize(X.stream), "hipStreamSynchronize");
    if (rc) return rc;
    long long total = 0;
    X.mov = false;
    for (int k : act) X.mov = X.mov || lats[k]->nmov > 0;
    const int bx = chunk_bx(X), by = chunk_by(X);
    for (size_t i = 0; i < act.size(); ++i) {
      vplbm_lattice *L = lats[act[i]];
      rc = resolve_pwin(L);
      if (rc) return fail(rc, "lattice " + std::to_string(act[i]) + ": " + L->err);
      void *slot = X.desc_host + i * dsz;
      switch (X.prec) {
        case VPLBM_F64: fill_desc<double>(L, (int)total, bx, by, slot); break;
        case VPLBM_F32: fill_desc<float>(L, (int)total, bx, by, slot); break;
        default: fill_desc<__half>(L, (int)total, bx, by, slot); break;
      }
      total += batch_tiles(L, bx, by);
    }
    X.aapar0 = -1;
    if (X.aa) {
      const int p0 = (int)((lats[act[0]]->nstep + 1) & 1);
      bool same = true;
      for (int k : act) same = same && (int)((lats[k]->nstep + 1) & 1) == p0;
      X.aapar0 = same ? p0 : -1;
    }
    if (total > X.tile_cap)
      return fail(VPLBM_EINVAL, "the batch's " + std::to_string(total) + " tiles exceed the tile table (" +
                                    std::to_string(X.tile_cap) + ")");
    const int nact = (int)act.size();
    rc = hipck(hipMemcpyAsync(X.desc_dev, X.desc_host, dsz * nact, hipMemcpyHostToDevice, X.stream),
               "batch descriptors");
    if (rc) return rc;
    (void)hipGetLastError();
    launch_fill_tiles(X, nact, (int)total);
    rc = hipck(hipGetLastError(), "k_fill_tile_case");
    if (rc) return rc;
    // launch 0 eagerly (it finalizes what the lattices left pending), then
    // pairs of launches (parities 1, 0), from a captured graph when allowed,
    // then a last one
    launch_batch(X, X.stream, (int)total, 0, 1);
    rc = hipck(hipGetLastError(), "k_step_batch");
    if (rc) return rc;
    long long done = 1;
    const long long pairs = (chunk - 1) / 2;
    // whole groups of GRAPH_PAIRS pairs replay from the graph (one launch
    // call per group); the remaining pairs are launched directly
    const long long groups = X.graph ? pairs / GRAPH_PAIRS : 0;
    if (groups > 0) {
      GraphKey key;
      key.nact = nact;
      key.bx = bx;
      key.mov = X.mov ? 1 : 0;
      key.aapar = X.aapar0;
      key.total = total;
      if (!*X.graph || *X.graph_key != key) {
        if (*X.graph) (void)hipGraphExecDestroy(*X.graph);
        *X.graph = nullptr;
        hipGraph_t g = nullptr;
        rc = hipck(hipStreamBeginCapture(X.cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        if (rc) return rc;
        for (int q = 0; q < GRAPH_PAIRS; ++q) {
          launch_batch(X, X.cap_stream, (int)total, 1, 0);
          launch_batch(X, X.cap_stream, (int)total, 0, 0);
        }
        rc = hipck(hipStreamEndCapture(X.cap_stream, &g), "end capture");
        if (!rc) rc = hipck(hipGraphInstantiate(X.graph, g, nullptr, nullptr, 0), "graph instantiate");
        if (g) (void)hipGraphDestroy(g);
        if (rc) return rc;
        *X.graph_key = key;
      }
      for (long long p = 0; p < groups && !rc; ++p) rc = hipck(hipGraphLaunch(*X.graph, X.stream), "graph launch");
      if (rc) return rc;
      done += 2 * GRAPH_PAIRS * groups;
    }
    for (long long p = groups * GRAPH_PAIRS; p < pairs; ++p) {
      launch_batch(X, X.stream, (int)total, 1, 0);
      launch_batch(X, X.stream, (int)total, 0, 0);
      rc = hipck(hipGetLastError(), "k_step_batch");
      if (rc) return rc;
      done += 2;
    }
    if (done < chunk) {
      launch_batch(X, X.stream, (int)total, 1, 0);
      rc = hipck(hipGetLastError(), "k_step_batch");
      if (rc) return rc;
      ++done;
    }
    for (int k : act) {
      vplbm_lattice *L = lats[k];
      L->nstep += chunk;
      L->cur ^= (int)(chunk & 1);
      L->pending = L->nmov == 0;  // the static bodies' forces, or the moving disks'
      L->mov_pending = L->nmov > 0;
      L->macro_valid = false;
      rem[k] -= chunk;
    }
  }
  return VPLBM_OK;
}

// ---- scratch of the allocation-free batched step --------------------------
// Descriptors, moving list and tile table of vplbm_batch_step_noalloc live in
// one file-scope device array; every GPU the library runs on holds its own
// copy until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
constexpr int NOALLOC_MAX_CASES = 256;
constexpr long long NOALLOC_MAX_TILES = 1 << 20;
constexpr size_t NOALLOC_DESC_BYTES = (size_t)NOALLOC_MAX_CASES * desc_size<double>();
constexpr size_t NOALLOC_TILE_OFF = (NOALLOC_DESC_BYTES + 255) / 256 * 256;
constexpr size_t NOALLOC_BYTES = NOALLOC_TILE_OFF + (size_t)(NOALLOC_MAX_TILES / TILE_BLOCK) * sizeof(BlockCase);
static_assert(NOALLOC_MAX_TILES % TILE_BLOCK == 0, "whole table blocks");
static_assert(desc_size<double>() >= desc_size<float>() && desc_size<double>() >= desc_size<__half>(),
              "descriptor slots sized for the largest descriptor");

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;  // guards the per-device addresses and the host staging below
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
unsigned char g_noalloc_desc_host[NOALLOC_DESC_BYTES];

}  // namespace

extern "C" {

int vplbm_batch_create(vplbm_lattice *const *lats, int n, vplbm_batch **out) {
  if (!out) return VPLBM_EINVAL;
  *out = nullptr;
  if (const char *why = batch_check(lats, n)) {
    if (lats && n >= 1 && lats[0]) lats[0]->fail(VPLBM_EINVAL, "%s", why);
    return VPLBM_EINVAL;
  }
  const int prec = lats[0]->p.precision;
  auto *B = new (std::nothrow) vplbm_batch();
  if (!B) return VPLBM_ENOMEM;
  B->cases.assign(lats, lats + n);
  B->stream = lats[0]->stream;
  B->prec = prec;
  B->trt = lats[0]->p.trt_lambda > 0.0;
  B->aa = lats[0]->aa();
  B->desc_host.assign(desc_size_of(prec) * n, 0);
  B->ncap = n;
  if (hipMalloc((void **)&B->desc_dev, B->desc_host.size()) != hipSuccess ||
      hipStreamCreate(&B->cap_stream) != hipSuccess) {
    (void)hipGetLastError();
    if (B->desc_dev) (void)hipFree(B->desc_dev);
    delete B;
    return VPLBM_ENOMEM;
  }
  *out = B;
  return VPLBM_OK;
}

int vplbm_batch_destroy(vplbm_batch *B) {
  if (!B) return VPLBM_EINVAL;
  (void)hipStreamSynchronize(B->stream);
  if (B->graph) (void)hipGraphExecDestroy(B->graph);
  (void)hipFree(B->desc_dev);
  if (B->tile_case_dev) (void)hipFree(B->tile_case_dev);
  (void)hipStreamDestroy(B->cap_stream);
  delete B;
  return VPLBM_OK;
}

const char *vplbm_batch_last_error(const vplbm_batch *B) { return B ? B->err.c_str() : "null batch"; }

int vplbm_batch_set_lattices(vplbm_batch *B, vplbm_lattice *const *lats, int n) {
  if (!B) return VPLBM_EINVAL;
  if (const char *why = batch_check(lats, n)) return B->fail(VPLBM_EINVAL, why);
  if (lats[0]->p.precision != B->prec || lats[0]->stream != B->stream ||
      (lats[0]->p.trt_lambda > 0.0) != B->trt || lats[0]->aa() != B->aa)
    return B->fail(VPLBM_EINVAL, "the lattices differ from the batch's precision, stream, collision or storage");
  if (n > B->ncap) {
    // room for n descriptors: wait for the work that reads the old table
    int rc = B->hip(hipStreamSynchronize(B->stream), "hipStreamSynchronize");
    if (rc) return rc;
    char *d = nullptr;
    if (hipMalloc((void **)&d, desc_size_of(B->prec) * n) != hipSuccess) {
      (void)hipGetLastError();
      return B->fail(VPLBM_ENOMEM, "batch tables");
    }
    (void)hipFree(B->desc_dev);
    B->desc_dev = d;
    B->ncap = n;
    B->desc_host.assign(desc_size_of(B->prec) * n, 0);
    if (B->graph) (void)hipGraphExecDestroy(B->graph);  // it holds the old tables' addresses
    B->graph = nullptr;
    B->graph_key = GraphKey();
  }
  B->cases.assign(lats, lats + n);
  return VPLBM_OK;
}

int vplbm_batch_set_tile(vplbm_batch *B, int bx, int by) {
  if (!B) return VPLBM_EINVAL;
  if (!batch_tile_ok(bx, by)) return B->fail(VPLBM_EINVAL, "batched launches run 64x4, 128x2 or 256x1 tiles");
  if (B->aa && (bx != 64 || by != 4)) return B->fail(VPLBM_EINVAL, "a batch of AA lattices runs 64x4 tiles");
  if (bx != B->bx || by != B->by) {
    if (B->graph) (void)hipGraphExecDestroy(B->graph);
    B->graph = nullptr;
    B->graph_key = GraphKey();
  }
  B->bx = bx;
  B->by = by;
  return VPLBM_OK;
}

int vplbm_batch_get_tile(const vplbm_batch *B, int *bx, int *by) {
  if (!B || !bx || !by) return VPLBM_EINVAL;
  *bx = B->bx;
  *by = B->by;
  return VPLBM_OK;
}

int vplbm_batch_step(vplbm_batch *B, const int *nsteps) {
  if (!B || !nsteps) return VPLBM_EINVAL;
  const int n = (int)B->cases.size();
  // the tile table holds the tiles of every lattice (its size when all are active)
  long long need = 0;
  // (chunks with moving disks or AA lattices run 64x4 tiles)
  for (vplbm_lattice *L : B->cases) need += std::max(batch_tiles(L, B->bx, B->by), batch_tiles(L, 64, 4));
  if (need > B->tile_case_cap) {
    int rc = B->hip(hipStreamSynchronize(B->stream), "hipStreamSynchronize");
    if (rc) return rc;
    if (B->tile_case_dev) (void)hipFree(B->tile_case_dev);
    B->tile_case_dev = nullptr;
    B->tile_case_cap = 0;
    if (B->graph) (void)hipGraphExecDestroy(B->graph);  // it holds the old table's address
    B->graph = nullptr;
    B->graph_key = GraphKey();
    rc = B->hip(hipMalloc((void **)&B->tile_case_dev, sizeof(BlockCase) * (size_t)table_entries(need)),
                "lattice table");
    if (rc) return rc;
    B->tile_case_cap = need;
  }
  BatchExec X;
  X.prec = B->prec;
  X.trt = B->trt;
  X.aa = B->aa;
  X.bx = B->bx;
  X.by = B->by;
  X.stream = B->stream;
  X.desc_dev = B->desc_dev;
  X.tile_dev = B->tile_case_dev;
  X.tile_cap = B->tile_case_cap;
  X.desc_host = B->desc_host.data();
  X.cap_stream = B->cap_stream;
  X.graph = &B->graph;
  X.graph_key = &B->graph_key;
  std::string err;
  const int rc = batch_run(X, B->cases.data(), n, nsteps, err);
  if (rc) B->err = err;
  return rc;
}

int vplbm_batch_step_noalloc(vplbm_lattice *const *lats, int n, const int *nsteps) {
  if (!lats || n < 1 || !lats[0]) return VPLBM_EINVAL;
  vplbm_lattice *L0 = lats[0];
  if (!nsteps) return L0->fail(VPLBM_EINVAL, "NULL step counts");
  if (const char *why = batch_check(lats, n)) return L0->fail(VPLBM_EINVAL, "%s", why);
  if (n > NOALLOC_MAX_CASES)
    return L0->fail(VPLBM_EINVAL, "vplbm_batch_step_noalloc takes at most %d lattices", NOALLOC_MAX_CASES);
  long long need = 0;
  for (int k = 0; k < n; ++k) need += batch_tiles(lats[k], 64, 4);
  if (need > NOALLOC_MAX_TILES)
    return L0->fail(VPLBM_EINVAL, "%lld tiles of 64x4 cells exceed the %lld of vplbm_batch_step_noalloc", need,
                    NOALLOC_MAX_TILES);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    (void)hipGetLastError();
    return L0->fail(VPLBM_EHIP, "no usable current device");
  }
  if (!g_scratch_ptr[dev]) {
    // once per device, with that device current: the array's device address
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return L0->fail(VPLBM_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
  }
  char *base = (char *)g_scratch_ptr[dev];
  BatchExec X;
  X.prec = L0->p.precision;
  X.trt = L0->p.trt_lambda > 0.0;
  X.aa = L0->aa();
  X.stream = L0->stream;
  X.desc_dev = base;
  X.tile_dev = (BlockCase *)(base + NOALLOC_TILE_OFF);
  X.tile_cap = NOALLOC_MAX_TILES;
  X.desc_host = (char *)g_noalloc_desc_host;
  std::string err;
  const int rc = batch_run(X, lats, n, nsteps, err);
  if (rc) L0->err = err;
  if (!rc) {
    // the host staging is reused by the next call: its copies must be done
    // before the lock is released
    const hipError_t e = hipStreamSynchronize(X.stream);
    if (e != hipSuccess) return L0->fail(VPLBM_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
  }
  return rc;
}

}  // extern "C"
