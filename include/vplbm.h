/*
 * vplbm.h -- C ABI of the MI355X (gfx950) VP-LBM library.
 *
 * One lattice = a D2Q9 lattice Boltzmann solver (Sec. 2.2 of Liberge &
 * Beghein, "About fluid forces computation for Volume Penalization coupled
 * with Lattice Boltzmann method") on an nx x ny grid, with one penalized
 * rigid body described by a solid indicator chi (Eq. fcar) and penalization
 * factor eta (Eq. 1; moment update Eqs. updatestep..updatestepm).  Each time
 * step is one fused HIP kernel: pull streaming (Eq. eqBd) with edge
 * conditions, moments, penalized velocity, BGK collision with the forcing
 * term, and the two force reductions the paper compares: momentum exchange
 * (Sec. 2.3.1, Eqs. MMEL and fluidtorque) and stress integration (Sec.
 * 2.3.2, Eq. defFf).  A free body follows Eqs. dep1/theta2 on the device.
 *
 * Conventions (all entry points):
 *   - Return 0 (VPLBM_OK) on success, a negative VPLBM_E* code on failure;
 *     no C++ exception crosses the boundary.  vplbm_last_error() returns a
 *     message owned by the handle, valid until the next call on it.
 *   - Units are lattice units (dx = dt = 1, c = 1, c_s^2 = 1/3).
 *   - Host arrays passed in are copied before the call returns; the caller
 *     keeps ownership.  Host output arrays are caller-allocated.
 *   - Field arrays are row-major [ny][nx] (index y*nx + x), cell centres at
 *     integer coordinates (x, y), x to the east, y to the north.
 *   - Work is queued on the HIP stream given at creation and runs
 *     asynchronously; calls that return data to the host synchronize that
 *     stream first.  Kernel faults surface as VPLBM_EHIP at the next
 *     synchronizing call.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Step numbering: "step n" is the n-th lattice update since the last
 *     initialization (vplbm_init_uniform / vplbm_set_fields), n >= 1.
 */
#ifndef VPLBM_H
#define VPLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vplbm_lattice vplbm_lattice; /* opaque */

/* Population storage.  The library stores deviations d_a = f_a - w_a rho0
 * in every precision and computes in FP64 (VPLBM_F64) or FP32 (others). */
enum {
  VPLBM_F64 = 0,    /* double storage, double arithmetic */
  VPLBM_F32 = 1,    /* float storage, float arithmetic */
  VPLBM_F16DEV = 2  /* IEEE half storage of d_a, float arithmetic */
};

/* Edge conditions (the Applications section uses an inlet with half-way
 * bounce-back, symmetry u.n = 0, no-slip walls and a free outflow). */
enum {
  VPLBM_BC_PERIODIC = 0, /* wrap around */
  VPLBM_BC_VELOCITY = 1, /* half-way bounce-back, wall half a cell outside the
                            edge, moving with (ux, uy); (0,0) = no-slip */
  VPLBM_BC_FREESLIP = 2, /* specular reflection (u.n = 0) */
  VPLBM_BC_OUTFLOW = 3,  /* zero-gradient: incoming populations copied from the
                            edge cell's own row/column */
  VPLBM_BC_CONVECTIVE = 4 /* convective outflow (the condition the Applications
                            section cites): an incoming population f at an edge
                            cell follows df/dt + U df/dn = 0, upwind and implicit,
                            f(t+1) = (f(t) + U f_inner(t+1)) / (1 + U), with
                            f_inner(t+1) the value the zero-gradient rule takes
                            and f(t) its own previous value (state kept per edge
                            cell, restarted by vplbm_init_uniform and
                            vplbm_set_fields).  U = ux >= 0 (lattice units); U = 0
                            freezes the incoming populations, large U tends to
                            zero-gradient.  At a corner the x edge decides. */
};

typedef struct {
  int kind;      /* VPLBM_BC_* */
  double ux, uy; /* wall / inflow velocity of VPLBM_BC_VELOCITY; ux is the
                    convection speed U of VPLBM_BC_CONVECTIVE */
} vplbm_edge;

typedef struct {
  int nx, ny;        /* lattice size, each >= 4, ny * pitch < 2^31 cells (pitch: nx
                        rounded up to a multiple of 64); populations are
                        indexed in 64 bits, cells in 32 */
  double tau;        /* BGK relaxation time, > 1/2; nu = (tau - 1/2)/3 (Eq. tauvisco) */
  double eta;        /* penalization factor, > 0; +inf switches penalization off */
  double rho0;       /* reference density (> 0; 1 in every workload here) */
  int precision;     /* VPLBM_F64 / VPLBM_F32 / VPLBM_F16DEV */
  vplbm_edge west, east, south, north;
  int hist_capacity; /* length of the device force-history ring in steps; 0 = 4096 */
  int max_si_points; /* capacity for stress-integration points; 0 = 4096 (max 4096) */
  int max_vertices;  /* capacity for polygon vertices; 0 = 4096 */
  double trt_lambda; /* 0: BGK collision.  > 0: two-relaxation-time collision
                        (Eq. TRT) with tau+ = tau and tau- = trt_lambda/(tau - 1/2)
                        + 1/2 (the paper uses 1/6); the forcing term is split the
                        same way, its odd part weighted by 1 - 1/(2 tau-) */
  int si_rule;       /* stress-integration stencil (Sec. 2.3.2): 0 = the paper's
                        nearest fluid node in the lattice direction closest to n;
                        1 = sigma interpolated (bilinear, 4 fluid nodes) at
                        x + 1.5 n, falling back to rule 0 when a node is solid;
                        rule 1 needs max_si_points in 1..1024 and keeps
                        up to 4 sample records per point */
  int max_bodies;    /* bodies one lattice can hold (ids 1..max_bodies in the
                        mask, see vplbm_set_body_ids); 0 = 1, max 63 */
  int max_interface_cells; /* momentum-exchange slots, one per interface cell
                        (a cell with a lattice link to the other phase);
                        0 = min(nx ny, 32 (nx + ny)).  Set-up fails with
                        VPLBM_EINVAL when the geometry has more.  A moving
                        disk keeps per-tile force sums here instead, for the
                        64 x 4 tiles its window of 2 h + 1 cells a side can
                        meet: 2 (ceil(2 h / 64) + 1) (ceil(2 h / 4) + 1)
                        slots, h = ceil(the larger of its radius and its
                        points' largest distance from its reference point)
                        + 8 */
  int streaming;     /* population storage (not a choice the paper makes):
                        VPLBM_STREAM_AB (0) = two buffers, one read and one
                        written per step; VPLBM_STREAM_AA (1) = one buffer
                        updated in place, odd and even steps alternating
                        (half the population memory, the same bytes moved
                        per cell update, the same arithmetic per cell: the
                        results agree with VPLBM_STREAM_AB to rounding).
                        AA runs with the 64x4 tile only; a batch takes
                        AA lattices when all of its lattices are AA */
} vplbm_params;

enum {
  VPLBM_STREAM_AB = 0,
  VPLBM_STREAM_AA = 1
};

/* Rigid-body state in lattice units: reference point (centre of a disk,
 * the given torque reference of a polygon), angle, translational and
 * angular velocity.  The velocity field of the body is
 * u_s(x) = (u - omega (y - y_G), v + omega (x - x_G)). */
typedef struct {
  double x, y, theta, u, v, omega;
} vplbm_body_state;

enum {
  VPLBM_OK = 0,
  VPLBM_EINVAL = -1,   /* invalid argument; nothing changed */
  VPLBM_ENOMEM = -2,   /* device memory too small or allocation failed */
  VPLBM_EHIP = -3,     /* HIP runtime error (including asynchronous kernel faults) */
  VPLBM_ESTATE = -4,   /* call not valid in the current state */
  VPLBM_EUNSTABLE = -5, /* the solution diverged: a step met a non-finite density
                           (reported by the next vplbm_sync or force read;
                           the state is then meaningless until re-initialized) */
  VPLBM_ENOSAMPLE = -6 /* a stress-integration point found no fluid sample node */
};

enum { VPLBM_FORCE_ME = 0, VPLBM_FORCE_SI = 1 };
enum { VPLBM_STEP_MACRO = 1 }; /* vplbm_step flag: write rho, u on the last step */

/* Exact device bytes a lattice with these parameters needs (populations
 * A and B, or one buffer with the AA pattern; mask, macroscopic fields,
 * per-cell force slots, force history, tables);
 * 0 if the parameters are invalid.  Sizes follow the D2Q9 lattice of
 * Sec. 2.2 (9 populations per cell). */
size_t vplbm_required_bytes(const vplbm_params *p);

/* Create a lattice: the fluid domain Omega of Sec. 2.1 discretized as the
 * D2Q9 lattice of Sec. 2.2, with relaxation time tau (Eq. tauvisco gives the
 * viscosity) and penalization factor eta (Eq. 1, Eq. fcar).  dev_mem: device
 * buffer of at least vplbm_required_bytes(p) bytes, 256-byte aligned,
 * borrowed for the lifetime of the handle (the caller frees it after
 * vplbm_destroy), or NULL to let the library allocate (and free) it.
 * hip_stream: a hipStream_t, or NULL for the default stream.  Populations
 * start at rest (f = f^eq(rho0, 0), Sec. 2.2), the mask is all fluid, the
 * body at rest at the origin.  VPLBM_EINVAL for invalid parameters (message
 * in vplbm_last_error(NULL)), VPLBM_ENOMEM for a buffer that is too small or
 * misaligned or a failed allocation. */
int vplbm_create(const vplbm_params *p, void *dev_mem, size_t dev_bytes, void *hip_stream,
                 vplbm_lattice **out);
/* Release a lattice (waits for its stream; frees the device buffer only if
 * the library allocated it).  VPLBM_EINVAL for NULL.  Resource handling of
 * this library, not a step of the paper's method. */
int vplbm_destroy(vplbm_lattice *lat);
/* Message of the last failed call on the handle; with lat == NULL, the
 * message of the last failed vplbm_create on the calling thread (error
 * reporting of this library, not part of the method). */
const char *vplbm_last_error(const vplbm_lattice *lat);

/* Set the populations to f^eq(rho, u) (second-order equilibrium, Sec. 2.2):
 * fluid cells take (ux, uy), solid cells the body velocity u_s(x).  Resets
 * the step counter and the force history. */
int vplbm_init_uniform(vplbm_lattice *lat, double rho, double ux, double uy);
/* Same with per-cell host fields rho, ux, uy ([ny][nx] each). */
int vplbm_set_fields(vplbm_lattice *lat, const double *rho, const double *ux, const double *uy);

/* Uniform external force density G added to the penalization force in every
 * cell (Eq. updatestep); (0, 0) by default. */
int vplbm_set_body_force(vplbm_lattice *lat, double gx, double gy);

/* Body geometry -> chi (Eq. fcar), built on the device.  Coordinates are
 * rounded to 1/4096 of a cell; a cell is solid when its centre lies inside
 * (disk: distance <= r; polygon: even-odd rule, points on an edge inside).
 * The reference point becomes (xc, yc) for a disk and (xref, yref) for a
 * polygon (nvert >= 3, implicitly closed).  Replaces any previous body. */
int vplbm_set_body_disk(vplbm_lattice *lat, double xc, double yc, double r);
int vplbm_set_body_polygon(vplbm_lattice *lat, const double *xy, int nvert, double xref,
                           double yref);
/* Arbitrary solid indicator (host, [ny][nx], nonzero = solid), static. */
int vplbm_set_mask(vplbm_lattice *lat, const uint8_t *solid);
/* Several static bodies in one lattice: ids [ny][nx] host bytes, 0 = fluid,
 * b in 1..nbody = solid cell of body b (nbody <= max_bodies); ref_xy[2*nbody]
 * the reference point of each body (its torques are taken about it).  Every
 * momentum-exchange link belongs to the body of its solid node, so a fluid
 * cell may be linked to one body only (bodies at least two cells apart;
 * VPLBM_EINVAL otherwise).  Replaces any previous body and removes all
 * stress-integration points.  Bodies set this way are static. */
int vplbm_set_body_ids(vplbm_lattice *lat, const uint8_t *ids, int nbody, const double *ref_xy);

/* Prescribed rigid motion: the state is applied now, and each step advances
 * the position and angle by the (constant) velocities; the disk's mask and
 * its stress-integration points follow the motion.  Polygon and host-mask
 * bodies are static: for them only the reference point and angle may be set
 * and the velocities must be zero (VPLBM_EINVAL otherwise). */
int vplbm_set_body_motion(vplbm_lattice *lat, const vplbm_body_state *s);

/* Free disk (Eqs. dep1, theta2): mass m = rho_s pi r^2, moment of inertia
 * m r^2 / 2, gravity (gx, gy) with buoyancy factor (1 - rho0/rho_s), driven
 * by the momentum-exchange (force_source = VPLBM_FORCE_ME) or
 * stress-integration (VPLBM_FORCE_SI) force of each step; semi-implicit
 * Euler, dt = 1, in FP64 on the device. */
int vplbm_set_body_dynamics(vplbm_lattice *lat, double rho_s, double gx, double gy,
                            int force_source);

/* One of several moving disks (vplbm_set_moving_disks): centre (x, y),
 * radius r, angle theta, velocities (u, v, omega); rho_s > 0 makes it free
 * (Eqs. dep1, theta2 with m = rho_s pi r^2, I = m r^2 / 2), rho_s = 0 gives
 * it the prescribed motion of its velocities. */
typedef struct {
  double x, y, r, theta, u, v, omega, rho_s;
} vplbm_disk;

/* Several moving disks in one lattice (n in 1..4, n <= max_bodies): disk k
 * becomes body k + 1.  Each follows its own motion (free or prescribed, as
 * for body 1 in vplbm_set_body_motion and vplbm_set_body_dynamics) with its
 * own momentum-exchange and stress-integration forces; the free ones share
 * the gravity (gx, gy) and the force that drives them (force_source).  The
 * paper moves one body at a time; this applies its single-body equations to
 * each disk, with no contact model: the disks must start at least two cells
 * apart and one cell inside the lattice, and a step that brings two of them
 * within one cell flags VPLBM_EINVAL ("a fluid cell is linked to two
 * different bodies") at the next check.  Replaces any previous body and
 * removes all stress-integration points (set them per disk with
 * vplbm_set_si_points_body).  The window each disk keeps must fit
 * max_interface_cells (see vplbm_params). */
int vplbm_set_moving_disks(vplbm_lattice *lat, const vplbm_disk *disks, int n, double gx, double gy,
                           int force_source);

/* Stress-integration points (Sec. 2.3.2): world coordinates xy[2*npts],
 * outward unit normals nrm[2*npts], integration lengths ds[npts], at the
 * current body state; they move rigidly with the body.  With si_rule 0 each
 * point takes its stress from a sample node: the lattice direction closest
 * to n, walked from the nearest node for up to 5 nodes until a fluid node is
 * met (VPLBM_ENOSAMPLE if none); with si_rule 1 from the bilinear
 * interpolation at x + 1.5 n (see vplbm_params).  npts = 0 removes the
 * points. */
int vplbm_set_si_points(vplbm_lattice *lat, const double *xy, const double *nrm, const double *ds,
                        int npts);
/* The same for body `body` (1..nbody) of a multi-body lattice; the points of
 * the other bodies stay.  All bodies' points together must fit
 * max_si_points, and a sample node may serve one body only (VPLBM_EINVAL).
 * vplbm_set_si_points is this call for body 1. */
int vplbm_set_si_points_body(vplbm_lattice *lat, int body, const double *xy, const double *nrm,
                             const double *ds, int npts);

/* Advance nsteps time steps (asynchronous).  One step n is the update of
 * Sec. 2.2 with the penalization of Eqs. updatestep..updatestepm: pull
 * streaming (Eq. eqBd), moments, penalized velocity and force density,
 * collision with the forcing term (Eq. TRT prefactor), and, fused into the
 * same kernel, the momentum exchange (Eqs. MMEL, fluidtorque) and stress
 * integration (Eq. defFf) of that step; a moving disk then follows Eqs.
 * dep1/theta2.  flags: VPLBM_STEP_MACRO makes the last step also store rho
 * and the penalized velocity u for vplbm_read_macro.  VPLBM_EINVAL for
 * nsteps < 0; nsteps = 0 does nothing. */
int vplbm_step(vplbm_lattice *lat, int nsteps, int flags);
/* Same as vplbm_step (the update of Sec. 2.2 with Eqs. updatestep..
 * updatestepm and the forces of Sec. 2.3), for measurement: HIP events
 * bracket every launch of the fused step kernel on the lattice's stream; on
 * return (the stream is synchronized) *kernel_ms holds the summed duration
 * of those launches in milliseconds.  The timing is this library's
 * instrumentation; the paper reports no kernel times. */
int vplbm_step_timed(vplbm_lattice *lat, int nsteps, int flags, double *kernel_ms);
/* Wait for the lattice's queued work and publish the last step's forces
 * (Sec. 2.3.1 and 2.3.2: the sums the next step would otherwise make).
 * Returns VPLBM_EUNSTABLE once a step met a non-finite density,
 * VPLBM_ENOSAMPLE when a moving body's point lost its sample node (the
 * sampling of Sec. 2.3.2 needs a fluid node along the normal), VPLBM_EHIP
 * for a kernel fault. */
int vplbm_sync(vplbm_lattice *lat);
/* Steps taken since the last initialization (-1 for NULL): the time index
 * n of Sec. 2.2 (dt = 1). */
long long vplbm_step_count(const vplbm_lattice *lat);
/* Workgroup tile of the step kernel (an execution choice, not one the
 * paper makes), bx cells along x times by rows: 64x1, 64x2, 64x4, 128x1,
 * 128x2 or 256x1.  The default is 64x4, or 128x2 when the two population
 * buffers exceed 1 GiB (FP64: 256 MB).  Results do not depend on it, forces
 * included: they are summed per interface cell and per sample record, in an
 * order fixed at geometry set-up.  A lattice with VPLBM_STREAM_AA or with
 * moving disks accepts 64x4 only (VPLBM_EINVAL otherwise).  Batched launches
 * use the batch's own tile (vplbm_batch_set_tile), not this setting. */
int vplbm_set_tile(vplbm_lattice *lat, int bx, int by);
/* The tile the lattice's own steps use (*bx cells along x, *by rows; see
 * vplbm_set_tile). */
int vplbm_get_tile(const vplbm_lattice *lat, int *bx, int *by);

/* Forces of the last step on body 1, out = (Fx, Fy, Tz), torque about the
 * body's reference point: vplbm_forces_me by momentum exchange (Sec. 2.3.1,
 * Eqs. MMEL and fluidtorque, summed over the links), evaluated on the
 * post-collision populations of step n-1; vplbm_forces_si by stress
 * integration (Sec. 2.3.2, Eq. defFf as the discrete sum over the registered
 * points, sigma of the streamed (pre-collision) populations of step n).
 * VPLBM_ESTATE before the first step. */
int vplbm_forces_me(vplbm_lattice *lat, double out[3]);
int vplbm_forces_si(vplbm_lattice *lat, double out[3]);
/* Stress integration over the given points on the current streamed state
 * (one-shot, not registered; sample nodes chosen as above). */
int vplbm_forces_si_at(vplbm_lattice *lat, const double *xy, const double *nrm, const double *ds,
                       int npts, double out[3]);
/* History: out[3*k..3*k+2] = forces of step first_step + k, k < n.  The
 * ring keeps the last hist_capacity steps (VPLBM_EINVAL outside it). */
int vplbm_force_history(vplbm_lattice *lat, int which, long long first_step, int n, double *out);
/* Per body (1..nbody) of a multi-body lattice: forces of the last step
 * (which = VPLBM_FORCE_ME or VPLBM_FORCE_SI) and their history.  The
 * single-body calls above are these for body 1. */
int vplbm_forces_body(vplbm_lattice *lat, int body, int which, double out[3]);
int vplbm_force_history_body(vplbm_lattice *lat, int body, int which, long long first_step, int n,
                             double *out);
/* State of body 1 for the next step: position, angle and velocities of the
 * rigid-body motion of Eqs. dep1 and theta2 (prescribed or free). */
int vplbm_get_body_state(vplbm_lattice *lat, vplbm_body_state *out);
/* The same for body `body` (1..nbody): a moving disk's state, or a static
 * body's reference point with zero angle and velocities. */
int vplbm_get_body_state_of(vplbm_lattice *lat, int body, vplbm_body_state *out);

/* rho (Eq. updatestep) and the penalized velocity u (Eq. updatestepm) of
 * the last step, which must have been run with VPLBM_STEP_MACRO
 * (VPLBM_ESTATE otherwise); host arrays [ny][nx], caller-owned. */
int vplbm_read_macro(vplbm_lattice *lat, double *rho, double *ux, double *uy);
/* The same (Eqs. updatestep, updatestepm) into caller-owned device arrays
 * [ny][nx] of the compute type (double for VPLBM_F64, float for VPLBM_F32 and
 * VPLBM_F16DEV), asynchronously on the lattice's stream (no host transfer). */
int vplbm_read_macro_device(vplbm_lattice *lat, void *rho, void *ux, void *uy);
/* The same (Eqs. updatestep, updatestepm) restricted to the window of w
 * columns from x0 and h rows from y0 (host arrays [h][w]); VPLBM_EINVAL if
 * it leaves the lattice. */
int vplbm_read_macro_window(vplbm_lattice *lat, int x0, int y0, int w, int h, double *rho, double *ux,
                            double *uy);
/* Post-collision populations f_a = w_a rho0 + d_a of the last step (or of the
 * initialization) as host doubles [9][ny][nx], in either storage mode: the
 * D2Q9 distributions of Sec. 2.2 after the collision of Eq. TRT. */
int vplbm_read_populations(vplbm_lattice *lat, double *f);
/* The same (Sec. 2.2) for a window, host array [9][h][w]. */
int vplbm_read_populations_window(vplbm_lattice *lat, int x0, int y0, int w, int h, double *f);
/* Mask bytes [ny][nx]: bits 0-5 body id (0 = fluid; chi of Eq. fcar is
 * id != 0), bit 6 stress-integration sample node (Sec. 2.3.2), bit 7
 * interface cell (a neighbour has the other phase: the cells whose links
 * enter the momentum exchange of Sec. 2.3.1). */
int vplbm_read_mask(vplbm_lattice *lat, uint8_t *out);

/* ---- batches --------------------------------------------------------------
 * The paper runs one case at a time; batching is an execution choice of
 * this library.  A batch steps several lattices with one launch of the fused
 * step kernel per time step (the step of vplbm_step: Sec. 2.2 with Eqs.
 * updatestep..updatestepm and the forces of Sec. 2.3): the tiles of all
 * active lattices are laid end to end and each workgroup finds its lattice
 * from a device table.  Each lattice computes exactly what vplbm_step would
 * (the same per-cell arithmetic and reduction order, whatever the tile), so
 * its results do not depend on what else is in the batch; moving disks are
 * stepped inside the same launch.  Runs of steps are replayed from a
 * captured HIP graph. */
typedef struct vplbm_batch vplbm_batch;

/* All lattices must share the precision, the collision (BGK or TRT of Eq.
 * TRT), the HIP stream and the storage scheme (all VPLBM_STREAM_AB or all
 * VPLBM_STREAM_AA; VPLBM_EINVAL otherwise); a lattice appears once.  The
 * handles stay owned by the caller and must outlive the batch; they must not
 * be stepped concurrently.  Destroy releases the batch's tables and graph;
 * last_error gives the message of its last failed call. */
int vplbm_batch_create(vplbm_lattice *const *lats, int n, vplbm_batch **out);
int vplbm_batch_destroy(vplbm_batch *b);
const char *vplbm_batch_last_error(const vplbm_batch *b);
/* Advance lattice k by nsteps[k] steps of Sec. 2.2 (0 = idle);
 * asynchronous.  Lattices with steps left run together; a lattice drops out
 * when its count is reached.  Forces (Sec. 2.3), histories and states are
 * read per lattice afterwards.  Launches with moving disks (Sec. 3.2) order
 * their tiles by where the disks were a step before, kept in 144 bytes of
 * static device memory per GPU that every batch shares: batches stepped at
 * the same time on one GPU may order each other's work less well, with the
 * same results. */
int vplbm_batch_step(vplbm_batch *b, const int *nsteps);
/* Replace the lattices of a batch (the rules of vplbm_batch_create; the
 * same precision, collision, stream and storage as the batch's first
 * lattices).  The device tables grow only when n exceeds every earlier
 * count, and a captured graph of the same launch shape is reused: a
 * continuous-batching server changes the resident set without rebuilding
 * the batch. */
int vplbm_batch_set_lattices(vplbm_batch *b, vplbm_lattice *const *lats, int n);
/* Tile of the batched launches (workgroup shape, not a choice the paper
 * makes): 64x4 (default), 128x2 or 256x1 cells (with moving disks a batch
 * runs 64x4 whatever this setting); a batch of AA lattices runs
 * 64x4 only (VPLBM_EINVAL otherwise).  Results do not depend on it (forces
 * are summed per interface cell and sample record in a fixed order). */
int vplbm_batch_set_tile(vplbm_batch *b, int bx, int by);
int vplbm_batch_get_tile(const vplbm_batch *b, int *bx, int *by);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the work
 * of vplbm_batch_step on lats[0..n) with nsteps[k] steps each, with 64x4
 * tiles and direct launches (no graph), without allocating anything.  Its
 * tables (lattice descriptors, the lattice of every block of 64 tiles) live
 * in one static device array of the library, 402 KiB per GPU, held
 * until the process ends; limits: n <= 256 lattices, 2^20 tiles of 64x4
 * cells in all (VPLBM_EINVAL beyond, message on lats[0]).  The lattices obey
 * the rules of vplbm_batch_create and are stepped on their common stream,
 * which must belong to the current device.  Every call shares that device's
 * array: calls are serialized inside the library (each returns after its
 * queued work has finished), and work of another thread that uses the same
 * lattices at the same time races.  Results are those of vplbm_batch_step,
 * bit for bit. */
int vplbm_batch_step_noalloc(vplbm_lattice *const *lats, int n, const int *nsteps);

#ifdef __cplusplus
}
#endif
#endif /* VPLBM_H */
