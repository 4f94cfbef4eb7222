/*
 * vplbm_oracle.c -- plain FP64 CPU oracle for the VP-LBM step and its two
 * fluid-force reductions.  TEST INFRASTRUCTURE ONLY: the tests, the smoke
 * check and the benchmark's CPU-baseline leg call it; the product path never
 * links or loads it.
 *
 * Everything here is written straight from the paper (Liberge & Beghein,
 * "About fluid forces computation for Volume Penalization coupled with
 * Lattice Boltzmann method") and is deliberately slow and obvious:
 * array-of-structures layout f[(y*nx + x)*9 + a], one pass per operation,
 * no fusion, no blocking.  It shares no code with the HIP library.
 *
 * One step n (state between steps: post-collision populations ft^{n-1}):
 *   1. momentum exchange on ft^{n-1}           (Sec. 2.3.1, Eqs. MMEL, total force, fluidtorque)
 *   2. streaming  f^n_a(x) = ft^{n-1}_a(x-c_a)  (Eq. eqBd, D2Q9 velocity set of Sec. 2.2)
 *   3. stress integration on f^n               (Sec. 2.3.2, Eq. defFf and the sigma definition)
 *   4. moments, penalized velocity            (Eqs. updatestep, updatestep3, updatestepm)
 *   5. equilibrium, forcing term, BGK         (BGK operator and f^eq of Sec. 2.2; forcing per Eq. eqBd
 *                                               and the (1 - dt/(2 tau)) prefactor of Eq. TRT)
 * Readings where the paper is silent (forcing-term form, edge rules, time
 * level of the forces, SI sample node) are listed in the design notes and
 * restated at each function below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 9

/* D2Q9 velocity set, Sec. 2.2: c_0 = 0, c_1..4 axis, c_5..8 diagonals. */
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* weights omega_alpha, Sec. 2.2: 4/9, 1/9 (axes), 1/36 (diagonals), summing
 * to one.  1/9 and 1/36 are the nearest doubles; the rest weight is the
 * double just above the one nearest to 4/9, the exact remainder
 * 1 - 4 w_1 - 4 w_5, so that the weights sum to exactly one in binary as they
 * do in the paper.  With the nearest double for 4/9 as well the sum falls
 * short by 2^-54, and every collision would remove that fraction of the
 * cell's mass divided by tau. */
static const double W[Q] = {0x1.c71c71c71c71dp-2, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* opposite direction alpha-bar, c_abar = -c_a (Sec. 2.2, TRT paragraph) */
static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0; /* c_s^2 = c^2/3 with c = 1 */

enum { EDGE_PERIODIC = 0, EDGE_VELOCITY = 1, EDGE_FREESLIP = 2, EDGE_OUTFLOW = 3, EDGE_CONVECTIVE = 4 };
enum { WEST = 0, EAST = 1, SOUTH = 2, NORTH = 3 };

typedef struct {
  int nx, ny;
  double tau, eta, rho0;
  int edge_kind[4];      /* west, east, south, north */
  double edge_u[4][2];   /* wall / inflow velocity of VELOCITY edges; [0] is the
                            convection speed U of CONVECTIVE edges */
  double gx, gy;         /* uniform external force density (tests) */
  double trt_lambda;     /* > 0: two-relaxation-time collision with this magic
                            parameter (Eq. TRT); <= 0: BGK */
} orc_params;

typedef struct {
  double x, y, theta, u, v, omega; /* reference point, angle, velocities */
} orc_body;

/* ------------------------------------------------------------------------ */
/* per-cell algebra                                                          */
/* ------------------------------------------------------------------------ */

/* Second-order equilibrium, Sec. 2.2:
 * f^eq_a = w_a rho (1 + c.u/cs^2 + uu:(cc - cs^2 I)/(2 cs^4)). */
void orc_equilibrium(double rho, double ux, double uy, double feq[Q]) {
  double uu = ux * ux + uy * uy;
  for (int a = 0; a < Q; ++a) {
    double cu = CX[a] * ux + CY[a] * uy; /* c_a . u, and uu:c_a c_a = (c_a . u)^2 */
    feq[a] = W[a] * rho * (1.0 + cu / CS2 + (cu * cu - CS2 * uu) / (2.0 * CS2 * CS2));
  }
}

/* Forcing term for a force density F, in the form of Guo, Zheng & Shi (2002),
 * which the paper cites for F_alpha without printing it:
 *   F_a = w_a [ (c_a - u)/cs^2 + (c_a.u) c_a / cs^4 ] . F
 * The (1 - 1/(2 tau)) prefactor is applied by the caller (Eq. TRT). */
void orc_forcing(double ux, double uy, double Fx, double Fy, double out[Q]) {
  for (int a = 0; a < Q; ++a) {
    double cu = CX[a] * ux + CY[a] * uy;
    double tx = (CX[a] - ux) / CS2 + cu * CX[a] / (CS2 * CS2);
    double ty = (CY[a] - uy) / CS2 + cu * CY[a] / (CS2 * CS2);
    out[a] = W[a] * (tx * Fx + ty * Fy);
  }
}

/* Rigid-body velocity at (x, y): u_s = u_G + omega e_z x (x - x_G). */
static void rigid_velocity(const orc_body *b, double x, double y, double *ux, double *uy) {
  *ux = b->u - b->omega * (y - b->y);
  *uy = b->v + b->omega * (x - b->x);
}

/* Moments and penalized velocity of one cell (Eqs. updatestep..updatestepm).
 *   rho = sum f,   m = sum c f,   k = chi/eta,
 *   u   = (m + G/2 + (k/2) rho u_s) / (rho (1 + k/2))      (Eq. updatestepm, with the
 *                                                           external density G added per Eq. updatestep)
 *   F   = G - rho k (u - u_s)                               (penalization term of Eq. 1 as a force density)
 * F is evaluated through the identity rho k (u - u_s) = k/(1 + k/2) (m + G/2 - rho u_s),
 * which follows from the line above and avoids multiplying a large k by a
 * difference of nearly equal numbers. */
void orc_cell_macro(const orc_params *p, const double f[Q], int chi, double usx, double usy,
                    double *rho, double *ux, double *uy, double *Fx, double *Fy) {
  double r = 0.0, mx = 0.0, my = 0.0;
  for (int a = 0; a < Q; ++a) {
    r += f[a];
    mx += CX[a] * f[a];
    my += CY[a] * f[a];
  }
  double k = chi ? 1.0 / p->eta : 0.0; /* eta = +inf switches penalization off */
  double hx = mx + 0.5 * p->gx, hy = my + 0.5 * p->gy;
  *rho = r;
  *ux = (hx + 0.5 * k * r * usx) / (r * (1.0 + 0.5 * k));
  *uy = (hy + 0.5 * k * r * usy) / (r * (1.0 + 0.5 * k));
  double kk = k / (1.0 + 0.5 * k);
  *Fx = p->gx - kk * (hx - r * usx);
  *Fy = p->gy - kk * (hy - r * usy);
}

/* ------------------------------------------------------------------------ */
/* streaming with edge rules (Eq. eqBd; edge conditions of the Applications  */
/* section: inlet half-way bounce-back, symmetry u.n = 0, no-slip walls,     */
/* free outflow).                                                            */
/* ------------------------------------------------------------------------ */

static int mirror_x(int a) { /* c -> (-cx, cy) */
  for (int b = 0; b < Q; ++b)
    if (CX[b] == -CX[a] && CY[b] == CY[a]) return b;
  return -1;
}
static int mirror_y(int a) { /* c -> (cx, -cy) */
  for (int b = 0; b < Q; ++b)
    if (CX[b] == CX[a] && CY[b] == -CY[a]) return b;
  return -1;
}

/* Value of population a arriving at (x, y) after streaming, read from the
 * post-collision field ft.  The source x - c_a is resolved axis by axis, x
 * first:
 *   periodic  : wrap the coordinate;
 *   outflow   : clamp to the edge (zero-gradient);
 *   free-slip : specular reflection -- take the mirrored population from the
 *               edge cell itself in that axis;
 *   velocity  : half-way bounce-back with wall velocity u_w, ends the search:
 *               f_a(x) = ft_abar(x) + 2 w_a rho0 (c_a . u_w) / cs^2;
 *   convective: the convective outflow condition (cited in the application
 *               section): the incoming population obeys df/dt + U df/dn = 0,
 *               upwind and implicit in the inner value,
 *                 f_a(x, t+1) = (f_a(x, t) + U f_a(x - n, t+1)) / (1 + U),
 *               where f_a(x - n, t+1), the value streamed into the inner
 *               neighbour, is the value the zero-gradient rule reads, and
 *               f_a(x, t) is this population's previous streamed value at x
 *               (fprev).  The first edge crossed (x first) decides; the other
 *               axis then only resolves the clamped source.                  */
double orc_stream_value(const orc_params *p, const double *ft, const double *fprev, int x, int y, int a) {
  int nx = p->nx, ny = p->ny;
  int sx = x - CX[a], sy = y - CY[a];
  int pop = a;
  int conv = -1; /* edge whose convective condition applies */
  if (sx < 0 || sx >= nx) {
    int e = sx < 0 ? WEST : EAST;
    int kind = p->edge_kind[e];
    if (kind == EDGE_VELOCITY) {
      double cu = CX[a] * p->edge_u[e][0] + CY[a] * p->edge_u[e][1];
      return ft[((size_t)y * nx + x) * Q + OPP[a]] + 2.0 * W[a] * p->rho0 * cu / CS2;
    } else if (kind == EDGE_PERIODIC) {
      sx = (sx + nx) % nx;
    } else if (kind == EDGE_OUTFLOW || kind == EDGE_CONVECTIVE) {
      sx = sx < 0 ? 0 : nx - 1;
      if (kind == EDGE_CONVECTIVE) conv = e;
    } else { /* free-slip */
      sx = x;
      pop = mirror_x(pop);
    }
  }
  if (sy < 0 || sy >= ny) {
    int e = sy < 0 ? SOUTH : NORTH;
    int kind = p->edge_kind[e];
    if (kind == EDGE_VELOCITY) {
      double cu = CX[a] * p->edge_u[e][0] + CY[a] * p->edge_u[e][1];
      return ft[((size_t)y * nx + x) * Q + OPP[a]] + 2.0 * W[a] * p->rho0 * cu / CS2;
    } else if (kind == EDGE_PERIODIC) {
      sy = (sy + ny) % ny;
    } else if (kind == EDGE_OUTFLOW || kind == EDGE_CONVECTIVE) {
      sy = sy < 0 ? 0 : ny - 1;
      if (kind == EDGE_CONVECTIVE && conv < 0) conv = e;
    } else {
      sy = y;
      pop = mirror_y(pop);
    }
  }
  double v = ft[((size_t)sy * nx + sx) * Q + pop];
  if (conv >= 0) {
    double U = p->edge_u[conv][0];
    v = (fprev[((size_t)y * nx + x) * Q + a] + U * v) / (1.0 + U);
  }
  return v;
}

/* fprev: the streamed field of the previous step (the initial field before
 * the first step); read only by convective edges, may be NULL without them */
void orc_stream(const orc_params *p, const double *ft, const double *fprev, double *f) {
  int nx = p->nx, ny = p->ny;
#pragma omp parallel for schedule(static) if ((long)nx * ny >= 65536)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x)
      for (int a = 0; a < Q; ++a)
        f[((size_t)y * nx + x) * Q + a] = orc_stream_value(p, ft, fprev, x, y, a);
}

/* Geometric neighbour x + c: wraps periodic axes, returns 0 when the
 * neighbour would lie beyond a non-periodic edge (no lattice link there). */
static int neighbour(const orc_params *p, int x, int y, int cx, int cy, int *ox, int *oy) {
  int nx = p->nx, ny = p->ny;
  int X = x + cx, Y = y + cy;
  if (X < 0 || X >= nx) {
    if (p->edge_kind[X < 0 ? WEST : EAST] != EDGE_PERIODIC) return 0;
    X = (X + nx) % nx;
  }
  if (Y < 0 || Y >= ny) {
    if (p->edge_kind[Y < 0 ? SOUTH : NORTH] != EDGE_PERIODIC) return 0;
    Y = (Y + ny) % ny;
  }
  *ox = X;
  *oy = Y;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* momentum exchange, Sec. 2.3.1                                             */
/* ------------------------------------------------------------------------ */

/* Link form: for every fluid node x_f and direction a whose neighbour
 * x_s = x_f + c_a is solid,
 *   F(x_G) = (c_a - u_G) ft_a(x_f) - (c_abar - u_G) ft_abar(x_s)       (Eq. MMEL)
 * summed over links (total force) and weighted by (x_G - x_ref) x F (Eq.
 * fluidtorque).  The interface point of a link is its midpoint,
 * x_f + c_a/2, measured from the fluid node; u_G there is the rigid-body
 * velocity.  ft is the post-collision field (the tilde of Eq. MMEL). */
void orc_momentum_exchange(const orc_params *p, const double *ft, const uint8_t *ids,
                           const orc_body *bodies, int nbody, double *out) {
  /* ids: body id of each cell (0 = fluid, 1..nbody); a link belongs to the
   * body of its solid node, its torque is taken about that body's reference
   * point and u_Gamma is that body's rigid velocity.  out[3 (b - 1) + k]. */
  for (int k = 0; k < 3 * nbody; ++k) out[k] = 0.0;
  int nx = p->nx, ny = p->ny;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      if (ids[(size_t)y * nx + x]) continue;
      for (int a = 1; a < Q; ++a) {
        int sx, sy;
        if (!neighbour(p, x, y, CX[a], CY[a], &sx, &sy)) continue;
        int id = ids[(size_t)sy * nx + sx];
        if (!id) continue;
        const orc_body *b = &bodies[id - 1];
        double gx = x + 0.5 * CX[a], gy = y + 0.5 * CY[a];
        double ugx, ugy;
        rigid_velocity(b, gx, gy, &ugx, &ugy);
        double fo = ft[((size_t)y * nx + x) * Q + a];
        double fi = ft[((size_t)sy * nx + sx) * Q + OPP[a]];
        double lx = (CX[a] - ugx) * fo - (CX[OPP[a]] - ugx) * fi;
        double ly = (CY[a] - ugy) * fo - (CY[OPP[a]] - ugy) * fi;
        double *o = &out[3 * (id - 1)];
        o[0] += lx;
        o[1] += ly;
        o[2] += (gx - b->x) * ly - (gy - b->y) * lx;
      }
    }
}

/* ------------------------------------------------------------------------ */
/* stress integration, Sec. 2.3.2                                           */
/* ------------------------------------------------------------------------ */

/* Stress at one fluid node from pre-collision populations f (Sec. 2.3.2):
 *   sigma = -(rho - rho0) cs^2 I - (1 - 1/(2 tau)) sum_a c_a c_a (f_a - f^eq_a)
 * with the pressure taken relative to rho0 (identical forces for closed
 * point sets; see the design notes).  u is the velocity of Eq. updatestep. */
void orc_node_stress(const orc_params *p, const double f[Q], double s[3]) {
  double rho, ux, uy, Fx, Fy, feq[Q];
  orc_cell_macro(p, f, 0, 0.0, 0.0, &rho, &ux, &uy, &Fx, &Fy);
  orc_equilibrium(rho, ux, uy, feq);
  double pxx = 0.0, pxy = 0.0, pyy = 0.0;
  for (int a = 0; a < Q; ++a) {
    double d = f[a] - feq[a];
    pxx += CX[a] * CX[a] * d;
    pxy += CX[a] * CY[a] * d;
    pyy += CY[a] * CY[a] * d;
  }
  double fac = 1.0 - 1.0 / (2.0 * p->tau);
  double pr = (rho - p->rho0) * CS2;
  s[0] = -pr - fac * pxx;
  s[1] = -fac * pxy;
  s[2] = -pr - fac * pyy;
}

/* F = sum_i S_i sigma(x_i) . n_i,  T = sum_i S_i r_i x sigma(x_i) . n_i
 * (Eq. defFf and its discrete form).  sigma(x_i) is the weighted sum of the
 * stresses of the point's stencil: up to 4 nodes node4[4i..4i+3] (index
 * y*nx + x, -1 = unused) with weights w4 (see orc_si_stencils). */
void orc_stress_integration(const orc_params *p, const double *f, int npts, const double *xy,
                            const double *nrm, const double *ds, const int *node4, const double *w4,
                            const int *pbody, const orc_body *bodies, int nbody, double *out) {
  /* pbody[i]: body (1..nbody) point i belongs to; out[3 (b - 1) + k] */
  for (int k = 0; k < 3 * nbody; ++k) out[k] = 0.0;
  for (int i = 0; i < npts; ++i) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 4; ++k) {
      if (node4[4 * i + k] < 0) continue;
      double sk[3];
      orc_node_stress(p, &f[(size_t)node4[4 * i + k] * Q], sk);
      for (int m = 0; m < 3; ++m) s[m] += w4[4 * i + k] * sk[m];
    }
    const orc_body *b = &bodies[pbody[i] - 1];
    double nx_ = nrm[2 * i], ny_ = nrm[2 * i + 1];
    double tx = ds[i] * (s[0] * nx_ + s[1] * ny_);
    double ty = ds[i] * (s[1] * nx_ + s[2] * ny_);
    double rx = xy[2 * i] - b->x, ry = xy[2 * i + 1] - b->y;
    double *o = &out[3 * (pbody[i] - 1)];
    o[0] += tx;
    o[1] += ty;
    o[2] += rx * ty - ry * tx;
  }
}

/* Sample node of each integration point.  Sec. 2.3.2 takes the populations
 * at the nearest fluid node in a lattice direction near the normal n; read
 * here as: the lattice direction beta with the largest (c_beta . n)/|c_beta|
 * (first one on ties), then, starting from the node nearest to x_i, the first
 * of up to five nodes along c_beta that is fluid and inside the domain.
 * Returns the number of points without a sample node (node = -1). */
int orc_si_nodes(int nx, int ny, const uint8_t *solid, int npts, const double *xy,
                 const double *nrm, int *node) {
  const double S = 0.70710678118654752440; /* 1/sqrt(2) */
  int missing = 0;
  for (int i = 0; i < npts; ++i) {
    double n0 = nrm[2 * i], n1 = nrm[2 * i + 1];
    double score[Q];
    score[1] = n0;
    score[2] = n1;
    score[3] = -n0;
    score[4] = -n1;
    score[5] = (n0 + n1) * S;
    score[6] = (-n0 + n1) * S;
    score[7] = (-n0 - n1) * S;
    score[8] = (n0 - n1) * S;
    int best = 1;
    for (int a = 2; a < Q; ++a)
      if (score[a] > score[best]) best = a;
    int ix = (int)floor(xy[2 * i] + 0.5), iy = (int)floor(xy[2 * i + 1] + 0.5);
    node[i] = -1;
    for (int k = 0; k <= 4; ++k) {
      int X = ix + k * CX[best], Y = iy + k * CY[best];
      if (X < 0 || X >= nx || Y < 0 || Y >= ny) continue;
      if (!solid[(size_t)Y * nx + X]) {
        node[i] = Y * nx + X;
        break;
      }
    }
    if (node[i] < 0) ++missing;
  }
  return missing;
}

/* Stencil of each integration point, as (node, weight) pairs.
 *  rule 0 -- the paper's extrapolation from the closest fluid node in the
 *            direction close to n: one node (orc_si_nodes), weight 1;
 *  rule 1 -- interpolation: the stress at p_i = x_i + 1.5 n_i, bilinear in
 *            the 4 nodes around p_i; when one of them is solid or outside the
 *            lattice the point falls back to rule 0.
 * Unused entries have node -1 and weight 0.  Returns the number of points
 * without a sample node. */
int orc_si_stencils(int nx, int ny, const uint8_t *solid, int npts, const double *xy,
                    const double *nrm, int rule, int *node4, double *w4) {
  int missing = 0;
  for (int i = 0; i < npts; ++i) {
    for (int k = 0; k < 4; ++k) {
      node4[4 * i + k] = -1;
      w4[4 * i + k] = 0.0;
    }
    if (rule == 1) {
      double px = xy[2 * i] + 1.5 * nrm[2 * i], py = xy[2 * i + 1] + 1.5 * nrm[2 * i + 1];
      int i0 = (int)floor(px), j0 = (int)floor(py);
      double fx = px - i0, fy = py - j0;
      int ok = i0 >= 0 && j0 >= 0 && i0 + 1 < nx && j0 + 1 < ny;
      for (int k = 0; k < 4 && ok; ++k) {
        int X = i0 + (k & 1), Y = j0 + (k >> 1);
        if (solid[(size_t)Y * nx + X]) ok = 0;
      }
      if (ok) {
        for (int k = 0; k < 4; ++k) {
          int X = i0 + (k & 1), Y = j0 + (k >> 1);
          node4[4 * i + k] = Y * nx + X;
          w4[4 * i + k] = ((k & 1) ? fx : 1.0 - fx) * ((k >> 1) ? fy : 1.0 - fy);
        }
        continue;
      }
    }
    int node;
    missing += orc_si_nodes(nx, ny, solid, 1, &xy[2 * i], &nrm[2 * i], &node);
    node4[4 * i] = node;
    w4[4 * i] = node >= 0 ? 1.0 : 0.0;
  }
  return missing;
}

/* ------------------------------------------------------------------------ */
/* one full step                                                              */
/* ------------------------------------------------------------------------ */

/* solid  : body id of each cell (0 = fluid, 1..nbody), chi = (id != 0)
 * bodies : the nbody rigid bodies (reference point, velocities)
 * ft_prev: post-collision field of step n-1 (input)
 * f_prev : streamed field of step n-1 (convective edges only; may be NULL)
 * f_work : scratch, receives the streamed pre-collision field f^n
 * ft_next: post-collision field of step n (output)
 * rho/ux/uy: macroscopic fields of step n (may be NULL)
 * me/si  : forces of step n per body, 3 each (ME of ft^{n-1}, SI of f^n);
 *          si may be NULL.  */
int orc_step(const orc_params *p, const double *ft_prev, const double *f_prev, double *f_work,
             double *ft_next, const uint8_t *solid, const orc_body *bodies, int nbody, int npts,
             const double *si_xy, const double *si_n, const double *si_ds, const int *si_body,
             const int *si_node4, const double *si_w4, double *rho_out, double *ux_out, double *uy_out,
             double *me, double *si) {
  int nx = p->nx, ny = p->ny;
  orc_momentum_exchange(p, ft_prev, solid, bodies, nbody, me);
  orc_stream(p, ft_prev, f_prev, f_work);
  if (si) {
    if (npts > 0)
      orc_stress_integration(p, f_work, npts, si_xy, si_n, si_ds, si_node4, si_w4, si_body, bodies, nbody, si);
    else
      for (int k = 0; k < 3 * nbody; ++k) si[k] = 0.0;
  }
  double fac = 1.0 - 1.0 / (2.0 * p->tau);
  /* TRT (Eq. TRT): tau+ = tau sets the viscosity, tau- = Lambda/(tau+ - 1/2) + 1/2 */
  double tau_m = p->trt_lambda > 0.0 ? p->trt_lambda / (p->tau - 0.5) + 0.5 : p->tau;
#pragma omp parallel for schedule(static) if ((long)nx * ny >= 65536)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t c = (size_t)y * nx + x;
      const double *f = &f_work[c * Q];
      int chi = solid[c] ? 1 : 0;
      double usx = 0.0, usy = 0.0;
      if (chi) rigid_velocity(&bodies[solid[c] - 1], (double)x, (double)y, &usx, &usy);
      double rho, ux, uy, Fx, Fy, feq[Q], Fa[Q];
      orc_cell_macro(p, f, chi, usx, usy, &rho, &ux, &uy, &Fx, &Fy);
      orc_equilibrium(rho, ux, uy, feq);
      orc_forcing(ux, uy, Fx, Fy, Fa);
      if (p->trt_lambda > 0.0) {
        /* symmetric / antisymmetric parts relax with tau+ / tau-.  The
         * forcing term is split the same way, its odd part carrying
         * (1 - 1/(2 tau-)): only then is the momentum put in per step exactly
         * F, as the half-force shift of Eq. updatestep presumes (for tau- =
         * tau+ this is the printed (1 - 1/(2 tau+)) F_alpha). */
        double fac_m = 1.0 - 1.0 / (2.0 * tau_m);
        for (int a = 0; a < Q; ++a) {
          double fp = 0.5 * (f[a] + f[OPP[a]]), fm = 0.5 * (f[a] - f[OPP[a]]);
          double ep = 0.5 * (feq[a] + feq[OPP[a]]), em = 0.5 * (feq[a] - feq[OPP[a]]);
          double Fp = 0.5 * (Fa[a] + Fa[OPP[a]]), Fm = 0.5 * (Fa[a] - Fa[OPP[a]]);
          ft_next[c * Q + a] = f[a] - (fp - ep) / p->tau - (fm - em) / tau_m + fac * Fp + fac_m * Fm;
        }
      } else {
        for (int a = 0; a < Q; ++a) /* BGK collision with forcing, Eq. eqBd */
          ft_next[c * Q + a] = f[a] - (f[a] - feq[a]) / p->tau + fac * Fa[a];
      }
      if (rho_out) rho_out[c] = rho;
      if (ux_out) ux_out[c] = ux;
      if (uy_out) uy_out[c] = uy;
    }
  return 0;
}

/* f = f^eq(rho, u) everywhere (initial state; solid cells get u_s). */
void orc_init_fields(const orc_params *p, const double *rho, const double *ux, const double *uy,
                     double *ft) {
  size_t n = (size_t)p->nx * p->ny;
  for (size_t c = 0; c < n; ++c) orc_equilibrium(rho[c], ux[c], uy[c], &ft[c * Q]);
}

/* ------------------------------------------------------------------------ */
/* solid indicator chi, Eq. fcar                                              */
/* ------------------------------------------------------------------------ */

/* Coordinates are taken on a fixed-point grid of 1/4096 cell so that the
 * inside/outside decision at a cell centre (integer coordinates) is exact
 * integer arithmetic. */
#define FIXQ 4096.0
static long long fixq(double v) { return llround(v * FIXQ); }

/* Disk: cell (i, j) is solid iff (i - xc)^2 + (j - yc)^2 <= r^2. */
int orc_mask_disk(int nx, int ny, double xc, double yc, double r, uint8_t *solid) {
  long long X = fixq(xc), Y = fixq(yc), R = fixq(r);
  int count = 0;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      long long dx = (long long)i * 4096 - X, dy = (long long)j * 4096 - Y;
      int in = dx * dx + dy * dy <= R * R;
      solid[(size_t)j * nx + i] = (uint8_t)in;
      count += in;
    }
  return count;
}

/* Polygon: even-odd rule at the cell centre; a centre lying exactly on an
 * edge counts as inside. */
static int point_in_polygon(long long px, long long py, int nv, const long long *vx,
                            const long long *vy) {
  int in = 0;
  for (int e = 0; e < nv; ++e) {
    long long ax = vx[e], ay = vy[e];
    long long bx = vx[(e + 1) % nv], by = vy[(e + 1) % nv];
    long long orient = (bx - ax) * (py - ay) - (by - ay) * (px - ax);
    if (orient == 0 && px >= (ax < bx ? ax : bx) && px <= (ax > bx ? ax : bx) &&
        py >= (ay < by ? ay : by) && py <= (ay > by ? ay : by))
      return 1; /* on the edge */
    if ((ay > py) != (by > py)) {
      /* the edge crosses the horizontal line through P to the right of P
       * iff orient has the sign of (by - ay) */
      if ((orient > 0) == (by > ay)) in = !in;
    }
  }
  return in;
}

int orc_mask_polygon(int nx, int ny, const double *xy, int nvert, uint8_t *solid) {
  if (nvert < 3) { /* no area: no cell inside */
    for (size_t c = 0; c < (size_t)nx * ny; ++c) solid[c] = 0;
    return 0;
  }
  long long *vx = (long long *)malloc(sizeof(long long) * nvert);
  long long *vy = (long long *)malloc(sizeof(long long) * nvert);
  for (int v = 0; v < nvert; ++v) {
    vx[v] = fixq(xy[2 * v]);
    vy[v] = fixq(xy[2 * v + 1]);
  }
  /* a centre outside the vertices' bounding box is neither inside nor on an edge */
  long long x0 = vx[0], x1 = vx[0], y0 = vy[0], y1 = vy[0];
  for (int v = 1; v < nvert; ++v) {
    x0 = vx[v] < x0 ? vx[v] : x0;
    x1 = vx[v] > x1 ? vx[v] : x1;
    y0 = vy[v] < y0 ? vy[v] : y0;
    y1 = vy[v] > y1 ? vy[v] : y1;
  }
  int count = 0;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const long long X = (long long)i * 4096, Y = (long long)j * 4096;
      int in = 0;
      if (X >= x0 && X <= x1 && Y >= y0 && Y <= y1) in = point_in_polygon(X, Y, nvert, vx, vy);
      solid[(size_t)j * nx + i] = (uint8_t)in;
      count += in;
    }
  free(vx);
  free(vy);
  return count;
}

/* ------------------------------------------------------------------------ */
/* rigid body, Eqs. dep1 and theta2                                           */
/* ------------------------------------------------------------------------ */

/* m d2x_G/dt2 = F + m (1 - rho/rho_s) g,  I d2theta/dt2 = T, advanced with
 * semi-implicit (symplectic) Euler and dt = 1: velocities first, then
 * positions with the new velocities. */
void orc_body_update(orc_body *b, const double FT[3], double mass, double inertia, double rho0,
                     double rho_s, double gx, double gy) {
  double buoy = 1.0 - rho0 / rho_s;
  b->u += FT[0] / mass + buoy * gx;
  b->v += FT[1] / mass + buoy * gy;
  b->omega += FT[2] / inertia;
  b->x += b->u;
  b->y += b->v;
  b->theta += b->omega;
}
