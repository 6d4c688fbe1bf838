/*
 * lbmref.c -- plain CPU FP64 oracle of the double-distribution-function
 * pseudopotential thermal lattice Boltzmann step of Li & Luo
 * (arXiv:1405.2232).
 *
 * TEST INFRASTRUCTURE ONLY: nothing in the product path may load this
 * library.  It is written to be read against the paper, not to be fast:
 * two full arrays (source and destination), one pass that evaluates the
 * moments and the pseudopotential of every node, and a second pass that
 * evaluates the force, collides and streams, node by node, in the order
 * the paper states the model.
 *
 * One time step from the post-streaming state (f, g) at time t:
 *   1. rho = sum_i f_i, j = sum_i e_i f_i, rho*cv*T = sum_i g_i
 *      (zeroth/first moments used in the Chapman-Enskog analysis, Eq. (13)).
 *   2. psi^2 = 2 (p_EOS - rho c_s^2) / (G c^2), psi = sqrt(psi^2)
 *      (Section II.A, the choice of psi that gives a desired EOS).
 *   3. F = pseudopotential force of Eq. (4) (Eq. (2) when beta = 1)
 *      plus the body force rho*(gx, gy) (buoyancy of Section III.B).
 *   4. u = (j + F/2)/rho, the velocity that goes with the forcing term.
 *   5. f_i* = f_i - (f_i - f_i^eq)/tau_f + F_i                    Eq. (1)
 *   6. g_i* = g_i - (g_i - g_i^eq)/tau_g, g_i^eq = cv T f_i^eq    Eq. (7)
 *      plus C_i of Eq. (25) for the corrected equation, Eq. (24).
 *   7. f_i(x + e_i, t + 1) = f_i*(x), the same for g.
 *
 * The third treatment (LBMREF_FD_RK2) replaces steps 6-7 for g by the
 * finite-difference solution of the temperature equation, Eq. (26), with
 * the two-stage Runge-Kutta scheme of Eq. (27); the temperature is then
 * carried as g_i = cv T f_i (so that sum_i g_i = rho cv T still holds).
 *
 * Readings where the paper is silent:
 *   - F_i is the forcing term of Guo et al. (the paper cites it as [21]):
 *     F_i = (1 - 1/(2 tau_f)) w_i [(e_i - u)/c_s^2 + (e_i.u) e_i / c_s^4] . F
 *   - the EOS temperature is the local T (the model is coupled) unless
 *     eos_fixed_T asks for a fixed temperature;
 *   - psi^2 < 0 (outside the EOS domain of a real psi) clamps psi to 0 and
 *     is counted; with beta = 0 only psi^2 enters Eq. (4) and nothing is
 *     clamped;
 *   - Eq. (27) as printed evaluates h2 at T^n + (dt/2) h1 but averages
 *     h1 and h2 with weight dt/2, which is not a second-order pair; it is
 *     read as Heun's method, h2 = K(T^n + dt h1), keeping the printed
 *     average.  The isotropic central differences of Eq. (26) are
 *     grad phi = sum_i w(|e_i|^2) phi(x + e_i) e_i and
 *     lap phi = 2 sum_i w(|e_i|^2) (phi(x + e_i) - phi(x)), with
 *     div(lambda grad T) = lambda lap T + grad lambda . grad T and
 *     lambda = (tau_g - 1/2) cv rho c_s^2 (the conductivity stated after
 *     Eq. (23)); u and rho are those of time t for both stages.  Beyond a
 *     Dirichlet wall the temperature ghost is 2 T_w - T(boundary node),
 *     beyond an adiabatic wall T(boundary node); rho mirrors;
 *   - with phi_divu the term phi div u of Eq. (5), phi = -T (dp_EOS/dT)_rho,
 *     which the paper omits (Eq. (6)), is kept: the finite-difference
 *     treatment adds phi div u / (rho cv) to K(T); the LB treatments add
 *     the source w_i phi div u to g_i* (zeroth moment phi div u, first and
 *     second moments zero; u of time t); div u by the same isotropic
 *     gradient (the velocity ghost beyond a wall is the boundary node's
 *     velocity reversed, for a no-slip wall halfway out);
 *   - open channel (wall_x = 2; the paper states inlet and outlet only as
 *     uniform inflow and fully developed outflow): the inlet sits halfway
 *     left of the first column, where f bounces back with the momentum of
 *     the inlet velocity, f_ib = f_i* - 2 w_i rho (e_i . u_in)/c_s^2, and
 *     g anti-bounces back with the inlet equilibrium's even part,
 *     g_ib = -g_i* + 2 w_i cv rho T_in (1 + 4.5 (e_i.u_in)^2 - 1.5 u_in^2)
 *     (bounces back when the left side is adiabatic); the outlet sits
 *     halfway right of the last column and holds the density rho_out with
 *     the node's own velocity and temperature (zero gradient) by
 *     anti-bounce-back, f_ib = -f_i* + 2 w_i rho_out (1 + 4.5 (e_i.u)^2 -
 *     1.5 u^2), g_ib = -g_i* + 2 w_i cv rho T (1 + 4.5 (e_i.u)^2 - 1.5 u^2);
 *     psi and the finite-difference temperature mirror there;
 *   - walls sit halfway between nodes; f bounces back; g bounces back
 *     (adiabatic) or anti-bounces back with the wall value rho(x) cv T_w
 *     (Dirichlet); the pseudopotential ghost beyond a wall mirrors the
 *     boundary node.  Where a diagonal leaves through a corner of a box,
 *     the corner is adiabatic if either wall is, else Dirichlet at the
 *     mean of the two wall temperatures (no axis preferred); at a corner
 *     of the open channel the plate's condition applies.
 */
#include "lbmref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* D2Q9: rest, four axis directions, four diagonals (Section II.A). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0; /* c_s^2 = c^2/3 with c = 1 */

static int opposite(int i) {
  for (int k = 0; k < 9; ++k)
    if (EX[k] == -EX[i] && EY[k] == -EY[i]) return k;
  return -1;
}

/* interaction weights of Eq. (2): w(1) = 1/3, w(2) = 1/12 */
static double w_sc(int i) {
  int e2 = EX[i] * EX[i] + EY[i] * EY[i];
  if (e2 == 1) return 1.0 / 3.0;
  if (e2 == 2) return 1.0 / 12.0;
  return 0.0;
}

struct lbmref_ctx {
  lbmref_params p;
  long n;
  double *f, *g, *f2, *g2;   /* [9][ny][nx] */
  double *rho, *jx, *jy, *E, *T, *psi, *psi2;
  double *ux, *uy, *K1, *K2, *Ts; /* FD treatment: velocity, stages */
  long clamp_count;
  long step;
  int have_fields;
};

#define IDX(h, x, y) ((long)(y) * (h)->p.nx + (x))
#define PL(h, q) ((long)(q) * (h)->n)

void lbmref_velocities(int *ex, int *ey, double *w) {
  for (int i = 0; i < 9; ++i) {
    ex[i] = EX[i];
    ey[i] = EY[i];
    w[i] = W[i];
  }
}

/* f_i^eq of Section II.A */
void lbmref_feq(double rho, double ux, double uy, double out[9]) {
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    double eu = EX[i] * ux + EY[i] * uy;
    out[i] = rho * W[i] * (1.0 + eu / CS2 + 0.5 * eu * eu / (CS2 * CS2) - 0.5 * uu / CS2);
  }
}

/* Guo forcing term F_i (the forcing term cited for Eq. (1)) */
void lbmref_guo(double tau_f, double ux, double uy, double Fx, double Fy, double out[9]) {
  for (int i = 0; i < 9; ++i) {
    double eu = EX[i] * ux + EY[i] * uy;
    double cx = (EX[i] - ux) / CS2 + eu * EX[i] / (CS2 * CS2);
    double cy = (EY[i] - uy) / CS2 + eu * EY[i] / (CS2 * CS2);
    out[i] = (1.0 - 1.0 / (2.0 * tau_f)) * W[i] * (cx * Fx + cy * Fy);
  }
}

/* correction term C_i of Eq. (25) */
void lbmref_corr(double tau_g, double cvT, double Fx, double Fy, double out[9]) {
  for (int i = 0; i < 9; ++i) {
    double eF = EX[i] * Fx + EY[i] * Fy;
    out[i] = (1.0 - 1.0 / (2.0 * tau_g)) * W[i] * cvT * eF / CS2;
  }
}

/* p_EOS: Carnahan-Starling (the non-ideal EOS used by the workloads) or
 * the ideal gas p = rho R T of Section III. */
double lbmref_pressure(const lbmref_params *p, double rho, double T) {
  if (p->eos == LBMREF_EOS_IDEAL) return rho * p->R * T;
  double eta = p->b * rho / 4.0;
  double num = 1.0 + eta + eta * eta - eta * eta * eta;
  double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
  return rho * p->R * T * num / den - p->a * rho * rho;
}

/* thermal condition beyond a wall of a box: side 0 left, 1 right, 2 bottom,
 * 3 top, -1 where that axis is not crossed.  Where both are crossed (a
 * diagonal leaving through a corner, or a ghost node beyond one), the
 * corner is adiabatic if either wall is, else Dirichlet at the mean of the
 * two wall temperatures: no axis is preferred, so the scheme stays
 * covariant under the exchange of x and y (the walls are a reading: the
 * paper's benchmarks state only which sides hold which condition).
 * Returns the condition and sets *Tw. */
static int wall_condition(const lbmref_params *p, int sx, int sy, double *Tw) {
  const int th[4] = {p->thermal_left, p->thermal_right, p->thermal_bottom, p->thermal_top};
  const double tw[4] = {p->T_left, p->T_right, p->T_bottom, p->T_top};
  if (sx >= 0 && sy >= 0) {
    *Tw = 0.5 * (tw[sx] + tw[sy]);
    if (th[sx] == LBMREF_THERMAL_ADIABATIC || th[sy] == LBMREF_THERMAL_ADIABATIC)
      return LBMREF_THERMAL_ADIABATIC;
    return LBMREF_THERMAL_DIRICHLET;
  }
  const int s = sx >= 0 ? sx : sy;
  *Tw = tw[s];
  return th[s];
}

/* neighbour index with periodic wrap or wall mirror; returns the node
 * whose psi stands in at (x, y) */
static void nb(int nx, int ny, int wall_x, int wall_y, int x, int y, int *xo, int *yo) {
  if (x < 0) x = wall_x ? 0 : x + nx;
  if (x >= nx) x = wall_x ? nx - 1 : x - nx;
  if (y < 0) y = wall_y ? 0 : y + ny;
  if (y >= ny) y = wall_y ? ny - 1 : y - ny;
  *xo = x;
  *yo = y;
}

/* Eq. (4): F = -G [beta psi(x) sum_i w psi(x+e_i) e_i
 *                  + (1-beta)/2 sum_i w psi^2(x+e_i) e_i]           */
void lbmref_sc_force_field(int nx, int ny, double G, double beta, int wall_x, int wall_y,
                           const double *psi, const double *psi2, double *Fx, double *Fy) {
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      double s1x = 0.0, s1y = 0.0, s2x = 0.0, s2y = 0.0;
      for (int i = 1; i < 9; ++i) {
        int xn, yn;
        nb(nx, ny, wall_x, wall_y, x + EX[i], y + EY[i], &xn, &yn);
        long k = (long)yn * nx + xn;
        s1x += w_sc(i) * psi[k] * EX[i];
        s1y += w_sc(i) * psi[k] * EY[i];
        s2x += w_sc(i) * psi2[k] * EX[i];
        s2y += w_sc(i) * psi2[k] * EY[i];
      }
      long c = (long)y * nx + x;
      Fx[c] = -G * (beta * psi[c] * s1x + 0.5 * (1.0 - beta) * s2x);
      Fy[c] = -G * (beta * psi[c] * s1y + 0.5 * (1.0 - beta) * s2y);
    }
  }
}

int lbmref_create(const lbmref_params *p, lbmref_handle *out) {
  if (!p || !out) return -1;
  if (p->nx < 1 || p->ny < 1 || !(p->tau_f > 0.5) || !(p->tau_g > 0.5) || !(p->cv > 0.0))
    return -1;
  struct lbmref_ctx *h = (struct lbmref_ctx *)calloc(1, sizeof(*h));
  if (!h) return -2;
  h->p = *p;
  h->n = (long)p->nx * p->ny;
  size_t dist = (size_t)9 * h->n * sizeof(double);
  size_t fld = (size_t)h->n * sizeof(double);
  h->f = (double *)malloc(dist);
  h->g = (double *)malloc(dist);
  h->f2 = (double *)malloc(dist);
  h->g2 = (double *)malloc(dist);
  h->rho = (double *)malloc(fld);
  h->jx = (double *)malloc(fld);
  h->jy = (double *)malloc(fld);
  h->E = (double *)malloc(fld);
  h->T = (double *)malloc(fld);
  h->psi = (double *)malloc(fld);
  h->psi2 = (double *)malloc(fld);
  h->ux = (double *)malloc(fld);
  h->uy = (double *)malloc(fld);
  h->K1 = (double *)malloc(fld);
  h->K2 = (double *)malloc(fld);
  h->Ts = (double *)malloc(fld);
  if (!h->f || !h->g || !h->f2 || !h->g2 || !h->rho || !h->jx || !h->jy || !h->E || !h->T ||
      !h->psi || !h->psi2 || !h->ux || !h->uy || !h->K1 || !h->K2 || !h->Ts) {
    lbmref_destroy(h);
    return -2;
  }
  *out = h;
  return 0;
}

int lbmref_destroy(lbmref_handle h) {
  if (!h) return -1;
  free(h->f);
  free(h->g);
  free(h->f2);
  free(h->g2);
  free(h->rho);
  free(h->jx);
  free(h->jy);
  free(h->E);
  free(h->T);
  free(h->psi);
  free(h->psi2);
  free(h->ux);
  free(h->uy);
  free(h->K1);
  free(h->K2);
  free(h->Ts);
  free(h);
  return 0;
}

int lbmref_init_fields(lbmref_handle h, const double *rho, const double *ux, const double *uy,
                       const double *T) {
  if (!h || !rho || !T) return -1;
  for (long c = 0; c < h->n; ++c) {
    double feq[9];
    double u = ux ? ux[c] : 0.0, v = uy ? uy[c] : 0.0;
    lbmref_feq(rho[c], u, v, feq);
    for (int i = 0; i < 9; ++i) {
      h->f[PL(h, i) + c] = feq[i];
      h->g[PL(h, i) + c] = h->p.cv * T[c] * feq[i];
    }
  }
  h->step = 0;
  h->clamp_count = 0;
  h->have_fields = 1;
  return 0;
}

/* pass 1: moments and pseudopotential of every node; returns clamps */
static long pass_moments(lbmref_handle h) {
  const lbmref_params *p = &h->p;
  long clamps = 0;
#pragma omp parallel for schedule(static) reduction(+ : clamps)
  for (int y = 0; y < p->ny; ++y) {
    for (int x = 0; x < p->nx; ++x) {
      long c = IDX(h, x, y);
      double r = 0.0, mx = 0.0, my = 0.0, e = 0.0;
      for (int i = 0; i < 9; ++i) {
        double fi = h->f[PL(h, i) + c];
        r += fi;
        mx += EX[i] * fi;
        my += EY[i] * fi;
        e += h->g[PL(h, i) + c];
      }
      h->rho[c] = r;
      h->jx[c] = mx;
      h->jy[c] = my;
      h->E[c] = e;
      h->T[c] = e / (r * p->cv);
      if (p->G == 0.0) {
        h->psi2[c] = 0.0;
        h->psi[c] = 0.0;
        continue;
      }
      double Te = p->eos_fixed_T ? p->T_eos : h->T[c];
      double s = 2.0 * (lbmref_pressure(p, r, Te) - r * CS2) / p->G;
      h->psi2[c] = s;
      if (s >= 0.0) {
        h->psi[c] = sqrt(s);
      } else {
        h->psi[c] = 0.0;
        if (p->beta != 0.0) clamps += 1;
      }
    }
  }
  return clamps;
}

/* total force: pseudopotential (Eq. (4)) plus body force */
static void total_force(lbmref_handle h, double *Fx, double *Fy) {
  const lbmref_params *p = &h->p;
  if (p->G != 0.0) {
    lbmref_sc_force_field(p->nx, p->ny, p->G, p->beta, p->wall_x, p->wall_y, h->psi, h->psi2,
                          Fx, Fy);
  } else {
    for (long c = 0; c < h->n; ++c) Fx[c] = Fy[c] = 0.0;
  }
  for (long c = 0; c < h->n; ++c) {
    Fx[c] += h->rho[c] * p->gx;
    Fy[c] += h->rho[c] * p->gy;
  }
}

static double phi_divu_at(lbmref_handle h, const double *T, int x, int y);

/* pass 2: collide (Eq. (1) and Eq. (7) or Eq. (24)) and stream.  With
 * phi_divu the LB g update also takes the source term of Eq. (5), whose
 * paper omits it (Eq. (6)): g_i* += w_i phi div u (dt = 1), the velocity
 * of time t; its divergence needs every node's velocity first. */
static void pass_collide_stream(lbmref_handle h, const double *Fx, const double *Fy,
                                int treatment) {
  const lbmref_params *p = &h->p;
  const int nx = p->nx, ny = p->ny;
  const int src = p->phi_divu && treatment != LBMREF_FD_RK2;
  if (src) {
    for (long c = 0; c < h->n; ++c) {
      h->ux[c] = (h->jx[c] + 0.5 * Fx[c]) / h->rho[c];
      h->uy[c] = (h->jy[c] + 0.5 * Fy[c]) / h->rho[c];
    }
  }
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      long c = IDX(h, x, y);
      double r = h->rho[c];
      double ux = (h->jx[c] + 0.5 * Fx[c]) / r;
      double uy = (h->jy[c] + 0.5 * Fy[c]) / r;
      if (!src) {
        h->ux[c] = ux;
        h->uy[c] = uy;
      }
      const double S = src ? phi_divu_at(h, h->T, x, y) : 0.0;
      double cvT = p->cv * h->T[c];
      double feq[9], fi_force[9], ci[9];
      lbmref_feq(r, ux, uy, feq);
      lbmref_guo(p->tau_f, ux, uy, Fx[c], Fy[c], fi_force);
      lbmref_corr(p->tau_g, cvT, Fx[c], Fy[c], ci);
      for (int i = 0; i < 9; ++i) {
        double fi = h->f[PL(h, i) + c];
        double gi = h->g[PL(h, i) + c];
        double fs = fi - (fi - feq[i]) / p->tau_f + fi_force[i];
        double geq = cvT * feq[i];
        double gs = gi - (gi - geq) / p->tau_g;
        if (treatment == LBMREF_CORRECTED) gs += ci[i];
        if (src) gs += W[i] * S;

        int xn = x + EX[i], yn = y + EY[i];
        int out_x = (xn < 0 || xn >= nx), out_y = (yn < 0 || yn >= ny);
        int hit_y = out_y && p->wall_y, hit_x = out_x && p->wall_x;
        int open = p->wall_x == 2;
        if (open && hit_x && !hit_y) {
          int o = opposite(i);
          if (xn >= nx) { /* outlet */
            double eu = EX[i] * ux + EY[i] * uy;
            double even = 1.0 + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy);
            h->f2[PL(h, o) + c] = -fs + 2.0 * W[i] * p->rho_out * even;
            h->g2[PL(h, o) + c] = -gs + 2.0 * W[i] * cvT * r * even;
            continue;
          }
          double eu = EX[i] * p->u_in; /* inlet */
          h->f2[PL(h, o) + c] = fs - 2.0 * W[i] * r * eu / CS2;
          if (p->thermal_left == LBMREF_THERMAL_DIRICHLET)
            h->g2[PL(h, o) + c] = -gs + 2.0 * W[i] * p->cv * r * p->T_left *
                                            (1.0 + 4.5 * eu * eu - 1.5 * p->u_in * p->u_in);
          else
            h->g2[PL(h, o) + c] = gs;
          continue;
        }
        if (hit_y || hit_x) {
          int o = opposite(i);
          /* at a corner of the open channel the plate's condition applies */
          int sx = hit_x && !open ? (xn < 0 ? 0 : 1) : -1;
          int sy = hit_y ? (yn < 0 ? 2 : 3) : -1;
          double Tw;
          int thermal = wall_condition(p, sx, sy, &Tw);
          h->f2[PL(h, o) + c] = fs;
          if (thermal == LBMREF_THERMAL_DIRICHLET)
            h->g2[PL(h, o) + c] = -gs + 2.0 * W[i] * p->cv * r * Tw;
          else
            h->g2[PL(h, o) + c] = gs;
        } else {
          if (xn < 0) xn += nx;
          if (xn >= nx) xn -= nx;
          if (yn < 0) yn += ny;
          if (yn >= ny) yn -= ny;
          long d = IDX(h, xn, yn);
          h->f2[PL(h, i) + d] = fs;
          h->g2[PL(h, i) + d] = gs;
        }
      }
    }
  }
}

/* value of a node field at (x, y), which may lie one node beyond a wall:
 * periodic wrap, or the mirrored boundary node; `dirichlet` gives the
 * temperature ghost 2 T_w - T(mirrored node) instead */
static double ghost(lbmref_handle h, const double *phi, int x, int y, int is_T) {
  const lbmref_params *p = &h->p;
  const int nx = p->nx, ny = p->ny;
  int xm = x, ym = y;
  int outx = x < 0 || x >= nx, outy = y < 0 || y >= ny;
  if (outx) xm = p->wall_x ? (x < 0 ? 0 : nx - 1) : (x < 0 ? x + nx : x - nx);
  if (outy) ym = p->wall_y ? (y < 0 ? 0 : ny - 1) : (y < 0 ? y + ny : y - ny);
  double v = phi[IDX(h, xm, ym)];
  if (!is_T) return v;
  int sx = outx && p->wall_x ? (x < 0 ? 0 : 1) : -1;
  int sy = outy && p->wall_y ? (y < 0 ? 2 : 3) : -1;
  if (p->wall_x == 2 && sy >= 0) sx = -1; /* open channel: the plate's condition at corners */
  if (sx < 0 && sy < 0) return v;
  double Tw;
  int th = wall_condition(p, sx, sy, &Tw);
  return th == LBMREF_THERMAL_DIRICHLET ? 2.0 * Tw - v : v;
}

/* (dp_EOS/dT) at fixed rho: Carnahan-Starling rho R Z(eta), ideal rho R */
static double dp_dT(const lbmref_params *p, double rho) {
  if (p->eos == LBMREF_EOS_IDEAL) return rho * p->R;
  double eta = p->b * rho / 4.0;
  double num = 1.0 + eta + eta * eta - eta * eta * eta;
  double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
  return rho * p->R * num / den;
}

/* velocity component at (x, y) one node beyond the lattice at most:
 * periodic wrap, or the boundary node's value reversed beyond a wall */
static double u_ghost(lbmref_handle h, const double *u, int x, int y) {
  const lbmref_params *p = &h->p;
  int outx = x < 0 || x >= p->nx, outy = y < 0 || y >= p->ny;
  double v = ghost(h, u, x, y, 0);
  if ((outx && p->wall_x) || (outy && p->wall_y)) v = -v;
  return v;
}

/* phi div u of Eq. (5) at node (x, y): phi = -T (dp_EOS/dT)_rho with the
 * node's T and rho, div u by the isotropic central difference
 * sum_i w(|e_i|^2) u(x + e_i) . e_i of the velocities in h->ux, h->uy */
static double phi_divu_at(lbmref_handle h, const double *T, int x, int y) {
  const lbmref_params *p = &h->p;
  long c = IDX(h, x, y);
  double du = 0.0;
  for (int i = 1; i < 9; ++i) {
    double w = w_sc(i);
    du += w * (u_ghost(h, h->ux, x + EX[i], y + EY[i]) * EX[i] +
               u_ghost(h, h->uy, x + EX[i], y + EY[i]) * EY[i]);
  }
  double phi = -T[c] * dp_dT(p, h->rho[c]);
  return phi * du;
}

/* K(T) of Eq. (26) at every node, with u and rho of time t */
static void fd_rhs(lbmref_handle h, const double *T, double *K) {
  const lbmref_params *p = &h->p;
  const double lam_per_rho = (p->tau_g - 0.5) * p->cv * CS2;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p->ny; ++y) {
    for (int x = 0; x < p->nx; ++x) {
      long c = IDX(h, x, y);
      double gTx = 0.0, gTy = 0.0, gLx = 0.0, gLy = 0.0, lapT = 0.0;
      for (int i = 1; i < 9; ++i) {
        double w = w_sc(i);
        double Tn = ghost(h, T, x + EX[i], y + EY[i], 1);
        double rn = ghost(h, h->rho, x + EX[i], y + EY[i], 0);
        gTx += w * Tn * EX[i];
        gTy += w * Tn * EY[i];
        gLx += w * lam_per_rho * rn * EX[i];
        gLy += w * lam_per_rho * rn * EY[i];
        lapT += 2.0 * w * (Tn - T[c]);
      }
      double lam = lam_per_rho * h->rho[c];
      double div = lam * lapT + gLx * gTx + gLy * gTy;
      K[c] = -(h->ux[c] * gTx + h->uy[c] * gTy) + div / (h->rho[c] * p->cv);
      if (p->phi_divu) K[c] += phi_divu_at(h, T, x, y) / (h->rho[c] * p->cv);
    }
  }
}

/* Eq. (27), read as Heun's method (dt = 1), then g = cv T f on the
 * streamed f */
static void fd_update(lbmref_handle h) {
  const long n = h->n;
  fd_rhs(h, h->T, h->K1);
  for (long c = 0; c < n; ++c) h->Ts[c] = h->T[c] + h->K1[c];
  fd_rhs(h, h->Ts, h->K2);
  for (long c = 0; c < n; ++c) {
    double Tn = h->T[c] + 0.5 * (h->K1[c] + h->K2[c]);
    for (int i = 0; i < 9; ++i) h->g2[PL(h, i) + c] = h->p.cv * Tn * h->f2[PL(h, i) + c];
  }
}

int lbmref_step(lbmref_handle h, int n, int treatment) {
  if (!h || n < 0) return -1;
  if (treatment != LBMREF_PLAIN && treatment != LBMREF_CORRECTED && treatment != LBMREF_FD_RK2)
    return -1;
  if (!h->have_fields) return -6;
  double *Fx = (double *)malloc((size_t)h->n * sizeof(double));
  double *Fy = (double *)malloc((size_t)h->n * sizeof(double));
  if (!Fx || !Fy) {
    free(Fx);
    free(Fy);
    return -2;
  }
  int status = 0;
  for (int s = 0; s < n; ++s) {
    long clamps = pass_moments(h);
    h->clamp_count += clamps;
    total_force(h, Fx, Fy);
    pass_collide_stream(h, Fx, Fy, treatment);
    if (treatment == LBMREF_FD_RK2) fd_update(h);
    double *t;
    t = h->f; h->f = h->f2; h->f2 = t;
    t = h->g; h->g = h->g2; h->g2 = t;
    h->step += 1;
    if (clamps > 0 && h->p.psi_policy == 1) {
      status = -5;
      break;
    }
  }
  free(Fx);
  free(Fy);
  return status;
}

int lbmref_force(lbmref_handle h, double *Fx, double *Fy) {
  if (!h || !h->have_fields) return -1;
  pass_moments(h);
  total_force(h, Fx, Fy);
  return 0;
}

int lbmref_psi(lbmref_handle h, double *psi, double *psi2) {
  if (!h || !h->have_fields) return -1;
  pass_moments(h);
  memcpy(psi, h->psi, (size_t)h->n * sizeof(double));
  memcpy(psi2, h->psi2, (size_t)h->n * sizeof(double));
  return 0;
}

int lbmref_moments(lbmref_handle h, double *rho, double *ux, double *uy, double *T) {
  if (!h || !h->have_fields) return -6;
  double *Fx = (double *)malloc((size_t)h->n * sizeof(double));
  double *Fy = (double *)malloc((size_t)h->n * sizeof(double));
  if (!Fx || !Fy) {
    free(Fx);
    free(Fy);
    return -2;
  }
  pass_moments(h);
  total_force(h, Fx, Fy);
  for (long c = 0; c < h->n; ++c) {
    if (rho) rho[c] = h->rho[c];
    if (ux) ux[c] = (h->jx[c] + 0.5 * Fx[c]) / h->rho[c];
    if (uy) uy[c] = (h->jy[c] + 0.5 * Fy[c]) / h->rho[c];
    if (T) T[c] = h->T[c];
  }
  free(Fx);
  free(Fy);
  return 0;
}

int lbmref_totals(lbmref_handle h, double out[8]) {
  if (!h || !h->have_fields) return -6;
  double *Fx = (double *)malloc((size_t)h->n * sizeof(double));
  double *Fy = (double *)malloc((size_t)h->n * sizeof(double));
  if (!Fx || !Fy) {
    free(Fx);
    free(Fy);
    return -2;
  }
  pass_moments(h);
  total_force(h, Fx, Fy);
  double m = 0.0, e = 0.0, px = 0.0, py = 0.0, bad = 0.0;
  for (long c = 0; c < h->n; ++c) {
    m += h->rho[c];
    e += h->E[c];
    px += h->jx[c] + 0.5 * Fx[c];
    py += h->jy[c] + 0.5 * Fy[c];
    if (!isfinite(h->rho[c]) || !isfinite(h->E[c])) bad += 1.0;
  }
  out[0] = m;
  out[1] = e;
  out[2] = px;
  out[3] = py;
  out[4] = bad;
  out[5] = (double)h->clamp_count;
  out[6] = (double)h->step;
  out[7] = 0.0;
  free(Fx);
  free(Fy);
  return 0;
}

int lbmref_get_state(lbmref_handle h, double *f, double *g) {
  if (!h || !h->have_fields) return -6;
  memcpy(f, h->f, (size_t)9 * h->n * sizeof(double));
  memcpy(g, h->g, (size_t)9 * h->n * sizeof(double));
  return 0;
}

int lbmref_set_state(lbmref_handle h, const double *f, const double *g) {
  if (!h) return -1;
  memcpy(h->f, f, (size_t)9 * h->n * sizeof(double));
  memcpy(h->g, g, (size_t)9 * h->n * sizeof(double));
  h->have_fields = 1;
  return 0;
}
