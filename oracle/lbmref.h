/*
 * lbmref.h -- plain CPU FP64 oracle of the double-distribution-function
 * pseudopotential thermal lattice Boltzmann step of Li & Luo,
 * "Effect of the forcing term in the pseudopotential lattice Boltzmann
 * modeling of thermal flows" (arXiv:1405.2232).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or helper with the HIP
 * library; its parameter struct is its own.
 *
 * Host arrays are row-major [ny][nx] (x fastest), FP64.
 * Distribution arrays are [9][ny][nx].
 */
#ifndef LBMREF_H
#define LBMREF_H

#ifdef __cplusplus
extern "C" {
#endif

enum { LBMREF_PLAIN = 0, LBMREF_CORRECTED = 1, LBMREF_FD_RK2 = 2 };
enum { LBMREF_EOS_CS = 0, LBMREF_EOS_IDEAL = 1 };
enum { LBMREF_THERMAL_DIRICHLET = 0, LBMREF_THERMAL_ADIABATIC = 1 };

typedef struct {
  int nx, ny;
  double tau_f, tau_g;      /* relaxation times of Eq. (1) and Eq. (7) */
  double G;                 /* interaction strength of Eqs. (2)-(4) */
  double beta;              /* mixing weight of Eq. (4); 1 gives Eq. (2) */
  int eos;                  /* LBMREF_EOS_* */
  double a, b, R;           /* EOS constants */
  int eos_fixed_T;          /* 1: EOS evaluated at T_eos instead of local T */
  double T_eos;
  double cv;                /* specific heat in g^eq = cv T f^eq */
  double gx, gy;            /* body acceleration: force rho*(gx, gy) */
  int wall_x, wall_y;       /* 0 periodic, 1 halfway bounce-back walls;
                               wall_x = 2: open, inlet on the left (velocity
                               (u_in, 0), temperature T_left), outlet on the
                               right (density rho_out, zero gradient of u
                               and T) */
  int thermal_left, thermal_right, thermal_bottom, thermal_top; /* LBMREF_THERMAL_* */
  double T_left, T_right, T_bottom, T_top;  /* Dirichlet wall temperatures */
  int psi_policy;           /* 0 clamp psi to 0 and count, 1 also flag an error */
  double u_in;              /* inlet velocity (wall_x = 2) */
  double rho_out;           /* outlet density (wall_x = 2) */
  int phi_divu;             /* 1: keep the phi div u term of Eq. (5): in K(T)
                               for the finite-difference treatment, as the
                               source w_i phi div u of g_i* for the LB ones */
} lbmref_params;

typedef struct lbmref_ctx *lbmref_handle;

int lbmref_create(const lbmref_params *p, lbmref_handle *out);
int lbmref_destroy(lbmref_handle h);
int lbmref_init_fields(lbmref_handle h, const double *rho, const double *ux,
                       const double *uy, const double *T);
int lbmref_step(lbmref_handle h, int n, int treatment);
int lbmref_moments(lbmref_handle h, double *rho, double *ux, double *uy, double *T);
/* out: mass, energy, px, py, nonfinite_count, clamp_count, step, 0 */
int lbmref_totals(lbmref_handle h, double out[8]);
int lbmref_get_state(lbmref_handle h, double *f, double *g);
int lbmref_set_state(lbmref_handle h, const double *f, const double *g);
/* total force (pseudopotential + body) at the current state */
int lbmref_force(lbmref_handle h, double *Fx, double *Fy);
int lbmref_psi(lbmref_handle h, double *psi, double *psi2);

/* single-node pieces, exposed for the closed-form checks */
void lbmref_velocities(int *ex, int *ey, double *w);
void lbmref_feq(double rho, double ux, double uy, double out[9]);
void lbmref_guo(double tau_f, double ux, double uy, double Fx, double Fy, double out[9]);
void lbmref_corr(double tau_g, double cvT, double Fx, double Fy, double out[9]);
double lbmref_pressure(const lbmref_params *p, double rho, double T);
/* pseudopotential force of Eq. (4) from given psi and psi^2 fields */
void lbmref_sc_force_field(int nx, int ny, double G, double beta, int wall_x, int wall_y,
                           const double *psi, const double *psi2, double *Fx, double *Fy);

#ifdef __cplusplus
}
#endif
#endif
