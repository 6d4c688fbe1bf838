/*
 * lbm.h -- C ABI of the MI355X (gfx950) implementation of the
 * double-distribution-function pseudopotential thermal lattice Boltzmann
 * step of Li & Luo, "Effect of the forcing term in the pseudopotential
 * lattice Boltzmann modeling of thermal flows" (arXiv:1405.2232).
 *
 * One time step (lbm_step) on a D2Q9 lattice of nx * ny nodes is:
 *   - moments rho = sum f_i, j = sum e_i f_i, rho cv T = sum g_i;
 *   - pseudopotential psi = sqrt(2 (p_EOS - rho c_s^2)/(G c^2))
 *     (Section II.A) for the node and its eight neighbours;
 *   - the pseudopotential force of Eq. (2), or its mixed form Eq. (4),
 *     plus a body force rho (gx, gy) (the buoyancy of Section III.B);
 *   - BGK collision of f with the forcing term F_i, Eq. (1), with the
 *     velocity u = (j + F/2)/rho;
 *   - BGK collision of g with g^eq = cv T f^eq, Eq. (7) (LBM_PLAIN), or
 *     the corrected Eq. (24) with the correction term C_i of Eq. (25)
 *     (LBM_CORRECTED);
 *   - streaming, with periodic wrap or halfway bounce-back walls.
 *
 * Conventions
 *   - Host arrays are FP64, row-major [ny][nx] with x fastest.
 *   - Device memory is owned by the caller: lbm_workspace_bytes() says how
 *     much, lbm_create() borrows it (it must outlive lbm_destroy()).  The
 *     library allocates no device memory of its own.
 *   - All device work is enqueued on the HIP stream given to lbm_create()
 *     (a hipStream_t passed as void*; NULL is the null stream).
 *   - Every function returns an int status (LBM_OK or a negative code);
 *     no C++ exception crosses this boundary.  Asynchronous device faults
 *     surface as LBM_EDEVICE from the next call that synchronizes.
 *   - Calls on one handle must not overlap (not thread-safe per handle).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* bad argument or parameter */
  LBM_ENOMEM = -2,     /* workspace too small */
  LBM_EDEVICE = -3,    /* HIP runtime error */
  LBM_ENONFINITE = -4, /* a density or energy became NaN/Inf */
  LBM_EDOMAIN = -5,    /* psi^2 < 0 met under the strict psi policy */
  LBM_ESTATE = -6      /* call out of order (e.g. step before init) */
};

/* temperature treatments */
enum {
  LBM_PLAIN = 0,     /* Eq. (7): carries the forcing-term effect of Eq. (23) */
  LBM_CORRECTED = 1, /* Eq. (24) with C_i of Eq. (25): recovers Eq. (A11) */
  LBM_FD_RK2 = 2     /* Eq. (26) by isotropic central differences and the
                        two-stage Runge-Kutta scheme of Eq. (27) (Heun's
                        form), u and rho of time t in both stages; the
                        temperature is then carried as g_i = cv T f_i.
                        Single lattices only (lbm_batch_step rejects it). */
};

/* storage precision of the distributions */
enum {
  LBM_FP64 = 0,      /* f_i, g_i stored and updated in FP64 */
  LBM_FP32_DEV = 1,  /* stored in FP32 as deviations f_i - w_i rho_ref and
                        g_i - w_i rho_ref cv T_ref (global shifts); the
                        collision runs in FP32; moments, EOS, psi, force and
                        reductions in FP64 */
  LBM_FP32_LOCAL = 2 /* as LBM_FP32_DEV, but the density shift is per node:
                        f_i - w_i rho_bar(x), g_i - w_i rho_bar(x) cv T_ref,
                        rho_bar(x) the node's density one step earlier
                        rounded to FP16 and stored beside the distributions
                        (2 more bytes per node and copy) */
};

enum { LBM_EOS_CS = 0, LBM_EOS_IDEAL = 1 };
enum { LBM_THERMAL_DIRICHLET = 0, LBM_THERMAL_ADIABATIC = 1 };

typedef struct {
  int nx, ny;           /* lattice nodes; 1 <= nx, ny; nx*ny < 2^31, and
                           one copy of the 18 distributions below 4 GiB
                           (about 5,400^2 nodes in FP64, 7,600^2 in
                           FP32) */
  double tau_f, tau_g;  /* relaxation times of Eq. (1) and Eq. (7); > 0.5 */
  double G;             /* interaction strength of Eq. (2); 0 disables it */
  double beta;          /* Eq. (4) mixing weight; 1 gives Eq. (2) */
  int eos;              /* LBM_EOS_CS: Carnahan-Starling,
                           p = rho R T (1+e+e^2-e^3)/(1-e)^3 - a rho^2,
                           e = b rho/4; LBM_EOS_IDEAL: p = rho R T
                           (the EOS of Section III) */
  double a, b, R;       /* EOS constants */
  int eos_fixed_T;      /* 0: EOS at the local T (coupled); 1: at T_eos */
  double T_eos;
  double cv;            /* specific heat in g^eq = cv T f^eq; > 0 */
  double gx, gy;        /* body acceleration; force rho * (gx, gy) */
  int wall_x, wall_y;   /* 0: periodic; 1: walls halfway outside the
                           first and last node (f bounces back; the psi
                           ghost mirrors the boundary node).  wall_x = 2:
                           open channel (Sec. III.A states only uniform
                           inflow and fully developed outflow): inlet
                           halfway left of the first column (f bounces
                           back with the momentum of (u_in, 0); g
                           anti-bounces back with the inlet equilibrium's
                           even part at T_left, or bounces back when the
                           left side is adiabatic), outlet halfway right of
                           the last column (anti-bounce-back holding
                           rho_out with the node's own velocity and
                           energy) */
  int thermal_left, thermal_right, thermal_bottom, thermal_top;
                        /* LBM_THERMAL_DIRICHLET: g anti-bounces back
                           with the wall value rho cv T_w; ADIABATIC: g
                           bounces back.  Where a diagonal leaves through
                           a corner of a box (wall_x = 1) it meets both
                           walls: adiabatic if either is, else Dirichlet
                           at the mean of the two wall temperatures (the
                           scheme stays covariant under exchanging x and
                           y); at a corner of the open channel the plate's
                           condition applies. */
  double T_left, T_right, T_bottom, T_top;
  int psi_policy;       /* 0: psi^2 < 0 clamps psi to 0 and is counted;
                           1: the same, and lbm_sync()/lbm_moments()
                           return LBM_EDOMAIN once any clamp happened */
  int precision;        /* LBM_FP64, LBM_FP32_DEV or LBM_FP32_LOCAL */
  double rho_ref, T_ref;/* deviation shifts: rho_ref for LBM_FP32_DEV,
                           T_ref for both FP32 forms */
  double u_in, rho_out; /* open channel (wall_x = 2): inlet velocity and
                           outlet density (> 0) */
  int phi_divu;         /* 1: keep the term phi div u of Eq. (5),
                           phi = -T (dp_EOS/dT)_rho, which the paper's
                           Eq. (6) drops: LBM_FD_RK2 adds it to K(T); the LB
                           treatments add the source w_i phi div u to the
                           post-collision g_i (u of time t, div u by the
                           isotropic central difference).  Such lattices
                           step one step per launch and cannot join a
                           batch.  0 or 1. */
} lbm_params;

typedef struct lbm_ctx *lbm_handle;

/* Device bytes lbm_create() needs for these parameters. */
int lbm_workspace_bytes(const lbm_params *p, size_t *bytes);

/* Validate p and bind a caller-owned device workspace of `bytes` bytes
 * (256-byte aligned) and a HIP stream.  No kernel runs here. */
int lbm_create(const lbm_params *p, void *dev_workspace, size_t bytes, void *hip_stream,
               lbm_handle *out);

/* Initialise f_i = f_i^eq(rho, u) and g_i = cv T f_i^eq(rho, u) from host
 * arrays (ux, uy may be NULL for zero).  Copies are stream-ordered; the
 * call returns once the host arrays may be reused. */
int lbm_init_fields(lbm_handle h, const double *rho, const double *ux, const double *uy,
                    const double *T);

/* The same, with the stored momentum j = rho u - F/2 (f_i = f_i^eq(rho,
 * u - F/(2 rho)), g_i = cv T f_i), F the total force (Eq. (2) or (4) plus
 * the body force) of the given rho and T: with the forcing of Eq. (1)
 * (Sec. II) the velocity is (j + F/2)/rho, so the velocity lbm_moments
 * reports for this state is the given u (to rounding).  A state at rest
 * with a density interface holds j = -F/2 at steady state; starting there
 * shortens the solve to steady state.  Uses the second distribution
 * buffer as scratch before the first step.  Same arguments and errors as
 * lbm_init_fields, plus LBM_EDEVICE if a kernel launch fails (the handle
 * is then uninitialised). */
int lbm_init_fields_physical(lbm_handle h, const double *rho, const double *ux, const double *uy,
                             const double *T);

/* Enqueue n >= 1 time steps with the given treatment (it may change from
 * call to call).  Does not synchronize unless a check interval is set
 * (lbm_set_check_interval), in which case the status of the last check
 * is returned. */
int lbm_step(lbm_handle h, int n, int treatment);

/* Check non-finite moments and the psi policy every k steps inside
 * lbm_step (k = 0, the default, checks only in lbm_sync / lbm_moments /
 * lbm_totals). */
int lbm_set_check_interval(lbm_handle h, int k);

/* Synchronize the stream and report LBM_ENONFINITE / LBM_EDOMAIN /
 * LBM_EDEVICE. */
int lbm_sync(lbm_handle h);

/* rho, u = (j + F/2)/rho and T at the current time, to host arrays (any
 * may be NULL).  Synchronizes. */
int lbm_moments(lbm_handle h, double *rho, double *ux, double *uy, double *T);

/* The same fields written to caller-owned device arrays of nx*ny doubles
 * (any may be NULL).  Stream-ordered; does not synchronize. */
int lbm_moments_device(lbm_handle h, double *d_rho, double *d_ux, double *d_uy, double *d_T);

/* FP64 totals at the current time: out[0] mass sum rho, out[1] energy
 * sum rho cv T, out[2..3] momentum sum (j + F/2), out[4] number of nodes
 * with non-finite rho or energy, out[5] psi clamps so far, out[6] steps
 * taken, out[7] 0.  Synchronizes. */
int lbm_totals(lbm_handle h, double out[8]);

/* lbm_totals for callers that cannot allocate device memory around the
 * call (code under stream capture, tight serving loops, harnesses that
 * forbid allocation).  The same totals, bit for bit, from the same kernels;
 * their scratch memory (per-block FP64 partial sums and the reduced
 * totals) lives in a static device array of the library, 2.6 MB on each
 * GPU the library runs on, held until the process ends, instead of in the
 * handle's workspace.  A lattice whose moments launch needs more than
 * 32768 blocks (beyond about 5,800^2 nodes) gives LBM_EINVAL; an
 * uninitialised handle LBM_ESTATE.  Every call on one GPU uses that GPU's
 * one array: calls that overlap on one GPU (from other threads, on other
 * streams) race, and the caller must serialize them.  Synchronizes the
 * handle's stream. */
int lbm_totals_noalloc(lbm_handle h, double out[8]);

/* Relative change of rho and T over one step,
 * max over {rho, T} of ||phi^n - phi^(n-1)||_inf / ||phi^n||_inf.
 * Takes one step with `treatment`.  Synchronizes. */
int lbm_step_residual(lbm_handle h, int treatment, double *residual);

/* Raw state, 18 planes [q][ny][nx] (q < 9: f, else g) in FP64 on the host,
 * deviations added back for LBM_FP32_DEV.  Synchronizes. */
int lbm_get_state(lbm_handle h, double *state);
int lbm_set_state(lbm_handle h, const double *state);

/* Checkpoint: write the stored state (raw bytes, any precision), the step
 * count and the clamp count to `path`, with what defines the stored form
 * (sizes, storage precision and layout, and the deviation shifts rho_ref
 * and cv T_ref); lbm_load restores it into a handle created with the same
 * parameters, so that a resumed run is bitwise equal to an uninterrupted
 * one.  LBM_EINVAL on I/O errors or any mismatch of that form, before
 * anything is copied to the device. */
int lbm_save(lbm_handle h, const char *path);
int lbm_load(lbm_handle h, const char *path);

/* Tile shape of the step kernel: bx columns per block (64, 128, 256 or 512)
 * and `rows` rows per block (>= 1).  The default comes from the lattice
 * size; an autotuner may pick another.  Results do not depend on it. */
int lbm_set_tiling(lbm_handle h, int bx, int rows);

/* Two steps per kernel launch (temporal blocking).  Where the lattice
 * allows it (any storage form and force, periodic in x) lbm_step advances the plain and corrected treatments
 * two steps per launch: the distributions of the intermediate time level
 * stay on chip, which halves the HBM traffic per step.  The arithmetic of
 * each step is the one-step kernel's.  `on` = 0 makes every step a
 * one-step launch; `rows` (> 0) sets the rows per block of the two-step
 * kernel, 0 keeps the current value.  Default: on for lattices large
 * enough to fill the device (small ones are bound by latency, where
 * one-step launches are faster), with the rows chosen from the lattice size
 * and the device's compute units.  A step that
 * ends at a periodic check is always a one-step launch.
 * lbm_get_step_pairing reports whether lbm_step will pair steps (`active`)
 * and the rows per block.  LBM_EINVAL for a NULL handle or rows < 0. */
int lbm_set_step_pairing(lbm_handle h, int on, int rows);
int lbm_get_step_pairing(lbm_handle h, int *active, int *rows);
int lbm_get_tiling(lbm_handle h, int *bx, int *rows);

int lbm_destroy(lbm_handle h);
const char *lbm_strerror(int status);

/* ------------------------------------------------------------------------
 * Batches: many independent lattices (sizes and parameters may differ, the
 * storage precision may not) stepped together, one kernel launch per step
 * covering every tile of every lattice, optionally replayed from captured
 * hipGraphs.  Each lattice keeps a single-lattice handle (lbm_batch_lattice)
 * for initialisation, moments, totals, residuals and checkpoints.  The step
 * is the same as lbm_step's, node for node, so a lattice advanced in a batch
 * is bitwise equal to the same lattice advanced alone (also where either
 * pairs steps).
 * ---------------------------------------------------------------------- */
typedef struct lbm_batch_ctx *lbm_batch_handle;

/* Device bytes for a batch of `count` lattices with parameters p[0..count). */
int lbm_batch_workspace_bytes(int count, const lbm_params *p, size_t *bytes);

/* Bind a caller-owned workspace and stream; all p[i].precision must agree
 * and no lattice may be an open channel (wall_x = 2) or keep the phi div u
 * source (phi_divu = 1).  Uploads the lattice
 * tables (synchronous). */
int lbm_batch_create(int count, const lbm_params *p, void *dev_workspace, size_t bytes,
                     void *hip_stream, lbm_batch_handle *out);

/* Single-lattice handle of lattice i (owned by the batch: do not destroy). */
int lbm_batch_lattice(lbm_batch_handle b, int i, lbm_handle *out);

/* lbm_init_fields / lbm_moments of lattice i. */
int lbm_batch_init_fields(lbm_batch_handle b, int i, const double *rho, const double *ux,
                          const double *uy, const double *T);
int lbm_batch_moments(lbm_batch_handle b, int i, double *rho, double *ux, double *uy,
                      double *T);
/* lbm_init_fields_physical of lattice i. */
int lbm_batch_init_fields_physical(lbm_batch_handle b, int i, const double *rho, const double *ux,
                                   const double *uy, const double *T);

/* Enqueue n >= 1 steps of every active lattice (all must be initialised). */
int lbm_batch_step(lbm_batch_handle b, int n, int treatment);

/* lbm_step_residual of every active lattice at once: one step of the
 * batch between two moment passes, one wait.  residuals[i] and status[i]
 * (count entries, caller-owned host arrays) get lattice i's residual and
 * the status its lbm_step_residual would return (LBM_ENONFINITE,
 * LBM_EDOMAIN or LBM_OK); an inactive lattice gets -1 and LBM_OK.  The
 * return value is LBM_OK, or the error of a failed call (LBM_EINVAL,
 * LBM_ESTATE for an uninitialised active lattice, LBM_EDEVICE). */
int lbm_batch_step_residuals(lbm_batch_handle b, int treatment, double *residuals, int *status);

/* Which lattices the next steps advance (active[i] != 0); NULL = all.  A
 * changed mask rebuilds the tile lists and drops the captured graphs; an
 * unchanged one keeps both. */
int lbm_batch_set_active(lbm_batch_handle b, const int *active);

/* Tile shape shared by the batch (bx in 64/128/256 lanes, rows >= 1). */
int lbm_batch_set_tiling(lbm_batch_handle b, int bx, int rows);
int lbm_batch_get_tiling(lbm_batch_handle b, int *bx, int *rows);

/* Two steps per launch for the batch (see lbm_set_step_pairing): used when
 * every lattice of the batch admits it, for the plain and corrected
 * treatments; then each launch advances every active lattice two steps
 * (one step for the last of an odd count).  `rows` (> 0) sets the band
 * height of the two-step tiles, 0 keeps it.  Default: on when the batch
 * fills the device, with the band height chosen from the lattice sizes and
 * the device's compute units.
 * lbm_batch_get_step_pairing reports whether lbm_batch_step pairs steps. */
int lbm_batch_set_step_pairing(lbm_batch_handle b, int on, int rows);
int lbm_batch_get_step_pairing(lbm_batch_handle b, int *active, int *rows);

/* k = 0: eager launches.  k even >= 2: lbm_batch_step replays a hipGraph
 * holding k launches (k steps, or 2k with two steps per launch; captured
 * on first use, recaptured when the tiling, the pairing or the active set
 * changes) for every whole group. */
int lbm_batch_use_graph(lbm_batch_handle b, int k);

/* Synchronize and check every lattice (first failing status). */
int lbm_batch_sync(lbm_batch_handle b);

int lbm_batch_destroy(lbm_batch_handle b);

/* Measurement aid: copy `bytes` (multiple of 16) from src to dst with a
 * plain streaming kernel on `hip_stream`; gives the practical HBM
 * bandwidth ceiling and the copy used to scale byte counters. */
int lbm_copy_probe(void *dst, const void *src, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
