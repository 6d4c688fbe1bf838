// Internal device-side interface of liblbm (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmdev {

// How the 18 distributions of a node are stored.
enum Storage {
  ST_F64 = 0,        // FP64 values
  ST_F32_GLOBAL = 1, // FP32 deviations from w_i rho_ref (g: w_i rho_ref cv T_ref)
  ST_F32_LOCAL = 2   // FP32 deviations from w_i rho_bar, rho_bar a per-node FP16
                     // density reference stored after the 18 planes
};

// Per-lattice constants of the model (Section II), pre-derived on the host.
struct Model {
  int nx, ny;
  int pitch;                 // elements between rows of one plane
  long long plane;           // elements between planes
  long long ref_off;         // bytes from a buffer to its FP16 reference plane
  long long ref_bytes;       // bytes of that plane
  int rpitch;                // elements between rows of the reference plane
  double inv_tau_f, inv_tau_g;
  double kf, kg;             // 1 - 1/(2 tau_f), 1 - 1/(2 tau_g)
  double G, beta;
  double two_over_G;         // 2/(G c^2) with c = 1
  int sc_on;                 // G != 0
  int beta_one;              // beta == 1: Eq. (2) only
  int count_clamps;          // beta != 0 (a real psi is needed)
  int eos;                   // 0 Carnahan-Starling, 1 ideal
  int eos_fixed_T;
  double a, b, R, T_eos;
  double cv, inv_cv;
  double gx, gy;
  int wall_x, wall_y;        // wall_x: 0 periodic, 1 walls, 2 inlet (left) / outlet (right)
  int thermal[4];            // left, right, bottom, top: 0 Dirichlet, 1 adiabatic
  double wall_E[4];          // cv * T_w per wall (multiplied by the node's rho)
  double rho_ref;            // ST_F32_GLOBAL density shift
  double cvT_ref;            // cv * T_ref: energy shift per unit reference density
  double lam_per_rho;        // (tau_g - 1/2) cv c_s^2: conductivity over density
  double u_in, rho_out;      // open channel (wall_x == 2): inlet velocity, outlet density
  int phi_divu;              // finite-difference treatment keeps phi div u (Eq. (5))
  double T_wall[4];          // wall temperatures (finite-difference treatment)
};

// What one launch of the tile kernel does.
// MODE_STEP_OPEN is MODE_STEP with the inlet/outlet code of the open
// channel compiled in (kept out of the other lattices' kernels, where its
// extra live values would push the row buffers into scratch memory)
// MODE_STEP_SRC is MODE_STEP with the source term phi div u of Eq. (5) in
// the g update, from velocity planes of time t passed in MomentsOut::ux, uy
// MODE_STEP_FD is the f half of MODE_STEP for the finite-difference
// treatment: it also writes rho, u and T of time t (the moments a
// MODE_MOMENTS launch would write) to MomentsOut::rho, ux, uy, T and
// stores no g, which the finite-difference update then writes whole
enum Mode { MODE_STEP = 0, MODE_MOMENTS = 1, MODE_STEP_OPEN = 2, MODE_STEP_SRC = 3, MODE_STEP_FD = 4 };

// Output/side buffers of a moments launch (all optional).
struct MomentsOut {
  double *rho, *ux, *uy, *T;     // dense [ny][nx]
  double *snap_rho, *snap_T;     // residual snapshot (dense)
  int write_snap;                // 1: store rho, T into snap_*
  int compare_snap;              // 1: accumulate max |phi - snap| and max |phi|
  double *partials;              // per-block partial sums [block][kPartials]
};

constexpr int kPartials = 10;    // mass, energy, px, py, nonfinite, |drho|max, |rho|max, |dT|max, |T|max, 0

// Tile geometry for one lattice.  A block of bx lanes covers bx consecutive
// columns starting one column left of its strip; the bx - 2 inner lanes own
// the strip, the two outer lanes only supply the psi halo.
struct Tiling {
  int bx;       // lanes per block
  int rows;     // rows per band
  int strips, bands;
  int xcd;      // 1: place consecutive bands on the same XCD
  int alt;      // 1: odd bands walk downwards
  int nt;       // 1: non-temporal stores
  int pf;       // rows of load look-ahead (1 or 2)
};

inline int strip_width(int bx) { return bx - 2; }

// Launchers (stream-ordered, no synchronization).  Return hipError_t.
hipError_t launch_step(const Model &m, const Tiling &t, int st, const void *src, void *dst,
                       int treatment, unsigned long long *clamp_counter, hipStream_t s);
// One step with the source term w_i phi div u of Eq. (5) added to the LB g
// update, phi = -T (dp_EOS/dT)_rho; ux, uy: dense [ny][nx] velocity planes of
// time t (the moments launch writes them).
hipError_t launch_step_fd(const Model &m, const Tiling &t, int st, const void *src, void *dst,
                          unsigned long long *cc, const MomentsOut &mo, hipStream_t s);
hipError_t launch_step_src(const Model &m, const Tiling &t, int st, const void *src, void *dst,
                           int treatment, unsigned long long *clamp_counter, const double *ux,
                           const double *uy, hipStream_t s);
// Two steps in one launch (x periodic; bx 64, 128 or 256 for FP32 storage
// with the force of Eq. (2), 128 for FP64 or the mixed force of Eq. (4);
// strips of bx - 6 owned columns): src holds time t, dst receives t + 2.
hipError_t launch_pair(const Model &m, const Tiling &t, int st, const void *src, void *dst,
                       int treatment, unsigned long long *clamp_counter, hipStream_t s);
hipError_t launch_moments(const Model &m, const Tiling &t, int st, const void *src,
                          const MomentsOut &o, hipStream_t s);
hipError_t launch_init(const Model &m, int st, void *dst, const double *rho, const double *ux,
                       const double *uy, const double *T, hipStream_t s);
hipError_t launch_finalize(const double *partials, int nblocks, double *out, hipStream_t s);
hipError_t launch_plane_to_f64(const Model &m, int st, const void *src, int q, double *out,
                               hipStream_t s);
hipError_t launch_plane_from_f64(const Model &m, int st, void *dst, int q, const double *in,
                                 hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
// Finite-difference temperature update (Eqs. (26)-(27)): from the moments of
// time t (dense planes mom[0..3] = rho, ux, uy, T, each nx*ny) and the
// streamed distributions in dst, writes g = cv T^(t+1) f into dst; k1 is a
// dense scratch plane.
hipError_t launch_fd(const Model &m, int st, const double *mom, double *k1, void *dst, hipStream_t s);

// Byte offset of the FP16 reference plane inside one distribution buffer.
__host__ __device__ inline size_t ref_plane_offset(const Model &m, int st) {
  return st == ST_F64 ? 0 : (size_t)m.ref_off;
}

// Batched step: many lattices, one launch.  Device tables, one entry per
// lattice: its model, the byte offsets (from `base`) of its two distribution
// buffers, the parity of the buffer that holds its current state relative to
// the batch-wide step parity, and its psi-clamp counter; plus the tile list.
struct BatchTile {
  int lattice, strip, band, rows;
  int dir;     // +1 up, -1 down
  int halves;  // two-step tiles: 1 = two 64-lane strips (one per wave) over
               // the lattice's last columns, bands `band` and `band2`
  int band2;   // the second wave's band (-1: none)
  int pad;
};
struct BatchTables {
  const Model *models;
  const long long *off0, *off1;
  const int *phase;
  unsigned long long *const *clamp;
  const BatchTile *tiles;
  int ntiles;
  int xcd;
};
hipError_t launch_batch_step(const BatchTables &t, int bx, int pf, int st, char *base, int parity,
                             int treatment, hipStream_t s);
// Two steps of every lattice whose tiles the table lists (pair tiles:
// strips of bx - 6 owned columns; bx 128; mix: some lattice uses the mixed
// force of Eq. (4)).
hipError_t launch_batch_pair(const BatchTables &t, int bx, int st, bool mix, char *base, int parity,
                             int treatment, hipStream_t s);

}  // namespace lbmdev
