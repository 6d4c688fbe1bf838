// Host side of the liblbm C ABI (include/lbm.h): parameter checks,
// workspace carving, stream-ordered launches and status reporting.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <new>
#include <vector>

#include "lbm_ctx.h"

using lbmdev::Model;
using lbmdev::Tiling;

namespace lbmhost {


// Compute units of the current device (256 on MI355X).
static int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return 256;
  return cus;
}

int one_step_bx(int nx) { return nx >= 192 ? 256 : (nx > 62 ? 128 : 64); }

// two-step blocks of bx lanes that fit on one CU: at most two waves per
// SIMD for FP32 storage and one for FP64 (registers), and no more than the
// 160 KB of LDS hold (the rings: 3 x 18 distributions, 2 x 4 psi rows, 2 x
// 4 references, and with the mixed force 2 x 4 psi^2 rows, per lane)
int pair_blocks_per_cu(int st, int bx, bool mix) {
  const int waves = st == lbmdev::ST_F64 ? 4 : 8;
  const long long lds = (long long)bx * (54 * (st == lbmdev::ST_F64 ? 8 : 4) + 64 + 32 + (mix ? 64 : 0));
  long long by_lds = 163840 / lds;
  long long by_waves = waves / (bx / 64);
  long long b = by_lds < by_waves ? by_lds : by_waves;
  return b < 1 ? 1 : (int)b;
}

// Band height shared by the lattices of a batch for the two-step kernel.
// half_strips[i] = 64-lane strips per band row of lattice i: two per full
// strip of 122 columns, plus one for a last strip of at most 58 columns
// (whose block covers two bands, one per wave) or two for a wider one.  For
// each candidate height the launch is simulated as the batch builds it:
// tiles grouped by lattice, cost = the taller band's rows + 7 pipeline rows,
// cut into eight runs of equal cost (one per XCD), each run longest first,
// each XCD filling its slots in list order; the height with the shortest
// simulated launch wins (the taller one on ties: fewer halo rows).
int pair_rows_for(const long long *half_strips, const int *ny, int count, int st, bool mix) {
  const long long slots = (long long)device_cus() * pair_blocks_per_cu(st, 128, mix);
  const int per_xcd = slots >= 8 ? (int)(slots / 8) : 1;
  int maxny = 6;
  for (int i = 0; i < count; ++i) maxny = ny[i] > maxny ? ny[i] : maxny;
  const int top = maxny < 160 ? maxny : 160;
  std::vector<int> cost;
  std::vector<long long> heap;
  long long best = -1;
  int rows = 6;
  for (int r = 6; r <= top; ++r) {
    cost.clear();
    long long total = 0;
    for (int i = 0; i < count; ++i) {
      const int rr = r < ny[i] ? r : ny[i];
      const int bands = (ny[i] + rr - 1) / rr;
      const long long full = half_strips[i] / 2;
      const bool half = (half_strips[i] & 1) != 0;
      for (int b = 0; b < bands; ++b) {
        const int n = (b + 1) * rr < ny[i] ? rr : ny[i] - b * rr;
        for (long long s = 0; s < full; ++s) cost.push_back(n + 7);
        if (half && (b & 1) == 0) {
          const int nb = b + 1 < bands ? ((b + 2) * rr < ny[i] ? rr : ny[i] - (b + 1) * rr) : 0;
          cost.push_back((n > nb ? n : nb) + 7);
        }
      }
    }
    for (int c : cost) total += c;
    long long make = 0, acc = 0;
    size_t k = 0;
    for (int x = 0; x < 8 && k < cost.size(); ++x) {
      const size_t first = k;
      while (k < cost.size() && (x == 7 || acc * 8 < total * (x + 1))) acc += cost[k++];
      std::vector<int> run(cost.begin() + first, cost.begin() + k);
      std::sort(run.begin(), run.end(), [](int a, int b) { return a > b; });
      heap.assign(per_xcd, 0);  // min-heap of slot finishing times
      for (int c : run) {
        std::pop_heap(heap.begin(), heap.end(), std::greater<long long>());
        heap.back() += c;
        std::push_heap(heap.begin(), heap.end(), std::greater<long long>());
      }
      make = std::max(make, *std::max_element(heap.begin(), heap.end()));
    }
    if (best < 0 || make <= best) {
      best = make;
      rows = r;
    }
  }
  return rows;
}

// Whether the work fills the chip: one-step blocks of bx lanes over
// `lanes` strip-rows would need bands of at least 6 rows to occupy every
// slot.  Smaller work is bound by the latency of each block's row walk,
// where a two-step launch (about n + 7 dependent row iterations for two
// steps of an n-row band) loses to two one-step launches with short bands
// (eight 64^2 FP64 lattices: 15.4 us per step paired, 7.0 unpaired).
bool fills_chip(long long lanes, int bx) {
  const long long slots = (long long)device_cus() * (512 / bx);
  return lanes >= 6 * slots;
}

// Band height of the one-step kernel for `lanes` strip-rows (strips x rows,
// summed over a batch's lattices) of blocks of bx lanes: `cap` rows when the
// work fills the chip many times over, fewer (down to 2) when the blocks
// would not fill the 2-waves-per-SIMD slots, because a block walks its band
// row after row and small lattices are bound by that latency (eight 64^2
// lattices: 14.3 us per step at 8 rows, 7.0 us at 2).
int one_step_rows(long long lanes, int bx, int cap) {
  const long long slots = (long long)device_cus() * (512 / bx);
  long long r = (lanes + slots - 1) / slots;
  if (r < 2) r = 2;
  if (r > cap) r = cap;
  return (int)r;
}

// Default tile shape: wide strips (inner width bx - 2) and bands of 6 rows
// (fewer on small lattices, see one_step_rows).  Short bands give many
// blocks (the step is latency-bound at two waves per SIMD) and their two
// halo rows are re-read from L2 by the neighbouring band running on the same
// XCD at the same time (2048^2: 6 rows 1.6 % faster than 8 in FP64, 0.7 % in
// FP32; 12 and 16 rows slower).
Tiling default_tiling(int nx, int ny, int precision) {
  Tiling t;
  t.bx = one_step_bx(nx);
  t.strips = (nx + t.bx - 3) / (t.bx - 2);
  t.rows = one_step_rows((long long)t.strips * ny, t.bx, 6);
  if (t.rows > ny) t.rows = ny;
  t.bands = (ny + t.rows - 1) / t.rows;
  t.xcd = 1;
  t.alt = 1;
  t.nt = 0;
  t.pf = 2;
  (void)precision;
  // experiment knobs (environment) override the defaults
  const long long ebx = env_ll("LBM_BX", 0), erows = env_ll("LBM_ROWS", 0);
  if (ebx == 64 || ebx == 128 || ebx == 256 || ebx == 512) t.bx = (int)ebx;
  if (erows >= 1) t.rows = (int)(erows < ny ? erows : ny);
  t.strips = (nx + t.bx - 3) / (t.bx - 2);
  t.bands = (ny + t.rows - 1) / t.rows;
  t.xcd = (int)env_ll("LBM_XCD", t.xcd);
  t.alt = (int)env_ll("LBM_ALT", t.alt);
  t.nt = (int)env_ll("LBM_NT", t.nt);
  t.pf = (int)env_ll("LBM_PF", t.pf);
  return t;
}

// Two-step tiling.  Blocks of 128 lanes (122 owned columns) run four to a
// CU for FP32 storage (two waves per SIMD; the LDS rings take 40 KB per
// block), two for FP64 (66 KB; one wave per SIMD).  The ny rows
// are split evenly into `bands` bands (heights differ by at most one row).
// A band of r rows costs its block about 2 r + 4 row collisions (the first
// step also runs on two rows beyond each band edge), and the blocks of a
// launch run in ceil(blocks / slots) rounds; rows <= 0 picks the fewest
// bands (tallest band at least 6 rows) that minimise rounds x (2 r_max + 4).
// That favours one round of tall bands: at 2048^2, 59 bands of 35 rows
// (1003 blocks for 1024 slots, 0.101 ms per step against 0.118 with 12-row
// bands in three rounds); at 4096^2, 30 bands of 137 rows (0.358 ms per
// step against 0.420 at 14 rows).  rows > 0 gives bands of at most `rows`
// rows.
Tiling pair_tiling(int nx, int ny, int rows, int st, bool mix) {
  Tiling t;
  const long long ebx = env_ll("LBM_PAIR_BX", 128);
  t.bx = ebx == 64 ? 64 : (ebx == 256 ? 256 : 128);
  if (st == lbmdev::ST_F64 || mix) t.bx = 128;  // the only width built for these
  t.strips = (nx + t.bx - 7) / (t.bx - 6);
  if (rows > 0) {
    t.bands = (ny + rows - 1) / rows;
  } else {
    const long long slots = (long long)device_cus() * pair_blocks_per_cu(st, t.bx, mix);
    long long best = -1;
    t.bands = 1;
    for (int bands = 1; bands <= (ny + 5) / 6; ++bands) {
      const long long blocks = (long long)t.strips * bands;
      const long long cost = ((blocks + slots - 1) / slots) * (2LL * ((ny + bands - 1) / bands) + 4);
      if (best < 0 || cost < best) {
        best = cost;
        t.bands = bands;
      }
    }
  }
  if (t.bands > ny) t.bands = ny;
  t.rows = (ny + t.bands - 1) / t.bands;  // the tallest band
  t.xcd = (int)env_ll("LBM_XCD", 1);
  t.alt = 0;
  t.nt = 0;
  t.pf = 1;
  return t;
}

// Tiling of the moments and reduction launches: a function of the lattice
// size alone, so that the per-block partials buffer it sizes does not
// depend on the device or the environment.  8-row bands where that still
// gives 1024 blocks; shorter bands (down to one row) on smaller lattices,
// whose moments pass is bound by one block's row walk (a 64^2 lattice:
// 8 blocks of 8 rows take about 20 us).
Tiling moments_tiling(int nx, int ny) {
  Tiling t;
  t.bx = one_step_bx(nx);
  t.strips = (nx + t.bx - 3) / (t.bx - 2);
  const long long want = (long long)t.strips * ny / 1024;  // rows per band for 1024 blocks
  t.rows = want >= 8 ? 8 : (want < 1 ? 1 : (int)want);
  if (t.rows > ny) t.rows = ny;
  t.bands = (ny + t.rows - 1) / t.rows;
  t.xcd = 1;
  t.alt = 1;
  t.nt = 0;
  t.pf = 1;
  return t;
}

long long env_ll(const char *name, long long dflt) {
  const char *s = getenv(name);
  if (!s || !*s) return dflt;
  return atoll(s);
}

int storage_of(const lbm_params *p) {
  return p->precision == LBM_FP64 ? lbmdev::ST_F64
         : (p->precision == LBM_FP32_DEV ? lbmdev::ST_F32_GLOBAL : lbmdev::ST_F32_LOCAL);
}

bool compute_layout(const lbm_params *p, Layout *L) {
  const int fp32 = p->precision != LBM_FP64;
  L->elem = fp32 ? 4 : 8;
  const int align_elems = (int)(kAlign / L->elem);
  const long long row = (long long)align_up((size_t)p->nx, (size_t)align_elems);
  if (env_ll("LBM_LAYOUT", 1) == 1) {
    // row-interleaved (default): the 18 rows (one per distribution) of
    // lattice row y are consecutive, each followed by a 256-byte stagger;
    // the kernels see a row stride (pitch) of 18 such rows and a
    // distribution stride (plane) of one.  A block's loads of one lattice
    // row then fall in one contiguous span instead of 18 planes far apart
    // (measured 4 % faster).  One row group past the end (plus 256
    // elements) holds the slots that lanes owning no node store into.
    L->plane = row + align_elems;
    L->pitch = (int)(18 * L->plane);
    // the reference rows get a 256-byte stagger too: with a power-of-two
    // row length, the rows that concurrent blocks touch would all map to
    // the same HBM channel (measured 2.5x slower)
    L->rpitch = (int)(row + 128);
    const long long body = (long long)p->ny * L->pitch + L->pitch + 512;
    L->ref_off = align_up((size_t)body * L->elem, kAlign);
    L->ref_bytes = ((size_t)p->ny * L->rpitch + 512) * 2;
  } else {
    // one plane per distribution, each ending in a 4 KiB pad: the pad
    // staggers the 18 streams of a row over HBM channels and holds the
    // slots that lanes owning no node store into (the kernels need at
    // least 512 elements there)
    L->pitch = (int)row;
    long long pad = env_ll("LBM_PLANE_PAD", 16) * align_elems;
    if (pad < 512) pad = 512;
    L->plane = (long long)align_up((size_t)L->pitch * (size_t)p->ny, (size_t)align_elems) + pad;
    L->rpitch = L->pitch;
    L->ref_off = (size_t)L->plane * 18 * L->elem;
    L->ref_bytes = (size_t)L->plane * 2;
  }
  // the distributions, then (LBM_FP32_LOCAL) one FP16 reference plane
  L->dist_bytes = align_up(L->ref_off + (p->precision == LBM_FP32_LOCAL ? L->ref_bytes : 0), kAlign);
  const size_t n = (size_t)p->nx * (size_t)p->ny;
  size_t off = 0;
  L->off_buf[0] = off;
  off += L->dist_bytes;
  L->off_buf[1] = off;
  off += L->dist_bytes;
  L->off_staging = off;
  off += align_up(4 * n * sizeof(double), kAlign);
  L->off_snap = off;
  off += align_up(2 * n * sizeof(double), kAlign);
  Tiling t = moments_tiling(p->nx, p->ny);
  L->max_blocks = t.strips * t.bands;
  L->off_partials = off;
  off += align_up((size_t)L->max_blocks * lbmdev::kPartials * sizeof(double), kAlign);
  L->off_out = off;
  off += align_up(lbmdev::kPartials * sizeof(double), kAlign);
  L->off_counters = off;
  off += align_up(8 * sizeof(unsigned long long), kAlign);
  L->off_fd = off;  // first stage of the finite-difference treatment
  off += align_up(n * sizeof(double), kAlign);
  L->total = off;
  return true;
}

int validate(const lbm_params *p) {
  if (!p) return LBM_EINVAL;
  if (p->nx < 1 || p->ny < 1) return LBM_EINVAL;
  if ((long long)p->nx * p->ny >= (1LL << 31)) return LBM_EINVAL;
  if (!(p->tau_f > 0.5) || !(p->tau_g > 0.5) || !isfinite(p->tau_f) || !isfinite(p->tau_g))
    return LBM_EINVAL;
  if (!(p->cv > 0.0) || !isfinite(p->cv)) return LBM_EINVAL;
  if (!isfinite(p->G) || !isfinite(p->beta)) return LBM_EINVAL;
  if (p->eos != LBM_EOS_CS && p->eos != LBM_EOS_IDEAL) return LBM_EINVAL;
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32_DEV && p->precision != LBM_FP32_LOCAL)
    return LBM_EINVAL;
  if (p->precision != LBM_FP64 && (!isfinite(p->rho_ref) || !isfinite(p->T_ref))) return LBM_EINVAL;
  const int th[4] = {p->thermal_left, p->thermal_right, p->thermal_bottom, p->thermal_top};
  for (int k = 0; k < 4; ++k)
    if (th[k] != LBM_THERMAL_DIRICHLET && th[k] != LBM_THERMAL_ADIABATIC) return LBM_EINVAL;
  if (p->psi_policy != 0 && p->psi_policy != 1) return LBM_EINVAL;
  if (p->wall_x != 0 && p->wall_x != 1 && p->wall_x != 2) return LBM_EINVAL;
  if (p->phi_divu != 0 && p->phi_divu != 1) return LBM_EINVAL;
  if (p->wall_x == 2 && (!(p->rho_out > 0.0) || !isfinite(p->rho_out) || !isfinite(p->u_in)))
    return LBM_EINVAL;
  if (p->wall_y != 0 && p->wall_y != 1) return LBM_EINVAL;
  return LBM_OK;
}

// the kernels address a distribution buffer with 32-bit byte offsets
bool fits_32bit(const Layout &L) {
  return (unsigned long long)L.ref_off + L.ref_bytes < (1ULL << 32);
}

Model make_model(const lbm_params *p, const Layout &L) {
  Model m;
  memset(&m, 0, sizeof(m));
  m.nx = p->nx;
  m.ny = p->ny;
  m.pitch = L.pitch;
  m.plane = L.plane;
  m.ref_off = (long long)L.ref_off;
  m.ref_bytes = (long long)L.ref_bytes;
  m.rpitch = L.rpitch;
  m.inv_tau_f = 1.0 / p->tau_f;
  m.inv_tau_g = 1.0 / p->tau_g;
  m.kf = 1.0 - 1.0 / (2.0 * p->tau_f);
  m.kg = 1.0 - 1.0 / (2.0 * p->tau_g);
  m.G = p->G;
  m.beta = p->beta;
  m.sc_on = p->G != 0.0;
  m.two_over_G = m.sc_on ? 2.0 / p->G : 0.0;
  m.beta_one = p->beta == 1.0;
  m.count_clamps = p->beta != 0.0;
  m.eos = p->eos;
  m.eos_fixed_T = p->eos_fixed_T != 0;
  m.a = p->a;
  m.b = p->b;
  m.R = p->R;
  m.T_eos = p->T_eos;
  m.cv = p->cv;
  m.inv_cv = 1.0 / p->cv;
  m.gx = p->gx;
  m.gy = p->gy;
  m.wall_x = p->wall_x;
  m.wall_y = p->wall_y;
  m.thermal[0] = p->thermal_left;
  m.thermal[1] = p->thermal_right;
  m.thermal[2] = p->thermal_bottom;
  m.thermal[3] = p->thermal_top;
  m.wall_E[0] = p->cv * p->T_left;
  m.wall_E[1] = p->cv * p->T_right;
  m.wall_E[2] = p->cv * p->T_bottom;
  m.wall_E[3] = p->cv * p->T_top;
  m.T_wall[0] = p->T_left;
  m.T_wall[1] = p->T_right;
  m.T_wall[2] = p->T_bottom;
  m.T_wall[3] = p->T_top;
  m.lam_per_rho = (p->tau_g - 0.5) * p->cv * (1.0 / 3.0);
  m.u_in = p->u_in;
  m.rho_out = p->rho_out;
  m.phi_divu = p->phi_divu != 0;
  if (p->precision == LBM_FP32_DEV) m.rho_ref = p->rho_ref;
  if (p->precision != LBM_FP64) m.cvT_ref = p->cv * p->T_ref;
  return m;
}

}  // namespace lbmhost

using namespace lbmhost;


#define HIPCHK(expr)                        \
  do {                                      \
    if ((expr) != hipSuccess) return LBM_EDEVICE; \
  } while (0)

namespace lbmhost {

int run_moments(lbm_ctx *h, double *rho, double *ux, double *uy, double *T, int write_snap,
                       int compare_snap) {
  lbmdev::MomentsOut mo;
  memset(&mo, 0, sizeof(mo));
  mo.rho = rho;
  mo.ux = ux;
  mo.uy = uy;
  mo.T = T;
  mo.snap_rho = h->snap;
  mo.snap_T = h->snap + (size_t)h->p.nx * h->p.ny;
  mo.write_snap = write_snap;
  mo.compare_snap = compare_snap;
  mo.partials = h->partials;
  HIPCHK(lbmdev::launch_moments(h->m, h->tm, h->st, h->buf[h->cur], mo, h->stream));
  HIPCHK(lbmdev::launch_finalize(h->partials, h->tm.strips * h->tm.bands, h->out, h->stream));
  return LBM_OK;
}

// read back reductions + clamp counter; synchronizes
int fetch_totals(lbm_ctx *h, double red[lbmdev::kPartials], unsigned long long *clamps) {
  HIPCHK(hipMemcpyAsync(red, h->out, lbmdev::kPartials * sizeof(double), hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipMemcpyAsync(clamps, h->counters, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int status_of(const lbm_ctx *h, const double red[lbmdev::kPartials], unsigned long long clamps) {
  if (red[4] > 0.0 || !isfinite(red[0]) || !isfinite(red[1])) return LBM_ENONFINITE;
  if (h->p.psi_policy == 1 && clamps > 0) return LBM_EDOMAIN;
  return LBM_OK;
}

int check(lbm_ctx *h) {
  int rc = run_moments(h, nullptr, nullptr, nullptr, nullptr, 0, 0);
  if (rc) return rc;
  double red[lbmdev::kPartials];
  unsigned long long clamps = 0;
  rc = fetch_totals(h, red, &clamps);
  if (rc) return rc;
  return status_of(h, red, clamps);
}

}  // namespace lbmhost

extern "C" {


int lbm_workspace_bytes(const lbm_params *p, size_t *bytes) {
  int rc = validate(p);
  if (rc) return rc;
  if (!bytes) return LBM_EINVAL;
  Layout L;
  compute_layout(p, &L);
  if (!fits_32bit(L)) return LBM_EINVAL;
  *bytes = L.total;
  return LBM_OK;
}

int lbm_create(const lbm_params *p, void *dev_workspace, size_t bytes, void *hip_stream,
               lbm_handle *out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  if (!dev_workspace || ((uintptr_t)dev_workspace % kAlign) != 0) return LBM_EINVAL;
  Layout L;
  compute_layout(p, &L);
  if (!fits_32bit(L)) return LBM_EINVAL;
  if (bytes < L.total) return LBM_ENOMEM;
  lbm_ctx *h = new (std::nothrow) lbm_ctx;
  if (!h) return LBM_ENOMEM;
  memset(h, 0, sizeof(*h));
  h->p = *p;
  h->L = L;
  h->m = make_model(p, L);
  h->st = storage_of(p);
  h->t = default_tiling(p->nx, p->ny, p->precision);
  h->tm = moments_tiling(p->nx, p->ny);
  h->tp = pair_tiling(p->nx, p->ny, (int)env_ll("LBM_PAIR_ROWS", 0), h->st,
                      h->m.sc_on && !h->m.beta_one);
  // two-step launches: periodic x, and no phi div u source (its velocity
  // planes are taken per step)
  h->pair_ok = p->wall_x == 0 && !p->phi_divu;
  h->pair_on = env_ll("LBM_PAIR", fills_chip((long long)h->t.strips * p->ny, h->t.bx) ? 1 : 0) != 0;
  h->stream = (hipStream_t)hip_stream;
  h->ws = (char *)dev_workspace;
  h->buf[0] = h->ws + L.off_buf[0];
  h->buf[1] = h->ws + L.off_buf[1];
  h->staging = (double *)(h->ws + L.off_staging);
  h->snap = (double *)(h->ws + L.off_snap);
  h->fd = (double *)(h->ws + L.off_fd);
  h->partials = (double *)(h->ws + L.off_partials);
  h->out = (double *)(h->ws + L.off_out);
  h->counters = (unsigned long long *)(h->ws + L.off_counters);
  *out = h;
  return LBM_OK;
}

int lbm_init_fields(lbm_handle h, const double *rho, const double *ux, const double *uy,
                    const double *T) {
  if (!h || !rho || !T) return LBM_EINVAL;
  const size_t n = (size_t)h->p.nx * h->p.ny;
  for (size_t c = 0; c < n; ++c) {
    if (!(rho[c] > 0.0) || !isfinite(rho[c]) || !isfinite(T[c])) return LBM_EINVAL;
    if (ux && !isfinite(ux[c])) return LBM_EINVAL;
    if (uy && !isfinite(uy[c])) return LBM_EINVAL;
  }
  double *d_rho = h->staging, *d_T = h->staging + n, *d_ux = h->staging + 2 * n,
         *d_uy = h->staging + 3 * n;
  HIPCHK(hipMemcpyAsync(d_rho, rho, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(d_T, T, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  if (ux) HIPCHK(hipMemcpyAsync(d_ux, ux, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  if (uy) HIPCHK(hipMemcpyAsync(d_uy, uy, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HIPCHK(lbmdev::launch_init(h->m, h->st, h->buf[0], d_rho, ux ? d_ux : nullptr,
                             uy ? d_uy : nullptr, d_T, h->stream));
  HIPCHK(hipMemsetAsync(h->counters, 0, 8 * sizeof(unsigned long long), h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->cur = 0;
  h->steps = 0;
  h->initialized = 1;
  return LBM_OK;
}

namespace {
bool treatment_ok(int t) { return t == LBM_PLAIN || t == LBM_CORRECTED || t == LBM_FD_RK2; }

// one time step; the finite-difference treatment takes the moments of time
// t first, runs the LB step for f (its g result is overwritten) and then
// the two finite-difference stages, which leave g = cv T f
hipError_t one_step(lbm_ctx *h, int treatment) {
  if (treatment == LBM_FD_RK2) {
    const size_t n = (size_t)h->p.nx * h->p.ny;
    lbmdev::MomentsOut mo{};
    mo.rho = h->staging;
    mo.ux = h->staging + n;
    mo.uy = h->staging + 2 * n;
    mo.T = h->staging + 3 * n;
    hipError_t e;
    if (h->p.wall_x != 2 && h->t.pf >= 2) {
      // one launch steps f and writes the moments of time t; the
      // finite-difference update then writes g whole
      e = lbmdev::launch_step_fd(h->m, h->t, h->st, h->buf[h->cur], h->buf[1 - h->cur], h->counters, mo,
                                 h->stream);
    } else {
      e = lbmdev::launch_moments(h->m, h->tm, h->st, h->buf[h->cur], mo, h->stream);
      if (e == hipSuccess)
        e = lbmdev::launch_step(h->m, h->t, h->st, h->buf[h->cur], h->buf[1 - h->cur], LBM_PLAIN,
                                h->counters, h->stream);
    }
    if (e != hipSuccess) return e;
    return lbmdev::launch_fd(h->m, h->st, h->staging, h->fd, h->buf[1 - h->cur], h->stream);
  }
  if (h->p.phi_divu) {
    // the source phi div u of Eq. (5) needs the velocity of time t at the
    // neighbours: the moments launch writes it to staging first
    const size_t n = (size_t)h->p.nx * h->p.ny;
    lbmdev::MomentsOut mo{};
    mo.rho = h->staging;
    mo.ux = h->staging + n;
    mo.uy = h->staging + 2 * n;
    mo.T = h->staging + 3 * n;
    hipError_t e = lbmdev::launch_moments(h->m, h->tm, h->st, h->buf[h->cur], mo, h->stream);
    if (e != hipSuccess) return e;
    return lbmdev::launch_step_src(h->m, h->t, h->st, h->buf[h->cur], h->buf[1 - h->cur], treatment,
                                   h->counters, mo.ux, mo.uy, h->stream);
  }
  return lbmdev::launch_step(h->m, h->t, h->st, h->buf[h->cur], h->buf[1 - h->cur], treatment,
                             h->counters, h->stream);
}
}  // namespace

int lbm_step(lbm_handle h, int n, int treatment) {
  if (!h || n < 1) return LBM_EINVAL;
  if (!treatment_ok(treatment)) return LBM_EINVAL;
  if (!h->initialized) return LBM_ESTATE;
  const bool pairs = h->pair_on && h->pair_ok && (treatment == LBM_PLAIN || treatment == LBM_CORRECTED);
  for (int k = 0; k < n;) {
    // two steps in one launch unless the first of them ends at a check
    if (pairs && k + 1 < n && !(h->check_every > 0 && (h->steps + 1) % h->check_every == 0)) {
      HIPCHK(lbmdev::launch_pair(h->m, h->tp, h->st, h->buf[h->cur], h->buf[1 - h->cur], treatment,
                                 h->counters, h->stream));
      h->steps += 2;
      k += 2;
    } else {
      HIPCHK(one_step(h, treatment));
      h->steps += 1;
      k += 1;
    }
    h->cur ^= 1;
    if (h->check_every > 0 && h->steps % h->check_every == 0) {
      int rc = check(h);
      if (rc) return rc;
    }
  }
  return LBM_OK;
}

int lbm_set_check_interval(lbm_handle h, int k) {
  if (!h || k < 0) return LBM_EINVAL;
  h->check_every = k;
  return LBM_OK;
}

int lbm_sync(lbm_handle h) {
  if (!h) return LBM_EINVAL;
  HIPCHK(hipStreamSynchronize(h->stream));
  if (!h->initialized) return LBM_OK;
  return check(h);
}

int lbm_moments(lbm_handle h, double *rho, double *ux, double *uy, double *T) {
  if (!h) return LBM_EINVAL;
  if (!h->initialized) return LBM_ESTATE;
  const size_t n = (size_t)h->p.nx * h->p.ny;
  double *s = h->staging;
  int rc = run_moments(h, rho ? s : nullptr, ux ? s + n : nullptr, uy ? s + 2 * n : nullptr,
                       T ? s + 3 * n : nullptr, 0, 0);
  if (rc) return rc;
  if (rho) HIPCHK(hipMemcpyAsync(rho, s, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (ux) HIPCHK(hipMemcpyAsync(ux, s + n, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (uy) HIPCHK(hipMemcpyAsync(uy, s + 2 * n, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (T) HIPCHK(hipMemcpyAsync(T, s + 3 * n, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  double red[lbmdev::kPartials];
  unsigned long long clamps = 0;
  rc = fetch_totals(h, red, &clamps);
  if (rc) return rc;
  return status_of(h, red, clamps);
}

int lbm_moments_device(lbm_handle h, double *d_rho, double *d_ux, double *d_uy, double *d_T) {
  if (!h) return LBM_EINVAL;
  if (!h->initialized) return LBM_ESTATE;
  return run_moments(h, d_rho, d_ux, d_uy, d_T, 0, 0);
}

int lbm_totals(lbm_handle h, double out[8]) {
  if (!h || !out) return LBM_EINVAL;
  if (!h->initialized) return LBM_ESTATE;
  int rc = run_moments(h, nullptr, nullptr, nullptr, nullptr, 0, 0);
  if (rc) return rc;
  double red[lbmdev::kPartials];
  unsigned long long clamps = 0;
  rc = fetch_totals(h, red, &clamps);
  if (rc) return rc;
  out[0] = red[0];
  out[1] = red[1];
  out[2] = red[2];
  out[3] = red[3];
  out[4] = red[4];
  out[5] = (double)clamps;
  out[6] = (double)h->steps;
  out[7] = 0.0;
  return LBM_OK;
}

int lbm_step_residual(lbm_handle h, int treatment, double *residual) {
  if (!h || !residual) return LBM_EINVAL;
  if (!treatment_ok(treatment)) return LBM_EINVAL;
  if (!h->initialized) return LBM_ESTATE;
  int rc = run_moments(h, nullptr, nullptr, nullptr, nullptr, 1, 0);
  if (rc) return rc;
  HIPCHK(one_step(h, treatment));
  h->cur ^= 1;
  h->steps += 1;
  rc = run_moments(h, nullptr, nullptr, nullptr, nullptr, 0, 1);
  if (rc) return rc;
  double red[lbmdev::kPartials];
  unsigned long long clamps = 0;
  rc = fetch_totals(h, red, &clamps);
  if (rc) return rc;
  const double r1 = red[6] > 0.0 ? red[5] / red[6] : 0.0;
  const double r2 = red[8] > 0.0 ? red[7] / red[8] : 0.0;
  *residual = r1 > r2 ? r1 : r2;
  return status_of(h, red, clamps);
}

int lbm_get_state(lbm_handle h, double *state) {
  if (!h || !state) return LBM_EINVAL;
  if (!h->initialized) return LBM_ESTATE;
  const size_t n = (size_t)h->p.nx * h->p.ny;
  for (int q = 0; q < 18; ++q) {
    HIPCHK(lbmdev::launch_plane_to_f64(h->m, h->st, h->buf[h->cur], q, h->staging, h->stream));
    HIPCHK(hipMemcpyAsync(state + (size_t)q * n, h->staging, n * sizeof(double),
                          hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  return LBM_OK;
}

int lbm_set_state(lbm_handle h, const double *state) {
  if (!h || !state) return LBM_EINVAL;
  const size_t n = (size_t)h->p.nx * h->p.ny;
  for (size_t c = 0; c < 18 * n; ++c)
    if (!isfinite(state[c])) return LBM_EINVAL;
  if (h->st == lbmdev::ST_F32_LOCAL) {
    // per-node reference from the density of the given state
    double *rho = (double *)malloc(n * sizeof(double));
    if (!rho) return LBM_ENOMEM;
    for (size_t c = 0; c < n; ++c) {
      double a = state[c];
      for (int q = 1; q < 9; ++q) a += state[(size_t)q * n + c];
      rho[c] = a;
    }
    hipError_t e = hipMemcpyAsync(h->staging, rho, n * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
      e = lbmdev::launch_plane_from_f64(h->m, h->st, h->buf[h->cur], -1, h->staging, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    free(rho);
    if (e != hipSuccess) return LBM_EDEVICE;
  }
  for (int q = 0; q < 18; ++q) {
    HIPCHK(hipMemcpyAsync(h->staging, state + (size_t)q * n, n * sizeof(double),
                          hipMemcpyHostToDevice, h->stream));
    HIPCHK(lbmdev::launch_plane_from_f64(h->m, h->st, h->buf[h->cur], q, h->staging, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  h->initialized = 1;
  return LBM_OK;
}

namespace {
// what defines the stored state: sizes, storage form and layout, and the
// deviation shifts (rho_ref, cv T_ref) the FP32 forms are taken from
struct CkptHeader {
  char magic[8];
  int nx, ny, precision, cur;
  long long steps;
  unsigned long long clamps;
  unsigned long long bytes;
  long long plane;
  int pitch, rpitch;
  double rho_ref, cvT_ref;
};

bool same_state_form(const CkptHeader &hd, const lbm_ctx *h, size_t bytes) {
  return memcmp(hd.magic, "LBMCKPT2", 8) == 0 && hd.nx == h->p.nx && hd.ny == h->p.ny &&
         hd.precision == h->p.precision && hd.bytes == bytes && hd.plane == h->L.plane &&
         hd.pitch == h->L.pitch && hd.rpitch == h->L.rpitch && hd.rho_ref == h->m.rho_ref &&
         hd.cvT_ref == h->m.cvT_ref;
}
}  // namespace

int lbm_save(lbm_handle h, const char *path) {
  if (!h || !path) return LBM_EINVAL;
  if (!h->initialized) return LBM_ESTATE;
  const size_t bytes = h->L.dist_bytes;
  char *buf = (char *)malloc(bytes);
  if (!buf) return LBM_ENOMEM;
  CkptHeader hd;
  memset(&hd, 0, sizeof(hd));
  memcpy(hd.magic, "LBMCKPT2", 8);
  hd.nx = h->p.nx;
  hd.ny = h->p.ny;
  hd.precision = h->p.precision;
  hd.steps = h->steps;
  hd.bytes = bytes;
  hd.plane = h->L.plane;
  hd.pitch = h->L.pitch;
  hd.rpitch = h->L.rpitch;
  hd.rho_ref = h->m.rho_ref;
  hd.cvT_ref = h->m.cvT_ref;
  hipError_t e = hipMemcpyAsync(buf, h->buf[h->cur], bytes, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&hd.clamps, h->counters, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                       h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    free(buf);
    return LBM_EDEVICE;
  }
  FILE *fp = fopen(path, "wb");
  int ok = fp && fwrite(&hd, sizeof(hd), 1, fp) == 1 && fwrite(buf, 1, bytes, fp) == bytes;
  if (fp && fclose(fp) != 0) ok = 0;
  free(buf);
  return ok ? LBM_OK : LBM_EINVAL;
}

int lbm_load(lbm_handle h, const char *path) {
  if (!h || !path) return LBM_EINVAL;
  FILE *fp = fopen(path, "rb");
  if (!fp) return LBM_EINVAL;
  CkptHeader hd;
  const size_t bytes = h->L.dist_bytes;
  if (fread(&hd, sizeof(hd), 1, fp) != 1 || !same_state_form(hd, h, bytes)) {
    fclose(fp);
    return LBM_EINVAL;
  }
  char *buf = (char *)malloc(bytes);
  if (!buf) {
    fclose(fp);
    return LBM_ENOMEM;
  }
  const int ok = fread(buf, 1, bytes, fp) == bytes;
  fclose(fp);
  if (!ok) {
    free(buf);
    return LBM_EINVAL;
  }
  hipError_t e = hipMemcpyAsync(h->buf[0], buf, bytes, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->counters, &hd.clamps, sizeof(unsigned long long), hipMemcpyHostToDevice,
                       h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  free(buf);
  if (e != hipSuccess) return LBM_EDEVICE;
  h->cur = 0;
  h->steps = hd.steps;
  h->initialized = 1;
  return LBM_OK;
}

int lbm_set_tiling(lbm_handle h, int bx, int rows) {
  if (!h) return LBM_EINVAL;
  if (bx != 64 && bx != 128 && bx != 256 && bx != 512) return LBM_EINVAL;
  if (rows < 1) return LBM_EINVAL;
  if (rows > h->p.ny) rows = h->p.ny;
  h->t.bx = bx;
  h->t.strips = (h->p.nx + bx - 3) / (bx - 2);
  h->t.rows = rows;
  h->t.bands = (h->p.ny + rows - 1) / rows;
  return LBM_OK;
}

int lbm_set_step_pairing(lbm_handle h, int on, int rows) {
  if (!h || rows < 0) return LBM_EINVAL;
  h->pair_on = on != 0;
  if (rows > 0)
    h->tp = lbmhost::pair_tiling(h->p.nx, h->p.ny, rows, h->st, h->m.sc_on && !h->m.beta_one);
  return LBM_OK;
}

int lbm_get_step_pairing(lbm_handle h, int *active, int *rows) {
  if (!h || !active || !rows) return LBM_EINVAL;
  *active = h->pair_on && h->pair_ok;
  *rows = h->tp.rows;
  return LBM_OK;
}

int lbm_get_tiling(lbm_handle h, int *bx, int *rows) {
  if (!h || !bx || !rows) return LBM_EINVAL;
  *bx = h->t.bx;
  *rows = h->t.rows;
  return LBM_OK;
}

int lbm_destroy(lbm_handle h) {
  if (!h) return LBM_EINVAL;
  delete h;
  return LBM_OK;
}

const char *lbm_strerror(int status) {
  switch (status) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "workspace too small";
    case LBM_EDEVICE: return "HIP runtime error";
    case LBM_ENONFINITE: return "non-finite density or energy";
    case LBM_EDOMAIN: return "pseudopotential outside its real domain";
    case LBM_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

int lbm_copy_probe(void *dst, const void *src, size_t bytes, void *hip_stream) {
  if (!dst || !src || bytes == 0 || bytes % 16 != 0) return LBM_EINVAL;
  HIPCHK(lbmdev::launch_copy(dst, src, bytes, (hipStream_t)hip_stream));
  return LBM_OK;
}

}  // extern "C"
