// Internal host-side declarations shared by the single-lattice and the
// batched parts of liblbm (not part of the C ABI).
#pragma once

#include <stddef.h>

#include "../../include/lbm.h"
#include "lbm_device.h"

namespace lbmhost {

using lbmdev::Model;
using lbmdev::Tiling;

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
  int pitch;
  int rpitch;             // row stride of the FP16 reference plane
  long long plane;        // elements
  size_t elem;            // bytes per stored value
  size_t dist_bytes;      // one buffer of 18 planes
  size_t ref_off;         // bytes from a buffer to its FP16 reference plane
  size_t ref_bytes;       // size of the reference plane
  size_t off_buf[2];
  size_t off_staging;     // 4 dense FP64 planes
  size_t off_snap;        // 2 dense FP64 planes
  size_t off_partials;
  int max_blocks;
  size_t off_out;         // kPartials doubles
  size_t off_counters;    // 8 u64
  size_t off_fd;          // 1 dense FP64 plane (finite-difference stage)
  size_t total;
};

long long env_ll(const char *name, long long dflt);
Tiling default_tiling(int nx, int ny, int precision);
Tiling moments_tiling(int nx, int ny);
int one_step_bx(int nx);
int one_step_rows(long long lanes, int bx, int cap);
bool fills_chip(long long lanes, int bx);
int pair_rows_for(const long long *half_strips, const int *ny, int count, int st, bool mix);
Tiling pair_tiling(int nx, int ny, int rows, int st, bool mix);
int pair_blocks_per_cu(int st, int bx, bool mix);
int storage_of(const lbm_params *p);
bool compute_layout(const lbm_params *p, Layout *L);
bool fits_32bit(const Layout &L);
int validate(const lbm_params *p);
Model make_model(const lbm_params *p, const Layout &L);

}  // namespace lbmhost

struct lbm_ctx {
  lbm_params p;
  lbmhost::Layout L;
  lbmdev::Model m;
  lbmdev::Tiling t;        // step tiling
  lbmdev::Tiling tm;       // moments tiling (fixed: sizes the partials buffer)
  lbmdev::Tiling tp;       // two-step tiling
  int pair_ok;             // the lattice admits two-step launches
  int pair_on;             // lbm_step uses them
  int st;          // lbmdev::Storage
  hipStream_t stream;
  char *ws;
  void *buf[2];
  int cur;
  double *staging, *snap, *partials, *out, *fd;
  unsigned long long *counters;
  long long steps;
  int initialized;
  int check_every;
};

namespace lbmhost {
int run_moments(lbm_ctx *h, double *rho, double *ux, double *uy, double *T, int write_snap,
                int compare_snap);
int fetch_totals(lbm_ctx *h, double red[lbmdev::kPartials], unsigned long long *clamps);
int status_of(const lbm_ctx *h, const double red[lbmdev::kPartials], unsigned long long clamps);
int check(lbm_ctx *h);
}  // namespace lbmhost
