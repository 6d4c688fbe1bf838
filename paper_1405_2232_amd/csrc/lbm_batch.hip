// Batched stepping of many independent lattices (lbm_batch_* in lbm.h).
//
// Every lattice owns a slice of the batch workspace laid out exactly as a
// single-lattice workspace, with its own lbm_ctx; the batch adds device
// tables (models, buffer offsets, parities, clamp counters, tiles) and one
// kernel launch per step, or per two steps where every lattice admits the
// two-step kernel, that walks the tiles of all active lattices.  Whole
// groups of k launches can be replayed from a captured hipGraph.  Every
// launch swaps each active lattice's two buffers, so `parity` counts
// launches, not steps.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "lbm_ctx.h"

using namespace lbmhost;
using lbmdev::BatchTables;
using lbmdev::BatchTile;

struct lbm_batch_ctx {
  int count;
  int st;
  hipStream_t stream;
  char *ws;
  std::vector<lbm_ctx *> lat;
  std::vector<size_t> lat_off;
  // device tables
  lbmdev::Model *d_models;
  long long *d_off0, *d_off1;
  int *d_phase;
  unsigned long long **d_clamp;
  BatchTile *d_tiles;
  int max_tiles;
  int ntiles;
  int bx, rows, pf;
  BatchTile *d_ptiles;  // tiles of the two-step kernel
  int nptiles;
  int pair_ok, pair_on, prows;
  bool pair_mix;  // some lattice uses the mixed force of Eq. (4)
  std::vector<int> active;
  std::vector<int> phase;  // host copy: lattice buffer = parity ^ phase
  int parity;
  int graph_k;
  hipStream_t cap;  // private stream the graphs are captured on
  hipGraphExec_t exec[2];
  hipGraph_t graph[2];
  int have_graph[2];  // 0, else 1 + treatment + 2 * (two-step launches)
};

namespace {

struct BatchLayout {
  std::vector<size_t> lat_off, lat_bytes;
  size_t off_models, off_off0, off_off1, off_phase, off_clamp, off_tiles, off_ptiles;
  int max_tiles;
  size_t total;
};

// one-row tiles of 64 lanes (62 owned columns) for every lattice fit in
// one round of the device's block slots (eight 64-lane blocks per CU)
bool thin_tiles_fit(int count, const lbm_params *p) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  long long blocks = 0;
  for (int i = 0; i < count; ++i) blocks += (long long)((p[i].nx + 61) / 62) * p[i].ny;
  return blocks <= 8LL * cus;
}

// tiles of one lattice for lanes bx and band height rows
int tiles_of(const lbm_params &p, int bx, int rows) {
  const int strips = (p.nx + bx - 3) / (bx - 2);
  const int r = rows < p.ny ? rows : p.ny;
  return strips * ((p.ny + r - 1) / r);
}

int batch_layout(int count, const lbm_params *p, BatchLayout *B) {
  if (count < 1 || !p) return LBM_EINVAL;
  size_t off = 0;
  B->lat_off.resize(count);
  B->lat_bytes.resize(count);
  long long tiles = 0;
  for (int i = 0; i < count; ++i) {
    int rc = validate(&p[i]);
    if (rc) return rc;
    if (p[i].precision != p[0].precision) return LBM_EINVAL;
    if (p[i].wall_x == 2) return LBM_EINVAL;  // open channels step alone
    if (p[i].phi_divu) return LBM_EINVAL;     // so do lattices with the phi div u source
    Layout L;
    compute_layout(&p[i], &L);
    if (!fits_32bit(L)) return LBM_EINVAL;
    B->lat_off[i] = off;
    B->lat_bytes[i] = L.total;
    off += align_up(L.total, kAlign);
    tiles += tiles_of(p[i], 64, 1);  // the most tiles any tiling can need
  }
  if (tiles > (1LL << 30)) return LBM_EINVAL;
  B->max_tiles = (int)tiles;
  B->off_models = off;
  off += align_up((size_t)count * sizeof(lbmdev::Model), kAlign);
  B->off_off0 = off;
  off += align_up((size_t)count * sizeof(long long), kAlign);
  B->off_off1 = off;
  off += align_up((size_t)count * sizeof(long long), kAlign);
  B->off_phase = off;
  off += align_up((size_t)count * sizeof(int), kAlign);
  B->off_clamp = off;
  off += align_up((size_t)count * sizeof(void *), kAlign);
  B->off_tiles = off;
  off += align_up((size_t)B->max_tiles * sizeof(BatchTile), kAlign);
  B->off_ptiles = off;  // strips of 122 columns: never more than the bound above
  off += align_up((size_t)B->max_tiles * sizeof(BatchTile), kAlign);
  B->total = off;
  return LBM_OK;
}

void drop_graphs(lbm_batch_ctx *b) {
  for (int k = 0; k < 2; ++k) {
    if (b->have_graph[k]) {
      (void)hipGraphExecDestroy(b->exec[k]);
      (void)hipGraphDestroy(b->graph[k]);
      b->have_graph[k] = 0;
    }
  }
}

// Row iterations a two-step tile runs (its block's duration in a full
// chip): the taller band's rows plus the seven of the pipeline.
int pair_cost(const BatchTile &x, const std::vector<lbm_ctx *> &lat) {
  const int ny = lat[x.lattice]->p.ny;
  const auto rows_of = [&](int band) { return band < 0 ? 0 : std::min(band * x.rows + x.rows, ny) - band * x.rows; };
  const int n = x.halves ? std::max(rows_of(x.band), rows_of(x.band2)) : rows_of(x.band);
  return n + 7;
}

// Orders two-step tiles for the launch's XCD mapping (block b runs list
// entry (b mod 8) * per + b / 8 on XCD b mod 8, so each XCD takes one
// contiguous run of the list in order).  The list, grouped by lattice, is
// cut into eight runs of equal row iterations; each run is sorted longest
// first (stably, so equal tiles of one lattice stay neighbours and share
// their halo rows in L2), which leaves the short ragged bands to fill the
// last slots; runs are padded to one length with empty tiles.
void order_for_xcds(std::vector<BatchTile> &pt, const std::vector<lbm_ctx *> &lat) {
  long long total = 0;
  for (const BatchTile &x : pt) total += pair_cost(x, lat);
  std::vector<std::vector<BatchTile>> run(8);
  long long acc = 0;
  int r = 0;
  for (const BatchTile &x : pt) {
    while (r < 7 && acc * 8 >= total * (r + 1)) ++r;
    run[r].push_back(x);
    acc += pair_cost(x, lat);
  }
  size_t per = 0;
  for (auto &v : run) {
    std::stable_sort(v.begin(), v.end(), [&](const BatchTile &a, const BatchTile &b) {
      return pair_cost(a, lat) > pair_cost(b, lat);
    });
    per = std::max(per, v.size());
  }
  BatchTile none;
  memset(&none, 0, sizeof(none));
  none.lattice = -1;
  pt.clear();
  for (auto &v : run) {
    v.resize(per, none);
    pt.insert(pt.end(), v.begin(), v.end());
  }
}

// tile list of the active lattices; consecutive tiles are neighbouring bands
// of one lattice (the kernel deals them to XCDs in runs); odd bands walk down
int upload_tiles(lbm_batch_ctx *b) {
  std::vector<BatchTile> t;
  t.reserve(b->max_tiles);
  for (int i = 0; i < b->count; ++i) {
    if (!b->active[i]) continue;
    const lbm_params &p = b->lat[i]->p;
    const int strips = (p.nx + b->bx - 3) / (b->bx - 2);
    const int rows = b->rows < p.ny ? b->rows : p.ny;
    const int bands = (p.ny + rows - 1) / rows;
    for (int band = 0; band < bands; ++band)
      for (int s = 0; s < strips; ++s) {
        BatchTile x;
        memset(&x, 0, sizeof(x));
        x.lattice = i;
        x.strip = s;
        x.band = band;
        x.rows = rows;
        x.dir = (band & 1) ? -1 : 1;
        t.push_back(x);
      }
  }
  if ((int)t.size() > b->max_tiles) return LBM_EINVAL;
  b->ntiles = (int)t.size();
  if (!t.empty() && hipMemcpyAsync(b->d_tiles, t.data(), t.size() * sizeof(BatchTile),
                                   hipMemcpyHostToDevice, b->stream) != hipSuccess)
    return LBM_EDEVICE;
  // two-step tiles: 128 lanes, strips of 122 owned columns; where a
  // lattice's last columns fit one wave's strip (at most 58), a block covers
  // them over two bands, one per wave
  std::vector<BatchTile> pt;
  if (b->pair_ok) {
    for (int i = 0; i < b->count; ++i) {
      if (!b->active[i]) continue;
      const lbm_params &p = b->lat[i]->p;
      const int full = p.nx / 122, rem = p.nx - 122 * full;
      const bool halves = rem > 0 && rem <= 58 && !env_ll("LBM_NO_HALVES", 0);
      const int strips = full + (rem > 0 && !halves ? 1 : 0);
      const int rows = b->prows < p.ny ? b->prows : p.ny;
      const int bands = (p.ny + rows - 1) / rows;
      for (int band = 0; band < bands; ++band) {
        for (int s = 0; s < strips; ++s) {
          BatchTile x;
          memset(&x, 0, sizeof(x));
          x.lattice = i;
          x.strip = s;
          x.band = band;
          x.rows = rows;
          x.dir = 1;
          pt.push_back(x);
        }
        if (halves && (band & 1) == 0) {
          BatchTile x;
          memset(&x, 0, sizeof(x));
          x.lattice = i;
          x.strip = full;
          x.band = band;
          x.band2 = band + 1 < bands ? band + 1 : -1;
          x.rows = rows;
          x.dir = 1;
          x.halves = 1;
          pt.push_back(x);
        }
      }
    }
  }
  if (!pt.empty() && env_ll("LBM_BATCH_ORDER", 1) != 0) {
    std::vector<BatchTile> ordered = pt;
    order_for_xcds(ordered, b->lat);
    if ((int)ordered.size() <= b->max_tiles) pt.swap(ordered);  // padding fits the table
  }
  if ((int)pt.size() > b->max_tiles) return LBM_EINVAL;
  b->nptiles = (int)pt.size();
  if (!pt.empty() && hipMemcpyAsync(b->d_ptiles, pt.data(), pt.size() * sizeof(BatchTile),
                                    hipMemcpyHostToDevice, b->stream) != hipSuccess)
    return LBM_EDEVICE;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_EDEVICE;
  drop_graphs(b);
  return LBM_OK;
}

// re-derive each lattice's parity phase from its handle (a member may have
// been stepped or re-initialised on its own)
int sync_phases(lbm_batch_ctx *b) {
  bool changed = false;
  for (int i = 0; i < b->count; ++i) {
    const int ph = b->lat[i]->cur ^ b->parity;
    if (ph != b->phase[i]) {
      b->phase[i] = ph;
      changed = true;
    }
  }
  if (!changed) return LBM_OK;
  if (hipMemcpyAsync(b->d_phase, b->phase.data(), b->count * sizeof(int), hipMemcpyHostToDevice,
                     b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return LBM_EDEVICE;
  drop_graphs(b);
  return LBM_OK;
}

BatchTables tables(const lbm_batch_ctx *b, bool pairs) {
  BatchTables t;
  t.models = b->d_models;
  t.off0 = b->d_off0;
  t.off1 = b->d_off1;
  t.phase = b->d_phase;
  t.clamp = b->d_clamp;
  t.tiles = pairs ? b->d_ptiles : b->d_tiles;
  t.ntiles = pairs ? b->nptiles : b->ntiles;
  t.xcd = 1;
  return t;
}

// `launches` launches of `per` steps each
void advance(lbm_batch_ctx *b, int launches, int per) {
  for (int i = 0; i < b->count; ++i)
    if (b->active[i]) {
      if (launches & 1) b->lat[i]->cur ^= 1;
      b->lat[i]->steps += (long long)launches * per;
    }
  if (launches & 1) b->parity ^= 1;
}

hipError_t launch(const lbm_batch_ctx *b, const BatchTables &t, bool pairs, int parity,
                  int treatment, hipStream_t s) {
  if (pairs) return lbmdev::launch_batch_pair(t, 128, b->st, b->pair_mix, b->ws, parity, treatment, s);
  return lbmdev::launch_batch_step(t, b->bx, b->pf, b->st, b->ws, parity, treatment, s);
}

// Record graph_k launches on the private stream (nothing runs); the graph
// is then replayed on the caller's stream.
int capture(lbm_batch_ctx *b, int treatment, bool pairs) {
  const int par = b->parity;
  if (!b->cap && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    b->cap = nullptr;
    return LBM_EDEVICE;
  }
  if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return LBM_EDEVICE;
  const BatchTables t = tables(b, pairs);
  hipError_t e = hipSuccess;
  for (int k = 0; k < b->graph_k && e == hipSuccess; ++k)
    e = launch(b, t, pairs, par ^ (k & 1), treatment, b->cap);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->cap, &g);
  if ((e != hipSuccess || e2 != hipSuccess) && g) (void)hipGraphDestroy(g);
  if (e != hipSuccess || e2 != hipSuccess) return LBM_EDEVICE;
  hipGraphExec_t x;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return LBM_EDEVICE;
  }
  b->graph[par] = g;
  b->exec[par] = x;
  b->have_graph[par] = 1 + treatment + 2 * (int)pairs;  // what it was captured with
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_workspace_bytes(int count, const lbm_params *p, size_t *bytes) {
  if (!bytes) return LBM_EINVAL;
  BatchLayout B;
  int rc = batch_layout(count, p, &B);
  if (rc) return rc;
  *bytes = B.total;
  return LBM_OK;
}

int lbm_batch_create(int count, const lbm_params *p, void *dev_workspace, size_t bytes,
                     void *hip_stream, lbm_batch_handle *out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  BatchLayout B;
  int rc = batch_layout(count, p, &B);
  if (rc) return rc;
  if (!dev_workspace || ((uintptr_t)dev_workspace % kAlign) != 0) return LBM_EINVAL;
  if (bytes < B.total) return LBM_ENOMEM;
  lbm_batch_ctx *b = new (std::nothrow) lbm_batch_ctx();
  if (!b) return LBM_ENOMEM;
  b->count = count;
  b->stream = (hipStream_t)hip_stream;
  b->ws = (char *)dev_workspace;
  b->lat.assign(count, nullptr);
  b->lat_off = B.lat_off;
  b->active.assign(count, 1);
  b->phase.assign(count, 0);
  b->parity = 0;
  b->max_tiles = B.max_tiles;
  b->graph_k = 0;
  b->cap = nullptr;
  b->have_graph[0] = b->have_graph[1] = 0;
  b->d_models = (lbmdev::Model *)(b->ws + B.off_models);
  b->d_off0 = (long long *)(b->ws + B.off_off0);
  b->d_off1 = (long long *)(b->ws + B.off_off1);
  b->d_phase = (int *)(b->ws + B.off_phase);
  b->d_clamp = (unsigned long long **)(b->ws + B.off_clamp);
  b->d_tiles = (BatchTile *)(b->ws + B.off_tiles);
  b->d_ptiles = (BatchTile *)(b->ws + B.off_ptiles);
  std::vector<lbmdev::Model> models(count);
  std::vector<long long> o0(count), o1(count);
  std::vector<unsigned long long *> cl(count);
  for (int i = 0; i < count; ++i) {
    rc = lbm_create(&p[i], b->ws + B.lat_off[i], B.lat_bytes[i], hip_stream, &b->lat[i]);
    if (rc) {
      lbm_batch_destroy(b);
      return rc;
    }
    models[i] = b->lat[i]->m;
    o0[i] = (long long)((char *)b->lat[i]->buf[0] - b->ws);
    o1[i] = (long long)((char *)b->lat[i]->buf[1] - b->ws);
    cl[i] = b->lat[i]->counters;
  }
  b->st = b->lat[0]->st;
  // shared tile shape: the batch's widest-lattice default, 8-row bands
  Tiling t0 = b->lat[0]->t;
  int maxnx = 0;
  for (int i = 0; i < count; ++i) maxnx = p[i].nx > maxnx ? p[i].nx : maxnx;
  b->bx = one_step_bx(maxnx);
  long long lanes = 0;
  for (int i = 0; i < count; ++i) lanes += (long long)((p[i].nx + b->bx - 3) / (b->bx - 2)) * p[i].ny;
  b->rows = one_step_rows(lanes, b->bx, 8);
  // a batch this small is bound by each block's row walk: one-row bands of
  // 64-lane blocks walk least (eight 64^2 FP64 lattices: 6.7 us per step
  // against 7.0 with 2-row 128-lane tiles, 4.9 against 6.5 once one
  // lattice is left open)
  if (env_ll("LBM_BATCH_THIN", 1) != 0 && thin_tiles_fit(count, p)) {
    b->bx = 64;
    b->rows = 1;
  }
  b->pf = t0.pf;
  b->pair_ok = 1;
  b->pair_mix = false;
  for (int i = 0; i < count; ++i) {
    b->pair_ok = b->pair_ok && b->lat[i]->pair_ok;
    b->pair_mix = b->pair_mix || (b->lat[i]->m.sc_on && !b->lat[i]->m.beta_one);
  }
  b->pair_on = env_ll("LBM_PAIR", fills_chip(lanes, b->bx) ? 1 : 0) != 0;
  {
    // blocks per band row in halves: two per full strip, one for a last
    // strip of at most 58 columns (two bands share its block), two otherwise
    std::vector<long long> st(count);
    std::vector<int> nys(count);
    for (int i = 0; i < count; ++i) {
      const int full = p[i].nx / 122, rem = p[i].nx - 122 * full;
      st[i] = 2LL * full + (rem == 0 ? 0 : (rem <= 58 ? 1 : 2));
      nys[i] = p[i].ny;
    }
    const long long er = env_ll("LBM_PAIR_ROWS", 0);
    b->prows = er > 0 ? (int)er : pair_rows_for(st.data(), nys.data(), count, b->lat[0]->st, b->pair_mix);
  }
  hipError_t e = hipMemcpyAsync(b->d_models, models.data(), count * sizeof(lbmdev::Model),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_off0, o0.data(), count * sizeof(long long), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_off1, o1.data(), count * sizeof(long long), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_phase, b->phase.data(), count * sizeof(int), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_clamp, cl.data(), count * sizeof(void *), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    lbm_batch_destroy(b);
    return LBM_EDEVICE;
  }
  rc = upload_tiles(b);
  if (rc) {
    lbm_batch_destroy(b);
    return rc;
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_lattice(lbm_batch_handle b, int i, lbm_handle *out) {
  if (!b || !out || i < 0 || i >= b->count) return LBM_EINVAL;
  *out = b->lat[i];
  return LBM_OK;
}

int lbm_batch_init_fields(lbm_batch_handle b, int i, const double *rho, const double *ux,
                          const double *uy, const double *T) {
  if (!b || i < 0 || i >= b->count) return LBM_EINVAL;
  return lbm_init_fields(b->lat[i], rho, ux, uy, T);
}

int lbm_batch_moments(lbm_batch_handle b, int i, double *rho, double *ux, double *uy, double *T) {
  if (!b || i < 0 || i >= b->count) return LBM_EINVAL;
  return lbm_moments(b->lat[i], rho, ux, uy, T);
}

int lbm_batch_step(lbm_batch_handle b, int n, int treatment) {
  if (!b || n < 1) return LBM_EINVAL;
  if (treatment != LBM_PLAIN && treatment != LBM_CORRECTED) return LBM_EINVAL;
  for (int i = 0; i < b->count; ++i)
    if (b->active[i] && !b->lat[i]->initialized) return LBM_ESTATE;
  int rc = sync_phases(b);
  if (rc) return rc;
  if (b->ntiles == 0) return LBM_OK;
  const bool pairs = b->pair_on && b->pair_ok && b->nptiles > 0;
  const int per = pairs ? 2 : 1;
  while (b->graph_k >= 2 && n >= b->graph_k * per) {
    const int par = b->parity;
    const int key = 1 + treatment + 2 * (int)pairs;
    if (b->have_graph[par] && b->have_graph[par] != key) {
      (void)hipGraphExecDestroy(b->exec[par]);
      (void)hipGraphDestroy(b->graph[par]);
      b->have_graph[par] = 0;
    }
    if (!b->have_graph[par]) {
      rc = capture(b, treatment, pairs);
      if (rc) return rc;
    }
    if (hipGraphLaunch(b->exec[par], b->stream) != hipSuccess) return LBM_EDEVICE;
    advance(b, b->graph_k, per);
    n -= b->graph_k * per;
  }
  // the rest eagerly: two-step launches, then one step if n is odd
  while (n > 0) {
    const bool two = pairs && n >= 2;
    if (launch(b, tables(b, two), two, b->parity, treatment, b->stream) != hipSuccess)
      return LBM_EDEVICE;
    advance(b, 1, two ? 2 : 1);
    n -= two ? 2 : 1;
  }
  return LBM_OK;
}

int lbm_batch_step_residuals(lbm_batch_handle b, int treatment, double *residuals, int *status) {
  if (!b || !residuals || !status) return LBM_EINVAL;
  if (treatment != LBM_PLAIN && treatment != LBM_CORRECTED) return LBM_EINVAL;
  for (int i = 0; i < b->count; ++i)
    if (b->active[i] && !b->lat[i]->initialized) return LBM_ESTATE;
  // everything is enqueued on the batch's stream before the first wait
  for (int i = 0; i < b->count; ++i) {
    if (!b->active[i]) continue;
    const int rc = run_moments(b->lat[i], nullptr, nullptr, nullptr, nullptr, 1, 0);
    if (rc) return rc;
  }
  int rc = lbm_batch_step(b, 1, treatment);
  if (rc) return rc;
  for (int i = 0; i < b->count; ++i) {
    if (!b->active[i]) continue;
    rc = run_moments(b->lat[i], nullptr, nullptr, nullptr, nullptr, 0, 1);
    if (rc) return rc;
  }
  // every lattice's totals and clamp counter come back before one wait
  std::vector<double> reds((size_t)b->count * lbmdev::kPartials, 0.0);
  std::vector<unsigned long long> clamp(b->count, 0);
  for (int i = 0; i < b->count; ++i) {
    if (!b->active[i]) continue;
    if (hipMemcpyAsync(&reds[(size_t)i * lbmdev::kPartials], b->lat[i]->out,
                       lbmdev::kPartials * sizeof(double), hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipMemcpyAsync(&clamp[i], b->lat[i]->counters, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                       b->stream) != hipSuccess)
      return LBM_EDEVICE;
  }
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_EDEVICE;
  for (int i = 0; i < b->count; ++i) {
    residuals[i] = -1.0;
    status[i] = LBM_OK;
    if (!b->active[i]) continue;
    const double *red = &reds[(size_t)i * lbmdev::kPartials];
    const unsigned long long clamps = clamp[i];
    const double r1 = red[6] > 0.0 ? red[5] / red[6] : 0.0;
    const double r2 = red[8] > 0.0 ? red[7] / red[8] : 0.0;
    residuals[i] = r1 > r2 ? r1 : r2;
    status[i] = status_of(b->lat[i], red, clamps);
  }
  return LBM_OK;
}

int lbm_batch_set_active(lbm_batch_handle b, const int *active) {
  if (!b) return LBM_EINVAL;
  bool same = true;
  for (int i = 0; i < b->count; ++i) {
    const int a = active ? (active[i] != 0) : 1;
    same = same && a == b->active[i];
    b->active[i] = a;
  }
  // an unchanged mask keeps the tile lists and the captured graphs
  return same ? LBM_OK : upload_tiles(b);
}

int lbm_batch_set_tiling(lbm_batch_handle b, int bx, int rows) {
  if (!b) return LBM_EINVAL;
  if (bx != 64 && bx != 128 && bx != 256) return LBM_EINVAL;
  if (rows < 1) return LBM_EINVAL;
  b->bx = bx;
  b->rows = rows;
  return upload_tiles(b);
}

int lbm_batch_set_step_pairing(lbm_batch_handle b, int on, int rows) {
  if (!b || rows < 0) return LBM_EINVAL;
  b->pair_on = on != 0;
  drop_graphs(b);
  if (rows > 0 && rows != b->prows) {
    b->prows = rows;
    return upload_tiles(b);
  }
  return LBM_OK;
}

int lbm_batch_get_step_pairing(lbm_batch_handle b, int *active, int *rows) {
  if (!b || !active || !rows) return LBM_EINVAL;
  *active = b->pair_on && b->pair_ok;
  *rows = b->prows;
  return LBM_OK;
}

int lbm_batch_get_tiling(lbm_batch_handle b, int *bx, int *rows) {
  if (!b || !bx || !rows) return LBM_EINVAL;
  *bx = b->bx;
  *rows = b->rows;
  return LBM_OK;
}

int lbm_batch_use_graph(lbm_batch_handle b, int k) {
  if (!b || k < 0 || k == 1 || (k & 1)) return LBM_EINVAL;
  if (k != b->graph_k) drop_graphs(b);
  b->graph_k = k;
  return LBM_OK;
}

int lbm_batch_sync(lbm_batch_handle b) {
  if (!b) return LBM_EINVAL;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_EDEVICE;
  for (int i = 0; i < b->count; ++i) {
    if (!b->lat[i]->initialized) continue;
    const int rc = lbm_sync(b->lat[i]);
    if (rc) return rc;
  }
  return LBM_OK;
}

int lbm_batch_destroy(lbm_batch_handle b) {
  if (!b) return LBM_EINVAL;
  drop_graphs(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (lbm_ctx *h : b->lat)
    if (h) lbm_destroy(h);
  delete b;
  return LBM_OK;
}

}  // extern "C"
