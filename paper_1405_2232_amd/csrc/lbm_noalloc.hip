// lbm_totals_noalloc: lbm_totals with its scratch memory (the per-block
// FP64 partial sums of the moments launch and the reduced totals) in a
// file-scope device array instead of the handle's workspace, for callers
// that cannot allocate device memory around the call.  Same kernels, same
// fixed reduction order, so the results equal lbm_totals' bit for bit.
#include <mutex>

#include "lbm_ctx.h"

namespace {

// Largest moments launch served: 32768 blocks (a lattice of up to about
// 5,800^2 nodes; at that size the moments tiling has 254-column strips and
// 8-row bands).
constexpr int kMaxBlocks = 32768;
constexpr size_t kPartialDoubles = (size_t)kMaxBlocks * lbmdev::kPartials;
// partials, then the reduced totals (kPartials doubles, 256-byte aligned)
constexpr size_t kScratchDoubles = kPartialDoubles + 32;

// One copy per GPU, alive until the process ends (2.6 MB).  Host code never
// passes this name to a kernel: it stands for a host-side shadow, not a
// device address.  The device address comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices];  // device address of `scratch` per device

// Device address of `scratch` on device `dev`, looked up once per device
// with that device current.
int scratch_of(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return LBM_EDEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return LBM_EDEVICE;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return LBM_EDEVICE;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return LBM_EDEVICE;
    g_scratch[dev] = (double *)p;
  }
  *out = g_scratch[dev];
  return LBM_OK;
}

}  // namespace

extern "C" int lbm_totals_noalloc(lbm_handle h, double out[8]) {
  if (!h || !out) return LBM_EINVAL;
  if (!h->initialized) return LBM_ESTATE;
  const int blocks = h->tm.strips * h->tm.bands;
  if (blocks < 1 || blocks > kMaxBlocks) return LBM_EINVAL;
  // the device that holds the handle's workspace
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, h->ws) != hipSuccess) return LBM_EDEVICE;
  double *base = nullptr;
  int rc = scratch_of(attr.device, &base);
  if (rc) return rc;
  double *partials = base;
  double *red_d = base + kPartialDoubles;
  // every block of the moments launch writes its own partials entry and the
  // finalize kernel writes every total, so nothing needs clearing first
  lbmdev::MomentsOut mo{};
  mo.partials = partials;
  if (lbmdev::launch_moments(h->m, h->tm, h->st, h->buf[h->cur], mo, h->stream) != hipSuccess)
    return LBM_EDEVICE;
  if (lbmdev::launch_finalize(partials, blocks, red_d, h->stream) != hipSuccess) return LBM_EDEVICE;
  double red[lbmdev::kPartials];
  unsigned long long clamps = 0;
  if (hipMemcpyAsync(red, red_d, sizeof(red), hipMemcpyDeviceToHost, h->stream) != hipSuccess)
    return LBM_EDEVICE;
  if (hipMemcpyAsync(&clamps, h->counters, sizeof(clamps), hipMemcpyDeviceToHost, h->stream) !=
      hipSuccess)
    return LBM_EDEVICE;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return LBM_EDEVICE;
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
