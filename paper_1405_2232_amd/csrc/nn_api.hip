// C ABI of the convolution-network kernels: argument checks and launches.
#include <math.h>
#include <stdint.h>

#include "lbm.h"
#include "lbmnn.h"
#include "nn_device.h"

using namespace lbmnn;

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

int status(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EDEVICE; }

bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

bool strides_ok(int cs, int co, int C) { return cs > 0 && co >= 0 && cs % 4 == 0 && co % 4 == 0 && co + C <= cs; }

bool dims_ok(int B, int H, int W) { return B > 0 && H > 0 && W > 0 && (long long)B * H * W < (1LL << 31); }

// rows of B*H per weight-gradient block: about 256 blocks per tap
int rows_per_chunk(int B, int H, int W) {
  long long rows = (long long)B * H;
  long long per = (rows + 255) / 256;
  // at least ~1024 pixels per block so the partial sums stay small
  const long long min_rows = (1024 + W - 1) / W;
  if (per < min_rows) per = min_rows;
  return (int)per;
}

int nchunks(int B, int H, int W) {
  const long long rows = (long long)B * H;
  const int r = rows_per_chunk(B, H, W);
  return (int)((rows + r - 1) / r);
}

bool norm_from(const float *shift, const float *scale, Norm *nm) {
  if (!shift || !scale) return false;
  for (int k = 0; k < 5; ++k) {
    if (!isfinite(shift[k]) || !isfinite(scale[k]) || scale[k] == 0.f) return false;
    nm->shift[k] = shift[k];
    nm->scale[k] = scale[k];
  }
  return true;
}

}  // namespace

extern "C" {

int lbmnn_conv3x3(const uint16_t *x, int xcs, int xco, const uint16_t *mask, int mcs, int mco,
                  const uint16_t *w, const float *bias, uint16_t *y, int ycs, int yco, int B, int H,
                  int W, int cin, int cout, int relu, int wrap_x, void *stream) {
  if (!x || !w || !y || !dims_ok(B, H, W)) return LBM_EINVAL;
  if (cin < 16 || cin % 16 || cout < 16 || cout % 16 || cout > 128) return LBM_EINVAL;
  if (!strides_ok(xcs, xco, cin) || !strides_ok(ycs, yco, cout)) return LBM_EINVAL;
  if (mask && !strides_ok(mcs, mco, cin)) return LBM_EINVAL;
  if (!aligned8(x) || !aligned8(w) || !aligned8(y) || (mask && !aligned8(mask))) return LBM_EINVAL;
  ConvArgs a{x, xcs, xco, mask, mcs, mco, w, bias, y, ycs, yco, B, H, W, cin, cout, relu != 0, wrap_x != 0};
  return status(launch_conv(a, as_stream(stream)));
}

int lbmnn_conv3x3_flip(const uint16_t *w, uint16_t *wt, int cin, int cout, void *stream) {
  if (!w || !wt || cin <= 0 || cout <= 0) return LBM_EINVAL;
  return status(launch_flip(w, wt, cin, cout, as_stream(stream)));
}

size_t lbmnn_wgrad_partials(int B, int H, int W, int cin, int cout) {
  if (!dims_ok(B, H, W) || cin <= 0 || cout <= 0) return 0;
  return (size_t)nchunks(B, H, W) * (9 * (size_t)cin * cout + cout);
}

int lbmnn_conv3x3_wgrad(const uint16_t *x, int xcs, int xco, const uint16_t *dy, int dcs, int dco,
                        const uint16_t *mask, int mcs, int mco, float *dw, float *db,
                        float *partials, int B, int H, int W, int cin, int cout, int wrap_x,
                        void *stream) {
  if (!x || !dy || !dw || !partials || !dims_ok(B, H, W)) return LBM_EINVAL;
  if (cin < 16 || cin % 16 || cin > 128 || cout < 16 || cout % 16 || cout > 128) return LBM_EINVAL;
  if ((cin / 16) * (cout / 16) > 32) return LBM_EINVAL;  // 8 tiles per wave
  if (!strides_ok(xcs, xco, cin) || !strides_ok(dcs, dco, cout)) return LBM_EINVAL;
  if (mask && !strides_ok(mcs, mco, cout)) return LBM_EINVAL;
  if (!aligned8(x) || !aligned8(dy) || (mask && !aligned8(mask))) return LBM_EINVAL;
  const int nc = nchunks(B, H, W);
  WgradArgs a{x, xcs, xco, dy, dcs, dco, mask, mcs, mco, partials,
              partials + (size_t)nc * 9 * cin * cout, B, H, W, cin, cout, wrap_x != 0,
              rows_per_chunk(B, H, W)};
  return status(launch_wgrad(a, nc, dw, db, as_stream(stream)));
}

int lbmnn_pool2(const uint16_t *x, int xcs, int xco, uint16_t *y, int ycs, int yco, int B, int H, int W,
                int C, void *stream) {
  if (!x || !y || !dims_ok(B, H, W) || H % 2 || W % 2 || C <= 0 || C % 4) return LBM_EINVAL;
  if (!strides_ok(xcs, xco, C) || !strides_ok(ycs, yco, C) || !aligned8(x) || !aligned8(y)) return LBM_EINVAL;
  return status(launch_pool2(x, xcs, xco, y, ycs, yco, B, H, W, C, as_stream(stream)));
}

int lbmnn_pool2_back(const uint16_t *dy, int dcs, int dco, uint16_t *dx, int xcs, int xco, int B, int H,
                     int W, int C, void *stream) {
  if (!dy || !dx || !dims_ok(B, H, W) || H % 2 || W % 2 || C <= 0 || C % 4) return LBM_EINVAL;
  if (!strides_ok(dcs, dco, C) || !strides_ok(xcs, xco, C) || !aligned8(dy) || !aligned8(dx)) return LBM_EINVAL;
  return status(launch_pool2_back(dy, dcs, dco, dx, xcs, xco, B, H, W, C, as_stream(stream)));
}

int lbmnn_up2(const uint16_t *x, int xcs, int xco, uint16_t *y, int ycs, int yco, int B, int H, int W,
              int C, void *stream) {
  if (!x || !y || !dims_ok(B, 2 * H, 2 * W) || C <= 0 || C % 4) return LBM_EINVAL;
  if (!strides_ok(xcs, xco, C) || !strides_ok(ycs, yco, C) || !aligned8(x) || !aligned8(y)) return LBM_EINVAL;
  return status(launch_up2(x, xcs, xco, y, ycs, yco, B, H, W, C, as_stream(stream)));
}

int lbmnn_up2_back(const uint16_t *dy, int dcs, int dco, uint16_t *dx, int xcs, int xco, int B, int H,
                   int W, int C, void *stream) {
  if (!dy || !dx || !dims_ok(B, 2 * H, 2 * W) || C <= 0 || C % 4) return LBM_EINVAL;
  if (!strides_ok(dcs, dco, C) || !strides_ok(xcs, xco, C) || !aligned8(dy) || !aligned8(dx)) return LBM_EINVAL;
  return status(launch_up2_back(dy, dcs, dco, dx, xcs, xco, B, H, W, C, as_stream(stream)));
}

int lbmnn_pack_input(const double *rho, const double *T, const double *s, double tc, const float *shift,
                     const float *scale, uint16_t *x0, float *base, int B, int H, int W, void *stream) {
  Norm nm;
  if (!rho || !T || !s || !x0 || !base || !dims_ok(B, H, W) || !(tc > 0) || !norm_from(shift, scale, &nm))
    return LBM_EINVAL;
  if (!aligned8(x0)) return LBM_EINVAL;
  return status(launch_pack_input(rho, T, s, tc, nm, x0, base, B, H * W, as_stream(stream)));
}

int lbmnn_pack_target(const double *rho, const double *T, double tc, const float *shift, const float *scale,
                      float *t, int B, int H, int W, void *stream) {
  Norm nm;
  if (!rho || !T || !t || !dims_ok(B, H, W) || !(tc > 0) || !norm_from(shift, scale, &nm)) return LBM_EINVAL;
  return status(launch_pack_target(rho, T, tc, nm, t, (size_t)B * H * W, as_stream(stream)));
}

int lbmnn_unpack_output(const float *pred, double tc, const float *shift, const float *scale, double *rho,
                        double *T, int B, int H, int W, void *stream) {
  Norm nm;
  if (!pred || !rho || !T || !dims_ok(B, H, W) || !(tc > 0) || !norm_from(shift, scale, &nm)) return LBM_EINVAL;
  return status(launch_unpack(pred, tc, nm, rho, T, (size_t)B * H * W, as_stream(stream)));
}

int lbmnn_head(const uint16_t *f, int fcs, int fco, const float *base, const float *wh, const float *bh,
               float *pred, int B, int H, int W, int C, void *stream) {
  if (!f || !base || !wh || !bh || !pred || !dims_ok(B, H, W) || (C != 16 && C != 32)) return LBM_EINVAL;
  if (!strides_ok(fcs, fco, C)) return LBM_EINVAL;
  return status(launch_head(f, fcs, fco, base, wh, bh, pred, (size_t)B * H * W, C, as_stream(stream)));
}

size_t lbmnn_head_partials(int B, int H, int W, int C) {
  if (!dims_ok(B, H, W) || C <= 0) return 0;
  return (size_t)head_blocks((size_t)B * H * W) * (3 + 2 * (size_t)C);
}

int lbmnn_head_loss(const uint16_t *f, int fcs, int fco, const float *base, const float *wh, const float *bh,
                    const float *t, float *loss, float *dwh, float *dbh, uint16_t *df, int dfcs, int dfco,
                    float *partials, int B, int H, int W, int C, void *stream) {
  if (!f || !base || !wh || !bh || !t || !loss || !dwh || !dbh || !df || !partials) return LBM_EINVAL;
  if (!dims_ok(B, H, W) || (C != 16 && C != 32)) return LBM_EINVAL;
  if (!strides_ok(fcs, fco, C) || !strides_ok(dfcs, dfco, C)) return LBM_EINVAL;
  return status(launch_head_loss(f, fcs, fco, base, wh, bh, t, loss, dwh, dbh, df, dfcs, dfco, partials,
                                 (size_t)B * H * W, C, as_stream(stream)));
}

int lbmnn_adam(float *w, uint16_t *w16, const float *g, float *m, float *v, size_t n, float lr, float beta1,
               float beta2, float eps, int t, void *stream) {
  if (!w || !w16 || !g || !m || !v || n == 0 || t < 1) return LBM_EINVAL;
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f)) return LBM_EINVAL;
  const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
  return status(launch_adam(w, w16, g, m, v, n, lr, beta1, beta2, eps, c1, c2, as_stream(stream)));
}

int lbmnn_to_bf16(const float *src, uint16_t *dst, size_t n, void *stream) {
  if (!src || !dst || n == 0) return LBM_EINVAL;
  return status(launch_to_bf16(src, dst, n, as_stream(stream)));
}

}  // extern "C"
