// Device-side declarations of the convolution-network kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmnn {

struct ConvArgs {
  const uint16_t *x;
  int xcs, xco;
  const uint16_t *mask;
  int mcs, mco;
  const uint16_t *w;
  const float *bias;
  uint16_t *y;
  int ycs, yco;
  int B, H, W, cin, cout, relu, wrap_x;
};

struct WgradArgs {
  const uint16_t *x;
  int xcs, xco;
  const uint16_t *dy;
  int dcs, dco;
  const uint16_t *mask;
  int mcs, mco;
  float *part;   // [nchunks][9][cout][cin]
  float *bpart;  // [nchunks][cout]
  int B, H, W, cin, cout, wrap_x, rows_per_chunk;
};

// per-channel normalisation (value - shift) / scale of the five input planes
struct Norm {
  double shift[5];
  double scale[5];
};

hipError_t launch_conv(const ConvArgs &a, hipStream_t s);
hipError_t launch_flip(const uint16_t *w, uint16_t *wt, int cin, int cout, hipStream_t s);
hipError_t launch_wgrad(const WgradArgs &a, int nchunks, float *dw, float *db, hipStream_t s);
hipError_t launch_pool2(const uint16_t *x, int xcs, int xco, uint16_t *y, int ycs, int yco, int B, int H,
                        int W, int C, hipStream_t s);
hipError_t launch_pool2_back(const uint16_t *dy, int dcs, int dco, uint16_t *dx, int xcs, int xco, int B,
                             int H, int W, int C, hipStream_t s);
hipError_t launch_up2(const uint16_t *x, int xcs, int xco, uint16_t *y, int ycs, int yco, int B, int H,
                      int W, int C, hipStream_t s);
hipError_t launch_up2_back(const uint16_t *dy, int dcs, int dco, uint16_t *dx, int xcs, int xco, int B,
                           int H, int W, int C, hipStream_t s);
hipError_t launch_pack_input(const double *rho, const double *T, const double *sc, double tc,
                             const Norm &nm, uint16_t *x0, float *base, int B, int HW, hipStream_t s);
hipError_t launch_pack_target(const double *rho, const double *T, double tc, const Norm &nm, float *t,
                              size_t n, hipStream_t s);
hipError_t launch_unpack(const float *pred, double tc, const Norm &nm, double *rho, double *T, size_t n,
                         hipStream_t s);
hipError_t launch_head(const uint16_t *f, int fcs, int fco, const float *base, const float *wh,
                       const float *bh, float *pred, size_t n, int C, hipStream_t s);
int head_blocks(size_t n);
hipError_t launch_head_loss(const uint16_t *f, int fcs, int fco, const float *base, const float *wh,
                            const float *bh, const float *tg, float *loss, float *dwh, float *dbh,
                            uint16_t *df, int dfcs, int dfco, float *part, size_t n, int C,
                            hipStream_t s);
hipError_t launch_adam(float *w, uint16_t *w16, const float *g, float *m, float *v, size_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_to_bf16(const float *src, uint16_t *dst, size_t n, hipStream_t s);

}  // namespace lbmnn
