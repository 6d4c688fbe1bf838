/*
 * lbmnn.h -- C ABI of the convolution-network kernels (gfx950) behind the
 * learned warm start of the thermal pseudopotential LB solver: a small
 * U-Net maps an initial state (density, temperature and the run's T0/T_c,
 * tau_f, tau_g as constant planes) to a near-steady density and
 * temperature from which the LB step (lbm.h) is started instead of the
 * initial state.  Training and inference run on these kernels only.
 *
 * The layers are the textbook ones (no passage of the paper defines
 * them): 3x3 convolution with bias and optional ReLU, 2x2 average pooling,
 * nearest-neighbour 2x upsampling, channel concatenation (by channel
 * offsets), a 1x1 output layer added to the input fields, a mean squared
 * error loss and Adam.
 *
 * Conventions
 *   - Activations are BF16 (uint16_t bit patterns, round to nearest even),
 *     layout NHWC: element (b, y, x, c) at ((b*H + y)*W + x)*cs + co + c,
 *     cs the channel stride and co the channel offset of the tensor (a
 *     concatenation is two tensors sharing one buffer at different
 *     offsets).  cs and co must be multiples of 4 and pointers 8-byte
 *     aligned.
 *   - Convolution weights are BF16 [cout][9][cin] (tap = 3*ky + kx, the
 *     input sample at (y + ky - 1, x + kx - 1)); biases FP32.  cin and cout
 *     must be multiples of 16 (pad the first layer's input channels with
 *     zeros); cout <= 128.  Products accumulate in FP32 on the matrix cores.
 *   - y is bounded by zeros (walls); x wraps periodically when wrap_x != 0,
 *     else it is bounded by zeros too.
 *   - All pointers are device pointers owned by the caller; every call
 *     enqueues work on `stream` (a hipStream_t, NULL = null stream) and does
 *     not synchronize.  Returns LBM_OK (0) or LBM_EINVAL (-1) for bad sizes
 *     or alignment, LBM_EDEVICE (-3) when a launch fails.
 */
#ifndef LBMNN_H
#define LBMNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* y = act(conv3x3(x) + bias); act = ReLU when relu != 0.  With `mask`
 * (nullable) every input value whose mask value is <= 0 reads as zero
 * (the ReLU derivative when x is the gradient of a ReLU layer's output
 * and mask that output).  bias may be NULL. */
int lbmnn_conv3x3(const uint16_t *x, int xcs, int xco, const uint16_t *mask, int mcs, int mco,
                  const uint16_t *w, const float *bias, uint16_t *y, int ycs, int yco, int B,
                  int H, int W, int cin, int cout, int relu, int wrap_x, void *stream);

/* Weights of the input-gradient convolution: wt[ci][8 - tap][co] =
 * w[co][tap][ci], so that lbmnn_conv3x3(dy, ..., wt, cin = cout,
 * cout = cin) gives the gradient with respect to the layer input. */
int lbmnn_conv3x3_flip(const uint16_t *w, uint16_t *wt, int cin, int cout, void *stream);

/* Size in floats of the partial-sum buffer lbmnn_conv3x3_wgrad needs. */
size_t lbmnn_wgrad_partials(int B, int H, int W, int cin, int cout);

/* Weight and bias gradients of y = act(conv3x3(x) + bias) given dy (the
 * gradient wrt y; mask = y applies the ReLU derivative, NULL for none):
 *   dw[co][tap][ci] = sum_p dy'(p, co) x(p + off(tap), ci),
 *   db[co] = sum_p dy'(p, co),
 * with dy' the masked dy.  Overwrites dw (FP32 [cout][9][cin]) and db
 * (FP32 [cout], may be NULL).  `partials` holds lbmnn_wgrad_partials()
 * floats; the sum over pixels runs in a fixed order (deterministic). */
int lbmnn_conv3x3_wgrad(const uint16_t *x, int xcs, int xco, const uint16_t *dy, int dcs, int dco,
                        const uint16_t *mask, int mcs, int mco, float *dw, float *db,
                        float *partials, int B, int H, int W, int cin, int cout, int wrap_x,
                        void *stream);

/* 2x2 average pooling (H, W even): y(b, y, x) = mean of x over the 2x2
 * block; lbmnn_pool2_back adds dy/4 to each of the four inputs'
 * gradients (accumulates into dx). */
int lbmnn_pool2(const uint16_t *x, int xcs, int xco, uint16_t *y, int ycs, int yco, int B, int H,
                int W, int C, void *stream);
int lbmnn_pool2_back(const uint16_t *dy, int dcs, int dco, uint16_t *dx, int xcs, int xco, int B,
                     int H, int W, int C, void *stream);

/* Nearest 2x upsampling from (H, W) to (2H, 2W); the backward sums the
 * four output gradients of each input (overwrites dx). */
int lbmnn_up2(const uint16_t *x, int xcs, int xco, uint16_t *y, int ycs, int yco, int B, int H,
              int W, int C, void *stream);
int lbmnn_up2_back(const uint16_t *dy, int dcs, int dco, uint16_t *dx, int xcs, int xco, int B,
                   int H, int W, int C, void *stream);

/* Input planes.  From FP64 fields rho, T [B][H][W] and per-image scalars
 * s[B][3] = (T0/T_c, tau_f, tau_g): x0 (BF16, 16 channels, NHWC) holds
 *   ((rho - shift[0]) / scale[0], (T/T_c - shift[1]) / scale[1],
 *    (s0 - shift[2]) / scale[2], (s1 - shift[3]) / scale[3],
 *    (s2 - shift[4]) / scale[4], 0, ..., 0),
 * and base (FP32, [B][H][W][2]) the first two channels unrounded.
 * tc is T_c. */
int lbmnn_pack_input(const double *rho, const double *T, const double *s, double tc,
                     const float *shift, const float *scale, uint16_t *x0, float *base, int B,
                     int H, int W, void *stream);

/* Normalised FP32 pair [B][H][W][2] from FP64 rho, T (the training
 * target), and back (pred to rho, T). */
int lbmnn_pack_target(const double *rho, const double *T, double tc, const float *shift,
                      const float *scale, float *t, int B, int H, int W, void *stream);
int lbmnn_unpack_output(const float *pred, double tc, const float *shift, const float *scale,
                        double *rho, double *T, int B, int H, int W, void *stream);

/* Output layer: pred(p, c) = base(p, c) + bh[c] + sum_k wh[c][k] f(p, k),
 * c < 2, k < C (f BF16 NHWC with stride fcs, offset fco; wh FP32 [2][C]).
 * pred is FP32 [B][H][W][2]. */
int lbmnn_head(const uint16_t *f, int fcs, int fco, const float *base, const float *wh,
               const float *bh, float *pred, int B, int H, int W, int C, void *stream);

/* Floats of partial sums lbmnn_head_loss needs. */
size_t lbmnn_head_partials(int B, int H, int W, int C);

/* Output layer, loss and their backward in one pass:
 *   loss = mean over (p, c) of (pred - t)^2 (written to *loss, FP32),
 *   dwh[2][C], dbh[2] (overwritten, FP32), df (BF16 NHWC, stride dfcs,
 *   offset dfco) = gradient of the loss wrt f. */
int lbmnn_head_loss(const uint16_t *f, int fcs, int fco, const float *base, const float *wh,
                    const float *bh, const float *t, float *loss, float *dwh, float *dbh,
                    uint16_t *df, int dfcs, int dfco, float *partials, int B, int H, int W, int C,
                    void *stream);

/* One Adam step over n FP32 parameters with FP32 gradients g and moments
 * m, v (step count t >= 1, bias-corrected); w16 receives the BF16 copy
 * of the updated parameters. */
int lbmnn_adam(float *w, uint16_t *w16, const float *g, float *m, float *v, size_t n, float lr,
               float beta1, float beta2, float eps, int t, void *stream);

/* BF16 copy of n FP32 values (weights after initialisation). */
int lbmnn_to_bf16(const float *src, uint16_t *dst, size_t n, void *stream);

#ifdef __cplusplus
}
#endif
#endif
