// Convolution-network kernels (gfx950) of the learned warm start: BF16
// activations and weights, FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x32_bf16 where the depth is a multiple of 32, else
// v_mfma_f32_16x16x16_bf16), FP32 biases, gradients of weights and the
// optimizer state.
//
// Matrix-core operand layout (one 64-lane wave, 16x16xKD product, KD = 16
// or 32, G = KD / 4 depth values per lane):
//   A (16 x KD, rows i, depth k): lane l holds A[l % 16][G (l / 16) + 0..G-1];
//   B (KD x 16, depth k, cols j): lane l holds B[G (l / 16) + 0..G-1][l % 16];
//   D (16 x 16):                  lane l holds D[4 (l / 16) + 0..3][l % 16].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_device.h"

namespace lbmnn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// one matrix-core product of depth 32: A, B eight BF16 values per lane
__device__ inline f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16v8, a),
                                                 __builtin_bit_cast(bf16v8, b), c, 0, 0, 0);
}

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even; NaN stays NaN
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline int wrap(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

// ---------------------------------------------------------------------------
// 3x3 convolution as an implicit product: rows = 16 pixels of one image row
// per wave (64 per block), depth = (tap, input channel) in chunks of KD (32
// when the input channels are a multiple of 32, else 16), columns = output
// channels in NB blocks of 16.  The A operand is read straight from the
// NHWC input (KD/4 consecutive channels per lane); the B operand from the
// [cout][9][cin] weights (cached).
template <int NB, int KD>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
  typedef short vec __attribute__((ext_vector_type(KD / 4)));
  constexpr int G = KD / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int segs = (a.W + 63) >> 6;
  int bid = blockIdx.x;
  const int seg = bid % segs;
  bid /= segs;
  const int yy = bid % a.H;
  const int b = bid / a.H;
  const int x0 = seg * 64 + wave * 16;
  const int px = x0 + (lane & 15);
  const int kg = (lane >> 4) * G;
  f32x4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (x0 < a.W) {
    for (int tap = 0; tap < 9; ++tap) {
      const int sy = yy + tap / 3 - 1;
      int sx = px + tap % 3 - 1;
      bool ok = sy >= 0 && sy < a.H && px < a.W;
      if (a.wrap_x)
        sx = wrap(sx, a.W);
      else
        ok = ok && sx >= 0 && sx < a.W;
      const size_t pix = ((size_t)b * a.H + (ok ? sy : 0)) * a.W + (ok ? sx : 0);
      const uint16_t *xp = a.x + pix * a.xcs + a.xco + kg;
      const uint16_t *mp = a.mask ? a.mask + pix * a.mcs + a.mco + kg : nullptr;
      const uint16_t *wp = a.w + ((size_t)(lane & 15) * 9 + tap) * a.cin + kg;
      for (int c0 = 0; c0 < a.cin; c0 += KD) {
        vec av = (vec)0;
        if (ok) {
          av = *(const vec *)(xp + c0);
          if (mp) {
            const vec mv = *(const vec *)(mp + c0);
#pragma unroll
            for (int j = 0; j < G; ++j)
              if (!(bf2f((uint16_t)mv[j]) > 0.f)) av[j] = 0;
          }
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const vec bv = *(const vec *)(wp + (size_t)nb * 16 * 9 * a.cin + c0);
          if constexpr (KD == 32)
            acc[nb] = mfma32(av, bv, acc[nb]);
          else
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[nb], 0, 0, 0);
        }
      }
    }
  }
  const int col = lane & 15;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int co = nb * 16 + col;
    if (co >= a.cout) continue;
    const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = x0 + (lane >> 4) * 4 + r;
      if (p >= a.W) continue;
      float v = acc[nb][r] + bias;
      if (a.relu) v = v > 0.f ? v : 0.f;
      a.y[(((size_t)b * a.H + yy) * a.W + p) * a.ycs + a.yco + co] = f2bf(v);
    }
  }
}

__global__ void k_flip(const uint16_t *w, uint16_t *wt, int cin, int cout) {
  const int n = cout * 9 * cin;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int ci = i % cin, tap = (i / cin) % 9, co = i / (9 * cin);
    wt[((size_t)ci * 9 + (8 - tap)) * cout + co] = w[i];
  }
}

// ---------------------------------------------------------------------------
// Weight gradient: for one tap per block (blockIdx.y) and one chunk of image
// rows (blockIdx.x), D[co][ci] = sum_p dy'(p, co) x(p + off, ci), depth =
// pixels.  Each 64-pixel segment of dy' and of the shifted x is staged in
// LDS transposed to [channel][pixel] (rows padded to 72 halves, 16-byte
// aligned), so that a lane's eight consecutive pixels are one 16-byte LDS
// read; two depth-32 products per segment.  The block's partial D goes to
// its own slot of `part`; k_wgrad_reduce sums the slots in order.
constexpr int kLdsPitch = 72;
constexpr int kMaxTilesPerWave = 8;

__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t lds_dy[128 * kLdsPitch];
  __shared__ __attribute__((aligned(16))) uint16_t lds_x[128 * kLdsPitch];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int tap = blockIdx.y;
  const int dyo = tap / 3 - 1, dxo = tap % 3 - 1;
  const int mb = a.cout >> 4, nbk = a.cin >> 4, ntiles = mb * nbk;
  const int rows_total = a.B * a.H;
  const int r0 = blockIdx.x * a.rows_per_chunk;
  const int r1 = min(rows_total, r0 + a.rows_per_chunk);
  const int segs = (a.W + 63) >> 6;
  f32x4 acc[kMaxTilesPerWave];
#pragma unroll
  for (int i = 0; i < kMaxTilesPerWave; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  const int p = t & 63, cg0 = t >> 6;
  for (int row = r0; row < r1; ++row) {
    const int b = row / a.H, yy = row % a.H;
    for (int seg = 0; seg < segs; ++seg) {
      const int x = seg * 64 + p;
      // stage dy' [cout][64]
      {
        const bool ok = x < a.W;
        const size_t pix = ((size_t)b * a.H + yy) * a.W + (ok ? x : 0);
        for (int cg = cg0; cg < (a.cout >> 2); cg += 4) {
          bf16x4 v = bf16x4{0, 0, 0, 0};
          if (ok) {
            v = *(const bf16x4 *)(a.dy + pix * a.dcs + a.dco + cg * 4);
            if (a.mask) {
              const bf16x4 mv = *(const bf16x4 *)(a.mask + pix * a.mcs + a.mco + cg * 4);
#pragma unroll
              for (int j = 0; j < 4; ++j)
                if (!(bf2f((uint16_t)mv[j]) > 0.f)) v[j] = 0;
            }
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) lds_dy[(cg * 4 + j) * kLdsPitch + p] = (uint16_t)v[j];
        }
      }
      // stage the shifted input [cin][64]
      {
        const int sy = yy + dyo;
        int sx = x + dxo;
        bool ok = x < a.W && sy >= 0 && sy < a.H;
        if (a.wrap_x)
          sx = wrap(sx, a.W);
        else
          ok = ok && sx >= 0 && sx < a.W;
        const size_t pix = ((size_t)b * a.H + (ok ? sy : 0)) * a.W + (ok ? sx : 0);
        for (int cg = cg0; cg < (a.cin >> 2); cg += 4) {
          bf16x4 v = bf16x4{0, 0, 0, 0};
          if (ok) v = *(const bf16x4 *)(a.x + pix * a.xcs + a.xco + cg * 4);
#pragma unroll
          for (int j = 0; j < 4; ++j) lds_x[(cg * 4 + j) * kLdsPitch + p] = (uint16_t)v[j];
        }
      }
      __syncthreads();
      if (tap == 4 && t < a.cout) {
        float s = 0.f;
        for (int q = 0; q < 64; ++q) s += bf2f(lds_dy[t * kLdsPitch + q]);
        bacc += s;
      }
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const int q8 = ks * 32 + (lane >> 4) * 8;
#pragma unroll
        for (int i = 0; i < kMaxTilesPerWave; ++i) {
          const int tile = wave + 4 * i;
          if (tile < ntiles) {
            const int ib = tile / nbk, jb = tile % nbk;
            const bf16x8 av = *(const bf16x8 *)(lds_dy + (ib * 16 + (lane & 15)) * kLdsPitch + q8);
            const bf16x8 bv = *(const bf16x8 *)(lds_x + (jb * 16 + (lane & 15)) * kLdsPitch + q8);
            acc[i] = mfma32(av, bv, acc[i]);
          }
        }
      }
      __syncthreads();
    }
  }
  float *out = a.part + ((size_t)blockIdx.x * 9 + tap) * a.cout * a.cin;
#pragma unroll
  for (int i = 0; i < kMaxTilesPerWave; ++i) {
    const int tile = wave + 4 * i;
    if (tile < ntiles) {
      const int ib = tile / nbk, jb = tile % nbk;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = ib * 16 + (lane >> 4) * 4 + r, ci = jb * 16 + (lane & 15);
        out[(size_t)co * a.cin + ci] = acc[i][r];
      }
    }
  }
  if (tap == 4 && t < a.cout) a.bpart[(size_t)blockIdx.x * a.cout + t] = bacc;
}

// dw[co][tap][ci] = sum over chunks (in order) of part[chunk][tap][co][ci]
__global__ void k_wgrad_reduce(const float *part, const float *bpart, float *dw, float *db,
                               int nchunks, int cin, int cout) {
  const int per = 9 * cout * cin;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < per) {
    const int ci = i % cin, tap = (i / cin) % 9, co = i / (9 * cin);
    const size_t src = ((size_t)tap * cout + co) * cin + ci;
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * per + src];
    dw[i] = s;
  } else if (db && i < per + cout) {
    const int co = i - per;
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += bpart[(size_t)c * cout + co];
    db[co] = s;
  }
}

// ---------------------------------------------------------------------------
// pooling / upsampling, one thread per (output pixel, 4 channels)
__global__ void k_pool2(const uint16_t *x, int xcs, int xco, uint16_t *y, int ycs, int yco, int B,
                        int H, int W, int C) {
  const int Ho = H / 2, Wo = W / 2, cg = C / 4;
  const size_t n = (size_t)B * Ho * Wo * cg;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % cg) * 4;
    size_t r = i / cg;
    const int xo = (int)(r % Wo);
    r /= Wo;
    const int yo = (int)(r % Ho);
    const int b = (int)(r / Ho);
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const size_t pix = ((size_t)b * H + 2 * yo + dy) * W + 2 * xo + dx;
        const bf16x4 v = *(const bf16x4 *)(x + pix * xcs + xco + c);
#pragma unroll
        for (int j = 0; j < 4; ++j) s[j] += bf2f((uint16_t)v[j]);
      }
    bf16x4 o;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = (short)f2bf(0.25f * s[j]);
    *(bf16x4 *)(y + (((size_t)b * Ho + yo) * Wo + xo) * ycs + yco + c) = o;
  }
}

__global__ void k_pool2_back(const uint16_t *dy, int dcs, int dco, uint16_t *dx, int xcs, int xco,
                             int B, int H, int W, int C) {
  const int Ho = H / 2, Wo = W / 2, cg = C / 4;
  const size_t n = (size_t)B * H * W * cg;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % cg) * 4;
    size_t r = i / cg;
    const int x = (int)(r % W);
    r /= W;
    const int y = (int)(r % H);
    const int b = (int)(r / H);
    const bf16x4 g = *(const bf16x4 *)(dy + (((size_t)b * Ho + y / 2) * Wo + x / 2) * dcs + dco + c);
    bf16x4 *dst = (bf16x4 *)(dx + (((size_t)b * H + y) * W + x) * xcs + xco + c);
    bf16x4 o = *dst;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = (short)f2bf(bf2f((uint16_t)o[j]) + 0.25f * bf2f((uint16_t)g[j]));
    *dst = o;
  }
}

__global__ void k_up2(const uint16_t *x, int xcs, int xco, uint16_t *y, int ycs, int yco, int B,
                      int H, int W, int C) {
  const int Ho = 2 * H, Wo = 2 * W, cg = C / 4;
  const size_t n = (size_t)B * Ho * Wo * cg;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % cg) * 4;
    size_t r = i / cg;
    const int xo = (int)(r % Wo);
    r /= Wo;
    const int yo = (int)(r % Ho);
    const int b = (int)(r / Ho);
    *(bf16x4 *)(y + (((size_t)b * Ho + yo) * Wo + xo) * ycs + yco + c) =
        *(const bf16x4 *)(x + (((size_t)b * H + yo / 2) * W + xo / 2) * xcs + xco + c);
  }
}

__global__ void k_up2_back(const uint16_t *dy, int dcs, int dco, uint16_t *dx, int xcs, int xco,
                           int B, int H, int W, int C) {
  const int Wo = 2 * W, cg = C / 4;
  const size_t n = (size_t)B * H * W * cg;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % cg) * 4;
    size_t r = i / cg;
    const int x = (int)(r % W);
    r /= W;
    const int y = (int)(r % H);
    const int b = (int)(r / H);
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    for (int dyy = 0; dyy < 2; ++dyy)
      for (int dxx = 0; dxx < 2; ++dxx) {
        const size_t pix = ((size_t)b * 2 * H + 2 * y + dyy) * Wo + 2 * x + dxx;
        const bf16x4 v = *(const bf16x4 *)(dy + pix * dcs + dco + c);
#pragma unroll
        for (int j = 0; j < 4; ++j) s[j] += bf2f((uint16_t)v[j]);
      }
    bf16x4 o;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = (short)f2bf(s[j]);
    *(bf16x4 *)(dx + (((size_t)b * H + y) * W + x) * xcs + xco + c) = o;
  }
}

// ---------------------------------------------------------------------------
// input / target / output planes
__global__ void k_pack_input(const double *rho, const double *T, const double *s, double tc,
                             Norm nm, uint16_t *x0, float *base, int B, int HW) {
  const size_t n = (size_t)B * HW;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / HW);
    const float c0 = (float)((rho[i] - nm.shift[0]) / nm.scale[0]);
    const float c1 = (float)((T[i] / tc - nm.shift[1]) / nm.scale[1]);
    float v[16];
    v[0] = c0;
    v[1] = c1;
    for (int k = 0; k < 3; ++k) v[2 + k] = (float)((s[3 * b + k] - nm.shift[2 + k]) / nm.scale[2 + k]);
    for (int k = 5; k < 16; ++k) v[k] = 0.f;
    bf16x4 *dst = (bf16x4 *)(x0 + i * 16);
    for (int q = 0; q < 4; ++q) {
      bf16x4 o;
#pragma unroll
      for (int j = 0; j < 4; ++j) o[j] = (short)f2bf(v[4 * q + j]);
      dst[q] = o;
    }
    base[2 * i] = c0;
    base[2 * i + 1] = c1;
  }
}

__global__ void k_pack_target(const double *rho, const double *T, double tc, Norm nm, float *t,
                              size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    t[2 * i] = (float)((rho[i] - nm.shift[0]) / nm.scale[0]);
    t[2 * i + 1] = (float)((T[i] / tc - nm.shift[1]) / nm.scale[1]);
  }
}

__global__ void k_unpack(const float *pred, double tc, Norm nm, double *rho, double *T, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    rho[i] = (double)pred[2 * i] * nm.scale[0] + nm.shift[0];
    T[i] = ((double)pred[2 * i + 1] * nm.scale[1] + nm.shift[1]) * tc;
  }
}

// ---------------------------------------------------------------------------
// output layer (1x1, C -> 2, residual on the input fields)
template <int C>
__global__ __launch_bounds__(256) void k_head(const uint16_t *f, int fcs, int fco, const float *base,
                                              const float *wh, const float *bh, float *pred, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    float o0 = base[2 * i] + bh[0], o1 = base[2 * i + 1] + bh[1];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const float v = bf2f(f[i * fcs + fco + k]);
      o0 += wh[k] * v;
      o1 += wh[C + k] * v;
    }
    pred[2 * i] = o0;
    pred[2 * i + 1] = o1;
  }
}

// one block per kHeadPix pixels; its partial sums (loss, dbh[2], dwh[2][C])
// go to its own slot, reduced in order by k_head_reduce
constexpr int kHeadPix = 1024;

template <int C>
__global__ __launch_bounds__(256) void k_head_loss(const uint16_t *f, int fcs, int fco,
                                                   const float *base, const float *wh,
                                                   const float *bh, const float *tg, uint16_t *df,
                                                   int dfcs, int dfco, float *part, size_t n) {
  __shared__ float red[256];
  const int t = threadIdx.x;
  const size_t p0 = (size_t)blockIdx.x * kHeadPix;
  const size_t p1 = p0 + kHeadPix < n ? p0 + kHeadPix : n;
  const float inv_n = 1.0f / (float)(2 * n);
  // thread-private partials: loss, dbh0, dbh1, dwh[2][C]
  float acc[3 + 2 * C];
#pragma unroll
  for (int k = 0; k < 3 + 2 * C; ++k) acc[k] = 0.f;
  for (size_t i = p0 + t; i < p1; i += 256) {
    float fv[C];
#pragma unroll
    for (int k = 0; k < C; ++k) fv[k] = bf2f(f[i * fcs + fco + k]);
    float o0 = base[2 * i] + bh[0], o1 = base[2 * i + 1] + bh[1];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      o0 += wh[k] * fv[k];
      o1 += wh[C + k] * fv[k];
    }
    const float e0 = o0 - tg[2 * i], e1 = o1 - tg[2 * i + 1];
    acc[0] += e0 * e0 + e1 * e1;
    const float g0 = 2.f * e0 * inv_n, g1 = 2.f * e1 * inv_n;
    acc[1] += g0;
    acc[2] += g1;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      acc[3 + k] += g0 * fv[k];
      acc[3 + C + k] += g1 * fv[k];
      df[i * dfcs + dfco + k] = f2bf(g0 * wh[k] + g1 * wh[C + k]);
    }
  }
  float *out = part + (size_t)blockIdx.x * (3 + 2 * C);
#pragma unroll
  for (int k = 0; k < 3 + 2 * C; ++k) {
    red[t] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) red[t] += red[t + s];
      __syncthreads();
    }
    if (t == 0) out[k] = red[0];
    __syncthreads();
  }
}

__global__ void k_head_reduce(const float *part, int nblk, int C, size_t n, float *loss, float *dwh,
                              float *dbh) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = 3 + 2 * C;
  if (k >= m) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * m + k];
  if (k == 0)
    *loss = s / (float)(2 * n);
  else if (k < 3)
    dbh[k - 1] = s;
  else
    dwh[k - 3] = s;
}

// ---------------------------------------------------------------------------
__global__ void k_adam(float *w, uint16_t *w16, const float *g, float *m, float *v, size_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    w16[i] = f2bf(wi);
  }
}

__global__ void k_to_bf16(const float *src, uint16_t *dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = f2bf(src[i]);
}

// ---------------------------------------------------------------------------
// launchers
static int grid_for(size_t n, int threads = 256) {
  size_t g = (n + threads - 1) / threads;
  if (g > 65536) g = 65536;
  return g < 1 ? 1 : (int)g;
}

template <int KD>
static hipError_t launch_conv_kd(const ConvArgs &a, int blocks, hipStream_t s) {
  switch ((a.cout + 15) / 16) {
    case 1: hipLaunchKernelGGL((k_conv<1, KD>), dim3(blocks), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_conv<2, KD>), dim3(blocks), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_conv<3, KD>), dim3(blocks), dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_conv<4, KD>), dim3(blocks), dim3(256), 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_conv<5, KD>), dim3(blocks), dim3(256), 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_conv<6, KD>), dim3(blocks), dim3(256), 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_conv<7, KD>), dim3(blocks), dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_conv<8, KD>), dim3(blocks), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_conv(const ConvArgs &a, hipStream_t s) {
  const int blocks = a.B * a.H * ((a.W + 63) / 64);
  // depth-32 products where the input channels allow them (every layer but
  // the first, whose 16 input planes are the padded fields) and their
  // 16-byte loads are aligned (channel strides and offsets multiples of 8)
  const bool kd32 = a.cin % 32 == 0 && a.xcs % 8 == 0 && a.xco % 8 == 0 &&
                    (!a.mask || (a.mcs % 8 == 0 && a.mco % 8 == 0));
  return kd32 ? launch_conv_kd<32>(a, blocks, s) : launch_conv_kd<16>(a, blocks, s);
}

hipError_t launch_flip(const uint16_t *w, uint16_t *wt, int cin, int cout, hipStream_t s) {
  hipLaunchKernelGGL(k_flip, dim3(grid_for((size_t)cout * 9 * cin)), dim3(256), 0, s, w, wt, cin, cout);
  return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs &a, int nchunks, float *dw, float *db, hipStream_t s) {
  hipLaunchKernelGGL(k_wgrad, dim3(nchunks, 9), dim3(256), 0, s, a);
  const int per = 9 * a.cout * a.cin + a.cout;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((per + 255) / 256), dim3(256), 0, s, a.part, a.bpart, dw, db,
                     nchunks, a.cin, a.cout);
  return hipGetLastError();
}

hipError_t launch_pool2(const uint16_t *x, int xcs, int xco, uint16_t *y, int ycs, int yco, int B, int H,
                        int W, int C, hipStream_t s) {
  hipLaunchKernelGGL(k_pool2, dim3(grid_for((size_t)B * (H / 2) * (W / 2) * (C / 4))), dim3(256), 0, s, x,
                     xcs, xco, y, ycs, yco, B, H, W, C);
  return hipGetLastError();
}

hipError_t launch_pool2_back(const uint16_t *dy, int dcs, int dco, uint16_t *dx, int xcs, int xco, int B,
                             int H, int W, int C, hipStream_t s) {
  hipLaunchKernelGGL(k_pool2_back, dim3(grid_for((size_t)B * H * W * (C / 4))), dim3(256), 0, s, dy, dcs,
                     dco, dx, xcs, xco, B, H, W, C);
  return hipGetLastError();
}

hipError_t launch_up2(const uint16_t *x, int xcs, int xco, uint16_t *y, int ycs, int yco, int B, int H,
                      int W, int C, hipStream_t s) {
  hipLaunchKernelGGL(k_up2, dim3(grid_for((size_t)B * 4 * H * W * (C / 4))), dim3(256), 0, s, x, xcs, xco,
                     y, ycs, yco, B, H, W, C);
  return hipGetLastError();
}

hipError_t launch_up2_back(const uint16_t *dy, int dcs, int dco, uint16_t *dx, int xcs, int xco, int B,
                           int H, int W, int C, hipStream_t s) {
  hipLaunchKernelGGL(k_up2_back, dim3(grid_for((size_t)B * H * W * (C / 4))), dim3(256), 0, s, dy, dcs,
                     dco, dx, xcs, xco, B, H, W, C);
  return hipGetLastError();
}

hipError_t launch_pack_input(const double *rho, const double *T, const double *sc, double tc,
                             const Norm &nm, uint16_t *x0, float *base, int B, int HW, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_input, dim3(grid_for((size_t)B * HW)), dim3(256), 0, s, rho, T, sc, tc, nm, x0,
                     base, B, HW);
  return hipGetLastError();
}

hipError_t launch_pack_target(const double *rho, const double *T, double tc, const Norm &nm, float *t,
                              size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_target, dim3(grid_for(n)), dim3(256), 0, s, rho, T, tc, nm, t, n);
  return hipGetLastError();
}

hipError_t launch_unpack(const float *pred, double tc, const Norm &nm, double *rho, double *T, size_t n,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_unpack, dim3(grid_for(n)), dim3(256), 0, s, pred, tc, nm, rho, T, n);
  return hipGetLastError();
}

hipError_t launch_head(const uint16_t *f, int fcs, int fco, const float *base, const float *wh,
                       const float *bh, float *pred, size_t n, int C, hipStream_t s) {
  if (C == 16)
    hipLaunchKernelGGL(k_head<16>, dim3(grid_for(n)), dim3(256), 0, s, f, fcs, fco, base, wh, bh, pred, n);
  else if (C == 32)
    hipLaunchKernelGGL(k_head<32>, dim3(grid_for(n)), dim3(256), 0, s, f, fcs, fco, base, wh, bh, pred, n);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int head_blocks(size_t n) { return (int)((n + kHeadPix - 1) / kHeadPix); }

hipError_t launch_head_loss(const uint16_t *f, int fcs, int fco, const float *base, const float *wh,
                            const float *bh, const float *tg, float *loss, float *dwh, float *dbh,
                            uint16_t *df, int dfcs, int dfco, float *part, size_t n, int C,
                            hipStream_t s) {
  const int nblk = head_blocks(n);
  if (C == 16)
    hipLaunchKernelGGL(k_head_loss<16>, dim3(nblk), dim3(256), 0, s, f, fcs, fco, base, wh, bh, tg, df, dfcs,
                       dfco, part, n);
  else if (C == 32)
    hipLaunchKernelGGL(k_head_loss<32>, dim3(nblk), dim3(256), 0, s, f, fcs, fco, base, wh, bh, tg, df, dfcs,
                       dfco, part, n);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_head_reduce, dim3(1), dim3(256), 0, s, part, nblk, C, n, loss, dwh, dbh);
  return hipGetLastError();
}

hipError_t launch_adam(float *w, uint16_t *w16, const float *g, float *m, float *v, size_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, s, w, w16, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float *src, uint16_t *dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace lbmnn
