// HIP kernels (gfx950) of the fused D2Q9 thermal pseudopotential LB step.
//
// Two kernels carry the step.  The one-step kernel (k_tile, k_batch) is
// described here; the two-step kernel (k_pair, k_pair_batch), which runs the
// same per-node arithmetic twice per launch with the intermediate time
// level in LDS, is described where it is defined.
//
// One step is one launch.  A block of BX lanes covers BX consecutive
// columns: the inner BX-2 lanes own a strip of columns, the two outer lanes
// supply the psi halo.  The block walks a band of rows (a sliding window
// along y; odd bands may walk downwards):
//   - the 18 distributions of the next rows are loaded one coalesced plane
//     at a time, PF rows ahead of use;
//   - the moments of row k+1 give rho and T, psi (Section II.A) goes to a
//     ring of four LDS rows;
//   - row k then reads the 3x3 psi stencil from LDS for the force of
//     Eq. (2)/(4), collides f (Eq. (1)) and g (Eq. (7) or Eq. (24)) and
//     pushes the results to the other buffer (ping-pong), with periodic
//     wrap or bounce-back at walls.
// Each distribution is read once and written once per step; only the psi
// halo (one row per band edge, one column per strip edge) is read twice.
// psi at a node needs the moments of its neighbours at the same time level,
// so an in-place (A-A) update would let one block read neighbour data that
// another block is overwriting; two buffers remove that race at no extra
// HBM traffic.
#include "lbm_device.h"

namespace lbmdev {

// D2Q9 velocity set, Section II.A: rest, E, N, W, S, NE, NW, SW, SE.
struct Q9 {
  static constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
};

template <typename S>
__device__ __host__ constexpr S wgt(int i) {
  return i == 0 ? S(4) / S(9) : (i < 5 ? S(1) / S(9) : S(1) / S(36));
}

// storage type S and arithmetic type C of each storage form: the per-node
// reference form keeps FP32 storage but collides in FP64 (FP64 and FP32
// vector ops issue at the same rate here, and rounding every intermediate
// to FP32 costs an order of magnitude in accuracy at the interfaces)
template <int ST>
struct Prec;
template <>
struct Prec<ST_F64> {
  using S = double;
  using C = double;
};
template <>
struct Prec<ST_F32_GLOBAL> {
  using S = float;
  using C = float;
};
template <>
struct Prec<ST_F32_LOCAL> {
  using S = float;
  using C = double;
};

// 1/x for x > 0 (not denormal): the hardware reciprocal estimate refined by
// two Newton-Raphson steps, e = 1 - x r, r <- r + r e, each of which
// squares the relative error; the result is within an ulp of the correctly
// rounded quotient, in five instructions instead of the ten of the
// correctly rounded division sequence (whose chain is also longer).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// sqrt(s) for s > 0 (not denormal): the hardware reciprocal-square-root
// estimate y, one Goldschmidt step on g = s y ~ sqrt(s) and h = y/2 ~
// 1/(2 sqrt(s)) (r = 1/2 - g h; g <- g + g r, h <- h + h r: both errors
// squared), then a Newton correction of g from the residual s - g^2.
// Within an ulp of the correctly rounded root, without the range scaling
// the general square root needs for denormal and huge arguments.
__device__ __forceinline__ double sqrt_pos(double s) {
  const double y = __builtin_amdgcn_rsq(s);
  double g = s * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, s);
  return fma(d, h, g);
}

__device__ inline double pressure(const Model &m, double rho, double T) {
  if (m.eos == 1) return rho * m.R * T;
  const double eta = 0.25 * m.b * rho;
  const double num = 1.0 + eta + eta * eta - eta * eta * eta;
  const double om = 1.0 - eta;
  return rho * m.R * T * num * recip(om * om * om) - m.a * rho * rho;
}

// psi^2 = 2 (p_EOS - rho c_s^2)/(G c^2); psi clamps to 0 outside the domain.
// ir = 1/rho
__device__ inline void node_psi(const Model &m, double rho, double E, double ir, double &psi,
                                double &s, int &clamped) {
  clamped = 0;
  if (!m.sc_on) {
    psi = 0.0;
    s = 0.0;
    return;
  }
  const double T = m.eos_fixed_T ? m.T_eos : E * m.inv_cv * ir;
  s = (pressure(m, rho, T) - rho * (1.0 / 3.0)) * m.two_over_G;
  if (s > 0.0) {
    psi = sqrt_pos(s);
  } else if (s == 0.0) {
    psi = 0.0;
  } else {
    psi = 0.0;
    clamped = m.count_clamps;
  }
}

// The density reference of a node in ST_F32_LOCAL storage: rho rounded to
// FP32 and then to FP16 (every block that computes a node's rho gets the
// same bits).  The empty asm keeps the two hardware conversions: without it
// the pair of roundings is folded into one FP64-to-FP16 rounding done in
// software, some thirty instructions.
__device__ inline float ref_of(double rho) {
  float f = (float)rho;
  asm volatile("" : "+v"(f));
  return (float)(_Float16)f;
}

// --- buffer addressing: one 32-bit byte offset per lane, plane offsets in SGPRs
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format

struct Bufs {
  __amdgpu_buffer_rsrc_t f, g, ref;
};

template <typename S>
__device__ inline Bufs make_bufs(const void *base, const Model &m) {
  const unsigned long long pb = (unsigned long long)m.plane * sizeof(S);
  Bufs b;
  char *p = (char *)base;
  b.f = __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)(unsigned)m.ref_off, kRsrcWord3);
  b.g = __builtin_amdgcn_make_buffer_rsrc(p + 9 * pb, (short)0, (int)(unsigned)(m.ref_off - 9 * pb),
                                          kRsrcWord3);
  b.ref = __builtin_amdgcn_make_buffer_rsrc(p + m.ref_off, (short)0, (int)(unsigned)m.ref_bytes,
                                            kRsrcWord3);
  return b;
}

__device__ inline float bld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float *) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ inline double bld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double *) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ inline void bst(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}
__device__ inline void bst(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, 0);
}

template <typename S>
struct Row {
  S v[18];
  float rb;  // reference density the stored deviations are taken from
};

template <typename C>
struct Mom {
  double rho, E, ir;  // ir = 1/rho (carried by the two-step kernel only)
  C jx, jy;  // first moment of f
  C sf, sg;  // deviation sums (rho - ref, E - ref * cvT_ref)
};

// Post-collision values of a node: Eq. (1) with the forcing term, and
// Eq. (7) or Eq. (24), with f_eq, g_eq = cv T f_eq and the forcing terms
// expanded in e_i.u and e_i.F (arithmetic in C, on deviations from the
// node's reference):
//   f_i* = (1 - 1/tau_f) f_i + w_i [K_f + e.u (A_f + B_f e.u + 9 k_f e.F) + 3 k_f e.F]
//   g_i* = (1 - 1/tau_g) g_i + w_i [K_g + e.u (A_g + B_g e.u) + k_c e.F]
// A_f = 3 rho/tau_f, B_f = 4.5 rho/tau_f, K_f = (drho - 1.5 rho u.u)/tau_f -
// 3 k_f u.F; A_g, B_g, K_g the same with rho cv T and dE; k_f = 1 -
// 1/(2 tau_f); k_c = (1 - 1/(2 tau_g)) 3 cv T for Eq. (24), 0 for Eq. (7).
// Every term is an explicit fma, so each kernel that uses it rounds alike.
template <typename C>
struct Post {
  C ux, uy, fx, fy, omf, omg, Kf, Af, Bf, kf3, kf9, Kg, Ag, Bg, kc;

  __device__ __forceinline__ void init(const Model &m, double rho, double E, double irho, C jx,
                                       C jy, C dr, C dE, double Fx, double Fy, int treatment) {
    const C rs = (C)rho, Es = (C)E;
    // FP64 arithmetic reuses 1/rho from the psi evaluation; FP32
    // arithmetic divides in FP32
    const C ir = sizeof(C) == sizeof(double) ? (C)irho : C(1) / rs;
    fx = (C)Fx;
    fy = (C)Fy;
    ux = fma(C(0.5), fx, jx) * ir;
    uy = fma(C(0.5), fy, jy) * ir;
    const C uu = fma(ux, ux, uy * uy);
    const C uF = fma(ux, fx, uy * fy);
    const C itf = (C)m.inv_tau_f, itg = (C)m.inv_tau_g, kf = (C)m.kf;
    omf = C(1) - itf;
    omg = C(1) - itg;
    const C tf = itf * rs, tg = itg * Es;
    Af = C(3) * tf;
    Bf = C(4.5) * tf;
    kf3 = C(3) * kf;
    kf9 = C(9) * kf;
    Kf = fma(-kf3, uF, fma(C(-1.5) * tf, uu, itf * dr));
    Ag = C(3) * tg;
    Bg = C(4.5) * tg;
    Kg = fma(C(-1.5) * tg, uu, itg * dE);
    kc = treatment == 1 ? (C)m.kg * (C(3) * Es * ir) : C(0);
  }

  // the two brackets of direction i
  __device__ __forceinline__ void bracket(int i, C &tf, C &tg) const {
    if (i == 0) {
      tf = Kf;
      tg = Kg;
      return;
    }
    const C sx = Q9::ex[i] > 0 ? ux : -ux, sy = Q9::ey[i] > 0 ? uy : -uy;
    const C gx = Q9::ex[i] > 0 ? fx : -fx, gy = Q9::ey[i] > 0 ? fy : -fy;
    const C eu = Q9::ex[i] == 0 ? sy : (Q9::ey[i] == 0 ? sx : sx + sy);
    const C eF = Q9::ex[i] == 0 ? gy : (Q9::ey[i] == 0 ? gx : gx + gy);
    tf = fma(kf3, eF, fma(eu, fma(kf9, eF, fma(Bf, eu, Af)), Kf));
    tg = fma(kc, eF, fma(eu, fma(Bg, eu, Ag), Kg));
  }

  // values relative to the node's own reference
  __device__ __forceinline__ void raw(int i, C fin, C gin, C &fs, C &gs) const {
    C tf, tg;
    bracket(i, tf, tg);
    fs = fma(wgt<C>(i), tf, omf * fin);
    gs = fma(wgt<C>(i), tg, omg * gin);
  }

  // values relative to a reference lower by dd (the node they land in);
  // cvTr converts a density reference to the energy reference
  __device__ __forceinline__ void shifted(int i, C fin, C gin, C dd, C cvTr, C &fo, C &go) const {
    C tf, tg;
    bracket(i, tf, tg);
    fo = fma(wgt<C>(i), tf + dd, omf * fin);
    go = fma(wgt<C>(i), fma(dd, cvTr, tg), omg * gin);
  }
};

__device__ inline long long fd_node(const Model &m, int x, int y, bool &ox, bool &oy);
__device__ inline double dp_dT(const Model &m, double rho);

// div u at node (x, y) by the isotropic central difference
// sum_i w(|e_i|^2) u(x + e_i) . e_i of dense velocity planes, periodic wrap
// or, beyond a wall, the boundary node's velocity reversed (no-slip wall
// halfway out)
__device__ inline double div_u_at(const Model &m, const double *uxa, const double *uya, int x, int y) {
  constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  double du = 0.0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const double w = i < 5 ? 1.0 / 3.0 : 1.0 / 12.0;
    const int xn = x + ex[i], yn = y + ey[i];
    bool ox, oy;
    const long long cn = fd_node(m, xn, yn, ox, oy);
    const double sgn = ((ox && m.wall_x) || (oy && m.wall_y)) ? -1.0 : 1.0;
    du += w * (sgn * uxa[cn] * ex[i] + sgn * uya[cn] * ey[i]);
  }
  return du;
}

template <int BX, typename S>
struct TileLds {
  double psi[4][BX];
  double s[4][BX];
  float rbn[4][BX];  // new per-node references (ST_F32_LOCAL)
  double red[BX];
};

template <int ST, int BX, int MODE, int PF>
__device__ void tile(const Model &m, const void *__restrict__ src_v, void *__restrict__ dst_v,
                     int strip, int y0, int y1, int dir, int nt, int treatment,
                     unsigned long long *clamp_counter, const MomentsOut &mo, TileLds<BX, typename Prec<ST>::S> &L,
                     int block_id) {
  using S = typename Prec<ST>::S;
  using C = typename Prec<ST>::C;
  const Bufs sb = make_bufs<S>(src_v, m);
  const Bufs db = make_bufs<S>(dst_v, m);
  const unsigned pb = (unsigned)(m.plane * (long long)sizeof(S));

  const int lane = threadIdx.x;
  const int nx = m.nx, ny = m.ny, pitch = m.pitch;
  const int x0 = strip * (BX - 2);
  const int nint = min(BX - 2, nx - x0);
  const bool active = lane <= nint + 1;
  const bool inner = lane >= 1 && lane <= nint;
  const int x = x0 - 1 + lane;  // own column (inner lanes)
  int xc = x;                   // column this lane loads: wrapped or mirrored
  if (xc < 0) xc = m.wall_x ? 0 : nx - 1;
  else if (xc >= nx) xc = m.wall_x ? nx - 1 : xc - nx;
  if (!active) xc = 0;          // idle lanes read a valid node and store nothing

  // push targets of an inner lane; -1 marks a wall
  const int xl = x > 0 ? x - 1 : (m.wall_x ? -1 : nx - 1);
  const int xr = x < nx - 1 ? x + 1 : (m.wall_x ? -1 : 0);

  auto map_row = [&](int r) -> int {
    if (r < 0) return m.wall_y ? 0 : r + ny;
    if (r >= ny) return m.wall_y ? ny - 1 : r - ny;
    return r;
  };

  const int n = y1 - y0;
  auto row_of = [&](int k) -> int { return dir > 0 ? y0 + k : y1 - 1 - k; };

  long long clamps = 0;

  auto load_row = [&](int k, Row<S> &d) {
    const unsigned cell = (unsigned)(map_row(row_of(k)) * pitch + xc);
    const unsigned off = cell * (unsigned)sizeof(S);
#pragma unroll
    for (int q = 0; q < 9; ++q) d.v[q] = bld(sb.f, off, (unsigned)q * pb, (S *)nullptr);
#pragma unroll
    for (int q = 0; q < 9; ++q) d.v[9 + q] = bld(sb.g, off, (unsigned)q * pb, (S *)nullptr);
    if (ST == ST_F32_LOCAL) {
      const unsigned rc = (unsigned)(map_row(row_of(k)) * m.rpitch + xc);
      const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(sb.ref, (int)(rc * 2u), 0, 0);
      d.rb = (float)__builtin_bit_cast(_Float16, h);
    }
  };

  // moments and psi of the row held in d; LDS ring slot = row & 3
  auto psi_row = [&](int k, const Row<S> &d, Mom<C> &mm, bool keep) {
    const int slot = row_of(k) & 3;
    double sf, sg;
    if (ST == ST_F32_LOCAL) {
      float a = d.v[0];
#pragma unroll
      for (int q = 1; q < 9; ++q) a += d.v[q];
      float b = d.v[9];
#pragma unroll
      for (int q = 10; q < 18; ++q) b += d.v[q];
      sf = (double)a;
      sg = (double)b;
    } else {
      double a = (double)d.v[0];
#pragma unroll
      for (int q = 1; q < 9; ++q) a += (double)d.v[q];
      double b = (double)d.v[9];
#pragma unroll
      for (int q = 10; q < 18; ++q) b += (double)d.v[q];
      sf = a;
      sg = b;
    }
    const C v1 = (C)d.v[1], v2 = (C)d.v[2], v3 = (C)d.v[3], v4 = (C)d.v[4], v5 = (C)d.v[5],
            v6 = (C)d.v[6], v7 = (C)d.v[7], v8 = (C)d.v[8];
    mm.jx = ((v1 - v3) + (v5 - v6)) + (v8 - v7);
    mm.jy = ((v2 - v4) + (v5 + v6)) - (v7 + v8);
    const double ref = ST == ST_F64 ? 0.0 : (ST == ST_F32_GLOBAL ? m.rho_ref : (double)d.rb);
    mm.sf = (C)sf;
    mm.sg = (C)sg;
    mm.rho = ref + sf;
    mm.E = ref * m.cvT_ref + sg;
    // 1/rho is recomputed at the collision (same bits) rather than carried:
    // two more live registers per row cost this kernel more than a division
    double psi, s;
    int cl;
    node_psi(m, mm.rho, mm.E, recip(mm.rho), psi, s, cl);
    L.psi[slot][lane] = psi;
    L.s[slot][lane] = s;
    if (ST == ST_F32_LOCAL) L.rbn[slot][lane] = ref_of(mm.rho);
    if (keep && inner) clamps += cl;
  };

  double acc[kPartials];
#pragma unroll
  for (int k = 0; k < kPartials; ++k) acc[k] = 0.0;

  auto collide_row = [&](int k, const Row<S> &d, const Mom<C> &mm) {
    if (MODE == MODE_MOMENTS && !inner) return;
    const int r = row_of(k);
    const int c = inner ? lane : 1;  // outer lanes compute on a valid stencil, store nothing
    const double *pm = L.psi[(r - 1) & 3];
    const double *p0 = L.psi[r & 3];
    const double *pp = L.psi[(r + 1) & 3];
    double Fx = 0.0, Fy = 0.0;
    if (m.sc_on) {
      // Eq. (2): w(1) = 1/3 on the axes, w(2) = 1/12 on the diagonals
      const double sx = (p0[c + 1] - p0[c - 1]) * (1.0 / 3.0) +
                        ((pp[c + 1] - pp[c - 1]) + (pm[c + 1] - pm[c - 1])) * (1.0 / 12.0);
      const double sy = (pp[c] - pm[c]) * (1.0 / 3.0) +
                        ((pp[c + 1] + pp[c - 1]) - (pm[c + 1] + pm[c - 1])) * (1.0 / 12.0);
      const double gb = -m.G * m.beta * p0[c];
      Fx = gb * sx;
      Fy = gb * sy;
      if (!m.beta_one) {  // second term of Eq. (4), from psi^2
        const double *qm = L.s[(r - 1) & 3];
        const double *q0 = L.s[r & 3];
        const double *qp = L.s[(r + 1) & 3];
        const double tx2 = (q0[c + 1] - q0[c - 1]) * (1.0 / 3.0) +
                           ((qp[c + 1] - qp[c - 1]) + (qm[c + 1] - qm[c - 1])) * (1.0 / 12.0);
        const double ty2 = (qp[c] - qm[c]) * (1.0 / 3.0) +
                           ((qp[c + 1] + qp[c - 1]) - (qm[c + 1] + qm[c - 1])) * (1.0 / 12.0);
        const double h = -m.G * 0.5 * (1.0 - m.beta);
        Fx += h * tx2;
        Fy += h * ty2;
      }
    }
    Fx += mm.rho * m.gx;
    Fy += mm.rho * m.gy;

    if (MODE == MODE_STEP_FD && inner) {
      // the moments of time t, as a MODE_MOMENTS launch writes them
      const long long o = (long long)r * nx + x;
      mo.rho[o] = mm.rho;
      mo.ux[o] = ((double)mm.jx + 0.5 * Fx) / mm.rho;
      mo.uy[o] = ((double)mm.jy + 0.5 * Fy) / mm.rho;
      mo.T[o] = mm.E * m.inv_cv / mm.rho;
    }

    if (MODE == MODE_MOMENTS) {
      const double ux = ((double)mm.jx + 0.5 * Fx) / mm.rho;
      const double uy = ((double)mm.jy + 0.5 * Fy) / mm.rho;
      const double T = mm.E * m.inv_cv / mm.rho;
      const long long o = (long long)r * nx + x;
      if (mo.rho) mo.rho[o] = mm.rho;
      if (mo.ux) mo.ux[o] = ux;
      if (mo.uy) mo.uy[o] = uy;
      if (mo.T) mo.T[o] = T;
      acc[0] += mm.rho;
      acc[1] += mm.E;
      acc[2] += (double)mm.jx + 0.5 * Fx;
      acc[3] += (double)mm.jy + 0.5 * Fy;
      acc[4] += (isfinite(mm.rho) && isfinite(mm.E)) ? 0.0 : 1.0;
      if (mo.compare_snap) {
        acc[5] = fmax(acc[5], fabs(mm.rho - mo.snap_rho[o]));
        acc[6] = fmax(acc[6], fabs(mm.rho));
        acc[7] = fmax(acc[7], fabs(T - mo.snap_T[o]));
        acc[8] = fmax(acc[8], fabs(T));
      }
      if (mo.write_snap) {
        mo.snap_rho[o] = mm.rho;
        mo.snap_T[o] = T;
      }
      return;
    }

    // collision, Eq. (1) with the forcing term and Eq. (7)/(24), in C, on
    // deviations from the node's own reference
    Post<C> P;
    P.init(m, mm.rho, mm.E, recip(mm.rho), mm.jx, mm.jy, mm.sf, mm.sg, Fx, Fy, treatment);
    if ((MODE == MODE_STEP_SRC || MODE == MODE_STEP_OPEN) && mo.ux) {
      // the source of Eq. (5), w_i phi div u with phi = -T (dp_EOS/dT)_rho,
      // from the velocity planes of time t (lanes owning no column read a
      // valid node and store nothing)
      const double Tn = mm.E * m.inv_cv * recip(mm.rho);
      P.Kg += (C)(-Tn * dp_dT(m, mm.rho) * div_u_at(m, mo.ux, mo.uy, inner ? x : 0, r));
    }
    const C rs = (C)mm.rho, Es = (C)mm.E;
    const C ux = P.ux, uy = P.uy;
    const C uu = ux * ux + uy * uy;
    const float rb_old = ST == ST_F32_LOCAL ? d.rb : 0.0f;
    const float *rn_m = L.rbn[(r - 1) & 3];
    const float *rn_0 = L.rbn[r & 3];
    const float *rn_p = L.rbn[(r + 1) & 3];
    const C cvTr = (C)m.cvT_ref;

    const int rD = r > 0 ? r - 1 : (m.wall_y ? -1 : ny - 1);
    const int rU = r < ny - 1 ? r + 1 : (m.wall_y ? -1 : 0);
    const bool row_wall = rD < 0 || rU < 0;  // uniform over the block
    const unsigned own = (unsigned)(r * pitch + x);
    if (ST == ST_F32_LOCAL)
      __builtin_amdgcn_raw_buffer_store_b16(
          __builtin_bit_cast(unsigned short, (_Float16)rn_0[c]), db.ref,
          (int)((unsigned)(inner ? r * m.rpitch + x : ny * m.rpitch + lane) * 2u), 0, 0);

    constexpr int kx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int ky[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    constexpr int ko[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    // post-collision values of direction i, shifted (ST_F32_LOCAL) to the
    // reference of the node with reference rd they land in
    auto post_to = [&](int i, float rd, C &fs, C &gs) {
      const C fin = (C)d.v[i], gin = (C)d.v[9 + i];
      if (ST == ST_F32_LOCAL) P.shifted(i, fin, gin, (C)(rb_old - rd), cvTr, fs, gs);
      else P.raw(i, fin, gin, fs, gs);
    };
    // Every lane issues the same 18 stores whatever its case, so the next
    // row's loads never wait for a store that sat in a masked branch; a lane
    // that owns no node writes into the unused pad past the end of the
    // plane, at a slot of its own.
    const unsigned dummy = (unsigned)(ny * pitch + lane);
    const unsigned sz = (unsigned)sizeof(S);
    if (!(row_wall || m.wall_x)) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        C fs, gs;
        const float *rr = ky[i] > 0 ? rn_p : (ky[i] < 0 ? rn_m : rn_0);
        post_to(i, ST == ST_F32_LOCAL ? rr[c + kx[i]] : 0.0f, fs, gs);
        const int col = kx[i] > 0 ? xr : (kx[i] < 0 ? xl : x);
        const int row = ky[i] > 0 ? rU : (ky[i] < 0 ? rD : r);
        const unsigned cell = inner ? (unsigned)(row * pitch + col) : dummy;
        bst(db.f, cell * sz, (unsigned)i * pb, (S)fs);  // plane offset in the scalar operand
        if (MODE != MODE_STEP_FD) bst(db.g, cell * sz, (unsigned)i * pb, (S)gs);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int exi = kx[i], eyi = ky[i];
        const int col = exi > 0 ? xr : (exi < 0 ? xl : x);
        const int row = eyi > 0 ? rU : (eyi < 0 ? rD : r);
        const bool stays = col >= 0 && row >= 0;
        const C wi = wgt<C>(i);
        // values in the reference of the node they land in (ST_F32_LOCAL),
        // and relative to the own reference (wall formulas)
        float rd = 0.0f;
        if (ST == ST_F32_LOCAL) {
          const float *rr = eyi > 0 ? rn_p : (eyi < 0 ? rn_m : rn_0);
          rd = stays ? rr[c + exi] : rn_0[c];
        }
        C fo, go, fs, gs;
        post_to(i, rd, fo, go);
        P.raw(i, (C)d.v[i], (C)d.v[9 + i], fs, gs);
        // halfway bounce-back into the same node; Dirichlet walls
        // anti-bounce-back with the wall value rho cv T_w.  A diagonal
        // leaving through a corner of a box meets both walls: adiabatic if
        // either is, else Dirichlet at the mean wall temperature (no axis
        // preferred); at a corner of the open channel the plate's rule holds
        const bool hy = row < 0;
        const int ky = eyi < 0 ? 2 : 3, kx = exi < 0 ? 0 : 1;
        int th = hy ? m.thermal[ky] : m.thermal[kx];
        double wE = hy ? m.wall_E[ky] : m.wall_E[kx];
        if (hy && col < 0 && m.wall_x == 1) {
          th = (m.thermal[kx] != 0 || m.thermal[ky] != 0) ? 1 : 0;
          wE = 0.5 * (m.wall_E[kx] + m.wall_E[ky]);
        }
        const double refE = ST == ST_F64 ? 0.0
                            : (ST == ST_F32_GLOBAL ? m.rho_ref * m.cvT_ref
                                                   : (double)rb_old * m.cvT_ref);
        const double refEn = ST == ST_F64 ? 0.0
                             : (ST == ST_F32_GLOBAL ? m.rho_ref * m.cvT_ref
                                                    : (double)rn_0[c] * m.cvT_ref);
        const C g_abb = -gs + wi * (C)(2.0 * mm.rho * wE - refE - refEn);
        C g_out = (stays || th != 0) ? go : g_abb;
        C f_out = fo;
        if (MODE == MODE_STEP_OPEN && m.wall_x == 2 && !stays && !hy) {
          const double refF = ST == ST_F64 ? 0.0 : (ST == ST_F32_GLOBAL ? m.rho_ref : (double)rb_old);
          const double refFn = ST == ST_F64 ? 0.0 : (ST == ST_F32_GLOBAL ? m.rho_ref : (double)rn_0[c]);
          if (exi > 0) {
            // outlet: density rho_out, the node's own velocity and energy
            const C eu = C(exi) * ux + C(eyi) * uy;
            const C even = C(1) + C(4.5) * eu * eu - C(1.5) * uu;
            f_out = -fs + wi * (C(2) * (C)m.rho_out * even - (C)(refF + refFn));
            g_out = -gs + wi * (C(2) * Es * even - (C)(refE + refEn));
          } else {
            // inlet: bounce-back carrying the inlet momentum; Dirichlet g
            // with the inlet equilibrium's even part
            const C eui = C(exi) * (C)m.u_in;
            f_out = fo - C(6) * wi * rs * eui;
            if (th == 0)
              g_out = -gs + wi * (C)(2.0 * mm.rho * wE * (1.0 + 3.0 * m.u_in * m.u_in) - refE - refEn);
          }
        }
        const unsigned q = stays ? (unsigned)i : (unsigned)ko[i];
        const unsigned cell = !inner ? dummy : (stays ? (unsigned)(row * pitch + col) : own);
        bst(db.f, cell * sz + q * pb, 0u, (S)f_out);
        if (MODE != MODE_STEP_FD) bst(db.g, cell * sz + q * pb, 0u, (S)g_out);
      }
    }
  };

  if (PF >= 2 && MODE != MODE_MOMENTS) {
    // PF + 1 row buffers in rotating roles: at row k the buffers hold rows
    // k (collide), k + 1 (psi) and k + 2 .. k + PF (loads in flight).  The
    // loop is unrolled over a full rotation so that every buffer index is a
    // constant and no loaded register is ever copied (a copy would wait for
    // the load in flight).
    // the moments of a row are kept from its psi evaluation to its
    // collision in two alternating slots; the unrolled span covers whole
    // rotations of both
    constexpr int NB = PF + 1;
    constexpr int SPAN = (NB % 2) ? 2 * NB : NB;
    Row<S> R[NB];
    Mom<C> M[2];
    load_row(-1, R[NB - 1]);
#pragma unroll
    for (int j = 0; j < PF; ++j) load_row(j, R[j]);
    psi_row(-1, R[NB - 1], M[1], false);
    psi_row(0, R[0], M[0], true);
    for (int k = 0; k < n; k += SPAN) {
#pragma unroll
      for (int j = 0; j < SPAN; ++j) {
        const int kk = k + j;
        if (kk < n) {
          // unconditional look-ahead: past the band it re-reads the band's
          // last (halo) row, which an earlier iteration left in cache
          load_row(min(kk + PF, n), R[(j + PF) % NB]);
          psi_row(kk + 1, R[(j + 1) % NB], M[(j + 1) & 1], kk + 1 < n);
          __syncthreads();
          collide_row(kk, R[j % NB], M[j & 1]);
        }
      }
    }
  } else {
    Row<S> R0, R1;
    Mom<C> M0, M1;
    load_row(-1, R1);
    psi_row(-1, R1, M1, false);
    load_row(0, R0);
    psi_row(0, R0, M0, true);
    auto iter = [&](int k, const Row<S> &cur, const Mom<C> &mc, Row<S> &nxt, Mom<C> &mn) {
      load_row(k + 1, nxt);
      psi_row(k + 1, nxt, mn, k + 1 < n);
      __syncthreads();
      collide_row(k, cur, mc);
    };
    for (int k = 0; k < n; k += 2) {
      iter(k, R0, M0, R1, M1);
      if (k + 1 < n) iter(k + 1, R1, M1, R0, M0);
    }
  }

  if (clamps && clamp_counter) atomicAdd(clamp_counter, (unsigned long long)clamps);

  if (MODE == MODE_MOMENTS && mo.partials) {
    // fixed-order block reduction of the per-lane partials
    for (int k = 0; k < kPartials; ++k) {
      __syncthreads();
      L.red[lane] = acc[k];
      __syncthreads();
      for (int w = BX / 2; w > 0; w >>= 1) {
        if (lane < w) L.red[lane] = (k >= 5) ? fmax(L.red[lane], L.red[lane + w]) : L.red[lane] + L.red[lane + w];
        __syncthreads();
      }
      if (lane == 0) mo.partials[(long long)block_id * kPartials + k] = L.red[0];
    }
  }
}

// block -> tile: with t.xcd the grid (a multiple of 8) is dealt so that the
// blocks landing on one XCD (round-robin dispatch) get consecutive tiles,
// i.e. neighbouring bands, whose halo rows then meet in that XCD's L2.
__device__ inline int tile_of_block(const Tiling &t) {
  const int b = blockIdx.x;
  if (!t.xcd) return b;
  const int per = (int)gridDim.x >> 3;
  return (b & 7) * per + (b >> 3);
}

template <int ST, int BX, int MODE, int PF>
__global__ __launch_bounds__(BX) void k_tile(Model m, Tiling t, const void *__restrict__ src,
                                             void *__restrict__ dst, int treatment,
                                             unsigned long long *clamp_counter, MomentsOut mo) {
  __shared__ TileLds<BX, typename Prec<ST>::S> L;
  const int tid = tile_of_block(t);
  if (tid >= t.strips * t.bands) return;
  const int strip = tid % t.strips;
  const int band = tid / t.strips;
  const int y0 = band * t.rows;
  const int y1 = min(y0 + t.rows, m.ny);
  const int dir = (t.alt && (band & 1)) ? -1 : 1;
  tile<ST, BX, MODE, PF>(m, src, dst, strip, y0, y1, dir, t.nt, treatment, clamp_counter, mo, L,
                         tid);
}

template <int ST, int BX, int PF>
__global__ __launch_bounds__(BX) void k_batch(BatchTables bt, char *__restrict__ base, int parity,
                                              int treatment) {
  __shared__ TileLds<BX, typename Prec<ST>::S> L;
  int tid = blockIdx.x;
  if (bt.xcd) {
    const int per = (int)gridDim.x >> 3;
    tid = (tid & 7) * per + (tid >> 3);
  }
  if (tid >= bt.ntiles) return;
  const BatchTile t = bt.tiles[tid];
  const Model m = bt.models[t.lattice];
  const int sb = parity ^ bt.phase[t.lattice];
  char *src = base + (sb ? bt.off1[t.lattice] : bt.off0[t.lattice]);
  char *dst = base + (sb ? bt.off0[t.lattice] : bt.off1[t.lattice]);
  const int y0 = t.band * t.rows;
  const int y1 = min(y0 + t.rows, m.ny);
  MomentsOut mo{};
  tile<ST, BX, MODE_STEP, PF>(m, src, dst, t.strip, y0, y1, t.dir, 0, treatment, bt.clamp[t.lattice],
                              mo, L, tid);
}

// ---------------------------------------------------------------------------
// Two time steps per launch (temporal blocking along the band).
//
// On lattices periodic in x, with the force of Eq. (2) alone, one launch
// advances the state by two steps and the distributions of the
// intermediate time level never reach HBM, which halves the HBM traffic per
// step.  A block of BX lanes covers BX consecutive columns; the
// inner BX - 6 lanes own a strip, and three halo columns per side supply
// psi of the first step, the first step's pushes into the owned columns'
// neighbours and psi of the second step.  At iteration j the block
//   - takes the moments and psi of the first step on row j       (ring psi1),
//   - takes the moments and psi of the second step on row j - 3, whose
//     first-step distributions became complete with the pushes of row j - 2
//     (ring psi2; the distributions are kept in registers),
//   - collides row j - 1 (first step) and pushes the results into an LDS
//     ring of three rows (in the storage precision),
//   - moves row j + 1 into place and loads row j + 2 into a spare register
//     row,
//   - collides row j - 4 (second step) and pushes the results to HBM with
//     the same stores as the one-step kernel.
// Rows are counted from three rows below the band (j = 0) to three rows
// above it; at y walls rows outside the lattice are not collided and the
// second step's psi ghost rows mirror the wall rows, as in the one-step
// kernel.  The arithmetic of each step is the one-step kernel's (the shared
// collision is written in explicit FMAs), on the same stored values, so two
// one-step launches and one two-step launch give the same result bit for
// bit.

template <int BX, typename S, bool MIX>
struct PairLds {
  S f1[3][18][BX];      // distributions after the first step, stored form
  double psi1[4][BX];
  double psi2[4][BX];
  float rb1[4][BX];     // per-node references after the first step (ST_F32_LOCAL)
  float rb2[4][BX];     // and after the second
  double s1[4][MIX ? BX : 1];  // psi^2 for the second term of Eq. (4)
  double s2[4][MIX ? BX : 1];
};

// two steps on the strip whose owned columns start at x0 and rows
// y0 .. y0 + n - 1 of one lattice.  The block's lanes form strips of sw
// lanes (sw = BX, or 64: each wave its own strip of 58 owned columns, used
// for the last columns of narrow lattices in a batch); each strip keeps to
// its own lanes of the LDS rings.  jb = iterations every wave of the block
// runs (the block's barriers), at least n + 7; a wave past its own n + 7
// only keeps the barriers.  (MIX: the lattice uses the mixed force of
// Eq. (4), beta != 1)
template <int ST, int BX, bool MIX>
__device__ void pair_tile(const Model &m, const void *__restrict__ src_v, void *__restrict__ dst_v,
                          int x0, int sw, int y0, int n, int jb, int treatment,
                          unsigned long long *clamp_counter, PairLds<BX, typename Prec<ST>::S, MIX> &L) {
  using S = typename Prec<ST>::S;
  using C = typename Prec<ST>::C;
  const Bufs sb = make_bufs<S>(src_v, m);
  const Bufs db = make_bufs<S>(dst_v, m);
  const unsigned pb = (unsigned)(m.plane * (long long)sizeof(S));
  constexpr unsigned sz = sizeof(S);

  const int lane = threadIdx.x;          // index into the LDS rings
  const int ll = lane & (sw - 1);          // lane within its strip
  const int lane0 = lane - ll;             // the strip's first lane
  const int nx = m.nx, ny = m.ny, pitch = m.pitch;
  const int nint = min(sw - 6, nx - x0);
  const bool active = ll < nint + 6;
  const bool own = ll >= 3 && ll < nint + 3;  // owns its column
  // a wave with no active lane (the last strip of a lattice, or no band)
  // only keeps the block's barriers
  const bool wave_live = (ll & ~63) < nint + 6 && n > 0;
  auto wrap = [](int v, int len) {
    const int r = v % len;
    return r < 0 ? r + len : r;
  };
  const int x = active ? wrap(x0 - 3 + ll, nx) : 0;
  const int xl = wrap(x - 1, nx), xr = wrap(x + 1, nx);
  // stencil centre in a ring row, inside the strip's lanes
  const int c = (ll >= 1 && ll <= sw - 2) ? lane : lane0 + 1;

  auto vrow = [&](int j) { return y0 - 3 + j; };
  auto inside = [&](int v) { return !m.wall_y || (v >= 0 && v < ny); };
  auto prow = [&](int v) { return m.wall_y ? min(max(v, 0), ny - 1) : wrap(v, ny); };

  long long clamps = 0;
  const C cvTr = (C)m.cvT_ref;

  auto load_row = [&](int j, Row<S> &d) {
    const int r = prow(vrow(j));
    const unsigned off = (unsigned)(r * pitch + x) * sz;
#pragma unroll
    for (int q = 0; q < 9; ++q) d.v[q] = bld(sb.f, off, (unsigned)q * pb, (S *)nullptr);
#pragma unroll
    for (int q = 0; q < 9; ++q) d.v[9 + q] = bld(sb.g, off, (unsigned)q * pb, (S *)nullptr);
    if (ST == ST_F32_LOCAL) {
      const unsigned rc = (unsigned)(r * m.rpitch + x);
      const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(sb.ref, (int)(rc * 2u), 0, 0);
      d.rb = (float)__builtin_bit_cast(_Float16, h);
    }
  };

  auto load_f1 = [&](int j, Row<S> &d) {
    const S *f = &L.f1[j % 3][0][0];
#pragma unroll
    for (int q = 0; q < 18; ++q) d.v[q] = f[q * BX + lane];
    if (ST == ST_F32_LOCAL) d.rb = L.rb1[j & 3][lane];
  };

  // rho, j, E of the stored values; the deviation sums in the one-step
  // kernel's precision (FP32 for per-node references, else FP64)
  auto moments = [&](const Row<S> &d, Mom<C> &mm) {
    double a, b;
    if (ST == ST_F32_LOCAL) {
      float fa = d.v[0];
#pragma unroll
      for (int q = 1; q < 9; ++q) fa += d.v[q];
      float fb = d.v[9];
#pragma unroll
      for (int q = 10; q < 18; ++q) fb += d.v[q];
      a = (double)fa;
      b = (double)fb;
    } else {
      a = (double)d.v[0];
#pragma unroll
      for (int q = 1; q < 9; ++q) a += (double)d.v[q];
      b = (double)d.v[9];
#pragma unroll
      for (int q = 10; q < 18; ++q) b += (double)d.v[q];
    }
    const C v1 = (C)d.v[1], v2 = (C)d.v[2], v3 = (C)d.v[3], v4 = (C)d.v[4], v5 = (C)d.v[5],
            v6 = (C)d.v[6], v7 = (C)d.v[7], v8 = (C)d.v[8];
    mm.jx = ((v1 - v3) + (v5 - v6)) + (v8 - v7);
    mm.jy = ((v2 - v4) + (v5 + v6)) - (v7 + v8);
    const double ref = ST == ST_F64 ? 0.0 : (ST == ST_F32_GLOBAL ? m.rho_ref : (double)d.rb);
    mm.sf = (C)a;
    mm.sg = (C)b;
    mm.rho = ref + a;
    mm.E = ref * m.cvT_ref + b;
    mm.ir = recip(mm.rho);
  };

  // force of Eq. (2), or of Eq. (4) with the psi^2 rings (MIX), from the
  // rings' rows j - 1, j, j + 1, plus the body force
  auto force = [&](const double (*ring)[BX], const double (*sring)[MIX ? BX : 1], int j,
                   double rho, double &Fx, double &Fy) {
    const double *pm = ring[(j - 1) & 3], *p0 = ring[j & 3], *pp = ring[(j + 1) & 3];
    Fx = 0.0;
    Fy = 0.0;
    if (m.sc_on) {
      const double sx = (p0[c + 1] - p0[c - 1]) * (1.0 / 3.0) +
                        ((pp[c + 1] - pp[c - 1]) + (pm[c + 1] - pm[c - 1])) * (1.0 / 12.0);
      const double sy = (pp[c] - pm[c]) * (1.0 / 3.0) +
                        ((pp[c + 1] + pp[c - 1]) - (pm[c + 1] + pm[c - 1])) * (1.0 / 12.0);
      const double gb = -m.G * m.beta * p0[c];
      Fx = gb * sx;
      Fy = gb * sy;
      if (MIX && !m.beta_one) {  // second term of Eq. (4), from psi^2
        const double *qm = sring[(j - 1) & 3], *q0 = sring[j & 3], *qp = sring[(j + 1) & 3];
        const double tx2 = (q0[c + 1] - q0[c - 1]) * (1.0 / 3.0) +
                           ((qp[c + 1] - qp[c - 1]) + (qm[c + 1] - qm[c - 1])) * (1.0 / 12.0);
        const double ty2 = (qp[c] - qm[c]) * (1.0 / 3.0) +
                           ((qp[c + 1] + qp[c - 1]) - (qm[c + 1] + qm[c - 1])) * (1.0 / 12.0);
        const double h = -m.G * 0.5 * (1.0 - m.beta);
        Fx += h * tx2;
        Fy += h * ty2;
      }
    }
    Fx += rho * m.gx;
    Fy += rho * m.gy;
  };

  // post-collision values of direction i in the reference rd of the node
  // they land in (ST_F32_LOCAL), and relative to the own reference
  auto post_to = [&](const Post<C> &P, const Row<S> &d, int i, float rd, C &fo, C &go) {
    const C fin = (C)d.v[i], gin = (C)d.v[9 + i];
    if (ST == ST_F32_LOCAL) P.shifted(i, fin, gin, (C)(d.rb - rd), cvTr, fo, go);
    else P.raw(i, fin, gin, fo, go);
  };

  // anti-bounce-back value of g at a Dirichlet y wall, from the value gs
  // relative to the own reference before the step (rb_old) and the own
  // reference after it (rb_new)
  auto g_wall = [&](int i, C gs, double rho, float rb_old, float rb_new) {
    const double wE = Q9::ey[i] < 0 ? m.wall_E[2] : m.wall_E[3];
    const double refE = ST == ST_F64 ? 0.0
                        : (ST == ST_F32_GLOBAL ? m.rho_ref * m.cvT_ref : (double)rb_old * m.cvT_ref);
    const double refEn = ST == ST_F64 ? 0.0
                         : (ST == ST_F32_GLOBAL ? m.rho_ref * m.cvT_ref : (double)rb_new * m.cvT_ref);
    return -gs + wgt<C>(i) * (C)(2.0 * rho * wE - refE - refEn);
  };

  auto psi_first = [&](int j, const Row<S> &d, Mom<C> &mm) {
    moments(d, mm);
    double psi, s;
    int cl;
    node_psi(m, mm.rho, mm.E, mm.ir, psi, s, cl);
    L.psi1[j & 3][lane] = psi;
    if (MIX) L.s1[j & 3][lane] = s;
    if (ST == ST_F32_LOCAL) L.rb1[j & 3][lane] = ref_of(mm.rho);
    const int v = vrow(j);
    if (own && v >= y0 && v < y0 + n) clamps += cl;
  };

  auto psi_second = [&](int j, Row<S> &d, Mom<C> &mm) {
    load_f1(j, d);
    moments(d, mm);
    double psi, s;
    int cl;
    node_psi(m, mm.rho, mm.E, mm.ir, psi, s, cl);
    const int v = vrow(j);
    L.psi2[j & 3][lane] = psi;
    if (MIX) L.s2[j & 3][lane] = s;
    if (ST == ST_F32_LOCAL) L.rb2[j & 3][lane] = ref_of(mm.rho);
    if (m.wall_y && v == 0) {  // mirror ghost rows
      L.psi2[(j - 1) & 3][lane] = psi;
      if (MIX) L.s2[(j - 1) & 3][lane] = s;
    }
    if (m.wall_y && v == ny - 1) {
      L.psi2[(j + 1) & 3][lane] = psi;
      if (MIX) L.s2[(j + 1) & 3][lane] = s;
    }
    if (own && v >= y0 && v < y0 + n) clamps += cl;
  };

  // first step of row j: pushes into the LDS ring (bounce-back at y walls)
  auto collide_first = [&](int j, const Row<S> &d, const Mom<C> &mm) {
    const int v = vrow(j);
    double Fx, Fy;
    force(L.psi1, L.s1, j, mm.rho, Fx, Fy);
    Post<C> P;
    P.init(m, mm.rho, mm.E, mm.ir, mm.jx, mm.jy, mm.sf, mm.sg, Fx, Fy, treatment);
    const float *rn_m = L.rb1[(j - 1) & 3];
    const float *rn_0 = L.rb1[j & 3];
    const float *rn_p = L.rb1[(j + 1) & 3];
    const bool wd = m.wall_y && v == 0, wu = m.wall_y && v == ny - 1;
    S *fm = &L.f1[(j + 2) % 3][0][0];
    S *f0 = &L.f1[j % 3][0][0];
    S *fp = &L.f1[(j + 1) % 3][0][0];
    // every lane stores: the lanes that do not collide in this step (the
    // two edges of the block) write inside the ring row, into entries that
    // no owned column reads
    const int tl = ll > 0 ? lane - 1 : lane, tr = ll < sw - 1 ? lane + 1 : lane;
    auto push = [&](int i, C fo, C go) {
      const int exi = Q9::ex[i], eyi = Q9::ey[i];
      S *f = eyi > 0 ? fp : (eyi < 0 ? fm : f0);
      const int to = exi > 0 ? tr : (exi < 0 ? tl : lane);
      f[i * BX + to] = (S)fo;
      f[(9 + i) * BX + to] = (S)go;
    };
    {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int exi = Q9::ex[i], eyi = Q9::ey[i];
        const bool hy = (eyi < 0 && wd) || (eyi > 0 && wu);
        float rd = 0.0f;
        if (ST == ST_F32_LOCAL) {
          const float *rr = eyi > 0 ? rn_p : (eyi < 0 ? rn_m : rn_0);
          rd = hy ? rn_0[c] : rr[c + exi];
        }
        C fo, go;
        post_to(P, d, i, rd, fo, go);
        if (!hy) {
          push(i, fo, go);
        } else {
          C fs, gs;
          P.raw(i, (C)d.v[i], (C)d.v[9 + i], fs, gs);
          const int th = eyi < 0 ? m.thermal[2] : m.thermal[3];
          const C g_out = th != 0 ? go : g_wall(i, gs, mm.rho, d.rb, rd);
          f0[Q9::opp[i] * BX + lane] = (S)fo;
          f0[(9 + Q9::opp[i]) * BX + lane] = (S)g_out;
        }
      }
    }
  };

  // second step of row j: pushes to HBM; every lane issues the same stores
  // (lanes that own no column write into the pad past the plane)
  auto collide_second = [&](int j, const Row<S> &d, const Mom<C> &mm) {
    const int r = vrow(j);
    double Fx, Fy;
    force(L.psi2, L.s2, j, mm.rho, Fx, Fy);
    Post<C> P;
    P.init(m, mm.rho, mm.E, mm.ir, mm.jx, mm.jy, mm.sf, mm.sg, Fx, Fy, treatment);
    const float *rn_m = L.rb2[(j - 1) & 3];
    const float *rn_0 = L.rb2[j & 3];
    const float *rn_p = L.rb2[(j + 1) & 3];
    const int rD = r > 0 ? r - 1 : (m.wall_y ? -1 : ny - 1);
    const int rU = r < ny - 1 ? r + 1 : (m.wall_y ? -1 : 0);
    const unsigned dummy = (unsigned)(ny * pitch + lane);
    const unsigned self = own ? (unsigned)(r * pitch + x) : dummy;
    if (ST == ST_F32_LOCAL)
      __builtin_amdgcn_raw_buffer_store_b16(
          __builtin_bit_cast(unsigned short, (_Float16)rn_0[c]), db.ref,
          (int)((unsigned)(own ? r * m.rpitch + x : ny * m.rpitch + lane) * 2u), 0, 0);
    if (rD >= 0 && rU >= 0) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int col = Q9::ex[i] > 0 ? xr : (Q9::ex[i] < 0 ? xl : x);
        const int row = Q9::ey[i] > 0 ? rU : (Q9::ey[i] < 0 ? rD : r);
        float rd = 0.0f;
        if (ST == ST_F32_LOCAL) {
          const float *rr = Q9::ey[i] > 0 ? rn_p : (Q9::ey[i] < 0 ? rn_m : rn_0);
          rd = rr[c + Q9::ex[i]];
        }
        C f_out, g_out;
        post_to(P, d, i, rd, f_out, g_out);
        const unsigned cell = own ? (unsigned)(row * pitch + col) : dummy;
        bst(db.f, cell * sz, (unsigned)i * pb, (S)f_out);  // plane offset in the scalar operand
        bst(db.g, cell * sz, (unsigned)i * pb, (S)g_out);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int exi = Q9::ex[i], eyi = Q9::ey[i];
        const int col = exi > 0 ? xr : (exi < 0 ? xl : x);
        const int row = eyi > 0 ? rU : (eyi < 0 ? rD : r);
        const bool stays = row >= 0;
        float rd = 0.0f;
        if (ST == ST_F32_LOCAL) {
          const float *rr = eyi > 0 ? rn_p : (eyi < 0 ? rn_m : rn_0);
          rd = stays ? rr[c + exi] : rn_0[c];
        }
        C f_out, g_out;
        post_to(P, d, i, rd, f_out, g_out);
        unsigned q = (unsigned)i, cell = own ? (unsigned)(row * pitch + col) : dummy;
        if (!stays) {
          const int th = eyi < 0 ? m.thermal[2] : m.thermal[3];
          if (th == 0) {
            C fs, gs;
            P.raw(i, (C)d.v[i], (C)d.v[9 + i], fs, gs);
            g_out = g_wall(i, gs, mm.rho, d.rb, rd);
          }
          q = (unsigned)Q9::opp[i];
          cell = self;
        }
        bst(db.f, cell * sz, q * pb, (S)f_out);  // q depends on the row only: uniform
        bst(db.g, cell * sz, q * pb, (S)g_out);
      }
    }
  };

  // the pipeline; register buffers alternate with the parity of j
  // P holds the row after next: loaded an iteration before it is copied
  // into its R slot, so a load has a whole iteration to arrive (the copy
  // is 19 moves; loading into R directly would leave half an iteration)
  Row<S> R[2], F[2], P;
  Mom<C> M[2], M2[2];
  // every stage below is guarded by n, so iterations past n + 7 do nothing
  const int J = jb;
  if (wave_live) {
    load_row(0, R[0]);
    load_row(1, P);
  }
  for (int j0 = 0; j0 < J; j0 += 2) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int j = j0 + u;
      if (j < J) {
        if (wave_live) {
          if (j < n + 6) psi_first(j, R[u], M[u]);
          const int j2 = j - 3;
          if (j2 >= 2 && j2 < n + 4 && inside(vrow(j2))) psi_second(j2, F[u ^ 1], M2[u ^ 1]);
        }
        __syncthreads();
        if (wave_live) {
          const int j1 = j - 1;
          if (j1 >= 1 && j1 < n + 5 && inside(vrow(j1))) collide_first(j1, R[u ^ 1], M[u ^ 1]);
          if (j + 1 < n + 6) R[u ^ 1] = P;
          if (j + 2 < n + 6) load_row(j + 2, P);
          const int j4 = j - 4;
          if (j4 >= 3 && j4 < n + 3) collide_second(j4, F[u], M2[u]);
        }
        __syncthreads();
      }
    }
  }
  if (clamps && clamp_counter) atomicAdd(clamp_counter, (unsigned long long)clamps);
}

template <int ST, int BX, bool MIX>
__global__ __launch_bounds__(BX) void k_pair(Model m, Tiling t, const void *__restrict__ src,
                                             void *__restrict__ dst, int treatment,
                                             unsigned long long *clamp_counter) {
  __shared__ PairLds<BX, typename Prec<ST>::S, MIX> L;
  const int tid = tile_of_block(t);
  if (tid >= t.strips * t.bands) return;
  const int strip = tid % t.strips;
  // t.bands bands over ny rows, heights differing by at most one row and
  // the taller ones spread evenly (consecutive tiles share an XCD)
  const int band = tid / t.strips;
  const int y0 = (int)((long long)band * m.ny / t.bands);
  const int y1 = (int)((long long)(band + 1) * m.ny / t.bands);
  pair_tile<ST, BX, MIX>(m, src, dst, strip * (BX - 6), BX, y0, y1 - y0, y1 - y0 + 7, treatment,
                         clamp_counter, L);
}

// Two steps of many lattices: one block per tile of the pair tile list
// (strips of BX - 6 owned columns).
template <int ST, int BX, bool MIX>
__global__ __launch_bounds__(BX) void k_pair_batch(BatchTables bt, char *__restrict__ base,
                                                   int parity, int treatment) {
  __shared__ PairLds<BX, typename Prec<ST>::S, MIX> L;
  int tid = blockIdx.x;
  if (bt.xcd) {
    const int per = (int)gridDim.x >> 3;
    tid = (tid & 7) * per + (tid >> 3);
  }
  if (tid >= bt.ntiles) return;
  const BatchTile t = bt.tiles[tid];
  if (t.lattice < 0) return;  // padding of an XCD's run
  const Model m = bt.models[t.lattice];
  const int sb = parity ^ bt.phase[t.lattice];
  char *src = base + (sb ? bt.off1[t.lattice] : bt.off0[t.lattice]);
  char *dst = base + (sb ? bt.off0[t.lattice] : bt.off1[t.lattice]);
  // a full strip of BX lanes over band t.band; or (t.halves) the last
  // columns of a narrow lattice (at most 58), one wave's strip per band: the
  // first wave band t.band, the second t.band2 (none when negative), the
  // block running the longer band's iterations
  const int na = min(t.band * t.rows + t.rows, m.ny) - t.band * t.rows;
  int sw = BX, band = t.band, n = na, jb = na + 7;
  if (t.halves) {
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nb = t.band2 >= 0 ? min(t.band2 * t.rows + t.rows, m.ny) - t.band2 * t.rows : 0;
    sw = 64;
    band = w == 0 ? t.band : max(t.band2, 0);
    n = w == 0 ? na : nb;
    jb = max(na, nb) + 7;
  }
  pair_tile<ST, BX, MIX>(m, src, dst, t.strip * (BX - 6), sw, band * t.rows, n, jb, treatment,
                         bt.clamp[t.lattice], L);
}

// ---------------------------------------------------------------------------

template <int ST>
__global__ void k_init(Model m, void *__restrict__ dst_v, const double *__restrict__ rho,
                       const double *__restrict__ ux, const double *__restrict__ uy,
                       const double *__restrict__ T) {
  using S = typename Prec<ST>::S;
  S *dst = (S *)dst_v;
  _Float16 *ref = (_Float16 *)((char *)dst_v + ref_plane_offset(m, ST));
  const long long n = (long long)m.nx * m.ny;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int x = (int)(c % m.nx), y = (int)(c / m.nx);
  const double r = rho[c];
  const double u = ux ? ux[c] : 0.0, v = uy ? uy[c] : 0.0;
  const double cvT = m.cv * T[c];
  const double uu = u * u + v * v;
  const long long idx = (long long)y * m.pitch + x;
  double rf = 0.0;
  if (ST == ST_F32_GLOBAL) rf = m.rho_ref;
  if (ST == ST_F32_LOCAL) {
    rf = (double)ref_of(r);
    ref[(long long)y * m.rpitch + x] = (_Float16)(float)rf;
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double eu = Q9::ex[i] * u + Q9::ey[i] * v;
    const double w = wgt<double>(i);
    const double feq = r * w * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    dst[i * m.plane + idx] = (S)(feq - w * rf);
    dst[(9 + i) * m.plane + idx] = (S)(cvT * feq - w * rf * m.cvT_ref);
  }
}

template <int ST>
__global__ void k_plane_to(Model m, const void *__restrict__ src_v, int q, double *__restrict__ out) {
  using S = typename Prec<ST>::S;
  const S *src = (const S *)src_v;
  const _Float16 *ref = (const _Float16 *)((const char *)src_v + ref_plane_offset(m, ST));
  const long long n = (long long)m.nx * m.ny;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int x = (int)(c % m.nx), y = (int)(c / m.nx);
  const long long idx = (long long)y * m.pitch + x;
  const int i = q < 9 ? q : q - 9;
  double rf = ST == ST_F64 ? 0.0
                           : (ST == ST_F32_GLOBAL ? m.rho_ref : (double)(float)ref[(long long)y * m.rpitch + x]);
  if (q >= 9) rf *= m.cvT_ref;
  out[c] = (double)src[q * m.plane + idx] + wgt<double>(i) * rf;
}

template <int ST>
__global__ void k_plane_from(Model m, void *__restrict__ dst_v, int q, const double *__restrict__ in) {
  using S = typename Prec<ST>::S;
  S *dst = (S *)dst_v;
  const _Float16 *ref = (const _Float16 *)((const char *)dst_v + ref_plane_offset(m, ST));
  const long long n = (long long)m.nx * m.ny;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int x = (int)(c % m.nx), y = (int)(c / m.nx);
  const long long idx = (long long)y * m.pitch + x;
  const int i = q < 9 ? q : q - 9;
  double rf = ST == ST_F64 ? 0.0
                           : (ST == ST_F32_GLOBAL ? m.rho_ref : (double)(float)ref[(long long)y * m.rpitch + x]);
  if (q >= 9) rf *= m.cvT_ref;
  dst[q * m.plane + idx] = (S)(in[c] - wgt<double>(i) * rf);
}

// reference plane of ST_F32_LOCAL from a dense FP64 density field
__global__ void k_ref_from_rho(Model m, void *__restrict__ dst_v, const double *__restrict__ rho) {
  _Float16 *ref = (_Float16 *)((char *)dst_v + ref_plane_offset(m, ST_F32_LOCAL));
  const long long n = (long long)m.nx * m.ny;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int x = (int)(c % m.nx), y = (int)(c / m.nx);
  ref[(long long)y * m.rpitch + x] = (_Float16)ref_of(rho[c]);
}

// Reduces the per-block partials (sums for entries 0-4, maxima for the
// rest) in one pass: each lane folds a strided set of blocks, the waves
// fold their lanes by butterfly shuffles, and the first lanes fold the four
// waves in a fixed order (the result is reproducible run to run).
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partials, int nblocks,
                                                  double *__restrict__ out) {
  __shared__ double red[kPartials][4];
  const int tx = threadIdx.x, lane = tx & 63, w = tx >> 6;
  double a[kPartials];
#pragma unroll
  for (int k = 0; k < kPartials; ++k) a[k] = 0.0;
  for (int b = tx; b < nblocks; b += 256) {
    const double *p = partials + (long long)b * kPartials;
#pragma unroll
    for (int k = 0; k < kPartials; ++k) a[k] = k >= 5 ? fmax(a[k], p[k]) : a[k] + p[k];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int k = 0; k < kPartials; ++k) {
      const double v = __shfl_xor(a[k], o, 64);
      a[k] = k >= 5 ? fmax(a[k], v) : a[k] + v;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kPartials; ++k) red[k][w] = a[k];
  }
  __syncthreads();
  if (tx < kPartials) {
    const int k = tx;
    out[k] = k >= 5 ? fmax(fmax(red[k][0], red[k][1]), fmax(red[k][2], red[k][3]))
                    : (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]);
  }
}

// ---------------------------------------------------------------------------
// Finite-difference temperature treatment, Eq. (26):
//   K(T) = -u . grad T + div(lambda grad T) / (rho cv),
//   lambda = (tau_g - 1/2) cv rho c_s^2,
// with the isotropic central differences grad phi = sum_i w_i phi(x+e_i) e_i
// and lap phi = 2 sum_i w_i (phi(x+e_i) - phi(x)) (w = 1/3 on the axes, 1/12
// on the diagonals) and div(lambda grad T) = lambda lap T + grad lambda .
// grad T; two stages per step, Eq. (27) taken as Heun's method:
//   k1 = K(T^t), T^(t+1) = T^t + (k1 + K(T^t + k1)) / 2,
// with rho and u of time t in both stages.

// a field one node beyond the lattice at most: periodic wrap or the
// mirrored boundary node
__device__ inline long long fd_node(const Model &m, int x, int y, bool &ox, bool &oy) {
  ox = x < 0 || x >= m.nx;
  oy = y < 0 || y >= m.ny;
  if (ox) x = m.wall_x ? (x < 0 ? 0 : m.nx - 1) : (x < 0 ? x + m.nx : x - m.nx);
  if (oy) y = m.wall_y ? (y < 0 ? 0 : m.ny - 1) : (y < 0 ? y + m.ny : y - m.ny);
  return (long long)y * m.nx + x;
}

// temperature ghost beyond a wall (halfway): 2 T_w - T(mirror) for a
// Dirichlet wall, T(mirror) for an adiabatic one.  Beyond a corner of a box
// (both walls crossed) the corner is adiabatic if either wall is, else
// Dirichlet at the mean of the two wall temperatures, so that neither axis
// is preferred; at a corner of the open channel the plate's condition holds.
__device__ inline double fd_T_ghost(const Model &m, double v, int x, int y, bool ox, bool oy) {
  const int kx = (ox && m.wall_x) ? (x < 0 ? 0 : 1) : -1;
  const int ky = (oy && m.wall_y) ? (y < 0 ? 2 : 3) : -1;
  if (ky >= 0 && kx >= 0 && m.wall_x == 1) {
    if (m.thermal[kx] != 0 || m.thermal[ky] != 0) return v;
    return 2.0 * (0.5 * (m.T_wall[kx] + m.T_wall[ky])) - v;
  }
  const int k = ky >= 0 ? ky : kx;
  if (k < 0) return v;
  return m.thermal[k] == 0 ? 2.0 * m.T_wall[k] - v : v;
}

// (dp_EOS/dT) at fixed rho: Carnahan-Starling rho R Z(eta), ideal rho R
__device__ inline double dp_dT(const Model &m, double rho) {
  if (m.eos == 1) return rho * m.R;
  const double eta = 0.25 * m.b * rho;
  const double om = 1.0 - eta;
  return rho * m.R * (1.0 + eta + eta * eta - eta * eta * eta) / (om * om * om);
}

// K at node (x, y); Tval(c) gives the stage temperature at an in-lattice
// node.  With m.phi_divu, K also carries phi div u / (rho cv) of Eq. (5),
// phi = -T (dp_EOS/dT)_rho, div u by the same gradient stencil (the
// velocity beyond a wall is the boundary node's, reversed)
template <typename TV>
__device__ inline double fd_K(const Model &m, const double *rho, const double *uxa, const double *uya,
                              int x, int y, long long c, TV Tval) {
  const double ux = uxa[c], uy = uya[c];
  constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const double Tc = Tval(c);
  double gTx = 0.0, gTy = 0.0, gLx = 0.0, gLy = 0.0, lap = 0.0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const double w = i < 5 ? 1.0 / 3.0 : 1.0 / 12.0;
    const int xn = x + ex[i], yn = y + ey[i];
    bool ox, oy;
    const long long cn = fd_node(m, xn, yn, ox, oy);
    const double Tn = fd_T_ghost(m, Tval(cn), xn, yn, ox, oy);
    const double ln = m.lam_per_rho * rho[cn];
    gTx += w * Tn * ex[i];
    gTy += w * Tn * ey[i];
    gLx += w * ln * ex[i];
    gLy += w * ln * ey[i];
    lap += 2.0 * w * (Tn - Tc);
  }
  const double div = m.lam_per_rho * rho[c] * lap + gLx * gTx + gLy * gTy;
  double K = -(ux * gTx + uy * gTy) + div / (rho[c] * m.cv);
  if (m.phi_divu) K += -Tc * dp_dT(m, rho[c]) * div_u_at(m, uxa, uya, x, y) / (rho[c] * m.cv);
  return K;
}

__global__ void k_fd1(Model m, const double *__restrict__ mom, double *__restrict__ k1) {
  const long long n = (long long)m.nx * m.ny;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int x = (int)(c % m.nx), y = (int)(c / m.nx);
  const double *rho = mom, *ux = mom + n, *uy = mom + 2 * n, *T = mom + 3 * n;
  k1[c] = fd_K(m, rho, ux, uy, x, y, c, [&](long long q) { return T[q]; });
}

template <int ST>
__global__ void k_fd2(Model m, const double *__restrict__ mom, const double *__restrict__ k1,
                      void *__restrict__ dst_v) {
  using S = typename Prec<ST>::S;
  const long long n = (long long)m.nx * m.ny;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int x = (int)(c % m.nx), y = (int)(c / m.nx);
  const double *rho = mom, *ux = mom + n, *uy = mom + 2 * n, *T = mom + 3 * n;
  const double k2 = fd_K(m, rho, ux, uy, x, y, c, [&](long long q) { return T[q] + k1[q]; });
  const double Tn = T[c] + 0.5 * (k1[c] + k2);
  S *dst = (S *)dst_v;
  const _Float16 *ref = (const _Float16 *)((const char *)dst_v + ref_plane_offset(m, ST));
  const long long idx = (long long)y * m.pitch + x;
  const double rf = ST == ST_F64 ? 0.0
                                 : (ST == ST_F32_GLOBAL ? m.rho_ref : (double)(float)ref[(long long)y * m.rpitch + x]);
  const double cvT = m.cv * Tn;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double w = wgt<double>(i);
    const double f = (double)dst[i * m.plane + idx] + w * rf;
    dst[(9 + i) * m.plane + idx] = (S)(cvT * f - w * rf * m.cvT_ref);
  }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// plain streaming copy: each lane moves four 16-byte words per trip
__global__ __launch_bounds__(256) void k_copy(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src,
                                              long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x * 4;
  for (long long i = ((long long)blockIdx.x * blockDim.x * 4) + threadIdx.x; i < n; i += stride) {
    u32x4 a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (i + k * 256 < n) a[k] = src[i + k * 256];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (i + k * 256 < n) __builtin_nontemporal_store(a[k], &dst[i + k * 256]);
  }
}

// ---------------------------------------------------------------------------

static inline unsigned grid1d(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

static inline unsigned tile_grid(const Tiling &t) {
  unsigned g = (unsigned)(t.strips * t.bands);
  if (t.xcd) g = (g + 7u) & ~7u;
  return g;
}

template <int ST, int MODE, int PF>
static hipError_t launch_tile_t(const Model &m, const Tiling &t, const void *src, void *dst,
                                int treatment, unsigned long long *cc, const MomentsOut &mo,
                                hipStream_t s) {
  const unsigned grid = tile_grid(t);
  switch (t.bx) {
    case 64:
      hipLaunchKernelGGL((k_tile<ST, 64, MODE, PF>), dim3(grid), dim3(64), 0, s, m, t, src, dst, treatment, cc, mo);
      break;
    case 128:
      hipLaunchKernelGGL((k_tile<ST, 128, MODE, PF>), dim3(grid), dim3(128), 0, s, m, t, src, dst, treatment, cc, mo);
      break;
    case 256:
      hipLaunchKernelGGL((k_tile<ST, 256, MODE, PF>), dim3(grid), dim3(256), 0, s, m, t, src, dst, treatment, cc, mo);
      break;
    case 512:
      hipLaunchKernelGGL((k_tile<ST, 512, MODE, PF>), dim3(grid), dim3(512), 0, s, m, t, src, dst, treatment, cc, mo);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODE, int PF>
static hipError_t launch_tile_st(const Model &m, const Tiling &t, int st, const void *src, void *dst,
                                 int treatment, unsigned long long *cc, const MomentsOut &mo,
                                 hipStream_t s) {
  switch (st) {
    case ST_F64: return launch_tile_t<ST_F64, MODE, PF>(m, t, src, dst, treatment, cc, mo, s);
    case ST_F32_GLOBAL: return launch_tile_t<ST_F32_GLOBAL, MODE, PF>(m, t, src, dst, treatment, cc, mo, s);
    case ST_F32_LOCAL: return launch_tile_t<ST_F32_LOCAL, MODE, PF>(m, t, src, dst, treatment, cc, mo, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step(const Model &m, const Tiling &t, int st, const void *src, void *dst,
                       int treatment, unsigned long long *cc, hipStream_t s) {
  MomentsOut mo{};
  if (m.wall_x == 2) {
    if (t.pf >= 2) return launch_tile_st<MODE_STEP_OPEN, 2>(m, t, st, src, dst, treatment, cc, mo, s);
    return launch_tile_st<MODE_STEP_OPEN, 1>(m, t, st, src, dst, treatment, cc, mo, s);
  }
  if (t.pf >= 2) return launch_tile_st<MODE_STEP, 2>(m, t, st, src, dst, treatment, cc, mo, s);
  return launch_tile_st<MODE_STEP, 1>(m, t, st, src, dst, treatment, cc, mo, s);
}

hipError_t launch_step_fd(const Model &m, const Tiling &t, int st, const void *src, void *dst,
                          unsigned long long *cc, const MomentsOut &mo, hipStream_t s) {
  if (!mo.rho || !mo.ux || !mo.uy || !mo.T || m.wall_x == 2 || t.pf < 2) return hipErrorInvalidValue;
  return launch_tile_st<MODE_STEP_FD, 2>(m, t, st, src, dst, 0, cc, mo, s);
}

hipError_t launch_step_src(const Model &m, const Tiling &t, int st, const void *src, void *dst,
                           int treatment, unsigned long long *cc, const double *ux, const double *uy,
                           hipStream_t s) {
  MomentsOut mo{};
  mo.ux = const_cast<double *>(ux);
  mo.uy = const_cast<double *>(uy);
  if (!ux || !uy) return hipErrorInvalidValue;
  if (m.wall_x == 2) return launch_tile_st<MODE_STEP_OPEN, 1>(m, t, st, src, dst, treatment, cc, mo, s);
  return launch_tile_st<MODE_STEP_SRC, 1>(m, t, st, src, dst, treatment, cc, mo, s);
}

hipError_t launch_pair(const Model &m, const Tiling &t, int st, const void *src, void *dst,
                       int treatment, unsigned long long *cc, hipStream_t s) {
  const unsigned grid = tile_grid(t);
  const bool mix = m.sc_on && !m.beta_one;
  if ((t.bx != 64 && t.bx != 128 && t.bx != 256) || m.wall_x != 0 ||
      ((st == ST_F64 || mix) && t.bx != 128))
    return hipErrorInvalidValue;
#define LBM_P(ST_, B_, MIX_) \
  hipLaunchKernelGGL((k_pair<ST_, B_, MIX_>), dim3(grid), dim3(B_), 0, s, m, t, src, dst, treatment, cc)
  if (mix) {
    if (st == ST_F64) LBM_P(ST_F64, 128, true);
    else if (st == ST_F32_GLOBAL) LBM_P(ST_F32_GLOBAL, 128, true);
    else if (st == ST_F32_LOCAL) LBM_P(ST_F32_LOCAL, 128, true);
    else return hipErrorInvalidValue;
  } else if (st == ST_F64) {
    LBM_P(ST_F64, 128, false);
  } else if (st == ST_F32_GLOBAL) {
    if (t.bx == 64) LBM_P(ST_F32_GLOBAL, 64, false);
    else if (t.bx == 128) LBM_P(ST_F32_GLOBAL, 128, false);
    else LBM_P(ST_F32_GLOBAL, 256, false);
  } else if (st == ST_F32_LOCAL) {
    if (t.bx == 64) LBM_P(ST_F32_LOCAL, 64, false);
    else if (t.bx == 128) LBM_P(ST_F32_LOCAL, 128, false);
    else LBM_P(ST_F32_LOCAL, 256, false);
  } else {
    return hipErrorInvalidValue;
  }
#undef LBM_P
  return hipGetLastError();
}

hipError_t launch_moments(const Model &m, const Tiling &t, int st, const void *src,
                          const MomentsOut &o, hipStream_t s) {
  return launch_tile_st<MODE_MOMENTS, 1>(m, t, st, src, nullptr, 0, nullptr, o, s);
}

hipError_t launch_fd(const Model &m, int st, const double *mom, double *k1, void *dst, hipStream_t s) {
  const long long n = (long long)m.nx * m.ny;
  const dim3 g(grid1d(n, 256)), b(256);
  hipLaunchKernelGGL(k_fd1, g, b, 0, s, m, mom, k1);
  switch (st) {
    case ST_F64: hipLaunchKernelGGL(k_fd2<ST_F64>, g, b, 0, s, m, mom, k1, dst); break;
    case ST_F32_GLOBAL: hipLaunchKernelGGL(k_fd2<ST_F32_GLOBAL>, g, b, 0, s, m, mom, k1, dst); break;
    case ST_F32_LOCAL: hipLaunchKernelGGL(k_fd2<ST_F32_LOCAL>, g, b, 0, s, m, mom, k1, dst); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_init(const Model &m, int st, void *dst, const double *rho, const double *ux,
                       const double *uy, const double *T, hipStream_t s) {
  const long long n = (long long)m.nx * m.ny;
  const dim3 g(grid1d(n, 256)), b(256);
  switch (st) {
    case ST_F64: hipLaunchKernelGGL(k_init<ST_F64>, g, b, 0, s, m, dst, rho, ux, uy, T); break;
    case ST_F32_GLOBAL: hipLaunchKernelGGL(k_init<ST_F32_GLOBAL>, g, b, 0, s, m, dst, rho, ux, uy, T); break;
    case ST_F32_LOCAL: hipLaunchKernelGGL(k_init<ST_F32_LOCAL>, g, b, 0, s, m, dst, rho, ux, uy, T); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int nblocks, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, partials, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_plane_to_f64(const Model &m, int st, const void *src, int q, double *out,
                               hipStream_t s) {
  const long long n = (long long)m.nx * m.ny;
  const dim3 g(grid1d(n, 256)), b(256);
  switch (st) {
    case ST_F64: hipLaunchKernelGGL(k_plane_to<ST_F64>, g, b, 0, s, m, src, q, out); break;
    case ST_F32_GLOBAL: hipLaunchKernelGGL(k_plane_to<ST_F32_GLOBAL>, g, b, 0, s, m, src, q, out); break;
    case ST_F32_LOCAL: hipLaunchKernelGGL(k_plane_to<ST_F32_LOCAL>, g, b, 0, s, m, src, q, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_plane_from_f64(const Model &m, int st, void *dst, int q, const double *in,
                                 hipStream_t s) {
  const long long n = (long long)m.nx * m.ny;
  const dim3 g(grid1d(n, 256)), b(256);
  switch (st) {
    case ST_F64: hipLaunchKernelGGL(k_plane_from<ST_F64>, g, b, 0, s, m, dst, q, in); break;
    case ST_F32_GLOBAL: hipLaunchKernelGGL(k_plane_from<ST_F32_GLOBAL>, g, b, 0, s, m, dst, q, in); break;
    case ST_F32_LOCAL:
      if (q < 0) hipLaunchKernelGGL(k_ref_from_rho, g, b, 0, s, m, dst, in);
      else hipLaunchKernelGGL(k_plane_from<ST_F32_LOCAL>, g, b, 0, s, m, dst, q, in);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s) {
  const long long n = (long long)(bytes / 16);
  long long blocks = (n + 1023) / 1024;
  if (blocks > 256 * 32) blocks = 256 * 32;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (u32x4 *)dst, (const u32x4 *)src, n);
  return hipGetLastError();
}

hipError_t launch_batch_pair(const BatchTables &t, int bx, int st, bool mix, char *base, int parity,
                             int treatment, hipStream_t s) {
  unsigned grid = (unsigned)t.ntiles;
  if (t.xcd) grid = (grid + 7u) & ~7u;
  if (grid == 0) return hipSuccess;
  const dim3 g(grid);
  if (bx != 128) return hipErrorInvalidValue;
#define LBM_PB(ST_, MIX_) \
  hipLaunchKernelGGL((k_pair_batch<ST_, 128, MIX_>), g, dim3(128), 0, s, t, base, parity, treatment)
  if (st == ST_F64) {
    if (mix) LBM_PB(ST_F64, true);
    else LBM_PB(ST_F64, false);
  } else if (st == ST_F32_GLOBAL) {
    if (mix) LBM_PB(ST_F32_GLOBAL, true);
    else LBM_PB(ST_F32_GLOBAL, false);
  } else if (st == ST_F32_LOCAL) {
    if (mix) LBM_PB(ST_F32_LOCAL, true);
    else LBM_PB(ST_F32_LOCAL, false);
  } else {
    return hipErrorInvalidValue;
  }
#undef LBM_PB
  return hipGetLastError();
}

hipError_t launch_batch_step(const BatchTables &t, int bx, int pf, int st, char *base, int parity,
                             int treatment, hipStream_t s) {
  unsigned grid = (unsigned)t.ntiles;
  if (t.xcd) grid = (grid + 7u) & ~7u;
  if (grid == 0) return hipSuccess;
  const dim3 g(grid);
#define LBM_B(ST_, B_, PF_) \
  hipLaunchKernelGGL((k_batch<ST_, B_, PF_>), g, dim3(B_), 0, s, t, base, parity, treatment)
#define LBM_BX(ST_, PF_)                      \
  do {                                        \
    if (bx == 64) LBM_B(ST_, 64, PF_);        \
    else if (bx == 128) LBM_B(ST_, 128, PF_); \
    else if (bx == 256) LBM_B(ST_, 256, PF_); \
    else return hipErrorInvalidValue;         \
  } while (0)
#define LBM_PF(ST_)                      \
  do {                                   \
    if (pf >= 2) LBM_BX(ST_, 2);         \
    else LBM_BX(ST_, 1);                 \
  } while (0)
  if (st == ST_F64) {
    LBM_PF(ST_F64);
  } else if (st == ST_F32_GLOBAL) {
    LBM_PF(ST_F32_GLOBAL);
  } else if (st == ST_F32_LOCAL) {
    LBM_PF(ST_F32_LOCAL);
  } else {
    return hipErrorInvalidValue;
  }
#undef LBM_PF
#undef LBM_BX
#undef LBM_B
  return hipGetLastError();
}

}  // namespace lbmdev
