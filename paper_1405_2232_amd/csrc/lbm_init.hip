// Initial states at mechanical balance with the forcing scheme.
//
// With the forcing of Eq. (1) (Guo's scheme, Sec. II) the fluid velocity
// is u = (j + F/2)/rho, j the first moment of the stored f.  A state
// initialised as f_eq(rho, u) stores j = rho u, so its velocity is
// u + F/(2 rho): near an interface, where the force of Eq. (2) or (4) is
// large, it starts far from the velocity asked for, and the LB step spends
// many steps relaxing that momentum.  lbm_init_fields_physical stores
// j = rho u - F/2 instead (f = f_eq(rho, u - F/(2 rho)), g = cv T f),
// with F the total force of the initial rho and T, so that the velocity
// the moments report is the given u.
#include <hip/hip_runtime.h>

#include "lbm_ctx.h"

namespace {

// u' = 2 u - u_rep, u_rep = (rho u + F/2)/rho reported for the state
// initialised with u: u' = u - F/(2 rho) to rounding
__global__ void k_balance_velocity(long long n, const double *__restrict__ rep,
                                   double *__restrict__ u, int have_u) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double u0 = have_u ? u[c] : 0.0;
  u[c] = 2.0 * u0 - rep[c];
}

hipError_t balance(lbm_ctx *h, int have_ux, int have_uy) {
  const long long n = (long long)h->p.nx * h->p.ny;
  // init_fields' staging layout: rho, T, ux, uy
  double *d_rho = h->staging, *d_T = h->staging + n, *d_ux = h->staging + 2 * n,
         *d_uy = h->staging + 3 * n;
  // the second distribution buffer is not read before the first step
  // writes it: it holds the reported velocity (2 n doubles; one buffer
  // holds at least 18 n FP32 values)
  double *rep = (double *)h->buf[1];
  lbmdev::MomentsOut mo{};
  mo.ux = rep;
  mo.uy = rep + n;
  mo.partials = h->partials;
  hipError_t e = lbmdev::launch_moments(h->m, h->tm, h->st, h->buf[0], mo, h->stream);
  if (e != hipSuccess) return e;
  const int tpb = 256;
  const unsigned grid = (unsigned)((n + tpb - 1) / tpb);
  k_balance_velocity<<<grid, tpb, 0, h->stream>>>(n, rep, d_ux, have_ux);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_balance_velocity<<<grid, tpb, 0, h->stream>>>(n, rep + n, d_uy, have_uy);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = lbmdev::launch_init(h->m, h->st, h->buf[0], d_rho, d_ux, d_uy, d_T, h->stream);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(h->counters, 0, 8 * sizeof(unsigned long long), h->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(h->stream);
}

}  // namespace

extern "C" {

int lbm_init_fields_physical(lbm_handle h, const double *rho, const double *ux, const double *uy,
                             const double *T) {
  const int rc = lbm_init_fields(h, rho, ux, uy, T);
  if (rc) return rc;
  if (balance(h, ux != nullptr, uy != nullptr) != hipSuccess) {
    h->initialized = 0;
    return LBM_EDEVICE;
  }
  h->cur = 0;
  h->steps = 0;
  return LBM_OK;
}

int lbm_batch_init_fields_physical(lbm_batch_handle b, int i, const double *rho, const double *ux,
                                   const double *uy, const double *T) {
  lbm_handle h = nullptr;
  const int rc = lbm_batch_lattice(b, i, &h);
  if (rc) return rc;
  return lbm_init_fields_physical(h, rho, ux, uy, T);
}

}  // extern "C"
