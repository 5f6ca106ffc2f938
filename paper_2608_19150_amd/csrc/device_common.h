// Device helpers shared by the DAG builder and the sweep kernels.
#pragma once

#include "internal.h"

namespace bgk {

// A kernel of a Picard iteration that was enqueued ahead of the host's view
// of convergence does nothing once the device-side stopping test has set
// *flag (null: always runs).  The flag is written by an earlier kernel on
// the same stream, so it is visible at launch.
__device__ __forceinline__ bool skip_launch(const int32_t* flag) {
  return flag != nullptr && *flag != 0;
}

// Facet fluxes fl_k = v.N_k (N_k = |e_k| n_k, outward) from the stored
// area-weighted normals, in a fixed operation order so that the DAG builder
// and the sweep classify every facet identically (inflow iff fl_k < 0).  A
// tangential facet, |v.n| <= 1e-12 |v|, gets exactly 0 (no edge, no flux):
// its computed flux is rounding noise whose sign means nothing.
template <int DIM>
__device__ __forceinline__ void facet_flux_raw(const double* __restrict__ geo, const double* v,
                                               double v2, double* fl, double* raw) {
#pragma unroll
  for (int k = 0; k <= DIM; ++k) {
    const double* N = geo + 1 + k * DIM;
    double s = N[0] * v[0];
    double n2 = N[0] * N[0];
#pragma unroll
    for (int d = 1; d < DIM; ++d) {
      s = __fma_rn(N[d], v[d], s);
      n2 = __fma_rn(N[d], N[d], n2);
    }
    raw[k] = s;
    fl[k] = (s * s <= 1e-24 * v2 * n2) ? 0.0 : s;
  }
}

template <int DIM>
__device__ __forceinline__ void facet_flux(const double* __restrict__ geo, const double* v,
                                           double v2, double* fl) {
  double raw[DIM + 1];
  facet_flux_raw<DIM>(geo, v, v2, fl, raw);
}

// Same, plus the stiffness weights w = |det J| J^{-1} v = -(d-1)! v.N_{b+1},
// taken from the unthresholded fluxes.
template <int DIM>
__device__ __forceinline__ void facet_flux_w(const double* __restrict__ geo, const double* v,
                                             double v2, double* fl, double* w) {
  double raw[DIM + 1];
  facet_flux_raw<DIM>(geo, v, v2, fl, raw);
  constexpr double f = (DIM == 2) ? -1.0 : -2.0;
#pragma unroll
  for (int b = 0; b < DIM; ++b) w[b] = f * raw[b + 1];
}

// bit k set: facet k of cell K is an interior inflow facet that is not
// lagged by the caller's mask
template <int DIM>
__device__ __forceinline__ int inflow_bits(const double* __restrict__ geo,
                                           const FacetRec* __restrict__ facet, int K,
                                           const double* v, int user_lag) {
  double fl[DIM + 1];
  double v2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) v2 = __fma_rn(v[d], v[d], v2);
  facet_flux<DIM>(geo + (size_t)K * GeoLayout<DIM>::STRIDE, v, v2, fl);
  int bits = 0;
#pragma unroll
  for (int k = 0; k <= DIM; ++k)
    if (fl[k] < 0.0 && facet[(size_t)K * (DIM + 1) + k].nb >= 0) bits |= 1 << k;
  return bits & ~user_lag;
}

// exp(x) by Cody-Waite reduction x = k ln2 + r (ln2 split into a high part
// with 21 trailing zero bits and a low part, so k*ln2_hi is exact for
// |k| < 2^11) and the degree-13 Taylor polynomial of exp(r) on
// |r| <= ln2/2 (truncation below 5e-18 relative), scaled by 2^k with ldexp
// (which also produces the gradual underflow).  Arguments below -745 give 0.
__device__ __forceinline__ double bgk_exp(double x) {
  if (x < -745.5) return 0.0;
  const double k = rint(x * 1.4426950408889634074);
  const double r = fma(-k, 1.9082149292705877000e-10, fma(-k, 6.93147180369123816490e-01, x));
  double p = 1.0 / 6227020800.0;           // 1/13!
  p = fma(p, r, 1.0 / 479001600.0);        // 1/12!
  p = fma(p, r, 1.0 / 39916800.0);         // 1/11!
  p = fma(p, r, 1.0 / 3628800.0);          // 1/10!
  p = fma(p, r, 1.0 / 362880.0);           // 1/9!
  p = fma(p, r, 1.0 / 40320.0);            // 1/8!
  p = fma(p, r, 1.0 / 5040.0);             // 1/7!
  p = fma(p, r, 1.0 / 720.0);              // 1/6!
  p = fma(p, r, 1.0 / 120.0);              // 1/5!
  p = fma(p, r, 1.0 / 24.0);               // 1/4!
  p = fma(p, r, 1.0 / 6.0);                // 1/3!
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)k);
}

// Maxwellian value exp(a + b.v + c|v|^2) from coefficients
template <int DIM>
__device__ __forceinline__ double maxw_eval(const double* __restrict__ coef, const double* v,
                                            double v2) {
  double e = coef[0];
#pragma unroll
  for (int d = 0; d < DIM; ++d) e = __fma_rn(coef[1 + d], v[d], e);
  e = __fma_rn(coef[1 + DIM], v2, e);
  return bgk_exp(e);
}

}  // namespace bgk
