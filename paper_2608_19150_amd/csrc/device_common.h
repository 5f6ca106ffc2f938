// Device helpers shared by the DAG builder and the sweep kernels.
#pragma once

#include "internal.h"

namespace bgk {

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

// Maxwellian value exp(a + b.v + c|v|^2) from coefficients
template <int DIM>
__device__ __forceinline__ double maxw_eval(const double* __restrict__ coef, const double* v,
                                            double v2) {
  double e = coef[0];
#pragma unroll
  for (int d = 0; d < DIM; ++d) e = __fma_rn(coef[1 + d], v[d], e);
  e = __fma_rn(coef[1 + DIM], v2, e);
  return exp(e);
}

}  // namespace bgk
