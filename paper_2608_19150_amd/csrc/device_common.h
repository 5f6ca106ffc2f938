// Device helpers shared by the DAG builder and the sweep kernels.
#pragma once

#include "internal.h"

namespace bgk {

// Facet fluxes v.N_k (N_k = |e_k| n_k, outward) of one cell from its
// D = |det J| J^{-1}: with w = D v,
//   v.N_0 = sum_b w_b / (d-1)!,   v.N_k = -w_{k-1} / (d-1)!   (k >= 1).
// Explicit fma calls fix the rounding so that the DAG builder and the sweep
// classify every facet identically (inflow iff v.N_k < 0).
template <int DIM>
__device__ __forceinline__ void facet_flux(const double* __restrict__ D, const double* v,
                                           double* fl) {
  double w[DIM];
#pragma unroll
  for (int r = 0; r < DIM; ++r) {
    double s = D[r * DIM] * v[0];
#pragma unroll
    for (int c = 1; c < DIM; ++c) s = __fma_rn(D[r * DIM + c], v[c], s);
    w[r] = s;
  }
  constexpr double inv = (DIM == 2) ? 1.0 : 0.5;
  double sum = w[0];
#pragma unroll
  for (int r = 1; r < DIM; ++r) sum += w[r];
  fl[0] = sum * inv;
#pragma unroll
  for (int k = 1; k <= DIM; ++k) fl[k] = -w[k - 1] * inv;
}

// Same as facet_flux but also returns w = D v (the stiffness weights).
template <int DIM>
__device__ __forceinline__ void facet_flux_w(const double* __restrict__ D, const double* v,
                                             double* fl, double* w) {
#pragma unroll
  for (int r = 0; r < DIM; ++r) {
    double s = D[r * DIM] * v[0];
#pragma unroll
    for (int c = 1; c < DIM; ++c) s = __fma_rn(D[r * DIM + c], v[c], s);
    w[r] = s;
  }
  constexpr double inv = (DIM == 2) ? 1.0 : 0.5;
  double sum = w[0];
#pragma unroll
  for (int r = 1; r < DIM; ++r) sum += w[r];
  fl[0] = sum * inv;
#pragma unroll
  for (int k = 1; k <= DIM; ++k) fl[k] = -w[k - 1] * inv;
}

// bit k set: facet k of cell K is an interior inflow facet that is not
// lagged by the caller's mask
template <int DIM>
__device__ __forceinline__ int inflow_bits(const double* __restrict__ geo,
                                           const FacetRec* __restrict__ facet, int K,
                                           const double* v, int user_lag) {
  double fl[DIM + 1];
  facet_flux<DIM>(geo + (size_t)K * GeoLayout<DIM>::STRIDE, v, fl);
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
