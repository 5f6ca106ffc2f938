// tgs_sweep: the topological-generation sweep (Sec. 4.1) of the Picard
// iteration eq. bgk-ss-picard, plus layout conversion kernels.
//
// Mapping: one workgroup owns one velocity j and walks that velocity's
// generations in order; the threads of the workgroup take the cells of a
// generation (a contiguous slot range in the sweep layout, so q and f move
// through HBM fully coalesced) and a workgroup barrier separates
// generations.  Velocities are independent, so no grid-wide barrier exists.
// Each thread assembles its cell's local system
//   A = |K| mass diag(sigma) - sum_b w_b stiff_b + sum_{v.N_k>0} (v.N_k) fmass_k
// (w = |det J| J^{-1} v, obtained from the facet fluxes) from compile-time
// reference matrices and solves it
// in registers by Gaussian elimination without pivoting (the symmetric part
// of A is positive definite: sigma > 0 plus the upwind facet terms).
#include "device_common.h"

namespace bgk {

struct SweepArgs {
  const double* geo;
  const FacetRec* facet;
  const int32_t* uid;
  const double* v;
  const int32_t* perm;
  const int32_t* pos;
  const int32_t* goff;
  const int64_t* gbase;
  const int32_t* G;
  const uint8_t* lag;
  const int32_t* vorder;
  const double* nu;
  const double* mcoef;
  const double* q;
  const double* bc_coef;
  const double* bc_dense;
  const double* f_prev;
  double* f_out;
  float* d32;      // FP32 correction traces (sweep layout), FP32 form only
  double sigma_shift;
  double q_scale;
  int n_cells;
  int n_v;
};

template <int N, typename T>
__device__ __forceinline__ void lu_solve(T (&A)[N][N], T (&b)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const T inv = T(1) / A[k][k];
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const T l = A[i][k] * inv;
#pragma unroll
      for (int c = k + 1; c < N; ++c) A[i][c] = fma(-l, A[k][c], A[i][c]);
      b[i] = fma(-l, b[k], b[i]);
    }
    A[k][k] = inv;
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    T s = b[i];
#pragma unroll
    for (int c = i + 1; c < N; ++c) s = fma(-A[i][c], b[c], s);
    b[i] = s * A[i][i];
  }
}

// Assemble the local matrix A and the volume part of the right-hand side
// for one (velocity, cell) item.
template <int DIM, int ORDER>
__device__ __forceinline__ void assemble(const double vol, const double* w, const double* fl,
                                         const double* sig, const double* src,
                                         double (&A)[Elem<DIM, ORDER>::NP][Elem<DIM, ORDER>::NP],
                                         double (&rhs)[Elem<DIM, ORDER>::NP]) {
  using E = Elem<DIM, ORDER>;
  constexpr int NP = E::NP, NF = E::NF;
#pragma unroll
  for (int a = 0; a < NP; ++a) {
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      double x = 0.0;
      if (E::T.mass[a][b] != 0.0) x = (vol * E::T.mass[a][b]) * sig[b];
#pragma unroll
      for (int be = 0; be < DIM; ++be)
        if (E::T.stiff[be][a][b] != 0.0) x = fma(-E::T.stiff[be][a][b], w[be], x);
      A[a][b] = x;
    }
    double r = 0.0;
#pragma unroll
    for (int b = 0; b < NP; ++b)
      if (E::T.mass[a][b] != 0.0) r = fma(E::T.mass[a][b], src[b], r);
    rhs[a] = vol * r;
  }
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const double out = fl[k] > 0.0 ? fl[k] : 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a)
#pragma unroll
      for (int b = 0; b < NP; ++b)
        if (E::T.fmass[k][a][b] != 0.0) A[a][b] = fma(out, E::T.fmass[k][a][b], A[a][b]);
  }
}

template <int DIM, int ORDER>
__global__ __launch_bounds__(1024) void k_sweep_fp64(SweepArgs a) {
  using E = Elem<DIM, ORDER>;
  constexpr int NP = E::NP, NF = E::NF, NFP = E::NFP, NC = DIM + 2;
  const int j = a.vorder[blockIdx.x];
  double v[DIM];
  double v2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    v[d] = a.v[(size_t)j * DIM + d];
    v2 = fma(v[d], v[d], v2);
  }
  const size_t base = (size_t)j * a.n_cells;
  const int32_t* __restrict__ perm = a.perm + base;
  const int32_t* __restrict__ pos = a.pos + base;
  const int32_t* __restrict__ go = a.goff + a.gbase[j];
  const int G = a.G[j];
  const double* __restrict__ q = a.q + base * NP;
  double* fo = a.f_out + base * NP;
  const double* fp = a.f_prev ? a.f_prev + base * NP : nullptr;
  const uint8_t* __restrict__ lag = a.lag ? a.lag + base : nullptr;
  const double qs = a.q_scale, shift = a.sigma_shift;

  for (int g = 0; g < G; ++g) {
    const int s0 = go[g], s1 = go[g + 1];
    for (int s = s0 + (int)threadIdx.x; s < s1; s += blockDim.x) {
      const int K = perm[s];
      const double* __restrict__ gk = a.geo + (size_t)K * GeoLayout<DIM>::STRIDE;
      const double vol = gk[0];
      double fl[NF], w[DIM];
      facet_flux_w<DIM>(gk, v, v2, fl, w);
      const size_t u = (size_t)a.uid[K];
      double sig[NP], src[NP];
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        const double M = maxw_eval<DIM>(a.mcoef + (u * NP + b) * NC, v, v2);
        const double nub = a.nu[u * NP + b];
        sig[b] = nub + shift;
        src[b] = fma(nub, M, qs * q[(size_t)s * NP + b]);
      }
      double A[NP][NP], rhs[NP];
      assemble<DIM, ORDER>(vol, w, fl, sig, src, A, rhs);
      const int lb = lag ? lag[K] : 0;
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        if (!(fl[k] < 0.0)) continue;
        const double inflow = -fl[k];
        const FacetRec fr = a.facet[(size_t)K * NF + k];
        double fh[NFP];
        if (fr.nb >= 0) {
          const size_t sl = (size_t)pos[fr.nb];
          const double* srcf = ((lb >> k) & 1) ? fp : fo;
#pragma unroll
          for (int p = 0; p < NFP; ++p) fh[p] = srcf[sl * NP + ((fr.pack >> (4 * (p + 1))) & 15)];
        } else {
          const size_t bf = (size_t)(-fr.nb - 1);
          if (a.bc_coef) {
#pragma unroll
            for (int p = 0; p < NFP; ++p) fh[p] = maxw_eval<DIM>(a.bc_coef + (bf * NFP + p) * NC, v, v2);
          } else {
#pragma unroll
            for (int p = 0; p < NFP; ++p) fh[p] = a.bc_dense[(bf * NFP + p) * a.n_v + j];
          }
        }
#pragma unroll
        for (int ia = 0; ia < NFP; ++ia) {
          const int ra = E::T.fnode[k][ia];
          double r = 0.0;
#pragma unroll
          for (int p = 0; p < NFP; ++p) r = fma(E::T.fmass[k][ra][E::T.fnode[k][p]], fh[p], r);
          rhs[ra] = fma(inflow, r, rhs[ra]);
        }
      }
      lu_solve<NP, double>(A, rhs);
#pragma unroll
      for (int b = 0; b < NP; ++b) fo[(size_t)s * NP + b] = rhs[b];
    }
    __syncthreads();
  }
}

// FP32 defect-correction sweep: per cell the FP64 residual of the previous
// iterate f_prev,
//   r = M_K(nu*M + q_scale*q) + inflow(f_prev) - A f_prev   (all FP64),
// then A delta = r + inflow(delta) solved in FP32 with upwind delta traces,
// and f_out = f_prev + delta stored in FP64.  At a fixed point of the Picard
// iteration delta -> 0, so the FP64 state converges to the FP64 solution.
template <int DIM, int ORDER>
__global__ __launch_bounds__(1024) void k_sweep_fp32c(SweepArgs a) {
  using E = Elem<DIM, ORDER>;
  constexpr int NP = E::NP, NF = E::NF, NFP = E::NFP, NC = DIM + 2;
  const int j = a.vorder[blockIdx.x];
  double v[DIM];
  double v2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    v[d] = a.v[(size_t)j * DIM + d];
    v2 = fma(v[d], v[d], v2);
  }
  const size_t base = (size_t)j * a.n_cells;
  const int32_t* __restrict__ perm = a.perm + base;
  const int32_t* __restrict__ pos = a.pos + base;
  const int32_t* __restrict__ go = a.goff + a.gbase[j];
  const int G = a.G[j];
  const double* __restrict__ q = a.q + base * NP;
  double* fo = a.f_out + base * NP;
  const double* __restrict__ fp = a.f_prev + base * NP;
  float* dl = a.d32 + base * NP;
  const uint8_t* __restrict__ lag = a.lag ? a.lag + base : nullptr;
  const double qs = a.q_scale, shift = a.sigma_shift;

  for (int g = 0; g < G; ++g) {
    const int s0 = go[g], s1 = go[g + 1];
    for (int s = s0 + (int)threadIdx.x; s < s1; s += blockDim.x) {
      const int K = perm[s];
      const double* __restrict__ gk = a.geo + (size_t)K * GeoLayout<DIM>::STRIDE;
      const double vol = gk[0];
      double fl[NF], w[DIM];
      facet_flux_w<DIM>(gk, v, v2, fl, w);
      const size_t u = (size_t)a.uid[K];
      double sig[NP], src[NP], fold[NP];
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        const double M = maxw_eval<DIM>(a.mcoef + (u * NP + b) * NC, v, v2);
        const double nub = a.nu[u * NP + b];
        sig[b] = nub + shift;
        src[b] = fma(nub, M, qs * q[(size_t)s * NP + b]);
        fold[b] = fp[(size_t)s * NP + b];
      }
      double A[NP][NP], r[NP];
      assemble<DIM, ORDER>(vol, w, fl, sig, src, A, r);
      const int lb = lag ? lag[K] : 0;
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        if (!(fl[k] < 0.0)) continue;
        const double inflow = -fl[k];
        const FacetRec fr = a.facet[(size_t)K * NF + k];
        double fh[NFP];
        if (fr.nb >= 0) {
          const size_t sl = (size_t)pos[fr.nb];
#pragma unroll
          for (int p = 0; p < NFP; ++p) fh[p] = fp[sl * NP + ((fr.pack >> (4 * (p + 1))) & 15)];
        } else {
          const size_t bf = (size_t)(-fr.nb - 1);
          if (a.bc_coef) {
#pragma unroll
            for (int p = 0; p < NFP; ++p) fh[p] = maxw_eval<DIM>(a.bc_coef + (bf * NFP + p) * NC, v, v2);
          } else {
#pragma unroll
            for (int p = 0; p < NFP; ++p) fh[p] = a.bc_dense[(bf * NFP + p) * a.n_v + j];
          }
        }
#pragma unroll
        for (int ia = 0; ia < NFP; ++ia) {
          const int ra = E::T.fnode[k][ia];
          double acc = 0.0;
#pragma unroll
          for (int p = 0; p < NFP; ++p) acc = fma(E::T.fmass[k][ra][E::T.fnode[k][p]], fh[p], acc);
          r[ra] = fma(inflow, acc, r[ra]);
        }
      }
      // FP64 residual r -= A f_prev; FP32 copy of A
      float Af[NP][NP], rf[NP];
#pragma unroll
      for (int ia = 0; ia < NP; ++ia) {
        double x = r[ia];
#pragma unroll
        for (int b = 0; b < NP; ++b) x = fma(-A[ia][b], fold[b], x);
        rf[ia] = (float)x;
#pragma unroll
        for (int b = 0; b < NP; ++b) Af[ia][b] = (float)A[ia][b];
      }
      // inflow of the correction through non-lagged interior facets (FP32)
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        if (!(fl[k] < 0.0)) continue;
        const FacetRec fr = a.facet[(size_t)K * NF + k];
        if (fr.nb < 0 || ((lb >> k) & 1)) continue;
        const float inflow = (float)(-fl[k]);
        const size_t sl = (size_t)pos[fr.nb];
        float dh[NFP];
#pragma unroll
        for (int p = 0; p < NFP; ++p) dh[p] = dl[sl * NP + ((fr.pack >> (4 * (p + 1))) & 15)];
#pragma unroll
        for (int ia = 0; ia < NFP; ++ia) {
          const int ra = E::T.fnode[k][ia];
          float acc = 0.0f;
#pragma unroll
          for (int p = 0; p < NFP; ++p)
            acc = fmaf((float)E::T.fmass[k][ra][E::T.fnode[k][p]], dh[p], acc);
          rf[ra] = fmaf(inflow, acc, rf[ra]);
        }
      }
      lu_solve<NP, float>(Af, rf);
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        dl[(size_t)s * NP + b] = rf[b];
        fo[(size_t)s * NP + b] = fold[b] + (double)rf[b];
      }
    }
    __syncthreads();
  }
}

// canonical f[user cell][node][v] <-> sweep f[v][slot][node]
__global__ void k_pack(const double* __restrict__ src, double* __restrict__ dst,
                       const int32_t* __restrict__ pos, const int32_t* __restrict__ uid, int nc,
                       int nv, int np, int to_sweep) {
  const size_t total = (size_t)nc * np * nv;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx % nv);
    const size_t r = idx / nv;
    const int aa = (int)(r % np);
    const int K = (int)(r / np);
    const size_t ci = ((size_t)uid[K] * np + aa) * nv + j;
    const size_t si = ((size_t)j * nc + pos[(size_t)j * nc + K]) * np + aa;
    if (to_sweep)
      dst[si] = src[ci];
    else
      dst[ci] = src[si];
  }
}

template <int DIM>
__global__ void k_eval_maxw(const double* __restrict__ coef, double* __restrict__ f,
                            const int32_t* __restrict__ perm, const int32_t* __restrict__ uid,
                            const double* __restrict__ vel, int nc, int nv, int np) {
  const size_t total = (size_t)nc * np * nv;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int aa = (int)(idx % np);
    const size_t r = idx / np;
    const size_t s = r % nc;
    const int j = (int)(r / nc);
    double v[DIM], v2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      v[d] = vel[(size_t)j * DIM + d];
      v2 = fma(v[d], v[d], v2);
    }
    const size_t u = uid[perm[(size_t)j * nc + s]];
    f[idx] = maxw_eval<DIM>(coef + (u * np + aa) * (DIM + 2), v, v2);
  }
}

int launch_sweep(const tgs_dag* d, const tgs_sweep_io* io, float* d32, hipStream_t stream) {
  SweepArgs a{d->d_geo,  d->d_facet, d->d_uid, d->d_v,   d->d_perm,   d->d_pos,
              d->d_goff, d->d_gbase, d->d_G,   d->d_lag, d->d_vorder, io->nu,
              io->mcoef, io->q,      io->bc_coef, io->bc_dense, io->f_prev, io->f_out,
              d32,       io->sigma_shift, io->q_scale, (int)d->n_cells, d->n_v};
  const dim3 grid(d->n_v), block(d->sweep_threads);
  const bool fp32 = io->precision == TGS_FP32_CORRECTION;
#define BGK_LAUNCH(D_, O_)                                                                 \
  if (fp32)                                                                                \
    hipLaunchKernelGGL((k_sweep_fp32c<D_, O_>), grid, block, 0, stream, a);                \
  else                                                                                     \
    hipLaunchKernelGGL((k_sweep_fp64<D_, O_>), grid, block, 0, stream, a);
  if (d->dim == 2 && d->order == 1) {
    BGK_LAUNCH(2, 1)
  } else if (d->dim == 2 && d->order == 2) {
    BGK_LAUNCH(2, 2)
  } else {
    BGK_LAUNCH(3, 1)
  }
#undef BGK_LAUNCH
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int grid_for(size_t total) {
  size_t g = (total + 255) / 256;
  return (int)std::min<size_t>(g, 65536);
}

}  // namespace bgk

using namespace bgk;

extern "C" int tgs_sweep(const tgs_dag* d, const tgs_sweep_io* io, bgk_stream_t stream) {
  if (!d || !io) return fail(BGK_E_INVALID, "null argument");
  if (!io->q || !io->f_out || !io->nu || !io->mcoef)
    return fail(BGK_E_INVALID, "q, f_out, nu and mcoef are required");
  if ((io->bc_coef == nullptr) == (io->bc_dense == nullptr))
    return fail(BGK_E_INVALID, "exactly one of bc_coef / bc_dense must be given");
  if (io->precision != TGS_FP64 && io->precision != TGS_FP32_CORRECTION)
    return fail(BGK_E_INVALID, "unknown precision");
  if ((d->d_lag || io->precision == TGS_FP32_CORRECTION) && !io->f_prev)
    return fail(BGK_E_INVALID, "f_prev is required with lagged facets or the FP32 form");
  if (io->f_prev && io->f_prev == io->f_out) return fail(BGK_E_INVALID, "f_out aliases f_prev");
  float* d32 = nullptr;
  if (io->precision == TGS_FP32_CORRECTION) {
    if (hipMallocAsync((void**)&d32, f_elems(d) * sizeof(float), (hipStream_t)stream) != hipSuccess)
      return fail(BGK_E_NOMEM, "correction buffer allocation failed");
  }
  int rc = launch_sweep(d, io, d32, (hipStream_t)stream);
  if (d32) (void)hipFreeAsync(d32, (hipStream_t)stream);
  return rc;
}

extern "C" int tgs_pack(const tgs_dag* d, const double* fc, double* fs, bgk_stream_t stream) {
  if (!d || !fc || !fs || (const void*)fc == (const void*)fs)
    return fail(BGK_E_INVALID, "bad arguments");
  const size_t total = f_elems(d);
  hipLaunchKernelGGL(k_pack, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, fc, fs,
                     d->d_pos, d->d_uid, (int)d->n_cells, d->n_v, d->n_p, 1);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

extern "C" int tgs_unpack(const tgs_dag* d, const double* fs, double* fc, bgk_stream_t stream) {
  if (!d || !fc || !fs || (const void*)fc == (const void*)fs)
    return fail(BGK_E_INVALID, "bad arguments");
  const size_t total = f_elems(d);
  hipLaunchKernelGGL(k_pack, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, fs, fc,
                     d->d_pos, d->d_uid, (int)d->n_cells, d->n_v, d->n_p, 0);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

extern "C" int tgs_eval_maxwellian(const tgs_dag* d, const double* coef, double* f,
                                   bgk_stream_t stream) {
  if (!d || !coef || !f) return fail(BGK_E_INVALID, "null argument");
  const size_t total = f_elems(d);
  if (d->dim == 2)
    hipLaunchKernelGGL(k_eval_maxw<2>, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream,
                       coef, f, d->d_perm, d->d_uid, d->d_v, (int)d->n_cells, d->n_v, d->n_p);
  else
    hipLaunchKernelGGL(k_eval_maxw<3>, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream,
                       coef, f, d->d_perm, d->d_uid, d->d_v, (int)d->n_cells, d->n_v, d->n_p);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}
