// tgs_sweep: the topological-generation sweep (Sec. 4.1) of the Picard
// iteration eq. bgk-ss-picard, plus layout conversion kernels.
//
// Mapping.  One workgroup owns one velocity j and walks that velocity's
// generations in order; each thread takes one cell of a generation (cells of
// a generation are a contiguous slot range of the sweep layout, so q and f
// stream through HBM coalesced).  Velocities are independent: there is no
// grid-wide barrier, only a workgroup barrier between generations.
//
// Per cell the thread assembles
//   A = |K| mass diag(sigma) - sum_b w_b stiff_b + sum_{v.N_k > 0} (v.N_k) fmass_k
//   b = |K| mass (nu*M + q_scale*q) + sum_{v.N_k < 0} |v.N_k| fmass_k fhat_k
// (w = |det J| J^{-1} v from the facet fluxes) with the reference matrices as
// compile-time integer tables, and solves A f = b in registers by Gaussian
// elimination without pivoting (A's symmetric part is positive definite:
// sigma > 0 plus the upwind facet terms).
//
// Latency.  Everything a cell needs except its upwind neighbours' new values
// (record, geometry, Maxwellian, sigma, source) is loaded ahead: in the
// pipelined walk (FP64) a whole solve ahead, over workgroup-sized chunks of
// the generations; in the plain walk (FP32 correction form, P1 triangles)
// the first chunk of the next generation before the barrier.  New values
// are also kept in an LDS ring of the last rs slots (a power of two, at
// least the workgroup size, at most RS); upwind reads are served from it
// when their slot is recent enough, so the per-generation barrier only
// orders LDS (s_waitcnt lgkmcnt + s_barrier) and global loads stay in
// flight across it.  Older upwind values are read from HBM after a full
// workgroup fence, which runs only when the ring no longer covers the
// generation's reach.
#include <climits>
#include <type_traits>

#include "device_common.h"
#include "sweep_args.h"
#include "walls.h"

namespace bgk {



// ---------------------------------------------------------------------------
// Integer-scaled reference tables.  Every normalised element integral is a
// rational whose denominator divides MS = (2k+d)!/d! (mass), SS = (2k-1+d)!
// (stiffness on the reference simplex) or FS = (2k+d-1)!/(d-1)! (facet
// mass); scaled by these the tables are small exact integers, so the kernel
// multiplies by integers and applies 1/MS, 1/SS, 1/FS once per cell.
// ---------------------------------------------------------------------------
constexpr double c_round(double x) {
  return x >= 0 ? (double)(long long)(x + 0.5) : -(double)(long long)(-x + 0.5);
}
constexpr double c_abs(double x) { return x < 0 ? -x : x; }

template <int DIM, int ORDER>
struct Scaled {
  using E = Elem<DIM, ORDER>;
  static constexpr int NP = E::NP, NF = E::NF, NFP = E::NFP;
  static constexpr double MS = cfact(2 * ORDER + DIM) / cfact(DIM);
  static constexpr double SS = cfact(2 * ORDER - 1 + DIM);
  static constexpr double FS = cfact(2 * ORDER + DIM - 1) / cfact(DIM - 1);
  struct Tab {
    double m[NP][NP] = {};
    double s[DIM][NP][NP] = {};
    double f[NF][NP][NP] = {};
    bool exact = true;
  };
  static constexpr Tab make() {
    Tab t;
    for (int a = 0; a < NP; ++a)
      for (int b = 0; b < NP; ++b) {
        const double m = E::T.mass[a][b] * MS;
        t.m[a][b] = c_round(m);
        if (c_abs(m - t.m[a][b]) > 1e-9) t.exact = false;
        for (int be = 0; be < DIM; ++be) {
          const double s = E::T.stiff[be][a][b] * SS;
          t.s[be][a][b] = c_round(s);
          if (c_abs(s - t.s[be][a][b]) > 1e-9) t.exact = false;
        }
        for (int k = 0; k < NF; ++k) {
          const double f = E::T.fmass[k][a][b] * FS;
          t.f[k][a][b] = c_round(f);
          if (c_abs(f - t.f[k][a][b]) > 1e-9) t.exact = false;
        }
      }
    return t;
  }
  static constexpr Tab T = make();
  static_assert(T.exact, "scaled reference tables must be integers");
};

template <int DIM, int ORDER>
struct SweepCfg {
  static constexpr int NP = Elem<DIM, ORDER>::NP;
  static constexpr int RS = (NP * 8 * 1024 <= 32768) ? 1024 : 512;  // LDS ring slots
};

// 1/x: hardware reciprocal estimate refined by two Newton steps (full
// double precision for the well-scaled pivots of the local systems).
__device__ __forceinline__ double recip(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Unpivoted LU in place: the multipliers below the diagonal, the
// reciprocal pivots on it, U above it.
template <int N, typename T>
__device__ __forceinline__ void lu_factor(T (&A)[N][N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const T inv = recip(A[k][k]);
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const T l = A[i][k] * inv;
#pragma unroll
      for (int c = k + 1; c < N; ++c) A[i][c] = fma(-l, A[k][c], A[i][c]);
      A[i][k] = l;
    }
    A[k][k] = inv;
  }
}

// Solves with lu_factor's result: forward elimination, back substitution
template <int N, typename T>
__device__ __forceinline__ void lu_apply(const T (&A)[N][N], T (&b)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int i = k + 1; i < N; ++i) b[i] = fma(-A[i][k], b[k], b[i]);
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    T s = b[i];
#pragma unroll
    for (int c = i + 1; c < N; ++c) s = fma(-A[i][c], b[c], s);
    b[i] = s * A[i][i];
  }
}

template <int N, typename T>
__device__ __forceinline__ void lu_solve(T (&A)[N][N], T (&b)[N]) {
  lu_factor<N, T>(A);
  lu_apply<N, T>(A, b);
}

// A cell prepared for its solve: everything but the upwind values.
template <int DIM, int ORDER>
struct Prep {
  static constexpr int NP = Elem<DIM, ORDER>::NP, NF = DIM + 1;
  int s;            // slot, -1: none
  int K;
  int code[NF];
  int pack;         // facet node maps (see tgs_dag::d_recx)
  double vol;
  double fl[NF];
  double w[DIM];
  double sig[NP];
  double src[NP];
};

template <int DIM>
__device__ __forceinline__ void load_rec(const SweepArgs& a, size_t base, int s, int& K,
                                         int (&code)[DIM + 1], int& pack) {
  const int4 r = reinterpret_cast<const int4*>(a.rec)[base + s];
  pack = a.recx[base + s];
  if (DIM == 2) {
    K = r.x;
    code[0] = r.y;
    code[1] = r.z;
    code[2] = r.w;
  } else {
    K = a.perm[base + s];
    code[0] = r.x;
    code[1] = r.y;
    code[2] = r.z;
    code[DIM] = r.w;
  }
}

// Raw inputs of one cell-velocity item, loaded a step before they are
// turned into a Prep (the pipelined walk): geometry, q, and either the
// Maxwellian factors of a tensor grid (TAB) or the node coefficients and nu.
template <int DIM, int ORDER, bool TAB>
struct Raw {
  static constexpr int NP = Elem<DIM, ORDER>::NP, NG = 1 + (DIM + 1) * DIM, NC = DIM + 2;
  static constexpr int NM = TAB ? 2 * NP : NP;                // (E_0, nu) pairs | nu
  static constexpr int NX = TAB ? NP : NP * NC;   // E_rest | coefficients
  double g[NG];
  double q[NP];
  double m[NM];
  double x[NX];
};

// Geometry taken from the table records (TabGeo): the last facet's
// area-weighted normal, g[1 + DIM*DIM ..], is minus the sum of the others
template <int DIM>
__device__ __forceinline__ void last_normal(double* g) {
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    double s = g[1 + d];
#pragma unroll
    for (int k = 1; k < DIM; ++k) s += g[1 + k * DIM + d];
    g[1 + DIM * DIM + d] = -s;
  }
}

// Plain loads of the raw inputs of slot s (cell K); nodal arrays in the
// internal cell order (no node map)
template <int DIM, int ORDER, bool TAB>
__device__ __forceinline__ void load_raw(const SweepArgs& a, size_t base, int s, int K,
                                         const double* const (&mrow)[2],
                                         Raw<DIM, ORDER, TAB>& R) {
  using RW = Raw<DIM, ORDER, TAB>;
  constexpr int NP = Elem<DIM, ORDER>::NP;
  constexpr bool TG = TAB && TabGeo<DIM, NP>::ON;
  if constexpr (!TG) {
    const double* __restrict__ gk = a.geo + (size_t)K * GeoLayout<DIM>::STRIDE;
#pragma unroll
    for (int i = 0; i < RW::NG; ++i) R.g[i] = gk[i];
  }
  const double* __restrict__ q = a.q + (base + s) * NP;
#pragma unroll
  for (int b = 0; b < NP; ++b) R.q[b] = q[b];
  const size_t u = (size_t)K;
  if constexpr (TAB) {
    constexpr int S0 = TabLayout::stride0(DIM, NP), S1 = TabLayout::stride1(DIM, NP);
    const double* __restrict__ e0 = mrow[0] + u * S0;
#pragma unroll
    for (int b = 0; b < RW::NM; ++b) R.m[b] = e0[b];
#pragma unroll
    for (int b = 0; b < NP; ++b) R.x[b] = mrow[1][u * S1 + b];
    if constexpr (TG) {
      using T = TabGeo<DIM, NP>;
#pragma unroll
      for (int i = 0; i < T::E0_N; ++i) R.g[i] = e0[T::E0_AT + i];
#pragma unroll
      for (int i = 0; i < T::REST_N; ++i) R.g[T::E0_N + i] = mrow[1][u * S1 + T::REST_AT + i];
    }
  } else {
#pragma unroll
    for (int b = 0; b < NP; ++b) R.m[b] = a.nu[u * NP + b];
    const double* __restrict__ mc = a.mcoef + u * NP * RW::NC;
#pragma unroll
    for (int i = 0; i < RW::NX; ++i) R.x[i] = mc[i];
  }
}

// the arithmetic of prepare<..., TAB>, in the same order, on loaded data
template <int DIM, int ORDER, bool TAB>
__device__ __forceinline__ void compute_prep(const SweepArgs& a, const double* v, double v2,
                                             const Raw<DIM, ORDER, TAB>& R,
                                             Prep<DIM, ORDER>& P) {
  using RW = Raw<DIM, ORDER, TAB>;
  constexpr int NP = Elem<DIM, ORDER>::NP, NF = DIM + 1;
  double g[RW::NG];
#pragma unroll
  for (int i = 0; i < RW::NG; ++i) g[i] = R.g[i];
  if constexpr (TAB && TabGeo<DIM, NP>::ON) last_normal<DIM>(g);
  P.vol = g[0];
  double raw[NF];
  facet_flux_raw<DIM>(g, v, v2, P.fl, raw);
  constexpr double wf = (DIM == 2) ? -1.0 : -2.0;
#pragma unroll
  for (int b = 0; b < DIM; ++b) P.w[b] = wf * raw[b + 1];
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    double M, nub;
    if constexpr (TAB) {
      M = R.m[2 * b] * R.x[b];
      nub = R.m[2 * b + 1];
    } else {
      M = maxw_eval<DIM>(R.x + b * RW::NC, v, v2);
      nub = R.m[b];
    }
    P.sig[b] = nub + a.sigma_shift;
    P.src[b] = fma(nub, M, a.q_scale * R.q[b]);
  }
}

template <int DIM, int ORDER, bool TAB>
__device__ __forceinline__ void prepare(const SweepArgs& a, const double* v, double v2,
                                        size_t base, const double* const (&mrow)[2],
                                        Prep<DIM, ORDER>& P) {
  constexpr int NP = Elem<DIM, ORDER>::NP, NF = DIM + 1, NC = DIM + 2;
  constexpr int NG = 1 + (DIM + 1) * DIM;
  const size_t u = (size_t)P.K;  // nodal arrays in the internal cell order
  double gk[NG];
  if constexpr (TAB && TabGeo<DIM, NP>::ON) {
    using T = TabGeo<DIM, NP>;
    const double* __restrict__ e0 = mrow[0] + u * TabLayout::stride0(DIM, NP);
    const double* __restrict__ er = mrow[1] + u * TabLayout::stride1(DIM, NP);
#pragma unroll
    for (int i = 0; i < T::E0_N; ++i) gk[i] = e0[T::E0_AT + i];
#pragma unroll
    for (int i = 0; i < T::REST_N; ++i) gk[T::E0_N + i] = er[T::REST_AT + i];
    last_normal<DIM>(gk);
  } else {
    const double* __restrict__ g = a.geo + (size_t)P.K * GeoLayout<DIM>::STRIDE;
#pragma unroll
    for (int i = 0; i < NG; ++i) gk[i] = g[i];
  }
  P.vol = gk[0];
  double raw[NF];
  facet_flux_raw<DIM>(gk, v, v2, P.fl, raw);
  constexpr double wf = (DIM == 2) ? -1.0 : -2.0;
#pragma unroll
  for (int b = 0; b < DIM; ++b) P.w[b] = wf * raw[b + 1];
  const double* __restrict__ q = a.q + (base + P.s) * NP;
  double M[NP], nu[NP];
  if constexpr (TAB) {
    // tensor grid: M = E_0[i_0][node] * E_rest[i_1..i_{d-1}][node]; the
    // first factor is stored interleaved with nu, so one gather brings both
    constexpr int S0 = TabLayout::stride0(DIM, NP), S1 = TabLayout::stride1(DIM, NP);
    const double* __restrict__ e0 = mrow[0] + u * S0;
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      M[b] = e0[2 * b] * mrow[1][u * S1 + b];
      nu[b] = e0[2 * b + 1];
    }
  } else {
#pragma unroll
    for (int b = 0; b < NP; ++b) nu[b] = a.nu[u * NP + b];
    const double* __restrict__ mc = a.mcoef + u * NP * NC;
#pragma unroll
    for (int b = 0; b < NP; ++b) M[b] = maxw_eval<DIM>(mc + b * NC, v, v2);
  }
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    const double nub = nu[b];
    P.sig[b] = nub + a.sigma_shift;
    P.src[b] = fma(nub, M[b], a.q_scale * q[b]);
  }
}

template <int DIM, int ORDER>
__device__ __forceinline__ void assemble(const Prep<DIM, ORDER>& P,
                                         double (&A)[Elem<DIM, ORDER>::NP][Elem<DIM, ORDER>::NP],
                                         double (&rhs)[Elem<DIM, ORDER>::NP]) {
  using S = Scaled<DIM, ORDER>;
  constexpr int NP = S::NP, NF = S::NF;
  const double vm = P.vol * (1.0 / S::MS);
  double vs[NP], ws[DIM], os[NF];
#pragma unroll
  for (int b = 0; b < NP; ++b) vs[b] = vm * P.sig[b];
#pragma unroll
  for (int be = 0; be < DIM; ++be) ws[be] = P.w[be] * (1.0 / S::SS);
#pragma unroll
  for (int k = 0; k < NF; ++k) os[k] = (P.fl[k] > 0.0 ? P.fl[k] : 0.0) * (1.0 / S::FS);
#pragma unroll
  for (int ia = 0; ia < NP; ++ia) {
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      double x = 0.0;
      if (S::T.m[ia][b] != 0.0) x = S::T.m[ia][b] * vs[b];
#pragma unroll
      for (int be = 0; be < DIM; ++be)
        if (S::T.s[be][ia][b] != 0.0) x = fma(-S::T.s[be][ia][b], ws[be], x);
#pragma unroll
      for (int k = 0; k < NF; ++k)
        if (S::T.f[k][ia][b] != 0.0) x = fma(S::T.f[k][ia][b], os[k], x);
      A[ia][b] = x;
    }
    double r = 0.0;
#pragma unroll
    for (int b = 0; b < NP; ++b)
      if (S::T.m[ia][b] != 0.0) r = fma(S::T.m[ia][b], P.src[b], r);
    rhs[ia] = vm * r;
  }
}

// Completes the load that produced x at this point: the empty asm reads x
// (so the compiler waits for that load here) and redefines it.  Used inside
// the rare branches that read global memory, so that code after the branch
// merge does not wait for outstanding loads: the vector-memory counter
// retires in order, and such a wait would also drain the loads prefetched
// for the following generations.
__device__ __forceinline__ void settle(double& x) { asm volatile("" : "+v"(x)); }

// upwind trace values of facet k at its nodes (in facet-node order)
template <int DIM, int ORDER, typename RT>
__device__ __forceinline__ void upwind_values(const SweepArgs& a, const Prep<DIM, ORDER>& P,
                                              int k, size_t base, int j, const double* v,
                                              double v2, const RT* ring, int rmask, int ring_lo,
                                              bool use_prev, double (&fh)[Elem<DIM, ORDER>::NFP]) {
  constexpr int NP = Elem<DIM, ORDER>::NP, NFP = Elem<DIM, ORDER>::NFP, NC = DIM + 2;
  constexpr int NB = NP <= 4 ? 2 : 3, NM = (1 << NB) - 1;
  const int c = P.code[k];
  if (c >= 0) {
    const int sl = c & REC_SLOT_MASK;
    const int pk = P.pack >> (NB * k * NFP);
    if (use_prev || (c & REC_LAG_BIT)) {
      const double* src = a.f_prev + (base + sl) * NP;
#pragma unroll
      for (int p = 0; p < NFP; ++p) fh[p] = src[(pk >> (NB * p)) & NM];
#pragma unroll
      for (int p = 0; p < NFP; ++p) settle(fh[p]);
    } else if (sl >= ring_lo) {
      const RT* src = ring + (sl & rmask) * NP;
#pragma unroll
      for (int p = 0; p < NFP; ++p) fh[p] = (double)src[(pk >> (NB * p)) & NM];
    } else {
      const double* src = a.f_out + (base + sl) * NP;
#pragma unroll
      for (int p = 0; p < NFP; ++p) fh[p] = src[(pk >> (NB * p)) & NM];
#pragma unroll
      for (int p = 0; p < NFP; ++p) settle(fh[p]);
    }
  } else {
    const size_t bf = (size_t)(-2 - c);
    if (a.bc_coef) {
#pragma unroll
      for (int p = 0; p < NFP; ++p) fh[p] = maxw_eval<DIM>(a.bc_coef + (bf * NFP + p) * NC, v, v2);
    } else {
#pragma unroll
      for (int p = 0; p < NFP; ++p) fh[p] = a.bc_dense[(bf * NFP + p) * a.n_v + j];
#pragma unroll
      for (int p = 0; p < NFP; ++p) settle(fh[p]);
    }
  }
}

// Issues the reads of facet k's upwind values without waiting for them: new
// values of recent slots from the LDS ring, older ones and lagged facets from
// HBM, boundary values from the dense boundary array (every launch of the
// FP64 sweep passes boundary data in dense form).
template <int DIM, int ORDER, typename RT>
__device__ __forceinline__ void fetch_upwind(const SweepArgs& a, const Prep<DIM, ORDER>& P, int k,
                                             size_t base, int j, const RT* ring, int rmask,
                                             int ring_lo, double (&fh)[Elem<DIM, ORDER>::NFP]) {
  constexpr int NP = Elem<DIM, ORDER>::NP, NFP = Elem<DIM, ORDER>::NFP;
  constexpr int NB = NP <= 4 ? 2 : 3, NM = (1 << NB) - 1;
  const int c = P.code[k];
  if (c >= 0) {
    const int sl = c & REC_SLOT_MASK;
    const int pk = P.pack >> (NB * k * NFP);
    if (c & REC_LAG_BIT) {
      const double* src = a.f_prev + (base + sl) * NP;
#pragma unroll
      for (int p = 0; p < NFP; ++p) fh[p] = src[(pk >> (NB * p)) & NM];
    } else if (sl >= ring_lo) {
      // the ring is LDS: an explicit LDS pointer keeps these reads apart from
      // the global ones in the other branches
      using lds_rt = __attribute__((address_space(3))) const RT;
      const lds_rt* src = (const lds_rt*)(ring + (sl & rmask) * NP);
#pragma unroll
      for (int p = 0; p < NFP; ++p) fh[p] = (double)src[(pk >> (NB * p)) & NM];
    } else {
      const double* src = a.f_out + (base + sl) * NP;
#pragma unroll
      for (int p = 0; p < NFP; ++p) fh[p] = src[(pk >> (NB * p)) & NM];
    }
    return;
  }
  const size_t bf = (size_t)(-2 - c);
#pragma unroll
  for (int p = 0; p < NFP; ++p) fh[p] = a.bc_dense[(bf * NFP + p) * a.n_v + j];
}

// The upwind values of every inflow facet of a prepared cell, read without
// waiting for them (facets with code -1 are left unset).
template <int DIM, int ORDER>
__device__ __forceinline__ void fetch_inflow(const SweepArgs& a, const Prep<DIM, ORDER>& P,
                                             size_t base, int j, const double* ring, int rmask,
                                             int ring_lo,
                                             double (&fh)[DIM + 1][Elem<DIM, ORDER>::NFP]) {
#pragma unroll
  for (int k = 0; k < DIM + 1; ++k)
    if (P.code[k] != -1) fetch_upwind<DIM, ORDER, double>(a, P, k, base, j, ring, rmask, ring_lo, fh[k]);
}

// FP64 solve of a prepared cell whose upwind values were fetched into fh:
// the local matrix is assembled (while those reads are in flight), the
// inflow terms are added in facet order, and the solution goes to rhs and,
// with RING, to the LDS ring.
template <int DIM, int ORDER, bool RING = true>
__device__ __forceinline__ void solve64_fetched(const Prep<DIM, ORDER>& P, double* ring, int rmask,
                                                double (&fh)[DIM + 1][Elem<DIM, ORDER>::NFP],
                                                double (&rhs)[Elem<DIM, ORDER>::NP]) {
  using S = Scaled<DIM, ORDER>;
  constexpr int NP = S::NP, NF = S::NF, NFP = S::NFP;
  double A[NP][NP];
  assemble<DIM, ORDER>(P, A, rhs);
  // the matrix does not depend on the upwind values: assemble and factor it
  // ahead of their first use, so the waits for their loads come after it
  lu_factor<NP, double>(A);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    if (P.code[k] == -1) continue;
    const double inflow = -P.fl[k] * (1.0 / S::FS);
#pragma unroll
    for (int ia = 0; ia < NFP; ++ia) {
      const int ra = Elem<DIM, ORDER>::T.fnode[k][ia];
      double r = 0.0;
#pragma unroll
      for (int p = 0; p < NFP; ++p)
        r = fma(S::T.f[k][ra][Elem<DIM, ORDER>::T.fnode[k][p]], fh[k][p], r);
      rhs[ra] = fma(inflow, r, rhs[ra]);
    }
  }
  lu_apply<NP, double>(A, rhs);
  if constexpr (RING) {
    double* rg = ring + (P.s & rmask) * NP;
#pragma unroll
    for (int b = 0; b < NP; ++b) rg[b] = rhs[b];
  }
}

// FP64 solve of a prepared cell into rhs, which also goes to the LDS ring
// (RING; without it every upwind value is read from HBM).  The upwind reads
// of every inflow facet are issued first, the local matrix is assembled while
// they are in flight, and the inflow terms are then added in facet order.
template <int DIM, int ORDER, bool RING = true>
__device__ __forceinline__ void solve64(const SweepArgs& a, const Prep<DIM, ORDER>& P, size_t base,
                                        int j, const double* v, double v2, double* ring,
                                        int rmask, int ring_lo,
                                        double (&rhs)[Elem<DIM, ORDER>::NP]) {
  double fh[DIM + 1][Elem<DIM, ORDER>::NFP];
  fetch_inflow<DIM, ORDER>(a, P, base, j, ring, rmask, ring_lo, fh);
  solve64_fetched<DIM, ORDER, RING>(P, ring, rmask, fh, rhs);
}

// FP64 solve of a prepared cell; the result goes to HBM and the LDS ring
template <int DIM, int ORDER, bool RING = true>
__device__ __forceinline__ void finish64(const SweepArgs& a, const Prep<DIM, ORDER>& P,
                                         size_t base, int j, const double* v, double v2,
                                         double* ring, int rmask, int ring_lo) {
  constexpr int NP = Elem<DIM, ORDER>::NP;
  double rhs[NP];
  solve64<DIM, ORDER, RING>(a, P, base, j, v, v2, ring, rmask, ring_lo, rhs);
  double* fo = a.f_out + (base + P.s) * NP;
#pragma unroll
  for (int b = 0; b < NP; ++b) fo[b] = rhs[b];
}

// FP32 defect correction of a prepared cell: FP64 residual of f_prev,
// FP32 solve for the correction with upwind correction traces, FP64 update.
template <int DIM, int ORDER>
__device__ __forceinline__ void finish32c(const SweepArgs& a, const Prep<DIM, ORDER>& P,
                                          size_t base, int j, const double* v, double v2,
                                          float* ring, int rmask, int ring_lo) {
  using S = Scaled<DIM, ORDER>;
  constexpr int NP = S::NP, NF = S::NF, NFP = S::NFP;
  double A[NP][NP], r[NP], fold[NP];
  assemble<DIM, ORDER>(P, A, r);
  const double* fp = a.f_prev + (base + P.s) * NP;
#pragma unroll
  for (int b = 0; b < NP; ++b) fold[b] = fp[b];
  // FP64 inflow of the previous iterate through every inflow facet
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    if (P.code[k] == -1) continue;
    double fh[NFP];
    upwind_values<DIM, ORDER, float>(a, P, k, base, j, v, v2, ring, rmask, ring_lo, true, fh);
    const double inflow = -P.fl[k] * (1.0 / S::FS);
#pragma unroll
    for (int ia = 0; ia < NFP; ++ia) {
      const int ra = Elem<DIM, ORDER>::T.fnode[k][ia];
      double acc = 0.0;
#pragma unroll
      for (int p = 0; p < NFP; ++p)
        acc = fma(S::T.f[k][ra][Elem<DIM, ORDER>::T.fnode[k][p]], fh[p], acc);
      r[ra] = fma(inflow, acc, r[ra]);
    }
  }
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
  // FP32 inflow of the corrections through non-lagged interior facets
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const int c = P.code[k];
    if (c < 0 || (c & REC_LAG_BIT)) continue;
    constexpr int NB = NP <= 4 ? 2 : 3, NM = (1 << NB) - 1;
    const int sl = c & REC_SLOT_MASK;
    const int pk = P.pack >> (NB * k * NFP);
    float dh[NFP];
    if (sl >= ring_lo) {
      const float* src = ring + (sl & rmask) * NP;
#pragma unroll
      for (int p = 0; p < NFP; ++p) dh[p] = src[(pk >> (NB * p)) & NM];
    } else {
      const float* src = a.d32 + (base + sl) * NP;
#pragma unroll
      for (int p = 0; p < NFP; ++p) dh[p] = src[(pk >> (NB * p)) & NM];
    }
    const float inflow = (float)(-P.fl[k] * (1.0 / S::FS));
#pragma unroll
    for (int ia = 0; ia < NFP; ++ia) {
      const int ra = Elem<DIM, ORDER>::T.fnode[k][ia];
      float acc = 0.0f;
#pragma unroll
      for (int p = 0; p < NFP; ++p)
        acc = fmaf((float)S::T.f[k][ra][Elem<DIM, ORDER>::T.fnode[k][p]], dh[p], acc);
      rf[ra] = fmaf(inflow, acc, rf[ra]);
    }
  }
  lu_solve<NP, float>(Af, rf);
  double* fo = a.f_out + (base + P.s) * NP;
  float* dg = a.d32 + (base + P.s) * NP;
  float* rg = ring + (P.s & rmask) * NP;
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    fo[b] = fold[b] + (double)rf[b];
    dg[b] = rf[b];
    rg[b] = rf[b];
  }
}

// Workgroup barrier that orders LDS only: global loads issued before it may
// stay in flight (the upwind values it protects live in the LDS ring).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One workgroup's walk over velocity j's generations; `ring` is LDS of
// SweepCfg::RS * NP values of the sweep's precision (rs * NP used).  PIPE takes the pipelined walk
// (FP64, nodal arrays in the internal order), which holds one cell's raw
// inputs in registers across a solve.
template <int DIM, int ORDER, bool F32, bool TAB, bool PIPE = false>
__device__ __forceinline__ void sweep_velocity(
    const SweepArgs& a, int j, typename std::conditional<F32, float, double>::type* ring) {
  constexpr int NF = DIM + 1;
  constexpr int NP = SweepCfg<DIM, ORDER>::NP;
  const int T = blockDim.x, tid = threadIdx.x;
  // ring slots: at least the workgroup size, so that two cells of one chunk
  // never share a ring slot (cells rs slots apart in a generation wider
  // than the ring are then separated by a barrier, below)
  int rs = a.ring_slots;
  while (rs < T) rs *= 2;
  const int rmask = rs - 1;
  double v[DIM], v2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    v[d] = a.v[(size_t)j * DIM + d];
    v2 = __fma_rn(v[d], v[d], v2);
  }
  const size_t base = (size_t)j * a.n_cells;
  // generation offsets and minimum upwind slots, read through the scalar
  // unit (constant address space: nothing writes them during the sweep):
  // their loads are then counted apart from the vector loads in flight, and
  // waiting for them does not drain the prefetched cell data
  using cint32 = __attribute__((address_space(4))) const int32_t;
  cint32* go = (cint32*)(a.goff + a.gbase[j]);
  cint32* gm = (cint32*)(a.gmin + a.gbase[j]);
  const int G = a.G[j];
  // rows of the factorised Maxwellian tables for this velocity (tensor
  // grids): axis 0's row and the rest's row; cell c's records are at
  // mrow[0] + c * s0 and mrow[1] + c * s1
  const double* mrow[2] = {nullptr, nullptr};
  if (a.mtab) {
    const TabLayout L(a.n_cells, a.n1, NP, DIM);
    mrow[0] = a.mtab + L.at(0, j / L.nr, 0);
    mrow[1] = a.mtab + L.at(1, j % L.nr, 0);
  }

  if constexpr (PIPE) {
    // Pipelined (FP64, no node map).  The walk is a sequence of steps, one per
    // T-cell chunk of a generation (a generation wider than the workgroup
    // takes several), with an LDS barrier after a generation's last chunk.
    // Step i: issue the record load of this thread's cell of step i+2, solve
    // step i, turn the raw inputs of step i+1 (loaded during step i-1) into
    // its Prep, issue the raw-input loads of step i+2, store step i's result.
    // Each load has a solve to complete under.  The vector-memory counter
    // retires in order, so a wait for one load waits for all issued before
    // it; the prefetch loads are therefore issued by every lane, whether or
    // not it has a cell in that step (an idle lane loads slot 0 and ignores
    // it), and a record is only copied between registers once it has arrived.
    static_assert(!F32, "the pipelined walk is FP64");
    using RawT = Raw<DIM, ORDER, TAB>;
    const auto next = [&](int& g, int& k) {
      if (g >= G) return;
      if (go[g] + (k + 1) * T < go[g + 1]) {
        ++k;
      } else {
        ++g;
        k = 0;
      }
    };
    const auto slot_of = [&](int g, int k) {
      if (g >= G) return -1;
      const int s = go[g] + k * T + tid;
      return s < go[g + 1] ? s : -1;
    };
    Prep<DIM, ORDER> P;
    RawT R, R2;
    int g0 = 0, k0 = 0;
    int g1 = 0, k1 = 0;
    next(g1, k1);
    int g2 = g1, k2 = k1;
    next(g2, k2);
    P.s = slot_of(g0, k0);
    if (P.s >= 0) {
      load_rec<DIM>(a, base, P.s, P.K, P.code, P.pack);
      prepare<DIM, ORDER, TAB>(a, v, v2, base, mrow, P);
    }
    // record of this thread's cell of step i+1 (its raw inputs are in R); a
    // slot of -1 marks an idle lane
    int n1s = slot_of(g1, k1), n1K = 0, n1code[NF], n1pack = 0;
    load_rec<DIM>(a, base, n1s >= 0 ? n1s : 0, n1K, n1code, n1pack);
    load_raw<DIM, ORDER, TAB>(a, base, n1s >= 0 ? n1s : 0, n1K, mrow, R);
    // record of step i+2, in flight at the start of step i
    int rsl = slot_of(g2, k2), rK, rcode[NF], rpack;
    load_rec<DIM>(a, base, rsl >= 0 ? rsl : 0, rK, rcode, rpack);
    int synced = 0;
    // One step of the walk (step i).  At its start `cur` holds the raw inputs
    // of step i+1 and the record of step i+2 is in flight, both issued a whole
    // step earlier.  The step issues step i's upwind reads, takes the record
    // of i+2 and issues its raw-input loads into `nxt`, issues the record load
    // of step i+3, then solves step i, turns `cur` into step i+1's Prep and
    // stores step i's result.  Every load has at least a whole step to
    // arrive, and the upwind reads, issued before the prefetches, are waited
    // for without waiting for those (the vector-memory counter retires in
    // order).  The loop alternates the two raw buffers and the record always
    // lands in the same registers, so no register that a load in flight will
    // write is copied at the loop's back edge (a copy would wait for it).
    const auto step = [&](RawT& cur, RawT& nxt) {
      const int s1 = go[g0 + 1];
      const int ring_lo = s1 - rs;
      if (k0 == 0 && gm[g0] < ring_lo && ring_lo > synced) {
        __syncthreads();
        synced = go[g0];
      }
      double fh[NF][Elem<DIM, ORDER>::NFP];
      if (P.s >= 0) fetch_inflow<DIM, ORDER>(a, P, base, j, ring, rmask, ring_lo, fh);
      // step i+2: its record (issued a step ago) and its raw-input loads
      const int n2s = rsl, n2K = rK, n2pack = rpack;
      int n2code[NF];
#pragma unroll
      for (int k = 0; k < NF; ++k) n2code[k] = rcode[k];
      load_raw<DIM, ORDER, TAB>(a, base, n2s >= 0 ? n2s : 0, n2K, mrow, nxt);
      // step i+3: its record
      int g3 = g2, k3 = k2;
      next(g3, k3);
      rsl = slot_of(g3, k3);
      load_rec<DIM>(a, base, rsl >= 0 ? rsl : 0, rK, rcode, rpack);
      // step i
      double out[NP];
      const int out_s = P.s;
      if (P.s >= 0) solve64_fetched<DIM, ORDER>(P, ring, rmask, fh, out);
      const bool last_chunk = go[g0] + (k0 + 1) * T >= s1;
      const bool wide = s1 - go[g0] > rs;
      // step i+1: Prep from the raw inputs loaded a step ago
      P.s = n1s;
      P.K = n1K;
      P.pack = n1pack;
#pragma unroll
      for (int k = 0; k < NF; ++k) P.code[k] = n1code[k];
      compute_prep<DIM, ORDER, TAB>(a, v, v2, cur, P);
      n1s = n2s;
      n1K = n2K;
      n1pack = n2pack;
#pragma unroll
      for (int k = 0; k < NF; ++k) n1code[k] = n2code[k];
      // step i's result
      if (out_s >= 0) {
        double* fo = a.f_out + (base + out_s) * NP;
#pragma unroll
        for (int b = 0; b < NP; ++b) fo[b] = out[b];
      }
      g0 = g1;
      k0 = k1;
      g1 = g2;
      k1 = k2;
      g2 = g3;
      k2 = k3;
      // after a generation's last chunk; and between the chunks of a
      // generation wider than the ring, whose cells rs slots apart share a
      // ring slot and must write it in slot order
      if (last_chunk || wide) lds_barrier();
    };
    while (g0 < G) {
      step(R, R2);
      if (g0 >= G) break;
      step(R2, R);
    }
    return;
  }

  Prep<DIM, ORDER> P;
  P.s = -1;
  if (go[0] + tid < go[1]) {
    P.s = go[0] + tid;
    load_rec<DIM>(a, base, P.s, P.K, P.code, P.pack);
    prepare<DIM, ORDER, TAB>(a, v, v2, base, mrow, P);
  }
  int ns = -1, nK = 0, ncode[NF], npack = 0;
  if (G > 1 && go[1] + tid < go[2]) {
    ns = go[1] + tid;
    load_rec<DIM>(a, base, ns, nK, ncode, npack);
  }
  int synced = 0;  // global stores of slots < synced are complete and visible
  for (int g = 0; g < G; ++g) {
    const int s0 = go[g], s1 = go[g + 1];
    const int ring_lo = s1 - rs;
    // values older than the ring come from HBM: fence only when this
    // generation reads one that may not be visible yet
    if (gm[g] < ring_lo && ring_lo > synced) {
      __syncthreads();
      synced = s0;
    }
    if (P.s >= 0) {
      if constexpr (F32)
        finish32c<DIM, ORDER>(a, P, base, j, v, v2, ring, rmask, ring_lo);
      else
        finish64<DIM, ORDER>(a, P, base, j, v, v2, ring, rmask, ring_lo);
    }
    // cells of a generation wider than the workgroup: further passes without
    // look-ahead, separated by a barrier when the generation is wider than
    // the ring (cells rs slots apart share a ring slot and must write it in
    // slot order)
    const bool wide = s1 - s0 > rs;
    for (int pass = s0 + T; pass < s1; pass += T) {
      if (wide) lds_barrier();
      const int s = pass + tid;
      if (s >= s1) continue;
      Prep<DIM, ORDER> Q;
      Q.s = s;
      load_rec<DIM>(a, base, s, Q.K, Q.code, Q.pack);
      prepare<DIM, ORDER, TAB>(a, v, v2, base, mrow, Q);
      if constexpr (F32)
        finish32c<DIM, ORDER>(a, Q, base, j, v, v2, ring, rmask, ring_lo);
      else
        finish64<DIM, ORDER>(a, Q, base, j, v, v2, ring, rmask, ring_lo);
    }
    // look-ahead: prepare this thread's cell of generation g+1, fetch the
    // record of generation g+2
    P.s = ns;
    if (ns >= 0) {
      P.K = nK;
      P.pack = npack;
#pragma unroll
      for (int k = 0; k < NF; ++k) P.code[k] = ncode[k];
      prepare<DIM, ORDER, TAB>(a, v, v2, base, mrow, P);
    }
    ns = -1;
    if (g + 3 <= G && go[g + 2] + tid < go[g + 3]) {
      ns = go[g + 2] + tid;
      load_rec<DIM>(a, base, ns, nK, ncode, npack);
    }
    lds_barrier();
  }
}

// Register budget: the plain P1-triangle walk fits 4 waves per SIMD; the
// pipelined walks and the other plain walks get 2 (up to 256 VGPRs, no
// spills): a sweep has at most a few velocities per CU resident anyway, and
// the spill-free kernel is faster (200k P2 triangles x 1024 velocities:
// 17.6 ms against 20.1 ms at 3, on the plain walk).
template <int DIM, int ORDER, bool F32, bool TAB, bool PIPE>
__global__ __launch_bounds__(256, (DIM == 2 && ORDER == 1 && !PIPE) ? 4 : 2) void k_sweep(SweepArgs a) {
  constexpr int RS = SweepCfg<DIM, ORDER>::RS, NP = SweepCfg<DIM, ORDER>::NP;
  using RT = typename std::conditional<F32, float, double>::type;
  __shared__ RT ring[RS * NP];
  if (skip_launch(a.skip)) return;
  sweep_velocity<DIM, ORDER, F32, TAB, PIPE>(a, a.vorder[blockIdx.x], ring);
}

// Packed walk (FP64): a 64-lane workgroup serves 64/L velocities, lane
// group t (lanes t L .. t L + L - 1) sweeping velocity vpack[block][t]
// through its generations L cells per step; every group advances one chunk
// per step, with a workgroup barrier between steps.  L = 1 is a thread
// walking its velocity's whole graph in order.  With 4 or more lanes per
// group each group keeps its last RS outputs in an LDS ring (RS a power of
// two >= 16 and >= L, from an 8 KB budget): a cell of generation g (slots
// [s0, s1)) reads upwind slots >= s1 - RS there, which no write of
// generation g can have overwritten (the same argument as the workgroup
// walk's ring), and older ones from memory; the barrier between steps then
// fences global memory only when some group is about to read such an older
// slot that may not be visible yet.  With 1 or 2 lanes (32-64 groups) the
// ring would hold too few slots to pay for its registers: every upwind
// value is read from memory, with a full fence between steps.  Each cell is
// prepared and solved by the same code as in the workgroup walk, so the
// results are bitwise equal.
template <int DIM, int ORDER, int L>
struct LanesCfg {
  static constexpr int NP = SweepCfg<DIM, ORDER>::NP, VPB = 64 / L;
  static constexpr int fit(int budget) {
    int r = 1;
    while (2 * r * VPB * NP * 8 <= budget) r *= 2;
    return r;
  }
  static constexpr int RS = fit(8192) < L ? L : fit(8192);
  static constexpr bool RING = RS >= 16;
};

// One 64-lane workgroup of the packed walk: lane group t sweeps velocity
// vblock[t] (-1: none).
template <int DIM, int ORDER, bool TAB, int L>
__device__ __forceinline__ void sweep_lanes_block(const SweepArgs& a,
                                                  const int32_t* __restrict__ vblock,
                                                  double* ring_all) {
  using C = LanesCfg<DIM, ORDER, L>;
  constexpr int NP = C::NP, RS = C::RS;
  const int lane = threadIdx.x, t = lane / L, r = lane - t * L;
  double* ring = ring_all + t * RS * NP;
  const int jj = vblock[t];
  const int j = jj < 0 ? 0 : jj;
  double v[DIM], v2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    v[d] = a.v[(size_t)j * DIM + d];
    v2 = __fma_rn(v[d], v[d], v2);
  }
  const size_t base = (size_t)j * a.n_cells;
  const int32_t* go = a.goff + a.gbase[j];
  const int32_t* gm = a.gmin + a.gbase[j];
  const int G = jj < 0 ? 0 : a.G[j];
  const double* mrow[2] = {nullptr, nullptr};
  if (a.mtab) {
    const TabLayout TL(a.n_cells, a.n1, NP, DIM);
    mrow[0] = a.mtab + TL.at(0, j / TL.nr, 0);
    mrow[1] = a.mtab + TL.at(1, j % TL.nr, 0);
  }
  int g = 0, s = 0, e = G > 0 ? go[1] : 0;
  int synced = 0;  // this group's slots below it are visible in global memory
  while (__ballot(g < G)) {
    // with the ring: a full fence when some group reads an upwind slot older
    // than its ring that was written after the last full fence
    const int ring_lo = C::RING ? e - RS : INT_MAX;
    if constexpr (C::RING) {
      const bool need = g < G && gm[g] < ring_lo && ring_lo > synced;
      if (__ballot(need)) {
        __syncthreads();
        synced = s;
      }
    }
    if (g < G) {
      if (s + r < e) {
        Prep<DIM, ORDER> P;
        P.s = s + r;
        load_rec<DIM>(a, base, P.s, P.K, P.code, P.pack);
        prepare<DIM, ORDER, TAB>(a, v, v2, base, mrow, P);
        finish64<DIM, ORDER, C::RING>(a, P, base, j, v, v2, ring, RS - 1, ring_lo);
      }
      s += L;
      if (s >= e) {
        ++g;
        s = e;
        if (g < G) e = go[g + 1];
      }
    }
    if constexpr (C::RING)
      lds_barrier();
    else
      __syncthreads();
  }
}

// P1 triangles on factorised tables fit five waves per SIMD (91 registers,
// no spills): 6.38 against 6.45-6.50 ms per sweep on the 3072-triangle strip
// with 36,864 velocities at L = 8, whose 4608 wavefronts then run at once
template <int DIM, int ORDER, bool TAB, int L>
__global__ __launch_bounds__(64, (DIM == 2 && ORDER == 1 && TAB) ? 5 : 1) void k_sweep_lanes(
    SweepArgs a) {
  using C = LanesCfg<DIM, ORDER, L>;
  __shared__ double ring_all[C::RING ? C::VPB * C::RS * C::NP : 1];
  if (skip_launch(a.skip)) return;
  sweep_lanes_block<DIM, ORDER, TAB, L>(a, a.vorder + blockIdx.x * C::VPB, ring_all);
}

// Batched packed walk: block b serves the 64/L velocities pvel[map[b].y ..]
// of instance map[b].x, unless that instance is done.
template <int DIM, int ORDER, bool TAB, int L>
__global__ __launch_bounds__(64) void k_sweep_batch_lanes(const SweepArgs* __restrict__ args,
                                                          const int2* __restrict__ map,
                                                          const int32_t* __restrict__ pvel,
                                                          const int32_t* __restrict__ done) {
  using C = LanesCfg<DIM, ORDER, L>;
  __shared__ double ring_all[C::RING ? C::VPB * C::RS * C::NP : 1];
  const int2 m = map[blockIdx.x];
  const int inst = __builtin_amdgcn_readfirstlane(m.x);
  const int off = __builtin_amdgcn_readfirstlane(m.y);
  if (done[inst]) return;
  const SweepArgs a = args[inst];
  sweep_lanes_block<DIM, ORDER, TAB, L>(a, pvel + off, ring_all);
}

// Batched FP64 sweep over many instances of one element type in one launch:
// block b sweeps velocity map[b].y (a position in its instance's velocity
// order) of instance map[b].x; instances flagged done skip.  One kernel per
// element type: a kernel holding both 2D walks would need the registers of
// both at once.
template <int DIM, int ORDER, bool TAB>
__global__ __launch_bounds__(256, 2) void k_sweep_batch(const SweepArgs* __restrict__ args,
                                                        const int2* __restrict__ map,
                                                        const int32_t* __restrict__ done) {
  constexpr int RS = SweepCfg<DIM, ORDER>::RS, NP = SweepCfg<DIM, ORDER>::NP;
  __shared__ double ring[RS * NP];
  // the block's instance and velocity are uniform: read them once through
  // the scalar unit, so the instance's arguments sit in scalar registers
  const int2 m = map[blockIdx.x];
  const int inst = __builtin_amdgcn_readfirstlane(m.x);
  const int vpos = __builtin_amdgcn_readfirstlane(m.y);
  if (done[inst]) return;
  const SweepArgs a = args[inst];
  const int j = __builtin_amdgcn_readfirstlane(a.vorder[vpos]);
  // batched instances are FP64 in the internal node order: pipelined walk on
  // factorised tables, the plain walk for node coefficients
  sweep_velocity<DIM, ORDER, false, TAB, TAB>(a, j, ring);
}

template <int DIM, int ORDER>
void launch_batch_kernel(bool tab, const SweepArgs* args, const BatchWalk& w, bool p1,
                         const int32_t* done, hipStream_t stream) {
  const int nb = p1 ? w.nb1 : w.nb2;
  const int2* map = p1 ? w.map + w.nb2 : w.map;
  if (w.lanes >= 64) {
    if (tab)
      hipLaunchKernelGGL((k_sweep_batch<DIM, ORDER, true>), dim3(nb), dim3(w.threads), 0, stream,
                         args, map, done);
    else
      hipLaunchKernelGGL((k_sweep_batch<DIM, ORDER, false>), dim3(nb), dim3(w.threads), 0,
                         stream, args, map, done);
    return;
  }
#define BGK_BL(L_)                                                                           \
  if (tab)                                                                                   \
    hipLaunchKernelGGL((k_sweep_batch_lanes<DIM, ORDER, true, L_>), dim3(nb), dim3(64), 0,   \
                       stream, args, map, w.pvel, done);                                     \
  else                                                                                       \
    hipLaunchKernelGGL((k_sweep_batch_lanes<DIM, ORDER, false, L_>), dim3(nb), dim3(64), 0,  \
                       stream, args, map, w.pvel, done);
  switch (w.lanes) {
    case 1: BGK_BL(1) break;
    case 2: BGK_BL(2) break;
    case 4: BGK_BL(4) break;
    case 8: BGK_BL(8) break;
    case 16: BGK_BL(16) break;
    default: BGK_BL(32) break;
  }
#undef BGK_BL
}

int launch_sweep_batch(int dim, bool tab, const SweepArgs* args, const BatchWalk& w,
                       const int32_t* done, hipStream_t stream, hipStream_t side, hipEvent_t fork,
                       hipEvent_t join) {
  if (dim == 3) {
    if (w.nb1 > 0) launch_batch_kernel<3, 1>(tab, args, w, true, done, stream);
    BGK_HIP(hipGetLastError());
    return BGK_OK;
  }
  if (w.nb2 > 0 && w.nb1 > 0) {
    // P1 instances on the side stream, forked from and joined back to the
    // main stream (under graph capture the two become parallel branches)
    BGK_HIP(hipEventRecord(fork, stream));
    BGK_HIP(hipStreamWaitEvent(side, fork, 0));
    launch_batch_kernel<2, 1>(tab, args, w, true, done, side);
    BGK_HIP(hipGetLastError());
    launch_batch_kernel<2, 2>(tab, args, w, false, done, stream);
    BGK_HIP(hipGetLastError());
    BGK_HIP(hipEventRecord(join, side));
    BGK_HIP(hipStreamWaitEvent(stream, join, 0));
    return BGK_OK;
  }
  if (w.nb2 > 0) launch_batch_kernel<2, 2>(tab, args, w, false, done, stream);
  if (w.nb1 > 0) launch_batch_kernel<2, 1>(tab, args, w, true, done, stream);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

// ring slots: the DAG's choice, else the most the element type's LDS ring holds
int ring_slots(const tgs_dag* d) {
  const int max = d->dim == 3 ? SweepCfg<3, 1>::RS : d->order == 1 ? SweepCfg<2, 1>::RS
                                                                   : SweepCfg<2, 2>::RS;
  return d->ring_slots > 0 ? std::min(d->ring_slots, max) : max;
}

SweepArgs make_sweep_args(const tgs_dag* d, const tgs_sweep_io* io,
                          const double* mtab, float* d32) {
  return SweepArgs{d->d_geo,   d->d_facet, d->d_v,      d->d_rec,   d->d_recx,  d->d_perm,
                   d->d_goff,  d->d_gmin,  d->d_gbase,  d->d_G,     d->d_vorder, io->nu,
                   io->mcoef,  mtab,       io->q,       io->bc_coef, io->bc_dense, io->f_prev,
                   io->f_out,  d32,        io->sigma_shift, io->q_scale, (int)d->n_cells, d->n_v,
                   d->n_1d,    ring_slots(d), d->order, nullptr};
}

int launch_sweep(const tgs_dag* d, const tgs_sweep_io* io, const double* mtab, float* d32,
                 hipStream_t stream, int threads, const int32_t* skip) {
  SweepArgs a = make_sweep_args(d, io, mtab, d32);
  a.skip = skip;
  const bool fp32 = io->precision == TGS_FP32_CORRECTION;
  if (threads <= 0) threads = d->sweep_threads;
  if (threads <= 0) {
    // 128 threads: the fastest measured on 200k P2 triangles x 1024
    // velocities (14.1 ms against 15.8 at 64, 15.5 at 192 and 14.8 at 256
    // threads), on 55k tetrahedra x 4096 velocities (15.9 ms against 17.6,
    // 16.9 and 16.5) and, pipelined, on 200k P1 triangles x 1024 velocities
    // (10.42 ms against 10.79, 12.31 and 10.46); smaller workgroups keep
    // more velocities per CU resident, and wider generations take a second
    // pass.  The plain P1-triangle walk (FP32 form, node coefficients): 256
    const bool plain_p1 = d->dim == 2 && d->order == 1 && (fp32 || !mtab);
    threads = plain_p1 ? 256 : 128;
  }
  if (!fp32 && d->sweep_lanes < 64) {
    SweepArgs ap = a;
    ap.vorder = d->d_vpack;
    const dim3 pgrid(d->vpack_blocks), pblock(64);
#define BGK_LANES(D_, O_, L_)                                                                \
  if (mtab)                                                                                \
    hipLaunchKernelGGL((k_sweep_lanes<D_, O_, true, L_>), pgrid, pblock, 0, stream, ap);   \
  else                                                                                     \
    hipLaunchKernelGGL((k_sweep_lanes<D_, O_, false, L_>), pgrid, pblock, 0, stream, ap);
#define BGK_LANES_L(D_, O_)   \
  switch (d->sweep_lanes) {   \
    case 1: BGK_LANES(D_, O_, 1) break;   \
    case 2: BGK_LANES(D_, O_, 2) break;   \
    case 4: BGK_LANES(D_, O_, 4) break;   \
    case 8: BGK_LANES(D_, O_, 8) break;   \
    case 16: BGK_LANES(D_, O_, 16) break; \
    default: BGK_LANES(D_, O_, 32) break; \
  }
    if (d->dim == 2 && d->order == 1) {
      BGK_LANES_L(2, 1)
    } else if (d->dim == 2 && d->order == 2) {
      BGK_LANES_L(2, 2)
    } else {
      BGK_LANES_L(3, 1)
    }
#undef BGK_LANES_L
#undef BGK_LANES
    BGK_HIP(hipGetLastError());
    return BGK_OK;
  }
  const dim3 grid(d->n_v), block(threads);
  // FP64 sweeps on factorised tables take the pipelined walk (sweeps that
  // evaluate the Maxwellian from node coefficients keep the plain walk:
  // their inputs do not fit twice in registers).  P1 triangles run it at
  // three waves per SIMD (165 registers) instead of the plain walk's four:
  // 10.5 against 12.4 ms on 200k P1 triangles x 1024 velocities, 0.74
  // against 0.80 ms per step on the 512-triangle case
#define BGK_LAUNCH(D_, O_)                                                                 \
  if (fp32 && mtab)                                                                        \
    hipLaunchKernelGGL((k_sweep<D_, O_, true, true, false>), grid, block, 0, stream, a);   \
  else if (fp32)                                                                           \
    hipLaunchKernelGGL((k_sweep<D_, O_, true, false, false>), grid, block, 0, stream, a);  \
  else if (mtab)                                                                           \
    hipLaunchKernelGGL((k_sweep<D_, O_, false, true, true>), grid, block, 0, stream, a);   \
  else                                                                                     \
    hipLaunchKernelGGL((k_sweep<D_, O_, false, false, false>), grid, block, 0, stream, a);
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

int grid_for(size_t total) {
  size_t g = (total + 255) / 256;
  return (int)std::min<size_t>(g, 65536);
}

}  // namespace bgk

using namespace bgk;

extern "C" int tgs_sweep(const tgs_dag* d, const tgs_sweep_io* io, bgk_stream_t stream) {
  return guarded([&]() -> int {
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
    // the kernels read nodal arrays in the internal cell order: nu and the
    // coefficients are permuted into scratch first; on a tensor velocity grid
    // the factorised Maxwellian tables are built from them, as in bgk_step, so
    // this is the solver's sweep kernel
    hipStream_t st = (hipStream_t)stream;
    const int np = d->n_p, nm = d->dim + 2;
    const size_t ntab = d->n_1d > 0 ? maxw_table_size(d) : 0;
    // boundary Maxwellians given by coefficients are evaluated once into the
    // dense boundary array the sweep reads
    const size_t nbc = io->bc_coef ? (size_t)d->n_bfaces * d->n_fp * d->n_v : 0;
    float* d32 = nullptr;
    double* nodal = nullptr;  // [n_nodes] nu, [n_nodes][dim+2] coefficients, tables, boundary
    if (hipMallocAsync((void**)&nodal,
                       ((size_t)d->n_nodes * (1 + nm) + ntab + nbc) * sizeof(double),
                       st) != hipSuccess)
      return fail(BGK_E_NOMEM, "scratch allocation failed");
    if (io->precision == TGS_FP32_CORRECTION &&
        hipMallocAsync((void**)&d32, f_elems(d) * sizeof(float), st) != hipSuccess) {
      (void)hipFreeAsync(nodal, st);
      return fail(BGK_E_NOMEM, "correction buffer allocation failed");
    }
    tgs_sweep_io io_i = *io;
    io_i.nu = nodal;
    io_i.mcoef = nodal + d->n_nodes;
    double* tab = ntab ? nodal + (size_t)d->n_nodes * (1 + nm) : nullptr;
    int rc = BGK_OK;
    if (nbc) {
      double* bcd = nodal + (size_t)d->n_nodes * (1 + nm) + ntab;
      rc = launch_bc_dense(d, io->bc_coef, bcd, st);
      io_i.bc_coef = nullptr;
      io_i.bc_dense = bcd;
    }
    if (!rc) rc = launch_nodal_rows(d, io->nu, nodal, np, 1, st);
    if (!rc) rc = launch_nodal_rows(d, io->mcoef, nodal + d->n_nodes, np * nm, 1, st);
    if (!rc && tab) rc = launch_maxw_tables(d, io_i.mcoef, io_i.nu, tab, st);
    if (!rc) rc = launch_sweep(d, &io_i, tab, d32, st, 0);
    if (d32) (void)hipFreeAsync(d32, st);
    (void)hipFreeAsync(nodal, st);
    return rc;
  });
}

extern "C" int tgs_pack(const tgs_dag* d, const double* fc, double* fs, bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!d || !fc || !fs || (const void*)fc == (const void*)fs)
      return fail(BGK_E_INVALID, "bad arguments");
    const size_t total = f_elems(d);
    hipLaunchKernelGGL(k_pack, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, fc, fs,
                       d->d_pos, d->d_uid, (int)d->n_cells, d->n_v, d->n_p, 1);
    BGK_HIP(hipGetLastError());
    return BGK_OK;
  });
}

extern "C" int tgs_unpack(const tgs_dag* d, const double* fs, double* fc, bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!d || !fc || !fs || (const void*)fc == (const void*)fs)
      return fail(BGK_E_INVALID, "bad arguments");
    const size_t total = f_elems(d);
    hipLaunchKernelGGL(k_pack, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, fs, fc,
                       d->d_pos, d->d_uid, (int)d->n_cells, d->n_v, d->n_p, 0);
    BGK_HIP(hipGetLastError());
    return BGK_OK;
  });
}

extern "C" int tgs_eval_maxwellian(const tgs_dag* d, const double* coef, double* f,
                                   bgk_stream_t stream) {
  return guarded([&]() -> int {
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
  });
}
