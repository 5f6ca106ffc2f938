// bgk_step: one DIRK time step (Sec. 3.5, App. A) whose stages are solved by
// the sweep-based Picard iteration (Sec. 4) with the stopping rule of
// eq. convergence-criteria.
//
// Stage bookkeeping (eq. q-stages, eq. dirk-recursive-def, eq. dirk-n) is
// carried as linear combinations over {f^k, f^(1), ..., f^(S)}:
//   F^(r) = f^(r)/(dt A_rr) - q^(r),
//   q^(s) = (f^k + dt sum_{r<s} A_sr F^(r)) / (dt A_ss),
//   f^{k+1} = f^k + dt sum_s b_s F^(s)   (= f^(S) for stiffly accurate tableaus).
// The first stage's source is f^k itself scaled inside the sweep (no extra
// pass); later stages materialise q^(s) with one fused combination kernel.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "device_common.h"
#include "kinetic_args.h"
#include "solver.h"
#include "sweep_args.h"
#include "walls.h"

namespace bgk {
int launch_nodal_perm(const tgs_dag* d, const double* src, double* dst, int to_internal,
                      hipStream_t stream);

// out = sum_i c_i x_i (NIN inputs, up to 5), grid-stride; out may be x0
// (each element is read before it is written by the same thread).  V = 2:
// pairs of doubles in 16-byte loads and stores (every pointer 16-byte
// aligned), the odd last element by the grid's first thread.  Each thread
// issues the loads of U grid-strided elements of every input before it
// combines any, so enough bytes are in flight to stream at the memory's
// rate; the arithmetic of each element is the same in every case.
template <int V, int NIN>
__global__ __launch_bounds__(256) void k_combine(double* out, const double* x0, const double* x1,
                                                 const double* x2, const double* x3,
                                                 const double* x4, double c0, double c1,
                                                 double c2, double c3, double c4, size_t n) {
  // the arrays are streamed once, with non-temporal loads and stores
  typedef double VT __attribute__((ext_vector_type(V)));
  constexpr int U = 4;
  const double* xs[5] = {x0, x1, x2, x3, x4};
  const double cs[5] = {c0, c1, c2, c3, c4};
  const size_t nv = n / V, stride = (size_t)gridDim.x * blockDim.x;
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < nv; i += U * stride) {
    VT t[NIN][U];
#pragma unroll
    for (int k = 0; k < NIN; ++k)
#pragma unroll
      for (int u = 0; u < U; ++u)
        t[k][u] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(xs[k]) + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      VT r;
#pragma unroll
      for (int e = 0; e < V; ++e) r[e] = cs[0] * t[0][u][e];
#pragma unroll
      for (int k = 1; k < NIN; ++k)
#pragma unroll
        for (int e = 0; e < V; ++e) r[e] = fma(cs[k], t[k][u][e], r[e]);
      __builtin_nontemporal_store(r, reinterpret_cast<VT*>(out) + i + u * stride);
    }
  }
  for (; i < nv; i += stride) {
    VT t[NIN];
#pragma unroll
    for (int k = 0; k < NIN; ++k)
      t[k] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(xs[k]) + i);
    VT r;
#pragma unroll
    for (int e = 0; e < V; ++e) r[e] = cs[0] * t[0][e];
#pragma unroll
    for (int k = 1; k < NIN; ++k)
#pragma unroll
      for (int e = 0; e < V; ++e) r[e] = fma(cs[k], t[k][e], r[e]);
    __builtin_nontemporal_store(r, reinterpret_cast<VT*>(out) + i);
  }
  if (V == 2 && (n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const size_t t = n - 1;
    double r = cs[0] * xs[0][t];
#pragma unroll
    for (int k = 1; k < NIN; ++k) r = fma(cs[k], xs[k][t], r);
    out[t] = r;
  }
}

// zero the per-iteration status words (a kernel, so the sequence stays
// capturable in a graph)
__global__ void k_reset(int32_t* status, unsigned long long* numax, const int32_t* skip) {
  if (threadIdx.x == 0 && !skip_launch(skip)) {
    status[0] = 0;
    status[1] = 0;
    *numax = 0ull;
  }
}

// control block of the chunked iteration at the start of a stage, and the
// status words of its first iteration
__global__ void k_ctl_init(int32_t* ctl, int32_t* status, unsigned long long* numax) {
  if (threadIdx.x < 8) ctl[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    reinterpret_cast<double*>(ctl)[4] = 0.0;
    status[0] = 0;
    status[1] = 0;
    *numax = 0ull;
  }
}

// The stopping test of one Picard iteration on the device (the host loop's
// rule: a non-physical or non-finite iterate fails the stage; with
// fixed_iters the count decides, else the max ratio of eq.
// convergence-criteria against tau / max(1, max nu dt); l_max iterations
// without stopping fail).  Once ctl[0] is set, later iterations skip.
// In the chunked iteration it first reduces the moment kernel's block pieces
// of the norms into the ratios (as k_ratio does) and afterwards clears the
// status words for the next iteration (the host loop's k_reset), so an
// iteration takes two launches fewer.
__global__ __launch_bounds__(256) void k_ratio_converge(
    int32_t* ctl, int32_t* __restrict__ status, unsigned long long* __restrict__ numax,
    const double* __restrict__ partial, int nblk, double* __restrict__ ratio, double tau,
    double dt, int fixed_iters, int l_max) {
  __shared__ double s[6][256];
  if (skip_launch(ctl)) return;
  ratio_block(partial, nblk, ratio, s);
  if (threadIdx.x != 0) return;
  const int32_t st0 = status[0], st1 = status[1];
  const unsigned long long nmax = *numax;
  status[0] = 0;
  status[1] = 0;
  *numax = 0ull;
  const int it = ctl[1] + 1;
  ctl[1] = it;
  ctl[2] += st0;
  if (st1 > 0) {
    ctl[0] = 2;
    ctl[3] = BGK_E_NONPHYSICAL;
    ctl[4] = st1;
    return;
  }
  const double last = ratio[3];
  reinterpret_cast<double*>(ctl)[4] = last;
  if (!isfinite(last)) {
    ctl[0] = 2;
    ctl[3] = BGK_E_NONPHYSICAL;
    return;
  }
  if (fixed_iters > 0) {
    if (it >= fixed_iters) {
      ctl[0] = 1;
      return;
    }
  } else {
    const double nm = __longlong_as_double((long long)nmax);
    if (last < tau / fmax(1.0, nm * dt)) {
      ctl[0] = 1;
      return;
    }
  }
  if (it >= l_max) {
    ctl[0] = 2;
    ctl[3] = BGK_E_NOT_CONVERGED;
  }
}

__global__ void k_clear_u8(uint8_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace bgk

using namespace bgk;


namespace bgk {

int set_tableau(bgk_solver* s, int tab) {
  std::memset(s->A, 0, sizeof(s->A));
  if (tab == BGK_TAB_BE) {
    s->S = 1;
    s->A[0][0] = 1.0;
    s->b[0] = 1.0;
  } else if (tab == BGK_TAB_DIRK2) {
    const double g = 1.0 - std::sqrt(2.0) / 2.0;
    s->S = 2;
    s->A[0][0] = g;
    s->A[1][0] = std::sqrt(2.0) / 2.0;
    s->A[1][1] = g;
    s->b[0] = s->A[1][0];
    s->b[1] = g;
  } else if (tab == BGK_TAB_DIRK3) {
    // gamma: the root of x^3 - 3x^2 + 3x/2 - 1/6 in (0.4, 0.5), by bisection
    double lo = 0.4, hi = 0.5;
    for (int i = 0; i < 200; ++i) {
      const double m = 0.5 * (lo + hi);
      if (m * m * m - 3 * m * m + 1.5 * m - 1.0 / 6.0 > 0) lo = m; else hi = m;
    }
    const double g = 0.5 * (lo + hi);
    s->S = 3;
    s->A[0][0] = s->A[1][1] = s->A[2][2] = g;
    s->A[1][0] = 0.5 * (1.0 - g);
    s->A[2][0] = -(6 * g * g - 16 * g + 1) / 4.0;
    s->A[2][1] = (6 * g * g - 20 * g + 5) / 4.0;
    for (int i = 0; i < 3; ++i) s->b[i] = s->A[2][i];
  } else if (tab == BGK_TAB_BDIRK2) {
    const double g = (3.0 + std::sqrt(3.0)) / 6.0;
    s->S = 2;
    s->A[0][0] = s->A[1][1] = g;
    s->A[1][0] = 1.0 - 2.0 * g;
    s->b[0] = s->b[1] = 0.5;
  } else {
    return fail(BGK_E_INVALID, "unknown tableau");
  }
  s->stiffly_accurate = true;
  for (int i = 0; i < s->S; ++i)
    if (s->b[i] != s->A[s->S - 1][i]) s->stiffly_accurate = false;
  // combination coefficients
  const double dt = s->opts.dt;
  std::memset(s->qcoef, 0, sizeof(s->qcoef));
  std::memset(s->Fcoef, 0, sizeof(s->Fcoef));
  std::memset(s->ncoef, 0, sizeof(s->ncoef));
  for (int st = 0; st < s->S; ++st) {
    double acc[5] = {1.0, 0, 0, 0, 0};
    for (int r = 0; r < st; ++r)
      for (int i = 0; i < 5; ++i) acc[i] += dt * s->A[st][r] * s->Fcoef[r][i];
    for (int i = 0; i < 5; ++i) s->qcoef[st][i] = acc[i] / (dt * s->A[st][st]);
    for (int i = 0; i < 5; ++i) s->Fcoef[st][i] = -s->qcoef[st][i];
    s->Fcoef[st][1 + st] += 1.0 / (dt * s->A[st][st]);
  }
  s->ncoef[0] = 1.0;
  for (int st = 0; st < s->S; ++st)
    for (int i = 0; i < 5; ++i) s->ncoef[i] += dt * s->b[st] * s->Fcoef[st][i];
  return BGK_OK;
}

}  // namespace bgk

namespace {

template <typename T>
int dmalloc(T** p, size_t n) {
  if (hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return fail(BGK_E_NOMEM, "solver workspace allocation failed");
  }
  return BGK_OK;
}

int combine(double* out, const double* const* xs, const double* cs, int nin, size_t n,
            hipStream_t stream) {
  const double* x[5] = {xs[0], nin > 1 ? xs[1] : xs[0], nin > 2 ? xs[2] : xs[0],
                        nin > 3 ? xs[3] : xs[0], nin > 4 ? xs[4] : xs[0]};
  double c[5] = {cs[0], nin > 1 ? cs[1] : 0, nin > 2 ? cs[2] : 0, nin > 3 ? cs[3] : 0,
                 nin > 4 ? cs[4] : 0};
  bool aligned = ((uintptr_t)out & 15) == 0;
  for (int i = 0; i < nin; ++i) aligned = aligned && ((uintptr_t)xs[i] & 15) == 0;
  const int V = aligned ? 2 : 1;
  // a large grid streams faster (2D workload, two inputs: 5.45 ms at up to
  // 131072 blocks against 5.96 at 8192)
  const int grid = std::max((int)std::min<size_t>((n / V + 255) / 256, 131072), 1);
#define BGK_COMB(V_, N_)                                                                      \
  hipLaunchKernelGGL((k_combine<V_, N_>), dim3(grid), dim3(256), 0, stream, out, x[0], x[1], \
                     x[2], x[3], x[4], c[0], c[1], c[2], c[3], c[4], n)
#define BGK_COMB_V(V_)                \
  switch (nin) {                      \
    case 1: BGK_COMB(V_, 1); break;   \
    case 2: BGK_COMB(V_, 2); break;   \
    case 3: BGK_COMB(V_, 3); break;   \
    case 4: BGK_COMB(V_, 4); break;   \
    default: BGK_COMB(V_, 5); break;  \
  }
  if (V == 2) {
    BGK_COMB_V(2)
  } else {
    BGK_COMB_V(1)
  }
#undef BGK_COMB_V
#undef BGK_COMB
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

}  // namespace

extern "C" int bgk_solver_create(const tgs_dag* d, const bgk_solver_opts* o, bgk_solver** out) {
  return guarded([&]() -> int {
    if (!d || !o || !out) return fail(BGK_E_INVALID, "null argument");
    *out = nullptr;
    if (!(o->dt > 0) || !(o->tau > 0) || o->l_max <= 0)
      return fail(BGK_E_INVALID, "dt, tau and l_max must be positive");
    if (!o->bc_coef) return fail(BGK_E_INVALID, "bc_coef is required");
    if (o->precision != TGS_FP64 && o->precision != TGS_FP32_CORRECTION)
      return fail(BGK_E_INVALID, "unknown precision");
    if (o->walls && walls_dag(o->walls) != d)
      return fail(BGK_E_INVALID, "walls belong to another DAG");
    if (o->maxw_mode == BGK_MAXW_PROJECTED && d->dg_cells <= 0)
      return fail(BGK_E_INVALID, "PROJECTED mode needs a Q2 velocity space (dg_cells > 0)");
    if (o->chunk_iters < 0) return fail(BGK_E_INVALID, "chunk_iters must be >= 0");
    if (o->chunk_iters > 1 && o->timing)
      return fail(BGK_E_INVALID, "per-kernel timing needs chunk_iters <= 1");
    bgk_solver* s = new (std::nothrow) bgk_solver();
    if (!s) return fail(BGK_E_NOMEM, "host allocation failed");
    s->dag = d;
    s->opts = *o;
    int rc = set_tableau(s, o->tableau);
    const size_t nf = f_elems(d);
    const size_t nn = (size_t)d->n_nodes * (d->dim + 2);
    if (!rc) rc = dmalloc(&s->fk, nf);
    for (int i = 0; i + 1 < s->S && !rc; ++i) rc = dmalloc(&s->fst[i], nf);
    if (!rc && !s->stiffly_accurate) rc = dmalloc(&s->fst[s->S - 1], nf);
    if (!rc && s->S > 1) rc = dmalloc(&s->q, nf);
    if (!rc && (d->d_lag || o->precision == TGS_FP32_CORRECTION)) rc = dmalloc(&s->fping, nf);
    if (!rc && o->precision == TGS_FP32_CORRECTION) rc = dmalloc(&s->d32, nf);
    if (!rc) rc = dmalloc(&s->U[0], nn);
    if (!rc) rc = dmalloc(&s->U[1], nn);
    if (!rc) rc = dmalloc(&s->mcoef, nn);
    if (!rc && d->n_1d > 0) rc = dmalloc(&s->mtab, maxw_table_size(d));
    if (!rc && o->maxw_mode == BGK_MAXW_PROJECTED) rc = dmalloc(&s->pr, proj_scratch_size(d));
    if (!rc) rc = dmalloc(&s->bcd, std::max<size_t>(1, (size_t)d->n_bfaces * d->n_fp * d->n_v));
    if (!rc) rc = dmalloc(&s->nu, (size_t)d->n_nodes);
    if (!rc) rc = dmalloc(&s->partial, (size_t)moment_partials(d) * 6);
    if (!rc && moment_split_doubles(d) > 0)
      rc = dmalloc(&s->msplit, (size_t)moment_split_doubles(d));
    if (!rc) rc = dmalloc(&s->ratio, 4);
    if (!rc) rc = dmalloc(&s->status, 2);
    if (!rc) rc = dmalloc(&s->numax, 1);
    if (!rc) rc = dmalloc(&s->sticky, (size_t)d->n_nodes);
    if (!rc) rc = dmalloc(&s->ctl, 16);
    if (!rc && o->chunk_iters > 1 && o->graph &&
        hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking) != hipSuccess)
      rc = fail(BGK_E_HIP, "hipStreamCreate failed");
    if (!rc && hipHostMalloc((void**)&s->h_info, 8 * sizeof(double)) != hipSuccess)
      rc = fail(BGK_E_NOMEM, "pinned host allocation failed");
    if (!rc && o->timing)
      for (int i = 0; i < 4 && !rc; ++i)
        if (hipEventCreate(&s->ev[i]) != hipSuccess) rc = fail(BGK_E_HIP, "hipEventCreate failed");
    if (rc) {
      bgk_solver_destroy(s);
      return rc;
    }
    *out = s;
    return BGK_OK;
  });
}

extern "C" int bgk_solver_destroy(bgk_solver* s) {
  return guarded([&]() -> int {
    if (!s) return BGK_OK;
    void* ptrs[] = {s->fk,    s->fst[0], s->fst[1], s->fst[2], s->fst[3], s->fping,
                    s->q,     s->d32,    s->U[0],   s->U[1],   s->mcoef,  s->mtab,
                    s->nu,    s->partial, s->ratio, s->status, s->numax, s->sticky, s->pr,
                    s->bcd,   s->ctl,    s->msplit};
    for (auto& g : s->graphs) (void)hipGraphExecDestroy(g.second);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    if (s->h_info) (void)hipHostFree(s->h_info);
    for (hipEvent_t e : s->ev)
      if (e) (void)hipEventDestroy(e);
    delete s;
    return BGK_OK;
  });
}

extern "C" int bgk_step(bgk_solver* s, double* f, const double* U_guess, double* U_out,
                        bgk_step_stats* stats, bgk_stream_t stream_) {
  return guarded([&]() -> int {
    if (!s || !f) return fail(BGK_E_INVALID, "null argument");
    const auto t0 = std::chrono::steady_clock::now();
    const tgs_dag* d = s->dag;
    const bgk_solver_opts& o = s->opts;
    hipStream_t stream = (hipStream_t)stream_;
    const size_t nf = f_elems(d);
    const size_t nn = (size_t)d->n_nodes * (d->dim + 2);
    const bool need_prev = d->d_lag != nullptr || o.precision == TGS_FP32_CORRECTION;
    bgk_step_stats st{};
    st.stages = s->S;
    int rc;
    // f^k is read by every stage's source and by the final combination.  The
    // last stage of a stiffly accurate tableau writes its iterates into f; with
    // two or more stages f^k is no longer needed by then (that stage's source
    // was formed before its first sweep), so only a one-stage tableau copies it
    const double* fk = f;
    if (s->stiffly_accurate && s->S == 1) {
      BGK_HIP(hipMemcpyAsync(s->fk, f, nf * sizeof(double), hipMemcpyDeviceToDevice, stream));
      fk = s->fk;
    }
    double* fst[4] = {s->fst[0], s->fst[1], s->fst[2], s->fst[3]};
    if (s->stiffly_accurate) fst[s->S - 1] = f;
    const double* stage_init = fk;   // initial Picard iterate of the stage
    int ucur = 0;
    // the sweep reads dense boundary data: the inflow facets' Maxwellians are
    // evaluated once per step (with walls, the wall facets' rows are replaced
    // before every sweep)
    if ((rc = launch_bc_dense(d, o.bc_coef, s->bcd, stream))) return rc;
    // nodal arrays (U, Maxwellian coefficients, nu) stay in the internal cell
    // order during the step; U_guess / U_out are in user order
    if (U_guess) {
      if ((rc = launch_nodal_perm(d, U_guess, s->U[0], 1, stream))) return rc;
    } else {
      if ((rc = launch_moments(d, fk, s->U[0], nullptr, nullptr, nullptr, stream, false,
                               s->msplit)))
        return rc;
    }
    const int K = o.chunk_iters > 1 ? o.chunk_iters : 1;
    const int nblk = moment_partials(d);  // pieces of the norms per moment pass
    // the buffer a Picard iteration writes, given the one it reads: with
    // lagged facets or the FP32 form the previous iterate must survive the
    // sweep, so iterates alternate between the stage's output and fping
    // (the first iteration reads the stage's initial iterate)
    const auto next_out = [&](const double* prev, double* out) -> double* {
      return need_prev ? (prev == out ? s->fping : out) : out;
    };
    for (int stg = 0; stg < s->S; ++stg) {
      const double shift = 1.0 / (o.dt * s->A[stg][stg]);
      const double* qsrc;
      double qscale;
      if (stg == 0) {
        qsrc = fk;
        qscale = s->qcoef[0][0];
      } else {
        const double* xs[5] = {fk, fst[0], fst[1], fst[2], fst[3]};
        if ((rc = combine(s->q, xs, s->qcoef[stg], stg + 1, nf, stream))) return rc;
        qsrc = s->q;
        qscale = 1.0;
      }
      double* out = fst[stg];
      // one Picard iteration reading moments U[ucur] and iterate prev,
      // writing U[ucur ^ 1] and cur_out; with `skip` every launch is a no-op
      // once the device-side stopping test has fired
      const auto enqueue_iter = [&](hipStream_t sm, int uc, const double* prv, double* cur,
                                    const int32_t* skip) -> int {
        int r;
        // the chunked iteration clears the status words and reduces the
        // norms in its stopping-test kernel
        if (!skip) hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, sm, s->status, s->numax, skip);
        if (o.timing) BGK_HIP(hipEventRecord(s->ev[0], sm));
        if ((r = launch_maxwellian(d, o.maxw_mode, s->U[uc], &o.nu_model, s->mcoef, s->nu,
                                   nullptr, s->status, s->numax, s->sticky, sm, skip)))
          return r;
        if (s->pr)
          r = launch_proj_tables(d, s->mcoef, s->nu, s->pr, s->mtab, sm, skip);
        else if (s->mtab)
          r = launch_maxw_tables(d, s->mcoef, s->nu, s->mtab, sm, skip);
        if (r) return r;
        if (o.timing) BGK_HIP(hipEventRecord(s->ev[1], sm));
        tgs_sweep_io io{};
        io.precision = o.precision;
        io.sigma_shift = shift;
        io.q_scale = qscale;
        io.nu = s->nu;
        io.mcoef = s->mcoef;
        io.q = qsrc;
        io.bc_coef = nullptr;
        io.bc_dense = s->bcd;
        io.f_prev = need_prev ? prv : nullptr;
        if (o.walls && (r = launch_wall_values(o.walls, prv, s->bcd, sm, skip))) return r;
        io.f_out = cur;
        if ((r = launch_sweep(d, &io, s->mtab, s->d32, sm, 0, skip))) return r;
        if (o.timing) BGK_HIP(hipEventRecord(s->ev[2], sm));
        if ((r = launch_moments(d, cur, s->U[uc ^ 1], s->U[uc], s->partial,
                                skip ? nullptr : s->ratio, sm, false, s->msplit, skip)))
          return r;
        if (o.timing) BGK_HIP(hipEventRecord(s->ev[3], sm));
        return BGK_OK;
      };
      // K iterations from (uc, prv), each followed by the device-side test
      const auto enqueue_chunk = [&](hipStream_t sm, int uc, const double* prv) -> int {
        for (int k = 0; k < K; ++k) {
          double* cur = next_out(prv, out);
          int r = enqueue_iter(sm, uc, prv, cur, s->ctl);
          if (r) return r;
          hipLaunchKernelGGL(k_ratio_converge, dim3(1), dim3(256), 0, sm, s->ctl, s->status,
                             s->numax, s->partial, nblk, s->ratio, o.tau, o.dt, o.fixed_iters,
                             o.l_max);
          BGK_HIP(hipGetLastError());
          uc ^= 1;
          prv = cur;
        }
        return BGK_OK;
      };
      const double* prev = stage_init;
      int it = 0;
      bool converged = false;
      double last = 0.0;
      // a node whose MATCHED solve fails stays on DIRECT for the rest of the
      // stage: an iterate switching between the two would not settle
      hipLaunchKernelGGL(k_clear_u8, dim3((unsigned)std::min<int64_t>((d->n_nodes + 255) / 256, 1024)),
                         dim3(256), 0, stream, s->sticky, d->n_nodes);
      if (K == 1) {
        while (it < o.l_max) {
          double* cur_out = next_out(prev, out);
          if ((rc = enqueue_iter(stream, ucur, prev, cur_out, nullptr))) return rc;
          BGK_HIP(hipMemcpyAsync(s->h_info, s->ratio, 4 * sizeof(double), hipMemcpyDeviceToHost,
                                 stream));
          BGK_HIP(hipMemcpyAsync(s->h_info + 4, s->numax, sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, stream));
          BGK_HIP(hipMemcpyAsync(s->h_info + 5, s->status, 2 * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, stream));
          BGK_HIP(hipStreamSynchronize(stream));
          if (o.timing) {
            float t01, t12, t23;
            BGK_HIP(hipEventElapsedTime(&t01, s->ev[0], s->ev[1]));
            BGK_HIP(hipEventElapsedTime(&t12, s->ev[1], s->ev[2]));
            BGK_HIP(hipEventElapsedTime(&t23, s->ev[2], s->ev[3]));
            st.maxwellian_ms += t01;
            st.sweep_ms += t12;
            st.moments_ms += t23;
          }
          ++st.sweeps;
          ++it;
          ucur ^= 1;
          prev = cur_out;
          int32_t stat[2];
          std::memcpy(stat, s->h_info + 5, sizeof(stat));
          st.maxw_fallbacks += stat[0];
          if (stat[1] > 0) {
            return fail(BGK_E_NONPHYSICAL, "non-physical moments (n <= 0 or theta <= 0) at " +
                                               std::to_string(stat[1]) + " nodes");
          }
          double numax;
          std::memcpy(&numax, s->h_info + 4, sizeof(double));
          last = s->h_info[3];
          if (!std::isfinite(last))
            return fail(BGK_E_NONPHYSICAL, "non-finite moments in the Picard iteration");
          if (o.fixed_iters > 0) {
            if (it >= o.fixed_iters) {
              converged = true;
              break;
            }
            continue;
          }
          if (last < o.tau / std::max(1.0, numax * o.dt)) {
            converged = true;
            break;
          }
        }
      } else {
        hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, stream, s->ctl, s->status, s->numax);
        BGK_HIP(hipGetLastError());
        int32_t done = 0;
        while (done == 0) {
          if (o.graph) {
            const ChunkKey key{stg, ucur, prev, out, fk, qsrc};
            hipGraphExec_t exec = nullptr;
            for (auto& g : s->graphs)
              if (g.first == key) exec = g.second;
            if (!exec) {
              if (s->graphs.size() >= 16) {
                for (auto& g : s->graphs) (void)hipGraphExecDestroy(g.second);
                s->graphs.clear();
              }
              BGK_HIP(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
              const int r = enqueue_chunk(s->cap, ucur, prev);
              hipGraph_t g = nullptr;
              const hipError_t e = hipStreamEndCapture(s->cap, &g);
              if (r || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return r ? r : fail(BGK_E_HIP, std::string("graph capture: ") +
                                                   hipGetErrorString(e));
              }
              const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
              (void)hipGraphDestroy(g);
              if (ei != hipSuccess)
                return fail(BGK_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
              s->graphs.emplace_back(key, exec);
            }
            BGK_HIP(hipGraphLaunch(exec, stream));
          } else if ((rc = enqueue_chunk(stream, ucur, prev))) {
            return rc;
          }
          BGK_HIP(hipMemcpyAsync(s->h_info, s->ctl, 16 * sizeof(int32_t), hipMemcpyDeviceToHost,
                                 stream));
          BGK_HIP(hipStreamSynchronize(stream));
          int32_t c[5];
          std::memcpy(c, s->h_info, sizeof(c));
          done = c[0];
          // the iterations that ran are a prefix of the chunk: follow their
          // buffer alternation
          for (int k = it; k < c[1]; ++k) {
            prev = next_out(prev, out);
            ucur ^= 1;
            ++st.sweeps;
          }
          it = c[1];
          last = s->h_info[4];
          if (done != 0) {
            st.maxw_fallbacks += c[2];
            if (done == 1) {
              converged = true;
            } else if (c[3] == BGK_E_NONPHYSICAL) {
              return c[4] > 0 ? fail(BGK_E_NONPHYSICAL,
                                     "non-physical moments (n <= 0 or theta <= 0) at " +
                                         std::to_string(c[4]) + " nodes")
                              : fail(BGK_E_NONPHYSICAL,
                                     "non-finite moments in the Picard iteration");
            }
          }
        }
      }
      if (prev != out) {
        BGK_HIP(hipMemcpyAsync(out, prev, nf * sizeof(double), hipMemcpyDeviceToDevice, stream));
      }
      st.iters[stg] = it;
      st.last_ratio[stg] = last;
      st.total_iters += it;
      if (!converged) {
        if (stats) *stats = st;
        return fail(BGK_E_NOT_CONVERGED, "Picard iteration reached l_max in stage " +
                                             std::to_string(stg + 1));
      }
      stage_init = out;
    }
    if (!s->stiffly_accurate) {
      const double* xs[5] = {fk, fst[0], fst[1], fst[2], fst[3]};
      if ((rc = combine(f, xs, s->ncoef, s->S + 1, nf, stream))) return rc;
      if (U_out &&
          (rc = launch_moments(d, f, s->U[ucur], nullptr, nullptr, nullptr, stream, false,
                               s->msplit)))
        return rc;
    }
    if (U_out && (rc = launch_nodal_perm(d, s->U[ucur], U_out, 0, stream))) return rc;
    BGK_HIP(hipStreamSynchronize(stream));
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return BGK_OK;
  });
}
