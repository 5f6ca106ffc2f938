// Batched stepping of many independent instances (an addition to the
// paper's method): every DIRK stage's Picard iteration (Sec. 4) runs for all
// instances at once — one launch each of the Maxwellian, the factorised
// tables, the sweep (a persistent launch over every instance's velocities,
// longest DAGs first), the moments and the convergence test — with the
// per-instance stopping rule of eq. convergence-criteria evaluated on the
// device.  An instance that has converged (or failed) is skipped by every
// later kernel of the stage, so a fixed chunk of iterations can be captured
// once in a hipGraph and replayed until every instance is done; the host
// polls one small control block per chunk.
//
// Per instance the arithmetic is that of bgk_step (same kernels' bodies,
// same combination order), so a batched step equals the single-instance
// step bit for bit.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <vector>

#include "device_common.h"
#include "kinetic_args.h"
#include "solver.h"
#include "sweep_args.h"
#include "walls.h"

namespace bgk {
namespace {

struct CombArgs {
  double* out;
  const double* x[5];
  double c[5];
  int nin;
  int64_t n;
};

struct ConvArgs {
  double tau, dt;
  int l_max, fixed_iters;
};

// out = sum_i c_i x_i per instance (blockIdx.y); same operation order as the
// single-instance combination.  Instances with done[i] == 2 (failed) skip.
__global__ void k_combine_batch(const CombArgs* __restrict__ args, const int32_t* __restrict__ done) {
  const int i = blockIdx.y;
  if (done && done[i] == 2) return;
  const CombArgs& a = args[i];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < a.n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = a.c[0] * a.x[0][e];
    if (a.nin > 1) s = fma(a.c[1], a.x[1][e], s);
    if (a.nin > 2) s = fma(a.c[2], a.x[2][e], s);
    if (a.nin > 3) s = fma(a.c[3], a.x[3][e], s);
    if (a.nin > 4) s = fma(a.c[4], a.x[4][e], s);
    a.out[e] = s;
  }
}

// control block, one entry per instance
struct Ctl {
  int32_t* done;       // 0 running, 1 stage converged, 2 failed
  int32_t* par;        // current moments are U[par]
  int32_t* iters;      // Picard iterations in the current stage
  int32_t* fallbacks;  // MATCHED fallbacks over the step
  int32_t* err;        // error code of a failed instance
  double* last;        // last max ratio
};

__global__ void k_step_init(Ctl c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  c.done[i] = 0;
  c.par[i] = 1;  // the initial moment pass writes U[par ^ 1] = U[0]
  c.iters[i] = 0;
  c.fallbacks[i] = 0;
  c.err[i] = 0;
  c.last[i] = 0.0;
}

__global__ void k_set_par(int32_t* par, int value, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) par[i] = value;
}

__global__ void k_stage_init(Ctl c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (c.done[i] != 2) c.done[i] = 0;
  c.iters[i] = 0;
}

__global__ void k_clear_bytes(uint8_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void k_iter_reset(const int32_t* __restrict__ done, int32_t* status,
                             unsigned long long* numax, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || done[i]) return;
  status[2 * i] = 0;
  status[2 * i + 1] = 0;
  numax[i] = 0ull;
}

// The stopping rule of one Picard iteration per instance (as bgk_step).
__global__ void k_converge(Ctl c, const ConvArgs* __restrict__ conv,
                           const int32_t* __restrict__ status,
                           const unsigned long long* __restrict__ numax,
                           const double* __restrict__ ratio, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || c.done[i]) return;
  const int it = c.iters[i] + 1;
  c.iters[i] = it;
  c.par[i] ^= 1;  // the new moments are current
  c.fallbacks[i] += status[2 * i];
  if (status[2 * i + 1] > 0) {
    c.done[i] = 2;
    c.err[i] = BGK_E_NONPHYSICAL;
    return;
  }
  const double last = ratio[4 * i + 3];
  c.last[i] = last;
  if (!isfinite(last)) {
    c.done[i] = 2;
    c.err[i] = BGK_E_NONPHYSICAL;
    return;
  }
  const ConvArgs& a = conv[i];
  if (a.fixed_iters > 0) {
    if (it >= a.fixed_iters) c.done[i] = 1;
    return;
  }
  const double nm = __longlong_as_double((long long)numax[i]);
  if (last < a.tau / fmax(1.0, nm * a.dt)) {
    c.done[i] = 1;
    return;
  }
  if (it >= a.l_max) {
    c.done[i] = 2;
    c.err[i] = BGK_E_NOT_CONVERGED;
  }
}

template <typename T>
int dalloc(T** p, size_t n) {
  if (hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return fail(BGK_E_NOMEM, "batch allocation failed");
  }
  return BGK_OK;
}

}  // namespace
}  // namespace bgk

using namespace bgk;

struct bgk_batch {
  int n = 0, dim = 0, S = 1;
  bool stiffly_accurate = true, tab = false;
  bgk_batch_opts opts{};
  std::vector<bgk_solver*> solvers;
  std::vector<double*> f_bound;      // caller f pointers the device arguments refer to
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;        // the P1 sweep kernel of mixed 2D batches
  hipEvent_t ev_in = nullptr, ev_out = nullptr, t0 = nullptr, t1 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // device arrays
  SweepArgs* sargs = nullptr;        // [S][n]
  SweepArgs* sargs_tune = nullptr;   // [n]
  BatchKin* kin = nullptr;           // [S + 2][n]: 0 init (f^k), 1 + s stage s, S + 1 caller f
  CombArgs* comb = nullptr;          // [S + 1][n]: 0 copy f -> f^k, s q^(s), S final
  ConvArgs* conv = nullptr;          // [n]
  int2* map = nullptr;               // sweep blocks: P2 instances' first, then P1's
  int nb2 = 0, nb1 = 0;
  // packed-walk block maps by lanes per velocity (built on first use, kept:
  // captured graphs refer to them)
  struct Packed {
    int2* map = nullptr;
    int32_t* pvel = nullptr;
    int nb2 = 0, nb1 = 0;
  };
  std::map<int, Packed> packed;
  int32_t* mom_first = nullptr;      // [n + 1]
  int mom_blocks = 0;
  int32_t* mx_inst = nullptr;        // Maxwellian blocks (128 nodes of one instance): instance
  int32_t* mx_first = nullptr;       // [n + 1] first Maxwellian block of each instance
  int mx_blocks = 0;
  int64_t n_nodes = 0;
  int64_t* tab_first = nullptr;      // [n + 1]
  int64_t n_tab = 0;
  int32_t* ctl_mem = nullptr;        // done, par, iters, fallbacks, err: 5n
  double* last = nullptr;            // [n]
  int32_t* status = nullptr;         // [2n]
  unsigned long long* numax = nullptr;  // [n]
  double* ratio = nullptr;           // [4n]
  double* partial = nullptr;         // moment block norms, per instance slices
  uint8_t* sticky = nullptr;         // [n_nodes]
  // host mirror of the control block (pinned): done, iters, fallbacks, err, last
  int32_t* h_ctl = nullptr;          // [5n]
  double* h_last = nullptr;          // [n]
  std::vector<hipGraphExec_t> exec;  // per stage, when graph capture is on
  std::vector<hipGraph_t> graphs;

  Ctl ctl() const {
    return Ctl{ctl_mem, ctl_mem + n, ctl_mem + 2 * n, ctl_mem + 3 * n, ctl_mem + 4 * n, last};
  }
};

namespace {

int batch_upload(bgk_batch* B, double* const* f) {
  const int n = B->n, S = B->S;
  std::vector<SweepArgs> sargs((size_t)S * n), tune(n);
  std::vector<BatchKin> kin((size_t)(S + 2) * n);
  std::vector<CombArgs> comb((size_t)(S + 1) * n);
  int64_t pfirst = 0;
  std::vector<int64_t> pbase(n);
  for (int i = 0; i < n; ++i) {
    pbase[i] = pfirst;
    pfirst += moment_blocks(B->solvers[i]->dag) * 6;
  }
  std::vector<int64_t> nfirst(n + 1, 0);
  for (int i = 0; i < n; ++i) nfirst[i + 1] = nfirst[i] + B->solvers[i]->dag->n_nodes;
  for (int i = 0; i < n; ++i) {
    bgk_solver* s = B->solvers[i];
    const tgs_dag* d = s->dag;
    const bgk_solver_opts& o = s->opts;
    const size_t nf = f_elems(d);
    double* out[4] = {s->fst[0], s->fst[1], s->fst[2], s->fst[3]};
    if (B->stiffly_accurate) out[S - 1] = f[i];
    double* mtab = B->tab ? s->mtab : nullptr;
    for (int st = 0; st < S; ++st) {
      tgs_sweep_io io{};
      io.precision = TGS_FP64;
      io.sigma_shift = 1.0 / (o.dt * s->A[st][st]);
      io.q_scale = st == 0 ? s->qcoef[0][0] : 1.0;
      io.nu = s->nu;
      io.mcoef = s->mcoef;
      io.q = st == 0 ? s->fk : s->q;
      io.bc_dense = s->bcd;
      io.f_out = out[st];
      sargs[(size_t)st * n + i] = make_sweep_args(d, &io, mtab, nullptr);
    }
    {
      // autotuning probe: read the caller's f as the source, write f^k
      tgs_sweep_io io{};
      io.precision = TGS_FP64;
      io.sigma_shift = 1.0 / (o.dt * s->A[0][0]);
      io.q_scale = s->qcoef[0][0];
      io.nu = s->nu;
      io.mcoef = s->mcoef;
      io.q = f[i];
      io.bc_dense = s->bcd;
      io.f_out = s->fk;
      tune[i] = make_sweep_args(d, &io, mtab, nullptr);
    }
    for (int k = 0; k < S + 2; ++k) {
      BatchKin& b = kin[(size_t)k * n + i];
      b = BatchKin{};
      b.maxw.coef = s->mcoef;
      b.maxw.nu = s->nu;
      b.maxw.M_dense = nullptr;
      b.maxw.status = B->status + 2 * i;
      b.maxw.numax = B->numax + i;
      b.maxw.v = d->d_v;
      b.maxw.w = d->d_w;
      b.maxw.x1 = d->d_nodes1d;
      b.maxw.w1 = d->d_weights1d;
      b.maxw.n1 = d->n_1d;
      b.maxw.n_v = d->n_v;
      b.maxw.n_nodes = d->n_nodes;
      b.maxw.mode = o.maxw_mode;
      b.maxw.nu_kind = o.nu_model.kind;
      b.maxw.nu_const = o.nu_model.nu_const;
      b.maxw.kn = o.nu_model.kn;
      b.maxw.L = d->L;
      b.maxw.dg_cells = d->dg_cells;
      b.maxw.sticky = B->sticky + nfirst[i];
      const double* mf = k == 0 ? s->fk : (k <= S ? out[k - 1] : f[i]);
      b.mom = MomArgs{mf,      d->d_pos, nullptr, d->d_v, d->d_w, nullptr, nullptr,
                      B->partial + pbase[i], (int)d->n_cells, d->n_v};
      b.U[0] = s->U[0];
      b.U[1] = s->U[1];
      b.mtab = mtab;
      b.geo = d->d_geo;
      b.x1 = d->d_nodes1d;
      b.n1 = d->n_1d;
      b.mom_vl = moment_vl(d);
      b.mom_blocks = moment_blocks(d);
      b.np = d->n_p;
      b.n_nodes = d->n_nodes;
      b.ratio = B->ratio + 4 * i;
    }
    const double* xs[5] = {s->fk, out[0], out[1], out[2], out[3]};
    for (int k = 0; k <= S; ++k) {
      CombArgs& c = comb[(size_t)k * n + i];
      c = CombArgs{};
      c.n = (int64_t)nf;
      if (k == 0) {  // f -> f^k
        c.out = s->fk;
        c.x[0] = f[i];
        c.c[0] = 1.0;
        c.nin = 1;
      } else if (k < S) {  // stage source q^(k)
        c.out = s->q;
        c.nin = k + 1;
        for (int r = 0; r < c.nin; ++r) {
          c.x[r] = xs[r];
          c.c[r] = s->qcoef[k][r];
        }
      } else {  // f^{k+1} for tableaus that are not stiffly accurate
        c.out = f[i];
        c.nin = S + 1;
        for (int r = 0; r < c.nin; ++r) {
          c.x[r] = xs[r];
          c.c[r] = s->ncoef[r];
        }
      }
      for (int r = c.nin; r < 5; ++r) c.x[r] = c.x[0];
    }
  }
  // the sweep reads dense boundary data: each instance's inflow Maxwellians,
  // evaluated once (batched instances have no walls)
  for (int i = 0; i < n; ++i) {
    const bgk_solver* s = B->solvers[i];
    int rc = launch_bc_dense(s->dag, s->opts.bc_coef, s->bcd, B->stream);
    if (rc) return rc;
  }
  BGK_HIP(hipMemcpyAsync(B->sargs, sargs.data(), sargs.size() * sizeof(SweepArgs),
                         hipMemcpyHostToDevice, B->stream));
  BGK_HIP(hipMemcpyAsync(B->sargs_tune, tune.data(), tune.size() * sizeof(SweepArgs),
                         hipMemcpyHostToDevice, B->stream));
  BGK_HIP(hipMemcpyAsync(B->kin, kin.data(), kin.size() * sizeof(BatchKin), hipMemcpyHostToDevice,
                         B->stream));
  BGK_HIP(hipMemcpyAsync(B->comb, comb.data(), comb.size() * sizeof(CombArgs),
                         hipMemcpyHostToDevice, B->stream));
  // the host vectors go out of scope: wait for the copies
  BGK_HIP(hipStreamSynchronize(B->stream));
  B->f_bound.assign(f, f + B->n);
  return BGK_OK;
}

int launch_combine(bgk_batch* B, int k, const int32_t* done) {
  hipLaunchKernelGGL(k_combine_batch, dim3(256, B->n), dim3(256), 0, B->stream,
                     B->comb + (size_t)k * B->n, done);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

dim3 inst_grid(int n) { return dim3((unsigned)((n + 63) / 64)); }

// The packed walk's blocks for `lanes` per velocity: each instance's
// velocities in direction order, 64/lanes to a block (angular neighbours,
// whose graphs are alike, so a block's lane groups finish together); P2
// instances' blocks first, then P1's, each part longest generation count
// first.
int packed_map(bgk_batch* B, int lanes, const bgk_batch::Packed** out) {
  auto it = B->packed.find(lanes);
  if (it == B->packed.end()) {
    const int vpb = 64 / lanes;
    std::vector<std::pair<int, int2>> blocks[2];
    std::vector<int32_t> pvel;
    for (int i = 0; i < B->n; ++i) {
      const tgs_dag* d = B->solvers[i]->dag;
      const std::vector<int32_t> order = angular_order(d);
      auto& part = blocks[d->dim == 2 && d->order == 2 ? 0 : 1];
      for (int b0 = 0; b0 < d->n_v; b0 += vpb) {
        const int off = (int)pvel.size();
        int gmax = 0;
        for (int t = 0; t < vpb; ++t) {
          const int j = b0 + t < d->n_v ? order[b0 + t] : -1;
          pvel.push_back(j);
          if (j >= 0) gmax = std::max(gmax, d->G_host[j]);
        }
        part.push_back({gmax, make_int2(i, off)});
      }
    }
    std::vector<int2> map;
    for (auto& part : blocks) {
      std::stable_sort(part.begin(), part.end(),
                       [](const std::pair<int, int2>& a, const std::pair<int, int2>& b) {
                         return a.first > b.first;
                       });
      for (const auto& b : part) map.push_back(b.second);
    }
    bgk_batch::Packed P;
    P.nb2 = (int)blocks[0].size();
    P.nb1 = (int)blocks[1].size();
    int rc = dalloc(&P.map, map.size());
    if (!rc) rc = dalloc(&P.pvel, pvel.size());
    if (!rc && (hipMemcpy(P.map, map.data(), map.size() * sizeof(int2), hipMemcpyHostToDevice) !=
                    hipSuccess ||
                hipMemcpy(P.pvel, pvel.data(), pvel.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice) != hipSuccess))
      rc = fail(BGK_E_HIP, "copy of the packed-walk map failed");
    if (rc) {
      if (P.map) (void)hipFree(P.map);
      if (P.pvel) (void)hipFree(P.pvel);
      return rc;
    }
    it = B->packed.emplace(lanes, P).first;
  }
  *out = &it->second;
  return BGK_OK;
}

// the walk of a batched sweep: the workgroup walk with `threads` (lanes 0
// or 64) or the packed walk with `lanes` per velocity
int batch_walk(bgk_batch* B, int threads, int lanes, BatchWalk* w) {
  if (lanes <= 0 || lanes >= 64) {
    *w = BatchWalk{threads, 64, B->map, B->nb2, B->nb1, nullptr};
    return BGK_OK;
  }
  const bgk_batch::Packed* P = nullptr;
  const int rc = packed_map(B, lanes, &P);
  if (rc) return rc;
  *w = BatchWalk{64, lanes, P->map, P->nb2, P->nb1, P->pvel};
  return BGK_OK;
}

bool valid_lanes(int lanes) {
  return lanes == 0 || lanes == 64 ||
         (lanes > 0 && lanes <= 32 && (lanes & (lanes - 1)) == 0);
}

// one Picard iteration of stage st for every running instance
int run_iteration(bgk_batch* B, int st, const SweepArgs* sargs, const BatchWalk& walk) {
  const int n = B->n;
  const Ctl c = B->ctl();
  const BatchKin* kin = B->kin + (size_t)(1 + st) * n;
  int rc;
  hipLaunchKernelGGL(k_iter_reset, inst_grid(n), dim3(64), 0, B->stream, c.done, B->status,
                     B->numax, n);
  BGK_HIP(hipGetLastError());
  if ((rc = launch_maxwellian_batch(B->dim, kin, c.par, c.done, B->mx_inst, B->mx_first, B->mx_blocks,
                                    B->stream)))
    return rc;
  if (B->tab &&
      (rc = launch_tables_batch(B->dim, kin, c.done, B->tab_first, n, B->n_tab, B->stream)))
    return rc;
  if ((rc = launch_sweep_batch(B->dim, B->tab, sargs, walk, c.done, B->stream, B->side,
                               B->ev_fork, B->ev_join)))
    return rc;
  if ((rc = launch_moments_batch(B->dim, kin, c.par, c.done, B->mom_first, n, B->mom_blocks, true,
                                 B->stream)))
    return rc;
  hipLaunchKernelGGL(k_converge, inst_grid(n), dim3(64), 0, B->stream, c, B->conv, B->status,
                     B->numax, B->ratio, n);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int run_chunk(bgk_batch* B, int st) {
  // the walk's maps were built at creation: nothing here allocates or copies
  BatchWalk walk;
  int rc = batch_walk(B, B->opts.sweep_threads, B->opts.sweep_lanes, &walk);
  for (int k = 0; k < B->opts.chunk_iters && !rc; ++k)
    rc = run_iteration(B, st, B->sargs + (size_t)st * B->n, walk);
  return rc;
}

int capture_graphs(bgk_batch* B) {
  B->graphs.assign(B->S, nullptr);
  B->exec.assign(B->S, nullptr);
  for (int st = 0; st < B->S; ++st) {
    BGK_HIP(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
    const int rc = run_chunk(B, st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(B->stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(BGK_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    B->graphs[st] = g;
    BGK_HIP(hipGraphInstantiate(&B->exec[st], g, nullptr, nullptr, 0));
  }
  return BGK_OK;
}

}  // namespace

extern "C" int bgk_batch_create(bgk_solver* const* solvers, int n, const bgk_batch_opts* opts,
                                bgk_batch** out) {
  return guarded([&]() -> int {
    if (!solvers || n <= 0 || !out) return fail(BGK_E_INVALID, "bad arguments");
    *out = nullptr;
    bgk_batch_opts o{};
    if (opts) o = *opts;
    if (o.chunk_iters <= 0) o.chunk_iters = 4;
    if (o.sweep_threads <= 0) o.sweep_threads = 128;
    if (o.sweep_threads % 64 || o.sweep_threads > 256)
      return fail(BGK_E_INVALID, "sweep_threads must be a multiple of 64 up to 256");
    if (!valid_lanes(o.sweep_lanes))
      return fail(BGK_E_INVALID, "sweep_lanes must be 0, 64 or a power of two up to 32");
    const bgk_solver* s0 = solvers[0];
    if (!s0) return fail(BGK_E_INVALID, "null solver");
    bool tab = true;
    int64_t n_nodes = 0, n_tab = 0, mx_total = 0;
    for (int i = 0; i < n; ++i) {
      const bgk_solver* s = solvers[i];
      if (!s) return fail(BGK_E_INVALID, "null solver");
      const tgs_dag* d = s->dag;
      if (d->dim != s0->dag->dim) return fail(BGK_E_UNSUPPORTED, "instances must share the dimension");
      if (s->opts.tableau != s0->opts.tableau)
        return fail(BGK_E_UNSUPPORTED, "instances must share the tableau");
      if (s->opts.precision != TGS_FP64)
        return fail(BGK_E_UNSUPPORTED, "batched stepping runs the FP64 sweep");
      if (d->d_lag) return fail(BGK_E_UNSUPPORTED, "batched stepping needs acyclic sweep graphs");
      if (d->dim == 3 && d->order != 1) return fail(BGK_E_UNSUPPORTED, "3D instances must be P1");
      if (s->opts.maxw_mode == BGK_MAXW_PROJECTED)
        return fail(BGK_E_UNSUPPORTED, "batched stepping has no projected Maxwellian");
      if (s->opts.walls) return fail(BGK_E_UNSUPPORTED, "batched stepping has no wall boundaries");
      tab = tab && s->mtab != nullptr;
      n_nodes += d->n_nodes;
      mx_total += (d->n_nodes + 127) / 128;
    }
    if (mx_total > INT32_MAX) return fail(BGK_E_INVALID, "too many nodes in the batch");
    bgk_batch* B = new (std::nothrow) bgk_batch();
    if (!B) return fail(BGK_E_NOMEM, "host allocation failed");
    B->n = n;
    B->dim = s0->dag->dim;
    B->S = s0->S;
    B->stiffly_accurate = s0->stiffly_accurate;
    B->tab = tab;
    B->opts = o;
    B->solvers.assign(solvers, solvers + n);
    B->n_nodes = n_nodes;
    int rc = BGK_OK;
    auto check = [&](hipError_t e, const char* what) {
      if (!rc && e != hipSuccess) rc = fail(BGK_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    };
    check(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking), "hipStreamCreate");
    check(hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking), "hipStreamCreate");
    check(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming), "hipEventCreate");
    check(hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming), "hipEventCreate");
    check(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming), "hipEventCreate");
    check(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming), "hipEventCreate");
    check(hipEventCreate(&B->t0), "hipEventCreate");
    check(hipEventCreate(&B->t1), "hipEventCreate");
    // per-instance layout tables
    std::vector<int64_t> tfirst(n + 1, 0);
    std::vector<int32_t> mfirst(n + 1, 0), xfirst(n + 1, 0), xinst;
    int64_t npart = 0;
    for (int i = 0; i < n; ++i) {
      const tgs_dag* d = solvers[i]->dag;
      const int64_t nb = (d->n_nodes + 127) / 128;
      xfirst[i + 1] = xfirst[i] + (int32_t)nb;
      xinst.insert(xinst.end(), (size_t)nb, i);
      tfirst[i + 1] =
          tfirst[i] + (tab ? table_threads(d->dim, d->n_cells, d->n_1d, d->n_p) : 0);  // table threads
      mfirst[i + 1] = mfirst[i] + moment_blocks(d);
      npart += (int64_t)moment_blocks(d) * 6;
    }
    n_tab = tfirst[n];
    B->n_tab = n_tab;
    B->mom_blocks = mfirst[n];
    // sweep blocks: every instance's velocities, P2 instances' first, each
    // part longest generation count first
    std::vector<std::pair<int, int2>> blocks[2];
    for (int i = 0; i < n && !rc; ++i) {
      const tgs_dag* d = solvers[i]->dag;
      std::vector<int32_t> vorder(d->n_v);
      check(hipMemcpy(vorder.data(), d->d_vorder, d->n_v * sizeof(int32_t), hipMemcpyDeviceToHost),
            "hipMemcpy");
      auto& part = blocks[d->dim == 2 && d->order == 2 ? 0 : 1];
      for (int y = 0; y < d->n_v; ++y) part.push_back({d->G_host[vorder[y]], make_int2(i, y)});
    }
    std::vector<int2> map;
    for (auto& part : blocks) {
      std::stable_sort(part.begin(), part.end(),
                       [](const std::pair<int, int2>& a, const std::pair<int, int2>& b) {
                         return a.first > b.first;
                       });
      for (const auto& b : part) map.push_back(b.second);
    }
    B->nb2 = (int)blocks[0].size();
    B->nb1 = (int)blocks[1].size();
    std::vector<ConvArgs> conv(n);
    for (int i = 0; i < n; ++i) {
      const bgk_solver_opts& so = solvers[i]->opts;
      conv[i] = ConvArgs{so.tau, so.dt, so.l_max, so.fixed_iters};
    }
    if (!rc) rc = dalloc(&B->sargs, (size_t)B->S * n);
    if (!rc) rc = dalloc(&B->sargs_tune, (size_t)n);
    if (!rc) rc = dalloc(&B->kin, (size_t)(B->S + 2) * n);
    if (!rc) rc = dalloc(&B->comb, (size_t)(B->S + 1) * n);
    if (!rc) rc = dalloc(&B->conv, (size_t)n);
    if (!rc) rc = dalloc(&B->map, map.size());
    if (!rc) rc = dalloc(&B->mom_first, (size_t)n + 1);
    B->mx_blocks = xfirst[n];
    if (!rc) rc = dalloc(&B->mx_inst, xinst.size());
    if (!rc) rc = dalloc(&B->mx_first, (size_t)n + 1);
    if (!rc) rc = dalloc(&B->tab_first, (size_t)n + 1);
    if (!rc) rc = dalloc(&B->ctl_mem, (size_t)5 * n);
    if (!rc) rc = dalloc(&B->last, (size_t)n);
    if (!rc) rc = dalloc(&B->status, (size_t)2 * n);
    if (!rc) rc = dalloc(&B->numax, (size_t)n);
    if (!rc) rc = dalloc(&B->ratio, (size_t)4 * n);
    if (!rc) rc = dalloc(&B->partial, (size_t)npart);
    if (!rc) rc = dalloc(&B->sticky, (size_t)n_nodes);
    if (!rc && hipHostMalloc((void**)&B->h_ctl, (size_t)5 * n * sizeof(int32_t)) != hipSuccess)
      rc = fail(BGK_E_NOMEM, "pinned allocation failed");
    if (!rc && hipHostMalloc((void**)&B->h_last, (size_t)n * sizeof(double)) != hipSuccess)
      rc = fail(BGK_E_NOMEM, "pinned allocation failed");
    if (!rc) {
      check(hipMemcpy(B->map, map.data(), map.size() * sizeof(int2), hipMemcpyHostToDevice), "hipMemcpy");
      check(hipMemcpy(B->mom_first, mfirst.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice),
            "hipMemcpy");
      check(hipMemcpy(B->mx_inst, xinst.data(), xinst.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice), "hipMemcpy");
      check(hipMemcpy(B->mx_first, xfirst.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice),
            "hipMemcpy");
      check(hipMemcpy(B->tab_first, tfirst.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice),
            "hipMemcpy");
      check(hipMemcpy(B->conv, conv.data(), n * sizeof(ConvArgs), hipMemcpyHostToDevice), "hipMemcpy");
    }
    // the packed walk's map now, so that captured chunks find it built
    BatchWalk walk;
    if (!rc) rc = batch_walk(B, o.sweep_threads, o.sweep_lanes, &walk);
    if (rc) {
      bgk_batch_destroy(B);
      return rc;
    }
    *out = B;
    return BGK_OK;
  });
}

extern "C" int bgk_batch_destroy(bgk_batch* B) {
  return guarded([&]() -> int {
    if (!B) return BGK_OK;
    for (hipGraphExec_t e : B->exec)
      if (e) (void)hipGraphExecDestroy(e);
    for (hipGraph_t g : B->graphs)
      if (g) (void)hipGraphDestroy(g);
    void* ptrs[] = {B->sargs,  B->sargs_tune, B->kin,    B->comb,   B->conv,   B->map,
                    B->mom_first, B->mx_inst, B->mx_first, B->tab_first, B->ctl_mem, B->last,
                    B->status,
                    B->numax,  B->ratio,      B->partial, B->sticky};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    for (auto& kv : B->packed) {
      if (kv.second.map) (void)hipFree(kv.second.map);
      if (kv.second.pvel) (void)hipFree(kv.second.pvel);
    }
    if (B->h_ctl) (void)hipHostFree(B->h_ctl);
    if (B->h_last) (void)hipHostFree(B->h_last);
    hipEvent_t evs[] = {B->ev_in, B->ev_out, B->t0, B->t1, B->ev_fork, B->ev_join};
    for (hipEvent_t e : evs)
      if (e) (void)hipEventDestroy(e);
    if (B->side) (void)hipStreamDestroy(B->side);
    if (B->stream) (void)hipStreamDestroy(B->stream);
    delete B;
    return BGK_OK;
  });
}

extern "C" int bgk_batch_step(bgk_batch* B, double* const* f, bgk_batch_stats* stats,
                              bgk_stream_t stream_) {
  return guarded([&]() -> int {
    if (!B || !f) return fail(BGK_E_INVALID, "null argument");
    for (int i = 0; i < B->n; ++i)
      if (!f[i]) return fail(BGK_E_INVALID, "null f for instance " + std::to_string(i));
    const auto t_start = std::chrono::steady_clock::now();
    const int n = B->n, S = B->S;
    hipStream_t caller = (hipStream_t)stream_;
    int rc;
    // order after the caller's prior work
    BGK_HIP(hipEventRecord(B->ev_in, caller));
    BGK_HIP(hipStreamWaitEvent(B->stream, B->ev_in, 0));
    if (B->f_bound.size() != (size_t)n || !std::equal(B->f_bound.begin(), B->f_bound.end(), f)) {
      if ((rc = batch_upload(B, f))) return rc;
    }
    if (B->opts.graph && B->exec.empty() && (rc = capture_graphs(B))) return rc;
    const Ctl c = B->ctl();
    std::vector<bgk_batch_stats> st(n);
    for (int i = 0; i < n; ++i) st[i].stages = S;
    std::vector<double> finish(n, 0.0);
    hipLaunchKernelGGL(k_step_init, inst_grid(n), dim3(64), 0, B->stream, c, n);
    BGK_HIP(hipGetLastError());
    if ((rc = launch_combine(B, 0, nullptr))) return rc;  // f^k
    if ((rc = launch_moments_batch(B->dim, B->kin, c.par, c.done, B->mom_first, n, B->mom_blocks,
                                   false, B->stream)))
      return rc;
    hipLaunchKernelGGL(k_set_par, inst_grid(n), dim3(64), 0, B->stream, c.par, 0, n);
    BGK_HIP(hipGetLastError());
    for (int s = 0; s < S; ++s) {
      if (s > 0 && (rc = launch_combine(B, s, c.done))) return rc;
      hipLaunchKernelGGL(k_stage_init, inst_grid(n), dim3(64), 0, B->stream, c, n);
      BGK_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_clear_bytes, dim3((unsigned)std::min<int64_t>((B->n_nodes + 255) / 256, 4096)),
                         dim3(256), 0, B->stream, B->sticky, B->n_nodes);
      BGK_HIP(hipGetLastError());
      std::vector<int> running(n, 1);
      for (;;) {
        if (B->opts.graph) {
          BGK_HIP(hipGraphLaunch(B->exec[s], B->stream));
        } else if ((rc = run_chunk(B, s))) {
          return rc;
        }
        BGK_HIP(hipMemcpyAsync(B->h_ctl, B->ctl_mem, (size_t)5 * n * sizeof(int32_t),
                               hipMemcpyDeviceToHost, B->stream));
        BGK_HIP(hipMemcpyAsync(B->h_last, B->last, (size_t)n * sizeof(double), hipMemcpyDeviceToHost,
                               B->stream));
        BGK_HIP(hipStreamSynchronize(B->stream));
        const double now =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        bool all = true;
        for (int i = 0; i < n; ++i) {
          const int done = B->h_ctl[i];
          if (done == 0) {
            all = false;
            continue;
          }
          if (running[i]) {
            running[i] = 0;
            st[i].iters[s] = B->h_ctl[2 * n + i];
            st[i].total_iters += st[i].iters[s];
            st[i].last_ratio[s] = B->h_last[i];
            if (done == 2 && st[i].status == BGK_OK) st[i].status = B->h_ctl[4 * n + i];
            if ((s == S - 1 || done == 2) && finish[i] == 0.0) finish[i] = now;
          }
        }
        if (all) break;
      }
    }
    if (!B->stiffly_accurate && (rc = launch_combine(B, S, c.done))) return rc;
    BGK_HIP(hipMemcpyAsync(B->h_ctl, B->ctl_mem, (size_t)5 * n * sizeof(int32_t),
                           hipMemcpyDeviceToHost, B->stream));
    BGK_HIP(hipStreamSynchronize(B->stream));
    BGK_HIP(hipEventRecord(B->ev_out, B->stream));
    BGK_HIP(hipStreamWaitEvent(caller, B->ev_out, 0));
    int first_err = BGK_OK, first_inst = -1;
    for (int i = 0; i < n; ++i) {
      st[i].maxw_fallbacks = B->h_ctl[3 * n + i];
      st[i].finish_ms = finish[i];
      if (st[i].status != BGK_OK && first_err == BGK_OK) {
        first_err = st[i].status;
        first_inst = i;
      }
    }
    if (stats) std::copy(st.begin(), st.end(), stats);
    if (first_err != BGK_OK)
      return fail(first_err, "instance " + std::to_string(first_inst) +
                                 (first_err == BGK_E_NONPHYSICAL ? ": non-physical moments"
                                                                 : ": Picard iteration reached l_max"));
    return BGK_OK;
  });
}

extern "C" int bgk_batch_time_sweep(bgk_batch* B, double* const* f, int threads, int lanes,
                                    int reps, float* ms, bgk_stream_t stream_) {
  return guarded([&]() -> int {
    if (!B || !f || !ms || reps <= 0) return fail(BGK_E_INVALID, "bad arguments");
    if (threads <= 0 || threads % 64 || threads > 256)
      return fail(BGK_E_INVALID, "threads must be a multiple of 64 up to 256");
    if (!valid_lanes(lanes))
      return fail(BGK_E_INVALID, "lanes must be 0, 64 or a power of two up to 32");
    for (int i = 0; i < B->n; ++i)
      if (!f[i]) return fail(BGK_E_INVALID, "null f");
    const int n = B->n;
    int rc;
    hipStream_t caller = (hipStream_t)stream_;
    BGK_HIP(hipEventRecord(B->ev_in, caller));
    BGK_HIP(hipStreamWaitEvent(B->stream, B->ev_in, 0));
    if (B->f_bound.size() != (size_t)n || !std::equal(B->f_bound.begin(), B->f_bound.end(), f)) {
      if ((rc = batch_upload(B, f))) return rc;
    }
    const Ctl c = B->ctl();
    // the Maxwellian of f's moments, then `reps` sweeps of f into f^k
    hipLaunchKernelGGL(k_step_init, inst_grid(n), dim3(64), 0, B->stream, c, n);
    BGK_HIP(hipGetLastError());
    if ((rc = launch_moments_batch(B->dim, B->kin + (size_t)(B->S + 1) * n, c.par, c.done,
                                   B->mom_first, n, B->mom_blocks, false, B->stream)))
      return rc;
    hipLaunchKernelGGL(k_set_par, inst_grid(n), dim3(64), 0, B->stream, c.par, 0, n);
    hipLaunchKernelGGL(k_clear_bytes, dim3((unsigned)std::min<int64_t>((B->n_nodes + 255) / 256, 4096)),
                       dim3(256), 0, B->stream, B->sticky, B->n_nodes);
    hipLaunchKernelGGL(k_iter_reset, inst_grid(n), dim3(64), 0, B->stream, c.done, B->status,
                       B->numax, n);
    BGK_HIP(hipGetLastError());
    const BatchKin* kin = B->kin + (size_t)n;
    if ((rc = launch_maxwellian_batch(B->dim, kin, c.par, c.done, B->mx_inst, B->mx_first, B->mx_blocks,
                                      B->stream)))
      return rc;
    if (B->tab &&
        (rc = launch_tables_batch(B->dim, kin, c.done, B->tab_first, n, B->n_tab, B->stream)))
      return rc;
    BatchWalk walk;
    if ((rc = batch_walk(B, threads, lanes, &walk))) return rc;
    BGK_HIP(hipEventRecord(B->t0, B->stream));
    for (int r = 0; r < reps; ++r)
      if ((rc = launch_sweep_batch(B->dim, B->tab, B->sargs_tune, walk, c.done, B->stream,
                                   B->side, B->ev_fork, B->ev_join)))
        return rc;
    BGK_HIP(hipEventRecord(B->t1, B->stream));
    BGK_HIP(hipEventSynchronize(B->t1));
    float t = 0.0f;
    BGK_HIP(hipEventElapsedTime(&t, B->t0, B->t1));
    *ms = t / reps;
    BGK_HIP(hipEventRecord(B->ev_out, B->stream));
    BGK_HIP(hipStreamWaitEvent(caller, B->ev_out, 0));
    return BGK_OK;
  });
}
