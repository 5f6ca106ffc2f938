// Arguments of the sweep kernels (one instance, one sweep).
#pragma once
#include <vector>

#include "internal.h"

namespace bgk {

struct SweepArgs {
  const double* geo;
  const FacetRec* facet;
  const double* v;
  const int32_t* rec;
  const int32_t* recx;
  const int32_t* perm;
  const int32_t* goff;
  const int32_t* gmin;
  const int64_t* gbase;
  const int32_t* G;
  const int32_t* vorder;
  const double* nu;
  const double* mcoef;
  const double* mtab;        // factorised Maxwellian tables (TabLayout, internal order) or null
  const double* q;
  const double* bc_coef;
  const double* bc_dense;
  const double* f_prev;
  double* f_out;
  float* d32;                // FP32 corrections (sweep layout), FP32 form only
  double sigma_shift;
  double q_scale;
  int n_cells;
  int n_v;
  int n1;                    // points per axis of a tensor velocity grid (mtab)
  int ring_slots;            // LDS ring of recent outputs, slots (power of two)
  int order;
  const int32_t* skip;       // nonzero *skip: the launch does nothing (nullable)
};

// The walk of a batched FP64 sweep.  lanes == 64: the workgroup walk, block
// b sweeping velocity position map[b].y of instance map[b].x with `threads`
// per workgroup.  lanes < 64: the packed walk, 64-lane block b serving the
// 64/lanes velocities pvel[map[b].y ..] (-1: none) of instance map[b].x.
// Either map holds the blocks of P2 instances first (nb2 of them), then
// those of P1 instances (nb1; every 3D instance is P1).
struct BatchWalk {
  int threads;
  int lanes;
  const int2* map;
  int nb2, nb1;
  const int32_t* pvel;
};

// One batched FP64 sweep; instances with done[i] skip.  In 2D with both
// element types present the two kernels run concurrently, the P1 one on
// `side` between the events fork (recorded on stream) and join (recorded on
// side, waited for on stream).
int launch_sweep_batch(int dim, bool tab, const SweepArgs* args, const BatchWalk& w,
                       const int32_t* done, hipStream_t stream, hipStream_t side, hipEvent_t fork,
                       hipEvent_t join);
SweepArgs make_sweep_args(const tgs_dag* d, const tgs_sweep_io* io,
                          const double* mtab, float* d32);
// the DAG's velocities sorted by direction (dag.hip): angular neighbours
// adjacent, the order the packed walk groups them in
std::vector<int32_t> angular_order(const tgs_dag* d);
// One single-instance sweep (sweep.hip): the DAG's walk, or the workgroup
// walk with `threads` per workgroup when threads > 0.  A non-null `skip`
// turns the launch into a no-op on the device while *skip is nonzero.
int launch_sweep(const tgs_dag* d, const tgs_sweep_io* io, const double* mtab, float* d32,
                 hipStream_t stream, int threads, const int32_t* skip = nullptr);
// factorised Maxwellian tables of a tensor velocity grid from nodal
// coefficients and nu (kinetic.hip), and their size in doubles
int launch_maxw_tables(const tgs_dag* d, const double* coef, const double* nu, double* tab,
                       hipStream_t stream, const int32_t* skip = nullptr);
// the same tables for the projected Maxwellian from primitive (n, u, theta)
// coefficients; pr is scratch of proj_scratch_size(d) doubles
int launch_proj_tables(const tgs_dag* d, const double* prim, const double* nu, double* pr,
                       double* tab, hipStream_t stream, const int32_t* skip = nullptr);
inline size_t proj_scratch_size(const tgs_dag* d) {
  return (size_t)d->dim * d->n_1d * d->n_nodes;
}
inline size_t maxw_table_size(const tgs_dag* d) {
  return (size_t)TabLayout(d->n_cells, d->n_1d, (int)(d->n_nodes / d->n_cells), d->dim).size();
}
// copies per-cell rows of `row` doubles between the user and the internal
// cell order (kinetic.hip)
int launch_nodal_rows(const tgs_dag* d, const double* src, double* dst, int row, int to_internal,
                      hipStream_t stream);

}  // namespace bgk
