// Arguments of the moment and Maxwellian kernels, and the batched launchers.
#pragma once
#include "internal.h"

namespace bgk {

constexpr int MOM_THREADS = 256;

struct MomArgs {
  const double* f;
  const int32_t* pos;
  const int32_t* uid;
  const double* v;
  const double* w;
  double* U;
  const double* U_prev;
  double* partial;  // [gridDim][6]: |dU_m|^2 (m = 0,1,2), |U_prev_m|^2
  int n_cells;
  int n_v;
  const int32_t* skip;  // nonzero *skip: the launch does nothing (nullable)
  double* split;        // velocity-split reduction: chunk sums [vb][cell][node][m]
  int jc;               // velocities per chunk
  int vb;               // chunks
};

struct MaxwArgs {
  const double* U;
  double* coef;
  double* nu;
  double* M_dense;          // canonical [n_nodes][n_v] or null
  int32_t* status;          // [0] fallbacks, [1] non-physical, or null
  unsigned long long* numax;  // bit pattern of max nu (nu >= 0), or null
  const double* v;
  const double* w;
  const double* x1;         // tensor 1-D nodes or null
  const double* w1;
  int n1;
  int n_v;
  int64_t n_nodes;
  int mode;
  int nu_kind;
  double nu_const, kn, L;
  int dg_cells;             // Q2 velocity cells per axis (PROJECTED), or 0
  // MATCHED: per node, set once its Newton solve has failed; such a node
  // keeps the DIRECT coefficients while the flag stays set (nullable)
  uint8_t* sticky;
  const int32_t* skip;  // nonzero *skip: the launch does nothing (nullable)
};

// Per-instance description for the batched kinetic kernels.  Nodal moments
// ping-pong between U[0] and U[1]: the current iterate is U[par[i]].
struct BatchKin {
  MaxwArgs maxw;       // .U is replaced by U[par]
  MomArgs mom;         // .U / .U_prev are replaced by U[par ^ 1] / U[par]
  const double* U[2];
  double* mtab;        // factorised tables or null
  const double* geo;   // cell geometry (carried in the tables' padding for P2 triangles)
  const double* x1;
  int n1;
  int mom_vl;          // velocity lanes of the moment kernel (1, 4, 16)
  int mom_blocks;
  int np;              // nodes per cell
  int64_t n_nodes;
  double* ratio;       // [4]
};

// Launchers over all instances; done[i] != 0 skips instance i.  blk_first
// is the exclusive prefix of per-instance block counts (n + 1 entries).
// The Maxwellian takes one 128-thread block per 128 nodes of an instance:
// blk_inst[b] is the instance of block b (n_blocks of them) and
// blk_first[i] the first block of instance i.
int launch_maxwellian_batch(int dim, const BatchKin* kin, const int32_t* par, const int32_t* done,
                            const int32_t* blk_inst, const int32_t* blk_first, int n_blocks,
                            hipStream_t stream);
int launch_tables_batch(int dim, const BatchKin* kin, const int32_t* done,
                        const int64_t* entry_first, int n_inst, int64_t n_total,
                        hipStream_t stream);
int launch_moments_batch(int dim, const BatchKin* kin, const int32_t* par, const int32_t* done,
                         const int32_t* blk_first, int n_inst, int n_blocks, bool with_ratio,
                         hipStream_t stream);
// Final reduction of the block pieces in a fixed order; writes
// out[0..2] = ratios, out[3] = max ratio.
__device__ __forceinline__ void ratio_block(const double* __restrict__ partial, int nblk,
                                            double* out, double (*s)[256]) {
  const int tid = threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int b = tid; b < nblk; b += 256)
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] += partial[(size_t)b * 6 + i];
#pragma unroll
  for (int i = 0; i < 6; ++i) s[i][tid] = acc[i];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off)
#pragma unroll
      for (int i = 0; i < 6; ++i) s[i][tid] += s[i][tid + off];
    __syncthreads();
  }
  if (tid == 0) {
    const double n0 = sqrt(s[3][0]);
    double mx = 0.0;
    for (int m = 0; m < 3; ++m) {
      double den = sqrt(s[3 + m][0]);
      if (m == 1) den = fmax(den, n0);
      const double r = sqrt(s[m][0]) / den;
      out[m] = r;
      mx = fmax(mx, r);
    }
    out[3] = mx;
  }
}

int moment_vl(const tgs_dag* d);
int moment_blocks(const tgs_dag* d);  // blocks of the unsplit kernel (the batch's)

// The single-instance moment pass of a mesh with few cells and many velocities
// splits the velocities into chunks (moment_split > 1): its chunk sums take
// moment_split_doubles doubles of scratch (at most MOM_SPLIT_DOUBLES), and its
// norms come in moment_partials pieces (moment_blocks without the split).
constexpr int64_t MOM_SPLIT_DOUBLES = (int64_t)1 << 21;
int moment_split(const tgs_dag* d);
int64_t moment_split_doubles(const tgs_dag* d);
int moment_partials(const tgs_dag* d);

// Single-instance launchers (kinetic.hip).  A non-null `skip` turns the
// launch into a no-op on the device while *skip is nonzero.  `split` is
// the chunk-sum scratch (moment_split_doubles; null when that is 0);
// `partial` holds 6 doubles per moment_partials piece.
int launch_moments(const tgs_dag* d, const double* f, double* U, const double* U_prev,
                   double* partial, double* ratio_out, hipStream_t stream, bool user_order,
                   double* split, const int32_t* skip = nullptr);
int launch_maxwellian(const tgs_dag* d, int mode, const double* U, const tgs_nu_model* nm,
                      double* coef, double* nu, double* M_dense, int32_t* status,
                      unsigned long long* numax, uint8_t* sticky, hipStream_t stream,
                      const int32_t* skip = nullptr);

}  // namespace bgk
