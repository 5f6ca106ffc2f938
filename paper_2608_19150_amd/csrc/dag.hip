// build_mesh_dag: host geometry and connectivity, then per-velocity upwind
// DAGs and longest-path generations on the GPU (Sec. 4.1).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>

#include "device_common.h"

namespace bgk {

namespace {

constexpr int DAG_THREADS = 256;

// ----------------------------------------------------------------------------
// host geometry
// ----------------------------------------------------------------------------
struct HostMesh {
  int dim, order, n_p, n_fp;
  int64_t n_cells;
  std::vector<double> geo;          // user order, [c][1 + (dim+1)*dim]: vol, normals
  std::vector<int32_t> nb;          // user order, [c][dim+1]: user nbr or -(1+bface)
  std::vector<int32_t> nb_face;     // [c][dim+1]
  std::vector<int32_t> nb_node;     // [c][dim+1][n_fp]
  std::vector<double> node_x;       // [c][n_p][dim]
  std::vector<double> bnode_x;      // [bf][n_fp][dim]
  std::vector<int32_t> bcell;       // [bf] user cell of the boundary facet
  std::vector<int32_t> bpack;       // [bf] its facet's local nodes, 4 bits each
  std::vector<double> bnormal;      // [bf][dim] outward unit normal
  std::vector<double> vol;          // [c]
  std::vector<double> centroid;     // [c][dim]
  int64_t n_bfaces = 0;
};

// local nodes on facet k (ascending), node key helpers
void facet_nodes(int dim, int order, int k, std::vector<int>& out) {
  out.clear();
  for (int a = 0; a <= dim; ++a)
    if (a != k) out.push_back(a);
  if (order == 2) {
    const int ii[3] = {0, 1, 2}, jj[3] = {1, 2, 0};
    for (int m = 0; m < 3; ++m)
      if (ii[m] != k && jj[m] != k) out.push_back(3 + m);
  }
}

// global identity of local node a of a cell: vertex id, or the sorted pair of
// an edge midpoint
std::array<int32_t, 2> node_key(const int32_t* cv, int a) {
  if (a < 3 || cv == nullptr) return {cv[a], -1};
  const int ii[3] = {0, 1, 2}, jj[3] = {1, 2, 0};
  int32_t x = cv[ii[a - 3]], y = cv[jj[a - 3]];
  return {std::min(x, y), std::max(x, y)};
}

int build_host_mesh(const tgs_mesh_desc* m, HostMesh& H) {
  const int dim = m->dim, order = m->order;
  BGK_CHECK(dim == 2 || dim == 3, BGK_E_UNSUPPORTED, "dim must be 2 or 3");
  BGK_CHECK(order == 1 || (order == 2 && dim == 2), BGK_E_UNSUPPORTED,
            "supported elements: P1 triangles/tetrahedra, P2 triangles");
  BGK_CHECK(m->n_cells > 0 && m->n_vert > dim && m->vert && m->cells, BGK_E_INVALID,
            "empty mesh");
  BGK_CHECK(m->n_cells < (int64_t)1 << 30, BGK_E_INVALID, "too many cells");
  H.dim = dim;
  H.order = order;
  H.n_p = order == 1 ? dim + 1 : 6;
  H.n_fp = order == 1 ? dim : 3;
  H.n_cells = m->n_cells;
  const int64_t nc = m->n_cells, nf = dim + 1;
  const int gs = 1 + (dim + 1) * dim;
  H.geo.assign(nc * gs, 0.0);
  H.vol.assign(nc, 0.0);
  H.centroid.assign(nc * dim, 0.0);
  H.node_x.assign(nc * H.n_p * dim, 0.0);
  for (int64_t c = 0; c < nc; ++c) {
    const int32_t* cv = m->cells + c * nf;
    double X[4][3] = {};
    for (int a = 0; a < nf; ++a) {
      BGK_CHECK(cv[a] >= 0 && cv[a] < m->n_vert, BGK_E_INVALID, "vertex id out of range");
      for (int d = 0; d < dim; ++d) X[a][d] = m->vert[(int64_t)cv[a] * dim + d];
    }
    double J[3][3] = {};  // columns X_{k+1} - X_0
    double hmax = 0.0;
    for (int r = 0; r < dim; ++r)
      for (int k = 0; k < dim; ++k) {
        J[r][k] = X[k + 1][r] - X[0][r];
        hmax = std::max(hmax, std::fabs(J[r][k]));
      }
    double det, inv[3][3];
    if (dim == 2) {
      det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      inv[0][0] = J[1][1] / det;
      inv[0][1] = -J[0][1] / det;
      inv[1][0] = -J[1][0] / det;
      inv[1][1] = J[0][0] / det;
    } else {
      const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
      inv[0][0] = c00 / det;
      inv[1][0] = c01 / det;
      inv[2][0] = c02 / det;
      inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
      inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
      inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
      inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
      inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
      inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    const double adet = std::fabs(det);
    BGK_CHECK(std::isfinite(det) && adet > 1e-13 * std::pow(hmax, dim), BGK_E_INVALID,
              "degenerate cell " + std::to_string(c));
    (void)inv;
    H.geo[c * gs] = adet / (dim == 2 ? 2.0 : 6.0);
    H.vol[c] = H.geo[c * gs];
    for (int d = 0; d < dim; ++d) {
      double s = 0;
      for (int a = 0; a < nf; ++a) s += X[a][d];
      H.centroid[c * dim + d] = s / nf;
    }
    for (int a = 0; a < H.n_p; ++a)
      for (int d = 0; d < dim; ++d) {
        double x;
        if (a < nf) {
          x = X[a][d];
        } else {
          const int ii[3] = {0, 1, 2}, jj[3] = {1, 2, 0};
          x = 0.5 * (X[ii[a - 3]][d] + X[jj[a - 3]][d]);
        }
        H.node_x[(c * H.n_p + a) * dim + d] = x;
      }
  }
  // facet matching by sorted vertex ids
  struct FKey {
    int32_t v[3];
    int32_t cell, k;
  };
  std::vector<FKey> keys(nc * nf);
  for (int64_t c = 0; c < nc; ++c)
    for (int k = 0; k < nf; ++k) {
      FKey& f = keys[c * nf + k];
      int p = 0;
      f.v[2] = -1;
      for (int a = 0; a < nf; ++a)
        if (a != k) f.v[p++] = m->cells[c * nf + a];
      std::sort(f.v, f.v + dim);
      f.cell = (int32_t)c;
      f.k = k;
    }
  std::sort(keys.begin(), keys.end(), [](const FKey& a, const FKey& b) {
    if (a.v[0] != b.v[0]) return a.v[0] < b.v[0];
    if (a.v[1] != b.v[1]) return a.v[1] < b.v[1];
    if (a.v[2] != b.v[2]) return a.v[2] < b.v[2];
    if (a.cell != b.cell) return a.cell < b.cell;
    return a.k < b.k;
  });
  H.nb.assign(nc * nf, INT32_MIN);
  H.nb_face.assign(nc * nf, -1);
  auto same = [&](const FKey& a, const FKey& b) {
    return a.v[0] == b.v[0] && a.v[1] == b.v[1] && a.v[2] == b.v[2];
  };
  for (size_t i = 0; i < keys.size();) {
    size_t e = i + 1;
    while (e < keys.size() && same(keys[i], keys[e])) ++e;
    BGK_CHECK(e - i <= 2, BGK_E_INVALID, "facet shared by more than two cells");
    if (e - i == 2) {
      const FKey &a = keys[i], &b = keys[i + 1];
      BGK_CHECK(a.cell != b.cell, BGK_E_INVALID, "cell with repeated vertices");
      H.nb[(int64_t)a.cell * nf + a.k] = b.cell;
      H.nb_face[(int64_t)a.cell * nf + a.k] = b.k;
      H.nb[(int64_t)b.cell * nf + b.k] = a.cell;
      H.nb_face[(int64_t)b.cell * nf + b.k] = a.k;
    }
    i = e;
  }
  // outward area-weighted facet normals N_k = |e_k| n_k: computed from the
  // lower-numbered cell's facet vertices (ascending local order), edge vector
  // rotated (2D) or half the cross product (3D), oriented away from the
  // centroid, and stored negated in the neighbour
  for (int64_t c = 0; c < nc; ++c)
    for (int k = 0; k < nf; ++k) {
      const int32_t nbc = H.nb[c * nf + k];
      if (nbc != INT32_MIN && nbc < c) continue;
      double P[3][3] = {};
      int p = 0;
      for (int a = 0; a < nf; ++a)
        if (a != k) {
          for (int d = 0; d < dim; ++d) P[p][d] = m->vert[(int64_t)m->cells[c * nf + a] * dim + d];
          ++p;
        }
      double N[3] = {0, 0, 0}, mid[3] = {0, 0, 0};
      if (dim == 2) {
        const double t0 = P[1][0] - P[0][0], t1 = P[1][1] - P[0][1];
        N[0] = t1;
        N[1] = -t0;
      } else {
        const double a0 = P[1][0] - P[0][0], a1 = P[1][1] - P[0][1], a2 = P[1][2] - P[0][2];
        const double b0 = P[2][0] - P[0][0], b1 = P[2][1] - P[0][1], b2 = P[2][2] - P[0][2];
        N[0] = 0.5 * (a1 * b2 - a2 * b1);
        N[1] = 0.5 * (a2 * b0 - a0 * b2);
        N[2] = 0.5 * (a0 * b1 - a1 * b0);
      }
      double dotc = 0.0;
      for (int d = 0; d < dim; ++d) {
        for (int q = 0; q < dim; ++q) mid[d] += P[q][d];
        mid[d] /= dim;
        dotc += N[d] * (mid[d] - H.centroid[c * dim + d]);
      }
      const double sgn = dotc < 0 ? -1.0 : 1.0;
      for (int d = 0; d < dim; ++d) H.geo[c * gs + 1 + k * dim + d] = sgn * N[d];
      if (nbc != INT32_MIN) {
        const int k2 = H.nb_face[c * nf + k];
        for (int d = 0; d < dim; ++d) H.geo[(int64_t)nbc * gs + 1 + k2 * dim + d] = -(sgn * N[d]);
      }
    }
  // boundary facets in ascending (cell, facet) order; node maps
  H.nb_node.assign(nc * nf * H.n_fp, -1);
  H.bnode_x.clear();
  std::vector<int> fn, fn2;
  int64_t nbf = 0;
  for (int64_t c = 0; c < nc; ++c)
    for (int k = 0; k < nf; ++k) {
      facet_nodes(dim, order, k, fn);
      const int64_t idx = c * nf + k;
      if (H.nb[idx] == INT32_MIN) {
        H.nb[idx] = -(int32_t)(1 + nbf);
        ++nbf;
        int32_t pack = 0;
        for (int p = 0; p < H.n_fp; ++p) {
          pack |= fn[p] << (4 * p);
          for (int d = 0; d < dim; ++d)
            H.bnode_x.push_back(H.node_x[(c * H.n_p + fn[p]) * dim + d]);
        }
        H.bcell.push_back((int32_t)c);
        H.bpack.push_back(pack);
        const double* nr = &H.geo[c * gs + 1 + k * dim];
        double len = 0.0;
        for (int d = 0; d < dim; ++d) len += nr[d] * nr[d];
        len = std::sqrt(len);
        for (int d = 0; d < dim; ++d) H.bnormal.push_back(nr[d] / len);
        continue;
      }
      const int32_t c2 = H.nb[idx];
      const int k2 = H.nb_face[idx];
      facet_nodes(dim, order, k2, fn2);
      for (int p = 0; p < H.n_fp; ++p) {
        auto key = order == 1 ? std::array<int32_t, 2>{m->cells[c * nf + fn[p]], -1}
                              : node_key(m->cells + c * nf, fn[p]);
        int found = -1;
        for (int q = 0; q < H.n_fp; ++q) {
          auto k2key = order == 1 ? std::array<int32_t, 2>{m->cells[(int64_t)c2 * nf + fn2[q]], -1}
                                  : node_key(m->cells + (int64_t)c2 * nf, fn2[q]);
          if (k2key == key) found = fn2[q];
        }
        BGK_CHECK(found >= 0, BGK_E_INVALID, "non-conforming facet");
        H.nb_node[idx * H.n_fp + p] = found;
      }
    }
  H.n_bfaces = nbf;
  return BGK_OK;
}

uint64_t spread_bits(uint64_t x, int dim) {
  // interleave the low bits of x with (dim-1) zero bits between them
  uint64_t r = 0;
  const int nb = dim == 2 ? 31 : 21;
  for (int b = 0; b < nb; ++b) r |= ((x >> b) & 1ull) << (b * dim);
  return r;
}

// ----------------------------------------------------------------------------
// GPU: per-velocity Kahn levels + stable counting sort by generation
// ----------------------------------------------------------------------------
struct DagArgs {
  const double* geo;
  const FacetRec* facet;
  const double* v;
  const uint8_t* user_lag;   // [n_v][n_cells] internal order, or null
  uint8_t* lag;              // [n_v][n_cells] output lag bits (may alias user_lag)
  int32_t* perm;             // [n_v][n_cells]
  int32_t* pos;              // [n_v][n_cells]
  int32_t* scratch_cnt;      // [batch][n_cells+1]  generation offsets (batch-local)
  int32_t* scratch_cur;      // [batch][n_cells+1]  in-degrees, then cursors
  int32_t* G;                // [n_v]
  unsigned long long* n_lagged;
  int n_cells;
};

template <int DIM>
__global__ __launch_bounds__(DAG_THREADS) void k_dag_levels(DagArgs a, int j0) {
  const int jb = blockIdx.x, j = j0 + jb, tid = threadIdx.x, bs = blockDim.x;
  const int nc = a.n_cells;
  double v[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) v[d] = a.v[(size_t)j * DIM + d];
  int32_t* indeg = a.scratch_cur + (size_t)jb * (nc + 1);
  int32_t* cnt = a.scratch_cnt + (size_t)jb * (nc + 1);
  int32_t* queue = a.perm + (size_t)j * nc;
  int32_t* gen = a.pos + (size_t)j * nc;
  const uint8_t* ulag = a.user_lag ? a.user_lag + (size_t)j * nc : nullptr;
  uint8_t* lag = a.lag ? a.lag + (size_t)j * nc : nullptr;

  __shared__ int s_tail, s_min;
  __shared__ int s_scan[DAG_THREADS];
  if (tid == 0) s_tail = 0;
  __syncthreads();
  // in-degrees and sources
  for (int K = tid; K < nc; K += bs) {
    const int ul = ulag ? ulag[K] : 0;
    const int bits = inflow_bits<DIM>(a.geo, a.facet, K, v, ul);
    indeg[K] = __popc(bits);
    gen[K] = -1;
    lag[K] = (uint8_t)ul;
  }
  __syncthreads();
  for (int K = tid; K < nc; K += bs)
    if (indeg[K] == 0) {
      const int p = atomicAdd(&s_tail, 1);
      queue[p] = K;
      gen[K] = 0;
    }
  __syncthreads();
  int head = 0, tail = s_tail, g = 0;
  while (head < nc) {
    if (head == tail) {
      // Every remaining cell still has an in-edge from another remaining
      // cell, so the remaining graph has a cycle.  Walk in-edges backwards
      // from the lowest-numbered remaining cell (each step to the in-neighbour
      // across the lowest-indexed facet) until a cell repeats: the edge that
      // closes that loop lies on a cycle and is lagged (its downwind cell
      // takes that facet's inflow from the previous iterate, Sec. 4.1).  One
      // edge per walk, walks repeated until a cell loses its last remaining
      // in-edge and is released.  Only edges that lie on a cycle are lagged.
      // The levels of this pass are not longest paths once something was
      // lagged; the host then repeats the pass on the final lagged set.
      if (tid == 0) s_min = INT32_MAX;
      __syncthreads();
      int mymin = INT32_MAX;
      for (int K = tid; K < nc; K += bs)
        if (gen[K] < 0) mymin = min(mymin, K);
      atomicMin(&s_min, mymin);
      __syncthreads();
      const int K0 = s_min;
      if (K0 == INT32_MAX) break;  // inconsistent bookkeeping: stop (G < cells flags it)
      if (tid == 0) {
        int32_t* path = cnt;  // scratch: free until the histogram below
        bool released = false, stuck = false;
        while (!released && !stuck) {
          int c = K0, len = 0;
          gen[c] = -2;
          path[len++] = c;
          for (;;) {
            const int cur = lag[c];
            const int bits = inflow_bits<DIM>(a.geo, a.facet, c, v, cur);
            int p = -1, kp = -1;
            for (int k = 0; k <= DIM && p < 0; ++k)
              if ((bits >> k) & 1) {
                const int nbk = a.facet[(size_t)c * (DIM + 1) + k].nb;
                if (gen[nbk] < 0) {
                  p = nbk;
                  kp = k;
                }
              }
            if (p < 0) {  // no remaining in-edge: cannot happen with indeg[c] > 0
              stuck = true;
              break;
            }
            if (gen[p] <= -2) {  // p is on this walk: the edge p -> c closes a cycle
              lag[c] = (uint8_t)(cur | (1 << kp));
              atomicAdd(a.n_lagged, 1ull);
              if (--indeg[c] == 0) {
                queue[tail] = c;
                gen[c] = g;
                released = true;
              }
              break;
            }
            gen[p] = -2;
            path[len++] = p;
            c = p;
          }
          for (int i = 0; i < len; ++i)
            if (gen[path[i]] == -2) gen[path[i]] = -1;
        }
        s_tail = released ? tail + 1 : tail;
      }
      __syncthreads();
      tail = s_tail;
      if (tail == head) break;  // nothing released: G < cells flags it
    }
    __syncthreads();
    if (tid == 0) s_tail = tail;
    __syncthreads();
    for (int idx = head + tid; idx < tail; idx += bs) {
      const int K = queue[idx];
#pragma unroll
      for (int k = 0; k <= DIM; ++k) {
        const FacetRec fr = a.facet[(size_t)K * (DIM + 1) + k];
        if (fr.nb < 0) continue;
        const int b = fr.nb, kb = fr.pack & 3;
        // lag[] holds the caller's bits and those added by cycle walks
        const int bits = inflow_bits<DIM>(a.geo, a.facet, b, v, lag[b]);
        if (!((bits >> kb) & 1)) continue;
        if (atomicSub(&indeg[b], 1) == 1) {
          const int p = atomicAdd(&s_tail, 1);
          queue[p] = b;
          gen[b] = g + 1;
        }
      }
    }
    __threadfence_block();
    __syncthreads();
    head = tail;
    tail = s_tail;
    ++g;
    __syncthreads();
  }
  if (head < nc) {  // not every cell was released: report, touch nothing else
    if (tid == 0) a.G[j] = -1;
    return;
  }
  const int G = g;
  if (tid == 0) a.G[j] = G;
  // histogram of generations
  for (int i = tid; i <= G; i += bs) cnt[i] = 0;
  __syncthreads();
  for (int K = tid; K < nc; K += bs) atomicAdd(&cnt[gen[K]], 1);
  __threadfence_block();
  __syncthreads();
  // exclusive scan of cnt[0..G] (cnt[G] = 0 -> becomes nc)
  int carry = 0;
  for (int base = 0; base <= G; base += bs) {
    const int i = base + tid;
    const int x = i <= G ? cnt[i] : 0;
    s_scan[tid] = x;
    __syncthreads();
    for (int off = 1; off < bs; off <<= 1) {
      const int y = tid >= off ? s_scan[tid - off] : 0;
      __syncthreads();
      s_scan[tid] += y;
      __syncthreads();
    }
    if (i <= G) {
      cnt[i] = carry + s_scan[tid] - x;
      indeg[i] = cnt[i];  // cursor
    }
    carry += s_scan[bs - 1];
    __syncthreads();
  }
  __threadfence_block();
  __syncthreads();
  // stable scatter in internal (Morton) order by one wavefront: within each
  // 64-cell chunk, equal generations keep their order via ballots
  if (tid < 64) {
    const int lane = tid;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int base = 0; base < nc; base += 64) {
      const int K = base + lane;
      const bool act = K < nc;
      const int gk = act ? gen[K] : -1;
      unsigned long long remaining = __ballot(act);
      int slot = 0;
      while (remaining) {
        const int leader = __ffsll((unsigned long long)remaining) - 1;
        const int gl = __shfl(gk, leader);
        const unsigned long long m = __ballot(act && gk == gl);
        int cur = 0;
        if (lane == leader) cur = atomicAdd(&indeg[gl], (int)__popcll(m));
        cur = __shfl(cur, leader);
        if (act && gk == gl) slot = cur + __popcll(m & below);
        remaining &= ~m;
      }
      if (act) {
        queue[slot] = K;
        gen[K] = slot;
      }
    }
  }
}

// Item records for the sweep: per (velocity, slot) the cell and, per facet,
// where its inflow comes from.  Uses the same facet classification as the
// level kernel and the sweep (facet_flux), so every inflow facet has a code.
template <int DIM>
__global__ void k_records(const double* __restrict__ geo, const FacetRec* __restrict__ facet,
                          const double* __restrict__ vel, const int32_t* __restrict__ perm,
                          const int32_t* __restrict__ pos, const uint8_t* __restrict__ lag,
                          int32_t* __restrict__ rec, int32_t* __restrict__ recx, int n_cells,
                          int n_fp, int j0, int nb) {
  const int64_t total = (int64_t)nb * n_cells;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int j = j0 + (int)(idx / n_cells);
    const size_t base = (size_t)j * n_cells;
    const int s = (int)(idx % n_cells);
    const int K = perm[base + s];
    double v[DIM], v2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      v[d] = vel[(size_t)j * DIM + d];
      v2 = __fma_rn(v[d], v[d], v2);
    }
    double fl[DIM + 1];
    facet_flux<DIM>(geo + (size_t)K * GeoLayout<DIM>::STRIDE, v, v2, fl);
    const int lb = lag ? lag[base + K] : 0;
    int code[4] = {-1, -1, -1, -1};
    const int nbits = n_fp == 3 && DIM == 2 ? 3 : 2;
    int packs = 0;
#pragma unroll
    for (int k = 0; k <= DIM; ++k) {
      const FacetRec fr = facet[(size_t)K * (DIM + 1) + k];
      for (int p = 0; p < n_fp; ++p)
        packs |= ((fr.pack >> (4 * (p + 1))) & 15) << (nbits * (k * n_fp + p));
      if (!(fl[k] < 0.0)) continue;
      if (fr.nb >= 0)
        code[k] = pos[base + fr.nb] | (((lb >> k) & 1) ? REC_LAG_BIT : 0);
      else
        code[k] = -2 - (-fr.nb - 1);
    }
    recx[base + s] = packs;
    int4 r;
    if (DIM == 2)
      r = make_int4(K, code[0], code[1], code[2]);
    else
      r = make_int4(code[0], code[1], code[2], code[3]);
    reinterpret_cast<int4*>(rec)[base + s] = r;
  }
}

// lowest upwind (non-lagged) slot read by each generation; one block per velocity
__global__ void k_gen_reach(const int32_t* __restrict__ rec, const int32_t* __restrict__ goff,
                            const int64_t* __restrict__ gbase, const int32_t* __restrict__ G,
                            int32_t* __restrict__ gmin, int n_cells, int dim) {
  const int j = blockIdx.x;
  const int32_t* go = goff + gbase[j];
  const size_t base = (size_t)j * n_cells;
  __shared__ int s_min;
  for (int g = 0; g < G[j]; ++g) {
    if (threadIdx.x == 0) s_min = INT32_MAX;
    __syncthreads();
    int m = INT32_MAX;
    for (int s = go[g] + threadIdx.x; s < go[g + 1]; s += blockDim.x) {
      const int4 r = reinterpret_cast<const int4*>(rec)[base + s];
      const int c[4] = {r.x, r.y, r.z, r.w};
      for (int k = (dim == 2 ? 1 : 0); k < 4; ++k)
        if (c[k] >= 0 && !(c[k] & REC_LAG_BIT)) m = min(m, c[k] & REC_SLOT_MASK);
    }
    atomicMin(&s_min, m);
    __syncthreads();
    if (threadIdx.x == 0) gmin[gbase[j] + g] = s_min;
    __syncthreads();
  }
}

template <typename T>
int dalloc(T** p, size_t n) {
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(BGK_E_NOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  return BGK_OK;
}

}  // namespace

void free_dag(tgs_dag* d) {
  if (!d) return;
  void* ptrs[] = {d->d_geo,  d->d_uid, d->d_facet, d->d_v,    d->d_w,    d->d_nodes1d,
                  d->d_weights1d, d->d_perm, d->d_pos, d->d_goff, d->d_gbase, d->d_G,
                  d->d_lag, d->d_vorder, d->d_rec, d->d_recx, d->d_gmin, d->d_vpack};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete d;
}

// direction key of a velocity: the angle (2D), or the octant then two
// angles (3D); sorting by it makes angular neighbours adjacent
double velocity_key(const double* vj, int dim) {
  if (dim == 2) return std::atan2(vj[1], vj[0]);
  const int oct = (vj[0] < 0) * 4 + (vj[1] < 0) * 2 + (vj[2] < 0);
  return oct * 10.0 + std::atan2(std::fabs(vj[1]), std::fabs(vj[0])) +
         std::atan2(std::fabs(vj[2]), std::hypot(vj[0], vj[1]));
}

std::vector<int32_t> angular_order(const tgs_dag* D) {
  std::vector<std::pair<double, int32_t>> key(D->n_v);
  for (int j = 0; j < D->n_v; ++j)
    key[j] = {velocity_key(&D->v_host[(size_t)j * D->dim], D->dim), j};
  std::stable_sort(key.begin(), key.end());
  std::vector<int32_t> out(D->n_v);
  for (int j = 0; j < D->n_v; ++j) out[j] = key[j].second;
  return out;
}

// Sorted positions 0..n-1 dealt to blocks: block b runs on XCD b % 8, and
// sector x (positions [x n/8, (x+1) n/8)) goes to XCD x, so block b takes
// the (b/8)-th position of sector b % 8 (sectors differ in size by at most
// one: a full sector falls through to the next with room)
std::vector<int32_t> deal_sectors(int n) {
  constexpr int NX = 8;
  std::vector<int32_t> out(n);
  std::vector<int> used(NX, 0);
  for (int b = 0; b < n; ++b) {
    int x = b % NX;
    int lo = (int)((int64_t)x * n / NX), hi = (int)((int64_t)(x + 1) * n / NX);
    for (int t = 0; t < NX && lo + used[x] >= hi; ++t) {
      x = (x + 1) % NX;
      lo = (int)((int64_t)x * n / NX);
      hi = (int)((int64_t)(x + 1) * n / NX);
    }
    out[b] = lo + used[x]++;
  }
  return out;
}

// The sweep walk: the workgroup walk with `threads` per workgroup (0: the
// element type's default), or the packed walk with `lanes` per velocity.
// lanes == 0 with threads == 0 takes the automatic rule: lanes from the mean
// generation width; a wavefront takes 64/L velocities that are angular
// neighbours (similar graphs, so its lane groups finish together), and the
// groups are dealt to the XCDs by sector like the workgroup walk's blocks.
int set_sweep_walk(tgs_dag* D, int threads, int lanes, hipStream_t stream) {
  const int nv = D->n_v, dim = D->dim;
  const int64_t nc = D->n_cells;
  D->sweep_threads = threads;
  if (lanes == 0 && threads == 0) {
    double sumG = 0.0;
    for (int j = 0; j < nv; ++j) sumG += D->G_host[j];
    const double width = (double)nc * nv / std::max(sumG, 1.0);
    int l0 = 1;
    while (l0 < 64 && l0 * 1.5 < width) l0 *= 2;
    // enough wavefronts to fill the GPU (4 per CU): fewer velocities per
    // wavefront when there are few velocities
    lanes = l0;
    while (lanes < 32 && (double)nv * lanes / 64 < 1024) lanes *= 2;
    if (l0 >= 32 || (double)nv * lanes / 64 < 1024) lanes = 64;
  }
  if (lanes == 0) lanes = 64;
  D->sweep_lanes = lanes;
  if (D->d_vpack) {
    (void)hipFree(D->d_vpack);
    D->d_vpack = nullptr;
  }
  D->vpack_blocks = 0;
  if (lanes < 64) {
    const int vpb = 64 / lanes;
    std::vector<std::pair<double, int32_t>> key(nv);
    for (int j = 0; j < nv; ++j) key[j] = {velocity_key(&D->v_host[(size_t)j * dim], dim), j};
    std::stable_sort(key.begin(), key.end());
    const int ng = (nv + vpb - 1) / vpb;
    const std::vector<int32_t> gorder = deal_sectors(ng);
    D->vpack_blocks = ng;
    std::vector<int32_t> vpack((size_t)ng * vpb, -1);
    for (int b = 0; b < ng; ++b)
      for (int t = 0; t < vpb; ++t) {
        const int pos = gorder[b] * vpb + t;
        if (pos < nv) vpack[(size_t)b * vpb + t] = key[pos].second;
      }
    int rc;
    if ((rc = dalloc(&D->d_vpack, vpack.size()))) return rc;
    BGK_HIP(hipMemcpyAsync(D->d_vpack, vpack.data(), vpack.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, stream));
    BGK_HIP(hipStreamSynchronize(stream));
  }
  return BGK_OK;
}

int build_dag_impl(const tgs_mesh_desc* mesh, const tgs_vgrid_desc* vg, const tgs_dag_opts* opts,
                   hipStream_t stream, tgs_dag* D) {
  HostMesh H;
  int rc = build_host_mesh(mesh, H);
  if (rc) return rc;
  const int dim = H.dim;
  BGK_CHECK(vg && vg->n_v > 0 && vg->v && vg->w, BGK_E_INVALID, "empty velocity grid");
  BGK_HIP(hipGetDevice(&D->device));
  D->dim = dim;
  D->order = H.order;
  D->n_p = H.n_p;
  D->n_fp = H.n_fp;
  D->n_cells = H.n_cells;
  D->n_vert = mesh->n_vert;
  D->n_bfaces = H.n_bfaces;
  D->n_nodes = H.n_cells * H.n_p;
  D->n_v = vg->n_v;
  D->L = vg->L;
  D->v_host.assign(vg->v, vg->v + (size_t)vg->n_v * dim);
  D->w_host.assign(vg->w, vg->w + vg->n_v);
  if (opts && opts->sweep_threads) {
    BGK_CHECK(opts->sweep_threads >= 64 && opts->sweep_threads <= 256 &&
                  opts->sweep_threads % 64 == 0,
              BGK_E_INVALID, "sweep_threads must be a multiple of 64 in [64, 256]");
    D->sweep_threads = opts->sweep_threads;
  }
  const int lanes_opt = opts ? opts->sweep_lanes : 0;
  BGK_CHECK(lanes_opt == 0 || (lanes_opt >= 1 && lanes_opt <= 64 && (lanes_opt & (lanes_opt - 1)) == 0),
            BGK_E_INVALID, "sweep_lanes must be 0 or a power of two up to 64");
  BGK_CHECK(!(opts && opts->sweep_threads && lanes_opt && lanes_opt < 64), BGK_E_INVALID,
            "sweep_threads sets the workgroup walk; it cannot be combined with packed lanes");
  if (opts && opts->ring_slots) {
    const int r = opts->ring_slots;
    BGK_CHECK(r >= 16 && r <= 1024 && (r & (r - 1)) == 0, BGK_E_INVALID,
              "ring_slots must be a power of two in [16, 1024]");
    D->ring_slots = r;
  }
  // tensor grid declaration
  D->n_1d = vg->n_1d;
  if (vg->n_1d > 0) {
    BGK_CHECK(vg->nodes_1d && vg->weights_1d, BGK_E_INVALID, "tensor grid without 1D factors");
    int64_t expect = 1;
    for (int d = 0; d < dim; ++d) expect *= vg->n_1d;
    BGK_CHECK(expect == vg->n_v, BGK_E_INVALID, "n_v != n_1d^dim");
    D->nodes_1d.assign(vg->nodes_1d, vg->nodes_1d + vg->n_1d);
    D->weights_1d.assign(vg->weights_1d, vg->weights_1d + vg->n_1d);
    for (int j = 0; j < vg->n_v; ++j) {
      int rem = j;
      double w = 1.0;
      int idx[3];
      for (int d = dim - 1; d >= 0; --d) {
        idx[d] = rem % vg->n_1d;
        rem /= vg->n_1d;
      }
      for (int d = 0; d < dim; ++d) {
        w *= vg->weights_1d[idx[d]];
        BGK_CHECK(vg->v[(size_t)j * dim + d] == vg->nodes_1d[idx[d]], BGK_E_INVALID,
                  "velocity grid is not the declared tensor product");
      }
      BGK_CHECK(std::fabs(w - vg->w[j]) <= 1e-13 * std::fabs(w), BGK_E_INVALID,
                "weights are not the declared tensor product");
    }
  }
  // Q2 discontinuous-Galerkin velocity space (Sec. 3.2): on each of the
  // dg_cells uniform cells of [-L, L] the 3-point Gauss-Legendre nodes
  // centre + (h/2) xi with weights (h/2) (5/9, 8/9, 5/9)
  if (vg->dg_cells) {
    const int nc1 = vg->dg_cells;
    BGK_CHECK(nc1 > 0, BGK_E_INVALID, "dg_cells must be positive");
    BGK_CHECK(vg->n_1d == 3 * nc1, BGK_E_INVALID, "a Q2 velocity space needs n_1d = 3*dg_cells");
    BGK_CHECK(vg->L > 0, BGK_E_INVALID, "a Q2 velocity space needs L > 0");
    const double h = 2.0 * vg->L / nc1;
    const double xi[3] = {-std::sqrt(0.6), 0.0, std::sqrt(0.6)};
    const double wr[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    for (int c = 0; c < nc1; ++c)
      for (int k = 0; k < 3; ++k) {
        const double x = -vg->L + h * (c + 0.5) + 0.5 * h * xi[k];
        const double w = 0.5 * h * wr[k];
        BGK_CHECK(std::fabs(vg->nodes_1d[3 * c + k] - x) <= 1e-12 * vg->L &&
                      std::fabs(vg->weights_1d[3 * c + k] - w) <= 1e-12 * w,
                  BGK_E_INVALID, "nodes_1d / weights_1d are not the Q2 Gauss-Legendre grid");
      }
    D->dg_cells = nc1;
  }
  const int64_t nc = H.n_cells;
  const int nf = dim + 1;
  // Morton order of centroids -> internal numbering
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t c = 0; c < nc; ++c)
    for (int d = 0; d < dim; ++d) {
      lo[d] = std::min(lo[d], H.centroid[c * dim + d]);
      hi[d] = std::max(hi[d], H.centroid[c * dim + d]);
    }
  std::vector<std::pair<uint64_t, int32_t>> mk(nc);
  const double scale = dim == 2 ? 2147483647.0 : 2097151.0;
  for (int64_t c = 0; c < nc; ++c) {
    uint64_t code = 0;
    for (int d = 0; d < dim; ++d) {
      const double t = (H.centroid[c * dim + d] - lo[d]) / std::max(hi[d] - lo[d], 1e-300);
      code |= spread_bits((uint64_t)(t * scale), dim) << d;
    }
    mk[c] = {code, (int32_t)c};
  }
  std::stable_sort(mk.begin(), mk.end(),
                   [](const auto& a, const auto& b) { return a.first < b.first; });
  D->uid_host.resize(nc);
  D->iid_host.resize(nc);
  for (int64_t i = 0; i < nc; ++i) {
    D->uid_host[i] = mk[i].second;
    D->iid_host[mk[i].second] = (int32_t)i;
  }
  // internal-order device records
  const int gs = 1 + (dim + 1) * dim;  // host record
  const int gstride = dim == 2 ? GeoLayout<2>::STRIDE : GeoLayout<3>::STRIDE;  // padded device record
  std::vector<double> geo_i(nc * gstride, 0.0);
  std::vector<FacetRec> fac_i(nc * nf);
  for (int64_t i = 0; i < nc; ++i) {
    const int64_t u = D->uid_host[i];
    std::copy(&H.geo[u * gs], &H.geo[u * gs] + gs, &geo_i[i * gstride]);
    for (int k = 0; k < nf; ++k) {
      const int32_t nb = H.nb[u * nf + k];
      FacetRec r;
      r.nb = nb >= 0 ? D->iid_host[nb] : nb;
      int pack = nb >= 0 ? (H.nb_face[u * nf + k] & 3) : 0;
      if (nb >= 0)
        for (int p = 0; p < H.n_fp; ++p) pack |= (H.nb_node[(u * nf + k) * H.n_fp + p] & 15) << (4 * (p + 1));
      r.pack = pack;
      fac_i[i * nf + k] = r;
    }
  }
  D->node_x = std::move(H.node_x);
  D->bnode_x = std::move(H.bnode_x);
  D->bface_cell = std::move(H.bcell);
  D->bface_pack = std::move(H.bpack);
  D->bface_normal = std::move(H.bnormal);
  D->vol_user = std::move(H.vol);
  const int nv = vg->n_v;
  if ((rc = dalloc(&D->d_geo, geo_i.size()))) return rc;
  if ((rc = dalloc(&D->d_uid, nc))) return rc;
  if ((rc = dalloc(&D->d_facet, fac_i.size()))) return rc;
  if ((rc = dalloc(&D->d_v, (size_t)nv * dim))) return rc;
  if ((rc = dalloc(&D->d_w, (size_t)nv))) return rc;
  if ((rc = dalloc(&D->d_perm, (size_t)nv * nc))) return rc;
  if ((rc = dalloc(&D->d_pos, (size_t)nv * nc))) return rc;
  if ((rc = dalloc(&D->d_G, (size_t)nv))) return rc;
  if ((rc = dalloc(&D->d_gbase, (size_t)nv))) return rc;
  if ((rc = dalloc(&D->d_vorder, (size_t)nv))) return rc;
  if ((rc = dalloc(&D->d_lag, (size_t)nv * nc))) return rc;
  BGK_HIP(hipMemcpyAsync(D->d_geo, geo_i.data(), geo_i.size() * sizeof(double),
                         hipMemcpyHostToDevice, stream));
  BGK_HIP(hipMemcpyAsync(D->d_uid, D->uid_host.data(), nc * sizeof(int32_t),
                         hipMemcpyHostToDevice, stream));
  BGK_HIP(hipMemcpyAsync(D->d_facet, fac_i.data(), fac_i.size() * sizeof(FacetRec),
                         hipMemcpyHostToDevice, stream));
  BGK_HIP(hipMemcpyAsync(D->d_v, D->v_host.data(), D->v_host.size() * sizeof(double),
                         hipMemcpyHostToDevice, stream));
  BGK_HIP(hipMemcpyAsync(D->d_w, D->w_host.data(), D->w_host.size() * sizeof(double),
                         hipMemcpyHostToDevice, stream));
  if (D->n_1d > 0) {
    if ((rc = dalloc(&D->d_nodes1d, D->n_1d))) return rc;
    if ((rc = dalloc(&D->d_weights1d, D->n_1d))) return rc;
    BGK_HIP(hipMemcpyAsync(D->d_nodes1d, D->nodes_1d.data(), D->n_1d * sizeof(double),
                           hipMemcpyHostToDevice, stream));
    BGK_HIP(hipMemcpyAsync(D->d_weights1d, D->weights_1d.data(), D->n_1d * sizeof(double),
                           hipMemcpyHostToDevice, stream));
  }
  uint8_t* d_ulag = nullptr;
  std::vector<uint8_t> ulag_i;
  if (opts && opts->lagged) {
    ulag_i.resize((size_t)nv * nc);
    for (int j = 0; j < nv; ++j)
      for (int64_t i = 0; i < nc; ++i)
        ulag_i[(size_t)j * nc + i] = opts->lagged[(size_t)j * nc + D->uid_host[i]] & ((1 << nf) - 1);
    if ((rc = dalloc(&d_ulag, ulag_i.size()))) return rc;
    BGK_HIP(hipMemcpyAsync(d_ulag, ulag_i.data(), ulag_i.size(), hipMemcpyHostToDevice, stream));
  }
  // batches of velocities bounded by ~1 GiB of scratch
  const size_t per_v = (size_t)2 * (nc + 1) * sizeof(int32_t);
  int batch = (int)std::max<size_t>(1, std::min<size_t>(nv, ((size_t)1 << 30) / per_v));
  int32_t *s_cnt = nullptr, *s_cur = nullptr;
  unsigned long long* d_nlag = nullptr;
  if ((rc = dalloc(&s_cnt, (size_t)batch * (nc + 1)))) return rc;
  if ((rc = dalloc(&s_cur, (size_t)batch * (nc + 1)))) return rc;
  if ((rc = dalloc(&d_nlag, 1))) return rc;
  BGK_HIP(hipMemsetAsync(d_nlag, 0, sizeof(unsigned long long), stream));
  DagArgs a{D->d_geo, D->d_facet, D->d_v, d_ulag, D->d_lag, D->d_perm, D->d_pos,
            s_cnt, s_cur, D->d_G, d_nlag, (int)nc};
  D->G_host.resize(nv);
  D->gbase_host.resize(nv);
  int64_t total_goff = 0;
  std::vector<int32_t> goff_host;
  // levels per batch of velocities; offsets copied to host per batch
  const auto levels = [&]() -> int {
    total_goff = 0;
    goff_host.clear();
    for (int j0 = 0; j0 < nv; j0 += batch) {
      const int nb = std::min(batch, nv - j0);
      if (dim == 2)
        hipLaunchKernelGGL(k_dag_levels<2>, dim3(nb), dim3(DAG_THREADS), 0, stream, a, j0);
      else
        hipLaunchKernelGGL(k_dag_levels<3>, dim3(nb), dim3(DAG_THREADS), 0, stream, a, j0);
      BGK_HIP(hipGetLastError());
      BGK_HIP(hipMemcpyAsync(D->G_host.data() + j0, D->d_G + j0, nb * sizeof(int32_t),
                             hipMemcpyDeviceToHost, stream));
      BGK_HIP(hipStreamSynchronize(stream));
      std::vector<int32_t> cnt_host((size_t)nb * (nc + 1));
      BGK_HIP(hipMemcpy(cnt_host.data(), s_cnt, cnt_host.size() * sizeof(int32_t),
                        hipMemcpyDeviceToHost));
      for (int jb = 0; jb < nb; ++jb) {
        const int j = j0 + jb;
        D->gbase_host[j] = total_goff;
        const int G = D->G_host[j];
        BGK_CHECK(G > 0, BGK_E_INVALID,
                  "generation construction failed for velocity " + std::to_string(j));
        goff_host.insert(goff_host.end(), cnt_host.begin() + (size_t)jb * (nc + 1),
                         cnt_host.begin() + (size_t)jb * (nc + 1) + G + 1);
        total_goff += G + 1;
      }
    }
    return BGK_OK;
  };
  if ((rc = levels())) return rc;
  unsigned long long nlag = 0;
  BGK_HIP(hipMemcpyAsync(&nlag, d_nlag, sizeof(nlag), hipMemcpyDeviceToHost, stream));
  BGK_HIP(hipStreamSynchronize(stream));
  if (nlag > 0) {
    // cycles were broken: the levels of that pass are not longest paths of
    // the lagged graph; repeat it with every lagged facet given (the graph is
    // now acyclic, so nothing more is lagged)
    a.user_lag = D->d_lag;
    if ((rc = levels())) return rc;
    unsigned long long nlag2 = 0;
    BGK_HIP(hipMemcpyAsync(&nlag2, d_nlag, sizeof(nlag2), hipMemcpyDeviceToHost, stream));
    BGK_HIP(hipStreamSynchronize(stream));
    BGK_CHECK(nlag2 == nlag, BGK_E_INVALID, "cycle breaking left a cycle");
  }
  if ((rc = dalloc(&D->d_goff, (size_t)total_goff))) return rc;
  BGK_HIP(hipMemcpyAsync(D->d_goff, goff_host.data(), total_goff * sizeof(int32_t),
                         hipMemcpyHostToDevice, stream));
  BGK_HIP(hipMemcpyAsync(D->d_gbase, D->gbase_host.data(), nv * sizeof(int64_t),
                         hipMemcpyHostToDevice, stream));
  BGK_HIP(hipStreamSynchronize(stream));
  (void)hipFree(s_cnt);
  (void)hipFree(s_cur);
  (void)hipFree(d_nlag);
  if (d_ulag) (void)hipFree(d_ulag);
  int64_t user_lag_bits = 0;
  for (uint8_t b : ulag_i) user_lag_bits += __builtin_popcount(b);
  D->n_lagged = (int64_t)nlag + user_lag_bits;
  if (D->n_lagged == 0) {
    (void)hipFree(D->d_lag);
    D->d_lag = nullptr;
  }
  D->max_G = 0;
  for (int j = 0; j < nv; ++j) D->max_G = std::max(D->max_G, D->G_host[j]);
  // sweep item records
  if ((rc = dalloc(&D->d_rec, (size_t)nv * nc * 4))) return rc;
  if ((rc = dalloc(&D->d_recx, (size_t)nv * nc))) return rc;
  {
    const int64_t total = (int64_t)nv * nc;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
    if (dim == 2)
      hipLaunchKernelGGL(k_records<2>, dim3(grid), dim3(256), 0, stream, D->d_geo, D->d_facet,
                         D->d_v, D->d_perm, D->d_pos, D->d_lag, D->d_rec, D->d_recx, (int)nc,
                         D->n_fp, 0, nv);
    else
      hipLaunchKernelGGL(k_records<3>, dim3(grid), dim3(256), 0, stream, D->d_geo, D->d_facet,
                         D->d_v, D->d_perm, D->d_pos, D->d_lag, D->d_rec, D->d_recx, (int)nc,
                         D->n_fp, 0, nv);
    BGK_HIP(hipGetLastError());
  }
  if ((rc = dalloc(&D->d_gmin, (size_t)total_goff))) return rc;
  hipLaunchKernelGGL(k_gen_reach, dim3(nv), dim3(256), 0, stream, D->d_rec, D->d_goff, D->d_gbase,
                     D->d_G, D->d_gmin, (int)nc, dim);
  BGK_HIP(hipGetLastError());
  // sweep block order.  Workgroups are dispatched round-robin over the 8
  // XCDs (block b -> XCD b % 8), each with its own L2.  Velocities sorted by
  // direction are dealt to XCDs in 8 contiguous angular sectors (2D) or by
  // octant (3D), so the velocities sharing an L2 sweep similar fronts and
  // reuse each other's cell data.  Within a sector, blocks that run together
  // are angular neighbours.
  std::vector<int32_t> vorder(nv);
  {
    std::vector<std::pair<double, int32_t>> key(nv);
    for (int j = 0; j < nv; ++j) key[j] = {velocity_key(&D->v_host[(size_t)j * dim], dim), j};
    std::stable_sort(key.begin(), key.end());
    const std::vector<int32_t> pos = deal_sectors(nv);
    for (int b = 0; b < nv; ++b) vorder[b] = key[pos[b]].second;
  }
  BGK_HIP(hipMemcpyAsync(D->d_vorder, vorder.data(), nv * sizeof(int32_t), hipMemcpyHostToDevice,
                         stream));
  if ((rc = set_sweep_walk(D, opts ? opts->sweep_threads : 0, lanes_opt, stream))) return rc;
  BGK_HIP(hipStreamSynchronize(stream));
  return BGK_OK;
}

}  // namespace bgk

using namespace bgk;

extern "C" int build_mesh_dag(const tgs_mesh_desc* mesh, const tgs_vgrid_desc* vgrid,
                              const tgs_dag_opts* opts, bgk_stream_t stream, tgs_dag** out) {
  return guarded([&]() -> int {
    if (!mesh || !vgrid || !out) return fail(BGK_E_INVALID, "null argument");
    *out = nullptr;
    if (vgrid->n_v <= 0) return fail(BGK_E_INVALID, "n_v must be positive");
    tgs_dag* D = new (std::nothrow) tgs_dag();
    if (!D) return fail(BGK_E_NOMEM, "host allocation failed");
    int rc;
    try {
      rc = build_dag_impl(mesh, vgrid, opts, (hipStream_t)stream, D);
    } catch (const std::exception& e) {
      rc = fail(BGK_E_NOMEM, std::string("host exception: ") + e.what());
    }
    if (rc) {
      free_dag(D);
      return rc;
    }
    *out = D;
    return BGK_OK;
  });
}

extern "C" int tgs_dag_destroy(tgs_dag* dag) {
  return guarded([&]() -> int {
    free_dag(dag);
    return BGK_OK;
  });
}

extern "C" int tgs_dag_sizes(const tgs_dag* d, int64_t s[9]) {
  return guarded([&]() -> int {
    if (!d || !s) return fail(BGK_E_INVALID, "null argument");
    s[0] = d->dim;
    s[1] = d->order;
    s[2] = d->n_p;
    s[3] = d->n_fp;
    s[4] = d->n_cells;
    s[5] = d->n_v;
    s[6] = d->n_bfaces;
    s[7] = d->max_G;
    s[8] = d->n_lagged;
    return BGK_OK;
  });
}

extern "C" int tgs_dag_generations(const tgs_dag* d, int32_t* gen, int32_t* G) {
  return guarded([&]() -> int {
    if (!d) return fail(BGK_E_INVALID, "null dag");
    if (G) std::copy(d->G_host.begin(), d->G_host.end(), G);
    if (!gen) return BGK_OK;
    const int64_t nc = d->n_cells;
    std::vector<int32_t> perm((size_t)d->n_v * nc);
    std::vector<int32_t> goff;
    BGK_HIP(hipMemcpy(perm.data(), d->d_perm, perm.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    int64_t total = 0;
    for (int j = 0; j < d->n_v; ++j) total += d->G_host[j] + 1;
    goff.resize(total);
    BGK_HIP(hipMemcpy(goff.data(), d->d_goff, total * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int j = 0; j < d->n_v; ++j) {
      const int32_t* go = goff.data() + d->gbase_host[j];
      for (int g = 0; g < d->G_host[j]; ++g)
        for (int s = go[g]; s < go[g + 1]; ++s)
          gen[(size_t)j * nc + d->uid_host[perm[(size_t)j * nc + s]]] = g;
    }
    return BGK_OK;
  });
}

extern "C" int tgs_dag_lagged(const tgs_dag* d, uint8_t* lagged) {
  return guarded([&]() -> int {
    if (!d || !lagged) return fail(BGK_E_INVALID, "null argument");
    const int64_t nc = d->n_cells;
    if (!d->d_lag) {
      std::memset(lagged, 0, (size_t)d->n_v * nc);
      return BGK_OK;
    }
    std::vector<uint8_t> tmp((size_t)d->n_v * nc);
    BGK_HIP(hipMemcpy(tmp.data(), d->d_lag, tmp.size(), hipMemcpyDeviceToHost));
    for (int j = 0; j < d->n_v; ++j)
      for (int64_t i = 0; i < nc; ++i) lagged[(size_t)j * nc + d->uid_host[i]] = tmp[(size_t)j * nc + i];
    return BGK_OK;
  });
}

extern "C" int tgs_dag_sweep_lanes(const tgs_dag* d) { return d ? d->sweep_lanes : 0; }
extern "C" int tgs_dag_set_walk(tgs_dag* d, int threads, int lanes) {
  return guarded([&]() -> int {
    if (!d) return fail(BGK_E_INVALID, "null argument");
    BGK_CHECK(threads == 0 || (threads >= 64 && threads <= 256 && threads % 64 == 0), BGK_E_INVALID,
              "threads must be 0 or a multiple of 64 in [64, 256]");
    BGK_CHECK(lanes == 0 || (lanes >= 1 && lanes <= 64 && (lanes & (lanes - 1)) == 0),
              BGK_E_INVALID, "lanes must be 0 or a power of two up to 64");
    BGK_CHECK(!(threads && lanes && lanes < 64), BGK_E_INVALID,
              "threads sets the workgroup walk; it cannot be combined with packed lanes");
    BGK_HIP(hipSetDevice(d->device));
    BGK_HIP(hipDeviceSynchronize());
    return set_sweep_walk(d, threads, lanes, nullptr);
  });
}

extern "C" int tgs_dag_explicit_dt(const tgs_dag* d, double cfl, double* dt) {
  return guarded([&]() -> int {
    if (!d || !dt) return fail(BGK_E_INVALID, "null argument");
    if (!(cfl > 0.0)) return fail(BGK_E_INVALID, "cfl must be positive");
    // eq. explicit-dt: h_min from the smallest cell measure, the largest speed
    double vmin = d->vol_user.empty() ? 0.0 : d->vol_user[0];
    for (double x : d->vol_user) vmin = std::min(vmin, x);
    double s2 = 0.0;
    for (int64_t j = 0; j < d->n_v; ++j) {
      double a = 0.0;
      for (int k = 0; k < d->dim; ++k) a += d->v_host[j * d->dim + k] * d->v_host[j * d->dim + k];
      s2 = std::max(s2, a);
    }
    if (!(s2 > 0.0) || !(vmin > 0.0)) return fail(BGK_E_INVALID, "zero speed or cell measure");
    const double hmin = std::pow(vmin, 1.0 / d->dim);
    *dt = cfl * (1.0 / d->dim) * (1.0 / (2 * d->order + 1)) * hmin / std::sqrt(s2);
    return BGK_OK;
  });
}

extern "C" int tgs_dag_geometry(const tgs_dag* d, double* node_x, double* bnode_x, double* vol) {
  return guarded([&]() -> int {
    if (!d) return fail(BGK_E_INVALID, "null dag");
    if (node_x) std::copy(d->node_x.begin(), d->node_x.end(), node_x);
    if (bnode_x) std::copy(d->bnode_x.begin(), d->bnode_x.end(), bnode_x);
    if (vol) std::copy(d->vol_user.begin(), d->vol_user.end(), vol);
    return BGK_OK;
  });
}
