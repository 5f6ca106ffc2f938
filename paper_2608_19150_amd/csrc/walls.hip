// Bounce-back and specular-reflection walls (Sec. "Boundary conditions"):
// f_bc(x, v) = f(x, T v) with T v = -v or T v = v - 2 (v.n) n.  On a
// velocity set closed under T the boundary value of velocity j at a wall
// facet node is the distribution of velocity T(j) at the same node, so the
// boundary update of a Picard iteration is a gather from the previous
// iterate into the dense boundary array the sweep reads.
#include <array>
#include <cmath>
#include <map>
#include <vector>

#include "device_common.h"
#include "walls.h"

struct tgs_walls {
  const tgs_dag* dag = nullptr;
  int64_t n_walls = 0;
  int n_maps = 0;
  int max_in = 0;             // longest incoming list
  int4* d_wall = nullptr;     // [n_walls]: boundary facet, internal cell, map, facet nodes
  int32_t* d_map = nullptr;   // [n_maps][n_v]: T(j)
  // per map: the velocities that can enter through such a wall (v.n <= 0 up
  // to the tangential tolerance), the only ones whose boundary data a sweep
  // reads; d_in_off[m] .. d_in_off[m + 1] index d_in
  int32_t* d_in = nullptr;
  int32_t* d_in_off = nullptr;
};

namespace bgk {

namespace {

// one thread per (wall facet, incoming velocity), velocities fastest: the
// writes of a wavefront to one boundary row are nearly contiguous
__global__ __launch_bounds__(256) void k_wall_values(const int4* __restrict__ wall,
                                                     const int32_t* __restrict__ map,
                                                     const int32_t* __restrict__ in,
                                                     const int32_t* __restrict__ in_off,
                                                     const int32_t* __restrict__ pos,
                                                     const double* __restrict__ f,
                                                     double* __restrict__ bc, int64_t n_walls,
                                                     int max_in, int n_v, int64_t n_cells,
                                                     int np, int nfp, const int32_t* skip) {
  if (skip_launch(skip)) return;
  const int64_t total = n_walls * max_in;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = t / max_in;
    const int k = (int)(t - w * max_in);
    const int4 W = wall[w];
    const int i0 = in_off[W.z];
    if (k >= in_off[W.z + 1] - i0) continue;
    const int j = in[i0 + k];
    const int jj = map[(int64_t)W.z * n_v + j];
    const int64_t slot = pos[(int64_t)jj * n_cells + W.y];
    const double* src = f + ((int64_t)jj * n_cells + slot) * np;
    for (int p = 0; p < nfp; ++p)
      bc[((int64_t)W.x * nfp + p) * n_v + j] = src[(W.w >> (4 * p)) & 15];
  }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_bc_dense(const double* __restrict__ coef,
                                                  const double* __restrict__ v,
                                                  double* __restrict__ bc, int64_t rows,
                                                  int n_v) {
  constexpr int NC = DIM + 2;
  const int64_t total = rows * n_v;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / n_v;
    const int j = (int)(t - r * n_v);
    double vv[DIM], v2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      vv[d] = v[(int64_t)j * DIM + d];
      v2 = fma(vv[d], vv[d], v2);
    }
    bc[t] = maxw_eval<DIM>(coef + r * NC, vv, v2);
  }
}

unsigned grid_of(int64_t total) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
}

// T(j) for every velocity by matching T v_j against the set: velocities are
// bucketed on a lattice of spacing 2 tol, so a match within tol lies in the
// image's bucket or a neighbouring one
int velocity_map(const tgs_dag* d, int kind, const double* nrm, std::vector<int32_t>& out) {
  const int dim = d->dim, nv = d->n_v;
  double scale = 1.0;
  for (double x : d->v_host) scale = std::max(scale, std::fabs(x));
  const double tol = 1e-9 * scale, cell = 2.0 * tol;
  using Key = std::array<int64_t, 3>;
  std::map<Key, std::vector<int32_t>> buckets;
  auto key_of = [&](const double* x) {
    Key k{0, 0, 0};
    for (int a = 0; a < dim; ++a) k[a] = (int64_t)std::floor(x[a] / cell);
    return k;
  };
  for (int j = 0; j < nv; ++j) buckets[key_of(&d->v_host[(size_t)j * dim])].push_back(j);
  out.assign(nv, -1);
  for (int j = 0; j < nv; ++j) {
    const double* vj = &d->v_host[(size_t)j * dim];
    double img[3] = {0, 0, 0};
    double vn = 0.0;
    for (int a = 0; a < dim; ++a) vn += vj[a] * nrm[a];
    for (int a = 0; a < dim; ++a)
      img[a] = kind == BGK_BC_BOUNCE_BACK ? -vj[a] : vj[a] - 2.0 * vn * nrm[a];
    const Key k = key_of(img);
    const int r1 = dim > 1 ? 1 : 0, r2 = dim > 2 ? 1 : 0;
    double best = tol;
    for (int o0 = -1; o0 <= 1; ++o0)
      for (int o1 = -r1; o1 <= r1; ++o1)
        for (int o2 = -r2; o2 <= r2; ++o2) {
          auto it = buckets.find(Key{k[0] + o0, k[1] + o1, k[2] + o2});
          if (it == buckets.end()) continue;
          for (int32_t c : it->second) {
            double dist = 0.0;
            for (int a = 0; a < dim; ++a)
              dist = std::max(dist, std::fabs(d->v_host[(size_t)c * dim + a] - img[a]));
            if (dist <= best) {
              best = dist;
              out[j] = c;
            }
          }
        }
    BGK_CHECK(out[j] >= 0, BGK_E_INVALID,
              "the velocity set is not closed under a wall's velocity map");
  }
  return BGK_OK;
}

}  // namespace

const tgs_dag* walls_dag(const tgs_walls* w) { return w->dag; }

int launch_wall_values(const tgs_walls* w, const double* f, double* bc_dense, hipStream_t stream,
                       const int32_t* skip) {
  const tgs_dag* d = w->dag;
  if (w->n_walls == 0 || w->max_in == 0) return BGK_OK;
  hipLaunchKernelGGL(k_wall_values, dim3(grid_of(w->n_walls * w->max_in)), dim3(256), 0, stream,
                     w->d_wall, w->d_map, w->d_in, w->d_in_off, d->d_pos, f, bc_dense, w->n_walls,
                     w->max_in, d->n_v, d->n_cells, d->n_p, d->n_fp, skip);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_bc_dense(const tgs_dag* d, const double* bc_coef, double* bc_dense,
                    hipStream_t stream) {
  const int64_t rows = d->n_bfaces * d->n_fp;
  if (rows == 0) return BGK_OK;
  if (d->dim == 2)
    hipLaunchKernelGGL(k_bc_dense<2>, dim3(grid_of(rows * d->n_v)), dim3(256), 0, stream,
                       bc_coef, d->d_v, bc_dense, rows, d->n_v);
  else
    hipLaunchKernelGGL(k_bc_dense<3>, dim3(grid_of(rows * d->n_v)), dim3(256), 0, stream,
                       bc_coef, d->d_v, bc_dense, rows, d->n_v);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

}  // namespace bgk

using namespace bgk;

extern "C" int tgs_walls_destroy(tgs_walls* w) {
  return guarded([&]() -> int {
    if (!w) return BGK_OK;
    if (w->d_wall) (void)hipFree(w->d_wall);
    if (w->d_map) (void)hipFree(w->d_map);
    if (w->d_in) (void)hipFree(w->d_in);
    if (w->d_in_off) (void)hipFree(w->d_in_off);
    delete w;
    return BGK_OK;
  });
}

extern "C" int tgs_walls_create(const tgs_dag* d, const int8_t* kind, tgs_walls** out) {
  return guarded([&]() -> int {
    if (!d || !out || (!kind && d->n_bfaces > 0)) return fail(BGK_E_INVALID, "null argument");
    *out = nullptr;
    const int dim = d->dim;
    std::vector<int4> wall;
    std::vector<int32_t> maps, in, in_off{0};
    std::map<std::array<double, 4>, int> map_id;   // (kind, unit normal) -> map
    for (int64_t bf = 0; bf < d->n_bfaces; ++bf) {
      const int k = kind[bf];
      if (k != BGK_BC_INFLOW && k != BGK_BC_BOUNCE_BACK && k != BGK_BC_REFLECT)
        return fail(BGK_E_INVALID, "unknown boundary kind at facet " + std::to_string(bf));
      if (k == BGK_BC_INFLOW) continue;
      const double* nrm = &d->bface_normal[(size_t)bf * dim];
      // one map per (kind, normal): the velocity map of bounce-back does not
      // depend on the normal, but the incoming velocities do
      std::array<double, 4> key{(double)k, 0, 0, 0};
      for (int a = 0; a < dim; ++a) key[1 + a] = nrm[a];
      auto it = map_id.find(key);
      int id;
      if (it == map_id.end()) {
        std::vector<int32_t> m;
        const int rc = velocity_map(d, k, nrm, m);
        if (rc) return rc;
        id = (int)map_id.size();
        map_id.emplace(key, id);
        maps.insert(maps.end(), m.begin(), m.end());
        // incoming velocities of this map (a superset of those the sweep reads:
        // it treats |v.N| <= 1e-12 |v| |N| as tangential)
        for (int j = 0; j < d->n_v; ++j) {
          double vn = 0.0, v2 = 0.0;
          for (int a = 0; a < dim; ++a) {
            const double x = d->v_host[(size_t)j * dim + a];
            vn += x * nrm[a];
            v2 += x * x;
          }
          if (vn <= 1e-9 * std::sqrt(v2)) in.push_back(j);
        }
        in_off.push_back((int32_t)in.size());
      } else {
        id = it->second;
      }
      wall.push_back(make_int4((int)bf, d->iid_host[d->bface_cell[bf]], id, d->bface_pack[bf]));
    }
    tgs_walls* w = new (std::nothrow) tgs_walls();
    if (!w) return fail(BGK_E_NOMEM, "host allocation failed");
    w->dag = d;
    w->n_walls = (int64_t)wall.size();
    w->n_maps = (int)map_id.size();
    for (size_t m = 0; m + 1 < in_off.size(); ++m)
      w->max_in = std::max(w->max_in, in_off[m + 1] - in_off[m]);
    if (!wall.empty()) {
      if (hipMalloc((void**)&w->d_wall, wall.size() * sizeof(int4)) != hipSuccess ||
          hipMalloc((void**)&w->d_map, maps.size() * sizeof(int32_t)) != hipSuccess ||
          hipMalloc((void**)&w->d_in, std::max<size_t>(in.size(), 1) * sizeof(int32_t)) !=
              hipSuccess ||
          hipMalloc((void**)&w->d_in_off, in_off.size() * sizeof(int32_t)) != hipSuccess) {
        tgs_walls_destroy(w);
        return fail(BGK_E_NOMEM, "wall arrays");
      }
      if (hipMemcpy(w->d_wall, wall.data(), wall.size() * sizeof(int4), hipMemcpyHostToDevice) !=
              hipSuccess ||
          hipMemcpy(w->d_map, maps.data(), maps.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
              hipSuccess ||
          (!in.empty() && hipMemcpy(w->d_in, in.data(), in.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice) != hipSuccess) ||
          hipMemcpy(w->d_in_off, in_off.data(), in_off.size() * sizeof(int32_t),
                    hipMemcpyHostToDevice) != hipSuccess) {
        tgs_walls_destroy(w);
        return fail(BGK_E_HIP, "wall arrays copy");
      }
    }
    *out = w;
    return BGK_OK;
  });
}

extern "C" int64_t tgs_walls_count(const tgs_walls* w) { return w ? w->n_walls : 0; }

extern "C" int tgs_wall_values(const tgs_walls* w, const double* f, double* bc_dense,
                               bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!w || !f || !bc_dense) return fail(BGK_E_INVALID, "null argument");
    return launch_wall_values(w, f, bc_dense, (hipStream_t)stream);
  });
}
