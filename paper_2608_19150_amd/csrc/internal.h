// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <new>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/bgktgs.h"

namespace bgk {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define BGK_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::bgk::fail(BGK_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define BGK_CHECK(cond, code, msg)       \
  do {                                   \
    if (!(cond)) return ::bgk::fail(code, msg); \
  } while (0)

// Records a fixed message without allocating (safe inside a catch handler).
int fail_static(int code, const char* msg) noexcept;

// Runs the body of an entry point so that no C++ exception crosses the C
// ABI: a host allocation failure (std::bad_alloc from a std::vector or
// std::map) or any other exception becomes BGK_E_NOMEM with its message.
template <class F>
int guarded(F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail_static(BGK_E_NOMEM, "host allocation failed (std::bad_alloc)");
  } catch (const std::exception& e) {
    try {
      return fail(BGK_E_NOMEM, std::string("host exception: ") + e.what());
    } catch (...) {
      return fail_static(BGK_E_NOMEM, "host exception");
    }
  } catch (...) {
    return fail_static(BGK_E_NOMEM, "unknown host exception");
  }
}

// ---------------------------------------------------------------------------
// Reference-element matrices, evaluated at compile time.
//
// Basis functions are polynomials in the barycentric coordinates
// lambda_0..lambda_d (P1: lambda_a; P2 triangle: lambda_k(2 lambda_k - 1) at
// vertices, 4 lambda_i lambda_j at edge midpoints (0,1),(1,2),(2,0)).  On a
// simplex of measure |K|,
//     int_K prod_i lambda_i^a_i = |K| d! prod_i a_i! / (sum a + d)!,
// which makes every element integral an exact rational; the tables hold
// those rationals rounded to double by the compiler.
// ---------------------------------------------------------------------------
struct Term {
  double c;
  int e[4];
};
struct Poly {
  int n = 0;
  Term t[24] = {};
};

constexpr double cfact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}
constexpr Poly p_mul(const Poly& a, const Poly& b) {
  Poly r;
  for (int i = 0; i < a.n; ++i)
    for (int j = 0; j < b.n; ++j) {
      Term t{a.t[i].c * b.t[j].c, {0, 0, 0, 0}};
      for (int k = 0; k < 4; ++k) t.e[k] = a.t[i].e[k] + b.t[j].e[k];
      r.t[r.n++] = t;
    }
  return r;
}
constexpr Poly p_dlam(const Poly& a, int var) {  // d/d lambda_var
  Poly r;
  for (int i = 0; i < a.n; ++i)
    if (a.t[i].e[var] > 0) {
      Term t = a.t[i];
      t.c *= t.e[var];
      t.e[var] -= 1;
      r.t[r.n++] = t;
    }
  return r;
}
// d/d xi_beta (beta = 1..d) with lambda_0 = 1 - sum xi, lambda_beta = xi_beta
constexpr Poly p_dxi(const Poly& a, int beta) {
  Poly r = p_dlam(a, beta);
  Poly m = p_dlam(a, 0);
  for (int i = 0; i < m.n; ++i) {
    Term t = m.t[i];
    t.c = -t.c;
    r.t[r.n++] = t;
  }
  return r;
}
// integral over a dim-simplex divided by its measure
constexpr double p_int_norm(const Poly& p, int dim) {
  double s = 0.0;
  for (int i = 0; i < p.n; ++i) {
    double num = 1.0;
    int deg = 0;
    for (int k = 0; k < 4; ++k) {
      num *= cfact(p.t[i].e[k]);
      deg += p.t[i].e[k];
    }
    s += p.t[i].c * cfact(dim) * num / cfact(deg + dim);
  }
  return s;
}
// integral over facet `drop` (lambda_drop = 0) divided by the facet measure
constexpr double p_int_facet_norm(const Poly& p, int dim, int drop) {
  double s = 0.0;
  for (int i = 0; i < p.n; ++i) {
    if (p.t[i].e[drop] != 0) continue;
    double num = 1.0;
    int deg = 0;
    for (int k = 0; k < 4; ++k) {
      num *= cfact(p.t[i].e[k]);
      deg += p.t[i].e[k];
    }
    s += p.t[i].c * cfact(dim - 1) * num / cfact(deg + dim - 1);
  }
  return s;
}
constexpr Poly p_lam(int i) {
  Poly r;
  r.n = 1;
  r.t[0] = Term{1.0, {0, 0, 0, 0}};
  r.t[0].e[i] = 1;
  return r;
}

template <int DIM, int ORDER>
struct Elem;

template <int DIM, int ORDER>
struct ElemBuild {
  static constexpr int NP = (ORDER == 1) ? DIM + 1 : 6;
  static constexpr int NF = DIM + 1;
  static constexpr int NFP = (ORDER == 1) ? DIM : 3;
  struct Tables {
    double mass[NP][NP] = {};             // (1/|K|) int phi_a phi_b
    double stiff[DIM][NP][NP] = {};       // int_ref phi_b d(phi_a)/d(xi_beta)
    double fmass[NF][NP][NP] = {};        // (1/|F_k|) int_{F_k} phi_a phi_b
    int fnode[NF][NFP] = {};              // local nodes on facet k, ascending
  };
  static constexpr Poly basis(int a) {
    if (ORDER == 1) return p_lam(a);
    // P2 triangle
    if (a < 3) {
      Poly r;
      r.n = 2;
      r.t[0] = Term{2.0, {0, 0, 0, 0}};
      r.t[0].e[a] = 2;
      r.t[1] = Term{-1.0, {0, 0, 0, 0}};
      r.t[1].e[a] = 1;
      return r;
    }
    const int ii[3] = {0, 1, 2}, jj[3] = {1, 2, 0};
    Poly r;
    r.n = 1;
    r.t[0] = Term{4.0, {0, 0, 0, 0}};
    r.t[0].e[ii[a - 3]] = 1;
    r.t[0].e[jj[a - 3]] += 1;
    return r;
  }
  // node a lies on facet k (lambda_k = 0 at the node)
  static constexpr bool on_facet(int a, int k) {
    if (a <= DIM) return a != k;  // vertices (and P2 vertices 0..2)
    const int ii[3] = {0, 1, 2}, jj[3] = {1, 2, 0};
    return ii[a - 3] != k && jj[a - 3] != k;
  }
  static constexpr Tables make() {
    Tables T;
    for (int a = 0; a < NP; ++a)
      for (int b = 0; b < NP; ++b) T.mass[a][b] = p_int_norm(p_mul(basis(a), basis(b)), DIM);
    for (int be = 0; be < DIM; ++be)
      for (int a = 0; a < NP; ++a)
        for (int b = 0; b < NP; ++b)
          T.stiff[be][a][b] =
              p_int_norm(p_mul(basis(b), p_dxi(basis(a), be + 1)), DIM) / cfact(DIM);
    for (int k = 0; k < NF; ++k) {
      int p = 0;
      for (int a = 0; a < NP; ++a)
        if (on_facet(a, k)) T.fnode[k][p++] = a;
      for (int a = 0; a < NP; ++a)
        for (int b = 0; b < NP; ++b)
          if (on_facet(a, k) && on_facet(b, k))
            T.fmass[k][a][b] = p_int_facet_norm(p_mul(basis(a), basis(b)), DIM, k);
    }
    return T;
  }
};

template <int DIM, int ORDER>
struct Elem {
  using B = ElemBuild<DIM, ORDER>;
  static constexpr int NP = B::NP, NF = B::NF, NFP = B::NFP;
  static constexpr typename B::Tables T = B::make();
};

// ---------------------------------------------------------------------------
// geometry record per internal cell (doubles):
//   [0] vol = |K|;  [1 + k*DIM + d] = N_k[d], the outward area-weighted
//   normal |e_k| n_k of facet k (facet opposite vertex k).
// Each interior facet's normal is computed once, from the lower-numbered
// cell's vertices, and stored negated in the other cell, so v.N is exactly
// antisymmetric across a facet.  Since N_k = -(1/(d-1)!) (row k-1 of
// |det J| J^{-1}) for k >= 1, the stiffness weights w = |det J| J^{-1} v are
// w_{k-1} = -(d-1)! v.N_k and J^{-1} need not be stored.
// internal cells are numbered in Morton order of their centroids
// ---------------------------------------------------------------------------
// A record is padded to a power of two of doubles, so that it never
// straddles a 128-byte cache line (the sweep gathers it per cell).
template <int DIM>
struct GeoLayout {
  static constexpr int USED = 1 + (DIM + 1) * DIM;  // doubles
  static constexpr int STRIDE = DIM == 2 ? 8 : 16;   // padded record
  static_assert(STRIDE >= USED, "record size");
};

// Factorised Maxwellian tables of a tensor velocity grid with n1 points per
// axis, per cell and padded like the geometry, in two parts: axis 0 as the
// cell's nodes' (E_0, nu) pairs, [n1][n_cells][s0]; then the product of the
// other axes' factors as one table, [n1^(d-1)][n_cells][s1], row r = the
// velocity's row-major index over axes 1..d-1 (s0, s1 = 2 n_p and n_p
// rounded up to a power of 2, doubled for P1 tetrahedra so that the padding
// holds their geometry: TabGeo).  A velocity's Maxwellian is then one
// multiply of two gathered factors in 2D and 3D alike.
struct TabLayout {
  int64_t nc;
  int n1, np, s0, s1, nr;
  __host__ __device__ static constexpr int pow2(int x) {
    int p = 1;
    while (p < x) p *= 2;
    return p;
  }
  __host__ __device__ static constexpr int stride0(int dim, int np) {
    return dim == 3 && np == 4 ? 16 : pow2(2 * np);
  }
  __host__ __device__ static constexpr int stride1(int dim, int np) {
    return dim == 3 && np == 4 ? 8 : pow2(np);
  }
  __host__ __device__ TabLayout(int64_t n_cells, int n1_, int np_, int dim)
      : nc(n_cells), n1(n1_), np(np_), s0(stride0(dim, np_)), s1(stride1(dim, np_)),
        nr(dim == 3 ? n1_ * n1_ : n1_) {}
  // first double of cell c's record on row i of part al (0: axis 0, 1: the rest)
  __host__ __device__ int64_t at(int al, int i, int64_t c) const {
    return al == 0 ? ((int64_t)i * nc + c) * s0
                   : (int64_t)n1 * nc * s0 + ((int64_t)i * nc + c) * s1;
  }
  __host__ __device__ int64_t size() const {
    return (int64_t)n1 * nc * s0 + (int64_t)nr * nc * s1;
  }
};

// P2 triangles and P1 tetrahedra: the padding of a cell's records carries its
// geometry (volume and the area-weighted normals of all facets but the
// last), so the sweep's table gathers bring it with no access of their own;
// the last facet's normal is minus the sum of the others (the normals of a
// closed simplex sum to zero).  Geometry doubles 0 .. E0_N-1 sit in axis
// 0's record from double E0_AT, the next REST_N in the rest's record from
// double REST_AT.  P2 triangles: records of 16 and 8 doubles (12 and 6
// used), (volume, N_0, N_1.x) and N_1.y.  P1 tetrahedra: records of 16 and
// 8 doubles (8 and 4 used), (volume, N_0, N_1, N_2.x) and N_2.yz.
template <int DIM, int NP>
struct TabGeo {
  static constexpr bool ON = (DIM == 2 && NP == 6) || (DIM == 3 && NP == 4);
  static constexpr int E0_AT = DIM == 2 ? 12 : 8, E0_N = DIM == 2 ? 4 : 8;
  static constexpr int REST_AT = DIM == 2 ? 6 : 4, REST_N = DIM == 2 ? 1 : 2;
};

// threads of the table kernels: one per (part, cell, 16-byte chunk of the
// cell's record), each writing its chunk on every row of its part
__host__ __device__ inline int64_t table_threads(int dim, int64_t n_cells, int n1, int np) {
  const TabLayout L(n_cells, n1, np, dim);
  return n_cells * (L.s0 / 2 + L.s1 / 2);
}

// 16-byte chunks of the tables (the unit the table kernels write)
__host__ __device__ inline int64_t table_chunks(int dim, int64_t n_cells, int n1, int np) {
  return TabLayout(n_cells, n1, np, dim).size() / 2;
}

// facet record: x = neighbour internal cell id, or -(1 + boundary facet id);
// y = bits 0..1 neighbour's facet index, bits 4*(p+1).. neighbour local node
// of facet node p (4 bits each)
struct FacetRec {
  int nb;
  int pack;
};

constexpr int REC_LAG_BIT = 1 << 30;
constexpr int REC_SLOT_MASK = REC_LAG_BIT - 1;

}  // namespace bgk

struct tgs_dag {
  int device = 0;
  int dim = 0, order = 0, n_p = 0, n_fp = 0;
  int64_t n_cells = 0, n_vert = 0, n_bfaces = 0, n_nodes = 0;
  int n_v = 0;
  int max_G = 0;
  int64_t n_lagged = 0;
  int sweep_threads = 0;   // 0: chosen per element type and precision
  int ring_slots = 0;      // 0: the element type's full LDS ring
  int sweep_lanes = 64;    // lanes per velocity of the FP64 sweep; 64: workgroup walk
  // host copies
  std::vector<double> v_host, w_host;       // [n_v][dim], [n_v]
  int n_1d = 0;
  std::vector<double> nodes_1d, weights_1d;
  double L = 0.0;
  int dg_cells = 0;                         // Q2 velocity cells per axis, or 0
  std::vector<int32_t> uid_host;            // internal -> user cell
  std::vector<int32_t> iid_host;            // user -> internal cell
  std::vector<double> node_x, bnode_x, vol_user;  // exports (user order)
  // boundary facets in ascending (user cell, local facet) order: cell, the
  // facet's local nodes (4 bits each), outward unit normal [dim]
  std::vector<int32_t> bface_cell, bface_pack;
  std::vector<double> bface_normal;
  std::vector<int32_t> G_host;              // [n_v]
  std::vector<int64_t> gbase_host;          // [n_v]
  // device arrays
  double* d_geo = nullptr;        // [n_cells][GeoLayout::STRIDE]
  int32_t* d_uid = nullptr;       // [n_cells] internal -> user
  bgk::FacetRec* d_facet = nullptr;  // [n_cells][dim+1]
  double* d_v = nullptr;          // [n_v][dim]
  double* d_w = nullptr;          // [n_v]
  double* d_nodes1d = nullptr;    // [n_1d]
  double* d_weights1d = nullptr;  // [n_1d]
  int32_t* d_perm = nullptr;      // [n_v][n_cells] slot -> internal cell
  int32_t* d_pos = nullptr;       // [n_v][n_cells] internal cell -> slot
  int32_t* d_goff = nullptr;      // flat generation offsets
  int64_t* d_gbase = nullptr;     // [n_v] base index of velocity j's offsets
  int32_t* d_G = nullptr;         // [n_v]
  uint8_t* d_lag = nullptr;       // [n_v][n_cells] lagged facet bits (internal), or null
  int32_t* d_vorder = nullptr;    // [n_v] velocity processed by sweep block b
  int32_t* d_vpack = nullptr;     // packed walk: [blocks][64 / sweep_lanes] velocity or -1
  int vpack_blocks = 0;
  // sweep item records, [n_v][n_cells][4] int32 per slot: 2D {K, c_0, c_1, c_2},
  // 3D {c_0, c_1, c_2, c_3} (K from d_perm); facet code c_k: -1 not an inflow
  // facet; >= 0 upwind neighbour's slot (bit 30 set when lagged); <= -2
  // boundary facet -2 - c
  int32_t* d_rec = nullptr;
  // [n_v][n_cells] facet node maps of the slot's cell: for facet k and facet
  // node p, the upwind neighbour's local node sits at bit NB*(k*n_fp + p)
  // with NB = 2 bits (n_p <= 4) or 3 bits (P2)
  int32_t* d_recx = nullptr;
  // per (velocity, generation), aligned with d_goff: the lowest slot any
  // cell of the generation reads a non-lagged upwind value from (INT32_MAX
  // if none); tells the sweep whether older values must come from HBM
  int32_t* d_gmin = nullptr;
};

namespace bgk {
inline size_t f_elems(const tgs_dag* d) { return (size_t)d->n_v * d->n_cells * d->n_p; }
}  // namespace bgk
