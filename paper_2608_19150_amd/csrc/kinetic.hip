// Velocity moments (eq. moments), the Picard stopping ratios
// (eq. convergence-criteria) and the discrete Maxwellian
// (eq. Maxwellian-projection) with the collision frequency.
#include <cmath>
#include <mutex>

#include "device_common.h"
#include "kinetic_args.h"
#include "sweep_args.h"

namespace bgk {

// ----------------------------------------------------------------------------
// moments: U[node][m] = sum_j w_j e_m(v_j) f_j(node)
//
// A block holds CB consecutive internal cells x VL velocity lanes (CB*VL =
// 256, cells fastest so a wavefront reads 64 consecutive entries of pos[j]).
// Lane l sums velocities j = l, l+VL, ... in increasing order; the VL partial
// sums are then added in lane order through LDS, so the result is bitwise
// reproducible.  Optionally the per-block pieces of the convergence norms
// are written for a fixed-order final reduction.
// ----------------------------------------------------------------------------


template <int DIM, int NP, int VL>
struct MomSmem {
  static constexpr int CB = MOM_THREADS / VL, NM = DIM + 2;
  static constexpr int RED = VL > 1 ? (VL - 1) * CB * NP * NM : 1;
  static constexpr int TOTAL = RED + 6 * CB;
};

// Sum over the velocities j0 + lane, j0 + lane + VL, ... below j1, in
// increasing order, of w_j e(v_j) times cell K's nodal values at its slot of
// velocity j.  UNR velocities' gathers (pos, then the NP values at that slot)
// are issued before any is summed, so each lane has UNR independent load
// chains in flight; the summation order is unchanged.
template <int DIM, int NP, int VL>
__device__ __forceinline__ void mom_accumulate(const MomArgs& a, int K, int lane, int j0, int j1,
                                               double (&acc)[NP][DIM + 2]) {
  constexpr int NM = DIM + 2;
  // the weights w_j e_m(v_j) of velocity j applied to one cell's nodal values
  auto accumulate = [&](int j, const double* fv) {
    const double wj = a.w[j];
    double e[NM];
    double v2 = 0.0;
    e[0] = wj;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double vd = a.v[(size_t)j * DIM + d];
      e[1 + d] = wj * vd;
      v2 = fma(vd, vd, v2);
    }
    e[NM - 1] = 0.5 * wj * v2;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int m = 0; m < NM; ++m) acc[p][m] = fma(e[m], fv[p], acc[p][m]);
  };
  constexpr int UNR = 8;
  int j = j0 + lane;
  for (; j + (UNR - 1) * VL < j1; j += UNR * VL) {
    double fv[UNR][NP];
    size_t slot[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      slot[u] = (size_t)a.pos[(size_t)(j + u * VL) * a.n_cells + K];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const double* fp = a.f + ((size_t)(j + u * VL) * a.n_cells + slot[u]) * NP;
#pragma unroll
      for (int p = 0; p < NP; ++p) fv[u][p] = fp[p];
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) accumulate(j + u * VL, fv[u]);
  }
  for (; j < j1; j += VL) {
    const size_t slot = (size_t)a.pos[(size_t)j * a.n_cells + K];
    const double* fp = a.f + ((size_t)j * a.n_cells + slot) * NP;
    double fv[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) fv[p] = fp[p];
    accumulate(j, fv);
  }
}

// The VL lanes' partial sums of cell c added in lane order through LDS
// (s_red: (VL - 1) * CB * NP * (DIM + 2) doubles); lane 0 ends with the sum.
template <int DIM, int NP, int VL, int CB>
__device__ __forceinline__ void mom_lanes(double* s_red, int c, int lane,
                                          double (&acc)[NP][DIM + 2]) {
  constexpr int NM = DIM + 2;
  if (lane > 0) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int m = 0; m < NM; ++m) s_red[(((lane - 1) * CB + c) * NP + p) * NM + m] = acc[p][m];
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll 1
    for (int l = 1; l < VL; ++l)
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int m = 0; m < NM; ++m) acc[p][m] += s_red[(((l - 1) * CB + c) * NP + p) * NM + m];
  }
}

// U of the block's CB cells (written by the threads that hold a cell's sum,
// threadIdx.x < CB) and, with U_prev, the block's piece of the convergence
// norms, reduced over the CB cells by a fixed-order tree (s_norm: 6 * CB
// doubles).
template <int DIM, int NP, int CB>
__device__ __forceinline__ void mom_finish(const MomArgs& a, int blk, int K, bool valid,
                                           bool writer, int c, const double (&acc)[NP][DIM + 2],
                                           double* s_norm) {
  constexpr int NM = DIM + 2;
  const int tid = threadIdx.x;
  if (writer) {
    double nrm[6] = {0, 0, 0, 0, 0, 0};
    if (valid) {
      const size_t u = a.uid ? (size_t)a.uid[K] : (size_t)K;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        double* Up = a.U + (u * NP + p) * NM;
#pragma unroll
        for (int m = 0; m < NM; ++m) Up[m] = acc[p][m];
        if (a.U_prev) {
          const double* Uo = a.U_prev + (u * NP + p) * NM;
#pragma unroll
          for (int m = 0; m < NM; ++m) {
            const int b = m == 0 ? 0 : (m == NM - 1 ? 2 : 1);
            const double dd = acc[p][m] - Uo[m];
            nrm[b] = fma(dd, dd, nrm[b]);
            nrm[3 + b] = fma(Uo[m], Uo[m], nrm[3 + b]);
          }
        }
      }
    }
    if (a.U_prev)
#pragma unroll
      for (int i = 0; i < 6; ++i) s_norm[i * CB + c] = nrm[i];
  }
  if (a.U_prev) {
    __syncthreads();
    // fixed-order tree over the CB cells of the block
    for (int off = CB / 2; off > 0; off >>= 1) {
      if (tid < off)
#pragma unroll
        for (int i = 0; i < 6; ++i) s_norm[i * CB + tid] += s_norm[i * CB + tid + off];
      __syncthreads();
    }
    if (tid < 6) a.partial[(size_t)blk * 6 + tid] = s_norm[tid * CB];
  }
}

// One block of the moment kernel: block `blk` of the instance; `smem` holds
// MomSmem<DIM, NP, VL>::TOTAL doubles of LDS.
template <int DIM, int NP, int VL>
__device__ __forceinline__ void moments_block(const MomArgs& a, int blk, double* smem) {
  constexpr int CB = MOM_THREADS / VL, NM = DIM + 2;
  double* s_red = smem;
  double* s_norm = smem + MomSmem<DIM, NP, VL>::RED;  // [6][CB]
  const int tid = threadIdx.x, c = tid % CB, lane = tid / CB;
  const int K = blk * CB + c;
  const bool valid = K < a.n_cells;
  double acc[NP][NM];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int m = 0; m < NM; ++m) acc[p][m] = 0.0;
  if (valid) mom_accumulate<DIM, NP, VL>(a, K, lane, 0, a.n_v, acc);
  if (VL > 1) mom_lanes<DIM, NP, VL, CB>(s_red, c, lane, acc);
  mom_finish<DIM, NP, CB>(a, blk, K, valid, lane == 0, c, acc, s_norm);
}

// Velocity-split moments for meshes with few cells and many velocities:
// block (b, v) sums the velocities of chunk v (jc of them, a multiple of
// the 4 lanes) for the 64 cells of block b, as moments_block does for all
// velocities, and writes the chunk's sums to split[v][cell]; k_moments_fold
// then adds the chunks in order and finishes as moments_block does.  The
// grid holds vb times the blocks, so such meshes still fill the GPU with
// wavefronts of 64 consecutive cells.
template <int DIM, int NP>
__global__ __launch_bounds__(MOM_THREADS) void k_moments_split(MomArgs a) {
  constexpr int VL = 4, CB = MOM_THREADS / VL, NM = DIM + 2;
  __shared__ double s_red[(VL - 1) * CB * NP * NM];
  if (skip_launch(a.skip)) return;
  const int tid = threadIdx.x, c = tid % CB, lane = tid / CB;
  const int K = blockIdx.x * CB + c;
  const int j0 = blockIdx.y * a.jc, j1 = min(a.n_v, j0 + a.jc);
  double acc[NP][NM];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int m = 0; m < NM; ++m) acc[p][m] = 0.0;
  if (K < a.n_cells) mom_accumulate<DIM, NP, VL>(a, K, lane, j0, j1, acc);
  mom_lanes<DIM, NP, VL, CB>(s_red, c, lane, acc);
  if (lane == 0 && K < a.n_cells) {
    double* P = a.split + ((size_t)blockIdx.y * a.n_cells + K) * NP * NM;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int m = 0; m < NM; ++m) P[p * NM + m] = acc[p][m];
  }
}

template <int DIM, int NP>
__global__ __launch_bounds__(64) void k_moments_fold(MomArgs a) {
  constexpr int CB = 64, NM = DIM + 2;
  __shared__ double s_norm[6 * CB];
  if (skip_launch(a.skip)) return;
  const int c = threadIdx.x, K = blockIdx.x * CB + c;
  const bool valid = K < a.n_cells;
  double acc[NP][NM];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int m = 0; m < NM; ++m) acc[p][m] = 0.0;
  if (valid)
    for (int v = 0; v < a.vb; ++v) {
      const double* P = a.split + ((size_t)v * a.n_cells + K) * NP * NM;
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int m = 0; m < NM; ++m) acc[p][m] += P[p * NM + m];
    }
  mom_finish<DIM, NP, CB>(a, blockIdx.x, K, valid, true, c, acc, s_norm);
}

template <int DIM, int NP, int VL>
__global__ __launch_bounds__(MOM_THREADS) void k_moments(MomArgs a) {
  __shared__ double smem[MomSmem<DIM, NP, VL>::TOTAL];
  if (skip_launch(a.skip)) return;
  moments_block<DIM, NP, VL>(a, blockIdx.x, smem);
}

// Wide blocks for large meshes: 256 consecutive cells x 4 velocity lanes
// (1024 threads), so the four wavefronts of one lane gather one velocity's
// values for 256 cells together and share the lines that neighbouring
// cells' slots fall in.  The lanes' sums are added in lane order through
// one LDS buffer, a lane at a time: the same order as moments_block<..., 4>.
template <int DIM, int NP>
__global__ __launch_bounds__(1024) void k_moments_wide(MomArgs a) {
  constexpr int VL = 4, CB = 256, NM = DIM + 2;
  __shared__ double s_buf[CB * NP * NM];
  __shared__ double s_norm[6 * CB];
  if (skip_launch(a.skip)) return;
  const int tid = threadIdx.x, c = tid % CB, lane = tid / CB;
  const int K = blockIdx.x * CB + c;
  const bool valid = K < a.n_cells;
  double acc[NP][NM];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int m = 0; m < NM; ++m) acc[p][m] = 0.0;
  if (valid) mom_accumulate<DIM, NP, VL>(a, K, lane, 0, a.n_v, acc);
#pragma unroll 1
  for (int l = 1; l < VL; ++l) {
    if (lane == l)
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int m = 0; m < NM; ++m) s_buf[(c * NP + p) * NM + m] = acc[p][m];
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int m = 0; m < NM; ++m) acc[p][m] += s_buf[(c * NP + p) * NM + m];
    __syncthreads();
  }
  mom_finish<DIM, NP, CB>(a, blockIdx.x, K, valid, lane == 0, c, acc, s_norm);
}

__global__ __launch_bounds__(256) void k_ratio(const double* __restrict__ partial, int nblk,
                                               double* out, const int32_t* skip) {
  __shared__ double s[6][256];
  if (skip_launch(skip)) return;
  ratio_block(partial, nblk, out, s);
}

// ----------------------------------------------------------------------------
// Maxwellian coefficients and collision frequency, one thread per node.
// ----------------------------------------------------------------------------


template <int N>
__device__ bool small_solve(double (&A)[N][N], double (&b)[N]) {
  // Gaussian elimination with partial pivoting on a (d+2)x(d+2) system
#pragma unroll
  for (int k = 0; k < N; ++k) {
    int piv = k;
    double best = fabs(A[k][k]);
#pragma unroll
    for (int i = k + 1; i < N; ++i)
      if (fabs(A[i][k]) > best) {
        best = fabs(A[i][k]);
        piv = i;
      }
    if (!(best > 0.0) || !isfinite(best)) return false;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (i == piv && piv != k) {
#pragma unroll
        for (int c = 0; c < N; ++c) {
          const double t = A[k][c];
          A[k][c] = A[i][c];
          A[i][c] = t;
        }
        const double t = b[k];
        b[k] = b[i];
        b[i] = t;
      }
    const double inv = 1.0 / A[k][k];
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const double l = A[i][k] * inv;
#pragma unroll
      for (int c = k; c < N; ++c) A[i][c] = fma(-l, A[k][c], A[i][c]);
      b[i] = fma(-l, b[k], b[i]);
    }
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double s = b[i];
#pragma unroll
    for (int c = i + 1; c < N; ++c) s = fma(-A[i][c], b[c], s);
    b[i] = s / A[i][i];
  }
  return true;
}

// F = sum_j w_j e_j M_j and the Jacobian J[r][c] = dF_r/dx_c for
// M_j = exp(a + b.v_j + c|v_j|^2), x = (a, b, c).
template <int DIM>
__device__ void matched_system(const MaxwArgs& p, const double (&x)[DIM + 2],
                               double (&F)[DIM + 2], double (&J)[DIM + 2][DIM + 2]) {
  constexpr int NM = DIM + 2;
  if (p.x1) {
    // tensor grid: per-axis sums Z[al][k] = sum_i w1_i x_i^k exp(b_al x_i + c x_i^2)
    double Z[DIM][5];
#pragma unroll
    for (int al = 0; al < DIM; ++al)
#pragma unroll
      for (int k = 0; k < 5; ++k) Z[al][k] = 0.0;
    for (int i = 0; i < p.n1; ++i) {
      const double xi = p.x1[i], wi = p.w1[i];
#pragma unroll
      for (int al = 0; al < DIM; ++al) {
        const double g = wi * exp(fma(x[1 + al], xi, x[1 + DIM] * xi * xi));
        double t = g;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          Z[al][k] += t;
          t *= xi;
        }
      }
    }
    const double ea = exp(x[0]);
    // moment of v^(k_al) summed: prod over axes of Z[al][k_al]
    auto P = [&](const int (&k)[DIM]) {
      double r = ea;
#pragma unroll
      for (int al = 0; al < DIM; ++al) r *= Z[al][k[al]];
      return r;
    };
    // F
    {
      int k0[DIM] = {};
      F[0] = P(k0);
#pragma unroll
      for (int be = 0; be < DIM; ++be) {
        int k[DIM] = {};
        k[be] = 1;
        F[1 + be] = P(k);
      }
      double e = 0.0;
#pragma unroll
      for (int be = 0; be < DIM; ++be) {
        int k[DIM] = {};
        k[be] = 2;
        e += P(k);
      }
      F[1 + DIM] = 0.5 * e;
    }
    // second moments m2[b][g] = sum w v_b v_g M, third t3[b] = sum w v_b |v|^2 M,
    // fourth q4 = sum w |v|^4 M
    double m2[DIM][DIM], t3[DIM], q4 = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
#pragma unroll
      for (int g = 0; g < DIM; ++g) {
        int k[DIM] = {};
        k[b] += 1;
        k[g] += 1;
        m2[b][g] = P(k);
      }
      double t = 0.0;
#pragma unroll
      for (int g = 0; g < DIM; ++g) {
        int k[DIM] = {};
        k[b] += 1;
        k[g] += 2;
        t += P(k);
      }
      t3[b] = t;
    }
#pragma unroll
    for (int b = 0; b < DIM; ++b)
#pragma unroll
      for (int g = 0; g < DIM; ++g) {
        int k[DIM] = {};
        k[b] += 2;
        k[g] += 2;
        q4 += P(k);
      }
    // Jacobian rows: mass, momentum, energy; columns: a, b, c
    J[0][0] = F[0];
#pragma unroll
    for (int be = 0; be < DIM; ++be) J[0][1 + be] = F[1 + be];
    J[0][1 + DIM] = 2.0 * F[1 + DIM];
#pragma unroll
    for (int g = 0; g < DIM; ++g) {
      J[1 + g][0] = F[1 + g];
#pragma unroll
      for (int be = 0; be < DIM; ++be) J[1 + g][1 + be] = m2[g][be];
      J[1 + g][1 + DIM] = t3[g];
    }
    J[1 + DIM][0] = F[1 + DIM];
#pragma unroll
    for (int be = 0; be < DIM; ++be) J[1 + DIM][1 + be] = 0.5 * t3[be];
    J[1 + DIM][1 + DIM] = 0.5 * q4;
    return;
  }
  // general velocity set: direct sums
#pragma unroll
  for (int r = 0; r < NM; ++r) {
    F[r] = 0.0;
#pragma unroll
    for (int c = 0; c < NM; ++c) J[r][c] = 0.0;
  }
  for (int j = 0; j < p.n_v; ++j) {
    double vv[DIM], v2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      vv[d] = p.v[(size_t)j * DIM + d];
      v2 = fma(vv[d], vv[d], v2);
    }
    double ex = x[0];
#pragma unroll
    for (int d = 0; d < DIM; ++d) ex = fma(x[1 + d], vv[d], ex);
    ex = fma(x[1 + DIM], v2, ex);
    const double wm = p.w[j] * exp(ex);
    double e[NM], pp[NM];
    e[0] = 1.0;
    pp[0] = 1.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) e[1 + d] = pp[1 + d] = vv[d];
    e[1 + DIM] = 0.5 * v2;
    pp[1 + DIM] = v2;
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      F[r] = fma(wm, e[r], F[r]);
#pragma unroll
      for (int c = 0; c < NM; ++c) J[r][c] = fma(wm * e[r], pp[c], J[r][c]);
    }
  }
}

// Projection onto the Q2 velocity space (App. B).  The Lagrange basis sits
// at the Gauss-Legendre nodes, so each cell's mass matrix is the diagonal of
// the quadrature weights and node k of cell c takes the value
//   (1/w_k) * integral over I_c of g(x) l_k(x) dx,   g = exp(-(x-u)^2/(2 theta)),
// where I_c is the cell except that the first cell extends to -infinity and
// the last to +infinity (the extension E of the projection's definition).
// With the cell's reference coordinate y (x = centre + (h/2) y) and the
// basis in monomials of y (reference nodes -s, 0, s with s^2 = 3/5, weights
// (h/2)(5/9, 8/9, 5/9)): l_0 = (y^2 - s y)/(2 s^2), l_1 = 1 - y^2/s^2,
// l_2 = (y^2 + s y)/(2 s^2), so the three values follow from the cell
// integrals m_k = integral of g y^k dx, k = 0, 1, 2.  Two evaluations of
// m_k, both exact up to rounding:
// * closed form: x = u + sigma t (sigma^2 = theta), y = alpha + beta t, and
//   G_m = integral of t^m exp(-t^2/2) over [t_a, t_b] from erfc:
//   G_0 = sqrt(pi/2) (A - B | B - A | 2 - A - B) with A = erfc(|t_a|/sqrt2),
//   B = erfc(|t_b|/sqrt2) as both limits are >= 0, <= 0 or straddle 0;
//   G_1 = e_a - e_b, G_2 = G_0 + t_a e_a - t_b e_b, e = exp(-t^2/2);
// * quadrature: t = t_c + r (t_c the cell centre, r in [-d, d] with
//   d = (h/2)/sigma): m_k = sigma beta^k exp(-t_c^2/2) K_k with
//   K_k = integral over [-d, d] of r^k exp(-t_c r - r^2/2) dr by 20-point
//   Gauss-Legendre, whose error for d <= 1 and |t_c| d <= 3 (an entire
//   integrand) is far below rounding.
// The closed form's expansion of (alpha + beta t)^2 cancels about
// 12 alpha^2 ulp when the cell lies many half-widths from u on a fine grid;
// the quadrature is used wherever it is exact (interior cells with d <= 1
// and |t_c| d <= 3), the closed form elsewhere (the extended end cells,
// cells wide against sigma).
__device__ __forceinline__ void proj_cell(double u, double sig, int c, int nc1, double L,
                                          double (&out)[3]) {
  constexpr double RT2 = 0.70710678118654752440;   // 1/sqrt(2)
  constexpr double SPI2 = 1.2533141373155002512;   // sqrt(pi/2)
  constexpr double S = 0.77459666924148337704;     // sqrt(3/5)
  // the 10 positive nodes of 20-point Gauss-Legendre on [-1, 1] and weights
  constexpr double GL[10][2] = {
      {7.65265211334973383e-02, 1.52753387130725782e-01},
      {2.27785851141645096e-01, 1.49172986472603658e-01},
      {3.73706088715419549e-01, 1.42096109318381875e-01},
      {5.10867001950827126e-01, 1.31688638449176526e-01},
      {6.36053680726515025e-01, 1.18194531961518245e-01},
      {7.46331906460150796e-01, 1.01930119817240261e-01},
      {8.39116971822218782e-01, 8.32767415767046715e-02},
      {9.12234428251325835e-01, 6.26720483341094425e-02},
      {9.63971927277913809e-01, 4.06014298003862170e-02},
      {9.93128599185094885e-01, 1.76140071391532732e-02}};
  const double hh = L / nc1;                       // half the cell width
  const double lo = -L + 2.0 * hh * c;
  const bool a_inf = c == 0, b_inf = c == nc1 - 1;
  const double be = sig / hh, d = hh / sig;
  const double tc = (lo + hh - u) / sig;
  double m0, m1, m2;
  if (!a_inf && !b_inf && d <= 1.0 && fabs(tc) * d <= 3.0) {
    double k0 = 0.0, k1 = 0.0, k2 = 0.0;
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      const double r = d * GL[q][0], w = d * GL[q][1];
      const double ep = w * bgk_exp(-tc * r - 0.5 * r * r);    // at +r
      const double em = w * bgk_exp(tc * r - 0.5 * r * r);     // at -r
      k0 += ep + em;
      k1 = fma(r, ep - em, k1);
      k2 = fma(r * r, ep + em, k2);
    }
    const double sc = sig * bgk_exp(-0.5 * tc * tc);
    m0 = sc * k0;
    m1 = sc * be * k1;
    m2 = sc * be * be * k2;
  } else {
    const double ta = (lo - u) / sig, tb = (lo + 2.0 * hh - u) / sig;
    const double A = a_inf ? 0.0 : erfc(fabs(ta) * RT2);
    const double B = b_inf ? 0.0 : erfc(fabs(tb) * RT2);
    const double g0 =
        SPI2 * (!a_inf && ta >= 0.0 ? A - B : (!b_inf && tb <= 0.0 ? B - A : 2.0 - A - B));
    const double ea = a_inf ? 0.0 : bgk_exp(-0.5 * ta * ta);
    const double eb = b_inf ? 0.0 : bgk_exp(-0.5 * tb * tb);
    const double g1 = ea - eb;
    const double g2 = g0 + (a_inf ? 0.0 : ta * ea) - (b_inf ? 0.0 : tb * eb);
    const double al = (u - (lo + hh)) / hh;
    m0 = sig * g0;
    m1 = sig * fma(al, g0, be * g1);
    m2 = sig * fma(al * al, g0, fma(2.0 * al * be, g1, be * be * g2));
  }
  out[0] = (m2 - S * m1) * (5.0 / 6.0) / (hh * (5.0 / 9.0));
  out[1] = (m0 - m2 * (5.0 / 3.0)) / (hh * (8.0 / 9.0));
  out[2] = (m2 + S * m1) * (5.0 / 6.0) / (hh * (5.0 / 9.0));
}

// value at 1-D node i = 3 c + k
__device__ __forceinline__ double proj_node(double u, double sig, int i, int nc1, double L) {
  const int c = i / 3, k = i - 3 * c;
  double p[3];
  proj_cell(u, sig, c, nc1, L, p);
  return k == 0 ? p[0] : (k == 1 ? p[1] : p[2]);
}

// What one node contributes to the kernel-wide status words; the caller
// adds a wavefront's contributions with one atomic each (flush_status).
struct NodeStatus {
  unsigned long long nubits = 0ull;  // bit pattern of nu (>= 0) of a physical node, else 0
  bool fallback = false;             // MATCHED solve failed or held on DIRECT
  bool nonphysical = false;
};

// One atomic per wavefront and status word: the wave's maximum nu bit
// pattern, its fallback and non-physical counts.  Every lane of the wave
// must call it (no lane may have left the kernel) and the targets must be
// the same for the whole wave.
__device__ __forceinline__ void flush_status(const NodeStatus& st, int32_t* status,
                                             unsigned long long* numax) {
  unsigned long long m = st.nubits;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(m, off);
    m = o > m ? o : m;
  }
  const unsigned long long fb = __ballot(st.fallback), np = __ballot(st.nonphysical);
  if (__lane_id() == 0) {
    if (numax && m) atomicMax(numax, m);
    if (status && fb) atomicAdd(&status[0], (int)__popcll(fb));
    if (status && np) atomicAdd(&status[1], (int)__popcll(np));
  }
}

template <int DIM>
__device__ __forceinline__ void maxwellian_node(const MaxwArgs& p, const double* __restrict__ Uin,
                                                int64_t i, NodeStatus& st) {
  constexpr int NM = DIM + 2;
  double U[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) U[m] = Uin[i * NM + m];
  const double n = U[0];
  double u[DIM], uu = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    u[d] = U[1 + d] / n;
    uu = fma(u[d], u[d], uu);
  }
  const double th = (2.0 * U[1 + DIM] / n - uu) / DIM;
  // theta enters unless the Maxwellian is the linear n/|V| with constant nu
  const bool needs_theta = !(p.mode == BGK_MAXW_LINEAR && p.nu_kind == BGK_NU_CONST);
  const bool physical = n > 0.0 && isfinite(n) && (!needs_theta || (th > 0.0 && isfinite(th)));
  // without collisions (constant nu = 0) no Maxwellian is needed: M = 0
  const bool collisional = !(p.nu_kind == BGK_NU_CONST && p.nu_const == 0.0);
  if (!collisional) {
    if (p.nu) p.nu[i] = 0.0;
    // PROJECTED keeps (n, u, theta): n = 0 makes its tables vanish
#pragma unroll
    for (int m = 0; m < NM; ++m)
      p.coef[i * NM + m] = p.mode == BGK_MAXW_PROJECTED ? (m == NM - 1 ? 1.0 : 0.0)
                                                         : (m == 0 ? -INFINITY : 0.0);
    if (p.M_dense)
      for (int j = 0; j < p.n_v; ++j) p.M_dense[i * p.n_v + j] = 0.0;
    return;
  }
  st.nonphysical = !physical;
  double nu = p.nu_kind == BGK_NU_CONST ? p.nu_const : n / sqrt(th) / p.kn;
  if (p.nu) p.nu[i] = nu;
  if (physical) st.nubits = (unsigned long long)__double_as_longlong(nu);
  if (p.mode == BGK_MAXW_PROJECTED) {
    // coefficients are the primitive variables (the values, if asked for,
    // come from k_proj_dense)
    p.coef[i * NM] = n;
#pragma unroll
    for (int d = 0; d < DIM; ++d) p.coef[i * NM + 1 + d] = u[d];
    p.coef[i * NM + 1 + DIM] = th;
    return;
  }
  double x[NM];
  if (p.mode == BGK_MAXW_LINEAR) {
    double vol = 1.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) vol *= 2.0 * p.L;
    x[0] = log(n / vol);
#pragma unroll
    for (int d = 0; d < DIM; ++d) x[1 + d] = 0.0;
    x[1 + DIM] = 0.0;
  } else {
    // DIRECT coefficients
    x[0] = log(n) - 0.5 * DIM * log(2.0 * M_PI * th) - 0.5 * uu / th;
#pragma unroll
    for (int d = 0; d < DIM; ++d) x[1 + d] = u[d] / th;
    x[1 + DIM] = -0.5 / th;
    if (p.mode == BGK_MAXW_MATCHED && physical && p.sticky && p.sticky[i]) {
      st.fallback = true;
    } else if (p.mode == BGK_MAXW_MATCHED && physical) {
      double Unorm = 0.0;
#pragma unroll
      for (int m = 0; m < NM; ++m) Unorm = fma(U[m], U[m], Unorm);
      Unorm = sqrt(Unorm);
      double y[NM];
#pragma unroll
      for (int m = 0; m < NM; ++m) y[m] = x[m];
      bool ok = false;
      for (int it = 0; it <= 30; ++it) {
        double F[NM], J[NM][NM];
        matched_system<DIM>(p, y, F, J);
        double rn = 0.0;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
          F[m] -= U[m];
          rn = fma(F[m], F[m], rn);
        }
        if (sqrt(rn) <= 1e-14 * Unorm) {
          ok = true;
          break;
        }
        if (!small_solve<NM>(J, F)) break;
        bool fin = true;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
          y[m] -= F[m];
          fin = fin && isfinite(y[m]);
        }
        if (!fin) break;
      }
      if (ok && y[1 + DIM] < 0.0) {
#pragma unroll
        for (int m = 0; m < NM; ++m) x[m] = y[m];
      } else {
        st.fallback = true;
        if (p.sticky) p.sticky[i] = 1;
      }
    }
  }
#pragma unroll
  for (int m = 0; m < NM; ++m) p.coef[i * NM + m] = x[m];
  if (p.M_dense) {
    for (int j = 0; j < p.n_v; ++j) {
      double vv[DIM], v2 = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        vv[d] = p.v[(size_t)j * DIM + d];
        v2 = fma(vv[d], vv[d], v2);
      }
      p.M_dense[i * p.n_v + j] = maxw_eval<DIM>(x, vv, v2);
    }
  }
}

// Projected Maxwellian values at every (node, velocity) from the primitive
// coefficients: n (2 pi theta)^(-d/2) times the product of the per-axis
// projections at the velocity's tensor indices (first axis slowest)
template <int DIM>
__global__ __launch_bounds__(256) void k_proj_dense(const double* __restrict__ prim,
                                                    double* __restrict__ M, int64_t n_nodes,
                                                    int n_v, int n1, int nc1, double L) {
  constexpr int NM = DIM + 2;
  const int64_t total = n_nodes * n_v;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = t / n_v;
    const int j = (int)(t - node * n_v);
    const double* P = prim + node * NM;
    const double th = P[1 + DIM], sig = sqrt(th);
    double val = P[0] / (DIM == 2 ? 2.0 * M_PI * th : 2.0 * M_PI * th * sqrt(2.0 * M_PI * th));
    int rem = j;
    for (int d = DIM - 1; d >= 0; --d) {
      const int ia = rem % n1;
      rem /= n1;
      val *= proj_node(P[1 + d], sig, ia, nc1, L);
    }
    M[t] = val;
  }
}

template <int DIM>
__global__ __launch_bounds__(128) void k_maxwellian(MaxwArgs p) {
  if (skip_launch(p.skip)) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  NodeStatus st;
  if (i < p.n_nodes) maxwellian_node<DIM>(p, p.U, i, st);
  flush_status(st, p.status, p.numax);
}

template <int DIM>
__global__ void k_coef_from_prim(const double* __restrict__ prim, double* __restrict__ coef,
                                 int64_t n) {
  constexpr int NM = DIM + 2;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double nn = prim[i * NM], th = prim[i * NM + 1 + DIM];
  double uu = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) uu = fma(prim[i * NM + 1 + d], prim[i * NM + 1 + d], uu);
  coef[i * NM] = log(nn) - 0.5 * DIM * log(2.0 * M_PI * th) - 0.5 * uu / th;
#pragma unroll
  for (int d = 0; d < DIM; ++d) coef[i * NM + 1 + d] = prim[i * NM + 1 + d] / th;
  coef[i * NM + 1 + DIM] = -0.5 / th;
}

// Factorised Maxwellian for tensor velocity grids: exp(a + b.v + c|v|^2) =
// E_0 E_rest with E_0 = exp(a + b_0 x_0 + c x_0^2) on axis 0 and E_rest =
// exp(sum over the other axes of b_al x_al + c x_al^2), both per node.  The
// padded per-cell records (TabLayout) are written as 16-byte chunks, pad
// included, consecutive chunks by consecutive threads: a chunk of axis 0 is
// node b of a record as (E_0, nu) (the sweep gathers both with one access),
// a chunk of the rest holds two nodes' entries.  Chunks are numbered
// through axis 0's records first, then through the rest's.
// Padding chunk h of cell c's record (axis 0 if first): zeros, or for P2
// triangles and P1 tetrahedra the cell's geometry (TabGeo)
template <int DIM>
__device__ __forceinline__ double2 pad_chunk(const double* __restrict__ geo, int np, bool first,
                                             int h, int64_t c) {
  if (DIM == 2 && np == 6) {
    const double* g = geo + c * GeoLayout<2>::STRIDE;
    if (first) return h == 6 ? make_double2(g[0], g[1]) : make_double2(g[2], g[3]);
    return make_double2(g[4], 0.0);
  }
  if (DIM == 3 && np == 4) {
    const double* g = geo + c * GeoLayout<3>::STRIDE;
    if (first) return make_double2(g[2 * (h - 4)], g[2 * (h - 4) + 1]);  // chunks 4..7
    return h == 2 ? make_double2(g[8], g[9]) : make_double2(0.0, 0.0);
  }
  return make_double2(0.0, 0.0);
}

// entry chunk h of cell c's record on row `row` of part `first` (axis 0) or
// the rest
template <int DIM>
__device__ __forceinline__ double2 table_value(const double* __restrict__ coef,
                                               const double* __restrict__ nu,
                                               const double* __restrict__ x1,
                                               const double* __restrict__ geo, int n1, int np,
                                               bool first, int64_t c, int h, int row) {
  constexpr int NM = DIM + 2;
  const auto entry = [&](int b) {
    const double* cf = coef + (c * np + b) * NM;
    double e;
    if (first) {
      const double x = x1[row];
      e = __fma_rn(cf[1 + DIM], x * x, cf[1] * x) + cf[0];
    } else if (DIM == 2) {
      const double x = x1[row];
      e = __fma_rn(cf[1 + DIM], x * x, cf[2] * x);
    } else {
      const double y = x1[row / n1], z = x1[row % n1];
      e = __fma_rn(cf[1 + DIM], y * y, cf[2] * y) + __fma_rn(cf[1 + DIM], z * z, cf[3] * z);
    }
    return bgk_exp(e);
  };
  if (first)
    return h < np ? make_double2(entry(h), nu[c * np + h]) : pad_chunk<DIM>(geo, np, true, h, c);
  if (2 * h >= np) return pad_chunk<DIM>(geo, np, false, h, c);
  return make_double2(entry(2 * h), 2 * h + 1 < np ? entry(2 * h + 1) : 0.0);
}

// Thread t of the table kernels (table_threads): part, cell and chunk, the
// chunk written on every row of the part, so each node's coefficients are
// read once rather than once per row; for every row, consecutive threads
// write consecutive chunks.
template <int DIM>
__device__ __forceinline__ void table_rows(const double* __restrict__ coef,
                                           const double* __restrict__ nu,
                                           const double* __restrict__ x1,
                                           const double* __restrict__ geo,
                                           double* __restrict__ tab, int64_t n_cells, int n1,
                                           int np, int64_t t) {
  const TabLayout L(n_cells, n1, np, DIM);
  const int h0 = L.s0 / 2, h1 = L.s1 / 2;
  const int64_t n0 = n_cells * h0;
  const bool first = t < n0;
  const int64_t u = first ? t : t - n0;
  const int half = first ? h0 : h1;
  const int64_t c = u / half;
  const int h = (int)(u - c * half);
  const int rows = first ? n1 : L.nr;
  for (int row = 0; row < rows; ++row)
    reinterpret_cast<double2*>(tab + L.at(first ? 0 : 1, row, c))[h] =
        table_value<DIM>(coef, nu, x1, geo, n1, np, first, c, h, row);
}

template <int DIM>
__global__ void k_maxw_tables(const double* __restrict__ coef, const double* __restrict__ nu,
                              const double* __restrict__ x1, const double* __restrict__ geo,
                              double* __restrict__ tab, int64_t n_cells, int n1, int np,
                              const int32_t* skip) {
  if (skip_launch(skip)) return;
  const int64_t total = table_threads(DIM, n_cells, n1, np);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x)
    table_rows<DIM>(coef, nu, x1, geo, tab, n_cells, n1, np, t);
}

int launch_maxw_tables(const tgs_dag* d, const double* coef, const double* nu, double* tab,
                       hipStream_t stream, const int32_t* skip) {
  const int np = (int)(d->n_nodes / d->n_cells);
  const int64_t total = table_threads(d->dim, d->n_cells, d->n_1d, np);
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  if (d->dim == 2)
    hipLaunchKernelGGL(k_maxw_tables<2>, dim3(grid), dim3(256), 0, stream, coef, nu, d->d_nodes1d,
                       d->d_geo, tab, d->n_cells, d->n_1d, np, skip);
  else
    hipLaunchKernelGGL(k_maxw_tables<3>, dim3(grid), dim3(256), 0, stream, coef, nu, d->d_nodes1d,
                       d->d_geo, tab, d->n_cells, d->n_1d, np, skip);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

// Projected-Maxwellian tables.  Pass 1: the per-axis projections of every
// node, pr[(a n1 + i) n_nodes + node] (axis 0 carrying n (2 pi theta)^(-d/2)),
// one thread per (node, axis, velocity cell) writing the cell's 3 values,
// consecutive nodes on consecutive threads.  Pass 2: the tables of the
// factorised layout from them, as 16-byte chunks like the exponential
// tables: axis 0's entry of 1-D node i0 paired with nu, the rest's entry
// pr_1[i1] (2D) or pr_1[i1] pr_2[i2] (3D, row i1 n1 + i2).
template <int DIM>
__global__ __launch_bounds__(256) void k_proj_axes(const double* __restrict__ prim,
                                                   double* __restrict__ pr, int64_t n_nodes,
                                                   int n1, int nc1, double L,
                                                   const int32_t* skip) {
  constexpr int NM = DIM + 2;
  if (skip_launch(skip)) return;
  const int64_t total = (int64_t)DIM * nc1 * n_nodes;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = t % n_nodes;
    const int ac = (int)(t / n_nodes);
    const int a = ac / nc1, c = ac - a * nc1;
    const double* P = prim + node * NM;
    const double th = P[1 + DIM];
    double p[3];
    proj_cell(P[1 + a], sqrt(th), c, nc1, L, p);
    const double f =
        a == 0 ? P[0] / (DIM == 2 ? 2.0 * M_PI * th : 2.0 * M_PI * th * sqrt(2.0 * M_PI * th))
               : 1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) pr[((int64_t)a * n1 + 3 * c + k) * n_nodes + node] = p[k] * f;
  }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_proj_tables(const double* __restrict__ pr,
                                                     const double* __restrict__ nu,
                                                     const double* __restrict__ geo,
                                                     double* __restrict__ tab, int64_t n_cells,
                                                     int n1, int np, const int32_t* skip) {
  if (skip_launch(skip)) return;
  const TabLayout L(n_cells, n1, np, DIM);
  const int64_t nn = n_cells * np;
  const int64_t a0 = (int64_t)n1 * n_cells * (L.s0 / 2);
  const int64_t total = table_chunks(DIM, n_cells, n1, np);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const bool first = t < a0;
    const int64_t u = first ? t : t - a0;
    const int half = (first ? L.s0 : L.s1) / 2;
    const int64_t q = u / half;
    const int h = (int)(u - q * half);
    const int64_t c = q % n_cells;
    const int row = (int)(q / n_cells);
    const auto rest = [&](int b) {
      const int64_t node = c * np + b;
      if (DIM == 2) return pr[((int64_t)n1 + row) * nn + node];
      return pr[((int64_t)n1 + row / n1) * nn + node] *
             pr[((int64_t)2 * n1 + row % n1) * nn + node];
    };
    double2 v;
    if (first)
      v = h < np ? make_double2(pr[(int64_t)row * nn + c * np + h], nu[c * np + h])
                 : pad_chunk<DIM>(geo, np, true, h, c);
    else if (2 * h >= np)
      v = pad_chunk<DIM>(geo, np, false, h, c);
    else
      v = make_double2(rest(2 * h), 2 * h + 1 < np ? rest(2 * h + 1) : 0.0);
    reinterpret_cast<double2*>(tab + L.at(first ? 0 : 1, row, c))[h] = v;
  }
}

int launch_proj_tables(const tgs_dag* d, const double* prim, const double* nu, double* pr,
                       double* tab, hipStream_t stream, const int32_t* skip) {
  BGK_CHECK(d->dg_cells > 0, BGK_E_INVALID, "projected tables need a Q2 velocity space");
  const int np = (int)(d->n_nodes / d->n_cells);
  const int64_t n_pr = (int64_t)d->dim * d->dg_cells * d->n_nodes;
  const int64_t total = table_chunks(d->dim, d->n_cells, d->n_1d, np);
  const int g1 = (int)std::min<int64_t>((n_pr + 255) / 256, 65536);
  const int g2 = (int)std::min<int64_t>((total + 255) / 256, 65536);
  if (d->dim == 2) {
    hipLaunchKernelGGL(k_proj_axes<2>, dim3(g1), dim3(256), 0, stream, prim, pr, d->n_nodes,
                       d->n_1d, d->dg_cells, d->L, skip);
    hipLaunchKernelGGL(k_proj_tables<2>, dim3(g2), dim3(256), 0, stream, pr, nu, d->d_geo, tab,
                       d->n_cells, d->n_1d, np, skip);
  } else {
    hipLaunchKernelGGL(k_proj_axes<3>, dim3(g1), dim3(256), 0, stream, prim, pr, d->n_nodes,
                       d->n_1d, d->dg_cells, d->L, skip);
    hipLaunchKernelGGL(k_proj_tables<3>, dim3(g2), dim3(256), 0, stream, pr, nu, d->d_geo, tab,
                       d->n_cells, d->n_1d, np, skip);
  }
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

// nodal rows between user order and internal order: to_internal:
// dst[K] = src[uid[K]], else dst[uid[K]] = src[K]; rows of `width` doubles
__global__ void k_nodal_perm(const double* __restrict__ src, double* __restrict__ dst,
                             const int32_t* __restrict__ uid, int64_t n_cells, int row,
                             int to_internal) {
  const int64_t total = n_cells * row;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t K = i / row, r = i % row;
    const int64_t u = uid[K];
    if (to_internal)
      dst[K * row + r] = src[u * row + r];
    else
      dst[u * row + r] = src[K * row + r];
  }
}

int launch_nodal_perm(const tgs_dag* d, const double* src, double* dst, int to_internal,
                      hipStream_t stream) {
  return launch_nodal_rows(d, src, dst, d->n_p * (d->dim + 2), to_internal, stream);
}

int launch_nodal_rows(const tgs_dag* d, const double* src, double* dst, int row, int to_internal,
                      hipStream_t stream) {
  const int64_t total = d->n_cells * row;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_nodal_perm, dim3(grid), dim3(256), 0, stream, src, dst, d->d_uid,
                     d->n_cells, row, to_internal);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

// Velocity lanes per cell for the moment kernel.  Fewer lanes put more
// consecutive cells of one velocity in a wavefront (their slots cluster, so
// the gathers coalesce better); more lanes give more threads, which the
// kernel needs to keep enough gathers in flight.  Measured: 3072 P1
// triangles x 36,864 velocities 1.7 ms at 64 lanes against 2.4 at 16;
// 10,523 tetrahedra x 110,592 velocities 19.6 ms at 4 against 24.1 at 16;
// 54,651 tetrahedra x 4096 velocities 3.00 ms at 4 against 3.22 at 1 and
// 3.90 at 16; 199,712 P2 triangles x 1024 velocities 3.43 ms at 4 against
// 3.68 at 1 and 4.20 at 16
int moment_vl(const tgs_dag* d) {
  const int64_t nc = d->n_cells;
  if (nc >= 16384) return 4;
  if (nc >= 4096) return d->n_v >= 65536 ? 4 : 16;
  return d->n_v < 2048 ? 16 : 64;
}

int moment_blocks(const tgs_dag* d) {
  const int vl = moment_vl(d);
  const int cb = MOM_THREADS / vl;
  return (int)((d->n_cells + cb - 1) / cb);
}

// Velocity chunks of the split moment reduction (1: none).  Meshes of 4096
// to 16,383 cells with 8192 velocities or more get enough chunks for about
// 4096 wavefronts of 64 cells (at least 256 velocities a chunk, at most 64
// chunks, at most MOM_SPLIT_DOUBLES of chunk sums).  Measured: 10,523
// tetrahedra x 110,592 velocities 17.6 ms in 7 chunks against 19.7 unsplit;
// 3072 P1 triangles x 36,864 velocities 1.84 ms in 22 chunks against 1.75
// unsplit at 64 lanes per cell, so smaller meshes stay unsplit.
int moment_split(const tgs_dag* d) {
  const int64_t nc = d->n_cells;
  if (nc < 4096 || nc >= 16384 || d->n_v < 8192) return 1;
  const int64_t blocks = (nc + 63) / 64;
  int64_t vb = (4096 + blocks * 4 - 1) / (blocks * 4);
  vb = std::min<int64_t>(vb, d->n_v / 256);
  vb = std::min<int64_t>(vb, 64);
  vb = std::min<int64_t>(vb, MOM_SPLIT_DOUBLES / (d->n_nodes * (d->dim + 2)));
  return vb < 2 ? 1 : (int)vb;
}

// velocities per chunk (a multiple of the 4 lanes) and the chunk count
static void split_chunks(const tgs_dag* d, int vb, int* jc, int* nchunks) {
  int c = (d->n_v + vb - 1) / vb;
  c = (c + 3) / 4 * 4;
  *jc = c;
  *nchunks = (d->n_v + c - 1) / c;
}

int64_t moment_split_doubles(const tgs_dag* d) {
  const int vb = moment_split(d);
  if (vb < 2) return 0;
  int jc, nch;
  split_chunks(d, vb, &jc, &nch);
  return (int64_t)nch * d->n_nodes * (d->dim + 2);
}

// Wide moment blocks (256 cells) for tetrahedral meshes of 16,384 cells or
// more.  Measured: 54,651 tetrahedra x 4096 velocities 2.28 ms against
// 2.90 in 64-cell blocks (32-byte slots, four to a line, shared by more
// neighbours); 199,712 P2 triangles x 1024 velocities 3.87 against 3.42,
// so triangles keep the 64-cell blocks.
bool moment_wide(const tgs_dag* d) { return d->dim == 3 && d->n_cells >= 16384; }

int moment_partials(const tgs_dag* d) {
  if (moment_split(d) > 1) return (int)((d->n_cells + 63) / 64);
  if (moment_wide(d)) return (int)((d->n_cells + 255) / 256);
  return moment_blocks(d);
}

int launch_moments(const tgs_dag* d, const double* f, double* U, const double* U_prev,
                   double* partial, double* ratio_out, hipStream_t stream, bool user_order,
                   double* split, const int32_t* skip) {
  MomArgs a{f,      d->d_pos, user_order ? d->d_uid : nullptr, d->d_v, d->d_w, U, U_prev, partial,
            (int)d->n_cells, d->n_v, skip};
  const int vb = moment_split(d);
  const int nblk = moment_partials(d);
  if (vb > 1) {
    BGK_CHECK(split != nullptr, BGK_E_INVALID, "split moment reduction without its scratch");
    int jc, nch;
    split_chunks(d, vb, &jc, &nch);
    a.split = split;
    a.jc = jc;
    a.vb = nch;
    const dim3 grid((unsigned)nblk, (unsigned)nch), block(MOM_THREADS);
#define BGK_MOMS(D_, P_)                                                                    \
  do {                                                                                      \
    hipLaunchKernelGGL((k_moments_split<D_, P_>), grid, block, 0, stream, a);             \
    hipLaunchKernelGGL((k_moments_fold<D_, P_>), dim3((unsigned)nblk), dim3(64), 0, stream, a); \
  } while (0)
    if (d->dim == 2 && d->order == 1)
      BGK_MOMS(2, 3);
    else if (d->dim == 2)
      BGK_MOMS(2, 6);
    else
      BGK_MOMS(3, 4);
#undef BGK_MOMS
  } else if (moment_wide(d)) {
    hipLaunchKernelGGL((k_moments_wide<3, 4>), dim3((unsigned)nblk), dim3(1024), 0, stream, a);
  } else {
    const int vl = moment_vl(d);
    const dim3 grid((unsigned)nblk), block(MOM_THREADS);
#define BGK_MOM(D_, P_)                                                                         \
  do {                                                                                          \
    if (vl == 1) hipLaunchKernelGGL((k_moments<D_, P_, 1>), grid, block, 0, stream, a);   \
    else if (vl == 4) hipLaunchKernelGGL((k_moments<D_, P_, 4>), grid, block, 0, stream, a); \
    else if (vl == 16) hipLaunchKernelGGL((k_moments<D_, P_, 16>), grid, block, 0, stream, a); \
    else hipLaunchKernelGGL((k_moments<D_, P_, 64>), grid, block, 0, stream, a);          \
  } while (0)
    if (d->dim == 2 && d->order == 1)
      BGK_MOM(2, 3);
    else if (d->dim == 2)
      BGK_MOM(2, 6);
    else
      BGK_MOM(3, 4);
#undef BGK_MOM
  }
  BGK_HIP(hipGetLastError());
  if (U_prev && ratio_out) {
    hipLaunchKernelGGL(k_ratio, dim3(1), dim3(256), 0, stream, partial, nblk, ratio_out, skip);
    BGK_HIP(hipGetLastError());
  }
  return BGK_OK;
}

int launch_maxwellian(const tgs_dag* d, int mode, const double* U, const tgs_nu_model* nm,
                      double* coef, double* nu, double* M_dense, int32_t* status,
                      unsigned long long* numax, uint8_t* sticky, hipStream_t stream,
                      const int32_t* skip) {
  BGK_CHECK(mode == BGK_MAXW_DIRECT || mode == BGK_MAXW_MATCHED || mode == BGK_MAXW_LINEAR ||
                mode == BGK_MAXW_PROJECTED,
            BGK_E_INVALID, "unknown Maxwellian mode");
  BGK_CHECK(mode != BGK_MAXW_PROJECTED || d->dg_cells > 0, BGK_E_INVALID,
            "PROJECTED mode needs a Q2 velocity space (dg_cells > 0)");
  BGK_CHECK(nm && (nm->kind == BGK_NU_CONST || (nm->kind == BGK_NU_KN && nm->kn > 0)),
            BGK_E_INVALID, "bad collision-frequency model");
  BGK_CHECK(mode != BGK_MAXW_LINEAR || d->L > 0, BGK_E_INVALID,
            "LINEAR mode needs the velocity box half-width L");
  MaxwArgs p{U,      coef,     nu,          M_dense,       status, numax,
             d->d_v, d->d_w,   d->d_nodes1d, d->d_weights1d, d->n_1d, d->n_v,
             d->n_nodes, mode, nm->kind,    nm->nu_const,  nm->kn, d->L, d->dg_cells, sticky,
             skip};
  const dim3 grid((unsigned)((d->n_nodes + 127) / 128)), block(128);
  if (d->dim == 2)
    hipLaunchKernelGGL(k_maxwellian<2>, grid, block, 0, stream, p);
  else
    hipLaunchKernelGGL(k_maxwellian<3>, grid, block, 0, stream, p);
  BGK_HIP(hipGetLastError());
  if (mode == BGK_MAXW_PROJECTED && M_dense) {
    const int64_t total = d->n_nodes * d->n_v;
    const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
    if (d->dim == 2)
      hipLaunchKernelGGL(k_proj_dense<2>, dim3(g), dim3(256), 0, stream, coef, M_dense,
                         d->n_nodes, d->n_v, d->n_1d, d->dg_cells, d->L);
    else
      hipLaunchKernelGGL(k_proj_dense<3>, dim3(g), dim3(256), 0, stream, coef, M_dense,
                         d->n_nodes, d->n_v, d->n_1d, d->dg_cells, d->L);
    BGK_HIP(hipGetLastError());
  }
  return BGK_OK;
}

// ----------------------------------------------------------------------------
// Batched forms: one launch over many instances (per-instance arguments in
// device memory; an instance whose done flag is set is skipped).
// ----------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int find_instance(const T* __restrict__ first, int n, T x) {
  int lo = 0, hi = n;  // first[lo] <= x < first[lo + 1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// One block per 128 nodes of one instance (instances' node ranges padded to
// whole blocks, blk_inst[b] the instance of block b, blk_first[i] its first
// block): the instance's arguments are wave-uniform, read through the scalar
// unit, and a finished instance's blocks leave at once.
template <int DIM>
__global__ __launch_bounds__(128) void k_maxwellian_batch(const BatchKin* __restrict__ kin,
                                                          const int32_t* __restrict__ par,
                                                          const int32_t* __restrict__ done,
                                                          const int32_t* __restrict__ blk_inst,
                                                          const int32_t* __restrict__ blk_first) {
  const int i = blk_inst[blockIdx.x];
  if (done[i]) return;
  const MaxwArgs& p = kin[i].maxw;
  const int64_t node = (int64_t)(blockIdx.x - blk_first[i]) * 128 + threadIdx.x;
  NodeStatus st;
  if (node < p.n_nodes) maxwellian_node<DIM>(p, kin[i].U[par[i]], node, st);
  flush_status(st, p.status, p.numax);
}

// Grid-stride over every instance's table threads; a thread that meets a
// finished instance (or one without tables) jumps to its first position past
// that instance's range, so finished instances cost O(instances) per thread.
template <int DIM>
__global__ void k_tables_batch(const BatchKin* __restrict__ kin, const int32_t* __restrict__ done,
                               const int64_t* __restrict__ first, int n_inst, int64_t total) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += stride) {
    const int i = find_instance<int64_t>(first, n_inst, g);
    if (done[i] || !kin[i].mtab) {
      const int64_t end = first[i + 1];
      if (end > g + stride) g += (end - g - 1) / stride * stride;
      continue;
    }
    // through a wave-uniform index when the wave is inside one instance
    // (scalar loads of its arguments), as in k_maxwellian_batch
    const auto chunk = [&](int ii) {
      const BatchKin& k = kin[ii];
      table_rows<DIM>(k.maxw.coef, k.maxw.nu, k.x1, k.geo, k.mtab, k.n_nodes / k.np, k.n1, k.np,
                      g - first[ii]);
    };
    const int i0 = __builtin_amdgcn_readfirstlane(i);
    if (__ballot(i != i0) == 0)
      chunk(i0);
    else
      chunk(i);
  }
}

template <int DIM, int NP>
__device__ __forceinline__ void moments_vl(const MomArgs& a, int vl, int blk, double* smem) {
  if (vl == 1)
    moments_block<DIM, NP, 1>(a, blk, smem);
  else if (vl == 4)
    moments_block<DIM, NP, 4>(a, blk, smem);
  else if (vl == 16)
    moments_block<DIM, NP, 16>(a, blk, smem);
  else
    moments_block<DIM, NP, 64>(a, blk, smem);
}

template <int DIM>
__global__ __launch_bounds__(MOM_THREADS) void k_moments_batch(
    const BatchKin* __restrict__ kin, const int32_t* __restrict__ par,
    const int32_t* __restrict__ done, const int32_t* __restrict__ first, int n_inst,
    int with_ratio) {
  constexpr int SM = DIM == 2 ? MomSmem<2, 6, 64>::TOTAL : MomSmem<3, 4, 64>::TOTAL;
  static_assert(DIM == 3 || (MomSmem<2, 3, 64>::TOTAL <= SM && MomSmem<2, 6, 16>::TOTAL <= SM &&
                             MomSmem<2, 6, 4>::TOTAL <= SM),
                "moment scratch");
  static_assert(DIM == 2 || MomSmem<3, 4, 16>::TOTAL <= SM, "moment scratch");
  __shared__ double smem[SM];
  const int i = find_instance<int32_t>(first, n_inst, (int32_t)blockIdx.x);
  if (done[i]) return;
  const BatchKin& k = kin[i];
  MomArgs a = k.mom;
  const int p = par[i];
  a.U = const_cast<double*>(k.U[p ^ 1]);
  a.U_prev = with_ratio ? k.U[p] : nullptr;
  const int blk = blockIdx.x - first[i];
  if constexpr (DIM == 2) {
    if (k.np == 3)
      moments_vl<2, 3>(a, k.mom_vl, blk, smem);
    else
      moments_vl<2, 6>(a, k.mom_vl, blk, smem);
  } else {
    moments_vl<3, 4>(a, k.mom_vl, blk, smem);
  }
}

__global__ __launch_bounds__(256) void k_ratio_batch(const BatchKin* __restrict__ kin,
                                                     const int32_t* __restrict__ done) {
  __shared__ double s[6][256];
  const int i = blockIdx.x;
  if (done[i]) return;
  ratio_block(kin[i].mom.partial, kin[i].mom_blocks, kin[i].ratio, s);
}

int launch_maxwellian_batch(int dim, const BatchKin* kin, const int32_t* par, const int32_t* done,
                            const int32_t* blk_inst, const int32_t* blk_first, int n_blocks,
                            hipStream_t stream) {
  if (n_blocks == 0) return BGK_OK;
  const dim3 grid((unsigned)n_blocks), block(128);
  if (dim == 2)
    hipLaunchKernelGGL(k_maxwellian_batch<2>, grid, block, 0, stream, kin, par, done, blk_inst,
                       blk_first);
  else
    hipLaunchKernelGGL(k_maxwellian_batch<3>, grid, block, 0, stream, kin, par, done, blk_inst,
                       blk_first);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_tables_batch(int dim, const BatchKin* kin, const int32_t* done,
                        const int64_t* entry_first, int n_inst, int64_t n_total,
                        hipStream_t stream) {
  if (n_total == 0) return BGK_OK;
  const int grid = (int)std::min<int64_t>((n_total + 255) / 256, 65536);
  if (dim == 2)
    hipLaunchKernelGGL(k_tables_batch<2>, dim3(grid), dim3(256), 0, stream, kin, done, entry_first,
                       n_inst, n_total);
  else
    hipLaunchKernelGGL(k_tables_batch<3>, dim3(grid), dim3(256), 0, stream, kin, done, entry_first,
                       n_inst, n_total);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_moments_batch(int dim, const BatchKin* kin, const int32_t* par, const int32_t* done,
                         const int32_t* blk_first, int n_inst, int n_blocks, bool with_ratio,
                         hipStream_t stream) {
  if (dim == 2)
    hipLaunchKernelGGL(k_moments_batch<2>, dim3(n_blocks), dim3(MOM_THREADS), 0, stream, kin, par,
                       done, blk_first, n_inst, (int)with_ratio);
  else
    hipLaunchKernelGGL(k_moments_batch<3>, dim3(n_blocks), dim3(MOM_THREADS), 0, stream, kin, par,
                       done, blk_first, n_inst, (int)with_ratio);
  BGK_HIP(hipGetLastError());
  if (with_ratio) {
    hipLaunchKernelGGL(k_ratio_batch, dim3(n_inst), dim3(256), 0, stream, kin, done);
    BGK_HIP(hipGetLastError());
  }
  return BGK_OK;
}

// Scratch of the allocation-free moments entry point (moments_noalloc):
// the chunk sums of a velocity-split moment pass, the per-block partial
// norms of the convergence ratios, then the ratios.
// One copy per device, held until the process ends.  Host code never uses
// the array's name as an address: it takes the device address from
// hipGetSymbolAddress once per device (noalloc_scratch below).
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = (int64_t)1 << 22;  // 32 MiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with it current).
int noalloc_scratch(double** out) {
  int dev = 0;
  BGK_HIP(hipGetDevice(&dev));
  BGK_CHECK(dev >= 0 && dev < NOALLOC_MAX_DEVICES, BGK_E_UNSUPPORTED, "device index too large");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    BGK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    BGK_CHECK(p != nullptr, BGK_E_HIP, "hipGetSymbolAddress returned no address");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return BGK_OK;
}

}  // namespace bgk

using namespace bgk;

extern "C" int moments(const tgs_dag* d, const double* f, double* U, const double* U_prev,
                       double* rel3, bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!d || !f || !U) return fail(BGK_E_INVALID, "null argument");
    if ((U_prev == nullptr) != (rel3 == nullptr))
      return fail(BGK_E_INVALID, "U_prev and rel3 go together");
    double* partial = nullptr;
    double* ratio = nullptr;
    double* split = nullptr;
    hipStream_t s = (hipStream_t)stream;
    const auto release = [&]() {
      if (partial) (void)hipFreeAsync(partial, s);
      if (ratio) (void)hipFreeAsync(ratio, s);
      if (split) (void)hipFreeAsync(split, s);
    };
    const int64_t nsplit = moment_split_doubles(d);
    if ((U_prev &&
         (hipMallocAsync((void**)&partial, (size_t)moment_partials(d) * 6 * sizeof(double), s) !=
              hipSuccess ||
          hipMallocAsync((void**)&ratio, 4 * sizeof(double), s) != hipSuccess)) ||
        (nsplit > 0 &&
         hipMallocAsync((void**)&split, (size_t)nsplit * sizeof(double), s) != hipSuccess)) {
      release();
      return fail(BGK_E_NOMEM, "scratch allocation failed");
    }
    int rc = launch_moments(d, f, U, U_prev, partial, ratio, s, true, split);
    if (rc == BGK_OK && U_prev) {
      if (hipMemcpyAsync(rel3, ratio, 3 * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = fail(BGK_E_HIP, "copy of ratios failed");
    }
    release();
    return rc;
  });
}

extern "C" int moments_noalloc(const tgs_dag* d, const double* f, double* U,
                               const double* U_prev, double* rel3, bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!d || !f || !U) return fail(BGK_E_INVALID, "null argument");
    if ((U_prev == nullptr) != (rel3 == nullptr))
      return fail(BGK_E_INVALID, "U_prev and rel3 go together");
    hipStream_t s = (hipStream_t)stream;
    double* partial = nullptr;
    double* ratio = nullptr;
    double* split = nullptr;
    // the scratch, each part 256-byte aligned: the chunk sums of a
    // velocity-split pass, the partial norms (6 per piece), the ratios
    const int64_t nsplit = moment_split_doubles(d);
    const int64_t at_part = (nsplit + 31) / 32 * 32;
    const int64_t need = U_prev ? (int64_t)moment_partials(d) * 6 : 0;
    const int64_t at_ratio = at_part + (need + 31) / 32 * 32;
    const int64_t total = at_ratio + (U_prev ? 4 : 0);
    if (total > NOALLOC_SCRATCH_DOUBLES)
      return fail(BGK_E_INVALID, "moments_noalloc: the mesh needs " + std::to_string(total) +
                                     " doubles of scratch, above the fixed " +
                                     std::to_string(NOALLOC_SCRATCH_DOUBLES) + " (use moments)");
    if (total > 0) {
      double* base = nullptr;
      int rc = noalloc_scratch(&base);
      if (rc) return rc;
      if (nsplit > 0) split = base;
      if (U_prev) {
        partial = base + at_part;
        ratio = base + at_ratio;
      }
    }
    // every chunk sum and every partial norm is written before it is read:
    // nothing in the scratch needs clearing
    int rc = launch_moments(d, f, U, U_prev, partial, ratio, s, true, split);
    if (rc == BGK_OK && U_prev) {
      if (hipMemcpyAsync(rel3, ratio, 3 * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = fail(BGK_E_HIP, "copy of ratios failed");
    }
    return rc;
  });
}

extern "C" int maxwellian(const tgs_dag* d, int mode, const double* U, const tgs_nu_model* nm,
                          double* coef, double* nu, double* M_dense, int32_t* status,
                          bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!d || !U || !coef || !nu) return fail(BGK_E_INVALID, "null argument");
    return launch_maxwellian(d, mode, U, nm, coef, nu, M_dense, status, nullptr, nullptr,
                             (hipStream_t)stream);
  });
}

extern "C" int maxwellian_coef_from_primitive(int dim, int64_t n, const double* prim, double* coef,
                                              bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!prim || !coef || n < 0 || (dim != 2 && dim != 3))
      return fail(BGK_E_INVALID, "bad arguments");
    if (n == 0) return BGK_OK;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (dim == 2)
      hipLaunchKernelGGL(k_coef_from_prim<2>, grid, block, 0, (hipStream_t)stream, prim, coef, n);
    else
      hipLaunchKernelGGL(k_coef_from_prim<3>, grid, block, 0, (hipStream_t)stream, prim, coef, n);
    BGK_HIP(hipGetLastError());
    return BGK_OK;
  });
}
