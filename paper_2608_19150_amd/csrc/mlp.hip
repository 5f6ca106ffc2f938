// Learned Picard initial guess: a per-node MLP 11 -> 64 -> 64 -> 64 -> 5
// (GELU hidden layers) run on BF16 MFMA with FP32 accumulation, trained on
// the GPU with back-propagation and Adam on FP32 master weights.
//
// Matrix products run on 16-row tiles (one tile per wavefront).  Products
// over the 64 hidden features use gfx950's v_mfma_f32_16x16x32_bf16 (two
// K-steps of 32); those over 16 (the padded inputs, the padded outputs in
// back-propagation, and the 16 rows of a tile in the weight gradients) use
// v_mfma_f32_16x16x16bf16_1k.  Operand fragments, lane l of 64, q = l / 16:
//   K = 32: A[l % 16][8q + i], B[8q + i][l % 16], i = 0..7
//   K = 16: A[l % 16][4q + i], B[4q + i][l % 16], i = 0..3
//   D (16 x 16, M x N): D[4q + i][l % 16], i = 0..3
// (the instruction pairs a lane's i-th A value with the i-th B value of the
// lanes of its column; any k order used alike by A and B is exact).
// Weights are kept as FP32 masters in a padded layout (inputs 11 -> 16,
// outputs 5 -> 16) and mirrored as BF16 B-operand fragments, both W (forward)
// and W^T (back-propagation), so each lane reads its values in one load.
// Activations live in LDS rows padded to 72 bf16 (16-byte aligned rows for
// the 8-value fragment reads).  Weight gradients are written per tile and
// summed over tiles in a fixed order, so training is bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.h"

namespace bgk {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int NI = 11, NO = 5, HD = 64, K1 = 16, N4 = 16;
// padded FP32 master layout
constexpr int OW1 = 0, OB1 = OW1 + K1 * HD, OW2 = OB1 + HD, OB2 = OW2 + HD * HD, OW3 = OB2 + HD,
              OB3 = OW3 + HD * HD, OW4 = OB3 + HD, OB4 = OW4 + HD * N4, NPAD = OB4 + N4;
// BF16 fragment buffer: forward W1, W2, W3, W4 then transposed W2, W3, W4
constexpr int FW1 = 0, FW2 = FW1 + K1 * HD, FW3 = FW2 + HD * HD, FW4 = FW3 + HD * HD,
              TW2 = FW4 + HD * N4, TW3 = TW2 + HD * HD, TW4 = TW3 + HD * HD, NFRAG = TW4 + N4 * HD;
constexpr int AST = 72;            // LDS row stride of activations (bf16, 16-byte rows)
constexpr int MLP_THREADS = 256;   // 4 wavefronts, one 16-row tile each
constexpr int GRAD_BLOCKS = 1024;  // gradient launches: one accumulator per wavefront

// Orders a wavefront's LDS writes before its later LDS reads by other lanes
// (DS operations of one wavefront complete in order; this stops the compiler
// from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma32(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// D (16 x NT*16) = act (16 x 16, LDS) * W (K = 16 fragments)
template <int NT>
__device__ __forceinline__ void mm_act_w16(const uint16_t* act, const uint16_t* __restrict__ frag,
                                           v4f (&acc)[NT], int lane) {
  const v4s* wf = reinterpret_cast<const v4s*>(frag);
  const v4s a = *reinterpret_cast<const v4s*>(act + (lane % 16) * AST + 4 * (lane / 16));
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma(a, wf[nt * 64 + lane], v4f{0.f, 0.f, 0.f, 0.f});
}

// D (16 x NT*16) = act (16 x 64, LDS) * W (K = 32 fragments, two K-steps)
template <int NT>
__device__ __forceinline__ void mm_act_w64(const uint16_t* act, const uint16_t* __restrict__ frag,
                                           v4f (&acc)[NT], int lane) {
  const v8bf* wf = reinterpret_cast<const v8bf*>(frag);
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < 2; ++kt) {
    const v8bf a =
        *reinterpret_cast<const v8bf*>(act + (lane % 16) * AST + kt * 32 + 8 * (lane / 16));
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma32(a, wf[(kt * NT + nt) * 64 + lane], acc[nt]);
  }
}

// D (MT*16 x NT*16) = h^T (features x 16 rows) * g (16 rows x features), both
// LDS; emits each 16 x NT*16 row block through sink(mt, nt, acc) as soon as it
// is complete, so only one block of accumulators is live.
template <int MT, int NT, class Sink>
__device__ __forceinline__ void mm_hT_g(const uint16_t* h, const uint16_t* g, int lane, Sink sink) {
  const int r = lane % 16, kq = lane / 16;
  v4s b[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) b[nt][i] = (short)g[(4 * kq + i) * AST + nt * 16 + r];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    v4s a;
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = (short)h[(4 * kq + i) * AST + mt * 16 + r];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) sink(mt, nt, mfma(a, b[nt], v4f{0.f, 0.f, 0.f, 0.f}));
  }
}

struct MlpArgs {
  const float* master;    // [NPAD]
  const uint16_t* frag;   // [NFRAG] BF16 fragments
  const float* stats;     // mean_in[11], std_in[11], mean_out[5], std_out[5]
};

// Hidden layer epilogue: z = acc + b (kept in registers, D layout, for the
// backward pass), h = gelu(z) -> bf16 act_out
__device__ __forceinline__ void hidden_epilogue(v4f (&acc)[4], const float* __restrict__ b,
                                                uint16_t* act_out, int lane) {
  const int r = lane % 16, kq = lane / 16;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int col = nt * 16 + r;
    const float bc = b[col];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float z = acc[nt][i] + bc;
      acc[nt][i] = z;
      act_out[(4 * kq + i) * AST + col] = f2bf(gelu(z));
    }
  }
  wave_sync();
}

// Forward pass of one 16-row tile whose normalised inputs are in act (rows
// 0..15); hidden activations go to act rows 16..63 (h1, h2, h3) and the
// pre-activations to z.  Returns the normalised outputs in D layout
// (column = lane % 16).
__device__ __forceinline__ v4f forward_tile(const MlpArgs& m, uint16_t* act, v4f (&z)[3][4],
                                            int lane) {
  mm_act_w16<4>(act, m.frag + FW1, z[0], lane);
  hidden_epilogue(z[0], m.master + OB1, act + 16 * AST, lane);
  mm_act_w64<4>(act + 16 * AST, m.frag + FW2, z[1], lane);
  hidden_epilogue(z[1], m.master + OB2, act + 32 * AST, lane);
  mm_act_w64<4>(act + 32 * AST, m.frag + FW3, z[2], lane);
  hidden_epilogue(z[2], m.master + OB3, act + 48 * AST, lane);
  v4f out[1];
  mm_act_w64<1>(act + 48 * AST, m.frag + FW4, out, lane);
  const float b4 = m.master[OB4 + lane % 16];
  return out[0] + v4f{b4, b4, b4, b4};
}

// Loads 16 rows of raw features, normalised, into act (bf16, cols 11..15 = 0)
__device__ __forceinline__ void load_inputs(const MlpArgs& m, const float* __restrict__ X, int64_t n,
                                            int64_t row0, uint16_t* act, int lane) {
  for (int idx = lane; idx < 16 * 16; idx += 64) {
    const int r = idx / 16, c = idx % 16;
    const int64_t row = row0 + r;
    float x = 0.0f;
    if (c < NI && row < n) x = (X[row * NI + c] - m.stats[c]) / m.stats[NI + c];
    act[r * AST + c] = f2bf(x);
  }
  wave_sync();
}

__global__ __launch_bounds__(MLP_THREADS) void k_mlp_forward(MlpArgs m, const float* __restrict__ X,
                                                             int64_t n, float* __restrict__ Y) {
  __shared__ __align__(16) uint16_t s_act[4][4 * 16 * AST];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  uint16_t* act = s_act[wave];
  const int64_t ntiles = (n + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t row0 = tile * 16;
    load_inputs(m, X, n, row0, act, lane);
    v4f z[3][4];
    const v4f y = forward_tile(m, act, z, lane);
    const int c = lane % 16;
    if (c < NO)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + 4 * (lane / 16) + i;
        if (row < n) Y[row * NO + c] = y[i] * m.stats[2 * NI + NO + c] + m.stats[2 * NI + c];
      }
    wave_sync();
  }
}

// sum over the 4 row-quads of each column (lanes r, r+16, r+32, r+48), fixed order
__device__ __forceinline__ float col_sum(float x, int lane) {
  const float a = __shfl(x, lane % 16), b = __shfl(x, lane % 16 + 16), c = __shfl(x, lane % 16 + 32),
              d = __shfl(x, lane % 16 + 48);
  return ((a + b) + c) + d;
}

// Loss and parameter gradients (padded layout), one wavefront per block.
// Block s takes tiles s, s + grid, ... and accumulates their gradients, in
// that order, in LDS (every index owned by one lane: race-free and
// reproducible), then writes partial[s][NPAD] and partial_loss[s].
__global__ __launch_bounds__(64) void k_mlp_grad(MlpArgs m, const float* __restrict__ X,
                                                 const float* __restrict__ T, int64_t n,
                                                 float* __restrict__ partial,
                                                 float* __restrict__ partial_loss) {
  __shared__ __align__(16) uint16_t act[4 * 16 * AST];
  __shared__ __align__(16) uint16_t g[16 * AST];
  __shared__ float gacc[NPAD];
  const int lane = threadIdx.x;
  const int r = lane % 16, kq = lane / 16;
  const int64_t ntiles = (n + 15) / 16;
  const int64_t slot = blockIdx.x;
  for (int p = lane; p < NPAD; p += 64) gacc[p] = 0.0f;
  wave_sync();
  const float inv = 2.0f / (float)(n * NO);
  float lacc = 0.0f;
  for (int64_t tile = slot; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * 16;
    load_inputs(m, X, n, row0, act, lane);
    v4f z[3][4];
    const v4f y = forward_tile(m, act, z, lane);
    // dY (normalised domain) and loss
    float lsum = 0.0f, dcol = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 4 * kq + i;
      const int64_t grow = row0 + row;
      float dy = 0.0f;
      if (r < NO && grow < n) {
        const float t = (T[grow * NO + r] - m.stats[2 * NI + r]) / m.stats[2 * NI + NO + r];
        const float diff = y[i] - t;
        lsum += diff * diff;
        dy = inv * diff;
      }
      dcol += dy;
      g[row * AST + r] = f2bf(dy);
    }
    wave_sync();
    {
      const float db = col_sum(dcol, lane);
      if (kq == 0) gacc[OB4 + r] += db;
    }
    // dW4 = h3^T dY   (64 x 16)
    mm_hT_g<4, 1>(act + 48 * AST, g, lane, [&](int mt, int, v4f d) {
#pragma unroll
      for (int i = 0; i < 4; ++i) gacc[OW4 + (mt * 16 + 4 * kq + i) * N4 + r] += d[i];
    });
    // back through the hidden layers: dh = g W^T, dz = dh * gelu'(z), dW = h_prev^T dz
#pragma unroll
    for (int L = 0; L < 3; ++L) {
      const int lay = 2 - L;  // hidden layer index of z (0-based)
      v4f dh[4];
      if (L == 0)
        mm_act_w16<4>(g, m.frag + TW4, dh, lane);
      else
        mm_act_w64<4>(g, m.frag + (L == 1 ? TW3 : TW2), dh, lane);
      wave_sync();  // every lane has read g before it is overwritten
      const int obias = L == 0 ? OB3 : (L == 1 ? OB2 : OB1);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int col = nt * 16 + r;
        float cs = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float dz = dh[nt][i] * gelu_grad(z[lay][nt][i]);
          cs += dz;
          g[(4 * kq + i) * AST + col] = f2bf(dz);
        }
        const float db = col_sum(cs, lane);
        if (kq == 0) gacc[obias + col] += db;
      }
      wave_sync();
      const uint16_t* hprev = act + lay * 16 * AST;
      const int ow = L == 0 ? OW3 : (L == 1 ? OW2 : OW1);
      auto sink = [&](int mt, int nt, v4f d) {
#pragma unroll
        for (int i = 0; i < 4; ++i) gacc[ow + (mt * 16 + 4 * kq + i) * HD + nt * 16 + r] += d[i];
      };
      if (L < 2)
        mm_hT_g<4, 4>(hprev, g, lane, sink);
      else
        mm_hT_g<1, 4>(hprev, g, lane, sink);
    }
    // loss: butterfly sum over the wavefront (same order on every lane)
    float ls = lsum;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ls += __shfl_xor(ls, off);
    lacc += ls;
    wave_sync();  // all reads of act / g done before the next tile's writes
  }
  wave_sync();
  if (slot < ntiles) {
    float* P = partial + (size_t)slot * NPAD;
    for (int p = lane; p < NPAD; p += 64) P[p] = gacc[p];
    if (lane == 0) partial_loss[slot] = lacc / (float)(n * NO);
  }
}

// grad[p] = sum over wavefront accumulators (slot order), loss likewise.
// The loads of 16 slots are issued before they are added (in slot order),
// so each thread keeps 16 loads in flight; 64-thread blocks spread the
// parameters over more compute units.
__global__ __launch_bounds__(64) void k_mlp_reduce(const float* __restrict__ partial,
                                                   const float* __restrict__ ploss,
                                                   int64_t nslots, float* __restrict__ grad,
                                                   float* __restrict__ loss) {
  constexpr int U = 16;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const auto ordered_sum = [&](const float* __restrict__ base, size_t stride) {
    float s = 0.0f;
    int64_t t = 0;
    for (; t + U <= nslots; t += U) {
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = base[(size_t)(t + u) * stride];
#pragma unroll
      for (int u = 0; u < U; ++u) s += v[u];
    }
    for (; t < nslots; ++t) s += base[(size_t)t * stride];
    return s;
  };
  if (p < NPAD) grad[p] = ordered_sum(partial + p, NPAD);
  if (p == NPAD && loss) *loss = ordered_sum(ploss, 1);
}

__global__ void k_mlp_adam(float* __restrict__ w, float* __restrict__ mo, float* __restrict__ ve,
                           const float* __restrict__ g, float lr, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPAD) return;
  const float gp = g[p];
  const float m = 0.9f * mo[p] + 0.1f * gp;
  const float v = 0.999f * ve[p] + 0.001f * gp * gp;
  mo[p] = m;
  ve[p] = v;
  w[p] -= lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
}

// BF16 fragments of the current master weights
__global__ void k_mlp_frag(const float* __restrict__ w, uint16_t* __restrict__ frag) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NFRAG) return;
  // decode (block, kt, nt, lane, i) for the layer this element belongs to
  int base, K, N, ow;
  bool trans;
  if (e < FW2) { base = FW1; K = K1; N = HD; ow = OW1; trans = false; }
  else if (e < FW3) { base = FW2; K = HD; N = HD; ow = OW2; trans = false; }
  else if (e < FW4) { base = FW3; K = HD; N = HD; ow = OW3; trans = false; }
  else if (e < TW2) { base = FW4; K = HD; N = N4; ow = OW4; trans = false; }
  else if (e < TW3) { base = TW2; K = HD; N = HD; ow = OW2; trans = true; }
  else if (e < TW4) { base = TW3; K = HD; N = HD; ow = OW3; trans = true; }
  else { base = TW4; K = N4; N = HD; ow = OW4; trans = true; }
  // K = 64 layers: 8-value fragments of 32-deep K-steps; K = 16: 4-value
  const int loc = e - base;
  const int V = K == HD ? 8 : 4;
  const int i = loc % V, lane = (loc / V) % 64, tileidx = loc / (64 * V);
  const int NT = N / 16;
  const int kt = tileidx / NT, nt = tileidx % NT;
  const int k = kt * 4 * V + V * (lane / 16) + i, nn = nt * 16 + lane % 16;
  // B operand value B[k][nn]: forward W[k][nn]; transposed W^T[k][nn] = W[nn][k]
  // (W stored [fan_in][fan_out] with row length N_out of that layer)
  float val;
  if (!trans) {
    val = w[ow + k * N + nn];
  } else {
    val = w[ow + nn * K + k];
  }
  frag[e] = f2bf(val);
}

// ---- features, targets and the fused guess ----------------------------------
template <int DIM>
__device__ __forceinline__ void prim5(const double* U, double (&p)[5]) {
  const double n = U[0];
  double uu = 0.0;
  p[0] = n;
  p[1] = p[2] = p[3] = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    p[1 + d] = U[1 + d] / n;
    uu = fma(p[1 + d], p[1 + d], uu);
  }
  p[4] = (2.0 * U[1 + DIM] / n - uu) / DIM;
}

template <int DIM>
__device__ __forceinline__ void node_features(const double* U1, const double* U2, int nu_kind,
                                              double nu_const, double kn, double dt, float* x) {
  double p1[5], p2[5];
  prim5<DIM>(U1, p1);
  prim5<DIM>(U2, p2);
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    x[c] = (float)p1[c];
    x[5 + c] = (float)(p1[c] - p2[c]);
  }
  const double nu = nu_kind == BGK_NU_CONST ? nu_const : p1[0] / sqrt(p1[4]) / kn;
  x[10] = (float)(dt * nu);
}

template <int DIM>
__global__ void k_mlp_features(const double* __restrict__ U1, const double* __restrict__ U2,
                               int64_t n, int nu_kind, double nu_const, double kn, double dt,
                               float* __restrict__ X) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x[NI];
  node_features<DIM>(U1 + i * (DIM + 2), U2 + i * (DIM + 2), nu_kind, nu_const, kn, dt, x);
#pragma unroll
  for (int c = 0; c < NI; ++c) X[i * NI + c] = x[c];
}

template <int DIM>
__global__ void k_mlp_targets(const double* __restrict__ Ut, const double* __restrict__ U1,
                              const double* __restrict__ U2, int64_t n, float* __restrict__ T) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double pt[5], p1[5], p2[5];
  prim5<DIM>(Ut + i * (DIM + 2), pt);
  prim5<DIM>(U1 + i * (DIM + 2), p1);
  prim5<DIM>(U2 + i * (DIM + 2), p2);
#pragma unroll
  for (int c = 0; c < NO; ++c) T[i * NO + c] = (float)(pt[c] - (p1[c] + (p1[c] - p2[c])));
}

template <int DIM>
__global__ __launch_bounds__(MLP_THREADS) void k_mlp_guess(MlpArgs m, const double* __restrict__ U1,
                                                           const double* __restrict__ U2, int64_t n,
                                                           int nu_kind, double nu_const, double kn,
                                                           double dt, double* __restrict__ Ug,
                                                           int32_t* fallback) {
  constexpr int NM = DIM + 2;
  __shared__ __align__(16) uint16_t s_act[4][4 * 16 * AST];
  __shared__ float s_y[4][16 * 17];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  uint16_t* act = s_act[wave];
  float* ys = s_y[wave];
  const int64_t ntiles = (n + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t row0 = tile * 16;
    // lanes 0..15: one node each
    if (lane < 16) {
      const int64_t node = row0 + lane;
      float x[NI];
      if (node < n) {
        node_features<DIM>(U1 + node * NM, U2 + node * NM, nu_kind, nu_const, kn, dt, x);
      } else {
#pragma unroll
        for (int c = 0; c < NI; ++c) x[c] = m.stats[c];
      }
#pragma unroll
      for (int c = 0; c < 16; ++c)
        act[lane * AST + c] = f2bf(c < NI ? (x[c] - m.stats[c]) / m.stats[NI + c] : 0.0f);
    }
    wave_sync();
    v4f z[3][4];
    const v4f y = forward_tile(m, act, z, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) ys[(4 * (lane / 16) + i) * 17 + lane % 16] = y[i];
    wave_sync();
    if (lane < 16) {
      const int64_t node = row0 + lane;
      if (node < n) {
        double p1[5], p2[5], q[5];
        prim5<DIM>(U1 + node * NM, p1);
        prim5<DIM>(U2 + node * NM, p2);
        bool ok = true;
#pragma unroll
        for (int c = 0; c < NO; ++c) {
          const double dlt = (double)(ys[lane * 17 + c] * m.stats[2 * NI + NO + c] + m.stats[2 * NI + c]);
          q[c] = p1[c] + (p1[c] - p2[c]) + dlt;
          ok = ok && isfinite(q[c]);
        }
        ok = ok && q[0] > 0.0 && q[4] > 0.0;
        double* out = Ug + node * NM;
        if (ok) {
          double uu = 0.0;
          out[0] = q[0];
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            out[1 + d] = q[0] * q[1 + d];
            uu = fma(q[1 + d], q[1 + d], uu);
          }
          out[1 + DIM] = 0.5 * q[0] * uu + 0.5 * DIM * q[0] * q[4];
        } else {
#pragma unroll
          for (int c = 0; c < NM; ++c) out[c] = U1[node * NM + c];
          if (fallback) atomicAdd(fallback, 1);
        }
      }
    }
    wave_sync();
  }
}

// logical <-> padded parameter layouts
void logical_to_padded(const float* src, float* dst) {
  std::memset(dst, 0, NPAD * sizeof(float));
  const float* p = src;
  for (int i = 0; i < NI; ++i)
    for (int j = 0; j < HD; ++j) dst[OW1 + i * HD + j] = *p++;
  for (int j = 0; j < HD; ++j) dst[OB1 + j] = *p++;
  for (int i = 0; i < HD * HD; ++i) dst[OW2 + i] = *p++;
  for (int j = 0; j < HD; ++j) dst[OB2 + j] = *p++;
  for (int i = 0; i < HD * HD; ++i) dst[OW3 + i] = *p++;
  for (int j = 0; j < HD; ++j) dst[OB3 + j] = *p++;
  for (int i = 0; i < HD; ++i)
    for (int j = 0; j < NO; ++j) dst[OW4 + i * N4 + j] = *p++;
  for (int j = 0; j < NO; ++j) dst[OB4 + j] = *p++;
}
void padded_to_logical(const float* src, float* dst) {
  float* p = dst;
  for (int i = 0; i < NI; ++i)
    for (int j = 0; j < HD; ++j) *p++ = src[OW1 + i * HD + j];
  for (int j = 0; j < HD; ++j) *p++ = src[OB1 + j];
  for (int i = 0; i < HD * HD; ++i) *p++ = src[OW2 + i];
  for (int j = 0; j < HD; ++j) *p++ = src[OB2 + j];
  for (int i = 0; i < HD * HD; ++i) *p++ = src[OW3 + i];
  for (int j = 0; j < HD; ++j) *p++ = src[OB3 + j];
  for (int i = 0; i < HD; ++i)
    for (int j = 0; j < NO; ++j) *p++ = src[OW4 + i * N4 + j];
  for (int j = 0; j < NO; ++j) *p++ = src[OB4 + j];
}

__global__ void k_padded_to_logical(const float* __restrict__ src, float* __restrict__ dst) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= BGK_MLP_PARAMS) return;
  int idx;
  int p = q;
  if (p < NI * HD) { idx = OW1 + p; }
  else if ((p -= NI * HD) < HD) { idx = OB1 + p; }
  else if ((p -= HD) < HD * HD) { idx = OW2 + p; }
  else if ((p -= HD * HD) < HD) { idx = OB2 + p; }
  else if ((p -= HD) < HD * HD) { idx = OW3 + p; }
  else if ((p -= HD * HD) < HD) { idx = OB3 + p; }
  else if ((p -= HD) < HD * NO) { idx = OW4 + (p / NO) * N4 + p % NO; }
  else { p -= HD * NO; idx = OB4 + p; }
  dst[q] = src[idx];
}

}  // namespace
}  // namespace bgk

using namespace bgk;

struct bgk_mlp {
  float* master = nullptr;   // [NPAD]
  float* m1 = nullptr;       // Adam first moment
  float* m2 = nullptr;       // Adam second moment
  uint16_t* frag = nullptr;  // [NFRAG]
  float* stats = nullptr;    // [32]
  float* grad = nullptr;     // [NPAD]
  float* partial = nullptr;  // [GRAD_BLOCKS][NPAD] per-wavefront gradient sums
  float* ploss = nullptr;    // [GRAD_BLOCKS]
  int step = 0;
};

namespace {
int mlp_sync(bgk_mlp* m, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_frag, dim3((NFRAG + 255) / 256), dim3(256), 0, s, m->master, m->frag);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}
MlpArgs margs(const bgk_mlp* m) {
  return MlpArgs{m->master, m->frag, m->stats};
}
int grid_tiles(int64_t ntiles) { return (int)std::max<int64_t>(1, std::min<int64_t>((ntiles + 3) / 4, 4096)); }
}  // namespace

extern "C" int bgk_mlp_create(const float* params, bgk_mlp** out) {
  return guarded([&]() -> int {
    if (!out) return fail(BGK_E_INVALID, "null argument");
    *out = nullptr;
    bgk_mlp* m = new (std::nothrow) bgk_mlp();
    if (!m) return fail(BGK_E_NOMEM, "host allocation failed");
    bool ok = hipMalloc((void**)&m->master, NPAD * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&m->m1, NPAD * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&m->m2, NPAD * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&m->grad, NPAD * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&m->frag, NFRAG * sizeof(uint16_t)) == hipSuccess &&
              hipMalloc((void**)&m->stats, 32 * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&m->partial, (size_t)GRAD_BLOCKS * NPAD * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&m->ploss, (size_t)GRAD_BLOCKS * sizeof(float)) == hipSuccess;
    if (!ok) {
      bgk_mlp_destroy(m);
      return fail(BGK_E_NOMEM, "MLP allocation failed");
    }
    std::vector<float> stats(32, 0.0f);
    for (int c = 0; c < NI; ++c) stats[NI + c] = 1.0f;
    for (int c = 0; c < NO; ++c) stats[2 * NI + NO + c] = 1.0f;
    if (hipMemcpy(m->stats, stats.data(), 32 * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      bgk_mlp_destroy(m);
      return fail(BGK_E_HIP, "stats upload failed");
    }
    int rc = bgk_mlp_set_params(m, params);
    if (rc) {
      bgk_mlp_destroy(m);
      return rc;
    }
    *out = m;
    return BGK_OK;
  });
}

extern "C" int bgk_mlp_destroy(bgk_mlp* m) {
  return guarded([&]() -> int {
    if (!m) return BGK_OK;
    void* ptrs[] = {m->master, m->m1, m->m2, m->frag, m->stats, m->grad, m->partial, m->ploss};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    delete m;
    return BGK_OK;
  });
}

extern "C" int bgk_mlp_set_params(bgk_mlp* m, const float* params) {
  return guarded([&]() -> int {
    if (!m) return fail(BGK_E_INVALID, "null mlp");
    std::vector<float> pad(NPAD, 0.0f);
    if (params) logical_to_padded(params, pad.data());
    BGK_HIP(hipMemcpy(m->master, pad.data(), NPAD * sizeof(float), hipMemcpyHostToDevice));
    BGK_HIP(hipMemset(m->m1, 0, NPAD * sizeof(float)));
    BGK_HIP(hipMemset(m->m2, 0, NPAD * sizeof(float)));
    m->step = 0;
    int rc = mlp_sync(m, nullptr);
    if (rc) return rc;
    BGK_HIP(hipDeviceSynchronize());
    return BGK_OK;
  });
}

extern "C" int bgk_mlp_get_params(const bgk_mlp* m, float* params) {
  return guarded([&]() -> int {
    if (!m || !params) return fail(BGK_E_INVALID, "null argument");
    std::vector<float> pad(NPAD);
    BGK_HIP(hipDeviceSynchronize());
    BGK_HIP(hipMemcpy(pad.data(), m->master, NPAD * sizeof(float), hipMemcpyDeviceToHost));
    padded_to_logical(pad.data(), params);
    return BGK_OK;
  });
}

extern "C" int bgk_mlp_set_normalization(bgk_mlp* m, const float* stats) {
  return guarded([&]() -> int {
    if (!m || !stats) return fail(BGK_E_INVALID, "null argument");
    for (int c = 0; c < NI; ++c)
      if (!(stats[NI + c] > 0.0f)) return fail(BGK_E_INVALID, "input std must be positive");
    for (int c = 0; c < NO; ++c)
      if (!(stats[2 * NI + NO + c] > 0.0f)) return fail(BGK_E_INVALID, "output std must be positive");
    BGK_HIP(hipMemcpy(m->stats, stats, 32 * sizeof(float), hipMemcpyHostToDevice));
    return BGK_OK;
  });
}

extern "C" int bgk_mlp_forward(bgk_mlp* m, const float* X, int64_t n, float* Y,
                               bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!m || !X || !Y || n < 0) return fail(BGK_E_INVALID, "bad arguments");
    if (n == 0) return BGK_OK;
    const int64_t ntiles = (n + 15) / 16;
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid_tiles(ntiles)), dim3(MLP_THREADS), 0,
                       (hipStream_t)stream, margs(m), X, n, Y);
    BGK_HIP(hipGetLastError());
    return BGK_OK;
  });
}

namespace {
int mlp_grad(bgk_mlp* m, const float* X, const float* T, int64_t n, float* loss, hipStream_t s) {
  const int64_t ntiles = (n + 15) / 16;
  const int grid = (int)std::min<int64_t>(ntiles, GRAD_BLOCKS);
  const int64_t nslots = grid;
  hipLaunchKernelGGL(k_mlp_grad, dim3(grid), dim3(64), 0, s, margs(m), X, T, n,
                     m->partial, m->ploss);
  BGK_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mlp_reduce, dim3((NPAD + 1 + 63) / 64), dim3(64), 0, s, m->partial,
                     m->ploss, nslots, m->grad, loss);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}
}  // namespace

extern "C" int bgk_mlp_loss_grad(bgk_mlp* m, const float* X, const float* T, int64_t n, float* grad,
                                 float* loss, bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!m || !X || !T || n <= 0) return fail(BGK_E_INVALID, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    int rc = mlp_grad(m, X, T, n, loss, s);
    if (rc) return rc;
    if (grad) {
      hipLaunchKernelGGL(k_padded_to_logical, dim3((BGK_MLP_PARAMS + 255) / 256), dim3(256), 0, s,
                         m->grad, grad);
      BGK_HIP(hipGetLastError());
    }
    return BGK_OK;
  });
}

extern "C" int bgk_mlp_adam_step(bgk_mlp* m, const float* X, const float* T, int64_t n, float lr,
                                 float* loss, bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!m || !X || !T || n <= 0 || !(lr > 0.0f)) return fail(BGK_E_INVALID, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    int rc = mlp_grad(m, X, T, n, loss, s);
    if (rc) return rc;
    m->step += 1;
    const float c1 = 1.0f - std::pow(0.9f, (float)m->step);
    const float c2 = 1.0f - std::pow(0.999f, (float)m->step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPAD + 255) / 256), dim3(256), 0, s, m->master, m->m1, m->m2,
                       m->grad, lr, c1, c2);
    BGK_HIP(hipGetLastError());
    return mlp_sync(m, s);
  });
}

extern "C" int bgk_mlp_features(const tgs_dag* d, const double* U1, const double* U2,
                                const tgs_nu_model* nm, double dt, float* X, bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!d || !U1 || !U2 || !nm || !X) return fail(BGK_E_INVALID, "null argument");
    const int64_t n = d->n_nodes;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (d->dim == 2)
      hipLaunchKernelGGL(k_mlp_features<2>, grid, block, 0, (hipStream_t)stream, U1, U2, n, nm->kind,
                         nm->nu_const, nm->kn, dt, X);
    else
      hipLaunchKernelGGL(k_mlp_features<3>, grid, block, 0, (hipStream_t)stream, U1, U2, n, nm->kind,
                         nm->nu_const, nm->kn, dt, X);
    BGK_HIP(hipGetLastError());
    return BGK_OK;
  });
}

extern "C" int bgk_mlp_targets(const tgs_dag* d, const double* Ut, const double* U1,
                               const double* U2, float* T, bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!d || !Ut || !U1 || !U2 || !T) return fail(BGK_E_INVALID, "null argument");
    const int64_t n = d->n_nodes;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (d->dim == 2)
      hipLaunchKernelGGL(k_mlp_targets<2>, grid, block, 0, (hipStream_t)stream, Ut, U1, U2, n, T);
    else
      hipLaunchKernelGGL(k_mlp_targets<3>, grid, block, 0, (hipStream_t)stream, Ut, U1, U2, n, T);
    BGK_HIP(hipGetLastError());
    return BGK_OK;
  });
}

extern "C" int bgk_mlp_guess(bgk_mlp* m, const tgs_dag* d, const double* U1, const double* U2,
                             const tgs_nu_model* nm, double dt, double* Ug, int32_t* fallback,
                             bgk_stream_t stream) {
  return guarded([&]() -> int {
    if (!m || !d || !U1 || !U2 || !nm || !Ug) return fail(BGK_E_INVALID, "null argument");
    const int64_t n = d->n_nodes;
    const int64_t ntiles = (n + 15) / 16;
    if (d->dim == 2)
      hipLaunchKernelGGL(k_mlp_guess<2>, dim3(grid_tiles(ntiles)), dim3(MLP_THREADS), 0,
                         (hipStream_t)stream, margs(m), U1, U2, n, nm->kind, nm->nu_const, nm->kn,
                         dt, Ug, fallback);
    else
      hipLaunchKernelGGL(k_mlp_guess<3>, dim3(grid_tiles(ntiles)), dim3(MLP_THREADS), 0,
                         (hipStream_t)stream, margs(m), U1, U2, n, nm->kind, nm->nu_const, nm->kn,
                         dt, Ug, fallback);
    BGK_HIP(hipGetLastError());
    return BGK_OK;
  });
}
