// Neural distance bound on the matrix cores.
//
// f(p) = a_s (||p|| - r0) + a_n NN(gamma(p)) + b      (eq. nnsdb, with a
// sphere prior that places the surface), gamma(p) = [p, sin(w_k p), cos(w_k p)],
// NN = w_out . softplus(W_D ... softplus(W_1 gamma + b_1) ... + b_D) + b_out.
//
// Two evaluators share the tile interface (points in sm.pts, values to sm.f):
//
// bf16 precisions (128 points per block, 32 per wave): the weights are the A
// operand and the activations the B operand of v_mfma_f32_32x32x16_bf16, so a
// wave holds every activation of its 32 points in registers from the
// features to the output dot, with no LDS traffic.  A layer's 32 x 32 output
// tile leaves lane l with 16 features of point l % 32; those registers are
// exactly the next layer's B fragments once the input features of that layer
// are permuted inside each group of 16 (swap of index bits 3 and 2), and
// sdb_describe packs the weights in that permuted order.  The layers work in
// base-2 units (first-layer weights and biases scaled by log2 e, output
// weights by ln 2), so the epilogue adds the bias, applies softplus with the
// hardware exp2/log2 and no multiply, and converts with the hardware bf16
// rounding.
//   BF16:   one product per fragment pair, activations and weights bf16
//   BF16x3: hi/lo bf16 splits of both, hi*hi + hi*lo + lo*hi with FP32
//           accumulation: about 2^-16 relative error
//
// FP32 (64 points per block): activations in LDS, v_mfma_f32_32x32x2f32 with
// the weights as B fragments; used for the FP32 bound, for re-evaluation of
// ambiguous bf16 values, and by the adjoint (which keeps pre-activations).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace gh {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int kMlpBlock = 256;
constexpr int kMlpMaxK = 256;           // widest layer input (features pad to <= 112)
constexpr int kBf16Rows = 128, kF32Rows = 64;
constexpr int kF32Stride = kMlpMaxK + 1;   // floats per LDS row (odd: no bank conflicts)
constexpr int kK0Steps = 7;                // bf16 first layer: 7 k-steps of 16 = 112 inputs
constexpr int kK0Mfma = 16 * kK0Steps;     // (3 + 6F <= 99 features, zero padded)
constexpr int kK0Store = 8;                // k-steps stored for the first layer (the 8th is zero)
constexpr int kChunkSteps = 2;             // k-steps per LDS chunk of A fragments
constexpr int kSpecRowsDefault = 32;       // network hop: rows of a draining tile given out as windows
constexpr int kStageElems = kChunkSteps * (kMlpMaxK / 32) * 512;  // bf16 per chunk buffer (W = 256)

enum : int { kPrecF32 = 0, kPrecBf16 = 1, kPrecBf16x3 = 2 };

struct MlpDesc {
  const uint16_t* wa;   // bf16 bits, packed A fragments of every hidden layer (register evaluator)
  const uint16_t* wal;  // bf16 bits of the remainders w - bf16(w), same packing
  const float* wf;      // float, packed B fragments of every hidden layer
  const float* wft;     // float, packed B fragments of W_l itself (l >= 1), for the adjoint
  const float* bias;    // [depth][W]
  const float* wout;    // [W]
  const float* bias2;   // [depth][W] bias x log2 e (register evaluator: base-2 pre-activations)
  const float* wout2;   // [W] output weights x ln 2 (register evaluator)
  const float* omegas;  // [F]
  const float* omrev;   // [16] w_k / 2pi (turns per unit; zero past F), for the hardware sine
  int F, W, depth, k1;  // k1 = 3 + 6F features
  int precision;
  int relu;             // hidden activation: 0 softplus, 1 ReLU max(z, 0)
  float act_one;        // 1 for softplus, 0 for ReLU (act_hw, act_f32)
  int split;            // tiles with few rows: 1 never split, 2 split <= 32 rows, 3 also <= 64 rows
  float a_s, r0, a_n, b, b_out;
  float eps;            // |f_bf16 - f_fp32| bound used by the hop test
  int hop_shrink;       // bf16 hop: 0 FP32 values for ambiguous steps, 1 steps of floor(max(|f| - eps, 0)/h)
  float eps3;           // plain bf16: |f_bf16x3 - f_fp32| bound for two-step corner certification (0: none)
  float off;            // plain bf16: offset subtracted from every plain bf16 value (0 elsewhere)
  int pool_tiles;       // network hop: ray slots of a block, in tiles (launch shape)
  int spec_rows;        // network hop: rows of a draining tile given out as windows ahead of the rays
};

// Input feature of a hidden layer (l >= 1) that sits in slot q (0..15) of a
// 16-wide k-step of the register evaluator: bits 3 and 2 of q swap places.
__host__ __device__ constexpr int mlpa_slot_feature(int q) {
  return (((q >> 2) & 1) << 3) | (((q >> 3) & 1) << 2) | (q & 3);
}
// Offset (bf16 elements) of layer l's A fragments: [k-step][m-tile][lane][8].
__host__ __device__ inline size_t mlpa_layer_offset(int l, int W) {
  return l == 0 ? 0 : (size_t)16 * kK0Store * W + (size_t)(l - 1) * W * W;
}

// FP32 evaluator: padded first-layer depth (k-steps of 2) and fragment offsets.
__host__ __device__ constexpr int mlp_k0(int k1) { return (k1 + 1) / 2 * 2; }
template <int P>
__host__ __device__ constexpr int mlp_rows() { return P == kPrecF32 ? kF32Rows : kBf16Rows; }
__host__ __device__ inline size_t mlp_layer_elems(int l, int k1, int W) {
  const int K = l == 0 ? mlp_k0(k1) : W;
  return (size_t)K * W;
}
__host__ __device__ inline size_t mlp_layer_offset(int l, int k1, int W) {
  return l == 0 ? 0 : mlp_layer_elems(0, k1, W) + (size_t)(l - 1) * W * W;
}

// LDS of one tile evaluation: FP32 activations (FP32 evaluator) or, in the
// same bytes, two chunk buffers of A fragments with their lo parts (register
// evaluator); the activation exchange of split tiles; the points and values
// of up to 128 rows; partial output dots.
struct MlpSmem {
  union {
    float af[kF32Rows * kF32Stride];
    uint16_t stage[2][2][kStageElems];
  };
  uint4 xch[2][2][kMlpMaxK / 16][64];  // split tiles: B fragments [group][hi/lo][k-step][lane]
  float pts[kBf16Rows][3];
  float f[kBf16Rows];
  float part[4][kBf16Rows];
};

// The plain bf16 register evaluator's part alone (hi fragments only, no FP32
// activations): about half of MlpSmem, so that two blocks fit one CU, for
// kernels that never run the FP32 or the split evaluator.
struct MlpSmemBf16 {
  uint16_t stage[2][1][kStageElems];
  uint4 xch[2][1][kMlpMaxK / 16][64];
  float pts[kBf16Rows][3];
  float f[kBf16Rows];
  float part[4][kBf16Rows];
};

// Resident weights for a small plain bf16 network: every layer's A fragments
// held in LDS for the whole kernel (no chunk copies, no per-chunk waits or
// barriers), with the points and values of a tile; at most 72 KB, so two
// blocks share a CU.  Tiles are never split (no exchange).  The first
// layer's zero k-step is not copied.
constexpr int kResidentW = 64;
constexpr int kResidentBytes = 70 * 1024;
struct MlpSmemRes {
  uint4 wres[kResidentBytes / 16];
  float pts[kBf16Rows][3];
  float f[kBf16Rows];
};
// The same layout for a ReLU network: its kernels apply max(z, 0) alone
// (bit-identical to the shared activation with c = 0, without the log term
// that c = 0 discards).
struct MlpSmemResRelu : MlpSmemRes {};
template <class Sm>
__host__ __device__ constexpr bool mlp_resident_layout() {
  return std::is_base_of_v<MlpSmemRes, Sm>;
}
// Offset (bf16 elements) of layer l's fragments in the resident copy, and
// the bytes of a network of the given depth.
__host__ __device__ constexpr size_t mlpr_layer_offset(int l, int W) {
  return l == 0 ? 0 : (size_t)16 * kK0Steps * W + (size_t)(l - 1) * W * W;
}
__host__ __device__ constexpr bool mlp_resident_fits(int depth, int W) {
  return W == kResidentW && depth >= 1 && mlpr_layer_offset(depth, W) * 2 <= (size_t)kResidentBytes;
}

// On the lean layout the widest network runs every tile split over two or
// more waves per group (at most 64 rows), so that a wave holds half of a
// layer's accumulators and two waves fit one SIMD.
template <int W, class Sm>
__host__ __device__ constexpr bool mlp_split_only() {
  return std::is_same_v<Sm, MlpSmemBf16> && W == kMlpMaxK;
}
template <int P, int W, class Sm>
__host__ __device__ constexpr int mlp_tile_rows() {
  return mlp_split_only<W, Sm>() ? 64 : (P == kPrecF32 ? kF32Rows : kBf16Rows);
}

// The FP32 evaluator's part alone (for kernels that never run the register
// evaluator).
struct MlpSmemF32 {
  float af[kF32Rows * kF32Stride];
  float pts[kBf16Rows][3];
  float f[kBf16Rows];
  float part[4][kBf16Rows];
};

// softplus(z) = max(z, 0) + log(1 + e^-|z|) with the accurate library
// functions (FP32 evaluator).
__device__ __forceinline__ float softplus_f32(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }

// Hidden-layer activation of the bf16 evaluators on a base-2 pre-activation
// z' = z log2 e (the weights are scaled for it, see sdb_describe):
// u = max(z', 0) + c log2(1 + 2^-|z'|) with the hardware base-2 exponential
// and logarithm (about 1 ulp each, far below the bf16 roundings that follow)
// is softplus(z) / ln 2 for c = 1 and ReLU(z) / ln 2 for c = 0 (the log term
// is finite, so c = 0 leaves max(z', 0) exactly).  One instruction stream
// for both: a branch on the activation here measurably slowed the softplus
// networks.
__device__ __forceinline__ float act_hw(float z, float c) {
  const float e = __builtin_amdgcn_exp2f(-fabsf(z));
  return fmaf(__builtin_amdgcn_logf(1.f + e), c, fmaxf(z, 0.f));
}

// act_hw for c = 0 without the log term: max(z, 0) + (+0), the same bits
// (the product of the finite log term and 0 is +0, which also turns -0 into
// +0).
__device__ __forceinline__ float act_relu(float z) { return fmaf(0.f, 0.f, fmaxf(z, 0.f)); }

// The same for the FP32 evaluator: max(z, 0) + c log(1 + e^-|z|), softplus
// for c = 1 (1 x is exact), ReLU for c = 0.
__device__ __forceinline__ float act_f32(float z, float c) { return fmaxf(z, 0.f) + c * log1pf(expf(-fabsf(z))); }

// Final value from NN (both evaluators).
__device__ __forceinline__ float mlp_value(const MlpDesc& m, float x, float y, float z, float nn) {
  const float rad = sqrtf((x * x + y * y) + z * z);
  return (m.a_s * (rad - m.r0) + m.a_n * nn) + m.b;
}

// =========================================================== FP32 evaluator
// Wave partition of the 64 x W output into 32 x 32 tiles (4 waves).
template <int W>
struct MlpShape {
  static constexpr int RT = kF32Rows / 32;
  static constexpr int CT = W / 32;
  static constexpr int NC = CT >= 4 ? CT / 4 : 1;
  static constexpr int NR = CT >= 4 ? RT : RT / 2;
  __device__ static int ct0(int w) { return CT >= 4 ? w * NC : (w & 1); }
  __device__ static int rt0(int w) { return CT >= 4 ? 0 : (w >> 1) * NR; }
};

// Features of rows [0, nrows) from sm.pts into the activation buffer
// (columns [k1, K0) are zero), then one sync.
template <class Sm>
__device__ __forceinline__ void mlp_features_f32(const MlpDesc& m, Sm& sm, int nrows) {
  const int K0 = mlp_k0(m.k1);
  const int per_row = 3 + 3 * m.F;  // p, then (sin, cos) for each (frequency, axis)
  for (int e = threadIdx.x; e < kF32Rows * per_row; e += blockDim.x) {
    const int r = e / per_row, q = e - r * per_row;
    float v0 = 0.f, v1 = 0.f;
    const int c0 = q < 3 ? q : 3 + 6 * ((q - 3) / 3) + (q - 3) % 3;
    const int c1 = q < 3 ? -1 : c0 + 3;
    if (r < nrows) {
      if (q < 3) v0 = sm.pts[r][q];
      else sincosf(m.omegas[(q - 3) / 3] * sm.pts[r][(q - 3) % 3], &v0, &v1);
    }
    sm.af[r * kF32Stride + c0] = v0;
    if (c1 >= 0) sm.af[r * kF32Stride + c1] = v1;
  }
  for (int e = threadIdx.x; e < kF32Rows * (K0 - m.k1); e += blockDim.x)
    sm.af[(e / (K0 - m.k1)) * kF32Stride + m.k1 + e % (K0 - m.k1)] = 0.f;
  __syncthreads();
}

// One hidden layer: act[:, :K] x W_l^T -> bias + softplus -> act[:, :W].
// With zout, the pre-activations are also stored there ([rows][W], FP32).
template <int W, class Sm>
__device__ __forceinline__ void mlp_layer_f32(const MlpDesc& m, Sm& sm, int l, int nrt, float* zout = nullptr) {
  using S = MlpShape<W>;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int K = l == 0 ? mlp_k0(m.k1) : W;
  const int ksteps = K / 2;
  const int ct0 = S::ct0(w), rt0 = S::rt0(w);
  f32x16_t acc[S::NR][S::NC];
#pragma unroll
  for (int rt = 0; rt < S::NR; ++rt)
#pragma unroll
    for (int ct = 0; ct < S::NC; ++ct)
#pragma unroll
      for (int t = 0; t < 16; ++t) acc[rt][ct][t] = 0.f;
  const int row_l = lane & 31, khalf = lane >> 5;
  const float* __restrict__ wl = m.wf + mlp_layer_offset(l, m.k1, W);
  // U k-steps per group: their weight loads are all in flight before the
  // group's products, so the products wait for memory once per group.
  constexpr int U = 8;
  for (int kt0 = 0; kt0 < ksteps; kt0 += U) {
    float bfr[U][S::NC];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kt = kt0 + u < ksteps ? kt0 + u : ksteps - 1;  // in bounds; unused past the end
#pragma unroll
      for (int ct = 0; ct < S::NC; ++ct) bfr[u][ct] = wl[(size_t)(kt * S::CT + ct0 + ct) * 64 + lane];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kt = kt0 + u;
      if (kt >= ksteps) break;
#pragma unroll
      for (int rt = 0; rt < S::NR; ++rt) {
        if (rt0 + rt >= nrt) break;
        const float afr = sm.af[((rt0 + rt) * 32 + row_l) * kF32Stride + kt * 2 + khalf];
#pragma unroll
        for (int ct = 0; ct < S::NC; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(afr, bfr[u][ct], acc[rt][ct], 0, 0, 0);
      }
    }
  }
  __syncthreads();  // every wave has read this layer's input
  const float* __restrict__ bias = m.bias + (size_t)l * W;
#pragma unroll
  for (int rt = 0; rt < S::NR; ++rt) {
    if (rt0 + rt >= nrt) break;
#pragma unroll
    for (int ct = 0; ct < S::NC; ++ct) {
      const int col = (ct0 + ct) * 32 + (lane & 31);
      const float bv = bias[col];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int row = (rt0 + rt) * 32 + 8 * (t >> 2) + 4 * (lane >> 5) + (t & 3);
        const float z = acc[rt][ct][t] + bv;
        if (zout) zout[row * W + col] = z;
        sm.af[row * kF32Stride + col] = act_f32(z, m.act_one);
      }
    }
  }
  __syncthreads();
}

template <int W, class Sm>
__device__ __forceinline__ void mlp_tile_f32(const MlpDesc& m, Sm& sm, int nrows) {
  constexpr int kParts = kMlpBlock / kF32Rows;  // threads per row in the output dot
  const int nrt = (nrows + 31) / 32;
  mlp_features_f32(m, sm, nrows);
  for (int l = 0; l < m.depth; ++l) mlp_layer_f32<W>(m, sm, l, nrt);
  const int q = threadIdx.x / kF32Rows, r = threadIdx.x % kF32Rows;
  if (r < nrows) {
    float s = 0.f;
    const int c0 = q * (W / kParts), c1 = c0 + W / kParts;
    for (int c = c0; c < c1; ++c) s += sm.af[r * kF32Stride + c] * m.wout[c];
    sm.part[q][r] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < nrows) {
    const int rr = threadIdx.x;
    float nn = m.b_out;
    for (int qq = 0; qq < kParts; ++qq) nn += sm.part[qq][rr];
    sm.f[rr] = mlp_value(m, sm.pts[rr][0], sm.pts[rr][1], sm.pts[rr][2], nn);
  }
  __syncthreads();
}

// ====================================================== register evaluator
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  const bf16x2_t v = {(__bf16)a, (__bf16)b};  // hardware round to nearest even
  return __builtin_bit_cast(uint32_t, v);
}

// Eight activations into a B fragment (and, for BF16x3, the fragment of the
// remainders a - bf16(a)).
template <int P>
__device__ __forceinline__ void pack_fragment(const float (&a)[8], bf16x8_t& hi, bf16x8_t& lo) {
  uint32_t h[4], r[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    h[i] = pack_bf16x2(a[2 * i], a[2 * i + 1]);
    if constexpr (P == kPrecBf16x3) {
      const float h0 = __uint_as_float(h[i] << 16), h1 = __uint_as_float(h[i] & 0xffff0000u);
      r[i] = pack_bf16x2(a[2 * i] - h0, a[2 * i + 1] - h1);
    }
  }
  hi = __builtin_bit_cast(bf16x8_t, h);
  if constexpr (P == kPrecBf16x3) lo = __builtin_bit_cast(bf16x8_t, r);
}

template <int P>
__device__ __forceinline__ f32x16_t mfma_step(const bf16x8_t& a, const bf16x8_t& al, const bf16x8_t& b,
                                              const bf16x8_t& bl, f32x16_t acc) {
  if constexpr (P == kPrecBf16x3) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bl, acc, 0, 0, 0);
  }
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
}

// Bias + activation of one layer's output tiles c0 .. c0 + NT - 1 (this
// wave's share); either packs them as B fragments of the next layer's
// k-steps 2(c0 + c) and 2(c0 + c) + 1 into x[2c], x[2c + 1], or, for the
// last hidden layer, returns this lane's
// part of the output dot.  Lane l holds feature 32c + 8j + 4(l / 32) + i of
// its point in acc[c - c0][4j + i].  The bias (and output weights) of the
// next tile are loaded while a tile is processed, and a scheduling barrier
// per tile keeps the compiler from hoisting every load of the layer (which
// would cost registers instead of latency).
template <int P, int W, int NT, bool kLast, bool kRelu = false>
__device__ __forceinline__ float mlp_epilogue(const MlpDesc& m, int l, int c0, f32x16_t (&acc)[NT],
                                              bf16x8_t (&x)[2 * NT], bf16x8_t (&xl)[2 * NT]) {
  const int h = (threadIdx.x >> 5) & 1;
  const float4* __restrict__ bias4 = reinterpret_cast<const float4*>(m.bias2 + (size_t)l * W) + h;
  const float4* __restrict__ wout4 = reinterpret_cast<const float4*>(m.wout2) + h;
  float dt[NT];  // per-tile output dots (kLast)
  float4 bv[4], wv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    bv[j] = bias4[8 * c0 + 2 * j];
    if constexpr (kLast) wv[j] = wout4[8 * c0 + 2 * j];
  }
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    float a[16];
    float dot = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[4 * j + 0] = kRelu ? act_relu(acc[c][4 * j + 0] + bv[j].x) : act_hw(acc[c][4 * j + 0] + bv[j].x, m.act_one);
      a[4 * j + 1] = kRelu ? act_relu(acc[c][4 * j + 1] + bv[j].y) : act_hw(acc[c][4 * j + 1] + bv[j].y, m.act_one);
      a[4 * j + 2] = kRelu ? act_relu(acc[c][4 * j + 2] + bv[j].z) : act_hw(acc[c][4 * j + 2] + bv[j].z, m.act_one);
      a[4 * j + 3] = kRelu ? act_relu(acc[c][4 * j + 3] + bv[j].w) : act_hw(acc[c][4 * j + 3] + bv[j].w, m.act_one);
      if constexpr (kLast) {
        dot += a[4 * j + 0] * wv[j].x;
        dot += a[4 * j + 1] * wv[j].y;
        dot += a[4 * j + 2] * wv[j].z;
        dot += a[4 * j + 3] * wv[j].w;
      }
    }
    dt[c] = dot;
    if (c + 1 < NT) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bv[j] = bias4[8 * (c0 + c + 1) + 2 * j];
        if constexpr (kLast) wv[j] = wout4[8 * (c0 + c + 1) + 2 * j];
      }
    }
    if constexpr (!kLast) {
      float a0[8], a1[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        a0[i] = a[i];
        a1[i] = a[8 + i];
      }
      pack_fragment<P>(a0, x[2 * c], xl[2 * c]);
      pack_fragment<P>(a1, x[2 * c + 1], xl[2 * c + 1]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  if constexpr (!kLast) return 0.f;
  // Tile dots of the whole point (both lane halves), then a pairwise tree
  // over the tiles: the same association for every split of the tiles over
  // waves, so a value does not depend on how full its tile was.
#pragma unroll
  for (int c = 0; c < NT; ++c) dt[c] += __shfl_xor(dt[c], 32, 64);
#pragma unroll
  for (int span = 1; span < NT; span *= 2)
#pragma unroll
    for (int c = 0; c + span < NT; c += 2 * span) dt[c] += dt[c + span];
  return dt[0];
}

// Features of k-step s of the first layer: slot 8h + i holds feature
// 16s + 8h + i of gamma(p) = [p, then per frequency sin(w p_x..z), cos(w p_x..z)],
// zero past 3 + 6F.  One hardware sine per feature (cos = sin + 1/4 turn).
// s is a constant once the caller's loop is unrolled.
template <int P>
__device__ __forceinline__ void mlp_features_reg(const MlpDesc& m, int s, float px, float py, float pz, bf16x8_t& x,
                                                 bf16x8_t& xl) {
  const int h = (threadIdx.x >> 5) & 1;
  float v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    float arg[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = 16 * s + 8 * q + i;
      if (k < 3) {
        arg[q] = k == 0 ? px : (k == 1 ? py : pz);
      } else {
        const int j = k - 3, fq = j / 6, r = j % 6, ax = r % 3;
        const float pa = ax == 0 ? px : (ax == 1 ? py : pz);
        arg[q] = fmaf(m.omrev[fq < 16 ? fq : 15], pa, r >= 3 ? 0.25f : 0.f);  // turns
      }
    }
    const float u = h ? arg[1] : arg[0];
    const bool lin = 16 * s + i < 3 && h == 0;
    v[i] = lin ? u : (16 * s + 8 * h + i < m.k1 ? __builtin_amdgcn_sinf(u) : 0.f);  // sin(2 pi u)
  }
  pack_fragment<P>(v, x, xl);
}

// A fragments stream through LDS in chunks of kChunkSteps k-steps (all
// m-tiles), double-buffered: while the waves multiply with one buffer, the
// next chunk (possibly the next layer's first) travels from global memory
// straight into the other buffer (global_load_lds, no registers); one wait
// and one barrier per chunk.
template <int P, int W>
struct ChunkDma {
  static constexpr int kPieces = kChunkSteps * (W / 32) / 4;  // 16-byte pieces per thread per part
  // Issues the copy of one chunk (hi and, for BF16x3, lo parts) into buffer buf.
  template <class Sm>
  __device__ static void issue(const uint16_t* __restrict__ ghi, const uint16_t* __restrict__ glo, Sm& sm,
                               int buf) {
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kPieces; ++q) {
      const int piece = threadIdx.x + q * kMlpBlock;  // lane l of wave w lands at (64w + 256q + l) * 16 bytes
      const int wave_base = (64 * w + q * kMlpBlock) * 8;
      __builtin_amdgcn_global_load_lds(ghi + (size_t)piece * 8,
                                       (__attribute__((address_space(3))) void*)&sm.stage[buf][0][wave_base], 16, 0, 0);
      if constexpr (P == kPrecBf16x3)
        __builtin_amdgcn_global_load_lds(glo + (size_t)piece * 8,
                                         (__attribute__((address_space(3))) void*)&sm.stage[buf][1][wave_base], 16, 0,
                                         0);
    }
  }
  // Waits for this thread's copies, then for the whole block.
  __device__ static void wait_and_sync() {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
  }
};

// One layer's products over NS input k-steps for this wave's NT m-tiles
// c0 .. c0 + NT - 1; its chunks start in buffer 0 (the number of chunks is
// even, so the next layer starts in buffer 0 too).  next_hi/next_lo: the
// following layer's fragments, copied during this layer's last chunk, or
// null.  Every wave of the block runs the same copies and barriers; with
// kActive false a wave only helps with the copies.  For the first layer
// (kFeat) the B fragments are the features, computed chunk by chunk.
template <int P, int W, int NT, int NS, bool kFeat, bool kActive, class Sm>
__device__ __forceinline__ void mlp_layer_reg(const MlpDesc& m, Sm& sm, int c0, const uint16_t* __restrict__ hi,
                                              const uint16_t* __restrict__ lo, const uint16_t* __restrict__ next_hi,
                                              const uint16_t* __restrict__ next_lo, f32x16_t (&acc)[NT],
                                              const bf16x8_t (&x)[W / 16], const bf16x8_t (&xl)[W / 16], float px,
                                              float py, float pz, size_t roff = 0) {
  constexpr int CT = W / 32;
  constexpr int NCH = (NS + kChunkSteps - 1) / kChunkSteps;
  constexpr int CE = kChunkSteps * CT * 512;  // bf16 elements per chunk
  static_assert(NCH % 2 == 0, "layers must have an even number of chunks");
  // resident weights: the layer's fragments sit in LDS at roff (bf16
  // elements) for the whole kernel, so nothing is copied or waited for
  constexpr bool kRes = mlp_resident_layout<Sm>();
  const int lane = threadIdx.x & 63;
  if constexpr (kActive) {
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int t = 0; t < 16; ++t) acc[c][t] = 0.f;
  }
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int cur = ch & 1;
    if constexpr (!kRes) {
      if (ch + 1 < NCH) ChunkDma<P, W>::issue(hi + (size_t)(ch + 1) * CE, lo + (size_t)(ch + 1) * CE, sm, cur ^ 1);
      else if (next_hi) ChunkDma<P, W>::issue(next_hi, next_lo, sm, cur ^ 1);
    }
    __builtin_amdgcn_sched_barrier(0);  // the copy starts before this chunk's products
    if constexpr (kActive) {
      const bf16x8_t* __restrict__ sa;
      if constexpr (kRes) sa = reinterpret_cast<const bf16x8_t*>(sm.wres) + (roff + (size_t)ch * CE) / 8;
      else sa = reinterpret_cast<const bf16x8_t*>(sm.stage[cur][0]);
      const bf16x8_t* __restrict__ sal = sa;  // the lo parts (BF16x3 only)
      if constexpr (P == kPrecBf16x3) sal = reinterpret_cast<const bf16x8_t*>(sm.stage[cur][1]);
      // Read the fragments of FS k-steps at once, then multiply: the reads
      // return in order, so each product waits only for its own fragment.
      constexpr int FS = P == kPrecBf16x3 || mlp_split_only<W, Sm>() ? 1 : kChunkSteps;
#pragma unroll
      for (int u0 = 0; u0 < kChunkSteps; u0 += FS) {
        bf16x8_t fa[FS][NT], fl[FS][NT];
#pragma unroll
        for (int u = 0; u < FS; ++u) {
          if (ch * kChunkSteps + u0 + u >= NS) break;
#pragma unroll
          for (int c = 0; c < NT; ++c) {
            const int o = ((u0 + u) * CT + c0 + c) * 64 + lane;
            fa[u][c] = sa[o];
            if constexpr (P == kPrecBf16x3) fl[u][c] = sal[o];
          }
        }
#pragma unroll
        for (int u = 0; u < FS; ++u) {
          const int s = ch * kChunkSteps + u0 + u;
          if (s >= NS) break;
          bf16x8_t xb, xbl;
          if constexpr (kFeat) {
            mlp_features_reg<P>(m, s, px, py, pz, xb, xbl);
          } else {
            xb = x[s];
            if constexpr (P == kPrecBf16x3) xbl = xl[s];
          }
#pragma unroll
          for (int c = 0; c < NT; ++c) acc[c] = mfma_step<P>(fa[u][c], fl[u][c], xb, xbl, acc[c]);
        }
        // Scheduling order of this group: every fragment read, then the
        // products (the compiler would otherwise serialise read -> wait ->
        // product to save registers).
        constexpr int kParts = P == kPrecBf16x3 ? 2 : 1;
        __builtin_amdgcn_sched_group_barrier(0x100, FS * NT * kParts, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, FS * NT * (P == kPrecBf16x3 ? 3 : 1), 0);
      }
    }
    __builtin_amdgcn_sched_barrier(0);  // and is waited for only after them
    if constexpr (!kRes) ChunkDma<P, W>::wait_and_sync();
  }
}

// Copies every layer's bf16 A fragments of the network into the resident
// layout (the first layer without its zero k-step), then synchronises.
template <int W>
__device__ __forceinline__ void mlp_load_resident(const MlpDesc& m, MlpSmemRes& sm) {  // either resident layout
  const size_t n0 = mlpr_layer_offset(1, W) / 8, nh = (mlpr_layer_offset(m.depth, W) - mlpr_layer_offset(1, W)) / 8;
  const uint4* __restrict__ g0 = reinterpret_cast<const uint4*>(m.wa);
  const uint4* __restrict__ g1 = reinterpret_cast<const uint4*>(m.wa + mlpa_layer_offset(1, W));
  for (size_t i = threadIdx.x; i < n0; i += blockDim.x) sm.wres[i] = g0[i];
  for (size_t i = threadIdx.x; i < nh; i += blockDim.x) sm.wres[n0 + i] = g1[i];
  __syncthreads();
}

// Hands this wave's new B fragments (tiles c0 .. c0 + NT - 1) to the other
// waves of its group through LDS and takes theirs (S > 1 only).  The chunk
// barriers of the following layer keep the next exchange from overwriting
// the buffer before every wave has read it.
template <int P, int W, int NT, class Sm>
__device__ __forceinline__ void mlp_exchange(Sm& sm, int grp, int c0, const bf16x8_t (&xo)[2 * NT],
                                             const bf16x8_t (&xol)[2 * NT], bf16x8_t (&x)[W / 16],
                                             bf16x8_t (&xl)[W / 16]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < 2 * NT; ++q) {
    sm.xch[grp][0][2 * c0 + q][lane] = __builtin_bit_cast(uint4, xo[q]);
    if constexpr (P == kPrecBf16x3) sm.xch[grp][1][2 * c0 + q][lane] = __builtin_bit_cast(uint4, xol[q]);
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < W / 16; ++s) {
    x[s] = __builtin_bit_cast(bf16x8_t, sm.xch[grp][0][s][lane]);
    if constexpr (P == kPrecBf16x3) xl[s] = __builtin_bit_cast(bf16x8_t, sm.xch[grp][1][s][lane]);
  }
}

// Part of NN(gamma(p)) of the group's 32 points that this wave computes: the
// S waves of a group (waves w with equal w / S) share its points, each taking
// W/32/S of the m-tiles of every layer.  Lanes l and l + 32 both pass point
// l % 32 and both receive its part.  Every wave of the block must call it
// with the same S (barriers inside), active or not.
template <int P, int W, int S, bool kActive, class Sm>
__device__ __forceinline__ float mlp_wave(const MlpDesc& m, Sm& sm, float px, float py, float pz) {
  constexpr int KS = W / 16, NT = W / 32 / S;
  constexpr bool kRelu = std::is_same_v<Sm, MlpSmemResRelu>;
  const int w = threadIdx.x >> 6;
  const int grp = w / S, c0 = (w % S) * NT;
  f32x16_t acc[NT];
  bf16x8_t x[KS], xl[KS];
  {
    if constexpr (!mlp_resident_layout<Sm>()) {
      ChunkDma<P, W>::issue(m.wa, m.wal, sm, 0);
      ChunkDma<P, W>::wait_and_sync();
    }
    const size_t on = mlpa_layer_offset(1, W);
    const bool deeper = m.depth > 1;
    mlp_layer_reg<P, W, NT, kK0Steps, true, kActive>(m, sm, c0, m.wa, m.wal, deeper ? m.wa + on : nullptr,
                                                     deeper ? m.wal + on : nullptr, acc, x, xl, px, py, pz,
                                                     mlpr_layer_offset(0, W));
  }
  float dot = 0.f;
  for (int l = 0;; ++l) {
    if (l + 1 == m.depth) {
      bf16x8_t xo[2 * NT], xol[2 * NT];  // unused by the last layer
      if constexpr (kActive) dot = mlp_epilogue<P, W, NT, true, kRelu>(m, l, c0, acc, xo, xol);
      break;
    }
    if constexpr (S == 1) {
      if constexpr (kActive) mlp_epilogue<P, W, NT, false, kRelu>(m, l, c0, acc, x, xl);
    } else {
      bf16x8_t xo[2 * NT], xol[2 * NT];
      if constexpr (kActive) mlp_epilogue<P, W, NT, false, kRelu>(m, l, c0, acc, xo, xol);
      mlp_exchange<P, W, NT>(sm, grp, c0, xo, xol, x, xl);
    }
    const size_t o = mlpa_layer_offset(l + 1, W), on = mlpa_layer_offset(l + 2, W);
    const bool deeper = l + 2 < m.depth;
    mlp_layer_reg<P, W, NT, KS, false, kActive>(m, sm, c0, m.wa + o, m.wal + o, deeper ? m.wa + on : nullptr,
                                                deeper ? m.wal + on : nullptr, acc, x, xl, px, py, pz,
                                                mlpr_layer_offset(l + 1, W));
  }
  return dot;
}

// Tile of nrows points with S waves per group of 32 points (4 / S groups).
template <int P, int W, int S, class Sm>
__device__ __forceinline__ void mlp_tile_split(const MlpDesc& m, Sm& sm, int nrows) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = w / S;
  const int row = 32 * grp + (lane & 31);
  const bool active = 32 * grp < nrows;  // wave-uniform
  const int rr = row < nrows ? row : 32 * grp;  // idle lanes evaluate a valid point
  float x = 0.f, y = 0.f, z = 0.f, part = 0.f;
  if (active) {
    x = sm.pts[rr][0];
    y = sm.pts[rr][1];
    z = sm.pts[rr][2];
    part = mlp_wave<P, W, S, true>(m, sm, x, y, z);
  } else {
    (void)mlp_wave<P, W, S, false>(m, sm, 0.f, 0.f, 0.f);
  }
  // plain bf16 values drop the measured offset of their error (exact for 0)
  const float off = P == kPrecBf16 ? m.off : 0.f;
  if constexpr (S == 1) {
    if (active && lane < 32 && row < nrows) sm.f[row] = mlp_value(m, x, y, z, m.b_out + part) - off;
  } else {
    if (active && lane < 32) sm.part[w % S][row] = part;
    __syncthreads();
    if (active && (w % S) == 0 && lane < 32 && row < nrows) {
      float p[S];
#pragma unroll
      for (int q = 0; q < S; ++q) p[q] = sm.part[q][row];
#pragma unroll
      for (int span = 1; span < S; span *= 2)  // the same pairwise tree as within a wave
#pragma unroll
        for (int q = 0; q + span < S; q += 2 * span) p[q] += p[q + span];
      sm.f[row] = mlp_value(m, x, y, z, m.b_out + p[0]) - off;
    }
  }
  __syncthreads();
}

// A tile with few rows spreads each group's layers over more waves: the
// round takes about as long as the largest share of one wave.
template <int P, int W, class Sm>
__device__ __forceinline__ void mlp_tile_reg(const MlpDesc& m, Sm& sm, int nrows) {
  constexpr int kS4 = W / 32 >= 4 ? 4 : W / 32;  // at least one m-tile per wave
  if constexpr (mlp_resident_layout<Sm>()) {
    mlp_tile_split<P, W, 1>(m, sm, nrows);  // resident weights: no exchange buffer
  } else if constexpr (mlp_split_only<W, Sm>()) {
    // nrows <= 64: every layer is split over two or four waves per group
    if (m.split >= 2 && nrows <= 32) mlp_tile_split<P, W, kS4>(m, sm, nrows);
    else mlp_tile_split<P, W, 2>(m, sm, nrows);
  } else {
    if (m.split >= 2 && nrows <= 32) mlp_tile_split<P, W, kS4>(m, sm, nrows);
    else if (m.split >= 3 && nrows <= 64) mlp_tile_split<P, W, 2>(m, sm, nrows);
    else mlp_tile_split<P, W, 1>(m, sm, nrows);
  }
}

// Evaluates f at sm.pts[0, nrows) into sm.f[0, nrows) (nrows <= mlp_rows<P>);
// sm.pts must be visible to the block (synchronised) before the call.
template <int P, int W, class Sm>
__device__ __forceinline__ void mlp_tile(const MlpDesc& m, Sm& sm, int nrows) {
  if constexpr (P == kPrecF32) mlp_tile_f32<W>(m, sm, nrows);
  else mlp_tile_reg<P, W>(m, sm, nrows);
}

// LDS of a kernel evaluating in precision P: the FP32-only layout when no
// bf16 tile runs (it leaves room for two blocks per CU).
template <int P>
using MlpSmemFor = std::conditional_t<P == kPrecF32, MlpSmemF32, MlpSmem>;

}  // namespace gh
