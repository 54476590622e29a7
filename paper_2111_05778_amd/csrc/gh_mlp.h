// Neural distance bound on the matrix cores.
//
// f(p) = a_s (||p|| - r0) + a_n NN(gamma(p)) + b      (eq. nnsdb, with a
// sphere prior that places the surface), gamma(p) = [p, sin(w_k p), cos(w_k p)],
// NN = w_out . softplus(W_D ... softplus(W_1 gamma + b_1) ... + b_D) + b_out.
//
// A block of four waves evaluates a tile of points: the features go to LDS,
// every hidden layer is a [rows x K] x [K x W] product on MFMA with FP32
// accumulation, its epilogue adds the bias, applies softplus and writes the
// next layer's input back to LDS, and a final FP32 dot gives NN.  Three
// precisions share the structure:
//   BF16:   v_mfma_f32_32x32x16_bf16, activations stored as bf16, 128 rows
//   BF16x3: the same instruction three times per product on hi/lo bf16
//           splits of activations and weights (hi*hi + hi*lo + lo*hi, FP32
//           accumulation): about 2^-16 relative error, 64 rows
//   FP32:   v_mfma_f32_32x32x2f32,    activations stored as f32,   64 rows
// Weights arrive pre-packed (sdb_describe) in the exact operand order of a
// 32 x 32 B fragment: one 16-byte (bf16) or 4-byte (f32) load per lane.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gh {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int kMlpBlock = 256;
constexpr int kMlpMaxK = 256;           // widest layer input (features pad to <= 112)
constexpr int kBf16Rows = 128, kF32Rows = 64;
constexpr int kBf16Stride = kMlpMaxK + 8;  // bf16 elements per LDS row (16-byte pad)
constexpr int kF32Stride = kMlpMaxK + 1;   // floats per LDS row (odd: no bank conflicts)

enum : int { kPrecF32 = 0, kPrecBf16 = 1, kPrecBf16x3 = 2 };

struct MlpDesc {
  const uint16_t* wb;   // bf16 bits, packed B fragments of every hidden layer
  const uint16_t* wbl;  // bf16 bits of the remainders w - bf16(w), same packing
  const float* wf;      // float, packed B fragments of every hidden layer
  const float* wft;     // float, packed B fragments of W_l itself (l >= 1), for the adjoint
  const float* bias;    // [depth][W]
  const float* wout;    // [W]
  const float* omegas;  // [F]
  int F, W, depth, k1;  // k1 = 3 + 6F features
  int precision;
  float a_s, r0, a_n, b, b_out;
  float eps;            // |f_bf16 - f_fp32| bound used by the hop test
};

// Padded first-layer depth of each precision's K steps.
__host__ __device__ constexpr int mlp_k0(int k1, int prec) { return prec != kPrecF32 ? (k1 + 15) / 16 * 16 : (k1 + 1) / 2 * 2; }
__host__ __device__ constexpr int mlp_kstep(int prec) { return prec != kPrecF32 ? 16 : 2; }
template <int P>
__host__ __device__ constexpr int mlp_rows() { return P == kPrecBf16 ? kBf16Rows : kF32Rows; }
// Elements of the packed fragments of layer l (0 = features -> W).
__host__ __device__ inline size_t mlp_layer_elems(int l, int k1, int W, int prec) {
  const int K = l == 0 ? mlp_k0(k1, prec) : W;
  return (size_t)K * W;
}
__host__ __device__ inline size_t mlp_layer_offset(int l, int k1, int W, int prec) {
  return l == 0 ? 0 : mlp_layer_elems(0, k1, W, prec) + (size_t)(l - 1) * W * W;
}

// LDS of one tile evaluation.  The activation layouts overlay; BF16x3 keeps
// the hi parts in rows [0, 64) and the lo parts in rows [64, 128).
struct MlpSmem {
  union {
    uint16_t ab[kBf16Rows * kBf16Stride];
    float af[kF32Rows * kF32Stride];
  } act;
  float pts[kBf16Rows][3];
  float f[kBf16Rows];
  float part[4][kBf16Rows];
};

__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (values are finite)
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// softplus(z) = max(z, 0) + log(1 + e^-|z|).  The BF16 path rounds the result
// to bf16 right after, so it uses the hardware exp/log; the FP32 path uses
// the accurate library functions.
template <int P>
__device__ __forceinline__ float softplus_t(float z) {
  if constexpr (P == kPrecBf16) {  // rounded to bf16 right after
    return fmaxf(z, 0.f) + __logf(1.f + __expf(-fabsf(z)));
  } else {
    return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));
  }
}

// Wave partition of the rows x W output into 32 x 32 tiles (4 waves).
template <int P, int W>
struct MlpShape {
  static constexpr int kRows = mlp_rows<P>();
  static constexpr int RT = kRows / 32;
  static constexpr int CT = W / 32;
  static constexpr int NC = CT >= 4 ? CT / 4 : 1;
  static constexpr int NR = CT >= 4 ? RT : RT / 2;
  __device__ static int ct0(int w) { return CT >= 4 ? w * NC : (w & 1); }
  __device__ static int rt0(int w) { return CT >= 4 ? 0 : (w >> 1) * NR; }
};

// Stores activation a of (row, col) in the layout of precision P.
template <int P>
__device__ __forceinline__ void act_store(MlpSmem& sm, int row, int col, float a) {
  if constexpr (P == kPrecBf16) {
    sm.act.ab[row * kBf16Stride + col] = f2bf(a);
  } else if constexpr (P == kPrecBf16x3) {
    const uint16_t hi = f2bf(a);
    sm.act.ab[row * kBf16Stride + col] = hi;
    sm.act.ab[(row + kF32Rows) * kBf16Stride + col] = f2bf(a - bf2f(hi));
  } else {
    sm.act.af[row * kF32Stride + col] = a;
  }
}
template <int P>
__device__ __forceinline__ float act_load(const MlpSmem& sm, int row, int col) {
  if constexpr (P == kPrecBf16) {
    return bf2f(sm.act.ab[row * kBf16Stride + col]);
  } else if constexpr (P == kPrecBf16x3) {
    return bf2f(sm.act.ab[row * kBf16Stride + col]) + bf2f(sm.act.ab[(row + kF32Rows) * kBf16Stride + col]);
  } else {
    return sm.act.af[row * kF32Stride + col];
  }
}

// Features of rows [0, nrows) from sm.pts into the activation buffer
// (columns [k1, K0) are zero), then one sync.
template <int P>
__device__ __forceinline__ void mlp_features(const MlpDesc& m, MlpSmem& sm, int nrows) {
  constexpr int kRows = mlp_rows<P>();
  const int K0 = mlp_k0(m.k1, P);
  const int per_row = 3 + 3 * m.F;  // p, then (sin, cos) for each (frequency, axis)
  for (int e = threadIdx.x; e < kRows * per_row; e += blockDim.x) {
    const int r = e / per_row, q = e - r * per_row;
    float v0 = 0.f, v1 = 0.f;
    const int c0 = q < 3 ? q : 3 + 6 * ((q - 3) / 3) + (q - 3) % 3;
    const int c1 = q < 3 ? -1 : c0 + 3;
    if (r < nrows) {
      if (q < 3) v0 = sm.pts[r][q];
      else sincosf(m.omegas[(q - 3) / 3] * sm.pts[r][(q - 3) % 3], &v0, &v1);
    }
    act_store<P>(sm, r, c0, v0);
    if (c1 >= 0) act_store<P>(sm, r, c1, v1);
  }
  for (int e = threadIdx.x; e < kRows * (K0 - m.k1); e += blockDim.x)
    act_store<P>(sm, e / (K0 - m.k1), m.k1 + e % (K0 - m.k1), 0.f);
  __syncthreads();
}

// One hidden layer: act[:, :K] x W_l^T -> bias + softplus -> act[:, :W].
// With zout, the pre-activations are also stored there ([rows][W], FP32).
template <int P, int W>
__device__ __forceinline__ void mlp_layer(const MlpDesc& m, MlpSmem& sm, int l, int nrt, float* zout = nullptr) {
  using S = MlpShape<P, W>;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int K = l == 0 ? mlp_k0(m.k1, P) : W;
  const int ksteps = K / mlp_kstep(P);
  const int ct0 = S::ct0(w), rt0 = S::rt0(w);
  f32x16_t acc[S::NR][S::NC];
#pragma unroll
  for (int rt = 0; rt < S::NR; ++rt)
#pragma unroll
    for (int ct = 0; ct < S::NC; ++ct)
#pragma unroll
      for (int t = 0; t < 16; ++t) acc[rt][ct][t] = 0.f;
  const int row_l = lane & 31, khalf = lane >> 5;
  if constexpr (P != kPrecF32) {
    const size_t off = mlp_layer_offset(l, m.k1, W, P);
    const uint16_t* __restrict__ wl = m.wb + off;
    const uint16_t* __restrict__ wll = m.wbl + off;
    for (int kt = 0; kt < ksteps; ++kt) {
      bf16x8_t bfr[S::NC], bfl[S::NC];
#pragma unroll
      for (int ct = 0; ct < S::NC; ++ct) {
        const size_t o = ((size_t)(kt * S::CT + ct0 + ct) * 64 + lane) * 8;
        bfr[ct] = *reinterpret_cast<const bf16x8_t*>(wl + o);
        if constexpr (P == kPrecBf16x3) bfl[ct] = *reinterpret_cast<const bf16x8_t*>(wll + o);
      }
#pragma unroll
      for (int rt = 0; rt < S::NR; ++rt) {
        if (rt0 + rt >= nrt) break;
        const int arow = (rt0 + rt) * 32 + row_l;
        const bf16x8_t afr =
            *reinterpret_cast<const bf16x8_t*>(&sm.act.ab[arow * kBf16Stride + kt * 16 + khalf * 8]);
        if constexpr (P == kPrecBf16x3) {
          const bf16x8_t afl = *reinterpret_cast<const bf16x8_t*>(
              &sm.act.ab[(arow + kF32Rows) * kBf16Stride + kt * 16 + khalf * 8]);
#pragma unroll
          for (int ct = 0; ct < S::NC; ++ct) {
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afl, bfr[ct], acc[rt][ct], 0, 0, 0);
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr, bfl[ct], acc[rt][ct], 0, 0, 0);
          }
        }
#pragma unroll
        for (int ct = 0; ct < S::NC; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr, bfr[ct], acc[rt][ct], 0, 0, 0);
      }
    }
  } else {
    const float* __restrict__ wl = m.wf + mlp_layer_offset(l, m.k1, W, P);
    for (int kt = 0; kt < ksteps; ++kt) {
      float bfr[S::NC];
#pragma unroll
      for (int ct = 0; ct < S::NC; ++ct) bfr[ct] = wl[(size_t)(kt * S::CT + ct0 + ct) * 64 + lane];
#pragma unroll
      for (int rt = 0; rt < S::NR; ++rt) {
        if (rt0 + rt >= nrt) break;
        const float afr = sm.act.af[((rt0 + rt) * 32 + row_l) * kF32Stride + kt * 2 + khalf];
#pragma unroll
        for (int ct = 0; ct < S::NC; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(afr, bfr[ct], acc[rt][ct], 0, 0, 0);
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
        act_store<P>(sm, row, col, softplus_t<P>(z));
      }
    }
  }
  __syncthreads();
}

// Evaluates f at sm.pts[0, nrows) into sm.f[0, nrows).
template <int P, int W>
__device__ __forceinline__ void mlp_tile(const MlpDesc& m, MlpSmem& sm, int nrows) {
  constexpr int kRows = mlp_rows<P>();
  constexpr int kParts = kMlpBlock / kRows;  // threads per row in the output dot
  const int nrt = (nrows + 31) / 32;
  mlp_features<P>(m, sm, nrows);
  for (int l = 0; l < m.depth; ++l) mlp_layer<P, W>(m, sm, l, nrt);
  const int q = threadIdx.x / kRows, r = threadIdx.x % kRows;
  if (r < nrows) {
    float s = 0.f;
    const int c0 = q * (W / kParts), c1 = c0 + W / kParts;
    for (int c = c0; c < c1; ++c) s += act_load<P>(sm, r, c) * m.wout[c];
    sm.part[q][r] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < nrows) {
    const int rr = threadIdx.x;
    float nn = m.b_out;
    for (int qq = 0; qq < kParts; ++qq) nn += sm.part[qq][rr];
    const float x = sm.pts[rr][0], y = sm.pts[rr][1], z = sm.pts[rr][2];
    const float rad = sqrtf((x * x + y * y) + z * z);
    sm.f[rr] = (m.a_s * (rad - m.r0) + m.a_n * nn) + m.b;
  }
  __syncthreads();
}

}  // namespace gh
