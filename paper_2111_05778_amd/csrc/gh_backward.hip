// Adjoint of a vertex loss with respect to the network parameters.
//
// A vertex on lattice edge a -> b (axis e) sits at P_a + t h e with
// t = f_a/(f_a - f_b), so dt/df_a = -f_b/(f_a - f_b)^2 and
// dt/df_b = f_a/(f_a - f_b)^2.  The cotangent of corner value f_c gathers
// (dL/dv . e) h dt/df_c over the (at most six) crossing edges through c, in
// a fixed order.  With f = a_s(||p|| - r0) + a_n NN + b, dL/dtheta =
// a_n sum_c gbar_c dNN(P_c)/dtheta: a tiled FP32 back-propagation through
// the network on the matrix cores.  Every sum runs in a fixed order (tiles
// block-strided, per-block partial gradients, then a reduction over blocks in
// block order), so the result is deterministic.

#include "gh_device.h"
#include "gh_launch.h"
#include "gh_layout.h"
#include "gh_mlp.h"

namespace gh {

constexpr int kVjpRows = kF32Rows;  // 64 corners per tile

// ----------------------------------------------------------- cotangents
__device__ __forceinline__ float corner_cotangent(const Workspace& ws, const Grid& g, size_t nl, int64_t ci,
                                                  int64_t m, const float* __restrict__ dldv) {
  const int n = g.n, n1 = n + 1;
  const int L = ws.cl[ci], k = ws.ck[ci];
  const int a = L / n1, b = L - a * n1;
  const float fc = ws.cf[ci];
  const uint32_t info = ws.cinfo[ci];
  const unsigned msk = cinfo_mask(info);
  const int64_t vb = cinfo_vbase(info);
  float s = 0.f;
  // c is the lower end a of its own crossing edges: dt/df_a = -f_b/(f_a - f_b)^2
  if (msk & 1u) {
    const float fb = ws.cf[corner_index(ws, nl, (size_t)L + n1, k)];
    const float d = fc - fb;
    s += dldv[3 * vb + 0] * g.h * (-fb / (d * d));
  }
  if (msk & 2u) {
    const float fb = ws.cf[corner_index(ws, nl, (size_t)L + 1, k)];
    const float d = fc - fb;
    s += dldv[3 * (vb + (msk & 1u)) + 1] * g.h * (-fb / (d * d));
  }
  if (msk & 4u) {
    const float fb = ws.cf[ci + 1];
    const float d = fc - fb;
    s += dldv[3 * (vb + __popc(msk & 3u)) + 2] * g.h * (-fb / (d * d));
  }
  // c is the upper end b of the edges from (a-1, b, k), (a, b-1, k), (a, b, k-1)
  if (a > 0) {
    const int64_t c2 = corner_index(ws, nl, (size_t)L - n1, k);
    if (c2 >= 0 && (cinfo_mask(ws.cinfo[c2]) & 1u)) {
      const float fa = ws.cf[c2], d = fa - fc;
      s += dldv[3 * cinfo_vbase(ws.cinfo[c2]) + 0] * g.h * (fa / (d * d));
    }
  }
  if (b > 0) {
    const int64_t c2 = corner_index(ws, nl, (size_t)L - 1, k);
    if (c2 >= 0 && (cinfo_mask(ws.cinfo[c2]) & 2u)) {
      const uint32_t inf = ws.cinfo[c2];
      const float fa = ws.cf[c2], d = fa - fc;
      s += dldv[3 * (cinfo_vbase(inf) + (cinfo_mask(inf) & 1u)) + 1] * g.h * (fa / (d * d));
    }
  }
  if (ci > 0 && ws.cl[ci - 1] == L && ws.ck[ci - 1] == k - 1 && (cinfo_mask(ws.cinfo[ci - 1]) & 4u)) {
    const uint32_t inf = ws.cinfo[ci - 1];
    const float fa = ws.cf[ci - 1], d = fa - fc;
    s += dldv[3 * (cinfo_vbase(inf) + __popc(cinfo_mask(inf) & 3u)) + 2] * g.h * (fa / (d * d));
  }
  (void)m;
  return s;
}

// Corner cotangents, compacted to the corners where they are non-zero
// (list order = corner order).  Four corners per lane, single-pass scan.
__global__ __launch_bounds__(kBlock) void k_cotangents(Grid g, Workspace ws, const float* __restrict__ dldv,
                                                       int32_t* __restrict__ cidx, float* __restrict__ cval,
                                                       int64_t* __restrict__ ccount, uint64_t* __restrict__ flags,
                                                       gh_counters* __restrict__ ctr) {
  const int64_t m = ws.nlist[0];
  if (m > ws.cap) {  // the forward overflowed its corner list: nothing to differentiate
    if (blockIdx.x == 0 && threadIdx.x == 0) *ccount = 0;
    return;
  }
  const size_t nl = (size_t)(g.n + 1) * (g.n + 1);
  constexpr int kItems = 4, kTile = kBlock * kItems;
  const int ntiles = (int)((m + kTile - 1) / kTile);
  if (ntiles == 0 && blockIdx.x == 0 && threadIdx.x == 0) *ccount = 0;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
    const int64_t c0 = (int64_t)tile * kTile + (int64_t)threadIdx.x * kItems;
    float cot[kItems];
    unsigned cnt = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      cot[r] = c0 + r < m ? corner_cotangent(ws, g, nl, c0 + r, m, dldv) : 0.f;
      cnt += cot[r] != 0.f;
    }
    const ScanOut so = block_scan_lookback(cnt, flags, tile, &ctr->flags);
    int64_t o = (int64_t)so.excl;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      if (cot[r] == 0.f) continue;
      cidx[o] = (int32_t)(c0 + r);
      cval[o] = cot[r];
      ++o;
    }
    if (threadIdx.x == 0 && tile == ntiles - 1) *ccount = (int64_t)so.total;
  }
}

// ------------------------------------------------------------- network VJP
struct VjpSmem {
  MlpSmemF32 fw;                         // activations (FP32 layout), points
  float g[kVjpRows * kF32Stride];     // dL/dz of the current layer
  float gout[kVjpRows];               // dL/dNN per row
};

__device__ __forceinline__ float sigmoidf(float z) { return 1.f / (1.f + expf(-z)); }

// part[o * K + k] += sum_r g[r][o] act[r][k] for o < W, k < K.
template <int W>
__device__ __forceinline__ void vjp_dw(VjpSmem& sm, float* __restrict__ part, int K) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int OT = W / 32, KT = (K + 31) / 32;
  for (int tt = w; tt < OT * KT; tt += 4) {
    const int ot = tt / KT, kt = tt - ot * KT;
    f32x16_t acc;
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = 0.f;
    for (int rs = 0; rs < kVjpRows / 2; ++rs) {
      const int r = 2 * rs + (lane >> 5);
      const float av = sm.g[r * kF32Stride + ot * 32 + (lane & 31)];
      const float bv = sm.fw.af[r * kF32Stride + kt * 32 + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
    const int kk = kt * 32 + (lane & 31);
    if (kk < K) {
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int o = ot * 32 + 8 * (t >> 2) + 4 * (lane >> 5) + (t & 3);
        part[(size_t)o * K + kk] += acc[t];
      }
    }
  }
}

// g <- (g x W_l) * sigmoid(z_{l-1}); the product on the matrix cores with
// the transposed packing of W_l.
template <int W>
__device__ __forceinline__ void vjp_dg(const MlpDesc& m, VjpSmem& sm, int l, const float* __restrict__ zprev) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int KT = W / 32;            // output column tiles
  constexpr int kPerWave = 2 * KT / 4;  // (2 row tiles x KT) over 4 waves
  const float* __restrict__ wt = m.wft + (size_t)(l - 1) * W * W;
  f32x16_t acc[kPerWave];
#pragma unroll
  for (int q = 0; q < kPerWave; ++q)
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[q][t] = 0.f;
  // U k-steps per group: the weight loads of a group are all in flight before
  // its products (W / 2 is a multiple of U for every supported width).
  constexpr int U = 8;
  for (int os0 = 0; os0 < W / 2; os0 += U) {
    float bv[U][kPerWave];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < kPerWave; ++q) {
        const int tt = w * kPerWave + q, kt = tt % KT;
        bv[u][q] = wt[(size_t)((os0 + u) * KT + kt) * 64 + lane];
      }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < kPerWave; ++q) {
        const int tt = w * kPerWave + q, rt = tt / KT;
        const float av = sm.g[(rt * 32 + (lane & 31)) * kF32Stride + 2 * (os0 + u) + (lane >> 5)];
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[u][q], acc[q], 0, 0, 0);
      }
  }
  __syncthreads();  // every wave has read g
#pragma unroll
  for (int q = 0; q < kPerWave; ++q) {
    const int tt = w * kPerWave + q, rt = tt / KT, kt = tt - rt * KT;
    const int col = kt * 32 + (lane & 31);
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int row = rt * 32 + 8 * (t >> 2) + 4 * (lane >> 5) + (t & 3);
      sm.g[row * kF32Stride + col] = acc[q][t] * sigmoidf(zprev[row * W + col]);
    }
  }
  __syncthreads();
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_mlp_vjp(MlpDesc m, Grid g, Workspace ws, const int32_t* __restrict__ cidx,
                                                    const float* __restrict__ cval, const int64_t* __restrict__ ccount,
                                                    float* __restrict__ zs_all, float* __restrict__ part_all,
                                                    int64_t nparams) {
  __shared__ VjpSmem sm;
  const int64_t count = *ccount;
  const int D = m.depth, n1 = g.n + 1;
  float* __restrict__ zs = zs_all + (size_t)blockIdx.x * D * kVjpRows * W;
  float* __restrict__ part = part_all + (size_t)blockIdx.x * nparams;
  for (int64_t p = threadIdx.x; p < nparams; p += kBlock) part[p] = 0.f;
  // parameter offsets: W_0, b_0, W_1, b_1, ..., W_D, b_D
  auto offW = [&](int l) -> int64_t {
    return l == 0 ? 0 : (int64_t)(m.k1 + 1) * W + (int64_t)(l - 1) * (W + 1) * W;
  };
  // W_l has fan_out (W, or 1 for the output layer) x fan_in (k1 for l = 0, else W) entries
  auto offb = [&](int l) -> int64_t { return offW(l) + (int64_t)(l == D ? 1 : W) * (l == 0 ? m.k1 : W); };
  const int64_t ntiles = (count + kVjpRows - 1) / kVjpRows;
  __syncthreads();
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int t = threadIdx.x;
    const int64_t i = tile * kVjpRows + t;
    if (t < kVjpRows) {
      float x = 0.f, y = 0.f, z = 0.f, go = 0.f;
      if (i < count) {
        const int64_t ci = cidx[i];
        const int L = ws.cl[ci], a = L / n1, b = L - a * n1;
        x = lattice(g, a);
        y = lattice(g, b);
        z = lattice(g, ws.ck[ci]);
        go = m.a_n * cval[i];
      }
      sm.fw.pts[t][0] = x;
      sm.fw.pts[t][1] = y;
      sm.fw.pts[t][2] = z;
      sm.gout[t] = go;
    }
    __syncthreads();
    // forward, keeping the pre-activations
    mlp_features_f32(m, sm.fw, kVjpRows);
    for (int l = 0; l < D; ++l) mlp_layer_f32<W>(m, sm.fw, l, kVjpRows / 32, zs + (size_t)l * kVjpRows * W);
    // output layer: dW_D[o] += sum_r gout_r act_D[r][o], db_D += sum_r gout_r
    for (int o = t; o < W; o += kBlock) {
      float s = 0.f;
      for (int r = 0; r < kVjpRows; ++r) s += sm.gout[r] * sm.fw.af[r * kF32Stride + o];
      part[offW(D) + o] += s;
    }
    if (t == 0) {
      float s = 0.f;
      for (int r = 0; r < kVjpRows; ++r) s += sm.gout[r];
      part[offb(D)] += s;
    }
    // dL/dz_{D-1} = gout x w_out * sigmoid(z_{D-1})
    const float* __restrict__ zl = zs + (size_t)(D - 1) * kVjpRows * W;
    for (int e = t; e < kVjpRows * W; e += kBlock) {
      const int r = e / W, o = e - r * W;
      sm.g[r * kF32Stride + o] = sm.gout[r] * m.wout[o] * sigmoidf(zl[r * W + o]);
    }
    __syncthreads();
    for (int l = D - 1; l >= 0; --l) {
      // input of layer l back into act
      if (l == 0) {
        mlp_features_f32(m, sm.fw, kVjpRows);
      } else {
        const float* __restrict__ zp = zs + (size_t)(l - 1) * kVjpRows * W;
        for (int e = t; e < kVjpRows * W; e += kBlock) {
          const int r = e / W, c = e - r * W;
          sm.fw.af[r * kF32Stride + c] = softplus_f32(zp[r * W + c]);
        }
        __syncthreads();
      }
      const int K = l == 0 ? m.k1 : W;
      vjp_dw<W>(sm, part + offW(l), K);
      for (int o = t; o < W; o += kBlock) {
        float s = 0.f;
        for (int r = 0; r < kVjpRows; ++r) s += sm.g[r * kF32Stride + o];
        part[offb(l) + o] += s;
      }
      __syncthreads();
      if (l > 0) vjp_dg<W>(m, sm, l, zs + (size_t)(l - 1) * kVjpRows * W);
    }
    __syncthreads();
  }
}

// dL/dtheta[p] = sum over blocks, in block order.
__global__ __launch_bounds__(kBlock) void k_vjp_reduce(const float* __restrict__ part_all, int blocks, int64_t nparams,
                                                       float* __restrict__ out) {
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < nparams; p += (int64_t)gridDim.x * kBlock) {
    float s = 0.f;
    for (int b = 0; b < blocks; ++b) s += part_all[(size_t)b * nparams + p];
    out[p] = s;
  }
}

__global__ void k_zero_u64(uint64_t* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// ================================================================ launcher
int64_t mlp_param_count(const MlpDesc& m) {
  const int64_t W = m.W;
  return (int64_t)(m.k1 + 1) * W + (int64_t)(m.depth - 1) * (W + 1) * W + (W + 1);
}

size_t backward_layout(const MlpDesc& m, int64_t cap, void* base, BackwardWs* bw) {
  const int64_t tiles = (cap + 1023) / 1024;
  const int64_t np = mlp_param_count(m);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t o_idx = take((size_t)cap * 4), o_val = take((size_t)cap * 4), o_cnt = take(8),
               o_flags = take((size_t)tiles * 8), o_zs = take((size_t)kVjpBlocks * m.depth * kVjpRows * m.W * 4),
               o_part = take((size_t)kVjpBlocks * np * 4);
  if (base && bw) {
    char* b = (char*)base;
    bw->cidx = (int32_t*)(b + o_idx);
    bw->cval = (float*)(b + o_val);
    bw->ccount = (int64_t*)(b + o_cnt);
    bw->flags = (uint64_t*)(b + o_flags);
    bw->nflags = (size_t)tiles;
    bw->zs = (float*)(b + o_zs);
    bw->part = (float*)(b + o_part);
    bw->nparams = np;
  }
  return off;
}

template <class K>
static int grid_for(K kernel, int64_t tiles, int max_per_cu) {
  int per_cu = 0;
  const int cus = cu_count();
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t cap = (int64_t)cus * (per_cu < max_per_cu ? per_cu : max_per_cu);
  const int64_t gsz = tiles < cap ? tiles : cap;
  return (int)(gsz < 1 ? 1 : gsz);
}

template <int W>
static void launch_vjp_w(const DevSdb& d, const Grid& g, const Workspace& ws, const BackwardWs& bw, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_vjp<W>, dim3(kVjpBlocks), dim3(kBlock), 0, s, d.mlp, g, ws, bw.cidx, bw.cval, bw.ccount,
                     bw.zs, bw.part, bw.nparams);
}

hipError_t launch_backward(const DevSdb& d, const Grid& g, const Workspace& ws, const BackwardWs& bw,
                           const float* dldv, float* dldtheta, gh_counters* ctr, hipStream_t s) {
  if (d.kind != GH_SDB_MLP) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(kBlock), 0, s, bw.flags, bw.nflags);
  const int64_t tiles = (ws.cap + 1023) / 1024;
  hipLaunchKernelGGL(k_cotangents, dim3(grid_for(k_cotangents, tiles, 4)), dim3(kBlock), 0, s, g, ws, dldv, bw.cidx,
                     bw.cval, bw.ccount, bw.flags, ctr);
  switch (d.mlp.W) {
    case 64: launch_vjp_w<64>(d, g, ws, bw, s); break;
    case 128: launch_vjp_w<128>(d, g, ws, bw, s); break;
    case 256: launch_vjp_w<256>(d, g, ws, bw, s); break;
    default: return hipErrorInvalidValue;
  }
  const int64_t rblocks = (bw.nparams + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_vjp_reduce, dim3((unsigned)(rblocks < 4096 ? rblocks : 4096)), dim3(kBlock), 0, s, bw.part,
                     kVjpBlocks, bw.nparams, dldtheta);
  return hipGetLastError();
}

}  // namespace gh
