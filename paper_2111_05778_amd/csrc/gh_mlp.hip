// Kernels of the neural bound: point lists, corner lists, enumeration and the
// hop, all built on the tile evaluator of gh_mlp.h.
//
// In the two bf16 precisions a value whose use depends on a decision it
// might get wrong is re-evaluated in FP32 before it is used, with margin
// eps >= |f_bf16 - f_fp32|:
//   hop test      floor((|f| - eps)/h) != floor((|f| + eps)/h)
//   corner sign   |f| < eps  (corners and enumeration signs)
// so the hop schedule and the sign of every corner are the FP32 ones.

#include <float.h>

#include "gh_device.h"
#include "gh_launch.h"
#include "gh_layout.h"
#include "gh_hop.h"
#include "gh_mlp.h"

namespace gh {

// ------------------------------------------------------------- point lists
template <int P, int W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_mlp_points(MlpDesc m, const float* __restrict__ xyz, float* __restrict__ f,
                                                       int64_t count) {
  __shared__ MlpSmemFor<P> sm;
  constexpr int R = mlp_rows<P>();
  const int64_t tiles = (count + R - 1) / R;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t i0 = tile * R;
    const int nrows = (int)(count - i0 < R ? count - i0 : R);
    if ((int)threadIdx.x < nrows) {
      const int64_t i = i0 + threadIdx.x;
      sm.pts[threadIdx.x][0] = xyz[3 * i];
      sm.pts[threadIdx.x][1] = xyz[3 * i + 1];
      sm.pts[threadIdx.x][2] = xyz[3 * i + 2];
    }
    __syncthreads();
    mlp_tile<P, W>(m, sm, nrows);
    if ((int)threadIdx.x < nrows) f[i0 + threadIdx.x] = sm.f[threadIdx.x];
    __syncthreads();
  }
}

// FP32 values of the corners whose indices are in s_idx[0, cnt) (cnt <=
// kF32Rows), written to the corner list.
template <int W, class Sm>
__device__ __forceinline__ void corners_fp32(const MlpDesc& m, const Grid& g, const Workspace& ws, Sm& sm,
                                             const int64_t* s_idx, int cnt) {
  const int n1 = g.n + 1;
  const int t = threadIdx.x;
  if (t < cnt) {
    const int64_t i = s_idx[t];
    const int L = ws.cl[i], a = L / n1, b = L - a * n1;
    sm.pts[t][0] = lattice(g, a);
    sm.pts[t][1] = lattice(g, b);
    sm.pts[t][2] = lattice(g, ws.ck[i]);
  }
  __syncthreads();
  mlp_tile<kPrecF32, W>(m, sm, cnt);
  if (t < cnt) ws.cf[s_idx[t]] = sm.f[t];
  __syncthreads();
}

// Split-bf16 values of the corners whose indices are in s_idx3[0, cnt) (cnt <=
// kBf16Rows): a value with |f| >= eps3 is certain of its sign and goes to
// the corner list, the others join the FP32 queue s_idx at *npend.
template <int W, class Sm>
__device__ __forceinline__ void corners_split(const MlpDesc& m, const Grid& g, const Workspace& ws, Sm& sm,
                                              int* s_cnt, const int64_t* s_idx3, int cnt, int64_t* s_idx,
                                              int& npend) {
  const int n1 = g.n + 1;
  const int t = threadIdx.x;
  if (t < cnt) {
    const int64_t i = s_idx3[t];
    const int L = ws.cl[i], a = L / n1, b = L - a * n1;
    sm.pts[t][0] = lattice(g, a);
    sm.pts[t][1] = lattice(g, b);
    sm.pts[t][2] = lattice(g, ws.ck[i]);
  }
  __syncthreads();
  mlp_tile<kPrecBf16x3, W>(m, sm, cnt);
  const float f = t < cnt ? sm.f[t] : 0.f;
  __syncthreads();
  const bool amb = t < cnt && fabsf(f) < m.eps3;
  int namb;
  const int r = block_rank(amb, s_cnt, namb);
  if (amb) s_idx[npend + r] = s_idx3[t];
  else if (t < cnt) ws.cf[s_idx3[t]] = f;
  npend += namb;
  __syncthreads();
}

// Bound at every corner of the corner list.  In the bf16 precisions a value
// with |f| < eps gets an FP32 value instead (its sign is then the FP32 sign);
// those corners are collected per block and evaluated in full FP32 tiles.
// Plain bf16 with eps3 > 0 certifies in two steps: such a corner first gets
// a split-bf16 value (full tiles of kBf16Rows), and only one within eps3 of
// zero goes on to FP32.  With kStored the bf16 values are already in the
// corner list (k_mlp_corners_lean) and this pass only certifies.
template <int P, int W, bool kStored = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_mlp_corners(
    MlpDesc m, Grid g, Workspace ws, gh_counters* __restrict__ ctr) {
  static_assert(!kStored || P == kPrecBf16, "stored values are plain bf16 ones");
  __shared__ MlpSmemFor<P> sm;
  __shared__ int s_cnt[kBlock / 64];
  __shared__ int64_t s_idx[kF32Rows + kBf16Rows];  // waiting for FP32: < kF32Rows + one tile's worth
  __shared__ int64_t s_idx3[P == kPrecBf16 ? 2 * kBf16Rows : 1];  // waiting for split bf16
  constexpr int R = mlp_rows<P>();
  const int64_t count = ws.nlist[0];
  if (count > ws.cap) return;
  const int n1 = g.n + 1;
  uint64_t reevals = 0;
  int npend = 0, npend3 = 0;  // block-uniform
  const bool two_step = P == kPrecBf16 && m.eps3 > 0.f;
  const int64_t tiles = (count + R - 1) / R;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t i0 = tile * R;
    const int nrows = (int)(count - i0 < R ? count - i0 : R);
    const bool mine = (int)threadIdx.x < nrows;
    float f = 0.f;
    if constexpr (kStored) {
      if (mine) f = ws.cf[i0 + threadIdx.x];
    } else {
      if (mine) {
        const int64_t i = i0 + threadIdx.x;
        const int L = ws.cl[i], a = L / n1, b = L - a * n1;
        sm.pts[threadIdx.x][0] = lattice(g, a);
        sm.pts[threadIdx.x][1] = lattice(g, b);
        sm.pts[threadIdx.x][2] = lattice(g, ws.ck[i]);
      }
      __syncthreads();
      mlp_tile<P, W>(m, sm, nrows);
      f = mine ? sm.f[threadIdx.x] : 0.f;
      __syncthreads();
    }
    if constexpr (P != kPrecF32) {
      const bool amb = mine && fabsf(f) < m.eps;
      int namb;
      const int r = block_rank(amb, s_cnt, namb);
      if constexpr (P == kPrecBf16) {
        if (two_step) {
          if (amb) s_idx3[npend3 + r] = i0 + threadIdx.x;
          npend3 += namb;
        } else {
          if (amb) s_idx[npend + r] = i0 + threadIdx.x;
          npend += namb;
        }
      } else {
        if (amb) s_idx[npend + r] = i0 + threadIdx.x;
        npend += namb;
      }
      if (!kStored && !amb && mine) ws.cf[i0 + threadIdx.x] = f;
      __syncthreads();
      if constexpr (P == kPrecBf16) {
        while (npend3 >= kBf16Rows) {  // each split tile adds at most kBf16Rows to a queue below kF32Rows
          npend3 -= kBf16Rows;
          corners_split<W>(m, g, ws, sm, s_cnt, s_idx3 + npend3, kBf16Rows, s_idx, npend);
          while (npend >= kF32Rows) {
            npend -= kF32Rows;
            corners_fp32<W>(m, g, ws, sm, s_idx + npend, kF32Rows);
            reevals += threadIdx.x == 0 ? kF32Rows : 0;
          }
        }
      }
      while (npend >= kF32Rows) {
        npend -= kF32Rows;
        corners_fp32<W>(m, g, ws, sm, s_idx + npend, kF32Rows);
        reevals += threadIdx.x == 0 ? kF32Rows : 0;
      }
    } else {
      if (mine) ws.cf[i0 + threadIdx.x] = f;
    }
  }
  if constexpr (P != kPrecF32) {
    if constexpr (P == kPrecBf16) {
      if (npend3 > 0) corners_split<W>(m, g, ws, sm, s_cnt, s_idx3, npend3, s_idx, npend);
    }
    while (npend > 0) {
      const int c = npend < kF32Rows ? npend : kF32Rows;
      npend -= c;
      corners_fp32<W>(m, g, ws, sm, s_idx + npend, c);
      reevals += threadIdx.x == 0 ? c : 0;
    }
    block_add_u64(reevals, (unsigned long long*)&ctr->n_reeval);
  }
}

// Plain bf16 values of every corner of the list on the lean layout (two
// blocks per CU); k_mlp_corners<kPrecBf16, W, true> then certifies the
// signs of those within eps of zero.
template <int W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mlp_corners_lean(
    MlpDesc m, Grid g, Workspace ws) {
  __shared__ MlpSmemBf16 sm;
  constexpr int R = mlp_tile_rows<kPrecBf16, W, MlpSmemBf16>();
  const int64_t count = ws.nlist[0];
  if (count > ws.cap) return;
  const int n1 = g.n + 1;
  const int64_t tiles = (count + R - 1) / R;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t i0 = tile * R;
    const int nrows = (int)(count - i0 < R ? count - i0 : R);
    const bool mine = (int)threadIdx.x < nrows;
    if (mine) {
      const int64_t i = i0 + threadIdx.x;
      const int L = ws.cl[i], a = L / n1, b = L - a * n1;
      sm.pts[threadIdx.x][0] = lattice(g, a);
      sm.pts[threadIdx.x][1] = lattice(g, b);
      sm.pts[threadIdx.x][2] = lattice(g, ws.ck[i]);
    }
    __syncthreads();
    mlp_tile<kPrecBf16, W>(m, sm, nrows);
    if (mine) ws.cf[i0 + threadIdx.x] = sm.f[threadIdx.x];
    __syncthreads();
  }
}

// Enumeration: a tile covers R/64 units of 64 consecutive lattice points c
// of one lattice column; each unit becomes two sign words (bit: f < 0).
template <int P, int W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_mlp_dense(MlpDesc m, Grid g, uint32_t* __restrict__ signs,
                                                      uint64_t* __restrict__ colmask, gh_counters* __restrict__ ctr) {
  __shared__ MlpSmemFor<P> sm;
  __shared__ int s_cnt[kBlock / 64];
  constexpr int R = mlp_rows<P>();
  constexpr int kUnits = R / 64;
  const int n1 = g.n + 1;
  const size_t nl = (size_t)n1 * n1, ncol = (size_t)g.n * g.n;
  const int chunks = (n1 + 63) / 64, words1 = (g.n + 32) / 32;
  const int64_t units = (int64_t)nl * chunks;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncol; c += (size_t)gridDim.x * blockDim.x)
    colmask[c] = 0;
  bool bad = false;
  uint64_t reevals = 0;
  const int64_t tiles = (units + kUnits - 1) / kUnits;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int r = threadIdx.x;
    const int64_t u = tile * kUnits + r / 64;
    const size_t L = (size_t)((u < units ? u : 0) % nl);
    const int chunk = (int)((u < units ? u : 0) / nl);
    const int c = 64 * chunk + (r & 63);
    const bool valid = r < R && u < units && c < n1;
    const float x = lattice(g, (int)(L / n1)), y = lattice(g, (int)(L % n1)), z = lattice(g, c < n1 ? c : n1 - 1);
    if (r < R) {
      sm.pts[r][0] = x;
      sm.pts[r][1] = y;
      sm.pts[r][2] = z;
    }
    __syncthreads();
    mlp_tile<P, W>(m, sm, R);
    float f = r < R ? sm.f[r] : 0.f;
    __syncthreads();
    if constexpr (P != kPrecF32) {
      bool amb = valid && fabsf(f) < m.eps;
      if constexpr (P == kPrecBf16) {
        if (m.eps3 > 0.f) {  // two steps: split bf16 first, FP32 only within eps3 of zero
          f = reeval_split<W>(m, sm, s_cnt, amb, x, y, z, f);
          amb = amb && fabsf(f) < m.eps3;
        }
      }
      f = reeval_fp32<W>(m, sm, s_cnt, amb, x, y, z, f, reevals);
    }
    bad |= valid && !(fabsf(f) <= FLT_MAX);
    const uint64_t msk = __ballot(valid && f < 0.f);
    if (r < R && (r & 63) == 0 && u < units) {
      signs[(size_t)(2 * chunk) * nl + L] = (uint32_t)msk;
      if (2 * chunk + 1 < words1) signs[(size_t)(2 * chunk + 1) * nl + L] = (uint32_t)(msk >> 32);
    }
  }
  if (bad) atomicOr(&ctr->flags, GH_FLAG_NONFINITE);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr->n_hop_evals = (int64_t)n1 * n1 * n1;
  if constexpr (P != kPrecF32) block_add_u64(reevals, (unsigned long long*)&ctr->n_reeval);
}

// --------------------------------------------------------------------- hop
// Rays from a global counter over all n^2 columns.
struct QueueRays {
  unsigned int* queue;
  int64_t first, end;
  __device__ unsigned int take(unsigned int k) const { return atomicAdd(queue, k); }
};

template <int P, int W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_hop_mlp(MlpDesc m, Grid g, uint64_t* __restrict__ colmask,
                                                    uint32_t* __restrict__ colbits, unsigned int* __restrict__ queue,
                                                    gh_counters* __restrict__ ctr) {
  __shared__ MlpSmemFor<P> sm;
  __shared__ int s_cnt[kBlock / 64];
  __shared__ unsigned int s_base;
  hop_mlp_pool<P, W>(m, g, colmask, colbits, ctr, sm, s_cnt, &s_base, QueueRays{queue, 0, (int64_t)g.n * g.n});
}

// The shrunk plain bf16 hop on the lean LDS layout (no FP32 activations, no
// lo fragments): two blocks share a CU, so one wave's epilogue can issue
// while the other wave of its SIMD runs products.  At W = 256 a wave with
// all eight m-tiles of its 32 points would need more registers than two
// waves per SIMD leave, so there every tile is split over two waves per
// group (64 rows per tile; mlp_split_only).
template <int W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_hop_mlp_lean(
    MlpDesc m, Grid g, uint64_t* __restrict__ colmask, uint32_t* __restrict__ colbits, unsigned int* __restrict__ queue,
    gh_counters* __restrict__ ctr) {
  __shared__ MlpSmemBf16 sm;
  __shared__ int s_cnt[kBlock / 64];
  __shared__ unsigned int s_base;
  hop_mlp_pool<kPrecBf16, W>(m, g, colmask, colbits, ctr, sm, s_cnt, &s_base, QueueRays{queue, 0, (int64_t)g.n * g.n});
}

// The same two kernels for a small network whose weights stay resident in
// LDS (mlp_resident_fits): loaded once per block, no copies per tile.  Sm is
// MlpSmemRes, or MlpSmemResRelu for a ReLU network (max(z, 0) alone).
template <int W, class Sm>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_hop_mlp_res(
    MlpDesc m, Grid g, uint64_t* __restrict__ colmask, uint32_t* __restrict__ colbits, unsigned int* __restrict__ queue,
    gh_counters* __restrict__ ctr) {
  __shared__ Sm sm;
  __shared__ int s_cnt[kBlock / 64];
  __shared__ unsigned int s_base;
  mlp_load_resident<W>(m, sm);
  hop_mlp_pool<kPrecBf16, W>(m, g, colmask, colbits, ctr, sm, s_cnt, &s_base, QueueRays{queue, 0, (int64_t)g.n * g.n});
}

template <int W, class Sm>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mlp_corners_res(
    MlpDesc m, Grid g, Workspace ws) {
  __shared__ Sm sm;
  constexpr int R = kBf16Rows;
  const int64_t count = ws.nlist[0];
  if (count > ws.cap) return;
  mlp_load_resident<W>(m, sm);
  const int n1 = g.n + 1;
  const int64_t tiles = (count + R - 1) / R;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t i0 = tile * R;
    const int nrows = (int)(count - i0 < R ? count - i0 : R);
    const bool mine = (int)threadIdx.x < nrows;
    if (mine) {
      const int64_t i = i0 + threadIdx.x;
      const int L = ws.cl[i], a = L / n1, b = L - a * n1;
      sm.pts[threadIdx.x][0] = lattice(g, a);
      sm.pts[threadIdx.x][1] = lattice(g, b);
      sm.pts[threadIdx.x][2] = lattice(g, ws.ck[i]);
    }
    __syncthreads();
    mlp_tile<kPrecBf16, W>(m, sm, nrows);
    if (mine) ws.cf[i0 + threadIdx.x] = sm.f[threadIdx.x];
    __syncthreads();
  }
}

// ================================================================ launchers
template <class K>
static int mlp_grid(K kernel, int64_t tiles) {
  int per_cu = 0;
  const int cus = cu_count();
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t cap = (int64_t)cus * per_cu;
  const int64_t gsz = tiles < cap ? tiles : cap;
  return (int)(gsz < 1 ? 1 : gsz);
}

template <int P, int W>
static hipError_t launch_mlp_w(int what, const DevSdb& d, const Grid& g, const Workspace* ws, uint32_t* signs,
                               const float* xyz, float* f, int64_t count, gh_counters* ctr, hipStream_t s) {
  constexpr int R = mlp_rows<P>();
  switch (what) {
    case 0: {  // points
      auto k = k_mlp_points<P, W>;
      hipLaunchKernelGGL(k, dim3(mlp_grid(k, (count + R - 1) / R)), dim3(kBlock), 0, s, d.mlp, xyz, f, count);
      break;
    }
    case 1: {  // corners
      if constexpr (P == kPrecBf16) {
        if (current_tuning().mlp_lean == 1) {  // all values on the lean layout, then the certification
          constexpr int RL = mlp_tile_rows<kPrecBf16, W, MlpSmemBf16>();
          bool res = false;
          if constexpr (W == kResidentW) {
            if ((res = mlp_resident_fits(d.mlp.depth, W))) {
              auto kr = d.mlp.relu ? k_mlp_corners_res<W, MlpSmemResRelu> : k_mlp_corners_res<W, MlpSmemRes>;
              hipLaunchKernelGGL(kr, dim3(mlp_grid(kr, (ws->cap + kBf16Rows - 1) / kBf16Rows)), dim3(kBlock), 0, s,
                                 d.mlp, g, *ws);
            }
          }
          if (!res) {
            auto ka = k_mlp_corners_lean<W>;
            hipLaunchKernelGGL(ka, dim3(mlp_grid(ka, (ws->cap + RL - 1) / RL)), dim3(kBlock), 0, s, d.mlp, g, *ws);
          }
          auto kb = k_mlp_corners<P, W, true>;
          hipLaunchKernelGGL(kb, dim3(mlp_grid(kb, (ws->cap + R - 1) / R)), dim3(kBlock), 0, s, d.mlp, g, *ws, ctr);
          break;
        }
      }
      auto k = k_mlp_corners<P, W>;
      hipLaunchKernelGGL(k, dim3(mlp_grid(k, (ws->cap + R - 1) / R)), dim3(kBlock), 0, s, d.mlp, g, *ws, ctr);
      break;
    }
    case 2: {  // enumeration
      auto k = k_mlp_dense<P, W>;
      const int64_t n1 = g.n + 1;
      const int64_t units = n1 * n1 * ((n1 + 63) / 64);
      hipLaunchKernelGGL(k, dim3(mlp_grid(k, (units + R / 64 - 1) / (R / 64))), dim3(kBlock), 0, s, d.mlp, g, signs,
                         ws->colmask, ctr);
      break;
    }
    case 3: {  // hop
      auto k = k_hop_mlp<P, W>;
      // the shrunk plain bf16 hop never waits for FP32 values: by default it
      // runs on the lean layout, two blocks per CU
      if constexpr (P == kPrecBf16) {
        if (d.mlp.hop_shrink && current_tuning().mlp_lean == 1) {
          k = k_hop_mlp_lean<W>;
          if constexpr (W == kResidentW)
            if (mlp_resident_fits(d.mlp.depth, W))
              k = d.mlp.relu ? k_hop_mlp_res<W, MlpSmemResRelu> : k_hop_mlp_res<W, MlpSmemRes>;
        }
      }
      const int64_t rays = (int64_t)g.n * g.n;
      hipLaunchKernelGGL(k, dim3(mlp_grid(k, (rays + R - 1) / R)), dim3(kBlock), 0, s, d.mlp, g, ws->colmask,
                         ws->colbits, &ws->ticket[kTicketRays], ctr);
      break;
    }
  }
  return hipGetLastError();
}

template <int P>
static hipError_t launch_mlp_p(int what, const DevSdb& d, const Grid& g, const Workspace* ws, uint32_t* signs,
                               const float* xyz, float* f, int64_t count, gh_counters* ctr, hipStream_t s) {
  switch (d.mlp.W) {
    case 64: return launch_mlp_w<P, 64>(what, d, g, ws, signs, xyz, f, count, ctr, s);
    case 128: return launch_mlp_w<P, 128>(what, d, g, ws, signs, xyz, f, count, ctr, s);
    case 256: return launch_mlp_w<P, 256>(what, d, g, ws, signs, xyz, f, count, ctr, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mlp(int what, const DevSdb& d0, const Grid& g, const Workspace* ws, uint32_t* signs,
                      const float* xyz, float* f, int64_t count, gh_counters* ctr, hipStream_t s) {
  if (d0.kind != GH_SDB_MLP) return hipErrorInvalidValue;
  DevSdb d = d0;
  const Tuning tu = current_tuning();
  d.mlp.split = tu.mlp_split;
  d.mlp.pool_tiles = tu.mlp_pool_tiles;
  d.mlp.spec_rows = tu.mlp_spec_rows;
  switch (d.mlp.precision) {
    case kPrecBf16: return launch_mlp_p<kPrecBf16>(what, d, g, ws, signs, xyz, f, count, ctr, s);
    case kPrecBf16x3: return launch_mlp_p<kPrecBf16x3>(what, d, g, ws, signs, xyz, f, count, ctr, s);
    default: return launch_mlp_p<kPrecF32>(what, d, g, ws, signs, xyz, f, count, ctr, s);
  }
}

// The margin of b against a with one block in a fixed order (no clearing,
// the same bits every run): with d_i = b[i] - a[i], factor * max |d_i| into
// *out, or with off non-null (max d + min d) / 2 into *off and factor *
// (max d - min d) / 2 into *out; NaN when a value or difference is not
// finite, so that the margin cannot pass for a valid one.
__global__ __launch_bounds__(1024) void k_margin(const float* __restrict__ a, const float* __restrict__ b, int64_t m,
                                                 float factor, float* __restrict__ out, float* __restrict__ off) {
  __shared__ float s_max[1024], s_min[1024];
  float mx = -FLT_MAX, mn = FLT_MAX;
  int bad = 0;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    const float d = b[i] - a[i];
    bad |= !(fabsf(d) <= FLT_MAX);
    mx = fmaxf(mx, d);
    mn = fminf(mn, d);
  }
  bad = __syncthreads_or(bad);
  s_max[threadIdx.x] = mx;
  s_min[threadIdx.x] = mn;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_max[threadIdx.x] = fmaxf(s_max[threadIdx.x], s_max[threadIdx.x + w]);
      s_min[threadIdx.x] = fminf(s_min[threadIdx.x], s_min[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float hi = m > 0 ? s_max[0] : 0.f, lo = m > 0 ? s_min[0] : 0.f;
    const float nan = __builtin_nanf("");
    if (off) {
      *off = bad ? nan : 0.5f * (hi + lo);
      *out = bad ? nan : factor * (0.5f * (hi - lo));
    } else {
      *out = bad ? nan : factor * fmaxf(hi, -lo);
    }
  }
}

hipError_t launch_bf16_margin(const DevSdb& d0, int prec, const float* xyz, int64_t m, float factor, float* f32,
                              float* flp, float* out, float* off, hipStream_t s) {
  if (d0.kind != GH_SDB_MLP) return hipErrorInvalidValue;
  DevSdb d = d0;
  d.mlp.off = 0.f;  // raw values: the offset is what is being measured
  hipError_t e = hipSuccess;
  if (m > 0) {
    d.mlp.precision = kPrecF32;
    if ((e = launch_mlp(0, d, Grid{}, nullptr, nullptr, xyz, f32, m, nullptr, s)) != hipSuccess) return e;
    d.mlp.precision = prec;
    if ((e = launch_mlp(0, d, Grid{}, nullptr, nullptr, xyz, flp, m, nullptr, s)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_margin, dim3(1), dim3(1024), 0, s, f32, flp, m, factor, out, off);
  return hipGetLastError();
}

}  // namespace gh
