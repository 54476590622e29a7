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
#include "gh_mlp.h"

namespace gh {

// Rank of this thread among the threads of the block with pred set, and
// their total.  Contains two barriers: every thread must call it.
__device__ __forceinline__ int block_rank(bool pred, int* s_cnt, int& total) {
  const uint64_t bal = __ballot(pred);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) s_cnt[w] = __popcll(bal);
  __syncthreads();
  int before = 0;
  total = 0;
#pragma unroll
  for (int q = 0; q < kBlock / 64; ++q) {
    const int c = s_cnt[q];
    if (q < w) before += c;
    total += c;
  }
  __syncthreads();
  return before + __popcll(bal & ((1ull << lane) - 1ull));
}

// FP32 re-evaluation of the points (x, y, z) of the threads with amb set, in
// tiles of kF32Rows; returns f updated for those threads.
template <int W>
__device__ __forceinline__ float reeval_fp32(const MlpDesc& m, MlpSmem& sm, int* s_cnt, bool amb, float x, float y,
                                             float z, float f, uint64_t& reevals) {
  int namb;
  const int arow = block_rank(amb, s_cnt, namb);
  for (int base = 0; base < namb; base += kF32Rows) {
    const bool mine = amb && arow >= base && arow < base + kF32Rows;
    if (mine) {
      sm.pts[arow - base][0] = x;
      sm.pts[arow - base][1] = y;
      sm.pts[arow - base][2] = z;
    }
    __syncthreads();
    mlp_tile<kPrecF32, W>(m, sm, namb - base < kF32Rows ? namb - base : kF32Rows);
    if (mine) f = sm.f[arow - base];
    __syncthreads();
  }
  reevals += amb ? 1 : 0;
  return f;
}

// ------------------------------------------------------------- point lists
template <int P, int W>
__global__ __launch_bounds__(kBlock) void k_mlp_points(MlpDesc m, const float* __restrict__ xyz, float* __restrict__ f,
                                                       int64_t count) {
  __shared__ MlpSmem sm;
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

// Bound at every corner of the corner list; signs certified (see above).
template <int P, int W>
__global__ __launch_bounds__(kBlock) void k_mlp_corners(MlpDesc m, Grid g, Workspace ws, gh_counters* __restrict__ ctr) {
  __shared__ MlpSmem sm;
  __shared__ int s_cnt[kBlock / 64];
  constexpr int R = mlp_rows<P>();
  const int64_t count = ws.nlist[0];
  if (count > ws.cap) return;
  const int n1 = g.n + 1;
  uint64_t reevals = 0;
  const int64_t tiles = (count + R - 1) / R;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t i0 = tile * R;
    const int nrows = (int)(count - i0 < R ? count - i0 : R);
    const bool mine = (int)threadIdx.x < nrows;
    float x = 0.f, y = 0.f, z = 0.f;
    if (mine) {
      const int64_t i = i0 + threadIdx.x;
      const int L = ws.cl[i], a = L / n1, b = L - a * n1;
      x = lattice(g, a);
      y = lattice(g, b);
      z = lattice(g, ws.ck[i]);
      sm.pts[threadIdx.x][0] = x;
      sm.pts[threadIdx.x][1] = y;
      sm.pts[threadIdx.x][2] = z;
    }
    __syncthreads();
    mlp_tile<P, W>(m, sm, nrows);
    float f = mine ? sm.f[threadIdx.x] : 0.f;
    __syncthreads();
    if constexpr (P != kPrecF32) f = reeval_fp32<W>(m, sm, s_cnt, mine && fabsf(f) < m.eps, x, y, z, f, reevals);
    if (mine) ws.cf[i0 + threadIdx.x] = f;
  }
  if constexpr (P != kPrecF32) block_add_u64(reevals, (unsigned long long*)&ctr->n_reeval);
}

// Enumeration: a tile covers R/64 units of 64 consecutive lattice points c
// of one lattice column; each unit becomes two sign words (bit: f < 0).
template <int P, int W>
__global__ __launch_bounds__(kBlock) void k_mlp_dense(MlpDesc m, Grid g, uint32_t* __restrict__ signs,
                                                      uint64_t* __restrict__ colmask, gh_counters* __restrict__ ctr) {
  __shared__ MlpSmem sm;
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
    if constexpr (P != kPrecF32) f = reeval_fp32<W>(m, sm, s_cnt, valid && fabsf(f) < m.eps, x, y, z, f, reevals);
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
// A block keeps a pool of R rays (one per owner thread, R = tile rows).  Each
// round it refills finished slots from a global ray counter, packs the live
// rays into the first rows, evaluates their current hop points as one tile
// (only the row tiles in use), certifies the bf16 values and applies the hop
// rule (Section 3, eq. iter, cell-quantised).
template <int P, int W>
__global__ __launch_bounds__(kBlock) void k_hop_mlp(MlpDesc m, Grid g, uint64_t* __restrict__ colmask,
                                                    uint32_t* __restrict__ colbits, unsigned int* __restrict__ queue,
                                                    gh_counters* __restrict__ ctr) {
  __shared__ MlpSmem sm;
  __shared__ int s_cnt[kBlock / 64];
  __shared__ unsigned int s_base;
  constexpr int R = mlp_rows<P>();
  const int n = g.n;
  const int64_t nrays = (int64_t)n * n;
  const size_t ncol = (size_t)nrays;
  const bool owner = (int)threadIdx.x < R;
  const float nf = (float)n;
  bool active = false, bad = false;
  size_t col = 0;
  int k = 0, wi = 0;
  uint32_t word = 0;
  uint64_t mask = 0;
  float x = 0.f, y = 0.f;
  uint64_t evals = 0, cands = 0, reevals = 0;
  for (;;) {
    // refill finished slots with the next rays
    int total;
    const bool want = owner && !active;
    const int fr = block_rank(want, s_cnt, total);
    if (threadIdx.x == 0) s_base = total ? atomicAdd(queue, (unsigned)total) : 0u;
    __syncthreads();
    if (want) {
      const int64_t idx = (int64_t)s_base + fr;
      if (idx < nrays) {
        active = true;
        col = (size_t)idx;
        x = centroid(g, (int)(idx / n));
        y = centroid(g, (int)(idx % n));
        k = 0;
        wi = 0;
        word = 0;
        mask = 0;
      }
    }
    // pack the live rays into rows [0, nact)
    int nact;
    const bool live = owner && active;
    const int row = block_rank(live, s_cnt, nact);
    if (nact == 0) break;  // uniform: the queue is empty and every slot is idle
    const float z = centroid(g, k);
    if (live) {
      sm.pts[row][0] = x;
      sm.pts[row][1] = y;
      sm.pts[row][2] = z;
    }
    __syncthreads();
    mlp_tile<P, W>(m, sm, nact);
    float d = live ? fabsf(sm.f[row]) : 0.f;
    __syncthreads();
    if constexpr (P != kPrecF32) {
      bool amb = false;
      if (live && d <= FLT_MAX)
        amb = floorf(fmaxf(d - m.eps, 0.f) * g.inv_h) != floorf((d + m.eps) * g.inv_h);
      d = fabsf(reeval_fp32<W>(m, sm, s_cnt, amb, x, y, z, d, reevals));
    }
    if (live) {
      ++evals;
      bool done = false;
      if (!(d <= FLT_MAX)) {
        bad = true;
        done = true;
      } else {
        const float s = floorf(d * g.inv_h);
        if (s == 0.f) {
          const int kw = k >> 5;
          if (kw != wi) {
            if (word) {
              colbits[(size_t)wi * ncol + col] = word;
              mask |= 1ull << wi;
            }
            word = 0;
            wi = kw;
          }
          word |= 1u << (k & 31);
          ++cands;
          ++k;
        } else {
          k += (int)fminf(s, nf);
        }
        done = k >= n;
      }
      if (done) {
        if (word) {
          colbits[(size_t)wi * ncol + col] = word;
          mask |= 1ull << wi;
        }
        colmask[col] = mask;
        active = false;
      }
    }
  }
  if (bad) atomicOr(&ctr->flags, GH_FLAG_NONFINITE);
  block_add_u64(evals, (unsigned long long*)&ctr->n_hop_evals);
  block_add_u64(cands, (unsigned long long*)&ctr->n_cand);
  block_add_u64(reevals, (unsigned long long*)&ctr->n_reeval);
}

// ================================================================ launchers
template <class K>
static int mlp_grid(K kernel, int64_t tiles) {
  int dev = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  const int cus = hipGetDeviceProperties(&prop, dev) == hipSuccess ? prop.multiProcessorCount : 1;
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

hipError_t launch_mlp(int what, const DevSdb& d, const Grid& g, const Workspace* ws, uint32_t* signs,
                      const float* xyz, float* f, int64_t count, gh_counters* ctr, hipStream_t s) {
  if (d.kind != GH_SDB_MLP) return hipErrorInvalidValue;
  switch (d.mlp.precision) {
    case kPrecBf16: return launch_mlp_p<kPrecBf16>(what, d, g, ws, signs, xyz, f, count, ctr, s);
    case kPrecBf16x3: return launch_mlp_p<kPrecBf16x3>(what, d, g, ws, signs, xyz, f, count, ctr, s);
    default: return launch_mlp_p<kPrecF32>(what, d, g, ws, signs, xyz, f, count, ctr, s);
  }
}

}  // namespace gh
