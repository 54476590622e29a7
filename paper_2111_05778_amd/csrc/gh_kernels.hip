// Grid hopping kernels for gfx950, with host launchers: counter reset, the
// analytic hop, the enumeration path and point evaluation.  The marching
// cubes on the hop's candidate cells are in the marching-cubes source.
//
// Pipeline of one polygonization (all on one stream):
//   k_clear      reset counters and look-back words
//   k_hop        R lanes per ray column: hop rule, candidate bitmap
//   marching cubes: k_corners, k_eval, k_verts, k_tris
// Enumeration replaces k_hop by k_dense_eval + k_dense_classify.

#include <float.h>

#include <algorithm>
#include <atomic>
#include <cmath>

#include "gh_device.h"
#include "gh_launch.h"
#include "gh_layout.h"
#include "gh_hop.h"

namespace gh {

// ------------------------------------------------------------------ clear
// Zeroes scan[begin, end), the given tickets and, before a hop, the
// counters.  (Marching cubes leave their own scans clean for the next pass.)
__global__ void k_clear(uint64_t* __restrict__ scan, size_t begin, size_t end, unsigned int* __restrict__ ticket,
                        unsigned ticket_mask, gh_counters* __restrict__ ctr, int mode) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = begin + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < end; i += stride) scan[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x < 8 && ((ticket_mask >> threadIdx.x) & 1)) ticket[threadIdx.x] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (mode == kClearAll) {
      ctr->n_hop_evals = 0;
      ctr->n_cand = 0;
      ctr->n_reeval = 0;
      ctr->flags = 0;
      ctr->reserved = 0;
      ctr->n_corner = 0;
      ctr->n_cells = 0;
      ctr->n_vert = 0;
      ctr->n_tri = 0;
    }
  }
}

// --------------------------------------------------------------------- hop
template <int R, bool kRegs, int kTypes = kAllTypes, bool kBudget = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_hop_prims(const float* __restrict__ prims, PrimGroups groups, Grid g,
                                                      uint64_t* __restrict__ colmask, uint32_t* __restrict__ colbits,
                                                      gh_counters* __restrict__ ctr, int budget,
                                                      uint32_t* __restrict__ park, unsigned int* __restrict__ npark) {
  __shared__ float4 s_rec[kMaxPrims * GH_PRIM_FLOATS / 4];
  stage_prims(s_rec, prims, groups.start[kPrimTypes]);
  hop_prims_tile<R, kRegs, kTypes, kBudget>(reinterpret_cast<const float*>(s_rec), groups, g, colmask, colbits, ctr,
                                            blockIdx.x,
                                   budget,
                           park, npark);
}

// Second pass of a hop with a step budget: the rays the first pass handed
// over, one wave and one window of cells each (see hop_window_rays).
template <int R, bool kRegs, int kTypes = kAllTypes>
__global__ __launch_bounds__(kBlock) void k_hop_long(const float* __restrict__ prims, PrimGroups groups, Grid g,
                                                     uint64_t* __restrict__ colmask, uint32_t* __restrict__ colbits,
                                                     const uint32_t* __restrict__ park,
                                                     const unsigned int* __restrict__ npark,
                                                     gh_counters* __restrict__ ctr) {
  __shared__ float4 s_rec[kMaxPrims * GH_PRIM_FLOATS / 4];
  stage_prims(s_rec, prims, groups.start[kPrimTypes]);
  hop_window_rays<R, kRegs, kTypes>(reinterpret_cast<const float*>(s_rec), groups, g, colmask, colbits, park, *npark,
                                    ctr);
}

// Algorithm 1 taken literally (see trace_prims_tile).
template <int R, bool kRegs = false, int kTypes = kAllTypes>
__global__ __launch_bounds__(kBlock) void k_trace_prims(const float* __restrict__ prims, PrimGroups groups, Grid g,
                                                        TraceConsts tc, uint64_t* __restrict__ colmask,
                                                        uint32_t* __restrict__ colbits,
                                                        gh_counters* __restrict__ ctr) {
  __shared__ float4 s_rec[kMaxPrims * GH_PRIM_FLOATS / 4];
  stage_prims(s_rec, prims, groups.start[kPrimTypes]);
  trace_prims_tile<R, kRegs, kTypes>(reinterpret_cast<const float*>(s_rec), groups, g, tc, colmask, colbits, ctr,
                                     blockIdx.x);
}

// ------------------------------------------------------------ enumeration
// Bound at every lattice point (Section 2, enumeration).  Classifying cells
// needs only the signs, so each wave evaluates 64 consecutive points c of
// one lattice column L and ballots them into two sign words of
// signs[W1][(n+1)^2] (bit set: f < 0).  Marching cubes re-evaluates the
// corners of the cells it keeps, exactly as after a hop.  Also clears the
// column masks that k_dense_classify sets.
template <class Eval>
__global__ __launch_bounds__(kBlock) void k_dense_eval(Eval ev, Grid g, uint32_t* __restrict__ signs,
                                                       uint64_t* __restrict__ colmask,
                                                       gh_counters* __restrict__ ctr) {
  const int n1 = g.n + 1;
  const size_t nl = (size_t)n1 * n1, ncol = (size_t)g.n * g.n;
  const int chunks = (n1 + 63) / 64, words1 = (g.n + 32) / 32;
  const size_t waves = nl * chunks;
  const size_t wstride = (size_t)gridDim.x * (kBlock / 64);
  const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t c = t0; c < ncol; c += (size_t)gridDim.x * blockDim.x) colmask[c] = 0;
  bool bad = false;
  for (size_t wv = (size_t)blockIdx.x * (kBlock / 64) + wave_id(); wv < waves; wv += wstride) {
    const size_t L = wv % nl;
    const int chunk = (int)(wv / nl);
    const int a = (int)(L / n1), b = (int)(L % n1);
    const int c = 64 * chunk + lane_id();
    bool neg = false;
    if (c < n1) {
      const float f = ev(lattice(g, a), lattice(g, b), lattice(g, c));
      neg = f < 0.f;
      bad |= !(fabsf(f) <= FLT_MAX);
    }
    const uint64_t m = __ballot(neg);
    if (lane_id() == 0) {
      signs[(size_t)(2 * chunk) * nl + L] = (uint32_t)m;
      if (2 * chunk + 1 < words1) signs[(size_t)(2 * chunk + 1) * nl + L] = (uint32_t)(m >> 32);
    }
  }
  if (bad) atomicOr(&ctr->flags, GH_FLAG_NONFINITE);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr->n_hop_evals = (int64_t)n1 * n1 * n1;
}

// Every cell whose eight corners do not share one side becomes a candidate.
// One thread builds one 32-cell word of one column from the sign words of
// its four lattice columns: cell k mixes signs when the OR over its corners
// (bits k and k+1 of each column) differs from their AND.
__global__ __launch_bounds__(kBlock) void k_dense_classify(Grid g, const uint32_t* __restrict__ signs,
                                                           uint64_t* __restrict__ colmask,
                                                           uint32_t* __restrict__ colbits,
                                                           gh_counters* __restrict__ ctr) {
  const int n = g.n, n1 = n + 1;
  const size_t ncol = (size_t)n * n, nl = (size_t)n1 * n1;
  const int words = (n + 31) >> 5, words1 = (n + 32) >> 5;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t col = tid % ncol;
  const int w = (int)(tid / ncol);
  uint64_t cands = 0;
  if (w < words) {
    const int i = (int)(col / n), j = (int)(col % n);
    const size_t L = (size_t)i * n1 + j;
    const size_t Ls[4] = {L, L + 1, L + n1, L + n1 + 1};
    uint32_t o = 0, an = ~0u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t cur = signs[(size_t)w * nl + Ls[q]];
      const uint32_t nxt = w + 1 < words1 ? signs[(size_t)(w + 1) * nl + Ls[q]] : 0u;
      const uint32_t up = (cur >> 1) | (nxt << 31);  // bit k: sign at k + 1
      o |= cur | up;
      an &= cur & up;
    }
    uint32_t word = o & ~an;
    const int valid = n - 32 * w;
    if (valid < 32) word &= (1u << valid) - 1u;
    if (word) {
      colbits[(size_t)w * ncol + col] = word;
      atomicOr((unsigned long long*)&colmask[col], 1ull << w);
      cands = __popc(word);
    }
  }
  block_add_u64(cands, (unsigned long long*)&ctr->n_cand);
}

template <class Eval>
__global__ __launch_bounds__(kBlock) void k_eval_points(Eval ev, const float* __restrict__ xyz, float* __restrict__ f,
                                                        int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += stride)
    f[p] = ev(xyz[3 * p], xyz[3 * p + 1], xyz[3 * p + 2]);
}

// ================================================================ launchers
hipError_t launch_clear(const Workspace& ws, gh_counters* ctr, ClearMode mode, hipStream_t s) {
  size_t begin = 0, end = scan_words(ws);
  unsigned tmask = 0xffu;
  if (mode == kClearCands) {
    begin = (size_t)(scan_cands(ws) - ws.scan);
    tmask = 1u << kTicketCands;
  }
  hipLaunchKernelGGL(k_clear, dim3(persistent_blocks((int64_t)(end - begin))), dim3(kBlock), 0, s, ws.scan, begin,
                     end, ws.ticket, tmask, ctr, (int)mode);
  return hipGetLastError();
}

template <int R>
static void launch_hop_r(const DevSdb& d, const Grid& g, const Workspace& ws, gh_counters* ctr, hipStream_t s) {
  using S = HopShape<R>;
  const int nbh = (g.n + S::kBlockH - 1) / S::kBlockH, nbw = (g.n + S::kBlockW - 1) / S::kBlockW;
  int most = 0;
  for (int t = 0; t < kPrimTypes; ++t) most = std::max(most, d.groups.start[t + 1] - d.groups.start[t]);
  const int budget = current_tuning().hop_step_budget;
  unsigned int* npark = &ws.ticket[kTicketPark];  // zeroed by the clear before every hop
  int present = 0;
  for (int t = 0; t < kPrimTypes; ++t) present |= (d.groups.start[t + 1] > d.groups.start[t] ? 1 : 0) << t;
  // Unions of spheres, boxes, tori and capsules (at most) get a kernel that
  // skips the other types; mixes covered by no special kernel take the
  // general one.
  constexpr int kSolids = (1 << kPrimSphere) | (1 << kPrimBox) | (1 << kPrimTorus) | (1 << kPrimCapsule);
  // The second pass (budget > 0) reads the count of handed-over rays on the
  // device; its grid fills the device once and strides over them.
  const int blocks = cu_count() * 8;
  // Register-record kernels take the hop square root: only where it gives
  // the exact root's decisions.
  const bool regs = most <= R && (d.flags & kSdbRadiiNormal) && g.h >= kHopRootMinH;
  // Unions of the solids, cylinders, cones and hexagonal prisms (the paper's
  // primitives) get a kernel that skips the other types.
  constexpr int kNoPlanes = kSolids | (1 << kPrimCylinder) | (1 << kPrimCone) | (1 << kPrimHexPrism);
  // Unions of Sierpinski records alone get a kernel that evaluates no other
  // type (the general kernel evaluates every type at every step).
  constexpr int kFractal = 1 << kPrimSierpinski;
  // The first pass without a budget carries no budget test.
  auto first = [&](auto kernel_nb, auto kernel_b) {
    if (budget > 0)
      hipLaunchKernelGGL(kernel_b, dim3(nbh * nbw), dim3(kBlock), 0, s, d.prims, d.groups, g, ws.colmask, ws.colbits,
                         ctr, budget, ws.park, npark);
    else
      hipLaunchKernelGGL(kernel_nb, dim3(nbh * nbw), dim3(kBlock), 0, s, d.prims, d.groups, g, ws.colmask,
                         ws.colbits, ctr, budget, ws.park, npark);
  };
  // all four solid types present, each with exactly R primitives: every lane
  // holds one record of each, and the kernel needs no presence select
  bool full = present == kSolids;
  for (int t = 0; t < kPrimTypes; ++t)
    if ((present >> t) & 1) full = full && d.groups.start[t + 1] - d.groups.start[t] == R;
  if (regs && full) {
    first(k_hop_prims<R, true, kSolids | kFullTypes, false>, k_hop_prims<R, true, kSolids | kFullTypes, true>);
    if (budget > 0)
      hipLaunchKernelGGL((k_hop_long<R, true, kSolids>), dim3(blocks), dim3(kBlock), 0, s, d.prims, d.groups, g,
                         ws.colmask, ws.colbits, ws.park, npark, ctr);
  } else if (regs && (present & ~kSolids) == 0) {
    first(k_hop_prims<R, true, kSolids, false>, k_hop_prims<R, true, kSolids, true>);
    if (budget > 0)
      hipLaunchKernelGGL((k_hop_long<R, true, kSolids>), dim3(blocks), dim3(kBlock), 0, s, d.prims, d.groups, g,
                         ws.colmask, ws.colbits, ws.park, npark, ctr);
  } else if (regs && (present & ~kNoPlanes) == 0) {
    first(k_hop_prims<R, true, kNoPlanes, false>, k_hop_prims<R, true, kNoPlanes, true>);
    if (budget > 0)
      hipLaunchKernelGGL((k_hop_long<R, true, kNoPlanes>), dim3(blocks), dim3(kBlock), 0, s, d.prims, d.groups, g,
                         ws.colmask, ws.colbits, ws.park, npark, ctr);
  } else if (regs && present == kFractal) {
    first(k_hop_prims<R, true, kFractal, false>, k_hop_prims<R, true, kFractal, true>);
    if (budget > 0)
      hipLaunchKernelGGL((k_hop_long<R, true, kFractal>), dim3(blocks), dim3(kBlock), 0, s, d.prims, d.groups, g,
                         ws.colmask, ws.colbits, ws.park, npark, ctr);
  } else {
    // Other unions read their records from LDS at every step, which only
    // touches the types present: holding a record of every type in
    // registers cost more (CSG-12 with a plane at N = 512, 0.43 against
    // 0.20 ms).
    first(k_hop_prims<R, false, kAllTypes, false>, k_hop_prims<R, false, kAllTypes, true>);
    if (budget > 0)
      hipLaunchKernelGGL((k_hop_long<R, false>), dim3(blocks), dim3(kBlock), 0, s, d.prims, d.groups, g, ws.colmask,
                         ws.colbits, ws.park, npark, ctr);
  }
}

hipError_t launch_hop(const DevSdb& d, const Grid& g, const Workspace& ws, gh_counters* ctr, int lanes_per_ray,
                      hipStream_t s) {
  if (d.kind == GH_SDB_MLP) return launch_mlp(3, d, g, &ws, nullptr, nullptr, nullptr, 0, ctr, s);
  if (d.kind != GH_SDB_PRIMS) return hipErrorInvalidValue;
  if (lanes_per_ray <= 0) {
    // Built-in choice: as many lanes as the largest type group has
    // primitives, so every lane of a group evaluates one of each type.
    int most = 1;
    for (int t = 0; t < kPrimTypes; ++t) most = std::max(most, d.groups.start[t + 1] - d.groups.start[t]);
    lanes_per_ray = most <= 4 ? most : 8;
  }
  switch (lanes_per_ray) {
    case 1: launch_hop_r<1>(d, g, ws, ctr, s); break;
    case 2: launch_hop_r<2>(d, g, ws, ctr, s); break;
    case 3: launch_hop_r<3>(d, g, ws, ctr, s); break;
    case 4: launch_hop_r<4>(d, g, ws, ctr, s); break;
    case 8: launch_hop_r<8>(d, g, ws, ctr, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int R>
static void launch_trace_r(const DevSdb& d, const Grid& g, const TraceConsts& tc, const Workspace& ws,
                           gh_counters* ctr, hipStream_t s) {
  using S = HopShape<R>;
  const int nbh = (g.n + S::kBlockH - 1) / S::kBlockH, nbw = (g.n + S::kBlockW - 1) / S::kBlockW;
  int most = 0, present = 0;
  for (int t = 0; t < kPrimTypes; ++t) {
    most = std::max(most, d.groups.start[t + 1] - d.groups.start[t]);
    present |= (d.groups.start[t + 1] > d.groups.start[t] ? 1 : 0) << t;
  }
  constexpr int kSolids = (1 << kPrimSphere) | (1 << kPrimBox) | (1 << kPrimTorus) | (1 << kPrimCapsule);
  if (most <= R && (present & ~kSolids) == 0)  // records in registers, solids only
    hipLaunchKernelGGL((k_trace_prims<R, true, kSolids>), dim3(nbh * nbw), dim3(kBlock), 0, s, d.prims, d.groups, g,
                       tc, ws.colmask, ws.colbits, ctr);
  else  // records read from LDS, as for the hop's other unions
    hipLaunchKernelGGL((k_trace_prims<R, false>), dim3(nbh * nbw), dim3(kBlock), 0, s, d.prims, d.groups, g, tc,
                       ws.colmask, ws.colbits, ctr);
}

hipError_t launch_hop_traced(const DevSdb& d, const Grid& g, const Workspace& ws, gh_counters* ctr,
                             int lanes_per_ray, hipStream_t s) {
  if (d.kind != GH_SDB_PRIMS) return hipErrorInvalidValue;
  const double h = g.h, side = (double)g.n * h;
  TraceConsts tc;
  tc.tau = (float)(std::sqrt(6.0) / 2.0 * h);
  tc.z_top = (float)((double)g.lo + side);
  tc.z_exit = (float)((double)g.lo + side / 2.0 + 1.05 * (side / 2.0));
  // Every trace advances by more than tau per evaluation and travels at
  // most 1.05 (N + 1/2) h, so a ray needs fewer than (N + 2)^2 evaluations.
  tc.max_steps = ((int64_t)g.n + 2) * ((int64_t)g.n + 2) + 64;
  if (lanes_per_ray <= 0) {
    int most = 1;
    for (int t = 0; t < kPrimTypes; ++t) most = std::max(most, d.groups.start[t + 1] - d.groups.start[t]);
    lanes_per_ray = most <= 4 ? most : 8;
  }
  switch (lanes_per_ray) {
    case 1: launch_trace_r<1>(d, g, tc, ws, ctr, s); break;
    case 2: launch_trace_r<2>(d, g, tc, ws, ctr, s); break;
    case 3: launch_trace_r<3>(d, g, tc, ws, ctr, s); break;
    case 4: launch_trace_r<4>(d, g, tc, ws, ctr, s); break;
    case 8: launch_trace_r<8>(d, g, tc, ws, ctr, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_dense(const DevSdb& d, const Grid& g, const Workspace& ws, uint32_t* signs, gh_counters* ctr,
                        hipStream_t s) {
  if (d.kind == GH_SDB_MLP) {
    const hipError_t e = launch_mlp(2, d, g, &ws, signs, nullptr, nullptr, 0, ctr, s);
    if (e != hipSuccess) return e;
  } else if (d.kind == GH_SDB_PRIMS) {
    const int64_t n1 = g.n + 1;
    const int64_t waves = n1 * n1 * ((n1 + 63) / 64);
    const int64_t blocks = (waves + 3) / 4;
    hipLaunchKernelGGL(k_dense_eval<PrimsEval>, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(kBlock), 0,
                       s, PrimsEval{d.prims, d.groups}, g, signs, ws.colmask, ctr);
  } else {
    return hipErrorInvalidValue;
  }
  const int64_t words = (g.n + 31) / 32;
  const int64_t threads = (int64_t)g.n * g.n * words;
  hipLaunchKernelGGL(k_dense_classify, dim3((unsigned)((threads + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g,
                     signs, ws.colmask, ws.colbits, ctr);
  return hipGetLastError();
}

int cu_count() {
  static std::atomic<int> cache[64];
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= 64) dev = 0;
  int c = cache[dev].load(std::memory_order_relaxed);
  if (c <= 0) {
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 1;
    cache[dev].store(c, std::memory_order_relaxed);
  }
  return c;
}

hipError_t launch_eval_points(const DevSdb& d, const float* xyz, float* f, int64_t m, hipStream_t s) {
  if (d.kind == GH_SDB_MLP) return launch_mlp(0, d, Grid{}, nullptr, nullptr, xyz, f, m, nullptr, s);
  if (d.kind != GH_SDB_PRIMS) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_eval_points<PrimsEval>, dim3(persistent_blocks(m)), dim3(kBlock), 0, s,
                     PrimsEval{d.prims, d.groups}, xyz, f, m);
  return hipGetLastError();
}

}  // namespace gh
