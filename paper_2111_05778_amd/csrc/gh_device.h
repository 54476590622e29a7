// Device-side building blocks shared by the kernels: grid and bound
// descriptors, the analytic bound evaluator, wave/block reductions and a
// single-pass block scan with decoupled look-back.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gh.h"

namespace gh {

constexpr int kBlock = 256;  // threads per block in every tiled kernel (4 waves)
constexpr int kMaxN = 2048;
constexpr int kMaxPrims = 64;

enum : int {
  kPrimSphere = 0,
  kPrimBox = 1,
  kPrimTorus = 2,
  kPrimCapsule = 3,
  kPrimPlane = 4,
  kPrimBoxBound = 5,
  kPrimCylinder = 6,
  kPrimCone = 7,
  kPrimHexPrism = 8,
  kPrimGenus2 = 9,
  kPrimSierpinski = 10
};

// Deepest Sierpinski record sdb_describe accepts.
constexpr int kSierpinskiMaxDepth = 16;

struct Grid {
  int n;        // cells per axis
  float lo;     // origin
  float h;      // cell size
  float inv_h;  // float32(1/h), computed in double and rounded once
  float cand_thr;  // candidate threshold float32((sqrt 3 / 2 + 1/32) h), or h on grids of cells small against
                   // the coordinates (h < 2^-12 max(1, |lo|, |lo + n h|)); in double, rounded once
};

// Cell centroid coordinate lo + (idx + 1/2) h (eq. cells): one rounded
// product and one rounded sum, no contraction.
__device__ __forceinline__ float centroid(const Grid& g, int idx) {
  return g.lo + ((float)idx + 0.5f) * g.h;
}
// Lattice coordinate lo + idx h.
__device__ __forceinline__ float lattice(const Grid& g, int idx) { return g.lo + (float)idx * g.h; }

// ------------------------------------------------------------ analytic bound
// Square root for hop decisions.  For a >= 2^-96 it is the correctly
// rounded root: the hardware estimate (within one ulp) or its neighbour on
// either side, chosen by the sign of the residual a - t s for each neighbour t
// (one fma, whose sign is exact); this range needs no scaling of the
// argument.  Below 2^-96 it returns the root of 2^-96 (2^-48).  A hop
// decision only needs floor(|f| / h), and in every formula a root below 2^-47
// either disappears when a term of magnitude >= 2^-23 is added (a radius or a
// face distance: the sum rounds to that term, as it does with the exact root)
// or leaves |f| < 2^-22, below h whenever h >= 2^-20, where both give s = 0.
// The torus's and the cylinder's first roots feed a second root instead,
// hence the condition |R| >= 2^-23 on the torus's ring radius and the
// cylinder's radius.  The cone's root is multiplied by c and followed by the
// subtraction of (a - qz) s, which either absorbs it or leaves a value below
// 2^-22 on both sides, so the maximum with the cap term gives s = 0 either
// way or the same cap value.  A Sierpinski record's edge and vertex roots are
// the value itself times 2^-d k, below 2^-48 k there, hence k < 2^27 for
// those records.  Kernels that use it run only when the grid and the union
// meet these conditions.
__device__ __forceinline__ float sqrt_hop(float a) {
  a = fmaxf(a, 0x1p-96f);
  const float s = __builtin_amdgcn_sqrtf(a);
  const float lo = __int_as_float(__float_as_int(s) - 1), hi = __int_as_float(__float_as_int(s) + 1);
  const float r = fmaf(-lo, s, a) <= 0.f ? lo : s;
  return fmaf(-hi, s, a) > 0.f ? hi : r;
}

// Smallest cell size for which sqrt_hop gives the decisions of the exact root.
constexpr float kHopRootMinH = 0x1p-20f;

// One primitive record (16 floats) at p, float32, one rounding per operation
// in exactly this order (the oracle's twin follows the same order):
//   d = p - c;  q_r = (M_r0 d_x + M_r1 d_y) + M_r2 d_z
//   sphere   sqrt((qx qx + qy qy) + qz qz) - r
//   box      u = |q| - b;  sqrt((mx mx + my my) + mz mz) + min(max(ux, max(uy, uz)), 0), m = max(u, 0)
//   boxbound max(ux, max(uy, uz))                         (Section 4.2, eq. boxdist)
//   torus    s = sqrt(qx qx + qz qz) - R;  sqrt(s s + qy qy) - r
//   capsule  w = qz - min(max(qz, -a), a);  sqrt((qx qx + qy qy) + w w) - r   (a >= 0)
//   plane    ((n_x x + n_y y) + n_z z) - d                 (Section 4.1, eq. plane)
//   cylinder rho = sqrt(qx qx + qy qy);  dx = rho - r, dz = |qz| - a, m = max(d, 0):
//            sqrt(mx mx + mz mz) + min(max(dx, dz), 0)     (capped, axis local z)
//   cone     rho = sqrt(qx qx + qy qy);  max(rho c - (a - qz) s, |qz| - a)
//            (apex at local z = a, half-angle with sine s and cosine c, cut at z = -a)
//   hexprism hx = qx/2, hy = (sqrt 3/2) qy;  max(|qx| - r, max(|hx + hy| - r,
//            max(|hy - hx| - r, |qz| - a)))                 (apothem r, axis local z)
//   genus2   k F(q), F = 2y(y^2 - 3x^2)(1 - z^2) + (x^2 + y^2)^2 - (9z^2 - 1)(1 - z^2)
//            (Section 5.1's implicit surface of genus 2; k normalises the
//            gradient over the grid to at most 1):  x2 = qx qx, y2, z2 alike,
//            w = 1 - z2;  ((((2 qy) (y2 - 3 x2)) w + (x2 + y2)(x2 + y2))
//            - (9 z2 - 1) w) k
//   sierpinski k S_d(q), the Sierpinski tetrahedron of depth d (Section 5.1's
//            fractal scene) on the tetrahedron T with vertices v_0 = (1,1,1),
//            v_1 = (1,-1,-1), v_2 = (-1,1,-1), v_3 = (-1,-1,1): d times
//            u = x + y, w = x - y, e = (-(u + z), z - w, w + z, u - z)
//            (e_i = -v_i . q), b = the least e_i (lowest i on ties), q = 2q - v_b;
//            then ldexp(t, -d) k with t the signed distance to T at the last q:
//            with the e_i sorted E1 >= E2 >= E3, a = E1 - 1, c = E2 - 1,
//              a float32(1/sqrt 3)                  if E1 + 3 E2 <= 4 (inside or beyond a face)
//              sqrt(0.375 (a a + c c) + 0.25 (a c))  if (E1 + E2) + 2 E3 <= 4 (beyond an edge)
//              |q - v_b| = sqrt((dx dx + dy dy) + dz dz)  otherwise (beyond the nearest vertex).
//            The copy at the nearest vertex is the nearest of the four (the
//            reflection swapping two vertices is a symmetry of the set), so
//            this is the signed distance to the set itself
// The type is a template argument: callers loop over primitives grouped by
// type, so no branch on the type sits inside the loop.  kHopRoot: the roots
// are taken by sqrt_hop (hop decisions only; the values themselves may differ
// from the exact ones below 2^-47).
template <int T, bool kHopRoot = false, class Ptr = const float*>
__device__ __forceinline__ float prim_eval_t(Ptr r, float x, float y, float z) {
  auto root = [](float v) { return kHopRoot ? sqrt_hop(v) : sqrtf(v); };
  if constexpr (T == kPrimPlane) {
    return ((r[4] * x + r[5] * y) + r[6] * z) - r[13];
  } else {
    const float dx = x - r[1], dy = y - r[2], dz = z - r[3];
    const float qx = (r[4] * dx + r[5] * dy) + r[6] * dz;
    const float qy = (r[7] * dx + r[8] * dy) + r[9] * dz;
    const float qz = (r[10] * dx + r[11] * dy) + r[12] * dz;
    if constexpr (T == kPrimSphere) {
      return root((qx * qx + qy * qy) + qz * qz) - r[13];
    } else if constexpr (T == kPrimTorus) {
      const float s = root(qx * qx + qz * qz) - r[13];
      return root(s * s + qy * qy) - r[14];
    } else if constexpr (T == kPrimCapsule) {
      // clamp(qz, -a, a) as one median of three (a >= 0 is validated on the
      // host; the result is the same input min(max(qz, -a), a) selects)
      const float w = qz - __builtin_amdgcn_fmed3f(qz, -r[13], r[13]);
      return root((qx * qx + qy * qy) + w * w) - r[14];
    } else if constexpr (T == kPrimCylinder) {
      const float rho = root(qx * qx + qy * qy);
      const float dx = rho - r[13], dz = fabsf(qz) - r[14];
      const float mx = fmaxf(dx, 0.f), mz = fmaxf(dz, 0.f);
      return root(mx * mx + mz * mz) + fminf(fmaxf(dx, dz), 0.f);
    } else if constexpr (T == kPrimCone) {
      const float rho = root(qx * qx + qy * qy);
      return fmaxf(rho * r[15] - (r[13] - qz) * r[14], fabsf(qz) - r[13]);
    } else if constexpr (T == kPrimGenus2) {
      const float x2 = qx * qx, y2 = qy * qy, z2 = qz * qz, w = 1.f - z2;
      const float r2 = x2 + y2;
      const float f = (((2.f * qy) * (y2 - 3.f * x2)) * w + r2 * r2) - (9.f * z2 - 1.f) * w;
      return f * r[13];
    } else if constexpr (T == kPrimSierpinski) {
      const int depth = (int)r[14];  // an integer in [0, kSierpinskiMaxDepth], validated on the host
      float x = qx, y = qy, z = qz;
      for (int l = 0; l < depth; ++l) {
        const float u = x + y, w = x - y;
        const float e0 = -(u + z), e1 = z - w, e2 = w + z, e3 = u - z;
        const bool odd01 = e1 < e0, odd23 = e3 < e2;  // the lesser of each pair, the lower index on a tie
        const float m01 = odd01 ? e1 : e0, m23 = odd23 ? e3 : e2;
        const bool low = !(m23 < m01);              // b in {0, 1}
        const float vx = low ? 1.f : -1.f, vy = (low ? odd01 : odd23) ? -1.f : 1.f;
        x = 2.f * x - vx;
        y = 2.f * y - vy;
        z = 2.f * z - vx * vy;                      // v_z = v_x v_y for the four vertices
      }
      // the distance to T at the last q: beyond one face (or inside), beyond
      // an edge, or beyond a vertex (the nearest one, picked as in the loop)
      const float u = x + y, w = x - y;
      const float e0 = -(u + z), e1 = z - w, e2 = w + z, e3 = u - z;
      const bool odd01 = e1 < e0, odd23 = e3 < e2;
      const bool low = !((odd23 ? e3 : e2) < (odd01 ? e1 : e0));
      const float vx = low ? 1.f : -1.f, vy = (low ? odd01 : odd23) ? -1.f : 1.f;
      const float h01 = fmaxf(e0, e1), l01 = fminf(e0, e1), h23 = fmaxf(e2, e3), l23 = fminf(e2, e3);
      const float mh = fminf(h01, h23), ml = fmaxf(l01, l23);
      const float E1 = fmaxf(h01, h23), E2 = fmaxf(mh, ml), E3 = fminf(mh, ml);  // the three largest e_i
      const float a = E1 - 1.f, c = E2 - 1.f;
      float t;
      if (E1 + 3.f * E2 <= 4.f) {
        t = a * 0.577350269189625764f;
      } else if ((E1 + E2) + 2.f * E3 <= 4.f) {
        t = root(0.375f * (a * a + c * c) + 0.25f * (a * c));
      } else {
        const float dx = x - vx, dy = y - vy, dz = z - vx * vy;
        t = root((dx * dx + dy * dy) + dz * dz);
      }
      return __builtin_amdgcn_ldexpf(t, -depth) * r[13];
    } else if constexpr (T == kPrimHexPrism) {
      const float hx = 0.5f * qx, hy = 0.866025403784438646f * qy;
      const float u1 = fabsf(qx) - r[13], u2 = fabsf(hx + hy) - r[13], u3 = fabsf(hy - hx) - r[13];
      return fmaxf(u1, fmaxf(u2, fmaxf(u3, fabsf(qz) - r[14])));
    } else {
      const float ux = fabsf(qx) - r[13], uy = fabsf(qy) - r[14], uz = fabsf(qz) - r[15];
      const float inner = fmaxf(ux, fmaxf(uy, uz));
      if constexpr (T == kPrimBoxBound) {
        return inner;
      } else {
        const float mx = fmaxf(ux, 0.f), my = fmaxf(uy, 0.f), mz = fmaxf(uz, 0.f);
        return root((mx * mx + my * my) + mz * mz) + fminf(inner, 0.f);
      }
    }
  }
}

constexpr int kPrimTypes = 11;
constexpr int kAllTypes = (1 << kPrimTypes) - 1;  // type mask with every type
constexpr int kFullTypes = 1 << 16;                 // flag beside a type mask: every lane holds every type

// Primitives sorted by type: group t occupies records [start[t], start[t+1]).
// The minimum is exact and commutative, so the order of the union does not
// change a single bit of the result (parameters are validated on the host so
// that no primitive can produce NaN).
struct PrimGroups {
  int start[kPrimTypes + 1];
};

template <int T, class F>
__device__ __forceinline__ void for_prims_of_type(const PrimGroups& g, int first, int step, F&& fn) {
  for (int p = g.start[T] + first; p < g.start[T + 1]; p += step) fn(p);
}

// Union over the primitives p = first, first + step, ... of every group.
template <class Rec>
__device__ __forceinline__ float union_strided(const PrimGroups& g, Rec rec, int first, int step, float x, float y,
                                               float z) {
  float f = __builtin_inff();
  for_prims_of_type<kPrimSphere>(g, first, step, [&](int p) { f = fminf(f, prim_eval_t<kPrimSphere>(rec(p), x, y, z)); });
  for_prims_of_type<kPrimBox>(g, first, step, [&](int p) { f = fminf(f, prim_eval_t<kPrimBox>(rec(p), x, y, z)); });
  for_prims_of_type<kPrimTorus>(g, first, step, [&](int p) { f = fminf(f, prim_eval_t<kPrimTorus>(rec(p), x, y, z)); });
  for_prims_of_type<kPrimCapsule>(g, first, step,
                                  [&](int p) { f = fminf(f, prim_eval_t<kPrimCapsule>(rec(p), x, y, z)); });
  for_prims_of_type<kPrimPlane>(g, first, step, [&](int p) { f = fminf(f, prim_eval_t<kPrimPlane>(rec(p), x, y, z)); });
  for_prims_of_type<kPrimBoxBound>(g, first, step,
                                   [&](int p) { f = fminf(f, prim_eval_t<kPrimBoxBound>(rec(p), x, y, z)); });
  for_prims_of_type<kPrimCylinder>(g, first, step,
                                   [&](int p) { f = fminf(f, prim_eval_t<kPrimCylinder>(rec(p), x, y, z)); });
  for_prims_of_type<kPrimCone>(g, first, step, [&](int p) { f = fminf(f, prim_eval_t<kPrimCone>(rec(p), x, y, z)); });
  for_prims_of_type<kPrimHexPrism>(g, first, step,
                                   [&](int p) { f = fminf(f, prim_eval_t<kPrimHexPrism>(rec(p), x, y, z)); });
  for_prims_of_type<kPrimGenus2>(g, first, step,
                                 [&](int p) { f = fminf(f, prim_eval_t<kPrimGenus2>(rec(p), x, y, z)); });
  for_prims_of_type<kPrimSierpinski>(g, first, step,
                                     [&](int p) { f = fminf(f, prim_eval_t<kPrimSierpinski>(rec(p), x, y, z)); });
  return f;
}

// Read-only global memory seen through the constant address space: a load
// at a wave-uniform address then becomes a scalar load into SGPRs instead of
// a vector load per lane.  Valid for data no kernel writes while it runs.
using ConstFloatPtr = const __attribute__((address_space(4))) float*;

// Min-union evaluated by one lane; every lane reads the same record at the
// same time, so the records come in by scalar loads.
struct PrimsEval {
  const float* __restrict__ prims;
  PrimGroups groups;
  __device__ __forceinline__ float operator()(float x, float y, float z) const {
    const ConstFloatPtr base = (ConstFloatPtr)prims;
    return union_strided(groups, [base](int p) { return base + p * GH_PRIM_FLOATS; }, 0, 1, x, y, z);
  }
};

// --------------------------------------------------------- wave/block sums
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  const int l = lane_id();
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(v, d, 64);
    if (l >= d) v += o;
  }
  return v;
}

// Adds v (per thread) over the block and atomically into *dst (one atomic per
// block).  The closing barrier lets the next call reuse the partials safely.
__device__ __forceinline__ void block_add_u64(uint64_t v, unsigned long long* dst) {
  __shared__ uint64_t s_part[kBlock / 64];
  v = wave_sum_u64(v);
  if (lane_id() == 0) s_part[wave_id()] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += s_part[w];
    if (t) atomicAdd(dst, (unsigned long long)t);
  }
  __syncthreads();
}

// ------------------------------------------------ single-pass block scan
// A tile publishes one 64-bit word per state change: status in the top two
// bits (1 = own aggregate, 2 = inclusive prefix), value in the low 62 bits.
// Tiles are taken in increasing order by block-strided loops over a grid of
// co-resident blocks, so every tile a block waits on is being processed.
constexpr uint64_t kScanAgg = 1ull << 62;
constexpr uint64_t kScanPrefix = 2ull << 62;
constexpr uint64_t kScanValMask = (1ull << 62) - 1;

struct ScanOut {
  uint64_t excl;   // exclusive prefix of this thread over the whole grid
  uint64_t base;   // exclusive prefix of this tile (its first output)
  uint64_t total;  // inclusive prefix at the end of this tile
};

// The whole block does the look-back over a window of kBlock * 4
// predecessors, thread t reading the words of tiles base - (r kBlock + t),
// r = 0..3 (distance 0 is the closest), so that consecutive lanes read
// consecutive words and a wave's load touches four cache lines.  A round
// consumes the words nearer than the closest unpublished one, up to and
// including the closest inclusive prefix; tiles before 0 read as prefix 0.
// A round that stopped at an unpublished word polls that word alone until it
// is published, then takes the next window from there.  All tiles of a kernel
// start at about the same time, so one wide window replaces a long chain of
// narrow ones, and the polls of waiting tiles stay one word each.  The wait is
// bounded: should it exceed kSpinLimit polls (only possible through a library
// bug), *err gets GH_FLAG_INTERNAL and the tile carries on with a partial
// prefix; every write stays inside its capacity check, so the result is
// flagged rather than the device hung.
//
// The scan comes in two halves so that a tile can do work that needs only
// its own offsets (staging outputs in LDS) while its predecessors finish:
// block_scan_publish scans the block and publishes the tile's aggregate,
// block_lookback returns the tile's base.  A coherent load of a look-back
// word takes microseconds while marching cubes keep memory busy.
constexpr int kSpinLimit = 1 << 22;
constexpr int kLookWindow = kBlock * 4;

struct NoAggHook {
  __device__ void operator()(uint64_t) const {}
};

struct LocalScan {
  uint64_t excl;  // exclusive prefix of this thread within the tile
  uint64_t agg;   // the tile's total
};

// on_agg(tile aggregate) runs in thread 0 before the tile publishes it.
template <class OnAgg = NoAggHook>
__device__ __forceinline__ LocalScan block_scan_publish(uint64_t v, uint64_t* flags, int tile,
                                                        OnAgg on_agg = OnAgg{}) {
  __shared__ uint64_t s_wave[kBlock / 64];
  const uint64_t incl = wave_incl_scan_u64(v);
  if (lane_id() == 63) s_wave[wave_id()] = incl;
  __syncthreads();
  uint64_t wave_off = 0, agg = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    const uint64_t s = s_wave[w];
    if (w < wave_id()) wave_off += s;
    agg += s;
  }
  if (threadIdx.x == 0) {
    on_agg(agg);
    __hip_atomic_store(&flags[tile], (tile == 0 ? kScanPrefix : kScanAgg) | (agg & kScanValMask), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();  // s_wave is free for the next tile
  return {wave_off + incl - v, agg};
}

// The tile's exclusive prefix over the grid; agg is its published total.
__device__ __forceinline__ uint64_t block_lookback(uint64_t* flags, int tile, uint64_t agg, unsigned int* err) {
  __shared__ uint64_t s_sum[kBlock / 64];
  __shared__ int s_first, s_empty, s_ready;
  __shared__ uint64_t s_prev;
  if (tile == 0) return 0;
  if (threadIdx.x == 0) s_prev = 0;
  int base = tile - 1;
  int spins = 0;
  bool probe = false;  // the last round stopped at an unpublished word: poll that one first
  while (true) {
    if (probe) {
      if (threadIdx.x == 0)
        s_ready = (__hip_atomic_load(&flags[base], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ~kScanValMask) != 0;
      __syncthreads();
      const bool ready = s_ready != 0;
      __syncthreads();
      if (!ready) {
        if (++spins > kSpinLimit) {
          if (threadIdx.x == 0) atomicOr(err, GH_FLAG_INTERNAL);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
    }
    uint64_t f[4];
    int first = kLookWindow, empty = kLookWindow;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pos = r * kBlock + (int)threadIdx.x;
      const int j = base - pos;
      f[r] = j >= 0 ? __hip_atomic_load(&flags[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kScanPrefix;
      const uint64_t st = f[r] & ~kScanValMask;
      if (st == kScanPrefix && pos < first) first = pos;
      if (st == 0 && pos < empty) empty = pos;
    }
    if (threadIdx.x == 0) {
      s_first = kLookWindow;
      s_empty = kLookWindow;
    }
    __syncthreads();
    if (first < kLookWindow) atomicMin(&s_first, first);
    if (empty < kLookWindow) atomicMin(&s_empty, empty);
    __syncthreads();
    first = s_first;
    empty = s_empty;
    const int last = first < empty ? first : empty - 1;
    uint64_t part = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (r * kBlock + (int)threadIdx.x <= last) part += f[r] & kScanValMask;
    part = wave_sum_u64(part);
    if (lane_id() == 0) s_sum[wave_id()] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t t = 0;
      for (int w = 0; w < kBlock / 64; ++w) t += s_sum[w];
      s_prev += t;
    }
    __syncthreads();
    if (first < empty) break;
    base -= empty;  // the closest unpublished word, or past the whole window
    probe = empty < kLookWindow;
  }
  if (threadIdx.x == 0)
    __hip_atomic_store(&flags[tile], kScanPrefix | ((s_prev + agg) & kScanValMask), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const uint64_t prev = s_prev;
  __syncthreads();  // s_prev is free for the next tile
  return prev;
}

// Both halves back to back.
template <class OnAgg = NoAggHook>
__device__ __forceinline__ ScanOut block_scan_lookback(uint64_t v, uint64_t* flags, int tile, unsigned int* err,
                                                       OnAgg on_agg = OnAgg{}) {
  const LocalScan ls = block_scan_publish(v, flags, tile, on_agg);
  const uint64_t base = block_lookback(flags, tile, ls.agg, err);
  ScanOut o;
  o.excl = base + ls.excl;
  o.base = base;
  o.total = base + ls.agg;
  return o;
}

}  // namespace gh
