// Hop kernels' device functions, shared by the single-bound and the batched
// launches: the analytic hop over one block tile of ray columns (and its
// optional long-ray pass over cell windows), the paper's per-column
// procedure taken literally over the same tiles, and the network hop over a
// pool of rays fed by a ray source.
#pragma once

#include <float.h>

#include "gh_device.h"
#include "gh_layout.h"
#include "gh_mlp.h"

namespace gh {

// --------------------------------------------------------------------- hop
// R lanes trace one ray together: lane q of the group evaluates primitives
// q, q + R, q + 2R, ... of each type group (records staged in LDS) and a
// reduction over the R lanes forms the union's minimum, which every lane of
// the group then holds bit for bit.  This divides the latency of one hop
// step by about R; it matters because the kernel lasts as long as its
// longest column, and a ray grazing a flat face steps cell by cell (the
// plane-parallel case of Section 4.1 costs N steps on such a column).
// A wave covers a compact patch of columns whose step counts are similar.
// R = 3 suits unions with three primitives of each type (21 rays per wave,
// the last lane idle).
template <int R>
struct HopShape {
  static constexpr int kWaveRays = 64 / R;
  static constexpr int kWaveW = R == 1 ? 8 : (R == 2 ? 8 : (R == 3 ? 7 : 4));
  static constexpr int kWaveH = kWaveRays / kWaveW;
  static constexpr int kBlockH = 2 * kWaveH, kBlockW = 2 * kWaveW;
  static_assert(kWaveH * kWaveW == kWaveRays, "wave patch must hold every ray of the wave");
};

// Minimum over the R lanes of each ray group, identical in every lane of the
// group (fminf is exact, so any order gives the same value).
template <int R>
__device__ __forceinline__ float group_min(float f, int q) {
  if constexpr ((R & (R - 1)) == 0) {
#pragma unroll
    for (int m = 1; m < R; m <<= 1) f = fminf(f, __shfl_xor(f, m, 64));
    return f;
  } else {
    const int base = lane_id() - q;
    float v = __shfl(f, base, 64);
#pragma unroll
    for (int t = 1; t < R; ++t) v = fminf(v, __shfl(f, base + t, 64));
    return v;
  }
}

// One lane's share of a cell's union value when R lanes evaluate a cell:
// lane q takes primitives q, q + R, q + 2R, ... of each type group.
// kRegs: every type group has at most R primitives, so the lane holds at
// most one record per type, loaded once by lane_records into registers.
// kHopRoot: the roots of the register path are taken by sqrt_hop, so such
// kernels run only on grids and unions that meet that root's conditions (the
// others take the LDS-record kernel, with exact roots).
// kTypes (kRegs only): bit t set when type t may be present; a type whose bit
// is clear is neither loaded nor evaluated.  With kFullTypes also set, every
// type of the mask is present with exactly R primitives, so every lane holds
// one record of each and no presence select is needed.
template <int R, int kTypes>
__device__ __forceinline__ void lane_records(const float* __restrict__ srec, const PrimGroups& groups, int q,
                                             float (&rec)[kPrimTypes][GH_PRIM_FLOATS], bool (&has)[kPrimTypes]) {
#pragma unroll
  for (int t = 0; t < kPrimTypes; ++t) {
    const int p = groups.start[t] + q;
    has[t] = p < groups.start[t + 1];
    if (!((kTypes >> t) & 1)) continue;
    const float* src = srec + (has[t] ? p : 0) * GH_PRIM_FLOATS;
#pragma unroll
    for (int e = 0; e < GH_PRIM_FLOATS; ++e) rec[t][e] = src[e];
  }
}

// One type's value in the register path: +inf for a type outside the mask.
template <int T, int kTypes, bool kHopRoot>
__device__ __forceinline__ float lane_type(const float (&rec)[kPrimTypes][GH_PRIM_FLOATS], float x, float y,
                                           float z) {
  if constexpr (!(kTypes & (1 << T)))
    return __builtin_inff();
  else
    return prim_eval_t<T, kHopRoot>(rec[T], x, y, z);
}

template <int R, bool kRegs, int kTypes, bool kHopRoot = true>
__device__ __forceinline__ float lane_union(const float* __restrict__ srec, const PrimGroups& groups, int q,
                                            const float (&rec)[kPrimTypes][GH_PRIM_FLOATS],
                                            const bool (&has)[kPrimTypes], float x, float y, float z) {
  if constexpr (kRegs) {
    float f = __builtin_inff();
    // Every type of the mask is evaluated (a lane without one holds another
    // record and discards the value): no lane-dependent branch splits the
    // step, so the independent chains of the formulas interleave.
    float v[kPrimTypes];
    v[kPrimSphere] = lane_type<kPrimSphere, kTypes, kHopRoot>(rec, x, y, z);
    v[kPrimBox] = lane_type<kPrimBox, kTypes, kHopRoot>(rec, x, y, z);
    v[kPrimTorus] = lane_type<kPrimTorus, kTypes, kHopRoot>(rec, x, y, z);
    v[kPrimCapsule] = lane_type<kPrimCapsule, kTypes, kHopRoot>(rec, x, y, z);
    v[kPrimPlane] = lane_type<kPrimPlane, kTypes, kHopRoot>(rec, x, y, z);
    v[kPrimBoxBound] = lane_type<kPrimBoxBound, kTypes, kHopRoot>(rec, x, y, z);
    v[kPrimCylinder] = lane_type<kPrimCylinder, kTypes, kHopRoot>(rec, x, y, z);
    v[kPrimCone] = lane_type<kPrimCone, kTypes, kHopRoot>(rec, x, y, z);
    v[kPrimHexPrism] = lane_type<kPrimHexPrism, kTypes, kHopRoot>(rec, x, y, z);
    v[kPrimGenus2] = lane_type<kPrimGenus2, kTypes, kHopRoot>(rec, x, y, z);
    v[kPrimSierpinski] = lane_type<kPrimSierpinski, kTypes, kHopRoot>(rec, x, y, z);
#pragma unroll
    for (int t = 0; t < kPrimTypes; ++t)
      if ((kTypes >> t) & 1) f = (kTypes & kFullTypes) || has[t] ? fminf(f, v[t]) : f;
    return f;
  } else {
    return union_strided(groups, [srec](int p) { return srec + p * GH_PRIM_FLOATS; }, q, R, x, y, z);
  }
}

// Hop rule (Section 3, eq. iter, cell-quantised): at the centroid of cell k,
// s = floor(|f| * inv_h); s >= 1 skips s cells, s == 0 moves to k + 1 and
// marks cell k as a candidate when |f| <= cand_thr (a cell with a sign
// change holds a zero within half its diagonal of the centroid, and |f| is
// at most the distance to it; cand_thr adds h/32 for float32 error); the
// ray ends when k >= n.  One block tile of
// columns; srec holds the primitive records in LDS.
// kRegs and kTypes as for lane_union: with kRegs the records live in
// registers for the whole ray instead of being read from LDS at every step.
// kBudget and budget > 0: a ray still running after that many steps is
// handed over with its state (column, k, the candidate word in progress and
// the word mask) to park[*park_count++]; the long-ray pass finishes it
// exactly as this loop would have (the hop is a function of the state
// alone).  Without kBudget the loop carries no budget test (about 18 scalar
// instructions per step).
template <int R, bool kRegs = false, int kTypes = kAllTypes, bool kBudget = false>
__device__ __forceinline__ void hop_prims_tile(const float* __restrict__ srec, const PrimGroups& groups, const Grid& g,
                                               uint64_t* __restrict__ colmask, uint32_t* __restrict__ colbits,
                                               gh_counters* __restrict__ ctr, int tile, int budget = 0,
                                               uint32_t* __restrict__ park = nullptr,
                                               unsigned int* __restrict__ park_count = nullptr) {
  using S = HopShape<R>;
  const int n = g.n;
  const int nbw = (n + S::kBlockW - 1) / S::kBlockW;
  const int bi = tile / nbw, bj = tile - bi * nbw;
  const int w = wave_id(), l = lane_id();
  const int r = l / R, q = l % R;
  const int i = bi * S::kBlockH + (w >> 1) * S::kWaveH + r / S::kWaveW;
  const int j = bj * S::kBlockW + (w & 1) * S::kWaveW + r % S::kWaveW;
  uint64_t evals = 0, cands = 0;
  bool bad = false, parked = false;
  const size_t ncol = (size_t)n * n, col = (size_t)i * n + j;
  int k = 0, wi = 0;
  uint32_t word = 0;
  uint64_t mask = 0;
  if (r < S::kWaveRays && i < n && j < n) {  // uniform over the R lanes of a ray
    const float x = centroid(g, i), y = centroid(g, j);
    const float nf = (float)n;
    float rec[kPrimTypes][GH_PRIM_FLOATS];
    bool has[kPrimTypes];
    if constexpr (kRegs) lane_records<R, kTypes>(srec, groups, q, rec, has);
    while (k < n) {
      if constexpr (kBudget) {
        if (budget > 0 && (int)evals >= budget) {
          parked = true;
          break;
        }
      }
      float f = lane_union<R, kRegs, kTypes>(srec, groups, q, rec, has, x, y, centroid(g, k));
      f = group_min<R>(f, q);
      ++evals;
      const float d = fabsf(f);
      // A non-finite value ends the ray without a branch out of the loop:
      // floor(inf) is inf and fminf(NaN, n) is n, so the step below is n.
      bad = bad || !(d <= FLT_MAX);
      const float s = floorf(d * g.inv_h);
      if (s == 0.f) {
        if (d <= g.cand_thr) {
          const int kw = k >> 5;
          if (kw != wi) {
            if (word && q == 0) colbits[(size_t)wi * ncol + col] = word;
            if (word) mask |= 1ull << wi;
            word = 0;
            wi = kw;
          }
          word |= 1u << (k & 31);
          ++cands;
        }
        ++k;
      } else {
        k += (int)fminf(s, nf);
      }
    }
    if (q == 0 && !parked) {
      if (word) {
        colbits[(size_t)wi * ncol + col] = word;
        mask |= 1ull << wi;
      }
      colmask[col] = mask;
    }
  }
  if constexpr (kBudget) {  // hand-over: one atomic per wave
    const bool give = parked && q == 0;
    const uint64_t gb = __ballot(give);
    if (gb) {
      const int first = __builtin_ctzll(gb);
      unsigned base = 0;
      if (l == first) base = atomicAdd(park_count, (unsigned)__popcll(gb));
      base = __shfl(base, first, 64);
      if (give) {
        uint32_t* o = park + 6 * (size_t)(base + __popcll(gb & ((1ull << l) - 1ull)));
        o[0] = (uint32_t)col;
        o[1] = (uint32_t)k;
        o[2] = (uint32_t)wi;
        o[3] = word;
        o[4] = (uint32_t)mask;
        o[5] = (uint32_t)(mask >> 32);
      }
    }
  }
  if (q != 0) evals = cands = 0;
  if (bad && q == 0) atomicOr(&ctr->flags, GH_FLAG_NONFINITE);
  block_add_u64(evals, (unsigned long long*)&ctr->n_hop_evals);
  block_add_u64(cands, (unsigned long long*)&ctr->n_cand);
}

// Long-ray pass over cell windows: each handed-over ray continues from its
// saved state with a whole wave.  The R lanes of group t evaluate cell
// k0 + t exactly as the first pass evaluates a cell, for the W = 64 / R cells
// k0 .. k0 + W - 1 of the window at once; the wave then applies the hop rule
// at each cell it lands on with that cell's value, until a step leaves the
// window, which starts the next round there.  Only the values at cells the
// ray reaches are used, so the steps, candidates and counts are those of the
// one-pass hop; a ray stepping one cell at a time along a surface advances W
// cells per round instead of one.  Wave v of the grid takes rays v, v + V,
// ... for V waves (a ticket shared by every wave costs more than the
// imbalance: its atomics serialise across the chip).
template <int R, bool kRegs, int kTypes>
__device__ __forceinline__ void hop_window_rays(const float* __restrict__ srec, const PrimGroups& groups, const Grid& g,
                                                uint64_t* __restrict__ colmask, uint32_t* __restrict__ colbits,
                                                const uint32_t* __restrict__ park, unsigned npark,
                                                gh_counters* __restrict__ ctr) {
  constexpr int W = 64 / R;
  const int n = g.n;
  const size_t ncol = (size_t)n * n;
  const int l = lane_id(), t = l / R, q = l % R;  // lanes past W * R evaluate a spare cell
  const float nf = (float)n;
  float rec[kPrimTypes][GH_PRIM_FLOATS];
  bool has[kPrimTypes];
  if constexpr (kRegs) lane_records<R, kTypes>(srec, groups, q, rec, has);
  uint64_t evals = 0, cands = 0;
  bool bad = false;
  const unsigned nwaves = gridDim.x * (kBlock / 64);
  for (unsigned ray = (unsigned)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kBlock / 64) + wave_id()));
       ray < npark; ray += nwaves) {  // uniform
    const uint32_t* st = park + 6 * (size_t)ray;
    const size_t col = (uint32_t)__builtin_amdgcn_readfirstlane((int)st[0]);
    int k = __builtin_amdgcn_readfirstlane((int)st[1]), wi = __builtin_amdgcn_readfirstlane((int)st[2]);
    uint32_t word = (uint32_t)__builtin_amdgcn_readfirstlane((int)st[3]);
    uint64_t mask = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)st[4]) |
                    ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)st[5]) << 32);
    const int i = (int)(col / n), j = (int)(col - (size_t)i * n);
    const float x = centroid(g, i), y = centroid(g, j);
    bool rbad = false;
    while (k < n && !rbad) {
      const int k0 = k, kt = k0 + t;
      float f = lane_union<R, kRegs, kTypes>(srec, groups, q, rec, has, x, y, centroid(g, kt < n ? kt : n - 1));
      f = group_min<R>(f, q);
      const float d = fabsf(f);
      while (k < n && k - k0 < W) {  // k grows at every step: at most W steps
        const float dk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), (k - k0) * R));
        ++evals;
        if (!(dk <= FLT_MAX)) {
          rbad = true;
          break;
        }
        const float s = floorf(dk * g.inv_h);
        if (s == 0.f) {
          if (dk <= g.cand_thr) {
            const int kw = k >> 5;
            if (kw != wi) {
              if (word && l == 0) colbits[(size_t)wi * ncol + col] = word;
              if (word) mask |= 1ull << wi;
              word = 0;
              wi = kw;
            }
            word |= 1u << (k & 31);
            ++cands;
          }
          ++k;
        } else {
          k += (int)fminf(s, nf);
        }
      }
    }
    if (l == 0) {
      if (word) {
        colbits[(size_t)wi * ncol + col] = word;
        mask |= 1ull << wi;
      }
      colmask[col] = mask;
    }
    bad = bad || rbad;
  }
  if (l != 0) evals = cands = 0;
  if (bad && l == 0) atomicOr(&ctr->flags, GH_FLAG_NONFINITE);
  block_add_u64(evals, (unsigned long long*)&ctr->n_hop_evals);
  block_add_u64(cands, (unsigned long long*)&ctr->n_cand);
}

// ------------------------------------------------------------ traced hop
// Constants of the paper's per-column procedure taken literally, each
// computed on the host in double from the float32 grid and rounded once:
// tau = sqrt(6)/2 h (eq. polydist), the top face z_top = lo + N h, and the
// overrun height lo + N h / 2 + 1.05 N h / 2 (Algorithm 1's exit test, the
// unit cube's 1.05/2 generalised).  max_steps bounds one ray's evaluations.
struct TraceConsts {
  float tau, z_top, z_exit;
  int64_t max_steps;
};

// Algorithm 1 as printed, over one block tile of columns (the same tiles,
// R-lane groups and record placement as hop_prims_tile, but exact roots,
// since the stopping test compares |f| itself): from the
// centroid of cell k the ray is sphere-traced (eq. iter) until |f| <= tau or
// the travel t reaches 1.05 (z_top - z_s); the cell of the last centroid at
// or below z_s + t (never below k) is a candidate unless it lies past the
// last cell or z_s + t is above the overrun height, and the ray resumes at
// the next cell.  Candidates rise strictly along a column, so they go to the
// same candidate words as the hop's.  The float32 operations are those of
// the oracle's FP32 twin, one rounding each, in the same order.
template <int R, bool kRegs = false, int kTypes = kAllTypes>
__device__ __forceinline__ void trace_prims_tile(const float* __restrict__ srec, const PrimGroups& groups,
                                                 const Grid& g, const TraceConsts tc, uint64_t* __restrict__ colmask,
                                                 uint32_t* __restrict__ colbits, gh_counters* __restrict__ ctr,
                                                 int tile) {
  using S = HopShape<R>;
  const int n = g.n;
  const int nbw = (n + S::kBlockW - 1) / S::kBlockW;
  const int bi = tile / nbw, bj = tile - bi * nbw;
  const int w = wave_id(), l = lane_id();
  const int r = l / R, q = l % R;
  const int i = bi * S::kBlockH + (w >> 1) * S::kWaveH + r / S::kWaveW;
  const int j = bj * S::kBlockW + (w & 1) * S::kWaveW + r % S::kWaveW;
  uint64_t evals = 0, cands = 0;
  bool bad = false, stuck = false;
  if (r < S::kWaveRays && i < n && j < n) {  // uniform over the R lanes of a ray
    const size_t ncol = (size_t)n * n, col = (size_t)i * n + j;
    const float x = centroid(g, i), y = centroid(g, j), z0 = centroid(g, 0);
    const float nf = (float)n;
    int k = 0, wi = 0;
    uint32_t word = 0;
    uint64_t mask = 0;
    float rec[kPrimTypes][GH_PRIM_FLOATS];
    bool has[kPrimTypes];
    if constexpr (kRegs) lane_records<R, kTypes>(srec, groups, q, rec, has);
    float zs = z0, t = 0.f, tmax = 1.05f * (tc.z_top - zs);
    for (int64_t steps = 0;; ++steps) {
      if (steps >= tc.max_steps) {
        stuck = true;
        break;
      }
      float f = lane_union<R, kRegs, kTypes, false>(srec, groups, q, rec, has, x, y, zs + t);  // exact roots
      f = group_min<R>(f, q);
      ++evals;
      const float d = fabsf(f);
      if (!(d <= FLT_MAX)) {
        bad = true;
        break;
      }
      const bool near = d <= tc.tau;
      const float tn = t + d;
      if (!near) t = tn;
      if (near || tn >= tmax) {
        const float z = zs + t;
        const float kf = floorf((z - z0) * g.inv_h);
        // max(k, kf), held below n + 1 so that it fits an int
        const int kk = kf > (float)k ? (kf < nf ? (int)kf : n) : k;
        if (kk > n - 1 || z > tc.z_exit) break;
        const int kw = kk >> 5;
        if (kw != wi) {
          if (word && q == 0) colbits[(size_t)wi * ncol + col] = word;
          if (word) mask |= 1ull << wi;
          word = 0;
          wi = kw;
        }
        word |= 1u << (kk & 31);
        ++cands;
        k = kk + 1;
        zs = centroid(g, k);
        t = 0.f;
        tmax = 1.05f * (tc.z_top - zs);
      }
    }
    if (q == 0) {
      if (word) {
        colbits[(size_t)wi * ncol + col] = word;
        mask |= 1ull << wi;
      }
      colmask[col] = mask;
    }
  }
  if (q != 0) evals = cands = 0;
  if (bad && q == 0) atomicOr(&ctr->flags, GH_FLAG_NONFINITE);
  if (stuck && q == 0) atomicOr(&ctr->flags, GH_FLAG_INTERNAL);
  block_add_u64(evals, (unsigned long long*)&ctr->n_hop_evals);
  block_add_u64(cands, (unsigned long long*)&ctr->n_cand);
}

// Copies the primitive records into LDS (then one barrier).
__device__ __forceinline__ void stage_prims(float4* s_rec, const float* __restrict__ prims, int np) {
  for (int t = threadIdx.x; t < np * (GH_PRIM_FLOATS / 4); t += kBlock) s_rec[t] = reinterpret_cast<const float4*>(prims)[t];
  __syncthreads();
}

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

// Split-bf16 re-evaluation of the points (x, y, z) of the threads with amb
// set, in tiles of kBf16Rows; returns f updated for those threads (the first
// step of the plain-bf16 sign certification).
template <int W, class Sm>
__device__ __forceinline__ float reeval_split(const MlpDesc& m, Sm& sm, int* s_cnt, bool amb, float x, float y,
                                              float z, float f) {
  int namb;
  const int arow = block_rank(amb, s_cnt, namb);
  for (int base = 0; base < namb; base += kBf16Rows) {
    const bool mine = amb && arow >= base && arow < base + kBf16Rows;
    if (mine) {
      sm.pts[arow - base][0] = x;
      sm.pts[arow - base][1] = y;
      sm.pts[arow - base][2] = z;
    }
    __syncthreads();
    mlp_tile<kPrecBf16x3, W>(m, sm, namb - base < kBf16Rows ? namb - base : kBf16Rows);
    if (mine) f = sm.f[arow - base];
    __syncthreads();
  }
  return f;
}

// FP32 re-evaluation of the points (x, y, z) of the threads with amb set, in
// tiles of kF32Rows; returns f updated for those threads.
template <int W, class Sm>
__device__ __forceinline__ float reeval_fp32(const MlpDesc& m, Sm& sm, int* s_cnt, bool amb, float x, float y,
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

// A block keeps a pool of up to 2R rays (one per owner thread; the launch
// shape mlp_pool_tiles picks one or two tiles of R rows).  Each round it refills finished slots from the ray source
// (rays [first, end) of the column order, taken through src.take), then
// evaluates one tile:
//  * normally the current hop points of up to R live rays (R = tile rows),
//    packed into the first rows, in the kernel's precision; in the bf16
//    precisions a value whose hop decision is ambiguous within the margin
//    (floor((d - eps)/h) != floor((d + eps)/h), or d - eps and d + eps on
//    either side of the candidate threshold) is not used: its ray waits for
//    an FP32 value;
//  * an FP32 tile of up to kF32Rows waiting rays once that many wait, or
//    when every live ray waits.
// Deferring the FP32 values fills their tiles instead of paying a mostly
// empty FP32 tile in every round that meets one ambiguous value.  The hop
// rule (Section 3, eq. iter, cell-quantised) is applied to every value used,
// so the schedule is the FP32 one.

template <int P, int W, class Src, class Sm>
__device__ __forceinline__ void hop_mlp_pool(const MlpDesc& m, const Grid& g, uint64_t* __restrict__ colmask,
                                             uint32_t* __restrict__ colbits, gh_counters* __restrict__ ctr,
                                             Sm& sm, int* s_cnt, unsigned int* s_base, Src src) {
  constexpr int R = mlp_tile_rows<P, W, Sm>();
  // The lean layout holds no FP32 activations: it serves the shrunk bf16 hop,
  // which never waits for an FP32 value.
  constexpr bool kLean = std::is_same_v<Sm, MlpSmemBf16> || mlp_resident_layout<Sm>();
  static_assert(!kLean || P == kPrecBf16, "the lean layout runs the plain bf16 evaluator only");
  const int n = g.n;
  const size_t ncol = (size_t)n * n;
  // Up to two tiles' worth of slots (a launch shape): ready rays fill the
  // tile while others wait for FP32 values, and the ray queue still balances
  // the work between blocks.
  const bool owner = (int)threadIdx.x < (m.pool_tiles == 1 ? 1 : 2) * R;
  const float nf = (float)n;
  bool active = false, pend = false, bad = false;
  size_t col = 0;
  int k = 0, wi = 0;
  uint32_t word = 0;
  uint64_t mask = 0;
  float x = 0.f, y = 0.f;
  uint64_t evals = 0, cands = 0, reevals = 0;
  // Hop rule with the value d at (x, y, centroid k); ends the ray when done.
  auto advance = [&](float d) {
    ++evals;
    bool done = false;
    if (!(d <= FLT_MAX)) {
      bad = true;
      done = true;
    } else {
      const float s = floorf(d * g.inv_h);
      if (s == 0.f) {
        if (d <= g.cand_thr) {
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
        }
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
  };
  for (;;) {
    // refill finished slots with the next rays
    int total;
    const bool want = owner && !active;
    const int fr = block_rank(want, s_cnt, total);
    if (threadIdx.x == 0) *s_base = total ? src.take((unsigned)total) : 0u;
    __syncthreads();
    if (want) {
      const int64_t idx = src.first + (int64_t)*s_base + fr;
      if (idx < src.end) {
        active = true;
        pend = false;
        col = (size_t)idx;
        x = centroid(g, (int)(idx / n));
        y = centroid(g, (int)(idx % n));
        k = 0;
        wi = 0;
        word = 0;
        mask = 0;
      }
    }
    int nrun, npend = 0;
    const bool ready = owner && active && !pend;
    const int row = block_rank(ready, s_cnt, nrun);
    const bool run = ready && row < R;  // the first R ready rays form this round's tile
    nrun = nrun < R ? nrun : R;
    int prow = 0;
    if constexpr (P != kPrecF32 && !kLean) prow = block_rank(owner && active && pend, s_cnt, npend);
    if (nrun == 0 && npend == 0) break;  // uniform: the queue is empty and every slot is idle
    const float z = centroid(g, k);
    if constexpr (!kLean) {
      if (npend >= kF32Rows || nrun == 0) {
        // FP32 values for up to kF32Rows waiting rays
        const bool mine = owner && active && pend && prow < kF32Rows;
        if (mine) {
          sm.pts[prow][0] = x;
          sm.pts[prow][1] = y;
          sm.pts[prow][2] = z;
        }
        __syncthreads();
        mlp_tile<kPrecF32, W>(m, sm, npend < kF32Rows ? npend : kF32Rows);
        const float d = mine ? fabsf(sm.f[prow]) : 0.f;
        __syncthreads();
        if (mine) {
          ++reevals;
          pend = false;
          advance(d);
        }
        continue;
      }
    }
    // Few ready rays (the pool draining): each also gets rows for its next
    // cells k + 1, ..., k + D - 1, filling a 32-row tile, which takes as long
    // as a tile of one row per ray.  A ray whose step (one cell as a
    // candidate, or a hop) lands inside that window takes the landing cell's
    // value at once; a value is used only at a cell the ray reaches, so the
    // steps and counts are unchanged.
    const int spec = m.spec_rows < R ? m.spec_rows : R;  // rows given out as windows (a launch shape)
    const int D = nrun <= spec ? spec / nrun : 1;
    if (run) {
#pragma unroll 1
      for (int t = 0; t < D; ++t) {
        sm.pts[row * D + t][0] = x;
        sm.pts[row * D + t][1] = y;
        sm.pts[row * D + t][2] = k + t < n ? centroid(g, k + t) : z;
      }
    }
    __syncthreads();
    mlp_tile<P, W>(m, sm, nrun * D);
    if (run) {
      const int k0 = k;
#pragma unroll 1
      while (active && k - k0 < D) {  // k grows with every step: at most D rounds
        float d = fabsf(sm.f[row * D + (k - k0)]);
        bool amb = false;
        if constexpr (P != kPrecF32) {
          if (kLean || m.hop_shrink) {
            // |f| - eps bounds |f_fp32| from below: the step is safe as it is
            // (a non-finite value stays non-finite)
            d = d <= FLT_MAX ? fmaxf(d - m.eps, 0.f) : d;
          } else {
            // the FP32 value lies in [d - eps, d + eps]: wait for it when the
            // step or the candidate test could differ there
            const float dl = fmaxf(d - m.eps, 0.f), dh = d + m.eps;
            amb = d <= FLT_MAX &&
                  (floorf(dl * g.inv_h) != floorf(dh * g.inv_h) || (dl <= g.cand_thr) != (dh <= g.cand_thr));
          }
        }
        if (amb) {
          pend = true;
          break;
        }
        advance(d);
      }
    }
    __syncthreads();
  }
  if (bad) atomicOr(&ctr->flags, GH_FLAG_NONFINITE);
  block_add_u64(evals, (unsigned long long*)&ctr->n_hop_evals);
  block_add_u64(cands, (unsigned long long*)&ctr->n_cand);
  block_add_u64(reevals, (unsigned long long*)&ctr->n_reeval);
}

}  // namespace gh
