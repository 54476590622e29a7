// Marching-cubes kernels for gfx950 on the candidate cells the hop leaves,
// with their host launchers.
//
//   k_corners    per lattice column: distinct corners of candidate cells,
//                single-pass scan -> CSR offsets, corner list
//   k_eval       bound at every corner, one lane per corner (analytic here,
//                network kernels in the network source)
//   k_verts      per lattice column: crossing edges owned by each corner,
//                scan -> one welded vertex per crossing lattice edge
//   k_tris       per cell column: case byte, triangles from the table,
//                scan -> triangle and cell emit
//   k_candidates candidate cells as a flat list (gh_candidates)

#include <float.h>

#include "gh_device.h"
#include "gh_launch.h"
#include "gh_layout.h"
#include "mc_table.h"

namespace gh {

__constant__ McTable g_mc = kMcTable;

// -------------------------------------------------------- candidate export
__global__ __launch_bounds__(kBlock) void k_candidates(Grid g, Workspace ws, int64_t* __restrict__ out, int64_t cap,
                                                      gh_counters* __restrict__ ctr) {
  const int n = g.n;
  const size_t ncol = (size_t)n * n;
  for (int tile = blockIdx.x; tile < (int)ws.tiles_col; tile += gridDim.x) {
  __syncthreads();
  const size_t col = (size_t)tile * kBlock + threadIdx.x;
  uint64_t m = 0;
  uint64_t cnt = 0;
  if (col < ncol) {
    m = ws.colmask[col];
    for (uint64_t r = m; r; r &= r - 1) cnt += __popc(ws.colbits[(size_t)__builtin_ctzll(r) * ncol + col]);
  }
  const ScanOut so = block_scan_lookback(cnt, scan_cands(ws), tile, &ctr->flags);
  if (col < ncol && so.excl + cnt <= (uint64_t)cap) {
    int64_t o = (int64_t)so.excl;
    for (uint64_t r = m; r; r &= r - 1) {
      const int w = __builtin_ctzll(r);
      for (uint32_t b = ws.colbits[(size_t)w * ncol + col]; b; b &= b - 1)
        out[o++] = (int64_t)col * n + 32 * w + __builtin_ctz(b);
    }
  }
  if (threadIdx.x == 0 && tile == (int)ws.tiles_col - 1 && so.total > (uint64_t)cap)
    atomicOr(&ctr->flags, GH_FLAG_CAPACITY);
  }
}

// Waits until this thread's device-scope atomic adds are performed, so that
// the tile's scan word, stored next, is seen only after them (a device-scope
// fence would also write back the whole L2 at every tile).
__device__ __forceinline__ void counts_done() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}

// Zeroes p[0, count) with the whole grid.
__device__ __forceinline__ void zero_words(uint64_t* __restrict__ p, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ------------------------------------------------------------------ corners
// Candidate words of the (up to four) cell columns around lattice column
// (a, b); a missing or empty column has mask 0.  Fixed-size and unrolled so
// that everything stays in registers.
struct LatAdj {
  uint32_t col[4];  // n * n < 2^32 for every supported n
  uint64_t mask[4];
  uint64_t uni;
};

__device__ __forceinline__ LatAdj lat_adjacent(int n, int a, int b, const uint64_t* __restrict__ colmask) {
  LatAdj A;
  A.uni = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = a - 1 + (q >> 1), j = b - 1 + (q & 1);
    const bool ok = i >= 0 && i < n && j >= 0 && j < n;
    const uint32_t c = ok ? (uint32_t)(i * n + j) : 0u;
    const uint64_t m = ok ? colmask[c] : 0ull;
    A.col[q] = c;
    A.mask[q] = m;
    A.uni |= m;
  }
  return A;
}

// OR over the wave, returned in scalar registers: loops over its bits are
// uniform, so every lane issues the load of word w in the same instruction
// (adjacent lanes are adjacent columns: one coalesced access per word).
__device__ __forceinline__ uint64_t wave_uniform_or(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) v |= __shfl_xor(v, d, 64);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Candidate word w of the four cell columns around a lattice column, OR-ed,
// and slot 3's word (the cell column (a, b) itself) on its own.  The four
// loads are unconditional (a missing column reads column 0 of the same word
// and is masked off), so no branch separates a load from its use and a group
// of words issues all its loads before the first wait.  0 <= w < words.
__device__ __forceinline__ uint32_t adj_cell_word_own(const LatAdj& A, const uint32_t* __restrict__ colbits,
                                                      size_t ncol, int w, uint32_t& own) {
  uint32_t v = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t x = colbits[(size_t)w * ncol + A.col[q]] & (0u - (uint32_t)((A.mask[q] >> w) & 1));
    v |= x;
    if (q == 3) own = x;
  }
  return v;
}

// Walks the corner words of the wave's columns in ascending order and calls
// fn(w, corner word, own cell word) for each; a lane without word w sees 0.
// Word w of a lattice column holds corners of cells w (bits k, k + 1) and
// w - 1 (its top corner at bit 0); cell words exist for w < words.  Words go
// in groups of kWalk whose loads are all issued before any is used (one
// memory round trip per group).  A word the walk skips is 0 in every lane of
// the wave, so the carry from the previous word needs no load.
constexpr int kWalk = 4;

template <class F>
__device__ __forceinline__ void walk_corner_words(const LatAdj& A, const uint32_t* __restrict__ colbits, size_t ncol,
                                                  int words, uint64_t wave_words, bool wave_hi, F&& fn) {
  int pw = -2;
  uint32_t pcur = 0;
  for (uint64_t r = wave_words; r;) {
    int wg[kWalk];
    uint32_t cur[kWalk], own[kWalk];
#pragma unroll
    for (int g = 0; g < kWalk; ++g) {
      const int w = r ? __builtin_ctzll(r) : -1;
      r &= r - 1;
      wg[g] = w;
      const bool cell = w >= 0 && w < words;  // uniform
      uint32_t o;
      const uint32_t c = adj_cell_word_own(A, colbits, ncol, cell ? w : 0, o);
      cur[g] = cell ? c : 0u;
      own[g] = cell ? o : 0u;
    }
#pragma unroll
    for (int g = 0; g < kWalk; ++g) {
      if (wg[g] < 0) break;
      const int w = wg[g];
      const uint32_t prv = pw == w - 1 ? pcur : 0u;
      pw = w;
      pcur = cur[g];
      fn(w, cur[g] | (cur[g] << 1) | (prv >> 31), own[g]);
    }
  }
  if (wave_hi) fn(64, pw == 63 ? pcur >> 31 : 0u, 0u);  // word 64: top corners of cell word 63 (n = 2048)
}

// Outputs a tile stages in LDS before writing them out with coalesced stores
// (a tile's outputs are one contiguous range of each list); a tile with more
// writes its entries directly.  A staged entry is one 32-bit word, the
// thread's index in the tile above a 12-bit corner or cell index k (k <= n
// <= 2048); the flush rebuilds the list values from the tile's first column.
constexpr int kStageCorners = 4096;
constexpr int kStageCands = 3072;
constexpr int kStageKBits = 12;
static_assert(kBlock <= (1 << (32 - kStageKBits)), "thread index field");
static_assert(kMaxN < (1 << kStageKBits), "corner index field");
static_assert(kBlock == kLatTile, "a corner tile is one block of lattice columns");

// One thread per lattice column (a, b): its corner words, the index of each
// word's first corner within the tile, its corners, and, when (a, b) is also
// a cell column, its candidate cells; thread 0 writes the tile's first list
// index to lbase.  One packed scan: (candidates << 31) | corners.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_corners(Grid g, Workspace ws,
                                                                                        gh_counters* __restrict__ ctr) {
  __shared__ __align__(16) uint32_t s_c[kStageCorners];
  __shared__ uint32_t s_k[kStageCands];
  const int n = g.n, n1 = n + 1;
  const size_t ncol = (size_t)n * n, nl = (size_t)n1 * n1;
  // A new pass: the capacity flag of an earlier one goes.  Every tile that
  // can set it does so after its look-back has seen tile 0 (block 0), so the
  // clear comes first.
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAnd(&ctr->flags, ~GH_FLAG_CAPACITY);
  for (int tile = blockIdx.x; tile < (int)ws.tiles_lat; tile += gridDim.x) {
  __syncthreads();
  const size_t L = (size_t)tile * kBlock + threadIdx.x;
  LatAdj A{{0, 0, 0, 0}, {0, 0, 0, 0}, 0};
  if (L < nl) A = lat_adjacent(n, (int)(L / n1), (int)(L % n1), ws.colmask);
  // Slot 3 is the cell column (a, b); its mask is 0 on the lattice's far faces.
  const uint64_t own = A.mask[3];
  const size_t own_col = A.col[3];  // valid where own != 0
  const uint64_t wave_words = wave_uniform_or(A.uni | (A.uni << 1));
  const bool wave_hi = wave_uniform_or(A.uni >> 63) != 0;
  uint64_t ncorner = 0, ncand = 0;
  // Corner words go to the records lrec as they are found (they do not
  // depend on the scan); the write pass reads them back.
  uint64_t lm = 0;
  uint32_t hi = 0;
  const int words = (n + 31) >> 5, words1 = (n + 32) >> 5;
  walk_corner_words(A, ws.colbits, ncol, words, wave_words, wave_hi, [&](int w, uint32_t cw, uint32_t ow) {
    ncand += __popc(ow);
    if (!cw) return;
    if (w < 64) lm |= 1ull << w; else hi = 1u;
    ws.lrec[(size_t)w * nl + L] = cw;  // the word now, its first index in the write pass
    ncorner += __popc(cw);
  });
  // Two 31-bit fields share the scan word.  On grids whose totals can reach
  // 2^31 ((n + 1)^3 corners), where a carry would spill into the other field,
  // each tile's own counts (far below 2^31) also go, exact, into 64-bit
  // totals, which the last tile compares with the scan's.
  unsigned long long* const pc = pack_counts(ws);
  const bool exact = (int64_t)n1 * n1 * n1 >= ((int64_t)1 << 31);
  const LocalScan ls = block_scan_publish((ncand << 31) | ncorner, scan_corners(ws), tile, [pc, exact](uint64_t agg) {
    if (!exact) return;
    atomicAdd(&pc[0], (unsigned long long)(agg & 0x7fffffffull));
    atomicAdd(&pc[1], (unsigned long long)(agg >> 31));
    counts_done();
  });
  const uint64_t tile_c = ls.agg & 0x7fffffffull, tile_k = ls.agg >> 31;
  const bool stage_c = tile_c <= (uint64_t)kStageCorners, stage_k = tile_k <= (uint64_t)kStageCands;
  // A tile whose corners and candidates both fit the stage emits them before
  // its look-back, so that the write pass overlaps the wait for the
  // predecessors; the word records carry list indices relative to the tile's
  // first corner (lbase holds that), so they need no base either.
  const bool early = stage_c && stage_k;
  const uint32_t tag = (uint32_t)threadIdx.x << kStageKBits;
  int64_t o = 0, oc = 0;        // this thread's next corner and candidate, within the tile
  int64_t cdst = 0, kdst = 0;   // list index of the tile's first corner and candidate (direct writes)
  bool on = false;              // whether this thread emits
  // A full word (32 consecutive corners, the columns along a wall parallel
  // to them) goes out as 16-byte stores once its position is 4-aligned.
  auto emit_staged = [&](int w, uint32_t cw) {
    int64_t i = o;
    if (cw == 0xffffffffu) {
      const uint32_t e0 = tag | (uint32_t)(32 * w);
      int j = 0;
      for (; j < 32 && (i & 3); ++j, ++i) s_c[i] = e0 + j;
      for (; j + 4 <= 32; j += 4, i += 4)
        *reinterpret_cast<uint4*>(s_c + i) = make_uint4(e0 + j, e0 + j + 1, e0 + j + 2, e0 + j + 3);
      for (; j < 32; ++j, ++i) s_c[i] = e0 + j;
    } else {
      for (uint32_t bb = cw; bb; bb &= bb - 1, ++i) s_c[i] = tag | (uint32_t)(32 * w + __builtin_ctz(bb));
    }
    o = i;
  };
  auto emit_direct = [&](int w, uint32_t cw) {
    const int32_t Li = (int32_t)L;
    int32_t* __restrict__ dk = ws.ck;
    int32_t* __restrict__ dl = ws.cl;
    int64_t i = cdst + o;
    if (cw == 0xffffffffu) {
      const int32_t k0 = 32 * w;
      int j = 0;
      for (; j < 32 && (i & 3); ++j, ++i) {
        dk[i] = k0 + j;
        dl[i] = Li;
      }
      for (; j + 4 <= 32; j += 4, i += 4) {
        *reinterpret_cast<int4*>(dk + i) = make_int4(k0 + j, k0 + j + 1, k0 + j + 2, k0 + j + 3);
        *reinterpret_cast<int4*>(dl + i) = make_int4(Li, Li, Li, Li);
      }
      for (; j < 32; ++j, ++i) {
        dk[i] = k0 + j;
        dl[i] = Li;
      }
    } else {
      for (uint32_t bb = cw; bb; bb &= bb - 1, ++i) {
        dk[i] = 32 * w + __builtin_ctz(bb);
        dl[i] = Li;
      }
    }
    o = i - cdst;
  };
  auto put = [&](int w, uint32_t cw, uint32_t ow) {
    if (cw) ws.lrec[(size_t)w * nl + L] = ((uint64_t)(uint32_t)o << 32) | cw;
    if (stage_c) emit_staged(w, cw);
    else emit_direct(w, cw);
    for (uint32_t bb = ow; bb; bb &= bb - 1) {
      const int kc = 32 * w + __builtin_ctz(bb);
      if (stage_k) s_k[oc] = tag | (uint32_t)kc;
      else ws.cand[kdst + oc] = (int64_t)own_col * n + kc;
      ++oc;
    }
  };
  // Write pass over the wave's corner words, loads grouped as in the walk;
  // every own cell word w has corner word w.
  auto write_pass = [&]() {
    o = (int64_t)(ls.excl & 0x7fffffffull);
    oc = (int64_t)(ls.excl >> 31);
    const uint64_t wave_lm = wave_uniform_or(on ? lm : 0ull);
    const size_t Lq = L < nl ? L : 0;
    for (uint64_t r = wave_lm; r;) {
      int wg[kWalk];
      uint32_t cw[kWalk], ow[kWalk];
#pragma unroll
      for (int g = 0; g < kWalk; ++g) {
        const int w = r ? __builtin_ctzll(r) : -1;
        r &= r - 1;
        wg[g] = w;
        // unconditional loads at clamped in-bounds addresses, masked after
        const int wl = w >= 0 && w < words1 ? w : 0, wc = w >= 0 && w < words ? w : 0;
        const uint32_t lw = (uint32_t)ws.lrec[(size_t)wl * nl + Lq];
        const uint32_t cwd = ws.colbits[(size_t)wc * ncol + own_col];
        cw[g] = on && w >= 0 && ((lm >> w) & 1) ? lw : 0u;
        ow[g] = on && w >= 0 && ((own >> w) & 1) ? cwd : 0u;
      }
#pragma unroll
      for (int g = 0; g < kWalk; ++g)
        if (wg[g] >= 0) put(wg[g], cw[g], ow[g]);
    }
    if (on && hi) put(64, (uint32_t)ws.lrec[(size_t)64 * nl + L], 0u);
  };
  if (early) {
    on = L < nl;
    write_pass();
  }
  const uint64_t base = block_lookback(scan_corners(ws), tile, ls.agg, &ctr->flags);
  const uint64_t total = base + ls.agg;
  const uint64_t cbase = base & 0x7fffffffull, kbase = base >> 31;
  // a field that wrapped inside this tile: the pass is void (flagged by the
  // last tile), and this tile writes nothing
  const bool wrapped = (total & 0x7fffffffull) < cbase || (total >> 31) < kbase;
  const bool fits = !wrapped && L < nl && cbase + (ls.excl & 0x7fffffffull) + ncorner <= (uint64_t)ws.cap;
  if (!early) {
    on = fits;
    cdst = (int64_t)cbase;
    kdst = (int64_t)kbase;
    write_pass();
  }
  if (threadIdx.x == 0) ws.lbase[tile] = (int64_t)cbase;
  __syncthreads();
  const int32_t Lt = tile * kBlock;  // the tile's first lattice column
  if (stage_c && !wrapped)
    for (int64_t i = threadIdx.x; i < (int64_t)tile_c; i += kBlock) {
      const int64_t gi = (int64_t)cbase + i;
      const uint32_t e = s_c[i];
      if (gi < ws.cap) {
        ws.ck[gi] = (int32_t)(e & ((1u << kStageKBits) - 1));
        ws.cl[gi] = Lt + (int32_t)(e >> kStageKBits);
      }
    }
  if (stage_k && !wrapped)
    for (int64_t i = threadIdx.x; i < (int64_t)tile_k; i += kBlock) {
      const int64_t gi = (int64_t)kbase + i;
      const uint32_t e = s_k[i];
      // the staging thread's lattice column (a, b) is cell column (a, b)
      const int32_t Le = Lt + (int32_t)(e >> kStageKBits), a = Le / n1, b = Le - a * n1;
      if (gi < ws.cap) ws.cand[gi] = ((int64_t)a * n + b) * n + (int64_t)(e & ((1u << kStageKBits) - 1));
    }
  if (L < nl) {
    ws.lmask[L] = fits ? lm : 0ull;
    ws.lmhi[L] = fits ? hi : 0u;
  }
  if (threadIdx.x == 0 && tile == (int)ws.tiles_lat - 1) {
    // every tile added its counts before publishing them, so they are all in
    int64_t tc = (int64_t)(total & 0x7fffffffull), tk = (int64_t)(total >> 31);
    if (exact) {
      const unsigned long long ec = __hip_atomic_load(&pc[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned long long ek = __hip_atomic_load(&pc[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (ec != (unsigned long long)tc || ek != (unsigned long long)tk) {  // carried: at least 2^31 > cap
        tc = (int64_t)ec;
        tk = (int64_t)ek;
        atomicOr(&ctr->flags, GH_FLAG_CAPACITY);
      }
      __hip_atomic_store(&pc[0], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // zero for the next pass
      __hip_atomic_store(&pc[1], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    ws.nlist[0] = tc;
    ws.nlist[1] = tk;
    ctr->n_corner = tc;
    if (tc > ws.cap) atomicOr(&ctr->flags, GH_FLAG_CAPACITY);
  }
  }
}

// Bound value at each corner point, one lane per corner.
template <class Eval>
__global__ __launch_bounds__(kBlock) void k_eval_corners(Eval ev, Grid g, Workspace ws) {
  const int64_t m = ws.nlist[0];
  if (m > ws.cap) return;
  const int n1 = g.n + 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < m; c += stride) {
    const int L = ws.cl[c];
    const int a = L / n1, b = L - a * n1;
    ws.cf[c] = ev(lattice(g, a), lattice(g, b), lattice(g, ws.ck[c]));
  }
}

// ------------------------------------------------------------------ vertices
// One thread per corner (a, b, k): the crossing edges it owns are the x edge
// to (a+1, b, k), the y edge to (a, b+1, k) and the z edge to (a, b, k+1),
// when the far end is a corner too and the signs differ.

// Each thread takes kItems consecutive list entries (a launch shape: 1, 2, 4
// or 8), so a tile covers kBlock * kItems entries and the entries keep their
// order in the output.  The thread's run of a 4-byte list is read with the
// widest aligned vector loads (the lists are 256-byte aligned and c0 is a
// multiple of kItems); entries past the list end are read but never used.
template <int kItems, class T>
__device__ __forceinline__ void load_run(const T* __restrict__ p, int64_t c0, int64_t cap, T (&out)[kItems]) {
  static_assert(sizeof(T) == 4, "4-byte lists");
  if (c0 + kItems <= cap) {
    if constexpr (kItems >= 4) {
#pragma unroll
      for (int r = 0; r < kItems; r += 4) {
        const uint4 v = *reinterpret_cast<const uint4*>(p + c0 + r);
        out[r] = __builtin_bit_cast(T, v.x);
        out[r + 1] = __builtin_bit_cast(T, v.y);
        out[r + 2] = __builtin_bit_cast(T, v.z);
        out[r + 3] = __builtin_bit_cast(T, v.w);
      }
    } else if constexpr (kItems == 2) {
      const uint2 v = *reinterpret_cast<const uint2*>(p + c0);
      out[0] = __builtin_bit_cast(T, v.x);
      out[1] = __builtin_bit_cast(T, v.y);
    } else {
      out[0] = p[c0];
    }
  } else {
#pragma unroll
    for (int r = 0; r < kItems; ++r) out[r] = c0 + r < cap ? p[c0 + r] : T{};
  }
}

template <int kItems>
__global__ __launch_bounds__(kBlock) void k_verts(Grid g, Workspace ws, float* __restrict__ verts,
                                                  int64_t* __restrict__ vert_edge, float* __restrict__ vert_t,
                                                  int64_t vert_cap, gh_counters* __restrict__ ctr) {
  constexpr int kTileItems = kBlock * kItems;
  // A tile stages up to one vertex per corner (0.4 on average).
  constexpr int kStageV = kTileItems;
  __shared__ float s_v[3 * kStageV];
  __shared__ int64_t s_e[kStageV];
  __shared__ float s_t[kStageV];
  // The scans keep themselves clean for the next pass, so that a pass needs
  // no clearing launch: the corner scan is done, the triangle scan is next.
  // (After any pass the corner and vertex scans are zero; a hop clears all.)
  zero_words(scan_corners(ws), (size_t)ws.tiles_lat);
  zero_words(scan_tris(ws), (size_t)ws.tiles_cap);
  const int64_t m = ws.nlist[0];
  if (m > ws.cap) {  // uniform: the corners overflowed, nothing to do
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->n_vert = 0;
    return;
  }
  const int n = g.n, n1 = n + 1;
  const size_t nl = (size_t)n1 * n1;
  const int ntiles = (int)((m + kTileItems - 1) / kTileItems);
  if (ntiles == 0 && blockIdx.x == 0 && threadIdx.x == 0) ctr->n_vert = 0;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
    const int64_t c0 = (int64_t)tile * kTileItems + (int64_t)threadIdx.x * kItems;
    int32_t Ls[kItems], ks[kItems];
    float fs[kItems];
    load_run<kItems>(ws.cl, c0, ws.cap, Ls);
    load_run<kItems>(ws.ck, c0, ws.cap, ks);
    load_run<kItems>(ws.cf, c0, ws.cap, fs);
    // The entry after the run is the next lane's first (one wave covers
    // consecutive runs); the last lane reads it.
    int32_t Lz = __shfl_down(Ls[0], 1, 64), kz = __shfl_down(ks[0], 1, 64);
    float fz = __shfl_down(fs[0], 1, 64);
    const int64_t cz = c0 + kItems;
    if (lane_id() == 63 && cz < m) {
      Lz = ws.cl[cz];
      kz = ws.ck[cz];
      fz = ws.cf[cz];
    }
    // Straight-line and unconditional (entries past the list end use
    // lattice column 0 and are masked): the index loads of all items go out
    // together, then the value loads.
    unsigned msk[kItems];
    float fe[kItems][3];
    int64_t ix[kItems], iy[kItems];
    bool xo[kItems], yo[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const bool valid = c0 + r < m;
      const int L = valid ? Ls[r] : 0, k = valid ? ks[r] : 0;
      const int a = L / n1, b = L - a * n1;
      xo[r] = valid && a < n;
      yo[r] = valid && b < n;
      ix[r] = corner_index(ws, nl, (size_t)(xo[r] ? L + n1 : L), k);
      iy[r] = corner_index(ws, nl, (size_t)(yo[r] ? L + 1 : L), k);
      xo[r] = xo[r] && ix[r] >= 0;
      yo[r] = yo[r] && iy[r] >= 0;
    }
    unsigned cnt = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const int64_t ci = c0 + r;
      const float fx = ws.cf[xo[r] ? ix[r] : 0], fy = ws.cf[yo[r] ? iy[r] : 0];
      const bool neg = fs[r] < 0.f;
      const int Ln = r + 1 < kItems ? Ls[r + 1 < kItems ? r + 1 : 0] : Lz;
      const int kn = r + 1 < kItems ? ks[r + 1 < kItems ? r + 1 : 0] : kz;
      const float fn = r + 1 < kItems ? fs[r + 1 < kItems ? r + 1 : 0] : fz;
      const bool zn = ci + 1 < m && Ln == Ls[r] && kn == ks[r] + 1;
      fe[r][0] = xo[r] ? fx : 0.f;
      fe[r][1] = yo[r] ? fy : 0.f;
      fe[r][2] = zn ? fn : 0.f;
      msk[r] = 0;
      if (xo[r] && ((fx < 0.f) != neg)) msk[r] |= 1u;
      if (yo[r] && ((fy < 0.f) != neg)) msk[r] |= 2u;
      if (zn && ((fn < 0.f) != neg)) msk[r] |= 4u;
      cnt += __popc(msk[r]);
    }
    const LocalScan ls = block_scan_publish(cnt, scan_verts(ws), tile);
    const int64_t tile_v = (int64_t)ls.agg;
    const bool stage = tile_v <= kStageV;
    // Vertices of item r from vertex vv on (a place in the tile's stage or
    // in the output).
    auto put_verts = [&](int r, int64_t vv, bool staged) {
      const int L = Ls[r], k = ks[r];
      const int a = L / n1, b = L - a * n1;
      const float fa = fs[r];
      const float xa = lattice(g, a), ya = lattice(g, b), za = lattice(g, k);
      const int64_t pid = ((int64_t)L * n1 + k) * 3;
#pragma unroll
      for (int axis = 0; axis < 3; ++axis) {
        if (!((msk[r] >> axis) & 1)) continue;
        const float fb = fe[r][axis];
        const float t = fa / (fa - fb);
        const float px = axis == 0 ? xa + t * g.h : xa;
        const float py = axis == 1 ? ya + t * g.h : ya;
        const float pz = axis == 2 ? za + t * g.h : za;
        if (staged) {
          s_v[3 * vv + 0] = px;
          s_v[3 * vv + 1] = py;
          s_v[3 * vv + 2] = pz;
          s_e[vv] = pid + axis;
          s_t[vv] = t;
        } else {
          verts[3 * vv + 0] = px;
          verts[3 * vv + 1] = py;
          verts[3 * vv + 2] = pz;
          if (vert_edge) vert_edge[vv] = pid + axis;
          if (vert_t) vert_t[vv] = t;
        }
        ++vv;
      }
    };
    // A staged tile computes its vertices into LDS before the look-back, so
    // that this work overlaps the wait for the predecessors.
    if (stage) {
      int64_t lv = (int64_t)ls.excl;
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        if (c0 + r >= m) break;
        if (msk[r]) put_verts(r, lv, true);
        lv += __popc(msk[r]);
      }
    }
    const int64_t vbase = (int64_t)block_lookback(scan_verts(ws), tile, ls.agg, &ctr->flags);
    const uint64_t total = (uint64_t)vbase + ls.agg;
    int64_t v = vbase + (int64_t)ls.excl;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const int64_t ci = c0 + r;
      if (ci >= m) break;
      ws.cinfo[ci] = cinfo_pack(v, msk[r], fs[r] < 0.f);
      if (!stage && msk[r] && v + __popc(msk[r]) <= vert_cap) put_verts(r, v, false);
      v += __popc(msk[r]);
    }
    __syncthreads();
    if (stage) {
      const int64_t nv = vbase + tile_v <= vert_cap ? tile_v : (vbase < vert_cap ? vert_cap - vbase : 0);
      for (int64_t i = threadIdx.x; i < 3 * nv; i += kBlock) verts[3 * vbase + i] = s_v[i];
      if (vert_edge)
        for (int64_t i = threadIdx.x; i < nv; i += kBlock) vert_edge[vbase + i] = s_e[i];
      if (vert_t)
        for (int64_t i = threadIdx.x; i < nv; i += kBlock) vert_t[vbase + i] = s_t[i];
    }
    if (threadIdx.x == 0 && tile == ntiles - 1) {
      ctr->n_vert = (int64_t)total;
      if (total > (uint64_t)vert_cap) atomicOr(&ctr->flags, GH_FLAG_CAPACITY);
    }
  }
}

// ----------------------------------------------------------------- triangles
// One thread per candidate cell (i, j, k): list indices of its corners in
// the four lattice columns (i+dx, j+dy) (the corner at k+1 follows the one
// at k in the list), their corner words (sign, owned crossing edges, first
// vertex), the case byte, and the table's triangles; each triangle vertex is
// the welded vertex of the cell edge, found in the word of its lower corner.
// Lower corner of each of the 12 cell edges, 3 bits per edge.
constexpr uint64_t edge_lower_pack() {
  uint64_t v = 0;
  for (int e = 0; e < 12; ++e) v |= (uint64_t)mc_edge_lower(e) << (3 * e);
  return v;
}
constexpr uint64_t kEdgeLower = edge_lower_pack();

struct CellCorners {
  uint32_t info[8];  // corner word of corner dx + 2 dy + 4 dz
};

// The corners of a candidate are corners by construction, so their list
// indices need only the word records (one load each, issued together), then
// the eight corner words (a second round trip).  Returns false when a record
// lacks its corner (inconsistent workspace contents).
__device__ __forceinline__ bool cell_corners(const Workspace& ws, int n, size_t nl, int64_t cell, CellCorners& C,
                                             unsigned& cs) {
  const int n1 = n + 1;
  const int64_t col = cell / n;
  const int k = (int)(cell - col * n);
  const int i = (int)(col / n), j = (int)(col - (int64_t)i * n);
  const size_t L = (size_t)i * n1 + j;
  bool ok = true;
  int64_t p[4];
  p[0] = corner_index_known(ws, nl, L, k, &ok);
  p[1] = corner_index_known(ws, nl, L + n1, k, &ok);
  p[2] = corner_index_known(ws, nl, L + 1, k, &ok);
  p[3] = corner_index_known(ws, nl, L + n1 + 1, k, &ok);
  cs = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    // clamped into the list, so that even a corrupt record reads in bounds
    const int64_t p0 = p[q] < 0 ? 0 : (p[q] < ws.cap ? p[q] : ws.cap - 1);
    const int64_t p1 = p0 + 1 < ws.cap ? p0 + 1 : p0;
    C.info[q] = ws.cinfo[p0];
    C.info[q + 4] = ws.cinfo[p1];
    cs |= (C.info[q] & 1u) << q;
    cs |= (C.info[q + 4] & 1u) << (q + 4);
  }
  return ok;
}

template <int kItems>
__global__ __launch_bounds__(kBlock) void k_tris(Grid g, Workspace ws, int32_t* __restrict__ tris, int64_t tri_cap,
                                                 int64_t* __restrict__ cells, uint8_t* __restrict__ cases,
                                                 int64_t cell_cap, int64_t vert_cap,
                                                 gh_counters* __restrict__ ctr) {
  constexpr int kTileItems = kBlock * kItems;
  // A tile stages up to 1.5 triangles per candidate (about 1.5 on average
  // for closed surfaces; a larger tile writes directly) and every cell.
  constexpr int kStageT = 3 * kTileItems / 2;
  __shared__ McCase s_mc[256];
  __shared__ int32_t s_tri[3 * kStageT];
  __shared__ int64_t s_cell[kTileItems];
  __shared__ uint8_t s_case[kTileItems];
  s_mc[threadIdx.x] = g_mc.c[threadIdx.x];
  __syncthreads();
  zero_words(scan_verts(ws), (size_t)ws.tiles_cap);  // done with; zero for the next pass
  if (ws.nlist[0] > ws.cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctr->n_tri = 0;
      ctr->n_cells = 0;
    }
    return;
  }
  const int64_t m = ws.nlist[1];
  const int n = g.n;
  const size_t nl = (size_t)(n + 1) * (n + 1);
  const bool verts_ok = ctr->n_vert <= vert_cap;
  const int ntiles = (int)((m + kTileItems - 1) / kTileItems);
  if (ntiles == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    ctr->n_tri = 0;
    ctr->n_cells = 0;
  }
  bool broken = false;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
    const int64_t q0 = (int64_t)tile * kTileItems + (int64_t)threadIdx.x * kItems;
    CellCorners C[kItems];
    unsigned cs[kItems], nt[kItems];
    int64_t cell[kItems];
    uint64_t pack = 0;
    bool vec = false;
    if constexpr (kItems >= 2) {
      // 16-byte loads of the thread's run of cell ids (as in load_run)
      vec = q0 + kItems <= ws.cap;
      if (vec)
#pragma unroll
        for (int r = 0; r < kItems; r += 2) {
          const uint4 v = *reinterpret_cast<const uint4*>(ws.cand + q0 + r);
          cell[r] = (int64_t)(((uint64_t)v.y << 32) | v.x);
          cell[r + 1] = (int64_t)(((uint64_t)v.w << 32) | v.z);
        }
    }
    if (!vec)
#pragma unroll
      for (int r = 0; r < kItems; ++r) cell[r] = q0 + r < m ? ws.cand[q0 + r] : 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const bool valid = q0 + r < m;
      if (!valid) cell[r] = 0;  // cell 0 keeps every address in bounds; masked below
      const bool ok = cell_corners(ws, n, nl, cell[r], C[r], cs[r]);
      nt[r] = valid && ok ? s_mc[cs[r]].ntri : 0u;
      broken = broken || (valid && !ok);
      // (cells << 31) | triangles: both stay below 2^31 for any mesh the outputs can index
      pack += ((uint64_t)(nt[r] ? 1 : 0) << 31) | nt[r];
    }
    // exact 64-bit totals beside the packed scan where the triangles (at
    // most 5 n^3) can reach 2^31, as in the corner pass
    unsigned long long* const pc = pack_counts(ws);
    const bool exact = (int64_t)5 * n * n * n >= ((int64_t)1 << 31);
    const LocalScan ls = block_scan_publish(pack, scan_tris(ws), tile, [pc, exact](uint64_t agg) {
      if (!exact) return;
      atomicAdd(&pc[2], (unsigned long long)(agg & 0x7fffffffull));
      atomicAdd(&pc[3], (unsigned long long)(agg >> 31));
      counts_done();
    });
    const int64_t tile_t = (int64_t)(ls.agg & 0x7fffffffull), tile_c = (int64_t)(ls.agg >> 31);
    const int64_t lt = (int64_t)(ls.excl & 0x7fffffffull), lc = (int64_t)(ls.excl >> 31);  // within the tile
    const bool stage = tile_t <= kStageT;  // the cells always fit: at most one per candidate
    // Welded vertex ids of item r's triangles, from triangle t on.
    auto put_tris = [&](int r, int64_t t, int32_t* __restrict__ dst) {
      const McCase mcc = s_mc[cs[r]];
#pragma unroll
      for (unsigned tq = 0; tq < 5; ++tq) {
        if (tq >= nt[r]) break;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          const int e = (int)((mcc.tri >> (12 * tq + 4 * v)) & 15);
          const int lcr = (int)((kEdgeLower >> (3 * e)) & 7), axis = e >> 2;
          uint32_t in = C[r].info[0];
#pragma unroll
          for (int q = 1; q < 7; ++q) in = lcr == q ? C[r].info[q] : in;
          dst[3 * (t + tq) + v] = (int32_t)(cinfo_vbase(in) + __popc(cinfo_mask(in) & ((1u << axis) - 1u)));
        }
      }
    };
    // Cells, cases and a staged tile's triangles go to LDS at their places in
    // the tile before the look-back, so that this work overlaps the wait for
    // the predecessors; only the flush needs the tile's place in the lists.
    if (verts_ok) {
      int64_t t = lt, c = lc;
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        if (!nt[r]) continue;
        s_cell[c] = cell[r];
        s_case[c] = (uint8_t)cs[r];
        if (stage) put_tris(r, t, s_tri);
        t += nt[r];
        ++c;
      }
    }
    const uint64_t base = block_lookback(scan_tris(ws), tile, ls.agg, &ctr->flags);
    const uint64_t total = base + ls.agg;
    const int64_t tbase = (int64_t)(base & 0x7fffffffull), cbase = (int64_t)(base >> 31);
    // a field wrapped here: the pass is void, write nothing
    const bool wrapped = (int64_t)(total & 0x7fffffffull) < tbase || (int64_t)(total >> 31) < cbase;
    if (verts_ok && !wrapped && !stage) {
      int64_t t0 = tbase + lt;
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        if (!nt[r]) continue;
        if (t0 + (int64_t)nt[r] <= tri_cap) put_tris(r, t0, tris);
        t0 += nt[r];
      }
    }
    __syncthreads();
    if (verts_ok && !wrapped) {
      if (stage) {
        const int64_t nt3 = 3 * (tbase + tile_t <= tri_cap ? tile_t : (tbase < tri_cap ? tri_cap - tbase : 0));
        for (int64_t i = threadIdx.x; i < nt3; i += kBlock) tris[3 * tbase + i] = s_tri[i];
      }
      const int64_t nc = cbase + tile_c <= cell_cap ? tile_c : (cbase < cell_cap ? cell_cap - cbase : 0);
      if (cells)
        for (int64_t i = threadIdx.x; i < nc; i += kBlock) cells[cbase + i] = s_cell[i];
      if (cases)
        for (int64_t i = threadIdx.x; i < nc; i += kBlock) cases[cbase + i] = s_case[i];
    }
    if (threadIdx.x == 0 && tile == ntiles - 1) {
      int64_t tt = (int64_t)(total & 0x7fffffffull), tc = (int64_t)(total >> 31);
      if (exact) {
        const unsigned long long et = __hip_atomic_load(&pc[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long ec = __hip_atomic_load(&pc[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (et != (unsigned long long)tt || ec != (unsigned long long)tc) {  // carried: at least 2^31 > tri_cap
          tt = (int64_t)et;
          tc = (int64_t)ec;
          atomicOr(&ctr->flags, GH_FLAG_CAPACITY);
        }
        __hip_atomic_store(&pc[2], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // zero for the next pass
        __hip_atomic_store(&pc[3], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      ctr->n_tri = tt;
      ctr->n_cells = tc;
      if (tt > tri_cap || ((cells || cases) && tc > cell_cap)) atomicOr(&ctr->flags, GH_FLAG_CAPACITY);
    }
  }
  if (broken) atomicOr(&ctr->flags, GH_FLAG_INTERNAL);
}

hipError_t launch_candidates(const Grid& g, const Workspace& ws, int64_t* out, int64_t cap, gh_counters* ctr,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_candidates, dim3(resident_grid(k_candidates, ws.tiles_col)), dim3(kBlock), 0, s, g, ws, out,
                     cap, ctr);
  return hipGetLastError();
}

hipError_t launch_mc(const DevSdb& d, const Grid& g, const Workspace& ws, float* verts, int64_t* vert_edge,
                     float* vert_t, int64_t vert_cap, int32_t* tris, int64_t tri_cap, int64_t* cells,
                     uint8_t* cases, int64_t cell_cap, gh_counters* ctr, hipStream_t s) {
  if (d.kind != GH_SDB_PRIMS && d.kind != GH_SDB_MLP) return hipErrorInvalidValue;
  const int items = current_tuning().mc_items_per_thread;
  const int64_t list_tiles = (ws.cap + (int64_t)kBlock * items - 1) / ((int64_t)kBlock * items);
  hipLaunchKernelGGL(k_corners, dim3(resident_grid(k_corners, ws.tiles_lat)), dim3(kBlock), 0, s, g, ws, ctr);
  if (d.kind == GH_SDB_MLP) {
    const hipError_t e = launch_mlp(1, d, g, &ws, nullptr, nullptr, nullptr, 0, ctr, s);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_eval_corners<PrimsEval>, dim3(persistent_blocks(ws.cap)), dim3(kBlock), 0, s,
                       PrimsEval{d.prims, d.groups}, g, ws);
  }
  auto emit = [&](auto kv, auto kt) {
    hipLaunchKernelGGL(kv, dim3(resident_grid(kv, list_tiles)), dim3(kBlock), 0, s, g, ws, verts, vert_edge, vert_t,
                       vert_cap, ctr);
    hipLaunchKernelGGL(kt, dim3(resident_grid(kt, list_tiles)), dim3(kBlock), 0, s, g, ws, tris, tri_cap, cells,
                       cases, cell_cap, vert_cap, ctr);
  };
  switch (items) {
    case 1: emit(k_verts<1>, k_tris<1>); break;
    case 2: emit(k_verts<2>, k_tris<2>); break;
    case 8: emit(k_verts<8>, k_tris<8>); break;
    default: emit(k_verts<4>, k_tris<4>); break;
  }
  return hipGetLastError();
}


}  // namespace gh
