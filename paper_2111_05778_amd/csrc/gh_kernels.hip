// Grid hopping and marching-cubes kernels for gfx950, with host launchers.
//
// Pipeline of one polygonization (all on one stream):
//   k_clear      reset counters and look-back words
//   k_hop        one lane per ray column: hop rule, candidate bitmap
//   k_corners    per lattice column: distinct corners of candidate cells,
//                single-pass scan -> CSR offsets, corner list
//   k_eval       bound at every corner, one lane per corner
//   k_verts      per lattice column: crossing edges owned by each corner,
//                scan -> one welded vertex per crossing lattice edge
//   k_tris       per cell column: case byte, triangles from the table,
//                scan -> triangle and cell emit
// Enumeration replaces k_hop by k_dense_eval + k_dense_classify.

#include <float.h>

#include <algorithm>
#include <atomic>

#include "gh_device.h"
#include "gh_launch.h"
#include "gh_layout.h"
#include "gh_hop.h"
#include "mc_table.h"

namespace gh {

__constant__ McTable g_mc = kMcTable;

// ------------------------------------------------------------------ clear
// Zeroes scan[begin, end), the given tickets and, per mode, the counters:
// all of them before a hop, the marching-cubes ones before gh_mc.
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
    }
    if (mode == kClearAll || mode == kClearMc) {
      ctr->n_corner = 0;
      ctr->n_cells = 0;
      ctr->n_vert = 0;
      ctr->n_tri = 0;
      ctr->flags &= ~GH_FLAG_CAPACITY;
    }
  }
}

// --------------------------------------------------------------------- hop
template <int R, bool kRegs>
__global__ __launch_bounds__(kBlock) void k_hop_prims(const float* __restrict__ prims, PrimGroups groups, Grid g,
                                                      uint64_t* __restrict__ colmask, uint32_t* __restrict__ colbits,
                                                      gh_counters* __restrict__ ctr) {
  __shared__ float4 s_rec[kMaxPrims * GH_PRIM_FLOATS / 4];
  stage_prims(s_rec, prims, groups.start[kPrimTypes]);
  hop_prims_tile<R, kRegs>(reinterpret_cast<const float*>(s_rec), groups, g, colmask, colbits, ctr, blockIdx.x);
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

// ------------------------------------------------------------------ corners
// Candidate words of the (up to four) cell columns around lattice column
// (a, b); a missing or empty column has mask 0.  Fixed-size and unrolled so
// that everything stays in registers.
struct LatAdj {
  size_t col[4];
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
    const size_t c = ok ? (size_t)i * n + j : 0;
    const uint64_t m = ok ? colmask[c] : 0ull;
    A.col[q] = c;
    A.mask[q] = m;
    A.uni |= m;
  }
  return A;
}

__device__ __forceinline__ uint32_t adj_cell_word(const LatAdj& A, const uint32_t* __restrict__ colbits,
                                                  size_t ncol, int w) {
  uint32_t v = 0;
  if (w < 0 || w >= 64) return 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if ((A.mask[q] >> w) & 1) v |= colbits[(size_t)w * ncol + A.col[q]];
  return v;
}

// Lattice points k of column (a, b) that are corners of a candidate cell:
// cell k of an adjacent column has corners k and k + 1.
__device__ __forceinline__ uint32_t corner_word(const LatAdj& A, const uint32_t* __restrict__ colbits, size_t ncol,
                                                int w) {
  const uint32_t cur = adj_cell_word(A, colbits, ncol, w);
  const uint32_t prev = adj_cell_word(A, colbits, ncol, w - 1);
  return cur | (cur << 1) | (prev >> 31);
}

template <class F>
__device__ __forceinline__ void for_corner_words(const LatAdj& A, F&& fn) {
  const uint64_t cw = A.uni | (A.uni << 1);
  for (uint64_t r = cw; r; r &= r - 1) fn(__builtin_ctzll(r));
  if ((A.uni >> 63) & 1) fn(64);
}

// One thread per lattice column (a, b): its corner words, their starting
// list indices, its corners, and, when (a, b) is also a cell column, its
// candidate cells.  One packed scan: (candidates << 31) | corners.
__global__ __launch_bounds__(kBlock) void k_corners(Grid g, Workspace ws, gh_counters* __restrict__ ctr) {
  const int n = g.n, n1 = n + 1;
  const size_t ncol = (size_t)n * n, nl = (size_t)n1 * n1;
  for (int tile = blockIdx.x; tile < (int)ws.tiles_lat; tile += gridDim.x) {
  __syncthreads();
  const size_t L = (size_t)tile * kBlock + threadIdx.x;
  LatAdj A{{0, 0, 0, 0}, {0, 0, 0, 0}, 0};
  int a = 0, b = 0;
  uint64_t ncorner = 0, ncand = 0, own = 0;
  size_t own_col = 0;
  // The first kCache corner words are kept for the write pass (most columns
  // have fewer); the rest are recomputed there.
  constexpr int kCache = 4;
  int cw_w[kCache];
  uint32_t cw_v[kCache];
  int nw = 0;
  if (L < nl) {
    a = (int)(L / n1);
    b = (int)(L % n1);
    A = lat_adjacent(n, a, b, ws.colmask);
    for_corner_words(A, [&](int w) {
      const uint32_t cw = corner_word(A, ws.colbits, ncol, w);
#pragma unroll
      for (int i = 0; i < kCache; ++i)
        if (i == nw) {
          cw_w[i] = w;
          cw_v[i] = cw;
        }
      ++nw;
      ncorner += __popc(cw);
    });
    if (a < n && b < n) {  // cell column (a, b) is slot 3 of the adjacency
      own = A.mask[3];
      own_col = A.col[3];
      for (uint64_t r = own; r; r &= r - 1) ncand += __popc(ws.colbits[(size_t)__builtin_ctzll(r) * ncol + own_col]);
    }
  }
  const ScanOut so = block_scan_lookback((ncand << 31) | ncorner, scan_corners(ws), tile, &ctr->flags);
  const uint64_t c0 = so.excl & 0x7fffffffull, k0 = so.excl >> 31;
  if (L < nl) {
    uint64_t lm = 0;
    uint32_t hi = 0;
    if (c0 + ncorner <= (uint64_t)ws.cap) {
      int64_t o = (int64_t)c0;
      auto put = [&](int w, uint32_t cw) {
        if (!cw) return;
        if (w < 64) lm |= 1ull << w; else hi = 1u;
        ws.lbits[(size_t)w * nl + L] = cw;
        ws.lwst[(size_t)w * nl + L] = (int32_t)o;
        for (uint32_t bb = cw; bb; bb &= bb - 1) {
          ws.ck[o] = 32 * w + __builtin_ctz(bb);
          ws.cl[o] = (int32_t)L;
          ++o;
        }
      };
      if (nw <= kCache) {
#pragma unroll
        for (int i = 0; i < kCache; ++i)
          if (i < nw) put(cw_w[i], cw_v[i]);
      } else {
        for_corner_words(A, [&](int w) { put(w, corner_word(A, ws.colbits, ncol, w)); });
      }
      int64_t oc = (int64_t)k0;
      for (uint64_t r = own; r; r &= r - 1) {
        const int w = __builtin_ctzll(r);
        for (uint32_t bb = ws.colbits[(size_t)w * ncol + own_col]; bb; bb &= bb - 1)
          ws.cand[oc++] = (int64_t)own_col * n + 32 * w + __builtin_ctz(bb);
      }
    }
    ws.lmask[L] = lm;
    ws.lmhi[L] = hi;
  }
  if (threadIdx.x == 0 && tile == (int)ws.tiles_lat - 1) {
    const int64_t tc = (int64_t)(so.total & 0x7fffffffull), tk = (int64_t)(so.total >> 31);
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
// Crossing edges of corner ci towards +x, +y, +z (bits 0..2); fe[axis] gets
// the value at the far end of each crossing edge, so the vertex pass needs
// no second round of loads.
__device__ __forceinline__ unsigned cross_mask(const Workspace& ws, const Grid& g, size_t nl, int64_t ci, int64_t m,
                                               float (&fe)[3]) {
  const int n = g.n, n1 = n + 1;
  const int L = ws.cl[ci], k = ws.ck[ci];
  const int a = L / n1, b = L - a * n1;
  const bool neg = ws.cf[ci] < 0.f;
  unsigned msk = 0;
  const int64_t ix = a < n ? corner_index(ws, nl, (size_t)L + n1, k) : -1;
  const int64_t iy = b < n ? corner_index(ws, nl, (size_t)L + 1, k) : -1;
  fe[0] = ix >= 0 ? ws.cf[ix] : 0.f;
  fe[1] = iy >= 0 ? ws.cf[iy] : 0.f;
  const bool zn = ci + 1 < m && ws.cl[ci + 1] == L && ws.ck[ci + 1] == k + 1;
  fe[2] = zn ? ws.cf[ci + 1] : 0.f;
  if (ix >= 0 && ((fe[0] < 0.f) != neg)) msk |= 1u;
  if (iy >= 0 && ((fe[1] < 0.f) != neg)) msk |= 2u;
  if (zn && ((fe[2] < 0.f) != neg)) msk |= 4u;
  return msk;
}

// Each thread takes kItems consecutive list entries (a launch shape: 1, 2, 4
// or 8), so a tile covers kBlock * kItems entries and the entries keep their
// order in the output.

template <int kItems>
__global__ __launch_bounds__(kBlock) void k_verts(Grid g, Workspace ws, float* __restrict__ verts,
                                                  int64_t* __restrict__ vert_edge, float* __restrict__ vert_t,
                                                  int64_t vert_cap, gh_counters* __restrict__ ctr) {
  constexpr int kTileItems = kBlock * kItems;
  const int64_t m = ws.nlist[0];
  if (m > ws.cap) return;  // uniform: the corners overflowed, nothing to do
  const int n1 = g.n + 1;
  const size_t nl = (size_t)n1 * n1;
  const int ntiles = (int)((m + kTileItems - 1) / kTileItems);
  if (ntiles == 0 && blockIdx.x == 0 && threadIdx.x == 0) ctr->n_vert = 0;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
    const int64_t c0 = (int64_t)tile * kTileItems + (int64_t)threadIdx.x * kItems;
    unsigned msk[kItems];
    float fe[kItems][3];
    unsigned cnt = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      msk[r] = 0;
      if (c0 + r < m) msk[r] = cross_mask(ws, g, nl, c0 + r, m, fe[r]);
      cnt += __popc(msk[r]);
    }
    const ScanOut so = block_scan_lookback(cnt, scan_verts(ws), tile, &ctr->flags);
    int64_t v = (int64_t)so.excl;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const int64_t ci = c0 + r;
      if (ci >= m) break;
      ws.cinfo[ci] = (v << 3) | (int64_t)msk[r];
      if (msk[r] && v + __popc(msk[r]) <= vert_cap) {
        const int L = ws.cl[ci], k = ws.ck[ci];
        const int a = L / n1, b = L - a * n1;
        const float fa = ws.cf[ci];
        const float xa = lattice(g, a), ya = lattice(g, b), za = lattice(g, k);
        const int64_t pid = ((int64_t)L * n1 + k) * 3;
        int64_t vv = v;
#pragma unroll
        for (int axis = 0; axis < 3; ++axis) {
          if (!((msk[r] >> axis) & 1)) continue;
          const float fb = fe[r][axis];
          const float t = fa / (fa - fb);
          verts[3 * vv + 0] = axis == 0 ? xa + t * g.h : xa;
          verts[3 * vv + 1] = axis == 1 ? ya + t * g.h : ya;
          verts[3 * vv + 2] = axis == 2 ? za + t * g.h : za;
          if (vert_edge) vert_edge[vv] = pid + axis;
          if (vert_t) vert_t[vv] = t;
          ++vv;
        }
      }
      v += __popc(msk[r]);
    }
    if (threadIdx.x == 0 && tile == ntiles - 1) {
      ctr->n_vert = (int64_t)so.total;
      if (so.total > (uint64_t)vert_cap) atomicOr(&ctr->flags, GH_FLAG_CAPACITY);
    }
  }
}

// ----------------------------------------------------------------- triangles
// One thread per candidate cell (i, j, k): list indices of its corners in
// the four lattice columns (i+dx, j+dy) (the corner at k+1 follows the one
// at k in the list), the case byte, and the table's triangles; each triangle
// vertex is the welded vertex of the cell edge, found at its lower corner.
struct CellCorners {
  int64_t p[4];  // list index of corner (i+dx, j+dy, k), slot dx + 2 dy
};

__device__ __forceinline__ bool cell_corners(const Workspace& ws, int n, size_t nl, int64_t cell, CellCorners& C,
                                             unsigned& cs, int& k) {
  const int n1 = n + 1;
  const int64_t col = cell / n;
  k = (int)(cell - col * n);
  const int i = (int)(col / n), j = (int)(col - (int64_t)i * n);
  const size_t L = (size_t)i * n1 + j;
  C.p[0] = corner_index(ws, nl, L, k);
  C.p[1] = corner_index(ws, nl, L + n1, k);
  C.p[2] = corner_index(ws, nl, L + 1, k);
  C.p[3] = corner_index(ws, nl, L + n1 + 1, k);
  cs = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (C.p[q] < 0) return false;
    cs |= (unsigned)(ws.cf[C.p[q]] < 0.f) << q;
    cs |= (unsigned)(ws.cf[C.p[q] + 1] < 0.f) << (q + 4);
  }
  return true;
}

template <int kItems>
__global__ __launch_bounds__(kBlock) void k_tris(Grid g, Workspace ws, int32_t* __restrict__ tris, int64_t tri_cap,
                                                 int64_t* __restrict__ cells, uint8_t* __restrict__ cases,
                                                 int64_t cell_cap, int64_t vert_cap,
                                                 gh_counters* __restrict__ ctr) {
  constexpr int kTileItems = kBlock * kItems;
  __shared__ McCase s_mc[256];
  s_mc[threadIdx.x] = g_mc.c[threadIdx.x];
  __syncthreads();
  if (ws.nlist[0] > ws.cap) return;
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
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      cs[r] = nt[r] = 0;
      cell[r] = 0;
      C[r] = CellCorners{{0, 0, 0, 0}};
      if (q0 + r < m) {
        int k;
        cell[r] = ws.cand[q0 + r];
        if (cell_corners(ws, n, nl, cell[r], C[r], cs[r], k)) nt[r] = s_mc[cs[r]].ntri;
        else broken = true;
      }
      // (cells << 31) | triangles: both stay below 2^31 for any mesh the outputs can index
      pack += ((uint64_t)(nt[r] ? 1 : 0) << 31) | nt[r];
    }
    const ScanOut so = block_scan_lookback(pack, scan_tris(ws), tile, &ctr->flags);
    int64_t t0 = (int64_t)(so.excl & 0x7fffffffull), c = (int64_t)(so.excl >> 31);
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      if (!nt[r]) continue;
      if (verts_ok) {
        if (c < cell_cap) {
          if (cells) cells[c] = cell[r];
          if (cases) cases[c] = (uint8_t)cs[r];
        }
        if (t0 + (int64_t)nt[r] <= tri_cap) {
          const McCase mcc = s_mc[cs[r]];
          for (unsigned tq = 0; tq < nt[r]; ++tq) {
#pragma unroll
            for (int v = 0; v < 3; ++v) {
              const int e = (int)((mcc.tri >> (12 * tq + 4 * v)) & 15);
              const int lc = mc_edge_lower(e), axis = e >> 2;
              const int slot = (lc & 1) + 2 * ((lc >> 1) & 1);
              const int64_t base =
                  slot == 0 ? C[r].p[0] : (slot == 1 ? C[r].p[1] : (slot == 2 ? C[r].p[2] : C[r].p[3]));
              const int64_t info = ws.cinfo[base + (lc >> 2)];
              tris[3 * (t0 + tq) + v] = (int32_t)((info >> 3) + __popc((unsigned)(info & 7) & ((1u << axis) - 1u)));
            }
          }
        }
      }
      t0 += nt[r];
      ++c;
    }
    if (threadIdx.x == 0 && tile == ntiles - 1) {
      const int64_t tt = (int64_t)(so.total & 0x7fffffffull), tc = (int64_t)(so.total >> 31);
      ctr->n_tri = tt;
      ctr->n_cells = tc;
      if (tt > tri_cap || ((cells || cases) && tc > cell_cap)) atomicOr(&ctr->flags, GH_FLAG_CAPACITY);
    }
  }
  if (broken) atomicOr(&ctr->flags, GH_FLAG_INTERNAL);
}

// Bound at arbitrary points.
template <class Eval>
__global__ __launch_bounds__(kBlock) void k_eval_points(Eval ev, const float* __restrict__ xyz, float* __restrict__ f,
                                                        int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += stride)
    f[p] = ev(xyz[3 * p], xyz[3 * p + 1], xyz[3 * p + 2]);
}

// ================================================================ launchers
static int persistent_blocks(int64_t work) {
  const int64_t want = (work + kBlock - 1) / kBlock;
  return (int)(want < 1 ? 1 : (want > 2048 ? 2048 : want));
}

hipError_t launch_clear(const Workspace& ws, gh_counters* ctr, ClearMode mode, hipStream_t s) {
  size_t begin = 0, end = scan_words(ws);
  unsigned tmask = 0xffu;
  if (mode == kClearMc) {
    end = (size_t)(scan_cands(ws) - ws.scan);
    tmask = (1u << kTicketCorners) | (1u << kTicketVerts) | (1u << kTicketTris);
  } else if (mode == kClearCands) {
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
  if (most <= R)
    hipLaunchKernelGGL((k_hop_prims<R, true>), dim3(nbh * nbw), dim3(kBlock), 0, s, d.prims, d.groups, g,
                       ws.colmask, ws.colbits, ctr);
  else
    hipLaunchKernelGGL((k_hop_prims<R, false>), dim3(nbh * nbw), dim3(kBlock), 0, s, d.prims, d.groups, g,
                       ws.colmask, ws.colbits, ctr);
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

// Look-back kernels run block-strided over their tiles with a grid no larger
// than the number of blocks the device holds at once: every tile a block
// waits on then belongs to a resident block that only waits on earlier
// tiles, so the scan always makes progress (no ticket counter needed).
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

template <class K>
static int resident_grid(K kernel, int64_t tiles) {
  const int cus = cu_count();
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  // One block per tile whenever every tile fits at once; otherwise the
  // tuned number of resident blocks per CU walks the tiles.
  if (tiles <= (int64_t)cus * per_cu) return (int)(tiles < 1 ? 1 : tiles);
  const int want = current_tuning().scan_blocks_per_cu;
  const int64_t cap = (int64_t)cus * (per_cu < want ? per_cu : want);
  const int64_t gsz = tiles < cap ? tiles : cap;
  return (int)(gsz < 1 ? 1 : gsz);
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

hipError_t launch_eval_points(const DevSdb& d, const float* xyz, float* f, int64_t m, hipStream_t s) {
  if (d.kind == GH_SDB_MLP) return launch_mlp(0, d, Grid{}, nullptr, nullptr, xyz, f, m, nullptr, s);
  if (d.kind != GH_SDB_PRIMS) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_eval_points<PrimsEval>, dim3(persistent_blocks(m)), dim3(kBlock), 0, s,
                     PrimsEval{d.prims, d.groups}, xyz, f, m);
  return hipGetLastError();
}

}  // namespace gh
