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
