// Workspace layout of one polygonization, carved from a caller-owned buffer.
//
// Candidate cells are kept per ray column as a bitmap over k (the hop writes
// only the non-zero 32-bit words and a 64-bit mask saying which words exist),
// so nothing has to be cleared between runs.  Corner points are listed by
// lattice column (a, b), then k; per lattice column a word bitmap over k with
// the index of each word's first corner (one 8-byte record per word, the
// index counted from the first corner of its tile of kLatTile lattice
// columns, whose list index lbase holds) gives any corner's list index in
// O(1).  Each corner carries its bound
// value and one 32-bit word with its sign, the crossing edges it owns and
// the index of its first welded vertex.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "gh.h"

namespace gh {

struct Workspace {
  uint64_t* colmask;   // [n*n] bit w set when word w of the column bitmap was written
  uint32_t* colbits;   // [W][n*n] candidate bitmap words, word-major (W = ceil(n/32))
  uint64_t* lmask;     // [(n+1)^2] bit w set when corner word w of lattice column L exists (w < 64)
  uint32_t* lmhi;      // [(n+1)^2] bit 0: corner word 64 exists (n = 2048 only)
  uint64_t* lrec;      // [W1][(n+1)^2] corner word w of a lattice column (k bits, low half) and the index of
                       // its first corner within the column's tile (high half), written where non-zero
                       // (W1 = ceil((n+1)/32))
  int64_t* lbase;      // [tiles_lat] list index of the first corner of each tile of lattice columns
  int32_t* ck;         // [cap] k of each corner (list ordered by lattice column, then k)
  int32_t* cl;         // [cap] lattice column a*(n+1) + b of each corner
  float* cf;           // [cap] bound value at the corner
  uint32_t* cinfo;     // [cap] (first vertex index << 4) | (crossing mask << 1) | (f < 0); mask x=1, y=2, z=4
  int64_t* cand;       // [cap] candidate cell ids in ascending order (never more than the corners)
  int64_t* nlist;      // [2] corners, candidates in the lists
  uint32_t* park;      // [n*n][6] rays handed to the long-ray pass: column, k, word index, word, mask lo/hi
  uint64_t* scan;      // look-back words: corners, vertices, triangles, candidates export
  unsigned int* ticket;// [8] tile tickets (one per scan) and spare
  int64_t cap;         // corner capacity
  int64_t tiles_lat;   // tiles over lattice columns
  int64_t tiles_col;   // tiles over cell columns
  int64_t tiles_cap;   // tiles over a list of cap items
  int words1;          // W1
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr int kPackCounts = 4;  // 64-bit words after the look-back words (see pack_counts)
constexpr int kLatTile = 256;   // lattice columns per corner tile

// Computes the layout; with base == nullptr only the size is produced.
inline size_t workspace_layout(int n, int64_t cap, void* base, Workspace* ws) {
  const size_t n2 = (size_t)n * n, n1 = (size_t)n + 1, nl = n1 * n1;
  const size_t words = ((size_t)n + 31) / 32, words1 = ((size_t)n + 32) / 32;
  const int64_t tiles_lat = (int64_t)((nl + kLatTile - 1) / kLatTile);
  const int64_t tiles_col = (int64_t)((n2 + 255) / 256);
  const int64_t tiles_cap = (int64_t)(((size_t)cap + 255) / 256);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t o_mask = take(n2 * 8);
  const size_t o_bits = take(words * n2 * 4);
  const size_t o_lmask = take(nl * 8);
  const size_t o_lmhi = take(nl * 4);
  const size_t o_lrec = take(words1 * nl * 8);
  const size_t o_lbase = take((size_t)tiles_lat * 8);
  const size_t o_ck = take((size_t)cap * 4);
  const size_t o_cl = take((size_t)cap * 4);
  const size_t o_cf = take((size_t)cap * 4);
  const size_t o_ci = take((size_t)cap * 4);
  const size_t o_cand = take((size_t)cap * 8);
  const size_t o_nlist = take(2 * 8);
  const size_t o_park = take(n2 * 6 * 4);
  const size_t scan_words = (size_t)(tiles_lat + 2 * tiles_cap + tiles_col) + kPackCounts;
  const size_t o_scan = take(scan_words * 8);
  const size_t o_ticket = take(8 * sizeof(unsigned int));
  if (base && ws) {
    char* b = (char*)base;
    ws->colmask = (uint64_t*)(b + o_mask);
    ws->colbits = (uint32_t*)(b + o_bits);
    ws->lmask = (uint64_t*)(b + o_lmask);
    ws->lmhi = (uint32_t*)(b + o_lmhi);
    ws->lrec = (uint64_t*)(b + o_lrec);
    ws->lbase = (int64_t*)(b + o_lbase);
    ws->ck = (int32_t*)(b + o_ck);
    ws->cl = (int32_t*)(b + o_cl);
    ws->cf = (float*)(b + o_cf);
    ws->cinfo = (uint32_t*)(b + o_ci);
    ws->cand = (int64_t*)(b + o_cand);
    ws->nlist = (int64_t*)(b + o_nlist);
    ws->park = (uint32_t*)(b + o_park);
    ws->scan = (uint64_t*)(b + o_scan);
    ws->ticket = (unsigned int*)(b + o_ticket);
    ws->cap = cap;
    ws->tiles_lat = tiles_lat;
    ws->tiles_col = tiles_col;
    ws->tiles_cap = tiles_cap;
    ws->words1 = (int)words1;
  }
  return off;
}

// Offsets of the four look-back arrays inside Workspace::scan.
__host__ __device__ inline uint64_t* scan_corners(const Workspace& w) { return w.scan; }
__host__ __device__ inline uint64_t* scan_verts(const Workspace& w) { return w.scan + w.tiles_lat; }
__host__ __device__ inline uint64_t* scan_tris(const Workspace& w) { return w.scan + w.tiles_lat + w.tiles_cap; }
__host__ __device__ inline uint64_t* scan_cands(const Workspace& w) {
  return w.scan + w.tiles_lat + 2 * w.tiles_cap;
}
__host__ __device__ inline size_t scan_words(const Workspace& w) {
  return (size_t)(w.tiles_lat + 2 * w.tiles_cap + w.tiles_col) + kPackCounts;
}
// Exact 64-bit totals behind the two packed scans (two 31-bit fields in one
// word, which a total of 2^31 would carry over): corners, candidates,
// triangles, cells.  Zero between passes.
__host__ __device__ inline unsigned long long* pack_counts(const Workspace& w) {
  return (unsigned long long*)(w.scan + w.tiles_lat + 2 * w.tiles_cap + w.tiles_col);
}

// List index of corner (L, k), or -1 when (L, k) is not a corner.  The mask,
// record and tile base loads are unconditional and issued together (one
// memory round trip); a record that was not written this run is read but
// never used.  k <= n, so the word index stays inside the W1 rows;
// L < (n+1)^2.  Word 64 exists only for n >= 2016, where its presence bit
// lives in lmhi.
__device__ __forceinline__ int64_t corner_index(const Workspace& ws, size_t nl, size_t L, int k) {
  const int w = k >> 5;
  const uint64_t lm = ws.lmask[L];
  const uint64_t rec = ws.lrec[(size_t)w * nl + L];
  const int64_t tb = ws.lbase[L / kLatTile];
  bool present;
  if (ws.words1 > 64) present = w < 64 ? ((lm >> (w & 63)) & 1) : (ws.lmhi[L] & 1);
  else present = (lm >> w) & 1;
  const uint32_t word = (uint32_t)rec;
  const uint32_t bit = 1u << (k & 31);
  const int64_t idx = tb + (int64_t)(int32_t)(rec >> 32) + __popc(word & (bit - 1u));
  return present && (word & bit) ? idx : -1;
}

// List index of a lattice point known to be a corner (a corner of a
// candidate cell): a record load and a tile base load, no presence test.  *ok
// is cleared when the record's word lacks the point (inconsistent workspace
// contents).
__device__ __forceinline__ int64_t corner_index_known(const Workspace& ws, size_t nl, size_t L, int k, bool* ok) {
  const uint64_t rec = ws.lrec[(size_t)(k >> 5) * nl + L];
  const int64_t tb = ws.lbase[L / kLatTile];
  const uint32_t word = (uint32_t)rec;
  const uint32_t bit = 1u << (k & 31);
  *ok = *ok && (word & bit);
  return tb + (int64_t)(int32_t)(rec >> 32) + __popc(word & (bit - 1u));
}

// The 32-bit corner word: sign, owned crossing edges, first vertex index.
constexpr int64_t kMaxVerts = (int64_t)1 << 28;  // vertex indices fit in 28 bits (vertex capacities stay below)
__host__ __device__ inline uint32_t cinfo_pack(int64_t vbase, unsigned mask, bool neg) {
  return ((uint32_t)vbase << 4) | (mask << 1) | (neg ? 1u : 0u);
}
__host__ __device__ inline int64_t cinfo_vbase(uint32_t c) { return (int64_t)(c >> 4); }
__host__ __device__ inline unsigned cinfo_mask(uint32_t c) { return (c >> 1) & 7u; }
__host__ __device__ inline bool cinfo_neg(uint32_t c) { return c & 1u; }

enum { kTicketCorners = 0, kTicketVerts = 1, kTicketTris = 2, kTicketCands = 3, kTicketRays = 4, kTicketPark = 5 };

}  // namespace gh
