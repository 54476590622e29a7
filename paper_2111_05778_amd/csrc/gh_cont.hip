// Continuation: the paper's surface-following comparator (Section 2,
// "cont").  From seed cells the search moves to the face neighbours of each
// cell it holds whose shared face has a sign change among its four corners,
// level by level, until no new cell appears.  Every cell reached is a
// sign-change cell; the set reached does not depend on the order.
//
// State in the caller's continuation workspace: a bitmap of reached cells
// (N^3 bits), a bitmap of evaluated lattice points ((N+1)^3 bits, so that each
// distinct corner counts as one evaluation) and two frontier lists.  The
// host drives the levels: one kernel per level, enqueued in batches, each
// reading its frontier's length on the device; after a batch the length
// comes back to the host, which ends the loop when it is zero.  The
// reached cells end as the candidate words of the hop workspace, so gh_mc
// follows as after gh_hop.
#include <hip/hip_runtime.h>

#include <float.h>

#include <algorithm>

#include "gh_device.h"
#include "gh_launch.h"
#include "gh_layout.h"

namespace gh {

namespace {

// Claims bit b of a bitmap; true for the one thread that set it.
__device__ __forceinline__ bool claim(uint32_t* __restrict__ bits, int64_t b) {
  const uint32_t m = 1u << (b & 31);
  return (atomicOr(&bits[b >> 5], m) & m) == 0;
}

__global__ __launch_bounds__(kBlock) void k_cont_seed(const int64_t* __restrict__ seeds, int64_t n_seeds, int n,
                                                      uint32_t* __restrict__ reached, int64_t* __restrict__ front,
                                                      unsigned long long* __restrict__ count) {
  const int64_t ncell = (int64_t)n * n * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_seeds; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t id = seeds[t];
    if (id < 0 || id >= ncell) continue;  // not a cell of the grid
    if (claim(reached, id)) front[atomicAdd(count, 1ull)] = id;  // at most n_seeds <= capacity entries
  }
}

// One level.  Eight lanes take each frontier cell: lane c evaluates corner
// c = dx + 2 dy + 4 dz (counted when it is the first to claim that lattice
// point), the group's signs come from one ballot, and lanes 0..5 take the
// faces (axis c / 2, upper side when c is odd): a face whose four corners do
// not share one sign leads to the neighbour behind it, which joins the next
// frontier if no one has reached it yet.
template <class Eval>
__global__ __launch_bounds__(kBlock) void k_cont_level(Eval ev, Grid g, const int64_t* __restrict__ front,
                                                       const unsigned long long* __restrict__ nfront_d,
                                                       int64_t* __restrict__ next,
                                                       unsigned long long* __restrict__ nnext, int64_t cap,
                                                       uint32_t* __restrict__ reached, uint32_t* __restrict__ known,
                                                       unsigned long long* __restrict__ levels,
                                                       unsigned long long* __restrict__ clear,
                                                       gh_counters* __restrict__ ctr) {
  const int n = g.n;
  const int64_t n1 = n + 1;
  // the frontier's length, as the previous level left it (held to the list's capacity)
  const int64_t nfront = (int64_t)*nfront_d < cap ? (int64_t)*nfront_d : cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (nfront > 0) atomicAdd(levels, 1ull);
    *clear = 0;  // the counter the next level fills (read by the previous one, which has finished)
  }
  const int lane = lane_id(), c = lane & 7;
  uint64_t evals = 0;
  bool bad = false, full = false;
  const int64_t groups = (int64_t)gridDim.x * (blockDim.x / 8);
  // uniform over the eight lanes of a group; waves run the loop the same
  // number of times except for the last round
  for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 8; t < nfront; t += groups) {
    const int64_t id = front[t];
    const int i = (int)(id / ((int64_t)n * n)), j = (int)((id / n) % n), k = (int)(id % n);
    const int a = i + (c & 1), b = j + ((c >> 1) & 1), z = k + ((c >> 2) & 1);
    const float f = ev(lattice(g, a), lattice(g, b), lattice(g, z));
    bad = bad || !(fabsf(f) <= FLT_MAX);
    if (claim(known, ((int64_t)a * n1 + b) * n1 + z)) ++evals;
    const unsigned neg = (unsigned)(__ballot(f < 0.f) >> (lane & ~7)) & 0xFFu;
    if (c < 6) {
      const int d = c >> 1, up = c & 1;
      constexpr unsigned kLow[3] = {0x55u, 0x33u, 0x0Fu};  // corners with bit 0, 1, 2 clear
      const unsigned face = up ? (~kLow[d] & 0xFFu) : kLow[d];
      const unsigned sgn = neg & face;
      const int ni = i + (d == 0 ? 2 * up - 1 : 0), nj = j + (d == 1 ? 2 * up - 1 : 0),
                nk = k + (d == 2 ? 2 * up - 1 : 0);
      if (sgn != 0 && sgn != face && ni >= 0 && ni < n && nj >= 0 && nj < n && nk >= 0 && nk < n) {
        const int64_t nb = ((int64_t)ni * n + nj) * n + nk;
        if (claim(reached, nb)) {
          const unsigned long long pos = atomicAdd(nnext, 1ull);
          if ((int64_t)pos < cap) next[pos] = nb;
          else full = true;
        }
      }
    }
  }
  if (bad) atomicOr(&ctr->flags, GH_FLAG_NONFINITE);
  if (full) atomicOr(&ctr->flags, GH_FLAG_CAPACITY);
  block_add_u64(evals, (unsigned long long*)&ctr->n_hop_evals);
}

// The reached cells as the hop's candidate words: word w of column col holds
// cells k = 32 w .. 32 w + 31, i.e. bits col n + 32 w .. of the cell bitmap.
__global__ __launch_bounds__(kBlock) void k_cont_columns(int n, const uint32_t* __restrict__ reached,
                                                         uint64_t* __restrict__ colmask,
                                                         uint32_t* __restrict__ colbits,
                                                         gh_counters* __restrict__ ctr) {
  const int64_t ncol = (int64_t)n * n;
  const int W = (n + 31) / 32;
  uint64_t cands = 0;
  for (int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; col < ncol; col += (int64_t)gridDim.x * blockDim.x) {
    uint64_t mask = 0;
    for (int w = 0; w < W; ++w) {
      const int64_t b0 = col * n + 32 * w;       // first bit of the word
      const int len = std::min(32, n - 32 * w);  // cells of this column in the word
      const int64_t q = b0 >> 5;
      const int sh = (int)(b0 & 31);
      uint64_t two = reached[q];
      if (sh + len > 32) two |= (uint64_t)reached[q + 1] << 32;  // in bounds: the word holds a cell of this column
      uint32_t word = (uint32_t)(two >> sh);
      if (len < 32) word &= (1u << len) - 1u;
      if (word) {
        colbits[(size_t)w * ncol + col] = word;
        mask |= 1ull << w;
        cands += __popc(word);
      }
    }
    colmask[col] = mask;
  }
  block_add_u64(cands, (unsigned long long*)&ctr->n_cand);
}

}  // namespace

size_t cont_layout(int n, int64_t cap, ContWorkspace* cw, void* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const int64_t cells = (int64_t)n * n * n, pts = (int64_t)(n + 1) * (n + 1) * (n + 1);
  const size_t o_reached = take((size_t)(cells / 32 + 1) * 4), o_known = take((size_t)(pts / 32 + 1) * 4),
               o_a = take((size_t)cap * 8), o_b = take((size_t)cap * 8), o_count = take(4 * 8);
  if (cw && base) {
    char* b = (char*)base;
    cw->reached = (uint32_t*)(b + o_reached);
    cw->known = (uint32_t*)(b + o_known);
    cw->front[0] = (int64_t*)(b + o_a);
    cw->front[1] = (int64_t*)(b + o_b);
    cw->count = (unsigned long long*)(b + o_count);
    cw->reached_bytes = (size_t)(cells / 32 + 1) * 4;
    cw->known_bytes = (size_t)(pts / 32 + 1) * 4;
    cw->cap = cap;
  }
  return off;
}

hipError_t run_cont(const DevSdb& d, const Grid& g, const Workspace& ws, const ContWorkspace& cw,
                    const int64_t* seeds, int64_t n_seeds, gh_counters* ctr, int64_t* levels, hipStream_t s) {
  if (d.kind != GH_SDB_PRIMS) return hipErrorInvalidValue;
  hipError_t e;
  if ((e = hipMemsetAsync(cw.reached, 0, cw.reached_bytes, s)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(cw.known, 0, cw.known_bytes, s)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(cw.count, 0, 4 * sizeof(unsigned long long), s)) != hipSuccess) return e;
  const int blocks = cu_count() * 8;
  hipLaunchKernelGGL(k_cont_seed, dim3(blocks), dim3(kBlock), 0, s, seeds, n_seeds, g.n, cw.reached, cw.front[0],
                     &cw.count[0]);
  // Levels are enqueued in batches: each level reads its frontier's length
  // on the device (a level past the end finds it zero and does nothing), so
  // the host waits once per batch instead of once per level.  Level l reads
  // counter l mod 3, fills counter (l + 1) mod 3 and clears (l + 2) mod 3 for
  // the level after it.  Every level with a frontier holds cells no earlier
  // level held, so N^3 levels bound the loop.
  constexpr int kBatch = 16;
  const int64_t max_levels = (int64_t)g.n * g.n * g.n + kBatch;
  const PrimsEval ev{d.prims, d.groups};
  const int lgrid = cu_count();
  for (int64_t level = 0; level < max_levels; level += kBatch) {
    for (int b = 0; b < kBatch; ++b) {
      const int64_t l = level + b;
      const int c0 = (int)(l % 3), c1 = (int)((l + 1) % 3), c2 = (int)((l + 2) % 3);
      hipLaunchKernelGGL(k_cont_level<PrimsEval>, dim3(lgrid), dim3(kBlock), 0, s, ev, g, cw.front[l & 1],
                         &cw.count[c0], cw.front[(l + 1) & 1], &cw.count[c1], cw.cap, cw.reached, cw.known,
                         &cw.count[3], &cw.count[c2], ctr);
    }
    unsigned long long nfront = 0;
    const int last = (int)((level + kBatch) % 3);  // the counter the next level would read
    if ((e = hipMemcpyAsync(&nfront, &cw.count[last], sizeof(nfront), hipMemcpyDeviceToHost, s)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (nfront == 0) break;
  }
  if (levels) {
    unsigned long long nl = 0;
    if ((e = hipMemcpyAsync(&nl, &cw.count[3], sizeof(nl), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    *levels = (int64_t)nl;
  }
  const int64_t ncol = (int64_t)g.n * g.n;
  hipLaunchKernelGGL(k_cont_columns, dim3((int)std::min<int64_t>((ncol + kBlock - 1) / kBlock, (int64_t)blocks)),
                     dim3(kBlock), 0, s, g.n, cw.reached, ws.colmask, ws.colbits, ctr);
  return hipGetLastError();
}

}  // namespace gh
