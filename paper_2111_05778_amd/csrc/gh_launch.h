// Host-side launchers of the kernels, and the device view of a bound.
#pragma once

#include <hip/hip_runtime.h>

#include "gh.h"
#include "gh_device.h"
#include "gh_layout.h"
#include "gh_mlp.h"

namespace gh {

// Launch shapes in effect (gh_set_tuning); every field resolved to a value.
struct Tuning {
  int hop_lanes_per_ray, scan_blocks_per_cu, batch_rays_per_item, mlp_split, mc_items_per_thread;
  int hop_step_budget;  // 0: no hand-over to the long-ray pass
  int mlp_pool_tiles, mlp_spec_rows;
  int mlp_lean;  // plain bf16 shrunk hop and corner values: 1 lean layout, 2 full layout
};
Tuning current_tuning();

// Compute units of the current device (cached per device).
int cu_count();

// Grid of a grid-strided kernel over `work` items, one thread each.
inline int persistent_blocks(int64_t work) {
  const int64_t want = (work + kBlock - 1) / kBlock;
  return (int)(want < 1 ? 1 : (want > 2048 ? 2048 : want));
}

// Look-back kernels run block-strided over their tiles with a grid no larger
// than the number of blocks the device holds at once: every tile a block
// waits on then belongs to a resident block that only waits on earlier
// tiles, so the scan always makes progress (no ticket counter needed).
// One block per tile whenever every tile fits at once; otherwise the tuned
// number of resident blocks per CU walks the tiles.
template <class K>
inline int resident_grid(K kernel, int64_t tiles) {
  const int cus = cu_count();
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  if (tiles <= (int64_t)cus * per_cu) return (int)(tiles < 1 ? 1 : tiles);
  const int want = current_tuning().scan_blocks_per_cu;
  const int64_t cap = (int64_t)cus * (per_cu < want ? per_cu : want);
  const int64_t gsz = tiles < cap ? tiles : cap;
  return (int)(gsz < 1 ? 1 : gsz);
}


// What the kernels need to evaluate a bound; lives inside gh_sdb_desc.
struct DevSdb {
  uint32_t magic;
  int32_t kind;
  int32_t n_prim;
  int32_t flags;       // kSdbRadiiNormal
  const float* prims;  // device, n_prim * GH_PRIM_FLOATS, sorted by type
  PrimGroups groups;   // type t occupies records [start[t], start[t+1])
  MlpDesc mlp;         // GH_SDB_MLP: packed network in the blob
};
constexpr uint32_t kDescMagic = 0x67687364u;  // "ghsd"
// Every torus ring radius and cylinder radius of the union has magnitude
// >= 2^-23 (one of the conditions for the hop square root, sqrt_hop).
constexpr int32_t kSdbRadiiNormal = 1;

enum ClearMode { kClearAll = 0, kClearCands = 2 };

// Continuation workspace (gh_cont): reached-cell and evaluated-point
// bitmaps, two frontier lists of cap cell ids, three rotating frontier
// counters and a level counter.
struct ContWorkspace {
  uint32_t* reached;
  uint32_t* known;
  int64_t* front[2];
  unsigned long long* count;
  size_t reached_bytes, known_bytes;
  int64_t cap;
};
// Layout of the continuation workspace for grid size n and frontier
// capacity cap; fills cw when base is given.  Returns the bytes needed.
size_t cont_layout(int n, int64_t cap, ContWorkspace* cw, void* base);
// Continuation from the seed cells (device list) to the candidate words of
// ws; host-driven levels, returns after the last one.  levels: out, may be null.
hipError_t run_cont(const DevSdb& d, const Grid& g, const Workspace& ws, const ContWorkspace& cw,
                    const int64_t* seeds, int64_t n_seeds, gh_counters* ctr, int64_t* levels, hipStream_t s);

hipError_t launch_clear(const Workspace& ws, gh_counters* ctr, ClearMode mode, hipStream_t s);
// lanes_per_ray: 1, 2, 3, 4 or 8 lanes trace one ray together (0 = chosen from the type groups).
hipError_t launch_hop(const DevSdb& d, const Grid& g, const Workspace& ws, gh_counters* ctr, int lanes_per_ray,
                      hipStream_t s);
// Algorithm 1 taken literally (analytic bounds): candidates into the same
// workspace words as launch_hop.
hipError_t launch_hop_traced(const DevSdb& d, const Grid& g, const Workspace& ws, gh_counters* ctr,
                             int lanes_per_ray, hipStream_t s);
hipError_t launch_dense(const DevSdb& d, const Grid& g, const Workspace& ws, uint32_t* signs, gh_counters* ctr,
                        hipStream_t s);
hipError_t launch_candidates(const Grid& g, const Workspace& ws, int64_t* out, int64_t cap, gh_counters* ctr,
                             hipStream_t s);
hipError_t launch_mc(const DevSdb& d, const Grid& g, const Workspace& ws, float* verts, int64_t* vert_edge,
                     float* vert_t, int64_t vert_cap, int32_t* tris, int64_t tri_cap, int64_t* cells,
                     uint8_t* cases, int64_t cell_cap, gh_counters* ctr, hipStream_t s);
hipError_t launch_eval_points(const DevSdb& d, const float* xyz, float* f, int64_t m, hipStream_t s);
// Network values at m points in FP32 (f32) and in bf16 precision prec (flp),
// then factor * max |flp - f32| into *out (NaN if any value is not finite).
hipError_t launch_bf16_margin(const DevSdb& d, int prec, const float* xyz, int64_t m, float factor, float* f32,
                              float* flp, float* margin, float* offset, hipStream_t s);
// Workspace of the adjoint (gh_backward).
constexpr int kVjpBlocks = 256;  // blocks of the network VJP, each with its own partial gradient
struct BackwardWs {
  int32_t* cidx;     // [cap] corners with a non-zero cotangent
  float* cval;       // [cap] their cotangents
  int64_t* ccount;   // number of them
  uint64_t* flags;   // look-back words of the compaction
  size_t nflags;
  float* zs;         // [kVjpBlocks][depth][64][W] pre-activations of the block's tile
  float* part;       // [kVjpBlocks][nparams] partial gradients
  int64_t nparams;
};
int64_t mlp_param_count(const MlpDesc& m);
size_t backward_layout(const MlpDesc& m, int64_t cap, void* base, BackwardWs* bw);
hipError_t launch_backward(const DevSdb& d, const Grid& g, const Workspace& ws, const BackwardWs& bw,
                           const float* dldv, float* dldtheta, gh_counters* ctr, hipStream_t s);

// Network kernels: what = 0 points, 1 corner list, 2 enumeration signs, 3 hop.
hipError_t launch_mlp(int what, const DevSdb& d, const Grid& g, const Workspace* ws, uint32_t* signs,
                      const float* xyz, float* f, int64_t count, gh_counters* ctr, hipStream_t s);

}  // namespace gh
