// Many bounds on uneven grids in two persistent hop launches.
//
// The plan holds a table of shapes (bound, grid, workspace, counters) and two
// lists of work items: block tiles of ray columns of the analytic bounds, and
// ranges of rays of the network bounds (gh_tuning.batch_rays_per_item).  Each
// list is ordered by estimated cost, longest first, and its persistent kernel
// takes items from its own counter, so uneven grids and widths keep the
// device busy until the end.  The analytic items run at the occupancy of the
// single-shape hop, the network items at one wave per SIMD (their activations
// fill the register file).  After the hops every shape gets its own
// marching-cubes pass; the whole sequence can be captured once into a
// hipGraph and replayed.  (The marching-cubes passes of different shapes stay
// in order on one stream: their look-back scans need every block of a kernel
// resident at once, which kernels running side by side would not ensure.)

#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "gh.h"
#include "gh_device.h"
#include "gh_hop.h"
#include "gh_launch.h"
#include "gh_layout.h"
#include "gh_mlp.h"

namespace gh {

struct BatchShape {
  DevSdb sdb;
  Grid grid;
  Workspace ws;
  gh_counters* ctr;
};

struct WorkItem {
  int32_t shape;
  int32_t pad;
  int64_t a, b;  // analytic: block tile a; network: rays [a, b) in column order
};

// Rays [first, end) handed out by a block-local counter.
struct RangeRays {
  unsigned int* counter;
  int64_t first, end;
  __device__ unsigned int take(unsigned int k) const {
    const unsigned int v = *counter;
    *counter = v + k;
    return v;
  }
};

// Zeroes every shape's counters, look-back words and tickets, and the two item counters.
__global__ void k_batch_clear(const BatchShape* __restrict__ shapes, int n_shapes, unsigned int* __restrict__ head) {
  if (blockIdx.x == 0 && threadIdx.x < 2) head[threadIdx.x] = 0;
  for (int s = blockIdx.x; s < n_shapes; s += gridDim.x) {
    const BatchShape& sh = shapes[s];
    const size_t nw = scan_words(sh.ws);
    for (size_t i = threadIdx.x; i < nw; i += blockDim.x) sh.ws.scan[i] = 0;
    if (threadIdx.x < 8) sh.ws.ticket[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
      gh_counters* c = sh.ctr;
      c->n_hop_evals = c->n_cand = c->n_corner = c->n_cells = c->n_vert = c->n_tri = c->n_reeval = 0;
      c->flags = 0;
      c->reserved = 0;
    }
  }
}

// Analytic items: a block tile of ray columns of one shape each.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_hop_batched_prims(
    const BatchShape* __restrict__ shapes, const WorkItem* __restrict__ items, int n_items,
    unsigned int* __restrict__ head) {
  __shared__ float4 s_rec[kMaxPrims * GH_PRIM_FLOATS / 4];
  __shared__ int s_item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = (int)atomicAdd(head, 1u);
    __syncthreads();
    const int it = s_item;
    if (it >= n_items) break;  // uniform: every block leaves once the list is exhausted
    const WorkItem wi = items[it];
    const BatchShape& sh = shapes[wi.shape];
    stage_prims(s_rec, sh.sdb.prims, sh.sdb.groups.start[kPrimTypes]);
    hop_prims_tile<4>(reinterpret_cast<const float*>(s_rec), sh.sdb.groups, sh.grid, sh.ws.colmask, sh.ws.colbits,
                      sh.ctr, (int)wi.a);
  }
}

// Network items: a range of rays of one shape each, through the ray pool,
// with the evaluator's LDS in sm.
template <int P, class Sm>
__device__ __forceinline__ void hop_batched_net(Sm& sm, const BatchShape* __restrict__ shapes,
                                                const WorkItem* __restrict__ items, int n_items,
                                                unsigned int* __restrict__ head) {
  __shared__ int s_cnt[kBlock / 64];
  __shared__ unsigned int s_base, s_next;
  __shared__ int s_item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = (int)atomicAdd(head, 1u);
    __syncthreads();
    const int it = s_item;
    if (it >= n_items) break;  // uniform: every block leaves once the list is exhausted
    const WorkItem wi = items[it];
    const BatchShape& sh = shapes[wi.shape];
    {
      if (threadIdx.x == 0) s_next = 0;
      __syncthreads();
      const RangeRays src{&s_next, wi.a, wi.b};
      switch (sh.sdb.mlp.W) {
        case 64:
          hop_mlp_pool<P, 64>(sh.sdb.mlp, sh.grid, sh.ws.colmask, sh.ws.colbits, sh.ctr, sm, s_cnt, &s_base, src);
          break;
        case 128:
          hop_mlp_pool<P, 128>(sh.sdb.mlp, sh.grid, sh.ws.colmask, sh.ws.colbits, sh.ctr, sm, s_cnt, &s_base, src);
          break;
        default:
          hop_mlp_pool<P, 256>(sh.sdb.mlp, sh.grid, sh.ws.colmask, sh.ws.colbits, sh.ctr, sm, s_cnt, &s_base, src);
          break;
      }
    }
  }
}

template <int P>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_hop_batched(
    const BatchShape* __restrict__ shapes, const WorkItem* __restrict__ items, int n_items,
    unsigned int* __restrict__ head) {
  __shared__ MlpSmem sm;
  hop_batched_net<P>(sm, shapes, items, n_items, head);
}

// Network items when every network shape takes the shrunk plain bf16 hop:
// the lean layout, two blocks per CU (as k_hop_mlp_lean).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_hop_batched_lean(
    const BatchShape* __restrict__ shapes, const WorkItem* __restrict__ items, int n_items,
    unsigned int* __restrict__ head) {
  __shared__ MlpSmemBf16 sm;
  hop_batched_net<kPrecBf16>(sm, shapes, items, n_items, head);
}

}  // namespace gh

// ==================================================================== host
struct gh_batch {
  std::vector<gh_batch_item> items;    // caller's per-shape buffers
  std::vector<gh::DevSdb> sdb;
  std::vector<gh::Grid> grids;
  std::vector<gh::Workspace> ws;
  gh::BatchShape* d_shapes = nullptr;  // in the caller's device buffer
  gh::WorkItem* d_items = nullptr;
  unsigned int* d_head = nullptr;      // [0] network item counter, [1] analytic item counter
  int n_items = 0;
  int n_prim_items = 0;                // the analytic items come first in d_items
  int precision = gh::kPrecF32;
  bool lean = false;                   // network items on the lean layout (every one shrunk plain bf16)
  hipGraphExec_t exec = nullptr;
};

namespace {

size_t batch_layout(int n_shapes, int64_t n_items, void* base, gh_batch* b) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = gh::align_up(off + bytes, 256);
    return o;
  };
  const size_t o_sh = take((size_t)n_shapes * sizeof(gh::BatchShape));
  const size_t o_it = take((size_t)n_items * sizeof(gh::WorkItem));
  const size_t o_hd = take(64);
  if (base && b) {
    char* p = (char*)base;
    b->d_shapes = (gh::BatchShape*)(p + o_sh);
    b->d_items = (gh::WorkItem*)(p + o_it);
    b->d_head = (unsigned int*)(p + o_hd);
  }
  return off;
}

// Work items of one shape with their estimated cost (bound evaluations x
// cost per evaluation; a ray takes about 2 log2 N + 4 steps).
void shape_items(int s, const gh::DevSdb& d, const gh::Grid& g, std::vector<std::pair<double, gh::WorkItem>>& out) {
  const double steps = 2.0 * log2((double)g.n) + 4.0;
  if (d.kind == GH_SDB_PRIMS) {
    using S = gh::HopShape<4>;
    const int nbh = (g.n + S::kBlockH - 1) / S::kBlockH, nbw = (g.n + S::kBlockW - 1) / S::kBlockW;
    const double cost = (double)S::kBlockH * S::kBlockW * steps * d.n_prim * 30.0;
    for (int t = 0; t < nbh * nbw; ++t) out.push_back({cost, gh::WorkItem{s, 0, t, 0}});
  } else {
    const int64_t rays = (int64_t)g.n * g.n;
    const int64_t per_item = gh::current_tuning().batch_rays_per_item;
    const double per_ray = steps * 2.0 * ((double)d.mlp.k1 * d.mlp.W + (double)(d.mlp.depth - 1) * d.mlp.W * d.mlp.W);
    for (int64_t a = 0; a < rays; a += per_item) {
      const int64_t e = std::min(rays, a + per_item);
      out.push_back({per_ray * (double)(e - a), gh::WorkItem{s, 0, a, e}});
    }
  }
}

hipError_t enqueue_batch(gh_batch* b, hipStream_t s) {
  const int ns = (int)b->items.size();
  hipLaunchKernelGGL(gh::k_batch_clear, dim3(ns < 1024 ? ns : 1024), dim3(gh::kBlock), 0, s, b->d_shapes, ns,
                     b->d_head);
  const int cus = gh::cu_count();
  auto hop = [&](auto kernel, const gh::WorkItem* items, int n, unsigned int* head) {
    if (n == 0) return;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, gh::kBlock, 0) != hipSuccess || per_cu < 1)
      per_cu = 1;
    const int blocks = std::max(1, std::min(n, cus * per_cu));
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(gh::kBlock), 0, s, b->d_shapes, items, n, head);
  };
  const int n_net = b->n_items - b->n_prim_items;
  hop(gh::k_hop_batched_prims, b->d_items, b->n_prim_items, b->d_head + 1);
  const gh::WorkItem* net_items = b->d_items + b->n_prim_items;
  switch (b->precision) {
    case gh::kPrecBf16:
      if (b->lean) hop(gh::k_hop_batched_lean, net_items, n_net, b->d_head);
      else hop(gh::k_hop_batched<gh::kPrecBf16>, net_items, n_net, b->d_head);
      break;
    case gh::kPrecBf16x3: hop(gh::k_hop_batched<gh::kPrecBf16x3>, net_items, n_net, b->d_head); break;
    default: hop(gh::k_hop_batched<gh::kPrecF32>, net_items, n_net, b->d_head); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int i = 0; i < ns; ++i) {
    const gh_batch_item& it = b->items[i];
    e = gh::launch_mc(b->sdb[i], b->grids[i], b->ws[i], it.verts, it.vert_edge, it.vert_t, it.vert_cap, it.tris,
                      it.tri_cap, it.cells, it.cases, (it.cells || it.cases) ? it.cell_cap : 0, it.ctr, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

// The C entry points validate through the single-bound ABI's helpers.
extern "C" gh_status gh_batch_validate_item(const gh_batch_item* it, int index, gh::DevSdb* d, gh::Grid* g,
                                            gh::Workspace* w);

extern "C" {

gh_status gh_batch_buffer_size(int n_shapes, const gh_batch_item* items_h, size_t* bytes_h) {
  if (n_shapes < 1 || !items_h || !bytes_h) return GH_EINVAL;
  int64_t n_items = 0;
  for (int i = 0; i < n_shapes; ++i) {
    gh::DevSdb d;
    gh::Grid g;
    gh::Workspace w;
    const gh_status st = gh_batch_validate_item(&items_h[i], i, &d, &g, &w);
    if (st != GH_OK) return st;
    std::vector<std::pair<double, gh::WorkItem>> v;
    shape_items(i, d, g, v);
    n_items += (int64_t)v.size();
  }
  *bytes_h = batch_layout(n_shapes, n_items, nullptr, nullptr);
  return GH_OK;
}

gh_status gh_batch_create(int n_shapes, const gh_batch_item* items_h, void* dev_buf, size_t dev_bytes, void* stream,
                          gh_batch** out_h) {
  if (n_shapes < 1 || !items_h || !dev_buf || !out_h) return GH_EINVAL;
  if (((uintptr_t)dev_buf) & 255) return GH_EINVAL;
  gh_batch* b = new gh_batch();
  std::vector<std::pair<double, gh::WorkItem>> work;
  int mlp_prec = -1;
  for (int i = 0; i < n_shapes; ++i) {
    gh::DevSdb d;
    gh::Grid g;
    gh::Workspace w;
    const gh_status st = gh_batch_validate_item(&items_h[i], i, &d, &g, &w);
    if (st != GH_OK) {
      delete b;
      return st;
    }
    if (d.kind == GH_SDB_MLP) {
      if (mlp_prec >= 0 && mlp_prec != d.mlp.precision) {
        delete b;
        return GH_EUNSUPPORTED;  // one network precision per batch
      }
      mlp_prec = d.mlp.precision;
    }
    b->items.push_back(items_h[i]);
    b->sdb.push_back(d);
    b->grids.push_back(g);
    b->ws.push_back(w);
    shape_items(i, d, g, work);
  }
  b->precision = mlp_prec < 0 ? gh::kPrecF32 : mlp_prec;
  b->lean = b->precision == gh::kPrecBf16 && gh::current_tuning().mlp_lean == 1;
  for (int i = 0; i < n_shapes; ++i)
    if (b->sdb[i].kind == GH_SDB_MLP && !b->sdb[i].mlp.hop_shrink) b->lean = false;
  // analytic items first, then network items, each by cost, longest first
  std::stable_sort(work.begin(), work.end(), [&](const auto& x, const auto& y) {
    const bool px = b->sdb[x.second.shape].kind == GH_SDB_PRIMS, py = b->sdb[y.second.shape].kind == GH_SDB_PRIMS;
    return px != py ? px : x.first > y.first;
  });
  b->n_items = (int)work.size();
  b->n_prim_items = 0;
  for (const auto& w : work) b->n_prim_items += b->sdb[w.second.shape].kind == GH_SDB_PRIMS ? 1 : 0;
  const size_t need = batch_layout(n_shapes, b->n_items, nullptr, nullptr);
  if (dev_bytes < need) {
    delete b;
    return GH_ECAPACITY;
  }
  batch_layout(n_shapes, b->n_items, dev_buf, b);
  std::vector<gh::BatchShape> shapes(n_shapes);
  const gh::Tuning tu = gh::current_tuning();
  for (int i = 0; i < n_shapes; ++i) {
    shapes[i] = gh::BatchShape{b->sdb[i], b->grids[i], b->ws[i], items_h[i].ctr};
    shapes[i].sdb.mlp.split = tu.mlp_split;
    shapes[i].sdb.mlp.pool_tiles = tu.mlp_pool_tiles;
    shapes[i].sdb.mlp.spec_rows = tu.mlp_spec_rows;
  }
  std::vector<gh::WorkItem> wi(b->n_items);
  for (int i = 0; i < b->n_items; ++i) wi[i] = work[i].second;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(b->d_shapes, shapes.data(), shapes.size() * sizeof(gh::BatchShape), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(b->d_items, wi.data(), wi.size() * sizeof(gh::WorkItem), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    delete b;
    return GH_EHIP;
  }
  *out_h = b;
  return GH_OK;
}

gh_status gh_batch_run(gh_batch* b, void* stream) {
  if (!b) return GH_EINVAL;
  return enqueue_batch(b, (hipStream_t)stream) == hipSuccess ? GH_OK : GH_EHIP;
}

gh_status gh_batch_capture(gh_batch* b, void* stream) {
  if (!b) return GH_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return GH_EHIP;
  const hipError_t e = enqueue_batch(b, s);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(s, &graph);
  if (e != hipSuccess || e2 != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return GH_EHIP;
  }
  const hipError_t e3 = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  return e3 == hipSuccess ? GH_OK : GH_EHIP;
}

gh_status gh_batch_replay(gh_batch* b, void* stream) {
  if (!b || !b->exec) return GH_EINVAL;
  return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? GH_OK : GH_EHIP;
}

gh_status gh_batch_item_count(const gh_batch* b, int64_t* n_items_h) {
  if (!b || !n_items_h) return GH_EINVAL;
  *n_items_h = b->n_items;
  return GH_OK;
}

gh_status gh_batch_destroy(gh_batch* b) {
  if (!b) return GH_EINVAL;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  delete b;
  return GH_OK;
}

}  // extern "C"
