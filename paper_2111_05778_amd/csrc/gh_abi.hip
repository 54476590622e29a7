// C ABI of the grid hopping polygonizer: argument checks, workspace
// carving and kernel launches.  No device memory is allocated here.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "gh.h"
#include "gh_launch.h"
#include "gh_layout.h"

static_assert(GH_PRIM_TYPES == gh::kPrimTypes, "record type count of the header and the evaluators");

namespace {

thread_local std::string g_last_error;
std::atomic<int> g_hop_lanes{0}, g_scan_blocks{0}, g_batch_rays{0}, g_mlp_split{0}, g_mc_items{0}, g_hop_budget{0},
    g_mlp_pool{0}, g_mlp_spec{0}, g_mlp_lean{0};

gh_status fail(gh_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

gh_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return GH_OK;
  return fail(GH_EHIP, "%s: %s", what, hipGetErrorString(e));
}

static_assert(sizeof(gh::DevSdb) <= sizeof(gh_sdb_desc), "descriptor does not fit");

gh_status read_desc(const gh_sdb_desc* desc_h, gh::DevSdb* d) {
  if (!desc_h) return fail(GH_EINVAL, "desc is NULL");
  memcpy(d, desc_h, sizeof(*d));
  if (d->magic != gh::kDescMagic) return fail(GH_EINVAL, "desc was not filled by sdb_describe");
  return GH_OK;
}

gh_status read_grid(const gh_grid* grid_h, gh::Grid* g) {
  if (!grid_h) return fail(GH_EINVAL, "grid is NULL");
  if (grid_h->n < 1) return fail(GH_EINVAL, "grid n = %d must be >= 1", grid_h->n);
  if (grid_h->n > gh::kMaxN) return fail(GH_EUNSUPPORTED, "grid n = %d exceeds %d", grid_h->n, gh::kMaxN);
  if (!(grid_h->h > 0.f) || !isfinite(grid_h->h)) return fail(GH_EINVAL, "grid h must be finite and > 0");
  if (!isfinite(grid_h->lo) || !isfinite(grid_h->lo + grid_h->n * grid_h->h))
    return fail(GH_EINVAL, "grid extent is not finite");
  g->n = grid_h->n;
  g->lo = grid_h->lo;
  g->h = grid_h->h;
  g->inv_h = (float)(1.0 / (double)grid_h->h);
  // Candidate threshold: half a cell's diagonal, where a cell the surface
  // crosses keeps its centroid value, plus h/32 for the float32 error of the
  // values (which must stay below h/64); on grids whose cells are small
  // against the coordinates, h (every cell with a zero step).
  const double hd = grid_h->h, lod = grid_h->lo;
  const double scale = fmax(1.0, fmax(fabs(lod), fabs(lod + grid_h->n * hd)));
  g->cand_thr = (float)((hd >= ldexp(1.0, -12) * scale ? sqrt(3.0) / 2.0 + 1.0 / 32.0 : 1.0) * hd);
  return GH_OK;
}

int64_t default_cap(int n) { return 16 * (int64_t)(n + 1) * (n + 1); }

gh_status carve(const gh::Grid& g, void* ws, size_t ws_bytes, int64_t cap, gh::Workspace* w) {
  if (!ws) return fail(GH_EINVAL, "workspace is NULL");
  if (cap <= 0) cap = default_cap(g.n);
  if (cap >= (int64_t)1 << 31) return fail(GH_EUNSUPPORTED, "corner_cap %lld too large", (long long)cap);
  const size_t need = gh::workspace_layout(g.n, cap, nullptr, nullptr);
  if (ws_bytes < need)
    return fail(GH_ECAPACITY, "workspace of %zu bytes, %zu needed for n=%d corner_cap=%lld", ws_bytes, need, g.n,
                (long long)cap);
  if (((uintptr_t)ws) & 255) return fail(GH_EINVAL, "workspace must be 256-byte aligned");
  gh::workspace_layout(g.n, cap, ws, w);
  return GH_OK;
}

uint16_t to_bf16(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even; values are finite
  return (uint16_t)(u >> 16);
}

bool finite_bounded(float v, float lim) { return fabsf(v) <= lim; }

// Packs the network into the blob: bf16 and f32 B fragments of every hidden
// layer (exact 32x32 MFMA operand order, zero-padded K), biases, output
// weights and frequencies.
gh_status describe_mlp(const gh_sdb_spec* sp, void* dev_blob, size_t blob_bytes, size_t* blob_needed_h,
                       gh_sdb_desc* desc_h, void* stream) {
  const int F = sp->n_freq, W = sp->width, D = sp->depth;
  if (F < 0 || F > 16) return fail(GH_EINVAL, "n_freq = %d must be in [0, 16]", F);
  if (!(W == 64 || W == 128 || W == 256)) return fail(GH_EUNSUPPORTED, "width %d: supported 64, 128, 256", W);
  if (D < 1 || D > 8) return fail(GH_EINVAL, "depth = %d must be in [1, 8]", D);
  if (!(sp->precision == GH_PREC_FP32 || sp->precision == GH_PREC_BF16 || sp->precision == GH_PREC_BF16X3))
    return fail(GH_EINVAL, "precision %d unknown", sp->precision);
  if (!sp->weights_h || !sp->biases_h || (F > 0 && !sp->omegas_h)) return fail(GH_EINVAL, "network arrays are NULL");
  const float scal[] = {sp->a_s, sp->r0, sp->a_n, sp->b, sp->bf16_margin};
  for (float v : scal)
    if (!finite_bounded(v, 1e6f)) return fail(GH_EINVAL, "network scalar not finite or above 1e6");
  if (sp->bf16_margin < 0.f) return fail(GH_EINVAL, "bf16_margin must be >= 0");
  // The bf16 modes take a hop or a sign only when it holds for every value
  // within bf16_margin, so their decisions are uncertified without one.
  if (sp->precision != GH_PREC_FP32 && !(sp->bf16_margin > 0.f))
    return fail(GH_EINVAL, "bf16 precisions need bf16_margin > 0 (>= max |f_bf16 - f_fp32|, see gh_bf16_margin)");
  if (!(sp->activation == GH_ACT_SOFTPLUS || sp->activation == GH_ACT_RELU))
    return fail(GH_EINVAL, "activation %d unknown", sp->activation);
  if (!(sp->bf16_hop == GH_BF16_HOP_FP32 || sp->bf16_hop == GH_BF16_HOP_SHRINK))
    return fail(GH_EINVAL, "bf16_hop %d unknown", sp->bf16_hop);
  if (!(sp->bf16x3_margin >= 0.f && sp->bf16x3_margin <= 1e6f)) return fail(GH_EINVAL, "bf16x3_margin must be >= 0");
  if (sp->bf16x3_margin > 0.f && sp->precision != GH_PREC_BF16)
    return fail(GH_EINVAL, "bf16x3_margin applies to GH_PREC_BF16 only");
  if (!(fabsf(sp->bf16_offset) <= 1e6f)) return fail(GH_EINVAL, "bf16_offset must be finite");
  if (sp->bf16_offset != 0.f && sp->precision != GH_PREC_BF16)
    return fail(GH_EINVAL, "bf16_offset applies to GH_PREC_BF16 only");
  const int k1 = 3 + 6 * F;
  for (int l = 0; l <= D; ++l) {
    const int fi = l == 0 ? k1 : W, fo = l == D ? 1 : W;
    if (!sp->weights_h[l] || !sp->biases_h[l]) return fail(GH_EINVAL, "layer %d arrays are NULL", l);
    for (int q = 0; q < fi * fo; ++q)
      if (!finite_bounded(sp->weights_h[l][q], 1e6f)) return fail(GH_EINVAL, "layer %d weight not finite", l);
    for (int q = 0; q < fo; ++q)
      if (!finite_bounded(sp->biases_h[l][q], 1e6f)) return fail(GH_EINVAL, "layer %d bias not finite", l);
  }
  for (int q = 0; q < F; ++q)
    if (!finite_bounded(sp->omegas_h[q], 1e4f)) return fail(GH_EINVAL, "frequency %d not finite", q);
  const size_t nb = gh::mlpa_layer_offset(D, W);
  size_t nf = 0;
  for (int l = 0; l < D; ++l) nf += gh::mlp_layer_elems(l, k1, W);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = gh::align_up(off + bytes, 256);
    return o;
  };
  const size_t nft = (size_t)(D - 1) * W * W;
  const size_t o_wa = take(nb * 2), o_wal = take(nb * 2), o_wf = take(nf * 4), o_wft = take(nft * 4 + 4),
               o_bias = take((size_t)D * W * 4), o_wout = take((size_t)W * 4), o_om = take(16 * 4),
               o_omrev = take(16 * 4), o_bias2 = take((size_t)D * W * 4), o_wout2 = take((size_t)W * 4);
  const size_t need = off;
  if (blob_needed_h) *blob_needed_h = need;
  if (!dev_blob) return desc_h ? fail(GH_EINVAL, "dev_blob is NULL") : GH_OK;
  if (blob_bytes < need) return fail(GH_ECAPACITY, "blob of %zu bytes, %zu needed", blob_bytes, need);
  if (!desc_h) return fail(GH_EINVAL, "desc is NULL");
  std::vector<unsigned char> host(need, 0);
  uint16_t* wa = (uint16_t*)(host.data() + o_wa);
  uint16_t* wal = (uint16_t*)(host.data() + o_wal);
  float* wf = (float*)(host.data() + o_wf);
  // Frequencies in turns per unit for the register evaluator's hardware sine.
  {
    float* om = (float*)(host.data() + o_omrev);
    for (int q = 0; q < F; ++q) om[q] = (float)((double)sp->omegas_h[q] / (2.0 * M_PI));
  }
  // The register evaluator works on pre-activations in base-2 units,
  // z' = z log2 e, so that its activation needs no multiply: the first
  // layer's weights and every bias are scaled by log2 e here, the hidden
  // layers' weights are not (a = ln 2 u with u = max(z', 0) + c log2(1 +
  // 2^-|z'|) is ln 2 times the activation, which the next layer's log2 e
  // cancels; ReLU is homogeneous, so c = 0 gives the same), and the output
  // weights are scaled by ln 2.
  const double kLog2e = 1.4426950408889634074, kLn2 = 0.6931471805599453094;
  for (int l = 0; l < D; ++l) {
    const float* Wl = sp->weights_h[l];  // W x fan_in, row-major
    const int fi = l == 0 ? k1 : W;
    const int CT = W / 32;
    // bf16 A fragments: (k-step s, m-tile c), lane, element i ->
    //   W_l[32c + lane%32][input of slot 16s + 8(lane/32) + i]; for l >= 1 the
    //   slot holds the permuted feature (the previous tile's register order).
    {
      const int KS = l == 0 ? gh::kK0Steps : W / 16;
      uint16_t* dst = wa + gh::mlpa_layer_offset(l, W);
      uint16_t* dstl = wal + gh::mlpa_layer_offset(l, W);
      for (int ks = 0; ks < KS; ++ks)
        for (int c = 0; c < CT; ++c)
          for (int lane = 0; lane < 64; ++lane)
            for (int i = 0; i < 8; ++i) {
              const int q = 8 * (lane / 32) + i;
              const int k = 16 * ks + (l == 0 ? q : gh::mlpa_slot_feature(q));
              const int row = c * 32 + lane % 32;
              const float v = k < fi ? (l == 0 ? (float)(Wl[(size_t)row * fi + k] * kLog2e)
                                                : Wl[(size_t)row * fi + k])
                                     : 0.f;
              const uint16_t hi = to_bf16(v);
              uint32_t hb = (uint32_t)hi << 16;
              float hv;
              memcpy(&hv, &hb, 4);
              const size_t o = ((size_t)(ks * CT + c) * 64 + lane) * 8 + i;
              dst[o] = hi;
              dstl[o] = to_bf16(v - hv);
            }
    }
    // f32: fragment (kt, ct), lane -> W[ct*32 + lane%32][2*kt + lane/32]
    {
      const int K = l == 0 ? gh::mlp_k0(k1) : W;
      float* dst = wf + gh::mlp_layer_offset(l, k1, W);
      for (int kt = 0; kt < K / 2; ++kt)
        for (int ct = 0; ct < CT; ++ct)
          for (int lane = 0; lane < 64; ++lane) {
            const int col = ct * 32 + lane % 32, k = 2 * kt + lane / 32;
            dst[(size_t)(kt * CT + ct) * 64 + lane] = k < fi ? Wl[(size_t)col * fi + k] : 0.f;
          }
    }
    // transposed f32 (l >= 1): fragment (ks, kt), lane -> W[2*ks + lane/32][kt*32 + lane%32]
    if (l >= 1) {
      float* dst = (float*)(host.data() + o_wft) + (size_t)(l - 1) * W * W;
      for (int ks = 0; ks < W / 2; ++ks)
        for (int kt = 0; kt < CT; ++kt)
          for (int lane = 0; lane < 64; ++lane)
            dst[(size_t)(ks * CT + kt) * 64 + lane] = Wl[(size_t)(2 * ks + lane / 32) * W + kt * 32 + lane % 32];
    }
    memcpy(host.data() + o_bias + (size_t)l * W * 4, sp->biases_h[l], (size_t)W * 4);
    float* b2 = (float*)(host.data() + o_bias2) + (size_t)l * W;
    for (int q = 0; q < W; ++q) b2[q] = (float)(sp->biases_h[l][q] * kLog2e);
  }
  memcpy(host.data() + o_wout, sp->weights_h[D], (size_t)W * 4);
  {
    float* w2 = (float*)(host.data() + o_wout2);
    for (int q = 0; q < W; ++q) w2[q] = (float)(sp->weights_h[D][q] * kLn2);
  }
  if (F > 0) memcpy(host.data() + o_om, sp->omegas_h, (size_t)F * 4);
  hipStream_t s = (hipStream_t)stream;
  gh_status st = hip_status(hipMemcpyAsync(dev_blob, host.data(), need, hipMemcpyHostToDevice, s), "upload");
  if (st != GH_OK) return st;
  st = hip_status(hipStreamSynchronize(s), "upload sync");
  if (st != GH_OK) return st;
  gh::DevSdb d{};
  d.magic = gh::kDescMagic;
  d.kind = GH_SDB_MLP;
  char* b = (char*)dev_blob;
  gh::MlpDesc& m = d.mlp;
  m.wa = (const uint16_t*)(b + o_wa);
  m.wal = (const uint16_t*)(b + o_wal);
  m.omrev = (const float*)(b + o_omrev);
  m.wf = (const float*)(b + o_wf);
  m.wft = (const float*)(b + o_wft);
  m.bias = (const float*)(b + o_bias);
  m.wout = (const float*)(b + o_wout);
  m.bias2 = (const float*)(b + o_bias2);
  m.wout2 = (const float*)(b + o_wout2);
  m.omegas = (const float*)(b + o_om);
  m.F = F;
  m.W = W;
  m.depth = D;
  m.k1 = k1;
  m.precision = sp->precision == GH_PREC_BF16 ? gh::kPrecBf16
                : (sp->precision == GH_PREC_BF16X3 ? gh::kPrecBf16x3 : gh::kPrecF32);
  m.a_s = sp->a_s;
  m.r0 = sp->r0;
  m.a_n = sp->a_n;
  m.b = sp->b;
  m.b_out = sp->biases_h[D][0];
  m.eps = sp->bf16_margin;
  m.hop_shrink = sp->precision != GH_PREC_FP32 && sp->bf16_hop == GH_BF16_HOP_SHRINK ? 1 : 0;
  m.eps3 = sp->bf16x3_margin;
  m.off = sp->bf16_offset;
  m.relu = sp->activation == GH_ACT_RELU ? 1 : 0;
  m.act_one = m.relu ? 0.f : 1.f;
  m.split = 3;
  m.pool_tiles = 2;
  m.spec_rows = gh::kSpecRowsDefault;
  memset(desc_h, 0, sizeof(*desc_h));
  memcpy(desc_h, &d, sizeof(d));
  return GH_OK;
}

}  // namespace

namespace gh {
Tuning current_tuning() {
  Tuning t;
  const int r = g_hop_lanes.load(std::memory_order_relaxed), sb = g_scan_blocks.load(std::memory_order_relaxed),
            br = g_batch_rays.load(std::memory_order_relaxed), ms = g_mlp_split.load(std::memory_order_relaxed);
  t.hop_lanes_per_ray = r;  // 0: chosen per bound by the launcher
  t.scan_blocks_per_cu = sb ? sb : 4;
  t.batch_rays_per_item = br ? br : 4096;
  t.mlp_split = ms ? ms : 3;
  const int mi = g_mc_items.load(std::memory_order_relaxed);
  t.mc_items_per_thread = mi ? mi : 4;
  const int hb = g_hop_budget.load(std::memory_order_relaxed);
  t.hop_step_budget = hb;  // 0: one pass
  const int mp = g_mlp_pool.load(std::memory_order_relaxed), msr = g_mlp_spec.load(std::memory_order_relaxed);
  t.mlp_pool_tiles = mp ? mp : 2;
  t.mlp_spec_rows = msr ? msr : 32;
  const int ml = g_mlp_lean.load(std::memory_order_relaxed);
  t.mlp_lean = ml ? ml : 1;
  return t;
}
}  // namespace gh

namespace {

// ------------------------------------------------- fixed workspace (no allocation)
// gh_polygonize_noalloc's workspace: one array per device, loaded with the
// code object and held until the process ends.  In host code `scratch` names
// a host-side stand-in, never the device memory: kernels and copies get the
// address that hipGetSymbolAddress returns for the current device.
__device__ __align__(256) static unsigned char scratch[GH_NOALLOC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, set on first use

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
gh_status scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(GH_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)");
    if (!p || ((uintptr_t)p & 255)) return fail(GH_EHIP, "fixed workspace address %p unusable", p);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GH_OK;
}

// Largest corner capacity whose workspace fits in `bytes` on this grid (0 if none).
int64_t largest_cap(int n, size_t bytes) {
  int64_t lo = 0, hi = ((int64_t)1 << 31) - 1;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (gh::workspace_layout(n, mid, nullptr, nullptr) <= bytes) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace

extern "C" {

const char* gh_last_error(void) { return g_last_error.c_str(); }

gh_status gh_set_tuning(const gh_tuning* t) {
  if (!t) return fail(GH_EINVAL, "tuning is NULL");
  const int r = t->hop_lanes_per_ray, sb = t->scan_blocks_per_cu, br = t->batch_rays_per_item, ms = t->mlp_split;
  if (!(r == 0 || r == 1 || r == 2 || r == 3 || r == 4 || r == 8))
    return fail(GH_EINVAL, "hop_lanes_per_ray = %d must be 0, 1, 2, 3, 4 or 8", r);
  if (!(sb == 0 || sb == 1 || sb == 2 || sb == 4 || sb == 8))
    return fail(GH_EINVAL, "scan_blocks_per_cu = %d must be 0, 1, 2, 4 or 8", sb);
  if (!(br == 0 || (br >= 256 && br <= 65536 && (br & (br - 1)) == 0)))
    return fail(GH_EINVAL, "batch_rays_per_item = %d must be 0 or a power of two in [256, 65536]", br);
  if (!(ms >= 0 && ms <= 3)) return fail(GH_EINVAL, "mlp_split = %d must be 0, 1, 2 or 3", ms);
  const int mi = t->mc_items_per_thread;
  if (!(mi == 0 || mi == 1 || mi == 2 || mi == 4 || mi == 8))
    return fail(GH_EINVAL, "mc_items_per_thread = %d must be 0, 1, 2, 4 or 8", mi);
  const int hb = t->hop_step_budget;
  if (!(hb >= 0 && hb <= 4096)) return fail(GH_EINVAL, "hop_step_budget = %d must be 0 or 1..4096", hb);
  const int mp = t->mlp_pool_tiles, msr = t->mlp_spec_rows;
  if (!(mp >= 0 && mp <= 2)) return fail(GH_EINVAL, "mlp_pool_tiles = %d must be 0, 1 or 2", mp);
  if (!(msr == 0 || msr == 1 || msr == 8 || msr == 16 || msr == 32))
    return fail(GH_EINVAL, "mlp_spec_rows = %d must be 0, 1, 8, 16 or 32", msr);
  const int ml = t->mlp_lean;
  if (!(ml >= 0 && ml <= 2)) return fail(GH_EINVAL, "mlp_lean = %d must be 0, 1 or 2", ml);
  if (t->reserved != 0) return fail(GH_EINVAL, "the reserved tuning field must be 0");
  g_hop_lanes.store(r, std::memory_order_relaxed);
  g_scan_blocks.store(sb, std::memory_order_relaxed);
  g_batch_rays.store(br, std::memory_order_relaxed);
  g_mlp_split.store(ms, std::memory_order_relaxed);
  g_mc_items.store(mi, std::memory_order_relaxed);
  g_hop_budget.store(hb, std::memory_order_relaxed);
  g_mlp_pool.store(mp, std::memory_order_relaxed);
  g_mlp_spec.store(msr, std::memory_order_relaxed);
  g_mlp_lean.store(ml, std::memory_order_relaxed);
  return GH_OK;
}

gh_status gh_get_tuning(gh_tuning* t) {
  if (!t) return fail(GH_EINVAL, "tuning is NULL");
  memset(t, 0, sizeof(*t));
  t->hop_lanes_per_ray = g_hop_lanes.load(std::memory_order_relaxed);
  t->scan_blocks_per_cu = g_scan_blocks.load(std::memory_order_relaxed);
  t->batch_rays_per_item = g_batch_rays.load(std::memory_order_relaxed);
  t->mlp_split = g_mlp_split.load(std::memory_order_relaxed);
  t->mc_items_per_thread = g_mc_items.load(std::memory_order_relaxed);
  t->hop_step_budget = g_hop_budget.load(std::memory_order_relaxed);
  t->mlp_pool_tiles = g_mlp_pool.load(std::memory_order_relaxed);
  t->mlp_spec_rows = g_mlp_spec.load(std::memory_order_relaxed);
  t->mlp_lean = g_mlp_lean.load(std::memory_order_relaxed);
  return GH_OK;
}

gh_status sdb_describe(const gh_sdb_spec* spec_h, void* dev_blob, size_t blob_bytes, size_t* blob_needed_h,
                       gh_sdb_desc* desc_h, void* stream) {
  if (!spec_h) return fail(GH_EINVAL, "spec is NULL");
  if (spec_h->kind == GH_SDB_MLP) return describe_mlp(spec_h, dev_blob, blob_bytes, blob_needed_h, desc_h, stream);
  if (spec_h->kind != GH_SDB_PRIMS)
    return fail(GH_EUNSUPPORTED, "bound kind %d is not supported by this library", spec_h->kind);
  const int np = spec_h->n_prim;
  if (np < 1 || np > gh::kMaxPrims) return fail(GH_EINVAL, "n_prim = %d must be in [1, %d]", np, gh::kMaxPrims);
  if (!spec_h->prims_h) return fail(GH_EINVAL, "prims_h is NULL");
  for (int p = 0; p < np; ++p) {
    const float* r = spec_h->prims_h + (size_t)p * GH_PRIM_FLOATS;
    const float t = r[0];
    if (!(t >= 0.f && t <= (float)(gh::kPrimTypes - 1) && t == floorf(t)))
      return fail(GH_EINVAL, "primitive %d has unknown type %g", p, (double)t);
    // Bounded magnitudes keep every intermediate finite or +inf, never NaN:
    // |M q| <= 3e33 and sums of squares can only overflow towards +inf.
    for (int q = 1; q < GH_PRIM_FLOATS; ++q) {
      const float lim = (q >= 4 && q <= 12) ? 1e3f : 1e30f;
      if (!(fabsf(r[q]) <= lim))
        return fail(GH_EINVAL, "primitive %d parameter %d = %g is not finite or exceeds %g", p, q, (double)r[q],
                    (double)lim);
    }
    if (t == 10.f && !(r[13] > 0.f && r[14] >= 0.f && r[14] <= (float)gh::kSierpinskiMaxDepth && r[14] == floorf(r[14])))
      return fail(GH_EINVAL, "sierpinski %d: needs k > 0 and an integer depth in [0, %d] (k = %g, depth = %g)", p,
                  gh::kSierpinskiMaxDepth, (double)r[13], (double)r[14]);
    if (t == 3.f && !(r[13] >= 0.f))
      return fail(GH_EINVAL, "capsule %d: half-length %g must be >= 0", p, (double)r[13]);
    // A cone's (sine, cosine) must not be longer than a unit vector: the
    // side term is then 1-Lipschitz and the record a distance bound.
    if (t == 7.f && !((double)r[14] * r[14] + (double)r[15] * r[15] <= 1.0 + 1e-6))
      return fail(GH_EINVAL, "cone %d: (sin, cos) = (%g, %g) is longer than a unit vector", p, (double)r[14],
                  (double)r[15]);
  }
  const size_t need = (size_t)np * GH_PRIM_FLOATS * sizeof(float);
  if (blob_needed_h) *blob_needed_h = need;
  if (!dev_blob) return desc_h ? fail(GH_EINVAL, "dev_blob is NULL") : GH_OK;
  if (blob_bytes < need) return fail(GH_ECAPACITY, "blob of %zu bytes, %zu needed", blob_bytes, need);
  if (!desc_h) return fail(GH_EINVAL, "desc is NULL");
  // Group the records by type (stable): the union's minimum does not depend
  // on the order, and the kernels then loop over one type at a time.
  std::vector<float> sorted((size_t)np * GH_PRIM_FLOATS);
  gh::PrimGroups groups{};
  {
    size_t o = 0;
    for (int t = 0; t < gh::kPrimTypes; ++t) {
      groups.start[t] = (int)(o / GH_PRIM_FLOATS);
      for (int p = 0; p < np; ++p) {
        const float* r = spec_h->prims_h + (size_t)p * GH_PRIM_FLOATS;
        if ((int)r[0] != t) continue;
        std::copy(r, r + GH_PRIM_FLOATS, sorted.begin() + o);
        o += GH_PRIM_FLOATS;
      }
    }
    groups.start[gh::kPrimTypes] = np;
  }
  hipStream_t s = (hipStream_t)stream;
  gh_status st = hip_status(hipMemcpyAsync(dev_blob, sorted.data(), need, hipMemcpyHostToDevice, s), "upload");
  if (st != GH_OK) return st;
  st = hip_status(hipStreamSynchronize(s), "upload sync");
  if (st != GH_OK) return st;
  gh::DevSdb d{};
  d.magic = gh::kDescMagic;
  d.kind = GH_SDB_PRIMS;
  d.n_prim = np;
  d.flags = gh::kSdbRadiiNormal;
  for (int t : {(int)gh::kPrimTorus, (int)gh::kPrimCylinder})
    for (int p = groups.start[t]; p < groups.start[t + 1]; ++p)
      if (!(fabsf(sorted[(size_t)p * GH_PRIM_FLOATS + 13]) >= 0x1p-23f)) d.flags &= ~gh::kSdbRadiiNormal;
  // A Sierpinski record's edge and vertex roots are scaled by 2^-d k: the
  // hop root's 2^-48 floor stays below 2^-21 <= h only for k < 2^27.
  for (int p = groups.start[gh::kPrimSierpinski]; p < groups.start[gh::kPrimSierpinski + 1]; ++p)
    if (!(sorted[(size_t)p * GH_PRIM_FLOATS + 13] < 0x1p27f)) d.flags &= ~gh::kSdbRadiiNormal;
  d.prims = (const float*)dev_blob;
  d.groups = groups;
  memset(desc_h, 0, sizeof(*desc_h));
  memcpy(desc_h, &d, sizeof(d));
  return GH_OK;
}

gh_status gh_dense_signs_size(const gh_grid* grid_h, size_t* bytes_h) {
  gh::Grid g;
  gh_status st = read_grid(grid_h, &g);
  if (st != GH_OK) return st;
  if (!bytes_h) return fail(GH_EINVAL, "bytes_h is NULL");
  const size_t n1 = (size_t)g.n + 1;
  *bytes_h = ((size_t)g.n + 32) / 32 * n1 * n1 * sizeof(uint32_t);
  return GH_OK;
}

gh_status gh_workspace_size(const gh_grid* grid_h, int64_t corner_cap, size_t* bytes_h) {
  gh::Grid g;
  gh_status st = read_grid(grid_h, &g);
  if (st != GH_OK) return st;
  if (!bytes_h) return fail(GH_EINVAL, "bytes_h is NULL");
  if (corner_cap <= 0) corner_cap = default_cap(g.n);
  if (corner_cap >= (int64_t)1 << 31) return fail(GH_EUNSUPPORTED, "corner_cap too large");
  *bytes_h = gh::workspace_layout(g.n, corner_cap, nullptr, nullptr);
  return GH_OK;
}

gh_status gh_hop(const gh_sdb_desc* desc_h, const gh_grid* grid_h, void* ws, size_t ws_bytes, int64_t corner_cap,
                 gh_counters* ctr, void* stream) {
  gh::DevSdb d;
  gh::Grid g;
  gh::Workspace w;
  gh_status st;
  if ((st = read_desc(desc_h, &d)) != GH_OK) return st;
  if ((st = read_grid(grid_h, &g)) != GH_OK) return st;
  if ((st = carve(g, ws, ws_bytes, corner_cap, &w)) != GH_OK) return st;
  if (!ctr) return fail(GH_EINVAL, "counters are NULL");
  hipStream_t s = (hipStream_t)stream;
  if ((st = hip_status(gh::launch_clear(w, ctr, gh::kClearAll, s), "clear")) != GH_OK) return st;
  return hip_status(gh::launch_hop(d, g, w, ctr, gh::current_tuning().hop_lanes_per_ray, s), "hop");
}

gh_status gh_hop_traced(const gh_sdb_desc* desc_h, const gh_grid* grid_h, void* ws, size_t ws_bytes,
                        int64_t corner_cap, gh_counters* ctr, void* stream) {
  gh::DevSdb d;
  gh::Grid g;
  gh::Workspace w;
  gh_status st;
  if ((st = read_desc(desc_h, &d)) != GH_OK) return st;
  if (d.kind != GH_SDB_PRIMS) return fail(GH_EUNSUPPORTED, "gh_hop_traced takes analytic bounds only");
  if ((st = read_grid(grid_h, &g)) != GH_OK) return st;
  if ((st = carve(g, ws, ws_bytes, corner_cap, &w)) != GH_OK) return st;
  if (!ctr) return fail(GH_EINVAL, "counters are NULL");
  hipStream_t s = (hipStream_t)stream;
  if ((st = hip_status(gh::launch_clear(w, ctr, gh::kClearAll, s), "clear")) != GH_OK) return st;
  return hip_status(gh::launch_hop_traced(d, g, w, ctr, gh::current_tuning().hop_lanes_per_ray, s), "traced hop");
}

gh_status gh_dense(const gh_sdb_desc* desc_h, const gh_grid* grid_h, void* ws, size_t ws_bytes, int64_t corner_cap,
                   uint32_t* signs, gh_counters* ctr, void* stream) {
  gh::DevSdb d;
  gh::Grid g;
  gh::Workspace w;
  gh_status st;
  if ((st = read_desc(desc_h, &d)) != GH_OK) return st;
  if ((st = read_grid(grid_h, &g)) != GH_OK) return st;
  if ((st = carve(g, ws, ws_bytes, corner_cap, &w)) != GH_OK) return st;
  if (!ctr || !signs) return fail(GH_EINVAL, "counters or sign buffer is NULL");
  hipStream_t s = (hipStream_t)stream;
  if ((st = hip_status(gh::launch_clear(w, ctr, gh::kClearAll, s), "clear")) != GH_OK) return st;
  return hip_status(gh::launch_dense(d, g, w, signs, ctr, s), "dense");
}

gh_status gh_mc(const gh_sdb_desc* desc_h, const gh_grid* grid_h, void* ws, size_t ws_bytes, int64_t corner_cap,
                float* verts, int64_t* vert_edge, float* vert_t, int64_t vert_cap, int32_t* tris, int64_t tri_cap,
                int64_t* cells, uint8_t* cases, int64_t cell_cap, gh_counters* ctr, void* stream) {
  gh::DevSdb d;
  gh::Grid g;
  gh::Workspace w;
  gh_status st;
  if ((st = read_desc(desc_h, &d)) != GH_OK) return st;
  if ((st = read_grid(grid_h, &g)) != GH_OK) return st;
  if ((st = carve(g, ws, ws_bytes, corner_cap, &w)) != GH_OK) return st;
  if (!ctr) return fail(GH_EINVAL, "counters are NULL");
  if (vert_cap < 0 || tri_cap < 0 || cell_cap < 0) return fail(GH_EINVAL, "negative capacity");
  if ((vert_cap > 0 && !verts) || (tri_cap > 0 && !tris)) return fail(GH_EINVAL, "output buffer is NULL");
  if (tri_cap >= ((int64_t)1 << 31) || vert_cap >= gh::kMaxVerts)
    return fail(GH_EUNSUPPORTED, "capacities must stay below 2^31 triangles and 2^28 vertices");
  if (!cells && !cases) cell_cap = 0;
  return hip_status(gh::launch_mc(d, g, w, verts, vert_edge, vert_t, vert_cap, tris, tri_cap, cells, cases, cell_cap,
                                  ctr, (hipStream_t)stream),
                    "mc");
}

gh_status gh_polygonize_noalloc(const gh_sdb_desc* desc_h, const gh_grid* grid_h, int64_t corner_cap, float* verts,
                                int64_t* vert_edge, float* vert_t, int64_t vert_cap, int32_t* tris, int64_t tri_cap,
                                int64_t* cells, uint8_t* cases, int64_t cell_cap, gh_counters* ctr, void* stream) {
  gh::DevSdb d;
  gh::Grid g;
  gh::Workspace w;
  gh_status st;
  if ((st = read_desc(desc_h, &d)) != GH_OK) return st;
  if ((st = read_grid(grid_h, &g)) != GH_OK) return st;
  if (!ctr) return fail(GH_EINVAL, "counters are NULL");
  if (vert_cap < 0 || tri_cap < 0 || cell_cap < 0) return fail(GH_EINVAL, "negative capacity");
  if ((vert_cap > 0 && !verts) || (tri_cap > 0 && !tris)) return fail(GH_EINVAL, "output buffer is NULL");
  if (tri_cap >= ((int64_t)1 << 31) || vert_cap >= gh::kMaxVerts)
    return fail(GH_EUNSUPPORTED, "capacities must stay below 2^31 triangles and 2^28 vertices");
  if (!cells && !cases) cell_cap = 0;
  const size_t bytes = GH_NOALLOC_WORKSPACE_BYTES;
  if (corner_cap <= 0) corner_cap = std::min(default_cap(g.n), largest_cap(g.n, bytes));
  if (corner_cap <= 0 || corner_cap >= ((int64_t)1 << 31) ||
      gh::workspace_layout(g.n, corner_cap, nullptr, nullptr) > bytes)
    return fail(GH_ECAPACITY,
                "the fixed workspace of %zu bytes holds n=%d with at most %lld corners (corner_cap %lld asked)",
                bytes, g.n, (long long)largest_cap(g.n, bytes), (long long)corner_cap);
  void* ws = nullptr;
  if ((st = scratch_of_current_device(&ws)) != GH_OK) return st;
  if ((st = carve(g, ws, bytes, corner_cap, &w)) != GH_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int lanes = gh::current_tuning().hop_lanes_per_ray;
  if ((st = hip_status(gh::launch_clear(w, ctr, gh::kClearAll, s), "clear")) != GH_OK) return st;
  if ((st = hip_status(gh::launch_hop(d, g, w, ctr, lanes, s), "hop")) != GH_OK) return st;
  return hip_status(gh::launch_mc(d, g, w, verts, vert_edge, vert_t, vert_cap, tris, tri_cap, cells, cases, cell_cap,
                                  ctr, s),
                    "mc");
}

gh_status gh_cont_workspace_size(const gh_grid* grid_h, int64_t frontier_cap, size_t* bytes_h) {
  gh::Grid g;
  gh_status st = read_grid(grid_h, &g);
  if (st != GH_OK) return st;
  if (!bytes_h) return fail(GH_EINVAL, "bytes_h is NULL");
  if (frontier_cap <= 0) frontier_cap = default_cap(g.n);
  *bytes_h = gh::cont_layout(g.n, frontier_cap, nullptr, nullptr);
  return GH_OK;
}

gh_status gh_cont(const gh_sdb_desc* desc_h, const gh_grid* grid_h, void* ws, size_t ws_bytes, int64_t corner_cap,
                  void* cws, size_t cws_bytes, int64_t frontier_cap, const int64_t* seeds, int64_t n_seeds,
                  gh_counters* ctr, int64_t* levels_h, void* stream) {
  gh::DevSdb d;
  gh::Grid g;
  gh::Workspace w;
  gh_status st;
  if ((st = read_desc(desc_h, &d)) != GH_OK) return st;
  if (d.kind != GH_SDB_PRIMS) return fail(GH_EUNSUPPORTED, "gh_cont takes analytic bounds only");
  if ((st = read_grid(grid_h, &g)) != GH_OK) return st;
  if ((st = carve(g, ws, ws_bytes, corner_cap, &w)) != GH_OK) return st;
  if (!ctr || !cws) return fail(GH_EINVAL, "counters or continuation workspace are NULL");
  if (((uintptr_t)cws) & 255) return fail(GH_EINVAL, "continuation workspace must be 256-byte aligned");
  if (frontier_cap <= 0) frontier_cap = default_cap(g.n);
  gh::ContWorkspace cw;
  const size_t need = gh::cont_layout(g.n, frontier_cap, &cw, cws);
  if (cws_bytes < need) return fail(GH_ECAPACITY, "continuation workspace of %zu bytes, %zu needed", cws_bytes, need);
  if (n_seeds < 0 || n_seeds > frontier_cap) return fail(GH_EINVAL, "n_seeds = %lld must be in [0, frontier_cap]",
                                                         (long long)n_seeds);
  if (n_seeds > 0 && !seeds) return fail(GH_EINVAL, "seeds are NULL");
  hipStream_t s = (hipStream_t)stream;
  if ((st = hip_status(gh::launch_clear(w, ctr, gh::kClearAll, s), "clear")) != GH_OK) return st;
  return hip_status(gh::run_cont(d, g, w, cw, seeds, n_seeds, ctr, levels_h, s), "continuation");
}

gh_status gh_candidates(const gh_grid* grid_h, void* ws, size_t ws_bytes, int64_t corner_cap, int64_t* out,
                        int64_t cap, gh_counters* ctr, void* stream) {
  gh::Grid g;
  gh::Workspace w;
  gh_status st;
  if ((st = read_grid(grid_h, &g)) != GH_OK) return st;
  if ((st = carve(g, ws, ws_bytes, corner_cap, &w)) != GH_OK) return st;
  if (!ctr || (cap > 0 && !out) || cap < 0) return fail(GH_EINVAL, "bad output or counters");
  hipStream_t s = (hipStream_t)stream;
  if ((st = hip_status(gh::launch_clear(w, ctr, gh::kClearCands, s), "clear")) != GH_OK) return st;
  return hip_status(gh::launch_candidates(g, w, out, cap, ctr, s), "candidates");
}

gh_status gh_batch_validate_item(const gh_batch_item* it, int index, gh::DevSdb* d, gh::Grid* g, gh::Workspace* w) {
  gh_status st;
  if (!it) return fail(GH_EINVAL, "batch item %d is NULL", index);
  if ((st = read_desc(&it->desc, d)) != GH_OK) return st;
  if ((st = read_grid(&it->grid, g)) != GH_OK) return st;
  if ((st = carve(*g, it->ws, it->ws_bytes, it->corner_cap, w)) != GH_OK) return st;
  if (!it->ctr) return fail(GH_EINVAL, "batch item %d has no counters", index);
  if (it->vert_cap < 0 || it->tri_cap < 0 || it->cell_cap < 0) return fail(GH_EINVAL, "negative capacity");
  if ((it->vert_cap > 0 && !it->verts) || (it->tri_cap > 0 && !it->tris))
    return fail(GH_EINVAL, "batch item %d output buffer is NULL", index);
  if (it->tri_cap >= ((int64_t)1 << 31) || it->vert_cap >= gh::kMaxVerts)
    return fail(GH_EUNSUPPORTED, "batch item %d: capacities must stay below 2^31 triangles and 2^28 vertices", index);
  return GH_OK;
}

gh_status gh_param_count(const gh_sdb_desc* desc_h, int64_t* count_h) {
  gh::DevSdb d;
  gh_status st;
  if ((st = read_desc(desc_h, &d)) != GH_OK) return st;
  if (d.kind != GH_SDB_MLP) return fail(GH_EUNSUPPORTED, "parameters exist for network bounds only");
  if (!count_h) return fail(GH_EINVAL, "count_h is NULL");
  *count_h = gh::mlp_param_count(d.mlp);
  return GH_OK;
}

gh_status gh_backward_workspace_size(const gh_sdb_desc* desc_h, int64_t corner_cap, size_t* bytes_h) {
  gh::DevSdb d;
  gh_status st;
  if ((st = read_desc(desc_h, &d)) != GH_OK) return st;
  if (d.kind != GH_SDB_MLP) return fail(GH_EUNSUPPORTED, "the adjoint exists for network bounds only");
  if (!bytes_h) return fail(GH_EINVAL, "bytes_h is NULL");
  if (corner_cap <= 0) return fail(GH_EINVAL, "corner_cap must be the workspace's (> 0)");
  *bytes_h = gh::backward_layout(d.mlp, corner_cap, nullptr, nullptr);
  return GH_OK;
}

gh_status gh_backward(const gh_sdb_desc* desc_h, const gh_grid* grid_h, void* ws, size_t ws_bytes, int64_t corner_cap,
                      const float* dL_dverts, float* dL_dtheta, void* bws, size_t bws_bytes, gh_counters* ctr,
                      void* stream) {
  gh::DevSdb d;
  gh::Grid g;
  gh::Workspace w;
  gh_status st;
  if ((st = read_desc(desc_h, &d)) != GH_OK) return st;
  if (d.kind != GH_SDB_MLP) return fail(GH_EUNSUPPORTED, "the adjoint exists for network bounds only");
  if (d.mlp.relu) return fail(GH_EUNSUPPORTED, "the adjoint takes softplus networks only");
  if ((st = read_grid(grid_h, &g)) != GH_OK) return st;
  if ((st = carve(g, ws, ws_bytes, corner_cap, &w)) != GH_OK) return st;
  if (!dL_dverts || !dL_dtheta || !ctr || !bws) return fail(GH_EINVAL, "NULL buffer");
  if (((uintptr_t)bws) & 255) return fail(GH_EINVAL, "backward workspace must be 256-byte aligned");
  const size_t need = gh::backward_layout(d.mlp, w.cap, nullptr, nullptr);
  if (bws_bytes < need) return fail(GH_ECAPACITY, "backward workspace of %zu bytes, %zu needed", bws_bytes, need);
  gh::BackwardWs bw;
  gh::backward_layout(d.mlp, w.cap, bws, &bw);
  return hip_status(gh::launch_backward(d, g, w, bw, dL_dverts, dL_dtheta, ctr, (hipStream_t)stream), "backward");
}

gh_status gh_bf16_margin(const gh_sdb_desc* desc_h, int32_t precision, const float* xyz, int64_t m, float factor,
                         float* f32, float* flp, float* margin, float* offset, void* stream) {
  gh::DevSdb d;
  gh_status st;
  if ((st = read_desc(desc_h, &d)) != GH_OK) return st;
  if (d.kind != GH_SDB_MLP) return fail(GH_EINVAL, "gh_bf16_margin takes a network bound");
  if (!(precision == GH_PREC_BF16 || precision == GH_PREC_BF16X3))
    return fail(GH_EINVAL, "precision %d: GH_PREC_BF16 or GH_PREC_BF16X3", precision);
  if (m < 0) return fail(GH_EINVAL, "negative point count");
  if (!(factor >= 1.f && factor <= 1e3f)) return fail(GH_EINVAL, "factor must be in [1, 1000]");
  if (!margin || (m > 0 && (!xyz || !f32 || !flp))) return fail(GH_EINVAL, "NULL buffer");
  const int prec = precision == GH_PREC_BF16 ? gh::kPrecBf16 : gh::kPrecBf16x3;
  return hip_status(gh::launch_bf16_margin(d, prec, xyz, m, factor, f32, flp, margin, offset, (hipStream_t)stream),
                    "bf16 margin");
}

gh_status gh_eval_points(const gh_sdb_desc* desc_h, const float* xyz, float* f, int64_t m, void* stream) {
  gh::DevSdb d;
  gh_status st;
  if ((st = read_desc(desc_h, &d)) != GH_OK) return st;
  if (m < 0) return fail(GH_EINVAL, "negative point count");
  if (m == 0) return GH_OK;
  if (!xyz || !f) return fail(GH_EINVAL, "points or output is NULL");
  return hip_status(gh::launch_eval_points(d, xyz, f, m, (hipStream_t)stream), "eval");
}

}  // extern "C"
