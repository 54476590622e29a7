/*
 * gh.h - grid hopping polygonizer for MI355X (gfx950), C ABI.
 *
 * The method (Markus & Suznjevic, "Theoretical and Empirical Analysis of a
 * Fast Algorithm for Extracting Polygons from Signed Distance Bounds"):
 * sphere tracing along the N^2 axis-aligned cell columns of an N^3 grid,
 * continued past the surface (Section 3, eq. iter and Algorithm 1), then
 * marching cubes on the cells the rays stop in.  Each step evaluates the
 * signed distance bound f at the centroid of cell (i, j, k) of the column and
 * skips s = floor(|f|/h) cells; s == 0 moves on by one and marks the cell as
 * a candidate when |f| <= (sqrt 3 / 2 + 1/32) h (a cell the surface crosses
 * holds a zero within half its diagonal of the centroid, and |f| is at most
 * the distance to the surface; h/32 covers float32 error up to h/64 in the
 * values, and grids with h below 2^-12 of the largest of 1, |lo| and
 * |lo + n h| take every cell with s == 0).  Section 5 requires the same mesh as marching
 * cubes over every cell ("enumeration", Section 2), which gh_dense provides
 * for comparison.
 *
 * Conventions shared by every entry point
 *  - Pointers are DEVICE pointers unless their name ends in _h (host).
 *  - Every call enqueues work on `stream` (a hipStream_t) and returns without
 *    synchronizing, except sdb_describe, which waits for its upload.
 *  - The library allocates no device memory.  The caller owns every buffer:
 *    descriptor blobs, workspaces, counters and outputs.
 *  - Argument errors are detected on the host before anything is enqueued
 *    and returned synchronously (GH_EINVAL, GH_EUNSUPPORTED); gh_last_error()
 *    then describes them.  Launch failures return GH_EHIP.
 *  - Data-dependent errors (an output or workspace capacity exceeded, a
 *    non-finite bound value) are reported asynchronously in gh_counters.flags.
 *    On overflow the counts still hold the sizes required and nothing is
 *    written past any capacity; the caller re-runs with larger buffers.
 *  - Calls that share a workspace or counters must be ordered on one stream.
 *
 * Grid: cube [lo, lo + n*h]^3 split into n^3 cells (Section 3, eq. cells, with
 * the unit cube generalised to any origin and step).  Lattice point
 * P(a, b, c) = lo + (a, b, c)*h, 0 <= a, b, c <= n; cell (i, j, k) spans
 * P(i, j, k)..P(i+1, j+1, k+1), centroid lo + (i + 1/2, j + 1/2, k + 1/2)*h.
 * Rays run along +z, one per column (i, j) (Section 3, the rays R_ij).
 * Ids: cell (i*n + j)*n + k; lattice point (a*(n+1) + b)*(n+1) + c;
 * lattice edge 3*point + axis (0 = x, 1 = y, 2 = z) from its lower end.
 * Supported: 1 <= n <= 2048.
 *
 * Arithmetic: the analytic bounds are evaluated in float32 with one rounding
 * per operation in a documented order (no contraction); the hop test
 * s = floor(|f| * inv_h), inv_h = float32(1/h), and the candidate test
 * |f| <= float32((sqrt 3 / 2 + 1/32) h) (factor and product in double,
 * rounded once) are taken in float32; vertex parameters t = f_a/(f_a - f_b)
 * are float32.
 */
#ifndef GH_H
#define GH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GH_OK = 0,
  GH_EINVAL = -1,        /* bad argument (null pointer, size, grid) */
  GH_ECAPACITY = -2,     /* a caller buffer or workspace is too small */
  GH_EHIP = -3,          /* the HIP runtime reported an error */
  GH_EUNSUPPORTED = -4,  /* valid but not supported (e.g. n > 2048) */
  GH_ENONFINITE = -5     /* the bound returned NaN or Inf */
} gh_status;

/* Bits of gh_counters.flags (asynchronous data errors). */
#define GH_FLAG_CAPACITY 1u  /* some output/workspace capacity was exceeded */
#define GH_FLAG_NONFINITE 2u /* a bound value was NaN or Inf */
#define GH_FLAG_INTERNAL 4u  /* inconsistent workspace contents (a library bug) */

typedef struct {
  int32_t n;  /* cells per axis */
  float lo;   /* cube origin (all three axes) */
  float h;    /* cell edge length, > 0 */
} gh_grid;

/* Device-resident statistics and data-error flags of a polygonization.
 * gh_hop (and gh_dense) reset the whole struct; gh_mc fills the rest. */
typedef struct {
  int64_t n_hop_evals;    /* bound evaluations by the hop (gh_dense: (n+1)^3) */
  int64_t n_cand;         /* candidate cells (gh_dense: sign-change cells) */
  int64_t n_corner;       /* distinct lattice points of candidates, evaluated once */
  int64_t n_cells;        /* cells that produced triangles */
  int64_t n_vert;         /* welded vertices (one per crossing lattice edge) */
  int64_t n_tri;          /* triangles */
  int64_t n_reeval;       /* float32 re-evaluations taken by the bf16 network path */
  uint32_t flags;         /* GH_FLAG_* */
  uint32_t reserved;
} gh_counters;

/* ----------------------------------------------------------------- bounds */
enum { GH_SDB_PRIMS = 1, GH_SDB_MLP = 2 };
/* Network arithmetic on the matrix cores, all with FP32 accumulation:
 *   FP32    v_mfma_f32_32x32x2f32 on float activations and weights
 *   BF16    v_mfma_f32_32x32x16_bf16 on bf16 activations and weights
 *   BF16X3  the bf16 instruction on hi + lo bf16 splits (hi*hi + hi*lo + lo*hi)
 * In both bf16 modes every decision a value feeds (the hop test, corner and
 * lattice signs) is re-evaluated in FP32 when it lies within bf16_margin of
 * changing, so schedules and signs are the FP32 ones (n_reeval counts). */
enum { GH_PREC_FP32 = 0, GH_PREC_BF16 = 1, GH_PREC_BF16X3 = 2 };
/* Activation of the hidden layers: softplus (the default, smooth) or ReLU
 * max(z, 0), the paper's choice (Section 5.2; batch normalisation folds into
 * the weights and biases at inference). */
enum { GH_ACT_SOFTPLUS = 0, GH_ACT_RELU = 1 };
/* Hop rule of the bf16 modes (the corner and lattice signs are certified in
 * either, so the mesh is the FP32 one):
 *   GH_BF16_HOP_FP32    a value whose step floor(|f|/h) or candidate test
 *                       could change within bf16_margin is re-evaluated in
 *                       FP32 first: the hop schedule, candidates and counts
 *                       are the FP32 ones
 *   GH_BF16_HOP_SHRINK  the step and the candidate test take
 *                       max(|f| - bf16_margin, 0) from the bf16 value alone
 *                       (it bounds the FP32 value's magnitude from below, so
 *                       no cell the surface crosses is skipped or left
 *                       unmarked): no FP32 in the hop, at the price of
 *                       shorter steps and more candidates */
enum { GH_BF16_HOP_FP32 = 0, GH_BF16_HOP_SHRINK = 1 };

/* Primitive record: 16 float32 values.
 *  [0] type: 0 sphere, 1 box (exact), 2 torus, 3 capsule, 4 plane,
 *            5 box bound (max of six face planes, Section 4.2 eq. boxdist),
 *            6 cylinder, 7 cone, 8 hexagonal prism (Section 5.1's primitives),
 *            9 the implicit surface of genus 2 of Section 5.1, scaled,
 *            10 the Sierpinski tetrahedron of Section 5.1's fractal scene
 *  [1..3] centre c;  [4..12] 3x3 matrix M row-major, local q = M (p - c)
 *  [13..15] sphere (r), box/box bound (bx, by, bz), torus (R, r) about local y,
 *           capsule (a, r) on local z in [-a, a] (a >= 0), plane (d) with f = M_row0 . p - d,
 *           cylinder (r, a) capped at local z = -a, a (exact distance),
 *           cone (a, s, c): apex at local z = a, axis -z, half-angle of sine s and
 *           cosine c (s^2 + c^2 <= 1), cut at z = -a (max of side and cap: a bound),
 *           hexagonal prism (r, a): apothem r with one pair of faces normal to local
 *           x, capped at z = -a, a (max of the face planes: a bound),
 *           genus 2 (k): k F(q) with F = 2y(y^2-3x^2)(1-z^2) + (x^2+y^2)^2 - (9z^2-1)(1-z^2);
 *           the caller picks k so that |grad| <= 1 wherever it is evaluated,
 *           Sierpinski (k, d): the tetrahedron of depth d (an integer in [0, 16])
 *           on the regular tetrahedron with vertices (1,1,1), (1,-1,-1), (-1,1,-1),
 *           (-1,-1,1) in local q; d times q = 2q - v_b with v_b the nearest vertex
 *           (largest v . q, lowest index on ties), then k 2^-d times the signed
 *           distance to the tetrahedron at the last q: the exact signed distance to
 *           the set in local units.  With M = s R (R a rotation) k = 1/s makes it
 *           the distance in world units; k > 0 (with k >= 2^27 the hop takes the
 *           LDS-record kernel with exact roots).
 * The bound is the minimum over the records (union, Section 4.3). */
#define GH_PRIM_FLOATS 16
/* Number of record types: the type field is an integer in [0, GH_PRIM_TYPES). */
#define GH_PRIM_TYPES 11

typedef struct {
  int32_t kind;                  /* GH_SDB_PRIMS or GH_SDB_MLP */
  /* GH_SDB_PRIMS */
  int32_t n_prim;                /* 1 .. 64 */
  const float* prims_h;          /* n_prim * GH_PRIM_FLOATS, host */
  /* GH_SDB_MLP (eq. nnsdb): f = a_s (||p|| - r0) + a_n NN(gamma(p)) + b,
   * gamma(p) = [p, for each k: sin(w_k p_x,y,z), cos(w_k p_x,y,z)],
   * NN = W_D ... act(W_1 gamma + b_1) ... + b_D, D = depth + 1 layers. */
  int32_t n_freq;                /* 0 .. 16 */
  int32_t width;                 /* 64, 128 or 256 */
  int32_t depth;                 /* hidden layers, 1 .. 8 */
  int32_t precision;             /* GH_PREC_FP32, GH_PREC_BF16 or GH_PREC_BF16X3 */
  const float* omegas_h;         /* n_freq, host */
  const float* const* weights_h; /* depth+1 host arrays, row-major fan_out x fan_in */
  const float* const* biases_h;  /* depth+1 host arrays of fan_out */
  float a_s, r0, a_n, b;
  float bf16_margin;             /* eps >= max |f_bf16 - f_fp32|, > 0 in the bf16 modes (gh_bf16_margin) */
  int32_t activation;            /* GH_ACT_SOFTPLUS (0) or GH_ACT_RELU; gh_backward takes softplus only */
  int32_t bf16_hop;              /* GH_BF16_HOP_FP32 (0) or GH_BF16_HOP_SHRINK (bf16 modes) */
  float bf16x3_margin;           /* GH_PREC_BF16 only: eps3 >= max |f_bf16x3 - f_fp32| > 0 certifies the corner
                                    values within bf16_margin of zero in two steps, bf16x3 first and FP32 only
                                    within eps3 of zero; 0: those corners go to FP32 directly */
  float bf16_offset;             /* GH_PREC_BF16 only: subtracted from every plain bf16 value (hop, corners,
                                    points); with the offset gh_bf16_margin measures, bf16_margin bounds
                                    |f_bf16 - bf16_offset - f_fp32|; 0 elsewhere */
} gh_sdb_spec;

/* Opaque, caller-owned, plain-old-data handle filled by sdb_describe.  It
 * refers to the device blob, which must outlive every call that uses it. */
typedef struct {
  uint64_t opaque[32];
} gh_sdb_desc;

/* Validate a bound and pack it into the caller's device blob.
 * spec_h: host.  dev_blob: device memory of blob_bytes (may be NULL to query
 * the size, written to *blob_needed_h).  desc_h: host, filled on success.
 * Uploads on `stream` and waits for the upload.  Returns GH_ECAPACITY when
 * blob_bytes < *blob_needed_h, GH_EINVAL / GH_EUNSUPPORTED on a bad spec. */
gh_status sdb_describe(const gh_sdb_spec* spec_h, void* dev_blob, size_t blob_bytes,
                       size_t* blob_needed_h, gh_sdb_desc* desc_h, void* stream);

/* Workspace bytes for gh_hop/gh_mc on this grid, holding up to corner_cap
 * distinct corner points (corner_cap <= 0 selects 16*(n+1)^2). */
gh_status gh_workspace_size(const gh_grid* grid_h, int64_t corner_cap, size_t* bytes_h);

/* Grid hopping over all n^2 columns (Section 3, Algorithm 1).  Records the
 * candidate cells in the workspace and resets *ctr, then sets n_hop_evals,
 * n_cand and flags.  ws: device, ws_bytes >= gh_workspace_size(grid, corner_cap). */
gh_status gh_hop(const gh_sdb_desc* desc_h, const gh_grid* grid_h, void* ws, size_t ws_bytes,
                 int64_t corner_cap, gh_counters* ctr, void* stream);

/* The paper's per-column procedure taken literally (Section 3: eq. iter,
 * eq. polydist and Algorithm 1), for comparison with gh_hop.  From the
 * centroid of cell k each ray is sphere-traced in +z until |f| <= sqrt(6)/2 h
 * or its travel reaches 1.05 x the distance to the top face; the cell of the
 * last centroid at or below the stopping point (never below k) is a
 * candidate unless it lies past the last cell or the stopping point is above
 * the overrun height lo + N h/2 + 1.05 N h/2; the ray resumes at the next
 * cell.  Unlike gh_hop this rule can miss cells that the surface crosses.
 * Same arguments, workspace contents and counters as gh_hop (n_hop_evals
 * counts every evaluation of the traces), so gh_mc can follow it.  Analytic
 * bounds only (GH_EUNSUPPORTED for a network).  GH_FLAG_INTERNAL if a ray
 * took (N+2)^2 + 64 evaluations, which the rule cannot need. */
gh_status gh_hop_traced(const gh_sdb_desc* desc_h, const gh_grid* grid_h, void* ws, size_t ws_bytes,
                        int64_t corner_cap, gh_counters* ctr, void* stream);

/* Bytes of the continuation workspace for this grid with room for
 * frontier_cap cells per level (frontier_cap <= 0 selects 16*(n+1)^2). */
gh_status gh_cont_workspace_size(const gh_grid* grid_h, int64_t frontier_cap, size_t* bytes_h);

/* Continuation, the paper's surface-following comparator (Section 2): from
 * the seed cells (device list of n_seeds cell ids (i*n + j)*n + k; ids outside
 * the grid are ignored) the search moves to every face neighbour behind a
 * face whose four corners do not share one sign, until no new cell appears.
 * It reaches every sign-change cell of each surface component holding a
 * seed, and only sign-change cells besides the seeds.  The cells reached go
 * to ws as candidates (gh_mc can follow); n_hop_evals counts the distinct
 * lattice points evaluated and n_cand the cells.  cws: device, 256-byte
 * aligned, cws_bytes >= gh_cont_workspace_size.  GH_FLAG_CAPACITY when a
 * level held more than frontier_cap cells (the search then goes on with the
 * first frontier_cap of them and its result is incomplete).  Runs one kernel
 * per level in batches and waits for each batch on `stream`: the call returns
 * when the search is done; *levels_h (may be NULL) receives the number of
 * levels.
 * Analytic bounds only (GH_EUNSUPPORTED for a network). */
gh_status gh_cont(const gh_sdb_desc* desc_h, const gh_grid* grid_h, void* ws, size_t ws_bytes, int64_t corner_cap,
                  void* cws, size_t cws_bytes, int64_t frontier_cap, const int64_t* seeds, int64_t n_seeds,
                  gh_counters* ctr, int64_t* levels_h, void* stream);

/* Marching cubes on the cells recorded in ws by gh_hop, gh_hop_traced, gh_cont or gh_dense
 * (Section 5: every reached cell is polygonized by marching cubes).
 * Evaluates the bound once per distinct corner point, welds one vertex per
 * crossing lattice edge and writes:
 *   verts     [vert_cap][3] float32 positions, ordered by lattice edge id
 *   vert_edge [vert_cap] int64 lattice edge id of each vertex (may be NULL)
 *   vert_t    [vert_cap] float32 edge parameter t (may be NULL)
 *   tris      [tri_cap][3] int32 vertex indices, facing from f < 0 to f >= 0,
 *             grouped by cell in cell-id order
 *   cells     [cell_cap] int64 ids of cells with triangles, ascending (may be NULL)
 *   cases     [cell_cap] uint8 inside-corner mask of those cells, corner
 *             dx + 2 dy + 4 dz inside when f < 0 (may be NULL)
 * Sets n_corner, n_cells, n_vert, n_tri; GH_FLAG_CAPACITY if any capacity
 * (including the workspace corner_cap) was too small.  Capacities must stay
 * below 2^28 vertices and 2^31 triangles (GH_EUNSUPPORTED). */
gh_status gh_mc(const gh_sdb_desc* desc_h, const gh_grid* grid_h, void* ws, size_t ws_bytes,
                int64_t corner_cap, float* verts, int64_t* vert_edge, float* vert_t, int64_t vert_cap,
                int32_t* tris, int64_t tri_cap, int64_t* cells, uint8_t* cases, int64_t cell_cap,
                gh_counters* ctr, void* stream);

/* Bytes of the fixed workspace of gh_polygonize_noalloc (128 MiB per device). */
#define GH_NOALLOC_WORKSPACE_BYTES ((size_t)128 << 20)

/* gh_hop followed by gh_mc with no workspace argument and no allocation, for
 * callers that cannot allocate device memory (code under hipGraph capture,
 * serving loops, hosts that forbid hipMalloc).  The workspace is a
 * GH_NOALLOC_WORKSPACE_BYTES array in the library's device code, one per
 * device, taken on the current device (the stream must belong to it) and
 * held until the process ends; this call allocates and frees nothing.
 * Outputs, capacities and counters are those of gh_mc; corner_cap <= 0
 * selects the default of gh_workspace_size or the largest capacity that
 * fits, whichever is smaller.  GH_ECAPACITY (synchronous, nothing enqueued)
 * when the grid with that corner capacity needs a larger workspace: the
 * array holds any n <= 512 with the default capacity up to n = 256 and about
 * 2.9e6 corners at n = 512.  Every call on one device shares the array, and
 * it keeps the last call's contents: calls that overlap on one device (other
 * streams, other threads) race and must be ordered by the caller. */
gh_status gh_polygonize_noalloc(const gh_sdb_desc* desc_h, const gh_grid* grid_h, int64_t corner_cap, float* verts,
                                int64_t* vert_edge, float* vert_t, int64_t vert_cap, int32_t* tris, int64_t tri_cap,
                                int64_t* cells, uint8_t* cases, int64_t cell_cap, gh_counters* ctr, void* stream);

/* Enumeration baseline (Section 2): evaluates f at every lattice point,
 * keeps only the signs in `signs` (device, gh_dense_signs_size bytes,
 * layout [w][a*(n+1) + b], bit c%32 of word w = c/32 set when
 * f(P(a, b, c)) < 0), records every sign-change cell in ws as the candidate
 * set and resets *ctr (n_hop_evals = (n+1)^3).  gh_mc then polygonizes
 * exactly as after gh_hop. */
gh_status gh_dense(const gh_sdb_desc* desc_h, const gh_grid* grid_h, void* ws, size_t ws_bytes,
                   int64_t corner_cap, uint32_t* signs, gh_counters* ctr, void* stream);

/* Bytes of the sign buffer of gh_dense: ceil((n+1)/32) * (n+1)^2 * 4. */
gh_status gh_dense_signs_size(const gh_grid* grid_h, size_t* bytes_h);

/* Export the candidate cells recorded in ws as ascending int64 cell ids into
 * out[cap]; the count is n_cand of *ctr.  Sets GH_FLAG_CAPACITY if cap is
 * too small. */
gh_status gh_candidates(const gh_grid* grid_h, void* ws, size_t ws_bytes, int64_t corner_cap,
                        int64_t* out, int64_t cap, gh_counters* ctr, void* stream);

/* Number of network parameters (GH_SDB_MLP): sum over layers of
 * (fan_in + 1) * fan_out, in the order W_0, b_0, W_1, b_1, ..., W_D, b_D
 * (each W row-major fan_out x fan_in). */
gh_status gh_param_count(const gh_sdb_desc* desc_h, int64_t* count_h);

/* Workspace bytes of gh_backward for this network and corner capacity. */
gh_status gh_backward_workspace_size(const gh_sdb_desc* desc_h, int64_t corner_cap, size_t* bytes_h);

/* Adjoint of a loss on the vertices of the last gh_mc on ws (network bounds).
 * A vertex on lattice edge a -> b sits at P_a + t h e_axis, t = f_a/(f_a - f_b);
 * the corner values get the cotangents (dL/dv . e) h dt/df, and the
 * network's parameters dL/dtheta = a_n sum_c gbar_c dNN(P_c)/dtheta by
 * back-propagation in FP32 on the matrix cores.  The cell set is piecewise
 * constant in theta and is not differentiated.
 *   dL_dverts  [n_vert][3] device, in the vertex order of gh_mc
 *   dL_dtheta  [gh_param_count] device, overwritten
 *   bws        device workspace of gh_backward_workspace_size bytes
 * The result is deterministic (fixed summation order). */
gh_status gh_backward(const gh_sdb_desc* desc_h, const gh_grid* grid_h, void* ws, size_t ws_bytes,
                      int64_t corner_cap, const float* dL_dverts, float* dL_dtheta, void* bws, size_t bws_bytes,
                      gh_counters* ctr, void* stream);

/* Margin of the bf16 decisions of a network bound.  The paper keeps a learned
 * bound safe by shrinking it (Section 5.2, the factor lambda); evaluating it
 * in bf16 adds an error that the hop test and the corner signs must also
 * absorb, and this measures it: the bound at m points xyz [m][3] in FP32 into
 * f32 [m] and in `precision` (GH_PREC_BF16 or GH_PREC_BF16X3) into flp [m],
 * both with the library's own evaluators (raw values: no bf16_offset), then,
 * with d_i = flp[i] - f32[i],
 *   offset NULL:  *margin = factor * max_i |d_i|
 *   otherwise:    *offset = (max_i d_i + min_i d_i) / 2 and
 *                 *margin = factor * (max_i d_i - min_i d_i) / 2
 * (one float each, device) with a fixed reduction order (the same bits every
 * run), or NaN when a value or difference is not finite.  The descriptor
 * may hold any precision (it carries both weight forms).  factor in
 * [1, 1000]; m = 0 gives 0.  Pass the results as gh_sdb_spec.bf16_margin
 * and bf16_offset (the offset only for GH_PREC_BF16): the offset removes
 * the part of the bf16 error that is the same everywhere (most of the
 * weights' rounding), which shrinks the margin.  It is a measured bound over
 * the points given, not a proof, so the points should cover the grid's
 * cube. */
gh_status gh_bf16_margin(const gh_sdb_desc* desc_h, int32_t precision, const float* xyz, int64_t m, float factor,
                         float* f32, float* flp, float* margin, float* offset, void* stream);

/* Evaluate the bound at m points xyz [m][3] (device) into f [m] (device). */
gh_status gh_eval_points(const gh_sdb_desc* desc_h, const float* xyz, float* f, int64_t m, void* stream);

/* ---------------------------------------------------------------- batches
 * Many bounds on their own grids in one persistent hop launch: work items
 * (a block tile of ray columns for an analytic bound, a range of rays for a
 * network) are ordered by estimated cost, longest first, and persistent
 * blocks take them from one counter; then every shape gets its marching
 * cubes.  All network bounds of a batch share one precision. */
typedef struct {
  gh_sdb_desc desc;                 /* from sdb_describe */
  gh_grid grid;
  void* ws;                         /* device workspace of this shape */
  size_t ws_bytes;
  int64_t corner_cap;
  float* verts;                     /* outputs as for gh_mc */
  int64_t* vert_edge;
  float* vert_t;
  int64_t vert_cap;
  int32_t* tris;
  int64_t tri_cap;
  int64_t* cells;
  uint8_t* cases;
  int64_t cell_cap;
  gh_counters* ctr;                 /* device, per shape */
} gh_batch_item;

typedef struct gh_batch gh_batch;   /* host object of a planned batch */

/* Device bytes of the plan (shape table, work items, item counter). */
gh_status gh_batch_buffer_size(int n_shapes, const gh_batch_item* items_h, size_t* bytes_h);
/* Plan a batch into dev_buf (uploads on stream and waits).  The items' buffers
 * must outlive the plan. */
gh_status gh_batch_create(int n_shapes, const gh_batch_item* items_h, void* dev_buf, size_t dev_bytes,
                          void* stream, gh_batch** batch_h);
/* Enqueue one run: reset counters, batched hop, marching cubes per shape. */
gh_status gh_batch_run(gh_batch* batch, void* stream);
/* Capture one run into a hipGraph (replaces a previous capture). */
gh_status gh_batch_capture(gh_batch* batch, void* stream);
/* Launch the captured graph on stream. */
gh_status gh_batch_replay(gh_batch* batch, void* stream);
gh_status gh_batch_item_count(const gh_batch* batch, int64_t* n_items_h);
gh_status gh_batch_destroy(gh_batch* batch);

/* Launch shapes of the kernels, process-wide (an autotuner sets them).
 * Fields left at 0 keep the built-in choice. */
typedef struct {
  int32_t hop_lanes_per_ray;   /* analytic hop: lanes tracing one ray together: 1, 2, 3, 4 or 8 (default:
                                  the largest number of primitives of one type, 8 above 4) */
  int32_t scan_blocks_per_cu;  /* marching-cubes look-back scans: resident blocks per CU, 1, 2, 4 or 8
                                  (default 4; never more than the occupancy allows) */
  int32_t batch_rays_per_item; /* batch: rays per network work item, a power of two in [256, 65536]
                                  (default 4096); read by gh_batch_create */
  int32_t mlp_split;           /* network tiles with few rows: 1 never split, 2 split tiles of <= 32 rows
                                  over four waves, 3 also tiles of <= 64 rows over two (default 3);
                                  values do not depend on it */
  int32_t mc_items_per_thread; /* marching cubes: list entries per thread of the vertex and triangle passes,
                                  1, 2, 4 or 8 (default 4) */
  int32_t hop_step_budget;     /* analytic hop: 0 one pass (default); 1..4096 steps a ray takes in the
                                  first pass, after which a ray still running continues in a second pass
                                  with one wave per ray, which evaluates a window of 64 / lanes cells at
                                  once and steps through it.  Results do not depend on it */
  int32_t mlp_pool_tiles;      /* network hop: rays a block keeps in its pool, in tiles of rows: 1 or 2
                                  (default 2; the second tile's rays wait while others are evaluated) */
  int32_t mlp_spec_rows;       /* network hop: rows of a draining pool's tile shared out as windows of cells
                                  ahead of each ray: 1 (no windows), 8, 16 or 32 (default 32); values and
                                  steps do not depend on it */
  int32_t mlp_lean;            /* plain bf16 networks: 1 (default) runs the shrunk hop (GH_BF16_HOP_SHRINK,
                                  which never waits for FP32 values) and the corner values on a lean LDS
                                  layout with two blocks per CU (at width 256 every tile is then split
                                  over two waves per group, 64 rows), the corner certification as a pass
                                  of its own; 2 runs both on the full layout, one block per CU (a batch
                                  reads it in gh_batch_create); values, steps and signs do not depend
                                  on it */
  int32_t reserved;
} gh_tuning;

/* Replace the process-wide launch shapes; GH_EINVAL for unsupported values. */
gh_status gh_set_tuning(const gh_tuning* tuning_h);
/* Read the launch shapes in effect. */
gh_status gh_get_tuning(gh_tuning* tuning_h);

/* Human-readable description of the last synchronous error on this thread. */
const char* gh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GH_H */
