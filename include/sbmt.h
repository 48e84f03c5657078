/*
 * sbmt.h -- C ABI of the MI355X (gfx950) implementation of Structured
 * Bitmap-to-Mesh Triangulation (SBMT, arXiv 2602.19474).
 *
 * The library turns a binary bitmap into a closed triangle mesh of its
 * foreground: the boundary extracted from the bitmap is embedded into a
 * regular equilateral grid by replacing only the cut base triangles with
 * templates from a finite lookup table (Sec. 3.3, Alg. 1 and Alg. 2, App. G).
 *
 * Conventions
 *  - Pixel (row r, column c) is a unit square centred at (x = c, y = r)
 *    (Sec. 3.3, structured triangular filling).  A nonzero byte is foreground.
 *  - grid_h is the edge length of the base equilateral grid in pixels, a
 *    dyadic rational h = p / 2^q with q <= 8 and 0 < h <= 6 (the paper's grid
 *    has h < 1, Sec. 3.3), with 3h <= 2s for the stride s below, and
 *    16 s 4^q (max(width, height) + 2s + 16) < 2^31 (exact predicates in
 *    64-bit integers); others return SBMT_E_UNSUPPORTED_GRID_H.  The boundary
 *    is taken from a raster coarsened by block majority with the stride
 *    s = min{s : s^2 > 2 h^2} (h = 1/2 -> 1, 1 -> 2, 3/2 -> 3, 2 -> 3, 4 -> 6)
 *    so that every boundary segment is longer than the base edge, as the
 *    geometric protocol of Sec. 3.2 requires.
 *  - Grid rows are horizontal: vertex (k, i) lies at
 *      x = x0 + h*i + (h/2)*(k mod 2),   y = -1 + k*h*sqrt(3)/2,
 *    x0 = -(2h+3)/4 for integer h, -(2h+3)/4 - 2^-(q+2) otherwise (so that no
 *    vertex lies on a boundary line).
 *  - Output vertices are FP64 (x, y) pairs; triangles are int32 index
 *    triples with positive signed area in (x, y); codes are one byte per
 *    triangle: 0 = uncut base triangle, 1..SBMT_NUM_CLASSES = canonical class
 *    of the cut parent triangle (the key kappa(K) of Sec. 3.3.3 reduced by
 *    rotation), bit 7 set = background side (only with SBMT_BOTH_SIDES).
 *  - Vertex and triangle order is canonical and independent of tiling:
 *    vertices by owner lattice vertex (row k, then i): the vertex itself (if
 *    emitted), the crossings on its edges to (k,i+1), (k+1,i+o-1), (k+1,i+o)
 *    (o = k mod 2) in order from the owner, the chain vertex in its triangle
 *    with apex on row k, then the one in its triangle with base on row k.
 *    Triangles by parent base triangle (row k, then i, apex-on-row-k first),
 *    each rotated to start at its smallest index, sorted within the parent.
 *
 * Memory and ownership
 *  - Every pointer named "device" is a device pointer on the handle's device;
 *    the caller allocates and owns all of them (bitmap, workspace, outputs).
 *    The library never allocates device memory on these paths; the handle only
 *    owns a small pinned host buffer used to return sizes.
 *  - Calls on one handle must not overlap (the pinned buffers are shared);
 *    batch objects keep a pointer to their handle, which must outlive them.
 *    Pinned host buffers of batch objects come from a pool of the handle
 *    and are reused, so a serving loop does not allocate pinned memory once
 *    warm.
 *  - The workspace holds the coarse raster, a two-byte code per lattice
 *    vertex, a four-byte word per lattice vertex for the persistent batch
 *    kernel, and 16-byte records of the owners classified exactly (by
 *    default room for half of the owners).
 *
 * Errors
 *  - Every call returns an sbmt_status.  Arguments are validated before any
 *    launch.  On error the output contents are undefined.
 */
#ifndef SBMT_H_
#define SBMT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SBMT_OK = 0,
  SBMT_E_INVALID_ARG = -1,        /* null pointer, negative size, stride < width ... */
  SBMT_E_UNSUPPORTED_GRID_H = -2, /* grid_h not p/2^q (q <= 8), above 6, or too fine for the image */
  SBMT_E_INDEX_OVERFLOW = -3,     /* more than INT32_MAX vertices */
  SBMT_E_WORKSPACE = -4,          /* workspace missing or smaller than required */
  SBMT_E_DEVICE = -5,             /* a HIP runtime call failed */
  SBMT_E_PROTOCOL = -6,           /* an inadmissible local pattern was seen (unreachable by design) */
  SBMT_E_CAPACITY = -7            /* outputs larger than the capacity given to a bounded call */
} sbmt_status;

/* flags */
#define SBMT_BOTH_SIDES 1u /* also emit background-side triangles and all lattice vertices */

typedef struct sbmt_context* sbmt_handle;

/* One image.  bitmap: device pointer to height rows of row_stride bytes,
 * row-major, nonzero = foreground.  width/height >= 0 (0 gives an empty mesh). */
typedef struct {
  const uint8_t* bitmap;
  int32_t width;
  int32_t height;
  int64_t row_stride;
  double grid_h;   /* p / 2^q pixels, see above */
  uint32_t flags;
} sbmt_image;

/* Sizes returned by planning. */
typedef struct {
  int64_t n_vertices;  /* rows of the vertex array (x, y) */
  int64_t n_triangles; /* rows of the triangle array and length of the code array */
  int64_t n_cut;       /* base triangles replaced by a template */
  int64_t n_segments;  /* boundary segments extracted from the coarsened bitmap (the
                          marching-squares polyline pieces, Sec. 3.2; each has length
                          s/sqrt2 or s pixels) */
} sbmt_sizes;

/* Per-image sizes record written to device memory by the asynchronous calls:
 * int64 [SBMT_SIZE_WORDS] = n_vertices, n_triangles, n_cut, status, n_segments. */
#define SBMT_SIZE_WORDS 5

/* Geometry of an image's grid (host-only computation). */
typedef struct {
  int32_t stride_s;      /* coarse stride s */
  int32_t coarse_w, coarse_h;
  int32_t grid_rows;     /* NK */
  int32_t grid_cols;     /* NI */
  size_t workspace_bytes;
} sbmt_layout;

/* Create a context on a HIP device (allocates a small pinned host buffer). */
sbmt_status sbmt_create(int device, sbmt_handle* out);
sbmt_status sbmt_destroy(sbmt_handle h);

/* Host-only: grid geometry and the workspace size for an image. */
sbmt_status sbmt_query(const sbmt_image* img, sbmt_layout* out);

/* Plan (Alg. 1 over every base triangle): extract the boundary, classify every
 * base triangle, count outputs and prefix-sum the output offsets into the
 * workspace.  Enqueued on `stream` (a hipStream_t, may be NULL for the null
 * stream); synchronises that stream to return the sizes in *out. */
sbmt_status sbmt_plan(sbmt_handle h, const sbmt_image* img, void* workspace, size_t ws_bytes,
                      sbmt_sizes* out, void* stream);

/* Run (Alg. 2 for every cut triangle, plus the uncut ones): write the mesh.
 * Requires the workspace produced by sbmt_plan for the same image.  Outputs:
 * verts [n_vertices][2] FP64, tris [n_triangles][3] int32, codes [n_triangles]
 * uint8, all device pointers.  Asynchronous on `stream`. */
sbmt_status sbmt_run(sbmt_handle h, const sbmt_image* img, void* workspace, size_t ws_bytes,
                     double* verts, int32_t* tris, uint8_t* codes, void* stream);

/* Plan and run in one asynchronous call, without a host round trip: outputs are
 * written only if they fit the capacities; the sizes record is written to the
 * device buffer `sizes_dev` (int64 [SBMT_SIZE_WORDS]: n_vertices, n_triangles,
 * n_cut, status, n_segments).  status = SBMT_E_CAPACITY if the mesh did not fit. */
sbmt_status sbmt_mesh_async(sbmt_handle h, const sbmt_image* img, void* workspace, size_t ws_bytes,
                            double* verts, int64_t vert_cap, int32_t* tris, uint8_t* codes,
                            int64_t tri_cap, int64_t* sizes_dev, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): sbmt_mesh_async
 * without the workspace arguments.  The workspace is a scratch array inside
 * the library, SBMT_NOALLOC_SCRATCH_BYTES bytes per GPU, held from the first
 * use of the library on that GPU until the process ends; its device address
 * is looked up once per handle by sbmt_create.  No device memory is allocated
 * by this call (the host does a few small bookkeeping allocations).
 *  - An image whose workspace (sbmt_layout.workspace_bytes of sbmt_query) is
 *    larger than SBMT_NOALLOC_SCRATCH_BYTES returns SBMT_E_WORKSPACE before
 *    any launch; 64 MiB covers an image of about 2200 x 2200 pixels at
 *    grid_h = 1 and 3500 x 3500 at grid_h = 2.
 *  - Every call on one GPU (through any handle of this process) uses the same
 *    array, which keeps the last call's contents: calls that overlap on one
 *    GPU (different streams, or different host threads) race and must be
 *    serialised by the caller.  Nothing in the array needs clearing between
 *    calls (the kernels clear what starts at zero).
 *  - Outputs, capacities, sizes_dev and errors are those of sbmt_mesh_async. */
#define SBMT_NOALLOC_SCRATCH_BYTES (64u << 20)
sbmt_status sbmt_mesh_noalloc(sbmt_handle h, const sbmt_image* img, double* verts, int64_t vert_cap,
                              int32_t* tris, uint8_t* codes, int64_t tri_cap, int64_t* sizes_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Batches: many images of different sizes and grid_h meshed by one set of
 * launches (or one persistent launch), e.g. inside a captured hipGraph.
 *
 * Life cycle:
 *   sbmt_batch_create  host only: validate the images, lay out the workspace
 *   sbmt_batch_bind    upload the image table (bitmaps, workspace regions and,
 *                      optionally, output views) into the workspace; waits for
 *                      the copy, so it is not capturable
 *   sbmt_batch_plan    classify and count every image; waits; per-image sizes
 *                      (sbmt_batch_plan_async + sbmt_batch_host_sizes: the
 *                      same without waiting, for schedulers)
 *   sbmt_batch_emit    write the planned meshes (asynchronous, capturable)
 *   sbmt_batch_mesh    the whole path without a host round trip (asynchronous,
 *                      capturable): an image is written only if it fits its
 *                      output capacities, sizes and statuses go to the
 *                      workspace (read with sbmt_batch_sizes) and to
 *                      sizes_dev if given
 *   sbmt_batch_tune    autotuner: times every candidate tuning on this batch
 *                      and keeps the fastest
 * A batch object and its workspace serve one call at a time; the image
 * bitmaps and outputs must stay valid while calls that use them run.
 * ------------------------------------------------------------------------- */
typedef struct sbmt_batch_s* sbmt_batch;

/* Output view of one image: device arrays with capacities in rows. */
typedef struct {
  double* verts;     /* [vert_cap][2] */
  int32_t* tris;     /* [tri_cap][3] */
  uint8_t* codes;    /* [tri_cap] */
  int64_t vert_cap;
  int64_t tri_cap;
} sbmt_outputs;

#define SBMT_STRATEGY_MULTI 0 /* coarsen, count, slow-owner, scan and emit kernels */
#define SBMT_STRATEGY_FUSED 1 /* coarsen, then one persistent classify-scan-emit kernel */

typedef struct {
  int32_t strategy;      /* SBMT_STRATEGY_* */
  int32_t tile_rows;     /* grid rows per tile or band: 4, 8 or 16 (16: multi only) */
  int32_t groups_per_cu; /* fused: resident workgroups per compute unit (0 = default) */
  int32_t reserved;
  int64_t record_cap;    /* slow-owner records in the workspace: 0 = default
                            (half of the owners), > 0 = that many; owners
                            beyond it are classified where they are needed */
} sbmt_tuning;

/* Host only.  tuning may be NULL (multi-kernel, 8-row tiles).  The fused
 * strategy needs per-image widths up to 12288 * grid_h pixels and at most
 * 2^31 / 10 lattice vertices per image; otherwise the batch uses the
 * multi-kernel strategy.  *ws_bytes receives the workspace size. */
sbmt_status sbmt_batch_create(sbmt_handle h, const sbmt_image* imgs, int32_t n, const sbmt_tuning* tuning,
                              size_t* ws_bytes, sbmt_batch* out);
sbmt_status sbmt_batch_destroy(sbmt_batch b);
/* outs: n output views, or NULL to bind none yet (plan only). */
sbmt_status sbmt_batch_bind(sbmt_batch b, void* workspace, size_t ws_bytes, const sbmt_outputs* outs, void* stream);
/* out: n host sizes.  Returns SBMT_E_PROTOCOL / SBMT_E_INDEX_OVERFLOW if an
 * image has that status (its sizes are still reported). */
sbmt_status sbmt_batch_plan(sbmt_batch b, sbmt_sizes* out, void* stream);
/* Asynchronous plan: the sizes land in a pinned host buffer of the batch once
 * the stream reaches this point (wait for an event recorded after this call,
 * then read them with sbmt_batch_host_sizes). */
sbmt_status sbmt_batch_plan_async(sbmt_batch b, void* stream);
/* Reads the pinned copy written by the last sbmt_batch_plan_async (no wait). */
sbmt_status sbmt_batch_host_sizes(sbmt_batch b, sbmt_sizes* out, int64_t* status);
/* sizes_dev: device int64 [n][SBMT_SIZE_WORDS] (n_vertices, n_triangles, n_cut, status,
 * n_segments) or NULL.
 * Emits what the last plan of this batch counted (with that plan's tile
 * height); SBMT_E_INVALID_ARG if the batch was never planned. */
sbmt_status sbmt_batch_emit(sbmt_batch b, int64_t* sizes_dev, void* stream);
sbmt_status sbmt_batch_mesh(sbmt_batch b, int64_t* sizes_dev, void* stream);
/* Host copy of the last call's per-image sizes and statuses (waits). */
sbmt_status sbmt_batch_sizes(sbmt_batch b, sbmt_sizes* out, int64_t* status, void* stream);
sbmt_status sbmt_batch_get_tuning(sbmt_batch b, sbmt_tuning* out);
sbmt_status sbmt_batch_set_tuning(sbmt_batch b, const sbmt_tuning* t);
/* reps timed runs per candidate; best / best_ms may be NULL. */
sbmt_status sbmt_batch_tune(sbmt_batch b, int32_t reps, sbmt_tuning* best, float* best_ms, void* stream);

/* ---------------------------------------------------------------------------
 * Geometric preprocessing of the grid (Alg. 3, Sec. 3.5; thresholds of
 * Sec. 3.3.4): before the polyline is embedded, the lattice of the image is
 * adapted to it in three steps.
 *   Step 1 (vertex snapping, distance a): a lattice vertex within a of a
 *          polyline vertex (a marching-squares midpoint whose two coarse
 *          samples differ) moves onto it;
 *   Step 2 (vertex repulsion, distance c): a vertex left in place that lies
 *          within c of a polyline segment moves along the segment's normal,
 *          on its own side, to distance exactly c;
 *   Step 3 (edge elimination, distance b): a polyline vertex that no lattice
 *          vertex snapped to and that lies within b of a side of a base
 *          triangle is inserted on that side, and each triangle of the side
 *          is replaced by the two triangles fanned around it.
 * The result is the preprocessed grid: lattice vertex (k, i) at index
 * k * grid_cols + i (after Steps 1 and 2), then the inserted polyline
 * vertices (by owner lattice vertex, then owned side E0, E1, E2), and the
 * triangles by base triangle slot (row k, then i, the slot with apex on row k
 * first; a fanned slot gives its two triangles in the order
 * (a0, m, a2), (m, a1, a2) for the split side a0 -> a1).  Every triangle has
 * positive signed area.  Distances are square roots of sums of squares in
 * FP64, thresholds compared strictly (closer than a, b, c).
 *
 * Thresholds must satisfy 0 <= b < a/2, 0 <= c < a/sqrt2, 0 <= a < h/2
 * (Sec. 3.3.4), or all be zero (the plain lattice); otherwise
 * SBMT_E_INVALID_ARG.  The paper's setting is
 * (a, b, c) = (0.26, 0.125, 0.183) * h / sqrt(0.45).  With admissible
 * thresholds every decision is local (one polyline vertex within a of a
 * lattice vertex, one segment within c of a vertex left in place, one side
 * within b of a polyline vertex and at most one split side per triangle);
 * an input that breaks one of these returns SBMT_E_PROTOCOL.
 * ------------------------------------------------------------------------- */

/* Host only.  Workspace bytes of sbmt_preprocess for this image and bounds on
 * its vertex and triangle counts: grid_rows * grid_cols plus
 * 2 (coarse_h + 2)(coarse_w + 2) (every sample edge of the padded coarse
 * raster), and 4 * grid_rows * grid_cols.  Any pointer may be NULL. */
sbmt_status sbmt_pre_query(const sbmt_image* img, size_t* workspace_bytes, int64_t* vert_bound, int64_t* tri_bound);

/* Preprocessed grid of one image on `stream`; waits for it.
 *  workspace    device, >= the bytes of sbmt_pre_query (else SBMT_E_WORKSPACE)
 *  verts        device double [vert_cap][2]; vert_cap must be at least
 *               grid_rows * grid_cols (else SBMT_E_CAPACITY before any launch)
 *  on_polyline  device uint8 [vert_cap]: 1 for a vertex on a polyline vertex
 *               (snapped or inserted), else 0
 *  tris         device int32 [tri_cap][3] (may be NULL with tri_cap = 0)
 *  counts       host int64 [6]: n_vertices, n_triangles, n_snapped,
 *               n_repelled, n_inserted, status
 * Rows beyond a capacity are not written and the call returns
 * SBMT_E_CAPACITY with the counts filled in (size the outputs from them and
 * call again); SBMT_E_PROTOCOL as above; SBMT_E_INDEX_OVERFLOW if a vertex
 * index does not fit int32. */
sbmt_status sbmt_preprocess(sbmt_handle h, const sbmt_image* img, double a, double b, double c, void* workspace,
                            size_t ws_bytes, double* verts, uint8_t* on_polyline, int64_t vert_cap, int32_t* tris,
                            int64_t tri_cap, int64_t* counts, void* stream);

/* The mesh of Alg. 3 (Sec. 3.5): the preprocessed grid above retriangulated
 * against the polyline.  Every grid triangle is cut by the polyline pieces
 * inside it (a corner on a polyline vertex is that vertex; a segment along a
 * grid edge cuts nothing), its faces are traced, and each foreground face is
 * triangulated by the template rule of Sec. 3.3 (fanned from the chain
 * vertex inside the triangle; the quadrilateral between two chords split by
 * the diagonal joining their exits; else fanned from the face's earliest
 * chain point); an uncut grid triangle is kept whole when it lies in the
 * foreground.  With admissible thresholds every triangle meets the angle and
 * area bounds of Sec. 3.3.4 (App. D).
 *
 * sbmt_pre_mesh_query (host only): workspace bytes, and a bound on the grid
 * vertices (grid_rows * grid_cols + 2 (coarse_h + 2)(coarse_w + 2)); the grid
 * phase keeps them in the workspace.
 *
 * sbmt_preprocess_mesh (waits for `stream`):
 *  workspace  device, >= the query's bytes (else SBMT_E_WORKSPACE)
 *  verts      device double [vert_cap][2]: the grid vertices some output
 *             triangle uses, in grid order (lattice vertex k * grid_cols + i,
 *             then the inserted polyline vertices), then the new vertices
 *             (crossings of grid edges, polyline vertices inside grid
 *             triangles) by owner lattice vertex.  Every row is used by a
 *             triangle.  May be NULL with vert_cap = 0 (a sizing call).
 *  tris       device int32 [tri_cap][3], positive signed area; codes device
 *             uint8 [tri_cap]: 0 = grid triangle kept whole, 1 = piece of a
 *             cut one.  May be NULL with tri_cap = 0.
 *  counts     host int64 [8]: n_vertices (all rows of verts written),
 *             n_triangles, n_snapped, n_repelled, n_inserted, status,
 *             n_grid_vertices (grid vertices kept), n_cut (grid triangles
 *             the polyline cuts)
 * Rows beyond a capacity are not written; SBMT_E_CAPACITY then comes with the
 * counts filled in (size the outputs from them and call again).  Errors as
 * for sbmt_preprocess, and SBMT_E_INDEX_OVERFLOW before any launch when the
 * query's grid vertex bound exceeds 2^31 - 1. */
sbmt_status sbmt_pre_mesh_query(const sbmt_image* img, size_t* workspace_bytes, int64_t* grid_vert_bound);
sbmt_status sbmt_preprocess_mesh(sbmt_handle h, const sbmt_image* img, double a, double b, double c,
                                 void* workspace, size_t ws_bytes, double* verts, int64_t vert_cap, int32_t* tris,
                                 uint8_t* codes, int64_t tri_cap, int64_t* counts, void* stream);

/* Number of canonical classes and the key code of class id c (1-based). */
int32_t sbmt_num_classes(void);
int32_t sbmt_class_code(int32_t class_id);

const char* sbmt_status_string(sbmt_status s);

#ifdef __cplusplus
}
#endif

#endif /* SBMT_H_ */
