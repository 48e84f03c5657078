/*
 * sbmt_post.h -- C ABI of the stages that consume an SBMT mesh on the GPU:
 * sampling a scalar field of the bitmap at the mesh vertices, the mesh
 * quality statistics the paper evaluates its meshes with, and the cotangent
 * Laplacian with explicit heat steps (the first PDE consumer).
 *
 * Both take the outputs of sbmt.h (vertices FP64 (x, y) pairs, triangles
 * int32 index triples) but accept any triangle mesh in that layout.  Every
 * array pointer is a device pointer on the current HIP device, allocated and
 * owned by the caller; the library allocates nothing.  Errors are returned as
 * sbmt_status codes (sbmt.h); arguments are checked before any launch.
 */
#ifndef SBMT_POST_H_
#define SBMT_POST_H_
#include <stddef.h>
#include <stdint.h>

#include "sbmt.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------------------
 * Scalar field sampling (the interpolation stage: a field of the bitmap is
 * carried onto the mesh, one value per vertex, linear over each triangle;
 * Sec. 3.3 structured filling and the interpolation cost of App. C).
 *
 * field: device FP32 image, `height` rows of `row_stride` elements, pixel
 * (r, c) centred at (x = c, y = r) like the bitmap.  The value at (x, y) is the
 * bilinear interpolant of the four surrounding pixel centres, with x clamped
 * to [0, width-1] and y to [0, height-1] (constant extension beyond the
 * outermost centres), computed in FP64.
 * ------------------------------------------------------------------------- */
typedef struct {
  const float* data;
  int32_t width;
  int32_t height;
  int64_t row_stride; /* elements, >= width */
} sbmt_field;

/* vert_values[i] = field at vertex i (n_vertices FP64 values).
 * tri_values (may be NULL): tri_values[t] = (v_a + v_b + v_c) / 3 for triangle
 * t = (a, b, c), the mean of the linear interpolant over the triangle; a
 * triangle with an index outside [0, n_vertices) gets NaN.
 * Needs width, height >= 1 when n_vertices > 0.  Asynchronous on `stream`. */
sbmt_status sbmt_sample_field(sbmt_handle h, const sbmt_field* field, const double* verts, int64_t n_vertices,
                              const int32_t* tris, int64_t n_triangles, double* vert_values, double* tri_values,
                              void* stream);

/* ---------------------------------------------------------------------------
 * Mesh quality (the statistics of the evaluation section: minimum angle,
 * minimum area, area variance, slivers, equilateral count (Tables 1, 3, 4),
 * aspect ratio AR = longest edge / shortest altitude with its median, 95th
 * percentile and maximum (Table 4), and the histogram of per-triangle
 * minimum angles in 2-degree bins).
 *
 * Per triangle (p0, p1, p2), in FP64 without contraction:
 *   squared edge lengths l0 = |p1-p0|^2, l1 = |p2-p1|^2, l2 = |p0-p2|^2;
 *   cross = (x1-x0)(y2-y0) - (y1-y0)(x2-x0) (twice the signed area);
 *   area = cross / 2;  AR = max(l) / |cross| (+inf when cross = 0);
 *   the smallest angle lies opposite the shortest edge j (ties: lowest j);
 *   with lu, lv the other two squared lengths, q = cross^2 / (lu lv) is the
 *   squared sine of that angle (0 when lu lv = 0).
 * Decisions taken on q (so that they do not depend on a trigonometric
 * routine): sliver iff q < sin^2(5 deg); histogram bin = number of
 * j in 1..29 with q >= sin^2(2j deg) (bin 29 = [58, 60] deg, the largest a
 * minimum angle can be); equilateral iff max(l) > 0 and
 * max(l) - min(l) <= 1e-6 max(l).  The reported minimum angle is
 * atan2(|u x w|, u . w) in degrees, u and w the edge vectors leaving the
 * vertex opposite edge j of the smallest-q triangle (lowest index among equal
 * q).  Vertices must be finite.  Percentiles are
 * nearest-rank over all counted triangles: element ceil(p n) - 1 of the sorted
 * AR values.  Mean and (population) variance of the areas are accumulated in
 * a fixed order (run to run identical).
 * ------------------------------------------------------------------------- */
#define SBMT_ANGLE_BINS 30
typedef struct {
  int64_t n_triangles;   /* triangles counted (indices in range) */
  int64_t n_invalid;     /* triangles with an index outside [0, n_vertices): skipped */
  int64_t n_nonpositive; /* cross <= 0 (not positively oriented) */
  int64_t n_slivers;     /* minimum angle below 5 degrees */
  int64_t n_equilateral;
  int64_t min_angle_tri; /* index of the triangle that gives min_angle_deg, -1 if none */
  double min_angle_deg;
  double min_area;
  double max_area;
  double mean_area;
  double var_area;
  double ar_median;
  double ar_p95;
  double ar_max;
  int64_t angle_hist[SBMT_ANGLE_BINS];
} sbmt_quality;

/* Workspace bytes for a mesh of n_triangles triangles (host only). */
sbmt_status sbmt_quality_workspace(int64_t n_triangles, size_t* bytes);

/* Asynchronous: the statistics land in the device struct *out_dev when the
 * stream reaches this point (FP fields are NaN and min_angle_tri is -1 when
 * no triangle is counted). */
sbmt_status sbmt_mesh_quality_async(sbmt_handle h, const double* verts, int64_t n_vertices, const int32_t* tris,
                                    int64_t n_triangles, void* workspace, size_t ws_bytes, sbmt_quality* out_dev,
                                    void* stream);

/* Same, copied to the host struct *out (waits for the stream).  Returns
 * SBMT_E_INVALID_ARG if a triangle had an index out of range (the statistics
 * of the others are still reported). */
sbmt_status sbmt_mesh_quality(sbmt_handle h, const double* verts, int64_t n_vertices, const int32_t* tris,
                              int64_t n_triangles, void* workspace, size_t ws_bytes, sbmt_quality* out,
                              void* stream);

/* ---------------------------------------------------------------------------
 * Cotangent Laplacian and explicit heat steps: linear finite elements on the
 * mesh for du/dt = alpha * Laplacian(u) with u = 0 on the boundary and a
 * Gaussian initial pulse (the diffusion setting of App. H).
 *
 * Per triangle T = (v0, v1, v2): cross_T = (x1-x0)(y2-y0) - (y1-y0)(x2-x0);
 * at vertex k, u = p(k+1) - p(k), w = p(k+2) - p(k) and
 * c_k = 0.5 * ((u . w) / cross_T) = cot(angle k) / 2 weighs the edge opposite
 * vertex k.  Row i of the stiffness matrix K lists the neighbours j of vertex
 * i in order of first appearance over the triangles containing i (ascending
 * triangle index; in each, the next vertex then the previous one), with
 * w_ij = the sum of that edge's weights in the same order; K is applied as
 * (K u)_i = sum_j w_ij (u_i - u_j) in row order.  Lumped mass
 * m_i = sum over the same triangles of (0.5 * cross_T) / 3.  A vertex is on
 * the boundary when one of its edges belongs to a single triangle.  Every
 * sum has a fixed order, so results are identical from run to run.
 * Triangles with an index out of range or repeated are skipped; the others
 * must be positively oriented.
 *
 * The workspace (sized by sbmt_laplacian_workspace for the mesh) holds the
 * assembled operator after sbmt_laplacian_assemble; the other calls take
 * that workspace and must see the same vertex count.
 * ------------------------------------------------------------------------- */
typedef struct {
  int64_t n_vertices;
  int64_t nnz;          /* stored off-diagonal entries (each undirected edge twice) */
  int64_t n_boundary;   /* vertices held at 0 */
  int64_t n_invalid;    /* skipped triangles */
  double min_mass;      /* smallest lumped mass (0 for a vertex in no triangle) */
  double lambda_bound;  /* Gershgorin bound on the eigenvalues of M^-1 K:
                           max_i (sum_j w_ij + sum_j |w_ij|) / m_i over m_i > 0;
                           explicit steps are stable for alpha dt <= 2 / lambda_bound */
} sbmt_laplacian_info;

/* Device pointers into an assembled workspace (valid while it lives):
 * row_off [n_v + 1] int64, col [nnz] int32, val [nnz] FP64, mass [n_v] FP64,
 * boundary [n_v] uint8 (1 = on the boundary). */
typedef struct {
  const int64_t* row_off;
  const int32_t* col;
  const double* val;
  const double* mass;
  const uint8_t* boundary;
} sbmt_csr;

/* Host only. */
sbmt_status sbmt_laplacian_workspace(int64_t n_vertices, int64_t n_triangles, size_t* bytes);

/* Assembles K, the masses and the boundary flags into the workspace and
 * returns the summary in *info (waits for the stream). */
sbmt_status sbmt_laplacian_assemble(sbmt_handle h, const double* verts, int64_t n_vertices, const int32_t* tris,
                                    int64_t n_triangles, void* workspace, size_t ws_bytes,
                                    sbmt_laplacian_info* info, void* stream);

/* Host only: the operator's arrays inside an assembled workspace. */
sbmt_status sbmt_laplacian_csr(void* workspace, size_t ws_bytes, int64_t n_vertices, int64_t n_triangles,
                               sbmt_csr* out);

/* y = K u (every row, boundary included).  Asynchronous. */
sbmt_status sbmt_laplacian_apply(sbmt_handle h, const void* workspace, size_t ws_bytes, int64_t n_vertices,
                                 int64_t n_triangles, const double* u, double* y, void* stream);

/* u_i = amp * exp(-((x_i - x0)^2 + (y_i - y0)^2) / (2 sigma^2)), 0 on the
 * boundary.  Asynchronous. */
sbmt_status sbmt_heat_init(sbmt_handle h, const void* workspace, size_t ws_bytes, const double* verts,
                           int64_t n_vertices, int64_t n_triangles, double x0, double y0, double sigma, double amp,
                           double* u, void* stream);

/* `steps` explicit Euler steps in place on u:
 * u_i <- 0 on the boundary, else u_i - ((dt * alpha) * (K u)_i) / m_i.
 * u_tmp [n_v] is scratch.  Asynchronous. */
sbmt_status sbmt_heat_steps(sbmt_handle h, const void* workspace, size_t ws_bytes, int64_t n_vertices,
                            int64_t n_triangles, double alpha, double dt, int32_t steps, double* u, double* u_tmp,
                            void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SBMT_POST_H_ */
