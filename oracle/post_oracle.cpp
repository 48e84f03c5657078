// SBMT CPU oracle, mesh consumers -- TEST INFRASTRUCTURE ONLY.
//
// Plain CPU definitions of the two stages that consume a mesh:
//   * scalar-field sampling at the mesh vertices (the interpolation stage of
//     the pipeline, one value per vertex, linear over each triangle; Sec. 3.3
//     structured filling, interpolation cost in App. C), with the per-triangle
//     mean of the linear interpolant;
//   * the mesh-quality statistics of the evaluation section (minimum angle,
//     minimum area, area variance, sliver count below 5 degrees, equilateral
//     count by an edge-length test: Tables 1 and 3; aspect ratio
//     AR = longest edge / shortest altitude with median, 95th percentile and
//     maximum: Table 4; histogram of per-triangle minimum angles in 2-degree
//     bins: the minimum-angle distribution figures).
//
// Only the tests, the smoke check and the CPU-baseline leg of the benchmark
// load this code; it shares nothing with the HIP path.  Everything is the
// textbook formula evaluated triangle by triangle in double precision (sums
// in long double), sorted with std::sort for the percentiles.
//
// Readings where the paper is silent:
//   * the field is bilinear between pixel centres, clamped at the outermost
//     centres (the paper names linear or barycentric schemes only);
//   * the edge-length test calls a triangle equilateral when its longest and
//     shortest squared edge lengths differ by at most 1e-6 of the longest (a
//     triangle whose three vertices coincide is not);
//   * a triangle of zero area has AR = +inf (its shortest altitude is 0);
//   * percentiles are nearest-rank (element ceil(p n) - 1 of the sorted list);
//   * the area variance is the population variance.
// The sliver and histogram decisions take the precision of the GPU kernels:
// the squared sine of the smallest angle against squared sines of the bin
// edges, not a rounded angle (an exact 30-degree angle sits on a bin edge).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace {

struct QualityOut {
  int64_t n_triangles, n_invalid, n_nonpositive, n_slivers, n_equilateral, min_angle_tri;
  double min_angle_deg, min_area, max_area, mean_area, var_area, ar_median, ar_p95, ar_max;
  int64_t angle_hist[30];
};

// Squared sine of d degrees.  pi / 180 goes through a volatile so that the
// value comes from the run-time sin, like the GPU library's host code.
double sin2_deg(int d) {
  volatile double rad = 3.14159265358979323846 / 180.0;
  const double s = std::sin(d * rad);
  return s * s;
}

// Bilinear value of the field at (x, y): the weights of the four pixel
// centres around the clamped point.
double bilinear(const float* f, int W, int H, int64_t ld, double x, double y) {
  double xc = x < 0.0 ? 0.0 : x, yc = y < 0.0 ? 0.0 : y;
  if (xc > W - 1) xc = W - 1;
  if (yc > H - 1) yc = H - 1;
  const int c0 = (int)std::floor(xc), r0 = (int)std::floor(yc);
  const int c1 = c0 + 1 < W ? c0 + 1 : W - 1, r1 = r0 + 1 < H ? r0 + 1 : H - 1;
  const double a = xc - c0, b = yc - r0;
  const double f00 = f[r0 * ld + c0], f01 = f[r0 * ld + c1];
  const double f10 = f[r1 * ld + c0], f11 = f[r1 * ld + c1];
  return (1.0 - a) * (1.0 - b) * f00 + a * (1.0 - b) * f01 + (1.0 - a) * b * f10 + a * b * f11;
}

}  // namespace

extern "C" {

void oracle_sample_field(const float* f, int W, int H, int64_t ld, const double* verts, int64_t nv,
                         const int32_t* tris, int64_t nt, double* vv, double* tv) {
  for (int64_t i = 0; i < nv; ++i) vv[i] = bilinear(f, W, H, ld, verts[2 * i], verts[2 * i + 1]);
  if (!tv) return;
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv) {
      tv[t] = NAN;
      continue;
    }
    tv[t] = (vv[a] + vv[b] + vv[c]) / 3.0;
  }
}

void oracle_mesh_quality(const double* verts, int64_t nv, const int32_t* tris, int64_t nt, QualityOut* out) {
  QualityOut q = {};
  q.min_angle_tri = -1;
  const double S5 = sin2_deg(5);
  double T[30];
  for (int j = 1; j < 30; ++j) T[j] = sin2_deg(2 * j);
  std::vector<double> ar, area;
  ar.reserve(nt);
  area.reserve(nt);
  double best_angle = INFINITY;
  q.min_area = INFINITY;
  q.max_area = -INFINITY;
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t id[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    if (id[0] < 0 || id[1] < 0 || id[2] < 0 || id[0] >= nv || id[1] >= nv || id[2] >= nv) {
      ++q.n_invalid;
      continue;
    }
    double x[3], y[3];
    for (int v = 0; v < 3; ++v) {
      x[v] = verts[2 * id[v]];
      y[v] = verts[2 * id[v] + 1];
    }
    // edge e runs from vertex e to vertex e+1
    double l[3];
    for (int e = 0; e < 3; ++e) {
      const double dx = x[(e + 1) % 3] - x[e], dy = y[(e + 1) % 3] - y[e];
      l[e] = dx * dx + dy * dy;
    }
    const double cross = (x[1] - x[0]) * (y[2] - y[0]) - (y[1] - y[0]) * (x[2] - x[0]);
    const double A = 0.5 * cross;
    const double lmax = std::max(l[0], std::max(l[1], l[2]));
    const double lmin = std::min(l[0], std::min(l[1], l[2]));
    ++q.n_triangles;
    if (cross <= 0.0) ++q.n_nonpositive;
    area.push_back(A);
    q.min_area = std::min(q.min_area, A);
    q.max_area = std::max(q.max_area, A);
    // a triangle of zero area has a zero altitude: AR = +inf
    ar.push_back(cross == 0.0 ? INFINITY : lmax / std::fabs(cross));
    if (lmax > 0.0 && lmax - lmin <= 1e-6 * lmax) ++q.n_equilateral;
    // smallest angle: opposite the shortest edge j (first of equal lengths);
    // the vertex opposite edge j is vertex j+2
    int j = 0;
    if (l[1] < l[j]) j = 1;
    if (l[2] < l[j]) j = 2;
    const double lu = l[(j + 1) % 3], lv = l[(j + 2) % 3];
    const double s2 = lu * lv > 0.0 ? (cross * cross) / (lu * lv) : 0.0;
    if (s2 < S5) ++q.n_slivers;
    int bin = 0;
    for (int b = 1; b < 30; ++b)
      if (s2 >= T[b]) bin = b;
    ++q.angle_hist[bin];
    // the angle itself: all three, by atan2, smallest kept
    for (int v = 0; v < 3; ++v) {
      const double ux = x[(v + 1) % 3] - x[v], uy = y[(v + 1) % 3] - y[v];
      const double wx = x[(v + 2) % 3] - x[v], wy = y[(v + 2) % 3] - y[v];
      const double ang = std::atan2(std::fabs(ux * wy - uy * wx), ux * wx + uy * wy) * (180.0 / 3.14159265358979323846);
      if (ang < best_angle) {
        best_angle = ang;
        q.min_angle_tri = t;
      }
    }
  }
  if (q.n_triangles == 0) {
    q.min_angle_deg = q.min_area = q.max_area = q.mean_area = q.var_area = NAN;
    q.ar_median = q.ar_p95 = q.ar_max = NAN;
  } else {
    q.min_angle_deg = best_angle;
    long double s = 0.0L;
    for (double a : area) s += a;
    const long double mean = s / (long double)area.size();
    long double m2 = 0.0L;
    for (double a : area) m2 += ((long double)a - mean) * ((long double)a - mean);
    q.mean_area = (double)mean;
    q.var_area = (double)(m2 / (long double)area.size());
    std::sort(ar.begin(), ar.end());
    const int64_t n = (int64_t)ar.size();
    q.ar_median = ar[(n + 1) / 2 - 1];        // ceil(n / 2) - 1
    q.ar_p95 = ar[(95 * n + 99) / 100 - 1];   // ceil(0.95 n) - 1
    q.ar_max = ar[n - 1];
  }
  *out = q;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Cotangent Laplacian and explicit heat steps (the parabolic experiment of
// App. H: du/dt = alpha * Laplacian(u), u = 0 on the boundary, Gaussian
// initial pulse), with linear finite elements on the mesh.
//
// Per triangle T = (v0, v1, v2): cross_T = (x1-x0)(y2-y0) - (y1-y0)(x2-x0);
// at vertex k, u = p(k+1) - p(k), w = p(k+2) - p(k), dot_k = u.w and
// c_k = 0.5 * (dot_k / cross_T) = cot(angle k) / 2, the weight of the edge
// opposite vertex k.  Row i of the stiffness matrix lists the neighbours j of
// i in order of first appearance over the triangles containing i (ascending
// triangle index; in each, the next vertex then the previous one), each with
// w_ij = the sum of its edge weights in that order.  (K u)_i = sum_j w_ij
// (u_i - u_j) in row order.  Lumped mass m_i = sum over the same triangles of
// (0.5 * cross_T) / 3.  A vertex is on the boundary when one of its edges
// belongs to a single triangle.  One explicit Euler step:
// u_i <- 0 on the boundary, else u_i - ((dt * alpha) * (K u)_i) / m_i.
// Triangles with an index out of range or repeated are skipped; the others
// must be positively oriented (a zero cross product gives infinite weights).
// The Laplacian is a reading of the App. H setting, which names linear
// finite elements without stating the time discretisation; the explicit
// step is the first consumer, not a claim about the paper's solver.
// ---------------------------------------------------------------------------
namespace {

struct Lap {
  std::vector<int64_t> row_off;  // n_v + 1
  std::vector<int32_t> col;
  std::vector<double> val, mass;
  std::vector<uint8_t> bnd;
  int64_t n_invalid = 0;
  double lambda_bound = 0.0;
};

Lap build_lap(const double* verts, int64_t nv, const int32_t* tris, int64_t nt) {
  Lap L;
  std::vector<std::vector<int64_t>> inc(nv);
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv || a == b || b == c || a == c) {
      ++L.n_invalid;  // an index out of range or repeated: skipped
      continue;
    }
    inc[a].push_back(t);
    inc[b].push_back(t);
    inc[c].push_back(t);
  }
  L.row_off.assign(nv + 1, 0);
  L.mass.assign(nv, 0.0);
  L.bnd.assign(nv, 0);
  for (int64_t i = 0; i < nv; ++i) {
    std::vector<int32_t> nb;
    std::vector<double> w;
    std::vector<int> mult;
    double m = 0.0;
    for (int64_t t : inc[i]) {
      const int32_t id[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
      double x[3], y[3];
      for (int v = 0; v < 3; ++v) {
        x[v] = verts[2 * id[v]];
        y[v] = verts[2 * id[v] + 1];
      }
      const double cross = (x[1] - x[0]) * (y[2] - y[0]) - (y[1] - y[0]) * (x[2] - x[0]);
      double c[3];
      for (int k = 0; k < 3; ++k) {
        const double ux = x[(k + 1) % 3] - x[k], uy = y[(k + 1) % 3] - y[k];
        const double wx = x[(k + 2) % 3] - x[k], wy = y[(k + 2) % 3] - y[k];
        c[k] = 0.5 * ((ux * wx + uy * wy) / cross);
      }
      m += (0.5 * cross) / 3.0;
      int k = 0;
      while (id[k] != i) ++k;
      const int32_t js[2] = {id[(k + 1) % 3], id[(k + 2) % 3]};
      const double cs[2] = {c[(k + 2) % 3], c[(k + 1) % 3]};
      for (int q = 0; q < 2; ++q) {
        size_t p = 0;
        while (p < nb.size() && nb[p] != js[q]) ++p;
        if (p == nb.size()) {
          nb.push_back(js[q]);
          w.push_back(cs[q]);
          mult.push_back(1);
        } else {
          w[p] += cs[q];
          ++mult[p];
        }
      }
    }
    for (int c : mult) L.bnd[i] |= c == 1;
    L.mass[i] = m;
    double diag = 0.0, offs = 0.0;
    for (double v : w) {
      diag += v;
      offs += std::fabs(v);
    }
    if (m > 0.0) L.lambda_bound = std::max(L.lambda_bound, (diag + offs) / m);
    L.col.insert(L.col.end(), nb.begin(), nb.end());
    L.val.insert(L.val.end(), w.begin(), w.end());
    L.row_off[i + 1] = (int64_t)L.col.size();
  }
  return L;
}

void apply_lap(const Lap& L, int64_t nv, const double* u, double* y) {
  for (int64_t i = 0; i < nv; ++i) {
    double s = 0.0;
    for (int64_t e = L.row_off[i]; e < L.row_off[i + 1]; ++e) s += L.val[e] * (u[i] - u[L.col[e]]);
    y[i] = s;
  }
}

}  // namespace

extern "C" {

struct OracleLapInfo {
  int64_t nnz, n_boundary, n_invalid;
  double min_mass, lambda_bound;
};

// Assembles and copies out: row_off [nv+1], col/val [nnz] (nnz from a first
// call with col == nullptr), mass [nv], bnd [nv].
void oracle_laplacian(const double* verts, int64_t nv, const int32_t* tris, int64_t nt, int64_t* row_off,
                      int32_t* col, double* val, double* mass, uint8_t* bnd, OracleLapInfo* info) {
  const Lap L = build_lap(verts, nv, tris, nt);
  info->nnz = (int64_t)L.col.size();
  info->n_invalid = L.n_invalid;
  info->n_boundary = 0;
  info->min_mass = INFINITY;
  for (int64_t i = 0; i < nv; ++i) {
    info->n_boundary += L.bnd[i];
    info->min_mass = std::min(info->min_mass, L.mass[i]);
  }
  info->lambda_bound = L.lambda_bound;
  if (!col) return;
  std::copy(L.row_off.begin(), L.row_off.end(), row_off);
  std::copy(L.col.begin(), L.col.end(), col);
  std::copy(L.val.begin(), L.val.end(), val);
  std::copy(L.mass.begin(), L.mass.end(), mass);
  std::copy(L.bnd.begin(), L.bnd.end(), bnd);
}

// y = K u
void oracle_laplacian_apply(const double* verts, int64_t nv, const int32_t* tris, int64_t nt, const double* u,
                            double* y) {
  const Lap L = build_lap(verts, nv, tris, nt);
  apply_lap(L, nv, u, y);
}

// Gaussian pulse amp * exp(-((x-x0)^2 + (y-y0)^2) / (2 sigma^2)), 0 on the boundary.
void oracle_heat_init(const double* verts, int64_t nv, const int32_t* tris, int64_t nt, double x0, double y0,
                      double sigma, double amp, double* u) {
  const Lap L = build_lap(verts, nv, tris, nt);
  for (int64_t i = 0; i < nv; ++i) {
    const double dx = verts[2 * i] - x0, dy = verts[2 * i + 1] - y0;
    u[i] = L.bnd[i] ? 0.0 : amp * std::exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma));
  }
}

// `steps` explicit Euler steps in place.
void oracle_heat_steps(const double* verts, int64_t nv, const int32_t* tris, int64_t nt, double alpha, double dt,
                       int32_t steps, double* u) {
  const Lap L = build_lap(verts, nv, tris, nt);
  std::vector<double> ku(nv);
  for (int32_t s = 0; s < steps; ++s) {
    apply_lap(L, nv, u, ku.data());
    for (int64_t i = 0; i < nv; ++i) u[i] = L.bnd[i] ? 0.0 : u[i] - ((dt * alpha) * ku[i]) / L.mass[i];
  }
}

}  // extern "C"
