// Cotangent Laplacian assembly and explicit heat steps on gfx950 (linear
// finite elements on an SBMT mesh; the diffusion setting of App. H).
//
// Assembly, all passes one thread per triangle or per vertex:
//   1. degree count (integer atomics) and validity of each triangle;
//   2. exclusive scan of the degrees -> incident-triangle offsets;
//   3. incident-triangle lists (slots by atomics, then sorted per vertex, so
//      the order is ascending triangle index whatever the atomics did);
//   4. per vertex: number of distinct neighbours, boundary flag (an edge seen
//      in one triangle), lumped mass;
//   5. exclusive scan of the row lengths -> CSR offsets;
//   6. per vertex: the row (neighbours in order of first appearance, edge
//      weights accumulated in triangle order) and the Gershgorin bound.
// Every floating-point sum runs in a fixed order, so the operator is the
// same bit for bit on every run.  For the steps the rows are also laid out in
// slices of 64 (entry e of the 64 rows of a slice side by side), so that one
// thread per row still sums its row in row order while a wave's loads of
// entry e coalesce (HBM bound: the operator is read once per step, the field
// values mostly from L2 because neighbours have nearby ids).  A mesh whose
// padded slices would not fit the space reserved for them steps on the rows.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/sbmt.h"
#include "../../include/sbmt_post.h"

namespace sbmt_pde {

constexpr int kThreads = 256;
constexpr int kScanPer = 8;  // elements per thread in the scans
constexpr int kScanBlock = kThreads * kScanPer;

struct Info {
  unsigned long long min_mass_key, lambda_key;  // order keys (see order_key)
  unsigned long long n_boundary, n_invalid;
};

__device__ __forceinline__ unsigned long long order_key(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ bool tri_valid(int32_t a, int32_t b, int32_t c, int64_t nv) {
  return a >= 0 && b >= 0 && c >= 0 && a < nv && b < nv && c < nv && a != b && b != c && a != c;
}

// Half-cotangents c_k of triangle t and its cross product.
__device__ __forceinline__ double tri_weights(const double2* __restrict__ v, const int32_t* id, double c[3]) {
  double x[3], y[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const double2 p = v[id[e]];
    x[e] = p.x;
    y[e] = p.y;
  }
  const double cross = (x[1] - x[0]) * (y[2] - y[0]) - (y[1] - y[0]) * (x[2] - x[0]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double ux = x[(k + 1) % 3] - x[k], uy = y[(k + 1) % 3] - y[k];
    const double wx = x[(k + 2) % 3] - x[k], wy = y[(k + 2) % 3] - y[k];
    c[k] = 0.5 * ((ux * wx + uy * wy) / cross);
  }
  return cross;
}

// The two neighbours of vertex i in triangle t (next, previous) and, if
// requested, their edge weights.
__device__ __forceinline__ void tri_neighbours(const int32_t* __restrict__ tris, int64_t t, int64_t i, int32_t j[2],
                                               int* kpos) {
  const int32_t a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
  const int k = a == i ? 0 : (b == i ? 1 : 2);
  const int32_t id[3] = {a, b, c};
  j[0] = id[(k + 1) % 3];
  j[1] = id[(k + 2) % 3];
  *kpos = k;
}

// ---------------------------------------------------------------------------
// Exclusive scan of int32 counts into int64 offsets (n + 1 entries).
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long block_excl_scan(long long x, long long* sh, long long* total) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    const long long add = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  const long long incl = sh[threadIdx.x];
  *total = sh[kThreads - 1];
  __syncthreads();
  return incl - x;
}

__global__ void __launch_bounds__(kThreads) k_scan_sums(const int32_t* __restrict__ in, int64_t n,
                                                        long long* __restrict__ sums) {
  __shared__ long long sh[kThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  long long s = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j)
    if (base + j < n) s += in[base + j];
  long long tot;
  block_excl_scan(s, sh, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the block sums in place.
__global__ void __launch_bounds__(kThreads) k_scan_top(long long* __restrict__ sums, int64_t nb) {
  __shared__ long long sh[kThreads];
  const int64_t per = (nb + kThreads - 1) / kThreads;
  const int64_t lo = (int64_t)threadIdx.x * per, hi = lo + per < nb ? lo + per : nb;
  long long s = 0;
  for (int64_t i = lo; i < hi; ++i) s += sums[i];
  long long tot;
  long long run = block_excl_scan(s, sh, &tot);
  for (int64_t i = lo; i < hi; ++i) {
    const long long v = sums[i];
    sums[i] = run;
    run += v;
  }
}

__global__ void __launch_bounds__(kThreads) k_scan_apply(const int32_t* __restrict__ in, int64_t n,
                                                         const long long* __restrict__ sums,
                                                         int64_t* __restrict__ out) {
  __shared__ long long sh[kThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  long long s = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j)
    if (base + j < n) s += in[base + j];
  long long tot;
  long long run = block_excl_scan(s, sh, &tot) + sums[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    if (base + j < n) {
      out[base + j] = run;
      run += in[base + j];
    }
  }
  if (base <= n - 1 && n - 1 < base + kScanPer) out[n] = run;  // the thread holding the last element
}

// ---------------------------------------------------------------------------
// Assembly passes.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_zero(int32_t* __restrict__ a, int64_t n, int32_t* __restrict__ b,
                                                   Info* __restrict__ info) {
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += step) {
    a[i] = 0;
    b[i] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    info->min_mass_key = ~0ull;
    info->lambda_key = 0ull;
    info->n_boundary = 0;
    info->n_invalid = 0;
  }
}

__global__ void __launch_bounds__(kThreads) k_degrees(const int32_t* __restrict__ tris, int64_t nt, int64_t nv,
                                                      int32_t* __restrict__ deg, Info* __restrict__ info) {
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < nt; t += step) {
    const int32_t a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    if (!tri_valid(a, b, c, nv)) {
      atomicAdd(&info->n_invalid, 1ull);
      continue;
    }
    atomicAdd(&deg[a], 1);
    atomicAdd(&deg[b], 1);
    atomicAdd(&deg[c], 1);
  }
}

__global__ void __launch_bounds__(kThreads) k_incident(const int32_t* __restrict__ tris, int64_t nt, int64_t nv,
                                                       const int64_t* __restrict__ inc_off,
                                                       int32_t* __restrict__ cursor, int32_t* __restrict__ inc) {
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < nt; t += step) {
    const int32_t id[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    if (!tri_valid(id[0], id[1], id[2], nv)) continue;
#pragma unroll
    for (int e = 0; e < 3; ++e) inc[inc_off[id[e]] + atomicAdd(&cursor[id[e]], 1)] = (int32_t)t;
  }
}

// Sorts each vertex's incident triangles; counts its distinct neighbours,
// flags the boundary and sums the lumped mass.
__global__ void __launch_bounds__(kThreads) k_rows_count(const double2* __restrict__ v, const int32_t* __restrict__ tris,
                                                         int64_t nv, const int64_t* __restrict__ inc_off,
                                                         int32_t* __restrict__ inc, int32_t* __restrict__ row_len,
                                                         double* __restrict__ mass, uint8_t* __restrict__ bnd,
                                                         Info* __restrict__ info) {
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nv; i += step) {
    const int64_t lo = inc_off[i], hi = inc_off[i + 1];
    // insertion sort (degrees are small)
    for (int64_t p = lo + 1; p < hi; ++p) {
      const int32_t x = inc[p];
      int64_t q = p - 1;
      while (q >= lo && inc[q] > x) {
        inc[q + 1] = inc[q];
        --q;
      }
      inc[q + 1] = x;
    }
    const int64_t ncand = 2 * (hi - lo);
    int32_t uniq = 0;
    bool boundary = false;
    double m = 0.0;
    for (int64_t p = 0; p < ncand; ++p) {
      int32_t jp[2];
      int kp;
      tri_neighbours(tris, inc[lo + p / 2], i, jp, &kp);
      const int32_t j = jp[p & 1];
      int mult = 0;
      bool first = true;
      for (int64_t q = 0; q < ncand; ++q) {
        int32_t jq[2];
        int kq;
        tri_neighbours(tris, inc[lo + q / 2], i, jq, &kq);
        if (jq[q & 1] == j) {
          ++mult;
          if (q < p) first = false;
        }
      }
      uniq += first;
      boundary |= mult == 1;
    }
    for (int64_t p = lo; p < hi; ++p) {
      const int64_t t = inc[p];
      const int32_t id[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
      double c[3];
      const double cross = tri_weights(v, id, c);
      m += (0.5 * cross) / 3.0;
    }
    row_len[i] = uniq;
    mass[i] = m;
    bnd[i] = boundary ? 1 : 0;
    if (boundary) atomicAdd(&info->n_boundary, 1ull);
    if (!isnan(m)) atomicMin(&info->min_mass_key, order_key(m));
  }
}

// Fills each row: neighbours in order of first appearance, weights summed in
// triangle order; the Gershgorin bound of the row.
__global__ void __launch_bounds__(kThreads) k_rows_fill(const double2* __restrict__ v, const int32_t* __restrict__ tris,
                                                        int64_t nv, const int64_t* __restrict__ inc_off,
                                                        const int32_t* __restrict__ inc,
                                                        const int64_t* __restrict__ row_off,
                                                        const double* __restrict__ mass, int32_t* __restrict__ col,
                                                        double* __restrict__ val, Info* __restrict__ info) {
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nv; i += step) {
    const int64_t lo = inc_off[i], hi = inc_off[i + 1], r0 = row_off[i];
    int64_t n = 0;
    for (int64_t p = lo; p < hi; ++p) {
      const int64_t t = inc[p];
      const int32_t id[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
      double c[3];
      tri_weights(v, id, c);
      const int k = id[0] == i ? 0 : (id[1] == i ? 1 : 2);
      const int32_t js[2] = {id[(k + 1) % 3], id[(k + 2) % 3]};
      const double cs[2] = {c[(k + 2) % 3], c[(k + 1) % 3]};
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        int64_t e = 0;
        while (e < n && col[r0 + e] != js[q]) ++e;
        if (e == n) {
          col[r0 + n] = js[q];
          val[r0 + n] = cs[q];
          ++n;
        } else {
          val[r0 + e] += cs[q];
        }
      }
    }
    double diag = 0.0, offs = 0.0;
    for (int64_t e = 0; e < n; ++e) {
      diag += val[r0 + e];
      offs += fabs(val[r0 + e]);
    }
    const double m = mass[i];
    if (m > 0.0) {
      const double lam = (diag + offs) / m;
      if (!isnan(lam)) atomicMax(&info->lambda_key, order_key(lam));
    }
  }
}

// ---------------------------------------------------------------------------
// Operator application and heat steps.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_apply(const int64_t* __restrict__ row_off,
                                                    const int32_t* __restrict__ col, const double* __restrict__ val,
                                                    int64_t nv, const double* __restrict__ u, double* __restrict__ y) {
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nv; i += step) {
    const double ui = u[i];
    double s = 0.0;
    for (int64_t e = row_off[i], end = row_off[i + 1]; e < end; ++e) s += val[e] * (ui - u[col[e]]);
    y[i] = s;
  }
}

// Slices of 64 rows: width = the longest row of the slice (times 64 entries).
__global__ void __launch_bounds__(kThreads) k_slice_width(const int32_t* __restrict__ row_len, int64_t nv,
                                                          int64_t nsl, int32_t* __restrict__ w64) {
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < nsl; q += step) {
    int m = 0;
    for (int j = 0; j < 64; ++j) {
      const int64_t i = q * 64 + j;
      if (i < nv) m = max(m, row_len[i]);
    }
    w64[q] = 64 * m;
  }
}

// Copies the rows into their slices (entry e of row i at
// slice_off[i / 64] + 64 e + i mod 64) when they fit the reserved space.
__global__ void __launch_bounds__(kThreads) k_slice_fill(const int64_t* __restrict__ row_off,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val,
                                                         const int32_t* __restrict__ row_len, int64_t nv,
                                                         const int64_t* __restrict__ slice_off, int64_t nsl,
                                                         int64_t cap, int32_t* __restrict__ col_s,
                                                         double* __restrict__ val_s) {
  if (slice_off[nsl] > cap) return;  // uniform: the steps use the rows
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nv; i += step) {
    const int64_t base = slice_off[i >> 6] + (i & 63), r0 = row_off[i];
    for (int e = 0; e < row_len[i]; ++e) {
      col_s[base + 64 * (int64_t)e] = col[r0 + e];
      val_s[base + 64 * (int64_t)e] = val[r0 + e];
    }
  }
}

struct Op {  // what a step reads
  const int64_t* row_off;
  const int32_t* col;
  const double* val;
  const int32_t* row_len;
  const int64_t* slice_off;
  const int32_t* col_s;
  const double* val_s;
  const double* mass;
  const uint8_t* bnd;
  int64_t nsl, cap;
};

__global__ void __launch_bounds__(kThreads) k_heat_step(Op op, int64_t nv, double dt_alpha,
                                                        const double* __restrict__ u, double* __restrict__ out) {
  const bool sliced = op.slice_off[op.nsl] <= op.cap;  // uniform
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nv; i += step) {
    if (op.bnd[i]) {
      out[i] = 0.0;
      continue;
    }
    const double ui = u[i];
    double s = 0.0;
    if (sliced) {
      const int64_t base = op.slice_off[i >> 6] + (i & 63);
      const int len = op.row_len[i];
      for (int e = 0; e < len; ++e) {
        const int64_t x = base + 64 * (int64_t)e;
        s += op.val_s[x] * (ui - u[op.col_s[x]]);
      }
    } else {
      for (int64_t e = op.row_off[i], end = op.row_off[i + 1]; e < end; ++e) s += op.val[e] * (ui - u[op.col[e]]);
    }
    out[i] = ui - (dt_alpha * s) / op.mass[i];
  }
}

__global__ void __launch_bounds__(kThreads) k_heat_init(const double2* __restrict__ v, const uint8_t* __restrict__ bnd,
                                                        int64_t nv, double x0, double y0, double sigma, double amp,
                                                        double* __restrict__ u) {
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nv; i += step) {
    const double2 p = v[i];
    const double dx = p.x - x0, dy = p.y - y0;
    u[i] = bnd[i] ? 0.0 : amp * exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma));
  }
}

__global__ void k_store_zero(int64_t* __restrict__ p) { *p = 0; }

__global__ void __launch_bounds__(kThreads) k_copy(const double* __restrict__ a, int64_t n, double* __restrict__ b) {
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += step) b[i] = a[i];
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t info, deg, cursor, inc_off, inc, row_len, row_off, col, val, mass, bnd, sums, slice_off, col_s, val_s,
      total;
  int64_t nsl, cap;
};

static int64_t scan_blocks(int64_t n) { return (n + kScanBlock - 1) / kScanBlock; }

static Layout layout(int64_t nv, int64_t nt) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.info = take(sizeof(Info));
  L.deg = take(4 * (size_t)nv);
  L.cursor = take(4 * (size_t)nv);
  L.inc_off = take(8 * (size_t)(nv + 1));
  L.inc = take(4 * 3 * (size_t)nt);
  L.row_len = take(4 * (size_t)nv);
  L.row_off = take(8 * (size_t)(nv + 1));
  L.col = take(4 * 6 * (size_t)nt);  // at most two distinct neighbours per incident triangle
  L.val = take(8 * 6 * (size_t)nt);
  L.mass = take(8 * (size_t)nv);
  L.bnd = take((size_t)nv);
  L.sums = take(8 * (size_t)(scan_blocks(nv) + 1));
  L.nsl = (nv + 63) / 64;
  L.cap = 6 * nt;  // as many entries as the rows may hold: padding beyond twice the entries falls back
  L.slice_off = take(8 * (size_t)(L.nsl + 1));
  L.col_s = take(4 * (size_t)L.cap);
  L.val_s = take(8 * (size_t)L.cap);
  L.total = o;
  return L;
}

static int grid_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

static sbmt_status scan(const int32_t* in, int64_t n, long long* sums, int64_t* out, hipStream_t s) {
  const int64_t nb = scan_blocks(n);
  if (nb == 0) {
    hipLaunchKernelGGL(k_store_zero, dim3(1), dim3(1), 0, s, out);
    return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
  }
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, s, sums, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, (const long long*)sums, out);
  return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
}

static double host_key_value(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  double d;
  memcpy(&d, &b, sizeof d);
  return d;
}

static bool sizes_ok(int64_t nv, int64_t nt) { return nv >= 0 && nt >= 0 && nv <= 0x7fffffffLL && nt <= 0x7fffffffLL; }

}  // namespace sbmt_pde

using namespace sbmt_pde;

extern "C" {

sbmt_status sbmt_laplacian_workspace(int64_t n_vertices, int64_t n_triangles, size_t* bytes) {
  if (!bytes || !sizes_ok(n_vertices, n_triangles)) return SBMT_E_INVALID_ARG;
  *bytes = layout(n_vertices, n_triangles).total;
  return SBMT_OK;
}

sbmt_status sbmt_laplacian_csr(void* workspace, size_t ws_bytes, int64_t n_vertices, int64_t n_triangles,
                               sbmt_csr* out) {
  if (!out || !sizes_ok(n_vertices, n_triangles)) return SBMT_E_INVALID_ARG;
  const Layout L = layout(n_vertices, n_triangles);
  if (!workspace || ws_bytes < L.total) return SBMT_E_WORKSPACE;
  char* w = (char*)workspace;
  out->row_off = (const int64_t*)(w + L.row_off);
  out->col = (const int32_t*)(w + L.col);
  out->val = (const double*)(w + L.val);
  out->mass = (const double*)(w + L.mass);
  out->boundary = (const uint8_t*)(w + L.bnd);
  return SBMT_OK;
}

sbmt_status sbmt_laplacian_assemble(sbmt_handle h, const double* verts, int64_t n_vertices, const int32_t* tris,
                                    int64_t n_triangles, void* workspace, size_t ws_bytes,
                                    sbmt_laplacian_info* info, void* stream) {
  if (!h || !info || !sizes_ok(n_vertices, n_triangles)) return SBMT_E_INVALID_ARG;
  if ((n_vertices > 0 && !verts) || (n_triangles > 0 && !tris)) return SBMT_E_INVALID_ARG;
  const Layout L = layout(n_vertices, n_triangles);
  if (!workspace || ws_bytes < L.total) return SBMT_E_WORKSPACE;
  char* w = (char*)workspace;
  hipStream_t s = (hipStream_t)stream;
  Info* dinfo = (Info*)(w + L.info);
  int32_t* deg = (int32_t*)(w + L.deg);
  int32_t* cursor = (int32_t*)(w + L.cursor);
  int64_t* inc_off = (int64_t*)(w + L.inc_off);
  int32_t* inc = (int32_t*)(w + L.inc);
  int32_t* row_len = (int32_t*)(w + L.row_len);
  int64_t* row_off = (int64_t*)(w + L.row_off);
  int32_t* col = (int32_t*)(w + L.col);
  double* val = (double*)(w + L.val);
  double* mass = (double*)(w + L.mass);
  uint8_t* bnd = (uint8_t*)(w + L.bnd);
  long long* sums = (long long*)(w + L.sums);
  const double2* v = (const double2*)verts;
  sbmt_status st;
  hipLaunchKernelGGL(k_zero, dim3(grid_for(n_vertices)), dim3(kThreads), 0, s, deg, n_vertices, cursor, dinfo);
  if (n_triangles > 0)
    hipLaunchKernelGGL(k_degrees, dim3(grid_for(n_triangles)), dim3(kThreads), 0, s, tris, n_triangles, n_vertices,
                       deg, dinfo);
  if ((st = scan(deg, n_vertices, sums, inc_off, s)) != SBMT_OK) return st;
  if (n_triangles > 0)
    hipLaunchKernelGGL(k_incident, dim3(grid_for(n_triangles)), dim3(kThreads), 0, s, tris, n_triangles,
                       n_vertices, (const int64_t*)inc_off, cursor, inc);
  if (n_vertices > 0)
    hipLaunchKernelGGL(k_rows_count, dim3(grid_for(n_vertices)), dim3(kThreads), 0, s, v, tris, n_vertices,
                       (const int64_t*)inc_off, inc, row_len, mass, bnd, dinfo);
  if ((st = scan(row_len, n_vertices, sums, row_off, s)) != SBMT_OK) return st;
  if (n_vertices > 0)
    hipLaunchKernelGGL(k_rows_fill, dim3(grid_for(n_vertices)), dim3(kThreads), 0, s, v, tris, n_vertices,
                       (const int64_t*)inc_off, (const int32_t*)inc, (const int64_t*)row_off, (const double*)mass,
                       col, val, dinfo);
  // the rows in slices of 64 for the steps (the slice widths reuse the
  // degree array, which is free by now)
  int64_t* slice_off = (int64_t*)(w + L.slice_off);
  hipLaunchKernelGGL(k_slice_width, dim3(grid_for(L.nsl)), dim3(kThreads), 0, s, (const int32_t*)row_len, n_vertices,
                     L.nsl, deg);
  if ((st = scan(deg, L.nsl, sums, slice_off, s)) != SBMT_OK) return st;
  if (n_vertices > 0)
    hipLaunchKernelGGL(k_slice_fill, dim3(grid_for(n_vertices)), dim3(kThreads), 0, s, (const int64_t*)row_off,
                       (const int32_t*)col, (const double*)val, (const int32_t*)row_len, n_vertices,
                       (const int64_t*)slice_off, L.nsl, L.cap, (int32_t*)(w + L.col_s), (double*)(w + L.val_s));
  if (hipGetLastError() != hipSuccess) return SBMT_E_DEVICE;
  Info hi;
  int64_t nnz = 0;
  if (hipMemcpyAsync(&hi, dinfo, sizeof(Info), hipMemcpyDeviceToHost, s) != hipSuccess) return SBMT_E_DEVICE;
  if (hipMemcpyAsync(&nnz, row_off + n_vertices, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess)
    return SBMT_E_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return SBMT_E_DEVICE;
  info->n_vertices = n_vertices;
  info->nnz = nnz;
  info->n_boundary = hi.n_boundary;
  info->n_invalid = hi.n_invalid;
  // no finite mass seen (no vertex, or NaN masses only): +inf like an empty minimum
  info->min_mass = hi.min_mass_key == ~0ull ? INFINITY : host_key_value(hi.min_mass_key);
  info->lambda_bound = hi.lambda_key == 0ull ? 0.0 : host_key_value(hi.lambda_key);
  return SBMT_OK;
}

sbmt_status sbmt_laplacian_apply(sbmt_handle h, const void* workspace, size_t ws_bytes, int64_t n_vertices,
                                 int64_t n_triangles, const double* u, double* y, void* stream) {
  if (!h || !sizes_ok(n_vertices, n_triangles) || (n_vertices > 0 && (!u || !y))) return SBMT_E_INVALID_ARG;
  const Layout L = layout(n_vertices, n_triangles);
  if (!workspace || ws_bytes < L.total) return SBMT_E_WORKSPACE;
  if (n_vertices == 0) return SBMT_OK;
  const char* w = (const char*)workspace;
  hipLaunchKernelGGL(k_apply, dim3(grid_for(n_vertices)), dim3(kThreads), 0, (hipStream_t)stream,
                     (const int64_t*)(w + L.row_off), (const int32_t*)(w + L.col), (const double*)(w + L.val),
                     n_vertices, u, y);
  return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
}

sbmt_status sbmt_heat_init(sbmt_handle h, const void* workspace, size_t ws_bytes, const double* verts,
                           int64_t n_vertices, int64_t n_triangles, double x0, double y0, double sigma, double amp,
                           double* u, void* stream) {
  if (!h || !sizes_ok(n_vertices, n_triangles) || (n_vertices > 0 && (!u || !verts)) || !(sigma > 0.0))
    return SBMT_E_INVALID_ARG;
  const Layout L = layout(n_vertices, n_triangles);
  if (!workspace || ws_bytes < L.total) return SBMT_E_WORKSPACE;
  if (n_vertices == 0) return SBMT_OK;
  const char* w = (const char*)workspace;
  hipLaunchKernelGGL(k_heat_init, dim3(grid_for(n_vertices)), dim3(kThreads), 0, (hipStream_t)stream,
                     (const double2*)verts, (const uint8_t*)(w + L.bnd), n_vertices, x0, y0, sigma, amp, u);
  return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
}

sbmt_status sbmt_heat_steps(sbmt_handle h, const void* workspace, size_t ws_bytes, int64_t n_vertices,
                            int64_t n_triangles, double alpha, double dt, int32_t steps, double* u, double* u_tmp,
                            void* stream) {
  if (!h || !sizes_ok(n_vertices, n_triangles) || steps < 0 || (n_vertices > 0 && (!u || !u_tmp)) || u == u_tmp)
    return SBMT_E_INVALID_ARG;
  const Layout L = layout(n_vertices, n_triangles);
  if (!workspace || ws_bytes < L.total) return SBMT_E_WORKSPACE;
  if (n_vertices == 0 || steps == 0) return SBMT_OK;
  const char* w = (const char*)workspace;
  hipStream_t s = (hipStream_t)stream;
  const double dt_alpha = dt * alpha;
  Op op;
  op.row_off = (const int64_t*)(w + L.row_off);
  op.col = (const int32_t*)(w + L.col);
  op.val = (const double*)(w + L.val);
  op.row_len = (const int32_t*)(w + L.row_len);
  op.slice_off = (const int64_t*)(w + L.slice_off);
  op.col_s = (const int32_t*)(w + L.col_s);
  op.val_s = (const double*)(w + L.val_s);
  op.mass = (const double*)(w + L.mass);
  op.bnd = (const uint8_t*)(w + L.bnd);
  op.nsl = L.nsl;
  op.cap = L.cap;
  double* a = u;
  double* b = u_tmp;
  for (int32_t k = 0; k < steps; ++k) {
    hipLaunchKernelGGL(k_heat_step, dim3(grid_for(n_vertices)), dim3(kThreads), 0, s, op, n_vertices, dt_alpha,
                       (const double*)a, b);
    double* t = a;
    a = b;
    b = t;
  }
  if (a != u) hipLaunchKernelGGL(k_copy, dim3(grid_for(n_vertices)), dim3(kThreads), 0, s, (const double*)a, n_vertices, u);
  return hipGetLastError() == hipSuccess ? SBMT_OK : SBMT_E_DEVICE;
}

}  // extern "C"
