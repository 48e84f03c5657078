// Mesh consumers on gfx950: sampling a scalar field at the mesh vertices and
// the mesh-quality statistics.
//
// Both are streaming passes over the mesh, bound by HBM bandwidth: one thread
// per vertex or triangle in a grid-stride loop; the three vertex gathers of a
// triangle hit L2 because triangles reference nearby vertex ids (vertices
// and triangles are numbered row by row).
//
// Quality: one pass computes every per-triangle quantity, reduces counts,
// extremes and the area moments per workgroup (fixed-order trees, so the
// floating-point results are identical from run to run) and writes a 64-bit
// order-preserving key of each aspect ratio.  The two nearest-rank
// percentiles are then found exactly by a most-significant-digit radix
// select over those keys: five digits of 12 or 13 bits, each an LDS histogram
// per workgroup (wave-aggregated atomics: most keys of a mesh share the digit
// of 2/sqrt3) merged into a global histogram, and a one-workgroup pick of the
// digit that holds each rank.  The top digit is histogrammed by the quality
// pass as it writes the keys, so the keys are read four times.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/sbmt.h"
#include "../../include/sbmt_post.h"

namespace sbmt_post {

constexpr int kThreads = 256;
constexpr int kBins = SBMT_ANGLE_BINS;
constexpr int kMaxDigit = 13;                 // bits per select pass
constexpr int kPasses = 5;                    // 12 + 4 x 13 = 64 bits
constexpr int kShift[kPasses] = {52, 39, 26, 13, 0};
constexpr int kDigit[kPasses] = {12, 13, 13, 13, 13};
constexpr int kTopDigit = 12;                 // pass 0, histogrammed by the quality pass itself
constexpr int kQualityBlocksMax = 2048;
constexpr int kSelectBlocks = 512;

// ---------------------------------------------------------------------------
// Field sampling.
// ---------------------------------------------------------------------------

// Bilinear value at (x, y) of the pixel-centred field, clamped to the centres'
// rectangle (no access outside it for any input, NaN included).
__device__ __forceinline__ double sample_at(const float* __restrict__ f, int W, int H, int64_t ld, double x,
                                            double y) {
  const double xc = fmin(fmax(x, 0.0), (double)(W - 1));
  const double yc = fmin(fmax(y, 0.0), (double)(H - 1));
  const int c0 = (int)xc, r0 = (int)yc;
  const int c1 = min(c0 + 1, W - 1), r1 = min(r0 + 1, H - 1);
  const double a = xc - (double)c0, b = yc - (double)r0;
  const float* row0 = f + (int64_t)r0 * ld;
  const float* row1 = f + (int64_t)r1 * ld;
  const double f00 = row0[c0], f01 = row0[c1], f10 = row1[c0], f11 = row1[c1];
  return (1.0 - a) * (1.0 - b) * f00 + a * (1.0 - b) * f01 + (1.0 - a) * b * f10 + a * b * f11;
}

__global__ void __launch_bounds__(kThreads) k_sample_vertices(const float* __restrict__ f, int W, int H, int64_t ld,
                                                              const double2* __restrict__ v, int64_t nv,
                                                              double* __restrict__ out) {
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nv; i += step) {
    const double2 p = v[i];
    out[i] = sample_at(f, W, H, ld, p.x, p.y);
  }
}

__global__ void __launch_bounds__(kThreads) k_sample_triangles(const double* __restrict__ vv, int64_t nv,
                                                               const int32_t* __restrict__ tris, int64_t nt,
                                                               double* __restrict__ out) {
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < nt; t += step) {
    const int32_t a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    const bool ok = a >= 0 && b >= 0 && c >= 0 && a < nv && b < nv && c < nv;
    out[t] = ok ? (vv[a] + vv[b] + vv[c]) / 3.0 : __longlong_as_double(0x7ff8000000000000ll);
  }
}

// ---------------------------------------------------------------------------
// Quality.
// ---------------------------------------------------------------------------
struct Thresholds {
  double sliver;     // sin^2(5 deg)
  double bin[kBins]; // bin[j] = sin^2(2j deg), j >= 1
};

// One workgroup's partial results.
struct Part {
  long long n, invalid, nonpos, sliver, equi;
  long long qidx;
  unsigned long long armax;
  double amin, amax, mean, m2, qmin;
};

struct SelState {
  unsigned long long prefix[2];
  long long rank[2];
  long long n;
  int same;  // both targets still share their prefix: one histogram serves both
};

// Monotone map of doubles to unsigned integers (NaN with the sign bit clear
// sorts above +inf).
__device__ __forceinline__ unsigned long long order_key(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double key_value(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)b);
}

// Adds 1 to h[bin] for every active lane: the lanes that share the first
// active lane's bin add once (a mesh's keys mostly share one digit).
__device__ __forceinline__ void hist_add(unsigned int* h, unsigned int bin) {
  const unsigned int b0 = __builtin_amdgcn_readfirstlane(bin);
  const unsigned long long same = __ballot(bin == b0);
  if (bin == b0) {
    if ((int)(threadIdx.x & 63) == __builtin_ctzll(same)) atomicAdd(&h[b0], (unsigned int)__popcll(same));
  } else {
    atomicAdd(&h[bin], 1u);
  }
}

// Chan et al.'s pairwise update of (count, mean, sum of squared deviations).
__device__ __forceinline__ void moments_merge(long long& n1, double& m1, double& M1, long long n2, double m2,
                                              double M2) {
  if (n2 == 0) return;
  if (n1 == 0) {
    n1 = n2;
    m1 = m2;
    M1 = M2;
    return;
  }
  const long long n = n1 + n2;
  const double d = m2 - m1;
  m1 = m1 + d * ((double)n2 / (double)n);
  M1 = M1 + M2 + d * d * ((double)n1 * (double)n2 / (double)n);
  n1 = n;
}

__device__ __forceinline__ void part_merge(Part& a, const Part& b) {
  a.invalid += b.invalid;
  a.nonpos += b.nonpos;
  a.sliver += b.sliver;
  a.equi += b.equi;
  if (b.n) {
    a.amin = fmin(a.amin, b.amin);
    a.amax = fmax(a.amax, b.amax);
    if (b.qmin < a.qmin || (b.qmin == a.qmin && b.qidx < a.qidx)) {
      a.qmin = b.qmin;
      a.qidx = b.qidx;
    }
    a.armax = a.armax > b.armax ? a.armax : b.armax;
  }
  moments_merge(a.n, a.mean, a.m2, b.n, b.mean, b.m2);
}

__device__ __forceinline__ Part part_empty() {
  Part p;
  p.n = p.invalid = p.nonpos = p.sliver = p.equi = 0;
  p.qidx = -1;
  p.armax = 0;
  p.amin = INFINITY;
  p.amax = -INFINITY;
  p.mean = p.m2 = 0.0;
  p.qmin = INFINITY;
  return p;
}

// Fixed-order tree over the workgroup's parts in LDS; the result is in ps[0].
__device__ __forceinline__ void part_tree(Part* ps) {
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part_merge(ps[threadIdx.x], ps[threadIdx.x + w]);
    __syncthreads();
  }
}

__global__ void k_quality_init(sbmt_quality* __restrict__ out, unsigned long long* __restrict__ ghist,
                               SelState* __restrict__ st) {
  for (int i = threadIdx.x; i < kBins; i += blockDim.x) out->angle_hist[i] = 0;
  for (int i = threadIdx.x; i < 2 << kMaxDigit; i += blockDim.x) ghist[i] = 0;
  if (threadIdx.x == 0) {
    st->prefix[0] = st->prefix[1] = 0;
    st->rank[0] = st->rank[1] = 0;
    st->n = 0;
    st->same = 1;
  }
}

__global__ void __launch_bounds__(kThreads) k_quality(const double2* __restrict__ v, int64_t nv,
                                                      const int32_t* __restrict__ tris, int64_t nt, Thresholds th,
                                                      unsigned long long* __restrict__ keys, Part* __restrict__ parts,
                                                      unsigned long long* __restrict__ ghist,
                                                      sbmt_quality* __restrict__ out) {
  // the top-digit histogram is flushed before the reduction reuses its LDS
  __shared__ union {
    unsigned int top_hist[1 << kTopDigit];  // first radix-select digit of the keys
    Part ps[kThreads];
  } lds;
  __shared__ unsigned int hist[kBins];
  unsigned int* top_hist = lds.top_hist;
  Part* ps = lds.ps;
  if (threadIdx.x < kBins) hist[threadIdx.x] = 0;
  for (int i = threadIdx.x; i < 1 << kTopDigit; i += kThreads) top_hist[i] = 0;
  __syncthreads();
  Part p = part_empty();
  unsigned int top = 0;  // bin kBins-1, the common one, counted in a register
  double shift = 0.0, s1 = 0.0, s2 = 0.0;
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < nt; t += step) {
    const int32_t ia = tris[3 * t], ib = tris[3 * t + 1], ic = tris[3 * t + 2];
    if (ia < 0 || ib < 0 || ic < 0 || ia >= nv || ib >= nv || ic >= nv) {
      ++p.invalid;
      keys[t] = ~0ull;
      hist_add(top_hist, (1u << kTopDigit) - 1u);
      continue;
    }
    const double2 p0 = v[ia], p1 = v[ib], p2 = v[ic];
    const double ax = p1.x - p0.x, ay = p1.y - p0.y;  // edge 0: vertex 0 -> 1
    const double bx = p2.x - p1.x, by = p2.y - p1.y;  // edge 1: vertex 1 -> 2
    const double cx = p0.x - p2.x, cy = p0.y - p2.y;  // edge 2: vertex 2 -> 0
    const double l0 = ax * ax + ay * ay, l1 = bx * bx + by * by, l2 = cx * cx + cy * cy;
    const double cross = ax * (p2.y - p0.y) - ay * (p2.x - p0.x);
    const double area = 0.5 * cross;
    const double lmax = fmax(l0, fmax(l1, l2)), lmin = fmin(l0, fmin(l1, l2));
    const unsigned long long key = order_key(cross == 0.0 ? INFINITY : lmax / fabs(cross));
    keys[t] = key;
    hist_add(top_hist, (unsigned int)(key >> (64 - kTopDigit)));
    p.armax = p.armax > key ? p.armax : key;
    p.nonpos += cross <= 0.0;
    p.equi += lmax > 0.0 && lmax - lmin <= 1e-6 * lmax;
    // the smallest angle is opposite the shortest edge (first of equal ones)
    const int j = l1 < l0 ? (l2 < l1 ? 2 : 1) : (l2 < l0 ? 2 : 0);
    const double den = j == 0 ? l1 * l2 : (j == 1 ? l2 * l0 : l0 * l1);
    const double q = den > 0.0 ? (cross * cross) / den : 0.0;
    p.sliver += q < th.sliver;
    if (q >= th.bin[kBins - 1]) {
      ++top;
    } else {
      int bin = 0;
#pragma unroll
      for (int b = 1; b < kBins - 1; ++b) bin += q >= th.bin[b];
      atomicAdd(&hist[bin], 1u);
    }
    if (q < p.qmin) {
      p.qmin = q;
      p.qidx = t;
    }
    p.amin = fmin(p.amin, area);
    p.amax = fmax(p.amax, area);
    if (p.n == 0) shift = area;
    const double d = area - shift;
    s1 += d;
    s2 += d * d;
    ++p.n;
  }
  if (p.n) {
    p.mean = shift + s1 / (double)p.n;
    p.m2 = fmax(s2 - s1 * s1 / (double)p.n, 0.0);
  }
  if (top) atomicAdd(&hist[kBins - 1], top);
  __syncthreads();
  for (int i = threadIdx.x; i < 1 << kTopDigit; i += kThreads)
    if (top_hist[i]) atomicAdd(&ghist[i], (unsigned long long)top_hist[i]);
  if (threadIdx.x < kBins && hist[threadIdx.x])
    atomicAdd((unsigned long long*)&out->angle_hist[threadIdx.x], (unsigned long long)hist[threadIdx.x]);
  __syncthreads();
  ps[threadIdx.x] = p;
  __syncthreads();
  part_tree(ps);
  if (threadIdx.x == 0) parts[blockIdx.x] = ps[0];
}

__global__ void __launch_bounds__(kThreads) k_quality_final(const double2* __restrict__ v,
                                                            const int32_t* __restrict__ tris,
                                                            const Part* __restrict__ parts, int nparts,
                                                            sbmt_quality* __restrict__ out, SelState* __restrict__ st) {
  __shared__ Part ps[kThreads];
  Part p = part_empty();
  for (int i = threadIdx.x; i < nparts; i += kThreads) part_merge(p, parts[i]);
  ps[threadIdx.x] = p;
  __syncthreads();
  part_tree(ps);
  if (threadIdx.x != 0) return;
  p = ps[0];
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  out->n_triangles = p.n;
  out->n_invalid = p.invalid;
  out->n_nonpositive = p.nonpos;
  out->n_slivers = p.sliver;
  out->n_equilateral = p.equi;
  out->min_angle_tri = p.n ? p.qidx : -1;  // -1 also when every q was NaN
  out->min_area = p.n ? p.amin : nan;
  out->max_area = p.n ? p.amax : nan;
  out->mean_area = p.n ? p.mean : nan;
  out->var_area = p.n ? p.m2 / (double)p.n : nan;
  out->ar_max = p.n ? key_value(p.armax) : nan;
  out->ar_median = out->ar_p95 = nan;
  out->min_angle_deg = nan;
  if (p.n && p.qidx >= 0) {
    // the angle at the vertex opposite the shortest edge of the smallest-q
    // triangle, from the two edge vectors leaving that vertex
    const int64_t t = p.qidx;
    double x[3], y[3];
    for (int e = 0; e < 3; ++e) {
      const double2 pe = v[tris[3 * t + e]];
      x[e] = pe.x;
      y[e] = pe.y;
    }
    double l[3];
    for (int e = 0; e < 3; ++e) {
      const double dx = x[(e + 1) % 3] - x[e], dy = y[(e + 1) % 3] - y[e];
      l[e] = dx * dx + dy * dy;
    }
    const int j = l[1] < l[0] ? (l[2] < l[1] ? 2 : 1) : (l[2] < l[0] ? 2 : 0);
    const int m = (j + 2) % 3;
    const double ux = x[(m + 1) % 3] - x[m], uy = y[(m + 1) % 3] - y[m];
    const double wx = x[(m + 2) % 3] - x[m], wy = y[(m + 2) % 3] - y[m];
    out->min_angle_deg = atan2(fabs(ux * wy - uy * wx), ux * wx + uy * wy) * (180.0 / 3.14159265358979323846);
  }
  st->n = p.n;
  st->rank[0] = (p.n + 1) / 2 - 1;          // ceil(n / 2) - 1
  st->rank[1] = (95 * p.n + 99) / 100 - 1;  // ceil(0.95 n) - 1
}

// One radix-select pass below the top digit: histogram of the digit at
// `shift` over the keys whose higher digits equal each target's prefix.
// Each thread keeps kSelUnroll key loads in flight.
constexpr int kSelUnroll = 8;
__global__ void __launch_bounds__(kThreads) k_select_hist(const unsigned long long* __restrict__ keys, int64_t n,
                                                          const SelState* __restrict__ st, int shift, int digit,
                                                          unsigned long long* __restrict__ ghist) {
  __shared__ unsigned int h[2][1 << kMaxDigit];
  if (st->n == 0) return;  // uniform: nothing counted
  const int nb = 1 << digit;
  const int ntg = st->same ? 1 : 2;
  for (int i = threadIdx.x; i < ntg * nb; i += kThreads) h[i / nb][i % nb] = 0;
  __syncthreads();
  const int hi = shift + digit;  // < 64: the top digit is counted by k_quality
  const unsigned long long pre0 = st->prefix[0] >> hi, pre1 = st->prefix[1] >> hi;
  const unsigned int mask = (unsigned int)nb - 1u;
  const int64_t chunk = (int64_t)gridDim.x * kThreads * kSelUnroll;
  for (int64_t base = (int64_t)blockIdx.x * kThreads * kSelUnroll + threadIdx.x; base < n; base += chunk) {
    unsigned long long k[kSelUnroll];
#pragma unroll
    for (int u = 0; u < kSelUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kThreads;
      k[u] = i < n ? keys[i] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < kSelUnroll; ++u) {
      if (base + (int64_t)u * kThreads >= n) break;
      const unsigned long long kh = k[u] >> hi;
      const unsigned int bin = (unsigned int)(k[u] >> shift) & mask;
      if (kh == pre0) hist_add(h[0], bin);
      if (ntg == 2 && kh == pre1) hist_add(h[1], bin);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ntg * nb; i += kThreads) {
    const unsigned int c = h[i / nb][i % nb];
    if (c) atomicAdd(&ghist[(i / nb) * (1 << kMaxDigit) + i % nb], (unsigned long long)c);
  }
}

// Finds the digit that holds each target rank (every thread sums its run of
// bins held in registers, a scan over the threads locates the run, its thread
// locates the bin), extends the prefixes and clears the global histogram;
// after the last pass writes the two percentiles.
template <int D>
__global__ void __launch_bounds__(kThreads) k_select_pick(unsigned long long* __restrict__ ghist,
                                                          SelState* __restrict__ st, int shift, int last,
                                                          sbmt_quality* __restrict__ out) {
  constexpr int per = (1 << D) / kThreads;
  __shared__ unsigned long long part[kThreads];
  __shared__ unsigned long long pick_bin[2], pick_below[2];
  if (st->n == 0) return;
  const int same = st->same;
  if (threadIdx.x < 2) pick_bin[threadIdx.x] = pick_below[threadIdx.x] = 0;
  for (int tg = 0; tg < 2; ++tg) {
    const unsigned long long* hg = ghist + (same ? 0 : tg) * (1 << kMaxDigit);
    unsigned long long c[per], sum = 0;
#pragma unroll
    for (int j = 0; j < per; ++j) {
      c[j] = hg[threadIdx.x * per + j];
      sum += c[j];
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
      const unsigned long long add = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0ull;
      __syncthreads();
      part[threadIdx.x] += add;
      __syncthreads();
    }
    const unsigned long long incl = part[threadIdx.x], excl = incl - sum;
    const unsigned long long r = (unsigned long long)st->rank[tg];
    if (r >= excl && r < incl) {
      unsigned long long below = excl;
      int b = 0;
#pragma unroll
      for (int j = 0; j < per; ++j) {
        if (b == j && below + c[j] <= r) {
          below += c[j];
          b = j + 1;
        }
      }
      pick_bin[tg] = (unsigned long long)(threadIdx.x * per + b);
      pick_below[tg] = below;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < 2 << kMaxDigit; i += kThreads) ghist[i] = 0;
  if (threadIdx.x == 0) {
    for (int tg = 0; tg < 2; ++tg) {
      st->prefix[tg] |= pick_bin[tg] << shift;
      st->rank[tg] -= (long long)pick_below[tg];
    }
    st->same = st->prefix[0] == st->prefix[1];
    if (last) {
      out->ar_median = key_value(st->prefix[0]);
      out->ar_p95 = key_value(st->prefix[1]);
    }
  }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int quality_blocks(int64_t nt) {
  const int64_t b = (nt + (int64_t)kThreads * 16 - 1) / ((int64_t)kThreads * 16);
  return (int)(b < 1 ? 1 : (b > kQualityBlocksMax ? kQualityBlocksMax : b));
}

struct QualityLayout {
  size_t out, parts, ghist, state, keys, total;
};

static QualityLayout quality_layout(int64_t nt) {
  QualityLayout L;
  L.out = 0;
  L.parts = align256(sizeof(sbmt_quality));
  L.ghist = L.parts + align256(sizeof(Part) * (size_t)quality_blocks(nt));
  L.state = L.ghist + align256(sizeof(unsigned long long) * (2u << kMaxDigit));
  L.keys = L.state + align256(sizeof(SelState));
  L.total = L.keys + align256(sizeof(unsigned long long) * (size_t)(nt > 0 ? nt : 0));
  return L;
}

// Squared sine of d degrees, from the run-time sin (pi / 180 through a
// volatile so that the compiler does not fold it).
static double sin2_deg(int d) {
  volatile double rad = 3.14159265358979323846 / 180.0;
  const double s = sin(d * rad);
  return s * s;
}

static Thresholds thresholds() {
  Thresholds t;
  t.sliver = sin2_deg(5);
  t.bin[0] = 0.0;
  for (int j = 1; j < kBins; ++j) t.bin[j] = sin2_deg(2 * j);
  return t;
}

static int grid_for(int64_t n, int cap) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace sbmt_post

using namespace sbmt_post;

extern "C" {

sbmt_status sbmt_sample_field(sbmt_handle h, const sbmt_field* field, const double* verts, int64_t n_vertices,
                              const int32_t* tris, int64_t n_triangles, double* vert_values, double* tri_values,
                              void* stream) {
  if (!h || !field || n_vertices < 0 || n_triangles < 0) return SBMT_E_INVALID_ARG;
  if (n_vertices > 0 && (!verts || !vert_values || !field->data || field->width < 1 || field->height < 1 ||
                         field->row_stride < field->width))
    return SBMT_E_INVALID_ARG;
  if (tri_values && n_triangles > 0 && (!tris || !vert_values)) return SBMT_E_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (n_vertices > 0) {
    hipLaunchKernelGGL(k_sample_vertices, dim3(grid_for(n_vertices, 1 << 16)), dim3(kThreads), 0, s, field->data,
                       field->width, field->height, field->row_stride, (const double2*)verts, n_vertices,
                       vert_values);
    if (hipGetLastError() != hipSuccess) return SBMT_E_DEVICE;
  }
  if (tri_values && n_triangles > 0) {
    hipLaunchKernelGGL(k_sample_triangles, dim3(grid_for(n_triangles, 1 << 16)), dim3(kThreads), 0, s,
                       vert_values, n_vertices, tris, n_triangles, tri_values);
    if (hipGetLastError() != hipSuccess) return SBMT_E_DEVICE;
  }
  return SBMT_OK;
}

sbmt_status sbmt_quality_workspace(int64_t n_triangles, size_t* bytes) {
  if (!bytes || n_triangles < 0) return SBMT_E_INVALID_ARG;
  *bytes = quality_layout(n_triangles).total;
  return SBMT_OK;
}

sbmt_status sbmt_mesh_quality_async(sbmt_handle h, const double* verts, int64_t n_vertices, const int32_t* tris,
                                    int64_t n_triangles, void* workspace, size_t ws_bytes, sbmt_quality* out_dev,
                                    void* stream) {
  if (!h || !out_dev || n_vertices < 0 || n_triangles < 0 || n_vertices > 0x7fffffffLL) return SBMT_E_INVALID_ARG;
  if (n_triangles > 0 && (!tris || (n_vertices > 0 && !verts))) return SBMT_E_INVALID_ARG;
  const QualityLayout L = quality_layout(n_triangles);
  if (!workspace || ws_bytes < L.total) return SBMT_E_WORKSPACE;
  char* ws = (char*)workspace;
  Part* parts = (Part*)(ws + L.parts);
  unsigned long long* ghist = (unsigned long long*)(ws + L.ghist);
  SelState* st = (SelState*)(ws + L.state);
  unsigned long long* keys = (unsigned long long*)(ws + L.keys);
  hipStream_t s = (hipStream_t)stream;
  const int nq = quality_blocks(n_triangles);
  hipLaunchKernelGGL(k_quality_init, dim3(1), dim3(kThreads), 0, s, out_dev, ghist, st);
  hipLaunchKernelGGL(k_quality, dim3(nq), dim3(kThreads), 0, s, (const double2*)verts, n_vertices, tris,
                     n_triangles, thresholds(), keys, parts, ghist, out_dev);
  hipLaunchKernelGGL(k_quality_final, dim3(1), dim3(kThreads), 0, s, (const double2*)verts, tris, parts, nq,
                     out_dev, st);
  const int nsel = grid_for((n_triangles + kSelUnroll - 1) / kSelUnroll, kSelectBlocks);
  static_assert(kShift[0] + kDigit[0] == 64 && kDigit[0] == kTopDigit, "top digit");
  static_assert(kDigit[1] == 13 && kDigit[2] == 13 && kDigit[3] == 13 && kDigit[4] == 13, "digits");
  for (int pass = 0; pass < kPasses; ++pass) {
    if (pass > 0)
      hipLaunchKernelGGL(k_select_hist, dim3(nsel), dim3(kThreads), 0, s, keys, n_triangles, st, kShift[pass],
                         kDigit[pass], ghist);
    const int last = pass == kPasses - 1 ? 1 : 0;
    if (kDigit[pass] == 12)
      hipLaunchKernelGGL(k_select_pick<12>, dim3(1), dim3(kThreads), 0, s, ghist, st, kShift[pass], last, out_dev);
    else
      hipLaunchKernelGGL(k_select_pick<13>, dim3(1), dim3(kThreads), 0, s, ghist, st, kShift[pass], last, out_dev);
  }
  if (hipGetLastError() != hipSuccess) return SBMT_E_DEVICE;
  return SBMT_OK;
}

sbmt_status sbmt_mesh_quality(sbmt_handle h, const double* verts, int64_t n_vertices, const int32_t* tris,
                              int64_t n_triangles, void* workspace, size_t ws_bytes, sbmt_quality* out,
                              void* stream) {
  if (!out) return SBMT_E_INVALID_ARG;
  sbmt_quality* dev = (sbmt_quality*)workspace;  // the layout's first slot
  sbmt_status st = sbmt_mesh_quality_async(h, verts, n_vertices, tris, n_triangles, workspace, ws_bytes, dev, stream);
  if (st != SBMT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(out, dev, sizeof(sbmt_quality), hipMemcpyDeviceToHost, s) != hipSuccess) return SBMT_E_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return SBMT_E_DEVICE;
  return out->n_invalid ? SBMT_E_INVALID_ARG : SBMT_OK;
}

}  // extern "C"
