// sbmt_pre.h -- geometric preprocessing of Alg. 3 (Sec. 3.5) and the
// retriangulation of the preprocessed grid: device code and workspace layout.
// Included by sbmt.hip inside namespace sbmt, after the meshing kernels whose
// helpers it uses (raster layout, row segments, scans).
#pragma once

// ---------------------------------------------------------------------------
// Geometric preprocessing of Alg. 3 (Sec. 3.5, thresholds of Sec. 3.3.4):
// Step 1 snaps a lattice vertex to the polyline vertex within distance a,
// Step 2 moves a vertex within c of a segment along that segment's normal to
// distance exactly c, Step 3 splits every mesh edge within b of a polyline
// vertex that no lattice vertex snapped to, at that vertex (the edge's one or
// two triangles become a fan around it).  The result is the preprocessed
// grid: lattice vertices (moved), inserted polyline vertices, and the base
// triangles with their split edges fanned.
//
// Polyline vertices are the marching-squares midpoints whose two coarse
// samples differ; distances are square roots of sums of squares in double
// precision, evaluated exactly as written (no contraction).  Admissible
// thresholds (b < a/2, c < a/sqrt2, a < h/2) keep every decision local: at
// most one polyline vertex within a of a lattice vertex, at most one segment
// within c of an unsnapped one, at most one edge within b of a polyline vertex
// and at most one polyline vertex within b of an edge, at most one split edge
// per triangle; the kernels flag a protocol error otherwise.
// ---------------------------------------------------------------------------
struct PreArgs {
  double a, b, c;
  double* verts;         // [NK NI + inserted][2]: lattice vertex k NI + i first
  uint8_t* on_polyline;  // per vertex: sits on a polyline vertex
  int32_t* tris;         // [triangles][3]
  int64_t vcap, tcap;
  uint8_t* mid;          // per midpoint: 1 if a lattice vertex snapped to it
  uint8_t* flags;        // per lattice vertex: bits 0-2 owned side E0-E2 split, 3 moved, 4 claimed, 5 snapped, 6 touched (mesh)
  int32_t* split;        // [NK NI][3]: midpoint splitting side E0, E1, E2 (written where split)
  int64_t* ins_base;     // [NK NI]: first inserted vertex of the owner (written where it has one)
  int64_t* counts;       // [8 + 512]: [2] error, [3] touched owners (mesh); from kPreTally 256 counters of snapped, then of repelled vertices
  int32_t* snap_mid;     // [NK NI]: the polyline vertex a lattice vertex snapped to (written where snapped)
  // retriangulation of the grid (sbmt_preprocess_mesh)
  uint32_t* rcount;      // [NK NI]: per-owner counts (pre_rc_*)
  uint32_t* rtri;        // [NK NI]: per grid triangle of the owner (4): output triangles (6 bits each), inner-vertex bits 24..27, cut bits 28..31
  int64_t* rbase;        // [NK NI]: first new vertex of the owner (written where it has one)
  const int64_t* gsizes; // the grid phase's sizes record (grid vertices first)
  int32_t* otris;        // [otcap][3]
  uint8_t* ocodes;       // [otcap]
  int64_t otcap;
  // compaction of the mesh's vertices: the grid vertices some output triangle
  // uses (marked in the count pass) keep their order and come first
  double* overts;        // [ovcap][2]: the mesh's vertices
  int64_t ovcap;
  uint8_t* used;         // [usedcap]: grid vertex used by an output triangle
  int64_t usedcap;
  int32_t* vmap;         // [usedcap]: its id in the mesh
  int32_t* tlist;        // [NK NI]: the touched owners, in owner order
  int64_t* rtbase;       // [NK NI]: a touched owner's first output triangle
  int64_t* vbsum;        // per block of kPreVScan grid vertices: used count, then base
  int64_t* nused;        // [1]: grid vertices in the mesh
  // a cut grid triangle's output kept by the count pass for the triangle pass
  int32_t* cbase;        // [NK NI]: cut grid triangles of the touched owners before list position t
  int64_t* cblk;         // per block of kPreVScan list positions: cut count, then base
  uint32_t* cstore;      // [ccap][1 + 3 kPreKeep]: number of triangles kept (or kPreNotKept), point refs
  int64_t ccap;
};
constexpr int kPreVScan = 16384;  // grid vertices (list positions) per block of the compaction (cut) scan
constexpr int kPreKeep = 4;       // output triangles a cut grid triangle keeps for the triangle pass
constexpr uint32_t kPreNotKept = 0xffffffffu;
constexpr uint8_t kPreMoved = 8;
constexpr int kPreTally = 8;
constexpr int kPreCounts = kPreTally + 512;

// Midpoint ids: horizontal midpoint between samples (R, C) and (R, C+1) is
// 2 ((R + 1)(CW + 2) + C + 1), the vertical one between (R, C) and (R+1, C)
// one more; R in -1 .. CH, C in -1 .. CW.
__device__ __forceinline__ int64_t mid_id(const Geo& g, int R, int C, int vert) {
  return 2 * ((int64_t)(R + 1) * (g.CW + 2) + (C + 1)) + vert;
}
__device__ __forceinline__ int sample_at(const Img& d, const Geo& g, int R, int C) {
  if (R < 0 || R >= g.CH || C < 0 || C >= g.CW) return 0;
  const int rr = R + kRing, cc = C + kRingC;
  return (int)((d.bits[(int64_t)rr * g.wpr + (cc >> 5)] >> (cc & 31)) & 1u);
}
// Sample (R, C) sits at pixel (s C + (s-1)/2, s R + (s-1)/2); the offset:
__device__ __forceinline__ double sample_off(const Geo& g) { return 0.5 * (g.s - 1); }
// Midpoint (R, C, vert) in pixels, and whether it is a polyline vertex.
__device__ __forceinline__ bool mid_point(const Img& d, const Geo& g, int R, int C, int vert, double& x, double& y) {
  const double half = 0.5 * g.s;
  x = (double)g.s * C + sample_off(g) + (vert ? 0.0 : half);
  y = (double)g.s * R + sample_off(g) + (vert ? half : 0.0);
  if (R < -1 || R > g.CH || C < -1 || C > g.CW) return false;
  return sample_at(d, g, R, C) != sample_at(d, g, vert ? R + 1 : R, vert ? C : C + 1);
}
__device__ __forceinline__ double euclid_d(double dx, double dy) { return __builtin_sqrt(dx * dx + dy * dy); }
// distance from (x, y) to segment P -> Q and the parameter of the closest point
__device__ __forceinline__ double seg_dist_d(double x, double y, double px, double py, double qx, double qy, double* tp) {
  const double dx = qx - px, dy = qy - py;
  double t = ((x - px) * dx + (y - py) * dy) / (dx * dx + dy * dy);
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  if (tp) *tp = t;
  return euclid_d(x - (px + t * dx), y - (py + t * dy));
}
__device__ __forceinline__ int nearest_index(const Geo& g, double v) {
  return (int)__builtin_floor((v - sample_off(g)) / g.s + 0.5);
}
__device__ __forceinline__ int floor_index(const Geo& g, double v) {
  return (int)__builtin_floor((v - sample_off(g)) / g.s);
}

// thresholds widened by a relative and absolute margin far above the rounding
// of the box bounds, so that a box never misses a candidate
__device__ __forceinline__ double widen(double r) { return r * (1.0 + 1e-12) + 1e-9; }
// Segment j of marching-squares case cs of dual cell (R, C): end points in pixels.
__device__ __forceinline__ void cell_segment(const Geo& g, int R, int C, uint32_t ms, int j, double& px, double& py,
                                             double& qx, double& qy) {
  const int ea = (int)((ms >> (2 + 4 * j)) & 3u), eb = (int)((ms >> (4 + 4 * j)) & 3u);
  // cell edges: 0 top, 1 right, 2 bottom, 3 left (midpoints relative to the TL sample, in s/2)
  const double x0 = (double)g.s * C + sample_off(g), y0 = (double)g.s * R + sample_off(g), hs = 0.5 * g.s;
  px = x0 + (ea == 0 || ea == 2 ? hs : (ea == 1 ? 2.0 * hs : 0.0));
  py = y0 + (ea == 1 || ea == 3 ? hs : (ea == 2 ? 2.0 * hs : 0.0));
  qx = x0 + (eb == 0 || eb == 2 ? hs : (eb == 1 ? 2.0 * hs : 0.0));
  qy = y0 + (eb == 1 || eb == 3 ? hs : (eb == 2 ? 2.0 * hs : 0.0));
}

// Base triangle slot t of owner (k, i) exists (all three corners in the lattice).
__device__ __forceinline__ bool pre_slot_ok(const Geo& g, int k, int i, int t) {
  const int o = k & 1;
  return t == 0 ? (k + 1 < g.NK && i + o - 1 >= 0 && i + o < g.NI) : (k + 1 < g.NK && i + 1 < g.NI && i + o < g.NI);
}
// Owned side e of (k, i) is a side of some base triangle: E0 of Ta(k, i) or of
// Tb of the owner above whose lower side it is, E1 of Tb(k, i) or of
// Ta(k, i-1), E2 of either triangle of (k, i).
__device__ __forceinline__ bool pre_edge_live(const Geo& g, int k, int i, int e) {
  if (e == 0) {
    const int ia = i + 1 - ((k - 1) & 1);
    return pre_slot_ok(g, k, i, 1) || (k >= 1 && ia >= 0 && ia < g.NI && pre_slot_ok(g, k - 1, ia, 0));
  }
  if (e == 1) return pre_slot_ok(g, k, i, 0) || (i >= 1 && pre_slot_ok(g, k, i - 1, 1));
  return pre_slot_ok(g, k, i, 0) || pre_slot_ok(g, k, i, 1);
}

// Flag bits per lattice vertex: 0-2 owned side E0-E2 split, 3 moved, 4 taken
// by a segment (Step 2), 5 snapped (Step 1).
constexpr uint32_t kPreClaim = 16;
constexpr uint32_t kPreSnapped = 32;
// ORs bits into the flag byte of vertex v; returns the byte before.
__device__ __forceinline__ uint32_t pre_flag_or(uint8_t* flags, int64_t v, uint32_t bits) {
  const int sh = 8 * (int)(v & 3);
  const uint32_t old = atomicOr(reinterpret_cast<uint32_t*>(flags + (v & ~(int64_t)3)), bits << sh);
  return (old >> sh) & 0xffu;
}
__device__ __forceinline__ void pre_error(const PreArgs& P) { atomicOr((unsigned long long*)&P.counts[2], 1ull); }
// Wave sum of n added to one of 256 counters of tally `which` (0 snapped,
// 1 repelled); every lane of the wave must call it.
__device__ __forceinline__ void pre_tally(const PreArgs& P, int which, int n) {
  const int tot = __builtin_amdgcn_readlane(wave_incl_scan_dpp(n), 63);
  if ((threadIdx.x & 63) == 0 && tot) {
    const int slot = (int)((blockIdx.x * 4u + (threadIdx.x >> 6)) & 255u);
    atomicAdd((unsigned long long*)&P.counts[kPreTally + 256 * which + slot], (unsigned long long)tot);
  }
}
// Lattice column pitch and row spacing in pixels (to locate rows and columns;
// positions themselves always come from lat_x / lat_y).
__device__ __forceinline__ double pre_hx(const Geo& g) { return (double)g.h / g.U; }
__device__ __forceinline__ double pre_hy(const Geo& g) { return pre_hx(g) * kHalfSqrt3; }
__device__ __forceinline__ int pre_row_floor(const Geo& g, double y) { return (int)__builtin_floor((y + 1.0) / pre_hy(g)); }
__device__ __forceinline__ int pre_lat_X(const Geo& g, int k, int i) { return g.X0 + 4 * g.h * i + 2 * g.h * (k & 1); }
// Owner column of x in row k, as a real number (column i sits at z = i).
__device__ __forceinline__ double pre_col(const Geo& g, int k, double x) {
  return (x - lat_x(g, pre_lat_X(g, k, 0))) / pre_hx(g);
}

// The unmoved lattice: every vertex at its lattice position, flags clear.
// Block: 1024 vertices of one row, four per thread (stride 256).
constexpr int kPreQuad = 4 * kCB;
__global__ void __launch_bounds__(256) k_pre_lattice(OneSrc src, PreArgs P, int nchunk) {
  const Geo g = src.d.g;
  const int k = (int)(blockIdx.x / (unsigned)nchunk);
  const int i0 = (int)(blockIdx.x - (unsigned)k * (unsigned)nchunk) * kPreQuad + (int)threadIdx.x;
  const double y = lat_y(g, k);
  double2* V = reinterpret_cast<double2*>(P.verts);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = i0 + j * kCB;
    if (i >= g.NI) break;
    const int64_t v = (int64_t)k * g.NI + i;
    if (v < P.vcap) {
      V[v] = make_double2(lat_x(g, pre_lat_X(g, k, i)), y);
      P.on_polyline[v] = 0;
    }
    P.flags[v] = 0;
  }
}

// The polyline is enumerated from the coarse raster: thread t of the launch
// takes stored word t of coarse rows -1 .. CH - 1.  Bit j concerns column
// C = C0 + j: dh marks the horizontal midpoint (R, C)-(R, C+1) as a polyline
// vertex, dv the vertical one (R, C)-(R+1, C), and cur / c1 / bel / b1 hold
// the samples (R, C), (R, C+1), (R+1, C), (R+1, C+1) of dual cell (R, C).
struct PreWord {
  int R, C0;
  uint32_t cur, c1, bel, b1, dh, dv;
};
__device__ __forceinline__ void pre_word_at(const Geo& g, uint32_t t, int& R, int& C0) {
  const uint32_t r = t / (uint32_t)g.wpr;
  R = (int)r - 1;
  C0 = 32 * (int)(t - r * (uint32_t)g.wpr) - kRingC;
}
__device__ __forceinline__ bool pre_word(const Img& d, const Geo& g, PreWord& W) {
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= (uint32_t)((g.CH + 1) * g.wpr)) return false;
  pre_word_at(g, t, W.R, W.C0);
  const int w = (W.C0 + kRingC) >> 5;
  const uint32_t* row = d.bits + (int64_t)(W.R + kRing) * g.wpr;
  const bool more = w + 1 < g.wpr;
  W.cur = row[w];
  W.bel = row[g.wpr + w];
  W.c1 = (W.cur >> 1) | ((more ? row[w + 1] : 0u) << 31);
  W.b1 = (W.bel >> 1) | ((more ? row[g.wpr + w + 1] : 0u) << 31);
  W.dh = W.cur ^ W.c1;
  W.dv = W.cur ^ W.bel;
  return true;
}
__device__ __forceinline__ void pre_mid_xy(const Geo& g, int R, int C, int vt, double& x, double& y) {
  x = (double)g.s * C + sample_off(g) + (vt ? 0.0 : 0.5 * g.s);
  y = (double)g.s * R + sample_off(g) + (vt ? 0.5 * g.s : 0.0);
}
// The items the lanes of a wave found (set bits of m0, then of m1; each with a
// 4-bit payload per bit read from pay0 / pay1 when given) are gathered in LDS
// and dealt round-robin to the lanes: f(source lane, which mask, bit, payload).
// Every thread of the block must call it (it synchronises the block).
constexpr int kPreDeal = 64 * 64;
template <class Pay, class F>
__device__ __forceinline__ void pre_deal(uint16_t (*lds)[kPreDeal], uint32_t m0, uint32_t m1, Pay pay, F f) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = __builtin_popcount(m0) + __builtin_popcount(m1);
  const int incl = wave_incl_scan_dpp(n);
  const int total = __builtin_amdgcn_readlane(incl, 63);
  int pos = incl - n;
  for (int which = 0; which < 2; ++which) {
    uint32_t m = which ? m1 : m0;
    while (m) {
      const int j = __builtin_ctz(m);
      m &= m - 1u;
      lds[wv][pos++] = (uint16_t)(lane | (which << 6) | (j << 7) | (pay(which, j) << 12));
    }
  }
  __syncthreads();
  for (int q = lane; q < total; q += 64) {
    const uint32_t e = lds[wv][q];
    f((int)(e & 63u), (int)((e >> 6) & 1u), (int)((e >> 7) & 31u), e >> 12);
  }
}
__device__ __forceinline__ uint32_t pre_no_pay(int, int) { return 0u; }

// Step 1 from the polyline side: the lattice vertex within a of polyline vertex
// (R, C, vt) at (mx, my) is the nearest one of a row within a of my (a < h/2:
// lattice vertices are h apart, so there is at most one); it moves onto the
// polyline vertex.  Returns the number of vertices snapped.
__device__ int pre_snap_one(const PreArgs& P, const Geo& g, int R, int C, int vt) {
  double mx, my;
  pre_mid_xy(g, R, C, vt, mx, my);
  const double aw = widen(P.a);
  int hits = 0;
  for (int k = max(0, pre_row_floor(g, my - aw)); k <= min(g.NK - 1, pre_row_floor(g, my + aw)); ++k) {
    const double yv = lat_y(g, k);
    if (!(__builtin_fabs(yv - my) <= aw)) continue;
    const int i = (int)__builtin_floor(pre_col(g, k, mx) + 0.5);
    if (i < 0 || i >= g.NI) continue;
    const double xv = lat_x(g, pre_lat_X(g, k, i));
    if (!(euclid_d(xv - mx, yv - my) < P.a)) continue;
    ++hits;
    const int64_t v = (int64_t)k * g.NI + i;
    if (pre_flag_or(P.flags, v, kPreSnapped | kPreMoved) & kPreSnapped) pre_error(P);  // two polyline vertices
    if (v < P.vcap) {
      reinterpret_cast<double2*>(P.verts)[v] = make_double2(mx, my);
      P.on_polyline[v] = 1;
    }
    P.mid[mid_id(g, R, C, vt)] = 1;
    P.snap_mid[v] = (int32_t)mid_id(g, R, C, vt);
  }
  if (hits > 1) pre_error(P);
  return hits;
}
__global__ void __launch_bounds__(256) k_pre_snap(OneSrc src, PreArgs P) {
  __shared__ uint16_t lds[4][kPreDeal];
  const Img& d = src.d;
  const Geo g = d.g;
  PreWord W;
  const bool on = P.a > 0.0 && pre_word(d, g, W);
  int n = 0;
  const uint32_t base = blockIdx.x * 256u + (threadIdx.x & ~63u);
  pre_deal(lds, on ? W.dh : 0u, on ? W.dv : 0u, pre_no_pay, [&](int sl, int vt, int j, uint32_t) {
    int R, C0;
    pre_word_at(g, base + sl, R, C0);
    n += pre_snap_one(P, g, R, C0 + j, vt);
  });
  pre_tally(P, 0, n);
}

// Step 2 from the segment side: every lattice vertex not snapped within c of
// segment P -> Q moves along the segment's left normal to distance c on its
// own side.  A vertex taken by two segments, or whose closest point is an end
// of the segment, is a protocol error (c < a/sqrt2 excludes both).  Returns
// the number of vertices moved.
__device__ int pre_repel_seg(const PreArgs& P, const Geo& g, double px, double py, double qx, double qy) {
  const double cw = widen(P.c);
  const double x0 = __builtin_fmin(px, qx) - cw, x1 = __builtin_fmax(px, qx) + cw;
  const double y0 = __builtin_fmin(py, qy) - cw, y1 = __builtin_fmax(py, qy) + cw;
  int n = 0;
  for (int k = max(0, pre_row_floor(g, y0)); k <= min(g.NK - 1, pre_row_floor(g, y1)); ++k) {
    const double yv = lat_y(g, k);
    if (yv < y0 || yv > y1) continue;
    const int i0 = max(0, (int)__builtin_floor(pre_col(g, k, x0))), i1 = min(g.NI - 1, (int)__builtin_floor(pre_col(g, k, x1)));
    for (int i = i0; i <= i1; ++i) {
      const double xv = lat_x(g, pre_lat_X(g, k, i));
      if (xv < x0 || xv > x1) continue;
      const int64_t v = (int64_t)k * g.NI + i;
      if (P.flags[v] & kPreSnapped) continue;
      double t;
      if (!(seg_dist_d(xv, yv, px, py, qx, qy, &t) < P.c)) continue;
      if (pre_flag_or(P.flags, v, kPreClaim | kPreMoved) & kPreClaim) pre_error(P);
      if (!(t > 0.0 && t < 1.0)) pre_error(P);
      const double dx = qx - px, dy = qy - py, L = euclid_d(dx, dy);
      const double nx = -dy / L, ny = dx / L;             // left normal
      const double ds = (xv - px) * nx + (yv - py) * ny;  // signed distance to the line
      const double move = (ds > 0 ? P.c : -P.c) - ds;
      if (v < P.vcap) reinterpret_cast<double2*>(P.verts)[v] = make_double2(xv + move * nx, yv + move * ny);
      ++n;
    }
  }
  return n;
}
__global__ void __launch_bounds__(256) k_pre_repel(OneSrc src, PreArgs P) {
  __shared__ uint16_t lds[4][kPreDeal];
  const Img& d = src.d;
  const Geo g = d.g;
  PreWord W;
  const bool on = P.c > 0.0 && pre_word(d, g, W);
  const uint32_t cells = on ? (W.dh | W.dv | (W.cur ^ W.b1)) : 0u;  // dual cells whose samples differ
  int n = 0;
  const uint32_t base = blockIdx.x * 256u + (threadIdx.x & ~63u);
  auto cs_of = [&](int, int j) {
    return ((W.cur >> j) & 1u) | (((W.c1 >> j) & 1u) << 1) | (((W.b1 >> j) & 1u) << 2) | (((W.bel >> j) & 1u) << 3);
  };
  pre_deal(lds, cells, 0u, cs_of, [&](int sl, int, int j, uint32_t cs) {
    int R, C0;
    pre_word_at(g, base + sl, R, C0);
    const uint32_t ms = ms_case((int)cs);
    for (int q = 0; q < (int)(ms & 3u); ++q) {
      double px, py, qx, qy;
      cell_segment(g, R, C0 + j, ms, q, px, py, qx, qy);
      n += pre_repel_seg(P, g, px, py, qx, qy);
    }
  });
  pre_tally(P, 1, n);
}

// Step 3 from the polyline side: a free polyline vertex (no lattice vertex
// snapped to it) finds the base triangle sides within b of it, on the moved
// vertices.  The vertices moved by less than a, so such a side lies within
// r = a + b of the polyline vertex on the lattice: per row, the owners whose
// side e spans x within r (E0 of rows within r of y, E1 and E2 of rows whose
// band reaches y within r).  One side: it is split there (its owner's flag
// bit and split record); more than one, or a side split twice, is a protocol
// error (b < a/2 excludes both).
__device__ void pre_split_one(const PreArgs& P, const Geo& g, int64_t id, double mx, double my) {
  const double r = widen(P.a + P.b), rr = r / pre_hx(g);
  const double2* V = reinterpret_cast<const double2*>(P.verts);
  int nh = 0;
  int64_t hv = -1;
  int he = 0;
  for (int k = max(0, pre_row_floor(g, my - r) - 1); k <= min(g.NK - 1, pre_row_floor(g, my + r)); ++k) {
    const double yu = lat_y(g, k), z = pre_col(g, k, mx);
    const int o = k & 1;
    for (int e = 0; e < 3; ++e) {
      // side e of owner i spans columns [i, i+1], [i-1/2, i], [i, i+1/2]
      const double lo = e == 0 ? z - 1.0 - rr : (e == 1 ? z - rr : z - 0.5 - rr);
      const double hi = e == 0 ? z + rr : (e == 1 ? z + 0.5 + rr : z + rr);
      const int kw = e == 0 ? k : k + 1;
      for (int i = max(0, (int)__builtin_floor(lo)); i <= min(g.NI - 1, (int)__builtin_floor(hi)); ++i) {
        if (!pre_edge_live(g, k, i, e)) continue;
        const int iw = e == 0 ? i + 1 : (e == 1 ? i + o - 1 : i + o);
        const double xu = lat_x(g, pre_lat_X(g, k, i)), xw = lat_x(g, pre_lat_X(g, kw, iw));
        const double yw = e == 0 ? yu : lat_y(g, kw);
        if (mx < __builtin_fmin(xu, xw) - r || mx > __builtin_fmax(xu, xw) + r || my < __builtin_fmin(yu, yw) - r ||
            my > __builtin_fmax(yu, yw) + r)
          continue;
        const int64_t v = (int64_t)k * g.NI + i;
        const double2 U = V[v], Wv = V[(int64_t)kw * g.NI + iw];
        // both orientations, as the side's two triangles see it
        if (seg_dist_d(mx, my, U.x, U.y, Wv.x, Wv.y, nullptr) < P.b ||
            seg_dist_d(mx, my, Wv.x, Wv.y, U.x, U.y, nullptr) < P.b) {
          ++nh;
          hv = v;
          he = e;
        }
      }
    }
  }
  if (nh > 1) pre_error(P);
  if (nh == 0) return;
  if (pre_flag_or(P.flags, hv, 1u << he) & (1u << he)) pre_error(P);  // a side split twice
  P.split[3 * hv + he] = (int32_t)id;
}
__global__ void __launch_bounds__(256) k_pre_split(OneSrc src, PreArgs P) {
  __shared__ uint16_t lds[4][kPreDeal];
  const Img& d = src.d;
  const Geo g = d.g;
  PreWord W;
  const bool on = P.b > 0.0 && pre_word(d, g, W);
  const uint32_t base = blockIdx.x * 256u + (threadIdx.x & ~63u);
  pre_deal(lds, on ? W.dh : 0u, on ? W.dv : 0u, pre_no_pay, [&](int sl, int vt, int j, uint32_t) {
    int R, C0;
    pre_word_at(g, base + sl, R, C0);
    const int64_t id = mid_id(g, R, C0 + j, vt);
    if (P.mid[id]) return;  // a lattice vertex sits on it
    double mx, my;
    pre_mid_xy(g, R, C0 + j, vt, mx, my);
    pre_split_one(P, g, id, mx, my);
  });
}

// Slots of owner (k, i): Tb = [v, vdr, vdl] has sides E2 of v, E0 of vdl, E1 of
// v; Ta = [v, vr, vdr] has E0 of v, E1 of vr, E2 of v.  Bit j of a slot's
// sides: side j (corner j to corner j+1) is split.  fv / fr / fdl: the flags
// of v, vr and vdl (the owners of the slot sides).
struct PreSlots {
  bool ok[2];
  uint32_t sides[2];
  bool moved[2];
  uint32_t fv, fr, fdl;
};
__device__ __forceinline__ PreSlots pre_owner_slots(const PreArgs& P, const Geo& g, int k, int i) {
  PreSlots S;
  const int o = k & 1;
  const int64_t v = (int64_t)k * g.NI + i, vd = (int64_t)(k + 1) * g.NI + i + o;  // vd: vdr
  S.ok[0] = pre_slot_ok(g, k, i, 0);
  S.ok[1] = pre_slot_ok(g, k, i, 1);
  S.fv = P.flags[v];
  S.fr = S.ok[1] ? P.flags[v + 1] : 0u;
  S.fdl = S.ok[0] ? P.flags[vd - 1] : 0u;
  const uint32_t fdr = (S.ok[0] || S.ok[1]) ? P.flags[vd] : 0u;
  const uint32_t fv = S.fv;
  S.sides[0] = S.ok[0] ? (((fv >> 2) & 1u) | ((S.fdl & 1u) << 1) | (((fv >> 1) & 1u) << 2)) : 0u;
  S.sides[1] = S.ok[1] ? ((fv & 1u) | (((S.fr >> 1) & 1u) << 1) | (((fv >> 2) & 1u) << 2)) : 0u;
  S.moved[0] = S.ok[0] && ((fv | fdr | S.fdl) & kPreMoved);
  S.moved[1] = S.ok[1] && ((fv | S.fr | fdr) & kPreMoved);
  return S;
}
// One wave per row segment of kCB owners; lane l takes owners i0 + l + 64 j,
// j = 0 .. 3, so that loads and stores of neighbouring lanes are adjacent.
__device__ __forceinline__ bool pre_segment(const Geo& g, const Shared& sh, int64_t& seg, int& k, int& i0) {
  const uint32_t sg = blockIdx.x * 4u + (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  seg = sg;
  if (seg >= sh.nseg) return false;
  const uint32_t kk = sg / (uint32_t)g.NCB;  // segment counts fit 32 bits (grid of nseg / 4 blocks)
  k = (int)kk;
  i0 = (int)(sg - kk * (uint32_t)g.NCB) * kCB;
  return true;
}

// Per row segment: inserted vertices (split sides owned) and triangles (one
// per slot, two for a slot with a split side).
__global__ void __launch_bounds__(256) k_pre_count(OneSrc src, PreArgs P, Shared sh) {
  const Geo g = src.d.g;
  int64_t seg;
  int k, i0;
  if (!pre_segment(g, sh, seg, k, i0)) return;  // wave-uniform
  int ni = 0, nt = 0;
  PreSlots S[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {  // every flag load of the lane first
    const int i = i0 + 64 * j + (int)(threadIdx.x & 63);
    S[j].ok[0] = S[j].ok[1] = false;
    if (i < g.NI) S[j] = pre_owner_slots(P, g, k, i);
  }
  const double2* V = reinterpret_cast<const double2*>(P.verts);
  const int o = k & 1;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = i0 + 64 * j + (int)(threadIdx.x & 63);
    if (i >= g.NI) break;
    ni += __builtin_popcount(S[j].fv & 7u);
    for (int t = 0; t < 2; ++t) {
      if (!S[j].ok[t]) continue;
      const int ns = __builtin_popcount(S[j].sides[t]);
      if (ns > 1) pre_error(P);  // a triangle with two split sides
      nt += ns ? 2 : 1;
      if (!S[j].moved[t] && !ns) continue;
      // positive orientation of the base triangle after the moves, and of
      // the two triangles fanned around an inserted vertex
      const int64_t v = (int64_t)k * g.NI + i;
      const int64_t C1 = t == 0 ? (int64_t)(k + 1) * g.NI + (i + o) : v + 1;
      const int64_t C2 = t == 0 ? (int64_t)(k + 1) * g.NI + (i + o - 1) : (int64_t)(k + 1) * g.NI + (i + o);
      const double2 Cp[3] = {V[v], V[C1], V[C2]};
      auto area2 = [](double2 A, double2 B, double2 C) {
        return (B.x - A.x) * (C.y - A.y) - (B.y - A.y) * (C.x - A.x);
      };
      if (!(area2(Cp[0], Cp[1], Cp[2]) > 0.0)) pre_error(P);
      if (!ns) continue;
      const int js = __builtin_ctz(S[j].sides[t]);
      const int64_t w = t == 0 ? (js == 1 ? C2 : v) : (js == 1 ? v + 1 : v);
      const int e = t == 0 ? (js == 0 ? 2 : (js == 1 ? 0 : 1)) : js;
      const int32_t m = P.split[3 * w + e];
      double2 M;
      pre_mid_xy(g, (m >> 1) / (g.CW + 2) - 1, (m >> 1) % (g.CW + 2) - 1, m & 1, M.x, M.y);
      const double2 a0 = Cp[js], a1 = Cp[(js + 1) % 3], a2 = Cp[(js + 2) % 3];
      if (!(area2(a0, M, a2) > 0.0) || !(area2(M, a1, a2) > 0.0)) pre_error(P);
    }
  }
  const int si = __builtin_amdgcn_readlane(wave_incl_scan_dpp(ni), 63);
  const int st = __builtin_amdgcn_readlane(wave_incl_scan_dpp(nt), 63);
  if ((threadIdx.x & 63) == 0) {
    sh.seg_cnt[seg] = make_int4(si, st, 0, 0);
    sh.seg_slow[seg] = 0ull;
  }
}

// Inserted vertices at their offsets (row segment base from the scan, owner
// offsets by wave scans), and the first inserted index of each owner that has one.
__global__ void __launch_bounds__(256) k_pre_inserted(OneSrc src, PreArgs P, Shared sh) {
  const Img& d = src.d;
  const Geo g = d.g;
  int64_t seg;
  int k, i0;
  if (!pre_segment(g, sh, seg, k, i0)) return;
  if (sh.seg_cnt[seg].x == 0) return;
  const int64_t nlat = (int64_t)g.NK * g.NI;
  int64_t base = sh.seg_off[seg].x;
  for (int j = 0; j < 4; ++j) {
    const int i = i0 + 64 * j + (int)(threadIdx.x & 63);
    const int64_t v = (int64_t)k * g.NI + i;
    const uint32_t f = i < g.NI ? (P.flags[v] & 7u) : 0u;
    const int n = __builtin_popcount(f);
    const int incl = wave_incl_scan_dpp(n);
    if (f) {
      int64_t pos = base + (incl - n);
      P.ins_base[v] = pos;
      for (int e = 0; e < 3; ++e) {
        if (!((f >> e) & 1u)) continue;
        const int32_t m = P.split[3 * v + e];
        const int R = (m >> 1) / (g.CW + 2) - 1, C = (m >> 1) % (g.CW + 2) - 1;
        double mx, my;
        pre_mid_xy(g, R, C, m & 1, mx, my);
        const int64_t id = nlat + pos++;
        if (id < P.vcap) {
          reinterpret_cast<double2*>(P.verts)[id] = make_double2(mx, my);
          P.on_polyline[id] = 1;
        }
      }
    }
    base += __builtin_amdgcn_readlane(incl, 63);
  }
}

// One wave copies n int32 values staged in LDS to dst (4-byte aligned):
// 16-byte stores over the 16-byte-aligned body, single words at its ends.
__device__ __forceinline__ void pre_wave_store(const int32_t* src, int32_t* dst, int n, int lane) {
  const int h = min((int)((16u - ((uint32_t)(uintptr_t)dst & 15u)) & 15u) >> 2, max(n, 0));
  if (lane < h) dst[lane] = src[lane];
  const int body = (n - h) >> 2;
  for (int q = lane; q < body; q += 64) {
    const int e = h + 4 * q;
    *reinterpret_cast<int4*>(dst + e) = make_int4(src[e], src[e + 1], src[e + 2], src[e + 3]);
  }
  const int t0 = h + 4 * max(body, 0);
  if (t0 + lane < n) dst[t0 + lane] = src[t0 + lane];
}

// Triangles of each row segment at their offsets (row segment base from the
// scan, owner offsets by wave scans).  Per 64 owners the wave stages its
// triangles in LDS and writes them as one contiguous run.  A slot with a split
// side j (corners a0 -> a1, opposite a2) becomes (a0, m, a2), (m, a1, a2)
// around the inserted vertex m.  Triangles with a moved or inserted corner are
// checked for positive orientation.
__global__ void __launch_bounds__(256) k_pre_triangles(OneSrc src, PreArgs P, Shared sh) {
  __shared__ int32_t stage[4][3 * 4 * 64];
  const Geo g = src.d.g;
  int64_t seg;
  int k, i0;
  if (!pre_segment(g, sh, seg, k, i0)) return;
  const int lane = (int)(threadIdx.x & 63);
  int32_t* st = stage[threadIdx.x >> 6];
  const int64_t nlat = (int64_t)g.NK * g.NI;
  const int o = k & 1;
  int64_t base = sh.seg_off[seg].y;
  PreSlots SS[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {  // every flag load of the lane first
    const int i = i0 + 64 * j + lane;
    SS[j].ok[0] = SS[j].ok[1] = false;
    if (i < g.NI) SS[j] = pre_owner_slots(P, g, k, i);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = i0 + 64 * j + lane;
    const PreSlots& S = SS[j];
    int nt = 0;
    for (int t = 0; t < 2; ++t) nt += S.ok[t] ? (S.sides[t] ? 2 : 1) : 0;
    const int incl = wave_incl_scan_dpp(nt);
    const int tot = __builtin_amdgcn_readlane(incl, 63);
    if (nt) {
      int pos = incl - nt;
      // (orientation checked by k_pre_count)
      auto put = [&](int64_t a, int64_t b, int64_t c, bool) {
        st[3 * pos] = (int32_t)a;
        st[3 * pos + 1] = (int32_t)b;
        st[3 * pos + 2] = (int32_t)c;
        ++pos;
      };
      const int64_t v = (int64_t)k * g.NI + i;
      for (int t = 0; t < 2; ++t) {
        if (!S.ok[t]) continue;
        const int64_t C0 = v;
        const int64_t C1 = t == 0 ? (int64_t)(k + 1) * g.NI + (i + o) : v + 1;
        const int64_t C2 = t == 0 ? (int64_t)(k + 1) * g.NI + (i + o - 1) : (int64_t)(k + 1) * g.NI + (i + o);
        if (!S.sides[t]) {
          put(C0, C1, C2, S.moved[t]);
          continue;
        }
        const int js = __builtin_ctz(S.sides[t]);
        // the owner and owned side of side js
        const int64_t w = t == 0 ? (js == 1 ? C2 : v) : (js == 1 ? v + 1 : v);
        const int e = t == 0 ? (js == 0 ? 2 : (js == 1 ? 0 : 1)) : js;
        const uint32_t fw = t == 0 ? (js == 1 ? S.fdl : S.fv) : (js == 1 ? S.fr : S.fv);
        const int64_t m = nlat + P.ins_base[w] + __builtin_popcount(fw & ((1u << e) - 1u));
        const int64_t Cs[3] = {C0, C1, C2};
        const int64_t a0 = Cs[js], a1 = Cs[(js + 1) % 3], a2 = Cs[(js + 2) % 3];
        put(a0, m, a2, true);
        put(m, a1, a2, true);
      }
    }
    // the wave's LDS writes are seen by its own later reads (one wave, program order)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t lim = 3 * (P.tcap - base);  // staged entries that fit the capacity
    pre_wave_store(st, P.tris + 3 * base, (int)min((int64_t)(3 * tot), max(lim, (int64_t)0)), lane);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    base += tot;
  }
}

__global__ void k_pre_clear(PreArgs P, int64_t nmid) {
  uint32_t* m4 = reinterpret_cast<uint32_t*>(P.mid);  // the region is padded to 256 bytes
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < (nmid + 3) / 4; q += (int64_t)gridDim.x * blockDim.x)
    m4[q] = 0u;
  for (int q = threadIdx.x; blockIdx.x == 0 && q < kPreCounts; q += blockDim.x) P.counts[q] = 0;
  if (P.used) {
    uint32_t* u4 = reinterpret_cast<uint32_t*>(P.used);  // padded to 256 bytes
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < (P.usedcap + 3) / 4;
         q += (int64_t)gridDim.x * blockDim.x)
      u4[q] = 0u;
  }
}

__global__ void k_pre_sizes(OneSrc src, PreArgs P, Shared sh, int64_t* out) {
  const Geo g = src.d.g;
  const longlong4 tot = sh.seg_off[sh.nseg];
  int64_t ns = 0, nr = 0;
  for (int q = 0; q < 256; ++q) {
    ns += P.counts[kPreTally + q];
    nr += P.counts[kPreTally + 256 + q];
  }
  out[0] = (int64_t)g.NK * g.NI + tot.x;  // vertices
  out[1] = tot.y;                          // triangles
  out[2] = ns;                             // snapped
  out[3] = nr;                             // repelled
  out[4] = tot.x;                          // inserted
  out[5] = P.counts[2] ? SBMT_E_PROTOCOL : ((out[0] > P.vcap || out[1] > P.tcap) ? SBMT_E_CAPACITY : SBMT_OK);
  if (out[0] > 0x7fffffffLL) out[5] = SBMT_E_INDEX_OVERFLOW;
}

// ---------------------------------------------------------------------------
// Retriangulation of the preprocessed grid against the polyline (the mesh of
// Alg. 3, Sec. 3.5): every grid triangle is cut by the polyline pieces inside
// it, its faces are traced along its boundary and the pieces, and the
// foreground faces are triangulated by the template rule (fanned from the
// chain vertex inside the triangle; the quadrilateral between two chords split
// by the diagonal joining their exits; else fanned from the face's earliest
// chain point); an uncut triangle is kept whole when it lies in the foreground.
// Decisions in FP64 on the moved points, as the oracle takes them; the margins
// c and b of Steps 2 and 3 keep them away from zero.  A corner that sits on a
// polyline vertex is that vertex by identity.
//
// Output vertices: the grid vertices (ids 0 .. NV-1, positions from the grid
// phase), then per owner (by the scan) its new vertices: the crossings of the
// grid edges it owns, edge slot by edge slot (slot 2e and 2e+1: side E_e, or
// its two halves around the inserted vertex; slot 6 + t: the fan edge of its
// split slot t), each edge's crossings in order from its lower-numbered end;
// then the polyline vertices strictly inside its slots' triangles.
// ---------------------------------------------------------------------------
struct PreSeg {
  double px, py, qx, qy;
  int32_t jp, jq;  // ids of the polyline vertices at the start and the end
};
__device__ __forceinline__ int32_t pre_cell_edge_mid(const Geo& g, int R, int C, int e) {
  // cell edges: 0 top, 1 right, 2 bottom, 3 left
  return (int32_t)(e == 0 ? mid_id(g, R, C, 0) : (e == 1 ? mid_id(g, R, C + 1, 1) : (e == 2 ? mid_id(g, R + 1, C, 0) : mid_id(g, R, C, 1))));
}
// A thread's copy of the coarse samples around one owner: rows R0 .. R0+nr-1,
// columns C0 .. C0+31 as row masks (background outside the stored raster).
struct PreBits {
  int R0, C0, nr;
  uint32_t rw[6];
};
__device__ __forceinline__ void pre_bits_load(const Img& d, const Geo& g, int R0, int C0, int nr, PreBits& B) {
  B.R0 = R0;
  B.C0 = C0;
  B.nr = nr;
  const int cc = C0 + kRingC;
  const int w0 = cc >> 5, sh = cc & 31;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    const int R = R0 + r;
    uint32_t w = 0;
    if (r < nr && R >= 0 && R < g.CH) {
      const uint32_t* row = d.bits + (int64_t)(R + kRing) * g.wpr;
      const uint64_t lo = (w0 >= 0 && w0 < g.wpr) ? row[w0] : 0u;
      const uint64_t hi = (w0 + 1 >= 0 && w0 + 1 < g.wpr) ? row[w0 + 1] : 0u;
      w = (uint32_t)((((hi << 32) | lo) >> sh));
      // columns outside the image are background
      const int cfirst = C0, clast = C0 + 31;
      if (cfirst < 0) w = -cfirst >= 32 ? 0u : (w & (~0u << (-cfirst)));
      if (clast >= g.CW) w &= (g.CW - C0) <= 0 ? 0u : (g.CW - C0 >= 32 ? ~0u : ((1u << (g.CW - C0)) - 1u));
    }
    B.rw[r] = w;
  }
}
// Row r of the block, selected rather than indexed (which would put rw in
// scratch memory).
__device__ __forceinline__ uint32_t pre_bits_row(const PreBits& B, int r) {
  uint32_t w = B.rw[0];
#pragma unroll
  for (int q = 1; q < 6; ++q) w = r == q ? B.rw[q] : w;
  return w;
}
__device__ __forceinline__ int pre_cell_case(const Img& d, const Geo& g, int R, int C, const PreBits* B = nullptr) {
  if (B && R >= B->R0 && R + 1 < B->R0 + B->nr && C >= B->C0 && C + 1 < B->C0 + 32) {
    const uint32_t t = pre_bits_row(*B, R - B->R0) >> (C - B->C0), u = pre_bits_row(*B, R + 1 - B->R0) >> (C - B->C0);
    return (int)((t & 1u) | ((t & 2u)) | ((u & 2u) << 1) | ((u & 1u) << 3));
  }
  return sample_at(d, g, R, C) | (sample_at(d, g, R, C + 1) << 1) | (sample_at(d, g, R + 1, C + 1) << 2) |
         (sample_at(d, g, R + 1, C) << 3);
}
// Calls f(seg) for every segment of the dual cells that contain a point of
// [x0, x1] x [y0, y1] (callers widen their boxes by a margin, so a cell that
// only touches the box's border holds no segment reaching inside it).
template <class F>
__device__ __forceinline__ void pre_segs_in_box(const Img& d, const Geo& g, double x0, double x1, double y0, double y1, F f,
                                                const PreBits* B = nullptr) {
  const int R0 = floor_index(g, y0), R1 = floor_index(g, y1);
  const int C0 = floor_index(g, x0), C1 = floor_index(g, x1);
  for (int R = R0; R <= R1; ++R)
    for (int C = C0; C <= C1; ++C) {
      const int cs = pre_cell_case(d, g, R, C, B);
      if (cs == 0 || cs == 15) continue;
      const uint32_t ms = ms_case(cs);
      for (int j = 0; j < (int)(ms & 3u); ++j) {
        PreSeg S;
        cell_segment(g, R, C, ms, j, S.px, S.py, S.qx, S.qy);
        S.jp = pre_cell_edge_mid(g, R, C, (int)((ms >> (2 + 4 * j)) & 3u));
        S.jq = pre_cell_edge_mid(g, R, C, (int)((ms >> (4 + 4 * j)) & 3u));
        f(S);
      }
    }
}
// Inside the foreground: the dual cell of the point, uniform or left of each
// of its segments (segments have the foreground on their left).  Used for
// points at a distance from the polyline (lattice corners off it, centroids of
// uncut triangles).
__device__ __forceinline__ int pre_inside_point(const Img& d, const Geo& g, double x, double y,
                                                const PreBits* B = nullptr) {
  const int R = floor_index(g, y), C = floor_index(g, x);
  const int cs = pre_cell_case(d, g, R, C, B);
  if (cs == 0 || cs == 15) return cs == 15;
  const uint32_t ms = ms_case(cs);
  for (int j = 0; j < (int)(ms & 3u); ++j) {
    double px, py, qx, qy;
    cell_segment(g, R, C, ms, j, px, py, qx, qy);
    if (!((qx - px) * (y - py) - (qy - py) * (x - px) > 0.0)) return 0;
  }
  return 1;
}
// Grid vertex: id, position, the polyline vertex it sits on (or -1).  Grid
// vertex and owner indices fit 32 bits (the entry points check it).
struct PreGV {
  int32_t id;
  int32_t bnd;
  double x, y;
};
__device__ __forceinline__ PreGV pre_lat_gv(const PreArgs& P, int64_t v) {
  PreGV r;
  r.id = (int32_t)v;
  const double2 p = reinterpret_cast<const double2*>(P.verts)[v];
  r.x = p.x;
  r.y = p.y;
  r.bnd = (P.flags[v] & kPreSnapped) ? P.snap_mid[v] : -1;
  return r;
}
// The vertex inserted on side e of owner w (flags fw).
__device__ __forceinline__ PreGV pre_ins_gv(const PreArgs& P, const Geo& g, int64_t w, int e, uint32_t fw) {
  PreGV r;
  r.id = (int32_t)((int64_t)g.NK * g.NI + P.ins_base[w] + __builtin_popcount(fw & ((1u << e) - 1u)));
  const double2 p = reinterpret_cast<const double2*>(P.verts)[r.id];
  r.x = p.x;
  r.y = p.y;
  r.bnd = P.split[3 * w + e];
  return r;
}
// Whether segment S crosses the grid edge U - W at an interior point of both
// (a segment end that is U's or W's polyline vertex lies on the edge's line);
// te: the crossing's position along U -> W (monotone, unnormalised).
__device__ __forceinline__ bool pre_crosses(const PreSeg& S, const PreGV& U, const PreGV& W, double* te) {
  const double gx = W.x - U.x, gy = W.y - U.y;
  const double dp = (S.jp == U.bnd || S.jp == W.bnd) ? 0.0 : gx * (S.py - U.y) - gy * (S.px - U.x);
  const double dq = (S.jq == U.bnd || S.jq == W.bnd) ? 0.0 : gx * (S.qy - U.y) - gy * (S.qx - U.x);
  if (!((dp > 0.0 && dq < 0.0) || (dp < 0.0 && dq > 0.0))) return false;
  const double hx = S.qx - S.px, hy = S.qy - S.py;
  const double eu = hx * (U.y - S.py) - hy * (U.x - S.px), ew = hx * (W.y - S.py) - hy * (W.x - S.px);
  if (!((eu > 0.0 && ew < 0.0) || (eu < 0.0 && ew > 0.0))) return false;
  if (te) {
    const double t = dp / (dp - dq);
    *te = (S.px + t * hx - U.x) * gx + (S.py + t * hy - U.y) * gy;
  }
  return true;
}
// The crossing point of grid edge (lo, hi), lo < hi, by segment S.
__device__ __forceinline__ void pre_crossing_xy(const PreSeg& S, const PreGV& L, const PreGV& H, double& x, double& y) {
  const double gx = H.x - L.x, gy = H.y - L.y;
  const double dp = gx * (S.py - L.y) - gy * (S.px - L.x);
  const double dq = gx * (S.qy - L.y) - gy * (S.qx - L.x);
  const double t = dp / (dp - dq);
  x = S.px + t * (S.qx - S.px);
  y = S.py + t * (S.qy - S.py);
}
// Calls f(seg, te) for every segment crossing grid edge U - W.
template <class F>
__device__ __forceinline__ void pre_edge_crossings(const Img& d, const Geo& g, const PreGV& U, const PreGV& W, F f,
                                                   const PreBits* B = nullptr) {
  const double m = 1e-9;
  pre_segs_in_box(d, g, fmin(U.x, W.x) - m, fmax(U.x, W.x) + m, fmin(U.y, W.y) - m, fmax(U.y, W.y) + m,
                  [&](const PreSeg& S) {
                    double te;
                    if (pre_crosses(S, U, W, &te)) f(S, te);
                  }, B);
}

// A grid triangle of an owner's slot: corners, and per edge e (corner e to
// e+1) the owner and edge slot that number its crossings.
struct PreGT {
  PreGV c[3];
  int32_t eo[3];
  int es[3];
};
// x, y or z for j = 0, 1, 2: selects rather than an indexed local array,
// which would live in scratch memory.
template <class V>
__device__ __forceinline__ V pre_sel3(const V& x, const V& y, const V& z, int j) {
  return j == 0 ? x : (j == 1 ? y : z);
}
// Edge slot q of owner (k, i): its ends (false if the owner has no such edge).
__device__ bool pre_edge_slot(const PreArgs& P, const Geo& g, int k, int i, const PreSlots& S, int q, PreGV& A,
                              PreGV& B) {
  const int o = k & 1;
  const int64_t v = (int64_t)k * g.NI + i;
  if (q < 6) {
    const int e = q >> 1;
    if (!pre_edge_live(g, k, i, e)) return false;
    const int kw = e == 0 ? k : k + 1, iw = e == 0 ? i + 1 : (e == 1 ? i + o - 1 : i + o);
    const bool split = (S.fv >> e) & 1u;
    if (!split && (q & 1)) return false;
    const PreGV U = pre_lat_gv(P, v), W = pre_lat_gv(P, (int64_t)kw * g.NI + iw);
    if (!split) {
      A = U;
      B = W;
      return true;
    }
    const PreGV M = pre_ins_gv(P, g, v, e, S.fv);
    A = (q & 1) ? M : U;
    B = (q & 1) ? W : M;
    return true;
  }
  const int t = q - 6;
  if (!S.ok[t] || !S.sides[t]) return false;
  const int js = __builtin_ctz(S.sides[t]);
  const int64_t C0 = v;
  const int64_t C1 = t == 0 ? (int64_t)(k + 1) * g.NI + (i + o) : v + 1;
  const int64_t C2 = t == 0 ? (int64_t)(k + 1) * g.NI + (i + o - 1) : (int64_t)(k + 1) * g.NI + (i + o);
  const int64_t w = t == 0 ? (js == 1 ? C2 : v) : (js == 1 ? v + 1 : v);
  const int e = t == 0 ? (js == 0 ? 2 : (js == 1 ? 0 : 1)) : js;
  const uint32_t fw = t == 0 ? (js == 1 ? S.fdl : S.fv) : (js == 1 ? S.fr : S.fv);
  A = pre_ins_gv(P, g, w, e, fw);
  B = pre_lat_gv(P, pre_sel3(C0, C1, C2, (js + 2) % 3));
  return true;
}
// The grid triangles of slot t of owner (k, i): one, or two fanned around the
// inserted vertex of its split side.  Returns their number.
__device__ int pre_slot_tris(const PreArgs& P, const Geo& g, int k, int i, const PreSlots& S, int t, PreGT* T) {
  if (!S.ok[t]) return 0;
  const int o = k & 1;
  const int64_t v = (int64_t)k * g.NI + i;
  const int64_t C0 = v;
  const int64_t C1 = t == 0 ? (int64_t)(k + 1) * g.NI + (i + o) : v + 1;
  const int64_t C2 = t == 0 ? (int64_t)(k + 1) * g.NI + (i + o - 1) : (int64_t)(k + 1) * g.NI + (i + o);
  // side j: owner, owned side, and whether corner j is that owner
  // Tb = [v, vdr, vdl]: E2 of v, E0 of vdl, E1 of v; Ta = [v, vr, vdr]: E0 of v, E1 of vr, E2 of v
  const int64_t so0 = v, so1 = t == 0 ? C2 : v + 1, so2 = v;
  const int se0 = t == 0 ? 2 : 0, se1 = t == 0 ? 0 : 1, se2 = t == 0 ? 1 : 2;
  const bool sa0 = true, sa1 = t != 0, sa2 = false;
  const PreGV G0 = pre_lat_gv(P, C0), G1 = pre_lat_gv(P, C1), G2 = pre_lat_gv(P, C2);
  if (!S.sides[t]) {
    T[0].c[0] = G0;
    T[0].c[1] = G1;
    T[0].c[2] = G2;
    T[0].eo[0] = so0;
    T[0].eo[1] = so1;
    T[0].eo[2] = so2;
    T[0].es[0] = 2 * se0;
    T[0].es[1] = 2 * se1;
    T[0].es[2] = 2 * se2;
    return 1;
  }
  const int js = __builtin_ctz(S.sides[t]);
  const uint32_t fw = t == 0 ? (js == 1 ? S.fdl : S.fv) : (js == 1 ? S.fr : S.fv);
  const int j1 = (js + 1) % 3, j2 = (js + 2) % 3;
  const int64_t soj = pre_sel3(so0, so1, so2, js);
  const int sej = pre_sel3(se0, se1, se2, js);
  const bool saj = pre_sel3(sa0, sa1, sa2, js);
  const PreGV M = pre_ins_gv(P, g, soj, sej, fw);
  const int h0 = 2 * sej + (saj ? 0 : 1), h1 = 2 * sej + (saj ? 1 : 0);
  const PreGV Gs = pre_sel3(G0, G1, G2, js), G1s = pre_sel3(G0, G1, G2, j1), G2s = pre_sel3(G0, G1, G2, j2);
  // (a0, m, a2): a0 -> m (half of the split side), m -> a2 (fan edge), a2 -> a0
  T[0].c[0] = Gs;
  T[0].c[1] = M;
  T[0].c[2] = G2s;
  T[0].eo[0] = soj;
  T[0].es[0] = h0;
  T[0].eo[1] = v;
  T[0].es[1] = 6 + t;
  T[0].eo[2] = pre_sel3(so0, so1, so2, j2);
  T[0].es[2] = 2 * pre_sel3(se0, se1, se2, j2);
  // (m, a1, a2): m -> a1 (other half), a1 -> a2, a2 -> m (fan edge)
  T[1].c[0] = M;
  T[1].c[1] = G1s;
  T[1].c[2] = G2s;
  T[1].eo[0] = soj;
  T[1].es[0] = h1;
  T[1].eo[1] = pre_sel3(so0, so1, so2, j1);
  T[1].es[1] = 2 * pre_sel3(se0, se1, se2, j1);
  T[1].eo[2] = v;
  T[1].es[2] = 6 + t;
  return 2;
}

// Per-owner counts of the retriangulation: crossings of edge slot q in bits
// 2q .. 2q+1, polyline vertices inside its triangles in 16 .. 18, output
// triangles in 19 .. 26, cut grid triangles in 27 .. 29.
__device__ __forceinline__ int pre_rc_cross(uint32_t rc, int q) { return (int)((rc >> (2 * q)) & 3u); }
__device__ __forceinline__ int pre_rc_before(uint32_t rc, int q) {  // crossings of slots before q
  int n = 0;
  for (int j = 0; j < q; ++j) n += pre_rc_cross(rc, j);
  return n;
}
__device__ __forceinline__ int pre_rc_inner(uint32_t rc) { return (int)((rc >> 16) & 7u); }
__device__ __forceinline__ int pre_rc_tris(uint32_t rc) { return (int)((rc >> 19) & 255u); }
__device__ __forceinline__ int pre_rc_cut(uint32_t rc) { return (int)((rc >> 27) & 7u); }

// A point of a triangle's subdivision: kind 0 grid vertex a; 1 crossing of
// grid edge (a, b), a < b, by segment s; 2 polyline vertex a strictly inside
// (s: the segment ending there).  ct: position along the chain.
struct PrePt {
  int32_t kind;
  int32_t a, b;
  int32_t s;
  double x, y, ct;
};
__device__ __forceinline__ bool pre_same(const PrePt& p, const PrePt& q) {
  return p.kind == q.kind && p.a == q.a && p.b == q.b && p.s == q.s;
}
struct PreSub {
  PreSeg S;
  double t0, t1;
  int e0, e1, c0, c1;
};

// Cuts grid triangle T by the polyline and triangulates its foreground faces,
// calling out(p0, p1, p2, code) per output triangle (code 0: the grid
// triangle kept whole, 1: a piece of a cut one).  Returns the number of
// polyline vertices strictly inside T (0 or 1) and sets *inner to it.  With
// kDefer, a cut triangle only sets *cut and returns -1 once its pieces are
// known (callers gather those and come back to them on full waves).
// With kCount, a foreground face of m points is reported as m - 2 triangles
// fanned from its first point: the same count and the same points as the
// template's triangles, without the template rule and its checks (for
// passes that only count; the pass that writes the triangles applies them).
template <bool kDefer = false, bool kCount = false, class Out>
__device__ int pre_tri_mesh(const Img& d, const Geo& g, const PreArgs& P, const PreGT& T, Out out, PrePt* inner,
                            bool* cut = nullptr, const PreBits* Bits = nullptr) {
  const int64_t NLAT = (int64_t)g.NK * g.NI;
  double minx = T.c[0].x, maxx = T.c[0].x, miny = T.c[0].y, maxy = T.c[0].y;
  for (int j = 1; j < 3; ++j) {
    minx = fmin(minx, T.c[j].x);
    maxx = fmax(maxx, T.c[j].x);
    miny = fmin(miny, T.c[j].y);
    maxy = fmax(maxy, T.c[j].y);
  }
  PreSub subs[3];
  int nsub = 0, edge_side = -1;
  bool bad = false;
  pre_segs_in_box(d, g, minx - 1e-9, maxx + 1e-9, miny - 1e-9, maxy + 1e-9, [&](const PreSeg& S) {
    if (fmax(S.px, S.qx) < minx - 1e-9 || fmin(S.px, S.qx) > maxx + 1e-9 || fmax(S.py, S.qy) < miny - 1e-9 ||
        fmin(S.py, S.qy) > maxy + 1e-9)
      return;
    // clip against the three edge half-planes (inside = left of each edge)
    double t0 = 0.0, t1 = 1.0;
    int e0 = -1, e1 = -1;
    for (int e = 0; e < 3; ++e) {
      const PreGV& A = T.c[e];
      const PreGV& B = T.c[(e + 1) % 3];
      // an end of the segment that is a corner of this edge lies on its line
      const double fp = (A.bnd == S.jp || B.bnd == S.jp) ? 0.0 : (B.x - A.x) * (S.py - A.y) - (B.y - A.y) * (S.px - A.x);
      const double fq = (A.bnd == S.jq || B.bnd == S.jq) ? 0.0 : (B.x - A.x) * (S.qy - A.y) - (B.y - A.y) * (S.qx - A.x);
      if (fp < 0 && fq < 0) return;
      if (fp >= 0 && fq >= 0) continue;
      const double t = fp / (fp - fq);
      if (fp < 0) {
        if (t > t0) {
          t0 = t;
          e0 = e;
        }
      } else if (t < t1) {
        t1 = t;
        e1 = e;
      }
    }
    if (!(t1 > t0)) return;
    PreSub sb;
    sb.S = S;
    sb.t0 = t0;
    sb.t1 = t1;
    sb.e0 = e0;
    sb.e1 = e1;
    sb.c0 = sb.c1 = -1;
    for (int j = 0; j < 3; ++j) {
      if (T.c[j].bnd == S.jp && t0 == 0.0) {
        sb.c0 = j;
        sb.e0 = -1;
      }
      if (T.c[j].bnd == S.jq && t1 == 1.0) {
        sb.c1 = j;
        sb.e1 = -1;
      }
    }
    if (sb.c0 >= 0 && sb.c1 >= 0) {
      // the segment joins two corners: it lies on their edge, and the
      // triangle lies on the side of its third corner
      const PreGV& T3 = T.c[3 - sb.c0 - sb.c1];
      edge_side = ((S.qx - S.px) * (T3.y - S.py) - (S.qy - S.py) * (T3.x - S.px)) > 0 ? 1 : 0;
      return;
    }
    if (!kDefer && nsub < 3) subs[nsub] = sb;  // (a probe only needs to know that there is one)
    ++nsub;
  }, Bits);
  if (nsub == 0) {
    // uncut: side from a segment along an edge, a lattice corner off the
    // polyline, else the centroid
    int fg = edge_side;
    for (int j = 0; j < 3 && fg < 0; ++j)
      if (T.c[j].id < NLAT && T.c[j].bnd < 0) fg = pre_inside_point(d, g, T.c[j].x, T.c[j].y, Bits);
    if (fg < 0) {
      double cx = 0, cy = 0;
      for (int j = 0; j < 3; ++j) {
        cx += T.c[j].x / 3;
        cy += T.c[j].y / 3;
      }
      fg = pre_inside_point(d, g, cx, cy, Bits);
    }
    if (fg) {
      PrePt p[3];
      for (int j = 0; j < 3; ++j) p[j] = PrePt{0, T.c[j].id, 0, -1, T.c[j].x, T.c[j].y, 0.0};
      out(p[0], p[1], p[2], 0);
    }
    return 0;
  }
  if (cut) *cut = true;
  if (kDefer) return -1;
  if (nsub > 2) {  // more than two segments in one triangle
    pre_error(P);
    return 0;
  }
  if (nsub == 2) {  // chain order
    if (subs[1].S.jq == subs[0].S.jp) {
      const PreSub tmp = subs[0];
      subs[0] = subs[1];
      subs[1] = tmp;
    }
    if (subs[0].S.jq != subs[1].S.jp) {
      pre_error(P);
      return 0;
    }
  }
  // Points of the subdivision in a pool (corners first); pieces, the boundary
  // cycle and the faces refer to them by index.
  PrePt pool[8];
  int np = 3;
  for (int j = 0; j < 3; ++j) pool[j] = PrePt{0, T.c[j].id, 0, -1, T.c[j].x, T.c[j].y, 0.0};
  auto cross_pt = [&](int e, const PreSeg& S) {
    const PreGV& A = T.c[e];
    const PreGV& B = T.c[(e + 1) % 3];
    const PreGV& L = A.id < B.id ? A : B;
    const PreGV& H = A.id < B.id ? B : A;
    PrePt p;
    p.kind = 1;
    p.a = L.id;
    p.b = H.id;
    p.s = S.jp;
    pre_crossing_xy(S, L, H, p.x, p.y);
    p.ct = 0.0;
    return p;
  };
  // pieces: the chain inside the triangle, from boundary to boundary
  uint8_t pc[2][3];
  int pn[2] = {0, 0}, npc = 0, ncur = 0;
  uint8_t cur[3];
  int inner_at = -1;
  for (int q = 0; q < nsub; ++q) {
    const PreSub& sb = subs[q];
    int st, en;
    if (sb.c0 >= 0) {
      st = sb.c0;
    } else {
      pool[np] = sb.e0 >= 0 ? cross_pt(sb.e0, sb.S) : PrePt{2, sb.S.jp, 0, sb.S.jp, sb.S.px, sb.S.py, 0.0};
      pool[np].ct = (double)q + sb.t0;
      st = np++;
    }
    if (ncur == 0) {
      cur[ncur++] = (uint8_t)st;
      // a corner point carries the chain position of the piece end it is (a
      // corner is a piece end at most once: checked with the cycle below)
      if (st < 3) pool[st].ct = (double)q + sb.t0;
    } else if (!(pool[st].kind == 2 && pool[cur[ncur - 1]].kind == 2 && pool[st].a == pool[cur[ncur - 1]].a)) {
      pre_error(P);  // pieces do not join
      return 0;
    } else {
      --np;  // the joint is the previous end
    }
    if (sb.c1 >= 0) {
      en = sb.c1;
      pool[en].ct = (double)q + sb.t1;
    } else {
      pool[np] = sb.e1 >= 0 ? cross_pt(sb.e1, sb.S) : PrePt{2, sb.S.jq, 0, sb.S.jp, sb.S.qx, sb.S.qy, 0.0};
      pool[np].ct = (double)q + sb.t1;
      en = np++;
    }
    cur[ncur++] = (uint8_t)en;
    if (pool[en].kind != 2) {
      for (int z = 0; z < ncur; ++z) pc[npc][z] = cur[z];
      pn[npc++] = ncur;
      ncur = 0;
    }
  }
  if (ncur != 0) {  // a piece ends inside the triangle
    pre_error(P);
    return 0;
  }
  int ninner = 0;
  for (int z = 3; z < np; ++z)
    if (pool[z].kind == 2) {
      ++ninner;
      inner_at = z;
    }
  if (ninner > 1) {
    pre_error(P);
    return 0;
  }
  if (inner_at >= 0) *inner = pool[inner_at];
  // boundary cycle: the corners and the piece ends on each edge, in order
  uint8_t cyc[8];
  int8_t cpiece[8], cend[8];
  double cpos[8];
  int n = 0;
  for (int j = 0; j < 3; ++j) {
    cyc[n] = (uint8_t)j;
    cpiece[n] = -1;
    cend[n] = -1;
    cpos[n] = 3.0 * j;
    ++n;
  }
  for (int q = 0; q < npc; ++q)
    for (int end = 0; end < 2; ++end) {
      const int pi = end == 0 ? pc[q][0] : pc[q][pn[q] - 1];
      const PrePt& p = pool[pi];
      if (p.kind == 0) {
        if (cpiece[pi] >= 0) {  // two pieces at one corner
          pre_error(P);
          return 0;
        }
        cpiece[pi] = (int8_t)q;
        cend[pi] = (int8_t)end;
        continue;
      }
      double pos = -1.0;
      for (int e = 0; e < 3; ++e) {
        const PreGV& A = T.c[e];
        const PreGV& B = T.c[(e + 1) % 3];
        if (p.kind == 1 && (A.id < B.id ? A.id : B.id) == p.a && (A.id < B.id ? B.id : A.id) == p.b) {
          const double L2 = (B.x - A.x) * (B.x - A.x) + (B.y - A.y) * (B.y - A.y);
          const double t = ((p.x - A.x) * (B.x - A.x) + (p.y - A.y) * (B.y - A.y)) / L2;
          if (!(t > 0 && t < 1)) {
            pre_error(P);
            return 0;
          }
          pos = 3.0 * e + 1.0 + t;
        }
      }
      if (pos < 0.0) {  // piece end not on the triangle
        pre_error(P);
        return 0;
      }
      cyc[n] = (uint8_t)pi;
      cpiece[n] = (int8_t)q;
      cend[n] = (int8_t)end;
      cpos[n] = pos;
      ++n;
    }
  for (int a = 1; a < n; ++a)  // insertion sort by position
    for (int b = a; b > 0 && cpos[b] < cpos[b - 1]; --b) {
      const uint8_t t0 = cyc[b];
      cyc[b] = cyc[b - 1];
      cyc[b - 1] = t0;
      const int8_t t1 = cpiece[b];
      cpiece[b] = cpiece[b - 1];
      cpiece[b - 1] = t1;
      const int8_t t2 = cend[b];
      cend[b] = cend[b - 1];
      cend[b - 1] = t2;
      const double t3 = cpos[b];
      cpos[b] = cpos[b - 1];
      cpos[b - 1] = t3;
    }
  // faces: walk the cycle; at a piece end reached along the boundary, follow the piece
  uint32_t used = 0;
  for (int st = 0; st < n; ++st) {
    if ((used >> st) & 1u) continue;
    uint8_t face[16];
    int m = 0, side = -1, at = st;
    for (int guard = 0; guard < 64; ++guard) {
      if ((used >> at) & 1u) break;
      used |= 1u << at;
      if (m < 16) face[m] = cyc[at];
      ++m;
      const int nx = (at + 1) % n;
      if (cpiece[nx] >= 0) {
        const int q = cpiece[nx];
        const bool fwd = cend[nx] == 0;
        const int s2 = fwd ? 1 : 0;
        if (side >= 0 && side != s2) {  // a face on both sides of the chain
          pre_error(P);
          return 0;
        }
        side = s2;
        if (fwd) {
          for (int z = 0; z + 1 < pn[q]; ++z) {
            if (m < 16) face[m] = pc[q][z];
            ++m;
          }
        } else {
          for (int z = pn[q] - 1; z > 0; --z) {
            if (m < 16) face[m] = pc[q][z];
            ++m;
          }
        }
        int oth = -1;
        for (int z = 0; z < n; ++z)
          if (cpiece[z] == q && cend[z] != cend[nx]) oth = z;
        if (oth < 0) {
          pre_error(P);
          return 0;
        }
        at = oth;
        if (at == st) break;
        continue;
      }
      at = nx;
      if (at == st) break;
    }
    if (side != 1) continue;
    if (m < 3 || m > 16) {  // degenerate face
      pre_error(P);
      return 0;
    }
    if (kCount) {
      for (int t = 1; t + 1 < m; ++t) out(pool[face[0]], pool[face[t]], pool[face[t + 1]], 1);
      continue;
    }
    // the template rule on this foreground face
    int apex = -1;
    for (int j = 0; j < m; ++j)
      if (pool[face[j]].kind == 2) apex = j;
    if (apex < 0 && m == 4 && npc == 2) {
      bool corners = false;
      for (int j = 0; j < m; ++j) corners = corners || face[j] < 3;
      if (!corners) {
        // the middle quadrilateral between two chords: diagonal joining their exits
        const int x1 = pc[0][pn[0] - 1], x2 = pc[1][pn[1] - 1];
        for (int j = 0; j < m; ++j)
          if (face[j] == x1) apex = j;
        if (apex < 0 || face[(apex + 2) % 4] != x2) {
          pre_error(P);  // nested exits not opposite
          return 0;
        }
      }
    }
    if (apex < 0) {
      // the earliest chain point: a piece point (corners only as piece ends)
      double best = 1e300;
      for (int j = 0; j < m; ++j) {
        const int pi = face[j];
        bool in_piece = false;
        for (int q = 0; q < npc; ++q)
          for (int z = 0; z < pn[q]; ++z) in_piece = in_piece || pc[q][z] == pi;
        if (!in_piece) continue;
        if (pool[pi].ct < best) {
          best = pool[pi].ct;
          apex = j;
        }
      }
    }
    if (apex < 0) {
      pre_error(P);
      return 0;
    }
    for (int t = 1; t + 1 < m; ++t) {
      const PrePt& a = pool[face[apex]];
      const PrePt& b = pool[face[(apex + t) % m]];
      const PrePt& c = pool[face[(apex + t + 1) % m]];
      if (!((b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x) > 0.0)) pre_error(P);
      out(a, b, c, 1);
    }
  }
  return ninner;

}

// Owners whose slot triangles a segment can reach: every segment marks the
// owners whose slot box on the lattice, widened by a + b (the moves and the
// inserted vertices stay within it), meets the segment's box.  An unmarked
// owner is quiet: its triangles are uncut, its corners are lattice vertices
// off the polyline, and the inside label of the owner vertex decides them.
constexpr uint32_t kPreTouched = 64;
__device__ void pre_touch_seg(const PreArgs& P, const Geo& g, double px, double py, double qx, double qy) {
  const double r = widen(P.a + P.b) + 1e-9, hx = pre_hx(g);
  const double x0 = fmin(px, qx) - r, x1 = fmax(px, qx) + r, y0 = fmin(py, qy) - r, y1 = fmax(py, qy) + r;
  for (int k = max(0, pre_row_floor(g, y0) - 1); k <= min(g.NK - 1, pre_row_floor(g, y1)); ++k) {
    const int ia = max(0, (int)__builtin_floor(pre_col(g, k, x0 - hx)));
    const int ib = min(g.NI - 1, (int)__builtin_floor(pre_col(g, k, x1 + 0.5 * hx)) + 1);
    for (int i = ia; i <= ib; ++i) {
      const int64_t v = (int64_t)k * g.NI + i;
      if (!(P.flags[v] & kPreTouched)) pre_flag_or(P.flags, v, kPreTouched);
    }
  }
}
__global__ void __launch_bounds__(256) k_pre_mesh_touch(OneSrc src, PreArgs P) {
  __shared__ uint16_t lds[4][kPreDeal];
  const Img& d = src.d;
  const Geo g = d.g;
  PreWord W;
  const bool on = pre_word(d, g, W);
  const uint32_t cells = on ? (W.dh | W.dv | (W.cur ^ W.b1)) : 0u;
  const uint32_t base = blockIdx.x * 256u + (threadIdx.x & ~63u);
  auto cs_of = [&](int, int j) {
    return ((W.cur >> j) & 1u) | (((W.c1 >> j) & 1u) << 1) | (((W.b1 >> j) & 1u) << 2) | (((W.bel >> j) & 1u) << 3);
  };
  pre_deal(lds, cells, 0u, cs_of, [&](int sl, int, int j, uint32_t cs) {
    int R, C0;
    pre_word_at(g, base + sl, R, C0);
    const uint32_t ms = ms_case((int)cs);
    for (int q = 0; q < (int)(ms & 3u); ++q) {
      double px, py, qx, qy;
      cell_segment(g, R, C0 + j, ms, q, px, py, qx, qy);
      pre_touch_seg(P, g, px, py, qx, qy);
    }
  });
}

// The samples around owner (k, i): the box of its two slots on the lattice
// widened by a + b (every moved or inserted corner stays in it), with the
// cells the enumerations of its edges and triangles look at (one more row and
// column on each side).
__device__ __forceinline__ void pre_owner_bits(const Img& d, const Geo& g, const PreArgs& P, int k, int i, PreBits& B) {
  const double hx = pre_hx(g), lx = lat_x(g, pre_lat_X(g, k, i));
  const double r = widen(P.a + P.b) + 1e-9;
  const int R0 = floor_index(g, lat_y(g, k) - r) - 1, R1 = floor_index(g, lat_y(g, k + 1) + r) + 1;
  const int C0 = floor_index(g, lx - 0.5 * hx - r) - 1;
  pre_bits_load(d, g, R0, C0, min(6, R1 - R0 + 1), B);
}

// Grid triangle z (slot z / 2, its z % 2-th triangle) of owner (k, i).
__device__ __forceinline__ bool pre_owner_tri(const PreArgs& P, const Geo& g, int k, int i, const PreSlots& S, int z,
                                              PreGT& T) {
  PreGT TT[2];
  const int m = pre_slot_tris(P, g, k, i, S, z >> 1, TT);
  if ((z & 1) >= m) return false;
  if (z & 1)  // constant indices keep TT in registers
    T = TT[1];
  else
    T = TT[0];
  return true;
}

// The crossings of edge slot q of owner (k, i) (cq of them, by position
// along the edge from its lower-numbered end), from mesh index `first`.
__device__ void pre_slot_vertices(const Img& d, const Geo& g, const PreArgs& P, int k, int i, int q, int cq,
                                  int64_t first) {
  double2* Vout = reinterpret_cast<double2*>(P.overts);
  const PreSlots S = pre_owner_slots(P, g, k, i);
  PreBits Bits;
  pre_owner_bits(d, g, P, k, i, Bits);
  PreGV A, B;
  pre_edge_slot(P, g, k, i, S, q, A, B);
  const PreGV& L = A.id < B.id ? A : B;
  const PreGV& H = A.id < B.id ? B : A;
  double te[3], xs[3], ys[3];
  int m = 0;
  pre_edge_crossings(d, g, L, H, [&](const PreSeg& Sg, double t) {
    if (m >= 3) return;
    te[m] = t;
    pre_crossing_xy(Sg, L, H, xs[m], ys[m]);
    for (int z = m++; z > 0 && te[z - 1] > te[z]; --z) {  // by position along the edge
      const double a = te[z], bx = xs[z], by = ys[z];
      te[z] = te[z - 1];
      xs[z] = xs[z - 1];
      ys[z] = ys[z - 1];
      te[z - 1] = a;
      xs[z - 1] = bx;
      ys[z - 1] = by;
    }
  }, &Bits);
  for (int z = 0; z < cq && z < m; ++z)
    if (first + z < P.ovcap) Vout[first + z] = make_double2(xs[z], ys[z]);
}
// The polyline vertex strictly inside grid triangle z of owner (k, i), at
// mesh index `at`.
__device__ void pre_inner_vertex(const Img& d, const Geo& g, const PreArgs& P, int k, int i, int z, int64_t at) {
  const PreSlots S = pre_owner_slots(P, g, k, i);
  PreGT T;
  if (!pre_owner_tri(P, g, k, i, S, z, T)) return;
  PreBits Bits;
  pre_owner_bits(d, g, P, k, i, Bits);
  PrePt in;
  if (pre_tri_mesh<false, true>(d, g, P, T, [](const PrePt&, const PrePt&, const PrePt&, int) {}, &in, nullptr,
                                &Bits) &&
      at < P.ovcap)
    reinterpret_cast<double2*>(P.overts)[at] = make_double2(in.x, in.y);
}

// A point of a cut triangle's output in 32 bits: bits 30..31 the kind; a
// grid vertex's id (below 2^30), a crossing's triangle edge (bits 28..29) and
// segment (below 2^28), nothing for the inner polyline vertex.  False if the
// point does not fit.
__device__ __forceinline__ bool pre_ref_pack(const PreGT& T, const PrePt& p, uint32_t& r) {
  if (p.kind == 0) {
    r = (uint32_t)p.a;
    return (uint32_t)p.a < (1u << 30);
  }
  if (p.kind == 2) {
    r = 2u << 30;
    return true;
  }
  if ((uint32_t)p.s >= (1u << 28)) return false;
  for (int e = 0; e < 3; ++e) {
    const int32_t ia = pre_sel3(T.c[0].id, T.c[1].id, T.c[2].id, e);
    const int32_t ib = pre_sel3(T.c[0].id, T.c[1].id, T.c[2].id, (e + 1) % 3);
    if (min(ia, ib) == p.a && max(ia, ib) == p.b) {
      r = (1u << 30) | ((uint32_t)e << 28) | (uint32_t)p.s;
      return true;
    }
  }
  return false;
}
// The slot of cut grid triangle z of list position t in the kept outputs.
__device__ __forceinline__ int64_t pre_cut_slot(const PreArgs& P, int64_t t, int z, uint32_t rt) {
  return (int64_t)P.cbase[t] + __builtin_popcount((rt >> 28) & ((1u << z) - 1u));
}

// Output triangles of grid triangle z of a touched owner, from position pos
// (kept: the count pass's output of a cut triangle, kn triangles of point refs).
__device__ void pre_owner_triangle(const Img& d, const Geo& g, const PreArgs& P, int k, int i, int z, uint32_t rc,
                                   uint32_t rt, int64_t pos, int64_t NV, const uint32_t* kept = nullptr, int kn = 0) {
  const int64_t v = (int64_t)k * g.NI + i;
  const PreSlots S = pre_owner_slots(P, g, k, i);
  PreBits Bits;
  pre_owner_bits(d, g, P, k, i, Bits);
  PreGT TT;
  if (!pre_owner_tri(P, g, k, i, S, z, TT)) return;
  const int64_t vbase = (pre_rc_before(rc, 8) + pre_rc_inner(rc)) ? P.rbase[v] : 0;
  const int64_t inner_id = NV + vbase + pre_rc_before(rc, 8) + __builtin_popcount((rt >> 24) & ((1u << z) - 1u));
  // per edge of the triangle: its owner's first crossing id and the
  // crossings' segments in order along the edge (at most three)
  int64_t ebase[3];
  int32_t eseg[3][3];
  int ecnt[3];
  for (int e = 0; e < 3; ++e) {
    const PreGV& A = TT.c[e];
    const PreGV& B = TT.c[(e + 1) % 3];
    const PreGV& L = A.id < B.id ? A : B;
    const PreGV& H = A.id < B.id ? B : A;
    const uint32_t rw = P.rcount[TT.eo[e]];
    ecnt[e] = pre_rc_cross(rw, TT.es[e]);
    ebase[e] = 0;
    if (!ecnt[e]) continue;
    ebase[e] = NV + P.rbase[TT.eo[e]] + pre_rc_before(rw, TT.es[e]);
    double te[3];
    int m = 0;
    pre_edge_crossings(d, g, L, H, [&](const PreSeg& Sg, double t) {
      if (m >= 3) return;
      te[m] = t;
      eseg[e][m] = Sg.jp;
      for (int z = m++; z > 0 && te[z - 1] > te[z]; --z) {
        const double t1 = te[z];
        te[z] = te[z - 1];
        te[z - 1] = t1;
        const int32_t s1 = eseg[e][z];
        eseg[e][z] = eseg[e][z - 1];
        eseg[e][z - 1] = s1;
      }
    }, &Bits);
    if (m != ecnt[e]) pre_error(P);
    ecnt[e] = min(m, ecnt[e]);
  }
  auto id_of = [&](const PrePt& p) -> int64_t {
    if (p.kind == 0) return P.vmap[p.a];
    if (p.kind == 2) return inner_id;
    for (int e = 0; e < 3; ++e) {
      const int64_t lo = TT.c[e].id < TT.c[(e + 1) % 3].id ? TT.c[e].id : TT.c[(e + 1) % 3].id;
      const int64_t hi = TT.c[e].id < TT.c[(e + 1) % 3].id ? TT.c[(e + 1) % 3].id : TT.c[e].id;
      if (lo != p.a || hi != p.b) continue;
      for (int r = 0; r < ecnt[e]; ++r)
        if (eseg[e][r] == p.s) return ebase[e] + r;
    }
    pre_error(P);
    return 0;
  };
  if (kept) {  // the count pass's output: ids from the point refs
    auto ref_id = [&](uint32_t r) -> int64_t {
      const uint32_t kind = r >> 30;
      if (kind == 0) return P.vmap[r & 0x3fffffffu];
      if (kind == 2) return inner_id;
      const int e = (int)((r >> 28) & 3u);
      const int32_t sg = (int32_t)(r & 0x0fffffffu);
      const int ne = pre_sel3(ecnt[0], ecnt[1], ecnt[2], e);
      for (int q = 0; q < ne; ++q) {
        const int32_t sq = e == 0 ? eseg[0][q] : (e == 1 ? eseg[1][q] : eseg[2][q]);
        if (sq == sg) return pre_sel3(ebase[0], ebase[1], ebase[2], e) + q;
      }
      pre_error(P);
      return 0;
    };
    for (int j = 0; j < kn; ++j, ++pos) {
      if (pos >= P.otcap) continue;
      int32_t* o = P.otris + 3 * pos;
      o[0] = (int32_t)ref_id(kept[3 * j]);
      o[1] = (int32_t)ref_id(kept[3 * j + 1]);
      o[2] = (int32_t)ref_id(kept[3 * j + 2]);
      P.ocodes[pos] = 1;
    }
    return;
  }
  PrePt in;
  (void)pre_tri_mesh(d, g, P, TT, [&](const PrePt& a, const PrePt& b, const PrePt& c, int code) {
    if (pos < P.otcap) {
      int32_t* o = P.otris + 3 * pos;
      o[0] = (int32_t)id_of(a);
      o[1] = (int32_t)id_of(b);
      o[2] = (int32_t)id_of(c);
      P.ocodes[pos] = (uint8_t)code;
    }
    ++pos;
  }, &in, nullptr, &Bits);
}


// The touched owners of each row segment (their list offsets come from a scan).
__global__ void __launch_bounds__(256) k_pre_mesh_tcount(OneSrc src, PreArgs P, Shared sh) {
  const Geo g = src.d.g;
  int64_t seg;
  int k, i0;
  if (!pre_segment(g, sh, seg, k, i0)) return;  // wave-uniform
  const int lane = threadIdx.x & 63;
  int n = 0;
  for (int j = 0; j < 4; ++j) {
    const int i = i0 + 64 * j + lane;
    n += (int)__popcll(__ballot(i < g.NI && (P.flags[(int64_t)k * g.NI + i] & kPreTouched)));
  }
  if (lane == 0) {
    sh.seg_cnt[seg] = make_int4(n, 0, 0, 0);
    sh.seg_slow[seg] = 0ull;
  }
}

// Quiet owners in place (their slots kept whole when the owner vertex is
// inside); the touched ones go to the list at their segment's offset, their
// counts cleared for the dense pass.
__global__ void __launch_bounds__(256) k_pre_mesh_count(OneSrc src, PreArgs P, Shared sh) {
  const Img& d = src.d;
  const Geo g = d.g;
  int64_t seg;
  int k, i0;
  if (!pre_segment(g, sh, seg, k, i0)) return;  // wave-uniform
  const int lane = threadIdx.x & 63;
  const double y = lat_y(g, k);
  int64_t at = sh.seg_off[seg].x;
  for (int j = 0; j < 4; ++j) {
    const int i = i0 + 64 * j + lane;
    const int64_t v = (int64_t)k * g.NI + i;
    const bool touched = i < g.NI && (P.flags[v] & kPreTouched);
    const unsigned long long bal = __ballot(touched);
    if (touched) {
      P.tlist[at + lanes_below(bal)] = (int32_t)v;
      P.rcount[v] = 0u;
      P.rtri[v] = 0u;
    } else if (i < g.NI) {
      const int nt = pre_inside_point(d, g, lat_x(g, pre_lat_X(g, k, i)), y)
                         ? (int)pre_slot_ok(g, k, i, 0) + (int)pre_slot_ok(g, k, i, 1)
                         : 0;
      P.rcount[v] = (uint32_t)nt << 19;
      if (nt) {  // the corners of its slots are in the mesh
        const int o = k & 1;
        P.used[v] = 1;
        if (pre_slot_ok(g, k, i, 0)) {
          P.used[(int64_t)(k + 1) * g.NI + (i + o)] = 1;
          P.used[(int64_t)(k + 1) * g.NI + (i + o - 1)] = 1;
        }
        if (pre_slot_ok(g, k, i, 1)) {
          P.used[v + 1] = 1;
          P.used[(int64_t)(k + 1) * g.NI + (i + o)] = 1;
        }
      }
    }
    at += (int64_t)__popcll(bal);
  }
}

// Work over n items in chunks of a block (a grid-stride loop): light(item)
// runs each item and returns true to put it off; put-off items are gathered
// in LDS and run by heavy(item) on full blocks, the rest at the end.  dl
// holds 2 * 256 entries; *nd starts at 0.
template <class Light, class Heavy>
__device__ __forceinline__ void pre_dense(int64_t n, int64_t* dl, int* nd, Light light, Heavy heavy) {
  for (int64_t base = (int64_t)blockIdx.x * 256;; base += (int64_t)gridDim.x * 256) {
    const bool more = base < n;  // uniform
    if (more) {
      const int64_t it = base + threadIdx.x;
      if (it < n && light(it)) dl[atomicAdd(nd, 1)] = it;
    }
    __syncthreads();
    int m = *nd;
    while (m >= 256 || (!more && m > 0)) {  // uniform
      const int take = m >= 256 ? 256 : m;
      if ((int)threadIdx.x < take) heavy(dl[m - take + threadIdx.x]);
      m -= take;
      __syncthreads();
    }
    if (threadIdx.x == 0) *nd = m;
    __syncthreads();
    if (!more) break;
  }
}
__device__ __forceinline__ void pre_tl_owner(const Geo& g, const PreArgs& P, int64_t t, int& k, int& i) {
  const uint32_t v = (uint32_t)P.tlist[t];
  const uint32_t kk = v / (uint32_t)g.NI;
  k = (int)kk;
  i = (int)(v - kk * (uint32_t)g.NI);
}

// Counts of a cut grid triangle of a touched owner (item t * 4 + z of the
// list): subdivision and template; triangles, inner vertex and the cut are
// added to the owner's words, and up to kPreKeep output triangles are kept in
// the triangle's slot for the triangle pass.
__device__ __forceinline__ void pre_mesh_cut_tri_count(const Img& d, const Geo& g, const PreArgs& P, int64_t t, int z) {
  int kk, ii;
  pre_tl_owner(g, P, t, kk, ii);
  const PreSlots S = pre_owner_slots(P, g, kk, ii);
  PreGT Tg;
  if (!pre_owner_tri(P, g, kk, ii, S, z, Tg)) return;
  PreBits Bits;
  pre_owner_bits(d, g, P, kk, ii, Bits);
  int nt = 0;
  PrePt in;
  bool cut = false;
  // the output is kept for the triangle pass when it fits its slot
  const uint32_t rt0 = P.rtri[(int64_t)kk * g.NI + ii];
  const int64_t slot = pre_cut_slot(P, t, z, rt0);
  uint32_t* kept = slot < P.ccap ? P.cstore + slot * (1 + 3 * kPreKeep) : nullptr;
  bool keep = kept != nullptr;
  const int nin = pre_tri_mesh(d, g, P, Tg, [&](const PrePt& a, const PrePt& b, const PrePt& c, int) {
    if (keep && nt < kPreKeep) {
      uint32_t ra, rb, rc;
      keep = pre_ref_pack(Tg, a, ra) && pre_ref_pack(Tg, b, rb) && pre_ref_pack(Tg, c, rc);
      kept[1 + 3 * nt] = ra;
      kept[2 + 3 * nt] = rb;
      kept[3 + 3 * nt] = rc;
    } else {
      keep = false;
    }
    ++nt;
    if (a.kind == 0) P.used[a.a] = 1;
    if (b.kind == 0) P.used[b.a] = 1;
    if (c.kind == 0) P.used[c.a] = 1;
  }, &in, &cut, &Bits);
  if (kept) kept[0] = keep ? (uint32_t)nt : kPreNotKept;
  if (nt > 63) {
    pre_error(P);
    nt = 63;
  }
  const int64_t v = (int64_t)kk * g.NI + ii;
  const uint32_t bits = ((uint32_t)nt << (6 * z)) | ((uint32_t)(nin ? 1 : 0) << (24 + z)) |
                        ((uint32_t)(cut ? 1 : 0) << (28 + z));
  if (bits) atomicOr(&P.rtri[v], bits);
  const uint32_t add = ((uint32_t)(nin ? 1 : 0) << 16) | ((uint32_t)nt << 19) | ((uint32_t)(cut ? 1 : 0) << 27);
  if (add) atomicAdd(&P.rcount[v], add);
}

// Counts of the touched owners, one lane per owner: its flags, slots and
// raster words are loaded once for its four grid triangles (the candidate
// segments clipped: an uncut triangle is counted, one triangle when in the
// foreground; a cut one gets its cut bit and is counted by
// k_pre_mesh_cut_count) and its eight edge slots (crossings); its words are
// written without atomics.  It takes 165 VGPRs (three waves per SIMD):
// held to 128 it spills and runs 7 % slower.
__global__ void __launch_bounds__(256) k_pre_mesh_probe_owner(OneSrc src, PreArgs P, Shared sh) {
  const Img& d = src.d;
  const Geo g = d.g;
  const int64_t T = sh.seg_off[sh.nseg].x;  // touched owners
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < T; t += (int64_t)gridDim.x * 256) {
    int kk, ii;
    pre_tl_owner(g, P, t, kk, ii);
    const int64_t v = (int64_t)kk * g.NI + ii;
    const PreSlots S = pre_owner_slots(P, g, kk, ii);
    PreBits Bits;
    pre_owner_bits(d, g, P, kk, ii, Bits);
    uint32_t rt = 0, rc = 0;
    for (int z = 0; z < 4; ++z) {
      PreGT Tg;
      if (!pre_owner_tri(P, g, kk, ii, S, z, Tg)) continue;
      int nt = 0;
      PrePt in;
      bool cut = false;
      const int nin = pre_tri_mesh<true>(d, g, P, Tg, [&](const PrePt& a, const PrePt& b, const PrePt& c, int) {
        ++nt;
        if (a.kind == 0) P.used[a.a] = 1;
        if (b.kind == 0) P.used[b.a] = 1;
        if (c.kind == 0) P.used[c.a] = 1;
      }, &in, &cut, &Bits);
      if (nin < 0) {  // cut: k_pre_mesh_cut_count takes it
        rt |= 1u << (28 + z);
        continue;
      }
      rt |= (uint32_t)nt << (6 * z);  // uncut: at most one triangle, no inner vertex
      rc += (uint32_t)nt << 19;
    }
    for (int e = 0; e < 8; ++e) {
      PreGV A, B;
      if (!pre_edge_slot(P, g, kk, ii, S, e, A, B)) continue;
      int c = 0;
      pre_edge_crossings(d, g, A, B, [&](const PreSeg&, double) { ++c; }, &Bits);
      if (c > 3) {  // more crossings of one grid edge than the numbering holds
        pre_error(P);
        c = 3;
      }
      rc |= (uint32_t)c << (2 * e);
    }
    P.rtri[v] = rt;
    P.rcount[v] = rc;
  }
}

// Exclusive scan in place of nblk block counts by one block; *total (if
// given) receives their sum.
__device__ __forceinline__ void pre_scan_blocks(int64_t* a, int64_t nblk, int64_t* total) {
  __shared__ int64_t part[4];
  int64_t run = 0;
  for (int64_t b = 0; b < nblk; b += 256) {
    const int64_t j = b + threadIdx.x;
    const int64_t x = j < nblk ? a[j] : 0;
    // block-wide exclusive scan of 256 int64 values (four waves of 64)
    int64_t incl = x;
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t y = __shfl_up(incl, off);
      if ((int)(threadIdx.x & 63) >= off) incl += y;
    }
    if ((threadIdx.x & 63) == 63) part[threadIdx.x >> 6] = incl;
    __syncthreads();
    int64_t before = run;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) before += part[w];
    if (j < nblk) a[j] = before + incl - x;
    run += part[0] + part[1] + part[2] + part[3];
    __syncthreads();
  }
  if (total && threadIdx.x == 0) *total = run;
}
// Slots of the cut grid triangles' kept outputs, in list order: per block of
// kPreVScan list positions the number of cut triangles; one block scans the
// counts; then each position's first slot (clamped to 32 bits: slots past the
// capacity keep nothing).
__device__ __forceinline__ int pre_cut_n(const PreArgs& P, int64_t t, int64_t T) {
  return t < T ? __builtin_popcount(P.rtri[P.tlist[t]] >> 28) : 0;
}
__global__ void __launch_bounds__(256) k_pre_cut_count(PreArgs P, Shared sh) {
  __shared__ int part[4];
  const int64_t T = sh.seg_off[sh.nseg].x;
  const int64_t b0 = (int64_t)blockIdx.x * kPreVScan;
  int n = 0;
  for (int q = threadIdx.x; q < kPreVScan && b0 < T; q += 256) n += pre_cut_n(P, b0 + q, T);
  const int w = __builtin_amdgcn_readlane(wave_incl_scan_dpp(n), 63);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) P.cblk[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}
__global__ void __launch_bounds__(256) k_pre_cut_top(PreArgs P, int64_t nblk) { pre_scan_blocks(P.cblk, nblk, nullptr); }
__global__ void __launch_bounds__(256) k_pre_cut_apply(PreArgs P, Shared sh) {
  __shared__ int part[4];
  const int64_t T = sh.seg_off[sh.nseg].x;
  const int64_t b0 = (int64_t)blockIdx.x * kPreVScan;
  if (b0 >= T) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t run = P.cblk[blockIdx.x];
  for (int c = 0; c < kPreVScan / 256; ++c) {
    const int64_t t = b0 + (int64_t)c * 256 + threadIdx.x;
    const int n = pre_cut_n(P, t, T);
    const int incl = wave_incl_scan_dpp(n);
    if (lane == 63) part[wv] = incl;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int tw = part[w];
      before += w < wv ? tw : 0;
      tot += tw;
    }
    if (t < T) P.cbase[t] = (int32_t)min(run + before + incl - n, (int64_t)0x7fffffff);
    run += tot;
    __syncthreads();
  }
}

// The cut grid triangles (cut bit set, no count yet), gathered per block and
// retriangulated on full blocks.  The retriangulating kernels are held to
// 128 VGPRs (four waves per SIMD): spilling more to scratch costs less than
// the latency two waves per SIMD leave uncovered.
__global__ void __launch_bounds__(256, 4) k_pre_mesh_cut_count(OneSrc src, PreArgs P, Shared sh) {
  __shared__ int64_t dl[512];
  __shared__ int nd;
  const Img& d = src.d;
  const Geo g = d.g;
  if (threadIdx.x == 0) nd = 0;
  __syncthreads();
  const int64_t T = sh.seg_off[sh.nseg].x;
  pre_dense(4 * T, dl, &nd, [&](int64_t it) -> bool {
    return (P.rtri[P.tlist[it >> 2]] >> (28 + (it & 3))) & 1u;
  }, [&](int64_t it) { pre_mesh_cut_tri_count(d, g, P, it >> 2, (int)(it & 3)); });
}

// Per row segment: new vertices, triangles and cut grid triangles of its
// owners, the input of the scan; counts[3] keeps the number of touched owners.
__global__ void __launch_bounds__(256) k_pre_mesh_segsum(OneSrc src, PreArgs P, Shared sh) {
  const Geo g = src.d.g;
  if (blockIdx.x == 0 && threadIdx.x == 0) P.counts[3] = sh.seg_off[sh.nseg].x;
  int64_t seg;
  int k, i0;
  if (!pre_segment(g, sh, seg, k, i0)) return;  // wave-uniform
  const int lane = threadIdx.x & 63;
  int nv = 0, nt = 0, nc = 0;
  for (int j = 0; j < 4; ++j) {
    const int i = i0 + 64 * j + lane;
    const uint32_t rc = i < g.NI ? P.rcount[(int64_t)k * g.NI + i] : 0u;
    nv += pre_rc_before(rc, 8) + pre_rc_inner(rc);
    nt += pre_rc_tris(rc);
    nc += pre_rc_cut(rc);
  }
  nv = __builtin_amdgcn_readlane(wave_incl_scan_dpp(nv), 63);
  nt = __builtin_amdgcn_readlane(wave_incl_scan_dpp(nt), 63);
  nc = __builtin_amdgcn_readlane(wave_incl_scan_dpp(nc), 63);
  if (lane == 0) {
    sh.seg_cnt[seg] = make_int4(nv, nt, nc, 0);
    sh.seg_slow[seg] = 0ull;
  }
}

// New vertices: the crossings of each owned edge slot in order from its
// lower-numbered end, then the polyline vertices inside the owner's
// triangles; each owner with new vertices records its first index (rbase,
// relative to the grid vertices kept).
__global__ void __launch_bounds__(256) k_pre_mesh_vbase(OneSrc src, PreArgs P, Shared sh) {
  const Geo g = src.d.g;
  int64_t seg;
  int k, i0;
  if (!pre_segment(g, sh, seg, k, i0) || sh.seg_cnt[seg].x == 0) return;  // wave-uniform
  const int lane = threadIdx.x & 63;
  int64_t acc = sh.seg_off[seg].x;
  for (int j = 0; j < 4; ++j) {
    const int i = i0 + 64 * j + lane;
    const int64_t v = (int64_t)k * g.NI + i;
    const uint32_t rc = i < g.NI ? P.rcount[v] : 0u;
    const int n = pre_rc_before(rc, 8) + pre_rc_inner(rc);
    const int incl = wave_incl_scan_dpp(n);
    if (n) P.rbase[v] = acc + (incl - n);
    acc += __builtin_amdgcn_readlane(incl, 63);
  }
}
// The crossings, one item per edge slot of the touched owners; the slots with
// crossings are gathered per block and done on full blocks.
__global__ void __launch_bounds__(256) k_pre_mesh_edge_verts(OneSrc src, PreArgs P) {
  __shared__ int64_t dl[512];
  __shared__ int nd;
  const Img& d = src.d;
  const Geo g = d.g;
  if (threadIdx.x == 0) nd = 0;
  __syncthreads();
  const int64_t T = P.counts[3];
  const int64_t NV = *P.nused;
  pre_dense(8 * T, dl, &nd, [&](int64_t e8) -> bool {
    return pre_rc_cross(P.rcount[P.tlist[e8 >> 3]], (int)(e8 & 7)) != 0;
  }, [&](int64_t e8) {
    int kk, ii;
    pre_tl_owner(g, P, e8 >> 3, kk, ii);
    const int q = (int)(e8 & 7);
    const int64_t v = (int64_t)kk * g.NI + ii;
    const uint32_t rc = P.rcount[v];
    pre_slot_vertices(d, g, P, kk, ii, q, pre_rc_cross(rc, q), NV + P.rbase[v] + pre_rc_before(rc, q));
  });
}
// The inner polyline vertices, one item per grid triangle of the touched
// owners; those with one are gathered per block and found on full blocks.
__global__ void __launch_bounds__(256, 4) k_pre_mesh_inner_verts(OneSrc src, PreArgs P) {
  __shared__ int64_t dl[512];
  __shared__ int nd;
  const Img& d = src.d;
  const Geo g = d.g;
  if (threadIdx.x == 0) nd = 0;
  __syncthreads();
  const int64_t T = P.counts[3];
  const int64_t NV = *P.nused;
  pre_dense(4 * T, dl, &nd, [&](int64_t it) -> bool {
    return (P.rtri[P.tlist[it >> 2]] >> (24 + (it & 3))) & 1u;
  }, [&](int64_t it) {
    int kk, ii;
    pre_tl_owner(g, P, it >> 2, kk, ii);
    const int z = (int)(it & 3);
    const int64_t v = (int64_t)kk * g.NI + ii;
    const uint32_t rc = P.rcount[v], rt = P.rtri[v];
    const int64_t at = NV + P.rbase[v] + pre_rc_before(rc, 8) + __builtin_popcount((rt >> 24) & ((1u << z) - 1u));
    pre_inner_vertex(d, g, P, kk, ii, z, at);
  });
}

// Output triangles at their offsets, with their codes: a quiet owner's slots
// as they are (code 0); a touched owner's first output triangle is recorded
// for the dense pass.  The 64 owners of a wave step hold consecutive output
// ranges: their triangles are staged in LDS by rank and lane j writes ranks j
// and j + 64 (a touched owner's ranks are left to the dense pass).
__global__ void __launch_bounds__(256) k_pre_mesh_triangles(OneSrc src, PreArgs P, Shared sh) {
  __shared__ Tri3 stage[4][128];
  __shared__ uint8_t full[4][128];
  const Geo g = src.d.g;
  int64_t seg;
  int k, i0;
  if (!pre_segment(g, sh, seg, k, i0)) return;  // wave-uniform
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t t0 = sh.seg_off[seg].y;
  const int o = k & 1;
  int acc = 0;
  for (int j = 0; j < 4; ++j) {
    const int i = i0 + 64 * j + lane;
    const int64_t v = (int64_t)k * g.NI + i;
    const uint32_t rc = i < g.NI ? P.rcount[v] : 0u;
    const int n = pre_rc_tris(rc);
    const int incl = wave_incl_scan_dpp(n);
    const int tot = __builtin_amdgcn_readlane(incl, 63);  // at most 4 * 64 (a touched owner: 4 * 63)
    const bool touched = n > 0 && (P.flags[v] & kPreTouched);
    if (touched) P.rtbase[v] = t0 + acc + (incl - n);
    for (int b = 0; b < tot; b += 128) {  // uniform
      full[wv][lane] = full[wv][lane + 64] = 0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (n > 0 && !touched) {
        int r = incl - n - b;
        for (int t = 0; t < 2; ++t) {
          if (!pre_slot_ok(g, k, i, t)) continue;
          if (r >= 0 && r < 128) {
            const int64_t c1 = t == 0 ? (int64_t)(k + 1) * g.NI + (i + o) : v + 1;
            const int64_t c2 = t == 0 ? (int64_t)(k + 1) * g.NI + (i + o - 1) : (int64_t)(k + 1) * g.NI + (i + o);
            Tri3 t3;
            t3.a = P.vmap[v];
            t3.b = P.vmap[c1];
            t3.c = P.vmap[c2];
            stage[wv][r] = t3;
            full[wv][r] = 1;
          }
          ++r;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = lane + 64 * h;
        const int64_t pos = t0 + acc + b + r;
        if (full[wv][r] && pos < P.otcap) {
          *reinterpret_cast<Tri3*>(P.otris + 3 * pos) = stage[wv][r];
          P.ocodes[pos] = 0;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    acc += tot;
  }
}

// Triangles of the touched owners, one item per grid triangle: an uncut one
// (in the foreground) is written as it is; the cut ones are retriangulated by
// k_pre_mesh_cut_tris.
__global__ void __launch_bounds__(256) k_pre_mesh_whole_tris(OneSrc src, PreArgs P) {
  const Geo g = src.d.g;
  const int64_t T = P.counts[3];
  for (int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x; it < 4 * T; it += (int64_t)gridDim.x * 256) {
    int kk, ii;
    pre_tl_owner(g, P, it >> 2, kk, ii);
    const int z = (int)(it & 3);
    const int64_t v = (int64_t)kk * g.NI + ii;
    const uint32_t rt = P.rtri[v];
    if (!((rt >> (6 * z)) & 63u) || ((rt >> (28 + z)) & 1u)) continue;
    int before = 0;
    for (int z2 = 0; z2 < z; ++z2) before += (int)((rt >> (6 * z2)) & 63u);
    const int64_t pos = P.rtbase[v] + before;
    const PreSlots S = pre_owner_slots(P, g, kk, ii);
    PreGT Tg;
    if (!pre_owner_tri(P, g, kk, ii, S, z, Tg)) continue;
    if (pos < P.otcap) {
      int32_t* o = P.otris + 3 * pos;
      o[0] = P.vmap[Tg.c[0].id];
      o[1] = P.vmap[Tg.c[1].id];
      o[2] = P.vmap[Tg.c[2].id];
      P.ocodes[pos] = 0;
    }
  }
}
__global__ void __launch_bounds__(256, 4) k_pre_mesh_cut_tris(OneSrc src, PreArgs P) {
  __shared__ int64_t dl[512];
  __shared__ int nd;
  const Img& d = src.d;
  const Geo g = d.g;
  if (threadIdx.x == 0) nd = 0;
  __syncthreads();
  const int64_t T = P.counts[3];
  const int64_t NV = *P.nused;
  pre_dense(4 * T, dl, &nd, [&](int64_t it) -> bool {
    const uint32_t rt = P.rtri[P.tlist[it >> 2]];
    const int z = (int)(it & 3);
    return ((rt >> (6 * z)) & 63u) && ((rt >> (28 + z)) & 1u);
  }, [&](int64_t it) {
    int kk, ii;
    pre_tl_owner(g, P, it >> 2, kk, ii);
    const int z = (int)(it & 3);
    const int64_t v = (int64_t)kk * g.NI + ii;
    const uint32_t rt = P.rtri[v];
    int before = 0;
    for (int z2 = 0; z2 < z; ++z2) before += (int)((rt >> (6 * z2)) & 63u);
    const int64_t slot = pre_cut_slot(P, it >> 2, z, rt);
    const uint32_t* kept = slot < P.ccap ? P.cstore + slot * (1 + 3 * kPreKeep) : nullptr;
    const uint32_t kn = kept ? kept[0] : kPreNotKept;
    if (kn != kPreNotKept && kn == ((rt >> (6 * z)) & 63u))
      pre_owner_triangle(d, g, P, kk, ii, z, P.rcount[v], rt, P.rtbase[v] + before, NV, kept + 1, (int)kn);
    else  // not kept: retriangulated again
      pre_owner_triangle(d, g, P, kk, ii, z, P.rcount[v], rt, P.rtbase[v] + before, NV);
  });
}

// Compaction of the grid vertices: the used ones keep their order.  Per block
// of kPreVScan grid vertices (of the NV the grid phase made): the used count;
// one block scans the counts; then each block numbers its used vertices and
// copies them into the mesh.
__global__ void __launch_bounds__(256) k_pre_vscan_count(PreArgs P) {
  __shared__ int part[4];
  const int64_t NV = P.gsizes[0] < P.usedcap ? P.gsizes[0] : P.usedcap;
  const int64_t b0 = (int64_t)blockIdx.x * kPreVScan;
  // four flags (bytes 0 or 1) per word, sixteen words per thread
  const uint32_t* u4 = reinterpret_cast<const uint32_t*>(P.used);
  int n = 0;
  for (int q = 0; q < kPreVScan / 1024; ++q) {
    const int64_t at = b0 + 4 * ((int64_t)q * 256 + threadIdx.x);
    if (at >= NV) break;
    uint32_t w = u4[at >> 2];
    if (NV - at < 4) w &= (1u << (8 * (NV - at))) - 1u;
    n += __builtin_popcount(w);
  }
  const int w = __builtin_amdgcn_readlane(wave_incl_scan_dpp(n), 63);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) P.vbsum[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}
__global__ void __launch_bounds__(256) k_pre_vscan_top(PreArgs P, int64_t nblk) { pre_scan_blocks(P.vbsum, nblk, P.nused); }
__global__ void __launch_bounds__(256) k_pre_vscan_apply(PreArgs P) {
  __shared__ int part[16][4];
  const int64_t NV = P.gsizes[0] < P.usedcap ? P.gsizes[0] : P.usedcap;
  const int64_t b0 = (int64_t)blockIdx.x * kPreVScan;
  if (b0 >= NV) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double2* G = reinterpret_cast<const double2*>(P.verts);
  double2* O = reinterpret_cast<double2*>(P.overts);
  int64_t run = P.vbsum[blockIdx.x];
  // rounds of 256 consecutive vertices, sixteen rounds per chunk: the ballots
  // of a chunk, the waves' counts in LDS, then the ids
  for (int c = 0; c < kPreVScan / 4096; ++c) {
    unsigned long long bal[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int64_t v = b0 + (int64_t)(16 * c + q) * 256 + threadIdx.x;
      bal[q] = __ballot(v < NV && P.used[v]);
      if (lane == 0) part[q][wv] = (int)__popcll(bal[q]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      int before = 0, tot = 0;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int tw = part[q][w];
        before += w < wv ? tw : 0;
        tot += tw;
      }
      const int64_t v = b0 + (int64_t)(16 * c + q) * 256 + threadIdx.x;
      if ((bal[q] >> lane) & 1ull) {
        const int64_t id = run + before + lanes_below(bal[q]);
        P.vmap[v] = (int32_t)id;
        if (id < P.ovcap) O[id] = G[v];
      }
      run += tot;
    }
    __syncthreads();
  }
}

__global__ void k_pre_mesh_sizes(PreArgs P, Shared sh, int64_t* out) {
  const longlong4 tot = sh.seg_off[sh.nseg];
  const int64_t NV = *P.nused;
  out[0] = NV + tot.x;        // vertices
  out[1] = tot.y;             // triangles
  out[2] = P.gsizes[2];       // snapped
  out[3] = P.gsizes[3];       // repelled
  out[4] = P.gsizes[4];       // inserted
  out[6] = NV;                // grid vertices in the mesh
  out[7] = tot.z;             // cut grid triangles
  int64_t st = P.gsizes[5];
  if (st == SBMT_OK || st == SBMT_E_CAPACITY) {
    if (P.counts[2]) st = SBMT_E_PROTOCOL;
    else if (out[0] > P.ovcap || out[1] > P.otcap) st = SBMT_E_CAPACITY;
    else st = SBMT_OK;
  }
  if (out[0] > 0x7fffffffLL) st = SBMT_E_INDEX_OVERFLOW;
  out[5] = st;
}

// Workspace of the preprocessing: the meshing layout of the image, then the
// per-midpoint words, the per-owner split sides, flags and first inserted
// indices, and the counters and sizes.
struct PreLayout {
  CallLayout L;
  size_t off_mid, off_split, off_flags, off_ins, off_counts, off_out, off_snap, total;
  // the retriangulation (sbmt_preprocess_mesh): grid on-polyline bytes, per-owner counts and bases, sizes
  size_t off_onp, off_rcount, off_rtri, off_rbase, off_out2, off_gverts, off_used, off_vmap, off_vbsum, off_nused,
      off_tlist, off_rtbase, off_cbase, off_cblk, off_cstore;
  int64_t ncblk, ccap;  // blocks of the cut scan; cut triangles whose output is kept
  int64_t nvblk;  // blocks of the vertex compaction scan
  int64_t nmid, nown;
};
static sbmt_status pre_layout(const sbmt_image* img, bool need_ptr, PreLayout* P, bool mesh = false) {
  sbmt_status st = make_call_layout(img, 1, 0, need_ptr, &P->L);
  if (st != SBMT_OK) return st;
  const Geo& g = P->L.g[0];
  P->nmid = 2LL * (g.CH + 2) * (g.CW + 2);
  P->nown = (int64_t)g.NK * g.NI;
  if (P->nmid >= (1LL << 31)) return SBMT_E_INVALID_ARG;  // midpoint ids are int32
  size_t off = align256(P->L.total);
  P->off_mid = off;
  off = align256(off + (size_t)P->nmid);
  P->off_split = off;
  off = align256(off + (size_t)P->nown * 12);
  P->off_flags = off;
  off = align256(off + (size_t)P->nown);
  P->off_ins = off;
  off = align256(off + (size_t)P->nown * 8);
  P->off_counts = off;
  off = align256(off + kPreCounts * 8);
  P->off_out = off;
  off = align256(off + 8 * 8);
  P->off_snap = off;
  off = align256(off + (size_t)P->nown * 4);
  P->off_onp = P->off_rcount = P->off_rtri = P->off_rbase = P->off_out2 = 0;
  P->off_gverts = P->off_used = P->off_vmap = P->off_vbsum = P->off_nused = P->off_tlist = P->off_rtbase = 0;
  P->off_cbase = P->off_cblk = P->off_cstore = 0;
  P->ncblk = P->ccap = 0;
  P->nvblk = 0;
  if (mesh) {
    P->off_onp = off;
    off = align256(off + (size_t)(P->nown + P->nmid));
    P->off_rcount = off;
    off = align256(off + (size_t)P->nown * 4);
    P->off_rtri = off;
    off = align256(off + (size_t)P->nown * 4);
    P->off_rbase = off;
    off = align256(off + (size_t)P->nown * 8);
    P->off_out2 = off;
    off = align256(off + 8 * 8);
    const int64_t ng = P->nown + P->nmid;  // bound on the grid vertices
    P->nvblk = (ng + kPreVScan - 1) / kPreVScan;
    P->off_gverts = off;
    off = align256(off + (size_t)ng * 16);
    P->off_used = off;
    off = align256(off + (size_t)ng);
    P->off_vmap = off;
    off = align256(off + (size_t)ng * 4);
    P->off_vbsum = off;
    off = align256(off + (size_t)P->nvblk * 8);
    P->off_nused = off;
    off = align256(off + 8);
    P->off_tlist = off;
    off = align256(off + (size_t)P->nown * 4);
    P->off_rtbase = off;
    off = align256(off + (size_t)P->nown * 8);
    // kept outputs of the cut grid triangles: room for one in 16 owners
    P->ncblk = (P->nown + kPreVScan - 1) / kPreVScan;
    P->ccap = std::max<int64_t>(65536, P->nown / 16);
    P->off_cbase = off;
    off = align256(off + (size_t)P->nown * 4);
    P->off_cblk = off;
    off = align256(off + (size_t)P->ncblk * 8);
    P->off_cstore = off;
    off = align256(off + (size_t)P->ccap * (1 + 3 * kPreKeep) * 4);
  }
  P->total = off;
  return SBMT_OK;
}
static bool pre_thresholds_ok(double a, double b, double c, double h) {
  if (!(a >= 0 && b >= 0 && c >= 0)) return false;
  if (a == 0 && b == 0 && c == 0) return true;
  return b < a / 2 && c * c < a * a / 2 && a < h / 2;
}
