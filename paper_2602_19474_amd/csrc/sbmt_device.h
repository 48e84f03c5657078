// Per-owner classification and emission of the SBMT hot path (gfx950 kernels).
//
// Every lattice vertex (k, i) of the equilateral grid "owns" its three
// forward edges E0 -> (k,i+1), E1 -> (k+1,i+o-1), E2 -> (k+1,i+o)
// (o = k mod 2) and two base triangles
//   Tb = [v(k,i), v(k+1,i+o), v(k+1,i+o-1)]  (apex on row k)
//   Ta = [v(k,i), v(k,i+1),   v(k+1,i+o)]    (base on row k),
// whose other edges are E3 = v(k,i+1) -> v(k+1,i+o) and
// E4 = v(k+1,i+o-1) -> v(k+1,i+o).  One thread classifies one owner:
//   fast path  the 3x3 coarse samples under Tb u Ta are uniform: no boundary
//              crosses the owner, every count follows from one bit;
//   slow path  marching-squares segments of the 2x2 dual cells, exact
//              segment/edge crossing tests (Alg. 1 restricted to proper
//              crossings), the order of two crossings on one edge, the chain
//              vertex inside each triangle, the inside bit of the owner
//              vertex, and the raw key of each cut triangle reduced to class
//              and rotation through the lookup table (Sec. 3.3.3, Alg. 2).
// Everything lives in registers: segment slots, crossing sets and orders are
// packed integers and bit masks indexed only by compile-time constants.
//
// Exact arithmetic: the grid edge is h = p / U pixels (U = 2^q, q <= 8) and
// coordinates are integers in units of 1 / (4U) pixel.  Boundary points are
// multiples of 2U (even); grid vertex (k,i) is at X = X0 + 4p*i + 2p*o with X0
// odd, and Y = -4U + 2pk*sqrt3.  Every predicate is sign(A + B*sqrt3) with
// integer A, B, never zero (x parity, irrationality of sqrt3).  Each is decided
// in integer arithmetic: per grid row, the floor of its line's ordinate and the
// floors of a / sqrt3 for the block's midpoint ordinates a (RowT) turn every
// sign into one integer comparison.  Geo::h holds p.
#pragma once
#include <stdint.h>

#ifndef SBMT_HD
#define SBMT_HD __host__ __device__ __forceinline__
#endif

namespace sbmt {

constexpr int kRing = 4;     // background sample rows stored above and below the raster
constexpr int kRingC = 32;   // background sample columns stored left of the raster (one word)

struct Geo {
  int32_t W, H;
  int64_t stride;
  int32_t h, s, CW, CH, NK, NI, NCB, wpr;  // h: the grid edge in units of 1/U pixel (p)
  int32_t X0;  // x of vertex (0,0) in units: -2p-3 (U = 1) or -(2p+3U)-1, odd
  int32_t q, U;  // U = 2^q: one unit is 1 / (4U) pixel
  uint32_t flags;
  float inv4s;    // 1 / (4 s)
  double xscale;  // 0.25 / U: units -> pixels
  double invU;    // 1 / U
};

// Sign of a + b*sqrt3, exact.  Zero only for a = b = 0.
SBMT_HD int z3sign(int64_t a, int64_t b) {
  if (a >= 0 && b >= 0) return (a | b) != 0 ? 1 : 0;
  if (a <= 0 && b <= 0) return -1;
  const int64_t a2 = a * a, b2 = 3 * b * b;
  return a > 0 ? (a2 > b2 ? 1 : -1) : (b2 > a2 ? 1 : -1);
}

constexpr double kSqrt3 = 1.7320508075688772;

// floor(sqrt(n)) for n < 2^62: a double estimate, then exact integer steps.
SBMT_HD uint64_t isqrt_u64(uint64_t n) {
  uint64_t r = (uint64_t)__builtin_sqrt((double)n);
  while (r * r > n) --r;
  while ((r + 1) * (r + 1) <= n) ++r;
  return r;
}

// floor(a / sqrt3) for |a| < 2^31: the largest m >= 0 with 3 m^2 < a^2 when
// a > 0 (a / sqrt3 is irrational for a != 0).
SBMT_HD int floor_div_sqrt3(int64_t a) {
  if (a == 0) return 0;
  const int m = (int)isqrt_u64(((uint64_t)(a * a) - 1u) / 3u);
  return a > 0 ? m : -m - 1;
}

// floor(n / (4 s U)) = floor((n >> q) / (4 s)) for |n >> q| < 2^24, through a
// float reciprocal and one correction.
SBMT_HD int div4s(const Geo& g, int n) {
  const int d = 4 * g.s;
  const int m = n >> g.q;
  int q = (int)__builtin_floorf((float)m * g.inv4s);
  q -= q * d > m ? 1 : 0;  // selects, not branches
  q += (q + 1) * d <= m ? 1 : 0;
  return q;
}

// Cell row of grid row k: the largest R with U (2sR + s + 1) <= k p sqrt3,
// i.e. floor((y_k - (s-1)/2) / s) for y_k = -1 + k h sqrt3 / 2, h = p / U.
SBMT_HD int row_cell(const Geo& g, int k) {
  const int s = g.s;
  const int64_t kp = (int64_t)k * g.h;
  // estimate in double precision (off by at most one), then exact steps
  int64_t R = (int64_t)__builtin_floor(((double)kp * kSqrt3 * g.invU - (double)(s + 1)) / (double)(2 * s));
  while (z3sign(-(int64_t)g.U * (2 * s * R + s + 1), kp) < 0) --R;
  while (z3sign(-(int64_t)g.U * (2 * s * (R + 1) + s + 1), kp) >= 0) ++R;
  return (int)R;
}

// Marching squares, corners in positive order TL, TR, BR, BL (bit 0..3); cell
// edge midpoints 0 top, 1 right, 2 bottom, 3 left.  A segment runs from each
// foreground->background transition to the next background->foreground one,
// so background corners are cut off (foreground 8-connected at saddles).
// Entry: count | (start0 | end0 << 2) << 2 | (start1 | end1 << 2) << 6.
constexpr uint32_t ms_entry(int n, int a0, int b0, int a1, int b1) {
  return (uint32_t)(n | ((a0 | (b0 << 2)) << 2) | ((a1 | (b1 << 2)) << 6));
}
constexpr uint64_t ms_pack4(uint32_t e0, uint32_t e1, uint32_t e2, uint32_t e3) {
  return (uint64_t)e0 | ((uint64_t)e1 << 16) | ((uint64_t)e2 << 32) | ((uint64_t)e3 << 48);
}
constexpr uint64_t kMS0 = ms_pack4(0, ms_entry(1, 0, 3, 0, 0), ms_entry(1, 1, 0, 0, 0), ms_entry(1, 1, 3, 0, 0));
constexpr uint64_t kMS1 = ms_pack4(ms_entry(1, 2, 1, 0, 0), ms_entry(2, 0, 1, 2, 3), ms_entry(1, 2, 0, 0, 0),
                                   ms_entry(1, 2, 3, 0, 0));
constexpr uint64_t kMS2 = ms_pack4(ms_entry(1, 3, 2, 0, 0), ms_entry(1, 0, 2, 0, 0), ms_entry(2, 1, 2, 3, 0),
                                   ms_entry(1, 1, 2, 0, 0));
constexpr uint64_t kMS3 = ms_pack4(ms_entry(1, 3, 1, 0, 0), ms_entry(1, 0, 1, 0, 0), ms_entry(1, 3, 0, 0, 0), 0);
SBMT_HD uint32_t ms_case(int c) {
  const uint64_t t = c < 8 ? (c < 4 ? kMS0 : kMS1) : (c < 12 ? kMS2 : kMS3);
  return (uint32_t)(t >> (16 * (c & 3))) & 0xffffu;
}

// Packed per-owner counts.
//  bit 0 self vertex emitted, 1-2 crossings on E0, 3-4 on E1, 5-6 on E2
//  (each in unary: 0, 1 or 3 for none, one or two, so that bits 0-8 count
//  the owner's vertices),
//  7 chain vertex in Tb, 8 chain vertex in Ta, 9-11 triangles of Tb,
//  12-14 triangles of Ta, 15 slow path, 16 owner vertex inside,
//  17 Tb cut, 18 Ta cut, 19 protocol error.
SBMT_HD int info_self(uint32_t f) { return f & 1; }
SBMT_HD int info_n(uint32_t f, int e) { return __builtin_popcount((f >> (1 + 2 * e)) & 3u); }
SBMT_HD int info_Ib(uint32_t f) { return (f >> 7) & 1; }
SBMT_HD int info_Ia(uint32_t f) { return (f >> 8) & 1; }
SBMT_HD int info_ntb(uint32_t f) { return (f >> 9) & 7; }
SBMT_HD int info_nta(uint32_t f) { return (f >> 12) & 7; }
SBMT_HD int info_slow(uint32_t f) { return (f >> 15) & 1; }
SBMT_HD int info_fg(uint32_t f) { return (f >> 16) & 1; }
SBMT_HD int info_ncut(uint32_t f) { return ((f >> 17) & 1) + ((f >> 18) & 1); }
SBMT_HD int info_err(uint32_t f) { return (f >> 19) & 1; }
SBMT_HD int info_nv(uint32_t f) { return __builtin_popcount(f & 0x1ffu); }  // self, crossings, chain vertices
SBMT_HD int info_nt(uint32_t f) { return info_ntb(f) + info_nta(f); }

// ---------------------------------------------------------------------------
// Owner frame and fast path.
// ---------------------------------------------------------------------------
struct Frame {
  int X;        // x4 x of the owner vertex
  int k, i, o;  // row, column, row parity
  int Rlo, Clo; // top-left dual cell of the 2x2 block under Tb u Ta
  uint32_t s9;  // 3x3 samples, bit (3 r + c) = sample (Rlo + r, Clo + c)
};

// A window of the packed coarse raster: rows rr0.., bit columns cc0.. (cc0 a
// multiple of 32) stored with `wpr` words per row.  The kernels stage the
// window a tile needs in LDS; the whole raster is the window (0, 0).
struct Bits {
  const uint32_t* p;
  int wpr, rr0, cc0;
};

SBMT_HD uint32_t sample3(const Bits& b, int rr, int cc) {
  const uint32_t* row = b.p + (rr - b.rr0) * b.wpr;
  const int c = cc - b.cc0;
  const int w = c >> 5, s = c & 31;
  const uint64_t v = ((uint64_t)row[w + 1] << 32) | row[w];
  return (uint32_t)(v >> s) & 7u;
}

SBMT_HD int clo_of(const Geo& g, int X) { return div4s(g, X - 2 * g.h - 2 * (g.s - 1) * g.U); }

SBMT_HD Frame owner_frame(const Geo& g, const Bits& bits, int k, int i, int Rlo) {
  Frame f;
  f.k = k;
  f.i = i;
  f.o = k & 1;
  f.X = g.X0 + 4 * g.h * i + 2 * g.h * f.o;
  f.Rlo = Rlo;
  f.Clo = clo_of(g, f.X);
  const int rr = Rlo + kRing, cc = f.Clo + kRingC;
  f.s9 = sample3(bits, rr, cc) | (sample3(bits, rr + 1, cc) << 3) | (sample3(bits, rr + 2, cc) << 6);
  return f;
}

// The same with the owner's window column Clo already known.
SBMT_HD Frame owner_frame_at(const Geo& g, const Bits& bits, int k, int i, int Rlo, int Clo) {
  Frame f;
  f.k = k;
  f.i = i;
  f.o = k & 1;
  f.X = g.X0 + 4 * g.h * i + 2 * g.h * f.o;
  f.Rlo = Rlo;
  f.Clo = Clo;
  const int rr = Rlo + kRing, cc = Clo + kRingC;
  f.s9 = sample3(bits, rr, cc) | (sample3(bits, rr + 1, cc) << 3) | (sample3(bits, rr + 2, cc) << 6);
  return f;
}

SBMT_HD bool frame_uniform(const Frame& f) { return f.s9 == 0u || f.s9 == 0x1ffu; }

// Counts of owner (k, i) whose window is uniform with inside bit fg.
SBMT_HD uint32_t fast_info_k(const Geo& g, int k, int i, int fg) {
  const bool both = (g.flags & 1u) != 0;
  const int o = k & 1;
  const bool tb_ok = (k + 1 < g.NK) && (i + o - 1 >= 0) && (i + o < g.NI);
  const bool ta_ok = (k + 1 < g.NK) && (i + 1 < g.NI) && (i + o < g.NI);
  const int self = both ? 1 : fg;
  const int ntb = (both || fg) ? (int)tb_ok : 0;
  const int nta = (both || fg) ? (int)ta_ok : 0;
  return (uint32_t)self | ((uint32_t)ntb << 9) | ((uint32_t)nta << 12) | ((uint32_t)fg << 16);
}
SBMT_HD uint32_t fast_info(const Geo& g, const Frame& f) { return fast_info_k(g, f.k, f.i, f.s9 != 0u); }

// Uniform-window masks of one grid row, for the tile kernels: bit (cc - cc0)
// of u0[w] / u1[w] is set when the samples of columns cc .. cc+2 in the three
// sample rows starting at the row's Rlo are all background / all foreground.
// An owner with window column Clo is then uniform iff its bit is set in one of
// them (window_kind).
SBMT_HD void window_masks_word(const Bits& b, int rr, int w, uint32_t& u0, uint32_t& u1) {
  const uint32_t* p0 = b.p + (rr - b.rr0) * b.wpr;
  const uint32_t* p1 = p0 + b.wpr;
  const uint32_t* p2 = p1 + b.wpr;
  const uint32_t o = p0[w] | p1[w] | p2[w], a = p0[w] & p1[w] & p2[w];
  const bool nx = w + 1 < b.wpr;
  const uint32_t on = nx ? (p0[w + 1] | p1[w + 1] | p2[w + 1]) : 0u;
  const uint32_t an = nx ? (p0[w + 1] & p1[w + 1] & p2[w + 1]) : 0u;
  const uint32_t x = o | ((o >> 1) | (on << 31)) | ((o >> 2) | (on << 30));
  const uint32_t y = a & ((a >> 1) | (an << 31)) & ((a >> 2) | (an << 30));
  u0 = ~x;
  u1 = y;
}
// 0: window not uniform, 1: all background, 2: all foreground.
SBMT_HD int window_kind(const Geo& g, const Bits& b, const uint32_t* u0, const uint32_t* u1, int X) {
  const int c = clo_of(g, X) + kRingC - b.cc0;
  const int w = c >> 5, sh = c & 31;
  return (int)((u0[w] >> sh) & 1u) | ((int)((u1[w] >> sh) & 1u) << 1);
}

// ---------------------------------------------------------------------------
// Slow path.
//
// Boundary points of the 2x2 block are the 12 cell-edge midpoints:
//   m = 2r + c       (r < 3, c < 2) between samples (r, c) and (r, c+1)
//   m = 6 + 3r + c   (r < 2, c < 3) between samples (r, c) and (r+1, c)
// Segment slot a = 2q + j holds segment j of dual cell q = 2 cr + cc.
// ---------------------------------------------------------------------------
// Segment slots of a block: nibble a of p (q) is the start (end) midpoint of
// slot a.
struct SegSlots {
  uint32_t p, q;
};

struct Slow {
  uint32_t info;
  uint32_t valid;  // segment slots present
  SegSlots seg;    // start and end midpoints of the segment slots
  uint64_t xm;     // edge e: crossing slot mask at bits [8e, 8e+8)
  uint64_t ord;    // edge e: first slot along U->V at [8e, 8e+4), second at [8e+4, 8e+8)
  uint32_t tri;    // t = 0 (Tb), 1 (Ta): class [8t, 8t+5), rotation [8t+5, 8t+7); chain vertex
                   // midpoint at [16 + 8t, 20 + 8t) (15 = none)
};

// Midpoint m sits at (xs + 2sU XI(m), ys + 2sU YI(m)) from the block's first sample.
constexpr uint64_t kMidXI = 0x420420313131ull;  // nibble m: 1,3,1,3,1,3, 0,2,4, 0,2,4 (from m = 0)
constexpr uint64_t kMidYI = 0x333111442200ull;  // nibble m: 0,0,2,2,4,4, 1,1,1, 3,3,3
SBMT_HD int mid_xi(int m) { return (int)((kMidXI >> (4 * m)) & 15u); }
SBMT_HD int mid_yi(int m) { return (int)((kMidYI >> (4 * m)) & 15u); }
// (both factors of the last product fit in 24 bits: a full-rate multiply)
SBMT_HD int mid_x(const Geo& g, const Frame& f, int m) {
  return g.U * (4 * g.s * f.Clo + 2 * (g.s - 1)) + (int)((uint32_t)(2 * g.s * g.U & 0xffff) * (uint32_t)mid_xi(m));
}
SBMT_HD int mid_y(const Geo& g, const Frame& f, int m) {
  return g.U * (4 * g.s * f.Rlo + 2 * (g.s - 1)) + (int)((uint32_t)(2 * g.s * g.U & 0xffff) * (uint32_t)mid_yi(m));
}
SBMT_HD int slot_p(const SegSlots& seg, int a) { return (int)((seg.p >> (4 * a)) & 15u); }
SBMT_HD int slot_q(const SegSlots& seg, int a) { return (int)((seg.q >> (4 * a)) & 15u); }
SBMT_HD void slot_set(SegSlots& seg, int a, uint32_t pa, uint32_t pb) {
  seg.p |= pa << (4 * a);
  seg.q |= pb << (4 * a);
}
SBMT_HD void slot_clear(SegSlots& seg) { seg.p = seg.q = 0u; }

// lattice vertex index of the ends of edge e (0 v, 1 vr, 2 vdl, 3 vdr)
SBMT_HD int edge_u(int e) { return e == 3 ? 1 : (e == 4 ? 2 : 0); }
SBMT_HD int edge_v(int e) { return e == 0 ? 1 : (e == 1 ? 2 : 3); }
// local edges of the two triangles in positive order: (edge id, direction)
//   Tb: (E2,+) (E4,-) (E1,-);  Ta: (E0,+) (E3,+) (E2,-)
SBMT_HD int tri_edge(int t, int j) {
  return t == 0 ? (j == 0 ? 2 : (j == 1 ? 4 : 1)) : (j == 0 ? 0 : (j == 1 ? 3 : 2));
}
SBMT_HD int tri_dir(int t, int j) { return t == 0 ? (j == 0 ? 1 : -1) : (j == 2 ? -1 : 1); }

SBMT_HD int popc8(uint32_t m) { return __builtin_popcount(m & 255u); }
SBMT_HD int ctz32(uint32_t m) { return __builtin_ctz(m); }
SBMT_HD int ctz8(uint32_t m) { return __builtin_ctz(m | 256u); }  // lowest set bit of m != 0 (8 for 0)

// Class lookup (generated tables), provided by the including translation unit.
SBMT_HD int lut_key(int code);
SBMT_HD int lut_nfg(int cls);
SBMT_HD int lut_ntri(int cls);
SBMT_HD uint32_t lut_tri(int cls, int j);

// Raw key of triangle t from the crossing sets, looked up into class | rot << 6.
// Returns 0 for an uncut triangle, -1 on a protocol violation.  The candidate
// token orders of all three key types are formed straight-line and selected.
SBMT_HD int tri_key(int t, uint64_t sp, const SegSlots& seg, uint64_t xm, uint64_t ord, int Imid) {
  uint32_t list = 0;  // per crossing (8 bits): slot | token << 3 | entry << 7
  int nc = 0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int eid = tri_edge(t, j), dir = tri_dir(t, j);
    const uint32_t m = (uint32_t)(xm >> (8 * eid)) & 255u;
    const int n = popc8(m);
#pragma unroll
    for (int re = 0; re < 2; ++re) {
      const int sl = (int)((ord >> (8 * eid + 4 * re)) & 15);
      const int rt = dir > 0 ? re : n - 1 - re;
      const int spos = (int)((sp >> (8 * sl + eid)) & 1u);  // start point on the positive side
      const int entry = dir > 0 ? !spos : spos;
      const uint32_t item = (uint32_t)(sl | ((2 * j + rt) << 3) | (entry << 7));
      const bool take = re < n && nc < 4;
      list |= take ? item << (8 * nc) : 0u;
      nc += re < n ? 1 : 0;
    }
  }
  if (nc == 0 && Imid == 15) return 0;
  const uint32_t i0 = list & 255u, i1 = (list >> 8) & 255u, i2 = (list >> 16) & 255u, i3 = (list >> 24) & 255u;
  const int s0 = i0 & 7, s1 = i1 & 7, s2 = i2 & 7, s3 = i3 & 7;
  const int k0 = (i0 >> 3) & 7, k1 = (i1 >> 3) & 7, k2 = (i2 >> 3) & 7, k3 = (i3 >> 3) & 7;
  const int e0 = (i0 >> 7) & 1, e1 = (i1 >> 7) & 1, e2 = (i2 >> 7) & 1, e3 = (i3 >> 7) & 1;
  int type = 0, t0 = 0, t1 = 0, t2 = 0, t3 = 0;
  bool good = false;
  if (Imid != 15) {
    // type 2: the crossing of the segment ending at I enters, the other leaves
    const bool in0 = slot_q(seg, s0) == Imid, out1 = slot_p(seg, s1) == Imid;
    const bool in1 = slot_q(seg, s1) == Imid, out0 = slot_p(seg, s0) == Imid;
    const bool a = in0 && out1 && e0 && !e1, b = in1 && out0 && e1 && !e0;
    good = nc == 2 && (a || b);
    type = 2;
    t0 = a ? k0 : k1;
    t1 = a ? k1 : k0;
  } else if (nc == 2) {
    good = s0 == s1 && e0 != e1;
    type = 1;
    t0 = e0 ? k0 : k1;
    t1 = e0 ? k1 : k0;
  } else if (nc == 4) {
    // two consecutive segments S1 -> S2; place each crossing by (segment, entry)
    const int sa = s0, sb = s1 != s0 ? s1 : (s2 != s0 ? s2 : s3);
    const bool ab = slot_q(seg, sa) == slot_p(seg, sb), ba = slot_q(seg, sb) == slot_p(seg, sa);
    const int S1 = ab ? sa : sb;
    const int q0 = (s0 == S1 ? 0 : 2) + (e0 ? 0 : 1), q1 = (s1 == S1 ? 0 : 2) + (e1 ? 0 : 1);
    const int q2 = (s2 == S1 ? 0 : 2) + (e2 ? 0 : 1), q3 = (s3 == S1 ? 0 : 2) + (e3 ? 0 : 1);
    const bool only2 = (s0 == sa || s0 == sb) && (s1 == sa || s1 == sb) && (s2 == sa || s2 == sb) &&
                       (s3 == sa || s3 == sb) && sa != sb;
    good = (ab || ba) && only2 && ((1 << q0) | (1 << q1) | (1 << q2) | (1 << q3)) == 15;
    type = 3;
    t0 = q0 == 0 ? k0 : (q1 == 0 ? k1 : (q2 == 0 ? k2 : k3));
    t1 = q0 == 1 ? k0 : (q1 == 1 ? k1 : (q2 == 1 ? k2 : k3));
    t2 = q0 == 2 ? k0 : (q1 == 2 ? k1 : (q2 == 2 ? k2 : k3));
    t3 = q0 == 3 ? k0 : (q1 == 3 ? k1 : (q2 == 3 ? k2 : k3));
  }
  if (!good) return -1;
  const int code = (type << 12) | (t0 << 9) | (t1 << 6) | (t2 << 3) | t3;
  const int kv = lut_key(code);
  return kv == 0 ? -1 : kv;
}

// Segments of the four dual cells of the block as slots (see Slow::seg).
template <class S>
SBMT_HD void block_segments(const Frame& f, S& seg, uint32_t& valid) {
#define SBMT_S(rr, cc) ((int)((f.s9 >> (3 * (rr) + (cc))) & 1u))
  slot_clear(seg);
  valid = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int cr = q >> 1, cc = q & 1;
    const int c = SBMT_S(cr, cc) | (SBMT_S(cr, cc + 1) << 1) | (SBMT_S(cr + 1, cc + 1) << 2) |
                  (SBMT_S(cr + 1, cc) << 3);
    const uint32_t ms = ms_case(c);
    const uint32_t lm = (uint32_t)((2 * cr + cc) | ((6 + 3 * cr + cc + 1) << 4) | ((2 * (cr + 1) + cc) << 8) |
                                   ((6 + 3 * cr + cc) << 12));
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j < (int)(ms & 3u)) {
        const uint32_t a = (ms >> (2 + 4 * j)) & 3u, b = (ms >> (4 + 4 * j)) & 3u;
        const uint32_t pa = (lm >> (4 * a)) & 15u, pb = (lm >> (4 * b)) & 15u;
        slot_set(seg, 2 * q + j, pa, pb);
        valid |= 1u << (2 * q + j);
      }
    }
  }
#undef SBMT_S
}

// Per 3x3 sample pattern s9, the block's segments in table form (entries
// written on the device by block_table_entry, from block_segments):
//   block_tab(2 s9)     x, y: the slots' start and end midpoints (SegSlots p, q),
//                       z: present slots, w: 0;
//   block_tab(2 s9 + 1) the slots' boxes in midpoint indices, nibble a of
//                       x: xlo, y: xhi, z: ylo, w: yhi of slot a (an absent
//                       slot has the empty box xlo = ylo = 7, xhi = yhi = 0).
SBMT_HD uint4 block_tab(int i);  // provided by the including translation unit

SBMT_HD void block_table_entry(uint32_t s9, uint4& A, uint4& B) {
  Frame f;
  f.X = f.k = f.i = f.o = f.Rlo = f.Clo = 0;
  f.s9 = s9;
  SegSlots seg;
  uint32_t valid;
  block_segments(f, seg, valid);
  uint32_t x0 = 0x77777777u, x1 = 0u, y0 = 0x77777777u, y1 = 0u;
  for (int a = 0; a < 8; ++a) {
    if (!((valid >> a) & 1u)) continue;
    const int pm = slot_p(seg, a), qm = slot_q(seg, a);
    const uint32_t m = ~(15u << (4 * a));
    x0 = (x0 & m) | ((uint32_t)min(mid_xi(pm), mid_xi(qm)) << (4 * a));
    x1 |= (uint32_t)max(mid_xi(pm), mid_xi(qm)) << (4 * a);
    y0 = (y0 & m) | ((uint32_t)min(mid_yi(pm), mid_yi(qm)) << (4 * a));
    y1 |= (uint32_t)max(mid_yi(pm), mid_yi(qm)) << (4 * a);
  }
  A = make_uint4(seg.p, seg.q, valid, 0u);
  B = make_uint4(x0, x1, y0, y1);
}

// floor(m / (2 s)) for |m| < 2^23, through a float reciprocal and one correction.
SBMT_HD int div2s(const Geo& g, int m) {
  const int d = 2 * g.s;
  int q = (int)__builtin_floorf((float)m * (2.0f * g.inv4s));
  q -= q * d > m ? 1 : 0;  // selects, not branches
  q += (q + 1) * d <= m ? 1 : 0;
  return q;
}
// floor(n / (2 s U)) = floor((n >> q) / (2 s)); ceil by symmetry.
SBMT_HD int floor_step(const Geo& g, int n) { return div2s(g, n >> g.q); }
SBMT_HD int ceil_step(const Geo& g, int n) { return -div2s(g, (-n) >> g.q); }

// A segment can cross an owned edge or end inside Tb or Ta only if its
// bounding box meets the box [X - h/2, X + h] x [y_k, y_{k+1}] of Tb u Ta
// (widened by one unit in y, rounded outwards).  With the block's midpoints at
// (xs + 2sU xi, ys + 2sU yi), the box of a slot [xlo, xhi] x [ylo, yhi] in
// midpoint indices meets it iff xhi >= x0, xlo <= x1, yhi >= y0, ylo <= y1.
// Every index lies in 0..4.
struct Reach {
  int x0, x1, y0, y1;
};
// The y range depends on the row only (k and its cell row Rlo).
SBMT_HD void row_reach(const Geo& g, int k, int Rlo, int& y0, int& y1) {
  const int ys = g.U * (4 * g.s * Rlo + 2 * (g.s - 1));
  const double yk = (double)(-4 * g.U) + (double)(2 * (int64_t)g.h * k) * kSqrt3;
  const int ylo = (int)__builtin_floor(yk) - 1;
  const int yhi = (int)__builtin_ceil(yk + 2.0 * g.h * kSqrt3) + 1;
  y0 = ceil_step(g, ylo - ys);
  y1 = floor_step(g, yhi - ys);
}
// The x range depends on the owner's abscissa only.
SBMT_HD void owner_xreach(const Geo& g, int X, int Clo, int& x0, int& x1) {
  const int xs = g.U * (4 * g.s * Clo + 2 * (g.s - 1));
  x0 = ceil_step(g, X - 2 * g.h - xs);
  x1 = floor_step(g, X + 4 * g.h - xs);
}
// Present slots whose box meets the reach box, as bit 4a + 3 for slot a: the
// four comparisons are made for the eight slots at once in nibble lanes
// ((8 + u) - v keeps bit 3 iff u >= v, with no borrow for u, v <= 7).
SBMT_HD uint32_t relevant_nib(const uint4& B, int x0, int x1, int y0, int y1) {
  constexpr uint32_t M8 = 0x88888888u, R1 = 0x11111111u;
  const uint32_t c1 = (B.y | M8) - (uint32_t)x0 * R1;
  const uint32_t c2 = ((uint32_t)x1 * R1 | M8) - B.x;
  const uint32_t c3 = (B.w | M8) - (uint32_t)y0 * R1;
  const uint32_t c4 = ((uint32_t)y1 * R1 | M8) - B.z;
  return c1 & c2 & c3 & c4 & M8;
}
SBMT_HD int nib_slot(uint32_t w) { return ctz32(w) >> 2; }

// Signs of the five point rows of a block (bit yi: the midpoint row yi lies
// below the line) against the horizontal edge lines of grid rows k (row0) and
// k + 1 (row4), exactly; they depend on the row only.
SBMT_HD void row_signs(const Geo& g, int k, int Rlo, uint32_t& row0, uint32_t& row4) {
  const int64_t hk = (int64_t)g.h * k;
  const int ys = g.U * (4 * g.s * Rlo + 2 * (g.s - 1));
  row0 = 0;
  row4 = 0;
  for (int yi = 0; yi < 5; ++yi) {
    const int Ay = ys + 2 * g.s * g.U * yi + 4 * g.U;
    row0 |= (uint32_t)(z3sign(Ay, -2 * hk) > 0) << yi;
    row4 |= (uint32_t)(z3sign(Ay, -2 * (hk + g.h)) > 0) << yi;
  }
}

// What the classification needs of the owner's row, packed in 32 bits:
// y0, y1 of row_reach as signed bytes, row0 in bits 16..20, row4 in 21..25.
SBMT_HD uint32_t pack_row(int y0, int y1, uint32_t row0, uint32_t row4) {
  return (uint32_t)(y0 & 255) | ((uint32_t)(y1 & 255) << 8) | (row0 << 16) | (row4 << 21);
}
SBMT_HD uint32_t row_info(const Geo& g, int k, int Rlo) {
  int y0, y1;
  uint32_t row0, row4;
  row_reach(g, k, Rlo, y0, y1);
  row_signs(g, k, Rlo, row0, row4);
  return pack_row(y0, y1, row0, row4);
}

// Everything the exact predicates need of grid row k, computed once per row:
//   R   its cell row (the Rlo of its owners' blocks)
//   FL  ceil(Y_k) - 1 for the row's ordinate Y_k = -4U + 2pk sqrt3 in units:
//       an integer n lies above the row line (n < Y_k) iff n <= FL
//   pk  row_info (reach in y, row0, row4)
//   TA  floor(a / sqrt3) for the ordinates a = ys + 2sU yi + 4U of the block's
//       midpoint rows yi = 0..4, measured from the line y = -4U through
//       vertex (0, 0) (ys: the block's first sample row)
struct RowT {
  int32_t R, FL;
  uint32_t pk;
  int32_t TA[5];
};

SBMT_HD RowT row_table_entry(const Geo& g, int k) {
  RowT t;
  t.R = row_cell(g, k);
  const int64_t pk = (int64_t)g.h * k;
  t.FL = k == 0 ? -4 * g.U - 1 : -4 * g.U + (int)isqrt_u64((uint64_t)(12 * pk * pk));
  t.pk = row_info(g, k, t.R);
  const int64_t ys = (int64_t)g.U * (4 * g.s * t.R + 2 * (g.s - 1));
  for (int yi = 0; yi < 5; ++yi) t.TA[yi] = floor_div_sqrt3(ys + 2LL * g.s * g.U * yi + 4 * g.U);
  return t;
}
SBMT_HD int row_ta(const RowT& t, int yi) {
  return yi == 0 ? t.TA[0] : (yi == 1 ? t.TA[1] : (yi == 2 ? t.TA[2] : (yi == 3 ? t.TA[3] : t.TA[4])));
}

// orient(P, Q, L) = ex (Ly - Py) - ey (Lx - Px) > 0 for a boundary segment
// P -> Q of the block (direction (dxi, dyi) in midpoint steps: axis-parallel or
// diagonal) and a lattice point L of a grid row, exactly.  The value is never
// zero: Lx is odd and Px even, and Ly is irrational or not a boundary ordinate.
//   vertical    -ey (Lx - Px)
//   horizontal  sign(ex) sign(Ly - Py); Py lies below L's row line iff `below`
//   diagonal    ey = sigma ex: sign(ex) sign(Ly - n), n = Py + sigma (Lx - Px),
//               with n < Ly iff n <= FL of L's row
SBMT_HD bool orient_pos(int dxi, int dyi, int px, int py, int Lx, bool below, int FL) {
  const bool diag_up = (dxi > 0) == (dyi > 0);
  const int n = py + (diag_up ? Lx - px : px - Lx);
  const bool hz = dyi == 0, vt = dxi == 0;
  const bool tdiag = (dxi > 0) == (n <= FL);
  const bool thz = (dxi > 0) == !below;
  const bool tvt = dyi > 0 ? Lx < px : Lx > px;
  return vt ? tvt : (hz ? thz : tdiag);
}

// Inside bit of the owner vertex: its dual cell (0, cv) of the block is
// uniform, or v lies left of every segment of that cell.
template <class S>
SBMT_HD int owner_inside(const Geo& g, const Frame& f, const S& seg, uint32_t valid, const RowT& rt) {
  const int X = f.X;
  const int cv = div4s(g, X - 2 * (g.s - 1) * g.U) - f.Clo;
  const int a = (int)((f.s9 >> cv) & 1u), b = (int)((f.s9 >> (cv + 1)) & 1u);
  const int c = (int)((f.s9 >> (4 + cv)) & 1u), d = (int)((f.s9 >> (3 + cv)) & 1u);
  if (a == b && b == c && c == d) return a;
  const uint32_t row0 = (rt.pk >> 16) & 31u;
  int fg = 1;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int sl = 2 * cv + j;
    if ((valid >> sl) & 1u) {
      const int pm = slot_p(seg, sl), qm = slot_q(seg, sl);
      const int pyi = mid_yi(pm);
      if (!orient_pos(mid_xi(qm) - mid_xi(pm), mid_yi(qm) - pyi, mid_x(g, f, pm), mid_y(g, f, pm), X,
                      (row0 >> pyi) & 1u, rt.FL))
        fg = 0;
    }
  }
  return fg;
}

// Inside bit of the owner vertex v of a quiet owner (no slot's box meets the
// reach box, which holds v).  Then v lies in none of the segment boxes of its
// dual cell (0, cv), i.e. in the part of the cell holding the corners that the
// marching-squares segments do not cut off: with one corner apart from the
// other three, that corner is cut off (a segment box is the quarter cell at
// the corner); at a saddle the background pair is cut off; with two adjacent
// corners apart the segment runs straight through the middle of the cell and
// v's side of it is one exact comparison (v never lies on a midline).
// rowp: the row's packed row_info (row0 bit 1: the block's middle point row
// lies below the row line).
SBMT_HD int quiet_inside(const Geo& g, const Frame& f, uint32_t rowp) {
  const int X = f.X;
  const int cv = div4s(g, X - 2 * (g.s - 1) * g.U) - f.Clo;
  const int a = (int)((f.s9 >> cv) & 1u), b = (int)((f.s9 >> (cv + 1)) & 1u);
  const int c = (int)((f.s9 >> (4 + cv)) & 1u), d = (int)((f.s9 >> (3 + cv)) & 1u);
  const int n = a + b + c + d;
  if (n != 2) return n >= 2 ? 1 : 0;
  if (a == c) return 1;  // saddle: foreground 8-connected
  // top pair apart from the bottom pair: the segment joins the left and right
  // midpoints (midpoint row 1); v above it sits with the top pair.  Left pair
  // apart from the right pair: the segment joins the top and bottom midpoints
  // at abscissa xm.
  if (a == b) return ((rowp >> 17) & 1u) ? a : d;
  return X < mid_x(g, f, cv) ? a : b;
}

// Counts of an owner whose window is not uniform but which no segment can
// reach (no relevant slot): like the fast path with the exact inside bit.
SBMT_HD uint32_t quiet_info(const Geo& g, const Frame& f, int fg) {
  Frame q = f;
  q.s9 = fg ? 0x1ffu : 0u;
  return fast_info(g, q);
}

// Signs of one segment slot of the block, exactly, as integer comparisons:
// e5p / e5q, both ends P, Q against the lines of the owned edges E0..E4 (E0 and
// E4 from the row's signs; E1, E2, E3 as comparisons with the row's floors of
// a / sqrt3), and l4, the lattice vertices v, vr, vdl, vdr against the segment
// line.  For an end point (px, py) with a = py + 4U > 0 (every boundary point
// lies below the line y = -4U) and d = px - X, each diagonal sign is that of
// a + sqrt3 (+-d - 2pk - ...), i.e. of an integer against -floor(a / sqrt3).
struct SlotGeo {
  int st, xs, ys, X, h, hk2;
  uint32_t row0, row4;
};
SBMT_HD SlotGeo slot_geo(const Geo& g, const Frame& f, const RowT& rt) {
  SlotGeo q;
  q.st = 2 * g.s * g.U;
  q.xs = g.U * (4 * g.s * f.Clo + 2 * (g.s - 1));
  q.ys = g.U * (4 * g.s * f.Rlo + 2 * (g.s - 1));
  q.X = f.X;
  q.h = g.h;
  q.hk2 = 2 * g.h * f.k;
  q.row0 = (rt.pk >> 16) & 31u;
  q.row4 = (rt.pk >> 21) & 31u;
  return q;
}
SBMT_HD void slot_signs(const SlotGeo& q, const RowT& rt, int FL1, int pm, int qm, uint32_t& e5p, uint32_t& e5q,
                        uint32_t& l4) {
  const int pxi = mid_xi(pm), pyi = mid_yi(pm), qxi = mid_xi(qm), qyi = mid_yi(qm);
#pragma unroll
  for (int z = 0; z < 2; ++z) {
    const int xi = z == 0 ? pxi : qxi, yi = z == 0 ? pyi : qyi;
    const int d = q.xs + q.st * xi - q.X, T = row_ta(rt, yi);
    uint32_t b5 = ((q.row0 >> yi) & 1u) | (((q.row4 >> yi) & 1u) << 4);
    b5 |= (uint32_t)(d - q.hk2 + T < 0) << 1;            // E1 line through v, vdl
    b5 |= (uint32_t)(T - d - q.hk2 >= 0) << 2;           // E2 line through v, vdr
    b5 |= (uint32_t)(d - 4 * q.h - q.hk2 + T < 0) << 3;  // E3 line through vr, vdr
    (z == 0 ? e5p : e5q) = b5;
  }
  const int px = q.xs + q.st * pxi, py = q.ys + q.st * pyi;
  const int dxi = qxi - pxi, dyi = qyi - pyi;
  const bool b0 = (q.row0 >> pyi) & 1u, b4 = (q.row4 >> pyi) & 1u;
  l4 = (uint32_t)orient_pos(dxi, dyi, px, py, q.X, b0, rt.FL);
  l4 |= (uint32_t)orient_pos(dxi, dyi, px, py, q.X + 4 * q.h, b0, rt.FL) << 1;
  l4 |= (uint32_t)orient_pos(dxi, dyi, px, py, q.X - 2 * q.h, b4, FL1) << 2;
  l4 |= (uint32_t)orient_pos(dxi, dyi, px, py, q.X + 2 * q.h, b4, FL1) << 3;
}

// Per relevant slot a, the 5-bit set of owned edges E0..E4 that its segment
// crosses: the ends lie on different sides of the edge line (d) and the edge
// ends on different sides of the segment line (l4: v, vr, vdl, vdr).
SBMT_HD uint32_t edge_split(uint32_t l4) {
  const uint32_t v = l4 & 1u, vr = (l4 >> 1) & 1u, vdl = (l4 >> 2) & 1u, vdr = (l4 >> 3) & 1u;
  return (v ^ vr) | ((v ^ vdl) << 1) | ((v ^ vdr) << 2) | ((vr ^ vdr) << 3) | ((vdl ^ vdr) << 4);
}

// Full classification of an owner from its row's table entry rt and the FL of
// the row below (FL1).
SBMT_HD void slow_classify(const Geo& g, const Frame& f, const RowT& rt, int FL1, Slow& r) {
  const bool both = (g.flags & 1u) != 0;
  const uint4 A = block_tab(2 * (int)f.s9), B = block_tab(2 * (int)f.s9 + 1);
  SegSlots seg;
  seg.p = A.x;
  seg.q = A.y;
  const uint32_t valid = A.z;
  int x0, x1;
  owner_xreach(g, f.X, f.Clo, x0, x1);
  const int y0 = (int)(int8_t)(rt.pk & 255u), y1 = (int)(int8_t)((rt.pk >> 8) & 255u);
  const uint32_t rel = relevant_nib(B, x0, x1, y0, y1);
  // per relevant slot: the signs of both ends (5 bits each at [8a, 8a+5) of
  // sp / sq), the owned edges its segment crosses (the ends lie on different
  // sides of the edge line and the edge ends on different sides of the
  // segment line; bit a of byte e of xm), and whether its end point is a chain
  // vertex inside Tb or Ta
  const SlotGeo q = slot_geo(g, f, rt);
  uint64_t sp = 0, sq = 0, xm = 0;
  bool err = false;
  int Ib = 15, Ia = 15;
  for (uint32_t w = rel; w; w &= w - 1) {
    const int a = nib_slot(w);
    const int pm = slot_p(seg, a), qm = slot_q(seg, a);
    uint32_t e5p, e5q, l4;
    slot_signs(q, rt, FL1, pm, qm, e5p, e5q, l4);
    sp |= (uint64_t)e5p << (8 * a);
    sq |= (uint64_t)e5q << (8 * a);
    const uint32_t x5 = (e5p ^ e5q) & edge_split(l4);
    xm |= ((uint64_t)(x5 & 1u) | ((uint64_t)((x5 >> 1) & 1u) << 8) | ((uint64_t)((x5 >> 2) & 1u) << 16) |
           ((uint64_t)((x5 >> 3) & 1u) << 24) | ((uint64_t)((x5 >> 4) & 1u) << 32))
          << a;
    const bool inb = ((e5q >> 2) & 1u) && !((e5q >> 4) & 1u) && !((e5q >> 1) & 1u);
    const bool ina = (e5q & 1u) && ((e5q >> 3) & 1u) && !((e5q >> 2) & 1u);
    if (inb) { if (Ib != 15) err = true; Ib = qm; }
    if (ina) { if (Ia != 15) err = true; Ia = qm; }
  }
  // order along each edge; two crossings come from consecutive segments S1 -> S2
  // sharing a vertex M, and S2's lies further along U->V iff
  // sign((P0 - M) x (P2 - M)) * sign(orient(U, V, M)) > 0
  uint64_t ord = 0;
#pragma unroll
  for (int e = 0; e < 5; ++e) {
    const uint32_t m = (uint32_t)(xm >> (8 * e)) & 255u;
    const int n = popc8(m);
    if (n > 2) err = true;
    if (n >= 1) {
      const int a = ctz8(m);
      const int b = n >= 2 ? ctz8(m & (m - 1)) : a;
      int first = a, second = b;
      if (n == 2) {
        int s1 = a, s2 = b;
        if (slot_q(seg, a) == slot_p(seg, b)) { s1 = a; s2 = b; }
        else if (slot_q(seg, b) == slot_p(seg, a)) { s1 = b; s2 = a; }
        else err = true;
        const int M = slot_q(seg, s1), P0 = slot_p(seg, s1), P2 = slot_q(seg, s2);
        const int mx = mid_x(g, f, M), my = mid_y(g, f, M);
        // offsets inside one block of 2 x 2 cells: |d| <= 8 s U, products fit in 32 bits
        const int cr = (mid_x(g, f, P0) - mx) * (mid_y(g, f, P2) - my) - (mid_y(g, f, P0) - my) * (mid_x(g, f, P2) - mx);
        const bool mpos = (sq >> (8 * s1 + e)) & 1u;
        const bool later = (cr > 0) == mpos;
        first = later ? s1 : s2;
        second = later ? s2 : s1;
      }
      ord |= (uint64_t)(first | (second << 4)) << (8 * e);
    }
  }
  const int fg = owner_inside(g, f, seg, valid, rt);
  const int kb = tri_key(0, sp, seg, xm, ord, Ib);
  const int ka = tri_key(1, sp, seg, xm, ord, Ia);
  if (kb < 0 || ka < 0) err = true;
  const int clsb = kb > 0 ? (kb & 63) : 0, clsa = ka > 0 ? (ka & 63) : 0;
  const int rotb = kb > 0 ? (kb >> 6) : 0, rota = ka > 0 ? (ka >> 6) : 0;
  const bool tb_ok = (f.k + 1 < g.NK) && (f.i + f.o - 1 >= 0) && (f.i + f.o < g.NI);
  const bool ta_ok = (f.k + 1 < g.NK) && (f.i + 1 < g.NI) && (f.i + f.o < g.NI);
  const int ntb = clsb ? (both ? lut_ntri(clsb) : lut_nfg(clsb)) : ((tb_ok && (both || fg)) ? 1 : 0);
  const int nta = clsa ? (both ? lut_ntri(clsa) : lut_nfg(clsa)) : ((ta_ok && (both || fg)) ? 1 : 0);
  const int self = both ? 1 : fg;
  const int n0 = popc8((uint32_t)xm & 255u), n1 = popc8((uint32_t)(xm >> 8) & 255u),
            n2 = popc8((uint32_t)(xm >> 16) & 255u);
  auto unary = [](int n) { return n >= 2 ? 3u : (uint32_t)n; };
  r.info = (uint32_t)self | (unary(n0) << 1) | (unary(n1) << 3) | (unary(n2) << 5) |
           ((uint32_t)(Ib != 15) << 7) | ((uint32_t)(Ia != 15) << 8) | ((uint32_t)ntb << 9) |
           ((uint32_t)nta << 12) | (1u << 15) | ((uint32_t)fg << 16) | ((uint32_t)(clsb != 0) << 17) |
           ((uint32_t)(clsa != 0) << 18) | ((uint32_t)err << 19);
  r.valid = valid;
  r.seg = seg;
  r.xm = xm;
  r.ord = ord;
  r.tri = (uint32_t)(clsb | (rotb << 5) | ((clsa | (rota << 5)) << 8) | (Ib << 16) | (Ia << 20));
}

// The same with the row data computed here (paths that classify few owners).
SBMT_HD void slow_classify(const Geo& g, const Frame& f, Slow& r) {
  const RowT rt = row_table_entry(g, f.k), rn = row_table_entry(g, f.k + 1);
  slow_classify(g, f, rt, rn.FL, r);
}

// Classify an owner whose window is not uniform: quiet (no segment can reach
// it: the fast counts with the exact inside bit) or slow.  Returns true if
// the full slow classification is needed.  x0, x1: the owner's reach in x
// (owner_xreach); rowp: its row's packed row_info.
SBMT_HD bool needs_slow(const Geo& g, const Frame& f, int x0, int x1, uint32_t rowp, uint32_t& info) {
  const int y0 = (int)(int8_t)(rowp & 255u), y1 = (int)(int8_t)((rowp >> 8) & 255u);
  if (relevant_nib(block_tab(2 * (int)f.s9 + 1), x0, x1, y0, y1)) return true;
  info = quiet_info(g, f, quiet_inside(g, f, rowp));
  return false;
}

// Compact classification of a slow owner (16 bytes), what emission needs:
//   info  packed counts
//   tri   class [0,5) rot [5,7) of Tb, class [8,13) rot [13,15) of Ta,
//         chain vertex midpoint of Tb [16,20) and Ta [20,24) (15 = none),
//         crossing counts of E3 [24,26) and E4 [26,28)
//   x     crossings on E0, E1, E2 in order from the owner, 8 bits each
//         (start midpoint | end midpoint << 4), E0 at bits [0,16), E1 [16,32),
//         E2 [32,48)
struct SlowRec {
  uint32_t info, tri;
  uint64_t x;
};

SBMT_HD SlowRec pack_slow(const Slow& r) {
  SlowRec o;
  o.info = r.info;
  const uint32_t n3 = (uint32_t)popc8((uint32_t)(r.xm >> 24) & 255u), n4 = (uint32_t)popc8((uint32_t)(r.xm >> 32) & 255u);
  o.tri = (r.tri & 0x00ffffffu) | (n3 << 24) | (n4 << 26);
  uint64_t x = 0;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int n = popc8((uint32_t)(r.xm >> (8 * e)) & 255u);
#pragma unroll
    for (int re = 0; re < 2; ++re) {
      const int sl = (int)((r.ord >> (8 * e + 4 * re)) & 15);
      const uint64_t pq = (uint64_t)(slot_p(r.seg, sl) | (slot_q(r.seg, sl) << 4));
      if (re < n) x |= pq << (16 * e + 8 * re);
    }
  }
  o.x = x;
  return o;
}

// ---------------------------------------------------------------------------
// Emission (Alg. 2, steps 2-4): vertices and sub-triangles of one owner with
// global ids taken from the owner offsets.
// ---------------------------------------------------------------------------
constexpr double kHalfSqrt3 = 0.86602540378443864676;
// pixel coordinates: x = X / (4U) (an exact scaling), y = -1 + (p k / U) sqrt3/2
SBMT_HD double lat_x(const Geo& g, int X) { return (double)X * g.xscale; }
SBMT_HD double to_px(const Geo& g, int v) { return (double)v * g.xscale; }
SBMT_HD double lat_y(const Geo& g, int k) { return -1.0 + ((double)((int64_t)g.h * k) * g.invU) * kHalfSqrt3; }

// Where emission writes: vertex p goes to v[p - vbase], triangle t to
// t[t - tbase] / c[t - tbase] (the kernels stage a row of output in LDS).
struct Out {
  double* v;
  int32_t* t;
  uint8_t* c;
  int64_t vbase, tbase;
};

struct Nb {  // ids one owner needs
  int vid;            // first vertex id of the owner
  int id_vr, id_vdl, id_vdr;
  int b0, b1, b2, b3, b4;  // first crossing id on E0..E4
  int bI;             // id of the chain vertex in Tb (the one in Ta follows)
};

SBMT_HD void put_vertex(double* verts, int64_t p, double x, double y) {
#ifdef SBMT_HOST_EMUL
  verts[2 * p] = x;
  verts[2 * p + 1] = y;
#else
  double2 v;
  v.x = x;
  v.y = y;
  *reinterpret_cast<double2*>(verts + 2 * p) = v;  // verts is 16-byte aligned
#endif
}

// One output triangle as a single 12-byte store.
struct __attribute__((aligned(4))) Tri3 {
  int32_t a, b, c;
};
SBMT_HD void put_tri(int32_t* tris, int64_t u, int a, int b, int c) {
#ifdef SBMT_HOST_EMUL
  tris[3 * u] = a;
  tris[3 * u + 1] = b;
  tris[3 * u + 2] = c;
#else
  Tri3 x;
  x.a = a;
  x.b = b;
  x.c = c;
  *reinterpret_cast<Tri3*>(tris + 3 * u) = x;
#endif
}

// Id of structural slot `sl` (see the emission table): a four-level select.
SBMT_HD int slot_id(const int (&ids)[16], int sl) {
  const int b0 = sl & 1, b1 = sl & 2, b2 = sl & 4, b3 = sl & 8;
  const int x0 = b0 ? ids[1] : ids[0], x1 = b0 ? ids[3] : ids[2], x2 = b0 ? ids[5] : ids[4], x3 = b0 ? ids[7] : ids[6];
  const int x4 = b0 ? ids[9] : ids[8], x5 = b0 ? ids[11] : ids[10], x6 = b0 ? ids[13] : ids[12],
            x7 = b0 ? ids[15] : ids[14];
  const int y0 = b1 ? x1 : x0, y1 = b1 ? x3 : x2, y2 = b1 ? x5 : x4, y3 = b1 ? x7 : x6;
  const int z0 = b2 ? y1 : y0, z1 = b2 ? y3 : y2;
  return b3 ? z1 : z0;
}

// Vertex `sub` of a slow owner, in the owner's vertex order (the vertex
// itself if emitted, the crossings on E0, E1, E2 in order from the owner, the
// chain vertex of Tb, then of Ta), written to id vid + sub.  Crossing
// X = P + t (Q - P), t = dP / (dP - dQ), dP = (V-U) x (P-U), dQ = (V-U) x (Q-U).
// uy, uy1: lat_y of the owner's row and of the row below.
SBMT_HD void emit_slow_vertex(const Geo& g, const Frame& f, const SlowRec& r, int sub, int64_t vid, double uy,
                              double uy1, const Out& out) {
  const uint32_t info = r.info;
  const int self = info_self(info);
  const int n0 = info_n(info, 0), n1 = info_n(info, 1), n2 = info_n(info, 2);
  const double ux = lat_x(g, f.X);
  double x = ux, y = uy;
  const int s = sub - self;
  if (s >= 0 && s < n0 + n1 + n2) {
    const int e = s < n0 ? 0 : (s < n0 + n1 ? 1 : 2);
    const int re = s - (e == 0 ? 0 : (e == 1 ? n0 : n0 + n1));
    const int vX = e == 0 ? f.X + 4 * g.h : (e == 1 ? f.X - 2 * g.h : f.X + 2 * g.h);
    const double vx = lat_x(g, vX), vy = e == 0 ? uy : uy1;
    const double gx = vx - ux, gy = vy - uy;
    const uint32_t pq = (uint32_t)(r.x >> (16 * e + 8 * re)) & 255u;
    const int pm = (int)(pq & 15u), qm = (int)(pq >> 4);
    const double px = to_px(g, mid_x(g, f, pm)), py = to_px(g, mid_y(g, f, pm));
    const double qx = to_px(g, mid_x(g, f, qm)), qy = to_px(g, mid_y(g, f, qm));
    const double dp = gx * (py - uy) - gy * (px - ux);
    const double dq = gx * (qy - uy) - gy * (qx - ux);
    const double tt = dp / (dp - dq);
    x = px + tt * (qx - px);
    y = py + tt * (qy - py);
  } else if (s >= 0) {
    const int mb = (int)((r.tri >> 16) & 15u), ma = (int)((r.tri >> 20) & 15u);
    const int m = (s == n0 + n1 + n2 && mb != 15) ? mb : ma;
    x = to_px(g, mid_x(g, f, m));
    y = to_px(g, mid_y(g, f, m));
  }
  put_vertex(out.v, vid + sub - out.vbase, x, y);
}

// Triangle `sub` of a slow owner, in the owner's triangle order (those of Tb,
// then of Ta; a cut triangle's emitted sub-triangles in table order), written
// to triangle to + sub.  `lut` is the emission table [class][rot][t][j] of the
// side mode: every entry with both sides, else the foreground ones (the
// kernels keep a copy in LDS, so that no table load waits behind the stores
// already issued).
SBMT_HD void emit_slow_triangle(const Geo& g, const SlowRec& r, int sub, const Nb& nb, int64_t to,
                                const Out& out, const uint16_t* lut) {
  const bool both = (g.flags & 1u) != 0;
  const uint32_t info = r.info;
  const int ntb = info_ntb(info);
  const int t = sub < ntb ? 0 : 1;
  const int j = sub - (t ? ntb : 0);
  const int cls = (int)((r.tri >> (8 * t)) & 31u);
  const int64_t u = to + sub - out.tbase;
  if (cls == 0) {
    put_tri(out.t, u, nb.vid, t == 0 ? nb.id_vdr : nb.id_vr, t == 0 ? nb.id_vdl : nb.id_vdr);
    out.c[u] = both && !info_fg(info) ? 0x80 : 0;
    return;
  }
  const int rot = (int)((r.tri >> (8 * t + 5)) & 3u);
  const int hasIb = ((r.tri >> 16) & 15u) != 15u;
  const int ids[16] = {nb.vid, nb.b0, nb.b0 + 1, nb.b1, nb.b1 + 1, nb.b2, nb.b2 + 1, nb.bI, nb.bI + hasIb,
                       nb.id_vr, nb.b3, nb.b3 + 1, nb.id_vdl, nb.b4, nb.b4 + 1, nb.id_vdr};
  // the j-th emitted entry of the template
  const uint32_t w = lut[((cls * 3 + rot) * 2 + t) * 5 + j];
  const int side = (int)((w >> 12) & 1u);
  put_tri(out.t, u, slot_id(ids, (int)(w & 15u)), slot_id(ids, (int)((w >> 4) & 15u)),
          slot_id(ids, (int)((w >> 8) & 15u)));
  out.c[u] = (uint8_t)(cls | (side ? 0 : 0x80));
}

// Emit one slow owner from its record (one thread for all its outputs).
SBMT_HD void emit_slow(const Geo& g, const Frame& f, const SlowRec& r, const Nb& nb, int64_t to, const Out& out,
                       const uint16_t* lut) {
  const int nv = info_nv(r.info), nt = info_nt(r.info);
  const double uy = lat_y(g, f.k), uy1 = lat_y(g, f.k + 1);
  for (int s = 0; s < nv; ++s) emit_slow_vertex(g, f, r, s, nb.vid, uy, uy1, out);
  for (int s = 0; s < nt; ++s) emit_slow_triangle(g, r, s, nb, to, out, lut);
}

}  // namespace sbmt
