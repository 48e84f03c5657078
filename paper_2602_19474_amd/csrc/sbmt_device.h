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
// Exact arithmetic: quarter-pixel integer coordinates ("x4 units").  Boundary
// points are even integers; grid vertex (k,i) is at X = -2h-3 + 4h*i + 2h*o
// (odd) and Y = -4 + 2hk*sqrt3.  Every predicate is sign(A + B*sqrt3) with
// integer A, B, never zero (x parity, irrationality of sqrt3), decided by a
// floating-point filter with an exact integer fallback.
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
  int32_t h, s, CW, CH, NK, NI, NCB, wpr;
  int32_t X0;  // x4 x-coordinate of vertex (0,0) = -2h-3
  uint32_t flags;
  float inv4s;  // 1 / (4 s)
};

// Sign of a + b*sqrt3, exact.  Zero only for a = b = 0.
SBMT_HD int z3sign(int64_t a, int64_t b) {
  if (a >= 0 && b >= 0) return (a | b) != 0 ? 1 : 0;
  if (a <= 0 && b <= 0) return -1;
  const int64_t a2 = a * a, b2 = 3 * b * b;
  return a > 0 ? (a2 > b2 ? 1 : -1) : (b2 > a2 ? 1 : -1);
}

// Same sign through a double-precision filter: |fl(a + b*c) - (a + b*sqrt3)|
// < 5e-16 (|a| + 2|b|) for |a|, |b| < 2^31, so a larger magnitude decides.
SBMT_HD int z3sign_f(int64_t a, int64_t b) {
  const double d = (double)a + (double)b * 1.7320508075688772;
  const double m = 4e-15 * ((double)(a < 0 ? -a : a) + 2.0 * (double)(b < 0 ? -b : b));
  if (d > m) return 1;
  if (d < -m) return -1;
  return z3sign(a, b);
}

constexpr double kSqrt3 = 1.7320508075688772;

// Sign of a quantity whose exact value is a + b*sqrt3 (integers a, b with
// |a|, |b| < 2^31) and whose double-precision evaluation in owner-local
// coordinates is v (absolute error below 1e-9 for coordinates below 2^20).
// Outside the +-1e-6 band the double decides; inside it the exact integer test.
SBMT_HD int sgn_filtered(double v, int64_t a, int64_t b) {
  if (v > 1e-6) return 1;
  if (v < -1e-6) return -1;
  return z3sign(a, b);
}

SBMT_HD int64_t floordiv(int64_t a, int64_t b) {  // b > 0
  const int64_t q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

// floor(n / (4 s)) for |n| < 2^24 through a float reciprocal and one correction.
SBMT_HD int div4s(const Geo& g, int n) {
  const int d = 4 * g.s;
  int q = (int)__builtin_floorf((float)n * g.inv4s);
  if (q * d > n) --q;
  else if ((q + 1) * d <= n) ++q;
  return q;
}

// Cell row of grid row k: the largest R with 2sR + s + 1 <= k*h*sqrt3, i.e.
// floor((y_k - (s-1)/2) / s) for y_k = -1 + k h sqrt3 / 2.
SBMT_HD int row_cell(int k, int h, int s) {
  const int64_t kh = (int64_t)k * h;
  int64_t R = floordiv(kh * 17320 / 10000 - s - 1, 2 * s);  // 1.732 < sqrt3 < 1.7321
  while (z3sign(-(2 * s * R + s + 1), kh) < 0) --R;
  while (z3sign(-(2 * s * (R + 1) + s + 1), kh) >= 0) ++R;
  return (int)R;
}

// Marching squares, corners in positive order TL, TR, BR, BL (bit 0..3); cell
// edge midpoints 0 top, 1 right, 2 bottom, 3 left.  A segment runs from each
// foreground->background transition to the next background->foreground one,
// so background corners are cut off (foreground 8-connected at saddles).
// Entry: count | (start0 | end0 << 2) << 2 | (start1 | end1 << 2) << 6.
#define SBMT_MS(n, a0, b0, a1, b1) (uint16_t)((n) | (((a0) | ((b0) << 2)) << 2) | (((a1) | ((b1) << 2)) << 6))
SBMT_HD uint16_t ms_case(int c) {
  switch (c) {
    case 1: return SBMT_MS(1, 0, 3, 0, 0);
    case 2: return SBMT_MS(1, 1, 0, 0, 0);
    case 3: return SBMT_MS(1, 1, 3, 0, 0);
    case 4: return SBMT_MS(1, 2, 1, 0, 0);
    case 5: return SBMT_MS(2, 0, 1, 2, 3);
    case 6: return SBMT_MS(1, 2, 0, 0, 0);
    case 7: return SBMT_MS(1, 2, 3, 0, 0);
    case 8: return SBMT_MS(1, 3, 2, 0, 0);
    case 9: return SBMT_MS(1, 0, 2, 0, 0);
    case 10: return SBMT_MS(2, 1, 2, 3, 0);
    case 11: return SBMT_MS(1, 1, 2, 0, 0);
    case 12: return SBMT_MS(1, 3, 1, 0, 0);
    case 13: return SBMT_MS(1, 0, 1, 0, 0);
    case 14: return SBMT_MS(1, 3, 0, 0, 0);
    default: return 0;
  }
}
#undef SBMT_MS

// Packed per-owner counts.
//  bit 0 self vertex emitted, 1-2 crossings on E0, 3-4 on E1, 5-6 on E2,
//  7 chain vertex in Tb, 8 chain vertex in Ta, 9-11 triangles of Tb,
//  12-14 triangles of Ta, 15 slow path, 16 owner vertex inside,
//  17 Tb cut, 18 Ta cut, 19 protocol error.
SBMT_HD int info_self(uint32_t f) { return f & 1; }
SBMT_HD int info_n(uint32_t f, int e) { return (f >> (1 + 2 * e)) & 3; }
SBMT_HD int info_Ib(uint32_t f) { return (f >> 7) & 1; }
SBMT_HD int info_Ia(uint32_t f) { return (f >> 8) & 1; }
SBMT_HD int info_ntb(uint32_t f) { return (f >> 9) & 7; }
SBMT_HD int info_nta(uint32_t f) { return (f >> 12) & 7; }
SBMT_HD int info_slow(uint32_t f) { return (f >> 15) & 1; }
SBMT_HD int info_fg(uint32_t f) { return (f >> 16) & 1; }
SBMT_HD int info_ncut(uint32_t f) { return ((f >> 17) & 1) + ((f >> 18) & 1); }
SBMT_HD int info_err(uint32_t f) { return (f >> 19) & 1; }
SBMT_HD int info_nv(uint32_t f) {
  return info_self(f) + info_n(f, 0) + info_n(f, 1) + info_n(f, 2) + info_Ib(f) + info_Ia(f);
}
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

SBMT_HD uint32_t sample3(const uint32_t* bits, int wpr, int rr, int cc) {
  const uint32_t* row = bits + (int64_t)rr * wpr;
  const int w = cc >> 5, b = cc & 31;
  const uint64_t v = ((uint64_t)row[w + 1] << 32) | row[w];
  return (uint32_t)(v >> b) & 7u;
}

SBMT_HD Frame owner_frame(const Geo& g, const uint32_t* bits, int k, int i, int Rlo) {
  Frame f;
  f.k = k;
  f.i = i;
  f.o = k & 1;
  f.X = g.X0 + 4 * g.h * i + 2 * g.h * f.o;
  f.Rlo = Rlo;
  f.Clo = div4s(g, f.X - 2 * g.h - 2 * (g.s - 1));
  const int rr = Rlo + kRing, cc = f.Clo + kRingC;
  f.s9 = sample3(bits, g.wpr, rr, cc) | (sample3(bits, g.wpr, rr + 1, cc) << 3) |
         (sample3(bits, g.wpr, rr + 2, cc) << 6);
  return f;
}

SBMT_HD bool frame_uniform(const Frame& f) { return f.s9 == 0u || f.s9 == 0x1ffu; }

// Counts of an owner whose window is uniform.
SBMT_HD uint32_t fast_info(const Geo& g, const Frame& f) {
  const bool both = (g.flags & 1u) != 0;
  const int fg = f.s9 != 0u;
  const bool tb_ok = (f.k + 1 < g.NK) && (f.i + f.o - 1 >= 0) && (f.i + f.o < g.NI);
  const bool ta_ok = (f.k + 1 < g.NK) && (f.i + 1 < g.NI) && (f.i + f.o < g.NI);
  const int self = both ? 1 : fg;
  const int ntb = (both || fg) ? (int)tb_ok : 0;
  const int nta = (both || fg) ? (int)ta_ok : 0;
  return (uint32_t)self | ((uint32_t)ntb << 9) | ((uint32_t)nta << 12) | ((uint32_t)fg << 16);
}

// ---------------------------------------------------------------------------
// Slow path.
//
// Boundary points of the 2x2 block are the 12 cell-edge midpoints:
//   m = 2r + c       (r < 3, c < 2) between samples (r, c) and (r, c+1)
//   m = 6 + 3r + c   (r < 2, c < 3) between samples (r, c) and (r+1, c)
// Segment slot a = 2q + j holds segment j of dual cell q = 2 cr + cc.
// ---------------------------------------------------------------------------
struct Slow {
  uint32_t info;
  uint32_t valid;  // segment slots present
  uint64_t seg;    // slot a: start midpoint bits [8a, 8a+4), end midpoint [8a+4, 8a+8)
  uint64_t xm;     // edge e: crossing slot mask at bits [8e, 8e+8)
  uint64_t ord;    // edge e: first slot along U->V at [8e, 8e+4), second at [8e+4, 8e+8)
  uint32_t tri;    // t = 0 (Tb), 1 (Ta): class [8t, 8t+5), rotation [8t+5, 8t+7); chain vertex
                   // midpoint at [16 + 8t, 20 + 8t) (15 = none)
};

SBMT_HD int mid_x(const Geo& g, const Frame& f, int m) {
  const int xs = 4 * g.s * f.Clo + 2 * (g.s - 1);
  return m < 6 ? xs + 4 * g.s * (m & 1) + 2 * g.s : xs + 4 * g.s * ((m - 6) % 3);
}
SBMT_HD int mid_y(const Geo& g, const Frame& f, int m) {
  const int ys = 4 * g.s * f.Rlo + 2 * (g.s - 1);
  return m < 6 ? ys + 4 * g.s * (m >> 1) : ys + 4 * g.s * ((m - 6) / 3) + 2 * g.s;
}
SBMT_HD int slot_p(uint64_t seg, int a) { return (int)((seg >> (8 * a)) & 15); }
SBMT_HD int slot_q(uint64_t seg, int a) { return (int)((seg >> (8 * a + 4)) & 15); }

// lattice vertex index of the ends of edge e (0 v, 1 vr, 2 vdl, 3 vdr)
SBMT_HD int edge_u(int e) { return e == 3 ? 1 : (e == 4 ? 2 : 0); }
SBMT_HD int edge_v(int e) { return e == 0 ? 1 : (e == 1 ? 2 : 3); }
// local edges of the two triangles in positive order: (edge id, direction)
//   Tb: (E2,+) (E4,-) (E1,-);  Ta: (E0,+) (E3,+) (E2,-)
SBMT_HD int tri_edge(int t, int j) {
  return t == 0 ? (j == 0 ? 2 : (j == 1 ? 4 : 1)) : (j == 0 ? 0 : (j == 1 ? 3 : 2));
}
SBMT_HD int tri_dir(int t, int j) { return t == 0 ? (j == 0 ? 1 : -1) : (j == 2 ? -1 : 1); }

SBMT_HD int popc8(uint32_t m) {
  m = m - ((m >> 1) & 0x55u);
  m = (m & 0x33u) + ((m >> 2) & 0x33u);
  return (int)((m + (m >> 4)) & 0x0fu);
}
SBMT_HD int ctz8(uint32_t m) {
  int n = 0;
  if (!(m & 0x0fu)) { n += 4; m >>= 4; }
  if (!(m & 0x03u)) { n += 2; m >>= 2; }
  if (!(m & 0x01u)) { n += 1; }
  return n;
}

// Class lookup (generated tables), provided by the including translation unit.
SBMT_HD int lut_key(int code);
SBMT_HD int lut_nfg(int cls);
SBMT_HD int lut_ntri(int cls);
SBMT_HD uint32_t lut_tri(int cls, int j);

// Raw key of triangle t from the crossing sets, looked up into class | rot << 6.
// Returns 0 for an uncut triangle, -1 on a protocol violation.
SBMT_HD int tri_key(int t, const uint32_t pos[5], uint64_t seg, uint64_t xm, uint64_t ord, int Imid) {
  uint32_t list = 0;  // per crossing: slot | local edge << 3 | rank << 5 | entry << 7
  int nc = 0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int eid = tri_edge(t, j), dir = tri_dir(t, j);
    const uint32_t m = (uint32_t)(xm >> (8 * eid)) & 255u;
    const int n = popc8(m);
#pragma unroll
    for (int re = 0; re < 2; ++re) {
      if (re < n) {
        const int sl = (int)((ord >> (8 * eid + 4 * re)) & 15);
        const int rt = dir > 0 ? re : n - 1 - re;
        const int sp = (int)((pos[eid] >> slot_p(seg, sl)) & 1u);
        const int entry = dir > 0 ? !sp : sp;
        if (nc < 4) list |= (uint32_t)(sl | (j << 3) | (rt << 5) | (entry << 7)) << (8 * nc);
        ++nc;
      }
    }
  }
  if (nc == 0 && Imid == 15) return 0;
  if (nc > 4) return -1;
  int type, t0 = 0, t1 = 0, t2 = 0, t3 = 0;
#define SBMT_TOK(c) ((int)((((list >> (8 * (c))) >> 3) & 3) * 2 + (((list >> (8 * (c))) >> 5) & 1)))
#define SBMT_SLOT(c) ((int)((list >> (8 * (c))) & 7))
#define SBMT_ENT(c) ((int)(((list >> (8 * (c))) >> 7) & 1))
  if (Imid != 15) {
    if (nc != 2) return -1;
    const int in0 = slot_q(seg, SBMT_SLOT(0)) == Imid, out0 = slot_p(seg, SBMT_SLOT(0)) == Imid;
    const int in1 = slot_q(seg, SBMT_SLOT(1)) == Imid, out1 = slot_p(seg, SBMT_SLOT(1)) == Imid;
    int ci, co;
    if (in0 && out1) { ci = 0; co = 1; }
    else if (in1 && out0) { ci = 1; co = 0; }
    else return -1;
    if (!SBMT_ENT(ci) || SBMT_ENT(co)) return -1;
    type = 2;
    t0 = ci == 0 ? SBMT_TOK(0) : SBMT_TOK(1);
    t1 = co == 0 ? SBMT_TOK(0) : SBMT_TOK(1);
  } else if (nc == 2) {
    if (SBMT_SLOT(0) != SBMT_SLOT(1) || SBMT_ENT(0) == SBMT_ENT(1)) return -1;
    type = 1;
    t0 = SBMT_ENT(0) ? SBMT_TOK(0) : SBMT_TOK(1);
    t1 = SBMT_ENT(0) ? SBMT_TOK(1) : SBMT_TOK(0);
  } else if (nc == 4) {
    const int sa = SBMT_SLOT(0);
    int sb = -1;
#pragma unroll
    for (int c = 1; c < 4; ++c)
      if (SBMT_SLOT(c) != sa) sb = SBMT_SLOT(c);
    if (sb < 0) return -1;
    int s1, s2;
    if (slot_q(seg, sa) == slot_p(seg, sb)) { s1 = sa; s2 = sb; }
    else if (slot_q(seg, sb) == slot_p(seg, sa)) { s1 = sb; s2 = sa; }
    else return -1;
    int have = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int sl = SBMT_SLOT(c), en = SBMT_ENT(c), tk = SBMT_TOK(c);
      const int q = (sl == s1 ? 0 : (sl == s2 ? 2 : 8)) + (en ? 0 : 1);
      if (q > 3) return -1;
      if (have & (1 << q)) return -1;
      have |= 1 << q;
      if (q == 0) t0 = tk;
      else if (q == 1) t1 = tk;
      else if (q == 2) t2 = tk;
      else t3 = tk;
    }
    type = 3;
  } else {
    return -1;
  }
#undef SBMT_TOK
#undef SBMT_SLOT
#undef SBMT_ENT
  const int code = (type << 12) | (t0 << 9) | (t1 << 6) | (t2 << 3) | t3;
  const int kv = lut_key(code);
  return kv == 0 ? -1 : kv;
}

SBMT_HD void slow_classify(const Geo& g, const Frame& f, Slow& r) {
  const bool both = (g.flags & 1u) != 0;
  const int h = g.h, X = f.X;
  const int64_t hk = (int64_t)h * f.k;
#define SBMT_S(rr, cc) ((int)((f.s9 >> (3 * (rr) + (cc))) & 1u))
  // signs of the 12 midpoints against the five edge lines (bit m = positive),
  // in coordinates local to the owner vertex: ly = (My + 4) - 2hk sqrt3
  const double yk = (double)(2 * hk) * kSqrt3;
  uint32_t pos[5] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll
  for (int m = 0; m < 12; ++m) {
    const int Ay = mid_y(g, f, m) + 4;
    const int lx = mid_x(g, f, m) - X;
    const double ly = (double)Ay - yk;
    pos[0] |= (uint32_t)(sgn_filtered(ly, Ay, -2 * hk) > 0) << m;
    pos[4] |= (uint32_t)(sgn_filtered(ly - 2.0 * h * kSqrt3, Ay, -2 * (hk + h)) > 0) << m;
    pos[2] |= (uint32_t)(sgn_filtered(ly - kSqrt3 * lx, Ay, -(lx + 2 * hk)) > 0) << m;
    pos[1] |= (uint32_t)(sgn_filtered(ly + kSqrt3 * lx, Ay, lx - 2 * hk) < 0) << m;
    pos[3] |= (uint32_t)(sgn_filtered(ly + kSqrt3 * (lx - 4 * h), Ay, lx - 4 * h - 2 * hk) < 0) << m;
  }
  // segments of the four dual cells
  uint64_t seg = 0;
  uint32_t valid = 0;
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
        seg |= (uint64_t)(pa | (pb << 4)) << (8 * (2 * q + j));
        valid |= 1u << (2 * q + j);
      }
    }
  }
  // signs of the four lattice vertices against each segment line: bit 4a + l;
  // orient(P, Q, L) = ex (Ly - Py) - ey (Lx - Px), Ly = -4 + LB sqrt3
  const int LX0 = X, LX1 = X + 4 * h, LX2 = X - 2 * h, LX3 = X + 2 * h;
  const int64_t LB01 = 2 * hk, LB23 = 2 * (hk + h);
  const double yb01 = (double)LB01 * kSqrt3, yb23 = (double)LB23 * kSqrt3;
  uint32_t lv = 0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    if ((valid >> a) & 1u) {
      const int pm = slot_p(seg, a), qm = slot_q(seg, a);
      const int px = mid_x(g, f, pm), py = mid_y(g, f, pm);
      const int ex = mid_x(g, f, qm) - px, ey = mid_y(g, f, qm) - py;
      const int64_t base = (int64_t)ex * (-4 - py);
      const double d01 = (double)(-4 - py) + yb01, d23 = (double)(-4 - py) + yb23;
      lv |= (uint32_t)(sgn_filtered(ex * d01 - (double)ey * (LX0 - px), base - (int64_t)ey * (LX0 - px), ex * LB01) > 0)
            << (4 * a);
      lv |= (uint32_t)(sgn_filtered(ex * d01 - (double)ey * (LX1 - px), base - (int64_t)ey * (LX1 - px), ex * LB01) > 0)
            << (4 * a + 1);
      lv |= (uint32_t)(sgn_filtered(ex * d23 - (double)ey * (LX2 - px), base - (int64_t)ey * (LX2 - px), ex * LB23) > 0)
            << (4 * a + 2);
      lv |= (uint32_t)(sgn_filtered(ex * d23 - (double)ey * (LX3 - px), base - (int64_t)ey * (LX3 - px), ex * LB23) > 0)
            << (4 * a + 3);
    }
  }
  // crossing sets: both segment ends on different sides of the edge line and
  // both edge ends on different sides of the segment line
  uint64_t xm = 0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    if ((valid >> a) & 1u) {
      const int pm = slot_p(seg, a), qm = slot_q(seg, a);
      const uint32_t l4 = (lv >> (4 * a)) & 15u;
#pragma unroll
      for (int e = 0; e < 5; ++e) {
        const uint32_t sp = (pos[e] >> pm) & 1u, sq = (pos[e] >> qm) & 1u;
        const uint32_t lu = (l4 >> edge_u(e)) & 1u, lw = (l4 >> edge_v(e)) & 1u;
        if (sp != sq && lu != lw) xm |= 1ull << (8 * e + a);
      }
    }
  }
  // order along each edge; two crossings come from consecutive segments S1 -> S2
  // sharing a vertex M, and S2's lies further along U->V iff
  // sign((P0 - M) x (P2 - M)) * sign(orient(U, V, M)) > 0
  bool err = false;
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
        const int64_t mx = mid_x(g, f, M), my = mid_y(g, f, M);
        const int64_t cr = (mid_x(g, f, P0) - mx) * (mid_y(g, f, P2) - my) -
                           (mid_y(g, f, P0) - my) * (mid_x(g, f, P2) - mx);
        const bool mpos = (pos[e] >> M) & 1u;
        const bool later = (cr > 0) == mpos;
        first = later ? s1 : s2;
        second = later ? s2 : s1;
      }
      ord |= (uint64_t)(first | (second << 4)) << (8 * e);
    }
  }
  // chain vertices: the midpoints between the centre sample and its neighbours
  int Ib = 15, Ia = 15;
  {
    const int c0 = SBMT_S(1, 1);
    const int cand[4] = {2, 3, 7, 10};
    const int ex[4] = {SBMT_S(1, 0) != c0, SBMT_S(1, 2) != c0, SBMT_S(0, 1) != c0, SBMT_S(2, 1) != c0};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (ex[q]) {
        const int m = cand[q];
        const bool inb = ((pos[2] >> m) & 1u) && !((pos[4] >> m) & 1u) && !((pos[1] >> m) & 1u);
        const bool ina = ((pos[0] >> m) & 1u) && ((pos[3] >> m) & 1u) && !((pos[2] >> m) & 1u);
        if (inb) { if (Ib != 15) err = true; Ib = m; }
        if (ina) { if (Ia != 15) err = true; Ia = m; }
      }
    }
  }
  // inside bit of the owner vertex: its dual cell (0, cv) of the block
  int fg;
  {
    const int cv = div4s(g, X - 2 * (g.s - 1)) - f.Clo;
    const int a = SBMT_S(0, cv), b = SBMT_S(0, cv + 1), c = SBMT_S(1, cv + 1), d = SBMT_S(1, cv);
    if (a == b && b == c && c == d) {
      fg = a;
    } else {
      fg = 1;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int sl = 2 * cv + j;
        if (((valid >> sl) & 1u) && !((lv >> (4 * sl)) & 1u)) fg = 0;
      }
    }
  }
#undef SBMT_S
  // keys of the two triangles
  const int kb = tri_key(0, pos, seg, xm, ord, Ib);
  const int ka = tri_key(1, pos, seg, xm, ord, Ia);
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
  r.info = (uint32_t)self | ((uint32_t)(n0 & 3) << 1) | ((uint32_t)(n1 & 3) << 3) | ((uint32_t)(n2 & 3) << 5) |
           ((uint32_t)(Ib != 15) << 7) | ((uint32_t)(Ia != 15) << 8) | ((uint32_t)ntb << 9) |
           ((uint32_t)nta << 12) | (1u << 15) | ((uint32_t)fg << 16) | ((uint32_t)(clsb != 0) << 17) |
           ((uint32_t)(clsa != 0) << 18) | ((uint32_t)err << 19);
  r.valid = valid;
  r.seg = seg;
  r.xm = xm;
  r.ord = ord;
  r.tri = (uint32_t)(clsb | (rotb << 5) | ((clsa | (rota << 5)) << 8) | (Ib << 16) | (Ia << 20));
}

// ---------------------------------------------------------------------------
// Emission (Alg. 2, steps 2-4): vertices and sub-triangles of one owner with
// global ids taken from the owner offsets.
// ---------------------------------------------------------------------------
constexpr double kHalfSqrt3 = 0.86602540378443864676;
SBMT_HD double lat_x(int X) { return 0.25 * (double)X; }
SBMT_HD double lat_y(int h, int k) { return -1.0 + (double)(h * k) * kHalfSqrt3; }

struct Nb {  // ids one owner needs
  int vid;            // first vertex id of the owner
  int id_vr, id_vdl, id_vdr;
  int b0, b1, b2, b3, b4;  // first crossing id on E0..E4
  int bI;             // id of the chain vertex in Tb (the one in Ta follows)
};

SBMT_HD void put_vertex(double* verts, int64_t p, double x, double y) {
  verts[2 * p] = x;
  verts[2 * p + 1] = y;
}

// Sub-triangle key for sorting: (a, b, c) rotated to start at the smallest id.
struct TriK {
  int a, b, c, code;
};
SBMT_HD TriK trik(int x, int y, int z, int code) {
  TriK t;
  if (y < x && y < z) { t.a = y; t.b = z; t.c = x; }
  else if (z < x && z < y) { t.a = z; t.b = x; t.c = y; }
  else { t.a = x; t.b = y; t.c = z; }
  t.code = code;
  return t;
}
SBMT_HD bool trik_less(const TriK& p, const TriK& q) {
  return p.a != q.a ? p.a < q.a : (p.b != q.b ? p.b < q.b : p.c < q.c);
}
SBMT_HD void trik_cx(TriK& p, TriK& q) {
  if (trik_less(q, p)) { TriK t = p; p = q; q = t; }
}

// Emit the sub-triangles of cut triangle t (sorted within the parent).
SBMT_HD void emit_cut(const Geo& g, const Slow& r, int t, const Nb& nb, int64_t& tp, int32_t* __restrict__ tris,
                      uint8_t* __restrict__ codes) {
  const bool both = (g.flags & 1u) != 0;
  const int cls = (int)((r.tri >> (8 * t)) & 31u), rot = (int)((r.tri >> (8 * t + 5)) & 3u);
  const int c1 = t == 0 ? nb.id_vdr : nb.id_vr, c2 = t == 0 ? nb.id_vdl : nb.id_vdr;
  const int idI = nb.bI + (t == 1 ? (int)(((r.tri >> 16) & 15u) != 15u) : 0);
  const int nt = lut_ntri(cls);
  const int bigc = 0x7fffffff;
  TriK q0 = {bigc, bigc, bigc, 0}, q1 = q0, q2 = q0, q3 = q0, q4 = q0;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    if (j < nt) {
      const uint32_t w = lut_tri(cls, j);
      const int side = (int)((w >> 12) & 1u);
      if (both || side) {
        int id3[3];
#pragma unroll
        for (int z = 0; z < 3; ++z) {
          const int lab = (int)((w >> (4 * z)) & 15u);
          int id;
          if (lab < 3) {
            const int li = (lab - rot + 3) % 3;
            id = li == 0 ? nb.vid : (li == 1 ? c1 : c2);
          } else if (lab < 9) {
            const int x = lab - 3, rr = x & 1;
            const int le = ((x >> 1) - rot + 3) % 3;
            // local edge le of triangle t: (edge id, direction)
            const int eid = t == 0 ? (le == 0 ? 2 : (le == 1 ? 4 : 1)) : (le == 0 ? 0 : (le == 1 ? 3 : 2));
            const int dir = t == 0 ? (le == 0 ? 1 : -1) : (le == 2 ? -1 : 1);
            const int n = popc8((uint32_t)(r.xm >> (8 * eid)) & 255u);
            const int base = eid == 0 ? nb.b0 : (eid == 1 ? nb.b1 : (eid == 2 ? nb.b2 : (eid == 3 ? nb.b3 : nb.b4)));
            id = base + (dir > 0 ? rr : n - 1 - rr);
          } else {
            id = idI;
          }
          id3[z] = id;
        }
        const TriK k = trik(id3[0], id3[1], id3[2], cls | (side ? 0 : 0x80));
        if (j == 0) q0 = k; else if (j == 1) q1 = k; else if (j == 2) q2 = k; else if (j == 3) q3 = k; else q4 = k;
      }
    }
  }
  // sorting network for five keys (unused slots sort last)
  trik_cx(q0, q1); trik_cx(q3, q4); trik_cx(q2, q4); trik_cx(q2, q3); trik_cx(q0, q3);
  trik_cx(q0, q2); trik_cx(q1, q4); trik_cx(q1, q3); trik_cx(q1, q2);
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const TriK& k = j == 0 ? q0 : (j == 1 ? q1 : (j == 2 ? q2 : (j == 3 ? q3 : q4)));
    if (k.a != bigc) {
      tris[3 * tp + 0] = k.a;
      tris[3 * tp + 1] = k.b;
      tris[3 * tp + 2] = k.c;
      codes[tp] = (uint8_t)k.code;
      ++tp;
    }
  }
}

// Emit one owner.  For a slow owner `r` holds its classification.
SBMT_HD void emit_owner(const Geo& g, const Frame& f, uint32_t info, const Slow* r, const Nb& nb, int64_t to,
                        double* __restrict__ verts, int32_t* __restrict__ tris, uint8_t* __restrict__ codes) {
  const bool both = (g.flags & 1u) != 0;
  const int fg = info_fg(info);
  const int self = info_self(info);
  const double ux = lat_x(f.X), uy = lat_y(g.h, f.k);
  int64_t p = nb.vid;
  if (self) put_vertex(verts, p++, ux, uy);
  int64_t tp = to;
  const uint8_t ucode = both && !fg ? 0x80 : 0;
  if (!info_slow(info)) {
    if (info_ntb(info)) {
      tris[3 * tp + 0] = nb.vid; tris[3 * tp + 1] = nb.id_vdr; tris[3 * tp + 2] = nb.id_vdl;
      codes[tp] = ucode;
      ++tp;
    }
    if (info_nta(info)) {
      tris[3 * tp + 0] = nb.vid; tris[3 * tp + 1] = nb.id_vr; tris[3 * tp + 2] = nb.id_vdr;
      codes[tp] = ucode;
    }
    return;
  }
  // crossings on E0, E1, E2 in order from the owner: X = P + t (Q - P),
  // t = dP / (dP - dQ), dP = (V-U) x (P-U), dQ = (V-U) x (Q-U)
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int n = popc8((uint32_t)(r->xm >> (8 * e)) & 255u);
    const int vX = e == 0 ? f.X + 4 * g.h : (e == 1 ? f.X - 2 * g.h : f.X + 2 * g.h);
    const double vx = lat_x(vX), vy = lat_y(g.h, e == 0 ? f.k : f.k + 1);
    const double gx = vx - ux, gy = vy - uy;
#pragma unroll
    for (int re = 0; re < 2; ++re) {
      if (re < n) {
        const int sl = (int)((r->ord >> (8 * e + 4 * re)) & 15);
        const int pm = slot_p(r->seg, sl), qm = slot_q(r->seg, sl);
        const double px = 0.25 * (double)mid_x(g, f, pm), py = 0.25 * (double)mid_y(g, f, pm);
        const double qx = 0.25 * (double)mid_x(g, f, qm), qy = 0.25 * (double)mid_y(g, f, qm);
        const double dp = gx * (py - uy) - gy * (px - ux);
        const double dq = gx * (qy - uy) - gy * (qx - ux);
        const double tt = dp / (dp - dq);
        put_vertex(verts, p++, px + tt * (qx - px), py + tt * (qy - py));
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int m = (int)((r->tri >> (16 + 4 * t)) & 15u);
    if (m != 15) put_vertex(verts, p++, 0.25 * (double)mid_x(g, f, m), 0.25 * (double)mid_y(g, f, m));
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int cls = (int)((r->tri >> (8 * t)) & 31u);
    if (cls == 0) {
      if ((t == 0 ? info_ntb(info) : info_nta(info)) != 0) {
        tris[3 * tp + 0] = nb.vid;
        tris[3 * tp + 1] = t == 0 ? nb.id_vdr : nb.id_vr;
        tris[3 * tp + 2] = t == 0 ? nb.id_vdl : nb.id_vdr;
        codes[tp] = ucode;
        ++tp;
      }
    } else {
      emit_cut(g, *r, t, nb, tp, tris, codes);
    }
  }
}

}  // namespace sbmt
