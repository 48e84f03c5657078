// Per-owner classification of the SBMT hot path (gfx950 kernels).
//
// Every lattice vertex (k, i) of the equilateral grid "owns" its three
// forward edges (to (k,i+1), (k+1,i+o-1), (k+1,i+o), o = k mod 2) and two base
// triangles: Tb = [v(k,i), v(k+1,i+o), v(k+1,i+o-1)] (apex on row k) and
// Ta = [v(k,i), v(k,i+1), v(k+1,i+o)] (base on row k).  One thread classifies
// one owner:
//   1. the 3x3 coarse samples under the owner's parallelogram Tb u Ta;
//      uniform samples mean no boundary nearby (fast path);
//   2. otherwise the marching-squares segments of the 2x2 dual cells, exact
//      segment/edge crossing tests (Alg. 1 restricted to proper crossings),
//      the order of two crossings on an edge, the chain vertex inside each
//      triangle, the inside bit of the owner vertex;
//   3. the raw key of each cut triangle (Sec. 3.3.3), reduced to its class and
//      rotation by the lookup table (Alg. 2, step 1).
//
// Exact arithmetic: quarter-pixel integer coordinates ("x4 units").  Boundary
// points are even; grid vertex (k,i) is at X = -2h-3 + 4h*i + 2h*(k&1) (odd),
// Y = -4 + 2hk*sqrt3.  Every predicate is sign(A + B*sqrt3) with integer A, B
// and is never zero (x parity, irrationality of sqrt3).
#pragma once
#include <stdint.h>

#ifndef SBMT_HD
#define SBMT_HD __host__ __device__ __forceinline__
#endif

namespace sbmt {

constexpr int kRing = 4;  // background samples stored around the coarse raster

struct Geo {
  int32_t W, H;
  int64_t stride;
  int32_t h, s, CW, CH, NK, NI, NCB, wpr;
  int32_t X0;  // x4 x-coordinate of vertex (0,0) = -2h-3
  uint32_t flags;
};

// Sign of a + b*sqrt3.  Zero only for a = b = 0.
SBMT_HD int z3sign(int64_t a, int64_t b) {
  if (a >= 0 && b >= 0) return (a | b) != 0 ? 1 : 0;
  if (a <= 0 && b <= 0) return -1;
  int64_t a2 = a * a, b2 = 3 * b * b;
  return a > 0 ? (a2 > b2 ? 1 : -1) : (b2 > a2 ? 1 : -1);
}

SBMT_HD int64_t floordiv(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

// Cell row of grid row k: the largest R with 2sR + s + 1 <= k*h*sqrt3, i.e.
// floor((y_k - (s-1)/2) / s) for y_k = -1 + k h sqrt3 / 2.
SBMT_HD int row_cell(int k, int h, int s) {
  int64_t kh = (int64_t)k * h;
  // integer estimate from 1.732 < sqrt3 < 1.7321, then exact fix-up
  int64_t R = floordiv(kh * 17320 / 10000 - s - 1, 2 * s);
  while (z3sign(-(2 * s * R + s + 1), kh) < 0) --R;
  while (z3sign(-(2 * s * (R + 1) + s + 1), kh) >= 0) ++R;
  return (int)R;
}

// Lattice point: x (odd, x4 units), y = -4 + b*sqrt3.
struct LPt {
  int32_t x, b;
};
// Boundary point: x, y even x4 units.
struct BPt {
  int32_t x, y;
};
struct Seg {
  BPt p, q;   // p -> q, foreground on the left
  int8_t cell;
};

// orient(U, V, P) for lattice U, V and boundary P
SBMT_HD int orient_llb(LPt U, LPt V, BPt P) {
  int64_t dx = V.x - U.x;
  int64_t A = dx * (int64_t)(P.y + 4);
  int64_t B = -dx * (int64_t)U.b - (int64_t)(V.b - U.b) * (int64_t)(P.x - U.x);
  return z3sign(A, B);
}
// orient(P, Q, U) for boundary P, Q and lattice U
SBMT_HD int orient_bbl(BPt P, BPt Q, LPt U) {
  int64_t ex = Q.x - P.x, ey = Q.y - P.y;
  int64_t A = ex * (int64_t)(-4 - P.y) - ey * (int64_t)(U.x - P.x);
  int64_t B = ex * (int64_t)U.b;
  return z3sign(A, B);
}

// Marching squares, corners in positive order TL, TR, BR, BL (bit 0..3); edge
// midpoints 0 top, 1 right, 2 bottom, 3 left.  A segment runs from each
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
//  bit 0 self vertex emitted, 1-2 crossings on the right edge, 3-4 down-left,
//  5-6 down-right, 7 chain vertex in Tb, 8 chain vertex in Ta, 9-11 triangles
//  of Tb, 12-14 triangles of Ta, 15 slow path, 16 owner vertex inside,
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

// Full classification of one owner (slow path).
struct Owner {
  uint32_t info;
  int nseg;
  Seg seg[8];
  // crossings on the five edges E0 v->vr, E1 v->vdl, E2 v->vdr, E3 vr->vdr,
  // E4 vdl->vdr, in order from the edge's first vertex
  int8_t nx[5];
  int8_t xseg[5][2];
  int8_t xd[5][2];   // sign of orient(U, V, P) of the crossing segment
  int16_t cls[2];    // 0 uncut; Tb = 0, Ta = 1
  int8_t rot[2];
  int8_t hasI[2];
  BPt I[2];
};

// Local edges of the two triangles as (edge id, direction) in positive order.
SBMT_HD int tri_edge(int t, int j) {
  // Tb: (E2,+) (E4,-) (E1,-); Ta: (E0,+) (E3,+) (E2,-)
  return t == 0 ? (j == 0 ? 2 : (j == 1 ? 4 : 1)) : (j == 0 ? 0 : (j == 1 ? 3 : 2));
}
SBMT_HD int tri_dir(int t, int j) { return t == 0 ? (j == 0 ? 1 : -1) : (j == 2 ? -1 : 1); }

SBMT_HD bool bpt_eq(BPt a, BPt b) { return a.x == b.x && a.y == b.y; }

SBMT_HD uint32_t sample3(const uint32_t* bits, int wpr, int rr, int cc) {
  const uint32_t* row = bits + (int64_t)rr * wpr;
  int w = cc >> 5, b = cc & 31;
  uint64_t v = ((uint64_t)row[w + 1] << 32) | row[w];
  return (uint32_t)(v >> b) & 7u;
}

struct Frame {
  int X, Yb, o;        // owner vertex (x4 x, y coefficient of sqrt3), row parity
  int Rlo, Clo;        // top-left dual cell of the 2x2 block
  uint32_t s9;         // 3x3 samples, bit (3*r + c)
};

SBMT_HD Frame owner_frame(const Geo& g, const uint32_t* bits, int k, int i, int Rlo) {
  Frame f;
  f.o = k & 1;
  f.X = g.X0 + 4 * g.h * i + 2 * g.h * f.o;
  f.Yb = 2 * g.h * k;
  f.Rlo = Rlo;
  f.Clo = (int)floordiv((int64_t)f.X - 2 * g.h - 2 * (g.s - 1), 4 * g.s);
  int rr = Rlo + kRing, cc = f.Clo + kRing;
  f.s9 = sample3(bits, g.wpr, rr, cc) | (sample3(bits, g.wpr, rr + 1, cc) << 3) |
         (sample3(bits, g.wpr, rr + 2, cc) << 6);
  return f;
}

SBMT_HD int frame_sample(const Frame& f, int r, int c) { return (f.s9 >> (3 * r + c)) & 1; }

// Class lookup tables (generated): key code -> class | rot << 6, templates.
// Provided by the including translation unit.
SBMT_HD int lut_key(int code);
SBMT_HD int lut_nfg(int cls);
SBMT_HD int lut_ntri(int cls);
SBMT_HD uint16_t lut_tri(int cls, int j);

// Build the raw key of triangle t and look up its class.  Returns false on a
// protocol violation.
SBMT_HD bool classify_tri(Owner& o, int t) {
  int nc = 0;
  int ce[4], cr[4], cs[4], cent[4];
  for (int j = 0; j < 3; ++j) {
    int eid = tri_edge(t, j), dir = tri_dir(t, j);
    int ne = o.nx[eid];
    for (int r = 0; r < ne; ++r) {
      if (nc >= 4) return false;
      ce[nc] = j;
      cr[nc] = dir > 0 ? r : ne - 1 - r;
      cs[nc] = o.xseg[eid][r];
      int d = o.xd[eid][r];
      cent[nc] = dir > 0 ? (d < 0) : (d > 0);
      ++nc;
    }
  }
  o.cls[t] = 0;
  o.rot[t] = 0;
  if (nc == 0 && !o.hasI[t]) return true;
  int type, tok[4] = {0, 0, 0, 0};
  if (o.hasI[t]) {
    if (nc != 2) return false;
    int sin = -1, sout = -1;
    for (int a = 0; a < o.nseg; ++a) {
      if (bpt_eq(o.seg[a].q, o.I[t])) sin = a;
      if (bpt_eq(o.seg[a].p, o.I[t])) sout = a;
    }
    int jin = -1, jout = -1;
    for (int c = 0; c < 2; ++c) {
      if (cs[c] == sin) jin = c;
      if (cs[c] == sout) jout = c;
    }
    if (jin < 0 || jout < 0 || jin == jout || !cent[jin] || cent[jout]) return false;
    type = 2;
    tok[0] = 2 * ce[jin] + cr[jin];
    tok[1] = 2 * ce[jout] + cr[jout];
  } else if (nc == 2) {
    if (cs[0] != cs[1] || cent[0] == cent[1]) return false;
    int a = cent[0] ? 0 : 1, b = 1 - a;
    type = 1;
    tok[0] = 2 * ce[a] + cr[a];
    tok[1] = 2 * ce[b] + cr[b];
  } else if (nc == 4) {
    int sa = cs[0], sb = -1;
    for (int c = 1; c < 4; ++c)
      if (cs[c] != sa) sb = cs[c];
    if (sb < 0) return false;
    int s1, s2;
    if (bpt_eq(o.seg[sa].q, o.seg[sb].p)) { s1 = sa; s2 = sb; }
    else if (bpt_eq(o.seg[sb].q, o.seg[sa].p)) { s1 = sb; s2 = sa; }
    else return false;
    int slot[4] = {-1, -1, -1, -1};
    for (int c = 0; c < 4; ++c) {
      int base = cs[c] == s1 ? 0 : (cs[c] == s2 ? 2 : -1);
      if (base < 0) return false;
      int q = base + (cent[c] ? 0 : 1);
      if (slot[q] >= 0) return false;
      slot[q] = c;
    }
    type = 3;
    for (int q = 0; q < 4; ++q) tok[q] = 2 * ce[slot[q]] + cr[slot[q]];
  } else {
    return false;
  }
  int code = (type << 12) | (tok[0] << 9) | (tok[1] << 6) | (tok[2] << 3) | tok[3];
  int kv = lut_key(code);
  if (kv == 0) return false;
  o.cls[t] = (int16_t)(kv & 63);
  o.rot[t] = (int8_t)(kv >> 6);
  return true;
}

// Classify owner (k, i).  FULL = false computes only the packed counts and
// returns early on the fast path; FULL = true also keeps what emission needs.
template <bool FULL>
SBMT_HD void classify_owner(const Geo& g, const uint32_t* bits, int k, int i, int Rlo, Owner& o) {
  const bool both = (g.flags & 1u) != 0;
  const Frame f = owner_frame(g, bits, k, i, Rlo);
  const int h = g.h, s = g.s;
  // existence of the owned triangles inside the grid extent
  const bool tb_ok = (k + 1 < g.NK) && (i + f.o - 1 >= 0) && (i + f.o < g.NI);
  const bool ta_ok = (k + 1 < g.NK) && (i + 1 < g.NI) && (i + f.o < g.NI);
  o.nseg = 0;
  for (int e = 0; e < 5; ++e) o.nx[e] = 0;
  o.hasI[0] = o.hasI[1] = 0;
  o.cls[0] = o.cls[1] = 0;
  o.rot[0] = o.rot[1] = 0;
  if (f.s9 == 0 || f.s9 == 0x1ffu) {
    const int fg = f.s9 != 0;
    const int self = both ? 1 : fg;
    const int ntb = both ? (int)tb_ok : (fg & tb_ok);
    const int nta = both ? (int)ta_ok : (fg & ta_ok);
    o.info = (uint32_t)self | ((uint32_t)ntb << 9) | ((uint32_t)nta << 12) | ((uint32_t)fg << 16);
    return;
  }
  // --- slow path: segments of the four dual cells -------------------------
  for (int cr = 0; cr < 2; ++cr)
    for (int cc = 0; cc < 2; ++cc) {
      int c = frame_sample(f, cr, cc) | (frame_sample(f, cr, cc + 1) << 1) |
              (frame_sample(f, cr + 1, cc + 1) << 2) | (frame_sample(f, cr + 1, cc) << 3);
      uint16_t m = ms_case(c);
      int X0c = 4 * s * (f.Clo + cc) + 2 * (s - 1), Y0c = 4 * s * (f.Rlo + cr) + 2 * (s - 1);
      BPt mid[4] = {{X0c + 2 * s, Y0c}, {X0c + 4 * s, Y0c + 2 * s}, {X0c + 2 * s, Y0c + 4 * s},
                    {X0c, Y0c + 2 * s}};
      for (int q = 0; q < (m & 3); ++q) {
        int a = (m >> (2 + 4 * q)) & 3, b = (m >> (4 + 4 * q)) & 3;
        o.seg[o.nseg].p = mid[a];
        o.seg[o.nseg].q = mid[b];
        o.seg[o.nseg].cell = (int8_t)(2 * cr + cc);
        ++o.nseg;
      }
    }
  // --- the five edges --------------------------------------------------------
  const LPt v = {f.X, f.Yb}, vr = {f.X + 4 * h, f.Yb}, vdl = {f.X - 2 * h, f.Yb + 2 * h},
            vdr = {f.X + 2 * h, f.Yb + 2 * h};
  const LPt EU[5] = {v, v, v, vr, vdl};
  const LPt EV[5] = {vr, vdl, vdr, vdr, vdr};
  bool err = false;
  for (int e = 0; e < 5; ++e) {
    int xlo = EU[e].x < EV[e].x ? EU[e].x : EV[e].x, xhi = EU[e].x < EV[e].x ? EV[e].x : EU[e].x;
    for (int a = 0; a < o.nseg; ++a) {
      const Seg& sg = o.seg[a];
      int sxlo = sg.p.x < sg.q.x ? sg.p.x : sg.q.x, sxhi = sg.p.x < sg.q.x ? sg.q.x : sg.p.x;
      if (sxhi < xlo || sxlo > xhi) continue;
      int s1 = orient_llb(EU[e], EV[e], sg.p), s2 = orient_llb(EU[e], EV[e], sg.q);
      if (s1 == s2) continue;
      int s3 = orient_bbl(sg.p, sg.q, EU[e]), s4 = orient_bbl(sg.p, sg.q, EV[e]);
      if (s3 == s4) continue;
      if (o.nx[e] >= 2) { err = true; continue; }
      o.xseg[e][o.nx[e]] = (int8_t)a;
      o.xd[e][o.nx[e]] = (int8_t)s1;
      ++o.nx[e];
    }
    if (o.nx[e] == 2) {
      // two crossings on one edge come from consecutive segments S1 -> S2 that
      // share a vertex M; S2's crossing lies further along U->V iff
      // sign((P0 - M) x (P2 - M)) * sign(orient(U, V, M)) > 0
      int a = o.xseg[e][0], b = o.xseg[e][1];
      int s1i, s2i;
      if (bpt_eq(o.seg[a].q, o.seg[b].p)) { s1i = a; s2i = b; }
      else if (bpt_eq(o.seg[b].q, o.seg[a].p)) { s1i = b; s2i = a; }
      else { err = true; continue; }
      BPt M = o.seg[s1i].q, P0 = o.seg[s1i].p, P2 = o.seg[s2i].q;
      int64_t cx = (int64_t)(P0.x - M.x) * (P2.y - M.y) - (int64_t)(P0.y - M.y) * (P2.x - M.x);
      int lam = (cx > 0 ? 1 : -1) * orient_llb(EU[e], EV[e], M);
      int first = lam > 0 ? s1i : s2i;
      if (o.xseg[e][0] != first) {
        int8_t ts = o.xseg[e][0], td = o.xd[e][0];
        o.xseg[e][0] = o.xseg[e][1]; o.xd[e][0] = o.xd[e][1];
        o.xseg[e][1] = ts; o.xd[e][1] = td;
      }
    }
  }
  // --- chain vertices: midpoints between the centre sample and its neighbours
  {
    const int c0 = frame_sample(f, 1, 1);
    const int Xc = 4 * s * (f.Clo + 1) + 2 * (s - 1), Yc = 4 * s * (f.Rlo + 1) + 2 * (s - 1);
    const int nb[4][2] = {{0, 1}, {2, 1}, {1, 0}, {1, 2}};
    const BPt mp[4] = {{Xc, Yc - 2 * s}, {Xc, Yc + 2 * s}, {Xc - 2 * s, Yc}, {Xc + 2 * s, Yc}};
    for (int q = 0; q < 4; ++q) {
      if (frame_sample(f, nb[q][0], nb[q][1]) == c0) continue;
      BPt M = mp[q];
      int o0 = orient_llb(v, vdr, M), o4 = orient_llb(vdl, vdr, M), o1 = orient_llb(v, vdl, M);
      int oR = orient_llb(v, vr, M), o3 = orient_llb(vr, vdr, M);
      if (o0 > 0 && o4 < 0 && o1 < 0) {
        if (o.hasI[0]) err = true;
        o.hasI[0] = 1; o.I[0] = M;
      }
      if (oR > 0 && o3 > 0 && o0 < 0) {
        if (o.hasI[1]) err = true;
        o.hasI[1] = 1; o.I[1] = M;
      }
    }
  }
  // --- inside bit of the owner vertex ------------------------------------------
  int fg;
  {
    int cc = (int)(floordiv((int64_t)f.X - 2 * (s - 1), 4 * s) - f.Clo);
    int a = frame_sample(f, 0, cc), b = frame_sample(f, 0, cc + 1), c = frame_sample(f, 1, cc + 1),
        d = frame_sample(f, 1, cc);
    if (a == b && b == c && c == d) {
      fg = a;
    } else {
      fg = 1;
      for (int q = 0; q < o.nseg; ++q)
        if (o.seg[q].cell == cc && orient_bbl(o.seg[q].p, o.seg[q].q, v) < 0) fg = 0;
    }
  }
  // --- keys of the two triangles ----------------------------------------------
  for (int t = 0; t < 2; ++t)
    if (!classify_tri(o, t)) err = true;
  int ntri[2];
  for (int t = 0; t < 2; ++t) {
    bool ok = t == 0 ? tb_ok : ta_ok;
    if (o.cls[t] == 0)
      ntri[t] = ok && (both || fg) ? 1 : 0;
    else
      ntri[t] = both ? lut_ntri(o.cls[t]) : lut_nfg(o.cls[t]);
  }
  const int self = both ? 1 : fg;
  o.info = (uint32_t)self | ((uint32_t)o.nx[0] << 1) | ((uint32_t)o.nx[1] << 3) | ((uint32_t)o.nx[2] << 5) |
           ((uint32_t)o.hasI[0] << 7) | ((uint32_t)o.hasI[1] << 8) | ((uint32_t)ntri[0] << 9) |
           ((uint32_t)ntri[1] << 12) | (1u << 15) | ((uint32_t)fg << 16) |
           ((uint32_t)(o.cls[0] != 0) << 17) | ((uint32_t)(o.cls[1] != 0) << 18) | ((uint32_t)err << 19);
  (void)FULL;
}

// ---------------------------------------------------------------------------
// Emission of one owner (Alg. 2, steps 2-4): its vertices and the sub-triangles
// of its two base triangles, with global ids from the owner offsets.
// ---------------------------------------------------------------------------
constexpr double kHalfSqrt3 = 0.86602540378443864676;
SBMT_HD double lat_x(int X) { return 0.25 * (double)X; }
SBMT_HD double lat_y(int h, int k) { return -1.0 + (double)(h * k) * kHalfSqrt3; }

struct Tri {
  int a, b, c, code;
};

SBMT_HD void rot_min(Tri& t) {
  if (t.b < t.a && t.b < t.c) { int x = t.a; t.a = t.b; t.b = t.c; t.c = x; }
  else if (t.c < t.a && t.c < t.b) { int x = t.c; t.c = t.b; t.b = t.a; t.a = x; }
}
SBMT_HD bool tri_less(const Tri& x, const Tri& y) {
  return x.a != y.a ? x.a < y.a : (x.b != y.b ? x.b < y.b : x.c < y.c);
}

struct Nb {  // ids needed by one owner
  int vid;               // first vertex id of the owner
  int id_vr, id_vdl, id_vdr;
  int base[5];           // first crossing id on edges E0..E4
  int baseI;             // id of the chain vertex in Tb (Ta follows)
};

SBMT_HD int inst_label(int lab, int rot) {
  if (lab < 3) return (lab - rot + 3) % 3;
  if (lab < 9) {
    int x = lab - 3, e = x >> 1, r = x & 1;
    return 3 + 2 * ((e - rot + 3) % 3) + r;
  }
  return lab;
}

SBMT_HD void put_vertex(double* verts, int64_t p, double x, double y) {
  double2 v;
  v.x = x;
  v.y = y;
  reinterpret_cast<double2*>(verts)[p] = v;
}

SBMT_HD void emit_owner(const Geo& g, const uint32_t* bits, int k, int c, int Rlo, uint32_t info,
                           const Nb& nb, int64_t to, double* __restrict__ verts, int32_t* __restrict__ tris,
                           uint8_t* __restrict__ codes) {
  const bool both = (g.flags & 1u) != 0;
  const int o_ = k & 1;
  const int X = g.X0 + 4 * g.h * c + 2 * g.h * o_;
  const int fg = info_fg(info);
  const int self = info_self(info);
  if (!info_slow(info)) {
    if (self) put_vertex(verts, nb.vid, lat_x(X), lat_y(g.h, k));
    const uint8_t code = both && !fg ? 0x80 : 0;
    int64_t tp = to;
    if (info_ntb(info)) {
      tris[3 * tp + 0] = nb.vid; tris[3 * tp + 1] = nb.id_vdr; tris[3 * tp + 2] = nb.id_vdl;
      codes[tp] = code; ++tp;
    }
    if (info_nta(info)) {
      tris[3 * tp + 0] = nb.vid; tris[3 * tp + 1] = nb.id_vr; tris[3 * tp + 2] = nb.id_vdr;
      codes[tp] = code;
    }
    return;
  }
  Owner o;
  classify_owner<true>(g, bits, k, c, Rlo, o);
  // vertices: self, crossings on E0, E1, E2 (from the owner), chain vertices
  int64_t p = nb.vid;
  const double ux = lat_x(X), uy = lat_y(g.h, k);
  if (self) put_vertex(verts, p++, ux, uy);
  const int EVx[3] = {X + 4 * g.h, X - 2 * g.h, X + 2 * g.h};
  const int EVk[3] = {k, k + 1, k + 1};
  for (int e = 0; e < 3; ++e) {
    const double vx = lat_x(EVx[e]), vy = lat_y(g.h, EVk[e]);
    const double gx = vx - ux, gy = vy - uy;
    for (int r = 0; r < o.nx[e]; ++r) {
      const Seg& sg = o.seg[o.xseg[e][r]];
      const double px = 0.25 * (double)sg.p.x, py = 0.25 * (double)sg.p.y;
      const double qx = 0.25 * (double)sg.q.x, qy = 0.25 * (double)sg.q.y;
      const double dp = gx * (py - uy) - gy * (px - ux);
      const double dq = gx * (qy - uy) - gy * (qx - ux);
      const double t = dp / (dp - dq);
      put_vertex(verts, p++, px + t * (qx - px), py + t * (qy - py));
    }
  }
  for (int t = 0; t < 2; ++t)
    if (o.hasI[t]) put_vertex(verts, p++, 0.25 * (double)o.I[t].x, 0.25 * (double)o.I[t].y);
  // triangles of Tb then Ta
  int64_t tp = to;
  for (int t = 0; t < 2; ++t) {
    const int cid[3] = {nb.vid, t == 0 ? nb.id_vdr : nb.id_vr, t == 0 ? nb.id_vdl : nb.id_vdr};
    if (o.cls[t] == 0) {
      if ((t == 0 ? info_ntb(info) : info_nta(info)) == 0) continue;
      tris[3 * tp + 0] = cid[0]; tris[3 * tp + 1] = cid[1]; tris[3 * tp + 2] = cid[2];
      codes[tp] = both && !fg ? 0x80 : 0;
      ++tp;
      continue;
    }
    const int cls = o.cls[t], rot = o.rot[t];
    Tri out[5];
    int n = 0;
    for (int j = 0; j < lut_ntri(cls); ++j) {
      const uint16_t w = lut_tri(cls, j);
      const int side = (w >> 12) & 1;
      if (!both && !side) continue;
      int id3[3];
      for (int q = 0; q < 3; ++q) {
        const int lab = inst_label((w >> (4 * q)) & 15, rot);
        int id;
        if (lab < 3) {
          id = cid[lab];
        } else if (lab < 9) {
          const int e = (lab - 3) >> 1, r = (lab - 3) & 1;
          const int eid = tri_edge(t, e), dir = tri_dir(t, e);
          const int ne = o.nx[eid];
          id = nb.base[eid] + (dir > 0 ? r : ne - 1 - r);
        } else {
          id = nb.baseI + (t == 1 ? (int)o.hasI[0] : 0);
        }
        id3[q] = id;
      }
      Tri tr = {id3[0], id3[1], id3[2], cls | (side ? 0 : 0x80)};
      rot_min(tr);
      int q = n++;
      while (q > 0 && tri_less(tr, out[q - 1])) { out[q] = out[q - 1]; --q; }
      out[q] = tr;
    }
    for (int j = 0; j < n; ++j) {
      tris[3 * tp + 0] = out[j].a; tris[3 * tp + 1] = out[j].b; tris[3 * tp + 2] = out[j].c;
      codes[tp] = (uint8_t)out[j].code;
      ++tp;
    }
  }
}

}  // namespace sbmt
