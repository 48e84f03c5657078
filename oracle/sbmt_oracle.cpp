// SBMT CPU oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, deliberately slow and obviously-correct CPU implementation of the
// Structured Bitmap-to-Mesh Triangulation path (arXiv 2602.19474): bitmap ->
// boundary polylines -> exact segment/triangle classification (Alg. 1) ->
// symmetry-canonical key (Sec. 3.3.3, the key kappa(K)) -> template
// retriangulation (Alg. 2, App. G) -> closed mesh.
//
// Only the test-suite, the smoke check and the CPU-baseline leg of the
// benchmark may load this library.  It shares no code, header, table or
// generator with the HIP path.  It takes a different route on purpose:
//   * segment-driven and global (the HIP path is triangle-driven and local);
//   * contours are traced sequentially into closed polylines;
//   * crossings are found per segment and stored in a per-edge registry
//     (the frozen registry R of Assumption 1), sorted by the exact parameter
//     along the grid edge (products in Z[sqrt3], 128-bit);
//   * lattice vertices are labelled inside/outside by ray parity along rows;
//   * chain vertices are located by exact point location;
//   * each cut triangle is split into faces by face tracing and every face is
//     triangulated procedurally from the stated rule (no lookup table);
//   * class ids come from a brute-force enumeration of all admissible keys.
//
// Exact arithmetic.  The grid edge is a dyadic rational h = p / U, U = 2^q
// (q <= 8), and coordinates are kept in units of 1 / (4U) pixel.  Boundary
// points are multiples of 2U (even).  Grid vertex (k,i) sits at
// X = X0 + 4p*i + 2p*(k&1) with X0 odd (X0 = -2p-3 for integer h, else
// -(2p + 3U) - 1) and Y = -4U + 2pk*sqrt3.  Every orientation predicate is
// therefore A + B*sqrt3 with integer A, B and is decided exactly.  With the
// coarse stride rule s^2 > 2h^2 no predicate of the global path is ever zero
// (the oracle asserts it).
//
// The paper leaves several points open; the readings taken here (boundary by
// marching squares on a block-majority coarsened raster, rotation-only
// canonicalisation, the template rule for free cases, output numbering) are
// listed in the repository's design notes and restated where they are used.
//
// The main path is the "all rules off" regime of the ablation (no
// preprocessing); its meshes carry no angle or area bound.  A second path,
// oracle_mesh_preprocessed, runs the preprocessing of Alg. 3 first (vertex
// snapping a, repulsion c, edge elimination b) and retriangulates against the
// polyline in double precision; it is pinned by the bounds of Sec. 3.3.4 and
// App. D on every triangle, by the mesh invariants and by reducing exactly to
// the main path when every threshold is zero.  oracle_pre_grid stops after the
// three steps and returns the preprocessed grid (pinned by brute force over
// the polyline): that is the part with a GPU counterpart.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

typedef __int128 i128;
typedef int64_t i64;

namespace {

struct OracleError : std::runtime_error {
  explicit OracleError(const std::string& m) : std::runtime_error(m) {}
};
#define ORACLE_CHECK(cond, msg)                                                  \
  do {                                                                           \
    if (!(cond)) throw OracleError(std::string("oracle: ") + (msg));             \
  } while (0)

// ---------------------------------------------------------------------------
// Exact arithmetic in Z[sqrt3].
// ---------------------------------------------------------------------------
struct Z3 {  // a + b*sqrt(3)
  i128 a, b;
};
static Z3 z3_sub(Z3 p, Z3 q) { return {p.a - q.a, p.b - q.b}; }
static Z3 z3_mul(Z3 p, Z3 q) { return {p.a * q.a + 3 * p.b * q.b, p.a * q.b + p.b * q.a}; }
static Z3 z3_scale(Z3 p, i128 s) { return {p.a * s, p.b * s}; }

// Sign of a + b*sqrt3, decided exactly: if both parts agree that is the sign,
// otherwise compare a^2 with 3b^2.
static int z3_sign(Z3 v) {
  i128 a = v.a, b = v.b;
  if (a >= 0 && b >= 0) return (a == 0 && b == 0) ? 0 : 1;
  if (a <= 0 && b <= 0) return -1;
  // opposite signs; |a|, |b| < 2^62 here so the squares fit in 128 bits
  i128 a2 = a * a, b2 = 3 * b * b;
  if (a > 0) return a2 > b2 ? 1 : (a2 < b2 ? -1 : 0);
  return b2 > a2 ? 1 : (b2 < a2 ? -1 : 0);
}

// A point whose x is an integer and whose y lies in Z[sqrt3].
struct Pt {
  i64 x;
  i64 ya, yb;  // y = ya + yb*sqrt3
};

// orient(p,q,r) = (q-p) x (r-p); x parts are rational so the result is in Z[sqrt3].
static Z3 orient(const Pt& p, const Pt& q, const Pt& r) {
  i128 qx = q.x - p.x, rx = r.x - p.x;
  Z3 qy{(i128)q.ya - p.ya, (i128)q.yb - p.yb};
  Z3 ry{(i128)r.ya - p.ya, (i128)r.yb - p.yb};
  return z3_sub(z3_scale(ry, qx), z3_scale(qy, rx));
}
static int orient_sign(const Pt& p, const Pt& q, const Pt& r) { return z3_sign(orient(p, q, r)); }

// ---------------------------------------------------------------------------
// Crossing parameter order along a directed edge U->V.
// A segment P->Q crossing the edge does so at mu = oU/(oU-oV) with
// oU = orient(P,Q,U), oV = orient(P,Q,V).  mu1 < mu2 is decided exactly by
// cross multiplication: sign(mu1-mu2) = sign(o2U*o1V - o1U*o2V)*sign(o1U)*sign(o2U).
// ---------------------------------------------------------------------------
static int mu_compare(Z3 o1U, Z3 o1V, Z3 o2U, Z3 o2V) {
  Z3 num = z3_sub(z3_mul(o2U, o1V), z3_mul(o1U, o2V));
  int s = z3_sign(num) * z3_sign(o1U) * z3_sign(o2U);
  return s;  // <0: mu1 < mu2
}

// ---------------------------------------------------------------------------
// Local configuration of one cut base triangle K and its template.
//
// Labels: corners c0,c1,c2 (positive orientation) -> 0,1,2; crossing slot
// X(e,r) on local edge e (c_e -> c_{e+1}) with rank r along that direction
// -> 3 + 2e + r; the chain vertex inside K (if any) -> 9.
//
// Key (Sec. 3.3.3): type 1 = one chord, type 2 = chain vertex inside,
// type 3 = two chords of consecutive segments.  Tokens follow chain order:
//   type 1: (entry, exit), type 2: (entry of S1, exit of S2),
//   type 3: (S1 entry, S1 exit, S2 entry, S2 exit), token X(e,r) = 2e + r.
// code = type*4096 + t0*512 + t1*64 + t2*8 + t3.
// The symmetry tag is the rotation j in {0,1,2} (e -> e+j mod 3) giving the
// smallest code (first such j); mirror images are distinct atomic cases
// (App. G, orientation handling), so reflections are not used.
// ---------------------------------------------------------------------------
struct Desc {
  int type = 0;
  int tok[4] = {0, 0, 0, 0};
};
static int desc_ntok(int type) { return type == 3 ? 4 : (type == 0 ? 0 : 2); }
static int desc_code(const Desc& d) {
  return d.type * 4096 + d.tok[0] * 512 + d.tok[1] * 64 + d.tok[2] * 8 + d.tok[3];
}
static Desc desc_rotate(const Desc& d, int j) {
  Desc r = d;
  for (int t = 0; t < desc_ntok(d.type); ++t) {
    int e = d.tok[t] / 2, rk = d.tok[t] % 2;
    r.tok[t] = 2 * ((e + j) % 3) + rk;
  }
  return r;
}
static void desc_canonical(const Desc& d, int* canon_code, int* rot) {
  int best = -1, bj = 0;
  for (int j = 0; j < 3; ++j) {
    int c = desc_code(desc_rotate(d, j));
    if (best < 0 || c < best) { best = c; bj = j; }
  }
  *canon_code = best;
  *rot = bj;
}

struct Tri3 {
  int v[3];
  int side;  // 1 = left of the chain (foreground), 0 = right
};

// Chain pieces of a configuration, as label pairs in chain direction.
struct LocalTemplate {
  bool ok = false;
  std::string why;
  std::vector<Tri3> tris;
};

// Cyclic boundary sequence of K: c0, X(0,0), X(0,1), c1, X(1,0), ... as labels
// restricted to the labels present.
static std::vector<int> boundary_cycle(const std::vector<int>& present_slots) {
  std::vector<int> cyc;
  for (int e = 0; e < 3; ++e) {
    cyc.push_back(e);
    for (int r = 0; r < 2; ++r) {
      int lab = 3 + 2 * e + r;
      if (std::find(present_slots.begin(), present_slots.end(), lab) != present_slots.end())
        cyc.push_back(lab);
    }
  }
  return cyc;
}

// Procedural triangulation of the key's faces (the template rule of App. G as
// read here):
//  * a face containing the chain vertex I is fanned from I (App. G, (1,1));
//  * the face between two nested chords (four crossings, no corner) is split
//    by the diagonal joining the exit crossings of the two chords
//    (App. G (2,2) cases d3 and a4);
//  * every other face is fanned from its chain-earliest crossing
//    (App. G single case (b), (2,2) case b1).
// Faces are found by tracing half-edges with the face on the left; the side of
// a face is "left" (foreground) when it uses a chain piece in chain direction.
static LocalTemplate triangulate(const Desc& d) {
  LocalTemplate out;
  const int I = 9;
  std::vector<int> slots;
  for (int t = 0; t < desc_ntok(d.type); ++t) slots.push_back(3 + d.tok[t]);
  // chain pieces (from,to) in chain direction, and chain position of labels
  std::vector<std::pair<int, int>> pieces;
  std::map<int, int> chainpos;
  if (d.type == 1) {
    pieces.push_back({slots[0], slots[1]});
    chainpos[slots[0]] = 0; chainpos[slots[1]] = 1;
  } else if (d.type == 2) {
    pieces.push_back({slots[0], I});
    pieces.push_back({I, slots[1]});
    chainpos[slots[0]] = 0; chainpos[I] = 1; chainpos[slots[1]] = 2;
  } else if (d.type == 3) {
    pieces.push_back({slots[0], slots[1]});
    pieces.push_back({slots[2], slots[3]});
    for (int t = 0; t < 4; ++t) chainpos[slots[t]] = t;
  } else {
    out.why = "bad type";
    return out;
  }
  std::vector<int> cyc = boundary_cycle(slots);
  const int n = (int)cyc.size();
  auto cyc_next = [&](int lab) {
    for (int j = 0; j < n; ++j)
      if (cyc[j] == lab) return cyc[(j + 1) % n];
    return -1;
  };
  // chain half-edge leaving a label (at most one per crossing; two at I)
  struct HE { int a, b; bool fwd; };
  std::vector<HE> chain_he;
  for (auto& p : pieces) {
    chain_he.push_back({p.first, p.second, true});
    chain_he.push_back({p.second, p.first, false});
  }
  // trace faces
  std::map<std::pair<int, int>, bool> used;
  std::vector<std::vector<int>> faces;
  std::vector<int> face_side;
  auto trace = [&](int a0, int b0, bool start_is_chain) -> bool {
    std::vector<int> face;
    int a = a0, b = b0;
    bool via_chain = start_is_chain;
    int side = -1;
    for (int guard = 0; guard < 32; ++guard) {
      if (used[{a, b}]) return false;
      used[{a, b}] = true;
      face.push_back(a);
      if (via_chain) {
        bool fwd = false;
        for (auto& h : chain_he)
          if (h.a == a && h.b == b) fwd = h.fwd;
        int s = fwd ? 1 : 0;
        if (side >= 0 && side != s) return false;  // inconsistent sides
        side = s;
      }
      // choose the next half-edge out of b
      int na = b, nb = -1;
      bool nchain = false;
      if (b == I) {
        for (auto& h : chain_he)
          if (h.a == I && h.b != a) { nb = h.b; }
        nchain = true;
      } else if (!via_chain && b >= 3) {
        for (auto& h : chain_he)
          if (h.a == b) { nb = h.b; }
        nchain = true;
      } else {
        nb = cyc_next(b);
        nchain = false;
      }
      if (nb < 0) return false;
      a = na; b = nb; via_chain = nchain;
      if (a == a0 && b == b0) {
        if (side < 0) return false;  // a face touching no chain piece
        faces.push_back(face);
        face_side.push_back(side);
        return true;
      }
    }
    return false;
  };
  for (int j = 0; j < n; ++j) {
    int a = cyc[j], b = cyc[(j + 1) % n];
    if (!used[{a, b}])
      if (!trace(a, b, false)) { out.why = "face tracing failed"; return out; }
  }
  for (auto& h : chain_he)
    if (!used[{h.a, h.b}]) { out.why = "unused chain half-edge"; return out; }
  // every boundary piece and chain piece must have been used exactly once;
  // total angle check is implicit in the consistent traversal.
  for (size_t f = 0; f < faces.size(); ++f) {
    const std::vector<int>& F = faces[f];
    int m = (int)F.size();
    if (m < 3) { out.why = "degenerate face"; return out; }
    int apex = -1;
    bool hasI = std::find(F.begin(), F.end(), I) != F.end();
    int ncorner = 0, ncross = 0;
    for (int lab : F) { if (lab < 3) ++ncorner; else if (lab != I) ++ncross; }
    if (hasI) {
      apex = I;
    } else if (d.type == 3 && ncorner == 0 && ncross == 4) {
      apex = slots[1];  // exit of S1; the diagonal reaches the exit of S2
      // the exit of S2 must be opposite the apex
      int pa = (int)(std::find(F.begin(), F.end(), apex) - F.begin());
      if (F[(pa + 2) % 4] != slots[3]) { out.why = "nested exits not opposite"; return out; }
    } else {
      int bestpos = 1 << 30;
      for (int lab : F)
        if (lab >= 3 && lab != I && chainpos.count(lab) && chainpos[lab] < bestpos) {
          bestpos = chainpos[lab];
          apex = lab;
        }
    }
    if (apex < 0) { out.why = "no apex"; return out; }
    int pa = (int)(std::find(F.begin(), F.end(), apex) - F.begin());
    for (int t = 1; t + 1 < m; ++t) {
      Tri3 tr;
      tr.v[0] = apex;
      tr.v[1] = F[(pa + t) % m];
      tr.v[2] = F[(pa + t + 1) % m];
      tr.side = face_side[f];
      out.tris.push_back(tr);
    }
  }
  out.ok = true;
  return out;
}

// Combinatorial admissibility of a key: slots distinct, ranks on an edge
// form {0} or {0,1}, chords join different edges, chords do not cross, and
// the induced faces carry consistent sides.
static bool desc_admissible(const Desc& d) {
  int nt = desc_ntok(d.type);
  if (nt == 0) return false;
  for (int a = 0; a < nt; ++a) {
    if (d.tok[a] < 0 || d.tok[a] > 5) return false;
    for (int b = a + 1; b < nt; ++b)
      if (d.tok[a] == d.tok[b]) return false;
  }
  for (int t = nt; t < 4; ++t)
    if (d.tok[t] != 0) return false;
  for (int e = 0; e < 3; ++e) {
    bool r0 = false, r1 = false;
    for (int t = 0; t < nt; ++t) {
      if (d.tok[t] == 2 * e) r0 = true;
      if (d.tok[t] == 2 * e + 1) r1 = true;
    }
    if (r1 && !r0) return false;
  }
  if (d.type == 1 || d.type == 3) {
    for (int c = 0; c < nt; c += 2)
      if (d.tok[c] / 2 == d.tok[c + 1] / 2) return false;
  }
  if (d.type == 3) {
    // positions on the boundary cycle: slot X(e,r) at 3e+1+r
    auto pos = [](int tok) { return 3 * (tok / 2) + 1 + tok % 2; };
    int a1 = pos(d.tok[0]), b1 = pos(d.tok[1]), a2 = pos(d.tok[2]), b2 = pos(d.tok[3]);
    int lo = std::min(a1, b1), hi = std::max(a1, b1);
    bool in2a = (a2 > lo && a2 < hi), in2b = (b2 > lo && b2 < hi);
    if (in2a != in2b) return false;  // chords cross
  }
  LocalTemplate t = triangulate(d);
  return t.ok;
}

static std::vector<int>& class_table() {
  static std::vector<int> table;
  if (!table.empty()) return table;
  std::vector<int> canon;
  for (int type = 1; type <= 3; ++type) {
    int nt = desc_ntok(type);
    int lim[4] = {6, 6, nt > 2 ? 6 : 1, nt > 3 ? 6 : 1};
    for (int a = 0; a < lim[0]; ++a)
      for (int b = 0; b < lim[1]; ++b)
        for (int c = 0; c < lim[2]; ++c)
          for (int e = 0; e < lim[3]; ++e) {
            Desc d;
            d.type = type;
            d.tok[0] = a; d.tok[1] = b; d.tok[2] = c; d.tok[3] = e;
            if (!desc_admissible(d)) continue;
            int cc, rot;
            desc_canonical(d, &cc, &rot);
            canon.push_back(cc);
          }
  }
  std::sort(canon.begin(), canon.end());
  canon.erase(std::unique(canon.begin(), canon.end()), canon.end());
  table = canon;
  return table;
}
static int class_id_of(int canon_code) {
  std::vector<int>& t = class_table();
  auto it = std::lower_bound(t.begin(), t.end(), canon_code);
  ORACLE_CHECK(it != t.end() && *it == canon_code, "key not in the admissible class table");
  return 1 + (int)(it - t.begin());
}

// ---------------------------------------------------------------------------
// Generic per-triangle classification (Alg. 1 restricted to proper crossings).
// Input: corners (positive orientation), the crossings found on each edge with
// the segment that makes them, and an optional chain vertex inside K.
// ---------------------------------------------------------------------------
struct LocalCrossing {
  int edge;      // local edge e (c_e -> c_{e+1})
  int rank;      // order along c_e -> c_{e+1}
  i64 seg;       // segment id
  bool entry;    // segment passes from outside to inside here
};
struct LocalInput {
  std::vector<LocalCrossing> xs;
  bool has_I = false;
  i64 seg_in = -1, seg_out = -1;  // segments ending / starting at I
  // chain order between two segments: first segment of a consecutive pair
  i64 first_seg = -1;
};

struct LocalResult {
  Desc d;
  int code = 0, canon = 0, rot = 0, cls = 0;
  int slot_seg[6];
  LocalTemplate tmpl;
};

static LocalResult classify_local(const LocalInput& in) {
  LocalResult r;
  for (int j = 0; j < 6; ++j) r.slot_seg[j] = -1;
  auto tok_of = [](const LocalCrossing& c) { return 2 * c.edge + c.rank; };
  const int nx = (int)in.xs.size();
  if (in.has_I) {
    ORACLE_CHECK(nx == 2, "protocol: a chain vertex inside K needs exactly two crossings");
    const LocalCrossing* cin = nullptr;
    const LocalCrossing* cout = nullptr;
    for (auto& c : in.xs) {
      if (c.seg == in.seg_in) cin = &c;
      if (c.seg == in.seg_out) cout = &c;
    }
    ORACLE_CHECK(cin && cout && cin != cout, "protocol: crossings do not match the chain at I");
    ORACLE_CHECK(cin->entry && !cout->entry, "protocol: entry/exit at I inconsistent");
    r.d.type = 2;
    r.d.tok[0] = tok_of(*cin);
    r.d.tok[1] = tok_of(*cout);
    r.slot_seg[r.d.tok[0]] = (int)cin->seg;
    r.slot_seg[r.d.tok[1]] = (int)cout->seg;
  } else if (nx == 2) {
    ORACLE_CHECK(in.xs[0].seg == in.xs[1].seg, "protocol: two crossings from different segments");
    const LocalCrossing& a = in.xs[0].entry ? in.xs[0] : in.xs[1];
    const LocalCrossing& b = in.xs[0].entry ? in.xs[1] : in.xs[0];
    ORACLE_CHECK(a.entry && !b.entry, "protocol: chord without entry/exit");
    r.d.type = 1;
    r.d.tok[0] = tok_of(a);
    r.d.tok[1] = tok_of(b);
    r.slot_seg[r.d.tok[0]] = (int)a.seg;
    r.slot_seg[r.d.tok[1]] = (int)b.seg;
  } else if (nx == 4) {
    ORACLE_CHECK(in.first_seg >= 0, "protocol: two chords need a chain order");
    const LocalCrossing *e1 = nullptr, *x1 = nullptr, *e2 = nullptr, *x2 = nullptr;
    int n1 = 0, n2 = 0;
    for (auto& c : in.xs) {
      bool first = (c.seg == in.first_seg);
      if (first) ++n1; else ++n2;
      if (first && c.entry) e1 = &c;
      if (first && !c.entry) x1 = &c;
      if (!first && c.entry) e2 = &c;
      if (!first && !c.entry) x2 = &c;
    }
    ORACLE_CHECK(n1 == 2 && n2 == 2 && e1 && x1 && e2 && x2, "protocol: two chords malformed");
    r.d.type = 3;
    r.d.tok[0] = tok_of(*e1); r.d.tok[1] = tok_of(*x1);
    r.d.tok[2] = tok_of(*e2); r.d.tok[3] = tok_of(*x2);
    r.slot_seg[r.d.tok[0]] = (int)e1->seg; r.slot_seg[r.d.tok[1]] = (int)x1->seg;
    r.slot_seg[r.d.tok[2]] = (int)e2->seg; r.slot_seg[r.d.tok[3]] = (int)x2->seg;
  } else {
    ORACLE_CHECK(false, "protocol: unsupported number of crossings on a base triangle");
  }
  r.code = desc_code(r.d);
  desc_canonical(r.d, &r.canon, &r.rot);
  r.cls = class_id_of(r.canon);
  r.tmpl = triangulate(r.d);
  ORACLE_CHECK(r.tmpl.ok, "template construction failed: " + r.tmpl.why);
  return r;
}

// ---------------------------------------------------------------------------
// Global pipeline.
// ---------------------------------------------------------------------------
struct Segment {
  Pt p, q;       // x4 units, p -> q with the foreground on the left
  i64 next = -1, prev = -1;
  i64 contour = -1;
};

struct Crossing {
  i64 edge_key;  // ((k*NI + i)*3 + d), d: 0 right, 1 down-left, 2 down-right
  i64 seg;
  int rank = 0;  // order from the edge owner along the edge
  i64 vid = -1;
  double x = 0, y = 0;
};

struct ChainVertex {
  i64 tri_key;   // (k*NI + i)*2 + t, t: 0 = apex-on-row-k triangle, 1 = base-on-row-k
  i64 seg_out;   // segment starting here
  i64 vid = -1;
};

struct Mesh {
  std::vector<double> verts;   // 2 per vertex
  std::vector<int32_t> tris;   // 3 per triangle
  std::vector<uint8_t> codes;
  i64 n_segments = 0, n_cut = 0, n_contours = 0;
  std::vector<i64> chain_xy;   // all segment start points, x4 units, contour by contour
  std::vector<i64> chain_start;
  int32_t NK = 0, NI = 0, s = 0;
};

static const double kHalfSqrt3 = 0.86602540378443864676;

class Oracle {
 public:
  Oracle(const uint8_t* bm, int W, int H, i64 stride, double grid_h, unsigned flags)
      : bm_(bm), W_(W), H_(H), stride_(stride), both_(flags & 1u) {
    // grid_h = p / 2^q exactly, q <= 8, reduced
    ORACLE_CHECK(grid_h > 0 && grid_h <= 64, "invalid grid edge");
    const double g256 = grid_h * 256.0;
    ORACLE_CHECK(g256 == std::floor(g256), "grid edge is not a multiple of 1/256");
    h_ = (i64)g256;
    U_ = 256;
    while (U_ > 1 && h_ % 2 == 0) { h_ /= 2; U_ /= 2; }
    ORACLE_CHECK(W >= 0 && H >= 0, "invalid arguments");
    ORACLE_CHECK(W == 0 || H == 0 || stride >= W, "row stride smaller than width");
    s_ = 1;
    while ((i64)s_ * s_ * U_ * U_ <= 2LL * h_ * h_) ++s_;  // smallest s with s^2 > 2h^2
    X0_ = U_ == 1 ? -2 * h_ - 3 : -(2 * h_ + 3 * U_) - 1;  // odd
    CW_ = (W + s_ - 1) / s_;
    CH_ = (H + s_ - 1) / s_;
    // rows: smallest m >= 1 with 3 m^2 h^2 > (2 s CH + 1)^2, NK = m + 1
    i64 m = 1;
    i128 rhs = (i128)U_ * U_ * (2LL * s_ * CH_ + 1) * (2LL * s_ * CH_ + 1);
    while ((i128)3 * m * m * h_ * h_ <= rhs) ++m;
    NK_ = m + 1;
    // columns: the last vertex lies right of x = s CW - 1/2
    NI_ = (4LL * U_ * s_ * CW_ - 2LL * U_ - X0_) / (4LL * h_) + 2;
  }

  // The polylines, grid and exact inside labels of the lattice vertices, for
  // the preprocessing pass of Alg. 3 (PreOracle below).
  struct Traced {
    std::vector<double> px, py;      // polyline vertex j = start of segment j, pixels
    std::vector<i64> next, prev;     // segment links along the closed contours
    std::vector<uint8_t> inside;     // lattice vertex (k, i) inside the polylines
    i64 NK = 0, NI = 0;
    int s = 1;
    double h = 1;
    std::vector<double> lx, ly;      // lattice vertex positions, pixels (lx per vertex, ly per row)
  };
  Traced traced() {
    coarsen();
    trace();
    build_registry();
    label_inside();
    Traced t;
    for (const Segment& sg : segs_) {
      t.px.push_back(to_px(sg.p.x));
      t.py.push_back(to_px(sg.p.ya));
      t.next.push_back(sg.next);
      t.prev.push_back(sg.prev);
    }
    t.inside = inside_;
    t.NK = NK_;
    t.NI = NI_;
    t.s = s_;
    t.h = (double)h_ / (double)U_;
    t.lx.resize((size_t)(NK_ * NI_));
    t.ly.resize((size_t)NK_);
    for (i64 k = 0; k < NK_; ++k) {
      t.ly[(size_t)k] = lat_yd(k);
      for (i64 i = 0; i < NI_; ++i) t.lx[(size_t)(k * NI_ + i)] = lat_xd(k, i);
    }
    return t;
  }

  Mesh run() {
    coarsen();
    trace();
    build_registry();
    locate_chain_vertices();
    label_inside();
    number_vertices();
    emit_triangles();
    mesh_.NK = (int32_t)NK_;
    mesh_.NI = (int32_t)NI_;
    mesh_.s = s_;
    return std::move(mesh_);
  }

 private:
  const uint8_t* bm_;
  int W_, H_;
  i64 stride_;
  i64 h_ = 1;   // grid edge numerator: h = h_ / U_ pixels
  i64 U_ = 1;   // 2^q: one coordinate unit is 1 / (4 U_) pixel
  i64 X0_ = 0;  // x of vertex (0, 0), odd
  bool both_;
  int s_ = 1;
  i64 CW_ = 0, CH_ = 0, NK_ = 0, NI_ = 0;
  std::vector<uint8_t> coarse_;
  std::vector<Segment> segs_;
  std::vector<Crossing> reg_;         // sorted by (edge_key, rank)
  std::vector<ChainVertex> chain_;    // sorted by tri_key
  std::vector<uint8_t> inside_;       // NK*NI
  std::vector<i64> lattice_id_;       // NK*NI, -1 if not a vertex
  std::vector<i64> cut_tris_;         // sorted unique tri keys
  Mesh mesh_;

  // --- geometry of the lattice -------------------------------------------
  Pt lat(i64 k, i64 i) const {
    return Pt{X0_ + 4LL * h_ * i + 2LL * h_ * (k & 1), -4 * U_, 2LL * h_ * k};
  }
  bool lat_ok(i64 k, i64 i) const { return k >= 0 && k < NK_ && i >= 0 && i < NI_; }
  // pixel coordinates (exact scalings by powers of two)
  double to_px(i64 v) const { return (double)v * (0.25 / (double)U_); }
  double lat_xd(i64 k, i64 i) const { return to_px(lat(k, i).x); }
  double lat_yd(i64 k) const { return -1.0 + ((double)(h_ * k) * (1.0 / (double)U_)) * kHalfSqrt3; }

  // endpoints of edge d of owner (k,i): 0 -> (k,i+1), 1 -> (k+1,i+o-1), 2 -> (k+1,i+o)
  void edge_ends(i64 k, i64 i, int d, i64* k2, i64* i2) const {
    i64 o = k & 1;
    if (d == 0) { *k2 = k; *i2 = i + 1; }
    else if (d == 1) { *k2 = k + 1; *i2 = i + o - 1; }
    else { *k2 = k + 1; *i2 = i + o; }
  }
  i64 ekey(i64 k, i64 i, int d) const { return (k * NI_ + i) * 3 + d; }
  i64 tkey(i64 k, i64 i, int t) const { return (k * NI_ + i) * 2 + t; }

  // corners of base triangle t of owner (k,i), positive orientation
  //  t = 0: [v(k,i), v(k+1,i+o), v(k+1,i+o-1)]  (apex on row k)
  //  t = 1: [v(k,i), v(k,i+1), v(k+1,i+o)]      (base on row k)
  void tri_corners(i64 k, i64 i, int t, i64 ck[3], i64 ci[3]) const {
    i64 o = k & 1;
    ck[0] = k; ci[0] = i;
    if (t == 0) { ck[1] = k + 1; ci[1] = i + o; ck[2] = k + 1; ci[2] = i + o - 1; }
    else { ck[1] = k; ci[1] = i + 1; ck[2] = k + 1; ci[2] = i + o; }
  }
  bool tri_exists(i64 k, i64 i, int t) const {
    i64 ck[3], ci[3];
    tri_corners(k, i, t, ck, ci);
    for (int j = 0; j < 3; ++j)
      if (!lat_ok(ck[j], ci[j])) return false;
    return true;
  }

  // --- step 1: block-majority coarsening ----------------------------------
  void coarsen() {
    coarse_.assign((size_t)(CW_ * CH_), 0);
    for (i64 R = 0; R < CH_; ++R)
      for (i64 C = 0; C < CW_; ++C) {
        i64 cnt = 0;
        for (i64 r = s_ * R; r < std::min<i64>(s_ * R + s_, H_); ++r)
          for (i64 c = s_ * C; c < std::min<i64>(s_ * C + s_, W_); ++c)
            if (bm_[r * stride_ + c] != 0) ++cnt;
        coarse_[R * CW_ + C] = (2 * cnt >= (i64)s_ * s_) ? 1 : 0;
      }
  }
  int sample(i64 R, i64 C) const {
    if (R < 0 || R >= CH_ || C < 0 || C >= CW_) return 0;
    return coarse_[R * CW_ + C];
  }

  // --- step 2: marching squares + sequential contour tracing --------------
  void trace() {
    // segments of every dual cell, keyed by their start point
    std::unordered_map<i64, i64> start_at;
    auto pkey = [](i64 X, i64 Y) { return (X + (1LL << 30)) * (1LL << 31) + (Y + (1LL << 30)); };
    for (i64 R = -1; R < CH_; ++R)
      for (i64 C = -1; C < CW_; ++C) {
        // corners in positive order TL, TR, BR, BL
        int v[4] = {sample(R, C), sample(R, C + 1), sample(R + 1, C + 1), sample(R + 1, C)};
        if (v[0] == v[1] && v[1] == v[2] && v[2] == v[3]) continue;
        // sample (R, C) sits at pixel (s C + (s-1)/2, s R + (s-1)/2)
        i64 X0 = U_ * (4LL * s_ * C + 2LL * (s_ - 1)), Y0 = U_ * (4LL * s_ * R + 2LL * (s_ - 1));
        const i64 hs = 2 * s_ * U_;  // half a cell
        i64 mx[4] = {X0 + hs, X0 + 2 * hs, X0 + hs, X0};
        i64 my[4] = {Y0, Y0 + hs, Y0 + 2 * hs, Y0 + hs};
        // a segment starts at each fg->bg transition (walking corners in positive
        // order) and ends at the next bg->fg transition; background corners are
        // cut off, so foreground is 8-connected at saddles.
        for (int j = 0; j < 4; ++j) {
          if (!(v[j] == 1 && v[(j + 1) % 4] == 0)) continue;
          int t = (j + 1) % 4;
          while (!(v[t] == 0 && v[(t + 1) % 4] == 1)) t = (t + 1) % 4;
          Segment sg;
          sg.p = Pt{mx[j], my[j], 0};
          sg.q = Pt{mx[t], my[t], 0};
          start_at[pkey(sg.p.x, sg.p.ya)] = (i64)segs_.size();
          segs_.push_back(sg);
        }
      }
    // link and walk the closed contours in order
    for (size_t a = 0; a < segs_.size(); ++a) {
      auto it = start_at.find(pkey(segs_[a].q.x, segs_[a].q.ya));
      ORACLE_CHECK(it != start_at.end(), "open contour");
      segs_[a].next = it->second;
      segs_[it->second].prev = (i64)a;
    }
    i64 ncont = 0;
    std::vector<Segment> ordered;
    std::vector<i64> newid(segs_.size(), -1);
    for (size_t a = 0; a < segs_.size(); ++a) {
      if (newid[a] >= 0) continue;
      mesh_.chain_start.push_back((i64)ordered.size());
      i64 cur = (i64)a;
      do {
        newid[cur] = (i64)ordered.size();
        Segment sg = segs_[cur];
        sg.contour = ncont;
        ordered.push_back(sg);
        cur = segs_[cur].next;
      } while (cur != (i64)a);
      ++ncont;
    }
    mesh_.chain_start.push_back((i64)ordered.size());
    for (auto& sg : ordered) {
      sg.next = newid[sg.next];
      sg.prev = newid[sg.prev];
    }
    segs_.swap(ordered);
    // protocol of Sec. 3.2: segment lengths s/sqrt2 or s, turns of at most 90 deg
    for (auto& sg : segs_) {
      i64 dx = sg.q.x - sg.p.x, dy = sg.q.ya - sg.p.ya;
      i64 l2 = dx * dx + dy * dy;
      ORACLE_CHECK(l2 == 8LL * s_ * s_ * U_ * U_ || l2 == 16LL * s_ * s_ * U_ * U_, "segment length");
      const Segment& nx = segs_[sg.next];
      i64 ex = nx.q.x - nx.p.x, ey = nx.q.ya - nx.p.ya;
      ORACLE_CHECK(dx * ex + dy * ey >= 0, "turn sharper than 90 degrees");
      mesh_.chain_xy.push_back(sg.p.x);
      mesh_.chain_xy.push_back(sg.p.ya);
    }
    mesh_.n_segments = (i64)segs_.size();
    mesh_.n_contours = ncont;
  }

  // --- step 3: registry of crossings (segment-driven) ---------------------
  // exact: is the rational y below grid row k in the picture (Y > -4U + 2pk*sqrt3)?
  int cmp_row(i64 Y, i64 k) const { return z3_sign(Z3{(i128)Y + 4 * U_, -(i128)2 * h_ * k}); }

  void build_registry() {
    std::vector<std::pair<i64, Crossing>> tmp;
    const double rowstep = 2.0 * h_ * std::sqrt(3.0);
    for (i64 sidx = 0; sidx < (i64)segs_.size(); ++sidx) {
      const Segment& sg = segs_[sidx];
      i64 ylo = std::min(sg.p.ya, sg.q.ya), yhi = std::max(sg.p.ya, sg.q.ya);
      i64 xlo = std::min(sg.p.x, sg.q.x), xhi = std::max(sg.p.x, sg.q.x);
      i64 k0 = (i64)std::floor((ylo + 4 * U_) / rowstep) - 2;
      i64 k1 = (i64)std::floor((yhi + 4 * U_) / rowstep) + 2;
      for (i64 k = std::max<i64>(k0, 0); k <= std::min<i64>(k1, NK_ - 1); ++k) {
        i64 X00 = lat(k, 0).x;
        i64 i0 = (xlo - 4LL * h_ - X00) / (4LL * h_) - 2;
        i64 i1 = (xhi + 2LL * h_ - X00) / (4LL * h_) + 2;
        for (i64 i = std::max<i64>(i0, 0); i <= std::min<i64>(i1, NI_ - 1); ++i)
          for (int d = 0; d < 3; ++d) {
            i64 k2, i2;
            edge_ends(k, i, d, &k2, &i2);
            if (!lat_ok(k2, i2)) continue;
            Pt U = lat(k, i), V = lat(k2, i2);
            int s1 = orient_sign(U, V, sg.p), s2 = orient_sign(U, V, sg.q);
            int s3 = orient_sign(sg.p, sg.q, U), s4 = orient_sign(sg.p, sg.q, V);
            ORACLE_CHECK(s1 != 0 && s2 != 0 && s3 != 0 && s4 != 0, "zero predicate");
            if (s1 == s2 || s3 == s4) continue;
            Crossing c;
            c.edge_key = ekey(k, i, d);
            c.seg = sidx;
            tmp.push_back({c.edge_key, c});
          }
      }
    }
    // group by edge and sort by exact parameter from the owner vertex
    std::sort(tmp.begin(), tmp.end(), [](const std::pair<i64, Crossing>& a,
                                         const std::pair<i64, Crossing>& b) {
      if (a.first != b.first) return a.first < b.first;
      return a.second.seg < b.second.seg;
    });
    for (size_t a = 0; a < tmp.size();) {
      size_t b = a;
      while (b < tmp.size() && tmp[b].first == tmp[a].first) ++b;
      std::vector<Crossing> grp;
      for (size_t j = a; j < b; ++j) grp.push_back(tmp[j].second);
      i64 key = tmp[a].first;
      i64 d = key % 3, owner = key / 3, k = owner / NI_, i = owner % NI_;
      i64 k2, i2;
      edge_ends(k, i, (int)d, &k2, &i2);
      Pt U = lat(k, i), V = lat(k2, i2);
      std::sort(grp.begin(), grp.end(), [&](const Crossing& c1, const Crossing& c2) {
        const Segment& g1 = segs_[c1.seg];
        const Segment& g2 = segs_[c2.seg];
        return mu_compare(orient(g1.p, g1.q, U), orient(g1.p, g1.q, V),
                          orient(g2.p, g2.q, U), orient(g2.p, g2.q, V)) < 0;
      });
      for (size_t j = 0; j < grp.size(); ++j) {
        grp[j].rank = (int)j;
        // crossing coordinates (FP64), along the boundary segment P->Q:
        //   t = dP / (dP - dQ),  dP = (V-U) x (P-U),  dQ = (V-U) x (Q-U),
        //   X = P + t (Q - P)
        const Segment& g = segs_[grp[j].seg];
        double px = to_px(g.p.x), py = to_px(g.p.ya);
        double qx = to_px(g.q.x), qy = to_px(g.q.ya);
        double ux = lat_xd(k, i), uy = lat_yd(k), vx = lat_xd(k2, i2), vy = lat_yd(k2);
        double gx = vx - ux, gy = vy - uy;
        double dp = gx * (py - uy) - gy * (px - ux);
        double dq = gx * (qy - uy) - gy * (qx - ux);
        double t = dp / (dp - dq);
        grp[j].x = px + t * (qx - px);
        grp[j].y = py + t * (qy - py);
        reg_.push_back(grp[j]);
      }
      a = b;
    }
  }

  // --- step 4: exact point location of chain vertices ---------------------
  void locate_chain_vertices() {
    const double rowstep = 2.0 * h_ * std::sqrt(3.0);
    for (i64 sidx = 0; sidx < (i64)segs_.size(); ++sidx) {
      const Pt& P = segs_[sidx].p;
      i64 k = (i64)std::floor((P.ya + 4 * U_) / rowstep);
      while (k > 0 && cmp_row(P.ya, k) < 0) --k;
      while (cmp_row(P.ya, k + 1) > 0) ++k;
      ORACLE_CHECK(cmp_row(P.ya, k) > 0 && cmp_row(P.ya, k + 1) < 0, "row location");
      i64 ic = (P.x - lat(k, 0).x) / (4LL * h_);
      int found = 0;
      i64 key = -1;
      for (i64 i = ic - 2; i <= ic + 2; ++i)
        for (int t = 0; t < 2; ++t) {
          if (i < 0 || i >= NI_ || !tri_exists(k, i, t)) continue;
          i64 ck[3], ci[3];
          tri_corners(k, i, t, ck, ci);
          bool in = true;
          for (int j = 0; j < 3; ++j) {
            int sgn = orient_sign(lat(ck[j], ci[j]), lat(ck[(j + 1) % 3], ci[(j + 1) % 3]), P);
            ORACLE_CHECK(sgn != 0, "chain vertex on a grid edge");
            if (sgn < 0) in = false;
          }
          if (in) { ++found; key = tkey(k, i, t); }
        }
      ORACLE_CHECK(found == 1, "chain vertex not in exactly one base triangle");
      ChainVertex cv;
      cv.tri_key = key;
      cv.seg_out = sidx;
      chain_.push_back(cv);
    }
    std::sort(chain_.begin(), chain_.end(),
              [](const ChainVertex& a, const ChainVertex& b) { return a.tri_key < b.tri_key; });
    for (size_t j = 1; j < chain_.size(); ++j)
      ORACLE_CHECK(chain_[j].tri_key != chain_[j - 1].tri_key,
                   "protocol: two chain vertices in one base triangle");
    // cut triangles: both neighbours of every crossed edge, plus chain triangles
    for (auto& c : reg_) {
      i64 d = c.edge_key % 3, owner = c.edge_key / 3, k = owner / NI_, i = owner % NI_;
      if (d == 0) {
        cut_tris_.push_back(tkey(k, i, 1));
        if (k >= 1) cut_tris_.push_back(tkey(k - 1, i + 1 - ((k - 1) & 1), 0));
      } else if (d == 1) {
        cut_tris_.push_back(tkey(k, i, 0));
        if (i >= 1) cut_tris_.push_back(tkey(k, i - 1, 1));
      } else {
        cut_tris_.push_back(tkey(k, i, 0));
        cut_tris_.push_back(tkey(k, i, 1));
      }
    }
    for (auto& cv : chain_) cut_tris_.push_back(cv.tri_key);
    std::sort(cut_tris_.begin(), cut_tris_.end());
    cut_tris_.erase(std::unique(cut_tris_.begin(), cut_tris_.end()), cut_tris_.end());
  }

  // --- step 5: inside/outside of lattice vertices by ray parity -----------
  void label_inside() {
    inside_.assign((size_t)(NK_ * NI_), 0);
    size_t p = 0;
    for (i64 k = 0; k < NK_; ++k) {
      int in = 0;  // v(k,0) lies left of the padded image: outside
      for (i64 i = 0; i < NI_; ++i) {
        inside_[k * NI_ + i] = (uint8_t)in;
        i64 key = ekey(k, i, 0);
        while (p < reg_.size() && reg_[p].edge_key < key) ++p;
        int cnt = 0;
        while (p < reg_.size() && reg_[p].edge_key == key) { ++cnt; ++p; }
        in ^= (cnt & 1);
      }
      ORACLE_CHECK(in == 0, "ray parity does not close on a row");
    }
  }

  // --- step 6: canonical vertex numbering ---------------------------------
  // Vertices are numbered by owner lattice vertex (row k, then i).  An owner
  // holds: itself (if foreground, or always in both-sides mode), the
  // crossings on its edges right, down-left, down-right (each in order from
  // the owner), then the chain vertex in its apex-on-row-k triangle, then the
  // chain vertex in its base-on-row-k triangle.
  void number_vertices() {
    lattice_id_.assign((size_t)(NK_ * NI_), -1);
    i64 nv = 0;
    size_t p = 0, q = 0;
    for (i64 k = 0; k < NK_; ++k)
      for (i64 i = 0; i < NI_; ++i) {
        if (both_ || inside_[k * NI_ + i]) {
          lattice_id_[k * NI_ + i] = nv++;
          mesh_.verts.push_back(lat_xd(k, i));
          mesh_.verts.push_back(lat_yd(k));
        }
        for (int d = 0; d < 3; ++d) {
          i64 key = ekey(k, i, d);
          while (p < reg_.size() && reg_[p].edge_key < key) ++p;
          while (p < reg_.size() && reg_[p].edge_key == key) {
            reg_[p].vid = nv++;
            mesh_.verts.push_back(reg_[p].x);
            mesh_.verts.push_back(reg_[p].y);
            ++p;
          }
        }
        for (int t = 0; t < 2; ++t) {
          i64 key = tkey(k, i, t);
          while (q < chain_.size() && chain_[q].tri_key < key) ++q;
          if (q < chain_.size() && chain_[q].tri_key == key) {
            chain_[q].vid = nv++;
            const Pt& P = segs_[chain_[q].seg_out].p;
            mesh_.verts.push_back(to_px(P.x));
            mesh_.verts.push_back(to_px(P.ya));
          }
        }
      }
    ORACLE_CHECK(nv <= 0x7fffffffLL, "vertex count exceeds int32");
  }

  const Crossing* reg_find(i64 key, int rank) const {
    auto it = std::lower_bound(reg_.begin(), reg_.end(), key,
                               [](const Crossing& c, i64 kk) { return c.edge_key < kk; });
    for (; it != reg_.end() && it->edge_key == key; ++it)
      if (it->rank == rank) return &*it;
    return nullptr;
  }
  int reg_count(i64 key) const {
    auto it = std::lower_bound(reg_.begin(), reg_.end(), key,
                               [](const Crossing& c, i64 kk) { return c.edge_key < kk; });
    int n = 0;
    for (; it != reg_.end() && it->edge_key == key; ++it) ++n;
    return n;
  }

  // the grid edge that joins two lattice vertices, and whether (a -> b)
  // runs along the owner's direction
  void edge_between(i64 ka, i64 ia, i64 kb, i64 ib, i64* key, bool* fwd) const {
    for (int pass = 0; pass < 2; ++pass) {
      i64 k = pass ? kb : ka, i = pass ? ib : ia;
      i64 ko = pass ? ka : kb, io = pass ? ia : ib;
      for (int d = 0; d < 3; ++d) {
        i64 k2, i2;
        edge_ends(k, i, d, &k2, &i2);
        if (k2 == ko && i2 == io) { *key = ekey(k, i, d); *fwd = (pass == 0); return; }
      }
    }
    ORACLE_CHECK(false, "no grid edge between vertices");
  }

  // --- step 7: triangles ---------------------------------------------------
  void emit_triangles() {
    size_t pc = 0;
    for (i64 k = 0; k < NK_; ++k)
      for (i64 i = 0; i < NI_; ++i)
        for (int t = 0; t < 2; ++t) {
          if (!tri_exists(k, i, t)) continue;
          i64 key = tkey(k, i, t);
          while (pc < cut_tris_.size() && cut_tris_[pc] < key) ++pc;
          bool cut = (pc < cut_tris_.size() && cut_tris_[pc] == key);
          i64 ck[3], ci[3];
          tri_corners(k, i, t, ck, ci);
          if (!cut) {
            int in0 = inside_[ck[0] * NI_ + ci[0]];
            ORACLE_CHECK(in0 == inside_[ck[1] * NI_ + ci[1]] && in0 == inside_[ck[2] * NI_ + ci[2]],
                         "uncut triangle with mixed corners");
            if (!in0 && !both_) continue;
            i64 a = lattice_id_[ck[0] * NI_ + ci[0]], b = lattice_id_[ck[1] * NI_ + ci[1]],
                c = lattice_id_[ck[2] * NI_ + ci[2]];
            std::vector<std::vector<i64>> one = {{a, b, c}};
            push_sorted(one, in0 ? 0 : 0x80);
            continue;
          }
          ++mesh_.n_cut;
          emit_cut(k, i, t, ck, ci);
        }
  }

  void push_sorted(std::vector<std::vector<i64>>& tl, int code) {
    for (auto& tr : tl) {
      int m = 0;
      for (int j = 1; j < 3; ++j)
        if (tr[j] < tr[m]) m = j;
      std::vector<i64> r = {tr[m], tr[(m + 1) % 3], tr[(m + 2) % 3]};
      tr = r;
    }
    std::sort(tl.begin(), tl.end());
    for (auto& tr : tl) {
      for (int j = 0; j < 3; ++j) {
        ORACLE_CHECK(tr[j] >= 0, "triangle refers to a missing vertex");
        mesh_.tris.push_back((int32_t)tr[j]);
      }
      mesh_.codes.push_back((uint8_t)code);
    }
  }

  void emit_cut(i64 k, i64 i, int t, const i64 ck[3], const i64 ci[3]) {
    Pt C[3];
    for (int j = 0; j < 3; ++j) C[j] = lat(ck[j], ci[j]);
    LocalInput in;
    // chain vertex inside this triangle
    i64 key = tkey(k, i, t);
    auto cit = std::lower_bound(chain_.begin(), chain_.end(), key,
                                [](const ChainVertex& a, i64 kk) { return a.tri_key < kk; });
    const ChainVertex* cvI = nullptr;
    if (cit != chain_.end() && cit->tri_key == key) {
      cvI = &*cit;
      in.has_I = true;
      in.seg_out = cvI->seg_out;
      in.seg_in = segs_[cvI->seg_out].prev;
    }
    // crossings on the three edges, ordered along the triangle's own direction
    i64 edge_key[3];
    bool edge_fwd[3];
    int edge_n[3];
    std::vector<i64> segs_seen;
    for (int e = 0; e < 3; ++e) {
      edge_between(ck[e], ci[e], ck[(e + 1) % 3], ci[(e + 1) % 3], &edge_key[e], &edge_fwd[e]);
      edge_n[e] = reg_count(edge_key[e]);
      for (int r = 0; r < edge_n[e]; ++r) {
        const Crossing* c = reg_find(edge_key[e], r);
        LocalCrossing lc;
        lc.edge = e;
        lc.rank = edge_fwd[e] ? r : edge_n[e] - 1 - r;
        lc.seg = c->seg;
        lc.entry = orient_sign(C[e], C[(e + 1) % 3], segs_[c->seg].p) < 0;
        in.xs.push_back(lc);
        if (std::find(segs_seen.begin(), segs_seen.end(), c->seg) == segs_seen.end())
          segs_seen.push_back(c->seg);
      }
    }
    if (segs_seen.size() == 2) {
      i64 a = segs_seen[0], b = segs_seen[1];
      if (segs_[a].next == b) in.first_seg = a;
      else if (segs_[b].next == a) in.first_seg = b;
      else ORACLE_CHECK(false, "protocol: two non-consecutive segments in one base triangle");
    }
    ORACLE_CHECK(segs_seen.size() <= 2, "protocol: more than two segments in one base triangle");
    LocalResult lr = classify_local(in);
    // label -> global vertex id
    auto label_id = [&](int lab) -> i64 {
      if (lab < 3) return lattice_id_[ck[lab] * NI_ + ci[lab]];
      if (lab == 9) return cvI->vid;
      int e = (lab - 3) / 2, r = (lab - 3) % 2;
      int er = edge_fwd[e] ? r : edge_n[e] - 1 - r;
      const Crossing* c = reg_find(edge_key[e], er);
      ORACLE_CHECK(c != nullptr, "template refers to a missing crossing");
      return c->vid;
    };
    std::vector<std::vector<i64>> fg, bg;
    for (auto& tr : lr.tmpl.tris) {
      std::vector<i64> g = {label_id(tr.v[0]), label_id(tr.v[1]), label_id(tr.v[2])};
      if (tr.side == 1) fg.push_back(g); else bg.push_back(g);
    }
    if (!both_) {
      push_sorted(fg, lr.cls);
    } else {
      // both sides: sort all sub-triangles together, the code carries the side bit
      std::vector<std::pair<std::vector<i64>, int>> tagged;
      for (auto& g : fg) tagged.push_back({rot_min(g), lr.cls});
      for (auto& g : bg) tagged.push_back({rot_min(g), lr.cls | 0x80});
      std::sort(tagged.begin(), tagged.end());
      for (auto& tg : tagged) {
        for (int j = 0; j < 3; ++j) mesh_.tris.push_back((int32_t)tg.first[j]);
        mesh_.codes.push_back((uint8_t)tg.second);
      }
    }
  }
  static std::vector<i64> rot_min(const std::vector<i64>& tr) {
    int m = 0;
    for (int j = 1; j < 3; ++j)
      if (tr[j] < tr[m]) m = j;
    return {tr[m], tr[(m + 1) % 3], tr[(m + 2) % 3]};
  }
};

// ===========================================================================
// Geometric preprocessing of Alg. 3 (Sec. 3.5), then the template
// retriangulation of the preprocessed mesh (Alg. 1 and 2 with corner contacts).
//
// Readings (the paper leaves them open):
//  * Step 1 snaps a lattice vertex to the closest polyline vertex (a boundary
//    point of the set L) within distance a; ties go to the lower polyline index.
//    (With the polyline vertices as the snapping targets, a vertex within c of
//    two segments meeting at a corner lies within c*sqrt2 < a of the corner and
//    is snapped, so no vertex is repelled by two segments: the reason given for
//    c < a/sqrt2.)
//  * Step 2 runs on the vertices Step 1 left in place: the closest segment
//    within distance c pushes the vertex along its normal to distance exactly
//    c, on the same side.
//  * Step 3 takes the polyline vertices in order: a mesh edge within distance b
//    of p_j (not ending at p_j) is removed with its triangles and the cavity is
//    fanned from p_j.
//  * Each triangle of the preprocessed mesh is cut by the pieces of the
//    polyline inside it (degenerate contacts: the polyline passes through a
//    corner that was snapped to, or inserted at, a polyline vertex); each
//    foreground face is triangulated by the template rule of the plain path:
//    fanned from the chain vertex inside the triangle if it has one, the
//    middle quadrilateral between two chords split by the diagonal joining the
//    chords' exits, else fanned from the face's earliest chain point.
// All decisions are taken in double precision: after the three steps every
// vertex off the polyline lies at least c from every segment and every
// polyline vertex off the mesh vertices at least b from every mesh edge, so
// each sign has a margin far above the rounding error; contacts at a corner are
// decided by identity (the corner is that polyline vertex).
// Output: vertices sorted by (y, x), triangles rotated to their smallest index
// and sorted; codes 0 for uncut triangles, 1 for pieces of cut ones.
// ===========================================================================
struct PreResult {
  std::vector<double> verts;
  std::vector<int32_t> tris;
  std::vector<uint8_t> codes;
  i64 n_snapped = 0, n_repelled = 0, n_inserted = 0, n_cut = 0;
  // the preprocessed grid (after Steps 1-3, before the retriangulation):
  // vertices (lattice k NI + i, then the inserted points in polyline order),
  // whether each sits on a polyline vertex, and the live triangles
  std::vector<double> grid_verts;
  std::vector<uint8_t> grid_on_polyline;
  std::vector<int64_t> grid_tris;
};

// Euclidean length as the square root of the sum of squares, in IEEE double
// operations (a plain formula that any implementation evaluates identically;
// every threshold decision below compares such lengths).
static double euclid(double dx, double dy) { return std::sqrt(dx * dx + dy * dy); }

class PreOracle {
 public:
  PreOracle(Oracle::Traced t, double a, double b, double c) : T_(std::move(t)), a_(a), b_(b), c_(c) {
    cs_ = std::max(T_.h, 1.0);
  }

  // grid_only: stop after Steps 1-3 (the preprocessed grid, no retriangulation)
  PreResult run(bool grid_only = false) {
    index_polyline();
    snap_and_repel();
    build_triangles();
    eliminate_edges();
    record_grid();
    if (grid_only) return out_;
    retriangulate();
    return finish();
  }

 private:
  struct V { double x, y; i64 bnd; };  // bnd: polyline vertex it sits on, or -1
  Oracle::Traced T_;
  double a_, b_, c_, cs_;
  std::vector<V> vs_;                  // mesh vertices: lattice (k NI + i), then inserted points
  std::vector<std::array<i64, 3>> tri_;
  std::vector<uint8_t> alive_;
  std::vector<std::vector<i64>> slot_;  // base triangle slot (k NI + i) * 2 + t -> its current triangles
  std::vector<i64> slot_of_;            // triangle -> base slot
  std::unordered_map<i64, std::vector<i64>> pcell_, scell_;  // cell -> polyline vertices / segments
  PreResult out_;
  // output points: key -> id, coordinates
  std::map<std::array<i64, 3>, i64> pkey_;
  std::vector<double> ox_, oy_;
  std::vector<std::array<i64, 3>> otri_;
  std::vector<uint8_t> ocode_;

  i64 nseg() const { return (i64)T_.px.size(); }
  double qx(i64 s) const { return T_.px[(size_t)T_.next[(size_t)s]]; }
  double qy(i64 s) const { return T_.py[(size_t)T_.next[(size_t)s]]; }
  i64 ckey(i64 cx, i64 cy) const { return (cx + (1LL << 30)) * (1LL << 31) + (cy + (1LL << 30)); }
  i64 cell(double v) const { return (i64)std::floor(v / cs_); }

  void index_polyline() {
    for (i64 j = 0; j < nseg(); ++j) {
      pcell_[ckey(cell(T_.px[(size_t)j]), cell(T_.py[(size_t)j]))].push_back(j);
      const double x0 = std::min(T_.px[(size_t)j], qx(j)) - 1.0, x1 = std::max(T_.px[(size_t)j], qx(j)) + 1.0;
      const double y0 = std::min(T_.py[(size_t)j], qy(j)) - 1.0, y1 = std::max(T_.py[(size_t)j], qy(j)) + 1.0;
      for (i64 cx = cell(x0); cx <= cell(x1); ++cx)
        for (i64 cy = cell(y0); cy <= cell(y1); ++cy) scell_[ckey(cx, cy)].push_back(j);
    }
  }
  template <class F>
  void near(const std::unordered_map<i64, std::vector<i64>>& m, double x, double y, double r, F f) const {
    for (i64 cx = cell(x - r); cx <= cell(x + r); ++cx)
      for (i64 cy = cell(y - r); cy <= cell(y + r); ++cy) {
        auto it = m.find(ckey(cx, cy));
        if (it == m.end()) continue;
        for (i64 j : it->second) f(j);
      }
  }
  // distance from (x, y) to segment j, and the parameter of the closest point
  double seg_dist(i64 j, double x, double y, double* tpar) const {
    const double px = T_.px[(size_t)j], py = T_.py[(size_t)j];
    const double dx = qx(j) - px, dy = qy(j) - py;
    double t = ((x - px) * dx + (y - py) * dy) / (dx * dx + dy * dy);
    t = std::min(1.0, std::max(0.0, t));
    if (tpar) *tpar = t;
    return euclid(x - (px + t * dx), y - (py + t * dy));
  }

  void record_grid() {
    for (const V& v : vs_) {
      out_.grid_verts.push_back(v.x);
      out_.grid_verts.push_back(v.y);
      out_.grid_on_polyline.push_back(v.bnd >= 0 ? 1 : 0);
    }
    for (size_t t = 0; t < tri_.size(); ++t)
      if (alive_[t])
        for (int j = 0; j < 3; ++j) out_.grid_tris.push_back(tri_[t][(size_t)j]);
  }

  // Steps 1 and 2: vertex snapping (a), then repulsion (c) of the vertices left
  void snap_and_repel() {
    const i64 NK = T_.NK, NI = T_.NI;
    vs_.resize((size_t)(NK * NI));
    for (i64 k = 0; k < NK; ++k)
      for (i64 i = 0; i < NI; ++i) {
        V& v = vs_[(size_t)(k * NI + i)];
        v.x = T_.lx[(size_t)(k * NI + i)];
        v.y = T_.ly[(size_t)k];
        v.bnd = -1;
        double best = a_;
        i64 bj = -1;
        near(pcell_, v.x, v.y, a_, [&](i64 j) {
          const double d = euclid(v.x - T_.px[(size_t)j], v.y - T_.py[(size_t)j]);
          if (d < best || (d == best && bj >= 0 && j < bj)) { best = d; bj = j; }
        });
        if (bj >= 0) {
          v.x = T_.px[(size_t)bj];
          v.y = T_.py[(size_t)bj];
          v.bnd = bj;
          ++out_.n_snapped;
        }
      }
    for (V& v : vs_) {
      if (v.bnd >= 0) continue;
      double best = c_;
      i64 bj = -1;
      std::vector<i64> close;
      near(scell_, v.x, v.y, c_, [&](i64 j) {
        double t;
        const double d = seg_dist(j, v.x, v.y, &t);
        if (d < c_) close.push_back(j);
        if (d < best || (d == best && bj >= 0 && j < bj)) { best = d; bj = j; }
      });
      std::sort(close.begin(), close.end());
      const int nclose = (int)(std::unique(close.begin(), close.end()) - close.begin());
      if (bj < 0) continue;
      // each vertex is acted upon by at most one segment (c < a / sqrt2)
      ORACLE_CHECK(nclose == 1, "a vertex within c of two segments");
      double t;
      seg_dist(bj, v.x, v.y, &t);
      ORACLE_CHECK(t > 0.0 && t < 1.0, "repulsion foot at a segment end");
      const double px = T_.px[(size_t)bj], py = T_.py[(size_t)bj];
      const double dx = qx(bj) - px, dy = qy(bj) - py, L = euclid(dx, dy);
      const double nx = -dy / L, ny = dx / L;                 // left normal
      const double d = (v.x - px) * nx + (v.y - py) * ny;     // signed distance to the line
      const double move = (d > 0 ? c_ : -c_) - d;
      v.x += move * nx;
      v.y += move * ny;
      ++out_.n_repelled;
    }
    // every vertex off the polyline now lies at least c from every segment
    for (const V& v : vs_) {
      if (v.bnd >= 0) continue;
      near(scell_, v.x, v.y, c_, [&](i64 j) {
        ORACLE_CHECK(seg_dist(j, v.x, v.y, nullptr) > c_ * (1.0 - 1e-9), "vertex closer than c after Step 2");
      });
    }
  }

  double area2(i64 a, i64 b, i64 c) const {
    const V &A = vs_[(size_t)a], &B = vs_[(size_t)b], &C = vs_[(size_t)c];
    return (B.x - A.x) * (C.y - A.y) - (B.y - A.y) * (C.x - A.x);
  }

  void build_triangles() {
    const i64 NK = T_.NK, NI = T_.NI;
    slot_.resize((size_t)(NK * NI * 2));
    for (i64 k = 0; k + 1 < NK; ++k)
      for (i64 i = 0; i < NI; ++i) {
        const i64 o = k & 1;
        for (int t = 0; t < 2; ++t) {
          i64 ck[3] = {k, t == 0 ? k + 1 : k, k + 1};
          i64 ci[3] = {i, t == 0 ? i + o : i + 1, t == 0 ? i + o - 1 : i + o};
          bool ok = true;
          for (int j = 0; j < 3; ++j) ok = ok && ci[j] >= 0 && ci[j] < NI;
          if (!ok) continue;
          std::array<i64, 3> tr = {ck[0] * NI + ci[0], ck[1] * NI + ci[1], ck[2] * NI + ci[2]};
          ORACLE_CHECK(area2(tr[0], tr[1], tr[2]) > 0, "a base triangle inverted by the vertex moves");
          add_tri(tr, (k * NI + i) * 2 + t);
        }
      }
  }
  void add_tri(const std::array<i64, 3>& tr, i64 slot) {
    slot_[(size_t)slot].push_back((i64)tri_.size());
    slot_of_.push_back(slot);
    tri_.push_back(tr);
    alive_.push_back(1);
  }

  static double pt_seg(double x, double y, double ax, double ay, double bx, double by) {
    const double dx = bx - ax, dy = by - ay;
    double t = ((x - ax) * dx + (y - ay) * dy) / (dx * dx + dy * dy);
    t = std::min(1.0, std::max(0.0, t));
    return euclid(x - (ax + t * dx), y - (ay + t * dy));
  }

  // Step 3: edge elimination (b) and cavity retriangulation around p_j
  void eliminate_edges() {
    const i64 NI = T_.NI;
    const double rh = T_.h * 0.86602540378443864676;
    std::vector<i64> on_vertex(nseg(), -1);
    for (size_t v = 0; v < vs_.size(); ++v)
      if (vs_[v].bnd >= 0) on_vertex[(size_t)vs_[v].bnd] = (i64)v;
    std::vector<uint8_t> touched(tri_.size(), 0);
    for (i64 j = 0; j < nseg(); ++j) {
      if (on_vertex[(size_t)j] >= 0) continue;
      const double x = T_.px[(size_t)j], y = T_.py[(size_t)j];
      // candidate triangles: the base slots around p_j (vertices moved by less than a < h/2)
      const i64 k0 = (i64)std::floor((y + 1.0) / rh);
      std::vector<std::pair<i64, i64>> edges;  // (u, w), u < w
      for (i64 k = k0 - 2; k <= k0 + 2; ++k) {
        if (k < 0 || k + 1 >= T_.NK) continue;
        const double xo = T_.lx[(size_t)(k * NI)];
        const i64 ic = (i64)std::floor((x - xo) / T_.h);
        for (i64 i = ic - 3; i <= ic + 3; ++i) {
          if (i < 0 || i >= NI) continue;
          for (int t = 0; t < 2; ++t)
            for (i64 tid : slot_[(size_t)((k * NI + i) * 2 + t)]) {
              if (!alive_[(size_t)tid]) continue;
              const auto& tr = tri_[(size_t)tid];
              for (int e = 0; e < 3; ++e) {
                const i64 u = tr[e], w = tr[(e + 1) % 3];
                if (vs_[(size_t)u].bnd == j || vs_[(size_t)w].bnd == j) continue;
                const V &U = vs_[(size_t)u], &W = vs_[(size_t)w];
                if (pt_seg(x, y, U.x, U.y, W.x, W.y) < b_) edges.push_back({std::min(u, w), std::max(u, w)});
              }
            }
        }
      }
      std::sort(edges.begin(), edges.end());
      edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
      if (edges.empty()) continue;
      // b < a/2: one edge per point, and no triangle with two flagged edges
      ORACLE_CHECK(edges.size() == 1, "a boundary point within b of two mesh edges");
      const i64 u = edges[0].first, w = edges[0].second;
      const i64 m = (i64)vs_.size();
      vs_.push_back(V{x, y, j});
      ++out_.n_inserted;
      int nt = 0;
      for (i64 k = k0 - 2; k <= k0 + 2; ++k) {
        if (k < 0 || k + 1 >= T_.NK) continue;
        const double xo = T_.lx[(size_t)(k * NI)];
        const i64 ic = (i64)std::floor((x - xo) / T_.h);
        for (i64 i = ic - 3; i <= ic + 3; ++i) {
          if (i < 0 || i >= NI) continue;
          for (int t = 0; t < 2; ++t) {
            const i64 slot = (k * NI + i) * 2 + t;
            const std::vector<i64> cur = slot_[(size_t)slot];
            for (i64 tid : cur) {
              if (!alive_[(size_t)tid]) continue;
              auto tr = tri_[(size_t)tid];
              int e = -1;
              for (int q = 0; q < 3; ++q)
                if (std::min(tr[q], tr[(q + 1) % 3]) == u && std::max(tr[q], tr[(q + 1) % 3]) == w) e = q;
              if (e < 0) continue;
              ORACLE_CHECK(!touched[(size_t)tid], "a triangle with two eliminated edges");
              alive_[(size_t)tid] = 0;
              ++nt;
              const i64 a0 = tr[e], a1 = tr[(e + 1) % 3], a2 = tr[(e + 2) % 3];
              std::array<i64, 3> t1 = {a0, m, a2}, t2 = {m, a1, a2};
              ORACLE_CHECK(area2(t1[0], t1[1], t1[2]) > 0 && area2(t2[0], t2[1], t2[2]) > 0,
                           "cavity fan not positively oriented");
              add_tri(t1, slot);
              add_tri(t2, slot);
              touched.resize(tri_.size(), 0);
              touched[tri_.size() - 1] = touched[tri_.size() - 2] = 1;
            }
          }
        }
      }
      ORACLE_CHECK(nt >= 1 && nt <= 2, "edge elimination found no triangle");
    }
  }

  // --- retriangulation against the polyline ------------------------------
  // a point of a triangle's subdivision: kind 0 mesh vertex, 1 crossing of
  // mesh edge (u, w) (u < w) by segment s, 2 polyline vertex strictly inside
  struct PP {
    int kind;
    i64 a, b, s;
    double x, y;
    double ct;  // chain parameter: segment order + t
  };
  i64 point_id(const PP& p) {
    std::array<i64, 3> key = p.kind == 0 ? std::array<i64, 3>{0, p.a, 0}
                           : (p.kind == 1 ? std::array<i64, 3>{1 + p.s, p.a, p.b} : std::array<i64, 3>{-1, p.a, 0});
    auto it = pkey_.find(key);
    if (it != pkey_.end()) return it->second;
    const i64 id = (i64)ox_.size();
    pkey_[key] = id;
    ox_.push_back(p.x);
    oy_.push_back(p.y);
    return id;
  }
  // crossing of mesh edge (u, w) by segment s, computed from the canonical
  // orientation u < w so that both triangles of the edge get the same point
  PP crossing(i64 u, i64 w, i64 s) const {
    const i64 lo = std::min(u, w), hi = std::max(u, w);
    const V &U = vs_[(size_t)lo], &W = vs_[(size_t)hi];
    const double px = T_.px[(size_t)s], py = T_.py[(size_t)s];
    const double gx = W.x - U.x, gy = W.y - U.y;
    const double dp = gx * (py - U.y) - gy * (px - U.x);
    const double dq = gx * (qy(s) - U.y) - gy * (qx(s) - U.x);
    const double t = dp / (dp - dq);
    PP p;
    p.kind = 1;
    p.a = lo;
    p.b = hi;
    p.s = s;
    p.x = px + t * (qx(s) - px);
    p.y = py + t * (qy(s) - py);
    p.ct = t;
    return p;
  }

  bool inside_point(double x, double y) const {
    // ray parity to -x against every segment (rarely needed: triangles with no
    // corner off the polyline and no piece inside)
    int n = 0;
    for (i64 j = 0; j < nseg(); ++j) {
      const double ay = T_.py[(size_t)j], by = qy(j);
      if ((ay > y) == (by > y)) continue;
      const double xc = T_.px[(size_t)j] + (y - ay) / (by - ay) * (qx(j) - T_.px[(size_t)j]);
      if (xc < x) ++n;
    }
    return n & 1;
  }

  void emit(const std::vector<i64>& f, int code) {
    otri_.push_back({f[0], f[1], f[2]});
    ocode_.push_back((uint8_t)code);
  }

  void retriangulate() {
    const i64 NLAT = T_.NK * T_.NI;
    for (size_t tid = 0; tid < tri_.size(); ++tid) {
      if (!alive_[tid]) continue;
      const auto C = tri_[tid];
      double minx = 1e300, maxx = -1e300, miny = 1e300, maxy = -1e300;
      for (int j = 0; j < 3; ++j) {
        minx = std::min(minx, vs_[(size_t)C[j]].x); maxx = std::max(maxx, vs_[(size_t)C[j]].x);
        miny = std::min(miny, vs_[(size_t)C[j]].y); maxy = std::max(maxy, vs_[(size_t)C[j]].y);
      }
      // segments meeting the triangle: pieces [t0, t1] of segment s inside it
      struct Sub { i64 s; double t0, t1; int e0, e1; int c0, c1; };  // e: edge of entry/exit (-1 none), c: corner (-1)
      std::vector<Sub> subs;
      int edge_side = -1;
      std::vector<i64> cand;
      near(scell_, 0.5 * (minx + maxx), 0.5 * (miny + maxy), 0.5 * std::max(maxx - minx, maxy - miny) + 1.0,
           [&](i64 j) { cand.push_back(j); });
      std::sort(cand.begin(), cand.end());
      cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
      for (i64 s : cand) {
        const i64 jp = s, jq = T_.next[(size_t)s];
        const double px = T_.px[(size_t)s], py = T_.py[(size_t)s], dx = qx(s) - px, dy = qy(s) - py;
        if (std::max(px, qx(s)) < minx - 1e-9 || std::min(px, qx(s)) > maxx + 1e-9 ||
            std::max(py, qy(s)) < miny - 1e-9 || std::min(py, qy(s)) > maxy + 1e-9)
          continue;
        // clip against the three edge half-planes (inside = left of each edge)
        double t0 = 0.0, t1 = 1.0;
        int e0 = -1, e1 = -1;
        bool empty = false;
        for (int e = 0; e < 3 && !empty; ++e) {
          const i64 ua = C[e], ub = C[(e + 1) % 3];
          const V &A = vs_[(size_t)ua], &B = vs_[(size_t)ub];
          auto side = [&](double x, double y) { return (B.x - A.x) * (y - A.y) - (B.y - A.y) * (x - A.x); };
          // an end of the segment that is a corner of this edge lies on its line
          double fp = (A.bnd == jp || B.bnd == jp) ? 0.0 : side(px, py);
          double fq = (A.bnd == jq || B.bnd == jq) ? 0.0 : side(qx(s), qy(s));
          if (fp < 0 && fq < 0) { empty = true; break; }
          if (fp >= 0 && fq >= 0) continue;
          const double t = fp / (fp - fq);
          if (fp < 0) { if (t > t0) { t0 = t; e0 = e; } }
          else { if (t < t1) { t1 = t; e1 = e; } }
        }
        if (empty || !(t1 > t0)) continue;
        Sub sb{s, t0, t1, e0, e1, -1, -1};
        for (int j = 0; j < 3; ++j) {
          if (vs_[(size_t)C[j]].bnd == jp && t0 == 0.0) { sb.c0 = j; sb.e0 = -1; }
          if (vs_[(size_t)C[j]].bnd == jq && t1 == 1.0) { sb.c1 = j; sb.e1 = -1; }
        }
        if (sb.c0 >= 0 && sb.c1 >= 0) {
          // the segment joins two corners: it lies on their edge and does not
          // enter the triangle, which lies on the side of its third corner
          const int third = 3 - sb.c0 - sb.c1;
          const V& T3 = vs_[(size_t)C[third]];
          edge_side = ((qx(s) - px) * (T3.y - py) - (qy(s) - py) * (T3.x - px)) > 0 ? 1 : 0;
          continue;
        }
        subs.push_back(sb);
      }
      if (subs.empty()) {
        // uncut: side from a boundary segment along an edge, a corner off the
        // polyline, else the centroid
        int fg = edge_side;
        for (int j = 0; j < 3 && fg < 0; ++j)
          if (C[j] < NLAT && vs_[(size_t)C[j]].bnd < 0) fg = T_.inside[(size_t)C[j]];
        if (fg < 0) {
          double cx = 0, cy = 0;
          for (int j = 0; j < 3; ++j) { cx += vs_[(size_t)C[j]].x / 3; cy += vs_[(size_t)C[j]].y / 3; }
          fg = inside_point(cx, cy);
        }
        if (fg) {
          std::vector<i64> f;
          for (int j = 0; j < 3; ++j) f.push_back(point_id(PP{0, C[j], 0, -1, vs_[(size_t)C[j]].x, vs_[(size_t)C[j]].y, 0}));
          emit(f, 0);
        }
        continue;
      }
      ++out_.n_cut;
      // chain order of the segments met: consecutive ones in polyline order
      std::sort(subs.begin(), subs.end(), [&](const Sub& x, const Sub& y) { return x.s < y.s; });
      if (subs.size() == 2 && T_.next[(size_t)subs[1].s] == subs[0].s) std::swap(subs[0], subs[1]);
      ORACLE_CHECK(subs.size() <= 2, "more than two segments in one triangle");
      if (subs.size() == 2)
        ORACLE_CHECK(T_.next[(size_t)subs[0].s] == subs[1].s, "two non-consecutive segments in one triangle");
      // points of the subdivision: boundary points (corners and crossings) and
      // the chain vertex inside
      auto corner_pp = [&](int j) {
        return PP{0, C[j], 0, -1, vs_[(size_t)C[j]].x, vs_[(size_t)C[j]].y, 0};
      };
      // pieces: sequences of points along the chain inside the triangle
      std::vector<std::vector<PP>> pieces;
      std::vector<PP> cur;
      std::vector<std::pair<int, double>> bpos;  // per piece end: position on the boundary cycle
      for (size_t q = 0; q < subs.size(); ++q) {
        const Sub& sb = subs[q];
        PP start, end;
        const double order = (double)q;
        if (sb.c0 >= 0) start = corner_pp(sb.c0);
        else if (sb.e0 >= 0) start = crossing(C[sb.e0], C[(sb.e0 + 1) % 3], sb.s);
        else { start = PP{2, sb.s, 0, sb.s, T_.px[(size_t)sb.s], T_.py[(size_t)sb.s], 0}; }
        if (sb.c1 >= 0) end = corner_pp(sb.c1);
        else if (sb.e1 >= 0) end = crossing(C[sb.e1], C[(sb.e1 + 1) % 3], sb.s);
        else { end = PP{2, T_.next[(size_t)sb.s], 0, sb.s, qx(sb.s), qy(sb.s), 0}; }
        start.ct = order + sb.t0;
        end.ct = order + sb.t1;
        if (cur.empty()) cur.push_back(start);
        else ORACLE_CHECK(start.kind == 2 && cur.back().kind == 2 && start.a == cur.back().a, "pieces do not join");
        cur.push_back(end);
        if (end.kind != 2) { pieces.push_back(cur); cur.clear(); }
      }
      ORACLE_CHECK(cur.empty(), "a piece ends inside the triangle");
      int ninner = 0;
      for (auto& pc : pieces)
        for (auto& p : pc) ninner += p.kind == 2;
      ORACLE_CHECK(ninner <= 1, "two chain vertices in one triangle");
      // boundary cycle: corners and the piece ends on each edge, in order
      struct BP { PP p; int piece; int end; double pos; };  // end 0 = piece start, 1 = piece end
      std::vector<BP> cyc;
      for (int j = 0; j < 3; ++j) cyc.push_back(BP{corner_pp(j), -1, -1, 3.0 * j});
      auto edge_pos = [&](const PP& p) -> double {
        for (int e = 0; e < 3; ++e) {
          if (p.kind == 0 && p.a == C[e]) return 3.0 * e;
          if (p.kind == 1 && std::min(C[e], C[(e + 1) % 3]) == p.a && std::max(C[e], C[(e + 1) % 3]) == p.b) {
            const V &A = vs_[(size_t)C[e]], &B = vs_[(size_t)C[(e + 1) % 3]];
            const double L2 = (B.x - A.x) * (B.x - A.x) + (B.y - A.y) * (B.y - A.y);
            const double t = ((p.x - A.x) * (B.x - A.x) + (p.y - A.y) * (B.y - A.y)) / L2;
            ORACLE_CHECK(t > 0 && t < 1, "crossing outside its edge");
            return 3.0 * e + 1.0 + t;  // strictly between the corners 3e and 3e+3
          }
        }
        ORACLE_CHECK(false, "piece end not on the triangle");
        return 0;
      };
      for (size_t q = 0; q < pieces.size(); ++q) {
        for (int end = 0; end < 2; ++end) {
          const PP& p = end == 0 ? pieces[q].front() : pieces[q].back();
          const double pos = edge_pos(p);
          if (p.kind == 0) {
            for (auto& bp : cyc)
              if (bp.p.kind == 0 && bp.p.a == p.a) {
                ORACLE_CHECK(bp.piece < 0, "two pieces at one corner");
                bp.piece = (int)q;
                bp.end = end;
              }
          } else {
            cyc.push_back(BP{p, (int)q, end, pos});
          }
        }
      }
      std::sort(cyc.begin(), cyc.end(), [](const BP& x, const BP& y) { return x.pos < y.pos; });
      const int n = (int)cyc.size();
      // faces: walk the cycle; at a piece end arrived along the boundary, follow the piece
      std::vector<uint8_t> used(n, 0);
      for (int st = 0; st < n; ++st) {
        if (used[st]) continue;
        std::vector<PP> face;
        int side = -1;  // 1: the face uses a piece in chain direction (foreground)
        int at = st;
        for (int guard = 0; guard < 64; ++guard) {
          if (used[at]) break;
          used[at] = 1;
          face.push_back(cyc[at].p);
          int nx = (at + 1) % n;
          if (cyc[nx].piece >= 0) {
            // arrive at a piece end along the boundary: follow the piece
            const auto& pc = pieces[(size_t)cyc[nx].piece];
            const bool fwd = cyc[nx].end == 0;
            const int s2 = fwd ? 1 : 0;
            ORACLE_CHECK(side < 0 || side == s2, "face on both sides of the chain");
            side = s2;
            if (fwd) for (size_t z = 0; z + 1 < pc.size(); ++z) face.push_back(pc[z]);
            else for (size_t z = pc.size() - 1; z > 0; --z) face.push_back(pc[z]);
            // the other end of the piece
            int oth = -1;
            for (int z = 0; z < n; ++z)
              if (cyc[z].piece == cyc[nx].piece && cyc[z].end != cyc[nx].end) oth = z;
            ORACLE_CHECK(oth >= 0, "piece end missing");
            used[nx] = used[nx];  // the entry end is visited by the face that leaves from it
            at = oth;
            if (at == st) break;
            continue;
          }
          at = nx;
          if (at == st) break;
        }
        if (side < 0) continue;  // cannot happen for a cut triangle's faces (each touches the chain)
        if (side != 1) continue;
        triangulate_face(face, pieces);
      }
    }
  }

  // the template rule on one foreground face (points in positive order)
  void triangulate_face(const std::vector<PP>& face, const std::vector<std::vector<PP>>& pieces) {
    const int m = (int)face.size();
    if (m < 3) {
      std::string d = "degenerate face of " + std::to_string(m) + " points:";
      for (auto& p : face) d += " (" + std::to_string(p.kind) + " " + std::to_string(p.x) + "," + std::to_string(p.y) + ")";
      d += "; pieces:";
      for (auto& pc : pieces) {
        d += " [";
        for (auto& p : pc) d += "(" + std::to_string(p.kind) + " " + std::to_string(p.x) + "," + std::to_string(p.y) + ")";
        d += "]";
      }
      ORACLE_CHECK(false, d);
    }
    int apex = -1;
    for (int j = 0; j < m; ++j)
      if (face[j].kind == 2) apex = j;
    if (apex < 0 && m == 4 && pieces.size() == 2) {
      bool corners = false;
      for (auto& p : face) corners = corners || p.kind == 0;
      if (!corners) {
        // middle quadrilateral between two chords: diagonal joining their exits
        const PP& x1 = pieces[0].back();
        for (int j = 0; j < m; ++j)
          if (face[j].kind == 1 && face[j].a == x1.a && face[j].b == x1.b && face[j].s == x1.s) apex = j;
        const PP& x2 = pieces[1].back();
        ORACLE_CHECK(apex >= 0 && face[(apex + 2) % 4].kind == 1 && face[(apex + 2) % 4].s == x2.s &&
                         face[(apex + 2) % 4].a == x2.a && face[(apex + 2) % 4].b == x2.b,
                     "nested exits not opposite");
      }
    }
    if (apex < 0) {
      double best = 1e300;
      for (int j = 0; j < m; ++j) {
        const bool on_chain = face[j].kind != 0 || vs_[(size_t)face[j].a].bnd >= 0;
        if (!on_chain) continue;
        // chain position: the piece point with the same identity
        double ct = 1e300;
        for (auto& pc : pieces)
          for (auto& p : pc)
            if (p.kind == face[j].kind && p.a == face[j].a && p.b == face[j].b && p.s == face[j].s) ct = p.ct;
        if (ct < best) { best = ct; apex = j; }
      }
    }
    ORACLE_CHECK(apex >= 0, "no apex");
    std::vector<i64> ids;
    for (int j = 0; j < m; ++j) ids.push_back(point_id(face[(apex + j) % m]));
    for (int t = 1; t + 1 < m; ++t) {
      const i64 a = ids[0], b = ids[t], c = ids[t + 1];
      const double ar = (ox_[(size_t)b] - ox_[(size_t)a]) * (oy_[(size_t)c] - oy_[(size_t)a]) -
                        (oy_[(size_t)b] - oy_[(size_t)a]) * (ox_[(size_t)c] - ox_[(size_t)a]);
      ORACLE_CHECK(ar > 0, "template triangle not positively oriented");
      emit({a, b, c}, 1);
    }
  }

  PreResult finish() {
    const i64 n = (i64)ox_.size();
    std::vector<i64> ord(n);
    for (i64 j = 0; j < n; ++j) ord[j] = j;
    std::sort(ord.begin(), ord.end(), [&](i64 a, i64 b) {
      return oy_[(size_t)a] != oy_[(size_t)b] ? oy_[(size_t)a] < oy_[(size_t)b] : ox_[(size_t)a] < ox_[(size_t)b];
    });
    std::vector<i64> rank(n);
    for (i64 j = 0; j < n; ++j) rank[(size_t)ord[(size_t)j]] = j;
    for (i64 j = 0; j < n; ++j) {
      out_.verts.push_back(ox_[(size_t)ord[(size_t)j]]);
      out_.verts.push_back(oy_[(size_t)ord[(size_t)j]]);
    }
    std::vector<std::pair<std::array<i64, 3>, uint8_t>> ts;
    for (size_t t = 0; t < otri_.size(); ++t) {
      std::array<i64, 3> r = {rank[(size_t)otri_[t][0]], rank[(size_t)otri_[t][1]], rank[(size_t)otri_[t][2]]};
      int mi = 0;
      for (int j = 1; j < 3; ++j)
        if (r[j] < r[mi]) mi = j;
      ts.push_back({{r[mi], r[(mi + 1) % 3], r[(mi + 2) % 3]}, ocode_[t]});
    }
    std::sort(ts.begin(), ts.end());
    for (auto& t : ts) {
      for (int j = 0; j < 3; ++j) out_.tris.push_back((int32_t)t.first[j]);
      out_.codes.push_back(t.second);
    }
    return std::move(out_);
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// C ABI (host pointers only).
// ---------------------------------------------------------------------------
extern "C" {

struct oracle_mesh {
  Mesh m;
};

oracle_mesh* oracle_mesh_from_bitmap(const uint8_t* bitmap, int32_t width, int32_t height,
                                     int64_t row_stride, double grid_h, uint32_t flags,
                                     char* err, int32_t errlen) {
  try {
    Oracle o(bitmap, width, height, row_stride, grid_h, flags);
    oracle_mesh* res = new oracle_mesh;
    res->m = o.run();
    return res;
  } catch (const std::exception& e) {
    if (err && errlen > 0) {
      std::snprintf(err, (size_t)errlen, "%s", e.what());
    }
    return nullptr;
  }
}

int64_t oracle_n_vertices(const oracle_mesh* r) { return (int64_t)r->m.verts.size() / 2; }
int64_t oracle_n_triangles(const oracle_mesh* r) { return (int64_t)r->m.codes.size(); }
int64_t oracle_n_segments(const oracle_mesh* r) { return r->m.n_segments; }
int64_t oracle_n_cut(const oracle_mesh* r) { return r->m.n_cut; }
int64_t oracle_n_contours(const oracle_mesh* r) { return r->m.n_contours; }
void oracle_grid_dims(const oracle_mesh* r, int32_t* nk, int32_t* ni, int32_t* s) {
  *nk = r->m.NK; *ni = r->m.NI; *s = r->m.s;
}
void oracle_copy(const oracle_mesh* r, double* verts, int32_t* tris, uint8_t* codes) {
  if (verts && !r->m.verts.empty()) std::memcpy(verts, r->m.verts.data(), r->m.verts.size() * 8);
  if (tris && !r->m.tris.empty()) std::memcpy(tris, r->m.tris.data(), r->m.tris.size() * 4);
  if (codes && !r->m.codes.empty()) std::memcpy(codes, r->m.codes.data(), r->m.codes.size());
}
// closed boundary polylines: chain_start has n_contours+1 entries, xy holds the
// start point of every segment (x4 units) contour by contour
void oracle_copy_chains(const oracle_mesh* r, int64_t* xy, int64_t* chain_start) {
  if (xy && !r->m.chain_xy.empty())
    std::memcpy(xy, r->m.chain_xy.data(), r->m.chain_xy.size() * 8);
  if (chain_start) std::memcpy(chain_start, r->m.chain_start.data(), r->m.chain_start.size() * 8);
}
void oracle_free(oracle_mesh* r) { delete r; }

// Mesh after the preprocessing of Alg. 3 with thresholds a, b, c (pixels).
struct oracle_pre {
  PreResult r;
};
oracle_pre* oracle_pre_run(const uint8_t* bitmap, int32_t width, int32_t height, int64_t row_stride, double grid_h,
                           double a, double b, double c, bool grid_only, char* err, int32_t errlen);

oracle_pre* oracle_mesh_preprocessed(const uint8_t* bitmap, int32_t width, int32_t height, int64_t row_stride,
                                     double grid_h, double a, double b, double c, char* err, int32_t errlen) {
  return oracle_pre_run(bitmap, width, height, row_stride, grid_h, a, b, c, false, err, errlen);
}

// Steps 1-3 only: the preprocessed grid (oracle_pre_grid_sizes / _copy /
// oracle_pre_counts read it; the mesh arrays stay empty).
oracle_pre* oracle_pre_grid(const uint8_t* bitmap, int32_t width, int32_t height, int64_t row_stride, double grid_h,
                            double a, double b, double c, char* err, int32_t errlen) {
  return oracle_pre_run(bitmap, width, height, row_stride, grid_h, a, b, c, true, err, errlen);
}

oracle_pre* oracle_pre_run(const uint8_t* bitmap, int32_t width, int32_t height, int64_t row_stride, double grid_h,
                           double a, double b, double c, bool grid_only, char* err, int32_t errlen) {
  try {
    // all rules off, or the admissible ranges of Sec. 3.3.4: b < a/2,
    // c < a/sqrt2, and a < h/2 (disjoint snapping neighbourhoods)
    ORACLE_CHECK(a >= 0 && b >= 0 && c >= 0, "negative threshold");
    const bool off = a == 0 && b == 0 && c == 0;
    ORACLE_CHECK(off || (b < a / 2 && c * c < a * a / 2 && a < grid_h / 2), "thresholds outside the admissible range");
    Oracle o(bitmap, width, height, row_stride, grid_h, 0);
    PreOracle p(o.traced(), a, b, c);
    oracle_pre* res = new oracle_pre;
    res->r = p.run(grid_only);
    return res;
  } catch (const std::exception& e) {
    if (err && errlen > 0) std::snprintf(err, (size_t)errlen, "%s", e.what());
    return nullptr;
  }
}
int64_t oracle_pre_n_vertices(const oracle_pre* r) { return (int64_t)r->r.verts.size() / 2; }
int64_t oracle_pre_n_triangles(const oracle_pre* r) { return (int64_t)r->r.codes.size(); }
void oracle_pre_counts(const oracle_pre* r, int64_t* out) {
  out[0] = r->r.n_snapped; out[1] = r->r.n_repelled; out[2] = r->r.n_inserted; out[3] = r->r.n_cut;
}
void oracle_pre_copy(const oracle_pre* r, double* verts, int32_t* tris, uint8_t* codes) {
  if (verts && !r->r.verts.empty()) std::memcpy(verts, r->r.verts.data(), r->r.verts.size() * 8);
  if (tris && !r->r.tris.empty()) std::memcpy(tris, r->r.tris.data(), r->r.tris.size() * 4);
  if (codes && !r->r.codes.empty()) std::memcpy(codes, r->r.codes.data(), r->r.codes.size());
}
void oracle_pre_free(oracle_pre* r) { delete r; }
// The preprocessed grid of Alg. 3 (Steps 1-3): vertices, on-polyline flags,
// live triangles (vertex indices).
void oracle_pre_grid_sizes(const oracle_pre* r, int64_t* out) {
  out[0] = (int64_t)r->r.grid_on_polyline.size();
  out[1] = (int64_t)r->r.grid_tris.size() / 3;
}
void oracle_pre_grid_copy(const oracle_pre* r, double* verts, uint8_t* on_polyline, int64_t* tris) {
  if (verts && !r->r.grid_verts.empty()) std::memcpy(verts, r->r.grid_verts.data(), r->r.grid_verts.size() * 8);
  if (on_polyline && !r->r.grid_on_polyline.empty())
    std::memcpy(on_polyline, r->r.grid_on_polyline.data(), r->r.grid_on_polyline.size());
  if (tris && !r->r.grid_tris.empty()) std::memcpy(tris, r->r.grid_tris.data(), r->r.grid_tris.size() * 8);
}

// Exact sign of a + b*sqrt3 (exposed for the arithmetic pin).
int32_t oracle_z3_sign(int64_t a, int64_t b) { return z3_sign(Z3{(i128)a, (i128)b}); }

// Admissible canonical key codes in ascending order; class id = 1 + index.
int32_t oracle_class_table(int32_t* out, int32_t cap) {
  std::vector<int>& t = class_table();
  for (int32_t j = 0; j < (int32_t)t.size() && j < cap; ++j) out[j] = t[j];
  return (int32_t)t.size();
}

// Canonical code and rotation tag of a raw key code (Sec. 3.3.3: the smallest
// code over the three rotations, the first rotation reaching it); -1 if the
// code is not admissible.
int32_t oracle_canonical(int32_t code, int32_t* canon_code, int32_t* rot) {
  Desc d;
  d.type = code / 4096;
  d.tok[0] = (code / 512) % 8; d.tok[1] = (code / 64) % 8;
  d.tok[2] = (code / 8) % 8; d.tok[3] = code % 8;
  if (!desc_admissible(d)) return -1;
  int cc = 0, r = 0;
  desc_canonical(d, &cc, &r);
  *canon_code = cc;
  *rot = r;
  return class_id_of(cc);
}

// Procedural template of one key (both sides).  out: up to 5 x (a,b,c,side).
int32_t oracle_template_of_code(int32_t code, int32_t* out) {
  Desc d;
  d.type = code / 4096;
  d.tok[0] = (code / 512) % 8; d.tok[1] = (code / 64) % 8;
  d.tok[2] = (code / 8) % 8; d.tok[3] = code % 8;
  if (!desc_admissible(d)) return -1;
  LocalTemplate t = triangulate(d);
  for (size_t j = 0; j < t.tris.size(); ++j) {
    out[4 * j + 0] = t.tris[j].v[0]; out[4 * j + 1] = t.tris[j].v[1];
    out[4 * j + 2] = t.tris[j].v[2]; out[4 * j + 3] = t.tris[j].side;
  }
  return (int32_t)t.tris.size();
}

// One base triangle against an explicit polyline (worked examples of the
// paper).  corners: 3 x (x, ya, yb), y = ya + yb*sqrt3; chain: m x (x, y);
// all in one common integer scale.  Only proper crossings are supported;
// a degenerate contact returns -2.
struct oracle_local_result {
  int32_t type, tok[4], code, canon_code, rot, class_id, paper_m, paper_n;
  int32_t n_tris;
  int32_t tris[5][4];
  int32_t slot_seg[6];
  double slot_xy[6][2];
  int32_t chain_vertex;
};

int32_t oracle_local(const int64_t* corners, const int64_t* chain, int32_t m, double unit,
                     oracle_local_result* out, char* err, int32_t errlen) {
  try {
    Pt C[3];
    for (int j = 0; j < 3; ++j) C[j] = Pt{corners[3 * j], corners[3 * j + 1], corners[3 * j + 2]};
    ORACLE_CHECK(orient_sign(C[0], C[1], C[2]) > 0, "corners not positively oriented");
    std::vector<Pt> P;
    for (int j = 0; j < m; ++j) P.push_back(Pt{chain[2 * j], chain[2 * j + 1], 0});
    LocalInput in;
    // chain vertex strictly inside K
    int inside_idx = -1;
    for (int j = 0; j < m; ++j) {
      int s0 = orient_sign(C[0], C[1], P[j]), s1 = orient_sign(C[1], C[2], P[j]),
          s2 = orient_sign(C[2], C[0], P[j]);
      if (s0 == 0 || s1 == 0 || s2 == 0) {
        bool outside = (s0 < 0 || s1 < 0 || s2 < 0);
        if (!outside) return -2;  // chain vertex on the boundary of K
        continue;
      }
      if (s0 > 0 && s1 > 0 && s2 > 0) {
        ORACLE_CHECK(inside_idx < 0, "more than one chain vertex inside K");
        inside_idx = j;
      }
    }
    struct Raw { int e; i64 seg; bool entry; Z3 oU, oV; };
    std::vector<Raw> raw;
    for (int sidx = 0; sidx + 1 < m; ++sidx) {
      for (int e = 0; e < 3; ++e) {
        const Pt& U = C[e];
        const Pt& V = C[(e + 1) % 3];
        int s1 = orient_sign(U, V, P[sidx]), s2 = orient_sign(U, V, P[sidx + 1]);
        int s3 = orient_sign(P[sidx], P[sidx + 1], U), s4 = orient_sign(P[sidx], P[sidx + 1], V);
        if (s1 == 0 || s2 == 0 || s3 == 0 || s4 == 0) {
          if (s1 * s2 <= 0 && s3 * s4 <= 0) return -2;  // touching contact
          continue;
        }
        if (s1 == s2 || s3 == s4) continue;
        raw.push_back({e, sidx, s1 < 0, orient(P[sidx], P[sidx + 1], U),
                       orient(P[sidx], P[sidx + 1], V)});
      }
    }
    std::vector<i64> segs_seen;
    for (auto& r : raw) {
      LocalCrossing lc;
      lc.edge = r.e;
      lc.rank = 0;
      for (auto& r2 : raw)
        if (r2.e == r.e && &r2 != &r && mu_compare(r2.oU, r2.oV, r.oU, r.oV) < 0) ++lc.rank;
      lc.seg = r.seg;
      lc.entry = r.entry;
      in.xs.push_back(lc);
      if (std::find(segs_seen.begin(), segs_seen.end(), r.seg) == segs_seen.end())
        segs_seen.push_back(r.seg);
    }
    if (inside_idx >= 0) {
      in.has_I = true;
      in.seg_in = inside_idx - 1;
      in.seg_out = inside_idx;
    }
    if (segs_seen.size() == 2) in.first_seg = std::min(segs_seen[0], segs_seen[1]);
    std::memset(out, 0, sizeof(*out));
    out->chain_vertex = inside_idx;
    for (int j = 0; j < 6; ++j) out->slot_seg[j] = -1;
    if (raw.empty() && inside_idx < 0) {
      out->type = 0;
      return 0;
    }
    LocalResult lr = classify_local(in);
    out->type = lr.d.type;
    for (int j = 0; j < 4; ++j) out->tok[j] = lr.d.tok[j];
    out->code = lr.code;
    out->canon_code = lr.canon;
    out->rot = lr.rot;
    out->class_id = lr.cls;
    out->paper_m = lr.d.type == 1 ? 0 : (lr.d.type == 2 ? 1 : 2);
    out->paper_n = lr.d.type == 1 ? 2 : (lr.d.type == 2 ? 1 : 2);
    out->n_tris = (int32_t)lr.tmpl.tris.size();
    for (int j = 0; j < out->n_tris && j < 5; ++j) {
      for (int q = 0; q < 3; ++q) out->tris[j][q] = lr.tmpl.tris[j].v[q];
      out->tris[j][3] = lr.tmpl.tris[j].side;
    }
    for (int j = 0; j < 6; ++j) out->slot_seg[j] = lr.slot_seg[j];
    // crossing coordinates for the figure check (floating point, display only)
    for (int j = 0; j < 6; ++j) {
      if (lr.slot_seg[j] < 0) continue;
      int e = j / 2;
      const Pt& U = C[e];
      const Pt& V = C[(e + 1) % 3];
      const Pt& A = P[lr.slot_seg[j]];
      const Pt& B = P[lr.slot_seg[j] + 1];
      double s3 = std::sqrt(3.0);
      double ux = U.x / unit, uy = (U.ya + U.yb * s3) / unit;
      double vx = V.x / unit, vy = (V.ya + V.yb * s3) / unit;
      double px = A.x / unit, py = A.ya / unit, qx = B.x / unit, qy = B.ya / unit;
      double gx = vx - ux, gy = vy - uy;
      double dp = gx * (py - uy) - gy * (px - ux);
      double dq = gx * (qy - uy) - gy * (qx - ux);
      double t = dp / (dp - dq);
      out->slot_xy[j][0] = px + t * (qx - px);
      out->slot_xy[j][1] = py + t * (qy - py);
    }
    return 0;
  } catch (const std::exception& e) {
    if (err && errlen > 0) std::snprintf(err, (size_t)errlen, "%s", e.what());
    return -1;
  }
}

}  // extern "C"
