"""Generate the lookup tables of the SBMT HIP kernels (``sbmt_tables.h``).

Run as ``python gen_tables.py [out.h]``; the build step runs it before hipcc.

The tables implement the finite template table of the paper (Alg. 2 and
App. G):

* ``sbmt_lut_key[16384]``: raw key code -> (class id | rotation << 6), 0 if the
  code is not an admissible configuration.  The raw code of a cut base triangle
  (corners c0, c1, c2 in positive orientation, local edge e = c_e -> c_{e+1})
  lists the boundary events in chain order, each as token 2e + r (r = rank of
  the crossing along edge e):
    type 1  one chord             (entry, exit)
    type 2  chain vertex inside   (entry of the first segment, exit of the second)
    type 3  two chords            (S1 entry, S1 exit, S2 entry, S2 exit)
  code = type*4096 + t0*512 + t1*64 + t2*8 + t3.  The canonical key is the
  smallest code over the three rotations e -> e+j (mirror images are distinct
  cases, App. G "Orientation handling"); the rotation stored is the first j
  reaching it.  Class ids number the admissible canonical codes in ascending
  order from 1 (0 = uncut).
* ``sbmt_lut_emit[class][rot][t][5]``: the same sub-triangles for triangle t
  (0 apex on the owner's row, 1 base on it) of an owner, seen through rotation
  rot, as triples of structural id slots in output order (see
  ``emission_order``), one uint16 per sub-triangle: a | b << 4 | c << 8 | side << 12.
* ``sbmt_lut_emit_fg[class][rot][t][5]``: the foreground entries of the same
  rows in the same order (what a foreground-only mesh emits), zero-padded, so
  that the j-th emitted sub-triangle is one lookup.
* ``sbmt_lut_tri[class][5]``: the template in canonical labels, one uint16 per
  sub-triangle: a | b << 4 | c << 8 | side << 12, labels 0..2 corners,
  3 + 2e + r crossing X(e, r), 9 the chain vertex; side 1 = left of the chain
  (foreground).  ``sbmt_lut_ntri`` / ``sbmt_lut_nfg`` count them.

Template rule (App. G, as read from its generic worked cases):
* a face that contains the chain vertex is fanned from it ((1,1) cases);
* the face between two nested chords (four crossings, no corner) takes the
  diagonal that joins the exit crossings of the two chords ((2,2) d3, a4);
* every other face is fanned from its earliest crossing along the chain
  (single-segment case (b), (2,2) b1).

This generator is written independently of the CPU oracle; tests compare the
two.  Faces are built here by splitting the boundary cycle into arcs.
"""
from __future__ import annotations

import sys

I_LABEL = 9


def ntok(typ: int) -> int:
    return 4 if typ == 3 else 2


def decode(code: int):
    typ = code >> 12
    t = [(code >> 9) & 7, (code >> 6) & 7, (code >> 3) & 7, code & 7]
    return typ, t


def encode(typ: int, t) -> int:
    return (typ << 12) | (t[0] << 9) | (t[1] << 6) | (t[2] << 3) | t[3]


def rotate(typ: int, t, j: int):
    n = ntok(typ)
    return [2 * (((x >> 1) + j) % 3) + (x & 1) if q < n else 0 for q, x in enumerate(t)]


def canonical(code: int):
    typ, t = decode(code)
    best, bj = None, 0
    for j in range(3):
        c = encode(typ, rotate(typ, t, j))
        if best is None or c < best:
            best, bj = c, j
    return best, bj


def _pos(label: int) -> int:
    """Position of a label on the boundary cycle (corner e at 3e, X(e,r) at 3e+1+r)."""
    if label < 3:
        return 3 * label
    x = label - 3
    return 3 * (x >> 1) + 1 + (x & 1)


def faces_of(code: int):
    """Faces of a key as CCW label lists with their side, or None if inadmissible."""
    typ, t = decode(code)
    if typ not in (1, 2, 3):
        return None
    n = ntok(typ)
    tok = t[:n]
    if any(x > 5 for x in tok) or any(x != 0 for x in t[n:]) or len(set(tok)) != n:
        return None
    for e in range(3):  # ranks on an edge must be {0} or {0, 1}
        if (2 * e + 1) in tok and (2 * e) not in tok:
            return None
    labels = [3 + x for x in tok]
    cycle = sorted([0, 1, 2] + labels, key=_pos)
    m = len(cycle)

    def arc(a, b):
        """Labels strictly after a up to strictly before b, walking the cycle CCW."""
        ia = cycle.index(a)
        out = []
        j = (ia + 1) % m
        while cycle[j] != b:
            out.append(cycle[j])
            j = (j + 1) % m
        return out

    if typ in (1, 3):
        for c in range(0, n, 2):
            if tok[c] >> 1 == tok[c + 1] >> 1:
                return None  # a straight chord cannot leave through the edge it entered
    if typ == 1:
        a, b = labels
        return [([a, b] + arc(b, a), 1), ([b, a] + arc(a, b), 0)]
    if typ == 2:
        a, b = labels
        return [([a, I_LABEL, b] + arc(b, a), 1), ([b, I_LABEL, a] + arc(a, b), 0)]
    a1, b1, a2, b2 = labels
    left1 = arc(b1, a1)          # boundary on the left of chord 1
    in_left = [a2 in left1, b2 in left1]
    if in_left[0] != in_left[1]:
        return None  # chords cross
    faces = []
    if in_left[0]:
        faces.append(([b1, a1] + arc(a1, b1), 0))      # chord 1's outer face is on its right
        mid_start, mid_first, side1 = a1, b1, 1
    else:
        faces.append(([a1, b1] + arc(b1, a1), 1))
        mid_start, mid_first, side1 = b1, a1, 0
    left2 = arc(b2, a2)
    if a1 in left2:
        if b1 not in left2:
            return None
        faces.append(([b2, a2] + arc(a2, b2), 0))
    else:
        faces.append(([a2, b2] + arc(b2, a2), 1))
    # middle face: along chord 1 on the middle side, then CCW to chord 2, along it, CCW back
    mid = [mid_start, mid_first]
    j = (cycle.index(mid_first) + 1) % m
    while cycle[j] not in (a2, b2):
        mid.append(cycle[j])
        j = (j + 1) % m
    u = cycle[j]
    w = b2 if u == a2 else a2
    side2 = 1 if (u, w) == (a2, b2) else 0
    if side2 != side1:
        return None  # the middle face would be on both sides of the chain
    mid += [u, w]
    j = (cycle.index(w) + 1) % m
    while cycle[j] != mid_start:
        mid.append(cycle[j])
        j = (j + 1) % m
    faces.append((mid, side1))
    return faces


def template_of(code: int):
    """Sub-triangles (a, b, c, side) of an admissible key, or None."""
    fs = faces_of(code)
    if fs is None:
        return None
    typ, t = decode(code)
    labels = [3 + x for x in t[:ntok(typ)]]
    chain_rank = {lab: q for q, lab in enumerate(labels)}
    tris = []
    for poly, side in fs:
        k = len(poly)
        corners = [p for p in poly if p < 3]
        if I_LABEL in poly:
            apex = I_LABEL
        elif typ == 3 and not corners and k == 4:
            apex = labels[1]  # exit of chord 1
            ia = poly.index(apex)
            if poly[(ia + 2) % 4] != labels[3]:
                return None
        else:
            apex = min((p for p in poly if p >= 3), key=lambda p: chain_rank[p])
        ia = poly.index(apex)
        rot = poly[ia:] + poly[:ia]
        for q in range(1, k - 1):
            tris.append((rot[0], rot[q], rot[q + 1], side))
    return tris


# Structural slots of the ids a base triangle of owner (k, i) can reference.
# Their numeric order is fixed by the owner numbering (own vertex, own
# crossings on E0, E1, E2, own chain vertices, then the next owner's vertex
# and its crossings on E3, then the row-below owners), so sorting by slot sorts
# by id:
#   0 v | 1,2 E0 | 3,4 E1 | 5,6 E2 | 7 I in Tb | 8 I in Ta | 9 vr | 10,11 E3 |
#   12 vdl | 13,14 E4 | 15 vdr
# Local edges of the triangles as (edge id, direction): Tb (t = 0):
# (E2,+) (E4,-) (E1,-); Ta (t = 1): (E0,+) (E3,+) (E2,-).
TRI_EDGE = {0: [(2, 1), (4, -1), (1, -1)], 1: [(0, 1), (3, 1), (2, -1)]}
EDGE_SLOT = {0: 1, 1: 3, 2: 5, 3: 10, 4: 13}
CORNER_SLOT = {0: [0, 15, 12], 1: [0, 9, 15]}


def emission_order(canon: int, rot: int, t: int):
    """Template of class `canon` seen through rotation `rot` on triangle t: the
    sub-triangles as slot triples rotated to start at the smallest slot and
    sorted, i.e. in output order; each with its side."""
    typ, tok = decode(canon)
    n = ntok(typ)
    # instance tokens: canonical edge e is instance edge e - rot
    inst = [2 * (((x >> 1) - rot) % 3) + (x & 1) for x in tok[:n]]
    count = [sum(1 for x in inst if x >> 1 == e) for e in range(3)]
    out = []
    for (a, b, c, side) in template_of(canon):
        slots = []
        for lab in (a, b, c):
            if lab < 3:
                slots.append(CORNER_SLOT[t][(lab - rot) % 3])
            elif lab < 9:
                x = lab - 3
                e, r = ((x >> 1) - rot) % 3, x & 1
                eid, d = TRI_EDGE[t][e]
                re = r if d > 0 else count[e] - 1 - r
                slots.append(EDGE_SLOT[eid] + re)
            else:
                slots.append(7 + t)
        m = slots.index(min(slots))
        out.append((tuple(slots[m:] + slots[:m]), side))
    out.sort()
    return out


def build():
    codes = [c for c in range(1 << 14) if faces_of(c) is not None]
    canon = sorted({canonical(c)[0] for c in codes})
    cls_of = {c: j + 1 for j, c in enumerate(canon)}
    key = [0] * (1 << 14)
    for c in codes:
        cc, j = canonical(c)
        key[c] = cls_of[cc] | (j << 6)
    tri = [[0] * 5]
    ntri, nfg = [0], [0]
    for cc in canon:
        ts = template_of(cc)
        assert ts is not None and len(ts) <= 5
        tri.append([a | (b << 4) | (c << 8) | (s << 12) for (a, b, c, s) in ts] + [0] * (5 - len(ts)))
        ntri.append(len(ts))
        nfg.append(sum(s for (_, _, _, s) in ts))
    emit = [[[[0] * 5 for _ in range(2)] for _ in range(3)]]
    for cc in canon:
        per_rot = []
        for rot in range(3):
            per_t = []
            for t in range(2):
                seq = emission_order(cc, rot, t)
                row = [a | (b << 4) | (c << 8) | (s << 12) for ((a, b, c), s) in seq]
                per_t.append(row + [0] * (5 - len(row)))
            per_rot.append(per_t)
        emit.append(per_rot)
    emit_fg = [[[[v for v in row if (v >> 12) & 1] for row in per_t] for per_t in per_rot] for per_rot in emit]
    emit_fg = [[[row + [0] * (5 - len(row)) for row in per_t] for per_t in per_rot] for per_rot in emit_fg]
    return {"canon": canon, "key": key, "tri": tri, "ntri": ntri, "nfg": nfg, "emit": emit, "emit_fg": emit_fg}


def emit_header(tables) -> str:
    canon = tables["canon"]
    lines = [
        "// Generated by gen_tables.py -- do not edit.",
        "// Template table of the SBMT lookup-driven retriangulation (Alg. 2, App. G).",
        "#pragma once",
        "#include <stdint.h>",
        "#ifndef SBMT_CONST",
        "#define SBMT_CONST __constant__",
        "#endif",
        f"#define SBMT_NUM_CLASSES {len(canon)}",
        "#define SBMT_CLASS_CODES_INIT 0, " + ", ".join(str(c) for c in canon),
        f"SBMT_CONST const int32_t sbmt_lut_class_code[{len(canon) + 1}] = {{0, "
        + ", ".join(str(c) for c in canon) + "};",
        f"SBMT_CONST const uint8_t sbmt_lut_ntri[{len(canon) + 1}] = {{"
        + ", ".join(str(v) for v in tables["ntri"]) + "};",
        f"SBMT_CONST const uint8_t sbmt_lut_nfg[{len(canon) + 1}] = {{"
        + ", ".join(str(v) for v in tables["nfg"]) + "};",
        f"SBMT_CONST const uint16_t sbmt_lut_tri[{len(canon) + 1}][5] = {{",
    ]
    lines += ["  {" + ", ".join(f"0x{v:04x}" for v in row) + "}," for row in tables["tri"]]
    lines.append("};")
    lines.append(f"SBMT_CONST const uint16_t sbmt_lut_emit[{len(canon) + 1}][3][2][5] = {{")
    for per_rot in tables["emit"]:
        lines.append("  {" + ", ".join("{" + ", ".join("{" + ", ".join(f"0x{v:04x}" for v in row) + "}"
                                                        for row in per_t) + "}" for per_t in per_rot) + "},")
    lines.append("};")
    lines.append(f"SBMT_CONST const uint16_t sbmt_lut_emit_fg[{len(canon) + 1}][3][2][5] = {{")
    for per_rot in tables["emit_fg"]:
        lines.append("  {" + ", ".join("{" + ", ".join("{" + ", ".join(f"0x{v:04x}" for v in row) + "}"
                                                        for row in per_t) + "}" for per_t in per_rot) + "},")
    lines.append("};")
    lines.append("SBMT_CONST const uint8_t sbmt_lut_key[16384] = {")
    key = tables["key"]
    for r in range(0, len(key), 32):
        lines.append("  " + ", ".join(str(v) for v in key[r:r + 32]) + ",")
    lines.append("};")
    return "\n".join(lines) + "\n"


def main(argv):
    import os

    out = argv[1] if len(argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                     "sbmt_tables.h")
    text = emit_header(build())
    old = open(out).read() if os.path.exists(out) else None
    if old != text:
        with open(out, "w") as f:
            f.write(text)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
