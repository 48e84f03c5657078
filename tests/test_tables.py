"""The kernels' lookup tables against the oracle, on every one of the 16384 key codes.

The HIP path reads three generated tables (``csrc/gen_tables.py`` writes
``csrc/sbmt_tables.h``): raw key code -> (class id, rotation tag), and per
(class, rotation, owned triangle) the template's sub-triangles as structural id
slots in output order.  The generator builds its templates by splitting the
boundary cycle into arcs; the oracle traces faces over half-edges.  Here every
code is taken through both:

* admissibility, class id and rotation tag (the canonical key of Sec. 3.3.3:
  smallest code over the three rotations, first rotation reaching it) must agree;
* the oracle's template of the raw code itself, computed directly in the
  instance frame, mapped onto the owner's id slots, must equal the table row
  that the kernels reach through (class, rotation) -- which also checks that
  templates are carried by rotations (equivariance, App. G orientation handling).

Slot contract (the owner numbering): owner v = (k, i) with o = k mod 2 owns
E0 = v -> (k, i+1), E1 = v -> (k+1, i+o-1), E2 = v -> (k+1, i+o) and the
triangles Tb = [v, vdr, vdl] (t = 0) and Ta = [v, vr, vdr] (t = 1), where
vr = (k, i+1), vdl = (k+1, i+o-1), vdr = (k+1, i+o); E3 = vr -> vdr and
E4 = vdl -> vdr belong to neighbours.  Slots: 0 v | 1, 2 crossings of E0 in
order along E0 | 3, 4 of E1 | 5, 6 of E2 | 7 chain vertex in Tb | 8 in Ta |
9 vr | 10, 11 E3 | 12 vdl | 13, 14 E4 | 15 vdr.
"""
from __future__ import annotations

import os
import sys

import pytest

import oracle

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2602_19474_amd", "csrc")


@pytest.fixture(scope="module")
def gen():
    sys.path.insert(0, CSRC)
    try:
        import gen_tables
    finally:
        sys.path.pop(0)
    return gen_tables


@pytest.fixture(scope="module")
def tables(gen):
    return gen.build()


# corners of Tb / Ta in positive orientation -> slots
CORNERS = {0: (0, 15, 12), 1: (0, 9, 15)}
# local edge e = c_e -> c_{e+1} of Tb / Ta -> (first slot of the grid edge, same direction as the grid edge?)
#   Tb: v -> vdr is E2 (+), vdr -> vdl is E4 reversed, vdl -> v is E1 reversed
#   Ta: v -> vr is E0 (+), vr -> vdr is E3 (+), vdr -> v is E2 reversed
EDGES = {0: ((5, True), (13, False), (3, False)), 1: ((1, True), (10, True), (5, False))}


def _slots_of(code, tmpl, t):
    typ = code // 4096
    tok = [(code // 512) % 8, (code // 64) % 8, (code // 8) % 8, code % 8][:4 if typ == 3 else 2]
    per_edge = [sum(1 for x in tok if x // 2 == e) for e in range(3)]
    out = []
    for (a, b, c, side) in tmpl:
        sl = []
        for lab in (a, b, c):
            if lab < 3:
                sl.append(CORNERS[t][lab])
            elif lab == 9:
                sl.append(7 + t)
            else:
                e, r = (lab - 3) // 2, (lab - 3) % 2
                first, fwd = EDGES[t][e]
                sl.append(first + (r if fwd else per_edge[e] - 1 - r))
        m = sl.index(min(sl))
        out.append((tuple(sl[m:] + sl[:m]), side))
    return sorted(out)


def _row(vals):
    return [((v & 15, (v >> 4) & 15, (v >> 8) & 15), (v >> 12) & 1) for v in vals]


def test_header_is_the_generator_output(gen, tables):
    with open(os.path.join(CSRC, "sbmt_tables.h")) as f:
        assert f.read() == gen.emit_header(tables)


def test_class_codes_equal_the_oracle_table(tables):
    assert list(tables["canon"]) == [int(c) for c in oracle.class_table()]


def test_every_key_code(tables):
    key, emit, emit_fg = tables["key"], tables["emit"], tables["emit_fg"]
    ntri, nfg = tables["ntri"], tables["nfg"]
    n_adm = 0
    for code in range(1 << 14):
        want = oracle.canonical(code)
        assert (key[code] != 0) == (want is not None), code
        if want is None:
            continue
        n_adm += 1
        cls, canon, rot = want
        assert key[code] & 63 == cls and key[code] >> 6 == rot, (code, key[code], want)
        tmpl = oracle.template_of_code(code)
        assert len(tmpl) == ntri[cls] and sum(s for *_, s in tmpl) == nfg[cls], code
        for t in (0, 1):
            got = _slots_of(code, tmpl, t)
            assert _row(emit[cls][rot][t][:ntri[cls]]) == got, (code, t)
            assert all(v == 0 for v in emit[cls][rot][t][ntri[cls]:])
            fg = [x for x in got if x[1] == 1]
            assert _row(emit_fg[cls][rot][t][:nfg[cls]]) == fg, (code, t)
            assert all(v == 0 for v in emit_fg[cls][rot][t][nfg[cls]:])
    # every class is reached by exactly three raw codes (no rotation fixes a key)
    assert n_adm == 3 * len(tables["canon"])
