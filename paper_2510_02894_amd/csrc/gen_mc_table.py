#!/usr/bin/env python3
"""Generate ``mc_table.h``: the per-case marching-cubes triangles used by the
HIP kernels, built from first principles (no table is copied).

Construction (the marching-cubes surface the paper's mesh pass builds, with
the ambiguity and triangulation rules fixed here):

* corner c of a cube sits at offset ((c>>2)&1, (c>>1)&1, c&1) along array
  axes (0, 1, 2); the case index has bit c set when corner c is inside;
* cube edge e = 4*a + 2*o_b + o_c runs along axis a from the corner with
  bit a clear, where b < c are the other two axes and (o_b, o_c) their
  offsets;
* on every face, the crossing edges are joined by segments: two crossings
  give one segment; four crossings (diagonal corners inside) give two
  segments, each cutting off one inside corner, so diagonal inside voxels
  stay separated (the region is 6-connected);
* every segment runs with the inside corners on its right when the face is
  seen from outside the cube; segments then chain into closed loops;
* each loop is fan-triangulated from its vertex with the smallest edge
  number, which makes every triangle normal point from inside to outside.

The header also carries, per case, integer data that lets the binary-mask
kernels compute area and volume without per-triangle geometry (vertices of a
binary mask sit at edge midpoints, so in half-voxel units every triangle has
small integer coordinates):

* ``l_e``: half-unit offset of edge e's midpoint inside the cube,
  2*offset(start corner) + e_axis;
* per triangle (a, b, c): the integer normal m = (l_b - l_a) x (l_c - l_a);
* per case: M = sum of m over its triangles and kappa = sum of
  l_a . (l_b x l_c).

Usage: ``python gen_mc_table.py [output]`` (default: ``mc_table.h`` beside
this script).
"""
from __future__ import annotations

import os
import sys

MAX_TRI = 5


def corner_offset(c):
    return ((c >> 2) & 1, (c >> 1) & 1, c & 1)


def corner_index(o):
    return (o[0] << 2) | (o[1] << 1) | o[2]


def edge_axis_start(e):
    a = e // 4
    ob, oc = (e % 4) >> 1, e & 1
    others = [x for x in range(3) if x != a]
    o = [0, 0, 0]
    o[others[0]] = ob
    o[others[1]] = oc
    return a, corner_index(o)


def edge_end(e):
    a, c0 = edge_axis_start(e)
    o = list(corner_offset(c0))
    o[a] = 1
    return corner_index(o)


EDGE_BY_CORNERS = {}
for _e in range(12):
    _c0, _c1 = edge_axis_start(_e)[1], edge_end(_e)
    EDGE_BY_CORNERS[frozenset((_c0, _c1))] = _e


def half_unit(e):
    """Edge midpoint in half-voxel units, relative to the cube's min corner."""
    a, c0 = edge_axis_start(e)
    o = corner_offset(c0)
    return tuple(2 * o[k] + (1 if k == a else 0) for k in range(3))


def faces():
    """Faces as (outward axis, side, corners in counter-clockwise order seen from outside).

    The 2-D frame (u, v) of a face is chosen right-handed with its outward
    normal, so a counter-clockwise walk around the face corners is the walk
    (0,0) -> (1,0) -> (1,1) -> (0,1) in (u, v).
    """
    out = []
    for f in range(3):
        g, h = [x for x in range(3) if x != f]
        for side in (0, 1):
            # (e_g, e_h, outward normal) right-handed? e_g x e_h = +e_f when (f, g, h) is
            # a cyclic permutation of (0, 1, 2); the outward normal is +e_f on side 1.
            cyclic = (f, g, h) in ((0, 1, 2), (1, 2, 0), (2, 0, 1))
            normal_sign = 1 if side == 1 else -1
            if (1 if cyclic else -1) == normal_sign:
                u_ax, v_ax = g, h
            else:
                u_ax, v_ax = h, g
            ring = []
            for (du, dv) in ((0, 0), (1, 0), (1, 1), (0, 1)):
                o = [0, 0, 0]
                o[f] = side
                o[u_ax] = du
                o[v_ax] = dv
                ring.append((corner_index(o), (du, dv)))
            out.append(ring)
    return out


FACES = faces()


def face_segments(case):
    """Directed segments (from_edge, to_edge) of all faces for one case."""
    segs = []
    for ring in FACES:
        ins = [(case >> c) & 1 for c, _ in ring]
        uv = [p for _, p in ring]
        cross = [k for k in range(4) if ins[k] != ins[(k + 1) % 4]]
        sides = [EDGE_BY_CORNERS[frozenset((ring[k][0], ring[(k + 1) % 4][0]))] for k in range(4)]
        mid = [((uv[k][0] + uv[(k + 1) % 4][0]) / 2, (uv[k][1] + uv[(k + 1) % 4][1]) / 2) for k in range(4)]
        pairs = []
        if len(cross) == 2:
            corner = next(k for k in range(4) if ins[k])
            pairs.append((cross[0], cross[1], corner))
        elif len(cross) == 4:
            for k in range(4):
                if ins[k]:
                    pairs.append(((k - 1) % 4, k, k))
        for s0, s1, corner in pairs:
            p, q, w = mid[s0], mid[s1], uv[corner]
            # 2-D cross product: > 0 means the corner lies left of p -> q.
            left = (q[0] - p[0]) * (w[1] - p[1]) - (q[1] - p[1]) * (w[0] - p[0])
            if left > 0:
                s0, s1 = s1, s0
            segs.append((sides[s0], sides[s1]))
    return segs


def case_triangles(case):
    nxt = {}
    for a, b in face_segments(case):
        assert a not in nxt, "edge with two successors"
        nxt[a] = b
    assert sorted(nxt) == sorted(nxt.values()), "segments do not close"
    tris = []
    done = set()
    for start in sorted(nxt):
        if start in done:
            continue
        loop = [start]
        done.add(start)
        cur = nxt[start]
        while cur != start:
            loop.append(cur)
            done.add(cur)
            cur = nxt[cur]
        # `start` is the smallest edge of its loop (edges are visited in order)
        for i in range(1, len(loop) - 1):
            tris.append((loop[0], loop[i], loop[i + 1]))
    return tris


def sub(a, b):
    return tuple(x - y for x, y in zip(a, b))


def cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def dot(a, b):
    return sum(x * y for x, y in zip(a, b))


def build():
    table = []
    for case in range(256):
        tris = case_triangles(case)
        assert len(tris) <= MAX_TRI
        normals, M, kappa = [], [0, 0, 0], 0
        for a, b, c in tris:
            la, lb, lc = half_unit(a), half_unit(b), half_unit(c)
            m = cross(sub(lb, la), sub(lc, la))
            normals.append(m)
            M = [M[k] + m[k] for k in range(3)]
            kappa += dot(la, cross(lb, lc))
        table.append(dict(tris=tris, normals=normals, M=M, kappa=kappa))
    return table


def render(table):
    lines = []
    w = lines.append
    w("// Generated by gen_mc_table.py -- do not edit.")
    w("// Marching-cubes triangles per case (corner c at offset ((c>>2)&1, (c>>1)&1, c&1);")
    w("// edge e = 4*axis + 2*o_b + o_c), ambiguous faces separate diagonal inside corners,")
    w("// loops fan-triangulated from their smallest edge, normals pointing inside -> outside.")
    w("#pragma once")
    w("#include <stdint.h>")
    w("")
    w("// Storage qualifier of the tables; device code defines it as __constant__ const.")
    w("#ifndef MC_TABLE_QUAL")
    w("#define MC_TABLE_QUAL const")
    w("#endif")
    w("")
    w("#define MC_MAX_TRI %d" % MAX_TRI)
    w("")
    w("// axis and start corner of each cube edge")
    w("static MC_TABLE_QUAL uint8_t MC_EDGE_AXIS[12] = {%s};" % ", ".join(str(edge_axis_start(e)[0]) for e in range(12)))
    w("static MC_TABLE_QUAL uint8_t MC_EDGE_C0[12] = {%s};" % ", ".join(str(edge_axis_start(e)[1]) for e in range(12)))
    w("// edge midpoint in half-voxel units relative to the cube's min corner")
    w("static MC_TABLE_QUAL int8_t MC_EDGE_HALF[12][3] = {%s};" % ", ".join(
        "{%d, %d, %d}" % half_unit(e) for e in range(12)))
    w("")
    w("static MC_TABLE_QUAL uint8_t MC_NTRI[256] = {")
    for r in range(0, 256, 16):
        w("    " + ", ".join("%d" % len(table[c]["tris"]) for c in range(r, r + 16)) + ",")
    w("};")
    w("")
    w("// triangles as cube-edge triples (unused slots are 0)")
    w("static MC_TABLE_QUAL uint8_t MC_TRI[256][MC_MAX_TRI][3] = {")
    for c in range(256):
        t = table[c]["tris"] + [(0, 0, 0)] * (MAX_TRI - len(table[c]["tris"]))
        w("    {%s}," % ", ".join("{%d, %d, %d}" % x for x in t))
    w("};")
    w("")
    w("// per-triangle integer normal (l_b - l_a) x (l_c - l_a) in half-voxel units")
    w("static MC_TABLE_QUAL int8_t MC_TRI_N[256][MC_MAX_TRI][3] = {")
    for c in range(256):
        n = table[c]["normals"] + [(0, 0, 0)] * (MAX_TRI - len(table[c]["normals"]))
        w("    {%s}," % ", ".join("{%d, %d, %d}" % x for x in n))
    w("};")
    w("")
    w("// per-case sum of triangle normals M and of l_a . (l_b x l_c) (kappa)")
    w("static MC_TABLE_QUAL int8_t MC_CASE_M[256][3] = {")
    for r in range(0, 256, 8):
        w("    " + ", ".join("{%d, %d, %d}" % tuple(table[c]["M"]) for c in range(r, r + 8)) + ",")
    w("};")
    w("static MC_TABLE_QUAL int16_t MC_CASE_KAPPA[256] = {")
    for r in range(0, 256, 16):
        w("    " + ", ".join("%d" % table[c]["kappa"] for c in range(r, r + 16)) + ",")
    w("};")
    w("")
    return "\n".join(lines)


def main(argv):
    out = argv[1] if len(argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)), "mc_table.h")
    text = render(build())
    with open(out, "w") as fh:
        fh.write(text)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
