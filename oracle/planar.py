"""TEST INFRASTRUCTURE -- the fractional Euler characteristic rule in 2D, on exact rationals.

Sec. 4.1.2 (Fig. topo_euler and the equation beside it) explains the rule on a planar triangle mesh: a mesh simplex
shared by k triangles carries weight 1/k inside each of them; when a triangle is clipped by a half-plane, a new
vertex inherits the weight of the edge it splits and a new edge inherits the weight of the triangle it splits (1);
the clipped polygon then contributes (sum of vertex weights) - (sum of edge weights) + (face weight) to the element's
Euler characteristic. This module applies exactly that rule, with Python ``Fraction`` arithmetic, so the paper's
printed numbers can be checked against it. The 3D oracle in ``rpd_oracle.cpp`` applies the same rule one dimension
up; the two share no code.
"""
from __future__ import annotations

from collections import Counter
from fractions import Fraction as Fr


def simplex_weights(tris):
    """k(sigma) per vertex and undirected edge: the number of triangles containing it; weight = 1/k."""
    kv = Counter()
    ke = Counter()
    for t in tris:
        for a in t:
            kv[a] += 1
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            ke[frozenset((a, b))] += 1
    return {v: Fr(1, k) for v, k in kv.items()}, {e: Fr(1, k) for e, k in ke.items()}


def triangle_polygon(pts, tri, wv, we):
    """A triangle as a weighted polygon: list of (point, vertex weight) and, per edge k (vertex k -> k+1), a weight."""
    verts = [(tuple(Fr(c) for c in pts[a]), wv[a]) for a in tri]
    edges = [we[frozenset((tri[k], tri[(k + 1) % 3]))] for k in range(3)]
    return verts, edges, Fr(1)


def clip(poly, line):
    """Keep the part with a*x + b*y + c >= 0 (Sutherland-Hodgman on one convex polygon, with inheritance)."""
    verts, edges, fw = poly
    a, b, c = (Fr(x) for x in line)

    def val(p):
        return a * p[0] + b * p[1] + c

    n = len(verts)
    out_v, out_e = [], []
    # walk the boundary; every kept piece of an old edge keeps its weight, the new edge on the line weighs fw
    for k in range(n):
        p, wp = verts[k]
        q, wq = verts[(k + 1) % n]
        sp, sq = val(p), val(q)
        if sp == 0 or sq == 0:
            raise ValueError("degenerate: a vertex lies on the clipping line")
        if sp > 0:
            out_v.append((p, wp))
            out_e.append(edges[k])
            if sq < 0:
                t = sp / (sp - sq)
                out_v.append(((p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])), edges[k]))
                out_e.append(fw)  # new edge along the clipping line
        else:
            if sq > 0:
                t = sp / (sp - sq)
                out_v.append(((p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])), edges[k]))
                out_e.append(edges[k])
    if not out_v:
        return None
    return out_v, out_e, fw


def polygon_chi(poly):
    """(sum of vertex weights, sum of edge weights, face weight, chi) of one weighted polygon."""
    verts, edges, fw = poly
    sv = sum((w for _, w in verts), Fr(0))
    se = sum(edges, Fr(0))
    return sv, se, fw, sv - se + fw


def cell_pieces(pts, tris, lines):
    """Clip every triangle by every half-plane of one cell; returns the per-triangle weighted polygons."""
    wv, we = simplex_weights(tris)
    out = []
    for t in tris:
        poly = triangle_polygon(pts, t, wv, we)
        for ln in lines:
            if poly is None:
                break
            poly = clip(poly, ln)
        out.append(poly)
    return out
