"""TEST INFRASTRUCTURE -- oracle of the dual medial mesh and its thinning (plain Python, slow, for small inputs).

Only the test-suite may import this module; the product package never imports anything under ``oracle/``.

* Duality (Sec. 3.2): a restricted power cell is dual to a medial vertex, an RPF to a medial edge, an RPE to a
  medial triangle and an RPV to a medial tet; the medial mesh's Euler characteristic is V - E + F - T (Sec. 6).
* Thinning (Sec. 5.3): the importance of a medial triangle f_ijk is the length of its dual RPE divided by the
  average diameter of spheres i, j, k. Tet-face simple pairs are removed, least important first, until no tet is
  left; then face-edge simple pairs whose triangle belonged to an original tet are removed, least important first,
  while the importance is below the stop value sigma. A pair (x, y) is simple when y lies on the boundary of x and
  of no other simplex left in the complex.
  Readings where the text is silent: ties in importance go to the lower triangle index (then the lower edge index);
  a face-edge pair's importance is its triangle's; vertices are never removed; tets that no simple pair reaches
  are left in place.
This module recomputes every simple pair from scratch at each step (quadratic time), so that each step can be
checked against the definition by eye.
"""
from __future__ import annotations

import numpy as np


def edge_alpha(lengths, keys, radii) -> np.ndarray:
    """Importance of the medial triangle dual to each RPE: |RPE_ijk| / ((2 r_i + 2 r_j + 2 r_k) / 3) (Sec. 5.3)."""
    r = np.asarray(radii, np.float64)
    out = np.empty(len(keys))
    for q, (i, j, k) in enumerate(np.asarray(keys).reshape(-1, 3)):
        mean_diam = (2 * r[i] + 2 * r[j] + 2 * r[k]) / 3.0
        out[q] = lengths[q] / mean_diam if mean_diam > 0 else np.inf
    return out


def medial_counts(res: dict):
    """(V, E, F, T) and chi = V - E + F - T of the dual medial mesh of an oracle result (Sec. 3.2, Sec. 6)."""
    V = int(np.count_nonzero(res["cell_beta0"] > 0))
    E, F, T = len(res["face_keys"]), len(res["edge_keys"]), len(res["rpv_keys"])
    return (V, E, F, T), V - E + F - T


def _faces_of(simplex):
    s = tuple(int(v) for v in simplex)
    return [tuple(s[:o] + s[o + 1:]) for o in range(len(s))]


def thin(n_vertices: int, edges, tris, alpha, tets, sigma: float):
    """Keep masks (edges, triangles, tets) after thinning; see the module docstring for the steps."""
    edges = [tuple(int(v) for v in e) for e in np.asarray(edges, np.int64).reshape(-1, 2)]
    tris = [tuple(int(v) for v in f) for f in np.asarray(tris, np.int64).reshape(-1, 3)]
    tets = [tuple(int(v) for v in t) for t in np.asarray(tets, np.int64).reshape(-1, 4)]
    alpha = [float(a) for a in np.asarray(alpha, np.float64).reshape(-1)]
    tri_index = {f: q for q, f in enumerate(tris)}
    edge_index = {e: q for q, e in enumerate(edges)}
    live_e, live_f, live_t = [True] * len(edges), [True] * len(tris), [True] * len(tets)

    # step 1: tet-face pairs
    while True:
        best = None
        for t, tet in enumerate(tets):
            if not live_t[t]:
                continue
            for face in _faces_of(tet):
                f = tri_index[face]
                others = [u for u, tet2 in enumerate(tets)
                          if live_t[u] and u != t and face in _faces_of(tet2)]
                if not others and (best is None or (alpha[f], f) < best[:2]):
                    best = (alpha[f], f, t)
        if best is None:
            break
        live_t[best[2]] = False
        live_f[best[1]] = False
    original = [any(f in _faces_of(tet) for tet in tets) for f in tris]

    # step 2: face-edge pairs of triangles of the original tets, while the importance is below sigma
    while True:
        best = None
        for f, tri in enumerate(tris):
            if not (live_f[f] and original[f]):
                continue
            if any(live_t[u] and tri in _faces_of(tet) for u, tet in enumerate(tets)):
                continue
            for edge in _faces_of(tri):
                e = edge_index[edge]
                if not live_e[e]:
                    continue
                on_e = [g for g, tri2 in enumerate(tris) if live_f[g] and edge in _faces_of(tri2)]
                if on_e == [f] and (best is None or (alpha[f], f, e) < best):
                    best = (alpha[f], f, e)
        if best is None or not best[0] < sigma:
            break
        live_f[best[1]] = False
        live_e[best[2]] = False
    return np.array(live_e, bool), np.array(live_f, bool), np.array(live_t, bool)
