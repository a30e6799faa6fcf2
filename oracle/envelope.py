"""TEST INFRASTRUCTURE -- oracle of the geometric-error metric (Sec. 4.3): distance from surface samples to the
enveloping volume of a medial mesh. FP64 numpy, vectorised over samples, one element at a time.

Only the test-suite and the benchmark's CPU baseline may import this module; the product package never imports
anything under ``oracle/``.

Enveloping elements (Sec. 3.2): a medial vertex's sphere; an edge's medial cone, the spheres interpolated linearly
between its two end spheres; a triangle's medial slab, the spheres interpolated over the triangle. For a sample q
and an element with spheres B(c(t), r(t)), the value is min over t of |q - c(t)| - r(t) (the distance to the
element's volume when q is outside it, negative inside). A sample's distance is the minimum over all elements.

Each element is evaluated on its own, boundary included, by listing candidate parameters that contain the
minimiser and taking the least value among them (every candidate is a point of the element, so the least is the
minimum):
* cone: t = 0, t = 1, and the roots in [0, 1] of the squared stationarity condition (a quadratic in t,
  solved in a cancellation-free form);
* slab: its three cones, and for each of the two planes tangent to all three spheres, the point where q's foot on
  the plane lies in the triangle of tangent points (the value there is q's signed distance to the plane).
"""
from __future__ import annotations

import numpy as np


def sphere_values(q: np.ndarray, c, r) -> np.ndarray:
    return np.linalg.norm(q - np.asarray(c, np.float64), axis=1) - float(r)


def cone_values(q: np.ndarray, c1, r1, c2, r2) -> np.ndarray:
    """min over t in [0, 1] of |q - (c1 + t e)| - (r1 + t dr), e = c2 - c1, dr = r2 - r1."""
    c1, c2 = np.asarray(c1, np.float64), np.asarray(c2, np.float64)
    r1, r2 = float(r1), float(r2)
    e, dr = c2 - c1, r2 - r1
    w = q - c1
    A = np.einsum("ij,ij->i", w, w)
    B = w @ e
    C = float(e @ e)

    def f(t):
        return np.sqrt(np.maximum(A - 2 * B * t + C * t * t, 0.0)) - r1 - dr * t

    best = np.minimum(f(np.zeros(len(q))), f(np.ones(len(q))))
    # f'(t) = 0: C t - B = dr |w - t e|; squared: C (C - dr^2) t^2 - 2 B (C - dr^2) t + B^2 - dr^2 A = 0, whose
    # discriminant over 4 C^2 (C - dr^2)^2 is dr^2 (A C - B^2) / (C - dr^2) with A C - B^2 = |w x e|^2, so the roots
    # are t = (B -+ |dr| |w x e| / sqrt(C - dr^2)) / C; both are candidates (squaring may add one)
    if C > dr * dr:
        wxe = np.linalg.norm(np.cross(w, e), axis=1)
        for sgn in (1.0, -1.0):
            t = (B + sgn * abs(dr) * wxe / np.sqrt(C - dr * dr)) / C
            inside = (t >= 0) & (t <= 1)
            best = np.where(inside, np.minimum(best, f(np.clip(t, 0, 1))), best)
    return best


def slab_values(q: np.ndarray, c, r) -> np.ndarray:
    """min over barycentric w of |q - sum w_i c_i| - sum w_i r_i for three spheres (c[i], r[i])."""
    c = np.asarray(c, np.float64).reshape(3, 3)
    r = np.asarray(r, np.float64).reshape(3)
    best = np.full(len(q), np.inf)
    for i, j in ((0, 1), (0, 2), (1, 2)):
        best = np.minimum(best, cone_values(q, c[i], r[i], c[j], r[j]))
    # tangent planes N.x = D with N.c_i + r_i = D for all i, |N| = 1: N = N0 + gamma n, N0 the least-norm solution
    # of N.(c_j - c_0) = -(r_j - r_0), n the unit normal of the centres' plane
    E = np.stack([c[1] - c[0], c[2] - c[0]])
    rhs = -np.array([r[1] - r[0], r[2] - r[0]])
    nc = np.cross(E[0], E[1])
    if np.linalg.norm(nc) == 0.0:
        return best
    n = nc / np.linalg.norm(nc)
    N0 = np.linalg.lstsq(E, rhs, rcond=None)[0]
    g2 = 1.0 - float(N0 @ N0)
    if g2 <= 0.0:
        return best
    for sgn in (1.0, -1.0):
        N = N0 + sgn * np.sqrt(g2) * n
        D = float(N @ c[0]) + r[0]
        h = q @ N - D                     # signed distance of q to the plane
        foot = q - h[:, None] * N[None, :]
        T = c + r[:, None] * N[None, :]   # tangent points
        # barycentric coordinates of the foot in the tangent triangle
        M = np.stack([T[1] - T[0], T[2] - T[0]], axis=1)  # 3 x 2
        ab = np.linalg.lstsq(M, (foot - T[0]).T, rcond=None)[0]  # 2 x m
        w = np.stack([1 - ab[0] - ab[1], ab[0], ab[1]])
        rstar = w.T @ r
        valid = (w >= 0).all(axis=0) & (rstar + h >= 0)
        best = np.where(valid, np.minimum(best, h), best)
    return best


def envelope_distance(spheres, edges, tris, samples):
    """(dist, nearest, values): per-sample minimum over all elements, the lowest element id reaching it, and a
    function giving one element's values (ids: spheres, then edges, then triangles)."""
    S = np.asarray(spheres, np.float64).reshape(-1, 4)
    E = np.asarray(edges, np.int64).reshape(-1, 2)
    F = np.asarray(tris, np.int64).reshape(-1, 3)
    q = np.asarray(samples, np.float64).reshape(-1, 3)

    def values(eid: int) -> np.ndarray:
        if eid < len(S):
            return sphere_values(q, S[eid, :3], S[eid, 3])
        eid -= len(S)
        if eid < len(E):
            i, j = E[eid]
            return cone_values(q, S[i, :3], S[i, 3], S[j, :3], S[j, 3])
        eid -= len(E)
        i, j, k = F[eid]
        return slab_values(q, S[[i, j, k], :3], S[[i, j, k], 3])

    dist = np.full(len(q), np.inf)
    nearest = np.full(len(q), -1, np.int64)
    for eid in range(len(S) + len(E) + len(F)):
        v = values(eid)
        better = v < dist
        dist = np.where(better, v, dist)
        nearest = np.where(better, eid, nearest)
    return dist, nearest, values
