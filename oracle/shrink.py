"""TEST INFRASTRUCTURE -- oracle of sphere shrinking (Sec. 5.1, Fig. tech_sphere_gen (a)). FP64 numpy.

Only the test-suite may import this module; the product package never imports anything under ``oracle/``.

The shrinking iteration of the paper's cited algorithm, in its order: start from a ball tangent at the pin p (inward
unit normal n) with a radius larger than the shape; find the surface point q nearest to the ball's centre; if q is
inside the ball, replace the radius by that of the ball tangent at p through q, r = |p - q|^2 / (2 n.(q - p)), and
repeat; stop when the nearest surface point is no longer inside. The nearest point on a triangle follows the
textbook region test (Voronoi regions of the vertices, edges and face of the triangle).
"""
from __future__ import annotations

import numpy as np


def closest_on_triangles(x: np.ndarray, a: np.ndarray, b: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Closest point of each triangle (a[k], b[k], c[k]) to the point x, (m, 3)."""
    ab, ac, ax = b - a, c - a, x - a
    d1, d2 = np.einsum("ij,ij->i", ab, ax), np.einsum("ij,ij->i", ac, ax)
    bx, cx = x - b, x - c
    d3, d4 = np.einsum("ij,ij->i", ab, bx), np.einsum("ij,ij->i", ac, bx)
    d5, d6 = np.einsum("ij,ij->i", ab, cx), np.einsum("ij,ij->i", ac, cx)
    va = d3 * d6 - d5 * d4
    vb = d5 * d2 - d1 * d6
    vc = d1 * d4 - d3 * d2
    out = np.empty_like(a)
    done = np.zeros(len(a), bool)

    def put(mask, pts):
        m = mask & ~done
        out[m] = pts[m]
        done[m] = True

    put((d1 <= 0) & (d2 <= 0), a)                                   # vertex a
    put((d3 >= 0) & (d4 <= d3), b)                                  # vertex b
    with np.errstate(divide="ignore", invalid="ignore"):
        v = d1 / (d1 - d3)
        put((vc <= 0) & (d1 >= 0) & (d3 <= 0), a + v[:, None] * ab)  # edge ab
        put((d6 >= 0) & (d5 <= d6), c)                              # vertex c
        w = d2 / (d2 - d6)
        put((vb <= 0) & (d2 >= 0) & (d6 <= 0), a + w[:, None] * ac)  # edge ac
        w2 = (d4 - d3) / ((d4 - d3) + (d5 - d6))
        put((va <= 0) & ((d4 - d3) >= 0) & ((d5 - d6) >= 0), b + w2[:, None] * (c - b))  # edge bc
        den = 1.0 / (va + vb + vc)
        v2, w3 = vb * den, vc * den
        put(np.ones(len(a), bool), a + v2[:, None] * ab + w3[:, None] * ac)  # face
    return out


def shrink(tris: np.ndarray, p, n, own: int = -1, r0: float = 4.0, max_iter: int = 1000):
    """Centre and radius of the maximal empty ball tangent at p (inward normal n) to the triangles (m, 3, 3)."""
    T = np.asarray(tris, np.float64)
    if own >= 0:
        T = np.delete(T, own, axis=0)
    a, b, c = T[:, 0], T[:, 1], T[:, 2]
    p, n = np.asarray(p, np.float64), np.asarray(n, np.float64)
    r = r0
    for _ in range(max_iter):
        ctr = p + r * n
        q = closest_on_triangles(ctr, a, b, c)
        d = np.linalg.norm(q - ctr, axis=1)
        k = int(np.argmin(d))
        if d[k] >= r * (1 - 1e-12):
            break
        w = q[k] - p
        r_new = float(w @ w) / (2.0 * float(n @ w))
        if not r_new < r:
            break
        r = r_new
    return p + r * n, r
