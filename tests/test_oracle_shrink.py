"""Pins of the sphere-shrinking oracle (Sec. 5.1, Fig. tech_sphere_gen (a)). CPU only.

* Kuhn cube [-1, 1]^3: the maximal ball tangent at a point (u, v) of a face touches the nearest side face or the
  opposite face, radius min(1 - |u|, 1 - |v|, 1) (closed form);
* the nearest-point routine against dense sampling of random triangles.
"""
import numpy as np

from oracle import shrink as S
from paper_2403_18761_amd import synth


def _cube_pins():
    prob = synth.make_problem(synth.cube_solid(4), 4, np.zeros((1, 3)), np.zeros(1))
    return synth.surface_pins(prob)


def test_cube_closed_form():
    tri, n, cen, _, _ = _cube_pins()
    for k in range(0, len(tri), 7):
        _, r = S.shrink(tri, cen[k], n[k], own=k)
        axis = int(np.argmax(np.abs(n[k])))
        u, v = (float(cen[k][a]) for a in range(3) if a != axis)
        assert abs(r - min(1 - abs(u), 1 - abs(v), 1.0)) < 1e-6, (k, r, u, v)


def test_closest_point_matches_dense_sampling():
    rng = np.random.default_rng(0)
    a, b, c = (rng.uniform(-1, 1, size=(40, 3)) for _ in range(3))
    for x in rng.uniform(-2, 2, size=(10, 3)):
        got = S.closest_on_triangles(x, a, b, c)
        s = np.linspace(0, 1, 201)
        uu, vv = np.meshgrid(s, s)
        m = uu + vv <= 1
        uu, vv = uu[m], vv[m]
        for k in range(len(a)):
            pts = a[k] + uu[:, None] * (b[k] - a[k]) + vv[:, None] * (c[k] - a[k])
            dmin = np.linalg.norm(pts - x, axis=1).min()
            dgot = np.linalg.norm(got[k] - x)
            assert dgot <= dmin + 1e-12 and dmin - dgot < 2e-2 * np.linalg.norm(b[k] - a[k]) + 1e-9
