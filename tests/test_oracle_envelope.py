"""Pins of the geometric-error oracle (Sec. 4.3; enveloping elements of Sec. 3.2). CPU only.

* sphere: |q - c| - r by definition (centre: -r);
* capsule (equal radii): point-segment distance minus r (textbook closed form);
* cones and slabs with any radii: direct numerical minimisation of |q - c(t)| - r(t) over the segment / triangle
  (dense grid, then a bounded local solver), independent of the oracle's candidate lists;
* an end sphere containing the other: the cone is that sphere;
* the union: the minimum over elements, reached by the reported element.
"""
import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

from oracle import envelope as env


def _brute_cone(q, c1, r1, c2, r2):
    c1, c2 = np.asarray(c1, float), np.asarray(c2, float)

    def f(t):
        return np.linalg.norm(q - (c1 + t * (c2 - c1))) - (r1 + t * (r2 - r1))

    ts = np.linspace(0, 1, 2001)
    t0 = ts[np.argmin([f(t) for t in ts])]
    res = minimize_scalar(f, bounds=(max(0, t0 - 1e-3), min(1, t0 + 1e-3)), method="bounded",
                          options={"xatol": 1e-12})
    return min(res.fun, f(0.0), f(1.0), f(t0))


def _brute_slab(q, c, r):
    c, r = np.asarray(c, float), np.asarray(r, float)

    def f(x):
        a, b = x
        w = np.array([1 - a - b, a, b])
        return np.linalg.norm(q - w @ c) - w @ r

    grid = [(a, b) for a in np.linspace(0, 1, 81) for b in np.linspace(0, 1, 81) if a + b <= 1]
    x0 = min(grid, key=f)
    res = minimize(f, x0, method="SLSQP", bounds=[(0, 1), (0, 1)],
                   constraints=[{"type": "ineq", "fun": lambda x: 1 - x[0] - x[1]}],
                   options={"ftol": 1e-14, "maxiter": 500})
    best = min(f(x0), res.fun if res.success else np.inf)
    for i, j in ((0, 1), (0, 2), (1, 2)):  # the solver may stop on a constraint edge: edges by the 1D brute force
        best = min(best, _brute_cone(q, c[i], r[i], c[j], r[j]))
    return best


def test_sphere_values():
    q = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    np.testing.assert_allclose(env.sphere_values(q, [0, 0, 0], 0.5), [-0.5, 2.5])


def test_capsule_is_segment_distance_minus_radius():
    rng = np.random.default_rng(0)
    c1, c2, r = np.array([-0.3, 0.1, 0.2]), np.array([0.4, -0.2, 0.5]), 0.15
    q = rng.uniform(-1, 1, size=(500, 3))
    e = c2 - c1
    t = np.clip((q - c1) @ e / (e @ e), 0, 1)
    want = np.linalg.norm(q - (c1 + t[:, None] * e), axis=1) - r
    np.testing.assert_allclose(env.cone_values(q, c1, r, c2, r), want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("seed", range(4))
def test_cone_matches_numerical_minimum(seed):
    rng = np.random.default_rng(seed)
    c1, c2 = rng.uniform(-0.5, 0.5, 3), rng.uniform(-0.5, 0.5, 3)
    L = np.linalg.norm(c2 - c1)
    r1 = rng.uniform(0, 0.3)
    r2 = max(0.0, r1 + rng.uniform(-0.9, 0.9) * L)  # |dr| < L: a proper cone
    q = rng.uniform(-1, 1, size=(40, 3))
    got = env.cone_values(q, c1, r1, c2, r2)
    want = np.array([_brute_cone(x, c1, r1, c2, r2) for x in q])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-9)


def test_cone_with_a_contained_end_sphere_is_the_big_sphere():
    c1, r1, c2, r2 = np.array([0.0, 0.0, 0.0]), 0.5, np.array([0.1, 0.0, 0.0]), 0.2
    q = np.random.default_rng(1).uniform(-1, 1, size=(200, 3))
    np.testing.assert_allclose(env.cone_values(q, c1, r1, c2, r2), env.sphere_values(q, c1, r1), atol=1e-13)


@pytest.mark.parametrize("seed,equal", [(0, True), (1, False), (2, False), (3, False)])
def test_slab_matches_numerical_minimum(seed, equal):
    rng = np.random.default_rng(10 + seed)
    c = rng.uniform(-0.5, 0.5, size=(3, 3))
    r = np.full(3, 0.1) if equal else rng.uniform(0.02, 0.2, 3)
    q = np.concatenate([rng.uniform(-1, 1, size=(20, 3)),
                        # points over the triangle's interior, off its plane: the tangent-plane case
                        (rng.dirichlet(np.ones(3), size=20) @ c) + 0.6 * np.cross(c[1] - c[0], c[2] - c[0])
                        / np.linalg.norm(np.cross(c[1] - c[0], c[2] - c[0])) * rng.choice([-1, 1], size=(20, 1))])
    got = env.slab_values(q, c, r)
    want = np.array([_brute_slab(x, c, r) for x in q])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-8)


def test_union_is_the_least_element():
    rng = np.random.default_rng(5)
    S = np.concatenate([rng.uniform(-0.5, 0.5, size=(5, 3)), rng.uniform(0.05, 0.2, size=(5, 1))], axis=1)
    E = np.array([[0, 1], [1, 2], [0, 2], [2, 3]])
    F = np.array([[0, 1, 2]])
    q = rng.uniform(-1, 1, size=(300, 3))
    d, near, values = env.envelope_distance(S, E, F, q)
    allv = np.stack([values(k) for k in range(len(S) + len(E) + len(F))])
    np.testing.assert_array_equal(d, allv.min(axis=0))
    np.testing.assert_array_equal(near, allv.argmin(axis=0))
    # a sample at a sphere centre lies inside by at least that radius
    d2, _, _ = env.envelope_distance(S, E, F, S[:, :3])
    assert np.all(d2 <= -S[:, 3] + 1e-15)
