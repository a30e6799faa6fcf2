"""Pins of the medial-mesh oracle (RPE lengths, importance, medial chi, thinning) and of the library's host
thinning against it. CPU only.

* RPE lengths: three equal spheres around a vertical axis meet along that axis (closed form), a fourth sphere on
  the axis cuts it at a height fixed by the power distances (Sec. 3.2 definitions).
* Medial chi: when every restricted element is contractible the nerve theorem (Sec. 3.1) gives chi(medial mesh) =
  chi(shape).
* Thinning (Sec. 5.3, Fig. tech_thinning): the single-tet example worked by hand; on Delaunay complexes every
  removal keeps chi, step 1 ends with no tet-face simple pair, step 2 ends with no qualifying face-edge pair below
  sigma, and removals come in pairs. The library's thinning must give the same masks as the oracle's.
"""
import itertools
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import medial
from paper_2403_18761_amd import synth

CX, CY, RHO = 13 / 128, 5 / 128, 3 / 8  # axis off every mesh plane of the N=4 Kuhn cube (x, y, x-y, x+y)


def _circle_problem(extra=None, radius=0.125):
    base = synth.cube_random(N=4, n_sites=3, seed=0)
    cen = [[CX + RHO, CY, 0.0], [CX - RHO, CY, 0.0], [CX, CY + RHO, 0.0]]
    if extra is not None:
        cen.append(extra)
    c = np.asarray(cen)
    return base.with_sites(c[:, 0], c[:, 1], c[:, 2], np.full(len(cen), radius))


def _lengths(r):
    return {tuple(int(v) for v in k): float(l) for k, l in zip(r["edge_keys"], r["edge_length"])}


def test_rpe_length_three_spheres_on_a_circle(oracle_lib):
    prob = _circle_problem()
    r = oracle_lib.rpd(prob)
    assert r["consistent"], r["report"]
    # the three cells meet along the vertical line through the circle's centre, across the whole cube
    assert _lengths(r) == pytest.approx({(0, 1, 2): 2.0}, abs=1e-12)
    a = medial.edge_alpha(r["edge_length"], r["edge_keys"], prob.sr)
    assert a[0] == pytest.approx(2.0 / (2 * float(prob.sr[0])), rel=1e-12)


def test_rpe_length_fourth_sphere_on_the_axis(oracle_lib):
    Z = 0.75
    prob = _circle_problem(extra=[CX, CY, Z])
    # equal radii: on the axis d_circle = rho^2 + z^2 and d_4 = (z - Z)^2, equal at z* = (Z^2 - rho^2) / (2 Z)
    zs = (Fr(Z) ** 2 - Fr(RHO) ** 2) / (2 * Fr(Z))
    r = oracle_lib.rpd(prob)
    assert r["consistent"], r["report"]
    L = _lengths(r)
    assert L[(0, 1, 2)] == pytest.approx(float(zs + 1), abs=1e-12)
    # on the plane x = CX (cells 0 and 1) with d_0 = d_3, z = z* and the cell of sphere 2 takes over at y = CY
    assert L[(0, 1, 3)] == pytest.approx(1 + CY, abs=1e-12)
    assert r["rpv_keys"].tolist() == [[0, 1, 2, 3]]


def test_medial_chi_equals_shape_chi_when_elements_are_contractible(oracle_lib):
    checked = 0
    for seed in range(6):
        prob = synth.cube_random(N=4, n_sites=10, seed=100 + seed)
        r = oracle_lib.rpd(prob)
        valid = all((r[k + "_chi"][r[k + "_beta0"] > 0] == 1).all() and (r[k + "_beta0"] <= 1).all()
                    for k in ("cell", "face", "edge"))
        if not valid:
            continue
        (V, E, F, T), chi = medial.medial_counts(r)
        assert V == np.count_nonzero(r["cell_npieces"])
        assert chi == r["mesh_chi"] == 1
        checked += 1
    assert checked >= 3


# ---------------------------------------------------------------------------------------------------- thinning
def _single_tet():
    edges = np.array(list(itertools.combinations(range(4), 2)))
    tris = np.array(list(itertools.combinations(range(4), 3)))
    tets = np.array([[0, 1, 2, 3]])
    alpha = np.array([0.05, 0.2, 0.1, 0.4])  # triangles 012, 013, 023, 123
    return edges, tris, alpha, tets


def _check_single_tet(ke, kf, kt):
    # step 1 removes the tet with its least important triangle 012; step 2 removes (023, edge 02) at 0.1, then
    # (013, edge 01) at 0.2 (its lower edge), and stops at 123 whose importance 0.4 is not below sigma = 0.3
    assert kt.tolist() == [False]
    assert kf.tolist() == [False, False, False, True]
    assert ke.tolist() == [False, False, True, True, True, True]  # 01, 02 gone; 03, 12, 13, 23 kept


def test_thin_single_tet_by_hand():
    e, f, a, t = _single_tet()
    _check_single_tet(*medial.thin(4, e, f, a, t, 0.3))


def test_library_thin_single_tet_by_hand():
    from paper_2403_18761_amd import rpd

    e, f, a, t = _single_tet()
    _check_single_tet(*rpd.thin(4, e, f, a, t, 0.3))


def _delaunay_complex(n, seed):
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    pts = rng.uniform(-1, 1, size=(n, 3))
    tets = np.sort(Delaunay(pts).simplices, axis=1)
    tets = np.unique(tets, axis=0)
    tris = np.unique(np.array([f for t in tets for f in itertools.combinations(t, 3)]), axis=0)
    edges = np.unique(np.array([e for f in tris for e in itertools.combinations(f, 2)]), axis=0)
    alpha = rng.uniform(0, 1, size=len(tris))
    alpha[rng.integers(0, len(tris), size=len(tris) // 5)] = 0.5  # ties
    return n, edges, tris, alpha, tets


def _chi(nv, ke, kf, kt):
    return nv - int(ke.sum()) + int(kf.sum()) - int(kt.sum())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_thin_invariants_on_delaunay_complexes(seed):
    nv, e, f, a, t = _delaunay_complex(14, seed)
    sigma = 0.4
    ke, kf, kt = medial.thin(nv, e, f, a, t, sigma)
    ones = np.ones
    assert _chi(nv, ke, kf, kt) == _chi(nv, ones(len(e), bool), ones(len(f), bool), ones(len(t), bool)) == 1
    faces = [set(itertools.combinations(tt, 3)) for tt in t.tolist()]
    tri_list = [tuple(x) for x in f.tolist()]
    # step 1 ended: no kept tet has a triangle that no other kept tet shares
    for u in np.flatnonzero(kt):
        for face in faces[u]:
            assert any(kt[w] and face in faces[w] for w in range(len(t)) if w != u)
    # step 2 ended: every remaining face-edge simple pair of an original triangle has importance >= sigma
    for q in np.flatnonzero(kf):
        if any(kt[w] and tri_list[q] in faces[w] for w in range(len(t))):
            continue
        for edge in itertools.combinations(tri_list[q], 2):
            k = int(np.flatnonzero((e == edge).all(axis=1))[0])
            on = [g for g in np.flatnonzero(kf) if set(edge) <= set(tri_list[g])]
            if ke[k] and on == [q]:
                assert a[q] >= sigma
    # removed edges and triangles come in pairs of step 2, tets and triangles in pairs of step 1
    assert (~kf).sum() == (~kt).sum() + (~ke).sum()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_library_thin_matches_oracle(seed):
    from paper_2403_18761_amd import rpd

    nv, e, f, a, t = _delaunay_complex(12 + 2 * seed, 10 + seed)
    for sigma in (0.0, 0.3, 2.0):
        want = medial.thin(nv, e, f, a, t, sigma)
        got = rpd.thin(nv, e, f, a, t, sigma)
        for w, g in zip(want, got):
            np.testing.assert_array_equal(g, w)


def test_library_thin_rejects_bad_complexes():
    from paper_2403_18761_amd import rpd

    e, f, a, t = _single_tet()
    with pytest.raises(rpd.RPDError):
        rpd.thin(4, e[:5], f, a, t, 0.3)  # a triangle's edge is missing
    with pytest.raises(rpd.RPDError):
        rpd.thin(4, e, f[::-1], a, t, 0.3)  # not sorted
    with pytest.raises(rpd.RPDError):
        rpd.thin(3, e, f, a, t, 0.3)  # vertex id out of range
    bad = a.copy()
    bad[1] = np.nan
    with pytest.raises(rpd.RPDError):
        rpd.thin(4, e, f, bad, t, 0.3)
