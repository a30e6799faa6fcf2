"""Pins of the oracle's tie-breaking by symbolic perturbation of the weights (simulation of simplicity: site s's
squared radius becomes r_s^2 + eps_s with eps_0 >> eps_1 >> ... > 0; the paper assumes a clean cut and does not say).

A degenerate input resolved symbolically must give the combinatorics of the same input with the lowest site's
radius grown by one grid unit (a real perturbation in the same direction, small enough to cross no other event),
and the volumes of the unperturbed input; the internal cross-checks (fractional chi = explicit V - E + F - C,
glued beta0 = skeleton beta0) and Euler additivity must hold.
"""
import numpy as np
import pytest

from paper_2403_18761_amd import synth

UNIT = 2.0 ** -20
COMBINATORIAL = ("cell_chi", "cell_beta0", "face_keys", "face_chi", "face_beta0", "edge_keys", "edge_chi",
                 "edge_beta0", "rpv_keys", "cell_npieces")


def _with(base, cen, rad):
    c = synth.quantize(np.asarray(cen, np.float64))
    r = synth.quantize(np.asarray(rad, np.float64))
    return base.with_sites(c[:, 0], c[:, 1], c[:, 2], r)


def degenerate_cases():
    """(name, problem): each has exact ties the weight perturbation has to break."""
    cube4 = synth.cube_random(N=4, n_sites=2, seed=0)
    rng = np.random.default_rng(3)
    extra = synth.quantize(rng.uniform(-0.9, 0.9, size=(10, 3)))
    cases = [
        # bisector x = 0 through a plane of mesh vertices
        ("mirror pair", _with(cube4, [[-0.375, 0.1, 0.2], [0.375, 0.1, 0.2]], [0.0, 0.0])),
        ("mirror pair + 10", _with(cube4, np.concatenate([[[-0.375, 0.1, 0.2], [0.375, 0.1, 0.2]], extra]),
                                   np.concatenate([[0.1, 0.1], rng.uniform(0, 0.1, 10)]))),
    ]
    # five equal spheres on a common sphere around a generic centre: a power vertex shared by five cells
    c0 = np.array([13, -7, 5]) / 128.0
    a = 0.375
    five = c0 + a * np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1]])
    cases.append(("five cospherical", _with(cube4, five, np.full(5, 0.125))))
    return cases


def _total_chi(r):
    return int(r["cell_chi"].sum()) - int(r["face_chi"].sum()) + int(r["edge_chi"].sum()) - len(r["rpv_keys"])


@pytest.mark.parametrize("name,prob", degenerate_cases(), ids=[c[0] for c in degenerate_cases()])
def test_ties_resolved_consistently(oracle_lib, name, prob):
    r = oracle_lib.rpd(prob)
    assert r["consistent"], r["report"]
    assert _total_chi(r) == r["mesh_chi"]
    assert abs(r["cell_vol"].sum() - 8.0) < 1e-12


@pytest.mark.parametrize("name,prob", degenerate_cases(), ids=[c[0] for c in degenerate_cases()])
def test_ties_match_a_real_perturbation(oracle_lib, name, prob):
    r = oracle_lib.rpd(prob)
    sr = prob.sr.copy()
    sr[0] = np.float32(float(sr[0]) + UNIT)  # site 0 (the dominant eps) grows by one grid unit
    q = oracle_lib.rpd(prob.with_sites(prob.sx, prob.sy, prob.sz, sr))
    for k in COMBINATORIAL:
        np.testing.assert_array_equal(r[k], q[k], err_msg=f"{name}: {k}")
    np.testing.assert_allclose(r["cell_vol"], q["cell_vol"], rtol=0, atol=1e-5)


def test_five_cospherical_vertex_is_split(oracle_lib):
    name, prob = degenerate_cases()[2]
    r = oracle_lib.rpd(prob)
    # the degree-5 vertex becomes RPVs of four cells each, joined by an infinitesimal RPE: more than one quadruple
    # among the five sites
    quads = [tuple(q) for q in r["rpv_keys"].tolist() if set(q) <= set(range(5))]
    assert len(quads) >= 2
