"""Pins of the oracle on general (non-voxel) tet meshes, where the fractional weights 1/k(sigma) need a
denominator beyond 2^31 and ownership weights replace them (one tet per mesh simplex carries its weight).

* On voxel meshes both weightings are definitions of the same chi (Sec. 4.1.2: the weights of a simplex sum to 1
  over the tets containing it): every element's chi and beta0 agree.
* On Delaunay meshes the oracle's own cross-check holds: the fractional chi equals the explicit V - E + F - C
  over merged keys (which uses no weights), the cell volumes partition the mesh, and the mesh's chi is 1.
"""
import numpy as np
import pytest

from paper_2403_18761_amd import synth

KINDS = ("cell_chi", "cell_beta0", "face_keys", "face_chi", "face_beta0", "edge_keys", "edge_chi", "edge_beta0",
         "rpv_keys", "cell_vol")


@pytest.mark.parametrize("which", ["torus", "cube"])
def test_owner_weights_give_the_same_chi_on_voxel_meshes(oracle_lib, which):
    prob = synth.torus_core(16, 64, 1) if which == "torus" else synth.cube_random(N=4, n_sites=30, seed=7)
    a = oracle_lib.rpd(prob)
    b = oracle_lib.rpd(prob, owner_weights=True)
    assert a["L"] > 1 and b["L"] == 1
    assert b["consistent"], b["report"]
    for k in KINDS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_delaunay_mesh_consistent(oracle_lib, seed):
    prob = synth.delaunay_ball(400, 40, seed)
    r = oracle_lib.rpd(prob)
    assert r["L"] == 1 and r["mesh_chi"] == 1 and r["mesh_components"] == 1
    assert r["consistent"], r["report"]
    np.testing.assert_array_equal(r["cell_chi"], r["cell_chi_asm"])
    np.testing.assert_array_equal(r["face_chi"], r["face_chi_asm"])
    np.testing.assert_array_equal(r["edge_chi"], r["edge_chi_asm"])
    P = np.stack([prob.vx, prob.vy, prob.vz], axis=1).astype(np.float64)
    t = prob.tv.reshape(-1, 4)
    vol = np.einsum("ij,ij->i", P[t[:, 1]] - P[t[:, 0]],
                    np.cross(P[t[:, 2]] - P[t[:, 0]], P[t[:, 3]] - P[t[:, 0]])).sum() / 6
    assert abs(r["cell_vol"].sum() - vol) < 1e-12 * vol


@pytest.mark.parametrize("kind", ["vertex", "edge"])
def test_pinched_meshes_are_rejected(oracle_lib, kind):
    """Sec. 3.3, Assumption: the input is a manifold tet mesh. A face-connected voxel mesh with a bow-tie vertex (two
    voxels that share only a corner) or a bow-tie edge (two voxels that share only an edge) is an input error; the same
    set with the pinch closed is accepted. Ground truth independent of the oracle: the voxel-level test for a
    manifold boundary (no edge- or vertex-critical 2x2 / 2x2x2 configuration)."""
    import numpy as np

    import oracle

    for fixed in (False, True):
        occ = np.zeros((4, 4, 4), dtype=bool)
        for c in synth.PINCHED[kind]["cells"] + (synth.PINCHED[kind]["fix"] if fixed else []):
            occ[c] = True
        assert synth.well_composed(occ) == fixed
    with pytest.raises(oracle.OracleError) as e:
        oracle.rpd(synth.pinched_voxels(kind))
    assert e.value.status == -2 and f"non-manifold {kind}" in e.value.msg, e.value.msg
    r = oracle.rpd(synth.pinched_voxels(kind, fixed=True))
    assert r["mesh_components"] == 1 and r["consistent"]
