"""The dual medial mesh of a GPU-built RPD and its thinning (Sec. 3.2 duality, Sec. 5.3).

The GPU's RPE lengths, importances and medial counts are compared with the oracle inside assert_parity; here the
library's thinning runs on the GPU-built medial mesh and is compared with the oracle's thinning on the same input,
mask for mask, and at full size the thinning keeps the medial chi.
"""
import numpy as np
import pytest

from paper_2403_18761_amd import synth
from tests.gpu_util import assert_parity, log, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle

    oracle.build(force=False)


def _medial(res_keys, n_sites):
    return n_sites, res_keys["face_keys"], res_keys["edge_keys"], res_keys["edge_alpha"], res_keys["rpv_keys"]


@pytest.mark.parametrize("case", ["torus16_n64", "cube4_n40"])
def test_thinning_of_gpu_medial_mesh_matches_oracle(case):
    import oracle
    from oracle import medial

    from paper_2403_18761_amd import rpd

    prob = {"torus16_n64": lambda: synth.torus_core(16, 64, 1),
            "cube4_n40": lambda: synth.cube_random(N=4, n_sites=40, seed=9)}[case]()
    log("case: thinning", case)
    r = oracle.rpd(prob, assemble=False)
    g = run_gpu(prob)
    assert_parity(g, r, label=case)
    nv, e, f, a, t = _medial(g, prob.n_sites)
    for sigma in (0.1, 0.3):
        got = rpd.thin(nv, e, f, a, t, sigma)
        want = medial.thin(nv, e, f, a, t, sigma)
        for name, x, y in zip(("edges", "triangles", "tets"), got, want):
            np.testing.assert_array_equal(x, y, err_msg=f"{case} sigma {sigma} {name}")
        ke, kf, kt = got
        chi = int(g["medial"][4])
        v_live = int(g["medial"][0])
        assert v_live - int(ke.sum()) + int(kf.sum()) - int(kt.sum()) == chi


def test_thinning_full_size_torus():
    import time

    from paper_2403_18761_amd import rpd

    prob = synth.torus_inside(64, 2000, 2)
    log("case: thinning torus N64 n2000")
    g = run_gpu(prob)
    nv, e, f, a, t = _medial(g, prob.n_sites)
    assert np.all(np.isfinite(a)) and np.all(a >= 0)
    t0 = time.perf_counter()
    ke, kf, kt = rpd.thin(nv, e, f, a, t, 0.3)
    log(f"thinning {len(t)} tets {len(f)} triangles {len(e)} edges: {1e3 * (time.perf_counter() - t0):.1f} ms, "
        f"tets left {int(kt.sum())}")
    V, E, F, T, chi = (int(x) for x in g["medial"])
    assert (V, E, F, T) == (int((g["cell_beta0"] > 0).sum()), len(e), len(f), len(t))
    assert V - int(ke.sum()) + int(kf.sum()) - int(kt.sum()) == chi
    assert (~kf).sum() == (~kt).sum() + (~ke).sum()
