"""The benchmark workloads at full size, in the launch configuration the benchmark times (autotuned first): tets
sampled at random are checked against the oracle piece by piece, and properties that hold at any size are checked on
the whole result (volumes partition the mesh, Euler additivity over the diagram, cell chi equal to the sum of its
pieces' fractional terms)."""
import os

import numpy as np
import pytest

from paper_2403_18761_amd import synth
from tests.gpu_util import ELEMENT_ARRAYS, extract, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle

    oracle.build(force=False)


def _dev(a, dt=None):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt or torch.float32, device="cuda:0")


def _mesh_sites(prob):
    import torch

    from paper_2403_18761_amd import rpd

    mesh = rpd.Mesh(_dev(prob.vx), _dev(prob.vy), _dev(prob.vz), _dev(prob.tv.reshape(-1), torch.int32))
    return mesh, (_dev(prob.sx), _dev(prob.sy), _dev(prob.sz), _dev(prob.sr))


def check_invariants(g, info, pieces=None, label=""):
    """Properties of any restricted power diagram of a mesh (exact integers, volumes to FP32 accuracy)."""
    vol = g["cell_vol"]
    assert abs(vol.sum() - info["volume"]) <= 1e-5 * info["volume"], (label, vol.sum(), info["volume"])
    live = vol > 0
    assert np.all(g["cell_beta0"][live] >= 1) and np.all(g["cell_beta0"][~live] == 0), label
    assert np.all(g["face_beta0"] >= 1) and np.all(g["edge_beta0"] >= 1), label
    additivity = int(g["cell_chi"].sum()) - int(g["face_chi"].sum()) + int(g["edge_chi"].sum()) - len(g["rpv_keys"])
    assert additivity == info["euler"], (label, additivity, info["euler"])
    if pieces is not None:
        num = np.zeros(len(vol), np.int64)
        np.add.at(num, pieces["i"], pieces["chi"])
        np.testing.assert_array_equal(num, g["cell_chi"].astype(np.int64) * info["L"], err_msg=f"{label} cell chi")


def sampled_against_oracle(prob, pieces, n_sample, seed, info, label):
    import oracle

    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(prob.n_tets, min(n_sample, prob.n_tets), replace=False))
    r = oracle.tet_pieces(prob, sel, threads=min(16, os.cpu_count() or 1))
    assert r["L"] == info["L"]
    want = {(p["t"], p["i"]): (p["chi_cell"], p["vol"]) for p in r["pieces"]}
    mask = np.isin(pieces["t"], sel)
    got = {(int(t), int(i)): (int(c), float(v))
           for t, i, c, v in zip(pieces["t"][mask], pieces["i"][mask], pieces["chi"][mask], pieces["geo"][mask, 0])}
    assert set(got) == set(want), (label, len(got), len(want), sorted(set(got) ^ set(want))[:5])
    # FP32 constructions err by about u |x| in the tet's frame, so a piece's volume error is absolute at the tet's
    # scale (surface h^2 times u h, about 6 u vol(t)): slivers get the floor 1e-6 vol(t), the rest 1e-5 relative
    v = np.stack([prob.vx, prob.vy, prob.vz], axis=1).astype(np.float64)
    p = v[prob.tv]
    tvol = np.abs(np.einsum("ij,ij->i", p[:, 1] - p[:, 0], np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]))) / 6.0
    for k, (c, vo) in want.items():
        assert got[k][0] == c, (label, k, got[k][0], c)
        assert abs(got[k][1] - vo) <= 1e-5 * vo + 1e-6 * tvol[k[0]], (label, k, got[k][1], vo, tvol[k[0]])
    return len(want)


def run_full(prob, n_sample, seed, label):
    from paper_2403_18761_amd import rpd

    mesh, sites = _mesh_sites(prob)
    best = rpd.autotune([mesh], [sites])
    log(label, "tets", prob.n_tets, "sites", prob.n_sites, "launch", best)
    res = rpd.build([mesh], [sites], block=best["block"], clip_budget=best["clip_budget"], flags=rpd.RPD_KEEP_PIECES)
    g = extract(res, 0)
    pieces = res.pieces(0)
    info = mesh.info()
    assert res.stats()["n_pairs"] == len(pieces["t"])
    check_invariants(g, info, pieces, label)
    n = sampled_against_oracle(prob, pieces, n_sample, seed, info, label)
    log(label, "sampled pieces", n, "total pieces", len(pieces["t"]))


def test_fullsize_torus():
    run_full(synth.torus_inside(64, 2000, 2), 400, 1, "torus N64 n2000")


def test_fullsize_genus3():
    run_full(synth.genus3_cad(128, 20000, 3), 200, 2, "genus3 N128 n20000")


def test_fullsize_batch_subset():
    """24 shapes of the 256-shape batch recipe (shape k is the batch's shape k) in one call."""
    from paper_2403_18761_amd import rpd

    t, s = synth.batch_sizes(256, 4)
    probs = [synth.batch_shape(k, int(t[k]), int(s[k])) for k in range(24)]
    made = [_mesh_sites(p) for p in probs]
    meshes, sites = [m for m, _ in made], [x for _, x in made]
    best = rpd.autotune(meshes, sites)
    log("batch subset tets", sum(p.n_tets for p in probs), "launch", best)
    res = rpd.build(meshes, sites, block=best["block"], clip_budget=best["clip_budget"], flags=rpd.RPD_KEEP_PIECES)
    total = 0
    for k, p in enumerate(probs):
        g = extract(res, k)
        pieces = res.pieces(k)
        info = meshes[k].info()
        check_invariants(g, info, pieces, f"batch shape {k}")
        total += sampled_against_oracle(p, pieces, 12, 100 + k, info, f"batch shape {k}")
    log("batch subset sampled pieces", total)


def test_fullsize_repair_session():
    """The repair workload at full size: after rounds of the session, the state equals a fresh build."""
    from paper_2403_18761_amd import rpd

    prob, table = synth.repair_problem(N=128, n_sites=500, seed=5)
    mesh, sites = _mesh_sites(prob)
    sess = rpd.Session(mesh, sites, tuple(_dev(x) for x in table), max_sites=500 + 64 * 4, max_insert=64)
    sess.run(3)
    info = sess.info()
    log("repair session", info)
    res = sess.result()
    a = extract(res, 0)
    s = sess.sites()
    fresh = rpd.build([mesh], [tuple(_dev(s[:, k]) for k in range(4))])
    b = extract(fresh, 0)
    for name in ELEMENT_ARRAYS:
        np.testing.assert_array_equal(a[name], b[name], err_msg=name)
    assert res.stats()["n_pairs"] == fresh.stats()["n_pairs"]
    check_invariants(a, mesh.info(), None, "repair session")
