"""Parity of the GPU geometric-error kernel (rpd_envelope_distance, Sec. 4.3) with the FP64 oracle.

Bar: per-sample distance within 1e-5 absolute + 1e-5 relative (FP32 evaluation of O(1) quantities: coordinates
and radii below 2, about ten rounded operations per value, element constants rounded once from FP64: a few units
of 6e-8 times 4 each, with margin); the reported nearest element's oracle value within the same bound of the
oracle's minimum (near-ties may pick another element).
"""
import numpy as np
import pytest

from paper_2403_18761_amd import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

ATOL, RTOL = 1e-5, 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(a, dt=None):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")


def _medial(prob, sigma=0.3):
    import torch

    from paper_2403_18761_amd import rpd

    mesh = rpd.Mesh(_dev(prob.vx, torch.float32), _dev(prob.vy, torch.float32), _dev(prob.vz, torch.float32),
                    _dev(prob.tv.reshape(-1), torch.int32))
    sites = tuple(_dev(x, torch.float32) for x in (prob.sx, prob.sy, prob.sz, prob.sr))
    res = rpd.build([mesh], [sites])
    xyzr = np.stack([prob.sx, prob.sy, prob.sz, prob.sr], axis=1)
    return res.medial_mesh(0, xyzr, sigma)


def _gpu_dist(S, E, F, q):
    import torch

    from paper_2403_18761_amd import rpd

    d, n = rpd.envelope_distance(_dev(S, torch.float32), _dev(E, torch.int32), _dev(F, torch.int32),
                                 _dev(q, torch.float32))
    torch.cuda.synchronize()
    return d.cpu().numpy(), n.cpu().numpy()


def _check(S, E, F, q, d, near, label):
    from oracle import envelope as env

    want, _, values = env.envelope_distance(S, E, F, q)
    tol = ATOL + RTOL * np.abs(want)
    fin = np.isfinite(want)
    np.testing.assert_array_equal(np.isfinite(d), fin, err_msg=label)
    err = np.abs(d[fin] - want[fin])
    assert np.all(err <= tol[fin]), (label, float(err.max()), int(np.argmax(err / tol[fin])))
    # the chosen element reaches the minimum within the bound
    for eid in np.unique(near[fin]):
        m = fin & (near == eid)
        assert np.all(np.abs(values(int(eid))[m] - want[m]) <= 2 * tol[m]), (label, int(eid))
    assert np.all(near[~fin] == -1)


@pytest.mark.parametrize("case,sigma", [("torus16_n64", 0.3), ("torus16_n64", None), ("cube4_n40", 0.1)])
def test_envelope_matches_oracle(case, sigma):
    prob = {"torus16_n64": lambda: synth.torus_core(16, 64, 1),
            "cube4_n40": lambda: synth.cube_random(N=4, n_sites=40, seed=9)}[case]()
    S, E, F = _medial(prob, sigma)
    q = synth.surface_samples(prob, 3001, seed=1)  # ragged against 1024 samples per workgroup
    log(f"case: envelope {case} sigma {sigma}: {len(S)} spheres {len(E)} cones {len(F)} slabs {len(q)} samples")
    d, near = _gpu_dist(S, E, F, q)
    _check(S, E, F, q, d, near, case)


def test_host_pointers_give_the_same_bits():
    from paper_2403_18761_amd import rpd

    prob = synth.torus_core(16, 64, 1)
    S, E, F = _medial(prob)
    q = synth.surface_samples(prob, 2000, seed=2)
    log("case: envelope host pointers")
    d0, n0 = _gpu_dist(S, E, F, q)
    d1, n1 = rpd.envelope_distance(S, E, F, q)
    np.testing.assert_array_equal(d0, d1)
    np.testing.assert_array_equal(n0, n1)


def test_edge_cases():
    from paper_2403_18761_amd import rpd

    rng = np.random.default_rng(3)
    q = rng.uniform(-1, 1, size=(777, 3)).astype(np.float32)
    S = np.array([[0.0, 0.0, 0.0, 0.5], [0.1, 0.0, 0.0, 0.2],      # cone with a contained end sphere
                  [0.5, 0.5, 0.0, 0.0], [-0.5, 0.5, 0.0, 0.0],     # zero radii: a segment
                  [0.0, -0.5, 0.25, 0.1], [0.25, -0.5, 0.25, 0.1], [0.5, -0.5, 0.25, 0.1],  # collinear centres
                  [0.0, 0.0, 0.75, 0.05], [0.5, 0.25, 0.75, 0.25], [-0.25, 0.5, 0.5, 0.125]], np.float32)
    E = np.array([[0, 1], [2, 3], [4, 5], [4, 6], [5, 6], [7, 8], [7, 9], [8, 9]], np.int32)
    F = np.array([[4, 5, 6], [7, 8, 9]], np.int32)
    log("case: envelope edge cases")
    for e, f in ((E, F), (E[:0], F[:0]), (E, F[:0])):
        d, near = _gpu_dist(S, e, f, q)
        _check(S, e, f, q, d, near, f"edge cases {len(e)} {len(f)}")
    d0, near0 = _gpu_dist(S, E, F, q)
    d1, none = rpd.envelope_distance(S, E, F, q, nearest=False)  # distances only: the same values
    assert none is None
    np.testing.assert_array_equal(d1, d0)
    d, near = rpd.envelope_distance(S[:0], E[:0], F[:0], q)  # no element at all
    assert np.all(np.isinf(d)) and np.all(near == -1)
    d, near = rpd.envelope_distance(S, E, F, q[:0])
    assert d.shape == (0,)
    with pytest.raises(rpd.RPDError):
        rpd.envelope_distance(S, np.array([[0, 10]], np.int32), F[:0], q)  # sphere id out of range


def test_envelope_full_size_torus_sampled():
    """The benchmark's configuration: the torus2000 medial mesh, 1M samples, distances only."""
    import time

    import torch

    from paper_2403_18761_amd import rpd

    prob = synth.torus_inside(64, 2000, 2)
    S, E, F = _medial(prob)
    q = synth.surface_samples(prob, 1_000_000, seed=4)
    log(f"case: envelope torus N64 n2000: {len(S)} spheres {len(E)} cones {len(F)} slabs, {len(q)} samples")
    t0 = time.perf_counter()
    dd, none = rpd.envelope_distance(_dev(S, torch.float32), _dev(E, torch.int32), _dev(F, torch.int32),
                                     _dev(q, torch.float32), nearest=False)
    torch.cuda.synchronize()
    log(f"gpu call {1e3 * (time.perf_counter() - t0):.1f} ms")
    d = dd.cpu().numpy()
    pick = np.random.default_rng(5).choice(len(q), size=1500, replace=False)
    d2, near2 = _gpu_dist(S, E, F, q[pick])  # the same samples with the nearest element
    np.testing.assert_array_equal(d[pick], d2)
    _check(S, E, F, q[pick], d2, near2, "torus2000 sampled")
    assert np.all(np.isfinite(d))
