"""The no-allocation entry point (rpd_envelope_distance_noalloc) through the C ABI: its results equal those of
rpd_envelope_distance bit for bit, on two calls in a row (the second with fewer samples and elements, so that it
reuses the scratch region the first one left behind), and inputs beyond its fixed region are rejected before any
device work."""
import numpy as np
import pytest

from paper_2403_18761_amd import synth
from tests.gpu_util import log


def _dev(a, dt):
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


def _both(S, E, F, q):
    import torch

    from paper_2403_18761_amd import rpd

    dS, dE, dF, dq = _dev(S, torch.float32), _dev(E, torch.int32), _dev(F, torch.int32), _dev(q, torch.float32)
    want_d, want_n = rpd.envelope_distance(dS, dE, dF, dq)
    dist = torch.full((len(q),), -7.0, dtype=torch.float32, device="cuda:0")
    near = torch.full((len(q),), -7, dtype=torch.int32, device="cuda:0")
    rpd.envelope_distance_noalloc(dS, dE, dF, dq, dist, near)
    only = torch.full((len(q),), -7.0, dtype=torch.float32, device="cuda:0")
    rpd.envelope_distance_noalloc(dS, dE, dF, dq, only, None)
    torch.cuda.synchronize()
    return (want_d.cpu().numpy(), want_n.cpu().numpy()), (dist.cpu().numpy(), near.cpu().numpy()), only.cpu().numpy()


@pytest.mark.gpu
def test_noalloc_equals_envelope_distance_twice():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    prob = synth.torus_inside(32, 400, 5)
    S, E, F = _medial(prob)
    big = synth.surface_samples(prob, 60000, seed=1)
    log(f"case: no-alloc envelope, {len(S)} spheres {len(E)} cones {len(F)} slabs, {len(big)} then fewer samples")
    (wd, wn), (gd, gn), only = _both(S, E, F, big)
    np.testing.assert_array_equal(gd, wd)
    np.testing.assert_array_equal(gn, wn)
    np.testing.assert_array_equal(only, wd)
    # second call: fewer samples and a sub-complex (spheres only and the first edges), so that stale minima or
    # records of the first call would show
    small = big[:7000] * np.float32(0.9)
    k = len(E) // 3
    sub_e = E[:k]
    (wd2, wn2), (gd2, gn2), only2 = _both(S, sub_e, np.zeros((0, 3), np.int32), small)
    np.testing.assert_array_equal(gd2, wd2)
    np.testing.assert_array_equal(gn2, wn2)
    np.testing.assert_array_equal(only2, wd2)
    assert np.all(np.isfinite(gd2)) and np.all(gn2 >= 0)


@pytest.mark.gpu
def test_noalloc_rejects_bad_ids():
    import torch

    from paper_2403_18761_amd import rpd

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S = _dev(np.array([[0, 0, 0, 0.5], [1, 0, 0, 0.5]], np.float32), torch.float32)
    E = _dev(np.array([[0, 5]], np.int32), torch.int32)
    F = _dev(np.zeros((0, 3), np.int32), torch.int32)
    q = _dev(np.zeros((4, 3), np.float32), torch.float32)
    dist = torch.empty(4, dtype=torch.float32, device="cuda:0")
    with pytest.raises(rpd.RPDError) as e:
        rpd.envelope_distance_noalloc(S, E, F, q, dist)
    assert e.value.code == rpd.RPD_E_INVALID
    E = _dev(np.array([[0, 1]], np.int32), torch.int32)
    rpd.envelope_distance_noalloc(S, E, F, q, dist)  # a valid call afterwards works
    torch.cuda.synchronize()
    assert np.allclose(dist.cpu().numpy(), -0.5)


def test_noalloc_limit_checked_before_device_work():
    """Over the region's size: RPD_E_NOMEM from the argument checks alone (no device is touched, so this runs on
    the CPU; the pointers are never dereferenced)."""
    import ctypes as C

    from paper_2403_18761_amd import rpd

    lib = rpd.load()
    dummy = np.zeros(16, np.float32)
    p = C.c_void_p(dummy.ctypes.data)
    n = rpd.RPD_NOALLOC_SCRATCH_BYTES // 8  # the per-sample minima alone fill the region
    rc = lib.rpd_envelope_distance_noalloc(p, 1, None, 0, None, 0, p, n, None, p, None)
    assert rc == rpd.RPD_E_NOMEM
    assert b"scratch" in lib.rpd_last_error()
    rc = lib.rpd_envelope_distance_noalloc(p, 1, None, -1, None, 0, p, 4, None, p, None)
    assert rc == rpd.RPD_E_INVALID
