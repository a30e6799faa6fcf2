"""Parity of the GPU sphere shrinking (rpd_shrink_spheres, Sec. 5.1) with the FP64 oracle of the shrinking
iteration. Bar: radius and centre within 1e-5 absolute + 1e-4 relative (FP32 ratio |q - p|^2 / 2 n.(q - p) and
edge quadratics on O(1) coordinates; the oracle stops its iteration at a relative gap of 1e-12)."""
import numpy as np
import pytest

from paper_2403_18761_amd import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(tri, n, cen, own, got, pick, label):
    from oracle import shrink as S

    for k in pick:
        c, r = S.shrink(tri, cen[k], n[k], own=int(own[k]))
        tol = 1e-5 + 1e-4 * r
        assert abs(got[k, 3] - r) <= tol, (label, int(k), float(got[k, 3]), r)
        assert np.abs(got[k, :3] - c).max() <= tol, (label, int(k))


@pytest.mark.parametrize("case", ["cube4", "torus16", "genus3_32"])
def test_shrink_matches_oracle(case):
    import torch

    from paper_2403_18761_amd import rpd

    prob = {"cube4": lambda: synth.make_problem(synth.cube_solid(4), 4, np.zeros((1, 3)), np.zeros(1)),
            "torus16": lambda: synth.torus_core(16, 64, 1),
            "genus3_32": lambda: synth.genus3_cad(N=32, n_sites=50, seed=14)}[case]()
    tri, n, cen, _, _ = synth.surface_pins(prob)
    own = np.arange(len(tri), dtype=np.int32)
    log(f"case: shrink {case}: {len(tri)} triangles")
    dev = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")
    got = rpd.shrink_spheres(dev(tri), dev(cen), dev(n), dev(own, torch.int32)).cpu().numpy()
    host = rpd.shrink_spheres(tri, cen, n, own)
    np.testing.assert_array_equal(got, host)
    assert np.all(np.isfinite(got))
    pick = np.random.default_rng(1).choice(len(tri), size=min(len(tri), 120), replace=False)
    _check(tri, n, cen, own, got, pick, case)
    if case == "cube4":  # closed form on every pin
        axis = np.argmax(np.abs(n), axis=1)
        uv = np.stack([np.delete(cen[k], axis[k]) for k in range(len(cen))])
        want = np.minimum(1 - np.abs(uv).max(axis=1), 1.0)
        np.testing.assert_allclose(got[:, 3], want, rtol=1e-5, atol=1e-6)
