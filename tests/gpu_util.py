"""Helpers for the GPU tests: run the HIP path through the C ABI and compare with the oracle."""
import sys

import numpy as np


def run_gpu(prob, precision=0, clip_budget=0, block=0, flags=0, device_ptrs=True, slots=0):
    import torch

    from paper_2403_18761_amd import rpd

    if device_ptrs:
        dev = torch.device("cuda:0")

        def t(a, dt=torch.float32):
            return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)

        mesh = rpd.Mesh(t(prob.vx), t(prob.vy), t(prob.vz), t(prob.tv.reshape(-1), torch.int32))
        sites = (t(prob.sx), t(prob.sy), t(prob.sz), t(prob.sr))
    else:
        mesh = rpd.Mesh(prob.vx, prob.vy, prob.vz, prob.tv.reshape(-1))
        sites = (prob.sx, prob.sy, prob.sz, prob.sr)
    res = rpd.build([mesh], [sites], precision=precision, clip_budget=clip_budget, block=block, flags=flags,
                    slots=slots)
    out = extract(res, 0)
    out["stats"] = res.stats()
    out["mesh_info"] = mesh.info()
    out["max_tet_vol"] = max_tet_volume(prob)
    out["radii"] = np.asarray(prob.sr, np.float64)
    if flags & rpd.RPD_KEEP_PIECES:
        out["pieces"] = res.pieces(0)
    return out


ELEMENT_ARRAYS = ("cell_chi", "cell_beta0", "face_keys", "face_chi", "face_beta0", "edge_keys", "edge_chi",
                  "edge_beta0", "rpv_keys", "cell_vol", "cell_cen", "edge_len", "edge_alpha", "medial")


def extract(res, k):
    """Every per-element array of shape k of a Result, as numpy arrays."""
    from paper_2403_18761_amd import rpd

    out = {}
    _, out["cell_chi"] = res.euler(k, rpd.RPD_CELL)
    _, out["cell_beta0"] = res.components(k, rpd.RPD_CELL)
    out["face_keys"], out["face_chi"] = res.euler(k, rpd.RPD_FACE)
    _, out["face_beta0"] = res.components(k, rpd.RPD_FACE)
    out["edge_keys"], out["edge_chi"] = res.euler(k, rpd.RPD_EDGE)
    _, out["edge_beta0"] = res.components(k, rpd.RPD_EDGE)
    out["rpv_keys"] = res.adjacency(k, rpd.RPD_VERTEX)
    out["cell_vol"], out["cell_cen"] = res.geometry(k)
    out["edge_len"], out["edge_alpha"] = res.edge_geometry(k)
    counts, chi = res.medial_euler(k)
    out["medial"] = np.array([*counts, chi], np.int64)  # V, E, F, T, chi of the dual medial mesh
    return out


def max_tet_volume(prob):
    v = np.stack([prob.vx, prob.vy, prob.vz], axis=1).astype(np.float64)
    p = v[prob.tv]
    d = np.einsum("ij,ij->i", p[:, 1] - p[:, 0], np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]))
    return float(np.abs(d).max()) / 6.0


def volume_floor(g, r, vol_rtol):
    """Absolute volume tolerance: a piece built from rounded vertices errs by about 6 u vol(t), at the scale of the
    tet it cuts and not of its own volume, so a cell of a few slivers carries that error whatever its size; the
    floor is vol_rtol / 10 times the largest tet volume (1e-6 vol(t) on the FP32 path), and never below vol_rtol
    1e-6 times the largest cell volume."""
    f = vol_rtol * 1e-6 * max(float(r["cell_vol"].max()), 1e-30)
    if "max_tet_vol" in g:
        f = max(f, 0.1 * vol_rtol * g["max_tet_vol"])
    return f


def assert_parity(g, r, vol_rtol=1e-5, label=""):
    """Bit-exact chi / beta0 / adjacency; volumes and first moments within FP32 tolerance."""
    # the oracle's own cross-checks (divisibility, cross-side symmetry, gluing symmetry) must hold before its result
    # serves as the reference
    if "consistent" in r:
        assert r["consistent"], (label, r.get("report"))
    np.testing.assert_array_equal(g["cell_chi"], r["cell_chi"], err_msg=f"{label} cell chi")
    np.testing.assert_array_equal(g["cell_beta0"], r["cell_beta0"], err_msg=f"{label} cell beta0")
    np.testing.assert_array_equal(g["face_keys"], r["face_keys"], err_msg=f"{label} face keys")
    np.testing.assert_array_equal(g["face_chi"], r["face_chi"], err_msg=f"{label} face chi")
    np.testing.assert_array_equal(g["face_beta0"], r["face_beta0"], err_msg=f"{label} face beta0")
    np.testing.assert_array_equal(g["edge_keys"], r["edge_keys"], err_msg=f"{label} edge keys")
    np.testing.assert_array_equal(g["edge_chi"], r["edge_chi"], err_msg=f"{label} edge chi")
    np.testing.assert_array_equal(g["edge_beta0"], r["edge_beta0"], err_msg=f"{label} edge beta0")
    np.testing.assert_array_equal(g["rpv_keys"], r["rpv_keys"], err_msg=f"{label} rpv keys")
    assert g["stats"]["n_pairs"] == r["n_pairs"], (label, g["stats"]["n_pairs"], r["n_pairs"])
    vr = r["cell_vol"]
    atol = volume_floor(g, r, vol_rtol)
    np.testing.assert_allclose(g["cell_vol"], vr, rtol=vol_rtol, atol=atol, err_msg=f"{label} volumes")
    ne = vr > 0
    np.testing.assert_array_equal(np.isnan(g["cell_cen"][:, 0]), ~ne, err_msg=f"{label} empty cells")
    # First moments M = vol * centroid, for every nonempty cell however small: a piece's moment is its volume times
    # a position with |x| <= sqrt 3 (plus the position's own rounding, far below), so the moment error of a cell is
    # at most sqrt 3 times its volume error; both volume terms (relative and absolute floor) carry over. Tiny cells are
    # held to the same absolute floor as their volumes.
    mg = g["cell_cen"][ne] * g["cell_vol"][ne, None]
    mr = r["cell_cen"][ne] * vr[ne, None]
    err = np.abs(mg - mr).max(axis=1, initial=0.0)
    bound = 2 * np.sqrt(3.0) * (vol_rtol * vr[ne] + atol)
    assert np.all(err <= bound), (label, "first moments", (err / bound).max(initial=0.0))
    # RPE lengths: a segment's endpoint is where the line of two bisector planes crosses a third plane; the planes
    # are rounded to the working precision, so the endpoint errs by u |x| / sin(angle of line and plane), and
    # shallow crossings amplify u = 6e-8 (FP32) by 10^2..10^3 where the volumes, integrals over the piece, average
    # it out. Lengths are held to 10x the volume tolerance (FP32: 1e-4 relative, 1e-5 absolute; FP64: 1e-8, 1e-9).
    len_rtol, len_atol = 10 * vol_rtol, vol_rtol
    np.testing.assert_allclose(g["edge_len"], r["edge_length"], rtol=len_rtol, atol=len_atol,
                               err_msg=f"{label} RPE lengths")
    from oracle import medial

    counts, chi = medial.medial_counts(r)
    np.testing.assert_array_equal(g["medial"], [*counts, chi], err_msg=f"{label} medial mesh counts")
    if "radii" in g:
        a_ref = medial.edge_alpha(r["edge_length"], r["edge_keys"], g["radii"])
        d = 2.0 * g["radii"][r["edge_keys"]].mean(axis=1) if len(a_ref) else np.zeros(0)
        tol = len_rtol * np.abs(a_ref) + len_atol / np.maximum(d, 1e-30)  # the length's tolerance over d
        finite = np.isfinite(a_ref)
        np.testing.assert_array_equal(np.isfinite(g["edge_alpha"]), finite, err_msg=f"{label} RPE importance")
        err = np.abs(g["edge_alpha"][finite] - a_ref[finite])
        assert np.all(err <= tol[finite]), (label, "RPE importance", (err / tol[finite]).max(initial=0.0))


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu_batch(probs, precision=0, flags=0):
    """Several shapes in one rpd_build call; returns one dict per shape in the layout of run_gpu."""
    import torch

    from paper_2403_18761_amd import rpd

    dev = torch.device("cuda:0")

    def t(a, dt=torch.float32):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)

    meshes = [rpd.Mesh(t(p.vx), t(p.vy), t(p.vz), t(p.tv.reshape(-1), torch.int32)) for p in probs]
    sites = [(t(p.sx), t(p.sy), t(p.sz), t(p.sr)) for p in probs]
    res = rpd.build(meshes, sites, precision=precision, flags=flags)
    outs = []
    for k in range(len(probs)):
        out = extract(res, k)
        out["mesh_info"] = meshes[k].info()
        out["max_tet_vol"] = max_tet_volume(probs[k])
        out["radii"] = np.asarray(probs[k].sr, np.float64)
        outs.append(out)
    return outs, res.stats()
