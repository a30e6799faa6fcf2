"""Seeded synthetic inputs: tetrahedral meshes of solids and medial-sphere site sets.

This module only *creates inputs*. It holds none of the restricted-power-diagram arithmetic: no clipping, no
power distances between sites, no Euler characteristics of diagram elements. Both the GPU path and the CPU oracle
consume what it writes, so it must not import either of them.

Input conventions (fixed by the boundary, see the paper's problem statement in Sec. 3.2-3.3):

* the domain is [-1, 1]^3; every coordinate and radius is a float32 value on the dyadic grid 2^-20
  (round-to-nearest-even), so both sides see bit-identical inputs and exact integer predicates have small
  fixed widths;
* the solid is discretised by voxels of an N^3 grid; a voxel is kept when all 8 of its corners lie inside the
  analytic solid; each kept voxel is split into the 6 Kuhn tetrahedra along its main diagonal;
* the kept voxel set must be well-composed (no edge- or vertex-critical 2x2 / 2x2x2 configurations), so its
  boundary is a 2-manifold, must be one 6-connected component without cavities, and must have the expected Euler
  characteristic; a generator that fails a check re-draws its jitter with the next attempt number;
* site centres never repeat exactly.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Callable

import numpy as np
from scipy import ndimage

QUANTUM = 2.0 ** -20


def quantize(a) -> np.ndarray:
    """Round to the 2^-20 grid (ties to even) and return float64 values that are exact in float32."""
    q = np.round(np.asarray(a, dtype=np.float64) / QUANTUM) * QUANTUM
    return q


@dataclasses.dataclass
class Problem:
    """One shape: a positively oriented tet mesh plus a site (medial sphere) set, all float32 on the 2^-20 grid."""

    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    tv: np.ndarray  # int32 [T, 4]
    sx: np.ndarray
    sy: np.ndarray
    sz: np.ndarray
    sr: np.ndarray
    meta: dict

    @property
    def n_verts(self) -> int:
        return int(self.vx.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tv.shape[0])

    @property
    def n_sites(self) -> int:
        return int(self.sx.shape[0])

    def with_sites(self, sx, sy, sz, sr, **meta) -> "Problem":
        m = dict(self.meta)
        m.update(meta)
        return Problem(self.vx, self.vy, self.vz, self.tv,
                       np.asarray(sx, np.float32), np.asarray(sy, np.float32),
                       np.asarray(sz, np.float32), np.asarray(sr, np.float32), m)


# ----------------------------------------------------------------------------------------------------------------
# analytic solids (signed distance: negative inside)
# ----------------------------------------------------------------------------------------------------------------

def torus_sdf(R: float, r: float, c) -> Callable[[np.ndarray], np.ndarray]:
    c = np.asarray(c, dtype=np.float64)

    def f(p: np.ndarray) -> np.ndarray:
        q = p - c
        rho = np.sqrt(q[..., 0] ** 2 + q[..., 1] ** 2)
        return np.sqrt((rho - R) ** 2 + q[..., 2] ** 2) - r

    return f


def box_sdf(lo, hi) -> Callable[[np.ndarray], np.ndarray]:
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    c = 0.5 * (lo + hi)
    h = 0.5 * (hi - lo)

    def f(p: np.ndarray) -> np.ndarray:
        d = np.abs(p - c) - h
        outside = np.linalg.norm(np.maximum(d, 0.0), axis=-1)
        inside = np.minimum(np.max(d, axis=-1), 0.0)
        return outside + inside

    return f


def cylinder_sdf(axis: int, centre, radius: float) -> Callable[[np.ndarray], np.ndarray]:
    """Infinite cylinder along a coordinate axis."""
    centre = np.asarray(centre, np.float64)
    others = [k for k in range(3) if k != axis]

    def f(p: np.ndarray) -> np.ndarray:
        d0 = p[..., others[0]] - centre[others[0]]
        d1 = p[..., others[1]] - centre[others[1]]
        return np.sqrt(d0 * d0 + d1 * d1) - radius

    return f


def union_sdf(*fs):
    def f(p):
        return np.min(np.stack([g(p) for g in fs]), axis=0)
    return f


def subtract_sdf(a, *bs):
    def f(p):
        return np.max(np.stack([a(p)] + [-b(p) for b in bs]), axis=0)
    return f


# ----------------------------------------------------------------------------------------------------------------
# voxelisation, validity checks and the Kuhn split
# ----------------------------------------------------------------------------------------------------------------

def grid_coords(N: int) -> np.ndarray:
    """Grid vertex coordinates -1 + 2k/N; N must be a power of two so that they lie on the 2^-20 grid."""
    if N < 1 or N > 2 ** 19 or (N & (N - 1)) != 0:
        raise ValueError(f"grid size N={N} must be a power of two")
    return -1.0 + 2.0 * np.arange(N + 1, dtype=np.float64) / N


def voxels_inside(sdf, N: int) -> np.ndarray:
    """Boolean [N,N,N] occupancy: voxel kept iff all 8 corners have sdf < 0."""
    g = grid_coords(N)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    inside = sdf(np.stack([X, Y, Z], axis=-1)) < 0.0
    occ = np.ones((N, N, N), dtype=bool)
    for dx, dy, dz in itertools.product((0, 1), repeat=3):
        occ &= inside[dx:dx + N, dy:dy + N, dz:dz + N]
    return occ


def voxel_euler(occ: np.ndarray) -> int:
    """V - E + F - C of the closed union of the kept unit cubes (a cubical complex count)."""
    N0, N1, N2 = occ.shape
    p = np.zeros((N0 + 2, N1 + 2, N2 + 2), dtype=bool)
    p[1:-1, 1:-1, 1:-1] = occ
    C = int(occ.sum())
    # faces normal to axis a: present if either adjacent cube is present
    F = 0
    E = 0
    for a in range(3):
        sl0 = [slice(None)] * 3
        sl1 = [slice(None)] * 3
        sl0[a] = slice(0, -1)
        sl1[a] = slice(1, None)
        F += int((p[tuple(sl0)] | p[tuple(sl1)]).sum())
    # edges along axis a: present if any of the 4 cubes around it is present
    for a in range(3):
        b, c = [k for k in range(3) if k != a]
        acc = None
        for db, dc in itertools.product((0, 1), repeat=2):
            sl = [slice(None)] * 3
            sl[b] = slice(db, p.shape[b] - 1 + db)
            sl[c] = slice(dc, p.shape[c] - 1 + dc)
            t = p[tuple(sl)]
            acc = t if acc is None else (acc | t)
        E += int(acc.sum())
    acc = None
    for d in itertools.product((0, 1), repeat=3):
        sl = tuple(slice(d[k], p.shape[k] - 1 + d[k]) for k in range(3))
        t = p[sl]
        acc = t if acc is None else (acc | t)
    V = int(acc.sum())
    return V - E + F - C


def well_composed(occ: np.ndarray) -> bool:
    """No edge-critical (diagonal pair in a 2x2 block) and no vertex-critical (antipodal pair or its complement in
    a 2x2x2 block) configuration; then the boundary of the voxel union is a 2-manifold."""
    p = np.zeros(tuple(s + 2 for s in occ.shape), dtype=bool)
    p[1:-1, 1:-1, 1:-1] = occ
    n = p.shape
    for a in range(3):
        b, c = [k for k in range(3) if k != a]

        def sl(db, dc):
            s = [slice(None)] * 3
            s[b] = slice(db, n[b] - 1 + db)
            s[c] = slice(dc, n[c] - 1 + dc)
            return p[tuple(s)]

        x00, x10, x01, x11 = sl(0, 0), sl(1, 0), sl(0, 1), sl(1, 1)
        if np.any((x00 & x11 & ~x10 & ~x01) | (x10 & x01 & ~x00 & ~x11)):
            return False
    cube = {}
    for d in itertools.product((0, 1), repeat=3):
        cube[d] = p[tuple(slice(d[k], n[k] - 1 + d[k]) for k in range(3))]
    count = sum(cube[d].astype(np.int8) for d in cube)
    for d in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        e = tuple(1 - x for x in d)
        pair = cube[d] & cube[e]
        nopair = ~cube[d] & ~cube[e]
        if np.any((count == 2) & pair) or np.any((count == 6) & nopair):
            return False
    return True


def voxel_set_ok(occ: np.ndarray, expected_chi: int) -> tuple[bool, str]:
    if not occ.any():
        return False, "empty"
    if not well_composed(occ):
        return False, "not well-composed"
    six = ndimage.generate_binary_structure(3, 1)
    _, ncomp = ndimage.label(occ, structure=six)
    if ncomp != 1:
        return False, f"{ncomp} components"
    comp = np.ones(tuple(s + 2 for s in occ.shape), dtype=bool)
    comp[1:-1, 1:-1, 1:-1] = ~occ
    _, nout = ndimage.label(comp, structure=six)
    if nout != 1:
        return False, "cavity"
    chi = voxel_euler(occ)
    if chi != expected_chi:
        return False, f"chi {chi} != {expected_chi}"
    return True, "ok"


_PERMS = list(itertools.permutations(range(3)))


def kuhn_mesh(occ: np.ndarray, N: int):
    """Split every kept voxel into 6 Kuhn tets {c, c+e_p0, c+e_p0+e_p1, c+1} (positively oriented).

    Returns float32 vertex coordinates (only the grid vertices that are used, numbered in raster order) and int32
    tets [T, 4]. Voxels are emitted in raster order (x slowest), tets of one voxel consecutively.
    """
    vox = np.argwhere(occ)  # raster order
    T = vox.shape[0] * 6
    corner = np.zeros((T, 4, 3), dtype=np.int64)
    for k, perm in enumerate(_PERMS):
        e = np.eye(3, dtype=np.int64)
        offs = [np.zeros(3, np.int64)]
        acc = np.zeros(3, np.int64)
        for a in perm:
            acc = acc + e[a]
            offs.append(acc.copy())
        offs = np.stack(offs)  # [4,3]
        # orientation sign of the permutation
        sgn = np.linalg.det(np.stack([offs[1] - offs[0], offs[2] - offs[0], offs[3] - offs[0]]).astype(float))
        if sgn < 0:
            offs = offs[[0, 1, 3, 2]]
        corner[k::6] = vox[:, None, :] + offs[None, :, :]
    M = N + 1
    lin = (corner[..., 0] * M + corner[..., 1]) * M + corner[..., 2]
    used, inv = np.unique(lin.ravel(), return_inverse=True)
    tv = inv.reshape(T, 4).astype(np.int32)
    ix = used // (M * M)
    iy = (used // M) % M
    iz = used % M
    g = grid_coords(N)
    vx = g[ix].astype(np.float32)
    vy = g[iy].astype(np.float32)
    vz = g[iz].astype(np.float32)
    return vx, vy, vz, tv


def mesh_from_sdf(sdf, N: int, expected_chi: int):
    occ = voxels_inside(sdf, N)
    ok, why = voxel_set_ok(occ, expected_chi)
    return occ, ok, why


# ----------------------------------------------------------------------------------------------------------------
# solids used by the workloads
# ----------------------------------------------------------------------------------------------------------------

def jittered_torus(N: int, seed: int, max_attempts: int = 64):
    """Solid torus, nominal R=0.6, r=0.25, jittered by a seeded draw; re-drawn until the voxel set is valid.

    Jitter recipe: g ~ N(0,1)^5 from numpy's PCG64 with the given seed (attempt a uses seed*1000+a):
    R = 0.6 (1 + 0.03 g0), r = 0.25 (1 + 0.03 g1), centre offset = 0.02 (g2, g3, g4).
    Attempt 0 with ``seed=None`` is the nominal, un-jittered torus.
    """
    for attempt in range(max_attempts):
        if seed is None:
            g = np.zeros(5)
        else:
            g = np.random.default_rng(seed * 1000 + attempt).standard_normal(5)
        R = 0.6 * (1 + 0.03 * g[0])
        r = 0.25 * (1 + 0.03 * g[1])
        c = 0.02 * g[2:5]
        sdf = torus_sdf(R, r, c)
        occ, ok, why = mesh_from_sdf(sdf, N, expected_chi=0)
        if ok:
            return dict(kind="torus", R=R, r=r, c=c.tolist(), attempt=attempt, sdf=sdf, occ=occ, genus=1)
        if seed is None:
            raise RuntimeError(f"nominal torus at N={N} invalid: {why}")
    raise RuntimeError("no valid torus voxelisation found")


def genus3_solid(N: int):
    """CAD-like genus-3 solid: union of three axis-aligned boxes minus three through-cylinders of radius 0.1.

    Boxes: a bar along x and two bars along y at its ends (an H-shaped plate), all 0.8 thick in z; one cylinder
    along z through each of the three bars. The union of the boxes is a ball (chi 1); each drilled hole adds a
    handle, so chi = 1 - 3 = -2.
    """
    zl, zh = -0.4, 0.4
    b0 = box_sdf([-0.8, -0.25, zl], [0.8, 0.25, zh])
    b1 = box_sdf([-0.85, -0.85, zl], [-0.4, 0.85, zh])
    b2 = box_sdf([0.4, -0.85, zl], [0.85, 0.85, zh])
    holes = [(0.0, 0.0), (-0.625, 0.5), (0.625, -0.5)]
    cyl = [cylinder_sdf(2, [x, y, 0.0], 0.1) for x, y in holes]
    sdf = subtract_sdf(union_sdf(b0, b1, b2), *cyl)
    occ, ok, why = mesh_from_sdf(sdf, N, expected_chi=-2)
    if not ok:
        raise RuntimeError(f"genus-3 solid at N={N} invalid: {why}")
    return dict(kind="genus3", sdf=sdf, occ=occ, genus=3, sharp_edges=_genus3_sharp_edges(zl, zh, holes))


def _genus3_sharp_edges(zl, zh, holes):
    """Sharp edges of the genus-3 solid as segments and circles (the H outline, its vertical corner edges and the
    hole rims), used to place sites near them."""
    segs = []
    outline = [(-0.85, -0.85), (-0.4, -0.85), (-0.4, -0.25), (0.4, -0.25), (0.4, -0.85), (0.85, -0.85),
               (0.85, 0.85), (0.4, 0.85), (0.4, 0.25), (-0.4, 0.25), (-0.4, 0.85), (-0.85, 0.85)]
    for k in range(len(outline)):
        a = outline[k]
        b = outline[(k + 1) % len(outline)]
        for z in (zl, zh):
            segs.append(("seg", (a[0], a[1], z), (b[0], b[1], z)))
        segs.append(("seg", (a[0], a[1], zl), (a[0], a[1], zh)))
    for cx, cy in holes:
        for z in (zl, zh):
            segs.append(("circ", (cx, cy, z), 0.1))
    return segs


def _sample_edges(edges, rng, m):
    out = np.zeros((m, 3))
    idx = rng.integers(0, len(edges), size=m)
    u = rng.random(m)
    for k in range(m):
        e = edges[idx[k]]
        if e[0] == "seg":
            a = np.asarray(e[1])
            b = np.asarray(e[2])
            out[k] = a + u[k] * (b - a)
        else:
            c = np.asarray(e[1])
            ang = 2 * math.pi * u[k]
            out[k] = c + e[2] * np.array([math.cos(ang), math.sin(ang), 0.0])
    return out


def metaball_solid(N: int, seed: int, n_balls: int, handles: bool = False, max_attempts: int = 64):
    """Metaball blobs sum_k exp(-|x-c_k|^2/s_k^2) > tau, optionally joined by thin capsule handles.

    The voxel set must be valid with chi = 1 - genus, where genus is measured on the voxel set itself.
    """
    for attempt in range(max_attempts):
        rng = np.random.default_rng(seed * 1000 + attempt)
        cs = rng.uniform(-0.55, 0.55, size=(n_balls, 3))
        ss = rng.uniform(0.22, 0.35, size=n_balls)
        tau = 0.5

        def f(p, cs=cs, ss=ss):
            acc = np.zeros(p.shape[:-1])
            for c, s in zip(cs, ss):
                acc += np.exp(-np.sum((p - c) ** 2, axis=-1) / (s * s))
            return tau - acc  # negative inside (not a true distance)

        fs = [f]
        caps = []
        if handles:
            order = rng.permutation(n_balls)
            for a, b in zip(order[:-1], order[1:]):
                caps.append((cs[a], cs[b]))
            caps.append((cs[order[-1]], cs[order[0]]))
            for (a, b) in caps:
                fs.append(_capsule_sdf(a, b, 0.04))
        sdf = union_sdf(*fs) if len(fs) > 1 else f
        occ = voxels_inside(sdf, N)
        if not occ.any() or not well_composed(occ):
            continue
        six = ndimage.generate_binary_structure(3, 1)
        _, ncomp = ndimage.label(occ, structure=six)
        if ncomp != 1:
            continue
        comp = np.ones(tuple(s + 2 for s in occ.shape), dtype=bool)
        comp[1:-1, 1:-1, 1:-1] = ~occ
        _, nout = ndimage.label(comp, structure=six)
        if nout != 1:
            continue
        chi = voxel_euler(occ)
        return dict(kind="metaballs", sdf=sdf, occ=occ, genus=1 - chi, attempt=attempt, handles=len(caps))
    raise RuntimeError("no valid metaball voxelisation found")


def _capsule_sdf(a, b, rad):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)

    def f(p):
        ab = b - a
        t = np.clip(np.sum((p - a) * ab, axis=-1) / np.dot(ab, ab), 0.0, 1.0)
        q = a + t[..., None] * ab
        return np.linalg.norm(p - q, axis=-1) - rad

    return f


def box_union_solid(N: int, seed: int, max_attempts: int = 64):
    """2-4 random axis-aligned boxes whose union is one valid component."""
    for attempt in range(max_attempts):
        rng = np.random.default_rng(seed * 1000 + attempt)
        k = int(rng.integers(2, 5))
        fs = []
        for _ in range(k):
            c = rng.uniform(-0.45, 0.45, size=3)
            h = rng.uniform(0.15, 0.45, size=3)
            fs.append(box_sdf(c - h, c + h))
        sdf = union_sdf(*fs)
        occ = voxels_inside(sdf, N)
        if not occ.any() or not well_composed(occ):
            continue
        six = ndimage.generate_binary_structure(3, 1)
        _, ncomp = ndimage.label(occ, structure=six)
        if ncomp != 1:
            continue
        comp = np.ones(tuple(s + 2 for s in occ.shape), dtype=bool)
        comp[1:-1, 1:-1, 1:-1] = ~occ
        _, nout = ndimage.label(comp, structure=six)
        if nout != 1:
            continue
        chi = voxel_euler(occ)
        return dict(kind="boxes", sdf=sdf, occ=occ, genus=1 - chi, attempt=attempt)
    raise RuntimeError("no valid box union found")


def cube_solid(N: int, lo: int = 0, hi: int | None = None):
    """A Kuhn-tessellated box made of voxels [lo, hi)^3 of the N^3 grid (a convex domain)."""
    hi = N if hi is None else hi
    occ = np.zeros((N, N, N), dtype=bool)
    occ[lo:hi, lo:hi, lo:hi] = True
    return dict(kind="cube", sdf=None, occ=occ, genus=0)


# Face-connected voxel sets on a 4^3 grid whose Kuhn meshes are not manifold: two voxels that touch only at the grid
# vertex (2, 2, 2) ("vertex") or only along the grid edge x = y = 2, 1 <= z <= 2 ("edge"), joined by a path of voxels
# that stays away from that vertex or edge. Adding the voxel listed under "fix" closes the pinch (a manifold mesh).
PINCHED = {
    "vertex": dict(cells=[(1, 1, 1), (0, 1, 1), (0, 2, 1), (0, 3, 1), (1, 3, 1), (2, 3, 1), (2, 3, 2), (2, 2, 2)],
                   fix=[(2, 1, 1), (2, 2, 1)]),
    "edge": dict(cells=[(1, 1, 1), (1, 1, 0), (2, 1, 0), (2, 2, 0), (2, 2, 1)], fix=[(2, 1, 1)]),
}


def pinched_voxels(kind: str, fixed: bool = False) -> Problem:
    """The Kuhn mesh of a PINCHED voxel set (with its fix when fixed), one site at the centre of the first voxel."""
    occ = np.zeros((4, 4, 4), dtype=bool)
    for c in PINCHED[kind]["cells"] + (PINCHED[kind]["fix"] if fixed else []):
        occ[c] = True
    c0 = -1.0 + (np.asarray(PINCHED[kind]["cells"][0], np.float64) + 0.5) * 0.5
    return make_problem(dict(kind=f"pinched_{kind}", sdf=None, occ=occ, genus=0), 4, c0[None, :], np.array([0.1]))


# ----------------------------------------------------------------------------------------------------------------
# sites
# ----------------------------------------------------------------------------------------------------------------

def _dedupe_centres(c: np.ndarray, r: np.ndarray):
    _, idx = np.unique(c, axis=0, return_index=True)
    idx = np.sort(idx)
    return c[idx], r[idx]


def sample_in_voxels(occ: np.ndarray, N: int, rng, m: int) -> np.ndarray:
    """Uniform points in the union of kept voxels (every voxel has the same volume)."""
    vox = np.argwhere(occ)
    pick = vox[rng.integers(0, vox.shape[0], size=m)]
    h = 2.0 / N
    return -1.0 + (pick + rng.random((m, 3))) * h


def make_problem(solid: dict, N: int, centres: np.ndarray, radii: np.ndarray, **meta) -> Problem:
    vx, vy, vz, tv = kuhn_mesh(solid["occ"], N)
    c = quantize(centres)
    r = np.maximum(quantize(radii), 0.0)
    c, r = _dedupe_centres(c, r)
    m = {k: v for k, v in solid.items() if k not in ("sdf", "occ", "sharp_edges")}
    m.update(meta)
    m["N"] = N
    return Problem(vx, vy, vz, tv, c[:, 0].astype(np.float32), c[:, 1].astype(np.float32),
                   c[:, 2].astype(np.float32), r.astype(np.float32), m)


def torus_core_sites(solid: dict, n: int, seed: int):
    """Centres uniform in angle on the core circle plus N(0, 0.02^2) jitter; r = distance to the torus surface."""
    rng = np.random.default_rng(seed)
    R, rt, c = solid["R"], solid["r"], np.asarray(solid["c"])
    phi = rng.uniform(0.0, 2 * math.pi, size=n)
    cen = np.stack([R * np.cos(phi), R * np.sin(phi), np.zeros(n)], axis=1) + c + rng.normal(0, 0.02, (n, 3))
    rad = np.maximum(-solid["sdf"](cen), 0.0)
    return cen, rad


def inside_sites(solid: dict, N: int, n: int, seed: int, scale: float):
    """Centres uniform inside the voxelised solid; r = scale * |sdf(centre)|."""
    rng = np.random.default_rng(seed)
    cen = sample_in_voxels(solid["occ"], N, rng, n)
    rad = scale * np.abs(solid["sdf"](cen))
    return cen, rad


# ----------------------------------------------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------------------------------------------

def torus_core(N: int = 16, n_sites: int = 64, seed: int = 1) -> Problem:
    """Solid torus (R=0.6, r=0.25, seed-jittered) on an N^3 grid, sites on the jittered core circle.

    N=16, 64 sites, seed 1 is the small torus workload (~0.9k tets)."""
    solid = jittered_torus(N, seed)
    cen, rad = torus_core_sites(solid, n_sites, seed)
    return make_problem(solid, N, cen, rad, workload=f"torus_core_N{N}_n{n_sites}_s{seed}", seed=seed)


def torus_inside(N: int = 64, n_sites: int = 2000, seed: int = 2) -> Problem:
    """Solid torus on an N^3 grid, sites uniform inside with r = 0.9 |sdf|.

    N=64, 2000 sites, seed 2 is the ~118k-tet torus workload."""
    solid = jittered_torus(N, seed)
    cen, rad = inside_sites(solid, N, n_sites, seed, 0.9)
    return make_problem(solid, N, cen, rad, workload=f"torus_inside_N{N}_n{n_sites}_s{seed}", seed=seed)


def genus3_cad(N: int = 128, n_sites: int = 20000, seed: int = 3, edge_frac: float = 0.3) -> Problem:
    """Genus-3 CAD-like solid; 70% of sites uniform inside (r=|sdf|), 30% within 0.02 of a sharp edge (kept inside
    the voxelised solid, r=|sdf|: tiny radii, near-degenerate bisectors). On grids coarser than N=200 the offset
    bound is widened to 4/N so that enough such points fall in kept voxels."""
    solid = genus3_solid(N)
    rng = np.random.default_rng(seed)
    n_edge = int(round(edge_frac * n_sites))
    n_in = n_sites - n_edge
    cen_in = sample_in_voxels(solid["occ"], N, rng, n_in)
    pts = []
    occ = solid["occ"]
    # offsets up to 0.02 (or two voxels on coarse grids, where the kept voxels sit deeper than 0.02)
    delta = max(0.02, 4.0 / N)
    for _ in range(1000):
        if len(pts) >= n_edge:
            break
        m = 2 * (n_edge - len(pts)) + 16
        base = _sample_edges(solid["sharp_edges"], rng, m)
        off = rng.uniform(-delta, delta, size=(m, 3))
        p = base + off
        ijk = np.floor((p + 1.0) * N / 2.0).astype(np.int64)
        ok = np.all((ijk >= 0) & (ijk < N), axis=1)
        ok[ok] = occ[ijk[ok, 0], ijk[ok, 1], ijk[ok, 2]]
        pts.extend(p[ok][: n_edge - len(pts)])
    if len(pts) < n_edge:
        raise RuntimeError("could not place sites near the sharp edges")
    cen = np.concatenate([cen_in, np.asarray(pts).reshape(-1, 3)])
    rad = np.abs(solid["sdf"](cen))
    return make_problem(solid, N, cen, rad, workload=f"genus3_N{N}_n{n_sites}_s{seed}", seed=seed)


def cube_random(N: int = 4, n_sites: int = 8, seed: int = 0, weights: bool = True) -> Problem:
    """Convex Kuhn cube with random sites inside (radii random or all zero)."""
    solid = cube_solid(N)
    rng = np.random.default_rng(seed)
    cen = rng.uniform(-1, 1, size=(n_sites, 3))
    rad = rng.uniform(0.0, 0.3, size=n_sites) if weights else np.zeros(n_sites)
    return make_problem(solid, N, cen, rad, workload=f"cube_N{N}_n{n_sites}_s{seed}", seed=seed)


def _scaled(sdf, scale: float):
    """The solid shrunk about the origin by ``scale`` (signed distances scale with it)."""
    return lambda p: sdf(p / scale) * scale


def batch_shape(k: int, tets_target: int, n_sites: int) -> Problem:
    """Shape k of the batched workload (seed 1000+k): torus, 2-4 box union or 3-6 metaballs on a 64^3 grid, shrunk
    about the origin so that its Kuhn mesh has about ``tets_target`` tets (targets above the unshrunk size are
    capped there). If no shrink of a drawn solid stays valid, the solid is redrawn (draw d uses seed+7919 d)."""
    N = 64
    for draw in range(16):
        seed = 1000 + k + 7919 * draw
        rng = np.random.default_rng(seed)
        kind = ["torus", "boxes", "metaballs"][int(rng.integers(0, 3))]
        n_balls = int(rng.integers(3, 7))
        if kind == "torus":
            base = jittered_torus(N, seed)
            expected = 0
        elif kind == "boxes":
            base = box_union_solid(N, seed)
            expected = 1 - base["genus"]
        else:
            base = metaball_solid(N, seed, n_balls)
            expected = 1 - base["genus"]
        full = int(base["occ"].sum()) * 6
        scale = min(1.0, (tets_target / max(full, 1)) ** (1.0 / 3.0))
        for attempt in range(24):  # shrink until the voxel set is valid again
            sdf = _scaled(base["sdf"], scale)
            occ = voxels_inside(sdf, N)
            ok, _ = voxel_set_ok(occ, expected)
            if ok:
                solid = dict(base, sdf=sdf, occ=occ, scale=scale)
                cen, rad = inside_sites(solid, N, n_sites, seed, 0.9)
                return make_problem(solid, N, cen, rad, workload=f"batch_{k}", seed=seed, kind=kind, draw=draw)
            scale *= 0.985
    raise RuntimeError(f"batch shape {k}: no valid scaled voxelisation")


def batch_problems(n_shapes: int = 256, seed: int = 4):
    """The batched workload: n_shapes shapes with log-uniform sizes (5k-200k tets, 100-5k sites)."""
    t, s = batch_sizes(n_shapes, seed)
    return [batch_shape(k, int(t[k]), int(s[k])) for k in range(n_shapes)]


def batch_sizes(n_shapes: int = 256, seed: int = 4):
    """Log-uniform tet targets in [5k, 200k] and site counts in [100, 5k] for the batched workload."""
    rng = np.random.default_rng(seed)
    t = np.exp(rng.uniform(math.log(5e3), math.log(2e5), size=n_shapes)).astype(int)
    s = np.exp(rng.uniform(math.log(100), math.log(5e3), size=n_shapes)).astype(int)
    return t, s


def blobs_with_handles(N: int, seed: int, n_blobs: int = 5, max_attempts: int = 64):
    """Separate metaball blobs on a jittered ring in the xy plane (field sum_k exp(-q_k(x)) > 1/2 with
    q_k = (dx^2 + dy^2)/s_k^2 + dz^2/(1.8 s_k)^2, tall ellipsoids), each joined to the next by a thin capsule
    handle (radius 0.06, at least 3.5 voxels on coarse grids), plus one chord handle from blob 0 to blob 2: a
    genus-2 solid whose cells spanning the thin handles are the first to violate the topology constraints."""
    hr = max(0.06, 3.5 * 2.0 / N)
    for attempt in range(max_attempts):
        rng = np.random.default_rng(seed * 1000 + attempt)
        ang = 2 * math.pi * (np.arange(n_blobs) + rng.uniform(-0.06, 0.06, n_blobs)) / n_blobs
        rad = 0.65 + rng.uniform(-0.02, 0.02, n_blobs)
        cs = np.stack([rad * np.cos(ang), rad * np.sin(ang), rng.uniform(-0.05, 0.05, n_blobs)], axis=1)
        ss = rng.uniform(0.295, 0.315, n_blobs)

        def field(p, cs=cs, ss=ss):
            acc = np.zeros(p.shape[:-1])
            for c, sc in zip(cs, ss):
                d = p - c
                acc += np.exp(-(d[..., 0] ** 2 + d[..., 1] ** 2) / (sc * sc) - d[..., 2] ** 2 / (1.8 * sc) ** 2)
            return 0.5 - acc

        pairs = [(k, (k + 1) % n_blobs) for k in range(n_blobs)] + [(0, 2)]
        sdf = union_sdf(field, *[_capsule_sdf(cs[a], cs[b], hr) for a, b in pairs])
        occ = voxels_inside(sdf, N)
        ok, _ = voxel_set_ok(occ, -1)
        if ok and voxel_euler(voxels_inside(field, N)) >= n_blobs - 2:  # most blobs alone stay apart
            return dict(kind="blobs_with_handles", sdf=sdf, occ=occ, genus=2, attempt=attempt, handles=len(pairs))
    raise RuntimeError("no valid blobs-with-handles voxelisation found")


def _jittered_centroids(prob: Problem, rng) -> np.ndarray:
    """Tet centroids moved by a uniform offset of up to an eighth of the tet's shortest bounding-box side per axis,
    so that inserted spheres sit in general position (bare centroids of a Kuhn grid lie on a lattice, where
    bisectors of equal spheres pass exactly through mesh vertices)."""
    v = np.stack([prob.vx, prob.vy, prob.vz], axis=1).astype(np.float64)
    p = v[prob.tv]
    ext = (p.max(axis=1) - p.min(axis=1)).min(axis=1)
    return p.mean(axis=1) + rng.uniform(-0.125, 0.125, size=(p.shape[0], 3)) * ext[:, None]


def centroid_table(prob: Problem, radius: float, seed: int = 0):
    """An insertion table for any mesh: for every tet a sphere near its centroid (jittered, see
    _jittered_centroids) with radius uniform in [0.9, 1.1] x radius."""
    rng = np.random.default_rng(seed)
    c = quantize(_jittered_centroids(prob, rng))
    r = quantize(radius * rng.uniform(0.9, 1.1, size=c.shape[0]))
    return (c[:, 0].astype(np.float32), c[:, 1].astype(np.float32), c[:, 2].astype(np.float32),
            r.astype(np.float32))


def _edt_radius(occ: np.ndarray, N: int, pts: np.ndarray, scale: float) -> np.ndarray:
    """scale x (distance from the point's voxel centre to the nearest removed voxel centre - h/2): a distance to
    the voxelised boundary that needs no analytic signed distance."""
    edt = ndimage.distance_transform_edt(np.pad(occ, 1))[1:-1, 1:-1, 1:-1]
    ijk = np.clip(np.floor((pts + 1.0) * N / 2.0).astype(np.int64), 0, N - 1)
    h = 2.0 / N
    return scale * np.maximum(edt[ijk[:, 0], ijk[:, 1], ijk[:, 2]] - 0.5, 0.0) * h


def repair_problem(N: int = 128, n_sites: int = 500, seed: int = 5):
    """The topology-repair workload: the genus-2 blobs-with-handles solid on an N^3 grid (about 1M Kuhn tets at
    N=128), n_sites initial spheres uniform inside, and the insertion table: for every tet, a sphere near its
    centroid (jittered into general position). Radii: 0.9 x (table: uniform 0.85-0.95 x) the voxel distance to
    the boundary. Returns (Problem, table) with table = (tx, ty, tz, tr) float32 arrays in the problem's tet
    order."""
    solid = blobs_with_handles(N, seed)
    rng = np.random.default_rng(seed)
    cen = sample_in_voxels(solid["occ"], N, rng, n_sites)
    rad = _edt_radius(solid["occ"], N, cen, 0.9)
    prob = make_problem(solid, N, cen, rad, workload=f"repair_N{N}_n{n_sites}_s{seed}", seed=seed)
    cent = _jittered_centroids(prob, rng)
    tc = quantize(cent)
    tr = np.maximum(quantize(_edt_radius(solid["occ"], N, cent, 1.0) * rng.uniform(0.85, 0.95, cent.shape[0])), 0.0)
    table = (tc[:, 0].astype(np.float32), tc[:, 1].astype(np.float32), tc[:, 2].astype(np.float32),
             tr.astype(np.float32))
    return prob, table


def tiny_two_tets() -> tuple:
    """Two positively oriented tets sharing one face (a bipyramid), vertices on the 2^-20 grid."""
    v = np.array([[0, 0, 0], [0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5], [0.25, 0.25, -0.5]], dtype=np.float64)
    tv = np.array([[0, 1, 2, 3], [0, 2, 1, 4]], dtype=np.int32)
    return v.astype(np.float32), tv


# ----------------------------------------------------------------------------------------------------------------
# surface samples (inputs of the geometric-error metric)
# ----------------------------------------------------------------------------------------------------------------

def boundary_triangles(prob: Problem) -> np.ndarray:
    """Faces of the tet mesh that belong to one tet only (the surface), as (m, 3) vertex ids."""
    tv = np.asarray(prob.tv).reshape(-1, 4)
    faces = np.concatenate([tv[:, [1, 2, 3]], tv[:, [0, 2, 3]], tv[:, [0, 1, 3]], tv[:, [0, 1, 2]]])
    key = np.sort(faces, axis=1)
    uniq, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    return uniq[cnt == 1]


def surface_samples(prob: Problem, n: int, seed: int) -> np.ndarray:
    """n points uniformly distributed over the surface of the tet mesh (area-weighted triangles, uniform
    barycentric), float32 (n, 3)."""
    rng = np.random.default_rng(seed)
    tri = boundary_triangles(prob)
    P = np.stack([prob.vx, prob.vy, prob.vz], axis=1).astype(np.float64)
    a, b, c = P[tri[:, 0]], P[tri[:, 1]], P[tri[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    pick = rng.choice(len(tri), size=n, p=area / area.sum())
    u, v = rng.random(n), rng.random(n)
    flip = u + v > 1
    u[flip], v[flip] = 1 - u[flip], 1 - v[flip]
    q = a[pick] + u[:, None] * (b[pick] - a[pick]) + v[:, None] * (c[pick] - a[pick])
    return q.astype(np.float32)


# ----------------------------------------------------------------------------------------------------------------
# general (non-voxel) tet meshes
# ----------------------------------------------------------------------------------------------------------------

def delaunay_ball(n_points: int = 400, n_sites: int = 40, seed: int = 0, radius: float = 0.9) -> Problem:
    """Delaunay tetrahedralisation of random grid points in a ball (a convex, single-component tet mesh whose
    vertex multiplicities are irregular, so the lcm of multiplicities is far beyond 2^31), with random weighted
    sites inside."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n_points, 3))
    pts = d / np.linalg.norm(d, axis=1, keepdims=True) * radius * rng.random((n_points, 1)) ** (1 / 3)
    pts = np.unique(quantize(pts), axis=0)
    tv = Delaunay(pts).simplices.astype(np.int64)
    P = np.round(pts * (1 << 20)).astype(np.int64)  # exact grid integers for the orientation test
    a, b, c, e = (P[tv[:, k]] for k in range(4))
    det = np.einsum("ij,ij->i", b - a, np.cross(c - a, e - a))
    if np.any(det == 0):
        raise ValueError("flat tet in the Delaunay tetrahedralisation; use another seed")
    neg = det < 0
    tv[neg, 0], tv[neg, 1] = tv[neg, 1].copy(), tv[neg, 0].copy()
    # sites: random points of random tets, radii up to 0.15
    pick = rng.integers(0, len(tv), n_sites)
    w = rng.dirichlet(np.ones(4), size=n_sites)
    cen = np.einsum("ik,ikj->ij", w, pts[tv[pick]])
    rad = rng.uniform(0.0, 0.15, size=n_sites)
    c = quantize(cen)
    r = np.maximum(quantize(rad), 0.0)
    c, r = _dedupe_centres(c, r)
    meta = dict(kind="delaunay_ball", workload=f"delaunay_ball_p{n_points}_n{n_sites}_s{seed}", seed=seed, N=0,
                genus=0)
    return Problem(pts[:, 0].astype(np.float32), pts[:, 1].astype(np.float32), pts[:, 2].astype(np.float32),
                   tv.astype(np.int32), c[:, 0].astype(np.float32), c[:, 1].astype(np.float32),
                   c[:, 2].astype(np.float32), r.astype(np.float32), meta)


def surface_pins(prob: Problem):
    """Boundary triangles of the tet mesh as (m, 3, 3) float32 vertex coordinates, their inward unit normals, their
    centroids (the pin points of sphere shrinking), and the (tet, local face) each comes from (face f is opposite the
    tet's vertex f)."""
    tv = np.asarray(prob.tv).reshape(-1, 4)
    nt = len(tv)
    faces = np.concatenate([tv[:, [1, 2, 3]], tv[:, [0, 2, 3]], tv[:, [0, 1, 3]], tv[:, [0, 1, 2]]])
    tet = np.tile(np.arange(nt), 4)
    loc = np.repeat(np.arange(4), nt)
    key = np.sort(faces, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    b = cnt[inv.reshape(-1)] == 1
    faces, tet, loc = faces[b], tet[b], loc[b]
    P = np.stack([prob.vx, prob.vy, prob.vz], axis=1).astype(np.float64)
    tri = P[faces]
    n = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    opp = P[tv[tet, loc]]
    flip = np.einsum("ij,ij->i", n, opp - tri[:, 0]) < 0
    n[flip] = -n[flip]
    order = np.lexsort((loc, tet))
    return (tri[order].astype(np.float32), n[order].astype(np.float32), tri[order].mean(axis=1).astype(np.float32),
            tet[order].astype(np.int32), loc[order].astype(np.int32))
