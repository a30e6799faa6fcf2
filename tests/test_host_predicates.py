"""The FP64 filter of the clipping kernels (side64 with the FP64 face and bisector planes, from rpd_device.h) compiled
for the host and checked against exact rational arithmetic: it may answer "undecided" (0), but a sign it returns must
be the exact sign, and an exact zero must come back undecided. Cases: large and nearly flat grid-aligned tets (where
the offsets of face planes carry many bits), bisectors, and exact ties (a bisector through a tet vertex)."""
import ctypes as C
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
Q = 2.0 ** -20


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("hostpred") / "libhostpred.so")
    src = os.path.join(HERE, "host_predicates.cpp")
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-shared", "-fPIC",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2403_18761_amd", "csrc"), src,
           "-o", out]
    if not os.path.exists(cmd[0]):
        pytest.skip("hipcc not available")
    subprocess.check_call(cmd)
    L = C.CDLL(out)
    L.host_side64.argtypes = [C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_int, C.POINTER(C.c_int),
                              C.POINTER(C.c_double)]
    L.host_side64.restype = C.c_int
    return L


def exact_planes(tv, sites, si, ids):
    """Exact rational planes in the tet-local frame (origin = vertex 0), float units."""
    y = [[Fraction(float(tv[v][k])) - Fraction(float(tv[0][k])) for k in range(3)] for v in range(4)]
    out = []
    for p in ids:
        if p < 4:
            o = [v for v in range(4) if v != p]
            u = [y[o[1]][k] - y[o[0]][k] for k in range(3)]
            w = [y[o[2]][k] - y[o[0]][k] for k in range(3)]
            n = [u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]]
            if sum(n[k] * (y[p][k] - y[o[0]][k]) for k in range(3)) < 0:
                n = [-x for x in n]
            out.append((n, -sum(n[k] * y[o[0]][k] for k in range(3))))
        else:
            ci = [Fraction(float(sites[si][k])) for k in range(3)]
            cj = [Fraction(float(sites[p - 4][k])) for k in range(3)]
            o = [Fraction(float(tv[0][k])) for k in range(3)]

            def D(c, r):
                return sum((c[k] - o[k]) ** 2 for k in range(3)) - Fraction(float(r)) ** 2

            n = [2 * (ci[k] - cj[k]) for k in range(3)]
            out.append((n, D(cj, sites[p - 4][3]) - D(ci, sites[si][3])))
    return out


def exact_sign(planes):
    (a, da), (b, db), (c, dc), (q, dq) = planes

    def det3(r0, r1, r2):
        return (r0[0] * (r1[1] * r2[2] - r1[2] * r2[1]) - r0[1] * (r1[0] * r2[2] - r1[2] * r2[0]) +
                r0[2] * (r1[0] * r2[1] - r1[1] * r2[0]))

    W = det3(a, b, c)
    if W == 0:
        return None
    rhs = [-da, -db, -dc]
    x = [det3(*[[rhs[r] if k == col else (a, b, c)[r][k] for k in range(3)] for r in range(3)]) / W
         for col in range(3)]
    v = sum(q[k] * x[k] for k in range(3)) + dq
    return (v > 0) - (v < 0)


def grid(rng, lo, hi, n):
    return np.round(rng.uniform(lo, hi, n) / Q) * Q


def call(lib, tv, sites, si, ids):
    tvf = np.ascontiguousarray(tv, np.float32).reshape(-1)
    sf = np.ascontiguousarray(sites, np.float32).reshape(-1)
    idc = np.ascontiguousarray(ids, np.int32)
    po = np.zeros(16)
    s = lib.host_side64(tvf.ctypes.data_as(C.POINTER(C.c_float)), sf.ctypes.data_as(C.POINTER(C.c_float)), si,
                        idc.ctypes.data_as(C.POINTER(C.c_int)), po.ctypes.data_as(C.POINTER(C.c_double)))
    return s, po.reshape(4, 4)


def positive(tv):
    a, b, c = tv[1] - tv[0], tv[2] - tv[0], tv[3] - tv[0]
    return np.dot(a.astype(np.float64), np.cross(b.astype(np.float64), c.astype(np.float64))) > 0


def flat_tet(rng):
    """Three large grid-aligned vertices and a fourth a few grid units off their plane (a nearly flat tet)."""
    while True:
        p = grid(rng, -1, 1, 9).reshape(3, 3)
        t = rng.uniform(0.1, 0.8, 2)
        apex = p[0] + t[0] * (p[1] - p[0]) + t[1] * (p[2] - p[0])
        n = np.cross(p[1] - p[0], p[2] - p[0])
        apex = apex + n / np.linalg.norm(n) * Q * rng.integers(1, 4)
        apex = np.round(apex / Q) * Q
        if np.all(np.abs(apex) <= 1):
            tv = np.vstack([p, apex])
            if not positive(tv):
                tv = tv[[1, 0, 2, 3]]
            if positive(tv):
                return tv


def test_side64_never_contradicts_exact(lib):
    rng = np.random.default_rng(7)
    wrong = undecided = decided = ties = 0
    for case in range(600):
        tv = flat_tet(rng) if case % 2 == 0 else np.vstack([grid(rng, -1, 1, 3) for _ in range(4)])
        if not positive(tv):
            tv = tv[[1, 0, 2, 3]]
        if not positive(tv):
            continue
        sites = np.hstack([grid(rng, -1, 1, 15).reshape(5, 3), grid(rng, 0, 0.5, 5)[:, None]])
        if case % 3 == 0:  # a bisector through a tet vertex: site 1 is site 0 reflected through vertex v
            v = tv[rng.integers(0, 4)]
            refl = 2 * v - sites[0, :3]
            if np.all(np.abs(refl) <= 1):
                sites[1, :3] = refl
                sites[1, 3] = sites[0, 3]
        for _ in range(6):
            kind = rng.integers(0, 3)
            if kind == 0:  # a tet vertex (three faces) against a bisector
                f = list(rng.permutation(4)[:3])
                ids = f + [4 + int(rng.integers(1, 5))]
            elif kind == 1:  # two faces and a bisector against another bisector
                f = list(rng.permutation(4)[:2])
                b = rng.permutation(np.arange(1, 5))[:2]
                ids = f + [4 + int(b[0]), 4 + int(b[1])]
            else:  # a bisector vertex against a face plane
                f = int(rng.integers(0, 4))
                b = rng.permutation(np.arange(1, 5))[:3]
                ids = [4 + int(b[0]), 4 + int(b[1]), 4 + int(b[2]), f]
            ex = exact_sign(exact_planes(tv, sites, 0, ids))
            if ex is None:
                continue
            s, _ = call(lib, tv, sites, 0, ids)
            if ex == 0:
                ties += 1
                assert s == 0, ("exact tie decided", case, ids, s)
            if s == 0:
                undecided += 1
            elif s != ex:
                wrong += 1
            else:
                decided += 1
    assert wrong == 0, wrong
    assert ties > 0 and decided > 100, (ties, decided)


def test_face_plane_offsets_are_once_rounded(lib):
    """The FP64 face plane equals the exact integer plane with the normal exact and the offset rounded once."""
    rng = np.random.default_rng(3)
    for _ in range(300):
        tv = flat_tet(rng)
        sites = np.zeros((1, 4))
        _, po = call(lib, tv, sites, 0, [0, 1, 2, 3])
        ex = exact_planes(tv, sites, 0, [0, 1, 2, 3])
        for k in range(4):
            n, d = ex[k]
            assert all(Fraction(po[k, c]) == n[c] for c in range(3))
            assert po[k, 3] == float(d)  # Python rounds a Fraction to the nearest double (ties to even)
