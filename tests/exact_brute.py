"""Exact-rational brute force for tiny inputs: an independent pin for the oracle (not the oracle itself).

It shares no algorithm with the oracle: instead of incremental clipping with plane-index bookkeeping and
fractional weights, every piece t & Omega_i is found by enumerating ALL triples of its bounding planes, solving each
exactly with Python ``Fraction`` arithmetic and keeping the feasible points; the Euler characteristic of every
restricted element is then counted as V - E + F - C on the complex obtained by merging the pieces' vertices, edges
and faces by their exact coordinates; beta0 is the number of connected components of that complex's 1-skeleton;
volumes are exact rationals. Only usable for a handful of tets and sites.
"""
from __future__ import annotations

import itertools
from fractions import Fraction as Fr


class Degenerate(Exception):
    pass


def _solve3(P):
    A = [[Fr(p[0]), Fr(p[1]), Fr(p[2]), -Fr(p[3])] for p in P]
    for col in range(3):
        piv = next((r for r in range(col, 3) if A[r][col] != 0), None)
        if piv is None:
            return None
        A[col], A[piv] = A[piv], A[col]
        for r in range(3):
            if r != col and A[r][col] != 0:
                f = A[r][col] / A[col][col]
                A[r] = [A[r][k] - f * A[col][k] for k in range(4)]
    return tuple(A[k][3] / A[k][k] for k in range(3))


def _val(pl, p):
    return pl[0] * p[0] + pl[1] * p[1] + pl[2] * p[2] + pl[3]


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _find(par, x):
    while par[x] != x:
        par[x] = par[par[x]]
        x = par[x]
    return x


def _components(points, edges):
    idx = {p: k for k, p in enumerate(points)}
    par = list(range(len(points)))
    for e in edges:
        a, b = tuple(e)
        ra, rb = _find(par, idx[a]), _find(par, idx[b])
        if ra != rb:
            par[ra] = rb
    return sum(1 for k in range(len(points)) if _find(par, k) == k)


def brute_rpd(prob):
    V = [tuple(Fr(float(c)) for c in (prob.vx[k], prob.vy[k], prob.vz[k])) for k in range(prob.n_verts)]
    S = [((Fr(float(prob.sx[k])), Fr(float(prob.sy[k])), Fr(float(prob.sz[k]))), Fr(float(prob.sr[k])) ** 2)
         for k in range(prob.n_sites)]
    n = len(S)
    pieces = {}  # (t, i) -> dict(points, tight, edges, faces, vol, mom)
    for t, tet in enumerate(prob.tv.tolist()):
        P = [V[a] for a in tet]
        faces = []
        for f in range(4):
            o = [P[k] for k in range(4) if k != f]
            nrm = _cross(_sub(o[1], o[0]), _sub(o[2], o[0]))
            if _dot(nrm, _sub(P[f], o[0])) < 0:
                nrm = tuple(-x for x in nrm)
            faces.append((nrm[0], nrm[1], nrm[2], -_dot(nrm, o[0])))
        for i in range(n):
            ci, wi = S[i]
            planes = [("f", f, faces[f]) for f in range(4)]
            for j in range(n):
                if j == i:
                    continue
                cj, wj = S[j]
                nrm = tuple(2 * (ci[k] - cj[k]) for k in range(3))
                d = _dot(cj, cj) - wj - _dot(ci, ci) + wi
                planes.append(("b", j, (nrm[0], nrm[1], nrm[2], d)))
            pts = {}
            for a, b, c in itertools.combinations(range(len(planes)), 3):
                p = _solve3([planes[a][2], planes[b][2], planes[c][2]])
                if p is None or p in pts:
                    continue
                vals = [_val(q[2], p) for q in planes]
                if all(v >= 0 for v in vals):
                    tight = frozenset(k for k, v in enumerate(vals) if v == 0)
                    if len(tight) != 3:
                        raise Degenerate("vertex on more than three planes")
                    pts[p] = tight
            if len(pts) < 4:
                if pts:
                    raise Degenerate("lower-dimensional piece")
                continue
            plist = list(pts)
            edges = []
            for u, w in itertools.combinations(plist, 2):
                sh = pts[u] & pts[w]
                if len(sh) == 2:
                    edges.append((u, w, sh))
            face_pl = {}
            for p in plist:
                for k in pts[p]:
                    face_pl.setdefault(k, []).append(p)
            apex = tuple(sum(p[k] for p in plist) / len(plist) for k in range(3))
            vol = Fr(0)
            mom = [Fr(0)] * 3
            for k, fv in face_pl.items():
                fe = [(u, w) for (u, w, sh) in edges if k in sh]
                cyc = [fv[0]]
                prev = None
                while len(cyc) < len(fv):
                    cur = cyc[-1]
                    nxt = next(o for (u, w) in fe for o in ((w,) if u == cur else (u,) if w == cur else ())
                               if o != prev)
                    prev = cur
                    cyc.append(nxt)
                for m in range(1, len(cyc) - 1):
                    a, b, c = cyc[0], cyc[m], cyc[m + 1]
                    det = _dot(_sub(b, a), _cross(_sub(c, a), _sub(apex, a)))
                    tv = abs(det) / 6
                    vol += tv
                    for d in range(3):
                        mom[d] += tv * (a[d] + b[d] + c[d] + apex[d]) / 4
            pieces[(t, i)] = dict(pts=pts, planes=planes, edges=edges, faces=face_pl, vol=vol, mom=mom)

    # ---- assembly by exact coordinates
    cells, faces, edges_el, rpv = {}, {}, {}, set()
    for i in range(n):
        Vs, Es, Fs, C = set(), set(), set(), 0
        vol = Fr(0)
        mom = [Fr(0)] * 3
        for (t, ii), pc in pieces.items():
            if ii != i:
                continue
            C += 1
            Vs |= set(pc["pts"])
            Es |= {frozenset((u, w)) for (u, w, _) in pc["edges"]}
            Fs |= {frozenset(fv) for fv in pc["faces"].values()}
            vol += pc["vol"]
            mom = [mom[d] + pc["mom"][d] for d in range(3)]
        chi = len(Vs) - len(Es) + len(Fs) - C
        b0 = _components(list(Vs), Es) if C else 0
        cells[i] = dict(chi=chi, beta0=b0, vol=vol, mom=mom)
    for (t, i), pc in pieces.items():
        pl = pc["planes"]
        for k, fv in pc["faces"].items():
            if pl[k][0] != "b":
                continue
            j = pl[k][1]
            if j < i:
                continue
            el = faces.setdefault((i, j), dict(V=set(), E=set(), F=set()))
            el["V"] |= set(fv)
            el["E"] |= {frozenset((u, w)) for (u, w, sh) in pc["edges"] if k in sh}
            el["F"].add(frozenset(fv))
        for (u, w, sh) in pc["edges"]:
            a, b = sorted(sh)
            if pl[a][0] == "b" and pl[b][0] == "b":
                j, k = sorted((pl[a][1], pl[b][1]))
                if j < i:
                    continue
                el = edges_el.setdefault((i, j, k), dict(V=set(), E=set()))
                el["V"] |= {u, w}
                el["E"].add(frozenset((u, w)))
        for p, tight in pc["pts"].items():
            if all(pl[k][0] == "b" for k in tight):
                rpv.add(tuple(sorted([i] + [pl[k][1] for k in tight])))
    face_out = {k: dict(chi=len(e["V"]) - len(e["E"]) + len(e["F"]), beta0=_components(list(e["V"]), e["E"]))
                for k, e in faces.items()}
    edge_out = {k: dict(chi=len(e["V"]) - len(e["E"]), beta0=_components(list(e["V"]), e["E"]))
                for k, e in edges_el.items()}
    return dict(cells=cells, faces=face_out, edges=edge_out, rpv=rpv, n_pairs=len(pieces),
                piece_vol={k: v["vol"] for k, v in pieces.items()})
