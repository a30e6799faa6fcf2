"""Writes ``piece_stats.json`` beside this script: the algorithmic work per nonempty piece of the benchmark workloads,
from the oracle's piece statistics (calls only ``oracle`` and ``paper_2403_18761_amd.synth``).

For a nonempty piece P_{t,i} with v vertices and f faces on bisector planes, the clipping method must evaluate each
bounding bisector at the piece's vertices (8 v f FLOP), construct every vertex once (about 30 v) and integrate the
volume and first moment over the face fans (about 25 v). The file stores, per workload, the mean of 8 v f + 55 v over
the pieces of the sampled tets (every tet of the torus workload), with the means of v and f beside it; the benchmark
multiplies it by the number of nonempty pieces of a build to get the build's algorithmic FLOPs.

Usage: ``python tests/golden/piece_stats.py [--threads N]``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "piece_stats.json")
SAMPLE_TETS = 150000  # tets sampled per workload when it has more (the torus is taken whole)


def flop_per_piece(v: np.ndarray, f: np.ndarray) -> np.ndarray:
    return 8.0 * v * f + 55.0 * v


def stats_of(probs, threads: int, seed: int) -> dict:
    import oracle

    rng = np.random.default_rng(seed)
    total = sum(p.n_tets for p in probs)
    frac = min(1.0, SAMPLE_TETS / total)
    vs, fs, tets = [], [], 0
    t0 = time.perf_counter()
    for p in probs:
        m = max(1, int(round(frac * p.n_tets)))
        sel = np.arange(p.n_tets) if m >= p.n_tets else np.sort(rng.choice(p.n_tets, m, replace=False))
        r = oracle.tet_pieces(p, sel, threads=threads)
        vs.extend(q["nverts"] for q in r["pieces"])
        fs.extend(len(q["face_terms"]) for q in r["pieces"])
        tets += len(sel)
    v, f = np.asarray(vs, np.float64), np.asarray(fs, np.float64)
    return dict(tets_sampled=tets, tets_total=total, pieces=len(v), mean_vertices=float(v.mean()),
                mean_bisector_faces=float(f.mean()), flop_per_piece=float(flop_per_piece(v, f).mean()),
                seconds=round(time.perf_counter() - t0, 1))


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    from paper_2403_18761_amd import synth

    out = {"formula": "mean over nonempty pieces of 8 v f + 55 v (v vertices, f faces on bisector planes)"}
    work = {
        "torus2000": lambda: [synth.torus_inside(N=64, n_sites=2000, seed=2)],
        "genus3": lambda: [synth.genus3_cad(N=128, n_sites=20000, seed=3)],
        "batch256": lambda: synth.batch_problems(256, 4),
    }
    for name, make in work.items():
        out[name] = stats_of(make(), args.threads, seed=7)
        print(name, out[name], flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
