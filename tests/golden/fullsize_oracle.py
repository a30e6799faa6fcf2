"""Writes the oracle's results for the full-size workloads into small digest files beside this script.

Calls only ``oracle`` (the CPU brute-force oracle) and ``paper_2403_18761_amd.synth`` (seeded inputs, no arithmetic of
the method); nothing here touches the HIP path. The whole oracle runs once per workload on the CPU (about one to a few
hours for the genus-3 solid and the 256-shape batch on 8 threads), and the GPU tests compare their own results with
the stored digests element list by element list.

What is stored per shape (``fullsize_<workload>.json``):

* ``input_sha256``: digest of the exact input arrays (the test regenerates the input and checks it first);
* ``n_pairs``, ``L`` and the element counts;
* ``sha256`` of every exact per-element array, in the byte layout ``digest_arrays`` defines: cell chi and beta0 (one
  entry per site), face keys/chi/beta0, edge keys/chi/beta0 (sorted by key), RPV keys;
* sums of chi and beta0 per kind (a mismatch then says which kind differs and by how much);
* the total cell volume and the volumes of 64 cells picked by a fixed seed (float64, for the 1e-5 check).

``repair50`` runs the oracle's own insertion loop (``oracle.repair``) for 50 rounds of at most 64 insertions on the
repair workload (975,462 tets, 500 initial sites, the per-tet sphere table) and stores the digest of the final site
array (float32 [n, 4]), the per-round counts and the record of the final RPD.

Usage: ``python tests/golden/fullsize_oracle.py torus2000|genus3|batch256|repair50 [--threads N]``. The batch file
is written after every shape, and a rerun resumes after the last stored shape of the same input.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

EXACT = ("cell_chi", "cell_beta0", "face_keys", "face_chi", "face_beta0", "edge_keys", "edge_chi", "edge_beta0",
         "rpv_keys")
N_VOL_SAMPLES = 64


def input_digest(prob) -> str:
    h = hashlib.sha256()
    for a, dt in ((prob.vx, np.float32), (prob.vy, np.float32), (prob.vz, np.float32), (prob.tv, np.int32),
                  (prob.sx, np.float32), (prob.sy, np.float32), (prob.sz, np.float32), (prob.sr, np.float32)):
        h.update(np.ascontiguousarray(a, dtype=dt).tobytes())
    return h.hexdigest()


def digest_arrays(res: dict) -> dict:
    """sha256 of each exact array as little-endian int32, row-major (the same layout on the GPU side)."""
    return {k: hashlib.sha256(np.ascontiguousarray(res[k], dtype="<i4").tobytes()).hexdigest() for k in EXACT}


def summary(res: dict) -> dict:
    return dict(
        n_cells_nonempty=int(np.count_nonzero(res["cell_vol"] > 0)),
        n_faces=int(len(res["face_keys"])), n_edges=int(len(res["edge_keys"])), n_rpv=int(len(res["rpv_keys"])),
        sum_cell_chi=int(np.sum(res["cell_chi"], dtype=np.int64)),
        sum_cell_beta0=int(np.sum(res["cell_beta0"], dtype=np.int64)),
        sum_face_chi=int(np.sum(res["face_chi"], dtype=np.int64)),
        sum_face_beta0=int(np.sum(res["face_beta0"], dtype=np.int64)),
        sum_edge_chi=int(np.sum(res["edge_chi"], dtype=np.int64)),
        sum_edge_beta0=int(np.sum(res["edge_beta0"], dtype=np.int64)),
    )


def volume_samples(n_sites: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_sites, min(N_VOL_SAMPLES, n_sites), replace=False))


def shape_record(prob, threads: int, seed: int) -> dict:
    import oracle

    t0 = time.perf_counter()
    r = oracle.rpd(prob, threads=threads, assemble=False)
    dt = time.perf_counter() - t0
    return record_of(prob, r, threads, seed, dt)


def record_of(prob, r: dict, threads: int, seed: int, dt: float) -> dict:
    if not r["consistent"]:
        raise RuntimeError(f"oracle reports an inconsistency: {r['report']}")
    pick = volume_samples(prob.n_sites, seed)
    return dict(
        input_sha256=input_digest(prob), n_tets=prob.n_tets, n_sites=prob.n_sites, L=r["L"],
        n_pairs=r["n_pairs"], sha256=digest_arrays(r), **summary(r),
        volume_total=float(np.sum(r["cell_vol"])), volume_sample_seed=seed,
        volume_sample_sites=[int(x) for x in pick], volume_sample=[float(r["cell_vol"][x]) for x in pick],
        oracle_seconds=round(dt, 1), oracle_threads=threads,
    )


def workload_problems(name: str):
    from paper_2403_18761_amd import synth

    if name == "torus2000":
        return [synth.torus_inside(N=64, n_sites=2000, seed=2)]
    if name == "genus3":
        return [synth.genus3_cad(N=128, n_sites=20000, seed=3)]
    if name == "batch256":
        return None  # generated shape by shape (see main)
    raise SystemExit(f"unknown workload {name}")


def path_for(name: str) -> str:
    return os.path.join(HERE, f"fullsize_{name}.json")


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=("torus2000", "genus3", "batch256", "repair50"))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    import oracle

    oracle.build(force=False)
    out = path_for(args.workload)
    if args.workload == "repair50":
        repair50(out, args.threads)
        return
    if args.workload != "batch256":
        prob = workload_problems(args.workload)[0]
        rec = shape_record(prob, args.threads, seed=11)
        with open(out, "w") as fh:
            json.dump({"workload": args.workload, "shapes": [rec]}, fh, indent=1)
        print(args.workload, "done in", rec["oracle_seconds"], "s", flush=True)
        return
    from paper_2403_18761_amd import synth

    tets, sites = synth.batch_sizes(256, 4)
    done = []
    partial = out + ".partial"  # shapes so far; renamed to the final name once all are in
    for path in (out, partial):
        if os.path.exists(path):
            with open(path) as fh:
                done = json.load(fh)["shapes"]
            break
    for k in range(len(done), 256):
        prob = synth.batch_shape(k, int(tets[k]), int(sites[k]))
        rec = shape_record(prob, args.threads, seed=1000 + k)
        rec["shape"] = k
        done.append(rec)
        tmp = out + ".tmp"
        with open(tmp, "w") as fh:
            json.dump({"workload": args.workload, "shapes": done}, fh, indent=1)
        os.replace(tmp, out if len(done) == 256 else partial)
        print(f"batch shape {k}: {prob.n_tets} tets, {prob.n_sites} sites, {rec['oracle_seconds']} s", flush=True)


REPAIR_ROUNDS, REPAIR_MAX_INSERT = 50, 64


def repair50(out: str, threads: int) -> None:
    from oracle import repair
    from paper_2403_18761_amd import synth

    prob, table = synth.repair_problem(N=128, n_sites=500, seed=5)
    max_sites = prob.n_sites + REPAIR_MAX_INSERT * REPAIR_ROUNDS
    t0 = time.perf_counter()
    sites, history, final = repair.repair_loop(prob, table, REPAIR_ROUNDS, REPAIR_MAX_INSERT, max_sites,
                                               threads=threads, log=lambda m: print(m, flush=True))
    dt = time.perf_counter() - t0
    fin = prob.with_sites(sites[:, 0], sites[:, 1], sites[:, 2], sites[:, 3])
    tab = np.stack([np.asarray(a, np.float32) for a in table], axis=1)
    rec = dict(workload="repair50", rounds=REPAIR_ROUNDS, max_insert=REPAIR_MAX_INSERT, max_sites=max_sites,
               initial_input_sha256=input_digest(prob),
               table_sha256=hashlib.sha256(np.ascontiguousarray(tab).tobytes()).hexdigest(),
               n_sites_final=int(sites.shape[0]),
               sites_sha256=hashlib.sha256(np.ascontiguousarray(sites, dtype="<f4").tobytes()).hexdigest(),
               history=[list(h) for h in history], loop_seconds=round(dt, 1),
               shapes=[record_of(fin, final, threads, 13, dt)])
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("repair50 done in", round(dt, 1), "s", flush=True)


if __name__ == "__main__":
    main()
