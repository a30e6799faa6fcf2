"""TEST INFRASTRUCTURE -- the sphere-insertion loop of topology repair, run on the CPU oracle.

Only the test-suite and the scripts that write stored expected values may import this module; it never imports the
product package.

The paper repairs topology by inserting spheres where a restricted element is not contractible and recomputing the
RPD (Sec. 4 overview; Sec. 4.1.3 places the new sphere). The placement used here is the deterministic table rule of
the library's table-insertion mode, so that the site sequence is a function of the exact combinatorics alone:

1. the whole RPD of the current sites, by the brute-force oracle (``oracle.rpd``);
2. the violating cells: nonempty, with chi != 1 or more than one component, the first ``max_insert`` in ascending
   site order;
3. for each such cell i, the candidate tets are those of its pieces whose table sphere is not in yet; for a cell with
   several components only the pieces outside the component of its piece in its smallest tet; the pick is the
   candidate t with the largest pair (h(t, round), t), h = the upper 32 bits of the splitmix64 finaliser of
   t * 2^32 + round (rounds counted from 0), and no pick when there is no candidate;
4. the picks are inserted in the order of the selected cells: cell k appends table[t_k] unless an earlier cell of
   the round picked the same tet, the sphere is in already, or the capacity ``max_sites`` is reached.
"""
from __future__ import annotations

import numpy as np

M64 = (1 << 64) - 1


def splitmix64_hi(x: int) -> int:
    """Upper 32 bits of the splitmix64 output function (Steele, Lea and Flood, 2014) applied to x + the golden-ratio
    increment."""
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return (z ^ (z >> 31)) >> 32


def select_and_pick(r: dict, used: np.ndarray, rnd: int, max_insert: int) -> list:
    """Steps 2 and 3 on one oracle result: the picked tet of every selected cell (None: no candidate)."""
    chi, b0, npc = r["cell_chi"], r["cell_beta0"], r["cell_npieces"]
    viol = np.nonzero((npc > 0) & ((chi != 1) | (b0 > 1)))[0][:max_insert]
    cp = r["cell_piece"]  # (t, i, component label), ordered by (i, t)
    picks = []
    for i in viol:
        lo, hi = np.searchsorted(cp[:, 1], [i, i + 1])
        ts, lab = cp[lo:hi, 0], cp[lo:hi, 2]
        ok = ~used[ts]
        if b0[i] > 1:
            ok &= lab != lab[np.argmin(ts)]
        best = None
        for t in ts[ok]:
            key = (splitmix64_hi((int(t) << 32) | rnd), int(t))
            if best is None or key > best:
                best = key
        picks.append(None if best is None or best == (0, 0) else best[1])
    return picks


def insert(picks: list, used: np.ndarray, table, sites: list, max_sites: int) -> int:
    """Step 4: appends the picked table spheres to ``sites`` (four lists x, y, z, r); returns how many."""
    added = 0
    for k, t in enumerate(picks):
        if t is None or t in picks[:k] or used[t]:
            continue
        if len(sites[0]) >= max_sites:
            break
        for c in range(4):
            sites[c].append(table[c][t])
        used[t] = True
        added += 1
    return added


def repair_loop(prob, table, rounds: int, max_insert: int, max_sites: int, threads: int = 0, log=None):
    """Runs ``rounds`` rounds from the sites of ``prob``; returns (final sites as float32 [n, 4], per-round counts of
    (selected cells, inserted spheres)) and the oracle result of the final site set."""
    import oracle

    sites = [list(np.asarray(a, np.float32)) for a in (prob.sx, prob.sy, prob.sz, prob.sr)]
    tab = [np.asarray(a, np.float32) for a in table]
    used = np.zeros(prob.n_tets, bool)
    history = []

    def current():
        a = [np.asarray(c, np.float32) for c in sites]
        return prob.with_sites(*a)

    for rnd in range(rounds):
        r = oracle.rpd(current(), threads=threads, assemble=False)
        if not r["consistent"]:
            raise RuntimeError(f"oracle inconsistency in round {rnd}: {r['report']}")
        picks = select_and_pick(r, used, rnd, max_insert)
        added = insert(picks, used, tab, sites, max_sites)
        history.append((len(picks), added))
        if log:
            log(f"round {rnd}: {len(picks)} violating cells selected, {added} spheres inserted, "
                f"{len(sites[0])} sites")
    final = oracle.rpd(current(), threads=threads, assemble=False)
    if not final["consistent"]:
        raise RuntimeError(f"oracle inconsistency after the last round: {final['report']}")
    return np.stack([np.asarray(c, np.float32) for c in sites], axis=1), history, final
