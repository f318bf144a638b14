"""Autotuner of the decomposition of each lattice of an ensemble run with
the persistent schedule.

The fragment edge F sets both the decomposition (part of the simulated
dynamics, so it is recorded with the results) and the cost: small F gives
many small tiles per phase, large F few tiles with long serial BKL chains.
F = 0 is the unfragmented method, plain BKL over the whole lattice, which
the library runs in LDS on one wavefront for lattices of at most 512
vacancies: one hop per step and no phases, the fastest choice for sparse
small lattices, whose fragment phases hold about one hop each.  For every
candidate the whole ensemble runs a short trial on the GPU; the kernel's
per-lattice busy timer and hop counters give the device time per hop, so
the time to reach the hop target is predicted per lattice, and each lattice
gets the candidate with the smallest prediction.  The critical path of the
ensemble is the slowest lattice, so the choice is made lattice by lattice.

The unfragmented candidate wins near ties (within PLAIN_MARGIN of the best
prediction, and still clear of the ensemble's slowest prediction): plain
BKL has no splitting error, and its cost per hop does not depend on how the
hops spread over tiles, which drifts as a lattice evolves from its initial
state (at low temperature the hops gather around the vacancies next to H
ions), while a short trial from the initial state sees only the start.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

# Per-lattice fragment edges chosen by tune() for the 512-lattice ensemble
# (seed 0xC4), stored so that runs of that ensemble simulate the same
# decomposition (the edge is part of the dynamics) without re-tuning.
ENSEMBLE_EDGES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned",
                              "ensemble_512_edges.json")

PLAIN_LDS_VACANCIES = 512
PLAIN_LDS_BYTES = 62_000
PLAIN_MARGIN = 0.05  # the unfragmented candidate wins within 5 % of the best prediction
PLAIN_CLEARANCE = 0.95  # ... when it stays below 95 % of the slowest lattice's prediction


def whole_if_sparse(spec) -> int:
    """One fragment (the whole lattice) for lattices of at most 32 cells and
    32 vacancies (the library's one-lane-block-per-vacancy path), else
    16-cell fragments."""
    return spec.L[0] if max(spec.L) <= 32 and spec.n_vac <= 32 else 16


def plain_if_sparse(spec) -> int:
    """Plain BKL (0) for lattices the library holds in LDS (at most 512
    vacancies; occupancy at 2 bits per site plus the rate cache inside one
    workgroup's share), else 16-cell fragments."""
    n = 3 * spec.L[0] * spec.L[1] * spec.L[2]
    slots = next(s for s in (64, 128, 256, 512) if spec.n_vac <= s) if spec.n_vac <= 512 else 512
    fits = (n + 15) // 16 * 4 + 4 * spec.n_vac + 9 * 8 * slots <= PLAIN_LDS_BYTES
    return 0 if spec.n_vac <= PLAIN_LDS_VACANCIES and fits else 16


DEFAULT_CANDIDATES = (4, 6, 8, 10, 12, 14, 16, 18, 20, 24, whole_if_sparse, plain_if_sparse)


def specs_digest(specs) -> str:
    """Digest of what identifies an ensemble's lattices (sizes, keys,
    compositions, temperatures, fields, windows), whatever their edges."""
    h = hashlib.sha256()
    for sp in specs:
        h.update(repr((tuple(sp.L), sp.seed, sp.lattice_id, sp.n_vac, sp.n_h, round(sp.T, 9),
                       round(sp.E_z, 3), sp.Ea_O, sp.Ea_H, float.hex(float(sp.t_sync)))).encode())
    return h.hexdigest()[:16]


def save_edges(path: str, specs, edges, report=None) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump({"lattices": len(specs), "digest": specs_digest(specs),
                   "edges": [int(e) for e in edges],
                   "histogram": {int(k): int(v) for k, v in zip(*np.unique(edges, return_counts=True))},
                   "report": report or {}}, f, indent=0)


def load_edges(path: str, specs):
    """Stored per-lattice edges for exactly these lattices, else None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("lattices") != len(specs) or d.get("digest") != specs_digest(specs):
        return None
    return np.array(d["edges"], dtype=np.int64)


def trial(specs, F, cycles: int, waves: int, plain_hops: int = 20_000):
    """Per-lattice (device ms, hops) of a short trial: `cycles` cycles for
    fragment lattices, then `plain_hops` hops for plain ones (a call with no
    cycles runs only the plain lattices)."""
    from paper_2004_09081_amd.workloads import to_gpu
    geoms, rates = to_gpu(specs, F)
    plain = np.array([sp.frag[0] == 0 for sp in specs])
    ts = [0.0 if p else sp.t_sync for p, sp in zip(plain, specs)]
    s = F.LatticeSet(geoms)
    try:
        s.init_random([sp.n_vac for sp in specs], [sp.n_h for sp in specs])
        s.set_rates(rates)
        s.set_schedule("persistent", waves)
        ms = np.zeros(len(specs))
        hops = np.zeros(len(specs))
        if not plain.all():
            s.advance(ts, max_cycles=cycles, min_hops=0)
            st = s.read_stats()
            ms[~plain] = np.array([x["busy_ms"] for x in st])[~plain]
            hops[~plain] = np.array([int(x["hops"][0]) + int(x["hops"][1]) for x in st])[~plain]
        if plain.any():
            s.advance(ts, max_cycles=0, min_hops=plain_hops)
            st = s.read_stats()
            ms[plain] = np.array([x["busy_ms"] for x in st])[plain]
            hops[plain] = np.array([int(x["hops"][0]) + int(x["hops"][1]) for x in st])[plain]
    finally:
        s.close()
    return ms, hops


def tune(make_specs, hop_target: int, candidates=DEFAULT_CANDIDATES, cycles: int = 128,
         waves: int = 4, log=None, repeats: int = 1):
    """make_specs(frag) -> list of LatticeSpec with fragment edge `frag`
    (cells).  A candidate is an edge, or a function of a lattice's spec
    giving its edge.  Each candidate's trial runs `repeats` times and a
    lattice's prediction is the median, which steadies the choice against
    timing noise.  Returns (per-lattice edge, report); the edge is the one
    the lattice ran with in its best trial."""
    from paper_2004_09081_amd import fkmc as F
    base = make_specs(8)
    n = len(base)
    best_t = np.full(n, np.inf)
    best_f = np.full(n, 8, dtype=np.int64)
    plain_t = np.full(n, np.inf)
    report = {}
    for c in candidates:
        label = c.__name__ if callable(c) else str(c)
        if callable(c):
            specs = make_specs(8)
            for sp in specs:
                sp.frag = (int(c(sp)),) * 3
        else:
            specs = make_specs(c)
        used = np.array([sp.frag[0] for sp in specs], dtype=np.int64)
        try:
            preds = []
            for _ in range(max(1, repeats)):
                ms, hops = trial(specs, F, cycles, waves)
                preds.append(ms * hop_target / np.maximum(hops, 1e-9))
        except F.FkmcError as e:
            report[label] = "infeasible: %s" % e
            if log:
                log("autotune F=%s: infeasible (%s)" % (label, e))
            continue
        pred = np.median(np.array(preds), axis=0)
        better = pred < best_t
        best_t[better] = pred[better]
        best_f[better] = used[better]
        plain_t = np.where(used == 0, np.minimum(plain_t, pred), plain_t)
        report[label] = {"max_pred_ms": float(pred.max()), "median_pred_ms": float(np.median(pred))}
        if log:
            log("autotune F=%s: slowest lattice predicted %.0f ms" % (label, pred.max()))
    near = (best_f != 0) & (plain_t <= best_t * (1.0 + PLAIN_MARGIN)) & \
        (plain_t <= PLAIN_CLEARANCE * best_t.max())
    best_f[near] = 0
    best_t[near] = plain_t[near]
    report["plain_near_ties"] = int(near.sum())
    if log:
        log("autotune: %d lattices take the unfragmented candidate on a near tie" % int(near.sum()))
    report["chosen_max_pred_ms"] = float(best_t.max())
    report["histogram"] = {int(k): int(v) for k, v in zip(*np.unique(best_f, return_counts=True))}
    return best_f, report
