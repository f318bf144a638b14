"""Autotuner of the fragment edge for an ensemble run with the persistent
schedule.

The fragment edge F sets both the decomposition (part of the simulated
dynamics, so it is recorded with the results) and the cost: small F gives
many small tiles per phase, large F few tiles with long serial BKL chains.
For every candidate F the whole ensemble runs a short trial on the GPU; the
kernel's per-lattice busy timer gives the device time per cycle and the hop
counters the hops per cycle, so the time to reach the hop target is
predicted per lattice, and each lattice gets the candidate with the smallest
prediction.  The critical path of the ensemble is the slowest lattice, so
the choice is made lattice by lattice.
"""
from __future__ import annotations

import numpy as np

def whole_if_sparse(spec) -> int:
    """One fragment (the whole lattice) for lattices of at most 32 cells and
    32 vacancies (the library's one-lane-block-per-vacancy path), else
    16-cell fragments."""
    return spec.L[0] if max(spec.L) <= 32 and spec.n_vac <= 32 else 16


DEFAULT_CANDIDATES = (4, 6, 8, 12, 16, 24, whole_if_sparse)


def trial(specs, F, ts, cycles: int, waves: int):
    """Per-lattice (ms per cycle, hops per cycle) for one fragment choice."""
    from paper_2004_09081_amd.workloads import to_gpu
    geoms, rates = to_gpu(specs, F)
    s = F.LatticeSet(geoms)
    try:
        s.init_random([sp.n_vac for sp in specs], [sp.n_h for sp in specs])
        s.set_rates(rates)
        s.set_schedule("persistent", waves)
        s.advance(ts, max_cycles=cycles, min_hops=0)
        st = s.read_stats()
    finally:
        s.close()
    ms = np.array([x["busy_ms"] for x in st]) / cycles
    hops = np.array([int(x["hops"][0]) + int(x["hops"][1]) for x in st], dtype=np.float64) / cycles
    return ms, hops


def tune(make_specs, hop_target: int, candidates=DEFAULT_CANDIDATES, cycles: int = 64,
         waves: int = 4, log=None):
    """make_specs(frag) -> list of LatticeSpec with fragment edge `frag`
    (cells).  A candidate is an edge, or a function of a lattice's spec
    giving its edge.  Returns (per-lattice edge, report); the edge is the
    one the lattice ran with in its best trial."""
    from paper_2004_09081_amd import fkmc as F
    base = make_specs(8)
    n = len(base)
    best_t = np.full(n, np.inf)
    best_f = np.full(n, 8, dtype=np.int64)
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
        ts = [sp.t_sync for sp in specs]
        try:
            ms, hpc = trial(specs, F, ts, cycles, waves)
        except F.FkmcError as e:
            report[label] = "infeasible: %s" % e
            if log:
                log("autotune F=%s: infeasible (%s)" % (label, e))
            continue
        pred = ms * hop_target / np.maximum(hpc, 1e-9)
        better = pred < best_t
        best_t[better] = pred[better]
        best_f[better] = used[better]
        report[label] = {"max_pred_ms": float(pred.max()), "median_pred_ms": float(np.median(pred))}
        if log:
            log("autotune F=%s: slowest lattice predicted %.0f ms" % (label, pred.max()))
    report["chosen_max_pred_ms"] = float(best_t.max())
    report["histogram"] = {int(k): int(v) for k, v in zip(*np.unique(best_f, return_counts=True))}
    return best_f, report
