"""Throughput benchmark of the fragment kMC hot path on one MI355X.

Default workload: the batched ensemble (512 independent lattices, cube edge
16-64 cells, T 300-900 K, H fraction 0-0.3, vacancy fraction 1e-3..1e-2,
field 0-1e7 V/m, 1e6 hops per lattice), all lattices advancing together in
one launch per phase.  One STEP = every lattice advances by its hop target
(1e6 hops) from the state left by the previous step; the inputs are resident
in HBM before the timed region.  Printed: one JSON line with whole-job hops/s,
the phase kernel's roofline figures (HIP-event timing), the one-lattice-per-
launch rate on a sample of the same lattices, and the CPU oracle's rate on a
bounded sample.

Other workloads (--workload): cfg3 (600^3 biased lattice, HBM-bound sweep),
cfg2 (48^3, five temperatures as one set).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "hops/s on 1 MI355X, batched fragment vs plain kMC; surrogate log10 D MAE"
HBM_PEAK_GBS = 8000.0
HOP_BYTES = 2 + 4 * 16  # two occupancy bytes written, two int32x4 displacements read+written


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def footprint_bytes(spec) -> int:
    """Bytes one cycle's 8 phases read: every sub-block once plus its three
    +faces (the footprint of each tile)."""
    tot = 0
    ws = []
    for a in range(3):
        L, F = spec.L[a], spec.frag[a]
        if F >= L:
            sizes = [L]
        else:
            nf, r = L // F, L % F
            sizes = [F] * nf
            if r >= 2:
                sizes.append(r)
            elif r == 1:
                sizes[-1] += 1
        w = []
        for s in sizes:
            w += [(s + 1) // 2, s // 2]
        ws.append(w)
    for x in ws[0]:
        for y in ws[1]:
            for z in ws[2]:
                tot += 3 * x * y * z + y * z + z * x + x * y
    return tot


def build_set(specs, F):
    from paper_2004_09081_amd.workloads import to_gpu
    geoms, rates = to_gpu(specs, F)
    s = F.LatticeSet(geoms)
    s.init_random([sp.n_vac for sp in specs], [sp.n_h for sp in specs])
    s.set_rates(rates)
    return s


def total_hops(stats) -> int:
    return int(sum(int(st["hops"][0]) + int(st["hops"][1]) for st in stats))


def cpu_baseline(specs, budget_s: float, hop_target: int):
    """The oracle, unchanged, on the first lattices of the workload (one
    host thread), cycle by cycle until each reaches its hop target or the
    time budget runs out."""
    from oracle import oracle as O
    done_hops = 0
    t_used = 0.0
    n_lat = 0
    partial = False
    for sp in specs:
        g = O.Geometry(L=sp.L, frag=sp.frag, a_angstrom=sp.a, seed=sp.seed,
                       lattice_id=sp.lattice_id, gb_period_cells=sp.gb_period,
                       gb_axes_mask=sp.gb_mask)
        lat = O.Lattice(g)
        lat.init_random(sp.n_vac, sp.n_h)
        lat.set_rates(O.RateParams(T=sp.T, Ea_O=sp.Ea_O, Ea_H=sp.Ea_H, E_z=sp.E_z, q=sp.q,
                                   gb_period_cells=sp.gb_period, gb_axes_mask=sp.gb_mask,
                                   gb_dE=sp.gb_dE))
        n_lat += 1
        h0 = 0
        t0 = time.perf_counter()
        while h0 < hop_target:
            lat.advance(sp.t_sync, max_cycles=1)
            h0 = int(lat.hops.sum())
            if t_used + time.perf_counter() - t0 > budget_s:
                partial = True
                break
        t_used += time.perf_counter() - t0
        done_hops += h0
        if t_used > budget_s:
            break
    return done_hops, t_used, n_lat, partial


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg4", choices=["cfg4", "cfg3", "cfg2"])
    ap.add_argument("--lattices", type=int, default=512, help="cfg4 ensemble size")
    ap.add_argument("--hops", type=int, default=1_000_000, help="cfg4 hops per lattice per step")
    ap.add_argument("--plain-sample", type=int, default=16)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--roofline-cycles", type=int, default=16)
    ap.add_argument("--frag", default="auto",
                    help="cfg4 fragment edge: cells, 'half' (ceil(L/2)) or 'auto' (autotuned per lattice)")
    ap.add_argument("--waves", type=int, default=0, help="waves per workgroup of the persistent kernel")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-train", type=int, default=4096)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (reference for the "
                         "HBM byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib << 20
        x = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copied_bytes": n}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the method would shard by lattice or by z-slab; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2004_09081_amd import fkmc as F
    from paper_2004_09081_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    F.lib()

    if args.workload == "cfg4":
        hop_target = args.hops
        tune_report = None
        if args.frag == "auto":
            from paper_2004_09081_amd import autotune
            t_tune = time.perf_counter()
            best, tune_report = autotune.tune(lambda fr: W.cfg4(n=args.lattices, hops=args.hops, frag=fr),
                                              hop_target, waves=args.waves or 4, log=log)
            per = {i: int(best[i]) for i in range(len(best))}
            specs = W.cfg4(n=args.lattices, hops=args.hops, frag=8)
            for i, sp in enumerate(specs):
                sp.frag = (per[i],) * 3
            log("autotune %.1f s: %s" % (time.perf_counter() - t_tune, tune_report["histogram"]))
        else:
            fr = (lambda L: (L + 1) // 2) if args.frag == "half" else int(args.frag)
            specs = W.cfg4(n=args.lattices, hops=args.hops, frag=fr)
        desc = ("cfg4 batched ensemble: %d lattices, cube edge 16-64 cells, T 300-900 K, "
                "x_H 0-0.3, x_V 1e-3..1e-2 log-uniform, E_z 0-1e7 V/m, fragment edge %s cells, "
                "%d hops per lattice per step" % (len(specs), args.frag, hop_target))
    elif args.workload == "cfg3":
        specs = [W.cfg3()]
        hop_target = 0
        desc = ("cfg3 600^3 cells (6.48e8 sites), 0.1%% V, 450 K, E_z 1e7 V/m, GB planes every "
                "50 cells +0.3 eV, 16^3-cell fragments, step = 4 cycles")
    else:
        specs = [W.cfg2(T) for T in W.CFG2_TEMPERATURES]
        hop_target = 10_000_000
        desc = "cfg2 48^3 cells, 12^3 fragments, x_H 0.10, x_V 0.005, T 300..800 K as one set, 1e7 hops each"

    t_setup = time.perf_counter()
    S = build_set(specs, F)
    if args.waves or args.workload == "cfg4":
        S.set_schedule("auto", args.waves or 4)
    torch.cuda.synchronize()
    log("setup %.2f s (%d lattices, %d sites)" % (time.perf_counter() - t_setup, len(specs),
                                                    sum(s.n_sites for s in specs)))
    ts = [s.t_sync for s in specs]

    def step():
        if args.workload == "cfg3":
            S.advance(ts, max_cycles=4, min_hops=0)
        else:
            S.advance(ts, max_cycles=10**9, min_hops=hop_target)

    for w in range(args.warmup):
        t0 = time.perf_counter()
        step()
        log("warmup %d: %.2f s" % (w, time.perf_counter() - t0))
    h_before = total_hops(S.read_stats())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = S.read_stats()
    hops = total_hops(stats) - h_before
    elapsed = t1 - t0
    value = hops / elapsed
    log("timed: %d hops in %.3f s -> %.4g hops/s" % (hops, elapsed, value))
    if args.workload == "cfg4":
        busy = np.array([st["busy_ms"] for st in stats])
        for i in np.argsort(-busy)[:8]:
            sp = specs[i]
            log("  lattice %d: busy %.1f ms, L=%d F=%d n_V=%d n_H=%d T=%.0f cycles=%d" % (
                i, busy[i], sp.L[0], sp.frag[0], sp.n_vac, sp.n_h, sp.T, stats[i]["cycles"]))

    # Roofline of the phase kernel: HIP-event timing of every phase launch
    # over a window of whole cycles in which every lattice is active.
    S.set_timing(True)
    h0 = total_hops(S.read_stats())
    S.advance(ts, max_cycles=args.roofline_cycles, min_hops=0)
    h1 = total_hops(S.read_stats())
    avg_ms, launches = S.phase_timing()
    S.set_timing(False)
    cyc = args.roofline_cycles
    fp = sum(footprint_bytes(s) for s in specs)
    bytes_per_launch = fp / 8.0 + (h1 - h0) * HOP_BYTES / (8.0 * cyc)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "kernel": "k_phase", "avg_launch_ms": avg_ms, "launches_timed": launches,
                "algorithmic_bytes_per_launch": bytes_per_launch}
    log("phase kernel: %.4f ms avg over %d launches, %.0f B/launch -> %.1f GB/s" %
        (avg_ms, launches, bytes_per_launch, achieved))

    out = {"metric": METRIC, "value": value, "unit": "hops/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded Philox placement, parameters drawn from the workload recipe)",
           "config": {"workload": desc, "lattices": len(specs),
                      "fragment_edges": ({int(k): int(v) for k, v in zip(*np.unique([sp.frag[0] for sp in specs], return_counts=True))}),
                      "sites": int(sum(s.n_sites for s in specs)),
                      "hops_timed": hops},
           "roofline": roofline}

    # one-lattice-per-launch path on a sample of the same lattices
    if args.workload == "cfg4" and args.plain_sample > 0:
        idx = np.linspace(0, len(specs) - 1, args.plain_sample).astype(int)
        ph, pt = 0, 0.0
        for i in idx:
            s1 = build_set([specs[i]], F)
            torch.cuda.synchronize()
            a = time.perf_counter()
            s1.advance([specs[i].t_sync], max_cycles=10**9, min_hops=hop_target)
            torch.cuda.synchronize()
            pt += time.perf_counter() - a
            ph += total_hops(s1.read_stats())
            s1.close()
        plain_rate = ph / pt
        out["one_lattice_per_launch"] = {"value": plain_rate, "unit": "hops/s",
                                         "sample": "%d of %d lattices, run one at a time" % (len(idx), len(specs)),
                                         "batched_over_plain": value / plain_rate}
        log("one-lattice-per-launch: %.4g hops/s (batched/plain = %.1f)" % (plain_rate, value / plain_rate))

    if args.workload == "cfg4" and not args.no_surrogate:
        from paper_2004_09081_amd import surrogate
        rep = surrogate.run_cfg5(n_train=args.surrogate_train, n_test=512, log=log)
        out["surrogate"] = rep
        log("surrogate: MAE %.4f decades on served points, served %.2f, kMC-only %.2f s vs "
            "surrogate+fallback %.2f s" % (rep["mae_log10D"], rep["served_fraction"],
                                           rep["time_kmc_only_s"], rep["time_surrogate_with_fallback_s"]))

    if not args.no_cpu_baseline:
        hops_c, tc, nl, partial = cpu_baseline(specs, args.cpu_budget, hop_target or 10**18)
        out["cpu_baseline"] = {"value": hops_c / tc, "unit": "hops/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "first %d lattice(s) of the workload, %d hops in %.1f s%s"
                                         % (nl, hops_c, tc, " (last one partial)" if partial else "")}
        log("cpu oracle: %.4g hops/s" % (hops_c / tc))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
