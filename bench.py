"""Throughput benchmark of the fragment kMC hot path on one MI355X.

Default workload: the batched ensemble (512 independent lattices, cube edge
16-64 cells, T 300-900 K, H fraction 0-0.3, vacancy fraction 1e-3..1e-2,
field 0-1e7 V/m, 1e6 hops per lattice), all lattices advancing in one
persistent launch per call.  One STEP = every lattice advances by its hop
target (1e6 hops) from the state left by the previous step; the inputs are
resident in HBM before the timed region.

Printed: one JSON line with whole-job hops/s; the roofline of the dominant
kernel of the timed region (HIP events around its launches); the fragment
sweep's roofline on the 600^3 biased lattice (lockstep phase kernel, HIP
events); the plain (unfragmented) kMC path and the fragment path run one
lattice per launch on a sample of the same lattices; the paper's
atom-selection scheme with null events on the lattices held in LDS, against
BKL on the same lattices; the surrogate report; and the CPU oracle's rate on
a bounded sample.

Other workloads (--workload): cfg3 (600^3 biased lattice), cfg2 (48^3, five
temperatures as one set).
"""
from __future__ import annotations

import argparse
import copy
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "hops/s on 1 MI355X, batched fragment vs plain kMC; surrogate log10 D MAE"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of one hop, what the method itself must move: the 9
# occupancy bytes around the moved vacancy read (its site and 8 neighbours),
# 2 written, and the int32x3 displacements of the two particles that swap
# read and written (2 x 12 B each way).
ALG_HOP_BYTES = 9 + 2 + 2 * 2 * 12
# Bytes a hop moves in this implementation's records: two occupancy bytes
# written, and the int32x4 displacement records of both particles read and
# written.
IMPL_HOP_BYTES = 2 + 4 * 16
# Sources (kernels and their launch set-up) whose change invalidates stored
# HBM traffic counts.
# The counter traffic belongs to these sources: the kernels, the host plan,
# and the autotuner that picks each ensemble lattice's decomposition.
KERNEL_SOURCES = ("paper_2004_09081_amd/csrc/fkmc_device.hip",
                  "paper_2004_09081_amd/csrc/fkmc_internal.h",
                  "paper_2004_09081_amd/csrc/fkmc_api.hip",
                  "paper_2004_09081_amd/autotune.py")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.md")
PLAIN_MAX_VACANCIES = 8192


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the counter summary, or None when there is
    none for this kernel and workload or the kernel sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    pat = re.compile(r"^traffic: kernel=(\S+) workload=(\S+) source=(\S+) bytes_per_launch=(\d+)")
    src = kernel_source_hash()
    with open(TRAFFIC_FILE) as f:
        for line in f:
            m = pat.match(line.strip())
            if m and m.group(1) == kernel and m.group(2) == workload and m.group(3) == src:
                return int(m.group(4))
    return None


def fragment_sizes(L: int, F: int):
    if F >= L:
        return [L]
    nf, r = L // F, L % F
    sizes = [F] * nf
    if r >= 2:
        sizes.append(r)
    elif r == 1:
        sizes[-1] += 1
    return sizes


def footprint_bytes(spec) -> int:
    """Occupancy bytes one cycle's 8 phases read: every sub-block once plus
    its three +faces (the footprint of each tile).  Plain lattices have no
    cycles (0)."""
    if spec.frag[0] == 0:
        return 0
    ws = []
    for a in range(3):
        w = []
        for s in fragment_sizes(spec.L[a], spec.frag[a]):
            w += [(s + 1) // 2, s // 2]
        ws.append(w)
    tot = 0
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


def hops_of(stats) -> np.ndarray:
    return np.array([int(st["hops"][0]) + int(st["hops"][1]) for st in stats], dtype=np.int64)


def roofline_obj(kernel, hops_per_launch, staging_per_launch, avg_ms, launches, workload, note):
    """Roofline of one kernel.  achieved/frac: the method's algorithmic bytes
    (ALG_HOP_BYTES per hop) per launch over the mean launch time.  The
    staging figures count what this design moves on purpose besides: each
    streamed lattice's footprints once per phase (HBM -> LDS), a resident
    lattice's occupancy in and out once per launch, and the displacement
    records of its hops."""
    sec = avg_ms * 1e-3
    alg = hops_per_launch * ALG_HOP_BYTES
    achieved = alg / sec / 1e9 if avg_ms > 0 else 0.0
    stg = staging_per_launch + hops_per_launch * IMPL_HOP_BYTES
    st_gbs = stg / sec / 1e9 if avg_ms > 0 else 0.0
    traffic = stored_traffic(kernel, workload)
    return {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic,
            "kernel": kernel, "avg_launch_ms": avg_ms, "launches_timed": launches,
            "hops_per_launch": float(hops_per_launch),
            "algorithmic_bytes_per_hop": ALG_HOP_BYTES,
            "algorithmic_bytes_per_launch": int(alg),
            "staging": {"bytes_per_launch": int(stg), "achieved": round(st_gbs, 3),
                        "frac": round(st_gbs / HBM_PEAK_GBS, 6)},
            "traffic_frac": (round(traffic / sec / 1e9 / HBM_PEAK_GBS, 6)
                             if traffic and avg_ms > 0 else None),
            "note": note}


def _oracle_lattice(sp):
    from oracle import oracle as O
    g = O.Geometry(L=sp.L, frag=sp.frag, a_angstrom=sp.a, seed=sp.seed, lattice_id=sp.lattice_id,
                   gb_period_cells=sp.gb_period, gb_axes_mask=sp.gb_mask)
    lat = O.Lattice(g)
    lat.init_random(sp.n_vac, sp.n_h)
    lat.set_rates(O.RateParams(T=sp.T, Ea_O=sp.Ea_O, Ea_H=sp.Ea_H, E_z=sp.E_z, q=sp.q,
                               gb_period_cells=sp.gb_period, gb_axes_mask=sp.gb_mask,
                               gb_dE=sp.gb_dE))
    return lat


def _oracle_run(sp, hop_target: int, budget_s: float):
    """The oracle, unchanged, on one lattice in the decomposition the GPU
    ran (plain BKL for edge 0, else fragment cycles), until the hop target
    or the time budget: (hops, seconds, finished)."""
    lat = _oracle_lattice(sp)
    h = 0
    t0 = time.perf_counter()
    while h < hop_target:
        if sp.frag[0] == 0:
            lat.advance_plain(min(20_000, hop_target - h))
        else:
            lat.advance(sp.t_sync, max_cycles=1)
        h = int(lat.hops.sum())
        if time.perf_counter() - t0 > budget_s:
            return h, time.perf_counter() - t0, False
    return h, time.perf_counter() - t0, True


def _oracle_worker(args):
    sp, hop_target, budget_s = args
    return _oracle_run(sp, hop_target, budget_s)


def cpu_model() -> str:
    """The host CPU's model name and its online and usable CPU counts."""
    name = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    if not name:
        import platform
        name = platform.processor() or "unknown"
    return "%s (%d CPUs online, %d usable by this process)" % (name, os.cpu_count() or 0,
                                                               len(os.sched_getaffinity(0)))


def cpu_baseline(specs, budget_s: float, hop_target: int, workers: int):
    """The oracle as it stands on the workload's first lattices: on one host
    thread, lattice after lattice until the budget runs out; then on
    `workers` processes at once, one lattice each (independent lattices, so
    the all-core rate is the sum of the per-process rates)."""
    import multiprocessing as mp
    done, used, n_lat, partial = 0, 0.0, 0, False
    for sp in specs:
        h, t, fin = _oracle_run(sp, hop_target, budget_s - used)
        done += h
        used += t
        n_lat += 1
        if not fin or used >= budget_s:
            partial = not fin
            break
    one = {"value": done / used, "hops": done, "seconds": used, "lattices": n_lat, "partial": partial}
    jobs = [(sp, hop_target, budget_s) for sp in specs[:workers]]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(len(jobs)) as pool:
        res = pool.map(_oracle_worker, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    allc = {"value": float(sum(h / t for h, t, _ in res)), "processes": len(jobs),
            "hops": int(sum(h for h, _, _ in res)), "wall_s": wall,
            "finished": int(sum(1 for _, _, f in res if f)),
            "per_process": [float(h / t) if t > 0 else 0.0 for h, t, _ in res]}
    return one, allc


def cpu_leg(args):
    """The cpu_baseline record of the workload bench.py times, from the
    oracle on the host's cores (cfg4: the stored autotuner decomposition when
    it matches, else 8-cell fragments)."""
    from paper_2004_09081_amd import workloads as W
    if args.workload == "cfg4":
        from paper_2004_09081_amd import autotune
        specs = W.cfg4(n=args.lattices, hops=args.hops, frag=8)
        edges = autotune.load_edges(autotune.ENSEMBLE_EDGES, specs)
        if edges is not None and args.frag in ("auto", "tune"):
            for sp, e in zip(specs, edges):
                sp.frag = (int(e),) * 3
        elif args.frag not in ("auto", "tune"):
            specs = W.cfg4(n=args.lattices, hops=args.hops,
                           frag=(lambda L: (L + 1) // 2) if args.frag == "half" else int(args.frag))
        hop_target = args.hops
    elif args.workload == "cfg3":
        specs, hop_target = [W.cfg3()], 10**18
    else:
        specs, hop_target = [W.cfg2(T) for T in W.CFG2_TEMPERATURES], 10_000_000
    workers = max(1, min(args.cpu_workers, len(os.sched_getaffinity(0))))
    one, allc = cpu_baseline(specs, args.cpu_budget, hop_target, workers)
    model = cpu_model()
    log("cpu oracle (%s): %.4g hops/s on 1 thread, %.4g hops/s on %d processes"
        % (model, one["value"], allc["value"], allc["processes"]))
    return {"value": one["value"], "unit": "hops/s", "cores": 1, "kind": "oracle", "cpu": model,
            "sample": "first %d lattice(s) of the workload in the decomposition the GPU runs (plain "
                      "BKL for unfragmented ones), %d hops in %.1f s on one thread%s"
                      % (one["lattices"], one["hops"], one["seconds"],
                         " (last one partial)" if one["partial"] else ""),
            "all_cores": {"value": allc["value"], "unit": "hops/s", "cores": allc["processes"],
                          "per_lattice": allc["per_process"],
                          "sample": "first %d lattices, one process each, up to %.0f s each (%d "
                                    "reached the hop target); rate = sum of per-process rates; "
                                    "per_lattice: each process's rate in lattice order (cfg2: one "
                                    "per temperature, 300-800 K)"
                                    % (allc["processes"], args.cpu_budget, allc["finished"])}}


def micro_run(F, W):
    """The reduced micro-scale BaTiO3 model (Voronoi grains with a +0.2 eV
    boundary layer, the paper's bias, 0.1 % vacancies, 450 K) run for 5 ms
    of simulated time: hops/s, and where the vacancies gather (on boundary
    sites against the boundary-site fraction; the densest 5^3-cell block
    against the mean)."""
    import torch
    t0 = time.perf_counter()
    spec, gmap = W.micro()
    t_map = time.perf_counter() - t0
    S = build_set([spec], F)
    S.set_gb_map(0, gmap)
    S.set_schedule("lockstep")
    cycles = int(math.ceil(spec.extra["t_end"] / spec.t_sync))
    torch.cuda.synchronize()
    a = time.perf_counter()
    S.advance([spec.t_sync], max_cycles=cycles, min_hops=0)
    torch.cuda.synchronize()
    el = time.perf_counter() - a
    st = S.read_stats()[0]
    occ, _ = S.read_state(0, with_disp=False)
    S.close()
    hops = int(st["hops"].sum())
    v = occ == 2
    L = spec.L
    cellv = v.reshape(L[2], L[1], L[0], 3).sum(axis=3)
    b = 5
    blocks = cellv[:L[2] // b * b, :L[1] // b * b, :L[0] // b * b].reshape(
        L[2] // b, b, L[1] // b, b, L[0] // b, b).sum(axis=(1, 3, 5))
    rep = {"hops": hops, "seconds": el, "hops_per_s": hops / el, "t_simulated_s": st["t"],
           "cycles": int(st["cycles"]), "vacancies": int(v.sum()),
           "boundary_site_fraction": float(gmap.mean()),
           "vacancies_on_boundary_sites": float(gmap[v].mean()),
           "densest_block_over_mean": float(blocks.max() / blocks.mean()),
           "drift_V_m_per_s": [float(x) * 1e-10 for x in st["drift"][2]],
           "map_seconds": t_map,
           "workload": "%dx%dx%d cells, %d Voronoi grains, boundary layer %.1f cell +%.1f eV, E_z %.3g V/m, "
                       "0.1%% V, %.0f K, %d^3 fragments, %.0e s" % (L[0], L[1], L[2], spec.extra["n_grains"],
                                                                  spec.extra["width"], spec.gb_dE, spec.E_z,
                                                                  spec.T, spec.frag[0], spec.extra["t_end"])}
    log("micro model: %d hops in %.2f s (%.3g hops/s) to t = %.3g s; vacancies on boundary sites %.3f "
        "(site fraction %.3f), densest 5^3 block %.1f x the mean" % (
            hops, el, rep["hops_per_s"], st["t"], rep["vacancies_on_boundary_sites"],
            rep["boundary_site_fraction"], rep["densest_block_over_mean"]))
    return rep


def sweep_leg(F, W, cycles: int, warm: int):
    """Lockstep fragment sweep of the 600^3 biased lattice: HIP-event time of
    every phase launch over `cycles` whole cycles after `warm` cycles."""
    import torch
    spec = W.cfg3()
    t0 = time.perf_counter()
    S = build_set([spec], F)
    S.set_schedule("lockstep")
    torch.cuda.synchronize()
    log("sweep leg: 600^3 set up in %.2f s" % (time.perf_counter() - t0))
    if warm:
        S.advance([spec.t_sync], max_cycles=warm, min_hops=0)
    h0 = int(hops_of(S.read_stats()).sum())
    S.set_timing(True)
    S.advance([spec.t_sync], max_cycles=cycles, min_hops=0)
    avg_ms, launches = S.phase_timing()
    S.set_timing(False)
    hops = int(hops_of(S.read_stats()).sum()) - h0
    S.close()
    del S
    torch.cuda.empty_cache()
    fp = footprint_bytes(spec)
    rf = roofline_obj("k_phase", hops / launches, fp / 8.0, avg_ms, launches, "cfg3",
                      "fragment sweep, one colour of every fragment per launch; staging = that "
                      "colour's footprints (sub-block plus three +faces) read HBM->LDS, written back")
    rf["hops_per_s"] = hops / (launches * avg_ms * 1e-3) if avg_ms > 0 else 0.0
    rf["workload"] = ("600^3 cells (6.48e8 sites), 0.1%% V, 450 K, E_z 1e7 V/m, GB z-planes every "
                      "50 cells +0.3 eV, 16^3-cell fragments, %d cycles" % cycles)
    log("sweep: k_phase %.4f ms avg over %d launches, %.0f hops/launch -> %.1f GB/s algorithmic "
        "(%.3f%% of peak), staging %.1f GB/s (%.2f%%), %.4g hops/s"
        % (avg_ms, launches, hops / launches, rf["achieved"], 100 * rf["frac"],
           rf["staging"]["achieved"], 100 * rf["staging"]["frac"], rf["hops_per_s"]))
    return rf


def one_per_launch(F, specs, idx, hop_target):
    """Each sampled lattice alone in its own set (its kernels carry one
    lattice per launch), advanced by hop_target hops."""
    import torch
    ph, pt = 0, 0.0
    for i in idx:
        s1 = build_set([specs[i]], F)
        torch.cuda.synchronize()
        a = time.perf_counter()
        s1.advance([specs[i].t_sync], max_cycles=10**9, min_hops=hop_target)
        torch.cuda.synchronize()
        pt += time.perf_counter() - a
        ph += int(hops_of(s1.read_stats()).sum())
        s1.close()
    return ph, pt


def atomic_leg(F, specs, n_frg, stages, replicas=1):
    """The paper's atom-selection scheme with null events (Eqs. AtomP and
    TimeStepFrg) on every ensemble lattice that fits in LDS unfragmented,
    all in one launch, against BKL on the same lattices from the same
    initial states: hops/s of both, and the ratio of the vacancy tracer D
    for n_frg selections per stage (the paper's parallel approximation) and
    for one (an exact kMC, so its ratio checks the estimator).  With
    replicas > 1 every such lattice runs that many times with its own
    random streams (lattice ids 512 apart), which narrows the D ratios."""
    import torch
    from paper_2004_09081_amd.autotune import plain_if_sparse
    sel = []
    for r in range(replicas):
        for sp in specs:
            if plain_if_sparse(sp) == 0:
                q = copy.copy(sp)
                q.frag = (0, 0, 0)
                q.t_sync = 0.0
                q.lattice_id = sp.lattice_id + 512 * r
                sel.append(q)
    n = len(sel)

    def run(fn):
        s = build_set(sel, F)
        try:
            torch.cuda.synchronize()
            a = time.perf_counter()
            fn(s)
            torch.cuda.synchronize()
            return time.perf_counter() - a, s.read_stats()
        finally:
            s.close()

    t_at, st_a = run(lambda s: s.advance_atomic(n_frg, stages))
    t_1, st_1 = run(lambda s: s.advance_atomic(1, stages))
    hops_a, hops_1 = hops_of(st_a), hops_of(st_1)

    def d_ratio(st):
        """Vacancy tracer D against BKL run to the same simulated time on
        each lattice (MSD/6t carries a short-time offset from local
        flicker, so equal times matter): the ratio of the summed estimates
        (a mean of per-lattice ratios of two noisy estimates is biased
        upwards), its error by the paired delta method."""
        horizon = [x["t"] for x in st]
        cap = 10 * int(hops_of(st).max()) + 100_000  # the horizon ends each run well before this
        tb, sb = run(lambda s: s.advance(horizon, 0, cap))
        assert all(y["t"] == h for y, h in zip(sb, horizon))
        da = np.array([x["D"][2] for x in st])
        db = np.array([y["D"][2] for y in sb])
        r = float(da.sum() / db.sum())
        return ({"value": r, "stderr": float(np.std(da - r * db, ddof=1) / np.sqrt(n) / db.mean())},
                float(hops_of(sb).sum() / tb))

    ra, bkl_rate = d_ratio(st_a)
    r1, _ = d_ratio(st_1)
    target = int(hops_a.mean())
    rep = {"value": float(hops_a.sum() / t_at), "unit": "hops/s", "lattices": n, "n_frg": n_frg,
           "stages": stages, "hops_per_stage": float(hops_a.sum() / (n * stages)),
           "kernel_ms": max(x["busy_ms"] for x in st_a),
           "bkl_same_lattices": {"value": bkl_rate, "unit": "hops/s",
                                 "mean_hops_per_lattice": target},
           "D_vacancy_ratio_to_bkl": ra,
           "one_selection": {"value": float(hops_1.sum() / t_1), "unit": "hops/s",
                             "hops_per_stage": float(hops_1.sum() / (n * stages)),
                             "D_vacancy_ratio_to_bkl": r1},
           "estimator": "D ratio = sum over lattices of D_V / the same sum for BKL run to the same "
                        "simulated time on each lattice",
           "sample": "%d of %d ensemble lattices (those held in LDS unfragmented) x %d replica(s), %d stages "
                     "of %d selections (and of 1), each against BKL to the same times"
                     % (n // replicas, len(specs), replicas, stages, n_frg)}
    log("atom selection (N_frg %d): %.4g hops/s on %d lattices, %.2f hops per stage, D_V ratio to BKL "
        "%.4f +- %.4f; N_frg 1: %.4g hops/s, D_V ratio %.4f +- %.4f; BKL on the same lattices %.4g hops/s"
        % (n_frg, rep["value"], n, rep["hops_per_stage"], ra["value"], ra["stderr"],
           rep["one_selection"]["value"], r1["value"], r1["stderr"], rep["bkl_same_lattices"]["value"]))
    return rep


def atomic_hbm_leg(F, specs, n_frg, stages):
    """The atom-selection scheme on the ensemble lattices of at most 8192
    vacancies that the persistent kernel does not hold in LDS (more than
    512 vacancies, or an occupancy too large for its LDS share), all in one
    call, against plain BKL making the same mean number of hops from the
    same initial states.  Those that fit the LDS atom-selection kernel's
    own limit run there, the rest keep their occupancy in HBM."""
    import torch
    from paper_2004_09081_amd.autotune import plain_if_sparse
    sel = []
    for sp in specs:
        if plain_if_sparse(sp) != 0 and sp.n_vac <= PLAIN_MAX_VACANCIES:
            q = copy.copy(sp)
            q.frag = (0, 0, 0)
            q.t_sync = 0.0
            sel.append(q)
    if not sel:
        return None

    def run(fn):
        s = build_set(sel, F)
        try:
            torch.cuda.synchronize()
            a = time.perf_counter()
            fn(s)
            torch.cuda.synchronize()
            return time.perf_counter() - a, s.read_stats()
        finally:
            s.close()

    t_at, st_a = run(lambda s: s.advance_atomic(n_frg, stages))
    hops_a = hops_of(st_a)
    target = int(hops_a.mean())
    t_b, st_b = run(lambda s: s.advance([0.0] * len(sel), 0, target))
    hops_b = hops_of(st_b)
    rep = {"value": float(hops_a.sum() / t_at), "unit": "hops/s", "lattices": len(sel), "n_frg": n_frg,
           "stages": stages, "hops_per_stage": float(hops_a.sum() / (len(sel) * stages)),
           "kernel_ms": max(x["busy_ms"] for x in st_a),
           "us_per_stage": 1e3 * max(x["busy_ms"] for x in st_a) / stages,
           "bkl_same_lattices": {"value": float(hops_b.sum() / t_b), "unit": "hops/s",
                                 "hops_per_lattice": target},
           "sample": "%d of %d ensemble lattices (at most 8192 vacancies, not held in LDS by the "
                     "persistent kernel; unfragmented), %d stages of %d selections; BKL the same mean "
                     "hop count" % (len(sel), len(specs), stages, n_frg)}
    log("atom selection on lattices past the persistent kernel's LDS (N_frg %d): %.4g hops/s on %d lattices, %.2f hops per stage, "
        "%.1f us per stage; BKL on the same lattices %.4g hops/s"
        % (n_frg, rep["value"], len(sel), rep["hops_per_stage"], rep["us_per_stage"],
           rep["bkl_same_lattices"]["value"]))
    return rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg4", choices=["cfg4", "cfg3", "cfg2", "micro"])
    ap.add_argument("--lattices", type=int, default=512, help="cfg4 ensemble size")
    ap.add_argument("--hops", type=int, default=1_000_000, help="cfg4 hops per lattice per step")
    ap.add_argument("--plain-sample", type=int, default=16,
                    help="lattices run one per launch for the comparison legs (0: skip)")
    ap.add_argument("--plain-hops", type=int, default=20_000,
                    help="hops per lattice of the unfragmented one-per-launch leg")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="processes of the all-core oracle leg (capped by the host's CPUs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep-cycles", type=int, default=4,
                    help="timed cycles of the 600^3 sweep leg (0: skip)")
    ap.add_argument("--frag", default="auto",
                    help="cfg4 fragment edge: cells, 'half' (ceil(L/2)), 'auto' (the stored autotuner "
                         "edges when they match the ensemble, else tuned now) or 'tune' (tuned now)")
    ap.add_argument("--tune-repeats", type=int, default=1,
                    help="autotuner trials per candidate (median per lattice)")
    ap.add_argument("--save-edges", default="", help="write the tuned per-lattice edges here")
    ap.add_argument("--waves", type=int, default=0, help="waves per workgroup of the persistent kernel")
    ap.add_argument("--atomic-stages", type=int, default=20000,
                    help="stages of the atom-selection leg (0: skip)")
    ap.add_argument("--atomic-frg", type=int, default=64, help="selections per stage of that leg")
    ap.add_argument("--atomic-replicas", type=int, default=1,
                    help="runs of each of that leg's lattices with their own random streams")
    ap.add_argument("--atomic-hbm-stages", type=int, default=2000,
                    help="stages of the atom-selection leg on lattices past the LDS kernel (0: skip)")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-train", type=int, default=4096)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (reference for the "
                         "HBM byte counters) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the method would shard by lattice or by z-slab; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    # The CPU oracle leg runs first, before this process touches the GPU, so
    # that its worker processes start from a process without GPU state.
    cpu_rep = None
    if not args.no_cpu_baseline and not args.calibrate_copy_mib and args.workload != "micro":
        cpu_rep = cpu_leg(args)

    import torch
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib << 20
        x = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copied_bytes": n}))
        return

    from paper_2004_09081_amd import fkmc as F
    from paper_2004_09081_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    F.lib()

    if args.workload == "micro":
        rep = micro_run(F, W)
        print(json.dumps({"metric": METRIC, "value": rep["hops_per_s"], "unit": "hops/s", "n_gpus": 1,
                          "steps": 1, "warmup": 0, "ms_per_step": rep["seconds"] * 1e3,
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic", "config": {"workload": rep["workload"]}, "micro": rep}),
              flush=True)
        return

    decomposition = None
    if args.workload == "cfg4":
        hop_target = args.hops
        if args.frag in ("auto", "tune"):
            from paper_2004_09081_amd import autotune
            specs = W.cfg4(n=args.lattices, hops=args.hops, frag=8)
            best = autotune.load_edges(autotune.ENSEMBLE_EDGES, specs) if args.frag == "auto" else None
            if best is not None:
                decomposition = "autotuner edges stored with the package (digest %s)" % autotune.specs_digest(specs)
                log("decomposition: stored autotuner edges %s" % dict(zip(*[x.tolist() for x in np.unique(best, return_counts=True)])))
            else:
                t_tune = time.perf_counter()
                best, tune_report = autotune.tune(lambda fr: W.cfg4(n=args.lattices, hops=args.hops, frag=fr),
                                                  hop_target, waves=args.waves or 4, log=log,
                                                  repeats=args.tune_repeats)
                log("autotune %.1f s: %s" % (time.perf_counter() - t_tune, tune_report["histogram"]))
                decomposition = "autotuned in this run (%d trial(s) per candidate)" % args.tune_repeats
                if args.save_edges:
                    autotune.save_edges(args.save_edges, specs, best, tune_report)
                    log("edges saved to %s" % args.save_edges)
            for i, sp in enumerate(specs):
                sp.frag = (int(best[i]),) * 3
        else:
            fr = (lambda L: (L + 1) // 2) if args.frag == "half" else int(args.frag)
            specs = W.cfg4(n=args.lattices, hops=args.hops, frag=fr)
        desc = ("cfg4 batched ensemble: %d lattices, cube edge 16-64 cells, T 300-900 K, "
                "x_H 0-0.3, x_V 1e-3..1e-2 log-uniform, E_z 0-1e7 V/m, fragment edge %s cells "
                "(0 = unfragmented BKL held in LDS), %d hops per lattice per step"
                % (len(specs), args.frag, hop_target))
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
    # plain lattices (fragment edge 0) take no horizon: exactly hop_target hops
    ts = [0.0 if s.frag[0] == 0 else s.t_sync for s in specs]

    def step():
        if args.workload == "cfg3":
            S.advance(ts, max_cycles=4, min_hops=0)
        else:
            S.advance(ts, max_cycles=10**9, min_hops=hop_target)

    for w in range(args.warmup):
        t0 = time.perf_counter()
        step()
        log("warmup %d: %.2f s" % (w, time.perf_counter() - t0))
    st0 = S.read_stats()
    h_before = hops_of(st0)
    c_before = np.array([st["cycles"] for st in st0], dtype=np.int64)
    # HIP events around every kernel launch of the timed steps (persistent
    # schedule: one launch per step; lockstep: one per phase).
    S.set_timing(True)
    ev_ms, ev_n = 0.0, 0
    step_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        a, n = S.phase_timing()
        ev_ms += a * n
        ev_n += n
        step_ms.append(round(a * n, 2))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log("timed steps, device ms each: %s" % step_ms)
    S.set_timing(False)
    stats = S.read_stats()
    hops_each = hops_of(stats) - h_before
    cyc_each = np.array([st["cycles"] for st in stats], dtype=np.int64) - c_before
    hops = int(hops_each.sum())
    elapsed = t1 - t0
    value = hops / elapsed
    log("timed: %d hops in %.3f s -> %.4g hops/s" % (hops, elapsed, value))
    avg_ms = ev_ms / ev_n if ev_n else 0.0
    res = np.array([st["lds_resident"] for st in stats], dtype=bool)
    fp = np.array([footprint_bytes(sp) for sp in specs], dtype=np.float64)
    sites = np.array([sp.n_sites for sp in specs], dtype=np.float64)
    if args.workload == "cfg4":
        busy = np.array([st["busy_ms"] for st in stats])
        fr = np.array([sp.frag[0] for sp in specs])
        for f in np.unique(fr):
            m = fr == f
            j = int(np.argmax(np.where(m, busy, -1.0)))
            log("  edge %d: %d lattices, busiest %d at %.1f ms (%.3f us/hop)" % (
                f, int(m.sum()), j, busy[j], 1e3 * busy[j] * args.steps / max(int(hops_each[j]), 1)))
        for i in np.argsort(-busy)[:8]:
            sp = specs[i]
            log("  lattice %d: busy %.1f ms, L=%d F=%d n_V=%d n_H=%d T=%.0f cycles=%d resident=%d" % (
                i, busy[i], sp.L[0], sp.frag[0], sp.n_vac, sp.n_h, sp.T, stats[i]["cycles"],
                stats[i]["lds_resident"]))
        # A lattice held in LDS moves its occupancy HBM->LDS->HBM once per
        # launch; any other lattice reads its footprints every cycle.
        sweep_b = float(np.where(res, 2.0 * sites * args.steps, cyc_each * fp).sum())
        roofline = roofline_obj(
            "k_batch", hops / max(ev_n, 1), sweep_b / max(ev_n, 1), avg_ms, ev_n, "cfg4",
            "persistent kernel, one workgroup per lattice; the launch lasts as long as the "
            "slowest lattice's serial BKL chain, so it is latency-bound, not HBM-bound: "
            "%d of %d lattices held in LDS" % (int(res.sum()), len(specs)))
    else:
        roofline = roofline_obj("k_phase", hops / max(ev_n, 1), float((cyc_each * fp).sum()) / max(ev_n, 1),
                                avg_ms, ev_n, args.workload,
                                "lockstep phase kernel, one colour of every fragment per launch")
    log("%s: %.4f ms avg over %d launches, %.4g hops/launch -> %.3f GB/s algorithmic, %.3f GB/s staging" % (
        roofline["kernel"], avg_ms, ev_n, roofline["hops_per_launch"], roofline["achieved"],
        roofline["staging"]["achieved"]))

    out = {"metric": METRIC, "value": value, "unit": "hops/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded Philox placement, parameters drawn from the workload recipe)",
           "config": {"workload": desc, "lattices": len(specs),
                      "fragment_edges": ({int(k): int(v) for k, v in zip(*np.unique([sp.frag[0] for sp in specs], return_counts=True))}),
                      "sites": int(sum(s.n_sites for s in specs)),
                      "decomposition": decomposition,
                      "hops_timed": hops},
           "step_device_ms": step_ms,
           "roofline": roofline}
    S.close()
    del S
    torch.cuda.empty_cache()

    if args.workload == "cfg4" and args.sweep_cycles > 0:
        out["roofline_sweep"] = sweep_leg(F, W, args.sweep_cycles, warm=1)

    if args.workload == "cfg4" and args.plain_sample > 0:
        idx = np.linspace(0, len(specs) - 1, args.plain_sample).astype(int)
        # plain (unfragmented) BKL, one lattice per launch; its kernel holds at
        # most PLAIN_MAX_VACANCIES vacancy slots
        pidx = [i for i in idx if specs[i].n_vac <= PLAIN_MAX_VACANCIES]
        plain_specs = []
        for sp in specs:
            q = copy.copy(sp)
            q.frag = (0, 0, 0)
            q.t_sync = 0.0  # plain mode: no time horizon, stop at the hop count
            plain_specs.append(q)
        ph, pt = one_per_launch(F, plain_specs, pidx, args.plain_hops)
        plain_rate = ph / pt
        out["plain_one_per_launch"] = {
            "value": plain_rate, "unit": "hops/s",
            "sample": "%d of %d lattices, unfragmented BKL, one lattice per launch, %d hops each"
                      % (len(pidx), len(specs), args.plain_hops),
            "batched_over_plain": value / plain_rate}
        log("plain kMC one-per-launch: %.4g hops/s (batched/plain = %.1f)" % (plain_rate, value / plain_rate))
        # the same fragment decomposition, one lattice per launch
        fh, ft = one_per_launch(F, specs, idx, hop_target)
        frag_rate = fh / ft
        out["fragment_one_per_launch"] = {
            "value": frag_rate, "unit": "hops/s",
            "sample": "%d of %d lattices, same fragments, one lattice per launch, %d hops each"
                      % (len(idx), len(specs), hop_target),
            "batched_over_one_per_launch": value / frag_rate}
        log("fragment kMC one-per-launch: %.4g hops/s (batched/one = %.1f)" % (frag_rate, value / frag_rate))

    if args.workload == "cfg4" and args.atomic_stages > 0:
        out["atom_selection"] = atomic_leg(F, specs, args.atomic_frg, args.atomic_stages, args.atomic_replicas)
        if args.atomic_hbm_stages > 0:
            out["atom_selection_hbm"] = atomic_hbm_leg(F, specs, args.atomic_frg, args.atomic_hbm_stages)

    if args.workload == "cfg4" and not args.no_surrogate:
        from paper_2004_09081_amd import surrogate
        rep = surrogate.run_cfg5(n_train=args.surrogate_train, n_test=512, log=log)
        out["surrogate"] = rep
        log("surrogate: MAE %.4f decades on served points, served %.2f, kMC-only %.2f s vs "
            "surrogate+fallback %.2f s" % (rep["mae_log10D"], rep["served_fraction"],
                                           rep["time_kmc_only_s"], rep["time_surrogate_with_fallback_s"]))

    if cpu_rep is not None:
        out["cpu_baseline"] = cpu_rep
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
