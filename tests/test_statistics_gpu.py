"""Statistical pins run through the HIP path: fragment kMC against the
unfragmented (plain) BKL it approximates, over 32 seeds (the paper's
accuracy criterion: the fragmentation changes D by less than its
statistical error)."""
import math

import numpy as np
import pytest

from tests.common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_09081_amd import fkmc
    return fkmc


def _run(F, frag, seeds, L, nv, nh, rp, t_end, t_sync):
    geoms = [F.Geometry.make(L, frag, 3.905, s, 7) for s in seeds]
    S = F.LatticeSet(geoms)
    S.init_random([nv] * len(seeds), [nh] * len(seeds))
    S.set_rates([F.RateParams.make(**rp)] * len(seeds))
    if frag[0] == 0:
        S.advance([t_end] * len(seeds), 0, 10**12)           # plain: stop at the horizon
    else:
        S.advance([t_sync] * len(seeds), max_cycles=int(round(t_end / t_sync)))
    st = S.read_stats()
    S.close()
    return np.array([x["D"] for x in st]), np.array([x["hops"] for x in st], dtype=float), st


def test_fragment_matches_unfragmented_within_3_sigma(F):
    say("fragment vs plain, 32 seeds")
    L, nv, nh = (12, 12, 12), 26, 518
    rp = dict(T=650.0, Ea_O=0.55, Ea_H=0.45)
    kB = 1.380649e-23 / 1.602176634e-19
    kO = 1e13 * math.exp(-0.55 / (kB * 650.0))
    kH = 1e13 * math.exp(-0.45 / (kB * 650.0))
    gamma = 8 * (0.1 * kH + 0.9 * kO)          # vacancy hop rate
    t_sync = 0.25 / gamma                      # about 0.25 hops per vacancy per cycle
    t_end = 1600 * t_sync
    seeds = list(range(32))
    Df, hf, sf = _run(F, (6, 6, 6), seeds, L, nv, nh, rp, t_end, t_sync)
    Dp, hp, sp = _run(F, (0, 0, 0), seeds, L, nv, nh, rp, t_end, t_sync)
    assert all(abs(x["t"] - t_end) <= 1e-12 * t_end for x in sf + sp)
    for X, name in ((2, "V"), (1, "H"), (0, "O")):
        a, b = Df[:, X], Dp[:, X]
        se = math.sqrt(a.var(ddof=1) / len(a) + b.var(ddof=1) / len(b))
        diff = a.mean() - b.mean()
        say("  D_%s frag %.4g plain %.4g diff/sigma %.2f" % (name, a.mean(), b.mean(), diff / se))
        assert abs(diff) < 3 * se, (name, a.mean(), b.mean(), se)
        assert se < 0.05 * b.mean(), (name, se / b.mean())
    assert hf.sum() > 2e5 and hp.sum() > 2e5


def test_cfg2_fragments_match_unfragmented_at_every_temperature(F):
    """The 48^3 lattice in 12^3-cell fragments (x_H 0.10, x_V 0.005, O 0.70
    eV, H 0.25 eV, t_sync 1e-9 s) at 300, 400, 500, 600 and 800 K, 32 seeds
    each, at least 1e7 hops per lattice; the unfragmented BKL reference
    starts from the same initial lattice and runs to the same simulated
    time (the paper's accuracy criterion, Sec. "Accuracy and parallel
    efficiency of the fragment kMC method", Table TABLE01).

    At 300, 400 and 500 K, D_V and D_H (and D_O at 500 K, where O hops
    number in the thousands) agree within 3 sigma of their difference over
    the 32 seeds.  At 600 and 800 K a window of 1e-9 s holds about 20 and
    200 hops per vacancy, and the edge-coloured splitting biases D (by 1-2 %
    at 600 K, 2-12 % at 800 K; the values are printed).  The bias shrinks
    with the window (1e-9/4, 1e-9/32 and 1e-9/128 s), and every D agrees with
    the unfragmented run within 3 sigma from 1e-9/32 s at 600 K and at
    1e-9/128 s at 800 K."""
    import copy
    from paper_2004_09081_amd import workloads as W
    seeds = list(range(32))
    n = len(seeds)
    temps = W.CFG2_TEMPERATURES
    hot = [600.0, 800.0]
    divs = [4, 32, 128]
    exact_from = {600.0: 32, 800.0: 128}   # windows from which 3 sigma must hold

    def build(specs):
        geoms, rates = W.to_gpu(specs, F)
        S = F.LatticeSet(geoms)
        S.init_random([sp.n_vac for sp in specs], [sp.n_h for sp in specs])
        S.set_rates(rates)
        return S

    def unfragmented(specs):
        out = []
        for sp in specs:
            q = copy.copy(sp)
            q.frag = (0, 0, 0)
            out.append(q)
        return out

    say("cfg2: %d fragment lattices to 1e7 hops each, window 1e-9 s" % (n * len(temps)))
    frag = [W.cfg2(T, seed=s) for T in temps for s in seeds]
    S = build(frag)
    S.set_schedule("persistent", 4)
    S.advance([sp.t_sync for sp in frag], max_cycles=10**9, min_hops=10_000_000)
    sf = S.read_stats()
    S.close()
    # shorter windows at 600 and 800 K, to the same simulated time for all seeds
    short, t_short = {}, []
    for T in hot:
        k = temps.index(T)
        cyc = int(np.median([x["cycles"] for x in sf[k * n:(k + 1) * n]]))
        for dv in divs:
            specs = [W.cfg2(T, seed=s) for s in seeds]
            for sp in specs:
                sp.t_sync = 1e-9 / dv
            say("cfg2 %.0f K: %d fragment lattices, window 1e-9/%d s, %d cycles" % (T, n, dv, cyc * dv))
            S = build(specs)
            S.set_schedule("persistent", 4)
            S.advance([sp.t_sync for sp in specs], max_cycles=cyc * dv, min_hops=0)
            short[(T, dv)] = S.read_stats()
            S.close()
            t_short += [x["t"] for x in short[(T, dv)]]
    base = [W.cfg2(T, seed=s) for T in temps for s in seeds]
    extra = [W.cfg2(T, seed=s) for T in hot for _ in divs for s in seeds]
    plain = unfragmented(base + extra)
    t_end = [x["t"] for x in sf] + t_short
    say("cfg2: %d unfragmented lattices to the same times" % len(plain))
    S = build(plain)
    S.advance(t_end, 0, 10**12)
    sp_all = S.read_stats()
    S.close()
    assert all(y["t"] == t for y, t in zip(sp_all, t_end))
    ref = {T: sp_all[k * n:(k + 1) * n] for k, T in enumerate(temps)}
    off = n * len(temps)
    ref_short = {}
    for T in hot:
        for dv in divs:
            ref_short[(T, dv)] = sp_all[off:off + n]
            off += n

    def compare(a, b, species, label):
        line = label
        out = {}
        for X, name in species:
            Df = np.array([x["D"][X] for x in a])
            Dp = np.array([x["D"][X] for x in b])
            se = math.sqrt(Df.var(ddof=1) / n + Dp.var(ddof=1) / n)
            diff = Df.mean() - Dp.mean()
            out[name] = (diff / se, diff / Dp.mean())
            line += "; D_%s %.5g vs %.5g A^2/us (%+.2f sigma, %+.2f %%)" % (
                name, 1e-6 * Df.mean(), 1e-6 * Dp.mean(), diff / se, 100 * diff / Dp.mean())
        say(line)
        return out

    bad = []
    for k, T in enumerate(temps):
        a, b = sf[k * n:(k + 1) * n], ref[T]
        hf = np.array([int(x["hops"].sum()) for x in a])
        assert (hf >= 10_000_000).all()
        o_hops = min(int(x["hops"][0]) for x in a + b)
        rate_f = hf.sum() / (1e-3 * max(x["busy_ms"] for x in a))
        rate_p = sum(int(x["hops"].sum()) for x in b) / (1e-3 * max(x["busy_ms"] for x in b)) \
            if b[0]["busy_ms"] > 0 else 0.0
        species = [(2, "V"), (1, "H")] + ([(0, "O")] if T >= 500 else [])
        res = compare(a, b, species, "  T %3.0f K, window 1e-9 s: cycles %d, hops %.4g, O hops >= %d, "
                      "%.3g hops/s (unfragmented %.3g)" % (T, a[0]["cycles"], hf.mean(), o_hops, rate_f, rate_p))
        if T >= 500 and o_hops <= 1000:
            bad.append((T, "O hops", o_hops))
        if T not in hot:
            bad += [(T, nm, sg) for nm, (sg, _) in res.items() if not abs(sg) < 3]
        else:
            prev = res
            for dv in divs:
                r = compare(short[(T, dv)], ref_short[(T, dv)], species,
                            "  T %3.0f K, window 1e-9/%d s" % (T, dv))
                for nm, (sg, rel) in r.items():
                    # the bias shrinks with the window, and is gone at 1/32
                    if abs(prev[nm][1]) > 0.02 and not abs(rel) < abs(prev[nm][1]):
                        bad.append((T, dv, nm, "bias did not shrink", rel, prev[nm][1]))
                    if dv >= exact_from[T] and not abs(sg) < 3:
                        bad.append((T, dv, nm, sg))
                prev = r
    assert not bad, bad


def test_fragment_site_energies_match_unfragmented_within_3_sigma(F):
    """The accuracy criterion on the site model (Table TABLEadd01 energies,
    vacancy-Fe and vacancy-vacancy): 24^3 cells, 0.2 % vacancies and Fe, 1000
    K, 32 seeds; fragment kMC in 12^3 and 8^3-cell fragments (6- and 4-cell
    sub-blocks, window about one hop per vacancy) against plain BKL with the
    same energies, all from the same initial lattices to the same simulated
    time: D_V agrees within 3 sigma of the difference."""
    from paper_2004_09081_amd import workloads as W
    L, T, xv, xfe, R = (24, 24, 24), 1000.0, 0.002, 0.002, 32
    nv, _ = W.counts(3 * 24**3, xv, 0.0)
    k0 = 1e13 * math.exp(-0.6 / (8.617333262e-5 * T))
    t_sync = 1.0 / (8 * k0)
    n_cyc = 300
    t_end = n_cyc * t_sync
    rp = F.RateParams.make(T=T, Ea_O=0.6)
    sets = {}
    for frag in (0, 12, 8):
        geoms = [F.Geometry.make(L, (frag,) * 3, 3.905, s, 0) for s in range(R)]
        S = F.LatticeSet(geoms)
        S.init_random([nv] * R, [0] * R)
        S.set_rates([rp] * R)
        for s in range(R):
            S.set_site_model(s, W.fe_map(L, xfe, s), W.SITE_E_FE_MEV, W.SITE_E_VV_MEV, 1200)
        if frag == 0:
            S.advance([t_end] * R, 0, 10**12)
        else:
            S.advance([t_sync] * R, max_cycles=n_cyc)
        st = S.read_stats()
        S.close()
        assert all(abs(x["t"] - t_end) <= 1e-12 * t_end for x in st)
        sets[frag] = np.array([x["D"][2] for x in st]), sum(int(x["hops"].sum()) for x in st)
    Dp = sets[0][0]
    for frag in (12, 8):
        Df = sets[frag][0]
        se = math.sqrt(Df.var(ddof=1) / R + Dp.var(ddof=1) / R)
        diff = Df.mean() - Dp.mean()
        say("  site model, %d^3 fragments: D_V %.5g vs %.5g A^2/us unfragmented (%+.2f sigma, %+.2f %%), "
            "%d hops" % (frag, 1e-6 * Df.mean(), 1e-6 * Dp.mean(), diff / se, 100 * diff / Dp.mean(),
                         sets[frag][1]))
        assert abs(diff) < 3 * se, (frag, Df.mean(), Dp.mean(), se)
        assert se < 0.05 * Dp.mean()
