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
    time.  Per temperature, D_V and D_H of the two agree within 3 sigma of
    their difference over the 32 seeds, and so does D_O where O hops are
    numerous (T >= 500 K, more than 1e3 O hops per lattice): the paper's
    accuracy criterion (Sec. "Accuracy and parallel efficiency of the
    fragment kMC method", Table TABLE01)."""
    import copy
    from paper_2004_09081_amd import workloads as W
    seeds = list(range(32))
    frag = [W.cfg2(T, seed=s) for T in W.CFG2_TEMPERATURES for s in seeds]
    plain = []
    for sp in frag:
        q = copy.copy(sp)
        q.frag = (0, 0, 0)
        plain.append(q)

    def build(specs):
        geoms, rates = W.to_gpu(specs, F)
        S = F.LatticeSet(geoms)
        S.init_random([sp.n_vac for sp in specs], [sp.n_h for sp in specs])
        S.set_rates(rates)
        return S

    say("cfg2: %d fragment lattices to 1e7 hops each" % len(frag))
    S = build(frag)
    S.set_schedule("persistent", 4)
    S.advance([sp.t_sync for sp in frag], max_cycles=10**9, min_hops=10_000_000)
    sf = S.read_stats()
    S.close()
    t_end = [x["t"] for x in sf]
    say("cfg2: %d unfragmented lattices to the same times" % len(plain))
    S = build(plain)
    S.advance(t_end, 0, 10**12)
    sp_ = S.read_stats()
    S.close()
    assert all(y["t"] == t for y, t in zip(sp_, t_end))
    n = len(seeds)
    bad = []
    for k, T in enumerate(W.CFG2_TEMPERATURES):
        a = sf[k * n:(k + 1) * n]
        b = sp_[k * n:(k + 1) * n]
        hf = np.array([int(x["hops"].sum()) for x in a])
        hp = np.array([int(x["hops"].sum()) for x in b])
        assert (hf >= 10_000_000).all()
        o_hops = min(int(x["hops"][0]) for x in a + b)
        rate_f = hf.sum() / (1e-3 * max(x["busy_ms"] for x in a)) if a[0]["busy_ms"] > 0 else 0.0
        line = "  T %3.0f K: cycles %d, hops frag %.4g plain %.4g, O hops >= %d, frag %.3g hops/s" % (
            T, a[0]["cycles"], hf.mean(), hp.mean(), o_hops, rate_f)
        species = [(2, "V"), (1, "H")] + ([(0, "O")] if T >= 500 else [])
        if T >= 500 and o_hops <= 1000:
            bad.append((T, "O hops", o_hops))
        for X, name in species:
            Df = np.array([x["D"][X] for x in a])
            Dp = np.array([x["D"][X] for x in b])
            se = math.sqrt(Df.var(ddof=1) / n + Dp.var(ddof=1) / n)
            diff = Df.mean() - Dp.mean()
            line += "; D_%s %.5g vs %.5g A^2/us (%+.2f sigma)" % (name, 1e-6 * Df.mean(), 1e-6 * Dp.mean(),
                                                               diff / se)
            if not abs(diff) < 3 * se:
                bad.append((T, name, Df.mean(), Dp.mean(), se))
        say(line)
    assert not bad, bad
