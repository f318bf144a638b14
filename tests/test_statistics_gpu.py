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
