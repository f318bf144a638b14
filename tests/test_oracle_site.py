"""Pins of the oracle's site-energy model (Sec. "Oxygen vacancy diffusion
with dopant and defect interaction", Table TABLEadd01): site energies
against a brute-force sum over real-space pair distances; plain BKL with all
pair energies zero equals plain BKL bit for bit; every hop pair obeys
detailed balance with respect to the total pair energy; and long runs
visit states with the Boltzmann weights exp(-U/k_B T) (the stationary law
of the master equation, which detailed balance fixes)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2004_09081_amd import workloads as W
from tests import brute

KB = brute.KB
TABLE = O.SiteParams(e_fe=W.SITE_E_FE_MEV, e_vv=W.SITE_E_VV_MEV, window=1500)
# shells by squared distance in (a/2)^2
FE_SHELL = {1: 0, 5: 1, 9: 2, 13: 3}
VV_SHELL = {2: 0, 4: 1, 6: 2, 8: 3, 10: 4, 16: 5}


def _n(d):
    """Squared minimum-image distance in (a/2)^2 of a real-space vector d
    (units of a)."""
    return int(round(4.0 * float((d * d).sum())))


def brute_energy(L, occ, fe, sp, s, skip=-1):
    """Site energy of O site s from real-space positions: O sites at the cube
    face centres, B (Fe) sites at the cube centres."""
    S = brute.sites(L)
    Lv = np.array(L, float)
    p = S[s][3]
    E = 0
    for (m, _, _, q) in S:
        if m in (s, skip) or occ[m] != 2:
            continue
        d = q - p
        d -= Lv * np.round(d / Lv)
        sh = VV_SHELL.get(_n(d))
        if sh is not None:
            E += sp.e_vv[sh]
    for k in range(L[2]):
        for j in range(L[1]):
            for i in range(L[0]):
                if not fe[(k * L[1] + j) * L[0] + i]:
                    continue
                d = np.array([i + 0.5, j + 0.5, k + 0.5]) - p
                d -= Lv * np.round(d / Lv)
                sh = FE_SHELL.get(_n(d))
                if sh is not None:
                    E += sp.e_fe[sh]
    return E


def _lattice(L, nv, nh, fe_frac, seed, T=1200.0, sp=TABLE, **rp):
    lat = O.Lattice(O.Geometry(L=L, seed=seed))
    lat.init_random(nv, nh)
    fe = W.fe_map(L, fe_frac, seed)
    lat.set_site_model(fe, sp, O.RateParams(T=T, **rp))
    return lat


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_site_energies_match_brute_force_pair_sums(seed):
    L = (5, 6, 5)
    lat = _lattice(L, 14, 10, 0.05, seed)
    vs = [int(v) for v in np.nonzero(lat.occ == 2)[0]]
    rng = np.random.default_rng(seed)
    assert lat.fe.sum() > 0
    for v in vs:
        assert lat.site_energy(v) == brute_energy(L, lat.occ, lat.fe, TABLE, v)
        skip = int(rng.choice(vs))
        assert lat.site_energy(v, skip) == brute_energy(L, lat.occ, lat.fe, TABLE, v, skip)
    # an ion site, excluding a vacancy next to it
    for s in rng.choice(lat.g.n_sites, 20, replace=False):
        if lat.occ[s] == 2:
            continue
        assert lat.site_energy(int(s), vs[0]) == brute_energy(L, lat.occ, lat.fe, TABLE, int(s), vs[0])


def test_zero_pair_energies_give_plain_bkl_bit_for_bit():
    L = (6, 5, 7)
    rp = dict(T=650.0, Ea_O=0.6, Ea_H=0.45, E_z=1e8, gb_period_cells=3, gb_axes_mask=5, gb_dE=0.05)
    a = O.Lattice(O.Geometry(L=L, seed=9, lattice_id=3, gb_period_cells=3, gb_axes_mask=5))
    a.init_random(20, 50)
    b = O.Lattice(O.Geometry(L=L, seed=9, lattice_id=3, gb_period_cells=3, gb_axes_mask=5))
    b.init_random(20, 50)
    a.set_rates(O.RateParams(**rp))
    b.set_site_model(W.fe_map(L, 0.1, 4), O.SiteParams(window=0), O.RateParams(**rp))
    assert np.array_equal(b.site_raw, O.absent_species_zeroed(O.rate_raw(O.RateParams(**rp), 3.905), b.occ))
    # the same quantum (n_ev of a plain domain) makes the rates identical
    assert a.q == b.site_q and np.array_equal(a.k12, np.rint(b.site_raw / b.site_q) * b.site_q)
    for n in (700, 1300):
        a.advance_plain(n)
        b.advance_plain_site(n)
        assert a.t == b.t and a.draws == b.draws
        assert np.array_equal(a.occ, b.occ) and np.array_equal(a.disp, b.disp)


def _total_energy(L, occ, fe, sp):
    """Total pair energy U (meV): vacancy-Fe pairs plus vacancy pairs once."""
    vs = [int(v) for v in np.nonzero(occ == 2)[0]]
    none = np.zeros_like(fe)
    U = 0
    for v in vs:
        U += brute_energy(L, occ, fe, O.SiteParams(e_fe=sp.e_fe, e_vv=(0,) * 6), v)
    for i, v in enumerate(vs):
        for w in vs[i + 1:]:
            occ2 = np.zeros_like(occ)
            occ2[w] = 2
            U += brute_energy(L, occ2, none, O.SiteParams(e_fe=(0,) * 4, e_vv=sp.e_vv), v)
    return U


def test_hops_obey_detailed_balance_with_the_total_pair_energy():
    L = (5, 5, 6)
    T = 900.0
    lat = _lattice(L, 10, 15, 0.06, 7, T=T, Ea_O=0.6, Ea_H=0.45)
    table = brute.neighbours(L)
    hop = O.hop_table()
    U0 = _total_energy(L, lat.occ, lat.fe, TABLE)
    checked = 0
    for v in [int(x) for x in np.nonzero(lat.occ == 2)[0]]:
        t_v = v % 3
        for d in range(8):
            tgt = O.hop_target(lat.g, v, d)
            if lat.occ[tgt] == 2:
                assert lat.site_rate(v, d) == 0.0
                continue
            kf = lat.site_rate(v, d)
            rev = O.Lattice(lat.g)
            rev.occ[:] = lat.occ
            rev.occ[v], rev.occ[tgt] = lat.occ[tgt], 2
            rev.set_site_model(lat.fe, TABLE, O.RateParams(T=T, Ea_O=0.6, Ea_H=0.45))
            # the reverse direction from tgt back to v
            dr = [e for e in range(8) if O.hop_target(lat.g, tgt, e) == v]
            assert len(dr) == 1
            kb = rev.site_rate(tgt, dr[0])
            U1 = _total_energy(L, rev.occ, lat.fe, TABLE)
            ratio = kf / kb
            ref = math.exp(-(U1 - U0) * 1e-3 / (KB * T))
            assert abs(ratio / ref - 1.0) < 4e-3, (v, d, ratio, ref, U1 - U0)
            checked += 1
    assert checked > 40


def _time_weighted(lat, n_hops, key, batches=20):
    """Fraction of time spent in each class key(lat) over n_hops single-hop
    calls, with batch means for the error."""
    per = n_hops // batches
    frac = []
    for b in range(batches):
        acc = {}
        for _ in range(per):
            k = key(lat)
            t0 = lat.t
            lat.advance_plain_site(1)
            acc[k] = acc.get(k, 0.0) + (lat.t - t0)
        tot = sum(acc.values())
        frac.append({k: x / tot for k, x in acc.items()})
    keys = sorted(set().union(*frac))
    m = {k: np.array([f.get(k, 0.0) for f in frac]) for k in keys}
    return {k: (v.mean(), v.std(ddof=1) / math.sqrt(batches)) for k, v in m.items()}


def test_one_vacancy_visits_fe_shells_with_boltzmann_weights():
    """One vacancy among two Fe dopants on a 5^3 lattice at 1500 K: the time
    fraction at each site energy equals sum over sites of that energy of
    exp(-E/k_B T), normalised."""
    L, T = (5, 5, 5), 1500.0
    lat = O.Lattice(O.Geometry(L=L, seed=11))
    lat.init_random(1, 0)
    fe = np.zeros(125, np.uint8)
    fe[[0, 62]] = 1
    lat.set_site_model(fe, TABLE, O.RateParams(T=T, Ea_O=0.6))
    E = np.array([brute_energy(L, np.zeros(375, np.int8), fe, TABLE, s) for s in range(375)])
    w = {}
    for e in E:
        w[int(e)] = w.get(int(e), 0.0) + math.exp(-e * 1e-3 / (KB * T))
    Z = sum(w.values())
    Es = {int(s): int(E[s]) for s in range(375)}
    res = _time_weighted(lat, 60000, lambda l: Es[int(np.nonzero(l.occ == 2)[0][0])])
    assert len(w) >= 4
    for e, x in w.items():
        m, se = res.get(e, (0.0, 0.0))
        assert abs(m - x / Z) < 4.5 * se + 2e-3, (e, m, x / Z, se)


def test_two_vacancies_visit_pair_shells_with_boltzmann_weights():
    """Two vacancies, no Fe, 5^3 lattice at 1200 K: the time fraction at each
    pair distance equals (pairs at that distance) exp(-e_VV/k_B T),
    normalised."""
    L, T = (5, 5, 5), 1200.0
    lat = O.Lattice(O.Geometry(L=L, seed=12))
    lat.init_random(2, 0)
    lat.set_site_model(np.zeros(125, np.uint8), TABLE, O.RateParams(T=T, Ea_O=0.6))
    S = brute.sites(L)
    pos = np.array([s[3] for s in S])
    Lv = np.array(L, float)

    def n_of(a, b):
        d = pos[b] - pos[a]
        d -= Lv * np.round(d / Lv)
        return _n(d)
    w = {}
    for a in range(375):
        for b in range(a + 1, 375):
            n = n_of(a, b)
            e = TABLE.e_vv[VV_SHELL[n]] if n in VV_SHELL else 0
            w[e] = w.get(e, 0.0) + math.exp(-e * 1e-3 / (KB * T))
    Z = sum(w.values())

    def key(l):
        a, b = [int(x) for x in np.nonzero(l.occ == 2)[0]]
        n = n_of(a, b)
        return TABLE.e_vv[VV_SHELL[n]] if n in VV_SHELL else 0
    res = _time_weighted(lat, 60000, key)
    for e, x in w.items():
        m, se = res.get(e, (0.0, 0.0))
        assert abs(m - x / Z) < 4.5 * se + 2e-3, (e, m, x / Z, se)


# --------------------------------------------------------------------------- fragment kMC
def _frag_pair(L, frag, nv, nh, rp, window, fe_frac=0.1, seed=9, **g):
    mk = lambda: O.Lattice(O.Geometry(L=L, frag=frag, seed=seed, lattice_id=3, **g))
    a, b = mk(), mk()
    a.init_random(nv, nh)
    b.init_random(nv, nh)
    return a, b


def test_zero_pair_energies_give_fragment_kmc_bit_for_bit():
    """Fragment kMC with site energies and every pair energy zero follows
    fragment kMC without them bit for bit (6- and 7-cell fragments: sub-blocks
    of 3 and 4 cells; field, boundary planes, H).  With nv below the smallest
    footprint's site count, both quanta come from n_ev = 8 nv."""
    L, frag = (12, 12, 13), (6, 6, 6)
    rp = dict(T=650.0, Ea_O=0.6, Ea_H=0.45, E_z=1e8, gb_period_cells=4, gb_axes_mask=6, gb_dE=0.05)
    a, b = _frag_pair(L, frag, 20, 60, rp, 0, gb_period_cells=4, gb_axes_mask=6)
    a.set_rates(O.RateParams(**rp))
    b.set_site_model(W.fe_map(L, 0.1, 4), O.SiteParams(window=0), O.RateParams(**rp))
    assert a.q == b.site_q and np.array_equal(a.k12, np.rint(b.site_raw / b.site_q) * b.site_q)
    t_sync = 2.0 / (8 * a.k12[0])
    for cyc in (3, 5):
        a.advance(t_sync, cyc)
        b.advance_site(t_sync, cyc)
        assert a.cycles == b.cycles and a.t == b.t
        assert np.array_equal(a.hops, b.hops) and int(a.hops.sum()) > 20
        assert np.array_equal(a.occ, b.occ) and np.array_equal(a.disp, b.disp)


def test_fragment_site_refuses_sub_blocks_within_the_vacancy_reach():
    """The paper's table reaches squared doubled distance 10 (the 6th
    vacancy-vacancy shell is 0): 1-cell sub-blocks are refused, 2-cell ones
    run; with a nonzero 6th shell (16) 2-cell sub-blocks are refused too."""
    L = (8, 8, 8)
    far = O.SiteParams(e_fe=W.SITE_E_FE_MEV, e_vv=W.SITE_E_VV_MEV[:5] + (60,), window=1500)
    for frag, sp, ok in (((2, 4, 4), TABLE, False), ((4, 4, 4), TABLE, True), ((4, 4, 4), far, False),
                         ((8, 8, 8), far, True)):
        lat = O.Lattice(O.Geometry(L=L, frag=frag, seed=2))
        lat.init_random(6, 0)
        lat.set_site_model(W.fe_map(L, 0.05, 2), sp, O.RateParams(T=900.0, Ea_O=0.6))
        if ok:
            lat.advance_site(1e-9, 1)
        else:
            with pytest.raises(ValueError, match="too narrow"):
                lat.advance_site(1e-9, 1)


def _phase_orders(L, frag, nv, seed, sp=TABLE, T=1100.0):
    """One cycle of site-model phases with each colour's sub-blocks taken in
    ascending and in descending fragment order; returns both final states."""
    out = []
    for order in (1, -1):
        lat = O.Lattice(O.Geometry(L=L, frag=frag, seed=seed))
        lat.init_random(nv, 0)
        lat.set_site_model(W.fe_map(L, 0.08, seed), sp, O.RateParams(T=T, Ea_O=0.6))
        t_sync = 40.0 / (8 * 1e13 * math.exp(-0.6 / (KB * T)))
        nf = lat.n_fragments
        for c in range(8):
            for f in range(nf)[::order]:
                lat.phase_site(t_sync, 0, c, f)
        out.append((lat.occ.copy(), lat.disp.copy()))
    return out


def test_sub_blocks_of_a_phase_are_independent_beyond_the_reach():
    """When every sub-block is wide enough for the vacancy-vacancy reach, no
    rate of a sub-block reads a site that another sub-block of the same
    colour changes, so the order in which a phase takes its sub-blocks does
    not matter: a cycle in ascending and in descending order ends in the
    same state (3- and 2-cell sub-blocks with the paper's table).  Within the
    reach (1-cell sub-blocks, or 2-cell ones with a nonzero 6th shell) the
    two orders differ."""
    far = O.SiteParams(e_fe=W.SITE_E_FE_MEV, e_vv=W.SITE_E_VV_MEV[:5] + (60,), window=1500)
    for L, frag, sp, same in (((12, 12, 12), (6, 6, 6), TABLE, True), ((8, 8, 8), (4, 4, 4), TABLE, True),
                              ((8, 8, 8), (4, 4, 4), far, False), ((8, 8, 8), (2, 2, 2), TABLE, False)):
        (o1, d1), (o2, d2) = _phase_orders(L, frag, 120, 5, sp)
        assert (np.array_equal(o1, o2) and np.array_equal(d1, d2)) == same, (L, frag, sp.e_vv)


def test_fragment_site_cycle_ends_sample_the_boltzmann_law():
    """Each phase is an exact BKL process on its edges whose rates obey
    detailed balance with respect to exp(-U/k_B T), so every phase, and the
    cycle, keeps that law: one vacancy among two Fe dopants on a 6^3 lattice
    (3-cell sub-blocks) at 1500 K, sampled at cycle ends, sits at each site
    energy with the Boltzmann weights."""
    L, T = (6, 6, 6), 1500.0
    lat = O.Lattice(O.Geometry(L=L, frag=(6, 6, 6), seed=13))
    lat.init_random(1, 0)
    fe = np.zeros(216, np.uint8)
    fe[[0, 129]] = 1
    lat.set_site_model(fe, TABLE, O.RateParams(T=T, Ea_O=0.6))
    n_sites = 3 * 216
    E = np.array([brute_energy(L, np.zeros(n_sites, np.int8), fe, TABLE, s) for s in range(n_sites)])
    w = {}
    for e in E:
        w[int(e)] = w.get(int(e), 0.0) + math.exp(-e * 1e-3 / (KB * T))
    Z = sum(w.values())
    t_sync = 3.0 / (8 * 1e13 * math.exp(-0.6 / (KB * T)))
    batches, per = 20, 1500
    frac = []
    for _ in range(batches):
        acc = {}
        for _ in range(per):
            lat.advance_site(t_sync, 1)
            e = int(E[int(np.nonzero(lat.occ == 2)[0][0])])
            acc[e] = acc.get(e, 0) + 1
        frac.append({k: v / per for k, v in acc.items()})
    assert len(w) >= 4
    for e, x in w.items():
        v = np.array([f.get(e, 0.0) for f in frac])
        m, se = v.mean(), v.std(ddof=1) / math.sqrt(batches)
        assert abs(m - x / Z) < 4.5 * se + 3e-3, (e, m, x / Z, se)
