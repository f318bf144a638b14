"""Pins of the oracle's atom-selection scheme with null events (Eqs. AtomP
and TimeStepFrg): with one selection per stage it is an exact kMC, so its
transient equals the master equation and its diffusion coefficient the
closed form; with many selections per stage the conflict rule keeps every
stage a set of hops on disjoint sites."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import brute

A = 3.905


def _rate_fn(p: O.RateParams, a=A):
    def fn(ion, d, src, dst):
        Ea = p.Ea_O if ion == 0 else p.Ea_H
        return brute.arrhenius(p.nu, Ea, p.T, p.E_z, p.q, d[2], a)
    return fn


def _state_at(lat, t):
    """Occupancy of a one-selection-per-stage run at time t (the state is
    constant between taken hops; a null stage leaves the clock alone)."""
    while True:
        occ = lat.occ.copy()
        n0 = lat.draws
        lat.advance_atomic(1, 1)
        assert lat.draws == n0 + 1
        if lat.t > t:
            return occ


@pytest.mark.parametrize("case", ["2V", "2V_field", "1V1H"])
def test_one_selection_transient_matches_master_equation(case):
    """P(state, t) with N^frg = 1 equals row s0 of expm(Q t): the null events
    (R_I < R^max when the two vacancies block each other, or next to H) make
    each taken hop's probability k_i / sum k and its waiting time
    exponential with rate sum k (Eq. AtomP and Eq. TimeStepFrg)."""
    L = (2, 2, 2)
    if case == "2V":
        p = O.RateParams(nu=1e13, T=600.0, Ea_O=0.6)
        nv, nh = 2, 0
    elif case == "2V_field":
        p = O.RateParams(nu=1e13, T=600.0, Ea_O=0.6, E_z=3e8, q=2.0)
        nv, nh = 2, 0
    else:
        p = O.RateParams(nu=1e13, T=600.0, Ea_O=0.6, Ea_H=0.55)
        nv, nh = 1, 1
    states, index, Q = brute.generator(L, nv, nh, _rate_fn(p))
    occ0 = states[7]
    k_o = brute.arrhenius(p.nu, p.Ea_O, p.T)
    t = 0.5 / k_o
    prob = brute.propagate(Q, t)[index[occ0.tobytes()]]
    R = 6000
    counts = np.zeros(len(states))
    for r in range(R):
        lat = O.Lattice(O.Geometry(L=L, seed=2024, lattice_id=r))
        lat.occ[:] = occ0
        lat.set_rates(p)
        counts[index[_state_at(lat, t).tobytes()]] += 1
    stat, pval = brute.chi2_pvalue(counts, prob)
    assert pval > 1e-4, (stat, pval)


@pytest.mark.parametrize("n_frg", [1, 8])
def test_single_vacancy_diffusion_closed_form(n_frg):
    """One vacancy: R^max = R_I, so no selection is null, and with several
    selections per stage all but the first touch the moved vacancy's old
    site: one hop per stage either way, D = Gamma_tot d^2 / 6."""
    p = O.RateParams(nu=1e13, T=600.0, Ea_O=0.6)
    k = brute.arrhenius(p.nu, p.Ea_O, p.T)
    gam = 8 * k
    L = (4, 4, 4)
    occ0 = np.zeros(3 * 64, np.int8)
    occ0[11] = 2
    R, n = 4000, 300
    r2 = np.zeros(R)
    t = np.zeros(R)
    for r in range(R):
        lat = O.Lattice(O.Geometry(L=L, seed=6, lattice_id=r))
        lat.occ[:] = occ0
        lat.set_rates(p)
        h = lat.advance_atomic(n_frg, n)
        assert sum(h) == n
        v = np.nonzero(lat.occ == 2)[0][0]
        r2[r] = (lat.disp[v].astype(float) ** 2).sum() * (A / 2) ** 2
        t[r] = lat.t
        assert lat.disp.sum(axis=0).tolist() == [0, 0, 0]
    # the clock: n hops at rate Gamma_tot each
    assert abs(t.mean() - n / gam) < 4 * t.std(ddof=1) / math.sqrt(R)
    D_est = r2.mean() / (6 * t.mean())
    D_ref = gam * (A / math.sqrt(2)) ** 2 / 6
    se = r2.std(ddof=1) / math.sqrt(R) / (6 * t.mean())
    assert abs(D_est - D_ref) < 4 * se + 0.01 * D_ref, (D_est, D_ref, se)


def test_crowded_stages_touch_disjoint_sites():
    """64 selections per stage on a crowded lattice: each stage's hops use
    distinct vacancies and distinct target ions (at most one hop per
    vacancy, never more than the vacancies), species are conserved, each
    particle's displacement travels with it (the sum is zero), and the
    clock moves by the number of hops times one waiting time."""
    g = O.Geometry(L=(3, 3, 3), seed=11, lattice_id=4)
    lat = O.Lattice(g)
    lat.init_random(12, 30)
    lat.set_rates(O.RateParams(nu=1e13, T=650.0, Ea_O=0.6, Ea_H=0.45))
    counts0 = np.bincount(lat.occ, minlength=3)
    total = 0
    for _ in range(300):
        occ = lat.occ.copy()
        h = lat.advance_atomic(64, 1)
        n = int(sum(h))
        total += n
        assert n <= 12
        changed = np.nonzero(occ != lat.occ)[0]
        # every hop swaps a vacancy with an ion: 2 changed sites per hop
        assert len(changed) == 2 * n
        assert (occ[changed] == 2).sum() == n and (lat.occ[changed] == 2).sum() == n
        assert np.bincount(lat.occ, minlength=3).tolist() == counts0.tolist()
        assert lat.disp.sum(axis=0).tolist() == [0, 0, 0]
    assert total > 300  # several hops per stage on average


@pytest.mark.parametrize("nv", [0, 24])
def test_no_possible_event_takes_no_stage(nv):
    """With no vacancy, or with every anion site of a 2x2x2 lattice vacant,
    K = 0: no stage runs, so the stage counter and the clock stay at zero
    and nothing moves."""
    lat = O.Lattice(O.Geometry(L=(2, 2, 2), seed=5, lattice_id=1))
    lat.init_random(nv, 0)
    lat.set_rates(O.RateParams(nu=1e13, T=600.0, Ea_O=0.6))
    occ0 = lat.occ.copy()
    h = lat.advance_atomic(8, 10)
    assert sum(h) == 0 and lat.draws == 0 and lat.t == 0.0
    assert np.array_equal(lat.occ, occ0)


def test_more_selections_than_vacancies():
    """64 selections per stage on 3 vacancies: at most 3 hops a stage (one
    per vacancy), and a stage with a taken hop always moves the clock."""
    lat = O.Lattice(O.Geometry(L=(4, 4, 4), seed=8, lattice_id=2))
    lat.init_random(3, 20)
    lat.set_rates(O.RateParams(nu=1e13, T=650.0, Ea_O=0.6, Ea_H=0.45))
    for _ in range(200):
        t0 = lat.t
        h = lat.advance_atomic(64, 1)
        n = int(sum(h))
        assert n <= 3
        assert (lat.t > t0) == (n > 0)
