"""Pins of the oracle's dynamics: the BKL step and clock against the exact
master equation, the phase splitting against the exact product of phase
propagators, and closed forms for diffusion and drift."""
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


def _run_plain_ensemble(L, occ0, p, t, R, key0=1000):
    """Final occupancies of R independent plain-BKL runs to time t."""
    finals = []
    for r in range(R):
        lat = O.Lattice(O.Geometry(L=L, seed=key0, lattice_id=r))
        lat.occ[:] = occ0
        lat.set_rates(p)
        lat.advance_plain(10**9, t_horizon=t)
        assert lat.t == t
        finals.append(lat.occ.copy())
    return finals


@pytest.mark.parametrize("case", ["1V", "1V_field", "1V1H"])
def test_bkl_transient_matches_master_equation(case):
    """P(state, t) of plain BKL (Eqs. TransitionProb, eventSelection and
    TimeStep) equals row s0 of expm(Q t) of the exact generator on 2x2x2."""
    L = (2, 2, 2)
    if case == "1V":
        p = O.RateParams(nu=1e13, T=600.0, Ea_O=0.6)
        nv, nh = 1, 0
    elif case == "1V_field":
        p = O.RateParams(nu=1e13, T=600.0, Ea_O=0.6, E_z=3e8, q=2.0)
        nv, nh = 1, 0
    else:
        p = O.RateParams(nu=1e13, T=600.0, Ea_O=0.6, Ea_H=0.5)
        nv, nh = 1, 1
    states, index, Q = brute.generator(L, nv, nh, _rate_fn(p))
    occ0 = states[5]
    k_o = brute.arrhenius(p.nu, p.Ea_O, p.T)
    t = 0.6 / k_o
    prob = brute.propagate(Q, t)[index[occ0.tobytes()]]
    R = 12000 if nh else 6000
    counts = np.zeros(len(states))
    for occ in _run_plain_ensemble(L, occ0, p, t, R):
        counts[index[occ.tobytes()]] += 1
    stat, pval = brute.chi2_pvalue(counts, prob)
    assert pval > 1e-4, (stat, pval)


def _phase_filter(L, F, colour):
    """Edges whose midpoint cell lies in a sub-block of the given colour
    (fragments of F cells per axis, each halved; here F divides L)."""
    def sub_colour(cell):
        c = 0
        for a in range(3):
            x = cell[a] % F[a]
            c |= (1 if x >= (F[a] + 1) // 2 else 0) << a
        return c
    S = brute.sites(L)
    Lv = np.array(L, float)
    pos = [s[3] for s in S]

    def filt(src, dst):
        d = pos[dst] - pos[src]
        d -= Lv * np.round(d / Lv)
        mid = np.mod(pos[src] + d / 2.0, Lv)
        cell = tuple(int(math.floor(x + 1e-9)) for x in mid)
        return sub_colour(cell) == colour
    return filt


@pytest.mark.parametrize("L,F,nv,field", [((4, 4, 4), (4, 4, 4), 1, 0.0),
                                          ((4, 2, 2), (2, 2, 2), 2, 0.0),
                                          ((4, 2, 2), (2, 2, 2), 2, 3e8)])
def test_fragment_cycle_matches_phase_propagators(L, F, nv, field):
    """One fragment-kMC cycle equals prod_c expm(t_sync Q_c) over the 8
    colour classes in order, where Q_c holds the hops whose edge midpoint
    lies in a sub-block of colour c; several tiles of one colour run at
    once, vacancies block each other, the window ends at t_sync."""
    p = O.RateParams(nu=1e13, T=600.0, Ea_O=0.6, E_z=field, q=2.0)
    rf = _rate_fn(p)
    states, index, _ = brute.generator(L, nv, 0, rf)
    P = np.eye(len(states))
    k_o = brute.arrhenius(p.nu, p.Ea_O, p.T)
    t_sync = 0.7 / k_o
    for c in range(8):
        _, _, Qc = brute.generator(L, nv, 0, rf, edge_filter=_phase_filter(L, F, c))
        P = P @ brute.propagate(Qc, t_sync)
    occ0 = states[len(states) // 3]
    prob = P[index[occ0.tobytes()]]
    R = 6000
    counts = np.zeros(len(states))
    for r in range(R):
        lat = O.Lattice(O.Geometry(L=L, frag=F, seed=77, lattice_id=r))
        lat.occ[:] = occ0
        lat.set_rates(p)
        lat.advance(t_sync, max_cycles=1)
        counts[index[lat.occ.tobytes()]] += 1
    stat, pval = brute.chi2_pvalue(counts, prob)
    assert pval > 1e-4, (stat, pval)


def test_single_vacancy_diffusion_closed_form():
    """One vacancy: MSD(t) = Gamma_tot d^2 t exactly in expectation, so
    D = Gamma_tot d^2 / 6 with Gamma_tot = 8 nu exp(-Ea/kB T), d = a/sqrt(2)."""
    p = O.RateParams(nu=1e13, T=600.0, Ea_O=0.6)
    k = brute.arrhenius(p.nu, p.Ea_O, p.T)
    gam = 8 * k
    t = 300.0 / gam
    L = (4, 4, 4)
    occ0 = np.zeros(3 * 64, np.int8)
    occ0[7] = 2
    R = 5000
    r2 = np.zeros(R)
    for r in range(R):
        lat = O.Lattice(O.Geometry(L=L, seed=5, lattice_id=r))
        lat.occ[:] = occ0
        lat.set_rates(p)
        lat.advance_plain(10**9, t_horizon=t)
        v = np.nonzero(lat.occ == 2)[0][0]
        r2[r] = (lat.disp[v].astype(float) ** 2).sum() * (A / 2) ** 2
        assert lat.disp.sum(axis=0).tolist() == [0, 0, 0]
    D_est = r2.mean() / (6 * t)
    se = r2.std(ddof=1) / math.sqrt(R) / (6 * t)
    D_ref = gam * (A / math.sqrt(2)) ** 2 / 6
    assert abs(D_est - D_ref) < 4 * se, (D_est, D_ref, se)
    assert se / D_ref < 0.03


def test_biased_drift_closed_form():
    """One vacancy under a field along z from a uniform start: the uniform
    law is stationary, so E[z(t)] = v t with v = (4a/3)(k+ - k-)."""
    p = O.RateParams(nu=1e13, T=600.0, Ea_O=0.6, E_z=2e8, q=2.0)
    kp = brute.arrhenius(p.nu, p.Ea_O, p.T, p.E_z, p.q, 0.5)
    km = brute.arrhenius(p.nu, p.Ea_O, p.T, p.E_z, p.q, -0.5)
    v_ref = 4 * A / 3 * (kp - km)
    t = 200.0 / (8 * kp)
    R = 3000
    z = np.zeros(R)
    for r in range(R):
        lat = O.Lattice(O.Geometry(L=(3, 3, 3), seed=9, lattice_id=r))
        lat.init_random(1, 0)
        lat.set_rates(p)
        lat.advance_plain(10**9, t_horizon=t)
        v = np.nonzero(lat.occ == 2)[0][0]
        z[r] = lat.disp[v, 2] * A / 2
    v_est = z.mean() / t
    se = z.std(ddof=1) / math.sqrt(R) / t
    assert abs(v_est - v_ref) < 4 * se, (v_est, v_ref, se)
    assert se / v_ref < 0.05


def test_displacements_conserved_and_observables():
    """Every hop adds h to the vacancy and -h to the ion, so the sum of all
    displacements stays zero; per-species sums then satisfy
    N_V <r_V> = -(N_O <r_O> + N_H <r_H>).  Observables follow their
    definitions on a small hand-made configuration."""
    g = O.Geometry(L=(6, 6, 6), frag=(3, 3, 3))
    lat = O.Lattice(g)
    lat.init_random(20, 60)
    lat.set_rates(O.RateParams(T=700.0, Ea_O=0.6, Ea_H=0.4, E_z=1e8, q=2.0))
    lat.advance(2e-8, max_cycles=3)
    assert lat.disp.sum(axis=0).tolist() == [0, 0, 0]
    st = lat.stats()
    assert (st.sum_r.sum(axis=0) == 0).all()
    assert st.count.tolist() == [648 - 80, 60, 20]
    # hand-made: two vacancies, one H
    occ = np.zeros(24, np.int8)
    occ[[0, 5]] = 2
    occ[7] = 1
    disp = np.zeros((24, 3), np.int32)
    disp[0] = [2, 0, -1]
    disp[5] = [0, 1, 1]
    disp[7] = [-2, -1, 0]
    st = O.observables(occ, disp, 4.0, 2.0)
    assert st.count.tolist() == [21, 1, 2]
    assert st.sum_r[2].tolist() == [2, 1, 0]
    assert st.msd[2] == pytest.approx(4.0 * (5 + 2) / 2)
    assert st.D[2] == pytest.approx(st.msd[2] / 12.0)
    assert st.drift[2, 0] == pytest.approx(2.0 * 2 / (2 * 2.0))
    assert st.Dtensor[2, 0, 0] == pytest.approx(4.0 * ((4 + 0) / 2 - 1.0) / 4.0)


def test_drift_with_boundary_planes_matches_projected_chain():
    """One vacancy under a field along z with boundary planes normal to z:
    rates depend only on the layer Z (doubled coordinate), and layers of one
    parity are alike, so Z alone is a Markov chain on a ring of 2 Lz layers.
    Starting from its stationary law, E[z(t)] = v t with v from that chain."""
    from scipy.linalg import null_space
    T, Ea, E, q, gbdE, P = 600.0, 0.6, 3e8, 2.0, 0.08, 3
    Lxy, Lz = 3, 6
    p = O.RateParams(nu=1e13, T=T, Ea_O=Ea, E_z=E, q=q, gb_period_cells=P, gb_axes_mask=4, gb_dE=gbdE)
    k = lambda dz, g: brute.arrhenius(1e13, Ea, T, E, q, dz / 2.0, A, gb=g * gbdE)
    nz = 2 * Lz
    Q = np.zeros((nz, nz))
    gb_layer = lambda Z: Z % 2 == 0 and (Z // 2) % P == 0
    for Z in range(nz):
        up, dn = (Z + 1) % nz, (Z - 1) % nz
        if Z % 2:   # types 0/1: two up and two down hops, the other end is even
            Q[Z, up] += 2 * k(+1, gb_layer(up))
            Q[Z, dn] += 2 * k(-1, gb_layer(dn))
        else:       # type 2: four up and four down hops
            Q[Z, up] += 4 * k(+1, gb_layer(Z))
            Q[Z, dn] += 4 * k(-1, gb_layer(Z))
    Q -= np.diag(Q.sum(1))
    pi = null_space(Q.T)[:, 0]
    pi = pi / pi.sum()
    v_ref = sum(pi[Z] * (Q[Z, (Z + 1) % nz] - Q[Z, (Z - 1) % nz]) for Z in range(nz)) * A / 2
    # sites of each layer, and the stationary start
    g = O.Geometry(L=(Lxy, Lxy, Lz), gb_period_cells=P, gb_axes_mask=4)
    N = g.n_sites
    layer_sites = {Z: [] for Z in range(nz)}
    for s in range(N):
        t = s % 3
        kc = s // 3 // (Lxy * Lxy)
        layer_sites[2 * kc + (t != 2)].append(s)
    rng = np.random.default_rng(5)
    R = 3000
    tend = 150.0 / (8 * k(0, 0))
    z = np.zeros(R)
    for r in range(R):
        Z = rng.choice(nz, p=pi)
        s0 = rng.choice(layer_sites[Z])
        lat = O.Lattice(O.Geometry(L=(Lxy, Lxy, Lz), seed=13, lattice_id=r, gb_period_cells=P,
                                   gb_axes_mask=4))
        lat.occ[s0] = 2
        lat.set_rates(p)
        lat.advance_plain(10**9, t_horizon=tend)
        v = np.nonzero(lat.occ == 2)[0][0]
        z[r] = lat.disp[v, 2] * A / 2
    v_est = z.mean() / tend
    se = z.std(ddof=1) / math.sqrt(R) / tend
    assert abs(v_est - v_ref) < 4 * se, (v_est, v_ref, se)
    assert se / abs(v_ref) < 0.1


def _tilted_msd(Q, disp, pi, t, lam=1e-3):
    """Exact E[x(t)^2] of the additive functional x (jump i -> j adds
    disp[i, j]) of a chain with generator Q started from law pi: the second
    derivative at 0 of pi exp(t Q(lam)) 1, where Q(lam) multiplies each
    off-diagonal rate by exp(lam disp), by a central difference."""
    def mgf(l):
        M = Q * np.exp(l * disp)
        np.fill_diagonal(M, np.diag(Q))
        return float(pi @ brute.propagate(M, t) @ np.ones(len(pi)))
    return (mgf(lam) - 2.0 * mgf(0.0) + mgf(-lam)) / lam**2


@pytest.mark.parametrize("axis", [0, 1])
def test_diffusion_across_boundary_planes_matches_projected_chain(axis):
    """One vacancy, no field, boundary planes normal to x (or y) every P
    cells.  A site lies on a plane when its coordinate along that axis is a
    multiple of P lattice constants (positions and neighbours from real
    space, not from the oracle's tables).  Every site of one layer (equal
    doubled coordinate along the axis) has the same rates to each other
    layer, which the test checks, so the layer index alone is a Markov
    chain; from the stationary (uniform) start its exact E[dx(t)^2] must
    match the oracle's runs.  The planes slow diffusion along the axis by
    about 3x, far outside the statistical error."""
    T, Ea, gbdE, P = 600.0, 0.6, 0.1, 3
    L = [3, 3, 3]
    L[axis] = 6
    L = tuple(L)
    mask = 1 << axis
    S = brute.sites(L)
    nb = brute.neighbours(L)
    N = len(S)
    pos = np.array([s[3] for s in S])
    on_plane = np.array([abs(p[axis] - round(p[axis])) < 1e-9 and int(round(p[axis])) % P == 0
                         for p in pos])
    X = np.rint(2 * pos[:, axis]).astype(int) % (2 * L[axis])
    nl = 2 * L[axis]
    k = lambda g: brute.arrhenius(1e13, Ea, T, gb=gbdE if g else 0.0)
    per_site = np.zeros((N, nl))
    step = np.zeros((nl, nl))
    for s in range(N):
        for m, d in nb[s]:
            per_site[s, X[m]] += k(on_plane[s] or on_plane[m])
            step[X[s], X[m]] = round(2 * d[axis])
    Q = np.zeros((nl, nl))
    for Xl in range(nl):
        rows = per_site[X == Xl]
        assert np.allclose(rows, rows[0], rtol=1e-14, atol=0), "layer %d is not lumpable" % Xl
        Q[Xl] = rows[0]
    np.fill_diagonal(Q, 0.0)
    Q -= np.diag(Q.sum(1))
    w = np.bincount(X, minlength=nl).astype(float)
    pi = w / w.sum()
    tend = 150.0 / (8 * k(0))
    msd_ref = _tilted_msd(Q, step.astype(float), pi, tend)
    # without planes the same chain gives a clearly different value
    Q0 = np.where(Q > 0, 0.0, Q)
    Q0 = np.zeros_like(Q)
    for Xl in range(nl):
        for Ym in range(nl):
            if step[Xl, Ym] != 0:
                Q0[Xl, Ym] = (4 if Xl % 2 == 0 else 2) * k(0)
    Q0 -= np.diag(Q0.sum(1))
    msd_free = _tilted_msd(Q0, step.astype(float), pi, tend)
    p = O.RateParams(nu=1e13, T=T, Ea_O=Ea, gb_period_cells=P, gb_axes_mask=mask, gb_dE=gbdE)
    rng = np.random.default_rng(17 + axis)
    R = 3000
    x2 = np.zeros(R)
    for r in range(R):
        s0 = int(rng.integers(N))
        lat = O.Lattice(O.Geometry(L=L, seed=31, lattice_id=r, gb_period_cells=P, gb_axes_mask=mask))
        lat.occ[s0] = 2
        lat.set_rates(p)
        lat.advance_plain(10**9, t_horizon=tend)
        v = np.nonzero(lat.occ == 2)[0][0]
        x2[r] = float(lat.disp[v, axis]) ** 2
    est = x2.mean()
    se = x2.std(ddof=1) / math.sqrt(R)
    assert abs(est - msd_ref) < 4 * se, (est, msd_ref, se)
    assert abs(msd_free - msd_ref) > 10 * se, (msd_free, msd_ref, se)


@pytest.mark.parametrize("plain", [False, True])
def test_boundary_site_map_of_planes_equals_planes(plain):
    """A boundary-site map that marks exactly the plane sites (type-a sites
    of the cells whose index along a masked axis a is a multiple of the
    period) gives the plane model's trajectories bit for bit, in fragment
    cycles and in plain BKL: the map path inherits the planes' pins."""
    L, frag, P, mask = (9, 8, 10), ((0, 0, 0) if plain else (4, 4, 5)), 3, 5
    rp = O.RateParams(T=650.0, Ea_O=0.6, Ea_H=0.45, E_z=1e8, gb_period_cells=P, gb_axes_mask=mask,
                      gb_dE=0.1)
    gmap = np.zeros(3 * L[0] * L[1] * L[2], np.uint8)
    for k in range(L[2]):
        for j in range(L[1]):
            for i in range(L[0]):
                for t, c in enumerate((i, j, k)):
                    if (mask >> t) & 1 and c % P == 0:
                        gmap[((k * L[1] + j) * L[0] + i) * 3 + t] = 1
    lats = []
    for m in (None, gmap):
        lat = O.Lattice(O.Geometry(L=L, frag=frag, seed=3, lattice_id=1, gb_period_cells=P, gb_axes_mask=mask,
                                   gb_map=m))
        lat.init_random(25, 60)
        lat.set_rates(rp)
        lats.append(lat)
    for _ in range(2):
        for lat in lats:
            if plain:
                lat.advance_plain(800)
            else:
                lat.advance(2.0 / (8 * lat.k12[0]), max_cycles=3)
    a, b = lats
    assert a.t == b.t and np.array_equal(a.occ, b.occ) and np.array_equal(a.disp, b.disp)
    assert int(a.hops.sum()) > 0
    # a different map changes the trajectory
    c = O.Lattice(O.Geometry(L=L, frag=frag, seed=3, lattice_id=1, gb_map=np.roll(gmap, 1)))
    c.init_random(25, 60)
    c.set_rates(rp)
    for _ in range(2):
        if plain:
            c.advance_plain(800)
        else:
            c.advance(2.0 / (8 * c.k12[0]), max_cycles=3)
    assert not np.array_equal(a.occ, c.occ)
