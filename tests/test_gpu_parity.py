"""GPU parity: the HIP path (through the C ABI) against the oracle,
element by element, on the same seeded inputs.  Integer state
(occupancy, displacements, hop counts, cycle counts) must be identical, and
so must the binary64 clock, because both sides follow the same sequence of
correctly rounded operations on exactly summable rates."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.common import Case, assert_same_state, gpu_set, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_09081_amd import fkmc
    fkmc.lib()


# Geometries: ragged remainders (>= 2 and == 1), single fragment along an
# axis, minimal L = 2, several tiles of each colour, H present, field, GB.
FRAG_CASES = {
    "cube12_w3": Case((12, 12, 12), (6, 6, 6), seed=1, nv=30, nh=100, T=700.0, Ea_O=0.6,
                      Ea_H=0.45),
    "ragged": Case((11, 9, 10), (4, 4, 3), seed=2, lattice_id=5, nv=25, nh=60, T=650.0,
                   Ea_O=0.55, Ea_H=0.5),
    "single_frag_axis": Case((8, 6, 4), (16, 3, 2), seed=3, nv=12, nh=0, T=600.0),
    "minimal_L2": Case((2, 2, 2), (2, 2, 2), seed=4, nv=3, nh=2, T=600.0, Ea_H=0.55),
    "field_gb": Case((16, 16, 20), (8, 8, 10), seed=5, nv=40, nh=0, T=500.0, Ea_O=0.5,
                     E_z=3e8, gb_period=5, gb_mask=4, gb_dE=0.1),
    "gb_all_axes": Case((12, 12, 12), (4, 4, 4), seed=6, nv=30, nh=30, T=600.0, Ea_O=0.55,
                        Ea_H=0.5, gb_period=3, gb_mask=7, gb_dE=0.05),
    "dense_vac": Case((8, 8, 8), (8, 8, 8), seed=7, nv=120, nh=40, T=600.0, Ea_H=0.5),
    # about 80 vacancies per footprint: the slot-recompute path
    "very_dense": Case((8, 8, 8), (8, 8, 8), seed=8, nv=500, nh=100, T=600.0, Ea_H=0.5),
}


@pytest.mark.parametrize("name", list(FRAG_CASES))
def test_init_matches_oracle(name):
    c = FRAG_CASES[name]
    say("init parity", name)
    g = gpu_set([c])
    assert_same_state(g, 0, c.oracle(), name)


@pytest.mark.parametrize("name", list(FRAG_CASES))
def test_fragment_cycles_match_oracle(name):
    c = FRAG_CASES[name]
    say("fragment parity", name)
    lat = c.oracle()
    k = lat.k12
    t_sync = 1.0 / (8.0 * k[0]) * 2.0
    g = gpu_set([c])
    assert g.get_rate_table(0).tobytes() == k.tobytes()
    for rep in range(2):
        lat.advance(t_sync, max_cycles=3)
        g.advance([t_sync], max_cycles=3)
        st = g.read_stats()[0]
        assert st["cycles"] == lat.cycles
        assert st["hops"].tolist() == [int(x) for x in lat.hops]
        assert st["t"] == lat.t
        assert_same_state(g, 0, lat, "%s rep %d" % (name, rep))
    assert int(lat.hops.sum()) > 0


def test_min_hops_stop_rule():
    c = FRAG_CASES["cube12_w3"]
    say("min_hops stop rule")
    lat = c.oracle()
    t_sync = 0.5 / (8.0 * lat.k12[0])
    lat.advance(t_sync, max_cycles=1000, min_hops=500)
    g = gpu_set([c])
    g.advance([t_sync], max_cycles=1000, min_hops=500)
    st = g.read_stats()[0]
    assert st["cycles"] == lat.cycles and st["hops"].tolist() == [int(x) for x in lat.hops]
    assert int(lat.hops.sum()) >= 500
    assert_same_state(g, 0, lat, "min_hops")


@pytest.mark.parametrize("name", ["ragged", "field_gb"])
def test_single_phase_matches_oracle(name):
    c = FRAG_CASES[name]
    say("single phase parity", name)
    lat = c.oracle()
    t_sync = 3.0 / (8.0 * lat.k12[0])
    g = gpu_set([c])
    for colour in (0, 5):
        for f in range(lat.n_fragments):
            lat.phase(t_sync, 0, colour, f)
        g.run_phase([t_sync], colour)
        assert_same_state(g, 0, lat, "%s colour %d" % (name, colour))


PLAIN_CASES = {
    "cfg1_8cube": Case((8, 8, 8), seed=0, nv=15, nh=0, T=600.0, Ea_O=0.6),
    "plain_H": Case((6, 5, 7), seed=9, lattice_id=3, nv=20, nh=50, T=650.0, Ea_O=0.6, Ea_H=0.45),
    "plain_field_gb": Case((6, 6, 6), seed=10, nv=8, nh=0, T=500.0, Ea_O=0.5, E_z=2e8,
                           gb_period=3, gb_dE=0.1),
    # 64 vacancies on 192 sites: most hops change a neighbouring slot too
    "dense_64": Case((4, 4, 4), seed=12, lattice_id=5, nv=64, nh=40, T=700.0, Ea_O=0.6, Ea_H=0.5),
    # LDS path with 2 and 4 slots per lane, at both ends of each range
    "dense_65": Case((5, 4, 4), seed=13, nv=65, nh=10, T=700.0, Ea_O=0.6, Ea_H=0.5),
    "slots_128": Case((6, 5, 5), seed=16, lattice_id=2, nv=128, nh=30, T=650.0, Ea_O=0.6, Ea_H=0.5),
    "slots_129": Case((6, 6, 5), seed=17, nv=129, nh=20, T=650.0, Ea_O=0.6, Ea_H=0.5, E_z=1e8),
    "slots_256": Case((8, 7, 6), seed=18, lattice_id=4, nv=256, nh=100, T=600.0, Ea_O=0.6,
                      Ea_H=0.45, gb_period=3, gb_dE=0.05),
    "slots_257": Case((8, 7, 6), seed=19, nv=257, nh=40, T=600.0, Ea_O=0.6, Ea_H=0.45),
    "slots_512": Case((10, 9, 8), seed=20, lattice_id=6, nv=512, nh=200, T=620.0, Ea_O=0.6,
                      Ea_H=0.45, E_z=5e7),
    # one vacancy more than the LDS path holds: the HBM kernel runs it
    "hbm_513": Case((10, 9, 8), seed=21, nv=513, nh=50, T=620.0, Ea_O=0.6, Ea_H=0.45),
    # 110,160 sites: held in LDS only at 2 bits per site
    "packed_big": Case((36, 34, 30), seed=22, lattice_id=7, nv=100, nh=5000, T=600.0, Ea_O=0.6,
                       Ea_H=0.4, E_z=2e7, gb_period=10, gb_dE=0.1),
    "edge2": Case((2, 3, 2), seed=14, nv=3, nh=4, T=650.0, Ea_O=0.6, Ea_H=0.5, E_z=1e8),
    "ragged_gb": Case((9, 7, 11), seed=15, lattice_id=9, nv=33, nh=90, T=550.0, Ea_O=0.55,
                      Ea_H=0.4, E_z=5e7, gb_period=4, gb_mask=7, gb_dE=0.08),
}


@pytest.mark.parametrize("lds", [True, False], ids=["lds", "hbm"])
@pytest.mark.parametrize("name", list(PLAIN_CASES))
def test_plain_matches_oracle(name, lds):
    """Plain BKL, in LDS on one wavefront (at most 512 vacancies) or in HBM
    on a workgroup: draws, clock, hop counts and state equal the oracle's."""
    c = PLAIN_CASES[name]
    say("plain parity", name, "lds" if lds else "hbm")
    lat = c.oracle()
    g = gpu_set([c])
    g.set_plain_lds(lds)
    for n_hops in (1000, 2500):
        lat.advance_plain(n_hops)
        g.advance([0.0], 0, n_hops)
        st = g.read_stats()[0]
        assert st["draws"] == lat.draws
        assert st["t"] == lat.t
        assert st["hops"].tolist() == [int(x) for x in lat.hops]
        assert_same_state(g, 0, lat, name)
    # horizon stop: the clock lands exactly on the horizon
    horizon = 50.0 / (8 * lat.k12[0])
    t0 = lat.t
    lat.advance_plain(10**9, t_horizon=horizon)
    g.advance([horizon - 0.0], 0, 10**9)
    st = g.read_stats()[0]
    assert lat.t == t0 + horizon
    assert st["t"] == lat.t and st["draws"] == lat.draws
    assert st["lds_resident"] == (1 if lds and c.nv <= 512 else 0)
    assert_same_state(g, 0, lat, name + " horizon")


# plain lattices past 4096 vacancies (the densest ensemble lattices hold up
# to 7,350): the HBM kernel sizes its LDS slot list per launch
PLAIN_BIG_CASES = [
    Case((16, 16, 17), seed=31, lattice_id=0, nv=4097, nh=800, T=620.0, Ea_O=0.6, Ea_H=0.45),
    Case((20, 20, 20), seed=32, lattice_id=1, nv=7350, nh=3000, T=600.0, Ea_O=0.6, Ea_H=0.45, E_z=1e8,
         gb_period=6, gb_dE=0.05),
    Case((20, 20, 21), seed=33, lattice_id=2, nv=8192, nh=0, T=650.0, Ea_O=0.6),
    Case((8, 7, 6), seed=34, lattice_id=3, nv=600, nh=40, T=650.0, Ea_O=0.6, Ea_H=0.45),
]


def test_plain_past_4096_vacancies_matches_oracle():
    """Plain BKL on the HBM kernel with 4097, 7350 and 8192 vacancies in one
    launch (slot list sized for the largest) beside a small lattice: draws,
    clock, hops and state equal the oracle's after two calls and a call
    stopped by its horizon; one vacancy more than the kernel holds is
    reported as FKMC_E_RANGE."""
    from paper_2004_09081_amd import fkmc as F
    say("plain parity past 4096 vacancies")
    lats = [c.oracle() for c in PLAIN_BIG_CASES]
    g = gpu_set(PLAIN_BIG_CASES)
    for n_hops in (800, 1200):
        for lat in lats:
            lat.advance_plain(n_hops)
        g.advance([0.0] * len(lats), 0, n_hops)
        stats = g.read_stats()
        for i, lat in enumerate(lats):
            assert stats[i]["lds_resident"] == 0
            assert stats[i]["draws"] == lat.draws and stats[i]["t"] == lat.t, i
            assert stats[i]["hops"].tolist() == [int(x) for x in lat.hops], i
            assert_same_state(g, i, lat, "plain big %d" % i)
    # about 300 hops' worth of time on each lattice
    hz = [300.0 / (8 * lat.k12[0] * c.nv) for lat, c in zip(lats, PLAIN_BIG_CASES)]
    h0 = [int(lat.hops.sum()) for lat in lats]
    for lat, h in zip(lats, hz):
        lat.advance_plain(10**9, t_horizon=h)
    g.advance(hz, 0, 10**9)
    stats = g.read_stats()
    for i, lat in enumerate(lats):
        assert 0 < int(lat.hops.sum()) - h0[i] < 20000
        assert stats[i]["draws"] == lat.draws and stats[i]["t"] == lat.t, i
        assert_same_state(g, i, lat, "plain big %d horizon" % i)
    g.close()
    g = gpu_set([Case((20, 20, 21), seed=2, nv=8193)])
    with pytest.raises(F.FkmcError) as e:
        g.advance([0.0], 0, 10)
    assert e.value.code == -4


# plain-mode degenerate cases: one vacancy, none, no ion to hop onto (no
# event at all), and a call ended by the horizon rather than the hop count
PLAIN_EDGE_CASES = {
    "one_vacancy": (Case((5, 4, 6), seed=5, nv=1, nh=10, T=650.0, Ea_O=0.6, Ea_H=0.45), 0.0),
    "no_vacancy": (Case((4, 4, 4), seed=4, nv=0, nh=5), 0.0),
    "no_ion": (Case((2, 2, 2), seed=3, nv=24, nh=0), 0.0),
    # 1,000 hops take 1.42e-8 s from this state in the oracle; the horizon
    # ends the second call part way
    "horizon": (Case((6, 5, 7), seed=9, lattice_id=3, nv=20, nh=50, T=650.0, Ea_O=0.6, Ea_H=0.45),
                0.6e-8),
}


@pytest.mark.parametrize("lds", [True, False], ids=["lds", "hbm"])
@pytest.mark.parametrize("name", list(PLAIN_EDGE_CASES))
def test_plain_edge_cases_match_oracle(name, lds):
    """Plain BKL with one vacancy, with none, with no event possible, and
    stopped by the horizon t_sync (the clock then takes t + t_sync and the
    draw is spent): draws, clock, hops and state equal the oracle's."""
    c, horizon = PLAIN_EDGE_CASES[name]
    say("plain edge parity", name, "lds" if lds else "hbm")
    lat = c.oracle()
    g = gpu_set([c])
    g.set_plain_lds(lds)
    for n_hops, h in ((500, 0.0), (10**6 if horizon else 1500, horizon)):
        lat.advance_plain(n_hops, h)
        g.advance([h], 0, n_hops)
        st = g.read_stats()[0]
        assert st["lds_resident"] == (1 if lds else 0)
        assert st["draws"] == lat.draws
        assert st["t"] == lat.t
        assert st["hops"].tolist() == [int(x) for x in lat.hops]
        assert_same_state(g, 0, lat, name)
    if name == "horizon":
        assert 0 < int(lat.hops.sum()) - 500 < 1000
    if name in ("no_vacancy", "no_ion"):
        assert lat.draws == 0 and int(lat.hops.sum()) == 0


# atom-selection scheme (Eqs. AtomP and TimeStepFrg): plain lattices in LDS
# with 0 to 512 vacancies, H, field, boundary planes, and no ion to hop onto
ATOMIC_CASES = [
    Case((5, 4, 6), seed=5, lattice_id=0, nv=1, nh=10, T=650.0, Ea_O=0.6, Ea_H=0.45),
    Case((8, 8, 8), seed=0, lattice_id=1, nv=15, nh=0, T=600.0, Ea_O=0.6),
    Case((6, 5, 7), seed=9, lattice_id=3, nv=20, nh=50, T=650.0, Ea_O=0.6, Ea_H=0.45),
    Case((6, 6, 6), seed=10, lattice_id=4, nv=8, nh=0, T=500.0, Ea_O=0.5, E_z=2e8, gb_period=3,
         gb_dE=0.1),
    Case((4, 4, 4), seed=12, lattice_id=5, nv=64, nh=40, T=700.0, Ea_O=0.6, Ea_H=0.5),
    Case((5, 4, 4), seed=13, lattice_id=6, nv=65, nh=10, T=700.0, Ea_O=0.6, Ea_H=0.5),
    Case((8, 7, 6), seed=18, lattice_id=7, nv=256, nh=100, T=600.0, Ea_O=0.6, Ea_H=0.45,
         gb_period=3, gb_dE=0.05),
    Case((10, 9, 8), seed=20, lattice_id=8, nv=512, nh=200, T=620.0, Ea_O=0.6, Ea_H=0.45, E_z=5e7),
    Case((4, 4, 4), seed=4, lattice_id=9, nv=0, nh=5),
    Case((2, 2, 2), seed=3, lattice_id=10, nv=24, nh=0),
    # past the LDS kernel: slots in LDS, occupancy in HBM
    Case((10, 9, 8), seed=21, lattice_id=11, nv=513, nh=50, T=620.0, Ea_O=0.6, Ea_H=0.45),
    Case((40, 30, 20), seed=23, lattice_id=12, nv=1200, nh=3000, T=650.0, Ea_O=0.6, Ea_H=0.45,
         E_z=1e8, gb_period=7, gb_dE=0.08),
    Case((16, 16, 16), seed=24, lattice_id=13, nv=4096, nh=0, T=600.0, Ea_O=0.6),
    # the largest slot count of the HBM kernel (one vacancy in three sites)
    Case((20, 20, 21), seed=25, lattice_id=14, nv=8192, nh=2000, T=600.0, Ea_O=0.6, Ea_H=0.45, E_z=5e7),
]


@pytest.mark.parametrize("lds", [True, False])
@pytest.mark.parametrize("n_frg", [1, 7, 64])
def test_atomic_matches_oracle(n_frg, lds):
    """The atom-selection scheme with null events on the GPU equals the
    oracle's bit for bit: stage counter, clock, hops and state, over calls
    of different lengths, and a plain BKL call in between (the two share
    the draw counter).  With lds off every lattice runs the HBM kernel."""
    say("atom-selection parity", n_frg, "lds" if lds else "hbm")
    lats = [c.oracle() for c in ATOMIC_CASES]
    g = gpu_set(ATOMIC_CASES)
    g.set_plain_lds(lds)
    for n_st, plain in ((40, 0), (90, 300), (25, 0)):
        for lat in lats:
            lat.advance_atomic(n_frg, n_st)
        g.advance_atomic(n_frg, n_st)
        if plain:
            for lat in lats:
                lat.advance_plain(plain)
            g.advance([0.0] * len(lats), 0, plain)
        stats = g.read_stats()
        for i, lat in enumerate(lats):
            assert stats[i]["draws"] == lat.draws, (i, n_st)
            assert stats[i]["t"] == lat.t, (i, n_st)
            assert stats[i]["hops"].tolist() == [int(x) for x in lat.hops], (i, n_st)
            assert_same_state(g, i, lat, "atom-selection member %d" % i)
    assert lats[0].draws == 155 + 300 and lats[8].draws == 0 and lats[9].draws == 0


def _random_plain_cases(seed, n):
    """n seeded random plain lattices of 2-16 cells per axis with 1 to 4096
    vacancies (from one vacancy to a third of the sites), H, field and
    boundary planes on random axes."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        L = tuple(int(x) for x in rng.integers(2, 17, size=3))
        sites = 3 * L[0] * L[1] * L[2]
        nv = int(min(4096, sites // 3, max(1, round(sites * 10 ** rng.uniform(-2.5, -0.4)))))
        if i % 6 == 0:  # one in six past the LDS kernel's 512 vacancies
            L = tuple(int(x) for x in rng.integers(12, 17, size=3))
            sites = 3 * L[0] * L[1] * L[2]
            nv = int(min(4096, sites // 3, rng.integers(513, 4097)))
        nh = int(rng.integers(0, (sites - nv) // 4 + 1))
        gb = int(rng.integers(2, 6)) if rng.random() < 0.4 else 0
        out.append(Case(L, seed=int(rng.integers(0, 1 << 30)), lattice_id=i, nv=nv, nh=nh,
                        T=float(rng.uniform(450, 800)), Ea_O=float(rng.uniform(0.5, 0.7)),
                        Ea_H=float(rng.uniform(0.35, 0.55)), E_z=float(rng.choice([0.0, 1e8, -2e8])),
                        gb_period=gb, gb_mask=int(rng.integers(1, 8)), gb_dE=0.07 if gb else 0.0))
    return out


@pytest.mark.parametrize("lds", [True, False])
def test_atomic_random_configurations_match_oracle(lds):
    """64 seeded random plain lattices (LDS and HBM kernels mixed, or all on
    the HBM kernel), three calls with random selection counts and stage
    counts, each against the oracle bit for bit."""
    cases = _random_plain_cases(911, 64)
    say("atom-selection random configurations", "lds" if lds else "hbm")
    rng = np.random.default_rng(912)
    lats = [c.oracle() for c in cases]
    g = gpu_set(cases)
    g.set_plain_lds(lds)
    for call in range(3):
        n_frg, n_st = int(rng.integers(1, 65)), int(rng.integers(20, 120))
        for lat in lats:
            lat.advance_atomic(n_frg, n_st)
        g.advance_atomic(n_frg, n_st)
        stats = g.read_stats()
        for i, lat in enumerate(lats):
            what = "member %d %s nv %d, call %d (n_frg %d)" % (i, cases[i].L, cases[i].nv, call, n_frg)
            assert stats[i]["draws"] == lat.draws and stats[i]["t"] == lat.t, what
            assert stats[i]["hops"].tolist() == [int(x) for x in lat.hops], what
            assert_same_state(g, i, lat, what)


def test_atomic_rejects_what_it_cannot_run():
    from paper_2004_09081_amd import fkmc as F
    g = gpu_set(ATOMIC_CASES[:2])
    for bad in (0, 65):
        with pytest.raises(F.FkmcError):
            g.advance_atomic(bad, 1)
    g = gpu_set([ATOMIC_CASES[0], Case((6, 6, 6), (3, 3, 3), seed=1, nv=4)])
    with pytest.raises(F.FkmcError):
        g.advance_atomic(1, 1)
    g = gpu_set([Case((20, 20, 21), seed=2, nv=8193)])
    with pytest.raises(F.FkmcError) as e:
        g.advance_atomic(1, 1)
    assert e.value.code == -6


def test_plain_lds_in_ensemble_launch():
    """Plain lattices held in LDS share the persistent launch with fragment
    lattices (hop targets: exact for plain, per cycle for fragments)."""
    cases = [Case((10, 10, 10), (5, 5, 5), seed=31, lattice_id=i, nv=12 + 3 * i, nh=20, T=650.0,
                  Ea_O=0.6, Ea_H=0.5) for i in range(3)]
    cases += [Case((7, 8, 6), seed=31, lattice_id=10 + i, nv=5 + 60 * i, nh=30, T=600.0 + 50 * i,
                   Ea_O=0.6, Ea_H=0.45, E_z=1e8 * i) for i in range(4)]
    say("plain LDS lattices in the persistent launch", len(cases))
    lats = [c.oracle() for c in cases]
    ts = [0.0 if l.g.plain else 1.0 / (8.0 * l.k12[0]) for l in lats]
    g = gpu_set(cases)
    g.set_schedule("persistent", 4)
    for rep in range(2):
        for lat, t in zip(lats, ts):
            if lat.g.plain:
                lat.advance_plain(1500)
            else:
                lat.advance(t, max_cycles=10**6, min_hops=1500)
        g.advance(ts, max_cycles=10**6, min_hops=1500)
        st = g.read_stats()
        for i, lat in enumerate(lats):
            assert_same_state(g, i, lat, "member %d call %d" % (i, rep))
            assert st[i]["t"] == lat.t
            assert st[i]["hops"].tolist() == [int(x) for x in lat.hops]
            if lat.g.plain:
                assert st[i]["draws"] == lat.draws and st[i]["lds_resident"] == 1


def test_batched_set_matches_oracle():
    """Lattices of different sizes, modes and parameters in one set, each
    identical to its own oracle run."""
    cases = [FRAG_CASES["cube12_w3"], FRAG_CASES["ragged"], PLAIN_CASES["plain_H"],
             FRAG_CASES["field_gb"], Case((20, 14, 9), (5, 7, 4), seed=11, lattice_id=77,
                                          nv=50, nh=120, T=800.0, Ea_O=0.7, Ea_H=0.5)]
    say("batched parity", len(cases))
    lats = [c.oracle() for c in cases]
    ts = [2.0 / (8.0 * l.k12[0]) for l in lats]
    g = gpu_set(cases)
    for lat, c, t in zip(lats, cases, ts):
        if lat.g.plain:
            lat.advance_plain(700)
        else:
            lat.advance(t, max_cycles=4)
    g.advance(ts, max_cycles=4, min_hops=0)
    # plain members make exactly min_hops hops; min_hops=0 means none
    for i, (lat, c) in enumerate(zip(lats, cases)):
        if lat.g.plain:
            continue
        assert_same_state(g, i, lat, "batch member %d" % i)
    stats = g.read_stats()
    for i, lat in enumerate(lats):
        if lat.g.plain:
            continue
        assert stats[i]["cycles"] == lat.cycles and stats[i]["t"] == lat.t


def test_stats_match_oracle_observables():
    c = FRAG_CASES["field_gb"]
    say("stats parity")
    lat = c.oracle()
    t_sync = 2.0 / (8.0 * lat.k12[0])
    lat.advance(t_sync, max_cycles=5)
    g = gpu_set([c])
    g.advance([t_sync], max_cycles=5)
    st = g.read_stats()[0]
    ref = lat.stats()
    assert st["count"].tolist() == ref.count.tolist()
    assert st["sum_r"].tolist() == ref.sum_r.tolist()
    rr = ref.sum_rr
    six = np.stack([rr[:, 0, 0], rr[:, 1, 1], rr[:, 2, 2], rr[:, 0, 1], rr[:, 0, 2], rr[:, 1, 2]], 1)
    assert st["sum_rr"].tolist() == six.tolist()
    np.testing.assert_allclose(st["msd"], ref.msd, rtol=1e-14)
    np.testing.assert_allclose(st["D"], ref.D, rtol=1e-14)
    np.testing.assert_allclose(st["drift"], ref.drift, rtol=1e-14)


def test_set_occupancy_and_rate_table_paths():
    """Caller-supplied occupancy and raw rate table give the oracle's run."""
    say("set_occupancy / set_rate_table")
    from paper_2004_09081_amd import fkmc as F
    c = FRAG_CASES["ragged"]
    lat = c.oracle()
    rng = np.random.default_rng(4)
    occ = np.zeros(lat.g.n_sites, np.int8)
    idx = rng.choice(lat.g.n_sites, 80, replace=False)
    occ[idx[:30]] = 2
    occ[idx[30:]] = 1
    lat.occ[:] = occ
    lat.disp[:] = 0
    raw = O.rate_raw(O.RateParams(T=700.0, Ea_O=0.5, Ea_H=0.45, E_z=1e8), lat.g.a_angstrom)
    nev = 8 * min(30, O.max_domain_sites(lat.g))
    lat.k12, _, _ = O.quantise(raw, nev)
    g = F.LatticeSet([c.gpu_geometry()])
    g.set_occupancy(0, occ)
    g.set_rate_table(0, raw)
    assert g.get_rate_table(0).tobytes() == lat.k12.tobytes()
    t_sync = 1.0 / (8 * lat.k12[0])
    lat.advance(t_sync, max_cycles=4)
    g.advance([t_sync], max_cycles=4)
    assert_same_state(g, 0, lat, "set_occupancy")


def test_no_vacancy_and_errors():
    say("edge cases: empty lattice, state errors")
    from paper_2004_09081_amd import fkmc as F
    c = Case((6, 6, 6), (3, 3, 3), nv=0, nh=10)
    g = gpu_set([c])
    g.advance([1e-9], max_cycles=3)
    st = g.read_stats()[0]
    assert st["cycles"] == 3 and st["hops"].tolist() == [0, 0]
    # rates invalidated by init_random: advance must refuse
    g.init_random([5], [0])
    with pytest.raises(F.FkmcError) as e:
        g.advance([1e-9], max_cycles=1)
    assert e.value.code == -2
    with pytest.raises(F.FkmcError):
        g.set_occupancy(0, np.full(g.geoms[0].n_sites, 3, np.int8))


@pytest.mark.parametrize("schedule", ["lockstep", "persistent"])
def test_crowded_domain_reports_range_error(schedule):
    """A BKL domain over the 128-vacancy cap is caught by the kernel's own
    bounds check and reported as FKMC_E_RANGE; reads keep reporting it
    until the lattice is initialised again, after which the set runs and
    matches the oracle."""
    say("crowded domain error", schedule)
    from paper_2004_09081_amd import fkmc as F
    # a fragment of edge 8 has 240-site domains: 1,100 vacancies put about
    # 170 in each
    cases = [Case((8, 8, 8), (8, 8, 8), seed=3, lattice_id=0, nv=1100),
             Case((8, 8, 8), (4, 4, 4), seed=3, lattice_id=1, nv=20)]
    g = gpu_set(cases)
    g.set_schedule(schedule, 4)
    with pytest.raises(F.FkmcError) as e:
        g.advance([1e-9, 1e-9], max_cycles=2)
    assert e.value.code == -4 and "lattice 0" in str(e.value)
    with pytest.raises(F.FkmcError):
        g.read_stats()
    cases[0].nv = 60
    g.init_random([c.nv for c in cases], [c.nh for c in cases])
    g.set_rates([c.gpu_rates() for c in cases])
    lats = [c.oracle() for c in cases]
    ts = [1.0 / (8.0 * l.k12[0]) for l in lats]
    for lat, t in zip(lats, ts):
        lat.advance(t, max_cycles=2)
    g.advance(ts, max_cycles=2)
    stats = g.read_stats()
    for i, lat in enumerate(lats):
        assert stats[i]["cycles"] == 2 and stats[i]["hops"].tolist() == [int(x) for x in lat.hops]
        assert_same_state(g, i, lat, "after re-initialisation %d" % i)


SCHED_CASES = [
    Case((30, 30, 28), (6, 6, 7), seed=21, lattice_id=0, nv=150, nh=600, T=700.0, Ea_O=0.6,
         Ea_H=0.45),                                    # 75,600 sites: not LDS-resident
    Case((10, 10, 10), (4, 4, 4), seed=21, lattice_id=1, nv=20, nh=30, T=650.0, Ea_O=0.55,
         Ea_H=0.5, E_z=2e8),                            # resident, ragged fragments
    Case((16, 16, 16), (8, 8, 8), seed=21, lattice_id=2, nv=40, nh=0, T=600.0, Ea_O=0.6,
         gb_period=4, gb_dE=0.1),                       # resident, boundary planes
    Case((6, 7, 5), (2, 3, 5), seed=21, lattice_id=3, nv=90, nh=20, T=600.0, Ea_H=0.5),  # > 64 slots possible
]


@pytest.mark.parametrize("schedule,waves", [("lockstep", 0), ("persistent", 1),
                                            ("persistent", 4), ("persistent", 8)])
def test_schedules_match_oracle(schedule, waves):
    """Lockstep launches and the persistent one-workgroup-per-lattice kernel
    (any wave count, LDS-resident or HBM-staged lattices) give the oracle's
    trajectories bit for bit."""
    say("schedule parity", schedule, waves)
    lats = [c.oracle() for c in SCHED_CASES]
    ts = [1.5 / (8.0 * l.k12[0]) for l in lats]
    for lat, t in zip(lats, ts):
        lat.advance(t, max_cycles=3)
    g = gpu_set(SCHED_CASES)
    g.set_schedule(schedule, waves)
    g.advance(ts, max_cycles=3)
    stats = g.read_stats()
    for i, lat in enumerate(lats):
        assert stats[i]["cycles"] == lat.cycles and stats[i]["t"] == lat.t
        assert stats[i]["hops"].tolist() == [int(x) for x in lat.hops]
        assert_same_state(g, i, lat, "%s/%d member %d" % (schedule, waves, i))


# a dense lattice whose single tile overflows 8 and 16 slots
GROUP_CASES = SCHED_CASES + [FRAG_CASES["dense_vac"]]


@pytest.mark.parametrize("schedule,group", [("lockstep", 8), ("lockstep", 4), ("lockstep", 2),
                                            ("lockstep", 1), ("persistent", 8), ("persistent", 4),
                                            ("persistent", 1)])
def test_tile_groups_match_oracle(schedule, group):
    """Every tile-group size (tiles per wavefront), including tiles whose
    vacancies overflow their segment's slots and run on the whole
    wavefront, reproduces the oracle bit for bit."""
    say("tile group parity", schedule, group)
    lats = [c.oracle() for c in GROUP_CASES]
    ts = [1.5 / (8.0 * l.k12[0]) for l in lats]
    for lat, t in zip(lats, ts):
        lat.advance(t, max_cycles=3)
    g = gpu_set(GROUP_CASES)
    g.set_schedule(schedule, 4)
    g.set_group(group)
    g.advance(ts, max_cycles=3)
    stats = g.read_stats()
    if schedule == "persistent":
        # every member ran the requested group, the HBM-staged one included
        assert [s["tile_group"] for s in stats] == [group] * len(stats)
        assert not stats[0]["lds_resident"] and stats[1]["lds_resident"]
    for i, lat in enumerate(lats):
        assert stats[i]["cycles"] == lat.cycles and stats[i]["t"] == lat.t
        assert stats[i]["hops"].tolist() == [int(x) for x in lat.hops]
        assert_same_state(g, i, lat, "%s/group %d member %d" % (schedule, group, i))


# one fragment, held in LDS, at most 32 vacancies: a block of lanes per vacancy
# (the 64-vacancy members take the tile path)
FAST_CASES = [
    Case((12, 10, 8), (12, 10, 8), seed=31, lattice_id=0, nv=20, nh=30, T=650.0, Ea_O=0.55,
         Ea_H=0.5, E_z=2e8, gb_period=3, gb_mask=5, gb_dE=0.08),
    Case((2, 2, 2), (2, 2, 2), seed=31, lattice_id=1, nv=3, nh=2, T=600.0, Ea_H=0.55),
    Case((9, 7, 5), (16, 16, 16), seed=31, lattice_id=2, nv=40, nh=10, T=700.0, Ea_O=0.6,
         Ea_H=0.45),
    Case((16, 16, 16), (16, 16, 16), seed=31, lattice_id=3, nv=64, nh=300, T=500.0, Ea_O=0.5,
         Ea_H=0.35),
    Case((5, 6, 7), (5, 6, 7), seed=31, lattice_id=4, nv=64, nh=0, T=600.0),
    Case((11, 3, 4), (20, 20, 20), seed=31, lattice_id=5, nv=1, nh=5, T=800.0, Ea_H=0.4),
]


@pytest.mark.parametrize("min_hops", [0, 1500])
def test_single_fragment_lattices_match_oracle(min_hops):
    """Single-fragment lattices held in LDS with a block of lanes per
    vacancy (the persistent schedule's path for up to 32 vacancies), odd
    sizes, L = 2, field and boundary planes on two axes: the oracle's
    trajectories bit for bit, over several calls, with and without a hop
    target."""
    say("single-fragment parity", min_hops)
    lats = [c.oracle() for c in FAST_CASES]
    ts = [1.3 / (8.0 * l.k12[0]) for l in lats]
    g = gpu_set(FAST_CASES)
    g.set_schedule("persistent", 4)
    for rep in range(2):
        for lat, t in zip(lats, ts):
            lat.advance(t, max_cycles=10**6 if min_hops else 5, min_hops=min_hops)
        g.advance(ts, max_cycles=10**6 if min_hops else 5, min_hops=min_hops)
        stats = g.read_stats()
        for i, lat in enumerate(lats):
            assert stats[i]["lds_resident"]
            assert stats[i]["cycles"] == lat.cycles and stats[i]["t"] == lat.t, (i, rep)
            assert stats[i]["hops"].tolist() == [int(x) for x in lat.hops], (i, rep)
            assert_same_state(g, i, lat, "single-fragment member %d rep %d" % (i, rep))


def test_schedule_rejects_oversized_workgroup():
    from paper_2004_09081_amd import fkmc as F
    g = gpu_set(SCHED_CASES[1:3])
    with pytest.raises(F.FkmcError):
        g.set_schedule("persistent", 16)


def test_persistent_min_hops_rule():
    say("persistent min_hops")
    lats = [c.oracle() for c in SCHED_CASES[1:3]]
    ts = [1.0 / (8.0 * l.k12[0]) for l in lats]
    for lat, t in zip(lats, ts):
        lat.advance(t, max_cycles=500, min_hops=300)
    g = gpu_set(SCHED_CASES[1:3])
    g.set_schedule("persistent", 4)
    g.advance(ts, max_cycles=500, min_hops=300)
    stats = g.read_stats()
    for i, lat in enumerate(lats):
        assert stats[i]["cycles"] == lat.cycles
        assert_same_state(g, i, lat, "member %d" % i)


def test_graph_replays_match_eager_and_oracle():
    """Lockstep cycles replayed from the HIP graph, several calls in a row
    with reads and eager work between them, equal the separately launched
    path and the oracle at every call (including max_cycles that is not a
    multiple of the graph's 8 cycles, and a hop target)."""
    say("graph replays")
    c = FRAG_CASES["ragged"]
    lat = c.oracle()
    t_sync = 1.5 / (8.0 * lat.k12[0])
    g = gpu_set([c])
    e = gpu_set([c])
    e.set_graph(False)
    for rep, (mc, mh) in enumerate([(3, 0), (11, 0), (1000, 400), (5, 0)]):
        lat.advance(t_sync, max_cycles=mc, min_hops=mh)
        g.advance([t_sync], max_cycles=mc, min_hops=mh)
        e.advance([t_sync], max_cycles=mc, min_hops=mh)
        sg, se = g.read_stats()[0], e.read_stats()[0]
        assert sg["cycles"] == se["cycles"] == lat.cycles, (rep, sg["cycles"], se["cycles"], lat.cycles)
        assert sg["t"] == lat.t and sg["hops"].tolist() == [int(x) for x in lat.hops]
        assert_same_state(g, 0, lat, "graph call %d" % rep)
        assert_same_state(e, 0, lat, "eager call %d" % rep)


@pytest.mark.parametrize("name", ["field_gb", "plain"])
def test_checkpoint_resume_is_bit_exact(name):
    """Checkpoint after some cycles, restore into a fresh handle, continue:
    identical to the uninterrupted run and to the oracle."""
    say("checkpoint/resume", name)
    c = FRAG_CASES["field_gb"] if name == "field_gb" else PLAIN_CASES["plain_H"]
    lat = c.oracle()
    t_sync = 2.0 / (8.0 * lat.k12[0])
    a = gpu_set([c])
    def step(s):
        if lat.g.plain:
            s.advance([0.0], 0, 700)
        else:
            s.advance([t_sync], max_cycles=3)
    step(a)
    blob = a.checkpoint(0)
    step(a)
    b = gpu_set([c])
    b.init_random([0], [0])          # wipe, then restore
    b.restore(0, blob)
    step(b)
    sa, sb = a.read_stats()[0], b.read_stats()[0]
    for k in ("t", "cycles", "draws"):
        assert sa[k] == sb[k], k
    assert sa["hops"].tolist() == sb["hops"].tolist()
    oa, da = a.read_state(0)
    ob, db = b.read_state(0)
    assert np.array_equal(oa, ob) and np.array_equal(da, db)
    if lat.g.plain:
        lat.advance_plain(700)
        lat.advance_plain(700)
    else:
        lat.advance(t_sync, max_cycles=3)
        lat.advance(t_sync, max_cycles=3)
    assert_same_state(b, 0, lat, "resumed " + name)
    assert sb["t"] == lat.t


def _random_cases(seed, n):
    """n seeded random small configurations: non-cubic lattices of 2-12
    cells per axis, fragment edges from 0 (plain) up to the lattice,
    vacancy fractions from one vacancy to crowded, H, field, boundary
    planes on random axes."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        L = tuple(int(x) for x in rng.integers(2, 13, size=3))
        sites = 3 * L[0] * L[1] * L[2]
        if rng.random() < 0.3:
            fr = (0, 0, 0)
        else:
            e = int(rng.integers(2, max(L) + 2))
            fr = (e, e, e)
        nv = int(min(sites // 3, max(1, round(sites * 10 ** rng.uniform(-2.5, -0.7)))))
        if fr[0]:
            # a BKL domain holds at most 128 vacancies: keep the mean per
            # domain at 40 or below, so none comes near the cap
            dom = O.max_domain_sites(O.Geometry(L=L, frag=fr))
            nv = max(1, min(nv, 128, 40 * sites // dom))
        nh = int(rng.integers(0, (sites - nv) // 4 + 1))
        gb = int(rng.integers(0, 5)) if rng.random() < 0.4 else 0
        out.append(Case(L, fr, seed=int(rng.integers(0, 1 << 30)), lattice_id=i, nv=nv, nh=nh,
                        T=float(rng.uniform(450, 800)), Ea_O=float(rng.uniform(0.5, 0.7)),
                        Ea_H=float(rng.uniform(0.35, 0.55)), E_z=float(rng.choice([0.0, 1e8, -2e8])),
                        gb_period=gb, gb_mask=int(rng.integers(1, 8)), gb_dE=0.07 if gb else 0.0))
    return out


@pytest.mark.parametrize("schedule", ["lockstep", "persistent"])
@pytest.mark.parametrize("seed", [20260, 7])
def test_random_configurations_match_oracle(schedule, seed):
    """96 seeded random configurations in one set, two calls (a cycle
    count, then a hop target), every lattice against the oracle bit for
    bit."""
    cases = _random_cases(seed, 96)
    say("random configurations", schedule, seed)
    lats = [c.oracle() for c in cases]
    ts = [0.0 if c.frag[0] == 0 else 1.2 / (8.0 * l.k12[0]) for c, l in zip(cases, lats)]
    g = gpu_set(cases)
    g.set_schedule(schedule, 4)
    for max_cycles, min_hops in ((3, 0), (10**6, 400)):
        for c, lat, t in zip(cases, lats, ts):
            if c.frag[0] == 0:
                lat.advance_plain(min_hops)  # plain: exactly min_hops hops
            else:
                lat.advance(t, max_cycles=max_cycles, min_hops=min_hops)
        g.advance(ts, max_cycles=max_cycles, min_hops=min_hops)
        stats = g.read_stats()
        for i, lat in enumerate(lats):
            assert stats[i]["cycles"] == lat.cycles and stats[i]["t"] == lat.t, (i, cases[i].L, cases[i].frag)
            assert stats[i]["hops"].tolist() == [int(x) for x in lat.hops], (i, cases[i].L, cases[i].frag)
            assert_same_state(g, i, lat, "random member %d %s %s" % (i, cases[i].L, cases[i].frag))



# Fragment edges of 14, 18, 20 and 24 cells (sub-blocks of 7, 9, 10 and 12
# cells, and the odd halves 8/7, 10/9, 11/10, 13/12 of merged remainders),
# each once small enough to be held in LDS by the persistent kernel and once
# staged from HBM, with a ragged remainder of >= 2 cells and one of 1 cell.
WIDE_CASES = [
    Case((26, 25, 24), (14, 14, 14), seed=41, lattice_id=0, nv=230, nh=4000, T=650.0, Ea_O=0.6,
         Ea_H=0.45, E_z=5e7),
    Case((30, 29, 28), (14, 14, 14), seed=41, lattice_id=1, nv=370, nh=7000, T=620.0, Ea_O=0.6,
         Ea_H=0.45, gb_period=7, gb_mask=7, gb_dE=0.06),
    Case((26, 23, 19), (18, 18, 18), seed=41, lattice_id=2, nv=170, nh=3000, T=700.0, Ea_O=0.6,
         Ea_H=0.45),
    Case((38, 37, 36), (18, 18, 18), seed=41, lattice_id=3, nv=760, nh=9000, T=600.0, Ea_O=0.6,
         Ea_H=0.45, E_z=1e8),
    Case((27, 21, 22), (20, 20, 20), seed=41, lattice_id=4, nv=190, nh=0, T=650.0, Ea_O=0.55,
         gb_period=10, gb_mask=4, gb_dE=0.1),
    Case((43, 40, 41), (20, 20, 20), seed=41, lattice_id=5, nv=1060, nh=6000, T=680.0, Ea_O=0.6,
         Ea_H=0.45),
    Case((25, 26, 24), (24, 24, 24), seed=41, lattice_id=6, nv=230, nh=2500, T=640.0, Ea_O=0.6,
         Ea_H=0.45, E_z=3e7),
    Case((50, 49, 48), (24, 24, 24), seed=41, lattice_id=7, nv=1760, nh=18000, T=600.0, Ea_O=0.6,
         Ea_H=0.45, gb_period=12, gb_mask=3, gb_dE=0.05),
]


@pytest.mark.parametrize("schedule,group", [("lockstep", 0), ("lockstep", 8), ("lockstep", 4),
                                            ("lockstep", 2), ("lockstep", 1), ("persistent", 0),
                                            ("persistent", 8), ("persistent", 4),
                                            ("persistent", 1)])
def test_wide_fragment_edges_match_oracle(schedule, group):
    """Sub-blocks of 7 to 13 cells (the wide fragment edges the autotuner
    can pick), held in LDS or staged, under both schedules and every tile
    group (0 = the library's own choice): the oracle's trajectories bit for
    bit over two calls (a cycle count, then a hop target)."""
    say("wide fragment edges", schedule, group)
    lats = [c.oracle() for c in WIDE_CASES]
    ts = [1.2 / (8.0 * l.k12[0]) for l in lats]
    g = gpu_set(WIDE_CASES)
    g.set_schedule(schedule, 4)
    g.set_group(group)
    for max_cycles, min_hops in ((2, 0), (10**6, 3000)):
        for lat, t in zip(lats, ts):
            lat.advance(t, max_cycles=max_cycles, min_hops=min_hops)
        g.advance(ts, max_cycles=max_cycles, min_hops=min_hops)
        stats = g.read_stats()
        if schedule == "persistent":
            res = [bool(s["lds_resident"]) for s in stats]
            assert res == [True, False] * 4, res
        for i, lat in enumerate(lats):
            what = "%s/%d member %d %s F=%d" % (schedule, group, i, WIDE_CASES[i].L, WIDE_CASES[i].frag[0])
            assert stats[i]["cycles"] == lat.cycles and stats[i]["t"] == lat.t, what
            assert stats[i]["hops"].tolist() == [int(x) for x in lat.hops], what
            assert_same_state(g, i, lat, what)


def test_transfers_larger_than_one_stage_chunk():
    """A lattice of 540,000 sites (more than the 2^19 sites one staging
    chunk of the work buffer holds): caller occupancy in, read back
    unchanged; two cycles equal the oracle's; a checkpoint restored into a
    fresh set continues identically."""
    say("chunked transfers, 540,000 sites")
    from paper_2004_09081_amd import fkmc as F
    c = Case((60, 60, 50), (15, 15, 10), seed=51, lattice_id=2, nv=0, nh=0, T=650.0, Ea_O=0.6,
             Ea_H=0.45, E_z=1e8)
    lat = c.oracle()
    n = lat.g.n_sites
    assert n > (1 << 19)
    rng = np.random.default_rng(52)
    occ = np.zeros(n, np.int8)
    idx = rng.choice(n, 3300, replace=False)
    occ[idx[:1100]] = 2
    occ[idx[1100:]] = 1
    lat.occ[:] = occ
    lat.disp[:] = 0
    raw = O.rate_raw(O.RateParams(**c.rp), lat.g.a_angstrom)
    lat.k12, _, _ = O.quantise(raw, 8 * min(1100, O.max_domain_sites(lat.g)))
    g = F.LatticeSet([c.gpu_geometry()])
    g.set_occupancy(0, occ)
    back, disp0 = g.read_state(0)
    assert np.array_equal(back, occ) and not disp0.any()
    g.set_rate_table(0, raw)
    t_sync = 1.5 / (8 * lat.k12[0])
    lat.advance(t_sync, max_cycles=2)
    g.advance([t_sync], max_cycles=2)
    assert_same_state(g, 0, lat, "chunked set_occupancy")
    blob = g.checkpoint(0)
    h = F.LatticeSet([c.gpu_geometry()])
    h.init_random([0], [0])
    h.restore(0, blob)
    for s in (g, h):
        s.advance([t_sync], max_cycles=1)
    lat.advance(t_sync, max_cycles=1)
    assert_same_state(h, 0, lat, "restored from checkpoint")
    assert_same_state(g, 0, lat, "uninterrupted")


# Voronoi grain boundaries as a site map (the micro-scale model's grains):
# fragment lattices held in LDS and staged, a plain lattice (HBM kernel)
VORONOI_CASES = [
    (Case((18, 16, 20), (6, 6, 6), seed=81, lattice_id=0, nv=60, nh=300, T=650.0, Ea_O=0.6, Ea_H=0.45,
          E_z=2e8, gb_dE=0.2), 6),
    (Case((34, 32, 30), (8, 8, 8), seed=81, lattice_id=1, nv=200, nh=0, T=600.0, Ea_O=0.55, E_z=1e8,
          gb_dE=0.2), 10),
    (Case((12, 10, 14), (12, 10, 14), seed=81, lattice_id=2, nv=20, nh=40, T=650.0, Ea_O=0.6, Ea_H=0.45,
          gb_dE=0.15), 3),
    (Case((10, 9, 11), seed=81, lattice_id=3, nv=30, nh=60, T=650.0, Ea_O=0.6, Ea_H=0.45, E_z=1e8,
          gb_dE=0.2), 4),
]


def _voronoi_oracle(c, n_grains):
    from paper_2004_09081_amd import workloads as W
    gmap = W.voronoi_boundary_map(c.L, n_grains, 1.0, c.lattice_id)
    g = O.Geometry(L=c.L, frag=c.frag, a_angstrom=c.a, seed=c.seed, lattice_id=c.lattice_id, gb_map=gmap)
    lat = O.Lattice(g)
    lat.init_random(c.nv, c.nh)
    lat.set_rates(O.RateParams(**c.rp))
    return lat, gmap


@pytest.mark.parametrize("schedule,group", [("lockstep", 0), ("persistent", 0), ("persistent", 8),
                                            ("persistent", 1)])
def test_voronoi_boundary_map_matches_oracle(schedule, group):
    """Grain boundaries from a Voronoi site map (barrier +gb_dE on every
    edge touching a boundary site) under both schedules and several tile
    groups, resident and staged fragments, one fragment, and plain BKL: the
    oracle's trajectories bit for bit."""
    say("Voronoi boundary map", schedule, group)
    cases = [c for c, _ in VORONOI_CASES]
    pairs = [_voronoi_oracle(c, n) for c, n in VORONOI_CASES]
    g = gpu_set(cases)
    for i, (_, gmap) in enumerate(pairs):
        g.set_gb_map(i, gmap)
    g.set_schedule(schedule, 4)
    g.set_group(group)
    ts = [0.0 if c.frag[0] == 0 else 1.3 / (8.0 * lat.k12[0]) for c, (lat, _) in zip(cases, pairs)]
    for max_cycles, min_hops in ((3, 0), (10**6, 1500)):
        # (plain members make exactly min_hops hops)
        for c, (lat, _), t in zip(cases, pairs, ts):
            if c.frag[0] == 0:
                lat.advance_plain(min_hops)
            else:
                lat.advance(t, max_cycles=max_cycles, min_hops=min_hops)
        g.advance(ts, max_cycles=max_cycles, min_hops=min_hops)
        st = g.read_stats()
        for i, (lat, _) in enumerate(pairs):
            what = "voronoi member %d %s" % (i, cases[i].L)
            assert st[i]["t"] == lat.t and st[i]["hops"].tolist() == [int(x) for x in lat.hops], what
            assert_same_state(g, i, lat, what)
