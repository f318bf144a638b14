"""Pins of the oracle's primitives against things other than itself:
a library Philox, libm/mpmath logarithms, real-space geometry, CODATA
constants, the exactness property of the quantised rates, and the
uniformity of the initial placement."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from oracle import gen_ln_constants
from tests import brute

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------------------- Philox
@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("rr") / "philox_rr")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-o", exe,
                           os.path.join(HERE, "philox_rocrand.cpp")], cwd="/tmp")
    return exe


def test_philox_matches_rocrand(rocrand_philox):
    """Philox4x32-10 outputs equal rocRAND's host engine for random and
    extreme counters/keys (Salmon et al., SC'11 generator)."""
    rng = np.random.default_rng(1234)
    cases = [[0] * 6, [2**32 - 1] * 6, [1, 2, 3, 4, 5, 6], [0, 0, 0xFFFFFFFF, 3, 0, 0]]
    cases += rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64).tolist()
    inp = "\n".join(" ".join(str(int(x)) for x in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_philox], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        ref = [int(x) for x in line.split()]
        got = O.philox(c[:4], c[4:]).tolist()
        assert got == ref, (c, got, ref)


# ----------------------------------------------------------------------------- ln
def _ulp_err(x, ref):
    return abs(x - ref) / math.ulp(ref) if ref != 0 else abs(x)


def test_philox_known_answer_vectors():
    """Published Philox4x32-10 test vectors (tests/golden/philox4x32_10_kat.txt)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    n = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        got = O.philox(tuple(v[0:4]), tuple(v[4:6]))
        assert [int(x) for x in got] == v[6:10], line
        n += 1
    assert n == 3


def test_ln_constants_match_mpmath():
    assert O.ln_constants() == gen_ln_constants.constants()


def test_ln_accuracy_against_mpmath_and_libm():
    """The oracle's ln (Cody-Waite + atanh series) is within 1 ulp of the
    correctly rounded log on the clock's whole input set u = m 2^-53."""
    import mpmath
    mpmath.mp.prec = 120
    rng = np.random.default_rng(7)
    m = rng.integers(1, 2**53 + 1, size=4000, dtype=np.uint64)
    us = [float(int(v)) * 2.0**-53 for v in m]
    us += [1.0, 2.0**-53, 0.5, 0.75, 1.0 - 2.0**-53, math.sqrt(0.5), 2.0**-26,
           math.nextafter(math.sqrt(0.5), 0), math.nextafter(math.sqrt(0.5), 1)]
    worst = 0.0
    for u in us:
        got = O.ln(u)
        if u == 1.0:
            assert got == 0.0
            continue
        ref = float(mpmath.log(mpmath.mpf(u)))
        worst = max(worst, _ulp_err(got, ref))
        assert _ulp_err(got, math.log(u)) <= 1.0
    assert worst <= 1.0, worst


# ----------------------------------------------------------------------------- geometry
@pytest.mark.parametrize("L", [(2, 2, 2), (3, 2, 4), (5, 3, 2)])
def test_hops_match_real_space_neighbours(L):
    """Every site has exactly 8 neighbours at a/sqrt(2); the oracle's hop
    targets are exactly those sites, with the same displacement vectors."""
    nb = brute.neighbours(L)
    g = O.Geometry(L=L)
    H = O.hop_table()
    for n, (_, _, t, _) in enumerate(brute.sites(L)):
        assert len(nb[n]) == 8
        ref = {m: tuple(np.round(2 * d).astype(int)) for m, d in nb[n]}
        got = {}
        for d in range(8):
            m = O.hop_target(g, n, d)
            got[m] = tuple(H[t, d])
        assert got == ref


def test_hop_order_lexicographic():
    H = O.hop_table()
    for t in range(3):
        rows = [tuple(r) for r in H[t]]
        assert rows == sorted(rows)
        # type-2 sites (even z) always change z; types 0 and 1 have four
        # in-plane hops
        nz = sorted(r[2] for r in rows)
        if t == 2:
            assert nz == [-1] * 4 + [1] * 4
        else:
            assert nz == [-1, -1, 0, 0, 0, 0, 1, 1]


# ----------------------------------------------------------------------------- rates
def test_rate_constant_and_arrhenius():
    """No field, no boundary: every O hop has nu exp(-Ea/(kB T)) with kB from
    scipy's CODATA constants (k/e)."""
    from scipy import constants as sc
    kB = sc.k / sc.e
    p = O.RateParams(nu=1e13, T=600.0, Ea_O=0.6, Ea_H=0.25)
    k = O.rate_raw(p, 3.905).reshape(2, 3, 2)
    assert np.allclose(k[0], 1e13 * math.exp(-0.6 / (kB * 600.0)), rtol=1e-12, atol=0)
    assert np.allclose(k[1], 1e13 * math.exp(-0.25 / (kB * 600.0)), rtol=1e-12, atol=0)


def test_rate_field_detailed_balance_and_boundary():
    """With a field the up/down ratio is exp(q E a /(2 kB T)) (the vacancy's
    energy falls by q E a/2 per up hop), symmetric about the flat hop; the
    boundary flag multiplies by exp(-dE_gb/(kB T))."""
    from scipy import constants as sc
    kB = sc.k / sc.e
    T, E, q, a = 450.0, 1e7, 2.0, 3.905
    p = O.RateParams(nu=1e13, T=T, Ea_O=0.75, E_z=E, q=q, gb_dE=0.3)
    k = O.rate_raw(p, a).reshape(2, 3, 2)
    up, flat, down = k[0, 2, 0], k[0, 1, 0], k[0, 0, 0]
    assert up > flat > down
    assert math.isclose(up / down, math.exp(q * E * a * 1e-10 / (2 * kB * T)), rel_tol=1e-12)
    assert math.isclose(up * down, flat * flat, rel_tol=1e-12)
    assert math.isclose(k[0, 1, 1] / k[0, 1, 0], math.exp(-0.3 / (kB * T)), rel_tol=1e-12)


def test_quantised_rates_sum_exactly_in_any_order():
    p = O.RateParams(nu=1e13, T=600.0, Ea_O=0.7, Ea_H=0.25, E_z=1e7, q=2.0, gb_dE=0.3)
    raw = O.rate_raw(p, 3.905)
    n_ev = 8 * 1000
    k, q, rel = O.quantise(raw, n_ev)
    assert q > 0 and math.log2(q) == int(math.log2(q))
    assert np.all(k / q == np.rint(k / q))
    assert n_ev * k.max() <= 2.0**53 * q
    assert rel <= 2.0**-10
    assert np.all(np.abs(k - raw) <= 0.5 * q)
    rng = np.random.default_rng(3)
    for _ in range(50):
        vals = k[rng.integers(0, 12, size=n_ev)]
        s1 = 0.0
        for v in vals:
            s1 += v
        s2 = 0.0
        for v in vals[::-1]:
            s2 += v
        assert s1 == s2 == math.fsum(vals)


def test_quantise_rejects_rate_below_floor():
    raw = np.array([1.0, 1e-30] + [0.0] * 10)
    with pytest.raises(ValueError):
        O.quantise(raw, 8)


# ----------------------------------------------------------------------------- init
def test_init_exact_counts_and_uniformity():
    """Exactly n_V vacancies and n_H H; every site equally likely to hold a
    vacancy (chi-square over 3000 independent keys)."""
    L = (2, 2, 2)
    N = 24
    cnt_v = np.zeros(N)
    cnt_h = np.zeros(N)
    R = 3000
    for s in range(R):
        lat = O.Lattice(O.Geometry(L=L, seed=s, lattice_id=11))
        lat.init_random(3, 5)
        assert (lat.occ == 2).sum() == 3 and (lat.occ == 1).sum() == 5
        cnt_v += lat.occ == 2
        cnt_h += lat.occ == 1
    _, p_v = brute.chi2_pvalue(cnt_v, np.full(N, 1 / N))
    _, p_h = brute.chi2_pvalue(cnt_h, np.full(N, 1 / N))
    assert p_v > 1e-4 and p_h > 1e-4


def test_init_distinct_keys_differ():
    a = O.Lattice(O.Geometry(L=(4, 4, 4), seed=0, lattice_id=0))
    b = O.Lattice(O.Geometry(L=(4, 4, 4), seed=0, lattice_id=1))
    a.init_random(10, 10)
    b.init_random(10, 10)
    assert not np.array_equal(a.occ, b.occ)


# ----------------------------------------------------------------------------- decomposition
GEOMS = [((4, 4, 4), (4, 4, 4)), ((8, 6, 5), (4, 3, 5)), ((7, 5, 9), (3, 4, 4)),
         ((2, 2, 2), (2, 2, 2)), ((6, 6, 6), (2, 2, 2))]


@pytest.mark.parametrize("L,F", GEOMS)
def test_decomposition_partitions_edges(L, F):
    """Sub-blocks tile the lattice; every hop edge is active in exactly one
    (fragment, colour) tile; each footprint holds both ends of its active
    edges; same-colour footprints are disjoint; the footprint size is the
    sub-block plus one face of type-a sites on each +a side."""
    g = O.Geometry(L=L, frag=F)
    nf = O.Lattice(g).n_fragments
    N = g.n_sites
    owner_count = {}
    cells = np.zeros(L[::-1], int)
    for c in range(8):
        used = np.zeros(N, bool)
        for f in range(nf):
            lo, hi = O.sub_block(g, f, c)
            w = [hi[a] - lo[a] for a in range(3)]
            cells[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += 1
            fp = set(O.footprint_sites(g, f, c).tolist())
            assert len(fp) == 3 * w[0] * w[1] * w[2] + w[1] * w[2] + w[2] * w[0] + w[0] * w[1]
            assert not used[list(fp)].any()
            used[list(fp)] = True
            for s in fp:
                for d in range(8):
                    if O.edge_active(g, s, d, f, c):
                        tgt = O.hop_target(g, s, d)
                        assert tgt in fp
                        key = (min(s, tgt), max(s, tgt))
                        owner_count[key] = owner_count.get(key, 0) + 1
    assert np.all(cells == 1)
    # each undirected edge seen from both ends, in exactly one tile
    assert len(owner_count) == N * 8 // 2
    assert set(owner_count.values()) == {2}
