"""Host-side checks of the C-ABI library that need no GPU: every declared
symbol is exported, and the host logic (rate tables, quantisation, domain
sizes, buffer sizes, argument checks) agrees with the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def F():
    from paper_2004_09081_amd import fkmc
    if not os.path.exists(fkmc.LIB_PATH):
        from paper_2004_09081_amd import build
        build.build()
    return fkmc


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "fkmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fkmc_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(F):
    syms = declared_symbols()
    assert len(syms) >= 20
    lib = C.CDLL(F.LIB_PATH)
    for s in syms:
        assert hasattr(lib, s), s
    from paper_2004_09081_amd import surrogate
    bound = set(F._SIGS) | set(surrogate._SIGS) | {"fkmc_mlp_param_count"}
    assert set(syms) == bound, "binding and header disagree: %s" % (set(syms) ^ bound)


@pytest.mark.parametrize("T,E,gb,Eh", [(600.0, 0.0, 0.0, 0.25), (450.0, 1e7, 0.3, 0.25),
                                       (300.0, 0.0, 0.0, 0.25), (900.0, 5e8, 0.2, 0.4),
                                       (800.0, -3e8, 0.0, 0.25)])
@pytest.mark.parametrize("n_ev", [8, 8 * 1659, 8 * 5000, 8 * 648000])
def test_rate_table_matches_oracle_bitwise(F, T, E, gb, Eh, n_ev):
    p = O.RateParams(nu=1e13, T=T, Ea_O=0.75, Ea_H=Eh, E_z=E, q=2.0, gb_dE=gb)
    raw_o = O.rate_raw(p, 3.905)
    try:
        k_o, q_o, rel_o = O.quantise(raw_o, n_ev)
        ok = True
    except ValueError:
        ok = False
    gp = F.RateParams.make(nu=1e13, T=T, Ea_O=0.75, Ea_H=Eh, E_z=E, q=2.0, gb_dE=gb)
    if not ok:
        with pytest.raises(F.FkmcError):
            F.rate_table_host(gp, 3.905, n_ev)
        return
    raw, k, q, rel = F.rate_table_host(gp, 3.905, n_ev)
    assert raw.tobytes() == raw_o.tobytes()
    assert k.tobytes() == k_o.tobytes()
    assert q == q_o and rel == rel_o


@pytest.mark.parametrize("L,Fr", [((8, 8, 8), (0, 0, 0)), ((48, 48, 48), (12, 12, 12)),
                                  ((600, 600, 600), (16, 16, 16)), ((7, 9, 5), (3, 4, 5)),
                                  ((10, 10, 10), (3, 3, 3)), ((4, 4, 4), (8, 8, 8))])
def test_domain_sites_match_oracle(F, L, Fr):
    g = F.Geometry.make(L, Fr)
    assert F.max_domain_sites(g) == O.max_domain_sites(O.Geometry(L=L, frag=Fr))


def test_domain_sites_brute_force(F):
    for L, Fr in [((7, 5, 9), (3, 4, 4)), ((6, 6, 6), (2, 2, 2)), ((5, 4, 3), (5, 4, 3))]:
        og = O.Geometry(L=L, frag=Fr)
        nf = O.Lattice(og).n_fragments
        best = max(len(O.footprint_sites(og, f, c)) for f in range(nf) for c in range(8))
        assert F.max_domain_sites(F.Geometry.make(L, Fr)) == best


def test_query_sizes_and_argument_checks(F):
    g = F.Geometry.make((600, 600, 600), (16, 16, 16))
    occ, disp, work = F.query_sizes([g])
    assert occ >= 648_000_000 and disp >= 16 * 648_000_000 and work > 0
    with pytest.raises(F.FkmcError) as e:
        F.query_sizes([F.Geometry.make((1, 4, 4), (0, 0, 0))])
    assert e.value.code == -1
    with pytest.raises(F.FkmcError):
        F.query_sizes([F.Geometry.make((8, 8, 8), (4, 0, 4))])
    with pytest.raises(F.FkmcError):
        F.rate_table_host(F.RateParams.make(T=-1.0), 3.905, 8)


def test_library_allocates_no_device_memory():
    """Device memory belongs to the caller: no library source allocates or
    frees device memory (canonical-order transfers stage through the work
    buffer)."""
    csrc = os.path.join(ROOT, "paper_2004_09081_amd", "csrc")
    pat = re.compile(r"\b(hipMalloc|hipMallocAsync|hipMallocManaged|hipExtMallocWithFlags|hipFree|"
                     r"hipFreeAsync|hipMallocPitch|hipMalloc3D|hipMallocArray)\s*\(")
    for name in sorted(os.listdir(csrc)):
        text = open(os.path.join(csrc, name)).read()
        text = re.sub(r"//[^\n]*", "", re.sub(r"/\*.*?\*/", "", text, flags=re.S))
        assert not pat.search(text), "%s allocates device memory: %s" % (name, pat.search(text).group(0))
