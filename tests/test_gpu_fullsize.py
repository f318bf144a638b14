"""Parity at the full size of the biased 600^3 workload (6.48e8 sites,
16^3-cell fragments, boundary planes, field): the whole initial occupancy
against the oracle, then one phase of colour 0 on the GPU against the oracle
run on a sample of fragments (their footprints are touched by no other tile
of that phase), plus invariants over the whole lattice."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.common import say

pytestmark = pytest.mark.gpu


def footprint_index(L, lo, hi):
    """Canonical indices of the footprint of sub-block [lo, hi): its cells'
    sites plus the type-a sites of the next cell layer along +a."""
    Lx, Ly, Lz = L
    xs, ys, zs = [np.arange(lo[a], hi[a]) for a in range(3)]
    def idx(i, j, k, t):
        return ((k * Ly + j) * Lx + i) * 3 + t
    I, J, K = np.meshgrid(xs, ys, zs, indexing="ij")
    own = np.concatenate([idx(I, J, K, t).ravel() for t in range(3)])
    J2, K2 = np.meshgrid(ys, zs, indexing="ij")
    fx = idx(hi[0] % Lx, J2, K2, 0).ravel()
    I2, K2 = np.meshgrid(xs, zs, indexing="ij")
    fy = idx(I2, hi[1] % Ly, K2, 1).ravel()
    I2, J2 = np.meshgrid(xs, ys, indexing="ij")
    fz = idx(I2, J2, hi[2] % Lz, 2).ravel()
    return np.concatenate([own, fx, fy, fz]).astype(np.int64)


def test_full_size_biased_lattice_init_and_phase():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_09081_amd import fkmc as F
    from paper_2004_09081_amd import workloads as W
    sp = W.cfg3()
    say("full size: init", sp.L, sp.n_vac)
    geoms, rates = W.to_gpu([sp], F)
    g = F.LatticeSet(geoms)
    g.init_random([sp.n_vac], [sp.n_h])
    g.set_rates(rates)
    og = O.Geometry(L=sp.L, frag=sp.frag, a_angstrom=sp.a, seed=sp.seed, lattice_id=sp.lattice_id,
                    gb_period_cells=sp.gb_period, gb_axes_mask=sp.gb_mask)
    lat = O.Lattice(og)
    lat.init_random(sp.n_vac, sp.n_h)
    occ0, _ = g.read_state(0, with_disp=False)
    assert np.array_equal(occ0, lat.occ), "initial occupancy differs"
    lat.set_rates(O.RateParams(T=sp.T, Ea_O=sp.Ea_O, Ea_H=sp.Ea_H, E_z=sp.E_z, q=sp.q,
                               gb_period_cells=sp.gb_period, gb_axes_mask=sp.gb_mask,
                               gb_dE=sp.gb_dE))
    assert g.get_rate_table(0).tobytes() == lat.k12.tobytes()
    say("full size: phase 0")
    g.run_phase([sp.t_sync], 0)
    occ1, disp1 = g.read_state(0)
    nf = lat.n_fragments
    rng = np.random.default_rng(11)
    sample = np.concatenate([[0, nf - 1], rng.choice(nf, 62, replace=False)])
    moved = 0
    for f in sample:
        lat.phase(sp.t_sync, 0, 0, int(f))
        lo, hi = O.sub_block(og, int(f), 0)
        fp = footprint_index(sp.L, lo, hi)
        assert np.array_equal(occ1[fp], lat.occ[fp]), "fragment %d occupancy" % f
        assert np.array_equal(disp1[fp], lat.disp[fp]), "fragment %d displacement" % f
        moved += int((lat.disp[fp] != 0).any(axis=1).sum())
    assert moved > 0
    # whole-lattice invariants: species conserved, displacements sum to zero
    assert np.bincount(occ1, minlength=3).tolist() == np.bincount(occ0, minlength=3).tolist()
    assert disp1.astype(np.int64).sum(axis=0).tolist() == [0, 0, 0]
    st = g.read_stats()[0]
    assert int(st["hops"].sum()) > 0 and st["count"][2] == sp.n_vac


def _oracle_of(sp):
    og = O.Geometry(L=sp.L, frag=sp.frag, a_angstrom=sp.a, seed=sp.seed, lattice_id=sp.lattice_id,
                    gb_period_cells=sp.gb_period, gb_axes_mask=sp.gb_mask)
    lat = O.Lattice(og)
    lat.init_random(sp.n_vac, sp.n_h)
    lat.set_rates(O.RateParams(T=sp.T, Ea_O=sp.Ea_O, Ea_H=sp.Ea_H, E_z=sp.E_z, q=sp.q,
                               gb_period_cells=sp.gb_period, gb_axes_mask=sp.gb_mask,
                               gb_dE=sp.gb_dE))
    return lat


def _run_ensemble_and_check(specs, sample, what):
    """The 512 lattices in the launch the benchmark times (one persistent
    launch per call, 4 wavefronts per workgroup, plain lattices held in LDS
    in the same launch, the second call in the launch order derived from the
    first call's device times); two calls of 1e5 hops per lattice (the
    benchmark's step is 1e6).  Every lattice conserves its species and a
    zero displacement sum; the sampled lattices equal the oracle's bit for
    bit."""
    from paper_2004_09081_amd import fkmc as F
    from paper_2004_09081_amd import workloads as W
    say(what, "samples", sample, "edges", sorted({specs[i].frag[0] for i in sample}))
    geoms, rates = W.to_gpu(specs, F)
    g = F.LatticeSet(geoms)
    g.init_random([sp.n_vac for sp in specs], [sp.n_h for sp in specs])
    g.set_rates(rates)
    g.set_schedule("auto", 4)
    ts = [sp.t_sync for sp in specs]
    H = 100_000
    for call in range(2):
        g.advance(ts, max_cycles=10**9, min_hops=H)
    st = g.read_stats()
    for i, s in enumerate(st):
        sp = specs[i]
        assert s["count"].tolist() == [3 * sp.L[0] ** 3 - sp.n_vac - sp.n_h, sp.n_h, sp.n_vac]
        assert s["sum_r"].sum(axis=0).tolist() == [0, 0, 0]
        assert int(s["hops"].sum()) >= 2 * H
    for i in sample:
        sp = specs[i]
        say("  oracle for lattice", i, sp.L, sp.frag, sp.n_vac, sp.n_h)
        lat = _oracle_of(sp)
        for call in range(2):
            if sp.frag[0] == 0:
                lat.advance_plain(H)
            else:
                lat.advance(sp.t_sync, max_cycles=10**9, min_hops=H)
        s = st[i]
        assert s["cycles"] == lat.cycles and s["t"] == lat.t, i
        assert s["hops"].tolist() == [int(x) for x in lat.hops], i
        occ, disp = g.read_state(i)
        assert np.array_equal(occ, lat.occ), "lattice %d occupancy" % i
        assert np.array_equal(disp, lat.disp), "lattice %d displacement" % i
    g.close()
    return st


def _one_per_edge(specs):
    """For every fragment edge in use, its lattice with the fewest sites
    (the oracle's cost)."""
    best = {}
    for i, sp in enumerate(specs):
        e = sp.frag[0]
        if e not in best or sp.n_sites < specs[best[e]].n_sites:
            best[e] = i
    return [best[e] for e in sorted(best)]


def test_full_ensemble_every_candidate_edge_matches_oracle():
    """Every decomposition the autotuner can choose, assigned round-robin
    over the 512 ensemble lattices (edges 4-24 cells, the whole lattice
    where sparse, unfragmented in LDS where it fits), with one sampled
    lattice per edge plus a resident, an HBM-staged and a crowded one."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_09081_amd import workloads as W
    from paper_2004_09081_amd.autotune import DEFAULT_CANDIDATES
    specs = W.cfg4(n=512, hops=10**6, frag=8)
    for i, sp in enumerate(specs):
        c = DEFAULT_CANDIDATES[i % len(DEFAULT_CANDIDATES)]
        sp.frag = (int(c(sp)) if callable(c) else int(c),) * 3
        if sp.frag[0] == 0:
            sp.t_sync = 0.0
    frag = [i for i, sp in enumerate(specs) if sp.frag[0] > 0]
    i_res = next(i for i in frag if specs[i].L[0] <= 20)
    i_stream = next(i for i in frag if 30 <= specs[i].L[0] <= 34 and specs[i].n_vac < 400)
    i_dense = max((i for i in frag if specs[i].L[0] <= 30),
                  key=lambda i: specs[i].extra["x_v"] * specs[i].frag[0] ** 3)
    sample = sorted(set(_one_per_edge(specs) + [i_res, i_stream, i_dense]))
    edges = {sp.frag[0] for sp in specs}
    assert edges >= {0, 4, 6, 8, 10, 12, 14, 16, 18, 20, 24}, edges
    st = _run_ensemble_and_check(specs, sample, "full ensemble, every candidate edge:")
    assert any(s["lds_resident"] and specs[i].frag[0] == 0 for i, s in enumerate(st))
    assert any(not s["lds_resident"] for s in st)
    groups = {s["tile_group"] for i, s in enumerate(st) if specs[i].frag[0] > 0}
    assert groups >= {1, 4, 8}, groups


def test_full_ensemble_benchmark_decomposition_matches_oracle():
    """The decomposition the benchmark runs by default (the autotuner's
    per-lattice edges, stored with the package), one sampled lattice per
    edge it uses plus the largest lattice of the most common edge."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_09081_amd import autotune
    from paper_2004_09081_amd import workloads as W
    specs = W.cfg4(n=512, hops=10**6, frag=8)
    edges = autotune.load_edges(autotune.ENSEMBLE_EDGES, specs)
    if edges is None:
        pytest.skip("no stored decomposition for this ensemble")
    for sp, e in zip(specs, edges):
        sp.frag = (int(e),) * 3
        if e == 0:
            sp.t_sync = 0.0
    sample = _one_per_edge(specs)
    common = max(set(edges.tolist()), key=edges.tolist().count)
    sample.append(max((i for i in range(len(specs)) if edges[i] == common),
                      key=lambda i: specs[i].n_sites))
    _run_ensemble_and_check(specs, sorted(set(sample)), "full ensemble, benchmark decomposition:")


def test_atom_selection_on_ensemble_lattices_matches_oracle():
    """The atom-selection scheme (Eqs. AtomP and TimeStepFrg) in the
    benchmark's configuration: every ensemble lattice held in LDS
    unfragmented, 64 selections per stage, one launch of 20,000 stages;
    three sampled lattices (fewest, median and most vacancies) equal the
    oracle's bit for bit."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import copy
    from paper_2004_09081_amd import fkmc as F
    from paper_2004_09081_amd import workloads as W
    from paper_2004_09081_amd.autotune import plain_if_sparse
    sel = []
    for sp in W.cfg4(n=512, hops=10**6, frag=8):
        if plain_if_sparse(sp) == 0:
            q = copy.copy(sp)
            q.frag = (0, 0, 0)
            sel.append(q)
    order = sorted(range(len(sel)), key=lambda i: sel[i].n_vac)
    sample = [order[0], order[len(order) // 2], order[-1]]
    say("atom selection on %d ensemble lattices, samples" % len(sel), sample)
    geoms, rates = W.to_gpu(sel, F)
    g = F.LatticeSet(geoms)
    g.init_random([sp.n_vac for sp in sel], [sp.n_h for sp in sel])
    g.set_rates(rates)
    g.advance_atomic(64, 20000)
    st = g.read_stats()
    for i in sample:
        sp = sel[i]
        say("  oracle for lattice", sp.lattice_id, sp.L, sp.n_vac)
        lat = _oracle_of(sp)
        lat.advance_atomic(64, 20000)
        assert st[i]["draws"] == lat.draws and st[i]["t"] == lat.t, i
        assert st[i]["hops"].tolist() == [int(x) for x in lat.hops], i
        occ, disp = g.read_state(i)
        assert np.array_equal(occ, lat.occ), "lattice %d occupancy" % sp.lattice_id
        assert np.array_equal(disp, lat.disp), "lattice %d displacement" % sp.lattice_id


def test_atom_selection_past_lds_matches_oracle():
    """The atom-selection scheme on the lattices the persistent kernel does
    not hold in LDS, in the benchmark's configuration: every ensemble
    lattice of at most 8192 vacancies among them, unfragmented, 64
    selections per stage, one call of 2,000 stages (most run with their
    occupancy in HBM); three sampled lattices (fewest, median and most
    vacancies) equal the oracle's bit for bit."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import copy
    from paper_2004_09081_amd import fkmc as F
    from paper_2004_09081_amd import workloads as W
    from paper_2004_09081_amd.autotune import plain_if_sparse
    sel = []
    for sp in W.cfg4(n=512, hops=10**6, frag=8):
        if plain_if_sparse(sp) != 0 and sp.n_vac <= 8192:
            q = copy.copy(sp)
            q.frag = (0, 0, 0)
            sel.append(q)
    order = sorted(range(len(sel)), key=lambda i: sel[i].n_vac)
    sample = [order[0], order[len(order) // 2], order[-1]]
    say("atom selection on %d ensemble lattices past the LDS, samples" % len(sel), sample)
    geoms, rates = W.to_gpu(sel, F)
    g = F.LatticeSet(geoms)
    g.init_random([sp.n_vac for sp in sel], [sp.n_h for sp in sel])
    g.set_rates(rates)
    g.advance_atomic(64, 2000)
    st = g.read_stats()
    assert sum(1 for x in st if not x["lds_resident"]) > 300
    for i in sample:
        sp = sel[i]
        say("  oracle for lattice", sp.lattice_id, sp.L, sp.n_vac)
        lat = _oracle_of(sp)
        lat.advance_atomic(64, 2000)
        assert st[i]["draws"] == lat.draws and st[i]["t"] == lat.t, i
        assert st[i]["hops"].tolist() == [int(x) for x in lat.hops], i
        occ, disp = g.read_state(i)
        assert np.array_equal(occ, lat.occ), "lattice %d occupancy" % sp.lattice_id
        assert np.array_equal(disp, lat.disp), "lattice %d displacement" % sp.lattice_id
