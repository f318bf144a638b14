"""The entry point that allocates nothing (fkmc_create_static: the work
space is the library's static per-device array) against the ordinary one
(fkmc_create with a caller work buffer), bit for bit, on two handles in a
row, the second over a smaller set; plus its refusals."""
import numpy as np
import pytest

from tests.common import Case, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_09081_amd import fkmc
    fkmc.lib()
    return fkmc


BIG = [Case((30, 30, 28), (6, 6, 7), seed=61, lattice_id=0, nv=150, nh=600, T=700.0, Ea_O=0.6,
            Ea_H=0.45),
       Case((16, 16, 16), (8, 8, 8), seed=61, lattice_id=1, nv=40, nh=0, T=600.0, gb_period=4,
            gb_dE=0.1),
       Case((10, 9, 8), seed=61, lattice_id=2, nv=60, nh=100, T=650.0, Ea_O=0.6, Ea_H=0.45),
       Case((12, 10, 11), seed=61, lattice_id=3, nv=600, nh=200, T=650.0, Ea_O=0.6, Ea_H=0.45,
            E_z=1e8)]
SMALL = [Case((8, 8, 8), (4, 4, 4), seed=62, lattice_id=0, nv=12, nh=20, T=650.0, Ea_O=0.6,
              Ea_H=0.45),
         Case((6, 5, 7), seed=62, lattice_id=1, nv=9, nh=30, T=600.0, Ea_O=0.6, Ea_H=0.45)]


def _make(F, cases, static):
    s = F.LatticeSet([c.gpu_geometry() for c in cases], static_work=static)
    s.init_random([c.nv for c in cases], [c.nh for c in cases])
    s.set_rates([c.gpu_rates() for c in cases])
    return s


def _run(s, cases, schedule):
    ts = [0.0 if c.frag[0] == 0 else 1.5 / (8.0 * s.get_rate_table(i)[0]) for i, c in enumerate(cases)]
    s.set_schedule(schedule, 4)
    s.advance(ts, max_cycles=3, min_hops=700)
    s.advance(ts, max_cycles=10**6, min_hops=900)
    return s.read_stats()


@pytest.mark.parametrize("schedule", ["lockstep", "persistent"])
def test_static_work_space_equals_caller_buffer(F, schedule):
    for cases in (BIG, SMALL):
        say("no-alloc entry point", schedule, len(cases), "lattices")
        a = _make(F, cases, False)
        b = _make(F, cases, True)
        sa, sb = _run(a, cases, schedule), _run(b, cases, schedule)
        for i in range(len(cases)):
            for k in ("t", "cycles", "draws"):
                assert sa[i][k] == sb[i][k], (i, k)
            assert sa[i]["hops"].tolist() == sb[i]["hops"].tolist()
            assert sa[i]["sum_r"].tolist() == sb[i]["sum_r"].tolist()
            oa, da = a.read_state(i)
            ob, db = b.read_state(i)
            assert np.array_equal(oa, ob) and np.array_equal(da, db), i
        assert int(sum(x["hops"].sum() for x in sb)) > 0
        a.close()
        b.close()


def test_static_work_space_refusals(F):
    say("no-alloc entry point: refusals")
    b = _make(F, SMALL, True)
    with pytest.raises(F.FkmcError) as e:
        _make(F, SMALL, True)
    assert e.value.code == -2
    b.close()
    c = _make(F, SMALL, True)      # released by close
    c.close()
    # 600^3 cells in 4-cell fragments: a tile table far beyond 64 MiB
    g = F.Geometry.make((600, 600, 600), (4, 4, 4), 3.905, 0, 0)
    arr = (F.Geometry * 1)(g)
    h = F.C.c_void_p()
    import torch
    tiny = torch.empty(256, dtype=torch.uint8, device="cuda:0")
    rc = F.lib().fkmc_create_static(arr, 1, tiny.data_ptr(), 256, tiny.data_ptr(), 256, None,
                                    F.C.byref(h))
    assert rc == -5 and not h.value
