"""Helpers pairing an oracle lattice with a GPU lattice of the same
geometry, key and rates."""
from __future__ import annotations

import sys

import numpy as np

from oracle import oracle as O


def gpu_modules():
    from paper_2004_09081_amd import fkmc as F
    return F


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Case:
    """One lattice configuration: geometry, composition and rates."""

    def __init__(self, L, frag=(0, 0, 0), seed=0, lattice_id=0, nv=10, nh=0, T=600.0,
                 Ea_O=0.6, Ea_H=0.25, E_z=0.0, q=2.0, gb_period=0, gb_mask=4, gb_dE=0.0,
                 a=3.905):
        self.L, self.frag, self.seed, self.lattice_id = tuple(L), tuple(frag), seed, lattice_id
        self.nv, self.nh = nv, nh
        self.rp = dict(T=T, Ea_O=Ea_O, Ea_H=Ea_H, E_z=E_z, q=q, gb_period_cells=gb_period,
                       gb_axes_mask=gb_mask, gb_dE=gb_dE)
        self.a = a

    def oracle(self) -> O.Lattice:
        g = O.Geometry(L=self.L, frag=self.frag, a_angstrom=self.a, seed=self.seed,
                       lattice_id=self.lattice_id, gb_period_cells=self.rp["gb_period_cells"],
                       gb_axes_mask=self.rp["gb_axes_mask"])
        lat = O.Lattice(g)
        lat.init_random(self.nv, self.nh)
        lat.set_rates(O.RateParams(**self.rp))
        return lat

    def gpu_geometry(self):
        F = gpu_modules()
        return F.Geometry.make(self.L, self.frag, self.a, self.seed, self.lattice_id)

    def gpu_rates(self):
        F = gpu_modules()
        return F.RateParams.make(**self.rp)


def gpu_set(cases):
    F = gpu_modules()
    s = F.LatticeSet([c.gpu_geometry() for c in cases])
    s.init_random([c.nv for c in cases], [c.nh for c in cases])
    s.set_rates([c.gpu_rates() for c in cases])
    return s


def assert_same_state(gset, i, lat: O.Lattice, what=""):
    occ, disp = gset.read_state(i)
    bad = np.nonzero(occ != lat.occ)[0]
    assert bad.size == 0, "%s occupancy differs at %d sites, first %s" % (what, bad.size, bad[:8])
    bad = np.nonzero((disp != lat.disp).any(axis=1))[0]
    assert bad.size == 0, "%s displacement differs at %d sites, first %s" % (what, bad.size, bad[:8])
