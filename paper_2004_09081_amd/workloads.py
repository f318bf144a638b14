"""Seeded synthetic workloads (input recipes only: sizes, compositions,
temperatures, fields, synchronisation windows).  No kMC arithmetic here.

Parameters follow the paper's systems (Sec. "Computational details": cubic
SrTiO3/BaTiO3-like anion sublattice, A = 1e13 1/s, O barrier 0.6-0.75 eV,
H barrier 0.17-0.28 eV, 0.1 % vacancies; the biased micro-scale run with
grain boundaries) at the sizes of the standard configurations below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

KB_EV = 1.380649e-23 / 1.602176634e-19  # eV/K
A_STO = 3.905                            # Angstrom


@dataclass
class LatticeSpec:
    L: tuple
    frag: tuple
    seed: int
    lattice_id: int
    n_vac: int
    n_h: int
    T: float
    Ea_O: float
    Ea_H: float
    E_z: float = 0.0
    q: float = 2.0
    gb_period: int = 0
    gb_mask: int = 4
    gb_dE: float = 0.0
    a: float = A_STO
    t_sync: float = 0.0
    extra: dict = field(default_factory=dict)

    @property
    def n_sites(self) -> int:
        return 3 * self.L[0] * self.L[1] * self.L[2]


def counts(n_sites: int, x_v: float, x_h: float):
    """Exact particle counts: nearest integer to fraction x site count."""
    return int(math.floor(x_v * n_sites + 0.5)), int(math.floor(x_h * n_sites + 0.5))


def window_one_hop(T, Ea_O, Ea_H, x_h, x_v, nu=1e13):
    """Synchronisation window giving about one hop per vacancy per cycle:
    1 / (8 (x_H k_H + x_O k_O)) with k = nu exp(-Ea/(k_B T)), no field."""
    kO = nu * math.exp(-Ea_O / (KB_EV * T))
    kH = nu * math.exp(-Ea_H / (KB_EV * T))
    x_o = 1.0 - x_h - x_v
    return 1.0 / (8.0 * (x_h * kH + x_o * kO))


def cfg1() -> LatticeSpec:
    """Plain serial BKL, 8^3 cells (1536 sites), 15 vacancies, O only,
    0.60 eV, 600 K, 1e5 hops."""
    return LatticeSpec(L=(8, 8, 8), frag=(0, 0, 0), seed=0, lattice_id=0, n_vac=15, n_h=0,
                       T=600.0, Ea_O=0.60, Ea_H=0.25, extra={"hops": 100_000})


def cfg2(T: float, seed: int = 0, frag: int = 12) -> LatticeSpec:
    """48^3 cells split in 4^3 fragments of 12^3; H on 10 % of the anion sites,
    0.5 % vacancies; O 0.70 eV, H 0.25 eV; window 1e-9 s; 1e7 hops per T."""
    L = (48, 48, 48)
    nv, nh = counts(3 * 48**3, 0.005, 0.10)
    return LatticeSpec(L=L, frag=(frag,) * 3, seed=seed, lattice_id=0, n_vac=nv, n_h=nh, T=T,
                       Ea_O=0.70, Ea_H=0.25, t_sync=1e-9, extra={"hops": 10_000_000})


CFG2_TEMPERATURES = (300.0, 400.0, 500.0, 600.0, 800.0)


def cfg3(L: int = 600, frag: int = 16) -> LatticeSpec:
    """600^3 cells (6.48e8 anion sites), 0.1 % vacancies, no H, O 0.75 eV,
    450 K, field 1e7 V/m along z (vacancy charge +2), grain-boundary planes
    normal to z every 50 cells with +0.3 eV, 16^3-cell fragments."""
    nv, _ = counts(3 * L**3, 0.001, 0.0)
    ts = window_one_hop(450.0, 0.75, 0.25, 0.0, 0.001)
    return LatticeSpec(L=(L, L, L), frag=(frag,) * 3, seed=0, lattice_id=0, n_vac=nv, n_h=0,
                       T=450.0, Ea_O=0.75, Ea_H=0.25, E_z=1e7, q=2.0, gb_period=50, gb_mask=4,
                       gb_dE=0.3, t_sync=ts)


def cfg4(n: int = 512, seed: int = 0xC4, frag=8, hops: int = 1_000_000):
    """Ensemble of n independent lattices: cube edge uniform in 16..64 cells,
    T uniform 300-900 K, H fraction uniform 0-0.3, vacancy fraction
    log-uniform 1e-3..1e-2, field uniform 0-1e7 V/m; O 0.70 eV, H 0.25 eV;
    window for about one hop per vacancy per cycle; 1e6 hops each."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        Lc = int(rng.integers(16, 65))
        T = float(rng.uniform(300.0, 900.0))
        xh = float(rng.uniform(0.0, 0.3))
        xv = float(10 ** rng.uniform(-3.0, -2.0))
        E = float(rng.uniform(0.0, 1e7))
        nv, nh = counts(3 * Lc**3, xv, xh)
        ts = window_one_hop(T, 0.70, 0.25, xh, xv)
        F = frag(Lc) if callable(frag) else int(frag)
        out.append(LatticeSpec(L=(Lc,) * 3, frag=(F,) * 3, seed=seed, lattice_id=i, n_vac=nv,
                               n_h=nh, T=T, Ea_O=0.70, Ea_H=0.25, E_z=E, q=2.0, t_sync=ts,
                               extra={"x_h": xh, "x_v": xv, "hops": hops}))
    return out


# Pair energies of the site-energy model (meV), from the paper's first-principles
# table of the vacancy-Fe and vacancy-vacancy interactions (Table TABLEadd01).
# Vacancy-Fe over the B-site shells at |r|^2 = 1, 5, 9, 13 (a/2)^2: the table
# gives 0, 0.510, 0.687, 0.709 eV relative to the nearest shell; taken here
# relative to the farthest tabulated shell, so that the interaction vanishes
# beyond it and a vacancy next to Fe is trapped by 0.709 eV.  Vacancy-vacancy
# over the O-site shells 2, 4, 6, 8, 10, 16 (a/2)^2 as tabulated (0 at 2a).
SITE_E_FE_MEV = (-709, -199, -22, 0)
SITE_E_VV_MEV = (343, 235, 200, 180, 23, 0)


def fe_map(L, x_fe: float, seed: int) -> np.ndarray:
    """Fe dopants on round(x_fe L0 L1 L2) distinct B sites (cube centres),
    uniformly at random: one byte per cell in canonical cell order
    ((k L1 + j) L0 + i), 1 = Fe."""
    n_cells = int(L[0] * L[1] * L[2])
    n = int(math.floor(x_fe * n_cells + 0.5))
    rng = np.random.default_rng(0xFE00 + int(seed))
    out = np.zeros(n_cells, dtype=np.uint8)
    out[rng.choice(n_cells, n, replace=False)] = 1
    return out


def voronoi_boundary_map(L, n_grains: int, width: float, seed: int) -> np.ndarray:
    """Grain-boundary sites of a periodic Voronoi tessellation of the x-z
    plane, extruded along y (the grain geometry of the paper's micro-scale
    BaTiO3 model, which it builds in two dimensions and runs in three):
    n_grains seeds drawn uniformly in the periodic x-z box; an anion site
    belongs to the boundary layer when its in-plane distance to the
    second-nearest seed exceeds that to the nearest by less than `width`
    (cells), a layer about `width` cells thick along every face between two
    grains.  One byte per site in canonical order ((k L1 + j) L0 + i) 3 +
    type, 1 = boundary site.  Built slab by slab along z."""
    rng = np.random.default_rng(0x6B00 + int(seed))
    Lv = np.array(L, dtype=np.float64)
    seeds = rng.random((int(n_grains), 3)) * Lv
    seeds[:, 1] = 0.0
    off = np.array([[0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])
    out = np.empty(3 * L[0] * L[1] * L[2], dtype=np.uint8)
    per_k = 3 * L[0] * L[1]
    slab = max(1, int(4_000_000 // max(per_k * int(n_grains), 1)))
    for k0 in range(0, L[2], slab):
        k1 = min(L[2], k0 + slab)
        k, j, i = np.meshgrid(np.arange(k0, k1), np.arange(L[1]), np.arange(L[0]), indexing="ij")
        cells = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
        pos = (cells[:, None, :] + off[None, :, :]).reshape(-1, 3)
        r = np.empty((pos.shape[0], int(n_grains)))
        for g in range(int(n_grains)):
            d = pos - seeds[g]
            d -= Lv * np.round(d / Lv)
            d[:, 1] = 0.0  # in-plane (x-z) distance
            r[:, g] = np.sqrt((d * d).sum(axis=1))
        r.sort(axis=1)
        out[k0 * per_k:k1 * per_k] = ((r[:, 1] - r[:, 0]) < width).astype(np.uint8)
    return out


def micro(L=(200, 50, 300), frag: int = 8, n_grains: int = 6, width: float = 1.0, seed: int = 0):
    """Reduced micro-scale BaTiO3 model (Sec. "Oxygen diffusion in
    micro-scale BaTiO3 model"): Voronoi grains separated by a boundary layer
    whose hops carry +0.2 eV (0.9 eV through the boundary against 0.7 eV in
    the grains), 0.1 % vacancies, the bias of the paper's model (20 V over
    962.4 nm along z, top +10 V: the field points to -z), open z boundary as
    periodic with unwrapped displacements, 450 K, 8^3-cell fragments (the
    vacancies pile up at the boundaries, past the 128 a BKL domain holds in
    16^3-cell fragments).  The box is 200 x 50 x 300 cells (78 x 20 x
    117 nm) instead of the paper's 1600 x 400 x 2400.  Returns the spec and
    its boundary-site map."""
    nv, _ = counts(3 * L[0] * L[1] * L[2], 0.001, 0.0)
    ts = window_one_hop(450.0, 0.70, 0.25, 0.0, 0.001)
    spec = LatticeSpec(L=tuple(L), frag=(frag,) * 3, seed=seed, lattice_id=0, n_vac=nv, n_h=0, T=450.0,
                       Ea_O=0.70, Ea_H=0.25, E_z=-20.0 / 962.4e-9, q=2.0, gb_period=0, gb_mask=0, gb_dE=0.2,
                       t_sync=ts, extra={"n_grains": n_grains, "width": width, "t_end": 5e-3})
    return spec, voronoi_boundary_map(L, n_grains, width, seed)


def surrogate_features(spec: LatticeSpec) -> np.ndarray:
    """(1000/T, x_H, log10 x_V, E / 1e7 V/m) of one lattice."""
    return np.array([1000.0 / spec.T, spec.extra.get("x_h", 0.0),
                     math.log10(max(spec.extra.get("x_v", 1e-3), 1e-12)), spec.E_z / 1e7])


def to_gpu(specs, F):
    """Geometries and rate parameters for the binding."""
    geoms = [F.Geometry.make(s.L, s.frag, s.a, s.seed, s.lattice_id) for s in specs]
    rates = [F.RateParams.make(T=s.T, Ea_O=s.Ea_O, Ea_H=s.Ea_H, E_z=s.E_z, q=s.q,
                               gb_period_cells=s.gb_period, gb_axes_mask=s.gb_mask,
                               gb_dE=s.gb_dE) for s in specs]
    return geoms, rates
