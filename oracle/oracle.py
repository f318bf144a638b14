"""ctypes front end of the C oracle (fkmc_oracle.c) plus exact observables.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg; never by the library.

All lattice arrays are in canonical site order n = ((k*Ly + j)*Lx + i)*3 + type;
occupancy int8 (O=0, H=1, V=2); displacement int32 [N, 3] in doubled units
(1 unit = a/2), travelling with the occupant.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fkmc_oracle.c")
LIB = os.path.join(HERE, "libfkmc_oracle.so")

SP_O, SP_H, SP_V = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared",
                               "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Geom(C.Structure):
    _fields_ = [("L", C.c_int32 * 3), ("frag", C.c_int32 * 3), ("a_angstrom", C.c_double),
                ("seed", C.c_uint32), ("lattice_id", C.c_uint32),
                ("gb_period_cells", C.c_int32), ("gb_axes_mask", C.c_int32),
                ("gb_map", C.c_void_p)]


class _SiteParams(C.Structure):
    _fields_ = [("e_fe", C.c_int32 * 4), ("e_vv", C.c_int32 * 6), ("window", C.c_int32)]


class _Rates(C.Structure):
    _fields_ = [("nu", C.c_double), ("T", C.c_double), ("Ea_O", C.c_double),
                ("Ea_H", C.c_double), ("E_z", C.c_double), ("q", C.c_double),
                ("gb_period_cells", C.c_int32), ("gb_axes_mask", C.c_int32),
                ("gb_dE", C.c_double)]


_lib = None


def lib():
    """The compiled oracle; FKMC_ORACLE_LIB names another build of the same
    source (the sanitizer test loads an instrumented one)."""
    global _lib
    if _lib is None:
        _lib = C.CDLL(os.environ.get("FKMC_ORACLE_LIB") or build())
        P = C.POINTER
        _lib.or_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        _lib.or_ln.argtypes = [C.c_double]
        _lib.or_ln.restype = C.c_double
        _lib.or_ln_constants.argtypes = [P(C.c_double)]
        _lib.or_hop_table.argtypes = [P(C.c_int32)]
        _lib.or_rate_raw.argtypes = [P(_Rates), C.c_double, P(C.c_double)]
        _lib.or_quantise.argtypes = [P(C.c_double), C.c_uint64, P(C.c_double), P(C.c_double),
                                     P(C.c_double)]
        _lib.or_init_random.argtypes = [P(_Geom), C.c_void_p, C.c_uint64, C.c_uint64,
                                        P(C.c_uint64)]
        _lib.or_phase.argtypes = [P(_Geom), P(C.c_double), C.c_void_p, C.c_void_p, C.c_double,
                                  C.c_uint64, C.c_int, C.c_int, P(C.c_uint64), P(C.c_uint64)]
        _lib.or_advance_frag.argtypes = [P(_Geom), P(C.c_double), C.c_void_p, C.c_void_p,
                                         C.c_double, C.c_uint64, C.c_uint64, C.c_uint64,
                                         P(C.c_uint64), P(C.c_uint64)]
        _lib.or_advance_plain.argtypes = [P(_Geom), P(C.c_double), C.c_void_p, C.c_void_p,
                                          P(C.c_uint64), P(C.c_double), C.c_double, C.c_uint64,
                                          P(C.c_uint64)]
        _lib.or_advance_atomic.argtypes = [P(_Geom), P(C.c_double), C.c_void_p, C.c_void_p,
                                           P(C.c_uint64), P(C.c_double), C.c_uint32, C.c_uint64,
                                           P(C.c_uint64)]
        _lib.or_num_fragments.argtypes = [P(_Geom)]
        _lib.or_footprint_sites.argtypes = [P(_Geom), C.c_int, C.c_int, P(C.c_int64), C.c_int64]
        _lib.or_edge_active.argtypes = [P(_Geom), C.c_int64, C.c_int, C.c_int, C.c_int]
        _lib.or_hop_target.argtypes = [P(_Geom), C.c_int64, C.c_int]
        _lib.or_hop_target.restype = C.c_int64
        _lib.or_is_gb_site.argtypes = [P(_Geom), C.c_int64]
        _lib.or_sub_block.argtypes = [P(_Geom), C.c_int, C.c_int, P(C.c_int32), P(C.c_int32)]
        _lib.or_site_energy.argtypes = [P(_Geom), C.c_void_p, C.c_void_p, P(_SiteParams), C.c_int64,
                                        C.c_int64]
        _lib.or_site_energy.restype = C.c_int32
        _lib.or_site_table.argtypes = [P(C.c_double), C.c_double, C.c_int32, C.c_uint64, P(C.c_double),
                                       P(C.c_double), P(C.c_double)]
        _lib.or_advance_plain_site.argtypes = [P(_Geom), P(C.c_double), P(C.c_double), C.c_double,
                                               C.c_void_p, P(_SiteParams), C.c_void_p, C.c_void_p,
                                               P(C.c_uint64), P(C.c_double), C.c_double, C.c_uint64,
                                               P(C.c_uint64)]
        _lib.or_advance_frag_site.argtypes = [P(_Geom), P(C.c_double), P(C.c_double), C.c_double,
                                              C.c_void_p, P(_SiteParams), C.c_void_p, C.c_void_p,
                                              C.c_double, C.c_uint64, C.c_uint64, C.c_uint64,
                                              P(C.c_uint64), P(C.c_uint64)]
        _lib.or_phase_site.argtypes = [P(_Geom), P(C.c_double), P(C.c_double), C.c_double, C.c_void_p,
                                       P(_SiteParams), C.c_void_p, C.c_void_p, C.c_double, C.c_uint64,
                                       C.c_int, C.c_int, P(C.c_uint64)]
        _lib.or_site_rate.argtypes = [P(_Geom), P(C.c_double), P(C.c_double), C.c_double, C.c_void_p,
                                      P(_SiteParams), C.c_void_p, C.c_int64, C.c_int]
        _lib.or_site_rate.restype = C.c_double
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# --------------------------------------------------------------------------- primitives
def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def ln(u: float) -> float:
    return lib().or_ln(float(u))


def ln_constants():
    o = (C.c_double * 3)()
    lib().or_ln_constants(o)
    return tuple(o)


def hop_table() -> np.ndarray:
    o = np.zeros((3, 8, 3), dtype=np.int32)
    lib().or_hop_table(o.ctypes.data_as(C.POINTER(C.c_int32)))
    return o


@dataclass
class RateParams:
    nu: float = 1e13
    T: float = 600.0
    Ea_O: float = 0.6
    Ea_H: float = 0.25
    E_z: float = 0.0
    q: float = 2.0
    gb_period_cells: int = 0
    gb_axes_mask: int = 4
    gb_dE: float = 0.0

    def c(self) -> _Rates:
        return _Rates(self.nu, self.T, self.Ea_O, self.Ea_H, self.E_z, self.q,
                      self.gb_period_cells, self.gb_axes_mask, self.gb_dE)


def rate_raw(p: RateParams, a_angstrom: float) -> np.ndarray:
    """12 unquantised rates, index (X*3 + dz+1)*2 + g."""
    o = np.zeros(12)
    r = p.c()
    lib().or_rate_raw(C.byref(r), float(a_angstrom), _dp(o))
    return o


def absent_species_zeroed(raw: np.ndarray, occ: np.ndarray) -> np.ndarray:
    """Copy of the 12-entry table with the entries of ion species that do
    not occur in occ set to zero (index (X*3 + dz+1)*2 + g, X = 0 O, 1 H)."""
    out = np.array(raw, dtype=np.float64)
    for X in (SP_O, SP_H):
        if not (occ == X).any():
            out[X * 6:(X + 1) * 6] = 0.0
    return out


def quantise(raw: np.ndarray, n_ev: int):
    raw = np.ascontiguousarray(raw, dtype=np.float64)
    o = np.zeros(12)
    q = C.c_double()
    rel = C.c_double()
    rc = lib().or_quantise(_dp(raw), int(n_ev), _dp(o), C.byref(q), C.byref(rel))
    if rc != 0:
        raise ValueError("rate quantisation failed (%d)" % rc)
    return o, q.value, rel.value


@dataclass
class SiteParams:
    """Pair energies (meV) of the site-energy model: vacancy-Fe over the B-site
    shells |r|^2 = 1, 5, 9, 13 (a/2)^2 and vacancy-vacancy over the O-site
    shells 2, 4, 6, 8, 10, 16; window = largest |dE_site| (meV) of a hop."""
    e_fe: tuple = (0, 0, 0, 0)
    e_vv: tuple = (0, 0, 0, 0, 0, 0)
    window: int = 1000

    def c(self) -> _SiteParams:
        p = _SiteParams()
        p.e_fe[:] = [int(x) for x in self.e_fe]
        p.e_vv[:] = [int(x) for x in self.e_vv]
        p.window = int(self.window)
        return p


def site_table(raw12: np.ndarray, T: float, window: int, n_ev: int):
    """(f, q, max_rel): f[j] = exp(-(j - window) meV/(2 k_B T)) and the
    quantum of the products raw12[i] f[j]."""
    raw12 = np.ascontiguousarray(raw12, dtype=np.float64)
    f = np.zeros(2 * int(window) + 1)
    q = C.c_double()
    rel = C.c_double()
    rc = lib().or_site_table(_dp(raw12), float(T), int(window), int(n_ev), _dp(f), C.byref(q), C.byref(rel))
    if rc != 0:
        raise ValueError("site rate table failed (%d)" % rc)
    return f, q.value, rel.value


# --------------------------------------------------------------------------- lattice
@dataclass
class Geometry:
    L: tuple = (8, 8, 8)
    frag: tuple = (0, 0, 0)
    a_angstrom: float = 3.905
    seed: int = 0
    lattice_id: int = 0
    gb_period_cells: int = 0
    gb_axes_mask: int = 4
    # one byte per site (canonical order), 1 = grain-boundary site; replaces
    # the planes when given (Voronoi grain boundaries)
    gb_map: np.ndarray = None

    def c(self) -> _Geom:
        g = _Geom()
        g.L[:] = list(self.L)
        g.frag[:] = list(self.frag)
        g.a_angstrom = self.a_angstrom
        g.seed = self.seed & 0xFFFFFFFF
        g.lattice_id = self.lattice_id & 0xFFFFFFFF
        g.gb_period_cells = self.gb_period_cells
        g.gb_axes_mask = self.gb_axes_mask
        if self.gb_map is not None:
            self._gb_keep = np.ascontiguousarray(self.gb_map, dtype=np.uint8).reshape(-1)
            assert self._gb_keep.size == self.n_sites
            g.gb_map = self._gb_keep.ctypes.data
        else:
            g.gb_map = None
        return g

    @property
    def n_sites(self) -> int:
        return 3 * self.L[0] * self.L[1] * self.L[2]

    @property
    def plain(self) -> bool:
        return all(f <= 0 for f in self.frag)


def _axis_halves(L: int, F: int):
    """Sub-block widths along one axis (fragments of F cells, halved)."""
    if F <= 0 or F >= L:
        sizes = [L]
    else:
        nf = L // F
        r = L - nf * F
        sizes = [F] * nf
        if r >= 2:
            sizes.append(r)
        elif r == 1:
            sizes[-1] += 1
    out = []
    for s in sizes:
        out += [(s + 1) // 2, s // 2]
    return out


def max_domain_sites(g: Geometry) -> int:
    """Largest number of sites one BKL domain can hold: the whole lattice in
    plain mode, else the largest footprint (sub-block sites plus one face of
    type-a sites on each +a side)."""
    if g.plain:
        return g.n_sites
    best = 0
    for wx in set(_axis_halves(g.L[0], g.frag[0])):
        for wy in set(_axis_halves(g.L[1], g.frag[1])):
            for wz in set(_axis_halves(g.L[2], g.frag[2])):
                best = max(best, 3 * wx * wy * wz + wy * wz + wz * wx + wx * wy)
    return best


class Lattice:
    """One lattice: canonical occupancy + displacement arrays, clock and counters."""

    def __init__(self, geom: Geometry, gb_dE: float = 0.0):
        self.g = geom
        self._gc = geom.c()
        N = geom.n_sites
        self.occ = np.zeros(N, dtype=np.int8)
        self.disp = np.zeros((N, 3), dtype=np.int32)
        self.k12 = np.zeros(12)
        self.t = 0.0
        self.cycles = 0
        self.draws = 0
        self.hops = np.zeros(2, dtype=np.uint64)  # O, H

    # -- set-up
    def init_random(self, n_vac: int, n_h: int) -> int:
        d = C.c_uint64()
        rc = lib().or_init_random(C.byref(self._gc), self.occ.ctypes.data, int(n_vac), int(n_h),
                                  C.byref(d))
        if rc != 0:
            raise ValueError("init failed")
        self.disp[:] = 0
        return d.value

    def set_rates(self, p: RateParams):
        """Rate table of Eq. RateCnst1 (field and boundary terms included),
        quantised for exact sums.  Species absent from the lattice (hops
        conserve the counts) get zero rates, so they do not set the quantum."""
        raw = rate_raw(p, self.g.a_angstrom)
        raw = absent_species_zeroed(raw, self.occ)
        nv = int((self.occ == SP_V).sum())
        n_ev = 8 * min(max(nv, 1), max_domain_sites(self.g))
        self.k12, self.q, self.max_rel = quantise(raw, n_ev)
        return self.k12

    # -- dynamics
    def advance(self, t_sync: float, max_cycles: int = 1, min_hops: int = 0):
        h = (C.c_uint64 * 2)()
        n = C.c_uint64()
        lib().or_advance_frag(C.byref(self._gc), _dp(self.k12), self.occ.ctypes.data,
                              self.disp.ctypes.data, float(t_sync), self.cycles, int(max_cycles),
                              int(min_hops), h, C.byref(n))
        self.cycles += n.value
        self.t = self.t + float(n.value) * float(t_sync)
        self.hops += np.array([h[0], h[1]], dtype=np.uint64)
        return n.value, (h[0], h[1])

    def phase(self, t_sync: float, cycle: int, colour: int, frag_index: int):
        h = (C.c_uint64 * 2)()
        st = C.c_uint64()
        lib().or_phase(C.byref(self._gc), _dp(self.k12), self.occ.ctypes.data,
                       self.disp.ctypes.data, float(t_sync), int(cycle), int(colour),
                       int(frag_index), h, C.byref(st))
        return (h[0], h[1]), st.value

    def advance_plain(self, n_hops: int, t_horizon: float = 0.0):
        h = (C.c_uint64 * 2)()
        d = C.c_uint64(self.draws)
        t = C.c_double(self.t)
        lib().or_advance_plain(C.byref(self._gc), _dp(self.k12), self.occ.ctypes.data,
                               self.disp.ctypes.data, C.byref(d), C.byref(t), float(t_horizon),
                               int(n_hops), h)
        self.draws = d.value
        self.t = t.value
        self.hops += np.array([h[0], h[1]], dtype=np.uint64)
        return (h[0], h[1])

    def advance_atomic(self, n_frg: int, n_stages: int):
        """Atom-selection fragment kMC with null events (Eqs. AtomP and
        TimeStepFrg): n_stages stages of n_frg selected vacancies each.  The
        stage counter is the plain draw counter `draws`."""
        h = (C.c_uint64 * 2)()
        d = C.c_uint64(self.draws)
        t = C.c_double(self.t)
        lib().or_advance_atomic(C.byref(self._gc), _dp(self.k12), self.occ.ctypes.data,
                                self.disp.ctypes.data, C.byref(d), C.byref(t), int(n_frg),
                                int(n_stages), h)
        self.draws = d.value
        self.t = t.value
        self.hops += np.array([h[0], h[1]], dtype=np.uint64)
        return (h[0], h[1])

    # -- site-energy interactions (plain BKL only)
    def set_site_model(self, fe: np.ndarray, sp: SiteParams, p: RateParams):
        """Fe map (one byte per cell, canonical cell order, 1 = Fe on its B
        site), pair energies and rate parameters of plain BKL with site
        energies; the quantum follows the largest possible rate."""
        L = self.g.L
        self.fe = np.ascontiguousarray(fe, dtype=np.uint8).reshape(L[0] * L[1] * L[2])
        self.sp = sp
        self._spc = sp.c()
        raw = absent_species_zeroed(rate_raw(p, self.g.a_angstrom), self.occ)
        nv = int((self.occ == SP_V).sum())
        n_ev = 8 * min(max(nv, 1), self.g.n_sites)
        self.site_raw = raw
        self.site_f, self.site_q, self.site_rel = site_table(raw, p.T, sp.window, n_ev)

    def site_energy(self, s: int, skip: int = -1) -> int:
        return lib().or_site_energy(C.byref(self._gc), self.occ.ctypes.data, self.fe.ctypes.data,
                                    C.byref(self._spc), int(s), int(skip))

    def site_rate(self, s: int, d: int) -> float:
        return lib().or_site_rate(C.byref(self._gc), _dp(self.site_raw), _dp(self.site_f), self.site_q,
                                  self.fe.ctypes.data, C.byref(self._spc), self.occ.ctypes.data, int(s), int(d))

    def advance_plain_site(self, n_hops: int, t_horizon: float = 0.0):
        """Plain BKL with site energies: same draws, clock and selection as
        advance_plain."""
        h = (C.c_uint64 * 2)()
        d = C.c_uint64(self.draws)
        t = C.c_double(self.t)
        rc = lib().or_advance_plain_site(C.byref(self._gc), _dp(self.site_raw), _dp(self.site_f), self.site_q,
                                         self.fe.ctypes.data, C.byref(self._spc), self.occ.ctypes.data,
                                         self.disp.ctypes.data, C.byref(d), C.byref(t), float(t_horizon),
                                         int(n_hops), h)
        self.draws = d.value
        self.t = t.value
        self.hops += np.array([h[0], h[1]], dtype=np.uint64)
        if rc != 0:
            raise ValueError("site-energy difference outside the window (%d)" % rc)
        return (h[0], h[1])

    def advance_site(self, t_sync: float, max_cycles: int = 1, min_hops: int = 0):
        """Fragment kMC with site energies: the cycles, phases, draws and
        clock of advance, the rates of advance_plain_site.  Every sub-block
        width w must satisfy 4 w^2 > the vacancy-vacancy reach (squared
        doubled distance of the farthest nonzero shell)."""
        h = (C.c_uint64 * 2)()
        n = C.c_uint64()
        rc = lib().or_advance_frag_site(C.byref(self._gc), _dp(self.site_raw), _dp(self.site_f), self.site_q,
                                        self.fe.ctypes.data, C.byref(self._spc), self.occ.ctypes.data,
                                        self.disp.ctypes.data, float(t_sync), self.cycles, int(max_cycles),
                                        int(min_hops), h, C.byref(n))
        if rc == -1:
            raise ValueError("a sub-block is too narrow for the vacancy-vacancy reach")
        self.cycles += n.value
        self.t = self.t + float(n.value) * float(t_sync)
        self.hops += np.array([h[0], h[1]], dtype=np.uint64)
        if rc != 0:
            raise ValueError("site-energy difference outside the window (%d)" % rc)
        return n.value, (h[0], h[1])

    def phase_site(self, t_sync: float, cycle: int, colour: int, frag_index: int):
        """One phase of advance_site (no sub-block width check)."""
        h = (C.c_uint64 * 2)()
        rc = lib().or_phase_site(C.byref(self._gc), _dp(self.site_raw), _dp(self.site_f), self.site_q,
                                 self.fe.ctypes.data, C.byref(self._spc), self.occ.ctypes.data,
                                 self.disp.ctypes.data, float(t_sync), int(cycle), int(colour),
                                 int(frag_index), h)
        if rc != 0:
            raise ValueError("site-energy difference outside the window (%d)" % rc)
        return (h[0], h[1])

    @property
    def n_fragments(self) -> int:
        return lib().or_num_fragments(C.byref(self._gc))

    def stats(self):
        return observables(self.occ, self.disp, self.g.a_angstrom, self.t)


def footprint_sites(g: Geometry, frag_index: int, colour: int) -> np.ndarray:
    gc = g.c()
    cap = g.n_sites
    out = np.zeros(cap, dtype=np.int64)
    n = lib().or_footprint_sites(C.byref(gc), frag_index, colour,
                                 out.ctypes.data_as(C.POINTER(C.c_int64)), cap)
    return out[:n]


def sub_block(g: Geometry, frag_index: int, colour: int):
    gc = g.c()
    lo = (C.c_int32 * 3)()
    hi = (C.c_int32 * 3)()
    lib().or_sub_block(C.byref(gc), frag_index, colour, lo, hi)
    return tuple(lo), tuple(hi)


def edge_active(g: Geometry, s: int, d: int, frag_index: int, colour: int) -> bool:
    gc = g.c()
    return bool(lib().or_edge_active(C.byref(gc), int(s), int(d), frag_index, colour))


def hop_target(g: Geometry, s: int, d: int) -> int:
    gc = g.c()
    return lib().or_hop_target(C.byref(gc), int(s), int(d))


def is_gb_site(g: Geometry, s: int) -> bool:
    gc = g.c()
    return bool(lib().or_is_gb_site(C.byref(gc), int(s)))


# --------------------------------------------------------------------------- observables
@dataclass
class Stats:
    count: np.ndarray            # [3] particles per species (O, H, V)
    sum_r: np.ndarray            # [3,3] int64, doubled units
    sum_rr: np.ndarray           # [3,3,3] int64 second moments
    t: float
    a: float
    msd: np.ndarray = field(default=None)     # [3] Angstrom^2
    D: np.ndarray = field(default=None)       # [3] Angstrom^2/s (Einstein, 6t)
    drift: np.ndarray = field(default=None)   # [3,3] Angstrom/s
    Dtensor: np.ndarray = field(default=None)  # [3,3,3] Angstrom^2/s


def observables(occ: np.ndarray, disp: np.ndarray, a: float, t: float) -> Stats:
    """Tracer statistics per species from the per-particle displacements
    (the paper tracks the trajectories of the respective atoms): exact int64
    sums, then MSD = (a/2)^2 sum|r|^2 / N, D = MSD/(6t), drift = (a/2) sum r/(N t),
    D_ab = (a/2)^2 (<r_a r_b> - <r_a><r_b>)/(2t)."""
    count = np.zeros(3, dtype=np.int64)
    sr = np.zeros((3, 3), dtype=np.int64)
    srr = np.zeros((3, 3, 3), dtype=np.int64)
    d64 = disp.astype(np.int64)
    for X in range(3):
        m = occ == X
        count[X] = int(m.sum())
        r = d64[m]
        sr[X] = r.sum(axis=0)
        srr[X] = r.T @ r
    st = Stats(count, sr, srr, t, a)
    h = a / 2.0
    with np.errstate(divide="ignore", invalid="ignore"):
        n = np.maximum(count, 1).astype(np.float64)
        st.msd = h * h * np.trace(srr, axis1=1, axis2=2).astype(np.float64) / n
        st.D = st.msd / (6.0 * t) if t > 0 else np.full(3, np.nan)
        st.drift = h * sr.astype(np.float64) / (n[:, None] * t) if t > 0 else np.full((3, 3), np.nan)
        mean = sr.astype(np.float64) / n[:, None]
        cov = srr.astype(np.float64) / n[:, None, None] - mean[:, :, None] * mean[:, None, :]
        st.Dtensor = h * h * cov / (2.0 * t) if t > 0 else np.full((3, 3, 3), np.nan)
    return st
