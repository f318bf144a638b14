"""Python binding of the C-ABI library libfkmc.so (include/fkmc.h).

Argument marshalling only: every step of the kMC path runs in the library's
HIP kernels.  PyTorch supplies the device buffers and the HIP stream.
The binding refuses to run if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfkmc.so")

FKMC_OK = 0
ERRORS = {-1: "E_INVALID", -2: "E_STATE", -3: "E_DEVICE", -4: "E_RANGE", -5: "E_NOMEM",
          -6: "E_UNSUPPORTED"}


class FkmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (ERRORS.get(code, code), msg))
        self.code = code


class Geometry(C.Structure):
    _fields_ = [("L", C.c_int32 * 3), ("frag", C.c_int32 * 3), ("a_angstrom", C.c_double),
                ("seed", C.c_uint32), ("lattice_id", C.c_uint32)]

    @staticmethod
    def make(L, frag=(0, 0, 0), a_angstrom=3.905, seed=0, lattice_id=0) -> "Geometry":
        g = Geometry()
        g.L[:] = [int(x) for x in L]
        g.frag[:] = [int(x) for x in frag]
        g.a_angstrom = float(a_angstrom)
        g.seed = int(seed) & 0xFFFFFFFF
        g.lattice_id = int(lattice_id) & 0xFFFFFFFF
        return g

    @property
    def n_sites(self) -> int:
        return 3 * self.L[0] * self.L[1] * self.L[2]


class RateParams(C.Structure):
    _fields_ = [("nu", C.c_double), ("T", C.c_double), ("Ea_O", C.c_double),
                ("Ea_H", C.c_double), ("E_z", C.c_double), ("q", C.c_double),
                ("gb_period_cells", C.c_int32), ("gb_axes_mask", C.c_int32),
                ("gb_dE", C.c_double)]

    @staticmethod
    def make(nu=1e13, T=600.0, Ea_O=0.6, Ea_H=0.25, E_z=0.0, q=2.0, gb_period_cells=0,
             gb_axes_mask=4, gb_dE=0.0) -> "RateParams":
        return RateParams(nu, T, Ea_O, Ea_H, E_z, q, gb_period_cells, gb_axes_mask, gb_dE)


class Buffers(C.Structure):
    _fields_ = [("occ", C.c_void_p), ("disp", C.c_void_p), ("work", C.c_void_p),
                ("bytes", C.c_size_t * 3)]


class Stats(C.Structure):
    _fields_ = [("t", C.c_double), ("cycles", C.c_uint64), ("draws", C.c_uint64),
                ("hops", C.c_uint64 * 2), ("count", C.c_uint64 * 3),
                ("sum_r", (C.c_int64 * 3) * 3), ("sum_rr", (C.c_int64 * 6) * 3),
                ("msd", C.c_double * 3), ("D", C.c_double * 3),
                ("drift", (C.c_double * 3) * 3), ("Dtensor", (C.c_double * 6) * 3),
                ("busy_ms", C.c_double), ("lds_resident", C.c_uint32), ("tile_group", C.c_uint32)]

    def to_dict(self) -> dict:
        return {
            "t": self.t, "cycles": self.cycles, "draws": self.draws,
            "hops": np.array(self.hops[:], dtype=np.uint64),
            "count": np.array(self.count[:], dtype=np.int64),
            "sum_r": np.array([r[:] for r in self.sum_r], dtype=np.int64),
            "sum_rr": np.array([r[:] for r in self.sum_rr], dtype=np.int64),
            "msd": np.array(self.msd[:]), "D": np.array(self.D[:]),
            "drift": np.array([r[:] for r in self.drift]),
            "Dtensor": np.array([r[:] for r in self.Dtensor]),
            "busy_ms": self.busy_ms, "lds_resident": bool(self.lds_resident),
            "tile_group": int(self.tile_group),
        }


# Exported symbols and their argument types (mirrors include/fkmc.h).
_P = C.POINTER
_SIGS = {
    "fkmc_query_sizes": [_P(Geometry), C.c_uint32, _P(C.c_size_t)],
    "fkmc_create": [_P(Geometry), C.c_uint32, _P(Buffers), C.c_void_p, _P(C.c_void_p)],
    "fkmc_create_static": [_P(Geometry), C.c_uint32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t,
                           C.c_void_p, _P(C.c_void_p)],
    "fkmc_destroy": [C.c_void_p],
    "fkmc_count": [C.c_void_p],
    "fkmc_init_random": [C.c_void_p, _P(C.c_uint64), _P(C.c_uint64)],
    "fkmc_set_occupancy": [C.c_void_p, C.c_uint32, C.c_void_p, C.c_size_t],
    "fkmc_set_rates": [C.c_void_p, _P(RateParams)],
    "fkmc_set_rate_table": [C.c_void_p, C.c_uint32, _P(C.c_double), C.c_size_t],
    "fkmc_get_rate_table": [C.c_void_p, C.c_uint32, _P(C.c_double), C.c_size_t],
    "fkmc_rate_table_host": [_P(RateParams), C.c_double, C.c_uint64, _P(C.c_double),
                             _P(C.c_double), _P(C.c_double), _P(C.c_double)],
    "fkmc_max_domain_sites": [_P(Geometry), _P(C.c_uint64)],
    "fkmc_advance": [C.c_void_p, _P(C.c_double), C.c_uint64, C.c_uint64],
    "fkmc_run_phase": [C.c_void_p, _P(C.c_double), C.c_int32],
    "fkmc_sync": [C.c_void_p],
    "fkmc_read_state": [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_size_t],
    "fkmc_read_stats": [C.c_void_p, _P(Stats)],
    "fkmc_set_timing": [C.c_void_p, C.c_int32],
    "fkmc_set_schedule": [C.c_void_p, C.c_int32, C.c_int32],
    "fkmc_set_graph": [C.c_void_p, C.c_int32],
    "fkmc_set_group": [C.c_void_p, C.c_int32],
    "fkmc_advance_atomic": [C.c_void_p, C.c_uint32, C.c_uint64],
    "fkmc_set_plain_lds": [C.c_void_p, C.c_int32],
    "fkmc_checkpoint_size": [C.c_void_p, C.c_uint32, _P(C.c_size_t)],
    "fkmc_checkpoint": [C.c_void_p, C.c_uint32, C.c_void_p, C.c_size_t],
    "fkmc_restore": [C.c_void_p, C.c_uint32, C.c_void_p, C.c_size_t],
    "fkmc_phase_timing": [C.c_void_p, _P(C.c_double), _P(C.c_uint64)],
    "fkmc_quantisation": [C.c_void_p, C.c_uint32, _P(C.c_double), _P(C.c_double)],
    "fkmc_site_model_bytes": [C.c_void_p, C.c_uint32, C.c_int32, _P(C.c_size_t)],
    "fkmc_gb_map_bytes": [C.c_void_p, C.c_uint32, _P(C.c_size_t)],
    "fkmc_set_gb_map": [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_size_t],
    "fkmc_set_site_model": [C.c_void_p, C.c_uint32, C.c_void_p, _P(C.c_int32), _P(C.c_int32), C.c_int32,
                            C.c_void_p, C.c_size_t],
    "fkmc_last_error": [],
}

_lib = None


def lib():
    """Load libfkmc.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfkmc.so is not built; run paper_2004_09081_amd.build.build()")
        _lib = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = C.c_int32
        _lib.fkmc_last_error.restype = C.c_char_p
        _lib.fkmc_count.restype = C.c_uint32
    return _lib


def _check(rc: int):
    if rc != FKMC_OK:
        raise FkmcError(rc, lib().fkmc_last_error().decode())


def _dbl(a) -> C.Array:
    a = [float(x) for x in a]
    return (C.c_double * len(a))(*a)


def rate_table_host(p: RateParams, a_angstrom: float, n_ev: int):
    raw = (C.c_double * 12)()
    qt = (C.c_double * 12)()
    q = C.c_double()
    rel = C.c_double()
    _check(lib().fkmc_rate_table_host(C.byref(p), float(a_angstrom), int(n_ev), raw, qt,
                                      C.byref(q), C.byref(rel)))
    return np.array(raw[:]), np.array(qt[:]), q.value, rel.value


def max_domain_sites(g: Geometry) -> int:
    o = C.c_uint64()
    _check(lib().fkmc_max_domain_sites(C.byref(g), C.byref(o)))
    return o.value


def query_sizes(geoms: Sequence[Geometry]):
    arr = (Geometry * len(geoms))(*geoms)
    out = (C.c_size_t * 3)()
    _check(lib().fkmc_query_sizes(arr, len(geoms), out))
    return tuple(out)


@dataclass
class LatticeSet:
    """A set of n >= 1 lattices in caller-owned (torch) device memory.  With
    static_work the handle comes from fkmc_create_static: only occupancy and
    displacements are allocated here, the work space is the library's."""
    geoms: list
    device: str = "cuda:0"
    static_work: bool = False
    _h: C.c_void_p = field(default=None, init=False, repr=False)

    def __post_init__(self):
        import torch
        self.geoms = list(self.geoms)
        self.n = len(self.geoms)
        lib()
        sizes = query_sizes(self.geoms)
        dev = torch.device(self.device)
        self.occ_buf = torch.empty(max(sizes[0], 1), dtype=torch.uint8, device=dev)
        self.disp_buf = torch.empty(max(sizes[1], 16), dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream(dev)
        arr = (Geometry * self.n)(*self.geoms)
        h = C.c_void_p()
        if self.static_work:
            self.work_buf = None
            _check(lib().fkmc_create_static(arr, self.n, self.occ_buf.data_ptr(), sizes[0],
                                            self.disp_buf.data_ptr(), sizes[1],
                                            C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        else:
            self.work_buf = torch.empty(max(sizes[2], 1), dtype=torch.uint8, device=dev)
            b = Buffers(self.occ_buf.data_ptr(), self.disp_buf.data_ptr(), self.work_buf.data_ptr(),
                        (C.c_size_t * 3)(*sizes))
            _check(lib().fkmc_create(arr, self.n, C.byref(b), C.c_void_p(self.stream.cuda_stream),
                                     C.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            _check(lib().fkmc_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- set-up
    def init_random(self, n_vac, n_h):
        nv = (C.c_uint64 * self.n)(*[int(x) for x in np.broadcast_to(n_vac, self.n)])
        nh = (C.c_uint64 * self.n)(*[int(x) for x in np.broadcast_to(n_h, self.n)])
        _check(lib().fkmc_init_random(self._h, nv, nh))

    def set_occupancy(self, i: int, occ: np.ndarray):
        occ = np.ascontiguousarray(occ, dtype=np.int8)
        _check(lib().fkmc_set_occupancy(self._h, i, occ.ctypes.data, occ.size))

    def set_rates(self, params: Sequence[RateParams]):
        if isinstance(params, RateParams):
            params = [params] * self.n
        arr = (RateParams * self.n)(*params)
        _check(lib().fkmc_set_rates(self._h, arr))

    def set_site_model(self, i: int, fe, e_fe, e_vv, window_meV: int):
        """Site energies on lattice i (fkmc_set_site_model): Fe map of
        one byte per cell, pair energies in meV; the device buffer is
        allocated here and kept with the set."""
        import torch
        n = C.c_size_t()
        _check(lib().fkmc_site_model_bytes(self._h, int(i), int(window_meV), C.byref(n)))
        buf = torch.empty(max(n.value, 1), dtype=torch.uint8, device=self.device)
        fe = np.ascontiguousarray(fe, dtype=np.uint8)
        ef = (C.c_int32 * 4)(*[int(x) for x in e_fe])
        ev = (C.c_int32 * 6)(*[int(x) for x in e_vv])
        _check(lib().fkmc_set_site_model(self._h, int(i), fe.ctypes.data, ef, ev, int(window_meV),
                                         buf.data_ptr(), n.value))
        if not hasattr(self, "_site_bufs"):
            self._site_bufs = {}
        self._site_bufs[int(i)] = buf

    def set_gb_map(self, i: int, gb_map):
        """Boundary sites of lattice i as a map (fkmc_set_gb_map): one byte
        per site in canonical order; None removes it."""
        import torch
        if gb_map is None:
            _check(lib().fkmc_set_gb_map(self._h, int(i), None, None, 0))
            return
        n = C.c_size_t()
        _check(lib().fkmc_gb_map_bytes(self._h, int(i), C.byref(n)))
        buf = torch.empty(max(n.value, 1), dtype=torch.uint8, device=self.device)
        m = np.ascontiguousarray(gb_map, dtype=np.uint8).reshape(-1)
        _check(lib().fkmc_set_gb_map(self._h, int(i), m.ctypes.data, buf.data_ptr(), n.value))
        if not hasattr(self, "_gb_bufs"):
            self._gb_bufs = {}
        self._gb_bufs[int(i)] = buf

    def set_rate_table(self, i: int, k12):
        _check(lib().fkmc_set_rate_table(self._h, i, _dbl(k12), 12))

    def get_rate_table(self, i: int) -> np.ndarray:
        o = (C.c_double * 12)()
        _check(lib().fkmc_get_rate_table(self._h, i, o, 12))
        return np.array(o[:])

    def quantisation(self, i: int):
        q = C.c_double()
        r = C.c_double()
        _check(lib().fkmc_quantisation(self._h, i, C.byref(q), C.byref(r)))
        return q.value, r.value

    # ---------------------------------------------------------------- dynamics
    def advance(self, t_sync, max_cycles: int = 1, min_hops: int = 0):
        ts = _dbl(np.broadcast_to(np.asarray(t_sync, dtype=np.float64), self.n))
        _check(lib().fkmc_advance(self._h, ts, int(max_cycles), int(min_hops)))

    def run_phase(self, t_sync, colour: int):
        ts = _dbl(np.broadcast_to(np.asarray(t_sync, dtype=np.float64), self.n))
        _check(lib().fkmc_run_phase(self._h, ts, int(colour)))

    def sync(self):
        _check(lib().fkmc_sync(self._h))

    SCHEDULES = {"auto": 0, "lockstep": 1, "persistent": 2}

    def set_schedule(self, schedule: str = "auto", waves: int = 0):
        _check(lib().fkmc_set_schedule(self._h, self.SCHEDULES[schedule], int(waves)))

    def checkpoint(self, i: int) -> bytes:
        n = C.c_size_t()
        _check(lib().fkmc_checkpoint_size(self._h, i, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().fkmc_checkpoint(self._h, i, buf, n.value))
        return buf.raw

    def restore(self, i: int, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        _check(lib().fkmc_restore(self._h, i, buf, len(data)))

    def set_graph(self, on: bool):
        _check(lib().fkmc_set_graph(self._h, 1 if on else 0))

    def advance_atomic(self, n_frg: int, n_stages: int):
        """Atom-selection fragment kMC with null events (Eqs. AtomP and
        TimeStepFrg) on a set of plain lattices of at most 8192 vacancies:
        n_stages stages of n_frg selected vacancies each."""
        _check(lib().fkmc_advance_atomic(self._h, int(n_frg), int(n_stages)))

    def set_group(self, group: int = 0):
        """Tiles per wavefront (0 automatic; 1, 2, 4 or 8)."""
        _check(lib().fkmc_set_group(self._h, int(group)))

    def set_plain_lds(self, on: bool):
        """Plain lattices that fit run in LDS in the persistent kernel (True,
        default) or every plain lattice runs the HBM kernel (False)."""
        _check(lib().fkmc_set_plain_lds(self._h, 1 if on else 0))

    def set_timing(self, on: bool):
        _check(lib().fkmc_set_timing(self._h, 1 if on else 0))

    def phase_timing(self):
        ms = C.c_double()
        n = C.c_uint64()
        _check(lib().fkmc_phase_timing(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # ---------------------------------------------------------------- read-out
    def read_state(self, i: int, with_disp: bool = True):
        N = self.geoms[i].n_sites
        occ = np.empty(N, dtype=np.int8)
        disp = np.empty((N, 3), dtype=np.int32) if with_disp else None
        _check(lib().fkmc_read_state(self._h, i, occ.ctypes.data,
                                     disp.ctypes.data if with_disp else None, N))
        return occ, disp

    def read_stats(self):
        arr = (Stats * self.n)()
        _check(lib().fkmc_read_stats(self._h, arr))
        return [s.to_dict() for s in arr]
