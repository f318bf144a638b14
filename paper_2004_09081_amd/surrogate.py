"""Python binding of the surrogate ensemble (fkmc_mlp_* in include/fkmc.h),
the kMC label generation for it, and the surrogate-with-fallback query.

Argument marshalling only: training and inference run in the library's
MFMA kernels; labels come from the library's batched kMC.
"""
from __future__ import annotations

import ctypes as C
import math
import time

import numpy as np

from . import fkmc as F

_SIGS = {
    "fkmc_mlp_query_sizes": [C.c_uint32, C.c_uint32, C.POINTER(C.c_size_t)],
    "fkmc_mlp_create": [C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p, C.c_size_t, C.c_void_p,
                        C.POINTER(C.c_void_p)],
    "fkmc_mlp_destroy": [C.c_void_p],
    "fkmc_mlp_set_data": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32],
    "fkmc_mlp_train": [C.c_void_p, C.c_uint32, C.c_uint32, C.c_float, C.c_void_p],
    "fkmc_mlp_grad": [C.c_void_p, C.c_void_p, C.c_void_p],
    "fkmc_mlp_predict": [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p],
    "fkmc_mlp_get_params": [C.c_void_p, C.c_void_p, C.c_size_t],
    "fkmc_mlp_set_params": [C.c_void_p, C.c_void_p, C.c_size_t],
    "fkmc_mlp_get_norm": [C.c_void_p, C.c_void_p],
}
_ready = False


def _lib():
    global _ready
    lib = F.lib()
    if not _ready:
        for name, args in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = C.c_int32
        lib.fkmc_mlp_param_count.restype = C.c_uint32
        _ready = True
    return lib


def _ok(rc, what):
    if rc != 0:
        raise F.FkmcError(rc, what)


N_PARAMS = 17410


class Ensemble:
    """members x MLP(4-128-128-2) in caller-owned device memory."""

    def __init__(self, members: int = 5, seed: int = 0, max_samples: int = 8192,
                 device: str = "cuda:0"):
        import torch
        lib = _lib()
        assert lib.fkmc_mlp_param_count() == N_PARAMS
        self.members = members
        nb = C.c_size_t()
        _ok(lib.fkmc_mlp_query_sizes(members, max_samples, C.byref(nb)), "query_sizes")
        self.dev = torch.device(device)
        self.work = torch.empty(nb.value, dtype=torch.uint8, device=self.dev)
        self.stream = torch.cuda.current_stream(self.dev)
        h = C.c_void_p()
        _ok(lib.fkmc_mlp_create(members, seed, max_samples, self.work.data_ptr(), nb.value,
                                C.c_void_p(self.stream.cuda_stream), C.byref(h)), "create")
        self._h = h
        self._data = None

    def close(self):
        if self._h:
            _lib().fkmc_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, shape):
        import torch
        t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(self.dev)
        assert tuple(t.shape) == shape
        return t

    def set_data(self, X, Y, M):
        n = len(X)
        self._data = (self._dev(X, (n, 4)), self._dev(Y, (n, 2)), self._dev(M, (n, 2)))
        _ok(_lib().fkmc_mlp_set_data(self._h, *[t.data_ptr() for t in self._data], n), "set_data")

    def train(self, steps: int, batch: int = 256, lr: float = 1e-3):
        loss = np.zeros(self.members, np.float32)
        _ok(_lib().fkmc_mlp_train(self._h, steps, batch, C.c_float(lr),
                                  loss.ctypes.data), "train")
        return loss

    def grad(self):
        g = np.zeros((self.members, N_PARAMS), np.float32)
        loss = np.zeros(self.members, np.float32)
        _ok(_lib().fkmc_mlp_grad(self._h, g.ctypes.data, loss.ctypes.data), "grad")
        return g, loss

    def predict(self, X, each: bool = False):
        import torch
        n = len(X)
        x = self._dev(X, (n, 4))
        mean = torch.empty((n, 2), dtype=torch.float32, device=self.dev)
        std = torch.empty_like(mean)
        ev = torch.empty((self.members, n, 2), dtype=torch.float32, device=self.dev) if each else None
        _ok(_lib().fkmc_mlp_predict(self._h, x.data_ptr(), n, mean.data_ptr(), std.data_ptr(),
                                    ev.data_ptr() if each else None), "predict")
        torch.cuda.synchronize(self.dev)
        out = (mean.cpu().numpy(), std.cpu().numpy())
        return out + ((ev.cpu().numpy(),) if each else ())

    def get_params(self):
        p = np.zeros((self.members, N_PARAMS), np.float32)
        _ok(_lib().fkmc_mlp_get_params(self._h, p.ctypes.data, p.size), "get_params")
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _ok(_lib().fkmc_mlp_set_params(self._h, p.ctypes.data, p.size), "set_params")

    def get_norm(self):
        o = np.zeros(12, np.float32)
        _ok(_lib().fkmc_mlp_get_norm(self._h, o.ctypes.data), "get_norm")
        return o


# --------------------------------------------------------------------------- kMC labels
MIN_HOPS = 1000  # a species' D is a label only with at least this many hops


def features(specs) -> np.ndarray:
    from .workloads import surrogate_features
    return np.stack([surrogate_features(s) for s in specs]).astype(np.float64)


def kmc_labels(specs, hop_target: int = 0, waves: int = 4, cycles: int = 0,
               schedule: str = "lockstep"):
    """Run the lattices as one batched set (to hop_target hops each, or for
    a fixed number of synchronisation cycles) and return log10 D (m^2/s) of
    O and H with validity masks (at least MIN_HOPS hops of that species).
    Lockstep by default: the label runs are set by their densest large
    lattices, whose tiles the lockstep launches spread over the whole GPU."""
    from .workloads import to_gpu
    geoms, rates = to_gpu(specs, F)
    s = F.LatticeSet(geoms)
    try:
        s.init_random([sp.n_vac for sp in specs], [sp.n_h for sp in specs])
        s.set_rates(rates)
        s.set_schedule(schedule, waves)
        ts = [0.0 if sp.frag[0] == 0 else sp.t_sync for sp in specs]  # plain: no horizon
        if cycles:
            s.advance(ts, max_cycles=cycles, min_hops=0)
        else:
            s.advance(ts, max_cycles=10**9, min_hops=hop_target)
        st = s.read_stats()
    finally:
        s.close()
    Y = np.zeros((len(specs), 2))
    M = np.zeros((len(specs), 2))
    for i, x in enumerate(st):
        for o, sp_idx in enumerate((0, 1)):
            D = x["D"][sp_idx] * 1e-20  # Angstrom^2/s -> m^2/s
            ok = int(x["hops"][sp_idx]) >= MIN_HOPS and x["count"][sp_idx] > 0 and D > 0
            M[i, o] = 1.0 if ok else 0.0
            Y[i, o] = math.log10(D) if ok else 0.0
    return Y, M


def query(ens: Ensemble, specs, hop_target: int = 0, threshold: float = 0.1, cycles: int = 0):
    """Answer log10 D for every spec: surrogate mean where the ensemble's
    population std of every output is <= threshold decades, else a kMC run
    (the fallback).  Returns (answers, served mask, seconds, n_fallback)."""
    t0 = time.perf_counter()
    X = features(specs)
    mean, std = ens.predict(X)
    served = (std <= threshold).all(axis=1)
    ans = mean.astype(np.float64).copy()
    fb = np.nonzero(~served)[0]
    if fb.size:
        Yf, Mf = kmc_labels([specs[i] for i in fb], hop_target, cycles=cycles)
        ans[fb] = np.where(Mf > 0, Yf, np.nan)
    return ans, served, time.perf_counter() - t0, int(fb.size)


# --------------------------------------------------------------------------- configuration 5
def label_fragment_edge(L: int) -> int:
    """Fragment edge of the label runs: 16-cell fragments from 32 cells up
    (few, larger tiles per phase), 8-cell below."""
    return 16 if L >= 32 else 8


def run_cfg5(n_train: int = 4096, n_test: int = 512, cycles: int = 2000, members: int = 5,
             steps: int = 6000, batch: int = 256, threshold: float = 0.1, frag=label_fragment_edge,
             chunk: int = 512, log=None, L_range=None, detail: bool = False):
    """Train the ensemble on kMC labels of n_train lattices drawn from the
    ensemble workload's parameter distribution (own key stream), evaluate on
    n_test held-out lattices (another stream): MAE of served answers against
    kMC, served fraction, and time-to-answer with and without the surrogate.
    Every run lasts `cycles` synchronisation windows (about that many hops
    per vacancy), so a label depends on the four inputs and not on the
    lattice size.  With detail, the report also holds the per-query
    answers, the served mask and the kMC labels with their masks."""
    hops = 0
    from . import workloads as W
    say = log or (lambda *a: None)

    def draw(n, seed):
        specs = W.cfg4(n=n, seed=seed, frag=frag, hops=hops)
        if L_range is not None:
            rng = np.random.default_rng(seed + 1)
            for s in specs:
                L = int(rng.integers(L_range[0], L_range[1] + 1))
                s.L = (L, L, L)
                F_ = frag(L) if callable(frag) else int(frag)
                s.frag = (F_, F_, F_)
                s.n_vac, s.n_h = W.counts(3 * L**3, s.extra["x_v"], s.extra["x_h"])
        return specs

    t0 = time.perf_counter()
    train_specs = draw(n_train, 0xC5A)
    Xtr = features(train_specs)
    Ytr = np.zeros((n_train, 2))
    Mtr = np.zeros((n_train, 2))
    for a in range(0, n_train, chunk):
        Y, M = kmc_labels(train_specs[a:a + chunk], cycles=cycles)
        Ytr[a:a + chunk], Mtr[a:a + chunk] = Y, M
        say("labels %d/%d (%.1f s)" % (min(a + chunk, n_train), n_train, time.perf_counter() - t0))
    t_labels = time.perf_counter() - t0
    ens = Ensemble(members=members, seed=0x5EED, max_samples=max(n_train, n_test))
    ens.set_data(Xtr, Ytr, Mtr)
    t1 = time.perf_counter()
    ens.train(steps // 2, batch=batch, lr=1e-3)
    loss = ens.train(steps - steps // 2, batch=batch, lr=3e-4)
    t_train = time.perf_counter() - t1
    say("trained %d steps in %.2f s, loss %s" % (steps, t_train, np.round(loss, 4)))

    test_specs = draw(n_test, 0xC5B)
    t2 = time.perf_counter()
    Yte, Mte = kmc_labels(test_specs, cycles=cycles)  # kMC alone answers every query
    t_kmc = time.perf_counter() - t2
    ans, served, t_surr, n_fb = query(ens, test_specs, threshold=threshold, cycles=cycles)
    sizes = np.array([s.n_sites for s in test_specs], dtype=np.float64)
    err = np.abs(ans - Yte)
    ok = (Mte > 0) & served[:, None]
    mae = float(err[ok].mean()) if ok.any() else float("nan")
    mae_o = float(err[:, 0][ok[:, 0]].mean()) if ok[:, 0].any() else float("nan")
    mae_h = float(err[:, 1][ok[:, 1]].mean()) if ok[:, 1].any() else float("nan")
    rep = {
        "mae_log10D": mae, "mae_log10D_O": mae_o, "mae_log10D_H": mae_h,
        "served_fraction": float(served.mean()), "fallbacks": n_fb,
        "label_coverage": [float(Mtr[:, 0].mean()), float(Mtr[:, 1].mean())],
        "time_kmc_only_s": t_kmc, "time_surrogate_with_fallback_s": t_surr,
        "speedup": t_kmc / t_surr if t_surr > 0 else None,
        "kmc_runs_fraction_with_surrogate": float(n_fb / max(n_test, 1)),
        "train_runs": n_train, "test_runs": n_test, "cycles_per_run": cycles, "members": members,
        "threshold_decades": threshold, "label_time_s": t_labels, "train_time_s": t_train,
        "final_loss": [float(x) for x in loss],
    }
    if detail:
        rep.update(answers=ans, served=served, kmc=Yte, kmc_mask=Mte)
    return rep
