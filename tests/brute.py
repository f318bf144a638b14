"""Brute-force checkers built independently of the oracle's code.

Geometry comes from real-space positions (anion sites at the cube face
centres, neighbours found by Euclidean distance a/sqrt(2)), not from any hop
table; generators of the continuous-time Markov chain are assembled by
enumerating configurations; propagators come from scipy.linalg.expm.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.linalg import expm

KB = 1.380649e-23 / 1.602176634e-19  # eV/K from the exact SI constants
OFF = np.array([[0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])  # face centres, units of a


def sites(L):
    """List of (index, cell, type, position in units of a) in canonical order."""
    Lx, Ly, Lz = L
    out = []
    for k in range(Lz):
        for j in range(Ly):
            for i in range(Lx):
                for t in range(3):
                    n = ((k * Ly + j) * Lx + i) * 3 + t
                    out.append((n, (i, j, k), t, np.array([i, j, k], float) + OFF[t]))
    return out


def neighbours(L):
    """For each site: list of (target index, displacement vector in units of a)
    over all sites at minimum-image distance sqrt(1/2)."""
    S = sites(L)
    Lv = np.array(L, float)
    pos = np.array([s[3] for s in S])
    nb = []
    for n, _, _, p in S:
        d = pos - p
        d -= Lv * np.round(d / Lv)
        r2 = (d * d).sum(axis=1)
        idx = np.nonzero(np.abs(r2 - 0.5) < 1e-9)[0]
        nb.append([(int(m), d[m]) for m in idx])
    return nb


def arrhenius(nu, Ea, T, E_z=0.0, q=0.0, dz_a=0.0, a=3.905, gb=0.0):
    """Rate of a vacancy hop whose z displacement is dz_a (units of a):
    barrier Ea + dE/2 with dE = -q E_z dz (eV), plus a boundary term."""
    dE = -q * E_z * dz_a * a * 1e-10
    return nu * math.exp(-(Ea + dE / 2.0 + gb) / (KB * T))


def generator(L, n_v, n_h, rate_fn, edge_filter=None):
    """Generator matrix Q (rows = from, Q[i,j] = rate i->j) over all placements
    of n_v vacancies and n_h H (rest O) on the lattice.  rate_fn(species of
    the ion, displacement of the vacancy, src, dst) gives each hop's rate;
    edge_filter(src, dst) restricts to a subset of edges (one phase)."""
    S = sites(L)
    N = len(S)
    nb = neighbours(L)
    states = []
    for vs in itertools.combinations(range(N), n_v):
        rest = [s for s in range(N) if s not in vs]
        for hs in itertools.combinations(rest, n_h):
            occ = np.zeros(N, np.int8)
            occ[list(vs)] = 2
            occ[list(hs)] = 1
            states.append(occ)
    index = {s.tobytes(): i for i, s in enumerate(states)}
    Q = np.zeros((len(states), len(states)))
    for i, occ in enumerate(states):
        for v in np.nonzero(occ == 2)[0]:
            for (m, d) in nb[v]:
                if occ[m] == 2:
                    continue
                if edge_filter is not None and not edge_filter(int(v), m):
                    continue
                new = occ.copy()
                new[v], new[m] = occ[m], 2
                j = index[new.tobytes()]
                Q[i, j] += rate_fn(int(occ[m]), d, int(v), m)
    Q -= np.diag(Q.sum(axis=1))
    return states, index, Q


def propagate(Q, t):
    return expm(Q * t)


def chi2_pvalue(counts, probs, min_expected=5.0):
    """Pearson chi-square p-value, pooling bins with small expectation."""
    from scipy.stats import chi2
    counts = np.asarray(counts, float)
    n = counts.sum()
    e = np.asarray(probs, float) * n
    order = np.argsort(e)
    c_s, e_s = counts[order], e[order]
    pc, pe, bc, be = [], [], 0.0, 0.0
    for c, x in zip(c_s, e_s):
        bc += c
        be += x
        if be >= min_expected:
            pc.append(bc)
            pe.append(be)
            bc, be = 0.0, 0.0
    if be > 0 and pe:
        pc[-1] += bc
        pe[-1] += be
    pc, pe = np.array(pc), np.array(pe)
    stat = ((pc - pe) ** 2 / pe).sum()
    dof = max(len(pc) - 1, 1)
    return stat, float(chi2.sf(stat, dof))
