"""Physics of the HIP path at scale: thousands of independent one-vacancy
lattices in one set, against the closed forms the oracle is pinned to
(Eqs. RateCnst1, TimeStep): D = Gamma_tot d^2 / 6 with Gamma_tot =
8 nu exp(-Ea/k_B T) and d = a/sqrt(2), and the biased drift
v = (4a/3)(k+ - k-).  The synchronisation window gives h = 0.1 hops per
vacancy per cycle; the exact phase propagators of these lattices put the
splitting bias of D and v there at 1e-4 to 2e-4, far inside the statistical
error of 2048 replicas."""
import math

import numpy as np
import pytest

from tests import brute
from tests.common import Case, gpu_set, say

pytestmark = pytest.mark.gpu

A = 3.905
KB = 1.380649e-23 / 1.602176634e-19


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _displacements(g, n):
    """Displacement (units of a/2) of the single vacancy of each lattice."""
    out = np.zeros((n, 3))
    for i in range(n):
        occ, disp = g.read_state(i)
        out[i] = disp[np.nonzero(occ == 2)[0][0]]
    return out


@pytest.mark.parametrize("L,frag,plain", [(4, 4, False), (4, 2, False), (4, 0, True)])
def test_single_vacancy_diffusion_closed_form(L, frag, plain):
    """Single-fragment path (frag 4 on 4^3), tile groups (frag 2), plain BKL."""
    T, Ea, R = 600.0, 0.6, 2048
    k = 1e13 * math.exp(-Ea / (KB * T))
    gam = 8 * k
    t_end = 300.0 / gam
    cases = [Case((L,) * 3, (frag,) * 3, seed=77, lattice_id=i, nv=1, nh=0, T=T, Ea_O=Ea)
             for i in range(R)]
    say("one-vacancy diffusion", L, frag, plain)
    g = gpu_set(cases)
    if plain:
        g.advance([t_end] * R, max_cycles=0, min_hops=10**9)
    else:
        t_sync = 0.1 / gam
        g.advance([t_sync] * R, max_cycles=int(round(t_end / t_sync)), min_hops=0)
    st = g.read_stats()
    t = np.array([s["t"] for s in st])
    assert np.allclose(t, t_end, rtol=1e-9)
    r2 = (_displacements(g, R) ** 2).sum(axis=1) * (A / 2) ** 2
    D_est = r2.mean() / (6 * t_end)
    se = r2.std(ddof=1) / math.sqrt(R) / (6 * t_end)
    D_ref = gam * (A / math.sqrt(2)) ** 2 / 6
    say("  D %.5g ref %.5g (%.2f sigma)" % (D_est, D_ref, (D_est - D_ref) / se))
    assert abs(D_est - D_ref) < 4 * se
    assert se / D_ref < 0.05


def test_biased_drift_closed_form():
    """One vacancy under a field along z, uniform start: v = (4a/3)(k+ - k-)."""
    T, Ea, E, R = 600.0, 0.6, 2e8, 2048
    kp = brute.arrhenius(1e13, Ea, T, E, 2.0, 0.5)
    km = brute.arrhenius(1e13, Ea, T, E, 2.0, -0.5)
    v_ref = 4 * A / 3 * (kp - km)
    gam = 8 * kp
    t_end = 200.0 / gam
    t_sync = 0.1 / gam
    cases = [Case((3, 3, 3), (3, 3, 3), seed=78, lattice_id=i, nv=1, nh=0, T=T, Ea_O=Ea, E_z=E)
             for i in range(R)]
    say("one-vacancy drift")
    g = gpu_set(cases)
    g.advance([t_sync] * R, max_cycles=int(round(t_end / t_sync)), min_hops=0)
    z = _displacements(g, R)[:, 2] * A / 2
    v_est = z.mean() / t_end
    se = z.std(ddof=1) / math.sqrt(R) / t_end
    say("  v %.5g ref %.5g (%.2f sigma)" % (v_est, v_ref, (v_est - v_ref) / se))
    assert abs(v_est - v_ref) < 4 * se
    assert se / v_ref < 0.05


@pytest.mark.parametrize("n_frg", [1, 8])
def test_atom_selection_single_vacancy_closed_form(n_frg):
    """The atom-selection scheme (Eqs. AtomP and TimeStepFrg) on one
    vacancy: never null, one hop per stage, D = Gamma_tot d^2 / 6."""
    T, Ea, R, n = 600.0, 0.6, 2048, 300
    k = 1e13 * math.exp(-Ea / (KB * T))
    gam = 8 * k
    cases = [Case((4, 4, 4), seed=79, lattice_id=i, nv=1, nh=0, T=T, Ea_O=Ea) for i in range(R)]
    say("one-vacancy atom selection", n_frg)
    g = gpu_set(cases)
    g.advance_atomic(n_frg, n)
    st = g.read_stats()
    assert all(int(s["hops"].sum()) == n for s in st)
    t = np.array([s["t"] for s in st])
    r2 = (_displacements(g, R) ** 2).sum(axis=1) * (A / 2) ** 2
    D_est = r2.mean() / (6 * t.mean())
    se = r2.std(ddof=1) / math.sqrt(R) / (6 * t.mean())
    D_ref = gam * (A / math.sqrt(2)) ** 2 / 6
    say("  D %.5g ref %.5g (%.2f sigma)" % (D_est, D_ref, (D_est - D_ref) / se))
    assert abs(t.mean() - n / gam) < 4 * t.std(ddof=1) / math.sqrt(R)
    assert abs(D_est - D_ref) < 4 * se + 0.01 * D_ref
    assert se / D_ref < 0.05

