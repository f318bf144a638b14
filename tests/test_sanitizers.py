"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU builds only; the GPU code is not
instrumented).  The oracle runs its own dynamics on ragged, minimal,
crowded, field and boundary-plane lattices in all three modes; the host
driver feeds the library's host entry points random and invalid
geometries and parameters."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ORACLE_RUN = r"""
import sys
sys.path.insert(0, %r)
from oracle import oracle as O
cases = [((5, 4, 6), (2, 3, 2), 6, 20), ((2, 2, 2), (2, 2, 2), 3, 4), ((7, 6, 5), (4, 4, 4), 40, 30),
         ((6, 6, 6), (0, 0, 0), 20, 40), ((4, 4, 4), (0, 0, 0), 60, 10), ((9, 7, 11), (4, 3, 5), 15, 0)]
for k, (L, F, nv, nh) in enumerate(cases):
    g = O.Geometry(L=L, frag=F, seed=7, lattice_id=k, gb_period_cells=2, gb_axes_mask=7)
    lat = O.Lattice(g)
    lat.init_random(nv, nh)
    lat.set_rates(O.RateParams(T=650.0, Ea_O=0.6, Ea_H=0.45, E_z=1e8, q=2.0, gb_period_cells=2,
                               gb_axes_mask=7, gb_dE=0.05))
    if F[0]:
        lat.advance(2.0 / (8 * lat.k12[0]), max_cycles=3)
        lat.advance(2.0 / (8 * lat.k12[0]), max_cycles=100, min_hops=200)
    else:
        lat.advance_plain(500)
        lat.advance_plain(10**6, t_horizon=20.0 / (8 * lat.k12[0]))
        lat.advance_atomic(7, 40)
    st = lat.stats()
print("oracle ok")
"""


def _asan_runtime():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    asan = _asan_runtime()
    if not asan:
        pytest.skip("no libasan")
    with tempfile.TemporaryDirectory() as d:
        so = os.path.join(d, "libfkmc_oracle_san.so")
        subprocess.check_call(["gcc", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                               "-o", so, os.path.join(ROOT, "oracle", "fkmc_oracle.c"), "-lm"])
        env = dict(os.environ, LD_PRELOAD=asan, FKMC_ORACLE_LIB=so,
                   ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([sys.executable, "-c", ORACLE_RUN % ROOT], env=env, capture_output=True,
                           text=True, timeout=600)
        assert r.returncode == 0 and "oracle ok" in r.stdout, r.stderr[-3000:]
        assert "runtime error" not in r.stderr, r.stderr[-3000:]


def test_library_host_code_under_address_and_undefined_behaviour_sanitizers():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("no hipcc")
    csrc = os.path.join(ROOT, "paper_2004_09081_amd", "csrc")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sanitize_host")
        cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=undefined",
               "-o", exe, os.path.join(ROOT, "tests", "sanitize_host.cpp"),
               os.path.join(csrc, "fkmc_api.hip"), os.path.join(csrc, "fkmc_device.hip"),
               os.path.join(csrc, "fkmc_mlp.hip")]
        subprocess.run(cmd, check=True, capture_output=True, timeout=900)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
        assert r.returncode == 0 and "0 unexpected" in r.stdout, (r.stdout, r.stderr[-3000:])
        assert "runtime error" not in r.stderr, r.stderr[-3000:]
