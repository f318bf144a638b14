"""MI355X-native fragment kinetic Monte Carlo (vacancy-mediated O/H
diffusion in cubic ABO3 perovskites; Nakata, arXiv:2004.09081).

The hot path lives in the HIP library libfkmc.so (C ABI in include/fkmc.h);
``fkmc`` is its Python binding and ``workloads`` holds the standard synthetic
configurations.
"""
from . import fkmc  # noqa: F401
