"""bsdmrg: block-sparse two-site DMRG effective-Hamiltonian engine for MI355X.

The compute path lives in libbsdmrg.so (HIP kernels for gfx950 behind the C
ABI of include/bsdmrg.h); ``lib`` is its ctypes binding and ``problems``
marshals seeded inputs into the canonical block layout.
"""
from . import lib  # noqa: F401
