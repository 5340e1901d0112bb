"""MI355X-native data-parallel Gibbs sampler for Horseshoe Probit regression.

The sampler itself is the HIP library libhsp.so behind the C ABI of
include/hsp.h; this package holds its sources (csrc/), its build script and a
thin ctypes binding (hsp.py).
"""
from .hsp import Batch, Sampler, HspError, load  # noqa: F401
