"""PMKRSA hot path on MI355X (gfx950): batched RSA encryption and CRT decryption.

The compute lives in libpmk.so (HIP kernels behind the C ABI of include/pmk.h);
``binding`` is its ctypes binding, ``inputs`` the seeded synthetic workloads.
"""
from . import binding, inputs  # noqa: F401
from .binding import Context, Plan, PmkError  # noqa: F401

__all__ = ["binding", "inputs", "Context", "Plan", "PmkError"]
