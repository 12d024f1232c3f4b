"""SISPH hot path on MI355X: HIP kernels behind the C ABI of include/sisph.h.

``cases`` builds the seeded synthetic inputs; ``sisph`` is the ctypes binding
of libsisph.so (loaded on first use, never replaced by a CPU path).
"""
from . import cases  # noqa: F401

__all__ = ["cases", "sisph"]
