"""MI355X-native flow-based sampler for lattice phi^4 (after arXiv 2208.08903).

The compute path is the HIP library liblfs.so (C ABI in include/lfs.h); the
``lfs`` module is its ctypes binding.  ``flow`` holds the training and
sampling drivers, ``serve`` the continuous-batching sampling server.
"""
from . import lfs  # noqa: F401

__all__ = ["lfs"]
