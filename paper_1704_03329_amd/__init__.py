"""mdpl: MI355X-native short-range molecular-dynamics pair loops.

The compute path is the HIP library ``libmdpl.so`` (sources in ``csrc/``,
ABI in ``include/mdpl.h``).  ``mdpl`` is its ctypes binding, ``sim`` holds
thin allocation helpers, ``autograd`` the differentiable energy.
"""
from . import mdpl  # noqa: F401

__all__ = ["mdpl"]
