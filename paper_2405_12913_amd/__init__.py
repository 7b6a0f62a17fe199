"""MI355X-native hot path of Hamiltonian ray tracing (arXiv:2405.12913).

The compute path is the HIP library libhrt.so (C ABI in include/hrt.h); ``hrt`` is its
thin Python binding with the same entry-point names.
"""
from . import hrt  # noqa: F401
from .hrt import Simulation, HRTError  # noqa: F401
