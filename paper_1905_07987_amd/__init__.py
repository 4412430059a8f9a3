"""MI355X-native ADER-DG step engine (ExaHyPE paper, Sec. 3.3-3.5).

The compute path is the HIP library ``libadg.so`` (sources in ``csrc/``,
C ABI in ``include/adg.h``); ``adg`` is its ctypes binding.
"""
from . import adg
from .adg import AdgError, Solver, basis_tables, max_order

__all__ = ["adg", "AdgError", "Solver", "basis_tables", "max_order"]
