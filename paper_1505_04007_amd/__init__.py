"""MI355X (gfx950) FDTD-PIC library for surface-plasmon excitation by an
electron bunch near a Drude metal film (arXiv:1505.04007).

The compute path is the HIP library ``libpic.so`` behind the C ABI in
``include/pic.h``; :mod:`paper_1505_04007_amd.native` is its ctypes binding.
"""
from .native import (BC_CPML, BC_PEC, BC_PERIODIC, FIELD_E, FIELD_H, FIELD_JB, FIELD_JPOL, Batch,  # noqa
                     PicError, Simulation, from_workload, load, query_sizes, spp_power, workload_sizes)

__all__ = ["Simulation", "Batch", "from_workload", "load", "spp_power", "query_sizes", "workload_sizes",
           "PicError", "BC_PEC", "BC_PERIODIC", "BC_CPML", "FIELD_E", "FIELD_H", "FIELD_JPOL", "FIELD_JB"]
