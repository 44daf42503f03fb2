"""MI355X implementation of the MORE-Stress hot path (arXiv 2411.12690).

The library ``libmos.so`` (HIP, gfx950) holds every stage: unit-cell FE
assembly, the multi-RHS local solves and Galerkin projection, the
element-by-element PCG solve of the reduced array system and the batched
stress reconstruction.  ``mos`` is its ctypes binding; ``build`` compiles it.
"""
from . import mos  # noqa: F401
from .mos import (Context, MosError, mos_array_layout, mos_build_cell, mos_cell_export,  # noqa: F401
                  mos_get_solution, mos_reconstruct, mos_reduce, mos_rom_export, mos_solve_array)
