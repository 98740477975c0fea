"""MI355X (gfx950) solver for the four-field double porosity/permeability
model: CG-VMS P1 assembly, Schur-complement fieldsplit preconditioner with
geometric multigrid V-cycles on the pressure Schur blocks, flexible GMRES,
mixed precision, adjoint.

Thin ctypes binding over ``libdpp.so`` (C ABI in ``include/dpp.h``).  torch
supplies device memory and streams; every numerical step runs in the HIP
library.  The binding fails loudly when the library is not built.
"""
from ._binding import (  # noqa: F401
    DppError, Problem, Precond, SolveStats, assemble, assemble_problem, default_opts,
    lib, lib_path, DppSolve, STATUS, profile_enable, profile_read, PROFILE_FAMILIES,
    Batch, assemble_batch, simplex_rule,
)
