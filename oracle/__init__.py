"""CPU oracle for the four-field DPP solve -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or link anything in this package.  The GPU
library never uses it; the two share no code.  Only the seeded input
generators (``dpp_inputs``) feed both.

Contents (each function cites the passage of the paper it follows):
  * ``dpp``:    mesh, CG-VMS assembly of K and f (C, FP64), field layout, block
                extraction, direct solves, ``selfp`` Schur approximation.
  * ``mg``:     the multigrid V-cycle used on the pressure Schur blocks, the
                Chebyshev smoother and its eigenvalue estimate.  The paper uses
                an algebraic multigrid package here; this build's own geometric
                V-cycle is defined in the module and is pinned by invariants,
                not by values printed in the paper.
  * ``solver``: the Schur-complement fieldsplit preconditioner, flexible GMRES,
                the adjoint solve and its parameter gradient.
  * ``post``:   L2 errors against the manufactured solutions, boundary fluxes
                and pressure integrals for the mass-balance check.
"""
