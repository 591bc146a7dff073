"""FP64 CPU oracle for Adaptive-Multilevel BDDC (Sousedik, Sistek, Mandel).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference the
GPU library is checked against.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the library never does,
and nothing here imports the library.  It shares no code with the GPU path
apart from the seeded input generators in ``workloads``.

Everything is dense numpy/scipy in float64, written step by step from the
paper's definitions:

* ``fem``          -- Q1 element matrices and assembly (Section 2 setting).
* ``substructure`` -- globs, interface, weights, initial constraints,
                      Schur complements, coarse basis (Sections 2, 5, 7).
* ``adaptive``     -- pair generalized eigenproblems, selection, constraint
                      rows (Section 4, eq. eig-matrix, Prop. 1, Alg. 2).
* ``bddc``         -- multilevel BDDC application (Alg. 1), the level
                      hierarchy (Alg. 3) and PCG with a Lanczos condition
                      estimate (Section 8).
* ``adjoint``      -- element log-coefficient gradient of a misfit.

Functions without an external pin say "parity unpinned" in their docstring.
"""
from .fem import (element_matrix_poisson, element_matrix_elasticity, element_matrices,
                  assemble_global, rigid_modes)
from .substructure import build_level, level1_input, LevelInput, Level
from .adaptive import pair_eigenproblem, enrich_level
from .bddc import (Hierarchy, setup_hierarchy, bddc_apply, pcg, lanczos_cond,
                   direct_solve, solve_problem, interior_solution)
from .adjoint import misfit_gradient

__all__ = [
    "element_matrix_poisson", "element_matrix_elasticity", "element_matrices",
    "assemble_global", "rigid_modes", "build_level", "level1_input", "LevelInput",
    "Level", "pair_eigenproblem", "enrich_level", "Hierarchy", "setup_hierarchy",
    "bddc_apply", "pcg", "lanczos_cond", "direct_solve", "solve_problem",
    "interior_solution", "misfit_gradient",
]
