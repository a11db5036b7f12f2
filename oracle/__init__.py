"""Plain, slow, FP64 CPU oracle of the SA-AMG preconditioned CG Poisson solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its Python
binding) imports, links or executes anything under ``oracle/``; only the test suite,
the smoke check and the benchmark's CPU-baseline leg use it.

The oracle follows the paper (Adelmann, Arbenz, Ineichen, "A fast parallel Poisson
solver on irregular domains applied to beam dynamics simulations"):

* ``grid``     - lattice, unknowns and wall distances (Section 2, Figure "boundary").
* ``operator`` - 7-point star with constant / linear / quadratic wall extrapolation
                 and the symmetric diagonal scaling (Section 2, eqs. 7pt-star,
                 const_extrapol, lin_extrapol, quad_extrapol, quad_extrapol1).
* ``amg``      - smoothed-aggregation AMG: aggregation into 3^d cubes, tentative and
                 smoothed prolongators, Galerkin coarse operators, Chebyshev smoother,
                 direct coarse solve and the V-cycle of Algorithm 1 (Section 3.2,
                 Table 1).
* ``pcg``      - preconditioned conjugate gradients with the relative-residual stop
                 (Section 3.1, Section 5 stopping criterion).
* ``rows``     - the residual of single rows, computed one by one from the wall rule,
                 for spot checks on grids too large to assemble quickly.

All arithmetic is float64 with numpy / scipy primitives (sparse products, dense
solves); no blocking or fusion is done beyond what the definitions state.
"""
from . import grid, operator, amg, pcg, rows, solve  # noqa: F401
