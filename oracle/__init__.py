"""Plain FP64 CPU oracle for the gradient-domain stack solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the HIP path.

What it computes (Kazhdan et al., "Gradient-Domain Processing for Large EM
Image Stacks"):

* ``grid``      -- the discrete gradient/divergence on a regular voxel grid with
                   natural (Neumann) boundaries, the screened anisotropic
                   operator (alpha - div W grad) of Sec. 4, the right-hand sides
                   of Eq. (1) (anisotropic diffusion, AD), Eq. (2)
                   (per-slice screened Poisson, SP) and of the general Sec. 4
                   system, and the discrete energies they minimise.
* ``assemble``  -- the same operator as an explicit sparse matrix.
* ``solvers``   -- the solution of those systems: dense direct solve (tiny
                   grids), conjugate gradients on the matrix-free operator, and
                   the exact DCT-II diagonalisation that is the discrete form of
                   the frequency-space analysis of Sec. 3.2.
* ``npr``       -- the gradient-modulation filter of Sec. 6 (the general
                   system with the input's gradients scaled by
                   lambda (1 - exp(-|grad|^2 / 2 sigma^2))), its limits and energy.
* ``hybrid``    -- the steps of the "Hybrid" discretisation of Sec. 4.2:
                   B-spline prolongation (1/2, 1, 1/2), its transpose, Galerkin
                   coarse operators from per-axis 1-D tables, 8-colour GS.
* ``linear``    -- the "Linear" discretisation of Sec. 4.2 (trilinear B-spline
                   finite elements): mass/stiffness tables, the AD right-hand
                   side and its solution (a different answer from the 7-point one).
* ``mgsteps``   -- single multigrid steps (Sec. 4.1): one red-black
                   Gauss-Seidel sweep, the residual, restriction by summing
                   children, constant and cell-centred trilinear prolongation,
                   and the canonical relative residual of the Table 1 caption.

Every array is float64, laid out ``[nz][ny][nx]`` (x fastest).  Weights are
``beta = (beta_x, beta_y, beta_z)``; grid spacing is 1 in every axis, so all
anisotropy enters through beta.

Parity pins (tests marked ``not gpu``) tie each function to something other
than itself: closed-form eigenvalues, dense solves, the DCT diagonalisation,
the identity and offset-removal invariants of Sec. 3, brute-force energy
minimisation on tiny grids, and the 1-D aliasing example of Fig. 2.
"""

from . import grid, assemble, solvers, mgsteps  # noqa: F401
