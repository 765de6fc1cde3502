"""CPU FP64 oracle for the FFT-accelerated multi-block Poisson solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or run this package; only the tests, the smoke check and the bench's CPU
baseline leg do.  It shares no code with the HIP library: no kernels, headers,
tables, constant generators, pre- or post-processing.

What it computes is the plain discrete solution p of L_h p = f, where L_h is
the cell-centred second-order finite-volume Laplacian of Eq. (8) (7-point
stencil) generalised to non-uniform x-y spacing, on a multi-block x-y
cross-section extruded along a uniform z direction, with homogeneous staggered
boundary conditions (Sec. 2, Sec. 3.1).  Three independent routes:

  * ``solve_alg1``   -- Algorithm 1: closed-form eigenfunction transform along z
                        (Table 1), one sparse direct 2D solve per mode of the
                        shifted system Eq. (9), inverse transform;
  * ``solve_separable`` -- single boxes: eigen-decomposition of the 1D
                        operators along all three axes (matrix decomposition,
                        the direct two-direction route of Sec. 2);
  * ``solve_dense``  -- tiny grids: full 3D matrix assembled cell by cell with
                        Python loops and solved by dense LU.

Where the operator is singular (no Dirichlet condition anywhere) the rhs must
have zero volume-weighted sum and the solution is gauged to zero
volume-weighted mean.
"""
from .transforms import basis, eigenvalues, table1_unnormalised, KINDS  # noqa: F401
from .grid import Geometry  # noqa: F401
from .operator import apply_3d, assemble_2d, assemble_3d_dense, second_difference_1d  # noqa: F401
from . import projection  # noqa: F401
from .solve import (  # noqa: F401
    solve, solve_alg1, solve_separable, solve_dense, residual, rel_residual,
    rel_error, project_compatible, remove_mean, is_singular, modal_rhs, solve_mode,
)
