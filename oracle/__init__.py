"""Plain FP64 CPU oracle for lagged-diffusivity TV deblurring with reflective
and anti-reflective boundary conditions.

Method: Bai, Donatelli, Serra-Capizzano, "Fast Preconditioners for Total
Variation Deblurring with Anti-Reflective Boundary Conditions" (arXiv
1011.5964).  Every function cites the section / equation it follows.

THIS PACKAGE IS TEST INFRASTRUCTURE.  It is the slow, obviously-correct
reference that the HIP path is checked against.  Only the test-suite, the
smoke check of the package entry point and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the GPU library: no kernels,
headers, tables, helpers or pre-/post-processing.  It imports nothing from the
GPU package; inputs are produced by the separate seeded generator and passed in.

Arithmetic is IEEE float64 throughout (the paper's MATLAB default precision).
Library primitives used as single steps: numpy/scipy convolution and
correlation, scipy.fft DCT-II/DST-I, dense matmul, numpy.linalg.solve.

Parity status of each part is recorded where it is defined; every public
function here is pinned by at least one test in tests/test_oracle_*.py.
"""

from .operators import (  # noqa: F401
    extension_matrix,
    extend,
    blur,
    blur_adjoint,
    forward_diff,
    forward_diff_adjoint,
    kappa,
    tv_apply,
    tv_diagonal,
    tv_objective,
    tv_gradient,
    normal_apply,
    dense_matrix,
)
from .transforms import (  # noqa: F401
    basis_matrix,
    transform_2d,
    inverse_transform_2d,
    symbol_grid,
    psf_symbol_eigenvalues,
)
from .precond import (  # noqa: F401
    VARIANTS,
    precond_setup,
    precond_setup_dense,
    precond_apply,
)
from .solver import pcg, fp_solve  # noqa: F401
from .adjoint import fp_adjoint, fp_adjoint_dense  # noqa: F401
from .reblur import (  # noqa: F401
    REBLUR_VARIANTS,
    ar_transform_matrix,
    ar_transform_inverse_matrix,
    ar_coefficients_2d,
    ar_synthesis_2d,
    ar_projection,
    ar_projection_level2,
    ar_end_weights,
    ar_extend_eigs,
    reblur_apply,
    reblur_precond_setup,
    reblur_precond_apply,
    pbicgstab,
    fp_solve_reblur,
)
