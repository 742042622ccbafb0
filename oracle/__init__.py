"""FP64 CPU oracle for the anelastic pressure projection.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow reference that the
HIP path is checked against. Only the tests, the smoke check and the bench's
CPU-baseline leg may import it; the product path never does.

Modules: projection (the separable projection, Sec. 4's FFT solver),
reductions (per-level horizontal mean and max, the I/O server's reduction
of Sec. 3) and variable (the projection with a density varying in x, y and
z, solved directly: the problem of the Krylov solver of Secs. 4-5).

Parity pinned: every function here is checked against brute force, a library
closed form, manufactured solutions, continuum convergence and invariants in
tests/test_oracle_pins.py.
"""
from .projection import (  # noqa: F401
    vertical_grid,
    divergence,
    gradient,
    tridiag_coefficients,
    modified_wavenumbers,
    forward_spectrum,
    solve_columns,
    inverse_spectrum,
    project,
    weighted_energy,
)
from .reductions import level_stats  # noqa: F401
from .variable import divergence_var, operator_matrix, project_var  # noqa: F401
