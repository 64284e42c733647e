"""FP64 CPU oracle for the IGR compressible-Euler right-hand side.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import
this package.  The product path (the HIP library and its Python binding)
never imports, calls or links anything here, and nothing here imports the
product package.

Paper: "Simulating many-engine spacecraft: Exceeding 1 quadrillion degrees of
freedom via information geometric regularization" (arXiv 2505.07392).
Section names below refer to that paper; equation numbers follow its LaTeX
order: (1)-(3) Navier-Stokes balances, (4) ideal-gas state equation,
(5) constitutive law, (6)-(8) the IGR-modified balances and (9) the
entropic-pressure (elliptic) equation.

Modules
-------
``igr_ref``  plain whole-array torch-float64 implementation of one RHS
             evaluation, the Sigma Jacobi solve, SSP-RK3, dt and sums.
``riemann``  exact Riemann solver for the 1D Euler equations (Sod pin).

Parity status of each function is stated in its module header.
"""

from . import igr_ref, riemann  # noqa: F401
