"""FP64 CPU oracle for Chebyshev-filtered subspace iteration on a real-space grid.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP path; the only common
code is the seeded input generator in ``synth``.

Every function is a plain, slow, obviously-correct restatement of what the
method computes (NumPy / SciPy, float64), citing the passage of the paper it
follows.  Where the paper is silent the reading used is stated next to the
code.  Layout conventions: vectors are ``[N, M]`` in *rank* order (the curve
order of the grid points), with the Euclidean inner product (no h^3 factor).
"""
from . import grid, hamiltonian, chfsi, scf  # noqa: F401
