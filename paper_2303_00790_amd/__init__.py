"""MI355X-native Chebyshev-filtered subspace iteration for real-space
finite-difference Kohn-Sham DFT (blockwise-Hilbert grids, KB projectors).

The compute path is the HIP library ``libchfsi.so`` (C ABI in
``include/chfsi.h``); ``binding`` marshals PyTorch tensors into it.
"""
from . import binding  # noqa: F401
from .binding import (CHF_F32, CHF_F64, ORDER_HILBERT, ORDER_LEX, ChfError, Context,  # noqa: F401
                      Hamiltonian, Scf, ScfParams, gram, orthonormalize, rayleigh_ritz)
