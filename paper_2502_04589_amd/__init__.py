"""MI355X (gfx950) augmented subspace eigensolver: Python binding of libpase.

Every step of the method runs in the HIP kernels of libpase.so; this module
only marshals arguments.  PyTorch provides device memory and the stream.
"""
from .solver import CsrMatrix, PaseError, Solver  # noqa: F401
from .learned import UNet  # noqa: F401
