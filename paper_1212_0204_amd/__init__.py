"""MI355X (gfx950) library for the High Order Fast Kinetic Scheme (HOFKS) of
Dimarco & Loubere, arXiv:1212.0204: Python binding over the C ABI of
``include/hofks.h``.  PyTorch provides the device workspace and the stream;
every step of the scheme runs in the library's HIP kernels.
"""
from .mlp import ClosureNet  # noqa: F401
from .solver import Batch, HofksError, Solver  # noqa: F401
