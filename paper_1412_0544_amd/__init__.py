"""MI355X-native classical RK4 for large periodic nearest-neighbour chains.

The HIP library (``libchainrk4.so``, C ABI in ``include/chain_rk4.h``) does
all of the arithmetic; this package only marshals arguments to it, with torch
supplying device memory and streams.
"""
from ._lib import ChainError, lib  # noqa: F401
from .chain import Chain, MODELS, METHODS, PRECS, RoesslerChain, state_dtype  # noqa: F401
from .batch import Batch  # noqa: F401

__all__ = ["Batch", "Chain", "ChainError", "lib", "MODELS", "METHODS", "PRECS", "RoesslerChain",
           "state_dtype"]
