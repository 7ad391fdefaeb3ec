"""Seeded synthetic inputs shared by the FP64 reference and the HIP library.

Holds random-number draws and gate-list layout only; no simulation arithmetic.
"""
from .circuits import *  # noqa: F401,F403
from .circuits import Gate, BitSwap  # noqa: F401
