"""FINGER search on MI355X (gfx950): a HIP library (libfinger.so, C ABI in
include/finger.h) and its thin Python binding.

Importing the package does not load the library; the first call does, and
fails loudly if it has not been built.
"""
from ._lib import (  # noqa: F401
    ANGULAR, CODE_BF16, CODE_F32, CODE_FP8E4M3, COUNTER_NAMES, L2, MODE_FINGER,
    MODE_GATED, MODE_PLAIN, NCOUNTERS, SIGMA_STD, SIGMA_VARIANCE, FingerError,
)
