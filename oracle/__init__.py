"""CPU oracle for SIDWT correlation -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product (the HIP library and its Python binding)
never does.
"""
from .sidwt_oracle import *  # noqa: F401,F403
from . import sidwt_oracle  # noqa: F401
