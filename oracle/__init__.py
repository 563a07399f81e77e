"""CPU oracle of the L-HWENO hot path (test infrastructure only).

Importable by the tests, the smoke check and the CPU-baseline leg of the
benchmark; never by the product package.
"""
from .hweno_ref import *  # noqa: F401,F403
