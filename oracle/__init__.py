"""FP64 CPU oracle for the t-SGNE optimisation loop.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library.
"""
from .oracle import *  # noqa: F401,F403
