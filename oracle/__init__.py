"""Plain FP64 CPU oracle for the frequency/time hybrid wave solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library
never calls it and shares no code, table or constant with it.
"""
from .fhw_oracle import *  # noqa: F401,F403
