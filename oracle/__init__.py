"""CPU FP64 oracle for Kerr backward ray tracing -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library.
"""
from .oracle import *  # noqa: F401,F403
