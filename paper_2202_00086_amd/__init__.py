"""MI355X (gfx950) backward ray tracing of null geodesics in Kerr spacetime.

The compute path is libkerrtrace.so (hand-written HIP kernels behind the C
ABI of include/kerrtrace.h); kerrtrace.py is its ctypes binding.
"""
