"""CPU oracle of the eduPIC PIC/MCC step -- TEST INFRASTRUCTURE ONLY.

Plain single-threaded C in FP64 (oracle.c), written from the paper's
algorithms, plus its ctypes binding (binding.py).  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the GPU library
never does.
"""
