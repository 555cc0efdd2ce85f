"""MI355X-native PIC/MCC hot path of the eduPIC method (arXiv:2103.09642).

The per-particle time step of a 1D3V electrostatic PIC/MCC simulation of an
argon capacitively coupled RF discharge -- field solve, leapfrog push, Monte
Carlo collisions, wall absorption, ionization births and charge deposition --
runs as hand-written HIP kernels for gfx950 behind the C ABI of
include/edupic.h.  `edupic` is the thin ctypes binding of that library.
"""
