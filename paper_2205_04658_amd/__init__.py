"""MI355X-native relativistic lattice-Boltzmann step (arXiv:2205.04658).

The compute path lives in the HIP/C++ shared library `librlb.so` (sources in
`csrc/`, C ABI in `include/rlb.h`).  `paper_2205_04658_amd.rlb` is a thin
ctypes binding over it; importing this package loads nothing until a
binding object is used.
"""
