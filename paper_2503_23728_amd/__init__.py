"""MI355X-native hot path of machine-learned-force-field ring-polymer
(path-integral) molecular dynamics: neighbour search, Behler-Parrinello
descriptors, per-element MLPs on MFMA, the hand-written adjoint for forces
and virial, and normal-mode PILE-L propagation, behind the C ABI of
include/pimd.h.

Modules: abi (ctypes binding of libpimd.so), pimd (torch-facing wrapper and
autograd Function), synthetic (seeded input generators), build (compiles the
library).  Importing the package loads nothing; abi.lib() loads the library.
"""
