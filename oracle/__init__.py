"""FP64 CPU oracle for ring-polymer (path-integral) MD with a
Behler-Parrinello neural potential.

This package is TEST INFRASTRUCTURE.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import or run it; the product
library never calls it and shares no code with it.  Every function states
the definition or the algorithm step it follows:

  constants    units and physical constants
  philox       Philox4x32-10 counter RNG + Box-Muller (Salmon et al., SC'11)
  neighbors    neighbour sets under the cutoff, brute force and cell list
  bpnn         symmetry-function descriptors, per-element MLP, analytic forces
  ring         normal modes, PILE-L OBABO integrator, estimators, harmonic V
  qho          quantum-harmonic-oscillator closed forms
  gfn          direct-force head in the graph-field-network form
  metad        well-tempered metadynamics on bead CVs (s_dimer, XRD)

The FP64 C core (bpnn_core.c) holds the triplet sums; oracle.build compiles
it with gcc.
"""
