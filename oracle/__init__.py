"""CPU FP64 reference implementation of subcycled RK4 with dense-output
refinement-boundary ghosts (Ji et al., "GPU-accelerated Subcycling Time
Integration with the Einstein Toolkit", arXiv:2503.09629, Sec. II).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct statement of what the method computes.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product library never does, and it shares no code, headers, tables or
constants with the GPU path.

Parts:
  splitmix   SplitMix64, the counter-based generator used by the block split
  hierarchy  block split, ghost classes, refinement-boundary lists,
             restriction pairs, nesting check, canonical map export
  dense      RK4 dense-output weights and fine-stage ghost weights, derived
             with exact rationals from the paper's formulas (Sec. II)
  stencil.c  wave right-hand side with Kreiss-Oliger dissipation and the RK4
             stage arithmetic as plain scalar loops (Sec. III.C, IV.A)
  evolve     per-block storage, ghost fills, prolongation, restriction and
             the recursive subcycling schedule (Sec. II, steps 1-7)

Parity status: every function is pinned by tests under tests/ against
closed forms, textbook special cases, brute force on tiny inputs or
invariants (see each module's header).
"""
