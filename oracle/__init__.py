"""ORACLE -- test infrastructure, not part of the product.

A plain, slow, obviously correct CPU implementation of what the arrow-SpMM
path computes.  Only the test suite, the smoke check and the benchmark's CPU
baseline leg may import it.  It shares no code with the HIP path; both only
consume the seeded inputs from :mod:`workloads`.

Contents (paper: Gianinazzi et al., "Arrow Matrix Decomposition", PPoPP'24):

* :mod:`oracle.spmm` -- FP64 CSR product Y = A X (the plain definition the
  method reaches exactly, Section 4 Eq. (1)), a pure-Python brute force for
  tiny inputs, and the iterated product with per-column renormalisation
  (Section 2, "Matrices": X_{t+1} = sigma(A X_t)).
* :mod:`oracle.decomp` -- the decomposition validator (arrow-width predicate of
  Section 1, exact reconstruction A = sum_i P_i B_i P_i^T of Section 4) and a
  step-by-step reference of LA-Decompose (Section 5.1) with the random
  spanning forest linear arrangement (Section 5.3) and smallest-first tree
  order (Section 5.4).
* :mod:`oracle.quant` -- decoders and round-to-nearest-even quantisers for
  BF16, FP16 and OCP FP8 E4M3FN written from the format definitions.
"""
