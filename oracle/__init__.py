"""CPU FP64 oracle for the sparse-grid time-DG streamline-diffusion method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the tests, the smoke check and the benchmark's CPU
baseline leg call it.  It shares no code with the HIP path: the only common
input is the seeded workload data from the `workloads` package.

Tiers:
  brute.py     O1: the space-time bilinear form a_j of (eq:weak_form_j)
               integrated by quadrature on the finest product mesh, with the
               coarse basis functions evaluated pointwise (no Kronecker
               factorisation, no transfer matrices).
  operator.py  O2: the Kronecker form of Sect. 4.2 (block formula for
               A_{l,l'}, factors from the finest level by the embedding
               matrices E, blockwise application in the factor order of
               Sect. 4.2).
  ct.py        the combination-technique preconditioner, Algorithm 1's body.
  krylov.py    flexible GMRES (outer) used around it.
  strip.py     right-hand side b_j and the strip-by-strip time stepping.

Parity status of each function is stated in its module header.
"""
