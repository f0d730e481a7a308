"""CPU oracle for sparse CP-ALS with MTTKRP -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct FP64 implementation of what the HIP library
computes, written from the paper (Section III, Algorithm 1) and pinned by the
``-m "not gpu"`` tests against brute force, closed forms and invariants.  It
shares no code with the HIP path (``paper_1812_05961_amd``): neither imports
the other.  Only the tests, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may use it.

Modules
  coo         MTTKRP on COO by a direct loop (C, FP64) and ||X||^2
  csf         CSF reference: stable lexicographic sort, duplicate merge, fiber
              compression, tile start nodes
  als         CP-ALS driver: Gram/Hadamard V, Cholesky solve with the
              pseudo-inverse fallback, column normalisation, fit, convergence
  dense_check dense tensor, unfolding and explicit Khatri-Rao product
              (brute force for tiny tensors)
  mlp         FP64 3-layer MLP forward/backward and Adam (selector reference)

Parity status per function is listed in each module's docstring.
"""
