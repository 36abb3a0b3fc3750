"""Plain CPU FP64 oracle for the accelerated SPD HSS construction.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package; the
product path (the HIP library and its Python binding) never does, and shares
no code with it.

It is a slow, literal, obviously checkable implementation of:

* the partition tree and admissibility lists (Section 2 notation, Section 5.1
  far-field sets, Section 5.2.2 block types);
* kernel-matrix entries (Section 6 kernel list, with length-scale
  parameterisation of the workloads);
* an H^2 representation built by proxy-point interpolative decomposition
  (Section 5.1 representation; the construction itself is not given in the
  paper, so the one here is this project's reading), its matrix-vector
  product and the level-masked sampling products of eq. (Yk);
* Algorithm 5.3 (accelerated SPD HSS construction), with Algorithm 5.1
  (randomized range finder) and Algorithm 5.2 (level-by-level special
  products), in both the eigen-decomposition form of the paper and the
  Cholesky form used by the GPU path;
* a nested-factor solve with the constructed HSS matrix, and PCG.

Every result is pinned in tests/ against dense brute force, closed forms,
library routines or the paper's identities.  Parts that no such pin fixes say
"parity unpinned" in their docstrings.
"""
