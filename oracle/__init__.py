"""CPU FP64 oracle for the PSLR preconditioner (Zheng, Xi, Saad; arXiv 2002.00917).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
restatement of the method, used by the test-suite, by the smoke check and by
the CPU timing leg of the benchmark.  The HIP library never imports, links or
calls it, and it shares no code with the library: the only module both sides
use is the seeded input generator ``paper_2002_00917_amd.workloads``.

Modules
  partition  -- domain-decomposition reordering (paper Sec. 2): labels,
                interface detection and the interiors-first permutation.
  pslr       -- block extraction, dense closed forms (eqs. matrixS, invS0,
                approx1, err1/err0/s1, schur, Sinv0/Sinv), Arnoldi, and the
                matrix-free application of Algorithm 3 and its transpose.
  krylov     -- right-preconditioned flexible GMRES, FP64.
  adjoint    -- gradient of a loss of z = A^{-1} b with respect to A's nonzeros.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against something other than itself (closed forms, textbook identities,
library routines, brute force); none is "parity unpinned".
"""
