"""CPU oracle for Accelerated Cyclic Reduction -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct FP64 reference implementations, written from
the paper (Chavez, Turkiyyah, Keyes, "A Direct Elliptic Solver Based on
Hierarchically Low-rank Schur Complements", arXiv:1604.00617):

* ``direct``  -- the plain definition: x = A^{-1} b by sparse/dense LU.
* ``bcr``     -- exact block cyclic reduction with dense blocks (Section 3:
                 even/odd permutation, Eq. "sche", Eq. "fund").
* ``hodlr``   -- HODLR (weak-admissibility H-matrix) storage, the truncation
                 rule T_eps, densify and matvec (Section 3, block tables).
* ``acr``     -- ACR: the BCR steps with every block held as a HODLR matrix and
                 every H-arithmetic operation realised as "exact dense result,
                 then compress" (formatted arithmetic with best truncation).
* ``refine``  -- iterative refinement with an FP64 residual (ACR used as a
                 preconditioner, Section 4 closing paragraph).
* ``krylov``  -- restarted flexible GMRES right-preconditioned by any
                 approximate inverse (the Krylov form of the same use).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU path and
never imports it; the only shared inputs come from ``workloads`` (seeded
problem generators that contain none of the method's arithmetic).
"""
