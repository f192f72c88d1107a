"""FP64 CPU oracle for the AMGe solve phase -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never calls it, and it shares
no code with the HIP path (the seeded input generators aside).

Modules
-------
fem        fine Kuhn mesh, incidence matrices, Whitney masses, fine operators
           (paper section 2, eq. (2.2); discrete derivatives of section 2.2)
hierarchy  structured 2x2x2 agglomeration, PV traces, local extensions,
           order-0 target filtering, Galerkin products, co-chain projectors
           (paper section 3, eqs. (3.2)-(3.9))
solve      l1 diagonals, hybrid smoother, V-cycle, dense Cholesky, inexact PCG
           (paper section 4, Algorithm 4.1, eq. (4.1); section 5.1 solver set-up)

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
closed forms, textbook identities, brute force or independent formulations.
Parity unpinned: PCG iteration counts (the paper's counts are for a mesh that
is not available), see the design notes.
"""
