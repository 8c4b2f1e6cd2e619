"""Plain FP64 CPU oracle for the bidomain per-step solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this package: only the tests, the smoke check and the benchmark's CPU
baseline leg do.  It shares no code with the HIP library; both consume the
seeded inputs of the `workloads` package and nothing else.

Modules
  fem       P1 assembly of stiffness and lumped mass (Sec. 3.1)
  ionic     Mitchell-Schaeffer reaction terms (the ionic model of the runs)
  bidomain  system matrix, Steps 1-3 of the resolution algorithm (Sec. 3.2),
            the normalised solve of Prop. 1
  blocklu   dense block-LU algebra of Sec. 4 (Prop. 2, Rem. 1, Prop. 3) and
            the block preconditioner of Def. 2 with the monodomain K_m
  mpnn      FP64 message-passing network used as the learned correction
  chebyshev polynomial P_K (Chebyshev acceleration of the Jacobi iteration
            on K_m, one of the free choices of Sec. 5.3) from its closed form
  record    activation times and probe (electrode) potentials of a run
            (the recordings of the test cases of Sec. 6)
"""
