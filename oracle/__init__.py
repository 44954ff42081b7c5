"""FP64 CPU oracle for HIF-preconditioned Crank-Nicolson solves (Feliu-Faba & Ying).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU
baseline leg may import or run anything in this package; the GPU library never does, and the
oracle never imports the GPU library.  The two share no code: only the seeded input generators
(``workloads``), which contain none of the method's arithmetic, feed both.

Modules (each function cites the passage of the paper it follows):
  fd          -- five/seven-point variable-coefficient stencil M, A = I - dt/2 M (Sec. 2, eq2)
  cn          -- Crank-Nicolson right-hand side, explicit reaction, PCG, Algorithm 1 (Sec. 2.1,
                 Sec. 2.3)
  geometry    -- quad/oct-tree levels, separator sets, grouping of active DOFs (Sec. 2.2)
  interp      -- interpolative decomposition by column-pivoted QR (Sec. 2.2 step 3, eq2_5)
  phif        -- block PHIF build (steps 1-3 per level, root) and apply of eqAinv (Sec. 2.2)
  phif_dense  -- dense-literal PHIF: the N x N factors of eqs eq2_3, jacobi-precond, eq_T,
                 eq2_9 formed and multiplied as written; pins ``phif`` on tiny grids
  estimate    -- power-iteration estimate of ||I - A F^-1||_2 (Sec. 3, Example 1)

Parity status: ``fd``, ``cn`` and the PHIF build/apply are pinned by tests (closed forms,
direct solves, the dense-literal transcription, the exactness at eps = 0, structural
identities).  The choice of skeleton DOFs inside each ID is one of several valid results of the
pivoted QR; exact factor entries are therefore compared only where both sides make the same
skeleton choice ("parity unpinned" beyond the invariants for that choice).
"""
