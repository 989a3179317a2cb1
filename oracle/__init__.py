"""CPU oracle for the HODLR-accelerated multifrontal preconditioner.

TEST INFRASTRUCTURE ONLY.  Plain, slow, float64 NumPy/SciPy code written from
the paper (Aminfar & Darve, "A Fast and Memory Efficient Sparse Solver with
Applications to Finite-Element Matrices").  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import it; the product path
never does.  It shares no code with the GPU library.

Modules
-------
symbolic   nested dissection, elimination tree, I_p, S_p, I_p^f (Sec. 4.1.1,
           Eq. couplingSet), relative maps, HODLR cluster trees, BDLR sets
           (Sec. 2.2).
dense_mf   conventional multifrontal Cholesky and solve (Sec. 4.1, Eq. update,
           Eq. upward, Eq. downward).
hodlr      HODLR matrices (Sec. 2.1, Eq. HODLR2): BDLR / SVD compression
           (Sec. 2.2, Eq. Bhat), recursive Sherman-Morrison-Woodbury factor and
           solve.
hodlr_mf   HODLR-accelerated multifrontal factor and solve (Sec. 4.2,
           Eq. update_HODLR, Eq. HODLR_EA_Expand, Eq. update_HODLR_Parent).
gmres      right-preconditioned flexible GMRES(m) (Sec. 3).
pcg        preconditioned conjugate gradients, flexible beta (Sec. 3: the
           preconditioner serves any Krylov solver, CG among them).

Parity status: every function is pinned by the tests under tests/ (see the
pin list in each module's docstring).  Iteration counts and the particular
skeleton pivots are heuristic outputs: reported, not pinned.
"""
