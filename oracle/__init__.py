"""FP64 CPU oracle for the null-space-free Maxwell eigensolver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links anything in this directory; only the test suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP path.

It computes, slowly and literally, what the paper defines:

* ``yee``    -- the Yee single-curl operator C built from K (Sec. 2, eqs. for
               C, C1..C3, K), the twisted DFT T and the diagonal Lambda's
               (Thm 2.1, Lemma 2.2).
* ``basis``  -- Pi_0, Pi_1, Pi_2 and the singular-vector matrices P, Q, P_r,
               Q_r by their defining formulas (Thm 2.3, the projection and
               curl constructions before Thm 2.4, Thm 2.5).
* ``medium`` -- the 3n x 3n material matrices eps_d, mu_d, xi_d, zeta_d from
               per-voxel 3x3 tensors (Sec. 3, Sec. 4.3).
* ``nfgep``  -- A_r and B_r of the HHPD null-space-free pencil (Thm 4.2), the
               discrete GEP (Sec. 3), plain CG (Sec. 4.2) and eigenvalues by
               dense LAPACK, by ARPACK on the pencil, and by sparse
               shift-invert on the 6n GEP.
* ``nfsep``  -- the null space free eigenvalue problem K y = omega y for any
               medium with a nonsingular B (Thm 3.2): K dense and matrix-free,
               GMRES, and shift-and-invert Arnoldi at zero shift (Sec. 4).
* ``grad``   -- eigenvalue derivatives w.r.t. per-voxel eps and gamma from the
               left/right eigenvectors of the GEP.

Every function states the passage it follows.  Pins (tests that tie these
functions to facts other than themselves) live in ``tests/test_oracle_*.py``.
Parity-unpinned items: none of the functions here; iteration counts and
timings are not computed by the oracle.
"""
