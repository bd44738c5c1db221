"""Plain, slow, obviously-correct CPU oracle of the two-stage Hermitian eigensolver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import, call or link anything in this
package.  It shares no code with the HIP library (``paper_1811_01277_amd``), and
neither imports the other; both take their inputs from ``workload``.

What it computes follows Sec. 2 of Kus et al., "Optimizations of the
Eigensolvers in the ELPA Library" (the two-stage method: full -> band ->
tridiagonal, tridiagonal eigensolve, and the two back-transformations of the
eigenvectors, Eqs. tridiagonalization, Esolv and the back-transformation
V~ = Q^H V^).  Readings of points the paper leaves open are listed in the
module docstrings where they are used.

Modules
-------
householder  LAPACK-convention reflector generation (larfg).
stage1       full -> band (panel Householder QR, two-sided update).
stage2       band -> tridiagonal one-column-per-step bulge chase (C).
tridiag      Sturm bisection + inverse iteration (C).
bt           back-transformations: tridiagonal->band (C, the hot path's
             definition) and band->full.
checks       residual / orthogonality invariants, cyclic Jacobi.
solve        the whole pipeline.
native       ctypes binding of oracle/csrc/oracle.c.
"""
