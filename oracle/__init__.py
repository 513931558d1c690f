"""CPU FP64 oracle for the augmented-Lagrangian Stokes multigrid (TEST INFRASTRUCTURE).

This package is test infrastructure. Only the test suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import it.
The GPU library never calls it and shares no code with it; the only common
input is the seeded workload description in ``workloads``.

It is a plain, slow, obviously-correct implementation written from the paper
(Shih, Stadler, Wechsung, "Robust multigrid techniques for augmented
Lagrangian preconditioning of incompressible Stokes equations with extreme
viscosity variations"):

* ``fem``        -- structured quad/hex hierarchy, [Q2]^d x P1disc spaces,
                    Gauss-Legendre quadrature (Section 4, definition of V_h^k, Q_h^{k-1}).
* ``coefficients`` -- multi-sinker viscosity and forcing (Section 5.2) and the
                    Newton tensor of a viscoplastic law (Section 5.3.1).
* ``assembly``   -- assembled sparse A, B, M_p, M_p(1/mu), A_gamma and the
                    right-hand side (Section 2, eq. (stokessys); Section 3, eq. (augstokessys)).
* ``multigrid``  -- vertex-star additive Schwarz smoother with dense LU patch
                    solves extracted from the assembled matrix (Section 4.1,
                    eq. (viim); Section 5.1), GMRES-accelerated relaxation,
                    the robust prolongation with local solves on coarse cells
                    (Section 4.2, eq. (Ptilde)), sparse-LU coarse solve, V-cycle.
* ``krylov``     -- FGMRES with the block preconditioner of eq. (precond) and
                    the Schur approximations P1/P2 of eq. (P1P2).
* ``direct``     -- direct solve of the bordered saddle-point system: the
                    plain definition of the discrete solution.

Every numerical step is FP64. Where the paper is silent or garbled, the
reading taken is stated at the function that implements it.
"""
