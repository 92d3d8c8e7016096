"""CPU FP64 oracle for the RVE corrector path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously correct NumPy/SciPy implementation of
what the GPU path computes, written from the paper (Khoromskaia, Khoromskij,
Otto, "Numerical study in stochastic homogenization for elliptic PDEs:
convergence rate in the size of representative volume elements"). It exists to
check the GPU path. Only the test suite, the smoke check in
``__graft_entry__.py`` and the CPU-baseline leg of ``bench.py`` may import or
call it; the product package never does, and shares no code with it.

Modules
-------
q1     Q1 Galerkin stiffness by Kronecker sums of 1D matrices (Sec. 3.1-3.2),
       Galerkin right-hand sides (eqn. FEM_discr_RHS), the constant-coefficient
       periodic symbol used by the preconditioner (Sec. 3.5).
pcg    Plain preconditioned CG with the constant-coefficient preconditioner
       applied by FFT (Sec. 3.5, eqn. DD_Eqn, Lemma Cond_Number).
ahom   One realization end to end: correctors, the homogenized 2x2 matrix in
       flux form (eqns. A_hom_m, Ahom_m_entry) and energy form (Sec. 4.3,
       symmetry argument for wg02), and dA_hom/da per cell.
stats  Ensemble statistics: empirical mean (A_hom_Empir), centred variances,
       the uncentred standard deviations Var1/Var2, and the quartic tensor
       (eqn. quartic).
fd5    The lumped five-point discretisation of Sec. 3.2 (eqns. Lapl_Kron_D,
       As_Kron) with the finite-difference Laplacian preconditioner (eqn.
       Lap_Kron): operator, right-hand sides, homogenized matrix, gradient.
lattice_sample
       The on-device sampler's law: lattice Poisson square centres decided by
       Philox4x32-10 words (Salmon et al., SC'11), squares painted into cells.
q1_3d  The three-dimensional corrector problems (d = 3; Sec. 2 and eqn.
       As_Kron_d): trilinear Q1 stiffness and right-hand sides, the rank-3
       constant-coefficient symbol and its FFT pseudo-inverse, PCG, and the
       3 x 3 homogenized matrix in energy and flux form.
dos    Spectral density of the stiffness matrix (Appendix, eqns. DOS,
       DOS_gauss): exact from eigenvalues, and the Chebyshev-moment estimate
       with probe vectors.

Pinning status: every function here is pinned by a ``-m "not gpu"`` test
against closed forms, brute force or invariants (see tests/test_oracle_*.py).
No function is "parity unpinned".
"""
from . import q1, pcg, ahom, stats, fd5, lattice_sample, dos, q1_3d  # noqa: F401
