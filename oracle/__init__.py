"""Plain CPU FP64 oracle for the real-space DFPT RPA correlation-energy hot path.

TEST INFRASTRUCTURE ONLY.  This package is a slow, obviously-correct restatement
of what the method computes, written from the paper (Zhang, Shah, Pask, Chow,
Suryanarayana, "Random Phase Approximation Correlation Energy using Real-Space
Density Functional Perturbation Theory", arXiv:2504.01816).  It exists so that
the GPU library can be checked against something independent of it.  Only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the product path never does.  It shares no code with the HIP library.

Every function works in float64 (complex128 where the paper's quantities are
complex) and cites the passage it follows: section, equation number (equations
numbered in order of appearance, Eq. 1 = the ACFD correlation energy through
Eq. 10 = the low-rank correlation energy), Algorithm 1 or a table.

Modules
-------
fd          12th-order periodic finite-difference Laplacian and Hamiltonian (Sec. 3, Eq. 4)
coulomb     nu^{1/2} by the Kronecker product of 1D eigenbases, and dense pseudo-inverse (Sec. 3, Eq. 5)
cocg        conjugate orthogonal conjugate gradient for complex-symmetric systems (Sec. 3)
chi0        chi0 applied by DFPT (Eqs. 7-9) and by the sum over states (Eq. 2)
subspace    Rayleigh-Ritz energy, Cholesky orthonormalisation, subspace iteration (Algorithm 1)
quadrature  Gauss-Legendre frequency rule mapped to [0, inf) (Sec. 3)
energy      full E_c over frequencies (Eq. 10, Algorithm 1)
gradient    dE_c/dV_loc with orbitals, eigenvalues and saved subspaces fixed
precond     Kronecker shifted-Laplacian preconditioner and preconditioned COCG (Sec. 3)
block       block COCG over the trial vectors that share one Sternheimer matrix (Sec. 3)
"""
