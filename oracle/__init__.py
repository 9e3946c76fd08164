"""CPU oracle for the WaveHoltz method with eigenvector deflation (FP64, numpy/scipy).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the HIP library: the only common dependency is the seeded
input generator ``workloads``.

Vectors here are *interior* unknowns of the unit-box grid with ``n`` cells per
side (``(n-1)**dim`` entries, x fastest); the boundary is homogeneous Dirichlet.

Modules
-------
discretization  L_h (face-averaged c^2), discrete Helmholtz matrix, direct solve
timeparams      time step, steps per period, adjusted frequency, filter weights
wavesolve       the filter operator Pi_h by explicit leapfrog + trapezoid rule
transfer        filter transfer functions beta (continuous) and beta_h (discrete)
modes           analytic Dirichlet sine eigenvectors and the deflation set
krylov          FPI, CG, DCG, GMRES(m), augmented GMRES, augmented BiCGStab
devd            direct eigenvector deflation (forcing deflation + inflation)
adjoint         misfit, direct-solve adjoint gradient, time-domain VJP, FD check

Parity status: every public function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against a closed form, an invariant, brute force, a
library routine applied to an independently built object (dense A from wave
solves, sparse LU) or a value the paper prints.  Among them: devd_solve in both
branches (CG; FPI with and without deflated iterates, against the direct solve
and the deflated rate of eq. WaveHoltzFPIconvergence) and transfer.kappa (the
2-norm condition number of the dense A).  No function is "parity unpinned".
"""
from . import discretization, timeparams, wavesolve, transfer, modes, krylov, devd, adjoint  # noqa: F401
