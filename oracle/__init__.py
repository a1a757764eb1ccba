"""FP64 CPU oracle for the TS2-GauSum split step (test infrastructure only).

This package is a plain, slow, float64 implementation of what the GPU library
computes, written from the paper (Antoine, Tang, Zhang, "On the ground states
and dynamics of space fractional nonlinear Schroedinger/Gross-Pitaevskii
equations with rotation term and nonlocal nonlinear interactions"):

* gausum      -- the Gaussian-sum (GauSum) nonlocal potential of Section 2:
                 sinc-quadrature Gaussian sum (eq. GS-Gene), the regular part
                 I1 through the separable tensor (eq. tensor), the near-field
                 Taylor correction I2 (eq. taylor), the 3D dipolar kernel via
                 the Coulomb potential of a modified density.
* scheme      -- the rotating-Lagrangian-coordinate time splitting of
                 Section 4.2 (eqs. 1step, 2stepA/B, solu_step2, int_poten and
                 the TS2-GauSum scheme tssp1-tssp3).
* diagnostics -- mass and energy (eqs. mass, energy), angular momentum
                 expectation (eq. AME), centre of mass (eq. CoM) and the
                 lab-frame operator apply H*psi (eq. SFSE).

It is test infrastructure: only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it.  It shares no code with the HIP
library; the GPU path never calls it.

Parity status of each function (what pins it, besides its own formula) is
listed in the module docstrings; every function here is pinned by a test in
tests/oracle/.
"""
from . import gausum, scheme, diagnostics  # noqa: F401
