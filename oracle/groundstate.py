"""Ground state by the gradient flow with discrete normalisation (GF-GauSum), float64.

Oracle (test infrastructure only).  Follows Section 3.2 of the paper:

* GFDN (eqs. gf-eq1 to gffg3): the imaginary-time flow of the operator
  (1/2)(-Lap+m^2)^s + V + beta|phi|^2 + lam Phi - Omega Lz, with the state
  renormalised to unit norm at every time level.
* Semi-implicit backward Euler (eqs. gf-eq2 to gffg33): with rho^n = |phi^n|^2
  and Phi^n = U * rho^n frozen over the step,
      A^{BE,n} phi1 = phi^n / dt,
      A^{BE,n} = I/dt + (1/2)(-Lap+m^2)^s + V + beta rho^n + lam Phi^n - Omega Lz,
  then phi^{n+1} = phi1 / ||phi1||.
* The first preconditioned system of eq. precond_type1, which the paper
  uses: with P_Delta = [I/dt + (1/2)(-Lap+m^2)^s]^{-1} (diagonal in Fourier
  space) and A_TF = V + beta rho^n + lam Phi^n - Omega Lz,
      (I + P_Delta A_TF) phi1 = P_Delta phi^n / dt,
  solved by BiCGStab.
* Stopping rule of the paper's experiments: ||phi^n - phi^{n+1}||_inf <= eps0 dt
  (run, run_to); run_to also stops on an energy change |E^{n+1} - E^n| below a
  tolerance, E of eq. energy in the frame of eq. SFSE.
* Initial guess (eq. ini_guess): ((1-Omega) phi_ho + Omega phi_ho^v), normalised.

Readings where the paper is silent:
* ||.||_2 is the discrete norm (h^d sum |phi|^2)^{1/2}, the mass of the dynamics.
* V is the trap in the frame where the energy carries -Omega Lz, i.e. V(x)
  unrotated (the functional whose minimiser is sought).
* The Krylov solver starts from phi^n and stops at a relative residual rtol of
  the preconditioned system (the paper gives no tolerance); here
  scipy.sparse.linalg.bicgstab.
* In 3D the initial guess carries the factor (gamma_z/pi)^{1/4} exp(-gamma_z z^2/2).

The operator is written out here from the equations (it does not call
diagnostics.apply_H), so that H psi of the diagnostics module pins it.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.sparse.linalg import LinearOperator, bicgstab

from .scheme import _bcast, axes, freqs, kinetic_symbol, lattice_potential
from . import _fft, diagnostics


def _norm(phi, N, L):
    vol = float(np.prod([2.0 * Lj / Nj for Nj, Lj in zip(N, L)]))
    return math.sqrt(vol * float(np.sum(np.abs(phi) ** 2)))


def initial_guess(N, L, Omega, gamma=(1.0, 1.0, 1.0)):
    """phi0 of eq. ini_guess (2D); in 3D times the normalised z Gaussian."""
    X = np.meshgrid(*axes(N, L), indexing="ij")
    r2 = X[0] ** 2 + X[1] ** 2
    ho = np.exp(-r2 / 2.0) / math.sqrt(math.pi)
    hov = (X[0] + 1j * X[1]) * np.exp(-r2 / 2.0) / math.sqrt(math.pi)
    phi = (1.0 - Omega) * ho + Omega * hov
    if len(N) == 3:
        gz = float(gamma[2])
        phi = phi * (gz / math.pi) ** 0.25 * np.exp(-gz * X[2] ** 2 / 2.0)
    return phi / _norm(phi, N, L)


class GroundState:
    """The backward-Euler GFDN of one problem (an oracle.scheme.Problem) at time step dt."""

    def __init__(self, prob, dt):
        self.prob, self.dt = prob, float(dt)
        N, L, d = prob.N, prob.L, prob.d
        self.N, self.L = N, L
        X = np.meshgrid(*axes(N, L), indexing="ij")
        self.X = X
        V = 0.5 * (prob.gamma[0] ** 2 * X[0] ** 2 + prob.gamma[1] ** 2 * X[1] ** 2)
        if d == 3:
            V = V + 0.5 * prob.gamma[2] ** 2 * X[2] ** 2
        self.V = V
        self.omega = kinetic_symbol(N, L, prob.s, prob.m)
        self.mu = [_bcast(m, j, d) for j, m in enumerate(freqs(N, L))]

    # -- operators ------------------------------------------------------------
    def P_delta(self, v):
        """[I/dt + (1/2)(-Lap+m^2)^s]^{-1} v, diagonal in Fourier space."""
        return _fft.ifftn(_fft.fftn(v) / (1.0 / self.dt + 0.5 * self.omega))

    def Lz(self, v):
        """-i (x d_y - y d_x) v with Fourier derivatives."""
        vh = _fft.fftn(v)
        dx = _fft.ifftn(1j * self.mu[0] * vh)
        dy = _fft.ifftn(1j * self.mu[1] * vh)
        return -1j * (self.X[0] * dy - self.X[1] * dx)

    def frozen(self, phi_n):
        """W^n = V + beta rho^n + lam Phi^n of the time level phi^n."""
        rho = np.abs(phi_n) ** 2
        V = self.V
        if getattr(self.prob, "lattice", None) is not None:
            V = V + lattice_potential(self.X, self.prob.lattice)  # the frame of eq. SFSE
        if getattr(self.prob, "U", None) is not None:
            if self.prob.Omega != 0.0:
                raise NotImplementedError("an external potential needs Omega = 0 in the ground-state step")
            V = V + self.prob.U
        return V + self.prob.beta * rho + self.prob.lam * self.prob.potential(rho)

    def A_TF(self, W, v):
        return W * v - self.prob.Omega * self.Lz(v)

    def system(self, phi_n):
        """(M, rhs) of the preconditioned system M phi1 = rhs, M = I + P_Delta A_TF."""
        W = self.frozen(phi_n)
        shape = phi_n.shape

        def mv(x):
            v = np.asarray(x).reshape(shape)
            return (v + self.P_delta(self.A_TF(W, v))).ravel()

        n = phi_n.size
        M = LinearOperator((n, n), matvec=mv, dtype=np.complex128)
        rhs = self.P_delta(phi_n / self.dt)
        return M, rhs

    # -- one backward-Euler step ---------------------------------------------
    def solve(self, phi_n, rtol=1e-12, maxiter=1000):
        """phi1 (not normalised) and (iterations, relative residual)."""
        M, rhs = self.system(phi_n)
        its = [0]

        def cb(_):
            its[0] += 1

        x, info = bicgstab(M, rhs.ravel(), x0=phi_n.ravel().astype(np.complex128), rtol=rtol,
                           maxiter=maxiter, callback=cb)
        if info < 0:
            raise RuntimeError(f"bicgstab breakdown ({info})")
        res = float(np.linalg.norm(M.matvec(x) - rhs.ravel()) / np.linalg.norm(rhs.ravel()))
        return x.reshape(phi_n.shape), (its[0], res)

    def step(self, phi_n, rtol=1e-12, maxiter=1000):
        """phi^{n+1} = phi1 / ||phi1|| and (iterations, residual, ||phi^n - phi^{n+1}||_inf)."""
        phi1, (its, res) = self.solve(phi_n, rtol, maxiter)
        phi = phi1 / _norm(phi1, self.N, self.L)
        return phi, (its, res, float(np.max(np.abs(phi - phi_n))))

    def run(self, phi0, eps0=1e-9, max_steps=100000, rtol=1e-12):
        """Iterate until ||phi^n - phi^{n+1}||_inf <= eps0 dt; returns (phi, steps, last stats)."""
        phi = phi0
        stats = None
        for n in range(1, int(max_steps) + 1):
            phi, stats = self.step(phi, rtol)
            if stats[2] <= eps0 * self.dt:
                return phi, n, stats
        return phi, int(max_steps), stats

    def energy(self, phi):
        """The functional the flow decreases: E(phi) of eq. energy in the frame of eq. SFSE (V unrotated, -Omega Lz)."""
        return diagnostics.energy_parts(self.prob, phi, 0.0)[5]

    def run_to(self, phi0, eps_diff=None, eps_energy=None, max_steps=100000, rtol=1e-12):
        """Iterate until a stopping rule holds after a step: the paper's ||phi^n - phi^{n+1}||_inf <= eps_diff dt
        (Section 3.3), or an energy change |E(phi^{n+1}) - E(phi^n)| <= eps_energy (None: rule not used), or
        max_steps.  Returns (phi, steps, rule, energies): rule 1 (difference), 2 (energy) or 0 (neither, after
        max_steps; the difference rule is tested first), energies = [E(phi0), E(phi^1), ...]."""
        phi = phi0
        energies = [self.energy(phi)]
        for n in range(1, int(max_steps) + 1):
            phi, stats = self.step(phi, rtol)
            energies.append(self.energy(phi))
            if eps_diff is not None and stats[2] <= eps_diff * self.dt:
                return phi, n, 1, energies
            if eps_energy is not None and abs(energies[-1] - energies[-2]) <= eps_energy:
                return phi, n, 2, energies
        return phi, int(max_steps), 0, energies
