"""TS2-GauSum time splitting in rotating Lagrangian coordinates, float64.

Oracle (test infrastructure only).  Follows Section 4.2 of the paper:

* The rotating Lagrangian coordinates x = A(t) x~ (eqs. Amatrix, transform)
  remove the rotation term; the potential becomes W(x~, t) = V(A(t) x~)
  (eq. FSE1_Rot).
* Linear sub-step (eq. 1step): i phi_t = (1/2)(-Lap + m^2)^s phi, integrated
  exactly in Fourier space on the periodic box: multiply the DFT coefficients
  by exp(-i tau (|mu|^2 + m^2)^s / 2).
* Nonlinear sub-step (eqs. 2stepA/B): the density is constant in time, so
  the solution is phi * exp(-i[tau beta rho + lam * K~ * rho + P]) with
  K~ = int U ds: tau * U for a Coulomb kernel, a dipole along z (the
  rotating axis m(t) = A^{-1} n equals n then) or any axis without
  rotation; for an axis that turns, the multiplier with the time average of
  m m^T over the sub-step (eq. Kernel_Rot), and P = int V(A(s) x~) ds (eq. int_poten).
* TS2-GauSum (eqs. tssp1-tssp3): half linear step, full nonlinear step,
  half linear step.
* A non-harmonic part of V: an optical lattice V_L = sum_j v_j sin^2(k_j x_j)
  in the frame of eq. SFSE (the form of the paper's second ground-state
  example).  Its time integral over a sub-step in rotating coordinates has no
  closed form; the paper leaves P to be computed numerically for a general V.
  Here: Gauss-Legendre quadrature in s with 32 nodes (Omega = 0: exactly
  tau V_L).
* Fourth order: the paper notes that TS2 extends to higher-order splitting
  (end of Section 4.2) without giving a scheme.  Reading: the symmetric
  triple-jump composition of Yoshida (1990), TS2 steps of lengths w1 dt,
  w0 dt, w1 dt with w1 = 1/(2 - 2^{1/3}), w0 = 1 - 2 w1 (negative); each
  sub-step is exact for negative lengths too.

Readings of the paper's text:
* Grid: N points per axis, x_l = -L + l h, h = 2L/N (the periodic endpoint
  of the paper's index set is dropped); frequencies mu_p = 2 pi p / (2L) in
  the order p = 0..N/2-1, -N/2..-1, the Nyquist index kept as p = -N/2.
* Half step: the paper's factor dt/4 is half a step of (1/2)(-Lap+m^2)^s, so
  a linear step of length tau multiplies by exp(-i tau omega / 2).
* Density of the nonlinear step: rho = |phi^(1)|^2, the state entering the
  nonlinear sub-step (the sub-problem conserves that density; reading the
  displayed |phi^n|^2 literally would make the scheme first order).
* Exact solution of the nonlinear sub-step: phi(t) = phi(t_n) * exp(...) (the
  displayed formula drops the factor phi(t_n)).
* P for the harmonic trap (derived here, theta = Omega t):
      V(A x~) = ((gx^2+gy^2)/4)(x~^2+y~^2) + (gz^2/2) z~^2
                + ((gx^2-gy^2)/4)[(x~^2-y~^2) cos 2theta + 2 x~ y~ sin 2theta]
  integrated over [t, t+tau]:
      int cos(2 Omega s) ds = cos(Omega(2t+tau)) sin(Omega tau)/Omega,
      int sin(2 Omega s) ds = sin(Omega(2t+tau)) sin(Omega tau)/Omega.

Parity: pinned by the exact free-evolution identity, the s = 1 free Gaussian
closed form, quadrature of P, unitarity (mass), reversibility, second-order
convergence, the s = 1 centre-of-mass ODE and conservation of <Lz>, and for a turning dipole axis the
second-order conservation of the rotating-frame energy (tests/oracle).
"""
from __future__ import annotations

import math

import numpy as np

from . import gausum
from . import _fft


def axes(N, L):
    return [-float(Lj) + np.arange(int(Nj)) * (2.0 * float(Lj) / int(Nj)) for Nj, Lj in zip(N, L)]


def freqs(N, L):
    """mu_{j,p} = 2 pi p / (2 L_j) in DFT order."""
    return [2.0 * math.pi * np.fft.fftfreq(int(Nj), d=2.0 * float(Lj) / int(Nj)) for Nj, Lj in zip(N, L)]


def _bcast(v, j, d):
    shape = [1] * d
    shape[j] = -1
    return v.reshape(shape)


def kinetic_symbol(N, L, s, m=0.0):
    """omega(mu) = (|mu|^2 + m^2)^s on the DFT grid."""
    d = len(N)
    mu = freqs(N, L)
    k2 = np.zeros(tuple(int(n) for n in N))
    for j in range(d):
        k2 = k2 + _bcast(mu[j], j, d) ** 2
    return (k2 + m * m) ** s


def kinetic(psi, N, L, s, tau, m=0.0):
    """Linear sub-step over time tau (eq. 1step, exact in Fourier space)."""
    om = kinetic_symbol(N, L, s, m)
    return _fft.ifftn(np.exp(-1j * tau * 0.5 * om) * _fft.fftn(psi))


def lattice_potential(X, lattice):
    """V_L = sum_j v_j sin^2(k_j x_j) at frame coordinates X (lattice = (v, k), per axis)."""
    v, k = lattice
    return sum(v[j] * np.sin(k[j] * X[j]) ** 2 for j in range(len(X)))


def _lab(X, Omega, t):
    th = Omega * t
    c, s_ = math.cos(th), math.sin(th)
    lab = list(X)
    lab[0] = c * X[0] + s_ * X[1]
    lab[1] = -s_ * X[0] + c * X[1]
    return lab


def lattice_integral(N, L, Omega, lattice, t, tau, nodes=32):
    """int_t^{t+tau} V_L(A(s) x~) ds by Gauss-Legendre in s."""
    X = np.meshgrid(*axes(N, L), indexing="ij")
    xg, wg = np.polynomial.legendre.leggauss(nodes)
    out = np.zeros(X[0].shape)
    for xi, wi in zip(xg, wg):
        out = out + 0.5 * tau * wi * lattice_potential(_lab(X, Omega, t + 0.5 * tau * (xi + 1.0)), lattice)
    return out


def trap(N, L, gamma, Omega, t, lattice=None):
    """W(x~, t) = V(A(t) x~) on the grid (rotating frame, eq. FSE1_Rot), lattice included."""
    d = len(N)
    X = np.meshgrid(*axes(N, L), indexing="ij")
    th = Omega * t
    c, s_ = math.cos(th), math.sin(th)
    x = c * X[0] + s_ * X[1]
    y = -s_ * X[0] + c * X[1]
    V = 0.5 * (gamma[0] ** 2 * x ** 2 + gamma[1] ** 2 * y ** 2)
    if d == 3:
        V = V + 0.5 * gamma[2] ** 2 * X[2] ** 2
    if lattice is not None:
        V = V + lattice_potential(_lab(X, Omega, t), lattice)
    return V


def trap_integral(N, L, gamma, Omega, t, tau, lattice=None):
    """P(x~; t, t+tau) = int_t^{t+tau} V(A(s) x~) ds: closed form for the harmonic trap
    (eq. int_poten), quadrature for a lattice."""
    d = len(N)
    X = np.meshgrid(*axes(N, L), indexing="ij")
    gx2, gy2 = gamma[0] ** 2, gamma[1] ** 2
    if Omega == 0.0:
        sc_int = math.cos(0.0) * tau
        ss_int = 0.0
    else:
        f = math.sin(Omega * tau) / Omega
        sc_int = math.cos(Omega * (2.0 * t + tau)) * f
        ss_int = math.sin(Omega * (2.0 * t + tau)) * f
    P = tau * (gx2 + gy2) / 4.0 * (X[0] ** 2 + X[1] ** 2)
    P = P + (gx2 - gy2) / 4.0 * ((X[0] ** 2 - X[1] ** 2) * sc_int + 2.0 * X[0] * X[1] * ss_int)
    if d == 3:
        P = P + tau * 0.5 * gamma[2] ** 2 * X[2] ** 2
    if lattice is not None:
        P = P + lattice_integral(N, L, Omega, lattice, t, tau)
    return P


class Problem:
    """Parameters of one instance plus its GauSum multiplier (built once)."""

    def __init__(self, d, N, L, s, Omega, gamma, beta, lam, kernel="coulomb", mu=1.0, c=1.0,
                 m=0.0, delta=None, axis=(0.0, 0.0, 1.0)):
        self.d, self.N, self.L = int(d), tuple(int(n) for n in N), tuple(float(x) for x in L)
        self.s, self.Omega, self.gamma = float(s), float(Omega), tuple(float(g) for g in gamma)
        self.beta, self.lam, self.kernel = float(beta), float(lam), kernel
        self.mu, self.c, self.m = float(mu), float(c), float(m)
        self.delta = delta
        self.axis = tuple(float(a) for a in axis)
        # optional real potential U(x~) on the computational grid, added to the
        # nonlinear phase as dt * U (static in the rotating Lagrangian coordinates)
        self.U = None
        # in the rotating Lagrangian coordinates the dipole axis m(t) = A^{-1}(t) n
        # turns unless n is the rotation axis (eq. Kernel_Rot)
        self.turning_axis = (kernel in ("ddi2", "ddi3") and self.Omega != 0.0
                             and (self.axis[0] != 0.0 or self.axis[1] != 0.0))
        self._K = None
        self._KC = None
        # optional optical lattice (v, k) per axis, in the frame of eq. SFSE
        self.lattice = None

    @classmethod
    def from_params(cls, p):
        return cls(p.d, p.N, p.L, p.s, p.Omega, p.gamma, p.beta, p.lam, kernel=p.kernel,
                   mu=p.mu, c=p.c, m=p.m, axis=p.axis)

    @property
    def h(self):
        return tuple(2.0 * L / N for L, N in zip(self.L, self.N))

    @property
    def K(self):
        if self._K is None and self.kernel != "none" and self.lam != 0.0:
            self._K = gausum.symbol(self.N, self.L, self.kernel, mu=self.mu, c=self.c,
                                    delta=self.delta, axis=self.axis)
        return self._K

    def K_at(self, t=0.0, tau=0.0):
        """Multiplier of the rotating-frame kernel over [t, t+tau] (its time average;
        tau = 0: at the instant t).  Equal to K unless the dipole axis turns."""
        if not self.turning_axis:
            return self.K
        if self._KC is None:
            c = 1.0 / ((4.0 if self.d == 3 else 2.0) * math.pi)
            self._KC = gausum.coulomb_symbol(self.N, self.L, mu=1.0, c=c, delta=self.delta)
        M = gausum.dipole_average(self.axis, self.Omega, t, tau)
        return gausum.dipole_form_symbol(self.N, self.L, self.kernel, M, KC=self._KC)

    def potential(self, rho, t=0.0, tau=0.0):
        """Nonlocal potential Phi[rho] = U * rho (zero if there is no kernel), in the rotating
        coordinates at time t (averaged over [t, t+tau]); t = 0 is also the frame of H psi."""
        if self.kernel == "none" or self.lam == 0.0:
            return np.zeros(self.N)
        return gausum.convolve(rho, self.K_at(t, tau))

    def nonlinear(self, phi, t, tau):
        """Nonlinear sub-step over [t, t+tau] (eqs. 2stepA, 2stepB, solu_step2)."""
        rho = np.abs(phi) ** 2
        theta = tau * self.beta * rho + self.lam * tau * self.potential(rho, t, tau)
        theta = theta + trap_integral(self.N, self.L, self.gamma, self.Omega, t, tau, self.lattice)
        if self.U is not None:
            theta = theta + tau * self.U
        return phi * np.exp(-1j * theta)

    def step(self, psi, t, dt):
        """One TS2-GauSum step (eqs. tssp1-tssp3); returns (psi, t + dt)."""
        p1 = kinetic(psi, self.N, self.L, self.s, 0.5 * dt, self.m)
        p2 = self.nonlinear(p1, t, dt)
        p3 = kinetic(p2, self.N, self.L, self.s, 0.5 * dt, self.m)
        return p3, t + dt

    def run(self, psi, nsteps, dt, t=0.0):
        for _ in range(int(nsteps)):
            psi, t = self.step(psi, t, dt)
        return psi, t

    def step4(self, psi, t, dt):
        """One fourth-order step: TS2 steps of lengths w1 dt, w0 dt, w1 dt."""
        w1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
        for w in (w1, 1.0 - 2.0 * w1, w1):
            psi, _ = self.step(psi, t, w * dt)
            t = t + w * dt
        return psi, t

    def run4(self, psi, nsteps, dt, t=0.0):
        t0 = t
        for k in range(int(nsteps)):
            psi, _ = self.step4(psi, t0 + k * dt, dt)
        return psi, t0 + nsteps * dt
