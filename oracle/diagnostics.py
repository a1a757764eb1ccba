"""Mass, energy, angular momentum, centre of mass and H*psi, float64.

Oracle (test infrastructure only).  Definitions from the paper:
* mass N = int |psi|^2 (eq. mass),
* energy E = int [ (1/2) psi^* (-Lap+m^2)^s psi + V |psi|^2 + (beta/2)|psi|^4
  + (lam/2) Phi |psi|^2 - Omega psi^* Lz psi ] (eq. energy), split here
  into its five parts,
* <Lz> = int psi^* Lz psi with Lz = -i (x d_y - y d_x) (eq. AME),
* centre of mass x_c = int x |psi|^2 (eq. CoM) and condensate widths
  delta_v = int v^2 |psi|^2 (eq. ConWidth, no square root), both in the lab
  frame: a state held in rotating Lagrangian coordinates x~ is read through
  x = A(t) x~ (eq. Amatrix), A = [[cos wt, sin wt], [-sin wt, cos wt]] on (x, y),
  w = Omega,
* H psi, the right-hand side operator of eq. SFSE in the lab frame, with an
  optional frozen density (the operator A^{BE,n} of Section 3.2 without its
  I/dt part uses rho = |phi^n|^2).

Discretisation: rectangle rule h^d sum over the periodic grid; Fourier
derivatives D_v = ifft(i mu_v fft(.)); the kinetic energy by Parseval,
(1/2)(h^d/n) sum omega(mu) |psi_hat|^2.  Energies of a state in the rotating
frame use W(x~, t) = V(A(t) x~); Lz and the other terms are rotation
invariant, so the sum is the lab-frame energy that the equation conserves.

Parity: pinned by closed forms for the harmonic-oscillator state and the
unit vortex (kinetic, potential, interaction energies, <Lz> = 1) and by
conservation laws (tests/oracle).
"""
from __future__ import annotations

import numpy as np

from .scheme import axes, freqs, kinetic_symbol, trap, _bcast
from . import _fft


def _vol(N, L):
    return float(np.prod([2.0 * Lj / Nj for Nj, Lj in zip(N, L)]))


def mass(psi, N, L):
    return _vol(N, L) * float(np.sum(np.abs(psi) ** 2))


def derivative(psi, N, L, axis):
    mu = freqs(N, L)[axis]
    return _fft.ifftn(1j * _bcast(mu, axis, len(N)) * _fft.fftn(psi))


def apply_Lz(psi, N, L):
    """Lz psi = -i (x D_y - y D_x) psi (eq. AME's operator) with spectral derivatives."""
    X = np.meshgrid(*axes(N, L), indexing="ij")
    return -1j * (X[0] * derivative(psi, N, L, 1) - X[1] * derivative(psi, N, L, 0))


def angular_momentum(psi, N, L):
    """<Lz> = h^d sum psi^* (-i)(x D_y - y D_x) psi (real part)."""
    X = np.meshgrid(*axes(N, L), indexing="ij")
    Dx = derivative(psi, N, L, 0)
    Dy = derivative(psi, N, L, 1)
    Lz = -1j * (X[0] * Dy - X[1] * Dx)
    return _vol(N, L) * float(np.real(np.sum(np.conj(psi) * Lz)))


def energy_parts(prob, psi, t=0.0):
    """(E_kin, E_pot, E_int, E_non, E_rot, E_total) of psi on prob's grid."""
    N, L = prob.N, prob.L
    vol = _vol(N, L)
    n = float(np.prod(N))
    om = kinetic_symbol(N, L, prob.s, prob.m)
    ph = _fft.fftn(psi)
    ekin = 0.5 * vol / n * float(np.sum(om * np.abs(ph) ** 2))
    rho = np.abs(psi) ** 2
    W = trap(N, L, prob.gamma, prob.Omega, t, getattr(prob, "lattice", None))
    if getattr(prob, "U", None) is not None:
        W = W + prob.U
    epot = vol * float(np.sum(W * rho))
    eint = 0.5 * prob.beta * vol * float(np.sum(rho ** 2))
    enon = 0.5 * prob.lam * vol * float(np.sum(prob.potential(rho, t) * rho))
    erot = -prob.Omega * angular_momentum(psi, N, L)
    return ekin, epot, eint, enon, erot, ekin + epot + eint + enon + erot


def center_of_mass(psi, N, L):
    X = np.meshgrid(*axes(N, L), indexing="ij")
    rho = np.abs(psi) ** 2
    vol = _vol(N, L)
    return np.array([vol * float(np.sum(Xj * rho)) for Xj in X])


def moments(psi, N, L, Omega=0.0, t=0.0):
    """(mass, x_c, delta) in the lab frame (eqs. mass, CoM, ConWidth).

    psi is given on the rotating-frame grid x~; with x = A(t) x~ the moments
    are transformed by rotating every grid point and summing directly.
    """
    d = len(N)
    X = np.meshgrid(*axes(N, L), indexing="ij")
    th = Omega * t
    lab = list(X)
    lab[0] = np.cos(th) * X[0] + np.sin(th) * X[1]
    lab[1] = -np.sin(th) * X[0] + np.cos(th) * X[1]
    rho = np.abs(psi) ** 2
    vol = _vol(N, L)
    xc = np.array([vol * float(np.sum(lab[j] * rho)) for j in range(d)])
    width = np.array([vol * float(np.sum(lab[j] ** 2 * rho)) for j in range(d)])
    return vol * float(np.sum(rho)), xc, width


def apply_H(prob, psi, rho_frozen=None):
    """H psi = (1/2)(-Lap+m^2)^s psi + (V + beta rho + lam Phi[rho]) psi - Omega Lz psi (lab frame)."""
    N, L = prob.N, prob.L
    om = kinetic_symbol(N, L, prob.s, prob.m)
    kin = _fft.ifftn(0.5 * om * _fft.fftn(psi))
    rho = np.abs(psi) ** 2 if rho_frozen is None else rho_frozen
    V = trap(N, L, prob.gamma, 0.0, 0.0, getattr(prob, "lattice", None))
    if getattr(prob, "U", None) is not None:
        if prob.Omega != 0.0:
            # U is static in the rotating Lagrangian coordinates, which turn
            # against the frame of H unless Omega = 0
            raise NotImplementedError("an external potential needs Omega = 0 in H psi")
        V = V + prob.U
    pot = (V + prob.beta * rho + prob.lam * prob.potential(rho)) * psi
    X = np.meshgrid(*axes(N, L), indexing="ij")
    Lz = -1j * (X[0] * derivative(psi, N, L, 1) - X[1] * derivative(psi, N, L, 0))
    return kin + pot - prob.Omega * Lz
