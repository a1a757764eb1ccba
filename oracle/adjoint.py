"""Discrete adjoint of the TS2-GauSum step, float64 (oracle; test infrastructure only).

The paper gives no adjoint.  This module is the reverse-mode derivative of
the oracle's own discrete scheme (scheme.Problem.step: eqs. tssp1-tssp3 in
rotating Lagrangian coordinates, with an optional potential U on the grid),
derived by hand.

Gradient convention (the one torch uses for complex tensors): for a real loss
L of a complex array psi, g = dL/dRe(psi) + i dL/dIm(psi), so that
dL = Re sum conj(g) dpsi.

One forward step over [t, t+dt]:
    psi1 = K psi,   K = exp(-i (dt/2) omega/2) in Fourier space (unitary),
    theta = dt beta |psi1|^2 + lam dt Phi[|psi1|^2] + P(x~; t, t+dt) + dt U,
    psi2 = psi1 exp(-i theta),
    psi' = K psi2.
Its reverse, given g' = dL/dpsi':
    g2 = K^H g',                         K^H = exp(+i (dt/2) omega/2)
    q  = Im(conj(g2) psi2)               (real; dL/dtheta = q)
    r  = dt beta q + lam dt Phi[q]       (Phi is self-adjoint: the padded circular
                                          convolution with a real, even multiplier)
    g1 = g2 exp(+i theta) + 2 r psi1     (theta depends on |psi1|^2)
    g  = K^H g1,      dL/dU += dt q.

Parity: pinned by central finite differences of the oracle's forward scheme
in random directions of psi0 and U (tests/oracle/test_adjoint.py).
"""
from __future__ import annotations

import numpy as np

from . import diagnostics as dg
from .scheme import kinetic, trap_integral


def _vol(N, L):
    return float(np.prod([2.0 * Lj / Nj for Nj, Lj in zip(N, L)]))


def _theta(prob, psi1, t, dt):
    rho = np.abs(psi1) ** 2
    th = dt * prob.beta * rho + prob.lam * dt * prob.potential(rho, t, dt)
    th = th + trap_integral(prob.N, prob.L, prob.gamma, prob.Omega, t, dt, prob.lattice)
    if prob.U is not None:
        th = th + dt * prob.U
    return th


def step_adjoint(prob, psi, t, dt, g_next):
    """Reverse of one step from psi at time t: returns (dL/dpsi, dL/dU contribution)."""
    N, L, s, m = prob.N, prob.L, prob.s, prob.m
    psi1 = kinetic(psi, N, L, s, 0.5 * dt, m)
    th = _theta(prob, psi1, t, dt)
    psi2 = psi1 * np.exp(-1j * th)
    g2 = kinetic(g_next, N, L, s, -0.5 * dt, m)
    q = np.imag(np.conj(g2) * psi2)
    r = dt * prob.beta * q + prob.lam * dt * prob.potential(q, t, dt)
    g1 = g2 * np.exp(1j * th) + 2.0 * r * psi1
    return kinetic(g1, N, L, s, -0.5 * dt, m), dt * q


def run_adjoint(prob, psi0, nsteps, dt, g_T, t=0.0):
    """dL/dpsi0 and dL/dU for nsteps steps from psi0 at time t, given g_T = dL/dpsi(T)."""
    states = [psi0]
    for k in range(int(nsteps) - 1):
        states.append(prob.step(states[-1], t + k * dt, dt)[0])
    g = g_T
    gU = np.zeros(prob.N)
    for k in reversed(range(int(nsteps))):
        g, dU = step_adjoint(prob, states[k], t + k * dt, dt, g)
        gU = gU + dU
    return g, gU


def loss_and_grad(psi, psi_target, N, L, w_lz=0.1):
    """L = |<psi_target, psi>|^2 + w_lz <Lz> and g = dL/dpsi.

    <a, b> = h^d sum conj(a) b; d|o|^2 = Re conj(2 h^d o a) db for o = <a, b>;
    <Lz> = h^d sum conj(psi) Lz psi with Lz Hermitian, so its gradient is
    2 h^d Lz psi.
    """
    vol = _vol(N, L)
    o = vol * np.sum(np.conj(psi_target) * psi)
    Lz = dg.apply_Lz(psi, N, L)
    lz = vol * float(np.real(np.sum(np.conj(psi) * Lz)))
    loss = float(abs(o) ** 2) + w_lz * lz
    g = 2.0 * vol * o * psi_target + w_lz * 2.0 * vol * Lz
    return loss, g
