"""Pins of the oracle's discrete adjoint (oracle/adjoint.py): central finite
differences of the oracle's own forward scheme in random directions."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as adj
from oracle import scheme


def _setup(d):
    rng = np.random.default_rng(11 + d)
    if d == 2:
        N, L = (32, 32), (6.0, 6.0)
        pr = scheme.Problem(2, N, L, 0.7, 0.5, (1.0, 1.3), 20.0, 3.0, kernel="coulomb", c=1 / (2 * math.pi))
        psi0 = W.harmonic_vortex_2d(N, L, seed=5)
        tgt = W.harmonic_vortex_2d(N, L, seed=6) * np.exp(0.3j * scheme.axes(N, L)[0][:, None])
    else:
        N, L = (16, 16, 12), (5.0, 5.0, 4.0)
        pr = scheme.Problem(3, N, L, 0.9, 0.4, (1.0, 1.0, 1.5), 30.0, 8.0, kernel="ddi3")
        psi0 = W.anisotropic_gaussian(N, L, (1.0, 1.0, 1.5), seed=5)
        tgt = W.anisotropic_gaussian(N, L, (1.2, 0.9, 1.5), seed=6)
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    pr.U = 0.3 * np.sin(X[0]) * np.cos(0.5 * X[1]) + 0.05 * rng.standard_normal(N)
    dpsi = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    dU = rng.standard_normal(N)
    return pr, psi0, tgt, dpsi, dU


def _loss(pr, psi0, tgt, nsteps, dt):
    psi, _ = pr.run(psi0, nsteps, dt)
    return adj.loss_and_grad(psi, tgt, pr.N, pr.L)[0]


def test_loss_gradient_by_finite_differences():
    pr, psi0, tgt, dpsi, _ = _setup(2)
    L0, g = adj.loss_and_grad(psi0, tgt, pr.N, pr.L)
    eps = 1e-6
    fd = (adj.loss_and_grad(psi0 + eps * dpsi, tgt, pr.N, pr.L)[0]
          - adj.loss_and_grad(psi0 - eps * dpsi, tgt, pr.N, pr.L)[0]) / (2 * eps)
    an = float(np.real(np.sum(np.conj(g) * dpsi)))
    assert abs(fd - an) < 1e-8 * max(1.0, abs(an))


@pytest.mark.parametrize("d", [2, 3])
def test_adjoint_by_finite_differences(d):
    # dL = Re sum conj(g0) dpsi0 + sum gU dU, against central differences of
    # the forward scheme (nonlinear phase, GauSum term, rotating trap integral, U)
    pr, psi0, tgt, dpsi, dU = _setup(d)
    nsteps, dt = 4, 0.05
    psiT, _ = pr.run(psi0, nsteps, dt)
    _, gT = adj.loss_and_grad(psiT, tgt, pr.N, pr.L)
    g0, gU = adj.run_adjoint(pr, psi0, nsteps, dt, gT)
    eps = 1e-6
    fd_psi = (_loss(pr, psi0 + eps * dpsi, tgt, nsteps, dt) - _loss(pr, psi0 - eps * dpsi, tgt, nsteps, dt)) / (2 * eps)
    an_psi = float(np.real(np.sum(np.conj(g0) * dpsi)))
    U0 = pr.U
    pr.U = U0 + eps * dU
    lp = _loss(pr, psi0, tgt, nsteps, dt)
    pr.U = U0 - eps * dU
    lm = _loss(pr, psi0, tgt, nsteps, dt)
    pr.U = U0
    fd_U = (lp - lm) / (2 * eps)
    an_U = float(np.sum(gU * dU))
    assert abs(fd_psi - an_psi) < 1e-7 * max(1.0, abs(an_psi)), (fd_psi, an_psi)
    assert abs(fd_U - an_U) < 1e-7 * max(1.0, abs(an_U)), (fd_U, an_U)
    # the directions are not trivial
    assert abs(an_psi) > 1e-3 and abs(an_U) > 1e-4


def test_linear_adjoint_is_the_inverse():
    # beta = lam = 0: the step is unitary, so its adjoint is its inverse; the
    # adjoint of psi(T) itself is psi0
    N, L = (32, 24), (6.0, 5.0)
    pr = scheme.Problem(2, N, L, 0.8, 0.6, (1.0, 1.2), 0.0, 0.0, kernel="none")
    psi0 = W.harmonic_vortex_2d(N, L, seed=7)
    psiT, _ = pr.run(psi0, 5, 0.04)
    g0, gU = adj.run_adjoint(pr, psi0, 5, 0.04, psiT)
    assert np.linalg.norm(g0 - psi0) / np.linalg.norm(psi0) < 1e-13
