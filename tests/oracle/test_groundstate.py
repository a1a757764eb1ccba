"""Pins of the ground-state oracle (backward-Euler GFDN with a preconditioned Krylov solve)."""
import math

import numpy as np

from oracle import diagnostics as dg
from oracle import groundstate as gs
from oracle.scheme import Problem, axes


def _prob(N, L, s, Omega, beta, lam, gamma=(1.0, 1.0, 1.0), kernel="coulomb"):
    d = len(N)
    c = 1.0 / (2 ** (d - 1) * math.pi)
    return Problem(d, N, L, s, Omega, gamma[:d], beta, lam, kernel=kernel, mu=1.0, c=c)


def test_step_solves_the_backward_euler_system():
    # A^{BE,n} phi1 = phi^n/dt, checked with the independently written H psi
    # (diagnostics.apply_H with the frozen density rho^n).
    p = _prob((16, 24), (6.0, 7.0), 0.7, 0.6, 20.0, 3.0)
    g = gs.GroundState(p, dt=0.05)
    phi_n = gs.initial_guess(p.N, p.L, 0.6)
    phi1, (its, res) = g.solve(phi_n, rtol=1e-13)
    lhs = dg.apply_H(p, phi1, rho_frozen=np.abs(phi_n) ** 2) + phi1 / g.dt
    rel = np.linalg.norm(lhs - phi_n / g.dt) / np.linalg.norm(phi_n / g.dt)
    assert res < 1e-12 and its > 0
    assert rel < 1e-10


def test_krylov_solution_equals_dense_solve():
    # brute force on a tiny grid: assemble A^{BE,n} column by column and solve directly
    p = _prob((8, 8), (4.0, 4.0), 0.8, 0.5, 10.0, 2.0)
    g = gs.GroundState(p, dt=0.1)
    phi_n = gs.initial_guess(p.N, p.L, 0.5)
    rho = np.abs(phi_n) ** 2
    n = phi_n.size
    A = np.zeros((n, n), dtype=complex)
    for k in range(n):
        e = np.zeros(n, dtype=complex)
        e[k] = 1.0
        E = e.reshape(p.N)
        A[:, k] = (dg.apply_H(p, E, rho_frozen=rho) + E / g.dt).ravel()
    direct = np.linalg.solve(A, (phi_n / g.dt).ravel()).reshape(p.N)
    phi1, _ = g.solve(phi_n, rtol=1e-14)
    assert np.linalg.norm(phi1 - direct) / np.linalg.norm(direct) < 1e-11


def _overlap(a, b, N, L):
    vol = float(np.prod([2.0 * Lj / Nj for Nj, Lj in zip(N, L)]))
    return vol * np.sum(np.conj(a) * b)


def test_linear_harmonic_ground_state_2d_rotating():
    # s = 1, beta = lam = 0, gamma = 1: for |Omega| < 1 the ground state of
    # H - Omega Lz is the Gaussian pi^{-1/2} exp(-|x|^2/2) with energy 1; the
    # initial guess carries a vortex component (energy 2 - Omega) that decays.
    p = _prob((32, 32), (8.0, 8.0), 1.0, 0.3, 0.0, 0.0)
    g = gs.GroundState(p, dt=1.0)
    phi, steps, stats = g.run(gs.initial_guess(p.N, p.L, 0.3), eps0=1e-10)
    X = np.meshgrid(*axes(p.N, p.L), indexing="ij")
    ho = np.exp(-(X[0] ** 2 + X[1] ** 2) / 2.0) / math.sqrt(math.pi)
    assert abs(abs(_overlap(ho, phi, p.N, p.L)) - 1.0) < 1e-10
    E = dg.energy_parts(p, phi)[5]
    assert abs(E - 1.0) < 1e-10
    assert steps < 200


def test_linear_harmonic_ground_state_3d():
    # anisotropic trap: energy (gx + gy + gz)/2 at s = 1
    p = _prob((24, 24, 24), (6.0, 6.0, 4.0), 1.0, 0.0, 0.0, 0.0, gamma=(1.0, 1.0, 2.0))
    g = gs.GroundState(p, dt=1.0)
    phi, steps, _ = g.run(gs.initial_guess(p.N, p.L, 0.0, p.gamma), eps0=1e-10)
    E = dg.energy_parts(p, phi)[5]
    assert abs(E - 2.0) < 1e-9


def test_fractional_nonlinear_energy_decreases_and_stationarity():
    # s = 0.6, repulsive contact and Coulomb terms, no rotation: the energy
    # decreases along the flow, and at convergence phi solves the
    # Euler-Lagrange equation H phi = mu phi (mu the chemical potential).
    p = _prob((32, 32), (8.0, 8.0), 0.6, 0.0, 50.0, 2.0)
    g = gs.GroundState(p, dt=0.2)
    phi = gs.initial_guess(p.N, p.L, 0.0)
    energies = [dg.energy_parts(p, phi)[5]]
    for _ in range(300):
        phi, stats = g.step(phi)
        energies.append(dg.energy_parts(p, phi)[5])
        if stats[2] <= 1e-11 * g.dt:
            break
    assert stats[2] <= 1e-11 * g.dt
    assert np.all(np.diff(energies) <= 1e-12)
    H = dg.apply_H(p, phi)
    mu = float(np.real(_overlap(phi, H, p.N, p.L)))
    res = np.linalg.norm(H - mu * phi) / np.linalg.norm(mu * phi)
    assert res < 1e-8


def test_run_to_stopping_rules():
    # The loop with the paper's difference rule stops where run() stops; with the
    # energy-change rule it stops once |E^{n+1} - E^n| <= eps, here at the s = 1
    # harmonic ground state (energy 1 exactly), the energies decreasing on the way.
    p = _prob((32, 32), (8.0, 8.0), 1.0, 0.3, 0.0, 0.0)
    g = gs.GroundState(p, dt=1.0)
    phi0 = gs.initial_guess(p.N, p.L, 0.3)
    a, na, _ = g.run(phi0, eps0=1e-10)
    b, nb, rule, en = g.run_to(phi0, eps_diff=1e-10)
    assert (nb, rule) == (na, 1) and np.array_equal(a, b)
    assert len(en) == nb + 1 and abs(en[-1] - dg.energy_parts(p, b)[5]) == 0.0
    c, nc, rule, en = g.run_to(phi0, eps_energy=1e-14)
    assert rule == 2 and abs(en[-1] - en[-2]) <= 1e-14 and nc < 200
    assert abs(en[-1] - 1.0) < 1e-10 and np.all(np.diff(en) <= 1e-15)
    _, nd, rule, en = g.run_to(phi0, eps_energy=1e-14, max_steps=3)
    assert (nd, rule, len(en)) == (3, 0, 4)
