"""Pins of the oracle's TS2-GauSum step (Section 4.2 of the paper)."""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import diagnostics as dg
from oracle import scheme


def test_free_evolution_is_one_multiplier():
    # beta = lam = 0, V = 0: n steps equal exp(-i n dt omega/2) for any s.
    N, L = (32, 32), (6.0, 6.0)
    for s in (0.4, 1.0, 1.5):
        pr = scheme.Problem(2, N, L, s, 0.3, (0.0, 0.0), 0.0, 0.0, kernel="none")
        psi0 = W.harmonic_vortex_2d(N, L, seed=1)
        psi, _ = pr.run(psi0, 7, 1e-2)
        om = scheme.kinetic_symbol(N, L, s)
        ref = np.fft.ifftn(np.exp(-1j * 7 * 1e-2 * om / 2) * np.fft.fftn(psi0))
        assert np.linalg.norm(psi - ref) / np.linalg.norm(ref) < 1e-13


@pytest.mark.parametrize("d", [2, 3])
def test_free_gaussian_s1_closed_form(d):
    # i psi_t = -(1/2) Lap psi, psi0 = pi^{-d/4} exp(-|x|^2/2):
    # psi(t) = pi^{-d/4} (1+it)^{-d/2} exp(-|x|^2 / (2(1+it))).
    N = (128, 128) if d == 2 else (64, 64, 64)
    L = (14.0,) * d if d == 2 else (10.0,) * d
    pr = scheme.Problem(d, N, L, 1.0, 0.0, (0.0,) * d, 0.0, 0.0, kernel="none")
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    r2 = sum(x * x for x in X)
    psi0 = math.pi ** (-d / 4) * np.exp(-r2 / 2) + 0j
    t = 0.5
    psi, _ = pr.run(psi0, 5, t / 5)
    exact = math.pi ** (-d / 4) * (1 + 1j * t) ** (-d / 2) * np.exp(-r2 / (2 * (1 + 1j * t)))
    assert np.linalg.norm(psi - exact) / np.linalg.norm(exact) < 1e-12


@pytest.mark.parametrize("s", [0.5, 0.75, 1.3])
def test_fractional_free_autocorrelation(s):
    # a(t) = <psi0, exp(-i t omega/2) psi0> for psi0 = phi_ho in 2D, against
    # the k-space rectangle rule (2L)^{-2} sum_k |phi_hat(k)|^2 exp(-i t |k|^{2s}/2)
    # of the closed-form transform |phi_hat|^2 = 4 pi exp(-|k|^2).
    N, L = (96, 96), (12.0, 12.0)
    pr = scheme.Problem(2, N, L, s, 0.0, (0.0, 0.0), 0.0, 0.0, kernel="none")
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    psi0 = np.exp(-(X[0] ** 2 + X[1] ** 2) / 2) / math.sqrt(math.pi) + 0j
    t = 0.8
    psi, _ = pr.run(psi0, 4, t / 4)
    vol = (2 * L[0] / N[0]) ** 2
    got = vol * np.sum(np.conj(psi0) * psi)
    ks = np.meshgrid(*[2 * math.pi * np.fft.fftfreq(n, d=2 * l / n) for n, l in zip(N, L)], indexing="ij")
    k2 = ks[0] ** 2 + ks[1] ** 2
    ref = np.sum(4 * math.pi * np.exp(-k2) * np.exp(-1j * t * k2 ** s / 2)) / (2 * L[0]) ** 2
    assert abs(got - ref) < 1e-13
    # and it tends to the continuum integral 2 int_0^inf exp(-k^2 - i t k^{2s}/2) k dk
    re, _ = integrate.quad(lambda k: 2 * math.exp(-k * k) * math.cos(t * k ** (2 * s) / 2) * k, 0, 12, epsabs=1e-15, limit=200)
    im, _ = integrate.quad(lambda k: -2 * math.exp(-k * k) * math.sin(t * k ** (2 * s) / 2) * k, 0, 12, epsabs=1e-15, limit=200)
    assert abs(got - (re + 1j * im)) < 5e-3


def test_trap_integral_matches_quadrature():
    N, L = (6, 5, 4), (3.0, 2.0, 2.5)
    gamma, Om = (1.0, 1.7, 0.6), 0.9
    t, tau = 0.37, 0.21
    P = scheme.trap_integral(N, L, gamma, Om, t, tau)
    for idx in [(0, 0, 0), (5, 4, 3), (2, 1, 2), (4, 2, 0)]:
        f = lambda s_: scheme.trap(N, L, gamma, Om, s_)[idx]
        ref, _ = integrate.quad(f, t, t + tau, epsabs=1e-15, epsrel=1e-14)
        assert abs(P[idx] - ref) < 1e-13 * max(1.0, abs(ref))
    # Omega -> 0 limit
    P0 = scheme.trap_integral(N, L, gamma, 0.0, t, tau)
    assert np.allclose(P0, tau * scheme.trap(N, L, gamma, 0.0, 0.0), rtol=1e-14, atol=0)


def test_nonlinear_substep_solves_the_pointwise_ode():
    # i phi_t = [V(A(t)x) + beta rho + lam Phi] phi with rho frozen: integrate
    # with an adaptive ODE solver at a few grid points.
    N, L = (16, 16), (4.0, 4.0)
    pr = scheme.Problem(2, N, L, 0.8, 0.7, (1.0, 1.4), 3.0, 2.0, kernel="coulomb", c=1 / (2 * math.pi))
    phi = W.harmonic_vortex_2d(N, L, seed=2)
    t0, tau = 0.3, 0.05
    out = pr.nonlinear(phi, t0, tau)
    rho = np.abs(phi) ** 2
    Phi = pr.potential(rho)
    for idx in [(3, 4), (8, 8), (15, 0), (10, 2)]:
        def rhs(t, y):
            z = y[0] + 1j * y[1]
            v = scheme.trap(N, L, pr.gamma, pr.Omega, t)[idx] + pr.beta * rho[idx] + pr.lam * Phi[idx]
            dz = -1j * v * z
            return [dz.real, dz.imag]
        sol = integrate.solve_ivp(rhs, (t0, t0 + tau), [phi[idx].real, phi[idx].imag], rtol=1e-12, atol=1e-14)
        ref = sol.y[0, -1] + 1j * sol.y[1, -1]
        assert abs(out[idx] - ref) < 1e-10 * max(abs(ref), 1e-3)


def test_mass_conserved_and_step_reversible():
    p = W.preset("plain2d")
    pr = scheme.Problem.from_params(p)
    psi0 = W.harmonic_vortex_2d(p.N, p.L, seed=0)
    psi, t = pr.run(psi0, 20, p.dt)
    assert abs(dg.mass(psi, p.N, p.L) - 1.0) < 1e-13
    back, tb = pr.run(psi, 20, -p.dt, t=t)
    assert abs(tb) < 1e-15
    assert np.linalg.norm(back - psi0) / np.linalg.norm(psi0) < 1e-12


def test_second_order_in_time():
    N, L = (64, 64), (8.0, 8.0)
    pr = scheme.Problem(2, N, L, 0.75, 0.5, (1.0, 1.2), 100.0, 1.0, kernel="coulomb", c=1 / (2 * math.pi))
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    psi0 = W.normalize((X[0] + 1j * X[1]) * np.exp(-(X[0] ** 2 + X[1] ** 2) / 2) * (1 + 0.2 * X[0]), pr.h)
    T = 0.1
    ref, _ = pr.run(psi0, 640, T / 640)
    errs = []
    for n in (20, 40, 80):
        p, _ = pr.run(psi0, n, T / n)
        errs.append(np.linalg.norm(p - ref) / np.linalg.norm(ref))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.9 < o < 2.15 for o in orders), (errs, orders)


def test_center_of_mass_follows_classical_ode_at_s1():
    # s = 1, harmonic V, Coulomb kernel: the lab-frame centre of mass solves
    # x'' - 2 Omega J x' + (Omega^2 J^2 + Lambda) x = 0 (remark after the
    # centre-of-mass lemma); the run is in rotating coordinates, x = A(t) x~.
    N, L = (64, 64), (8.0, 8.0)
    g, Om = (1.0, 1.3), 0.4
    pr = scheme.Problem(2, N, L, 1.0, Om, g, 10.0, 2.0, kernel="coulomb", c=1 / (2 * math.pi))
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    psi = np.exp(-((X[0] - 1.0) ** 2 + (X[1] - 0.5) ** 2) / 2) / math.sqrt(math.pi) + 0j
    x0 = dg.center_of_mass(psi, N, L)
    T, n = 1.0, 500
    psi, t = pr.run(psi, n, T / n)
    A = np.array([[math.cos(Om * t), math.sin(Om * t)], [-math.sin(Om * t), math.cos(Om * t)]])
    xl = A @ dg.center_of_mass(psi, N, L)
    J = np.array([[0.0, 1.0], [-1.0, 0.0]])
    Lam = np.diag([g[0] ** 2, g[1] ** 2])

    def f(_, y):
        x, v = y[:2], y[2:]
        return np.r_[v, 2 * Om * J @ v - (Om * Om * J @ J + Lam) @ x]
    # A real initial state has no momentum: x' - Omega J x = 0 at t = 0.
    sol = integrate.solve_ivp(f, (0, T), np.r_[x0, Om * J @ x0], rtol=1e-12, atol=1e-12)
    assert np.max(np.abs(xl - sol.y[:2, -1])) < 1e-6


def test_center_of_mass_3d_ddi_nonrotating():
    # s = 1, Omega = 0, z-dipole: x_c(t) = x0 cos(gamma t) on each axis.
    N, L = (32, 32, 32), (6.0, 6.0, 6.0)
    g = (1.0, 1.0, 1.5)
    pr = scheme.Problem(3, N, L, 1.0, 0.0, g, 5.0, 3.0, kernel="ddi3")
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    x0 = np.array([0.5, -0.3, 0.4])
    psi = np.exp(-sum((X[i] - x0[i]) ** 2 for i in range(3)) / 2) + 0j
    psi = W.normalize(psi, pr.h)
    T, n = 0.6, 120
    psi, t = pr.run(psi, n, T / n)
    xc = dg.center_of_mass(psi, N, L)
    assert np.max(np.abs(xc - x0 * np.cos(np.array(g) * T))) < 2e-5


def test_angular_momentum_conserved_isotropic_s1():
    # Lemma on <Lz>: radial V and a Coulomb kernel conserve <Lz>.
    N, L = (64, 64), (8.0, 8.0)
    pr = scheme.Problem(2, N, L, 1.0, 0.5, (1.0, 1.0), 50.0, 1.0, kernel="coulomb", c=1 / (2 * math.pi))
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    psi0 = W.normalize((X[0] + 1j * X[1]) * np.exp(-(X[0] ** 2 + X[1] ** 2) / 2) * (1 + 0.3 * X[0]), pr.h)
    lz0 = dg.angular_momentum(psi0, N, L)
    psi, _ = pr.run(psi0, 100, 1e-3)
    # Continuum law; on the grid the drift is a spatial discretisation error.
    assert abs(dg.angular_momentum(psi, N, L) - lz0) < 2e-7


def test_energy_conserved_to_second_order():
    # Rotating frame, isotropic trap: the lab energy drifts as O(dt^2) + <Lz> drift.
    N, L = (64, 64), (8.0, 8.0)
    pr = scheme.Problem(2, N, L, 1.0, 0.5, (1.0, 1.0), 50.0, 1.0, kernel="coulomb", c=1 / (2 * math.pi))
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    psi0 = W.normalize((X[0] + 1j * X[1]) * np.exp(-(X[0] ** 2 + X[1] ** 2) / 2) * (1 + 0.3 * X[0]), pr.h)
    e0 = dg.energy_parts(pr, psi0)[-1]
    drift = []
    for dt in (4e-3, 2e-3):
        psi, t = pr.run(psi0, int(round(0.2 / dt)), dt)
        drift.append(abs(dg.energy_parts(pr, psi, t)[-1] - e0))
    assert drift[1] < drift[0] / 3.0
    assert drift[1] < 1e-4


def test_widths_follow_2d_virial_law_at_s1():
    # s = 1, isotropic trap gamma, cubic nonlinearity, d = 2: the virial
    # identity gives d^2<r^2>/dt^2 = 4 E0 - 4 gamma^2 <r^2>, E0 the energy
    # without the rotation term (conserved, like <Lz>, for a radial trap), so
    # for a real initial state <r^2>(t) = E0/gamma^2 + (<r^2>(0) - E0/gamma^2) cos(2 gamma t).
    # <r^2> = delta_x + delta_y (eq. ConWidth) read in the lab frame.
    N, L = (64, 64), (8.0, 8.0)
    gam, Om = 1.2, 0.5
    pr = scheme.Problem(2, N, L, 1.0, Om, (gam, gam), 5.0, 0.0, kernel="none")
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    psi = W.normalize(np.exp(-(X[0] - 0.4) ** 2 / 1.6 - X[1] ** 2 / 0.9) + 0j, pr.h)
    ek, ep, ei, _, _, _ = dg.energy_parts(pr, psi)
    E0 = ek + ep + ei
    r0 = float(np.sum(dg.moments(psi, N, L)[2]))
    T, n = 1.0, 1000
    psi, t = pr.run(psi, n, T / n)
    r2 = float(np.sum(dg.moments(psi, N, L, Omega=Om, t=t)[2]))
    exact = E0 / gam ** 2 + (r0 - E0 / gam ** 2) * math.cos(2 * gam * t)
    # second-order splitting error: 6e-7, 1.5e-7, 3.4e-8 at 500, 1000, 2000 steps
    assert abs(r2 - exact) < 5e-7


def test_fourth_order_composition_converges_at_order_4():
    # the triple-jump composition of TS2 steps: error ratio ~16 per halving
    # (TS2 itself gives ~4), rotating anisotropic trap and Coulomb kernel
    N, L = (64, 64), (8.0, 8.0)
    pr = scheme.Problem(2, N, L, 0.8, 0.6, (1.0, 1.3), 30.0, 2.0, kernel="coulomb", c=1 / (2 * math.pi))
    psi0 = W.harmonic_vortex_2d(N, L, seed=3)
    T = 0.4
    ref, tr = pr.run4(psi0, 256, T / 256)
    assert abs(tr - T) < 1e-15
    errs = []
    for n in (8, 16, 32):
        p, _ = pr.run4(psi0, n, T / n)
        errs.append(np.linalg.norm(p - ref) / np.linalg.norm(ref))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.6 < o < 4.4 for o in orders), (errs, orders)


def test_fourth_order_free_evolution_is_exact():
    # no trap and no interaction: every sub-step is the exact kinetic flow and
    # the lengths sum to dt, so n steps equal one kinetic step of length n dt
    N, L = (32, 48), (6.0, 7.0)
    pr = scheme.Problem(2, N, L, 0.7, 0.0, (0.0, 0.0), 0.0, 0.0, kernel="none")
    psi0 = W.harmonic_vortex_2d(N, L, seed=4)
    p, _ = pr.run4(psi0, 5, 0.03)
    q = scheme.kinetic(psi0, N, L, 0.7, 0.15)
    assert np.linalg.norm(p - q) / np.linalg.norm(q) < 1e-13


def _turning_dipole_drift(sign, nsteps):
    # 3D dipole along a tilted axis with rotation: in the rotating Lagrangian
    # coordinates the axis turns, m(t) = A^{-1}(t) n; the rotating-frame energy
    # (its instantaneous kernel at time t) is conserved by the equation.
    from oracle import gausum
    orig = gausum.dipole_average
    gausum.dipole_average = lambda axis, Omega=0.0, t=0.0, tau=0.0: orig(axis, sign * Omega, t, tau)
    try:
        N, L = (24, 24, 24), (5.0, 5.0, 5.0)
        pr = scheme.Problem(3, N, L, 0.9, 0.5, (1.0, 1.0, 1.2), 20.0, 20.0, kernel="ddi3", axis=(0.6, 0.0, 0.8))
        X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
        psi = W.normalize(np.exp(-X[0] ** 2 / 1.2 - X[1] ** 2 / 0.7 - X[2] ** 2) * (1 + 0.2 * X[0] + 0.3j * X[1]),
                          pr.h)
        E0 = dg.energy_parts(pr, psi, 0.0)[5]
        psi, t = pr.run(psi, nsteps, 1.0 / nsteps)
        return dg.energy_parts(pr, psi, t)[5] - E0
    finally:
        gausum.dipole_average = orig


def test_turning_dipole_axis_conserves_the_rotating_frame_energy():
    # second-order drift (2.6e-3, 6.6e-4 over t = 1 at 50, 100 steps); the axis
    # turned the wrong way (m = A n) drifts by 1.7e-2 and does not converge
    d50, d100 = _turning_dipole_drift(1, 50), _turning_dipole_drift(1, 100)
    assert abs(d100) < 1e-3 and 3.5 < d50 / d100 < 4.5
    assert abs(_turning_dipole_drift(-1, 100)) > 10 * abs(d100)


def test_plane_wave_phase_with_mass_term():
    # free evolution (no trap, no interaction) of a grid plane wave exp(i k.x):
    # exp(-i T (|k|^2 + m^2)^s / 2) (eq. SFSE with the mass term)
    N, L = (32, 24), (4.0, 3.0)
    s, m = 0.7, 1.3
    pr = scheme.Problem(2, N, L, s, 0.0, (0.0, 0.0), 0.0, 0.0, kernel="none", m=m)
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    k = (3 * math.pi / L[0], -2 * math.pi / L[1])
    psi0 = np.exp(1j * (k[0] * X[0] + k[1] * X[1]))
    psi, t = pr.run(psi0, 7, 0.11)
    om = (k[0] ** 2 + k[1] ** 2 + m * m) ** s
    assert np.max(np.abs(psi - psi0 * np.exp(-0.5j * t * om))) < 1e-13


def test_lattice_time_integral_against_adaptive_quadrature():
    # int_t^{t+tau} V_L(A(s) x~) ds on the grid against scipy's adaptive quad at sample points
    N, L = (16, 12), (4.0, 3.0)
    lat = ((10.0, 7.0, 0.0), (math.pi, 1.3, 0.0))
    Om, t, tau = 0.8, 0.9, 0.3
    P = scheme.lattice_integral(N, L, Om, lat, t, tau)
    ax = scheme.axes(N, L)
    for i, j in [(0, 0), (3, 7), (11, 2), (15, 11)]:
        x, y = ax[0][i], ax[1][j]

        def f(s):
            c, sn = math.cos(Om * s), math.sin(Om * s)
            return 10.0 * math.sin(math.pi * (c * x + sn * y)) ** 2 + 7.0 * math.sin(1.3 * (-sn * x + c * y)) ** 2
        ref, _ = integrate.quad(f, t, t + tau, epsabs=1e-14, epsrel=1e-14)
        assert abs(P[i, j] - ref) < 1e-13 * max(1.0, abs(ref))
    # without rotation: exactly tau V_L
    P0 = scheme.lattice_integral(N, L, 0.0, lat, t, tau)
    X = np.meshgrid(*ax, indexing="ij")
    assert np.max(np.abs(P0 - tau * scheme.lattice_potential(X, lat))) < 1e-13


def _lattice_drift(nsteps):
    N, L = (48, 48), (6.0, 6.0)
    pr = scheme.Problem(2, N, L, 0.9, 0.5, (1.0, 1.0), 10.0, 0.0, kernel="none")
    pr.lattice = ((2.0, 2.0, 0.0), (0.5 * math.pi, 0.5 * math.pi, 0.0))
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    psi = W.normalize(np.exp(-(X[0] - 0.5) ** 2 / 1.2 - X[1] ** 2 / 0.8) * (1 + 0.3j * X[1]) + 0j, pr.h)
    E0 = dg.energy_parts(pr, psi, 0.0)[5]
    psi, t = pr.run(psi, nsteps, 1.0 / nsteps)
    return dg.energy_parts(pr, psi, t)[5] - E0


def test_rotating_lattice_conserves_the_rotating_frame_energy():
    # the lattice is static in the frame of eq. SFSE, where the Hamiltonian does
    # not depend on time; in rotating coordinates it turns, and the energy with
    # W(x~, t) = V(A(t) x~) is conserved up to the splitting error (order 2)
    d50, d100 = _lattice_drift(50), _lattice_drift(100)
    assert abs(d100) < 1e-3 and 3.5 < d50 / d100 < 4.5
