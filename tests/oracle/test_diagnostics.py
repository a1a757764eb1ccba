"""Pins of the oracle's mass, energy, <Lz> and H*psi against closed forms."""
import math

import numpy as np
import pytest
from scipy import special

import workloads as W
from oracle import diagnostics as dg
from oracle import scheme


def _ho(N, L):
    d = len(N)
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    r2 = sum(x * x for x in X)
    return X, math.pi ** (-d / 4) * np.exp(-r2 / 2) + 0j


def _kspace_rectangle_rule(N, L, s):
    # (1/2)(2L)^{-d} sum_k |k|^{2s} |phi_hat(k)|^2 with the closed-form
    # transform phi_hat(k) = pi^{-d/4} (2 pi)^{d/2} exp(-|k|^2/2) on the DFT grid.
    d = len(N)
    ks = np.meshgrid(*[2 * math.pi * np.fft.fftfreq(n, d=2 * l / n) for n, l in zip(N, L)], indexing="ij")
    k2 = sum(k * k for k in ks)
    ph2 = math.pi ** (-d / 2) * (2 * math.pi) ** d * np.exp(-k2)
    return 0.5 * float(np.sum(k2 ** s * ph2)) / float(np.prod([2 * l for l in L]))


@pytest.mark.parametrize("d,s", [(2, 0.5), (2, 0.75), (2, 1.0), (2, 2.0), (3, 0.8), (3, 1.0)])
def test_energies_of_harmonic_ground_state(d, s):
    # Continuum: E_kin = Gamma(d/2+s)/(2 Gamma(d/2)); E_pot = d/4 (gamma = 1);
    # E_int = (beta/2)(2 pi)^{-d/2}; mass 1; <Lz> = 0.  For fractional s the
    # symbol |k|^{2s} has a cusp at k = 0, so the grid value is the k-space
    # rectangle rule of the closed-form transform (checked to round-off) and
    # approaches the continuum value only as the box grows.
    N = (128, 128) if d == 2 else (64, 64, 64)
    L = (12.0,) * d if d == 2 else (10.0,) * d
    beta = 3.0
    pr = scheme.Problem(d, N, L, s, 0.0, (1.0,) * d, beta, 0.0, kernel="none")
    _, psi = _ho(N, L)
    ek, ep, ei, en, er, et = dg.energy_parts(pr, psi)
    assert abs(ek - _kspace_rectangle_rule(N, L, s)) < 1e-12
    cont = special.gamma(d / 2 + s) / (2 * special.gamma(d / 2))
    if float(s).is_integer():
        assert abs(ek - cont) < 1e-12
    else:
        assert abs(ek - cont) < 5e-3
    assert abs(ep - d / 4) < 1e-12
    assert abs(ei - beta / 2 * (2 * math.pi) ** (-d / 2)) < 1e-12
    assert abs(dg.mass(psi, N, L) - 1.0) < 1e-12
    assert abs(dg.angular_momentum(psi, N, L)) < 1e-12


def test_vortex_angular_momentum_and_s1_energy():
    N, L = (128, 128), (12.0, 12.0)
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    psi = (X[0] + 1j * X[1]) * np.exp(-(X[0] ** 2 + X[1] ** 2) / 2) / math.sqrt(math.pi)
    assert abs(dg.angular_momentum(psi, N, L) - 1.0) < 1e-12
    Om = 0.3
    pr = scheme.Problem(2, N, L, 1.0, Om, (1.0, 1.0), 0.0, 0.0, kernel="none")
    ek, ep, ei, en, er, et = dg.energy_parts(pr, psi)
    # 2D oscillator state with one quantum: E_kin = E_pot = 1; E_rot = -Omega.
    assert abs(ek - 1.0) < 1e-12 and abs(ep - 1.0) < 1e-12
    assert abs(er + Om) < 1e-12 and abs(et - (2.0 - Om)) < 1e-12


def test_nonlocal_energy_closed_form():
    N, L = (48, 48, 48), (6.0, 6.0, 6.0)
    X, psi = _ho(N, L)  # rho = pi^{-3/2} exp(-r^2)
    lam = 2.0
    pr = scheme.Problem(3, N, L, 1.0, 0.0, (1.0,) * 3, 0.0, lam, kernel="coulomb", c=1 / (4 * math.pi))
    en = dg.energy_parts(pr, psi)[3]
    assert abs(en - lam / 2 * math.sqrt(2 / math.pi) / (4 * math.pi)) < 1e-13


def test_apply_H_eigenstates_s1():
    # H phi_ho = (d/2) phi_ho;  H phi_v = (2 - Omega) phi_v in 2D (Lz phi_v = phi_v).
    N, L = (64, 64), (10.0, 10.0)
    X, ho = _ho(N, L)
    pr = scheme.Problem(2, N, L, 1.0, 0.0, (1.0, 1.0), 0.0, 0.0, kernel="none")
    assert np.max(np.abs(dg.apply_H(pr, ho) - 1.0 * ho)) < 1e-12
    vort = (X[0] + 1j * X[1]) * np.exp(-(X[0] ** 2 + X[1] ** 2) / 2) / math.sqrt(math.pi)
    Om = 0.35
    pr = scheme.Problem(2, N, L, 1.0, Om, (1.0, 1.0), 0.0, 0.0, kernel="none")
    assert np.max(np.abs(dg.apply_H(pr, vort) - (2.0 - Om) * vort)) < 1e-12


def test_apply_H_expectation_is_energy_plus_interactions():
    # <psi, H psi> = E + E_int + E_non (the chemical-potential identity).
    p = W.preset("plain2d")
    pr = scheme.Problem.from_params(p)
    psi = W.harmonic_vortex_2d(p.N, p.L, seed=4)
    vol = np.prod(pr.h)
    lhs = vol * np.sum(np.conj(psi) * dg.apply_H(pr, psi))
    ek, ep, ei, en, er, et = dg.energy_parts(pr, psi)
    assert abs(lhs.imag) < 1e-10
    assert abs(lhs.real - (et + ei + en)) < 1e-10 * abs(et)


def test_apply_H_frozen_density():
    p = W.preset("plain2d")
    pr = scheme.Problem.from_params(p)
    psi = W.harmonic_vortex_2d(p.N, p.L, seed=5)
    rho = np.abs(psi) ** 2
    assert np.allclose(dg.apply_H(pr, psi, rho_frozen=rho), dg.apply_H(pr, psi), rtol=0, atol=1e-13)
    rho2 = 0.5 * rho
    diff = dg.apply_H(pr, psi, rho_frozen=rho2) - dg.apply_H(pr, psi)
    expect = (pr.beta * (rho2 - rho) + pr.lam * pr.potential(rho2 - rho)) * psi
    assert np.max(np.abs(diff - expect)) < 1e-11


@pytest.mark.parametrize("d", [2, 3])
def test_lab_frame_moments_of_rotated_anisotropic_gaussian(d):
    # |psi|^2 is a Gaussian with mean c and covariance S = diag(a_j^2 / 2) in the
    # rotating coordinates x~; in the lab frame x = A(t) x~ its mean is A c and
    # its covariance A S A^T, so x_c = A c and delta_v = (A S A^T)_vv + (A c)_v^2.
    N = (64, 72, 48)[:d]
    L = (9.0, 10.0, 8.0)[:d]
    a = np.array([1.0, 0.7, 1.3][:d])
    c = np.array([0.8, -0.5, 0.3][:d])
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    psi = np.exp(-sum((X[j] - c[j]) ** 2 / (2 * a[j] ** 2) for j in range(d))) / math.sqrt(math.pi ** (d / 2) * np.prod(a))
    Om, t = 0.6, 1.3
    th = Om * t
    A = np.eye(d)
    A[:2, :2] = [[math.cos(th), math.sin(th)], [-math.sin(th), math.cos(th)]]
    S = np.diag(a ** 2 / 2)
    mean = A @ c
    cov = A @ S @ A.T
    m, xc, width = dg.moments(psi, N, L, Omega=Om, t=t)
    assert abs(m - 1.0) < 1e-13
    assert np.max(np.abs(xc - mean)) < 1e-13
    assert np.max(np.abs(width - (np.diag(cov) + mean ** 2))) < 1e-12
    # without rotation the moments are those of the grid coordinates
    m0, xc0, w0 = dg.moments(psi, N, L)
    assert np.max(np.abs(xc0 - c)) < 1e-13 and np.max(np.abs(w0 - (a ** 2 / 2 + c ** 2))) < 1e-12
