"""Pins of the oracle's GauSum nonlocal potential (Section 2 of the paper).

Each check compares the oracle with something other than itself: closed-form
potentials of Gaussian densities, direct numerical quadrature of the
truncated kernel's Fourier integral, a brute-force linear convolution and an
independent evaluation of the 1D integrals.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import gausum, scheme


def _radius(N, L):
    X = np.meshgrid(*scheme.axes(N, L), indexing="ij")
    return X, np.sqrt(sum(x * x for x in X))


@pytest.mark.parametrize("c", [1.0, 1.0 / (4.0 * math.pi)])
def test_coulomb_3d_gaussian_closed_form(c):
    # U = c/|x|, rho = pi^{-3/2} exp(-r^2)  =>  Phi = c erf(r)/r.
    N, L = (48, 48, 48), (6.0, 6.0, 6.0)
    X, r = _radius(N, L)
    rho = math.pi ** -1.5 * np.exp(-r ** 2)
    phi = gausum.potential(rho, N, L, "coulomb", mu=1.0, c=c)
    rs = np.where(r > 0, r, 1.0)
    exact = c * np.where(r > 0, special.erf(rs) / rs, 2.0 / math.sqrt(math.pi))
    assert np.linalg.norm(phi - exact) / np.linalg.norm(exact) < 1e-13
    # Interaction integral int Phi rho = c sqrt(2/pi).
    vol = np.prod([2 * l / n for n, l in zip(N, L)])
    assert abs(vol * np.sum(phi * rho) - c * math.sqrt(2.0 / math.pi)) < 1e-13


def test_coulomb_2d_gaussian_closed_form():
    # U = c/|x| in 2D, rho = exp(-r^2)/pi  =>  Phi = c sqrt(pi) exp(-r^2/2) I0(r^2/2).
    N, L = (64, 64), (8.0, 8.0)
    c = 1.0 / (2.0 * math.pi)
    X, r = _radius(N, L)
    rho = np.exp(-r ** 2) / math.pi
    phi = gausum.potential(rho, N, L, "coulomb", mu=1.0, c=c)
    exact = c * math.sqrt(math.pi) * special.i0e(r ** 2 / 2.0)
    assert np.linalg.norm(phi - exact) / np.linalg.norm(exact) < 1e-13
    vol = np.prod([2 * l / n for n, l in zip(N, L)])
    assert abs(vol * np.sum(phi * rho) - c * math.sqrt(math.pi / 2.0)) < 1e-13


@pytest.mark.parametrize("ax", [2, 0, 1])
def test_ddi3_gaussian_closed_form(ax):
    # Phi = -rho - 3 d_nn [erf(r)/(4 pi r)] for a dipole along coordinate axis ax.
    N, L = (48, 48, 48), (6.0, 6.0, 6.0)
    X, r = _radius(N, L)
    rho = math.pi ** -1.5 * np.exp(-r ** 2)
    axis = tuple(1.0 if j == ax else 0.0 for j in range(3))
    phi = gausum.potential(rho, N, L, "ddi3", axis=axis)
    rs = np.where(r > 0, r, 1.0)
    g = 2.0 / math.sqrt(math.pi) * np.exp(-rs ** 2)
    fp = g / rs - special.erf(rs) / rs ** 2
    fpp = -2.0 * g - 2.0 * g / rs ** 2 + 2.0 * special.erf(rs) / rs ** 3
    z = X[ax]
    dzz = fpp * z ** 2 / rs ** 2 + fp * (1.0 / rs - z ** 2 / rs ** 3)
    dzz = np.where(r > 0, dzz, -4.0 / (3.0 * math.sqrt(math.pi)))
    exact = -rho - 3.0 * dzz / (4.0 * math.pi)
    assert np.linalg.norm(phi - exact) / np.linalg.norm(exact) < 1e-13
    # Isotropic density: the dipolar interaction energy vanishes.
    vol = np.prod([2 * l / n for n, l in zip(N, L)])
    assert abs(vol * np.sum(phi * rho)) < 1e-13


def test_ddi3_anisotropic_energy_by_radial_quadrature():
    # For rho = Gaussian with widths (a, a, b): int Phi rho = (2pi)^-3 int Khat |rho_hat|^2,
    # Khat = -1 + 3 cos^2(theta_k); reduced to a 1D integral over cos(theta_k).
    a, b = 1.0, 0.7
    N, L = (48, 48, 48), (6.0, 6.0, 6.0)
    X, _ = _radius(N, L)
    rho = np.exp(-(X[0] ** 2 + X[1] ** 2) / a ** 2 - X[2] ** 2 / b ** 2) / (math.pi ** 1.5 * a * a * b)
    phi = gausum.potential(rho, N, L, "ddi3")
    vol = np.prod([2 * l / n for n, l in zip(N, L)])
    got = vol * np.sum(phi * rho)

    # |rho_hat|^2 = exp(-(k_perp^2 a^2 + k_z^2 b^2)/2); integrate k radially in closed form.
    def integrand(u):  # u = cos(theta_k)
        s2 = (1 - u * u) * a * a + u * u * b * b
        radial = 0.5 * math.gamma(1.5) * (2.0 / s2) ** 1.5  # int_0^inf k^2 exp(-k^2 s2/2) dk
        return (-1.0 + 3.0 * u * u) * radial
    val, _ = integrate.quad(integrand, -1.0, 1.0, epsabs=1e-15, epsrel=1e-14)
    exact = 2.0 * math.pi * val / (2.0 * math.pi) ** 3
    assert abs(got - exact) < 1e-12 * max(1.0, abs(exact))


def _ddi2_exact(X, axis):
    # Phi = -(3/2)[d_{n_perp n_perp} - n3^2 Lap_perp] f with f = c sqrt(pi) e^{-a} I0(a),
    # a = r^2/2, c = 1/(2 pi) (the 2D Coulomb potential of rho = exp(-r^2)/pi).
    # With g(a) = e^{-a} I0(a): d_ij f = c sqrt(pi) [g'(a) delta_ij + g''(a) x_i x_j].
    x, y = X
    a = (x * x + y * y) / 2.0
    i0, i1 = special.i0e(a), special.i1e(a)
    i1_over_a = np.where(a > 0, i1 / np.where(a > 0, a, 1.0), 0.5)
    g1 = i1 - i0
    g2 = 2.0 * i0 - 2.0 * i1 - i1_over_a
    pre = math.sqrt(math.pi) / (2.0 * math.pi)
    dxx, dyy, dxy = pre * (g1 + g2 * x * x), pre * (g1 + g2 * y * y), pre * g2 * x * y
    n1, n2, n3 = axis
    return -1.5 * (n1 * n1 * dxx + 2.0 * n1 * n2 * dxy + n2 * n2 * dyy - n3 * n3 * (dxx + dyy))


@pytest.mark.parametrize("axis", [(0.0, 0.0, 1.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.6, 0.0, 0.8),
                                  (0.36, 0.48, 0.8)])
def test_ddi2_gaussian_closed_form(axis):
    # 2D dipole (eq. Kernel): Phi = -(3/2)(d_{n_perp n_perp} - n3^2 Lap_perp)(1/(2 pi |x|)) * rho,
    # rho = exp(-r^2)/pi, against the second derivatives of the Bessel form.
    # A non-square box separates the two in-plane axes.
    N, L = (64, 56), (8.0, 7.0)
    X, r = _radius(N, L)
    rho = np.exp(-r ** 2) / math.pi
    phi = gausum.potential(rho, N, L, "ddi2", axis=axis)
    exact = _ddi2_exact(X, axis)
    assert np.linalg.norm(phi - exact) / np.linalg.norm(exact) < 1e-12
    # Interaction energy (2 pi)^-2 int m(k) |rho_hat|^2 dk with rho_hat = exp(-k^2/4):
    # m = (3/2)|k|[(n_perp.k_hat)^2 - n3^2]; angular mean of (n_perp.k_hat)^2 is |n_perp|^2/2.
    vol = np.prod([2 * l / n for n, l in zip(N, L)])
    nperp2 = axis[0] ** 2 + axis[1] ** 2
    exact_e = 1.5 * (nperp2 / 2.0 - axis[2] ** 2) * math.sqrt(math.pi / 2.0) / (2.0 * math.pi)
    assert abs(vol * np.sum(phi * rho) - exact_e) < 1e-12


def test_ddi2_energy_of_anisotropic_gaussian_by_angular_quadrature():
    # rho with widths (a, b): int Phi rho = (2 pi)^-2 int m(k) |rho_hat|^2 dk,
    # |rho_hat|^2 = exp(-(k1^2 a^2 + k2^2 b^2)/2); the radial integral in closed form.
    a, b = 1.0, 0.6
    axis = (1.0, 0.0, 0.0)
    N, L = (64, 64), (8.0, 8.0)
    X, _ = _radius(N, L)
    rho = np.exp(-X[0] ** 2 / a ** 2 - X[1] ** 2 / b ** 2) / (math.pi * a * b)
    phi = gausum.potential(rho, N, L, "ddi2", axis=axis)
    vol = np.prod([2 * l / n for n, l in zip(N, L)])
    got = vol * np.sum(phi * rho)

    def integrand(th):
        c, s = math.cos(th), math.sin(th)
        s2 = c * c * a * a + s * s * b * b
        radial = math.sqrt(math.pi / 2.0) / s2 ** 1.5  # int_0^inf k^2 exp(-k^2 s2/2) dk
        return 1.5 * (c * c) * radial
    val, _ = integrate.quad(integrand, 0.0, 2.0 * math.pi, epsabs=1e-15, epsrel=1e-14)
    exact = val / (2.0 * math.pi) ** 2
    assert abs(got - exact) < 1e-12 * max(1.0, abs(exact))


def test_fft_machinery_equals_brute_force_linear_convolution():
    # Phi_i = sum_j k[(i - j) mod M] rho_j with k the discrete kernel: checks
    # padding position, crop and the normalisation of the transforms.
    rng = np.random.default_rng(3)
    for N, L in [((8, 6), (2.0, 1.5)), ((6, 4, 4), (1.5, 1.0, 1.0))]:
        K = gausum.coulomb_symbol(N, L, mu=1.0, c=1.0)
        k = gausum.real_space_kernel(K)
        rho = rng.random(N)
        phi = gausum.convolve(rho, K)
        M = K.shape
        ref = np.zeros(N)
        for i in np.ndindex(*N):
            acc = 0.0
            for j in np.ndindex(*N):
                acc += k[tuple((a - b) % m for a, b, m in zip(i, j, M))] * rho[j]
            ref[i] = acc
        assert np.max(np.abs(phi - ref)) < 1e-13 * np.max(np.abs(ref))


def test_symbol_equals_truncated_kernel_fourier_integral():
    # Khat(kappa) = int_{[-2L,2L]^2} c/|y| exp(-i kappa.y) dy, evaluated by
    # direct 2D quadrature in polar pieces (independent of the Gaussian sum
    # and of the near-field constants).
    N, L = (16, 16), (2.0, 2.0)
    c = 1.0
    K = gausum.coulomb_symbol(N, L, mu=1.0, c=c)
    kap = gausum.padded_frequencies(N, L)
    D = 2.0 * L[0]

    def fourier_integral(k0, k1):
        # integrate over the square [-D, D]^2 in polar coordinates: the 1/r
        # singularity cancels against the Jacobian r.
        def inner(theta):
            ct, st = math.cos(theta), math.sin(theta)
            rmax = D / max(abs(ct), abs(st))
            f = lambda r: math.cos(r * (k0 * ct + k1 * st))
            v, _ = integrate.quad(f, 0.0, rmax, epsabs=1e-13, epsrel=1e-13, limit=200)
            return v
        tot = 0.0
        for q in range(8):  # split at the square's corners and axes
            a, b = q * math.pi / 4, (q + 1) * math.pi / 4
            v, _ = integrate.quad(inner, a, b, epsabs=1e-12, epsrel=1e-12, limit=200)
            tot += v
        return c * tot

    for (i, j) in [(0, 0), (1, 0), (3, 2), (5, 7), (16, 3)]:
        ref = fourier_integral(kap[0][i], kap[1][j])
        assert abs(K[i, j] - ref) < 1e-9 * max(1.0, abs(ref)), (i, j, K[i, j], ref)


def test_G_faddeeva_and_legendre_agree():
    w, tau = gausum.sinc_gaussian_sum(1.0, 1.0, 3, 8.0, 8e-4)
    kap = gausum.padded_frequencies((64,), (8.0,))[0]
    D = 16.0
    sel = (tau * D > 0.5) & (tau * D < 40.0)
    a = gausum.G_table(tau[sel], kap, D, method="faddeeva")
    b = np.array([gausum._G_legendre(t, kap, D) for t in tau[sel]])
    scale = np.max(np.abs(b), axis=1, keepdims=True)
    assert np.max(np.abs(a - b) / scale) < 1e-14


def test_G_limits():
    # tau -> 0: G -> 2 sin(kappa D)/kappa (= 2D at kappa=0, 0 on the DFT grid);
    # large tau: G -> sqrt(pi)/tau exp(-kappa^2/(4 tau^2)).
    D = 4.0
    kap = np.array([0.0, math.pi / D, 5 * math.pi / D])
    g0 = gausum.G_table(np.array([1e-9]), kap, D)[0]
    assert abs(g0[0] - 2 * D) < 1e-12
    assert np.max(np.abs(g0[1:])) < 1e-12
    tau = 7.0
    g1 = gausum.G_table(np.array([tau]), kap, D)[0]
    assert np.allclose(g1, math.sqrt(math.pi) / tau * np.exp(-kap ** 2 / (4 * tau * tau)), rtol=1e-14, atol=0)


@pytest.mark.parametrize("mu,d", [(1.0, 2), (1.0, 3), (0.5, 2), (1.7, 3)])
def test_gaussian_sum_relative_accuracy(mu, d):
    L = 12.0
    delta = gausum.default_delta((L,))
    w, tau = gausum.sinc_gaussian_sum(mu, 1.0, d, L, delta)
    r = np.geomspace(delta, 2.0 * math.sqrt(d) * L, 3000)
    err = np.max(np.abs(gausum.gaussian_sum_eval(r, w, tau) * r ** mu - 1.0))
    assert err < 1e-14


def test_near_field_constants_against_direct_radial_quadrature():
    d, mu, c = 2, 1.0, 1.0 / (2 * math.pi)
    delta = 8e-4
    w, tau = gausum.sinc_gaussian_sum(mu, c, d, 8.0, delta)
    C0, C2 = gausum.near_field_constants(mu, c, d, delta, w, tau)
    Sd = 2 * math.pi
    diff = lambda r: c / r ** mu - np.sum(w * np.exp(-(tau * r) ** 2))
    i0, _ = integrate.quad(lambda r: diff(r) * r ** (d - 1), 0.0, delta, epsabs=1e-20, epsrel=1e-11, limit=400)
    i2, _ = integrate.quad(lambda r: diff(r) * r ** (d + 1), 0.0, delta, epsabs=1e-30, epsrel=1e-11, limit=400)
    assert abs(C0 - Sd * i0) < 1e-9 * abs(C0)
    assert abs(C2 - Sd * i2 / (2 * d)) < 1e-8 * abs(C2)
    assert C0 > 1e-6  # the zeroth-order term is far above round-off: it cannot be dropped


@pytest.mark.parametrize("t,tau", [(0.3, 0.05), (1.7, -0.08), (0.0, 0.0), (2.0, 1.3)])
def test_dipole_time_average_by_quadrature(t, tau):
    # M = (1/tau) int m m^T ds with m(s) = A(s)^{-1} n, against Gauss-Legendre in s
    n = np.array([0.48, -0.36, 0.8])
    Om = 0.7
    M = gausum.dipole_average(n, Om, t, tau)

    def m(s):
        c, si = math.cos(Om * s), math.sin(Om * s)
        A = np.array([[c, si, 0.0], [-si, c, 0.0], [0.0, 0.0, 1.0]])
        return np.linalg.solve(A, n)
    if tau == 0.0:
        ref = np.outer(m(t), m(t))
    else:
        x, w = np.polynomial.legendre.leggauss(40)
        ss = t + 0.5 * tau * (x + 1.0)
        ref = sum(wi * np.outer(m(si), m(si)) for wi, si in zip(w, ss)) * 0.5
    assert np.max(np.abs(M - ref)) < 1e-14
    assert abs(np.trace(M) - 1.0) < 1e-14


def test_tilted_dipole_symbol_is_even_and_matches_its_axis_products():
    # a tilted axis: multiplier even under kappa -> -kappa on the padded grid
    # (odd products vanish at Nyquist indices) and, away from them, equal to
    # -1 + 3 (n.kappa)^2 Khat_C
    N, L = (16, 12, 10), (4.0, 3.0, 3.0)
    n = np.array([0.48, -0.36, 0.8])
    K = gausum.ddi3_symbol(N, L, axis=tuple(n))
    neg = K[np.ix_(*[(-np.arange(2 * m)) % (2 * m) for m in N])]
    assert np.max(np.abs(K - neg)) == 0.0
    KC = gausum.coulomb_symbol(N, L, mu=1.0, c=1.0 / (4.0 * math.pi))
    kap = gausum.padded_frequencies(N, L)
    nk = n[0] * kap[0][:, None, None] + n[1] * kap[1][None, :, None] + n[2] * kap[2][None, None, :]
    full = -1.0 + 3.0 * nk ** 2 * KC
    inner = np.ix_(*[np.r_[0:m, m + 1:2 * m] for m in N])
    assert np.max(np.abs(K[inner] - full[inner])) < 1e-13 * np.max(np.abs(full))
