"""GauSum nonlocal potential, float64 (oracle; test infrastructure only).

Follows Section 2 of the paper (the review of the Gaussian-sum method) with
the readings below, which the paper leaves open:

* Kernel normalisation: U(x) = c/|x|^mu with an explicit prefactor c (the
  paper's Coulomb-type kernel, eq. Kernel, has c = 1/(2^{d-1} pi)).
* Gaussian sum (eq. GS-Gene): trapezoidal (sinc) quadrature of
      r^{-mu} = (2/Gamma(mu/2)) * int_R exp(-r^2 e^{2t} + mu t) dt,
  nodes t_q = t_lo + q*ht, tau_q = e^{t_q}, w_q = c*2*ht*e^{mu t_q}/Gamma(mu/2),
  ht = 0.14, t_lo = ln(1e-17)/mu - ln(2 sqrt(d) L) - 1, t_hi = ln(9/delta).
  Accuracy is asked on [delta, 2 sqrt(d) L] (the diagonal of the
  integration box B2 = [-2L, 2L]^d, which the paper's [delta, 2] misses).
* delta = 1e-4 * L (the low end of the paper's range, scaled to the box).
* Padding factor 2: the density on [-L, L)^d is zero-padded to a period-4L
  box with 2N points per axis and the kernel is truncated to [-2L, 2L]^d;
  for x in the box this truncated circular convolution equals the linear one.
* Near field (eq. taylor): the zeroth-order Taylor term is kept together with
  the Laplacian term, giving the Fourier multiplier C0 - C2 |kappa|^2.
* 3D dipole along n: Phi = -rho - 3 (1/(4 pi |x|)) * d_nn rho, i.e. the
  multiplier -1 + 3 (n.kappa)^2 Khat_C with Khat_C the symbol of the
  truncated 1/(4 pi |x|) kernel.  This is the kernel's own symbol in eq.
  Kernel; the displayed reformulation at the end of Section 2 carries a sign
  and factor slip.
* Dipole axes with off-diagonal products n_i n_j (a tilted axis, or any
  axis that turns in the rotating frame): the multiplier is c0 + Khat_C
  kappa^T M kappa with a symmetric M; its odd terms kappa_i kappa_j (i != j)
  are taken as zero at Nyquist indices, where kappa and -kappa share an
  index, so that the multiplier stays even under kappa -> -kappa on the grid
  and the potential of a real density is real.
* An axis that turns in the rotating Lagrangian coordinates, m(t) = A^{-1}(t) n
  (eq. Kernel_Rot), enters a nonlinear sub-step over [t, t+tau] through the
  time average M = (1/tau) int m m^T ds (the sub-step integrates the
  potential over time with the density frozen); in closed form each
  harmonic cos/sin(a + b s) averages to its value at the midpoint times
  sinc(b tau / 2).
* 2D dipole along n = (n_perp, n3): Phi = -(3/2)(d_{n_perp n_perp} - n3^2
  Lap_perp)(1/(2 pi |x|)) * rho (eq. Kernel), i.e. the multiplier
  (3/2)[(n_perp.kappa)^2 - n3^2 |kappa|^2] Khat_C with Khat_C the symbol of
  the truncated 1/(2 pi |x|) kernel; applying the Coulomb kernel to the
  modified density of Section 2 is the same product in Fourier space.

Parity: pinned by closed forms (erf(r)/r Coulomb potential of a 3D
Gaussian, the 2D Bessel form, the 3D and 2D dipolar derivative forms), a brute-force
O(N^{2d}) linear convolution on tiny grids, the Gaussian-sum accuracy check
and two independent evaluations of the 1D integrals G (tests/oracle).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from . import _fft


SURFACE = {2: 2.0 * math.pi, 3: 4.0 * math.pi}  # |S^{d-1}|


def default_delta(L):
    return 1e-4 * float(np.max(L))


def sinc_gaussian_sum(mu, c, d, Lmax, delta, ht=0.14, eps=1e-17):
    """Weights w_q and exponents tau_q of U_GS(r) = sum_q w_q exp(-tau_q^2 r^2).

    Sinc (trapezoidal) quadrature of the integral representation of r^{-mu}
    (eq. GS-Gene; details of the quadrature are the reading stated above).
    """
    t_lo = math.log(eps) / mu - math.log(2.0 * math.sqrt(d) * Lmax) - 1.0
    t_hi = math.log(9.0 / delta)
    Q = int(math.ceil((t_hi - t_lo) / ht))
    t = t_lo + ht * np.arange(Q + 1, dtype=np.float64)
    tau = np.exp(t)
    w = c * 2.0 * ht * np.exp(mu * t) / special.gamma(mu / 2.0)
    return w, tau


def gaussian_sum_eval(r, w, tau):
    """U_GS(r) for an array of radii."""
    r = np.asarray(r, dtype=np.float64)
    return np.sum(w[:, None] * np.exp(-(tau[:, None] ** 2) * r[None, :] ** 2), axis=0)


def _G_faddeeva(tau, kappa, D):
    """2 int_0^D exp(-tau^2 y^2) cos(kappa y) dy via the Faddeeva function.

    Full-line Gaussian transform minus the two tails; each tail is
    (sqrt(pi)/(2 tau)) exp(-tau^2 D^2 + i kappa D) w(kappa/(2 tau) + i tau D).
    Used where tau*D >= 2, so that exp(-tau^2 D^2) is small and nothing cancels.
    """
    z = kappa / (2.0 * tau) + 1j * tau * D
    tail = np.real(np.exp(-(tau * D) ** 2 + 1j * kappa * D) * special.wofz(z))
    return (math.sqrt(math.pi) / tau) * (np.exp(-(kappa / (2.0 * tau)) ** 2) - tail)


def _G_legendre(tau, kappa, D, nodes_per_panel=24):
    """2 int_0^D exp(-tau^2 y^2) cos(kappa y) dy by composite Gauss-Legendre."""
    kappa = np.asarray(kappa, dtype=np.float64)
    periods = float(np.max(np.abs(kappa))) * D / (2.0 * math.pi)
    panels = int(max(8, math.ceil(2.0 * periods) + 4))
    x, wt = np.polynomial.legendre.leggauss(nodes_per_panel)
    edges = np.linspace(0.0, D, panels + 1)
    a, b = edges[:-1], edges[1:]
    y = (0.5 * (b - a)[:, None] * (x[None, :] + 1.0) + a[:, None]).ravel()
    wy = (0.5 * (b - a)[:, None] * wt[None, :]).ravel()
    f = np.exp(-(tau * y) ** 2) * wy
    return 2.0 * np.cos(np.outer(kappa, y)) @ f


def G_table(tau, kappa, D, method="auto"):
    """Table G[q, j] = 2 int_0^D exp(-tau_q^2 y^2) cos(kappa_j y) dy (eq. tensor).

    method="auto": Faddeeva form for tau*D >= 2, Gauss-Legendre below (the
    Faddeeva form would cancel catastrophically for tiny tau).
    """
    tau = np.asarray(tau, dtype=np.float64)
    kappa = np.asarray(kappa, dtype=np.float64)
    out = np.empty((tau.size, kappa.size))
    for q, tq in enumerate(tau):
        use_fad = (method == "faddeeva") or (method == "auto" and tq * D >= 2.0)
        out[q] = _G_faddeeva(tq, kappa, D) if use_fad else _G_legendre(tq, kappa, D)
    return out


def near_field_constants(mu, c, d, delta, w, tau):
    """C0, C2 of the near-field correction I2 = C0*rho + C2*Lap(rho) (eq. taylor).

    C0 = int_{|y|<delta} (U - U_GS) dy,
    C2 = (1/(2d)) int_{|y|<delta} (U - U_GS) |y|^2 dy,
    with the Gaussian ball integrals written through the regularised lower
    incomplete gamma function P(a, x).
    """
    Sd = SURFACE[d]
    a0, a2 = d / 2.0, d / 2.0 + 1.0
    x = (tau * delta) ** 2
    ball_g0 = Sd * special.gamma(a0) * special.gammainc(a0, x) / (2.0 * tau ** d)
    ball_g2 = Sd * special.gamma(a2) * special.gammainc(a2, x) / (2.0 * tau ** (d + 2))
    C0 = c * Sd * delta ** (d - mu) / (d - mu) - np.sum(w * ball_g0)
    C2 = (c * Sd * delta ** (d + 2 - mu) / (d + 2 - mu) - np.sum(w * ball_g2)) / (2.0 * d)
    return float(C0), float(C2)


def padded_frequencies(N, L):
    """kappa_j on the padded grid: M_j = 2 N_j points of spacing h_j = 2L_j/N_j."""
    return [2.0 * math.pi * np.fft.fftfreq(2 * int(Nj), d=2.0 * float(Lj) / int(Nj))
            for Nj, Lj in zip(N, L)]


def coulomb_symbol(N, L, mu=1.0, c=1.0, delta=None, ht=0.14, g_method="auto"):
    """Khat_C on the full padded frequency grid (shape 2N per axis), float64.

    Khat_C(kappa) = sum_q w_q prod_j G(tau_q, kappa_j, 2 L_j) + C0 - C2 |kappa|^2.
    """
    d = len(N)
    Lmax = float(np.max(L))
    delta = default_delta(L) if delta is None else delta
    w, tau = sinc_gaussian_sum(mu, c, d, Lmax, delta, ht=ht)
    kap = padded_frequencies(N, L)
    tables = [G_table(tau, kap[j], 2.0 * float(L[j]), method=g_method) for j in range(d)]
    K = np.zeros(tuple(2 * int(n) for n in N))
    for q in range(tau.size):
        term = tables[0][q]
        for j in range(1, d):
            term = np.multiply.outer(term, tables[j][q])
        K += w[q] * term
    C0, C2 = near_field_constants(mu, c, d, delta, w, tau)
    k2 = np.zeros_like(K)
    for j in range(d):
        shape = [1] * d
        shape[j] = -1
        k2 = k2 + kap[j].reshape(shape) ** 2
    return K + C0 - C2 * k2


def dipole_average(axis, Omega=0.0, t=0.0, tau=0.0):
    """M = (1/tau) int_t^{t+tau} m(s) m(s)^T ds with m(s) = A(s)^{-1} n (eq. Kernel_Rot);
    tau = 0 gives m(t) m(t)^T.  A(s) turns (x, y) by the angle Omega s, so A^{-1} n
    is n_perp turned by +Omega s and n3 unchanged."""
    n1, n2, n3 = (float(a) for a in axis)
    r = math.hypot(n1, n2)
    phi0 = math.atan2(n2, n1) if r > 0.0 else 0.0

    def sinc(x):
        return 1.0 if x == 0.0 else math.sin(x) / x

    def avg_cos(k):  # mean of cos(k (phi0 + Omega s)) over [t, t + tau]
        return math.cos(k * (phi0 + Omega * (t + 0.5 * tau))) * sinc(0.5 * k * Omega * tau)

    def avg_sin(k):
        return math.sin(k * (phi0 + Omega * (t + 0.5 * tau))) * sinc(0.5 * k * Omega * tau)
    M = np.zeros((3, 3))
    M[0, 0] = r * r * (0.5 + 0.5 * avg_cos(2))
    M[1, 1] = r * r * (0.5 - 0.5 * avg_cos(2))
    M[0, 1] = M[1, 0] = r * r * 0.5 * avg_sin(2)
    M[0, 2] = M[2, 0] = n3 * r * avg_cos(1)
    M[1, 2] = M[2, 1] = n3 * r * avg_sin(1)
    M[2, 2] = n3 * n3
    return M


def dipole_form_symbol(N, L, kernel, M, delta=None, ht=0.14, KC=None):
    """Dipolar multiplier for an axis second-moment matrix M (M = n n^T for a fixed axis):
    3D  -1 + 3 Khat_C kappa^T M kappa,                 Khat_C for 1/(4 pi |x|);
    2D  (3/2) Khat_C (kappa^T M_perp kappa - M_33 |kappa|^2),  Khat_C for 1/(2 pi |x|).
    Odd terms (i != j) use kappa = 0 at Nyquist indices."""
    d = len(N)
    if KC is None:
        KC = coulomb_symbol(N, L, mu=1.0, c=1.0 / ((4.0 if d == 3 else 2.0) * math.pi), delta=delta, ht=ht)
    kap = padded_frequencies(N, L)
    kx = []
    for j in range(d):
        k = kap[j].copy()
        k[int(N[j])] = 0.0  # the Nyquist index of the 2N_j-point padded axis
        kx.append(k)

    def b(v, j):
        shape = [1] * d
        shape[j] = -1
        return v.reshape(shape)
    Q = np.zeros(KC.shape)
    for i in range(d):
        Q = Q + M[i, i] * b(kap[i], i) ** 2
        for j in range(i + 1, d):
            Q = Q + 2.0 * M[i, j] * b(kx[i], i) * b(kx[j], j)
    if d == 3:
        return -1.0 + 3.0 * KC * Q
    k2 = sum(b(kap[i], i) ** 2 for i in range(2))
    return 1.5 * KC * (Q - M[2, 2] * k2)


def ddi3_symbol(N, L, delta=None, ht=0.14, axis=(0.0, 0.0, 1.0)):
    """3D dipolar multiplier -1 + 3 (n.kappa)^2 Khat_C, Khat_C for 1/(4 pi |x|)."""
    n = np.asarray(axis, dtype=np.float64)
    return dipole_form_symbol(N, L, "ddi3", np.outer(n, n), delta=delta, ht=ht)


def ddi2_symbol(N, L, delta=None, ht=0.14, axis=(0.0, 0.0, 1.0)):
    """2D dipolar multiplier (3/2)[(n_perp.kappa)^2 - n3^2 |kappa|^2] Khat_C, Khat_C for 1/(2 pi |x|)."""
    n = np.asarray(axis, dtype=np.float64)
    return dipole_form_symbol(N, L, "ddi2", np.outer(n, n), delta=delta, ht=ht)


def symbol(N, L, kernel, mu=1.0, c=1.0, delta=None, axis=(0.0, 0.0, 1.0)):
    if kernel == "coulomb":
        return coulomb_symbol(N, L, mu=mu, c=c, delta=delta)
    if kernel == "ddi3":
        if len(N) != 3:
            raise ValueError("the 3D dipolar kernel needs d = 3")
        return ddi3_symbol(N, L, delta=delta, axis=axis)
    if kernel == "ddi2":
        if len(N) != 2:
            raise ValueError("the 2D dipolar kernel needs d = 2")
        return ddi2_symbol(N, L, delta=delta, axis=axis)
    raise ValueError(kernel)


def convolve(rho, K):
    """Phi = crop_N ifftn_M( K * fftn_M(pad(rho)) ): rho at indices [0, N) of the 2N box."""
    N = rho.shape
    M = K.shape
    pad = np.zeros(M)
    pad[tuple(slice(0, n) for n in N)] = rho
    out = _fft.ifftn(K * _fft.fftn(pad))
    return np.real(out[tuple(slice(0, n) for n in N)])


def potential(rho, N, L, kernel, mu=1.0, c=1.0, delta=None, K=None, axis=(0.0, 0.0, 1.0)):
    """Phi[rho] = (U * rho) on the grid, via the GauSum multiplier."""
    if K is None:
        K = symbol(N, L, kernel, mu=mu, c=c, delta=delta, axis=axis)
    return convolve(rho, K)


def real_space_kernel(K):
    """k = ifftn(K): the discrete kernel whose circular convolution the FFT path applies."""
    return np.real(_fft.ifftn(K))
