"""Seeded synthetic inputs and named parameter sets.

This module is shared by the tests, the benchmark and the oracle checks.  It
holds no step of the numerical method: it only lays out uniform grids, draws
seeded random numbers and builds initial wave functions of the shapes the
paper's experiments use (harmonic-oscillator ground states, a unit vortex,
Gaussians), normalised to unit discrete mass.

Grid convention (periodic box, N points per axis, no duplicated endpoint):
    x_l = -L + l*h,  l = 0..N-1,  h = 2L/N
which is the paper's uniform grid of the time-splitting scheme (Section 4.2)
with the periodic endpoint dropped.
"""
from __future__ import annotations

import dataclasses
import math
import os
import re
from typing import Sequence

import numpy as np

__all__ = [
    "Params",
    "grid_axes",
    "mesh",
    "normalize",
    "harmonic_vortex_2d",
    "anisotropic_gaussian",
    "ground_state_guess",
    "vortex_lattice_2d",
    "PRESETS",
    "preset",
    "batch_sweep",
    "stored_long_run",
]


@dataclasses.dataclass(frozen=True)
class Params:
    """Physical and numerical parameters of one problem instance.

    d: dimension (2 or 3); N: points per axis; L: half-widths of the box
    [-L_j, L_j]; s: fractional order; Omega: rotation speed; gamma: trap
    frequencies of V = sum_v gamma_v^2 v^2 / 2; beta, lam: local and nonlocal
    interaction strengths; kernel: "none", "coulomb", "ddi3" or "ddi2";
    axis: unit dipole axis n (a 2D dipole keeps its third component as the
    out-of-plane part n3); mu: Coulomb exponent; coef: prefactor c of U = c/|x|^mu (the paper's
    Coulomb-type kernel uses c = 1/(2^{d-1} pi)); m: mass term of the
    fractional operator; dt: time step; steps: number of steps of the run.
    """

    d: int
    N: tuple
    L: tuple
    s: float
    Omega: float
    gamma: tuple
    beta: float
    lam: float
    kernel: str = "coulomb"
    axis: tuple = (0.0, 0.0, 1.0)
    mu: float = 1.0
    coef: float | None = None
    m: float = 0.0
    dt: float = 1e-3
    steps: int = 1
    name: str = ""

    @property
    def c(self) -> float:
        if self.coef is not None:
            return float(self.coef)
        if self.kernel == "ddi3":
            return 1.0 / (4.0 * math.pi)
        return 1.0 / (2 ** (self.d - 1) * math.pi)

    @property
    def h(self) -> tuple:
        return tuple(2.0 * L / N for L, N in zip(self.L, self.N))

    @property
    def npts(self) -> int:
        return int(np.prod(self.N))

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


def grid_axes(N: Sequence[int], L: Sequence[float]):
    """1D coordinate arrays x_l = -L + l*h, h = 2L/N (float64)."""
    return [(-float(Lj) + np.arange(int(Nj), dtype=np.float64) * (2.0 * float(Lj) / int(Nj)))
            for Nj, Lj in zip(N, L)]


def mesh(N, L):
    return np.meshgrid(*grid_axes(N, L), indexing="ij")


def normalize(psi: np.ndarray, h: Sequence[float]) -> np.ndarray:
    """Scale psi so that prod(h) * sum |psi|^2 = 1."""
    vol = float(np.prod(h))
    nrm = math.sqrt(vol * float(np.sum(np.abs(psi) ** 2)))
    return psi / nrm


def _noise(shape, seed, amp):
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return amp * (re + 1j * im)


def harmonic_vortex_2d(N, L, seed=0, noise=1e-3):
    """Unit vortex (x+iy) exp(-|x|^2/2)/sqrt(pi) plus seeded complex noise.

    The vortex profile is the paper's initial-guess component for rotating
    ground states (Section 3.3, the initial guess); the noise breaks its
    symmetry so that every Fourier mode is populated.
    """
    X, Y = mesh(N, L)
    psi = (X + 1j * Y) * np.exp(-(X ** 2 + Y ** 2) / 2.0) / math.sqrt(math.pi)
    psi = psi + _noise(psi.shape, seed, noise)
    return normalize(psi, [2.0 * Lj / Nj for Nj, Lj in zip(N, L)])


def anisotropic_gaussian(N, L, gamma, seed=0, noise=1e-3):
    """exp(-sum_v gamma_v v^2 / 2) * (1 + noise*(xi1 + i xi2)), normalised."""
    grids = mesh(N, L)
    arg = np.zeros(grids[0].shape)
    for g, X in zip(gamma, grids):
        arg += g * X ** 2
    psi = np.exp(-arg / 2.0).astype(np.complex128)
    psi = psi * (1.0 + _noise(psi.shape, seed, noise))
    return normalize(psi, [2.0 * Lj / Nj for Nj, Lj in zip(N, L)])


def ground_state_guess(N, L, Omega, gamma=None, seed=0, noise=1e-3):
    """((1-Omega) phi_ho + Omega phi_ho^v), normalised (Section 3.3 initial guess).

    In 3D the planar profile is multiplied by (g_z/pi)^{1/4} exp(-g_z z^2/2).
    """
    grids = mesh(N, L)
    X, Y = grids[0], grids[1]
    r2 = X ** 2 + Y ** 2
    ho = np.exp(-r2 / 2.0) / math.sqrt(math.pi)
    hov = (X + 1j * Y) * ho
    psi = (1.0 - Omega) * ho + Omega * hov
    if len(N) == 3:
        gz = 1.0 if gamma is None else gamma[2]
        psi = psi * (gz / math.pi) ** 0.25 * np.exp(-gz * grids[2] ** 2 / 2.0)
    psi = psi + _noise(psi.shape, seed, noise)
    return normalize(psi, [2.0 * Lj / Nj for Nj, Lj in zip(N, L)])


def vortex_lattice_2d(N, L, seed=0, nv=7, radius=1.5, jitter=0.05, width2=2.0):
    """Gaussian envelope exp(-|x|^2/width2) times a product of nv unit vortices.

    width2 = 2 keeps the degree-nv profile inside the [-8, 8]^2 box of the
    2D cases (boundary density below 1e-15 of the peak).

    Vortex centres: the origin plus a hexagon of the given radius, each
    jittered by a seeded normal displacement.  Used for the batched sweep.
    """
    rng = np.random.default_rng(seed)
    X, Y = mesh(N, L)
    centres = [(0.0, 0.0)] + [(radius * math.cos(k * math.pi / 3), radius * math.sin(k * math.pi / 3))
                              for k in range(max(nv - 1, 0))]
    psi = np.exp(-(X ** 2 + Y ** 2) / width2).astype(np.complex128)
    for (cx, cy) in centres[:nv]:
        jx, jy = rng.normal(0.0, jitter, 2)
        psi = psi * ((X - cx - jx) + 1j * (Y - cy - jy))
    return normalize(psi, [2.0 * Lj / Nj for Nj, Lj in zip(N, L)])


# ---------------------------------------------------------------------------
# Named parameter sets.
#   plain2d:      2D plain method, 64^2 on [-8,8]^2, Coulomb GauSum on 128^2 padding.
#   dipole3d_128: 3D 128^3 on [-12,12]^3, z-dipole GauSum on 256^3 padding.
#   dipole3d_256: the same physics on a 256^3 grid (512^3 padding): the
#         headline 3D 256^3 split step.
#   coulomb3d_96: 3D 96^3 Coulomb (used here only as a parity case).
#   adjoint3d_96: the differentiation case: the same physics with the trap
#         given as a grid potential V(x) = |x|^2/2 (gamma = 0 in the plan), the
#         parameter whose gradient is taken.
# ---------------------------------------------------------------------------
PRESETS = {
    "plain2d": Params(d=2, N=(64, 64), L=(8.0, 8.0), s=0.75, Omega=0.5, gamma=(1.0, 1.0),
                   beta=100.0, lam=1.0, kernel="coulomb", mu=1.0, dt=1e-3, steps=100,
                   name="plain2d-64"),
    "dipole3d_128": Params(d=3, N=(128, 128, 128), L=(12.0, 12.0, 12.0), s=0.8, Omega=0.7,
                   gamma=(1.0, 1.0, 2.0), beta=200.0, lam=50.0, kernel="ddi3", mu=1.0,
                   dt=5e-4, steps=1000, name="dipole3d-128"),
    "dipole3d_256": Params(d=3, N=(256, 256, 256), L=(12.0, 12.0, 12.0), s=0.8, Omega=0.7,
                 gamma=(1.0, 1.0, 2.0), beta=200.0, lam=50.0, kernel="ddi3", mu=1.0,
                 dt=5e-4, steps=100, name="dipole3d-256"),
    "coulomb3d_96": Params(d=3, N=(96, 96, 96), L=(12.0, 12.0, 12.0), s=0.6, Omega=0.4,
                   gamma=(1.0, 1.0, 1.0), beta=100.0, lam=1.0, kernel="coulomb", mu=1.0,
                   dt=1e-3, steps=200, name="coulomb3d-96"),
    "adjoint3d_96": Params(d=3, N=(96, 96, 96), L=(12.0, 12.0, 12.0), s=0.6, Omega=0.4,
                   gamma=(0.0, 0.0, 0.0), beta=100.0, lam=1.0, kernel="coulomb", mu=1.0,
                   dt=1e-3, steps=200, name="adjoint3d-96"),
    # ground-state solve at scale: trap and time step not stated; gamma = 1 and
    # the paper's ground-state time step dt = 1e-3 are taken
    "gs3d_256": Params(d=3, N=(256, 256, 256), L=(16.0, 16.0, 16.0), s=0.9, Omega=0.8,
                   gamma=(1.0, 1.0, 1.0), beta=1000.0, lam=-50.0, kernel="ddi3", mu=1.0,
                   dt=1e-3, steps=2, name="groundstate3d-256"),
}


def preset(name: str, **kw) -> Params:
    p = PRESETS[name]
    return p.replace(**kw) if kw else p


def initial_state(p: Params, seed: int = 0) -> np.ndarray:
    """The seeded initial state used for a parameter set (complex128)."""
    if p.d == 2 and p.name.startswith("plain2d"):
        return harmonic_vortex_2d(p.N, p.L, seed=seed)
    if p.d == 2:
        return vortex_lattice_2d(p.N, p.L, seed=seed)
    return anisotropic_gaussian(p.N, p.L, p.gamma, seed=seed)


def harmonic_potential(N, L, gamma) -> np.ndarray:
    """V(x) = sum_v gamma_v^2 v^2 / 2 sampled on the grid (float64)."""
    V = np.zeros(tuple(int(n) for n in N))
    for g, X in zip(gamma, mesh(N, L)):
        V = V + 0.5 * g * g * X ** 2
    return V


def adjoint_case_inputs(p: Params):
    """psi0, V(x) = |x|^2/2 and the target state of the differentiation case (complex128 / float64):
    the Gaussian initial state of the 96^3 cases (seed 0), the isotropic harmonic trap as a grid array, and
    the displaced target (seed 1)."""
    return (anisotropic_gaussian(p.N, p.L, (1.0,) * p.d, seed=0), harmonic_potential(p.N, p.L, (1.0,) * p.d),
            adjoint_target(p.N, p.L, seed=1))


def adjoint_target(N, L, seed=1):
    """Target state of the differentiation case: a Gaussian displaced by half a
    unit along x with a phase ramp along y, plus seeded noise, normalised."""
    grids = mesh(N, L)
    arg = (grids[0] - 0.5) ** 2
    for X in grids[1:]:
        arg = arg + X ** 2
    psi = np.exp(-arg / 2.0 + 0.3j * grids[1]) * (1.0 + _noise(grids[0].shape, seed, 1e-3))
    return normalize(psi, [2.0 * Lj / Nj for Nj, Lj in zip(N, L)])


def batch_sweep(count=64, sizes=(128, 256, 384, 512), seed=0, beta=500.0, lam=1.0,
                L=8.0, dt=1e-3, steps=500):
    """The batched sweep: count 2D instances on uneven grids in equal shares.

    s_i ~ U[0.3, 1.0] and Omega_i ~ U[0, 0.9] from one seeded generator; box,
    time step, trap and nonlocal strength as in the 2D plain-method case.
    """
    rng = np.random.default_rng(seed)
    s_vals = rng.uniform(0.3, 1.0, count)
    om_vals = rng.uniform(0.0, 0.9, count)
    out = []
    for i in range(count):
        n = sizes[i * len(sizes) // count]
        out.append(Params(d=2, N=(n, n), L=(L, L), s=float(s_vals[i]), Omega=float(om_vals[i]),
                          gamma=(1.0, 1.0), beta=beta, lam=lam, kernel="coulomb", mu=1.0,
                          dt=dt, steps=steps, name=f"batch-{i}-{n}"))
    return out


# ---------------------------------------------------------------------------
# Stored oracle values of the full-length runs (tests/golden/*_long.txt,
# written by tests/golden/make_long_runs.py, which calls only the oracle).
# ---------------------------------------------------------------------------
GOLDEN_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden")


def stored_long_run(name: str):
    """Parse tests/golden/<name>_long.txt.

    Returns (scalars, samples): scalars[key] = (mass, energy, lz) and
    samples[key] = (index tuple of arrays, complex128 values), where key is the
    step (single runs) or the instance number (the batched sweep, whose scalars
    are keyed (k, step)).
    """
    path = os.path.join(GOLDEN_DIR, f"{name}_long.txt")
    scalars, rows = {}, []
    with open(path) as f:
        for line in f:
            if line.startswith("# scalars"):
                kv = dict(re.findall(r"(\w+)=(\S+)", line))
                key = (int(kv["k"]), int(kv["step"])) if "k" in kv else int(kv["step"])
                scalars[key] = (float(kv["mass"]), float(kv["energy"]), float(kv["lz"]))
            elif line.strip() and not line.startswith("#"):
                rows.append(line.split())
    data = np.array(rows, dtype=float)
    samples = {}
    for key in np.unique(data[:, 0]).astype(int):
        r = data[data[:, 0] == key]
        idx = tuple(r[:, j].astype(int) for j in range(1, r.shape[1] - 2))
        samples[int(key)] = (idx, r[:, -2] + 1j * r[:, -1])
    return scalars, samples
