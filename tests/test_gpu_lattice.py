"""GPU parity of the optical lattice trap (fse_set_lattice): its time integral
by quadrature in the rotating frame, its value in the energy, H psi and the
ground state, and the adjoint, against the oracle."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as adj
from oracle import diagnostics as dg
from oracle import groundstate as ogs
from oracle import scheme

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1512_03210_amd import fse  # noqa: E402


def _note(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fse.lib()


CASES = {
    # rotating 2D Coulomb with the paper's lattice form, amplitude 10, k = pi
    "rot2d": (W.Params(d=2, N=(64, 48), L=(6.0, 5.0), s=0.8, Omega=0.5, gamma=(1.0, 1.0), beta=20.0, lam=2.0,
                       kernel="coulomb", coef=1.0 / (2.0 * math.pi), dt=2e-3, name="lat-rot2d"),
              ((10.0, 10.0), (math.pi, math.pi))),
    # rotating 3D dipole along z, anisotropic lattice with a z part
    "rot3d": (W.Params(d=3, N=(24, 32, 16), L=(5.0, 6.0, 4.0), s=0.9, Omega=0.7, gamma=(1.0, 1.2, 1.5), beta=30.0,
                       lam=10.0, kernel="ddi3", dt=2e-3, name="lat-rot3d"),
              ((3.0, 5.0, 2.0), (1.1, 0.7, 1.6))),
    # no rotation: the integral is exact
    "still2d": (W.Params(d=2, N=(48, 48), L=(5.0, 5.0), s=1.2, Omega=0.0, gamma=(1.0, 1.0), beta=40.0, lam=0.0,
                         kernel="none", dt=2e-3, name="lat-still2d"),
                ((4.0, 6.0), (1.5, 2.0))),
}
_PR = {}


def _prob(name):
    if name not in _PR:
        p, (v, k) = CASES[name]
        pr = scheme.Problem.from_params(p)
        pr.lattice = (tuple(v) + (0.0,) * (3 - len(v)), tuple(k) + (0.0,) * (3 - len(k)))
        _PR[name] = pr
    return _PR[name]


def _plan(name, prec):
    p, (v, k) = CASES[name]
    plan = fse.Plan.from_params(p, prec)
    plan.set_lattice(v, k)
    return plan


def _psi0(p, seed=0):
    if p.d == 2:
        return W.harmonic_vortex_2d(p.N, p.L, seed=seed)
    return W.anisotropic_gaussian(p.N, p.L, p.gamma, seed=seed)


def _dev(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex128 if prec == fse.C128 else np.complex64))).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-11), (fse.C64, 2e-5)])
def test_steps_against_oracle(name, prec, tol):
    p = CASES[name][0]
    pr = _prob(name)
    psi0 = _psi0(p)
    plan = _plan(name, prec)
    for n, order in ((1, 2), (10, 2), (3, 4)):
        ref, _ = (pr.run if order == 2 else pr.run4)(psi0, n, p.dt)
        plan.time = 0.0
        x = _dev(psi0, prec)
        plan.step(x, n, p.dt, order=order)
        err = _rel(x.cpu().numpy().astype(np.complex128), ref)
        _note(f"[lattice] {name} prec={prec} steps={n} order={order}: {err:.3e}")
        assert err < tol


@pytest.mark.parametrize("name", list(CASES))
def test_energy_H_and_ground_state(name):
    p = CASES[name][0]
    pr = _prob(name)
    psi = _psi0(p, seed=1)
    plan = _plan(name, fse.C128)
    plan.time = 1.3  # the lattice has turned by Omega t in the rotating coordinates
    x = _dev(psi, fse.C128)
    e = plan.energy(x).cpu().numpy()
    eo = np.array(dg.energy_parts(pr, psi, t=1.3))
    assert np.all(np.abs(e - eo) <= 1e-11 * np.maximum(1.0, np.abs(eo)))
    H = plan.apply_H(x).cpu().numpy()
    assert _rel(H, dg.apply_H(pr, psi)) < 1e-12
    g = ogs.GroundState(pr, 0.05)
    ref, _ = g.step(psi, rtol=1e-12)
    plan.gs_step(x, 0.05, tol=1e-12)
    err = _rel(x.cpu().numpy(), ref)
    _note(f"[lattice] {name}: energy max diff {np.max(np.abs(e - eo)):.2e}, ground-state step {err:.3e}")
    assert err < 1e-10


def test_adjoint_with_a_turning_lattice_and_grid_potential():
    name = "rot2d"
    p = CASES[name][0]
    pr = _prob(name)
    X = np.meshgrid(*scheme.axes(p.N, p.L), indexing="ij")
    U = 0.2 * np.cos(X[0]) * np.sin(0.7 * X[1])
    pr.U = U
    try:
        psi0 = _psi0(p, seed=2)
        tgt = W.adjoint_target(p.N, p.L, seed=3)
        n = 5
        psiT, _ = pr.run(psi0, n, p.dt)
        _, gT = adj.loss_and_grad(psiT, tgt, p.N, p.L)
        g_ref, gU_ref = adj.run_adjoint(pr, psi0, n, p.dt, gT)
    finally:
        pr.U = None
    plan = _plan(name, fse.C128)
    plan.set_potential(torch.from_numpy(U).cuda())
    g = _dev(gT, fse.C128)
    gU = torch.zeros(p.N, dtype=torch.float64, device="cuda:0")
    plan.step_adjoint(_dev(psi0, fse.C128), n, p.dt, g, gU)
    e1, e2 = _rel(g.cpu().numpy(), g_ref), _rel(gU.cpu().numpy(), gU_ref)
    _note(f"[lattice] adjoint: {e1:.3e} {e2:.3e}")
    assert e1 < 1e-11 and e2 < 1e-11


def test_rotating_lattice_energy_is_conserved_on_the_gpu():
    # the oracle pin's case: drift of the rotating-frame energy second order in dt
    p = W.Params(d=2, N=(48, 48), L=(6.0, 6.0), s=0.9, Omega=0.5, gamma=(1.0, 1.0), beta=10.0, lam=0.0,
                 kernel="none", dt=0.01, name="lat-energy")
    X = np.meshgrid(*scheme.axes(p.N, p.L), indexing="ij")
    psi0 = W.normalize(np.exp(-(X[0] - 0.5) ** 2 / 1.2 - X[1] ** 2 / 0.8) * (1 + 0.3j * X[1]) + 0j, p.h)
    drift = []
    for n in (50, 100):
        plan = fse.Plan.from_params(p, fse.C128)
        plan.set_lattice((2.0, 2.0), (0.5 * math.pi, 0.5 * math.pi))
        x = _dev(psi0, fse.C128)
        E0 = plan.energy(x).cpu().numpy()[5]
        plan.step(x, n, 1.0 / n)
        drift.append(plan.energy(x).cpu().numpy()[5] - E0)
    _note(f"[lattice] energy drift over t = 1: {drift}")
    assert abs(drift[1]) < 1e-3 and 3.5 < drift[0] / drift[1] < 4.5
    plan.set_lattice(None)  # removed: back to the harmonic trap
