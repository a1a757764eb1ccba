"""GPU parity for dipole axes applied as a quadratic form in the padded
convolution: tilted axes (products n_i n_j) and axes that turn in the
rotating Lagrangian coordinates (m(t) = A^{-1}(t) n), against the oracle."""
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
    "tilt3d": W.Params(d=3, N=(24, 32, 16), L=(5.0, 6.0, 4.0), s=0.9, Omega=0.0, gamma=(1.0, 1.2, 1.5), beta=50.0,
                       lam=20.0, kernel="ddi3", axis=(0.48, -0.36, 0.8), dt=2e-3, name="tilt3d"),
    "turn3d": W.Params(d=3, N=(24, 24, 32), L=(5.0, 5.0, 6.0), s=0.8, Omega=0.6, gamma=(1.0, 1.3, 1.1), beta=50.0,
                       lam=20.0, kernel="ddi3", axis=(0.6, 0.0, 0.8), dt=2e-3, name="turn3d"),
    "turn2d": W.Params(d=2, N=(48, 64), L=(6.0, 7.0), s=0.7, Omega=0.6, gamma=(1.0, 1.2), beta=30.0, lam=-6.0,
                       kernel="ddi2", axis=(0.8, 0.0, 0.6), dt=2e-3, name="turn2d"),
    "tilt2d": W.Params(d=2, N=(64, 48), L=(7.0, 6.0), s=1.1, Omega=0.0, gamma=(1.0, 0.9), beta=30.0, lam=8.0,
                       kernel="ddi2", axis=(0.36, 0.48, 0.8), dt=2e-3, name="tilt2d"),
}
_PR = {}


def _prob(name):
    if name not in _PR:
        _PR[name] = scheme.Problem.from_params(CASES[name])
    return _PR[name]


def _psi0(p, seed=0):
    X = np.meshgrid(*scheme.axes(p.N, p.L), indexing="ij")
    if p.d == 2:
        psi = W.harmonic_vortex_2d(p.N, p.L, seed=seed)
    else:
        psi = W.anisotropic_gaussian(p.N, p.L, p.gamma, seed=seed)
    return W.normalize(psi * (1.0 + 0.3 * X[0] + 0.2j * X[1]), p.h)


def _dev(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex128 if prec == fse.C128 else np.complex64))).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-11), (fse.C64, 2e-5)])
def test_steps_against_oracle(name, prec, tol):
    p = CASES[name]
    pr = _prob(name)
    psi0 = _psi0(p)
    plan = fse.Plan.from_params(p, prec)
    for n, order in ((1, 2), (10, 2), (3, 4)):
        ref, t = (pr.run if order == 2 else pr.run4)(psi0, n, p.dt)
        plan.time = 0.0
        x = _dev(psi0, prec)
        plan.step(x, n, p.dt, order=order)
        err = _rel(x.cpu().numpy().astype(np.complex128), ref)
        _note(f"[axes] {name} prec={prec} steps={n} order={order}: {err:.3e}")
        assert err < tol


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-11), (fse.C64, 1e-5)])
def test_potential_and_energy_at_a_turned_time(name, prec, tol):
    p = CASES[name]
    pr = _prob(name)
    psi = _psi0(p, seed=1)
    t = 1.9
    plan = fse.Plan.from_params(p, prec)
    plan.time = t
    x = _dev(psi, prec)
    xin = x.cpu().numpy().astype(np.complex128)
    phi = plan.nonlocal_potential(x).cpu().numpy().astype(np.float64)
    ref = pr.potential(np.abs(xin) ** 2, t)
    e1 = _rel(phi, ref)
    e = plan.energy(x).cpu().numpy()
    eo = np.array(dg.energy_parts(pr, xin, t=t))
    _note(f"[axes] {name} prec={prec}: potential {e1:.3e}, max dE {np.max(np.abs(e - eo)):.3e}")
    assert e1 < tol
    assert np.all(np.abs(e - eo) <= tol * np.maximum(1.0, np.abs(eo)))


@pytest.mark.parametrize("name", list(CASES))
def test_H_and_ground_state_in_the_frame_of_the_axis(name):
    p = CASES[name]
    pr = _prob(name)
    psi = _psi0(p, seed=2)
    plan = fse.Plan.from_params(p, fse.C128)
    plan.time = 0.7  # H psi and the ground state do not depend on the step's time
    H = plan.apply_H(_dev(psi, fse.C128)).cpu().numpy()
    assert _rel(H, dg.apply_H(pr, psi)) < 1e-12
    g = ogs.GroundState(pr, 0.05)
    ref, _ = g.step(psi, rtol=1e-12)
    x = _dev(psi, fse.C128)
    plan.gs_step(x, 0.05, tol=1e-12)
    err = _rel(x.cpu().numpy(), ref)
    _note(f"[axes] {name} ground-state step: {err:.3e}")
    assert err < 1e-10


@pytest.mark.parametrize("name", ["turn3d", "turn2d"])
def test_adjoint_with_a_turning_axis(name):
    p = CASES[name]
    pr = _prob(name)
    psi0 = _psi0(p, seed=3)
    tgt = W.adjoint_target(p.N, p.L, seed=4)
    n = 5
    psiT, _ = pr.run(psi0, n, p.dt)
    _, gT = adj.loss_and_grad(psiT, tgt, p.N, p.L)
    g_ref, gU_ref = adj.run_adjoint(pr, psi0, n, p.dt, gT)
    plan = fse.Plan.from_params(p, fse.C128)
    g = _dev(gT, fse.C128)
    gU = torch.zeros(p.N, dtype=torch.float64, device="cuda:0")
    plan.step_adjoint(_dev(psi0, fse.C128), n, p.dt, g, gU)
    e1, e2 = _rel(g.cpu().numpy(), g_ref), _rel(gU.cpu().numpy(), gU_ref)
    _note(f"[axes] adjoint {name}: {e1:.3e} {e2:.3e}")
    assert e1 < 1e-11 and e2 < 1e-11


def test_rotating_frame_energy_is_conserved_on_the_gpu():
    # the oracle pin's case: 3D tilted axis turning with Omega = 0.5; drift of
    # the rotating-frame energy second order in dt
    p = W.Params(d=3, N=(24, 24, 24), L=(5.0, 5.0, 5.0), s=0.9, Omega=0.5, gamma=(1.0, 1.0, 1.2), beta=20.0,
                 lam=20.0, kernel="ddi3", axis=(0.6, 0.0, 0.8), dt=0.01, name="turn-energy")
    X = np.meshgrid(*scheme.axes(p.N, p.L), indexing="ij")
    psi0 = W.normalize(np.exp(-X[0] ** 2 / 1.2 - X[1] ** 2 / 0.7 - X[2] ** 2) * (1 + 0.2 * X[0] + 0.3j * X[1]), p.h)
    drift = []
    for n in (50, 100):
        plan = fse.Plan.from_params(p, fse.C128)
        x = _dev(psi0, fse.C128)
        E0 = plan.energy(x).cpu().numpy()[5]
        plan.step(x, n, 1.0 / n)
        drift.append(plan.energy(x).cpu().numpy()[5] - E0)
    _note(f"[axes] energy drift over t = 1: {drift}")
    assert abs(drift[1]) < 1e-3 and 3.5 < drift[0] / drift[1] < 4.5


def test_batch_rejects_a_turning_axis():
    p = CASES["turn2d"].replace(N=(64, 64), L=(8.0, 8.0))
    with pytest.raises(fse.FseError):
        fse.Batch([p], fse.C64)
