"""Drift of the GPU path against the FP64 oracle over 1000 steps of the 2D plain case
(64^2, s = 0.75, Omega = 0.5, beta = 100, Coulomb GauSum, dt = 1e-3).

One step is gated at 1e-12 (FP64) and 1e-5 (complex64) elsewhere; over many steps the
nonlinear dynamics amplify round-off, so these bounds are loose and the measured values
are printed for the record."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import diagnostics as dg
from oracle import scheme

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1512_03210_amd import fse  # noqa: E402

STEPS = 1000


def _note(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fse.lib()


@pytest.fixture(scope="module")
def oracle_run():
    p = W.preset("plain2d")
    psi0 = W.initial_state(p, seed=0)
    pr = scheme.Problem.from_params(p)
    ref, t = pr.run(psi0, STEPS, p.dt)
    return p, psi0, pr, ref, t


@pytest.mark.parametrize("prec,tol_state,tol_scalar", [(fse.C128, 1e-8, 1e-10), (fse.C64, 5e-3, 2e-3)])
def test_drift_1000_steps(oracle_run, prec, tol_state, tol_scalar):
    p, psi0, pr, ref, t = oracle_run
    dt_np = np.complex128 if prec == fse.C128 else np.complex64
    plan = fse.Plan.from_params(p, prec)
    x = torch.from_numpy(psi0.astype(dt_np)).cuda()
    plan.step(x, STEPS, p.dt)
    e = plan.energy(x).cpu().numpy()
    m = plan.mass(x).item()
    lz = plan.angular_momentum(x).item()
    y = x.cpu().numpy().astype(np.complex128)
    err = float(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    eo = np.array(dg.energy_parts(pr, ref, t=t))
    mo, lzo = dg.mass(ref, p.N, p.L), dg.angular_momentum(ref, p.N, p.L)
    _note(f"[drift] {STEPS} steps prec={prec}: state rel L2 {err:.3e}; |dmass| {abs(m - mo):.2e}, "
          f"|dE_total| {abs(e[5] - eo[5]):.2e}, |dLz| {abs(lz - lzo):.2e} (oracle E {eo[5]:.6f}, Lz {lzo:.6f})")
    assert abs(plan.time - t) < 1e-12
    assert err < tol_state
    assert abs(m - mo) < tol_scalar
    assert abs(e[5] - eo[5]) < tol_scalar * max(1.0, abs(eo[5]))
    assert abs(lz - lzo) < tol_scalar * max(1.0, abs(lzo))
