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


@pytest.mark.parametrize("name", ["plain2d", "dipole3d_128"])
def test_complex64_mass_renormalisation(name):
    # complex64, 1000 steps in one call: with the FP64 renormalisation (the default) the call returns the mass it
    # was given; without it the FP32 twiddle residuals bias the mass by a few 1e-8 per step
    p = W.preset(name)
    psi0 = W.initial_state(p, seed=0).astype(np.complex64)
    out = {}
    for on in (True, False):
        plan = fse.Plan.from_params(p, fse.C64)
        assert plan.mass_renorm()[0]  # on by default for complex64
        plan.set_mass_renorm(on)
        x = torch.from_numpy(psi0).cuda()
        m0 = plan.mass(x).item()
        plan.step(x, STEPS, p.dt)
        m1 = plan.mass(x).item()
        out[on] = (m1 - m0, plan.mass_renorm(), x.to(torch.complex128))
    ref = fse.Plan.from_params(p, fse.C128)
    assert not ref.mass_renorm()[0]  # off for complex128
    y = torch.from_numpy(W.initial_state(p, seed=0)).cuda()
    ref.step(y, STEPS, p.dt)
    e_on = float(torch.linalg.vector_norm(out[True][2] - y) / torch.linalg.vector_norm(y))
    e_off = float(torch.linalg.vector_norm(out[False][2] - y) / torch.linalg.vector_norm(y))
    _note(f"[renorm] {name}: dmass on {out[True][0]:.2e}, off {out[False][0]:.2e}; factor {out[True][1][1]!r}; "
          f"state vs FP64 on {e_on:.3e}, off {e_off:.3e}")
    # the exit transform, after the mass is measured, adds its own FP32 rounding (~1e-8)
    assert abs(out[True][0]) < 1e-7
    assert abs(out[True][1][1] - 1.0) < 1e-3 and out[True][1][1] != 1.0
    assert e_on <= e_off * 1.05
