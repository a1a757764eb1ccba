"""Diagnostic calls recorded into a HIP graph (torch.cuda.graph) and replayed.

Every replay follows eager work that changes the state (and overwrites the outputs) and a synchronisation, and
must equal the eager calls on the current state bit for bit: the graph reads the live buffers, and no call
records a runtime memset (the buffers a call clears are cleared by a fill kernel).
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")

from paper_1512_03210_amd import fse  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fse.lib()


def _params(kernel="ddi3", lam=50.0):
    return W.Params(d=3, N=(32, 32, 24), L=(6.0, 6.0, 5.0), s=0.8, Omega=0.7, gamma=(1.0, 1.2, 2.0), beta=200.0,
                    lam=lam, kernel=kernel, dt=5e-4)


def _dev(a, prec):
    return torch.from_numpy(a.astype(np.complex128 if prec == fse.C128 else np.complex64)).to("cuda:0")


@pytest.mark.parametrize("prec", [fse.C128, fse.C64])
def test_diagnostics_replay_equal_eager_calls(prec):
    p = _params()
    p0 = _params(kernel="none", lam=0.0)
    psi = _dev(W.anisotropic_gaussian(p.N, p.L, p.gamma, seed=3), prec)
    plan = fse.Plan.from_params(p, prec)
    plan0 = fse.Plan.from_params(p0, prec)
    # first calls allocate the plans' diagnostic buffers (nothing may be allocated while capturing)
    plan.energy(psi), plan.mass(psi), plan.angular_momentum(psi), plan.apply_Lz(psi), plan0.nonlocal_potential(psi)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        e = plan.energy(psi)
        m = plan.mass(psi)
        lz = plan.angular_momentum(psi)
        lzpsi = plan.apply_Lz(psi)
        phi0 = plan0.nonlocal_potential(psi)
    torch.cuda.synchronize()
    for k in range(4):
        # eager work between replays: a new state, garbage in every output
        psi.mul_(0.97 - 0.01 * k)
        psi[k, 2 * k, 3] += 0.05
        for t in (e, m, lz):
            t.fill_(-1.0)
        lzpsi.fill_(7.0)
        phi0.fill_(1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(e, plan.energy(psi))
        assert torch.equal(m, plan.mass(psi))
        assert torch.equal(lz, plan.angular_momentum(psi))
        assert torch.equal(lzpsi, plan.apply_Lz(psi))
        assert torch.count_nonzero(phi0).item() == 0
        torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# Steps recorded into a graph: the time of the state lives in device memory, so a replay runs at the time the
# plan has when it runs (the trap integral P(x~; t, t+dt) of an anisotropic rotating trap, eq. int_poten; a
# dipole axis that turns in the rotating frame, eq. Kernel_Rot; a turning optical lattice), not at the time of
# the capture.
# ---------------------------------------------------------------------------
import math  # noqa: E402

from oracle import diagnostics as odg  # noqa: E402
from oracle import scheme  # noqa: E402

STEP_CASES = {
    # anisotropic trap under rotation: P depends on t
    "aniso2d": (W.Params(d=2, N=(48, 64), L=(6.0, 7.0), s=0.8, Omega=0.7, gamma=(1.0, 1.4), beta=30.0, lam=2.0,
                         kernel="coulomb", dt=2e-3, name="cap-aniso2d"), None),
    # dipole axis off z under rotation: the multiplier turns with t
    "turning3d": (W.Params(d=3, N=(24, 32, 16), L=(5.0, 6.0, 4.0), s=0.9, Omega=0.6, gamma=(1.0, 1.2, 1.5),
                           beta=30.0, lam=10.0, kernel="ddi3", axis=(1.0, 0.0, 0.0), dt=2e-3, name="cap-turn3d"),
                  None),
    # optical lattice under rotation: its time integral turns with t
    "lattice2d": (W.Params(d=2, N=(64, 48), L=(6.0, 5.0), s=0.8, Omega=0.5, gamma=(1.0, 1.0), beta=20.0, lam=2.0,
                           kernel="coulomb", coef=1.0 / (2.0 * math.pi), dt=2e-3, name="cap-lat2d"),
                  ((10.0, 10.0), (math.pi, math.pi))),
}


def _case_plan(name, prec):
    p, lat = STEP_CASES[name]
    plan = fse.Plan.from_params(p, prec)
    if lat is not None:
        plan.set_lattice(*lat)
    return plan


def _case_psi0(p):
    if p.d == 2:
        return W.harmonic_vortex_2d(p.N, p.L, seed=5)
    return W.anisotropic_gaussian(p.N, p.L, p.gamma, seed=5)


@pytest.mark.parametrize("name", list(STEP_CASES))
@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-12), (fse.C64, 1e-5)])
def test_captured_steps_replay_at_the_current_time(name, prec, tol):
    p, lat = STEP_CASES[name]
    psi0 = _case_psi0(p)
    pg, pe = _case_plan(name, prec), _case_plan(name, prec)
    xg, xe = _dev(psi0, prec), _dev(psi0, prec)
    # first calls build the kinetic tables of this dt and the diagnostic buffers
    w = xg.clone()
    pg.step(w, 2, p.dt)
    pg.energy(w), pg.moments(w)
    pg.time = 0.0
    del w
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pg.step(xg, 2, p.dt)
        e = pg.energy(xg)
        mo = pg.moments(xg)
    torch.cuda.synchronize()
    assert pg.time == 0.0  # capturing runs nothing
    for k in range(3):
        # eager work between replays: the eager twin advances, and other calls run on the captured plan
        pe.step(xe, 2, p.dt)
        junk = pg.mass(xe)
        e.fill_(-1.0)
        mo.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(xg, xe), (name, k)
        assert torch.equal(e, pe.energy(xe)), (name, k)
        assert torch.equal(mo, pe.moments(xe)), (name, k)
        assert abs(pg.time - 2 * (k + 1) * p.dt) < 1e-15 and pg.time == pe.time
        del junk
    # the replayed trajectory (6 steps, three different start times) against the oracle
    pr = scheme.Problem.from_params(p)
    if lat is not None:
        pr.lattice = (tuple(lat[0]) + (0.0,), tuple(lat[1]) + (0.0,))
    ref, t = pr.run(psi0, 6, p.dt)
    out = xg.cpu().numpy().astype(np.complex128)
    err = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    assert err < tol, (name, err)
    eo = odg.energy_parts(pr, ref, t)
    eg = e.cpu().numpy()
    assert abs(eg[5] - eo[5]) < (1e-11 if prec == fse.C128 else 1e-4) * max(1.0, abs(eo[5])), (name, eg, eo)
