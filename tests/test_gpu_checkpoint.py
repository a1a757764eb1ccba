"""Resume from a checkpoint continues the trajectory; the diagnostics log records the invariants."""
import json
import os

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")

from paper_1512_03210_amd import checkpoint, fse  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fse.lib()


def _params():
    return W.Params(d=3, N=(32, 32, 24), L=(6.0, 6.0, 5.0), s=0.8, Omega=0.7, gamma=(1.0, 1.2, 2.0), beta=200.0,
                    lam=50.0, kernel="ddi3", dt=5e-4)


@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-13), (fse.C64, 2e-6)])
def test_resume_equals_an_uninterrupted_run(tmp_path, prec, tol):
    p = _params()
    dt = np.complex128 if prec == fse.C128 else np.complex64
    psi0 = W.anisotropic_gaussian(p.N, p.L, p.gamma, seed=5).astype(dt)
    a = torch.from_numpy(psi0).to("cuda:0")
    plan = fse.Plan.from_params(p, prec)
    plan.step(a, 12, p.dt)
    b = torch.from_numpy(psi0).to("cuda:0")
    first = fse.Plan.from_params(p, prec)
    first.step(b, 7, p.dt)
    prefix = os.path.join(tmp_path, "ck")
    checkpoint.save(prefix, p, b, first.time, prec)
    del first, b
    plan2, c, p2 = checkpoint.resume(prefix, W.Params)
    assert p2 == p and abs(plan2.time - 7 * p.dt) < 1e-15
    plan2.step(c, 5, p.dt)
    assert abs(plan2.time - plan.time) < 1e-15
    err = float(torch.linalg.vector_norm(c - a) / torch.linalg.vector_norm(a))
    assert err < tol
    # a second resume from the same files repeats the continuation bit for bit
    plan3, c3, _ = checkpoint.resume(prefix, W.Params)
    plan3.step(c3, 5, p.dt)
    assert torch.equal(c3, c)


def test_logged_run_writes_one_line_per_chunk(tmp_path):
    p = _params()
    psi = torch.from_numpy(W.anisotropic_gaussian(p.N, p.L, p.gamma, seed=6)).to("cuda:0")
    plan = fse.Plan.from_params(p, fse.C128)
    m0 = plan.mass(psi).item()
    log = os.path.join(tmp_path, "diag.jsonl")
    checkpoint.run_logged(plan, psi, 23, p.dt, 5, log)
    recs = [json.loads(line) for line in open(log)]
    assert [r["steps"] for r in recs] == [5, 10, 15, 20, 23]
    assert abs(recs[-1]["t"] - 23 * p.dt) < 1e-15
    for r in recs:
        assert abs(r["mass"] - m0) < 1e-12 * m0
        e = r["energy"]
        assert abs(e["total"] - (e["kin"] + e["pot"] + e["int"] + e["non"] + e["rot"])) < 1e-12 * abs(e["total"])
    assert abs(recs[-1]["energy"]["total"] - recs[0]["energy"]["total"]) < 1e-3 * abs(recs[0]["energy"]["total"])


@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-13), (fse.C64, 2e-6)])
def test_resume_keeps_the_plan_state(tmp_path, prec, tol):
    # a plan with a grid potential, a turning optical lattice and non-default kernel options: the resumed plan
    # rebuilds all of them and continues the uninterrupted run
    import math
    p = W.Params(d=2, N=(48, 64), L=(6.0, 7.0), s=0.8, Omega=0.5, gamma=(1.0, 1.2), beta=20.0, lam=2.0,
                 kernel="coulomb", coef=1.0 / (2.0 * math.pi), dt=2e-3)
    cd, rd = (np.complex128, np.float64) if prec == fse.C128 else (np.complex64, np.float32)
    psi0 = W.harmonic_vortex_2d(p.N, p.L, seed=8).astype(cd)
    X, Y = W.mesh(p.N, p.L)
    U = torch.from_numpy((0.3 * np.cos(X) * np.sin(0.5 * Y)).astype(rd)).to("cuda:0")
    lat = ((4.0, 6.0), (1.5, 2.0))
    opts = dict(delta=2e-3, ht=0.12)

    def make():
        pl = fse.Plan.from_params(p, prec, **opts)
        pl.set_potential(U.clone())
        pl.set_lattice(*lat)
        return pl

    a = torch.from_numpy(psi0).to("cuda:0")
    whole = make()
    whole.step(a, 12, p.dt)
    b = torch.from_numpy(psi0).to("cuda:0")
    first = make()
    first.step(b, 7, p.dt)
    prefix = os.path.join(tmp_path, "ck")
    checkpoint.save(prefix, p, b, first.time, prec, plan=first)
    del first, b
    plan2, c, _ = checkpoint.resume(prefix, W.Params)
    plan2.step(c, 5, p.dt)
    err = float(torch.linalg.vector_norm(c - a) / torch.linalg.vector_norm(a))
    assert err < tol, err
    # without the lattice and the potential the continuation differs
    bare = fse.Plan.from_params(p, prec)
    d = torch.from_numpy(psi0).to("cuda:0")
    bare.step(d, 12, p.dt)
    assert float(torch.linalg.vector_norm(d - a) / torch.linalg.vector_norm(a)) > 1e3 * tol
