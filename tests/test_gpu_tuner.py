"""The pass-schedule autotuner (fse_plan_tune): every schedule it can choose
matches the oracle, tuning is stable, and the file cache round-trips."""
import itertools
import math
import os
import sys

import numpy as np
import pytest

import workloads as W
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


# contiguous axis of 256 points: the kinetic lines (256) and the convolution
# lines (512) both have an alternative radix schedule; a 256-point axis 0 (or
# axis 1 in 3D) has an alternative column plan
CASES = {
    "rot3d": W.Params(d=3, N=(16, 24, 256), L=(4.0, 5.0, 12.0), s=0.8, Omega=0.5, gamma=(1.0, 1.2, 0.3),
                      beta=50.0, lam=5.0, kernel="coulomb", dt=1e-3, name="rot3d"),
    "rot2d": W.Params(d=2, N=(48, 256), L=(6.0, 12.0), s=0.7, Omega=0.6, gamma=(1.0, 0.5), beta=40.0, lam=2.0,
                      kernel="coulomb", dt=1e-3, name="rot2d"),
    "cols3d": W.Params(d=3, N=(24, 256, 16), L=(5.0, 12.0, 4.0), s=0.9, Omega=0.4, gamma=(1.2, 0.3, 1.5),
                       beta=30.0, lam=4.0, kernel="ddi3", dt=1e-3, name="cols3d"),
    "cols2d": W.Params(d=2, N=(256, 48), L=(12.0, 6.0), s=0.8, Omega=0.5, gamma=(0.4, 1.1), beta=40.0, lam=2.0,
                       kernel="coulomb", dt=1e-3, name="cols2d"),
    # 256-point axis 0 in 3D: both column plans and both radix plans of the fused phase pass
    "fused3d": W.Params(d=3, N=(256, 16, 24), L=(12.0, 4.0, 5.0), s=0.7, Omega=0.5, gamma=(0.3, 1.2, 1.0),
                        beta=40.0, lam=3.0, kernel="ddi3", dt=1e-3, name="fused3d"),
}
_REF = {}


def _psi0(p):
    if p.d == 2:
        return W.harmonic_vortex_2d(p.N, p.L, seed=2)
    return W.anisotropic_gaussian(p.N, p.L, p.gamma, seed=2)


def _ref(name):
    if name not in _REF:
        p = CASES[name]
        pr = scheme.Problem.from_params(p)
        psi0 = _psi0(p)
        _REF[name] = (psi0, pr.run(psi0, 2, p.dt)[0])
    return _REF[name]


def _schedules(plan):
    """Every schedule the plan accepts."""
    out = []
    for sc in itertools.product((0, 1), repeat=fse.NSCHED):
        try:
            plan.set_schedule(list(sc))
        except fse.FseError:
            continue
        out.append(list(sc))
    return out


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-12), (fse.C64, 1e-5)])
def test_every_schedule_against_oracle(name, prec, tol):
    p = CASES[name]
    psi0, ref = _ref(name)
    cd = np.complex128 if prec == fse.C128 else np.complex64
    plan = fse.Plan.from_params(p, prec)
    scheds = _schedules(plan)
    assert len(scheds) == {"rot3d": 8, "rot2d": 4, "cols3d": 4, "cols2d": 4, "fused3d": 8}[name]
    for sc in scheds:
        plan.set_schedule(sc)
        plan.time = 0.0
        x = torch.from_numpy(psi0.astype(cd)).cuda()
        plan.step(x, 2, p.dt)
        err = float(np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref))
        _note(f"[tuner] {name} prec={prec} schedule {sc}: {err:.3e}")
        assert err < tol


def test_tune_is_stable_and_file_cache_round_trips(tmp_path):
    p = CASES["rot3d"]
    path = str(tmp_path / "tune.txt")
    a = fse.Plan.from_params(p, fse.C64)
    r1 = a.tune(cache_path=path)
    _note(f"[tuner] rot3d c64: {r1}")
    assert all(v in (0, 1) for v in r1["schedule"]) and len(r1["schedule"]) == fse.NSCHED
    # every allowed schedule timed (3D, line alternatives at 256 and 512, no 256-point column axis): 8 of 16
    assert sum(t > 0 for t in r1["tuned_ms"]) == 8 and all(t == -1.0 for t in r1["tuned_ms"][8:])
    assert a.time == 0.0  # tuning runs steps on scratch and restores the plan's time
    with open(path) as f:
        lines = [l for l in f.read().splitlines() if l]
    assert len(lines) == 1 and lines[0].endswith(" ".join(map(str, r1["schedule"])))
    # a second plan of the same shape takes the cached choice without timing
    b = fse.Plan.from_params(p, fse.C64)
    r2 = b.tune(cache_path=path)
    assert r2["schedule"] == r1["schedule"] and all(t == -1.0 for t in r2["tuned_ms"])
    # the tuned plan still matches the oracle
    psi0, ref = _ref("rot3d")
    x = torch.from_numpy(psi0.astype(np.complex64)).cuda()
    b.step(x, 2, p.dt)
    assert float(np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)) < 1e-5


def test_invalid_schedules_rejected():
    p2 = CASES["rot2d"]
    plan = fse.Plan.from_params(p2, fse.C128)
    with pytest.raises(fse.FseError):
        plan.set_schedule([0, 0, 1])  # mirrored order is 3D only
    with pytest.raises(fse.FseError):
        plan.set_schedule([2, 0, 0])
    small = fse.Plan.from_params(W.preset("plain2d"), fse.C128)  # 64-point lines: no alternative
    with pytest.raises(fse.FseError):
        small.set_schedule([1, 0, 0])
    assert small.schedule()["schedule"] == [0, 0, 0, 0, 0]
    with pytest.raises(fse.FseError):
        small.set_schedule([0, 0, 0, 1])  # 64-point columns: no alternative plan
    with pytest.raises(fse.FseError):
        small.set_schedule([0, 0, 0, 0, 1])  # 64-point fused pass: one plan
    cols = fse.Plan.from_params(CASES["cols2d"], fse.C128)
    cols.set_schedule([0, 0, 0, 1])
    assert cols.schedule()["schedule"] == [0, 0, 0, 1, 0]
    cols.set_schedule([0, 0, 0, 1, 1])
    assert cols.schedule()["schedule"] == [0, 0, 0, 1, 1]


def test_tuning_a_fused_axis_of_256_points():
    p = CASES["fused3d"]
    plan = fse.Plan.from_params(p, fse.C64)
    r = plan.tune()
    _note(f"[tuner] fused3d c64: {r}")
    timed = [i for i, t in enumerate(r["tuned_ms"]) if t > 0]
    assert len(timed) == 8 and sum(1 for i in timed if i & 16) == 4  # both fused plans timed
    psi0, ref = _ref("fused3d")
    x = torch.from_numpy(psi0.astype(np.complex64)).cuda()
    plan.step(x, 2, p.dt)
    assert float(np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)) < 1e-5


def test_tuning_a_column_axis_of_256_points():
    p = CASES["cols3d"]
    plan = fse.Plan.from_params(p, fse.C128)
    r = plan.tune()
    _note(f"[tuner] cols3d c128: {r}")
    timed = [i for i, t in enumerate(r["tuned_ms"]) if t > 0]
    assert len(timed) == 4 and all(i & 8 for i in timed[2:])  # the column plan alternative was timed
    psi0, ref = _ref("cols3d")
    x = torch.from_numpy(psi0).cuda()
    plan.step(x, 2, p.dt)
    assert float(np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)) < 1e-12
