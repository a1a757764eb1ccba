"""Numeric guard (fse_set_guard / fse_guard_status), a failure-detection aid the paper does not have.

The failing conditions are planted from the host in the state (a NaN value, a rescaled state); every
kernel still runs to completion (NaN arithmetic does not fault), and the guard must report them.
"""
import math

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")

from paper_1512_03210_amd import fse  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {fse.C128: 1e-8, fse.C64: 1e-4}


@pytest.fixture(scope="module", autouse=True)
def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fse.lib()


def _setup(prec):
    p = W.preset("plain2d")
    psi0 = W.harmonic_vortex_2d(p.N, p.L, seed=0)
    dt = np.complex128 if prec == fse.C128 else np.complex64
    x = torch.from_numpy(psi0.astype(dt)).to("cuda:0")
    return p, fse.Plan.from_params(p, prec), x


@pytest.mark.parametrize("prec", [fse.C128, fse.C64])
def test_guard_is_off_by_default_and_quiet_on_a_good_run(prec):
    p, plan, x = _setup(prec)
    plan.step(x, 5, p.dt)
    tripped, m0, m = plan.guard_status()
    assert not tripped and math.isnan(m0) and math.isnan(m)
    plan.set_guard(TOL[prec])
    plan.step(x, 10, p.dt)
    ref = plan.mass(x).item()
    for _ in range(3):
        plan.step(x, 10, p.dt)
        plan.step(x, 2, p.dt, order=4)
    tripped, m0, m = plan.guard_status()
    assert not tripped
    assert abs(m0 - ref) <= 1e-14 * ref  # the reference is the mass after the first guarded call
    assert abs(m - plan.mass(x).item()) <= 1e-14 * ref
    assert abs(m - m0) <= TOL[prec] * m0


@pytest.mark.parametrize("prec", [fse.C128, fse.C64])
def test_guard_trips_on_a_nan_and_blocks_later_steps_until_reset(prec):
    p, plan, x = _setup(prec)
    good = x.clone()
    plan.set_guard(TOL[prec])
    plan.step(x, 2, p.dt)
    x[3, 5] = complex("nan")
    plan.step(x, 2, p.dt)  # its own check trips; the call itself has launched normally
    torch.cuda.synchronize()
    with pytest.raises(fse.FseError) as e:
        plan.step(x, 1, p.dt)
    assert e.value.status == fse.STATUS_CODES["FSE_ERR_NUMERIC"]
    with pytest.raises(fse.FseError):
        plan.step(x, 1, p.dt, order=4)  # stays tripped
    tripped, m0, m = plan.guard_status()
    assert tripped and math.isfinite(m0) and math.isnan(m)
    # restart from a good state: re-arming clears the flag and the reference
    x.copy_(good)
    plan.set_guard(TOL[prec])
    plan.step(x, 3, p.dt)
    assert not plan.guard_status()[0]
    plan.step(x, 3, p.dt)
    assert not plan.guard_status()[0]


@pytest.mark.parametrize("prec", [fse.C128, fse.C64])
def test_guard_trips_on_a_mass_change_and_can_be_turned_off(prec):
    p, plan, x = _setup(prec)
    plan.set_guard(TOL[prec])
    plan.step(x, 2, p.dt)
    x.mul_(1.01)
    plan.step(x, 2, p.dt)
    tripped, m0, m = plan.guard_status()
    assert tripped and abs(m / m0 - 1.0201) < 1e-3
    plan.set_guard(0.0)  # off: steps run again and nothing is checked
    plan.step(x, 2, p.dt)
    assert plan.guard_status()[0] is False


def test_guard_rejects_a_non_finite_tolerance():
    _, plan, _ = _setup(fse.C128)
    with pytest.raises(fse.FseError) as e:
        plan.set_guard(float("nan"))
    assert e.value.status == fse.STATUS_CODES["FSE_ERR_ARG"]
