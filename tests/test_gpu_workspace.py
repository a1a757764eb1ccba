"""Caller-owned step scratch (fse_scratch_size, fse_set_workspace)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1512_03210_amd import fse  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fse.lib()


@pytest.mark.parametrize("prec", [fse.C128, fse.C64])
def test_caller_scratch_gives_identical_steps(prec):
    p = W.Params(d=3, N=(32, 24, 16), L=(6.0, 5.0, 4.0), s=0.8, Omega=0.7, gamma=(1.0, 1.3, 2.0), beta=50.0,
                 lam=5.0, kernel="coulomb", dt=1e-3, name="ws3d")
    cd = np.complex128 if prec == fse.C128 else np.complex64
    psi0 = W.anisotropic_gaussian(p.N, p.L, p.gamma, seed=3).astype(cd)
    a = fse.Plan.from_params(p, prec)
    b = fse.Plan.from_params(p, prec)
    need = b.scratch_bytes()
    assert need >= (p.N[0] + 1) * p.N[1] * p.N[2] * (16 if prec == fse.C128 else 8)
    held = b.workspace_bytes()
    buf = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    b.set_workspace(buf)
    assert b.workspace_bytes() < held
    x, y = torch.from_numpy(psi0).cuda(), torch.from_numpy(psi0).cuda()
    a.step(x, 5, p.dt)
    buf.fill_(0xFF)  # the scratch carries nothing between calls
    b.step(y, 5, p.dt)
    assert torch.equal(x, y)
    assert torch.equal(a.energy(x), b.energy(y))
    before = b.workspace_bytes()  # now with the diagnostics buffer of the energy call
    b.set_workspace(None)  # back to plan-owned scratch: X1 and X2 allocated again
    cs = 16 if prec == fse.C128 else 8
    assert b.workspace_bytes() - before == 3 * (p.N[0] + 1) * p.N[1] * p.N[2] * cs
    b.step(y, 1, p.dt)
    a.step(x, 1, p.dt)
    assert torch.equal(x, y)


def test_workspace_errors_and_local_plans():
    p = W.preset("plain2d")
    plan = fse.Plan.from_params(p, fse.C128)
    need = plan.scratch_bytes()
    with pytest.raises(fse.FseError):
        plan.set_workspace(torch.empty(need - 256, dtype=torch.uint8, device="cuda:0"))
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(fse.FseError):
        plan.set_workspace(big[1:])  # not 256-byte aligned
    local = fse.Plan.from_params(p.replace(lam=0.0, kernel="none"), fse.C128)
    assert local.scratch_bytes() == 0
    local.set_workspace(torch.empty(16, dtype=torch.uint8, device="cuda:0"))  # nothing to take: accepted
