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
