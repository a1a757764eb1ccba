"""fse_mass_noalloc (the allocation-free variant of fse_mass) against fse_mass, through the C ABI.

Two calls in a row on one device, the second on a smaller grid, each against fse_mass of the same state:
the variant runs the same kernels on the same data, so the FP64 masses agree bit for bit.  The second call
reuses the device array that the first one filled.
"""
import ctypes

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


def _state(p, prec, seed):
    cd = np.complex128 if prec == fse.C128 else np.complex64
    return torch.from_numpy(W.initial_state(p, seed=seed).astype(cd)).to("cuda:0")


@pytest.mark.parametrize("prec", [fse.C128, fse.C64])
def test_noalloc_mass_matches_fse_mass_on_two_calls(prec):
    big = W.preset("dipole3d_128")
    small = W.preset("plain2d")
    L = fse.lib()
    st = fse._stream(None)
    for p, seed in ((big, 1), (small, 2)):
        plan = fse.Plan.from_params(p, prec)
        x = _state(p, prec, seed)
        x.mul_(1.25)  # mass 1.5625, not the normalised 1
        ref = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda:0")
        out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda:0")
        assert L.fse_mass(plan._h, fse._ptr(x), fse._ptr(ref), st) == 0
        assert L.fse_mass_noalloc(plan._h, fse._ptr(x), fse._ptr(out), st) == 0, L.fse_last_error()
        torch.cuda.synchronize()
        assert out.item() == ref.item(), (p.name, out.item(), ref.item())
        tol = 1e-12 if prec == fse.C128 else 1e-5
        assert abs(ref.item() - 1.5625) < tol
        del plan


def test_noalloc_mass_argument_errors():
    p = W.preset("plain2d")
    plan = fse.Plan.from_params(p, fse.C128)
    L = fse.lib()
    x = _state(p, fse.C128, 0)
    assert L.fse_mass_noalloc(None, fse._ptr(x), fse._ptr(x), fse._stream(None)) == -1
    assert L.fse_mass_noalloc(plan._h, None, fse._ptr(x), fse._stream(None)) == -1
    assert L.fse_mass_noalloc(plan._h, fse._ptr(x), ctypes.c_void_p(), fse._stream(None)) == -1
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    plan.mass_noalloc(x, out)
    torch.cuda.synchronize()
    assert abs(out.item() - 1.0) < 1e-13
