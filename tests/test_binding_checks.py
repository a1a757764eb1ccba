"""The binding refuses buffers of the wrong dtype, shape, layout or device before any library call (a wrong buffer
would make a kernel write or read out of bounds).  Runs on the CPU: the plan is a bare binding object and the
tensors are stand-ins that report the properties the checks look at."""
import pytest

torch = pytest.importorskip("torch")

from paper_1512_03210_amd import fse  # noqa: E402


class _T:
    """Tensor stand-in: dtype, shape, device flag and contiguity."""

    def __init__(self, dtype, shape, cuda=True, contiguous=True):
        self.dtype, self.shape, self.is_cuda, self._c = dtype, shape, cuda, contiguous
        self.device = "cuda:0"

    def is_contiguous(self):
        return self._c

    def data_ptr(self):
        raise AssertionError("the library must not be reached")


def _plan(N=(16, 16)):
    p = fse.Plan.__new__(fse.Plan)
    p.N, p.cdtype, p.rdtype, p._h = N, torch.complex128, torch.float64, None
    return p


@pytest.mark.parametrize("bad", [
    _T(torch.float32, (16, 16)),                       # wrong precision
    _T(torch.float64, (16, 8)),                        # wrong shape: the kernel would write past its end
    _T(torch.float64, (16, 16), cuda=False),           # host memory
    _T(torch.float64, (16, 16), contiguous=False),
])
def test_nonlocal_potential_out_and_frozen_density_are_checked(bad):
    p = _plan()
    psi = _T(torch.complex128, (16, 16))
    with pytest.raises(ValueError):
        p.nonlocal_potential(psi, out=bad)
    with pytest.raises(ValueError):
        p.apply_H(psi, out=_T(torch.complex128, (16, 16)), rho_frozen=bad)


def test_state_checks():
    p = _plan()
    for bad in (_T(torch.complex64, (16, 16)), _T(torch.complex128, (16,)), _T(torch.complex128, (16, 16), cuda=False)):
        with pytest.raises(ValueError):
            p.mass(bad)
        with pytest.raises(ValueError):
            p.step(bad, 1, 1e-3)
