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

    def numel(self):
        n = 1
        for k in self.shape:
            n *= k
        return n

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


_BAD_STATES = [_T(torch.complex64, (16, 16)), _T(torch.complex128, (16,)), _T(torch.complex128, (16, 16), cuda=False),
               _T(torch.complex128, (16, 16), contiguous=False)]


@pytest.mark.parametrize("bad", _BAD_STATES)
@pytest.mark.parametrize("call", [
    lambda p, x: p.step(x, 1, 1e-3, order=4),
    lambda p, x: p.energy(x),
    lambda p, x: p.angular_momentum(x),
    lambda p, x: p.moments(x),
    lambda p, x: p.mass_noalloc(x, _T(torch.float64, (1,))),
    lambda p, x: p.apply_Lz(x),
    lambda p, x: p.apply_Lz(_T(torch.complex128, (16, 16)), out=x),
    lambda p, x: p.angular_momentum_grad(x),
    lambda p, x: p.apply_H(x),
    lambda p, x: p.nonlocal_potential(x),
    lambda p, x: p.gs_step(x, 0.01),
    lambda p, x: p.gs_run(x, 0.01, max_steps=2),
    lambda p, x: p.step_adjoint(x, 1, 1e-3, _T(torch.complex128, (16, 16))),
    lambda p, x: p.step_adjoint(_T(torch.complex128, (16, 16)), 1, 1e-3, x),
])
def test_every_state_argument_is_checked(call, bad):
    with pytest.raises(ValueError):
        call(_plan(), bad)


@pytest.mark.parametrize("bad", [_T(torch.float32, (16, 16)), _T(torch.float64, (16, 8)),
                                 _T(torch.float64, (16, 16), cuda=False)])
def test_real_grid_arguments_are_checked(bad):
    p = _plan()
    with pytest.raises(ValueError):
        p.set_potential(bad)
    with pytest.raises(ValueError):
        p.step_adjoint(_T(torch.complex128, (16, 16)), 1, 1e-3, _T(torch.complex128, (16, 16)), grad_U=bad)


def test_scalar_outputs_are_checked():
    p = _plan()
    psi = _T(torch.complex128, (16, 16))
    for bad in (_T(torch.float32, (1,)), _T(torch.float64, (0,)), _T(torch.float64, (1,), cuda=False)):
        with pytest.raises(ValueError):
            p.mass_noalloc(psi, bad)
    for g in (_T(torch.float32, (1,)), _T(torch.float64, (2,)), _T(torch.float64, (1,), cuda=False)):
        with pytest.raises(ValueError):
            p.angular_momentum_grad(psi, g=g, out=_T(torch.complex128, (16, 16)))


def test_batch_packed_state_is_checked():
    b = fse.Batch.__new__(fse.Batch)
    b.cdtype, b.offsets, b.count, b._h = torch.complex64, [0, 256], 1, None
    for bad in (_T(torch.complex128, (256,)), _T(torch.complex64, (255,)), _T(torch.complex64, (256,), cuda=False),
                _T(torch.complex64, (256,), contiguous=False)):
        with pytest.raises(ValueError):
            b.step(bad, 1)
        with pytest.raises(ValueError):
            b.reduce(bad)
