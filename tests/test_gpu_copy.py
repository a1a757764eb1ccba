"""The library's streaming copy kernel (the HBM-counter calibration reference)."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1512_03210_amd import fse  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fse.lib()


@pytest.mark.parametrize("nt", [False, True])
@pytest.mark.parametrize("n16", [1, 255, 1024, 1025, 3 * 1024 + 17, 1 << 20])
def test_copy_exact(n16, nt):
    # sizes below, at and across the 1024-element workgroup, with a ragged tail
    g = torch.Generator(device="cpu").manual_seed(n16)
    src = torch.randn(2 * n16, dtype=torch.float64, generator=g).cuda()
    guard = 64
    dst = torch.full((2 * n16 + guard,), -7.0, dtype=torch.float64, device="cuda")
    fse.device_copy(dst, src, 16 * n16, nontemporal=nt)
    torch.cuda.synchronize()
    assert torch.equal(dst[: 2 * n16], src)
    assert torch.all(dst[2 * n16:] == -7.0)  # nothing written past the end


def test_copy_rejects_bad_arguments():
    a = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(fse.FseError):
        fse.device_copy(a, a[1:], 16)  # misaligned source
    with pytest.raises(fse.FseError):
        fse.device_copy(a, a, 24)  # not a multiple of 16
    with pytest.raises(fse.FseError):
        fse.device_copy(a, a[1:], 16, nontemporal=True)
