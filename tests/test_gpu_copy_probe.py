"""The streaming-copy probe used as the measured HBM ceiling copies its bytes exactly."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0707_1299_amd import lbm  # noqa: E402


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, (1 << 20) * 3 + 48])
def test_copy_probe_copies_exactly(nbytes):
    g = torch.Generator(device="cuda").manual_seed(7)
    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros_like(src)
    lbm.lb_copy_probe(src, dst, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert int(dst[nbytes:].count_nonzero()) == 0
