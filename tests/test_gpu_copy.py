"""The roofline reference copy kernel (rtm_device_copy) moves every byte."""
import pytest
import torch

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [4, 1000, 1 << 20, 3 * (1 << 20) + 12])
def test_device_copy_exact(n):
    require_gpu()
    import paper_2201_06914_amd as P
    from paper_2201_06914_amd.api import device_copy
    g = torch.Generator(device="cuda").manual_seed(n)
    src = torch.randn(n, device="cuda", generator=g)
    dst = torch.full_like(src, float("nan"))
    device_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    assert P is not None
