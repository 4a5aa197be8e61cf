"""The GPU and the HIP library are visible to the test process."""
import pytest

pytestmark = pytest.mark.gpu


def test_device_and_library_visible():
    import torch
    assert torch.cuda.is_available(), "no ROCm device visible to this process"
    import paper_1412_0659_amd as bh
    t = bh.Tree(16)
    t.close()
