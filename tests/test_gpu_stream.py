"""The streaming reference kernels (roofline yardstick): the copies are exact
and the read kernels write one sum per workgroup."""
import pytest

from paper_1402_1763_amd import binding

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)


@pytest.mark.parametrize("mode", ["copy", "copy_nt"])
def test_copies_are_exact(mode):
    import torch
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (3 * 2 ** 20 + 64,), dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    binding.stream_reference(src, dst, mode, 37)       # grid smaller than the buffer: strides
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


@pytest.mark.parametrize("mode", ["read", "read_nt"])
def test_reads_write_one_sum_per_workgroup(mode):
    import torch
    src = torch.zeros(2 ** 20, dtype=torch.int32, device="cuda")
    out = torch.full((128,), 7, dtype=torch.int32, device="cuda")
    binding.stream_reference(src, out, mode, 64)
    torch.cuda.synchronize()
    assert bool((out[:64] == 0).all()) and bool((out[64:] == 7).all())


def test_rejects_bad_arguments():
    import torch
    src = torch.zeros(1000, dtype=torch.int32, device="cuda")
    with pytest.raises(binding.MFError):
        binding.stream_reference(src[1:], src, "copy", 4)      # 3996 bytes, unaligned
    with pytest.raises(binding.MFError):
        binding.stream_reference(src, src, "read", 0)
