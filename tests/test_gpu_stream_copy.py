"""The measurement aid lbm_stream_copy (the streaming-kernel bandwidth ceiling of
bench.py): a byte-exact copy, through the C ABI."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2101_01702_amd import lbm
    return lbm.load()


@pytest.mark.parametrize("nbytes", [16, 16 * 1_000_003, 64 << 20])
def test_stream_copy_is_exact(lib, nbytes):
    import torch
    rng = np.random.default_rng(nbytes % 9973)
    src = torch.as_tensor(rng.integers(0, 256, size=nbytes, dtype=np.uint8)).cuda()
    dst = torch.zeros_like(src)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.lbm_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, st) == 0
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
