"""lbm_stream_probe (the streaming-ceiling measurement aid): it copies the
population bytes of nbricks bricks exactly, in both layouts, and times them."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("grouped", [0, 1])
def test_stream_probe_copies_exactly(grouped):
    import torch

    from paper_1507_06565_amd._lib import check, lib

    nb = 1000  # 62 full workgroups of 16 bricks and a ragged one of 8
    n = nb * 64 * 19
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.full((n + 64,), -1.0, dtype=torch.float32, device="cuda")  # 64 guard values after the end
    s = torch.cuda.current_stream()
    ms = C.c_double()
    check(lib.lbm_stream_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nb, grouped, 3,
                               C.c_void_p(s.cuda_stream), C.byref(ms)), "lbm_stream_probe")
    assert ms.value > 0.0
    d = dst.cpu().numpy()
    assert np.array_equal(d[:n], src.cpu().numpy())
    assert np.all(d[n:] == -1.0)
