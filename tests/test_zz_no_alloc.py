"""mlp_loss_noalloc, the variant of mlp_loss whose loss partials live in the
library's static device array, against mlp_loss with a caller-provided
partials buffer: identical dy and loss bit for bit, on two calls in a row
(the second with fewer rows, so stale partials of the first would show), and
rows beyond the static limit refused."""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _p(t):
    return C.c_void_p(t.data_ptr())


def _inputs(B, seed, dev):
    rng = np.random.default_rng(seed)
    y = torch.tensor(rng.standard_normal((B, 16)).astype(np.float32), device=dev)
    t = torch.tensor(rng.standard_normal((B, 2)).astype(np.float32), device=dev)
    m = torch.tensor((rng.uniform(size=(B, 2)) < 0.7).astype(np.float32), device=dev)
    return y, t, m, float(m.sum().item())


def test_noalloc_loss_equals_loss_on_two_calls():
    from paper_1507_06565_amd._lib import check, lib

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s = torch.cuda.current_stream(dev)
    stream = C.c_void_p(s.cuda_stream)
    for B, seed in ((65536, 1), (4096 + 64 * 3, 2)):
        print(f"mlp_loss_noalloc vs mlp_loss: B={B} seed={seed}", file=sys.stderr, flush=True)
        y, t, m, ms = _inputs(B, seed, dev)
        dy_ref = torch.empty_like(y)
        part = torch.empty((B + 255) // 256, dtype=torch.float64, device=dev)
        L_ref = C.c_double()
        check(lib.mlp_loss(_p(y), _p(t), _p(m), B, ms, _p(dy_ref), _p(part), C.byref(L_ref), stream), "mlp_loss")
        dy = torch.full_like(y, float("nan"))
        L = C.c_double(float("nan"))
        check(lib.mlp_loss_noalloc(_p(y), _p(t), _p(m), B, ms, _p(dy), C.byref(L), stream), "mlp_loss_noalloc")
        assert torch.equal(dy, dy_ref)
        assert L.value == L_ref.value, (L.value, L_ref.value)
        # the loss is the masked mean squared error of the two used outputs
        e = ((y[:, :2] - t) * m).double()
        ref = float((e * e).sum().item()) * float(np.float32(1.0 / ms))
        assert abs(L.value / ref - 1) < 1e-6
    # null loss pointer: dy only
    dy2 = torch.empty_like(y)
    check(lib.mlp_loss_noalloc(_p(y), _p(t), _p(m), B, ms, _p(dy2), None, stream), "mlp_loss_noalloc")
    assert torch.equal(dy2, dy_ref)


def test_noalloc_loss_refuses_rows_beyond_its_scratch():
    from paper_1507_06565_amd._lib import lib

    dev = torch.device("cuda:0")
    stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    big = 4194304 + 64
    one = torch.zeros(1, dtype=torch.float32, device=dev)
    L = C.c_double()
    st = lib.mlp_loss_noalloc(_p(one), _p(one), _p(one), big, 1.0, _p(one), C.byref(L), stream)
    assert st == -1
    assert b"limit" in lib.lbm_last_error()
    # not a multiple of 64 rows either
    assert lib.mlp_loss_noalloc(_p(one), _p(one), _p(one), 100, 1.0, _p(one), C.byref(L), stream) == -1
