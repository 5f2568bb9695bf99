"""z4c_mlp_backward_noalloc (the backward pass for callers that cannot
allocate: its work buffer is the library's per-GPU device array) against
z4c_mlp_backward with a caller-allocated work buffer, through the C ABI:
two calls in a row, the second with a smaller batch, both bitwise equal
(same kernels, same reduction order); a batch above the array's limit is
rejected."""
import ctypes as C

import numpy as np
import pytest

from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def z():
    import paper_2409_10383_amd as m
    return m


def _ptr(t):
    return C.c_void_p(t.data_ptr())


@pytest.mark.parametrize("seed", [0])
def test_noalloc_backward_equals_backward(seed):
    L = z().lib()
    rng = np.random.default_rng(seed)
    params = torch.tensor(omlp.init(5).astype(np.float32), device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    maxb = 4096
    for B in (maxb, 1500):   # the largest allowed batch, then a smaller one
        X = torch.tensor(rng.standard_normal((B, 16)).astype(np.float32), device="cuda")
        T = torch.tensor(rng.standard_normal(B).astype(np.float32), device="cuda")
        Y = torch.empty(B, dtype=torch.float32, device="cuda")
        cache = torch.empty(B * 128, dtype=torch.float32, device="cuda")
        assert L.z4c_mlp_forward(_ptr(params), _ptr(X), B, _ptr(Y), _ptr(cache), stream) == 0
        g_ref = torch.empty(5313, dtype=torch.float32, device="cuda")
        l_ref = torch.empty(1, dtype=torch.float32, device="cuda")
        work = torch.empty(z().mlp_work_floats(B), dtype=torch.float32, device="cuda")
        assert L.z4c_mlp_backward(_ptr(params), _ptr(X), _ptr(Y), _ptr(T), _ptr(cache), B, _ptr(g_ref),
                                  _ptr(l_ref), _ptr(work), stream) == 0
        g = torch.full((5313,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        assert L.z4c_mlp_backward_noalloc(_ptr(params), _ptr(X), _ptr(Y), _ptr(T), _ptr(cache), B, _ptr(g),
                                          _ptr(loss), stream) == 0
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), B
        assert torch.equal(loss, l_ref), B
        assert torch.isfinite(g).all()
    # above the limit: rejected before any launch
    B = maxb + 1
    X = torch.zeros((B, 16), dtype=torch.float32, device="cuda")
    T = torch.zeros(B, dtype=torch.float32, device="cuda")
    cache = torch.zeros(B * 128, dtype=torch.float32, device="cuda")
    assert L.z4c_mlp_backward_noalloc(_ptr(params), _ptr(X), _ptr(T), _ptr(T), _ptr(cache), B, _ptr(g),
                                      None, stream) == -1
