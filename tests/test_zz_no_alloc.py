"""The allocation-free MLP forward entry point (dgmg_mlp_forward_noalloc, work area
in a static device array of the library) against dgmg_mlp_forward with a caller
work buffer, called through the C ABI: two calls in a row, the second with fewer
rows, each bit for bit equal to the buffered entry point (the same kernel and
the same per-row arithmetic; the static array keeps the first call's rows, which
the second must not see); the row limit is enforced."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_1603_02524_amd import dgmg as D  # noqa: E402

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _buffered(lib, params, X):
    B = X.shape[0]
    Y = torch.full((B, D.MLP_OUT), float("nan"), dtype=torch.float32, device="cuda")
    work = torch.empty((B, 2 * D.MLP_HIDDEN), dtype=torch.float32, device="cuda")
    assert lib.dgmg_mlp_forward(_ptr(params), _ptr(X), B, _ptr(Y), _ptr(work), _stream()) == 0
    return Y


def _noalloc(lib, params, X):
    B = X.shape[0]
    Y = torch.full((B, D.MLP_OUT), float("nan"), dtype=torch.float32, device="cuda")
    assert lib.dgmg_mlp_forward_noalloc(_ptr(params), _ptr(X), B, _ptr(Y), _stream()) == 0
    return Y


def test_noalloc_forward_matches_buffered_on_two_calls():
    lib = D.load_library()
    rng = np.random.default_rng(77)
    params = torch.tensor(rng.normal(0, 0.3, D.mlp_param_count()), dtype=torch.float32, device="cuda")
    for B in (D.MLP_NOALLOC_MAX_ROWS, 517):          # the full array, then a smaller input
        X = torch.tensor(rng.uniform(-1, 1, (B, D.MLP_IN)), dtype=torch.float32, device="cuda")
        y_ref = _buffered(lib, params, X)
        y = _noalloc(lib, params, X)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        assert torch.equal(y, y_ref), B


def test_noalloc_forward_limits():
    lib = D.load_library()
    params = torch.zeros(D.mlp_param_count(), dtype=torch.float32, device="cuda")
    B = D.MLP_NOALLOC_MAX_ROWS + 1
    X = torch.zeros((B, D.MLP_IN), dtype=torch.float32, device="cuda")
    Y = torch.zeros((B, D.MLP_OUT), dtype=torch.float32, device="cuda")
    rc = lib.dgmg_mlp_forward_noalloc(_ptr(params), _ptr(X), B, _ptr(Y), _stream())
    assert rc == -1
    assert b"exceed the maximum" in lib.dgmg_last_error(None)
    assert lib.dgmg_mlp_forward_noalloc(_ptr(params), _ptr(X), 0, _ptr(Y), _stream()) == 0
    y = D.mlp_forward_noalloc(params, X[:5])
    assert torch.equal(y, torch.zeros_like(y))       # zero network: outputs are the zero biases
