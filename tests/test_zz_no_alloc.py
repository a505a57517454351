"""The allocation-free apply (cm_apply_noalloc) against cm_apply, through the
C ABI: two calls in a row on one GPU, the second with a smaller input (the
fixed scratch array keeps the first call's contents), and the size limit."""
import ctypes as C

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

K0 = 2 * np.pi


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _noalloc(torch, op, opname, X):
    from paper_1412_1756_amd import _lib
    Y = torch.empty_like(X)
    st = _lib.lib().cm_apply_noalloc(op._h, _lib.OPS[opname], C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()),
                                     X.stride(0), X.shape[1], _lib.CM_C128 if X.dtype == torch.complex128 else
                                     _lib.CM_C64, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, Y


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_noalloc_apply_matches_apply_on_two_calls(torch_cuda):
    torch = torch_cuda
    from paper_1412_1756_amd import Operator, _lib
    # first call: 7,680 unknowns, 4 levels, 8 columns, FP32 far field (27 MiB of workspace)
    V, F = workloads.icosphere(4, 1.0)
    big = Operator(V, F, K0, nlv=4, d0=5.0, interp_p=10, max_cols=16)
    Xb = torch.tensor(workloads.cn01_block(big.N, 8, 100), dtype=torch.complex64, device="cuda")
    print("noalloc call 1: N=7680 ncols=8 c64 op Z", flush=True)
    st, Yn = _noalloc(torch, big, "Z", Xb)
    assert st == _lib.CM_OK, _lib.lib().cm_last_error()
    Ya = big.apply(Xb, "Z")
    torch.cuda.synchronize()
    e1 = _relerr(Yn.cpu().numpy(), Ya.cpu().numpy())
    print(f"  rel diff to cm_apply {e1:.3e}, bitwise equal {bool(torch.equal(Yn, Ya))}", flush=True)
    assert e1 < 1e-6
    # the size limit: 16 FP64 columns need 108 MiB, more than the fixed array
    Xw = torch.zeros((big.N, 16), dtype=torch.complex128, device="cuda")
    st, _ = _noalloc(torch, big, "Z", Xw)
    assert st == _lib.CM_E_BADARG
    assert "exceeds" in _lib.lib().cm_last_error().decode()
    # second call, smaller: 1,920 unknowns, 3 levels, 3 columns, FP64, R x
    V, F = workloads.icosphere(3, 0.5)
    small = Operator(V, F, K0, nlv=3, d0=6.0, interp_p=12, max_cols=4)
    Xs = torch.tensor(workloads.cn01_block(small.N, 3, 200), dtype=torch.complex128, device="cuda")
    print("noalloc call 2: N=1920 ncols=3 c128 op R", flush=True)
    st, Yn = _noalloc(torch, small, "R", Xs)
    assert st == _lib.CM_OK, _lib.lib().cm_last_error()
    Ya = small.apply(Xs, "R")
    torch.cuda.synchronize()
    e2 = _relerr(Yn.cpu().numpy(), Ya.cpu().numpy())
    print(f"  rel diff to cm_apply {e2:.3e}, bitwise equal {bool(torch.equal(Yn, Ya))}", flush=True)
    assert e2 < 1e-13
    # and the first handle again after the second (stale scratch contents)
    st, Yn = _noalloc(torch, big, "Z", Xb)
    assert st == _lib.CM_OK
    torch.cuda.synchronize()
    e3 = _relerr(Yn.cpu().numpy(), big.apply(Xb, "Z").cpu().numpy())
    print(f"noalloc call 3 (first handle again): rel diff {e3:.3e}", flush=True)
    assert e3 < 1e-6
