"""pwa_mlp_forward_noalloc (the forward pass with its buffers in the
library's fixed device array) against pwa_mlp_forward with a caller-owned
workspace: same kernels, same inputs, so the outputs must be identical.
Two calls in a row, the second with a smaller batch, then a batch beyond the
array's limit, which must be refused."""

import ctypes
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

DIMS = (1024, 512, 512, 48)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_forward_noalloc_matches_forward():
    from paper_2403_09225_amd import _lib as L
    from paper_2403_09225_amd.learned_start import MLP
    net = MLP(DIMS, seed=3)
    lib = net.lib
    gen = np.random.Generator(np.random.PCG64(17))
    for B in (200, 37):
        say(f"[no-alloc] forward batch {B}")
        x = torch.tensor(gen.random((B, DIMS[0])), dtype=torch.float32, device="cuda")
        ref = net.forward(x)
        y = torch.full((B, DIMS[3]), float("nan"), dtype=torch.float32, device="cuda")
        code = lib.pwa_mlp_forward_noalloc(ctypes.byref(net.dims), _ptr(net.w), _ptr(net.wbf),
                                           _ptr(x), B, _ptr(y), _stream())
        assert code == L.PWA_OK, L.status_str(code) if hasattr(L, "status_str") else code
        torch.cuda.synchronize()
        assert torch.equal(y, ref), float((y - ref).abs().max())
    # beyond the fixed array (4 MiB of forward buffers: 336 rows at these
    # widths) the call is refused before any launch
    x = torch.zeros((352, DIMS[0]), dtype=torch.float32, device="cuda")
    y = torch.empty((352, DIMS[3]), dtype=torch.float32, device="cuda")
    assert lib.pwa_mlp_forward_noalloc(ctypes.byref(net.dims), _ptr(net.w), _ptr(net.wbf), _ptr(x),
                                       352, _ptr(y), _stream()) == L.PWA_E_WORKSPACE
    code = lib.pwa_mlp_forward_noalloc(ctypes.byref(net.dims), _ptr(net.w), _ptr(net.wbf), _ptr(x),
                                       336, _ptr(y), _stream())
    assert code == L.PWA_OK
    torch.cuda.synchronize()
    assert torch.equal(y[:336], net.forward(x[:336]))
