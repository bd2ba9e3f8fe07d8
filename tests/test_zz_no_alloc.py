"""The no-allocation network forward pass (ctf_cnn_forward_noalloc) against the workspace form
(ctf_cnn_forward) through the C-ABI: the same kernels, so the outputs agree bit for bit, on two
calls in a row (the second smaller, which reuses the scratch array the first one filled), in
float32 and bf16-MFMA modes; and the size limit is refused on the host with CTF_EINVAL."""
import sys

import numpy as np
import pytest

from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu


def _inputs(B, H, W, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(B, 3, H, W)).astype(np.float32)


@pytest.mark.parametrize("bf16", [False, True])
def test_noalloc_forward_equals_workspace_forward(bf16):
    import torch
    from paper_2301_09991_amd import ctf
    theta = ocnn.init_params(11).astype(np.float32)
    theta[-1] = 0.05
    th = torch.as_tensor(theta, device="cuda")
    # the first call nearly fills the array (32 x 32 x 30 = 30720 of 32768 pixels), the second
    # is smaller and reads nothing the first left behind
    for (B, H, W), seed in (((30, 32, 32), 1), ((2, 12, 20), 2)):
        print(f"[no_alloc] bf16={bf16} batch={B} h={H} w={W}", file=sys.stderr, flush=True)
        x = torch.as_tensor(_inputs(B, H, W, seed), device="cuda")
        ref = torch.empty((B, 1, H, W), dtype=torch.float32, device="cuda")
        got = torch.full((B, 1, H, W), float("nan"), dtype=torch.float32, device="cuda")
        ctf.Cnn(B, H, W).forward(th, x, ref, bf16=bf16)
        ctf.cnn_forward_noalloc(th, x, got, bf16=bf16)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        assert torch.isfinite(got).all()


def test_noalloc_forward_refuses_oversized_input():
    import torch
    from paper_2301_09991_amd import ctf
    th = torch.zeros(ctf.cnn_param_count(), dtype=torch.float32, device="cuda")
    # batch * h * w = 182 * 182 = 33124 > 32768: rejected on the host before anything is launched;
    # the buffers still have the full size, so a launch would stay inside them
    B, H, W = 1, 182, 182
    assert B * H * W > ctf.CNN_NOALLOC_MAX_PIXELS
    x = torch.zeros((B, 3, H, W), dtype=torch.float32, device="cuda")
    out = torch.zeros((B, 1, H, W), dtype=torch.float32, device="cuda")
    lib = ctf.load()
    s = torch.cuda.current_stream().cuda_stream
    import ctypes
    rc = lib.ctf_cnn_forward_noalloc(ctypes.c_void_p(th.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), B, H, W, 0, ctypes.c_void_p(s))
    assert rc == ctf.CTF_EINVAL
    assert b"no-allocation limit" in lib.ctf_last_error()
