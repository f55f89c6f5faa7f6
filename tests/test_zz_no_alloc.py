"""Allocation-free gradient of the closure network (pc_mlp_grad_noalloc,
its scratch a device array of the library) against pc_mlp_grad with a
caller-allocated scratch, through the C ABI: the same kernels and the same
fixed-order reduction, so gradients and losses must be bitwise equal, on two
calls in a row with the second batch smaller than the first (the array keeps
the first call's contents); batches above the maximum are refused."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_noalloc_gradient_equals_scratch_gradient(torch_cuda):
    torch = torch_cuda
    from oracle import mlp as O
    from paper_2202_03215_amd import mlp as M
    net = M.ClosureNet(O.init_params(11), max_batch=16384)
    L = M._lib()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    g = torch.Generator(device="cpu").manual_seed(5)
    for n in (16384, 12000, 1537):
        x = torch.randn(n, 5, generator=g).cuda()
        t = torch.randn(n, 2, generator=g).cuda()
        g_ref, l_ref = net.grad_loss(x, t)
        g_ref, l_ref = g_ref.clone(), l_ref.clone()
        grad = torch.full((M.N_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        rc = L.pc_mlp_grad_noalloc(net.packed.data_ptr(), x.data_ptr(), t.data_ptr(), n, grad.data_ptr(),
                                   loss.data_ptr(), stream)
        assert rc == 0, L.pc_mlp_last_error()
        torch.cuda.synchronize()
        assert torch.isfinite(grad).all() and torch.isfinite(loss).all()
        assert torch.equal(grad, g_ref), (n, float((grad - g_ref).abs().max()))
        assert torch.equal(loss, l_ref), n
    x = torch.zeros(16385, 5, device="cuda")
    t = torch.zeros(16385, 2, device="cuda")
    grad = torch.zeros(M.N_PARAMS, dtype=torch.float32, device="cuda")
    rc = L.pc_mlp_grad_noalloc(net.packed.data_ptr(), x.data_ptr(), t.data_ptr(), 16385, grad.data_ptr(), None,
                               stream)
    assert rc == -1
    assert b"16384" in L.pc_mlp_last_error()
