"""The allocation-free gradient entry point against the one with a caller
work area, through the C ABI: two calls in a row on fresh data, the second
with fewer samples, bit for bit."""
import ctypes

import numpy as np
import pytest

gpu = pytest.mark.gpu


@gpu
def test_mlp_grad_noalloc_matches_work_area_entry_point():
    import torch
    from paper_1212_0204_amd import _lib
    from paper_1212_0204_amd.mlp import ClosureNet, init_params
    L = _lib.lib()
    net = ClosureNet(init_params(21))
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(31)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    for n, use_idx in ((5000, False), (1234, True)):
        print("CASE noalloc n =", n, "idx" if use_idx else "rows", flush=True)
        x = torch.tensor(rng.standard_normal((n + 17, 37)).astype(np.float32), device="cuda")
        t = torch.tensor(rng.standard_normal((n + 17, 4)).astype(np.float32), device="cuda")
        idx = torch.tensor(rng.integers(0, n + 17, n).astype(np.int32), device="cuda") if use_idx else None
        g_ref = torch.empty(net.nparam, dtype=torch.float32, device="cuda")
        l_ref = torch.empty(1, dtype=torch.float32, device="cuda")
        nb = L.hofks_mlp_grad_work_bytes(n)
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        assert L.hofks_mlp_grad(vp(net.packed), vp(x), vp(t), vp(idx) if use_idx else None, n,
                                vp(g_ref), vp(l_ref), vp(work), nb, stream) == 0
        g = torch.full((net.nparam,), float("nan"), dtype=torch.float32, device="cuda")
        l = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        assert L.hofks_mlp_grad_noalloc(vp(net.packed), vp(x), vp(t), vp(idx) if use_idx else None,
                                        n, vp(g), vp(l), stream) == 0
        torch.cuda.synchronize()
        assert torch.isfinite(g).all() and torch.isfinite(l).all()
        assert torch.equal(g, g_ref) and torch.equal(l, l_ref)
    # bad arguments are refused before anything runs
    assert L.hofks_mlp_grad_noalloc(vp(net.packed), vp(x), vp(t), None, 0, vp(g), vp(l), stream) == -1
