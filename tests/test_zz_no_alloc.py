"""pt_mlp_forward_static, the network's forward pass that allocates nothing (its hidden
activations live in a fixed device array of the library), against pt_mlp_forward with a
caller workspace: the same kernels, so the logits must be identical bit for bit.  Two
calls in a row, the second with a smaller batch (the array keeps the first call's
values), then the largest batch and a refused one."""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_forward_static_matches_workspace_forward():
    import torch
    from paper_1004_0023_amd import ptqmc
    torch.cuda.set_device(0)
    L = ptqmc.lib()
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(11)
    params = torch.from_numpy(ptqmc.init_ladder_params(5, out_bias=0.1)).cuda()
    # a non-zero output layer, so every logit depends on both hidden layers
    w3 = slice(128 * 32 + 128 + 128 * 128 + 128, 128 * 32 + 128 + 128 * 128 + 128 + 64 * 128)
    params[w3] = torch.from_numpy(rng.normal(0, 0.1, 64 * 128).astype(np.float32)).cuda()
    for batch in (300, 37, ptqmc.MLP_STATIC_MAX_BATCH):
        print(f"case: pt_mlp_forward_static, batch {batch}", flush=True)
        sys.stdout.flush()
        x = torch.from_numpy(rng.normal(0, 1, (batch, 32)).astype(np.float32)).cuda()
        ws = torch.empty(int(L.pt_mlp_workspace_bytes(batch)), dtype=torch.uint8, device="cuda")
        want = torch.empty((batch, 64), dtype=torch.float32, device="cuda")
        got = torch.full((batch, 64), float("nan"), dtype=torch.float32, device="cuda")
        assert L.pt_mlp_forward(params.data_ptr(), x.data_ptr(), want.data_ptr(), batch,
                                ws.data_ptr(), C.c_void_p(stream)) == 0
        assert L.pt_mlp_forward_static(params.data_ptr(), x.data_ptr(), got.data_ptr(), batch,
                                       C.c_void_p(stream)) == 0
        torch.cuda.synchronize()
        w, g = want.cpu().numpy(), got.cpu().numpy()
        assert np.all(np.isfinite(g))
        assert np.array_equal(w.view(np.uint32), g.view(np.uint32)), batch
        assert float(np.abs(w).max()) > 0.0
    big = ptqmc.MLP_STATIC_MAX_BATCH + 1
    x = torch.zeros((big, 32), dtype=torch.float32, device="cuda")
    out = torch.zeros((big, 64), dtype=torch.float32, device="cuda")
    rc = L.pt_mlp_forward_static(params.data_ptr(), x.data_ptr(), out.data_ptr(), big,
                                 C.c_void_p(stream))
    assert rc == ptqmc.PT_EINVAL
    assert b"PT_MLP_STATIC_MAX_BATCH" in L.pt_last_error()
