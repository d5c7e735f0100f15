"""hdc_bundle_noalloc (the bundling entry point for callers that cannot
allocate) against hdc_bundle, through the C ABI: two calls in a row on the
library's per-device scratch, the second on a smaller input, each bit for
bit equal to hdc_bundle with a workspace of its own."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def _inputs(n, nbits, K, seed):
    g = np.random.default_rng(seed)
    W = (nbits + 63) // 64
    bits = g.integers(0, 2, size=(n, W * 64), dtype=np.uint8)
    bits[:, nbits:] = 0
    H = np.packbits(bits, axis=1, bitorder="little").view(np.int64).reshape(n, W)
    y = g.integers(0, K, size=n).astype(np.int32)
    return torch.as_tensor(H).cuda(), torch.as_tensor(y).cuda()


def test_bundle_noalloc_matches_bundle():
    from paper_2606_26547_amd import hdc
    lib = hdc.lib()
    assert lib.hdc_bundle_noalloc_limit_bytes() == 32 << 20
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    # the multi-block grouping path twice (the second call on a smaller
    # input reuses the scratch the first one left behind), then a small
    # bundle (one kernel, no scratch)
    for n, nbits, K in ((40000, 10240, 26), (20000, 4096, 40), (3000, 2048, 10)):
        say("bundle_noalloc", n, nbits, K)
        assert lib.hdc_bundle_workspace_bytes(n, nbits, K) <= lib.hdc_bundle_noalloc_limit_bytes()
        H, y = _inputs(n, nbits, K, n)
        W = H.shape[1]
        C1 = torch.full((K, W), -1, dtype=torch.int64, device="cuda")
        c1 = torch.full((K,), -1, dtype=torch.int32, device="cuda")
        rc = lib.hdc_bundle_noalloc(st, C.c_void_p(H.data_ptr()), n, nbits, W, C.c_void_p(y.data_ptr()), K,
                                    C.c_void_p(C1.data_ptr()), W, C.c_void_p(c1.data_ptr()))
        assert rc == 0, hdc.STATUS[rc]
        C2, c2 = hdc.bundle(H, nbits, y, K)
        torch.cuda.synchronize()
        assert torch.equal(C1, C2)
        assert torch.equal(c1, c2)
        assert int(c1.sum().item()) == n
