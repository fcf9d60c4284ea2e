"""The allocation-free orthonormalisation (snect_orthonormalize_noalloc,
fixed per-device scratch) against the allocating one (snect_orthonormalize)
through the C ABI: identical bits on two calls in a row, the second on a
smaller problem, so the second call runs on scratch the first one filled."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _factors(sn, ts):
    f = sn.Factors()
    f.A, f.B, f.C, f.G = (t.data_ptr() for t in ts)
    return f


def _draw(seed, dims, ranks):
    import torch
    rng = np.random.default_rng(seed)
    U = [rng.standard_normal((d, r)).astype(np.float32) * 0.5 for d, r in zip(dims, ranks)]
    G = rng.standard_normal(ranks).astype(np.float32)
    return [torch.tensor(a, device="cuda") for a in U + [G]]


def test_noalloc_equals_allocating_orthonormalize():
    import torch
    import paper_1711_08095_amd as sn
    lib = sn.load()
    fn = lib.snect_orthonormalize_noalloc
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p] + [ctypes.c_int32] * 6 + [ctypes.POINTER(sn.Factors)]
    ctx = sn.Context(0)
    for n, (dims, ranks) in enumerate((((4500, 14000, 5), (20, 20, 5)), ((300, 257, 7), (10, 3, 7)))):
        print(f"no-alloc QR call {n}: dims {dims} ranks {ranks}", flush=True)
        a = _draw(100 + n, dims, ranks)
        b = [t.clone() for t in a]
        fa = _factors(sn, a)
        rc = lib.snect_orthonormalize(ctx.h, *dims, *ranks, ctypes.byref(fa))
        assert rc == 0
        fb = _factors(sn, b)
        rc = fn(ctx.h, *dims, *ranks, ctypes.byref(fb))
        assert rc == 0, lib.snect_last_error(ctx.h)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x, y)
        for q in b[:3]:
            qq = q.double().cpu().numpy()
            np.testing.assert_allclose(qq.T @ qq, np.eye(qq.shape[1]), atol=1e-5)
    # the fixed scratch holds 32 x 32 Gram matrices: larger ranks are refused
    big = _draw(7, (40, 40, 40), (33, 2, 2))
    rc = fn(ctx.h, 40, 40, 40, 33, 2, 2, ctypes.byref(_factors(sn, big)))
    assert rc == -4
    # a rank-deficient factor is reported, as by the allocating call
    A = torch.zeros((20, 3), device="cuda")
    A[:, 0] = 1.0
    A[:, 2] = torch.arange(20, device="cuda", dtype=torch.float32)
    rest = [torch.randn((30, 2), device="cuda"), torch.randn((4, 2), device="cuda"),
            torch.randn((3, 2, 2), device="cuda")]
    rc = fn(ctx.h, 20, 30, 4, 3, 2, 2, ctypes.byref(_factors(sn, [A] + rest)))
    assert rc == -1
    ctx.close()
