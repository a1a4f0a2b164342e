"""bhpp_topk_noalloc (working memory in a static device array, no
allocation) against bhpp_topk through the C ABI: two calls in a row on the
same stream, the second with a smaller input, in both dtypes; the results
must be bit-identical (index work), and the limits are rejected before any
work is enqueued."""
import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _call(fn, scores, k, exclude, dt):
    import torch
    import paper_2312_06724_amd as bh
    rows, n = scores.shape
    ids = torch.full((rows, k), -7, dtype=torch.int32, device="cuda")
    vals = torch.full((rows, k), -7.0, dtype=scores.dtype, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fn(scores.data_ptr(), rows, n, k, exclude.data_ptr() if exclude is not None else None, dt,
            ids.data_ptr(), vals.data_ptr(), stream)
    assert rc == 0, bh.BhppError(rc, "top-k")
    return ids, vals


def test_topk_noalloc_matches_topk():
    import torch
    import paper_2312_06724_amd as bh
    L = bh.load_library()
    rng = np.random.default_rng(31)
    for dt, tdt in ((bh.DTYPE_F32, torch.float32), (bh.DTYPE_F64, torch.float64)):
        # the second call is smaller than the first (rows, length and k)
        for rows, n, k in ((64, 200_003, 4096), (5, 9_001, 100)):
            # few distinct values (ties broken by id), zeros of both signs
            a = rng.integers(0, 50, size=(rows, n)).astype(np.float64) * 1e-3
            a[:, ::7] = -0.0
            sc = torch.from_numpy(a).to(device="cuda", dtype=tdt)
            ex = torch.from_numpy(rng.integers(0, n, size=rows).astype(np.int32)).cuda()
            for exclude in (ex, None):
                i1, v1 = _call(L.bhpp_topk, sc, k, exclude, dt)
                i2, v2 = _call(L.bhpp_topk_noalloc, sc, k, exclude, dt)
                torch.cuda.synchronize()
                assert torch.equal(i1, i2)
                assert torch.equal(v1.view(torch.int32 if dt == bh.DTYPE_F32 else torch.int64),
                                   v2.view(torch.int32 if dt == bh.DTYPE_F32 else torch.int64))
            # and one row against the brute-force sort
            rid, _ = oracle.topk_bruteforce(a[-1].astype(np.float32 if dt == bh.DTYPE_F32 else np.float64), k,
                                            exclude=-1)
            assert np.array_equal(i2[-1].cpu().numpy(), rid)
    # limits: more rows or a larger k than the static array holds
    sc = torch.zeros((65, 5000), dtype=torch.float32, device="cuda")
    ids = torch.empty((65, 8), dtype=torch.int32, device="cuda")
    vals = torch.empty((65, 8), dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.bhpp_topk_noalloc(sc.data_ptr(), 65, 5000, 8, None, bh.DTYPE_F32, ids.data_ptr(), vals.data_ptr(),
                               s) == -7
    assert L.bhpp_topk_noalloc(sc.data_ptr(), 1, 5000, 4097, None, bh.DTYPE_F32, ids.data_ptr(), vals.data_ptr(),
                               s) == -7
