"""bhpp_topk against the brute-force full sort (bit-exact ids and values)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bh():
    import paper_2312_06724_amd as bh
    return bh


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n,k", [(1, 1), (7, 7), (100, 5), (4096, 100), (4097, 100), (50000, 100), (20000, 1000)])
def test_topk_random(bh, dtype, n, k):
    import torch
    rng = np.random.default_rng(n * 7 + k)
    rows = 3
    x = rng.random((rows, n))
    x[:, ::7] = 0.0                       # many ties at zero
    a = np.arange(1, n, 11)
    b = a + 1
    keep = b < n
    x[:, a[keep]] = x[:, b[keep]]         # and ties between neighbours
    if dtype == "f32":
        x = x.astype(np.float32)
    t = torch.from_numpy(x).cuda()
    ids, vals = bh.topk(t, k)
    for r in range(rows):
        rid, rv = oracle.topk_bruteforce(x[r], k)
        assert np.array_equal(ids[r].cpu().numpy(), rid)
        assert np.array_equal(vals[r].cpu().numpy(), rv.astype(x.dtype))


def test_topk_ties_negzero_exclude(bh):
    import torch
    x = np.array([[0.5, 0.7, 0.7, -0.0, 0.0, 0.1], [0.0, -0.0, 0.0, 0.0, -1.0, 0.0]], dtype=np.float32)
    ids, _ = bh.topk(torch.from_numpy(x).cuda(), 4, exclude=np.array([1, 0], np.int32))
    assert ids[0].cpu().numpy().tolist() == [2, 0, 5, 3]
    assert ids[1].cpu().numpy().tolist() == [1, 2, 3, 5]


def test_topk_all_equal(bh):
    import torch
    x = np.full((2, 9000), 0.25, dtype=np.float64)
    ids, _ = bh.topk(torch.from_numpy(x).cuda(), 33)
    assert ids[0].cpu().numpy().tolist() == list(range(33))
