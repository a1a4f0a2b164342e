"""The oracle's adjacency build against an independent numpy construction."""
import math

import numpy as np
import pytest

import oracle
import synth


def _numpy_csr(n_rows, a, b, w):
    order = np.lexsort((b, a))            # by a, then b (stable)
    a_s, b_s, w_s = a[order], b[order], w[order]
    rp = np.zeros(n_rows + 1, np.int64)
    np.add.at(rp, a_s + 1, 1)
    return np.cumsum(rp), b_s.astype(np.int32), w_s


@pytest.mark.parametrize("wl_seed", [1, 2])
def test_build_matches_numpy(wl_seed):
    el = synth.chung_lu(300, 500, 4000, 2.1, "lognormal", wl_seed)
    g = oracle.Graph.from_edges(el)
    ex = g.export()
    rp, ci, w = _numpy_csr(el.n_u, el.u, el.v, el.w)
    assert np.array_equal(ex["rp_u"], rp) and np.array_equal(ex["ci_u"], ci) and np.array_equal(ex["w_u"], w)
    rp, ci, w = _numpy_csr(el.n_v, el.v, el.u, el.w)
    assert np.array_equal(ex["rp_v"], rp) and np.array_equal(ex["ci_v"], ci) and np.array_equal(ex["w_v"], w)
    # Eq. (d): within one rounding step of the exactly rounded sum
    for side, n in (("u", el.n_u), ("v", el.n_v)):
        rp, w, ws = ex["rp_" + side], ex["w_" + side], ex["ws_" + side]
        for i in range(n):
            f = math.fsum(w[rp[i]:rp[i + 1]])
            assert abs(ws[i] - f) <= 1e-14 * max(f, 1.0)


def test_duplicates_merged_in_input_order():
    eu = np.array([1, 0, 1, 1, 0], np.int32)
    ev = np.array([2, 0, 2, 0, 0], np.int32)
    w = np.array([0.1, 2.0, 0.2, 5.0, 3.0])
    g = oracle.Graph(2, 3, eu, ev, w)
    ex = g.export()
    assert g.n_e == 3
    assert ex["rp_u"].tolist() == [0, 1, 3]
    assert ex["ci_u"].tolist() == [0, 0, 2]
    assert ex["w_u"].tolist() == [2.0 + 3.0, 5.0, 0.1 + 0.2]
    assert ex["ws_u"].tolist() == [5.0, 5.0 + (0.1 + 0.2)]


@pytest.mark.parametrize("bad", ["range_u", "range_v", "zero", "neg", "nan", "inf"])
def test_build_rejects_bad_input(bad):
    eu = np.array([0, 1], np.int32)
    ev = np.array([0, 1], np.int32)
    w = np.array([1.0, 2.0])
    if bad == "range_u":
        eu[1] = 2
    elif bad == "range_v":
        ev[1] = -1
    elif bad == "zero":
        w[0] = 0.0
    elif bad == "neg":
        w[0] = -1.0
    elif bad == "nan":
        w[0] = np.nan
    else:
        w[0] = np.inf
    with pytest.raises(ValueError):
        oracle.Graph(2, 2, eu, ev, w)
