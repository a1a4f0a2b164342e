"""Pins of the oracle's warm start (signed residues, Lemma 1 for any start,
two-sided bound, fallback). The dense solve of Pi = alpha (I - (1-alpha) P)^-1
is the independent source of truth."""
import numpy as np

import oracle


def test_signed_residue_satisfies_lemma1_for_any_start(small_graph):
    s = small_graph
    g, Pi, alpha = s["g"], s["Pi"], s["wl"].alpha
    rng = np.random.default_rng(1)
    for u in s["sources"][:4]:
        u = int(u)
        for y in (rng.normal(0, 1e-3, g.n_u), Pi[:, u] * (1 + rng.normal(0, 0.5, g.n_u)), np.zeros(g.n_u)):
            r = g.warm_residue(u, alpha, y)
            # pi(., u) = y + Pi r  (Lemma 1 with pi_b = y)
            lhs = y + Pi @ r
            assert np.abs(lhs - Pi[:, u]).max() < 1e-12
    # y = 0 gives the cold start e_u
    r = g.warm_residue(int(s["sources"][0]), alpha, np.zeros(g.n_u))
    e = np.zeros(g.n_u)
    e[int(s["sources"][0])] = 1.0
    assert np.array_equal(r, e)


def test_exact_start_needs_no_push(small_graph):
    s = small_graph
    g, Pi, wl = s["g"], s["Pi"], s["wl"]
    src = s["sources"][:4]
    y0 = np.stack([Pi[:, int(u)] for u in src])
    beta, st, wi = g.approx_bhpp_warm_many(src, wl.alpha, wl.eps, y0)
    for i, u in enumerate(src):
        exact = oracle.bhpp_from_dense(Pi, int(u))
        assert wi[i]["fell_back"] == 0 and wi[i]["res_max"] < 1e-12
        assert np.abs(beta[i] - exact).max() < 1e-11
        assert st[i]["pi_returned"] == 1


def test_two_sided_bound_for_noisy_starts(small_graph):
    s = small_graph
    g, Pi, wl = s["g"], s["Pi"], s["wl"]
    rng = np.random.default_rng(2)
    src = s["sources"][:8]
    starts = []
    for j, u in enumerate(src):
        col = Pi[:, int(u)]
        if j % 2:
            starts.append(col * (1 + rng.normal(0, 0.05, g.n_u)))                 # relative noise
        else:
            starts.append(np.maximum(0, col + rng.normal(0, 2e-5, g.n_u)))       # absolute noise
    y0 = np.stack(starts)
    eps = 1e-6
    beta, st, wi = g.approx_bhpp_warm_many(src, wl.alpha, eps, y0)
    lo = hi = 0.0
    for i, u in enumerate(src):
        assert wi[i]["fell_back"] == 0
        d = oracle.bhpp_from_dense(Pi, int(u)) - beta[i]
        assert np.abs(d).max() <= eps + 1e-12, (i, np.abs(d).max())
        lo, hi = min(lo, d.min()), max(hi, d.max())
    assert lo < 0 < hi          # the guarantee is two-sided: both signs occur


def test_bad_start_falls_back_to_cold(small_graph):
    s = small_graph
    g, Pi, wl = s["g"], s["Pi"], s["wl"]
    src = s["sources"][:3]
    y0 = np.stack([10.0 * Pi[:, int(u)] for u in src[:2]] + [np.zeros(g.n_u)])
    beta, st, wi = g.approx_bhpp_warm_many(src, wl.alpha, wl.eps, y0)
    cold, cst = g.approx_bhpp_many(src, wl.alpha, wl.eps)
    for i in range(3):
        assert wi[i]["fell_back"] == 1
        assert np.array_equal(beta[i], cold[i])
    assert wi[2]["res_l1"] == 1.0 and wi[2]["res_max"] == 1.0   # y = 0 is the cold start exactly


def test_warm_start_cuts_work_when_close(small_graph):
    """A start within 1% of the answer needs fewer sweeps than a cold start."""
    s = small_graph
    g, Pi, wl = s["g"], s["Pi"], s["wl"]
    rng = np.random.default_rng(3)
    src = s["sources"][:6]
    y0 = np.stack([Pi[:, int(u)] * (1 + rng.normal(0, 0.01, g.n_u)) for u in src])
    _, wst, wi = g.approx_bhpp_warm_many(src, wl.alpha, wl.eps, y0)
    _, cst = g.approx_bhpp_many(src, wl.alpha, wl.eps)
    sweeps = lambda x: x["ss_sel_iters"] + x["ss_seq_iters"] + x["pi_sel_iters"] + x["t"]
    assert sum(sweeps(x) for x in wst) < sum(sweeps(x) for x in cst)
    assert all(w["res_l1"] < 0.1 for w in wi)
