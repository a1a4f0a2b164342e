"""GPU parity on the 2k x 3k, 20k-edge graph (FP64) and small FP32 graphs.

Reference values come only from the FP64 oracle (dense exact solve, truncated
series, O-method) on the same seeded inputs.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bh():
    import paper_2312_06724_amd as bh
    return bh


@pytest.fixture(scope="module")
def small(small_graph, bh):
    s = small_graph
    el = s["el"]
    print(f"[gpu] building small graph {el.n_u}x{el.n_v} {el.n_e} edges (f64)", flush=True)
    G = bh.Graph.from_edges(el, alpha=0.15, dtype="f64", keep_external=True)
    return dict(s, G=G)


def test_graph_index_bit_exact(small):
    ex = {k: v.cpu().numpy() for k, v in small["G"].export().items()}
    ref = small["g"].export()
    for k in ("rp_u", "ci_u", "rp_v", "ci_v"):
        assert np.array_equal(ex[k], ref[k]), k
    for k in ("w_u", "w_v", "ws_u", "ws_v"):
        assert np.array_equal(ex[k], ref[k]), k   # FP64 sums in the same order


def test_graph_info_and_lambda(small):
    inf = small["G"].info()
    g = small["g"]
    assert inf["n_edges"] == g.n_e
    assert inf["tau"] == g.default_tau(0.15)
    lam_ref = g.lambda_(0.15)
    assert abs(inf["lambda"] - lam_ref) <= 1e-9 * lam_ref
    assert abs(inf["eps_b_ratio"] - g.eps_b(1.0)) <= 1e-15
    assert inf["isolated_u"] == int((g.ws_u == 0).sum())
    # Lemma 4 against the dense solve
    assert inf["lambda"] >= small["Pi"].sum(0).max() - 1e-9


def test_single_queries_theorem3_and_oracle(small):
    G, Pi, g = small["G"], small["Pi"], small["g"]
    eps = 1e-7
    for u in small["sources"]:
        u = int(u)
        print(f"[gpu] single query u={u}", flush=True)
        b, st = G.query(u, eps)
        b = b.cpu().numpy()
        beta = Pi[u, :] + Pi[:, u]
        d = beta - b
        assert d.min() >= -1e-10 and d.max() <= eps + 1e-10, (u, d.min(), d.max())
        ref, _, _, st_ref = g.approx_bhpp(u, 0.15, eps)
        assert np.abs(ref - b).max() <= eps
        # same algorithm, same FP64 arithmetic up to summation order
        assert st["t"] == st_ref["t"] and st["ss_switched"] == st_ref["ss_switched"], (st, st_ref)


def test_batch_equals_single_and_topk_bit_exact(small):
    G, Pi = small["G"], small["Pi"]
    src = small["sources"]
    eps, k = 1e-7, 50
    print(f"[gpu] batch of {len(src)} sources, top-{k}", flush=True)
    out = G.query_batch(src, eps, k=k, exclude_self=True)
    S = out["scores"].cpu().numpy()
    ids = out["ids"].cpu().numpy()
    vals = out["vals"].cpu().numpy()
    for i, u in enumerate(src):
        u = int(u)
        one = G.query(u, eps)[0].cpu().numpy()
        assert np.abs(one - S[i]).max() <= 1e-12
        beta = Pi[u, :] + Pi[:, u]
        d = beta - S[i]
        assert d.min() >= -1e-10 and d.max() <= eps + 1e-10
        rid, rval = oracle.topk_bruteforce(S[i], k, exclude=u)
        assert np.array_equal(ids[i], rid)
        assert np.array_equal(vals[i], rval)
        # against the exact scores: identical sets unless the k-th gap is within eps
        eid, ev = oracle.topk_bruteforce(beta, k + 1, exclude=u)
        if ev[k - 1] - ev[k] > eps + 1e-9:
            assert set(ids[i]) == set(eid[:k])


def test_mixed_eps_in_one_batch(small):
    G, Pi = small["G"], small["Pi"]
    src = small["sources"][:6]
    eps = np.array([1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7])
    S = G.query_batch(src, eps)["scores"].cpu().numpy()
    for i, u in enumerate(src):
        u = int(u)
        d = (Pi[u, :] + Pi[:, u]) - S[i]
        assert d.min() >= -1e-10 and d.max() <= eps[i] + 1e-10


def test_error_codes(small, bh):
    G, g = small["G"], small["g"]
    iso = int(np.nonzero(g.ws_u == 0)[0][0])
    with pytest.raises(bh.BhppError) as e:
        G.query(iso, 1e-6)
    assert e.value.code == -3
    with pytest.raises(bh.BhppError) as e:
        G.query(g.n_u, 1e-6)
    assert e.value.code == -2
    with pytest.raises(bh.BhppError) as e:
        G.query(int(small["sources"][0]), 0.0)
    assert e.value.code == -1
    with pytest.raises(bh.BhppError) as e:
        G.query_batch(small["sources"][:2], 1e-6, k=g.n_u)
    assert e.value.code == -1


def test_degenerate_inputs(small, bh):
    """An empty batch; a graph of one edge, where P = [1], so pi(u, u) = 1 and
    beta(u, u) = 2; a graph without edges (every node isolated); and the
    largest k (every other node, in (score, id) order)."""
    G, g = small["G"], small["g"]
    out = G.query_batch(np.array([], np.int32), 1e-6, k=5)
    assert tuple(out["scores"].shape) == (0, g.n_u) and tuple(out["ids"].shape) == (0, 5)
    assert out["stats"] == []
    one = np.array([0], np.int32)
    for dt, tol in (("f64", 1e-12), ("f32", 1e-6)):
        G1 = bh.Graph(1, 1, one, one, np.array([2.5]), dtype=dt)
        s = G1.query(0, 1e-6)[0].double().cpu().numpy()
        assert 2.0 - 1e-6 - tol <= s[0] <= 2.0 + tol, (dt, s)
        b = G1.query_batch([0, 0], 1e-6, k=1, exclude_self=False)
        assert np.array_equal(b["ids"].cpu().numpy(), [[0], [0]])
        assert np.array_equal(b["scores"].double().cpu().numpy()[:, 0], [s[0], s[0]])
    G0 = bh.Graph(3, 2, np.array([], np.int32), np.array([], np.int32), np.array([]))
    info = G0.info()
    assert info["n_edges"] == 0 and info["isolated_u"] == 3 and info["isolated_v"] == 2
    with pytest.raises(bh.BhppError) as e:
        G0.query(1, 1e-6)
    assert e.value.code == -3
    u = int(small["sources"][0])
    out = G.query_batch([u], 1e-7, k=g.n_u - 1, exclude_self=True)
    S = out["scores"].cpu().numpy()[0]
    rid, rval = oracle.topk_bruteforce(S, g.n_u - 1, exclude=u)
    assert np.array_equal(out["ids"].cpu().numpy()[0], rid)
    assert np.array_equal(out["vals"].cpu().numpy()[0], rval)


def test_build_rejects_bad_input(bh):
    eu = np.array([0, 1], np.int32)
    ev = np.array([0, 1], np.int32)
    with pytest.raises(bh.BhppError) as e:
        bh.Graph(2, 2, eu, ev, np.array([1.0, -1.0]))
    assert e.value.code == -4
    with pytest.raises(bh.BhppError) as e:
        bh.Graph(2, 2, eu, np.array([0, 2], np.int32), np.array([1.0, 1.0]))
    assert e.value.code == -2


def test_closed_form_graphs(bh):
    import pins_lib
    for name, mk in pins_lib.CLOSED_FORMS.items():
        (nu, nv, eu, ev, w), Pi = mk()
        for dt in ("f64", "f32"):
            G = bh.Graph(nu, nv, eu, ev, w, dtype=dt)
            S = G.query_batch(np.arange(nu), 1e-6)["scores"].cpu().numpy()
            for u in range(nu):
                d = (Pi[u, :] + Pi[:, u]) - S[u]
                tol = 1e-10 if dt == "f64" else 2e-6
                assert d.min() >= -tol and d.max() <= 1e-6 + tol, (name, dt, u)


def test_duplicate_edges_merged(bh):
    eu = np.array([1, 0, 1, 1, 0], np.int32)
    ev = np.array([2, 0, 2, 0, 0], np.int32)
    w = np.array([0.1, 2.0, 0.2, 5.0, 3.0])
    G = bh.Graph(2, 3, eu, ev, w, dtype="f64", keep_external=True)
    ex = {k: v.cpu().numpy() for k, v in G.export().items()}
    ref = oracle.Graph(2, 3, eu, ev, w).export()
    for k in ("rp_u", "ci_u", "w_u", "rp_v", "ci_v", "w_v", "ws_u", "ws_v"):
        assert np.array_equal(ex[k], ref[k]), k


def test_graph_index_many_sort_tiles(bh):
    """The build's radix sort over many tiles: 300k edges with repeated
    pairs (input-order FP64 merges), (u, v) and (v, u) keys of 30 bits (four
    digit passes, an even count; the 2k x 3k graph's keys take three), and the
    degree sorts of 20k and 40k nodes (eight passes)."""
    el = synth.chung_lu(20000, 40000, 300000, 2.1, "lognormal", 31)
    rng = np.random.default_rng(12)
    dup = rng.integers(0, el.n_e, 20000)
    eu = np.concatenate([el.u, el.u[dup]]).astype(np.int32)
    ev = np.concatenate([el.v, el.v[dup]]).astype(np.int32)
    w = np.concatenate([el.w, rng.uniform(0.5, 2.0, dup.size)])
    perm = rng.permutation(eu.size)
    eu, ev, w = eu[perm], ev[perm], w[perm]
    print(f"[gpu] build sort: {eu.size} edges over 20k x 40k", flush=True)
    G = bh.Graph(20000, 40000, eu, ev, w, dtype="f64", keep_external=True)
    ex = {k: v.cpu().numpy() for k, v in G.export().items()}
    ref = oracle.Graph(20000, 40000, eu, ev, w).export()
    for k in ("rp_u", "ci_u", "w_u", "rp_v", "ci_v", "w_v", "ws_u", "ws_v"):
        assert np.array_equal(ex[k], ref[k]), k


@pytest.mark.parametrize("reorder", [True, False])
def test_fp32_random_graph_batch(bh, reorder):
    """FP32 values and accumulation; several tiles, split rows and a ragged
    last source block (70 sources = 64 + 6)."""
    el = synth.chung_lu(3000, 5000, 60000, 2.1, "lognormal", 77)
    g = oracle.Graph.from_edges(el)
    src = synth.sample_sources(el, 70, "uniform", 5)
    G = bh.Graph.from_edges(el, dtype="f32", reorder=reorder)
    eps = 1e-6
    print(f"[gpu] fp32 random graph reorder={reorder}", flush=True)
    out = G.query_batch(src, eps, k=20)
    S = out["scores"].cpu().numpy().astype(np.float64)
    ex = g.exact_beta_many(src, 0.15, tail=1e-12)
    d = ex - S
    assert d.min() >= -1e-6 and d.max() <= eps + 1e-6, (d.min(), d.max())
    ids = out["ids"].cpu().numpy()
    for i, u in enumerate(src):
        rid, _ = oracle.topk_bruteforce(out["scores"][i].cpu().numpy(), 20, exclude=int(u))
        assert np.array_equal(ids[i], rid)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sparse_frontier_steps_match_dense(small, bh, dtype):
    """One-source queries take SS-Push's selective iterations as sparse
    frontier pushes; the result and every phase counter match the dense
    sweeps of the same graph (up to summation order), and the bound holds."""
    el, Pi = small["el"], small["Pi"]
    Gs = bh.Graph.from_edges(el, dtype=dtype)
    Gd = bh.Graph.from_edges(el, dtype=dtype, sparse=False)
    eps = 1e-7 if dtype == "f64" else 1e-6
    tol = 1e-12 if dtype == "f64" else 1e-6
    for u in small["sources"][:8]:
        u = int(u)
        bs, ss = Gs.query(u, eps)
        bd, sd = Gd.query(u, eps)
        bs, bd = bs.double().cpu().numpy(), bd.double().cpu().numpy()
        assert np.abs(bs - bd).max() <= tol, u
        for key in ("ss_sel_iters", "ss_seq_iters", "pi_sel_iters", "t", "ss_switched", "pi_returned"):
            assert ss[key] == sd[key], (u, key, ss, sd)
        assert abs(ss["np_ss"] - sd["np_ss"]) <= 1e-9 * max(1.0, sd["np_ss"])
        beta = Pi[u, :] + Pi[:, u]
        d = beta - bs
        assert d.min() >= -tol and d.max() <= eps + tol


def test_eps_b_split_keeps_the_bound(small, bh):
    """Theorem 3 holds for any eps_b in (0, eps): queries with a set split stay
    in [beta - eps, beta], follow the oracle run with the same eps_b phase for
    phase, and the tuner keeps one of its candidates."""
    el, Pi, g = small["el"], small["Pi"], small["g"]
    G = bh.Graph.from_edges(el, dtype="f64")
    paper = G.info()["eps_b_ratio"]
    eps = 1e-7
    src = small["sources"][:6]
    for ratio in (0.05, 0.9):
        G.set_eps_b_ratio(ratio)
        assert abs(G.info()["eps_b_ratio"] - ratio) < 1e-15
        out = G.query_batch(src, eps)
        S = out["scores"].cpu().numpy()
        for i, u in enumerate(src):
            u = int(u)
            d = Pi[u, :] + Pi[:, u] - S[i]
            assert d.min() >= -1e-10 and d.max() <= eps + 1e-10, (ratio, u)
            _, _, _, st = g.approx_bhpp(u, 0.15, eps, eps_b=ratio * eps)
            assert out["stats"][i]["t"] == st["t"] and out["stats"][i]["ss_switched"] == st["ss_switched"]
    best, ms, gm, sw = G.tune_eps_b(small["sources"][6:], eps, [0.05, 0.2, paper], curve=True)
    assert best in (0.05, 0.2, paper) and np.all(ms > 0) and np.all(sw > 0)
    # Fig. 1's shape: gamma does not grow with eps_b (a larger eps_b leaves more residue)...
    # here measured on the same sources: gamma at 0.05 <= gamma at the paper's ratio
    assert gm[0] <= gm[2] + 1e-12
    G.set_eps_b_ratio(0.0)
    assert G.info()["eps_b_ratio"] == paper
    with pytest.raises(bh.BhppError):
        G.set_eps_b_ratio(1.0)


def test_single_direction_hpp(small, bh):
    """pi(u, .) by PI-Push alone (Theorem 2) and pi(., u) by SS-Push alone
    (Theorem 1), each within [pi - eps, pi] of the dense solve; batches of
    one (sparse steps) and of many give the same values."""
    G, Pi = small["G"], small["Pi"]
    src = small["sources"][:10]
    for eps in (1e-4, 1e-7):
        fwd, fst = G.query_hpp(src, eps, "forward")
        bwd, bst = G.query_hpp(src, eps, "backward")
        F, B = fwd.cpu().numpy(), bwd.cpu().numpy()
        for i, u in enumerate(src):
            u = int(u)
            df = Pi[u, :] - F[i]
            db = Pi[:, u] - B[i]
            assert df.min() >= -1e-10 and df.max() <= eps + 1e-10, ("fwd", eps, u, df.min(), df.max())
            assert db.min() >= -1e-10 and db.max() <= eps + 1e-10, ("bwd", eps, u, db.min(), db.max())
            assert fst[i]["ss_sel_iters"] == 0 and bst[i]["pi_sel_iters"] == 0 and bst[i]["t"] == 0
        one, _ = G.query_hpp(src[:1], eps, "backward")
        assert np.abs(one.cpu().numpy()[0] - B[0]).max() <= 1e-12
    with pytest.raises(bh.BhppError):
        G.query_hpp(src, 1e-6, "forward", alpha=2.0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_hub_lds_is_bit_neutral(small, bh, dtype, monkeypatch):
    """One-source gathers read the hub slice of their vector from an LDS copy;
    the values are the same as the global ones, so dense one-source queries
    give the same bits with the copy on or off."""
    el = small["el"]
    monkeypatch.setenv("BHPP_TUNE", "hub=0")
    G0 = bh.Graph.from_edges(el, dtype=dtype, sparse=False)
    monkeypatch.setenv("BHPP_TUNE", "hub=1")
    G1 = bh.Graph.from_edges(el, dtype=dtype, sparse=False)
    for u in small["sources"][:6]:
        b0, s0 = G0.query(int(u), 1e-7)
        b1, s1 = G1.query(int(u), 1e-7)
        assert s0 == s1
        assert np.array_equal(b0.cpu().numpy().view(np.uint8), b1.cpu().numpy().view(np.uint8)), int(u)
    G0.close()
    G1.close()
