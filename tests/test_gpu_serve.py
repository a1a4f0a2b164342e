"""Serving: continuous batching of top-k queries through a resident block
(bhpp_server_*). A request's answer is the same alone and in a mix, equals the
plain batched path's, and meets the error bound against the exact scores."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import paper_2312_06724_amd as bh
    el = synth.chung_lu(20000, 40000, 300000, 2.1, "lognormal", 41)
    src = synth.sample_sources(el, 150, "degree", 12)
    eps = np.random.default_rng(5).choice([1e-5, 1e-6, 1e-7], size=src.size)
    print(f"[gpu] serve: graph 20k x 40k, 300k edges; {src.size} requests", flush=True)
    # the plain batched path gives the bits a server gives (columns keep their positions here)
    G = bh.Graph.from_edges(el, dtype="f32", fixed_width=True)
    return dict(bh=bh, el=el, src=src, eps=eps, G=G)


def drain(S, submit_plan):
    """Feed requests per poll as planned ({poll index: [(tag, src, eps)]}), poll
    until everything finished; returns {tag: (ids, vals, stats)}."""
    res, p = {}, 0
    total = sum(len(v) for v in submit_plan.values())
    while len(res) < total:
        for tag, u, e in submit_plan.get(p, []):
            S.submit(u, e, tag)
        for tag, ids, vals, st in S.poll(stats=True):
            assert tag not in res
            res[tag] = (ids, vals, st)
        p += 1
        assert p < 100000
    return res


def test_staggered_mix_matches_batched_and_alone(setup):
    s = setup
    bh, G, src, eps = s["bh"], s["G"], s["src"], s["eps"]
    k = 20
    S = bh.Server(G, k=k)
    assert S.width == 64
    rng = np.random.default_rng(3)
    plan = {}
    for i in range(src.size):          # arrivals spread over polls, several per poll
        plan.setdefault(int(rng.integers(0, 40)), []).append((i, int(src[i]), float(eps[i])))
    mix = drain(S, plan)
    inf = S.info()
    assert inf["completed"] == src.size and inf["queued"] == 0 and inf["running"] == 0
    # the plain batched path (64-column block, same kernels) gives the same bits
    b = G.query_batch(src, eps, k=k, scores=False)
    bi, bv = b["ids"].cpu().numpy(), b["vals"].cpu().numpy()
    for i in range(src.size):
        assert np.array_equal(mix[i][0], bi[i]), i
        assert np.array_equal(mix[i][1], bv[i]), i
        assert mix[i][2]["steps"] == b["stats"][i]["steps"]
    # alone: one request in an otherwise empty block
    for i in (0, 7, 149):
        alone = drain(S, {0: [(1000 + i, int(src[i]), float(eps[i]))]})[1000 + i]
        assert np.array_equal(alone[0], mix[i][0]) and np.array_equal(alone[1], mix[i][1])
    S.close()


def test_served_results_within_bound(setup):
    s = setup
    bh, G, src, eps = s["bh"], s["G"], s["src"][:24], s["eps"][:24]
    k = 30
    S = bh.Server(G, k=k, max_width=16)
    assert S.width == 16
    res = drain(S, {0: [(i, int(src[i]), float(eps[i])) for i in range(src.size)]})
    S.close()
    ex = oracle.Graph.from_edges(s["el"]).exact_beta_many(src, 0.15, tail=1e-11, nthreads=16)
    for i, u in enumerate(src):
        ids, vals, _ = res[i]
        row = ex[i].copy()
        row[u] = -np.inf
        # each returned value is beta' of that id: within the bound of the exact score
        d = row[ids] - vals.astype(np.float64)
        assert d.min() >= -1e-6 and d.max() <= eps[i] + 1e-6, (i, d.min(), d.max())
        # the k-th exact score is matched within the bound (band rule on ties)
        kth = np.sort(row)[::-1][k - 1]
        assert vals[-1] >= kth - eps[i] - 1e-6


def test_memory_budget_sets_width_and_errors(setup):
    s = setup
    bh, G = s["bh"], s["G"]
    big = bh.Server(G, k=10)
    full = big.info()["resident_bytes"]
    big.close()
    S = bh.Server(G, k=10, mem_budget_bytes=full / 3)
    assert S.width in (8, 16) and S.info()["resident_bytes"] <= full / 3
    with pytest.raises(bh.BhppError):
        S.submit(-1, 1e-6, 0)
    with pytest.raises(bh.BhppError):
        S.submit(0, -1.0, 0)
    with pytest.raises(bh.BhppError):            # launch settings are fixed while a server exists
        G.set_launch_config(G.launch_config())
    assert S.poll() == []                       # nothing queued
    S.close()
    G.set_launch_config(G.launch_config())
    with pytest.raises(bh.BhppError):
        bh.Server(G, k=10, mem_budget_bytes=1000.0)


def test_warm_started_serving(setup):
    """Serving with a model: the structural self term alone (network output
    zero) never falls back; each result meets the bound and matches the same
    request served alone within the tolerance."""
    s = setup
    bh, G, src, eps = s["bh"], s["G"], s["src"][:40], s["eps"][:40]
    M0 = bh.Model(G, seed=1)
    M0.set_params(np.zeros(bh.MODEL_PARAMS, np.float32))
    M0.embed()
    k = 20
    S = bh.Server(G, k=k, model=M0)
    rng = np.random.default_rng(8)
    plan = {}
    for i in range(src.size):
        plan.setdefault(int(rng.integers(0, 20)), []).append((i, int(src[i]), float(eps[i])))
    mix = drain(S, plan)
    inf = S.info()
    assert inf["warm_started"] == src.size and inf["warm_fell_back"] == 0
    assert all(mix[i][2]["fell_back"] == 0 and mix[i][2]["res_l1"] < 1 for i in range(src.size))
    for i in (0, 13, 39):
        alone = drain(S, {0: [(500 + i, int(src[i]), float(eps[i]))]})[500 + i]
        assert np.abs(alone[1].astype(np.float64) - mix[i][1]).max() <= 1e-6
    S.close()
    ex = oracle.Graph.from_edges(s["el"]).exact_beta_many(src[:6], 0.15, tail=1e-11, nthreads=16)
    for i in range(6):
        row = ex[i].copy()
        row[src[i]] = -np.inf
        d = row[mix[i][0]] - mix[i][1].astype(np.float64)
        assert np.abs(d).max() <= eps[i] + 1e-6, (i, np.abs(d).max())
    M0.close()


def test_server_stops_using_a_useless_model(setup):
    s = setup
    bh, G, src = s["bh"], s["G"], s["src"]
    M1 = bh.Model(G, seed=2)
    M1.set_params(np.random.default_rng(3).normal(0, 0.5, bh.MODEL_PARAMS).astype(np.float32))
    M1.embed()
    S = bh.Server(G, k=10, model=M1)
    res = drain(S, {p: [(p * 10 + j, int(src[(p * 10 + j) % src.size]), 1e-5) for j in range(10)] for p in range(40)})
    inf = S.info()
    assert len(res) == 400
    assert inf["warm_fell_back"] >= 32 and inf["warm_started"] < 300
    S.close()
    M1.close()


def test_submit_from_another_thread(setup):
    """Requests submitted by a second thread while the first one polls (the
    server's queue takes submits beside a running poll): each request is
    answered once, with the bits of the plain batched path."""
    import threading
    import time
    s = setup
    bh, G, src, eps = s["bh"], s["G"], s["src"], s["eps"]
    k = 10
    S = bh.Server(G, k=k)
    done = threading.Event()

    def feeder():
        rng = np.random.default_rng(8)
        for i in range(src.size):
            S.submit(int(src[i]), float(eps[i]), i)
            if rng.random() < 0.3:
                time.sleep(0.002)
        done.set()

    t = threading.Thread(target=feeder)
    t.start()
    res, polls = {}, 0
    while not (done.is_set() and len(res) == src.size):
        for tag, ids, vals, st in S.poll(stats=True):
            assert tag not in res
            res[tag] = (ids, vals, st)
        polls += 1
        assert polls < 1000000
    t.join()
    assert S.info()["completed"] == src.size
    b = G.query_batch(src, eps, k=k, scores=False)
    bi, bv = b["ids"].cpu().numpy(), b["vals"].cpu().numpy()
    for i in range(src.size):
        assert np.array_equal(res[i][0], bi[i]), i
        assert np.array_equal(res[i][1], bv[i]), i
    S.close()
