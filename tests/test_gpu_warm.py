"""Learned warm start on the GPU: the MFMA GEMM's lane layout, the node
features and the network's gradients against the FP64 oracle, training, and
warm-started queries (signed residues) against the exact scores and against
the oracle's warm start from the same start."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp

pytestmark = pytest.mark.gpu


def bf16_tensor(torch, a):
    """FP32 numpy -> device bf16 tensor (round to nearest even) and the rounded values as float64."""
    r = mlp.bf16_round(a)
    t = torch.from_numpy(r.astype(np.float32)).to("cuda").to(torch.bfloat16)
    return t.view(torch.int16), r


@pytest.mark.parametrize("M,N,K,ta,tb", [(64, 64, 32, 0, 0), (100, 70, 50, 0, 0), (37, 129, 200, 1, 0),
                                         (130, 33, 64, 0, 1), (65, 65, 300, 1, 1),
                                         # 16-byte staging: k contiguous with a ragged K, rows contiguous
                                         (64, 48, 104, 0, 1), (72, 40, 100, 1, 0)])
def test_gemm_lane_layout(M, N, K, ta, tb):
    import torch
    import paper_2312_06724_amd as bh
    print(f"[gpu] gemm {M}x{N}x{K} ta={ta} tb={tb}", flush=True)
    rng = np.random.default_rng(M * 7 + N)
    A = rng.normal(0, 1, (K, M) if ta else (M, K)).astype(np.float32)
    B = rng.normal(0, 1, (N, K) if tb else (K, N)).astype(np.float32)
    At, Ar = bf16_tensor(torch, A)
    Bt, Br = bf16_tensor(torch, B)
    C = bh.gemm_bf16(At, Bt, bool(ta), bool(tb)).cpu().numpy().astype(np.float64)
    ref = (Ar.T if ta else Ar) @ (Br.T if tb else Br)
    assert np.abs(C - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())


@pytest.fixture(scope="module")
def small():
    import paper_2312_06724_amd as bh
    wl = synth.SMALL
    el = wl.graph()
    print("[gpu] warm: 2k x 3k graph", flush=True)
    G = bh.Graph.from_edges(el, alpha=wl.alpha, dtype="f64", fixed_width=True)
    g = oracle.Graph.from_edges(el)
    Pi, _, _ = oracle.exact_dense(el.n_u, el.n_v, el.u, el.v, el.w, wl.alpha)
    return dict(bh=bh, wl=wl, el=el, G=G, g=g, Pi=Pi, src=wl.sources(el))


def test_features_match_oracle(small):
    M = small["bh"].Model(small["G"], seed=3)
    F = M.features().cpu().numpy().astype(np.float64)
    ref = mlp.features(small["g"])
    assert np.abs(F - ref).max() < 1e-5
    M.close()


def test_gradients_match_oracle(small):
    s = small
    M = s["bh"].Model(s["G"], seed=4)
    rng = np.random.default_rng(5)
    theta = M.params().astype(np.float64)
    theta += rng.normal(0, 0.05, theta.size)          # non-zero biases too
    M.set_params(theta.astype(np.float32))
    theta32 = M.params().astype(np.float64)
    c, sigma = M.scales()
    g = s["g"]
    live = np.nonzero(g.deg_u > 0)[0]
    src = s["src"][:8]
    cand = np.concatenate([src[:3], rng.choice(np.setdiff1d(live, src), 37, replace=False)]).astype(np.int32)
    Pi = s["Pi"]
    ws = g.ws_u
    T = np.stack([Pi[int(u), cand] for u in src])      # pi(u, x)
    loss, grad = M.loss_grad(src, cand, T)
    # oracle: same BF16 inputs and weights (biases stay FP32, as on the GPU)
    X = mlp.bf16_round(M.features().cpu().numpy())
    th = theta32.copy()
    o = 0
    for _ in range(2):
        for shp in mlp.SHAPES:
            n = int(np.prod(shp))
            if len(shp) == 2:
                th[o:o + n] = mlp.bf16_round(th[o:o + n].astype(np.float32))
            o += n
    prior = mlp.self_prior(g, s["wl"].alpha)
    E = np.where(cand[None, :] == src[:, None], prior[src][:, None], 0.0)
    lo, go = mlp.loss_and_grad(th, X[src], X[cand], ws[cand], T, c, sigma, E)
    assert abs(loss - lo) <= 2e-2 * lo, (loss, lo)
    o = 0
    for t in range(2):
        for shp in mlp.SHAPES:
            n = int(np.prod(shp))
            a, b = grad[o:o + n].astype(np.float64), go[o:o + n]
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-300)
            assert rel < 5e-2 and cos > 0.998, (t, shp, rel, cos)
            o += n
    M.close()


def value_lists(rows, live, rng, top=64, rand=64):
    """Per source: its top entries plus entries at random nodes, with values."""
    ids, vals = [], []
    for b in rows:
        t = np.argsort(-b, kind="stable")[:top]
        r = rng.choice(live, rand, replace=False)
        i = np.unique(np.concatenate([t, r]))
        i = np.concatenate([i, np.full(top + rand - i.size, -1)])
        ids.append(i)
        vals.append(np.where(i >= 0, b[np.maximum(i, 0)], 0.0))
    return np.array(ids, dtype=np.int32), np.array(vals, dtype=np.float32)


def test_training_reduces_loss(small):
    s = small
    M = s["bh"].Model(s["G"], seed=6)
    g, Pi = s["g"], s["Pi"]
    live = np.nonzero(g.deg_u > 0)[0]
    train = live[::3].astype(np.int32)
    # lists of exact beta (the plain path's output would do the same)
    ids, vals = value_lists([oracle.bhpp_from_dense(Pi, int(u)) for u in train], live, np.random.default_rng(1))
    # a fixed held-out batch: 16 other sources, all their listed pairs known
    held = live[1::3][:16].astype(np.int32)
    hid, hval = value_lists([oracle.bhpp_from_dense(Pi, int(u)) for u in held], live, np.random.default_rng(2))
    cand = np.unique(hid[hid >= 0]).astype(np.int32)
    T = np.full((held.size, cand.size), np.nan)
    ws = g.ws_u
    for i, u in enumerate(held):
        k = hid[i] >= 0
        T[i, np.searchsorted(cand, hid[i][k])] = Pi[int(u), hid[i][k]]
    before, _ = M.loss_grad(held, cand, T, want_grad=False)
    losses = M.train(train, ids, vals, steps=300, batch_src=16, batch_cand=2048, lr=5e-4)
    after, _ = M.loss_grad(held, cand, T, want_grad=False)
    print(f"[gpu] held-out loss {before:.4g} -> {after:.4g}", flush=True)
    assert np.all(np.isfinite(losses)) and after < 0.7 * before
    M.close()


def test_caller_starts_match_oracle_warm(small):
    """Warm starts given directly (the exact column with relative noise): the
    GPU's signed-residue run and the oracle's agree, and both are within eps
    of the exact scores on both sides."""
    s = small
    G, g, Pi, wl = s["G"], s["g"], s["Pi"], s["wl"]
    rng = np.random.default_rng(8)
    src = s["src"][:12]
    ws = g.ws_u
    eps = 1e-7
    # starts in forward form: p(u, x) ~ pi(u, x); rows 10, 11 are useless (fall back)
    P = np.stack([Pi[int(u)] * (1 + rng.normal(0, 0.05, g.n_u)) for u in src])
    P[10] *= 30.0
    P[11] = 0.0
    out = G.query_batch(src, eps, starts=P, k=wl.k)
    S = out["scores"].cpu().numpy()
    # the oracle from the same start (backward form y(x) = ws(u)/ws(x) p(u, x))
    inv = np.divide(1.0, ws, out=np.zeros_like(ws), where=ws > 0)
    Y0 = np.stack([ws[int(u)] * inv * P[i].astype(np.float32).astype(np.float64) for i, u in enumerate(src)])
    ob, ost, owi = g.approx_bhpp_warm_many(src, wl.alpha, eps, Y0)
    lo = 0.0
    for i, u in enumerate(src):
        ex = oracle.bhpp_from_dense(Pi, int(u))
        d = ex - S[i]
        assert np.abs(d).max() <= eps + 1e-9, (i, np.abs(d).max())
        lo = min(lo, d.min())
        w = out["warm"][i]
        assert w["fell_back"] == owi[i]["fell_back"], i
        assert abs(w["res_l1"] - owi[i]["res_l1"]) <= 1e-9 * max(1.0, owi[i]["res_l1"])
        assert np.abs(S[i] - ob[i]).max() <= eps, i
    assert out["warm"][10]["fell_back"] == 1 and out["warm"][11]["fell_back"] == 1
    assert sum(w["fell_back"] for w in out["warm"][:10]) == 0
    assert lo < 0          # warm starts can land above the exact score
    # a fallen-back query is the cold query, bit for bit (same block width)
    cold = G.query_batch(src, eps, k=wl.k)
    assert np.array_equal(cold["scores"].cpu().numpy()[10:12], S[10:12])


def test_model_warm_queries_within_bound(small):
    s = small
    G, g, Pi, wl = s["G"], s["g"], s["Pi"], s["wl"]
    M = s["bh"].Model(G, seed=7)
    live = np.nonzero(g.deg_u > 0)[0]
    ids, vals = value_lists([oracle.bhpp_from_dense(Pi, int(u)) for u in live], live, np.random.default_rng(2))
    M.train(live.astype(np.int32), ids, vals, steps=600, batch_src=16, batch_cand=2048, lr=5e-4)
    M.embed()
    src = s["src"]
    out = G.query_batch(src, wl.eps, model=M, k=wl.k)
    S = out["scores"].cpu().numpy()
    for i, u in enumerate(src):
        d = oracle.bhpp_from_dense(Pi, int(u)) - S[i]
        assert np.abs(d).max() <= wl.eps + 1e-9, (i, np.abs(d).max())
    r = np.array([w["res_l1"] for w in out["warm"]])
    fb = np.array([w["fell_back"] for w in out["warm"]])
    assert np.all((r >= 1) <= (fb == 1))
    print(f"[gpu] warm res_l1 median {np.median(r):.3f}, fallback {fb.mean():.2f}", flush=True)
    M.close()


@pytest.fixture(scope="module")
def trained():
    """A 20k x 40k graph (FP32): training data from the plain GPU path, then
    the same evaluation queries cold, warm from the structural self term alone
    (the network's output set to zero: the no-network ablation) and warm from
    the trained network."""
    import paper_2312_06724_amd as bh
    import torch
    el = synth.chung_lu(20000, 40000, 300000, 2.1, "lognormal", 51)
    G = bh.Graph.from_edges(el, dtype="f32")
    live = np.nonzero(el.degrees_u() > 0)[0]
    rng = np.random.default_rng(6)
    train = synth.sample_sources(el, 1024, "uniform", 17)
    evals = np.setdiff1d(synth.sample_sources(el, 80, "uniform", 18), train)[:48]
    ids, vals = [], []
    for i in range(0, train.size, 64):
        chunk = train[i:i + 64]
        out = G.query_batch(chunk, 1e-6, k=64, exclude_self=False, scores=True, stats=False)
        r = torch.from_numpy(rng.choice(live, (chunk.size, 64))).to("cuda")
        rv = torch.gather(out["scores"], 1, r.long())
        ii = torch.cat([out["ids"], r.int()], 1).cpu().numpy()
        vv = torch.cat([out["vals"], rv], 1).cpu().numpy()
        for a, b in zip(ii, vv):
            _, keep = np.unique(a, return_index=True)
            a2 = np.full(128, -1, np.int32)
            b2 = np.zeros(128, np.float32)
            a2[:keep.size], b2[:keep.size] = a[keep], b[keep]
            ids.append(a2)
            vals.append(b2)
    print(f"[gpu] training data: {train.size} sources", flush=True)
    cold = G.query_batch(evals, 1e-6, k=50)
    M0 = bh.Model(G, seed=9)
    M0.set_params(np.zeros(bh.MODEL_PARAMS, np.float32))
    M0.embed()
    prior_only = G.query_batch(evals, 1e-6, k=50, model=M0)
    M = bh.Model(G, seed=9)
    losses = M.train(train, np.array(ids), np.array(vals), steps=1500, batch_src=32, batch_cand=4096, lr=5e-4)
    M.embed()
    warm = G.query_batch(evals, 1e-6, k=50, model=M)
    sw = lambda o: float(np.mean([x["steps"] for x in o["stats"]]))
    rep = {}
    for name, o in (("prior only", prior_only), ("trained", warm)):
        r = np.array([w["res_l1"] for w in o["warm"]])
        fb = np.array([w["fell_back"] for w in o["warm"]])
        rep[name] = dict(res_l1_median=round(float(np.median(r)), 3), fallback=float(fb.mean()), sweeps=sw(o))
    print(f"[gpu] loss {losses[:50].mean():.4g} -> {losses[-50:].mean():.4g}; sweeps cold {sw(cold):.1f}; "
          f"{rep}", flush=True)
    yield dict(bh=bh, el=el, G=G, evals=evals, cold=cold, prior_only=prior_only, warm=warm, M=M, M0=M0, rep=rep,
               sweeps=sw)
    M.close()
    M0.close()
    G.close()


def test_trained_network_against_cold_start(trained):
    """Cold, self-term-only and trained starts all stay within eps of the
    exact scores; a start is dropped exactly when its residual is no better
    than the cold start's; the self term alone always beats the cold start."""
    t = trained
    ex = oracle.Graph.from_edges(t["el"]).exact_beta_many(t["evals"][:6], 0.15, tail=1e-11, nthreads=16)
    for name in ("cold", "prior_only", "warm"):
        S = t[name]["scores"][:6].double().cpu().numpy()
        assert np.abs(ex - S).max() <= 1e-6 + 1e-6, name
    for name in ("prior_only", "warm"):
        r = np.array([w["res_l1"] for w in t[name]["warm"]])
        fb = np.array([w["fell_back"] for w in t[name]["warm"]])
        assert np.all((r >= 1) <= (fb == 1))
    assert t["rep"]["prior only"]["fallback"] == 0.0


@pytest.mark.xfail(strict=False, reason="negative result on random power-law graphs: the trained towers' starts "
                                        "leave a larger signed residue than the structural self term alone (the "
                                        "residue amplifies the prediction error by about 1/alpha); recorded in the "
                                        "design notes with the curve against training-set size")
def test_trained_network_beats_self_term(trained):
    """What the trained network gains over the method without it: a smaller
    median residual than the self-term-only start, starts that are kept, and
    fewer sweeps than that ablation."""
    rep = trained["rep"]
    assert rep["trained"]["res_l1_median"] < rep["prior only"]["res_l1_median"]
    assert rep["trained"]["fallback"] < 1.0
    assert rep["trained"]["sweeps"] < rep["prior only"]["sweeps"]


def test_model_predictions_are_the_warm_starts(trained):
    """bhpp_model_predict exports the start each warm query uses: giving the
    exported starts back through bhpp_query_batch_start reproduces the model's
    warm queries bit for bit (residuals, fallbacks, scores)."""
    t = trained
    p = t["M0"].predict(t["evals"])
    assert p.shape == (t["evals"].size, t["el"].n_u) and float(p.min()) >= 0.0
    a = t["G"].query_batch(t["evals"], 1e-6, k=50, starts=p)
    b = t["prior_only"]
    assert np.array_equal(a["scores"].cpu().numpy(), b["scores"].cpu().numpy())
    assert [w["fell_back"] for w in a["warm"]] == [w["fell_back"] for w in b["warm"]]
    assert np.allclose([w["res_l1"] for w in a["warm"]], [w["res_l1"] for w in b["warm"]], rtol=0, atol=0)
