"""The MCSP baseline on the GPU (Sec. 3.3, Baselines and Challenges):
MonteCarlo walks drawn from Philox4x32-10 and Walker alias tables plus
SelectivePush with eps/2. The generator's counters and the tables are fixed
by their definitions, so the GPU's walks are the oracle's walks: same end
counts (checked through beta' in FP64 to 1e-12, far below one count's
1/n_r), and beta' within eps of the exact scores."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_mcsp_fp64_equals_oracle_walks(small_graph):
    import paper_2312_06724_amd as bh
    s = small_graph
    G = bh.Graph.from_edges(s["el"], alpha=0.15, dtype="f64", mcsp=True)
    src = s["sources"][:6]
    eps, seed = 2e-2, 20231206
    out = G.query_mcsp(src, eps, seed=seed, k=20)
    S = out["scores"].cpu().numpy()
    assert out["walks"] == oracle.mc_walks(s["el"].n_u, eps / 2, 1e-6)
    for i, u in enumerate(src):
        u = int(u)
        ref, cnt, pib, n_r = s["g"].mcsp(u, 0.15, eps, 1e-6, seed)
        assert n_r == out["walks"]
        assert np.abs(S[i] - ref).max() <= 1e-12, (u, np.abs(S[i] - ref).max())
        beta = s["Pi"][u, :] + s["Pi"][:, u]
        assert np.abs(beta - S[i]).max() <= eps
        rid, _ = oracle.topk_bruteforce(S[i], 20, exclude=u)
        assert np.array_equal(out["ids"][i].cpu().numpy(), rid)
    # a batch of one (sparse SelectivePush steps) gives the same row
    one = G.query_mcsp(src[:1], eps, seed=seed)["scores"][0].cpu().numpy()
    assert np.abs(one - S[0]).max() <= 1e-13
    G.close()


def test_mcsp_fp32_random_graph():
    import paper_2312_06724_amd as bh
    el = synth.chung_lu(3000, 5000, 40000, 2.1, "lognormal", 55)
    g = oracle.Graph.from_edges(el)
    Pi, _, _ = oracle.exact_dense(el.n_u, el.n_v, el.u, el.v, el.w, 0.15)
    G = bh.Graph.from_edges(el, alpha=0.15, dtype="f32", mcsp=True)
    src = synth.sample_sources(el, 5, "degree", 3)
    eps = 2e-2
    out = G.query_mcsp(src, eps, seed=5)
    S = out["scores"].double().cpu().numpy()
    for i, u in enumerate(src):
        ref, _, _, _ = g.mcsp(int(u), 0.15, eps, 1e-6, 5)
        assert np.abs(S[i] - ref).max() <= 2e-6, int(u)
        assert np.abs(Pi[u, :] + Pi[:, u] - S[i]).max() <= eps + 1e-6
    G.close()


def test_mcsp_needs_its_tables(small_graph):
    import paper_2312_06724_amd as bh
    G = bh.Graph.from_edges(small_graph["el"], alpha=0.15, dtype="f64")
    with pytest.raises(bh.BhppError):
        G.query_mcsp(small_graph["sources"][:1], 1e-2)
    G.close()
