"""Queue-fed query blocks (many uneven sources), graph replay and launch settings."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import paper_2312_06724_amd as bh
    el = synth.chung_lu(20000, 40000, 300000, 2.1, "lognormal", 31)
    src = synth.sample_sources(el, 200, "degree", 8)       # uneven: hubs and tail nodes
    rng = np.random.default_rng(4)
    eps = rng.choice([1e-4, 1e-5, 1e-6], size=src.size)
    print(f"[gpu] graph 20k x 40k, 300k edges; {src.size} degree-proportional sources", flush=True)
    G = bh.Graph.from_edges(el, dtype="f32")
    Gf = bh.Graph.from_edges(el, dtype="f32", fixed_width=True)
    g = oracle.Graph.from_edges(el)
    return dict(bh=bh, el=el, src=src, eps=eps, G=G, Gf=Gf, g=g)


def test_many_uneven_sources_against_exact(setup):
    s = setup
    out = s["G"].query_batch(s["src"], s["eps"], k=20)
    S = out["scores"].double().cpu().numpy()
    ex = s["g"].exact_beta_many(s["src"], 0.15, tail=1e-11, nthreads=16)
    d = ex - S
    tol = 1e-6
    assert d.min() >= -tol, d.min()
    assert np.all(d.max(axis=1) <= s["eps"] + tol), (d.max(axis=1) - s["eps"]).max()
    ids = out["ids"].cpu().numpy()
    Sf = out["scores"].cpu().numpy()
    for i, u in enumerate(s["src"]):
        rid, _ = oracle.topk_bruteforce(Sf[i], 20, exclude=int(u))
        assert np.array_equal(ids[i], rid)
    st = out["stats"]
    steps = np.array([x["steps"] for x in st])
    assert steps.min() > 0 and steps.max() > steps.min()    # uneven work per source


def test_alone_and_in_mix_identical(setup):
    """With a fixed block width, a query's result does not depend on the other
    queries sharing its block (64 columns), nor on its column or position."""
    s = setup
    src, eps = s["src"], s["eps"]
    a = s["Gf"].query_batch(src, eps, k=10)
    perm = np.random.default_rng(9).permutation(src.size)
    b = s["Gf"].query_batch(src[perm], eps[perm], k=10)
    Sa, Sb = a["scores"].cpu().numpy(), b["scores"].cpu().numpy()
    assert np.array_equal(Sa[perm], Sb)
    assert np.array_equal(a["ids"].cpu().numpy()[perm], b["ids"].cpu().numpy())
    # one query with 63 others vs with 63 different others
    c = s["Gf"].query_batch(np.concatenate([src[:1], src[100:163]]), np.concatenate([eps[:1], eps[100:163]]))
    assert np.array_equal(c["scores"][0].cpu().numpy(), Sa[0])


def test_narrowing_blocks_match_fixed_width(setup):
    """A batch that packs its running sources into the low columns as others
    finish gives every source the bits of a block that never packs: each
    column is computed independently of its position (a full queue-fed run,
    one block that packs once, and a 40-source batch)."""
    s = setup
    for sl in (slice(0, 64), slice(0, 200), slice(10, 50)):
        src, eps = s["src"][sl], s["eps"][sl]
        a = s["G"].query_batch(src, eps, k=10)
        b = s["Gf"].query_batch(src, eps, k=10)
        assert np.array_equal(a["scores"].cpu().numpy(), b["scores"].cpu().numpy()), sl
        assert np.array_equal(a["ids"].cpu().numpy(), b["ids"].cpu().numpy()), sl
        assert a["stats"] == b["stats"], sl


def test_launch_settings_do_not_change_results(setup):
    s = setup
    G = s["G"]
    src, eps = s["src"][:70], s["eps"][:70]
    base = G.query_batch(src, eps)["scores"].cpu().numpy()
    cfg0 = G.launch_config()
    for te, inf, nt, gr in [(256, 4, 0, 0), (1024, 16, 1, 1), (512, 8, 0, 1)]:
        G.set_launch_config(dict(tile_edges=te, inflight=inf, nt_stream=nt, graphs=gr))
        S = G.query_batch(src, eps)["scores"].cpu().numpy()
        assert np.abs(S - base).max() <= 1e-6
    best = G.autotune()
    assert best["tile_edges"] in (512, 1024, 2048, 4096) and best["inflight"] in (4, 8, 16)
    S = G.query_batch(src, eps)["scores"].cpu().numpy()
    assert np.abs(S - base).max() <= 1e-6
    G.set_launch_config(cfg0)


def test_fused_select_matches_select_pass(setup, monkeypatch):
    """In 64-column blocks gather A applies the push rule itself (S = y/ws for
    the pushed x) instead of reading a copy written by a select pass: same
    products in the same order, so the same bits. 200 sources refill the
    columns, so sweeps in which columns start a query (y = e_src taken in the
    gather) are mixed in; PISP's batch adds the mid-query residue restart.
    The fused gather's rows come by buffer loads by default; bufa=0 takes
    global loads: same bits."""
    s = setup
    monkeypatch.setenv("BHPP_TUNE", "fuse=0")
    G0 = s["bh"].Graph.from_edges(s["el"], dtype="f32", fixed_width=True)
    monkeypatch.setenv("BHPP_TUNE", "bufa=0")
    G1 = s["bh"].Graph.from_edges(s["el"], dtype="f32", fixed_width=True)
    monkeypatch.delenv("BHPP_TUNE")
    G0.set_launch_config(s["Gf"].launch_config())
    G1.set_launch_config(s["Gf"].launch_config())
    src, eps = s["src"], s["eps"]
    a = s["Gf"].query_batch(src, eps, k=10)
    for Gx in (G0, G1):
        b = Gx.query_batch(src, eps, k=10)
        assert np.array_equal(a["scores"].cpu().numpy(), b["scores"].cpu().numpy())
        assert np.array_equal(a["ids"].cpu().numpy(), b["ids"].cpu().numpy())
        assert a["stats"] == b["stats"]
    a = s["Gf"].query_batch(src[:80], 1e-5, k=10, method="pisp")
    b = G0.query_batch(src[:80], 1e-5, k=10, method="pisp")
    assert np.array_equal(a["scores"].cpu().numpy(), b["scores"].cpu().numpy())
    assert np.array_equal(a["ids"].cpu().numpy(), b["ids"].cpu().numpy())
    assert a["stats"] == b["stats"]


def test_async_admission_matches_draining_rounds(setup, monkeypatch):
    """Batches of more than 64 sources admit new queries without draining the
    stream (the host reads copies of the column states a chunk behind and
    queues extraction, top-k and admission behind the running sweeps). With
    chunks of 1, 2 or 8 sweeps, packing on or off, every query gets the bits
    and counters of the draining export rounds: a query's arithmetic does not
    depend on when it is admitted or which column it takes."""
    s = setup
    src, eps = s["src"], s["eps"]
    monkeypatch.setenv("BHPP_TUNE", "async=0")
    Gh = s["bh"].Graph.from_edges(s["el"], dtype="f32", fixed_width=True)
    Gh.set_launch_config(s["Gf"].launch_config())
    base = Gh.query_batch(src, eps, k=10)
    Gh.close()
    for chunk, fixed in ((1, False), (2, True), (8, False)):
        monkeypatch.setenv("BHPP_TUNE", f"async=1,chunk={chunk}")
        Ga = s["bh"].Graph.from_edges(s["el"], dtype="f32", fixed_width=fixed)
        Ga.set_launch_config(s["Gf"].launch_config())
        out = Ga.query_batch(src, eps, k=10)
        assert np.array_equal(out["scores"].cpu().numpy(), base["scores"].cpu().numpy()), chunk
        assert np.array_equal(out["ids"].cpu().numpy(), base["ids"].cpu().numpy()), chunk
        assert out["stats"] == base["stats"], chunk
        # without scores or top-k outputs only the statistics come back
        st = Ga.query_batch(src, eps, k=0, scores=False)["stats"]
        assert st == base["stats"], chunk
        Ga.close()
    monkeypatch.delenv("BHPP_TUNE")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_fused_update_matches_update_pass(setup, monkeypatch, dtype):
    """In 64-column blocks the U-side gather applies the update itself: a
    tile's row sums stay in LDS and each entry of y and ACC is computed from
    the same operands in the same order as the update pass, so the scores and
    top-k match bit for bit. Only the order of the FP64 per-source sums
    changes (the gather's tiles instead of the update's blocks): counters are
    equal and the sums agree to rounding."""
    s = setup
    src, eps = s["src"][:150], s["eps"][:150]
    monkeypatch.setenv("BHPP_TUNE", "upd=0")
    G0 = s["bh"].Graph.from_edges(s["el"], dtype=dtype, fixed_width=True)
    monkeypatch.setenv("BHPP_TUNE", "upd=1")
    G1 = s["bh"].Graph.from_edges(s["el"], dtype=dtype, fixed_width=True)
    monkeypatch.delenv("BHPP_TUNE")
    G1.set_launch_config(G0.launch_config())
    a = G1.query_batch(src, eps, k=10)
    b = G0.query_batch(src, eps, k=10)
    assert np.array_equal(a["scores"].cpu().numpy(), b["scores"].cpu().numpy())
    assert np.array_equal(a["ids"].cpu().numpy(), b["ids"].cpu().numpy())
    for x, y in zip(a["stats"], b["stats"]):
        assert x.keys() == y.keys()
        for key in x:
            if isinstance(x[key], float):
                assert abs(x[key] - y[key]) <= 1e-12 * max(1.0, abs(y[key])), key
            else:
                assert x[key] == y[key], key
    G0.close()
    G1.close()


def test_admission_order_does_not_change_results(setup, monkeypatch):
    """Queues admit the longest expected queries first (smaller eps, then lower
    degree); with the caller's order instead every query gets the same bits and
    counters, and outputs stay in the caller's order either way."""
    s = setup
    src, eps = s["src"], s["eps"]
    monkeypatch.setenv("BHPP_TUNE", "order=0")
    G0 = s["bh"].Graph.from_edges(s["el"], dtype="f32")
    monkeypatch.delenv("BHPP_TUNE")
    G0.set_launch_config(s["G"].launch_config())
    a = s["G"].query_batch(src, eps, k=10)
    b = G0.query_batch(src, eps, k=10)
    assert np.array_equal(a["scores"].cpu().numpy(), b["scores"].cpu().numpy())
    assert np.array_equal(a["ids"].cpu().numpy(), b["ids"].cpu().numpy())
    assert a["stats"] == b["stats"]
    G0.close()
