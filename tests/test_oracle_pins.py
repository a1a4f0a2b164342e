"""Pins of the FP64 oracle against facts other than itself (CPU only)."""
import numpy as np
import pytest

import oracle
from pins_lib import (pin_closed_forms, pin_dense_invariants, pin_eps_b, pin_golden_gamma,
                      pin_golden_rounds, pin_lambda, pin_lemma1_and_mass, pin_mcsp, pin_pisp, pin_power_mass,
                      pin_random_walk, pin_series_agree, pin_theorems)


def test_closed_forms():
    assert pin_closed_forms() == []


def test_random_walk_simulation():
    assert pin_random_walk() == []


def test_dense_invariants(small_graph):
    assert pin_dense_invariants(small_graph["Pi"], small_graph["ws"]) == []


def test_series_forward_backward_lemma3(small_graph):
    s = small_graph
    assert pin_series_agree(s["g"], s["sources"], s["wl"].alpha) == []


def test_series_match_dense(small_graph):
    s = small_graph
    for u in s["sources"][:4]:
        u = int(u)
        assert np.allclose(s["g"].hpp_forward(u, 0.15, 1e-14), s["Pi"][u, :], atol=1e-12)
        assert np.allclose(s["g"].hpp_backward(u, 0.15, 1e-14), s["Pi"][:, u], atol=1e-12)


def test_theorems_every_source(small_graph):
    s = small_graph
    out, seen = pin_theorems(s["g"], s["Pi"], s["sources"], s["wl"].alpha, [1e-2, 1e-4, 1e-7])
    assert out == []
    # every branch of Algorithms 3-4 was exercised by these queries
    assert any(st["ss_switched"] for st in seen) and any(not st["ss_switched"] for st in seen)
    assert any(st["t"] > 0 for st in seen)


def test_pi_push_early_return_branch():
    """Eq. (fwd-eps) ending PI-Push (no power iterations) is exercised by the
    closed-form graphs, where the theorem bands were checked above."""
    from pins_lib import CLOSED_FORMS
    hits = 0
    for mk in CLOSED_FORMS.values():
        (nu, nv, eu, ev, w), _ = mk()
        g = oracle.Graph(nu, nv, eu, ev, w)
        hits += sum(g.approx_bhpp(u, 0.15, 1e-2)[3]["pi_returned"] for u in range(nu))
    assert hits > 0


@pytest.mark.parametrize("k", [0, 1, 5])
def test_lemma1_every_iteration(small_graph, k):
    s = small_graph
    assert pin_lemma1_and_mass(s["g"], s["Pi"], int(s["sources"][k]), 0.15, 1e-7) == []


def test_lambda_lemma4(small_graph):
    s = small_graph
    assert pin_lambda(s["g"], s["Pi"], 0.15) == []


def test_power_iteration_mass(small_graph):
    assert pin_power_mass(small_graph["g"], 0.15) == []


def test_golden_gamma_fig1(small_graph):
    s = small_graph
    assert pin_golden_gamma(s["g"], s["sources"], 0.15) == []


def test_golden_power_rounds():
    assert pin_golden_rounds() == []


def test_eps_b_closed_form():
    assert pin_eps_b() == []


def test_gamma_decreases_with_eps_b(small_graph):
    """Sec. 4.3: as eps_b decreases and SS-Push progresses, gamma decreases (Fig. 1)."""
    g = small_graph["g"]
    for u in small_graph["sources"][:4]:
        gam = []
        for eb in (0.5, 0.1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
            gam.append(g.approx_bhpp(int(u), 0.15, 2 * eb, eps_b=eb)[3]["gamma"])
        assert all(b <= a + 1e-12 for a, b in zip(gam, gam[1:])), gam


def test_random_graphs_theorem3():
    """Theorem 3 on several random graphs, including ones with isolated nodes
    and hub-heavy degree sequences."""
    import synth
    for seed, (nu, nv, ne, gam) in enumerate([(50, 80, 300, 2.1), (200, 40, 900, 2.5),
                                               (120, 300, 400, 2.05)]):
        el = synth.chung_lu(nu, nv, ne, gam, "lognormal", 90 + seed)
        g = oracle.Graph.from_edges(el)
        Pi, _, ws = oracle.exact_dense(nu, nv, el.u, el.v, el.w, 0.15)
        assert pin_dense_invariants(Pi, ws) == []
        src = np.nonzero(ws > 0)[0][:10]
        out, _ = pin_theorems(g, Pi, src, 0.15, [1e-3, 1e-8])
        assert out == []
        assert pin_lambda(g, Pi, 0.15) == []


def test_isolated_source_rejected():
    import synth
    el = synth.chung_lu(40, 60, 50, 2.1, "int10", 4)
    g = oracle.Graph.from_edges(el)
    iso = np.nonzero(g.ws_u == 0)[0]
    assert iso.size > 0
    with pytest.raises(ValueError, match="isolated"):
        g.approx_bhpp(int(iso[0]), 0.15, 1e-4)


def test_topk_bruteforce_hand_example():
    # ties broken by ascending id, -0 ranks as +0, excluded id left out
    s = np.array([0.5, 0.7, 0.7, -0.0, 0.0, 0.1])
    ids, vals = oracle.topk_bruteforce(s, 4, exclude=1)
    assert ids.tolist() == [2, 0, 5, 3]
    ids, _ = oracle.topk_bruteforce(s, 6, exclude=-1)
    assert ids.tolist() == [1, 2, 0, 5, 3, 4]


def test_block_series_matches_single_and_dense(small_graph):
    """The block form of the exact series gives each source's single-source
    series bit for bit (the same products in the same order), and so matches
    the dense solve; an isolated source keeps alpha e_u, as the single form."""
    import synth
    s = small_graph
    src = np.asarray(s["sources"][:7])
    blk = s["g"].hpp_forward_block(src, 0.15, 1e-12, nthreads=3)
    for i, u in enumerate(src):
        one = s["g"].hpp_forward(int(u), 0.15, 1e-12)
        assert np.array_equal(blk[i], one), int(u)
        assert np.allclose(blk[i], s["Pi"][int(u), :], atol=1e-11)
    el = synth.chung_lu(40, 60, 50, 2.1, "int10", 4)
    g = oracle.Graph.from_edges(el)
    iso = np.nonzero(g.ws_u == 0)[0][:1]
    live = np.nonzero(g.ws_u > 0)[0][:3]
    both = np.concatenate([live, iso, live[:1]])
    blk = g.hpp_forward_block(both, 0.15, 1e-10)
    for i, u in enumerate(both):
        assert np.array_equal(blk[i], g.hpp_forward(int(u), 0.15, 1e-10)), int(u)
    ex = g.exact_beta_many(live, 0.15, tail=1e-10)
    ex0 = g.exact_beta_many(live, 0.15, tail=1e-10, block=0)
    assert np.array_equal(ex, ex0)


def test_pisp_bands_every_source(small_graph):
    """PISP (Sec. 3.3) on every source of the 2k x 3k graph at three eps."""
    s = small_graph
    assert pin_pisp(s["g"], s["Pi"], s["sources"], s["wl"].alpha) == []


def test_pisp_closed_forms():
    """PISP on the hand-built graphs: the bands against the closed forms."""
    from pins_lib import CLOSED_FORMS
    for mk in CLOSED_FORMS.values():
        (nu, nv, eu, ev, w), Pi = mk()
        g = oracle.Graph(nu, nv, eu, ev, w)
        assert pin_pisp(g, Pi, range(nu), 0.15, (1e-2, 1e-5)) == []


def test_bounded_sample_counts_the_work(small_graph):
    """The CPU baseline's bounded sample (Algorithm 5 stopped after a number
    of push iterations) counts the edges touched: uncapped, that is the
    statistics' n_p of both sub-algorithms plus 2|E| per PowerIteration round;
    capped, a part of it."""
    s = small_graph
    g, src = s["g"], s["sources"][:4]
    full = g.approx_bhpp_sample(src, 0.15, 1e-7, 100000)
    _, st = g.approx_bhpp_many(src, 0.15, 1e-7)
    for i in range(len(src)):
        want = st[i]["np_ss"] + st[i]["np_pi"] + 2 * g.n_e * st[i]["t"]
        assert abs(full[i] - want) <= 1e-9 * want
    part = g.approx_bhpp_sample(src, 0.15, 1e-7, 3)
    assert np.all(part > 0) and np.all(part < full)


def test_mcsp_generator_alias_walks_and_band(small_graph):
    """MCSP (Sec. 3.3): Philox known answers, alias tables, the walk count,
    walk frequencies against the dense solve and the eps band."""
    s = small_graph
    assert pin_mcsp(s["g"], s["Pi"], s["sources"], s["wl"].alpha) == []


def test_mc_walks_on_the_walk_graph():
    """The walks against the random-walk definition on a small irregular graph
    (asymmetric P): frequencies within 5 standard errors of the dense row."""
    from pins_lib import walk_graph
    nu, nv, eu, ev, w = walk_graph()
    g = oracle.Graph(nu, nv, eu, ev, w)
    Pi, _, _ = oracle.exact_dense(nu, nv, eu, ev, w, 0.15)
    n_r = 400000
    for u in range(nu):
        cnt, _ = g.mc_counts(u, 0.15, n_r, 99 + u)
        sig = np.sqrt(Pi[u] * (1 - Pi[u]) / n_r)
        assert np.all(np.abs(cnt / n_r - Pi[u]) <= 5 * sig + 1e-9), u
