"""The seeded input generator: determinism and the promised structure."""
import numpy as np

import synth


def test_deterministic_and_distinct():
    a = synth.chung_lu(500, 700, 5000, 2.1, "lognormal", 9)
    b = synth.chung_lu(500, 700, 5000, 2.1, "lognormal", 9)
    c = synth.chung_lu(500, 700, 5000, 2.1, "lognormal", 10)
    assert np.array_equal(a.u, b.u) and np.array_equal(a.v, b.v) and np.array_equal(a.w, b.w)
    assert not np.array_equal(a.u, c.u)
    keys = a.u.astype(np.int64) * a.n_v + a.v
    assert np.unique(keys).size == a.n_e
    assert a.u.min() >= 0 and a.u.max() < 500 and a.v.min() >= 0 and a.v.max() < 700
    assert np.all(a.w > 0) and np.all(a.w.astype(np.float32).astype(np.float64) == a.w)


def test_int_weights_and_power_law():
    el = synth.SMALL.graph()
    assert el.n_e == 20000
    assert set(np.unique(el.w)) <= set(range(1, 11))
    d = el.degrees_u()
    assert d.max() > 20 * d.mean()          # hubs exist
    assert (d == 0).sum() > 0               # and isolated nodes


def test_sources():
    el = synth.SMALL.graph()
    s = synth.sample_sources(el, 16, "uniform", 3)
    assert np.unique(s).size == 16 and np.all(el.degrees_u()[s] > 0)
    s2 = synth.sample_sources(el, 200, "degree", 3)
    assert el.degrees_u()[s2].mean() > el.degrees_u()[el.degrees_u() > 0].mean()
