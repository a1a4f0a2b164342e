"""Shared pytest setup: the ``gpu`` marker and small-graph fixtures."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(scope="session")
def small_graph():
    """The 2k x 3k, 20k-edge power-law graph (DBLP scale) with its dense exact Pi."""
    import oracle
    import synth
    wl = synth.SMALL
    el = wl.graph()
    g = oracle.Graph.from_edges(el)
    Pi, P, ws = oracle.exact_dense(el.n_u, el.n_v, el.u, el.v, el.w, wl.alpha)
    return dict(wl=wl, el=el, g=g, Pi=Pi, P=P, ws=ws, sources=wl.sources(el))


def tiny_random(n_u, n_v, n_e, seed, gamma=2.3, weights="lognormal"):
    import synth
    return synth.chung_lu(n_u, n_v, n_e, gamma, weights, seed)


@pytest.fixture(scope="session")
def uncaptured(request):
    """Context manager that lets output through pytest's capture, so long
    oracle computations inside a test show their own progress lines."""
    import contextlib
    capman = request.config.pluginmanager.getplugin("capturemanager")

    @contextlib.contextmanager
    def cm():
        if capman is None:
            yield
        else:
            with capman.global_and_fixture_disabled():
                yield
    return cm
