"""Pins of the FP64 network and feature reference (oracle/mlp.py): closed
forms of GELU, BF16 rounding, hand-computed features, and the analytic
gradient against central finite differences."""
import math

import numpy as np

import oracle
from oracle import mlp


def test_gelu_closed_forms():
    z = np.array([0.0, 1.0, -1.0, 10.0, -10.0])
    phi1 = 0.5 * (1 + math.erf(1 / math.sqrt(2)))          # Phi(1) = 0.8413447460685429
    assert abs(phi1 - 0.8413447460685429) < 1e-15
    g = mlp.gelu(z)
    assert g[0] == 0.0 and abs(g[1] - phi1) < 1e-15 and abs(g[2] + (1 - phi1)) < 1e-15
    assert abs(g[3] - 10.0) < 1e-12 and abs(g[4]) < 1e-12
    d = mlp.gelu_grad(z)
    assert d[0] == 0.5 and abs(d[1] - (phi1 + math.exp(-0.5) / math.sqrt(2 * math.pi))) < 1e-15
    # derivative against a central difference
    h = 1e-6
    zz = np.linspace(-4, 4, 17)
    fd = (mlp.gelu(zz + h) - mlp.gelu(zz - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(zz)).max() < 1e-8


def test_bf16_rounding():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 3.0e-3], dtype=np.float32)
    r = mlp.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1 + 2 ** -6 and r[3] == -2.5   # ties to even
    assert abs(r[4] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_features_hand_example():
    # U0 - V0 (w 1), U0 - V1 (w 3), U1 - V1 (w 2); U2 isolated
    g = oracle.Graph(3, 2, np.array([0, 0, 1]), np.array([0, 1, 1]), np.array([1.0, 3.0, 2.0]))
    F = mlp.features(g)
    b0, b1 = mlp.bucket(np.array([0, 1]))
    assert np.all(F[2] == 0)
    assert F[0, 0] == 1 and abs(F[0, 1] - math.log(3) / 8) < 1e-15 and abs(F[0, 2] - math.log(4) / 8) < 1e-15
    # neighbour log-degrees: d(V0) = 1, d(V1) = 2
    assert abs(F[0, 3] - (0.25 * math.log(2) + 0.75 * math.log(3)) / 8) < 1e-15
    assert abs(F[1, 3] - math.log(3) / 8) < 1e-15
    assert abs(F[0, 4 + b0] - (0.25 if b0 != b1 else 1.0)) < 1e-15
    assert abs(F[1, 4 + b1] - 1.0) < 1e-15
    assert np.all(mlp.bucket(np.arange(1000)) < mlp.N_BUCKETS)


def test_feature_buckets_sum_to_one(small_graph):
    F = mlp.features(small_graph["g"])
    live = small_graph["g"].deg_u > 0
    assert np.abs(F[live, 4:].sum(1) - 1).max() < 1e-12
    assert np.all(F[~live] == 0)


def init(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, mlp.N_PARAMS) / np.sqrt(np.concatenate(
        [np.full(int(np.prod(s)), s[0] if len(s) == 2 else 1.0) for s in mlp.SHAPES] * 2))


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = init(1)
    Xu, Xx = rng.normal(0, 1, (3, mlp.IN)), rng.normal(0, 1, (5, mlp.IN))
    ws = rng.uniform(1, 5, 5)
    T = rng.uniform(0, 1e-2, (3, 5))
    T[1, 2] = T[0, 4] = np.nan                     # unknown targets are left out
    c, sigma = 0.05, 1e-4
    loss, grad = mlp.loss_and_grad(theta, Xu, Xx, ws, T, c, sigma)
    # the loss is what predict() implies
    p = mlp.predict(theta, Xu, Xx, ws, c)
    k = np.isfinite(T)
    assert abs(loss - ((p[k] - T[k]) ** 2 / (T[k] + sigma)).mean()) < 1e-12 * max(1.0, loss)
    # coordinates in every block of both towers
    offs, o = [], 0
    for _ in range(2):
        for s in mlp.SHAPES:
            n = int(np.prod(s))
            offs += list(o + rng.choice(n, size=min(4, n), replace=False))
            o += n
    h = 1e-6
    for i in offs:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, Xu, Xx, ws, T, c, sigma)[0] - mlp.loss_and_grad(tm, Xu, Xx, ws, T, c, sigma)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, grad[i])


def test_self_prior_matches_dense(small_graph):
    s = small_graph
    a = s["wl"].alpha
    D = mlp.self_prior(s["g"], a)
    live = s["g"].deg_u > 0
    ref = a + a * (1 - a) * np.diag(s["P"])
    assert np.abs(D[live] - ref[live]).max() < 1e-14 and np.all(D[~live] == 0)
    # a lower bound of pi(u, u) (both dropped terms are non-negative)
    assert np.all(D[live] <= np.diag(s["Pi"])[live] + 1e-15)


def test_extra_term_only_shifts_the_prediction():
    rng = np.random.default_rng(3)
    theta = init(2)
    Xu, Xx = rng.normal(0, 1, (2, mlp.IN)), rng.normal(0, 1, (4, mlp.IN))
    ws = rng.uniform(1, 5, 4)
    E = np.zeros((2, 4))
    E[1, 3] = 0.2
    p0 = mlp.predict(theta, Xu, Xx, ws, 0.05)
    p1 = mlp.predict(theta, Xu, Xx, ws, 0.05, E)
    assert np.array_equal(p1 - p0, E)
    T = p1.copy()
    loss, grad = mlp.loss_and_grad(theta, Xu, Xx, ws, T, 0.05, 1e-4, E)
    assert loss < 1e-20 and np.abs(grad).max() < 1e-12
