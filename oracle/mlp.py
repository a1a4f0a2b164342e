"""FP64 reference of the warm-start network and its node features.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU baseline
leg of the benchmark use this module; the GPU library never does.

The warm start is not in the paper; it seeds Lemma 1's invariant (any start
y of pi(., u) with the signed residue r = e_u - (y - (1-alpha) P y)/alpha).
Its prediction uses the symmetric kernel of Lemma 3,
K(u, x) = pi(u, x)/ws(x) = pi(x, u)/ws(u), modelled by two towers f and g:
    p_hat(u, x) = c * ws(x) * <f(feat(u)), g(feat(x))> + [x = u] D(u)
(estimates pi(u, x)), where D(u) = alpha + alpha (1-alpha) P(u,u) is the
structural self term (the first two terms of the return series, which a
low-rank product cannot express); y(x) = ws(u)/ws(x) p_hat(u, x) then
estimates pi(x, u).

Towers: 64 -> 256 -> 256 -> 128, GELU after the two hidden layers,
GELU(z) = z Phi(z) (exact form with erf). Parameters are one flat vector:
tower f then tower g, each W1[64][256], b1[256], W2[256][256], b2[256],
W3[256][128], b3[128] (row-major, y = x W + b).

Training loss on a batch of sources u_i and candidates x_j with targets
T[i][j] = pi(u_i, x_j) (NaN where unknown: left out):
    L = mean over known (i, j) of (p_hat(u_i, x_j) - T[i][j])^2 / (T[i][j] + tau),
a squared relative error weighted by the mass T, so the many small entries
of the far field count by their mass as they do in the residue's L1 norm.
Everything here is FP64 with no intermediate rounding.
"""
from __future__ import annotations

import math

import numpy as np

IN, HID, OUT = 64, 256, 128
N_BUCKETS = IN - 4
SHAPES = [(IN, HID), (HID,), (HID, HID), (HID,), (HID, OUT), (OUT,)]
TOWER = sum(int(np.prod(s)) for s in SHAPES)
N_PARAMS = 2 * TOWER


def bucket(v):
    """Neighbour-id bucket of a V node (its external id): a multiplicative hash."""
    h = (np.asarray(v, dtype=np.uint64) * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)
    return ((h >> np.uint64(16)) % np.uint64(N_BUCKETS)).astype(np.int64)


def features(g):
    """64 features per U node of an oracle.Graph (rows of isolated nodes are 0):
    [0] 1, [1] ln(1+d(x))/8, [2] ln ws(x)/8, [3] sum_v w(x,v)/ws(x) ln(1+d(v))/8,
    [4+b] sum over neighbours v in bucket b of w(x,v)/ws(x)."""
    ex = g.export()
    rp_u, ci_u, w_u, rp_v = ex["rp_u"], ex["ci_u"], ex["w_u"], ex["rp_v"]
    ws_u = ex["ws_u"]
    deg_u = np.diff(rp_u)
    deg_v = np.diff(rp_v)
    F = np.zeros((g.n_u, IN))
    rows = np.repeat(np.arange(g.n_u), deg_u)
    live = deg_u > 0
    F[live, 0] = 1.0
    F[live, 1] = np.log1p(deg_u[live]) / 8.0
    F[live, 2] = np.log(ws_u[live]) / 8.0
    frac = w_u / ws_u[rows]
    np.add.at(F[:, 3], rows, frac * np.log1p(deg_v[ci_u]) / 8.0)
    np.add.at(F, (rows, 4 + bucket(ci_u)), frac)
    return F


def self_prior(g, alpha):
    """Structural self term added to the prediction at x = u: the first two
    terms of the return series of Eq. (hpp), alpha + alpha (1-alpha) P(u,u),
    with P(u,u) = sum_v w(u,v)^2 / (ws(u) ws(v)) (Eq. (pmatrix)); 0 if isolated."""
    ex = g.export()
    rp_u, ci_u, w_u, ws_u, ws_v = ex["rp_u"], ex["ci_u"], ex["w_u"], ex["ws_u"], ex["ws_v"]
    deg = np.diff(rp_u)
    rows = np.repeat(np.arange(g.n_u), deg)
    s = np.zeros(g.n_u)
    np.add.at(s, rows, w_u * w_u / ws_v[ci_u])
    out = np.zeros(g.n_u)
    live = deg > 0
    out[live] = alpha + alpha * (1 - alpha) * s[live] / ws_u[live]
    return out


def split(theta):
    """Flat parameter vector -> (tower f, tower g), each a list of 6 arrays."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == N_PARAMS
    towers, o = [], 0
    for _ in range(2):
        t = []
        for s in SHAPES:
            n = int(np.prod(s))
            t.append(theta[o:o + n].reshape(s))
            o += n
        towers.append(t)
    return towers


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


_erf = np.vectorize(math.erf, otypes=[np.float64])


def tower_forward(p, X):
    W1, b1, W2, b2, W3, b3 = p
    z1 = X @ W1 + b1
    a1 = gelu(z1)
    z2 = a1 @ W2 + b2
    a2 = gelu(z2)
    z3 = a2 @ W3 + b3
    return z3, (X, z1, a1, z2, a2)


def tower_backward(p, cache, dz3):
    W1, b1, W2, b2, W3, b3 = p
    X, z1, a1, z2, a2 = cache
    gW3 = a2.T @ dz3
    gb3 = dz3.sum(0)
    dz2 = (dz3 @ W3.T) * gelu_grad(z2)
    gW2 = a1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * gelu_grad(z1)
    gW1 = X.T @ dz1
    gb1 = dz1.sum(0)
    return [gW1, gb1, gW2, gb2, gW3, gb3]


def predict(theta, Xu, Xx, ws_x, c, extra=None):
    """p_hat[i][j] = c ws(x_j) <f(Xu_i), g(Xx_j)> (+ extra[i][j], the self term)."""
    pf, pg = split(theta)
    F, _ = tower_forward(pf, Xu)
    Gm, _ = tower_forward(pg, Xx)
    p = c * (F @ Gm.T) * np.asarray(ws_x)[None, :]
    return p if extra is None else p + extra


def loss_and_grad(theta, Xu, Xx, ws_x, T, c, tau, extra=None):
    """The training loss and its gradient (flat, same layout as theta);
    extra[i][j] is added to the prediction (the self term where x_j = u_i)."""
    pf, pg = split(theta)
    F, cf = tower_forward(pf, Xu)
    Gm, cg = tower_forward(pg, Xx)
    ws_x = np.asarray(ws_x, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    known = np.isfinite(T)
    Tk = np.where(known, T, 0.0)
    wgt = np.where(known, 1.0 / np.sqrt(np.abs(Tk) + tau), 0.0)
    pred = c * (F @ Gm.T) * ws_x[None, :]
    if extra is not None:
        pred = pred + extra
    diff = (pred - Tk) * wgt
    n = int(known.sum())
    loss = float((diff * diff).sum() / n)
    dpred = 2.0 * diff * wgt / n
    dK = dpred * c * ws_x[None, :]
    dF = dK @ Gm
    dG = dK.T @ F
    grads = tower_backward(pf, cf, dF) + tower_backward(pg, cg, dG)
    return loss, np.concatenate([x.ravel() for x in grads])


def bf16_round(a):
    """Round FP32 values to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
