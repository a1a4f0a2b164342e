"""Checks that pin the FP64 oracle to facts other than itself.

Each ``pin_*`` function returns a list of failure strings (empty = pass). The
pin tests assert they all pass against the real oracle; the mutation tests
assert that every deliberately broken copy of the oracle fails at least one.

Sources of truth used here, none of them the oracle's own formulas:
  * closed forms of Eq. (hpp) on graphs whose P is known in closed form
    (rank-one P, P = I, complete bipartite), derived by hand;
  * a Monte-Carlo simulation of the random walk with restart that defines
    HPP (Sec. 3.2), which pins the direction of P;
  * the dense LU solve of Pi = alpha (I - (1-alpha) P)^-1 (a library routine);
  * the paper's theorems as inequalities: Theorems 1-3, Lemma 1, Lemma 3, Lemma 4;
  * values the paper prints (tests/golden/).
"""
import math
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return rows


def _fail(cond, msg, out):
    if not cond:
        out.append(msg)


# ---------------------------------------------------------------------------
# hand-built graphs with closed-form HPP
# ---------------------------------------------------------------------------

def star_graph(n_u=7, seed=3):
    """Every U node linked to the single V node 0 (V node 1 isolated).
    P = 1 s^T with s(y) = w(y,0)/ws(0), so by Sherman-Morrison
    Pi = alpha I + (1-alpha) 1 s^T."""
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 10, n_u).astype(np.float64)
    eu = np.arange(n_u, dtype=np.int32)
    ev = np.zeros(n_u, dtype=np.int32)
    s = w / w.sum()
    Pi = 0.15 * np.eye(n_u) + 0.85 * np.outer(np.ones(n_u), s)
    return (n_u, 2, eu, ev, w), Pi


def matching_graph(n=6):
    """Edges (i, i): P = I, so pi(u, x) = 1[x = u]."""
    eu = np.arange(n, dtype=np.int32)
    w = np.arange(1, n + 1, dtype=np.float64)
    return (n, n, eu, eu.copy(), w), np.eye(n)


def complete_graph(n_u=5, n_v=4, wt=2.5):
    """K_{n_u,n_v} with equal weights: P(x, y) = 1/n_u, so
    pi(u, x) = alpha 1[x=u] + (1-alpha)/n_u."""
    eu = np.repeat(np.arange(n_u, dtype=np.int32), n_v)
    ev = np.tile(np.arange(n_v, dtype=np.int32), n_u)
    w = np.full(eu.size, wt)
    Pi = 0.15 * np.eye(n_u) + 0.85 / n_u * np.ones((n_u, n_u))
    return (n_u, n_v, eu, ev, w), Pi


def two_components():
    """Two disjoint complete blocks: beta vanishes across blocks."""
    (a_nu, a_nv, a_u, a_v, a_w), PiA = complete_graph(3, 2, 1.0)
    (b_nu, b_nv, b_u, b_v, b_w), PiB = complete_graph(4, 3, 3.0)
    eu = np.concatenate([a_u, b_u + a_nu]).astype(np.int32)
    ev = np.concatenate([a_v, b_v + a_nv]).astype(np.int32)
    w = np.concatenate([a_w, b_w])
    Pi = np.zeros((a_nu + b_nu, a_nu + b_nu))
    Pi[:a_nu, :a_nu] = PiA
    Pi[a_nu:, a_nu:] = PiB
    return (a_nu + b_nu, a_nv + b_nv, eu, ev, w), Pi


CLOSED_FORMS = {"star": star_graph, "matching": matching_graph,
                "complete": complete_graph, "two_components": two_components}


def walk_graph():
    """A small irregular graph for the random-walk simulation (asymmetric P)."""
    eu = np.array([0, 0, 1, 1, 2, 3, 3, 4, 4, 4], dtype=np.int32)
    ev = np.array([0, 1, 1, 2, 0, 2, 3, 0, 3, 1], dtype=np.int32)
    w = np.array([1.0, 3.0, 2.0, 1.0, 5.0, 1.0, 4.0, 2.0, 1.0, 1.0])
    return 5, 4, eu, ev, w


def simulate_rwr(n_u, n_v, eu, ev, w, alpha, src, n_walks, seed):
    """Estimate pi(src, .) by simulating random walks with restart on the
    bipartite graph itself: at each U node the walk stops with probability
    alpha, otherwise it steps U->V with probability w/ws(u) and then V->U with
    probability w/ws(v) (Sec. 3.2). Returns end-node frequencies. All walks
    advance together; a neighbour is drawn by inverting the running sum of
    the edge weights of the current node."""
    rng = np.random.default_rng(seed)
    eu, ev, w = np.asarray(eu), np.asarray(ev), np.asarray(w, dtype=np.float64)

    def side(a, b, n):
        order = np.lexsort((b, a))
        a_s, b_s, w_s = a[order], b[order], w[order]
        cw = np.cumsum(w_s)
        start = np.searchsorted(a_s, np.arange(n), side="left")
        base = np.where(start > 0, cw[np.maximum(start - 1, 0)], 0.0)
        tot = np.bincount(a_s, weights=w_s, minlength=n)
        return cw, base, tot, b_s

    cu, bu, tu, nu_to_v = side(eu, ev, n_u)
    cv, bv, tv, nv_to_u = side(ev, eu, n_v)
    x = np.full(n_walks, src, dtype=np.int64)
    alive = np.ones(n_walks, dtype=bool)
    while alive.any():
        idx = np.nonzero(alive)[0]
        stop = rng.random(idx.size) < alpha
        alive[idx[stop]] = False
        idx = idx[~stop]
        if idx.size == 0:
            break
        cur = x[idx]
        e = np.searchsorted(cu, bu[cur] + rng.random(idx.size) * tu[cur], side="right")
        vv = nu_to_v[np.minimum(e, cu.size - 1)]
        e = np.searchsorted(cv, bv[vv] + rng.random(idx.size) * tv[vv], side="right")
        x[idx] = nv_to_u[np.minimum(e, cv.size - 1)]
    return np.bincount(x, minlength=n_u) / n_walks


# ---------------------------------------------------------------------------
# pins
# ---------------------------------------------------------------------------

def pin_closed_forms(alpha=0.15):
    out = []
    for name, mk in CLOSED_FORMS.items():
        (nu, nv, eu, ev, w), Pi_cf = mk()
        g = oracle.Graph(nu, nv, eu, ev, w)
        for u in range(nu):
            pf = g.hpp_forward(u, alpha, 1e-14)
            pb = g.hpp_backward(u, alpha, 1e-14)
            _fail(np.allclose(pf, Pi_cf[u, :], atol=1e-12), f"{name}: forward series row {u}", out)
            _fail(np.allclose(pb, Pi_cf[:, u], atol=1e-12), f"{name}: backward series col {u}", out)
            beta_cf = Pi_cf[u, :] + Pi_cf[:, u]
            for eps in (1e-2, 1e-5):
                b, _, _, _ = g.approx_bhpp(u, alpha, eps)
                d = beta_cf - b
                _fail(d.min() >= -1e-12 and d.max() <= eps + 1e-12,
                      f"{name}: Theorem 3 band u={u} eps={eps} [{d.min()},{d.max()}]", out)
            # Algorithm 1 from a one-hot start approaches row u of Pi
            p = g.power_iteration(np.eye(nu)[u], alpha, 200)
            _fail(np.allclose(p, Pi_cf[u, :], atol=1e-12), f"{name}: PowerIteration row {u}", out)
        Pi_d, _, _ = oracle.exact_dense(nu, nv, eu, ev, w, alpha)
        _fail(np.allclose(Pi_d, Pi_cf, atol=1e-12), f"{name}: dense solve", out)
    return out


def pin_random_walk(alpha=0.15, n_walks=400000):
    """The oracle's forward HPP row and beta' against simulated random walks
    (each entry within 5 standard errors, plus 1e-3)."""
    out = []
    nu, nv, eu, ev, w = walk_graph()
    g = oracle.Graph(nu, nv, eu, ev, w)
    Pi_d, _, _ = oracle.exact_dense(nu, nv, eu, ev, w, alpha)
    est = np.array([simulate_rwr(nu, nv, eu, ev, w, alpha, x, n_walks, 11 + x) for x in range(nu)])
    sig = np.sqrt(np.maximum(est * (1 - est), 1e-6) / n_walks)
    for src in range(nu):
        pf = g.hpp_forward(src, alpha, 1e-14)
        _fail(np.all(np.abs(est[src] - pf) <= 5 * sig[src] + 1e-3), f"walks vs forward row {src}", out)
        _fail(np.allclose(Pi_d[src, :], pf, atol=1e-12), f"dense row {src}", out)
        b, _, _, _ = g.approx_bhpp(src, alpha, 1e-6)
        beta_mc = est[src, :] + est[:, src]
        tol = 5 * (sig[src, :] + sig[:, src]) + 2e-3
        _fail(np.all(np.abs(beta_mc - b) <= tol), f"walks vs beta' src {src}", out)
    return out


def pin_dense_invariants(Pi, ws, out=None):
    """Rows of Pi sum to 1 on non-isolated rows, Pi >= 0, and Lemma 3:
    ws(i) pi(i, j) = ws(j) pi(j, i)."""
    out = [] if out is None else out
    nz = ws > 0
    _fail(np.allclose(Pi[nz].sum(1), 1.0, atol=1e-10), "row sums", out)
    _fail(Pi.min() >= -1e-15, "non-negative", out)
    S = ws[:, None] * Pi
    _fail(np.allclose(S, S.T, atol=1e-12 * max(1.0, np.abs(S).max())), "Lemma 3 symmetry", out)
    return out


def pin_theorems(g, Pi, sources, alpha, eps_list):
    """Theorems 1-3 on every source: 0 <= pi(x,u) - pi_b <= eps_b,
    0 <= pi(u,x) - pi_f <= eps_f, 0 <= beta - beta' <= eps (plus FP64 slack)."""
    out, seen = [], []
    for eps in eps_list:
        eps_b = g.eps_b(eps)
        for u in sources:
            u = int(u)
            b, pf, pb, st = g.approx_bhpp(u, alpha, eps)
            seen.append(st)
            d_b = Pi[:, u] - pb
            d_f = Pi[u, :] - pf
            d = (Pi[u, :] + Pi[:, u]) - b
            tol = 1e-12
            _fail(d_b.min() >= -tol and d_b.max() <= eps_b + tol, f"Thm1 u={u} eps={eps}", out)
            _fail(d_f.min() >= -tol and d_f.max() <= eps - eps_b + tol, f"Thm2 u={u} eps={eps}", out)
            _fail(d.min() >= -tol and d.max() <= eps + tol, f"Thm3 u={u} eps={eps}", out)
    return out, seen


def pin_lemma1_and_mass(g, Pi, u, alpha, eps):
    """Lemma 1 at the end of every push iteration, pi(., u) = pi_b + Pi r, and
    the mass invariant sum_x ws(x) (pi_b(x) + r(x)) = ws(u) that follows from
    it (Lemma 3 makes ws^T Pi = ws^T)."""
    out = []
    ws = g.ws_u
    col = Pi[:, u]
    worst = [0.0, 0.0]
    def cb(phase, it, pib, r):
        worst[0] = max(worst[0], np.abs(col - (pib + Pi @ r)).max())
        worst[1] = max(worst[1], abs((ws * (pib + r)).sum() - ws[u]) / ws[u])
    g.approx_bhpp(u, alpha, eps, trace=cb)
    _fail(worst[0] <= 1e-12, f"Lemma 1 u={u}: {worst[0]}", out)
    _fail(worst[1] <= 1e-12, f"mass u={u}: {worst[1]}", out)
    return out


def pin_lambda(g, Pi, alpha):
    """Lemma 4: lambda >= max column sum of Pi for any tau, and lambda <= the
    ws ratio branch of Eq. (lambda)."""
    out = []
    colmax = Pi.sum(0).max()
    ws = g.ws_u
    ratio = ws.max() / ws[ws > 0].min()
    for tau in (0, 3, 10, None):
        lam = g.lambda_(alpha, tau)
        _fail(lam >= colmax - 1e-9, f"lambda tau={tau}: {lam} < {colmax}", out)
        _fail(lam <= ratio * (1 + 1e-12), f"lambda tau={tau} above ws ratio", out)
    # tau large: the rho branch is tight (within |U| (1-alpha)^(tau+1))
    lam = g.lambda_(alpha, 400)
    _fail(lam <= colmax + 1e-6 or lam == ratio, f"lambda tau=400 not tight: {lam} vs {colmax}", out)
    return out


def pin_power_mass(g, alpha):
    """Algorithm 1 keeps exact mass: sum PowerIteration(e, t) =
    (1 - (1-alpha)^(t+1)) sum e for e >= 0 supported on non-isolated nodes."""
    out = []
    rng = np.random.default_rng(5)
    e = rng.random(g.n_u) * (g.ws_u > 0)
    for t in (0, 1, 7, 30):
        p = g.power_iteration(e, alpha, t)
        want = (1 - (1 - alpha) ** (t + 1)) * e.sum()
        _fail(abs(p.sum() - want) <= 1e-12 * e.sum(), f"PowerIteration mass t={t}", out)
    return out


def pin_golden_gamma(g, sources, alpha):
    """Fig. 1 first DBLP point (tests/golden/fig1_gamma_dblp.txt): gamma = 0.85
    at eps_b = 0.5 whenever one push of the source ends SS-Push."""
    out = []
    (a, eb, gamma), = read_golden("fig1_gamma_dblp.txt")
    hit = 0
    for u in sources:
        _, _, _, st = g.approx_bhpp(int(u), a, 1.0, eps_b=eb)
        if st["ss_sel_iters"] == 1 and st["ss_switched"] == 0:
            hit += 1
            _fail(abs(st["gamma"] - gamma) <= 1e-12, f"gamma u={u}: {st['gamma']}", out)
    _fail(hit > 0, "no source ended SS-Push after one push", out)
    return out


def pin_golden_rounds():
    out = []
    (a, s, ef, t), = read_golden("powiter_rounds.txt")
    _fail(oracle.t_of(s, ef, a) == int(t), f"Eq. (t) rounds: {oracle.t_of(s, ef, a)} != {int(t)}", out)
    # and the rounding is what Theorem 2's proof needs: (1-a)^(t+1) s <= ef < (1-a)^t s
    for sr, e in ((1.0, 0.1), (0.3, 1e-6), (2.0e-3, 5e-7), (1e-7, 1e-6)):
        tt = oracle.t_of(sr, e, a)
        _fail((1 - a) ** (tt + 1) * sr <= e * (1 + 1e-12), f"t too small {sr},{e}", out)
        _fail(tt == 0 or (1 - a) ** tt * sr > e, f"t too large {sr},{e}", out)
    return out


def pin_eps_b():
    """Eq. (epsilon-b) at the workload sizes, worked by hand:
    2000x3000, 20000 edges: mu = sqrt(6e6)/2e4 = 0.122474..., ratio = 0.46738...
    1Mx2M, 20M edges: mu = sqrt(2e12)/2e7 = 0.0707107, ratio = 0.48168...
    and mu >= 1 (a perfect matching of 4: mu = 1) falls back to eps/2."""
    out = []
    g1 = oracle.Graph(2000, 3000, np.array([0], np.int32), np.array([0], np.int32), np.ones(1))
    _fail(abs(oracle._load().orc_eps_b(2000, 3000, 20000, 1.0) - 0.46738) < 1e-5, "eps_b small", out)
    _fail(abs(oracle._load().orc_eps_b(1000000, 2000000, 20000000, 1.0) - 0.48168) < 1e-5, "eps_b medium", out)
    _fail(abs(oracle._load().orc_eps_b(4, 4, 4, 1.0) - 0.5) < 1e-15, "eps_b fallback", out)
    del g1
    return out


def pin_series_agree(g, sources, alpha):
    """Forward and backward series are computed independently; Lemma 3 links
    them: ws(u) pi(u, x) = ws(x) pi(x, u)."""
    out = []
    ws = g.ws_u
    for u in sources[:3]:
        u = int(u)
        pf = g.hpp_forward(u, alpha, 1e-13)
        pb = g.hpp_backward(u, alpha, 1e-13)
        lhs, rhs = ws[u] * pf, ws * pb
        _fail(np.allclose(lhs, rhs, atol=1e-10 * ws[u]), f"series Lemma 3 u={u}", out)
    return out


def pin_warm_start(g, Pi, sources, alpha, eps=1e-6):
    """Warm start: Lemma 1 for the signed residue of arbitrary starts, an
    exact start returns the exact beta, noisy starts stay within eps on both
    sides, and a useless start is the cold start."""
    out = []
    rng = np.random.default_rng(11)
    src = [int(u) for u in sources[:4]]
    for u in src[:2]:
        y = Pi[:, u] * (1 + rng.normal(0, 0.3, g.n_u))
        r = g.warm_residue(u, alpha, y)
        _fail(np.abs(y + Pi @ r - Pi[:, u]).max() < 1e-12, f"warm residue breaks Lemma 1 (u={u})", out)
    exact = np.stack([oracle.bhpp_from_dense(Pi, u) for u in src])
    y0 = np.stack([Pi[:, u] for u in src])
    b, st, wi = g.approx_bhpp_warm_many(src, alpha, eps, y0)
    _fail(np.abs(b - exact).max() < 1e-11, "exact warm start does not return beta", out)
    y0 = np.stack([Pi[:, u] * (1 + rng.normal(0, 0.05, g.n_u)) for u in src])
    b, st, wi = g.approx_bhpp_warm_many(src, alpha, eps, y0)
    _fail(all(w["fell_back"] == 0 for w in wi), "noisy warm start fell back", out)
    _fail(np.abs(b - exact).max() <= eps + 1e-12, f"warm start outside eps: {np.abs(b - exact).max()}", out)
    b, st, wi = g.approx_bhpp_warm_many(src[:1], alpha, eps, np.zeros((1, g.n_u)))
    cold, _ = g.approx_bhpp_many(src[:1], alpha, eps)
    _fail(wi[0]["fell_back"] == 1 and np.array_equal(b[0], cold[0]), "zero start is not the cold start", out)
    return out


def pisp_rounds(alpha, eps):
    """The PowerIteration rounds of PISP by their definition: the smallest
    t >= 0 whose dropped mass (1-alpha)^(t+1) is at most eps/2 (a loop, not
    the log formula)."""
    t, m = 0, 1.0 - alpha
    while m > eps / 2:
        m *= 1.0 - alpha
        t += 1
    return t


def pin_pisp(g, Pi, sources, alpha, eps_list=(1e-2, 1e-4, 1e-7)):
    """PISP (Sec. 3.3): the forward part is short of pi(u, .) by exactly
    the dropped mass (1-alpha)^(t+1) in total and by at most eps/2 per entry,
    the backward part is within [pi(., u) - eps/2, pi(., u)] (SelectivePush's
    guarantee), so 0 <= beta - beta' <= eps. The rounds at alpha = 0.15,
    worked by hand: (1-a)^(t+1) <= eps/2 gives t = 32, 89, 103 at eps = 1e-2,
    1e-6, 1e-7 (0.85^33 = 0.00469 <= 0.005 < 0.85^32 = 0.00551)."""
    out = []
    hand = {1e-2: 32, 1e-6: 89, 1e-7: 103}
    for e, t in hand.items():
        _fail(pisp_rounds(0.15, e) == t, f"PISP rounds by hand eps={e}", out)
    for eps in eps_list:
        for u in sources:
            u = int(u)
            b, pf, pb, st = g.pisp(u, alpha, eps)
            t = pisp_rounds(alpha, eps)
            _fail(st["t"] == t, f"PISP t u={u} eps={eps}: {st['t']} != {t}", out)
            _fail(abs(pf.sum() - (1 - (1 - alpha) ** (t + 1))) <= 1e-12, f"PISP forward mass u={u} eps={eps}", out)
            d_f = Pi[u, :] - pf
            d_b = Pi[:, u] - pb
            d = (Pi[u, :] + Pi[:, u]) - b
            tol = 1e-12
            _fail(d_f.min() >= -tol and d_f.max() <= eps / 2 + tol, f"PISP forward band u={u} eps={eps}", out)
            _fail(d_b.min() >= -tol and d_b.max() <= eps / 2 + tol, f"PISP backward band u={u} eps={eps}", out)
            _fail(d.min() >= -tol and d.max() <= eps + tol, f"PISP band u={u} eps={eps}", out)
            _fail(st["sp_iters"] >= 1, f"PISP no SelectivePush iteration u={u}", out)
    return out


PHILOX_KAT = [  # Philox4x32-10 known-answer vectors of its authors (Random123): counter, key -> output
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


def pin_mcsp(g, Pi, sources, alpha=0.15):
    """MCSP (Sec. 3.3): the generator reproduces Philox4x32-10's published
    known answers; every alias table encodes its row's distribution
    w(x, .)/ws(x); the walk count for |U| = 2000, eps_f = 5e-3, p_f = 1e-6 is
    2 (1 + 5e-3/3) ln(2e9) / 2.5e-5 = 1716168.56..., rounded up (worked by
    hand); walk frequencies agree with the dense Pi within 5 standard errors;
    and beta' is within eps of beta (both parts' errors are at most eps/2, the
    MonteCarlo part with probability 1 - p_f)."""
    out = []
    for ctr, key, want in PHILOX_KAT:
        got = oracle.philox4x32_10(ctr, key)
        _fail([int(x) for x in got] == list(want), f"Philox known answer {ctr}", out)
    _fail(oracle.mc_walks(2000, 5e-3, 1e-6) == 1716169, "MonteCarlo walk count", out)
    exp = g.export()
    for side, (rp, w, ws) in enumerate(((exp["rp_u"], exp["w_u"], exp["ws_u"]), (exp["rp_v"], exp["w_v"], exp["ws_v"]))):
        prob, alias = g.alias_tables(side)
        worst = 0.0
        for r in range(rp.size - 1):
            b, e = rp[r], rp[r + 1]
            d = e - b
            if d == 0:
                continue
            mass = prob[b:e].copy()
            np.add.at(mass, alias[b:e], 1.0 - prob[b:e])
            worst = max(worst, np.abs(mass / d - w[b:e] / ws[r]).max())
        _fail(worst <= 1e-12, f"alias tables side {side}: {worst}", out)
    n_r = 200000
    for u in sources[:2]:
        u = int(u)
        cnt, steps = g.mc_counts(u, alpha, n_r, 12345)
        est = cnt / n_r
        sig = np.sqrt(np.maximum(Pi[u] * (1 - Pi[u]), 1e-7) / n_r)
        _fail(np.all(np.abs(est - Pi[u]) <= 5 * sig + 1e-4), f"walk frequencies u={u}", out)
        _fail(cnt.sum() == n_r, "every walk ends once", out)
        _fail(abs(steps / n_r - (1 - alpha) / alpha) <= 0.05, f"mean walk length u={u}: {steps / n_r}", out)
    for u in sources[:2]:
        u = int(u)
        eps = 2e-2
        b, cnt, pib, nr = g.mcsp(u, alpha, eps, 1e-6, 7)
        beta = Pi[u, :] + Pi[:, u]
        _fail(np.abs(beta - b).max() <= eps, f"MCSP band u={u}: {np.abs(beta - b).max()}", out)
        d_b = Pi[:, u] - pib
        _fail(d_b.min() >= -1e-12 and d_b.max() <= eps / 2 + 1e-12, f"MCSP backward band u={u}", out)
        _fail(nr == oracle.mc_walks(g.n_u, eps / 2, 1e-6) and cnt.sum() == nr, f"MCSP walks u={u}", out)
    return out


def run_core_pins(small, stop_early=False):
    """The pins the mutation tests rely on; fast enough to run per mutant.
    ``small`` holds the edge list and the dense Pi (computed with numpy, not
    the C oracle); the oracle's graph is rebuilt with whichever library is
    loaded."""
    el, Pi, src, a = small["el"], small["Pi"], small["sources"], small["wl"].alpha
    g = oracle.Graph.from_edges(el)
    checks = [pin_golden_rounds,
              lambda: pin_closed_forms(a),
              lambda: pin_power_mass(g, a),
              lambda: pin_golden_gamma(g, src, a),
              lambda: pin_theorems(g, Pi, src[:4], a, [1e-3, 1e-6])[0],
              lambda: pin_lemma1_and_mass(g, Pi, int(src[0]), a, 1e-5),
              lambda: pin_lambda(g, Pi, a),
              lambda: pin_warm_start(g, Pi, src, a),
              lambda: pin_pisp(g, Pi, src[:4], a),
              lambda: pin_mcsp(g, Pi, src, a)]
    out = []
    for c in checks:
        try:
            out += c()
        except ValueError as e:      # an oracle error code counts as a failed pin
            out.append(str(e))
        if out and stop_early:
            break
    return out

if __name__ == "__main__":
    # python pins_lib.py <oracle .so>: run the core pins against that library
    # and print the number of failures (used by the mutation tests).
    import json
    import sys
    import synth
    oracle.use_library(sys.argv[1])
    wl = synth.SMALL
    el = wl.graph()
    Pi, _, _ = oracle.exact_dense(el.n_u, el.n_v, el.u, el.v, el.w, wl.alpha)
    res = run_core_pins(dict(el=el, Pi=Pi, sources=wl.sources(el), wl=wl), stop_early=len(sys.argv) > 2)
    print(json.dumps({"failures": len(res), "first": res[:3]}))
