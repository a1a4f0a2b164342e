"""FP64 CPU oracle for approximate BHPP (Yang, WWW '22).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the GPU library and the GPU library never calls it.

Two parts:
  * O-exact: the plain definition of the result. ``exact_dense`` forms P
    densely from Eq. (pmatrix) and solves Pi = alpha (I - (1-alpha) P)^-1
    (Eq. (hpp) summed in closed form; a library LU solve is the only step).
    ``hpp_forward`` / ``hpp_backward`` sum Eq. (hpp) as a truncated series in
    C for graphs too large for a dense solve.
  * O-method: Algorithms 1-5 step by step in C (``approx_bhpp``), with
    Lemma 4 (``lambda_``) and Eq. (epsilon-b) (``eps_b``).
Plus a brute-force top-k by full sort.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bhpp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lib_path_override = None

ORC_ERRORS = {-1: "invalid argument", -2: "id out of range", -3: "isolated source",
              -4: "bad weight", -5: "out of memory", -6: "no convergence"}


def build(force: bool = False) -> str:
    """Compile the C oracle (-O3, no fast-math, OpenMP across queries only)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=native", "-fno-fast-math", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Stats(ctypes.Structure):
    _fields_ = [("ss_sel_iters", ctypes.c_int32), ("ss_seq_iters", ctypes.c_int32),
                ("pi_sel_iters", ctypes.c_int32), ("t", ctypes.c_int32),
                ("ss_switched", ctypes.c_int32), ("pi_returned", ctypes.c_int32),
                ("np_ss", ctypes.c_double), ("np_pi", ctypes.c_double),
                ("gamma", ctypes.c_double), ("sum_r_ss", ctypes.c_double),
                ("sum_rf", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class WarmInfo(ctypes.Structure):
    _fields_ = [("res_l1", ctypes.c_double), ("res_max", ctypes.c_double), ("fell_back", ctypes.c_int32),
                ("pad", ctypes.c_int32)]

    def as_dict(self):
        return dict(res_l1=self.res_l1, res_max=self.res_max, fell_back=self.fell_back)


class PispStats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int32), ("sp_iters", ctypes.c_int32), ("np", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


TRACE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))


def use_library(path):
    """Load the oracle from another shared object (the mutation tests build
    deliberately broken copies of the oracle and point the wrappers at them).
    ``None`` restores the real oracle."""
    global _lib, _lib_path_override
    _lib = None
    _lib_path_override = path


def _load():
    global _lib
    if _lib is None:
        if _lib_path_override is None:
            build()
        L = ctypes.CDLL(_lib_path_override or _LIB_PATH)
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.orc_build.restype = P
        L.orc_build.argtypes = [I32, I32, I64, P, P, P, ctypes.POINTER(ctypes.c_int)]
        L.orc_free.argtypes = [P]
        L.orc_nnz.restype = I64
        L.orc_nnz.argtypes = [P]
        L.orc_export.argtypes = [P] + [P] * 8
        L.orc_power_iteration.argtypes = [P, P, D, I32, P]
        L.orc_hpp_forward.argtypes = [P, I32, D, D, P, P]
        L.orc_hpp_backward.argtypes = [P, I32, D, D, P, P]
        L.orc_hpp_forward_many.argtypes = [P, I32, P, D, D, P, I32]
        L.orc_hpp_forward_block.argtypes = [P, I32, P, D, D, P, I32, I32]
        L.orc_eps_b.restype = D
        L.orc_eps_b.argtypes = [I32, I32, I64, D]
        L.orc_default_tau.restype = I32
        L.orc_default_tau.argtypes = [I32, D]
        L.orc_lambda.argtypes = [P, D, I32, ctypes.POINTER(D), ctypes.POINTER(D)]
        L.orc_approx_bhpp.argtypes = [P, I32, D, D, D, D, P, P, P, ctypes.POINTER(Stats), TRACE_FN, P]
        L.orc_approx_bhpp_many.argtypes = [P, I32, P, D, D, D, D, P, P, I32]
        L.orc_warm_residue.argtypes = [P, I32, D, P, P]
        L.orc_approx_bhpp_warm.argtypes = [P, I32, D, D, D, D, P, P, ctypes.POINTER(Stats),
                                           ctypes.POINTER(WarmInfo)]
        L.orc_approx_bhpp_warm_many.argtypes = [P, I32, P, D, D, D, D, P, P, P, P, I32]
        L.orc_pisp.argtypes = [P, I32, D, D, P, P, P, P]
        L.orc_approx_bhpp_sample.argtypes = [P, I32, P, D, D, D, D, I32, P, I32]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_alias_tables.argtypes = [P, I32, P, P]
        L.orc_mc_walks.restype = I64
        L.orc_mc_walks.argtypes = [I32, D, D]
        L.orc_mc_counts.argtypes = [P, I32, D, I64, ctypes.c_uint64, P, P]
        L.orc_mcsp.argtypes = [P, I32, D, D, D, ctypes.c_uint64, P, P, P, P]
        L.orc_pisp_many.argtypes = [P, I32, P, D, D, P, P, I32]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_t.restype = I32
        L.orc_t.argtypes = [D, D, D]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle error {rc}: {ORC_ERRORS.get(rc, '?')}")


def _ptr(a):
    return a.ctypes.data if a is not None else None


class Graph:
    """The oracle's own CSR/CSC build of W (Sec. 3.1), with ws from Eq. (d)."""

    def __init__(self, n_u, n_v, eu, ev, w):
        L = _load()
        self._eu = np.ascontiguousarray(eu, dtype=np.int32)
        self._ev = np.ascontiguousarray(ev, dtype=np.int32)
        self._w = np.ascontiguousarray(w, dtype=np.float64)
        err = ctypes.c_int(0)
        h = L.orc_build(n_u, n_v, self._eu.size, _ptr(self._eu), _ptr(self._ev), _ptr(self._w),
                        ctypes.byref(err))
        if not h:
            _check(err.value)
        self._h = h
        self.n_u, self.n_v = int(n_u), int(n_v)
        self.n_e = int(L.orc_nnz(h))
        self._exp = None

    @classmethod
    def from_edges(cls, el):
        return cls(el.n_u, el.n_v, el.u, el.v, el.w)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_free(self._h)
            self._h = None

    def export(self):
        """CSR of W (rows U) and of W^T (rows V), and ws, as numpy arrays."""
        if self._exp is None:
            nu, nv, m = self.n_u, self.n_v, self.n_e
            d = dict(rp_u=np.empty(nu + 1, np.int64), ci_u=np.empty(m, np.int32), w_u=np.empty(m),
                     rp_v=np.empty(nv + 1, np.int64), ci_v=np.empty(m, np.int32), w_v=np.empty(m),
                     ws_u=np.empty(nu), ws_v=np.empty(nv))
            _load().orc_export(self._h, *[_ptr(d[k]) for k in
                                          ("rp_u", "ci_u", "w_u", "rp_v", "ci_v", "w_v", "ws_u", "ws_v")])
            self._exp = d
        return self._exp

    @property
    def ws_u(self):
        return self.export()["ws_u"]

    @property
    def deg_u(self):
        return np.diff(self.export()["rp_u"])

    # ---- Algorithm 1 ----
    def power_iteration(self, e, alpha, t):
        e = np.ascontiguousarray(e, dtype=np.float64)
        out = np.empty(self.n_u)
        _check(_load().orc_power_iteration(self._h, _ptr(e), alpha, int(t), _ptr(out)))
        return out

    # ---- Eq. (hpp) as truncated series ----
    def hpp_forward(self, u, alpha, tail=1e-12):
        out = np.empty(self.n_u)
        _check(_load().orc_hpp_forward(self._h, int(u), alpha, tail, _ptr(out), None))
        return out

    def hpp_backward(self, u, alpha, tail=1e-12):
        out = np.empty(self.n_u)
        _check(_load().orc_hpp_backward(self._h, int(u), alpha, tail, _ptr(out), None))
        return out

    def hpp_forward_many(self, sources, alpha, tail=1e-10, nthreads=0):
        src = np.ascontiguousarray(sources, dtype=np.int32)
        out = np.empty((src.size, self.n_u))
        _check(_load().orc_hpp_forward_many(self._h, src.size, _ptr(src), alpha, tail, _ptr(out),
                                            int(nthreads)))
        return out

    def hpp_forward_block(self, sources, alpha, tail=1e-10, nthreads=0, progress=0):
        """The series of ``hpp_forward`` for several sources in one pass over
        the adjacency per term (rows split over threads); every row equals
        ``hpp_forward`` of its source bit for bit. ``progress`` > 0 prints a
        line to stderr every that many terms."""
        src = np.ascontiguousarray(sources, dtype=np.int32)
        out = np.empty((src.size, self.n_u))
        _check(_load().orc_hpp_forward_block(self._h, src.size, _ptr(src), alpha, tail, _ptr(out),
                                             int(nthreads), int(progress)))
        return out

    def exact_beta_many(self, sources, alpha, tail=1e-10, nthreads=0, block=64, progress=0):
        """beta(u, x) = pi(u, x) + pi(x, u), the second term from Lemma 3:
        pi(x, u) = pi(u, x) ws(u) / ws(x). Each entry is short of the exact
        value by at most 2 * tail: the dropped terms of pi(u, x) are at most
        tail * max_l P^l(u, x) and P^l(u, x) <= min(1, ws(x)/ws(u)) by the same
        reversibility. Isolated x score 0 (x != u). ``block`` > 0 runs the
        series for up to that many sources per adjacency pass
        (``hpp_forward_block``, the same bits); 0 runs one source per thread."""
        src = np.asarray(sources)
        if block > 0:
            pf = np.concatenate([self.hpp_forward_block(src[i:i + block], alpha, tail, nthreads, progress)
                                 for i in range(0, src.size, block)]) if src.size else np.empty((0, self.n_u))
        else:
            pf = self.hpp_forward_many(sources, alpha, tail, nthreads)
        ws = self.ws_u
        out = np.empty_like(pf)
        for i, u in enumerate(np.asarray(sources)):
            ratio = np.divide(ws[u], ws, out=np.zeros_like(ws), where=ws > 0)
            out[i] = pf[i] * (1.0 + ratio)
        return out

    # ---- preprocessing ----
    def eps_b(self, eps):
        return float(_load().orc_eps_b(self.n_u, self.n_v, self.n_e, eps))

    def default_tau(self, alpha):
        return int(_load().orc_default_tau(self.n_u, alpha))

    def lambda_(self, alpha, tau=None):
        tau = self.default_tau(alpha) if tau is None else tau
        lam, rmax = ctypes.c_double(), ctypes.c_double()
        _check(_load().orc_lambda(self._h, alpha, int(tau), ctypes.byref(lam), ctypes.byref(rmax)))
        return float(lam.value)

    # ---- Algorithm 5 ----
    def approx_bhpp(self, u, alpha, eps, eps_b=None, lam=None, trace=None):
        """Returns (beta', pi_f, pi_b, stats dict). ``trace(phase, iter, pi_b, r)``
        is called after every push iteration with copies of the arrays."""
        eps_b = self.eps_b(eps) if eps_b is None else eps_b
        lam = self.lambda_(alpha) if lam is None else lam
        beta, pif, pib = np.empty(self.n_u), np.empty(self.n_u), np.empty(self.n_u)
        st = Stats()
        nu = self.n_u
        if trace is not None:
            def _cb(ctx, phase, it, pb, r):
                trace(int(phase), int(it), np.ctypeslib.as_array(pb, (nu,)).copy(),
                      np.ctypeslib.as_array(r, (nu,)).copy())
            cb = TRACE_FN(_cb)
        else:
            cb = TRACE_FN()
        _check(_load().orc_approx_bhpp(self._h, int(u), alpha, eps, eps_b, lam, _ptr(beta), _ptr(pif),
                                       _ptr(pib), ctypes.byref(st), cb, None))
        return beta, pif, pib, st.as_dict()

    def approx_bhpp_many(self, sources, alpha, eps, eps_b=None, lam=None, nthreads=0, keep=True):
        eps_b = self.eps_b(eps) if eps_b is None else eps_b
        lam = self.lambda_(alpha) if lam is None else lam
        src = np.ascontiguousarray(sources, dtype=np.int32)
        beta = np.empty((src.size, self.n_u)) if keep else None
        st = (Stats * max(1, src.size))()
        _check(_load().orc_approx_bhpp_many(self._h, src.size, _ptr(src), alpha, eps, eps_b, lam,
                                            _ptr(beta), ctypes.cast(st, ctypes.c_void_p),
                                            int(nthreads)))
        return beta, [st[i].as_dict() for i in range(src.size)]

    # ---- PISP (Sec. 3.3, Baselines and Challenges) ----
    def pisp(self, u, alpha, eps):
        """The PISP baseline: PowerIteration for pi(u, .) with t rounds
        ((1-alpha)^(t+1) <= eps/2) plus SelectivePush for pi(., u) with
        eps_b = eps/2. Returns (beta', pi_f, pi_b, stats dict)."""
        beta, pif, pib = np.empty(self.n_u), np.empty(self.n_u), np.empty(self.n_u)
        st = PispStats()
        _check(_load().orc_pisp(self._h, int(u), alpha, eps, _ptr(beta), _ptr(pif), _ptr(pib), ctypes.byref(st)))
        return beta, pif, pib, st.as_dict()

    def pisp_many(self, sources, alpha, eps, nthreads=0, keep=True):
        src = np.ascontiguousarray(sources, dtype=np.int32)
        beta = np.empty((src.size, self.n_u)) if keep else None
        st = (PispStats * max(1, src.size))()
        _check(_load().orc_pisp_many(self._h, src.size, _ptr(src), alpha, eps, _ptr(beta),
                                     ctypes.cast(st, ctypes.c_void_p), int(nthreads)))
        return beta, [st[i].as_dict() for i in range(src.size)]

    def approx_bhpp_sample(self, sources, alpha, eps, max_iters, eps_b=None, lam=None, nthreads=0):
        """Algorithm 5 for each source, stopped after max_iters push
        iterations (a bounded sample for timing); returns the edges each
        query touched."""
        eps_b = self.eps_b(eps) if eps_b is None else eps_b
        lam = self.lambda_(alpha) if lam is None else lam
        src = np.ascontiguousarray(sources, dtype=np.int32)
        work = np.zeros(src.size)
        _check(_load().orc_approx_bhpp_sample(self._h, src.size, _ptr(src), alpha, eps, eps_b, lam, int(max_iters),
                                              _ptr(work), int(nthreads)))
        return work

    # ---- MCSP (Sec. 3.3, Baselines and Challenges) ----
    def alias_tables(self, side):
        """Walker alias tables (Vose's construction) of the rows of U
        (side 0, entries as in export()['ci_u']) or of V (side 1)."""
        prob = np.empty(self.n_e)
        alias = np.empty(self.n_e, np.int32)
        _check(_load().orc_alias_tables(self._h, int(side), _ptr(prob), _ptr(alias)))
        return prob, alias

    def mc_counts(self, u, alpha, n_r, seed):
        """End nodes of n_r random walks with restart from u (Philox draws)."""
        counts = np.empty(self.n_u, np.int64)
        steps = ctypes.c_double()
        _check(_load().orc_mc_counts(self._h, int(u), alpha, int(n_r), ctypes.c_uint64(seed), _ptr(counts),
                                     ctypes.byref(steps)))
        return counts, steps.value

    def mcsp(self, u, alpha, eps, p_f=1e-6, seed=0):
        """The MCSP baseline: MonteCarlo with eps/2 plus SelectivePush with
        eps/2. Returns (beta', counts, pi_b, n_r)."""
        beta, pib = np.empty(self.n_u), np.empty(self.n_u)
        counts = np.empty(self.n_u, np.int64)
        n_r = ctypes.c_int64()
        _check(_load().orc_mcsp(self._h, int(u), alpha, eps, p_f, ctypes.c_uint64(seed), _ptr(beta), _ptr(counts),
                                _ptr(pib), ctypes.byref(n_r)))
        return beta, counts, pib, int(n_r.value)

    def warm_residue(self, u, alpha, y):
        """Signed residue of a warm start y (estimates of pi(x, u)):
        r = e_u - (y - (1-alpha) P y) / alpha (Lemma 1 holds for it)."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        r = np.empty(self.n_u)
        _check(_load().orc_warm_residue(self._h, int(u), alpha, _ptr(y), _ptr(r)))
        return r

    def approx_bhpp_warm_many(self, sources, alpha, eps, y0, eps_b=None, lam=None, nthreads=0):
        """Approx-BHPP from warm starts y0[i] (backward coordinates) with signed
        residues; falls back to the cold start when the start is no better.
        Returns (beta, stats, warm infos)."""
        eps_b = self.eps_b(eps) if eps_b is None else eps_b
        lam = self.lambda_(alpha) if lam is None else lam
        src = np.ascontiguousarray(sources, dtype=np.int32)
        y0 = np.ascontiguousarray(y0, dtype=np.float64).reshape(src.size, self.n_u)
        beta = np.empty((src.size, self.n_u))
        st = (Stats * max(1, src.size))()
        wi = (WarmInfo * max(1, src.size))()
        _check(_load().orc_approx_bhpp_warm_many(self._h, src.size, _ptr(src), alpha, eps, eps_b, lam, _ptr(y0),
                                                 _ptr(beta), ctypes.cast(st, ctypes.c_void_p),
                                                 ctypes.cast(wi, ctypes.c_void_p), int(nthreads)))
        return beta, [st[i].as_dict() for i in range(src.size)], [wi[i].as_dict() for i in range(src.size)]


def philox4x32_10(ctr, key):
    """One block of Philox4x32-10: four 32-bit counters and two 32-bit key
    words in, four 32-bit numbers out."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def mc_walks(n_u, eps_f, p_f):
    """MonteCarlo's walk count for an eps_f error with failure probability p_f."""
    return int(_load().orc_mc_walks(int(n_u), eps_f, p_f))


def max_threads() -> int:
    return int(_load().orc_max_threads())


# ---------------------------------------------------------------------------
# O-exact by a dense solve (tiny graphs only)
# ---------------------------------------------------------------------------

def dense_P(n_u, n_v, eu, ev, w):
    """Eq. (pmatrix): P = D_U^-1 W D_V^-1 W^T, formed densely. Rows of isolated
    U nodes are zero. Duplicate pairs add their weights."""
    W = np.zeros((n_u, n_v))
    np.add.at(W, (np.asarray(eu), np.asarray(ev)), np.asarray(w, dtype=np.float64))
    ws_u, ws_v = W.sum(1), W.sum(0)
    inv_u = np.divide(1.0, ws_u, out=np.zeros_like(ws_u), where=ws_u > 0)
    inv_v = np.divide(1.0, ws_v, out=np.zeros_like(ws_v), where=ws_v > 0)
    Um = W * inv_u[:, None]        # forward transition U (Sec. 3.1)
    Vm = W.T * inv_v[:, None]      # backward transition V
    return Um @ Vm, ws_u


def exact_dense(n_u, n_v, eu, ev, w, alpha):
    """Pi with Pi[i, j] = pi(i, j) = sum_l alpha (1-alpha)^l P^l (Eq. (hpp)),
    i.e. alpha (I - (1-alpha) P)^-1, plus ws_u."""
    P, ws_u = dense_P(n_u, n_v, eu, ev, w)
    A = np.eye(n_u) - (1.0 - alpha) * P
    Pi = np.linalg.solve(A, alpha * np.eye(n_u))
    return Pi, P, ws_u


def bhpp_from_dense(Pi, u):
    """beta(u, x) = pi(u, x) + pi(x, u) for all x (Sec. 3.2)."""
    return Pi[u, :] + Pi[:, u]


# ---------------------------------------------------------------------------
# Brute-force top-k
# ---------------------------------------------------------------------------

def topk_bruteforce(scores, k, exclude=-1):
    """The k best entries ordered by (score descending, id ascending), with -0
    treated as +0 and ``exclude`` (if >= 0) left out. Full sort, no selection."""
    s = np.asarray(scores).copy()
    s[s == 0] = 0.0
    ids = np.arange(s.size)
    keep = ids != exclude
    s, ids = s[keep], ids[keep]
    order = np.lexsort((ids, -s))
    order = order[:k]
    return ids[order].astype(np.int32), s[order]


def t_of(sum_rf, eps_f, alpha):
    """Eq. (t) as the C oracle rounds it (up, clamped at 0)."""
    return int(_load().orc_t(sum_rf, eps_f, alpha))
