"""MI355X (gfx950) approximate BHPP queries: Python binding of libbhpp.so.

The binding only marshals arguments: device buffers come from PyTorch tensors
(``data_ptr``) and work is enqueued on torch's current HIP stream. Every step
of the computation runs in the HIP kernels of ``csrc/``; there is no CPU
fallback. Importing works without a GPU (for symbol checks); any call that
needs the device fails loudly when the library or the GPU is missing.

Method: Yang, "Efficient and Effective Similarity Search over Bipartite
Graphs", WWW '22 (Algorithms 1-5).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libbhpp.so")

STATUS = {0: "ok", -1: "invalid argument", -2: "node id out of range", -3: "source node has no edge",
          -4: "edge weight not finite and positive", -5: "out of memory", -6: "HIP device error",
          -7: "not supported", -8: "step limit reached"}

DTYPE_F32, DTYPE_F64 = 0, 1
BUILD_KEEP_EXTERNAL, BUILD_NO_REORDER, BUILD_DENSE_ONLY, BUILD_FIXED_WIDTH, BUILD_MCSP = 1, 2, 4, 8, 16

# names exported by include/bhpp.h
EXPORTED = ["bhpp_build_graph", "bhpp_query", "bhpp_query_batch", "bhpp_topk", "bhpp_topk_noalloc", "bhpp_graph_info",
            "bhpp_graph_export", "bhpp_profile_enable", "bhpp_profile_read", "bhpp_profile_sweeps", "bhpp_autotune",
            "bhpp_set_launch_config", "bhpp_get_launch_config", "bhpp_set_schedule", "bhpp_get_schedule", "bhpp_server_create", "bhpp_server_submit",
            "bhpp_server_poll", "bhpp_server_info", "bhpp_server_destroy", "bhpp_model_create", "bhpp_model_params",
            "bhpp_model_features", "bhpp_model_loss_grad", "bhpp_model_train", "bhpp_model_embed", "bhpp_model_predict",
            "bhpp_model_free",
            "bhpp_query_batch_warm", "bhpp_query_batch_start", "bhpp_gemm_bf16", "bhpp_set_eps_b_ratio",
            "bhpp_tune_eps_b", "bhpp_query_hpp", "bhpp_query_batch_pisp", "bhpp_query_batch_mcsp", "bhpp_free_graph",
            "bhpp_status_string"]
MODEL_PARAMS = 230656
MODEL_FEATURES = 64


class BhppError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} ({code})")


class GraphOpts(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("tau", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class QueryStats(ctypes.Structure):
    _fields_ = [("ss_sel_iters", ctypes.c_int32), ("ss_seq_iters", ctypes.c_int32),
                ("pi_sel_iters", ctypes.c_int32), ("t", ctypes.c_int32),
                ("ss_switched", ctypes.c_int32), ("pi_returned", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("sparse_sweeps", ctypes.c_int32),
                ("np_ss", ctypes.c_double), ("np_pi", ctypes.c_double), ("gamma", ctypes.c_double),
                ("sum_r_ss", ctypes.c_double), ("sum_rf", ctypes.c_double),
                ("visits_u", ctypes.c_double), ("visits_v", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class GraphSummary(ctypes.Structure):
    _fields_ = [("n_u", ctypes.c_int32), ("n_v", ctypes.c_int32), ("n_edges", ctypes.c_int64),
                ("isolated_u", ctypes.c_int32), ("isolated_v", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("tau", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("lambda_", ctypes.c_double), ("mu", ctypes.c_double),
                ("eps_b_ratio", ctypes.c_double), ("ws_u_max", ctypes.c_double),
                ("ws_u_min", ctypes.c_double), ("build_ms", ctypes.c_double)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["lambda"] = d.pop("lambda_")
        return d


class WarmStats(ctypes.Structure):
    _fields_ = [("res_l1", ctypes.c_double), ("res_max", ctypes.c_double), ("fell_back", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return dict(res_l1=self.res_l1, res_max=self.res_max, fell_back=self.fell_back)


class ServerSummary(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("k", ctypes.c_int32), ("queued", ctypes.c_int64),
                ("running", ctypes.c_int64), ("completed", ctypes.c_int64), ("sweeps", ctypes.c_int64),
                ("resident_bytes", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("warm_started", ctypes.c_int64), ("warm_fell_back", ctypes.c_int64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["lambda"] = d.pop("lambda_")
        return d


_lib = None


def load_library():
    """Load libbhpp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() or "
                           "python paper_2312_06724_amd/build_lib.py")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.bhpp_build_graph.restype = I32
    L.bhpp_build_graph.argtypes = [I32, I32, I64, P, P, P, ctypes.POINTER(GraphOpts), P, ctypes.POINTER(P)]
    L.bhpp_query.restype = I32
    L.bhpp_query.argtypes = [P, I32, D, D, P, ctypes.POINTER(QueryStats), P]
    L.bhpp_query_batch.restype = I32
    L.bhpp_query_batch.argtypes = [P, I32, P, P, D, D, P, I32, I32, P, P, P, P]
    L.bhpp_query_batch_pisp.restype = I32
    L.bhpp_query_batch_pisp.argtypes = [P, I32, P, P, D, D, P, I32, I32, P, P, P, P]
    L.bhpp_query_batch_mcsp.restype = I32
    L.bhpp_query_batch_mcsp.argtypes = [P, I32, P, D, D, D, ctypes.c_uint64, P, I32, I32, P, P, P, P, P]
    L.bhpp_topk.restype = I32
    L.bhpp_topk.argtypes = [P, I32, I32, I32, P, I32, P, P, P]
    L.bhpp_topk_noalloc.restype = I32
    L.bhpp_topk_noalloc.argtypes = [P, I32, I32, I32, P, I32, P, P, P]
    L.bhpp_graph_info.restype = I32
    L.bhpp_graph_info.argtypes = [P, ctypes.POINTER(GraphSummary)]
    L.bhpp_graph_export.restype = I32
    L.bhpp_graph_export.argtypes = [P] * 9 + [P]
    L.bhpp_profile_enable.restype = I32
    L.bhpp_profile_enable.argtypes = [P, I32]
    L.bhpp_profile_read.restype = I32
    L.bhpp_profile_read.argtypes = [P, P, P, P]
    L.bhpp_profile_sweeps.restype = I32
    L.bhpp_profile_sweeps.argtypes = [P, P]
    L.bhpp_autotune.restype = I32
    L.bhpp_autotune.argtypes = [P, P, P]
    L.bhpp_set_launch_config.restype = I32
    L.bhpp_set_launch_config.argtypes = [P, P]
    L.bhpp_get_launch_config.restype = I32
    L.bhpp_get_launch_config.argtypes = [P, P]
    L.bhpp_set_schedule.restype = I32
    L.bhpp_set_schedule.argtypes = [P, P]
    L.bhpp_get_schedule.restype = I32
    L.bhpp_get_schedule.argtypes = [P, P]
    L.bhpp_server_create.restype = I32
    L.bhpp_server_create.argtypes = [P, P, I32, D, D, I32, I32, ctypes.POINTER(P)]
    L.bhpp_server_submit.restype = I32
    L.bhpp_server_submit.argtypes = [P, I32, D, I64]
    L.bhpp_server_poll.restype = I32
    L.bhpp_server_poll.argtypes = [P, I32, P, P, P, P, P, P]
    L.bhpp_model_create.restype = I32
    L.bhpp_model_create.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(P)]
    L.bhpp_model_params.restype = I32
    L.bhpp_model_params.argtypes = [P, P, P, P, P]
    L.bhpp_model_features.restype = I32
    L.bhpp_model_features.argtypes = [P, P, P]
    L.bhpp_model_loss_grad.restype = I32
    L.bhpp_model_loss_grad.argtypes = [P, I32, P, I32, P, P, P, P]
    L.bhpp_model_train.restype = I32
    L.bhpp_model_train.argtypes = [P, I32, P, I32, P, P, I32, I32, I32, D, ctypes.c_uint64, P]
    L.bhpp_model_embed.restype = I32
    L.bhpp_model_embed.argtypes = [P]
    L.bhpp_model_predict.restype = I32
    L.bhpp_model_predict.argtypes = [P, I32, P, P, P]
    L.bhpp_model_free.restype = None
    L.bhpp_model_free.argtypes = [P]
    L.bhpp_query_batch_warm.restype = I32
    L.bhpp_query_batch_warm.argtypes = [P, P, I32, P, P, D, D, P, I32, I32, P, P, P, P, P]
    L.bhpp_query_batch_start.restype = I32
    L.bhpp_query_batch_start.argtypes = [P, P, I32, P, P, D, D, P, I32, I32, P, P, P, P, P]
    L.bhpp_set_eps_b_ratio.restype = I32
    L.bhpp_set_eps_b_ratio.argtypes = [P, D]
    L.bhpp_tune_eps_b.restype = I32
    L.bhpp_tune_eps_b.argtypes = [P, I32, P, D, D, I32, P, P, P, P, P, P]
    L.bhpp_query_hpp.restype = I32
    L.bhpp_query_hpp.argtypes = [P, I32, P, P, D, D, I32, P, P, P]
    L.bhpp_gemm_bf16.restype = I32
    L.bhpp_gemm_bf16.argtypes = [I32, I32, I32, P, I32, P, I32, P, P]
    L.bhpp_server_info.restype = I32
    L.bhpp_server_info.argtypes = [P, ctypes.POINTER(ServerSummary)]
    L.bhpp_server_destroy.restype = None
    L.bhpp_server_destroy.argtypes = [P]
    L.bhpp_free_graph.restype = None
    L.bhpp_free_graph.argtypes = [P]
    L.bhpp_status_string.restype = ctypes.c_char_p
    L.bhpp_status_string.argtypes = [I32]
    _lib = L
    return L


def _check(rc, where):
    if rc != 0:
        raise BhppError(rc, where)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the BHPP library runs on the GPU only")
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x, dtype):
    """A contiguous device tensor of `dtype` holding x (numpy or tensor)."""
    torch = _torch()
    if isinstance(x, torch.Tensor):
        return x.to(device="cuda", dtype=dtype).contiguous()
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


class Graph:
    """A built bipartite graph resident in HBM (bhpp_build_graph)."""

    def __init__(self, n_u, n_v, edge_u, edge_v, edge_w, alpha=0.15, dtype="f32", tau=-1,
                 keep_external=False, reorder=True, sparse=True, fixed_width=False, mcsp=False):
        torch = _torch()
        L = load_library()
        self.dtype = dtype
        self._tdtype = torch.float64 if dtype == "f64" else torch.float32
        eu = _dev(edge_u, torch.int32)
        ev = _dev(edge_v, torch.int32)
        ew = _dev(edge_w, self._tdtype)
        flags = ((BUILD_KEEP_EXTERNAL if keep_external else 0) | (0 if reorder else BUILD_NO_REORDER) |
                 (0 if sparse else BUILD_DENSE_ONLY) | (BUILD_FIXED_WIDTH if fixed_width else 0) |
                 (BUILD_MCSP if mcsp else 0))
        opts = GraphOpts(alpha, tau, DTYPE_F64 if dtype == "f64" else DTYPE_F32, flags)
        h = ctypes.c_void_p()
        rc = L.bhpp_build_graph(n_u, n_v, eu.numel(), eu.data_ptr(), ev.data_ptr(), ew.data_ptr(),
                                ctypes.byref(opts), _stream(), ctypes.byref(h))
        _check(rc, "bhpp_build_graph")
        self._h = h
        self.n_u, self.n_v = int(n_u), int(n_v)
        self.alpha = alpha

    @classmethod
    def from_edges(cls, el, **kw):
        return cls(el.n_u, el.n_v, el.u, el.v, el.w, **kw)

    def close(self):
        if getattr(self, "_h", None):
            load_library().bhpp_free_graph(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        s = GraphSummary()
        _check(load_library().bhpp_graph_info(self._h, ctypes.byref(s)), "bhpp_graph_info")
        return s.as_dict()

    def export(self):
        """External-id adjacency and ws (needs keep_external=True)."""
        torch = _torch()
        inf = self.info()
        m = inf["n_edges"]
        out = dict(rp_u=torch.empty(self.n_u + 1, dtype=torch.int64, device="cuda"),
                   ci_u=torch.empty(max(m, 1), dtype=torch.int32, device="cuda"),
                   w_u=torch.empty(max(m, 1), dtype=self._tdtype, device="cuda"),
                   rp_v=torch.empty(self.n_v + 1, dtype=torch.int64, device="cuda"),
                   ci_v=torch.empty(max(m, 1), dtype=torch.int32, device="cuda"),
                   w_v=torch.empty(max(m, 1), dtype=self._tdtype, device="cuda"),
                   ws_u=torch.empty(self.n_u, dtype=self._tdtype, device="cuda"),
                   ws_v=torch.empty(self.n_v, dtype=self._tdtype, device="cuda"))
        keys = ("rp_u", "ci_u", "w_u", "rp_v", "ci_v", "w_v", "ws_u", "ws_v")
        rc = load_library().bhpp_graph_export(self._h, *[out[k].data_ptr() for k in keys], _stream())
        _check(rc, "bhpp_graph_export")
        for k in ("ci_u", "w_u", "ci_v", "w_v"):
            out[k] = out[k][:m]
        return out

    def query(self, source, eps, alpha=None, with_stats=True):
        """One query (bhpp_query): beta'(u, x) for every x, as a device tensor."""
        torch = _torch()
        out = torch.empty(self.n_u, dtype=self._tdtype, device="cuda")
        st = QueryStats()
        rc = load_library().bhpp_query(self._h, int(source), alpha or self.alpha, eps, out.data_ptr(),
                                       ctypes.byref(st), _stream())
        _check(rc, "bhpp_query")
        return (out, st.as_dict()) if with_stats else out

    def query_batch(self, sources, eps, alpha=None, k=0, exclude_self=True, scores=True, stats=True, model=None,
                    starts=None, method="approx"):
        """Many queries (bhpp_query_batch; bhpp_query_batch_warm with a Model;
        bhpp_query_batch_start with starts = [n, n_u] estimates of pi(u, x);
        bhpp_query_batch_pisp with method="pisp", the paper's PISP baseline).
        ``eps`` is a float or one per source. Returns dict(scores=[n, n_u]
        tensor or None, ids, vals, stats, warm)."""
        torch = _torch()
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
        n = src.size
        eps_arr = np.broadcast_to(np.asarray(eps, dtype=np.float64), (n,)).copy()
        sc = torch.empty((n, self.n_u), dtype=self._tdtype, device="cuda") if scores else None
        ids = torch.empty((n, k), dtype=torch.int32, device="cuda") if k else None
        vals = torch.empty((n, k), dtype=self._tdtype, device="cuda") if k else None
        st = (QueryStats * max(1, n))()
        common = (n, src.ctypes.data, eps_arr.ctypes.data, alpha or self.alpha, (float(eps_arr[0]) if n else 0.0),
                  sc.data_ptr() if sc is not None else None, int(k), 1 if exclude_self else 0,
                  ids.data_ptr() if ids is not None else None, vals.data_ptr() if vals is not None else None,
                  ctypes.cast(st, ctypes.c_void_p) if stats else None)
        warm = None
        if starts is not None:
            st0 = _dev(starts, self._tdtype)
            assert tuple(st0.shape) == (n, self.n_u)
            ws = (WarmStats * max(1, n))()
            rc = load_library().bhpp_query_batch_start(self._h, st0.data_ptr(), *common,
                                                       ctypes.cast(ws, ctypes.c_void_p), _stream())
            _check(rc, "bhpp_query_batch_start")
            warm = [ws[i].as_dict() for i in range(n)]
        elif method == "pisp":
            rc = load_library().bhpp_query_batch_pisp(self._h, *common, _stream())
            _check(rc, "bhpp_query_batch_pisp")
        elif model is None:
            rc = load_library().bhpp_query_batch(self._h, *common, _stream())
            _check(rc, "bhpp_query_batch")
        else:
            ws = (WarmStats * max(1, n))()
            rc = load_library().bhpp_query_batch_warm(self._h, model._h, *common, ctypes.cast(ws, ctypes.c_void_p),
                                                      _stream())
            _check(rc, "bhpp_query_batch_warm")
            warm = [ws[i].as_dict() for i in range(n)]
        return dict(scores=sc, ids=ids, vals=vals, stats=[st[i].as_dict() for i in range(n)] if stats else None,
                    warm=warm)

    def query_mcsp(self, sources, eps, alpha=None, p_f=1e-6, seed=0, k=0, exclude_self=True, scores=True,
                   stats=True):
        """The MCSP baseline (bhpp_query_batch_mcsp; the graph needs mcsp=True).
        Returns dict(scores, ids, vals, stats, walks)."""
        torch = _torch()
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
        n = src.size
        sc = torch.empty((n, self.n_u), dtype=self._tdtype, device="cuda") if scores else None
        ids = torch.empty((n, k), dtype=torch.int32, device="cuda") if k else None
        vals = torch.empty((n, k), dtype=self._tdtype, device="cuda") if k else None
        st = (QueryStats * max(1, n))()
        walks = ctypes.c_int64()
        rc = load_library().bhpp_query_batch_mcsp(
            self._h, n, src.ctypes.data, float(eps), alpha or self.alpha, float(p_f), ctypes.c_uint64(seed),
            sc.data_ptr() if sc is not None else None, int(k), 1 if exclude_self else 0,
            ids.data_ptr() if ids is not None else None, vals.data_ptr() if vals is not None else None,
            ctypes.cast(st, ctypes.c_void_p) if stats else None, ctypes.byref(walks), _stream())
        _check(rc, "bhpp_query_batch_mcsp")
        return dict(scores=sc, ids=ids, vals=vals, stats=[st[i].as_dict() for i in range(n)] if stats else None,
                    walks=int(walks.value))

    def autotune(self, cache_path=None):
        """Pick the fastest launch setting for this graph (bhpp_autotune) and
        remember it in a JSON cache keyed by the graph's shape, so later builds
        of the same graph can reuse it with apply_cached_config()."""
        import json
        cfg = (ctypes.c_int32 * 4)()
        _check(load_library().bhpp_autotune(self._h, _stream(), cfg), "bhpp_autotune")
        out = dict(tile_edges=cfg[0], inflight=cfg[1], nt_stream=cfg[2], graphs=cfg[3])
        if cache_path:
            data = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
            data[self.cache_key()] = out
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
        return out

    def cache_key(self):
        inf = self.info()
        return f"{inf['n_u']}x{inf['n_v']}x{inf['n_edges']}:{self.dtype}"

    def apply_cached_config(self, cache_path):
        import json
        if not os.path.exists(cache_path):
            return None
        ent = json.load(open(cache_path)).get(self.cache_key())
        if ent:
            self.set_launch_config(ent)
        return ent

    def set_launch_config(self, cfg):
        arr = (ctypes.c_int32 * 4)(cfg["tile_edges"], cfg["inflight"], cfg["nt_stream"], cfg["graphs"])
        _check(load_library().bhpp_set_launch_config(self._h, arr), "bhpp_set_launch_config")

    def schedule(self):
        """(sweeps per chunk, asynchronous admission) of query batches."""
        a = (ctypes.c_int32 * 2)()
        _check(load_library().bhpp_get_schedule(self._h, a), "bhpp_get_schedule")
        return dict(chunk_sweeps=a[0], async_admission=a[1])

    def set_schedule(self, chunk_sweeps, async_admission=True):
        a = (ctypes.c_int32 * 2)(int(chunk_sweeps), 1 if async_admission else 0)
        _check(load_library().bhpp_set_schedule(self._h, a), "bhpp_set_schedule")

    def launch_config(self):
        cfg = (ctypes.c_int32 * 4)()
        _check(load_library().bhpp_get_launch_config(self._h, cfg), "bhpp_get_launch_config")
        return dict(tile_edges=cfg[0], inflight=cfg[1], nt_stream=cfg[2], graphs=cfg[3])

    def query_hpp(self, sources, eps, direction="forward", alpha=None, stats=True):
        """One direction of HPP (bhpp_query_hpp): "forward" pi(u, .) or
        "backward" pi(., u) for each source; returns ([n, n_u] tensor, stats)."""
        torch = _torch()
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
        n = src.size
        eps_arr = np.broadcast_to(np.asarray(eps, dtype=np.float64), (n,)).copy()
        out = torch.empty((n, self.n_u), dtype=self._tdtype, device="cuda")
        st = (QueryStats * max(1, n))()
        d = {"forward": 0, "backward": 1}[direction]
        rc = load_library().bhpp_query_hpp(self._h, n, src.ctypes.data, eps_arr.ctypes.data, alpha or self.alpha,
                                           (float(eps_arr[0]) if n else 0.0), d, out.data_ptr(),
                                           ctypes.cast(st, ctypes.c_void_p) if stats else None, _stream())
        _check(rc, "bhpp_query_hpp")
        return out, ([st[i].as_dict() for i in range(n)] if stats else None)

    def set_eps_b_ratio(self, ratio):
        """eps_b = ratio * eps for later queries; 0 restores Eq. (epsilon-b)."""
        _check(load_library().bhpp_set_eps_b_ratio(self._h, float(ratio)), "bhpp_set_eps_b_ratio")

    def tune_eps_b(self, sources, eps, ratios, alpha=None, curve=False):
        """Time the sample once per candidate ratio, keep the fastest;
        returns (best ratio, ms per candidate[, mean gamma, mean sweeps])."""
        src = np.ascontiguousarray(sources, dtype=np.int32)
        r = np.ascontiguousarray(ratios, dtype=np.float64)
        ms, gm, sw = np.zeros(r.size), np.zeros(r.size), np.zeros(r.size)
        best = ctypes.c_double()
        _check(load_library().bhpp_tune_eps_b(self._h, src.size, src.ctypes.data, float(eps), alpha or self.alpha,
                                              r.size, r.ctypes.data, ms.ctypes.data, gm.ctypes.data, sw.ctypes.data,
                                              ctypes.byref(best), _stream()), "bhpp_tune_eps_b")
        return (best.value, ms, gm, sw) if curve else (best.value, ms)

    def profile(self, enable):
        _check(load_library().bhpp_profile_enable(self._h, 1 if enable else 0), "bhpp_profile_enable")

    def profile_read(self):
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_int64 * 4)()
        b = (ctypes.c_double * 4)()
        _check(load_library().bhpp_profile_read(self._h, ms, n, b), "bhpp_profile_read")
        live = ctypes.c_int64()
        _check(load_library().bhpp_profile_sweeps(self._h, ctypes.byref(live)), "bhpp_profile_sweeps")
        return dict(ms=list(ms), launches=list(n), bytes=list(b), live_sweeps=int(live.value))


class Server:
    """A resident query block fed by a request queue (bhpp_server_*):
    continuous batching of top-k queries on one graph."""

    def __init__(self, graph, k=100, max_width=64, mem_budget_bytes=0.0, alpha=None, exclude_self=True, model=None):
        _torch()
        L = load_library()
        h = ctypes.c_void_p()
        rc = L.bhpp_server_create(graph._h, model._h if model is not None else None, int(max_width),
                                  float(mem_budget_bytes), alpha or graph.alpha, int(k), 1 if exclude_self else 0,
                                  ctypes.byref(h))
        _check(rc, "bhpp_server_create")
        self._h = h
        self.graph = graph          # keeps the graph (and model) alive while the server exists
        self.model = model
        self.k = int(k)
        self.width = self.info()["width"]
        self._vdt = np.float64 if graph.dtype == "f64" else np.float32
        self._tags = np.empty(self.width, dtype=np.int64)
        self._ids = np.empty((self.width, self.k), dtype=np.int32)
        self._vals = np.empty((self.width, self.k), dtype=self._vdt)
        self._st = (QueryStats * self.width)()
        self._ws = (WarmStats * self.width)()

    def submit(self, source, eps, tag):
        _check(load_library().bhpp_server_submit(self._h, int(source), float(eps), int(tag)), "bhpp_server_submit")

    def poll(self, stats=False):
        """Run one chunk; returns [(tag, ids, vals[, stats])] of the finished
        requests (stats includes the warm-start report when there is a model)."""
        n = ctypes.c_int32()
        rc = load_library().bhpp_server_poll(self._h, self.width, self._tags.ctypes.data, self._ids.ctypes.data,
                                             self._vals.ctypes.data, ctypes.cast(self._st, ctypes.c_void_p),
                                             ctypes.cast(self._ws, ctypes.c_void_p), ctypes.byref(n))
        _check(rc, "bhpp_server_poll")
        out = []
        for j in range(n.value):
            r = (int(self._tags[j]), self._ids[j].copy(), self._vals[j].copy())
            if stats:
                d = self._st[j].as_dict()
                if self.model is not None:
                    d.update(self._ws[j].as_dict())
                r = r + (d,)
            out.append(r)
        return out

    def info(self):
        s = ServerSummary()
        _check(load_library().bhpp_server_info(self._h, ctypes.byref(s)), "bhpp_server_info")
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load_library().bhpp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """The warm-start network of a graph (bhpp_model_*): features, two BF16
    towers trained on the GPU, node embeddings."""

    def __init__(self, graph, seed=0):
        _torch()
        h = ctypes.c_void_p()
        _check(load_library().bhpp_model_create(graph._h, ctypes.c_uint64(seed), ctypes.byref(h)), "bhpp_model_create")
        self._h = h
        self.graph = graph

    def params(self):
        out = np.empty(MODEL_PARAMS, dtype=np.float32)
        _check(load_library().bhpp_model_params(self._h, out.ctypes.data, None, None, None), "bhpp_model_params")
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        assert theta.size == MODEL_PARAMS
        _check(load_library().bhpp_model_params(self._h, None, theta.ctypes.data, None, None), "bhpp_model_params")

    def scales(self):
        c, sg = ctypes.c_double(), ctypes.c_double()
        _check(load_library().bhpp_model_params(self._h, None, None, ctypes.byref(c), ctypes.byref(sg)),
               "bhpp_model_params")
        return c.value, sg.value

    def features(self):
        torch = _torch()
        out = torch.empty((self.graph.n_u, MODEL_FEATURES), dtype=torch.float32, device="cuda")
        _check(load_library().bhpp_model_features(self._h, out.data_ptr(), _stream()), "bhpp_model_features")
        torch.cuda.synchronize()
        return out

    def loss_grad(self, src, cand, targets, want_grad=True):
        src = np.ascontiguousarray(src, dtype=np.int32)
        cand = np.ascontiguousarray(cand, dtype=np.int32)
        T = np.ascontiguousarray(targets, dtype=np.float32).reshape(src.size, cand.size)
        loss = ctypes.c_double()
        g = np.empty(MODEL_PARAMS, dtype=np.float32) if want_grad else None
        _check(load_library().bhpp_model_loss_grad(self._h, src.size, src.ctypes.data, cand.size, cand.ctypes.data,
                                                   T.ctypes.data, ctypes.byref(loss),
                                                   g.ctypes.data if g is not None else None), "bhpp_model_loss_grad")
        return loss.value, g

    def train(self, src, ids, vals, steps, batch_src=32, batch_cand=4096, lr=1e-3, seed=1):
        src = np.ascontiguousarray(src, dtype=np.int32)
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        vals = np.ascontiguousarray(vals, dtype=np.float32)
        M = ids.shape[1]
        losses = np.empty(max(1, steps), dtype=np.float32)
        _check(load_library().bhpp_model_train(self._h, src.size, src.ctypes.data, M, ids.ctypes.data,
                                               vals.ctypes.data, int(steps), int(batch_src), int(batch_cand),
                                               float(lr), ctypes.c_uint64(seed), losses.ctypes.data),
               "bhpp_model_train")
        return losses[:steps]

    def predict(self, sources):
        """The model's start for each source (bhpp_model_predict): [n, n_u]
        device FP32 estimates of pi(u, x)."""
        torch = _torch()
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
        out = torch.empty((src.size, self.graph.n_u), dtype=torch.float32, device="cuda")
        _check(load_library().bhpp_model_predict(self._h, src.size, src.ctypes.data, out.data_ptr(), _stream()),
               "bhpp_model_predict")
        return out

    def embed(self):
        _check(load_library().bhpp_model_embed(self._h), "bhpp_model_embed")

    def close(self):
        if getattr(self, "_h", None):
            load_library().bhpp_model_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm_bf16(A, B, trans_a=False, trans_b=False):
    """bhpp_gemm_bf16 on device bf16 tensors: A @ B in FP32 (operands given
    transposed when trans_a / trans_b)."""
    torch = _torch()
    A = A.contiguous()
    B = B.contiguous()
    M, K = (A.shape[1], A.shape[0]) if trans_a else A.shape
    N = B.shape[0] if trans_b else B.shape[1]
    C = torch.empty((M, N), dtype=torch.float32, device="cuda")
    _check(load_library().bhpp_gemm_bf16(M, N, K, A.data_ptr(), 1 if trans_a else 0, B.data_ptr(),
                                         1 if trans_b else 0, C.data_ptr(), _stream()), "bhpp_gemm_bf16")
    return C


def topk(scores, k, exclude=None):
    """bhpp_topk on a [rows, n] device tensor: (ids int32, vals)."""
    torch = _torch()
    scores = scores.contiguous()
    if scores.dim() == 1:
        scores = scores[None, :]
    rows, n = scores.shape
    dt = DTYPE_F64 if scores.dtype == torch.float64 else DTYPE_F32
    ids = torch.empty((rows, k), dtype=torch.int32, device="cuda")
    vals = torch.empty((rows, k), dtype=scores.dtype, device="cuda")
    ex = _dev(exclude, torch.int32) if exclude is not None else None
    rc = load_library().bhpp_topk(scores.data_ptr(), rows, n, k, ex.data_ptr() if ex is not None else None,
                                  dt, ids.data_ptr(), vals.data_ptr(), _stream())
    _check(rc, "bhpp_topk")
    return ids, vals
