"""Benchmark: approximate BHPP queries per second on one MI355X.

Headline workload (one "step"): 256 query sources run as one batch through
the queue-fed 64-column residue block, on a seeded Chung-Lu bipartite graph
with |U| = 5M, |V| = 10M, 100M edges, degree exponent 2.1, lognormal(0,1)
weights. The sources are a fixed set of 1,024 non-isolated U nodes drawn with
probability proportional to degree (their frontiers differ by more than
1000x); step i runs quarter (i mod 4) of the set, so every four steps cover
all 1,024. alpha = 0.15, eps = 1e-6; each query runs Algorithm 5 and returns
its top-100 (FP32 values and accumulation). Inputs are resident in HBM before
timing starts.

Prints ONE JSON line. Besides the headline it reports the roofline of the
dominant kernel (HIP events on the query stream over the timed steps, bytes
counted in edge visits from the queries' own counters), the FP64 CPU oracle
timed on a bounded sample of the same queries, the plain single-source GPU
path on the same graph, and, on the 1M x 2M graph (the learned start's and
the serving workload's graph): plain batched and single-source queries, the
eps_b split tuning, the learned warm start and continuous-batching serving.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
KINDS = ["gather_a", "gather_b", "update", "select"]
KIND_NAMES = ["V-side gather with the push rule (k_gather64, SIDE_A)", "U-side gather (k_gather64)",
              "U-side update (k_update)", "push selection (k_select)"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_digest(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = int(omp) if omp and omp.isdigit() and int(omp) > 0 else aff
    return dict(cpu_model=model, nproc=os.cpu_count(), affinity=aff, threads=min(threads, aff))


def stored_traffic(workload, kernel):
    """HBM bytes per launch (mean over the profiled dispatches) from rocprofv3
    FETCH_SIZE/WRITE_SIZE, if the counters were taken on the current kernel
    source for this workload."""
    p = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    cur = source_digest(os.path.join(ROOT, "paper_2312_06724_amd", "csrc", "sweep.hip"))
    ent = d.get(workload, {}).get(kernel)
    if not ent or ent.get("sweep_hip_sha") != cur:
        return None
    return ent.get("bytes_per_launch")


def copy_ceiling(torch):
    """Read + write GB/s of a 1 GiB device-to-device copy (best of 10 timed on
    the copy's own stream): the streaming rate the memory system sustains."""
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2.0 * (1 << 30) / (best * 1e-3) / 1e9


def roofline(prof, stats, info, workload):
    """Roofline of the dominant sweep kernel over the timed steps.

    Unit of work: the edge visit, the increment of the push cost n_p in
    Algorithms 3 and 4, counted by the queries themselves over every sweep
    (visits_u: edges of the pushed U nodes, the entries the V-side gather
    reads with a non-zero value; visits_v: edges of the V nodes with a
    non-zero residue, read by the U-side gather). Algorithmic bytes:
      structure: 8 B per adjacency entry (index + weight) and 8 B per row
                 (offsets) for every sweep in which a query ran (the block
                 shares one adjacency read among its columns);
      visits:    4 B per visit (the neighbour's value);
      outputs:   4 B per output row and running column (column-sweeps).
    The update reads degree and 1/ws once per sweep (8 B per node) and per
    node and running column reads y, ACC, G and writes y, ACC (20 B); fused
    into the U-side gather it drops G (the gather's output row) and keeps
    16 B per node and column.
    Each gather read counts as a memory read (no reuse); the per-entry 1/ws
    the V-side gather streams beside the adjacency is overhead, not counted.
    """
    import numpy as np
    E = float(info["n_edges"])
    U1 = float(info["n_u"] - info["isolated_u"])
    V1 = float(info["n_v"] - info["isolated_v"])
    L = float(prof["live_sweeps"])
    CS = float(sum(s["steps"] for s in stats))
    VU = float(sum(s["visits_u"] for s in stats))
    VV = float(sum(s["visits_v"] for s in stats))
    alg = [L * (8 * E + 8 * V1) + 4 * VU + 4 * V1 * CS,
           L * (8 * E + 8 * U1) + 4 * VV + 4 * U1 * CS,
           L * 8 * U1 + 20 * U1 * CS,
           0.0]
    comp = [L * (8 * E + 8 * V1) + 4 * (U1 + V1) * CS,
            L * (8 * E + 8 * U1) + 4 * (U1 + V1) * CS,
            L * 8 * U1 + 20 * U1 * CS,
            0.0]
    # the U-side gather with the update fused (no update launches): it takes
    # on the update's node terms without G (8 B per node per sweep; read y,
    # ACC and write y, ACC: 16 B per node and column) and no longer writes
    # its G row (4 B per node and column)
    fused_update = prof["launches"][2] == 0 and prof["launches"][1] > 0
    if fused_update:
        alg[1] += L * 8 * U1 + 12 * U1 * CS
        comp[1] += L * 8 * U1 + 12 * U1 * CS
    dom = int(np.argmax(prof["ms"]))
    sec = prof["ms"][dom] * 1e-3
    launches = max(1, prof["launches"][dom])
    avg_ms = prof["ms"][dom] / launches
    achieved = alg[dom] / sec / 1e9
    paper_units = sum(s["np_ss"] + s["np_pi"] + 2 * E * s["t"] for s in stats)
    traffic = stored_traffic(workload, KINDS[dom])
    name = KIND_NAMES[dom]
    if dom == 1 and fused_update:
        name = "U-side gather with the update fused (k_gather64, UPD)"
    out = dict(bound="hbm", kernel=name, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
               frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
               avg_launch_ms=round(avg_ms, 4), launches=prof["launches"][dom], live_sweeps=int(L),
               algorithmic_bytes_per_launch=int(alg[dom] / launches),
               counts=dict(column_sweeps=int(CS), visits_u=VU, visits_v=VV, edge_visits=VU + VV,
                           paper_work_units=paper_units,
                           sparse_column_sweeps=int(sum(s["sparse_sweeps"] for s in stats)),
                           column_use=round(CS / max(1.0, 64.0 * L), 4)),
               compulsory=dict(bytes_per_launch=int(comp[dom] / launches), achieved=round(comp[dom] / sec / 1e9, 1),
                               frac=round(comp[dom] / sec / 1e9 / HBM_PEAK_GBS, 4)),
               kernels={k: dict(avg_ms=round(prof["ms"][i] / max(1, prof["launches"][i]), 4),
                                launches=prof["launches"][i],
                                gbs=round(alg[i] / (prof["ms"][i] * 1e-3) / 1e9, 1) if prof["ms"][i] > 0 else None)
                        for i, k in enumerate(KINDS) if prof["launches"][i] > 0})
    if traffic:
        out["traffic_gbs"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
    return out


def cpu_baseline(el, sources, wl, threads, work_per_query, iters):
    """The FP64 oracle (Algorithm 5 as it stands, one query per thread) on a
    bounded sample: the first `threads` sources of the set, each stopped after
    `iters` push iterations (a whole query takes minutes on this graph). The
    sample's rate of edge visits (the paper's work unit n_p, 2|E| per
    PowerIteration round) over all threads, divided by the mean work of a
    whole query of the same sources (from their GPU statistics: n_p of both
    sub-algorithms plus 2|E| t, the same iteration sequence), gives queries/s."""
    import oracle
    t0 = time.perf_counter()
    g = oracle.Graph.from_edges(el)
    # lambda only sets PI-Push's thresholds, which the sampled iterations
    # (SS-Push's first pushes) never reach: the ws-ratio branch of Eq. (lambda),
    # a valid bound by Lemma 4, spares the oracle's long power iteration
    ws = g.ws_u
    lam = float(ws.max() / ws[ws > 0].min())
    eps_b = g.eps_b(wl.eps)
    t_pre = time.perf_counter() - t0
    sample = sources[:threads]
    t0 = time.perf_counter()
    work = g.approx_bhpp_sample(sample, wl.alpha, wl.eps, iters, eps_b, lam, nthreads=threads)
    dt = time.perf_counter() - t0
    rate = float(work.sum()) / dt
    return dict(value=rate / work_per_query, unit="queries/s", cores=threads, kind="oracle",
                edge_visits_per_s=round(rate, 1), work_per_query=work_per_query,
                s_per_query_per_thread=round(work_per_query / (rate / threads), 1),
                sample=f"{len(sample)} of the {len(sources)} sources of {wl.name}, one query per thread, FP64 "
                       f"Approx-BHPP (Algorithms 1-5) stopped after {iters} push iterations: "
                       f"{work.sum():.4g} edge visits in {dt:.1f} s wall; a whole query of these sources does "
                       f"{work_per_query:.4g} (mean, from their GPU statistics); graph build, lambda and eps_b "
                       f"({t_pre:.1f} s) not timed")


def run_headline(bh, torch, np, args, hinfo):
    import synth
    wl = synth.LARGE
    t0 = time.perf_counter()
    el = wl.graph()
    src = wl.sources(el)
    log(f"graph {wl.name}: {el.n_e} edges generated in {time.perf_counter() - t0:.1f}s")
    G = bh.Graph.from_edges(el, alpha=wl.alpha, dtype="f32")
    info = G.info()
    if args.launch:
        t, i, n, c = (int(x) for x in args.launch.split(","))
        cfg = dict(tile_edges=t, inflight=i, nt_stream=n, graphs=1)
        G.set_launch_config(cfg)
        G.set_schedule(c)
    else:
        cfg = G.autotune()
    cfg.update(G.schedule())
    log(f"built on GPU in {info['build_ms']:.0f} ms; lambda={info['lambda']:.1f} "
        f"eps_b/eps={info['eps_b_ratio']:.4f}; autotuned {cfg}")
    per = args.sources_per_step
    parts = max(1, src.size // per)

    def step(i):
        part = src[(i % parts) * per:(i % parts + 1) * per]
        return G.query_batch(part, wl.eps, k=wl.k, exclude_self=True, scores=False, stats=True)

    G.profile(True)
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    G.profile(True)            # clears the totals
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        stats += step(i)["stats"]
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = G.profile_read()
    G.profile(False)
    qps = per * args.steps / dt
    roof = roofline(prof, stats, info, wl.name)
    roof["copy_gbs"] = round(copy_ceiling(torch), 1)
    if roof.get("traffic_gbs"):
        roof["traffic_frac_of_copy"] = round(roof["traffic_gbs"] / roof["copy_gbs"], 4)
    roof["share_of_step"] = round(sum(prof["ms"]) / (dt * 1e3), 3)
    log(f"headline {qps:.2f} q/s; dominant kernel {roof['kernel']} {roof['avg_launch_ms']} ms, "
        f"{roof['achieved']} GB/s (frac {roof['frac']}); copy {roof['copy_gbs']} GB/s")
    steps_q = np.array([s["steps"] for s in stats])
    single = None
    if args.single > 0:
        G.query(int(src[0]), wl.eps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for u in src[:args.single]:
            G.query(int(u), wl.eps, with_stats=False)
        torch.cuda.synchronize()
        single = args.single / (time.perf_counter() - t1)
        log(f"single-source on {wl.name}: {single:.2f} q/s")
    G.close()
    head = dict(value=qps, dt=dt, steps_q=steps_q, wl=wl, info=info, cfg=cfg, roof=roof, single=single,
                parts=parts)
    cpu = None
    if not args.no_cpu_baseline:
        n = args.cpu_threads or hinfo["threads"]
        E = float(info["n_edges"])
        # whole-query work of the sampled sources (the first n of the set), from the timed steps' statistics
        first = {int(u): s for u, s in zip(np.concatenate([src[(i % parts) * per:(i % parts + 1) * per]
                                                           for i in range(args.steps)]), stats)}
        w = [first[int(u)]["np_ss"] + first[int(u)]["np_pi"] + 2 * E * first[int(u)]["t"]
             for u in src[:n] if int(u) in first]
        if not w:
            w = [s["np_ss"] + s["np_pi"] + 2 * E * s["t"] for s in stats]
        log(f"CPU oracle baseline on {n} threads ...")
        cpu = cpu_baseline(el, src, wl, n, float(np.mean(w)), args.cpu_iters)
        cpu.update(cpu_model=hinfo["cpu_model"], nproc=hinfo["nproc"], affinity=hinfo["affinity"])
        log(f"CPU oracle: {cpu['value']:.4f} q/s")
    head["cpu"] = cpu
    return head


def run_learned(bh, torch, np, G, el, wl, src, n_train, steps, reps):
    """Learned warm start: training data from the plain GPU path (top-64 of
    beta' plus 64 random entries per source, for n_train uniform sources
    disjoint from the evaluation sources), GPU training, then the evaluation
    sources batched and warm-started, beside the no-network ablation (the
    structural self term alone)."""
    import synth
    live = np.nonzero(el.degrees_u() > 0)[0]
    rng = np.random.default_rng(77)
    cand = synth.sample_sources(el, n_train + src.size, "uniform", 4242)
    train = np.setdiff1d(cand, src)[:n_train].astype(np.int32)
    t0 = time.perf_counter()
    ids, vals = [], []
    for i in range(0, train.size, 64):
        chunk = train[i:i + 64]
        out = G.query_batch(chunk, wl.eps, k=64, exclude_self=False, scores=True, stats=False)
        r = torch.from_numpy(rng.choice(live, (chunk.size, 64))).to("cuda")
        rv = torch.gather(out["scores"], 1, r.long())
        ii = torch.cat([out["ids"], r.int()], 1).cpu().numpy()
        vv = torch.cat([out["vals"], rv], 1).cpu().numpy()
        for a, b in zip(ii, vv):
            _, keep = np.unique(a, return_index=True)
            a2 = np.full(128, -1, np.int32)
            b2 = np.zeros(128, np.float32)
            a2[:keep.size], b2[:keep.size] = a[keep], b[keep]
            ids.append(a2)
            vals.append(b2)
        del out
    t_data = time.perf_counter() - t0
    log(f"learned: training data from {train.size} plain queries in {t_data:.1f}s")
    t0 = time.perf_counter()
    M = bh.Model(G, seed=1)
    losses = M.train(train, np.array(ids), np.array(vals), steps=steps, batch_src=32, batch_cand=4096, lr=5e-4)
    M.embed()
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"learned: {steps} training steps + embedding in {t_train:.1f}s, loss {losses[:50].mean():.3g} -> "
        f"{losses[-50:].mean():.3g}")

    def timed(model):
        model_q = lambda: G.query_batch(src, wl.eps, k=wl.k, exclude_self=True, scores=True, stats=True, model=model)
        model_q()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            o = model_q()
        torch.cuda.synchronize()
        qps = src.size * reps / (time.perf_counter() - t1)
        r = np.array([w["res_l1"] for w in o["warm"]])
        fb = np.array([w["fell_back"] for w in o["warm"]])
        return dict(queries_per_s=round(qps, 3), res_l1_median=round(float(np.median(r)), 4),
                    res_l1_max=round(float(r.max()), 4), fallback_rate=round(float(fb.mean()), 3),
                    mean_sweeps_per_query=float(np.mean([x["steps"] for x in o["stats"]])))

    learned = timed(M)
    M0 = bh.Model(G, seed=1)
    M0.set_params(np.zeros(bh.MODEL_PARAMS, np.float32))
    M0.embed()
    ablation = timed(M0)
    M0.close()
    log(f"learned: {learned}; self term only: {ablation}")
    return M, dict(train_sources=int(train.size), train_steps=steps, batch="32 sources x 4096 candidates",
                   data_s=round(t_data, 1), train_s=round(t_train, 1),
                   loss_first=float(losses[:50].mean()), loss_last=float(losses[-50:].mean()),
                   batched_learned=learned, ablation_self_term_only=ablation)


def run_learned_curve(bh, torch, np, G, el, wl, src, sizes):
    """The learned start against training-set size: training data (top-64 of
    beta' plus 64 random entries) from the plain GPU path for max(sizes)
    uniform sources disjoint from the evaluation sources; for each size a
    fresh model is trained on the first `size` of them. On the evaluation
    sources it reports the prediction error ||p_hat(u, .) - pi(u, .)||_1 (pi
    from the plain path's beta' by Lemma 3: pi(u, x) = beta' ws(x)/(ws(u) +
    ws(x))), the start's residual norm, the fallback rate and the sweeps,
    beside the structural self term alone (size 0)."""
    import synth
    n_max = max(sizes)
    live = np.nonzero(el.degrees_u() > 0)[0]
    rng = np.random.default_rng(78)
    cand = synth.sample_sources(el, n_max + src.size, "uniform", 4343)
    train = np.setdiff1d(cand, src)[:n_max].astype(np.int32)
    rng.shuffle(train)
    ws = np.bincount(el.u, weights=el.w, minlength=el.n_u)
    ws_t = torch.from_numpy(ws).to("cuda")
    ref = G.query_batch(src, wl.eps, k=0, exclude_self=False, scores=True, stats=True)
    pi = ref["scores"].double() * ws_t[None, :] / (ws_t[src.astype(np.int64)][:, None] + ws_t[None, :])
    cold_sweeps = float(np.mean([x["steps"] for x in ref["stats"]]))
    t0 = time.perf_counter()
    ids = np.full((train.size, 128), -1, np.int32)
    vals = np.zeros((train.size, 128), np.float32)
    for i in range(0, train.size, 64):
        chunk = train[i:i + 64]
        out = G.query_batch(chunk, wl.eps, k=64, exclude_self=False, scores=True, stats=False)
        r = torch.from_numpy(rng.choice(live, (chunk.size, 64))).to("cuda")
        rv = torch.gather(out["scores"], 1, r.long())
        ii = torch.cat([out["ids"], r.int()], 1).cpu().numpy()
        vv = torch.cat([out["vals"], rv], 1).cpu().numpy()
        for j, (a, b) in enumerate(zip(ii, vv)):
            _, keep = np.unique(a, return_index=True)
            ids[i + j, :keep.size], vals[i + j, :keep.size] = a[keep], b[keep]
        del out
        if (i // 64) % 200 == 0:
            log(f"learned curve: training data {i + chunk.size}/{train.size}")
    t_data = time.perf_counter() - t0
    log(f"learned curve: training data from {train.size} plain queries in {t_data:.1f}s")
    rows = []
    for n in [0] + sorted(sizes):
        M = bh.Model(G, seed=1)
        steps = 0
        if n == 0:
            M.set_params(np.zeros(bh.MODEL_PARAMS, np.float32))
            losses = np.zeros(1)
        else:
            steps = int(min(20000, max(2000, n // 10)))
            losses = M.train(train[:n], ids[:n], vals[:n], steps=steps, batch_src=32, batch_cand=4096, lr=5e-4)
        M.embed()
        p_hat = M.predict(src).double()
        dp = (p_hat - pi).abs().sum(1).cpu().numpy()
        o = G.query_batch(src, wl.eps, k=0, scores=False, stats=True, model=M)
        r = np.array([w["res_l1"] for w in o["warm"]])
        fb = np.array([w["fell_back"] for w in o["warm"]])
        rows.append(dict(train_sources=int(n), train_steps=steps, loss_last=float(np.mean(losses[-50:])),
                         dp_l1_median=round(float(np.median(dp)), 4), dp_l1_max=round(float(dp.max()), 4),
                         res_l1_median=round(float(np.median(r)), 4), fallback_rate=round(float(fb.mean()), 3),
                         mean_sweeps_per_query=float(np.mean([x["steps"] for x in o["stats"]]))))
        log(f"learned curve: {rows[-1]}")
        M.close()
        del p_hat
    return dict(eval_sources=int(src.size), data_s=round(t_data, 1), cold_mean_sweeps=cold_sweeps, curve=rows)


def run_serving(bh, G, el, wl, rates, duration, np, model=None):
    """Continuous batching on the resident graph: Poisson arrivals at each rate
    for `duration` seconds, degree-proportional sources, eps uniform on
    {1e-5, 1e-6, 1e-7}, top-k per request. Latency = arrival to result. When
    a rate overloads the device, results stop being collected `duration` + 6 s
    after the start; the latencies of the requests still unfinished then are
    at least the time they have waited, which the *_all percentiles use (lower
    bounds)."""
    import synth

    def new_server():
        S = bh.Server(G, k=wl.k, model=model)
        warm = synth.sample_sources(el, 4, "degree", 90)   # capture the sweep chunk once
        for i, u in enumerate(warm):
            S.submit(int(u), 1e-5, -1 - i)
        while S.info()["completed"] < warm.size:
            S.poll()
        return S

    S = new_server()
    out = []
    for j, rate in enumerate(rates):
        rng = np.random.default_rng(1000 + j)
        n = max(1, int(rate * duration))
        arr = np.cumsum(rng.exponential(1.0 / rate, size=n))
        src = synth.sample_sources(el, n, "degree", 2000 + j)
        eps = rng.choice([1e-5, 1e-6, 1e-7], size=n)
        lat = np.full(n, np.nan)
        inf0 = S.info()
        t0 = time.perf_counter()
        i = done = 0
        cap = duration + 6.0
        t = 0.0
        while done < n:
            now = time.perf_counter() - t0
            while i < n and arr[i] <= now:
                S.submit(int(src[i]), float(eps[i]), i)
                i += 1
            res = S.poll()
            t = time.perf_counter() - t0
            for tag, _, _ in res:
                lat[tag] = t - arr[tag]
                done += 1
            if t > cap:
                break
            if not res and i < n:
                inf = S.info()
                if inf["running"] == 0 and inf["queued"] == 0:
                    time.sleep(max(0.0, arr[i] - (time.perf_counter() - t0)))
        wall = time.perf_counter() - t0
        ok = lat[~np.isnan(lat)]
        inf = S.info()
        rec = dict(offered_qps=rate, requests=n, completed=int(ok.size), completion=round(ok.size / n, 4),
                   wall_s=round(wall, 2), served_qps=round(ok.size / wall, 2),
                   p50_ms=round(float(np.percentile(ok, 50)) * 1e3, 1) if ok.size else None,
                   p99_ms=round(float(np.percentile(ok, 99)) * 1e3, 1) if ok.size else None,
                   backlog=int(n - ok.size), sweeps=int(inf["sweeps"] - inf0["sweeps"]),
                   warm_started=int(inf["warm_started"] - inf0["warm_started"]),
                   warm_fell_back=int(inf["warm_fell_back"] - inf0["warm_fell_back"]))
        if ok.size < n:
            # unfinished requests: latency at least (cutoff - arrival); never-submitted ones count from arrival too
            lb = lat.copy()
            miss = np.isnan(lb)
            lb[miss] = np.maximum(0.0, t - arr[miss])
            rec["p50_ms_all"] = round(float(np.percentile(lb, 50)) * 1e3, 1)
            rec["p99_ms_all"] = round(float(np.percentile(lb, 99)) * 1e3, 1)
            rec["all_percentiles"] = "lower bounds: unfinished requests counted at the time waited"
        out.append(rec)
        log(f"serve {rate} q/s: {rec}")
        if ok.size < n:   # overloaded: drop what is left before the next rate
            S.close()
            S = new_server()
    res = dict(width=S.width, k=wl.k, resident_bytes=int(S.info()["resident_bytes"]),
               learned_warm_start=model is not None, eps_mix=[1e-5, 1e-6, 1e-7],
               source_sampling="degree-proportional", duration_s=duration, rates=out)
    S.close()
    return res


def run_baselines(bh, torch, np, G, wl, src):
    """The paper's comparison (Sec. 5.4, Fig. 3) on the GPU: Approx-BHPP
    against PISP and MCSP (Sec. 3.3) on the same sources, batched, at several
    eps. Time per batch, best of two runs after a warm-up; MCSP only where
    its walk count stays small (the paper drops it at small eps too)."""
    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(2):
            t0 = time.perf_counter()
            o = fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return o, best
    rows = []
    for eps in (1e-2, 1e-4, 1e-6, 1e-7):
        a, ta = timed(lambda: G.query_batch(src, eps, k=wl.k, scores=False, stats=True))
        p, tp = timed(lambda: G.query_batch(src, eps, k=wl.k, scores=False, stats=True, method="pisp"))
        rec = dict(eps=eps, approx_qps=round(src.size / ta, 2), pisp_qps=round(src.size / tp, 2),
                   approx_sweeps=float(np.mean([x["steps"] for x in a["stats"]])),
                   pisp_sweeps=float(np.mean([x["steps"] for x in p["stats"]])),
                   approx_edge_visits=float(np.mean([x["visits_u"] + x["visits_v"] for x in a["stats"]])),
                   pisp_edge_visits=float(np.mean([x["visits_u"] + x["visits_v"] for x in p["stats"]])),
                   speedup_over_pisp=round(tp / ta, 3))
        if eps >= 1e-2:
            m, tm = timed(lambda: G.query_mcsp(src, eps, p_f=1e-6, seed=1, k=wl.k, scores=False, stats=False))
            rec.update(mcsp_qps=round(src.size / tm, 2), mcsp_walks_per_query=m["walks"],
                       speedup_over_mcsp=round(tm / ta, 3))
        rows.append(rec)
        log(f"baselines eps={eps}: {rec}")
    return rows


def run_medium(bh, torch, np, args):
    """The 1M x 2M graph: plain batched (64 uniform sources per batch) and
    single-source queries, eps_b tuning, learned warm start, serving."""
    import synth
    wl = synth.MEDIUM
    t0 = time.perf_counter()
    el = wl.graph()
    src = wl.sources(el)
    log(f"graph {wl.name}: {el.n_e} edges generated in {time.perf_counter() - t0:.1f}s")
    G = bh.Graph.from_edges(el, alpha=wl.alpha, dtype="f32", mcsp=not args.no_baselines)
    info = G.info()
    out = dict(workload=wl.name, sources=int(src.size), source_sampling="uniform non-isolated",
               lambda_=round(info["lambda"], 3))

    def batch():
        return G.query_batch(src, wl.eps, k=wl.k, exclude_self=True, scores=True, stats=True)

    batch()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    reps = max(1, args.medium_reps)
    for _ in range(reps):
        o = batch()
    torch.cuda.synchronize()
    out["batched_qps"] = round(src.size * reps / (time.perf_counter() - t1), 3)
    out["mean_sweeps_per_query"] = float(np.mean([x["steps"] for x in o["stats"]]))
    log(f"{wl.name}: plain batched {out['batched_qps']} q/s")
    if args.single > 0:
        G.query(int(src[0]), wl.eps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for u in src[:args.single]:
            G.query(int(u), wl.eps, with_stats=False)
        torch.cuda.synchronize()
        out["single_source_qps"] = round(args.single / (time.perf_counter() - t1), 3)
        log(f"{wl.name}: single-source {out['single_source_qps']} q/s")
    if not args.no_baselines:
        out["baselines"] = run_baselines(bh, torch, np, G, wl, src)
    if not args.no_tune_eps_b:
        paper = info["eps_b_ratio"]
        sample = np.setdiff1d(synth.sample_sources(el, 128, "uniform", 9090), src)[:64]
        ratios = [0.01, 0.03, 0.1, 0.2, paper]
        best, ms, gm, swc = G.tune_eps_b(sample, wl.eps, ratios, curve=True)
        batch()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            o = batch()
        torch.cuda.synchronize()
        tq = src.size * reps / (time.perf_counter() - t1)
        sw = float(np.mean([x["steps"] for x in o["stats"]]))
        G.set_eps_b_ratio(0.0)
        out["tuned_eps_b"] = dict(candidates=[round(r, 4) for r in ratios], sample_ms=[round(m, 1) for m in ms],
                                  gamma_curve=[round(float(x), 5) for x in gm],
                                  sample_sweeps=[round(float(x), 1) for x in swc], best_ratio=round(best, 4),
                                  paper_ratio=round(paper, 4), queries_per_s=round(tq, 3), mean_sweeps_per_query=sw)
        log(f"tuned eps_b ratio {best:.3f}: {tq:.1f} q/s, {sw:.1f} sweeps per query")
    model = None
    if not args.no_learned:
        model, out["learned"] = run_learned(bh, torch, np, G, el, wl, src, args.train_sources, args.train_steps, 2)
        if out.get("single_source_qps"):
            out["learned"]["gain_over_single_source"] = round(
                out["learned"]["batched_learned"]["queries_per_s"] / out["single_source_qps"], 2)
    if args.learned_curve:
        sizes = [int(x) for x in args.learned_curve.split(",") if x.strip()]
        out["learned_curve"] = run_learned_curve(bh, torch, np, G, el, wl, src, sizes)
    rates = [float(x) for x in args.serve.split(",") if x.strip()]
    if rates:
        out["serving"] = run_serving(bh, G, el, wl, rates, args.serve_seconds, np, model)
    if model is not None:
        model.close()
    G.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sources-per-step", type=int, default=256,
                    help="sources per step, a slice of the 1024-source set (1024 = the whole set)")
    ap.add_argument("--single", type=int, default=4, help="sources timed one at a time on each graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--cpu-iters", type=int, default=6, help="push iterations per query of the CPU sample")
    ap.add_argument("--no-medium", action="store_true", help="skip the 1M x 2M graph's measurements")
    ap.add_argument("--medium-reps", type=int, default=5)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm start")
    ap.add_argument("--no-baselines", action="store_true", help="skip the PISP / MCSP comparison")
    ap.add_argument("--no-tune-eps-b", action="store_true", help="skip the eps_b split tuning")
    ap.add_argument("--train-sources", type=int, default=2048)
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--learned-curve", default="",
                    help="training-set sizes for the learned-start curve on the 1M x 2M graph, e.g. 2048,20000,200000")
    ap.add_argument("--no-headline", action="store_true", help="skip the 100M-edge headline (extras only)")
    ap.add_argument("--launch", default="",
                    help="tile,inflight,nt,chunk launch setting for the headline graph instead of autotuning "
                         "(profiling runs)")
    ap.add_argument("--serve", default="150,300,2000,20000",
                    help="Poisson arrival rates (q/s) for the serving run; empty to skip")
    ap.add_argument("--serve-seconds", type=float, default=6.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB device-to-device copy first (known-size kernel for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(sources shard across GPUs without communication; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2312_06724_amd as bh

    hinfo = host_info()
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 1 GiB read + 1 GiB written")
        del a, b

    if args.no_headline:   # extras only (experiments); no headline value
        medium = run_medium(bh, torch, np, args)
        print(json.dumps({"metric": "BHPP queries/s at eps=1e-6 (plain vs batched+learned); HBM GB/s; p99 ms",
                          "value": None, "unit": "queries/s", "n_gpus": 1, "host": hinfo, "medium": medium}),
              flush=True)
        return
    head = run_headline(bh, torch, np, args, hinfo)
    medium = None if args.no_medium else run_medium(bh, torch, np, args)
    wl, info = head["wl"], head["info"]
    out = {
        "metric": "BHPP queries/s at eps=1e-6 (plain vs batched+learned); HBM GB/s; p99 ms",
        "value": round(head["value"], 3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["dt"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_u": info["n_u"], "n_v": info["n_v"], "n_edges": info["n_edges"],
                   "sources_per_step": args.sources_per_step, "source_set": int(wl.n_sources),
                   "source_sampling": "degree-proportional", "alpha": wl.alpha, "eps": wl.eps, "k": wl.k,
                   "lambda": round(info["lambda"], 3), "launch_config": head["cfg"]},
        "roofline": head["roof"],
        "cpu_baseline": head["cpu"],
        "single_source_qps": round(head["single"], 3) if head["single"] else None,
        "sweeps_per_query": dict(min=int(head["steps_q"].min()), mean=float(head["steps_q"].mean()),
                                 max=int(head["steps_q"].max())),
        "host": hinfo,
        "medium": medium,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
