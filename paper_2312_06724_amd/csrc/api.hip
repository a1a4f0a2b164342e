// C ABI entry points (include/bhpp.h): argument checking, handle ownership,
// error mapping. All computation happens in the kernels of build.hip,
// sweep.hip and topk.hip.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "common.h"

using bhpp::Graph;

struct bhpp_graph {
    Graph* g;
};

struct bhpp_server {
    bhpp_graph* h;
    bhpp::Server* sv;
    int32_t width;
};

struct bhpp_model {
    bhpp_graph* h;
    bhpp::Model* m;
};

namespace {

hipStream_t stream_of(void* s) { return reinterpret_cast<hipStream_t>(s); }

bool valid_alpha(double a) { return a > 0.0 && a < 1.0 && std::isfinite(a); }
bool valid_eps(double e) { return e > 0.0 && e < 1e30 && std::isfinite(e); }

bhpp_status sticky(Graph* g, bhpp_status rc) {
    if (rc == BHPP_DEVICE_ERROR) g->sticky_error = true;
    return rc;
}

// lambda for this alpha (Lemma 4), computed once per alpha and cached
bhpp_status lambda_for(Graph* g, double alpha, hipStream_t s, double* out) {
    auto it = g->lambda_cache.find(alpha);
    if (it != g->lambda_cache.end()) {
        *out = it->second;
        return BHPP_OK;
    }
    int32_t tau = 0;
    double mm = (double)g->nu * (1.0 - alpha);
    while (mm > 1.0) { mm *= (1.0 - alpha); ++tau; }
    bhpp_status rc = bhpp::compute_lambda(g, alpha, tau, s, out);
    if (rc == BHPP_OK) g->lambda_cache[alpha] = *out;
    return rc;
}

}  // namespace

extern "C" {

const char* bhpp_status_string(bhpp_status s) {
    switch (s) {
        case BHPP_OK: return "ok";
        case BHPP_INVALID_ARG: return "invalid argument";
        case BHPP_OUT_OF_RANGE: return "node id out of range";
        case BHPP_ISOLATED_SOURCE: return "source node has no edge";
        case BHPP_BAD_WEIGHT: return "edge weight not finite and positive";
        case BHPP_OUT_OF_MEMORY: return "out of memory";
        case BHPP_DEVICE_ERROR: return "HIP device error";
        case BHPP_NOT_SUPPORTED: return "not supported";
        case BHPP_NO_CONVERGENCE: return "step limit reached";
        default: return "unknown status";
    }
}

bhpp_status bhpp_build_graph(int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* edge_u,
                             const int32_t* edge_v, const void* edge_w, const bhpp_graph_opts* opts,
                             void* hip_stream, bhpp_graph** out) {
    if (!out) return BHPP_INVALID_ARG;
    *out = nullptr;
    bhpp_graph_opts o{0.15, -1, BHPP_DTYPE_F32, 0u};
    if (opts) o = *opts;
    if (n_u <= 0 || n_v <= 0 || n_edges < 0 || n_edges > 0x7FFFFFFFLL) return BHPP_INVALID_ARG;
    if (n_edges > 0 && (!edge_u || !edge_v || !edge_w)) return BHPP_INVALID_ARG;
    if (!valid_alpha(o.alpha)) return BHPP_INVALID_ARG;
    if (o.dtype != BHPP_DTYPE_F32 && o.dtype != BHPP_DTYPE_F64) return BHPP_NOT_SUPPORTED;
    try {
        Graph* g = nullptr;
        bhpp_status rc = bhpp::build_graph(n_u, n_v, n_edges, edge_u, edge_v, edge_w, o, stream_of(hip_stream), &g);
        if (rc) return rc;
        bhpp_graph* h = new (std::nothrow) bhpp_graph{g};
        if (!h) {
            bhpp::free_graph(g);
            return BHPP_OUT_OF_MEMORY;
        }
        *out = h;
        return BHPP_OK;
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

static bhpp_status query_batch_impl(bhpp_graph* h, bhpp_model* model, const void* starts, int32_t target,
                                    int32_t n_src, const int32_t* sources,
                                    const double* eps, double alpha, double eps_all, void* scores_out, int32_t k,
                                    int32_t exclude_self, int32_t* topk_ids, void* topk_vals,
                                    bhpp_query_stats* stats, bhpp_warm_stats* wstats, void* hip_stream) {
    if (!h || !h->g) return BHPP_INVALID_ARG;
    Graph* g = h->g;
    if (g->sticky_error) return BHPP_DEVICE_ERROR;
    if (n_src < 0 || (n_src > 0 && !sources) || !valid_alpha(alpha)) return BHPP_INVALID_ARG;
    if (model && (model->h != h || !bhpp::model_ready(model->m))) return BHPP_INVALID_ARG;
    if (n_src == 0) return BHPP_OK;
    if (k < 0 || k > bhpp::kTopkTmpK || k > g->nu - (exclude_self ? 1 : 0)) return BHPP_INVALID_ARG;
    if (k > 0 && (!topk_ids || !topk_vals)) return BHPP_INVALID_ARG;
    std::vector<double> e((size_t)n_src);
    for (int32_t i = 0; i < n_src; ++i) {
        e[i] = eps ? eps[i] : eps_all;
        if (!valid_eps(e[i])) return BHPP_INVALID_ARG;
    }
    for (int32_t i = 0; i < n_src; ++i) {
        if (sources[i] < 0 || sources[i] >= g->nu) return BHPP_OUT_OF_RANGE;
        if (!(g->h_ws_u[sources[i]] > 0.0)) return BHPP_ISOLATED_SOURCE;
    }
    try {
        std::lock_guard<std::mutex> lock(g->mu);
        hipStream_t s = stream_of(hip_stream);
        double lam = 0.0;
        bhpp_status rc = lambda_for(g, alpha, s, &lam);
        if (rc) return sticky(g, rc);
        rc = bhpp::run_queries(g, model ? model->m : nullptr, starts, wstats, target, n_src, sources, e.data(), alpha,
                               lam,
                               scores_out, k, exclude_self, topk_ids, topk_vals, stats, s);
        if (rc == BHPP_OK && hipStreamSynchronize(s) != hipSuccess) rc = BHPP_DEVICE_ERROR;
        return sticky(g, rc);
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

bhpp_status bhpp_query_batch(bhpp_graph* h, int32_t n_src, const int32_t* sources, const double* eps,
                             double alpha, double eps_all, void* scores_out, int32_t k, int32_t exclude_self,
                             int32_t* topk_ids, void* topk_vals, bhpp_query_stats* stats, void* hip_stream) {
    return query_batch_impl(h, nullptr, nullptr, 0, n_src, sources, eps, alpha, eps_all, scores_out, k, exclude_self,
                            topk_ids, topk_vals, stats, nullptr, hip_stream);
}

bhpp_status bhpp_query_batch_warm(bhpp_graph* h, bhpp_model* m, int32_t n_src, const int32_t* sources,
                                  const double* eps, double alpha, double eps_all, void* scores_out, int32_t k,
                                  int32_t exclude_self, int32_t* topk_ids, void* topk_vals, bhpp_query_stats* stats,
                                  bhpp_warm_stats* warm_out, void* hip_stream) {
    if (!m || !m->m) return BHPP_INVALID_ARG;
    return query_batch_impl(h, m, nullptr, 0, n_src, sources, eps, alpha, eps_all, scores_out, k, exclude_self,
                            topk_ids, topk_vals, stats, warm_out, hip_stream);
}

bhpp_status bhpp_query_batch_start(bhpp_graph* h, const void* starts, int32_t n_src, const int32_t* sources,
                                   const double* eps, double alpha, double eps_all, void* scores_out, int32_t k,
                                   int32_t exclude_self, int32_t* topk_ids, void* topk_vals, bhpp_query_stats* stats,
                                   bhpp_warm_stats* warm_out, void* hip_stream) {
    if (!starts) return BHPP_INVALID_ARG;
    return query_batch_impl(h, nullptr, starts, 0, n_src, sources, eps, alpha, eps_all, scores_out, k, exclude_self,
                            topk_ids, topk_vals, stats, warm_out, hip_stream);
}

bhpp_status bhpp_query_batch_pisp(bhpp_graph* h, int32_t n_src, const int32_t* sources, const double* eps,
                                  double alpha, double eps_all, void* scores_out, int32_t k, int32_t exclude_self,
                                  int32_t* topk_ids, void* topk_vals, bhpp_query_stats* stats, void* hip_stream) {
    return query_batch_impl(h, nullptr, nullptr, 3, n_src, sources, eps, alpha, eps_all, scores_out, k, exclude_self,
                            topk_ids, topk_vals, stats, nullptr, hip_stream);
}

bhpp_status bhpp_query_batch_mcsp(bhpp_graph* h, int32_t n_src, const int32_t* sources, double eps, double alpha,
                                  double p_f, uint64_t seed, void* scores_out, int32_t k, int32_t exclude_self,
                                  int32_t* topk_ids, void* topk_vals, bhpp_query_stats* stats, int64_t* walks_out,
                                  void* hip_stream) {
    if (!h || !h->g) return BHPP_INVALID_ARG;
    Graph* g = h->g;
    if (g->sticky_error) return BHPP_DEVICE_ERROR;
    if (!g->mc_prob_u) return BHPP_NOT_SUPPORTED;
    if (!valid_eps(eps) || !(p_f > 0.0 && p_f < 1.0)) return BHPP_INVALID_ARG;
    if (n_src < 0 || (n_src > 0 && !sources) || !valid_alpha(alpha)) return BHPP_INVALID_ARG;
    if (n_src == 0) return BHPP_OK;
    if (k < 0 || k > bhpp::kTopkTmpK || k > g->nu - (exclude_self ? 1 : 0)) return BHPP_INVALID_ARG;
    if (k > 0 && (!topk_ids || !topk_vals)) return BHPP_INVALID_ARG;
    for (int32_t i = 0; i < n_src; ++i) {
        if (sources[i] < 0 || sources[i] >= g->nu) return BHPP_OUT_OF_RANGE;
        if (!(g->h_ws_u[sources[i]] > 0.0)) return BHPP_ISOLATED_SOURCE;
    }
    const int64_t n_r = bhpp::mc_walk_count(g->nu, 0.5 * eps, p_f);
    if (n_r > 0xFFFFFFFFll) return BHPP_NOT_SUPPORTED;   // walks are numbered with 32 bits
    if (walks_out) *walks_out = n_r;
    try {
        std::lock_guard<std::mutex> lock(g->mu);
        hipStream_t s = stream_of(hip_stream);
        double lam = 0.0;
        bhpp_status rc = lambda_for(g, alpha, s, &lam);
        if (rc) return sticky(g, rc);
        const size_t rows_bytes = (size_t)n_src * g->nu * g->elem;
        void* rows = scores_out;
        uint32_t* counts = nullptr;
        if (!rows && hipMalloc(&rows, rows_bytes) != hipSuccess) {
            (void)hipGetLastError();
            return BHPP_OUT_OF_MEMORY;
        }
        if (hipMalloc((void**)&counts, 4 * (size_t)n_src * g->nu) != hipSuccess) {
            (void)hipGetLastError();
            if (!scores_out) hipFree(rows);
            return BHPP_OUT_OF_MEMORY;
        }
        std::vector<double> e((size_t)n_src, eps);
        // backward part: SelectivePush with eps/2 (control mode 4) into the rows
        rc = bhpp::run_queries(g, nullptr, nullptr, nullptr, 4, n_src, sources, e.data(), alpha, lam, rows, 0, 0,
                               nullptr, nullptr, stats, s);
        // forward part: the walks, then beta' = counts / n_r + pi_b
        if (rc == BHPP_OK) rc = bhpp::mcsp_counts(g, n_src, sources, alpha, n_r, seed, counts, s);
        if (rc == BHPP_OK) rc = bhpp::mcsp_combine(g, rows, counts, n_src, n_r, s);
        if (rc == BHPP_OK && k > 0) {
            std::vector<int32_t> ex((size_t)n_src, -1);
            if (exclude_self)
                for (int32_t i = 0; i < n_src; ++i) ex[i] = sources[i];
            int32_t* d_ex = nullptr;
            if (hipMalloc((void**)&d_ex, 4 * (size_t)n_src) != hipSuccess) {
                (void)hipGetLastError();
                rc = BHPP_OUT_OF_MEMORY;
            } else {
                if (hipMemcpyAsync(d_ex, ex.data(), 4 * (size_t)n_src, hipMemcpyHostToDevice, s) != hipSuccess)
                    rc = BHPP_DEVICE_ERROR;
                if (rc == BHPP_OK)
                    rc = bhpp::topk_rows(rows, n_src, g->nu, k, d_ex, g->dtype, topk_ids, topk_vals, s);
                if (hipStreamSynchronize(s) != hipSuccess && rc == BHPP_OK) rc = BHPP_DEVICE_ERROR;
                hipFree(d_ex);
            }
        }
        if (rc == BHPP_OK && hipStreamSynchronize(s) != hipSuccess) rc = BHPP_DEVICE_ERROR;
        hipFree(counts);
        if (!scores_out) hipFree(rows);
        return sticky(g, rc);
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

bhpp_status bhpp_query_hpp(bhpp_graph* h, int32_t n_src, const int32_t* sources, const double* eps, double alpha,
                           double eps_all, int32_t direction, void* scores_out, bhpp_query_stats* stats,
                           void* hip_stream) {
    if (direction != BHPP_HPP_FORWARD && direction != BHPP_HPP_BACKWARD) return BHPP_INVALID_ARG;
    if (!scores_out && n_src > 0) return BHPP_INVALID_ARG;
    return query_batch_impl(h, nullptr, nullptr, direction == BHPP_HPP_FORWARD ? 1 : 2, n_src, sources, eps, alpha,
                            eps_all, scores_out, 0, 0, nullptr, nullptr, stats, nullptr, hip_stream);
}

bhpp_status bhpp_query(bhpp_graph* h, int32_t source, double alpha, double eps, void* scores_out,
                       bhpp_query_stats* stats, void* hip_stream) {
    if (!scores_out) return BHPP_INVALID_ARG;
    return bhpp_query_batch(h, 1, &source, nullptr, alpha, eps, scores_out, 0, 0, nullptr, nullptr, stats,
                            hip_stream);
}

bhpp_status bhpp_topk(const void* scores, int32_t n_rows, int32_t n, int32_t k, const int32_t* exclude_ids,
                      int32_t dtype, int32_t* ids_out, void* vals_out, void* hip_stream) {
    if (n_rows < 0 || n <= 0 || k < 1 || k > n) return BHPP_INVALID_ARG;
    if (n_rows > 0 && (!scores || !ids_out || !vals_out)) return BHPP_INVALID_ARG;
    if (dtype != BHPP_DTYPE_F32 && dtype != BHPP_DTYPE_F64) return BHPP_NOT_SUPPORTED;
    if (exclude_ids && k > n - 1) return BHPP_INVALID_ARG;
    try {
        return bhpp::topk_rows(scores, n_rows, n, k, exclude_ids, dtype, ids_out, vals_out, stream_of(hip_stream));
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

bhpp_status bhpp_topk_noalloc(const void* scores, int32_t n_rows, int32_t n, int32_t k, const int32_t* exclude_ids,
                              int32_t dtype, int32_t* ids_out, void* vals_out, void* hip_stream) {
    if (n_rows < 0 || n <= 0 || k < 1 || k > n) return BHPP_INVALID_ARG;
    if (n_rows > 0 && (!scores || !ids_out || !vals_out)) return BHPP_INVALID_ARG;
    if (dtype != BHPP_DTYPE_F32 && dtype != BHPP_DTYPE_F64) return BHPP_NOT_SUPPORTED;
    if (exclude_ids && k > n - 1) return BHPP_INVALID_ARG;
    if (n_rows > BHPP_TOPK_NOALLOC_MAX_ROWS || k > BHPP_TOPK_NOALLOC_MAX_K) return BHPP_NOT_SUPPORTED;
    return bhpp::topk_rows_static(scores, n_rows, n, k, exclude_ids, dtype, ids_out, vals_out, stream_of(hip_stream));
}

bhpp_status bhpp_graph_info(const bhpp_graph* h, bhpp_graph_summary* out) {
    if (!h || !h->g || !out) return BHPP_INVALID_ARG;
    *out = h->g->info;
    return BHPP_OK;
}

bhpp_status bhpp_graph_export(const bhpp_graph* h, int64_t* rp_u, int32_t* ci_u, void* w_u, int64_t* rp_v,
                              int32_t* ci_v, void* w_v, void* ws_u, void* ws_v, void* hip_stream) {
    if (!h || !h->g) return BHPP_INVALID_ARG;
    Graph* g = h->g;
    if (!g->x_rp_u) return BHPP_NOT_SUPPORTED;
    if (!rp_u || !ci_u || !w_u || !rp_v || !ci_v || !w_v || !ws_u || !ws_v) return BHPP_INVALID_ARG;
    hipStream_t s = stream_of(hip_stream);
    const size_t m = (size_t)g->ne, e = (size_t)g->elem;
    BHPP_HIP(hipMemcpyAsync(rp_u, g->x_rp_u, 8 * ((size_t)g->nu + 1), hipMemcpyDeviceToDevice, s));
    BHPP_HIP(hipMemcpyAsync(rp_v, g->x_rp_v, 8 * ((size_t)g->nv + 1), hipMemcpyDeviceToDevice, s));
    if (m > 0) {
        BHPP_HIP(hipMemcpyAsync(ci_u, g->x_ci_u, 4 * m, hipMemcpyDeviceToDevice, s));
        BHPP_HIP(hipMemcpyAsync(ci_v, g->x_ci_v, 4 * m, hipMemcpyDeviceToDevice, s));
        BHPP_HIP(hipMemcpyAsync(w_u, g->x_w_u, e * m, hipMemcpyDeviceToDevice, s));
        BHPP_HIP(hipMemcpyAsync(w_v, g->x_w_v, e * m, hipMemcpyDeviceToDevice, s));
    }
    BHPP_HIP(hipMemcpyAsync(ws_u, g->x_ws_u, e * g->nu, hipMemcpyDeviceToDevice, s));
    BHPP_HIP(hipMemcpyAsync(ws_v, g->x_ws_v, e * g->nv, hipMemcpyDeviceToDevice, s));
    BHPP_HIP(hipStreamSynchronize(s));
    return BHPP_OK;
}

bhpp_status bhpp_profile_enable(bhpp_graph* h, int32_t enable) {
    if (!h || !h->g) return BHPP_INVALID_ARG;
    Graph* g = h->g;
    std::lock_guard<std::mutex> lock(g->mu);
    if (enable) {
        for (hipEvent_t e : g->prof_ev) hipEventDestroy(e);
        g->prof_ev.clear();
        g->prof_kind.clear();
        g->prof_b.clear();
        for (int k = 0; k < 4; ++k) {
            g->prof_ms[k] = 0.0;
            g->prof_n[k] = 0;
            g->prof_bytes[k] = 0.0;
        }
        g->prof_live = 0;
    }
    g->prof_on = enable != 0;
    return BHPP_OK;
}

bhpp_status bhpp_profile_sweeps(bhpp_graph* h, int64_t* live_out) {
    if (!h || !h->g || !live_out) return BHPP_INVALID_ARG;
    Graph* g = h->g;
    std::lock_guard<std::mutex> lock(g->mu);
    *live_out = g->prof_live;
    return BHPP_OK;
}

bhpp_status bhpp_profile_read(bhpp_graph* h, double ms[4], int64_t launches[4], double bytes[4]) {
    if (!h || !h->g || !ms || !launches || !bytes) return BHPP_INVALID_ARG;
    Graph* g = h->g;
    std::lock_guard<std::mutex> lock(g->mu);
    // fold the recorded event pairs into the totals
    const size_t pairs = g->prof_ev.size() / 2;
    for (size_t i = 0; i < pairs; ++i) {
        hipEvent_t a = g->prof_ev[2 * i], b = g->prof_ev[2 * i + 1];
        if (hipEventSynchronize(b) != hipSuccess) return BHPP_DEVICE_ERROR;
        float t = 0.f;
        if (hipEventElapsedTime(&t, a, b) != hipSuccess) return BHPP_DEVICE_ERROR;
        const int kind = g->prof_kind[i];
        g->prof_ms[kind] += t;
        g->prof_n[kind] += 1;
        g->prof_bytes[kind] += g->prof_b[i];
        hipEventDestroy(a);
        hipEventDestroy(b);
    }
    g->prof_ev.clear();
    g->prof_kind.clear();
    g->prof_b.clear();
    for (int k = 0; k < 4; ++k) {
        ms[k] = g->prof_ms[k];
        launches[k] = g->prof_n[k];
        bytes[k] = g->prof_bytes[k];
    }
    return BHPP_OK;
}

bhpp_status bhpp_autotune(bhpp_graph* h, void* hip_stream, int32_t config_out[4]) {
    if (!h || !h->g || !config_out) return BHPP_INVALID_ARG;
    Graph* g = h->g;
    if (g->sticky_error) return BHPP_DEVICE_ERROR;
    try {
        std::lock_guard<std::mutex> lock(g->mu);
        if (g->n_servers > 0) return BHPP_INVALID_ARG;
        int cfg[4];
        bhpp_status rc = bhpp::autotune(g, stream_of(hip_stream), cfg);
        if (rc == BHPP_OK)
            for (int i = 0; i < 4; ++i) config_out[i] = cfg[i];
        return sticky(g, rc);
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

bhpp_status bhpp_set_launch_config(bhpp_graph* h, const int32_t config[4]) {
    if (!h || !h->g || !config) return BHPP_INVALID_ARG;
    Graph* g = h->g;
    try {
        std::lock_guard<std::mutex> lock(g->mu);
        if (g->n_servers > 0) return BHPP_INVALID_ARG;
        int cfg[4] = {config[0], config[1], config[2], config[3]};
        return sticky(g, bhpp::set_launch_config(g, cfg));
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

bhpp_status bhpp_get_launch_config(const bhpp_graph* h, int32_t config_out[4]) {
    if (!h || !h->g || !config_out) return BHPP_INVALID_ARG;
    const Graph* g = h->g;
    config_out[0] = g->tile_edges;
    config_out[1] = g->inflight;
    config_out[2] = g->nt_stream;
    config_out[3] = g->use_graphs;
    return BHPP_OK;
}

bhpp_status bhpp_set_schedule(bhpp_graph* h, const int32_t sched[2]) {
    if (!h || !h->g || !sched || sched[0] < 1 || sched[0] > 8) return BHPP_INVALID_ARG;
    Graph* g = h->g;
    std::lock_guard<std::mutex> lock(g->mu);
    if (g->n_servers > 0) return BHPP_INVALID_ARG;
    if (sched[0] != g->chunk_sweeps) bhpp::drop_chunk_graphs(g);
    g->chunk_sweeps = sched[0];
    g->async_sched = sched[1] ? 1 : 0;
    return BHPP_OK;
}

bhpp_status bhpp_get_schedule(const bhpp_graph* h, int32_t sched_out[2]) {
    if (!h || !h->g || !sched_out) return BHPP_INVALID_ARG;
    sched_out[0] = h->g->chunk_sweeps;
    sched_out[1] = h->g->async_sched;
    return BHPP_OK;
}

bhpp_status bhpp_server_create(bhpp_graph* h, bhpp_model* model, int32_t max_width, double mem_budget_bytes,
                               double alpha, int32_t k, int32_t exclude_self, bhpp_server** out) {
    if (!out) return BHPP_INVALID_ARG;
    *out = nullptr;
    if (!h || !h->g || !valid_alpha(alpha) || max_width < 1 || max_width > 64) return BHPP_INVALID_ARG;
    if (model && (model->h != h || !bhpp::model_ready(model->m))) return BHPP_INVALID_ARG;
    Graph* g = h->g;
    if (g->sticky_error) return BHPP_DEVICE_ERROR;
    if (k < 1 || k > bhpp::kTopkTmpK || k > g->nu - (exclude_self ? 1 : 0)) return BHPP_INVALID_ARG;
    if (!(mem_budget_bytes <= 0.0 || std::isfinite(mem_budget_bytes))) return BHPP_INVALID_ARG;
    try {
        std::lock_guard<std::mutex> lock(g->mu);
        double lam = 0.0;
        bhpp_status rc = lambda_for(g, alpha, nullptr, &lam);
        if (rc) return sticky(g, rc);
        bhpp::Server* sv = nullptr;
        rc = bhpp::server_create(g, model ? model->m : nullptr, max_width, mem_budget_bytes, alpha, lam, k,
                                 exclude_self ? 1 : 0, &sv);
        if (rc) return sticky(g, rc);
        bhpp_server* s = new (std::nothrow) bhpp_server{h, sv, 0};
        if (!s) {
            bhpp::server_destroy(sv);
            return BHPP_OUT_OF_MEMORY;
        }
        bhpp_server_summary i;
        bhpp::server_info(sv, &i);
        s->width = i.width;
        *out = s;
        return BHPP_OK;
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

bhpp_status bhpp_server_submit(bhpp_server* s, int32_t source, double eps, int64_t tag) {
    if (!s || !s->sv || !valid_eps(eps)) return BHPP_INVALID_ARG;
    Graph* g = s->h->g;
    if (source < 0 || source >= g->nu) return BHPP_OUT_OF_RANGE;
    if (!(g->h_ws_u[source] > 0.0)) return BHPP_ISOLATED_SOURCE;
    try {
        return bhpp::server_submit(s->sv, source, eps, tag);
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

bhpp_status bhpp_server_poll(bhpp_server* s, int32_t capacity, int64_t* tags_out, int32_t* ids_out, void* vals_out,
                             bhpp_query_stats* stats_out, bhpp_warm_stats* warm_out, int32_t* n_out) {
    if (!s || !s->sv || !n_out) return BHPP_INVALID_ARG;
    *n_out = 0;
    if (capacity < s->width || !tags_out || !ids_out || !vals_out) return BHPP_INVALID_ARG;
    Graph* g = s->h->g;
    if (g->sticky_error) return BHPP_DEVICE_ERROR;
    try {
        std::lock_guard<std::mutex> lock(g->mu);
        return sticky(g, bhpp::server_poll(s->sv, tags_out, ids_out, vals_out, stats_out, warm_out, n_out));
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

bhpp_status bhpp_server_info(const bhpp_server* s, bhpp_server_summary* out) {
    if (!s || !s->sv || !out) return BHPP_INVALID_ARG;
    bhpp::server_info(s->sv, out);
    return BHPP_OK;
}

void bhpp_server_destroy(bhpp_server* s) {
    if (!s) return;
    if (s->sv) {
        std::lock_guard<std::mutex> lock(s->h->g->mu);
        bhpp::server_destroy(s->sv);
    }
    delete s;
}

bhpp_status bhpp_model_create(bhpp_graph* h, uint64_t seed, bhpp_model** out) {
    if (!out) return BHPP_INVALID_ARG;
    *out = nullptr;
    if (!h || !h->g) return BHPP_INVALID_ARG;
    Graph* g = h->g;
    if (g->sticky_error) return BHPP_DEVICE_ERROR;
    try {
        std::lock_guard<std::mutex> lock(g->mu);
        bhpp::Model* m = nullptr;
        bhpp_status rc = bhpp::model_create(g, seed, &m);
        if (rc) return sticky(g, rc);
        bhpp_model* o = new (std::nothrow) bhpp_model{h, m};
        if (!o) {
            bhpp::model_free(m);
            return BHPP_OUT_OF_MEMORY;
        }
        *out = o;
        return BHPP_OK;
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

bhpp_status bhpp_model_params(bhpp_model* m, float* get_out, const float* set_in, double* c_out, double* sigma_out) {
    if (!m || !m->m) return BHPP_INVALID_ARG;
    std::lock_guard<std::mutex> lock(m->h->g->mu);
    if (get_out) {
        bhpp_status rc = bhpp::model_get_params(m->m, get_out);
        if (rc) return rc;
    }
    if (set_in) {
        for (int64_t i = 0; i < bhpp::model_num_params(); ++i)
            if (!std::isfinite(set_in[i])) return BHPP_INVALID_ARG;
        bhpp_status rc = bhpp::model_set_params(m->m, set_in);
        if (rc) return rc;
    }
    double c = 0.0, sg = 0.0;
    bhpp::model_scales(m->m, &c, &sg);
    if (c_out) *c_out = c;
    if (sigma_out) *sigma_out = sg;
    return BHPP_OK;
}

bhpp_status bhpp_model_features(bhpp_model* m, float* out, void* hip_stream) {
    if (!m || !m->m || !out) return BHPP_INVALID_ARG;
    std::lock_guard<std::mutex> lock(m->h->g->mu);
    return bhpp::model_features(m->m, out, stream_of(hip_stream));
}

static bool valid_nodes(const Graph* g, int32_t n, const int32_t* ids) {
    for (int32_t i = 0; i < n; ++i)
        if (ids[i] < 0 || ids[i] >= g->nu || !(g->h_ws_u[ids[i]] > 0.0)) return false;
    return true;
}

bhpp_status bhpp_model_loss_grad(bhpp_model* m, int32_t n_src, const int32_t* src, int32_t n_cand,
                                 const int32_t* cand, const float* targets, double* loss_out, float* grad_out) {
    if (!m || !m->m || n_src < 1 || n_cand < 1 || !src || !cand || !targets || !loss_out) return BHPP_INVALID_ARG;
    Graph* g = m->h->g;
    if (!valid_nodes(g, n_src, src) || !valid_nodes(g, n_cand, cand)) return BHPP_OUT_OF_RANGE;
    try {
        std::lock_guard<std::mutex> lock(g->mu);
        return sticky(g, bhpp::model_loss_grad(m->m, n_src, src, n_cand, cand, targets, loss_out, grad_out));
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

bhpp_status bhpp_model_train(bhpp_model* m, int32_t n_src, const int32_t* src, int32_t M, const int32_t* ids,
                             const float* vals, int32_t steps, int32_t batch_src, int32_t batch_cand, double lr,
                             uint64_t seed, float* loss_out) {
    if (!m || !m->m || n_src < 1 || M < 1 || !src || !ids || !vals || steps < 0 || batch_src < 1 ||
        batch_cand < 1 || !(lr > 0.0) || !std::isfinite(lr))
        return BHPP_INVALID_ARG;
    Graph* g = m->h->g;
    if (!valid_nodes(g, n_src, src)) return BHPP_OUT_OF_RANGE;
    try {
        std::lock_guard<std::mutex> lock(g->mu);
        return sticky(g, bhpp::model_train(m->m, n_src, src, M, ids, vals, steps, batch_src, batch_cand, lr, seed,
                                           loss_out));
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

bhpp_status bhpp_model_embed(bhpp_model* m) {
    if (!m || !m->m) return BHPP_INVALID_ARG;
    Graph* g = m->h->g;
    try {
        std::lock_guard<std::mutex> lock(g->mu);
        return sticky(g, bhpp::model_embed(m->m));
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

bhpp_status bhpp_model_predict(bhpp_model* m, int32_t n_src, const int32_t* sources, float* out, void* hip_stream) {
    if (!m || !m->m || n_src < 0 || (n_src > 0 && (!sources || !out))) return BHPP_INVALID_ARG;
    Graph* g = m->h->g;
    if (g->sticky_error) return BHPP_DEVICE_ERROR;
    if (!bhpp::model_ready(m->m)) return BHPP_INVALID_ARG;
    for (int32_t i = 0; i < n_src; ++i) {
        if (sources[i] < 0 || sources[i] >= g->nu) return BHPP_OUT_OF_RANGE;
        if (!(g->h_ws_u[sources[i]] > 0.0)) return BHPP_ISOLATED_SOURCE;
    }
    if (n_src == 0) return BHPP_OK;
    try {
        std::lock_guard<std::mutex> lock(g->mu);
        return sticky(g, bhpp::model_predict_ext(m->m, n_src, sources, out, stream_of(hip_stream)));
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

void bhpp_model_free(bhpp_model* m) {
    if (!m) return;
    if (m->m) {
        std::lock_guard<std::mutex> lock(m->h->g->mu);
        bhpp::model_free(m->m);
    }
    delete m;
}

bhpp_status bhpp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, int32_t trans_a, const uint16_t* B,
                           int32_t trans_b, float* C, void* hip_stream) {
    if (M < 1 || N < 1 || K < 1 || !A || !B || !C) return BHPP_INVALID_ARG;
    return bhpp::gemm_test(M, N, K, A, trans_a, B, trans_b, C, stream_of(hip_stream));
}

bhpp_status bhpp_set_eps_b_ratio(bhpp_graph* h, double ratio) {
    if (!h || !h->g || !(ratio >= 0.0 && ratio < 1.0)) return BHPP_INVALID_ARG;
    Graph* g = h->g;
    std::lock_guard<std::mutex> lock(g->mu);
    g->info.eps_b_ratio = ratio > 0.0 ? ratio : g->eps_b_paper;
    return BHPP_OK;
}

bhpp_status bhpp_tune_eps_b(bhpp_graph* h, int32_t n_src, const int32_t* sources, double eps, double alpha,
                            int32_t n_ratios, const double* ratios, double* ms_out, double* gamma_out,
                            double* sweeps_out, double* best_out, void* hip_stream) {
    if (!h || !h->g || n_src < 1 || !sources || n_ratios < 1 || !ratios || !best_out || !valid_eps(eps) ||
        !valid_alpha(alpha))
        return BHPP_INVALID_ARG;
    Graph* g = h->g;
    if (g->sticky_error) return BHPP_DEVICE_ERROR;
    for (int32_t i = 0; i < n_ratios; ++i)
        if (!(ratios[i] > 0.0 && ratios[i] < 1.0)) return BHPP_INVALID_ARG;
    for (int32_t i = 0; i < n_src; ++i) {
        if (sources[i] < 0 || sources[i] >= g->nu) return BHPP_OUT_OF_RANGE;
        if (!(g->h_ws_u[sources[i]] > 0.0)) return BHPP_ISOLATED_SOURCE;
    }
    try {
        std::lock_guard<std::mutex> lock(g->mu);
        hipStream_t s = stream_of(hip_stream);
        double lam = 0.0;
        bhpp_status rc = lambda_for(g, alpha, s, &lam);
        if (rc) return sticky(g, rc);
        const double saved = g->info.eps_b_ratio;
        std::vector<double> e((size_t)n_src, eps);
        std::vector<bhpp_query_stats> st((size_t)n_src);
        double best_ms = 0.0, best = saved;
        for (int32_t i = 0; i < n_ratios && rc == BHPP_OK; ++i) {
            g->info.eps_b_ratio = ratios[i];
            const auto t0 = std::chrono::steady_clock::now();
            rc = bhpp::run_queries(g, nullptr, nullptr, nullptr, 0, n_src, sources, e.data(), alpha, lam, nullptr, 0,
                                   0, nullptr, nullptr, st.data(), s);
            if (rc == BHPP_OK && hipStreamSynchronize(s) != hipSuccess) rc = BHPP_DEVICE_ERROR;
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (ms_out) ms_out[i] = ms;
            double gm = 0.0, sw = 0.0;
            for (const bhpp_query_stats& q : st) {
                gm += q.gamma;
                sw += q.steps;
            }
            if (gamma_out) gamma_out[i] = gm / n_src;   // Eq. (gamma) averaged over the sample (Fig. 1's quantity)
            if (sweeps_out) sweeps_out[i] = sw / n_src;
            if (rc == BHPP_OK && (i == 0 || ms < best_ms)) {
                best_ms = ms;
                best = ratios[i];
            }
        }
        g->info.eps_b_ratio = rc == BHPP_OK ? best : saved;
        *best_out = g->info.eps_b_ratio;
        return sticky(g, rc);
    } catch (...) {
        return BHPP_OUT_OF_MEMORY;
    }
}

void bhpp_free_graph(bhpp_graph* h) {
    if (!h) return;
    if (h->g) {
        hipDeviceSynchronize();
        bhpp::free_graph(h->g);
    }
    delete h;
}

}  // extern "C"
