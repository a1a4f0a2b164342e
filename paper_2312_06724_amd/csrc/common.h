// Internal declarations of the BHPP library (gfx950). Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/bhpp.h"

namespace bhpp {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kTileEdges = 512;      // target adjacency entries per work tile (the build scales it with |E|)
constexpr int kMaxCols = 64;         // sources per dense residue block (one per lane)
constexpr int kPassThreads = 256;    // threads per block of the sweep kernels
constexpr int kNumRed = 5;           // per-source reductions after a step (see Red)
constexpr int kTopkTmpK = 4096;      // largest k of the batched top-k

// A unit of work for one wavefront: either a run of whole rows whose degrees
// are similar (rows are numbered by decreasing degree) or one piece of a row
// that is longer than kTileEdges. Pieces of a split row write partial sums to
// slot `slot`; a fix-up pass adds them in slot order.
struct Tile {
    int32_t row_begin, row_end;   // rows [row_begin, row_end)
    int64_t e_begin, e_end;       // adjacency range covered
    int32_t slot;                 // partial-sum slot, -1 for whole rows
    int32_t epar_log2;            // log2 of the edge-parallel lanes per row
};

struct SplitRow {
    int32_t row;
    int32_t slot_begin, slot_end; // pieces in order
    int32_t pad;
};

struct TileSet {
    Tile* tiles = nullptr;        // device
    int32_t n_tiles = 0;
    SplitRow* split = nullptr;    // device
    int32_t n_split = 0;
    int32_t n_slots = 0;
};

// Push rule of a source for one half of a sweep (which nodes x are pushed).
enum Rule : int32_t {
    RULE_NONE = 0,   // nothing
    RULE_SS = 1,     // r(x) > eps_b, i.e. y(x)/ws(x) > eps_b/ws(u)     (Algorithm 3, selective)
    RULE_PI = 2,     // r_f(x) > eps_f/lambda, i.e. y(x) > eps_f/lambda (Algorithm 4, selective)
    RULE_ALL = 3,    // every x with y(x) > 0                           (sequential pushes, PowerIteration)
};

// Phase of a source.
enum Mode : int32_t {
    MODE_SS_SEL = 0, MODE_SS_SEQ = 1, MODE_PI_SEL = 2, MODE_POWER = 3,
    MODE_FINAL = 4, MODE_DONE = 5,
};

// Reductions taken over U after every sweep, per source.
enum Red : int32_t {
    RED_NP = 0,      // push cost n_p of the sweep (edges of pushed U and active V nodes): the V-side
                     // part in the gather slots [0, off_u), the U-side part in the update slots
    RED_CNT_SS = 1,  // #{x : r(x) > eps_b}
    RED_SUM_R = 2,   // sum_x y(x)/ws(x)   (times ws(u) = sum of r)
    RED_CNT_PI = 3,  // #{x : y(x) > eps_f/lambda}
    RED_SUM_Y = 4,   // sum_x y(x)          (= sum of the forward residue)
};

// Per-source state. The sweep kernels read the first block; the control
// kernel owns the rest.
struct ColState {
    int32_t ruleA, ruleB, convert, mode;
    double k_ss;         // eps_b / ws(u)
    double k_pi;         // eps_f / lambda
    double ws_src;       // ws(u)
    double alpha;
    // control
    double eps, eps_b, eps_f;
    double np;           // n_p of the current sub-algorithm
    double gamma;
    double two_e;        // 2|E|
    double ln_inv;       // ln(1/(1-alpha))
    int32_t t_rem;
    int32_t steps;
    // statistics
    int32_t ss_sel_iters, ss_seq_iters, pi_sel_iters, t, ss_switched, pi_returned;
    double np_ss, np_pi, sum_r_ss, sum_rf;
    double visits_u, visits_v;   // edge visits of all sweeps: pushed U nodes' edges, active V nodes' edges
    int32_t sparse_sweeps;       // sweeps whose pushed U nodes have fewer than |E|/16 edges
    // scheduling: a column reused for a new query keeps the old query's Y and
    // ACC until its first sweep, which reads them as y = e_src and ACC = 0
    int32_t fresh;
    int32_t src_row;     // internal id of the source
    int32_t qid;         // index of the query in the caller's arrays, -1 if none
    // warm start: signed residues; the combine uses pi_b as SS-Push returned it,
    // whose forward image the update stores in SNAP in the sweep after (snap)
    int32_t warm;
    int32_t snap;
    int32_t fell_back;   // a warm start was no better than the cold start: ran cold
    int32_t target;      // 0: beta (Algorithm 5); 1: pi(u, .) (PI-Push alone); 2: pi(., u) (SS-Push alone);
                         // 3: beta by PISP (SelectivePush, then PowerIteration from e_u);
                         // 4: pi(., u) by SelectivePush alone (MCSP's backward part)
    int32_t reset_y;     // the next sweep reads y = e_src (PISP's forward part) but keeps ACC
    double res_l1;       // sum_x |r_f(x)| of the warm start
    double res_max;      // max_x |r(x)|
};

struct Workspace {
    int cols = 0;                // allocated column count (power of 2)
    int elem = 0;                // bytes per value
    void* Y = nullptr;           // [n_u][cols] forward residue y = (ws/ws(u)) r
    void* ACC = nullptr;         // [n_u][cols] push estimate, later beta'
    void* S = nullptr;           // [n_u][cols] y/ws of the nodes pushed in the current sweep
    void* Q = nullptr;           // [n_v][cols] V-side residue of the current sweep
    void* partA = nullptr;       // [slots_v][cols] split-row partial sums
    void* partB = nullptr;       // [slots_u][cols]
    double* red = nullptr;       // [kNumRed][cols][n_part] per-block reductions
    int n_part = 0;
    ColState* st = nullptr;      // [cols]
    int32_t* n_active = nullptr; // device counter of unfinished sources
    int32_t* h_active = nullptr; // pinned host mirror
    void* SNAP = nullptr;        // [n_u][cols] warm starts: ACC when SS-Push returned (allocated on demand)
    void* scores = nullptr;      // [cols][n_u]: G during sweeps, row-major score scratch for top-k
    int32_t* ids_tmp = nullptr;  // [cols][kTopkTmpK] top-k scratch
    void* vals_tmp = nullptr;
    int32_t* ex_tmp = nullptr;   // [3][64]: exported columns, their excluded ids, a narrowing map
    ColState* adm = nullptr;     // [64] states of queries being admitted (asynchronous batches)
    size_t bytes = 0;
    // warm starts: an FP64 block that applies the two-hop operator to the
    // predictions of newly admitted queries (allocated on demand)
    int wcols = 0;
    void *wY = nullptr, *wS = nullptr, *wG = nullptr, *wQ = nullptr, *wpartA = nullptr, *wpartB = nullptr;
    double* wred = nullptr;
    ColState* wst = nullptr;
    int32_t* wn_active = nullptr;
    float* wP = nullptr;         // [n_u][wcols] predictions
    double* wres = nullptr;      // [2][wcols][blocks] residual norms per block
    int32_t* wcol_ids = nullptr; // [64] block column of each new query
    // sparse frontier steps of a one-source block (allocated on demand)
    int32_t* fF = nullptr;       // [n_u] frontier
    void* fS = nullptr;          // [n_u] y/ws of the frontier
    int64_t* fDeg = nullptr;     // [max(n_u, n_v)] degrees, then their inclusive scan in fOffs
    int64_t* fOffs = nullptr;
    int32_t* fTV = nullptr;      // [n_v] touched V nodes
    void* fQ = nullptr;          // [n_v] V-side residue of a sparse step, kept zero between steps
    int32_t* fMark = nullptr;    // [n_v] touched marks, kept zero between steps
    void* fCnt = nullptr;        // counters: |F|, |T_V|, sum d over F, sum d over T_V
    void* fScanTmp = nullptr;
    size_t fScanBytes = 0;
    unsigned long long* h_fCnt = nullptr;   // pinned mirror
    // sweep chunks captured as HIP graphs (one per column count), replayed per chunk
    hipGraphExec_t chunk_exec[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
};

struct Graph {
    int32_t nu = 0, nv = 0;
    int64_t ne = 0;
    int32_t dtype = BHPP_DTYPE_F32;
    int elem = 4;
    // internal (degree-ordered) adjacency
    int64_t* rp_u = nullptr; int32_t* ci_u = nullptr; void* w_u = nullptr;   // w_u holds w(x,v)/ws(v)
    int64_t* rp_v = nullptr; int32_t* ci_v = nullptr; void* w_v = nullptr;   // w_v holds w(x,v)
    void* iw_v = nullptr;            // per entry of W^T's rows: 1/ws of the entry's U node (graph dtype)
    float* inv_ws_u_f = nullptr; float* inv_ws_v_f = nullptr;     // F32 graphs
    double* inv_ws_u_d = nullptr; double* inv_ws_v_d = nullptr;   // both dtypes
    int32_t* deg_u = nullptr;    // degree of each internal U row
    uint64_t* end_bits_u = nullptr;  // bit e set iff entry e of the U rows ends its row
    uint64_t* end_bits_v = nullptr;
    int32_t* perm_u = nullptr;   // external U id -> internal
    int32_t* iperm_u = nullptr;  // internal -> external
    int32_t* iperm_v = nullptr;  // internal V id -> external
    TileSet tiles_u, tiles_v;
    // tiles_u with at most upd_rows(elem) whole rows per tile: the U-side gather
    // of 64-column blocks that applies the update itself keeps a tile's row sums
    // in LDS until the tile ends
    TileSet tiles_uf;
    // MCSP's alias tables (BHPP_BUILD_MCSP): rows of W and of W^T in caller ids
    int64_t *mc_rp_u = nullptr, *mc_rp_v = nullptr;
    double *mc_prob_u = nullptr, *mc_prob_v = nullptr;
    int32_t *mc_keep_u = nullptr, *mc_keep_v = nullptr, *mc_alias_u = nullptr, *mc_alias_v = nullptr;
    // external-order copies (BHPP_BUILD_KEEP_EXTERNAL)
    int64_t* x_rp_u = nullptr; int32_t* x_ci_u = nullptr; void* x_w_u = nullptr;
    int64_t* x_rp_v = nullptr; int32_t* x_ci_v = nullptr; void* x_w_v = nullptr;
    void* x_ws_u = nullptr; void* x_ws_v = nullptr;
    // host copies
    std::vector<double> h_ws_u;       // external order, FP64
    std::vector<int32_t> h_perm_u;    // external -> internal
    std::vector<int64_t> h_rp_u, h_rp_v;   // internal row offsets (tiles are rebuilt from them)
    bhpp_graph_summary info{};
    std::map<double, double> lambda_cache;   // alpha -> lambda
    int32_t tau = 0;
    // runtime
    std::mutex mu;
    Workspace ws;
    hipStream_t work = nullptr;      // the library's own stream (capturable), joined to the caller's
    // launch settings chosen by the autotuner (or defaults / BHPP_TUNE)
    int tile_edges = kTileEdges;
    int inflight = 8;
    int nt_stream = 0;
    int use_graphs = 1;
    int fuse_select = 1;             // 64-column blocks: gather A applies the push rule (no select pass)
    int sparse_steps = 1;            // one-source queries: sparse frontier steps while the frontier is small
    int narrow = 1;                  // batches narrow their block as sources finish
    int hub_lds = 0;                 // one-source gathers read the hub slice of their vector from LDS (hub=1)
    int buf_rows = 1;                // gather A (push rule applied, FP32) reads rows with buffer loads (bufa=1)
    int chunk_sweeps = 8;            // sweeps per launched chunk (captured graph), 1..8
    int async_sched = 1;             // queue-fed 64-column batches admit without draining the stream
    int fuse_update = 1;             // 64-column blocks: the U-side gather applies the update (no G array)
    int order_admit = 1;             // batches admit the longest expected queries first
    int upd_inflight = 2;            // rows whose y and ACC loads the fused update keeps in flight (2 or 4)
    double eps_b_paper = 0.5;        // eps_b / eps of Eq. (epsilon-b); info.eps_b_ratio is the one in use
    bool sticky_error = false;
    int n_servers = 0;               // live servers hold captured graphs of the tiles
    // profiling of the sweep kernels
    bool prof_on = false;
    double prof_ms[4] = {0, 0, 0, 0};
    int64_t prof_n[4] = {0, 0, 0, 0};
    double prof_bytes[4] = {0, 0, 0, 0};
    int64_t prof_live = 0;                // sweeps in which some query still ran
    std::vector<hipEvent_t> prof_ev;      // pairs, recorded on the query stream
    std::vector<int32_t> prof_kind;
    std::vector<double> prof_b;
};

// Push test of a lane's source: the rule becomes (compare y/ws(x) or y,
// threshold); RULE_NONE gets an infinite threshold. Residues of a warm-started
// query are signed, so callers pass |y| and |y/ws(x)| (cold-start residues are
// never negative, for them this is the plain test).
template <typename VT>
struct PushTest {
    bool by_ws;
    VT thr;
    __device__ __forceinline__ PushTest(int rule, VT kss, VT kpi) {
        by_ws = rule == RULE_SS;
        thr = rule == RULE_SS ? kss : rule == RULE_PI ? kpi : rule == RULE_ALL ? VT(0) : VT(INFINITY);
    }
    __device__ __forceinline__ bool operator()(VT y, VT yw) const { return (by_ws ? yw : y) > thr; }
};

// ---- host helpers (api.hip / build.hip / sweep.hip / topk.hip) ----
#define BHPP_HIP(expr)                                      \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return BHPP_DEVICE_ERROR;     \
    } while (0)

bhpp_status build_graph(int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* eu,
                        const int32_t* ev, const void* ew, const bhpp_graph_opts& opts,
                        hipStream_t s, Graph** out);
void free_graph(Graph* g);
bhpp_status compute_lambda(Graph* g, double alpha, int32_t tau, hipStream_t s, double* lambda_out);
// MCSP (mcsp.hip)
int64_t mc_walk_count(int32_t nu, double eps_f, double p_f);
bhpp_status mcsp_build_tables(Graph* g, const int64_t* xrp_u, const int32_t* xci_u, const double* xw_u,
                              const double* ws_u, const int64_t* xrp_v, const int32_t* xci_v, const double* xw_v,
                              const double* ws_v, hipStream_t s);
bhpp_status mcsp_counts(Graph* g, int32_t n, const int32_t* src_ext, double alpha, int64_t n_r, uint64_t seed,
                        uint32_t* counts, hipStream_t s);
bhpp_status mcsp_combine(Graph* g, void* rows, const uint32_t* counts, int32_t n, int64_t n_r, hipStream_t s);
// One sparse push step of a one-source block (frontier.hip): sparse_front
// (frontier, take, U->V scatter into w.fQ), then the caller's dense U-side
// gather of w.fQ into G, then sparse_finish (y += (1-alpha) G, reductions).
struct SparseStep {
    int64_t max_work = 0;   // in: above this sum of frontier degrees the step is not taken
    int red_blocks = 0, n_part = 0, off_u = 0;   // in: reduction slots of the phase control
    int32_t frontier = 0;   // out: |F|
    int64_t work_u = 0;     // out: sum of d(x) over F
    bool done = false;      // out: the step was taken
};
bhpp_status ensure_sparse(Graph* g, Workspace& w, hipStream_t s);
bhpp_status sparse_front(Graph* g, Workspace& w, SparseStep& io, hipStream_t s);
bhpp_status sparse_finish(Graph* g, Workspace& w, const SparseStep& io, const void* G, hipStream_t s);

struct Model;
bhpp_status run_queries(Graph* g, Model* model, const void* starts, bhpp_warm_stats* wstats, int32_t target,
                        int32_t n, const int32_t* src_ext, const double* eps, double alpha,
                        double lambda, void* scores_out, int32_t k, int32_t exclude_self,
                        int32_t* topk_ids, void* topk_vals, bhpp_query_stats* stats, hipStream_t s);
bhpp_status topk_rows(const void* scores, int32_t n_rows, int32_t n, int32_t k, const int32_t* exclude,
                      int32_t dtype, int32_t* ids_out, void* vals_out, hipStream_t s);
bhpp_status topk_rows_static(const void* scores, int32_t n_rows, int32_t n, int32_t k, const int32_t* exclude,
                             int32_t dtype, int32_t* ids_out, void* vals_out, hipStream_t s);
size_t topk_static_scratch_bytes();
bhpp_status ensure_workspace(Graph* g, int cols, hipStream_t s);
bhpp_status ensure_workspace(Graph* g, Workspace& w, int cols, hipStream_t s);
size_t workspace_bytes(const Graph* g, int cols);
struct Server;
bhpp_status server_create(Graph* g, Model* model, int max_width, double mem_budget, double alpha, double lambda, int k,
                          int excl, Server** out);
bhpp_status server_submit(Server* sv, int32_t src, double eps, int64_t tag);
bhpp_status server_poll(Server* sv, int64_t* tags, int32_t* ids, void* vals, bhpp_query_stats* st,
                        bhpp_warm_stats* wst, int32_t* n_out);
void server_info(Server* sv, bhpp_server_summary* out);
void server_destroy(Server* sv);
bhpp_status model_create(Graph* g, uint64_t seed, Model** out);
void model_free(Model* m);
int64_t model_num_params();
bhpp_status model_set_params(Model* m, const float* host);
bhpp_status model_get_params(Model* m, float* host);
void model_scales(const Model* m, double* c, double* sigma);
bhpp_status model_features(Model* m, float* out_ext, hipStream_t s);
bhpp_status model_loss_grad(Model* m, int n_src, const int32_t* src, int n_cand, const int32_t* cand,
                            const float* target, double* loss, float* grad_host);
bhpp_status model_train(Model* m, int n_src, const int32_t* src, int M, const int32_t* ids, const float* vals,
                        int steps, int batch_src, int batch_cand, double lr, uint64_t seed, float* loss_out);
bhpp_status model_embed(Model* m);
bool model_ready(const Model* m);
bhpp_status model_predict(Model* m, const int32_t* src_rows_host, int n, int cols, float* out, hipStream_t s);
bhpp_status model_predict_ext(Model* m, int n, const int32_t* src_ext, float* out, hipStream_t s);
bhpp_status gemm_test(int M, int N, int K, const uint16_t* A, int trans_a, const uint16_t* B, int trans_b, float* C,
                      hipStream_t s);
bhpp_status set_launch_config(Graph* g, const int* cfg);
bhpp_status build_tiles(const std::vector<int64_t>& rp, int32_t n_rows, int tile_edges, TileSet* ts,
                        int max_rows = 512);
// Rows per tile of tiles_uf: 4 KB of row sums (64 columns) per wavefront.
inline int upd_rows(int elem) { return 4096 / (64 * elem); }
void free_workspace(Workspace& w);
bhpp_status autotune(Graph* g, hipStream_t s, int* out_cfg);
void drop_chunk_graphs(Graph* g);
void free_tiles(TileSet* ts);

inline int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace bhpp
