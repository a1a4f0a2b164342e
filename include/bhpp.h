/*
 * bhpp.h -- C ABI of the MI355X (gfx950) library for approximate BHPP queries.
 *
 * Method: Yang, "Efficient and Effective Similarity Search over Bipartite
 * Graphs", WWW '22 (arXiv 2312.06724).
 *
 * Problem (Sec. 3.2, Definition 1): given a weighted undirected bipartite graph
 * G = (U u V, E), a restart probability alpha in (0,1) and a query node u in U,
 * return for every x in U a value beta'(u,x) with |beta(u,x) - beta'(u,x)| <= eps,
 * where beta(u,x) = pi(u,x) + pi(x,u) and pi is hidden personalized PageRank,
 * the random walk with restart over the two-hop U->V->U transition
 * P = D_U^-1 W D_V^-1 W^T (Sec. 3.1, Eq. (pmatrix); Eq. (hpp)).
 * The library runs Approx-BHPP (Algorithm 5): SS-Push (Algorithm 3), then
 * PI-Push (Algorithm 4, which ends with PowerIteration, Algorithm 1), then
 * beta' = pi_f + pi_b. For the cold start every returned value also satisfies
 * 0 <= beta - beta' <= eps up to floating-point rounding (Theorems 1-3).
 *
 * Conventions shared by every entry point:
 *  - Pointers documented as "device" must point to GPU memory of the current
 *    HIP device; pointers documented as "host" to CPU memory.
 *  - hip_stream is a hipStream_t (NULL = the null stream). All GPU work is
 *    enqueued on it. Calls return once the work is enqueued unless stated
 *    otherwise; the caller synchronises the stream before reading outputs.
 *  - Argument errors are detected before any work is enqueued and return a
 *    negative status; outputs are then untouched.
 *  - A HIP runtime failure returns BHPP_DEVICE_ERROR and is remembered on the
 *    graph handle: every later call on that handle returns BHPP_DEVICE_ERROR.
 *  - No C++ exception crosses this interface.
 *  - Node ids are 0-based: U ids in [0, n_u), V ids in [0, n_v).
 */
#ifndef BHPP_H
#define BHPP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bhpp_status;
#define BHPP_OK               0
#define BHPP_INVALID_ARG     -1  /* alpha not in (0,1), eps <= 0, k < 1, n < 0, NULL pointer, ... */
#define BHPP_OUT_OF_RANGE    -2  /* a node id outside [0,n_u) or [0,n_v) */
#define BHPP_ISOLATED_SOURCE -3  /* query source with no edge: ws(u) = 0 */
#define BHPP_BAD_WEIGHT      -4  /* an edge weight that is <= 0, NaN or infinite */
#define BHPP_OUT_OF_MEMORY   -5  /* a device or host allocation failed */
#define BHPP_DEVICE_ERROR    -6  /* HIP runtime error; sticky on the handle */
#define BHPP_NOT_SUPPORTED   -7  /* unsupported dtype or option */
#define BHPP_NO_CONVERGENCE  -8  /* the step limit of a query was reached */

#define BHPP_DTYPE_F32 0        /* FP32 weights, residues and scores, FP32 accumulation */
#define BHPP_DTYPE_F64 1        /* FP64 throughout */

/* Graph build options. */
typedef struct {
    double alpha;       /* restart probability in (0,1) used for lambda (Lemma 4) */
    int32_t tau;        /* PowerIteration rounds for lambda; < 0 selects the smallest tau
                           with n_u (1-alpha)^(tau+1) <= 1 */
    int32_t dtype;      /* BHPP_DTYPE_F32 or BHPP_DTYPE_F64; edge_w has this type */
    uint32_t flags;     /* bitwise OR of BHPP_BUILD_* */
} bhpp_graph_opts;

/* Keep the external-id CSR/CSC after the build so bhpp_graph_export can return
   them (doubles the structure memory). */
#define BHPP_BUILD_KEEP_EXTERNAL 1u
/* Do not renumber nodes by degree internally (identity order). */
#define BHPP_BUILD_NO_REORDER    2u
/* One-source queries sweep densely from the start. By default SS-Push's
   selective iterations of a lone source run as sparse frontier pushes (work
   proportional to the frontier's edges) while the frontier's edges number
   under |E|/16. */
#define BHPP_BUILD_DENSE_ONLY    4u
/* A batch keeps its sources in the columns they started in. By default, once
   no source is waiting and at most 32 of a 64-column block's columns are still
   running, the running columns are moved to the lowest columns and the sweeps
   skip the others (cheaper sweeps). Every column is computed independently of
   its position, so both give the same bits; the flag only turns the packing
   off.
   Launch settings can also be set at build time through the environment
   variable BHPP_TUNE, a comma-separated list of tile=<entries per work tile>,
   inflight=<4|8|16>, nt=<0|1> (non-temporal adjacency loads), graphs=<0|1>
   (replay sweeps as HIP graphs), sparse=<0|1> (as BHPP_BUILD_DENSE_ONLY),
   narrow=<0|1> (as BHPP_BUILD_FIXED_WIDTH), fuse=<0|1> (64-column blocks:
   the V-side gather applies the push rule itself instead of a separate
   selection pass; same bits either way), upd=<0|1> (64-column blocks: the
   U-side gather applies the update itself instead of a separate update
   pass; same bits per entry, per-source sums added in another order; on by
   default), bufa=<0|1> (64-column FP32 blocks: the V-side gather reads its
   rows with buffer loads; same bits either way; on by default) and
   hub=<0|1> (one-source gathers read the values of the
   highest-degree nodes from a copy in LDS; same bits either way; off by
   default). */
#define BHPP_BUILD_FIXED_WIDTH   8u
/* Build MCSP's Walker alias tables (bhpp_query_batch_mcsp): 16 bytes per
   adjacency entry per side. */
#define BHPP_BUILD_MCSP         16u

typedef struct bhpp_graph bhpp_graph;  /* opaque; owns all of its device memory */

/* Per-query counters of the two sub-algorithms. */
typedef struct {
    int32_t ss_sel_iters;   /* selective push iterations of SS-Push (Algorithm 3) */
    int32_t ss_seq_iters;   /* sequential push iterations of SS-Push */
    int32_t pi_sel_iters;   /* selective push iterations of PI-Push (Algorithm 4) */
    int32_t t;              /* PowerIteration rounds, Eq. (t); 0 if PI-Push returned early */
    int32_t ss_switched;    /* 1 if Eq. (bwd-np) switched SS-Push to sequential pushes */
    int32_t pi_returned;    /* 1 if Eq. (fwd-eps) ended PI-Push without power iterations */
    int32_t steps;          /* two-hop sweeps executed for this source */
    int32_t sparse_sweeps;  /* of those, sweeps whose pushed U nodes have fewer than |E|/16 edges
                               (a frontier small enough for edge-parallel push steps) */
    double np_ss;           /* push cost n_p recorded by SS-Push (edges touched) */
    double np_pi;           /* push cost n_p recorded by PI-Push */
    double gamma;           /* Eq. (gamma) */
    double sum_r_ss;        /* sum of the residue r when SS-Push returned */
    double sum_rf;          /* sum of the forward residue entering PowerIteration */
    /* Edge visits of every sweep of the query (all phases), split by side:
       visits_u sums d(x) over the U nodes pushed (the entries the V-side half
       reads with a non-zero value), visits_v sums d(v) over the V nodes with a
       non-zero residue. Their sum over the phases is the work measure n_p of
       Algorithms 3-4 extended to the sequential and PowerIteration sweeps. */
    double visits_u;
    double visits_v;
} bhpp_query_stats;

/* Graph summary and preprocessing results (Lemma 4, Eq. (epsilon-b)). */
typedef struct {
    int32_t n_u, n_v;
    int64_t n_edges;          /* distinct (u,v) pairs after merging duplicates */
    int32_t isolated_u;       /* U nodes with no edge */
    int32_t isolated_v;
    int32_t dtype;
    int32_t tau;              /* rounds used for lambda */
    double alpha;             /* alpha that lambda was computed for */
    double lambda;            /* Eq. (lambda) */
    double mu;                /* sqrt(|U||V|)/|E| */
    double eps_b_ratio;       /* eps_b / eps in use: Eq. (epsilon-b) (0.5 when mu >= 1) unless set or tuned */
    double ws_u_max, ws_u_min;/* over U nodes with at least one edge */
    double build_ms;          /* device time of the build, preprocessing included */
} bhpp_graph_summary;

/* Per-query report of a warm start (bhpp_query_batch_warm, servers with a model). */
typedef struct {
    double res_l1;        /* sum_x ws(x)/ws(u) |r(x)| of the start's signed residue (cold start: 1) */
    double res_max;       /* max_x |r(x)| (cold start: 1) */
    int32_t fell_back;    /* 1: the start was no better than the cold start, the query ran cold */
    int32_t reserved;
} bhpp_warm_stats;

/*
 * Build the graph and run the preprocessing step (Sec. 3.1; Lemma 4;
 * Eq. (epsilon-b); the paper excludes this step from query time, Sec. 5.4).
 *   n_u, n_v       partition sizes (> 0)
 *   n_edges        number of input edges (>= 0)
 *   edge_u, edge_v device int32[n_edges], endpoint ids
 *   edge_w         device float[n_edges] or double[n_edges] (opts->dtype), weights > 0
 *   opts           host; NULL = {alpha 0.15, tau auto, F32, no flags}
 *   out            host; receives the new handle
 * Duplicate (u,v) pairs are merged by summing their weights in FP64 in input
 * order. Input buffers are only read during the call and may be freed after
 * the stream has synchronised. This call synchronises hip_stream.
 * Errors: INVALID_ARG, OUT_OF_RANGE, BAD_WEIGHT, OUT_OF_MEMORY, DEVICE_ERROR,
 * NOT_SUPPORTED (dtype).
 */
bhpp_status bhpp_build_graph(int32_t n_u, int32_t n_v, int64_t n_edges,
                             const int32_t* edge_u, const int32_t* edge_v, const void* edge_w,
                             const bhpp_graph_opts* opts, void* hip_stream, bhpp_graph** out);

/*
 * One eps-approximate BHPP query (Definition 1, Algorithm 5) from source u.
 *   scores_out  device array of n_u values of the graph dtype; receives
 *               beta'(u, x) for every x in U, including u itself.
 *               Isolated x receive 0.
 *   stats       host, nullable
 * eps_b = eps * info.eps_b_ratio and eps_f = eps - eps_b (Algorithm 5).
 * If alpha differs from the graph's alpha, lambda is recomputed for it and cached.
 * Synchronises hip_stream before returning (phase control runs on the device;
 * the host waits for the source to finish).
 * Errors: INVALID_ARG, OUT_OF_RANGE, ISOLATED_SOURCE, NO_CONVERGENCE, DEVICE_ERROR.
 */
bhpp_status bhpp_query(bhpp_graph* g, int32_t source, double alpha, double eps,
                       void* scores_out, bhpp_query_stats* stats, void* hip_stream);

/*
 * n_src independent queries executed together: up to 64 sources share every
 * two-hop sweep as columns of one dense residue block, each source with its
 * own phase, thresholds and stopping point. With more than 64 sources the
 * block is fed from a queue: as sources finish, their results are written out
 * and the next sources take their columns, so sources of very different cost
 * share the sweeps without waiting for each other. Sources enter the block
 * longest expected first (smaller eps, then lower degree); outputs stay in
 * the caller's order, and a source's result does not depend on when it
 * entered.
 *   sources      host int32[n_src]
 *   eps          host double[n_src] (per-source error threshold) or NULL to use eps_all
 *   scores_out   device [n_src][n_u] row-major of the graph dtype, or NULL
 *   k            top-k size, 0 to skip top-k, else 1 <= k <= min(4096, n_u - (exclude_self != 0))
 *   exclude_self nonzero: the source itself is left out of its own top-k
 *   topk_ids     device int32[n_src][k] (required if k > 0)
 *   topk_vals    device [n_src][k] of the graph dtype (required if k > 0)
 *   stats        host bhpp_query_stats[n_src], nullable
 * Top-k order is (score descending, node id ascending). Synchronises hip_stream.
 * Errors: as bhpp_query.
 */
bhpp_status bhpp_query_batch(bhpp_graph* g, int32_t n_src, const int32_t* sources,
                             const double* eps, double alpha, double eps_all,
                             void* scores_out, int32_t k, int32_t exclude_self,
                             int32_t* topk_ids, void* topk_vals,
                             bhpp_query_stats* stats, void* hip_stream);

/*
 * Top-k of each row of a score matrix, ordered by (score descending, id
 * ascending); -0 ranks as +0. Used for the paper's retrieval of the nodes most
 * similar to a query node (Sec. 1; Sec. 5).
 *   scores       device [n_rows][n] row-major, float (dtype F32) or double (F64)
 *   exclude_ids  device int32[n_rows] id to leave out per row (-1 none), or NULL
 *   ids_out      device int32[n_rows][k]
 *   vals_out     device [n_rows][k] of dtype
 * Requires 1 <= k <= n (k <= n-1 for a row with an exclusion); k above 4096
 * returns NOT_SUPPORTED. Scores must not be NaN (the order of NaN is
 * unspecified). Does not synchronise.
 * Errors: INVALID_ARG, NOT_SUPPORTED, OUT_OF_MEMORY, DEVICE_ERROR.
 */
bhpp_status bhpp_topk(const void* scores, int32_t n_rows, int32_t n, int32_t k,
                      const int32_t* exclude_ids, int32_t dtype,
                      int32_t* ids_out, void* vals_out, void* hip_stream);

/*
 * bhpp_topk without any allocation, for callers that cannot allocate device
 * memory: code recorded into a HIP graph by stream capture, tight serving
 * loops, harnesses that forbid hipMalloc. Same arguments, order and results
 * as bhpp_topk; the caller still provides scores and outputs. The working
 * memory of the selection (per row: a state record, a 256-bin histogram and
 * k candidates) comes from one static device array of about 4.3 MB that the
 * library holds on each device it runs on until the process ends; its device
 * address is looked up on the first call on a device. Limits: n_rows <=
 * BHPP_TOPK_NOALLOC_MAX_ROWS and k <= BHPP_TOPK_NOALLOC_MAX_K, else
 * NOT_SUPPORTED before any work is enqueued. Every call on a device uses the
 * same array: calls that overlap on one device (different streams, or
 * threads enqueueing concurrently) race and must be serialised by the
 * caller; consecutive calls on one stream are safe (each clears what it uses
 * with a kernel, not a memset). Does not synchronise.
 * Errors: INVALID_ARG, NOT_SUPPORTED, DEVICE_ERROR.
 */
#define BHPP_TOPK_NOALLOC_MAX_ROWS 64
#define BHPP_TOPK_NOALLOC_MAX_K 4096
bhpp_status bhpp_topk_noalloc(const void* scores, int32_t n_rows, int32_t n, int32_t k,
                              const int32_t* exclude_ids, int32_t dtype,
                              int32_t* ids_out, void* vals_out, void* hip_stream);

/* Fill *out (host) with the graph summary. Errors: INVALID_ARG. */
bhpp_status bhpp_graph_info(const bhpp_graph* g, bhpp_graph_summary* out);

/*
 * Copy the external-id adjacency (requires BHPP_BUILD_KEEP_EXTERNAL):
 * rows of U with ascending v (rp_u int64[n_u+1], ci_u int32[nnz], w_u), rows of
 * V with ascending u (rp_v int64[n_v+1], ci_v int32[nnz], w_v), and the weighted
 * degrees of Eq. (d) ws_u[n_u], ws_v[n_v], each summed in FP64 along the row
 * in stored order and rounded once to the dtype. Weight and ws arrays have the
 * graph dtype. All pointers are device. Synchronises hip_stream.
 * Errors: INVALID_ARG, NOT_SUPPORTED (handle built without the flag), DEVICE_ERROR.
 */
bhpp_status bhpp_graph_export(const bhpp_graph* g, int64_t* rp_u, int32_t* ci_u, void* w_u,
                              int64_t* rp_v, int32_t* ci_v, void* w_v, void* ws_u, void* ws_v,
                              void* hip_stream);

/*
 * Device-time profile of the sweep kernels. While enabled, every launch of the
 * V-side gather (kind 0), the U-side gather (kind 1; in 64-column blocks it
 * also applies the update, and kind 2 then has no launches), the U-side update
 * (kind 2) and the push selection (kind 3; none in 64-column blocks, whose
 * V-side gather applies the push rule itself) on a query stream is bracketed by
 * HIP events on that stream and the
 * elapsed times are accumulated; bhpp_profile_read synchronises and returns,
 * per kind, the total milliseconds, the number of launches and the
 * algorithmic bytes those launches moved in total (per launch: the adjacency
 * read once plus each dense vector read or written once, for every column of
 * the block whether its source still runs or not: an upper bound when some
 * columns have finished; the query statistics give the sweeps each source
 * ran, from which the bytes of the running columns follow). enable = 0 stops
 * recording; enable = 1 also clears the totals. Errors: INVALID_ARG,
 * DEVICE_ERROR.
 */
bhpp_status bhpp_profile_enable(bhpp_graph* g, int32_t enable);
bhpp_status bhpp_profile_read(bhpp_graph* g, double ms[4], int64_t launches[4], double bytes[4]);
/* Number of sweeps run by query batches while profiling was on in which at
   least one query of the block was still running (host, *live_out). A batch
   runs its sweeps in chunks, so its last chunk can hold sweeps whose kernels
   find nothing to do and return at once; those are not counted. The
   launches of each kernel kind that did work equal this count. Errors:
   INVALID_ARG. */
bhpp_status bhpp_profile_sweeps(bhpp_graph* g, int64_t* live_out);

/*
 * Launch settings of the sweep kernels: config[0] entries per work tile (rows
 * longer than this are split into pieces), config[1] row gathers kept in
 * flight per wavefront in the 64-source gather (4, 8 or 16), config[2] 1 to
 * stream adjacency loads and row outputs past the caches, config[3] 1 to
 * replay each chunk of sweeps as a captured HIP graph. Results do not depend
 * on them, only the time does.
 *
 * bhpp_autotune times a few sweeps of a 64-source block for each candidate
 * (tile sizes 512/1024/2048/4096, 4/8/16 gathers in flight, streaming
 * off/on) on hip_stream's device, keeps the fastest and writes it to
 * config_out (host); it then sets the sweeps per chunk so that a chunk takes
 * about 2 ms. It synchronises hip_stream. bhpp_set_launch_config applies a setting saved
 * earlier (e.g. a cache keyed by the graph); bhpp_get_launch_config reads the
 * current one. Errors: INVALID_ARG (also while a server of this graph
 * exists: its captured sweeps refer to the current tiles), OUT_OF_MEMORY,
 * DEVICE_ERROR.
 */
bhpp_status bhpp_autotune(bhpp_graph* g, void* hip_stream, int32_t config_out[4]);
/*
 * Scheduling of query batches: sched[0] sweeps per launched chunk (1..8;
 * phase control runs on the device every sweep, the host looks at the block
 * only between chunks), sched[1] 1 to let queue-fed batches of more than 64
 * sources admit new queries without draining the stream (the host reads
 * copies of the column states one chunk behind and queues the finished
 * queries' extraction, top-k and the next admissions behind the running
 * sweeps), 0 for draining export rounds. Results do not depend on them.
 * The build sets sched[0] from an estimate of a 64-column sweep (chunks of
 * about 2 ms: 1 sweep from some 10M edges up, 8 on small graphs), and
 * bhpp_autotune from the sweep time it measured. Errors: INVALID_ARG (also
 * while a server of this graph exists).
 */
bhpp_status bhpp_set_schedule(bhpp_graph* g, const int32_t sched[2]);
bhpp_status bhpp_get_schedule(const bhpp_graph* g, int32_t sched_out[2]);
bhpp_status bhpp_set_launch_config(bhpp_graph* g, const int32_t config[4]);
bhpp_status bhpp_get_launch_config(const bhpp_graph* g, int32_t config_out[4]);

/* ------------------------------------------------------------------------
 * Learned warm start (an extension, not in the paper; it rests on Lemma 1 and
 * Lemma 3).
 *
 * Lemma 1's invariant pi(., u) = pi_b + Pi r holds for ANY start pi_b = y when
 * r = e_u - (y - (1-alpha) P y)/alpha (signed). A model predicts the start;
 * the residue is computed with one two-hop sweep accumulated in FP64, and
 * Algorithms 3-5 then run with |r| in every threshold, sum and budget test.
 * The combine takes pi_b as SS-Push returned it, so |beta - beta'| <= eps on
 * both sides (a cold start is within [0, eps]). A start whose residue is no
 * better than the cold start's (sum_x ws(x)/ws(u)|r(x)| >= 1 or max|r| >= 1)
 * is dropped and the query runs cold.
 *
 * The model: 64 hashed features per U node (degree, ws, neighbour-id
 * buckets), two towers f, g: 64 -> 256 -> 256 -> 128 with GELU, BF16 weights
 * and activations with FP32 accumulation (MFMA), and the prediction
 *     p_hat(u, x) = c ws(x) <f(u), g(x)>  of pi(u, x), clamped at 0
 * (the start y(x) = ws(u)/ws(x) p_hat(u, x)). Parameters are one FP32 vector of
 * BHPP_MODEL_PARAMS values: tower f then tower g, each W1[64][256] b1[256]
 * W2[256][256] b2[256] W3[256][128] b3[128] (row-major, y = x W + b).
 *
 * bhpp_model_create      computes the features, draws Glorot-uniform weights
 *                        from `seed` (host RNG), zero biases. The model keeps
 *                        a pointer to the graph: free it first.
 * bhpp_model_params      copies the FP32 parameters out (get, host, nullable)
 *                        and/or in (set, host, nullable; resets the optimizer).
 *                        c_out / tau_out (nullable): the score scale c and
 *                        the loss's tau.
 * bhpp_model_features    features of every U node, device FP32 [n_u][64], rows
 *                        in caller ids.
 * bhpp_model_loss_grad   one forward and backward pass (no update) on a batch:
 *                        sources src[n_src], candidates cand[n_cand] (host,
 *                        caller ids), targets[n_src][n_cand] (host FP32,
 *                        estimates of pi(u, x), NaN where unknown);
 *                        loss = mean over known T of (p_hat - T)^2 / (T + tau);
 *                        grad_out host FP32[BHPP_MODEL_PARAMS], nullable.
 * bhpp_model_train       Adam (lr, betas 0.9/0.999) for `steps` steps on lists
 *                        of BHPP values: ids[n_src][M] (caller ids, -1 for
 *                        none) and vals[n_src][M] = beta'(src_i, x), e.g. the
 *                        top entries of each vector from bhpp_query_batch
 *                        (exclude_self = 0) plus entries at random nodes.
 *                        Target of a listed pair: pi(u,x) = beta'(u,x)
 *                        ws(x)/(ws(u)+ws(x)) (Lemma 3); other pairs are left
 *                        out. Each step takes batch_src sources drawn from
 *                        `seed` and, as candidates, their listed nodes (at
 *                        most batch_cand). loss_out: host float[steps], nullable.
 * bhpp_model_embed       embeddings of every U node by both towers; needed
 *                        after training and before warm queries.
 * bhpp_query_batch_warm  bhpp_query_batch with every query warm-started from
 *                        the model; warm_out: host bhpp_warm_stats[n_src],
 *                        nullable. Errors as bhpp_query_batch, and
 *                        INVALID_ARG if the model has no embeddings.
 * ---------------------------------------------------------------------- */
#define BHPP_MODEL_FEATURES 64
#define BHPP_MODEL_PARAMS 230656

typedef struct bhpp_model bhpp_model;

bhpp_status bhpp_model_create(bhpp_graph* g, uint64_t seed, bhpp_model** out);
bhpp_status bhpp_model_params(bhpp_model* m, float* get_out, const float* set_in, double* c_out, double* tau_out);
bhpp_status bhpp_model_features(bhpp_model* m, float* out, void* hip_stream);
bhpp_status bhpp_model_loss_grad(bhpp_model* m, int32_t n_src, const int32_t* src, int32_t n_cand,
                                 const int32_t* cand, const float* targets, double* loss_out, float* grad_out);
bhpp_status bhpp_model_train(bhpp_model* m, int32_t n_src, const int32_t* src, int32_t M, const int32_t* ids,
                             const float* vals, int32_t steps, int32_t batch_src, int32_t batch_cand, double lr,
                             uint64_t seed, float* loss_out);
bhpp_status bhpp_model_embed(bhpp_model* m);
/* The start the model gives each source, as estimates of pi(u, x) (the warm
   queries' p_hat, self term included, clamped at 0): out device FP32
   [n_src][n_u], caller ids; sources host, caller ids. Needs embeddings.
   Synchronises hip_stream. Errors: INVALID_ARG, OUT_OF_RANGE,
   ISOLATED_SOURCE, OUT_OF_MEMORY, DEVICE_ERROR. */
bhpp_status bhpp_model_predict(bhpp_model* m, int32_t n_src, const int32_t* sources, float* out, void* hip_stream);
void bhpp_model_free(bhpp_model* m);
bhpp_status bhpp_query_batch_warm(bhpp_graph* g, bhpp_model* m, int32_t n_src, const int32_t* sources,
                                  const double* eps, double alpha, double eps_all, void* scores_out, int32_t k,
                                  int32_t exclude_self, int32_t* topk_ids, void* topk_vals, bhpp_query_stats* stats,
                                  bhpp_warm_stats* warm_out, void* hip_stream);

/* ------------------------------------------------------------------------
 * One direction of HPP alone (the sub-results Algorithm 5 combines), for
 * n_src sources as in bhpp_query_batch (no top-k):
 *   BHPP_HPP_FORWARD   scores_out[i][x] ~ pi(u_i, x), single-source HPP
 *                      (Eq. (hpp), a row of Pi) by PI-Push (Algorithm 4) from
 *                      (pi_b, r) = (0, e_u) with eps_f = eps: within
 *                      [pi - eps, pi] (Theorem 2);
 *   BHPP_HPP_BACKWARD  scores_out[i][x] ~ pi(x, u_i), single-target HPP (a
 *                      column of Pi) by SS-Push (Algorithm 3) with
 *                      eps_b = eps: within [pi - eps, pi] (Theorem 1).
 * scores_out: device [n_src][n_u] of the graph dtype (required). Errors: as
 * bhpp_query_batch, INVALID_ARG for another direction.
 * ---------------------------------------------------------------------- */
#define BHPP_HPP_FORWARD  0
#define BHPP_HPP_BACKWARD 1
bhpp_status bhpp_query_hpp(bhpp_graph* g, int32_t n_src, const int32_t* sources, const double* eps, double alpha,
                           double eps_all, int32_t direction, void* scores_out, bhpp_query_stats* stats,
                           void* hip_stream);

/* ------------------------------------------------------------------------
 * PISP, the baseline the paper compares Approx-BHPP with (Sec. 3.3,
 * Baselines and Challenges; Sec. 5.4, Fig. 3): for each source u, the
 * forward part pi(u, .) by PowerIteration (Algorithm 1) from e_u with t rounds,
 * t = log_{1/(1-alpha)}(2/eps) - 1 rounded up (the smallest t with
 * (1-alpha)^(t+1) <= eps/2), plus the backward part pi(., u) by SelectivePush
 * (Algorithm 2) with eps_b = eps/2 run until no U residue exceeds eps_b;
 * beta' = pi_f + pi_b, within [beta - eps, beta]. Arguments, outputs, batching
 * and errors as bhpp_query_batch. In the statistics ss_sel_iters counts the
 * SelectivePush iterations, np_ss their push cost and t the PowerIteration
 * rounds; the other phase counters stay 0.
 * ---------------------------------------------------------------------- */
bhpp_status bhpp_query_batch_pisp(bhpp_graph* g, int32_t n_src, const int32_t* sources,
                                  const double* eps, double alpha, double eps_all,
                                  void* scores_out, int32_t k, int32_t exclude_self,
                                  int32_t* topk_ids, void* topk_vals,
                                  bhpp_query_stats* stats, void* hip_stream);

/* ------------------------------------------------------------------------
 * MCSP, the paper's other baseline (Sec. 3.3, Baselines and Challenges;
 * Sec. 5.4, Fig. 3), on a graph built with BHPP_BUILD_MCSP: for each source
 * u, pi(u, .) estimated by MonteCarlo, n_r = 2 (1 + eps_f/3) ln(|U|/p_f) /
 * eps_f^2 random walks with restart (eps_f = eps/2, rounded up; the paper's
 * experiments use p_f = 1e-6), whose steps draw neighbours from Walker alias
 * tables (weights w/ws of the row); plus pi(., u) by SelectivePush
 * (Algorithm 2) with eps_b = eps/2; beta' = (walks ending at x)/n_r + pi_b(x),
 * within eps of beta with probability at least 1 - p_f.
 * The walks draw from Philox4x32-10 under the 64-bit seed: walk w of source u
 * takes at step s the counters (w, u, 2s, 0x4D435350) and (w, u, 2s + 1,
 * 0x4D435350) under the key (seed low 32 bits, seed high 32 bits); r0 of the
 * first block stops the walk if r0 < alpha 2^32, else (r1, r2) pick the U->V
 * step and (r3, first number of the second block) the V->U step: slot =
 * (r d) >> 32 of a row of d entries, kept iff r' 2^-32 < prob(slot), else
 * its alias. Outputs, top-k and statistics (of SelectivePush) as
 * bhpp_query_batch; scores_out may be NULL (the rows are then held in a
 * temporary buffer for the top-k); walks_out (host, nullable) receives n_r.
 * Synchronises hip_stream.
 * Errors: as bhpp_query_batch, NOT_SUPPORTED without the tables or when n_r
 * exceeds 2^32 - 1 (eps too small).
 * ---------------------------------------------------------------------- */
bhpp_status bhpp_query_batch_mcsp(bhpp_graph* g, int32_t n_src, const int32_t* sources, double eps,
                                  double alpha, double p_f, uint64_t seed, void* scores_out, int32_t k,
                                  int32_t exclude_self, int32_t* topk_ids, void* topk_vals,
                                  bhpp_query_stats* stats, int64_t* walks_out, void* hip_stream);

/* Warm start from caller-given starts instead of a model: starts is device
   [n_src][n_u] of the graph dtype, row i = estimates of pi(sources[i], x) for
   every x (caller ids; any sign; the start is rounded to FP32). Same
   residue, phases, bound and fallback as bhpp_query_batch_warm. */
bhpp_status bhpp_query_batch_start(bhpp_graph* g, const void* starts, int32_t n_src, const int32_t* sources,
                                   const double* eps, double alpha, double eps_all, void* scores_out, int32_t k,
                                   int32_t exclude_self, int32_t* topk_ids, void* topk_vals, bhpp_query_stats* stats,
                                   bhpp_warm_stats* warm_out, void* hip_stream);

/* GEMM on the matrix cores as the model runs it, exposed for its layout test:
   C[M][N] = A B, A BF16 [M][K] (or [K][M] if trans_a), B BF16 [K][N] (or
   [N][K] if trans_b), C FP32 [M][N]; all device. Errors: INVALID_ARG. */
bhpp_status bhpp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, int32_t trans_a, const uint16_t* B,
                           int32_t trans_b, float* C, void* hip_stream);

/* ------------------------------------------------------------------------
 * Serving (continuous batching). Requests are the queries of Definition 1
 * (source u, error bound eps) answered by Algorithm 5 and reduced to their
 * top-k; they arrive one at a time and leave when done.
 *
 * A server owns a resident query block of `width` columns on its own HIP
 * stream: width is the largest power of two <= max_width (1..64) whose
 * device workspace fits in mem_budget_bytes (<= 0: no cap); the workspace of
 * width 64 on a 1M x 2M graph is about 1.6 GB in FP32 (plus about 3 GB with a
 * model, for the warm starts). k: 1 <= k <= min(4096, n_u - (exclude_self
 * != 0)). Admission: a request enters the block at the next poll, in the
 * lowest free column (the sweeps skip the columns above the highest one
 * held). With a model (nullable; it must have
 * embeddings) admitted requests are warm-started as in bhpp_query_batch_warm
 * (warm_out of the poll, nullable, reports it); once the model's recent
 * starts fall back in 90% of cases (after 32 tries) only every 16th admission
 * is warm-started, until the rate improves: a useless start only costs time.
 *
 * bhpp_server_submit queues a request (host call, no device work; source in
 * caller ids, eps > 0, tag is returned with the result). It may run on
 * another thread while a poll runs.
 * bhpp_server_poll admits queued requests into free columns, runs one chunk
 * of sweeps (8) and synchronises, then writes the requests that finished:
 * n_out entries of tags_out[n], ids_out[n][k] and vals_out[n][k] (HOST
 * memory, values in the graph's dtype, order as bhpp_topk) and, if not NULL,
 * stats_out[n]. capacity (entries the outputs hold) must be >= width. With
 * nothing queued or running it returns at once with n_out = 0.
 * A request's result does not depend on the other requests in the block.
 * Destroy every server of a graph before freeing the graph.
 * Errors: INVALID_ARG, OUT_OF_RANGE, ISOLATED_SOURCE (submit checks the
 * source), OUT_OF_MEMORY (create: the budget does not fit width 1),
 * NO_CONVERGENCE, DEVICE_ERROR.
 * ---------------------------------------------------------------------- */
typedef struct bhpp_server bhpp_server;

typedef struct {
    int32_t width;          /* columns of the resident block */
    int32_t k;
    int64_t queued;         /* submitted, not yet admitted */
    int64_t running;        /* admitted, not finished */
    int64_t completed;
    int64_t sweeps;         /* sweeps run by this server */
    double resident_bytes;  /* device bytes of its workspace */
    double lambda;          /* Lemma 4 bound used by its PI-Push thresholds */
    int64_t warm_started;   /* requests that got a warm start from the model */
    int64_t warm_fell_back; /* ... whose start was dropped for the cold start */
} bhpp_server_summary;

bhpp_status bhpp_server_create(bhpp_graph* g, bhpp_model* model, int32_t max_width, double mem_budget_bytes,
                               double alpha, int32_t k, int32_t exclude_self, bhpp_server** out);
bhpp_status bhpp_server_submit(bhpp_server* s, int32_t source, double eps, int64_t tag);
bhpp_status bhpp_server_poll(bhpp_server* s, int32_t capacity, int64_t* tags_out, int32_t* ids_out,
                             void* vals_out, bhpp_query_stats* stats_out, bhpp_warm_stats* warm_out,
                             int32_t* n_out);
bhpp_status bhpp_server_info(const bhpp_server* s, bhpp_server_summary* out);
void bhpp_server_destroy(bhpp_server* s);

/* ------------------------------------------------------------------------
 * The split of eps between SS-Push and PI-Push. Theorem 3 holds for any
 * eps_b in (0, eps); Eq. (epsilon-b) picks eps_b from mu, which only affects
 * speed. bhpp_set_eps_b_ratio sets eps_b = ratio * eps for later queries
 * (0 < ratio < 1; ratio = 0 restores Eq. (epsilon-b)). bhpp_tune_eps_b runs
 * the sample sources (host ids, eps, alpha; no outputs) once per candidate
 * ratio and writes, per candidate (host arrays [n_ratios], each nullable),
 * the run's wall time in ms, the mean gamma of Eq. (gamma) over the sample
 * (the quantity of Fig. 1) and the mean number of sweeps per source; it keeps
 * the fastest ratio and returns it in *best_out. It synchronises hip_stream.
 * Errors: INVALID_ARG, OUT_OF_RANGE, ISOLATED_SOURCE, NO_CONVERGENCE,
 * DEVICE_ERROR.
 * ---------------------------------------------------------------------- */
bhpp_status bhpp_set_eps_b_ratio(bhpp_graph* g, double ratio);
bhpp_status bhpp_tune_eps_b(bhpp_graph* g, int32_t n_src, const int32_t* sources, double eps, double alpha,
                            int32_t n_ratios, const double* ratios, double* ms_out, double* gamma_out,
                            double* sweeps_out, double* best_out, void* hip_stream);

/* Free the handle and all device memory it owns (NULL is ignored). The caller
   must make sure no work using it is still running. */
void bhpp_free_graph(bhpp_graph* g);

/* Static description of a status code. */
const char* bhpp_status_string(bhpp_status s);

#ifdef __cplusplus
}
#endif

#endif /* BHPP_H */
