/*
 * FP64 CPU oracle for approximate BHPP queries.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this code. It shares no code, header
 * or table with the GPU library, and the GPU library never calls it.
 *
 * It follows Yang, "Efficient and Effective Similarity Search over Bipartite
 * Graphs" (WWW '22), in the paper's own notation:
 *   ws(.)            weighted degree, Eq. (d)                        Sec. 3.1
 *   U = D_U^-1 W, V = D_V^-1 W^T, P = U V (never formed here)         Sec. 3.1, Eq. (pmatrix)
 *   pi(u,x) = sum_l alpha (1-alpha)^l P^l(u,x)                        Eq. (hpp)
 *   PowerIteration                                                    Algorithm 1 (Sec. 3.3)
 *   one push iteration (U->V then V->U)                               Algorithm 2 (Sec. 3.3)
 *   SS-Push: selective pushes, budget Eq. (bwd-np), sequential pushes Algorithm 3 (Sec. 4.1)
 *   PI-Push: thresholds ws(u)/ws(x) eps_f/lambda, Eq. (fwd-eps),
 *            Eq. (gamma), Eq. (fwd-np), Eq. (fppr), Eq. (fresidue),
 *            Eq. (t), then PowerIteration                              Algorithm 4 (Sec. 4.2)
 *   Approx-BHPP: beta' = pi_f + pi_b                                  Algorithm 5 (Sec. 4.3)
 *   lambda                                                            Lemma 4, Eq. (lambda)
 *   eps_b                                                             Eq. (epsilon-b) (Sec. 4.3)
 * Everything is FP64 and single-threaded per query; loops run over node ids in
 * increasing order. The only parallelism is across independent queries, and
 * in the block form of the exact series (orc_hpp_forward_block), whose output
 * rows are split over threads while each value keeps the single-source order
 * of operations.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nu, nv;
    int64_t ne;              /* distinct edges after merging duplicates */
    int64_t* rp_u;           /* CSR of W, rows = U: rp_u[nu+1] */
    int32_t* ci_u;           /* neighbour v of each entry, ascending per row */
    double* w_u;             /* w(u,v) */
    int64_t* rp_v;           /* CSR of W^T, rows = V */
    int32_t* ci_v;           /* neighbour u, ascending per row */
    double* w_v;
    double* ws_u;            /* Eq. (d), summed in the row order above */
    double* ws_v;
} orc_graph;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ERANGE = -2, ORC_EISOLATED = -3, ORC_EWEIGHT = -4, ORC_ENOMEM = -5,
       ORC_ENOCONV = -6 };

/* A query needs O(log 1/eps) push iterations (Sec. 4.3); this cap only turns a
 * runaway loop into an error. */
#define ORC_MAX_ITERS 20000

void orc_free(orc_graph* g) {
    if (!g) return;
    free(g->rp_u); free(g->ci_u); free(g->w_u);
    free(g->rp_v); free(g->ci_v); free(g->w_v);
    free(g->ws_u); free(g->ws_v);
    free(g);
}

/* Stable counting sort of idx[0..n) by key[idx[i]] in [0, nk). */
static int counting_sort(const int32_t* key, int32_t nk, const int64_t* idx, int64_t n, int64_t* out) {
    int64_t* cnt = (int64_t*)calloc((size_t)nk + 1, sizeof(int64_t));
    if (!cnt) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; ++i) cnt[key[idx[i]] + 1]++;
    for (int32_t k = 0; k < nk; ++k) cnt[k + 1] += cnt[k];
    for (int64_t i = 0; i < n; ++i) out[cnt[key[idx[i]]]++] = idx[i];
    free(cnt);
    return ORC_OK;
}

/*
 * Build both adjacency directions of the undirected bipartite graph (Sec. 3.1).
 * Duplicate (u,v) pairs are merged by summing their weights in input order.
 * Returns NULL and sets *err on failure.
 */
orc_graph* orc_build(int32_t nu, int32_t nv, int64_t ne, const int32_t* eu, const int32_t* ev,
                     const double* w, int* err) {
    *err = ORC_OK;
    if (nu <= 0 || nv <= 0 || ne < 0) { *err = ORC_EINVAL; return NULL; }
    for (int64_t i = 0; i < ne; ++i) {
        if (eu[i] < 0 || eu[i] >= nu || ev[i] < 0 || ev[i] >= nv) { *err = ORC_ERANGE; return NULL; }
        if (!(w[i] > 0.0) || !isfinite(w[i])) { *err = ORC_EWEIGHT; return NULL; }
    }
    orc_graph* g = (orc_graph*)calloc(1, sizeof(orc_graph));
    int64_t* a = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ne > 0 ? ne : 1));
    int64_t* b = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ne > 0 ? ne : 1));
    if (!g || !a || !b) { *err = ORC_ENOMEM; free(a); free(b); orc_free(g); return NULL; }
    g->nu = nu; g->nv = nv;
    for (int64_t i = 0; i < ne; ++i) a[i] = i;
    /* LSD: stable by v, then stable by u => ordered by (u, v, input position) */
    if (counting_sort(ev, nv, a, ne, b) || counting_sort(eu, nu, b, ne, a)) {
        *err = ORC_ENOMEM; free(a); free(b); orc_free(g); return NULL;
    }
    /* merge duplicates */
    int64_t m = 0;
    int32_t* su = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    int32_t* sv = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    double* sw = (double*)malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
    if (!su || !sv || !sw) { *err = ORC_ENOMEM; return NULL; }
    for (int64_t i = 0; i < ne; ++i) {
        int64_t e = a[i];
        if (m > 0 && su[m - 1] == eu[e] && sv[m - 1] == ev[e]) {
            sw[m - 1] += w[e];
        } else {
            su[m] = eu[e]; sv[m] = ev[e]; sw[m] = w[e]; ++m;
        }
    }
    g->ne = m;
    g->rp_u = (int64_t*)calloc((size_t)nu + 1, sizeof(int64_t));
    g->rp_v = (int64_t*)calloc((size_t)nv + 1, sizeof(int64_t));
    g->ci_u = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    g->ci_v = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    g->w_u = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    g->w_v = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    g->ws_u = (double*)calloc((size_t)nu, sizeof(double));
    g->ws_v = (double*)calloc((size_t)nv, sizeof(double));
    if (!g->rp_u || !g->rp_v || !g->ci_u || !g->ci_v || !g->w_u || !g->w_v || !g->ws_u || !g->ws_v) {
        *err = ORC_ENOMEM; orc_free(g); return NULL;
    }
    for (int64_t i = 0; i < m; ++i) {
        g->rp_u[su[i] + 1]++;
        g->rp_v[sv[i] + 1]++;
        g->ci_u[i] = sv[i];
        g->w_u[i] = sw[i];
    }
    for (int32_t x = 0; x < nu; ++x) g->rp_u[x + 1] += g->rp_u[x];
    for (int32_t y = 0; y < nv; ++y) g->rp_v[y + 1] += g->rp_v[y];
    /* transpose: walking CSR rows in order keeps each V row sorted by u */
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)nv);
    if (!fill) { *err = ORC_ENOMEM; orc_free(g); return NULL; }
    for (int32_t y = 0; y < nv; ++y) fill[y] = g->rp_v[y];
    for (int64_t i = 0; i < m; ++i) {
        int64_t p = fill[sv[i]]++;
        g->ci_v[p] = su[i];
        g->w_v[p] = sw[i];
    }
    free(fill);
    /* Eq. (d): weighted degrees, summed along each row in stored order */
    for (int32_t x = 0; x < nu; ++x) {
        double s = 0.0;
        for (int64_t p = g->rp_u[x]; p < g->rp_u[x + 1]; ++p) s += g->w_u[p];
        g->ws_u[x] = s;
    }
    for (int32_t y = 0; y < nv; ++y) {
        double s = 0.0;
        for (int64_t p = g->rp_v[y]; p < g->rp_v[y + 1]; ++p) s += g->w_v[p];
        g->ws_v[y] = s;
    }
    free(a); free(b); free(su); free(sv); free(sw);
    return g;
}

int64_t orc_nnz(const orc_graph* g) { return g->ne; }

void orc_export(const orc_graph* g, int64_t* rp_u, int32_t* ci_u, double* w_u, int64_t* rp_v,
                int32_t* ci_v, double* w_v, double* ws_u, double* ws_v) {
    memcpy(rp_u, g->rp_u, sizeof(int64_t) * ((size_t)g->nu + 1));
    memcpy(rp_v, g->rp_v, sizeof(int64_t) * ((size_t)g->nv + 1));
    memcpy(ci_u, g->ci_u, sizeof(int32_t) * (size_t)g->ne);
    memcpy(ci_v, g->ci_v, sizeof(int32_t) * (size_t)g->ne);
    memcpy(w_u, g->w_u, sizeof(double) * (size_t)g->ne);
    memcpy(w_v, g->w_v, sizeof(double) * (size_t)g->ne);
    memcpy(ws_u, g->ws_u, sizeof(double) * (size_t)g->nu);
    memcpy(ws_v, g->ws_v, sizeof(double) * (size_t)g->nv);
}

/* ---------------------------------------------------------------------------
 * Row-vector and column-vector products with P = U V, without forming P.
 * ------------------------------------------------------------------------- */

/* out = p * U * V  (row vector p over U; Algorithm 1's (pi U) V) */
static void row_times_P(const orc_graph* g, const double* p, double* tmp_v, double* out) {
    for (int32_t y = 0; y < g->nv; ++y) {        /* (p U)(v) = sum_x p(x) w(x,v)/ws(x) */
        double s = 0.0;
        for (int64_t q = g->rp_v[y]; q < g->rp_v[y + 1]; ++q) {
            int32_t x = g->ci_v[q];
            s += p[x] * g->w_v[q] / g->ws_u[x];
        }
        tmp_v[y] = s;
    }
    for (int32_t x = 0; x < g->nu; ++x) {        /* ((pU) V)(x) = sum_v (pU)(v) w(v,x)/ws(v) */
        double s = 0.0;
        for (int64_t q = g->rp_u[x]; q < g->rp_u[x + 1]; ++q) {
            int32_t y = g->ci_u[q];
            s += tmp_v[y] * g->w_u[q] / g->ws_v[y];
        }
        out[x] = s;
    }
}

/* out = P * c  (column vector c over U): (P c)(x) = sum_v U(x,v) sum_y V(v,y) c(y) */
static void P_times_col(const orc_graph* g, const double* c, double* tmp_v, double* out) {
    for (int32_t y = 0; y < g->nv; ++y) {
        double s = 0.0;
        for (int64_t q = g->rp_v[y]; q < g->rp_v[y + 1]; ++q) s += g->w_v[q] * c[g->ci_v[q]];
        tmp_v[y] = g->ws_v[y] > 0.0 ? s / g->ws_v[y] : 0.0;
    }
    for (int32_t x = 0; x < g->nu; ++x) {
        if (g->ws_u[x] == 0.0) { out[x] = 0.0; continue; }
        double s = 0.0;
        for (int64_t q = g->rp_u[x]; q < g->rp_u[x + 1]; ++q) s += g->w_u[q] * tmp_v[g->ci_u[q]];
        out[x] = s / g->ws_u[x];
    }
}

/*
 * Algorithm 1 (PowerIteration): pi <- e; t times pi <- e + (1-alpha) (pi U) V;
 * return alpha * pi. e and out are row vectors over U; out may alias nothing.
 */
int orc_power_iteration(const orc_graph* g, const double* e, double alpha, int32_t t, double* out) {
    double* pi = (double*)malloc(sizeof(double) * (size_t)g->nu);
    double* nx = (double*)malloc(sizeof(double) * (size_t)g->nu);
    double* tv = (double*)malloc(sizeof(double) * (size_t)g->nv);
    if (!pi || !nx || !tv) { free(pi); free(nx); free(tv); return ORC_ENOMEM; }
    memcpy(pi, e, sizeof(double) * (size_t)g->nu);
    for (int32_t i = 1; i <= t; ++i) {
        row_times_P(g, pi, tv, nx);
        for (int32_t x = 0; x < g->nu; ++x) pi[x] = e[x] + (1.0 - alpha) * nx[x];
    }
    for (int32_t x = 0; x < g->nu; ++x) out[x] = alpha * pi[x];
    free(pi); free(nx); free(tv);
    return ORC_OK;
}

/* Number of series terms L so that the dropped mass (1-alpha)^(L+1) <= tail. */
static int32_t series_terms(double alpha, double tail) {
    int32_t L = 0;
    double m = 1.0 - alpha;
    while (m > tail) { m *= (1.0 - alpha); ++L; }
    return L;
}

/*
 * Eq. (hpp) summed directly as a truncated series, forward direction:
 * out(x) = sum_{l=0..L} alpha (1-alpha)^l (e_u P^l)(x), i.e. pi(u, x).
 * Every entry is short of the exact value by at most the tail (1-alpha)^(L+1).
 */
int orc_hpp_forward(const orc_graph* g, int32_t u, double alpha, double tail, double* out, int32_t* terms) {
    if (u < 0 || u >= g->nu) return ORC_ERANGE;
    int32_t L = series_terms(alpha, tail);
    double* p = (double*)calloc((size_t)g->nu, sizeof(double));
    double* nx = (double*)malloc(sizeof(double) * (size_t)g->nu);
    double* tv = (double*)malloc(sizeof(double) * (size_t)g->nv);
    if (!p || !nx || !tv) { free(p); free(nx); free(tv); return ORC_ENOMEM; }
    p[u] = 1.0;
    double c = alpha;
    for (int32_t x = 0; x < g->nu; ++x) out[x] = c * p[x];
    for (int32_t l = 1; l <= L; ++l) {
        if (g->ws_u[u] == 0.0) break;
        row_times_P(g, p, tv, nx);
        double* t = p; p = nx; nx = t;
        c *= (1.0 - alpha);
        for (int32_t x = 0; x < g->nu; ++x) out[x] += c * p[x];
    }
    if (terms) *terms = L;
    free(p); free(nx); free(tv);
    return ORC_OK;
}

/* Eq. (hpp), backward direction: out(x) = pi(x, u) = sum_l alpha (1-alpha)^l (P^l e_u)(x). */
int orc_hpp_backward(const orc_graph* g, int32_t u, double alpha, double tail, double* out, int32_t* terms) {
    if (u < 0 || u >= g->nu) return ORC_ERANGE;
    int32_t L = series_terms(alpha, tail);
    double* c = (double*)calloc((size_t)g->nu, sizeof(double));
    double* nx = (double*)malloc(sizeof(double) * (size_t)g->nu);
    double* tv = (double*)malloc(sizeof(double) * (size_t)g->nv);
    if (!c || !nx || !tv) { free(c); free(nx); free(tv); return ORC_ENOMEM; }
    c[u] = 1.0;
    double k = alpha;
    for (int32_t x = 0; x < g->nu; ++x) out[x] = k * c[x];
    for (int32_t l = 1; l <= L; ++l) {
        P_times_col(g, c, tv, nx);
        double* t = c; c = nx; nx = t;
        k *= (1.0 - alpha);
        for (int32_t x = 0; x < g->nu; ++x) out[x] += k * c[x];
    }
    if (terms) *terms = L;
    free(c); free(nx); free(tv);
    return ORC_OK;
}

int orc_hpp_forward_many(const orc_graph* g, int32_t n, const int32_t* src, double alpha, double tail,
                         double* out, int32_t nthreads) {
    int rc = ORC_OK;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
#endif
    for (int32_t i = 0; i < n; ++i) {
        int r = orc_hpp_forward(g, src[i], alpha, tail, out + (size_t)i * (size_t)g->nu, NULL);
        if (r != ORC_OK) rc = r;
    }
    (void)nthreads;
    return rc;
}

int orc_max_threads(void);

/*
 * Eq. (hpp), forward direction, for n sources at once: out[i][x] = pi(src[i], x),
 * the same truncated series as orc_hpp_forward. The n row vectors are kept
 * node-major (p[x][i]) so one pass over the adjacency serves all of them; for
 * every source the products and sums are the ones orc_hpp_forward makes, in
 * the same order, so each row of out equals its single-source value bit for
 * bit. Rows of the two products are split over threads (each output row is
 * written by one thread; nothing is shared). Isolated sources give e_u alpha.
 */
int orc_hpp_forward_block(const orc_graph* g, int32_t n, const int32_t* src, double alpha, double tail,
                          double* out, int32_t nthreads, int32_t progress) {
    if (n <= 0) return ORC_OK;
    for (int32_t i = 0; i < n; ++i)
        if (src[i] < 0 || src[i] >= g->nu) return ORC_ERANGE;
    const int32_t L = series_terms(alpha, tail);
    const size_t nu = (size_t)g->nu, nv = (size_t)g->nv, m = (size_t)n;
    double* p = (double*)calloc(nu * m, sizeof(double));
    double* nx = (double*)malloc(sizeof(double) * nu * m);
    double* tv = (double*)malloc(sizeof(double) * nv * m);
    double* acc = (double*)malloc(sizeof(double) * nu * m);
    if (!p || !nx || !tv || !acc) {
        free(p); free(nx); free(tv); free(acc);
        return ORC_ENOMEM;
    }
    for (int32_t i = 0; i < n; ++i) p[(size_t)src[i] * m + i] = 1.0;
    double c = alpha;
    for (size_t j = 0; j < nu * m; ++j) acc[j] = c * p[j];
    const int nt = nthreads > 0 ? nthreads : orc_max_threads();
    for (int32_t l = 1; l <= L; ++l) {
        /* (p U)(v) = sum_x p(x) w(x,v)/ws(x), per source, as row_times_P */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4096) num_threads(nt)
#endif
        for (int32_t y = 0; y < g->nv; ++y) {
            double* s = tv + (size_t)y * m;
            for (size_t i = 0; i < m; ++i) s[i] = 0.0;
            for (int64_t q = g->rp_v[y]; q < g->rp_v[y + 1]; ++q) {
                const int32_t x = g->ci_v[q];
                const double* px = p + (size_t)x * m;
                for (size_t i = 0; i < m; ++i) s[i] += px[i] * g->w_v[q] / g->ws_u[x];
            }
        }
        /* ((pU) V)(x) = sum_v (pU)(v) w(v,x)/ws(v) */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4096) num_threads(nt)
#endif
        for (int32_t x = 0; x < g->nu; ++x) {
            double* s = nx + (size_t)x * m;
            for (size_t i = 0; i < m; ++i) s[i] = 0.0;
            for (int64_t q = g->rp_u[x]; q < g->rp_u[x + 1]; ++q) {
                const int32_t y = g->ci_u[q];
                const double* ty = tv + (size_t)y * m;
                for (size_t i = 0; i < m; ++i) s[i] += ty[i] * g->w_u[q] / g->ws_v[y];
            }
        }
        /* a source without edges keeps p = e_u and stops adding (orc_hpp_forward breaks) */
        for (int32_t i = 0; i < n; ++i)
            if (g->ws_u[src[i]] == 0.0)
                for (size_t x = 0; x < nu; ++x) nx[x * m + i] = 0.0;
        double* t = p; p = nx; nx = t;
        c *= (1.0 - alpha);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
        for (int64_t x = 0; x < (int64_t)nu; ++x)
            for (size_t i = 0; i < m; ++i) acc[(size_t)x * m + i] += c * p[(size_t)x * m + i];
        if (progress > 0 && (l % progress == 0 || l == L)) {
            fprintf(stderr, "[oracle] exact series of %d sources: term %d of %d\n", (int)n, (int)l, (int)L);
            fflush(stderr);
        }
    }
    for (size_t i = 0; i < m; ++i)
        for (size_t x = 0; x < nu; ++x) out[i * nu + x] = acc[x * m + i];
    free(p); free(nx); free(tv); free(acc);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Preprocessing: Lemma 4 and Eq. (epsilon-b)
 * ------------------------------------------------------------------------- */

/* Eq. (epsilon-b): eps_b = eps (1-mu)/(2-mu), mu = sqrt(|U||V|)/|E|; if mu >= 1
 * the formula leaves (0, eps), and eps/2 is used instead. */
double orc_eps_b(int32_t nu, int32_t nv, int64_t ne, double eps) {
    double mu = sqrt((double)nu * (double)nv) / (double)ne;
    if (!(mu < 1.0)) return 0.5 * eps;
    return eps * (1.0 - mu) / (2.0 - mu);
}

/* tau for Lemma 4: the smallest tau with |U| (1-alpha)^(tau+1) <= 1 */
int32_t orc_default_tau(int32_t nu, double alpha) {
    int32_t tau = 0;
    double m = (double)nu * (1.0 - alpha);
    while (m > 1.0) { m *= (1.0 - alpha); ++tau; }
    return tau;
}

/*
 * Lemma 4, Eq. (lambda): rho = PowerIteration(e = 1, t = tau);
 * lambda = min(max rho + |U| (1-alpha)^(tau+1), max ws / min ws), where the
 * ws ratio runs over nodes with ws > 0 (an isolated node's column sum is alpha).
 */
int orc_lambda(const orc_graph* g, double alpha, int32_t tau, double* lambda_out, double* rho_max_out) {
    double* one = (double*)malloc(sizeof(double) * (size_t)g->nu);
    double* rho = (double*)malloc(sizeof(double) * (size_t)g->nu);
    if (!one || !rho) { free(one); free(rho); return ORC_ENOMEM; }
    for (int32_t x = 0; x < g->nu; ++x) one[x] = 1.0;
    int rc = orc_power_iteration(g, one, alpha, tau, rho);
    if (rc) { free(one); free(rho); return rc; }
    double rmax = 0.0, wmax = 0.0, wmin = INFINITY;
    for (int32_t x = 0; x < g->nu; ++x) {
        if (rho[x] > rmax) rmax = rho[x];
        if (g->ws_u[x] > 0.0) {
            if (g->ws_u[x] > wmax) wmax = g->ws_u[x];
            if (g->ws_u[x] < wmin) wmin = g->ws_u[x];
        }
    }
    double a = rmax + (double)g->nu * pow(1.0 - alpha, (double)tau + 1.0);
    double b = wmax / wmin;
    *lambda_out = a < b ? a : b;
    if (rho_max_out) *rho_max_out = rmax;
    free(one); free(rho);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Approx-BHPP (Algorithms 2-5)
 * ------------------------------------------------------------------------- */

typedef struct {
    int32_t ss_sel_iters, ss_seq_iters, pi_sel_iters, t;
    int32_t ss_switched;     /* 1 if Eq. (bwd-np) sent SS-Push to sequential pushes */
    int32_t pi_returned;     /* 1 if Eq. (fwd-eps) ended PI-Push (no power iterations) */
    double np_ss, np_pi;     /* push cost n_p recorded in each algorithm */
    double gamma;            /* Eq. (gamma) */
    double sum_r_ss;         /* sum of r when SS-Push returned */
    double sum_rf;           /* sum of the forward residue entering PowerIteration */
} orc_stats;

/* phase ids passed to the trace callback */
enum { PH_SS_SEL = 0, PH_SS_SEQ = 1, PH_PI_SEL = 2 };
typedef void (*orc_trace_fn)(void* ctx, int32_t phase, int32_t iter, const double* pi_b, const double* r);

typedef struct {
    double* r;     /* residue on U */
    double* rv;    /* residue on V */
    double* pib;   /* pi_b(x, u) */
    double* thr;   /* per-node push threshold of the current phase */
    double* tmp;
} orc_work;

static void work_free(orc_work* w) { free(w->r); free(w->rv); free(w->pib); free(w->thr); free(w->tmp); }

static int work_alloc(orc_work* w, const orc_graph* g) {
    memset(w, 0, sizeof(*w));
    w->r = (double*)calloc((size_t)g->nu, sizeof(double));
    w->rv = (double*)calloc((size_t)g->nv, sizeof(double));
    w->pib = (double*)calloc((size_t)g->nu, sizeof(double));
    w->thr = (double*)calloc((size_t)g->nu, sizeof(double));
    w->tmp = (double*)calloc((size_t)g->nu, sizeof(double));
    if (!w->r || !w->rv || !w->pib || !w->thr || !w->tmp) { work_free(w); return ORC_ENOMEM; }
    return ORC_OK;
}

/*
 * One iteration of Algorithm 2's loop body with per-node threshold thr:
 * every x in U with r(x) > thr(x) gives alpha r(x) to pi_b(x) and sends
 * (1-alpha) w(x,v)/ws(v) r(x) to each neighbour v, then r(x) <- 0; next every v
 * in V with r(v) > 0 sends w(y,v)/ws(y) r(v) to each neighbour y, then r(v) <- 0.
 * The U loop changes only V residues and the pushed node's own residue, so
 * testing r(x) while walking x in id order selects exactly the nodes that were
 * above threshold when the loop started. Returns the edges touched (n_p).
 */
static double push_iteration(const orc_graph* g, orc_work* w, double alpha) {
    double np = 0.0;
    for (int32_t x = 0; x < g->nu; ++x) {
        double rx = w->r[x];
        if (!(rx > w->thr[x])) continue;
        for (int64_t q = g->rp_u[x]; q < g->rp_u[x + 1]; ++q) {
            int32_t v = g->ci_u[q];
            w->rv[v] += (1.0 - alpha) * g->w_u[q] / g->ws_v[v] * rx;
        }
        w->pib[x] += alpha * rx;
        w->r[x] = 0.0;
        np += (double)(g->rp_u[x + 1] - g->rp_u[x]);
    }
    for (int32_t v = 0; v < g->nv; ++v) {
        double rv = w->rv[v];
        if (!(rv > 0.0)) continue;
        for (int64_t q = g->rp_v[v]; q < g->rp_v[v + 1]; ++q) {
            int32_t y = g->ci_v[q];
            w->r[y] += g->w_v[q] / g->ws_u[y] * rv;
        }
        w->rv[v] = 0.0;
        np += (double)(g->rp_v[v + 1] - g->rp_v[v]);
    }
    return np;
}

static double log_base(double alpha, double x) { return log(x) / log(1.0 / (1.0 - alpha)); }

int32_t orc_t(double sum_rf, double eps_f, double alpha);

/*
 * Algorithm 5 for source u. Outputs (each |U| doubles, NULL to skip):
 *   beta   = beta'(u, x)
 *   pi_f   = the forward estimate of pi(u, x)  (Algorithm 4's output)
 *   pi_b   = the backward estimate of pi(x, u) (after PI-Push's pushes)
 */
/* Algorithm 5 with a cap on the push iterations (ORC_ENOCONV past it); work,
 * if not NULL, receives the edges touched: the n_p of every push iteration
 * and 2|E| per PowerIteration round. */
static int approx_bhpp_core(const orc_graph* g, int32_t u, double alpha, double eps, double eps_b, double lambda,
                            double* beta, double* pi_f_out, double* pi_b_out, orc_stats* st,
                            orc_trace_fn trace, void* ctx, int32_t cap, double* work);

int orc_approx_bhpp(const orc_graph* g, int32_t u, double alpha, double eps, double eps_b, double lambda,
                    double* beta, double* pi_f_out, double* pi_b_out, orc_stats* st,
                    orc_trace_fn trace, void* ctx) {
    return approx_bhpp_core(g, u, alpha, eps, eps_b, lambda, beta, pi_f_out, pi_b_out, st, trace, ctx,
                            ORC_MAX_ITERS, NULL);
}

static int approx_bhpp_core(const orc_graph* g, int32_t u, double alpha, double eps, double eps_b, double lambda,
                            double* beta, double* pi_f_out, double* pi_b_out, orc_stats* st,
                            orc_trace_fn trace, void* ctx, int32_t cap, double* work) {
    if (u < 0 || u >= g->nu) return ORC_ERANGE;
    if (!(alpha > 0.0 && alpha < 1.0) || !(eps > 0.0) || !(eps_b > 0.0 && eps_b < eps) || !(lambda > 0.0))
        return ORC_EINVAL;
    if (g->ws_u[u] == 0.0) return ORC_EISOLATED;
    orc_stats s;
    memset(&s, 0, sizeof(s));
    orc_work w;
    if (work_alloc(&w, g)) return ORC_ENOMEM;
    const int32_t nu = g->nu;
    const double E2 = 2.0 * (double)g->ne;
    const double wsu = g->ws_u[u];

    /* ---- Algorithm 3 (SS-Push), target u ---- */
    w.r[u] = 1.0;
    for (int32_t x = 0; x < nu; ++x) w.thr[x] = eps_b;
    double np = 0.0;
    int ss_done = 0;
    int32_t iters = 0;
    for (;;) {                                   /* selective pushes */
        if (++iters > cap) { work_free(&w); return ORC_ENOCONV; }
        { const double d = push_iteration(g, &w, alpha); np += d; if (work) *work += d; }
        ++s.ss_sel_iters;
        if (trace) trace(ctx, PH_SS_SEL, s.ss_sel_iters, w.pib, w.r);
        double rmax = 0.0, rsum = 0.0;
        for (int32_t x = 0; x < nu; ++x) { if (w.r[x] > rmax) rmax = w.r[x]; rsum += w.r[x]; }
        if (rmax <= eps_b || rsum <= eps_b) { ss_done = 1; break; }
        if (np >= E2 * log_base(alpha, 1.0 / rsum)) break;   /* Eq. (bwd-np) */
    }
    s.np_ss = np;
    if (!ss_done) {
        s.ss_switched = 1;
        for (int32_t x = 0; x < nu; ++x) w.thr[x] = 0.0;     /* eps_b replaced by 0 */
        for (;;) {                               /* sequential pushes */
            double rmax = 0.0, rsum = 0.0;
            for (int32_t x = 0; x < nu; ++x) { if (w.r[x] > rmax) rmax = w.r[x]; rsum += w.r[x]; }
            if (!(rmax > eps_b && rsum > eps_b)) break;
            if (++iters > cap) { work_free(&w); return ORC_ENOCONV; }
            { const double d = push_iteration(g, &w, alpha); s.np_ss += d; if (work) *work += d; }
            ++s.ss_seq_iters;
            if (trace) trace(ctx, PH_SS_SEQ, s.ss_seq_iters, w.pib, w.r);
        }
    }
    {
        double rsum = 0.0;
        for (int32_t x = 0; x < nu; ++x) rsum += w.r[x];
        s.sum_r_ss = rsum;
    }

    /* ---- Algorithm 4 (PI-Push), source u ---- */
    const double eps_f = eps - eps_b;            /* Algorithm 5 */
    double gamma = 0.0;                          /* Eq. (gamma) */
    for (int32_t x = 0; x < nu; ++x) gamma += g->ws_u[x] / wsu * w.r[x];
    s.gamma = gamma;
    for (int32_t x = 0; x < nu; ++x)             /* threshold ws(u)/ws(x) eps_f/lambda */
        w.thr[x] = g->ws_u[x] > 0.0 ? wsu / g->ws_u[x] * eps_f / lambda : INFINITY;
    np = 0.0;
    int pi_returned = 0;
    for (;;) {
        if (++iters > cap) { work_free(&w); return ORC_ENOCONV; }
        { const double d = push_iteration(g, &w, alpha); np += d; if (work) *work += d; }
        ++s.pi_sel_iters;
        if (trace) trace(ctx, PH_PI_SEL, s.pi_sel_iters, w.pib, w.r);
        int all_below = 1;                       /* Eq. (fwd-eps) for every node */
        double fsum = 0.0;
        for (int32_t x = 0; x < nu; ++x) {
            if (w.r[x] > w.thr[x]) all_below = 0;
            fsum += g->ws_u[x] / wsu * w.r[x];
        }
        if (all_below) { pi_returned = 1; break; }
        if (np >= E2 * log_base(alpha, gamma / fsum)) break; /* Eq. (fwd-np) */
    }
    s.np_pi = np;
    s.pi_returned = pi_returned;
    double* pif = w.tmp;
    for (int32_t x = 0; x < nu; ++x) pif[x] = g->ws_u[x] / wsu * w.pib[x];   /* Eq. (fppr) */
    if (!pi_returned) {
        double* rf = (double*)malloc(sizeof(double) * (size_t)nu);
        double* pr = (double*)malloc(sizeof(double) * (size_t)nu);
        if (!rf || !pr) { free(rf); free(pr); work_free(&w); return ORC_ENOMEM; }
        double fsum = 0.0;
        for (int32_t x = 0; x < nu; ++x) { rf[x] = g->ws_u[x] / wsu * w.r[x]; fsum += rf[x]; }  /* Eq. (fresidue) */
        s.sum_rf = fsum;
        int32_t t = orc_t(fsum, eps_f, alpha);                                              /* Eq. (t) */
        s.t = t;
        if (work) *work += E2 * (double)t;
        int rc = orc_power_iteration(g, rf, alpha, t, pr);                                   /* Algorithm 1 */
        if (rc) { free(rf); free(pr); work_free(&w); return rc; }
        for (int32_t x = 0; x < nu; ++x) pif[x] += pr[x];
        free(rf); free(pr);
    }

    /* ---- Algorithm 5, combine ---- */
    if (beta) for (int32_t x = 0; x < nu; ++x) beta[x] = pif[x] + w.pib[x];
    if (pi_f_out) memcpy(pi_f_out, pif, sizeof(double) * (size_t)nu);
    if (pi_b_out) memcpy(pi_b_out, w.pib, sizeof(double) * (size_t)nu);
    if (st) *st = s;
    work_free(&w);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Warm start (not in the paper; it rests on Lemma 1 and Lemma 3).
 *
 * Lemma 1's invariant pi(., u) = pi_b + Pi r (Pi = alpha (I - (1-alpha) P)^-1
 * applied to the column vector r) holds for ANY start pi_b = y if the residue
 * is the signed r = e_u - (y - (1-alpha) P y) / alpha, since
 * Pi (I - (1-alpha) P) = alpha I; every push keeps it, whatever the signs.
 * With signed residues every test of Algorithms 3 and 4 uses |r|, and a V
 * node is pushed when its residue is non-zero.
 *
 * Error bound (two-sided). With pi_b* the backward estimate when SS-Push
 * returns and r* its residue, |pi(x,u) - pi_b*(x)| = |(Pi r*)(x)| <= max|r*|
 * (rows of Pi sum to 1, Pi >= 0), and max|r*| <= eps_b or sum|r*| <= eps_b
 * when SS-Push returns. PI-Push then continues on (pi_b, r); by Lemma 3 the
 * forward value is pi(u,x) = ws(x)/ws(u) pi_b(x) + (r_f Pi)(x) with
 * r_f = ws/ws(u) r, whose remainder after PowerIteration with t sweeps is at
 * most (1-alpha)^(t+1) sum|r_f| <= eps_f in L1, and at most
 * max|r_f| lambda <= eps_f when PI-Push returns (Lemma 4). The combine
 * therefore takes pi_b* (the backward estimate as SS-Push returned it):
 * beta' = pi_f + pi_b*, |beta - beta'| <= eps_b + eps_f = eps.
 *
 * Fallback: if the start is no better than a cold start
 * (sum|r_f| >= 1 or max|r| >= 1), the query runs cold (orc_approx_bhpp).
 * ---------------------------------------------------------------------- */
typedef struct {
    double res_l1;      /* sum_x ws(x)/ws(u) |r(x)| of the warm start */
    double res_max;     /* max_x |r(x)| */
    int32_t fell_back;  /* 1: ran cold */
    int32_t pad;
} orc_warm_info;

/* (P y)(x) = sum_v w(x,v)/ws(x) sum_x' w(x',v)/ws(v) y(x') (Eq. (pmatrix)), into out. */
static void apply_P(const orc_graph* g, const double* y, double* yv, double* out) {
    for (int32_t v = 0; v < g->nv; ++v) {
        double s = 0.0;
        for (int64_t q = g->rp_v[v]; q < g->rp_v[v + 1]; ++q) s += g->w_v[q] * y[g->ci_v[q]];
        yv[v] = g->ws_v[v] > 0.0 ? s / g->ws_v[v] : 0.0;
    }
    for (int32_t x = 0; x < g->nu; ++x) {
        double s = 0.0;
        for (int64_t q = g->rp_u[x]; q < g->rp_u[x + 1]; ++q) s += g->w_u[q] * yv[g->ci_u[q]];
        out[x] = g->ws_u[x] > 0.0 ? s / g->ws_u[x] : 0.0;
    }
}

/* Algorithm 2's loop body with signed residues: push x if |r(x)| > thr(x),
 * then every v with r(v) != 0. Returns n_p. */
static double push_iteration_signed(const orc_graph* g, orc_work* w, double alpha) {
    double np = 0.0;
    for (int32_t x = 0; x < g->nu; ++x) {
        double rx = w->r[x];
        if (!(fabs(rx) > w->thr[x])) continue;
        for (int64_t q = g->rp_u[x]; q < g->rp_u[x + 1]; ++q) {
            int32_t v = g->ci_u[q];
            w->rv[v] += (1.0 - alpha) * g->w_u[q] / g->ws_v[v] * rx;
        }
        w->pib[x] += alpha * rx;
        w->r[x] = 0.0;
        np += (double)(g->rp_u[x + 1] - g->rp_u[x]);
    }
    for (int32_t v = 0; v < g->nv; ++v) {
        double rv = w->rv[v];
        if (rv == 0.0) continue;
        for (int64_t q = g->rp_v[v]; q < g->rp_v[v + 1]; ++q) {
            int32_t y = g->ci_v[q];
            w->r[y] += g->w_v[q] / g->ws_u[y] * rv;
        }
        w->rv[v] = 0.0;
        np += (double)(g->rp_v[v + 1] - g->rp_v[v]);
    }
    return np;
}

/* Warm-start residue of a start y (backward coordinates: y(x) estimates
 * pi(x,u)): r = e_u - (y - (1-alpha) P y)/alpha. */
int orc_warm_residue(const orc_graph* g, int32_t u, double alpha, const double* y, double* r_out) {
    if (u < 0 || u >= g->nu) return ORC_ERANGE;
    double* yv = (double*)malloc(sizeof(double) * (size_t)g->nv);
    double* py = (double*)malloc(sizeof(double) * (size_t)g->nu);
    if (!yv || !py) { free(yv); free(py); return ORC_ENOMEM; }
    apply_P(g, y, yv, py);
    for (int32_t x = 0; x < g->nu; ++x)
        r_out[x] = (x == u ? 1.0 : 0.0) - (y[x] - (1.0 - alpha) * py[x]) / alpha;
    free(yv); free(py);
    return ORC_OK;
}

int orc_approx_bhpp_warm(const orc_graph* g, int32_t u, double alpha, double eps, double eps_b, double lambda,
                         const double* y0, double* beta, orc_stats* st, orc_warm_info* wi) {
    if (u < 0 || u >= g->nu) return ORC_ERANGE;
    if (!(alpha > 0.0 && alpha < 1.0) || !(eps > 0.0) || !(eps_b > 0.0 && eps_b < eps) || !(lambda > 0.0))
        return ORC_EINVAL;
    if (g->ws_u[u] == 0.0) return ORC_EISOLATED;
    const int32_t nu = g->nu;
    const double wsu = g->ws_u[u];
    orc_warm_info info;
    memset(&info, 0, sizeof(info));
    orc_work w;
    if (work_alloc(&w, g)) return ORC_ENOMEM;
    int rc = orc_warm_residue(g, u, alpha, y0, w.r);
    if (rc) { work_free(&w); return rc; }
    for (int32_t x = 0; x < nu; ++x) {
        if (g->ws_u[x] == 0.0) continue;
        info.res_l1 += g->ws_u[x] / wsu * fabs(w.r[x]);
        if (fabs(w.r[x]) > info.res_max) info.res_max = fabs(w.r[x]);
    }
    if (!(info.res_l1 < 1.0 && info.res_max < 1.0)) {
        info.fell_back = 1;
        work_free(&w);
        if (wi) *wi = info;
        return orc_approx_bhpp(g, u, alpha, eps, eps_b, lambda, beta, NULL, NULL, st, NULL, NULL);
    }
    for (int32_t x = 0; x < nu; ++x) w.pib[x] = y0[x];
    orc_stats s;
    memset(&s, 0, sizeof(s));
    const double E2 = 2.0 * (double)g->ne;

    /* ---- Algorithm 3 with |r| ---- */
    for (int32_t x = 0; x < nu; ++x) w.thr[x] = eps_b;
    double np = 0.0;
    int ss_done = 0;
    int32_t iters = 0;
    for (;;) {
        if (++iters > ORC_MAX_ITERS) { work_free(&w); return ORC_ENOCONV; }
        np += push_iteration_signed(g, &w, alpha);
        ++s.ss_sel_iters;
        double rmax = 0.0, rsum = 0.0;
        for (int32_t x = 0; x < nu; ++x) { double a = fabs(w.r[x]); if (a > rmax) rmax = a; rsum += a; }
        if (rmax <= eps_b || rsum <= eps_b) { ss_done = 1; break; }
        if (np >= E2 * log_base(alpha, 1.0 / rsum)) break;
    }
    s.np_ss = np;
    if (!ss_done) {
        s.ss_switched = 1;
        for (int32_t x = 0; x < nu; ++x) w.thr[x] = 0.0;
        for (;;) {
            double rmax = 0.0, rsum = 0.0;
            for (int32_t x = 0; x < nu; ++x) { double a = fabs(w.r[x]); if (a > rmax) rmax = a; rsum += a; }
            if (!(rmax > eps_b && rsum > eps_b)) break;
            if (++iters > ORC_MAX_ITERS) { work_free(&w); return ORC_ENOCONV; }
            s.np_ss += push_iteration_signed(g, &w, alpha);
            ++s.ss_seq_iters;
        }
    }
    double* pib_ss = (double*)malloc(sizeof(double) * (size_t)nu);
    if (!pib_ss) { work_free(&w); return ORC_ENOMEM; }
    memcpy(pib_ss, w.pib, sizeof(double) * (size_t)nu);      /* pi_b* */
    {
        double rsum = 0.0;
        for (int32_t x = 0; x < nu; ++x) rsum += fabs(w.r[x]);
        s.sum_r_ss = rsum;
    }

    /* ---- Algorithm 4 with |r| ---- */
    const double eps_f = eps - eps_b;
    double gamma = 0.0;
    for (int32_t x = 0; x < nu; ++x) gamma += g->ws_u[x] / wsu * fabs(w.r[x]);
    s.gamma = gamma;
    for (int32_t x = 0; x < nu; ++x)
        w.thr[x] = g->ws_u[x] > 0.0 ? wsu / g->ws_u[x] * eps_f / lambda : INFINITY;
    np = 0.0;
    int pi_returned = 0;
    for (;;) {
        if (++iters > ORC_MAX_ITERS) { free(pib_ss); work_free(&w); return ORC_ENOCONV; }
        np += push_iteration_signed(g, &w, alpha);
        ++s.pi_sel_iters;
        int all_below = 1;
        double fsum = 0.0;
        for (int32_t x = 0; x < nu; ++x) {
            if (fabs(w.r[x]) > w.thr[x]) all_below = 0;
            fsum += g->ws_u[x] / wsu * fabs(w.r[x]);
        }
        if (all_below) { pi_returned = 1; break; }
        if (np >= E2 * log_base(alpha, gamma / fsum)) break;
    }
    s.np_pi = np;
    s.pi_returned = pi_returned;
    double* pif = w.tmp;
    for (int32_t x = 0; x < nu; ++x) pif[x] = g->ws_u[x] / wsu * w.pib[x];   /* Eq. (fppr) */
    if (!pi_returned) {
        double* rf = (double*)malloc(sizeof(double) * (size_t)nu);
        double* pr = (double*)malloc(sizeof(double) * (size_t)nu);
        if (!rf || !pr) { free(rf); free(pr); free(pib_ss); work_free(&w); return ORC_ENOMEM; }
        double fsum = 0.0;
        for (int32_t x = 0; x < nu; ++x) { rf[x] = g->ws_u[x] / wsu * w.r[x]; fsum += fabs(rf[x]); }
        s.sum_rf = fsum;
        int32_t t = orc_t(fsum, eps_f, alpha);
        s.t = t;
        rc = orc_power_iteration(g, rf, alpha, t, pr);
        if (rc) { free(rf); free(pr); free(pib_ss); work_free(&w); return rc; }
        for (int32_t x = 0; x < nu; ++x) pif[x] += pr[x];
        free(rf); free(pr);
    }
    if (beta) for (int32_t x = 0; x < nu; ++x) beta[x] = pif[x] + pib_ss[x];
    if (st) *st = s;
    if (wi) *wi = info;
    free(pib_ss);
    work_free(&w);
    return ORC_OK;
}

/* Warm-started queries over a thread pool; y0 is [n][nu]. */
int orc_approx_bhpp_warm_many(const orc_graph* g, int32_t n, const int32_t* src, double alpha, double eps,
                              double eps_b, double lambda, const double* y0, double* beta, orc_stats* st,
                              orc_warm_info* wi, int32_t nthreads) {
    int rc = ORC_OK;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
#endif
    for (int32_t i = 0; i < n; ++i) {
        int r = orc_approx_bhpp_warm(g, src[i], alpha, eps, eps_b, lambda, y0 + (size_t)i * (size_t)g->nu,
                                     beta ? beta + (size_t)i * (size_t)g->nu : NULL, st ? st + i : NULL,
                                     wi ? wi + i : NULL);
        if (r != ORC_OK) rc = r;
    }
    (void)nthreads;
    return rc;
}

/* Independent queries over a thread pool: the CPU baseline. */
int orc_approx_bhpp_many(const orc_graph* g, int32_t n, const int32_t* src, double alpha, double eps,
                         double eps_b, double lambda, double* beta, orc_stats* st, int32_t nthreads) {
    int rc = ORC_OK;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
#endif
    for (int32_t i = 0; i < n; ++i) {
        int r = orc_approx_bhpp(g, src[i], alpha, eps, eps_b, lambda,
                                beta ? beta + (size_t)i * (size_t)g->nu : NULL, NULL, NULL,
                                st ? st + i : NULL, NULL, NULL);
        if (r != ORC_OK) rc = r;
    }
    (void)nthreads;
    return rc;
}

/*
 * PISP, the baseline of Sec. 3.3 (Baselines and Challenges) against which the
 * paper measures Approx-BHPP (Sec. 5.4, Fig. 3). Two independent parts:
 *   forward:  pi_f = PowerIteration(e_u, t) (Algorithm 1), t the paper's
 *             log_{1/(1-alpha)}(2/eps) - 1 rounded up (as Eq. (t) with a
 *             unit residue and eps_f = eps/2), so that the dropped mass
 *             (1-alpha)^(t+1) is at most eps/2;
 *   backward: pi_b = SelectivePush (Algorithm 2) from r = e_u with
 *             eps_b = eps/2: push iterations with threshold eps_b until no U
 *             residue exceeds eps_b (its loop's only exit), so that
 *             0 <= pi(x, u) - pi_b(x) <= eps/2;
 * beta' = pi_f + pi_b. Outputs as orc_approx_bhpp (NULL to skip).
 */
typedef struct {
    int32_t t;          /* PowerIteration rounds */
    int32_t sp_iters;   /* SelectivePush iterations */
    double np;          /* edges touched by SelectivePush */
} orc_pisp_stats;

/* SelectivePush (Algorithm 2) from r = e_u: push iterations with threshold
 * thr_b (its eps_b) until no U residue exceeds it (the loop's only exit); pib
 * receives pi_b(x, u), within [pi(x, u) - thr_b, pi(x, u)]. */
static int selective_push(const orc_graph* g, int32_t u, double alpha, double thr_b, double* pib, int32_t* iters,
                          double* np) {
    orc_work w;
    if (work_alloc(&w, g)) return ORC_ENOMEM;
    for (int32_t x = 0; x < g->nu; ++x) w.thr[x] = thr_b;
    w.r[u] = 1.0;
    *iters = 0;
    *np = 0.0;
    for (;;) {
        if (*iters >= ORC_MAX_ITERS) { work_free(&w); return ORC_ENOCONV; }
        *np += push_iteration(g, &w, alpha);
        *iters += 1;
        double rmax = 0.0;
        for (int32_t x = 0; x < g->nu; ++x) rmax = w.r[x] > rmax ? w.r[x] : rmax;
        if (!(rmax > thr_b)) break;
    }
    memcpy(pib, w.pib, sizeof(double) * (size_t)g->nu);
    work_free(&w);
    return ORC_OK;
}

int orc_pisp(const orc_graph* g, int32_t u, double alpha, double eps, double* beta, double* pi_f_out,
             double* pi_b_out, orc_pisp_stats* st) {
    if (u < 0 || u >= g->nu) return ORC_ERANGE;
    if (!(alpha > 0.0 && alpha < 1.0) || !(eps > 0.0)) return ORC_EINVAL;
    if (g->ws_u[u] == 0.0) return ORC_EISOLATED;
    orc_pisp_stats s;
    memset(&s, 0, sizeof(s));
    /* forward part */
    s.t = orc_t(1.0, 0.5 * eps, alpha);
    double* e = (double*)calloc((size_t)g->nu, sizeof(double));
    double* pif = (double*)malloc(sizeof(double) * (size_t)g->nu);
    if (!e || !pif) { free(e); free(pif); return ORC_ENOMEM; }
    e[u] = 1.0;
    int rc = orc_power_iteration(g, e, alpha, s.t, pif);
    free(e);
    if (rc) { free(pif); return rc; }
    /* backward part */
    double* pib = (double*)malloc(sizeof(double) * (size_t)g->nu);
    if (!pib) { free(pif); return ORC_ENOMEM; }
    rc = selective_push(g, u, alpha, 0.5 * eps, pib, &s.sp_iters, &s.np);
    if (rc) { free(pib); free(pif); return rc; }
    for (int32_t x = 0; x < g->nu; ++x) {
        if (beta) beta[x] = pif[x] + pib[x];
        if (pi_f_out) pi_f_out[x] = pif[x];
        if (pi_b_out) pi_b_out[x] = pib[x];
    }
    if (st) *st = s;
    free(pib);
    free(pif);
    return ORC_OK;
}

int orc_pisp_many(const orc_graph* g, int32_t n, const int32_t* src, double alpha, double eps, double* beta,
                  orc_pisp_stats* st, int32_t nthreads) {
    int rc = ORC_OK;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
#endif
    for (int32_t i = 0; i < n; ++i) {
        int r = orc_pisp(g, src[i], alpha, eps, beta ? beta + (size_t)i * (size_t)g->nu : NULL, NULL, NULL,
                         st ? st + i : NULL);
        if (r != ORC_OK) rc = r;
    }
    (void)nthreads;
    return rc;
}

/* ---------------------------------------------------------------------------
 * MCSP, the other baseline of Sec. 3.3 (Baselines and Challenges): pi(u, .)
 * by MonteCarlo, random walks with restart whose steps draw neighbours from
 * Walker alias tables (the structures Sec. 3.3 names), with eps_f = eps/2 and
 * n_r = 2 (1 + eps_f/3) ln(|U|/p_f) / eps_f^2 walks (the count behind Eq. (mc),
 * rounded up); plus pi(., u) by SelectivePush (Algorithm 2) with
 * eps_b = eps/2; beta' = pi_f + pi_b.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011), a
 * counter-based generator, so that any implementation of its definition draws
 * the same walks. Walk w from source u takes, at step s, the eight 32-bit
 * numbers of the counters (w, u, 2s, TAG) and (w, u, 2s + 1, TAG) under the
 * key (seed low, seed high): r0 decides the stop (stop iff r0 < alpha 2^32),
 * r1, r2 draw the U->V step and r3, r4 the V->U step (slot = (r d) >> 32 of a
 * row with d entries; keep the slot iff r' 2^-32 < prob[slot], else take its
 * alias).
 * ------------------------------------------------------------------------- */
#define ORC_MC_TAG 0x4D435350u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }     /* key schedule (Weyl sequence) */
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Vose's construction of Walker's alias table for each row of a CSR: row r
 * with d entries of weights w and sum ws gets prob[e] and alias[e] (a slot of
 * the same row) with, for every slot j,
 *   (prob[j] + sum over slots i with alias[i] = j of (1 - prob[i])) / d = w_j / ws. */
static int alias_rows(int32_t n, const int64_t* rp, const double* w, const double* ws, double* prob, int32_t* alias) {
    int64_t maxd = 0;
    for (int32_t r = 0; r < n; ++r) if (rp[r + 1] - rp[r] > maxd) maxd = rp[r + 1] - rp[r];
    double* q = (double*)malloc(sizeof(double) * (size_t)(maxd > 0 ? maxd : 1));
    int32_t* sm = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxd > 0 ? maxd : 1));
    int32_t* lg = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxd > 0 ? maxd : 1));
    if (!q || !sm || !lg) { free(q); free(sm); free(lg); return ORC_ENOMEM; }
    for (int32_t r = 0; r < n; ++r) {
        const int64_t b = rp[r];
        const int32_t d = (int32_t)(rp[r + 1] - b);
        if (d == 0) continue;
        int32_t ns = 0, nl = 0;
        for (int32_t j = 0; j < d; ++j) {
            q[j] = w[b + j] * (double)d / ws[r];
            if (q[j] < 1.0) sm[ns++] = j; else lg[nl++] = j;
        }
        while (ns > 0 && nl > 0) {
            const int32_t a = sm[--ns], l = lg[--nl];
            prob[b + a] = q[a];
            alias[b + a] = l;
            q[l] = (q[l] + q[a]) - 1.0;
            if (q[l] < 1.0) sm[ns++] = l; else lg[nl++] = l;
        }
        while (nl > 0) { const int32_t l = lg[--nl]; prob[b + l] = 1.0; alias[b + l] = l; }
        while (ns > 0) { const int32_t a = sm[--ns]; prob[b + a] = 1.0; alias[b + a] = a; }
    }
    free(q); free(sm); free(lg);
    return ORC_OK;
}

/* side 0: rows of U (entries as in rp_u/ci_u), side 1: rows of V */
int orc_alias_tables(const orc_graph* g, int32_t side, double* prob, int32_t* alias) {
    return side == 0 ? alias_rows(g->nu, g->rp_u, g->w_u, g->ws_u, prob, alias)
                     : alias_rows(g->nv, g->rp_v, g->w_v, g->ws_v, prob, alias);
}

/* Walks of MonteCarlo: n_r = 2 (1 + eps_f/3) ln(|U|/p_f) / eps_f^2, rounded up. */
int64_t orc_mc_walks(int32_t nu, double eps_f, double p_f) {
    return (int64_t)ceil(2.0 * (1.0 + eps_f / 3.0) * log((double)nu / p_f) / (eps_f * eps_f));
}

static int32_t alias_draw_row(const int64_t* rp, const int32_t* ci, const double* prob, const int32_t* alias,
                              int32_t r, uint32_t rs, uint32_t rc) {
    const int64_t b = rp[r];
    const uint64_t d = (uint64_t)(rp[r + 1] - b);
    const int64_t slot = (int64_t)(((uint64_t)rs * d) >> 32);
    const int64_t pick = (double)rc * 0x1.0p-32 < prob[b + slot] ? slot : (int64_t)alias[b + slot];
    return ci[b + pick];
}

/* counts[x] = number of the n_r walks from u that end at x (walks numbered 0..n_r-1) */
int orc_mc_counts(const orc_graph* g, int32_t u, double alpha, int64_t n_r, uint64_t seed, int64_t* counts,
                  double* steps_out) {
    if (u < 0 || u >= g->nu) return ORC_ERANGE;
    if (g->ws_u[u] == 0.0) return ORC_EISOLATED;
    if (n_r > 0xFFFFFFFFll) return ORC_EINVAL;
    double* pu = (double*)malloc(sizeof(double) * (size_t)(g->ne > 0 ? g->ne : 1));
    double* pv = (double*)malloc(sizeof(double) * (size_t)(g->ne > 0 ? g->ne : 1));
    int32_t* au = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->ne > 0 ? g->ne : 1));
    int32_t* av = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->ne > 0 ? g->ne : 1));
    if (!pu || !pv || !au || !av) { free(pu); free(pv); free(au); free(av); return ORC_ENOMEM; }
    if (orc_alias_tables(g, 0, pu, au) || orc_alias_tables(g, 1, pv, av)) {
        free(pu); free(pv); free(au); free(av); return ORC_ENOMEM;
    }
    for (int32_t x = 0; x < g->nu; ++x) counts[x] = 0;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const double stop_thr = alpha * 4294967296.0;
    double steps = 0.0;
    for (int64_t wk = 0; wk < n_r; ++wk) {
        int32_t x = u;
        for (uint32_t st = 0;; ++st) {
            uint32_t c[4] = {(uint32_t)wk, (uint32_t)u, 2u * st, ORC_MC_TAG}, a[4], b[4];
            orc_philox4x32_10(c, key, a);
            c[2] = 2u * st + 1u;
            orc_philox4x32_10(c, key, b);
            if ((double)a[0] < stop_thr) break;                                  /* the walk stops at x */
            const int32_t v = alias_draw_row(g->rp_u, g->ci_u, pu, au, x, a[1], a[2]);   /* U -> V */
            x = alias_draw_row(g->rp_v, g->ci_v, pv, av, v, a[3], b[0]);                 /* V -> U */
            steps += 1.0;
        }
        counts[x] += 1;
    }
    if (steps_out) *steps_out = steps;
    free(pu); free(pv); free(au); free(av);
    return ORC_OK;
}

/* MCSP: beta' = counts / n_r + pi_b (SelectivePush at eps/2); pi_b_out and
 * counts_out are optional. */
int orc_mcsp(const orc_graph* g, int32_t u, double alpha, double eps, double p_f, uint64_t seed, double* beta,
             int64_t* counts_out, double* pi_b_out, int64_t* n_r_out) {
    if (u < 0 || u >= g->nu) return ORC_ERANGE;
    if (!(alpha > 0.0 && alpha < 1.0) || !(eps > 0.0) || !(p_f > 0.0 && p_f < 1.0)) return ORC_EINVAL;
    if (g->ws_u[u] == 0.0) return ORC_EISOLATED;
    const int64_t n_r = orc_mc_walks(g->nu, 0.5 * eps, p_f);
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)g->nu);
    double* pib = (double*)malloc(sizeof(double) * (size_t)g->nu);
    if (!cnt || !pib) { free(cnt); free(pib); return ORC_ENOMEM; }
    int rc = orc_mc_counts(g, u, alpha, n_r, seed, cnt, NULL);
    int32_t it = 0;
    double np = 0.0;
    if (rc == ORC_OK) rc = selective_push(g, u, alpha, 0.5 * eps, pib, &it, &np);
    if (rc == ORC_OK) {
        for (int32_t x = 0; x < g->nu; ++x) {
            if (beta) beta[x] = (double)cnt[x] / (double)n_r + pib[x];
            if (counts_out) counts_out[x] = cnt[x];
            if (pi_b_out) pi_b_out[x] = pib[x];
        }
        if (n_r_out) *n_r_out = n_r;
    }
    free(cnt); free(pib);
    return rc;
}

/* A bounded sample of the CPU baseline: each source runs Algorithm 5 as
 * orc_approx_bhpp does, stopped after max_iters push iterations; work[i]
 * receives the edges its query touched. The rate of edge visits per second
 * scales the oracle's speed to whole queries. */
int orc_approx_bhpp_sample(const orc_graph* g, int32_t n, const int32_t* src, double alpha, double eps,
                           double eps_b, double lambda, int32_t max_iters, double* work, int32_t nthreads) {
    int rc = ORC_OK;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
#endif
    for (int32_t i = 0; i < n; ++i) {
        work[i] = 0.0;
        int r = approx_bhpp_core(g, src[i], alpha, eps, eps_b, lambda, NULL, NULL, NULL, NULL, NULL, NULL,
                                 max_iters, work + i);
        if (r != ORC_OK && r != ORC_ENOCONV) rc = r;
    }
    (void)nthreads;
    return rc;
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Eq. (t) rounded up and clamped at 0: the smallest integer t with
 * (1-alpha)^(t+1) * sum_rf <= eps_f, which is what the proof of Theorem 2 needs. */
int32_t orc_t(double sum_rf, double eps_f, double alpha) {
    double tr = ceil(log_base(alpha, sum_rf / eps_f) - 1.0);
    return tr > 0.0 ? (int32_t)tr : 0;
}
