// MCSP, the baseline of Sec. 3.3 (Baselines and Challenges) built from
// MonteCarlo and SelectivePush: pi(u, .) from random walks with restart over
// the bipartite graph (eps_f = eps/2, n_r walks from the count behind
// Eq. (mc)), pi(., u) from SelectivePush with eps_b = eps/2 (the sweep
// kernels' control mode 4), beta' = counts / n_r + pi_b.
//
// Walk steps draw neighbours from Walker alias tables, one per row of W and
// of W^T in caller ids, built at graph build time (BHPP_BUILD_MCSP) by Vose's
// construction in FP64 from the merged weights, one thread per row.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011), a
// counter-based generator: walk w from source u takes at step s the numbers
// of the counters (w, u, 2s, TAG) and (w, u, 2s + 1, TAG) under the key
// (seed low, seed high). r0 decides the stop (r0 < alpha 2^32), (r1, r2) the
// U->V step and (r3, r4) the V->U step: slot = (r d) >> 32 in a row of d
// entries, kept iff r' 2^-32 < prob[slot], else its alias. Every quantity the
// walk compares is exact, so a walk depends only on its counter, the key and
// the tables.
#include <cmath>
#include <vector>

#include "common.h"

namespace bhpp {

namespace {

constexpr uint32_t kMcTag = 0x4D435350u;

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;   // key schedule: the Weyl sequence of the definition
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Vose's construction for each row, one thread per row (rows of hubs are long,
// but the tables are built once per graph). q, small and large are scratch
// arrays of one entry per adjacency entry, used at the row's own offsets.
// keep[e] is the neighbour at slot e, alias_to[e] the neighbour of its alias.
__global__ void k_alias_rows(int32_t n_rows, const int64_t* rp, const int32_t* ci, const double* w, const double* ws,
                             double* q, int32_t* sm, int32_t* lg, double* prob, int32_t* keep, int32_t* alias_to) {
#pragma clang fp contract(off)
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int64_t b = rp[r];
    const int32_t d = (int32_t)(rp[r + 1] - b);
    if (d == 0) return;
    double* qr = q + b;
    int32_t* S = sm + b;
    int32_t* L = lg + b;
    int32_t ns = 0, nl = 0;
    const double wsr = ws[r];
    for (int32_t j = 0; j < d; ++j) {
        const double v = w[b + j] * (double)d / wsr;
        qr[j] = v;
        if (v < 1.0) S[ns++] = j; else L[nl++] = j;
    }
    while (ns > 0 && nl > 0) {
        const int32_t a = S[--ns], l = L[--nl];
        prob[b + a] = qr[a];
        alias_to[b + a] = ci[b + l];
        qr[l] = (qr[l] + qr[a]) - 1.0;
        if (qr[l] < 1.0) S[ns++] = l; else L[nl++] = l;
    }
    while (nl > 0) {
        const int32_t l = L[--nl];
        prob[b + l] = 1.0;
        alias_to[b + l] = ci[b + l];
    }
    while (ns > 0) {
        const int32_t a = S[--ns];
        prob[b + a] = 1.0;
        alias_to[b + a] = ci[b + a];
    }
    for (int32_t j = 0; j < d; ++j) keep[b + j] = ci[b + j];
}

__device__ __forceinline__ int32_t draw(const int64_t* rp, const double* prob, const int32_t* keep,
                                        const int32_t* alias_to, int32_t row, uint32_t rs, uint32_t rc) {
    const int64_t b = rp[row];
    const uint64_t d = (uint64_t)(rp[row + 1] - b);
    const int64_t e = b + (int64_t)(((uint64_t)rs * d) >> 32);
    return (double)rc * 0x1.0p-32 < prob[e] ? keep[e] : alias_to[e];
}

struct McTables {
    const int64_t *rp_u, *rp_v;
    const double *prob_u, *prob_v;
    const int32_t *keep_u, *keep_v, *alias_u, *alias_v;
};

// Walks 0..n_r-1 of every source (blockIdx.y), grid-stride; counts[i][x] +=
// 1 for the node where walk ends. Walks are geometric in length (mean
// (1-alpha)/alpha steps); a walk that reached 2^31 steps would wrap its step
// counter, which has probability (1-alpha)^(2^31), so no cap is needed for
// alpha in (0, 1) at double precision.
__global__ __launch_bounds__(256) void k_mc_walks(McTables t, const int32_t* src, int64_t n_r, double stop_thr,
                                                  uint32_t k0, uint32_t k1, uint32_t* counts, int32_t n_u) {
    const int32_t i = blockIdx.y;
    const int32_t u = src[i];
    uint32_t* cnt = counts + (size_t)i * n_u;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < n_r; w += (int64_t)gridDim.x * blockDim.x) {
        int32_t x = u;
        for (uint32_t st = 0;; ++st) {
            uint32_t a[4], b[4];
            philox4x32_10((uint32_t)w, (uint32_t)u, 2u * st, kMcTag, k0, k1, a);
            philox4x32_10((uint32_t)w, (uint32_t)u, 2u * st + 1u, kMcTag, k0, k1, b);
            if ((double)a[0] < stop_thr) break;
            const int32_t v = draw(t.rp_u, t.prob_u, t.keep_u, t.alias_u, x, a[1], a[2]);
            x = draw(t.rp_v, t.prob_v, t.keep_v, t.alias_v, v, a[3], b[0]);
        }
        atomicAdd(&cnt[x], 1u);
    }
}

// rows[i][x] = counts[i][x] / n_r + rows[i][x] (caller ids), in FP64 then rounded once
template <typename VT>
__global__ void k_mc_combine(VT* rows, const uint32_t* counts, int64_t total, double nr) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        rows[i] = (VT)((double)counts[i] / nr + (double)rows[i]);
}

}  // namespace

int64_t mc_walk_count(int32_t nu, double eps_f, double p_f) {
    return (int64_t)ceil(2.0 * (1.0 + eps_f / 3.0) * log((double)nu / p_f) / (eps_f * eps_f));
}

bhpp_status mcsp_build_tables(Graph* g, const int64_t* xrp_u, const int32_t* xci_u, const double* xw_u,
                              const double* ws_u, const int64_t* xrp_v, const int32_t* xci_v, const double* xw_v,
                              const double* ws_v, hipStream_t s) {
    const size_t m = (size_t)std::max<int64_t>(g->ne, 1);
    const size_t nu = (size_t)g->nu, nv = (size_t)g->nv;
    double* q = nullptr;
    int32_t *sm = nullptr, *lg = nullptr;
    bool ok = hipMalloc((void**)&g->mc_rp_u, 8 * (nu + 1)) == hipSuccess &&
              hipMalloc((void**)&g->mc_rp_v, 8 * (nv + 1)) == hipSuccess &&
              hipMalloc((void**)&g->mc_prob_u, 8 * m) == hipSuccess &&
              hipMalloc((void**)&g->mc_prob_v, 8 * m) == hipSuccess &&
              hipMalloc((void**)&g->mc_keep_u, 4 * m) == hipSuccess &&
              hipMalloc((void**)&g->mc_keep_v, 4 * m) == hipSuccess &&
              hipMalloc((void**)&g->mc_alias_u, 4 * m) == hipSuccess &&
              hipMalloc((void**)&g->mc_alias_v, 4 * m) == hipSuccess &&
              hipMalloc((void**)&q, 8 * m) == hipSuccess && hipMalloc((void**)&sm, 4 * m) == hipSuccess &&
              hipMalloc((void**)&lg, 4 * m) == hipSuccess;
    bhpp_status rc = ok ? BHPP_OK : BHPP_OUT_OF_MEMORY;
    if (ok) {
        if (hipMemcpyAsync(g->mc_rp_u, xrp_u, 8 * (nu + 1), hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(g->mc_rp_v, xrp_v, 8 * (nv + 1), hipMemcpyDeviceToDevice, s) != hipSuccess)
            rc = BHPP_DEVICE_ERROR;
        hipLaunchKernelGGL(k_alias_rows, dim3((unsigned)((nu + 255) / 256)), dim3(256), 0, s, g->nu, xrp_u, xci_u,
                           xw_u, ws_u, q, sm, lg, g->mc_prob_u, g->mc_keep_u, g->mc_alias_u);
        hipLaunchKernelGGL(k_alias_rows, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, g->nv, xrp_v, xci_v,
                           xw_v, ws_v, q, sm, lg, g->mc_prob_v, g->mc_keep_v, g->mc_alias_v);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) rc = BHPP_DEVICE_ERROR;
    } else {
        (void)hipGetLastError();
    }
    hipFree(q);
    hipFree(sm);
    hipFree(lg);
    return rc;
}

bhpp_status mcsp_counts(Graph* g, int32_t n, const int32_t* src_ext, double alpha, int64_t n_r, uint64_t seed,
                        uint32_t* counts, hipStream_t s) {
    if (!g->mc_prob_u) return BHPP_NOT_SUPPORTED;
    McTables t{g->mc_rp_u, g->mc_rp_v, g->mc_prob_u, g->mc_prob_v, g->mc_keep_u, g->mc_keep_v, g->mc_alias_u,
               g->mc_alias_v};
    int32_t* d_src = nullptr;
    if (hipMalloc((void**)&d_src, 4 * (size_t)n) != hipSuccess) {
        (void)hipGetLastError();
        return BHPP_OUT_OF_MEMORY;
    }
    bhpp_status rc = BHPP_OK;
    if (hipMemcpyAsync(d_src, src_ext, 4 * (size_t)n, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(counts, 0, 4 * (size_t)n * g->nu, s) != hipSuccess)
        rc = BHPP_DEVICE_ERROR;
    if (rc == BHPP_OK) {
        const int64_t blocks = std::min<int64_t>((n_r + 255) / 256, 4096);
        hipLaunchKernelGGL(k_mc_walks, dim3((unsigned)std::max<int64_t>(blocks, 1), (unsigned)n), dim3(256), 0, s, t,
                           d_src, n_r, alpha * 4294967296.0, (uint32_t)seed, (uint32_t)(seed >> 32), counts, g->nu);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) rc = BHPP_DEVICE_ERROR;
    }
    hipFree(d_src);
    return rc;
}

bhpp_status mcsp_combine(Graph* g, void* rows, const uint32_t* counts, int32_t n, int64_t n_r, hipStream_t s) {
    const int64_t total = (int64_t)n * g->nu;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
    if (g->dtype == BHPP_DTYPE_F64)
        hipLaunchKernelGGL(k_mc_combine<double>, dim3(std::max(blocks, 1u)), dim3(256), 0, s, (double*)rows, counts,
                           total, (double)n_r);
    else
        hipLaunchKernelGGL(k_mc_combine<float>, dim3(std::max(blocks, 1u)), dim3(256), 0, s, (float*)rows, counts,
                           total, (double)n_r);
    return hipGetLastError() == hipSuccess ? BHPP_OK : BHPP_DEVICE_ERROR;
}

}  // namespace bhpp
