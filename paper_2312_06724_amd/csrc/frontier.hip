// Sparse two-hop push step for one source: one iteration of Algorithm 2's
// loop body over an explicit frontier, for the selective phase of SS-Push
// (Algorithm 3) while its frontier is small. Same arithmetic as a dense
// sweep (forward coordinates, Lemma 3):
//   1. frontier: every x whose residue passes the push test; a wavefront
//      compacts its hits with a ballot and a prefix count (one atomic per
//      wavefront), and adds up their degrees;
//   2. take: ACC(x) += alpha y(x), S(x) = y(x)/ws(x), y(x) = 0 for x in F;
//   3. U->V scatter, edge-parallel over the frontier's edges (an inclusive
//      scan of their degrees, scan.h's three-launch tile scan, maps a thread
//      to its edge):
//      Q(v) += w(x,v) S(x) into a V vector kept zero between steps; the first
//      touch of v lists it and adds d(v) to n_p;
//   4. V->U: the dense U-side gather of the sweep kernels over Q (its zeros
//      cost reads only), then y += (1-alpha) G with the per-source reductions
//      of the dense update, and Q is cleared on the listed nodes.
// The U->V scatter uses atomic adds, so its summation order (not the result
// up to rounding) depends on timing.
#include <algorithm>

#include "common.h"
#include "scan.h"

namespace bhpp {

namespace {

template <typename VT>
__global__ __launch_bounds__(256) void k_frontier(const VT* __restrict__ Y, const VT* __restrict__ inv_ws,
                                                  const int32_t* __restrict__ deg, int32_t nu, const ColState* st,
                                                  int32_t* F, unsigned long long* cnt) {
    const ColState& cs = st[0];
    const PushTest<VT> test(cs.ruleA, (VT)cs.k_ss, (VT)cs.k_pi);
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = wave0; base < nu; base += stride) {   // uniform per wavefront
        const int64_t x = base + lane;
        bool pred = false;
        int32_t d = 0;
        if (x < nu) {
            d = deg[x];
            const VT y = Y[x];
            pred = d > 0 && test(fabs(y), fabs(y * inv_ws[x]));
        }
        const uint64_t m = __ballot(pred);
        if (m == 0) continue;
        unsigned long long dsum = pred ? (unsigned long long)d : 0ull;
        for (int o = 32; o > 0; o >>= 1) dsum += __shfl_xor(dsum, o);
        unsigned long long at = 0;
        if (lane == 0) {
            at = atomicAdd(&cnt[0], (unsigned long long)__popcll(m));
            atomicAdd(&cnt[2], dsum);
        }
        at = __shfl(at, 0);
        if (pred) F[at + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)x;
    }
}

template <typename VT>
__global__ void k_take(const int32_t* F, int32_t nF, VT* Y, VT* ACC, const VT* inv_ws, const int32_t* deg,
                       const ColState* st, VT* S, int64_t* dF) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nF) return;
    const int32_t x = F[i];
    const VT y = Y[x];
    ACC[x] += (VT)st[0].alpha * y;
    Y[x] = VT(0);
    S[i] = y * inv_ws[x];
    dF[i] = deg[x];
}

__device__ inline int32_t upper_index(const int64_t* offs, int32_t n, int64_t t) {
    // first i with offs[i] > t (offs is an inclusive scan, offs[n-1] > t)
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (offs[mid] > t) hi = mid; else lo = mid + 1;
    }
    return lo;
}

template <typename VT, typename WT>
__global__ void k_scatter_u(const int32_t* F, const int64_t* offs, int32_t nF, int64_t total, const VT* S,
                            const int64_t* rp_u, const int32_t* ci_u, const WT* w_u, const VT* inv_ws_v,
                            const int64_t* rp_v, VT* Q, int32_t* mark, int32_t* TV, unsigned long long* cnt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const int32_t i = upper_index(offs, nF, t);
        const int64_t first = i > 0 ? offs[i - 1] : 0;
        const int64_t e = rp_u[F[i]] + (t - first);
        const int32_t v = ci_u[e];
        atomicAdd(&Q[v], (VT)w_u[e] / inv_ws_v[v] * S[i]);   // w_u holds w(x,v)/ws(v)
        if (mark[v] == 0 && atomicCAS(&mark[v], 0, 1) == 0) {
            TV[atomicAdd(&cnt[1], 1ull)] = v;
            atomicAdd(&cnt[3], (unsigned long long)(rp_v[v + 1] - rp_v[v]));
        }
    }
}

template <typename VT>
__global__ void k_clear_v(const int32_t* TV, const unsigned long long* cnt, VT* Q, int32_t* mark) {
    const int64_t n = (int64_t)cnt[1];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        Q[TV[j]] = VT(0);
        mark[TV[j]] = 0;
    }
}

// y += (1-alpha) G over all of U, then the reductions k_update makes after a
// dense sweep, into the update slots [off_u, off_u + gridDim.x); n_p goes
// where a dense sweep puts it: the edges of F (U side) to slot off_u, the
// edges of the touched V nodes (V side) to slot 0 of the gather slots
// [0, off_u), whose other slots are zeroed.
template <typename VT>
__global__ __launch_bounds__(256) void k_sparse_finish(VT* Y, const VT* G, const VT* inv_ws, const int32_t* deg,
                                                       int32_t nu, const ColState* st, double* red, int n_part,
                                                       int off_u, const unsigned long long* cnt) {
    __shared__ double sh[4][256];
    const ColState& cs = st[0];
    const VT kss = (VT)cs.k_ss, kpi = (VT)cs.k_pi, oma = VT(1) - (VT)cs.alpha;
    double r[4] = {0, 0, 0, 0};
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < nu; x += (int64_t)gridDim.x * blockDim.x) {
        if (deg[x] == 0) continue;
        const VT y = Y[x] + oma * G[x];
        Y[x] = y;
        const VT tn = fabs(y * inv_ws[x]), ya = fabs(y);
        r[0] += (tn > kss) ? 1.0 : 0.0;
        r[1] += (double)tn;
        r[2] += (ya > kpi) ? 1.0 : 0.0;
        r[3] += (double)ya;
    }
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = r[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int slot = off_u + blockIdx.x;
        red[(size_t)RED_NP * n_part + slot] = blockIdx.x == 0 ? (double)cnt[2] : 0.0;
        red[(size_t)RED_CNT_SS * n_part + slot] = sh[0][0];
        red[(size_t)RED_SUM_R * n_part + slot] = sh[1][0];
        red[(size_t)RED_CNT_PI * n_part + slot] = sh[2][0];
        red[(size_t)RED_SUM_Y * n_part + slot] = sh[3][0];
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < off_u; i += gridDim.x * blockDim.x)
        red[(size_t)RED_NP * n_part + i] = i == 0 ? (double)cnt[3] : 0.0;
}

unsigned grid_of(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 4096); }

template <typename VT, typename WT>
bhpp_status sparse_front_impl(Graph* g, Workspace& w, SparseStep& io, hipStream_t s) {
    const int32_t nu = g->nu;
    const VT* inv_ws = reinterpret_cast<const VT*>(sizeof(VT) == 8 ? (const void*)g->inv_ws_u_d
                                                                    : (const void*)g->inv_ws_u_f);
    const VT* inv_ws_v = reinterpret_cast<const VT*>(sizeof(VT) == 8 ? (const void*)g->inv_ws_v_d
                                                                      : (const void*)g->inv_ws_v_f);
    VT* Y = reinterpret_cast<VT*>(w.Y);
    VT* ACC = reinterpret_cast<VT*>(w.ACC);
    VT* S = reinterpret_cast<VT*>(w.fS);
    BHPP_HIP(hipMemsetAsync(w.fCnt, 0, 4 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_frontier<VT>, dim3(grid_of(nu)), dim3(256), 0, s, Y, inv_ws, g->deg_u, nu, w.st, w.fF,
                       (unsigned long long*)w.fCnt);
    BHPP_HIP(hipMemcpyAsync(w.h_fCnt, w.fCnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    BHPP_HIP(hipStreamSynchronize(s));
    const int32_t nF = (int32_t)w.h_fCnt[0];
    const int64_t workF = (int64_t)w.h_fCnt[2];
    io.frontier = nF;
    io.work_u = workF;
    io.done = workF <= io.max_work;   // else too much work for a sparse step: the caller sweeps densely
    if (!io.done || nF == 0) return BHPP_OK;
    hipLaunchKernelGGL(k_take<VT>, dim3(grid_of(nF)), dim3(256), 0, s, w.fF, nF, Y, ACC, inv_ws, g->deg_u, w.st, S,
                       w.fDeg);
    BHPP_HIP((scan_many<int64_t, int64_t, false>(w.fDeg, w.fOffs, nF, (int64_t*)w.fScanTmp, s)));
    hipLaunchKernelGGL((k_scatter_u<VT, WT>), dim3(grid_of(workF)), dim3(256), 0, s, w.fF, w.fOffs, nF, workF, S,
                       g->rp_u, g->ci_u, reinterpret_cast<const WT*>(g->w_u), inv_ws_v, g->rp_v,
                       reinterpret_cast<VT*>(w.fQ), w.fMark, w.fTV, (unsigned long long*)w.fCnt);
    BHPP_HIP(hipGetLastError());
    return BHPP_OK;
}

template <typename VT>
bhpp_status sparse_finish_impl(Graph* g, Workspace& w, const SparseStep& io, const void* G, hipStream_t s) {
    const VT* inv_ws = reinterpret_cast<const VT*>(sizeof(VT) == 8 ? (const void*)g->inv_ws_u_d
                                                                    : (const void*)g->inv_ws_u_f);
    hipLaunchKernelGGL(k_sparse_finish<VT>, dim3(io.red_blocks), dim3(256), 0, s, reinterpret_cast<VT*>(w.Y),
                       reinterpret_cast<const VT*>(G), inv_ws, g->deg_u, g->nu, w.st, w.red, io.n_part, io.off_u,
                       (const unsigned long long*)w.fCnt);
    hipLaunchKernelGGL(k_clear_v<VT>, dim3(256), dim3(256), 0, s, w.fTV, (const unsigned long long*)w.fCnt,
                       reinterpret_cast<VT*>(w.fQ), w.fMark);
    BHPP_HIP(hipGetLastError());
    return BHPP_OK;
}

}  // namespace

bhpp_status ensure_sparse(Graph* g, Workspace& w, hipStream_t s) {
    if (w.fF) return BHPP_OK;
    const size_t nu = (size_t)g->nu, nv = (size_t)g->nv, e = (size_t)g->elem, nm = std::max(nu, nv);
    const size_t tb = (size_t)scan_tiles((int64_t)nm) * 8;
    auto A = [&](void** p, size_t bytes) { return hipMalloc(p, bytes ? bytes : 256) == hipSuccess; };
    const bool ok = A((void**)&w.fF, nu * 4) && A(&w.fS, nu * e) && A((void**)&w.fDeg, nm * 8) &&
                    A((void**)&w.fOffs, nm * 8) && A((void**)&w.fTV, nv * 4) && A(&w.fQ, nv * e) &&
                    A((void**)&w.fMark, nv * 4) && A((void**)&w.fCnt, 64) && A(&w.fScanTmp, tb) &&
                    hipHostMalloc((void**)&w.h_fCnt, 64) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return BHPP_OUT_OF_MEMORY;
    }
    w.fScanBytes = tb;
    BHPP_HIP(hipMemsetAsync(w.fQ, 0, nv * e, s));
    BHPP_HIP(hipMemsetAsync(w.fMark, 0, nv * 4, s));
    return BHPP_OK;
}

bhpp_status sparse_front(Graph* g, Workspace& w, SparseStep& io, hipStream_t s) {
    if (g->dtype == BHPP_DTYPE_F64) return sparse_front_impl<double, double>(g, w, io, s);
    return sparse_front_impl<float, float>(g, w, io, s);
}

bhpp_status sparse_finish(Graph* g, Workspace& w, const SparseStep& io, const void* G, hipStream_t s) {
    if (g->dtype == BHPP_DTYPE_F64) return sparse_finish_impl<double>(g, w, io, G, s);
    return sparse_finish_impl<float>(g, w, io, G, s);
}

}  // namespace bhpp
