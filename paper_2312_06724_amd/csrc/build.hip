// Graph build and preprocessing (Sec. 3.1; Lemma 4; Eq. (epsilon-b)).
//
// From an unsorted device edge list the build produces, on the device:
//  1. the external-id adjacency of W sorted by (u, v) and of W^T sorted by
//     (v, u), duplicates merged by an FP64 sum in input order;
//  2. ws(u), ws(v) of Eq. (d), each an FP64 sum along its sorted row, rounded
//     once to the graph dtype (the same sum a plain CPU loop computes);
//  3. an internal numbering of U and of V by decreasing degree (ties by id),
//     so hub rows come first, rows of similar degree share work tiles, and
//     the heavily reused hub entries of the dense vectors sit together;
//  4. the internal adjacency in both directions, 1/ws vectors, work tiles;
//  5. lambda (Lemma 4) by PowerIteration from the all-ones vector and
//     eps_b / eps (Eq. (epsilon-b)).
// Sorting is a stable LSD radix sort on 8-bit digits written below (tile
// histograms, one prefix sum over them, a stable scatter); prefix sums use
// scan.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "common.h"
#include "scan.h"

namespace bhpp {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <typename WT>
__global__ void k_validate(int64_t n, const int32_t* eu, const int32_t* ev, const WT* ew, int32_t nu, int32_t nv,
                           int32_t* flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int f = 0;
    for (; i < n; i += stride) {
        if (eu[i] < 0 || eu[i] >= nu || ev[i] < 0 || ev[i] >= nv) f |= 1;
        const double w = (double)ew[i];
        if (!(w > 0.0) || !isfinite(w)) f |= 2;
    }
    if (f) atomicOr(flags, f);
}

__global__ void k_keys_pair(int64_t n, const int32_t* a, const int32_t* b, int64_t nb, uint64_t* keys,
                            int32_t* idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        keys[i] = (uint64_t)a[i] * (uint64_t)nb + (uint64_t)b[i];
        idx[i] = (int32_t)i;
    }
}

__global__ void k_heads(int64_t n, const uint64_t* keys, int32_t* head) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// One thread per run of equal keys: merged weight = FP64 sum in input order
// (the stable sort kept input order inside a run).
template <typename WT>
__global__ void k_merge(int64_t n, const uint64_t* keys, const int32_t* idx, const int32_t* head, const int32_t* pos,
                        const WT* ew, int64_t nv, int32_t* u_of, int32_t* v_of, double* w_of) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !head[i]) return;
    double s = 0.0;
    int64_t j = i;
    do {
        s += (double)ew[idx[j]];
        ++j;
    } while (j < n && !head[j]);
    const int32_t d = pos[i];
    u_of[d] = (int32_t)(keys[i] / (uint64_t)nv);
    v_of[d] = (int32_t)(keys[i] % (uint64_t)nv);
    w_of[d] = s;
}

// rp[x] = first position p with rows[p] >= x, for x in [0, n_rows]
__global__ void k_row_ptr(int32_t n_rows, int64_t m, const int32_t* rows, int64_t* rp) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x > n_rows) return;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (rows[mid] < x) lo = mid + 1; else hi = mid;
    }
    rp[x] = lo;
}

// Eq. (d): sequential FP64 sum along each sorted row
__global__ void k_row_sums(int32_t n_rows, const int64_t* rp, const double* w, double* ws) {
    int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n_rows) return;
    double s = 0.0;
    for (int64_t p = rp[x]; p < rp[x + 1]; ++p) s += w[p];
    ws[x] = s;
}

// gather by permutation: out[i] = in[order[i]] (optionally mapped through a table)
__global__ void k_gather_i32(int64_t n, const int32_t* order, const int32_t* in, const int32_t* map, int32_t* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int32_t v = in[order[i]];
        out[i] = map ? map[v] : v;
    }
}
// out[i] = map[in[i]]
__global__ void k_map_i32(int64_t n, const int32_t* in, const int32_t* map, int32_t* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = map[in[i]];
}
__global__ void k_gather_f64(int64_t n, const int32_t* order, const double* in, double* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[order[i]];
}
// U rows store w(x,v)/ws(v): the U-side gather then needs no per-row scaling
template <typename WT>
__global__ void k_scale_by_col(int64_t n, const double* w, const int32_t* col, const int32_t* iperm_col,
                               const double* ws_col_ext, WT* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (WT)(w[i] / ws_col_ext[iperm_col[col[i]]]);
}
template <typename WT>
__global__ void k_cast(int64_t n, const double* in, WT* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (WT)in[i];
}
__global__ void k_rows_from_keys(int64_t n, const uint64_t* keys, int64_t div, int32_t* rows) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rows[i] = (int32_t)(keys[i] / (uint64_t)div);
}

// key = (INT32_MAX - degree) << 32 | id : ascending key = descending degree, then id
__global__ void k_degree_keys(int32_t n, const int64_t* rp, int reorder, uint64_t* keys) {
    int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const uint64_t d = (uint64_t)(rp[x + 1] - rp[x]);
    keys[x] = reorder ? (((uint64_t)0x7FFFFFFF - d) << 32) | (uint64_t)x : (uint64_t)x;
}
// out[i] = vals[idx[i]]
template <typename T>
__global__ void k_take(int64_t n, const int32_t* idx, const T* vals, T* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = vals[idx[i]];
}

__global__ void k_perm_from_keys(int32_t n, const uint64_t* keys, int32_t* iperm, int32_t* perm) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t x = (int32_t)(keys[i] & 0xFFFFFFFFull);
    iperm[i] = x;
    perm[x] = i;
}
// bit e of bits is set iff adjacency entry e is the last entry of its row
__global__ void k_end_bits(int32_t n, const int64_t* rp, unsigned long long* bits) {
    int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n || rp[x + 1] == rp[x]) return;
    const int64_t e = rp[x + 1] - 1;
    atomicOr(&bits[e >> 6], 1ull << (e & 63));
}
__global__ void k_degrees(int32_t n, const int64_t* rp, int32_t* deg) {
    int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) deg[x] = (int32_t)(rp[x + 1] - rp[x]);
}
// inverse weighted degree in internal order; 0 for isolated nodes
template <typename VT>
__global__ void k_inv_ws(int32_t n, const int32_t* iperm, const double* ws_ext, VT* out) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double w = ws_ext[iperm[i]];
    out[i] = w > 0.0 ? (VT)(1.0 / w) : VT(0);
}

static inline dim3 grid_for(int64_t n, int t = 256) { return dim3((unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1)); }

static int bits_for(uint64_t maxval) {
    int b = 1;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b;
}

// ---------------------------------------------------------------------------
// work tiles (host): rows grouped so each tile covers about kTileEdges
// adjacency entries; rows longer than that are split into pieces.
// ---------------------------------------------------------------------------
bhpp_status build_tiles(const std::vector<int64_t>& rp, int32_t n_rows, int tile_edges, TileSet* ts, int max_rows) {
    std::vector<Tile> tiles;
    std::vector<SplitRow> split;
    int32_t slot = 0;
    int32_t end = n_rows;
    while (end > 0 && rp[end] == rp[end - 1]) --end;   // isolated suffix (degree order) needs no work
    int32_t row = 0;
    const int64_t T = tile_edges;
    auto log2ceil = [](int64_t d) {
        int l = 0;
        while ((1LL << l) < d && l < 6) ++l;
        return l;
    };
    while (row < end) {
        const int64_t d = rp[row + 1] - rp[row];
        if (d == 0) {   // rows without edges need no work and stay out of every tile
            ++row;
            continue;
        }
        if (d > T) {
            SplitRow s{row, slot, 0, 0};
            for (int64_t e0 = rp[row]; e0 < rp[row + 1]; e0 += T) {
                const int64_t e1 = std::min(e0 + T, rp[row + 1]);
                tiles.push_back(Tile{row, row + 1, e0, e1, slot++, 6});
            }
            s.slot_end = slot;
            split.push_back(s);
            ++row;
            continue;
        }
        const int32_t start = row;
        int64_t edges = 0, maxd = 0;
        while (row < end) {
            const int64_t dd = rp[row + 1] - rp[row];
            if (dd == 0 || dd > T) break;
            if (row > start && (edges + dd > T || row - start >= max_rows)) break;
            edges += dd;
            maxd = std::max(maxd, dd);
            ++row;
        }
        tiles.push_back(Tile{start, row, rp[start], rp[row], -1, log2ceil(std::max<int64_t>(1, maxd))});
    }
    ts->n_tiles = (int32_t)tiles.size();
    ts->n_split = (int32_t)split.size();
    ts->n_slots = slot;
    if (hipMalloc((void**)&ts->tiles, sizeof(Tile) * std::max<size_t>(1, tiles.size())) != hipSuccess ||
        hipMalloc((void**)&ts->split, sizeof(SplitRow) * std::max<size_t>(1, split.size())) != hipSuccess)
        return BHPP_OUT_OF_MEMORY;
    if (!tiles.empty() && hipMemcpy(ts->tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice) != hipSuccess)
        return BHPP_DEVICE_ERROR;
    if (!split.empty() && hipMemcpy(ts->split, split.data(), sizeof(SplitRow) * split.size(), hipMemcpyHostToDevice) != hipSuccess)
        return BHPP_DEVICE_ERROR;
    return BHPP_OK;
}

void free_tiles(TileSet* ts) {
    hipFree(ts->tiles);
    hipFree(ts->split);
    *ts = TileSet{};
}

void free_graph(Graph* g) {
    if (!g) return;
    void* ptrs[] = {g->rp_u, g->ci_u, g->w_u, g->rp_v, g->ci_v, g->w_v, g->iw_v, g->inv_ws_u_f, g->inv_ws_v_f, g->deg_u, g->end_bits_u, g->end_bits_v,
                    g->mc_rp_u, g->mc_rp_v, g->mc_prob_u, g->mc_prob_v, g->mc_keep_u, g->mc_keep_v, g->mc_alias_u,
                    g->mc_alias_v,
                    g->inv_ws_u_d, g->inv_ws_v_d, g->perm_u, g->iperm_u, g->iperm_v, g->x_rp_u, g->x_ci_u, g->x_w_u,
                    g->x_rp_v, g->x_ci_v, g->x_w_v, g->x_ws_u, g->x_ws_v};
    for (void* p : ptrs) hipFree(p);
    free_tiles(&g->tiles_u);
    free_tiles(&g->tiles_v);
    free_tiles(&g->tiles_uf);
    free_workspace(g->ws);
    for (hipEvent_t e : g->prof_ev) hipEventDestroy(e);
    if (g->work) hipStreamDestroy(g->work);
    delete g;
}

// ---------------------------------------------------------------------------
// the build
// ---------------------------------------------------------------------------
namespace {

// Scoped device allocations for the build's temporaries.
struct Tmp {
    std::vector<void*> ptrs;
    bool ok = true;
    template <typename T>
    T* get(size_t n) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
            ok = false;
            return nullptr;
        }
        ptrs.push_back(p);
        return (T*)p;
    }
    ~Tmp() {
        for (void* p : ptrs) hipFree(p);
    }
};

// Stable LSD radix sort, one launch pair per 8-bit digit. The keys are cut
// into tiles of kRsTile consecutive entries, one workgroup each:
//   k_rs_hist: the tile's digit counts, stored digit-major (digit d of tile t
//     at d * n_tiles + t), so one exclusive prefix sum over them gives every
//     (digit, tile) its first output position;
//   k_rs_scatter: the tile's keys in input order, 256 at a time; a key's rank
//     among equal digits of its wavefront comes from eight ballots, the counts
//     of the earlier wavefronts and rounds from LDS, so equal digits keep
//     their input order.
constexpr int kRsItems = 16;
constexpr int kRsTile = 256 * kRsItems;

__global__ __launch_bounds__(256) void k_rs_hist(const uint64_t* keys, int64_t n, int shift, int32_t n_tiles,
                                                 int32_t* hist) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
        const int64_t i = base + (int64_t)r * 256 + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

template <bool PAIRS>
__global__ __launch_bounds__(256) void k_rs_scatter(const uint64_t* keys, const int32_t* vals, int64_t n, int shift,
                                                    int32_t n_tiles, const int32_t* offs, uint64_t* keys_out,
                                                    int32_t* vals_out) {
    __shared__ int32_t run[256];        // position of the next key with digit d in this tile's output range
    __shared__ int32_t wcnt[4][256];    // keys with digit d in wavefront w of the current round
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    run[t] = offs[(int64_t)t * n_tiles + blockIdx.x];
    for (int k = 0; k < 4; ++k) wcnt[k][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int r = 0; r < kRsItems; ++r) {
        const int64_t i = base + (int64_t)r * 256 + t;
        const bool ok = i < n;
        uint64_t key = 0;
        int32_t val = 0;
        if (ok) {
            key = keys[i];
            if (PAIRS) val = vals[i];
        }
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t same = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t on = __ballot((d >> b) & 1u);
            same &= ((d >> b) & 1u) ? on : ~on;
        }
        const int rank = __popcll(same & lt);
        if (ok && rank == 0) wcnt[wid][d] = __popcll(same);
        __syncthreads();
        if (ok) {
            int32_t pos = run[d] + rank;
            for (int k = 0; k < wid; ++k) pos += wcnt[k][d];
            keys_out[pos] = key;
            if (PAIRS) vals_out[pos] = val;
        }
        __syncthreads();
        run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
        for (int k = 0; k < 4; ++k) wcnt[k][t] = 0;
        __syncthreads();
    }
}

// Stable sort on the low `bits` bits; the result lands in keys_out (and
// idx_out); keys_in and idx_in serve as the other buffer of the passes and are
// overwritten.
static bool radix_sort(Tmp& tmp, uint64_t* keys_in, uint64_t* keys_out, int32_t* idx_in, int32_t* idx_out, int64_t n,
                       int bits, hipStream_t s) {
    if (n <= 0) return true;
    const int32_t n_tiles = (int32_t)((n + kRsTile - 1) / kRsTile);
    const int64_t nh = (int64_t)n_tiles * 256;
    int32_t* hist = tmp.get<int32_t>(nh);
    int32_t* ts = tmp.get<int32_t>(scan_tiles(nh));
    if (!tmp.ok) return false;
    const bool pairs = idx_in != nullptr;
    const int passes = std::max(1, (bits + 7) / 8);
    uint64_t* ka = keys_in;
    uint64_t* kb = keys_out;
    int32_t* va = idx_in;
    int32_t* vb = idx_out;
    if (passes % 2 == 0) {   // an even number of passes ends where it starts: begin from a copy in keys_out
        if (hipMemcpyAsync(keys_out, keys_in, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return false;
        if (pairs && hipMemcpyAsync(idx_out, idx_in, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return false;
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3(n_tiles), dim3(256), 0, s, ka, n, shift, n_tiles, hist);
        if (scan_many<int32_t, int32_t, true>(hist, hist, nh, ts, s) != hipSuccess) return false;
        if (pairs)
            hipLaunchKernelGGL(k_rs_scatter<true>, dim3(n_tiles), dim3(256), 0, s, ka, va, n, shift, n_tiles, hist,
                               kb, vb);
        else
            hipLaunchKernelGGL(k_rs_scatter<false>, dim3(n_tiles), dim3(256), 0, s, ka, va, n, shift, n_tiles, hist,
                               kb, vb);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    return hipGetLastError() == hipSuccess;
}

static bool sort_pairs(Tmp& tmp, uint64_t* keys_in, uint64_t* keys_out, int32_t* idx_in, int32_t* idx_out, int64_t n,
                       int bits, hipStream_t s) {
    return radix_sort(tmp, keys_in, keys_out, idx_in, idx_out, n, bits, s);
}

static bool sort_keys(Tmp& tmp, uint64_t* in, uint64_t* out, int64_t n, int bits, hipStream_t s) {
    return radix_sort(tmp, in, out, nullptr, nullptr, n, bits, s);
}

static bool exclusive_sum(Tmp& tmp, const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
    int32_t* ts = tmp.get<int32_t>(scan_tiles(n));
    if (!tmp.ok) return false;
    return scan_many<int32_t, int32_t, true>(in, out, n, ts, s) == hipSuccess;
}

// CSR of the edge list (a[i] -> b[i], weight w[i]) sorted by (a, b).
// Outputs rp[n_a+1], ci[m] (b mapped through map_b if given), w (FP64), and
// the row-sorted a of each entry (rows_sorted).
static bhpp_status csr_from(Tmp& tmp, int64_t m, const int32_t* a, const int32_t* b, const double* w, int32_t n_a,
                            int32_t n_b, const int32_t* map_b, int64_t* rp, int32_t* ci, double* w_out, hipStream_t s) {
    uint64_t* k0 = tmp.get<uint64_t>(m);
    uint64_t* k1 = tmp.get<uint64_t>(m);
    int32_t* i0 = tmp.get<int32_t>(m);
    int32_t* i1 = tmp.get<int32_t>(m);
    int32_t* rows = tmp.get<int32_t>(m);
    if (!tmp.ok) return BHPP_OUT_OF_MEMORY;
    if (m > 0) {
        hipLaunchKernelGGL(k_keys_pair, grid_for(m), dim3(256), 0, s, m, a, b, (int64_t)n_b, k0, i0);
        const int bits = bits_for((uint64_t)n_a * (uint64_t)n_b);
        if (!sort_pairs(tmp, k0, k1, i0, i1, m, bits, s)) return BHPP_DEVICE_ERROR;
        hipLaunchKernelGGL(k_rows_from_keys, grid_for(m), dim3(256), 0, s, m, k1, (int64_t)n_b, rows);
        hipLaunchKernelGGL(k_gather_i32, grid_for(m), dim3(256), 0, s, m, i1, b, map_b, ci);
        hipLaunchKernelGGL(k_gather_f64, grid_for(m), dim3(256), 0, s, m, i1, w, w_out);
    }
    hipLaunchKernelGGL(k_row_ptr, grid_for((int64_t)n_a + 1), dim3(256), 0, s, n_a, m, rows, rp);
    BHPP_HIP(hipGetLastError());
    return BHPP_OK;
}

template <typename WT>
bhpp_status build_impl(int32_t nu, int32_t nv, int64_t n, const int32_t* eu, const int32_t* ev, const WT* ew,
                       const bhpp_graph_opts& opts, hipStream_t s, Graph* g) {
    Tmp tmp;
    hipEvent_t e0, e1;
    BHPP_HIP(hipEventCreate(&e0));
    BHPP_HIP(hipEventCreate(&e1));
    BHPP_HIP(hipEventRecord(e0, s));
    // 1. validate
    int32_t* flags = tmp.get<int32_t>(1);
    if (!tmp.ok) return BHPP_OUT_OF_MEMORY;
    BHPP_HIP(hipMemsetAsync(flags, 0, sizeof(int32_t), s));
    if (n > 0) hipLaunchKernelGGL(k_validate<WT>, dim3(1024), dim3(256), 0, s, n, eu, ev, ew, nu, nv, flags);
    int32_t hflags = 0;
    BHPP_HIP(hipMemcpyAsync(&hflags, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BHPP_HIP(hipStreamSynchronize(s));
    if (hflags & 1) return BHPP_OUT_OF_RANGE;
    if (hflags & 2) return BHPP_BAD_WEIGHT;

    // 2. sort by (u, v), merge duplicates
    uint64_t* k0 = tmp.get<uint64_t>(n);
    uint64_t* k1 = tmp.get<uint64_t>(n);
    int32_t* i0 = tmp.get<int32_t>(n);
    int32_t* i1 = tmp.get<int32_t>(n);
    int32_t* head = tmp.get<int32_t>(n);
    int32_t* pos = tmp.get<int32_t>(n);
    if (!tmp.ok) return BHPP_OUT_OF_MEMORY;
    int64_t m = 0;
    if (n > 0) {
        hipLaunchKernelGGL(k_keys_pair, grid_for(n), dim3(256), 0, s, n, eu, ev, (int64_t)nv, k0, i0);
        if (!sort_pairs(tmp, k0, k1, i0, i1, n, bits_for((uint64_t)nu * (uint64_t)nv), s)) return BHPP_DEVICE_ERROR;
        hipLaunchKernelGGL(k_heads, grid_for(n), dim3(256), 0, s, n, k1, head);
        if (!exclusive_sum(tmp, head, pos, n, s)) return BHPP_DEVICE_ERROR;
        int32_t last_pos = 0, last_head = 0;
        BHPP_HIP(hipMemcpyAsync(&last_pos, pos + (n - 1), 4, hipMemcpyDeviceToHost, s));
        BHPP_HIP(hipMemcpyAsync(&last_head, head + (n - 1), 4, hipMemcpyDeviceToHost, s));
        BHPP_HIP(hipStreamSynchronize(s));
        m = (int64_t)last_pos + last_head;
    }
    int32_t* u_of = tmp.get<int32_t>(m);
    int32_t* v_of = tmp.get<int32_t>(m);
    double* w_of = tmp.get<double>(m);
    if (!tmp.ok) return BHPP_OUT_OF_MEMORY;
    if (n > 0)
        hipLaunchKernelGGL(k_merge<WT>, grid_for(n), dim3(256), 0, s, n, k1, i1, head, pos, ew, (int64_t)nv, u_of,
                           v_of, w_of);
    g->ne = m;

    // 3. external adjacency in both directions and Eq. (d)
    int64_t* xrp_u = tmp.get<int64_t>((size_t)nu + 1);
    int32_t* xci_u = tmp.get<int32_t>(m);
    double* xw_u = tmp.get<double>(m);
    int64_t* xrp_v = tmp.get<int64_t>((size_t)nv + 1);
    int32_t* xci_v = tmp.get<int32_t>(m);
    double* xw_v = tmp.get<double>(m);
    double* ws_u = tmp.get<double>(nu);
    double* ws_v = tmp.get<double>(nv);
    if (!tmp.ok) return BHPP_OUT_OF_MEMORY;
    bhpp_status rc = csr_from(tmp, m, u_of, v_of, w_of, nu, nv, nullptr, xrp_u, xci_u, xw_u, s);
    if (rc) return rc;
    rc = csr_from(tmp, m, v_of, u_of, w_of, nv, nu, nullptr, xrp_v, xci_v, xw_v, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_row_sums, grid_for(nu), dim3(256), 0, s, nu, xrp_u, xw_u, ws_u);
    hipLaunchKernelGGL(k_row_sums, grid_for(nv), dim3(256), 0, s, nv, xrp_v, xw_v, ws_v);
    BHPP_HIP(hipGetLastError());

    // 4. degree order
    const int reorder = (opts.flags & BHPP_BUILD_NO_REORDER) ? 0 : 1;
    int32_t* perm_v = tmp.get<int32_t>(nv);
    int32_t* iperm_v = tmp.get<int32_t>(nv);
    uint64_t* dk0 = tmp.get<uint64_t>(std::max(nu, nv));
    uint64_t* dk1 = tmp.get<uint64_t>(std::max(nu, nv));
    if (!tmp.ok) return BHPP_OUT_OF_MEMORY;
    BHPP_HIP(hipMalloc((void**)&g->perm_u, sizeof(int32_t) * nu));
    BHPP_HIP(hipMalloc((void**)&g->iperm_u, sizeof(int32_t) * nu));
    hipLaunchKernelGGL(k_degree_keys, grid_for(nu), dim3(256), 0, s, nu, xrp_u, reorder, dk0);
    if (!sort_keys(tmp, dk0, dk1, nu, 64, s)) return BHPP_DEVICE_ERROR;
    hipLaunchKernelGGL(k_perm_from_keys, grid_for(nu), dim3(256), 0, s, nu, dk1, g->iperm_u, g->perm_u);
    hipLaunchKernelGGL(k_degree_keys, grid_for(nv), dim3(256), 0, s, nv, xrp_v, reorder, dk0);
    if (!sort_keys(tmp, dk0, dk1, nv, 64, s)) return BHPP_DEVICE_ERROR;
    hipLaunchKernelGGL(k_perm_from_keys, grid_for(nv), dim3(256), 0, s, nv, dk1, iperm_v, perm_v);
    BHPP_HIP(hipGetLastError());
    BHPP_HIP(hipMalloc((void**)&g->iperm_v, sizeof(int32_t) * nv));
    BHPP_HIP(hipMemcpyAsync(g->iperm_v, iperm_v, sizeof(int32_t) * nv, hipMemcpyDeviceToDevice, s));

    // 5. internal adjacency: relabel, then sort each direction
    int32_t* iu = tmp.get<int32_t>(m);
    int32_t* iv = tmp.get<int32_t>(m);
    if (!tmp.ok) return BHPP_OUT_OF_MEMORY;
    if (m > 0) {
        hipLaunchKernelGGL(k_map_i32, grid_for(m), dim3(256), 0, s, m, u_of, g->perm_u, iu);
        hipLaunchKernelGGL(k_map_i32, grid_for(m), dim3(256), 0, s, m, v_of, perm_v, iv);
    }
    double* w_int_u = tmp.get<double>(m);
    double* w_int_v = tmp.get<double>(m);
    if (!tmp.ok) return BHPP_OUT_OF_MEMORY;
    BHPP_HIP(hipMalloc((void**)&g->rp_u, sizeof(int64_t) * ((size_t)nu + 1)));
    BHPP_HIP(hipMalloc((void**)&g->ci_u, sizeof(int32_t) * std::max<int64_t>(m, 1)));
    BHPP_HIP(hipMalloc((void**)&g->rp_v, sizeof(int64_t) * ((size_t)nv + 1)));
    BHPP_HIP(hipMalloc((void**)&g->ci_v, sizeof(int32_t) * std::max<int64_t>(m, 1)));
    BHPP_HIP(hipMalloc(&g->w_u, sizeof(WT) * std::max<int64_t>(m, 1)));
    BHPP_HIP(hipMalloc(&g->w_v, sizeof(WT) * std::max<int64_t>(m, 1)));
    rc = csr_from(tmp, m, iu, iv, w_of, nu, nv, nullptr, g->rp_u, g->ci_u, w_int_u, s);
    if (rc) return rc;
    rc = csr_from(tmp, m, iv, iu, w_of, nv, nu, nullptr, g->rp_v, g->ci_v, w_int_v, s);
    if (rc) return rc;
    if (m > 0) {
        hipLaunchKernelGGL(k_scale_by_col<WT>, grid_for(m), dim3(256), 0, s, m, w_int_u, g->ci_u, iperm_v, ws_v,
                           (WT*)g->w_u);
        hipLaunchKernelGGL(k_cast<WT>, grid_for(m), dim3(256), 0, s, m, w_int_v, (WT*)g->w_v);
    }
    {   // row-end bitmaps (one spare word so a reader may load word i+1)
        const size_t words = (size_t)(m >> 6) + 2;
        BHPP_HIP(hipMalloc((void**)&g->end_bits_u, 8 * words));
        BHPP_HIP(hipMalloc((void**)&g->end_bits_v, 8 * words));
        BHPP_HIP(hipMemsetAsync(g->end_bits_u, 0, 8 * words, s));
        BHPP_HIP(hipMemsetAsync(g->end_bits_v, 0, 8 * words, s));
        hipLaunchKernelGGL(k_end_bits, grid_for(nu), dim3(256), 0, s, nu, g->rp_u, (unsigned long long*)g->end_bits_u);
        hipLaunchKernelGGL(k_end_bits, grid_for(nv), dim3(256), 0, s, nv, g->rp_v, (unsigned long long*)g->end_bits_v);
    }
    BHPP_HIP(hipMalloc((void**)&g->deg_u, sizeof(int32_t) * nu));
    hipLaunchKernelGGL(k_degrees, grid_for(nu), dim3(256), 0, s, nu, g->rp_u, g->deg_u);
    BHPP_HIP(hipMalloc((void**)&g->inv_ws_u_d, sizeof(double) * nu));
    BHPP_HIP(hipMalloc((void**)&g->inv_ws_v_d, sizeof(double) * nv));
    hipLaunchKernelGGL(k_inv_ws<double>, grid_for(nu), dim3(256), 0, s, nu, g->iperm_u, ws_u, g->inv_ws_u_d);
    hipLaunchKernelGGL(k_inv_ws<double>, grid_for(nv), dim3(256), 0, s, nv, iperm_v, ws_v, g->inv_ws_v_d);
    if (sizeof(WT) == 4) {
        BHPP_HIP(hipMalloc((void**)&g->inv_ws_u_f, sizeof(float) * nu));
        BHPP_HIP(hipMalloc((void**)&g->inv_ws_v_f, sizeof(float) * nv));
        hipLaunchKernelGGL(k_inv_ws<float>, grid_for(nu), dim3(256), 0, s, nu, g->iperm_u, ws_u, g->inv_ws_u_f);
        hipLaunchKernelGGL(k_inv_ws<float>, grid_for(nv), dim3(256), 0, s, nv, iperm_v, ws_v, g->inv_ws_v_f);
    }
    // 1/ws of each entry's U node along the rows of W^T, stored beside the
    // adjacency: the 64-column V-side gather reads it with the indices when it
    // applies the push rule itself
    BHPP_HIP(hipMalloc(&g->iw_v, sizeof(WT) * std::max<int64_t>(m, 1)));
    hipLaunchKernelGGL(k_take<WT>, grid_for(m), dim3(256), 0, s, m, g->ci_v,
                       sizeof(WT) == 4 ? (const WT*)g->inv_ws_u_f : (const WT*)g->inv_ws_u_d, (WT*)g->iw_v);
    BHPP_HIP(hipGetLastError());

    // 6. external copies for export
    if (opts.flags & BHPP_BUILD_KEEP_EXTERNAL) {
        BHPP_HIP(hipMalloc((void**)&g->x_rp_u, sizeof(int64_t) * ((size_t)nu + 1)));
        BHPP_HIP(hipMalloc((void**)&g->x_rp_v, sizeof(int64_t) * ((size_t)nv + 1)));
        BHPP_HIP(hipMalloc((void**)&g->x_ci_u, sizeof(int32_t) * std::max<int64_t>(m, 1)));
        BHPP_HIP(hipMalloc((void**)&g->x_ci_v, sizeof(int32_t) * std::max<int64_t>(m, 1)));
        BHPP_HIP(hipMalloc(&g->x_w_u, sizeof(WT) * std::max<int64_t>(m, 1)));
        BHPP_HIP(hipMalloc(&g->x_w_v, sizeof(WT) * std::max<int64_t>(m, 1)));
        BHPP_HIP(hipMalloc(&g->x_ws_u, sizeof(WT) * nu));
        BHPP_HIP(hipMalloc(&g->x_ws_v, sizeof(WT) * nv));
        BHPP_HIP(hipMemcpyAsync(g->x_rp_u, xrp_u, sizeof(int64_t) * ((size_t)nu + 1), hipMemcpyDeviceToDevice, s));
        BHPP_HIP(hipMemcpyAsync(g->x_rp_v, xrp_v, sizeof(int64_t) * ((size_t)nv + 1), hipMemcpyDeviceToDevice, s));
        if (m > 0) {
            BHPP_HIP(hipMemcpyAsync(g->x_ci_u, xci_u, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, s));
            BHPP_HIP(hipMemcpyAsync(g->x_ci_v, xci_v, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL(k_cast<WT>, grid_for(m), dim3(256), 0, s, m, xw_u, (WT*)g->x_w_u);
            hipLaunchKernelGGL(k_cast<WT>, grid_for(m), dim3(256), 0, s, m, xw_v, (WT*)g->x_w_v);
        }
        hipLaunchKernelGGL(k_cast<WT>, grid_for(nu), dim3(256), 0, s, (int64_t)nu, ws_u, (WT*)g->x_ws_u);
        hipLaunchKernelGGL(k_cast<WT>, grid_for(nv), dim3(256), 0, s, (int64_t)nv, ws_v, (WT*)g->x_ws_v);
        BHPP_HIP(hipGetLastError());
    }
    // 7. MCSP's alias tables from the merged FP64 weights in caller ids
    if (opts.flags & BHPP_BUILD_MCSP) {
        rc = mcsp_build_tables(g, xrp_u, xci_u, xw_u, ws_u, xrp_v, xci_v, xw_v, ws_v, s);
        if (rc) return rc;
    }

    // 7. host-side summaries and tiles
    g->h_ws_u.resize(nu);
    g->h_perm_u.resize(nu);
    std::vector<double> h_ws_v(nv);
    std::vector<int64_t> h_rp_u((size_t)nu + 1), h_rp_v((size_t)nv + 1);
    BHPP_HIP(hipMemcpyAsync(g->h_ws_u.data(), ws_u, sizeof(double) * nu, hipMemcpyDeviceToHost, s));
    BHPP_HIP(hipMemcpyAsync(h_ws_v.data(), ws_v, sizeof(double) * nv, hipMemcpyDeviceToHost, s));
    BHPP_HIP(hipMemcpyAsync(g->h_perm_u.data(), g->perm_u, sizeof(int32_t) * nu, hipMemcpyDeviceToHost, s));
    BHPP_HIP(hipMemcpyAsync(h_rp_u.data(), g->rp_u, sizeof(int64_t) * ((size_t)nu + 1), hipMemcpyDeviceToHost, s));
    BHPP_HIP(hipMemcpyAsync(h_rp_v.data(), g->rp_v, sizeof(int64_t) * ((size_t)nv + 1), hipMemcpyDeviceToHost, s));
    BHPP_HIP(hipStreamSynchronize(s));
    rc = build_tiles(h_rp_u, nu, g->tile_edges, &g->tiles_u);
    if (rc) return rc;
    rc = build_tiles(h_rp_v, nv, g->tile_edges, &g->tiles_v);
    if (rc) return rc;
    rc = build_tiles(h_rp_u, nu, g->tile_edges, &g->tiles_uf, upd_rows(g->elem));
    if (rc) return rc;
    g->h_rp_u = std::move(h_rp_u);
    g->h_rp_v = std::move(h_rp_v);

    bhpp_graph_summary& I = g->info;
    I.n_u = nu;
    I.n_v = nv;
    I.n_edges = m;
    I.dtype = g->dtype;
    I.isolated_u = 0;
    I.isolated_v = 0;
    I.ws_u_max = 0.0;
    I.ws_u_min = INFINITY;
    for (int32_t x = 0; x < nu; ++x) {
        const double w = g->h_ws_u[x];
        if (w > 0.0) {
            I.ws_u_max = std::max(I.ws_u_max, w);
            I.ws_u_min = std::min(I.ws_u_min, w);
        } else {
            I.isolated_u++;
        }
    }
    for (int32_t y = 0; y < nv; ++y)
        if (!(h_ws_v[y] > 0.0)) I.isolated_v++;
    if (!(I.ws_u_min < INFINITY)) I.ws_u_min = 0.0;
    // Eq. (epsilon-b); mu >= 1 would leave (0, eps), then eps/2
    I.mu = m > 0 ? std::sqrt((double)nu * (double)nv) / (double)m : INFINITY;
    I.eps_b_ratio = I.mu < 1.0 ? (1.0 - I.mu) / (2.0 - I.mu) : 0.5;
    g->eps_b_paper = I.eps_b_ratio;

    // 8. lambda (Lemma 4)
    I.alpha = opts.alpha;
    int32_t tau = opts.tau;
    if (tau < 0) {   // smallest tau with |U| (1-alpha)^(tau+1) <= 1
        tau = 0;
        double mm = (double)nu * (1.0 - opts.alpha);
        while (mm > 1.0) { mm *= (1.0 - opts.alpha); ++tau; }
    }
    g->tau = tau;
    I.tau = tau;
    double lam = 1.0;
    if (m > 0) {
        rc = compute_lambda(g, opts.alpha, tau, s, &lam);
        if (rc) return rc;
    }
    I.lambda = lam;
    g->lambda_cache[opts.alpha] = lam;
    BHPP_HIP(hipEventRecord(e1, s));
    BHPP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    I.build_ms = ms;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return BHPP_OK;
}

}  // namespace

bhpp_status build_graph(int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* eu, const int32_t* ev,
                        const void* ew, const bhpp_graph_opts& opts, hipStream_t s, Graph** out) {
    Graph* g = new (std::nothrow) Graph();
    if (!g) return BHPP_OUT_OF_MEMORY;
    // launch settings: defaults, or BHPP_TUNE="tile=512,inflight=8,nt=0,graphs=1" (also sparse=, narrow=, fuse=,
    // hub=, chunk=, async=, upd=, urows=, order=)
    bool chunk_set = false, tile_set = false;
    if (const char* e = getenv("BHPP_TUNE")) {
        int v;
        const char* q;
        if ((q = strstr(e, "tile=")) && sscanf(q, "tile=%d", &v) == 1 && v >= 64) {
            g->tile_edges = v;
            tile_set = true;
        }
        if ((q = strstr(e, "inflight=")) && sscanf(q, "inflight=%d", &v) == 1 && (v == 4 || v == 8 || v == 16))
            g->inflight = v;
        if ((q = strstr(e, "nt=")) && sscanf(q, "nt=%d", &v) == 1) g->nt_stream = v ? 1 : 0;
        if ((q = strstr(e, "graphs=")) && sscanf(q, "graphs=%d", &v) == 1) g->use_graphs = v ? 1 : 0;
        if ((q = strstr(e, "sparse=")) && sscanf(q, "sparse=%d", &v) == 1) g->sparse_steps = v ? 1 : 0;
        if ((q = strstr(e, "narrow=")) && sscanf(q, "narrow=%d", &v) == 1) g->narrow = v ? 1 : 0;
        if ((q = strstr(e, "fuse=")) && sscanf(q, "fuse=%d", &v) == 1) g->fuse_select = v ? 1 : 0;
        if ((q = strstr(e, "hub=")) && sscanf(q, "hub=%d", &v) == 1) g->hub_lds = v ? 1 : 0;
        if ((q = strstr(e, "bufa=")) && sscanf(q, "bufa=%d", &v) == 1) g->buf_rows = v ? 1 : 0;
        if ((q = strstr(e, "chunk=")) && sscanf(q, "chunk=%d", &v) == 1 && v >= 1 && v <= 8) {
            g->chunk_sweeps = v;
            chunk_set = true;
        }
        if ((q = strstr(e, "async=")) && sscanf(q, "async=%d", &v) == 1) g->async_sched = v ? 1 : 0;
        if ((q = strstr(e, "upd=")) && sscanf(q, "upd=%d", &v) == 1) g->fuse_update = v ? 1 : 0;
        if ((q = strstr(e, "urows=")) && sscanf(q, "urows=%d", &v) == 1 && (v == 2 || v == 4)) g->upd_inflight = v;
        if ((q = strstr(e, "order=")) && sscanf(q, "order=%d", &v) == 1) g->order_admit = v ? 1 : 0;
    }
    if (opts.flags & BHPP_BUILD_DENSE_ONLY) g->sparse_steps = 0;
    if (opts.flags & BHPP_BUILD_FIXED_WIDTH) g->narrow = 0;
    if (!tile_set) {
        // entries per work tile before any autotuning: about three tiles per
        // wavefront of the gathers' largest grid (2048 blocks of 4 waves),
        // a power of two in [256, 4096] (4096 measured best on 100M edges)
        int te = 256;
        while (te < 4096 && (double)te * 3.0 * 8192.0 < (double)n_edges) te *= 2;
        g->tile_edges = te;
    }
    g->nu = n_u;
    g->nv = n_v;
    g->dtype = opts.dtype;
    g->elem = opts.dtype == BHPP_DTYPE_F64 ? 8 : 4;
    bhpp_status rc;
    if (opts.dtype == BHPP_DTYPE_F64)
        rc = build_impl<double>(n_u, n_v, n_edges, eu, ev, (const double*)ew, opts, s, g);
    else
        rc = build_impl<float>(n_u, n_v, n_edges, eu, ev, (const float*)ew, opts, s, g);
    if (rc) {
        (void)hipGetLastError();
        free_graph(g);
        return rc;
    }
    if (!chunk_set) {
        // sweeps per chunk before any autotuning, by the autotuner's rule (about
        // 2 ms of sweeps per chunk) on an estimate of a 64-column sweep: both
        // gathers read a 256-byte row per entry at about 6 TB/s
        const double sweep_ms = 2.0 * (double)g->ne * 264.0 / 6.0e9;
        int chunk = 8;
        while (chunk > 1 && chunk * sweep_ms > 2.0) chunk /= 2;
        g->chunk_sweeps = chunk;
    }
    *out = g;
    return BHPP_OK;
}

}  // namespace bhpp
