// Top-k of each row of a score matrix, ordered by (score descending, id
// ascending): the retrieval of the nodes most similar to a query node
// (Sec. 1; Sec. 5 uses the top-k of BHPP). -0 ranks as +0.
//
// Every element gets a unique key: the order-preserving bit pattern of its
// score followed by the complement of its id, so "larger key" = "better".
// A most-significant-digit radix select (8-bit digits) finds, row by row, the
// shortest key prefix whose bucket completes the top k; one collect pass
// gathers exactly the k keys at or above it, and a bitonic sort in LDS orders
// them. All passes read rows with coalesced loads; many blocks share a row.
#include <cstring>
#include <mutex>

#include "common.h"

namespace bhpp {

constexpr int kTopkThreads = 256;
constexpr int kTopkPerThread = 16;
constexpr int kTopkChunk = kTopkThreads * kTopkPerThread;
constexpr int kTopkMaxK = 4096;
constexpr int kTopkStaticRows = 64;   // rows per call of the allocation-free top-k

struct TopkRow {
    uint64_t pre_hi;   // chosen digits so far (left-aligned in a 96-bit key)
    uint32_t pre_lo;
    int32_t depth;     // number of chosen digits
    int32_t kk;        // elements still to take from the current bucket
    int32_t done;
    int32_t count;     // collected candidates
    int32_t pad;
};

// 96-bit key = [hi: 64 bits][lo: 32 bits]. FP32: hi = ord(score) << 32 | ~id,
// lo = 0 (8 digits used). FP64: hi = ord(score), lo = ~id (12 digits).
struct Key {
    uint64_t hi;
    uint32_t lo;
};

__device__ __forceinline__ uint32_t ord32(float s) {
    uint32_t u = __float_as_uint(s == 0.0f ? 0.0f : s);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ uint64_t ord64(double s) {
    uint64_t u = (uint64_t)__double_as_longlong(s == 0.0 ? 0.0 : s);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

template <typename VT>
struct KeyOf;
template <>
struct KeyOf<float> {
    static constexpr int kDigits = 8;
    __device__ static Key make(float s, uint32_t id) { return Key{((uint64_t)ord32(s) << 32) | (uint64_t)(~id), 0u}; }
};
template <>
struct KeyOf<double> {
    static constexpr int kDigits = 12;
    __device__ static Key make(double s, uint32_t id) { return Key{ord64(s), ~id}; }
};

__device__ __forceinline__ uint32_t digit_of(const Key& k, int d) {
    return d < 8 ? (uint32_t)(k.hi >> (56 - 8 * d)) & 0xFFu : (k.lo >> (24 - 8 * (d - 8))) & 0xFFu;
}

// top `depth` digits of k compared with the chosen prefix: -1, 0, +1
__device__ __forceinline__ int cmp_prefix(const Key& k, uint64_t pre_hi, uint32_t pre_lo, int depth) {
    if (depth == 0) return 0;
    if (depth <= 8) {
        const uint64_t a = k.hi >> (64 - 8 * depth), b = pre_hi >> (64 - 8 * depth);
        return a < b ? -1 : (a > b ? 1 : 0);
    }
    if (k.hi != pre_hi) return k.hi < pre_hi ? -1 : 1;
    const int dl = depth - 8;
    const uint32_t a = k.lo >> (32 - 8 * dl), b = pre_lo >> (32 - 8 * dl);
    return a < b ? -1 : (a > b ? 1 : 0);
}

__device__ __forceinline__ Key excluded_key() { return Key{0ull, 0u}; }

template <typename VT>
__device__ __forceinline__ Key load_key(const VT* row, int32_t i, int32_t ex) {
    return i == ex ? excluded_key() : KeyOf<VT>::make(row[i], (uint32_t)i);
}

__global__ void k_topk_init(TopkRow* st, int n_rows, int k, uint32_t* hist) {
    int r = blockIdx.x;
    if (threadIdx.x == 0) {
        TopkRow t;
        memset(&t, 0, sizeof(t));
        t.kk = k;
        st[r] = t;
    }
    hist[(size_t)r * 256 + threadIdx.x] = 0;
}

template <typename VT>
__global__ __launch_bounds__(kTopkThreads) void k_topk_hist(const VT* scores, int32_t n, const int32_t* exclude,
                                                           const TopkRow* st, int d, uint32_t* hist) {
    __shared__ uint32_t h[256];
    const int row = blockIdx.y;
    const TopkRow t = st[row];
    if (t.done) return;
    h[threadIdx.x] = 0;
    __syncthreads();
    const VT* R = scores + (size_t)row * n;
    const int32_t ex = exclude ? exclude[row] : -1;
    const int32_t base = blockIdx.x * kTopkChunk;
    for (int j = 0; j < kTopkPerThread; ++j) {
        const int32_t i = base + j * kTopkThreads + threadIdx.x;
        if (i >= n) break;
        const Key key = load_key<VT>(R, i, ex);
        if (cmp_prefix(key, t.pre_hi, t.pre_lo, t.depth) == 0) atomicAdd(&h[digit_of(key, d)], 1u);
    }
    __syncthreads();
    const uint32_t c = h[threadIdx.x];
    if (c) atomicAdd(&hist[(size_t)row * 256 + threadIdx.x], c);
}

// Pick the bucket holding the kk-th largest remaining key.
__global__ __launch_bounds__(256) void k_topk_select(TopkRow* st, int d, uint32_t* hist, int last_digit) {
    __shared__ uint32_t cnt[256];
    __shared__ uint32_t scan[256];
    const int row = blockIdx.x;
    uint32_t* H = hist + (size_t)row * 256;
    TopkRow t = st[row];
    // bucket 255 first: thread j looks at bucket 255 - j
    const uint32_t c = H[255 - threadIdx.x];
    cnt[threadIdx.x] = c;
    scan[threadIdx.x] = c;
    H[255 - threadIdx.x] = 0;
    __syncthreads();
    if (t.done) return;
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0u;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    const uint32_t incl = scan[threadIdx.x];
    const uint32_t excl = incl - cnt[threadIdx.x];
    if (excl < (uint32_t)t.kk && incl >= (uint32_t)t.kk) {
        const uint32_t b = 255u - threadIdx.x;
        t.kk -= (int32_t)excl;
        if (d < 8)
            t.pre_hi |= (uint64_t)b << (56 - 8 * d);
        else
            t.pre_lo |= b << (24 - 8 * (d - 8));
        t.depth = d + 1;
        if (cnt[threadIdx.x] == (uint32_t)t.kk || d == last_digit) t.done = 1;
        st[row] = t;
    }
}

struct Cand {
    uint64_t hi;
    uint32_t lo;
    int32_t id;
};

template <typename VT>
__global__ __launch_bounds__(kTopkThreads) void k_topk_collect(const VT* scores, int32_t n, const int32_t* exclude,
                                                              TopkRow* st, int k, Cand* cand) {
    const int row = blockIdx.y;
    const TopkRow t = st[row];
    const VT* R = scores + (size_t)row * n;
    const int32_t ex = exclude ? exclude[row] : -1;
    const int32_t base = blockIdx.x * kTopkChunk;
    for (int j = 0; j < kTopkPerThread; ++j) {
        const int32_t i = base + j * kTopkThreads + threadIdx.x;
        if (i >= n) break;
        if (i == ex) continue;
        const Key key = load_key<VT>(R, i, ex);
        if (cmp_prefix(key, t.pre_hi, t.pre_lo, t.depth) >= 0) {
            const int p = atomicAdd(&st[row].count, 1);
            if (p < k) cand[(size_t)row * k + p] = Cand{key.hi, key.lo, i};
        }
    }
}

__device__ __forceinline__ bool key_less(const Cand& a, const Cand& b) {
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

// Bitonic sort of the k candidates of a row, descending by key.
template <typename VT>
__global__ __launch_bounds__(1024) void k_topk_sort(const VT* scores, int32_t n, const Cand* cand, const TopkRow* st,
                                                   int k, int kp2, int32_t* ids_out, VT* vals_out) {
    extern __shared__ Cand sh[];
    const int row = blockIdx.x;
    const int have = min(st[row].count, k);   // == k unless the selection went wrong
    for (int i = threadIdx.x; i < kp2; i += blockDim.x)
        sh[i] = i < have ? cand[(size_t)row * k + i] : Cand{0ull, 0u, -1};
    __syncthreads();
    for (int size = 2; size <= kp2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < kp2; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool desc = (i & size) == 0;
                    const Cand a = sh[i], b = sh[j];
                    const bool swap = desc ? key_less(a, b) : key_less(b, a);
                    if (swap) {
                        sh[i] = b;
                        sh[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const int id = sh[i].id;
        const bool ok = id >= 0 && id < n;
        ids_out[(size_t)row * k + i] = ok ? id : -1;
        vals_out[(size_t)row * k + i] = ok ? scores[(size_t)row * n + id] : VT(0);
    }
}

// The passes over n_rows rows with the scratch st[n_rows], hist[n_rows][256]
// and cand[n_rows][k] given by the caller; k_topk_init clears what must
// start at zero (no memset, so the passes can be captured in a graph).
template <typename VT>
static void topk_passes(const VT* scores, int32_t n_rows, int32_t n, int32_t k, const int32_t* exclude,
                        int32_t* ids_out, VT* vals_out, TopkRow* st, uint32_t* hist, Cand* cand, hipStream_t s) {
    const int digits = KeyOf<VT>::kDigits;
    const dim3 grid((n + kTopkChunk - 1) / kTopkChunk, n_rows);
    hipLaunchKernelGGL(k_topk_init, dim3(n_rows), dim3(256), 0, s, st, n_rows, k, hist);
    for (int d = 0; d < digits; ++d) {
        hipLaunchKernelGGL(k_topk_hist<VT>, grid, dim3(kTopkThreads), 0, s, scores, n, exclude, st, d, hist);
        hipLaunchKernelGGL(k_topk_select, dim3(n_rows), dim3(256), 0, s, st, d, hist, digits - 1);
    }
    hipLaunchKernelGGL(k_topk_collect<VT>, grid, dim3(kTopkThreads), 0, s, scores, n, exclude, st, k, cand);
    const int kp2 = next_pow2(k);
    const int threads = kp2 < 1024 ? (kp2 < 64 ? 64 : kp2) : 1024;
    hipLaunchKernelGGL(k_topk_sort<VT>, dim3(n_rows), dim3(threads), sizeof(Cand) * kp2, s, scores, n, cand, st, k,
                       kp2, ids_out, vals_out);
}

template <typename VT>
static bhpp_status topk_impl(const VT* scores, int32_t n_rows, int32_t n, int32_t k, const int32_t* exclude,
                             int32_t* ids_out, VT* vals_out, hipStream_t s) {
    TopkRow* st = nullptr;
    uint32_t* hist = nullptr;
    Cand* cand = nullptr;
    if (hipMallocAsync((void**)&st, sizeof(TopkRow) * n_rows, s) != hipSuccess ||
        hipMallocAsync((void**)&hist, sizeof(uint32_t) * 256 * n_rows, s) != hipSuccess ||
        hipMallocAsync((void**)&cand, sizeof(Cand) * (size_t)k * n_rows, s) != hipSuccess) {
        if (st) hipFreeAsync(st, s);
        if (hist) hipFreeAsync(hist, s);
        (void)hipGetLastError();
        return BHPP_OUT_OF_MEMORY;
    }
    topk_passes<VT>(scores, n_rows, n, k, exclude, ids_out, vals_out, st, hist, cand, s);
    hipError_t e = hipGetLastError();
    hipFreeAsync(st, s);
    hipFreeAsync(hist, s);
    hipFreeAsync(cand, s);
    return e == hipSuccess ? BHPP_OK : BHPP_DEVICE_ERROR;
}

bhpp_status topk_rows(const void* scores, int32_t n_rows, int32_t n, int32_t k, const int32_t* exclude,
                      int32_t dtype, int32_t* ids_out, void* vals_out, hipStream_t s) {
    if (k > kTopkMaxK) return BHPP_NOT_SUPPORTED;
    if (dtype != BHPP_DTYPE_F64 && dtype != BHPP_DTYPE_F32) return BHPP_NOT_SUPPORTED;
    const int per = 32768;   // rows per launch (grid.y limit)
    const size_t e = dtype == BHPP_DTYPE_F64 ? 8 : 4;
    for (int32_t r0 = 0; r0 < n_rows; r0 += per) {
        const int32_t nr = n_rows - r0 < per ? n_rows - r0 : per;
        const char* sc = (const char*)scores + (size_t)r0 * n * e;
        const int32_t* ex = exclude ? exclude + r0 : nullptr;
        int32_t* ids = ids_out + (size_t)r0 * k;
        char* vals = (char*)vals_out + (size_t)r0 * k * e;
        bhpp_status rc = dtype == BHPP_DTYPE_F64
                             ? topk_impl<double>((const double*)sc, nr, n, k, ex, ids, (double*)vals, s)
                             : topk_impl<float>((const float*)sc, nr, n, k, ex, ids, (float*)vals, s);
        if (rc) return rc;
    }
    return BHPP_OK;
}

// ---------------------------------------------------------------------------
// Top-k without allocation: the scratch of up to kTopkStaticRows rows at the
// largest k lives in one file-scope device array, `scratch`, that every call
// on a device shares (each device holds its own copy until the process ends).
// Host code never passes the array's name to a kernel: its device address is
// looked up once per device with hipGetSymbolAddress and kept in
// g_scratch_ptr.
// ---------------------------------------------------------------------------
constexpr size_t kScratchSt = 256 * ((sizeof(TopkRow) * kTopkStaticRows + 255) / 256);
constexpr size_t kScratchHist = sizeof(uint32_t) * 256 * kTopkStaticRows;
constexpr size_t kScratchCand = sizeof(Cand) * (size_t)kTopkMaxK * kTopkStaticRows;
constexpr size_t kScratchBytes = kScratchSt + kScratchHist + kScratchCand;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with it current).
static bhpp_status scratch_of_current_device(unsigned char** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BHPP_DEVICE_ERROR;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return BHPP_DEVICE_ERROR;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return BHPP_OK;
}

size_t topk_static_scratch_bytes() { return kScratchBytes; }

bhpp_status topk_rows_static(const void* scores, int32_t n_rows, int32_t n, int32_t k, const int32_t* exclude,
                             int32_t dtype, int32_t* ids_out, void* vals_out, hipStream_t s) {
    if (k > kTopkMaxK || n_rows > kTopkStaticRows) return BHPP_NOT_SUPPORTED;
    if (dtype != BHPP_DTYPE_F64 && dtype != BHPP_DTYPE_F32) return BHPP_NOT_SUPPORTED;
    if (n_rows == 0) return BHPP_OK;
    unsigned char* base = nullptr;
    bhpp_status rc = scratch_of_current_device(&base);
    if (rc) return rc;
    TopkRow* st = reinterpret_cast<TopkRow*>(base);
    uint32_t* hist = reinterpret_cast<uint32_t*>(base + kScratchSt);
    Cand* cand = reinterpret_cast<Cand*>(base + kScratchSt + kScratchHist);
    if (dtype == BHPP_DTYPE_F64)
        topk_passes<double>((const double*)scores, n_rows, n, k, exclude, ids_out, (double*)vals_out, st, hist, cand,
                            s);
    else
        topk_passes<float>((const float*)scores, n_rows, n, k, exclude, ids_out, (float*)vals_out, st, hist, cand, s);
    return hipGetLastError() == hipSuccess ? BHPP_OK : BHPP_DEVICE_ERROR;
}

}  // namespace bhpp
