// Warm-start network (gfx950): node features, a two-tower MLP in BF16 with
// FP32 accumulation on MFMA (forward, backward, Adam), node embeddings, and
// the per-query prediction that seeds the signed residue.
//
// The warm start is not part of the paper. It uses Lemma 1 (the push
// invariant holds for any start pi_b = y with residue
// r = e_u - (y - (1-alpha) P y)/alpha) and Lemma 3 (ws(u) pi(u,x) =
// ws(x) pi(x,u), so K(u,x) = pi(u,x)/ws(x) is symmetric). The network models
//     p_hat(u, x) = c ws(x) <f(feat(u)), g(feat(x))>   ~ pi(u, x),
// i.e. a start y(x) = ws(u)/ws(x) p_hat(u, x) of pi(x, u). In the sweep
// kernels' forward coordinates the start is ACC = p_hat directly.
//
// Towers f and g: 64 -> 256 -> 256 -> 128, GELU after both hidden layers.
// Parameters (FP32 master copy, BF16 compute copy) are one flat vector:
// tower f then tower g, each W1[64][256] b1[256] W2[256][256] b2[256]
// W3[256][128] b3[128], row-major, y = x W + b.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <unordered_map>

#include "common.h"

namespace bhpp {

namespace {

constexpr int kIn = 64, kHid = 256, kOut = 128, kBuckets = kIn - 4;
constexpr int64_t kOffW1 = 0, kOffB1 = kOffW1 + kIn * kHid, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
                  kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid * kOut, kTower = kOffB3 + kOut;
constexpr int64_t kParams = 2 * kTower;
constexpr int kEmbedChunk = 32768;   // rows per tower pass when embedding all nodes

typedef uint16_t bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__host__ __device__ inline bf16 to_bf16(float f) {   // round to nearest, ties to even
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16)(u >> 16);
}
__device__ inline float from_bf16(bf16 h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ---------------------------------------------------------------------------
// GEMM on MFMA: C[M][N] = A[M][K] B[K][N], A and B BF16 with arbitrary element
// strides (so transposed operands need no copy), FP32 accumulation, and an
// epilogue. A workgroup of 4 waves owns a 64x64 tile of C; each wave a 32x32
// quarter computed by gfx950's v_mfma_f32_32x32x16_bf16 over K chunks of 32
// staged in LDS (A as [row][k], B as [col][k], so each lane's operand is 8
// contiguous k: one 16-byte LDS read).
// ---------------------------------------------------------------------------
enum Epi { EPI_F32 = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_BWD = 3, EPI_PRED = 4, EPI_LOSS = 5 };

struct GemmArgs {
    int M, N, K;
    const bf16* A;
    int64_t a_rs, a_cs;      // A(i,k) = A[i*a_rs + k*a_cs]
    const bf16* B;
    int64_t b_rs, b_cs;      // B(k,j) = B[k*b_rs + j*b_cs]
    int epi;
    const float* bias;       // [N]                                    BIAS, BIAS_GELU
    float* outf;             // FP32 result [M][ld_f] (nullable)
    int64_t ld_f;
    bf16* outh;              // BF16 result [M][ld_h] (nullable)
    int64_t ld_h;
    const float* aux;        // GELU_BWD: pre-activation z [M][ld_f]; LOSS: targets [M][N]
    const float* vec;        // PRED: per-row ws(x); LOSS: per-column ws(x_j)
    float scale;             // PRED, LOSS: c
    float sigma;             // LOSS: tau of the weight 1/(T + tau)
    float inv_n;             // LOSS: 1 / (number of known targets)
    float* loss_part;        // LOSS: one partial per workgroup
    // structural self term: prior[node] is added where row node == column node
    const float* prior;      // PRED, LOSS (nullable)
    const int32_t* row_node; // LOSS: node of each row
    const int32_t* col_node; // PRED, LOSS: node of each column (-1: none)
};

// Stage the 64 x 32 block X(r, k) = X[r rs + k ks], rows r0.., k from k0,
// into S[r][k] (zero outside n_r x K). Where k (or r) is the contiguous
// dimension and 8 entries stay in range on 16-byte boundaries, a thread moves
// them with one 16-byte load; otherwise entry by entry.
__device__ inline void stage_block(bf16 (*S)[40], const bf16* X, int64_t rs, int64_t ks, int n_r, int K, int r0,
                                   int k0, bool vec_ok, int tid) {
    if (ks == 1 && vec_ok) {   // 4 threads per row, 8 k each
        const int r = tid >> 2, kk = (tid & 3) * 8, i = r0 + r, k = k0 + kk;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (i < n_r && k + 8 <= K) {
            v = *reinterpret_cast<const uint4*>(X + (int64_t)i * rs + k);
        } else if (i < n_r) {
            bf16 t[8];
            for (int q = 0; q < 8; ++q) t[q] = k + q < K ? X[(int64_t)i * rs + k + q] : (bf16)0;
            memcpy(&v, t, 16);
        }
        *reinterpret_cast<uint4*>(&S[r][kk]) = v;
        return;
    }
    if (rs == 1 && vec_ok) {   // 8 threads per k, 8 rows each
        const int kk = tid >> 3, r = (tid & 7) * 8, i = r0 + r, k = k0 + kk;
        bf16 t[8];
        if (k < K && i + 8 <= n_r) {
            const uint4 v = *reinterpret_cast<const uint4*>(X + (int64_t)k * ks + i);
            memcpy(t, &v, 16);
        } else {
            for (int q = 0; q < 8; ++q) t[q] = (k < K && i + q < n_r) ? X[(int64_t)k * ks + i + q] : (bf16)0;
        }
        for (int q = 0; q < 8; ++q) S[r + q][kk] = t[q];
        return;
    }
    for (int e = tid; e < 64 * 32; e += 256) {
        // the loop index runs along whichever dimension is contiguous in memory
        const bool kfast = ks == 1;
        const int r = kfast ? e >> 5 : e & 63, kk = kfast ? e & 31 : e >> 6;
        const int i = r0 + r, k = k0 + kk;
        S[r][kk] = (i < n_r && k < K) ? X[(int64_t)i * rs + (int64_t)k * ks] : (bf16)0;
    }
}

__global__ __launch_bounds__(256) void k_gemm(GemmArgs p) {
    __shared__ __align__(16) bf16 As[64][40];   // rows of 80 bytes: 16-byte aligned reads
    __shared__ __align__(16) bf16 Bs[64][40];
    __shared__ float red[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wr = wave >> 1, wc = wave & 1;
    const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;   // rows on x: up to 2^31 tiles
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    // 16-byte moves need 16-byte aligned bases and strides of the non-contiguous dimension
    const bool a_vec = ((uintptr_t)p.A & 15) == 0 && ((p.a_cs == 1 && p.a_rs % 8 == 0) || (p.a_rs == 1 && p.a_cs % 8 == 0));
    const bool b_vec = ((uintptr_t)p.B & 15) == 0 && ((p.b_rs == 1 && p.b_cs % 8 == 0) || (p.b_cs == 1 && p.b_rs % 8 == 0));
    for (int k0 = 0; k0 < p.K; k0 += 32) {
        stage_block(As, p.A, p.a_rs, p.a_cs, p.M, p.K, row0, k0, a_vec, tid);
        stage_block(Bs, p.B, p.b_cs, p.b_rs, p.N, p.K, col0, k0, b_vec, tid);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 32; kk += 16) {
            // lane l holds row (col) l % 32 and k = kk + 8 (l / 32) + 0..7
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wr * 32 + (lane & 31)][kk + (lane >> 5) * 8]);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[wc * 32 + (lane & 31)][kk + (lane >> 5) * 8]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    float lsum = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        // D[i][j] of the 32x32 block: i = 8 (r/4) + 4 (lane/32) + r%4, j = lane%32
        const int i = row0 + wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int j = col0 + wc * 32 + (lane & 31);
        if (i >= p.M || j >= p.N) continue;
        float v = acc[r];
        const int64_t fi = (int64_t)i * p.ld_f + j, hi = (int64_t)i * p.ld_h + j;
        switch (p.epi) {
            case EPI_F32:
                if (p.outf) p.outf[fi] = v;
                if (p.outh) p.outh[hi] = to_bf16(v);
                break;
            case EPI_BIAS:
                v += p.bias[j];
                if (p.outf) p.outf[fi] = v;
                if (p.outh) p.outh[hi] = to_bf16(v);
                break;
            case EPI_BIAS_GELU:
                v += p.bias[j];
                if (p.outf) p.outf[fi] = v;
                p.outh[hi] = to_bf16(gelu(v));
                break;
            case EPI_GELU_BWD:
                v *= gelu_grad(p.aux[fi]);
                if (p.outf) p.outf[fi] = v;
                p.outh[hi] = to_bf16(v);
                break;
            case EPI_PRED: {
                const float w = p.vec[i];
                v = w > 0.0f ? fmaxf(0.0f, v * p.scale * w) : 0.0f;
                if (p.prior && p.col_node[j] == i) v += p.prior[i];
                p.outf[fi] = v;
                break;
            }
            case EPI_LOSS: {
                // (p_hat - T)^2 / (T + tau) over the known targets (NaN: unknown)
                const float t = p.aux[(int64_t)i * p.N + j];
                float gk = 0.0f;
                if (isfinite(t)) {
                    const float w = p.vec[j];
                    const float wt = rsqrtf(fabsf(t) + p.sigma);
                    const int32_t nd = p.row_node[i];
                    const float pr = (p.prior && nd == p.col_node[j]) ? p.prior[nd] : 0.0f;
                    const float d = (v * p.scale * w + pr - t) * wt;
                    lsum += d * d;
                    gk = 2.0f * d * wt * p.inv_n * p.scale * w;
                }
                p.outh[hi] = to_bf16(gk);
                break;
            }
            default:
                break;
        }
    }
    if (p.epi == EPI_LOSS) {
        red[tid] = lsum;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0) p.loss_part[blockIdx.y * gridDim.x + blockIdx.x] = red[0];   // any fixed slot per tile
    }
}

void gemm(const GemmArgs& a, hipStream_t s) {
    dim3 grid((a.M + 63) / 64, (a.N + 63) / 64);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, a);
}

GemmArgs gemm_args(int M, int N, int K, const bf16* A, int64_t a_rs, int64_t a_cs, const bf16* B, int64_t b_rs,
                   int64_t b_cs, int epi) {
    GemmArgs g;
    memset(&g, 0, sizeof(g));
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.a_rs = a_rs; g.a_cs = a_cs;
    g.B = B; g.b_rs = b_rs; g.b_cs = b_cs;
    g.epi = epi;
    g.ld_f = N;
    g.ld_h = N;
    return g;
}

// Column sums of an FP32 [rows][cols] matrix (bias gradients) in a fixed
// order: block (b, c) sums rows b, b + kColSplit, ... of 64 columns with 4
// row-interleaved lanes per column into part[b][cols]; k_colsum_fin adds the
// kColSplit partials of each column in order.
constexpr int kColSplit = 32;

__global__ __launch_bounds__(256) void k_colsum(const float* X, int rows, int cols, float* part) {
    __shared__ float sh[4][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int j = blockIdx.y * 64 + c;
    float s = 0.0f;
    if (j < cols)
        for (int i = blockIdx.x + g * kColSplit; i < rows; i += 4 * kColSplit) s += X[(int64_t)i * cols + j];
    sh[g][c] = s;
    __syncthreads();
    if (g == 0 && j < cols) part[(int64_t)blockIdx.x * cols + j] = (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
}

__global__ void k_colsum_fin(const float* part, int cols, float* out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float s = 0.0f;
    for (int b = 0; b < kColSplit; ++b) s += part[(int64_t)b * cols + j];
    out[j] = s;
}

__global__ void k_gather_rows(const bf16* src, int width, const int32_t* idx, int n, bf16* dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * width) return;
    const int r = (int)(t / width), c = (int)(t % width);
    const int32_t i = idx[r];
    dst[t] = i >= 0 ? src[(int64_t)i * width + c] : (bf16)0;
}

__global__ void k_adam(float* theta, bf16* theta_h, const float* grad, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float t = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
    theta[i] = t;
    theta_h[i] = to_bf16(t);
}

__global__ void k_to_bf16(const float* x, int64_t n, bf16* y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = to_bf16(x[i]);
}

// ---------------------------------------------------------------------------
// Node features, one wave per U row (internal order), written to row
// out_row[x] of out (FP32, 64 per row); isolated rows are 0:
//   [0] 1, [1] ln(1+d(x))/8, [2] ln ws(x)/8,
//   [3] sum_v w(x,v)/ws(x) ln(1+d(v))/8,
//   [4+b] sum of w(x,v)/ws(x) over neighbours v whose external id hashes to b.
// Each lane sums its own entries into its own LDS column, then the lanes are
// added in a fixed order, so the result does not depend on timing.
// ---------------------------------------------------------------------------
__device__ inline int id_bucket(int32_t v_ext) {
    const uint32_t h = (uint32_t)((uint64_t)(uint32_t)v_ext * 0x9E3779B1ull);
    return (int)((h >> 16) % (uint32_t)kBuckets);
}

template <typename WT>
__global__ __launch_bounds__(256) void k_features(int32_t nu, const int64_t* rp_u, const int32_t* ci_u,
                                                  const WT* w_u, const int64_t* rp_v, const int32_t* iperm_v,
                                                  const double* inv_ws_u, const double* inv_ws_v,
                                                  const int32_t* out_row, float* out) {
    __shared__ float bins[4][kBuckets + 1][kWave];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int32_t x = blockIdx.x * 4 + wv;
    const bool valid = x < nu;
    for (int b = 0; b <= kBuckets; ++b) bins[wv][b][lane] = 0.0f;
    const int64_t e0 = valid ? rp_u[x] : 0, e1 = valid ? rp_u[x + 1] : 0;
    const double iwx = valid ? inv_ws_u[x] : 0.0;
    for (int64_t e = e0 + lane; e < e1; e += kWave) {
        const int32_t v = ci_u[e];
        const double w = (double)w_u[e] / inv_ws_v[v];       // w_u holds w(x,v)/ws(v)
        const float frac = (float)(w * iwx);
        const float dv = (float)(rp_v[v + 1] - rp_v[v]);
        bins[wv][id_bucket(iperm_v[v])][lane] += frac;
        bins[wv][kBuckets][lane] += frac * log1pf(dv) * 0.125f;
    }
    __syncthreads();   // lanes below read the columns of the other lanes
    if (!valid) return;
    float* o = out + (int64_t)out_row[x] * kIn;
    const int64_t d = e1 - e0;
    // lane b <= kBuckets adds bin b over the 64 lanes in order
    if (lane <= kBuckets) {
        float s = 0.0f;
        for (int l = 0; l < kWave; ++l) s += bins[wv][lane][l];
        if (lane < kBuckets) o[4 + lane] = d > 0 ? s : 0.0f;
        else o[3] = d > 0 ? s : 0.0f;
    }
    if (lane == 0) {
        o[0] = d > 0 ? 1.0f : 0.0f;
        o[1] = d > 0 ? (float)(log1p((double)d) * 0.125) : 0.0f;
        o[2] = d > 0 ? (float)(-log(iwx) * 0.125) : 0.0f;
    }
}

__global__ void k_identity(int32_t n, int32_t* out) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = i;
}

__global__ void k_ws_of(int32_t n, const double* inv_ws, float* ws) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ws[i] = inv_ws[i] > 0.0 ? (float)(1.0 / inv_ws[i]) : 0.0f;
}

// Structural self term of the prediction: the first two terms of the return
// series of Eq. (hpp), alpha + alpha (1-alpha) P(x,x), with
// P(x,x) = sum_v w(x,v)^2 / (ws(x) ws(v)) (Eq. (pmatrix)); one wavefront per row.
template <typename WT>
__global__ __launch_bounds__(256) void k_self_prior(int32_t nu, const int64_t* rp_u, const WT* w_u, const int32_t* ci_u,
                                                    const double* inv_ws_u, const double* inv_ws_v, double alpha,
                                                    float* out) {
    // one wavefront per row; lanes take strided entries, then a fixed tree
    const int lane = threadIdx.x & 63;
    const int32_t x = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (x >= nu) return;   // whole wavefront
    const int64_t e0 = rp_u[x], e1 = rp_u[x + 1];
    double s = 0.0;
    for (int64_t e = e0 + lane; e < e1; e += 64) {
        const double q = (double)w_u[e];                  // w(x,v)/ws(v)
        s += q * q / inv_ws_v[ci_u[e]];                   // w^2 / ws(v)
    }
    for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m);
    if (lane == 0) out[x] = e1 > e0 ? (float)(alpha + alpha * (1.0 - alpha) * s * inv_ws_u[x]) : 0.0f;
}

uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
double uniform01(uint64_t& s) { return (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace

// activations of one tower pass over `cap` rows
struct TowerBuf {
    int cap = 0;
    bf16* X = nullptr;                       // [cap][64]
    float* z1 = nullptr; bf16* a1 = nullptr; // [cap][256]
    float* z2 = nullptr; bf16* a2 = nullptr;
    float* z3 = nullptr; bf16* z3h = nullptr; // [cap][128]
    float* d3 = nullptr; bf16* d3h = nullptr; // gradients w.r.t. z3, z2, z1
    float* d2 = nullptr; bf16* d2h = nullptr;
    float* d1 = nullptr; bf16* d1h = nullptr;
};

struct Model {
    Graph* g = nullptr;
    hipStream_t s = nullptr;
    float* theta = nullptr;   // FP32 master parameters
    bf16* theta_h = nullptr;  // BF16 copy used by the kernels
    float* grad = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    int64_t t = 0;
    bf16* X = nullptr;        // [n_u][64] features, internal order
    float* ws = nullptr;      // [n_u] ws(x), internal order (0 for isolated)
    float* prior = nullptr;   // [n_u] structural self term, internal order
    std::vector<float> h_prior;
    bf16* Femb = nullptr;     // [n_u][128] tower f, internal order
    bf16* Gemb = nullptr;     // [n_u][128] tower g
    bool emb_valid = false;
    double c = 1.0, sigma = 1e-9;   // score scale c and the loss's tau
    TowerBuf tf, tg;
    bf16* dK = nullptr;       // [cap_u][cap_x]
    float* T = nullptr;       // [cap_u][cap_x] targets
    float* wsx = nullptr;     // [cap_x]
    int32_t* idx = nullptr;   // [cap_u + cap_x] batch rows (internal ids)
    float* loss_part = nullptr;
    int cap_u = 0, cap_x = 0;
    bf16* fsel = nullptr;     // [64][128] tower-f rows of the sources being predicted
    float* csum = nullptr;    // [kColSplit][256] partial column sums
    int32_t* d_rows = nullptr;
};

namespace {

void free_tower(TowerBuf& b) {
    void* p[] = {b.X, b.z1, b.a1, b.z2, b.a2, b.z3, b.z3h, b.d3, b.d3h, b.d2, b.d2h, b.d1, b.d1h};
    for (void* q : p) hipFree(q);
    b = TowerBuf{};
}

bhpp_status alloc_tower(TowerBuf& b, int cap) {
    if (b.cap >= cap) return BHPP_OK;
    free_tower(b);
    const size_t c = (size_t)cap;
    bool ok = hipMalloc((void**)&b.X, c * kIn * 2) == hipSuccess &&
              hipMalloc((void**)&b.z1, c * kHid * 4) == hipSuccess && hipMalloc((void**)&b.a1, c * kHid * 2) == hipSuccess &&
              hipMalloc((void**)&b.z2, c * kHid * 4) == hipSuccess && hipMalloc((void**)&b.a2, c * kHid * 2) == hipSuccess &&
              hipMalloc((void**)&b.z3, c * kOut * 4) == hipSuccess && hipMalloc((void**)&b.z3h, c * kOut * 2) == hipSuccess &&
              hipMalloc((void**)&b.d3, c * kOut * 4) == hipSuccess && hipMalloc((void**)&b.d3h, c * kOut * 2) == hipSuccess &&
              hipMalloc((void**)&b.d2, c * kHid * 4) == hipSuccess && hipMalloc((void**)&b.d2h, c * kHid * 2) == hipSuccess &&
              hipMalloc((void**)&b.d1, c * kHid * 4) == hipSuccess && hipMalloc((void**)&b.d1h, c * kHid * 2) == hipSuccess;
    if (!ok) {
        free_tower(b);
        (void)hipGetLastError();
        return BHPP_OUT_OF_MEMORY;
    }
    b.cap = cap;
    return BHPP_OK;
}

void colsum(const float* X, int rows, int cols, float* part, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3(kColSplit, (cols + 63) / 64), dim3(256), 0, s, X, rows, cols, part);
    hipLaunchKernelGGL(k_colsum_fin, dim3((cols + 127) / 128), dim3(128), 0, s, part, cols, out);
}

// forward pass of one tower over rows b.X[0..n): z3 (FP32) and z3h (BF16)
void tower_forward(const Model* m, int tower, TowerBuf& b, int n, hipStream_t s) {
    const bf16* P = m->theta_h + tower * kTower;
    const float* Pf = m->theta + tower * kTower;
    GemmArgs a = gemm_args(n, kHid, kIn, b.X, kIn, 1, P + kOffW1, kHid, 1, EPI_BIAS_GELU);
    a.bias = Pf + kOffB1; a.outf = b.z1; a.outh = b.a1;
    gemm(a, s);
    a = gemm_args(n, kHid, kHid, b.a1, kHid, 1, P + kOffW2, kHid, 1, EPI_BIAS_GELU);
    a.bias = Pf + kOffB2; a.outf = b.z2; a.outh = b.a2;
    gemm(a, s);
    a = gemm_args(n, kOut, kHid, b.a2, kHid, 1, P + kOffW3, kOut, 1, EPI_BIAS);
    a.bias = Pf + kOffB3; a.outf = b.z3; a.outh = b.z3h;
    gemm(a, s);
}

// backward pass of one tower from b.d3h / b.d3 (gradient w.r.t. z3) into grad
void tower_backward(Model* m, int tower, TowerBuf& b, int n, hipStream_t s) {
    const bf16* P = m->theta_h + tower * kTower;
    float* G = m->grad + tower * kTower;
    // W3: a2^T d3
    GemmArgs a = gemm_args(kHid, kOut, n, b.a2, 1, kHid, b.d3h, kOut, 1, EPI_F32);
    a.outf = G + kOffW3;
    gemm(a, s);
    colsum(b.d3, n, kOut, m->csum, G + kOffB3, s);
    // d2 = (d3 W3^T) * gelu'(z2)
    a = gemm_args(n, kHid, kOut, b.d3h, kOut, 1, P + kOffW3, 1, kOut, EPI_GELU_BWD);
    a.aux = b.z2; a.outf = b.d2; a.outh = b.d2h;
    gemm(a, s);
    a = gemm_args(kHid, kHid, n, b.a1, 1, kHid, b.d2h, kHid, 1, EPI_F32);
    a.outf = G + kOffW2;
    gemm(a, s);
    colsum(b.d2, n, kHid, m->csum, G + kOffB2, s);
    // d1 = (d2 W2^T) * gelu'(z1)
    a = gemm_args(n, kHid, kHid, b.d2h, kHid, 1, P + kOffW2, 1, kHid, EPI_GELU_BWD);
    a.aux = b.z1; a.outf = b.d1; a.outh = b.d1h;
    gemm(a, s);
    a = gemm_args(kIn, kHid, n, b.X, 1, kIn, b.d1h, kHid, 1, EPI_F32);
    a.outf = G + kOffW1;
    gemm(a, s);
    colsum(b.d1, n, kHid, m->csum, G + kOffB1, s);
}

bhpp_status ensure_batch(Model* m, int nu_b, int nx_b) {
    bhpp_status rc = alloc_tower(m->tf, std::max(nu_b, 64));
    if (rc) return rc;
    rc = alloc_tower(m->tg, std::max(nx_b, 64));
    if (rc) return rc;
    if (m->cap_u >= nu_b && m->cap_x >= nx_b) return BHPP_OK;
    hipFree(m->dK); hipFree(m->T); hipFree(m->wsx); hipFree(m->idx); hipFree(m->loss_part);
    const size_t cu = (size_t)std::max(nu_b, m->cap_u), cx = (size_t)std::max(nx_b, m->cap_x);
    const size_t tiles = ((cu + 63) / 64) * ((cx + 63) / 64);
    bool ok = hipMalloc((void**)&m->dK, cu * cx * 2) == hipSuccess && hipMalloc((void**)&m->T, cu * cx * 4) == hipSuccess &&
              hipMalloc((void**)&m->wsx, cx * 4) == hipSuccess && hipMalloc((void**)&m->idx, (cu + cx) * 4) == hipSuccess &&
              hipMalloc((void**)&m->loss_part, tiles * 4) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        m->cap_u = m->cap_x = 0;
        return BHPP_OUT_OF_MEMORY;
    }
    m->cap_u = (int)cu;
    m->cap_x = (int)cx;
    return BHPP_OK;
}

// One forward + backward over a batch: rows idx[0..nu_b) of the features feed
// tower f, rows idx[nu_b..nu_b+nx_b) tower g; targets T, ws of the candidates
// wsx (device, already uploaded). Leaves the gradient in m->grad and the loss
// partials in m->loss_part.
void batch_pass(Model* m, int nu_b, int nx_b, int64_t n_known, hipStream_t s) {
    const int64_t tot_f = (int64_t)nu_b * kIn, tot_g = (int64_t)nx_b * kIn;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((tot_f + 255) / 256)), dim3(256), 0, s, m->X, kIn, m->idx, nu_b,
                       m->tf.X);
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((tot_g + 255) / 256)), dim3(256), 0, s, m->X, kIn,
                       m->idx + nu_b, nx_b, m->tg.X);
    tower_forward(m, 0, m->tf, nu_b, s);
    tower_forward(m, 1, m->tg, nx_b, s);
    // p_hat = c ws(x_j) <f_i, g_j>, loss and dL/dK
    GemmArgs a = gemm_args(nu_b, nx_b, kOut, m->tf.z3h, kOut, 1, m->tg.z3h, 1, kOut, EPI_LOSS);
    a.aux = m->T; a.vec = m->wsx; a.scale = (float)m->c; a.sigma = (float)m->sigma;
    a.inv_n = 1.0f / (float)std::max<int64_t>(n_known, 1);
    a.outh = m->dK; a.ld_h = nx_b; a.loss_part = m->loss_part;
    a.prior = m->prior; a.row_node = m->idx; a.col_node = m->idx + nu_b;
    gemm(a, s);
    // dF = dK G, dG = dK^T F
    a = gemm_args(nu_b, kOut, nx_b, m->dK, nx_b, 1, m->tg.z3h, kOut, 1, EPI_F32);
    a.outf = m->tf.d3; a.outh = m->tf.d3h;
    gemm(a, s);
    a = gemm_args(nx_b, kOut, nu_b, m->dK, 1, nx_b, m->tf.z3h, kOut, 1, EPI_F32);
    a.outf = m->tg.d3; a.outh = m->tg.d3h;
    gemm(a, s);
    tower_backward(m, 0, m->tf, nu_b, s);
    tower_backward(m, 1, m->tg, nx_b, s);
}

int loss_tiles(int nu_b, int nx_b) { return ((nu_b + 63) / 64) * ((nx_b + 63) / 64); }

}  // namespace

void model_free(Model* m) {
    if (!m) return;
    if (m->s) hipStreamSynchronize(m->s);
    void* p[] = {m->theta, m->theta_h, m->grad, m->adam_m, m->adam_v, m->X, m->ws, m->prior, m->Femb, m->Gemb,
                 m->dK, m->T, m->wsx, m->idx, m->loss_part, m->fsel, m->d_rows, m->csum};
    for (void* q : p) hipFree(q);
    free_tower(m->tf);
    free_tower(m->tg);
    if (m->s) hipStreamDestroy(m->s);
    delete m;
}

int64_t model_num_params() { return kParams; }

// Features of every U node into out (FP32 [n_u][64]); ext_order: rows in the
// caller's ids, else internal order.
static bhpp_status compute_features(const Graph* g, float* out, bool ext_order, hipStream_t s) {
    int32_t* rows = nullptr;
    BHPP_HIP(hipMalloc((void**)&rows, sizeof(int32_t) * (size_t)g->nu));
    if (ext_order)
        BHPP_HIP(hipMemcpyAsync(rows, g->iperm_u, sizeof(int32_t) * (size_t)g->nu, hipMemcpyDeviceToDevice, s));
    else
        hipLaunchKernelGGL(k_identity, dim3((g->nu + 255) / 256), dim3(256), 0, s, g->nu, rows);
    BHPP_HIP(hipMemsetAsync(out, 0, sizeof(float) * (size_t)g->nu * kIn, s));
    const dim3 grid((g->nu + 3) / 4);
    if (g->dtype == BHPP_DTYPE_F64)
        hipLaunchKernelGGL(k_features<double>, grid, dim3(256), 0, s, g->nu, g->rp_u, g->ci_u, (const double*)g->w_u,
                           g->rp_v, g->iperm_v, g->inv_ws_u_d, g->inv_ws_v_d, rows, out);
    else
        hipLaunchKernelGGL(k_features<float>, grid, dim3(256), 0, s, g->nu, g->rp_u, g->ci_u, (const float*)g->w_u,
                           g->rp_v, g->iperm_v, g->inv_ws_u_d, g->inv_ws_v_d, rows, out);
    BHPP_HIP(hipGetLastError());
    BHPP_HIP(hipStreamSynchronize(s));
    hipFree(rows);
    return BHPP_OK;
}

bhpp_status model_features(Model* m, float* out_ext, hipStream_t s) { return compute_features(m->g, out_ext, true, s); }

bhpp_status model_create(Graph* g, uint64_t seed, Model** out) {
    Model* m = new (std::nothrow) Model();
    if (!m) return BHPP_OUT_OF_MEMORY;
    m->g = g;
    const size_t nu = (size_t)g->nu;
    bool ok = hipStreamCreateWithFlags(&m->s, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc((void**)&m->theta, kParams * 4) == hipSuccess &&
              hipMalloc((void**)&m->theta_h, kParams * 2) == hipSuccess &&
              hipMalloc((void**)&m->grad, kParams * 4) == hipSuccess &&
              hipMalloc((void**)&m->adam_m, kParams * 4) == hipSuccess &&
              hipMalloc((void**)&m->adam_v, kParams * 4) == hipSuccess &&
              hipMalloc((void**)&m->X, nu * kIn * 2) == hipSuccess && hipMalloc((void**)&m->ws, nu * 4) == hipSuccess &&
              hipMalloc((void**)&m->prior, nu * 4) == hipSuccess &&
              hipMalloc((void**)&m->Femb, nu * kOut * 2) == hipSuccess &&
              hipMalloc((void**)&m->Gemb, nu * kOut * 2) == hipSuccess &&
              hipMalloc((void**)&m->fsel, (size_t)kMaxCols * kOut * 2) == hipSuccess &&
              hipMalloc((void**)&m->d_rows, (size_t)kMaxCols * 4) == hipSuccess &&
              hipMalloc((void**)&m->csum, (size_t)kColSplit * kHid * 4) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        model_free(m);
        return BHPP_OUT_OF_MEMORY;
    }
    hipStream_t s = m->s;
    // features (internal order) -> BF16
    float* F = nullptr;
    if (hipMalloc((void**)&F, nu * kIn * 4) != hipSuccess) {
        (void)hipGetLastError();
        model_free(m);
        return BHPP_OUT_OF_MEMORY;
    }
    bhpp_status rc = compute_features(g, F, false, s);
    if (rc == BHPP_OK) {
        hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((nu * kIn + 255) / 256)), dim3(256), 0, s, F, (int64_t)(nu * kIn),
                           m->X);
        hipLaunchKernelGGL(k_ws_of, dim3((g->nu + 255) / 256), dim3(256), 0, s, g->nu, g->inv_ws_u_d, m->ws);
        if (g->dtype == BHPP_DTYPE_F64)
            hipLaunchKernelGGL(k_self_prior<double>, dim3((g->nu + 3) / 4), dim3(256), 0, s, g->nu, g->rp_u,
                               (const double*)g->w_u, g->ci_u, g->inv_ws_u_d, g->inv_ws_v_d, g->info.alpha, m->prior);
        else
            hipLaunchKernelGGL(k_self_prior<float>, dim3((g->nu + 3) / 4), dim3(256), 0, s, g->nu, g->rp_u,
                               (const float*)g->w_u, g->ci_u, g->inv_ws_u_d, g->inv_ws_v_d, g->info.alpha, m->prior);
        m->h_prior.resize(nu);
        if (hipMemcpyAsync(m->h_prior.data(), m->prior, 4 * nu, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = BHPP_DEVICE_ERROR;
    }
    hipFree(F);
    if (rc) {
        model_free(m);
        return rc;
    }
    // Glorot-uniform weights, zero biases (host RNG: splitmix64)
    std::vector<float> th((size_t)kParams, 0.0f);
    uint64_t st = seed;
    for (int tw = 0; tw < 2; ++tw) {
        const int64_t base = tw * kTower;
        const int64_t offs[3] = {kOffW1, kOffW2, kOffW3};
        const int fin[3] = {kIn, kHid, kHid}, fout[3] = {kHid, kHid, kOut};
        for (int l = 0; l < 3; ++l) {
            const double a = sqrt(6.0 / (double)(fin[l] + fout[l]));
            for (int64_t i = 0; i < (int64_t)fin[l] * fout[l]; ++i)
                th[base + offs[l] + i] = (float)((2.0 * uniform01(st) - 1.0) * a);
        }
    }
    // scale of the score: c = 1e-3 / mean ws over non-isolated nodes, so that
    // <f, g> of order 1 predicts pi of order 1e-3 at average ws
    double sum = 0.0;
    int64_t cnt = 0;
    for (double w : g->h_ws_u)
        if (w > 0.0) { sum += w; ++cnt; }
    m->c = cnt > 0 ? 1e-3 / (sum / (double)cnt) : 1.0;
    // tau of the loss weight 1/(T + tau): far below the average pi(u, x) = 1/|U|
    m->sigma = cnt > 0 ? 1e-3 / (double)cnt : 1e-9;
    rc = model_set_params(m, th.data());
    if (rc) {
        model_free(m);
        return rc;
    }
    *out = m;
    return BHPP_OK;
}

bhpp_status model_set_params(Model* m, const float* host) {
    hipStream_t s = m->s;
    BHPP_HIP(hipMemcpyAsync(m->theta, host, kParams * 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, s, m->theta, kParams,
                       m->theta_h);
    BHPP_HIP(hipMemsetAsync(m->adam_m, 0, kParams * 4, s));
    BHPP_HIP(hipMemsetAsync(m->adam_v, 0, kParams * 4, s));
    BHPP_HIP(hipStreamSynchronize(s));
    m->t = 0;
    m->emb_valid = false;
    return BHPP_OK;
}

bhpp_status model_get_params(Model* m, float* host) {
    BHPP_HIP(hipMemcpy(host, m->theta, kParams * 4, hipMemcpyDeviceToHost));
    return BHPP_OK;
}

void model_scales(const Model* m, double* c, double* sigma) {
    *c = m->c;
    *sigma = m->sigma;
}

// Upload one batch: source rows, candidate rows (internal ids), targets and
// candidate ws.
static bhpp_status upload_batch(Model* m, const std::vector<int32_t>& rows_u, const std::vector<int32_t>& rows_x,
                                const std::vector<float>& T, const std::vector<float>& wsx) {
    hipStream_t s = m->s;
    const int nu_b = (int)rows_u.size(), nx_b = (int)rows_x.size();
    bhpp_status rc = ensure_batch(m, nu_b, nx_b);
    if (rc) return rc;
    BHPP_HIP(hipMemcpyAsync(m->idx, rows_u.data(), 4 * (size_t)nu_b, hipMemcpyHostToDevice, s));
    BHPP_HIP(hipMemcpyAsync(m->idx + nu_b, rows_x.data(), 4 * (size_t)nx_b, hipMemcpyHostToDevice, s));
    BHPP_HIP(hipMemcpyAsync(m->T, T.data(), 4 * T.size(), hipMemcpyHostToDevice, s));
    BHPP_HIP(hipMemcpyAsync(m->wsx, wsx.data(), 4 * wsx.size(), hipMemcpyHostToDevice, s));
    return BHPP_OK;
}

static bhpp_status read_loss(Model* m, int nu_b, int nx_b, int64_t n_known, double* loss) {
    std::vector<float> lp((size_t)loss_tiles(nu_b, nx_b));
    BHPP_HIP(hipMemcpyAsync(lp.data(), m->loss_part, 4 * lp.size(), hipMemcpyDeviceToHost, m->s));
    BHPP_HIP(hipStreamSynchronize(m->s));
    double l = 0.0;
    for (float v : lp) l += v;
    *loss = l / (double)std::max<int64_t>(n_known, 1);
    return BHPP_OK;
}

static int64_t count_known(const std::vector<float>& T) {
    int64_t n = 0;
    for (float t : T) n += std::isfinite(t) ? 1 : 0;
    return n;
}

bhpp_status model_loss_grad(Model* m, int n_src, const int32_t* src, int n_cand, const int32_t* cand,
                            const float* target, double* loss, float* grad_host) {
    const Graph* g = m->g;
    std::vector<int32_t> ru(n_src), rx(n_cand);
    std::vector<float> wsx(n_cand), T((size_t)n_src * n_cand);
    for (int i = 0; i < n_src; ++i) ru[i] = g->h_perm_u[src[i]];
    for (int j = 0; j < n_cand; ++j) {
        rx[j] = g->h_perm_u[cand[j]];
        wsx[j] = (float)g->h_ws_u[cand[j]];
    }
    memcpy(T.data(), target, 4 * T.size());
    const int64_t nk = count_known(T);
    if (nk == 0) return BHPP_INVALID_ARG;
    bhpp_status rc = upload_batch(m, ru, rx, T, wsx);
    if (rc) return rc;
    batch_pass(m, n_src, n_cand, nk, m->s);
    BHPP_HIP(hipGetLastError());
    rc = read_loss(m, n_src, n_cand, nk, loss);
    if (rc) return rc;
    if (grad_host) BHPP_HIP(hipMemcpy(grad_host, m->grad, kParams * 4, hipMemcpyDeviceToHost));
    return BHPP_OK;
}

// Training on lists of BHPP values from the plain path: ids[i][*] (caller
// ids, -1 for none) and vals[i][*] = beta'(src_i, x), e.g. the top entries of
// each vector plus entries at random nodes (the far field). The target of a
// listed pair is pi(u, x) = beta'(u, x) ws(x) / (ws(u) + ws(x)) (Lemma 3);
// pairs that are not listed are unknown and left out of the loss. Each step
// takes batch_src random sources and, as candidates, their listed nodes (at
// most batch_cand).
bhpp_status model_train(Model* m, int n_src, const int32_t* src, int M, const int32_t* ids, const float* vals,
                        int steps, int batch_src, int batch_cand, double lr, uint64_t seed, float* loss_out) {
    const Graph* g = m->g;
    const int32_t nu = g->nu;
    std::vector<std::unordered_map<int32_t, float>> tgt((size_t)n_src);
    for (int i = 0; i < n_src; ++i) {
        const double wu = g->h_ws_u[src[i]];
        tgt[i].reserve((size_t)M * 2);
        for (int j = 0; j < M; ++j) {
            const int32_t x = ids[(size_t)i * M + j];
            if (x < 0 || x >= nu) continue;
            const double wx = g->h_ws_u[x];
            if (!(wx > 0.0)) continue;
            tgt[i][x] = (float)((double)vals[(size_t)i * M + j] * wx / (wu + wx));
        }
    }
    std::vector<int32_t> mark((size_t)nu, -1);
    uint64_t st = seed;
    std::vector<int32_t> bsrc, cand, ru, rx;
    std::vector<float> T, wsx;
    const float nan = std::numeric_limits<float>::quiet_NaN();
    for (int step = 0; step < steps; ++step) {
        bsrc.clear();
        cand.clear();
        for (int i = 0; i < batch_src; ++i) bsrc.push_back((int32_t)(splitmix(st) % (uint64_t)n_src));
        for (int32_t i : bsrc)
            for (const auto& kv : tgt[i])
                if ((int)cand.size() < batch_cand && mark[kv.first] != step) {
                    mark[kv.first] = step;
                    cand.push_back(kv.first);
                }
        const int nx_b = (int)cand.size();
        if (nx_b == 0) return BHPP_INVALID_ARG;
        ru.resize(batch_src);
        rx.resize(nx_b);
        wsx.resize(nx_b);
        T.assign((size_t)batch_src * nx_b, nan);
        for (int i = 0; i < batch_src; ++i) ru[i] = g->h_perm_u[src[bsrc[i]]];
        for (int j = 0; j < nx_b; ++j) {
            rx[j] = g->h_perm_u[cand[j]];
            wsx[j] = (float)g->h_ws_u[cand[j]];
        }
        for (int i = 0; i < batch_src; ++i) {
            const auto& mp = tgt[bsrc[i]];
            for (int j = 0; j < nx_b; ++j) {
                auto it = mp.find(cand[j]);
                if (it != mp.end()) T[(size_t)i * nx_b + j] = it->second;
            }
        }
        const int64_t nk = count_known(T);
        bhpp_status rc = upload_batch(m, ru, rx, T, wsx);
        if (rc) return rc;
        batch_pass(m, batch_src, nx_b, nk, m->s);
        m->t += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - powf(b1, (float)m->t), c2 = 1.0f - powf(b2, (float)m->t);
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, m->s, m->theta, m->theta_h,
                           m->grad, m->adam_m, m->adam_v, kParams, (float)lr, b1, b2, c1, c2);
        BHPP_HIP(hipGetLastError());
        double l = 0.0;
        rc = read_loss(m, batch_src, nx_b, nk, &l);   // also keeps the host buffers free for the next step
        if (rc) return rc;
        if (loss_out) loss_out[step] = (float)l;
    }
    m->emb_valid = false;
    return BHPP_OK;
}

// Embeddings of every U node by both towers (internal order).
bhpp_status model_embed(Model* m) {
    const Graph* g = m->g;
    hipStream_t s = m->s;
    bhpp_status rc = alloc_tower(m->tf, kEmbedChunk);
    if (rc) return rc;
    std::vector<int32_t> rows(kEmbedChunk);
    int32_t* d_idx = nullptr;
    BHPP_HIP(hipMalloc((void**)&d_idx, 4 * (size_t)kEmbedChunk));
    for (int tw = 0; tw < 2 && rc == BHPP_OK; ++tw) {
        bf16* dst = tw == 0 ? m->Femb : m->Gemb;
        for (int32_t r0 = 0; r0 < g->nu; r0 += kEmbedChunk) {
            const int n = std::min(kEmbedChunk, g->nu - r0);
            for (int i = 0; i < n; ++i) rows[i] = r0 + i;
            if (hipMemcpyAsync(d_idx, rows.data(), 4 * (size_t)n, hipMemcpyHostToDevice, s) != hipSuccess) {
                rc = BHPP_DEVICE_ERROR;
                break;
            }
            const int64_t tot = (int64_t)n * kIn;
            hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m->X, kIn, d_idx, n,
                               m->tf.X);
            tower_forward(m, tw, m->tf, n, s);
            if (hipMemcpyAsync(dst + (size_t)r0 * kOut, m->tf.z3h, 2 * (size_t)n * kOut, hipMemcpyDeviceToDevice, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {   // rows[] is reused by the next chunk
                rc = BHPP_DEVICE_ERROR;
                break;
            }
        }
    }
    hipFree(d_idx);
    if (rc == BHPP_OK) m->emb_valid = true;
    return rc;
}

bool model_ready(const Model* m) { return m && m->emb_valid; }

// Predictions for up to 64 sources (internal rows src_rows[0..m)):
// out[x][j] = max(0, c ws(x) <F[src_j], G[x]>) for every internal x, in an
// [n_u][cols] FP32 array (columns j >= m are 0). Runs on stream s.
bhpp_status model_predict(Model* m, const int32_t* src_rows_host, int n, int cols, float* out, hipStream_t s) {
    if (!m->emb_valid || n > kMaxCols || cols > kMaxCols || n > cols) return BHPP_INVALID_ARG;
    std::vector<int32_t> r((size_t)kMaxCols, -1);
    for (int j = 0; j < n; ++j) r[j] = src_rows_host[j];
    BHPP_HIP(hipMemcpyAsync(m->d_rows, r.data(), 4 * (size_t)kMaxCols, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_gather_rows, dim3((kMaxCols * kOut + 255) / 256), dim3(256), 0, s, m->Femb, kOut, m->d_rows,
                       kMaxCols, m->fsel);
    GemmArgs a = gemm_args(m->g->nu, cols, kOut, m->Gemb, kOut, 1, m->fsel, 1, kOut, EPI_PRED);
    a.vec = m->ws;
    a.scale = (float)m->c;
    a.prior = m->prior;
    a.col_node = m->d_rows;
    a.outf = out;
    a.ld_f = cols;
    gemm(a, s);
    BHPP_HIP(hipGetLastError());
    // the host array r must stay valid until the copy has run
    BHPP_HIP(hipStreamSynchronize(s));
    return BHPP_OK;
}

// Predictions in caller ids: out[j][x] = tmp[perm_u[x]][j] for j < m.
__global__ void k_pred_rows(const float* tmp, int cols, int m, const int32_t* perm, int32_t nu, float* out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)m * nu) return;
    const int j = (int)(i / nu);
    const int32_t x = (int32_t)(i % nu);
    out[i] = tmp[(size_t)perm[x] * cols + j];
}

// The start the model gives each source (caller ids): out[i][x] = p_hat(src_i, x).
bhpp_status model_predict_ext(Model* m, int n, const int32_t* src_ext, float* out, hipStream_t s) {
    if (!m->emb_valid) return BHPP_INVALID_ARG;
    Graph* g = m->g;
    float* tmp = nullptr;
    if (hipMalloc((void**)&tmp, (size_t)g->nu * kMaxCols * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        return BHPP_OUT_OF_MEMORY;
    }
    bhpp_status rc = BHPP_OK;
    for (int i0 = 0; i0 < n && rc == BHPP_OK; i0 += kMaxCols) {
        const int c = n - i0 < kMaxCols ? n - i0 : kMaxCols;
        std::vector<int32_t> rows(c);
        for (int j = 0; j < c; ++j) rows[j] = g->h_perm_u[src_ext[i0 + j]];
        rc = model_predict(m, rows.data(), c, kMaxCols, tmp, s);
        if (rc) break;
        const size_t tot = (size_t)c * g->nu;
        hipLaunchKernelGGL(k_pred_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, tmp, kMaxCols, c,
                           g->perm_u, g->nu, out + (size_t)i0 * g->nu);
        if (hipGetLastError() != hipSuccess) rc = BHPP_DEVICE_ERROR;
    }
    if (hipStreamSynchronize(s) != hipSuccess && rc == BHPP_OK) rc = BHPP_DEVICE_ERROR;
    hipFree(tmp);
    return rc;
}

// Raw GEMM for the layout test: C = A B with A [M][K], B [K][N] BF16 (device),
// C FP32 [M][N]; trans_a / trans_b read A as [K][M] / B as [N][K].
bhpp_status gemm_test(int M, int N, int K, const uint16_t* A, int trans_a, const uint16_t* B, int trans_b, float* C,
                      hipStream_t s) {
    GemmArgs a = gemm_args(M, N, K, A, trans_a ? 1 : K, trans_a ? M : 1, B, trans_b ? 1 : N, trans_b ? K : 1, EPI_F32);
    a.outf = C;
    gemm(a, s);
    BHPP_HIP(hipGetLastError());
    return BHPP_OK;
}

}  // namespace bhpp
