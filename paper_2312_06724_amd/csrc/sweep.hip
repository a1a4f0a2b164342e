// Two-hop sweep kernels and device-side phase control for Approx-BHPP.
//
// Coordinates. The kernels keep, per source u and node x in U, the forward
// residue y(x) = ws(x)/ws(u) * r(x) (Eq. (fresidue)) instead of the backward
// residue r of Algorithms 2-3. By Lemma 3 a backward push of r is the same
// operation as a forward push of y (Eq. (bwd2fwd)), so one array serves
// SS-Push, PI-Push and PowerIteration, and only the push rule changes:
//   SS-Push:   push x iff r(x) > eps_b        <=> y(x)/ws(x) > eps_b/ws(u)
//   PI-Push:   push x iff r(x) > ws(u)/ws(x) eps_f/lambda <=> y(x) > eps_f/lambda
//   sequential pushes and PowerIteration: push every x with y(x) > 0.
// Pushing a set S (Algorithm 2, one iteration): ACC(x) += alpha y(x) for x in
// S, then y <- y - y_S + (1-alpha) y_S P with P = D_U^-1 W D_V^-1 W^T. ACC
// then equals pi_f = ws/ws(u) pi_b (Eq. (fppr)); at the end it is converted to
// beta' = pi_f + pi_b = ACC (1 + ws(u)/ws(x)) plus the PowerIteration part
// (Algorithm 5). PowerIteration(y, t) (Algorithm 1) is t pushes of every node
// followed by ACC += alpha y: alpha sum_{l<=t} (1-alpha)^l y P^l.
//
// One sweep (one iteration of Algorithm 2's loop) is:
//   gather A (rows v of W^T): Q(v) = (1-alpha)/ws(v) * sum_x w(x,v) y_S(x)/ws(x)
//   gather B (rows x of W):   G(x) = sum_v w(x,v) Q(v)
//   update (rows x of U):     y(x) <- y(x) - y_S(x) + G(x), ACC(x) += alpha y_S(x),
//                             and the per-source reductions the phase control needs
//   control (one block per source): the tests of Algorithms 3-4.
// Up to 64 sources run together; source c of a block occupies column c of the
// node-major arrays Y[n_u][C], ACC[n_u][C], G[n_u][C], Q[n_v][C], so one
// adjacency entry feeds C lanes with one contiguous load. The gathers contain
// no loads besides the row gathers inside their inner loop (row metadata is
// loaded per chunk of entries), so the row gathers stay in flight.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include <deque>
#include <new>

#include "common.h"

namespace bhpp {

// ---------------------------------------------------------------------------
// launch geometry
// ---------------------------------------------------------------------------
constexpr int kWavesPerBlock = kPassThreads / kWave;
constexpr int kFixThreads = 1024;   // split-row fix-ups: 16 slot groups of 64 columns
constexpr int kMaxPassBlocks = 2048;
constexpr int kMaxFixBlocks = 1024;
constexpr int kUpdateBlocks = 2048;
constexpr int kUpdateBlocks1 = 512;   // one-column blocks: 1/64 of the work, fewer partial sums

struct Geometry {
    int blkA, blkFA, blkB, blkFB, blkU, blkU1, blkBU;
    // reduction slots: gather A, fix-up A, then the update's: k_update's blocks,
    // or (update fused into gather B) gather B's blocks followed by its fix-up's
    int offA, offFA, offU, n_part;
};

// Partial-sum slots of the U-side split rows (tiles_u and tiles_uf split the
// same rows into the same pieces).
static int32_t slots_u(const Graph* g) { return std::max(g->tiles_u.n_slots, g->tiles_uf.n_slots); }

static Geometry geometry(const Graph* g) {
    Geometry G;
    auto clampi = [](long v, int lo, int hi) { return (int)(v < lo ? lo : (v > hi ? hi : v)); };
    G.blkA = clampi((g->tiles_v.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock, 1, kMaxPassBlocks);
    G.blkB = clampi((g->tiles_u.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock, 1, kMaxPassBlocks);
    G.blkFA = clampi(g->tiles_v.n_split, 1, kMaxFixBlocks);
    G.blkFB = clampi(g->tiles_u.n_split, 1, kMaxFixBlocks);
    G.blkU = kUpdateBlocks;
    G.blkU1 = kUpdateBlocks1;
    G.blkBU = clampi((g->tiles_uf.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock, 1, kMaxPassBlocks);
    G.offA = 0;
    G.offFA = G.blkA;
    G.offU = G.offFA + G.blkFA;
    G.n_part = G.offU + std::max(G.blkU, G.blkBU + G.blkFB);
    return G;
}

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
// Sum `v` over the lanes of the block that serve the same column and store
// it at out[col * n_part + slot] (fixed order, so results are deterministic).
template <int COLS, int NW = kWavesPerBlock>
__device__ __forceinline__ void block_column_sum(double v, double* sh, double* out, int n_part, int slot) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int m = COLS; m < kWave; m <<= 1) v += __shfl_xor(v, m);
    sh[wid * kWave + lane] = v;
    __syncthreads();
    if ((int)threadIdx.x < COLS) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += sh[w * kWave + threadIdx.x];
        out[(size_t)threadIdx.x * n_part + slot] = s;
    }
    __syncthreads();
}

// Broadcast lane j's value to the whole wavefront (j uniform).
__device__ __forceinline__ int32_t rl(int32_t v, int j) { return __builtin_amdgcn_readlane(v, j); }
// Word 3 of a buffer resource for untyped 32-bit accesses (data format 32) on
// this GPU family; the base, a zero stride and the byte size fill the rest.
constexpr int kRawBufferFlags = 0x00020000;
__device__ __forceinline__ float rl(float v, int j) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j)); }
__device__ __forceinline__ int64_t rl(int64_t v, int j) {
    const int32_t lo = __builtin_amdgcn_readlane((int32_t)(v & 0xFFFFFFFF), j);
    const int32_t hi = __builtin_amdgcn_readlane((int32_t)(v >> 32), j);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double rl(double v, int j) { return __longlong_as_double(rl((int64_t)__double_as_longlong(v), j)); }

// Index of the calling wavefront in its block, as a wave-uniform (scalar)
// value: tile indices derived from it then stay in scalar registers, so the
// per-entry bounds tests are scalar branches instead of exec-masked regions.
__device__ __forceinline__ int wave_in_block() { return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); }

// A work tile read by a whole wavefront, broadcast from lane 0 so that its
// fields are known to be wave-uniform (the loads themselves may be vector
// loads, since the kernels also store to memory).
__device__ __forceinline__ Tile load_tile(const Tile* tiles, int t) {
    const Tile T = tiles[t];
    Tile U;
    U.row_begin = __builtin_amdgcn_readfirstlane(T.row_begin);
    U.row_end = __builtin_amdgcn_readfirstlane(T.row_end);
    U.e_begin = rl(T.e_begin, 0);
    U.e_end = rl(T.e_end, 0);
    U.slot = __builtin_amdgcn_readfirstlane(T.slot);
    U.epar_log2 = __builtin_amdgcn_readfirstlane(T.epar_log2);
    return U;
}

// DPP move of v from another lane (0 where the source is outside the row or
// the destination row is masked off): CTRL 0x111..0x118 shift right within a
// row of 16 lanes, 0x142 broadcasts lane 15 of each row to the next row,
// 0x143 broadcasts lane 31 to rows 2 and 3.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_mov(double v) {
    const int64_t b = __double_as_longlong(v);
    const int32_t lo = __builtin_amdgcn_update_dpp(0, (int32_t)(b & 0xFFFFFFFF), CTRL, ROWS, 0xF, true);
    const int32_t hi = __builtin_amdgcn_update_dpp(0, (int32_t)(b >> 32), CTRL, ROWS, 0xF, true);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Segmented inclusive sum across the wavefront: lane L returns the sum of
// lanes start..L (start <= L is the first lane of L's segment), added in a
// fixed order. Hillis-Steele steps of 1, 2, 4 and 8 lanes inside each row of
// 16, then the lane-15 and lane-31 broadcasts carry row totals across rows;
// every step adds only a source lane of the same segment.
template <typename VT>
__device__ __forceinline__ VT segmented_sum(VT v, int lane, int start) {
    const int lr = lane & 15;
    VT t;
    t = dpp_mov<0x111, 0xF>(v);
    if (lr >= 1 && lane - 1 >= start) v += t;
    t = dpp_mov<0x112, 0xF>(v);
    if (lr >= 2 && lane - 2 >= start) v += t;
    t = dpp_mov<0x114, 0xF>(v);
    if (lr >= 4 && lane - 4 >= start) v += t;
    t = dpp_mov<0x118, 0xF>(v);
    if (lr >= 8 && lane - 8 >= start) v += t;
    t = dpp_mov<0x142, 0xA>(v);                       // rows 1 and 3 take lanes 15 and 47
    if ((lane & 16) && start <= (lane & ~15) - 1) v += t;
    t = dpp_mov<0x143, 0xC>(v);                       // rows 2 and 3 take lane 31
    if ((lane & 32) && start <= 31) v += t;
    return v;
}

template <typename T>
__device__ __forceinline__ T ld_nt(const T* p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_nt(T* p, T v) { __builtin_nontemporal_store(v, p); }

template <typename VT, typename WT>
struct GatherArgs {
    const Tile* tiles;
    int n_tiles;
    const int64_t* rp;
    const int32_t* ci;
    const WT* w;            // gather A: w(x,v); gather B: w(x,v)/ws(v)
    const VT* X;            // gathered vector: gather A S (over U), gather B Q (over V)
    VT* OUT;                // gather A: Q, gather B: G
    VT* part;               // split-row partial sums [slots][COLS]
    const uint64_t* end_bits;  // bit e set iff entry e is the last of its row
    const int32_t* n_active;
    double* red;            // [kNumRed][COLS][n_part]
    int n_part;
    int red_slot;           // first reduction slot of this launch
    int nt_stream;          // stream adjacency and row outputs past the caches
    // k_gather64, gather A: when Yf is set the gather applies the push rule
    // itself, S(x) = y(x)/ws(x) for the pushed x, reading Y, 1/ws of each
    // entry's neighbour (iwf, stored beside the adjacency so that it arrives
    // with the indices) and the column states (stf) instead of a selected copy
    // S; a column that starts a query in this sweep (lazy reset, or PISP's
    // residue restart) takes y = e_src instead of its Y
    const VT* Yf = nullptr;
    const VT* iwf = nullptr;     // per adjacency entry, beside ci and w
    const ColState* stf = nullptr;
    // k_gather1: length of X and how many of its leading entries each block
    // stages in LDS (nodes are numbered by decreasing degree, so the first
    // entries are the hubs most adjacency entries point at); 0: none
    int32_t n_x = 0;
    int32_t hub = 0;
    // k_gather64 / k_fixup, gather B with the update fused (64 columns): the
    // row sums stay on chip and the update of those rows follows, as k_update
    // does it, with its reductions in the slots from red_slot
    VT* Yu = nullptr;
    VT* ACCu = nullptr;
    VT* SNAPu = nullptr;
    const VT* iwu = nullptr;       // 1/ws of the U rows
    const int32_t* degu = nullptr;
    const ColState* stu = nullptr;
};

// ---------------------------------------------------------------------------
// Update of one U row and column (k_update, and gather B with the update
// fused): the push of x decided by ruleB (ACC += alpha y, y = 0), the
// conversion of ACC the control asks for, y += (1-alpha) G, and the per-source
// reductions. Both kernels call apply() with the same operands, so they
// produce the same bits.
// ---------------------------------------------------------------------------
template <typename VT>
struct UpdateRule {
    PushTest<VT> test;
    VT kss, kpi, ws_src, alpha, oma;
    int convert;
    bool warm, snap, fresh, y_src;
    int32_t src_row;
    // has_snap: the block has a SNAP array (the host never marks a column
    // warm in a block without one; the check only keeps a slip in bounds)
    __device__ __forceinline__ UpdateRule(const ColState& cs, bool has_snap)
        : test(cs.ruleB, (VT)cs.k_ss, (VT)cs.k_pi) {
        convert = cs.convert;
        warm = cs.warm != 0 && has_snap;   // combine with pi_b as SS-Push left it
        snap = warm && cs.snap != 0;
        kss = (VT)cs.k_ss;
        kpi = (VT)cs.k_pi;
        ws_src = (VT)cs.ws_src;
        alpha = (VT)cs.alpha;
        oma = VT(1) - alpha;
        fresh = cs.fresh != 0;
        y_src = fresh || cs.reset_y != 0;   // y = e_src this sweep (ACC kept unless fresh)
        src_row = cs.src_row;
    }
    // y and ACC of row x as this sweep reads them (a new query: y = e_src, ACC = 0)
    __device__ __forceinline__ VT y_of(const VT* Y, size_t i, int32_t x) const {
        return y_src ? (x == src_row ? VT(1) : VT(0)) : Y[i];
    }
    __device__ __forceinline__ VT acc_of(const VT* ACC, size_t i) const { return fresh ? VT(0) : ACC[i]; }
    __device__ __forceinline__ void apply(VT y, VT a, VT g, VT iw, int32_t d, size_t i, VT* Y, VT* ACC, VT* SNAP,
                                          double* r) const {
        const VT yw = y * iw;
        const bool sel = test(fabs(y), fabs(yw));
        const VT s = sel ? y : VT(0);
        VT acc = a;
        if (snap) SNAP[i] = acc;                              // forward image of pi_b when SS-Push returned
        if (convert == 1) {
            // Eq. (fppr) plus the backward part of Alg. 5's combine: ACC -> beta' part
            if (warm) acc = acc + ws_src * iw * (snap ? acc : SNAP[i]);
            else acc = acc * (VT(1) + ws_src * iw);
        } else if (convert == 3) {
            acc = acc * ws_src * iw;   // SS-Push alone: the forward image back to pi_b(x) ~ pi(x, u)
        }                              // convert == 2 (PI-Push alone): ACC already holds pi_f's part
        acc += alpha * s;
        const VT yn = (y - s) + oma * g;
        Y[i] = yn;
        ACC[i] = acc;
        const VT tn = fabs(yn * iw), ya = fabs(yn);
        r[RED_NP] += sel ? (double)d : 0.0;
        r[RED_CNT_SS] += (tn > kss) ? 1.0 : 0.0;
        r[RED_SUM_R] += (double)tn;
        r[RED_CNT_PI] += (ya > kpi) ? 1.0 : 0.0;
        r[RED_SUM_Y] += (double)ya;
    }
};

// Columns of a block in use: n_active[1] (0: all). A batch keeps its running
// sources in the low columns, so lanes at or past the bound skip their loads
// and stores (a 64-wide row read of 32 columns fetches one 128-byte line).
__device__ __forceinline__ int live_cols(const int32_t* n_active, int cols) {
    const int c = n_active[1];
    return c > 0 && c < cols ? c : cols;
}

// Gather A (rows v of W^T) forms Q(v) = sum_x w(x,v) S(x) with S(x) = y(x)/ws(x)
// for the pushed x and 0 otherwise; gather B (rows x of W) forms
// G(x) = sum_v w(x,v)/ws(v) Q(v); the update then adds (1-alpha) G(x). Both are
// the same weighted gather; gather A also counts the push cost of the V side:
// d(v) for every v with a pushed neighbour, i.e. Q(v) > 0 (each pushed
// neighbour adds a positive term).

// ---------------------------------------------------------------------------
// Gathers for 2..32 sources: a wavefront takes a tile; lanes are (row group,
// edge slot, column); rows of a tile have similar degree (degree order), so
// the edge slots per row follow the tile's largest degree.
// ---------------------------------------------------------------------------
template <int COLS, typename VT, typename WT, bool SIDE_A>
__global__ __launch_bounds__(kPassThreads) void k_gather(GatherArgs<VT, WT> p) {
    __shared__ double sh[kPassThreads];
    if (*p.n_active == 0) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = wave_in_block();
    const int col = lane & (COLS - 1);
    double np = 0.0;
    const int n_waves = gridDim.x * kWavesPerBlock;
    for (int t = blockIdx.x * kWavesPerBlock + wid; t < p.n_tiles; t += n_waves) {
        const Tile T = load_tile(p.tiles, t);
        const int epar = min(1 << T.epar_log2, kWave / COLS);
        const int gl = epar * COLS;            // lanes per row
        const int ngroups = kWave / gl;
        const int grp = lane / gl;
        const int slot = (lane % gl) / COLS;
        for (int r0 = T.row_begin; r0 < T.row_end; r0 += ngroups) {
            const int row = r0 + grp;
            const bool valid = row < T.row_end;
            int64_t e0 = 0, e1 = 0;
            if (T.slot >= 0) {
                e0 = T.e_begin;
                e1 = T.e_end;
            } else if (valid) {
                e0 = p.rp[row];
                e1 = p.rp[row + 1];
            }
            VT acc = VT(0);
#pragma unroll 4
            for (int64_t e = e0 + slot; e < e1; e += epar)
                acc += (VT)p.w[e] * p.X[(size_t)p.ci[e] * COLS + col];
#pragma unroll
            for (int m = COLS; m < kWave; m <<= 1)
                if (m < gl) acc += __shfl_xor(acc, m);
            if (slot == 0 && valid) {
                if (T.slot >= 0) {
                    p.part[(size_t)T.slot * COLS + col] = acc;
                } else {
                    p.OUT[(size_t)row * COLS + col] = acc;
                    if (SIDE_A && acc != VT(0)) np += (double)(e1 - e0);
                }
            }
        }
    }
    if (SIDE_A) block_column_sum<COLS>(np, sh, p.red + (size_t)RED_NP * COLS * p.n_part, p.n_part,
                                       p.red_slot + blockIdx.x);
}

// ---------------------------------------------------------------------------
// Gather for 64 sources: one lane per source, one row at a time. Per chunk of
// 64 adjacency entries the wavefront loads, one entry or row per lane, the
// neighbour ids, weights and the end offsets of the next 64 rows; it then
// keeps INF row gathers in flight, taking each entry's neighbour id from its
// lane with readlane. A row whose last entry is reached is flushed with a
// store. Tiles hold no empty rows. Tile bounds, chunk sizes and row ends are
// wave-uniform (scalar registers); the live-column mask only guards the
// stores.
// ---------------------------------------------------------------------------
template <typename VT, typename WT>
struct Gather64State {
    int row;          // current output row
    int rend;         // its end, relative to the chunk start (> 64: later chunk)
    int64_t rbeg;     // its first entry
    VT acc;           // this lane's partial sum of the row
    double np;        // this lane's push cost (gather A)
};

// One chunk of n entries starting at cb. FULL: n == 64, so no entry needs a
// bounds test; otherwise loads past n re-read entry n-1 and are not used.
// UPD: whole rows go to this wavefront's LDS rows (lrow, row st.row at
// (st.row - T.row_begin) * 64) for the update at the end of the tile.
// BUF (FP32): the row reads are buffer loads through xr (X as a buffer of at
// most 2 GiB): the row's byte offset goes in a scalar register and the lane's
// column offset in a vector register, so no 64-bit address is formed per entry.
template <typename VT, typename WT, bool SIDE_A, int INF, bool FULL, int FUSED, bool UPD, bool BUF>
__device__ __forceinline__ void gather64_chunk(const GatherArgs<VT, WT>& p, const VT* X, __amdgpu_buffer_rsrc_t xr,
                                               const PushTest<VT>& test,
                                               bool ysrc, int32_t src_row, const Tile& T, bool split, bool ns,
                                               bool on, int col, int xcol, int64_t cb, int n, int32_t lx, VT lw,
                                               VT liw, int mbase, int m_rel, Gather64State<VT, WT>& st, VT* lrow) {
    constexpr int COLS = 64;
    const int jend = FULL ? kWave : n;
    for (int j0 = 0; j0 < jend; j0 += INF) {
        VT v[INF];
#pragma unroll
        for (int jj = 0; jj < INF; ++jj) {
            const int j = FULL ? j0 + jj : min(j0 + jj, n - 1);
            if constexpr (BUF && sizeof(VT) == 4)
                v[jj] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                    xr, xcol * 4, (int)((uint32_t)rl(lx, j) * (COLS * 4u)), 0));
            else
                v[jj] = X[(size_t)(uint32_t)rl(lx, j) * COLS + xcol];
        }
#pragma unroll
        for (int jj = 0; jj < INF; ++jj) {
            const int j = j0 + jj;
            if (FULL || j < n) {
                VT sv = v[jj];
                if (FUSED) {   // the select pass's arithmetic: S = y/ws if pushed, else 0
                    if (FUSED == 2 && ysrc) sv = rl(lx, j) == src_row ? VT(1) : VT(0);   // a new query: y = e_src
                    const VT yw = sv * rl(liw, j);
                    sv = test(fabs(sv), fabs(yw)) ? yw : VT(0);
                }
                st.acc += rl(lw, j) * sv;
                if (j + 1 == st.rend) {                 // last entry of the row: flush
                    if (split) {
                        if (on) p.part[(size_t)T.slot * COLS + col] = st.acc;
                    } else {
                        if (UPD) {
                            if (on) lrow[(st.row - T.row_begin) * COLS + col] = st.acc;
                        } else {
                            const size_t idx = (size_t)st.row * COLS + col;
                            if (on) {
                                if (ns) st_nt(&p.OUT[idx], st.acc); else p.OUT[idx] = st.acc;
                            }
                        }
                        const int64_t rend_abs = cb + st.rend;
                        if (SIDE_A && st.acc != VT(0)) st.np += (double)(rend_abs - st.rbeg);
                        st.rbeg = rend_abs;
                    }
                    st.acc = VT(0);
                    ++st.row;
                    st.rend = st.row - mbase < kWave ? rl(m_rel, st.row - mbase) : (1 << 30);
                }
            }
        }
    }
}

// The update of a tile's rows [rb, re) from their sums in lrow (gather B with
// the update fused): B rows' loads in flight, then UpdateRule::apply.
template <typename VT, typename WT, int B>
__device__ __forceinline__ void update_tile_rows(const GatherArgs<VT, WT>& p, const VT* lrow, int rb, int re, int col,
                                                 double* r) {
    constexpr int COLS = 64;
    const UpdateRule<VT> u(p.stu[col], p.SNAPu != nullptr);
    for (int x0 = rb; x0 < re; x0 += B) {
        VT y[B], a[B], iw[B];
        int32_t d[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int x = x0 + k;
            const bool in = x < re;
            const size_t i = (size_t)x * COLS + col;
            d[k] = in ? p.degu[x] : 0;
            iw[k] = in ? p.iwu[x] : VT(0);
            y[k] = in ? u.y_of(p.Yu, i, x) : VT(0);
            a[k] = in ? u.acc_of(p.ACCu, i) : VT(0);
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int x = x0 + k;
            if (x < re && d[k] != 0)
                u.apply(y[k], a[k], lrow[(x - rb) * COLS + col], iw[k], d[k], (size_t)x * COLS + col, p.Yu, p.ACCu,
                        p.SNAPu, r);
        }
    }
}

// AM (gather A): 0 reads S written by the select pass; 1 applies the push rule
// itself (GatherArgs::Yf); 2 does so with buffer-load row reads (FP32, the
// gathered block under 2 GiB). Each mode is a kernel of its own, which keeps
// the code of one launch small.
// UPD > 0 (gather B only; UPD rows' loads in flight in the update): tiles of
// at most upd_rows whole rows, whose sums stay
// in LDS (each lane writes and reads only its own column: no barrier); after
// each whole-row tile its rows are updated. Split pieces go to the partial
// sums as usual (their rows are updated by the fix-up). The block's update
// reductions go to slots red_slot + blockIdx.x.
template <typename VT, typename WT, bool SIDE_A, int INF, int UPD, int AM>
__global__ __launch_bounds__(kPassThreads) void k_gather64(GatherArgs<VT, WT> p) {
    constexpr int COLS = 64;
    constexpr int LROWS = UPD ? 4096 / (COLS * (int)sizeof(VT)) : 1;   // upd_rows()
    __shared__ double sh[kPassThreads];
    __shared__ VT lds_rows[UPD ? kWavesPerBlock * LROWS * COLS : 1];
    if (*p.n_active == 0) return;
    const bool ns = p.nt_stream != 0;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = wave_in_block();
    const int col = lane;
    const bool on = col < live_cols(p.n_active, COLS);
    VT* lrow = UPD ? lds_rows + wid * LROWS * COLS : nullptr;
    // lanes of unused columns read column 0 of the same row (lane 0's cache
    // line, so no extra traffic and no divergent branch around the loads);
    // their sums are never stored and their push cost is dropped
    const int xcol = on ? col : 0;
    // gather A with the push rule applied here (see GatherArgs::Yf)
    constexpr bool fused = SIDE_A && AM > 0;
    constexpr bool kBuf = fused && AM == 2 && sizeof(VT) == 4;
    PushTest<VT> test(RULE_NONE, VT(0), VT(0));
    bool ysrc = false;
    int32_t src_row = -1;
    if (fused) {
        const ColState& cs = p.stf[col];
        test = PushTest<VT>(cs.ruleA, (VT)cs.k_ss, (VT)cs.k_pi);
        ysrc = on && (cs.fresh != 0 || cs.reset_y != 0);
        src_row = cs.src_row;
    }
    // the comparison with the source's row only in sweeps where a column starts
    // a query (wave-uniform: every wavefront holds all 64 columns)
    const bool new_q = fused && __ballot(ysrc) != 0ull;
    const VT* X = fused ? p.Yf : p.X;
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
        (void*)X, (short)0, kBuf ? (int)((uint32_t)p.n_x * (COLS * 4u)) : 0, kRawBufferFlags);   // kBuf only
    Gather64State<VT, WT> st;
    st.np = 0.0;
    double r[kNumRed] = {0, 0, 0, 0, 0};   // UPD: the update's reductions
    const int n_waves = gridDim.x * kWavesPerBlock;
    for (int t = blockIdx.x * kWavesPerBlock + wid; t < p.n_tiles; t += n_waves) {
        const Tile T = load_tile(p.tiles, t);
        const bool split = T.slot >= 0;
        st.row = T.row_begin;
        st.rbeg = T.e_begin;
        st.acc = VT(0);
        for (int64_t cb = T.e_begin; cb < T.e_end; cb += kWave) {
            const int n = (int)min((int64_t)kWave, T.e_end - cb);
            const int32_t lx = lane < n ? (ns ? ld_nt(&p.ci[cb + lane]) : p.ci[cb + lane]) : 0;
            const VT lw = lane < n ? (VT)(ns ? ld_nt(&p.w[cb + lane]) : p.w[cb + lane]) : VT(0);
            const VT liw = fused && lane < n ? p.iwf[cb + lane] : VT(0);   // 1/ws of each entry's neighbour
            const int mbase = st.row;
            const int mr = mbase + lane;
            const int64_t m_end = split ? T.e_end : (mr < T.row_end ? p.rp[mr + 1] : T.e_end);
            // row ends relative to the chunk start (> 64: not in this chunk)
            const int m_rel = (int)min(m_end - cb, (int64_t)(1 << 30));
            st.rend = rl(m_rel, 0);
            // FUSED: 0 the select pass's S, 1 the push rule applied here, 2 also
            // y = e_src for the columns that start a query in this sweep
#define BHPP_CHUNK(FULL, FUSED)                                                                          \
    gather64_chunk<VT, WT, SIDE_A, INF, FULL, FUSED, (UPD > 0), kBuf>(p, X, xr, test, ysrc, src_row, T, split, \
                                                                      ns, on, col, xcol, cb, n, lx, lw, liw,    \
                                                                      mbase, m_rel, st, lrow)
            if constexpr (fused) {
                if (n == kWave) {
                    if (new_q) BHPP_CHUNK(true, 2); else BHPP_CHUNK(true, 1);
                } else {
                    if (new_q) BHPP_CHUNK(false, 2); else BHPP_CHUNK(false, 1);
                }
            } else {
                if (n == kWave) BHPP_CHUNK(true, 0); else BHPP_CHUNK(false, 0);
            }
#undef BHPP_CHUNK
        }
        if (UPD && !split && on) update_tile_rows<VT, WT, (UPD > 0 ? UPD : 1)>(p, lrow, T.row_begin, T.row_end, col, r);
    }
    if (!on) st.np = 0.0;
    if (SIDE_A) block_column_sum<COLS>(st.np, sh, p.red + (size_t)RED_NP * COLS * p.n_part, p.n_part,
                                       p.red_slot + blockIdx.x);
    if (UPD) {
#pragma unroll
        for (int k = 0; k < kNumRed; ++k)
            block_column_sum<COLS>(r[k], sh, p.red + (size_t)k * COLS * p.n_part, p.n_part, p.red_slot + blockIdx.x);
    }
}

// ---------------------------------------------------------------------------
// Gather for one source: lanes are adjacency entries. A wavefront walks its
// tile in groups of UNR chunks of 64 entries (coalesced index and weight
// loads, one gather per lane, all UNR chunks in flight); the row-end bitmap
// gives the lanes that end a row, and a segmented inclusive scan across the
// lanes (fixed order) sums each row. The row still open at the end of a chunk
// carries its partial sum into the next one. Tiles hold no empty rows.
// ---------------------------------------------------------------------------
constexpr int kHubLdsBytes = 32768;   // LDS per block for the hub slice of X (k_gather1)

template <typename VT, typename WT, bool SIDE_A>
__global__ __launch_bounds__(kPassThreads) void k_gather1(GatherArgs<VT, WT> p) {
    constexpr int UNR = 4;
    constexpr int HUB = kHubLdsBytes / (int)sizeof(VT);
    __shared__ double sh[kPassThreads];
    __shared__ VT hub[HUB];
    if (*p.n_active == 0) return;
    // the hub slice X[0, nh): one coalesced copy per block, then LDS reads
    // instead of L2 requests for every entry that points at a hub
    const int32_t nh = min(min(HUB, p.hub), p.n_x);
    for (int32_t i = threadIdx.x; i < nh; i += kPassThreads) hub[i] = p.X[i];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = wave_in_block();
    const uint64_t lt_mask = lane ? (~0ull >> (kWave - lane)) : 0ull;   // lanes below this one
    double np = 0.0;
    const int n_waves = gridDim.x * kWavesPerBlock;
    for (int t = blockIdx.x * kWavesPerBlock + wid; t < p.n_tiles; t += n_waves) {
        const Tile T = load_tile(p.tiles, t);
        const bool split = T.slot >= 0;
        int row = T.row_begin;
        int64_t open_begin = T.e_begin;   // first entry of the row still open
        VT carry = VT(0);                 // its partial sum (uniform)
        VT part = VT(0);                  // split pieces: per-lane partial sums
        for (int64_t cb0 = T.e_begin; cb0 < T.e_end; cb0 += (int64_t)kWave * UNR) {
            int n[UNR];
            int32_t x[UNR];
            VT ww[UNR], v[UNR];
            uint64_t mask[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int64_t cb = cb0 + (int64_t)u * kWave;
                n[u] = (int)max((int64_t)0, min((int64_t)kWave, T.e_end - cb));
                const bool valid = lane < n[u];
                x[u] = valid ? p.ci[cb + lane] : 0;
                ww[u] = valid ? (VT)p.w[cb + lane] : VT(0);
                mask[u] = 0;
                if (!split && n[u] > 0) {
                    const int64_t wi = cb >> 6;
                    const int bs = (int)(cb & 63);
                    const uint64_t w0 = p.end_bits[wi];
                    const uint64_t w1 = bs ? p.end_bits[wi + 1] : 0ull;
                    uint64_t m = bs ? ((w0 >> bs) | (w1 << (64 - bs))) : w0;
                    if (n[u] < kWave) m &= (1ull << n[u]) - 1ull;
                    mask[u] = m;
                }
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) v[u] = lane < n[u] ? (x[u] < nh ? hub[x[u]] : p.X[x[u]]) : VT(0);
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                if (n[u] == 0) break;
                const VT term = ww[u] * v[u];
                if (split) {
                    part += term;
                    continue;
                }
                const int64_t cb = cb0 + (int64_t)u * kWave;
                const uint64_t before = mask[u] & lt_mask;
                const int seg = __popcll(before);                           // rows ended before this lane
                const int start = before ? kWave - __clzll(before) : 0;      // first lane of this lane's row
                VT sum = segmented_sum(term, lane, start);
                if (seg == 0) sum += carry;
                if ((mask[u] >> lane) & 1ull) {
                    p.OUT[(size_t)(row + seg)] = sum;
                    if (SIDE_A && sum != VT(0)) {
                        const int64_t beg = seg == 0 ? open_begin : cb + start;
                        np += (double)(cb + lane + 1 - beg);
                    }
                }
                const VT last = rl(sum, n[u] - 1);
                if (mask[u]) {
                    const int h = kWave - 1 - __clzll(mask[u]);              // last row end in the chunk
                    open_begin = cb + h + 1;
                    carry = h == n[u] - 1 ? VT(0) : last;
                } else {
                    carry = last;
                }
                row += __popcll(mask[u]);
            }
        }
        if (split) {
#pragma unroll
            for (int m = 1; m < kWave; m <<= 1) part += __shfl_xor(part, m);
            if (lane == 0) p.part[T.slot] = part;
        }
    }
    if (SIDE_A) block_column_sum<1>(np, sh, p.red + (size_t)RED_NP * p.n_part, p.n_part, p.red_slot + blockIdx.x);
}

// Fix-up of split rows for one source: one wavefront per row, lane l adding
// pieces l, l + 64, ... (four loads in flight), then a butterfly across the
// lanes (every lane ends with the same bits: each step adds two equal pairs).
template <typename VT, typename WT, bool SIDE_A>
__global__ __launch_bounds__(kPassThreads) void k_fixup1(GatherArgs<VT, WT> p, const SplitRow* split, int n_split) {
    __shared__ double sh[kPassThreads];
    if (*p.n_active == 0) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = wave_in_block();
    double np = 0.0;
    for (int i = blockIdx.x * kWavesPerBlock + wid; i < n_split; i += gridDim.x * kWavesPerBlock) {
        const SplitRow S = split[i];
        VT a0 = VT(0), a1 = VT(0), a2 = VT(0), a3 = VT(0);
        int sl = S.slot_begin + lane;
        for (; sl + 3 * kWave < S.slot_end; sl += 4 * kWave) {
            a0 += p.part[sl];
            a1 += p.part[sl + kWave];
            a2 += p.part[sl + 2 * kWave];
            a3 += p.part[sl + 3 * kWave];
        }
        for (; sl < S.slot_end; sl += kWave) a0 += p.part[sl];
        VT v = (a0 + a1) + (a2 + a3);
#pragma unroll
        for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m);
        if (lane == 0) {
            p.OUT[S.row] = v;
            // gather A: the V node's push cost counts when its residue is non-zero
            if (SIDE_A && v != VT(0)) np += (double)(p.rp[S.row + 1] - p.rp[S.row]);
        }
    }
    if (SIDE_A) block_column_sum<1>(np, sh, p.red + (size_t)RED_NP * p.n_part, p.n_part, p.red_slot + blockIdx.x);
}

// Fix-up of split rows, one block per row: thread (sl, col) adds the pieces
// sl, sl + L, sl + 2L, ... (L = threads / COLS) into eight running sums (eight
// loads in flight: a hub row has hundreds of pieces), the block then adds the
// L partial sums in a fixed tree, and writes the row like the gather.
// UPD (gather B with the update fused): the row is updated instead of
// written to OUT, and the block's update reductions go to red_slot + blockIdx.x
// (written even when there is no split row).
template <int COLS, typename VT, typename WT, bool SIDE_A, bool UPD = false>
__global__ __launch_bounds__(kFixThreads) void k_fixup(GatherArgs<VT, WT> p, const SplitRow* split, int n_split) {
    __shared__ double sh[kFixThreads];
    __shared__ VT sv[kFixThreads];
    if (*p.n_active == 0) return;
    constexpr int L = kFixThreads / COLS;
    const int tid = threadIdx.x;
    const int col = tid & (COLS - 1);
    const int sl = tid / COLS;
    const bool on = col < live_cols(p.n_active, COLS);
    double np = 0.0;
    double r[kNumRed] = {0, 0, 0, 0, 0};
    for (int i = blockIdx.x; i < n_split; i += gridDim.x) {
        const SplitRow S = split[i];
        VT a[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = VT(0);
        int s = on ? S.slot_begin + sl : S.slot_end;
        for (; s + 7 * L < S.slot_end; s += 8 * L) {   // eight independent loads in flight
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] += p.part[(size_t)(s + j * L) * COLS + col];
        }
        for (; s < S.slot_end; s += L) a[0] += p.part[(size_t)s * COLS + col];
        sv[tid] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        __syncthreads();
        for (int h = L / 2; h > 0; h >>= 1) {
            if (sl < h) sv[tid] += sv[tid + h * COLS];
            __syncthreads();
        }
        if (sl == 0 && on) {
            const int row = S.row;
            const VT q = sv[tid];
            const size_t i = (size_t)row * COLS + col;
            if (UPD) {
                const UpdateRule<VT> u(p.stu[col], p.SNAPu != nullptr);
                const int32_t d = p.degu[row];
                if (d != 0)
                    u.apply(u.y_of(p.Yu, i, row), u.acc_of(p.ACCu, i), q, p.iwu[row], d, i, p.Yu, p.ACCu, p.SNAPu, r);
            } else {
                p.OUT[i] = q;
            }
            // gather A: the V node is pushed (its cost counted) when its residue is
            // non-zero, the rule the unsplit rows apply to their sums
            if (SIDE_A && q != VT(0)) np += (double)(p.rp[row + 1] - p.rp[row]);
        }
        __syncthreads();
    }
    if (SIDE_A)
        block_column_sum<COLS, kFixThreads / kWave>(np, sh, p.red + (size_t)RED_NP * COLS * p.n_part, p.n_part,
                                                    p.red_slot + blockIdx.x);
    if (UPD) {
#pragma unroll
        for (int k = 0; k < kNumRed; ++k)
            block_column_sum<COLS, kFixThreads / kWave>(r[k], sh, p.red + (size_t)k * COLS * p.n_part, p.n_part,
                                                        p.red_slot + blockIdx.x);
    }
}

// ---------------------------------------------------------------------------
// Select: S(x) = y(x)/ws(x) for every x the source pushes in this sweep
// (its rule for the V-side half), else 0.
// ---------------------------------------------------------------------------
template <int COLS, typename VT>
__global__ __launch_bounds__(kPassThreads) void k_select(const VT* __restrict__ Y, VT* __restrict__ S,
                                                        const VT* __restrict__ inv_ws, int32_t n_rows,
                                                        const ColState* st, const int32_t* n_active) {
    if (*n_active == 0) return;
    const int col = threadIdx.x & (COLS - 1);
    if (col >= live_cols(n_active, COLS)) return;   // no barrier below
    const ColState& cs = st[col];
    const PushTest<VT> test(cs.ruleA, (VT)cs.k_ss, (VT)cs.k_pi);
    const bool fresh = cs.fresh != 0 || cs.reset_y != 0;   // y = e_src this sweep
    const int32_t src_row = cs.src_row;
    const size_t n = (size_t)n_rows * COLS;
    const size_t stride = (size_t)gridDim.x * kPassThreads;
    constexpr int U = 4;
    for (size_t i0 = (size_t)blockIdx.x * kPassThreads + threadIdx.x; i0 < n; i0 += U * stride) {
        VT y[U], iw[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const size_t i = i0 + k * stride;
            const int32_t x = (int32_t)(i / COLS);
            y[k] = i < n ? (fresh ? (x == src_row ? VT(1) : VT(0)) : Y[i]) : VT(0);   // new query: y = e_src
            iw[k] = i < n ? inv_ws[x] : VT(0);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const size_t i = i0 + k * stride;
            const VT yw = y[k] * iw[k];
            if (i < n) S[i] = test(fabs(y[k]), fabs(yw)) ? yw : VT(0);
        }
    }
}

// ---------------------------------------------------------------------------
// Update of U rows: apply the push of x decided by ruleB, add (1-alpha) G,
// convert ACC when the control asks for it, and reduce per source.
// ---------------------------------------------------------------------------
template <int COLS, typename VT>
__global__ __launch_bounds__(kPassThreads) void k_update(VT* __restrict__ Y, VT* __restrict__ ACC,
                                                        const VT* __restrict__ G, const VT* __restrict__ inv_ws,
                                                        const int32_t* __restrict__ deg, int32_t n_rows,
                                                        const ColState* st, const int32_t* n_active, double* red,
                                                        int n_part, int red_slot, VT* __restrict__ SNAP) {
    __shared__ double sh[kPassThreads];
    if (*n_active == 0) return;
    const int col = threadIdx.x & (COLS - 1);
    const UpdateRule<VT> u(st[col], SNAP != nullptr);
    double r[kNumRed] = {0, 0, 0, 0, 0};
    const size_t n = col < live_cols(n_active, COLS) ? (size_t)n_rows * COLS : 0;   // unused columns: no work
    const size_t stride = (size_t)gridDim.x * kPassThreads;   // a multiple of COLS: the column stays fixed
    constexpr int U = 4;
    for (size_t i0 = (size_t)blockIdx.x * kPassThreads + threadIdx.x; i0 < n; i0 += U * stride) {
        VT y[U], a[U], g[U], iw[U];
        int32_t d[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const size_t i = i0 + k * stride;
            const bool in = i < n;
            const int32_t x = in ? (int32_t)(i / COLS) : 0;
            d[k] = in ? deg[x] : 0;
            iw[k] = in ? inv_ws[x] : VT(0);
            y[k] = in ? u.y_of(Y, i, x) : VT(0);
            a[k] = in ? u.acc_of(ACC, i) : VT(0);
            g[k] = in ? G[i] : VT(0);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (d[k] == 0) continue;                          // isolated or past the end: untouched
            u.apply(y[k], a[k], g[k], iw[k], d[k], i0 + k * stride, Y, ACC, SNAP, r);
        }
    }
#pragma unroll
    for (int k = 0; k < kNumRed; ++k)
        block_column_sum<COLS>(r[k], sh, red + (size_t)k * COLS * n_part, n_part, red_slot + blockIdx.x);
}

// ---------------------------------------------------------------------------
// phase control (Algorithms 3 and 4), one block per source
// ---------------------------------------------------------------------------
__device__ void set_rules(ColState& s, int mode, int ra, int rb, int conv) {
    s.mode = mode;
    s.ruleA = ra;
    s.ruleB = rb;
    s.convert = conv;
}

// SS-Push returned: start PI-Push (Algorithm 5).
__device__ void enter_pi(ColState& s, const double* R, double sum_r) {
    s.np_ss = s.np;
    s.sum_r_ss = sum_r;
    if (s.target == 2) {        // single-target HPP: SS-Push's pi_b is the result (Theorem 1)
        set_rules(s, MODE_FINAL, RULE_NONE, RULE_NONE, 3);
        return;
    }
    s.gamma = R[RED_SUM_Y];     // Eq. (gamma): sum_x ws(x)/ws(u) |r(x)| = sum_x |y(x)|
    s.np = 0.0;                 // Algorithm 4 repeats Algorithm 3's push loop, which starts from n_p = 0
    s.snap = s.warm;            // a warm start keeps pi_b as it is now for the combine
    if (R[RED_CNT_PI] == 0.0) {
        // the first selective iteration would push nothing and Eq. (fwd-eps)
        // would hold: return pi_f from Eq. (fppr)
        s.pi_sel_iters = 1;
        s.pi_returned = 1;
        set_rules(s, MODE_FINAL, RULE_NONE, RULE_NONE, s.target == 1 ? 2 : 1);
    } else {
        set_rules(s, MODE_PI_SEL, RULE_PI, RULE_PI, 0);
    }
}

// R[RED_NP] is the sweep's whole push cost, np_v its V-side part.
// PISP: SelectivePush has ended; the next sweep converts ACC to pi_b (the
// backward part, convert 3), restarts the residue from y = e_u and begins the
// t rounds of PowerIteration (Algorithm 1) that add pi_f into ACC.
__device__ void enter_pisp_power(ColState& s, double sum_r) {
    s.np_ss = s.np;
    s.sum_r_ss = sum_r;
    s.reset_y = 1;
    if (s.t == 0) {
        set_rules(s, MODE_FINAL, RULE_NONE, RULE_ALL, 3);
    } else {
        s.t_rem = s.t;
        set_rules(s, MODE_POWER, RULE_ALL, RULE_ALL, 3);
    }
}

__device__ void control_update(ColState& s, const double* R, double np_v, int32_t* n_active) {
    s.fresh = 0;   // after its first sweep a column holds its own query's Y and ACC
    s.snap = 0;    // the snapshot (if any) was taken by the sweep that just ran
    s.reset_y = 0; // likewise the residue restart of PISP
    const int m = s.mode;
    if (m == MODE_DONE) return;
    s.steps += 1;
    // edge visits of this sweep; the U-side count is the update's push set,
    // which the V-side half read unless its rule was NONE (the last sweep of
    // PowerIteration only adds alpha y)
    if (s.ruleA != RULE_NONE) {
        s.visits_u += R[RED_NP] - np_v;
        if (R[RED_NP] - np_v < s.two_e / 32.0) s.sparse_sweeps += 1;
    }
    s.visits_v += np_v;
    const double sum_r = R[RED_SUM_R] * s.ws_src;     // sum_x |r(x)|
    const double sum_y = R[RED_SUM_Y];                // sum_x |r_f(x)|
    const bool ss_stop = (R[RED_CNT_SS] == 0.0) || (sum_r <= s.eps_b);
    switch (m) {
        case MODE_SS_SEL:
            s.np += R[RED_NP];
            s.ss_sel_iters += 1;
            if (s.target == 3 || s.target == 4) {
                // SelectivePush (Algorithm 2): its loop ends when no U residue
                // exceeds eps_b; there is no budget test. PISP goes on with
                // PowerIteration; MCSP's backward part ends here (pi_b)
                if (R[RED_CNT_SS] == 0.0) {
                    if (s.target == 3) {
                        enter_pisp_power(s, sum_r);
                    } else {
                        s.np_ss = s.np;
                        s.sum_r_ss = sum_r;
                        set_rules(s, MODE_FINAL, RULE_NONE, RULE_NONE, 3);
                    }
                }
            } else if (ss_stop) {
                enter_pi(s, R, sum_r);
            } else if (s.np >= s.two_e * (log(1.0 / sum_r) / s.ln_inv)) {      // Eq. (bwd-np)
                s.ss_switched = 1;
                set_rules(s, MODE_SS_SEQ, RULE_ALL, RULE_ALL, 0);
            }
            break;
        case MODE_SS_SEQ:
            s.np += R[RED_NP];
            s.ss_seq_iters += 1;
            if (ss_stop) enter_pi(s, R, sum_r);
            break;
        case MODE_PI_SEL:
            s.np += R[RED_NP];
            s.pi_sel_iters += 1;
            if (R[RED_CNT_PI] == 0.0) {                                         // Eq. (fwd-eps)
                s.np_pi = s.np;
                s.pi_returned = 1;
                set_rules(s, MODE_FINAL, RULE_NONE, RULE_NONE, s.target == 1 ? 2 : 1);
            } else if (s.np >= s.two_e * (log(s.gamma / sum_y) / s.ln_inv)) {  // Eq. (fwd-np)
                s.np_pi = s.np;
                s.sum_rf = sum_y;
                const double tr = ceil(log(sum_y / s.eps_f) / s.ln_inv - 1.0);   // Eq. (t)
                const int t = tr > 0.0 ? (int)tr : 0;
                s.t = t;
                const int cv = s.target == 1 ? 2 : 1;
                if (t == 0) {
                    set_rules(s, MODE_FINAL, RULE_NONE, RULE_ALL, cv);
                } else {
                    s.t_rem = t;
                    set_rules(s, MODE_POWER, RULE_ALL, RULE_ALL, cv);
                }
            }
            break;
        case MODE_POWER:
            s.convert = 0;
            s.t_rem -= 1;
            if (s.t_rem == 0) set_rules(s, MODE_FINAL, RULE_NONE, RULE_ALL, 0);
            break;
        case MODE_FINAL:
            set_rules(s, MODE_DONE, RULE_NONE, RULE_NONE, 0);
            atomicSub(n_active, 1);
            break;
        default:
            break;
    }
}

// Reduction slots [0, off_u) carry only n_p (gather A and its fix-up);
// [off_u, n_used) carry all reductions (the update's blocks); n_part is the
// stride of the slot arrays.
constexpr int kControlWaves = 3;                                    // wavefronts per reduction
constexpr int kControlThreads = kNumRed * kControlWaves * kWave;
template <int COLS>
__global__ __launch_bounds__(kControlThreads) void k_control(ColState* st, const double* red, int n_part, int n_used,
                                                             int off_u, int32_t* n_active) {
    __shared__ double P[kNumRed][kControlWaves];
    __shared__ double PV[kControlWaves];
    __shared__ double R[kNumRed];
    if (*n_active == 0) return;
    const int col = blockIdx.x;
    if (col >= live_cols(n_active, COLS)) return;   // whole block
    // n_active[4] counts the sweeps in which some query of the block ran
    if (col == 0 && threadIdx.x == 0) n_active[4] += 1;
    const int wv = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int k = wv / kControlWaves, sub = wv % kControlWaves;
    const double* src = red + ((size_t)k * COLS + col) * n_part;
    constexpr int stride = kControlWaves * kWave;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = (k == RED_NP ? 0 : off_u) + sub * kWave + lane;
    // n_p: the gather slots [0, off_u) (V side) first, kept apart
    double av = 0.0;
    if (k == RED_NP) {
        for (; i < off_u; i += stride) av += src[i];
    }
    for (; i + 3 * stride < n_used; i += 4 * stride) {
        a0 += src[i];
        a1 += src[i + stride];
        a2 += src[i + 2 * stride];
        a3 += src[i + 3 * stride];
    }
    for (; i < n_used; i += stride) a0 += src[i];
    double v = (a0 + a1) + (a2 + a3);
#pragma unroll
    for (int m = kWave / 2; m > 0; m >>= 1) {
        v += __shfl_xor(v, m);
        av += __shfl_xor(av, m);
    }
    if (lane == 0) {
        P[k][sub] = v;
        if (k == RED_NP) PV[sub] = av;
    }
    __syncthreads();
    if ((int)threadIdx.x < kNumRed) {
        double t = 0.0;
        for (int j = 0; j < kControlWaves; ++j) t += P[threadIdx.x][j];
        if (threadIdx.x == RED_NP) {
            double tv = 0.0;
            for (int j = 0; j < kControlWaves; ++j) tv += PV[j];
            PV[0] = tv;   // read below, after the barrier
            t += tv;
        }
        R[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) control_update(st[col], R, PV[0], n_active);
}

// ---------------------------------------------------------------------------
// initialisation and output
// ---------------------------------------------------------------------------
template <typename VT>
__global__ void k_fill(VT* a, size_t n, VT v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) a[i] = v;
}

template <typename VT>
__global__ void k_seed(VT* Y, const int32_t* rows, int ncols, int cols) {
    int c = threadIdx.x;
    if (c < ncols) Y[(size_t)rows[c] * cols + c] = VT(1);
}

// Block narrowing: column j of the c2-wide dst is column map[j] of the
// c1-wide src (map[j] < 0: zero).
template <typename VT>
__global__ void k_compact(const VT* src, int c1, VT* dst, int c2, const int32_t* map, int32_t nu) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)nu * c2) return;
    const size_t x = i / c2;
    const int m = map[i % c2];
    dst[i] = m >= 0 ? src[x * c1 + m] : VT(0);
}

// Finished columns cols[0..m) of ACC (internal node order) -> out[j][external x]
// (row-major, one row per finished query). The internal rows of the block's 64
// nodes are looked up once into LDS; then either the whole 64-column rows go
// through an LDS tile (reads and writes both coalesced), or, for one or two
// columns, only those entries are read (a row's 256 bytes span two cache
// lines; one column needs one).
// Isolated nodes score 0; their rows of ACC are never written by the sweeps
// (and may hold another block width's data), so they are not read.
template <int COLS, typename VT>
__global__ __launch_bounds__(256) void k_extract(const VT* ACC, const int32_t* perm, const int32_t* deg, int32_t nu,
                                                 const int32_t* cols, int m, VT* out) {
    __shared__ VT tile[64][COLS + (COLS == 1 ? 0 : 1)];
    __shared__ int32_t rowx[64];   // internal row of node x0 + i; -1: isolated or past the end
    const int x0 = blockIdx.x * 64;
    if (threadIdx.x < 64) {
        const int x = x0 + (int)threadIdx.x;
        int32_t xi = -1;
        if (x < nu) {
            xi = perm[x];
            if (deg[xi] == 0) xi = -1;
        }
        rowx[threadIdx.x] = xi;
    }
    __syncthreads();
    if (COLS > 1 && m <= 2) {
        for (int idx = threadIdx.x; idx < 64 * m; idx += 256) {
            const int j = idx / 64, i = idx % 64;
            const int x = x0 + i;
            const int32_t xi = rowx[i];
            if (x < nu) out[(size_t)j * nu + x] = xi >= 0 ? ACC[(size_t)xi * COLS + cols[j]] : VT(0);
        }
        return;
    }
    for (int idx = threadIdx.x; idx < 64 * COLS; idx += 256) {
        const int i = idx / COLS, c = idx % COLS;
        const int32_t xi = rowx[i];
        tile[i][c] = xi >= 0 ? ACC[(size_t)xi * COLS + c] : VT(0);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * m; idx += 256) {
        const int j = idx / 64, i = idx % 64;
        const int x = x0 + i;
        if (x < nu) out[(size_t)j * nu + x] = tile[i][cols[j]];
    }
}

// ---------------------------------------------------------------------------
// Warm start of newly admitted queries (columns cols[j], j < m). With the
// prediction p = ACC start (forward image of pi_b = y) and G the two-hop image
// of p computed in FP64, the signed residue of Lemma 1 in forward coordinates
// is y0 = e_src - (p - (1-alpha) G) / alpha. Per column the kernel also
// reduces sum_x |y0| (= sum |r_f|) and max_x ws(u)/ws(x) |y0| (= max |r|) on
// the stored values.
// ---------------------------------------------------------------------------
__global__ void k_warm_load(const float* P, double* Y, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) Y[i] = (double)P[i];
}

template <int COLS, typename VT>
__global__ __launch_bounds__(kPassThreads) void k_warm_finish(const float* P, const double* G, int ct, int m,
                                                             const int32_t* cols, const ColState* st,
                                                             const double* inv_ws, const int32_t* deg, int32_t nu,
                                                             VT* Y, VT* ACC, double* res) {
    __shared__ double s1[kPassThreads], s2[kPassThreads];
    const int j = threadIdx.x % ct;    // ct is a power of two <= 64: it divides the block
    const int per = kPassThreads / ct;
    double l1 = 0.0, mx = 0.0;
    if (j < m) {
        const int c = cols[j];
        const double alpha = st[c].alpha, wsu = st[c].ws_src;
        const int32_t src = st[c].src_row;
        for (int32_t x = blockIdx.x * per + threadIdx.x / ct; x < nu; x += gridDim.x * per) {
            const size_t ij = (size_t)x * ct + j;
            VT yv = VT(0), pv = VT(0);
            if (deg[x] > 0) {
                const double p = (double)P[ij];
                yv = (VT)((x == src ? 1.0 : 0.0) - (p - (1.0 - alpha) * G[ij]) / alpha);
                pv = (VT)p;
                l1 += fabs((double)yv);
                mx = fmax(mx, wsu * inv_ws[x] * fabs((double)yv));
            }
            Y[(size_t)x * COLS + c] = yv;
            ACC[(size_t)x * COLS + c] = pv;
        }
    }
    s1[threadIdx.x] = l1;
    s2[threadIdx.x] = mx;
    __syncthreads();
    if ((int)threadIdx.x < ct) {
        double a = 0.0, b = 0.0;
        for (int t = threadIdx.x; t < kPassThreads; t += ct) {
            a += s1[t];
            b = fmax(b, s2[t]);
        }
        res[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = a;
        res[((size_t)ct + threadIdx.x) * gridDim.x + blockIdx.x] = b;
    }
}

// Caller-given starts (row q of starts, caller ids, forward coordinates:
// estimates of pi(u, x)) of the new columns into P [n_u][ct] (internal rows).
template <typename T>
__global__ void k_starts_gather(const T* starts, int32_t nu, const int32_t* qids, const int32_t* iperm, int ct,
                                int m, float* P) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)nu * ct) return;
    const int32_t x = (int32_t)(i / ct);
    const int j = (int)(i % ct);
    P[i] = j < m ? (float)starts[(size_t)qids[j] * nu + iperm[x]] : 0.0f;
}

// Keep a warm start only if it beats the cold start (sum |r_f| < 1 and
// max |r| < 1, the cold start's values); otherwise the column restarts cold.
__global__ void k_warm_decide(ColState* st, const double* res, int ct, int m, const int32_t* cols, int nblk) {
    const int j = threadIdx.x;
    if (j >= m) return;
    double l1 = 0.0, mx = 0.0;
    for (int b = 0; b < nblk; ++b) {
        l1 += res[(size_t)j * nblk + b];
        mx = fmax(mx, res[((size_t)ct + j) * nblk + b]);
    }
    ColState& c = st[cols[j]];
    c.res_l1 = l1;
    c.res_max = mx;
    const bool fb = !(l1 < 1.0 && mx < 1.0);
    c.fell_back = fb ? 1 : 0;
    c.warm = fb ? 0 : 1;
    c.fresh = fb ? 1 : 0;     // a cold restart reads y = e_src, ACC = 0 in its first sweep
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <typename VT>
static VT* as(void* p) { return reinterpret_cast<VT*>(p); }

template <typename VT>
static const VT* inv_ws_u_of(const Graph* g);
template <>
const float* inv_ws_u_of<float>(const Graph* g) { return g->inv_ws_u_f; }
template <>
const double* inv_ws_u_of<double>(const Graph* g) { return g->inv_ws_u_d; }
template <typename VT>
static const VT* inv_ws_v_of(const Graph* g);
template <>
const float* inv_ws_v_of<float>(const Graph* g) { return g->inv_ws_v_f; }
template <>
const double* inv_ws_v_of<double>(const Graph* g) { return g->inv_ws_v_d; }

// Buffers of one dense residue block (the graph's workspace or a private one).
struct Block {
    void* Y;
    void* ACC;
    void* S;
    void* G;
    void* Q;
    void* partA;
    void* partB;
    double* red;
    ColState* st;
    int32_t* n_active;
    int32_t* h_active;
    void* SNAP;          // warm starts only (else null)
};

// Gather A's kernel (the AM of k_gather64): with the push rule applied in the
// gather, FP32 blocks under 2 GiB (so that every byte offset is a positive
// 32-bit value) read their rows with buffer loads (measured 1% faster for
// gather A; the U-side gather keeps global loads, which measured faster there).
template <typename VT>
static int gather_a_mode(const Graph* g, bool fuse) {
    if (!fuse) return 0;
    return g->buf_rows && sizeof(VT) == 4 && (uint64_t)g->nu * 64 * sizeof(VT) < (1ull << 31) ? 2 : 1;
}

template <typename VT, typename WT, bool SIDE_A, int UPD = 0>
static void launch_gather64(int inflight, int blocks, hipStream_t s, const GatherArgs<VT, WT>& a, int am = 0) {
#define BHPP_G64(I, M) \
    hipLaunchKernelGGL((k_gather64<VT, WT, SIDE_A, I, UPD, M>), dim3(blocks), dim3(kPassThreads), 0, s, a)
#define BHPP_G64_AM(I)                    \
    do {                                  \
        if constexpr (!SIDE_A) {          \
            BHPP_G64(I, 0);               \
        } else {                          \
            if (am == 0) BHPP_G64(I, 0);  \
            else if (am == 1) BHPP_G64(I, 1); \
            else BHPP_G64(I, 2);          \
        }                                 \
    } while (0)
    switch (inflight) {
        case 4:
            BHPP_G64_AM(4);
            break;
        case 16:
            BHPP_G64_AM(16);
            break;
        default:
            BHPP_G64_AM(8);
            break;
    }
#undef BHPP_G64_AM
#undef BHPP_G64
}

static void prof_begin(Graph* g, hipStream_t s, int kind, double bytes, hipEvent_t* ev) {
    ev[0] = ev[1] = nullptr;
    if (!g->prof_on) return;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
        hipEventDestroy(a);
        return;
    }
    hipEventRecord(a, s);
    ev[0] = a;
    ev[1] = b;
    g->prof_kind.push_back(kind);
    g->prof_b.push_back(bytes);
}
static void prof_end(Graph* g, hipStream_t s, hipEvent_t* ev) {
    if (ev[1] == nullptr) return;
    hipEventRecord(ev[1], s);
    g->prof_ev.push_back(ev[0]);
    g->prof_ev.push_back(ev[1]);
}

// Algorithmic bytes of one launch, counted per unit of the method's own cost
// measure (an edge visit, the increment of n_p in Algorithms 3 and 4):
// a C-column gather visits every entry once per column; the entry's index and
// weight are shared by the C columns and each column reads one value of the
// neighbour's row, so an entry-column costs (4 + sizeof(W)) / C + sizeof(V)
// bytes; every non-isolated output row is written once, with its two offsets.
// Node passes count each value read or written once per column.
// kind 0: gather A (rows V), 1: gather B (rows U), 2: update (rows U),
// 3: select (rows U), 4: gather B with the update fused (timed as kind 1).
template <typename VT, typename WT>
static double launch_bytes(const Graph* g, int cols, int kind) {
    const double nnz = (double)g->ne;
    const double nu = (double)(g->nu - g->info.isolated_u), nv = (double)(g->nv - g->info.isolated_v);
    const double vt = sizeof(VT);
    const double visits = nnz * ((4.0 + sizeof(WT)) + cols * vt);
    // gather A applying the push rule also reads 1/ws of each entry's
    // neighbour; there is no select pass then
    const bool fused = cols == 64 && g->fuse_select && vt == (double)g->elem;
    if (kind == 0) return visits + (fused ? nnz * vt : 0.0) + nv * (8.0 + cols * vt);
    if (kind == 3 && fused) return 0.0;
    if (kind == 1) return visits + nu * (8.0 + cols * vt);
    if (kind == 2)   // degrees, 1/ws_u; read Y, ACC, G; write Y, ACC
        return nu * 4.0 + nu * vt + 5.0 * nu * cols * vt;
    if (kind == 4)   // gather B with the update fused: the gather's reads, then read Y, ACC; write Y, ACC
        return visits + nu * 8.0 + nu * 4.0 + nu * vt + 4.0 * nu * cols * vt;
    return (double)g->nu * (vt + 2.0 * cols * vt);   // select: 1/ws_u, read Y, write S
}

// The V-side half and the U-side gather of one sweep: select, gather A and its
// fix-up, gather B and its fix-up (G = the two-hop image of S). `prof` adds
// HIP-event timing when profiling is on.
// upd (64 columns): gather B applies the update itself over tiles_uf (its
// reduction slots from G.offU, then its fix-up's), and no G is written.
template <int COLS, typename VT, typename WT>
static void launch_front(Graph* g, const Block& b, const Geometry& G, hipStream_t s, bool prof, bool upd = false) {
    GatherArgs<VT, WT> A;
    A.tiles = g->tiles_v.tiles;
    A.n_tiles = g->tiles_v.n_tiles;
    A.rp = g->rp_v;
    A.ci = g->ci_v;
    A.w = reinterpret_cast<const WT*>(g->w_v);
    A.X = as<VT>(b.S);
    A.OUT = as<VT>(b.Q);
    A.part = as<VT>(b.partA);
    A.end_bits = g->end_bits_v;
    A.n_active = b.n_active;
    A.red = b.red;
    A.n_part = G.n_part;
    A.nt_stream = g->nt_stream;
    A.n_x = g->nu;
    A.hub = g->hub_lds ? kHubLdsBytes / (int)sizeof(VT) : 0;
    GatherArgs<VT, WT> B = A;
    B.tiles = g->tiles_u.tiles;
    B.n_tiles = g->tiles_u.n_tiles;
    B.rp = g->rp_u;
    B.ci = g->ci_u;
    B.w = reinterpret_cast<const WT*>(g->w_u);
    B.X = as<VT>(b.Q);
    B.OUT = as<VT>(b.G);
    B.part = as<VT>(b.partB);
    B.end_bits = g->end_bits_u;
    B.n_x = g->nv;
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto pb = [&](int kind) {
        if (prof) prof_begin(g, s, kind, launch_bytes<VT, WT>(g, COLS, kind), ev);
    };

    const bool fuse = COLS == 64 && g->fuse_select && sizeof(VT) == (size_t)g->elem;
    if (fuse) {
        A.Yf = as<VT>(b.Y);
        A.iwf = reinterpret_cast<const VT*>(g->iw_v);
        A.stf = b.st;
    }
    if (!fuse) {
        pb(3);
        hipLaunchKernelGGL((k_select<COLS, VT>), dim3(G.blkU), dim3(kPassThreads), 0, s, as<VT>(b.Y), as<VT>(b.S),
                           inv_ws_u_of<VT>(g), g->nu, b.st, b.n_active);
        prof_end(g, s, ev);
    }
    pb(0);
    A.red_slot = G.offA;
    if (COLS == 64)
        launch_gather64<VT, WT, true>(g->inflight, G.blkA, s, A, gather_a_mode<VT>(g, fuse));
    else if (COLS == 1)
        hipLaunchKernelGGL((k_gather1<VT, WT, true>), dim3(G.blkA), dim3(kPassThreads), 0, s, A);
    else
        hipLaunchKernelGGL((k_gather<COLS, VT, WT, true>), dim3(G.blkA), dim3(kPassThreads), 0, s, A);
    prof_end(g, s, ev);
    // the fix-up always runs: its blocks also write their reduction slots
    A.red_slot = G.offFA;
    if (COLS == 1)
        hipLaunchKernelGGL((k_fixup1<VT, WT, true>), dim3(G.blkFA), dim3(kPassThreads), 0, s, A, g->tiles_v.split,
                           g->tiles_v.n_split);
    else
        hipLaunchKernelGGL((k_fixup<COLS, VT, WT, true>), dim3(G.blkFA), dim3(kFixThreads), 0, s, A,
                           g->tiles_v.split, g->tiles_v.n_split);
    if (COLS == 64 && upd) {
        B.tiles = g->tiles_uf.tiles;
        B.n_tiles = g->tiles_uf.n_tiles;
        B.Yu = as<VT>(b.Y);
        B.ACCu = as<VT>(b.ACC);
        B.SNAPu = as<VT>(b.SNAP);
        B.iwu = inv_ws_u_of<VT>(g);
        B.degu = g->deg_u;
        B.stu = b.st;
        B.OUT = nullptr;
        if (prof) prof_begin(g, s, 1, launch_bytes<VT, WT>(g, COLS, 4), ev);
        B.red_slot = G.offU;
        if (g->upd_inflight == 4)
            launch_gather64<VT, WT, false, 4>(g->inflight, G.blkBU, s, B);
        else
            launch_gather64<VT, WT, false, 2>(g->inflight, G.blkBU, s, B);
        prof_end(g, s, ev);
        B.red_slot = G.offU + G.blkBU;
        hipLaunchKernelGGL((k_fixup<COLS, VT, WT, false, true>), dim3(G.blkFB), dim3(kFixThreads), 0, s, B,
                           g->tiles_uf.split, g->tiles_uf.n_split);
        return;
    }
    pb(1);
    B.red_slot = 0;
    if (COLS == 64)
        launch_gather64<VT, WT, false>(g->inflight, G.blkB, s, B);
    else if (COLS == 1)
        hipLaunchKernelGGL((k_gather1<VT, WT, false>), dim3(G.blkB), dim3(kPassThreads), 0, s, B);
    else
        hipLaunchKernelGGL((k_gather<COLS, VT, WT, false>), dim3(G.blkB), dim3(kPassThreads), 0, s, B);
    prof_end(g, s, ev);
    if (g->tiles_u.n_split > 0) {
        if (COLS == 1)
            hipLaunchKernelGGL((k_fixup1<VT, WT, false>), dim3(G.blkFB), dim3(kPassThreads), 0, s, B,
                               g->tiles_u.split, g->tiles_u.n_split);
        else
            hipLaunchKernelGGL((k_fixup<COLS, VT, WT, false>), dim3(G.blkFB), dim3(kFixThreads), 0, s, B,
                               g->tiles_u.split, g->tiles_u.n_split);
    }
}

template <int COLS, typename VT, typename WT>
static bhpp_status launch_step(Graph* g, const Block& b, const Geometry& G, hipStream_t s) {
    const bool upd = COLS == 64 && g->fuse_update && sizeof(VT) == (size_t)g->elem && g->tiles_uf.tiles != nullptr;
    launch_front<COLS, VT, WT>(g, b, G, s, true, upd);
    int n_used;   // reduction slots of the sweep
    if (upd) {
        n_used = G.offU + G.blkBU + G.blkFB;
    } else {
        hipEvent_t ev[2] = {nullptr, nullptr};
        prof_begin(g, s, 2, launch_bytes<VT, WT>(g, COLS, 2), ev);
        const int blkU = COLS == 1 ? G.blkU1 : G.blkU;   // its blocks fill reduction slots [offU, offU + blkU)
        hipLaunchKernelGGL((k_update<COLS, VT>), dim3(blkU), dim3(kPassThreads), 0, s, as<VT>(b.Y), as<VT>(b.ACC),
                           as<VT>(b.G), inv_ws_u_of<VT>(g), g->deg_u, g->nu, b.st, b.n_active, b.red, G.n_part,
                           G.offU, as<VT>(b.SNAP));
        prof_end(g, s, ev);
        n_used = G.offU + blkU;
    }
    hipLaunchKernelGGL((k_control<COLS>), dim3(COLS), dim3(kControlThreads), 0, s, b.st, b.red, G.n_part, n_used,
                       G.offU, b.n_active);
    BHPP_HIP(hipGetLastError());
    return BHPP_OK;
}

constexpr int kMaxSteps = 4000;   // sweeps without a finished query; a query needs O(log 1/eps)

// One chunk of g->chunk_sweeps sweeps. Unless the kernels are being profiled,
// the chunk is captured once as a HIP graph (all state lives in device
// memory, so every replay continues where the last one stopped) and replayed.
template <int COLS, typename VT, typename WT>
static bhpp_status launch_chunk(Graph* g, const Block& b, const Geometry& G, hipStream_t s, hipGraphExec_t* cache) {
    if (cache && g->use_graphs && !g->prof_on) {
        if (*cache == nullptr) {
            if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return BHPP_DEVICE_ERROR;
            bhpp_status rc = BHPP_OK;
            for (int i = 0; i < g->chunk_sweeps && rc == BHPP_OK; ++i) rc = launch_step<COLS, VT, WT>(g, b, G, s);
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &graph);
            if (rc != BHPP_OK || e != hipSuccess || graph == nullptr) {
                if (graph) hipGraphDestroy(graph);
                (void)hipGetLastError();
                return rc != BHPP_OK ? rc : BHPP_DEVICE_ERROR;
            }
            const hipError_t e2 = hipGraphInstantiate(cache, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (e2 != hipSuccess) {
                *cache = nullptr;
                return BHPP_DEVICE_ERROR;
            }
        }
        BHPP_HIP(hipGraphLaunch(*cache, s));
        return BHPP_OK;
    }
    for (int i = 0; i < g->chunk_sweeps; ++i) {
        const bhpp_status rc = launch_step<COLS, VT, WT>(g, b, G, s);
        if (rc) return rc;
    }
    return BHPP_OK;
}

// Run the block until no source is active (no refill): used for lambda.
template <int COLS, typename VT, typename WT>
static bhpp_status run_plain(Graph* g, const Block& b, hipStream_t s) {
    const Geometry G = geometry(g);
    int steps = 0;
    for (;;) {
        bhpp_status rc = launch_chunk<COLS, VT, WT>(g, b, G, s, nullptr);
        if (rc) return rc;
        steps += g->chunk_sweeps;
        BHPP_HIP(hipMemcpyAsync(b.h_active, b.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        BHPP_HIP(hipStreamSynchronize(s));
        if (b.h_active[0] == 0) return BHPP_OK;
        if (steps > kMaxSteps) return BHPP_NO_CONVERGENCE;
    }
}

static void init_state(ColState& c, double alpha, double ws_src, double eps, double eps_b_ratio, double lambda,
                       int64_t ne, int target = 0) {
    memset(&c, 0, sizeof(c));
    c.alpha = alpha;
    c.ws_src = ws_src;
    c.eps = eps;
    c.target = target;
    // Algorithm 5's split of eps; one direction alone takes the whole eps;
    // PISP halves it (Sec. 3.3)
    c.eps_b = target == 1 ? 0.0 : target == 2 ? eps : (target == 3 || target == 4) ? 0.5 * eps : eps * eps_b_ratio;
    c.eps_f = eps - c.eps_b;
    c.k_ss = ws_src > 0 ? c.eps_b / ws_src : 0.0;
    c.k_pi = c.eps_f / lambda;
    c.two_e = 2.0 * (double)ne;
    c.ln_inv = log(1.0 / (1.0 - alpha));
    c.convert = 0;
    c.qid = -1;
    if (target == 1) {
        // single-source HPP: Algorithm 4 from (pi_b, r) = (0, e_u), gamma = 1
        c.mode = MODE_PI_SEL;
        c.ruleA = c.ruleB = RULE_PI;
        c.gamma = 1.0;
    } else if (target == 3) {
        // PISP: SelectivePush first; PowerIteration's rounds t are the
        // smallest with (1-alpha)^(t+1) <= eps/2, i.e. log_{1/(1-alpha)}(2/eps) - 1
        // rounded up (Sec. 3.3)
        c.mode = MODE_SS_SEL;
        c.ruleA = c.ruleB = RULE_SS;
        const double tr = ceil(log(1.0 / c.eps_f) / c.ln_inv - 1.0);
        c.t = tr > 0.0 ? (int)tr : 0;
    } else {
        c.mode = MODE_SS_SEL;                // Algorithm 3 starts with selective pushes
        c.ruleA = c.ruleB = RULE_SS;
    }
}

static void done_state(ColState& c) {
    memset(&c, 0, sizeof(c));
    c.mode = MODE_DONE;
    c.alpha = 0.5;
    c.k_ss = c.k_pi = 1e300;
    c.qid = -1;
}

static void fill_stats(const ColState& cs, bhpp_query_stats& q) {
    q.ss_sel_iters = cs.ss_sel_iters;
    q.ss_seq_iters = cs.ss_seq_iters;
    q.pi_sel_iters = cs.pi_sel_iters;
    q.t = cs.t;
    q.ss_switched = cs.ss_switched;
    q.pi_returned = cs.pi_returned;
    q.steps = cs.steps;
    q.sparse_sweeps = cs.sparse_sweeps;
    q.np_ss = cs.np_ss;
    q.np_pi = cs.np_pi;
    q.gamma = cs.gamma;
    q.sum_r_ss = cs.sum_r_ss;
    q.sum_rf = cs.sum_rf;
    q.visits_u = cs.visits_u;
    q.visits_v = cs.visits_v;
}

static int log2i(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

static bhpp_status ensure_warm(Graph* g, Workspace& w, int ct, hipStream_t s) {
    if (!w.SNAP) {
        if (hipMalloc(&w.SNAP, (size_t)g->nu * w.cols * w.elem) != hipSuccess) {
            (void)hipGetLastError();
            return BHPP_OUT_OF_MEMORY;
        }
        w.bytes += (size_t)g->nu * w.cols * w.elem;
    }
    if (w.wcols >= ct) return BHPP_OK;
    void* old[] = {w.wY, w.wS, w.wG, w.wQ, w.wpartA, w.wpartB, w.wred, w.wst, w.wn_active, w.wP,
                   w.wres, w.wcol_ids};
    for (void* p : old) hipFree(p);
    w.wcols = 0;
    const Geometry G = geometry(g);
    const size_t c = (size_t)ct, nu = (size_t)g->nu, nv = (size_t)g->nv;
    auto A = [&](void** p, size_t bytes) { return hipMalloc(p, bytes ? bytes : 256) == hipSuccess; };
    const bool ok = A(&w.wY, nu * c * 8) && A(&w.wS, nu * c * 8) && A(&w.wG, nu * c * 8) && A(&w.wQ, nv * c * 8) &&
                    A(&w.wpartA, (size_t)g->tiles_v.n_slots * c * 8) &&
                    A(&w.wpartB, (size_t)slots_u(g) * c * 8) &&
                    A((void**)&w.wred, (size_t)kNumRed * c * G.n_part * 8) &&
                    A((void**)&w.wst, sizeof(ColState) * c) && A((void**)&w.wn_active, 64) &&
                    A((void**)&w.wP, nu * c * 4) && A((void**)&w.wres, 2 * c * kUpdateBlocks * 8) &&
                    A((void**)&w.wcol_ids, (size_t)kMaxCols * 4);
    if (!ok) {
        (void)hipGetLastError();
        return BHPP_OUT_OF_MEMORY;
    }
    w.wcols = ct;
    (void)s;
    return BHPP_OK;
}

template <int CT, typename WT>
static void warm_front(Graph* g, Workspace& w, hipStream_t s) {
    const Block tb{w.wY, nullptr, w.wS, w.wG, w.wQ, w.wpartA, w.wpartB, w.wred, w.wst, w.wn_active,
                   nullptr, nullptr};
    launch_front<CT, double, WT>(g, tb, geometry(g), s, false);
}

// Seed the block columns `cols` (their states already uploaded) from the
// model's predictions: ACC = p, Y = the signed residue, then keep or reject
// each start on the device.
// Where warm starts come from: the model, or starts given by the caller
// (device [n_query][n_u] of the graph dtype, row = query index).
struct WarmSource {
    Model* model = nullptr;
    const void* starts = nullptr;
    bool any() const { return model != nullptr || starts != nullptr; }
};

template <int COLS, typename VT, typename WT>
static bhpp_status warm_init(Graph* g, const WarmSource& src, Workspace& w, const Block& b,
                             const std::vector<int32_t>& cols, const std::vector<ColState>& hs, hipStream_t s) {
    const int m = (int)cols.size();
    if (m == 0) return BHPP_OK;
    const int ct = next_pow2(m);
    bhpp_status rc = ensure_warm(g, w, ct, s);
    if (rc) return rc;
    if (src.model) {
        std::vector<int32_t> rows(m);
        for (int j = 0; j < m; ++j) rows[j] = hs[cols[j]].src_row;
        rc = model_predict(src.model, rows.data(), m, ct, w.wP, s);
        if (rc) return rc;
    } else {
        std::vector<int32_t> q(m);
        for (int j = 0; j < m; ++j) q[j] = hs[cols[j]].qid;
        BHPP_HIP(hipMemcpyAsync(w.wcol_ids, q.data(), 4 * (size_t)m, hipMemcpyHostToDevice, s));
        const size_t n = (size_t)g->nu * ct;
        hipLaunchKernelGGL(k_starts_gather<VT>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (const VT*)src.starts, g->nu, w.wcol_ids, g->iperm_u, ct, m, w.wP);
        BHPP_HIP(hipStreamSynchronize(s));   // q is read by the copy
    }
    const size_t n = (size_t)g->nu * ct;
    hipLaunchKernelGGL(k_warm_load, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w.wP, (double*)w.wY, n);
    std::vector<ColState> ts(ct);
    for (ColState& c : ts) {
        done_state(c);
        c.mode = MODE_POWER;
        c.ruleA = c.ruleB = RULE_ALL;
    }
    const int32_t one[2] = {1, 0};   // one active; all columns in use
    BHPP_HIP(hipMemcpyAsync(w.wst, ts.data(), sizeof(ColState) * ct, hipMemcpyHostToDevice, s));
    BHPP_HIP(hipMemcpyAsync(w.wn_active, one, 8, hipMemcpyHostToDevice, s));
    BHPP_HIP(hipMemcpyAsync(w.wcol_ids, cols.data(), 4 * (size_t)m, hipMemcpyHostToDevice, s));
    switch (ct) {
        case 1: warm_front<1, WT>(g, w, s); break;
        case 2: warm_front<2, WT>(g, w, s); break;
        case 4: warm_front<4, WT>(g, w, s); break;
        case 8: warm_front<8, WT>(g, w, s); break;
        case 16: warm_front<16, WT>(g, w, s); break;
        case 32: warm_front<32, WT>(g, w, s); break;
        default: warm_front<64, WT>(g, w, s); break;
    }
    hipLaunchKernelGGL((k_warm_finish<COLS, VT>), dim3(kUpdateBlocks), dim3(kPassThreads), 0, s, w.wP,
                       (const double*)w.wG, ct, m, w.wcol_ids, b.st, g->inv_ws_u_d, g->deg_u, g->nu, as<VT>(b.Y),
                       as<VT>(b.ACC), w.wres);
    hipLaunchKernelGGL(k_warm_decide, dim3(1), dim3(64), 0, s, b.st, w.wres, ct, m, w.wcol_ids, kUpdateBlocks);
    BHPP_HIP(hipGetLastError());
    // the host vectors above must outlive their copies
    BHPP_HIP(hipStreamSynchronize(s));
    return BHPP_OK;
}

static void fill_warm(const ColState& c, bhpp_warm_stats& o) {
    o.res_l1 = c.res_l1;
    o.res_max = c.res_max;
    o.fell_back = c.fell_back;
    o.reserved = 0;
}

// SS-Push's selective iterations of a lone source as sparse frontier steps
// (frontier.hip: frontier compaction and U->V scatter; the V->U half is the
// dense U-side gather) while the frontier's edges are few (at most |E|/16);
// the first larger frontier, or the end of the selective phase, hands the
// state (Y, ACC and the source's phase control, all on the device) over to
// the dense sweeps. Counts toward the same per-query statistics.
template <typename VT, typename WT>
static bhpp_status sparse_phase(Graph* g, Workspace& w, std::vector<ColState>& hs, hipStream_t s) {
    bhpp_status rc = ensure_sparse(g, w, s);
    if (rc) return rc;
    const Geometry G = geometry(g);
    // explicit start y = e_src, ACC = 0 (instead of the lazy reset of the first dense sweep)
    const size_t nu = (size_t)g->nu;
    hipLaunchKernelGGL(k_fill<VT>, dim3(1024), dim3(256), 0, s, as<VT>(w.Y), nu, VT(0));
    hipLaunchKernelGGL(k_fill<VT>, dim3(1024), dim3(256), 0, s, as<VT>(w.ACC), nu, VT(0));
    int32_t one_row[1] = {hs[0].src_row};
    BHPP_HIP(hipMemcpyAsync(w.ex_tmp, one_row, 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_seed<VT>, dim3(1), dim3(64), 0, s, as<VT>(w.Y), w.ex_tmp, 1, 1);
    hs[0].fresh = 0;
    BHPP_HIP(hipMemcpyAsync(w.st, hs.data(), sizeof(ColState), hipMemcpyHostToDevice, s));
    BHPP_HIP(hipStreamSynchronize(s));
    GatherArgs<VT, WT> B;
    B.tiles = g->tiles_u.tiles;
    B.n_tiles = g->tiles_u.n_tiles;
    B.rp = g->rp_u;
    B.ci = g->ci_u;
    B.w = reinterpret_cast<const WT*>(g->w_u);
    B.X = as<VT>(w.fQ);
    B.OUT = as<VT>(w.scores);
    B.part = as<VT>(w.partB);
    B.end_bits = g->end_bits_u;
    B.n_active = w.n_active;
    B.red = w.red;
    B.n_part = G.n_part;
    B.nt_stream = g->nt_stream;
    B.red_slot = 0;
    B.n_x = g->nv;
    B.hub = g->hub_lds ? kHubLdsBytes / (int)sizeof(VT) : 0;
    for (int it = 0; it < kMaxSteps; ++it) {
        SparseStep io;
        io.max_work = g->ne / 16;
        io.red_blocks = G.blkU1;   // as the one-column update: slots [offU, offU + blkU1)
        io.n_part = G.n_part;
        io.off_u = G.offU;
        rc = sparse_front(g, w, io, s);
        if (rc) return rc;
        if (!io.done) break;
        hipLaunchKernelGGL((k_gather1<VT, WT, false>), dim3(G.blkB), dim3(kPassThreads), 0, s, B);
        if (g->tiles_u.n_split > 0)
            hipLaunchKernelGGL((k_fixup1<VT, WT, false>), dim3(G.blkFB), dim3(kPassThreads), 0, s, B,
                               g->tiles_u.split, g->tiles_u.n_split);
        rc = sparse_finish(g, w, io, w.scores, s);
        if (rc) return rc;
        hipLaunchKernelGGL((k_control<1>), dim3(1), dim3(kControlThreads), 0, s, w.st, w.red, G.n_part,
                           G.offU + G.blkU1, G.offU, w.n_active);
        BHPP_HIP(hipGetLastError());
        BHPP_HIP(hipMemcpyAsync(hs.data(), w.st, sizeof(ColState), hipMemcpyDeviceToHost, s));
        BHPP_HIP(hipStreamSynchronize(s));
        if (hs[0].mode != MODE_SS_SEL) break;
    }
    return BHPP_OK;
}

// Order in which a batch's queries enter the block: longest expected first,
// so that the block's last columns run out together (a longest-processing-
// time-first schedule). Smaller eps needs more sweeps, and so does a source of
// lower degree (on the 100M-edge workload's 1,024 sources, sweeps and log
// degree correlate at -0.62), which the internal numbering (by decreasing
// degree) gives directly: eps ascending, then internal row descending. The
// caller's order when ordering is off. Each query's result does not depend
// on when it is admitted.
static std::vector<int32_t> admission_order(const Graph* g, int n, const int32_t* src_ext, const double* eps) {
    std::vector<int32_t> ord((size_t)n);
    for (int i = 0; i < n; ++i) ord[(size_t)i] = i;
    if (g->order_admit)
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
            if (eps[a] != eps[b]) return eps[a] < eps[b];
            return g->h_perm_u[src_ext[a]] > g->h_perm_u[src_ext[b]];
        });
    return ord;
}

// Queries are fed to a block of COLS columns from a queue. When enough
// columns have finished (or the queue is empty and all have), their beta'
// rows are extracted, their top-k computed, and the free columns take the
// next queries; a reused column needs no reset pass (ColState::fresh).
template <int COLS, typename VT, typename WT>
static bhpp_status run_sched(Graph* g, const WarmSource& warm, bhpp_warm_stats* wstats, int target, int n,
                             const int32_t* src_ext,
                             const double* eps, double alpha, double lambda, void* scores_out, int k,
                             int exclude_self, int32_t* ids_out, void* vals_out, bhpp_query_stats* stats,
                             hipStream_t s) {
    Workspace& w = g->ws;
    const Block b{w.Y, w.ACC, w.S, w.scores, w.Q, w.partA, w.partB, w.red, w.st, w.n_active, w.h_active,
                  w.SNAP};
    const Geometry G = geometry(g);
    const size_t nu = (size_t)g->nu, e = (size_t)g->elem;
    std::vector<ColState> hs(COLS);
    for (int c = 0; c < COLS; ++c) done_state(hs[c]);
    int next = 0;
    int ncols = n < COLS ? n : COLS;   // columns in use (the kernels skip the others)
    std::vector<int32_t> newcols;   // columns given a query since the last upload (warm starts)
    const std::vector<int32_t> order = admission_order(g, n, src_ext, eps);
    auto assign = [&](int c) {
        const int q = order[(size_t)next++];
        const int32_t u = src_ext[q];
        init_state(hs[c], alpha, g->h_ws_u[u], eps[q], g->info.eps_b_ratio, lambda, g->ne, target);
        hs[c].fresh = 1;
        hs[c].src_row = g->h_perm_u[u];
        hs[c].qid = q;
        if (warm.any()) newcols.push_back(c);
    };
    for (int c = 0; c < COLS && next < n; ++c) assign(c);
    auto upload = [&]() -> bhpp_status {
        int32_t act = 0;
        for (int c = 0; c < COLS; ++c) act += hs[c].mode != MODE_DONE ? 1 : 0;
        w.h_active[2] = act;
        w.h_active[3] = ncols;
        BHPP_HIP(hipMemcpyAsync(w.st, hs.data(), sizeof(ColState) * COLS, hipMemcpyHostToDevice, s));
        BHPP_HIP(hipMemcpyAsync(w.n_active, &w.h_active[2], 2 * sizeof(int32_t), hipMemcpyHostToDevice, s));
        if (warm.any() && !newcols.empty()) {
            const bhpp_status r = warm_init<COLS, VT, WT>(g, warm, w, b, newcols, hs, s);
            newcols.clear();
            if (r) return r;
        }
        return BHPP_OK;
    };
    bhpp_status rc = upload();
    if (rc) return rc;
    if (g->prof_on) BHPP_HIP(hipMemsetAsync(w.n_active + 4, 0, sizeof(int32_t), s));   // live sweeps
    if (COLS == 1 && n == 1 && target != 1 && !warm.any() && g->sparse_steps && !g->prof_on) {
        rc = sparse_phase<VT, WT>(g, w, hs, s);
        if (rc) return rc;
    }
    int live = 0;
    for (int c = 0; c < COLS; ++c) live += hs[c].qid >= 0 ? 1 : 0;
    const int R = COLS >= 8 ? COLS / 8 : 1;   // finished columns that trigger an export round
    hipGraphExec_t* cache = &w.chunk_exec[log2i(COLS)];
    hipEvent_t evs[2];
    BHPP_HIP(hipEventCreateWithFlags(&evs[0], hipEventDisableTiming));
    BHPP_HIP(hipEventCreateWithFlags(&evs[1], hipEventDisableTiming));
    int chunk = 0, steps = 0;
    bool pending = false;
    std::vector<int32_t> cols, ex;
    while (live > 0) {
        rc = launch_chunk<COLS, VT, WT>(g, b, G, s, cache);
        if (rc) break;
        steps += g->chunk_sweeps;
        const int slot = chunk & 1;
        if (hipMemcpyAsync(&w.h_active[slot], w.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipEventRecord(evs[slot], s) != hipSuccess) {
            rc = BHPP_DEVICE_ERROR;
            break;
        }
        bool round = false;
        if (pending) {   // the count after the previous chunk
            if (hipEventSynchronize(evs[slot ^ 1]) != hipSuccess) { rc = BHPP_DEVICE_ERROR; break; }
            const int act = w.h_active[slot ^ 1];
            const int done = live - act;
            // with an empty queue, a block whose running sources fit in 32 columns packs them there
            round = act == 0 || (next < n && done >= R) || (g->narrow && next >= n && ncols > 32 && act <= 32);
        }
        pending = true;
        ++chunk;
        if (!round) {
            if (steps > kMaxSteps) { rc = BHPP_NO_CONVERGENCE; break; }
            continue;
        }
        // export round: wait for the chunk in flight, then read every column's state
        if (hipStreamSynchronize(s) != hipSuccess ||
            hipMemcpy(hs.data(), w.st, sizeof(ColState) * COLS, hipMemcpyDeviceToHost) != hipSuccess) {
            rc = BHPP_DEVICE_ERROR;
            break;
        }
        cols.clear();
        ex.clear();
        for (int c = 0; c < COLS; ++c)
            if (hs[c].qid >= 0 && hs[c].mode == MODE_DONE) {
                cols.push_back(c);
                ex.push_back(exclude_self ? src_ext[hs[c].qid] : -1);
            }
        const int m = (int)cols.size();
        if (m > 0) {
            int32_t* d_cols = w.ex_tmp;
            int32_t* d_ex = w.ex_tmp + kMaxCols;
            BHPP_HIP(hipMemcpyAsync(d_cols, cols.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
            BHPP_HIP(hipMemcpyAsync(d_ex, ex.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
            VT* rows = as<VT>(w.scores);   // [m][nu]; G is rewritten by the next sweep
            hipLaunchKernelGGL((k_extract<COLS, VT>), dim3((g->nu + 63) / 64), dim3(256), 0, s, as<VT>(w.ACC),
                               g->perm_u, g->deg_u, g->nu, d_cols, m, rows);
            BHPP_HIP(hipGetLastError());
            if (k > 0) {
                rc = topk_rows(rows, m, g->nu, k, d_ex, g->dtype, w.ids_tmp, w.vals_tmp, s);
                if (rc) break;
            }
            for (int j = 0; j < m; ++j) {
                const int q = hs[cols[j]].qid;
                if (scores_out)
                    BHPP_HIP(hipMemcpyAsync((char*)scores_out + (size_t)q * nu * e, (char*)rows + (size_t)j * nu * e,
                                            nu * e, hipMemcpyDeviceToDevice, s));
                if (k > 0) {
                    BHPP_HIP(hipMemcpyAsync(ids_out + (size_t)q * k, w.ids_tmp + (size_t)j * k, sizeof(int32_t) * k,
                                            hipMemcpyDeviceToDevice, s));
                    BHPP_HIP(hipMemcpyAsync((char*)vals_out + (size_t)q * k * e, (char*)w.vals_tmp + (size_t)j * k * e,
                                            e * k, hipMemcpyDeviceToDevice, s));
                }
                if (stats) fill_stats(hs[cols[j]], stats[q]);
                if (wstats) fill_warm(hs[cols[j]], wstats[q]);
                hs[cols[j]].qid = -1;
                --live;
                if (next < n) {
                    assign(cols[j]);
                    ++live;
                }
            }
            rc = upload();
            if (rc) break;
            steps = 0;
        }
        pending = false;
        chunk = 0;
        if (g->narrow && next >= n && live > 0 && ncols > 32 && live <= 32) {
            // pack: the running columns move to columns [0, live), in order
            // (states re-read: warm starts of this round were decided on the device)
            if (hipStreamSynchronize(s) != hipSuccess ||
                hipMemcpy(hs.data(), w.st, sizeof(ColState) * COLS, hipMemcpyDeviceToHost) != hipSuccess) {
                rc = BHPP_DEVICE_ERROR;
                break;
            }
            std::vector<int32_t> map(kMaxCols, -1);
            std::vector<ColState> nh(COLS);
            for (auto& c : nh) done_state(c);
            int j = 0;
            for (int c = 0; c < COLS; ++c)
                if (hs[c].qid >= 0) {
                    map[j] = c;
                    nh[j] = hs[c];
                    ++j;
                }
            int32_t* d_map = w.ex_tmp + 2 * kMaxCols;
            BHPP_HIP(hipMemcpyAsync(d_map, map.data(), sizeof(int32_t) * kMaxCols, hipMemcpyHostToDevice, s));
            const size_t tot = nu * COLS;
            void* arrays[3] = {w.Y, w.ACC, w.SNAP};
            for (void* a : arrays) {
                if (!a) continue;
                hipLaunchKernelGGL(k_compact<VT>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, as<VT>(a), COLS,
                                   as<VT>(w.S), COLS, d_map, g->nu);
                BHPP_HIP(hipMemcpyAsync(a, w.S, tot * e, hipMemcpyDeviceToDevice, s));
            }
            BHPP_HIP(hipGetLastError());
            hs = nh;
            ncols = live;
            rc = upload();
            if (rc) break;
            BHPP_HIP(hipStreamSynchronize(s));   // map is read by the copy above
        }
    }
    if (rc == BHPP_OK && hipStreamSynchronize(s) != hipSuccess) rc = BHPP_DEVICE_ERROR;
    if (rc == BHPP_OK && g->prof_on) {
        int32_t live_sweeps = 0;
        if (hipMemcpy(&live_sweeps, w.n_active + 4, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
            rc = BHPP_DEVICE_ERROR;
        g->prof_live += live_sweeps;
    }
    hipEventDestroy(evs[0]);
    hipEventDestroy(evs[1]);
    return rc;
}

// Admission of the next queries into freed columns: st[cols[j]] = adm[j];
// the queries among them count as active.
__global__ void k_admit(ColState* st, const ColState* adm, const int32_t* cols, int m, int32_t* n_active) {
    const int j = threadIdx.x;
    const bool act = j < m && adm[j].mode != MODE_DONE;
    if (j < m) st[cols[j]] = adm[j];
    const uint64_t b = __ballot(act);
    if (j == 0 && b) atomicAdd(n_active, (int32_t)__popcll(b));
}

// A queue-fed 64-column batch that never drains the stream to admit queries.
// After every chunk the column states are copied to a pinned host ring; the
// host reads the copy of chunk i while chunk i+1 runs and, for the columns
// whose query finished by chunk i or runs its last sweep (MODE_FINAL) in chunk
// i+1, enqueues behind chunk i+1: the extraction
// of their beta' rows, their top-k and output copies, then the admission of
// the next queries into those columns (k_admit). A finished column is inert
// (its rules are NONE: its ACC is rewritten with the same bits), so reading
// it a chunk later gives the values it finished with. Packing the running
// columns into the low half once the queue is empty drains the stream once.
template <typename VT, typename WT>
static bhpp_status run_sched_async(Graph* g, int target, int n, const int32_t* src_ext, const double* eps,
                                   double alpha, double lambda, void* scores_out, int k, int exclude_self,
                                   int32_t* ids_out, void* vals_out, bhpp_query_stats* stats, hipStream_t s) {
    constexpr int COLS = 64;
    constexpr int NS = 4;   // pinned slots: state copies and admission lists
    Workspace& w = g->ws;
    const Block b{w.Y, w.ACC, w.S, w.scores, w.Q, w.partA, w.partB, w.red, w.st, w.n_active, w.h_active,
                  w.SNAP};
    const Geometry G = geometry(g);
    const size_t nu = (size_t)g->nu, e = (size_t)g->elem;
    ColState* h_snap = nullptr;   // [NS][COLS]
    ColState* h_adm = nullptr;    // [NS][COLS]
    int32_t* h_lists = nullptr;   // [NS][2][COLS]: columns, excluded ids
    int32_t* h_cnt = nullptr;     // [NS] active counts
    if (hipHostMalloc((void**)&h_snap, sizeof(ColState) * NS * COLS) != hipSuccess ||
        hipHostMalloc((void**)&h_adm, sizeof(ColState) * NS * COLS) != hipSuccess ||
        hipHostMalloc((void**)&h_lists, sizeof(int32_t) * NS * 2 * COLS) != hipSuccess ||
        hipHostMalloc((void**)&h_cnt, sizeof(int32_t) * NS) != hipSuccess) {
        if (h_snap) hipHostFree(h_snap);
        if (h_adm) hipHostFree(h_adm);
        if (h_lists) hipHostFree(h_lists);
        (void)hipGetLastError();
        return BHPP_OUT_OF_MEMORY;
    }
    hipEvent_t ev_snap[NS], ev_adm[NS];
    bool adm_busy[NS] = {false, false, false, false};
    for (int i = 0; i < NS; ++i) {
        hipEventCreateWithFlags(&ev_snap[i], hipEventDisableTiming);
        hipEventCreateWithFlags(&ev_adm[i], hipEventDisableTiming);
    }
    std::vector<ColState> hs(COLS);
    std::vector<int32_t> qid(COLS, -1);   // the query each column holds (host view), -1 none
    for (int c = 0; c < COLS; ++c) done_state(hs[c]);
    int next = 0, ncols = COLS, exported = 0;
    const std::vector<int32_t> order = admission_order(g, n, src_ext, eps);
    auto init_q = [&](ColState& c, int col) {
        const int q = order[(size_t)next++];
        const int32_t u = src_ext[q];
        init_state(c, alpha, g->h_ws_u[u], eps[q], g->info.eps_b_ratio, lambda, g->ne, target);
        c.fresh = 1;
        c.src_row = g->h_perm_u[u];
        c.qid = q;
        qid[col] = q;
    };
    for (int c = 0; c < COLS && next < n; ++c) init_q(hs[c], c);
    bhpp_status rc = BHPP_OK;
    {
        int32_t act = 0;
        for (int c = 0; c < COLS; ++c) act += hs[c].mode != MODE_DONE ? 1 : 0;
        w.h_active[2] = act;
        w.h_active[3] = 0;
        if (hipMemcpyAsync(w.st, hs.data(), sizeof(ColState) * COLS, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(w.n_active, &w.h_active[2], 2 * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess)
            rc = BHPP_DEVICE_ERROR;
        if (g->prof_on && hipMemsetAsync(w.n_active + 4, 0, sizeof(int32_t), s) != hipSuccess) rc = BHPP_DEVICE_ERROR;
        if (hipStreamSynchronize(s) != hipSuccess) rc = BHPP_DEVICE_ERROR;   // w.h_active is read by the copy
    }
    hipGraphExec_t* cache = &w.chunk_exec[log2i(COLS)];
    int64_t chunk = 0, idle_sweeps = 0, rounds = 0;
    // a query exported in its last sweep gets its statistics from the state
    // copy of that chunk (taken before the admission that reuses its column)
    struct PendingStats {
        int32_t col, q;
        int64_t copy;   // index of the state copy to read
    };
    std::vector<PendingStats> pend;
    auto flush_stats = [&](int64_t copy, const ColState* snap) {
        size_t keep = 0;
        for (size_t i = 0; i < pend.size(); ++i) {
            if (pend[i].copy == copy) {
                if (stats) fill_stats(snap[pend[i].col], stats[pend[i].q]);
            } else {
                pend[keep++] = pend[i];
            }
        }
        pend.resize(keep);
    };
    // after the stream has drained: every pending copy is in the ring (none
    // newer was taken)
    auto flush_all_stats = [&]() {
        for (const PendingStats& p : pend)
            if (stats) fill_stats(h_snap[(size_t)(p.copy % NS) * COLS + p.col], stats[p.q]);
        pend.clear();
    };
    // export the columns `cols` (finished as of the state copy `snap`) and
    // admit the next queries into them, behind the work already queued
    auto export_round = [&](const std::vector<int32_t>& cols, const ColState* snap) -> bhpp_status {
        const int m = (int)cols.size();
        // a pinned slot whose copies have run (rounds use the slots in turn)
        const int slot = (int)(rounds % NS);
        if (adm_busy[slot] && hipEventSynchronize(ev_adm[slot]) != hipSuccess) return BHPP_DEVICE_ERROR;
        ++rounds;
        int32_t* lc = h_lists + (size_t)slot * 2 * COLS;
        int32_t* lx = lc + COLS;
        ColState* ad = h_adm + (size_t)slot * COLS;
        for (int j = 0; j < m; ++j) {
            const int c = cols[j];
            const int q = snap[c].qid;
            lc[j] = c;
            lx[j] = exclude_self ? src_ext[q] : -1;
            if (snap[c].mode == MODE_FINAL)
                pend.push_back(PendingStats{c, q, chunk - 1});   // the copy behind the chunk just launched
            else if (stats)
                fill_stats(snap[c], stats[q]);
        }
        BHPP_HIP(hipMemcpyAsync(w.ex_tmp, lc, sizeof(int32_t) * 2 * COLS, hipMemcpyHostToDevice, s));
        VT* rows = as<VT>(w.scores);   // [m][nu]; G is rewritten by the next sweep
        if (scores_out || k > 0) {
            hipLaunchKernelGGL((k_extract<COLS, VT>), dim3((g->nu + 63) / 64), dim3(256), 0, s, as<VT>(w.ACC),
                               g->perm_u, g->deg_u, g->nu, w.ex_tmp, m, rows);
            BHPP_HIP(hipGetLastError());
        }
        if (k > 0) {
            const bhpp_status r = topk_rows(rows, m, g->nu, k, w.ex_tmp + COLS, g->dtype, w.ids_tmp, w.vals_tmp, s);
            if (r) return r;
        }
        for (int j = 0; j < m; ++j) {
            const int q = snap[cols[j]].qid;
            if (scores_out)
                BHPP_HIP(hipMemcpyAsync((char*)scores_out + (size_t)q * nu * e, (char*)rows + (size_t)j * nu * e,
                                        nu * e, hipMemcpyDeviceToDevice, s));
            if (k > 0) {
                BHPP_HIP(hipMemcpyAsync(ids_out + (size_t)q * k, w.ids_tmp + (size_t)j * k, sizeof(int32_t) * k,
                                        hipMemcpyDeviceToDevice, s));
                BHPP_HIP(hipMemcpyAsync((char*)vals_out + (size_t)q * k * e, (char*)w.vals_tmp + (size_t)j * k * e,
                                        e * k, hipMemcpyDeviceToDevice, s));
            }
        }
        exported += m;
        // admission: the next queries, or nothing, into the freed columns
        for (int j = 0; j < m; ++j) {
            const int c = cols[j];
            if (next < n) {
                init_q(ad[j], c);
            } else {
                done_state(ad[j]);
                qid[c] = -1;
            }
        }
        BHPP_HIP(hipMemcpyAsync(w.adm, ad, sizeof(ColState) * m, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_admit, dim3(1), dim3(COLS), 0, s, w.st, w.adm, w.ex_tmp, m, w.n_active);
        BHPP_HIP(hipGetLastError());
        BHPP_HIP(hipEventRecord(ev_adm[slot], s));
        adm_busy[slot] = true;
        return BHPP_OK;
    };
    std::vector<int32_t> fin;
    while (rc == BHPP_OK && exported < n) {
        rc = launch_chunk<COLS, VT, WT>(g, b, G, s, cache);
        if (rc) break;
        const int cs = (int)(chunk % NS);
        if (hipMemcpyAsync(h_snap + (size_t)cs * COLS, w.st, sizeof(ColState) * COLS, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipMemcpyAsync(h_cnt + cs, w.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipEventRecord(ev_snap[cs], s) != hipSuccess) {
            rc = BHPP_DEVICE_ERROR;
            break;
        }
        ++chunk;
        if (chunk < 2) continue;
        // the state copy of the chunk before the one just launched
        const int ps = (int)((chunk - 2) % NS);
        if (hipEventSynchronize(ev_snap[ps]) != hipSuccess) { rc = BHPP_DEVICE_ERROR; break; }
        const ColState* snap = h_snap + (size_t)ps * COLS;
        flush_stats(chunk - 2, snap);
        fin.clear();
        for (int c = 0; c < ncols; ++c)
            if (qid[c] >= 0 && snap[c].qid == qid[c] && (snap[c].mode == MODE_DONE || snap[c].mode == MODE_FINAL))
                fin.push_back(c);
        if (!fin.empty()) {
            rc = export_round(fin, snap);
            idle_sweeps = 0;
        } else {
            idle_sweeps += g->chunk_sweeps;
            if (idle_sweeps > kMaxSteps) rc = BHPP_NO_CONVERGENCE;
        }
        if (rc) break;
        // once the queue is empty and at most 32 columns run, move them to the
        // low columns (same bits: columns are independent of their position)
        int live = 0;
        for (int c = 0; c < ncols; ++c) live += qid[c] >= 0 ? 1 : 0;
        if (g->narrow && next >= n && ncols > 32 && live > 0 && live <= 32) {
            if (hipStreamSynchronize(s) != hipSuccess ||
                hipMemcpy(hs.data(), w.st, sizeof(ColState) * COLS, hipMemcpyDeviceToHost) != hipSuccess) {
                rc = BHPP_DEVICE_ERROR;
                break;
            }
            for (int i = 0; i < NS; ++i) adm_busy[i] = false;   // the stream has drained
            flush_all_stats();
            // columns that finished since the last copy leave first
            fin.clear();
            for (int c = 0; c < ncols; ++c)
                if (qid[c] >= 0 && hs[c].qid == qid[c] && hs[c].mode == MODE_DONE) fin.push_back(c);
            if (!fin.empty()) {
                rc = export_round(fin, hs.data());
                if (rc) break;
                if (hipStreamSynchronize(s) != hipSuccess ||
                    hipMemcpy(hs.data(), w.st, sizeof(ColState) * COLS, hipMemcpyDeviceToHost) != hipSuccess) {
                    rc = BHPP_DEVICE_ERROR;
                    break;
                }
                for (int i = 0; i < NS; ++i) adm_busy[i] = false;
            }
            std::vector<int32_t> map(kMaxCols, -1), nq(COLS, -1);
            std::vector<ColState> nh(COLS);
            for (auto& c : nh) done_state(c);
            int j = 0;
            for (int c = 0; c < COLS; ++c)
                if (qid[c] >= 0) {
                    map[j] = c;
                    nh[j] = hs[c];
                    nq[j] = qid[c];
                    ++j;
                }
            if (j > 0) {
                int32_t* d_map = w.ex_tmp + 2 * kMaxCols;
                BHPP_HIP(hipMemcpyAsync(d_map, map.data(), sizeof(int32_t) * kMaxCols, hipMemcpyHostToDevice, s));
                const size_t tot = nu * COLS;
                void* arrays[2] = {w.Y, w.ACC};
                for (void* a : arrays) {
                    hipLaunchKernelGGL(k_compact<VT>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, as<VT>(a),
                                       COLS, as<VT>(w.S), COLS, d_map, g->nu);
                    BHPP_HIP(hipMemcpyAsync(a, w.S, tot * e, hipMemcpyDeviceToDevice, s));
                }
                BHPP_HIP(hipGetLastError());
                ncols = j;
                qid = nq;
                int32_t act = 0;
                for (int c = 0; c < COLS; ++c) act += nh[c].mode != MODE_DONE ? 1 : 0;
                w.h_active[2] = act;
                w.h_active[3] = ncols;
                BHPP_HIP(hipMemcpyAsync(w.st, nh.data(), sizeof(ColState) * COLS, hipMemcpyHostToDevice, s));
                BHPP_HIP(hipMemcpyAsync(w.n_active, &w.h_active[2], 2 * sizeof(int32_t), hipMemcpyHostToDevice, s));
                BHPP_HIP(hipStreamSynchronize(s));   // map, nh and h_active are read by the copies
            }
            chunk = 0;   // the state copies in flight predate the packing
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess && rc == BHPP_OK) rc = BHPP_DEVICE_ERROR;
    if (rc == BHPP_OK) flush_all_stats();
    if (rc == BHPP_OK && g->prof_on) {
        int32_t live_sweeps = 0;
        if (hipMemcpy(&live_sweeps, w.n_active + 4, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
            rc = BHPP_DEVICE_ERROR;
        g->prof_live += live_sweeps;
    }
    for (int i = 0; i < NS; ++i) {
        hipEventDestroy(ev_snap[i]);
        hipEventDestroy(ev_adm[i]);
    }
    hipHostFree(h_snap);
    hipHostFree(h_adm);
    hipHostFree(h_lists);
    hipHostFree(h_cnt);
    return rc;
}

template <typename VT, typename WT>
static bhpp_status run_sched_dispatch(Graph* g, const WarmSource& model, bhpp_warm_stats* ws, int target, int cols,
                                      int n,
                                      const int32_t* src, const double* eps, double alpha, double lambda,
                                      void* scores, int k, int ex, int32_t* ids, void* vals, bhpp_query_stats* st,
                                      hipStream_t s) {
#define BHPP_RUN(C) \
    return run_sched<C, VT, WT>(g, model, ws, target, n, src, eps, alpha, lambda, scores, k, ex, ids, vals, st, s)
    if (cols == 64 && n > 64 && !model.any() && g->async_sched)
        return run_sched_async<VT, WT>(g, target, n, src, eps, alpha, lambda, scores, k, ex, ids, vals, st, s);
    switch (cols) {
        case 1: BHPP_RUN(1);
        case 2: BHPP_RUN(2);
        case 4: BHPP_RUN(4);
        case 8: BHPP_RUN(8);
        case 64: BHPP_RUN(64);
        default: return BHPP_INVALID_ARG;
    }
#undef BHPP_RUN
}

void free_workspace(Workspace& w) {
    for (hipGraphExec_t& x : w.chunk_exec)
        if (x) {
            hipGraphExecDestroy(x);
            x = nullptr;
        }
    void* ptrs[] = {w.Y, w.ACC, w.S, w.Q, w.partA, w.partB, w.red, w.st, w.n_active, w.scores, w.adm,
                    w.ids_tmp, w.vals_tmp, w.ex_tmp, w.SNAP, w.wY, w.wS, w.wG, w.wQ, w.wpartA, w.wpartB,
                    w.wred, w.wst, w.wn_active, w.wP, w.wres, w.wcol_ids, w.fF, w.fS, w.fDeg,
                    w.fOffs, w.fTV, w.fQ, w.fMark, w.fCnt, w.fScanTmp};
    for (void* p : ptrs) hipFree(p);
    if (w.h_active) hipHostFree(w.h_active);
    if (w.h_fCnt) hipHostFree(w.h_fCnt);
    w = Workspace{};
}

// Workspace of the query block. w.scores doubles as G during the sweeps and
// as the row-major score rows of finished queries between sweeps. Blocks of
// fewer columns reuse the buffers with a smaller row stride; rows of isolated
// nodes are never read (S and the update skip them, the extract writes 0).
size_t workspace_bytes(const Graph* g, int cols) {
    const Geometry G = geometry(g);
    const size_t e = (size_t)g->elem, c = (size_t)cols;
    return (size_t)g->nu * c * e * 4 + (size_t)g->nv * c * e + (size_t)g->tiles_v.n_slots * c * e +
           (size_t)slots_u(g) * c * e + (size_t)kNumRed * c * G.n_part * 8 + sizeof(ColState) * c +
           (size_t)kMaxCols * kTopkTmpK * (4 + e) + sizeof(ColState) * kMaxCols + 4096;
}

bhpp_status ensure_workspace(Graph* g, int cols, hipStream_t s) { return ensure_workspace(g, g->ws, cols, s); }

bhpp_status ensure_workspace(Graph* g, Workspace& w, int cols, hipStream_t s) {
    const Geometry G = geometry(g);
    if (w.cols >= cols && w.n_part >= G.n_part) return BHPP_OK;
    free_workspace(w);
    const size_t e = (size_t)g->elem;
    const size_t c = (size_t)cols;
    auto alloc = [&](void** p, size_t bytes) -> bool {
        if (bytes == 0) bytes = 256;
        w.bytes += bytes;
        return hipMalloc(p, bytes) == hipSuccess;
    };
    bool ok = alloc(&w.Y, (size_t)g->nu * c * e) && alloc(&w.ACC, (size_t)g->nu * c * e) &&
              alloc(&w.S, (size_t)g->nu * c * e) &&
              alloc(&w.Q, (size_t)g->nv * c * e) && alloc(&w.partA, (size_t)g->tiles_v.n_slots * c * e) &&
              alloc(&w.partB, (size_t)slots_u(g) * c * e) &&
              alloc((void**)&w.red, (size_t)kNumRed * c * G.n_part * 8 + 64 * 4) &&
              alloc((void**)&w.st, sizeof(ColState) * c) && alloc((void**)&w.n_active, 64) &&
              alloc(&w.scores, (size_t)g->nu * c * e) &&
              alloc((void**)&w.ids_tmp, (size_t)kMaxCols * kTopkTmpK * 4) &&
              alloc(&w.vals_tmp, (size_t)kMaxCols * kTopkTmpK * e) &&
              alloc((void**)&w.ex_tmp, (size_t)3 * kMaxCols * 4) &&
              alloc((void**)&w.adm, sizeof(ColState) * kMaxCols);
    if (ok) ok = hipHostMalloc((void**)&w.h_active, 64) == hipSuccess;
    if (!ok) {
        free_workspace(w);
        (void)hipGetLastError();
        return BHPP_OUT_OF_MEMORY;
    }
    BHPP_HIP(hipMemsetAsync(w.n_active, 0, 64, s));   // [0] active sources, [1] columns in use (0: all)
    const size_t nU = (size_t)g->nu * c;
    if (e == 8) {
        hipLaunchKernelGGL(k_fill<double>, dim3(2048), dim3(256), 0, s, as<double>(w.Y), nU, 0.0);
        hipLaunchKernelGGL(k_fill<double>, dim3(2048), dim3(256), 0, s, as<double>(w.ACC), nU, 0.0);
    } else {
        hipLaunchKernelGGL(k_fill<float>, dim3(2048), dim3(256), 0, s, as<float>(w.Y), nU, 0.0f);
        hipLaunchKernelGGL(k_fill<float>, dim3(2048), dim3(256), 0, s, as<float>(w.ACC), nU, 0.0f);
    }
    BHPP_HIP(hipGetLastError());
    w.cols = cols;
    w.elem = g->elem;
    w.n_part = G.n_part;
    return BHPP_OK;
}

bhpp_status run_queries(Graph* g, Model* model, const void* starts, bhpp_warm_stats* wstats, int32_t target,
                        int32_t n, const int32_t* src_ext, const double* eps, double alpha, double lambda,
                        void* scores_out,
                        int32_t k, int32_t exclude_self, int32_t* topk_ids, void* topk_vals, bhpp_query_stats* stats,
                        hipStream_t caller) {
    WarmSource warm;
    warm.model = model;
    warm.starts = starts;
    if (k > kTopkTmpK) return BHPP_NOT_SUPPORTED;
    if (!g->work) BHPP_HIP(hipStreamCreateWithFlags(&g->work, hipStreamNonBlocking));
    hipStream_t s = g->work;
    // the library's stream waits for the caller's prior work
    hipEvent_t ev;
    BHPP_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    BHPP_HIP(hipEventRecord(ev, caller));
    BHPP_HIP(hipStreamWaitEvent(s, ev, 0));
    // one source: the entry-parallel kernels; up to 8: a block of that many
    // columns; more: the 64-column kernels, with the columns past the batch
    // skipped (measured faster than the narrower kernels from 16 columns on)
    const int cols = n <= 8 ? next_pow2(n) : kMaxCols;
    bhpp_status rc = ensure_workspace(g, cols, s);
    if (rc == BHPP_OK) {
        if (g->dtype == BHPP_DTYPE_F64)
            rc = run_sched_dispatch<double, double>(g, warm, wstats, target, cols, n, src_ext, eps, alpha, lambda,
                                                    scores_out, k, exclude_self, topk_ids, topk_vals, stats, s);
        else
            rc = run_sched_dispatch<float, float>(g, warm, wstats, target, cols, n, src_ext, eps, alpha, lambda,
                                                  scores_out, k, exclude_self, topk_ids, topk_vals, stats, s);
    }
    // and the caller's stream waits for the library's work
    if (hipEventRecord(ev, s) != hipSuccess || hipStreamWaitEvent(caller, ev, 0) != hipSuccess) rc = BHPP_DEVICE_ERROR;
    hipEventDestroy(ev);
    return rc;
}

// Lemma 4: rho = PowerIteration(e = 1, tau) computed in FP64 with one column
// in a private workspace; lambda = min(max rho + |U| (1-alpha)^(tau+1),
// max ws / min ws).
template <typename WT>
static bhpp_status lambda_impl(Graph* g, double alpha, int32_t tau, hipStream_t s, double* out) {
    const Geometry G = geometry(g);
    Block b{};
    const size_t nU = (size_t)g->nu, nV = (size_t)g->nv;
    auto A = [&](void** p, size_t bytes) { return hipMalloc(p, bytes ? bytes : 256) == hipSuccess; };
    bool ok = A(&b.Y, nU * 8) && A(&b.ACC, nU * 8) && A(&b.S, nU * 8) && A(&b.G, nU * 8) && A(&b.Q, nV * 8) &&
              A(&b.partA, (size_t)g->tiles_v.n_slots * 8) &&
              A(&b.partB, (size_t)slots_u(g) * 8) && A((void**)&b.red, (size_t)kNumRed * G.n_part * 8) &&
              A((void**)&b.st, sizeof(ColState)) && A((void**)&b.n_active, 64) &&
              hipHostMalloc((void**)&b.h_active, 64) == hipSuccess;
    bhpp_status rc = ok ? BHPP_OK : BHPP_OUT_OF_MEMORY;
    const bool saved_prof = g->prof_on;
    g->prof_on = false;
    if (rc == BHPP_OK) {
        ColState c;
        done_state(c);
        c.alpha = alpha;
        c.ln_inv = log(1.0 / (1.0 - alpha));
        if (tau > 0) {
            c.t_rem = tau;
            c.mode = MODE_POWER;
            c.ruleA = c.ruleB = RULE_ALL;
        } else {
            c.mode = MODE_FINAL;
            c.ruleA = RULE_NONE;
            c.ruleB = RULE_ALL;
        }
        int32_t one[2] = {1, 0};
        if (hipMemcpyAsync(b.st, &c, sizeof(c), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(b.n_active, one, 8, hipMemcpyHostToDevice, s) != hipSuccess)
            rc = BHPP_DEVICE_ERROR;
        hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, s, as<double>(b.Y), nU, 1.0);
        hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, s, as<double>(b.ACC), nU, 0.0);
        if (rc == BHPP_OK) rc = run_plain<1, double, WT>(g, b, s);
        if (rc == BHPP_OK) {
            std::vector<double> rho(nU);
            if (hipMemcpy(rho.data(), b.ACC, nU * 8, hipMemcpyDeviceToHost) != hipSuccess) rc = BHPP_DEVICE_ERROR;
            double rmax = 0.0;
            for (double v : rho) rmax = v > rmax ? v : rmax;
            const double a = rmax + (double)g->nu * pow(1.0 - alpha, (double)tau + 1.0);
            const double bnd = g->info.ws_u_max / g->info.ws_u_min;
            *out = a < bnd ? a : bnd;
        }
    }
    g->prof_on = saved_prof;
    void* ptrs[] = {b.Y, b.ACC, b.S, b.G, b.Q, b.partA, b.partB, b.red, b.st, b.n_active};
    for (void* p : ptrs) hipFree(p);
    if (b.h_active) hipHostFree(b.h_active);
    return rc;
}

bhpp_status compute_lambda(Graph* g, double alpha, int32_t tau, hipStream_t s, double* lambda_out) {
    if (g->dtype == BHPP_DTYPE_F64) return lambda_impl<double>(g, alpha, tau, s, lambda_out);
    return lambda_impl<float>(g, alpha, tau, s, lambda_out);
}

// ---------------------------------------------------------------------------
// Autotuner: times sweeps of a 64-column block in PowerIteration mode for each
// candidate launch setting (work-tile size, row gathers in flight, streaming
// loads, graph replay) and keeps the fastest. The results do not depend on
// the setting; only the time does.
// ---------------------------------------------------------------------------
template <typename VT, typename WT>
static bhpp_status time_setting(Graph* g, hipStream_t s, int reps, float* ms_out) {
    const int COLS_T = 64;
    bhpp_status rc = ensure_workspace(g, COLS_T, s);
    if (rc) return rc;
    Workspace& w = g->ws;
    const Block b{w.Y, w.ACC, w.S, w.scores, w.Q, w.partA, w.partB, w.red, w.st, w.n_active, w.h_active,
                  w.SNAP};
    const Geometry G = geometry(g);
    std::vector<ColState> hs(COLS_T);
    for (int c = 0; c < COLS_T; ++c) {
        done_state(hs[c]);
        hs[c].alpha = g->info.alpha;
        hs[c].mode = MODE_POWER;
        hs[c].ruleA = hs[c].ruleB = RULE_ALL;
        hs[c].t_rem = 1 << 20;               // never finishes within the timing
        hs[c].fresh = 1;
        hs[c].src_row = c % g->nu;           // hubs first in internal order
    }
    int32_t act[2] = {COLS_T, 0};
    BHPP_HIP(hipMemcpyAsync(w.st, hs.data(), sizeof(ColState) * COLS_T, hipMemcpyHostToDevice, s));
    BHPP_HIP(hipMemcpyAsync(w.n_active, act, 8, hipMemcpyHostToDevice, s));
    hipGraphExec_t* cache = &w.chunk_exec[log2i(COLS_T)];
    rc = launch_chunk<COLS_T, VT, WT>(g, b, G, s, cache);   // warm-up (and capture)
    if (rc) return rc;
    hipEvent_t e0, e1;
    BHPP_HIP(hipEventCreate(&e0));
    BHPP_HIP(hipEventCreate(&e1));
    BHPP_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps && rc == BHPP_OK; ++r) rc = launch_chunk<COLS_T, VT, WT>(g, b, G, s, cache);
    BHPP_HIP(hipEventRecord(e1, s));
    BHPP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *ms_out = ms / (float)(reps * g->chunk_sweeps);
    // leave the block inactive
    done_state(hs[0]);
    for (int c = 0; c < COLS_T; ++c) done_state(hs[c]);
    act[0] = 0;
    BHPP_HIP(hipMemcpyAsync(w.st, hs.data(), sizeof(ColState) * COLS_T, hipMemcpyHostToDevice, s));
    BHPP_HIP(hipMemcpyAsync(w.n_active, act, 8, hipMemcpyHostToDevice, s));
    BHPP_HIP(hipStreamSynchronize(s));
    return rc;
}

void drop_chunk_graphs(Graph* g) {
    for (hipGraphExec_t& x : g->ws.chunk_exec)
        if (x) {
            hipGraphExecDestroy(x);
            x = nullptr;
        }
}

static bhpp_status apply_setting(Graph* g, int tile_edges, int inflight, int nt, int graphs) {
    drop_chunk_graphs(g);
    if (tile_edges != g->tile_edges) {
        free_tiles(&g->tiles_u);
        free_tiles(&g->tiles_v);
        free_tiles(&g->tiles_uf);
        g->tile_edges = tile_edges;
        bhpp_status rc = build_tiles(g->h_rp_u, g->nu, tile_edges, &g->tiles_u);
        if (rc) return rc;
        rc = build_tiles(g->h_rp_v, g->nv, tile_edges, &g->tiles_v);
        if (rc) return rc;
        rc = build_tiles(g->h_rp_u, g->nu, tile_edges, &g->tiles_uf, upd_rows(g->elem));
        if (rc) return rc;
        free_workspace(g->ws);   // slot counts changed
    }
    g->inflight = inflight;
    g->nt_stream = nt;
    g->use_graphs = graphs;
    return BHPP_OK;
}

bhpp_status autotune(Graph* g, hipStream_t s, int* out_cfg) {
    if (!g->work) BHPP_HIP(hipStreamCreateWithFlags(&g->work, hipStreamNonBlocking));
    hipStream_t ws = g->work;
    BHPP_HIP(hipStreamSynchronize(s));
    const int tiles[] = {512, 1024, 2048, 4096};
    const int infl[] = {4, 8, 16};
    int best[4] = {g->tile_edges, g->inflight, g->nt_stream, g->use_graphs};
    float best_ms = 1e30f;
    for (int te : tiles)
        for (int inf : infl)
            for (int nt = 0; nt < 2; ++nt) {
                bhpp_status rc = apply_setting(g, te, inf, nt, 1);
                if (rc) return rc;
                float ms = 0.f;
                rc = g->dtype == BHPP_DTYPE_F64 ? time_setting<double, double>(g, ws, 2, &ms)
                                                : time_setting<float, float>(g, ws, 2, &ms);
                if (rc) return rc;
                if (ms < best_ms) {
                    best_ms = ms;
                    best[0] = te;
                    best[1] = inf;
                    best[2] = nt;
                    best[3] = 1;
                }
            }
    bhpp_status rc = apply_setting(g, best[0], best[1], best[2], best[3]);
    for (int i = 0; i < 4; ++i) out_cfg[i] = best[i];
    // sweeps per chunk: a query that finishes waits for the chunk boundary
    // (and, in queue-fed batches, one more chunk) before its column is
    // refilled, while each chunk costs the host a launch and a state copy;
    // chunks of about 2 ms of sweeps keep the host far ahead of the device
    int chunk = 8;
    while (chunk > 1 && chunk * (double)best_ms > 2.0) chunk /= 2;
    if (chunk != g->chunk_sweeps) drop_chunk_graphs(g);
    g->chunk_sweeps = chunk;
    return rc;
}

bhpp_status set_launch_config(Graph* g, const int* cfg) {
    if (cfg[0] < 64 || cfg[0] > 1 << 16 || (cfg[1] != 4 && cfg[1] != 8 && cfg[1] != 16)) return BHPP_INVALID_ARG;
    return apply_setting(g, cfg[0], cfg[1], cfg[2] ? 1 : 0, cfg[3] ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Serving: a resident query block fed by a request queue (continuous
// batching). Each poll admits waiting requests into free columns, runs one
// chunk of sweeps, and returns the top-k of every request that finished. The
// block width is fixed at creation by the memory budget; a request is
// admitted when a column is free. Columns are independent, so a request's
// result does not depend on the requests it shares the block with.
// ---------------------------------------------------------------------------
struct Server {
    Graph* g = nullptr;
    Model* model = nullptr;               // warm starts for admitted requests (nullable)
    Workspace ws;
    int cols = 0, k = 0, excl = 0;
    double alpha = 0.0, lambda = 0.0;
    hipStream_t s = nullptr;
    std::mutex qmu;                       // guards the queue (submit may run beside poll)
    struct Req { int32_t src; double eps; int64_t tag; };
    std::deque<Req> queue;
    std::vector<ColState> hs;
    std::vector<int64_t> tag;
    std::vector<int32_t> src;
    int32_t* h_ids = nullptr;             // pinned [cols][k]
    void* h_vals = nullptr;
    int64_t completed = 0, sweeps = 0, since_done = 0;
    bool dirty = false;                   // host states changed since the last upload
    // adaptive warm starts: a model whose starts keep falling back only costs
    // time, so after a while it is used for every 16th admission only, until
    // its recent fallback rate drops below 0.9
    std::vector<uint8_t> tried;           // per column: the request was warm-started
    double w_tries = 0.0, w_falls = 0.0;  // decayed counts over recent warm starts
    int64_t admitted = 0, warm_started = 0, warm_fell_back = 0;
};

// Upload the column states, the number of unfinished requests and the column
// bound: requests take the lowest free columns, so at light load the sweep
// kernels skip the loads and stores of the columns above the highest one held.
static bhpp_status server_upload(Server* sv) {
    int32_t act = 0, bound = 0;
    for (int c = 0; c < sv->cols; ++c) {
        act += sv->hs[c].mode != MODE_DONE ? 1 : 0;
        if (sv->hs[c].qid >= 0) bound = c + 1;
    }
    sv->ws.h_active[2] = act;
    sv->ws.h_active[3] = bound < sv->cols ? bound : 0;   // 0: every column
    BHPP_HIP(hipMemcpyAsync(sv->ws.st, sv->hs.data(), sizeof(ColState) * sv->cols, hipMemcpyHostToDevice, sv->s));
    BHPP_HIP(hipMemcpyAsync(sv->ws.n_active, &sv->ws.h_active[2], 2 * sizeof(int32_t), hipMemcpyHostToDevice, sv->s));
    return BHPP_OK;
}

template <int COLS, typename VT, typename WT>
static bhpp_status server_poll_impl(Server* sv, int64_t* tags, int32_t* ids, void* vals, bhpp_query_stats* st,
                                    bhpp_warm_stats* wst, int32_t* n_out) {
    Graph* g = sv->g;
    Workspace& w = sv->ws;
    const Block b{w.Y, w.ACC, w.S, w.scores, w.Q, w.partA, w.partB, w.red, w.st, w.n_active, w.h_active,
                  w.SNAP};
    std::vector<int32_t> newcols;
    const Geometry G = geometry(g);
    hipStream_t s = sv->s;
    *n_out = 0;
    bool dirty = sv->dirty;
    {
        std::lock_guard<std::mutex> lock(sv->qmu);
        for (int c = 0; c < COLS && !sv->queue.empty(); ++c) {
            if (sv->hs[c].qid >= 0) continue;
            const Server::Req r = sv->queue.front();
            sv->queue.pop_front();
            init_state(sv->hs[c], sv->alpha, g->h_ws_u[r.src], r.eps, g->info.eps_b_ratio, sv->lambda, g->ne);
            sv->hs[c].fresh = 1;
            sv->hs[c].src_row = g->h_perm_u[r.src];
            sv->hs[c].qid = c;
            sv->tag[c] = r.tag;
            sv->src[c] = r.src;
            const bool useful = sv->w_tries < 32.0 || sv->w_falls < 0.9 * sv->w_tries;
            const bool warm = sv->model && (useful || sv->admitted % 16 == 0);
            sv->tried[c] = warm ? 1 : 0;
            if (warm) newcols.push_back(c);
            sv->admitted += 1;
            dirty = true;
        }
    }
    if (dirty) {
        bhpp_status rc = server_upload(sv);
        if (rc) return rc;
        sv->dirty = false;
        if (!newcols.empty()) {
            WarmSource ws;
            ws.model = sv->model;
            rc = warm_init<COLS, VT, WT>(g, ws, w, b, newcols, sv->hs, sv->s);
            if (rc) return rc;
        }
    }
    int live = 0;
    for (int c = 0; c < COLS; ++c) live += sv->hs[c].qid >= 0 ? 1 : 0;
    if (live == 0) return BHPP_OK;
    bhpp_status rc = launch_chunk<COLS, VT, WT>(g, b, G, s, &w.chunk_exec[log2i(COLS)]);
    if (rc) return rc;
    sv->sweeps += g->chunk_sweeps;
    sv->since_done += g->chunk_sweeps;
    BHPP_HIP(hipStreamSynchronize(s));
    BHPP_HIP(hipMemcpy(sv->hs.data(), w.st, sizeof(ColState) * COLS, hipMemcpyDeviceToHost));
    std::vector<int32_t> cols, ex;
    for (int c = 0; c < COLS; ++c)
        if (sv->hs[c].qid >= 0 && sv->hs[c].mode == MODE_DONE) {
            cols.push_back(c);
            ex.push_back(sv->excl ? sv->src[c] : -1);
        }
    const int m = (int)cols.size();
    if (m == 0) return sv->since_done > kMaxSteps ? BHPP_NO_CONVERGENCE : BHPP_OK;
    sv->since_done = 0;
    const size_t nu = (size_t)g->nu, e = (size_t)g->elem, kk = (size_t)sv->k;
    int32_t* d_cols = w.ex_tmp;
    int32_t* d_ex = w.ex_tmp + kMaxCols;
    BHPP_HIP(hipMemcpyAsync(d_cols, cols.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
    BHPP_HIP(hipMemcpyAsync(d_ex, ex.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
    VT* rows = as<VT>(w.scores);
    hipLaunchKernelGGL((k_extract<COLS, VT>), dim3((g->nu + 63) / 64), dim3(256), 0, s, as<VT>(w.ACC), g->perm_u,
                       g->deg_u, g->nu, d_cols, m, rows);
    BHPP_HIP(hipGetLastError());
    rc = topk_rows(rows, m, g->nu, sv->k, d_ex, g->dtype, w.ids_tmp, w.vals_tmp, s);
    if (rc) return rc;
    BHPP_HIP(hipMemcpyAsync(sv->h_ids, w.ids_tmp, sizeof(int32_t) * kk * m, hipMemcpyDeviceToHost, s));
    BHPP_HIP(hipMemcpyAsync(sv->h_vals, w.vals_tmp, e * kk * m, hipMemcpyDeviceToHost, s));
    BHPP_HIP(hipStreamSynchronize(s));
    (void)nu;
    for (int j = 0; j < m; ++j) {
        const int c = cols[j];
        tags[j] = sv->tag[c];
        memcpy(ids + (size_t)j * kk, sv->h_ids + (size_t)j * kk, sizeof(int32_t) * kk);
        memcpy((char*)vals + (size_t)j * kk * e, (char*)sv->h_vals + (size_t)j * kk * e, e * kk);
        if (st) fill_stats(sv->hs[c], st[j]);
        if (wst) {
            fill_warm(sv->hs[c], wst[j]);
            if (!sv->tried[c]) {   // admitted cold: report the cold start's values
                wst[j].res_l1 = wst[j].res_max = 1.0;
                wst[j].fell_back = 1;
            }
        }
        if (sv->tried[c]) {
            const int fb = sv->hs[c].fell_back;
            sv->w_tries = 0.99 * sv->w_tries + 1.0;
            sv->w_falls = 0.99 * sv->w_falls + (fb ? 1.0 : 0.0);
            sv->warm_started += 1;
            sv->warm_fell_back += fb;
        }
        sv->hs[c].qid = -1;
    }
    sv->dirty = true;   // freed columns: the device copy still names their request
    sv->completed += m;
    *n_out = m;
    return BHPP_OK;
}

template <typename VT, typename WT>
static bhpp_status server_poll_dispatch(Server* sv, int64_t* t, int32_t* i, void* v, bhpp_query_stats* st,
                                        bhpp_warm_stats* ws, int32_t* n) {
    switch (sv->cols) {
        case 1: return server_poll_impl<1, VT, WT>(sv, t, i, v, st, ws, n);
        case 2: return server_poll_impl<2, VT, WT>(sv, t, i, v, st, ws, n);
        case 4: return server_poll_impl<4, VT, WT>(sv, t, i, v, st, ws, n);
        case 8: return server_poll_impl<8, VT, WT>(sv, t, i, v, st, ws, n);
        case 16: return server_poll_impl<16, VT, WT>(sv, t, i, v, st, ws, n);
        case 32: return server_poll_impl<32, VT, WT>(sv, t, i, v, st, ws, n);
        case 64: return server_poll_impl<64, VT, WT>(sv, t, i, v, st, ws, n);
        default: return BHPP_INVALID_ARG;
    }
}

void server_destroy(Server* sv) {
    if (!sv) return;
    if (sv->s) hipStreamSynchronize(sv->s);
    free_workspace(sv->ws);
    if (sv->h_ids) hipHostFree(sv->h_ids);
    if (sv->h_vals) hipHostFree(sv->h_vals);
    if (sv->s) hipStreamDestroy(sv->s);
    if (sv->g) sv->g->n_servers -= 1;
    delete sv;
}

// device bytes of the warm-start side of a block of `cols` columns: SNAP and
// the FP64 block that computes the residues of up to `cols` new queries
static size_t warm_bytes(const Graph* g, int cols) {
    const Geometry G = geometry(g);
    const size_t c = (size_t)cols, nu = (size_t)g->nu, nv = (size_t)g->nv;
    return nu * c * g->elem + nu * c * (3 * 8 + 4) + nv * c * 8 + (size_t)g->tiles_v.n_slots * c * 8 +
           (size_t)slots_u(g) * c * 8 + (size_t)kNumRed * c * G.n_part * 8 + 2 * c * kUpdateBlocks * 8 + 4096;
}

bhpp_status server_create(Graph* g, Model* model, int max_width, double mem_budget, double alpha, double lambda, int k,
                          int excl, Server** out) {
    auto need = [&](int c) { return (double)workspace_bytes(g, c) + (model ? (double)warm_bytes(g, c) : 0.0); };
    int cols = 1;
    while (cols * 2 <= max_width && cols * 2 <= kMaxCols) cols *= 2;
    if (mem_budget > 0.0)
        while (cols > 1 && need(cols) > mem_budget) cols /= 2;
    if (mem_budget > 0.0 && need(cols) > mem_budget) return BHPP_OUT_OF_MEMORY;
    Server* sv = new (std::nothrow) Server();
    if (!sv) return BHPP_OUT_OF_MEMORY;
    sv->g = g;
    sv->model = model;
    g->n_servers += 1;
    sv->cols = cols;
    sv->k = k;
    sv->excl = excl;
    sv->alpha = alpha;
    sv->lambda = lambda;
    sv->hs.resize(cols);
    for (ColState& c : sv->hs) done_state(c);
    sv->tag.assign(cols, -1);
    sv->src.assign(cols, -1);
    sv->tried.assign(cols, 0);
    bhpp_status rc = BHPP_OK;
    if (hipStreamCreateWithFlags(&sv->s, hipStreamNonBlocking) != hipSuccess) rc = BHPP_DEVICE_ERROR;
    if (rc == BHPP_OK) rc = ensure_workspace(g, sv->ws, cols, sv->s);
    if (rc == BHPP_OK && model) rc = ensure_warm(g, sv->ws, cols, sv->s);
    if (rc == BHPP_OK && (hipHostMalloc((void**)&sv->h_ids, sizeof(int32_t) * (size_t)cols * k) != hipSuccess ||
                          hipHostMalloc(&sv->h_vals, (size_t)g->elem * cols * k) != hipSuccess))
        rc = BHPP_OUT_OF_MEMORY;
    if (rc == BHPP_OK) rc = server_upload(sv);
    if (rc == BHPP_OK && hipStreamSynchronize(sv->s) != hipSuccess) rc = BHPP_DEVICE_ERROR;
    if (rc) {
        (void)hipGetLastError();
        server_destroy(sv);
        return rc;
    }
    *out = sv;
    return BHPP_OK;
}

bhpp_status server_submit(Server* sv, int32_t src, double eps, int64_t tag) {
    std::lock_guard<std::mutex> lock(sv->qmu);
    sv->queue.push_back(Server::Req{src, eps, tag});
    return BHPP_OK;
}

bhpp_status server_poll(Server* sv, int64_t* tags, int32_t* ids, void* vals, bhpp_query_stats* st,
                        bhpp_warm_stats* wst, int32_t* n_out) {
    if (sv->g->dtype == BHPP_DTYPE_F64)
        return server_poll_dispatch<double, double>(sv, tags, ids, vals, st, wst, n_out);
    return server_poll_dispatch<float, float>(sv, tags, ids, vals, st, wst, n_out);
}

void server_info(Server* sv, bhpp_server_summary* o) {
    memset(o, 0, sizeof(*o));
    o->width = sv->cols;
    o->k = sv->k;
    {
        std::lock_guard<std::mutex> lock(sv->qmu);
        o->queued = (int64_t)sv->queue.size();
    }
    int64_t run = 0;
    for (const ColState& c : sv->hs) run += c.qid >= 0 ? 1 : 0;
    o->running = run;
    o->completed = sv->completed;
    o->sweeps = sv->sweeps;
    o->resident_bytes = (double)sv->ws.bytes;
    o->lambda = sv->lambda;
    o->warm_started = sv->warm_started;
    o->warm_fell_back = sv->warm_fell_back;
}

}  // namespace bhpp
