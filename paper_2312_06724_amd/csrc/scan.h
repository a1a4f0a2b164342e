// Device prefix sums without waits between workgroups, in three launches:
//   1. every tile of kScanTile entries is scanned in registers (kScanItems
//      consecutive entries per thread), across a wavefront with lane shuffles
//      and across the workgroup's four wavefronts through LDS; the tile's
//      total goes to tile_sum;
//   2. one workgroup turns the tile totals into exclusive tile offsets;
//   3. every tile after the first adds its offset.
// A scan of at most one tile is the first launch alone. The output may alias
// the input. Integer sums, so the result does not depend on the tiling.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bhpp {

constexpr int kScanItems = 8;
constexpr int kScanTile = 256 * kScanItems;

// Tile totals scan_many needs for n entries.
inline int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

template <typename T>
__device__ inline T wave_inclusive(T v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

template <typename TI, typename TO, bool EXCL>
__global__ __launch_bounds__(256) void k_scan_tile(const TI* in, TO* out, int64_t n, TO* tile_sum) {
    __shared__ TO wsum[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    TO v[kScanItems];
    TO run = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const TO x = base + i < n ? (TO)in[base + i] : TO(0);
        v[i] = EXCL ? run : run + x;
        run += x;
    }
    const TO incl = wave_inclusive(run, lane);
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    TO pre = incl - run;
    for (int k = 0; k < wid; ++k) pre += wsum[k];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) out[base + i] = v[i] + pre;
    if (threadIdx.x == 255) tile_sum[blockIdx.x] = pre + run;
}

// Exclusive scan of the t tile totals in place, by one workgroup.
template <typename TO>
__global__ __launch_bounds__(256) void k_scan_offsets(TO* ts, int64_t t) {
    __shared__ TO wsum[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    TO carry = 0;
    for (int64_t b = 0; b < t; b += 256) {
        const int64_t i = b + threadIdx.x;
        const TO v = i < t ? ts[i] : TO(0);
        const TO incl = wave_inclusive(v, lane);
        if (lane == 63) wsum[wid] = incl;
        __syncthreads();
        TO pre = carry + incl - v;
        for (int k = 0; k < wid; ++k) pre += wsum[k];
        const TO tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();   // every wavefront has read wsum before the next round writes it
        if (i < t) ts[i] = pre;
        carry += tot;
    }
}

// Tile blockIdx.x + 1 adds its offset.
template <typename TO>
__global__ __launch_bounds__(256) void k_scan_add(TO* out, int64_t n, const TO* ts) {
    const int64_t tile = (int64_t)blockIdx.x + 1;
    const TO off = ts[tile];
    const int64_t b = tile * kScanTile;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t j = b + (int64_t)k * 256 + threadIdx.x;
        if (j < n) out[j] += off;
    }
}

// Inclusive (EXCL false) or exclusive prefix sum of in[0, n) into out, with
// tile_sum holding at least scan_tiles(n) entries. Returns the launch status.
template <typename TI, typename TO, bool EXCL>
inline hipError_t scan_many(const TI* in, TO* out, int64_t n, TO* tile_sum, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t t = scan_tiles(n);
    hipLaunchKernelGGL((k_scan_tile<TI, TO, EXCL>), dim3((unsigned)t), dim3(256), 0, s, in, out, n, tile_sum);
    if (t > 1) {
        hipLaunchKernelGGL(k_scan_offsets<TO>, dim3(1), dim3(256), 0, s, tile_sum, t);
        hipLaunchKernelGGL(k_scan_add<TO>, dim3((unsigned)(t - 1)), dim3(256), 0, s, out, n, (const TO*)tile_sum);
    }
    return hipGetLastError();
}

}  // namespace bhpp
