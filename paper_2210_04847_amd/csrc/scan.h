// Exact integer scan turning per-ray counts into packed_info starts, shared
// by the compacting passes (marching, visibility pruning).  The counting
// kernels leave one int64 sum per workgroup of kRaysPerBlock rays; the scan
// and finalize_starts_kernel turn them into each ray's start and the
// device-side total.
#pragma once

#include "common.h"

namespace {

using namespace nacc;
using namespace nacc::dev;

constexpr int kRaysPerBlock = 64;  // rays per workgroup of the counting passes

// Exclusive scan of n int64 values in place (exact, deterministic), in
// tiles of kScanTile values: one workgroup per tile adds its values, one
// workgroup scans the tile sums, and one workgroup per tile rewrites its
// values as offsets from its tile's offset.  Each thread of a tile takes a
// contiguous run of kScanPer values; the runs' sums are scanned in LDS.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;
constexpr int64_t kScanTile = static_cast<int64_t>(kScanThreads) * kScanPer;

__global__ __launch_bounds__(kScanThreads) void scan_tile_sums_kernel(const int64_t* __restrict__ v, int64_t n,
                                                                      int64_t* __restrict__ tile_sums) {
    __shared__ int64_t part[kScanThreads];
    const int t = threadIdx.x;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = base + static_cast<int64_t>(k) * kScanThreads + t;  // coalesced
        if (i < n) s += v[i];
    }
    part[t] = s;
    __syncthreads();
    for (int off = kScanThreads / 2; off > 0; off >>= 1) {
        if (t < off) part[t] += part[t + off];
        __syncthreads();
    }
    if (t == 0) tile_sums[blockIdx.x] = part[0];
}

// tile_offsets: the scanned tile sums (nullptr: one tile, offset 0); total
// (nullable) receives the sum of all n values.
__global__ __launch_bounds__(kScanThreads) void scan_tiles_kernel(int64_t* __restrict__ v, int64_t n,
                                                                  const int64_t* __restrict__ tile_offsets,
                                                                  int64_t* __restrict__ total) {
    __shared__ int64_t part[kScanThreads];
    const int t = threadIdx.x;
    const int64_t a = static_cast<int64_t>(blockIdx.x) * kScanTile + static_cast<int64_t>(t) * kScanPer;
    int64_t run[kScanPer];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        run[k] = a + k < n ? v[a + k] : 0;
        s += run[k];
    }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int64_t x = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    int64_t off = (tile_offsets != nullptr ? tile_offsets[blockIdx.x] : 0) + (part[t] - s);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (a + k < n) v[a + k] = off;
        off += run[k];
    }
    if (total != nullptr && blockIdx.x == gridDim.x - 1 && t == kScanThreads - 1) *total = off;
}

// int64 scratch values scan_exclusive needs for n values (the tile sums).
inline int64_t scan_scratch_values(int64_t n) {
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    return tiles > 1 ? tiles : 0;
}

// Launches the exclusive scan of v[0, n) on stream s; *total (nullable, on
// the device) receives the sum.  n <= kScanTile^2.
inline void scan_exclusive(int64_t* v, int64_t n, int64_t* total, int64_t* scratch, hipStream_t s) {
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles <= 1) {
        hipLaunchKernelGGL(scan_tiles_kernel, dim3(1), dim3(kScanThreads), 0, s, v, n, nullptr, total);
        return;
    }
    hipLaunchKernelGGL(scan_tile_sums_kernel, dim3(static_cast<unsigned>(tiles)), dim3(kScanThreads), 0, s, v, n,
                       scratch);
    hipLaunchKernelGGL(scan_tiles_kernel, dim3(1), dim3(kScanThreads), 0, s, scratch, tiles, nullptr, nullptr);
    hipLaunchKernelGGL(scan_tiles_kernel, dim3(static_cast<unsigned>(tiles)), dim3(kScanThreads), 0, s, v, n,
                       scratch, total);
}

// packed_info[r].start = offset of r's workgroup + exclusive scan of the
// counts inside it (one wave = the workgroup's 64 rays).  Starts that do
// not fit int32 saturate; the fill pass then reports NACC_ECAPACITY.
__global__ __launch_bounds__(kRaysPerBlock) void finalize_starts_kernel(
    const int64_t* __restrict__ block_offsets, int64_t n_rays, int32_t* __restrict__ packed_info) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kRaysPerBlock + threadIdx.x;
    const int n = r < n_rays ? packed_info[2 * r + 1] : 0;
    const int incl = wave_inclusive_sum(n);
    const int64_t start = block_offsets[blockIdx.x] + (incl - n);
    if (r < n_rays) packed_info[2 * r] = static_cast<int32_t>(min(start, static_cast<int64_t>(INT32_MAX)));
}

int64_t num_blocks(int64_t n_rays) { return (n_rays + kRaysPerBlock - 1) / kRaysPerBlock; }

}  // namespace
