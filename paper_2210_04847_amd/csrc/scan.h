// Exact integer scan turning per-ray counts into packed_info starts, shared
// by the compacting passes (marching, visibility pruning).  The counting
// kernels leave one int64 sum per workgroup of kRaysPerBlock rays; these two
// kernels turn them into each ray's start and the device-side total.
#pragma once

#include "common.h"

namespace {

using namespace nacc;
using namespace nacc::dev;

constexpr int kRaysPerBlock = 64;  // rays per workgroup of the counting passes

// Exclusive scan of the per-workgroup sums, in place, by one workgroup:
// each thread sums a contiguous run, the 1024 run totals are scanned in LDS,
// then each thread rewrites its run as exclusive offsets.  Integer, exact.
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void scan_block_sums_kernel(
    int64_t* __restrict__ sums, int64_t nb, int64_t* __restrict__ total) {
    __shared__ int64_t part[kScanThreads];
    const int t = threadIdx.x;
    const int64_t per = (nb + kScanThreads - 1) / kScanThreads;
    const int64_t a = min(nb, static_cast<int64_t>(t) * per);
    const int64_t b = min(nb, a + per);
    int64_t s = 0;
    for (int64_t i = a; i < b; ++i) s += sums[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    for (int64_t i = a; i < b; ++i) {
        const int64_t v = sums[i];
        sums[i] = run;
        run += v;
    }
    if (t == kScanThreads - 1) *total = part[t];
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
