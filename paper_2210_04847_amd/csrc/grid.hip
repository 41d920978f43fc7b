// Occupancy-grid update on gfx950 (NerfAcc, Sec. 2.1: a binary grid cached
// and updated during training).  The update rule is delegated by the paper to
// Instant-NGP; it is read here as: decay every cell, take the maximum with
// fresh density samples at random jittered cell positions, threshold.
//
//   decay        occ[c] *= decay                       (streaming, float4)
//   sample_cells Philox4x64-10 per sample -> cell, jittered position
//   update_max   atomic max on the FP32 bit patterns (order-independent)
//   pack         one ballot per wavefront -> two 32-bit words of bits
#include <cmath>

#include "common.h"

#pragma clang fp contract(off)

namespace {

using namespace nacc;
using namespace nacc::dev;

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void decay_kernel(float* __restrict__ occ, int64_t n, float decay) {
    const int64_t n4 = n / 4;
    float4* occ4 = reinterpret_cast<float4*>(occ);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n4; i += stride) {
        float4 v = occ4[i];
        v.x = v.x * decay;
        v.y = v.y * decay;
        v.z = v.z * decay;
        v.w = v.w * decay;
        occ4[i] = v;
    }
    for (int64_t i = 4 * n4 + static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
        occ[i] = occ[i] * decay;
    }
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of two
// 64x64 -> 128-bit products with the published multipliers, keys bumped by
// the published Weyl constants between rounds.
struct U64x4 {
    uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                               uint64_t k1) {
    constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t kMul1 = 0xCA5A826395121157ull;
    constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
    constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t lo0 = kMul0 * c0, hi0 = __umul64hi(kMul0, c0);
        const uint64_t lo1 = kMul1 * c2, hi1 = __umul64hi(kMul1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return U64x4{{c0, c1, c2, c3}};
}

__global__ __launch_bounds__(kThreads) void sample_cells_kernel(uint64_t seed, uint64_t step,
                                                                 const uint64_t* __restrict__ step_dev, int64_t n,
                                                                 int res,
                                                                 uint64_t n_cells, float lo0, float lo1, float lo2,
                                                                 float h0, float h1, float h2, int cascade,
                                                                 int32_t* __restrict__ cells,
                                                                 float* __restrict__ positions) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (q >= n) return;
    const uint64_t update = step_dev != nullptr ? *step_dev : step;
    const U64x4 r = philox4x64_10(static_cast<uint64_t>(q), update, 0, 0, seed, 0);
    const uint64_t cell = ((r.v[0] >> 32) * n_cells) >> 32;
    cells[q] = static_cast<int32_t>(cell);
    const uint64_t per_grid = static_cast<uint64_t>(res) * res * res;
    const int level = cascade ? static_cast<int>(cell / per_grid) : 0;
    const uint64_t local = cell % per_grid;
    const int j0 = static_cast<int>(local / (static_cast<uint64_t>(res) * res));
    const int j1 = static_cast<int>((local / res) % res);
    const int j2 = static_cast<int>(local % res);
    const float jit0 = static_cast<float>(r.v[1] >> 40) * 0x1p-24f;
    const float jit1 = static_cast<float>(r.v[2] >> 40) * 0x1p-24f;
    const float jit2 = static_cast<float>(r.v[3] >> 40) * 0x1p-24f;
    positions[3 * q] = ldexpf(lo0 + (static_cast<float>(j0) + jit0) * h0, level);
    positions[3 * q + 1] = ldexpf(lo1 + (static_cast<float>(j1) + jit1) * h1, level);
    positions[3 * q + 2] = ldexpf(lo2 + (static_cast<float>(j2) + jit2) * h2, level);
}

// max on FP32 through integer atomics: non-negative floats order like their
// signed bit patterns, negative floats order in reverse of their unsigned
// bit patterns, and every non-negative pattern is below every negative one
// as unsigned.  NaN values are skipped.
__global__ __launch_bounds__(kThreads) void update_max_kernel(float* __restrict__ occ,
                                                               const int32_t* __restrict__ cells,
                                                               const float* __restrict__ values, int64_t n,
                                                               int64_t n_cells) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (q >= n) return;
    const int32_t c = cells[q];
    const float v = values[q];
    if (c < 0 || c >= n_cells || v != v) return;
    if (!signbit(v)) {
        atomicMax(reinterpret_cast<int*>(occ) + c, __float_as_int(v));
    } else {
        atomicMin(reinterpret_cast<unsigned int*>(occ) + c, __float_as_uint(v));
    }
}

// One lane per cell; the wave's ballot is bits [64 w, 64 w + 64).
__global__ __launch_bounds__(kThreads) void pack_kernel(const float* __restrict__ occ, int64_t n_cells,
                                                         float threshold, uint32_t* __restrict__ bits) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    const bool set = i < n_cells && occ[i] > threshold;
    const uint64_t m = ballot(set);
    const int lane = lane_id();
    const int64_t word = (i - lane) / 32;
    if (lane == 0 && word < n_cells / 32) bits[word] = static_cast<uint32_t>(m);
    if (lane == 32 && word + 1 < n_cells / 32) bits[word + 1] = static_cast<uint32_t>(m >> 32);
}

// Skip field, per grid: one byte per coarse cell of 4x4x4 fine cells (C
// order), min(NACC_SKIP_CAP, Chebyshev distance in coarse cells to the
// nearest coarse cell that holds an occupied fine cell).  The L-infinity
// distance separates over the axes,
//   dist(a,b,c) = min_da max(|da|, min_db max(|db|, min_dc max(|dc|, e))),
// e = 0 at occupied coarse cells and the cap elsewhere, so it is built by a
// coarse-occupancy pass and one windowed pass per axis (window +-cap).

// Coarse occupancy: one lane per coarse cell, 16 fine-row reads (the 4 bits
// of a row lie in one word since 4 | res).
__global__ __launch_bounds__(kThreads) void coarse_kernel(const uint32_t* __restrict__ bits, int res, int n_grids,
                                                          uint32_t words, uint8_t* __restrict__ out) {
    const int c = res / 4;
    const int64_t per_grid = static_cast<int64_t>(c) * c * c;
    const int64_t id = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (id >= per_grid * n_grids) return;
    const int grid = static_cast<int>(id / per_grid);
    const int64_t cell = id % per_grid;
    const int cx = static_cast<int>(cell / (static_cast<int64_t>(c) * c));
    const int cy = static_cast<int>((cell / c) % c);
    const int cz = static_cast<int>(cell % c);
    const uint32_t* fine = bits + static_cast<int64_t>(grid) * words;
    uint32_t any = 0u;
    for (int x = 4 * cx; x < 4 * cx + 4; ++x) {
        for (int y = 4 * cy; y < 4 * cy + 4; ++y) {
            const int64_t b = (static_cast<int64_t>(x) * res + y) * res + 4 * cz;
            any |= (fine[b >> 5] >> (b & 31)) & 0xFu;
        }
    }
    out[id] = any != 0u ? 0 : NACC_SKIP_CAP;
}

// One axis of the distance: out = min over |t| <= cap of max(|t|, in[cell + t
// along the axis]), inside the grid.  stride: cells between neighbours along
// the axis (c^2, c or 1).
__global__ __launch_bounds__(kThreads) void distance_pass_kernel(const uint8_t* __restrict__ in, int c,
                                                                 int64_t n_cells, int64_t stride,
                                                                 uint8_t* __restrict__ out) {
    const int64_t id = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (id >= n_cells) return;
    const int pos = static_cast<int>((id / stride) % c);
    int best = in[id];
    for (int t = 1; t <= NACC_SKIP_CAP && t < best; ++t) {
        const int lo = pos - t, hi = pos + t;
        int v = NACC_SKIP_CAP;
        if (lo >= 0) v = min(v, static_cast<int>(in[id - t * stride]));
        if (hi < c) v = min(v, static_cast<int>(in[id + t * stride]));
        best = min(best, max(t, v));
    }
    out[id] = static_cast<uint8_t>(best);
}

// Halo bits: one lane per cell of 2^3 fine cells; the lane ORs the fine
// bits within kHaloReach cells of its own on every axis (up to 6 x 6 rows of
// 6 bits, clipped to the grid; the 6 bits of a row lie in at most two
// words), and each wave packs its 64 cells into two words by a ballot.  The
// lanes of a grid are rounded up to whole waves, so no wave spans two grids.
__global__ __launch_bounds__(kThreads) void halo_kernel(const uint32_t* __restrict__ bits, int res, int n_grids,
                                                        uint32_t words, uint32_t out_words,
                                                        uint32_t* __restrict__ out) {
    const int h = res / 2;
    const int64_t cells = static_cast<int64_t>(h) * h * h;
    const int64_t per_grid = static_cast<int64_t>(out_words) * 32;  // lanes per grid, whole waves
    const int64_t id = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t total = per_grid * n_grids;
    const int64_t grid = id / per_grid;
    const int64_t cell = id % per_grid;
    bool any = false;
    if (id < total && cell < cells) {
        const int cx = static_cast<int>(cell / (static_cast<int64_t>(h) * h));
        const int cy = static_cast<int>((cell / h) % h);
        const int cz = static_cast<int>(cell % h);
        const uint32_t* fine = bits + grid * words;
        const int x0 = max(2 * cx - kHaloReach, 0), x1 = min(2 * cx + 1 + kHaloReach, res - 1);
        const int y0 = max(2 * cy - kHaloReach, 0), y1 = min(2 * cy + 1 + kHaloReach, res - 1);
        const int z0 = max(2 * cz - kHaloReach, 0), z1 = min(2 * cz + 1 + kHaloReach, res - 1);
        const uint64_t want = (1ull << (z1 - z0 + 1)) - 1ull;
        for (int x = x0; x <= x1 && !any; ++x) {
            for (int y = y0; y <= y1; ++y) {
                const int64_t a = (static_cast<int64_t>(x) * res + y) * res + z0;  // first bit of the run
                const int64_t b = a + (z1 - z0);                                  // last bit
                const uint64_t lo = fine[a >> 5];
                const uint64_t hi = (b >> 5) != (a >> 5) ? fine[b >> 5] : 0u;
                if ((((hi << 32) | lo) >> (a & 31)) & want) {
                    any = true;
                    break;
                }
            }
        }
    }
    const uint64_t m = ballot(any);
    const int lane = lane_id();
    const int64_t word = (id - lane) / 32;  // id - lane: the wave's first lane, a multiple of 64
    if (lane == 0 && id - lane < total) {
        out[word] = static_cast<uint32_t>(m);
        out[word + 1] = static_cast<uint32_t>(m >> 32);
    }
}

unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kThreads - 1) / kThreads); }

}  // namespace

extern "C" {

int nacc_grid_decay(float* occ, int64_t n_cells, float decay, void* stream) {
    clear_error();
    NACC_REQUIRE(n_cells >= 0, NACC_EINVAL, "n_cells < 0");
    NACC_REQUIRE(n_cells == 0 || occ != nullptr, NACC_EINVAL, "occ must be non-NULL");
    NACC_REQUIRE(reinterpret_cast<uintptr_t>(occ) % 16 == 0, NACC_EINVAL, "occ must be 16-byte aligned");
    if (n_cells == 0) return NACC_OK;
    const int64_t work = (n_cells + 3) / 4;
    const unsigned nb = static_cast<unsigned>(std::min<int64_t>(blocks_for(work), 8192));
    hipLaunchKernelGGL(decay_kernel, dim3(nb), dim3(kThreads), 0, as_stream(stream), occ, n_cells, decay);
    return check_launch("grid decay");
}

int nacc_grid_sample_cells(uint64_t seed, uint64_t step, const uint64_t* step_dev, int64_t n,
                           const nacc_grid_desc* grid, int32_t levels, int32_t* cells, float* positions,
                           void* stream) {
    clear_error();
    NACC_REQUIRE(grid != nullptr, NACC_EINVAL, "grid must be non-NULL");
    NACC_REQUIRE(n >= 0 && n <= INT32_MAX, NACC_EINVAL, "n = %lld out of [0, 2^31-1]", static_cast<long long>(n));
    NACC_REQUIRE(n == 0 || (cells != nullptr && positions != nullptr), NACC_EINVAL, "outputs must be non-NULL");
    NACC_REQUIRE(grid->res >= 1 && grid->res <= 1024, NACC_EINVAL, "grid res = %d out of [1, 1024]", grid->res);
    const bool cascade = grid->lookup == NACC_LOOKUP_CASCADE;
    NACC_REQUIRE(levels >= 1 && (!cascade || levels <= 16), NACC_EINVAL, "levels = %d out of [1, %s]", levels,
                 cascade ? "16" : "2^31");
    const uint64_t n_cells = static_cast<uint64_t>(grid->res) * grid->res * grid->res * levels;
    NACC_REQUIRE(n_cells <= static_cast<uint64_t>(INT32_MAX), NACC_ESHAPE, "too many cells for int32 indices");
    for (int i = 0; i < 3; ++i) {
        NACC_REQUIRE(std::isfinite(grid->lo[i]) && std::isfinite(grid->hi[i]) && grid->lo[i] < grid->hi[i],
                     NACC_EINVAL, "grid box axis %d is empty or not finite", i);
    }
    if (n == 0) return NACC_OK;
    float h[3];
    for (int i = 0; i < 3; ++i) {
        h[i] = static_cast<float>((static_cast<double>(grid->hi[i]) - static_cast<double>(grid->lo[i])) /
                                  static_cast<double>(grid->res));
    }
    hipLaunchKernelGGL(sample_cells_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, as_stream(stream), seed, step,
                       step_dev, n, grid->res, n_cells, grid->lo[0], grid->lo[1], grid->lo[2], h[0], h[1], h[2],
                       cascade ? 1 : 0, cells, positions);
    return check_launch("grid sample cells");
}

int nacc_grid_update_max(float* occ, const int32_t* cells, const float* values, int64_t n, int64_t n_cells,
                         void* stream) {
    clear_error();
    NACC_REQUIRE(n >= 0 && n_cells >= 0, NACC_EINVAL, "negative size");
    NACC_REQUIRE(n == 0 || (occ != nullptr && cells != nullptr && values != nullptr), NACC_EINVAL,
                 "arguments must be non-NULL");
    if (n == 0) return NACC_OK;
    hipLaunchKernelGGL(update_max_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, as_stream(stream), occ, cells,
                       values, n, n_cells);
    return check_launch("grid update max");
}

int64_t nacc_grid_skip_bytes(const nacc_grid_desc* grid) {
    if (grid == nullptr || grid->res < 4 || grid->res % 4 != 0 || grid->n_grids < 1) return 0;
    return halo_offset(grid->res, grid->n_grids) + halo_words(grid->res) * 4 * grid->n_grids;
}

int nacc_grid_build_skip(const uint32_t* bits, const nacc_grid_desc* grid, uint8_t* skip, void* stream) {
    clear_error();
    NACC_REQUIRE(grid != nullptr, NACC_EINVAL, "grid must be non-NULL");
    NACC_REQUIRE(grid->res >= 4 && grid->res <= 1024 && grid->res % 4 == 0, NACC_ENOTSUP,
                 "the skip field needs res %% 4 == 0 (res = %d)", grid->res);
    NACC_REQUIRE(grid->n_grids >= 1, NACC_EINVAL, "n_grids = %d < 1", grid->n_grids);
    const int64_t cells = static_cast<int64_t>(grid->res) * grid->res * grid->res;
    NACC_REQUIRE(cells % 32 == 0, NACC_ESHAPE, "res^3 is not a multiple of 32");
    NACC_REQUIRE(bits != nullptr && skip != nullptr, NACC_EINVAL, "bits and skip must be non-NULL");
    NACC_REQUIRE(reinterpret_cast<uintptr_t>(skip) % 4 == 0, NACC_EINVAL, "skip must be 4-byte aligned");
    const int c = grid->res / 4;
    const int64_t n = static_cast<int64_t>(c) * c * c * grid->n_grids;
    uint8_t* field = skip;
    uint8_t* scratch = skip + n;
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(coarse_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, s, bits, grid->res, grid->n_grids,
                       static_cast<uint32_t>(cells / 32), scratch);
    int st = check_launch("grid skip coarse");
    if (st != NACC_OK) return st;
    const int64_t strides[3] = {1, c, static_cast<int64_t>(c) * c};
    uint8_t* src = scratch;
    uint8_t* dst = field;
    for (int axis = 0; axis < 3; ++axis) {  // z, y, x: the third pass lands in `field`
        hipLaunchKernelGGL(distance_pass_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, s, src, c, n,
                           strides[axis], dst);
        st = check_launch("grid skip distance");
        if (st != NACC_OK) return st;
        uint8_t* t = src;
        src = dst;
        dst = t;
    }
    const int64_t hw = halo_words(grid->res);
    uint32_t* halo = reinterpret_cast<uint32_t*>(skip + halo_offset(grid->res, grid->n_grids));
    hipLaunchKernelGGL(halo_kernel, dim3(blocks_for(hw * 32 * grid->n_grids)), dim3(kThreads), 0, s, bits,
                       grid->res, grid->n_grids, static_cast<uint32_t>(cells / 32), static_cast<uint32_t>(hw),
                       halo);
    return check_launch("grid skip halo");
}

int nacc_grid_pack(const float* occ, int64_t n_cells, float threshold, uint32_t* bits, void* stream) {
    clear_error();
    NACC_REQUIRE(n_cells >= 0 && n_cells % 32 == 0, NACC_ESHAPE, "n_cells = %lld must be a multiple of 32",
                 static_cast<long long>(n_cells));
    NACC_REQUIRE(n_cells == 0 || (occ != nullptr && bits != nullptr), NACC_EINVAL, "arguments must be non-NULL");
    if (n_cells == 0) return NACC_OK;
    hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(n_cells)), dim3(kThreads), 0, as_stream(stream), occ, n_cells,
                       threshold, bits);
    return check_launch("grid pack");
}

}  // extern "C"
