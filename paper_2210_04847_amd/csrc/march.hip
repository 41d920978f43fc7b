// Occupancy-grid ray marching on gfx950 (NerfAcc, Sec. 2.1 "Ray Marching",
// "Pruning Empty and Occluded Regions", "GPU Memory Efficiency").
//
// Samples are the lattice intervals of each ray whose midpoint lies in an
// occupied cell.  Empty space is pruned while marching, so the ragged output
// is produced by three steps:
//   count  every ray's sample count, plus one partial sum per workgroup;
//   scan   exclusive scan of the workgroup sums, then of the counts inside
//          each workgroup -> packed_info (start, count) and the total;
//   fill   the same traversal again, writing each sample at its offset.
//
// Uniform steps: one wavefront per ray, the 64 lanes test 64 consecutive
// lattice candidates at once, so the 64 grid-word loads of an iteration are
// independent (they overlap in flight instead of forming a dependent chain)
// and the 256 KiB bit grid stays resident in the XCD's L2.  A ballot of the
// occupied lanes gives the count (popcount) and, in the fill pass, each
// lane's output slot (mbcnt), so the writes of a wave are contiguous.
//
// Cone steps: the lattice is a recurrence in t, so one lane walks one ray.
//
// All lattice arithmetic follows the FP32 contract in nacc.h: this file is
// compiled with -ffp-contract=off and `fp contract(off)`, and uses only
// correctly rounded + - * / sqrt, min/max, ldexp and float->int truncation of
// non-negative values.
#include <cmath>

#include "common.h"

#pragma clang fp contract(off)

namespace {

using namespace nacc;
using namespace nacc::dev;

constexpr int kRaysPerBlock = 64;     // rays per workgroup in count/fill/scan
constexpr int kMaxCandidates = 1 << 24;

struct GridK {
    float lo[3];
    float s[3];        // fl32(res / (hi - lo))
    float top;         // (float)(res - 1)
    float base;        // cascade: half-extent of level 0
    int res;
    int n_grids;
    uint32_t words;    // 32-bit words per grid
    int coarse;        // coarse cells per axis of the skip grid (res / 4)
    uint32_t mip_words;  // 32-bit words per grid of the skip grid (dilated half first)
};

struct ClipK {
    float lo[3];
    float hi[3];
};

struct StepK {
    float near_plane, far_plane, dt, dt_max, cone;
    int max_per_ray;
};

// Ray against the clip box (FP32 slab test of the contract).
__device__ __forceinline__ bool clip_ray(const float o[3], const float d[3], const ClipK& c,
                                         float near_plane, float far_plane, float& t_near,
                                         float& t_far) {
    float t_enter = -INFINITY, t_exit = INFINITY;
    bool miss = false;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (d[i] != 0.0f) {
            float ta = (c.lo[i] - o[i]) / d[i];
            float tb = (c.hi[i] - o[i]) / d[i];
            t_enter = fmaxf(t_enter, fminf(ta, tb));
            t_exit = fminf(t_exit, fmaxf(ta, tb));
        } else if (!(o[i] >= c.lo[i] && o[i] <= c.hi[i])) {
            miss = true;
        }
    }
    t_near = fmaxf(t_enter, near_plane);
    t_far = fminf(t_exit, far_plane);
    return !miss && t_near < t_far;
}

// Occupancy bit of point x.  `word0` is the first word of the ray's grid
// (box / contraction lookups); the cascade picks its level itself.
template <int LOOKUP>
__device__ __forceinline__ bool occupied(const uint32_t* __restrict__ bits, uint32_t word0,
                                         const GridK& g, float x0, float x1, float x2) {
    if (LOOKUP == NACC_LOOKUP_CASCADE) {
        // level = number of level boxes the point lies outside of, i.e. the
        // smallest l with max|x_i| <= b 2^l, clamped to the last level.
        float m = fmaxf(fmaxf(fabsf(x0), fabsf(x1)), fabsf(x2));
        int level = 0;
        for (int l = 0; l < g.n_grids - 1; ++l) level += (m > ldexpf(g.base, l)) ? 1 : 0;
        x0 = ldexpf(x0, -level);
        x1 = ldexpf(x1, -level);
        x2 = ldexpf(x2, -level);
        word0 = static_cast<uint32_t>(level) * g.words;
    } else if (LOOKUP == NACC_LOOKUP_CONTRACT) {
        float n = sqrtf((x0 * x0 + x1 * x1) + x2 * x2);
        if (n > 1.0f) {
            float f = (2.0f - 1.0f / n) / n;
            x0 = x0 * f;
            x1 = x1 * f;
            x2 = x2 * f;
        }
    }
    float u0 = fminf(fmaxf((x0 - g.lo[0]) * g.s[0], 0.0f), g.top);
    float u1 = fminf(fmaxf((x1 - g.lo[1]) * g.s[1], 0.0f), g.top);
    float u2 = fminf(fmaxf((x2 - g.lo[2]) * g.s[2], 0.0f), g.top);
    uint32_t res = static_cast<uint32_t>(g.res);
    uint32_t cell = (static_cast<uint32_t>(static_cast<int>(u0)) * res +
                     static_cast<uint32_t>(static_cast<int>(u1))) * res +
                    static_cast<uint32_t>(static_cast<int>(u2));
    uint32_t word = bits[word0 + (cell >> 5)];
    return ((word >> (cell & 31u)) & 1u) != 0u;
}

// Fine cell indices (j_0, j_1, j_2) of point x under the box lookup.
__device__ __forceinline__ void cell_indices(const GridK& g, float x0, float x1, float x2, uint32_t& j0, uint32_t& j1,
                                             uint32_t& j2) {
    j0 = static_cast<uint32_t>(static_cast<int>(fminf(fmaxf((x0 - g.lo[0]) * g.s[0], 0.0f), g.top)));
    j1 = static_cast<uint32_t>(static_cast<int>(fminf(fmaxf((x1 - g.lo[1]) * g.s[1], 0.0f), g.top)));
    j2 = static_cast<uint32_t>(static_cast<int>(fminf(fmaxf((x2 - g.lo[2]) * g.s[2], 0.0f), g.top)));
}

// Bit of the dilated skip grid at the coarse cell holding fine cell j: it is
// clear only if every fine cell within one coarse cell (4 fine cells) of
// it, in every direction, is empty.
__device__ __forceinline__ bool skip_bit(const uint32_t* __restrict__ mip, uint32_t mip0, const GridK& g,
                                         uint32_t j0, uint32_t j1, uint32_t j2) {
    const uint32_t c = static_cast<uint32_t>(g.coarse);
    const uint32_t cell = ((j0 >> 2) * c + (j1 >> 2)) * c + (j2 >> 2);
    return ((mip[mip0 + (cell >> 5)] >> (cell & 31u)) & 1u) != 0u;
}

// Largest group size G in {64, 32, 16, 8} such that the midpoints of any
// two candidates at most G/2 steps apart fall in fine cells at most 4 apart
// on every axis (bound on |u_k - u_t| below 3.9, with a generous allowance
// for FP32 rounding of t, x and u), so that one test point per group plus
// the one-coarse-cell dilation covers every candidate of the group.
// 0: no grouping for this ray.
__device__ __forceinline__ int group_size(const GridK& g, const float o[3], const float d[3], float t_near,
                                          float t_far, float dt) {
    const float tmax = fmaxf(fabsf(t_near), fabsf(t_far));
    float slope = 0.0f, slack = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float sd = g.s[i] * fabsf(d[i]);
        slope = fmaxf(slope, sd * dt);
        slack = fmaxf(slack, g.s[i] * (fabsf(o[i]) + fabsf(g.lo[i]) + 2.0f * fabsf(d[i]) * tmax));
    }
    slack = (slack + static_cast<float>(g.res)) * 0x1p-16f;
    for (int G = 64; G >= 8; G >>= 1) {
        if (slope * static_cast<float>(G / 2) + slack <= 3.9f) return G;
    }
    return 0;
}

// First word of the ray's grid, or false for an invalid grid id (the ray is
// then treated as a miss).
template <int LOOKUP>
__device__ __forceinline__ bool grid_of_ray(const int32_t* __restrict__ grid_id, int64_t r,
                                            const GridK& g, uint32_t& word0) {
    word0 = 0;
    if (LOOKUP != NACC_LOOKUP_CASCADE && grid_id != nullptr) {
        int gid = grid_id[r];
        if (gid < 0 || gid >= g.n_grids) return false;
        word0 = static_cast<uint32_t>(gid) * g.words;
    }
    return true;
}

// One ray, uniform steps, whole wave.  Returns the ray's sample count (the
// same value in every lane).  FILL writes samples [0, limit) at `start`.
//
// With a skip grid (MIP, box lookup only), candidates are grouped G at a
// time; one test point per group (its middle candidate, computed with the
// same contract formulae) is looked up in the dilated skip grid, 64 groups
// per wave.  A chunk of 64 candidates whose groups are all clear is skipped
// without touching its candidates, and lanes in clear groups skip their
// fine lookup: their cells are empty by construction, so the sample set is
// exactly the one of the plain traversal.
template <int LOOKUP, bool FILL, bool MIP>
__device__ __forceinline__ int march_ray_uniform(
    int64_t r, const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const int32_t* __restrict__ grid_id, const uint32_t* __restrict__ bits, const uint32_t* __restrict__ mip,
    const GridK& g, const ClipK& c, const StepK& p, int64_t start, int limit, int64_t capacity,
    int32_t* __restrict__ ray_indices, float* __restrict__ t_starts, float* __restrict__ t_ends,
    bool& overflow, uint64_t* __restrict__ masks = nullptr, int n_masks = 0, int first_chunk = 0,
    int count0 = 0) {
    const int lane = lane_id();
    float o[3], d[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o[i] = rays_o[3 * r + i];
        d[i] = rays_d[3 * r + i];
    }
    uint32_t word0;
    if (!grid_of_ray<LOOKUP>(grid_id, r, g, word0)) return 0;
    float t_near, t_far;
    if (!clip_ray(o, d, c, p.near_plane, p.far_plane, t_near, t_far)) return 0;
    const uint32_t mip0 = MIP ? (word0 / g.words) * g.mip_words : 0u;
    int G = MIP ? uniform<int>(group_size(g, o, d, t_near, t_far, p.dt)) : 0;
    uint64_t live_groups = ~0ull;  // groups [window * 64, window * 64 + 64) as bits
    uint64_t live_chunks = ~0ull;  // chunks of the window as bits
    int window_chunk = -(1 << 30);  // first chunk of the current window
    uint64_t my_mask = 0ull;        // count pass: lane j keeps the ballot of chunk j
    int count = count0;
    for (int k0 = first_chunk * kWave; k0 < kMaxCandidates; k0 += kWave) {
        const int chunk = k0 / kWave;
        bool lane_live = true;
        if (MIP && G > 0) {
            if (chunk >= window_chunk + G && k0 + kWave * G > kMaxCandidates) {
                // test points past 2^24 would not be exact lattice points:
                // plain traversal from here on
                G = 0;
            }
        }
        if (MIP && G > 0) {
            if (chunk >= window_chunk + G) {
                // new window: 64 groups of G candidates = G chunks
                window_chunk = chunk;
                const int kt = k0 + lane * G + G / 2;
                const float a0 = t_near + static_cast<float>(kt) * p.dt;
                const float a1 = t_near + static_cast<float>(kt + 1) * p.dt;
                const float am = (a0 + a1) * 0.5f;
                uint32_t j0, j1, j2;
                cell_indices(g, o[0] + d[0] * am, o[1] + d[1] * am, o[2] + d[2] * am, j0, j1, j2);
                live_groups = ballot(skip_bit(mip, mip0, g, j0, j1, j2));
                const int per_chunk = kWave / G;  // groups per chunk: 1, 2, 4 or 8
                const uint64_t group_mask = (1ull << per_chunk) - 1ull;
                live_chunks = ballot(lane < G && ((live_groups >> (lane * per_chunk)) & group_mask) != 0ull);
            }
            const int rel = chunk - window_chunk;
            if (((live_chunks >> rel) & 1ull) == 0ull) {
                // every candidate of this chunk lies in empty cells
                if (!(t_near + static_cast<float>(k0) * p.dt < t_far)) break;
                continue;
            }
            lane_live = ((live_groups >> ((rel * kWave + lane) / G)) & 1ull) != 0ull;
        }
        const int k = k0 + lane;
        const float t0 = t_near + static_cast<float>(k) * p.dt;
        const bool live = t0 < t_far;
        if (ballot(live) == 0) break;  // t_k is non-decreasing in k
        const float t1 = t_near + static_cast<float>(k + 1) * p.dt;
        const float tm = (t0 + t1) * 0.5f;
        bool hit = false;
        if (live && lane_live) {
            hit = occupied<LOOKUP>(bits, word0, g, o[0] + d[0] * tm, o[1] + d[1] * tm, o[2] + d[2] * tm);
        }
        const uint64_t m = ballot(hit);
        if (!FILL && lane == chunk) my_mask = m;
        if (FILL && hit) {
            const int idx = count + bits_below(m);
            if (idx < limit) {
                const int64_t pos = start + idx;
                if (pos >= 0 && pos < capacity) {
                    ray_indices[pos] = static_cast<int32_t>(r);
                    t_starts[pos] = t0;
                    t_ends[pos] = t1;
                } else {
                    overflow = true;
                }
            }
        }
        count += __popcll(m);
        if (p.max_per_ray > 0 && count >= p.max_per_ray) {
            count = p.max_per_ray;
            break;
        }
        if (FILL && count >= limit) break;
    }
    if (!FILL && lane < n_masks) masks[lane] = my_mask;
    return count;
}

template <int LOOKUP, bool MIP, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void count_uniform_kernel(
    const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const int32_t* __restrict__ grid_id, int64_t n_rays, const uint32_t* __restrict__ bits,
    const uint32_t* __restrict__ mip, GridK g, ClipK c, StepK p, int32_t* __restrict__ packed_info,
    int64_t* __restrict__ block_sums, uint64_t* __restrict__ masks, int n_masks) {
    __shared__ int64_t wave_total[WAVES];
    const int wave = uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kRaysPerBlock;
    int64_t total = 0;
    bool unused = false;
    for (int i = wave; i < kRaysPerBlock; i += WAVES) {
        const int64_t r = first + i;
        if (r >= n_rays) break;
        const int n = march_ray_uniform<LOOKUP, false, MIP>(
            r, rays_o, rays_d, grid_id, bits, mip, g, c, p, 0, 0, 0, nullptr, nullptr, nullptr, unused,
            masks != nullptr ? masks + r * n_masks : nullptr, masks != nullptr ? n_masks : 0);
        if (lane_id() == 0) packed_info[2 * r + 1] = n;
        total += n;
    }
    if (lane_id() == 0) wave_total[wave] = total;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int w = 0; w < WAVES; ++w) s += wave_total[w];
        block_sums[blockIdx.x] = s;
    }
}

// Writes the samples of one ray from the per-chunk occupancy masks stored by
// the count pass (the first n_masks chunks), so the grid is not traversed a
// second time; a ray whose samples continue past those chunks is traversed
// from there on.
template <int LOOKUP, bool MIP>
__device__ __forceinline__ void fill_ray_from_masks(
    int64_t r, const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const int32_t* __restrict__ grid_id, const uint32_t* __restrict__ bits, const uint32_t* __restrict__ mip,
    const GridK& g, const ClipK& c, const StepK& p, int64_t start, int limit, int64_t capacity,
    int32_t* __restrict__ ray_indices, float* __restrict__ t_starts, float* __restrict__ t_ends, bool& overflow,
    const uint64_t* __restrict__ masks, int n_masks) {
    const int lane = lane_id();
    float o[3], d[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o[i] = rays_o[3 * r + i];
        d[i] = rays_d[3 * r + i];
    }
    float t_near, t_far;
    clip_ray(o, d, c, p.near_plane, p.far_plane, t_near, t_far);
    const uint64_t mine = lane < n_masks ? masks[lane] : 0ull;  // one load: lane j holds chunk j
    int written = 0;
    for (int j = 0; j < n_masks && written < limit; ++j) {
        const uint64_t m = (static_cast<uint64_t>(static_cast<uint32_t>(
                                __builtin_amdgcn_readlane(static_cast<int>(mine >> 32), j)))
                            << 32) |
                           static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(mine), j));
        if (m == 0ull) continue;
        if ((m >> lane) & 1ull) {
            const int idx = written + bits_below(m);
            if (idx < limit) {
                const int k = j * kWave + lane;
                const int64_t pos = start + idx;
                if (pos >= 0 && pos < capacity) {
                    ray_indices[pos] = static_cast<int32_t>(r);
                    t_starts[pos] = t_near + static_cast<float>(k) * p.dt;
                    t_ends[pos] = t_near + static_cast<float>(k + 1) * p.dt;
                } else {
                    overflow = true;
                }
            }
        }
        written += __popcll(m);
    }
    if (written < limit) {
        march_ray_uniform<LOOKUP, true, MIP>(r, rays_o, rays_d, grid_id, bits, mip, g, c, p, start, limit, capacity,
                                             ray_indices, t_starts, t_ends, overflow, nullptr, 0, n_masks, written);
    }
}

template <int LOOKUP, bool MIP, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void fill_uniform_kernel(
    const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const int32_t* __restrict__ grid_id, int64_t n_rays, const uint32_t* __restrict__ bits,
    const uint32_t* __restrict__ mip, GridK g, ClipK c, StepK p, const int32_t* __restrict__ packed_info,
    int64_t capacity, int32_t* __restrict__ ray_indices, float* __restrict__ t_starts, float* __restrict__ t_ends,
    int32_t* __restrict__ status, const uint64_t* __restrict__ masks, int n_masks) {
    const int wave = uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kRaysPerBlock;
    bool overflow = false;
    for (int i = wave; i < kRaysPerBlock; i += WAVES) {
        const int64_t r = first + i;
        if (r >= n_rays) break;
        const int64_t start = packed_info[2 * r];
        const int limit = uniform<int>(packed_info[2 * r + 1]);
        if (limit == 0) continue;
        if (masks != nullptr) {
            fill_ray_from_masks<LOOKUP, MIP>(r, rays_o, rays_d, grid_id, bits, mip, g, c, p, start, limit, capacity,
                                             ray_indices, t_starts, t_ends, overflow, masks + r * n_masks, n_masks);
        } else {
            march_ray_uniform<LOOKUP, true, MIP>(r, rays_o, rays_d, grid_id, bits, mip, g, c, p, start, limit,
                                                 capacity, ray_indices, t_starts, t_ends, overflow);
        }
    }
    if (overflow && status != nullptr) *status = NACC_ECAPACITY;
}

// One ray per lane, cone steps (the lattice is a recurrence in t).
template <int LOOKUP, bool FILL>
__device__ __forceinline__ int march_ray_cone(
    int64_t r, const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const int32_t* __restrict__ grid_id, const uint32_t* __restrict__ bits, const GridK& g,
    const ClipK& c, const StepK& p, int64_t start, int limit, int64_t capacity,
    int32_t* __restrict__ ray_indices, float* __restrict__ t_starts, float* __restrict__ t_ends,
    bool& overflow) {
    float o[3], d[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o[i] = rays_o[3 * r + i];
        d[i] = rays_d[3 * r + i];
    }
    uint32_t word0;
    if (!grid_of_ray<LOOKUP>(grid_id, r, g, word0)) return 0;
    float t_near, t_far;
    if (!clip_ray(o, d, c, p.near_plane, p.far_plane, t_near, t_far)) return 0;
    int count = 0;
    float t0 = t_near;
    for (int k = 0; k < kMaxCandidates; ++k) {
        if (!(t0 < t_far)) break;
        const float step = fminf(fmaxf(t0 * p.cone, p.dt), p.dt_max);
        const float t1 = t0 + step;
        if (!(t1 > t0)) break;
        const float tm = (t0 + t1) * 0.5f;
        if (occupied<LOOKUP>(bits, word0, g, o[0] + d[0] * tm, o[1] + d[1] * tm,
                             o[2] + d[2] * tm)) {
            if (p.max_per_ray > 0 && count >= p.max_per_ray) break;
            if (FILL) {
                if (count >= limit) break;
                const int64_t pos = start + count;
                if (pos >= 0 && pos < capacity) {
                    ray_indices[pos] = static_cast<int32_t>(r);
                    t_starts[pos] = t0;
                    t_ends[pos] = t1;
                } else {
                    overflow = true;
                }
            }
            ++count;
        }
        t0 = t1;
    }
    return count;
}

template <int LOOKUP>
__global__ __launch_bounds__(kRaysPerBlock) void count_cone_kernel(
    const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const int32_t* __restrict__ grid_id, int64_t n_rays, const uint32_t* __restrict__ bits,
    GridK g, ClipK c, StepK p, int32_t* __restrict__ packed_info,
    int64_t* __restrict__ block_sums) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kRaysPerBlock + threadIdx.x;
    bool unused = false;
    int n = 0;
    if (r < n_rays) {
        n = march_ray_cone<LOOKUP, false>(r, rays_o, rays_d, grid_id, bits, g, c, p, 0, 0, 0,
                                          nullptr, nullptr, nullptr, unused);
        packed_info[2 * r + 1] = n;
    }
    const int s = wave_sum(n);  // <= 64 * 2^24 fits int32
    if (threadIdx.x == 0) block_sums[blockIdx.x] = s;
}

template <int LOOKUP>
__global__ __launch_bounds__(kRaysPerBlock) void fill_cone_kernel(
    const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const int32_t* __restrict__ grid_id, int64_t n_rays, const uint32_t* __restrict__ bits,
    GridK g, ClipK c, StepK p, const int32_t* __restrict__ packed_info, int64_t capacity,
    int32_t* __restrict__ ray_indices, float* __restrict__ t_starts, float* __restrict__ t_ends,
    int32_t* __restrict__ status) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kRaysPerBlock + threadIdx.x;
    if (r >= n_rays) return;
    const int limit = packed_info[2 * r + 1];
    if (limit == 0) return;
    bool overflow = false;
    march_ray_cone<LOOKUP, true>(r, rays_o, rays_d, grid_id, bits, g, c, p, packed_info[2 * r],
                                 limit, capacity, ray_indices, t_starts, t_ends, overflow);
    if (overflow && status != nullptr) *status = NACC_ECAPACITY;
}

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

__global__ void set_status_kernel(int32_t* status, int32_t value) { *status = value; }

// --------------------------------------------------------------------------
// Host side: validation and launch.
// --------------------------------------------------------------------------

int64_t num_blocks(int64_t n_rays) { return (n_rays + kRaysPerBlock - 1) / kRaysPerBlock; }

constexpr int kMaxMaskChunks = 32;

// Workspace of the marching calls: the per-workgroup sums of the scan, then
// (uniform steps only) n_masks 64-bit occupancy masks per ray, one per chunk
// of 64 candidates, written by the count pass and replayed by the fill pass.
// n_masks covers the longest chord of the clip box (or far - near) in steps.
struct Layout {
    int64_t sums_bytes;
    int n_masks;
    int64_t bytes;
};

Layout workspace_layout(int64_t n_rays, const nacc_grid_desc& grid, const nacc_march_params& p) {
    Layout l;
    l.sums_bytes = ((num_blocks(n_rays) * static_cast<int64_t>(sizeof(int64_t)) + 255) / 256) * 256;
    l.n_masks = 0;
    if (p.cone == 0.0f && p.dt > 0.0f) {
        double span = static_cast<double>(p.far_plane) - static_cast<double>(p.near_plane);
        if (grid.lookup != NACC_LOOKUP_CONTRACT) {
            const double scale = grid.lookup == NACC_LOOKUP_CASCADE ? std::ldexp(1.0, grid.n_grids - 1) : 1.0;
            double d2 = 0.0;
            for (int i = 0; i < 3; ++i) {
                const double e = (static_cast<double>(grid.hi[i]) - static_cast<double>(grid.lo[i])) * scale;
                d2 += e * e;
            }
            span = std::min(span, std::sqrt(d2));
        }
        if (std::isfinite(span) && span > 0.0) {
            const double chunks = std::ceil((span / p.dt + 2.0) / kWave);
            l.n_masks = static_cast<int>(std::min<double>(chunks, kMaxMaskChunks));
        } else if (!std::isfinite(span)) {
            l.n_masks = kMaxMaskChunks;
        }
    }
    l.bytes = l.sums_bytes + n_rays * l.n_masks * static_cast<int64_t>(sizeof(uint64_t));
    return l;
}

int validate(const float* rays_o, const float* rays_d, int64_t n_rays, const uint32_t* bits,
             const nacc_grid_desc* grid, const nacc_march_params* params) {
    NACC_REQUIRE(grid != nullptr && params != nullptr, NACC_EINVAL, "grid and params must be non-NULL");
    NACC_REQUIRE(n_rays >= 0 && n_rays <= INT32_MAX, NACC_EINVAL, "n_rays = %lld out of [0, 2^31-1]",
                 static_cast<long long>(n_rays));
    NACC_REQUIRE(n_rays == 0 || (rays_o != nullptr && rays_d != nullptr && bits != nullptr),
                 NACC_EINVAL, "rays_o, rays_d and grid_bits must be non-NULL");
    const int res = grid->res;
    NACC_REQUIRE(res >= 1 && res <= 1024, NACC_EINVAL, "grid res = %d out of [1, 1024]", res);
    const int64_t cells = static_cast<int64_t>(res) * res * res;
    NACC_REQUIRE(cells % 32 == 0, NACC_ESHAPE, "res^3 = %lld is not a multiple of 32",
                 static_cast<long long>(cells));
    NACC_REQUIRE(grid->lookup >= 0 && grid->lookup <= 2, NACC_EINVAL, "unknown lookup mode %d", grid->lookup);
    NACC_REQUIRE(grid->n_grids >= 1, NACC_EINVAL, "n_grids = %d < 1", grid->n_grids);
    NACC_REQUIRE(static_cast<int64_t>(grid->n_grids) * (cells / 32) <= UINT32_MAX, NACC_ESHAPE,
                 "grid array exceeds 2^32 words");
    for (int i = 0; i < 3; ++i) {
        NACC_REQUIRE(std::isfinite(grid->lo[i]) && std::isfinite(grid->hi[i]) && grid->lo[i] < grid->hi[i],
                     NACC_EINVAL, "grid box axis %d is empty or not finite", i);
    }
    if (grid->lookup == NACC_LOOKUP_CASCADE) {
        NACC_REQUIRE(grid->n_grids <= 16, NACC_EINVAL, "cascade levels = %d > 16", grid->n_grids);
        int e = 0;
        const float b = grid->hi[0];
        NACC_REQUIRE(std::frexp(b, &e) == 0.5f, NACC_EINVAL, "cascade half-extent %g is not a power of two", b);
        for (int i = 0; i < 3; ++i) {
            NACC_REQUIRE(grid->hi[i] == b && grid->lo[i] == -b, NACC_EINVAL,
                         "cascade level-0 box must be [-b, b]^3");
        }
    }
    const nacc_march_params& p = *params;
    NACC_REQUIRE(std::isfinite(p.dt) && p.dt > 0.0f, NACC_EINVAL, "dt = %g must be finite and > 0", p.dt);
    NACC_REQUIRE(std::isfinite(p.cone) && p.cone >= 0.0f, NACC_EINVAL, "cone = %g must be finite and >= 0",
                 p.cone);
    NACC_REQUIRE(p.cone == 0.0f || p.dt_max >= p.dt, NACC_EINVAL, "dt_max = %g < dt = %g", p.dt_max, p.dt);
    NACC_REQUIRE(!std::isnan(p.near_plane) && !std::isnan(p.far_plane), NACC_EINVAL, "near/far is NaN");
    NACC_REQUIRE(p.max_per_ray >= 0, NACC_EINVAL, "max_per_ray = %d < 0", p.max_per_ray);
    return NACC_OK;
}

void make_constants(const nacc_grid_desc& grid, const nacc_march_params& params, GridK& g, ClipK& c,
                    StepK& p) {
    for (int i = 0; i < 3; ++i) {
        g.lo[i] = grid.lo[i];
        g.s[i] = axis_scale(grid.res, grid.lo[i], grid.hi[i]);
        c.lo[i] = grid.lo[i];
        c.hi[i] = grid.hi[i];
        if (grid.lookup == NACC_LOOKUP_CASCADE) {
            c.lo[i] = std::ldexp(grid.lo[i], grid.n_grids - 1);
            c.hi[i] = std::ldexp(grid.hi[i], grid.n_grids - 1);
        } else if (grid.lookup == NACC_LOOKUP_CONTRACT) {
            c.lo[i] = -INFINITY;
            c.hi[i] = INFINITY;
        }
    }
    g.top = static_cast<float>(grid.res - 1);
    g.base = grid.hi[0];
    g.res = grid.res;
    g.n_grids = grid.n_grids;
    g.words = static_cast<uint32_t>(static_cast<int64_t>(grid.res) * grid.res * grid.res / 32);
    g.coarse = grid.res / 4;
    g.mip_words = static_cast<uint32_t>(nacc_grid_mip_words(&grid) / std::max(grid.n_grids, 1));
    p.near_plane = params.near_plane;
    p.far_plane = params.far_plane;
    p.dt = params.dt;
    p.dt_max = params.dt_max;
    p.cone = params.cone;
    p.max_per_ray = params.max_per_ray;
}

template <int LOOKUP, bool MIP, int WAVES>
void launch_count_uniform(int64_t nb, hipStream_t s, const float* o, const float* d, const int32_t* gid, int64_t n,
                          const uint32_t* bits, const uint32_t* mip, const GridK& g, const ClipK& c, const StepK& p,
                          int32_t* packed, int64_t* sums, uint64_t* masks, int n_masks) {
    hipLaunchKernelGGL((count_uniform_kernel<LOOKUP, MIP, WAVES>), dim3(nb), dim3(WAVES * kWave), 0, s, o, d, gid, n,
                       bits, mip, g, c, p, packed, sums, masks, n_masks);
}

template <int LOOKUP, bool MIP, int WAVES>
void launch_fill_uniform(int64_t nb, hipStream_t s, const float* o, const float* d, const int32_t* gid, int64_t n,
                         const uint32_t* bits, const uint32_t* mip, const GridK& g, const ClipK& c, const StepK& p,
                         const int32_t* packed, int64_t capacity, int32_t* ri, float* ts, float* te, int32_t* status,
                         const uint64_t* masks, int n_masks) {
    hipLaunchKernelGGL((fill_uniform_kernel<LOOKUP, MIP, WAVES>), dim3(nb), dim3(WAVES * kWave), 0, s, o, d, gid, n,
                       bits, mip, g, c, p, packed, capacity, ri, ts, te, status, masks, n_masks);
}

template <int LOOKUP, bool MIP, typename... A>
void count_by_waves(int waves, A&&... a) {
    if (waves == 1) launch_count_uniform<LOOKUP, MIP, 1>(a...);
    else if (waves == 2) launch_count_uniform<LOOKUP, MIP, 2>(a...);
    else launch_count_uniform<LOOKUP, MIP, 4>(a...);
}

template <int LOOKUP, bool MIP, typename... A>
void fill_by_waves(int waves, A&&... a) {
    if (waves == 1) launch_fill_uniform<LOOKUP, MIP, 1>(a...);
    else if (waves == 2) launch_fill_uniform<LOOKUP, MIP, 2>(a...);
    else launch_fill_uniform<LOOKUP, MIP, 4>(a...);
}

template <int LOOKUP>
void launch_count(bool cone, int64_t nb, hipStream_t s, const float* o, const float* d, const int32_t* gid,
                  int64_t n, const uint32_t* bits, const uint32_t* mip, const GridK& g, const ClipK& c,
                  const StepK& p, int32_t* packed, int64_t* sums, uint64_t* masks, int n_masks) {
    const int waves = tuning().march_waves_per_group;
    if (cone) {
        hipLaunchKernelGGL(count_cone_kernel<LOOKUP>, dim3(nb), dim3(kRaysPerBlock), 0, s, o, d, gid, n,
                           bits, g, c, p, packed, sums);
    } else if (mip != nullptr && LOOKUP == NACC_LOOKUP_AABB) {
        count_by_waves<LOOKUP, true>(waves, nb, s, o, d, gid, n, bits, mip, g, c, p, packed, sums, masks, n_masks);
    } else {
        count_by_waves<LOOKUP, false>(waves, nb, s, o, d, gid, n, bits, mip, g, c, p, packed, sums, masks, n_masks);
    }
}

template <int LOOKUP>
void launch_fill(bool cone, int64_t nb, hipStream_t s, const float* o, const float* d, const int32_t* gid,
                 int64_t n, const uint32_t* bits, const uint32_t* mip, const GridK& g, const ClipK& c,
                 const StepK& p, const int32_t* packed, int64_t capacity, int32_t* ri, float* ts, float* te,
                 int32_t* status, const uint64_t* masks, int n_masks) {
    const int waves = tuning().march_waves_per_group;
    if (cone) {
        hipLaunchKernelGGL(fill_cone_kernel<LOOKUP>, dim3(nb), dim3(kRaysPerBlock), 0, s, o, d, gid, n, bits,
                           g, c, p, packed, capacity, ri, ts, te, status);
    } else if (mip != nullptr && LOOKUP == NACC_LOOKUP_AABB) {
        fill_by_waves<LOOKUP, true>(waves, nb, s, o, d, gid, n, bits, mip, g, c, p, packed, capacity, ri, ts, te,
                                    status, masks, n_masks);
    } else {
        fill_by_waves<LOOKUP, false>(waves, nb, s, o, d, gid, n, bits, mip, g, c, p, packed, capacity, ri, ts, te,
                                     status, masks, n_masks);
    }
}

// The skip grid is used by uniform steps with the box lookup and needs
// res % 4 == 0; anything else marches without it.
const uint32_t* usable_mip(const uint32_t* mip, const nacc_grid_desc& grid, const nacc_march_params& p) {
    if (mip == nullptr || grid.lookup != NACC_LOOKUP_AABB || p.cone != 0.0f || grid.res % 4 != 0) return nullptr;
    return mip;
}

}  // namespace

extern "C" {

int64_t nacc_march_workspace_size(int64_t n_rays, const nacc_grid_desc* grid, const nacc_march_params* params) {
    clear_error();
    if (n_rays < 0 || grid == nullptr || params == nullptr) return -1;
    if (validate(nullptr, nullptr, 0, nullptr, grid, params) != NACC_OK) return -1;
    return workspace_layout(n_rays, *grid, *params).bytes;
}

int nacc_march_count(const float* rays_o, const float* rays_d, const int32_t* grid_id, int64_t n_rays,
                     const uint32_t* grid_bits, const uint32_t* grid_mip, const nacc_grid_desc* grid,
                     const nacc_march_params* params,
                     int32_t* packed_info, int64_t* total, void* workspace, size_t workspace_bytes,
                     void* stream) {
    clear_error();
    int st = validate(rays_o, rays_d, n_rays, grid_bits, grid, params);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(total != nullptr, NACC_EINVAL, "total must be non-NULL");
    NACC_REQUIRE(n_rays == 0 || packed_info != nullptr, NACC_EINVAL, "packed_info must be non-NULL");
    const Layout lay = workspace_layout(n_rays, *grid, *params);
    const int64_t need = lay.bytes;
    NACC_REQUIRE(need == 0 || workspace != nullptr, NACC_EINVAL, "workspace must be non-NULL");
    NACC_REQUIRE(static_cast<int64_t>(workspace_bytes) >= need, NACC_ESHAPE,
                 "workspace of %zu bytes, need %lld", workspace_bytes, static_cast<long long>(need));
    uint64_t* masks = lay.n_masks > 0 ? reinterpret_cast<uint64_t*>(static_cast<char*>(workspace) + lay.sums_bytes)
                                      : nullptr;
    GridK g;
    ClipK c;
    StepK p;
    make_constants(*grid, *params, g, c, p);
    hipStream_t s = as_stream(stream);
    const int64_t nb = num_blocks(n_rays);
    int64_t* sums = static_cast<int64_t*>(workspace);
    const bool cone = params->cone > 0.0f;
    const uint32_t* mip = usable_mip(grid_mip, *grid, *params);
    if (nb > 0) {
        switch (grid->lookup) {
            case NACC_LOOKUP_AABB:
                launch_count<NACC_LOOKUP_AABB>(cone, nb, s, rays_o, rays_d, grid_id, n_rays, grid_bits, mip, g, c, p,
                                               packed_info, sums, masks, lay.n_masks);
                break;
            case NACC_LOOKUP_CASCADE:
                launch_count<NACC_LOOKUP_CASCADE>(cone, nb, s, rays_o, rays_d, grid_id, n_rays, grid_bits, mip, g, c,
                                                  p, packed_info, sums, masks, lay.n_masks);
                break;
            default:
                launch_count<NACC_LOOKUP_CONTRACT>(cone, nb, s, rays_o, rays_d, grid_id, n_rays, grid_bits, mip, g,
                                                   c, p, packed_info, sums, masks, lay.n_masks);
                break;
        }
        st = check_launch("march count");
        if (st != NACC_OK) return st;
    }
    hipLaunchKernelGGL(scan_block_sums_kernel, dim3(1), dim3(kScanThreads), 0, s, sums, nb, total);
    st = check_launch("march scan");
    if (st != NACC_OK) return st;
    if (nb > 0) {
        hipLaunchKernelGGL(finalize_starts_kernel, dim3(nb), dim3(kRaysPerBlock), 0, s, sums, n_rays,
                           packed_info);
        st = check_launch("march starts");
    }
    return st;
}

int nacc_march_fill(const float* rays_o, const float* rays_d, const int32_t* grid_id, int64_t n_rays,
                    const uint32_t* grid_bits, const uint32_t* grid_mip, const nacc_grid_desc* grid,
                    const nacc_march_params* params,
                    const int32_t* packed_info, const void* workspace, size_t workspace_bytes, int64_t capacity,
                    int32_t* ray_indices, float* t_starts, float* t_ends, int32_t* status, void* stream) {
    clear_error();
    int st = validate(rays_o, rays_d, n_rays, grid_bits, grid, params);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(capacity >= 0 && capacity <= INT32_MAX, NACC_ECAPACITY,
                 "capacity = %lld out of [0, 2^31-1]", static_cast<long long>(capacity));
    NACC_REQUIRE(n_rays == 0 || packed_info != nullptr, NACC_EINVAL, "packed_info must be non-NULL");
    NACC_REQUIRE(capacity == 0 || (ray_indices != nullptr && t_starts != nullptr && t_ends != nullptr),
                 NACC_EINVAL, "sample outputs must be non-NULL");
    GridK g;
    ClipK c;
    StepK p;
    make_constants(*grid, *params, g, c, p);
    hipStream_t s = as_stream(stream);
    if (status != nullptr) {
        hipLaunchKernelGGL(set_status_kernel, dim3(1), dim3(1), 0, s, status, static_cast<int32_t>(NACC_OK));
        st = check_launch("march status");
        if (st != NACC_OK) return st;
    }
    const int64_t nb = num_blocks(n_rays);
    if (nb == 0) return NACC_OK;
    const bool cone = params->cone > 0.0f;
    const uint32_t* mip = usable_mip(grid_mip, *grid, *params);
    const Layout lay = workspace_layout(n_rays, *grid, *params);
    NACC_REQUIRE(workspace == nullptr || static_cast<int64_t>(workspace_bytes) >= lay.bytes, NACC_ESHAPE,
                 "workspace of %zu bytes, need %lld", workspace_bytes, static_cast<long long>(lay.bytes));
    const uint64_t* masks =
        workspace != nullptr && lay.n_masks > 0
            ? reinterpret_cast<const uint64_t*>(static_cast<const char*>(workspace) + lay.sums_bytes)
            : nullptr;
    switch (grid->lookup) {
        case NACC_LOOKUP_AABB:
            launch_fill<NACC_LOOKUP_AABB>(cone, nb, s, rays_o, rays_d, grid_id, n_rays, grid_bits, mip, g, c, p,
                                          packed_info, capacity, ray_indices, t_starts, t_ends, status, masks, lay.n_masks);
            break;
        case NACC_LOOKUP_CASCADE:
            launch_fill<NACC_LOOKUP_CASCADE>(cone, nb, s, rays_o, rays_d, grid_id, n_rays, grid_bits, mip, g, c, p,
                                             packed_info, capacity, ray_indices, t_starts, t_ends, status, masks, lay.n_masks);
            break;
        default:
            launch_fill<NACC_LOOKUP_CONTRACT>(cone, nb, s, rays_o, rays_d, grid_id, n_rays, grid_bits, mip, g, c, p,
                                              packed_info, capacity, ray_indices, t_starts, t_ends, status, masks, lay.n_masks);
            break;
    }
    return check_launch("march fill");
}

}  // extern "C"
