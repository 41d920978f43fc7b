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
// Empty space: with a skip field (nacc_grid_build_skip), a test at one
// candidate's midpoint gives a stretch of t ahead in which every candidate
// midpoint is sure to fall in empty cells of the same grid level; those
// candidates are passed over without grid lookups.  The bound allows for
// the FP32 rounding of positions, so the sample set is exactly the one of
// the plain traversal.
//
// All lattice arithmetic follows the FP32 contract in nacc.h: this file is
// compiled with -ffp-contract=off and `fp contract(off)`, and uses only
// correctly rounded + - * / sqrt, min/max, ldexp and float->int truncation of
// non-negative values.
#include <cmath>

#include "common.h"
#include "lattice.h"
#include "scan.h"

#pragma clang fp contract(off)

namespace {

using namespace nacc;
using namespace nacc::dev;

// Per-ray constants of the skip-field test.
//   slack_x: allowance for the FP32 rounding of sample positions: two
//            positions of the ray differ by at most |d_i| |tm_k - tm_0| plus
//            slack_x on every axis (a few ulps of the largest coordinate the
//            ray reaches, taken generously);
//   inv_v:   1 / (fine cells per unit t on the fastest axis, at level 0);
//   inv_dmax: 1 / max_i |d_i|.
//   contraction lookup: t_out, from which on the ray moves away from the
//   origin (past its closest approach, rounded up), |d| rounded up, the
//   largest |o_i|, |d_i| and the grid's largest cells-per-unit scale.
struct SkipRay {
    float slack_x;
    float slack_s;  // slack_x in fine cells at level 0
    float inv_v;
    float inv_dmax;
    float t_out, dnorm, omax, dmax, smax;
};

__device__ __forceinline__ SkipRay skip_ray(const GridK& g, const float o[3], const float d[3], float t_far) {
    SkipRay k;
    const float omax = fmaxf(fmaxf(fabsf(o[0]), fabsf(o[1])), fabsf(o[2]));
    const float dmax = fmaxf(fmaxf(fabsf(d[0]), fabsf(d[1])), fabsf(d[2]));
    k.slack_x = (omax + dmax * fabsf(t_far) + 1.0f) * 0x1p-20f;
    const float smax = fmaxf(fmaxf(g.s[0], g.s[1]), g.s[2]);
    k.slack_s = smax * k.slack_x;
    k.inv_v = 1.0f / fmaxf(fmaxf(g.s[0] * fabsf(d[0]), g.s[1] * fabsf(d[1])), g.s[2] * fabsf(d[2]));
    k.inv_dmax = 1.0f / dmax;
    const float dd = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    const float od = (o[0] * d[0] + o[1] * d[1]) + o[2] * d[2];
    const float t_star = -od / dd;
    k.t_out = t_star + (fabsf(t_star) + 1.0f) * 0x1p-16f;
    k.dnorm = sqrtf(dd) * (1.0f + 0x1p-18f);
    k.omax = omax;
    k.dmax = dmax;
    k.smax = smax;
    return k;
}

// Contraction lookup: the end of the stretch past tm whose candidates all
// map to empty fine cells.  The contraction c(x) = (2 - 1/|x|) x/|x| is
// Lipschitz with constant L(r) = (2 - 1/r)/r on |x| >= r >= 1 (its
// derivative stretches tangential directions by that factor and the radial
// one by 1/r^2 <= L(r); L <= 1 everywhere).  Past the closest approach |x|
// only grows along the ray, so candidates a distance D_t further along t
// map within L(r) |d| D_t of c(x(tm)), r a lower bound of |x(tm)|; before
// it L = 1.  The byte `dist` guarantees empty fine cells within
// 4 (dist - 1) cells on every axis; the stretch is kept inside that after
// allowing for the FP32 rounding of positions (a few ulps of the largest
// coordinate reached, at most 2 tm + 1 along the ray: the stretch is capped
// there) and of the contraction (2^-16 in contracted units).
__device__ __forceinline__ float skip_end_contract(const SkipRay& k, const Probe& q, int dist, float tm, int res) {
    float lip = 1.0f;
    if (tm > k.t_out) {
        const float t_reach = 2.0f * fabsf(tm) + 1.0f;
        const float slack = (k.omax + k.dmax * t_reach + 1.0f) * 0x1p-20f;
        const float r = q.m * (1.0f - 0x1p-18f) - 2.0f * slack;
        if (r > 1.0f) lip = ((2.0f - 1.0f / r) / r) * (1.0f + 0x1p-18f);
    }
    const float slack_pos = (k.omax + k.dmax * (2.0f * fabsf(tm) + 1.0f) + 1.0f) * 0x1p-20f;
    const float slack_cells = k.smax * 3.5f * (lip * slack_pos + 0x1p-16f) + static_cast<float>(res) * 0x1p-18f;
    const float budget = 4.0f * static_cast<float>(dist - 1) - slack_cells;
    float span = budget / (k.smax * lip * k.dnorm);
    span = fminf(span, fabsf(tm) + 1.0f);  // the reach the slack allows for
    span = span * (1.0f - 0x1p-10f) - fabsf(tm) * 0x1p-21f;
    return (dist >= 2 && span > 0.0f) ? tm + span : -INFINITY;
}

// End (in t) of the stretch past the candidate midpoint tm over which every
// candidate midpoint of the ray falls in an empty fine cell, from the skip
// byte `dist` of tm's coarse cell (probe q); -inf if there is none.  The
// byte bounds the stretch at 4 (dist - 1) fine cells on every axis of q's
// grid level; a cascade stretch also ends before the point could change
// level.  Rounding margins keep the bound strict.
template <int LOOKUP>
__device__ __forceinline__ float skip_end_at(const GridK& g, const SkipRay& k, const Probe& q, int dist, float tm) {
    if (LOOKUP == NACC_LOOKUP_CONTRACT) return skip_end_contract(k, q, dist, tm, g.res);
    // fine cells at level l are 2^l times larger: the slack in fine cells
    // shrinks and the stretch in t grows by 2^l
    const float budget =
        4.0f * static_cast<float>(dist - 1) - (ldexpf(k.slack_s, -q.level) + static_cast<float>(g.res) * 0x1p-18f);
    float span = ldexpf(budget * k.inv_v, q.level);
    if (LOOKUP == NACC_LOOKUP_CASCADE) {
        float room = INFINITY;
        if (q.level < g.n_grids - 1) room = fminf(room, ldexpf(g.base, q.level) - q.m);
        if (q.level > 0) room = fminf(room, q.m - ldexpf(g.base, q.level - 1));
        span = fminf(span, (room - k.slack_x) * k.inv_dmax);
    }
    span = span * (1.0f - 0x1p-10f) - fabsf(tm) * 0x1p-21f;
    return (dist >= 2 && span > 0.0f) ? tm + span : -INFINITY;
}

// DPP move that leaves a lane's own value where the source lane is out of
// range or its row is masked off (the identity for max).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_or_self(float v) {
    const int b = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, CTRL, ROW_MASK, 0xf, false));
}

// Maximum over the 64 lanes (every lane active): prefix maxima within each
// row of 16 lanes, then the row maxima carried by two row broadcasts.
__device__ __forceinline__ float wave_max(float x) {
    x = fmaxf(x, dpp_or_self<kRowShr1>(x));
    x = fmaxf(x, dpp_or_self<kRowShr2>(x));
    x = fmaxf(x, dpp_or_self<kRowShr4>(x));
    x = fmaxf(x, dpp_or_self<kRowShr8>(x));
    x = fmaxf(x, dpp_or_self<kRowBcast15, 0xa>(x));
    x = fmaxf(x, dpp_or_self<kRowBcast31, 0xc>(x));
    return read_lane(x, kWave - 1);
}

// Chunk masks of the count pass, one per lane: lane j holds the ballot of
// chunk j (as two 32-bit halves).  The chunk index and the ballot are
// wave-uniform, so the ballot is written into lane j directly.
struct ChunkMasks {
    int lo = 0, hi = 0;
    __device__ __forceinline__ void keep(int chunk, uint64_t m) {
        if (chunk < kWave) {
            const uint32_t m_lo = static_cast<uint32_t>(m), m_hi = static_cast<uint32_t>(m >> 32);
            // one scalar operand per instruction: the lane select goes in m0
            asm volatile("v_writelane_b32 %0, %1, m0" : "+v"(lo) : "s"(m_lo), "{m0}"(chunk));
            asm volatile("v_writelane_b32 %0, %1, m0" : "+v"(hi) : "s"(m_hi), "{m0}"(chunk));
        }
    }
    __device__ __forceinline__ uint64_t mine() const {
        return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
    }
};

// Uniform steps without the skip field, two chunks of 64 candidates per
// iteration: both chunks' grid words are loaded before either is tested, so
// each wave keeps two lookups in flight instead of waiting on one at a time
// (a chunk past the ray's end is looked up and ignored; its cell indices are
// clamped into the grid like any other).  Same samples, same order, same
// masks as one chunk at a time.
template <int LOOKUP, bool FILL>
__device__ __forceinline__ int march_ray_uniform_x2(
    int64_t r, const RaySpan& span, const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const uint32_t* __restrict__ bits, const GridK& g, const StepK& p, int64_t start, int limit,
    int64_t capacity, int32_t* __restrict__ ray_indices, float* __restrict__ t_starts, float* __restrict__ t_ends,
    bool& overflow, uint64_t* __restrict__ masks, int n_masks, int first_chunk, int count0) {
    if (!span.valid) return 0;
    const int lane = lane_id();
    const float* o = span.o;
    const float* d = span.d;
    const uint32_t word0 = span.word0;
    const float t_near = span.t_near, t_far = span.t_far;
    ChunkMasks my_masks;  // count pass
    int count = count0;
    bool done = false;
    for (int k0 = first_chunk * kWave; k0 < kMaxCandidates && !done; k0 += 2 * kWave) {
        float t0[2], t1[2];
        uint64_t live[2];  // ballots of t0 < t_far
        uint64_t ms[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int k = k0 + u * kWave + lane;
            t0[u] = t_near + static_cast<float>(k) * p.dt;
            live[u] = ballot(t0[u] < t_far);
            t1[u] = t_near + static_cast<float>(k + 1) * p.dt;
        }
        if (live[0] == 0ull) break;  // t_k is non-decreasing in k
        // both words are loaded, and both ballots taken, before any branch
        // on them (a ballot cannot move into a branch)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const float tm = (t0[u] + t1[u]) * 0.5f;
            const Probe q = probe<LOOKUP>(g, word0, o[0] + d[0] * tm, o[1] + d[1] * tm, o[2] + d[2] * tm);
            const uint32_t w = grid_word(grid_rsrc(bits, g), q.word);  // every lane: the index is clamped into the grid
            // ballots of plain comparisons, combined as masks (a ballot of
            // a combined condition costs two more vector instructions)
            ms[u] = live[u] & ballot(((w >> q.bit) & 1u) != 0u);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int chunk = k0 / kWave + u;
            if (u == 1 && (live[1] == 0ull || k0 + kWave >= kMaxCandidates)) {
                done = true;
                break;
            }
            const uint64_t m = ms[u];
            const bool hit = ((m >> lane) & 1ull) != 0ull;
            if (!FILL) my_masks.keep(chunk, m);
            if (FILL && hit) {
                const int idx = count + bits_below(m);
                if (idx < limit) {
                    const int64_t pos = start + idx;
                    if (pos >= 0 && pos < capacity) {
                        ray_indices[pos] = static_cast<int32_t>(r);
                        t_starts[pos] = t0[u];
                        t_ends[pos] = t1[u];
                    } else {
                        overflow = true;
                    }
                }
            }
            count += __popcll(m);
            if (p.max_per_ray > 0 && count >= p.max_per_ray) {
                count = p.max_per_ray;
                done = true;
                break;
            }
            if (FILL && count >= limit) {
                done = true;
                break;
            }
        }
    }
    if (!FILL && lane < n_masks) masks[lane] = my_masks.mine();
    return count;
}

// One ray, uniform steps, whole wave.  Returns the ray's sample count (the
// same value in every lane).  FILL writes samples [0, limit) at `start`.
// With SKIP, candidates inside a stretch the skip field clears are not
// looked up; a chunk of 64 candidates that lies wholly inside one is passed
// over at the cost of its lattice arithmetic.
template <int LOOKUP, bool FILL, bool SKIP>
__device__ __forceinline__ int march_ray_uniform(
    int64_t r, const RaySpan& span, const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const uint32_t* __restrict__ bits, const uint8_t* __restrict__ skip,
    const GridK& g, const StepK& p, int64_t start, int limit, int64_t capacity,
    int32_t* __restrict__ ray_indices, float* __restrict__ t_starts, float* __restrict__ t_ends,
    bool& overflow, uint64_t* __restrict__ masks = nullptr, int n_masks = 0, int first_chunk = 0,
    int count0 = 0) {
    if constexpr (!SKIP) {
        return march_ray_uniform_x2<LOOKUP, FILL>(r, span, rays_o, rays_d, bits, g, p, start, limit, capacity,
                                                  ray_indices, t_starts, t_ends, overflow, masks, n_masks,
                                                  first_chunk, count0);
    }
    if (!span.valid) return 0;
    const int lane = lane_id();
    const float* o = span.o;
    const float* d = span.d;
    const uint32_t word0 = span.word0;
    const float t_near = span.t_near, t_far = span.t_far;
    SkipRay sk{};
    if (SKIP) sk = skip_ray(g, o, d, t_far);
    float skip_end = -INFINITY;  // candidates with midpoint below it are empty
    ChunkMasks my_masks;         // count pass
    int count = count0;
    for (int k0 = first_chunk * kWave; k0 < kMaxCandidates; k0 += kWave) {
        const int chunk = k0 / kWave;
        const int k = k0 + lane;
        const float t0 = t_near + static_cast<float>(k) * p.dt;
        const bool live = t0 < t_far;
        if (ballot(live) == 0) break;  // t_k is non-decreasing in k
        const float t1 = t_near + static_cast<float>(k + 1) * p.dt;
        const float tm = (t0 + t1) * 0.5f;
        const bool todo = live && !(tm < skip_end);
        bool hit = false;
        if (ballot(todo) != 0ull) {
            // every lane probes its candidate (the index is in range whatever
            // the candidate), so the grid word and the skip byte are loaded
            // together; lanes inside a cleared stretch ignore the word
            const Probe q = probe<LOOKUP>(g, word0, o[0] + d[0] * tm, o[1] + d[1] * tm, o[2] + d[2] * tm);
            const uint32_t w = grid_word(grid_rsrc(bits, g), q.word);
            if (SKIP) {
                const int dist = skip[q.coarse];
                const float e = live ? skip_end_at<LOOKUP>(g, sk, q, dist, tm) : -INFINITY;
                // the stretches start at this chunk's candidates, so any of
                // them that reaches past the chunk covers the next candidates
                skip_end = fmaxf(skip_end, wave_max(e));
            }
            hit = todo && ((w >> q.bit) & 1u) != 0u;
        }
        const uint64_t m = ballot(hit);
        if (!FILL) my_masks.keep(chunk, m);
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
    if (!FILL && lane < n_masks) masks[lane] = my_masks.mine();
    return count;
}

// Count pass of one ray by segments (whole wave): looks up every candidate
// of the live segments, 64 at a time.  The occupancy ballots are turned
// back into the plain traversal's chunk masks (chunk j: candidates
// [64 j, 64 j + 64)), so the fill pass replays them exactly as it does for
// the plain traversal: each segment's G bits lie inside one chunk (G
// divides 64, segments are aligned to G), and the first lane of each
// segment ORs them into that chunk's mask in this wave's LDS slice
// (`chunk_masks`, 64 entries; chunks from n_masks on are not stored and the
// fill traverses them again).  `list` is this wave's 64-byte LDS slice for
// a block's live segments.  Returns the ray's count.
__device__ __forceinline__ int count_ray_segments(const RaySpan& span, const uint32_t* __restrict__ bits,
                                                  const uint32_t* __restrict__ halo, const GridK& g,
                                                  const StepK& p, const SegRay& sg, uint8_t* list,
                                                  uint64_t* chunk_masks, uint64_t* __restrict__ masks,
                                                  int n_masks) {
    const int lane = lane_id();
    const int log_g = sg.log_g;
    const int gmask = (1 << log_g) - 1;
    const int per_iter = kWave >> log_g;  // segments per wave iteration
    const uint64_t field = (1ull << (1 << log_g)) - 1ull;
    chunk_masks[lane] = 0ull;
    int count = 0;
    bool done = false;
    for (int b = 0; !done; ++b) {
        uint64_t vm;
        const uint64_t lm = live_segments(span, halo, g, p, sg, b, vm);
        if (vm == 0ull) break;  // t at a segment's first candidate is non-decreasing in j
        if (((lm >> lane) & 1ull) != 0ull) list[bits_below(lm)] = static_cast<uint8_t>(lane);
        wave_lds_sync();
        const int n_live = static_cast<int>(__popcll(lm));
        // two chunks per iteration, both chunks' grid words in flight before
        // either is tested (a chunk past the live segments looks up clamped
        // cells and counts nothing)
        for (int q = 0; q < n_live && !done; q += 2 * per_iter) {
            int k[2];
            float t0[2], t1[2];
            uint64_t alive[2], m[2];
            Probe pq[2];
            uint32_t w[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int slot = q + u * per_iter + (lane >> log_g);
                const bool in = slot < n_live;
                const int seg = in ? static_cast<int>(list[slot]) : 0;
                k[u] = ((b * kWave + seg) << log_g) + (lane & gmask);
                t0[u] = span.t_near + static_cast<float>(k[u]) * p.dt;
                t1[u] = span.t_near + static_cast<float>(k[u] + 1) * p.dt;
                alive[u] = ballot(in && t0[u] < span.t_far);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float tm = (t0[u] + t1[u]) * 0.5f;
                pq[u] = probe<NACC_LOOKUP_AABB>(g, span.word0, span.o[0] + span.d[0] * tm,
                                                span.o[1] + span.d[1] * tm, span.o[2] + span.d[2] * tm);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) w[u] = grid_word(grid_rsrc(bits, g), pq[u].word);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                m[u] = alive[u] & ballot(((w[u] >> pq[u].bit) & 1u) != 0u);
                if ((lane & gmask) == 0 && (k[u] >> kWaveLog2) < n_masks) {
                    const uint64_t part = (m[u] >> lane) & field;  // this segment's hits
                    if (part != 0ull) {
                        __hip_atomic_fetch_or(chunk_masks + (k[u] >> kWaveLog2), part << (k[u] & (kWave - 1)),
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    }
                }
            }
            count += static_cast<int>(__popcll(m[0])) + static_cast<int>(__popcll(m[1]));
            if (p.max_per_ray > 0 && count >= p.max_per_ray) {
                count = p.max_per_ray;
                done = true;
            }
        }
        if (vm != ~0ull) break;  // the ray's segments end in this block
        wave_lds_sync();         // the list is written again by the next block
    }
    wave_lds_sync();
    if (masks != nullptr && lane < n_masks) masks[lane] = chunk_masks[lane];
    wave_lds_sync();  // read before the next ray clears them
    return count;
}

// The box lookup with a skip buffer marches by segments (its halo bits).
template <int LOOKUP, bool SKIP>
constexpr bool kSegments = LOOKUP == NACC_LOOKUP_AABB && SKIP;

template <int LOOKUP, bool SKIP, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void count_uniform_kernel(
    const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const int32_t* __restrict__ grid_id, int64_t n_rays, const uint32_t* __restrict__ bits,
    const uint8_t* __restrict__ skip, const uint32_t* __restrict__ halo, GridK g, ClipK c, StepK p,
    int32_t* __restrict__ packed_info, int64_t* __restrict__ block_sums, uint64_t* __restrict__ masks, int n_masks,
    int split) {
    __shared__ int64_t wave_total[WAVES];
    // segments: each wave's chunk masks, then its list of live segments
    __shared__ uint64_t seg_masks[kSegments<LOOKUP, SKIP> ? WAVES * kWave : 1];
    __shared__ uint8_t seg_lists[kSegments<LOOKUP, SKIP> ? WAVES * kWave : 1];
    const int wave = uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    // workgroup b takes part b % split of the group of kRaysPerBlock rays
    // b / split: per = kRaysPerBlock / split rays from `first`
    const int per = kRaysPerBlock / split;
    const int64_t group = static_cast<int64_t>(blockIdx.x) / split;
    const int64_t first = group * kRaysPerBlock + static_cast<int64_t>(blockIdx.x % split) * per;
    // this wave's rays are first + wave + j WAVES; lane j clips ray j
    const int64_t mine = first + wave + static_cast<int64_t>(lane_id()) * WAVES;
    RaySpan spans{};
    if (wave + lane_id() * WAVES < per && mine < n_rays) {
        spans = ray_span<LOOKUP>(mine, rays_o, rays_d, grid_id, g, c, p);
    }
    int64_t total = 0;
    bool unused = false;
    for (int i = wave; i < per; i += WAVES) {
        const int64_t r = first + i;
        if (r >= n_rays) break;
        const RaySpan span = read_span(spans, i / WAVES);
        uint64_t* ray_masks = masks != nullptr ? masks + r * n_masks : nullptr;
        const int ray_n_masks = masks != nullptr ? n_masks : 0;
        int n;
        if constexpr (kSegments<LOOKUP, SKIP>) {
            const SegRay sg = span.valid ? seg_ray(g, span, p) : SegRay{0, 0u};
            if (sg.log_g != 0) {
                n = count_ray_segments(span, bits, halo, g, p, sg, seg_lists + wave * kWave,
                                       seg_masks + wave * kWave, ray_masks, ray_n_masks);
            } else {
                n = march_ray_uniform<LOOKUP, false, false>(r, span, rays_o, rays_d, bits, skip, g, p, 0, 0, 0,
                                                            nullptr, nullptr, nullptr, unused, ray_masks,
                                                            ray_n_masks);
            }
        } else {
            n = march_ray_uniform<LOOKUP, false, SKIP>(r, span, rays_o, rays_d, bits, skip, g, p, 0, 0, 0, nullptr,
                                                       nullptr, nullptr, unused, ray_masks, ray_n_masks);
        }
        if (lane_id() == 0) packed_info[2 * r + 1] = n;
        total += n;
    }
    if (lane_id() == 0) wave_total[wave] = total;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int w = 0; w < WAVES; ++w) s += wave_total[w];
        if (split == 1) {
            block_sums[group] = s;
        } else {  // the group's parts add up (integers: exact in any order)
            atomicAdd(reinterpret_cast<unsigned long long*>(block_sums + group), static_cast<unsigned long long>(s));
        }
    }
}

// Zeroes the per-group sums that the parts of split groups add into (a
// kernel, not a memset node, so that captured graphs replay it faithfully).
__global__ __launch_bounds__(256) void zero_sums_kernel(int64_t* __restrict__ sums, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) sums[i] = 0;
}

// The fill pass writes the samples of a ray from the per-chunk occupancy
// masks stored by the count pass (the first n_masks chunks), so the grid is
// not traversed a second time; a ray whose samples continue past those
// chunks is traversed from there on.
// The samples of the stored chunks of one ray (lane j of `mine` holds
// chunk j's mask), up to `limit`; only the chunks holding samples are
// visited, in order.  Returns the number written (or, CHECKED, taken).
template <bool CHECKED>
__device__ __forceinline__ int fill_chunks(int64_t r, float t_near, float dt, int64_t start, int limit,
                                           int64_t capacity, int32_t* __restrict__ ray_indices,
                                           float* __restrict__ t_starts, float* __restrict__ t_ends, bool& overflow,
                                           uint64_t mine) {
    const int lane = lane_id();
    int written = 0;
    for (uint64_t todo = ballot(mine != 0ull); todo != 0ull && written < limit; todo &= todo - 1ull) {
        const int j = static_cast<int>(__builtin_ctzll(todo));
        const uint64_t m = (static_cast<uint64_t>(static_cast<uint32_t>(
                                __builtin_amdgcn_readlane(static_cast<int>(mine >> 32), j)))
                            << 32) |
                           static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(mine), j));
        const int pc = static_cast<int>(__popcll(m));
        const int n_take = pc < limit - written ? pc : limit - written;
        const int rank = bits_below(m);
        if (((m >> lane) & 1ull) != 0ull && rank < n_take) {
            const int k = j * kWave + lane;
            const float t0 = t_near + static_cast<float>(k) * dt;
            const float t1 = t_near + static_cast<float>(k + 1) * dt;
            if (!CHECKED) {
                // wave-uniform bases, 32-bit lane offsets
                const int64_t base = start + written;
                const uint32_t off = static_cast<uint32_t>(rank);
                (ray_indices + base)[off] = static_cast<int32_t>(r);
                (t_starts + base)[off] = t0;
                (t_ends + base)[off] = t1;
            } else {
                const int64_t pos = start + written + rank;
                if (pos >= 0 && pos < capacity) {
                    ray_indices[pos] = static_cast<int32_t>(r);
                    t_starts[pos] = t0;
                    t_ends[pos] = t1;
                } else {
                    overflow = true;
                }
            }
        }
        written += n_take;
    }
    return written;
}

constexpr int kFillBatch = 8;  // rays per wave whose loads the fill issues together

template <int LOOKUP, bool SKIP, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void fill_uniform_kernel(
    const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const int32_t* __restrict__ grid_id, int64_t n_rays, const uint32_t* __restrict__ bits,
    const uint8_t* __restrict__ skip, GridK g, ClipK c, StepK p, const int32_t* __restrict__ packed_info,
    int64_t capacity, int32_t* __restrict__ ray_indices, float* __restrict__ t_starts, float* __restrict__ t_ends,
    int32_t* __restrict__ status, const uint64_t* __restrict__ masks, int n_masks, int split) {
    const int wave = uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    const int per = kRaysPerBlock / split;  // rays of this workgroup, as in the count pass
    const int64_t first = static_cast<int64_t>(blockIdx.x) * per;
    const int64_t mine = first + wave + static_cast<int64_t>(lane_id()) * WAVES;
    RaySpan spans{};
    if (wave + lane_id() * WAVES < per && mine < n_rays && packed_info[2 * mine + 1] > 0) {
        spans = ray_span<LOOKUP>(mine, rays_o, rays_d, grid_id, g, c, p);
    }
    bool overflow = false;
    // the box lookup's count pass leaves the plain traversal's masks also
    // when it marched by segments
    constexpr bool kFillSkip = SKIP && !kSegments<LOOKUP, SKIP>;
    if (masks != nullptr) {
        // kFillBatch rays at a time: their ranges and masks are all loaded
        // before any of their samples is stored.  A wave waits on its loads
        // only after its earlier stores have completed too (one counter
        // covers both), so loading ray by ray would put a store round trip
        // between consecutive rays.
        for (int i0 = wave; i0 < per; i0 += WAVES * kFillBatch) {
            int my_start = 0, my_limit = 0;  // lane b: ray i0 + b WAVES
            {
                const int ib = i0 + lane_id() * WAVES;
                const int64_t rb = first + ib;
                if (lane_id() < kFillBatch && ib < per && rb < n_rays) {
                    my_start = packed_info[2 * rb];
                    my_limit = packed_info[2 * rb + 1];
                }
            }
            uint64_t mk[kFillBatch];
#pragma unroll
            for (int b = 0; b < kFillBatch; ++b) {
                const int i = i0 + b * WAVES;
                const int64_t r = first + i;
                mk[b] = i < per && r < n_rays && lane_id() < n_masks ? masks[r * n_masks + lane_id()] : 0ull;
            }
            // every loaded value is read here, before the batch's first
            // store, so the wait for the loads is not a wait for stores
            int lim[kFillBatch], beg[kFillBatch];
            uint64_t any = 0ull;
#pragma unroll
            for (int b = 0; b < kFillBatch; ++b) {
                lim[b] = read_lane(my_limit, b);
                beg[b] = read_lane(my_start, b);
                any |= ballot(mk[b] != 0ull) | static_cast<uint64_t>(lim[b]);
            }
            if (any == 0ull) continue;  // no ray of the batch has samples
#pragma unroll
            for (int b = 0; b < kFillBatch; ++b) {
                const int i = i0 + b * WAVES;
                const int64_t r = first + i;
                if (i >= per || r >= n_rays) break;
                const int limit = lim[b];
                if (limit == 0) continue;
                const int64_t start = beg[b];
                const RaySpan span = read_span(spans, i / WAVES);
                int written;
                if (start >= 0 && start + limit <= capacity) {
                    written = fill_chunks<false>(r, span.t_near, p.dt, start, limit, capacity, ray_indices,
                                                 t_starts, t_ends, overflow, mk[b]);
                } else {
                    written = fill_chunks<true>(r, span.t_near, p.dt, start, limit, capacity, ray_indices,
                                                t_starts, t_ends, overflow, mk[b]);
                }
                if (written < limit) {  // samples past the stored chunks: traverse from there
                    march_ray_uniform<LOOKUP, true, kFillSkip>(r, span, rays_o, rays_d, bits, skip, g, p, start,
                                                               limit, capacity, ray_indices, t_starts, t_ends,
                                                               overflow, nullptr, 0, n_masks, written);
                }
            }
        }
        if (overflow && status != nullptr) *status = NACC_ECAPACITY;
        return;
    }
    for (int i = wave; i < per; i += WAVES) {
        const int64_t r = first + i;
        if (r >= n_rays) break;
        const int64_t start = packed_info[2 * r];
        const int limit = uniform<int>(packed_info[2 * r + 1]);
        if (limit == 0) continue;
        const RaySpan span = read_span(spans, i / WAVES);
        if constexpr (kSegments<LOOKUP, SKIP>) {
            // no stored masks: the segment count pass finds the samples with
            // fewer lookups; its ballots are written here directly
            march_ray_uniform<LOOKUP, true, false>(r, span, rays_o, rays_d, bits, skip, g, p, start, limit,
                                                   capacity, ray_indices, t_starts, t_ends, overflow);
        } else {
            march_ray_uniform<LOOKUP, true, SKIP>(r, span, rays_o, rays_d, bits, skip, g, p, start, limit, capacity,
                                                  ray_indices, t_starts, t_ends, overflow);
        }
    }
    if (overflow && status != nullptr) *status = NACC_ECAPACITY;
}

// Cone steps: the lattice is a recurrence in t, t_{k+1} = t_k +
// min(max(t_k c, dt), dt_max), so a lane walks a stretch of one ray.
// Candidates are taken kConeBatch at a time: the recurrence first (a few
// dependent FP32 operations per candidate), then the batch's grid words are
// all loaded before any is tested, so each lane keeps several loads in
// flight.  The count pass stores the occupancy bits of each chunk of 64
// candidates chunk-major (masks[chunk * n_rays + r]), and the fill pass
// replays them, running only the recurrence.
constexpr int kConeBatch = 8;
static_assert(kWave % kConeBatch == 0, "a batch must not straddle two chunks");

// The next kConeBatch cone steps from t: interval ends tb[0..kConeBatch] and
// how many of the batch's candidates lie inside the ray (a candidate is in
// while t_k < t_far and the step still advances t).
__device__ __forceinline__ int cone_steps(float t, float t_far, const StepK& p, float tb[kConeBatch + 1]) {
    tb[0] = t;
    int n_valid = kConeBatch;
#pragma unroll
    for (int u = 0; u < kConeBatch; ++u) {
        // min(max(t c, dt), dt_max) as one median (dt <= dt_max)
        const float step = __builtin_amdgcn_fmed3f(tb[u] * p.cone, p.dt, p.dt_max);
        tb[u + 1] = tb[u] + step;
        if (n_valid == kConeBatch && !(tb[u] < t_far && tb[u + 1] > tb[u])) n_valid = u;
    }
    return n_valid;
}

// Occupancy bits of a batch's candidates (bit u for candidate u < n_valid).
// All the batch's words (and one skip byte) are loaded before any is
// tested; every index is in range whatever the candidate.  Candidates
// inside a stretch cleared by the skip field are not looked up, and the
// batch's last candidate extends that stretch for the next batches.
template <int LOOKUP, bool SKIP>
__device__ __forceinline__ uint32_t cone_hits(const uint32_t* __restrict__ bits, const uint8_t* __restrict__ skip,
                                              const GridK& g, const SkipRay& sk, float& skip_end, uint32_t word0,
                                              const float o[3], const float d[3], const float tb[kConeBatch + 1],
                                              int n_valid) {
    float tm[kConeBatch];
    uint32_t todo = (1u << n_valid) - 1u;
#pragma unroll
    for (int u = 0; u < kConeBatch; ++u) {
        tm[u] = (tb[u] + tb[u + 1]) * 0.5f;
        if (SKIP && tm[u] < skip_end) todo &= ~(1u << u);
    }
    uint32_t hits = 0u;
    if (todo != 0u) {
        Probe q[kConeBatch];
        uint32_t w[kConeBatch];
#pragma unroll
        for (int u = 0; u < kConeBatch; ++u) {
            q[u] = probe<LOOKUP>(g, word0, o[0] + d[0] * tm[u], o[1] + d[1] * tm[u], o[2] + d[2] * tm[u]);
        }
#pragma unroll
        for (int u = 0; u < kConeBatch; ++u) w[u] = grid_word(grid_rsrc(bits, g), q[u].word);
        const int dist = SKIP ? static_cast<int>(skip[q[kConeBatch - 1].coarse]) : 0;
#pragma unroll
        for (int u = 0; u < kConeBatch; ++u) {
            if (((todo >> u) & 1u) != 0u && ((w[u] >> q[u].bit) & 1u) != 0u) hits |= 1u << u;
        }
        if (SKIP && n_valid == kConeBatch) {
            skip_end = fmaxf(skip_end, skip_end_at<LOOKUP>(g, sk, q[kConeBatch - 1], dist, tm[kConeBatch - 1]));
        }
    }
    return hits;
}

// One ray, cone steps, one lane, traversing the grid: the fill pass when no
// count-pass workspace is given (the same samples as the chunk-parallel
// passes, for checking them and for callers that keep no workspace).
template <int LOOKUP, bool SKIP>
__device__ __forceinline__ void fill_ray_cone(
    int64_t r, const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const int32_t* __restrict__ grid_id, const uint32_t* __restrict__ bits,
    const uint8_t* __restrict__ skip, const GridK& g,
    const ClipK& c, const StepK& p, int64_t start, int limit, int64_t capacity,
    float* __restrict__ t_starts, float* __restrict__ t_ends, bool& overflow) {
    float o[3], d[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o[i] = rays_o[3 * r + i];
        d[i] = rays_d[3 * r + i];
    }
    uint32_t word0;
    if (!grid_of_ray<LOOKUP>(grid_id, r, g, word0)) return;
    float t_near, t_far;
    if (!clip_ray(o, d, c, p.near_plane, p.far_plane, t_near, t_far)) return;
    SkipRay sk{};
    if (SKIP) sk = skip_ray(g, o, d, t_far);
    float skip_end = -INFINITY;  // candidates with midpoint below it are empty
    int count = 0;
    float t = t_near;
    for (int k0 = 0; k0 < kMaxCandidates && count < limit; k0 += kConeBatch) {
        float tb[kConeBatch + 1];
        const int n_valid = cone_steps(t, t_far, p, tb);
        const uint32_t hits =
            cone_hits<LOOKUP, SKIP>(bits, skip, g, sk, skip_end, word0, o, d, tb, n_valid) & ((1u << n_valid) - 1u);
#pragma unroll
        for (int u = 0; u < kConeBatch; ++u) {
            if (((hits >> u) & 1u) == 0u || count >= limit) continue;
            const int64_t pos = start + count;
            if (pos >= 0 && pos < capacity) {
                t_starts[pos] = tb[u];
                t_ends[pos] = tb[u + 1];
            } else {
                overflow = true;
            }
            ++count;
        }
        if (n_valid < kConeBatch) break;
        t = tb[kConeBatch];
    }
}

struct ConeHalo {
    float v;     // max_i s_i |d_i|: level-0 cells per unit t on the fastest axis
    float smax;  // max_i s_i
    float omax, dmax, dnorm;
    float onorm;  // |o|, rounded up
};

__device__ __forceinline__ ConeHalo cone_halo_ray(const GridK& g, const float o[3], const float d[3]) {
    ConeHalo k;
    k.v = fmaxf(fmaxf(g.s[0] * fabsf(d[0]), g.s[1] * fabsf(d[1])), g.s[2] * fabsf(d[2]));
    k.smax = fmaxf(fmaxf(g.s[0], g.s[1]), g.s[2]);
    k.omax = fmaxf(fmaxf(fabsf(o[0]), fabsf(o[1])), fabsf(o[2]));
    k.dmax = fmaxf(fmaxf(fabsf(d[0]), fabsf(d[1])), fabsf(d[2]));
    k.dnorm = sqrtf((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]) * (1.0f + 0x1p-18f);
    k.onorm = sqrtf((o[0] * o[0] + o[1] * o[1]) + o[2] * o[2]) * (1.0f + 0x1p-18f);
    return k;
}

// Whether a segment of candidates whose midpoints lie in [ta, tb] may hold
// samples (see above): false only when the centre's halo bit is clear and
// the bound holds.  Branch-free, so the segments' halo words are all in
// flight together.
template <int LOOKUP>
__device__ __forceinline__ bool cone_segment_live(const GridK& g, __amdgpu_buffer_rsrc_t hrs, uint32_t grid,
                                                  const float o[3], const float d[3], const ConeHalo& k, float ta,
                                                  float tb) {
    const float tc = (ta + tb) * 0.5f;
    const float h = (tb - ta) * 0.5f + fabsf(tb) * 0x1p-20f;  // half-extent, with the rounding of the t values
    float x0 = o[0] + d[0] * tc, x1 = o[1] + d[1] * tc, x2 = o[2] + d[2] * tc;
    // the rounding of positions (a few ulps of the largest coordinate
    // reached, for both points) and of cell coordinates, generously
    const float slack_x = (k.omax + k.dmax * fabsf(tb) + 1.0f) * 0x1p-19f;
    const float cell_slack = static_cast<float>(g.res) * 0x1p-17f;
    float dev;  // bound of |u_i(midpoint) - u_i(centre)| in cells
    bool open = false;  // the bound cannot be established
    uint32_t hgrid = grid;
    if (LOOKUP == NACC_LOOKUP_CASCADE) {
        const float m = fmaxf(fmaxf(fabsf(x0), fabsf(x1)), fabsf(x2));
        const float dm = k.dmax * h + slack_x;
        const int l_lo = cascade_level(fmaxf(m - dm, 0.0f), g);
        const int l_hi = cascade_level(m + dm, g);
        open = l_lo != l_hi;  // a midpoint may lie on another level
        hgrid = static_cast<uint32_t>(l_hi);
        x0 = ldexpf(x0, -l_hi);
        x1 = ldexpf(x1, -l_hi);
        x2 = ldexpf(x2, -l_hi);
        dev = ldexpf(k.v * h + k.smax * slack_x, -l_hi) + cell_slack;
    } else if (LOOKUP == NACC_LOOKUP_CONTRACT) {
        // The hardware square root and reciprocal (within a few ulps) serve
        // here: every quantity below is a bound that carries a margin far
        // above their error (2^-18 relative on |x|, L and the motion factor;
        // 2^-16 contracted units on the centre's position).
        const float n = __builtin_amdgcn_sqrtf((x0 * x0 + x1 * x1) + x2 * x2);
        // r_min bounds |x| from below over the segment; beyond radius r > 1
        // the contraction shrinks distances by at most (2 - 1/r)/r, and a
        // motion along the ray by at most (1 + 2|o|)/r^2: its radial part
        // shrinks by 1/r^2, its tangential part, at most |o||d|/r long, by
        // (2 - 1/r)/r < 2/r
        const float r_min = n * (1.0f - 0x1p-18f) - k.dnorm * h - 2.0f * slack_x;
        float lip = 1.0f, along = 1.0f;
        if (r_min > 1.0f) {
            const float ir = __builtin_amdgcn_rcpf(r_min);
            lip = ((2.0f - ir) * ir) * (1.0f + 0x1p-18f);
            along = fminf(lip, ((1.0f + 2.0f * k.onorm) * (ir * ir)) * (1.0f + 0x1p-18f));
        }
        if (n > 1.0f) {
            const float in = __builtin_amdgcn_rcpf(n);
            const float f = (2.0f - in) * in;
            x0 = x0 * f;
            x1 = x1 * f;
            x2 = x2 * f;
        }
        dev = k.smax * (along * k.dnorm * h + lip * 3.5f * slack_x + 3.5f * 0x1p-16f) + cell_slack;
    } else {
        dev = k.v * h + k.smax * slack_x + cell_slack;
    }
    open = open || !(dev <= static_cast<float>(kHaloReach) * (1.0f - 0x1p-10f));
    const bool hb = halo_bit(hrs, g, hgrid * g.halo_words, x0, x1, x2);  // loaded in every case
    return open | hb;
}

// The cone-step lattice from the near plane, shared by every ray that
// starts there (rays from inside the clip box, or with no box at all, start
// at the near plane): t at every 8th candidate, computed once on the host
// in FP32 with the device's operations (each correctly rounded; the
// median of three is the clamp), and passed by value.  The recurrence only
// depends on t, so a chunk of any ray whose first t equals the table's
// entry continues along the table; the starts and count passes then read
// chunk and segment starts instead of walking them.  Left empty (n = 0) if
// the steps stall within the table (t + step == t), which the walks handle.
constexpr int kMaxMaskChunks = 64;  // one per lane of a wave
constexpr int kTableStride = kWave / kConeBatch;  // table entries per chunk
struct ConeTable {
    float t[kMaxMaskChunks * kTableStride + 1];
    int n;  // entries: n_masks 8 + 1, or 0
};

ConeTable cone_table(const StepK& p, int n_masks) {
    ConeTable tab;
    tab.n = 0;
    float t = p.near_plane;
    if (n_masks <= 0 || !std::isfinite(t)) return tab;
    const int n = n_masks * kTableStride + 1;
    for (int i = 0; i < n; ++i) {
        tab.t[i] = t;
        for (int u = 0; u < kConeBatch && i + 1 < n; ++u) {
            const float step = std::fmin(std::fmax(t * p.cone, p.dt), p.dt_max);
            const float t1 = t + step;
            if (!(t1 > t)) return tab;  // stalls: no table
            t = t1;
        }
    }
    tab.n = n;
    return tab;
}

// Chunk-parallel cone marching.  The recurrence itself is cheap (four FP32
// operations per candidate) but serial; the grid lookups are not.  A
// pre-pass walks each ray's recurrence once, one lane per ray, and records
// t at the start of every chunk of 64 candidates; the count and fill passes
// then take one lane per (ray, chunk), so a launch has ~12 times as many
// independent lanes as rays to hide the lookup latency.  Tasks are ordered
// chunk-major (task = chunk * n_rays + ray): a wave's loads and stores of
// the per-chunk arrays are contiguous.  A ray longer than the stored chunks
// is finished by the task of its last stored chunk.
// CULL (contraction lookup with halo bits): a chunk whose candidates all
// provably map into halo-clear cells (one test of the chunk's whole extent,
// see cone_segment_live) is marked by a NaN start, which the segment count
// and fill passes take for a chunk without samples.  Far from the scene the
// contraction maps a whole chunk of candidates into a fraction of a cell.
// The last stored chunk is never marked: the passes continue the ray from it.
template <int LOOKUP, bool CULL>
__global__ __launch_bounds__(kRaysPerBlock) void cone_starts_kernel(
    const float* __restrict__ rays_o, const float* __restrict__ rays_d, const int32_t* __restrict__ grid_id,
    int64_t n_rays, GridK g, ClipK c, StepK p, int n_masks, float* __restrict__ chunk_t,
    float* __restrict__ t_far_out, int32_t* __restrict__ extra, const uint32_t* __restrict__ halo,
    uint64_t* __restrict__ live_chunks, int64_t* __restrict__ task_sums, ConeTable tab) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kRaysPerBlock + threadIdx.x;
    uint64_t listed = 0ull;  // CULL: chunks with candidates that may hold samples
    if (r < n_rays) {
        float o[3], d[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            o[i] = rays_o[3 * r + i];
            d[i] = rays_d[3 * r + i];
        }
        uint32_t word0;
        float t_near = 0.0f, t_far = 0.0f;
        bool live = grid_of_ray<LOOKUP>(grid_id, r, g, word0);
        live = clip_ray(o, d, c, p.near_plane, p.far_plane, t_near, t_far) && live;
        t_far_out[r] = live ? t_far : -INFINITY;
        extra[r] = 0;
        const ConeHalo k = cone_halo_ray(g, o, d);  // (unused unless CULL)
        const __amdgpu_buffer_rsrc_t hrs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint32_t*>(halo), 0, static_cast<int>(g.halo_bytes), kBufferWord3);
        float t = t_near;
        const bool tabled = tab.n > 0 && t_near == tab.t[0];  // starts at the near plane
        const bool all_tabled = __builtin_amdgcn_ballot_w64(live && !tabled) == 0ull;
        if (all_tabled) {
            // every live ray of the wave follows the table: eight chunks at
            // a time, so that their culling tests' loads are in flight
            // together
            for (int j0 = 0; j0 < n_masks; j0 += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int j = j0 + u;
                    if (j < n_masks) {
                        const float ta = tab.t[kTableStride * j];
                        const bool has = live && ta < t_far;
                        float start = has ? ta : INFINITY;
                        if (CULL && has && j < n_masks - 1 &&
                            !cone_segment_live<LOOKUP>(g, hrs, word0 / g.words, o, d, k, ta,
                                                       tab.t[kTableStride * (j + 1)])) {
                            start = __builtin_nanf("");
                        }
                        if (CULL && start < INFINITY) listed |= 1ull << j;
                        chunk_t[static_cast<int64_t>(j) * n_rays + r] = start;
                    }
                }
            }
        }
        for (int j = 0; j < (all_tabled ? 0 : n_masks); ++j) {
            live = live && t < t_far;  // the chunk's first candidate exists
            const float ta = t;
            const bool has = live;
            if (__builtin_amdgcn_ballot_w64(live && !tabled) == 0ull) {
                // the wave's live rays all follow the table (or have all
                // ended): the next chunk's start, past the ray's end too
                if (tabled) t = tab.t[kTableStride * (j + 1)];
            } else if (p.no_stall) {
                // every step advances, so the candidates inside the ray are a
                // prefix: the steps are taken without tests (past the ray's
                // end t runs on; the next chunk's test sees that)
#pragma unroll 8
                for (int u = 0; u < kWave; ++u) t = t + __builtin_amdgcn_fmed3f(t * p.cone, p.dt, p.dt_max);
            } else {
                // 64 steps without branches: a ray that ends keeps its last t
#pragma unroll 8
                for (int u = 0; u < kWave; ++u) {
                    const float t1 = t + __builtin_amdgcn_fmed3f(t * p.cone, p.dt, p.dt_max);
                    live = live && t < t_far && t1 > t;
                    t = live ? t1 : t;
                }
            }
            float start = has ? ta : INFINITY;
            if (CULL && has && j < n_masks - 1 &&
                !cone_segment_live<LOOKUP>(g, hrs, word0 / g.words, o, d, k, ta, t)) {
                start = __builtin_nanf("");
            }
            if (CULL && start < INFINITY) listed |= 1ull << j;
            chunk_t[static_cast<int64_t>(j) * n_rays + r] = start;
        }
        if (CULL) live_chunks[r] = listed;
    }
    if (CULL) {
        // the workgroup's (one wave of 64 rays) listed rays per chunk,
        // chunk-major ([chunk][workgroup]), for the scan that places the
        // tasks in the list chunk by chunk, rays in order within a chunk
        for (int j = 0; j < n_masks; ++j) {
            const uint64_t b = __builtin_amdgcn_ballot_w64(((listed >> j) & 1ull) != 0ull);
            if (threadIdx.x == 0) task_sums[static_cast<int64_t>(j) * gridDim.x + blockIdx.x] = __popcll(b);
        }
    }
}

// The task list of the segment passes under CULL: the listed chunks, chunk
// by chunk, rays in order within a chunk (task = j n_rays + r), so that
// neighbouring tasks read and write neighbouring entries of the per-chunk
// arrays.  offsets: the exclusive scan of the per-(chunk, workgroup) counts.
__global__ __launch_bounds__(kRaysPerBlock) void task_list_kernel(const int64_t* __restrict__ offsets,
                                                                  int64_t n_rays, int n_masks,
                                                                  const uint64_t* __restrict__ live_chunks,
                                                                  int32_t* __restrict__ task_list) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kRaysPerBlock + threadIdx.x;
    const uint64_t m = r < n_rays ? live_chunks[r] : 0ull;
    for (int j = 0; j < n_masks; ++j) {
        const bool on = ((m >> j) & 1ull) != 0ull;
        const uint64_t b = __builtin_amdgcn_ballot_w64(on);
        if (on) {
            const int64_t pos = offsets[static_cast<int64_t>(j) * gridDim.x + blockIdx.x] + bits_below(b);
            task_list[pos] = static_cast<int32_t>(static_cast<int64_t>(j) * n_rays + r);
        }
    }
}

// Occupancy bits of the 64 candidates of one chunk from its first t; `ended`
// tells whether the ray's candidates stop inside the chunk.
template <int LOOKUP, bool SKIP>
__device__ __forceinline__ uint64_t cone_chunk_bits(const uint32_t* __restrict__ bits,
                                                    const uint8_t* __restrict__ skip, const GridK& g,
                                                    const SkipRay& sk, float& skip_end, uint32_t word0,
                                                    const float o[3], const float d[3], float& t, float t_far,
                                                    const StepK& p, bool& ended) {
    uint64_t m = 0ull;
    ended = false;
#pragma unroll 1
    for (int b = 0; b < kWave / kConeBatch; ++b) {
        float tb[kConeBatch + 1];
        const int n_valid = cone_steps(t, t_far, p, tb);
        const uint32_t hits =
            cone_hits<LOOKUP, SKIP>(bits, skip, g, sk, skip_end, word0, o, d, tb, n_valid) & ((1u << n_valid) - 1u);
        m |= static_cast<uint64_t>(hits) << (b * kConeBatch);
        if (n_valid < kConeBatch) {
            ended = true;
            break;
        }
        t = tb[kConeBatch];
    }
    return m;
}

constexpr int kTaskThreads = 256;

template <int LOOKUP, bool SKIP>
__global__ __launch_bounds__(kTaskThreads) void count_cone_chunks_kernel(
    const float* __restrict__ rays_o, const float* __restrict__ rays_d, const int32_t* __restrict__ grid_id,
    int64_t n_rays, const uint32_t* __restrict__ bits, const uint8_t* __restrict__ skip, GridK g, StepK p,
    int n_masks, const float* __restrict__ chunk_t, const float* __restrict__ t_far_in,
    uint64_t* __restrict__ masks, int32_t* __restrict__ extra) {
    const int64_t task = static_cast<int64_t>(blockIdx.x) * kTaskThreads + threadIdx.x;
    if (task >= static_cast<int64_t>(n_masks) * n_rays) return;
    const int j = static_cast<int>(task / n_rays);
    const int64_t r = task - static_cast<int64_t>(j) * n_rays;
    float t = chunk_t[task];
    if (!(t < INFINITY)) {
        masks[task] = 0ull;
        return;
    }
    const float t_far = t_far_in[r];
    float o[3], d[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o[i] = rays_o[3 * r + i];
        d[i] = rays_d[3 * r + i];
    }
    uint32_t word0;
    grid_of_ray<LOOKUP>(grid_id, r, g, word0);  // valid: the ray has candidates
    SkipRay sk{};
    if (SKIP) sk = skip_ray(g, o, d, t_far);
    float skip_end = -INFINITY;
    bool ended;
    masks[task] = cone_chunk_bits<LOOKUP, SKIP>(bits, skip, g, sk, skip_end, word0, o, d, t, t_far, p, ended);
    if (j == n_masks - 1 && !ended) {
        // past the stored chunks: count the rest of the ray here
        int count = 0;
        for (int k0 = n_masks * kWave; k0 < kMaxCandidates; k0 += kWave) {
            count += __popcll(
                cone_chunk_bits<LOOKUP, SKIP>(bits, skip, g, sk, skip_end, word0, o, d, t, t_far, p, ended));
            if (ended) break;
        }
        extra[r] = count;
    }
}

// Per-ray counts from the chunk masks (capped at max_per_ray) and the
// workgroup sums of the scan.  For the segment fill (nullable): the samples
// of each ray before each chunk, and per ray the bits of the chunks holding
// samples (sample_chunks may be live_chunks itself: each ray's word is read
// before it is written).
__global__ __launch_bounds__(kRaysPerBlock) void cone_counts_kernel(int64_t n_rays, int n_masks, int max_per_ray,
                                                                    const uint64_t* __restrict__ masks,
                                                                    const int32_t* __restrict__ extra,
                                                                    int32_t* __restrict__ packed_info,
                                                                    int64_t* __restrict__ block_sums,
                                                                    int32_t* __restrict__ chunk_base,
                                                                    const uint64_t* live_chunks,
                                                                    uint64_t* sample_chunks) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kRaysPerBlock + threadIdx.x;
    int n = 0;
    if (r < n_rays) {
        // with a task list, the chunks left out of it hold no samples (their
        // masks were not written)
        const uint64_t listed = live_chunks != nullptr ? live_chunks[r] : ~0ull;
        uint64_t holding = 0ull;
        int64_t total = 0;
        // eight chunks' masks loaded together, then taken in order
        constexpr int kGroup = 8;
        for (int j0 = 0; j0 < n_masks; j0 += kGroup) {
            uint64_t mg[kGroup];
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                const int j = j0 + u;
                mg[u] = j < n_masks && ((listed >> j) & 1ull) != 0ull ? masks[static_cast<int64_t>(j) * n_rays + r]
                                                                       : 0ull;
            }
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                const int j = j0 + u;
                const uint64_t m = mg[u];
                // samples of the ray before chunk j, for the segment fill,
                // which reads it for the chunks holding samples and the last
                if (chunk_base != nullptr && j < n_masks && (m != 0ull || j == n_masks - 1)) {
                    chunk_base[static_cast<int64_t>(j) * n_rays + r] =
                        static_cast<int32_t>(min(total, static_cast<int64_t>(kMaxCandidates)));
                }
                total += __popcll(m);
                if (m != 0ull) holding |= 1ull << j;
            }
        }
        if (sample_chunks != nullptr) sample_chunks[r] = holding;
        total += extra[r];
        if (max_per_ray > 0) total = min(total, static_cast<int64_t>(max_per_ray));
        n = static_cast<int>(min(total, static_cast<int64_t>(kMaxCandidates)));
        packed_info[2 * r + 1] = n;
    }
    const int sum = wave_sum(n);  // <= 64 * 2^24 fits int32
    if (threadIdx.x == 0) block_sums[blockIdx.x] = sum;
}

template <int LOOKUP, bool SKIP>
__global__ __launch_bounds__(kTaskThreads) void fill_cone_chunks_kernel(
    const float* __restrict__ rays_o, const float* __restrict__ rays_d, const int32_t* __restrict__ grid_id,
    int64_t n_rays, const uint32_t* __restrict__ bits, const uint8_t* __restrict__ skip, GridK g, StepK p,
    int n_masks, const float* __restrict__ chunk_t, const float* __restrict__ t_far_in,
    const uint64_t* __restrict__ masks, const int32_t* __restrict__ packed_info, int64_t capacity,
    float* __restrict__ t_starts, float* __restrict__ t_ends, int32_t* __restrict__ status) {
    const int64_t task = static_cast<int64_t>(blockIdx.x) * kTaskThreads + threadIdx.x;
    if (task >= static_cast<int64_t>(n_masks) * n_rays) return;
    const int j = static_cast<int>(task / n_rays);
    const int64_t r = task - static_cast<int64_t>(j) * n_rays;
    float t = chunk_t[task];
    if (!(t < INFINITY)) return;
    const int limit = packed_info[2 * r + 1];
    int idx = 0;  // samples of the ray before this chunk
    for (int q = 0; q < j; ++q) idx += __popcll(masks[static_cast<int64_t>(q) * n_rays + r]);
    if (idx >= limit) return;
    const int64_t start = packed_info[2 * r];
    const float t_far = t_far_in[r];
    bool overflow = false;
    auto emit = [&](float a, float b) {
        const int64_t pos = start + idx;
        if (pos >= 0 && pos < capacity) {
            t_starts[pos] = a;
            t_ends[pos] = b;
        } else {
            overflow = true;
        }
        ++idx;
    };
    const uint64_t m = masks[task];
    bool ended = false;
#pragma unroll 1
    for (int b = 0; b < kWave / kConeBatch && idx < limit; ++b) {
        float tb[kConeBatch + 1];
        const int n_valid = cone_steps(t, t_far, p, tb);
        const uint32_t hits = static_cast<uint32_t>(m >> (b * kConeBatch)) & ((1u << n_valid) - 1u);
#pragma unroll
        for (int u = 0; u < kConeBatch; ++u) {
            if (((hits >> u) & 1u) != 0u && idx < limit) emit(tb[u], tb[u + 1]);
        }
        if (n_valid < kConeBatch) {
            ended = true;
            break;
        }
        t = tb[kConeBatch];
    }
    if (j == n_masks - 1 && !ended && idx < limit) {
        // past the stored chunks: look the rest of the ray up again
        float o[3], d[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            o[i] = rays_o[3 * r + i];
            d[i] = rays_d[3 * r + i];
        }
        uint32_t word0;
        grid_of_ray<LOOKUP>(grid_id, r, g, word0);
        SkipRay sk{};
        if (SKIP) sk = skip_ray(g, o, d, t_far);
        float skip_end = -INFINITY;
        for (int k0 = n_masks * kWave; k0 < kMaxCandidates && idx < limit; k0 += kConeBatch) {
            float tb[kConeBatch + 1];
            const int n_valid = cone_steps(t, t_far, p, tb);
            const uint32_t hits = cone_hits<LOOKUP, SKIP>(bits, skip, g, sk, skip_end, word0, o, d, tb, n_valid) &
                                  ((1u << n_valid) - 1u);
#pragma unroll
            for (int u = 0; u < kConeBatch; ++u) {
                if (((hits >> u) & 1u) != 0u && idx < limit) emit(tb[u], tb[u + 1]);
            }
            if (n_valid < kConeBatch) break;
            t = tb[kConeBatch];
        }
    }
    if (overflow && status != nullptr) *status = NACC_ECAPACITY;
}

// ---------------------------------------------------------------------------
// Cone steps with the halo bits of the skip buffer.  A chunk's 64 candidates
// form 8 segments of kConeBatch; the count pass walks the chunk's recurrence
// once (one lane per chunk) and tests one halo bit per segment at its
// centre.  The segments that may hold samples are queued per wave in LDS
// and then looked up 64 at a time, one segment per lane, so that the lanes
// stay busy although only a few segments of a chunk are live.  Each looked-up
// segment's 8 occupancy bits are ORed into its chunk's mask (byte s of the
// mask, as in the plain passes), and the t at the start of every segment
// holding samples is stored, so the fill pass writes them without walking
// the recurrence again.
//
// A clear halo bit proves a segment empty when all its midpoints provably
// map within kHaloReach cells of the centre's cell in the grid the centre is
// looked up in: the midpoints lie within h of the centre in t (h half the
// segment's extent plus rounding), so within |d_i| h plus the rounding of
// positions on axis i; cascades also need every midpoint on the centre's
// level (its max |x_i| bracketed on both sides), and the contraction
// shrinks distances by at most L(r) = (2 - 1/r)/r beyond radius r >= 1
// (at most 1 everywhere).  Where the bound fails the segment is looked up.
// ---------------------------------------------------------------------------
constexpr int kSegsPerChunk = kWave / kConeBatch;
constexpr int kTaskWaves = kTaskThreads / kWave;
constexpr int kSegQueue = kWave * kSegsPerChunk;  // every segment of a wave's chunks

// 32-bit value of lane `src` (per lane) through the LDS crossbar; every lane
// must be active.
__device__ __forceinline__ float lane_value(float v, int src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ int lane_value(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }

template <int LOOKUP>
__global__ __launch_bounds__(kTaskThreads) void count_cone_segments_kernel(
    const float* __restrict__ rays_o, const float* __restrict__ rays_d, const int32_t* __restrict__ grid_id,
    int64_t n_rays, const uint32_t* __restrict__ bits, const uint32_t* __restrict__ halo, GridK g, StepK p,
    int n_masks, const float* __restrict__ chunk_t, const float* __restrict__ t_far_in,
    uint64_t* __restrict__ masks, int32_t* __restrict__ extra, float* __restrict__ seg_t,
    const int32_t* __restrict__ task_list, const int64_t* __restrict__ task_total, ConeTable tab) {
    __shared__ float q_t[kTaskWaves][kSegQueue];
    __shared__ uint16_t q_id[kTaskWaves][kSegQueue];
    __shared__ uint64_t q_mask[kTaskWaves][kWave];
    const int lane = lane_id();
    const int wave = uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    // task = chunk j n_rays + ray r; lane i of the launch takes task i, or,
    // with a task list, its i-th entry
    const int64_t first_idx = static_cast<int64_t>(blockIdx.x) * kTaskThreads + wave * kWave;
    const int64_t idx = first_idx + lane;
    bool in_range;
    int64_t task = idx;
    if (task_list != nullptr) {
        in_range = idx < *task_total;
        if (in_range) task = task_list[idx];
    } else {
        in_range = idx < static_cast<int64_t>(n_masks) * n_rays;
    }
    int j = 0;
    int64_t r = 0;
    float t = INFINITY;
    if (in_range) {
        j = static_cast<int>(task / n_rays);
        r = task - static_cast<int64_t>(j) * n_rays;
        t = chunk_t[task];
    }
    const bool active = t < INFINITY;  // (NaN: a chunk the starts pass proved empty)
    if (ballot(active) == 0ull) {     // the whole wave: nothing to look up
        if (in_range) masks[task] = 0ull;
        return;
    }
    float o[3] = {0.0f, 0.0f, 0.0f}, d[3] = {0.0f, 0.0f, 0.0f};
    float t_far = -INFINITY;
    uint32_t word0 = 0;
    if (active) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            o[i] = rays_o[3 * r + i];
            d[i] = rays_d[3 * r + i];
        }
        t_far = t_far_in[r];
        grid_of_ray<LOOKUP>(grid_id, r, g, word0);  // valid: the ray has candidates
    }
    // walk the chunk's recurrence once; test each segment's halo bit
    const ConeHalo k = cone_halo_ray(g, o, d);
    const __amdgpu_buffer_rsrc_t hrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(halo), 0, static_cast<int>(g.halo_bytes), kBufferWord3);
    const uint32_t grid = word0 / g.words;
    float st[kSegsPerChunk];
    uint32_t live = 0u;
    bool alive = active;
    // a chunk that starts on the near-plane lattice (not the last stored
    // one, whose end the continuation needs) reads its segment starts; the
    // wave's tasks are chunk-major, so they nearly always share one chunk
    // index, whose entries are then read with scalar loads
    const int j0 = uniform<int>(j);
    const bool tabled = tab.n > 0 && active && j == j0 && j0 < n_masks - 1 && t == tab.t[kTableStride * j0];
    if (ballot(active && !tabled) == 0ull) {
#pragma unroll
        for (int s = 0; s < kSegsPerChunk; ++s) {
            const float ta = tabled ? tab.t[kTableStride * j0 + s] : t;
            const float tb = tabled ? tab.t[kTableStride * j0 + s + 1] : t;
            st[s] = ta;
            const bool any = active && ta < t_far;
            live |= static_cast<uint32_t>(cone_segment_live<LOOKUP>(g, hrs, grid, o, d, k, ta, tb) & any) << s;
        }
    } else if (p.no_stall) {
        // every step advances: a segment holds candidates inside the ray iff
        // its first t lies before t_far; its extent is taken past the ray's
        // end (a larger interval only weakens the test)
        float t_last = t;  // t of the chunk's last candidate
#pragma unroll
        for (int s = 0; s < kSegsPerChunk; ++s) {
            const float ta = t;
#pragma unroll
            for (int u = 0; u < kConeBatch; ++u) {
                t_last = t;
                t = t + __builtin_amdgcn_fmed3f(t * p.cone, p.dt, p.dt_max);
            }
            st[s] = ta;
            const bool any = active && ta < t_far;
            live |= static_cast<uint32_t>(cone_segment_live<LOOKUP>(g, hrs, grid, o, d, k, ta, t) & any) << s;
        }
        alive = active && t_last < t_far;
    } else {
#pragma unroll
        for (int s = 0; s < kSegsPerChunk; ++s) {
            const float ta = t;
            bool any = false;  // some candidate of the segment lies inside the ray
#pragma unroll
            for (int u = 0; u < kConeBatch; ++u) {
                const float t1 = t + __builtin_amdgcn_fmed3f(t * p.cone, p.dt, p.dt_max);
                alive = alive && t < t_far && t1 > t;
                any = any || alive;
                t = alive ? t1 : t;
            }
            st[s] = ta;
            live |= static_cast<uint32_t>(cone_segment_live<LOOKUP>(g, hrs, grid, o, d, k, ta, t) & any) << s;
        }
    }
    const bool ended = !alive;
    // queue the live segments of the wave's chunks in LDS, in lane order
    const int n_items = __popc(live);
    const int before = wave_inclusive_sum(n_items) - n_items;
    const int total = read_lane(before + n_items, kWave - 1);
    {
        int pos = before;
#pragma unroll
        for (int s = 0; s < kSegsPerChunk; ++s) {
            if (((live >> s) & 1u) != 0u) {
                q_t[wave][pos] = st[s];
                q_id[wave][pos] = static_cast<uint16_t>(lane | (s << kWaveLog2));
                ++pos;
            }
        }
    }
    q_mask[wave][lane] = 0ull;
    wave_lds_sync();
    // look the queued segments up, one per lane
    for (int base = 0; base < total; base += kWave) {
        const int i = base + lane;
        const bool has = i < total;
        const float t0 = has ? q_t[wave][i] : 0.0f;
        const int id = has ? static_cast<int>(q_id[wave][i]) : 0;
        const int src = id & (kWave - 1);
        const int s = id >> kWaveLog2;
        float so[3], sd[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            so[c] = lane_value(o[c], src);
            sd[c] = lane_value(d[c], src);
        }
        // every lane takes part in the crossbar reads (a lane left out would
        // not provide its value to the lanes reading it)
        const float src_far = lane_value(t_far, src);
        const float s_far = has ? src_far : -INFINITY;
        const uint32_t s_word0 = static_cast<uint32_t>(lane_value(static_cast<int>(word0), src));
        float tb[kConeBatch + 1];
        const int n_valid = cone_steps(t0, s_far, p, tb);
        SkipRay sk{};
        float skip_end = -INFINITY;
        const uint32_t hits =
            cone_hits<LOOKUP, false>(bits, nullptr, g, sk, skip_end, s_word0, so, sd, tb, n_valid) &
            ((1u << n_valid) - 1u);
        const int64_t s_task =
            task_list != nullptr ? static_cast<int64_t>(lane_value(static_cast<int>(task), src)) : first_idx + src;
        if (has && hits != 0u) {
            __hip_atomic_fetch_or(&q_mask[wave][src], static_cast<uint64_t>(hits) << (s * kConeBatch),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            seg_t[s_task * kSegsPerChunk + s] = t0;
        }
    }
    wave_lds_sync();
    if (in_range) masks[task] = q_mask[wave][lane];
    if (active && j == n_masks - 1 && !ended) {
        // past the stored chunks: count the rest of the ray here
        SkipRay sk{};
        float skip_end = -INFINITY;
        bool e2 = false;
        int count = 0;
        for (int k0 = n_masks * kWave; k0 < kMaxCandidates; k0 += kWave) {
            count += __popcll(cone_chunk_bits<LOOKUP, false>(bits, nullptr, g, sk, skip_end, word0, o, d, t, t_far,
                                                             p, e2));
            if (e2) break;
        }
        extra[r] = count;
    }
}

// Fill pass of the segment count, ray-major with staged stores.  A wave
// takes kFillRays consecutive rays and lists their (ray, chunk) tasks for the
// chunks that hold samples (cone_counts_kernel leaves their bits per ray),
// ray by ray, chunk by chunk, so the segments that hold samples, queued in
// that order, are in the order of their samples in the output.  The queue
// is written 64 segments at a time: one lane per segment runs its 8
// recurrence steps from the stored t at its start and puts its samples
// (t_start, t_end) into this wave's LDS slots in output order; then the
// wave stores the slots, 64 consecutive positions at a time, with the ray
// indices, so every store is coalesced (each segment's samples stored from
// its own lane scatter 4-byte writes over as many cache lines as lanes).
// A ray longer than the stored chunks is finished past them by its lane.
constexpr int kFillSlots = kWave * kConeBatch;  // the samples of 64 segments at most
// Rays per wave: their tasks still spread over all 64 lanes, and more,
// shorter waves hide the latency of each round's permutes, LDS round trips
// and stores better (contraction lookup: 111 -> 94 us at 262,144 rays; 8
// rays per wave lose again).
constexpr int kFillRays = 16;

// Position of the k-th set bit of v (k < popcount(v)).
__device__ __forceinline__ int nth_set_bit(uint64_t v, int k) {
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const int c = static_cast<int>(__popcll(v & ((1ull << w) - 1ull)));
        if (k >= c) {
            k -= c;
            v >>= w;
            pos += w;
        }
    }
    return pos;
}

template <int LOOKUP>
__global__ __launch_bounds__(kTaskThreads) void fill_cone_rays_kernel(
    const float* __restrict__ rays_o, const float* __restrict__ rays_d, const int32_t* __restrict__ grid_id,
    int64_t n_rays, const uint32_t* __restrict__ bits, GridK g, StepK p, int n_masks,
    const float* __restrict__ chunk_t, const float* __restrict__ t_far_in, const uint64_t* __restrict__ masks,
    const int32_t* __restrict__ chunk_base, const float* __restrict__ seg_t,
    const uint64_t* __restrict__ sample_chunks, const int32_t* __restrict__ packed_info, int64_t capacity,
    int32_t* __restrict__ ray_indices, float* __restrict__ t_starts, float* __restrict__ t_ends,
    int32_t* __restrict__ status) {
    __shared__ uint16_t q_id[kTaskWaves][kSegQueue];
    __shared__ float s_t0[kTaskWaves][kFillSlots];
    __shared__ float s_t1[kTaskWaves][kFillSlots];
    __shared__ uint8_t s_entry[kTaskWaves][kFillSlots];  // the queue entry (of this round) a slot belongs to
    __shared__ int64_t e_pos[kTaskWaves][kWave];         // output position of an entry's first sample
    __shared__ int32_t e_slot[kTaskWaves][kWave];        // its first slot
    __shared__ int32_t e_ray[kTaskWaves][kWave];
    const int lane = lane_id();
    const int wave = uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    // lane i: ray first + i
    const int64_t ray = (static_cast<int64_t>(blockIdx.x) * kTaskWaves + wave) * kFillRays + lane;
    int limit = 0;
    int64_t start = 0;
    uint64_t nz = 0ull;
    if (lane < kFillRays && ray < n_rays) {
        limit = packed_info[2 * ray + 1];
        if (limit > 0) {
            start = packed_info[2 * ray];
            nz = sample_chunks[ray];
        }
    }
    // a ray whose last stored chunk exists may go on past the stored chunks
    const float t_last = limit > 0 ? chunk_t[static_cast<int64_t>(n_masks - 1) * n_rays + ray] : INFINITY;
    const int n_tasks = static_cast<int>(__popcll(nz));
    const int t_before = wave_inclusive_sum(n_tasks) - n_tasks;
    const int t_total = read_lane(t_before + n_tasks, kWave - 1);
    bool overflow = false;
    const int start_lo = static_cast<int>(start), start_hi = static_cast<int>(start >> 32);
    const int nz_lo = static_cast<int>(nz), nz_hi = static_cast<int>(nz >> 32);
    for (int tb0 = 0; tb0 < t_total; tb0 += kWave) {
        // task i of the wave: the ray lane L whose tasks hold it, and its
        // (i - first task of L)-th chunk holding samples
        const int i = tb0 + lane;
        int L = 0;
#pragma unroll
        for (int step = kWave / 2; step >= 1; step >>= 1) {
            const int probe_lane = L + step;  // < 64
            if (lane_value(t_before, probe_lane) <= i) L = probe_lane;
        }
        const bool has_task = i < t_total;
        const uint64_t l_nz = (static_cast<uint64_t>(static_cast<uint32_t>(lane_value(nz_hi, L))) << 32) |
                              static_cast<uint32_t>(lane_value(nz_lo, L));
        const int l_first = lane_value(t_before, L);
        const int l_limit = lane_value(limit, L);
        const int64_t l_start = (static_cast<int64_t>(lane_value(start_hi, L)) << 32) |
                                static_cast<uint32_t>(lane_value(start_lo, L));
        const int64_t r = (static_cast<int64_t>(blockIdx.x) * kTaskWaves + wave) * kFillRays + L;
        uint64_t m = 0ull;
        int base = 0;
        int64_t task = 0;
        float t_far = -INFINITY;
        if (has_task) {
            const int j = nth_set_bit(l_nz, i - l_first);
            task = static_cast<int64_t>(j) * n_rays + r;
            m = masks[task];
            base = chunk_base[task];
            t_far = t_far_in[r];
        }
        // segments holding samples that fall before the ray's limit
        uint32_t todo = 0u;
#pragma unroll
        for (int s = 0; s < kSegsPerChunk; ++s) {
            const bool holds = ((m >> (s * kConeBatch)) & 0xffull) != 0ull;
            const int idx = base + static_cast<int>(__popcll(m & ((1ull << (s * kConeBatch)) - 1ull)));
            if (holds && idx < l_limit) todo |= 1u << s;
        }
        const int n_items = __popc(todo);
        const int before = wave_inclusive_sum(n_items) - n_items;
        const int total = read_lane(before + n_items, kWave - 1);
        {
            int pos = before;
#pragma unroll
            for (int s = 0; s < kSegsPerChunk; ++s) {
                if (((todo >> s) & 1u) != 0u) {
                    q_id[wave][pos] = static_cast<uint16_t>(lane | (s << kWaveLog2));
                    ++pos;
                }
            }
        }
        wave_lds_sync();
        const int m_lo = static_cast<int>(m), m_hi = static_cast<int>(m >> 32);
        const int task_lo = static_cast<int>(task), task_hi = static_cast<int>(task >> 32);
        // the stored starts of every round's segments (round k: queue entry
        // 64 k + lane; at most 8 rounds), all loaded before the first round
        // stores anything: one counter tracks a wave's loads and stores, so
        // a load issued after stores is waited for together with them
        float t_seg[kSegsPerChunk];
#pragma unroll
        for (int k = 0; k < kSegsPerChunk; ++k) {
            t_seg[k] = 0.0f;
            if (k * kWave < total) {
                const int q = k * kWave + lane;
                const bool has = q < total;
                const int id = has ? static_cast<int>(q_id[wave][q]) : 0;
                const int src = id & (kWave - 1);
                const int64_t s_task = (static_cast<int64_t>(lane_value(task_hi, src)) << 32) |
                                       static_cast<uint32_t>(lane_value(task_lo, src));
                if (has) t_seg[k] = seg_t[s_task * kSegsPerChunk + (id >> kWaveLog2)];
            }
        }
        for (int qb = 0; qb < total; qb += kWave) {
            const int q = qb + lane;
            const bool has = q < total;
            const int id = has ? static_cast<int>(q_id[wave][q]) : 0;
            const int src = id & (kWave - 1);
            const int s = id >> kWaveLog2;
            const float seg_t0 = t_seg[0];
#pragma unroll
            for (int k = 0; k + 1 < kSegsPerChunk; ++k) t_seg[k] = t_seg[k + 1];  // the next round's first
            // the queued segment's task, gathered from its lane (every lane
            // takes part in the permutes)
            const float s_far = lane_value(t_far, src);
            const int s_limit = lane_value(l_limit, src);
            const int s_base = lane_value(base, src);
            const int s_ray = lane_value(static_cast<int>(r), src);
            const int64_t s_start = (static_cast<int64_t>(lane_value(static_cast<int>(l_start >> 32), src)) << 32) |
                                    static_cast<uint32_t>(lane_value(static_cast<int>(l_start), src));
            const uint64_t s_m = (static_cast<uint64_t>(static_cast<uint32_t>(lane_value(m_hi, src))) << 32) |
                                 static_cast<uint32_t>(lane_value(m_lo, src));
            float tb[kConeBatch + 1];
            uint32_t hits = 0u;
            int first = 0;  // the segment's first sample within its ray
            if (has) {
                const int n_valid = cone_steps(seg_t0, s_far, p, tb);
                hits = static_cast<uint32_t>(s_m >> (s * kConeBatch)) & 0xffu & ((1u << n_valid) - 1u);
                first = s_base + static_cast<int>(__popcll(s_m & ((1ull << (s * kConeBatch)) - 1ull)));
            }
            const int n_out = has ? min(__popc(hits), max(s_limit - first, 0)) : 0;
            const int slot0 = wave_inclusive_sum(n_out) - n_out;
            const int n_slots = read_lane(slot0 + n_out, kWave - 1);
            if (has) {
                e_pos[wave][lane] = s_start + first;
                e_slot[wave][lane] = slot0;
                e_ray[wave][lane] = s_ray;
                int k = 0;
#pragma unroll
                for (int u = 0; u < kConeBatch; ++u) {
                    if (((hits >> u) & 1u) != 0u && k < n_out) {
                        s_t0[wave][slot0 + k] = tb[u];
                        s_t1[wave][slot0 + k] = tb[u + 1];
                        s_entry[wave][slot0 + k] = static_cast<uint8_t>(lane);
                        ++k;
                    }
                }
            }
            wave_lds_sync();
            for (int k = lane; k < n_slots; k += kWave) {
                const int e = s_entry[wave][k];
                const int64_t pos = e_pos[wave][e] + (k - e_slot[wave][e]);
                if (pos >= 0 && pos < capacity) {
                    t_starts[pos] = s_t0[wave][k];
                    t_ends[pos] = s_t1[wave][k];
                    ray_indices[pos] = e_ray[wave][e];
                } else {
                    overflow = true;
                }
            }
            wave_lds_sync();  // the queue and the slots are written again next round
        }
    }
    if (t_last < INFINITY) {
        // the last stored chunk: walk it, then look the rest of the ray up
        // again (rays of more than n_masks chunks of candidates, rare)
        const int64_t last = static_cast<int64_t>(n_masks - 1) * n_rays + ray;
        const uint64_t m = masks[last];
        int idx = chunk_base[last] + static_cast<int>(__popcll(m));
        const float t_far = t_far_in[ray];
        float t = t_last;
        bool ended = false;
        for (int s = 0; s < kSegsPerChunk && !ended; ++s) {
            float tb[kConeBatch + 1];
            const int n_valid = cone_steps(t, t_far, p, tb);
            ended = n_valid < kConeBatch;
            t = tb[kConeBatch];
        }
        if (!ended && idx < limit) {
            float o[3], d[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                o[c] = rays_o[3 * ray + c];
                d[c] = rays_d[3 * ray + c];
            }
            uint32_t word0;
            grid_of_ray<LOOKUP>(grid_id, ray, g, word0);
            SkipRay sk{};
            float skip_end = -INFINITY;
            for (int k0 = n_masks * kWave; k0 < kMaxCandidates && idx < limit; k0 += kConeBatch) {
                float tb[kConeBatch + 1];
                const int n_valid = cone_steps(t, t_far, p, tb);
                const uint32_t hits =
                    cone_hits<LOOKUP, false>(bits, nullptr, g, sk, skip_end, word0, o, d, tb, n_valid) &
                    ((1u << n_valid) - 1u);
#pragma unroll
                for (int u = 0; u < kConeBatch; ++u) {
                    if (((hits >> u) & 1u) != 0u && idx < limit) {
                        const int64_t pos = start + idx;
                        if (pos >= 0 && pos < capacity) {
                            t_starts[pos] = tb[u];
                            t_ends[pos] = tb[u + 1];
                            ray_indices[pos] = static_cast<int32_t>(ray);
                        } else {
                            overflow = true;
                        }
                        ++idx;
                    }
                }
                if (n_valid < kConeBatch) break;
                t = tb[kConeBatch];
            }
        }
    }
    if (overflow && status != nullptr) *status = NACC_ECAPACITY;
}

template <int LOOKUP, bool SKIP>
__global__ __launch_bounds__(kRaysPerBlock) void fill_cone_kernel(
    const float* __restrict__ rays_o, const float* __restrict__ rays_d,
    const int32_t* __restrict__ grid_id, int64_t n_rays, const uint32_t* __restrict__ bits,
    const uint8_t* __restrict__ skip, GridK g, ClipK c, StepK p, const int32_t* __restrict__ packed_info,
    int64_t capacity, float* __restrict__ t_starts, float* __restrict__ t_ends, int32_t* __restrict__ status) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kRaysPerBlock + threadIdx.x;
    if (r >= n_rays) return;
    const int limit = packed_info[2 * r + 1];
    if (limit == 0) return;
    bool overflow = false;
    // the ray indices are written by expand_rays_kernel, contiguously
    fill_ray_cone<LOOKUP, SKIP>(r, rays_o, rays_d, grid_id, bits, skip, g, c, p, packed_info[2 * r], limit, capacity,
                                t_starts, t_ends, overflow);
    if (overflow && status != nullptr) *status = NACC_ECAPACITY;
}

// ray_indices[start_r + i] = r for i < count_r: one wave per ray at a time,
// 64 consecutive slots per store (the lane-per-ray fill would scatter them).
constexpr int kExpandThreads = 256;

__global__ __launch_bounds__(kExpandThreads) void expand_rays_kernel(const int32_t* __restrict__ packed_info,
                                                                     int64_t n_rays, int64_t capacity,
                                                                     int32_t* __restrict__ ray_indices) {
    const int lane = lane_id();
    const int64_t waves = static_cast<int64_t>(gridDim.x) * (kExpandThreads / kWave);
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * (kExpandThreads / kWave) + threadIdx.x / kWave; r < n_rays;
         r += waves) {
        const int64_t start = packed_info[2 * r];
        const int count = packed_info[2 * r + 1];
        for (int i = lane; i < count; i += kWave) {
            const int64_t pos = start + i;
            if (pos >= 0 && pos < capacity) ray_indices[pos] = static_cast<int32_t>(r);
        }
    }
}

__global__ void set_status_kernel(int32_t* status, int32_t value) { *status = value; }

// --------------------------------------------------------------------------
// Host side: validation and launch.
// --------------------------------------------------------------------------


// Longest [t_near, t_far) a ray can have: far - near, and (unless the
// lookup contracts space, which has no clip box) the clip box's diagonal.
double clip_span(const nacc_grid_desc& grid, const nacc_march_params& p) {
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
    return span;
}

// Upper bound of the lattice candidates of one ray (at most kMaxCandidates).
// Cone steps never shrink as t grows, so a ray entering later than the near
// plane covers its (at most span long) range in no more steps than the
// recurrence started at the near plane; two extra candidates absorb the
// rounding of the sums.
int64_t candidate_bound(const nacc_grid_desc& grid, const nacc_march_params& p) {
    const double span = clip_span(grid, p);
    if (!(span > 0.0)) return 0;
    if (!std::isfinite(span)) return kMaxCandidates;
    if (p.cone == 0.0f) {
        return std::min<int64_t>(kMaxCandidates, static_cast<int64_t>(std::ceil(span / p.dt)) + 2);
    }
    const double end = static_cast<double>(p.near_plane) + span;
    float t = p.near_plane;
    int64_t k = 0;
    while (k < kMaxCandidates && static_cast<double>(t) < end) {
        const float step = fminf(fmaxf(t * p.cone, p.dt), p.dt_max);
        const float t1 = t + step;
        if (!(t1 > t)) return kMaxCandidates;
        t = t1;
        ++k;
    }
    return std::min<int64_t>(kMaxCandidates, k + 2);
}

// Workspace of the marching calls: the per-workgroup sums of the scan, then
// n_masks 64-bit occupancy masks per ray, one per chunk of 64 candidates,
// written by the count pass and replayed by the fill pass.  n_masks covers
// the longest possible ray (up to kMaxMaskChunks chunks).
// Cone steps add, for the chunk-parallel passes: t at the start of every
// chunk (chunk-major, +inf past the ray's candidates), each ray's t_far
// (-inf: no samples) and its hits past the stored chunks.
struct Layout {
    int64_t sums_bytes;
    int n_masks;
    int64_t chunk_t_off, t_far_off, extra_off;  // cone steps only (0 otherwise)
    int64_t base_off, seg_t_off;                // cone steps, segment passes
    int64_t live_off, tsum_off, tlist_off;      // cone steps, the task list of the segment passes
    int64_t bytes;
};

int64_t align256(int64_t b) { return ((b + 255) / 256) * 256; }

Layout workspace_layout(int64_t n_rays, const nacc_grid_desc& grid, const nacc_march_params& p) {
    Layout l;
    // the workgroup sums, then the scan's scratch
    const int64_t nb = num_blocks(n_rays);
    l.sums_bytes = align256((nb + scan_scratch_values(nb)) * static_cast<int64_t>(sizeof(int64_t)));
    l.n_masks = 0;
    if (p.dt > 0.0f) {
        const int64_t k = candidate_bound(grid, p);
        l.n_masks = static_cast<int>(std::min<int64_t>((k + kWave - 1) / kWave, kMaxMaskChunks));
    }
    l.bytes = l.sums_bytes + align256(n_rays * l.n_masks * static_cast<int64_t>(sizeof(uint64_t)));
    l.chunk_t_off = l.t_far_off = l.extra_off = l.base_off = l.seg_t_off = 0;
    l.live_off = l.tsum_off = l.tlist_off = 0;
    if (p.cone > 0.0f) {
        l.chunk_t_off = l.bytes;
        l.t_far_off = l.chunk_t_off + align256(n_rays * l.n_masks * static_cast<int64_t>(sizeof(float)));
        l.extra_off = l.t_far_off + align256(n_rays * static_cast<int64_t>(sizeof(float)));
        l.base_off = l.extra_off + align256(n_rays * static_cast<int64_t>(sizeof(int32_t)));
        l.seg_t_off = l.base_off + align256(n_rays * l.n_masks * static_cast<int64_t>(sizeof(int32_t)));
        l.live_off = l.seg_t_off + align256(n_rays * l.n_masks * kSegsPerChunk * static_cast<int64_t>(sizeof(float)));
        l.tsum_off = l.live_off + align256(n_rays * static_cast<int64_t>(sizeof(uint64_t)));
        const int64_t n_sums = nb * l.n_masks;  // per (chunk, workgroup), the total, the scan's scratch
        l.tlist_off = l.tsum_off + align256((n_sums + 1 + scan_scratch_values(n_sums)) *
                                            static_cast<int64_t>(sizeof(int64_t)));
        l.bytes = l.tlist_off + align256(n_rays * l.n_masks * static_cast<int64_t>(sizeof(int32_t)));
    }
    return l;
}

struct ConeWork {
    uint64_t* masks;      // [n_masks][n_rays]
    float* chunk_t;       // [n_masks][n_rays]
    float* t_far;         // [n_rays]
    int32_t* extra;       // [n_rays]
    int32_t* chunk_base;  // [n_masks][n_rays]: samples of the ray before each chunk
    float* seg_t;         // [n_masks][n_rays][kSegsPerChunk]: t at the start of segments holding samples
    uint64_t* live_chunks;  // [n_rays]: chunks in the task list (contraction lookup)
    int64_t* task_sums;     // [n_masks][workgroups] + 1: scan of the task counts, then the total
    int32_t* task_list;     // [n_masks * n_rays]
    int n_masks;
};

ConeWork cone_work(void* workspace, const Layout& l) {
    char* b = static_cast<char*>(workspace);
    ConeWork w;
    w.masks = reinterpret_cast<uint64_t*>(b + l.sums_bytes);
    w.chunk_t = reinterpret_cast<float*>(b + l.chunk_t_off);
    w.t_far = reinterpret_cast<float*>(b + l.t_far_off);
    w.extra = reinterpret_cast<int32_t*>(b + l.extra_off);
    w.chunk_base = reinterpret_cast<int32_t*>(b + l.base_off);
    w.seg_t = reinterpret_cast<float*>(b + l.seg_t_off);
    w.live_chunks = reinterpret_cast<uint64_t*>(b + l.live_off);
    w.task_sums = reinterpret_cast<int64_t*>(b + l.tsum_off);
    w.task_list = reinterpret_cast<int32_t*>(b + l.tlist_off);
    w.n_masks = l.n_masks;
    return w;
}

// Workgroups per group of kRaysPerBlock rays in the uniform-step kernels:
// small batches are spread over more workgroups (the chip has 256 CUs), so
// that each wave walks fewer rays one after the other; results do not
// depend on it.
int march_split(int64_t groups) { return groups < 256 ? 4 : (groups < 512 ? 2 : 1); }

// Halo bits of a skip buffer (see halo_offset).
const uint32_t* halo_of(const uint8_t* skip, const GridK& g) {
    return skip == nullptr ? nullptr
                           : reinterpret_cast<const uint32_t*>(skip + halo_offset(g.res, g.n_grids));
}

template <int LOOKUP, bool SKIP, int WAVES>
void launch_count_uniform(int64_t nb, hipStream_t s, const float* o, const float* d, const int32_t* gid, int64_t n,
                          const uint32_t* bits, const uint8_t* skip, const GridK& g, const ClipK& c, const StepK& p,
                          int32_t* packed, int64_t* sums, uint64_t* masks, int n_masks) {
    const int split = march_split(nb);
    if (split > 1) {
        hipLaunchKernelGGL(zero_sums_kernel, dim3(static_cast<unsigned>((nb + 255) / 256)), dim3(256), 0, s, sums,
                           nb);
    }
    hipLaunchKernelGGL((count_uniform_kernel<LOOKUP, SKIP, WAVES>), dim3(static_cast<unsigned>(nb * split)),
                       dim3(WAVES * kWave), 0, s, o, d, gid, n, bits, skip, halo_of(skip, g), g, c, p, packed, sums,
                       masks, n_masks, split);
}

template <int LOOKUP, bool SKIP, int WAVES>
void launch_fill_uniform(int64_t nb, hipStream_t s, const float* o, const float* d, const int32_t* gid, int64_t n,
                         const uint32_t* bits, const uint8_t* skip, const GridK& g, const ClipK& c, const StepK& p,
                         const int32_t* packed, int64_t capacity, int32_t* ri, float* ts, float* te, int32_t* status,
                         const uint64_t* masks, int n_masks) {
    const int split = march_split(nb);
    hipLaunchKernelGGL((fill_uniform_kernel<LOOKUP, SKIP, WAVES>), dim3(static_cast<unsigned>(nb * split)),
                       dim3(WAVES * kWave), 0, s, o, d, gid, n, bits, skip, g, c, p, packed, capacity, ri, ts, te,
                       status, masks, n_masks, split);
}

unsigned task_blocks(int n_masks, int64_t n_rays) {
    return static_cast<unsigned>((static_cast<int64_t>(n_masks) * n_rays + kTaskThreads - 1) / kTaskThreads);
}

// The segment passes run over a task list of the chunks the starts pass
// could not prove empty: contraction lookup with halo bits, task ids within
// int32.
template <int LOOKUP, bool SKIP>
bool cone_task_list(const ConeWork& cw, int64_t n_rays) {
    return SKIP && LOOKUP == NACC_LOOKUP_CONTRACT && cw.n_masks > 0 &&
           static_cast<int64_t>(cw.n_masks) * n_rays <= INT32_MAX;
}

template <int LOOKUP, bool SKIP>
void launch_count_impl(const ConeWork* cw, int64_t nb, hipStream_t s, const float* o, const float* d,
                       const int32_t* gid, int64_t n, const uint32_t* bits, const uint8_t* skip, const GridK& g,
                       const ClipK& c, const StepK& p, int32_t* packed, int64_t* sums, uint64_t* masks, int n_masks) {
    if (cw != nullptr) {  // cone steps
        const bool listed = cone_task_list<LOOKUP, SKIP>(*cw, n);
        const ConeTable tab = cone_table(p, cw->n_masks);
        if (listed) {
            hipLaunchKernelGGL((cone_starts_kernel<LOOKUP, true>), dim3(nb), dim3(kRaysPerBlock), 0, s, o, d, gid, n,
                               g, c, p, cw->n_masks, cw->chunk_t, cw->t_far, cw->extra, halo_of(skip, g),
                               cw->live_chunks, cw->task_sums, tab);
            const int64_t n_sums = nb * cw->n_masks;
            scan_exclusive(cw->task_sums, n_sums, cw->task_sums + n_sums, cw->task_sums + n_sums + 1, s);
            hipLaunchKernelGGL(task_list_kernel, dim3(nb), dim3(kRaysPerBlock), 0, s, cw->task_sums, n,
                               cw->n_masks, cw->live_chunks, cw->task_list);
        } else {
            hipLaunchKernelGGL((cone_starts_kernel<LOOKUP, false>), dim3(nb), dim3(kRaysPerBlock), 0, s, o, d, gid, n,
                               g, c, p, cw->n_masks, cw->chunk_t, cw->t_far, cw->extra, nullptr, nullptr, nullptr, tab);
        }
        if (cw->n_masks > 0 && SKIP) {  // segments through the halo bits
            hipLaunchKernelGGL((count_cone_segments_kernel<LOOKUP>), dim3(task_blocks(cw->n_masks, n)),
                               dim3(kTaskThreads), 0, s, o, d, gid, n, bits, halo_of(skip, g), g, p, cw->n_masks,
                               cw->chunk_t, cw->t_far, cw->masks, cw->extra, cw->seg_t,
                               listed ? cw->task_list : nullptr,
                               listed ? cw->task_sums + nb * cw->n_masks : nullptr, tab);
        } else if (cw->n_masks > 0) {
            hipLaunchKernelGGL((count_cone_chunks_kernel<LOOKUP, false>), dim3(task_blocks(cw->n_masks, n)),
                               dim3(kTaskThreads), 0, s, o, d, gid, n, bits, skip, g, p, cw->n_masks, cw->chunk_t,
                               cw->t_far, cw->masks, cw->extra);
        }
        hipLaunchKernelGGL(cone_counts_kernel, dim3(nb), dim3(kRaysPerBlock), 0, s, n, cw->n_masks, p.max_per_ray,
                           cw->masks, cw->extra, packed, sums, SKIP ? cw->chunk_base : nullptr,
                           listed ? cw->live_chunks : nullptr, SKIP ? cw->live_chunks : nullptr);
        return;
    }
    switch (tuning().march_waves_per_group) {
        case 1: launch_count_uniform<LOOKUP, SKIP, 1>(nb, s, o, d, gid, n, bits, skip, g, c, p, packed, sums, masks, n_masks); break;
        case 2: launch_count_uniform<LOOKUP, SKIP, 2>(nb, s, o, d, gid, n, bits, skip, g, c, p, packed, sums, masks, n_masks); break;
        case 8: launch_count_uniform<LOOKUP, SKIP, 8>(nb, s, o, d, gid, n, bits, skip, g, c, p, packed, sums, masks, n_masks); break;
        case 16: launch_count_uniform<LOOKUP, SKIP, 16>(nb, s, o, d, gid, n, bits, skip, g, c, p, packed, sums, masks, n_masks); break;
        default: launch_count_uniform<LOOKUP, SKIP, 4>(nb, s, o, d, gid, n, bits, skip, g, c, p, packed, sums, masks, n_masks); break;
    }
}

template <int LOOKUP, bool SKIP>
void launch_fill_impl(bool cone, const ConeWork* cw, int64_t nb, hipStream_t s, const float* o, const float* d,
                      const int32_t* gid, int64_t n, const uint32_t* bits, const uint8_t* skip, const GridK& g,
                      const ClipK& c, const StepK& p, const int32_t* packed, int64_t capacity, int32_t* ri, float* ts,
                      float* te, int32_t* status, const uint64_t* masks, int n_masks) {
    if (cone) {
        if (cw != nullptr && cw->n_masks > 0 && SKIP) {
            // the segment count's masks, segment starts and chunks holding
            // samples, ray-major (the ray indices written with the samples)
            const int64_t per_block = static_cast<int64_t>(kTaskWaves) * kFillRays;
            const unsigned blocks = static_cast<unsigned>((n + per_block - 1) / per_block);
            hipLaunchKernelGGL((fill_cone_rays_kernel<LOOKUP>), dim3(blocks), dim3(kTaskThreads), 0, s, o, d, gid, n,
                               bits, g, p, cw->n_masks, cw->chunk_t, cw->t_far, cw->masks, cw->chunk_base,
                               cw->seg_t, cw->live_chunks, packed, capacity, ri, ts, te, status);
            return;
        } else if (cw != nullptr && cw->n_masks > 0) {  // replay the count pass's chunks, one lane per chunk
            hipLaunchKernelGGL((fill_cone_chunks_kernel<LOOKUP, false>), dim3(task_blocks(cw->n_masks, n)),
                               dim3(kTaskThreads), 0, s, o, d, gid, n, bits, skip, g, p, cw->n_masks, cw->chunk_t,
                               cw->t_far, cw->masks, packed, capacity, ts, te, status);
        } else {  // traversal, one lane per ray
            hipLaunchKernelGGL((fill_cone_kernel<LOOKUP, SKIP>), dim3(nb), dim3(kRaysPerBlock), 0, s, o, d, gid, n,
                               bits, skip, g, c, p, packed, capacity, ts, te, status);
        }
        const int64_t blocks = std::min<int64_t>((n + kExpandThreads / kWave - 1) / (kExpandThreads / kWave),
                                                 256 * 64);
        hipLaunchKernelGGL(expand_rays_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kExpandThreads), 0, s,
                           packed, n, capacity, ri);
        return;
    }
    switch (tuning().march_waves_per_group) {
        case 1: launch_fill_uniform<LOOKUP, SKIP, 1>(nb, s, o, d, gid, n, bits, skip, g, c, p, packed, capacity, ri, ts, te, status, masks, n_masks); break;
        case 2: launch_fill_uniform<LOOKUP, SKIP, 2>(nb, s, o, d, gid, n, bits, skip, g, c, p, packed, capacity, ri, ts, te, status, masks, n_masks); break;
        case 8: launch_fill_uniform<LOOKUP, SKIP, 8>(nb, s, o, d, gid, n, bits, skip, g, c, p, packed, capacity, ri, ts, te, status, masks, n_masks); break;
        case 16: launch_fill_uniform<LOOKUP, SKIP, 16>(nb, s, o, d, gid, n, bits, skip, g, c, p, packed, capacity, ri, ts, te, status, masks, n_masks); break;
        default: launch_fill_uniform<LOOKUP, SKIP, 4>(nb, s, o, d, gid, n, bits, skip, g, c, p, packed, capacity, ri, ts, te, status, masks, n_masks); break;
    }
}

// The skip field serves every lookup (res % 4 == 0).
template <int LOOKUP, typename... A>
void dispatch_count(const uint8_t* skip, const ConeWork* cw, int64_t nb, hipStream_t s, const float* o,
                    const float* d, const int32_t* gid, int64_t n, const uint32_t* bits, A&&... a) {
    if (skip != nullptr) {
        launch_count_impl<LOOKUP, true>(cw, nb, s, o, d, gid, n, bits, skip, a...);
        return;
    }
    launch_count_impl<LOOKUP, false>(cw, nb, s, o, d, gid, n, bits, nullptr, a...);
}

template <int LOOKUP, typename... A>
void dispatch_fill(const uint8_t* skip, bool cone, const ConeWork* cw, int64_t nb, hipStream_t s, const float* o,
                   const float* d, const int32_t* gid, int64_t n, const uint32_t* bits, A&&... a) {
    if (skip != nullptr) {
        launch_fill_impl<LOOKUP, true>(cone, cw, nb, s, o, d, gid, n, bits, skip, a...);
        return;
    }
    launch_fill_impl<LOOKUP, false>(cone, cw, nb, s, o, d, gid, n, bits, nullptr, a...);
}

const uint8_t* usable_skip(const uint8_t* skip, const nacc_grid_desc& grid) {
    if (skip == nullptr || grid.res % 4 != 0) return nullptr;
    return skip;
}

// Count, scan and starts of one marching call, given the scan sums and (for
// uniform steps, nullable) the chunk masks or (cone steps) the cone
// workspace.
int march_count_launch(const float* rays_o, const float* rays_d, const int32_t* grid_id, int64_t n_rays,
                       const uint32_t* grid_bits, const uint8_t* grid_skip, const nacc_grid_desc* grid,
                       const nacc_march_params* params, int32_t* packed_info, int64_t* total, int64_t* sums,
                       uint64_t* masks, int n_masks, const ConeWork* cw, hipStream_t s) {
    GridK g;
    ClipK c;
    StepK p;
    make_constants(*grid, *params, g, c, p);
    const int64_t nb = num_blocks(n_rays);
    const uint8_t* skip = usable_skip(grid_skip, *grid);
    int st = NACC_OK;
    if (nb > 0) {
        switch (grid->lookup) {
            case NACC_LOOKUP_AABB:
                dispatch_count<NACC_LOOKUP_AABB>(skip, cw, nb, s, rays_o, rays_d, grid_id, n_rays, grid_bits, g, c,
                                                 p, packed_info, sums, masks, n_masks);
                break;
            case NACC_LOOKUP_CASCADE:
                dispatch_count<NACC_LOOKUP_CASCADE>(skip, cw, nb, s, rays_o, rays_d, grid_id, n_rays, grid_bits, g,
                                                    c, p, packed_info, sums, masks, n_masks);
                break;
            default:
                dispatch_count<NACC_LOOKUP_CONTRACT>(skip, cw, nb, s, rays_o, rays_d, grid_id, n_rays, grid_bits,
                                                     g, c, p, packed_info, sums, masks, n_masks);
                break;
        }
        st = check_launch("march count");
        if (st != NACC_OK) return st;
    }
    scan_exclusive(sums, nb, total, sums + nb, s);
    st = check_launch("march scan");
    if (st != NACC_OK) return st;
    if (nb > 0) {
        hipLaunchKernelGGL(finalize_starts_kernel, dim3(nb), dim3(kRaysPerBlock), 0, s, sums, n_rays,
                           packed_info);
        st = check_launch("march starts");
    }
    return st;
}

}  // namespace

extern "C" {

int64_t nacc_march_workspace_size(int64_t n_rays, const nacc_grid_desc* grid, const nacc_march_params* params) {
    clear_error();
    if (n_rays < 0 || grid == nullptr || params == nullptr) return -1;
    if (validate(nullptr, nullptr, 0, nullptr, grid, params) != NACC_OK) return -1;
    return workspace_layout(n_rays, *grid, *params).bytes;
}

int64_t nacc_march_max_samples_per_ray(const nacc_grid_desc* grid, const nacc_march_params* params) {
    clear_error();
    if (grid == nullptr || params == nullptr) {
        set_error(NACC_EINVAL, "grid and params must be non-NULL");
        return -1;
    }
    const nacc_march_params& p = *params;
    if (!(std::isfinite(p.dt) && p.dt > 0.0f) || !(p.cone >= 0.0f) || std::isnan(p.near_plane) ||
        std::isnan(p.far_plane)) {
        set_error(NACC_EINVAL, "invalid marching parameters");
        return -1;
    }
    int64_t bound = candidate_bound(*grid, p);
    if (p.max_per_ray > 0) bound = std::min<int64_t>(bound, p.max_per_ray);
    return bound;
}

int nacc_march_count(const float* rays_o, const float* rays_d, const int32_t* grid_id, int64_t n_rays,
                     const uint32_t* grid_bits, const uint8_t* grid_skip, const nacc_grid_desc* grid,
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
    ConeWork cw_store{};
    const ConeWork* cw = nullptr;
    if (params->cone > 0.0f) {
        cw_store = cone_work(workspace, lay);
        cw = &cw_store;
    }
    return march_count_launch(rays_o, rays_d, grid_id, n_rays, grid_bits, grid_skip, grid, params, packed_info,
                              total, static_cast<int64_t*>(workspace), masks, lay.n_masks, cw, as_stream(stream));
}

int nacc_march_fill(const float* rays_o, const float* rays_d, const int32_t* grid_id, int64_t n_rays,
                    const uint32_t* grid_bits, const uint8_t* grid_skip, const nacc_grid_desc* grid,
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
    const uint8_t* skip = usable_skip(grid_skip, *grid);
    const Layout lay = workspace_layout(n_rays, *grid, *params);
    NACC_REQUIRE(workspace == nullptr || static_cast<int64_t>(workspace_bytes) >= lay.bytes, NACC_ESHAPE,
                 "workspace of %zu bytes, need %lld", workspace_bytes, static_cast<long long>(lay.bytes));
    const uint64_t* masks =
        workspace != nullptr && lay.n_masks > 0
            ? reinterpret_cast<const uint64_t*>(static_cast<const char*>(workspace) + lay.sums_bytes)
            : nullptr;
    ConeWork cw_store{};
    const ConeWork* cw = nullptr;
    if (cone && workspace != nullptr) {
        cw_store = cone_work(const_cast<void*>(workspace), lay);
        cw = &cw_store;
    }
    switch (grid->lookup) {
        case NACC_LOOKUP_AABB:
            dispatch_fill<NACC_LOOKUP_AABB>(skip, cone, cw, nb, s, rays_o, rays_d, grid_id, n_rays, grid_bits, g, c, p,
                                            packed_info, capacity, ray_indices, t_starts, t_ends, status, masks,
                                            lay.n_masks);
            break;
        case NACC_LOOKUP_CASCADE:
            dispatch_fill<NACC_LOOKUP_CASCADE>(skip, cone, cw, nb, s, rays_o, rays_d, grid_id, n_rays, grid_bits, g, c,
                                               p, packed_info, capacity, ray_indices, t_starts, t_ends, status, masks,
                                               lay.n_masks);
            break;
        default:
            dispatch_fill<NACC_LOOKUP_CONTRACT>(skip, cone, cw, nb, s, rays_o, rays_d, grid_id, n_rays, grid_bits, g, c,
                                                p, packed_info, capacity, ray_indices, t_starts, t_ends, status,
                                                masks, lay.n_masks);
            break;
    }
    return check_launch("march fill");
}

}  // extern "C"
