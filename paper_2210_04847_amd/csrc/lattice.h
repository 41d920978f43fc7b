// Shared by the marching kernels and the fused inference kernel: the FP32
// lattice contract of nacc.h (ray clip, cell lookup through the box,
// cascade or contraction transforms), the per-launch constants and the
// host-side validation of grid and marching parameters.  Every operation is
// one correctly rounded FP32 operation without FMA (the including files are
// compiled with -ffp-contract=off).
#pragma once

#include <cmath>

#include "common.h"

#pragma clang fp contract(off)

namespace {

using namespace nacc;
using namespace nacc::dev;

constexpr int kMaxCandidates = 1 << 24;

struct GridK {
    float lo[3];
    float s[3];        // fl32(res / (hi - lo))
    float top;         // (float)(res - 1)
    float base;        // cascade: half-extent of level 0 (a power of two)
    float inv_base;    // 1 / base (exact)
    int res;
    int n_grids;
    uint32_t words;    // 32-bit words per grid
    int coarse;          // coarse cells per axis of the skip field (res / 4)
    uint32_t skip_cells;  // bytes per grid of the skip field (coarse^3)
    uint32_t res2, coarse2;  // res^2, coarse^2
    uint32_t bytes;          // bytes of all grids' bit arrays (< 2^32)
    int halo_res;            // halo cells per axis (res / 2)
    uint32_t halo_res2;      // halo_res^2
    uint32_t halo_words;     // 32-bit words per grid of the halo bits
    uint32_t halo_bytes;     // bytes of all grids' halo bits
    float contract_delta;    // contraction lookup: see probe
};

// The grids' words are read through a buffer resource: 32-bit byte offsets
// (no 64-bit address arithmetic per lookup) and a hardware range check (a
// word past the arrays reads as 0; the cell indices are clamped, so none
// is).  The resource's last word selects 32-bit untyped data.
constexpr int kBufferWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t grid_rsrc(const uint32_t* bits, const GridK& g) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(bits), 0, static_cast<int>(g.bytes), kBufferWord3);
}

__device__ __forceinline__ uint32_t grid_word(__amdgpu_buffer_rsrc_t rs, uint32_t word) {
    return __builtin_amdgcn_raw_buffer_load_b32(rs, word << 2, 0, 0);
}

struct ClipK {
    float lo[3];
    float hi[3];
};

struct StepK {
    float near_plane, far_plane, dt, dt_max, cone;
    int max_per_ray;
    // cone steps: every step from a t between the near and far planes
    // advances t (dt exceeds twice an ulp of the largest such |t|), so the
    // recurrence can be walked without testing each step for a stall
    int no_stall;
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

// min(max(u, 0), top) in one instruction (the median of the three; no NaN
// reaches it for finite rays).
__device__ __forceinline__ float clamp_cell(float u, float top) { return __builtin_amdgcn_fmed3f(u, 0.0f, top); }

// Cascade level of a point with m = max_i |x_i|: the number of levels
// l < n_grids - 1 with m > base 2^l, i.e. the smallest l with m <= base 2^l,
// clamped to the last level.  q = m / base is exact (base is a power of
// two), and the smallest l with q <= 2^l is read off q's exponent and
// mantissa: q = 1.f 2^(e-127) gives e - 127, plus one unless f = 0.  Zero,
// subnormal and NaN m give level 0, as the comparisons do.
__device__ __forceinline__ int cascade_level(float m, const GridK& g) {
    const uint32_t b = __float_as_uint(m * g.inv_base);
    const int e = static_cast<int>(b >> 23);
    int level = e - 127 + ((b & 0x7fffffu) != 0u ? 1 : 0);
    if (e == 0 || !(m == m)) level = 0;
    return min(max(level, 0), g.n_grids - 1);
}

// Where point x is looked up: the grid word and bit of its fine cell, the
// byte of its coarse cell in the skip field, and (cascade) its level and
// m = max_i |x_i|.  `word0` is the first word of the ray's grid (box /
// contraction lookups); the cascade picks its level itself.
struct Probe {
    uint32_t word;
    uint32_t bit;
    uint32_t coarse;
    int level;
    float m;
};

template <int LOOKUP>
__device__ __forceinline__ Probe probe(const GridK& g, uint32_t word0, float x0, float x1, float x2) {
    Probe q;
    q.level = 0;
    q.m = 0.0f;
    uint32_t grid = word0 / g.words;
    if (LOOKUP == NACC_LOOKUP_CASCADE) {
        q.m = fmaxf(fmaxf(fabsf(x0), fabsf(x1)), fabsf(x2));
        q.level = cascade_level(q.m, g);
        x0 = ldexpf(x0, -q.level);
        x1 = ldexpf(x1, -q.level);
        x2 = ldexpf(x2, -q.level);
        grid = static_cast<uint32_t>(q.level);
        word0 = grid * g.words;
    }
    float u0, u1, u2;  // cell coordinates
    if (LOOKUP == NACC_LOOKUP_CONTRACT) {
        // The FP32 contract contracts x with a correctly rounded square root
        // and divisions: n = |x|, f = (2 - 1/n) / n.  The cell is decided
        // first from the hardware square root and reciprocal (a few ulps);
        // it is the contract's cell wherever the fast cell coordinates lie
        // farther than contract_delta from a cell boundary (an integer) and
        // |x| is not near 1, because the two evaluations differ by less:
        // with every hardware result within 2 ulps, the fast u is within
        // s (48.8 + 2 |lo|) 2^-24 of the exact value and the contract's
        // within s (22.4 + 2 |lo|) 2^-24 (|y| < 2 after contraction), and
        // contract_delta is twice their sum.  Other lanes evaluate the
        // contract itself.
        const float n2 = (x0 * x0 + x1 * x1) + x2 * x2;
        const float na = __builtin_amdgcn_sqrtf(n2);
        q.m = na;  // |x|, for the skip bound (which allows 2^-18 relative)
        bool exact = fabsf(na - 1.0f) <= 0x1p-20f;
        if (na > 1.0f) {
            const float ia = __builtin_amdgcn_rcpf(na);
            const float fa = (2.0f - ia) * ia;
            u0 = (x0 * fa - g.lo[0]) * g.s[0];
            u1 = (x1 * fa - g.lo[1]) * g.s[1];
            u2 = (x2 * fa - g.lo[2]) * g.s[2];
            exact = exact || fabsf(u0 - rintf(u0)) <= g.contract_delta ||
                    fabsf(u1 - rintf(u1)) <= g.contract_delta || fabsf(u2 - rintf(u2)) <= g.contract_delta;
        } else {  // not contracted, as in the contract
            u0 = (x0 - g.lo[0]) * g.s[0];
            u1 = (x1 - g.lo[1]) * g.s[1];
            u2 = (x2 - g.lo[2]) * g.s[2];
        }
        if (exact) {
            const float n = sqrtf(n2);
            if (n > 1.0f) {
                const float f = (2.0f - 1.0f / n) / n;
                x0 = x0 * f;
                x1 = x1 * f;
                x2 = x2 * f;
            }
            u0 = (x0 - g.lo[0]) * g.s[0];
            u1 = (x1 - g.lo[1]) * g.s[1];
            u2 = (x2 - g.lo[2]) * g.s[2];
        }
    } else {
        u0 = (x0 - g.lo[0]) * g.s[0];
        u1 = (x1 - g.lo[1]) * g.s[1];
        u2 = (x2 - g.lo[2]) * g.s[2];
    }
    const uint32_t j0 = static_cast<uint32_t>(static_cast<int>(clamp_cell(u0, g.top)));
    const uint32_t j1 = static_cast<uint32_t>(static_cast<int>(clamp_cell(u1, g.top)));
    const uint32_t j2 = static_cast<uint32_t>(static_cast<int>(clamp_cell(u2, g.top)));
    // j < res <= 1024 and res^2 <= 2^20: every factor fits the 24-bit
    // multiplier, every product 32 bits
    const uint32_t res = static_cast<uint32_t>(g.res);
    const uint32_t cell = __umul24(j0, g.res2) + (__umul24(j1, res) + j2);
    q.word = word0 + (cell >> 5);
    q.bit = cell & 31u;
    const uint32_t cc = static_cast<uint32_t>(g.coarse);
    q.coarse = grid * g.skip_cells + (__umul24(j0 >> 2, g.coarse2) + (__umul24(j1 >> 2, cc) + (j2 >> 2)));
    return q;
}

// Occupancy bit of point x.
template <int LOOKUP>
__device__ __forceinline__ bool occupied(const uint32_t* __restrict__ bits, uint32_t word0,
                                         const GridK& g, float x0, float x1, float x2) {
    const Probe q = probe<LOOKUP>(g, word0, x0, x1, x2);
    return ((grid_word(grid_rsrc(bits, g), q.word) >> q.bit) & 1u) != 0u;
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

// Where a ray is marched: its clipped range and the first word of its grid
// (valid = false: an invalid grid id or a miss, no samples).  The uniform
// kernels compute the spans of a wave's rays lane-parallel, one ray per
// lane, and broadcast each one as the wave reaches its ray.
struct RaySpan {
    float t_near, t_far;
    uint32_t word0;
    uint32_t grid;  // index of the ray's grid (box / contraction lookups)
    bool valid;
    float o[3], d[3];  // the ray itself
};

template <int LOOKUP>
__device__ __forceinline__ RaySpan ray_span(int64_t r, const float* __restrict__ rays_o,
                                            const float* __restrict__ rays_d, const int32_t* __restrict__ grid_id,
                                            const GridK& g, const ClipK& c, const StepK& p) {
    RaySpan s;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        s.o[i] = rays_o[3 * r + i];
        s.d[i] = rays_d[3 * r + i];
    }
    s.valid = grid_of_ray<LOOKUP>(grid_id, r, g, s.word0);
    s.grid = s.word0 / g.words;  // one ray per lane: once per 64 rays of a wave
    s.valid = clip_ray(s.o, s.d, c, p.near_plane, p.far_plane, s.t_near, s.t_far) && s.valid;
    return s;
}

// Lane `lane`'s span (and ray) in every lane: the rays of a wave are loaded
// and clipped lane-parallel once, then broadcast one at a time, so no ray
// waits on loads of its own.
__device__ __forceinline__ RaySpan read_span(const RaySpan& s, int lane) {
    RaySpan b;
    b.t_near = read_lane(s.t_near, lane);
    b.t_far = read_lane(s.t_far, lane);
    b.word0 = static_cast<uint32_t>(read_lane(static_cast<int>(s.word0), lane));
    b.grid = static_cast<uint32_t>(read_lane(static_cast<int>(s.grid), lane));
    b.valid = read_lane(s.valid ? 1 : 0, lane) != 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        b.o[i] = read_lane(s.o[i], lane);
        b.d[i] = read_lane(s.d[i], lane);
    }
    return b;
}

// ---------------------------------------------------------------------------
// Uniform steps through the box lookup with the halo bits of the skip
// buffer.  A ray's candidates are grouped into segments of G consecutive
// ones (segment j: candidates [j G, j G + G)); a wave tests 64 segments at
// once, one halo bit each at the segment's centre, and then looks up one by
// one only the candidates of the segments whose bit is set, 64 at a time
// (64 / G segments per iteration, in segment order, so the ballots still
// list the samples in t order).
//
// A clear bit proves its segment empty.  The segment's midpoints lie within
// (G/2) dt of its centre in t, so their fine-cell coordinates
// u_i = (x_i - lo_i) s_i differ from the centre's by less than
// v (G/2) dt plus rounding, v = max_i s_i |d_i|.  G is the largest power of
// two up to 32 that keeps this below kHaloReach cells; the cells of the
// midpoints then lie within kHaloReach cells of the centre's cell (clamping
// into the grid only brings coordinates closer), so within kHaloReach cells
// of the centre's 2x2x2 halo cell on every axis, and a clear halo bit says
// none of those cells is occupied.  Rays that would need G < 8 are marched
// candidate by candidate.  The samples are exactly those of the plain
// traversal.
// ---------------------------------------------------------------------------
constexpr int kMinSegmentLog2 = 3;  // segments of 8, 16 or 32 candidates

struct SegRay {
    int log_g;       // log2 of the candidates per segment; 0: no segments
    uint32_t halo0;  // first halo word of the ray's grid
};

__device__ __forceinline__ SegRay seg_ray(const GridK& g, const RaySpan& span, const StepK& p) {
    SegRay sg{0, 0u};
    const float* o = span.o;
    const float* d = span.d;
    const float v = fmaxf(fmaxf(g.s[0] * fabsf(d[0]), g.s[1] * fabsf(d[1])), g.s[2] * fabsf(d[2]));
    const float smax = fmaxf(fmaxf(g.s[0], g.s[1]), g.s[2]);
    const float omax = fmaxf(fmaxf(fabsf(o[0]), fabsf(o[1])), fabsf(o[2]));
    const float dmax = fmaxf(fmaxf(fabsf(d[0]), fabsf(d[1])), fabsf(d[2]));
    const float tmax = fmaxf(fabsf(span.t_near), fabsf(span.t_far));
    // allowances in cells, each taken generously: the rounding of both
    // positions (a few ulps of the largest coordinate the ray reaches), of
    // the cell coordinates, and of the t values (a few ulps of t, times v)
    const float slack_x = (omax + dmax * tmax + 1.0f) * 0x1p-20f;
    const float slack = 2.0f * smax * slack_x + static_cast<float>(g.res) * 0x1p-17f + v * tmax * 0x1p-20f;
    const float budget = static_cast<float>(kHaloReach) - slack;
    int lg = 5;
    while (lg >= kMinSegmentLog2 && !(v * ldexpf(p.dt, lg - 1) * (1.0f + 0x1p-10f) <= budget)) --lg;
    if (lg >= kMinSegmentLog2) {
        sg.log_g = lg;
        sg.halo0 = span.grid * g.halo_words;
    }
    return sg;
}

// Halo bit of the cell holding point x (the box lookup's clamped cell
// coordinates, halved).
__device__ __forceinline__ bool halo_bit(__amdgpu_buffer_rsrc_t rs, const GridK& g, uint32_t halo0, float x0,
                                         float x1, float x2) {
    const uint32_t j0 = static_cast<uint32_t>(static_cast<int>(clamp_cell((x0 - g.lo[0]) * g.s[0], g.top)));
    const uint32_t j1 = static_cast<uint32_t>(static_cast<int>(clamp_cell((x1 - g.lo[1]) * g.s[1], g.top)));
    const uint32_t j2 = static_cast<uint32_t>(static_cast<int>(clamp_cell((x2 - g.lo[2]) * g.s[2], g.top)));
    const uint32_t cell =
        __umul24(j0 >> 1, g.halo_res2) + (__umul24(j1 >> 1, static_cast<uint32_t>(g.halo_res)) + (j2 >> 1));
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(rs, (halo0 + (cell >> 5)) << 2, 0, 0);
    return ((w >> (cell & 31u)) & 1u) != 0u;
}

// Live-segment ballot of block b of a ray's segments (segment j = b 64 +
// lane): its first candidate lies before t_far (ballot `vm`, returned too)
// and the halo bit at its centre is set.
__device__ __forceinline__ uint64_t live_segments(const RaySpan& span, const uint32_t* __restrict__ halo,
                                                  const GridK& g, const StepK& p, const SegRay& sg, int b,
                                                  uint64_t& vm) {
    const int lane = lane_id();
    const int log_g = sg.log_g;
    const int k_first = (b * kWave + lane) << log_g;
    // kMaxCandidates is a multiple of every G: a segment starting below it
    // ends at or below it
    const bool valid = k_first < kMaxCandidates && span.t_near + static_cast<float>(k_first) * p.dt < span.t_far;
    vm = ballot(valid);
    if (vm == 0ull) return 0ull;
    const __amdgpu_buffer_rsrc_t hrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(halo), 0, static_cast<int>(g.halo_bytes), kBufferWord3);
    const float tc = span.t_near + static_cast<float>(k_first + (1 << (log_g - 1))) * p.dt;
    const bool hb = halo_bit(hrs, g, sg.halo0, span.o[0] + span.d[0] * tc, span.o[1] + span.d[1] * tc,
                             span.o[2] + span.d[2] * tc);
    return vm & ballot(hb);
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
    NACC_REQUIRE(static_cast<int64_t>(grid->n_grids) * (cells / 8) <= INT32_MAX, NACC_ESHAPE,
                 "grid arrays of %lld bytes exceed 2^31 - 1", static_cast<long long>(grid->n_grids * (cells / 8)));
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
    g.inv_base = 1.0f / grid.hi[0];
    g.res = grid.res;
    g.n_grids = grid.n_grids;
    g.words = static_cast<uint32_t>(static_cast<int64_t>(grid.res) * grid.res * grid.res / 32);
    g.coarse = grid.res / 4;
    g.skip_cells = static_cast<uint32_t>(g.coarse) * g.coarse * g.coarse;
    g.res2 = static_cast<uint32_t>(grid.res) * static_cast<uint32_t>(grid.res);
    g.coarse2 = static_cast<uint32_t>(g.coarse) * static_cast<uint32_t>(g.coarse);
    g.bytes = static_cast<uint32_t>(static_cast<int64_t>(grid.n_grids) * g.words * 4);
    g.halo_res = grid.res / 2;
    g.halo_res2 = static_cast<uint32_t>(g.halo_res) * static_cast<uint32_t>(g.halo_res);
    g.halo_words = static_cast<uint32_t>(halo_words(grid.res));
    g.halo_bytes = static_cast<uint32_t>(static_cast<int64_t>(grid.n_grids) * g.halo_words * 4);
    float smax = 0.0f, lmax = 0.0f;
    for (int i = 0; i < 3; ++i) {
        smax = std::fmax(smax, g.s[i]);
        lmax = std::fmax(lmax, std::fabs(g.lo[i]));
    }
    g.contract_delta = static_cast<float>(2.0 * 0x1p-24 * smax * (72.0 + 4.0 * lmax));
    p.near_plane = params.near_plane;
    p.far_plane = params.far_plane;
    p.dt = params.dt;
    p.dt_max = params.dt_max;
    p.cone = params.cone;
    p.max_per_ray = params.max_per_ray;
    const double t_abs = std::fmax(std::fabs(static_cast<double>(params.near_plane)),
                                   std::fabs(static_cast<double>(params.far_plane)));
    p.no_stall = std::isfinite(t_abs) && t_abs * 0x1p-21 < static_cast<double>(params.dt) ? 1 : 0;
}

}  // namespace
