// Fused inference: marching, an in-kernel field and the forward render of
// each ray in one wavefront, without writing the samples out (NerfAcc
// Sec. 2.1 marching with early termination, Eq. 1 rendering; the field is
// the synthetic blob field, the one field the library can evaluate itself).
//
// One wavefront per ray.  The wave marches 64 lattice candidates per
// iteration exactly as the marching kernels do (uniform steps) and appends
// the occupied ones, in t order, to a ring of candidate indices in its LDS
// slice (two chunks of candidates per iteration, so two grid lookups are in
// flight).  Whenever the ring holds 64 of them (or the ray's candidates are
// exhausted) the wave takes them as one chunk: each lane evaluates the field
// at its sample's midpoint and the chunk is rendered with the same
// transmittance routine as the rendering kernels.  The chunks are the ray's
// samples 64 at a time, the same chunks the rendering kernels read from the
// packed arrays, so colour, opacity and depth are bit for bit those of
// marching + field + rendering as three steps.  Marching stops at the
// early-termination cut, which the three-step form cannot do (it marches the
// whole ray before any density is known).  Through the box lookup with the
// halo bits of a skip buffer, a ray is marched by segments as in the count
// pass: 64 segments' halo bits tested at once, then only the candidates of
// the live segments looked up, in t order, so the queued samples are the
// same.
#include <cmath>

#include "blob_field.h"
#include "common.h"
#include "lattice.h"
#include "nacc_synth.h"
#include "transmittance.h"

#pragma clang fp contract(off)

namespace {

using namespace nacc;
using namespace nacc::dev;
using namespace nacc::blob;
using namespace nacc::vr;

constexpr int kFusedWaves = 4;
constexpr int kFusedRays = 64;  // rays per workgroup: lane j of a wave clips its j-th ray
constexpr int kRing = 256;      // candidate indices per wave: < 64 held + 128 appended

// Appends the occupied candidates of one wave iteration (ballot m of the
// candidates k, lanes in t order) to the ring, at most up to max_per_ray
// samples; returns false when the cap ends the ray.
__device__ __forceinline__ bool append_hits(uint64_t m, bool hit, int k, int head, int& queued, int& marched,
                                            const StepK& p, int* __restrict__ ring) {
    int n_new = __popcll(m);
    bool more = true;
    if (p.max_per_ray > 0 && marched + n_new >= p.max_per_ray) {
        n_new = p.max_per_ray - marched;  // the first ones in t order
        hit = hit && bits_below(m) < n_new;
        more = false;
    }
    if (hit) ring[(head + queued + bits_below(m)) & (kRing - 1)] = k;
    queued += n_new;
    marched += n_new;
    return more;
}

// Where the segment walk of a ray stands between chunks.
struct SegWalk {
    int block = 0;      // next block of 64 segments to test
    int slot = 0;       // next entry of the current block's live list
    int n_live = 0;     // entries of that list
    bool last = false;  // the current block is the ray's last
};

template <int LOOKUP, bool PER_SET, bool SEG>
__device__ __forceinline__ void render_ray_fused(int64_t r, const RaySpan& span, const float* __restrict__ table,
                                                 int n_blobs, int n_sets, const int32_t* __restrict__ ray_set,
                                                 const float* __restrict__ rays_o, const float* __restrict__ rays_d,
                                                 const uint32_t* __restrict__ bits,
                                                 const uint32_t* __restrict__ halo, const GridK& g, const StepK& p,
                                                 float eps, int* __restrict__ ring, uint8_t* __restrict__ list,
                                                 float* __restrict__ color, float* __restrict__ opacity,
                                                 float* __restrict__ depth, int32_t* __restrict__ kept) {
    const int lane = lane_id();
    const float* o = span.o;  // loaded lane-parallel with the wave's other rays
    const float* d = span.d;
    int set = 0;
    if (PER_SET) {
        set = uniform<int>(ray_set[r]);
        set = set < 0 ? 0 : (set >= n_sets ? n_sets - 1 : set);
    }
    const float* cc = table + static_cast<int64_t>(n_sets) * n_blobs * kBlobStride;
    const bool contract = cc[12] != 0.0f;
    const float t_near = span.t_near, t_far = span.t_far;
    double carry = 0.0;
    float acc_r = 0.0f, acc_g = 0.0f, acc_b = 0.0f, acc_a = 0.0f, acc_d = 0.0f;
    int head = 0;      // ring slot of the oldest queued candidate
    int queued = 0;    // candidates in the ring
    int marched = 0;   // samples appended so far (max_per_ray)
    int rendered = 0;  // samples taken as chunks so far
    int n_kept = -1;
    bool more = span.valid;
    int k0 = 0;
    SegRay sg{0, 0u};
    if (SEG && span.valid) sg = seg_ray(g, span, p);
    SegWalk sw;
    while (true) {
        // march until a whole chunk is queued or the ray's candidates end,
        // by segments: two iterations of live segments' candidates at a time
        // (both grid words loaded before either is tested)
        while (SEG && sg.log_g != 0 && more && queued < kWave) {
            if (sw.slot >= sw.n_live) {  // the next block of segments
                uint64_t vm;
                const uint64_t lm = sw.last ? 0ull : live_segments(span, halo, g, p, sg, sw.block, vm);
                if (sw.last || vm == 0ull) {
                    more = false;
                    break;
                }
                wave_lds_sync();  // the previous block's list has been read
                if (((lm >> lane) & 1ull) != 0ull) list[bits_below(lm)] = static_cast<uint8_t>(lane);
                wave_lds_sync();
                sw.n_live = static_cast<int>(__popcll(lm));
                sw.slot = 0;
                sw.last = vm != ~0ull;
                ++sw.block;
                continue;
            }
            const int log_g = sg.log_g;
            const int per_iter = kWave >> log_g;
            int k[2];
            float t0[2], t1[2];
            bool alive[2];
            uint64_t ms[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int slot = sw.slot + u * per_iter + (lane >> log_g);
                const bool in = slot < sw.n_live;
                const int seg = in ? static_cast<int>(list[slot]) : 0;
                k[u] = (((sw.block - 1) * kWave + seg) << log_g) + (lane & ((1 << log_g) - 1));
                t0[u] = t_near + static_cast<float>(k[u]) * p.dt;
                t1[u] = t_near + static_cast<float>(k[u] + 1) * p.dt;
                alive[u] = in && t0[u] < t_far;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float tm = (t0[u] + t1[u]) * 0.5f;
                const Probe q =
                    probe<LOOKUP>(g, span.word0, o[0] + d[0] * tm, o[1] + d[1] * tm, o[2] + d[2] * tm);
                const uint32_t w = grid_word(grid_rsrc(bits, g), q.word);  // every lane: the index is clamped into the grid
                ms[u] = ballot(alive[u] & (((w >> q.bit) & 1u) != 0u));
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (!append_hits(ms[u], ((ms[u] >> lane) & 1ull) != 0ull, k[u], head, queued, marched, p, ring)) {
                    more = false;
                    break;
                }
            }
            sw.slot += 2 * per_iter;
        }
        while (!(SEG && sg.log_g != 0) && more && queued < kWave) {
            float t0[2], t1[2];
            bool live[2];
            uint64_t ms[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int k = k0 + u * kWave + lane;
                t0[u] = t_near + static_cast<float>(k) * p.dt;
                live[u] = t0[u] < t_far;
                t1[u] = t_near + static_cast<float>(k + 1) * p.dt;
            }
            if (ballot(live[0]) == 0ull || k0 >= kMaxCandidates) {  // t_k is non-decreasing in k
                more = false;
                break;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float tm = (t0[u] + t1[u]) * 0.5f;
                const Probe q =
                    probe<LOOKUP>(g, span.word0, o[0] + d[0] * tm, o[1] + d[1] * tm, o[2] + d[2] * tm);
                const uint32_t w = grid_word(grid_rsrc(bits, g), q.word);  // every lane: the index is clamped into the grid
                ms[u] = ballot(live[u] & (((w >> q.bit) & 1u) != 0u));
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u == 1 && (ballot(live[1]) == 0ull || k0 + kWave >= kMaxCandidates)) {
                    more = false;
                    break;
                }
                if (!append_hits(ms[u], ((ms[u] >> lane) & 1ull) != 0ull, k0 + u * kWave + lane, head, queued,
                                 marched, p, ring)) {
                    more = false;
                    break;
                }
            }
            k0 += 2 * kWave;
        }
        if (queued == 0) break;
        wave_lds_sync();
        // one chunk: the next min(queued, 64) samples of the ray
        const int n_chunk = min(queued, kWave);
        const bool valid = lane < n_chunk;
        float t0 = 0.0f, t1 = 0.0f, sigma = 0.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
        if (valid) {
            const int k = ring[(head + lane) & (kRing - 1)];
            t0 = t_near + static_cast<float>(k) * p.dt;
            t1 = t_near + static_cast<float>(k + 1) * p.dt;
            float x0 = midpoint_coord(o[0], d[0], t0, t1);
            float x1 = midpoint_coord(o[1], d[1], t0, t1);
            float x2 = midpoint_coord(o[2], d[2], t0, t1);
            to_scene(contract, x0, x1, x2);
            eval_field(table, n_blobs, set, x0, x1, x2, sigma);
            eval_rgb(cc, x0, x1, x2, cr, cg, cb);
        }
        wave_lds_sync();
        head = (head + n_chunk) & (kRing - 1);
        queued -= n_chunk;
        const Trans t = transmittance_of(sigma * (t1 - t0), carry);
        const int keep_n = chunk_keep(valid, t.t_in, eps);
        const bool keep = valid && lane < keep_n;
        const float w = keep ? t.t_in * alpha_of(t.tau) : 0.0f;
        acc_r = __builtin_fmaf(w, cr, acc_r);
        acc_g = __builtin_fmaf(w, cg, acc_g);
        acc_b = __builtin_fmaf(w, cb, acc_b);
        acc_a += w;
        acc_d = __builtin_fmaf(w, (t0 + t1) * 0.5f, acc_d);
        carry += static_cast<double>(read_lane(t.incl, 63));
        if (keep_n < kWave) {
            n_kept = rendered + keep_n;
            break;
        }
        rendered += n_chunk;
    }
    wave_sum4(acc_r, acc_g, acc_b, acc_a);
    acc_d = wave_sum1(acc_d);
    if (lane == 0) {
        color[3 * r] = acc_r;
        color[3 * r + 1] = acc_g;
        color[3 * r + 2] = acc_b;
        opacity[r] = acc_a;
        depth[r] = acc_d;
        if (kept != nullptr) kept[r] = n_kept >= 0 ? n_kept : rendered;
    }
}

// clocks (nullable): the device wall clock when the workgroup started and
// when its last wave finished, per workgroup of kFusedRays rays.
template <int LOOKUP, bool PER_SET, bool SEG>
__global__ __launch_bounds__(kFusedWaves * kWave) void fused_render_kernel(
    const float* __restrict__ table, int n_blobs, int n_sets, const int32_t* __restrict__ ray_set,
    const float* __restrict__ rays_o, const float* __restrict__ rays_d, const int32_t* __restrict__ grid_id,
    int64_t n_rays, const uint32_t* __restrict__ bits, const uint32_t* __restrict__ halo, GridK g, ClipK c,
    StepK p, float eps, float* __restrict__ color, float* __restrict__ opacity, float* __restrict__ depth,
    int32_t* __restrict__ kept, uint64_t* __restrict__ clocks) {
    __shared__ int rings[kFusedWaves][kRing];
    __shared__ uint8_t lists[kFusedWaves][SEG ? kWave : 1];
    const uint64_t t_start = clocks != nullptr ? wall_clock64() : 0ull;
    const int wave = uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kFusedRays;
    // this wave's rays are first + wave + j kFusedWaves; lane j clips ray j
    const int64_t mine = first + wave + static_cast<int64_t>(lane_id()) * kFusedWaves;
    RaySpan spans{};
    if (lane_id() < kFusedRays / kFusedWaves && mine < n_rays) {
        spans = ray_span<LOOKUP>(mine, rays_o, rays_d, grid_id, g, c, p);
    }
    for (int i = wave; i < kFusedRays; i += kFusedWaves) {
        const int64_t r = first + i;
        if (r >= n_rays) break;
        const RaySpan span = read_span(spans, i / kFusedWaves);
        render_ray_fused<LOOKUP, PER_SET, SEG>(r, span, table, n_blobs, n_sets, ray_set, rays_o, rays_d, bits, halo,
                                               g, p, eps, rings[wave], lists[wave], color, opacity, depth, kept);
    }
    if (clocks != nullptr) {
        __syncthreads();
        if (threadIdx.x == 0) {
            clocks[2 * blockIdx.x] = t_start;
            clocks[2 * blockIdx.x + 1] = wall_clock64();
        }
    }
}

template <int LOOKUP, bool SEG>
void launch_fused_seg(bool per_set, unsigned nb, hipStream_t s, const float* table, int n_blobs, int n_sets,
                      const int32_t* ray_set, const float* o, const float* d, const int32_t* gid, int64_t n,
                      const uint32_t* bits, const uint32_t* halo, const GridK& g, const ClipK& c, const StepK& p,
                      float eps, float* color, float* opacity, float* depth, int32_t* kept, uint64_t* clocks) {
    if (per_set) {
        hipLaunchKernelGGL((fused_render_kernel<LOOKUP, true, SEG>), dim3(nb), dim3(kFusedWaves * kWave), 0, s,
                           table, n_blobs, n_sets, ray_set, o, d, gid, n, bits, halo, g, c, p, eps, color, opacity,
                           depth, kept, clocks);
    } else {
        hipLaunchKernelGGL((fused_render_kernel<LOOKUP, false, SEG>), dim3(nb), dim3(kFusedWaves * kWave), 0, s,
                           table, n_blobs, n_sets, ray_set, o, d, gid, n, bits, halo, g, c, p, eps, color, opacity,
                           depth, kept, clocks);
    }
}

}  // namespace

extern "C" {

int64_t nacc_wall_clock_khz(int32_t device) {
    clear_error();
    int khz = 0;
    const hipError_t e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device);
    if (e != hipSuccess) return set_error(NACC_EHIP, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
    return khz;
}

int nacc_synth_render_fused(const void* table, int32_t n_blobs, int32_t n_sets, const int32_t* ray_set,
                            const float* rays_o, const float* rays_d, const int32_t* grid_id, int64_t n_rays,
                            const uint32_t* grid_bits, const uint8_t* grid_skip, const nacc_grid_desc* grid,
                            const nacc_march_params* params, float early_stop_eps, float* color, float* opacity,
                            float* depth, int32_t* kept, uint64_t* clocks, void* stream) {
    clear_error();
    int st = validate(rays_o, rays_d, n_rays, grid_bits, grid, params);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(params->cone == 0.0f, NACC_ENOTSUP, "the fused kernel marches uniform steps only (cone = %g)",
                 params->cone);
    NACC_REQUIRE(table != nullptr && n_blobs >= 1 && n_sets >= 1, NACC_EINVAL,
                 "table must be non-NULL with n_blobs, n_sets >= 1");
    NACC_REQUIRE(std::isfinite(early_stop_eps) && early_stop_eps >= 0.0f, NACC_EINVAL,
                 "early_stop_eps = %g must be finite and >= 0", early_stop_eps);
    NACC_REQUIRE(n_rays == 0 || (color != nullptr && opacity != nullptr && depth != nullptr), NACC_EINVAL,
                 "color, opacity and depth must be non-NULL");
    if (n_rays == 0) return NACC_OK;
    GridK g;
    ClipK c;
    StepK p;
    make_constants(*grid, *params, g, c, p);
    const unsigned nb = static_cast<unsigned>((n_rays + kFusedRays - 1) / kFusedRays);
    hipStream_t s = as_stream(stream);
    const float* tb = static_cast<const float*>(table);
    const bool per_set = ray_set != nullptr;
    // the halo bits of the skip buffer (box lookup, res a multiple of 4)
    const uint32_t* halo = grid_skip != nullptr && grid->res % 4 == 0 && grid->lookup == NACC_LOOKUP_AABB
                               ? reinterpret_cast<const uint32_t*>(grid_skip + halo_offset(g.res, g.n_grids))
                               : nullptr;
    switch (grid->lookup) {
        case NACC_LOOKUP_AABB:
            if (halo != nullptr) {
                launch_fused_seg<NACC_LOOKUP_AABB, true>(per_set, nb, s, tb, n_blobs, n_sets, ray_set, rays_o,
                                                         rays_d, grid_id, n_rays, grid_bits, halo, g, c, p,
                                                         early_stop_eps, color, opacity, depth, kept, clocks);
            } else {
                launch_fused_seg<NACC_LOOKUP_AABB, false>(per_set, nb, s, tb, n_blobs, n_sets, ray_set, rays_o,
                                                          rays_d, grid_id, n_rays, grid_bits, nullptr, g, c, p,
                                                          early_stop_eps, color, opacity, depth, kept, clocks);
            }
            break;
        case NACC_LOOKUP_CASCADE:
            launch_fused_seg<NACC_LOOKUP_CASCADE, false>(per_set, nb, s, tb, n_blobs, n_sets, ray_set, rays_o, rays_d,
                                                         grid_id, n_rays, grid_bits, nullptr, g, c, p,
                                                         early_stop_eps, color, opacity, depth, kept, clocks);
            break;
        default:
            launch_fused_seg<NACC_LOOKUP_CONTRACT, false>(per_set, nb, s, tb, n_blobs, n_sets, ray_set, rays_o,
                                                          rays_d, grid_id, n_rays, grid_bits, nullptr, g, c, p,
                                                          early_stop_eps, color, opacity, depth, kept, clocks);
            break;
    }
    return check_launch("fused render");
}

}  // extern "C"
