// Packed differentiable volume rendering on gfx950 (NerfAcc, Eq. 1 and
// Sec. 2.2 "Differentiable Rendering"; early termination from Sec. 2.1).
//
// One wavefront per ray.  The ray's samples are read in chunks of 64, one per
// lane, with coalesced loads of the packed arrays through buffer resources
// that span the ray's samples (SampleSpan below).  Inside a chunk the
// exclusive transmittance comes from a DPP prefix sum of tau = sigma * delta
// over the 64 lanes; the running prefix across chunks is carried in FP64.
// The same routine (chunk_transmittance) produces T in the forward, the
// backward and the fused kernels, so all three place the early-termination
// cut on the same sample.
//
// Backward: g_sigma_i = delta_i (T_{i+1} v_i - S_i), S_i = sum_{k>i} w_k v_k.
// S_i is a true suffix sum, accumulated from the end of the ray (chunks in
// reverse, a DPP suffix scan inside each chunk), so it stays accurate
// relative to its own terms however small T gets; a
// total-minus-prefix form would lose every digit once T falls below the
// rounding of the total.  The first chunks of each ray stay in registers
// between the forward and the backward pass (no second read, no second
// transmittance evaluation for them).
#include <cmath>
#include <mutex>

#include "common.h"
#include "scan.h"
#include "transmittance.h"

#pragma clang fp contract(off)

namespace {

using namespace nacc;
using namespace nacc::dev;
using namespace nacc::vr;

constexpr int kRenderThreads = 256;  // 4 waves
constexpr int kRaysPerRenderBlock = kRenderThreads / kWave;

struct Sample {
    float t0, t1, sigma, r, g, b;
};

// A ray's samples are consecutive in every packed array, so a span of them
// is read and written through buffer resources: a resource covers `count`
// samples from `first`, sample i of the span sits at the byte offset 4 i
// (12 i for colours), so each lane's offset is a constant of the kernel and
// no address is formed per access, and the hardware range check reads 0
// for every lane past the span and drops its stores.  Spans cover at most
// 64 K samples (one resource per chunk past the first K), so every offset
// stays far inside 32 bits however long the ray.  The last word of a
// resource selects 32-bit untyped data.  Only 32-bit buffer accesses are
// used (a colour is three of them at neighbouring offsets): this compiler's
// 64- and 96-bit buffer-load builtins can come out as a 32-bit load whose
// other words are lost.
constexpr int kRawBufferWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const float* base, int64_t first, int count, int width) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base) + first * width, 0, count * width * 4,
                                             kRawBufferWord3);
}

struct SampleSpan {
    __amdgpu_buffer_rsrc_t ts, te, sig, rgb;
};

__device__ __forceinline__ SampleSpan sample_span(const float* ts, const float* te, const float* sig,
                                                  const float* rgb, int64_t first, int count) {
    return SampleSpan{span_rsrc(ts, first, count, 1), span_rsrc(te, first, count, 1),
                      span_rsrc(sig, first, count, 1), span_rsrc(rgb, first, count, 3)};
}

// Byte offsets of the calling lane's sample in a span: 4 i in the 32-bit
// arrays, 12 i in the colours.  Chunk c of a span adds the constants 256 c
// and 768 c, which the compiler places in the instructions' immediate
// offsets; the lane's part is made opaque (an empty asm statement that
// claims to change it, no instruction) so that the sums are not hoisted out
// of the ray loop into registers of their own.
struct LaneOffset {
    uint32_t o4, o12;
};

__device__ __forceinline__ LaneOffset lane_offset() {
    uint32_t o4 = static_cast<uint32_t>(lane_id()) * 4u, o12 = static_cast<uint32_t>(lane_id()) * 12u;
    asm volatile("" : "+v"(o4), "+v"(o12));
    return LaneOffset{o4, o12};
}

__device__ __forceinline__ LaneOffset chunk_offset(const LaneOffset& l, int c) {
    return LaneOffset{l.o4 + static_cast<uint32_t>(c) * 256u, l.o12 + static_cast<uint32_t>(c) * 768u};
}

// The sample at offset o of the span (zeros past its end).
__device__ __forceinline__ Sample load_span(const SampleSpan& sp, const LaneOffset& o) {
    Sample x;
    x.t0 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sp.ts, o.o4, 0, 0));
    x.t1 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sp.te, o.o4, 0, 0));
    x.sigma = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sp.sig, o.o4, 0, 0));
    x.r = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sp.rgb, o.o12, 0, 0));
    x.g = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sp.rgb, o.o12 + 4u, 0, 0));
    x.b = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sp.rgb, o.o12 + 8u, 0, 0));
    return x;
}

// The first samples of a ray (the first chunk of the next ray, or the K
// register-cached chunks), at most `cap`.
__device__ __forceinline__ SampleSpan head_span(const float* ts, const float* te, const float* sig, const float* rgb,
                                                int64_t start, int n, int cap) {
    return sample_span(ts, te, sig, rgb, start, min(n, cap));
}

// Where a span's gradients go.
struct GradSpan {
    __amdgpu_buffer_rsrc_t sig, rgb;
};

__device__ __forceinline__ GradSpan grad_span(float* g_sigmas, float* g_rgbs, int64_t first, int count) {
    return GradSpan{span_rsrc(g_sigmas, first, count, 1), span_rsrc(g_rgbs, first, count, 3)};
}

__device__ __forceinline__ void store_grads(const GradSpan& d, const LaneOffset& o, float gs, float gr, float gg,
                                            float gb) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, gs), d.sig, o.o4, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, gr), d.rgb, o.o12, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, gg), d.rgb, o.o12 + 4u, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, gb), d.rgb, o.o12 + 8u, 0, 0);
}

__device__ __forceinline__ Trans chunk_transmittance(const Sample& x, double carry) {
    return transmittance_of(x.sigma * (x.t1 - x.t0), carry);
}

template <bool WEIGHTS>
__global__ __launch_bounds__(kRenderThreads) void render_fwd_kernel(
    const int32_t* __restrict__ packed_info, int64_t n_rays, int64_t n_samples, const float* __restrict__ ts,
    const float* __restrict__ te, const float* __restrict__ sig, const float* __restrict__ rgb, float eps,
    float* __restrict__ color, float* __restrict__ opacity, float* __restrict__ depth,
    float* __restrict__ weights, int32_t* __restrict__ kept) {
    const int lane = lane_id();
    const int64_t r = xcd_grouped<16>(blockIdx.x, gridDim.x) * kRaysPerRenderBlock +
                      uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    if (r >= n_rays) return;
    int64_t start;
    int n;
    ray_range(packed_info, r, n_samples, start, n);
    double carry = 0.0;
    float acc_r = 0.0f, acc_g = 0.0f, acc_b = 0.0f, acc_a = 0.0f, acc_d = 0.0f;
    int c = 0;
    int n_kept = n;
    for (; c < n; c += kWave) {
        const int i = c + lane;
        const bool valid = i < n;
        const int64_t s = start + i;
        const Sample x = load_span(sample_span(ts, te, sig, rgb, start + c, min(n - c, kWave)), lane_offset());
        const Trans t = chunk_transmittance(x, carry);
        const int keep_n = chunk_keep_n(n - c, t.t_in, eps);
        const bool keep = lane < min(keep_n, n - c);
        const float w = keep ? t.t_in * alpha_of(t.tau) : 0.0f;
        acc_r = __builtin_fmaf(w, x.r, acc_r);
        acc_g = __builtin_fmaf(w, x.g, acc_g);
        acc_b = __builtin_fmaf(w, x.b, acc_b);
        acc_a += w;
        acc_d = __builtin_fmaf(w, (x.t0 + x.t1) * 0.5f, acc_d);
        if (WEIGHTS && valid) weights[s] = w;
        carry += static_cast<double>(read_lane(t.incl, 63));
        if (keep_n < kWave) {
            n_kept = c + keep_n;
            c += kWave;
            break;
        }
    }
    if (WEIGHTS) {
        for (; c < n; c += kWave) {
            if (c + lane < n) weights[start + c + lane] = 0.0f;
        }
    }
    wave_sum4(acc_r, acc_g, acc_b, acc_a);
    acc_d = wave_sum1(acc_d);
    if (lane == 0) {
        color[3 * r] = acc_r;
        color[3 * r + 1] = acc_g;
        color[3 * r + 2] = acc_b;
        opacity[r] = acc_a;
        depth[r] = acc_d;
        if (kept != nullptr) kept[r] = n_kept;
    }
}

// Upstream gradient of one ray: v_i = gc . rgb_i + ga + gd * m_i.
struct RayGrad {
    float gr, gg, gb, ga, gd;
};

// What the backward needs of a sample: its interval length, midpoint and
// colour (its density only enters through w and T, formed in the forward).
struct GradInput {
    float delta, m, r, g, b;
};

__device__ __forceinline__ GradInput grad_input(const Sample& x) {
    return GradInput{x.t1 - x.t0, (x.t0 + x.t1) * 0.5f, x.r, x.g, x.b};
}

// v = gc . rgb + (ga + gd m), with fused multiply-adds in a fixed order
// (the attribute kernels form their dot product the same way).  NO_AD:
// ga = gd = 0 is known (the loss reads the colour only), and ga + gd m is
// then +0 for every finite m, so m is not needed and the sum is the general
// one bit for bit.
template <bool NO_AD>
__device__ __forceinline__ float vdot(const RayGrad& q, const GradInput& x) {
    const float c = __builtin_fmaf(q.gb, x.b, __builtin_fmaf(q.gg, x.g, q.gr * x.r));
    return NO_AD ? c + 0.0f : c + __builtin_fmaf(q.gd, x.m, q.ga);
}

// Gradients of one chunk (lane i = sample c + i) given w_i and T_{i+1};
// `above` is sum_k w_k v_k over the samples after the chunk.  Returns the
// same sum over the samples from the chunk on.  S_i = above + (suffix of
// w v inside the chunk past i): every partial sum is formed from the end of
// the ray, so it is accurate relative to the terms it adds however small T
// gets.  Lanes at or past the cut get zeros.
template <bool NO_AD>
__device__ __forceinline__ float chunk_grads(const RayGrad& q, const GradInput& x, float w, float t_next, bool keep,
                                             const GradSpan& dst, const LaneOffset& o, float above) {
    const float v = vdot<NO_AD>(q, x);
    const float wv = keep ? w * v : 0.0f;
    const float incl = wave_inclusive_suffix(wv);
    const float suffix = above + shift_down_one(incl);
    const float gs = x.delta * __builtin_fmaf(t_next, v, -suffix);
    store_grads(dst, o, keep ? gs : 0.0f, keep ? w * q.gr : 0.0f, keep ? w * q.gg : 0.0f, keep ? w * q.gb : 0.0f);
    return above + read_lane(incl, 0);
}

// Forward pass of one ray shared by the backward and the fused kernels.
// The first K chunks are loaded up front; what the backward needs of them
// (GradInput, w_i and T_{i+1}) stays in registers; later chunks are
// streamed.  Produces the cut, the FP64 tau prefix at the start of the
// chunk holding the last kept sample, and (ACCUM) the rendered colour /
// opacity / depth.
template <int K>
struct RayCache {
    GradInput x[K];
    float w[K];
    float t_next[K];
    double carries;  // lane j: FP64 tau prefix at the start of chunk j (j < 64)
};

// The first S chunks past the register-cached ones can be kept in LDS: per
// chunk and lane what the backward reads of a sample (interval length,
// colour, w_i and T_{i+1}, 6 floats; the midpoint's term is +0 in the loss
// kernels), so that their backward pass neither reloads them from memory nor
// forms T again.  Each lane reads back only its own slots, in the wave's own
// order of LDS accesses.
constexpr int kStashFloats = 6;
constexpr int kStashChunks = 3;  // 18 KiB of LDS per workgroup of 4 waves: 8 workgroups per CU

template <int K, bool ACCUM, bool PRELOADED = false, int S = 0>
__device__ __forceinline__ void ray_forward(int64_t start, int n, const float* __restrict__ ts,
                                            const float* __restrict__ te, const float* __restrict__ sig,
                                            const float* __restrict__ rgb, float eps, RayCache<K>& cache, int& kept,
                                            double& prefix_hi, float acc[3], float& acc_a, float& acc_d,
                                            const Sample& chunk0 = Sample{}, float* stash = nullptr) {
    const int lane = lane_id();
    const LaneOffset lo = lane_offset();
    // chunks past the ray's end are neither loaded nor read
    Sample x[K];
    const SampleSpan head = head_span(ts, te, sig, rgb, start, n, K * kWave);
#pragma unroll
    for (int c = 0; c < K; ++c) {
        if (c * kWave >= n) continue;
        if (PRELOADED && c == 0) {
            x[0] = chunk0;  // loaded while the previous ray was finished
        } else {
            x[c] = load_span(head, chunk_offset(lo, c));
        }
    }
    double carry = 0.0, carry_prev = 0.0;
    kept = n;
    prefix_hi = 0.0;
    cache.carries = 0.0;
    bool stopped = false;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        cache.w[c] = 0.0f;
        cache.t_next[c] = 0.0f;
        if (c * kWave >= n) continue;
        cache.x[c] = grad_input(x[c]);
        if (stopped) continue;
        if (lane == c) cache.carries = carry;
        const int n_valid = n - c * kWave;
        const Trans t = chunk_transmittance(x[c], carry);
        const int keep_n = chunk_keep_n(n_valid, t.t_in, eps);
        const bool keep = lane < min(keep_n, n_valid);
        const float w = keep ? t.t_in * alpha_of(t.tau) : 0.0f;
        cache.w[c] = w;
        cache.t_next[c] = t.t_next;
        if (ACCUM) {
            acc[0] = __builtin_fmaf(w, x[c].r, acc[0]);
            acc[1] = __builtin_fmaf(w, x[c].g, acc[1]);
            acc[2] = __builtin_fmaf(w, x[c].b, acc[2]);
            acc_a += w;
            acc_d = __builtin_fmaf(w, (x[c].t0 + x[c].t1) * 0.5f, acc_d);
        }
        if (keep_n < kWave) {
            kept = c * kWave + keep_n;
            prefix_hi = keep_n > 0 ? carry : carry_prev;
            stopped = true;
        } else {
            carry_prev = carry;
            carry += static_cast<double>(read_lane(t.incl, 63));
            prefix_hi = carry_prev;
        }
    }
    for (int c = K * kWave; !stopped && c < n; c += kWave) {
        if (lane == c / kWave) cache.carries = carry;
        const Sample x = load_span(sample_span(ts, te, sig, rgb, start + c, min(n - c, kWave)), lo);
        const Trans t = chunk_transmittance(x, carry);
        const int keep_n = chunk_keep_n(n - c, t.t_in, eps);
        if (ACCUM || S > 0) {
            const bool keep = lane < min(keep_n, n - c);
            const float w = keep ? t.t_in * alpha_of(t.tau) : 0.0f;
            if (ACCUM) {
                acc[0] = __builtin_fmaf(w, x.r, acc[0]);
                acc[1] = __builtin_fmaf(w, x.g, acc[1]);
                acc[2] = __builtin_fmaf(w, x.b, acc[2]);
                acc_a += w;
                acc_d = __builtin_fmaf(w, (x.t0 + x.t1) * 0.5f, acc_d);
            }
            const int slot = c / kWave - K;
            if (S > 0 && slot < S) {
                float* st = stash + slot * kStashFloats * kWave + lane;
                st[0] = x.t1 - x.t0;
                st[kWave] = x.r;
                st[2 * kWave] = x.g;
                st[3 * kWave] = x.b;
                st[4 * kWave] = w;
                st[5 * kWave] = t.t_next;
            }
        }
        if (keep_n < kWave) {
            kept = c + keep_n;
            prefix_hi = keep_n > 0 ? carry : carry_prev;
            stopped = true;
        } else {
            carry_prev = carry;
            carry += static_cast<double>(read_lane(t.incl, 63));
            prefix_hi = carry_prev;
        }
    }
}

// Backward pass of one ray: chunks from the last kept one down to the first.
// Streamed chunks rebuild T from the FP64 prefix at their end (walked down
// from prefix_hi); cached chunks reuse w and T_{i+1} from the forward pass.
template <int K, bool NO_AD, int S = 0>
__device__ __forceinline__ void ray_backward(int64_t start, int n, int kept, double prefix_hi,
                                             const float* __restrict__ ts, const float* __restrict__ te,
                                             const float* __restrict__ sig, const float* __restrict__ rgb,
                                             const RayCache<K>& cache, const RayGrad& q, float* __restrict__ g_sigmas,
                                             float* __restrict__ g_rgbs, const float* stash = nullptr) {
    static_assert(S == 0 || NO_AD, "the stash leaves out the midpoint");
    const int lane = lane_id();
    const LaneOffset lo = lane_offset();
    const int cached_end = K * kWave;
    const int c_hi = kept > 0 ? ((kept - 1) / kWave) * kWave : -kWave;
    float above = 0.0f;
    double p_end = 0.0;  // tau prefix at the end of the chunk being processed
    for (int c = c_hi; c >= cached_end; c -= kWave) {
        const int i = c + lane;
        const bool keep = i < kept;
        const int slot = c / kWave - K;
        if (S > 0 && slot < S) {  // the forward's values, from LDS (chunk < 64: p_end is not needed below)
            const float* st = stash + slot * kStashFloats * kWave + lane;
            const GradInput gx{st[0], 0.0f, st[kWave], st[2 * kWave], st[3 * kWave]};
            above = chunk_grads<NO_AD>(q, gx, st[4 * kWave], st[5 * kWave], keep,
                                       grad_span(g_sigmas, g_rgbs, start + c, min(n - c, kWave)), lo, above);
            continue;
        }
        // samples past the cut read as zeros, as in the forward pass's sums
        const Sample x = load_span(sample_span(ts, te, sig, rgb, start + c, min(kept - c, kWave)), lo);
        const float tau = x.sigma * (x.t1 - x.t0);
        const float chunk_tau = wave_sum(tau);
        // the forward pass's own carry (so T is bit for bit the forward T)
        // for the first 64 chunks, else the prefix walked down from the end
        const int chunk = c / kWave;
        const double p_start = chunk < kWave ? read_lane(cache.carries, chunk)
                                             : (c == c_hi ? prefix_hi : p_end - static_cast<double>(chunk_tau));
        const Trans t = chunk_transmittance(x, p_start);
        const float w = keep ? t.t_in * alpha_of(t.tau) : 0.0f;
        const float t_next = t.t_next;
        above = chunk_grads<NO_AD>(q, grad_input(x), w, t_next, keep,
                                   grad_span(g_sigmas, g_rgbs, start + c, min(n - c, kWave)), lo, above);
        p_end = p_start;
    }
    const GradSpan head = grad_span(g_sigmas, g_rgbs, start, min(n, cached_end));
#pragma unroll
    for (int c = K - 1; c >= 0; --c) {
        if (c * kWave >= n) continue;
        const int i = c * kWave + lane;
        above = chunk_grads<NO_AD>(q, cache.x[c], cache.w[c], cache.t_next[c], i < kept, head, chunk_offset(lo, c),
                                   above);
    }
    // streamed chunks past the cut: zeros, no loads (stored last, so no wait
    // on memory above waits for them)
    for (int c = max(c_hi + kWave, cached_end); c < n; c += kWave) {
        store_grads(grad_span(g_sigmas, g_rgbs, start + c, min(n - c, kWave)), lo, 0.0f, 0.0f, 0.0f, 0.0f);
    }
}

template <int K>
__global__ __launch_bounds__(kRenderThreads) void render_bwd_kernel(
    const int32_t* __restrict__ packed_info, int64_t n_rays, int64_t n_samples, const float* __restrict__ ts,
    const float* __restrict__ te, const float* __restrict__ sig, const float* __restrict__ rgb, float eps,
    const float* __restrict__ g_color, const float* __restrict__ g_opacity, const float* __restrict__ g_depth,
    float* __restrict__ g_sigmas, float* __restrict__ g_rgbs) {
    const int64_t r = xcd_grouped<16>(blockIdx.x, gridDim.x) * kRaysPerRenderBlock +
                      uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    if (r >= n_rays) return;
    int64_t start;
    int n;
    ray_range(packed_info, r, n_samples, start, n);
    if (n == 0) return;
    RayGrad q;
    q.gr = uniform<float>(g_color[3 * r]);
    q.gg = uniform<float>(g_color[3 * r + 1]);
    q.gb = uniform<float>(g_color[3 * r + 2]);
    q.ga = g_opacity != nullptr ? uniform<float>(g_opacity[r]) : 0.0f;
    q.gd = g_depth != nullptr ? uniform<float>(g_depth[r]) : 0.0f;
    RayCache<K> cache;
    int kept;
    double prefix_hi;
    float acc[3] = {0.0f, 0.0f, 0.0f};
    float acc_a = 0.0f, acc_d = 0.0f;
    ray_forward<K, false>(start, n, ts, te, sig, rgb, eps, cache, kept, prefix_hi, acc, acc_a, acc_d);
    ray_backward<K, false>(start, n, kept, prefix_hi, ts, te, sig, rgb, cache, q, g_sigmas, g_rgbs);
}

// Fused forward + MSE + backward.  The forward gives the colour, the loss
// gradient g_C = 2 (C - target) / (3 n_rays) follows, then the backward runs
// on the cached chunks.  Rays are walked grid-stride (one ray per wave at
// the largest grid); each wave leaves one partial sum of the loss.  8 waves
// per SIMD (at most 64 VGPRs) wherever that needs no spill (7 with K = 4
// and the prefetch); with the buffer addressing 8 waves run no faster than
// 7, and no slower.
template <int K, bool PREFETCH>
__global__ __launch_bounds__(kRenderThreads)
__attribute__((amdgpu_waves_per_eu(K == 4 && PREFETCH ? 7 : 8))) void render_mse_kernel(
    const int32_t* __restrict__ packed_info, int64_t n_rays, int64_t n_samples, const float* __restrict__ ts,
    const float* __restrict__ te, const float* __restrict__ sig, const float* __restrict__ rgb, float eps,
    const float* __restrict__ target, float inv_count2, float* __restrict__ color, float* __restrict__ opacity,
    float* __restrict__ depth, float* __restrict__ g_sigmas, float* __restrict__ g_rgbs,
    double* __restrict__ loss_partial) {
    const int lane = lane_id();
    const int wave = uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    __shared__ float stash_all[kRaysPerRenderBlock * kStashChunks * kStashFloats * kWave];
    float* stash = stash_all + wave * kStashChunks * kStashFloats * kWave;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kRaysPerRenderBlock;
    double wave_total = 0.0;
    // PREFETCH: the next ray's range is read when a ray starts and its first
    // chunk is loaded before the ray's backward pass, so those loads are in
    // flight while the backward runs
    int64_t r = xcd_grouped<16>(blockIdx.x, gridDim.x) * kRaysPerRenderBlock + wave;
    int64_t start = 0;
    int n = 0;
    Sample pre{};
    if (PREFETCH && r < n_rays) {
        ray_range(packed_info, r, n_samples, start, n);
        pre = load_span(head_span(ts, te, sig, rgb, start, n, kWave), lane_offset());
    }
    for (; r < n_rays; r += stride) {
        if (!PREFETCH) ray_range(packed_info, r, n_samples, start, n);
        // the target is read with the ray's first samples, not after its
        // forward pass, so its latency overlaps theirs
        const float tr = target[3 * r], tg = target[3 * r + 1], tb = target[3 * r + 2];
        const int64_t r_next = r + stride;
        int64_t start_next = 0;
        int n_next = 0;
        if (PREFETCH && r_next < n_rays) ray_range(packed_info, r_next, n_samples, start_next, n_next);
        RayCache<K> cache;
        int kept;
        double prefix_hi;
        float acc[3] = {0.0f, 0.0f, 0.0f};
        float acc_a = 0.0f, acc_d = 0.0f;
        ray_forward<K, true, PREFETCH, kStashChunks>(start, n, ts, te, sig, rgb, eps, cache, kept, prefix_hi, acc,
                                                     acc_a, acc_d, pre, stash);
        wave_sum4(acc[0], acc[1], acc[2], acc_a);
        acc_d = wave_sum1(acc_d);
        const float cr = acc[0], cg = acc[1], cb = acc[2];
        const float er = cr - tr, eg = cg - tg, eb = cb - tb;
        RayGrad q;
        q.gr = uniform<float>(er * inv_count2);
        q.gg = uniform<float>(eg * inv_count2);
        q.gb = uniform<float>(eb * inv_count2);
        q.ga = 0.0f;
        q.gd = 0.0f;
        wave_total += static_cast<double>(er) * er + static_cast<double>(eg) * eg + static_cast<double>(eb) * eb;
        if (PREFETCH) pre = load_span(head_span(ts, te, sig, rgb, start_next, n_next, kWave), lane_offset());
        if (n > 0) {
            ray_backward<K, true, kStashChunks>(start, n, kept, prefix_hi, ts, te, sig, rgb, cache, q, g_sigmas,
                                                g_rgbs, stash);
        }
        // stored after the backward: a store before it would make the
        // backward's first wait on memory also wait for the store
        if (lane == 0) {
            color[3 * r] = cr;
            color[3 * r + 1] = cg;
            color[3 * r + 2] = cb;
            opacity[r] = acc_a;
            depth[r] = acc_d;
        }
        if (PREFETCH) {
            start = start_next;
            n = n_next;
        }
    }
    // one partial per wave: no workgroup barrier, which would make every
    // wave wait for its gradient stores to complete before it could exit
    if (lane == 0) loss_partial[static_cast<int64_t>(blockIdx.x) * kRaysPerRenderBlock + wave] = wave_total;
}

// The fused loss kernel for launches with fewer waves than rays (each wave
// takes several rays): rays without samples are finished lane-parallel.
// Occupancy as in render_mse_kernel: 8 waves per SIMD, 7 or 6 where more
// registers are live (K = 3 with the prefetch, K = 4).
template <int K, bool PREFETCH>
__global__ __launch_bounds__(kRenderThreads)
__attribute__((amdgpu_waves_per_eu(K + PREFETCH >= 5 ? 6 : (K + PREFETCH >= 4 ? 7 : 8)))) void render_mse_grouped_kernel(
    const int32_t* __restrict__ packed_info, int64_t n_rays, int64_t n_samples, const float* __restrict__ ts,
    const float* __restrict__ te, const float* __restrict__ sig, const float* __restrict__ rgb, float eps,
    const float* __restrict__ target, float inv_count2, float* __restrict__ color, float* __restrict__ opacity,
    float* __restrict__ depth, float* __restrict__ g_sigmas, float* __restrict__ g_rgbs,
    double* __restrict__ loss_partial) {
    const int lane = lane_id();
    const int wave = uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    __shared__ float stash_all[kRaysPerRenderBlock * kStashChunks * kStashFloats * kWave];
    float* stash = stash_all + wave * kStashChunks * kStashFloats * kWave;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kRaysPerRenderBlock;
    const int64_t r0 = xcd_grouped<16>(blockIdx.x, gridDim.x) * kRaysPerRenderBlock + wave;
    double wave_total = 0.0;  // squared errors of the wave's rays
    // The wave's rays are r0 + i stride, taken 64 at a time: lane i reads the
    // range of ray i, so a ray without samples is finished by its lane alone
    // (colour 0, the squared error of its target) and the rays with samples
    // are rendered one after the other by the whole wave.
    for (int64_t rb = r0; rb < n_rays; rb += stride * kWave) {
        const int64_t my_r = rb + static_cast<int64_t>(lane) * stride;
        const bool mine = my_r < n_rays;
        int my_n = 0, my_start = 0;
        if (mine) {
            const int s0 = packed_info[2 * my_r], c0 = packed_info[2 * my_r + 1];
            const bool ok = s0 >= 0 && c0 >= 0 && static_cast<int64_t>(s0) + c0 <= n_samples;
            my_n = ok ? c0 : 0;
            my_start = ok ? s0 : 0;
        }
        if (ballot(mine && my_n == 0) != 0ull) {
            double sq = 0.0;
            if (mine && my_n == 0) {
                // the rendered colour is the wave sum of zeros, +0
                const float er = 0.0f - target[3 * my_r], eg = 0.0f - target[3 * my_r + 1],
                            eb = 0.0f - target[3 * my_r + 2];
                sq = static_cast<double>(er) * er + static_cast<double>(eg) * eg + static_cast<double>(eb) * eb;
                color[3 * my_r] = 0.0f;
                color[3 * my_r + 1] = 0.0f;
                color[3 * my_r + 2] = 0.0f;
                opacity[my_r] = 0.0f;
                depth[my_r] = 0.0f;
            }
            wave_total += wave_sum(sq);
        }
        uint64_t todo = ballot(mine && my_n > 0);
        // PREFETCH: a ray's first chunk is loaded during the previous ray's
        // backward pass
        Sample pre{};
        // (a ray's range is taken from its lane's registers, not loaded
        // again: no memory round trip before its samples are requested)
        if (PREFETCH && todo != 0ull) {
            const int j = static_cast<int>(__builtin_ctzll(todo));
            pre = load_span(head_span(ts, te, sig, rgb, read_lane(my_start, j), read_lane(my_n, j), kWave),
                            lane_offset());
        }
        while (todo != 0ull) {
            const int i = static_cast<int>(__builtin_ctzll(todo));
            todo &= todo - 1ull;
            const int64_t r = rb + static_cast<int64_t>(i) * stride;
            const int64_t start = read_lane(my_start, i);
            const int n = read_lane(my_n, i);
            // the target's address is wave-uniform: scalar loads
            const float tr = target[3 * r], tg = target[3 * r + 1], tb = target[3 * r + 2];
            RayCache<K> cache;
            int kept;
            double prefix_hi;
            float acc[3] = {0.0f, 0.0f, 0.0f};
            float acc_a = 0.0f, acc_d = 0.0f;
            ray_forward<K, true, PREFETCH, kStashChunks>(start, n, ts, te, sig, rgb, eps, cache, kept, prefix_hi,
                                                         acc, acc_a, acc_d, pre, stash);
            wave_sum4(acc[0], acc[1], acc[2], acc_a);
            acc_d = wave_sum1(acc_d);
            const float cr = acc[0], cg = acc[1], cb = acc[2];
            const float er = cr - tr, eg = cg - tg, eb = cb - tb;
            RayGrad q;
            q.gr = uniform<float>(er * inv_count2);
            q.gg = uniform<float>(eg * inv_count2);
            q.gb = uniform<float>(eb * inv_count2);
            q.ga = 0.0f;
            q.gd = 0.0f;
            wave_total += static_cast<double>(er) * er + static_cast<double>(eg) * eg + static_cast<double>(eb) * eb;
            if (PREFETCH && todo != 0ull) {
                const int j = static_cast<int>(__builtin_ctzll(todo));
                pre = load_span(head_span(ts, te, sig, rgb, read_lane(my_start, j), read_lane(my_n, j), kWave),
                                lane_offset());
            }
            ray_backward<K, true, kStashChunks>(start, n, kept, prefix_hi, ts, te, sig, rgb, cache, q, g_sigmas,
                                                g_rgbs, stash);
            // stored after the backward: a store before it would make the
            // backward's first wait on memory also wait for the store
            if (lane == 0) {
                color[3 * r] = cr;
                color[3 * r + 1] = cg;
                color[3 * r + 2] = cb;
                opacity[r] = acc_a;
                depth[r] = acc_d;
            }
        }
    }
    // one partial per wave: no workgroup barrier, which would make every
    // wave wait for its gradient stores to complete before it could exit
    if (lane == 0) loss_partial[static_cast<int64_t>(blockIdx.x) * kRaysPerRenderBlock + wave] = wave_total;
}

// First level of the loss sum: workgroup b adds partials
// [b * kSumSpan, (b + 1) * kSumSpan) in a fixed order.
constexpr int kSumThreads = 256;
constexpr int kSumPerThread = 16;
constexpr int64_t kSumSpan = static_cast<int64_t>(kSumThreads) * kSumPerThread;

__global__ __launch_bounds__(kSumThreads) void loss_sum_kernel(const double* __restrict__ partial, int64_t n,
                                                               double* __restrict__ out) {
    __shared__ double part[kSumThreads];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kSumSpan + threadIdx.x;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kSumPerThread; ++j) {
        const int64_t i = base + static_cast<int64_t>(j) * kSumThreads;
        s += i < n ? partial[i] : 0.0;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = kSumThreads / 2; off > 0; off >>= 1) {
        if (static_cast<int>(threadIdx.x) < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

// loss = (sum of the partials, in a fixed order) / (3 n_rays).
constexpr int kLossThreads = 1024;

__global__ __launch_bounds__(kLossThreads) void loss_reduce_kernel(const double* __restrict__ partial, int64_t nb,
                                                                   double inv_count, float* __restrict__ loss) {
    __shared__ double part[kLossThreads];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += kLossThreads) s += partial[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = kLossThreads / 2; off > 0; off >>= 1) {
        if (static_cast<int>(threadIdx.x) < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = static_cast<float>(part[0] * inv_count);
}

int64_t render_blocks(int64_t n_rays) { return (n_rays + kRaysPerRenderBlock - 1) / kRaysPerRenderBlock; }

// The fused kernel walks the rays grid-stride with at most
// tuning().render_mse_max_blocks workgroups (one ray per wave when that is
// at least render_blocks).
int64_t mse_blocks(int64_t n_rays) {
    return std::max<int64_t>(1, std::min<int64_t>(render_blocks(n_rays), tuning().render_mse_max_blocks));
}

// Partials of the fused loss at any tuning: one per wave of the largest
// grid, then one per workgroup of loss_sum_kernel.
int64_t mse_partials(int64_t n_rays) { return std::max<int64_t>(1, render_blocks(n_rays)) * kRaysPerRenderBlock; }
int64_t mse_sums(int64_t n_rays) { return (mse_partials(n_rays) + kSumSpan - 1) / kSumSpan; }

// Kernels instantiated for 1..4 register-cached chunks per ray.
template <template <int> class F, typename... A>
void dispatch_cached(int k, A&&... a) {
    switch (k) {
        case 1: F<1>::run(a...); break;
        case 3: F<3>::run(a...); break;
        case 4: F<4>::run(a...); break;
        default: F<2>::run(a...); break;
    }
}

template <int K>
struct LaunchBwd {
    static void run(dim3 grid, hipStream_t s, const int32_t* packed_info, int64_t n_rays, int64_t n_samples,
                    const float* ts, const float* te, const float* sig, const float* rgb, float eps, const float* gc,
                    const float* go, const float* gd, float* g_sig, float* g_rgb) {
        hipLaunchKernelGGL(render_bwd_kernel<K>, grid, dim3(kRenderThreads), 0, s, packed_info, n_rays, n_samples, ts,
                           te, sig, rgb, eps, gc, go, gd, g_sig, g_rgb);
    }
};

template <int K>
struct LaunchMse {
    static void run(dim3 grid, hipStream_t s, const int32_t* packed_info, int64_t n_rays, int64_t n_samples,
                    const float* ts, const float* te, const float* sig, const float* rgb, float eps, const float* target,
                    float inv_count2, float* color, float* opacity, float* depth, float* g_sig, float* g_rgb,
                    double* partial) {
        // one wave per ray: the plain kernel; several rays per wave: the
        // grouped one, which finishes the rays without samples lane-parallel
        const bool grouped = static_cast<int64_t>(grid.x) * kRaysPerRenderBlock < n_rays;
        if (tuning().render_prefetch != 0 && grouped) {
            hipLaunchKernelGGL((render_mse_grouped_kernel<K, true>), grid, dim3(kRenderThreads), 0, s, packed_info,
                               n_rays, n_samples, ts, te, sig, rgb, eps, target, inv_count2, color, opacity, depth,
                               g_sig, g_rgb, partial);
        } else if (grouped) {
            hipLaunchKernelGGL((render_mse_grouped_kernel<K, false>), grid, dim3(kRenderThreads), 0, s, packed_info,
                               n_rays, n_samples, ts, te, sig, rgb, eps, target, inv_count2, color, opacity, depth,
                               g_sig, g_rgb, partial);
        } else if (tuning().render_prefetch != 0) {
            hipLaunchKernelGGL((render_mse_kernel<K, true>), grid, dim3(kRenderThreads), 0, s, packed_info, n_rays,
                               n_samples, ts, te, sig, rgb, eps, target, inv_count2, color, opacity, depth, g_sig,
                               g_rgb, partial);
        } else {
            hipLaunchKernelGGL((render_mse_kernel<K, false>), grid, dim3(kRenderThreads), 0, s, packed_info, n_rays,
                               n_samples, ts, te, sig, rgb, eps, target, inv_count2, color, opacity, depth, g_sig,
                               g_rgb, partial);
        }
    }
};

// ---------------------------------------------------------------------------
// Visibility pruning while marching (Sec. 2.1, "Pruning Empty and Occluded
// Regions"; Sec. 3, ray_marching with sigma_fn / early_stop_eps /
// alpha_thre): with the densities of the marched samples, keep a sample iff
// its transmittance is at least eps and its opacity at least alpha_thre.
// The transmittance is the renderer's (chunk_transmittance + chunk_keep), so
// the cut falls where rendering would place it.  The compaction reuses the
// marching scan: count (keep flags + per-ray counts), scan, fill.
// ---------------------------------------------------------------------------

// One wave per ray, four waves per workgroup of kRaysPerBlock rays.
template <bool PRUNE_FILL>
__global__ __launch_bounds__(kRenderThreads) void prune_kernel(
    const int32_t* __restrict__ packed_info, int64_t n_rays, int64_t n_samples, const float* __restrict__ ts,
    const float* __restrict__ te, const float* __restrict__ sig, float eps, float alpha_thre,
    uint8_t* __restrict__ keep, int32_t* __restrict__ packed_out, int64_t* __restrict__ block_sums,
    int64_t capacity, int32_t* __restrict__ ri_out, float* __restrict__ ts_out, float* __restrict__ te_out,
    float* __restrict__ sig_out, int32_t* __restrict__ status) {
    __shared__ int64_t wave_total[kRaysPerRenderBlock];
    const int lane = lane_id();
    const int wave = uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kRaysPerBlock;
    int64_t total = 0;
    bool overflow = false;
    for (int j = wave; j < kRaysPerBlock; j += kRaysPerRenderBlock) {
        const int64_t r = first + j;
        if (r >= n_rays) break;
        int64_t start;
        int n;
        ray_range(packed_info, r, n_samples, start, n);
        if (!PRUNE_FILL) {
            double carry = 0.0;
            int count = 0;
            int c = 0;
            for (; c < n; c += kWave) {
                const int i = c + lane;
                const bool valid = i < n;
                const int64_t s = start + i;
                Sample x{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                if (valid) {
                    x.t0 = ts[s];
                    x.t1 = te[s];
                    x.sigma = sig[s];
                }
                const Trans t = chunk_transmittance(x, carry);
                const int keep_n = chunk_keep(valid, t.t_in, eps);
                const bool k = valid && lane < keep_n && alpha_of(t.tau) >= alpha_thre;
                if (valid) keep[s] = k ? 1 : 0;
                count += __popcll(ballot(k));
                carry += static_cast<double>(read_lane(t.incl, 63));
                if (keep_n < kWave) {
                    c += kWave;
                    break;
                }
            }
            for (; c < n; c += kWave) {  // behind the cut
                if (c + lane < n) keep[start + c + lane] = 0;
            }
            if (lane == 0) packed_out[2 * r + 1] = count;
            total += count;
        } else {
            const int64_t out0 = packed_out[2 * r];
            const int limit = uniform<int>(packed_out[2 * r + 1]);
            int written = 0;
            for (int c = 0; c < n && written < limit; c += kWave) {
                const int i = c + lane;
                const int64_t s = start + i;
                const bool k = i < n && keep[s] != 0;
                const uint64_t m = ballot(k);
                const int idx = written + bits_below(m);
                if (k && idx < limit) {
                    const int64_t pos = out0 + idx;
                    if (pos >= 0 && pos < capacity) {
                        ri_out[pos] = static_cast<int32_t>(r);
                        ts_out[pos] = ts[s];
                        te_out[pos] = te[s];
                        if (sig_out != nullptr) sig_out[pos] = sig[s];
                    } else {
                        overflow = true;
                    }
                }
                written += __popcll(m);
            }
        }
    }
    if (!PRUNE_FILL) {
        if (lane == 0) wave_total[wave] = total;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t sum = 0;
            for (int w = 0; w < kRaysPerRenderBlock; ++w) sum += wave_total[w];
            block_sums[blockIdx.x] = sum;
        }
    } else if (overflow && status != nullptr) {
        *status = NACC_ECAPACITY;
    }
}

__global__ void prune_status_kernel(int32_t* status) { *status = NACC_OK; }

int validate_render(const int32_t* packed_info, int64_t n_rays, int64_t n_samples, const float* ts,
                    const float* te, const float* sig, const float* rgb, float eps) {
    NACC_REQUIRE(n_rays >= 0 && n_rays <= INT32_MAX, NACC_EINVAL, "n_rays = %lld out of [0, 2^31-1]",
                 static_cast<long long>(n_rays));
    NACC_REQUIRE(n_samples >= 0 && n_samples <= INT32_MAX, NACC_EINVAL, "n_samples = %lld out of [0, 2^31-1]",
                 static_cast<long long>(n_samples));
    NACC_REQUIRE(n_rays == 0 || packed_info != nullptr, NACC_EINVAL, "packed_info must be non-NULL");
    NACC_REQUIRE(n_samples == 0 || (ts != nullptr && te != nullptr && sig != nullptr && rgb != nullptr),
                 NACC_EINVAL, "sample inputs must be non-NULL");
    NACC_REQUIRE(!std::isnan(eps) && eps >= 0.0f && eps < 1.0f, NACC_EINVAL, "early_stop_eps = %g out of [0, 1)",
                 eps);
    return NACC_OK;
}

}  // namespace

extern "C" {

int nacc_render_fwd(const int32_t* packed_info, int64_t n_rays, int64_t n_samples, const float* t_starts,
                    const float* t_ends, const float* sigmas, const float* rgbs, float early_stop_eps, float* color,
                    float* opacity, float* depth, float* weights, int32_t* kept, void* stream) {
    clear_error();
    int st = validate_render(packed_info, n_rays, n_samples, t_starts, t_ends, sigmas, rgbs, early_stop_eps);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(n_rays == 0 || (color != nullptr && opacity != nullptr && depth != nullptr), NACC_EINVAL,
                 "color, opacity and depth must be non-NULL");
    if (n_rays == 0) return NACC_OK;
    hipStream_t s = as_stream(stream);
    const dim3 grid(static_cast<unsigned>(render_blocks(n_rays)));
    if (weights != nullptr) {
        hipLaunchKernelGGL(render_fwd_kernel<true>, grid, dim3(kRenderThreads), 0, s, packed_info, n_rays,
                           n_samples, t_starts, t_ends, sigmas, rgbs, early_stop_eps, color, opacity, depth, weights,
                           kept);
    } else {
        hipLaunchKernelGGL(render_fwd_kernel<false>, grid, dim3(kRenderThreads), 0, s, packed_info, n_rays,
                           n_samples, t_starts, t_ends, sigmas, rgbs, early_stop_eps, color, opacity, depth, weights,
                           kept);
    }
    return check_launch("render fwd");
}

int nacc_render_bwd(const int32_t* packed_info, int64_t n_rays, int64_t n_samples, const float* t_starts,
                    const float* t_ends,
                    const float* sigmas, const float* rgbs, float early_stop_eps, const float* g_color,
                    const float* g_opacity, const float* g_depth, float* g_sigmas, float* g_rgbs, void* stream) {
    clear_error();
    int st = validate_render(packed_info, n_rays, n_samples, t_starts, t_ends, sigmas, rgbs, early_stop_eps);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(n_rays == 0 || (g_color != nullptr && g_sigmas != nullptr && g_rgbs != nullptr), NACC_EINVAL,
                 "g_color, g_sigmas and g_rgbs must be non-NULL");
    if (n_rays == 0) return NACC_OK;
    hipStream_t s = as_stream(stream);
    dispatch_cached<LaunchBwd>(tuning().render_cached_chunks, dim3(static_cast<unsigned>(render_blocks(n_rays))), s,
                               packed_info, n_rays, n_samples, t_starts, t_ends, sigmas, rgbs, early_stop_eps, g_color,
                               g_opacity, g_depth, g_sigmas, g_rgbs);
    return check_launch("render bwd");
}

int64_t nacc_render_mse_workspace_size(int64_t n_rays) {
    if (n_rays < 0) return -1;
    // the same at any tuning (render_blocks bounds mse_blocks)
    return (((mse_partials(n_rays) + mse_sums(n_rays)) * static_cast<int64_t>(sizeof(double)) + 255) / 256) * 256;
}

}  // extern "C"

namespace {

// The fused loss call after validation of everything but the workspace:
// `partial` holds mse_partials(n_rays) + mse_sums(n_rays) doubles.  Every
// entry the call reads is written earlier in the same call (one partial per
// wave of the grid, one first-level sum per summing workgroup), so the
// workspace needs no clearing.
int render_mse_launch(const int32_t* packed_info, int64_t n_rays, int64_t n_samples, const float* t_starts,
                      const float* t_ends, const float* sigmas, const float* rgbs, float early_stop_eps,
                      const float* target, int64_t loss_rays, float* color, float* opacity, float* depth,
                      float* g_sigmas, float* g_rgbs, float* loss, double* partial, hipStream_t s) {
    const int64_t nb = mse_blocks(n_rays);
    const double count = 3.0 * static_cast<double>(loss_rays);
    const float inv_count2 = static_cast<float>(2.0 / count);
    dispatch_cached<LaunchMse>(tuning().render_cached_chunks, dim3(static_cast<unsigned>(nb)), s, packed_info, n_rays,
                               n_samples, t_starts, t_ends, sigmas, rgbs, early_stop_eps, target, inv_count2, color,
                               opacity, depth, g_sigmas, g_rgbs, partial);
    int st = check_launch("render fwd+bwd+mse");
    if (st != NACC_OK) return st;
    const int64_t n_part = nb * kRaysPerRenderBlock;
    const int64_t n_sums = (n_part + kSumSpan - 1) / kSumSpan;
    double* sums = partial + mse_partials(n_rays);
    hipLaunchKernelGGL(loss_sum_kernel, dim3(static_cast<unsigned>(n_sums)), dim3(kSumThreads), 0, s, partial, n_part,
                       sums);
    st = check_launch("render loss sum");
    if (st != NACC_OK) return st;
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(kLossThreads), 0, s, sums, n_sums, 1.0 / count, loss);
    return check_launch("render loss");
}

// Argument checks shared by both forms of the fused loss call; the
// workspace is checked by each form.
int validate_mse(const int32_t* packed_info, int64_t n_rays, int64_t n_samples, const float* t_starts,
                 const float* t_ends, const float* sigmas, const float* rgbs, float early_stop_eps,
                 const float* target, int64_t& loss_rays, float* color, float* opacity, float* depth,
                 float* g_sigmas, float* g_rgbs, float* loss) {
    int st = validate_render(packed_info, n_rays, n_samples, t_starts, t_ends, sigmas, rgbs, early_stop_eps);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(n_rays > 0, NACC_EINVAL, "the mean squared error needs n_rays > 0");
    if (loss_rays == 0) loss_rays = n_rays;
    NACC_REQUIRE(loss_rays >= n_rays, NACC_EINVAL, "loss_rays = %lld < n_rays = %lld",
                 static_cast<long long>(loss_rays), static_cast<long long>(n_rays));
    NACC_REQUIRE(target != nullptr && color != nullptr && opacity != nullptr && depth != nullptr &&
                     g_sigmas != nullptr && g_rgbs != nullptr && loss != nullptr,
                 NACC_EINVAL, "outputs and target must be non-NULL");
    return NACC_OK;
}

}  // namespace

// Device memory of nacc_render_fwd_bwd_mse_noalloc, in place of a caller's
// workspace: every GPU the library runs on holds its own copy until the
// process ends.  Host code never passes this name to a kernel (on the host it
// is only a stand-in for the symbol); it uses the device address resolved
// for the current device by mse_static_scratch.
static __device__ __align__(256) unsigned char scratch[NACC_MSE_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device, resolved once per
// device (hipGetSymbolAddress with that device current; no allocation).
int mse_static_scratch(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    NACC_REQUIRE(e == hipSuccess, NACC_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    NACC_REQUIRE(dev >= 0 && dev < kMaxDevices, NACC_ENOTSUP, "device %d beyond the %d devices supported", dev,
                 kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        NACC_REQUIRE(e == hipSuccess && p != nullptr, NACC_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                     hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<double*>(g_scratch_ptr[dev]);
    return NACC_OK;
}

}  // namespace

extern "C" {

int nacc_render_fwd_bwd_mse(const int32_t* packed_info, int64_t n_rays, int64_t n_samples, const float* t_starts,
                            const float* t_ends, const float* sigmas, const float* rgbs, float early_stop_eps,
                            const float* target, int64_t loss_rays, float* color, float* opacity, float* depth,
                            float* g_sigmas, float* g_rgbs, float* loss, void* workspace, size_t workspace_bytes,
                            void* stream) {
    clear_error();
    int st = validate_mse(packed_info, n_rays, n_samples, t_starts, t_ends, sigmas, rgbs, early_stop_eps, target,
                          loss_rays, color, opacity, depth, g_sigmas, g_rgbs, loss);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(workspace != nullptr, NACC_EINVAL, "workspace must be non-NULL");
    const int64_t need = nacc_render_mse_workspace_size(n_rays);
    NACC_REQUIRE(static_cast<int64_t>(workspace_bytes) >= need, NACC_ESHAPE, "workspace of %zu bytes, need %lld",
                 workspace_bytes, static_cast<long long>(need));
    return render_mse_launch(packed_info, n_rays, n_samples, t_starts, t_ends, sigmas, rgbs, early_stop_eps, target,
                             loss_rays, color, opacity, depth, g_sigmas, g_rgbs, loss,
                             static_cast<double*>(workspace), as_stream(stream));
}

int nacc_render_fwd_bwd_mse_noalloc(const int32_t* packed_info, int64_t n_rays, int64_t n_samples,
                                    const float* t_starts, const float* t_ends, const float* sigmas,
                                    const float* rgbs, float early_stop_eps, const float* target, int64_t loss_rays,
                                    float* color, float* opacity, float* depth, float* g_sigmas, float* g_rgbs,
                                    float* loss, void* stream) {
    clear_error();
    int st = validate_mse(packed_info, n_rays, n_samples, t_starts, t_ends, sigmas, rgbs, early_stop_eps, target,
                          loss_rays, color, opacity, depth, g_sigmas, g_rgbs, loss);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(n_rays <= NACC_MSE_NOALLOC_MAX_RAYS, NACC_ECAPACITY,
                 "n_rays = %lld exceeds the %lld rays the static scratch of %lld bytes holds",
                 static_cast<long long>(n_rays), static_cast<long long>(NACC_MSE_NOALLOC_MAX_RAYS),
                 static_cast<long long>(NACC_MSE_NOALLOC_SCRATCH_BYTES));
    NACC_REQUIRE(nacc_render_mse_workspace_size(n_rays) <= NACC_MSE_NOALLOC_SCRATCH_BYTES, NACC_ECAPACITY,
                 "n_rays = %lld needs %lld bytes of scratch, more than the static %lld",
                 static_cast<long long>(n_rays), static_cast<long long>(nacc_render_mse_workspace_size(n_rays)),
                 static_cast<long long>(NACC_MSE_NOALLOC_SCRATCH_BYTES));
    double* partial = nullptr;
    st = mse_static_scratch(&partial);
    if (st != NACC_OK) return st;
    return render_mse_launch(packed_info, n_rays, n_samples, t_starts, t_ends, sigmas, rgbs, early_stop_eps, target,
                             loss_rays, color, opacity, depth, g_sigmas, g_rgbs, loss, partial, as_stream(stream));
}

int64_t nacc_prune_workspace_size(int64_t n_rays) {
    if (n_rays < 0) return -1;
    const int64_t nb = num_blocks(n_rays);  // the workgroup sums, then the scan's scratch
    return (((nb + scan_scratch_values(nb)) * static_cast<int64_t>(sizeof(int64_t)) + 255) / 256) * 256;
}

int nacc_prune_count(const int32_t* packed_info, int64_t n_rays, int64_t n_samples, const float* t_starts,
                     const float* t_ends, const float* sigmas, float early_stop_eps, float alpha_thre,
                     uint8_t* keep, int32_t* packed_out, int64_t* total, void* workspace, size_t workspace_bytes,
                     void* stream) {
    clear_error();
    NACC_REQUIRE(n_rays >= 0 && n_rays <= INT32_MAX, NACC_EINVAL, "n_rays = %lld out of [0, 2^31-1]",
                 static_cast<long long>(n_rays));
    NACC_REQUIRE(n_samples >= 0 && n_samples <= INT32_MAX, NACC_EINVAL, "n_samples = %lld out of [0, 2^31-1]",
                 static_cast<long long>(n_samples));
    NACC_REQUIRE(total != nullptr, NACC_EINVAL, "total must be non-NULL");
    NACC_REQUIRE(n_rays == 0 || (packed_info != nullptr && packed_out != nullptr), NACC_EINVAL,
                 "packed_info and packed_out must be non-NULL");
    NACC_REQUIRE(n_samples == 0 || (t_starts != nullptr && t_ends != nullptr && sigmas != nullptr && keep != nullptr),
                 NACC_EINVAL, "sample arrays and keep must be non-NULL");
    NACC_REQUIRE(!std::isnan(early_stop_eps) && early_stop_eps >= 0.0f, NACC_EINVAL,
                 "early_stop_eps = %g must be >= 0", early_stop_eps);
    NACC_REQUIRE(!std::isnan(alpha_thre), NACC_EINVAL, "alpha_thre is NaN");
    const int64_t need = nacc_prune_workspace_size(n_rays);
    NACC_REQUIRE(workspace != nullptr && static_cast<int64_t>(workspace_bytes) >= need, NACC_ESHAPE,
                 "workspace of %zu bytes, need %lld", workspace_bytes, static_cast<long long>(need));
    hipStream_t s = as_stream(stream);
    int64_t* sums = static_cast<int64_t*>(workspace);
    const int64_t nb = num_blocks(n_rays);
    if (nb > 0) {
        hipLaunchKernelGGL(prune_kernel<false>, dim3(static_cast<unsigned>(nb)), dim3(kRenderThreads), 0, s,
                           packed_info, n_rays, n_samples, t_starts, t_ends, sigmas, early_stop_eps, alpha_thre, keep,
                           packed_out, sums, 0, nullptr, nullptr, nullptr, nullptr, nullptr);
        int st = check_launch("prune count");
        if (st != NACC_OK) return st;
    }
    scan_exclusive(sums, nb, total, sums + nb, s);
    int st = check_launch("prune scan");
    if (st != NACC_OK || nb == 0) return st;
    hipLaunchKernelGGL(finalize_starts_kernel, dim3(static_cast<unsigned>(nb)), dim3(kRaysPerBlock), 0, s, sums,
                       n_rays, packed_out);
    return check_launch("prune starts");
}

int nacc_prune_fill(const int32_t* packed_info, int64_t n_rays, int64_t n_samples, const float* t_starts,
                    const float* t_ends, const float* sigmas, const uint8_t* keep, const int32_t* packed_out,
                    int64_t capacity, int32_t* ray_indices_out, float* t_starts_out, float* t_ends_out,
                    float* sigmas_out, int32_t* status, void* stream) {
    clear_error();
    NACC_REQUIRE(n_rays >= 0 && n_rays <= INT32_MAX, NACC_EINVAL, "n_rays = %lld out of [0, 2^31-1]",
                 static_cast<long long>(n_rays));
    NACC_REQUIRE(n_samples >= 0 && n_samples <= INT32_MAX, NACC_EINVAL, "n_samples = %lld out of [0, 2^31-1]",
                 static_cast<long long>(n_samples));
    NACC_REQUIRE(capacity >= 0 && capacity <= INT32_MAX, NACC_ECAPACITY, "capacity = %lld out of [0, 2^31-1]",
                 static_cast<long long>(capacity));
    NACC_REQUIRE(n_rays == 0 || (packed_info != nullptr && packed_out != nullptr), NACC_EINVAL,
                 "packed_info and packed_out must be non-NULL");
    NACC_REQUIRE(n_samples == 0 || (t_starts != nullptr && t_ends != nullptr && keep != nullptr), NACC_EINVAL,
                 "sample arrays and keep must be non-NULL");
    NACC_REQUIRE(sigmas_out == nullptr || n_samples == 0 || sigmas != nullptr, NACC_EINVAL,
                 "sigmas_out needs sigmas");
    NACC_REQUIRE(capacity == 0 || (ray_indices_out != nullptr && t_starts_out != nullptr && t_ends_out != nullptr),
                 NACC_EINVAL, "outputs must be non-NULL");
    hipStream_t s = as_stream(stream);
    if (status != nullptr) {
        hipLaunchKernelGGL(prune_status_kernel, dim3(1), dim3(1), 0, s, status);
        int st = check_launch("prune status");
        if (st != NACC_OK) return st;
    }
    const int64_t nb = num_blocks(n_rays);
    if (nb == 0) return NACC_OK;
    hipLaunchKernelGGL(prune_kernel<true>, dim3(static_cast<unsigned>(nb)), dim3(kRenderThreads), 0, s, packed_info,
                       n_rays, n_samples, t_starts, t_ends, sigmas, 0.0f, 0.0f, const_cast<uint8_t*>(keep),
                       const_cast<int32_t*>(packed_out), nullptr, capacity, ray_indices_out, t_starts_out, t_ends_out,
                       sigmas_out, status);
    return check_launch("prune fill");
}

}  // extern "C"
