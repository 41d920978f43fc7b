// Differentiable rendering of arbitrary per-sample attributes (NerfAcc
// Sec. 2.2: any sample attribute, not only colour, is rendered the way
// Eq. 1 renders colour), with a constant background blended by 1 - opacity
// (the constant background of the Instant-NGP example, Sec. 4) and an
// opacity threshold below which a sample counts as empty.
//
// One wavefront per ray, chunks of 64 samples, the transmittance routine of
// the colour kernels (transmittance.h); a sample whose opacity is below the
// threshold enters the scan with tau = 0, so it neither contributes nor
// attenuates, the same as a ray from which it was dropped.  Attributes go
// through the lanes' registers 16 channels at a time: the forward walks the
// ray once per block of 16 channels (re-reading only t and sigma), the
// backward forms v_i = g . a_i over all blocks, then writes w_i g.  With 3
// channels, no background and no threshold the results are bit for bit
// those of the colour kernels.
#include <cmath>

#include "common.h"
#include "transmittance.h"

#pragma clang fp contract(off)

namespace {

using namespace nacc;
using namespace nacc::dev;
using namespace nacc::vr;

constexpr int kAttrThreads = 256;  // 4 waves, one ray each
constexpr int kAttrRays = kAttrThreads / kWave;
constexpr int kBlock = 16;  // channels held per lane at a time

struct Interval {
    float t0, t1, sigma;
};

__device__ __forceinline__ Interval load_interval(bool valid, int64_t s, const float* __restrict__ ts,
                                                  const float* __restrict__ te, const float* __restrict__ sig) {
    Interval x{0.0f, 0.0f, 0.0f};
    if (valid) {
        x.t0 = ts[s];
        x.t1 = te[s];
        x.sigma = sig[s];
    }
    return x;
}

// Opacity, the tau entering the scan, and whether the sample counts (its
// opacity reaches the threshold; a threshold <= 0 keeps every sample).
struct Masked {
    float tau, alpha;
    bool on;
};

__device__ __forceinline__ Masked masked(const Interval& x, float alpha_thre) {
    Masked m;
    const float tau = x.sigma * (x.t1 - x.t0);
    m.alpha = alpha_of(tau);
    m.on = !(alpha_thre > 0.0f) || m.alpha >= alpha_thre;
    m.tau = m.on ? tau : 0.0f;
    return m;
}

// Channels [c0, c0 + cb) of sample s (cb <= kBlock, wave-uniform), zeros
// past cb.  VEC4: rows start 16-byte aligned and cb is a multiple of 4.
template <bool VEC4>
__device__ __forceinline__ void load_block(bool valid, int64_t s, const float* __restrict__ attrs, int n_ch, int c0,
                                           int cb, float a[kBlock]) {
    const float* row = attrs + s * n_ch + c0;
#pragma unroll
    for (int k = 0; k < kBlock; k += 4) {
        if (k < cb) {
            if (VEC4) {
                const float4 v = valid ? *reinterpret_cast<const float4*>(row + k) : make_float4(0.f, 0.f, 0.f, 0.f);
                a[k] = v.x;
                a[k + 1] = v.y;
                a[k + 2] = v.z;
                a[k + 3] = v.w;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) a[k + j] = (valid && k + j < cb) ? row[k + j] : 0.0f;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) a[k + j] = 0.0f;
        }
    }
}

// Row s of the attribute gradient: w * g, or zeros (positive zeros, as the
// colour kernels write) when `zero`.
template <bool VEC4>
__device__ __forceinline__ void store_scaled(int64_t s, float* __restrict__ g_attrs, int n_ch,
                                             const float* __restrict__ g, float w, bool zero) {
    float* row = g_attrs + s * n_ch;
    if (VEC4) {
        for (int k = 0; k < n_ch; k += 4) {
            *reinterpret_cast<float4*>(row + k) =
                zero ? make_float4(0.0f, 0.0f, 0.0f, 0.0f)
                     : make_float4(w * uniform<float>(g[k]), w * uniform<float>(g[k + 1]),
                                   w * uniform<float>(g[k + 2]), w * uniform<float>(g[k + 3]));
        }
    } else {
        for (int k = 0; k < n_ch; ++k) row[k] = zero ? 0.0f : w * uniform<float>(g[k]);
    }
}

// Rows of 4 or 8 channels, or of a multiple of 16 (16-byte aligned rows),
// move between memory and the lanes through LDS, one block of up to 16
// channels at a time: the wave reads and writes a chunk's 64 row segments
// as whole float4s in address order (runs of 1 KB, or of 64 bytes per row
// for wider rows) instead of each lane touching its own row, which stalls
// the vector L1 on tag lookups.  Row r's float4 j sits in slot j ^ (r & 3)
// of the row's four, so that lanes reading their own rows spread over the
// LDS banks.
struct Staged {
    int qpr;  // float4s per block of a row: 1, 2 or 4
    int sh;   // log2(qpr)
    int rs;   // float4s per row
};

__device__ __forceinline__ Staged staged_rows(int n_ch) {
    const int qpr = n_ch >= kBlock ? 4 : n_ch >> 2;
    return Staged{qpr, qpr == 4 ? 2 : (qpr == 2 ? 1 : 0), n_ch >> 2};
}

// Rows [0, rows) of the chunk starting at `first`, as this lane's share of
// whole float4s in address order (zeros past `rows`).  Issued early; the
// values are only needed by exchange_rows.
struct RowQuads {
    float4 v[4];
};

template <bool WIDE>
__device__ __forceinline__ RowQuads fetch_rows(const Staged& g, const float* __restrict__ attrs, int64_t first,
                                               int rows, int c0) {
    const int lane = lane_id();
    const float4* src = reinterpret_cast<const float4*>(attrs) + first * g.rs + (c0 >> 2);
    RowQuads r;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        r.v[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (k < g.qpr) {
            const int q = lane + kWave * k;
            const int row = q >> g.sh, quad = q & (g.qpr - 1);
            // rows of one block are contiguous: their float4s run in order
            if (row < rows) r.v[k] = src[WIDE ? row * g.rs + quad : q];
        }
    }
    return r;
}

// The fetched float4s, regrouped through `stage` so that lane i holds row i
// in a[] (zeros past n_ch).
__device__ __forceinline__ void exchange_rows(const Staged& g, const RowQuads& r, float4* __restrict__ stage,
                                              float a[kBlock]) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < g.qpr) {
            const int q = lane + kWave * k;
            const int row = q >> g.sh, quad = q & (g.qpr - 1);
            stage[row * 4 + (quad ^ (row & 3))] = r.v[k];
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (j < g.qpr) v = stage[lane * 4 + (j ^ (lane & 3))];
        a[4 * j] = v.x;
        a[4 * j + 1] = v.y;
        a[4 * j + 2] = v.z;
        a[4 * j + 3] = v.w;
    }
    wave_lds_sync();  // the stage is rewritten by the next chunk
}

// Value of `x` in lane `src` (all lanes active).
__device__ __forceinline__ float lane_value(float x, int src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, x)));
}

// Block c0 of rows [0, rows) of the gradient chunk starting at `first`:
// row i = w_i g, or zeros where lane i's `keep` is false, written as whole
// float4s in address order; gq holds g's float4 c0 / 4 + (lane & (qpr - 1)),
// which is the one every float4 this lane writes needs.
template <bool WIDE>
__device__ __forceinline__ void store_rows_staged(const Staged& g, float* __restrict__ g_attrs, int64_t first,
                                                  int rows, int c0, float w, bool keep, const float gq[4]) {
    const int lane = lane_id();
    float4* dst = reinterpret_cast<float4*>(g_attrs) + first * g.rs + (c0 >> 2);
    const float kf = keep ? 1.0f : 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < g.qpr) {
            const int q = lane + kWave * k;
            const int row = q >> g.sh, quad = q & (g.qpr - 1);
            const float wr = lane_value(w, row);
            const bool kr = lane_value(kf, row) != 0.0f;
            if (row < rows) {
                dst[WIDE ? row * g.rs + quad : q] = kr ? make_float4(wr * gq[0], wr * gq[1], wr * gq[2], wr * gq[3])
                            : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
    }
}

template <bool VEC4, int STAGE>
__global__ __launch_bounds__(kAttrThreads) void attrs_fwd_kernel(
    const int32_t* __restrict__ packed_info, int64_t n_rays, int64_t n_samples, const float* __restrict__ ts,
    const float* __restrict__ te, const float* __restrict__ sig, const float* __restrict__ attrs, int n_ch,
    float eps, float alpha_thre, const float* __restrict__ background, float* __restrict__ out,
    float* __restrict__ opacity, float* __restrict__ depth, float* __restrict__ weights) {
    // STAGE 0: per-lane rows; 1: rows of one block (4, 8 or 16 channels)
    // through LDS; 2: rows of several blocks of 16 through LDS
    constexpr bool STAGED = STAGE > 0, WIDE = STAGE == 2;
    const int lane = lane_id();
    const int64_t r = xcd_grouped<16>(blockIdx.x, gridDim.x) * kAttrRays + uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    if (r >= n_rays) return;
    int64_t start;
    int n;
    ray_range(packed_info, r, n_samples, start, n);
    // STAGED (aligned rows of 4 or 8 channels or a multiple of 16): rows
    // through LDS
    __shared__ float4 stage_all[STAGED ? kAttrRays * kWave * 4 : 1];
    float4* stage = stage_all + (STAGED ? uniform<int>(static_cast<int>(threadIdx.x) / kWave) * kWave * 4 : 0);
    const Staged sg = staged_rows(n_ch);
    float total_a = 0.0f;
    for (int c0 = 0; c0 < n_ch && (WIDE || c0 == 0 || !STAGED); c0 += kBlock) {
        const int cb = min(kBlock, n_ch - c0);
        const bool first = c0 == 0;
        float acc[kBlock];
#pragma unroll
        for (int k = 0; k < kBlock; ++k) acc[k] = 0.0f;
        float acc_a = 0.0f, acc_d = 0.0f;
        double carry = 0.0;
        int c = 0;
        for (; c < n; c += kWave) {
            const int i = c + lane;
            const bool valid = i < n;
            const int64_t s = start + i;
            const Interval x = load_interval(valid, s, ts, te, sig);
            RowQuads rq;
            if (STAGED) rq = fetch_rows<WIDE>(sg, attrs, start + c, min(n - c, kWave), c0);
            const Masked m = masked(x, alpha_thre);
            const Trans t = transmittance_of(m.tau, carry);
            const int keep_n = chunk_keep(valid, t.t_in, eps);
            const bool keep = valid && lane < keep_n && m.on;
            const float w = keep ? t.t_in * m.alpha : 0.0f;
            float a[kBlock];
            if (STAGED) {
                exchange_rows(sg, rq, stage, a);
            } else {
                load_block<VEC4>(valid, s, attrs, n_ch, c0, cb, a);
            }
#pragma unroll
            for (int k = 0; k < kBlock; ++k) acc[k] = __builtin_fmaf(w, a[k], acc[k]);
            if (first) {
                acc_a += w;
                acc_d = __builtin_fmaf(w, (x.t0 + x.t1) * 0.5f, acc_d);
                if (weights != nullptr && valid) weights[s] = w;
            }
            carry += static_cast<double>(read_lane(t.incl, 63));
            if (keep_n < kWave) {
                c += kWave;
                break;
            }
        }
        if (first) {
            if (weights != nullptr) {
                for (; c < n; c += kWave) {
                    if (c + lane < n) weights[start + c + lane] = 0.0f;
                }
            }
            total_a = wave_sum1(acc_a);
            acc_d = wave_sum1(acc_d);
            if (lane == 0) {
                if (opacity != nullptr) opacity[r] = total_a;
                if (depth != nullptr) depth[r] = acc_d;
            }
        }
#pragma unroll
        for (int k = 0; k < kBlock; ++k) {
            if (k < cb) {
                float v = wave_sum1(acc[k]);
                if (background != nullptr) v += background[c0 + k] * (1.0f - total_a);
                if (lane == 0) out[r * n_ch + c0 + k] = v;
            }
        }
    }
}

template <bool VEC4, int STAGE>
__global__ __launch_bounds__(kAttrThreads) void attrs_bwd_kernel(
    const int32_t* __restrict__ packed_info, int64_t n_rays, int64_t n_samples, const float* __restrict__ ts,
    const float* __restrict__ te, const float* __restrict__ sig, const float* __restrict__ attrs, int n_ch,
    float eps, float alpha_thre, const float* __restrict__ background, const float* __restrict__ g_out,
    const float* __restrict__ g_opacity, const float* __restrict__ g_depth, float* __restrict__ g_sigmas,
    float* __restrict__ g_attrs) {
    // STAGE 0: per-lane rows; 1: rows of one block (4, 8 or 16 channels)
    // through LDS; 2: rows of several blocks of 16 through LDS
    constexpr bool STAGED = STAGE > 0, WIDE = STAGE == 2;
    const int lane = lane_id();
    const int64_t r = xcd_grouped<16>(blockIdx.x, gridDim.x) * kAttrRays + uniform<int>(static_cast<int>(threadIdx.x) / kWave);
    if (r >= n_rays) return;
    int64_t start;
    int n;
    ray_range(packed_info, r, n_samples, start, n);
    if (n == 0) return;
    const float* g = g_out + r * n_ch;
    // STAGED (aligned rows of 4 or 8 channels or a multiple of 16): rows
    // through LDS
    __shared__ float4 stage_all[STAGED ? kAttrRays * kWave * 4 : 1];
    float4* stage = stage_all + (STAGED ? uniform<int>(static_cast<int>(threadIdx.x) / kWave) * kWave * 4 : 0);
    const Staged sg = staged_rows(n_ch);
    // the float4 of g's first block this lane's staged stores need, once per
    // ray (wider rows load their other blocks' per chunk)
    float gq0[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (STAGED) {
        const int quad = lane & (sg.qpr - 1);
#pragma unroll
        for (int m = 0; m < 4; ++m) gq0[m] = g[4 * quad + m];
    }
    // the background adds -g . background to the opacity's gradient
    float ga = g_opacity != nullptr ? uniform<float>(g_opacity[r]) : 0.0f;
    if (background != nullptr) {
        float gb = 0.0f;
        for (int k = 0; k < n_ch; ++k) gb += uniform<float>(g[k]) * background[k];
        ga -= gb;
    }
    const float gd = g_depth != nullptr ? uniform<float>(g_depth[r]) : 0.0f;
    // forward: the cut and the FP64 tau prefix at the start of every chunk
    // (lane j holds chunk j's for the first 64 chunks)
    double carry = 0.0, carry_prev = 0.0, prefix_hi = 0.0, carries = 0.0;
    int kept = n;
    for (int c = 0; c < n; c += kWave) {
        if (lane == c / kWave) carries = carry;
        const int i = c + lane;
        const bool valid = i < n;
        const Masked m = masked(load_interval(valid, start + i, ts, te, sig), alpha_thre);
        const Trans t = transmittance_of(m.tau, carry);
        const int keep_n = chunk_keep(valid, t.t_in, eps);
        if (keep_n < kWave) {
            kept = c + keep_n;
            prefix_hi = keep_n > 0 ? carry : carry_prev;
            break;
        }
        carry_prev = carry;
        carry += static_cast<double>(read_lane(t.incl, 63));
        prefix_hi = carry_prev;
    }
    const int c_hi = kept > 0 ? ((kept - 1) / kWave) * kWave : -kWave;
    // chunks past the cut: zeros
    for (int c = c_hi + kWave; c < n; c += kWave) {
        const int i = c + lane;
        if (i < n) {
            const int64_t s = start + i;
            g_sigmas[s] = 0.0f;
            store_scaled<VEC4>(s, g_attrs, n_ch, g, 0.0f, true);
        }
    }
    // backward, from the last kept chunk down
    float above = 0.0f;
    double p_end = 0.0;
    for (int c = c_hi; c >= 0; c -= kWave) {
        const int i = c + lane;
        const bool valid = i < n;
        const int64_t s = start + i;
        const Interval x = load_interval(i < kept, s, ts, te, sig);
        RowQuads rq;
        const int rows_read = max(0, min(kept - c, kWave));
        if (STAGED) rq = fetch_rows<WIDE>(sg, attrs, start + c, rows_read, 0);
        const Masked m = masked(x, alpha_thre);
        const float chunk_tau = wave_sum(m.tau);
        const int chunk = c / kWave;
        const double p_start = chunk < kWave ? read_lane(carries, chunk)
                                             : (c == c_hi ? prefix_hi : p_end - static_cast<double>(chunk_tau));
        const Trans t = transmittance_of(m.tau, p_start);
        const bool keep = i < kept && m.on;
        const float w = keep ? t.t_in * m.alpha : 0.0f;
        // v_i = g . a_i + (g_opacity - g . background) + g_depth m_i
        float dot = 0.0f;
        for (int c0 = 0; c0 < n_ch && (WIDE || c0 == 0 || !STAGED); c0 += kBlock) {
            const int cb = min(kBlock, n_ch - c0);
            float a[kBlock];
            if (STAGED) {
                if (WIDE && c0 > 0) rq = fetch_rows<WIDE>(sg, attrs, start + c, rows_read, c0);
                exchange_rows(sg, rq, stage, a);
            } else {
                load_block<VEC4>(i < kept, s, attrs, n_ch, c0, cb, a);
            }
#pragma unroll
            for (int k = 0; k < kBlock; ++k) {
                if (k < cb) {
                    dot = c0 + k == 0 ? uniform<float>(g[0]) * a[0]
                                      : __builtin_fmaf(uniform<float>(g[c0 + k]), a[k], dot);
                }
            }
        }
        const float v = dot + __builtin_fmaf(gd, (x.t0 + x.t1) * 0.5f, ga);
        const float wv = keep ? w * v : 0.0f;
        const float incl = wave_inclusive_suffix(wv);
        const float suffix = above + shift_down_one(incl);
        if (valid) g_sigmas[s] = keep ? (x.t1 - x.t0) * __builtin_fmaf(t.t_next, v, -suffix) : 0.0f;
        if (STAGED) {
            store_rows_staged<WIDE>(sg, g_attrs, start + c, min(n - c, kWave), 0, w, keep, gq0);
            for (int c0 = kBlock; WIDE && c0 < n_ch; c0 += kBlock) {
                const int quad = lane & (sg.qpr - 1);
                float gq[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) gq[m] = g[c0 + 4 * quad + m];
                store_rows_staged<WIDE>(sg, g_attrs, start + c, min(n - c, kWave), c0, w, keep, gq);
            }
        } else if (valid) {
            store_scaled<VEC4>(s, g_attrs, n_ch, g, w, !keep);
        }
        above = above + read_lane(incl, 0);
        p_end = p_start;
    }
}

int validate_attrs(const int32_t* packed_info, int64_t n_rays, int64_t n_samples, const float* ts, const float* te,
                   const float* sig, const float* attrs, int32_t n_ch, float eps, float alpha_thre) {
    NACC_REQUIRE(n_rays >= 0 && n_rays <= INT32_MAX, NACC_EINVAL, "n_rays = %lld out of [0, 2^31-1]",
                 static_cast<long long>(n_rays));
    NACC_REQUIRE(n_samples >= 0 && n_samples <= INT32_MAX, NACC_EINVAL, "n_samples = %lld out of [0, 2^31-1]",
                 static_cast<long long>(n_samples));
    NACC_REQUIRE(n_ch >= 1 && n_ch <= 4096, NACC_EINVAL, "n_ch = %d out of [1, 4096]", n_ch);
    NACC_REQUIRE(n_samples * static_cast<int64_t>(n_ch) <= (int64_t{1} << 40), NACC_ESHAPE,
                 "n_samples * n_ch exceeds 2^40");
    NACC_REQUIRE(n_rays == 0 || packed_info != nullptr, NACC_EINVAL, "packed_info must be non-NULL");
    NACC_REQUIRE(n_samples == 0 || (ts != nullptr && te != nullptr && sig != nullptr && attrs != nullptr),
                 NACC_EINVAL, "sample inputs must be non-NULL");
    NACC_REQUIRE(!std::isnan(eps) && eps >= 0.0f && eps < 1.0f, NACC_EINVAL, "early_stop_eps = %g out of [0, 1)",
                 eps);
    NACC_REQUIRE(std::isfinite(alpha_thre), NACC_EINVAL, "alpha_thre = %g must be finite", alpha_thre);
    return NACC_OK;
}

// Row widths that go through LDS: 4 or 8 channels, or whole blocks of
// kBlock.
bool staged_width(int32_t n_ch) { return n_ch == 4 || n_ch == 8 || n_ch % kBlock == 0; }

// Rows of 16-byte aligned float4s (attribute and gradient arrays alike).
bool vec4_rows(const float* a, const float* b, int32_t n_ch) {
    return n_ch % 4 == 0 && (reinterpret_cast<uintptr_t>(a) % 16) == 0 && (reinterpret_cast<uintptr_t>(b) % 16) == 0;
}

}  // namespace

extern "C" {

int nacc_render_attrs_fwd(const int32_t* packed_info, int64_t n_rays, int64_t n_samples, const float* t_starts,
                          const float* t_ends, const float* sigmas, const float* attrs, int32_t n_ch,
                          float early_stop_eps, float alpha_thre, const float* background, float* out,
                          float* opacity, float* depth, float* weights, void* stream) {
    clear_error();
    int st = validate_attrs(packed_info, n_rays, n_samples, t_starts, t_ends, sigmas, attrs, n_ch, early_stop_eps,
                            alpha_thre);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(n_rays == 0 || out != nullptr, NACC_EINVAL, "out must be non-NULL");
    if (n_rays == 0) return NACC_OK;
    const dim3 grid(static_cast<unsigned>((n_rays + kAttrRays - 1) / kAttrRays));
    hipStream_t s = as_stream(stream);
    const bool vec4 = vec4_rows(attrs, attrs, n_ch);
    auto kernel = vec4 ? (n_ch <= kBlock ? (staged_width(n_ch) ? attrs_fwd_kernel<true, 1> : attrs_fwd_kernel<true, 0>)
                                         : (staged_width(n_ch) ? attrs_fwd_kernel<true, 2> : attrs_fwd_kernel<true, 0>))
                       : attrs_fwd_kernel<false, 0>;
    hipLaunchKernelGGL(kernel, grid, dim3(kAttrThreads), 0, s, packed_info, n_rays, n_samples, t_starts, t_ends,
                       sigmas, attrs, n_ch, early_stop_eps, alpha_thre, background, out, opacity, depth, weights);
    return check_launch("render attrs fwd");
}

int nacc_render_attrs_bwd(const int32_t* packed_info, int64_t n_rays, int64_t n_samples, const float* t_starts,
                          const float* t_ends, const float* sigmas, const float* attrs, int32_t n_ch,
                          float early_stop_eps, float alpha_thre, const float* background, const float* g_out,
                          const float* g_opacity, const float* g_depth, float* g_sigmas, float* g_attrs,
                          void* stream) {
    clear_error();
    int st = validate_attrs(packed_info, n_rays, n_samples, t_starts, t_ends, sigmas, attrs, n_ch, early_stop_eps,
                            alpha_thre);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(n_rays == 0 || (g_out != nullptr && g_sigmas != nullptr && g_attrs != nullptr), NACC_EINVAL,
                 "g_out, g_sigmas and g_attrs must be non-NULL");
    if (n_rays == 0) return NACC_OK;
    const dim3 grid(static_cast<unsigned>((n_rays + kAttrRays - 1) / kAttrRays));
    hipStream_t s = as_stream(stream);
    const bool vec4 = vec4_rows(attrs, g_attrs, n_ch);
    auto kernel = vec4 ? (n_ch <= kBlock ? (staged_width(n_ch) ? attrs_bwd_kernel<true, 1> : attrs_bwd_kernel<true, 0>)
                                         : (staged_width(n_ch) ? attrs_bwd_kernel<true, 2> : attrs_bwd_kernel<true, 0>))
                       : attrs_bwd_kernel<false, 0>;
    hipLaunchKernelGGL(kernel, grid, dim3(kAttrThreads), 0, s, packed_info, n_rays, n_samples, t_starts, t_ends,
                       sigmas, attrs, n_ch, early_stop_eps, alpha_thre, background, g_out, g_opacity, g_depth,
                       g_sigmas, g_attrs);
    return check_launch("render attrs bwd");
}

}  // extern "C"
