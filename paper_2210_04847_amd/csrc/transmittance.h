// Transmittance, opacity and the early-termination cut of one chunk of 64
// samples (Eq. 1; Sec. 2.1 early termination), shared by the rendering
// kernels and the fused inference kernel so that all of them weight a
// sample bit for bit alike.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace nacc {
namespace vr {

using namespace nacc::dev;

constexpr float kLog2e = 1.4426950408889634f;

// e^-x for x >= 0 on the hardware exp2 (relative error a few ulp).
__device__ __forceinline__ float exp_neg(float x) { return __builtin_amdgcn_exp2f(-x * kLog2e); }

// alpha = 1 - e^-tau without cancellation: for tau <= 1/4, tau times the
// Taylor series of (1 - e^-tau) / tau = sum_k (-tau)^k / (k + 1)! through
// k = 5, in Horner form with fused multiply-adds (truncation below
// tau^6 / 5040 < 5e-8 relative, rounding a few ulp); above it 1 - e^-tau
// directly (e^-tau <= 0.78, so the subtraction loses at most a few ulp).
__device__ __forceinline__ float alpha_of(float tau) {
    if (tau <= 0.25f) {
        float p = __builtin_fmaf(tau, -1.0f / 720.0f, 1.0f / 120.0f);
        p = __builtin_fmaf(p, tau, -1.0f / 24.0f);
        p = __builtin_fmaf(p, tau, 1.0f / 6.0f);
        p = __builtin_fmaf(p, tau, -0.5f);
        p = __builtin_fmaf(p, tau, 1.0f);
        return tau * p;
    }
    return 1.0f - exp_neg(tau);
}

// Transmittance of each lane's sample in a chunk, given the FP64 prefix of
// tau before the chunk: T_i = e^-carry * e^-(exclusive chunk prefix).  The
// chunk factor comes from the FP64 carry rounded once to FP32, the lane
// factor from a short FP32 prefix inside the chunk; relative error about
// (carry + chunk prefix) * log2(e) * 2^-24 plus a few ulp.
struct Trans {
    float tau;     // sigma * delta
    float incl;    // inclusive prefix of tau inside the chunk
    float t_in;    // T_i
    float t_next;  // T_{i+1}
};

// The value of the lane below, 1 in lane 0.
__device__ __forceinline__ float shift_up_one_or_one(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, 1.0f),
                                                                 __builtin_bit_cast(int, x), kWaveShr1, 0xf, 0xf,
                                                                 false));
}

__device__ __forceinline__ Trans transmittance_of(float tau, double carry) {
    Trans t;
    t.tau = tau;
    t.incl = wave_inclusive_sum(t.tau);
    const float t0 = uniform<float>(exp_neg(static_cast<float>(carry)));
    // lane i's exclusive prefix is lane i-1's inclusive one (0 in lane 0,
    // where e^-0 = 1), so e^-excl is the neighbour's e^-incl, bit for bit
    const float e_incl = exp_neg(t.incl);
    t.t_in = t0 * shift_up_one_or_one(e_incl);
    t.t_next = t0 * e_incl;
    return t;
}

// Sums over the 64 lanes of a ray's accumulators (colour, opacity, depth,
// attribute channels) in one fixed association, the same for every value
// whatever its slot, so that every rendering kernel produces the same bits:
// lanes i and i + 32 are added (i < 32), then of those i and i + 16
// (i < 16), then the 16 partial sums by the row scan's tree (lane 15 of the
// row).  gfx950's lane swaps (v_permlane32_swap: the upper half of the
// first register with the lower half of the second; v_permlane16_swap: the
// odd rows of the first with the even rows of the second) place the halves
// of two values side by side, so that one addition folds both: four values
// cost the folds of one.
__device__ __forceinline__ uint32_t as_bits(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ float as_float(uint32_t x) { return __builtin_bit_cast(float, x); }

// Tree sum of each row of 16 lanes, in its lane 15.
__device__ __forceinline__ float row_tree(float x) {
    x = x + dpp<kRowShr1>(x);
    x = x + dpp<kRowShr2>(x);
    x = x + dpp<kRowShr4>(x);
    x = x + dpp<kRowShr8>(x);
    return x;
}

__device__ __forceinline__ void wave_sum4(float& a, float& b, float& c, float& d) {
    const auto ab = __builtin_amdgcn_permlane32_swap(as_bits(a), as_bits(b), false, false);
    const float s1 = as_float(ab[0]) + as_float(ab[1]);  // lanes < 32: a, else b
    const auto cd = __builtin_amdgcn_permlane32_swap(as_bits(c), as_bits(d), false, false);
    const float s2 = as_float(cd[0]) + as_float(cd[1]);  // lanes < 32: c, else d
    const auto q = __builtin_amdgcn_permlane16_swap(as_bits(s1), as_bits(s2), false, false);
    const float t = row_tree(as_float(q[0]) + as_float(q[1]));  // rows: a, c, b, d
    a = read_lane(t, 15);
    c = read_lane(t, 31);
    b = read_lane(t, 47);
    d = read_lane(t, 63);
}

__device__ __forceinline__ float wave_sum1(float x) {
    const auto h = __builtin_amdgcn_permlane32_swap(as_bits(x), as_bits(x), false, false);
    const float y = as_float(h[0]) + as_float(h[1]);
    const auto q = __builtin_amdgcn_permlane16_swap(as_bits(y), as_bits(y), false, false);
    return read_lane(row_tree(as_float(q[0]) + as_float(q[1])), 15);
}

// Number of leading lanes kept in this chunk: the first valid lane with
// T < eps and every lane after it are cut (64 = no cut here).
__device__ __forceinline__ int chunk_keep(bool valid, float t_in, float eps) {
    if (!(eps > 0.0f)) return kWave;
    const uint64_t m = ballot(valid && t_in < eps);
    return m == 0 ? kWave : static_cast<int>(__builtin_ctzll(m));
}

// The same for a chunk whose first n_valid > 0 lanes hold samples (n_valid
// wave-uniform): the valid lanes' mask is formed in scalar registers.
__device__ __forceinline__ int chunk_keep_n(int n_valid, float t_in, float eps) {
    if (!(eps > 0.0f)) return kWave;
    const uint64_t valid = n_valid >= kWave ? ~0ull : (1ull << n_valid) - 1ull;
    const uint64_t m = ballot(t_in < eps) & valid;
    return m == 0 ? kWave : static_cast<int>(__builtin_ctzll(m));
}

// The ray's sample range from packed_info; a range that does not lie inside
// [0, n_samples) is treated as an empty ray, so no access leaves the arrays.
__device__ __forceinline__ void ray_range(const int32_t* __restrict__ packed_info, int64_t r, int64_t n_samples,
                                          int64_t& start, int& n) {
    const int s0 = uniform<int>(packed_info[2 * r]);
    const int c0 = uniform<int>(packed_info[2 * r + 1]);
    const bool ok = s0 >= 0 && c0 >= 0 && static_cast<int64_t>(s0) + c0 <= n_samples;
    start = ok ? s0 : 0;
    n = ok ? c0 : 0;
}

}  // namespace vr
}  // namespace nacc
