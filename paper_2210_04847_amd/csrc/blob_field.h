// The synthetic Gaussian-blob field's device code (test and benchmark input,
// standing in for the user's radiance field), shared by the field kernels
// and the fused inference kernel, which must evaluate it bit for bit alike.
//
// The coefficient table holds, per blob, (c_x, c_y, c_z, k, peak) with
// k = -log2(e) / (2 std^2), so each blob costs one exp2 on the hardware
// transcendental unit; the 9 + 3 colour coefficients follow the blobs, then
// the flags word (1.0f: the scene is defined in contracted coordinates).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace nacc {
namespace blob {

constexpr int kBlobStride = 5;
constexpr float kLog2e = 1.4426950408889634f;

inline int64_t table_floats(int32_t n_blobs, int32_t n_sets) {
    return static_cast<int64_t>(n_sets) * n_blobs * kBlobStride + 13;
}

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ void eval_field(const float* __restrict__ table, int n_blobs, int set, float x0, float x1,
                                           float x2, float& sigma) {
    const float* blob = table + static_cast<int64_t>(set) * n_blobs * kBlobStride;
    float acc = 0.0f;
#pragma unroll 4
    for (int b = 0; b < n_blobs; ++b) {
        const float dx = x0 - blob[kBlobStride * b];
        const float dy = x1 - blob[kBlobStride * b + 1];
        const float dz = x2 - blob[kBlobStride * b + 2];
        const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        acc = fmaf(blob[kBlobStride * b + 4], exp2_fast(d2 * blob[kBlobStride * b + 3]), acc);
    }
    sigma = acc;
}

__device__ __forceinline__ void eval_rgb(const float* __restrict__ cc, float x0, float x1, float x2, float& r,
                                         float& g, float& b) {
    const float z0 = fmaf(cc[0], x0, fmaf(cc[1], x1, fmaf(cc[2], x2, cc[9])));
    const float z1 = fmaf(cc[3], x0, fmaf(cc[4], x1, fmaf(cc[5], x2, cc[10])));
    const float z2 = fmaf(cc[6], x0, fmaf(cc[7], x1, fmaf(cc[8], x2, cc[11])));
    r = 1.0f / (1.0f + exp2_fast(-z0 * kLog2e));
    g = 1.0f / (1.0f + exp2_fast(-z1 * kLog2e));
    b = 1.0f / (1.0f + exp2_fast(-z2 * kLog2e));
}

// Sample midpoint, FP32, no fused multiply-add (matches the positions of the
// tests).
__device__ __forceinline__ float midpoint_coord(float o, float d, float t0, float t1) {
#pragma clang fp contract(off)
    const float tm = (t0 + t1) * 0.5f;
    return o + d * tm;
}

// Scene coordinates of a world point when the scene is defined in
// contracted space: beyond the unit ball, x -> (2 - 1/|x|) x / |x|.
__device__ __forceinline__ void to_scene(bool contract, float& x0, float& x1, float& x2) {
    if (!contract) return;
    const float n2 = fmaf(x2, x2, fmaf(x1, x1, x0 * x0));
    if (n2 > 1.0f) {
        const float n = sqrtf(n2);
        const float f = (2.0f - 1.0f / n) / n;
        x0 *= f;
        x1 *= f;
        x2 *= f;
    }
}

}  // namespace blob
}  // namespace nacc
