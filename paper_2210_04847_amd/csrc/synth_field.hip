// Synthetic Gaussian-blob radiance field (test and benchmark input only; it
// stands in for the user's field of Sec. 3 and is not part of the method).
// The coefficient table and its evaluation are in blob_field.h.
#include <cmath>

#include "blob_field.h"
#include "common.h"
#include "nacc_synth.h"

namespace {

using namespace nacc;
using namespace nacc::blob;
using namespace nacc::dev;

constexpr int kThreads = 256;

__global__ void prepare_kernel(const float* __restrict__ centres, const float* __restrict__ stds,
                               const float* __restrict__ peaks, const float* __restrict__ w,
                               const float* __restrict__ bias, int32_t n_blobs, int32_t n_sets,
                               int32_t flags, float* __restrict__ table) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nb = static_cast<int64_t>(n_sets) * n_blobs;
    if (i < nb) {
        const int b = static_cast<int>(i % n_blobs);
        const float s = stds[b];
        float* e = table + kBlobStride * i;
        e[0] = centres[3 * i];
        e[1] = centres[3 * i + 1];
        e[2] = centres[3 * i + 2];
        e[3] = -kLog2e / (2.0f * s * s);
        e[4] = peaks[b];
    } else if (i < nb + 13) {
        const int j = static_cast<int>(i - nb);
        table[kBlobStride * nb + j] = j < 9 ? w[j] : (j < 12 ? bias[j - 9] : static_cast<float>(flags & 1));
    }
}

// With a single centre set (PER_SET false) every lane reads the same blob
// parameters, which the compiler then fetches with scalar loads.
template <bool PER_SET>
__global__ __launch_bounds__(kThreads) void field_samples_kernel(
    const float* __restrict__ table, int n_blobs, int n_sets, const float* __restrict__ rays_o,
    const float* __restrict__ rays_d, int64_t n_rays, const int32_t* __restrict__ ray_set,
    const int32_t* __restrict__ ray_indices,
    const float* __restrict__ ts, const float* __restrict__ te, int64_t n_cap, const int64_t* __restrict__ n_dev,
    float* __restrict__ sigmas, float* __restrict__ rgbs) {
    const int64_t n = n_dev != nullptr ? min(n_cap, *n_dev) : n_cap;
    const float* cc = table + static_cast<int64_t>(n_sets) * n_blobs * kBlobStride;
    const bool contract = cc[12] != 0.0f;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    for (int64_t s = xcd_grouped<16>(blockIdx.x, gridDim.x) * kThreads + threadIdx.x; s < n; s += stride) {
        const int64_t r = ray_indices[s];
        if (r < 0 || r >= n_rays) {
            sigmas[s] = 0.0f;
            if (rgbs != nullptr) rgbs[3 * s] = rgbs[3 * s + 1] = rgbs[3 * s + 2] = 0.0f;
            continue;
        }
        const float t0 = ts[s], t1 = te[s];
        float x0 = midpoint_coord(rays_o[3 * r], rays_d[3 * r], t0, t1);
        float x1 = midpoint_coord(rays_o[3 * r + 1], rays_d[3 * r + 1], t0, t1);
        float x2 = midpoint_coord(rays_o[3 * r + 2], rays_d[3 * r + 2], t0, t1);
        to_scene(contract, x0, x1, x2);
        int set = 0;
        if (PER_SET) {
            set = ray_set[r];
            set = set < 0 ? 0 : (set >= n_sets ? n_sets - 1 : set);
        }
        float sigma;
        eval_field(table, n_blobs, set, x0, x1, x2, sigma);
        sigmas[s] = sigma;
        if (rgbs != nullptr) {
            float cr, cg, cb;
            eval_rgb(cc, x0, x1, x2, cr, cg, cb);
            rgbs[3 * s] = cr;
            rgbs[3 * s + 1] = cg;
            rgbs[3 * s + 2] = cb;
        }
    }
}

// Centre set per point: point_set[q], or point_cell[q] / cells_per_set when
// the points were drawn as cells of several grids.
template <bool PER_SET>
__global__ __launch_bounds__(kThreads) void field_points_kernel(const float* __restrict__ table, int n_blobs,
                                                                 int n_sets, const float* __restrict__ points,
                                                                 const int32_t* __restrict__ point_set,
                                                                 const int32_t* __restrict__ point_cell,
                                                                 int64_t cells_per_set, int64_t n,
                                                                 float* __restrict__ sigmas,
                                                                 float* __restrict__ rgbs) {
    const float* cc = table + static_cast<int64_t>(n_sets) * n_blobs * kBlobStride;
    const bool contract = cc[12] != 0.0f;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; q < n; q += stride) {
        float x0 = points[3 * q], x1 = points[3 * q + 1], x2 = points[3 * q + 2];
        to_scene(contract, x0, x1, x2);
        int set = 0;
        if (PER_SET) {
            set = point_set != nullptr ? point_set[q] : static_cast<int>(point_cell[q] / cells_per_set);
            set = set < 0 ? 0 : (set >= n_sets ? n_sets - 1 : set);
        }
        float sigma;
        eval_field(table, n_blobs, set, x0, x1, x2, sigma);
        sigmas[q] = sigma;
        if (rgbs != nullptr) {
            float cr, cg, cb;
            eval_rgb(cc, x0, x1, x2, cr, cg, cb);
            rgbs[3 * q] = cr;
            rgbs[3 * q + 1] = cg;
            rgbs[3 * q + 2] = cb;
        }
    }
}

unsigned field_blocks(int64_t n) {
    const int64_t want = (n + kThreads - 1) / kThreads;
    return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(want, 256 * 16)));
}

}  // namespace

extern "C" {

int64_t nacc_synth_table_size(int32_t n_blobs, int32_t n_sets) {
    if (n_blobs < 1 || n_sets < 1) return -1;
    return table_floats(n_blobs, n_sets) * static_cast<int64_t>(sizeof(float));
}

int nacc_synth_prepare(const float* centres, const float* stds, const float* peaks, const float* w, const float* bias,
                       int32_t n_blobs, int32_t n_sets, int32_t flags, void* table, void* stream) {
    clear_error();
    NACC_REQUIRE(n_blobs >= 1 && n_sets >= 1, NACC_EINVAL, "n_blobs and n_sets must be >= 1");
    NACC_REQUIRE(centres && stds && peaks && w && bias && table, NACC_EINVAL, "arguments must be non-NULL");
    NACC_REQUIRE((flags & ~NACC_SYNTH_CONTRACT) == 0, NACC_EINVAL, "unknown flags 0x%x", flags);
    const int64_t total = static_cast<int64_t>(n_sets) * n_blobs + 13;
    hipLaunchKernelGGL(prepare_kernel, dim3(static_cast<unsigned>((total + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, as_stream(stream), centres, stds, peaks, w, bias, n_blobs, n_sets,
                       flags, static_cast<float*>(table));
    return check_launch("synth prepare");
}

int nacc_synth_field_samples(const void* table, int32_t n_blobs, int32_t n_sets, const float* rays_o,
                             const float* rays_d, int64_t n_rays, const int32_t* ray_set,
                             const int32_t* ray_indices,
                             const float* t_starts, const float* t_ends, int64_t n_samples,
                             const int64_t* n_samples_dev, float* sigmas, float* rgbs, void* stream) {
    clear_error();
    NACC_REQUIRE(n_blobs >= 1 && n_sets >= 1, NACC_EINVAL, "n_blobs and n_sets must be >= 1");
    NACC_REQUIRE(n_samples >= 0, NACC_EINVAL, "n_samples < 0");
    NACC_REQUIRE(n_samples == 0 || (table && rays_o && rays_d && ray_indices && t_starts && t_ends && sigmas),
                 NACC_EINVAL, "arguments must be non-NULL");
    if (n_samples == 0) return NACC_OK;
    auto kernel = ray_set != nullptr ? field_samples_kernel<true> : field_samples_kernel<false>;
    hipLaunchKernelGGL(kernel, dim3(field_blocks(n_samples)), dim3(kThreads), 0, as_stream(stream),
                       static_cast<const float*>(table), n_blobs, n_sets, rays_o, rays_d, n_rays, ray_set,
                       ray_indices,
                       t_starts, t_ends, n_samples, n_samples_dev, sigmas, rgbs);
    return check_launch("synth field samples");
}

int nacc_synth_field_points(const void* table, int32_t n_blobs, int32_t n_sets, const float* points,
                            const int32_t* point_set, const int32_t* point_cell, int64_t cells_per_set, int64_t n,
                            float* sigmas, float* rgbs, void* stream) {
    clear_error();
    NACC_REQUIRE(n_blobs >= 1 && n_sets >= 1, NACC_EINVAL, "n_blobs and n_sets must be >= 1");
    NACC_REQUIRE(n >= 0, NACC_EINVAL, "n < 0");
    NACC_REQUIRE(n == 0 || (table && points && sigmas), NACC_EINVAL, "arguments must be non-NULL");
    NACC_REQUIRE(point_cell == nullptr || cells_per_set > 0, NACC_EINVAL, "cells_per_set must be > 0");
    if (n == 0) return NACC_OK;
    const bool per_set = point_set != nullptr || point_cell != nullptr;
    auto kernel = per_set ? field_points_kernel<true> : field_points_kernel<false>;
    hipLaunchKernelGGL(kernel, dim3(field_blocks(n)), dim3(kThreads), 0, as_stream(stream),
                       static_cast<const float*>(table), n_blobs, n_sets, points, point_set, point_cell,
                       cells_per_set, n, sigmas, rgbs);
    return check_launch("synth field points");
}

int nacc_synth_samples_stage_run(void* stage, void* stream) {
    clear_error();
    NACC_REQUIRE(stage != nullptr, NACC_EINVAL, "stage must be non-NULL");
    const auto* a = static_cast<const nacc_synth_samples_stage*>(stage);
    NACC_REQUIRE(a->n_samples_dev != nullptr, NACC_EINVAL, "the samples stage needs n_samples_dev");
    return nacc_synth_field_samples(a->table, a->n_blobs, a->n_sets, a->rays_o, a->rays_d, a->n_rays, a->ray_set,
                                    a->ray_indices, a->t_starts, a->t_ends, a->n_samples, a->n_samples_dev,
                                    a->sigmas, a->rgbs, stream);
}

int nacc_synth_points_stage_run(void* stage, void* stream) {
    clear_error();
    NACC_REQUIRE(stage != nullptr, NACC_EINVAL, "stage must be non-NULL");
    const auto* a = static_cast<const nacc_synth_points_stage*>(stage);
    return nacc_synth_field_points(a->table, a->n_blobs, a->n_sets, a->points, a->point_set, a->point_cell,
                                   a->cells_per_set, a->n, a->sigmas, a->rgbs, stream);
}

}  // extern "C"
