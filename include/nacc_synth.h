/*
 * nacc_synth.h -- a synthetic radiance field for tests and benchmarks.
 *
 * NOT part of the method.  NerfAcc is field-agnostic: the user's radiance
 * field is evaluated between marching and rendering (Sec. 3, sigma_fn /
 * rgb_sigma_fn).  This analytic field stands in for that user field so the
 * library can be exercised end to end without trained weights:
 *   sigma(x) = sum_b peak_b * exp(-|x - c_b|^2 / (2 std_b^2))
 *   rgb(x)   = 1 / (1 + exp(-(W x + bias)))          (W row-major 3x3)
 * Sample positions are the FP32 midpoints x = o + d * ((t_start + t_end) * 0.5f)
 * (no fused multiply-add).  Accuracy: a few FP32 ulps of the exponent
 * arguments (relative error of sigma and rgb below 1e-5 without contraction;
 * with it, the FP32 rounding of the contracted point adds about
 * 1e-6 |d| / std^2 per blob, d the distance to the blob's centre).
 *
 * Conventions as in nacc.h: device pointers, caller-owned memory, stream as
 * void*, status codes, nacc_last_error() for messages.
 */
#ifndef NACC_SYNTH_H
#define NACC_SYNTH_H

#include <stddef.h>
#include <stdint.h>

#include "nacc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of the prepared coefficient table for n_sets * n_blobs blobs. */
int64_t nacc_synth_table_size(int32_t n_blobs, int32_t n_sets);

/* flags of nacc_synth_prepare: the scene is defined in contracted
 * coordinates, i.e. sigma and rgb are evaluated at y = x for |x| <= 1 and
 * y = (2 - 1/|x|) x / |x| beyond (FP32, Euclidean norm), as for unbounded
 * scenes (Sec. 2.1). */
#define NACC_SYNTH_CONTRACT 1

/*
 * Prepares the coefficient table (device memory of nacc_synth_table_size
 * bytes) from the blob parameters:
 *   centres float[n_sets][n_blobs][3] (one centre set per frame),
 *   stds, peaks float[n_blobs], w float[3][3], bias float[3],
 *   flags 0 or NACC_SYNTH_CONTRACT.
 */
int nacc_synth_prepare(const float* centres, const float* stds, const float* peaks, const float* w,
                       const float* bias, int32_t n_blobs, int32_t n_sets, int32_t flags, void* table,
                       void* stream);

/*
 * sigma and rgb at the midpoints of packed samples.
 *   n_rays    rays in rays_o / rays_d; samples naming another ray get 0.
 *   ray_set   int32[n_rays] centre set of each ray, or NULL for set 0.
 *   n_samples number of samples (or an upper bound when n_samples_dev is
 *             given: then only the first *n_samples_dev are evaluated).
 *   sigmas    out float[n_samples]; rgbs out float[n_samples][3] (nullable).
 */
int nacc_synth_field_samples(const void* table, int32_t n_blobs, int32_t n_sets, const float* rays_o,
                             const float* rays_d, int64_t n_rays, const int32_t* ray_set,
                             const int32_t* ray_indices,
                             const float* t_starts, const float* t_ends, int64_t n_samples,
                             const int64_t* n_samples_dev, float* sigmas, float* rgbs, void* stream);

/* sigma (and rgb, nullable) at points float[n][3].  The centre set of point
 * q is point_set[q] if point_set is given, else point_cell[q] / cells_per_set
 * if point_cell is given (cells drawn over several grids by
 * nacc_grid_sample_cells), else 0. */
int nacc_synth_field_points(const void* table, int32_t n_blobs, int32_t n_sets, const float* points,
                            const int32_t* point_set, const int32_t* point_cell, int64_t cells_per_set,
                            int64_t n, float* sigmas, float* rgbs, void* stream);

/*
 * Fused inference (Sec. 2.1 marching with early termination, Eq. 1
 * rendering, forward only): marches each ray through the occupancy grid,
 * evaluates this synthetic field at the occupied samples and renders them,
 * in one kernel, without writing the samples out.  For fields that can be
 * evaluated inside the kernel only (this one).
 *   Arguments as in nacc_march_count / nacc_march_fill (rays_o, rays_d,
 *   grid_id nullable, grid_bits, grid_skip nullable, grid, params) and
 *   nacc_synth_field_samples (table, n_blobs, n_sets, ray_set nullable);
 *   uniform steps only (params->cone must be 0, else NACC_ENOTSUP).  With
 *   a skip buffer the box lookup marches by the segments of its halo bits
 *   (the sample set is the same); the other lookups ignore it.
 *   early_stop_eps  as in nacc_render_fwd (0 disables the cut).
 *   color float[n_rays][3], opacity, depth float[n_rays]: outputs as from
 *   nacc_render_fwd; kept int32[n_rays] (nullable): samples before the cut.
 *   clocks  uint64[ceil(n_rays / 64)][2] (nullable): for each group of 64
 *           consecutive rays (rendered by one workgroup), the device wall
 *           clock (hipDeviceAttributeWallClockRate, kHz) when its workgroup
 *           started and when the group's last ray was finished, so that a
 *           caller rendering several images in one launch can tell when
 *           each image was done.
 * The samples are those nacc_march_fill would write and the chunks those
 * nacc_render_fwd would read, so the outputs equal, bit for bit, marching,
 * then nacc_synth_field_samples, then nacc_render_fwd.  Marching stops at
 * the early-termination cut.  Errors: NACC_EINVAL / NACC_ESHAPE for invalid
 * arguments (checked on the host before any launch), NACC_EHIP for a
 * failed launch.
 */
int nacc_synth_render_fused(const void* table, int32_t n_blobs, int32_t n_sets, const int32_t* ray_set,
                            const float* rays_o, const float* rays_d, const int32_t* grid_id, int64_t n_rays,
                            const uint32_t* grid_bits, const uint8_t* grid_skip,
                            const nacc_grid_desc* grid, const nacc_march_params* params,
                            float early_stop_eps, float* color, float* opacity, float* depth,
                            int32_t* kept, uint64_t* clocks, void* stream);

/* Frequency (kHz) of the device wall clock the clocks output above counts,
 * for device `device`; a negative status if the runtime cannot say. */
int64_t nacc_wall_clock_khz(int32_t device);

/*
 * The two field evaluations above as stages of a step plan (nacc_plan.h):
 * each *_stage_run has the nacc_stage_fn signature and takes a pointer to
 * its struct (which must outlive the plan) as `user`; the struct's fields
 * are the arguments of the call of the same name.  The samples stage
 * evaluates the first *n_samples_dev samples (required: the plan's total).
 */
typedef struct nacc_synth_samples_stage {
    const void* table;
    int32_t n_blobs;
    int32_t n_sets;
    const float* rays_o;
    const float* rays_d;
    int64_t n_rays;
    const int32_t* ray_set;
    const int32_t* ray_indices;
    const float* t_starts;
    const float* t_ends;
    int64_t n_samples;
    const int64_t* n_samples_dev;
    float* sigmas;
    float* rgbs;
} nacc_synth_samples_stage;

typedef struct nacc_synth_points_stage {
    const void* table;
    int32_t n_blobs;
    int32_t n_sets;
    const float* points;
    const int32_t* point_set;
    const int32_t* point_cell;
    int64_t cells_per_set;
    int64_t n;
    float* sigmas;
    float* rgbs;
} nacc_synth_points_stage;

int nacc_synth_samples_stage_run(void* stage, void* stream);
int nacc_synth_points_stage_run(void* stage, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NACC_SYNTH_H */
