/*
 * nacc_plan.h -- step plans: one training (or rendering) step of the
 * method, described once, launched eagerly or replayed as a HIP graph, with
 * its launch parameters tuned on the step itself.
 *
 * A step is the sequence of Sec. 3 (the example training loop): marching
 * through the occupancy grid (nacc_march_count, nacc_march_fill), the
 * caller's radiance field at the marched samples, then differentiable
 * rendering with the loss and its backward (nacc_render_fwd_bwd_mse) or
 * forward rendering alone (nacc_render_fwd), then optionally more of the
 * caller's work (the field's backward, an optimiser).  The occupancy grid
 * update of Sec. 2.1 (decay, fresh densities at random cells, threshold;
 * every few steps) is a second, optional sequence of the same plan.
 *
 * Ownership.  Every array named in nacc_plan_desc is device memory owned by
 * the caller and must stay valid, at the same address, for the plan's
 * lifetime; a captured graph holds the addresses.  The plan owns the
 * marching and loss workspaces, a HIP stream for capture and tuning, and
 * the graphs; nacc_plan_destroy frees them.  Creating a plan allocates
 * device memory (hipMalloc); launching one does not.
 *
 * Stages.  The caller's work enters as nacc_stage_fn callbacks, called on
 * the host thread that launches or captures, in step order, with the stream
 * the step runs on.  A stage enqueues its work on that stream and returns
 * 0, or a nonzero status that ends the step with that status.  During
 * capture the stream is capturing: a stage must not synchronise, allocate,
 * copy synchronously or record hipMemsetAsync (use a fill kernel), and must
 * enqueue all of its device work on the given stream.  A stage reads the
 * sample count from the device (`total`), never from the host.
 *
 * Threads and devices.  A plan is not thread-safe; calls on it must come
 * from one thread at a time, with the device that created it current
 * (NACC_EINVAL otherwise).  Graph replays on different streams, or a replay
 * concurrent with an eager step of the same plan, race on the plan's
 * buffers.
 */
#ifndef NACC_PLAN_H
#define NACC_PLAN_H

#include <stddef.h>
#include <stdint.h>

#include "nacc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* A stage of the caller's: enqueue work on `stream` (a hipStream_t),
 * return 0 or a nonzero status. */
typedef int (*nacc_stage_fn)(void* user, void* stream);

/*
 * One step, as the entry points of nacc.h take it.
 *   rays_o, rays_d, grid_id, n_rays, grid_bits, grid_skip, grid, params
 *       as for nacc_march_count (grid_id and grid_skip may be NULL).
 *   capacity  length of ray_indices, t_starts, t_ends, sigmas, rgbs,
 *       g_sigmas, g_rgbs (rgbs and g_rgbs: capacity rows of 3);
 *       n_rays * nacc_march_max_samples_per_ray(grid, params) samples never
 *       overflow; fewer make *status report NACC_ECAPACITY when a step
 *       overflows (rendering then reads only the samples that fit).
 *   packed_info, ray_indices, t_starts, t_ends, total, status
 *       the marching outputs (status may be NULL).
 *   field, field_user  writes sigmas[0, *total) and rgbs[0, *total) for
 *       the marched samples (required).
 *   sigmas, rgbs  the field's outputs, read by rendering.
 *   early_stop_eps  as for nacc_render_fwd.
 *   target    float[n_rays][3]: training step with the MSE loss
 *       (nacc_render_fwd_bwd_mse, mean over loss_rays, 0 = n_rays), writing
 *       g_sigmas, g_rgbs and loss; NULL: forward rendering only
 *       (nacc_render_fwd), and g_sigmas, g_rgbs, loss are not used.
 *   color, opacity, depth  rendering outputs (required).
 *   after, after_user  optional stage run last (e.g. the field's backward).
 * Grid update (all ignored when occ is NULL):
 *   occ       float[n_cells], n_cells = n_grids * res^3: the density grid
 *       grid_bits is packed from; update_cells cells are drawn per update.
 *   decay, threshold, seed  as for nacc_grid_decay, nacc_grid_pack and
 *       nacc_grid_sample_cells.
 *   update_counter  uint64[1] on the device: the update number, read by the
 *       cell draw and incremented by each update (set it to resume).
 *   update_cell_ids int32[update_cells], update_positions
 *       float[update_cells][3], update_values float[update_cells]: the drawn
 *       cells, their jittered points, and the densities there.
 *   update_field, update_field_user  writes update_values from
 *       update_positions (and update_cell_ids) (required with occ).
 * An update runs decay, draw, update_field, max update, pack, and rebuilds
 * grid_skip (when given) from the new bits.
 */
typedef struct nacc_plan_desc {
    const float* rays_o;
    const float* rays_d;
    const int32_t* grid_id;
    int64_t n_rays;
    uint32_t* grid_bits;
    uint8_t* grid_skip;
    nacc_grid_desc grid;
    nacc_march_params params;
    int64_t capacity;
    int32_t* packed_info;
    int32_t* ray_indices;
    float* t_starts;
    float* t_ends;
    int64_t* total;
    int32_t* status;
    nacc_stage_fn field;
    void* field_user;
    const float* sigmas;
    const float* rgbs;
    float early_stop_eps;
    const float* target;
    int64_t loss_rays;
    float* color;
    float* opacity;
    float* depth;
    float* g_sigmas;
    float* g_rgbs;
    float* loss;
    nacc_stage_fn after;
    void* after_user;
    float* occ;
    float decay;
    float threshold;
    uint64_t seed;
    int64_t update_cells;
    uint64_t* update_counter;
    int32_t* update_cell_ids;
    float* update_positions;
    float* update_values;
    nacc_stage_fn update_field;
    void* update_field_user;
} nacc_plan_desc;

typedef struct nacc_plan nacc_plan;

/*
 * Validates `desc` on the host (NACC_EINVAL / NACC_ESHAPE with a message,
 * nothing allocated), then allocates the plan and its workspaces on the
 * current device (NACC_EHIP if that fails).  *out is set only on success.
 */
int nacc_plan_create(const nacc_plan_desc* desc, nacc_plan** out);

/* Frees the plan, its workspaces, stream and graphs (after waiting for its
 * own stream).  NULL is accepted.  Work the caller enqueued on other
 * streams that uses the plan must have finished. */
int nacc_plan_destroy(nacc_plan* plan);

/* Enqueues one step eagerly on `stream` (NULL = the default stream), with
 * the process's current nacc_tuning. */
int nacc_plan_step(nacc_plan* plan, void* stream);

/* Enqueues one grid update eagerly on `stream`; NACC_EINVAL if the plan has
 * no update (occ NULL). */
int nacc_plan_update(nacc_plan* plan, void* stream);

/*
 * Captures the step (and the update, if the plan has one) into HIP graphs
 * on the plan's own stream, with the current nacc_tuning, replacing any
 * earlier capture.  Synchronous: returns when the graphs are instantiated.
 * Stages run once, capturing.  Nothing is executed on the device.
 */
int nacc_plan_capture_step(nacc_plan* plan);

/* Replays the captured step on `stream`, then the captured update when
 * with_update != 0.  NACC_EINVAL before nacc_plan_capture_step. */
int nacc_plan_launch(nacc_plan* plan, int32_t with_update, void* stream);

/*
 * Tunes the launch parameters (nacc_tuning) on this step: two rounds of
 * coordinate descent over every knob, each setting captured and timed over
 * `repeats` graph replays (>= 1) after two warm-up replays, and accepted
 * only if a checksum of every word of the step's outputs (packed_info,
 * total, color, opacity, depth, all marched samples and, when training,
 * their gradients) equals that of the starting setting.  Synchronous; it
 * waits for `stream` first.
 * Runs steps (not updates) on the device, overwriting the step's outputs.
 * Leaves the best setting as the process's nacc_tuning, writes it to *best
 * (nullable) and its time per step to *best_ms (nullable), and re-captures
 * the plan's graphs if it had any.
 */
int nacc_plan_autotune(nacc_plan* plan, int32_t repeats, void* stream, nacc_tuning* best,
                       float* best_ms);

#ifdef __cplusplus
}
#endif

#endif /* NACC_PLAN_H */
