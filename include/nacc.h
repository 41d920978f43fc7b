/*
 * nacc.h -- C ABI of the MI355X (gfx950) library for occupancy-grid ray
 * marching and packed differentiable volume rendering, after NerfAcc
 * (Li, Tancik, Kanazawa, arXiv 2210.04847).
 *
 * The calls follow the paper's two-step statement of the problem (Sec. 2):
 * ray marching emits ragged samples, then differentiable rendering
 * accumulates them along each ray.  Between the two the caller evaluates its
 * own radiance field (Sec. 3: sigma_fn / rgb_sigma_fn); callbacks never cross
 * this boundary.
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers to contiguous memory owned by
 *     the caller, unless stated otherwise.  The library allocates nothing in
 *     these calls and keeps no pointer after returning.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued asynchronously on it; nothing blocks the host unless
 *     stated.
 *   - Arguments are validated on the host before anything is launched.  A
 *     call returns NACC_OK (0) or a negative status; it never aborts or
 *     throws.  nacc_last_error() returns a message for the calling thread's
 *     most recent failure.
 *   - Ray and sample counts are int64; ray_indices and packed_info entries are
 *     int32, so a call whose sample total would exceed 2^31-1 is rejected
 *     (NACC_ECAPACITY).
 *   - Floating point is IEEE FP32.  Marching follows the FP32 lattice
 *     contract written out below, so its sample sets are reproducible
 *     bit for bit on any IEEE machine.
 *
 * Packed sample layout (Sec. 3, the ragged outputs of ray_marching):
 *   packed_info  int32[n_rays][2]: (first sample index, sample count) of
 *                each ray; rays are stored consecutively in ray order.
 *   ray_indices  int32[n_samples]: the ray of each sample.
 *   t_starts, t_ends  float[n_samples]: the sample interval along the ray;
 *                within a ray the intervals are in increasing t and adjacent
 *                candidates share endpoints bit for bit.
 *   sigmas       float[n_samples]: post-activation density.
 *   rgbs         float[n_samples][3]: post-activation colour.
 *
 * FP32 lattice contract (our reading of Sec. 2.1; the paper states the
 * method, not the formulae):
 *   clip   per axis i with d_i != 0: ta = (lo_i - o_i) / d_i,
 *          tb = (hi_i - o_i) / d_i, tmin_i = min(ta, tb),
 *          tmax_i = max(ta, tb); an axis with d_i == 0 imposes nothing when
 *          lo_i <= o_i <= hi_i and otherwise the ray misses.
 *          t_near = max(max_i tmin_i, near_plane),
 *          t_far = min(min_i tmax_i, far_plane); hit iff t_near < t_far.
 *   steps  uniform (cone == 0): t_k = t_near + (float)k * dt.
 *          cone (cone > 0): t_0 = t_near,
 *          t_{k+1} = t_k + min(max(t_k * cone, dt), dt_max).
 *          Candidate k exists while t_k < t_far and k < 2^24 (cone: also
 *          while t_{k+1} > t_k).  Its interval is [t_k, t_{k+1}], not
 *          clamped to t_far.
 *   point  t_m = (t_k + t_{k+1}) * 0.5f, x_i = o_i + d_i * t_m.
 *   cell   u_i = (x_i - lo_i) * s_i, s_i = fl32(res / (hi_i - lo_i)) (FP64
 *          quotient rounded once); j_i = floor(min(max(u_i, 0), res - 1));
 *          cell = (j_0 * res + j_1) * res + j_2 (x-major, C order);
 *          occupied iff bit (cell & 31) of word bits[cell >> 5] is set.
 *   Each operation above is one correctly rounded FP32 operation, with no
 *   fused multiply-add.
 */
#ifndef NACC_H
#define NACC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
    NACC_OK = 0,
    NACC_EINVAL = -1,    /* a null pointer, a negative size, a bad mode */
    NACC_ESHAPE = -2,    /* sizes inconsistent with each other */
    NACC_ECAPACITY = -3, /* an output would not fit its buffer or int32 */
    NACC_EHIP = -4,      /* the HIP runtime reported an error */
    NACC_ENOTSUP = -5    /* a valid request the library does not support */
};

/* Grid lookup modes. */
enum {
    NACC_LOOKUP_AABB = 0,     /* grid over the box [lo, hi]; the box is also
                                 the clip box */
    NACC_LOOKUP_CASCADE = 1,  /* n_grids nested grids over [-b,b]^3 * 2^l
                                 (multi-scale grids, Sec. 2.1 footnote); the
                                 clip box is the largest one */
    NACC_LOOKUP_CONTRACT = 2  /* scene contraction x -> (2 - 1/|x|) x/|x|
                                 for |x| > 1 before the lookup (Sec. 2.1,
                                 "Scene Contraction"); no clip box */
};

/*
 * Occupancy grid description (Sec. 2.1, "Pruning Empty and Occluded
 * Regions": a binary grid cached and updated during training).
 * The bit array has n_grids * res^3 bits, grid g occupying words
 * [g * res^3 / 32, (g+1) * res^3 / 32); all grids together at most
 * 2^31 - 1 bytes (NACC_ESHAPE otherwise).
 *   lo, hi   AABB and CONTRACT: the box the grid covers.  CASCADE: the
 *            level-0 cube, lo = -b, hi = +b on every axis, b a power of two;
 *            level l covers [-b 2^l, b 2^l]^3, and a point goes to the
 *            smallest level that holds it (max_i |x_i| <= b 2^l), the last
 *            level holding everything else.
 *   res      cells per axis; res^3 must be a multiple of 32; res <= 1024.
 *   n_grids  AABB/CONTRACT: grids selectable per ray by grid_id;
 *            CASCADE: number of levels (1..16).
 *   lookup   NACC_LOOKUP_*.
 */
typedef struct nacc_grid_desc {
    float lo[3];
    float hi[3];
    int32_t res;
    int32_t n_grids;
    int32_t lookup;
    int32_t reserved;
} nacc_grid_desc;

/*
 * Marching parameters (Sec. 3, ray_marching's near_plane / far_plane and
 * the render step size; cone stepping for large scenes).
 *   near_plane, far_plane  the t range before the clip.
 *   dt        uniform step (cone == 0) or the smallest cone step; > 0.
 *   dt_max    largest cone step (ignored when cone == 0); >= dt.
 *   cone      0 for uniform steps; > 0 scales the step with t.
 *   max_per_ray  0 for no cap; otherwise each ray keeps only its first
 *             max_per_ray samples.
 */
typedef struct nacc_march_params {
    float near_plane;
    float far_plane;
    float dt;
    float dt_max;
    float cone;
    int32_t max_per_ray;
} nacc_march_params;

/* Library version string; never NULL. */
const char* nacc_version(void);

/*
 * Launch parameters that change speed, never results: every setting
 * produces bit-identical marching output and rendering results, since the
 * per-ray arithmetic does not depend on them (rendering of rays longer than
 * 64 chunks of 64 samples aside, whose backward may then differ in the last
 * bits); the fused loss value is a sum in a different order.  Process-wide;
 * set them before launching, not concurrently with launches.
 *   march_waves_per_group  wavefronts sharing each group of 64 rays in the
 *                          uniform-step marching kernels: 1, 2, 4, 8 or 16
 *                          (4; more waves suit small batches).
 *   render_cached_chunks   chunks of 64 samples per ray kept in registers
 *                          between the forward and the backward pass: 1..4
 *                          (4).
 *   render_mse_max_blocks  workgroups of the fused loss kernel, 1..2^20
 *                          (16384); at n_rays / 4 or more, one ray per
 *                          wave.
 *   render_prefetch        0 or 1 (0): the fused loss kernel loads the
 *                          next ray's first chunk during a ray's backward.
 * Workspace sizes do not depend on these settings.
 */
typedef struct nacc_tuning {
    int32_t march_waves_per_group;
    int32_t render_cached_chunks;
    int32_t render_mse_max_blocks;
    int32_t render_prefetch;
} nacc_tuning;

void nacc_get_tuning(nacc_tuning* out);
int nacc_set_tuning(const nacc_tuning* tuning);

/* Message of the calling thread's most recent failed call ("" if none). */
const char* nacc_last_error(void);

/* Name of a status code. */
const char* nacc_status_str(int status);

/* Bytes of device workspace the marching calls need for n_rays rays with
 * this grid and these parameters (>= 0); -1 for invalid arguments.  The
 * workspace holds the scan's partial sums and, for uniform steps, one 64-bit
 * occupancy mask per ray and chunk of 64 candidates (enough chunks for the
 * longest chord of the clip box), which let nacc_march_fill write the
 * samples without traversing the grid again. */
int64_t nacc_march_workspace_size(int64_t n_rays, const nacc_grid_desc* grid,
                                  const nacc_march_params* params);

/*
 * Upper bound of the samples one ray can emit under `grid` and `params`
 * (the longest possible [t_near, t_far) divided into lattice steps, at most
 * 2^24, capped by max_per_ray).  n_rays times this bound sizes sample
 * buffers that no call can overflow, so that a step never has to read the
 * sample total back to the host.  Returns -1 (and sets the message) for
 * invalid arguments.
 */
int64_t nacc_march_max_samples_per_ray(const nacc_grid_desc* grid,
                                       const nacc_march_params* params);

/*
 * Marching, pass 1 of 2: count the samples of every ray and lay them out
 * (Sec. 2.1, "GPU Memory Efficiency": empty space is pruned while marching,
 * so only the samples in occupied cells are ever stored).
 *   rays_o, rays_d  float[n_rays][3]: origins and directions (normalised
 *                   directions are expected but not required).
 *   grid_id         int32[n_rays] grid of each ray, or NULL for grid 0
 *                   (ignored for CASCADE); a ray whose grid id is outside
 *                   [0, n_grids) gets no samples.
 *   grid_bits       uint32[n_grids * res^3 / 32], LSB-first bit order.
 *   grid_skip       the skip field built from grid_bits by
 *                   nacc_grid_build_skip, or NULL.  It only lets the kernels
 *                   pass over candidates that lie in empty cells without
 *                   looking them up, so results are identical with and
 *                   without it; it must be rebuilt whenever grid_bits
 *                   changes.  Used by every lookup when res % 4 == 0,
 *                   ignored otherwise (the contraction lookup bounds its
 *                   stretches through the contraction's Lipschitz
 *                   constant, (2 - 1/r)/r beyond radius r >= 1).
 *   packed_info     out int32[n_rays][2]: (start, count) per ray.
 *   total           out int64[1]: the sample total, on the device.
 *   workspace       device scratch of nacc_march_workspace_size bytes;
 *                   contents on entry are irrelevant; pass the same buffer,
 *                   unmodified, to nacc_march_fill.
 * Errors: NACC_EINVAL / NACC_ESHAPE for bad arguments; NACC_EHIP if a launch
 * fails.  A total above 2^31-1 is reported by nacc_march_fill.
 */
int nacc_march_count(const float* rays_o, const float* rays_d,
                     const int32_t* grid_id, int64_t n_rays,
                     const uint32_t* grid_bits, const uint8_t* grid_skip,
                     const nacc_grid_desc* grid,
                     const nacc_march_params* params, int32_t* packed_info,
                     int64_t* total, void* workspace, size_t workspace_bytes,
                     void* stream);

/*
 * Marching, pass 2 of 2: write the samples laid out by nacc_march_count
 * (the same rays, grid and parameters, its packed_info and its workspace;
 * workspace may be NULL, the grid is then traversed again).
 *   capacity        length of ray_indices / t_starts / t_ends.
 *   ray_indices     out int32[capacity], t_starts / t_ends out float[capacity].
 *   status          out int32[1] on the device: NACC_OK, or NACC_ECAPACITY
 *                   when some sample fell at or beyond `capacity` (those
 *                   samples are not written; the others are).  May be NULL.
 */
int nacc_march_fill(const float* rays_o, const float* rays_d,
                    const int32_t* grid_id, int64_t n_rays,
                    const uint32_t* grid_bits, const uint8_t* grid_skip,
                    const nacc_grid_desc* grid,
                    const nacc_march_params* params,
                    const int32_t* packed_info, const void* workspace,
                    size_t workspace_bytes, int64_t capacity,
                    int32_t* ray_indices, float* t_starts, float* t_ends,
                    int32_t* status, void* stream);

/*
 * Rendering forward, Eq. 1 (Sec. 2.2): per ray
 *   alpha_i = 1 - exp(-sigma_i delta_i), delta_i = t_end_i - t_start_i,
 *   T_i = exp(-sum_{j<i} sigma_j delta_j), w_i = T_i alpha_i,
 *   color = sum w_i rgb_i, opacity = sum w_i,
 *   depth = sum w_i (t_start_i + t_end_i) / 2.
 * Early termination (Sec. 2.1): with early_stop_eps > 0 the first sample
 * with T_i < early_stop_eps and every later sample of the ray get w = 0.
 *   color out float[n_rays][3]; opacity, depth out float[n_rays];
 *   weights out float[n_samples] or NULL (zero past the cut).
 *   kept    out int32[n_rays] or NULL: samples before the cut per ray.
 *   n_samples  length of the sample arrays (they may be NULL when it is 0).
 * Only samples referenced by packed_info are read.  A ray whose range
 * [start, start + count) does not lie inside [0, n_samples) is rendered as
 * an empty ray (zeros), so malformed packed_info never reads out of bounds.
 */
int nacc_render_fwd(const int32_t* packed_info, int64_t n_rays,
                    int64_t n_samples, const float* t_starts, const float* t_ends,
                    const float* sigmas, const float* rgbs,
                    float early_stop_eps, float* color, float* opacity,
                    float* depth, float* weights, int32_t* kept,
                    void* stream);

/*
 * Rendering backward (Sec. 2.2: all outputs of the radiance field receive
 * gradients).  Inputs as nacc_render_fwd plus the upstream gradients
 * g_color float[n_rays][3] and g_opacity, g_depth float[n_rays] (either may
 * be NULL = zero).  With v_i = g_color . rgb_i + g_opacity + g_depth m_i:
 *   g_rgbs_i   = w_i g_color
 *   g_sigmas_i = delta_i (T_{i+1} v_i - sum_{k>i} w_k v_k)
 * both zero at and past the early-termination cut, which is recomputed
 * exactly as in the forward call.  Transmittance is recomputed, not stored.
 *   g_sigmas out float[n_samples], g_rgbs out float[n_samples][3]; every
 *   sample referenced by packed_info is written.
 */
int nacc_render_bwd(const int32_t* packed_info, int64_t n_rays,
                    int64_t n_samples, const float* t_starts, const float* t_ends,
                    const float* sigmas, const float* rgbs,
                    float early_stop_eps, const float* g_color,
                    const float* g_opacity, const float* g_depth,
                    float* g_sigmas, float* g_rgbs, void* stream);

/*
 * Rendering of arbitrary per-sample attributes (Sec. 2.2: any sample
 * attribute, not only colour, is rendered differentiably by Eq. 1), with
 * a constant background and an opacity threshold.
 *   packed_info, n_rays, n_samples, t_starts, t_ends, sigmas,
 *   early_stop_eps   as for nacc_render_fwd.
 *   attrs        float[n_samples][n_ch], rows contiguous; 1 <= n_ch <= 4096.
 *   alpha_thre   if > 0, a sample with alpha_i = 1 - exp(-sigma_i delta_i)
 *                below it is empty: weight 0 and no attenuation of the
 *                samples behind it (the same as dropping it from the ray);
 *                <= 0 keeps every sample.  The decision is taken on the
 *                FP32 alpha.
 *   background   float[n_ch] or NULL: out += background * (1 - opacity)
 *                (the constant background of the Sec. 4 examples).
 *   out          out float[n_rays][n_ch] = sum_i w_i attrs_i (+ background).
 *   opacity, depth, weights   out float[n_rays], float[n_rays],
 *                float[n_samples]; each may be NULL (not written).
 * With n_ch = 3, no background and no threshold the outputs equal those of
 * nacc_render_fwd bit for bit.  Validation errors as nacc_render_fwd.
 */
int nacc_render_attrs_fwd(const int32_t* packed_info, int64_t n_rays,
                          int64_t n_samples, const float* t_starts,
                          const float* t_ends, const float* sigmas,
                          const float* attrs, int32_t n_ch, float early_stop_eps,
                          float alpha_thre, const float* background, float* out,
                          float* opacity, float* depth, float* weights,
                          void* stream);

/*
 * Backward of nacc_render_attrs_fwd (the cut and the empty samples held
 * fixed).  Inputs as the forward plus g_out float[n_rays][n_ch] and
 * g_opacity, g_depth float[n_rays] (NULL = zero).  With
 * v_i = g_out . attrs_i + (g_opacity - g_out . background) + g_depth m_i:
 *   g_attrs_i  = w_i g_out                        float[n_samples][n_ch]
 *   g_sigmas_i = delta_i (T_{i+1} v_i - sum_{k>i} w_k v_k)
 * both zero for empty samples and at and past the cut; every sample
 * referenced by packed_info is written.  With n_ch = 3, no background and
 * no threshold the gradients equal nacc_render_bwd's bit for bit.
 */
int nacc_render_attrs_bwd(const int32_t* packed_info, int64_t n_rays,
                          int64_t n_samples, const float* t_starts,
                          const float* t_ends, const float* sigmas,
                          const float* attrs, int32_t n_ch, float early_stop_eps,
                          float alpha_thre, const float* background,
                          const float* g_out, const float* g_opacity,
                          const float* g_depth, float* g_sigmas, float* g_attrs,
                          void* stream);

/*
 * Visibility pruning of marched samples (Sec. 2.1, "Pruning Empty and
 * Occluded Regions"; the ray_marching call of Sec. 3 with sigma_fn,
 * early_stop_eps and alpha_thre): given the densities of the samples (the
 * caller's field evaluated without gradients), sample i of a ray is kept
 * iff its transmittance T_i is at least early_stop_eps (the renderer's
 * transmittance and cut: everything from the first T_i < eps on is
 * dropped; eps = 0 keeps every sample) and its opacity
 * alpha_i = 1 - exp(-sigma_i delta_i) is at least alpha_thre.  Dropped
 * samples still attenuate the ones behind them.  Compaction follows the
 * marching pattern: count + scan, then fill.
 */
/* Bytes of device workspace nacc_prune_count needs (>= 0). */
int64_t nacc_prune_workspace_size(int64_t n_rays);

/*
 * Pass 1: keep flags and the packed layout of the kept samples.
 *   packed_info, n_rays, n_samples, t_starts, t_ends, sigmas: the marched
 *               samples as for the rendering calls.
 *   keep        out uint8[n_samples]: 1 = kept (every sample of a ray
 *               whose range lies inside n_samples is written).
 *   packed_out  out int32[n_rays][2]: (start, count) of the kept samples.
 *   total       out int64[1]: number kept, on the device.
 *   workspace   device scratch of nacc_prune_workspace_size bytes.
 */
int nacc_prune_count(const int32_t* packed_info, int64_t n_rays,
                     int64_t n_samples, const float* t_starts,
                     const float* t_ends, const float* sigmas,
                     float early_stop_eps, float alpha_thre, uint8_t* keep,
                     int32_t* packed_out, int64_t* total, void* workspace,
                     size_t workspace_bytes, void* stream);

/*
 * Pass 2: writes the kept samples in order at their packed_out slots:
 * ray_indices_out, t_starts_out, t_ends_out (and sigmas_out, nullable:
 * the densities, so the caller need not evaluate them again), each with
 * room for `capacity` samples.  Samples past capacity are dropped and
 * *status (nullable, device) is set to NACC_ECAPACITY.
 */
int nacc_prune_fill(const int32_t* packed_info, int64_t n_rays,
                    int64_t n_samples, const float* t_starts,
                    const float* t_ends, const float* sigmas,
                    const uint8_t* keep, const int32_t* packed_out,
                    int64_t capacity, int32_t* ray_indices_out,
                    float* t_starts_out, float* t_ends_out,
                    float* sigmas_out, int32_t* status, void* stream);

/* Bytes of device workspace nacc_render_fwd_bwd_mse needs (>= 0; the same
 * under every nacc_tuning, so a workspace stays valid after retuning). */
int64_t nacc_render_mse_workspace_size(int64_t n_rays);

/*
 * Fused forward + mean-squared-error loss + backward (the training step of
 * Sec. 3: loss = mse(color, target), then backward), in one pass per ray.
 *   target     float[n_rays][3].
 *   loss_rays  rays the mean is taken over (0 = n_rays; >= n_rays): a batch
 *              split over several calls passes its total, so that the calls'
 *              gradients equal those of one call over the whole batch and
 *              their losses add up to its loss.
 *   loss       out float[1] on the device: sum of squared errors of these
 *              rays divided by 3 loss_rays.
 *   color, opacity, depth, g_sigmas, g_rgbs as in the calls above, with
 *   g_color = 2 (color - target) / (3 loss_rays), g_opacity = g_depth = 0.
 *   workspace  device scratch of nacc_render_mse_workspace_size bytes.
 */
int nacc_render_fwd_bwd_mse(const int32_t* packed_info, int64_t n_rays,
                            int64_t n_samples, const float* t_starts,
                            const float* t_ends,
                            const float* sigmas, const float* rgbs,
                            float early_stop_eps, const float* target,
                            int64_t loss_rays,
                            float* color, float* opacity, float* depth,
                            float* g_sigmas, float* g_rgbs, float* loss,
                            void* workspace, size_t workspace_bytes,
                            void* stream);

/*
 * The fused loss call of nacc_render_fwd_bwd_mse without a workspace
 * argument, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 * Arguments, outputs and results are those of nacc_render_fwd_bwd_mse (the
 * same kernels); the per-wave partial losses go to a static device array of
 * NACC_MSE_NOALLOC_SCRATCH_BYTES instead.  The call allocates nothing: the
 * first call on a device resolves that device's copy of the array (no
 * allocation; each GPU keeps its copy until the process ends), later calls
 * reuse it.  Every entry the call reads is written earlier in the same call,
 * so no state carries over from one call to the next.
 * Limits: n_rays <= NACC_MSE_NOALLOC_MAX_RAYS, else NACC_ECAPACITY with
 * nothing launched.  Calls that overlap on one GPU (several streams, several
 * host threads) share the array and race: serialise them.
 */
#define NACC_MSE_NOALLOC_SCRATCH_BYTES (8ll << 20)
#define NACC_MSE_NOALLOC_MAX_RAYS 1044480ll
int nacc_render_fwd_bwd_mse_noalloc(const int32_t* packed_info, int64_t n_rays,
                                    int64_t n_samples, const float* t_starts,
                                    const float* t_ends, const float* sigmas,
                                    const float* rgbs, float early_stop_eps,
                                    const float* target, int64_t loss_rays,
                                    float* color, float* opacity, float* depth,
                                    float* g_sigmas, float* g_rgbs, float* loss,
                                    void* stream);

/*
 * Occupancy-grid update (Sec. 2.1: the grid is cached and updated during
 * training; the update rule is delegated by the paper to Instant-NGP and
 * read here as: decay every cell, take the max with fresh density samples at
 * random cells, threshold).  The state is float occ[n_cells].
 */

/* occ[c] = occ[c] * decay for every cell (FP32 multiply). */
int nacc_grid_decay(float* occ, int64_t n_cells, float decay, void* stream);

/*
 * n random cells of update `step` with jittered positions inside them.
 * Sample q draws Philox4x64-10 (Salmon et al., SC 2011) at
 * counter (q, step, 0, 0), key (seed, 0) -> (r0, r1, r2, r3):
 *   cell     = ((r0 >> 32) * n_cells) >> 32, n_cells = levels * res^3
 *   jitter_i = (float)(r_{i+1} >> 40) * 2^-24
 *   x_i      = lo_i + ((float)j_i + jitter_i) * h_i,
 *              h_i = fl32((hi_i - lo_i) / res), (j_0, j_1, j_2) the C-order
 *              index of the cell within its grid, grid = cell / res^3.
 * CASCADE grids: `levels` (1..16) is the number of levels and x is then
 * scaled by 2^grid (exact).  Otherwise `levels` (>= 1) counts independent
 * grids over the same box (grid = cell / res^3) and x is left in the box.
 * n_cells must fit int32 (NACC_ESHAPE otherwise).
 *   step_dev  uint64[1] on the device, or NULL: when given, the update number
 *             is read from it at run time (so that a captured graph can
 *             replay updates with advancing numbers) and `step` is ignored.
 *   cells out int32[n] (global cell index); positions out float[n][3].
 */
int nacc_grid_sample_cells(uint64_t seed, uint64_t step,
                           const uint64_t* step_dev, int64_t n,
                           const nacc_grid_desc* grid, int32_t levels,
                           int32_t* cells, float* positions, void* stream);

/* occ[cells[q]] = max(occ[cells[q]], values[q]) for q < n; independent of
 * the order of duplicate cells; NaN values are ignored. */
int nacc_grid_update_max(float* occ, const int32_t* cells,
                         const float* values, int64_t n, int64_t n_cells,
                         void* stream);

/* Largest distance the skip field stores (coarse cells). */
#define NACC_SKIP_CAP 15

/* Bytes of the skip buffer of `grid` (n_grids grids), 0 if res % 4 != 0:
 * the distance field (n_grids * (res/4)^3 bytes), as much scratch for its
 * build, then, from the next multiple of 256 bytes, the halo bits
 * (n_grids * 2 * ceil((res/2)^3 / 64) 32-bit words). */
int64_t nacc_grid_skip_bytes(const nacc_grid_desc* grid);

/*
 * Builds the skip field the marching calls use to pass over empty space
 * (Sec. 2.1, "Pruning Empty and Occluded Regions"): per grid, one byte per
 * coarse cell of 4x4x4 fine cells (C order),
 *   min(NACC_SKIP_CAP, Chebyshev distance in coarse cells to the nearest
 *       coarse cell holding an occupied fine cell),
 * so 0 marks coarse cells with occupied cells.  A point whose coarse cell
 * has distance D >= 2 has only empty fine cells within 4 (D - 1) fine cells
 * of it along every axis.  The field is the first n_grids * (res/4)^3 bytes
 * of `skip`, followed by scratch of the build.  The halo bits come after
 * (layout at nacc_grid_skip_bytes): per grid, one bit per cell of 2x2x2 fine
 * cells (C order over (res/2)^3 cells, LSB first), set iff some occupied
 * fine cell lies within 2 fine cells of it on every axis; the uniform-step
 * box lookup tests them once per run of candidates whose midpoints stay
 * within that reach.
 *   bits  uint32[n_grids * res^3 / 32]; skip out uint8[nacc_grid_skip_bytes],
 *         4-byte aligned.
 * NACC_ENOTSUP unless res % 4 == 0.
 */
int nacc_grid_build_skip(const uint32_t* bits, const nacc_grid_desc* grid,
                         uint8_t* skip, void* stream);

/* bits: bit c is set iff occ[c] > threshold (strict); n_cells % 32 == 0;
 * bits is uint32[n_cells / 32], LSB first. */
int nacc_grid_pack(const float* occ, int64_t n_cells, float threshold,
                   uint32_t* bits, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NACC_H */
