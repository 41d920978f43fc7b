/*
 * oracle.c -- plain, slow CPU reference for occupancy-grid ray marching,
 * packed volume rendering and the occupancy-grid update of NerfAcc
 * (Li, Tancik, Kanazawa, "NerfAcc: A General NeRF Acceleration Toolbox",
 * arXiv 2210.04847).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or constant table with
 * the HIP library; both sides are written separately against the same
 * definitions (the FP32 lattice contract below, Eq. 1 of the paper, and the
 * published Philox4x64-10 generator).
 *
 * Precision.
 *   - Marching is defined on an FP32 lattice (the "lattice contract"); the
 *     oracle evaluates it by brute force: every candidate interval is tested
 *     against a dense 0/1 mask, no skipping of any kind.  Built with
 *     -ffp-contract=off and no fast-math, so every + - * / is one IEEE
 *     round-to-nearest-even operation, exactly as written.
 *   - Rendering and its gradient are Eq. 1 evaluated in FP64 on the FP32
 *     inputs.
 *   - The occupancy-grid state is FP32 by definition, so the EMA update uses
 *     the same FP32 operations (each a single correctly rounded operation).
 *
 * Lattice contract (our reading; the paper gives no formulae for marching):
 *   clip   per axis i with d_i != 0: ta = (lo_i - o_i) / d_i,
 *          tb = (hi_i - o_i) / d_i; tmin_i = min(ta,tb), tmax_i = max(ta,tb).
 *          An axis with d_i == 0 imposes no limit if lo_i <= o_i <= hi_i and
 *          otherwise misses.  t_near = max(max_i tmin_i, near),
 *          t_far = min(min_i tmax_i, far); the ray hits iff t_near < t_far.
 *   steps  uniform: t_k = t_near + (float)k * dt (product rounded, then sum).
 *          cone:    t_0 = t_near, t_{k+1} = t_k + min(max(t_k*cone, dt), dt_max).
 *          Candidate k exists while t_k < t_far (and k < 2^24; for the cone
 *          recurrence also while t_{k+1} > t_k).  Its interval is
 *          [t_k, t_{k+1}]; the last interval is not clamped to t_far.
 *   point  t_m = (t_k + t_{k+1}) * 0.5, x_i = o_i + d_i * t_m.
 *   cell   u_i = (x_i - lo_i) * s_i with s_i = fl32(res / (hi_i - lo_i))
 *          (computed in FP64, rounded once); j_i = floor(clamp(u_i, 0,
 *          res-1)); cell = (j_0*res + j_1)*res + j_2.
 *          cascade lookup: m = max_i |x_i|; level l = the smallest l with
 *          m <= b*2^l, clamped to [0, levels-1]; the point is scaled by 2^-l
 *          (exact) and looked up in grid l over the base box [-b, b]^3.
 *          contraction lookup: n = sqrt((x0*x0 + x1*x1) + x2*x2); if n > 1
 *          the point becomes x_i * ((2 - 1/n) / n); looked up over the box.
 *   emit   candidate k is a sample iff its cell is occupied; samples are
 *          stored ray-major, k ascending (optionally capped per ray).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_CANDIDATES (1 << 24)

/* ------------------------------------------------------------------------ */
/* Marching (Sec. 2.1, "Ray Marching" and "Pruning Empty and Occluded       */
/* Regions"): samples are the lattice intervals whose midpoint lies in an   */
/* occupied cell of the occupancy grid.                                     */
/* ------------------------------------------------------------------------ */

/* Ray against an axis-aligned box, FP32.  Returns 1 on a hit. */
static int clip_ray(const float o[3], const float d[3], const float lo[3],
                    const float hi[3], float near_plane, float far_plane,
                    float* t_near, float* t_far) {
    float t_enter = -INFINITY;
    float t_exit = INFINITY;
    for (int i = 0; i < 3; ++i) {
        if (d[i] != 0.0f) {
            float ta = (lo[i] - o[i]) / d[i];
            float tb = (hi[i] - o[i]) / d[i];
            float tmin = ta < tb ? ta : tb;
            float tmax = ta < tb ? tb : ta;
            if (tmin > t_enter) t_enter = tmin;
            if (tmax < t_exit) t_exit = tmax;
        } else if (!(o[i] >= lo[i] && o[i] <= hi[i])) {
            return 0;
        }
    }
    float tn = t_enter > near_plane ? t_enter : near_plane;
    float tf = t_exit < far_plane ? t_exit : far_plane;
    *t_near = tn;
    *t_far = tf;
    return tn < tf;
}

/* fl32(res / (hi - lo)), computed in double and rounded once. */
static float axis_scale(int32_t res, float lo, float hi) {
    return (float)((double)res / ((double)hi - (double)lo));
}

/* Index of the cell holding x in a res^3 grid over [lo, hi]. */
static int64_t cell_of(const float x[3], const float lo[3], const float s[3],
                       int32_t res) {
    int64_t j[3];
    for (int i = 0; i < 3; ++i) {
        float u = (x[i] - lo[i]) * s[i];
        if (!(u > 0.0f)) u = 0.0f; /* also maps NaN to 0 */
        if (u > (float)(res - 1)) u = (float)(res - 1);
        j[i] = (int64_t)floorf(u);
    }
    return (j[0] * res + j[1]) * res + j[2];
}

/* Occupancy of the point x, for the given lookup mode.  mask is the dense
 * 0/1 grid array [n_grids][res][res][res]; grid selects one of them for the
 * box and contraction lookups. */
static int occupied_at(const float x[3], const uint8_t* mask, int32_t res,
                       int32_t n_grids, int32_t lookup, const float lo[3],
                       const float hi[3], int64_t grid) {
    int64_t cells = (int64_t)res * res * res;
    float s[3];
    for (int i = 0; i < 3; ++i) s[i] = axis_scale(res, lo[i], hi[i]);
    if (lookup == 0) {
        return mask[grid * cells + cell_of(x, lo, s, res)] != 0;
    }
    if (lookup == 1) {
        /* Multi-scale grids: the level is the smallest l with
         * max|x_i| <= b * 2^l, where b = hi[0] is the half-extent of the
         * level-0 cube (a power of two). */
        float m = fabsf(x[0]);
        if (fabsf(x[1]) > m) m = fabsf(x[1]);
        if (fabsf(x[2]) > m) m = fabsf(x[2]);
        int level = 0;
        while (level < n_grids - 1 && m > ldexpf(hi[0], level)) ++level;
        float y[3];
        for (int i = 0; i < 3; ++i) y[i] = ldexpf(x[i], -level);
        return mask[(int64_t)level * cells + cell_of(y, lo, s, res)] != 0;
    }
    /* lookup == 2: scene contraction (Sec. 2.1, "Scene Contraction for
     * Unbounded Scene"): points outside the unit ball are pulled inside the
     * ball of radius 2 before the grid is queried. */
    float n2 = (x[0] * x[0] + x[1] * x[1]) + x[2] * x[2];
    float n = sqrtf(n2);
    float y[3] = {x[0], x[1], x[2]};
    if (n > 1.0f) {
        float f = (2.0f - 1.0f / n) / n;
        for (int i = 0; i < 3; ++i) y[i] = x[i] * f;
    }
    return mask[grid * cells + cell_of(y, lo, s, res)] != 0;
}

/*
 * Brute-force marching.  For every ray: clip, walk every lattice candidate,
 * test its midpoint against the dense mask, keep the occupied ones.
 *
 * counts[n_rays] always receives the per-ray sample count.  When ray_indices
 * (and t_starts, t_ends) is non-NULL the samples are written in ray-major
 * order; samples beyond `capacity` are not written.  Returns the total.
 *
 * lookup 0: box lookup, the box is also the clip box; grid_id (nullable)
 *           picks the grid per ray.
 * lookup 1: cascaded grids, level-0 box [-b,b]^3, clip box [-b,b]^3 scaled
 *           by 2^(n_grids-1).
 * lookup 2: contraction, box = contracted grid box, no clipping (near/far
 *           only); grid_id (nullable) picks the grid per ray.
 */
int64_t oracle_march(const float* rays_o, const float* rays_d,
                     const int32_t* grid_id, int64_t n_rays,
                     const uint8_t* mask, int32_t res, int32_t n_grids,
                     int32_t lookup, const float* box, float near_plane,
                     float far_plane, float dt, float dt_max, float cone,
                     int32_t max_per_ray, int32_t* counts, int64_t capacity,
                     int32_t* ray_indices, float* t_starts, float* t_ends) {
    const float* lo = box;
    const float* hi = box + 3;
    float clip_lo[3], clip_hi[3];
    for (int i = 0; i < 3; ++i) {
        clip_lo[i] = lo[i];
        clip_hi[i] = hi[i];
        if (lookup == 1) {
            clip_lo[i] = ldexpf(lo[i], n_grids - 1);
            clip_hi[i] = ldexpf(hi[i], n_grids - 1);
        } else if (lookup == 2) {
            clip_lo[i] = -INFINITY;
            clip_hi[i] = INFINITY;
        }
    }
    int64_t total = 0;
    for (int64_t r = 0; r < n_rays; ++r) {
        const float* o = rays_o + 3 * r;
        const float* d = rays_d + 3 * r;
        int64_t grid = (grid_id != NULL && lookup != 1) ? grid_id[r] : 0;
        int32_t count = 0;
        float t_near, t_far;
        /* a ray naming a grid that does not exist is a miss */
        int valid_grid = grid >= 0 && grid < n_grids;
        if (valid_grid && clip_ray(o, d, clip_lo, clip_hi, near_plane, far_plane,
                                   &t_near, &t_far)) {
            float t0 = t_near;
            for (int64_t k = 0; k < ORACLE_MAX_CANDIDATES; ++k) {
                float t1;
                if (cone == 0.0f) {
                    /* uniform lattice, anchored at t_near */
                    t0 = t_near + (float)k * dt;
                    if (!(t0 < t_far)) break;
                    t1 = t_near + (float)(k + 1) * dt;
                } else {
                    /* cone-scaled steps: a recurrence on t */
                    if (!(t0 < t_far)) break;
                    float step = t0 * cone;
                    if (step < dt) step = dt;
                    if (step > dt_max) step = dt_max;
                    t1 = t0 + step;
                    if (!(t1 > t0)) break;
                }
                float tm = (t0 + t1) * 0.5f;
                float x[3];
                for (int i = 0; i < 3; ++i) x[i] = o[i] + d[i] * tm;
                if (occupied_at(x, mask, res, n_grids, lookup, lo, hi, grid)) {
                    if (max_per_ray > 0 && count >= max_per_ray) break;
                    int64_t at = total + count;
                    if (ray_indices != NULL && at < capacity) {
                        ray_indices[at] = (int32_t)r;
                        t_starts[at] = t0;
                        t_ends[at] = t1;
                    }
                    ++count;
                }
                t0 = t1;
            }
        }
        counts[r] = count;
        total += count;
    }
    return total;
}

/* The clip interval alone, for closed-form tests of the clip step. */
void oracle_clip(const float* rays_o, const float* rays_d, int64_t n_rays,
                 const float* box, float near_plane, float far_plane,
                 float* t_near, float* t_far, int32_t* hit) {
    for (int64_t r = 0; r < n_rays; ++r) {
        hit[r] = clip_ray(rays_o + 3 * r, rays_d + 3 * r, box, box + 3,
                          near_plane, far_plane, t_near + r, t_far + r);
    }
}

/* ------------------------------------------------------------------------ */
/* Rendering, Eq. 1 (Sec. 2.2 "Differentiable Rendering"):                  */
/*   C = sum_i T_i alpha_i c_i,  T_i = exp(-sum_{j<i} sigma_j delta_j),     */
/*   alpha_i = 1 - exp(-sigma_i delta_i),  delta_i = t_end - t_start.       */
/* Early termination (Sec. 2.1): sample i and everything after it is        */
/* dropped once T_i < eps (eps = 0 disables it).                            */
/* ------------------------------------------------------------------------ */

/* Visibility pruning while marching (Sec. 2.1, "Pruning Empty and Occluded
 * Regions"; the ray_marching call of Sec. 3 with sigma_fn, early_stop_eps and
 * alpha_thre): with the densities of the marched samples, sample i of a ray
 * is kept iff its transmittance T_i = exp(-sum_{j<i} sigma_j delta_j) is at
 * least eps (so everything from the first T_i < eps on is dropped) and its
 * opacity alpha_i = 1 - exp(-sigma_i delta_i) is at least alpha_thre.  Every
 * sample, kept or not, adds to the transmittance of the ones after it.
 * FP64.  Outputs keep[n_samples] (0/1) and counts[n_rays]; returns the
 * number kept. */
int64_t oracle_prune(const int32_t* packed_info, int64_t n_rays,
                     const double* t_starts, const double* t_ends,
                     const double* sigmas, double eps, double alpha_thre,
                     uint8_t* keep, int32_t* counts) {
    int64_t total = 0;
    for (int64_t r = 0; r < n_rays; ++r) {
        int64_t start = packed_info[2 * r], n = packed_info[2 * r + 1];
        double prefix = 0.0;
        int32_t kept = 0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t s = start + i;
            double tau = sigmas[s] * (t_ends[s] - t_starts[s]);
            double trans = exp(-prefix);
            double alpha = -expm1(-tau);
            int k = trans >= eps && alpha >= alpha_thre;
            keep[s] = (uint8_t)k;
            kept += k;
            prefix += tau;
        }
        counts[r] = kept;
        total += kept;
    }
    return total;
}

/* Forward in FP64 (inputs are FP64 arrays; FP32 data converts exactly).
 * Outputs: color[n_rays*3], opacity[n_rays], depth[n_rays]
 * (depth = sum w * (t_start + t_end) / 2), weights[n_samples] (nullable,
 * zero past the cut), kept[n_rays] (nullable: samples before the cut). */
void oracle_render_fwd(const int32_t* packed_info, int64_t n_rays,
                       const double* t_starts, const double* t_ends,
                       const double* sigmas, const double* rgbs, double eps,
                       double* color, double* opacity, double* depth,
                       double* weights, int32_t* kept) {
    for (int64_t r = 0; r < n_rays; ++r) {
        int64_t start = packed_info[2 * r];
        int64_t n = packed_info[2 * r + 1];
        double c[3] = {0.0, 0.0, 0.0};
        double a = 0.0, dep = 0.0;
        double prefix = 0.0; /* sum_{j<i} sigma_j delta_j */
        int64_t cut = n;
        for (int64_t i = 0; i < n; ++i) {
            int64_t s = start + i;
            double ts = t_starts[s], te = t_ends[s];
            double tau = sigmas[s] * (te - ts);
            double trans = exp(-prefix);
            if (eps > 0.0 && trans < eps) {
                cut = i;
                break;
            }
            double alpha = -expm1(-tau);
            double w = trans * alpha;
            for (int ch = 0; ch < 3; ++ch) c[ch] += w * rgbs[3 * s + ch];
            a += w;
            dep += w * (ts + te) * 0.5;
            if (weights != NULL) weights[s] = w;
            prefix += tau;
        }
        if (weights != NULL)
            for (int64_t i = cut; i < n; ++i) weights[start + i] = 0.0;
        for (int ch = 0; ch < 3; ++ch) color[3 * r + ch] = c[ch];
        opacity[r] = a;
        depth[r] = dep;
        if (kept != NULL) kept[r] = (int32_t)cut;
    }
}

/*
 * Backward of oracle_render_fwd in FP64 (Sec. 2.2: every field output
 * receives a gradient).  With v_i = g_C . c_i + g_A + g_D * m_i,
 * m_i = (t_start + t_end) / 2, and the cut treated as locally constant:
 *   dL/dc_i     = w_i * g_C
 *   dL/dsigma_i = delta_i * (T_{i+1} v_i - sum_{k>i, k<cut} w_k v_k)
 * both zero at and after the cut.  g_opacity and g_depth are nullable (zero).
 * scale (nullable) receives delta_i * (T_{i+1} |v|_i + sum_{k>i} w_k |v|_k),
 * the magnitude of the terms that form dL/dsigma_i: |v|_i is the sum of the
 * magnitudes of the terms of v_i (|g_C,ch c_i,ch| over channels, |g_A|,
 * |g_D m_i|), since v_i is itself a sum of terms of either sign.
 */
int oracle_render_bwd(const int32_t* packed_info, int64_t n_rays,
                       const double* t_starts, const double* t_ends,
                       const double* sigmas, const double* rgbs, double eps,
                       const double* g_color, const double* g_opacity,
                       const double* g_depth, double* g_sigmas, double* g_rgbs,
                       double* scale) {
    int64_t longest = 0;
    for (int64_t r = 0; r < n_rays; ++r)
        if (packed_info[2 * r + 1] > longest) longest = packed_info[2 * r + 1];
    double* pre = (double*)malloc((size_t)(longest > 0 ? longest : 1) * sizeof(double));
    if (pre == NULL) return -1;
    for (int64_t r = 0; r < n_rays; ++r) {
        int64_t start = packed_info[2 * r];
        int64_t n = packed_info[2 * r + 1];
        double gc[3] = {g_color[3 * r], g_color[3 * r + 1], g_color[3 * r + 2]};
        double ga = g_opacity != NULL ? g_opacity[r] : 0.0;
        double gd = g_depth != NULL ? g_depth[r] : 0.0;
        /* Forward quantities: the exclusive prefix sum_{j<i} tau_j per
         * sample, and the cut. */
        double prefix = 0.0;
        int64_t cut = n;
        for (int64_t i = 0; i < n; ++i) {
            if (eps > 0.0 && exp(-prefix) < eps) {
                cut = i;
                break;
            }
            int64_t s = start + i;
            pre[i] = prefix;
            prefix += sigmas[s] * (t_ends[s] - t_starts[s]);
        }
        /* Reverse pass: suffix sums of w_k v_k (and of w_k |v_k|). */
        double suffix = 0.0, suffix_abs = 0.0;
        for (int64_t i = cut - 1; i >= 0; --i) {
            int64_t s = start + i;
            double ts = t_starts[s], te = t_ends[s];
            double delta = te - ts;
            double tau = sigmas[s] * delta;
            double t_i = exp(-pre[i]);
            double t_next = exp(-(pre[i] + tau));
            double w = t_i * -expm1(-tau);
            double v = gc[0] * rgbs[3 * s] + gc[1] * rgbs[3 * s + 1] +
                       gc[2] * rgbs[3 * s + 2] + ga + gd * (ts + te) * 0.5;
            double v_abs = fabs(gc[0] * rgbs[3 * s]) + fabs(gc[1] * rgbs[3 * s + 1]) +
                           fabs(gc[2] * rgbs[3 * s + 2]) + fabs(ga) +
                           fabs(gd * (ts + te) * 0.5);
            double dtau = t_next * v - suffix;
            g_sigmas[s] = delta * dtau;
            if (scale != NULL) scale[s] = delta * (t_next * v_abs + suffix_abs);
            for (int ch = 0; ch < 3; ++ch) g_rgbs[3 * s + ch] = w * gc[ch];
            suffix += w * v;
            suffix_abs += w * v_abs;
        }
        for (int64_t i = cut; i < n; ++i) {
            int64_t s = start + i;
            g_sigmas[s] = 0.0;
            if (scale != NULL) scale[s] = 0.0;
            for (int ch = 0; ch < 3; ++ch) g_rgbs[3 * s + ch] = 0.0;
        }
    }
    free(pre);
    return 0;
}

/*
 * Rendering of arbitrary per-sample attributes (Sec. 2.2: any sample
 * attribute, not only colour, is rendered differentiably), in FP64, with
 * two options:
 *   background (nullable, n_ch values): the rendered attribute is
 *     sum_i w_i a_i + background * (1 - opacity), the constant background
 *     of the Instant-NGP example's evaluation (Sec. 4);
 *   alpha_thre: if > 0, a sample with alpha_i < alpha_thre is empty
 *     (weight 0, no attenuation of later samples), the same as dropping it
 *     from the ray before rendering; 0 keeps every sample.
 * attrs: n_samples rows of n_ch values, row stride `stride` (>= n_ch).
 * Outputs: out[n_rays * n_ch], opacity, depth (as oracle_render_fwd),
 * weights[n_samples] (nullable).  The cut is the first sample whose
 * transmittance (over the samples that are not empty) is below eps.
 */
void oracle_render_attrs_fwd(const int32_t* packed_info, int64_t n_rays,
                             const double* t_starts, const double* t_ends,
                             const double* sigmas, const double* attrs, int64_t n_ch,
                             int64_t stride, double eps, double alpha_thre,
                             const double* background, double* out, double* opacity,
                             double* depth, double* weights) {
    for (int64_t r = 0; r < n_rays; ++r) {
        int64_t start = packed_info[2 * r];
        int64_t n = packed_info[2 * r + 1];
        double a = 0.0, dep = 0.0, prefix = 0.0;
        for (int64_t ch = 0; ch < n_ch; ++ch) out[r * n_ch + ch] = 0.0;
        int64_t cut = n;
        for (int64_t i = 0; i < n; ++i) {
            int64_t s = start + i;
            double ts = t_starts[s], te = t_ends[s];
            double tau = sigmas[s] * (te - ts);
            double trans = exp(-prefix);
            if (eps > 0.0 && trans < eps) {
                cut = i;
                break;
            }
            double alpha = -expm1(-tau);
            double w = 0.0;
            if (!(alpha_thre > 0.0) || alpha >= alpha_thre) {
                w = trans * alpha;
                prefix += tau;
            }
            for (int64_t ch = 0; ch < n_ch; ++ch) out[r * n_ch + ch] += w * attrs[s * stride + ch];
            a += w;
            dep += w * (ts + te) * 0.5;
            if (weights != NULL) weights[s] = w;
        }
        if (weights != NULL)
            for (int64_t i = cut; i < n; ++i) weights[start + i] = 0.0;
        if (background != NULL)
            for (int64_t ch = 0; ch < n_ch; ++ch) out[r * n_ch + ch] += background[ch] * (1.0 - a);
        opacity[r] = a;
        depth[r] = dep;
    }
}

/*
 * Backward of oracle_render_attrs_fwd (cut and empty samples locally
 * constant).  The background term adds -g_out . background to the opacity
 * gradient, so with
 *   v_i = g_out . a_i + (g_opacity - g_out . background) + g_depth * m_i:
 *   dL/da_i     = w_i * g_out
 *   dL/dsigma_i = delta_i * (T_{i+1} v_i - sum_{k>i} w_k v_k)
 * for samples before the cut that are not empty; zero for the others.
 * g_opacity, g_depth, background nullable; scale as in oracle_render_bwd.
 */
int oracle_render_attrs_bwd(const int32_t* packed_info, int64_t n_rays,
                            const double* t_starts, const double* t_ends,
                            const double* sigmas, const double* attrs, int64_t n_ch,
                            int64_t stride, double eps, double alpha_thre,
                            const double* background, const double* g_out,
                            const double* g_opacity, const double* g_depth,
                            double* g_sigmas, double* g_attrs, double* scale) {
    int64_t longest = 0;
    for (int64_t r = 0; r < n_rays; ++r)
        if (packed_info[2 * r + 1] > longest) longest = packed_info[2 * r + 1];
    double* pre = (double*)malloc((size_t)(longest > 0 ? longest : 1) * sizeof(double));
    if (pre == NULL) return -1;
    for (int64_t r = 0; r < n_rays; ++r) {
        int64_t start = packed_info[2 * r];
        int64_t n = packed_info[2 * r + 1];
        const double* g = g_out + r * n_ch;
        double ga = g_opacity != NULL ? g_opacity[r] : 0.0;
        double gd = g_depth != NULL ? g_depth[r] : 0.0;
        double ga_abs = fabs(ga);
        if (background != NULL)
            for (int64_t ch = 0; ch < n_ch; ++ch) {
                ga -= g[ch] * background[ch];
                ga_abs += fabs(g[ch] * background[ch]);
            }
        double prefix = 0.0;
        int64_t cut = n;
        for (int64_t i = 0; i < n; ++i) {
            if (eps > 0.0 && exp(-prefix) < eps) {
                cut = i;
                break;
            }
            int64_t s = start + i;
            pre[i] = prefix;
            double tau = sigmas[s] * (t_ends[s] - t_starts[s]);
            if (!(alpha_thre > 0.0) || -expm1(-tau) >= alpha_thre) prefix += tau;
        }
        double suffix = 0.0, suffix_abs = 0.0;
        for (int64_t i = n - 1; i >= 0; --i) {
            int64_t s = start + i;
            double ts = t_starts[s], te = t_ends[s];
            double delta = te - ts;
            double tau = sigmas[s] * delta;
            double alpha = -expm1(-tau);
            if (i >= cut || (alpha_thre > 0.0 && alpha < alpha_thre)) {
                g_sigmas[s] = 0.0;
                if (scale != NULL) scale[s] = 0.0;
                for (int64_t ch = 0; ch < n_ch; ++ch) g_attrs[s * stride + ch] = 0.0;
                continue;
            }
            double t_i = exp(-pre[i]);
            double t_next = exp(-(pre[i] + tau));
            double w = t_i * alpha;
            double v = ga + gd * (ts + te) * 0.5;
            double v_abs = ga_abs + fabs(gd * (ts + te) * 0.5);
            for (int64_t ch = 0; ch < n_ch; ++ch) {
                v += g[ch] * attrs[s * stride + ch];
                v_abs += fabs(g[ch] * attrs[s * stride + ch]);
            }
            g_sigmas[s] = delta * (t_next * v - suffix);
            if (scale != NULL) scale[s] = delta * (t_next * v_abs + suffix_abs);
            for (int64_t ch = 0; ch < n_ch; ++ch) g_attrs[s * stride + ch] = w * g[ch];
            suffix += w * v;
            suffix_abs += w * v_abs;
        }
    }
    free(pre);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Occupancy-grid update (Sec. 2.1: the binary grid is cached and updated   */
/* during training).  Our reading of the update: every cell decays by a     */
/* factor, sampled cells take the max with fresh density samples, and the   */
/* bit is set where the stored value exceeds a threshold.  FP32 state.      */
/* ------------------------------------------------------------------------ */

/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): ten rounds of two 64x64->128 multiplications
 * with the published multipliers and Weyl key increments. */
void oracle_philox4x64_10(const uint64_t* counter, const uint64_t* key,
                          uint64_t* out) {
    const uint64_t mul0 = 0xD2E7470EE14C6C93ULL;
    const uint64_t mul1 = 0xCA5A826395121157ULL;
    const uint64_t weyl0 = 0x9E3779B97F4A7C15ULL;
    const uint64_t weyl1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = counter[0], c1 = counter[1], c2 = counter[2], c3 = counter[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        unsigned __int128 p0 = (unsigned __int128)mul0 * c0;
        unsigned __int128 p1 = (unsigned __int128)mul1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += weyl0;
        k1 += weyl1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/*
 * Random cells for update number `step`: sample n uses
 * Philox4x64-10(counter = (n, step, 0, 0), key = (seed, 0)) -> (r0..r3).
 *   cell     = ((r0 >> 32) * n_cells) >> 32        (uniform in [0, n_cells))
 *   jitter_i = (float)(r_{i+1} >> 40) * 2^-24       (uniform in [0, 1))
 * With n_cells = levels * res^3 the cell also names its level (grid).  The
 * position is x_i = lo_i + ((float)j_i + jitter_i) * h_i scaled by 2^level
 * (level = cell / res^3; cascades only, levels = 1 otherwise), where
 * h_i = fl32((hi_i - lo_i) / res) and (j_0, j_1, j_2) is the C-order cell.
 */
void oracle_grid_sample_cells(uint64_t seed, uint64_t step, int64_t n,
                              int32_t res, int32_t levels, int32_t cascade,
                              const float* box,
                              int32_t* cells, float* positions) {
    int64_t per_grid = (int64_t)res * res * res;
    uint64_t n_cells = (uint64_t)per_grid * (uint64_t)levels;
    float h[3];
    for (int i = 0; i < 3; ++i)
        h[i] = (float)(((double)box[3 + i] - (double)box[i]) / (double)res);
    for (int64_t q = 0; q < n; ++q) {
        uint64_t ctr[4] = {(uint64_t)q, step, 0, 0};
        uint64_t key[2] = {seed, 0};
        uint64_t rnd[4];
        oracle_philox4x64_10(ctr, key, rnd);
        uint64_t cell = ((rnd[0] >> 32) * n_cells) >> 32;
        cells[q] = (int32_t)cell;
        int64_t level = cascade ? (int64_t)cell / per_grid : 0;
        int64_t local = (int64_t)cell % per_grid;
        int64_t j[3] = {local / ((int64_t)res * res), (local / res) % res, local % res};
        for (int i = 0; i < 3; ++i) {
            float jit = (float)(rnd[i + 1] >> 40) * 0x1p-24f;
            float x = box[i] + ((float)j[i] + jit) * h[i];
            positions[3 * q + i] = ldexpf(x, (int)level);
        }
    }
}

void oracle_grid_decay(float* occ, int64_t n_cells, float decay) {
    for (int64_t c = 0; c < n_cells; ++c) occ[c] = occ[c] * decay;
}

void oracle_grid_update_max(float* occ, const int32_t* cells,
                            const float* values, int64_t n) {
    for (int64_t q = 0; q < n; ++q) {
        float v = values[q];
        if (v > occ[cells[q]]) occ[cells[q]] = v;
    }
}

void oracle_grid_threshold(const float* occ, int64_t n_cells, float threshold,
                           uint8_t* mask) {
    for (int64_t c = 0; c < n_cells; ++c) mask[c] = occ[c] > threshold ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Synthetic radiance field used as test input (a stand-in for the user's   */
/* field of Sec. 3; not part of the method).  FP64 evaluation at FP32       */
/* positions x = o + d * ((t_start + t_end) * 0.5), computed in FP32.       */
/*   sigma(x) = sum_b peak_b * exp(-|x - c_b|^2 / (2 std_b^2))              */
/*   rgb(x)   = 1 / (1 + exp(-(W x + bias)))                                */
/* ------------------------------------------------------------------------ */

void oracle_sample_positions(const float* rays_o, const float* rays_d,
                             const int32_t* ray_indices, const float* t_starts,
                             const float* t_ends, int64_t n, float* positions) {
    for (int64_t s = 0; s < n; ++s) {
        int64_t r = ray_indices[s];
        float tm = (t_starts[s] + t_ends[s]) * 0.5f;
        for (int i = 0; i < 3; ++i)
            positions[3 * s + i] = rays_o[3 * r + i] + rays_d[3 * r + i] * tm;
    }
}

/* blob_set (nullable) selects, per point, which set of n_blobs centres is
 * used (per-frame scenes); centres has shape [sets][n_blobs][3]. */
void oracle_blob_field(const float* positions, const int32_t* blob_set,
                       int64_t n, const float* centres, const float* stds,
                       const float* peaks, int32_t n_blobs, const float* w,
                       const float* bias, int32_t contract, double* sigma,
                       double* rgb) {
    for (int64_t q = 0; q < n; ++q) {
        double x[3] = {positions[3 * q], positions[3 * q + 1], positions[3 * q + 2]};
        if (contract) {
            /* scene defined in contracted coordinates (Sec. 2.1, unbounded
             * scenes): points beyond the unit ball are pulled inside the
             * radius-2 ball, the norm mapping to 2 - 1/norm */
            double nrm = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
            if (nrm > 1.0) {
                double f = (2.0 - 1.0 / nrm) / nrm;
                for (int i = 0; i < 3; ++i) x[i] *= f;
            }
        }
        const float* cset = centres + (blob_set != NULL ? (int64_t)blob_set[q] * n_blobs * 3 : 0);
        double acc = 0.0;
        for (int32_t b = 0; b < n_blobs; ++b) {
            double d2 = 0.0;
            for (int i = 0; i < 3; ++i) {
                double e = x[i] - (double)cset[3 * b + i];
                d2 += e * e;
            }
            double sd = stds[b];
            acc += (double)peaks[b] * exp(-d2 / (2.0 * sd * sd));
        }
        if (sigma != NULL) sigma[q] = acc;
        if (rgb != NULL) {
            for (int ch = 0; ch < 3; ++ch) {
                double z = bias[ch];
                for (int i = 0; i < 3; ++i) z += (double)w[3 * ch + i] * x[i];
                rgb[3 * q + ch] = 1.0 / (1.0 + exp(-z));
            }
        }
    }
}
