// Step plans (nacc_plan.h): one step of Sec. 3's training loop (marching,
// the caller's field, rendering with the loss and its backward) and the
// occupancy-grid update of Sec. 2.1, launched eagerly through the entry
// points of nacc.h, or captured into HIP graphs and replayed; plus a tuner
// of the launch parameters that times graph replays of the step itself.
#include <algorithm>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "nacc_plan.h"

using namespace nacc;

struct nacc_plan {
    nacc_plan_desc d;
    int device = 0;
    void* march_ws = nullptr;
    size_t march_ws_bytes = 0;
    void* mse_ws = nullptr;
    size_t mse_ws_bytes = 0;
    hipStream_t own = nullptr;  // capture and tuning stream (default priority)
    hipGraphExec_t step_exec = nullptr;
    hipGraphExec_t update_exec = nullptr;
};

namespace {

__global__ void increment_kernel(uint64_t* counter) {
    if (threadIdx.x == 0) counter[0] += 1;
}

int hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return NACC_OK;
    return set_error(NACC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int validate(const nacc_plan_desc* d) {
    NACC_REQUIRE(d != nullptr, NACC_EINVAL, "plan description must be non-NULL");
    NACC_REQUIRE(d->n_rays >= 0, NACC_EINVAL, "n_rays < 0");
    NACC_REQUIRE(d->capacity >= 0 && d->capacity <= INT32_MAX, NACC_EINVAL,
                 "capacity = %lld not in [0, 2^31-1]", static_cast<long long>(d->capacity));
    NACC_REQUIRE(d->rays_o && d->rays_d && d->grid_bits && d->packed_info && d->total, NACC_EINVAL,
                 "rays, grid bits, packed_info and total must be non-NULL");
    NACC_REQUIRE(d->capacity == 0 || (d->ray_indices && d->t_starts && d->t_ends && d->sigmas && d->rgbs),
                 NACC_EINVAL, "sample arrays must be non-NULL");
    NACC_REQUIRE(d->field != nullptr, NACC_EINVAL, "the field stage is required");
    NACC_REQUIRE(d->color && d->opacity && d->depth, NACC_EINVAL, "color, opacity and depth must be non-NULL");
    NACC_REQUIRE(d->early_stop_eps >= 0.0f, NACC_EINVAL, "early_stop_eps must be >= 0");
    if (d->target != nullptr) {
        NACC_REQUIRE(d->loss != nullptr, NACC_EINVAL, "a training step needs loss");
        NACC_REQUIRE(d->capacity == 0 || (d->g_sigmas && d->g_rgbs), NACC_EINVAL,
                     "a training step needs g_sigmas and g_rgbs");
        NACC_REQUIRE(d->loss_rays == 0 || d->loss_rays >= d->n_rays, NACC_EINVAL, "loss_rays must be 0 or >= n_rays");
    }
    // the grid and the marching parameters, as the marching calls check them
    if (nacc_march_workspace_size(d->n_rays, &d->grid, &d->params) < 0) return NACC_EINVAL;
    if (d->occ != nullptr) {
        NACC_REQUIRE(d->update_cells > 0, NACC_EINVAL, "update_cells must be > 0");
        NACC_REQUIRE(d->update_counter && d->update_cell_ids && d->update_positions && d->update_values,
                     NACC_EINVAL, "the update's arrays must be non-NULL");
        NACC_REQUIRE(d->update_field != nullptr, NACC_EINVAL, "the update needs its field stage");
        NACC_REQUIRE(d->decay >= 0.0f && d->decay <= 1.0f, NACC_EINVAL, "decay must lie in [0, 1]");
        NACC_REQUIRE(d->threshold == d->threshold, NACC_EINVAL, "threshold is NaN");
    }
    return NACC_OK;
}

int check_device(const nacc_plan* p) {
    NACC_REQUIRE(p != nullptr, NACC_EINVAL, "plan must be non-NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
        return set_error(NACC_EINVAL, "the plan belongs to device %d, current is %d", p->device, dev);
    }
    return NACC_OK;
}

int stage(nacc_stage_fn fn, void* user, hipStream_t s, const char* what) {
    const int st = fn(user, s);
    if (st != 0 && nacc_last_error()[0] == '\0') set_error(st, "%s stage returned %d", what, st);
    return st;
}

int run_step(nacc_plan* p, hipStream_t s) {
    const nacc_plan_desc& d = p->d;
    int st = nacc_march_count(d.rays_o, d.rays_d, d.grid_id, d.n_rays, d.grid_bits, d.grid_skip, &d.grid,
                              &d.params, d.packed_info, d.total, p->march_ws, p->march_ws_bytes, s);
    if (st != NACC_OK) return st;
    st = nacc_march_fill(d.rays_o, d.rays_d, d.grid_id, d.n_rays, d.grid_bits, d.grid_skip, &d.grid, &d.params,
                         d.packed_info, p->march_ws, p->march_ws_bytes, d.capacity, d.ray_indices, d.t_starts,
                         d.t_ends, d.status, s);
    if (st != NACC_OK) return st;
    if ((st = stage(d.field, d.field_user, s, "field")) != 0) return st;
    if (d.target != nullptr) {
        st = nacc_render_fwd_bwd_mse(d.packed_info, d.n_rays, d.capacity, d.t_starts, d.t_ends, d.sigmas, d.rgbs,
                                     d.early_stop_eps, d.target, d.loss_rays, d.color, d.opacity, d.depth,
                                     d.g_sigmas, d.g_rgbs, d.loss, p->mse_ws, p->mse_ws_bytes, s);
    } else {
        st = nacc_render_fwd(d.packed_info, d.n_rays, d.capacity, d.t_starts, d.t_ends, d.sigmas, d.rgbs,
                             d.early_stop_eps, d.color, d.opacity, d.depth, nullptr, nullptr, s);
    }
    if (st != NACC_OK) return st;
    if (d.after != nullptr && (st = stage(d.after, d.after_user, s, "after")) != 0) return st;
    return NACC_OK;
}

int run_update(nacc_plan* p, hipStream_t s) {
    const nacc_plan_desc& d = p->d;
    const int64_t n_cells = static_cast<int64_t>(d.grid.n_grids) * d.grid.res * d.grid.res * d.grid.res;
    int st = nacc_grid_decay(d.occ, n_cells, d.decay, s);
    if (st != NACC_OK) return st;
    st = nacc_grid_sample_cells(d.seed, 0, d.update_counter, d.update_cells, &d.grid, d.grid.n_grids,
                                d.update_cell_ids, d.update_positions, s);
    if (st != NACC_OK) return st;
    if ((st = stage(d.update_field, d.update_field_user, s, "update field")) != 0) return st;
    if ((st = nacc_grid_update_max(d.occ, d.update_cell_ids, d.update_values, d.update_cells, n_cells, s)) != NACC_OK)
        return st;
    if ((st = nacc_grid_pack(d.occ, n_cells, d.threshold, d.grid_bits, s)) != NACC_OK) return st;
    if (d.grid_skip != nullptr && (st = nacc_grid_build_skip(d.grid_bits, &d.grid, d.grid_skip, s)) != NACC_OK)
        return st;
    hipLaunchKernelGGL(increment_kernel, dim3(1), dim3(kWave), 0, s, d.update_counter);
    return check_launch("update counter");
}

// Captures `run` on the plan's stream into an instantiated graph.
template <typename Run>
int capture(nacc_plan* p, Run run, hipGraphExec_t* out) {
    int st = hip_status(hipStreamBeginCapture(p->own, hipStreamCaptureModeThreadLocal), "begin capture");
    if (st != NACC_OK) return st;
    const int run_st = run(p, p->own);
    hipGraph_t graph = nullptr;
    const hipError_t end = hipStreamEndCapture(p->own, &graph);
    if (run_st != NACC_OK) {
        if (graph != nullptr) (void)hipGraphDestroy(graph);
        return run_st;
    }
    if ((st = hip_status(end, "end capture")) != NACC_OK) return st;
    hipGraphExec_t exec = nullptr;
    st = hip_status(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate");
    (void)hipGraphDestroy(graph);
    if (st != NACC_OK) return st;
    *out = exec;
    return NACC_OK;
}

void drop_graphs(nacc_plan* p) {
    if (p->step_exec != nullptr) (void)hipGraphExecDestroy(p->step_exec);
    if (p->update_exec != nullptr) (void)hipGraphExecDestroy(p->update_exec);
    p->step_exec = p->update_exec = nullptr;
}

int capture_all(nacc_plan* p) {
    drop_graphs(p);
    int st = capture(p, run_step, &p->step_exec);
    if (st == NACC_OK && p->d.occ != nullptr) st = capture(p, run_update, &p->update_exec);
    if (st != NACC_OK) drop_graphs(p);
    return st;
}

// The outputs a change of launch parameters must leave bit-identical: the
// sample total and, for every output array, a position-dependent checksum of
// all its 32-bit words (sum over i of mix(i, word_i) modulo 2^64, so the
// order in which threads add does not matter), taken on the device.
struct Snapshot {
    std::vector<unsigned long long> sums;
};

__device__ inline unsigned long long mix64(unsigned long long z) {
    // the finaliser of SplitMix64 (Steele, Lea, Flood, OOPSLA 2014)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void checksum_kernel(const uint32_t* __restrict__ words, int64_t n_words,
                                unsigned long long* __restrict__ out) {
    unsigned long long acc = 0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n_words; i += stride) {
        acc += mix64((static_cast<unsigned long long>(i) << 32) ^ words[i] ^ 0x9E3779B97F4A7C15ull);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & (kWave - 1)) == 0 && acc != 0) atomicAdd(out, acc);
}

int snapshot(const nacc_plan* p, Snapshot* snap) {
    const nacc_plan_desc& d = p->d;
    int64_t total = 0;
    int st = hip_status(hipMemcpy(&total, d.total, sizeof(total), hipMemcpyDeviceToHost), "snapshot copy");
    if (st != NACC_OK) return st;
    const size_t e = static_cast<size_t>(std::max<int64_t>(0, std::min<int64_t>(total, d.capacity)));
    const size_t r = static_cast<size_t>(d.n_rays);
    const std::pair<const void*, size_t> parts[] = {
        {d.packed_info, r * 2},
        {d.color, r * 3},
        {d.opacity, r},
        {d.depth, r},
        {d.ray_indices, e},
        {d.t_starts, e},
        {d.t_ends, e},
        {d.target != nullptr ? d.g_sigmas : nullptr, e},
        {d.target != nullptr ? d.g_rgbs : nullptr, e * 3},
    };
    constexpr int kParts = sizeof(parts) / sizeof(parts[0]);
    unsigned long long* sums = nullptr;
    st = hip_status(hipMalloc(&sums, kParts * sizeof(unsigned long long)), "hipMalloc");
    if (st == NACC_OK)
        st = hip_status(hipMemsetAsync(sums, 0, kParts * sizeof(unsigned long long), p->own), "memset");
    for (int i = 0; st == NACC_OK && i < kParts; ++i) {
        const int64_t n = parts[i].first != nullptr ? static_cast<int64_t>(parts[i].second) : 0;
        if (n == 0) continue;
        const int64_t blocks = std::min<int64_t>(2048, (n + 255) / 256);
        hipLaunchKernelGGL(checksum_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, p->own,
                           static_cast<const uint32_t*>(parts[i].first), n, sums + i);
        st = check_launch("checksum");
    }
    snap->sums.assign(kParts + 1, 0ull);
    snap->sums[kParts] = static_cast<unsigned long long>(total);
    if (st == NACC_OK) st = hip_status(hipStreamSynchronize(p->own), "synchronize");
    if (st == NACC_OK)
        st = hip_status(hipMemcpy(snap->sums.data(), sums, kParts * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost), "snapshot copy");
    if (sums != nullptr) (void)hipFree(sums);
    return st;
}

// Milliseconds per replay of the step captured under `t`; also its snapshot.
int time_setting(nacc_plan* p, const nacc_tuning& t, int repeats, hipEvent_t a, hipEvent_t b, float* ms,
                 Snapshot* snap) {
    int st = nacc_set_tuning(&t);
    if (st != NACC_OK) return st;
    hipGraphExec_t exec = nullptr;
    if ((st = capture(p, run_step, &exec)) != NACC_OK) return st;
    st = hip_status(hipGraphLaunch(exec, p->own), "graph launch");
    if (st == NACC_OK) st = hip_status(hipStreamSynchronize(p->own), "synchronize");
    if (st == NACC_OK) st = snapshot(p, snap);
    if (st == NACC_OK) st = hip_status(hipGraphLaunch(exec, p->own), "graph launch");
    if (st == NACC_OK) st = hip_status(hipEventRecord(a, p->own), "event record");
    for (int i = 0; st == NACC_OK && i < repeats; ++i) st = hip_status(hipGraphLaunch(exec, p->own), "graph launch");
    if (st == NACC_OK) st = hip_status(hipEventRecord(b, p->own), "event record");
    if (st == NACC_OK) st = hip_status(hipEventSynchronize(b), "event synchronize");
    if (st == NACC_OK) st = hip_status(hipEventElapsedTime(ms, a, b), "elapsed time");
    (void)hipGraphExecDestroy(exec);
    if (st == NACC_OK) *ms /= static_cast<float>(repeats);
    return st;
}

int set_knob(nacc_tuning* t, int knob, int value) {
    switch (knob) {
        case 0: t->march_waves_per_group = value; break;
        case 1: t->render_cached_chunks = value; break;
        case 2: t->render_mse_max_blocks = value; break;
        default: t->render_prefetch = value; break;
    }
    return value;
}

int get_knob(const nacc_tuning& t, int knob) {
    switch (knob) {
        case 0: return t.march_waves_per_group;
        case 1: return t.render_cached_chunks;
        case 2: return t.render_mse_max_blocks;
        default: return t.render_prefetch;
    }
}

int autotune(nacc_plan* p, int repeats, nacc_tuning* best_out, float* best_ms_out) {
    static const std::vector<int> kValues[4] = {
        {1, 2, 4, 8, 16}, {1, 2, 3, 4}, {4096, 8192, 16384, 65536}, {0, 1}};
    const bool training = p->d.target != nullptr;
    nacc_tuning best;
    nacc_get_tuning(&best);
    hipEvent_t a = nullptr, b = nullptr;
    int st = hip_status(hipEventCreate(&a), "event create");
    if (st == NACC_OK) st = hip_status(hipEventCreate(&b), "event create");
    Snapshot reference, trial_snap;
    float best_ms = 0.0f;
    if (st == NACC_OK) st = time_setting(p, best, repeats, a, b, &best_ms, &reference);
    // two rounds of coordinate descent: a knob's best value can change once
    // the later knobs have moved
    for (int round = 0; round < 2; ++round)
    for (int knob = 0; st == NACC_OK && knob < 4; ++knob) {
        if (!training && knob >= 1) break;  // the rendering knobs act on the fused loss kernel only
        for (int v : kValues[knob]) {
            if (v == get_knob(best, knob)) continue;
            nacc_tuning trial = best;
            set_knob(&trial, knob, v);
            float ms = 0.0f;
            st = time_setting(p, trial, repeats, a, b, &ms, &trial_snap);
            if (st != NACC_OK) break;
            if (trial_snap.sums != reference.sums) continue;  // changed a result: rejected
            if (ms < best_ms) {
                best = trial;
                best_ms = ms;
            }
        }
    }
    (void)nacc_set_tuning(&best);
    if (a != nullptr) (void)hipEventDestroy(a);
    if (b != nullptr) (void)hipEventDestroy(b);
    if (st != NACC_OK) return st;
    if (best_out != nullptr) *best_out = best;
    if (best_ms_out != nullptr) *best_ms_out = best_ms;
    return NACC_OK;
}

}  // namespace

extern "C" {

int nacc_plan_create(const nacc_plan_desc* desc, nacc_plan** out) {
    clear_error();
    NACC_REQUIRE(out != nullptr, NACC_EINVAL, "out must be non-NULL");
    int st = validate(desc);
    if (st != NACC_OK) return st;
    auto* p = new nacc_plan();
    p->d = *desc;
    st = hip_status(hipGetDevice(&p->device), "get device");
    p->march_ws_bytes = static_cast<size_t>(nacc_march_workspace_size(desc->n_rays, &desc->grid, &desc->params));
    p->mse_ws_bytes = static_cast<size_t>(nacc_render_mse_workspace_size(desc->n_rays));
    if (st == NACC_OK && p->march_ws_bytes > 0) st = hip_status(hipMalloc(&p->march_ws, p->march_ws_bytes), "hipMalloc");
    if (st == NACC_OK && p->mse_ws_bytes > 0 && desc->target != nullptr)
        st = hip_status(hipMalloc(&p->mse_ws, p->mse_ws_bytes), "hipMalloc");
    if (st == NACC_OK) st = hip_status(hipStreamCreateWithFlags(&p->own, hipStreamNonBlocking), "stream create");
    if (st != NACC_OK) {
        const std::string msg = nacc_last_error();
        nacc_plan_destroy(p);
        return set_error(st, "%s", msg.c_str());
    }
    *out = p;
    return NACC_OK;
}

int nacc_plan_destroy(nacc_plan* p) {
    clear_error();
    if (p == nullptr) return NACC_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != p->device) (void)hipSetDevice(p->device);
    if (p->own != nullptr) (void)hipStreamSynchronize(p->own);
    drop_graphs(p);
    if (p->march_ws != nullptr) (void)hipFree(p->march_ws);
    if (p->mse_ws != nullptr) (void)hipFree(p->mse_ws);
    if (p->own != nullptr) (void)hipStreamDestroy(p->own);
    if (prev >= 0 && prev != p->device) (void)hipSetDevice(prev);
    delete p;
    return NACC_OK;
}

int nacc_plan_step(nacc_plan* p, void* stream) {
    clear_error();
    int st = check_device(p);
    return st != NACC_OK ? st : run_step(p, as_stream(stream));
}

int nacc_plan_update(nacc_plan* p, void* stream) {
    clear_error();
    int st = check_device(p);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(p->d.occ != nullptr, NACC_EINVAL, "the plan has no grid update (occ is NULL)");
    return run_update(p, as_stream(stream));
}

int nacc_plan_capture_step(nacc_plan* p) {
    clear_error();
    int st = check_device(p);
    if (st != NACC_OK) return st;
    st = capture_all(p);
    if (st == NACC_OK) st = hip_status(hipStreamSynchronize(p->own), "synchronize");
    return st;
}

int nacc_plan_launch(nacc_plan* p, int32_t with_update, void* stream) {
    clear_error();
    int st = check_device(p);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(p->step_exec != nullptr, NACC_EINVAL, "nacc_plan_capture_step has not been called");
    NACC_REQUIRE(!with_update || p->update_exec != nullptr, NACC_EINVAL, "the plan has no grid update");
    st = hip_status(hipGraphLaunch(p->step_exec, as_stream(stream)), "graph launch");
    if (st == NACC_OK && with_update) st = hip_status(hipGraphLaunch(p->update_exec, as_stream(stream)), "graph launch");
    return st;
}

int nacc_plan_autotune(nacc_plan* p, int32_t repeats, void* stream, nacc_tuning* best, float* best_ms) {
    clear_error();
    int st = check_device(p);
    if (st != NACC_OK) return st;
    NACC_REQUIRE(repeats >= 1, NACC_EINVAL, "repeats must be >= 1");
    if ((st = hip_status(hipStreamSynchronize(as_stream(stream)), "synchronize")) != NACC_OK) return st;
    const bool had_graphs = p->step_exec != nullptr;
    drop_graphs(p);
    st = autotune(p, repeats, best, best_ms);
    if (st == NACC_OK && had_graphs) st = capture_all(p);
    if (st == NACC_OK) st = hip_status(hipStreamSynchronize(p->own), "synchronize");
    return st;
}

}  // extern "C"
