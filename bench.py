#!/usr/bin/env python3
"""Benchmark of occupancy-grid ray marching + packed differentiable rendering
on one MI355X.

Default workload (train_262k): one training step = march (count, scan, fill)
-> synthetic field at the samples -> fused render forward + MSE + backward,
plus the occupancy-grid update (decay, 2^18 random cells, field, max, pack)
every 16 steps.  262,144 rays, 128^3 grid of 32 blobs.  Inputs are seeded,
synthetic and resident in HBM before the timed region; outputs go to
capacity-sized buffers, so no step waits on the host.  The step runs as the
library's step plan (nacc_plan): its launch parameters tuned by the plan on
this step, then the step and the grid update captured by the library into
two HIP graphs and replayed; per-phase times come from an eager pass with
HIP events on the launch stream.

--workload dynamic_64: 64 frames with their own grids (~262k rays, Poisson
counts per frame); 64 per-frame plain calls (each sized by a host read of the
sample total, like the paper's API) against one batched graph-captured step
over all frames; their outputs are checked bit for bit.  dynamic_64_shared:
the same frames marched through one grid shared by all frames (the maximum
of their densities over time).

--workload unbounded_262k / unbounded_contract_262k: 262,144 rays from
inside the unit ball, cone-scaled steps to far = 1e4, a scene defined in
contracted coordinates; four world-space cascades, or one grid over the
contracted space read through the contraction (at most 1024 samples per
ray).

--workload images_8: four 800x800 and four 1920x1080 images rendered
forward: one fused launch for all images (marching, field and render per
wavefront) against one plain call sequence per image, bit for bit.

--workload attrs_262k: the training rays with 16-channel feature vectors
rendered (background, opacity threshold) forward and backward.

--workload plain_fwd_4k: 4,096 rays, 8 blobs, forward only, no early
termination.

Prints one JSON line.  --gpus N > 1 is not supported (one GPU).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "marched+rendered samples/s (fwd+bwd) and % HBM peak; batched vs plain, 1 GPU"
HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s
EMA_EVERY = 16
EMA_CELLS = 1 << 18
EMA_DECAY = 0.95
THRESHOLD = 0.01


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="train_262k",
                    choices=["train_262k", "plain_fwd_4k", "unbounded_262k",
                             "unbounded_contract_262k", "dynamic_64", "dynamic_64_shared",
                             "images_8", "attrs_262k"])
    ap.add_argument("--form", choices=["plan", "graph", "eager"], default="plan",
                    help="time the step as the library's step plan (its own HIP graphs and "
                         "tuner), captured in HIP graphs through torch, or launched eagerly "
                         "(training workloads; steps with visibility pruning, the attribute "
                         "and image workloads use torch graphs for \"plan\")")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning", default=None,
                    help="launch parameters to use instead of tuning, as key=value,... (the "
                         "fields of nacc_tuning), e.g. to take hardware counters under the "
                         "setting a tuned run chose")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rays", type=int, default=131072)
    ap.add_argument("--skip-field", choices=["auto", "on", "off"], default="auto",
                    help="march with the grid's skip buffer (empty-space skipping: its halo bits "
                         "let the count pass test runs of 8 to 32 candidates at once); auto uses "
                         "it for every workload")
    ap.add_argument("--alpha-thre", type=float, default=None,
                    help="prune the marched samples by visibility before shading them, as the "
                         "paper's ray_marching with sigma_fn (T >= early_stop_eps, alpha >= this; "
                         "the paper's listing uses 1e-2)")
    ap.add_argument("--attrs-channels", type=int, default=16,
                    help="attrs_262k: feature channels per sample")
    ap.add_argument("--rows", choices=["all", "none"], default="all",
                    help="with the default workload (train_262k) also measure the HBM probe "
                         "and the other workloads (plain_fwd_4k, unbounded_262k, "
                         "unbounded_contract_262k, dynamic_64, images_8) and attach them to "
                         "the JSON line as rows")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB on the device (a plain copy of "
                         "known size, for calibrating hardware traffic counters)")
    return ap.parse_args()


def fixed_tuning(args, nacc):
    """Sets the launch parameters given by --tuning; returns them all."""
    kv = dict(item.split("=", 1) for item in args.tuning.split(",") if item)
    nacc._lib.set_tuning(**{k: int(v) for k, v in kv.items()})
    tuned = nacc._lib.get_tuning()
    log(f"tuning set: {tuned}")
    return tuned


def use_skip(args, w):
    """Whether a workload marches with the grid's skip buffer."""
    if args.skip_field != "auto":
        return args.skip_field == "on"
    return True


def grid_label(w):
    lookup = getattr(w, "lookup", "aabb")
    if lookup == "cascade":
        return f"{w.cascades} cascades of {w.res}^3 bit-packed"
    if lookup == "contract":
        return (f"{w.res}^3 bit-packed over the contracted space [-2,2]^3, "
                f"at most {w.max_per_ray} samples per ray")
    return f"{w.res}^3 bit-packed"


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


class Step:
    """Buffers and launches of one step over the rays with grid(s) `grid`
    (everything on torch's current stream).  grid_id (optional, per ray)
    picks the grid and the field's centre set; ray_set (optional) picks the
    centre set alone (rays of several frames through one shared grid), and
    update_set the centre set the grid update reads per drawn cell."""

    def __init__(self, torch, nacc, w, rays_o, rays_d, targets, grid, field, grid_id=None,
                 skip_field=False, forward_only=False, loss_rays=0, seed=0, alpha_thre=None,
                 ray_set=None, update_set=None):
        self.torch, self.nacc, self.lib = torch, nacc, nacc._lib
        dev = rays_o.device
        self.w = w
        self.n = rays_o.shape[0]
        self.rays_o, self.rays_d, self.target = rays_o, rays_d, targets
        self.grid, self.field = grid, field
        self.grid_id = grid_id
        self.ray_set = grid_id if ray_set is None else ray_set
        self.update_set = update_set
        self.forward_only = forward_only
        self.loss_rays = loss_rays
        self.params = self.lib.march_params(w.near, w.far, w.dt, getattr(w, "dt_max", 1e10),
                                            getattr(w, "cone", 0.0),
                                            max_per_ray=getattr(w, "max_per_ray", 0))
        # sample buffers no step can overflow, so no step reads the total back
        self.capacity = self.n * self.lib.march_max_samples_per_ray(grid.desc, self.params)
        n, cap = self.n, self.capacity
        i32, f32 = torch.int32, torch.float32
        self.packed = torch.empty((n, 2), dtype=i32, device=dev)
        self.total = torch.empty(1, dtype=torch.int64, device=dev)
        self.ws = torch.empty(max(self.lib.march_workspace_size(n, grid.desc, self.params), 1),
                              dtype=torch.uint8, device=dev)
        self.ray_indices = torch.empty(cap, dtype=i32, device=dev)
        self.t_starts = torch.empty(cap, dtype=f32, device=dev)
        self.t_ends = torch.empty(cap, dtype=f32, device=dev)
        self.status = torch.zeros(1, dtype=i32, device=dev)
        self.sigmas = torch.empty(cap, dtype=f32, device=dev)
        self.rgbs = torch.empty((cap, 3), dtype=f32, device=dev)
        self.g_sigmas = torch.empty(cap, dtype=f32, device=dev)
        self.g_rgbs = torch.empty((cap, 3), dtype=f32, device=dev)
        self.color = torch.empty((n, 3), dtype=f32, device=dev)
        self.opacity = torch.empty(n, dtype=f32, device=dev)
        self.depth = torch.empty(n, dtype=f32, device=dev)
        self.loss = torch.empty(1, dtype=f32, device=dev)
        self.mse_ws = torch.empty(max(self.lib.render_mse_workspace_size(n), 1), dtype=torch.uint8,
                                  device=dev)
        self.ema_cells = torch.empty(EMA_CELLS, dtype=i32, device=dev)
        self.ema_pos = torch.empty((EMA_CELLS, 3), dtype=f32, device=dev)
        self.ema_sigma = torch.empty(EMA_CELLS, dtype=f32, device=dev)
        self.updates = torch.zeros(1, dtype=torch.int64, device=dev)  # read by the kernel
        self.seed = seed
        self.skip = grid.skip if skip_field else None
        # visibility pruning (the paper's ray_marching with sigma_fn): densities
        # of all marched samples, then only the kept ones are shaded and rendered
        self.prune = alpha_thre is not None
        self.alpha_thre = alpha_thre
        self.cur = (self.packed, self.ray_indices, self.t_starts, self.t_ends, self.total)
        if self.prune:
            self.sig_all = torch.empty(cap, dtype=f32, device=dev)
            self.keep = torch.empty(cap, dtype=torch.uint8, device=dev)
            self.prune_ws = torch.empty(max(self.lib.prune_workspace_size(n), 1), dtype=torch.uint8,
                                        device=dev)
            self.cur = (torch.empty((n, 2), dtype=i32, device=dev),
                        torch.empty(cap, dtype=i32, device=dev),
                        torch.empty(cap, dtype=f32, device=dev),
                        torch.empty(cap, dtype=f32, device=dev),
                        torch.empty(1, dtype=torch.int64, device=dev))
        self.PHASES = (("march_count", "march_fill") + (("field_sigma", "prune") if self.prune
                                                         else ()) + ("field", "render", "grid_update"))

    def march_count(self):
        self.lib.march_count(self.rays_o, self.rays_d, self.grid_id, self.grid.bits, self.grid.desc,
                             self.params, self.packed, self.total, self.ws, self.skip)

    def march_fill(self):
        self.lib.march_fill(self.rays_o, self.rays_d, self.grid_id, self.grid.bits, self.grid.desc,
                            self.params, self.packed, self.ray_indices, self.t_starts, self.t_ends,
                            self.status, self.skip, self.ws)

    def field_sigma(self):
        """Densities only, of every marched sample (the sigma_fn of the paper)."""
        self.lib.synth_field_samples(self.field.table, self.field.n_blobs, self.field.n_sets,
                                     self.rays_o, self.rays_d, self.ray_set, self.ray_indices,
                                     self.t_starts, self.t_ends, self.sig_all, None, self.total)

    def prune_samples(self):
        packed_k, ri_k, ts_k, te_k, total_k = self.cur
        self.lib.prune_count(self.packed, self.t_starts, self.t_ends, self.sig_all,
                             self.w.early_stop_eps, self.alpha_thre, self.keep, packed_k, total_k,
                             self.prune_ws)
        self.lib.prune_fill(self.packed, self.t_starts, self.t_ends, self.sig_all, self.keep,
                            packed_k, ri_k, ts_k, te_k, None, self.status)

    def field_eval(self):
        packed, ri, ts, te, total = self.cur
        self.lib.synth_field_samples(self.field.table, self.field.n_blobs, self.field.n_sets,
                                     self.rays_o, self.rays_d, self.ray_set, ri, ts, te,
                                     self.sigmas, self.rgbs, total)

    def render(self):
        packed, _, ts, te, _ = self.cur
        if self.forward_only:
            self.lib.render_fwd(packed, ts, te, self.sigmas, self.rgbs,
                                self.w.early_stop_eps, self.color, self.opacity, self.depth)
        else:
            self.lib.render_fwd_bwd_mse(packed, ts, te, self.sigmas,
                                        self.rgbs, self.w.early_stop_eps, self.target, self.color,
                                        self.opacity, self.depth, self.g_sigmas, self.g_rgbs,
                                        self.loss, self.mse_ws, self.loss_rays)

    def grid_update(self):
        lib, g = self.lib, self.grid
        lib.grid_decay(g.occ, EMA_DECAY)
        lib.grid_sample_cells(self.seed, self.updates, EMA_CELLS, g.desc, g.n_grids,
                              self.ema_cells, self.ema_pos)
        # a contraction-lookup grid draws its positions in the contracted space
        table = (self.field.table_contracted if g.lookup == self.lib.LOOKUP_CONTRACT
                 else self.field.table)
        per_cell = self.field.n_sets > 1 and self.update_set is None
        lib.synth_field_points(table, self.field.n_blobs, self.field.n_sets,
                               self.ema_pos, self.update_set, self.ema_sigma,
                               point_cell=self.ema_cells if per_cell else None,
                               cells_per_set=g.res ** 3)
        lib.grid_update_max(g.occ, self.ema_cells, self.ema_sigma)
        lib.grid_pack(g.occ, THRESHOLD, g.bits)
        if g.skip is not None:
            lib.grid_build_skip(g.bits, g.desc, g.skip)
        self.updates.add_(1)

    def step(self, update=False, events=None):
        """One step; events (optional): len(PHASES) + 1 HIP events, recorded
        before each phase and after the last."""
        fns = [self.march_count, self.march_fill]
        if self.prune:
            fns += [self.field_sigma, self.prune_samples]
        fns += [self.field_eval, self.render]
        for j, fn in enumerate(fns):
            if events is not None:
                events[j].record()
            fn()
        if events is not None:
            events[len(fns)].record()
        if update:
            self.grid_update()
        if events is not None:
            events[len(fns) + 1].record()

    def plan(self):
        """This step (and its grid update) as the library's step plan: the
        same launches on the same buffers, with the synthetic field as native
        stages, captured and replayed by the library itself."""
        if self.prune:
            raise ValueError("a step plan has no visibility-pruning stage")
        lib, f, g = self.lib, self.field, self.grid
        field = lib.synth_samples_stage(f.table, f.n_blobs, f.n_sets, self.rays_o, self.rays_d,
                                        self.ray_set, self.ray_indices, self.t_starts,
                                        self.t_ends, self.sigmas, self.rgbs, self.total)
        table = f.table_contracted if g.lookup == lib.LOOKUP_CONTRACT else f.table
        per_cell = f.n_sets > 1 and self.update_set is None
        update_field = lib.synth_points_stage(table, f.n_blobs, f.n_sets, self.ema_pos,
                                              self.update_set, self.ema_sigma,
                                              point_cell=self.ema_cells if per_cell else None,
                                              cells_per_set=g.res ** 3)
        train = not self.forward_only
        return lib.Plan(self.rays_o, self.rays_d, g.bits, g.desc, self.params, self.packed,
                        self.ray_indices, self.t_starts, self.t_ends, self.total, field,
                        self.sigmas, self.rgbs, self.color, self.opacity, self.depth,
                        early_stop_eps=self.w.early_stop_eps, grid_id=self.grid_id,
                        grid_skip=self.skip, status=self.status,
                        target=self.target if train else None, loss_rays=self.loss_rays,
                        g_sigmas=self.g_sigmas if train else None,
                        g_rgbs=self.g_rgbs if train else None, loss=self.loss if train else None,
                        occ=g.occ, decay=EMA_DECAY, threshold=THRESHOLD, seed=self.seed,
                        update_counter=self.updates, update_cell_ids=self.ema_cells,
                        update_positions=self.ema_pos, update_values=self.ema_sigma,
                        update_field=update_field)

    def outputs(self):
        """Tensors a change of launch parameters must leave bit-identical."""
        return (self.packed, self.ray_indices[:1 << 20], self.t_starts[:1 << 20], self.color,
                self.g_sigmas[:1 << 20], self.g_rgbs[:1 << 18])


def capture(torch, fn):
    """fn captured in a HIP graph (warmed up on a side stream first)."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def algorithmic_bytes(n_rays, e, v, forward_only=False):
    """Bytes each phase must move (reads of its inputs + writes of its
    outputs, each once), for one step with e samples of which v precede the
    early-termination cut."""
    return {
        # rays in (24 B/ray), counts + starts out and back (4 + 4 + 4 B/ray)
        "march_count": 24 * n_rays + 12 * n_rays,
        # rays + packed_info in, 12 B per sample out
        "march_fill": 32 * n_rays + 12 * e,
        # ray index + interval in (12 B), sigma + rgb out (16 B), rays once
        "field": 28 * e + 24 * n_rays,
        # forward: kept samples read once (24 B) + packed_info in, colour /
        # opacity / depth out; fused: also gradients of every sample written
        # (16 B) and the target read (40 B/ray in all)
        "render": (24 * v + 28 * n_rays) if forward_only else (24 * v + 16 * e + 40 * n_rays),
    }


# The synthetic field per sample: per blob 3 differences, the squared
# distance (multiply, 2 multiply-adds), the exponent argument, exp2 and the
# accumulation (9); the colour's 3 affine rows (9 multiply-adds) and 3
# sigmoids (multiply, exp2, add, reciprocal: 12); the midpoint and position
# (8).  The render per sample: tau (2), the chunk scan (6), two exponentials
# with their scalings (4), the opacity series (12), the weight (1) and five
# accumulations (5).
FIELD_OPS_PER_BLOB = 9
FIELD_OPS_FIXED = 29
RENDER_OPS = 30


# VALU lane operations per second: the 157.3 TFLOP/s FP32 vector figure with
# an FMA counted as one operation, 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz.
# Single-issue, unpacked code (the library compiles without packed FP32) is
# held near half of it, 16 lanes per SIMD per clock; the counters show the
# count kernels issuing slightly above that half, so only the full figure is
# a ceiling.
ALU_PEAK = 256 * 4 * 32 * 2.4e9


def lattice_candidates(w, rays_o, rays_d):
    """Lattice candidates of the rays, each of which the count pass decides
    (FP64 slab clip; cone steps by running the recurrence in FP32 for all rays
    at once)."""
    import numpy as np
    o = rays_o.astype(np.float64)
    d = rays_d.astype(np.float64)
    cascades = getattr(w, "cascades", 1)
    lo = np.asarray(w.box[:3], np.float64) * 2.0 ** (cascades - 1)
    hi = np.asarray(w.box[3:], np.float64) * 2.0 ** (cascades - 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        ta = (lo - o) / d
        tb = (hi - o) / d
    t_in = np.nanmax(np.minimum(ta, tb), axis=1)
    t_out = np.nanmin(np.maximum(ta, tb), axis=1)
    if getattr(w, "lookup", "aabb") == "contract":  # no clip box
        t_in = np.full(o.shape[0], -np.inf)
        t_out = np.full(o.shape[0], np.inf)
    t_near = np.maximum(t_in, w.near)
    t_far = np.minimum(t_out, w.far)
    hit = t_near < t_far
    cone = getattr(w, "cone", 0.0)
    if cone == 0.0:
        return int(np.ceil((t_far[hit] - t_near[hit]) / w.dt).sum())
    t = t_near[hit].astype(np.float32)
    tf = t_far[hit].astype(np.float32)
    c, dt, dmax = np.float32(cone), np.float32(w.dt), np.float32(getattr(w, "dt_max", 1e10))
    n = 0
    live = t < tf
    while live.any():
        n += int(live.sum())
        t = np.where(live, t + np.minimum(np.maximum(t * c, dt), dmax), t)
        live = t < tf
    return n


RENDER_SOURCES = ("paper_2210_04847_amd/csrc/render.hip+paper_2210_04847_amd/csrc/transmittance.h+"
                  "paper_2210_04847_amd/csrc/common.h")
MARCH_SOURCES = ("paper_2210_04847_amd/csrc/march.hip+paper_2210_04847_amd/csrc/lattice.h+"
                 "paper_2210_04847_amd/csrc/scan.h+paper_2210_04847_amd/csrc/common.h")


def recorded_traffic(kernel, source, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    counter summaries (profiles/*.md, lines 'traffic_record: ...'), or None
    when none was taken on this workload or none matches the current source
    of the kernel (the counters are then stale)."""
    import glob
    import hashlib
    # `source`: the kernel's files joined by '+', hashed in that order
    h = hashlib.sha256()
    for part in source.split("+"):
        h.update(open(os.path.join(ROOT, part), "rb").read())
    digest = h.hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic_record:"):
                continue
            kv = dict(item.split("=", 1) for item in line.split()[1:])
            if (kv.get("kernel") == kernel and kv.get("workload") == workload
                    and kv.get("source") == source and kv.get("sha256_16") == digest):
                return float(kv["read_bytes"]) + float(kv["write_bytes"])
    return None


def recorded_valu(phase, source, workload):
    """VALU instructions per step of a phase's kernels on `workload` from the
    committed counter summaries (lines 'valu_record: ...'), or None when
    none matches the current source."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for part in source.split("+"):
        h.update(open(os.path.join(ROOT, part), "rb").read())
    digest = h.hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("valu_record:"):
                continue
            kv = dict(item.split("=", 1) for item in line.split()[1:])
            if (kv.get("phase") == phase and kv.get("workload") == workload
                    and kv.get("source") == source and kv.get("sha256_16") == digest):
                return float(kv["valu_insts"])
    return None


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) and usable threads."""
    name = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return name, usable


def _oracle_chunk(w, inp, mask, lookup, a, b, forward_only):
    """The oracle, as it stands, on rays [a, b): brute-force marching, FP64
    field, FP64 forward (+ MSE + backward).  Returns the samples marched."""
    import numpy as np

    import oracle
    o, d = inp["rays_o"][a:b], inp["rays_d"][a:b]
    packed, ri, ts, te = oracle.march(o, d, mask, w.res, np.asarray(w.box, np.float32), w.near,
                                      w.far, w.dt, dt_max=getattr(w, "dt_max", 1e10),
                                      cone=getattr(w, "cone", 0.0), lookup=lookup,
                                      n_grids=getattr(w, "cascades", 1),
                                      max_per_ray=getattr(w, "max_per_ray", 0))
    pos = oracle.sample_positions(o, d, ri, ts, te)
    sig, rgb = oracle.blob_field(inp["scene"], pos)
    fwd = oracle.render_fwd(packed, ts, te, sig, rgb, w.early_stop_eps)
    if not forward_only:
        _, g_color = oracle.mse_loss_and_grad(fwd["color"], inp["targets"][a:b])
        oracle.render_bwd(packed, ts, te, sig, rgb, g_color, eps=w.early_stop_eps)
    return int(ri.size)


def cpu_baseline(w, inp, n_single, n_all, forward_only=False, max_threads=16):
    """The oracle timed on the host: one thread on the first n_single rays,
    then all usable threads (at most max_threads; rays split into chunks run
    by a thread pool, the oracle's C calls release the interpreter lock) on
    the first n_all rays.  The arithmetic per ray is the oracle's, unchanged."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    mask = oracle.grid_threshold(inp["occ"], THRESHOLD)
    lookup = {"contract": oracle.LOOKUP_CONTRACT, "cascade": oracle.LOOKUP_CASCADE}.get(
        getattr(w, "lookup", "aabb"), oracle.LOOKUP_AABB)
    name, usable = cpu_model()
    threads = max(1, min(usable, max_threads))
    t0 = time.perf_counter()
    e1 = _oracle_chunk(w, inp, mask, lookup, 0, n_single, forward_only)
    dt1 = time.perf_counter() - t0
    chunk = max(1, -(-n_all // (threads * 8)))
    bounds = [(a, min(a + chunk, n_all)) for a in range(0, n_all, chunk)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as pool:
        ek = sum(pool.map(lambda ab: _oracle_chunk(w, inp, mask, lookup, ab[0], ab[1],
                                                   forward_only), bounds))
    dtk = time.perf_counter() - t0
    what = "march+field+fwd" if forward_only else "march+field+fwd+bwd"
    return {"value": ek / dtk, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_all} of {inp['rays_o'].shape[0]} rays ({ek} samples), {what}, "
                      f"{threads} threads over rays, {dtk:.1f} s; host: {name}, {usable} usable "
                      f"hardware threads",
            "single_thread": {"value": e1 / dt1, "unit": "samples/s",
                              "sample": f"first {n_single} rays ({e1} samples), {dt1:.1f} s"},
            "cpu_model": name, "usable_threads": usable}


def hbm_probe(torch, nacc, mib=4096, repeats=8):
    """Achievable HBM bandwidth on this device: read-only, write-only and
    copy passes of the library's streaming probe over buffers of `mib` MiB
    (well past the 256 MB last-level cache), best over a sweep of launch
    sizes, HIP events on the launch stream.  Copy counts read + write bytes."""
    import numpy as np
    lib = nacc._lib
    n_bytes = mib << 20
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for kind, name, factor in ((lib.PROBE_READ, "read", 1), (lib.PROBE_WRITE, "write", 1),
                               (lib.PROBE_COPY, "copy", 2)):
        best = (0.0, 0)
        for blocks in (2048, 4096, 8192, 16384, 32768):
            lib.probe_hbm(kind, src, dst, n_bytes, blocks)  # warm-up
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(repeats + 1)]
            ev[0].record()
            for k in range(repeats):
                lib.probe_hbm(kind, src, dst, n_bytes, blocks)
                ev[k + 1].record()
            torch.cuda.synchronize()
            ms = float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(repeats)]))
            gbps = factor * n_bytes / (ms * 1e-3) / 1e9
            if gbps > best[0]:
                best = (gbps, blocks)
        out[name] = {"GB/s": best[0], "blocks": best[1], "frac_of_peak": best[0] * 1e9 / HBM_PEAK}
    del src, dst
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    out["bytes"] = n_bytes
    return out


def kept_fraction(st, e_last):
    """Rendered samples before the early-termination cut / rendered samples,
    from one forward with per-ray kept counts (outside the timed region)."""
    torch = st.torch
    packed, _, ts, te, _ = st.cur
    kept = torch.empty(st.n, dtype=torch.int32, device="cuda")
    st.lib.render_fwd(packed, ts, te, st.sigmas, st.rgbs, st.w.early_stop_eps,
                      st.color, st.opacity, st.depth, None, kept)
    return int(kept.sum().item()) / max(e_last, 1)


def phase_timing(torch, st, steps, first_index, updates=True):
    """Per-phase HIP-event times of `steps` eager steps (grid update every 16
    steps, if `updates`)."""
    import numpy as np
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(st.PHASES) + 1)]
              for _ in range(steps)]
    upd = [updates and (first_index + k) % EMA_EVERY == 0 for k in range(steps)]
    for k in range(steps):
        st.step(update=upd[k], events=events[k])
    torch.cuda.synchronize()
    out = {p: [] for p in st.PHASES}
    for k in range(steps):
        for j, p in enumerate(st.PHASES):
            if p == "grid_update" and not upd[k]:
                continue
            out[p].append(events[k][j].elapsed_time(events[k][j + 1]))
    return {p: (float(np.mean(v)) if v else 0.0) for p, v in out.items()}


def step_latency(torch, launch, n):
    """p10 / p50 / p90 of n single launches, each bracketed by HIP events on
    the launch stream (ms)."""
    import numpy as np
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n)]
    for a, b in ev:
        a.record()
        launch()
        b.record()
    torch.cuda.synchronize()
    v = np.array([a.elapsed_time(b) for a, b in ev])
    return {"p10": float(np.percentile(v, 10)), "p50": float(np.percentile(v, 50)),
            "p90": float(np.percentile(v, 90)), "launches": n}


def unfused_render(torch, st, repeats=16):
    """The render forward and backward as two calls (nacc_render_fwd, then
    nacc_render_bwd with the MSE gradient of the colour as a given input) on
    the step's samples, timed per call with HIP events; algorithmic bytes:
    forward 24 B per sample before the cut + 28 B per ray (packed_info in,
    colour / opacity / depth out); backward the same samples again, 16 B of
    gradients written for every sample, packed_info and g_color in
    (20 B per ray)."""
    import numpy as np
    lib = st.lib
    e = int(st.total.item())
    n = st.n
    ts, te, sg, rg = st.t_starts[:e], st.t_ends[:e], st.sigmas[:e], st.rgbs[:e]
    color = torch.empty_like(st.color)
    opac = torch.empty_like(st.opacity)
    depth = torch.empty_like(st.depth)
    kept = torch.empty(n, dtype=torch.int32, device=st.color.device)
    gs = torch.empty(e, dtype=torch.float32, device=st.color.device)
    gr = torch.empty((e, 3), dtype=torch.float32, device=st.color.device)
    eps = st.w.early_stop_eps
    lib.render_fwd(st.packed, ts, te, sg, rg, eps, color, opac, depth, kept=kept)
    # the loss's gradient (an input here), as the fused kernel forms it
    g_color = (color - st.target) * float(np.float32(2.0 / (3 * n)))
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(repeats)]
    for a, b, c in ev:
        a.record()
        lib.render_fwd(st.packed, ts, te, sg, rg, eps, color, opac, depth)
        b.record()
        lib.render_bwd(st.packed, ts, te, sg, rg, eps, g_color, None, None, gs, gr)
        c.record()
    torch.cuda.synchronize()
    fwd = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    bwd = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    v = int(kept.sum().item())
    fwd_bytes = 24 * v + 28 * n
    bwd_bytes = 24 * v + 16 * e + 20 * n
    same = bool(torch.equal(gs.view(torch.int32), st.g_sigmas[:e].view(torch.int32)) and
                torch.equal(color.view(torch.int32), st.color.view(torch.int32)))
    return {"fwd_ms": fwd, "bwd_ms": bwd, "samples_per_s": e / ((fwd + bwd) * 1e-3),
            "alg_bytes": fwd_bytes + bwd_bytes,
            "hbm_frac": (fwd_bytes + bwd_bytes) / ((fwd + bwd) * 1e-3) / HBM_PEAK,
            "fwd_hbm_frac": fwd_bytes / (fwd * 1e-3) / HBM_PEAK,
            "bwd_hbm_frac": bwd_bytes / (bwd * 1e-3) / HBM_PEAK,
            "identical_to_fused": same}


def bench_train(args, torch, nacc):
    import synth
    unbounded = args.workload in synth.UNBOUNDED_WORKLOADS
    w = (synth.UNBOUNDED_WORKLOADS if unbounded else synth.WORKLOADS)[args.workload]
    forward_only = args.workload == "plain_fwd_4k"
    t_gen = time.perf_counter()
    inp = synth.unbounded_inputs(w) if unbounded else synth.workload_inputs(w)
    log(f"inputs generated in {time.perf_counter() - t_gen:.1f} s")
    dev = torch.device("cuda")
    t = lambda a: torch.from_numpy(a).to(dev)
    if unbounded:
        grid = nacc.OccupancyGrid(w.box, w.res, n_grids=w.cascades, lookup=w.lookup, device=dev)
    else:
        grid = nacc.OccupancyGrid(w.box, w.res, device=dev)
    grid.set_occupancy(t(inp["occ"]), THRESHOLD)
    field = nacc.BlobField(inp["scene"], device=dev)
    st = Step(torch, nacc, w, t(inp["rays_o"]), t(inp["rays_d"]), t(inp["targets"]), grid, field,
              skip_field=use_skip(args, w), forward_only=forward_only, seed=4000 + w.seed_base,
              alpha_thre=args.alpha_thre)
    torch.cuda.synchronize()
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    form = args.form if not (args.form == "plan" and st.prune) else "graph"
    plan = st.plan() if form == "plan" else None
    tuned = None
    if args.tuning:
        tuned = fixed_tuning(args, nacc)
    elif plan is not None and not args.no_autotune:
        tuned, tuned_ms = plan.autotune(repeats=20)
        log(f"tuned by the plan: {tuned} ({tuned_ms:.4f} ms per step)")
    elif not args.no_autotune:
        from paper_2210_04847_amd import autotune
        cands = dict(autotune.CANDIDATES)
        if forward_only:
            cands = {"march_waves_per_group": cands["march_waves_per_group"]}
        tuned, _ = autotune.autotune(lambda: st.step(), st.outputs, cands, log=log)
        log(f"tuned: {tuned}")
    steps, warmup = args.steps, args.warmup
    for k in range(warmup):
        st.step(update=k % EMA_EVERY == 0)
    torch.cuda.synchronize()
    log(f"warmup done ({warmup} steps)")

    graphs = None
    if plan is not None:
        plan.capture()
        log("captured the step plan's HIP graphs")
    elif form == "graph":
        graphs = (capture(torch, lambda: st.step(update=False)),
                  capture(torch, lambda: st.step(update=True)))
        log("captured the step in HIP graphs")

    # A step's sample total changes only when the grid does: marching the
    # same rays through the same bits gives the same samples, bit for bit.
    # So the totals are copied out (a small copy kernel each) only at the
    # first step and at each step after one that updated the grid, and hold
    # in between; the last step's total is checked against that afterwards.
    totals = torch.zeros(steps, dtype=torch.int64, device="cuda")
    rendered = torch.zeros(steps, dtype=torch.int64, device="cuda")
    copied = []
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record()
    prev_upd = True
    for k in range(steps):
        upd = (warmup + k) % EMA_EVERY == 0
        if plan is not None:
            plan.launch(with_update=upd)
        elif graphs is not None:
            graphs[1 if upd else 0].replay()
        else:
            st.step(update=upd)
        if prev_upd:
            totals[k:k + 1].copy_(st.total)
            rendered[k:k + 1].copy_(st.cur[4])
            copied.append(k)
        prev_upd = upd
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_total = start.elapsed_time(stop)
    if int(st.status.item()) != 0:
        raise RuntimeError("capacity overflow in the timed region")
    last_total, last_rendered = int(st.total.item()), int(st.cur[4].item())
    e_steps, k_steps = totals.cpu().numpy(), rendered.cpu().numpy()
    for k in range(steps):
        if k not in copied:
            e_steps[k], k_steps[k] = e_steps[k - 1], k_steps[k - 1]
    if (e_steps[-1], k_steps[-1]) != (last_total, last_rendered):
        raise RuntimeError("a step's sample total changed without a grid update")
    e_total = int(e_steps.sum())
    phase_avg = phase_timing(torch, st, min(steps, 32), warmup + steps)
    if plan is not None:
        one = lambda: plan.launch()
    elif graphs is not None:
        one = graphs[0].replay
    else:
        one = lambda: st.step()
    latency = step_latency(torch, one, 100 if forward_only else 32)
    unfused = None if (forward_only or st.prune) else unfused_render(torch, st)
    e_mean = e_total / steps
    k_mean = float(k_steps.mean())  # samples shaded and rendered (= e_mean unpruned)
    v_frac = kept_fraction(st, int(k_steps[-1]))
    alg = algorithmic_bytes(st.n, k_mean, k_mean * v_frac, forward_only)
    # marching moves the marched samples; the field and render the rendered ones
    alg["march_fill"] = algorithmic_bytes(st.n, e_mean, e_mean, forward_only)["march_fill"]
    if st.prune:
        # densities in, keep flags out; then flags in, kept intervals copied
        alg["prune"] = 13 * e_mean + 16 * st.n + (1 * e_mean + 8 * k_mean + 12 * k_mean)
        alg["field_sigma"] = 16 * e_mean + 24 * st.n
    # the dominant kernel of the path itself (the synthetic field stands in for
    # the user's radiance field and is reported, not ranked)
    per_launch = {p: phase_avg[p] for p in alg if p not in ("field", "field_sigma")}
    dominant = max(per_launch, key=per_launch.get)
    step_ms = ms_total / steps
    step_bytes = sum(alg.values())
    render_bps = alg["render"] / (phase_avg["render"] * 1e-3)
    render_roofline = {
        "bound": "hbm", "kernel": "render", "achieved": render_bps / 1e9, "peak": HBM_PEAK / 1e9,
        "unit": "GB/s", "frac": render_bps / HBM_PEAK,
        "traffic": (recorded_traffic("render_mse", RENDER_SOURCES, w.name)
                    if not forward_only else None)}
    if dominant == "march_count":
        # The count pass is bound by its arithmetic.  With the halo bits it
        # looks up only part of the lattice, so its work is not a fixed
        # number of operations per lattice candidate: `achieved` counts the
        # VALU lane operations the phase's kernels executed per step
        # (SQ_INSTS_VALU x 64 from the committed counter record of this
        # workload and source; null when none matches), per phase time.
        cands = lattice_candidates(w, inp["rays_o"], inp["rays_d"])
        valu = recorded_valu("march_count", MARCH_SOURCES, w.name)
        secs = phase_avg["march_count"] * 1e-3
        ops_s = valu * 64 / secs if valu is not None else None
        roofline = {"bound": "alu", "kernel": "march_count",
                    "achieved": ops_s / 1e12 if ops_s is not None else None,
                    "peak": ALU_PEAK / 1e12, "unit": "TOP/s",
                    "frac": ops_s / ALU_PEAK if ops_s is not None else None,
                    "traffic": recorded_traffic("march_count", MARCH_SOURCES, w.name),
                    "measure": "VALU lane operations executed (SQ_INSTS_VALU x 64, committed "
                               "counter record)",
                    "candidates": cands, "candidates_per_s": cands / secs}
    elif dominant == "render":
        roofline = render_roofline
    else:
        bps = alg[dominant] / (phase_avg[dominant] * 1e-3)
        roofline = {"bound": "hbm", "kernel": dominant, "achieved": bps / 1e9,
                    "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": bps / HBM_PEAK,
                    "traffic": None}
    # the marching + rendering path as a whole (count with its scan, fill,
    # fused render; the synthetic field and the grid update left out)
    path_keys = [k for k in ("march_count", "march_fill", "prune", "render") if k in alg]
    path_bytes = sum(alg[k] for k in path_keys)
    path_ms = sum(phase_avg[k] for k in path_keys)
    path_bps = path_bytes / (path_ms * 1e-3)
    path_roofline = {"bound": "hbm", "kernels": path_keys, "achieved": path_bps / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": path_bps / HBM_PEAK,
                     "ms": path_ms, "alg_bytes": path_bytes,
                     "limiter": max(path_keys, key=lambda k: phase_avg[k])}
    result = {
        "metric": METRIC,
        "value": e_total / (ms_total * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "rays": w.n_rays,
                   "grid": grid_label(w),
                   "blobs": inp["scene"].n_blobs, "dt": w.dt,
                   "cone": getattr(w, "cone", 0.0), "early_stop_eps": w.early_stop_eps,
                   "pass": "forward" if forward_only else "forward+mse+backward",
                   "grid_update_every": EMA_EVERY, "grid_update_cells": EMA_CELLS,
                   "form": form, "skip_field": "on" if use_skip(args, w) else "off", "tuning": tuned,
                   "visibility_pruning": (None if args.alpha_thre is None else
                                          {"early_stop_eps": w.early_stop_eps,
                                           "alpha_thre": args.alpha_thre}),
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "roofline_render": render_roofline,
        "roofline_path": path_roofline,
        "samples_per_step": e_mean,
        "rendered_samples_per_step": k_mean,
        "kept_fraction": v_frac,
        "phase_ms": phase_avg,
        "phase_gbps": {p: alg[p] / (phase_avg[p] * 1e-3) / 1e9 for p in alg if phase_avg[p] > 0},
        "step_alg_bytes": step_bytes,
        "step_hbm_frac": step_bytes / (step_ms * 1e-3) / HBM_PEAK,
        "step_latency_ms": latency,
        "render_unfused": unfused,
        "path_samples_per_s": e_mean / (1e-3 * (step_ms - phase_avg["field"]
                                                - phase_avg.get("field_sigma", 0.0))),
        "wall_s": wall,
        "cpu_baseline": None,
    }
    if plan is not None:
        plan.close()  # its graphs and workspaces, before the interpreter tears down the runtime
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        result["cpu_baseline"] = cpu_baseline(w, inp, min(args.cpu_sample_rays // 2, w.n_rays),
                                              min(args.cpu_sample_rays * 2, w.n_rays),
                                              forward_only)
    return result


def bench_dynamic(args, torch, nacc):
    """Per-frame plain calls vs one batched graph-captured step."""
    import numpy as np

    import synth
    w = synth.DYNAMIC_WORKLOADS[args.workload]
    t_gen = time.perf_counter()
    inp = synth.dynamic_inputs(w)
    log(f"inputs generated in {time.perf_counter() - t_gen:.1f} s")
    dev = torch.device("cuda")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    nf, res = w.n_frames, inp["res"]
    shared = w.shared_grid  # one grid for all frames (the maximum over time)
    grid = nacc.OccupancyGrid(w.box, res, n_grids=1 if shared else nf, device=dev)
    grid.set_occupancy(t(inp["occ"]), THRESHOLD)
    field = nacc.BlobField(inp["scene"], device=dev)
    rays_o, rays_d = t(inp["rays_o"]), t(inp["rays_d"])
    tgt, frame = t(inp["targets"]), t(inp["frame"])
    n_total = rays_o.shape[0]
    upd_set = t(synth.update_frames(EMA_CELLS, nf, 4100 + w.seed_base)) if shared else None
    batched = Step(torch, nacc, w, rays_o, rays_d, tgt, grid, field,
                   grid_id=None if shared else frame, ray_set=frame, update_set=upd_set,
                   seed=4000 + w.seed_base, skip_field=use_skip(args, w))
    lib = nacc._lib
    words = res ** 3 // 32
    starts = np.concatenate([[0], np.cumsum(inp["counts"])]).astype(np.int64)
    desc1 = lib.grid_desc(w.box[:3], w.box[3:], res)
    params = lib.march_params(w.near, w.far, w.dt)

    # each frame's own skip buffer, built once like the grid state it comes
    # from, only when the batched step marches with it too
    frame_skip = {}
    if use_skip(args, w):
        for f in range(nf):
            g = 0 if shared else f
            if g not in frame_skip:
                buf = torch.empty(lib.grid_skip_bytes(desc1), dtype=torch.uint8, device=dev)
                lib.grid_build_skip(grid.bits[g * words:(g + 1) * words], desc1, buf)
                frame_skip[g] = buf

    def plain_frames(keep=None):
        """One plain call sequence per frame: its rays, its grid (a view of the
        frame's words), outputs sized exactly after a host read of the total,
        gradients normalised by the whole batch (loss_rays)."""
        for f in range(nf):
            a, b = int(starts[f]), int(starts[f + 1])
            n = b - a
            if n == 0:
                continue
            o, d = rays_o[a:b], rays_d[a:b]
            g = 0 if shared else f
            bits = grid.bits[g * words:(g + 1) * words]
            skip = frame_skip.get(g)
            packed = torch.empty((n, 2), dtype=torch.int32, device=dev)
            total = torch.empty(1, dtype=torch.int64, device=dev)
            ws = torch.empty(lib.march_workspace_size(n, desc1, params), dtype=torch.uint8,
                             device=dev)
            lib.march_count(o, d, None, bits, desc1, params, packed, total, ws, skip)
            e = int(total.item())
            ri = torch.empty(e, dtype=torch.int32, device=dev)
            ts = torch.empty(e, dtype=torch.float32, device=dev)
            te = torch.empty(e, dtype=torch.float32, device=dev)
            lib.march_fill(o, d, None, bits, desc1, params, packed, ri, ts, te, None, skip, ws)
            sig = torch.empty(e, dtype=torch.float32, device=dev)
            rgb = torch.empty((e, 3), dtype=torch.float32, device=dev)
            lib.synth_field_samples(field.table, field.n_blobs, field.n_sets, o, d, frame[a:b], ri,
                                    ts, te, sig, rgb)
            color = torch.empty((n, 3), dtype=torch.float32, device=dev)
            opac = torch.empty(n, dtype=torch.float32, device=dev)
            dep = torch.empty(n, dtype=torch.float32, device=dev)
            gs = torch.empty(e, dtype=torch.float32, device=dev)
            gr = torch.empty((e, 3), dtype=torch.float32, device=dev)
            loss = torch.empty(1, dtype=torch.float32, device=dev)
            mws = torch.empty(lib.render_mse_workspace_size(n), dtype=torch.uint8, device=dev)
            lib.render_fwd_bwd_mse(packed, ts, te, sig, rgb, w.early_stop_eps, tgt[a:b], color,
                                   opac, dep, gs, gr, loss, mws, n_total)
            if keep is not None:
                keep.append((packed, ri + a, ts, color, gs, gr))

    plan = batched.plan() if args.form == "plan" else None
    tuned = None
    if args.tuning:
        tuned = fixed_tuning(args, nacc)
    elif plan is not None and not args.no_autotune:
        tuned, tuned_ms = plan.autotune(repeats=20)
        log(f"tuned by the plan: {tuned} ({tuned_ms:.4f} ms per step)")
    elif not args.no_autotune:
        from paper_2210_04847_amd import autotune
        tuned, _ = autotune.autotune(lambda: batched.step(), batched.outputs, log=log)
        log(f"tuned: {tuned}")
    for _ in range(3):
        batched.step()
        plain_frames()
    torch.cuda.synchronize()

    # the batched step against the plain calls, bit for bit
    kept = []
    plain_frames(kept)
    batched.step()
    torch.cuda.synchronize()
    e_b = int(batched.total.item())
    cat = lambda j: torch.cat([k[j].reshape(-1) for k in kept])
    bits32 = lambda x: x.contiguous().view(torch.int32)
    same = {
        "counts": bool(torch.equal(batched.packed[:, 1], cat(0).reshape(-1, 2)[:, 1])),
        "ray_indices": bool(torch.equal(batched.ray_indices[:e_b], cat(1))),
        "t_starts": bool(torch.equal(bits32(batched.t_starts[:e_b]), bits32(cat(2)))),
        "color": bool(torch.equal(bits32(batched.color.reshape(-1)), bits32(cat(3)))),
        "g_sigmas": bool(torch.equal(bits32(batched.g_sigmas[:e_b]), bits32(cat(4)))),
        "g_rgbs": bool(torch.equal(bits32(batched.g_rgbs[:e_b].reshape(-1)), bits32(cat(5)))),
    }
    log(f"batched vs plain identical: {same}")

    steps = args.steps
    reps = max(steps // 8, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plain_frames()
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3 / reps
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        batched.step()
    stop.record()
    torch.cuda.synchronize()
    eager_ms = start.elapsed_time(stop) / steps
    if plan is not None:
        plan.capture()
        replay = lambda: plan.launch()
    else:
        g = capture(torch, lambda: batched.step())
        replay = g.replay
    start.record()
    for _ in range(steps):
        replay()
    stop.record()
    torch.cuda.synchronize()
    graph_ms = start.elapsed_time(stop) / steps
    if plan is not None:
        plan.close()
    phase_avg = phase_timing(torch, batched, min(steps, 16), 1, updates=False)
    v_frac = kept_fraction(batched, e_b)
    alg = algorithmic_bytes(n_total, e_b, e_b * v_frac)
    achieved = alg["render"] / (phase_avg["render"] * 1e-3)
    return {
        "metric": METRIC,
        "value": e_b / (graph_ms * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 3,
        "ms_per_step": graph_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "frames": nf, "rays": n_total,
                   "grid": (f"one {res}^3 shared by the {nf} frames" if shared
                            else f"{nf} x {res}^3"),
                   "blobs": w.n_blobs, "early_stop_eps": w.early_stop_eps,
                   "pass": "forward+mse+backward",
                   "form": ("batched, the library's step plan (one HIP graph per step)"
                            if plan is not None else "batched, one HIP graph per step"),
                   "tuning": tuned, "skip_field": "on" if use_skip(args, w) else "off",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "render", "achieved": achieved / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK,
                     "traffic": None},
        "samples_per_step": e_b,
        "batched_graph_ms": graph_ms,
        "batched_eager_ms": eager_ms,
        "plain_per_frame_ms": plain_ms,
        "batched_over_plain": plain_ms / graph_ms,
        "identical_outputs": same,
        "phase_ms": phase_avg,
        "cpu_baseline": None,
    }


def bench_attrs(args, torch, nacc):
    """The training workload with per-sample feature vectors instead of
    colours: march, field densities, then the attribute render forward and
    backward (16 channels, a background, opacity threshold 0.01) given an
    upstream gradient of the rendered features, as a feature-decoding model
    would supply it.  Step captured in a HIP graph."""
    import numpy as np

    import synth
    w = synth.WORKLOADS["train_262k"]
    ch, thre = args.attrs_channels, 0.01
    inp = synth.workload_inputs(w)
    dev = torch.device("cuda")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    grid = nacc.OccupancyGrid(w.box, w.res, device=dev)
    grid.set_occupancy(t(inp["occ"]), THRESHOLD)
    field = nacc.BlobField(inp["scene"], device=dev)
    st = Step(torch, nacc, w, t(inp["rays_o"]), t(inp["rays_d"]), t(inp["targets"]), grid, field,
              seed=4000 + w.seed_base)
    lib = nacc._lib
    gen = torch.Generator(device=dev)
    gen.manual_seed(5000 + w.seed_base)
    feats = torch.randn((st.capacity, ch), generator=gen, device=dev)
    g_out = torch.randn((st.n, ch), generator=gen, device=dev)
    bg = torch.linspace(0.0, 1.0, ch, device=dev)
    out = torch.empty((st.n, ch), device=dev)
    g_feats = torch.empty_like(feats)
    eps = w.early_stop_eps

    def fwd():
        lib.render_attrs_fwd(st.packed, st.t_starts, st.t_ends, st.sigmas, feats, eps, thre, bg,
                             out, st.opacity, st.depth)

    def bwd():
        lib.render_attrs_bwd(st.packed, st.t_starts, st.t_ends, st.sigmas, feats, eps, thre, bg,
                             g_out, None, None, st.g_sigmas, g_feats)

    def step():
        st.march_count()
        st.march_fill()
        st.field_eval()
        fwd()
        bwd()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    g = capture(torch, step)
    steps = args.steps
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        g.replay()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    e = int(st.total.item())
    # per-phase times (eager, HIP events on the launch stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    phases = {"march_count": [], "march_fill": [], "field": [], "attrs_fwd": [], "attrs_bwd": []}
    for _ in range(16):
        fns = (st.march_count, st.march_fill, st.field_eval, fwd, bwd)
        for j, fn in enumerate(fns):
            ev[j].record()
            fn()
        ev[5].record()
        torch.cuda.synchronize()
        for j, name in enumerate(phases):
            phases[name].append(ev[j].elapsed_time(ev[j + 1]))
    ph = {k: float(np.mean(v)) for k, v in phases.items()}
    # samples before the cut (FP32 opacity mask included) from the weights
    wts = torch.empty(st.capacity, device=dev)
    lib.render_attrs_fwd(st.packed, st.t_starts, st.t_ends, st.sigmas, feats, eps, thre, bg,
                         out, None, None, wts)
    torch.cuda.synchronize()
    counts = st.packed[:, 1].long()
    ray_of = torch.repeat_interleave(torch.arange(st.n, device=dev), counts)
    last = torch.zeros(st.n, dtype=torch.long, device=dev)
    idx = torch.arange(e, device=dev)
    nz = wts[:e] > 0
    last.scatter_reduce_(0, ray_of[nz], idx[nz] - st.packed[:, 0].long()[ray_of[nz]] + 1, "amax")
    v = int(last.sum().item())  # samples up to the last weighted one: a lower bound of those read
    blocks = -(-ch // 16)
    fwd_bytes = v * (12 * blocks + 4 * ch) + st.n * (8 + 4 * ch + 8)
    bwd_bytes = v * (12 + 12 + 4 * ch) + e * (4 + 4 * ch) + st.n * (8 + 4 * ch)
    dominant = "attrs_bwd" if ph["attrs_bwd"] >= ph["attrs_fwd"] else "attrs_fwd"
    bps = (bwd_bytes if dominant == "attrs_bwd" else fwd_bytes) / (ph[dominant] * 1e-3)
    return {
        "metric": METRIC,
        "value": e / (ms * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"attrs{ch}_262k", "rays": w.n_rays, "grid": f"{w.res}^3 bit-packed",
                   "channels": ch, "background": "linspace(0, 1)", "alpha_thre": thre,
                   "early_stop_eps": eps, "pass": "attribute render forward + backward",
                   "form": "graph", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": bps / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": bps / HBM_PEAK,
                     "traffic": None},
        "samples_per_step": e,
        "samples_read_per_step": v,
        "phase_ms": ph,
        "phase_gbps": {"attrs_fwd": fwd_bytes / (ph["attrs_fwd"] * 1e-3) / 1e9,
                       "attrs_bwd": bwd_bytes / (ph["attrs_bwd"] * 1e-3) / 1e9},
        "cpu_baseline": None,
    }


def bench_images(args, torch, nacc):
    """Whole images forward (march, field, render).  The batched form is one
    fused launch over all images (marching, field and render per wavefront,
    no samples written); the plain form is one three-step call sequence per
    image (march count -> host read of the total -> fill -> field -> render,
    outputs sized exactly).  A batched three-step sequence over all images is
    timed too.  All colours are checked bit for bit against each other."""
    import numpy as np

    import synth
    w = synth.IMAGE_WORKLOADS[args.workload]
    t_gen = time.perf_counter()
    inp = synth.image_inputs(w)
    log(f"inputs generated in {time.perf_counter() - t_gen:.1f} s")
    sw = inp["scene_workload"]
    dev = torch.device("cuda")
    lib = nacc._lib
    grid = nacc.OccupancyGrid(sw.box, sw.res, device=dev)
    grid.set_occupancy(torch.from_numpy(inp["occ"]).to(dev), THRESHOLD)
    field = nacc.BlobField(inp["scene"], device=dev)
    rays_o = torch.from_numpy(inp["rays_o"]).to(dev)
    rays_d = torch.from_numpy(inp["rays_d"]).to(dev)
    counts = inp["counts"]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    params = lib.march_params(sw.near, sw.far, sw.dt)
    skip = grid.skip if use_skip(args, sw) else None
    eps = w.early_stop_eps
    i32, f32 = torch.int32, torch.float32

    def render(o, d, events=None):
        """march count -> host read of the total -> fill -> field -> render."""
        n = o.shape[0]
        rec = (lambda j: events[j].record()) if events is not None else (lambda j: None)
        rec(0)
        packed = torch.empty((n, 2), dtype=i32, device=dev)
        total = torch.empty(1, dtype=torch.int64, device=dev)
        ws = torch.empty(lib.march_workspace_size(n, grid.desc, params), dtype=torch.uint8,
                         device=dev)
        lib.march_count(o, d, None, grid.bits, grid.desc, params, packed, total, ws, skip)
        rec(1)
        e = int(total.item())
        ri = torch.empty(e, dtype=i32, device=dev)
        ts = torch.empty(e, dtype=f32, device=dev)
        te = torch.empty(e, dtype=f32, device=dev)
        lib.march_fill(o, d, None, grid.bits, grid.desc, params, packed, ri, ts, te, None, skip, ws)
        rec(2)
        sig = torch.empty(e, dtype=f32, device=dev)
        rgb = torch.empty((e, 3), dtype=f32, device=dev)
        lib.synth_field_samples(field.table, field.n_blobs, field.n_sets, o, d, None, ri, ts, te,
                                sig, rgb)
        rec(3)
        color = torch.empty((n, 3), dtype=f32, device=dev)
        opacity = torch.empty(n, dtype=f32, device=dev)
        depth = torch.empty(n, dtype=f32, device=dev)
        lib.render_fwd(packed, ts, te, sig, rgb, eps, color, opacity, depth)
        rec(4)
        return e, color

    def batched():
        return render(rays_o, rays_d)

    def plain(done=None):
        e = 0
        for k in range(len(counts)):
            a, b = int(offs[k]), int(offs[k + 1])
            ek, _ = render(rays_o[a:b], rays_d[a:b])
            e += ek
            if done is not None:
                done[k].record()
        return e

    n_all = rays_o.shape[0]
    f_color = torch.empty((n_all, 3), dtype=f32, device=dev)
    f_opacity = torch.empty(n_all, dtype=f32, device=dev)
    f_depth = torch.empty(n_all, dtype=f32, device=dev)
    f_kept = torch.empty(n_all, dtype=i32, device=dev)

    # per workgroup of 64 rays: device wall clock at its start and its end
    clocks = torch.zeros(2 * ((n_all + 63) // 64), dtype=torch.int64, device=dev)
    clock_khz = lib.wall_clock_khz(dev.index or 0)

    def fused(a=0, b=None, clk=None):
        """marching + field + render in one kernel, no samples written."""
        b = n_all if b is None else b
        lib.synth_render_fused(field.table, field.n_blobs, field.n_sets, None, rays_o[a:b],
                               rays_d[a:b], None, grid.bits, grid.desc, params, eps,
                               f_color[a:b], f_opacity[a:b], f_depth[a:b], f_kept[a:b], skip, clk)

    def image_done_ms():
        """Completion of each image in the last launch with clocks, from the
        start of its first workgroup (every image is a whole number of
        64-ray groups here; a group shared by two images counts for both)."""
        c = clocks.view(-1, 2).cpu().numpy()
        t0 = int(c[:, 0].min())
        out = []
        for k in range(len(counts)):
            g0, g1 = int(offs[k]) // 64, (int(offs[k + 1]) + 63) // 64
            out.append((int(c[g0:g1, 1].max()) - t0) / clock_khz)
        return out

    # warm-up (also fills the allocator's cache) and equality checks
    e_b, color_b = batched()
    colors = []
    for k in range(len(counts)):
        a, b = int(offs[k]), int(offs[k + 1])
        colors.append(render(rays_o[a:b], rays_d[a:b])[1])
    fused()
    torch.cuda.synchronize()
    same = bool(torch.equal(color_b.view(torch.int32), torch.cat(colors).view(torch.int32)))
    same_fused = bool(torch.equal(color_b.view(torch.int32), f_color.view(torch.int32)))
    kept_total = int(f_kept.sum().item())
    log(f"batched vs per-image colours identical: {same}; fused identical: {same_fused}; "
        f"{e_b} samples, {kept_total} before the cut")
    del colors, color_b

    runs = max(args.steps // 3, 3)
    lat_b, lat_p, ms_b, ms_p = [], [], [], []
    for _ in range(runs):
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        batched()
        stop.record()
        torch.cuda.synchronize()
        t = start.elapsed_time(stop)
        ms_b.append(t)
        lat_b += [t] * len(counts)  # every image completes with the batch
        done = [torch.cuda.Event(enable_timing=True) for _ in counts]
        start.record()
        plain(done)
        torch.cuda.synchronize()
        lat_p += [start.elapsed_time(ev) for ev in done]
        ms_p.append(start.elapsed_time(done[-1]))
    # fused: all images in one launch, and one launch per image
    ms_f, lat_f, lat_fb = [], [], []
    for _ in range(runs):
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        fused(clk=clocks)
        stop.record()
        torch.cuda.synchronize()
        ms_f.append(start.elapsed_time(stop))
        lat_fb += image_done_ms()
        done = [torch.cuda.Event(enable_timing=True) for _ in counts]
        start.record()
        for k in range(len(counts)):
            fused(int(offs[k]), int(offs[k + 1]))
            done[k].record()
        torch.cuda.synchronize()
        lat_f += [start.elapsed_time(ev) for ev in done]
    med_f = float(np.median(ms_f))
    # lane operations the fused kernel must at least do: the field and the
    # render of every sample before the cut (marching not counted)
    ops_f = kept_total * (FIELD_OPS_PER_BLOB * field.n_blobs + FIELD_OPS_FIXED + RENDER_OPS)
    events = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    render(rays_o, rays_d, events)
    torch.cuda.synchronize()
    names = ("march_count", "march_fill", "field", "render")
    phase = {nm: events[j].elapsed_time(events[j + 1]) for j, nm in enumerate(names)}
    n_rays = int(offs[-1])
    alg = algorithmic_bytes(n_rays, e_b, e_b, forward_only=True)  # upper bound on V
    achieved = alg["render"] / (phase["render"] * 1e-3)
    pct = lambda v, q: float(np.percentile(v, q))
    med_b, med_p = float(np.median(ms_b)), float(np.median(ms_p))
    perc = lambda v: {"p50": pct(v, 50), "p90": pct(v, 90), "p99": pct(v, 99)}
    ops_s = ops_f / (med_f * 1e-3)
    return {
        "metric": METRIC,
        # the batched form: one fused launch over all eight images (marching,
        # field and render per wavefront); its samples are the marched ones
        # before the early-termination cut, which it renders
        "value": kept_total / (med_f * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": runs,
        "warmup": 1,
        "ms_per_step": med_f,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "images": [list(sz) for sz in w.sizes], "rays": n_rays,
                   "grid": f"{sw.res}^3 bit-packed", "blobs": sw.n_blobs,
                   "early_stop_eps": eps, "pass": "forward",
                   "form": "one fused launch for all images vs per-image plain call sequences",
                   "skip_field": "on" if use_skip(args, sw) else "off", "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "fused_render", "achieved": ops_s / 1e12,
                     "peak": ALU_PEAK / 1e12, "unit": "TOP/s", "frac": ops_s / ALU_PEAK,
                     "traffic": None,
                     "note": "lower bound: the field and render of the samples before the cut only"},
        "samples_before_cut": kept_total,
        "rays_per_s": n_rays / (med_f * 1e-3),
        "batched_ms": med_f,
        "plain_ms": med_p,
        "batched_over_plain": med_p / med_f,
        "identical_to_plain": same_fused and same,
        # per-image completion inside the one launch (device wall clock at the
        # end of each image's last workgroup, from the first workgroup's start)
        "latency_ms": {"batched": perc(lat_fb),
                       "batched_per_image_ms": [float(np.median(lat_fb[k::len(counts)]))
                                                for k in range(len(counts))],
                       "plain": perc(lat_p),
                       "fused_per_image_launches": perc(lat_f)},
        "three_step_batched": {"ms": med_b, "samples_per_s": e_b / (med_b * 1e-3),
                               "samples": e_b, "over_plain": med_p / med_b,
                               "latency_ms": perc(lat_b), "identical_to_plain": same,
                               "phase_ms": phase,
                               "roofline_render": {"bound": "hbm", "kernel": "render",
                                                   "achieved": achieved / 1e9,
                                                   "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                                   "frac": achieved / HBM_PEAK}},
        "cpu_baseline": None,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; the benchmark runs on one GPU "
              "(rays shard across GPUs without communication except the grid update; see the "
              "design notes)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2210_04847_amd as nacc
    result = run_workload(args, torch, nacc)
    if args.workload == "train_262k" and args.rows == "all":
        attach_rows(args, torch, nacc, result)
    print(json.dumps(result), flush=True)


def run_workload(args, torch, nacc):
    if args.workload.startswith("dynamic"):
        return bench_dynamic(args, torch, nacc)
    if args.workload.startswith("images"):
        return bench_images(args, torch, nacc)
    if args.workload == "attrs_262k":
        return bench_attrs(args, torch, nacc)
    return bench_train(args, torch, nacc)


ROWS = ("plain_fwd_4k", "unbounded_262k", "unbounded_contract_262k", "dynamic_64", "images_8")
# keys of a workload's line that the headline line already carries
_ROW_DROP = ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "dtype", "data",
             "cpu_baseline", "unit")


def attach_rows(args, torch, nacc, result):
    """The HBM probe and every other workload, each measured as its own
    `--workload` run would measure it, attached to the headline line."""
    import copy
    log("HBM probe")
    probe = hbm_probe(torch, nacc)
    result["hbm_probe"] = probe
    measured = max(probe["read"]["GB/s"], probe["copy"]["GB/s"], probe["write"]["GB/s"])

    def with_measured(r):
        if isinstance(r, dict) and r.get("unit") == "GB/s" and r.get("achieved"):
            r["frac_of_measured"] = r["achieved"] / measured
        return r

    for key in ("roofline", "roofline_render", "roofline_path"):
        with_measured(result.get(key))
    rows = {}
    for name in ROWS:
        sub = copy.copy(args)
        sub.workload = name
        sub.no_cpu_baseline = True
        log(f"row {name}")
        t0 = time.perf_counter()
        try:
            r = run_workload(sub, torch, nacc)
        except Exception as exc:  # a failed row is reported, the others still run
            rows[name] = {"error": f"{type(exc).__name__}: {exc}"}
            log(f"row {name} failed: {exc}")
            continue
        finally:
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
        r = {k: v for k, v in r.items() if k not in _ROW_DROP}
        r["samples_per_s"] = r.pop("value")
        for key in ("roofline", "roofline_render", "roofline_path"):
            with_measured(r.get(key))
        r["wall_s_row"] = time.perf_counter() - t0
        rows[name] = r
    result["rows"] = rows
    dyn = rows.get("dynamic_64", {})
    if "batched_over_plain" in dyn:
        result["batched_over_plain"] = {"dynamic_64": dyn["batched_over_plain"],
                                        "identical": all(dyn["identical_outputs"].values())}


if __name__ == "__main__":
    main()
