#!/usr/bin/env python3
"""Benchmark of the marching + rendering training step on one MI355X.

One step = march (count, scan, fill) -> synthetic field at the samples ->
fused render forward + MSE + backward, plus the occupancy-grid update
(decay, 2^18 random cells, field, max, pack) every 16 steps.  Inputs are
synthetic, seeded and resident in HBM before the timed region; outputs are
written into capacity-sized buffers, so no step waits on the host.

Prints one JSON line (see the keys below).  --gpus N > 1 is not supported:
the path runs on one GPU.
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
    ap.add_argument("--workload", default="train_262k", choices=["train_262k", "plain_fwd_4k"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-grid", choices=["on", "off"], default="off",
                    help="march with the dilated coarse skip grid")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB on the device (a plain copy of "
                         "known size, for calibrating hardware traffic counters)")
    ap.add_argument("--cpu-sample-rays", type=int, default=131072)
    return ap.parse_args()


class TrainStep:
    """Buffers and launches of one training step (everything on torch's
    current stream)."""

    def __init__(self, w, inp, torch, nacc, skip_grid=False):
        self.torch, self.nacc, self.lib = torch, nacc, nacc._lib
        dev = torch.device("cuda")
        t = lambda a: torch.from_numpy(a).to(dev)
        self.w = w
        self.n = w.n_rays
        self.rays_o, self.rays_d = t(inp["rays_o"]), t(inp["rays_d"])
        self.target = t(inp["targets"])
        self.grid = nacc.OccupancyGrid(w.box, w.res, device=dev)
        self.grid.set_occupancy(t(inp["occ"]), THRESHOLD)
        self.field = nacc.BlobField(inp["scene"], device=dev)
        diag = math.sqrt(sum((w.box[3 + i] - w.box[i]) ** 2 for i in range(3)))
        self.capacity = self.n * (int(math.ceil(diag / w.dt)) + 2)
        n, cap = self.n, self.capacity
        i32, f32 = torch.int32, torch.float32
        self.params = self.lib.march_params(w.near, w.far, w.dt)
        self.packed = torch.empty((n, 2), dtype=i32, device=dev)
        self.total = torch.empty(1, dtype=torch.int64, device=dev)
        self.ws = torch.empty(self.lib.march_workspace_size(n, self.grid.desc, self.params),
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
        self.mse_ws = torch.empty(self.lib.render_mse_workspace_size(n), dtype=torch.uint8, device=dev)
        self.ema_cells = torch.empty(EMA_CELLS, dtype=i32, device=dev)
        self.ema_pos = torch.empty((EMA_CELLS, 3), dtype=f32, device=dev)
        self.ema_sigma = torch.empty(EMA_CELLS, dtype=f32, device=dev)
        self.updates = 0
        self.seed = 4000 + w.seed_base
        self.mip = self.grid.mip if skip_grid else None

    # phases ------------------------------------------------------------
    def march_count(self):
        self.lib.march_count(self.rays_o, self.rays_d, None, self.grid.bits, self.grid.desc,
                             self.params, self.packed, self.total, self.ws, self.mip)

    def march_fill(self):
        self.lib.march_fill(self.rays_o, self.rays_d, None, self.grid.bits, self.grid.desc,
                            self.params, self.packed, self.ray_indices, self.t_starts, self.t_ends,
                            self.status, self.mip, self.ws)

    def field_eval(self):
        self.lib.synth_field_samples(self.field.table, self.field.n_blobs, self.field.n_sets,
                                     self.rays_o, self.rays_d, None, self.ray_indices,
                                     self.t_starts, self.t_ends, self.sigmas, self.rgbs,
                                     self.total)

    def render(self):
        e = self.capacity
        self.lib.render_fwd_bwd_mse(self.packed, self.t_starts[:e], self.t_ends[:e],
                                    self.sigmas[:e], self.rgbs[:e], self.w.early_stop_eps,
                                    self.target, self.color, self.opacity, self.depth,
                                    self.g_sigmas, self.g_rgbs, self.loss, self.mse_ws)

    def grid_update(self):
        lib, g = self.lib, self.grid
        lib.grid_decay(g.occ, EMA_DECAY)
        lib.grid_sample_cells(self.seed, self.updates, EMA_CELLS, g.desc, 1, self.ema_cells,
                              self.ema_pos)
        lib.synth_field_points(self.field.table, self.field.n_blobs, self.field.n_sets,
                               self.ema_pos, None, self.ema_sigma)
        lib.grid_update_max(g.occ, self.ema_cells, self.ema_sigma)
        lib.grid_pack(g.occ, THRESHOLD, g.bits)
        lib.grid_build_mip(g.bits, g.desc, g.mip)
        self.updates += 1

    PHASES = ("march_count", "march_fill", "field", "render", "grid_update")

    def step(self, k, events=None):
        ev = events
        if ev is not None:
            ev[0].record()
        self.march_count()
        if ev is not None:
            ev[1].record()
        self.march_fill()
        if ev is not None:
            ev[2].record()
        self.field_eval()
        if ev is not None:
            ev[3].record()
        self.render()
        if ev is not None:
            ev[4].record()
        if k % EMA_EVERY == 0:
            self.grid_update()
        if ev is not None:
            ev[5].record()


def algorithmic_bytes(n_rays, e, v):
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
        # kept samples read once (24 B), gradients of every sample written
        # (16 B), packed_info + target in, colour/opacity/depth out (40 B/ray)
        "render": 24 * v + 16 * e + 40 * n_rays,
    }


def recorded_traffic(kernel, source):
    """HBM bytes per launch of `kernel` from the committed counter summaries
    (profiles/*.md, lines 'traffic_record: ...'), or None when none matches
    the current source of the kernel (the counters are then stale)."""
    import glob
    import hashlib
    src = os.path.join(ROOT, source)
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic_record:"):
                continue
            kv = dict(item.split("=", 1) for item in line.split()[1:])
            if kv.get("kernel") == kernel and kv.get("source") == source and kv.get("sha256_16") == digest:
                return float(kv["read_bytes"]) + float(kv["write_bytes"])
    return None


def cpu_baseline(w, inp, n_sample):
    """The oracle, as it stands, on the first n_sample rays of the workload:
    brute-force marching, FP64 field, FP64 forward + MSE + backward."""
    import numpy as np

    import oracle
    o = inp["rays_o"][:n_sample]
    d = inp["rays_d"][:n_sample]
    mask = oracle.grid_threshold(inp["occ"], THRESHOLD)
    t0 = time.perf_counter()
    packed, ri, ts, te = oracle.march(o, d, mask, w.res, np.asarray(w.box, np.float32), w.near,
                                      w.far, w.dt)
    pos = oracle.sample_positions(o, d, ri, ts, te)
    sig, rgb = oracle.blob_field(inp["scene"], pos)
    fwd = oracle.render_fwd(packed, ts, te, sig, rgb, w.early_stop_eps)
    _, g_color = oracle.mse_loss_and_grad(fwd["color"], inp["targets"][:n_sample])
    oracle.render_bwd(packed, ts, te, sig, rgb, g_color, eps=w.early_stop_eps)
    dt = time.perf_counter() - t0
    return {"value": ri.size / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_sample} of {w.n_rays} rays ({ri.size} samples), "
                      f"march+field+fwd+bwd, one thread, {dt:.1f} s, host {platform.processor() or platform.machine()}"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this build runs on one GPU "
              "(rays shard across GPUs without communication except the grid update; see the "
              "design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_2210_04847_amd as nacc

    w = synth.WORKLOADS[args.workload]
    t_gen = time.perf_counter()
    inp = synth.workload_inputs(w)
    print(f"# inputs generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    st = TrainStep(w, inp, torch, nacc, skip_grid=args.skip_grid == "on")
    torch.cuda.synchronize()
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    steps, warmup = args.steps, args.warmup
    for k in range(warmup):
        st.step(k)
    torch.cuda.synchronize()
    print(f"# warmup done ({warmup} steps)", file=sys.stderr, flush=True)

    totals = torch.empty(steps, dtype=torch.int64, device="cuda")
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record()
    for k in range(steps):
        st.step(warmup + k, events[k])
        totals[k:k + 1].copy_(st.total)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_total = start.elapsed_time(stop)
    if int(st.status.item()) != 0:
        raise RuntimeError("capacity overflow in the timed region")

    e_steps = totals.cpu().numpy()
    e_total = int(e_steps.sum())
    phase_ms = {p: [] for p in TrainStep.PHASES}
    for k in range(steps):
        ev = events[k]
        for j, p in enumerate(TrainStep.PHASES):
            if p == "grid_update" and (warmup + k) % EMA_EVERY != 0:
                continue
            phase_ms[p].append(ev[j].elapsed_time(ev[j + 1]))
    phase_avg = {p: (float(np.mean(v)) if v else 0.0) for p, v in phase_ms.items()}

    # samples before the cut (V): one forward with the per-ray kept counts,
    # outside the timed region, on the final step's samples
    e_last = int(e_steps[-1])
    kept = torch.empty(st.n, dtype=torch.int32, device="cuda")
    nacc._lib.render_fwd(st.packed, st.t_starts[:e_last], st.t_ends[:e_last], st.sigmas[:e_last],
                         st.rgbs[:e_last], w.early_stop_eps, st.color, st.opacity, st.depth,
                         None, kept)
    v_last = int(kept.sum().item())
    v_frac = v_last / max(e_last, 1)

    e_mean = e_total / steps
    v_mean = e_mean * v_frac
    alg = algorithmic_bytes(st.n, e_mean, v_mean)
    # the dominant kernel of the path itself (the synthetic field stands in
    # for the user's radiance field and is reported, not ranked)
    per_launch = {p: phase_avg[p] for p in alg if p != "field"}
    dominant = max(per_launch, key=per_launch.get)
    achieved = alg[dominant] / (phase_avg[dominant] * 1e-3)
    step_ms = ms_total / steps
    step_bytes = sum(alg.values())

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
        "config": {"workload": w.name, "rays": w.n_rays, "grid": f"{w.res}^3 bit-packed",
                   "blobs": w.n_blobs, "dt": w.dt, "early_stop_eps": w.early_stop_eps,
                   "grid_update_every": EMA_EVERY, "grid_update_cells": EMA_CELLS,
                   "form": "plain", "skip_grid": args.skip_grid, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": achieved / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK,
                     "traffic": (recorded_traffic("render_mse_kernel",
                                                  "paper_2210_04847_amd/csrc/render.hip")
                                 if dominant == "render" else None)},
        "samples_per_step": e_mean,
        "kept_fraction": v_frac,
        "phase_ms": phase_avg,
        "phase_gbps": {p: alg[p] / (phase_avg[p] * 1e-3) / 1e9 for p in alg if phase_avg[p] > 0},
        "step_alg_bytes": step_bytes,
        "step_hbm_frac": step_bytes / (step_ms * 1e-3) / HBM_PEAK,
        "path_samples_per_s": e_mean / (1e-3 * (step_ms - phase_avg["field"])),
        "wall_s": wall,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        print("# timing the oracle on the host", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(w, inp, min(args.cpu_sample_rays, w.n_rays))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
