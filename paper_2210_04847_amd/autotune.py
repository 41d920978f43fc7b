"""Autotuner for the library's launch parameters (nacc_tuning).

The knobs change speed, not results: rays per marching wave group, chunks of
64 samples kept in registers per ray between the forward and backward
passes, the fused loss kernel's workgroup count and whether it loads the
next ray's first chunk early.  Tuning is coordinate
descent over the knobs on the caller's real workload: each candidate is timed
with HIP events over a few steps and accepted only if the step's outputs are
bit-identical to those of the reference setting (a candidate that changed a
result would be a bug, and is rejected).
"""
from __future__ import annotations

import torch

from . import _lib

CANDIDATES = {
    "render_cached_chunks": (1, 2, 3, 4),
    "march_waves_per_group": (1, 2, 4, 8, 16),
    "render_mse_max_blocks": (4096, 8192, 16384, 65536),
    "render_prefetch": (0, 1),
}


def _time(step, repeats, warmup):
    for _ in range(warmup):
        step()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(repeats):
        step()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / repeats


def _snapshot(outputs):
    return [t.detach().clone() for t in outputs()]


def _identical(a, b):
    return all(x.shape == y.shape and torch.equal(x.view(torch.int32) if x.dtype == torch.float32
                                                   else x, y.view(torch.int32)
                                                   if y.dtype == torch.float32 else y)
               for x, y in zip(a, b))


def autotune(step, outputs, candidates=None, repeats=5, warmup=2, log=None):
    """Picks the fastest setting of every knob in `candidates` (default
    CANDIDATES) for `step` (launches one step on the current stream) and
    leaves it set.  outputs() returns the tensors that must not change.
    Returns (best setting, {setting repr: ms per step})."""
    cands = CANDIDATES if candidates is None else candidates
    best = _lib.get_tuning()
    step()
    torch.cuda.synchronize()
    reference = _snapshot(outputs)
    timings = {}
    best_ms = _time(step, repeats, warmup)
    timings[repr(sorted(best.items()))] = best_ms
    for knob, values in cands.items():
        for v in values:
            if v == best[knob]:
                continue
            trial = dict(best, **{knob: v})
            _lib.set_tuning(**trial)
            step()
            torch.cuda.synchronize()
            if not _identical(_snapshot(outputs), reference):
                if log:
                    log(f"autotune: {knob}={v} changed an output; rejected")
                continue
            ms = _time(step, repeats, warmup)
            timings[repr(sorted(trial.items()))] = ms
            if log:
                log(f"autotune: {knob}={v}: {ms:.4f} ms (best {best_ms:.4f})")
            if ms < best_ms:
                best, best_ms = trial, ms
        _lib.set_tuning(**best)
    return best, timings
