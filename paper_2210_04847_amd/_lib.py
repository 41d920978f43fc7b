"""ctypes binding of the gfx950 library (libnacc.so): argument marshalling only.

Every call takes torch tensors that live on the GPU, checks dtype, device and
contiguity, and passes raw pointers plus torch's current HIP stream to the C
ABI declared in include/*.h.  No arithmetic of the
method happens here.  If the library has not been built, importing this module
raises ImportError: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads torch's HIP runtime first; libnacc.so then binds to it

_HERE = os.path.dirname(os.path.abspath(__file__))
# NACC_LIBRARY: another build of the library (A/B timing of two builds)
LIB_PATH = os.environ.get("NACC_LIBRARY") or os.path.join(_HERE, "libnacc.so")

NACC_OK, NACC_EINVAL, NACC_ESHAPE, NACC_ECAPACITY, NACC_EHIP, NACC_ENOTSUP = 0, -1, -2, -3, -4, -5
LOOKUP_AABB, LOOKUP_CASCADE, LOOKUP_CONTRACT = 0, 1, 2


class NaccError(RuntimeError):
    """A call into libnacc.so returned a non-zero status."""

    def __init__(self, name, status, message):
        super().__init__(f"{name}: {status_name(status)} ({status}): {message}")
        self.status = status


class GridDesc(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_float * 3), ("hi", ctypes.c_float * 3),
                ("res", ctypes.c_int32), ("n_grids", ctypes.c_int32),
                ("lookup", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("march_waves_per_group", ctypes.c_int32), ("render_cached_chunks", ctypes.c_int32),
                ("render_mse_max_blocks", ctypes.c_int32), ("render_prefetch", ctypes.c_int32)]


class MarchParams(ctypes.Structure):
    _fields_ = [("near_plane", ctypes.c_float), ("far_plane", ctypes.c_float),
                ("dt", ctypes.c_float), ("dt_max", ctypes.c_float),
                ("cone", ctypes.c_float), ("max_per_ray", ctypes.c_int32)]


class PlanDesc(ctypes.Structure):
    """nacc_plan_desc (include/nacc_plan.h); stage functions as addresses."""
    _fields_ = [("rays_o", ctypes.c_void_p), ("rays_d", ctypes.c_void_p),
                ("grid_id", ctypes.c_void_p), ("n_rays", ctypes.c_int64),
                ("grid_bits", ctypes.c_void_p), ("grid_skip", ctypes.c_void_p),
                ("grid", GridDesc), ("params", MarchParams), ("capacity", ctypes.c_int64),
                ("packed_info", ctypes.c_void_p), ("ray_indices", ctypes.c_void_p),
                ("t_starts", ctypes.c_void_p), ("t_ends", ctypes.c_void_p),
                ("total", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("field", ctypes.c_void_p), ("field_user", ctypes.c_void_p),
                ("sigmas", ctypes.c_void_p), ("rgbs", ctypes.c_void_p),
                ("early_stop_eps", ctypes.c_float), ("target", ctypes.c_void_p),
                ("loss_rays", ctypes.c_int64), ("color", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("depth", ctypes.c_void_p),
                ("g_sigmas", ctypes.c_void_p), ("g_rgbs", ctypes.c_void_p),
                ("loss", ctypes.c_void_p), ("after", ctypes.c_void_p),
                ("after_user", ctypes.c_void_p), ("occ", ctypes.c_void_p),
                ("decay", ctypes.c_float), ("threshold", ctypes.c_float),
                ("seed", ctypes.c_uint64), ("update_cells", ctypes.c_int64),
                ("update_counter", ctypes.c_void_p), ("update_cell_ids", ctypes.c_void_p),
                ("update_positions", ctypes.c_void_p), ("update_values", ctypes.c_void_p),
                ("update_field", ctypes.c_void_p), ("update_field_user", ctypes.c_void_p)]


class SynthSamplesStage(ctypes.Structure):
    _fields_ = [("table", ctypes.c_void_p), ("n_blobs", ctypes.c_int32),
                ("n_sets", ctypes.c_int32), ("rays_o", ctypes.c_void_p),
                ("rays_d", ctypes.c_void_p), ("n_rays", ctypes.c_int64),
                ("ray_set", ctypes.c_void_p), ("ray_indices", ctypes.c_void_p),
                ("t_starts", ctypes.c_void_p), ("t_ends", ctypes.c_void_p),
                ("n_samples", ctypes.c_int64), ("n_samples_dev", ctypes.c_void_p),
                ("sigmas", ctypes.c_void_p), ("rgbs", ctypes.c_void_p)]


class SynthPointsStage(ctypes.Structure):
    _fields_ = [("table", ctypes.c_void_p), ("n_blobs", ctypes.c_int32),
                ("n_sets", ctypes.c_int32), ("points", ctypes.c_void_p),
                ("point_set", ctypes.c_void_p), ("point_cell", ctypes.c_void_p),
                ("cells_per_set", ctypes.c_int64), ("n", ctypes.c_int64),
                ("sigmas", ctypes.c_void_p), ("rgbs", ctypes.c_void_p)]


STAGE_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p)


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_U64 = ctypes.c_uint64
_F = ctypes.c_float
_SZ = ctypes.c_size_t
_INT = ctypes.c_int

_SIGNATURES = {
    "nacc_version": (ctypes.c_char_p, []),
    "nacc_get_tuning": (None, [ctypes.POINTER(Tuning)]),
    "nacc_set_tuning": (_INT, [ctypes.POINTER(Tuning)]),
    "nacc_last_error": (ctypes.c_char_p, []),
    "nacc_status_str": (ctypes.c_char_p, [_INT]),
    "nacc_march_workspace_size": (_I64, [_I64, ctypes.POINTER(GridDesc), ctypes.POINTER(MarchParams)]),
    "nacc_march_max_samples_per_ray": (_I64, [ctypes.POINTER(GridDesc), ctypes.POINTER(MarchParams)]),
    "nacc_march_count": (_INT, [_P, _P, _P, _I64, _P, _P, ctypes.POINTER(GridDesc),
                                ctypes.POINTER(MarchParams), _P, _P, _P, _SZ, _P]),
    "nacc_march_fill": (_INT, [_P, _P, _P, _I64, _P, _P, ctypes.POINTER(GridDesc),
                               ctypes.POINTER(MarchParams), _P, _P, _SZ, _I64, _P, _P, _P, _P, _P]),
    "nacc_render_fwd": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _F, _P, _P, _P, _P, _P, _P]),
    "nacc_render_bwd": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _F, _P, _P, _P, _P, _P, _P]),
    "nacc_render_attrs_fwd": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _I32, _F, _F, _P, _P, _P,
                                     _P, _P, _P]),
    "nacc_render_attrs_bwd": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _I32, _F, _F, _P, _P, _P,
                                     _P, _P, _P, _P]),
    "nacc_render_mse_workspace_size": (_I64, [_I64]),
    "nacc_render_fwd_bwd_mse": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _F, _P, _I64, _P, _P, _P,
                                       _P, _P, _P, _P, _SZ, _P]),
    "nacc_render_fwd_bwd_mse_noalloc": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _F, _P, _I64, _P,
                                               _P, _P, _P, _P, _P, _P]),
    "nacc_grid_decay": (_INT, [_P, _I64, _F, _P]),
    "nacc_grid_sample_cells": (_INT, [_U64, _U64, _P, _I64, ctypes.POINTER(GridDesc), _I32,
                                      _P, _P, _P]),
    "nacc_grid_update_max": (_INT, [_P, _P, _P, _I64, _I64, _P]),
    "nacc_grid_pack": (_INT, [_P, _I64, _F, _P, _P]),
    "nacc_grid_skip_bytes": (_I64, [ctypes.POINTER(GridDesc)]),
    "nacc_grid_build_skip": (_INT, [_P, ctypes.POINTER(GridDesc), _P, _P]),
    "nacc_prune_workspace_size": (_I64, [_I64]),
    "nacc_prune_count": (_INT, [_P, _I64, _I64, _P, _P, _P, _F, _F, _P, _P, _P, _P, _SZ, _P]),
    "nacc_prune_fill": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _P, _I64, _P, _P, _P, _P, _P, _P]),
    "nacc_synth_table_size": (_I64, [_I32, _I32]),
    "nacc_synth_prepare": (_INT, [_P, _P, _P, _P, _P, _I32, _I32, _I32, _P, _P]),
    "nacc_synth_field_samples": (_INT, [_P, _I32, _I32, _P, _P, _I64, _P, _P, _P, _P, _I64,
                                        _P, _P, _P, _P]),
    "nacc_synth_field_points": (_INT, [_P, _I32, _I32, _P, _P, _P, _I64, _I64, _P, _P, _P]),
    "nacc_synth_samples_stage_run": (_INT, [_P, _P]),
    "nacc_synth_points_stage_run": (_INT, [_P, _P]),
    "nacc_plan_create": (_INT, [ctypes.POINTER(PlanDesc), ctypes.POINTER(_P)]),
    "nacc_plan_destroy": (_INT, [_P]),
    "nacc_plan_step": (_INT, [_P, _P]),
    "nacc_plan_update": (_INT, [_P, _P]),
    "nacc_plan_capture_step": (_INT, [_P]),
    "nacc_plan_launch": (_INT, [_P, _I32, _P]),
    "nacc_plan_autotune": (_INT, [_P, _I32, _P, ctypes.POINTER(Tuning), ctypes.POINTER(_F)]),
    "nacc_wall_clock_khz": (_I64, [_I32]),
    "nacc_synth_render_fused": (_INT, [_P, _I32, _I32, _P, _P, _P, _P, _I64, _P, _P,
                                       ctypes.POINTER(GridDesc), ctypes.POINTER(MarchParams), _F,
                                       _P, _P, _P, _P, _P, _P]),
    "nacc_probe_hbm": (_INT, [_I32, _P, _P, _I64, _I32, _P]),
    "nacc_probe_fast_sqrt_rcp": (_INT, [_P, _I64, _P, _P, _P]),
}

# Symbols declared in the headers under include/.
EXPORTED = tuple(_SIGNATURES)


def _load():
    how = "run `python paper_2210_04847_amd/build.py` (or __graft_entry__.build())"
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; {how} first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        if not hasattr(lib, name):
            raise ImportError(f"{LIB_PATH} predates its sources (no {name}); {how}")
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def status_name(status: int) -> str:
    return lib.nacc_status_str(status).decode()


def version() -> str:
    return lib.nacc_version().decode()


def get_tuning() -> dict:
    t = Tuning()
    lib.nacc_get_tuning(ctypes.byref(t))
    return {name: getattr(t, name) for name, _ in Tuning._fields_}


def set_tuning(**kw) -> None:
    """Changes launch parameters (never results); unspecified keys keep their
    current values."""
    cur = get_tuning()
    cur.update(kw)
    t = Tuning(cur["march_waves_per_group"], cur["render_cached_chunks"],
               cur["render_mse_max_blocks"], cur["render_prefetch"])
    _check("nacc_set_tuning", lib.nacc_set_tuning(ctypes.byref(t)))


def _check(name, status):
    if status != NACC_OK:
        raise NaccError(name, status, lib.nacc_last_error().decode())


def _ptr(t):
    """Device pointer of a tensor (None -> NULL)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, dtype, name, numel=None):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")


def grid_desc(lo, hi, res, n_grids=1, lookup=LOOKUP_AABB) -> GridDesc:
    d = GridDesc()
    for i in range(3):
        d.lo[i] = float(lo[i])
        d.hi[i] = float(hi[i])
    d.res, d.n_grids, d.lookup, d.reserved = int(res), int(n_grids), int(lookup), 0
    return d


def march_params(near_plane, far_plane, dt, dt_max=1e10, cone=0.0, max_per_ray=0) -> MarchParams:
    p = MarchParams()
    p.near_plane, p.far_plane, p.dt = float(near_plane), float(far_plane), float(dt)
    p.dt_max, p.cone, p.max_per_ray = float(dt_max), float(cone), int(max_per_ray)
    return p


# ---------------------------------------------------------------------------
# Thin wrappers, one per C entry point (same names without the prefix).
# ---------------------------------------------------------------------------

def march_workspace_size(n_rays: int, desc, params) -> int:
    n = int(lib.nacc_march_workspace_size(n_rays, ctypes.byref(desc), ctypes.byref(params)))
    if n < 0:
        raise NaccError("nacc_march_workspace_size", NACC_EINVAL, lib.nacc_last_error().decode())
    return n


def march_max_samples_per_ray(desc, params) -> int:
    n = int(lib.nacc_march_max_samples_per_ray(ctypes.byref(desc), ctypes.byref(params)))
    if n < 0:
        raise NaccError("nacc_march_max_samples_per_ray", NACC_EINVAL,
                        lib.nacc_last_error().decode())
    return n


def _grid_words(desc):
    return desc.n_grids * desc.res ** 3 // 32


def march_count(rays_o, rays_d, grid_id, grid_bits, desc, params, packed_info, total,
                workspace, grid_skip=None, stream=None):
    n = rays_o.shape[0]
    _need(rays_o, torch.float32, "rays_o", 3 * n)
    _need(rays_d, torch.float32, "rays_d", 3 * n)
    _need(grid_id, torch.int32, "grid_id", n)
    _need(grid_bits, torch.int32, "grid_bits", _grid_words(desc))
    _need(packed_info, torch.int32, "packed_info", 2 * n)
    _need(total, torch.int64, "total", 1)
    _need(workspace, torch.uint8, "workspace")
    _need(grid_skip, torch.uint8, "grid_skip", grid_skip_bytes(desc))
    _check("nacc_march_count", lib.nacc_march_count(
        _ptr(rays_o), _ptr(rays_d), _ptr(grid_id), n, _ptr(grid_bits), _ptr(grid_skip),
        ctypes.byref(desc),
        ctypes.byref(params), _ptr(packed_info), _ptr(total), _ptr(workspace),
        workspace.numel() if workspace is not None else 0, _stream(stream)))


def march_fill(rays_o, rays_d, grid_id, grid_bits, desc, params, packed_info, ray_indices,
               t_starts, t_ends, status=None, grid_skip=None, workspace=None, stream=None):
    n = rays_o.shape[0]
    cap = ray_indices.numel()
    _need(rays_o, torch.float32, "rays_o", 3 * n)
    _need(rays_d, torch.float32, "rays_d", 3 * n)
    _need(grid_id, torch.int32, "grid_id", n)
    _need(grid_bits, torch.int32, "grid_bits", _grid_words(desc))
    _need(packed_info, torch.int32, "packed_info", 2 * n)
    _need(ray_indices, torch.int32, "ray_indices")
    _need(t_starts, torch.float32, "t_starts", cap)
    _need(t_ends, torch.float32, "t_ends", cap)
    _need(status, torch.int32, "status", 1)
    _need(grid_skip, torch.uint8, "grid_skip", grid_skip_bytes(desc))
    _need(workspace, torch.uint8, "workspace")
    _check("nacc_march_fill", lib.nacc_march_fill(
        _ptr(rays_o), _ptr(rays_d), _ptr(grid_id), n, _ptr(grid_bits), _ptr(grid_skip),
        ctypes.byref(desc), ctypes.byref(params), _ptr(packed_info), _ptr(workspace),
        workspace.numel() if workspace is not None else 0, cap, _ptr(ray_indices),
        _ptr(t_starts), _ptr(t_ends), _ptr(status), _stream(stream)))


def _render_inputs(packed_info, t_starts, t_ends, sigmas, rgbs):
    n = packed_info.shape[0]
    e = t_starts.numel()
    _need(packed_info, torch.int32, "packed_info", 2 * n)
    _need(t_starts, torch.float32, "t_starts")
    _need(t_ends, torch.float32, "t_ends", e)
    _need(sigmas, torch.float32, "sigmas", e)
    _need(rgbs, torch.float32, "rgbs", 3 * e)
    return n, e


def render_fwd(packed_info, t_starts, t_ends, sigmas, rgbs, early_stop_eps, color, opacity,
               depth, weights=None, kept=None, stream=None):
    n, e = _render_inputs(packed_info, t_starts, t_ends, sigmas, rgbs)
    _need(color, torch.float32, "color", 3 * n)
    _need(opacity, torch.float32, "opacity", n)
    _need(depth, torch.float32, "depth", n)
    _need(weights, torch.float32, "weights", e)
    _need(kept, torch.int32, "kept", n)
    _check("nacc_render_fwd", lib.nacc_render_fwd(
        _ptr(packed_info), n, e, _ptr(t_starts), _ptr(t_ends), _ptr(sigmas), _ptr(rgbs),
        float(early_stop_eps), _ptr(color), _ptr(opacity), _ptr(depth), _ptr(weights),
        _ptr(kept), _stream(stream)))


def render_bwd(packed_info, t_starts, t_ends, sigmas, rgbs, early_stop_eps, g_color,
               g_opacity, g_depth, g_sigmas, g_rgbs, stream=None):
    n, e = _render_inputs(packed_info, t_starts, t_ends, sigmas, rgbs)
    _need(g_color, torch.float32, "g_color", 3 * n)
    _need(g_opacity, torch.float32, "g_opacity", n)
    _need(g_depth, torch.float32, "g_depth", n)
    _need(g_sigmas, torch.float32, "g_sigmas", e)
    _need(g_rgbs, torch.float32, "g_rgbs", 3 * e)
    _check("nacc_render_bwd", lib.nacc_render_bwd(
        _ptr(packed_info), n, e, _ptr(t_starts), _ptr(t_ends), _ptr(sigmas), _ptr(rgbs),
        float(early_stop_eps), _ptr(g_color), _ptr(g_opacity), _ptr(g_depth), _ptr(g_sigmas),
        _ptr(g_rgbs), _stream(stream)))


def render_mse_workspace_size(n_rays: int) -> int:
    return int(lib.nacc_render_mse_workspace_size(n_rays))


def render_fwd_bwd_mse(packed_info, t_starts, t_ends, sigmas, rgbs, early_stop_eps, target,
                       color, opacity, depth, g_sigmas, g_rgbs, loss, workspace, loss_rays=0,
                       stream=None):
    n, e = _render_inputs(packed_info, t_starts, t_ends, sigmas, rgbs)
    _need(target, torch.float32, "target", 3 * n)
    _need(color, torch.float32, "color", 3 * n)
    _need(opacity, torch.float32, "opacity", n)
    _need(depth, torch.float32, "depth", n)
    _need(g_sigmas, torch.float32, "g_sigmas", e)
    _need(g_rgbs, torch.float32, "g_rgbs", 3 * e)
    _need(loss, torch.float32, "loss", 1)
    _need(workspace, torch.uint8, "workspace")
    _check("nacc_render_fwd_bwd_mse", lib.nacc_render_fwd_bwd_mse(
        _ptr(packed_info), n, e, _ptr(t_starts), _ptr(t_ends), _ptr(sigmas), _ptr(rgbs),
        float(early_stop_eps), _ptr(target), int(loss_rays), _ptr(color), _ptr(opacity),
        _ptr(depth), _ptr(g_sigmas), _ptr(g_rgbs), _ptr(loss), _ptr(workspace), workspace.numel(),
        _stream(stream)))


# rays the allocation-free fused loss call takes (its static device scratch)
MSE_NOALLOC_MAX_RAYS = 1044480


def render_fwd_bwd_mse_noalloc(packed_info, t_starts, t_ends, sigmas, rgbs, early_stop_eps,
                               target, color, opacity, depth, g_sigmas, g_rgbs, loss,
                               loss_rays=0, stream=None):
    n, e = _render_inputs(packed_info, t_starts, t_ends, sigmas, rgbs)
    _need(target, torch.float32, "target", 3 * n)
    _need(color, torch.float32, "color", 3 * n)
    _need(opacity, torch.float32, "opacity", n)
    _need(depth, torch.float32, "depth", n)
    _need(g_sigmas, torch.float32, "g_sigmas", e)
    _need(g_rgbs, torch.float32, "g_rgbs", 3 * e)
    _need(loss, torch.float32, "loss", 1)
    _check("nacc_render_fwd_bwd_mse_noalloc", lib.nacc_render_fwd_bwd_mse_noalloc(
        _ptr(packed_info), n, e, _ptr(t_starts), _ptr(t_ends), _ptr(sigmas), _ptr(rgbs),
        float(early_stop_eps), _ptr(target), int(loss_rays), _ptr(color), _ptr(opacity),
        _ptr(depth), _ptr(g_sigmas), _ptr(g_rgbs), _ptr(loss), _stream(stream)))


def grid_decay(occ, decay, stream=None):
    _need(occ, torch.float32, "occ")
    _check("nacc_grid_decay", lib.nacc_grid_decay(_ptr(occ), occ.numel(), float(decay),
                                                  _stream(stream)))


def grid_sample_cells(seed, step, n, desc, levels, cells, positions, step_dev=None, stream=None):
    """step: the update number, or a one-element int64 GPU tensor holding it."""
    if torch.is_tensor(step):
        _need(step, torch.int64, "step", 1)
        step, step_dev = 0, step
    _need(cells, torch.int32, "cells", n)
    _need(positions, torch.float32, "positions", 3 * n)
    _check("nacc_grid_sample_cells", lib.nacc_grid_sample_cells(
        int(seed), int(step), _ptr(step_dev), int(n), ctypes.byref(desc), int(levels),
        _ptr(cells), _ptr(positions), _stream(stream)))


def grid_update_max(occ, cells, values, stream=None):
    n = cells.numel()
    _need(occ, torch.float32, "occ")
    _need(cells, torch.int32, "cells")
    _need(values, torch.float32, "values", n)
    _check("nacc_grid_update_max", lib.nacc_grid_update_max(
        _ptr(occ), _ptr(cells), _ptr(values), n, occ.numel(), _stream(stream)))


def grid_skip_bytes(desc) -> int:
    return int(lib.nacc_grid_skip_bytes(ctypes.byref(desc)))


def grid_build_skip(bits, desc, skip, stream=None):
    _need(bits, torch.int32, "bits", _grid_words(desc))
    _need(skip, torch.uint8, "skip", grid_skip_bytes(desc))
    _check("nacc_grid_build_skip", lib.nacc_grid_build_skip(_ptr(bits), ctypes.byref(desc), _ptr(skip),
                                                             _stream(stream)))


def grid_pack(occ, threshold, bits, stream=None):
    _need(occ, torch.float32, "occ")
    _need(bits, torch.int32, "bits", occ.numel() // 32)
    _check("nacc_grid_pack", lib.nacc_grid_pack(_ptr(occ), occ.numel(), float(threshold),
                                                _ptr(bits), _stream(stream)))


def synth_table_size(n_blobs, n_sets) -> int:
    return int(lib.nacc_synth_table_size(n_blobs, n_sets))


def prune_workspace_size(n_rays: int) -> int:
    return int(lib.nacc_prune_workspace_size(int(n_rays)))


def prune_count(packed_info, t_starts, t_ends, sigmas, early_stop_eps, alpha_thre, keep, packed_out,
                total, workspace, stream=None):
    n = packed_info.shape[0]
    e = t_starts.numel()
    _need(packed_info, torch.int32, "packed_info", 2 * n)
    _need(packed_out, torch.int32, "packed_out", 2 * n)
    for t, nm in ((t_starts, "t_starts"), (t_ends, "t_ends"), (sigmas, "sigmas")):
        _need(t, torch.float32, nm, e)
    _need(keep, torch.uint8, "keep", e)
    _need(total, torch.int64, "total", 1)
    _need(workspace, torch.uint8, "workspace")
    _check("nacc_prune_count", lib.nacc_prune_count(
        _ptr(packed_info), n, e, _ptr(t_starts), _ptr(t_ends), _ptr(sigmas), float(early_stop_eps),
        float(alpha_thre), _ptr(keep), _ptr(packed_out), _ptr(total), _ptr(workspace),
        workspace.numel(), _stream(stream)))


def prune_fill(packed_info, t_starts, t_ends, sigmas, keep, packed_out, ray_indices_out,
               t_starts_out, t_ends_out, sigmas_out=None, status=None, stream=None):
    n = packed_info.shape[0]
    e = t_starts.numel()
    cap = t_starts_out.numel()
    _need(packed_info, torch.int32, "packed_info", 2 * n)
    _need(packed_out, torch.int32, "packed_out", 2 * n)
    for t, nm in ((t_starts, "t_starts"), (t_ends, "t_ends")):
        _need(t, torch.float32, nm, e)
    _need(sigmas, torch.float32, "sigmas", e)
    _need(keep, torch.uint8, "keep", e)
    _need(ray_indices_out, torch.int32, "ray_indices_out", cap)
    _need(t_ends_out, torch.float32, "t_ends_out", cap)
    _need(sigmas_out, torch.float32, "sigmas_out", cap)
    _need(status, torch.int32, "status", 1)
    _check("nacc_prune_fill", lib.nacc_prune_fill(
        _ptr(packed_info), n, e, _ptr(t_starts), _ptr(t_ends), _ptr(sigmas), _ptr(keep),
        _ptr(packed_out), cap, _ptr(ray_indices_out), _ptr(t_starts_out), _ptr(t_ends_out),
        _ptr(sigmas_out), _ptr(status), _stream(stream)))


SYNTH_CONTRACT = 1


def synth_prepare(centres, stds, peaks, w, bias, table, flags=0, stream=None):
    n_sets, n_blobs = centres.shape[0], centres.shape[1]
    for t, nm in ((centres, "centres"), (stds, "stds"), (peaks, "peaks"), (w, "w"), (bias, "bias"),
                  (table, "table")):
        _need(t, torch.float32, nm)
    _check("nacc_synth_prepare", lib.nacc_synth_prepare(
        _ptr(centres), _ptr(stds), _ptr(peaks), _ptr(w), _ptr(bias), n_blobs, n_sets,
        int(flags), _ptr(table), _stream(stream)))


def synth_field_samples(table, n_blobs, n_sets, rays_o, rays_d, ray_set, ray_indices, t_starts,
                        t_ends, sigmas, rgbs=None, n_samples_dev=None, stream=None):
    n = ray_indices.numel()
    _need(table, torch.float32, "table")
    _need(ray_indices, torch.int32, "ray_indices")
    _need(ray_set, torch.int32, "ray_set", rays_o.numel() // 3)
    _need(sigmas, torch.float32, "sigmas", n)
    _need(rgbs, torch.float32, "rgbs", 3 * n)
    _need(n_samples_dev, torch.int64, "n_samples_dev", 1)
    _need(rays_o, torch.float32, "rays_o")
    _need(rays_d, torch.float32, "rays_d", rays_o.numel())
    _check("nacc_synth_field_samples", lib.nacc_synth_field_samples(
        _ptr(table), n_blobs, n_sets, _ptr(rays_o), _ptr(rays_d), rays_o.numel() // 3,
        _ptr(ray_set), _ptr(ray_indices),
        _ptr(t_starts), _ptr(t_ends), n, _ptr(n_samples_dev), _ptr(sigmas), _ptr(rgbs),
        _stream(stream)))


def synth_field_points(table, n_blobs, n_sets, points, point_set, sigmas, rgbs=None,
                       point_cell=None, cells_per_set=0, stream=None):
    n = points.shape[0]
    _need(table, torch.float32, "table")
    _need(points, torch.float32, "points", 3 * n)
    _need(point_set, torch.int32, "point_set", n)
    _need(point_cell, torch.int32, "point_cell", n)
    _need(sigmas, torch.float32, "sigmas", n)
    _need(rgbs, torch.float32, "rgbs", 3 * n)
    _check("nacc_synth_field_points", lib.nacc_synth_field_points(
        _ptr(table), n_blobs, n_sets, _ptr(points), _ptr(point_set), _ptr(point_cell),
        int(cells_per_set), n, _ptr(sigmas), _ptr(rgbs), _stream(stream)))


def wall_clock_khz(device: int = 0) -> int:
    """Frequency of the device wall clock that the fused kernel's clocks count."""
    khz = int(lib.nacc_wall_clock_khz(device))
    if khz <= 0:
        raise NaccError("nacc_wall_clock_khz", khz if khz < 0 else NACC_EHIP,
                        lib.nacc_last_error().decode())
    return khz


def synth_render_fused(table, n_blobs, n_sets, ray_set, rays_o, rays_d, grid_id, grid_bits, desc,
                       params, early_stop_eps, color, opacity, depth, kept=None, grid_skip=None,
                       clocks=None, stream=None):
    n = rays_o.shape[0]
    _need(table, torch.float32, "table")
    _need(ray_set, torch.int32, "ray_set", n)
    _need(rays_o, torch.float32, "rays_o", 3 * n)
    _need(rays_d, torch.float32, "rays_d", 3 * n)
    _need(grid_id, torch.int32, "grid_id", n)
    _need(grid_bits, torch.int32, "grid_bits", _grid_words(desc))
    _need(color, torch.float32, "color", 3 * n)
    _need(opacity, torch.float32, "opacity", n)
    _need(depth, torch.float32, "depth", n)
    _need(kept, torch.int32, "kept", n)
    _need(grid_skip, torch.uint8, "grid_skip", grid_skip_bytes(desc))
    _need(clocks, torch.int64, "clocks", 2 * ((n + 63) // 64))
    _check("nacc_synth_render_fused", lib.nacc_synth_render_fused(
        _ptr(table), n_blobs, n_sets, _ptr(ray_set), _ptr(rays_o), _ptr(rays_d), _ptr(grid_id), n,
        _ptr(grid_bits), _ptr(grid_skip), ctypes.byref(desc), ctypes.byref(params),
        float(early_stop_eps), _ptr(color), _ptr(opacity), _ptr(depth), _ptr(kept), _ptr(clocks),
        _stream(stream)))


def render_attrs_fwd(packed_info, t_starts, t_ends, sigmas, attrs, early_stop_eps, alpha_thre,
                     background, out, opacity=None, depth=None, weights=None, stream=None):
    n = packed_info.shape[0]
    e = t_starts.numel()
    ch = attrs.shape[1] if attrs.dim() == 2 else 1
    _need(packed_info, torch.int32, "packed_info", 2 * n)
    _need(t_starts, torch.float32, "t_starts")
    _need(t_ends, torch.float32, "t_ends", e)
    _need(sigmas, torch.float32, "sigmas", e)
    _need(attrs, torch.float32, "attrs", e * ch)
    _need(background, torch.float32, "background", ch)
    _need(out, torch.float32, "out", n * ch)
    _need(opacity, torch.float32, "opacity", n)
    _need(depth, torch.float32, "depth", n)
    _need(weights, torch.float32, "weights", e)
    _check("nacc_render_attrs_fwd", lib.nacc_render_attrs_fwd(
        _ptr(packed_info), n, e, _ptr(t_starts), _ptr(t_ends), _ptr(sigmas), _ptr(attrs), ch,
        float(early_stop_eps), float(alpha_thre), _ptr(background), _ptr(out), _ptr(opacity),
        _ptr(depth), _ptr(weights), _stream(stream)))


def render_attrs_bwd(packed_info, t_starts, t_ends, sigmas, attrs, early_stop_eps, alpha_thre,
                     background, g_out, g_opacity, g_depth, g_sigmas, g_attrs, stream=None):
    n = packed_info.shape[0]
    e = t_starts.numel()
    ch = attrs.shape[1] if attrs.dim() == 2 else 1
    _need(packed_info, torch.int32, "packed_info", 2 * n)
    _need(t_starts, torch.float32, "t_starts")
    _need(t_ends, torch.float32, "t_ends", e)
    _need(sigmas, torch.float32, "sigmas", e)
    _need(attrs, torch.float32, "attrs", e * ch)
    _need(background, torch.float32, "background", ch)
    _need(g_out, torch.float32, "g_out", n * ch)
    _need(g_opacity, torch.float32, "g_opacity", n)
    _need(g_depth, torch.float32, "g_depth", n)
    _need(g_sigmas, torch.float32, "g_sigmas", e)
    _need(g_attrs, torch.float32, "g_attrs", e * ch)
    _check("nacc_render_attrs_bwd", lib.nacc_render_attrs_bwd(
        _ptr(packed_info), n, e, _ptr(t_starts), _ptr(t_ends), _ptr(sigmas), _ptr(attrs), ch,
        float(early_stop_eps), float(alpha_thre), _ptr(background), _ptr(g_out), _ptr(g_opacity),
        _ptr(g_depth), _ptr(g_sigmas), _ptr(g_attrs), _stream(stream)))


# ---------------------------------------------------------------------------
# Step plans (include/nacc_plan.h).
# ---------------------------------------------------------------------------

class Stage:
    """A stage of a step plan: the address of a nacc_stage_fn and its `user`
    pointer, plus the objects that must stay alive while a plan uses it."""

    def __init__(self, fn_address, user, keep=()):
        self.fn = ctypes.c_void_p(fn_address)
        self.user = user
        self.keep = keep


def _address(fn):
    return ctypes.cast(fn, ctypes.c_void_p).value


def synth_samples_stage(table, n_blobs, n_sets, rays_o, rays_d, ray_set, ray_indices, t_starts,
                        t_ends, sigmas, rgbs, n_samples_dev) -> Stage:
    """nacc_synth_field_samples as a native stage (the first *n_samples_dev
    samples of ray_indices / t_starts / t_ends)."""
    n = ray_indices.numel()
    _need(table, torch.float32, "table")
    _need(rays_o, torch.float32, "rays_o")
    _need(rays_d, torch.float32, "rays_d", rays_o.numel())
    _need(ray_set, torch.int32, "ray_set", rays_o.numel() // 3)
    _need(ray_indices, torch.int32, "ray_indices")
    _need(t_starts, torch.float32, "t_starts", n)
    _need(t_ends, torch.float32, "t_ends", n)
    _need(sigmas, torch.float32, "sigmas", n)
    _need(rgbs, torch.float32, "rgbs", 3 * n)
    _need(n_samples_dev, torch.int64, "n_samples_dev", 1)
    if n_samples_dev is None:
        raise ValueError("the samples stage needs n_samples_dev")
    st = SynthSamplesStage(_ptr(table), n_blobs, n_sets, _ptr(rays_o), _ptr(rays_d),
                           rays_o.numel() // 3, _ptr(ray_set), _ptr(ray_indices), _ptr(t_starts),
                           _ptr(t_ends), n, _ptr(n_samples_dev), _ptr(sigmas), _ptr(rgbs))
    keep = (st, table, rays_o, rays_d, ray_set, ray_indices, t_starts, t_ends, sigmas, rgbs,
            n_samples_dev)
    return Stage(_address(lib.nacc_synth_samples_stage_run), ctypes.addressof(st), keep)


def synth_points_stage(table, n_blobs, n_sets, points, point_set, sigmas, point_cell=None,
                       cells_per_set=0) -> Stage:
    """nacc_synth_field_points (densities only) as a native stage."""
    n = points.shape[0]
    _need(table, torch.float32, "table")
    _need(points, torch.float32, "points", 3 * n)
    _need(point_set, torch.int32, "point_set", n)
    _need(point_cell, torch.int32, "point_cell", n)
    _need(sigmas, torch.float32, "sigmas", n)
    st = SynthPointsStage(_ptr(table), n_blobs, n_sets, _ptr(points), _ptr(point_set),
                          _ptr(point_cell), int(cells_per_set), n, _ptr(sigmas), None)
    keep = (st, table, points, point_set, point_cell, sigmas)
    return Stage(_address(lib.nacc_synth_points_stage_run), ctypes.addressof(st), keep)


def python_stage(fn) -> Stage:
    """A Python callable as a stage: fn(stream) enqueues its work on `stream`
    (a torch.cuda.ExternalStream, or the default stream; also made torch's
    current stream).  It must
    not allocate device memory or synchronise if the plan is captured.  An
    exception ends the step; it is raised again by the plan call."""
    errors = []

    def trampoline(_user, stream):
        try:
            ext = (torch.cuda.ExternalStream(stream) if stream else
                   torch.cuda.default_stream())
            with torch.cuda.stream(ext):
                fn(ext)
            return 0
        except BaseException as e:  # reported by the plan call that ran the stage
            errors.append(e)
            return NACC_EINVAL

    cb = STAGE_FN(trampoline)
    stage = Stage(_address(cb), None, (cb, fn))
    stage.errors = errors
    return stage


class Plan:
    """A step plan (nacc_plan_create): marching, the field stage, rendering
    (with the MSE loss and its backward when `target` is given), an optional
    `after` stage and an optional grid update (when `occ` is given).  Keeps
    every tensor and stage it was given alive until close()."""

    def __init__(self, rays_o, rays_d, grid_bits, desc, params, packed_info, ray_indices,
                 t_starts, t_ends, total, field, sigmas, rgbs, color, opacity, depth,
                 early_stop_eps=1e-4, grid_id=None, grid_skip=None, status=None, target=None,
                 loss_rays=0, g_sigmas=None, g_rgbs=None, loss=None, after=None, occ=None,
                 decay=0.95, threshold=0.01, seed=0, update_counter=None, update_cell_ids=None,
                 update_positions=None, update_values=None, update_field=None):
        n = rays_o.shape[0]
        cap = ray_indices.numel()
        _need(rays_o, torch.float32, "rays_o", 3 * n)
        _need(rays_d, torch.float32, "rays_d", 3 * n)
        _need(grid_id, torch.int32, "grid_id", n)
        _need(grid_bits, torch.int32, "grid_bits", _grid_words(desc))
        _need(grid_skip, torch.uint8, "grid_skip", grid_skip_bytes(desc))
        _need(packed_info, torch.int32, "packed_info", 2 * n)
        _need(ray_indices, torch.int32, "ray_indices")
        for t, nm, k in ((t_starts, "t_starts", 1), (t_ends, "t_ends", 1), (sigmas, "sigmas", 1),
                         (rgbs, "rgbs", 3), (g_sigmas, "g_sigmas", 1), (g_rgbs, "g_rgbs", 3)):
            _need(t, torch.float32, nm, k * cap)
        _need(total, torch.int64, "total", 1)
        _need(status, torch.int32, "status", 1)
        _need(target, torch.float32, "target", 3 * n)
        for t, nm, k in ((color, "color", 3), (opacity, "opacity", 1), (depth, "depth", 1)):
            _need(t, torch.float32, nm, k * n)
        _need(loss, torch.float32, "loss", 1)
        m = int(update_cell_ids.numel()) if update_cell_ids is not None else 0
        if occ is not None:
            _need(occ, torch.float32, "occ", desc.n_grids * desc.res ** 3)
            _need(update_counter, torch.int64, "update_counter", 1)
            _need(update_cell_ids, torch.int32, "update_cell_ids")
            _need(update_positions, torch.float32, "update_positions", 3 * m)
            _need(update_values, torch.float32, "update_values", m)
        stages = [x for x in (field, after, update_field) if x is not None]
        d = PlanDesc()
        d.rays_o, d.rays_d, d.grid_id, d.n_rays = _ptr(rays_o), _ptr(rays_d), _ptr(grid_id), n
        d.grid_bits, d.grid_skip, d.grid, d.params = _ptr(grid_bits), _ptr(grid_skip), desc, params
        d.capacity = cap
        d.packed_info, d.ray_indices = _ptr(packed_info), _ptr(ray_indices)
        d.t_starts, d.t_ends, d.total, d.status = _ptr(t_starts), _ptr(t_ends), _ptr(total), _ptr(status)
        d.field = field.fn if field is not None else None
        d.field_user = field.user if field is not None else None
        d.sigmas, d.rgbs, d.early_stop_eps = _ptr(sigmas), _ptr(rgbs), float(early_stop_eps)
        d.target, d.loss_rays = _ptr(target), int(loss_rays)
        d.color, d.opacity, d.depth = _ptr(color), _ptr(opacity), _ptr(depth)
        d.g_sigmas, d.g_rgbs, d.loss = _ptr(g_sigmas), _ptr(g_rgbs), _ptr(loss)
        d.after = after.fn if after is not None else None
        d.after_user = after.user if after is not None else None
        d.occ, d.decay, d.threshold, d.seed = _ptr(occ), float(decay), float(threshold), int(seed)
        d.update_cells, d.update_counter = m, _ptr(update_counter)
        d.update_cell_ids, d.update_positions = _ptr(update_cell_ids), _ptr(update_positions)
        d.update_values = _ptr(update_values)
        d.update_field = update_field.fn if update_field is not None else None
        d.update_field_user = update_field.user if update_field is not None else None
        self._keep = (rays_o, rays_d, grid_id, grid_bits, grid_skip, packed_info, ray_indices,
                      t_starts, t_ends, total, status, sigmas, rgbs, target, color, opacity, depth,
                      g_sigmas, g_rgbs, loss, occ, update_counter, update_cell_ids,
                      update_positions, update_values, stages)
        self._stages = stages
        handle = ctypes.c_void_p()
        self._call("nacc_plan_create", lib.nacc_plan_create(ctypes.byref(d), ctypes.byref(handle)))
        self.handle = handle

    def _call(self, name, status):
        for st in self._stages:
            errs = getattr(st, "errors", None)
            if errs:
                e = errs.pop()
                errs.clear()
                raise e
        _check(name, status)

    def step(self, stream=None):
        self._call("nacc_plan_step", lib.nacc_plan_step(self.handle, _stream(stream)))

    def update(self, stream=None):
        self._call("nacc_plan_update", lib.nacc_plan_update(self.handle, _stream(stream)))

    def capture(self):
        self._call("nacc_plan_capture_step", lib.nacc_plan_capture_step(self.handle))

    def launch(self, with_update=False, stream=None):
        self._call("nacc_plan_launch", lib.nacc_plan_launch(self.handle, int(bool(with_update)),
                                                            _stream(stream)))

    def autotune(self, repeats=5, stream=None):
        """Returns (the chosen tuning, its ms per step); see nacc_plan_autotune."""
        t, ms = Tuning(), ctypes.c_float()
        self._call("nacc_plan_autotune", lib.nacc_plan_autotune(
            self.handle, int(repeats), _stream(stream), ctypes.byref(t), ctypes.byref(ms)))
        return {name: getattr(t, name) for name, _ in Tuning._fields_}, ms.value

    def close(self):
        if getattr(self, "handle", None):
            lib.nacc_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PROBE_READ, PROBE_WRITE, PROBE_COPY = 0, 1, 2


def probe_hbm(kind, src, dst, n_bytes, blocks, stream=None):
    """One streaming pass of the HBM probe (include/nacc_probe.h)."""
    _need(src, src.dtype if src is not None else None, "src")
    _need(dst, dst.dtype, "dst")
    if src is not None and src.numel() * src.element_size() < n_bytes:
        raise ValueError("src is smaller than n_bytes")
    if kind != PROBE_READ and dst.numel() * dst.element_size() < n_bytes:
        raise ValueError("dst is smaller than n_bytes")
    _check("nacc_probe_hbm", lib.nacc_probe_hbm(int(kind), _ptr(src), _ptr(dst), int(n_bytes),
                                                int(blocks), _stream(stream)))


def probe_fast_sqrt_rcp(x, sqrt_out, rcp_out, stream=None):
    """The hardware square root and reciprocal of x (float32 device tensors)."""
    n = x.numel()
    _need(x, torch.float32, "x")
    _need(sqrt_out, torch.float32, "sqrt_out", n)
    _need(rcp_out, torch.float32, "rcp_out", n)
    _check("nacc_probe_fast_sqrt_rcp", lib.nacc_probe_fast_sqrt_rcp(
        _ptr(x), n, _ptr(sqrt_out), _ptr(rcp_out), _stream(stream)))
