"""The paper-shaped Python API (NerfAcc, Sec. 3 "Plug-and-Play").

    packed_info, ray_indices, t_starts, t_ends = ray_marching(rays_o, rays_d, grid, ...)
    color, opacity, depth = rendering(packed_info, t_starts, t_ends, sigmas, rgbs, ...)
    color, opacity, depth = rendering(rgb_sigma_fn, packed_info, t_starts, t_ends, ray_indices)

Every step runs in the HIP library; this module allocates outputs with torch
and marshals arguments.  ray_marching returns ray_indices explicitly, which the
paper's sigma_fn consumes.
"""
from __future__ import annotations

import math

import torch

from . import _lib

STEP_1024 = float(torch.tensor(3.0 * math.sqrt(3.0) / 1024.0, dtype=torch.float32))

_LOOKUPS = {"aabb": _lib.LOOKUP_AABB, "cascade": _lib.LOOKUP_CASCADE,
            "contract": _lib.LOOKUP_CONTRACT}


def _dev(device):
    return torch.device(device if device is not None else "cuda")


class OccupancyGrid:
    """Bit-packed occupancy grid(s) with the FP32 density state behind them
    (Sec. 2.1: a binary grid cached and updated during training).

    lookup "aabb": n_grids grids over `box`, a ray picks one by grid_id.
    lookup "cascade": n_grids nested levels, level l over box * 2^l (box must
    be [-b, b]^3 with b a power of two).
    lookup "contract": grid over the contracted space `box` (normally [-2,2]^3).
    """

    def __init__(self, box, resolution=128, n_grids=1, lookup="aabb", device=None):
        self.box = tuple(float(v) for v in box)
        self.res = int(resolution)
        self.n_grids = int(n_grids)
        self.lookup = _LOOKUPS[lookup] if isinstance(lookup, str) else int(lookup)
        self.cells = self.n_grids * self.res ** 3
        if self.cells % 32:
            raise ValueError("n_grids * res^3 must be a multiple of 32")
        dev = _dev(device)
        self.occ = torch.zeros(self.cells, dtype=torch.float32, device=dev)
        self.bits = torch.zeros(self.cells // 32, dtype=torch.int32, device=dev)
        self.desc = _lib.grid_desc(self.box[:3], self.box[3:], self.res, self.n_grids,
                                   self.lookup)
        # skip field for passing over empty space (res % 4 == 0)
        sb = _lib.grid_skip_bytes(self.desc)
        self.skip = torch.zeros(sb, dtype=torch.uint8, device=dev) if sb > 0 else None
        self.updates = 0

    def _repack(self, threshold):
        _lib.grid_pack(self.occ, threshold, self.bits)
        if self.skip is not None:
            _lib.grid_build_skip(self.bits, self.desc, self.skip)

    def set_occupancy(self, occ, threshold=0.01):
        """Replaces the density state and repacks the bits (occ > threshold)."""
        occ = torch.as_tensor(occ, dtype=torch.float32).reshape(-1)
        if occ.numel() != self.cells:
            raise ValueError(f"expected {self.cells} values, got {occ.numel()}")
        self.occ.copy_(occ)
        self._repack(threshold)

    def update(self, sigma_fn, decay=0.95, threshold=0.01, n_samples=1 << 18, seed=0):
        """One update: decay all cells, max with sigma_fn at n random jittered
        cell positions (Philox4x64-10 keyed by seed, counter = update number),
        repack.  sigma_fn maps positions [n, 3] (and, for several independent
        grids, the grid index [n]) to densities [n]; box and cascade positions
        are in world space, contraction-lookup positions in the contracted
        space the grid covers (a field defined in contracted coordinates reads
        them directly; points of norm >= 2 have no world preimage)."""
        dev = self.occ.device
        cells = torch.empty(n_samples, dtype=torch.int32, device=dev)
        pos = torch.empty((n_samples, 3), dtype=torch.float32, device=dev)
        _lib.grid_decay(self.occ, decay)
        _lib.grid_sample_cells(seed, self.updates, n_samples, self.desc, self.n_grids, cells, pos)
        if self.n_grids == 1 or self.lookup == _lib.LOOKUP_CASCADE:
            sig = sigma_fn(pos)
        else:
            sig = sigma_fn(pos, torch.div(cells, self.res ** 3, rounding_mode="floor"))
        sig = torch.as_tensor(sig, dtype=torch.float32, device=dev).reshape(-1).contiguous()
        _lib.grid_update_max(self.occ, cells, sig)
        self._repack(threshold)
        self.updates += 1

    def update_every(self, step, sigma_fn, every=16, **kw):
        """The training loop's grid maintenance (Sec. 2.1): update() at steps
        0, every, 2 every, ...; returns whether it ran.  Keyword arguments go
        to update()."""
        if step % every != 0:
            return False
        self.update(sigma_fn, **kw)
        return True

    def state_dict(self):
        return {"occ": self.occ.clone(), "bits": self.bits.clone(), "updates": self.updates,
                "box": self.box, "res": self.res, "n_grids": self.n_grids,
                "lookup": self.lookup}

    def load_state_dict(self, state):
        self.occ.copy_(state["occ"])
        self.bits.copy_(state["bits"])
        if self.skip is not None:
            _lib.grid_build_skip(self.bits, self.desc, self.skip)
        self.updates = int(state["updates"])


def ray_marching(rays_o, rays_d, grid: OccupancyGrid, near_plane=0.0, far_plane=1e10,
                 render_step_size=STEP_1024, cone_angle=0.0, dt_max=1e10, max_per_ray=0,
                 grid_id=None, skip_empty=False, replay_masks=True, sigma_fn=None,
                 early_stop_eps=1e-4, alpha_thre=0.0):
    """Marches the rays through the occupancy grid (Sec. 2.1) and returns the
    packed samples (Sec. 3): packed_info [R, 2] int32 (start, count),
    ray_indices [E] int32, t_starts [E], t_ends [E] float32.  One device-to-host
    copy of the total sizes the outputs exactly.  skip_empty uses the grid's
    skip field and replay_masks lets the fill pass reuse the count pass's
    occupancy masks (same samples either way).  With sigma_fn(t_starts,
    t_ends, ray_indices) -> densities, the samples are then pruned by
    visibility (prune_samples: T >= early_stop_eps, alpha >= alpha_thre),
    evaluating sigma_fn without gradients."""
    out = _march(rays_o, rays_d, grid, near_plane, far_plane, render_step_size, cone_angle, dt_max,
                 max_per_ray, grid_id, skip_empty, replay_masks)
    if sigma_fn is None:
        return out
    packed, ray_indices, t_starts, t_ends = out
    with torch.no_grad():
        sig = sigma_fn(t_starts, t_ends, ray_indices)
    sig = torch.as_tensor(sig, dtype=torch.float32).reshape(-1).contiguous()
    return prune_samples(packed, t_starts, t_ends, sig, early_stop_eps, alpha_thre)[:4]


def prune_samples(packed_info, t_starts, t_ends, sigmas, early_stop_eps=1e-4, alpha_thre=0.0):
    """Visibility pruning (Sec. 2.1, occluded regions): keeps the samples whose
    transmittance is at least early_stop_eps and whose opacity is at least
    alpha_thre, given their densities.  Returns (packed_info, ray_indices,
    t_starts, t_ends, sigmas) of the kept samples."""
    n = packed_info.shape[0]
    e = t_starts.numel()
    dev = t_starts.device
    keep = torch.empty(max(e, 1), dtype=torch.uint8, device=dev)[:e]
    packed_out = torch.empty((n, 2), dtype=torch.int32, device=dev)
    total = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(max(_lib.prune_workspace_size(n), 1), dtype=torch.uint8, device=dev)
    ts, te, sg = _flat(t_starts), _flat(t_ends), sigmas.reshape(-1).contiguous()
    _lib.prune_count(packed_info.contiguous(), ts, te, sg, early_stop_eps, alpha_thre, keep,
                     packed_out, total, ws)
    k = int(total.item())
    ri = torch.empty(k, dtype=torch.int32, device=dev)
    ts_o = torch.empty(k, dtype=torch.float32, device=dev)
    te_o = torch.empty(k, dtype=torch.float32, device=dev)
    sg_o = torch.empty(k, dtype=torch.float32, device=dev)
    _lib.prune_fill(packed_info.contiguous(), ts, te, sg, keep, packed_out, ri, ts_o, te_o, sg_o)
    return packed_out, ri, ts_o, te_o, sg_o


def _march(rays_o, rays_d, grid, near_plane, far_plane, render_step_size, cone_angle, dt_max,
           max_per_ray, grid_id, skip_empty, replay_masks):
    rays_o = rays_o.reshape(-1, 3).contiguous()
    rays_d = rays_d.reshape(-1, 3).contiguous()
    n = rays_o.shape[0]
    dev = rays_o.device
    params = _lib.march_params(near_plane, far_plane, render_step_size, dt_max, cone_angle,
                               max_per_ray)
    packed = torch.empty((n, 2), dtype=torch.int32, device=dev)
    total = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(max(_lib.march_workspace_size(n, grid.desc, params), 1), dtype=torch.uint8,
                     device=dev)
    gid = None if grid_id is None else grid_id.to(torch.int32).contiguous()
    skip = grid.skip if skip_empty else None
    _lib.march_count(rays_o, rays_d, gid, grid.bits, grid.desc, params, packed, total, ws, skip)
    e = int(total.item())
    if e > 2 ** 31 - 1:
        raise _lib.NaccError("ray_marching", _lib.NACC_ECAPACITY,
                             f"{e} samples exceed the int32 index range")
    ray_indices = torch.empty(e, dtype=torch.int32, device=dev)
    t_starts = torch.empty(e, dtype=torch.float32, device=dev)
    t_ends = torch.empty(e, dtype=torch.float32, device=dev)
    _lib.march_fill(rays_o, rays_d, gid, grid.bits, grid.desc, params, packed, ray_indices,
                    t_starts, t_ends, None, skip, ws if replay_masks else None)
    return packed, ray_indices, t_starts, t_ends


class RenderFn(torch.autograd.Function):
    """Eq. 1 forward and its hand-written backward (Sec. 2.2): gradients flow
    to the per-sample densities and colours; transmittance is recomputed in
    the backward kernel rather than stored."""

    @staticmethod
    def forward(ctx, packed_info, t_starts, t_ends, sigmas, rgbs, early_stop_eps):
        n = packed_info.shape[0]
        dev = sigmas.device
        color = torch.empty((n, 3), dtype=torch.float32, device=dev)
        opacity = torch.empty((n, 1), dtype=torch.float32, device=dev)
        depth = torch.empty((n, 1), dtype=torch.float32, device=dev)
        _lib.render_fwd(packed_info, t_starts, t_ends, sigmas, rgbs, early_stop_eps, color,
                        opacity, depth)
        ctx.save_for_backward(packed_info, t_starts, t_ends, sigmas, rgbs)
        ctx.eps = early_stop_eps
        return color, opacity, depth

    @staticmethod
    def backward(ctx, g_color, g_opacity, g_depth):
        packed_info, t_starts, t_ends, sigmas, rgbs = ctx.saved_tensors
        g_sigmas = torch.empty_like(sigmas)
        g_rgbs = torch.empty_like(rgbs)
        gc = g_color.contiguous() if g_color is not None else torch.zeros(
            (packed_info.shape[0], 3), dtype=torch.float32, device=sigmas.device)
        go = g_opacity.reshape(-1).contiguous() if g_opacity is not None else None
        gd = g_depth.reshape(-1).contiguous() if g_depth is not None else None
        _lib.render_bwd(packed_info, t_starts, t_ends, sigmas, rgbs, ctx.eps, gc, go, gd,
                        g_sigmas, g_rgbs)
        return None, None, None, g_sigmas, g_rgbs, None


def _flat(x, cols=None):
    x = x.contiguous()
    return x.reshape(-1) if cols is None else x.reshape(-1, cols)


def rendering(*args, early_stop_eps=1e-4, ray_indices=None):
    """rendering(packed_info, t_starts, t_ends, sigmas, rgbs) or
    rendering(rgb_sigma_fn, packed_info, t_starts, t_ends, ray_indices=...)
    -> color [R, 3], opacity [R, 1], depth [R, 1]; differentiable in sigmas
    and rgbs.  (n, 1)-shaped sample tensors are accepted."""
    if callable(args[0]):
        rgb_sigma_fn, packed_info, t_starts, t_ends = args
        rgbs, sigmas = rgb_sigma_fn(t_starts, t_ends, ray_indices)
    else:
        packed_info, t_starts, t_ends, sigmas, rgbs = args
    sig = sigmas.reshape(-1)
    col = rgbs.reshape(-1, 3)
    if not sig.is_contiguous():
        sig = sig.contiguous()
    if not col.is_contiguous():
        col = col.contiguous()
    return RenderFn.apply(packed_info.contiguous(), _flat(t_starts), _flat(t_ends), sig, col,
                          float(early_stop_eps))


class AttrsFn(torch.autograd.Function):
    """Rendering of arbitrary per-sample attributes (Sec. 2.2) with a
    background and an opacity threshold; hand-written backward to the
    densities and the attributes."""

    @staticmethod
    def forward(ctx, packed_info, t_starts, t_ends, sigmas, attrs, early_stop_eps, alpha_thre,
                background):
        n = packed_info.shape[0]
        dev = sigmas.device
        out = torch.empty((n, attrs.shape[1]), dtype=torch.float32, device=dev)
        opacity = torch.empty((n, 1), dtype=torch.float32, device=dev)
        depth = torch.empty((n, 1), dtype=torch.float32, device=dev)
        _lib.render_attrs_fwd(packed_info, t_starts, t_ends, sigmas, attrs, early_stop_eps,
                              alpha_thre, background, out, opacity, depth)
        ctx.save_for_backward(packed_info, t_starts, t_ends, sigmas, attrs, background)
        ctx.eps, ctx.thre = early_stop_eps, alpha_thre
        return out, opacity, depth

    @staticmethod
    def backward(ctx, g_out, g_opacity, g_depth):
        packed_info, t_starts, t_ends, sigmas, attrs, background = ctx.saved_tensors
        g_sigmas = torch.empty_like(sigmas)
        g_attrs = torch.empty_like(attrs)
        go = g_out.contiguous() if g_out is not None else torch.zeros(
            (packed_info.shape[0], attrs.shape[1]), dtype=torch.float32, device=sigmas.device)
        ga = g_opacity.reshape(-1).contiguous() if g_opacity is not None else None
        gd = g_depth.reshape(-1).contiguous() if g_depth is not None else None
        _lib.render_attrs_bwd(packed_info, t_starts, t_ends, sigmas, attrs, ctx.eps, ctx.thre,
                              background, go, ga, gd, g_sigmas, g_attrs)
        return None, None, None, g_sigmas, g_attrs, None, None, None


def render_attrs(packed_info, t_starts, t_ends, sigmas, attrs, early_stop_eps=1e-4,
                 alpha_thre=0.0, background=None):
    """Renders per-sample attributes attrs [E, C] (any C >= 1: features,
    normals, ...) as Eq. 1 renders colour (Sec. 2.2) -> out [R, C],
    opacity [R, 1], depth [R, 1]; differentiable in sigmas and attrs.
    background [C] (optional) is blended in by 1 - opacity; samples whose
    opacity is below alpha_thre (> 0) count as empty."""
    sig = sigmas.reshape(-1).contiguous()
    at = attrs.reshape(sig.numel(), -1).contiguous()
    bg = None if background is None else torch.as_tensor(
        background, dtype=torch.float32, device=sig.device).reshape(-1).contiguous()
    return AttrsFn.apply(packed_info.contiguous(), _flat(t_starts), _flat(t_ends), sig, at,
                         float(early_stop_eps), float(alpha_thre), bg)


def render_mse(packed_info, t_starts, t_ends, sigmas, rgbs, target, early_stop_eps=1e-4):
    """Fused forward + MSE loss + backward in one kernel pass per ray.
    Returns (loss [1], color, opacity, depth, g_sigmas, g_rgbs)."""
    n = packed_info.shape[0]
    dev = sigmas.device
    color = torch.empty((n, 3), dtype=torch.float32, device=dev)
    opacity = torch.empty(n, dtype=torch.float32, device=dev)
    depth = torch.empty(n, dtype=torch.float32, device=dev)
    g_sigmas = torch.empty_like(sigmas)
    g_rgbs = torch.empty_like(rgbs)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ws = torch.empty(max(_lib.render_mse_workspace_size(n), 1), dtype=torch.uint8, device=dev)
    _lib.render_fwd_bwd_mse(packed_info, t_starts, t_ends, sigmas, rgbs, early_stop_eps,
                            target.contiguous(), color, opacity, depth, g_sigmas, g_rgbs, loss, ws)
    return loss, color, opacity, depth, g_sigmas, g_rgbs


class BlobField:
    """The synthetic Gaussian-blob field (test and benchmark input, standing in
    for the user's radiance field of Sec. 3), evaluated by HIP kernels."""

    def __init__(self, scene, device=None):
        dev = _dev(device)
        self.n_blobs = scene.n_blobs
        self.n_sets = scene.n_sets
        t = lambda a: torch.as_tensor(a, dtype=torch.float32).contiguous().to(dev)
        self.table = torch.empty(_lib.synth_table_size(self.n_blobs, self.n_sets) // 4,
                                 dtype=torch.float32, device=dev)
        self.contract = bool(getattr(scene, "contract", False))
        _lib.synth_prepare(t(scene.centres), t(scene.stds), t(scene.peaks), t(scene.w),
                           t(scene.bias), self.table,
                           _lib.SYNTH_CONTRACT if self.contract else 0)
        # the same scene read at points already in its contracted coordinates
        # (the positions a contraction-lookup grid update draws)
        self.table_contracted = self.table
        if self.contract:
            self.table_contracted = torch.empty_like(self.table)
            _lib.synth_prepare(t(scene.centres), t(scene.stds), t(scene.peaks), t(scene.w),
                               t(scene.bias), self.table_contracted, 0)

    def samples(self, rays_o, rays_d, ray_indices, t_starts, t_ends, ray_set=None,
                n_samples_dev=None, sigmas=None, rgbs=None):
        e = ray_indices.numel()
        dev = ray_indices.device
        sig = sigmas if sigmas is not None else torch.empty(e, dtype=torch.float32, device=dev)
        rgb = rgbs if rgbs is not None else torch.empty((e, 3), dtype=torch.float32, device=dev)
        _lib.synth_field_samples(self.table, self.n_blobs, self.n_sets, rays_o, rays_d, ray_set,
                                 ray_indices, t_starts, t_ends, sig, rgb, n_samples_dev)
        return sig, rgb

    def points(self, points, point_set=None, want_rgb=False, contracted=False):
        """Field at points [n, 3]; contracted: the points are already in the
        scene's contracted coordinates."""
        n = points.shape[0]
        dev = points.device
        sig = torch.empty(n, dtype=torch.float32, device=dev)
        rgb = torch.empty((n, 3), dtype=torch.float32, device=dev) if want_rgb else None
        ps = None if point_set is None else point_set.to(torch.int32).contiguous()
        _lib.synth_field_points(self.table_contracted if contracted else self.table, self.n_blobs,
                                self.n_sets, points.contiguous(), ps, sig, rgb)
        return (sig, rgb) if want_rgb else sig


def render_fused(field: BlobField, rays_o, rays_d, grid: OccupancyGrid, near_plane=0.0,
                 far_plane=1e10, render_step_size=STEP_1024, early_stop_eps=1e-4, max_per_ray=0,
                 grid_id=None, ray_set=None, return_kept=False, skip_empty=True):
    """Inference in one kernel (Sec. 2.1 marching with early termination and
    Eq. 1, forward only) for a field the library evaluates itself: marches,
    evaluates `field` at the occupied samples and renders them without
    writing the samples out.  Returns (color [R, 3], opacity [R], depth [R])
    (and the samples before the cut per ray, with return_kept), equal bit
    for bit to ray_marching -> field.samples -> rendering.  Uniform steps
    only.  With skip_empty the box lookup marches by the halo bits of the
    grid's skip buffer (same samples)."""
    n = rays_o.shape[0]
    dev = rays_o.device
    color = torch.empty((n, 3), dtype=torch.float32, device=dev)
    opacity = torch.empty(n, dtype=torch.float32, device=dev)
    depth = torch.empty(n, dtype=torch.float32, device=dev)
    kept = torch.empty(n, dtype=torch.int32, device=dev) if return_kept else None
    params = _lib.march_params(near_plane, far_plane, render_step_size, max_per_ray=max_per_ray)
    gid = None if grid_id is None else grid_id.to(torch.int32).contiguous()
    rs = None if ray_set is None else ray_set.to(torch.int32).contiguous()
    _lib.synth_render_fused(field.table, field.n_blobs, field.n_sets, rs, rays_o.contiguous(),
                            rays_d.contiguous(), gid, grid.bits, grid.desc, params, early_stop_eps,
                            color, opacity, depth, kept, grid.skip if skip_empty else None)
    return (color, opacity, depth, kept) if return_kept else (color, opacity, depth)
