"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws inputs: rays, a Gaussian-blob scene standing in for the
user's radiance field (the paper's method is field-agnostic, Sec. 3), the
initial occupancy values of the grid, render-only inputs and loss targets.  It
holds none of the marching, rendering or grid-update arithmetic; the HIP
library and the oracle each implement those on their own.

Everything is drawn in FP64 with ``numpy.random.Generator(PCG64(seed))`` and
cast to FP32 once.  The paper's datasets (NeRF-Synthetic, D-NeRF, Mip-NeRF 360)
are not available; these distributions stand in for them with the sparsity of a
converged scene (Sec. 2.1 reports up to 98% of samples pruned).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Step of the dense sampling used by the bounded configurations: the diagonal
# of the [-1.5, 1.5]^3 box over 1024 samples (Sec. 4.1 samples 1024 per ray).
STEP_1024 = float(np.float32(3.0 * math.sqrt(3.0) / 1024.0))

BOX_1_5 = (-1.5, -1.5, -1.5, 1.5, 1.5, 1.5)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def rays_toward_origin(n: int, seed: int, radius: float = 4.0,
                       jitter_std: float = 0.1):
    """Origins uniform on a sphere of `radius`; each direction points at a
    target drawn from N(0, jitter_std^2 I) and is normalised."""
    g = _rng(seed)
    o = g.standard_normal((n, 3))
    o = radius * o / np.linalg.norm(o, axis=1, keepdims=True)
    p = jitter_std * g.standard_normal((n, 3))
    d = p - o
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


def rays_unbounded(n: int, seed: int):
    """Origins uniform in the unit ball, directions uniform on the sphere."""
    g = _rng(seed)
    v = g.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    rad = g.random(n) ** (1.0 / 3.0)
    o = v * rad[:, None]
    d = g.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


@dataclass
class BlobScene:
    """Sum of isotropic Gaussian blobs (density) plus a sigmoid of a linear map
    of position (colour).  centres has shape [n_sets, n_blobs, 3]; n_sets > 1
    holds one centre set per frame of a dynamic scene."""
    centres: np.ndarray  # f32 [S, B, 3]
    stds: np.ndarray     # f32 [B]
    peaks: np.ndarray    # f32 [B]
    w: np.ndarray        # f32 [3, 3]
    bias: np.ndarray     # f32 [3]

    @property
    def n_blobs(self) -> int:
        return int(self.stds.shape[0])

    @property
    def n_sets(self) -> int:
        return int(self.centres.shape[0])


def blob_scene(n_blobs: int, seed: int, peak: float = 50.0,
               centre_range: float = 1.0, radius_range=(0.1, 0.3)) -> BlobScene:
    """Centres U[-centre_range, centre_range]^3, radius U[radius_range] read as
    three standard deviations, the given peak density, colour map W, b ~ N(0,1).
    """
    g = _rng(seed)
    centres = g.uniform(-centre_range, centre_range, (1, n_blobs, 3))
    radii = g.uniform(radius_range[0], radius_range[1], n_blobs)
    w = g.standard_normal((3, 3))
    bias = g.standard_normal(3)
    return BlobScene(centres=centres.astype(np.float32),
                     stds=(radii / 3.0).astype(np.float32),
                     peaks=np.full(n_blobs, peak, np.float32),
                     w=w.astype(np.float32), bias=bias.astype(np.float32))


def moving_blob_scene(n_blobs: int, n_frames: int, seed: int,
                      peak: float = 50.0) -> BlobScene:
    """A blob scene whose centres move linearly in time: frame f at time
    f / (n_frames - 1) has centres c + v * time, v ~ U[-0.5, 0.5]^3."""
    base = blob_scene(n_blobs, seed, peak)
    g = _rng(seed + 7919)
    vel = g.uniform(-0.5, 0.5, (n_blobs, 3))
    times = np.arange(n_frames) / max(n_frames - 1, 1)
    c = base.centres[0].astype(np.float64)[None] + times[:, None, None] * vel[None]
    base.centres = c.astype(np.float32)
    return base


def blob_density(scene: BlobScene, points: np.ndarray, set_index: int = 0,
                 chunk: int = 1 << 18) -> np.ndarray:
    """FP64 density of the scene at FP64 points [n, 3] (centre set
    `set_index`).  Used to draw the initial occupancy values."""
    c = scene.centres[set_index].astype(np.float64)
    s = scene.stds.astype(np.float64)
    pk = scene.peaks.astype(np.float64)
    out = np.empty(points.shape[0], np.float64)
    for a in range(0, points.shape[0], chunk):
        p = points[a:a + chunk]
        d2 = ((p[:, None, :] - c[None, :, :]) ** 2).sum(-1)
        out[a:a + chunk] = (pk[None] * np.exp(-d2 / (2.0 * s[None] ** 2))).sum(-1)
    return out


def cell_centres(res: int, box) -> np.ndarray:
    """FP64 centres of a res^3 grid over box (lo[3], hi[3]) in C order
    (x-major), shape [res^3, 3]."""
    lo = np.asarray(box[:3], np.float64)
    hi = np.asarray(box[3:], np.float64)
    ax = [lo[i] + (np.arange(res) + 0.5) * (hi[i] - lo[i]) / res for i in range(3)]
    gx, gy, gz = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    return np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)


def initial_occupancy(scene: BlobScene, res: int, box, set_index: int = 0,
                      level_scale: float = 1.0) -> np.ndarray:
    """FP32 occupancy values: the scene density at every cell centre of a
    res^3 grid over box * level_scale, in C order."""
    pts = cell_centres(res, box) * level_scale
    return blob_density(scene, pts, set_index).astype(np.float32)


def local_occupancy(scene: BlobScene, res: int, box, set_index: int = 0,
                    reach: float = 7.0) -> np.ndarray:
    """FP32 occupancy values of one centre set: each blob adds its density
    at the cell centres within `reach` standard deviations of its centre
    (per axis), evaluated separably as a product of three 1-D Gaussians in
    FP64.  This is the input definition of the per-frame grids (the
    contributions it leaves out are below 50 e^-24.5 ~ 1e-9)."""
    lo = np.asarray(box[:3], np.float64)
    hi = np.asarray(box[3:], np.float64)
    h = (hi - lo) / res
    occ = np.zeros((res, res, res), np.float64)
    for b in range(scene.n_blobs):
        c = scene.centres[set_index, b].astype(np.float64)
        sd = float(scene.stds[b])
        span = []
        for i in range(3):
            a = max(0, int(np.floor((c[i] - reach * sd - lo[i]) / h[i] - 0.5)))
            e = min(res, int(np.ceil((c[i] + reach * sd - lo[i]) / h[i] + 0.5)))
            span.append((a, e))
        if any(a >= e for a, e in span):
            continue
        g = []
        for i, (a, e) in enumerate(span):
            x = lo[i] + (np.arange(a, e) + 0.5) * h[i]
            g.append(np.exp(-((x - c[i]) ** 2) / (2.0 * sd * sd)))
        blk = float(scene.peaks[b]) * g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :]
        (a0, e0), (a1, e1), (a2, e2) = span
        occ[a0:e0, a1:e1, a2:e2] += blk
    return occ.astype(np.float32).ravel()


def random_mask(n_cells: int, p: float, seed: int) -> np.ndarray:
    """uint8 0/1 occupancy mask with P(1) = p."""
    return (_rng(seed).random(n_cells) < p).astype(np.uint8)


def targets(n: int, seed: int) -> np.ndarray:
    """Loss targets U[0, 1], f32 [n, 3]."""
    return _rng(seed).random((n, 3)).astype(np.float32)


def ragged_render_inputs(n_rays: int, seed: int, mean_count: float = 40.0,
                         max_count: int = 300, dt: float = 0.01,
                         sigma_max: float = 60.0, empty_frac: float = 0.1):
    """Render-only inputs: ragged per-ray sample counts (Poisson, a fraction of
    empty rays, clipped to max_count), increasing sample intervals per ray,
    densities mixing empty stretches with dense blobs, colours in [0, 1].

    Returns packed_info i32 [n_rays, 2], t_starts, t_ends, sigmas f32 [E],
    rgbs f32 [E, 3].
    """
    g = _rng(seed)
    counts = np.minimum(g.poisson(mean_count, n_rays), max_count)
    counts[g.random(n_rays) < empty_frac] = 0
    counts = counts.astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    e = int(counts.sum())
    gaps = np.where(g.random(e) < 0.8, 0.0, g.exponential(0.05, e))
    widths = dt * g.uniform(0.5, 1.5, e)
    ray_of = np.repeat(np.arange(n_rays), counts)
    steps = widths + gaps
    cs = np.cumsum(steps)
    before = np.concatenate([[0.0], cs])[starts]  # sum of steps before each ray
    t0 = 0.5 + g.random(n_rays)
    t_ends = t0[ray_of] + cs - before[ray_of]
    t_starts = t_ends - widths
    sig = np.where(g.random(e) < 0.3, 0.0, g.uniform(0.0, sigma_max, e))
    sig *= (g.random(e) < 0.5)  # sparse
    rgbs = g.random((e, 3))
    packed = np.stack([starts, counts], axis=1).astype(np.int32)
    t_s = t_starts.astype(np.float32)
    t_e = t_ends.astype(np.float32)
    # keep intervals ordered after rounding to FP32
    t_e = np.maximum(t_e, t_s)
    return packed, t_s, t_e, sig.astype(np.float32), rgbs.astype(np.float32)


# --------------------------------------------------------------------------
# Workload definitions (sizes and seeds).  Seeds: field 1000 + c,
# rays 2000 + c, targets 3000 + c, grid-update key 4000 + c.
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n_rays: int
    n_blobs: int
    res: int
    box: tuple
    dt: float
    early_stop_eps: float
    near: float
    far: float
    seed_base: int


WORKLOADS = {
    "plain_fwd_4k": Workload("plain_fwd_4k", 4096, 8, 128, BOX_1_5, STEP_1024,
                             0.0, 0.0, 1e10, 0),
    "train_262k": Workload("train_262k", 262144, 32, 128, BOX_1_5, STEP_1024,
                           1e-4, 0.0, 1e10, 1),
}


@dataclass
class DynamicWorkload:
    name: str
    n_frames: int
    mean_rays: float
    n_blobs: int
    res: int
    box: tuple
    dt: float
    early_stop_eps: float
    near: float
    far: float
    seed_base: int


DYNAMIC_WORKLOADS = {
    "dynamic_64": DynamicWorkload("dynamic_64", 64, 4096.0, 32, 128, BOX_1_5, STEP_1024, 1e-4,
                                  0.0, 1e10, 3),
}


def dynamic_inputs(w: DynamicWorkload, n_frames: int | None = None, res: int | None = None,
                   mean_rays: float | None = None):
    """Rays (grouped by frame, frame f at time f / (F - 1)), their frame ids,
    the moving blob scene, one occupancy grid per frame and loss targets.
    Ray counts per frame ~ Poisson(mean_rays)."""
    nf = w.n_frames if n_frames is None else n_frames
    rs = w.res if res is None else res
    mean = w.mean_rays if mean_rays is None else mean_rays
    g = _rng(2000 + w.seed_base)
    counts = g.poisson(mean, nf).astype(np.int64)
    n = int(counts.sum())
    o, d = rays_toward_origin(n, 2100 + w.seed_base)
    frame = np.repeat(np.arange(nf), counts).astype(np.int32)
    scene = moving_blob_scene(w.n_blobs, nf, 1000 + w.seed_base)
    occ = np.concatenate([local_occupancy(scene, rs, w.box, f) for f in range(nf)])
    tgt = targets(n, 3000 + w.seed_base)
    return dict(rays_o=o, rays_d=d, frame=frame, counts=counts, scene=scene, occ=occ,
                targets=tgt, res=rs)


def workload_inputs(w: Workload, n_rays: int | None = None):
    """Rays, scene, initial occupancy and targets for a bounded workload.
    n_rays (optional) takes the first rays of the full set's generator stream
    only when equal to the full count; a smaller count draws its own rays."""
    n = w.n_rays if n_rays is None else n_rays
    o, d = rays_toward_origin(n, 2000 + w.seed_base)
    scene = blob_scene(w.n_blobs, 1000 + w.seed_base)
    occ = initial_occupancy(scene, w.res, w.box)
    tgt = targets(n, 3000 + w.seed_base)
    return dict(rays_o=o, rays_d=d, scene=scene, occ=occ, targets=tgt)
