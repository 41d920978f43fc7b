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
# the grid of a contraction lookup covers the contracted space, a ball of radius 2
CONTRACT_BOX = (-2.0, -2.0, -2.0, 2.0, 2.0, 2.0)


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
    # True: the scene is defined in contracted coordinates (density and colour
    # are evaluated at the image of x under the unbounded-scene contraction)
    contract: bool = False

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


def contracted(points: np.ndarray) -> np.ndarray:
    """Scene coordinates of world points for a scene defined in contracted
    space: points beyond the unit ball map to radius 2 - 1/|x| (FP64).  This
    is part of the synthetic scene's definition."""
    nrm = np.linalg.norm(points, axis=1, keepdims=True)
    f = np.where(nrm > 1.0, (2.0 - 1.0 / np.maximum(nrm, 1.0)) / np.maximum(nrm, 1.0), 1.0)
    return points * f


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
        if scene.contract:
            p = contracted(p)
        d2 = ((p[:, None, :] - c[None, :, :]) ** 2).sum(-1)
        out[a:a + chunk] = (pk[None] * np.exp(-d2 / (2.0 * s[None] ** 2))).sum(-1)
    return out


def unbounded_blob_scene(levels: int, per_level: int, seed: int,
                         std_range=(0.04, 0.12), depth_range=(2.0, 6.0)) -> BlobScene:
    """A scene for unbounded rays, defined in contracted coordinates: level
    l = 0..levels-1 holds `per_level` blobs whose centres are the contracted
    images of world points at radius 2^(3 l / (levels - 1)) (1 to 8) in
    uniformly drawn directions.  Contracted standard deviations are drawn
    from std_range; each peak is set so that the optical depth through the
    blob's centre along the radius, in world units, is drawn from depth_range
    whatever the level (the contraction stretches radii by |x|^2 there)."""
    g = _rng(seed)
    n = levels * per_level
    lvl = np.repeat(np.arange(levels), per_level)
    radius = 2.0 ** (3.0 * lvl / max(levels - 1, 1))
    v = g.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    centres = contracted(v * radius[:, None])
    std = g.uniform(std_range[0], std_range[1], n)
    depth = g.uniform(depth_range[0], depth_range[1], n)
    stretch = np.maximum(radius, 1.0) ** 2
    peaks = depth / (math.sqrt(2.0 * math.pi) * std * stretch)
    w = g.standard_normal((3, 3))
    bias = g.standard_normal(3)
    return BlobScene(centres=centres[None].astype(np.float32), stds=std.astype(np.float32),
                     peaks=peaks.astype(np.float32), w=w.astype(np.float32),
                     bias=bias.astype(np.float32), contract=True)


def _sparse_density(scene: BlobScene, p: np.ndarray, cut: float) -> np.ndarray:
    """FP64 density of the scene's first centre set at scene-space points p,
    skipping blobs at points where they contribute below `cut`."""
    s = scene.stds.astype(np.float64)
    pk = scene.peaks.astype(np.float64)
    c = scene.centres[0].astype(np.float64)
    reach = s * np.sqrt(2.0 * np.log(np.maximum(pk / cut, 1.0)))
    acc = np.zeros(p.shape[0], np.float64)
    for b in range(scene.n_blobs):
        e = p - c[b]
        near = np.all(np.abs(e) < reach[b], axis=1)
        if not near.any():
            continue
        d2 = (e[near] ** 2).sum(1)
        acc[near] += pk[b] * np.exp(-d2 / (2.0 * s[b] ** 2))
    return acc


def cascade_occupancy(scene: BlobScene, res: int, levels: int, base: float = 1.0,
                      threshold_hint: float = 1e-2, chunk: int = 1 << 20) -> np.ndarray:
    """FP32 occupancy values of `levels` cascaded res^3 grids, level l over
    [-base 2^l, base 2^l]^3: the scene density at every cell centre (world
    coordinates), level-major then C order.  Blobs are skipped at points
    where they contribute below threshold_hint * 1e-6 (a sum of such
    contributions cannot cross the threshold)."""
    out = []
    cut = threshold_hint * 1e-6
    for lvl in range(levels):
        h = base * 2.0 ** lvl
        pts = cell_centres(res, (-h, -h, -h, h, h, h))
        occ = np.zeros(pts.shape[0], np.float64)
        for a in range(0, pts.shape[0], chunk):
            p = pts[a:a + chunk]
            if scene.contract:
                p = contracted(p)
            occ[a:a + chunk] = _sparse_density(scene, p, cut)
        out.append(occ)
    return np.concatenate(out).astype(np.float32)


def contracted_occupancy(scene: BlobScene, res: int, threshold_hint: float = 1e-2,
                         chunk: int = 1 << 20) -> np.ndarray:
    """FP32 occupancy values of one res^3 grid over the contracted space
    [-2, 2]^3 (the grid of a contraction lookup): the density of a scene
    defined in contracted coordinates, read at every cell centre directly,
    C order."""
    assert scene.contract
    pts = cell_centres(res, CONTRACT_BOX)
    occ = np.zeros(pts.shape[0], np.float64)
    cut = threshold_hint * 1e-6
    for a in range(0, pts.shape[0], chunk):
        occ[a:a + chunk] = _sparse_density(scene, pts[a:a + chunk], cut)
    return occ.astype(np.float32)


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


def camera_rays(width: int, height: int, index: int, n_cameras: int = 8, radius: float = 4.0,
                focal_scale: float = 1.2):
    """Pinhole camera `index` of n_cameras on the z = 0 circle of `radius`
    (azimuth 2 pi index / n_cameras) looking at the origin, up = +z, focal
    length focal_scale * width pixels, principal point at the image centre;
    one ray through every pixel centre, row-major from the top-left pixel.
    Returns origins and unit directions, f32 [height * width, 3]."""
    az = 2.0 * math.pi * index / n_cameras
    eye = radius * np.array([math.cos(az), math.sin(az), 0.0])
    fwd = -eye / np.linalg.norm(eye)
    right = np.cross(fwd, [0.0, 0.0, 1.0])
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    f = focal_scale * width
    x = (np.arange(width) + 0.5 - 0.5 * width) / f
    y = -(np.arange(height) + 0.5 - 0.5 * height) / f
    d = fwd[None, None, :] + x[None, :, None] * right + y[:, None, None] * up
    d = d.reshape(-1, 3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(eye, d.shape)
    return np.ascontiguousarray(o, np.float32), np.ascontiguousarray(d, np.float32)


@dataclass
class ImageWorkload:
    """Whole images rendered forward through the training scene's grid and
    field (blob scene and 128^3 grid of the train_262k workload)."""
    name: str
    sizes: tuple        # (width, height) per image; image k uses camera k
    n_cameras: int
    scene_workload: str
    early_stop_eps: float

    @property
    def n_rays(self) -> int:
        return sum(w * h for w, h in self.sizes)


IMAGE_WORKLOADS = {
    "images_8": ImageWorkload("images_8", ((800, 800),) * 4 + ((1920, 1080),) * 4, 8, "train_262k",
                              1e-4),
}


def image_inputs(w: ImageWorkload, scale: int = 1):
    """Rays of every image (concatenated in image order), the ray count of
    each image, and the scene and occupancy of the scene workload.  scale > 1
    divides every image size by it (smaller cases for tests)."""
    os_, ds_, counts = [], [], []
    for k, (wd, ht) in enumerate(w.sizes):
        o, d = camera_rays(wd // scale, ht // scale, k, w.n_cameras)
        os_.append(o)
        ds_.append(d)
        counts.append(o.shape[0])
    sw = WORKLOADS[w.scene_workload]
    scene = blob_scene(sw.n_blobs, 1000 + sw.seed_base)
    occ = initial_occupancy(scene, sw.res, sw.box)
    return dict(rays_o=np.ascontiguousarray(np.concatenate(os_)),
                rays_d=np.ascontiguousarray(np.concatenate(ds_)),
                counts=np.array(counts, np.int64), scene=scene, occ=occ, scene_workload=sw)


@dataclass
class UnboundedWorkload:
    """Rays from inside the unit ball in all directions, cone-scaled steps
    and a scene defined in contracted coordinates.  lookup "cascade": grids
    level l over [-2^l, 2^l]^3 in world space (the rays are clipped to the
    largest); lookup "contract": one grid over the contracted space [-2, 2]^3
    read through the scene contraction (no clip box: the lattice runs from
    near to far, at most max_per_ray samples per ray)."""
    name: str
    n_rays: int
    blob_levels: int
    blobs_per_level: int
    res: int
    cascades: int
    dt: float
    cone: float
    dt_max: float
    early_stop_eps: float
    near: float
    far: float
    seed_base: int
    lookup: str = "cascade"
    max_per_ray: int = 0

    @property
    def box(self):
        if self.lookup == "contract":
            return CONTRACT_BOX
        return (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)  # level 0; level l is box * 2^l


UNBOUNDED_WORKLOADS = {
    "unbounded_262k": UnboundedWorkload("unbounded_262k", 262144, 8, 4, 128, 4, STEP_1024,
                                        1.0 / 256.0, 1e10, 1e-4, 0.2, 1e4, 2),
    # the paper's own unbounded mechanism: contraction inside the grid lookup
    "unbounded_contract_262k": UnboundedWorkload("unbounded_contract_262k", 262144, 8, 4, 128, 1,
                                                 STEP_1024, 1.0 / 256.0, 1e10, 1e-4, 0.2, 1e4, 2,
                                                 lookup="contract", max_per_ray=1024),
}


def unbounded_inputs(w: UnboundedWorkload, n_rays: int | None = None, res: int | None = None):
    """Rays, scene, occupancy values (cascaded grids, or the contracted-space
    grid) and targets of an unbounded workload (smaller ray counts or
    resolutions for tests)."""
    n = w.n_rays if n_rays is None else n_rays
    rs = w.res if res is None else res
    o, d = rays_unbounded(n, 2000 + w.seed_base)
    scene = unbounded_blob_scene(w.blob_levels, w.blobs_per_level, 1000 + w.seed_base)
    if w.lookup == "contract":
        occ = contracted_occupancy(scene, rs)
    else:
        occ = cascade_occupancy(scene, rs, w.cascades)
    tgt = targets(n, 3000 + w.seed_base)
    return dict(rays_o=o, rays_d=d, scene=scene, occ=occ, targets=tgt, res=rs)


@dataclass
class DynamicWorkload:
    """Frames of a moving scene.  Each frame has its own occupancy grid, or
    (shared_grid) all frames march through one grid holding the maximum of
    the frames' densities, which the grid update keeps by reading the field
    at a random frame per drawn cell."""
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
    shared_grid: bool = False


DYNAMIC_WORKLOADS = {
    "dynamic_64": DynamicWorkload("dynamic_64", 64, 4096.0, 32, 128, BOX_1_5, STEP_1024, 1e-4,
                                  0.0, 1e10, 3),
    "dynamic_64_shared": DynamicWorkload("dynamic_64_shared", 64, 4096.0, 32, 128, BOX_1_5,
                                         STEP_1024, 1e-4, 0.0, 1e10, 3, shared_grid=True),
}


def update_frames(n: int, n_frames: int, seed: int) -> np.ndarray:
    """The frame at which a shared grid's update reads the field, per drawn
    cell slot (uniform over the frames, int32 [n]); fixed across updates
    while the drawn cells change."""
    return _rng(seed).integers(0, n_frames, n).astype(np.int32)


def dynamic_inputs(w: DynamicWorkload, n_frames: int | None = None, res: int | None = None,
                   mean_rays: float | None = None):
    """Rays (grouped by frame, frame f at time f / (F - 1)), their frame ids,
    the moving blob scene, one occupancy grid per frame (or the shared one:
    the maximum over the frames) and loss targets.  Ray counts per frame ~
    Poisson(mean_rays)."""
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
    if w.shared_grid:
        occ = occ.reshape(nf, -1).max(0)
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
