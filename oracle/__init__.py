"""Plain CPU oracle for NerfAcc-style ray marching and volume rendering.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this package; the product path (the HIP library and
its Python binding) never imports it.  The arithmetic lives in ``oracle.c``
(plain C, built with gcc -O2 -ffp-contract=off); this module only marshals
numpy arrays through ctypes and takes exclusive prefix sums of per-ray counts.

Every function cites the passage of the paper it follows; the FP32 lattice
contract the marching follows is written out at the top of ``oracle.c``.

Parity status: every function below is pinned by a CPU test against closed
forms, brute force, finite differences or a library routine (see
``tests/test_oracle_pins.py``); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
             "-fno-finite-math-only", "-Wall", "-Wextra", "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_F = ctypes.c_float
_D = ctypes.c_double
_U64 = ctypes.c_uint64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_march.restype = _I64
    lib.oracle_march.argtypes = [_P, _P, _P, _I64, _P, _I32, _I32, _I32, _P,
                                 _F, _F, _F, _F, _F, _I32, _P, _I64, _P, _P, _P]
    lib.oracle_clip.restype = None
    lib.oracle_clip.argtypes = [_P, _P, _I64, _P, _F, _F, _P, _P, _P]
    lib.oracle_render_fwd.restype = None
    lib.oracle_render_fwd.argtypes = [_P, _I64, _P, _P, _P, _P, _D,
                                      _P, _P, _P, _P, _P]
    lib.oracle_render_bwd.restype = ctypes.c_int
    lib.oracle_render_bwd.argtypes = [_P, _I64, _P, _P, _P, _P, _D,
                                      _P, _P, _P, _P, _P, _P]
    lib.oracle_render_attrs_fwd.restype = None
    lib.oracle_render_attrs_fwd.argtypes = [_P, _I64, _P, _P, _P, _P, _I64, _I64, _D, _D, _P,
                                            _P, _P, _P, _P]
    lib.oracle_render_attrs_bwd.restype = ctypes.c_int
    lib.oracle_render_attrs_bwd.argtypes = [_P, _I64, _P, _P, _P, _P, _I64, _I64, _D, _D, _P,
                                            _P, _P, _P, _P, _P, _P]
    lib.oracle_philox4x64_10.restype = None
    lib.oracle_philox4x64_10.argtypes = [_P, _P, _P]
    lib.oracle_grid_sample_cells.restype = None
    lib.oracle_grid_sample_cells.argtypes = [_U64, _U64, _I64, _I32, _I32,
                                             _I32, _P, _P, _P]
    lib.oracle_grid_decay.restype = None
    lib.oracle_grid_decay.argtypes = [_P, _I64, _F]
    lib.oracle_grid_update_max.restype = None
    lib.oracle_grid_update_max.argtypes = [_P, _P, _P, _I64]
    lib.oracle_grid_threshold.restype = None
    lib.oracle_grid_threshold.argtypes = [_P, _I64, _F, _P]
    lib.oracle_sample_positions.restype = None
    lib.oracle_sample_positions.argtypes = [_P, _P, _P, _P, _P, _I64, _P]
    lib.oracle_prune.restype = _I64
    lib.oracle_prune.argtypes = [_P, _I64, _P, _P, _P, ctypes.c_double, ctypes.c_double, _P, _P]
    lib.oracle_blob_field.restype = None
    lib.oracle_blob_field.argtypes = [_P, _P, _I64, _P, _P, _P, _I32, _P, _P,
                                      _I32, _P, _P]
    _lib = lib
    return lib


def _c(a, dtype):
    """Contiguous array of the given dtype (a copy only when needed)."""
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Marching (Sec. 2.1)
# --------------------------------------------------------------------------

LOOKUP_AABB, LOOKUP_CASCADE, LOOKUP_CONTRACT = 0, 1, 2


def march(rays_o, rays_d, mask, res, box, near, far, dt, dt_max=1e10,
          cone=0.0, lookup=LOOKUP_AABB, n_grids=1, grid_id=None,
          max_per_ray=0):
    """Brute-force marching (every lattice candidate tested, no skipping).

    mask: uint8 0/1 [n_grids * res^3] dense occupancy (C order per grid).
    Returns (packed_info i32 [R, 2], ray_indices i32 [E], t_starts f32 [E],
    t_ends f32 [E]).  packed_info[:, 0] is the exclusive prefix sum of the
    counts (the packed layout of Sec. 3).
    """
    lib = _load()
    o = _c(rays_o, np.float32).reshape(-1, 3)
    d = _c(rays_d, np.float32).reshape(-1, 3)
    n = o.shape[0]
    m = _c(mask, np.uint8).ravel()
    assert m.size == n_grids * res ** 3
    bx = _c(box, np.float32).ravel()
    gid = None if grid_id is None else _c(grid_id, np.int32)
    counts = np.zeros(n, np.int32)
    args = (_ptr(o), _ptr(d), _ptr(gid), n, _ptr(m), res, n_grids, lookup,
            _ptr(bx), near, far, dt, dt_max, cone, max_per_ray)
    total = lib.oracle_march(*args, _ptr(counts), 0, None, None, None)
    ri = np.zeros(total, np.int32)
    ts = np.zeros(total, np.float32)
    te = np.zeros(total, np.float32)
    total2 = lib.oracle_march(*args, _ptr(counts), total, _ptr(ri), _ptr(ts),
                              _ptr(te))
    assert total2 == total
    starts = np.zeros(n, np.int64)
    if n > 1:
        starts[1:] = np.cumsum(counts.astype(np.int64))[:-1]
    packed = np.stack([starts, counts.astype(np.int64)], 1).astype(np.int32)
    return packed, ri, ts, te


def clip(rays_o, rays_d, box, near, far):
    """The ray-box clip alone: (t_near f32 [R], t_far f32 [R], hit bool [R])."""
    lib = _load()
    o = _c(rays_o, np.float32).reshape(-1, 3)
    d = _c(rays_d, np.float32).reshape(-1, 3)
    n = o.shape[0]
    bx = _c(box, np.float32).ravel()
    tn = np.zeros(n, np.float32)
    tf = np.zeros(n, np.float32)
    hit = np.zeros(n, np.int32)
    lib.oracle_clip(_ptr(o), _ptr(d), n, _ptr(bx), near, far, _ptr(tn),
                    _ptr(tf), _ptr(hit))
    return tn, tf, hit.astype(bool)


# --------------------------------------------------------------------------
# Rendering, Eq. 1 (Sec. 2.2) and its gradient
# --------------------------------------------------------------------------

def render_fwd(packed_info, t_starts, t_ends, sigmas, rgbs, eps=0.0):
    """FP64 forward.  Returns dict(color [R,3], opacity [R], depth [R],
    weights [E], kept [R]) as float64 / int32 arrays."""
    lib = _load()
    p = _c(packed_info, np.int32).reshape(-1, 2)
    n = p.shape[0]
    ts = _c(t_starts, np.float64).ravel()
    te = _c(t_ends, np.float64).ravel()
    sg = _c(sigmas, np.float64).ravel()
    cl = _c(rgbs, np.float64).reshape(-1, 3)
    color = np.zeros((n, 3))
    opacity = np.zeros(n)
    depth = np.zeros(n)
    weights = np.zeros(ts.size)
    kept = np.zeros(n, np.int32)
    lib.oracle_render_fwd(_ptr(p), n, _ptr(ts), _ptr(te), _ptr(sg), _ptr(cl),
                          float(eps), _ptr(color), _ptr(opacity), _ptr(depth),
                          _ptr(weights), _ptr(kept))
    return dict(color=color, opacity=opacity, depth=depth, weights=weights,
                kept=kept)


def render_bwd(packed_info, t_starts, t_ends, sigmas, rgbs, g_color,
               g_opacity=None, g_depth=None, eps=0.0):
    """FP64 backward.  Returns dict(g_sigmas [E], g_rgbs [E,3], scale [E]);
    scale is the magnitude of the terms that form each sigma gradient (the
    two terms of its difference, each with v summed in magnitude over its own
    terms)."""
    lib = _load()
    p = _c(packed_info, np.int32).reshape(-1, 2)
    n = p.shape[0]
    ts = _c(t_starts, np.float64).ravel()
    te = _c(t_ends, np.float64).ravel()
    sg = _c(sigmas, np.float64).ravel()
    cl = _c(rgbs, np.float64).reshape(-1, 3)
    gc = _c(g_color, np.float64).reshape(-1, 3)
    ga = None if g_opacity is None else _c(g_opacity, np.float64).ravel()
    gd = None if g_depth is None else _c(g_depth, np.float64).ravel()
    gs = np.zeros(ts.size)
    gr = np.zeros((ts.size, 3))
    scale = np.zeros(ts.size)
    rc = lib.oracle_render_bwd(_ptr(p), n, _ptr(ts), _ptr(te), _ptr(sg),
                               _ptr(cl), float(eps), _ptr(gc), _ptr(ga),
                               _ptr(gd), _ptr(gs), _ptr(gr), _ptr(scale))
    if rc != 0:
        raise MemoryError("oracle_render_bwd: allocation failed")
    return dict(g_sigmas=gs, g_rgbs=gr, scale=scale)


def render_attrs_fwd(packed_info, t_starts, t_ends, sigmas, attrs, eps=0.0, alpha_thre=0.0,
                     background=None):
    """FP64 rendering of per-sample attributes attrs [E, C] (Sec. 2.2: any
    sample attribute is rendered), with an optional constant background
    blended by 1 - opacity and samples with alpha < alpha_thre treated as
    empty.  Returns dict(out [R, C], opacity [R], depth [R], weights [E])."""
    lib = _load()
    p = _c(packed_info, np.int32).reshape(-1, 2)
    n = p.shape[0]
    ts = _c(t_starts, np.float64).ravel()
    te = _c(t_ends, np.float64).ravel()
    sg = _c(sigmas, np.float64).ravel()
    at = _c(attrs, np.float64).reshape(ts.size, -1)
    ch = at.shape[1]
    bg = None if background is None else _c(background, np.float64).ravel()
    out = np.zeros((n, ch))
    opacity = np.zeros(n)
    depth = np.zeros(n)
    weights = np.zeros(ts.size)
    lib.oracle_render_attrs_fwd(_ptr(p), n, _ptr(ts), _ptr(te), _ptr(sg), _ptr(at), ch, ch,
                                float(eps), float(alpha_thre), _ptr(bg), _ptr(out),
                                _ptr(opacity), _ptr(depth), _ptr(weights))
    return dict(out=out, opacity=opacity, depth=depth, weights=weights)


def render_attrs_bwd(packed_info, t_starts, t_ends, sigmas, attrs, g_out, g_opacity=None,
                     g_depth=None, eps=0.0, alpha_thre=0.0, background=None):
    """FP64 backward of render_attrs_fwd.  Returns dict(g_sigmas [E],
    g_attrs [E, C], scale [E]) (scale as in render_bwd)."""
    lib = _load()
    p = _c(packed_info, np.int32).reshape(-1, 2)
    n = p.shape[0]
    ts = _c(t_starts, np.float64).ravel()
    te = _c(t_ends, np.float64).ravel()
    sg = _c(sigmas, np.float64).ravel()
    at = _c(attrs, np.float64).reshape(ts.size, -1)
    ch = at.shape[1]
    gout = _c(g_out, np.float64).reshape(n, ch)
    ga = None if g_opacity is None else _c(g_opacity, np.float64).ravel()
    gd = None if g_depth is None else _c(g_depth, np.float64).ravel()
    bg = None if background is None else _c(background, np.float64).ravel()
    gs = np.zeros(ts.size)
    gat = np.zeros((ts.size, ch))
    scale = np.zeros(ts.size)
    rc = lib.oracle_render_attrs_bwd(_ptr(p), n, _ptr(ts), _ptr(te), _ptr(sg), _ptr(at), ch, ch,
                                     float(eps), float(alpha_thre), _ptr(bg), _ptr(gout),
                                     _ptr(ga), _ptr(gd), _ptr(gs), _ptr(gat), _ptr(scale))
    if rc != 0:
        raise MemoryError("oracle_render_attrs_bwd: allocation failed")
    return dict(g_sigmas=gs, g_attrs=gat, scale=scale)


def prune(packed_info, t_starts, t_ends, sigmas, eps=1e-4, alpha_thre=0.0):
    """Visibility pruning of marched samples (Sec. 2.1 occluded regions;
    Sec. 3 ray_marching with sigma_fn): keep iff T_i >= eps and alpha_i >=
    alpha_thre, FP64.  Returns (keep u8 [E], counts i32 [R])."""
    lib = _load()
    pk = _c(packed_info, np.int32).reshape(-1, 2)
    ts = _c(t_starts, np.float64)
    te = _c(t_ends, np.float64)
    sg = _c(sigmas, np.float64)
    keep = np.zeros(ts.size, np.uint8)
    counts = np.zeros(pk.shape[0], np.int32)
    lib.oracle_prune(_ptr(pk), pk.shape[0], _ptr(ts), _ptr(te), _ptr(sg), float(eps),
                     float(alpha_thre), _ptr(keep), _ptr(counts))
    return keep, counts


def mse_loss_and_grad(color, target):
    """loss = mean((color - target)^2) over all R*3 values (the loss of the
    training step in Sec. 3) and its gradient 2 (color - target) / (3R)."""
    c = np.asarray(color, np.float64)
    t = np.asarray(target, np.float64)
    diff = c - t
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


# --------------------------------------------------------------------------
# Occupancy-grid update (Sec. 2.1; update rule read from Instant-NGP)
# --------------------------------------------------------------------------

def philox4x64_10(counter, key):
    """One Philox4x64-10 block: counter (4 x uint64), key (2 x uint64)."""
    lib = _load()
    c = _c(counter, np.uint64)
    k = _c(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib.oracle_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def grid_sample_cells(seed, step, n, res, box, levels=1, cascade=False):
    """Random cells and jittered positions of update `step` (positions scaled
    by 2^level for cascaded grids)."""
    lib = _load()
    bx = _c(box, np.float32).ravel()
    cells = np.zeros(n, np.int32)
    pos = np.zeros((n, 3), np.float32)
    lib.oracle_grid_sample_cells(seed, step, n, res, levels, int(cascade), _ptr(bx),
                                 _ptr(cells), _ptr(pos))
    return cells, pos


def grid_decay(occ, decay):
    lib = _load()
    o = np.array(occ, np.float32, copy=True).ravel()
    lib.oracle_grid_decay(_ptr(o), o.size, decay)
    return o


def grid_update_max(occ, cells, values):
    lib = _load()
    o = np.array(occ, np.float32, copy=True).ravel()
    c = _c(cells, np.int32)
    v = _c(values, np.float32)
    lib.oracle_grid_update_max(_ptr(o), _ptr(c), _ptr(v), c.size)
    return o


def grid_threshold(occ, threshold):
    """Dense 0/1 mask: occ > threshold."""
    lib = _load()
    o = _c(occ, np.float32).ravel()
    m = np.zeros(o.size, np.uint8)
    lib.oracle_grid_threshold(_ptr(o), o.size, threshold, _ptr(m))
    return m


# --------------------------------------------------------------------------
# Synthetic stand-in field (test input, not the method)
# --------------------------------------------------------------------------

def sample_positions(rays_o, rays_d, ray_indices, t_starts, t_ends):
    """FP32 sample midpoints x = o + d * ((t_start + t_end) * 0.5)."""
    lib = _load()
    o = _c(rays_o, np.float32).reshape(-1, 3)
    d = _c(rays_d, np.float32).reshape(-1, 3)
    ri = _c(ray_indices, np.int32)
    ts = _c(t_starts, np.float32)
    te = _c(t_ends, np.float32)
    pos = np.zeros((ri.size, 3), np.float32)
    lib.oracle_sample_positions(_ptr(o), _ptr(d), _ptr(ri), _ptr(ts), _ptr(te),
                                ri.size, _ptr(pos))
    return pos


def blob_field(scene, positions, blob_set=None, want_rgb=True):
    """FP64 density (and colour) of a synth.BlobScene at FP32 positions
    (a scene with `contract` set is defined in contracted coordinates)."""
    lib = _load()
    pos = _c(positions, np.float32).reshape(-1, 3)
    n = pos.shape[0]
    bs = None if blob_set is None else _c(blob_set, np.int32)
    cen = _c(scene.centres, np.float32)
    std = _c(scene.stds, np.float32)
    pk = _c(scene.peaks, np.float32)
    w = _c(scene.w, np.float32)
    b = _c(scene.bias, np.float32)
    sigma = np.zeros(n)
    rgb = np.zeros((n, 3)) if want_rgb else None
    lib.oracle_blob_field(_ptr(pos), _ptr(bs), n, _ptr(cen), _ptr(std),
                          _ptr(pk), scene.n_blobs, _ptr(w), _ptr(b),
                          int(bool(getattr(scene, "contract", False))),
                          _ptr(sigma), _ptr(rgb))
    return (sigma, rgb) if want_rgb else sigma
