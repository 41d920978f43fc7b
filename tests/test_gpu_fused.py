"""GPU tests of the fused inference kernel (marching, the synthetic field and
the forward render of each ray in one kernel, no samples written out).

Its chunks are the ray's samples 64 at a time, the chunks the rendering
kernel reads, so it must give the bits of the three-step form (marching,
then the field at the samples, then the forward render) on every ray; that
form is itself checked against the oracle elsewhere.  Here the fused outputs
are also compared with the oracle directly: against the oracle's render of
the same samples and field values (the render tolerances), and end to end
against the oracle's marching, FP64 field and render, with the error of the
FP32 field propagated through the render's sensitivities.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth
from parity import RENDER_RTOL, assert_bit_exact, check_forward

pytestmark = pytest.mark.gpu

BOX = np.array(synth.BOX_1_5, np.float32)


def _nacc():
    import paper_2210_04847_amd as nacc
    return nacc


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bits(t):
    return t.contiguous().view(torch.int32)


def _three_step(nacc, field, grid, o, d, near, far, dt, eps, max_per_ray=0, grid_id=None,
                ray_set=None):
    packed, ri, ts, te = nacc.ray_marching(o, d, grid, near, far, dt, max_per_ray=max_per_ray,
                                           grid_id=grid_id)
    rs = None if ray_set is None else ray_set.to(torch.int32).contiguous()
    sig, rgb = field.samples(o, d, ri, ts, te, ray_set=rs)
    kept = torch.empty(o.shape[0], dtype=torch.int32, device="cuda")
    color = torch.empty((o.shape[0], 3), dtype=torch.float32, device="cuda")
    opac = torch.empty(o.shape[0], dtype=torch.float32, device="cuda")
    dep = torch.empty(o.shape[0], dtype=torch.float32, device="cuda")
    nacc._lib.render_fwd(packed, ts, te, sig, rgb, eps, color, opac, dep, None, kept)
    torch.cuda.synchronize()
    return dict(packed=packed, ri=ri, ts=ts, te=te, sig=sig, rgb=rgb, color=color, opacity=opac,
                depth=dep, kept=kept)


def _assert_same(fused, ref):
    color, opacity, depth, kept = fused
    assert torch.equal(_bits(color), _bits(ref["color"])), "color"
    assert torch.equal(_bits(opacity), _bits(ref["opacity"])), "opacity"
    assert torch.equal(_bits(depth), _bits(ref["depth"])), "depth"
    assert torch.equal(kept, ref["kept"]), "samples before the cut"


@pytest.fixture(scope="module")
def train4k():
    nacc = _nacc()
    w = synth.WORKLOADS["train_262k"]
    inp = synth.workload_inputs(w, 4099)  # a ragged last workgroup
    grid = nacc.OccupancyGrid(w.box, w.res)
    grid.set_occupancy(_cuda(inp["occ"]), 0.01)
    field = nacc.BlobField(inp["scene"])
    return nacc, w, inp, grid, field


@pytest.mark.parametrize("skip", [True, False])
@pytest.mark.parametrize("eps", [1e-4, 0.0, 0.05])
def test_fused_equals_three_steps(train4k, eps, skip):
    """With the grid's skip buffer (marching by the segments of its halo
    bits) and without."""
    nacc, w, inp, grid, field = train4k
    o, d = _cuda(inp["rays_o"]), _cuda(inp["rays_d"])
    ref = _three_step(nacc, field, grid, o, d, w.near, w.far, w.dt, eps)
    fused = nacc.render_fused(field, o, d, grid, w.near, w.far, w.dt, eps, return_kept=True,
                              skip_empty=skip)
    torch.cuda.synchronize()
    _assert_same(fused, ref)
    counts = ref["packed"][:, 1]
    assert int(counts.max()) > 128 and int((counts == 0).sum()) > 0
    if eps > 0.01:
        assert int((ref["kept"] < counts).sum()) > 100  # the cut stops many rays early


@pytest.mark.parametrize("seed", range(16))
def test_fused_random_scenes_equal_three_steps(seed):
    """Random blob scenes, grid resolutions and thresholds, ray counts (the
    64-ray workgroup edges), step sizes, cut thresholds, caps and skip
    settings: the fused kernel gives the three-step form's bits on every ray."""
    nacc = _nacc()
    rng = np.random.default_rng(5000 + seed)
    scene = synth.blob_scene(int(rng.integers(1, 40)), 6000 + seed, peak=float(rng.choice([5.0, 50.0, 500.0])))
    res = int(rng.choice([16, 32, 64, 128]))
    grid = nacc.OccupancyGrid(tuple(BOX[:3]) + tuple(BOX[3:]), res)
    grid.set_occupancy(_cuda(synth.initial_occupancy(scene, res, BOX)), float(rng.choice([1e-3, 0.01, 1.0])))
    field = nacc.BlobField(scene)
    n = int(rng.choice([1, 63, 64, 65, 700, 3000]))
    o, d = synth.rays_toward_origin(n, 7000 + seed, jitter_std=float(rng.choice([0.1, 1.0])))
    o, d = _cuda(o), _cuda(d)
    dt = float(np.float32(3 ** 0.5 * 3 / float(rng.choice([256, 1024, 4096]))))
    eps = float(rng.choice([0.0, 1e-4, 1e-2]))
    cap = int(rng.choice([0, 0, 50, 300]))
    skip = bool(rng.integers(0, 2))
    ref = _three_step(nacc, field, grid, o, d, 0.0, 1e10, dt, eps, max_per_ray=cap)
    fused = nacc.render_fused(field, o, d, grid, 0.0, 1e10, dt, eps, max_per_ray=cap, return_kept=True,
                              skip_empty=skip)
    torch.cuda.synchronize()
    _assert_same(fused, ref)


def test_fused_matches_oracle_render_of_its_samples(train4k):
    """Against the oracle's FP64 render of the marched samples at the field
    values the field kernel gives them (the render tolerances)."""
    nacc, w, inp, grid, field = train4k
    o, d = _cuda(inp["rays_o"]), _cuda(inp["rays_d"])
    ref = _three_step(nacc, field, grid, o, d, w.near, w.far, w.dt, w.early_stop_eps)
    color, opacity, depth = nacc.render_fused(field, o, d, grid, w.near, w.far, w.dt,
                                              w.early_stop_eps)
    torch.cuda.synchronize()
    e = ref["ri"].numel()
    got = dict(color=color.cpu().numpy(), opacity=opacity.cpu().numpy(), depth=depth.cpu().numpy())
    check_forward(got, ref["packed"].cpu().numpy(), ref["ts"].cpu().numpy(), ref["te"].cpu().numpy(),
                  ref["sig"][:e].cpu().numpy(), ref["rgb"][:e].cpu().numpy(), w.early_stop_eps)


def test_fused_end_to_end_against_oracle(train4k):
    """Oracle marching (bit for bit the same samples), the oracle's FP64
    field and FP64 render.  The FP32 field's error (2e-5 relative in sigma,
    1e-5 relative + 4e-6 in rgb) moves the render by at most
    sum_s |dC/dsigma_s| |d sigma_s| + sum_s w_s |d c_s|; |dC/dsigma_s| is
    bounded by the oracle's gradient term magnitudes with unit upstream
    gradient.  Rays whose transmittance passes within 1e-3 of eps may cut at
    a neighbouring sample and are held to eps * (max colour + 1)."""
    nacc, w, inp, grid, field = train4k
    o, d = _cuda(inp["rays_o"]), _cuda(inp["rays_d"])
    eps = w.early_stop_eps
    color, opacity, depth = nacc.render_fused(field, o, d, grid, w.near, w.far, w.dt, eps)
    torch.cuda.synchronize()
    mask = oracle.grid_threshold(inp["occ"], 0.01)
    packed, ri, ts, te = oracle.march(inp["rays_o"], inp["rays_d"], mask, w.res, BOX, w.near, w.far,
                                      w.dt)
    pos = oracle.sample_positions(inp["rays_o"], inp["rays_d"], ri, ts, te)
    sig, rgb = oracle.blob_field(inp["scene"], pos)
    ref = oracle.render_fwd(packed, ts, te, sig, rgb, eps)
    n = packed.shape[0]
    ray_of = np.repeat(np.arange(n), packed[:, 1])
    d_sig = 2e-5 * sig
    d_rgb = 1e-5 * rgb + 4e-6
    outs = dict(color=color.cpu().numpy().astype(np.float64),
                opacity=opacity.cpu().numpy().astype(np.float64),
                depth=depth.cpu().numpy().astype(np.float64))
    m = 0.5 * (ts.astype(np.float64) + te.astype(np.float64))
    # sensitivities: unit upstream gradient on one output at a time
    sens = {}
    for k in range(3):
        g = np.zeros((n, 3))
        g[:, k] = 1.0
        sens[("color", k)] = oracle.render_bwd(packed, ts, te, sig, rgb, g, eps=eps)["scale"]
    zero = np.zeros((n, 3))
    sens[("opacity", 0)] = oracle.render_bwd(packed, ts, te, sig, rgb, zero, np.ones(n),
                                             eps=eps)["scale"]
    sens[("depth", 0)] = oracle.render_bwd(packed, ts, te, sig, rgb, zero, None, np.ones(n),
                                           eps=eps)["scale"]
    # rays whose cut is ambiguous under the field's error
    tau = sig * (te.astype(np.float64) - ts.astype(np.float64))
    amb = np.zeros(n, bool)
    for r in np.flatnonzero(packed[:, 1]):
        a, c = packed[r]
        trans = np.exp(-np.concatenate([[0.0], np.cumsum(tau[a:a + c])[:-1]]))
        amb[r] = np.any(np.abs(trans - eps) <= 1e-3 * eps)
    for name, chans in (("color", 3), ("opacity", 1), ("depth", 1)):
        got = outs[name].reshape(n, chans)
        want = ref[name].reshape(n, chans)
        for k in range(chans):
            prop = np.bincount(ray_of, sens[(name, k)] * d_sig, minlength=n)
            if name == "color":
                prop += np.bincount(ray_of, ref["weights"] * d_rgb[:, k], minlength=n)
            tol = RENDER_RTOL * np.abs(want[:, k]) + 1e-12 + prop
            tol = np.where(amb, np.maximum(tol, eps * (np.abs(want[:, k]).max() + 1.0) + prop), tol)
            bad = np.flatnonzero(np.abs(got[:, k] - want[:, k]) > tol)
            assert bad.size == 0, (f"{name}[{k}]: {bad.size} rays, e.g. {bad[0]}: "
                                   f"{got[bad[0], k]} vs {want[bad[0], k]} (tol {tol[bad[0]]})")
    assert amb.sum() < 0.01 * n


def test_fused_max_per_ray_and_lookups():
    """A per-ray cap falling inside a 64-candidate chunk, and uniform steps
    through cascades and through the contraction lookup."""
    nacc = _nacc()
    w = synth.WORKLOADS["train_262k"]
    inp = synth.workload_inputs(w, 1500)
    grid = nacc.OccupancyGrid(w.box, w.res)
    grid.set_occupancy(_cuda(inp["occ"]), 0.01)
    field = nacc.BlobField(inp["scene"])
    o, d = _cuda(inp["rays_o"]), _cuda(inp["rays_d"])
    for cap in (37, 64, 100):
        ref = _three_step(nacc, field, grid, o, d, w.near, w.far, w.dt, 1e-4, max_per_ray=cap)
        assert int(ref["packed"][:, 1].max()) == cap
        for skip in (True, False):
            _assert_same(nacc.render_fused(field, o, d, grid, w.near, w.far, w.dt, 1e-4,
                                           max_per_ray=cap, return_kept=True, skip_empty=skip), ref)
    uw = synth.UNBOUNDED_WORKLOADS["unbounded_262k"]
    uin = synth.unbounded_inputs(uw, 1200, 32)
    uf = nacc.BlobField(uin["scene"])
    uo, ud = _cuda(uin["rays_o"]), _cuda(uin["rays_d"])
    cg = nacc.OccupancyGrid(uw.box, 32, n_grids=uw.cascades, lookup="cascade")
    cg.set_occupancy(_cuda(uin["occ"]), 0.01)
    ref = _three_step(nacc, uf, cg, uo, ud, uw.near, 30.0, 0.02, 1e-4)
    assert ref["ri"].numel() > 10000
    _assert_same(nacc.render_fused(uf, uo, ud, cg, uw.near, 30.0, 0.02, 1e-4, return_kept=True),
                 ref)
    kw = synth.UNBOUNDED_WORKLOADS["unbounded_contract_262k"]
    kin = synth.unbounded_inputs(kw, 1200, 32)
    kg = nacc.OccupancyGrid(kw.box, 32, lookup="contract")
    kg.set_occupancy(_cuda(kin["occ"]), 0.01)
    ref = _three_step(nacc, uf, kg, uo, ud, kw.near, 200.0, 0.02, 1e-4, max_per_ray=1024)
    assert ref["ri"].numel() > 10000
    _assert_same(nacc.render_fused(uf, uo, ud, kg, kw.near, 200.0, 0.02, 1e-4, max_per_ray=1024,
                                   return_kept=True), ref)


def test_fused_coarse_steps_and_workgroup_clocks(train4k):
    """Steps too long for segments (each ray marched candidate by candidate
    although the skip buffer is given), and the per-workgroup clocks: set
    for every group of 64 rays, start before end, within the launch, and
    the colours the same as without them."""
    nacc, w, inp, grid, field = train4k
    lib = nacc._lib
    o, d = _cuda(inp["rays_o"]), _cuda(inp["rays_d"])
    ref = _three_step(nacc, field, grid, o, d, w.near, w.far, 0.05, 1e-4)
    _assert_same(nacc.render_fused(field, o, d, grid, w.near, w.far, 0.05, 1e-4, return_kept=True),
                 ref)
    n = o.shape[0]
    groups = (n + 63) // 64
    clocks = torch.zeros(2 * groups, dtype=torch.int64, device="cuda")
    color = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    opacity = torch.empty(n, dtype=torch.float32, device="cuda")
    depth = torch.empty(n, dtype=torch.float32, device="cuda")
    kept = torch.empty(n, dtype=torch.int32, device="cuda")
    params = lib.march_params(w.near, w.far, w.dt)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    lib.synth_render_fused(field.table, field.n_blobs, field.n_sets, None, o, d, None, grid.bits,
                           grid.desc, params, 1e-4, color, opacity, depth, kept, grid.skip, clocks)
    stop.record()
    torch.cuda.synchronize()
    want = _three_step(nacc, field, grid, o, d, w.near, w.far, w.dt, 1e-4)
    _assert_same((color, opacity, depth, kept), want)
    c = clocks.view(groups, 2).cpu().numpy()
    assert (c > 0).all() and (c[:, 1] >= c[:, 0]).all()
    khz = lib.wall_clock_khz(0)
    assert khz > 0
    span_ms = (int(c[:, 1].max()) - int(c[:, 0].min())) / khz
    assert 0 < span_ms <= start.elapsed_time(stop) * 1.05 + 0.05


def test_fused_frames_grid_ids_and_edge_cases():
    """Per-ray grids and centre sets (frames of a dynamic scene, invalid ids
    included), no rays, and cone steps refused."""
    nacc = _nacc()
    w = synth.DYNAMIC_WORKLOADS["dynamic_64"]
    inp = synth.dynamic_inputs(w, 5, 32, 300)
    grid = nacc.OccupancyGrid(w.box, 32, n_grids=5)
    grid.set_occupancy(_cuda(inp["occ"]), 0.01)
    field = nacc.BlobField(inp["scene"])
    o, d = _cuda(inp["rays_o"]), _cuda(inp["rays_d"])
    gid = inp["frame"].copy()
    gid[::97] = -1
    gid[1::89] = 5  # out of range: no samples
    g_t, s_t = _cuda(gid), _cuda(inp["frame"])
    ref = _three_step(nacc, field, grid, o, d, w.near, w.far, w.dt, 1e-4, grid_id=g_t, ray_set=s_t)
    _assert_same(nacc.render_fused(field, o, d, grid, w.near, w.far, w.dt, 1e-4, grid_id=g_t,
                                   ray_set=s_t, return_kept=True), ref)
    assert int(ref["packed"][::97, 1].sum()) == 0
    empty = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    c, a, dd = nacc.render_fused(field, empty, empty, grid, w.near, w.far, w.dt)
    assert c.shape == (0, 3) and a.numel() == 0
    lib = nacc._lib
    with pytest.raises(lib.NaccError) as err:
        lib.synth_render_fused(field.table, field.n_blobs, field.n_sets, None, o, d, None,
                               grid.bits, grid.desc, lib.march_params(0.2, 100.0, 0.01, cone=0.01),
                               1e-4, torch.empty((o.shape[0], 3), device="cuda"),
                               torch.empty(o.shape[0], device="cuda"),
                               torch.empty(o.shape[0], device="cuda"))
    assert err.value.status == lib.NACC_ENOTSUP


def test_fused_images_equal_three_steps():
    """The eight orbit images at one tenth of their size: every pixel."""
    nacc = _nacc()
    w = synth.IMAGE_WORKLOADS["images_8"]
    inp = synth.image_inputs(w, scale=10)
    sw = inp["scene_workload"]
    grid = nacc.OccupancyGrid(sw.box, sw.res)
    grid.set_occupancy(_cuda(inp["occ"]), 0.01)
    field = nacc.BlobField(inp["scene"])
    o, d = _cuda(inp["rays_o"]), _cuda(inp["rays_d"])
    ref = _three_step(nacc, field, grid, o, d, sw.near, sw.far, sw.dt, w.early_stop_eps)
    _assert_same(nacc.render_fused(field, o, d, grid, sw.near, sw.far, sw.dt, w.early_stop_eps,
                                   return_kept=True), ref)
