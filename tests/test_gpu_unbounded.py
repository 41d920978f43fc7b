"""GPU parity of the unbounded-scene path at a size the oracle covers whole:
rays from inside the unit ball in all directions (3,000 of them: a ragged
last workgroup), cone-scaled steps t_{k+1} = t_k + clamp(t_k / 256, dt,
dt_max) from near = 0.2, and a scene defined in contracted coordinates, for
both unbounded grid layouts, marched with the skip field: four cascaded
32^3 grids (level l over [-2^l, 2^l]^3) and the paper's contraction lookup
(one 32^3 grid over the contracted space [-2, 2]^3, lattice to far = 1e4,
at most 1024 samples per ray).  Marching is compared bit for bit, the field
within its FP32 tolerance, and the fused render + MSE + backward on the
step's own samples within the render and gradient tolerances."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth
from parity import assert_bit_exact, check_backward, check_forward
from steps import field_tolerance, make_step, march_kwargs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["unbounded_262k", "unbounded_contract_262k"])
def small(request):
    # with the skip field (the cascade benchmark marches without it)
    return make_step(request.param, n_rays=3000, res=32, skip_field=True)


def test_unbounded_march_all_rays(small):
    w, inp, st = small
    e = int(st.total.item())
    mask = oracle.grid_threshold(inp["occ"], 0.01)
    packed, ri, ts, te = oracle.march(inp["rays_o"], inp["rays_d"], mask, inp["res"],
                                      np.asarray(w.box, np.float32), w.near, w.far, w.dt,
                                      **march_kwargs(w))
    assert e == ri.size and e > 10000
    counts = packed[:, 1]
    assert (counts == 0).mean() < 0.9 and counts.max() > 100  # ragged
    assert_bit_exact(st.packed.cpu().numpy(), packed, "packed_info")
    assert_bit_exact(st.ray_indices[:e].cpu().numpy(), ri, "ray_indices")
    assert_bit_exact(st.t_starts[:e].cpu().numpy(), ts, "t_starts")
    assert_bit_exact(st.t_ends[:e].cpu().numpy(), te, "t_ends")
    # the capacity bound covers every ray
    lib = st.lib
    assert counts.max() <= lib.march_max_samples_per_ray(st.grid.desc, st.params)
    if w.max_per_ray:
        assert counts.max() <= w.max_per_ray


def test_unbounded_field_all_samples(small):
    w, inp, st = small
    e = int(st.total.item())
    ri = st.ray_indices[:e].cpu().numpy()
    pos = oracle.sample_positions(inp["rays_o"], inp["rays_d"], ri, st.t_starts[:e].cpu().numpy(),
                                  st.t_ends[:e].cpu().numpy())
    s_o, c_o = oracle.blob_field(inp["scene"], pos)
    tol = field_tolerance(inp["scene"], pos, s_o)
    assert np.all(np.abs(st.sigmas[:e].cpu().numpy() - s_o) <= tol)
    assert np.all(np.abs(st.rgbs[:e].cpu().numpy() - c_o) <= 1e-5 * c_o + 4e-6)


def test_unbounded_fused_render(small):
    w, inp, st = small
    st.render()
    torch.cuda.synchronize()
    e = int(st.total.item())
    n = st.n
    packed = st.packed.cpu().numpy()
    ts, te = st.t_starts[:e].cpu().numpy(), st.t_ends[:e].cpu().numpy()
    sg, cl = st.sigmas[:e].cpu().numpy(), st.rgbs[:e].cpu().numpy()
    eps = w.early_stop_eps
    got = dict(color=st.color.cpu().numpy(), opacity=st.opacity.cpu().numpy(),
               depth=st.depth.cpu().numpy())
    ref, _ = check_forward(got, packed, ts, te, sg, cl, eps)
    diff = ref["color"] - inp["targets"].astype(np.float64)
    want_loss = float(np.mean(diff * diff))
    assert abs(float(st.loss.item()) - want_loss) <= 1e-5 * want_loss
    g_color = 2.0 * diff / (3 * n)
    dg = 2.0 / (3 * n) * 1e-5 * np.abs(ref["color"]).max(1)
    prop = oracle.render_bwd(packed, ts, te, sg, cl, np.repeat(dg[:, None], 3, 1), eps=eps)
    ray_of = np.repeat(np.arange(n), packed[:, 1])
    check_backward(st.g_sigmas[:e].cpu().numpy(), st.g_rgbs[:e].cpu().numpy(), packed, ts, te,
                   sg, cl, g_color, None, None, eps, extra_scale=prop["scale"],
                   extra_rgb=(ref["weights"] * dg[ray_of])[:, None])


def test_unbounded_grid_update(small):
    """One grid update: cascades draw cells over all levels, positions scaled
    to their level, and read the field at the contraction of the world
    position; the contraction lookup draws positions in the contracted space
    and reads the field there directly.  Then max into the decayed
    densities and repack."""
    w, inp, st = small
    occ0 = inp["occ"]
    st.grid.set_occupancy(torch.from_numpy(occ0).cuda(), 0.01)
    st.updates.zero_()
    st.grid_update()
    torch.cuda.synchronize()
    res = inp["res"]
    cascade = w.lookup == "cascade"
    cells, pos = oracle.grid_sample_cells(st.seed, 0, 1 << 18, res,
                                          np.asarray(w.box, np.float32), w.cascades, cascade)
    # the scene as a field of contracted-space points
    scene = inp["scene"] if cascade else dataclasses.replace(inp["scene"], contract=False)
    sig = oracle.blob_field(scene, pos, want_rgb=False)
    got_sig = st.ema_sigma.cpu().numpy()
    assert_bit_exact(st.ema_cells.cpu().numpy(), cells, "cells")
    assert_bit_exact(st.ema_pos.cpu().numpy(), pos, "positions")
    assert np.all(np.abs(got_sig - sig) <= field_tolerance(scene, pos, sig))
    if not cascade:
        assert np.abs(pos).max() > 1.9 and (sig > 0.01).mean() > 0.001
    # with the GPU's own densities the update is bit-exact
    want = oracle.grid_update_max(oracle.grid_decay(occ0, 0.95), cells, got_sig)
    assert_bit_exact(st.grid.occ.cpu().numpy(), want, "occupancy after the update")
    bits = np.packbits(oracle.grid_threshold(want, 0.01).astype(np.uint8),
                       bitorder="little").view("<u4").view(np.int32)
    assert_bit_exact(st.grid.bits.cpu().numpy(), bits, "repacked bits")
