"""GPU parity of whole-image forward rendering (pinhole cameras on an orbit
around the training scene), at one tenth of the image sizes: marching bit
for bit against the oracle on every ray, rendering against the oracle on
sampled rays, and all images in one call sequence against one call
sequence per image, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import assert_bit_exact, check_forward

pytestmark = pytest.mark.gpu

SCALE = 10


@pytest.fixture(scope="module")
def images():
    import paper_2210_04847_amd as nacc
    w = synth.IMAGE_WORKLOADS["images_8"]
    inp = synth.image_inputs(w, scale=SCALE)
    sw = inp["scene_workload"]
    grid = nacc.OccupancyGrid(sw.box, sw.res)
    grid.set_occupancy(torch.from_numpy(inp["occ"]).cuda(), 0.01)
    field = nacc.BlobField(inp["scene"])
    return w, inp, sw, grid, field, nacc


def _render(nacc, grid, field, sw, eps, o, d):
    packed, ri, ts, te = nacc.ray_marching(o, d, grid, sw.near, sw.far, sw.dt)
    sig, rgb = field.samples(o, d, ri, ts, te)
    color, opacity, depth = nacc.rendering(packed, ts, te, sig, rgb, early_stop_eps=eps)
    torch.cuda.synchronize()
    return packed, ri, ts, te, sig, rgb, color, opacity, depth


def test_images_march_and_render(images):
    w, inp, sw, grid, field, nacc = images
    o = torch.from_numpy(inp["rays_o"]).cuda()
    d = torch.from_numpy(inp["rays_d"]).cuda()
    packed, ri, ts, te, sig, rgb, color, opacity, depth = _render(nacc, grid, field, sw,
                                                                   w.early_stop_eps, o, d)
    mask = oracle.grid_threshold(inp["occ"], 0.01)
    p_o, ri_o, ts_o, te_o = oracle.march(inp["rays_o"], inp["rays_d"], mask, sw.res,
                                         np.asarray(sw.box, np.float32), sw.near, sw.far, sw.dt)
    assert ri_o.size > 100000 and (p_o[:, 1] == 0).any()  # corners miss the box
    assert_bit_exact(packed.cpu().numpy(), p_o, "packed_info")
    assert_bit_exact(ri.cpu().numpy(), ri_o, "ray_indices")
    assert_bit_exact(ts.cpu().numpy(), ts_o, "t_starts")
    assert_bit_exact(te.cpu().numpy(), te_o, "t_ends")
    rays = np.sort(np.random.default_rng(61).choice(packed.shape[0], 3000, replace=False))
    pk = p_o[rays].copy()
    idx = np.concatenate([np.arange(a, a + n) for a, n in pk]).astype(np.int64)
    pk[:, 0] = np.concatenate([[0], np.cumsum(pk[:-1, 1])])
    got = dict(color=color.cpu().numpy()[rays], opacity=opacity.cpu().numpy()[rays],
               depth=depth.cpu().numpy()[rays])
    check_forward(got, pk, ts_o[idx], te_o[idx], sig.cpu().numpy()[idx], rgb.cpu().numpy()[idx],
                  w.early_stop_eps)


def test_images_batched_equals_per_image(images):
    w, inp, sw, grid, field, nacc = images
    o = torch.from_numpy(inp["rays_o"]).cuda()
    d = torch.from_numpy(inp["rays_d"]).cuda()
    all_out = _render(nacc, grid, field, sw, w.early_stop_eps, o, d)
    offs = np.concatenate([[0], np.cumsum(inp["counts"])])
    parts = [_render(nacc, grid, field, sw, w.early_stop_eps, o[a:b], d[a:b])
             for a, b in zip(offs[:-1], offs[1:])]
    for j, name in ((6, "color"), (7, "opacity"), (8, "depth")):
        cat = torch.cat([p[j] for p in parts])
        assert torch.equal(all_out[j].view(torch.int32), cat.view(torch.int32)), name
    counts = torch.cat([p[0][:, 1] for p in parts])
    assert torch.equal(all_out[0][:, 1], counts)
