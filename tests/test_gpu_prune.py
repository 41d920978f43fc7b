"""GPU parity of visibility pruning (keep a marched sample iff its
transmittance is at least eps and its opacity at least alpha_thre) against
the FP64 oracle.

The keep decision compares an FP32 quantity with a threshold, so a sample
whose oracle value lies within a relative band of the threshold may go
either way; keep is monotone in both thresholds, so the GPU's flags must lie
between the oracle's flags at thresholds raised and lowered by the band.
Everything else is exact: the per-ray counts are the sums of the flags, and
the compacted samples are the input samples the flags select, bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import assert_bit_exact

pytestmark = pytest.mark.gpu

BAND = 2e-5  # relative error of the FP32 transmittance and opacity, generously


def _lib():
    import paper_2210_04847_amd as nacc
    return nacc._lib


def _gpu_prune(packed, ts, te, sg, eps, thre):
    lib = _lib()
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    p_d, ts_d, te_d, sg_d = cu(packed), cu(ts), cu(te), cu(sg)
    n, e = packed.shape[0], ts.size
    keep = torch.full((max(e, 1),), 7, dtype=torch.uint8, device="cuda")[:e]
    p_out = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    total = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(max(lib.prune_workspace_size(n), 1), dtype=torch.uint8, device="cuda")
    lib.prune_count(p_d, ts_d, te_d, sg_d, eps, thre, keep, p_out, total, ws)
    k = int(total.item())
    ri = torch.empty(k, dtype=torch.int32, device="cuda")
    ts_o = torch.empty(k, dtype=torch.float32, device="cuda")
    te_o = torch.empty(k, dtype=torch.float32, device="cuda")
    sg_o = torch.empty(k, dtype=torch.float32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    lib.prune_fill(p_d, ts_d, te_d, sg_d, keep, p_out, ri, ts_o, te_o, sg_o, status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    return (keep.cpu().numpy(), p_out.cpu().numpy(), ri.cpu().numpy(), ts_o.cpu().numpy(),
            te_o.cpu().numpy(), sg_o.cpu().numpy())


def check_prune(packed, ts, te, sg, eps, thre):
    keep, p_out, ri, ts_o, te_o, sg_o = _gpu_prune(packed, ts, te, sg, eps, thre)
    assert set(np.unique(keep)) <= {0, 1}
    # between the oracle at thresholds raised and lowered by the band
    strict, _ = oracle.prune(packed, ts, te, sg, eps * (1 + BAND), thre * (1 + BAND))
    loose, _ = oracle.prune(packed, ts, te, sg, eps * (1 - BAND), thre * (1 - BAND))
    exact, _ = oracle.prune(packed, ts, te, sg, eps, thre)
    assert np.all(strict <= keep) and np.all(keep <= loose)
    assert keep.size == 0 or np.mean(keep == exact) > 0.999
    # counts, starts and the compacted samples follow the flags exactly
    n = packed.shape[0]
    ray_of = np.repeat(np.arange(n), packed[:, 1])
    counts = np.bincount(ray_of[keep == 1], minlength=n)
    assert_bit_exact(p_out[:, 1], counts.astype(np.int32), "kept counts")
    assert_bit_exact(p_out[:, 0], (np.cumsum(counts) - counts).astype(np.int32), "kept starts")
    sel = keep == 1
    assert_bit_exact(ri, ray_of[sel].astype(np.int32), "ray_indices")
    assert_bit_exact(ts_o, ts[sel], "t_starts")
    assert_bit_exact(te_o, te[sel], "t_ends")
    assert_bit_exact(sg_o, sg[sel], "sigmas")
    return keep


@pytest.mark.parametrize("eps,thre", [(1e-4, 0.0), (1e-4, 1e-2), (0.0, 1e-2), (1e-2, 0.3),
                                      (0.0, 0.0)])
def test_prune_ragged(eps, thre):
    packed, ts, te, sg, _ = synth.ragged_render_inputs(3000, 81, mean_count=60, max_count=700)
    keep = check_prune(packed, ts, te, sg, eps, thre)
    if eps == 0.0 and thre == 0.0:
        assert keep.all()
    else:
        assert 0 < keep.mean() < 1


def test_prune_empty_and_long_rays():
    packed, ts, te, sg, _ = synth.ragged_render_inputs(200, 82, mean_count=400, max_count=3000,
                                                       sigma_max=2.0, empty_frac=0.3)
    check_prune(packed, ts, te, sg, 1e-4, 1e-3)
    check_prune(packed[:0], ts[:0], te[:0], sg[:0], 1e-4, 1e-3)


def test_prune_marched_training_samples():
    """The training workload's own samples (4,096 rays), densities from the
    synthetic field: the pruning the paper's ray_marching applies with a
    sigma_fn, through the library's Python entry point."""
    import paper_2210_04847_amd as nacc
    w = synth.WORKLOADS["train_262k"]
    inp = synth.workload_inputs(w, 4096)
    grid = nacc.OccupancyGrid(w.box, w.res)
    grid.set_occupancy(torch.from_numpy(inp["occ"]).cuda(), 0.01)
    field = nacc.BlobField(inp["scene"])
    o = torch.from_numpy(inp["rays_o"]).cuda()
    d = torch.from_numpy(inp["rays_d"]).cuda()
    packed, ri, ts, te = nacc.ray_marching(o, d, grid, w.near, w.far, w.dt)
    sig, _ = field.samples(o, d, ri, ts, te)
    keep = check_prune(packed.cpu().numpy(), ts.cpu().numpy(), te.cpu().numpy(),
                       sig.cpu().numpy(), 1e-4, 1e-2)
    assert keep.mean() < 0.9
    # the same through ray_marching(sigma_fn=...)
    sigma_fn = lambda t0, t1, r: field.samples(o, d, r, t0, t1)[0]
    p2, ri2, ts2, te2 = nacc.ray_marching(o, d, grid, w.near, w.far, w.dt, sigma_fn=sigma_fn,
                                          early_stop_eps=1e-4, alpha_thre=1e-2)
    torch.cuda.synchronize()
    sel = keep == 1
    assert_bit_exact(ts2.cpu().numpy(), ts.cpu().numpy()[sel], "t_starts via sigma_fn")
    assert_bit_exact(ri2.cpu().numpy(), ri.cpu().numpy()[sel], "ray_indices via sigma_fn")


def test_pruned_training_step():
    """The benchmark's pruned step (densities of every marched sample,
    pruning, shading and the fused render of the kept ones), against the
    same calls made one by one through the Python entry points."""
    import bench
    import paper_2210_04847_amd as nacc
    w = synth.WORKLOADS["train_262k"]
    inp = synth.workload_inputs(w, 4096)
    t = lambda a: torch.from_numpy(a).cuda()
    grid = nacc.OccupancyGrid(w.box, w.res)
    grid.set_occupancy(t(inp["occ"]), 0.01)
    field = nacc.BlobField(inp["scene"])
    o, d = t(inp["rays_o"]), t(inp["rays_d"])
    st = bench.Step(torch, nacc, w, o, d, t(inp["targets"]), grid, field, alpha_thre=1e-2)
    st.step()
    torch.cuda.synchronize()
    packed_k, ri_k, ts_k, te_k, total_k = st.cur
    k = int(total_k.item())
    sigma_fn = lambda t0, t1, r: field.samples(o, d, r, t0, t1)[0]
    p2, ri2, ts2, te2 = nacc.ray_marching(o, d, grid, w.near, w.far, w.dt, sigma_fn=sigma_fn,
                                          early_stop_eps=w.early_stop_eps, alpha_thre=1e-2)
    torch.cuda.synchronize()
    assert k == ri2.numel() and k < int(st.total.item())
    assert_bit_exact(packed_k.cpu().numpy(), p2.cpu().numpy(), "packed_info")
    assert_bit_exact(ts_k[:k].cpu().numpy(), ts2.cpu().numpy(), "t_starts")
    assert_bit_exact(te_k[:k].cpu().numpy(), te2.cpu().numpy(), "t_ends")
    assert_bit_exact(ri_k[:k].cpu().numpy(), ri2.cpu().numpy(), "ray_indices")
    sig2, rgb2 = field.samples(o, d, ri2, ts2, te2)
    loss, color, _, _, g_sig, g_rgb = nacc.render_mse(p2, ts2, te2, sig2, rgb2, t(inp["targets"]),
                                                      early_stop_eps=w.early_stop_eps)
    torch.cuda.synchronize()
    assert torch.equal(st.color.view(torch.int32), color.view(torch.int32))
    assert torch.equal(st.g_sigmas[:k].view(torch.int32), g_sig.view(torch.int32))


@pytest.mark.parametrize("seed", range(64))
def test_prune_random_configurations(seed):
    """Random batch sizes, ray lengths, densities and both thresholds."""
    rng = np.random.default_rng(600 + seed)
    n = int(rng.choice([1, 63, 64, 65, 700, 3000]))
    mean = float(rng.choice([5, 60, 300]))
    smax = float(rng.choice([1.0, 40.0, 500.0]))
    eps = float(rng.choice([0.0, 1e-4, 1e-2]))
    thre = float(rng.choice([0.0, 1e-3, 1e-2, 0.2]))
    packed, ts, te, sg, _ = synth.ragged_render_inputs(n, 650 + seed, mean_count=mean,
                                                       max_count=int(3 * mean) + 1,
                                                       sigma_max=smax)
    check_prune(packed, ts, te, sg, eps, thre)
