"""GPU tests of the batched form and of graph-captured steps.

The batched form marches and renders the rays of many frames, each frame with
its own occupancy grid (per-ray grid ids), in one call sequence with outputs
in capacity-sized buffers, so that no call waits on the host.  It must give
the oracle's samples bit for bit, and the same bits as one plain call
sequence per frame.  A step replayed from a HIP graph must give the bits of
the same step launched eagerly, replay after replay; the grid update inside
a graph must draw new cells at every replay.  Launch-parameter settings
(nacc_set_tuning) must leave every result bit-identical.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import assert_bit_exact, check_backward, check_forward

pytestmark = pytest.mark.gpu

N_FRAMES, RES, MEAN_RAYS = 6, 32, 300
THRESHOLD = 0.01


@pytest.fixture(scope="module")
def dyn():
    w = synth.DYNAMIC_WORKLOADS["dynamic_64"]
    inp = synth.dynamic_inputs(w, N_FRAMES, RES, MEAN_RAYS)
    return w, inp


def _nacc():
    import paper_2210_04847_amd as nacc
    return nacc


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _batched_step(w, inp, **kw):
    import bench
    nacc = _nacc()
    grid = nacc.OccupancyGrid(w.box, inp["res"], n_grids=N_FRAMES)
    grid.set_occupancy(_cuda(inp["occ"]), THRESHOLD)
    field = nacc.BlobField(inp["scene"])
    return bench.Step(torch, nacc, w, _cuda(inp["rays_o"]), _cuda(inp["rays_d"]),
                      _cuda(inp["targets"]), grid, field, grid_id=_cuda(inp["frame"]), **kw)


def _bits(t):
    t = t.detach().contiguous()
    return t.view(torch.int32) if t.dtype == torch.float32 else t


def _same(a, b):
    return a.shape == b.shape and torch.equal(_bits(a), _bits(b))


def test_batched_march_and_field_match_oracle(dyn):
    w, inp = dyn
    st = _batched_step(w, inp)
    st.march_count()
    st.march_fill()
    st.field_eval()
    torch.cuda.synchronize()
    e = int(st.total.item())
    mask = oracle.grid_threshold(inp["occ"], THRESHOLD)
    packed, ri, ts, te = oracle.march(inp["rays_o"], inp["rays_d"], mask, RES,
                                      np.asarray(w.box, np.float32), w.near, w.far, w.dt,
                                      n_grids=N_FRAMES, grid_id=inp["frame"])
    assert e == ri.size and e > 1000
    assert_bit_exact(st.packed.cpu().numpy(), packed, "packed_info")
    assert_bit_exact(st.ray_indices[:e].cpu().numpy(), ri, "ray_indices")
    assert_bit_exact(st.t_starts[:e].cpu().numpy(), ts, "t_starts")
    assert_bit_exact(st.t_ends[:e].cpu().numpy(), te, "t_ends")
    assert int(st.status.item()) == 0
    # each sample's field comes from its ray's frame
    pos = oracle.sample_positions(inp["rays_o"], inp["rays_d"], ri, ts, te)
    sig, rgb = oracle.blob_field(inp["scene"], pos, blob_set=inp["frame"][ri])
    got_s = st.sigmas[:e].cpu().numpy().astype(np.float64)
    got_c = st.rgbs[:e].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got_s - sig) <= 2e-5 * np.abs(sig) + 1e-30)
    assert np.all(np.abs(got_c - rgb) <= 1e-5 * np.abs(rgb) + 1e-12)


def test_shared_grid_march_field_and_update(dyn):
    """All frames through one grid shared over time (the maximum of the
    frames' densities, so the OR of their bits), each sample's field from its
    ray's frame; the grid update reads the field at a fixed random frame per
    drawn cell slot.  Marching bit for bit against the oracle with the OR
    mask, the field within its tolerance, the update bit for bit given the
    GPU's densities."""
    import bench
    w = synth.DYNAMIC_WORKLOADS["dynamic_64_shared"]
    inp = synth.dynamic_inputs(w, N_FRAMES, RES, MEAN_RAYS)
    occ_frames = dyn[1]["occ"].reshape(N_FRAMES, -1)
    assert_bit_exact(inp["occ"], occ_frames.max(0), "shared occupancy = max over frames")
    nacc = _nacc()
    grid = nacc.OccupancyGrid(w.box, RES)
    grid.set_occupancy(_cuda(inp["occ"]), THRESHOLD)
    field = nacc.BlobField(inp["scene"])
    upd = synth.update_frames(1 << 18, N_FRAMES, 4100 + w.seed_base)
    st = bench.Step(torch, nacc, w, _cuda(inp["rays_o"]), _cuda(inp["rays_d"]),
                    _cuda(inp["targets"]), grid, field, ray_set=_cuda(inp["frame"]),
                    update_set=_cuda(upd), seed=7)
    st.step()
    torch.cuda.synchronize()
    e = int(st.total.item())
    mask = oracle.grid_threshold(inp["occ"], THRESHOLD)
    assert_bit_exact(mask, oracle.grid_threshold(occ_frames, THRESHOLD).reshape(N_FRAMES, -1)
                     .max(0), "shared mask = OR of the frames' masks")
    packed, ri, ts, te = oracle.march(inp["rays_o"], inp["rays_d"], mask, RES,
                                      np.asarray(w.box, np.float32), w.near, w.far, w.dt)
    assert e == ri.size and e > 1000
    assert_bit_exact(st.packed.cpu().numpy(), packed, "packed_info")
    assert_bit_exact(st.ray_indices[:e].cpu().numpy(), ri, "ray_indices")
    assert_bit_exact(st.t_starts[:e].cpu().numpy(), ts, "t_starts")
    pos = oracle.sample_positions(inp["rays_o"], inp["rays_d"], ri, ts, te)
    sig = oracle.blob_field(inp["scene"], pos, blob_set=inp["frame"][ri], want_rgb=False)
    got_s = st.sigmas[:e].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got_s - sig) <= 2e-5 * np.abs(sig) + 1e-30)
    # the looser shared grid marches more samples than the per-frame grids
    per_frame = oracle.march(inp["rays_o"], inp["rays_d"],
                             oracle.grid_threshold(dyn[1]["occ"], THRESHOLD), RES,
                             np.asarray(w.box, np.float32), w.near, w.far, w.dt,
                             n_grids=N_FRAMES, grid_id=inp["frame"])[1].size
    assert e > per_frame
    # grid update: cells of the one grid, field at the slot's frame
    occ0 = inp["occ"]
    st.grid.set_occupancy(_cuda(occ0), THRESHOLD)
    st.updates.zero_()
    st.grid_update()
    torch.cuda.synchronize()
    cells, p_o = oracle.grid_sample_cells(7, 0, 1 << 18, RES, np.asarray(w.box, np.float32))
    assert_bit_exact(st.ema_cells.cpu().numpy(), cells, "cells")
    assert_bit_exact(st.ema_pos.cpu().numpy(), p_o, "positions")
    s_o = oracle.blob_field(inp["scene"], p_o, blob_set=upd, want_rgb=False)
    got = st.ema_sigma.cpu().numpy()
    assert np.all(np.abs(got - s_o) <= 2e-5 * np.abs(s_o) + 1e-30)
    want = oracle.grid_update_max(oracle.grid_decay(occ0, 0.95), cells, got)
    assert_bit_exact(st.grid.occ.cpu().numpy(), want, "occupancy after the update")


def test_batched_render_and_loss_rays_match_oracle(dyn):
    """The fused render of the batched step against the oracle on the step's
    own samples, with the loss normalised over all rays of the batch and over
    four times as many (loss_rays: the batch is a part of a larger one)."""
    w, inp = dyn
    n = inp["rays_o"].shape[0]
    for loss_rays in (0, 4 * n):
        st = _batched_step(w, inp, loss_rays=loss_rays)
        st.step()
        torch.cuda.synchronize()
        e = int(st.total.item())
        packed = st.packed.cpu().numpy()
        ts, te = st.t_starts[:e].cpu().numpy(), st.t_ends[:e].cpu().numpy()
        sg, cl = st.sigmas[:e].cpu().numpy(), st.rgbs[:e].cpu().numpy()
        eps = w.early_stop_eps
        got = dict(color=st.color.cpu().numpy(), opacity=st.opacity.cpu().numpy(),
                   depth=st.depth.cpu().numpy())
        ref, _ = check_forward(got, packed, ts, te, sg, cl, eps)
        big_l = n if loss_rays == 0 else loss_rays
        diff = ref["color"] - inp["targets"].astype(np.float64)
        want_loss = float(np.sum(diff * diff)) / (3 * big_l)
        assert abs(float(st.loss.item()) - want_loss) <= 1e-5 * want_loss
        g_color = 2.0 * diff / (3 * big_l)
        dg = 2.0 / (3 * big_l) * 1e-5 * np.abs(ref["color"]).max(1)
        prop = oracle.render_bwd(packed, ts, te, sg, cl, np.repeat(dg[:, None], 3, 1), eps=eps)
        ray_of = np.repeat(np.arange(n), packed[:, 1])
        extra_rgb = (ref["weights"] * dg[ray_of])[:, None]
        check_backward(st.g_sigmas[:e].cpu().numpy(), st.g_rgbs[:e].cpu().numpy(), packed, ts,
                       te, sg, cl, g_color, None, None, eps, extra_scale=prop["scale"],
                       extra_rgb=extra_rgb)


def test_batched_equals_plain_frames(dyn):
    """One batched step over all frames gives the bits of one plain call
    sequence per frame (its rays, a view of its grid, exactly sized outputs
    after a host read of its sample total)."""
    w, inp = dyn
    lib = _nacc()._lib
    st = _batched_step(w, inp)
    st.step()
    torch.cuda.synchronize()
    e_b = int(st.total.item())
    n_total = inp["rays_o"].shape[0]
    starts = np.concatenate([[0], np.cumsum(inp["counts"])]).astype(np.int64)
    words = RES ** 3 // 32
    desc1 = lib.grid_desc(w.box[:3], w.box[3:], RES)
    o_all, d_all, f_all = st.rays_o, st.rays_d, st.grid_id
    loss_sum = 0.0
    pieces = {k: [] for k in ("count", "ri", "ts", "te", "sig", "color", "gs", "gr")}
    for f in range(N_FRAMES):
        a, b = int(starts[f]), int(starts[f + 1])
        n = b - a
        if n == 0:
            continue
        o, d = o_all[a:b], d_all[a:b]
        bits = st.grid.bits[f * words:(f + 1) * words]
        packed = torch.empty((n, 2), dtype=torch.int32, device="cuda")
        total = torch.empty(1, dtype=torch.int64, device="cuda")
        ws = torch.empty(lib.march_workspace_size(n, desc1, st.params), dtype=torch.uint8,
                         device="cuda")
        lib.march_count(o, d, None, bits, desc1, st.params, packed, total, ws)
        e = int(total.item())
        ri = torch.empty(e, dtype=torch.int32, device="cuda")
        ts = torch.empty(e, dtype=torch.float32, device="cuda")
        te = torch.empty(e, dtype=torch.float32, device="cuda")
        lib.march_fill(o, d, None, bits, desc1, st.params, packed, ri, ts, te, None, None, ws)
        sig = torch.empty(e, dtype=torch.float32, device="cuda")
        rgb = torch.empty((e, 3), dtype=torch.float32, device="cuda")
        lib.synth_field_samples(st.field.table, st.field.n_blobs, st.field.n_sets, o, d,
                                f_all[a:b], ri, ts, te, sig, rgb)
        color = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        opac = torch.empty(n, dtype=torch.float32, device="cuda")
        dep = torch.empty(n, dtype=torch.float32, device="cuda")
        gs = torch.empty(e, dtype=torch.float32, device="cuda")
        gr = torch.empty((e, 3), dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        mws = torch.empty(lib.render_mse_workspace_size(n), dtype=torch.uint8, device="cuda")
        lib.render_fwd_bwd_mse(packed, ts, te, sig, rgb, w.early_stop_eps, st.target[a:b], color,
                               opac, dep, gs, gr, loss, mws, n_total)
        torch.cuda.synchronize()
        loss_sum += float(loss.item())
        for k, v in (("count", packed[:, 1]), ("ri", ri + a), ("ts", ts), ("te", te),
                     ("sig", sig), ("color", color), ("gs", gs), ("gr", gr)):
            pieces[k].append(v)
    cat = {k: torch.cat(v) for k, v in pieces.items()}
    assert cat["ri"].numel() == e_b
    assert _same(st.packed[:, 1], cat["count"])
    assert _same(st.ray_indices[:e_b], cat["ri"])
    assert _same(st.t_starts[:e_b], cat["ts"])
    assert _same(st.t_ends[:e_b], cat["te"])
    assert _same(st.sigmas[:e_b], cat["sig"])
    assert _same(st.color, cat["color"])
    assert _same(st.g_sigmas[:e_b], cat["gs"])
    assert _same(st.g_rgbs[:e_b], cat["gr"])
    # losses of the parts, each normalised by the whole batch, add up to the
    # batch loss (up to the order of FP32 partial sums)
    assert abs(float(st.loss.item()) - loss_sum) <= 1e-5 * loss_sum


def _snapshot(st):
    e = int(st.total.item())
    return [x.clone() for x in (st.packed, st.ray_indices[:e], st.t_starts[:e], st.t_ends[:e],
                                st.sigmas[:e], st.color, st.opacity, st.depth, st.g_sigmas[:e],
                                st.g_rgbs[:e], st.loss)]


def test_graph_replays_match_eager(dyn):
    """A step captured in a HIP graph, replayed several times with eager work
    (another eager step, unrelated torch kernels, host synchronisation)
    between the replays, gives the eager step's bits at every replay."""
    import bench
    w, inp = dyn
    st = _batched_step(w, inp)
    st.step()
    torch.cuda.synchronize()
    want = _snapshot(st)
    g = bench.capture(torch, lambda: st.step())
    scratch = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        # scribble over every output so a replay that wrote nothing fails
        for x in (st.packed, st.ray_indices, st.t_starts, st.color, st.g_sigmas, st.loss):
            x.view(torch.int32).fill_(-1) if x.dtype == torch.float32 else x.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        got = _snapshot(st)
        for k, (a, b) in enumerate(zip(got, want)):
            assert _same(a, b), f"replay {rep}: output {k} differs from the eager step"
        scratch.mul_(1.0001).add_(scratch.sum() * 1e-9)
        st.step()
        torch.cuda.synchronize()


def test_graph_grid_update_advances(dyn):
    """The grid update captured in a graph draws the cells of update k at its
    k-th replay (the update number is read on the device), and leaves the
    grid exactly as the same number of eager updates."""
    import bench
    w, inp = dyn
    lib = _nacc()._lib
    # the cell draw alone, against the oracle
    desc = lib.grid_desc(w.box[:3], w.box[3:], 64)
    step = torch.zeros(1, dtype=torch.int64, device="cuda")
    n = 100003
    cells = torch.empty(n, dtype=torch.int32, device="cuda")
    pos = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    g = bench.capture(torch, lambda: lib.grid_sample_cells(77, step, n, desc, 1, cells, pos))
    for k in (0, 1, 5):
        step.fill_(k)
        g.replay()
        torch.cuda.synchronize()
        c_o, p_o = oracle.grid_sample_cells(77, k, n, 64, np.asarray(w.box, np.float32))
        assert_bit_exact(cells.cpu().numpy(), c_o, f"cells of update {k}")
        assert_bit_exact(pos.cpu().numpy(), p_o, f"positions of update {k}")
    # whole updates: eager against graph-replayed, three in a row
    eager = _batched_step(w, inp, seed=4003)
    for _ in range(3):
        eager.grid_update()
    torch.cuda.synchronize()
    graphed = _batched_step(w, inp, seed=4003)
    g2 = bench.capture(torch, lambda: graphed.grid_update())
    # capture() ran the update once (warm-up); start again from the inputs
    graphed.grid.set_occupancy(_cuda(inp["occ"]), THRESHOLD)
    graphed.updates.zero_()
    for _ in range(3):
        g2.replay()
        torch.cuda.synchronize()
    assert int(graphed.updates.item()) == 3
    assert _same(graphed.grid.occ, eager.grid.occ)
    assert _same(graphed.grid.bits, eager.grid.bits)


@pytest.mark.parametrize("knob,values", [
    ("render_cached_chunks", (1, 2, 3, 4)),
    ("march_waves_per_group", (1, 2, 4, 8, 16)),
    ("render_mse_max_blocks", (1, 3, 1024, 8192, 1 << 20)),
    ("render_prefetch", (0, 1)),
])
def test_tuning_leaves_results_identical(dyn, knob, values):
    w, inp = dyn
    lib = _nacc()._lib
    base = lib.get_tuning()
    st = _batched_step(w, inp)
    try:
        st.step()
        torch.cuda.synchronize()
        want = _snapshot(st)
        for v in values:
            lib.set_tuning(**dict(base, **{knob: v}))
            st.step()
            torch.cuda.synchronize()
            got = _snapshot(st)
            # the loss (last) is a sum over workgroup partials: its rounding
            # may follow the workgroup count
            for k, (a, b) in enumerate(zip(got[:-1], want[:-1])):
                assert _same(a, b), f"{knob}={v}: output {k} changed"
            assert abs(float(got[-1].item()) - float(want[-1].item())) <= 1e-6 * float(
                want[-1].item())
    finally:
        lib.set_tuning(**base)


def test_autotune_keeps_outputs(dyn):
    from paper_2210_04847_amd import autotune
    w, inp = dyn
    lib = _nacc()._lib
    base = lib.get_tuning()
    st = _batched_step(w, inp)
    try:
        st.step()
        torch.cuda.synchronize()
        want = _snapshot(st)
        best, timings = autotune.autotune(lambda: st.step(), st.outputs,
                                          {"render_cached_chunks": (1, 3),
                                           "march_waves_per_group": (2,)}, repeats=2, warmup=1)
        assert lib.get_tuning() == best and len(timings) >= 2
        st.step()
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(_snapshot(st)[:-1], want[:-1])):
            assert _same(a, b), f"output {k} changed after autotuning"
    finally:
        lib.set_tuning(**base)
