"""GPU tests of step plans (include/nacc_plan.h).

A plan runs the same launches as the individual calls, so its outputs must
be the calls' bits: eagerly, and replayed from the library's own HIP graphs
(with eager work between the replays); its grid update must leave the grid
exactly as the same number of update call sequences; its tuner must leave
every compared output unchanged; a sample buffer that is too small must be
reported, not overrun; a failing stage must end the step with its error.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

N_FRAMES, RES, MEAN_RAYS = 6, 32, 300
THRESHOLD = 0.01


@pytest.fixture(scope="module")
def dyn():
    w = synth.DYNAMIC_WORKLOADS["dynamic_64"]
    inp = synth.dynamic_inputs(w, N_FRAMES, RES, MEAN_RAYS)
    return w, inp


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _step(w, inp, **kw):
    import bench
    import paper_2210_04847_amd as nacc
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


def _snapshot(st, loss=True):
    e = int(st.total.item())
    out = [st.packed, st.ray_indices[:e], st.t_starts[:e], st.t_ends[:e], st.sigmas[:e],
           st.rgbs[:e], st.color, st.opacity, st.depth]
    if not st.forward_only:
        out += [st.g_sigmas[:e], st.g_rgbs[:e]] + ([st.loss] if loss else [])
    return [x.clone() for x in out]


def _scribble(st):
    for x in (st.packed, st.ray_indices, st.t_starts, st.t_ends, st.sigmas, st.rgbs, st.color,
              st.opacity, st.depth, st.g_sigmas, st.g_rgbs, st.loss):
        x.view(torch.int32).fill_(-1) if x.dtype == torch.float32 else x.fill_(-1)


def _check(got, want, what):
    assert len(got) == len(want)
    for k, (a, b) in enumerate(zip(got, want)):
        assert _same(a, b), f"{what}: output {k} differs from the individual calls"


@pytest.mark.parametrize("forward_only", [False, True])
def test_plan_step_and_replays_equal_the_calls(dyn, forward_only):
    w, inp = dyn
    st = _step(w, inp, forward_only=forward_only)
    st.step()
    torch.cuda.synchronize()
    want = _snapshot(st)
    plan = st.plan()
    try:
        _scribble(st)
        plan.step()
        torch.cuda.synchronize()
        _check(_snapshot(st), want, "eager plan step")
        plan.capture()
        scratch = torch.randn(1 << 20, device="cuda")
        for rep in range(4):
            _scribble(st)
            plan.launch()
            torch.cuda.synchronize()
            _check(_snapshot(st), want, f"replay {rep}")
            scratch.mul_(1.0001).add_(scratch.sum() * 1e-9)
            st.step()  # eager calls on the same buffers between replays
            torch.cuda.synchronize()
        # a replay on a side stream, ordered after the default stream's work
        side = torch.cuda.Stream()
        _scribble(st)
        side.wait_stream(torch.cuda.current_stream())
        plan.launch(stream=side)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        _check(_snapshot(st), want, "replay on a side stream")
    finally:
        plan.close()


def test_plan_update_equals_the_calls(dyn):
    """Eager and replayed plan updates draw the cells of update 0, 1, 2, ...
    (the counter on the device) and leave occ, bits and the skip field as
    the individual update calls do."""
    w, inp = dyn
    eager = _step(w, inp, seed=4003, skip_field=True)
    for _ in range(3):
        eager.grid_update()
    eager.step()
    torch.cuda.synchronize()
    want = _snapshot(eager)
    st = _step(w, inp, seed=4003, skip_field=True)
    plan = st.plan()
    try:
        plan.update()
        plan.capture()  # captures, does not run
        torch.cuda.synchronize()
        assert int(st.updates.item()) == 1
        plan.launch(with_update=True)
        plan.launch(with_update=True)
        plan.launch()
        torch.cuda.synchronize()
        assert int(st.updates.item()) == 3
        assert _same(st.grid.occ, eager.grid.occ)
        assert _same(st.grid.bits, eager.grid.bits)
        assert _same(st.grid.skip, eager.grid.skip)
        _check(_snapshot(st), want, "step after three updates")
    finally:
        plan.close()


def test_plan_autotune_keeps_outputs(dyn):
    w, inp = dyn
    import paper_2210_04847_amd as nacc
    lib = nacc._lib
    base = lib.get_tuning()
    st = _step(w, inp)
    st.step()
    torch.cuda.synchronize()
    want = _snapshot(st, loss=False)
    want_loss = float(st.loss.item())
    plan = st.plan()
    try:
        plan.capture()
        best, ms = plan.autotune(repeats=2)
        assert ms > 0 and lib.get_tuning() == best
        _scribble(st)
        plan.launch()  # re-captured under the chosen setting
        torch.cuda.synchronize()
        _check(_snapshot(st, loss=False), want, "after autotune")
        # the loss is a sum over workgroup partials: its rounding may follow
        # the workgroup count
        assert abs(float(st.loss.item()) - want_loss) <= 1e-6 * want_loss
    finally:
        plan.close()
        lib.set_tuning(**base)


def test_plan_capacity_overflow_is_reported(dyn):
    """With room for fewer samples than a step marches, the plan reports
    NACC_ECAPACITY in status, writes only what fits, and renders every ray
    whose samples all fit exactly as with room for all of them."""
    import paper_2210_04847_amd as nacc
    w, inp = dyn
    full = _step(w, inp)
    full.step()
    torch.cuda.synchronize()
    e = int(full.total.item())
    packed = full.packed.clone()
    small = _step(w, inp)
    cap = e // 2
    lib = nacc._lib
    f, g = small.field, small.grid
    ri = torch.empty(cap, dtype=torch.int32, device="cuda")
    ts = torch.empty(cap, dtype=torch.float32, device="cuda")
    te = torch.empty(cap, dtype=torch.float32, device="cuda")
    sig = torch.empty(cap, dtype=torch.float32, device="cuda")
    rgb = torch.empty((cap, 3), dtype=torch.float32, device="cuda")
    gs = torch.empty(cap, dtype=torch.float32, device="cuda")
    gr = torch.empty((cap, 3), dtype=torch.float32, device="cuda")
    field = lib.synth_samples_stage(f.table, f.n_blobs, f.n_sets, small.rays_o, small.rays_d,
                                    small.ray_set, ri, ts, te, sig, rgb, small.total)
    plan = lib.Plan(small.rays_o, small.rays_d, g.bits, g.desc, small.params, small.packed, ri,
                    ts, te, small.total, field, sig, rgb, small.color, small.opacity, small.depth,
                    early_stop_eps=w.early_stop_eps, grid_id=small.grid_id, status=small.status,
                    target=small.target, g_sigmas=gs, g_rgbs=gr, loss=small.loss)
    try:
        plan.step()
        torch.cuda.synchronize()
        assert int(small.status.item()) == lib.NACC_ECAPACITY
        assert int(small.total.item()) == e and torch.equal(small.packed, packed)
        assert _same(ri, full.ray_indices[:cap]) and _same(ts, full.t_starts[:cap])
        fits = (packed[:, 0] + packed[:, 1]) <= cap
        assert int(fits.sum()) > 0
        assert _same(small.color[fits], full.color[fits])
        end = int((packed[:, 0] + packed[:, 1])[fits].max())
        assert _same(gs[:end], full.g_sigmas[:end])
        assert not bool(torch.isnan(small.color).any())
    finally:
        plan.close()


def test_python_stage_and_its_errors(dyn):
    """A Python callable as the field stage: eager and captured steps give the
    native stage's bits; an exception inside the stage ends the step and is
    raised by the plan call."""
    import paper_2210_04847_amd as nacc
    lib = nacc._lib
    w, inp = dyn
    st = _step(w, inp)
    st.step()
    torch.cuda.synchronize()
    want = _snapshot(st)
    f = st.field

    def field_fn(stream):
        lib.synth_field_samples(f.table, f.n_blobs, f.n_sets, st.rays_o, st.rays_d, st.ray_set,
                                st.ray_indices, st.t_starts, st.t_ends, st.sigmas, st.rgbs,
                                st.total, stream=stream)

    g = st.grid
    plan = lib.Plan(st.rays_o, st.rays_d, g.bits, g.desc, st.params, st.packed, st.ray_indices,
                    st.t_starts, st.t_ends, st.total, lib.python_stage(field_fn), st.sigmas,
                    st.rgbs, st.color, st.opacity, st.depth, early_stop_eps=w.early_stop_eps,
                    grid_id=st.grid_id, status=st.status, target=st.target, g_sigmas=st.g_sigmas,
                    g_rgbs=st.g_rgbs, loss=st.loss)
    try:
        _scribble(st)
        plan.step()
        torch.cuda.synchronize()
        _check(_snapshot(st), want, "python stage, eager")
        plan.capture()
        _scribble(st)
        plan.launch()
        torch.cuda.synchronize()
        _check(_snapshot(st), want, "python stage, replayed")
    finally:
        plan.close()

    class Boom(RuntimeError):
        pass

    def failing(stream):
        raise Boom("field failed")

    bad = lib.Plan(st.rays_o, st.rays_d, g.bits, g.desc, st.params, st.packed, st.ray_indices,
                   st.t_starts, st.t_ends, st.total, lib.python_stage(failing), st.sigmas,
                   st.rgbs, st.color, st.opacity, st.depth, grid_id=st.grid_id)
    try:
        with pytest.raises(Boom):
            bad.step()
        with pytest.raises(Boom):
            bad.capture()
        with pytest.raises(lib.NaccError):
            bad.launch()  # nothing was captured
        with pytest.raises(lib.NaccError):
            bad.update()  # the plan has no update
    finally:
        torch.cuda.synchronize()
        bad.close()


@pytest.mark.parametrize("name", ["unbounded_262k", "unbounded_contract_262k"])
def test_plan_unbounded_equals_the_calls(name):
    """Cone steps through cascades and through the contraction lookup, with
    the skip field: the plan's eager step, replays and update give the bits
    of the individual calls."""
    from steps import make_step
    _, _, st = make_step(name, n_rays=3000, res=32, skip_field=True)
    st.step(update=True)
    st.step()
    torch.cuda.synchronize()
    want = _snapshot(st)
    grid_bits = st.grid.bits.clone()
    _, _, other = make_step(name, n_rays=3000, res=32, skip_field=True)
    plan = other.plan()
    try:
        plan.capture()
        plan.launch(with_update=True)
        _scribble(other)
        plan.launch()
        torch.cuda.synchronize()
        assert _same(other.grid.bits, grid_bits)
        _check(_snapshot(other), want, f"{name}: replays")
        _scribble(other)
        plan.step()
        torch.cuda.synchronize()
        _check(_snapshot(other), want, f"{name}: eager plan step")
    finally:
        plan.close()


def test_after_stage_runs_last(dyn):
    """The optional after-stage runs after rendering, on the step's stream,
    eagerly and in the captured graph: here it copies the gradients out."""
    import paper_2210_04847_amd as nacc
    lib = nacc._lib
    w, inp = dyn
    st = _step(w, inp)
    st.step()
    torch.cuda.synchronize()
    e = int(st.total.item())
    want = st.g_sigmas[:e].clone()
    copied = torch.full_like(st.g_sigmas, -1.0)

    def after(stream):
        torch.mul(st.g_sigmas, 1.0, out=copied)  # an elementwise kernel, no allocation

    f, g = st.field, st.grid
    field = lib.synth_samples_stage(f.table, f.n_blobs, f.n_sets, st.rays_o, st.rays_d, st.ray_set,
                                    st.ray_indices, st.t_starts, st.t_ends, st.sigmas, st.rgbs,
                                    st.total)
    plan = lib.Plan(st.rays_o, st.rays_d, g.bits, g.desc, st.params, st.packed, st.ray_indices,
                    st.t_starts, st.t_ends, st.total, field, st.sigmas, st.rgbs, st.color,
                    st.opacity, st.depth, early_stop_eps=w.early_stop_eps, grid_id=st.grid_id,
                    status=st.status, target=st.target, g_sigmas=st.g_sigmas, g_rgbs=st.g_rgbs,
                    loss=st.loss, after=lib.python_stage(after))
    try:
        plan.step()
        torch.cuda.synchronize()
        assert _same(copied[:e], want)
        plan.capture()
        for _ in range(2):
            copied.fill_(-1.0)
            st.g_sigmas.fill_(7.0)
            plan.launch()
            torch.cuda.synchronize()
            assert _same(copied[:e], want) and _same(st.g_sigmas[:e], want)
    finally:
        plan.close()
