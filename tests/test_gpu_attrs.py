"""GPU parity of the rendering of arbitrary per-sample attributes (Sec. 2.2),
with a constant background and an opacity threshold, against the FP64
oracle; with three channels, no background and no threshold it must give
the colour kernels' bits.

Tolerances (derived like the colour ones): an attribute channel is a signed
sum, so its error is bounded relative to the magnitude of its terms,
1e-5 (sum_i w_i |a_i| + |b| (1 - A) + |b|), the last term for the FP32
rounding of 1 - A; attribute gradients 1e-5 |w_i g|; density gradients
1e-4 of delta_i (T_{i+1} |v|_i + sum_{k>i} w_k |v|_k), where |v|_i sums
the magnitudes of the terms of v_i = g . a_i + g_opacity - g . b + g_depth
m_i (a dot product over many signed channels can cancel, and its FP32
rounding is relative to its terms).  The opacity
threshold is decided on the FP32 opacity: rays holding a sample whose
oracle opacity lies within a relative 2e-5 of the threshold, or whose
transmittance passes within 1e-5 of eps, are left out of the elementwise
comparison (and counted).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import GRAD_RTOL, assert_bit_exact

pytestmark = pytest.mark.gpu


def _nacc():
    import paper_2210_04847_amd as nacc
    return nacc


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _gpu(packed, ts, te, sg, attrs, eps, thre, bg, g_out, g_op, g_dep, attrs_t=None):
    lib = _nacc()._lib
    n, e = packed.shape[0], ts.size
    ch = attrs.shape[1]
    p, t0, t1, s = _cuda(packed), _cuda(ts), _cuda(te), _cuda(sg)
    a = _cuda(attrs) if attrs_t is None else attrs_t
    b = None if bg is None else _cuda(bg.astype(np.float32))
    out = torch.full((n, ch), 7.0, device="cuda")
    op = torch.full((n,), 7.0, device="cuda")
    dep = torch.full((n,), 7.0, device="cuda")
    wts = torch.full((max(e, 1),), 7.0, device="cuda")[:e]
    lib.render_attrs_fwd(p, t0, t1, s, a, eps, thre, b, out, op, dep, wts)
    gs = torch.full((max(e, 1),), 7.0, device="cuda")[:e]
    ga = torch.full((max(e * ch, 1),), 7.0, device="cuda")[:e * ch].view(e, ch)
    lib.render_attrs_bwd(p, t0, t1, s, a, eps, thre, b, _cuda(g_out.astype(np.float32)),
                         _cuda(g_op.astype(np.float32)), _cuda(g_dep.astype(np.float32)), gs, ga)
    torch.cuda.synchronize()
    return dict(out=out.cpu().numpy(), opacity=op.cpu().numpy(), depth=dep.cpu().numpy(),
                weights=wts.cpu().numpy(), g_sigmas=gs.cpu().numpy(), g_attrs=ga.cpu().numpy())


def _excluded_rays(packed, ts, te, sg, eps, thre):
    """Rays with a sample near the opacity threshold or the cut."""
    tau = sg.astype(np.float64) * (te.astype(np.float64) - ts.astype(np.float64))
    alpha = -np.expm1(-tau)
    near_thre = (np.abs(alpha - thre) <= 2e-5 * thre) if thre > 0 else np.zeros(ts.size, bool)
    on = alpha >= thre if thre > 0 else np.ones(ts.size, bool)
    n = packed.shape[0]
    bad = np.zeros(n, bool)
    ray_of = np.repeat(np.arange(n), packed[:, 1])
    bad[ray_of[near_thre]] = True
    if eps > 0:
        tm = np.where(on, tau, 0.0)
        for r in np.flatnonzero(packed[:, 1]):
            a, c = packed[r]
            trans = np.exp(-np.concatenate([[0.0], np.cumsum(tm[a:a + c])[:-1]]))
            bad[r] |= np.any(np.abs(trans - eps) <= 1e-5 * eps)
    return bad


def _check(packed, ts, te, sg, attrs, eps, thre, bg, seed):
    g = np.random.default_rng(seed)
    n, ch = packed.shape[0], attrs.shape[1]
    g_out = g.standard_normal((n, ch))
    g_op = g.standard_normal(n)
    g_dep = g.standard_normal(n)
    got = _gpu(packed, ts, te, sg, attrs, eps, thre, bg, g_out, g_op, g_dep)
    a64 = attrs.astype(np.float64)
    bg = None if bg is None else bg.astype(np.float32).astype(np.float64)  # what the GPU reads
    want = oracle.render_attrs_fwd(packed, ts, te, sg, a64, eps, thre, bg)
    grad = oracle.render_attrs_bwd(packed, ts, te, sg, a64, g_out.astype(np.float32),
                                   g_op.astype(np.float32), g_dep.astype(np.float32), eps, thre, bg)
    skip = _excluded_rays(packed, ts, te, sg, eps, thre)
    ok = ~skip
    ray_of = np.repeat(np.arange(n), packed[:, 1])
    oks = ok[ray_of]
    w = want["weights"]
    terms = np.zeros((n, ch))
    np.add.at(terms, ray_of, w[:, None] * np.abs(a64))
    b = np.zeros(ch) if bg is None else np.abs(bg.astype(np.float64))
    tol = 1e-5 * (terms + b[None] * (1 - want["opacity"][:, None]) + b[None]) + 1e-12
    err = np.abs(got["out"] - want["out"])
    assert np.all(err[ok] <= tol[ok]), f"out: worst {np.max(err[ok] / tol[ok])} x tolerance"
    for name in ("opacity", "depth"):
        e_ = np.abs(got[name] - want[name])
        assert np.all(e_[ok] <= 1e-5 * np.abs(want[name][ok]) + 1e-12), name
    assert np.all(np.abs(got["weights"][oks] - w[oks]) <= 1e-5 * w[oks] + 1e-12), "weights"
    # gradients
    gw = np.abs(w[:, None] * g_out.astype(np.float32)[ray_of])
    ea = np.abs(got["g_attrs"] - grad["g_attrs"])
    assert np.all(ea[oks] <= 1e-5 * gw[oks] + 1e-12), "g_attrs"
    # the magnitude of the terms of v: the oracle's scale with every term
    # of v made non-negative
    g_abs_op = np.abs(g_op.astype(np.float32)).astype(np.float64)
    if bg is not None:
        g_abs_op = g_abs_op + np.abs(g_out.astype(np.float32)) @ np.abs(bg)
    scale = oracle.render_attrs_bwd(packed, ts, te, sg, np.abs(a64),
                                    np.abs(g_out.astype(np.float32)), g_abs_op,
                                    np.abs(g_dep.astype(np.float32)), eps, thre)["scale"]
    es = np.abs(got["g_sigmas"] - grad["g_sigmas"])
    tol_s = GRAD_RTOL * (np.abs(grad["g_sigmas"]) + scale) + 1e-12
    assert np.all(es[oks] <= tol_s[oks]), f"g_sigmas: worst {np.max(es[oks] / tol_s[oks])}"
    if thre > 0:
        alpha = -np.expm1(-sg.astype(np.float64) * (te.astype(np.float64) - ts.astype(np.float64)))
        low = (alpha < thre * (1 - 2e-5)) & oks
        assert np.all(got["weights"][low] == 0) and np.all(got["g_sigmas"][low] == 0)
    return skip


@pytest.mark.parametrize("ch,thre,with_bg,eps", [(1, 0.0, False, 1e-4), (5, 0.05, True, 1e-4),
                                                 (16, 0.0, True, 0.0), (20, 0.02, True, 1e-4),
                                                 (64, 0.05, False, 1e-4), (3, 0.05, True, 1e-2)])
def test_attrs_match_oracle(ch, thre, with_bg, eps):
    packed, ts, te, sg, _ = synth.ragged_render_inputs(1500, 31 + ch, mean_count=70, max_count=400,
                                                       sigma_max=30.0)
    rng = np.random.default_rng(ch)
    attrs = rng.standard_normal((ts.size, ch)).astype(np.float32)
    bg = rng.standard_normal(ch) if with_bg else None
    skip = _check(packed, ts, te, sg, attrs, eps, thre, bg, 100 + ch)
    assert skip.mean() < 0.02


def test_attrs_three_channels_equal_colour_kernels():
    """n_ch = 3, no background, no threshold: the colour kernels' bits."""
    lib = _nacc()._lib
    packed, ts, te, sg, cl = synth.ragged_render_inputs(2000, 41, mean_count=90, max_count=700)
    n, e = packed.shape[0], ts.size
    g = np.random.default_rng(41)
    gc, go, gd = (g.standard_normal((n, 3)).astype(np.float32), g.standard_normal(n).astype(np.float32),
                  g.standard_normal(n).astype(np.float32))
    for eps in (1e-4, 0.0):
        got = _gpu(packed, ts, te, sg, cl, eps, 0.0, None, gc, go, gd)
        p, t0, t1, s, c = _cuda(packed), _cuda(ts), _cuda(te), _cuda(sg), _cuda(cl)
        color = torch.empty((n, 3), device="cuda")
        op = torch.empty(n, device="cuda")
        dep = torch.empty(n, device="cuda")
        wts = torch.empty(e, device="cuda")
        lib.render_fwd(p, t0, t1, s, c, eps, color, op, dep, wts)
        g_s = torch.empty(e, device="cuda")
        g_c = torch.empty((e, 3), device="cuda")
        lib.render_bwd(p, t0, t1, s, c, eps, _cuda(gc), _cuda(go), _cuda(gd), g_s, g_c)
        torch.cuda.synchronize()
        assert_bit_exact(got["out"], color.cpu().numpy(), "colour")
        assert_bit_exact(got["opacity"], op.cpu().numpy(), "opacity")
        assert_bit_exact(got["depth"], dep.cpu().numpy(), "depth")
        assert_bit_exact(got["weights"], wts.cpu().numpy(), "weights")
        assert_bit_exact(got["g_sigmas"], g_s.cpu().numpy(), "g_sigmas")
        assert_bit_exact(got["g_attrs"], g_c.cpu().numpy(), "g_rgbs")


@pytest.mark.parametrize("ch", [4, 8, 12, 16, 32, 48])
def test_attrs_unaligned_rows_and_empty_rays(ch):
    """Rows that are not 16-byte aligned take the per-lane scalar path and
    give the aligned path's bits (4, 8 and multiples of 16 channels: rows
    staged through LDS; 12: per-lane float4 rows); empty rays render the
    background."""
    packed, ts, te, sg, _ = synth.ragged_render_inputs(500, 43, mean_count=40, max_count=200,
                                                       empty_frac=0.3)
    attrs = np.random.default_rng(43).standard_normal((ts.size, ch)).astype(np.float32)
    bg = np.linspace(-1, 1, ch)
    g = np.random.default_rng(44)
    args = (g.standard_normal((500, ch)), g.standard_normal(500), g.standard_normal(500))
    aligned = _gpu(packed, ts, te, sg, attrs, 1e-4, 0.02, bg, *args)
    big = torch.zeros(attrs.size + 1, device="cuda")
    big[1:] = _cuda(attrs.ravel())
    shifted = big[1:].view(ts.size, ch)  # 4-byte offset
    assert shifted.data_ptr() % 16 != 0
    unaligned = _gpu(packed, ts, te, sg, attrs, 1e-4, 0.02, bg, *args, attrs_t=shifted)
    for k in aligned:
        assert_bit_exact(unaligned[k], aligned[k], k)
    empty = packed[:, 1] == 0
    assert empty.sum() > 50
    assert_bit_exact(aligned["out"][empty], np.tile(bg.astype(np.float32), (empty.sum(), 1)),
                     "background of empty rays")


def test_attrs_autograd():
    """render_attrs under torch.autograd gives the backward call's
    gradients."""
    nacc = _nacc()
    packed, ts, te, sg, _ = synth.ragged_render_inputs(300, 45, mean_count=50, max_count=300)
    ch = 12
    attrs = np.random.default_rng(45).standard_normal((ts.size, ch)).astype(np.float32)
    bg = np.random.default_rng(46).standard_normal(ch)
    s_t = _cuda(sg).requires_grad_(True)
    a_t = _cuda(attrs).requires_grad_(True)
    out, op, dep = nacc.render_attrs(_cuda(packed), _cuda(ts), _cuda(te), s_t, a_t,
                                     early_stop_eps=1e-4, alpha_thre=0.01, background=bg)
    g = np.random.default_rng(47)
    g_out = g.standard_normal((300, ch)).astype(np.float32)
    g_op = g.standard_normal(300).astype(np.float32)
    loss = (out * _cuda(g_out)).sum() + (op.reshape(-1) * _cuda(g_op)).sum()
    loss.backward()
    got = _gpu(packed, ts, te, sg, attrs, 1e-4, 0.01, bg, g_out, g_op, np.zeros(300, np.float32))
    assert_bit_exact(out.detach().cpu().numpy(), got["out"], "out")
    assert_bit_exact(s_t.grad.cpu().numpy(), got["g_sigmas"], "g_sigmas")
    assert_bit_exact(a_t.grad.cpu().numpy(), got["g_attrs"], "g_attrs")


@pytest.mark.parametrize("seed", range(64))
def test_attrs_random_configurations(seed):
    """Random channel counts (staged and per-lane widths), batch sizes, ray
    lengths, thresholds, cuts and backgrounds against the oracle."""
    rng = np.random.default_rng(300 + seed)
    ch = int(rng.choice([1, 2, 4, 7, 8, 12, 16, 32]))
    n = int(rng.choice([3, 64, 65, 600]))
    mean = float(rng.choice([10, 70, 200]))
    thre = float(rng.choice([0.0, 0.02]))
    eps = float(rng.choice([0.0, 1e-4]))
    packed, ts, te, sg, _ = synth.ragged_render_inputs(n, 350 + seed, mean_count=mean,
                                                       max_count=int(3 * mean) + 1,
                                                       sigma_max=float(rng.choice([5.0, 40.0])))
    attrs = rng.standard_normal((ts.size, ch)).astype(np.float32)
    bg = rng.standard_normal(ch) if rng.random() < 0.5 else None
    skip = _check(packed, ts, te, sg, attrs, eps, thre, bg, 400 + seed)
    # at most 5% of the rays (or one ray, for batches of a few rays) may be
    # set aside as undecidable at the threshold or the cut
    assert skip.sum() <= max(1.0, 0.05 * skip.size)
