"""Comparison helpers for the GPU parity tests (no GPU needed to import).

Tolerances, derived from the arithmetic:
  * marching outputs (counts, starts, ray indices, t values) are compared bit
    for bit: both sides follow the same FP32 lattice contract;
  * rendered colour, opacity, depth and weights: |gpu - oracle| <= 1e-5 |oracle|
    (+ a floor of 1e-12 absolute).  Every rendered value is a sum of
    non-negative terms, so the FP32 result is relatively accurate; the FP32
    transmittance carries a relative error of about (log2(64) + 2) u P with
    P <= -ln(1e-4) ~ 9.2 inside the kept samples, i.e. below 1e-5;
  * gradients: |gpu - oracle| <= 1e-4 (|oracle| + scale), where scale is the
    magnitude of the terms that form the gradient
    (delta (T_{i+1} |v|_i + sum_{k>i} w_k |v|_k), |v|_i the sum of the
    magnitudes of the terms of v_i = g_C . c_i + g_A + g_D m_i).  The sigma
    gradient is a difference of two such terms, and v_i a sum of terms of
    either sign (colour channels weighted by a signed loss gradient); both
    are small exactly where they cancel, and no FP32 evaluation can be
    elementwise-relative there, so relative accuracy is measured against the
    size of the terms.  On samples whose gradient keeps at least half the
    size of its terms (no cancellation) the error is also held elementwise to
    1e-4 of the value itself, and the largest such error is reported;
  * early termination: where the oracle's FP64 transmittance lies within a
    relative 1e-5 of eps at the deciding sample, FP32 may place the cut one
    sample earlier or later; such rays are accepted if they match the oracle
    evaluated with either cut.
"""
import numpy as np

import oracle

RENDER_RTOL = 1e-5
GRAD_RTOL = 1e-4
CUT_BAND = 1e-5


def bits(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.float32:
        return a.view(np.int32)
    return a


def assert_bit_exact(got, want, what):
    g, w = bits(got), bits(want)
    assert g.shape == w.shape, f"{what}: shape {g.shape} != {w.shape}"
    bad = np.flatnonzero(g.ravel() != w.ravel())
    assert bad.size == 0, (f"{what}: {bad.size} of {g.size} entries differ, first at "
                           f"{bad[:5]}: got {np.asarray(got).ravel()[bad[:5]]} want "
                           f"{np.asarray(want).ravel()[bad[:5]]}")


def ambiguous_rays(packed, t_starts, t_ends, sigmas, eps):
    """Rays whose oracle transmittance is within CUT_BAND of eps at some
    sample up to and including the cut."""
    amb = np.zeros(packed.shape[0], bool)
    if eps <= 0:
        return amb
    tau = sigmas.astype(np.float64) * (t_ends.astype(np.float64) - t_starts.astype(np.float64))
    for r in range(packed.shape[0]):
        a, n = int(packed[r, 0]), int(packed[r, 1])
        if n == 0:
            continue
        pre = np.concatenate([[0.0], np.cumsum(tau[a:a + n])[:-1]])
        trans = np.exp(-pre)
        if np.any(np.abs(trans - eps) <= CUT_BAND * eps):
            amb[r] = True
    return amb


def _close(got, want, rtol, scale=None, floor=1e-12):
    tol = rtol * (np.abs(want) + (0 if scale is None else scale)) + floor
    return np.abs(got - want) <= tol


def check_forward(got, packed, t_starts, t_ends, sigmas, rgbs, eps, weights_got=None):
    """got: dict(color [R,3], opacity [R], depth [R]) from the GPU."""
    ref = oracle.render_fwd(packed, t_starts, t_ends, sigmas, rgbs, eps)
    amb = ambiguous_rays(packed, t_starts, t_ends, sigmas, eps)
    alts = []
    if amb.any():
        alts = [oracle.render_fwd(packed, t_starts, t_ends, sigmas, rgbs, eps * (1 + f * CUT_BAND))
                for f in (-1.5, 1.5)]
    ok = np.ones(packed.shape[0], bool)
    for name in ("color", "opacity", "depth"):
        g = np.asarray(got[name], np.float64).reshape(ref[name].shape)
        c = _close(g, ref[name], RENDER_RTOL)
        c = c.reshape(packed.shape[0], -1).all(1)
        for alt in alts:
            c |= amb & _close(g, alt[name], RENDER_RTOL).reshape(packed.shape[0], -1).all(1)
        ok &= c
    bad = np.flatnonzero(~ok)
    assert bad.size == 0, (f"forward: {bad.size} rays outside tolerance, e.g. ray {bad[0]}: "
                           f"color {np.asarray(got['color']).reshape(-1, 3)[bad[0]]} vs "
                           f"{ref['color'][bad[0]]}")
    if weights_got is not None:
        ray_of = np.repeat(np.arange(packed.shape[0]), packed[:, 1])
        wc = _close(np.asarray(weights_got, np.float64), ref["weights"], RENDER_RTOL)
        for alt in alts:
            wc |= amb[ray_of] & _close(np.asarray(weights_got, np.float64), alt["weights"],
                                       RENDER_RTOL)
        assert wc.all(), f"weights: {np.count_nonzero(~wc)} samples outside tolerance"
    return ref, amb


def check_backward(g_sig, g_rgb, packed, t_starts, t_ends, sigmas, rgbs, g_color, g_opacity,
                   g_depth, eps, extra_scale=None, extra_rgb=None):
    """Compares GPU gradients with the oracle's.  extra_scale / extra_rgb are
    absolute bounds of error propagated from an input the kernel computes
    itself (the fused loss gradient, from its own FP32 colour)."""
    ref = oracle.render_bwd(packed, t_starts, t_ends, sigmas, rgbs, g_color, g_opacity, g_depth,
                            eps)
    amb = ambiguous_rays(packed, t_starts, t_ends, sigmas, eps)
    ray_of = np.repeat(np.arange(packed.shape[0]), packed[:, 1])
    alts = []
    if amb.any():
        alts = [oracle.render_bwd(packed, t_starts, t_ends, sigmas, rgbs, g_color, g_opacity,
                                  g_depth, eps * (1 + f * CUT_BAND)) for f in (-1.5, 1.5)]

    def within(r):
        # extra_scale is an absolute bound of propagated input error
        floor = 1e-20 + (0 if extra_scale is None else extra_scale)
        ok_s = _close(np.asarray(g_sig, np.float64), r["g_sigmas"], GRAD_RTOL, r["scale"], floor)
        ex = 0 if extra_rgb is None else extra_rgb
        ok_c = (np.abs(np.asarray(g_rgb, np.float64).reshape(-1, 3) - r["g_rgbs"])
                <= GRAD_RTOL * np.abs(r["g_rgbs"]) + ex + 1e-20).all(1)
        return ok_s & ok_c

    ok = within(ref)
    for alt in alts:
        ok |= amb[ray_of] & within(alt)
    bad = np.flatnonzero(~ok)
    assert bad.size == 0, (f"backward: {bad.size} samples outside tolerance, e.g. sample "
                           f"{bad[0]} (ray {ray_of[bad[0]]}): g_sigma {np.asarray(g_sig)[bad[0]]} "
                           f"vs {ref['g_sigmas'][bad[0]]} (scale {ref['scale'][bad[0]]})")
    # strict elementwise check where the gradient does not cancel: on samples
    # (of unambiguous rays) whose oracle value is at least half the size of
    # its terms, the error must stay within GRAD_RTOL of the value itself
    gs = np.asarray(g_sig, np.float64)
    floor = 1e-20 + (0 if extra_scale is None else extra_scale)
    strict = np.maximum(np.abs(gs - ref["g_sigmas"]) - floor, 0.0) / np.maximum(
        np.abs(ref["g_sigmas"]), 1e-30)
    plain = (~amb[ray_of]) & (np.abs(ref["g_sigmas"]) >= 0.5 * ref["scale"]) & (
        np.abs(ref["g_sigmas"]) > 0)
    worst = float(strict[plain].max()) if plain.any() else 0.0
    assert worst <= GRAD_RTOL, (f"backward: strict relative error {worst:.3e} on a sample whose "
                                f"gradient does not cancel")
    STRICT_REPORT.append(dict(strict_max=worst, strict_all=float(strict[~amb[ray_of]].max())
                              if (~amb[ray_of]).any() else 0.0, n_plain=int(plain.sum())))
    return ref, amb


# Largest strict elementwise relative gradient errors seen by check_backward
# (on non-cancelling samples, and on all samples), for the test reports.
STRICT_REPORT = []
