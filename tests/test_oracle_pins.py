"""Pins of the oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself or retypes its formulae: each
checks a closed form, an invariant, an exact geometric property, a library
routine, or finite differences, chosen so that a dropped term, a wrong sign
or index, or a transposed operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import synth

BOX = np.array([-1.5, -1.5, -1.5, 1.5, 1.5, 1.5], np.float32)


def _rays(n, seed):
    return synth.rays_toward_origin(n, seed)


# ---------------------------------------------------------------------------
# Clip (Sec. 2.1: rays are clipped to the scene box before marching)
# ---------------------------------------------------------------------------

def test_clip_axis_aligned_closed_form():
    # A ray along each axis, both directions, from outside the box: the
    # entry and exit are the two faces, at distances |o_i| -/+ 1.5.
    for axis in range(3):
        for sgn in (1.0, -1.0):
            o = np.zeros((1, 3), np.float32)
            d = np.zeros((1, 3), np.float32)
            o[0, axis] = -sgn * 4.0
            o[0, (axis + 1) % 3] = 0.25
            d[0, axis] = sgn
            tn, tf, hit = oracle.clip(o, d, BOX, 0.0, 1e10)
            assert hit[0]
            assert tn[0] == np.float32(2.5) and tf[0] == np.float32(5.5)


def test_clip_geometry_random_rays():
    # Entry and exit points lie on the box surface; points strictly between
    # lie inside; misses never come within the box.
    g = np.random.default_rng(5)
    o = g.uniform(-4, 4, (4000, 3)).astype(np.float32)
    d = g.standard_normal((4000, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    tn, tf, hit = oracle.clip(o, d, BOX, 0.0, 1e10)
    o64, d64 = o.astype(np.float64), d.astype(np.float64)
    for t, name in ((tn, "entry"), (tf, "exit")):
        p = o64[hit] + d64[hit] * t[hit, None].astype(np.float64)
        inside_start = (np.abs(o64[hit]) <= 1.5).all(1) & (name == "entry")
        on_face = np.abs(np.abs(p).max(1) - 1.5) < 1e-5
        assert np.all(on_face | inside_start)
    mid = o64[hit] + d64[hit] * (0.5 * (tn[hit] + tf[hit]))[:, None]
    assert np.all(np.abs(mid) <= 1.5 + 1e-5)
    # brute force for the misses: dense points along the ray stay outside
    ts = np.linspace(0, 12, 4001)
    pts = o64[~hit, None, :] + d64[~hit, None, :] * ts[None, :, None]
    assert not np.any((np.abs(pts) < 1.5 - 1e-4).all(-1))
    # an origin inside the box starts at near = 0
    tn2, tf2, hit2 = oracle.clip(np.zeros((1, 3), np.float32),
                                 np.array([[1, 0, 0]], np.float32), BOX, 0.0, 1e10)
    assert hit2[0] and tn2[0] == 0.0 and tf2[0] == np.float32(1.5)


def test_clip_zero_direction_component():
    o = np.array([[0.2, -4.0, 0.1], [2.0, -4.0, 0.0]], np.float32)
    d = np.array([[0.0, 1.0, 0.0], [0.0, 1.0, 0.0]], np.float32)
    tn, tf, hit = oracle.clip(o, d, BOX, 0.0, 1e10)
    assert hit[0] and tn[0] == np.float32(2.5) and tf[0] == np.float32(5.5)
    assert not hit[1]  # x = 2 lies outside the slab, direction parallel


# ---------------------------------------------------------------------------
# Marching (Sec. 2.1: keep only samples in occupied cells)
# ---------------------------------------------------------------------------

def test_empty_grid_gives_no_samples():
    o, d = _rays(500, 1)
    mask = np.zeros(32 ** 3, np.uint8)
    packed, ri, ts, te = oracle.march(o, d, mask, 32, BOX, 0.0, 1e10,
                                      synth.STEP_1024)
    assert ri.size == 0 and np.all(packed[:, 1] == 0)


def test_full_grid_count_closed_form():
    # With every cell occupied, ray r gets every lattice candidate:
    # ceil((t_far - t_near) / dt) of them.
    o, d = _rays(3000, 2)
    mask = np.ones(16 ** 3, np.uint8)
    dt = synth.STEP_1024
    packed, ri, ts, te = oracle.march(o, d, mask, 16, BOX, 0.0, 1e10, dt)
    tn, tf, hit = oracle.clip(o, d, BOX, 0.0, 1e10)
    q = (tf.astype(np.float64) - tn.astype(np.float64)) / np.float64(np.float32(dt))
    expect = np.where(hit, np.ceil(q), 0)
    clear = np.abs(q - np.round(q)) > 1e-3
    assert clear.mean() > 0.99
    assert np.array_equal(packed[clear, 1], expect[clear].astype(np.int32))
    assert np.all(np.abs(packed[~clear, 1] - expect[~clear]) <= 1)
    # consecutive samples of a ray share endpoints bit for bit
    same_ray = ri[1:] == ri[:-1]
    assert np.array_equal(te[:-1][same_ray], ts[1:][same_ray])
    assert np.all(ts[1:][same_ray] > ts[:-1][same_ray])
    # the first sample starts at the clip entry
    first = packed[packed[:, 1] > 0, 0]
    assert np.array_equal(ts[first], tn[packed[:, 1] > 0])
    # ray_indices are the rays repeated by their counts
    assert np.array_equal(ri, np.repeat(np.arange(o.shape[0]), packed[:, 1]))


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sgn", [1.0, -1.0])
def test_single_cell_axis_rays(axis, sgn):
    # One occupied cell at an asymmetric index; a ray along `axis` through
    # its column must emit exactly the candidates whose midpoint lies inside
    # that cell's extent along the axis.  A ray through the transposed column
    # emits nothing (catches axis-order mistakes).
    res = 8
    h = 3.0 / res
    idx = [5, 2, 6]
    mask = np.zeros((res, res, res), np.uint8)
    mask[idx[0], idx[1], idx[2]] = 1
    dt = 0.02
    o = np.zeros((2, 3), np.float32)
    d = np.zeros((2, 3), np.float32)
    for r, col in enumerate((idx, idx[::-1])):
        for i in range(3):
            if i != axis:
                o[r, i] = -1.5 + (col[i] + 0.37) * h
        o[r, axis] = -sgn * 3.0
        d[r, axis] = sgn
    packed, ri, ts, te = oracle.march(o, d, mask.ravel(), res, BOX, 0.0, 1e10, dt)
    tn, tf, hit = oracle.clip(o, d, BOX, 0.0, 1e10)
    # exact geometry in FP64: midpoint coordinate along the axis
    k = np.arange(int((tf[0] - tn[0]) / dt) + 2)
    mids = o[0, axis] + sgn * (tn[0] + (k + 0.5) * dt)
    lo_face = -1.5 + idx[axis] * h
    inside = (mids >= lo_face) & (mids < lo_face + h)
    near_face = (np.abs(mids - lo_face) < 1e-5) | (np.abs(mids - lo_face - h) < 1e-5)
    got = np.zeros_like(inside)
    kk = np.round((ts[ri == 0] - tn[0]) / dt).astype(int)
    got[kk] = True
    assert np.array_equal(got[~near_face], inside[~near_face])
    assert 18 <= inside.sum() <= 19
    if idx[::-1] != idx:
        assert packed[1, 1] == 0


def test_dense_mask_sampling_tiny_grids():
    # Marching equals dense sampling of the ray at the lattice midpoints with
    # an exact FP64 cell test, except for midpoints within 1e-5 of a face.
    for res, seed in ((4, 11), (8, 12), (16, 13)):
        mask = synth.random_mask(res ** 3, 0.35, seed)
        o, d = _rays(300, seed)
        dt = 0.013
        packed, ri, ts, te = oracle.march(o, d, mask, res, BOX, 0.0, 1e10, dt)
        tn, tf, hit = oracle.clip(o, d, BOX, 0.0, 1e10)
        m3 = mask.reshape(res, res, res)
        for r in range(o.shape[0]):
            if not hit[r]:
                assert packed[r, 1] == 0
                continue
            n_cand = int(np.ceil((float(tf[r]) - float(tn[r])) / dt)) + 1
            k = np.arange(n_cand)
            tm = float(tn[r]) + (k + 0.5) * dt
            valid = float(tn[r]) + k * dt < float(tf[r])
            x = o[r].astype(np.float64) + d[r].astype(np.float64) * tm[:, None]
            u = (x + 1.5) * res / 3.0
            amb = (np.abs(u - np.round(u)) < 1e-4).any(1)
            # also ambiguous: candidates at the far end of the lattice
            amb |= np.abs(float(tn[r]) + k * dt - float(tf[r])) < 1e-5
            j = np.clip(np.floor(u), 0, res - 1).astype(int)
            occ = m3[j[:, 0], j[:, 1], j[:, 2]].astype(bool) & valid
            sel = ri == r
            got = np.zeros(n_cand, bool)
            kk = np.round((ts[sel].astype(np.float64) - float(tn[r])) / dt).astype(int)
            got[kk] = True
            assert np.array_equal(got[~amb], occ[~amb]), (res, r)


def test_per_ray_grid_selection():
    # Two grids behind one call: grid 0 empty, grid 1 full.  A ray naming
    # grid 1 must get every lattice candidate, ceil((t_far - t_near)/dt) of
    # them; a ray naming grid 0 none; a ray naming a grid that does not exist
    # (-1 or 2) none.  Ignoring grid_id (always grid 0) or reading the wrong
    # grid's slice of the mask fails this.
    res = 8
    o, d = _rays(400, 21)
    dt = synth.STEP_1024
    mask = np.concatenate([np.zeros(res ** 3, np.uint8), np.ones(res ** 3, np.uint8)])
    gid = np.resize(np.array([1, 0, 1, -1, 2, 1], np.int32), o.shape[0])
    packed, ri, ts, te = oracle.march(o, d, mask, res, BOX, 0.0, 1e10, dt,
                                      n_grids=2, grid_id=gid)
    tn, tf, hit = oracle.clip(o, d, BOX, 0.0, 1e10)
    q = (tf.astype(np.float64) - tn.astype(np.float64)) / np.float64(np.float32(dt))
    full = np.where(hit, np.ceil(q), 0)
    clear = np.abs(q - np.round(q)) > 1e-3
    on1 = gid == 1
    assert on1.sum() > 100 and (on1 & hit).sum() > 50
    assert np.all(packed[~on1, 1] == 0)
    assert np.array_equal(packed[on1 & clear, 1], full[on1 & clear].astype(np.int32))
    assert np.all(np.abs(packed[on1 & ~clear, 1] - full[on1 & ~clear]) <= 1)
    assert np.array_equal(ri, np.repeat(np.arange(o.shape[0]), packed[:, 1]))


@pytest.mark.parametrize("lookup", [0, 2])
def test_per_ray_grids_equal_separate_calls(lookup):
    # Rays over three different random grids in one call equal, ray by ray
    # and bit for bit, one single-grid call per grid on that grid alone.
    res = 8
    o, d = _rays(300, 22)
    box = BOX if lookup == 0 else np.array([-2, -2, -2, 2, 2, 2], np.float32)
    far = 1e10 if lookup == 0 else 6.0
    masks = [synth.random_mask(res ** 3, f, 30 + i) for i, f in enumerate((0.2, 0.5, 0.8))]
    gid = np.random.default_rng(23).integers(0, 3, o.shape[0]).astype(np.int32)
    packed, ri, ts, te = oracle.march(o, d, np.concatenate(masks), res, box, 0.0,
                                      far, 0.02, lookup=lookup, n_grids=3, grid_id=gid)
    for g in range(3):
        sel = np.flatnonzero(gid == g)
        p1, r1, s1, e1 = oracle.march(o[sel], d[sel], masks[g], res, box, 0.0,
                                      far, 0.02, lookup=lookup)
        assert np.array_equal(packed[sel, 1], p1[:, 1]), g
        for j, r in enumerate(sel):
            a, n = packed[r]
            b, m = p1[j]
            assert np.array_equal(ts[a:a + n], s1[b:b + m])
            assert np.array_equal(te[a:a + n], e1[b:b + m])
    # distinct grids really give distinct samples (the test can fail)
    assert len({int(packed[gid == g, 1].sum()) for g in range(3)}) == 3


def _round_f32(q):
    """Round an exact rational to the nearest float32 (ties to even)."""
    from fractions import Fraction
    if q == 0:
        return np.float32(0.0)
    sign = -1 if q < 0 else 1
    q = abs(Fraction(q))
    e = math.floor(math.log2(q.numerator) - math.log2(q.denominator))
    while Fraction(2) ** e > q:
        e -= 1
    while Fraction(2) ** (e + 1) <= q:
        e += 1
    ulp = Fraction(2) ** (e - 23)
    m = q / ulp
    lo = math.floor(m)
    rem = m - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    return np.float32(sign * float(lo * ulp))


def test_lattice_is_two_roundings_not_fma():
    # The lattice point t_k is fl(t_near + fl(k * dt)): the product is
    # rounded to FP32 before the sum.  Evaluated here by exact rational
    # arithmetic; on the candidates where that differs from the singly
    # rounded fl(t_near + k * dt) (a fused multiply-add) the oracle must give
    # the two-rounding value.
    from fractions import Fraction
    dt = np.float32(synth.STEP_1024)
    res = 4
    mask = np.ones(res ** 3, np.uint8)
    n_diff = 0
    for a in (0.123456789, 0.7071067, 1.1, 2.3456):
        o = np.array([[-1.5 - a, 0.1, 0.2]], np.float32)
        d = np.array([[1.0, 0.0, 0.0]], np.float32)
        packed, ri, ts, te = oracle.march(o, d, mask, res, BOX, 0.0, 1e10, float(dt))
        tn, tf, hit = oracle.clip(o, d, BOX, 0.0, 1e10)
        t0 = Fraction(float(tn[0]))
        for k in range(1, packed[0, 1]):
            prod = _round_f32(Fraction(k) * Fraction(float(dt)))
            two = _round_f32(t0 + Fraction(float(prod)))
            fma = _round_f32(t0 + Fraction(k) * Fraction(float(dt)))
            assert ts[k] == two, (a, k)
            n_diff += int(two != fma)
    assert n_diff >= 20  # the fixture does tell the two forms apart


def test_rays_missing_box_and_max_per_ray():
    o = np.array([[0.0, 3.0, -4.0], [0.0, 0.0, -4.0]], np.float32)
    d = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0]], np.float32)
    mask = np.ones(8 ** 3, np.uint8)
    packed, ri, ts, te = oracle.march(o, d, mask, 8, BOX, 0.0, 1e10, 0.05)
    assert packed[0, 1] == 0 and packed[1, 1] == 60
    packed, ri, ts, te = oracle.march(o, d, mask, 8, BOX, 0.0, 1e10, 0.05,
                                      max_per_ray=7)
    assert packed[1, 1] == 7 and ri.size == 7


def test_near_far_planes():
    o = np.array([[0.0, 0.0, -4.0]], np.float32)
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    mask = np.ones(8 ** 3, np.uint8)
    packed, ri, ts, te = oracle.march(o, d, mask, 8, BOX, 3.0, 4.0, 0.1)
    assert ts[0] == np.float32(3.0)
    assert packed[0, 1] == 10


def test_cone_steps_count_closed_form():
    # Full grid, cone stepping: steps of dt until t * cone reaches dt, then a
    # geometric progression with ratio (1 + cone): count ~ (t* - t_near) / dt
    # + ln(t_far / t*) / ln(1 + cone), t* = dt / cone.
    cone, dt = 1.0 / 256, 1.0 / 512
    o = np.array([[0.0, 0.0, 0.0]], np.float32)
    d = np.array([[1.0, 0.0, 0.0]], np.float32)
    box = np.array([-64, -64, -64, 64, 64, 64], np.float32)
    mask = np.ones(4 ** 3, np.uint8)
    packed, ri, ts, te = oracle.march(o, d, mask, 4, box, 0.1, 60.0, dt,
                                      dt_max=1e10, cone=cone)
    t_star = dt / cone
    expect = (t_star - 0.1) / dt + math.log(60.0 / t_star) / math.log1p(cone)
    assert abs(packed[0, 1] - expect) <= 2.0
    steps = te - ts
    assert np.all(np.diff(ts) > 0)
    assert np.all(steps >= np.float32(dt) * (1 - 1e-4))
    big = ts > 2 * t_star
    assert np.allclose(steps[big] / ts[big], cone, rtol=1e-4)
    # dt_max caps the step
    packed2, ri2, ts2, te2 = oracle.march(o, d, mask, 4, box, 0.1, 60.0, dt,
                                          dt_max=0.05, cone=cone)
    assert np.max(te2 - ts2) <= np.float32(0.05) * (1 + 1e-4)


def test_cascade_level_selection():
    # Cascaded grids over [-1,1]^3 * 2^l, l = 0..3: occupy only level 2.
    # Samples must be exactly those whose midpoint has 2 < max|x| <= 4.
    res, levels = 8, 4
    mask = np.zeros((levels, res ** 3), np.uint8)
    mask[2] = 1
    base = np.array([-1, -1, -1, 1, 1, 1], np.float32)
    o, d = synth.rays_unbounded(200, 21)
    packed, ri, ts, te = oracle.march(o, d, mask.ravel(), res, base, 0.0, 1e10,
                                      0.01, lookup=oracle.LOOKUP_CASCADE,
                                      n_grids=levels)
    tn, tf, hit = oracle.clip(o, d, base * 8, 0.0, 1e10)
    for r in range(0, 200, 7):
        k = np.arange(int(np.ceil((float(tf[r]) - float(tn[r])) / 0.01)) + 1)
        tm = float(tn[r]) + (k + 0.5) * 0.01
        x = o[r].astype(np.float64) + d[r].astype(np.float64) * tm[:, None]
        m = np.abs(x).max(1)
        want = (m > 2) & (m <= 4) & (float(tn[r]) + k * 0.01 < float(tf[r]))
        amb = (np.abs(m - 2) < 1e-5) | (np.abs(m - 4) < 1e-5)
        got = np.zeros(k.size, bool)
        kk = np.round((ts[ri == r].astype(np.float64) - float(tn[r])) / 0.01).astype(int)
        got[kk] = True
        assert np.array_equal(got[~amb], want[~amb])
    # a point exactly on a level boundary (max|x| = 2^l) belongs to level l
    o1 = np.array([[2.0, 0.0, -9.0]], np.float32)
    d1 = np.array([[0.0, 0.0, 1.0]], np.float32)
    mask1 = np.zeros((levels, res ** 3), np.uint8)
    mask1[1] = 1
    packed1, _, ts1, te1 = oracle.march(o1, d1, mask1.ravel(), res, base, 0.0,
                                        1e10, 0.25, lookup=oracle.LOOKUP_CASCADE,
                                        n_grids=levels)
    mids = -9.0 + (ts1.astype(np.float64) + te1) / 2
    assert packed1[0, 1] > 0 and np.all(np.abs(mids) <= 2.0)


@pytest.mark.parametrize("x0,t_min", [(0.5, 0.5), (1.5, 2.0)])
def test_contraction_axis(x0, t_min):
    # Contracted grid over [-2,2]^3 occupied where x' >= x0.  Along +x from the
    # origin, x' = t for t <= 1 and 2 - 1/t beyond: samples start at t = t_min.
    res = 64
    mask = np.zeros((res, res, res), np.uint8)
    j0 = int(round((x0 + 2.0) * res / 4.0))
    mask[j0:] = 1
    box = np.array([-2, -2, -2, 2, 2, 2], np.float32)
    o = np.array([[0.0, 0.0, 0.0]], np.float32)
    d = np.array([[1.0, 0.0, 0.0]], np.float32)
    dt = 0.004
    packed, ri, ts, te = oracle.march(o, d, mask.ravel(), res, box, 0.0, 50.0,
                                      dt, lookup=oracle.LOOKUP_CONTRACT)
    mids = (ts.astype(np.float64) + te) / 2
    assert abs(mids[0] - t_min) <= dt
    assert packed[0, 1] == int(np.ceil((50.0 - 0.0) / dt)) - int(np.floor(t_min / dt))


def test_contraction_uses_euclidean_norm():
    # Along (1,1,0)/sqrt(2): x'_0 = (2 - 1/t) / sqrt(2) beyond t = 1, so a grid
    # occupied for x'_0 >= 1 starts at t = 1 / (2 - sqrt(2)).
    res = 64
    mask = np.zeros((res, res, res), np.uint8)
    mask[48:] = 1  # x' >= 1.0
    box = np.array([-2, -2, -2, 2, 2, 2], np.float32)
    o = np.zeros((1, 3), np.float32)
    d = np.array([[1.0, 1.0, 0.0]], np.float32) / np.float32(math.sqrt(2.0))
    packed, ri, ts, te = oracle.march(o, d, mask.ravel(), res, box, 0.0, 20.0,
                                      0.002, lookup=oracle.LOOKUP_CONTRACT)
    first_mid = (float(ts[0]) + float(te[0])) / 2
    assert abs(first_mid - 1.0 / (2.0 - math.sqrt(2.0))) < 0.003


# ---------------------------------------------------------------------------
# Rendering, Eq. 1 (Sec. 2.2)
# ---------------------------------------------------------------------------

def _uniform_segment(n, t0, dt, sigma, color):
    ts = t0 + dt * np.arange(n)
    te = ts + dt
    packed = np.array([[0, n]], np.int32)
    return packed, ts, te, np.full(n, sigma), np.tile(color, (n, 1))


def test_constant_density_closed_form():
    n, t0, dt, sigma = 50, 1.25, 0.02, 7.0
    c = np.array([0.2, 0.5, 0.9])
    packed, ts, te, sg, cl = _uniform_segment(n, t0, dt, sigma, c)
    out = oracle.render_fwd(packed, ts, te, sg, cl)
    q = math.exp(-sigma * dt)
    a = 1 - q ** n
    assert out["opacity"][0] == pytest.approx(a, rel=1e-13)
    assert np.allclose(out["color"][0], c * a, rtol=1e-13)
    # depth: (1-q) sum_k q^k (t0 + (k + 1/2) dt)
    s0 = (1 - q ** n) / (1 - q)
    s1 = q * (1 - n * q ** (n - 1) + (n - 1) * q ** n) / (1 - q) ** 2
    depth = (1 - q) * ((t0 + 0.5 * dt) * s0 + dt * s1)
    assert out["depth"][0] == pytest.approx(depth, rel=1e-12)
    # transmittance T_k = exp(-sigma k dt): weights are (1-q) q^k
    assert np.allclose(out["weights"], (1 - q) * q ** np.arange(n), rtol=1e-12)


def test_weights_telescope():
    packed, ts, te, sg, cl = synth.ragged_render_inputs(200, 3)
    out = oracle.render_fwd(packed, ts, te, sg, cl)
    tau = sg.astype(np.float64) * (te.astype(np.float64) - ts)
    for r in range(200):
        a, n = packed[r]
        t_final = math.exp(-tau[a:a + n].sum())
        assert out["opacity"][r] == pytest.approx(1 - t_final, rel=1e-12, abs=1e-15)
        assert out["weights"][a:a + n].sum() == pytest.approx(1 - t_final,
                                                             rel=1e-12, abs=1e-15)
    assert np.all(out["weights"] >= 0) and np.all(out["opacity"] <= 1)


def test_early_termination_cut():
    packed, ts, te, sg, cl = synth.ragged_render_inputs(300, 4, sigma_max=400.0)
    eps = 1e-4
    out = oracle.render_fwd(packed, ts, te, sg, cl, eps)
    tau = sg.astype(np.float64) * (te.astype(np.float64) - ts)
    n_cut = 0
    for r in range(300):
        a, n = packed[r]
        k = out["kept"][r]
        pre = np.concatenate([[0.0], np.cumsum(tau[a:a + n])])
        trans = np.exp(-pre)
        assert np.all(trans[:k] >= eps)
        if k < n:
            n_cut += 1
            assert trans[k] < eps
            assert np.all(out["weights"][a + k:a + n] == 0)
        assert out["opacity"][r] == pytest.approx(1 - trans[k], rel=1e-12, abs=1e-15)
    assert n_cut > 20


def test_single_sample_weight_is_alpha():
    packed = np.array([[0, 1]], np.int32)
    out = oracle.render_fwd(packed, [2.0], [2.5], [3.0], [[0.1, 0.6, 1.0]])
    alpha = 1 - math.exp(-1.5)
    assert out["weights"][0] == pytest.approx(alpha, rel=1e-15)
    assert np.allclose(out["color"][0], alpha * np.array([0.1, 0.6, 1.0]), rtol=1e-15)
    assert out["depth"][0] == pytest.approx(alpha * 2.25, rel=1e-15)


def test_first_opaque_sample_terminates():
    # A first sample with tau = 40 leaves T_1 = e^-40 < 1e-4: only it counts.
    packed = np.array([[0, 3]], np.int32)
    out = oracle.render_fwd(packed, [0, 1, 2], [1, 2, 3], [40.0, 1.0, 1.0],
                            [[1, 0, 0], [0, 1, 0], [0, 0, 1]], eps=1e-4)
    assert out["kept"][0] == 1
    assert out["color"][0][1] == 0 and out["color"][0][2] == 0


# ---------------------------------------------------------------------------
# Gradients (Sec. 2.2: every field output receives a gradient)
# ---------------------------------------------------------------------------

def test_single_sample_gradient_closed_form():
    sigma, dt = 3.0, 0.5
    c = np.array([0.1, 0.6, 1.0])
    gc = np.array([0.3, -0.7, 0.2])
    ga, gd = 0.4, -0.05
    packed = np.array([[0, 1]], np.int32)
    out = oracle.render_bwd(packed, [2.0], [2.5], [sigma], [c], [gc], [ga], [gd])
    v = gc @ c + ga + gd * 2.25
    assert out["g_sigmas"][0] == pytest.approx(dt * math.exp(-sigma * dt) * v, rel=1e-14)
    alpha = 1 - math.exp(-sigma * dt)
    assert np.allclose(out["g_rgbs"][0], alpha * gc, rtol=1e-14)


def test_two_sample_gradient_closed_form():
    # L = g . (w0 c0 + w1 c1), w0 = 1 - e^-t0, w1 = e^-t0 (1 - e^-t1):
    # dL/dtau0 = e^-t0 g.c0 - e^-t0 (1 - e^-t1) g.c1, dL/dtau1 = e^-(t0+t1) g.c1
    s0, s1, d0, d1 = 2.0, 5.0, 0.25, 0.125
    c0, c1 = np.array([1.0, 0.0, 0.5]), np.array([0.0, 1.0, 0.25])
    g = np.array([0.7, -0.2, 0.4])
    packed = np.array([[0, 2]], np.int32)
    out = oracle.render_bwd(packed, [0.0, 1.0], [d0, 1.0 + d1], [s0, s1],
                            [c0, c1], [g])
    t0, t1 = s0 * d0, s1 * d1
    dtau0 = math.exp(-t0) * g @ c0 - math.exp(-t0) * (1 - math.exp(-t1)) * g @ c1
    dtau1 = math.exp(-t0 - t1) * g @ c1
    assert out["g_sigmas"][0] == pytest.approx(d0 * dtau0, rel=1e-13)
    assert out["g_sigmas"][1] == pytest.approx(d1 * dtau1, rel=1e-13)


@pytest.mark.parametrize("eps", [0.0, 1e-4])
def test_gradient_matches_finite_differences(eps):
    packed, ts, te, sg, cl = synth.ragged_render_inputs(40, 6, mean_count=25,
                                                        sigma_max=120.0)
    g = np.random.default_rng(7)
    gc = g.standard_normal((40, 3))
    ga = g.standard_normal(40)
    gd = g.standard_normal(40)
    sg64 = sg.astype(np.float64)
    cl64 = cl.astype(np.float64)

    def loss(s, c):
        o = oracle.render_fwd(packed, ts, te, s, c, eps)
        return float((o["color"] * gc).sum() + (o["opacity"] * ga).sum()
                     + (o["depth"] * gd).sum())

    out = oracle.render_bwd(packed, ts, te, sg64, cl64, gc, ga, gd, eps)
    fwd = oracle.render_fwd(packed, ts, te, sg64, cl64, eps)
    idx = g.choice(sg.size, 60, replace=False)
    for s in idx:
        r = np.searchsorted(packed[:, 0], s, side="right") - 1
        while packed[r, 1] == 0 or s >= packed[r, 0] + packed[r, 1]:
            r -= 1
        # skip samples next to the early-termination cut (not differentiable)
        k = s - packed[r, 0]
        if eps > 0 and abs(k - fwd["kept"][r]) <= 1:
            continue
        h = 1e-6 * max(abs(sg64[s]), 1.0)
        sp, sm = sg64.copy(), sg64.copy()
        sp[s] += h
        sm[s] -= h
        fd = (loss(sp, cl64) - loss(sm, cl64)) / (2 * h)
        assert fd == pytest.approx(out["g_sigmas"][s],
                                   abs=1e-7 * max(1.0, out["scale"][s] / 1e-2))
        for ch in range(3):
            cp, cm = cl64.copy(), cl64.copy()
            cp[s, ch] += 1e-6
            cm[s, ch] -= 1e-6
            fdc = (loss(sg64, cp) - loss(sg64, cm)) / 2e-6
            assert fdc == pytest.approx(out["g_rgbs"][s, ch], abs=1e-8)


# ---------------------------------------------------------------------------
# Rendering of arbitrary attributes, background, opacity threshold (Sec. 2.2
# "any sample attributes"; Sec. 4 constant background)
# ---------------------------------------------------------------------------

def test_attrs_constant_density_background_closed_form():
    # n equal intervals of width h at density s, every sample carrying the
    # same attributes a: out = a A + b (1 - A), A = 1 - e^(-s n h),
    # depth = sum_i T_i alpha (t_i + h/2) with T_i = e^(-s h i)
    n, h, s = 50, 0.02, 3.0
    a = np.array([0.2, -1.5, 7.0, 0.0, 3.25, 1.0, -0.5])
    b = np.array([1.0, 0.5, -2.0, 4.0, 0.0, 0.25, 1.0])
    ts = h * np.arange(n)
    packed = np.array([[0, n], [n, 0]], np.int32)  # the second ray is empty
    out = oracle.render_attrs_fwd(packed, ts, ts + h, np.full(n, s), np.tile(a, (n, 1)),
                                  background=b)
    big_a = 1.0 - math.exp(-s * n * h)
    assert out["opacity"][0] == pytest.approx(big_a, rel=1e-13)
    assert np.allclose(out["out"][0], a * big_a + b * (1 - big_a), rtol=1e-13, atol=1e-15)
    alpha = 1.0 - math.exp(-s * h)
    dep = sum(math.exp(-s * h * i) * alpha * (h * i + h / 2) for i in range(n))
    assert out["depth"][0] == pytest.approx(dep, rel=1e-13)
    assert np.array_equal(out["out"][1], b) and out["opacity"][1] == 0.0


def test_attrs_opacity_threshold_closed_form():
    # three samples, the first below the threshold: it neither contributes
    # nor attenuates, so w_2 = alpha_2 and w_3 = (1 - alpha_2) alpha_3
    sig = np.array([0.5, 1.0, 2.0])
    ts = np.array([0.0, 1.0, 2.0])
    a = np.array([[10.0, 1.0], [2.0, -1.0], [3.0, 5.0]])
    out = oracle.render_attrs_fwd(np.array([[0, 3]], np.int32), ts, ts + 1.0, sig, a,
                                  alpha_thre=0.5)
    a1, a2 = 1 - math.exp(-1.0), 1 - math.exp(-2.0)
    w = np.array([0.0, a1, (1 - a1) * a2])
    assert np.allclose(out["weights"], w, rtol=1e-14)
    assert np.allclose(out["out"][0], w @ a, rtol=1e-14)


@pytest.mark.parametrize("eps", [0.0, 1e-2])
def test_attrs_threshold_equals_dropping_the_samples(eps):
    """Samples below the opacity threshold are as if they were not on the
    ray: rendering with the threshold equals rendering, without it, the
    samples that remain (their opacity taken here with numpy)."""
    packed, ts, te, sg, _ = synth.ragged_render_inputs(60, 21, mean_count=30, sigma_max=40.0)
    attrs = np.random.default_rng(21).standard_normal((ts.size, 5))
    bg = np.array([0.5, -1.0, 2.0, 0.0, 1.0])
    alpha = -np.expm1(-sg.astype(np.float64) * (te.astype(np.float64) - ts.astype(np.float64)))
    thre = 0.1
    keep = alpha >= thre
    assert 0.1 < keep.mean() < 0.9
    ray_of = np.repeat(np.arange(packed.shape[0]), packed[:, 1])
    counts = np.bincount(ray_of[keep], minlength=packed.shape[0])
    packed_k = np.stack([np.concatenate([[0], np.cumsum(counts)[:-1]]), counts], 1).astype(np.int32)
    masked = oracle.render_attrs_fwd(packed, ts, te, sg, attrs, eps, thre, bg)
    dropped = oracle.render_attrs_fwd(packed_k, ts[keep], te[keep], sg[keep], attrs[keep], eps, 0.0,
                                      bg)
    for name in ("out", "opacity", "depth"):
        assert np.allclose(masked[name], dropped[name], rtol=1e-13, atol=1e-15)
    assert np.all(masked["weights"][~keep] == 0.0)


@pytest.mark.parametrize("eps,thre", [(0.0, 0.0), (1e-3, 0.2)])
def test_attrs_gradient_matches_finite_differences(eps, thre):
    packed, ts, te, sg, _ = synth.ragged_render_inputs(30, 22, mean_count=20, sigma_max=60.0)
    g = np.random.default_rng(22)
    ch = 6
    attrs = g.standard_normal((ts.size, ch))
    bg = g.standard_normal(ch)
    g_out = g.standard_normal((30, ch))
    ga = g.standard_normal(30)
    gd = g.standard_normal(30)
    sg64 = sg.astype(np.float64)

    def loss(s, a):
        o = oracle.render_attrs_fwd(packed, ts, te, s, a, eps, thre, bg)
        return float((o["out"] * g_out).sum() + (o["opacity"] * ga).sum()
                     + (o["depth"] * gd).sum())

    out = oracle.render_attrs_bwd(packed, ts, te, sg64, attrs, g_out, ga, gd, eps, thre, bg)
    alpha = -np.expm1(-sg64 * (te.astype(np.float64) - ts.astype(np.float64)))
    # the transmittance at each sample, to stay away from the cut
    tau = np.where(alpha >= thre, sg64 * (te.astype(np.float64) - ts.astype(np.float64)), 0.0)
    checked = 0
    for s in g.choice(sg.size, 120, replace=False):
        r = np.searchsorted(packed[:, 0], s, side="right") - 1
        while packed[r, 1] == 0 or s >= packed[r, 0] + packed[r, 1]:
            r -= 1
        a0 = packed[r, 0]
        trans = math.exp(-tau[a0:s].sum())
        if (abs(alpha[s] - thre) < 1e-3 or (eps > 0 and abs(trans / eps - 1) < 0.5)
                or sg64[s] == 0.0):
            continue  # not differentiable across the threshold or the cut (a
            # zero density lies on the threshold 0: sigma - h is below it)
        h = 1e-6 * max(abs(sg64[s]), 1.0)
        sp, sm = sg64.copy(), sg64.copy()
        sp[s] += h
        sm[s] -= h
        fd = (loss(sp, attrs) - loss(sm, attrs)) / (2 * h)
        assert fd == pytest.approx(out["g_sigmas"][s], abs=1e-7 * max(1.0, out["scale"][s] / 1e-2))
        for k in range(ch):
            ap, am = attrs.copy(), attrs.copy()
            ap[s, k] += 1e-6
            am[s, k] -= 1e-6
            fda = (loss(sg64, ap) - loss(sg64, am)) / 2e-6
            assert fda == pytest.approx(out["g_attrs"][s, k], abs=1e-8)
        checked += 1
    assert checked > 30
    if thre > 0:
        assert np.all(out["g_sigmas"][alpha < thre] == 0.0)


def test_gradient_zero_past_cut():
    packed = np.array([[0, 3]], np.int32)
    out = oracle.render_bwd(packed, [0, 1, 2], [1, 2, 3], [40.0, 1.0, 1.0],
                            [[1, 0, 0], [0, 1, 0], [0, 0, 1]], [[1, 1, 1]],
                            eps=1e-4)
    assert out["g_sigmas"][1] == 0 and out["g_sigmas"][2] == 0
    assert np.all(out["g_rgbs"][1:] == 0)


# ---------------------------------------------------------------------------
# Occupancy-grid update
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((5, 17, 0, 0), (123456789, 0)),
    ((2 ** 64 - 1, 3, 2 ** 63, 7), (2 ** 64 - 1, 2 ** 40 + 3)),
])
def test_philox_matches_numpy(counter, key):
    # numpy's Philox bit generator is Philox4x64-10; it increments its
    # counter before producing a block, so start it one step behind.
    value = sum(int(w) << (64 * i) for i, w in enumerate(counter))
    value = (value - 1) % (1 << 256)
    prev = np.array([(value >> (64 * i)) & (2 ** 64 - 1) for i in range(4)],
                    np.uint64)
    bg = np.random.Philox(counter=prev, key=np.array(key, np.uint64))
    want = bg.random_raw(4)
    got = oracle.philox4x64_10(np.array(counter, np.uint64), np.array(key, np.uint64))
    assert np.array_equal(got, want)


def test_sample_cells_inside_and_uniform():
    res = 16
    cells, pos = oracle.grid_sample_cells(99, 3, 200000, res, BOX)
    assert cells.min() >= 0 and cells.max() < res ** 3
    j = np.stack([cells // (res * res), (cells // res) % res, cells % res], 1)
    h = 3.0 / res
    lo = -1.5 + j * h
    assert np.all(pos >= lo - 1e-6) and np.all(pos <= lo + h + 1e-6)
    hist = np.bincount(cells, minlength=res ** 3)
    expect = 200000 / res ** 3
    chi2 = ((hist - expect) ** 2 / expect).sum()
    assert chi2 < res ** 3 + 6 * math.sqrt(2 * res ** 3)
    # different steps give different draws, the same step the same draws
    c2, _ = oracle.grid_sample_cells(99, 4, 1000, res, BOX)
    c3, _ = oracle.grid_sample_cells(99, 3, 1000, res, BOX)
    assert not np.array_equal(c2, cells[:1000]) and np.array_equal(c3, cells[:1000])


def test_sample_cells_cascade_levels():
    res, levels = 8, 4
    base = np.array([-1, -1, -1, 1, 1, 1], np.float32)
    cells, pos = oracle.grid_sample_cells(5, 0, 50000, res, base, levels, cascade=True)
    lvl = cells // res ** 3
    assert set(np.unique(lvl)) == {0, 1, 2, 3}
    m = np.abs(pos).max(1)
    assert np.all(m <= 2.0 ** lvl + 1e-6)


def test_decay_update_threshold():
    g = np.random.default_rng(8)
    occ0 = g.uniform(0, 1, 4096).astype(np.float32)
    o = occ0
    for _ in range(5):
        o = oracle.grid_decay(o, 0.95)
    want = occ0.copy()
    for _ in range(5):
        want = (want * np.float32(0.95)).astype(np.float32)
    assert np.array_equal(o, want)
    cells = g.integers(0, 4096, 10000).astype(np.int32)
    vals = g.uniform(0, 1.2, 10000).astype(np.float32)
    got = oracle.grid_update_max(o, cells, vals)
    ref = o.copy()
    np.maximum.at(ref, cells, vals)
    assert np.array_equal(got, ref)
    perm = g.permutation(10000)
    assert np.array_equal(oracle.grid_update_max(o, cells[perm], vals[perm]), got)
    m = oracle.grid_threshold(got, 0.5)
    assert np.array_equal(m.astype(bool), got > np.float32(0.5))
    # strict threshold
    assert oracle.grid_threshold(np.array([0.5, 0.5000001], np.float32), 0.5).tolist() == [0, 1]


# ---------------------------------------------------------------------------
# Synthetic field (test input)
# ---------------------------------------------------------------------------

def test_blob_field_closed_form():
    scene = synth.blob_scene(1, 3)
    c = scene.centres[0, 0].astype(np.float64)
    s = float(scene.stds[0])
    pts = np.array([c, c + [s, 0, 0], c + [0, 2 * s, 0]], np.float32)
    sigma, rgb = oracle.blob_field(scene, pts)
    p64 = pts.astype(np.float64)
    r2 = ((p64 - c) ** 2).sum(1)
    assert np.allclose(sigma, 50.0 * np.exp(-r2 / (2 * s * s)), rtol=1e-12)
    z = p64 @ scene.w.astype(np.float64).T + scene.bias
    from scipy.special import expit
    assert np.allclose(rgb, expit(z), rtol=1e-12)


def test_blob_field_in_contracted_space():
    """A scene defined in contracted coordinates: world points beyond the
    unit ball are evaluated at radius 2 - 1/|x| along their own direction
    (Euclidean norm), points inside it unchanged.  Values with closed forms:
    (2,0,0) -> (1.5,0,0); (4,0,0) -> (1.75,0,0); (2,2,1) (norm 3) ->
    (10/9, 10/9, 5/9); (0.625,0,0) -> itself."""
    import dataclasses
    from scipy.special import expit
    base = synth.BlobScene(centres=np.array([[[1.5, 0.0, 0.0]]], np.float32),
                           stds=np.array([0.125], np.float32), peaks=np.array([7.0], np.float32),
                           w=np.eye(3, dtype=np.float32), bias=np.zeros(3, np.float32),
                           contract=True)
    pts = np.array([[2, 0, 0], [4, 0, 0], [0.625, 0, 0], [-2, 0, 0]], np.float32)
    sigma, rgb = oracle.blob_field(base, pts)
    k = 1.0 / (2 * 0.125 ** 2)
    want = 7.0 * np.exp(-k * np.array([0.0, 0.25 ** 2, 0.875 ** 2, 3.0 ** 2]))
    assert np.allclose(sigma, want, rtol=1e-12, atol=0)
    assert np.allclose(rgb[0], expit([1.5, 0.0, 0.0]), rtol=1e-12)
    assert np.allclose(rgb[3], expit([-1.5, 0.0, 0.0]), rtol=1e-12)
    diag = dataclasses.replace(base, centres=np.array([[[10 / 9, 10 / 9, 5 / 9]]], np.float32))
    s2 = oracle.blob_field(diag, np.array([[2, 2, 1]], np.float32), want_rgb=False)
    c = np.array([10 / 9, 10 / 9, 5 / 9])
    d2 = ((c - c.astype(np.float32)) ** 2).sum()  # the centre is stored in FP32
    assert abs(s2[0] - 7.0 * np.exp(-k * d2)) <= 1e-12
    # without the flag the same scene is evaluated in world coordinates
    plain = dataclasses.replace(base, contract=False)
    s3 = oracle.blob_field(plain, np.array([[2, 0, 0]], np.float32), want_rgb=False)
    assert np.isclose(s3[0], 7.0 * np.exp(-k * 0.25), rtol=1e-12)


def test_unbounded_scene_generator():
    """Blob centres of the unbounded scene sit at the contracted images of
    world radii 1 .. 8 (contracted radius 2 - 1/R), and a blob's optical
    depth along its radius is level-independent by construction."""
    scene = synth.unbounded_blob_scene(8, 4, 5)
    r = np.linalg.norm(scene.centres[0].astype(np.float64), axis=1)
    world = 2.0 ** (3.0 * np.repeat(np.arange(8), 4) / 7.0)
    assert np.allclose(r, 2.0 - 1.0 / world, rtol=1e-6)
    depth = (scene.peaks.astype(np.float64) * np.sqrt(2 * np.pi) * scene.stds * world ** 2)
    assert depth.min() >= 2.0 - 1e-5 and depth.max() <= 6.0 + 1e-5


def test_contracted_grid_occupancy_generator():
    """The contraction lookup's grid holds the scene density at its cell
    centres read directly in contracted coordinates, the same values the
    cascades read at the contraction of their world cell centres: a cell
    centre of the contracted grid inside the unit ball is its own world
    point, so the two generators agree where a level-0 cascade cell centre
    coincides with it."""
    import dataclasses
    scene = synth.unbounded_blob_scene(8, 4, 5)
    res = 16
    occ = synth.contracted_occupancy(scene, res)
    pts = synth.cell_centres(res, synth.CONTRACT_BOX)
    direct = oracle.blob_field(dataclasses.replace(scene, contract=False), pts.astype(np.float32),
                               want_rgb=False)
    assert np.all(np.abs(occ - direct) <= 1e-5 * direct + 1e-7)
    # cascade level 0 over [-1, 1]^3 at resolution res / 2 has the same cell
    # centres as the inner half of the contracted grid, where c(x) = x
    cas = synth.cascade_occupancy(scene, res // 2, 1).reshape(res // 2, res // 2, res // 2)
    inner = occ.reshape(res, res, res)[res // 4:3 * res // 4, res // 4:3 * res // 4,
                                       res // 4:3 * res // 4]
    c = synth.cell_centres(res // 2, (-1, -1, -1, 1, 1, 1)).reshape(res // 2, res // 2, res // 2, 3)
    inside = np.linalg.norm(c, axis=-1) <= 1.0
    assert inside.sum() > 100
    assert np.array_equal(cas[inside], inner[inside])


# ---------------------------------------------------------------------------
# Visibility pruning while marching (Sec. 2.1 occluded regions, Sec. 3)
# ---------------------------------------------------------------------------

def _packed(counts):
    counts = np.asarray(counts, np.int64)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    return np.stack([starts, counts], 1).astype(np.int32)


def test_prune_constant_density_closed_form():
    # n equal intervals of width h at density s: T_i = exp(-s h i), so the
    # samples with s h i <= ln(1/eps) survive: floor(ln(1/eps) / (s h)) + 1
    h, n = 0.01, 400
    for s, eps in ((30.0, 1e-4), (7.0, 1e-3), (123.0, 1e-2)):
        ts = np.arange(n) * h
        keep, counts = oracle.prune(_packed([n]), ts, ts + h, np.full(n, s), eps, 0.0)
        q = math.log(1.0 / eps) / (s * h)
        assert abs(q - round(q)) > 1e-6
        want = min(n, math.floor(q) + 1)
        assert counts[0] == want and keep.sum() == want
        assert np.all(keep[:want] == 1) and np.all(keep[want:] == 0)


def test_prune_alpha_threshold_and_transmittance_of_dropped_samples():
    # alpha_i = 1 - exp(-s_i h) >= thre  <=>  s_i h >= -ln(1 - thre); a dropped
    # low-opacity sample still darkens the ones after it
    h = 0.1
    thre = 0.05
    s_cut = -math.log(1 - thre) / h       # ~0.513
    sig = np.array([0.0, 0.3, 0.6, 5.0, 0.2, 80.0, 1.0, 0.0, 3.0])
    ts = np.arange(sig.size) * h
    keep, counts = oracle.prune(_packed([sig.size]), ts, ts + h, sig, 0.0, thre)
    assert np.array_equal(keep, (sig >= s_cut).astype(np.uint8))
    # with the transmittance test at eps 2e-4: sample 6 sits behind
    # T = exp(-(0 + .3 + .6 + 5 + .2 + 80) * .1) = exp(-8.61) ~ 1.8e-4 and is
    # dropped, as is everything after it; sample 3 (T = exp(-.09)) is kept
    keep2, _ = oracle.prune(_packed([sig.size]), ts, ts + h, sig, 2e-4, thre)
    pre = np.concatenate([[0.0], np.cumsum(sig * h)[:-1]])
    want = ((np.exp(-pre) >= 2e-4) & (sig >= s_cut)).astype(np.uint8)
    assert np.array_equal(keep2, want) and keep2[3] == 1 and keep2[6] == 0


def test_prune_dropped_sample_still_attenuates():
    # An opaque sample (tau = 8.0), then a faint one below the opacity
    # threshold (tau = 0.03, alpha = 0.0296 < 0.05), then a dense one.  The
    # third sample's transmittance is exp(-8.03) = 3.2585e-4 when the dropped
    # sample attenuates and exp(-8.0) = 3.3546e-4 if it did not; eps =
    # 3.3e-4 lies between, so only the attenuating rule drops sample 2.
    h = 0.1
    sig = np.array([80.0, 0.3, 5.0])
    ts = np.arange(sig.size) * h
    assert math.exp(-8.03) < 3.3e-4 < math.exp(-8.0)
    keep, counts = oracle.prune(_packed([3]), ts, ts + h, sig, 3.3e-4, 0.05)
    assert keep.tolist() == [1, 0, 0] and counts[0] == 1
    # the same ray without the faint sample keeps the dense one
    keep2, _ = oracle.prune(_packed([2]), ts[[0, 2]], ts[[0, 2]] + h, sig[[0, 2]],
                            3.3e-4, 0.05)
    assert keep2.tolist() == [1, 1]


def test_prune_degenerate_settings_keep_everything():
    packed, ts, te, sg, _ = synth.ragged_render_inputs(300, 71)
    keep, counts = oracle.prune(packed, ts, te, sg, 0.0, 0.0)
    assert keep.all() and np.array_equal(counts, packed[:, 1])
    # eps > 1 drops everything (T_0 = 1 < eps)
    keep, counts = oracle.prune(packed, ts, te, sg, 1.5, 0.0)
    assert not keep.any() and not counts.any()


def test_prune_matches_render_cut():
    # with alpha_thre = 0 the kept samples are exactly those before the
    # renderer's early-termination cut
    packed, ts, te, sg, rgb = synth.ragged_render_inputs(500, 72)
    keep, counts = oracle.prune(packed, ts, te, sg, 1e-4, 0.0)
    fwd = oracle.render_fwd(packed, ts, te, sg, rgb, 1e-4)
    assert np.array_equal(counts, fwd["kept"])
