"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the headers declare, carries gfx950 code, and rejects bad
arguments on the host before any launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include"))) if h.endswith(".h")]


def declared_symbols():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(nacc_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_headers_declare_the_binding():
    from paper_2210_04847_amd import _lib
    assert set(declared_symbols()) == set(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    from paper_2210_04847_amd import _lib
    raw = ctypes.CDLL(_lib.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(raw, s)]
    assert not missing, missing


def test_library_holds_gfx950_code():
    from paper_2210_04847_amd import _lib
    data = open(_lib.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_status_strings_and_version():
    from paper_2210_04847_amd import _lib
    assert _lib.version().startswith("nacc")
    assert _lib.status_name(_lib.NACC_ECAPACITY) == "NACC_ECAPACITY"
    assert _lib.status_name(12345) == "NACC_UNKNOWN"


def _march_count_raw(lib, n_rays, desc, params, ws_bytes=1 << 20):
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    return lib.nacc_march_count(fake, fake, None, n_rays, fake, None, ctypes.byref(desc),
                                ctypes.byref(params), fake, fake, fake, ws_bytes, None)


@pytest.mark.parametrize("field,value", [
    ("res", 0), ("res", 2000), ("lookup", 7), ("n_grids", 0), ("res", 3),
])
def test_bad_grid_rejected_on_host(field, value):
    from paper_2210_04847_amd import _lib
    desc = _lib.grid_desc((-1, -1, -1), (1, 1, 1), 8)
    setattr(desc, field, value)
    params = _lib.march_params(0.0, 10.0, 0.01)
    st = _march_count_raw(_lib.lib, 10, desc, params)
    assert st in (_lib.NACC_EINVAL, _lib.NACC_ESHAPE)
    assert _lib.lib.nacc_last_error().decode()


@pytest.mark.parametrize("kw", [dict(dt=0.0), dict(dt=float("nan")), dict(cone=-1.0),
                                dict(cone=0.01, dt_max=0.001), dict(max_per_ray=-2),
                                dict(near_plane=float("nan"))])
def test_bad_params_rejected_on_host(kw):
    from paper_2210_04847_amd import _lib
    desc = _lib.grid_desc((-1, -1, -1), (1, 1, 1), 8)
    args = dict(near_plane=0.0, far_plane=10.0, dt=0.01, dt_max=1e10, cone=0.0, max_per_ray=0)
    args.update(kw)
    params = _lib.march_params(**args)
    assert _march_count_raw(_lib.lib, 10, desc, params) == _lib.NACC_EINVAL


def test_bad_cascade_box_rejected():
    from paper_2210_04847_amd import _lib
    desc = _lib.grid_desc((-1.5, -1.5, -1.5), (1.5, 1.5, 1.5), 8, 4, _lib.LOOKUP_CASCADE)
    params = _lib.march_params(0.0, 10.0, 0.01)
    assert _march_count_raw(_lib.lib, 10, desc, params) == _lib.NACC_EINVAL


def test_small_workspace_and_bad_sizes_rejected():
    from paper_2210_04847_amd import _lib
    desc = _lib.grid_desc((-1, -1, -1), (1, 1, 1), 8)
    params = _lib.march_params(0.0, 10.0, 0.01)
    assert _march_count_raw(_lib.lib, 100000, desc, params, ws_bytes=8) == _lib.NACC_ESHAPE
    assert _march_count_raw(_lib.lib, -1, desc, params) == _lib.NACC_EINVAL
    fake = ctypes.c_void_p(0x1000)
    lib = _lib.lib
    assert lib.nacc_render_fwd(fake, 10, 5, fake, fake, fake, fake, 1.5, fake, fake, fake, None,
                               None, None) == _lib.NACC_EINVAL
    assert lib.nacc_render_fwd(fake, 10, 5, None, fake, fake, fake, 0.0, fake, fake, fake, None,
                               None, None) == _lib.NACC_EINVAL
    assert lib.nacc_grid_pack(fake, 33, 0.5, fake, None) == _lib.NACC_ESHAPE
    assert lib.nacc_render_fwd_bwd_mse(fake, 0, 0, None, None, None, None, 0.0, fake, 0, fake, fake,
                                       fake, fake, fake, fake, fake, 1 << 20,
                                       None) == _lib.NACC_EINVAL
    assert lib.nacc_render_fwd_bwd_mse(fake, 10, 5, fake, fake, fake, fake, 0.0, fake, 3, fake, fake,
                                       fake, fake, fake, fake, fake, 1 << 20,
                                       None) == _lib.NACC_EINVAL  # loss_rays < n_rays
    assert lib.nacc_march_workspace_size(-5, ctypes.byref(desc), ctypes.byref(params)) == -1
    assert lib.nacc_march_workspace_size(64, ctypes.byref(desc), ctypes.byref(params)) >= 8
    bad = _lib.march_params(0.0, 10.0, -1.0)
    assert lib.nacc_march_workspace_size(64, ctypes.byref(desc), ctypes.byref(bad)) == -1


def test_tuning_validated_and_round_trips():
    from paper_2210_04847_amd import _lib
    before = _lib.get_tuning()
    _lib.set_tuning(render_cached_chunks=3, march_waves_per_group=2)
    assert _lib.get_tuning()["render_cached_chunks"] == 3
    for bad in (dict(render_cached_chunks=0), dict(march_waves_per_group=3),
                dict(render_mse_max_blocks=0), dict(render_prefetch=2)):
        with pytest.raises(_lib.NaccError):
            _lib.set_tuning(**bad)
    _lib.set_tuning(**before)
    assert _lib.get_tuning() == before


def test_workspace_sizes_do_not_follow_tuning():
    """A workspace sized once stays valid whatever the autotuner picks."""
    from paper_2210_04847_amd import _lib
    before = _lib.get_tuning()
    desc = _lib.grid_desc((-1.5,) * 3, (1.5,) * 3, 128)
    params = _lib.march_params(0.0, 1e10, 3 ** 0.5 * 3 / 1024)
    sizes = set()
    try:
        for blocks in (1, 4096, 1 << 20):
            for waves in (1, 2, 4):
                _lib.set_tuning(**dict(before, render_mse_max_blocks=blocks,
                                       march_waves_per_group=waves))
                sizes.add((_lib.render_mse_workspace_size(262144),
                           _lib.march_workspace_size(262144, desc, params)))
    finally:
        _lib.set_tuning(**before)
    assert len(sizes) == 1


def test_zero_rays_launch_nothing_but_need_total():
    from paper_2210_04847_amd import _lib
    desc = _lib.grid_desc((-1, -1, -1), (1, 1, 1), 8)
    params = _lib.march_params(0.0, 10.0, 0.01)
    fake = ctypes.c_void_p(0x1000)
    st = _lib.lib.nacc_march_count(fake, fake, None, 0, fake, None, ctypes.byref(desc),
                                   ctypes.byref(params), None, None, None, 0, None)
    assert st == _lib.NACC_EINVAL  # total is required even for zero rays


def _plan_desc_raw(_lib, **over):
    """A plan description whose pointers are never dereferenced: every case
    below fails validation on the host, before any device call."""
    fake = 0x1000
    d = _lib.PlanDesc()
    d.rays_o = d.rays_d = d.grid_bits = d.packed_info = d.total = fake
    d.ray_indices = d.t_starts = d.t_ends = d.sigmas = d.rgbs = fake
    d.color = d.opacity = d.depth = fake
    d.field = fake
    d.n_rays, d.capacity = 16, 1024
    d.grid = _lib.grid_desc((-1, -1, -1), (1, 1, 1), 8)
    d.params = _lib.march_params(0.0, 10.0, 0.01)
    for k, v in over.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("over", [
    dict(field=None), dict(color=None), dict(n_rays=-1), dict(capacity=-1),
    dict(capacity=1 << 31), dict(early_stop_eps=-1.0), dict(sigmas=None),
    dict(target=0x1000),                          # training without loss / gradients
    dict(target=0x1000, loss=0x1000, g_sigmas=0x1000, g_rgbs=0x1000, loss_rays=3),
    dict(occ=0x1000),                             # update without its arrays
    dict(occ=0x1000, update_cells=8, update_counter=0x1000, update_cell_ids=0x1000,
         update_positions=0x1000, update_values=0x1000),  # ... without its field stage
])
def test_bad_plan_rejected_on_host(over):
    from paper_2210_04847_amd import _lib
    d = _plan_desc_raw(_lib, **over)
    out = ctypes.c_void_p(0x1234)
    st = _lib.lib.nacc_plan_create(ctypes.byref(d), ctypes.byref(out))
    assert st == _lib.NACC_EINVAL
    assert out.value == 0x1234  # untouched on failure
    assert _lib.lib.nacc_last_error().decode()


def test_bad_plan_grid_rejected_on_host():
    from paper_2210_04847_amd import _lib
    out = ctypes.c_void_p()
    for over in (dict(grid=_lib.grid_desc((-1, -1, -1), (1, 1, 1), 3)),
                 dict(params=_lib.march_params(0.0, 10.0, 0.0))):
        d = _plan_desc_raw(_lib, **over)
        assert _lib.lib.nacc_plan_create(ctypes.byref(d), ctypes.byref(out)) == _lib.NACC_EINVAL


def test_plan_calls_on_null_plan_rejected():
    from paper_2210_04847_amd import _lib
    lib = _lib.lib
    assert lib.nacc_plan_destroy(None) == _lib.NACC_OK
    for st in (lib.nacc_plan_step(None, None), lib.nacc_plan_update(None, None),
               lib.nacc_plan_capture_step(None), lib.nacc_plan_launch(None, 0, None),
               lib.nacc_plan_autotune(None, 3, None, None, None)):
        assert st == _lib.NACC_EINVAL
    assert lib.nacc_synth_samples_stage_run(None, None) == _lib.NACC_EINVAL

