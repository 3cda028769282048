"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes

import numpy as np
import os
import re

import pytest

from paper_1412_4933_amd import pedsim, scenarios

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pedsim.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sim_create", "sim_step_lem", "sim_step_aco", "sim_stats", "sim_scratch_bytes",
              "sim_read_state", "sim_destroy", "sim_strerror", "sim_attach_tour",
              "sim_step_aco_tour", "sim_set_neighbours"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = pedsim.lib()
    for n in declared_functions():
        assert hasattr(L, n), n


def test_strerror_names_every_code():
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert pedsim.sim_strerror(code) not in ("", "unknown error")
    assert pedsim.sim_strerror(-99) == "unknown error"


def _params(**kw):
    base = dict(W=64, H=32, seed=1, step0=0, rho=0.1, dtau=1.0, alpha=1, beta=2, cross_a=4,
                cross_b=4)
    base.update(kw)
    return pedsim.SimParams(**base)


def test_scratch_bytes_cover_one_byte_per_cell():
    for W, H in ((1, 1), (64, 32), (200, 100), (1024, 512), (4096, 2048), (777, 3)):
        n = pedsim.sim_scratch_bytes(_params(W=W, H=H, cross_a=0, cross_b=0))
        assert n >= W * H and n % 256 == 0


@pytest.mark.parametrize("bad", [
    dict(W=0), dict(H=0), dict(W=-3), dict(W=65536, H=32768), dict(rho=0.0), dict(rho=1.5),
    dict(rho=float("nan")), dict(dtau=-1.0), dict(dtau=float("inf")), dict(alpha=-1),
    dict(alpha=9), dict(beta=9), dict(cross_a=65), dict(cross_b=-1)])
def test_bad_parameters_rejected_on_host(bad):
    p = _params(**bad)
    with pytest.raises(pedsim.SimError) as e:
        pedsim.sim_scratch_bytes(p)
    assert e.value.code == pedsim.SIM_EINVAL
    h = ctypes.c_void_p()
    rc = pedsim.lib().sim_create(ctypes.byref(p), 16, 16, None, 16, 1 << 20, None, ctypes.byref(h))
    assert rc == pedsim.SIM_EINVAL and not h.value


def test_missing_buffers_and_small_scratch_rejected_on_host():
    p = _params()
    need = pedsim.sim_scratch_bytes(p)
    h = ctypes.c_void_p()
    L = pedsim.lib()
    assert L.sim_create(ctypes.byref(p), None, 16, None, 16, need, None, ctypes.byref(h)) == pedsim.SIM_EINVAL
    assert L.sim_create(ctypes.byref(p), 16, 16, None, None, need, None, ctypes.byref(h)) == pedsim.SIM_ESCRATCH
    assert L.sim_create(ctypes.byref(p), 16, 16, None, 16, need - 1, None, ctypes.byref(h)) == pedsim.SIM_ESCRATCH
    assert L.sim_step_lem(None, 1, None) == pedsim.SIM_EINVAL
    assert L.sim_step_aco(None, 1, None) == pedsim.SIM_EINVAL


def test_params_of_scenario():
    s = scenarios.lem_200x100()
    p = pedsim.params_of(s)
    assert (p.W, p.H, p.seed, p.cross_a, p.cross_b) == (200, 100, 1, 11, 11)
    assert s.band_a == 11 and s.n_a == 1000


def test_scenario_bands_follow_the_band_rule():
    s = scenarios.aco_1024x512()
    assert s.band_a == 99 and s.band_b == 99 and s.agents == 100000
    import numpy as np
    assert np.all(s.code[:, 99:1024 - 99] != scenarios.GROUP_A)
    assert np.count_nonzero(s.code == scenarios.GROUP_A) == 50000
    assert sorted(s.ids[s.ids != 0].tolist()) == list(range(1, 100001))


def test_serving_requests_are_poisson_and_sized():
    from paper_1412_4933_amd import serve
    specs = scenarios.served_requests(64)
    reqs = serve.poisson_requests(specs, rate=100.0, seed=1)
    t = [r.arrival for r in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
    gaps = np.diff([0.0] + t)
    assert 0.005 < gaps.mean() < 0.02  # rate 100/s
    for r, (W, H, N, band, mode, steps, seed) in zip(reqs, specs):
        assert 200 <= r.steps <= 2000 and r.agents == N
        assert r.nbytes >= W * H * (5 + (8 if mode == 1 else 0))


def test_batch_shapes_follow_the_recipe():
    shapes = scenarios.batch_shapes(256)
    assert len(shapes) == 256
    for i, (W, H, N, band, mode) in enumerate(shapes):
        assert 64 <= W <= 2048 and W % 2 == 0 and H == W // 2
        assert 500 <= N <= 100000 and N % 2 == 0 and N <= 2 * (W // 4) * (H - 2)
        assert mode == (i % 2)


def test_library_loads_after_torch_runtime():
    """The library shares torch's HIP runtime: loading it brings torch in first."""
    import sys
    pedsim.lib()
    assert "torch" in sys.modules


def test_tour_calls_reject_null_handle():
    L = pedsim.lib()
    assert L.sim_step_aco_tour(None, 1, None) == pedsim.SIM_EINVAL
    assert L.sim_attach_tour(None, None, None, None) == pedsim.SIM_EINVAL
    assert L.sim_set_neighbours(None, 8) == pedsim.SIM_EINVAL
    assert L.sim_batch_set_neighbours(None, 8) == pedsim.SIM_EINVAL
    assert L.sim_batch_attach_tour(None, 0, None, None, None) == pedsim.SIM_EINVAL


def test_range_calls_reject_null_handle():
    L = pedsim.lib()
    out = (ctypes.c_int32 * 4)()
    assert L.sim_set_ranges(None, 3, 2) == pedsim.SIM_EINVAL
    assert L.sim_set_range_tiling(None, 64, 32, 2, 512) == pedsim.SIM_EINVAL
    assert L.sim_get_range_tiling(None, out) == pedsim.SIM_EINVAL


def test_noalloc_rejects_bad_arguments_on_host():
    """Refused before any device work: bad parameters, missing planes, an
    unknown or tour mode, negative steps, ACO without pheromone, and a grid
    whose scratch exceeds the static array."""
    L = pedsim.lib()
    st = pedsim.SimStats()
    good = _params()
    bad = _params(W=0)
    assert L.sim_run_noalloc(ctypes.byref(bad), 0, 16, 16, None, 1, None, ctypes.byref(st)) == pedsim.SIM_EINVAL
    assert L.sim_run_noalloc(ctypes.byref(good), 0, None, 16, None, 1, None, ctypes.byref(st)) == pedsim.SIM_EINVAL
    assert L.sim_run_noalloc(ctypes.byref(good), 2, 16, 16, 16, 1, None, ctypes.byref(st)) == pedsim.SIM_EINVAL
    assert L.sim_run_noalloc(ctypes.byref(good), 0, 16, 16, None, -1, None, ctypes.byref(st)) == pedsim.SIM_EINVAL
    assert L.sim_run_noalloc(ctypes.byref(good), 1, 16, 16, None, 1, None, ctypes.byref(st)) == pedsim.SIM_ENOTAU
    big = _params(W=4096, H=2048, cross_a=4, cross_b=4)
    assert L.sim_run_noalloc(ctypes.byref(big), 0, 16, 16, None, 1, None, ctypes.byref(st)) == pedsim.SIM_ESCRATCH
