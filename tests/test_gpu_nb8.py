"""GPU parity of the eight-neighbour candidate set (backward cells ranked
last): code, ids, both pheromone planes, tour lengths and counters identical
to the oracle's, bit for bit, for LEM, ACO and the tour variant across
tilings, ragged grids, every 4x4 grid with up to five agents, and the
population sweep's shape."""
import numpy as np
import pytest

import oracle
from paper_1412_4933_amd import scenarios as S

pytestmark = pytest.mark.gpu

MODES = [S.MODE_LEM, S.MODE_ACO, S.MODE_ACO_TOUR]


@pytest.fixture(scope="module")
def pedsim():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_4933_amd import pedsim as P
    P.lib()
    return P


def say(*a):
    print("[gpu-case]", *a, flush=True)


def assert_same(sim, st, mode, what=""):
    code, ids, tau = sim.state()
    assert np.array_equal(code, st.code), f"code differs {what}: {np.argwhere(code != st.code)[:5]}"
    assert np.array_equal(ids, st.ids), f"ids differ {what}: {np.argwhere(ids != st.ids)[:5]}"
    if mode != S.MODE_LEM:
        bad = tau.view(np.uint32) != st.tau.view(np.uint32)
        assert not bad.any(), f"pheromone differs {what}: {np.argwhere(bad)[:5]}"
    if mode == S.MODE_ACO_TOUR:
        tour = sim.tour_lengths()
        assert np.array_equal(tour.view(np.uint32), st.tour.view(np.uint32)), f"tour differs {what}"
    s = sim.stats()
    a, b, ca, cb = st.counts()
    assert (s["agents_a"], s["agents_b"], s["crossed_a"], s["crossed_b"]) == (a, b, ca, cb), what
    assert s["step"] == st.t


def run_both(pedsim, scn, mode, steps, chunks=(1,), tiling=None):
    sim = pedsim.Sim(scn)
    if tiling is not None:
        sim.set_tiling(mode, *tiling)
    st = oracle.State.from_scenario(scn)
    done = 0
    for c in chunks:
        if done + c > steps:
            break
        sim.step(c, mode)
        moved = st.run(mode, c)
        done += c
        assert sim.stats()["moved_last"] == moved
        assert_same(sim, st, mode, f"after {done} steps")
    if done < steps:
        sim.step(steps - done, mode)
        moved = st.run(mode, steps - done)
        assert sim.stats()["moved_last"] == moved
        assert_same(sim, st, mode, f"after {steps} steps")
    sim.close()


TILINGS = [None, (0, 48, 2, 256), (0, 64, 8, 256), (0, 32, 1, 128), (0, 48, 3, 512), (0, 64, 1, 64)]


@pytest.mark.parametrize("tiling", TILINGS)
@pytest.mark.parametrize("mode", MODES)
def test_nb8_200x100_full_run(pedsim, mode, tiling):
    scn = S.make_scenario(200, 100, 1000, 1000, band_a=10, seed=1, mode=mode, steps=500,
                          with_tau=True, neighbours=8)
    say("nb8 200x100", mode, tiling)
    run_both(pedsim, scn, mode, 500, chunks=(1, 1, 1, 2, 5, 10, 30, 50, 100), tiling=tiling)


@pytest.mark.parametrize("W,H,na,nb,obst,seed", [
    (67, 13, 90, 80, 0.0, 11),
    (130, 37, 300, 280, 0.07, 12),
    (3, 40, 20, 0, 0.0, 13),
    (257, 9, 150, 160, 0.0, 14),
    (64, 8, 0, 0, 0.0, 15),
])
@pytest.mark.parametrize("mode", MODES)
def test_nb8_ragged_grids(pedsim, W, H, na, nb, obst, seed, mode):
    band = max(1, min(W // 2, 6))
    scn = S.make_scenario(W, H, na, nb, band_a=band, seed=seed, mode=mode, obstacle_frac=obst,
                          with_tau=True, neighbours=8)
    say("nb8 ragged", W, H, mode)
    run_both(pedsim, scn, mode, 60, chunks=(1, 1, 3, 10), tiling=(0, 40, 3, 512))


@pytest.mark.parametrize("alpha,beta,rho,dtau", [(2, 3, 0.05, 0.5), (0, 1, 1.0, 2.0), (1, 2, 0.9, 1.0)])
@pytest.mark.parametrize("mode", [S.MODE_ACO, S.MODE_ACO_TOUR])
def test_nb8_aco_parameters(pedsim, alpha, beta, rho, dtau, mode):
    scn = S.make_scenario(150, 60, 700, 650, band_a=8, seed=21, mode=mode, obstacle_frac=0.04,
                          alpha=alpha, beta=beta, rho=rho, dtau=dtau, neighbours=8)
    say("nb8 aco params", mode, alpha, beta, rho, dtau)
    run_both(pedsim, scn, mode, 120, chunks=(1, 10, 40))


def _mosaic_all_small_grids(max_agents):
    from itertools import combinations, product
    grids = []
    for m in range(max_agents + 1):
        for pos in combinations(range(16), m):
            for groups in product((1, 2), repeat=m):
                g = np.zeros(16, np.uint8)
                g[list(pos)] = groups
                grids.append(g.reshape(4, 4))
    per_row = 512
    rows = (len(grids) + per_row - 1) // per_row
    code = np.full((rows * 5 + 1, per_row * 5 + 1), S.WALL, np.uint8)
    for i, g in enumerate(grids):
        oy, ox = 1 + (i // per_row) * 5, 1 + (i % per_row) * 5
        code[oy:oy + 4, ox:ox + 4] = g
    return code, len(grids)


@pytest.mark.parametrize("mode", MODES)
def test_nb8_bruteforce_all_4x4_grids_up_to_5_agents(pedsim, mode):
    code, n = _mosaic_all_small_grids(5)
    assert n == 173889
    H, W = code.shape
    rng = np.random.default_rng(10)
    tau = rng.uniform(0.0, 2.0, size=(2, H, W)).astype(np.float32)
    scn = S.from_grid(code, seed=78, tau=tau, mode=mode, neighbours=8)
    say("nb8 bruteforce", mode, W, H)
    run_both(pedsim, scn, mode, 3, chunks=(1, 1, 1))


@pytest.mark.parametrize("mode", [S.MODE_LEM, S.MODE_ACO])
def test_nb8_sweep_shape(pedsim, mode):
    """480 x 480 with 2,560 agents in 3-column bands (the sweep's lowest
    density): the fronts meet and pass within the run."""
    scn = S.paper_sweep([1], repeats=1, steps=600, modes=(mode,), neighbours=8)[0]
    say("nb8 sweep shape", mode)
    run_both(pedsim, scn, mode, 600, chunks=(100, 200))


def test_nb8_errors(pedsim):
    scn = S.make_scenario(64, 32, 100, 100, band_a=6, seed=3, mode=S.MODE_ACO, neighbours=8)
    sim = pedsim.Sim(scn)
    for nw in (1, 2, 3):  # only the row-lane engine with the pheromone in LDS
        with pytest.raises(pedsim.SimError) as e:
            sim.set_tiling(S.MODE_ACO, nw, 32, 1, 256)
        assert e.value.code == pedsim.SIM_EINVAL
    with pytest.raises(pedsim.SimError) as e:
        pedsim.sim_set_neighbours(sim.h, 7)
    assert e.value.code == pedsim.SIM_EINVAL
    assert sim.tiling(S.MODE_ACO)[0] == 0
    sim.close()


@pytest.mark.parametrize("mode", [S.MODE_ACO, S.MODE_ACO_TOUR])
def test_nb8_1024x512_default_tiling(pedsim, mode):
    """The benchmark's eight-neighbour workload in its launch configuration."""
    scn = S.aco_nb8_1024x512()
    scn.mode = mode
    say("nb8 1024x512", mode)
    run_both(pedsim, scn, mode, 200, chunks=(1, 7, 40))
