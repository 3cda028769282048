"""GPU parity of larger scanning and moving ranges (the paper's future work,
Sec. VII): the range kernel against the oracle's range step, bit for bit on
codes, ids, both pheromone planes and the counters.

Cases: every (scan, move) pair family from (1, 1) to (8, 8) on a ragged grid
with obstacles, LEM and ACO, in chunks of odd and even length; (1, 1) against
the oracle's base step as well; ragged and degenerate grids (narrower than a
tile, a single free row, no agents, a full grid); every launch shape family;
a mosaic of small walled-off grids crowded enough that most landing cells are
contested; ACO parameter variants; checkpoint/resume; and the 1024x512
workload with ranges (4, 2) through all 2,000 steps against the all-core
oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1412_4933_amd import scenarios as S

pytestmark = pytest.mark.gpu

THREADS = oracle.cpu_threads()


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


def assert_same(sim, st, what=""):
    code, ids, tau = sim.state()
    assert np.array_equal(code, st.code), f"code differs {what}: {np.argwhere(code != st.code)[:5]}"
    assert np.array_equal(ids, st.ids), f"ids differ {what}: {np.argwhere(ids != st.ids)[:5]}"
    if st.tau is not None and tau is not None:
        bad = tau.view(np.uint32) != st.tau.view(np.uint32)
        assert not bad.any(), f"pheromone differs {what}: {np.argwhere(bad)[:5]}"
    s = sim.stats()
    a, b, ca, cb = st.counts()
    assert (s["agents_a"], s["agents_b"], s["crossed_a"], s["crossed_b"]) == (a, b, ca, cb), what
    assert s["step"] == st.t, what
    return s


def run_both(pedsim, scn, mode, ranges, chunks, tiling=None, base_oracle=False):
    """Advance the GPU (range kernel) and the oracle together, comparing after
    every chunk; base_oracle=True steps the oracle's base model instead."""
    sim = pedsim.Sim(scn)
    sim.set_ranges(*ranges)
    if tiling is not None:
        sim.set_range_tiling(*tiling)
    st = oracle.State.from_scenario(scn, threads=THREADS)
    st.ranges = None if base_oracle else ranges
    done = 0
    for c in chunks:
        sim.step(c, mode)
        moved = st.run(mode, c)
        done += c
        s = assert_same(sim, st, f"{ranges} after {done} steps")
        if c > 0:
            assert s["moved_last"] == moved, f"moved after {done} steps"
    sim.close()
    return st


PAIRS = [(1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (3, 3), (4, 2), (4, 4), (5, 3), (6, 6), (7, 2),
         (8, 1), (8, 5), (8, 8)]


@pytest.mark.parametrize("ranges", PAIRS)
@pytest.mark.parametrize("mode", [S.MODE_LEM, S.MODE_ACO])
def test_range_pairs_match_oracle(pedsim, mode, ranges):
    scn = S.make_scenario(203, 77, 1400, 1300, band_a=12, seed=40 + ranges[0] * 8 + ranges[1], mode=mode,
                          obstacle_frac=0.05, with_tau=True)
    say("range pair", ranges, "mode", mode)
    run_both(pedsim, scn, mode, ranges, chunks=(1, 2, 5, 12, 33, 7))


@pytest.mark.parametrize("mode", [S.MODE_LEM, S.MODE_ACO])
def test_range_one_one_is_the_base_step(pedsim, mode):
    scn = S.make_scenario(150, 50, 900, 900, band_a=9, seed=77, mode=mode, obstacle_frac=0.04,
                          with_tau=True)
    say("range (1,1) vs base oracle, mode", mode)
    run_both(pedsim, scn, mode, (1, 1), chunks=(3, 20, 17), base_oracle=True)


# launch shapes (interior cols, rows, steps per launch, threads); the longest
# ranges need the most LDS per cell, so they get the smaller shapes
TILINGS = [((3, 2), t) for t in [(16, 8, 1, 64), (32, 8, 1, 128), (64, 16, 1, 256), (64, 32, 1, 512),
                                   (128, 24, 1, 256), (48, 40, 1, 192), (256, 8, 1, 512), (64, 64, 1, 256),
                                   (64, 32, 2, 512), (64, 16, 3, 512), (32, 16, 4, 256), (16, 8, 4, 64),
                                   (48, 24, 2, 320)]] + \
          [((8, 8), t) for t in [(16, 8, 1, 64), (32, 8, 1, 128), (64, 16, 1, 256), (32, 16, 1, 512),
                                   (96, 8, 1, 256), (40, 24, 1, 192), (24, 24, 1, 320), (16, 16, 1, 128)]] + \
          [((1, 1), t) for t in [(64, 32, 4, 512), (32, 8, 3, 128)]] + \
          [((4, 2), t) for t in [(64, 32, 2, 512), (64, 24, 2, 256)]]


@pytest.mark.parametrize("ranges,tiling", TILINGS)
def test_range_tilings(pedsim, tiling, ranges):
    scn = S.make_scenario(333, 95, 2500, 2400, band_a=14, seed=5, mode=S.MODE_ACO, obstacle_frac=0.06)
    say("range tiling", tiling, ranges)
    run_both(pedsim, scn, S.MODE_ACO, ranges, chunks=(1, 6, 9, 2, 5), tiling=tiling)


@pytest.mark.parametrize("shape", [(3, 3), (5, 4), (7, 3), (1, 5), (9, 2), (65, 9), (64, 8), (130, 17)])
@pytest.mark.parametrize("ranges", [(2, 2), (8, 3)])
def test_range_ragged_grids(pedsim, shape, ranges):
    W, H = shape
    rng = np.random.default_rng(W * 100 + H)
    code = np.zeros((H, W), np.uint8)
    if H >= 3:
        code[0, :] = S.WALL
        code[-1, :] = S.WALL
    free = np.argwhere(code == S.EMPTY)
    if len(free):
        pick = rng.choice(len(free), size=max(1, len(free) // 2), replace=False)
        for i, (y, x) in enumerate(free[pick]):
            code[y, x] = S.GROUP_A if i % 2 == 0 else S.GROUP_B
    tau = np.full((2, H, W), np.float32(1.0), np.float32)
    scn = S.from_grid(code, seed=3, tau=tau, mode=S.MODE_ACO)
    say("range ragged", shape, ranges)
    run_both(pedsim, scn, S.MODE_ACO, ranges, chunks=(1, 4, 3))


def test_range_no_agents_and_full_grid(pedsim):
    empty = S.wall_frame(90, 20)
    tau = np.full((2, 20, 90), np.float32(0.5), np.float32)
    run_both(pedsim, S.from_grid(empty, tau=tau, mode=S.MODE_ACO), S.MODE_ACO, (4, 3), chunks=(5, 2))
    full = S.wall_frame(70, 12)
    full[1:-1, :35] = S.GROUP_A
    full[1:-1, 35:] = S.GROUP_B
    tau = np.full((2, 12, 70), np.float32(2.0), np.float32)
    run_both(pedsim, S.from_grid(full, tau=tau, mode=S.MODE_ACO), S.MODE_ACO, (5, 5), chunks=(3, 4))


def _mosaic(seed, cells=6, reps_x=40, reps_y=20, fill=0.55):
    """Many small grids separated by wall lines: agents see and move only
    inside their own sub-grid, so each one is an independent crowded case."""
    rng = np.random.default_rng(seed)
    W, H = reps_x * (cells + 1) + 1, reps_y * (cells + 1) + 1
    code = np.full((H, W), S.WALL, np.uint8)
    for j in range(reps_y):
        for i in range(reps_x):
            y0, x0 = 1 + j * (cells + 1), 1 + i * (cells + 1)
            sub = rng.random((cells, cells))
            blk = np.where(sub < fill / 2, S.GROUP_A, np.where(sub < fill, S.GROUP_B, S.EMPTY))
            code[y0:y0 + cells, x0:x0 + cells] = blk
    return code


@pytest.mark.parametrize("ranges", [(2, 2), (4, 3), (6, 6)])
@pytest.mark.parametrize("mode", [S.MODE_LEM, S.MODE_ACO])
def test_range_contested_mosaic(pedsim, mode, ranges):
    code = _mosaic(11 + ranges[1])
    H, W = code.shape
    rng = np.random.default_rng(5)
    tau = rng.uniform(0.0, 3.0, size=(2, H, W)).astype(np.float32)
    scn = S.from_grid(code, seed=9, tau=tau, mode=mode)
    say("range mosaic", ranges, "mode", mode, f"{W}x{H}", scn.agents, "agents")
    run_both(pedsim, scn, mode, ranges, chunks=(1, 1, 2, 4, 8))


@pytest.mark.parametrize("alpha,beta,rho,dtau", [(2, 3, 0.25, 0.5), (0, 1, 1.0, 2.0), (3, 0, 0.05, 0.0),
                                                 (1, 8, 0.5, 3.0)])
def test_range_aco_parameters(pedsim, alpha, beta, rho, dtau):
    scn = S.make_scenario(180, 60, 1200, 1200, band_a=12, seed=8, mode=S.MODE_ACO, obstacle_frac=0.03,
                          alpha=alpha, beta=beta, rho=rho, dtau=dtau)
    say("range ACO params", alpha, beta, rho, dtau)
    run_both(pedsim, scn, S.MODE_ACO, (5, 2), chunks=(2, 15, 8))


def test_range_checkpoint_resume(pedsim):
    scn = S.make_scenario(140, 40, 700, 700, band_a=8, seed=12, mode=S.MODE_ACO)
    sim = pedsim.Sim(scn)
    sim.set_ranges(4, 2)
    sim.step(13)
    code, ids, tau = sim.state()
    t = sim.stats()["step"]
    sim.close()
    resumed = scn.copy()
    resumed.code, resumed.ids, resumed.tau = code, ids, tau
    sim2 = pedsim.Sim(resumed, step0=t)
    sim2.set_ranges(4, 2)
    sim2.step(20)
    st = oracle.State.from_scenario(scn)
    st.ranges = (4, 2)
    st.run(S.MODE_ACO, 33)
    assert_same(sim2, st, "after resume")
    sim2.close()


def test_range_switch_back_to_base(pedsim):
    scn = S.make_scenario(128, 40, 600, 600, band_a=8, seed=14, mode=S.MODE_ACO)
    sim = pedsim.Sim(scn)
    st = oracle.State.from_scenario(scn)
    sim.set_ranges(3, 2)
    st.ranges = (3, 2)
    sim.step(9)
    st.run(S.MODE_ACO, 9)
    sim.set_ranges(0, 0)
    st.ranges = None
    sim.step(10)
    st.run(S.MODE_ACO, 10)
    assert_same(sim, st, "ranges then base")
    sim.close()


def test_range_rejections(pedsim):
    scn = S.make_scenario(64, 20, 100, 100, band_a=4, seed=1, mode=S.MODE_ACO)
    sim = pedsim.Sim(scn)
    for bad in ((9, 1), (2, 3), (0, 1), (1, 0), (-1, -1)):
        with pytest.raises(pedsim.SimError):
            sim.set_ranges(*bad)
    sim.set_ranges(3, 2)
    with pytest.raises(pedsim.SimError):
        pedsim.sim_set_neighbours(sim.h, 8)
    with pytest.raises(pedsim.SimError):
        sim.set_range_tiling(8, 8, 1, 256)
    with pytest.raises(pedsim.SimError):
        sim.set_range_tiling(64, 32, 1, 100)
    with pytest.raises(pedsim.SimError):
        sim.set_range_tiling(64, 32, 5, 256)
    with pytest.raises(pedsim.SimError):
        sim.set_range_tiling(64, 32, 0, 256)
    sim.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", [S.MODE_ACO, S.MODE_LEM])
def test_range_1024x512_all_2000_steps(pedsim, mode):
    scn = S.range_1024x512(mode)
    say("range 1024x512 x2000, mode", mode, "ranges", scn.ranges, "oracle threads", THREADS)
    run_both(pedsim, scn, mode, scn.ranges, chunks=(1, 99, 400, 1500))
