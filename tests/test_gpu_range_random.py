"""Seeded random configurations of the range model (larger scanning and moving
ranges, the paper's future work, Sec. VII): grid shape, population, obstacles,
mode, scanning and moving range, ACO parameters and the range kernel's launch
shape (tile, steps per launch, threads) are drawn at random; every case must
match the oracle's range step bit for bit after a few calls of random
length."""
import numpy as np
import pytest

import oracle
from paper_1412_4933_amd import scenarios as S

pytestmark = pytest.mark.gpu

SHAPES = [(16, 8), (32, 8), (32, 16), (48, 24), (64, 16), (64, 32), (96, 8), (128, 16)]


def draw_case(i):
    rng = np.random.default_rng(7700 + i)
    W = int(rng.integers(3, 300))
    H = int(rng.integers(3, 120))
    mode = int(rng.choice([S.MODE_LEM, S.MODE_ACO]))
    scan = int(rng.integers(1, 9))
    move = int(rng.integers(1, scan + 1))
    cap = max(0, (W // 4) * (H - 2))
    N = int(rng.integers(0, min(cap, 3000) + 1)) if cap else 0
    obst = float(rng.choice([0.0, 0.0, 0.04, 0.1]))
    kw = dict(alpha=int(rng.integers(0, 4)), beta=int(rng.integers(0, 5)),
              rho=float(rng.choice([0.05, 0.1, 0.5, 1.0])), dtau=float(rng.choice([0.0, 0.5, 1.0, 2.0])))
    try:
        scn = S.make_scenario(W, H, N // 2, N - N // 2, band_a=max(1, W // 8), seed=int(rng.integers(1, 1 << 40)),
                              mode=mode, obstacle_frac=obst, with_tau=True, **kw)
    except ValueError:  # the obstacles left no room for the population
        scn = S.make_scenario(W, H, 0, 0, band_a=1, seed=1, mode=mode, with_tau=True, **kw)
    cols, rows = SHAPES[int(rng.integers(0, len(SHAPES)))]
    tiling = (cols, rows, int(rng.integers(1, 5)), int(rng.choice([64, 128, 256, 512])))
    steps = [int(v) for v in rng.integers(1, 10, size=3)]
    return scn, (scan, move), tiling, steps


@pytest.mark.parametrize("i", range(60))
def test_random_range_configuration_matches_oracle(i):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_4933_amd import pedsim
    scn, ranges, tiling, steps = draw_case(i)
    sim = pedsim.Sim(scn, autotune=False)
    sim.set_ranges(*ranges)
    try:
        sim.set_range_tiling(*tiling)
    except pedsim.SimError:
        pass  # does not fit the LDS with these ranges: keep the default shape
    print(f"[gpu-case] range random {i}: {scn.W}x{scn.H} agents {scn.n_a + scn.n_b} mode {scn.mode} "
          f"ranges {ranges} tiling {sim.range_tiling()} steps {steps}", flush=True)
    st = oracle.State.from_scenario(scn)
    st.ranges = ranges
    for k in steps:
        sim.step(k, scn.mode)
        moved = st.run(scn.mode, k)
        code, ids, tau = sim.state()
        assert np.array_equal(code, st.code) and np.array_equal(ids, st.ids)
        if scn.mode != S.MODE_LEM:
            assert np.array_equal(tau.view(np.uint32), st.tau.view(np.uint32))
        s = sim.stats()
        a, b, ca, cb = st.counts()
        assert (s["agents_a"], s["agents_b"], s["crossed_a"], s["crossed_b"], s["moved_last"]) == (a, b, ca, cb, moved)
    sim.close()
