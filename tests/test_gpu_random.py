"""Seeded random configurations: grid shape, population, obstacles, mode
(LEM, ACO, tour variant), candidate set, ACO parameters, initial tour
lengths and tiling are drawn at random; every case must match the oracle
bit for bit after a few launches."""
import numpy as np
import pytest

import oracle
from paper_1412_4933_amd import scenarios as S

pytestmark = pytest.mark.gpu

ROW_TILINGS = [(0, 32, 1, 64), (0, 40, 2, 256), (0, 48, 3, 512), (0, 56, 4, 512), (0, 64, 2, 128),
               (0, 52, 4, 512), (0, 64, 6, 512)]
OTHER_TILINGS = [(1, 32, 1, 256), (1, 32, 2, 512), (2, 48, 2, 1024), (3, 48, 2, 256), (3, 40, 3, 128)]


def draw_case(i):
    rng = np.random.default_rng(9000 + i)
    W = int(rng.integers(3, 400))
    H = int(rng.integers(3, 160))
    neighbours = 8 if rng.random() < 0.4 else 5
    mode = int(rng.choice([S.MODE_LEM, S.MODE_ACO, S.MODE_ACO_TOUR]))
    cap = max(0, (W // 4) * (H - 2))
    N = int(rng.integers(0, min(cap, 4000) + 1)) if cap else 0
    obst = float(rng.choice([0.0, 0.0, 0.03, 0.08]))
    kw = dict(alpha=int(rng.integers(0, 4)), beta=int(rng.integers(0, 4)),
              rho=float(rng.choice([0.05, 0.1, 0.5, 0.9, 1.0])), dtau=float(rng.choice([0.0, 0.5, 1.0, 2.0])))
    try:
        scn = S.make_scenario(W, H, N // 2, N - N // 2, band_a=max(1, W // 8), seed=int(rng.integers(1, 1 << 40)),
                              mode=mode, obstacle_frac=obst, with_tau=True, neighbours=neighbours, **kw)
    except ValueError:  # the obstacles left no room for the population
        scn = S.make_scenario(W, H, 0, 0, band_a=1, seed=1, mode=mode, with_tau=True,
                              neighbours=neighbours, **kw)
    if mode == S.MODE_ACO_TOUR and rng.random() < 0.5:
        scn.tour = (rng.random(scn.agents) * 20).astype(np.float32)
    pool = ROW_TILINGS if (neighbours == 8 or mode == S.MODE_ACO_TOUR) else ROW_TILINGS + OTHER_TILINGS
    tiling = pool[int(rng.integers(0, len(pool)))]
    steps = [int(v) for v in rng.integers(1, 12, size=3)]
    return scn, tiling, steps


@pytest.mark.parametrize("i", range(120))
def test_random_configuration_matches_oracle(i):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_4933_amd import pedsim
    scn, tiling, steps = draw_case(i)
    print(f"[gpu-case] random {i}: {scn.W}x{scn.H} agents {scn.agents} mode {scn.mode} "
          f"neighbours {scn.neighbours} tiling {tiling} steps {steps}", flush=True)
    sim = pedsim.Sim(scn)
    try:
        sim.set_tiling(scn.mode, *tiling)
    except pedsim.SimError:
        pass  # shape too large for this grid's tile bound: keep the default
    st = oracle.State.from_scenario(scn)
    for k in steps:
        sim.step(k, scn.mode)
        moved = st.run(scn.mode, k)
        code, ids, tau = sim.state()
        assert np.array_equal(code, st.code) and np.array_equal(ids, st.ids)
        if scn.mode != S.MODE_LEM:
            assert np.array_equal(tau.view(np.uint32), st.tau.view(np.uint32))
        if scn.mode == S.MODE_ACO_TOUR and scn.agents:
            assert np.array_equal(sim.tour_lengths().view(np.uint32), st.tour.view(np.uint32))
        s = sim.stats()
        a, b, ca, cb = st.counts()
        assert (s["agents_a"], s["agents_b"], s["crossed_a"], s["crossed_b"], s["moved_last"]) == (a, b, ca, cb, moved)
    sim.close()
