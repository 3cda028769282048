"""Row-lane launches on grids with more tiles than the device runs at once deal
out their tiles in the order the previous launch recorded (the tiles that held
agents first). The order decides only which workgroup takes which tile, so the
results must stay identical to the oracle's: through many launches, when the
tiling or the mode changes (a new tile grid starts again from row-major order),
with the eight-neighbour set, and on the 4096x2048 workload's tiling."""
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


def same(sim, st, what):
    code, ids, tau = sim.state()
    assert np.array_equal(code, st.code), what
    assert np.array_equal(ids, st.ids), what
    if tau is not None and st.tau is not None:
        assert np.array_equal(tau.view(np.uint32), st.tau.view(np.uint32)), what
    s = sim.stats()
    a, b, ca, cb = st.counts()
    assert (s["agents_a"], s["agents_b"], s["crossed_a"], s["crossed_b"]) == (a, b, ca, cb), what


# Regions of 56 or 64 rows with six steps per launch hold one ACO workgroup
# (two LEM ones) per compute unit: the 784 and 1,092 tiles of 768x768 are more
# than the device runs at once. Tiling and mode changes start a new order.
PLAN = [(S.MODE_ACO, (0, 64, 6, 512), 30), (S.MODE_ACO, (0, 56, 6, 512), 12), (S.MODE_LEM, (0, 64, 6, 512), 12),
        (S.MODE_ACO, (0, 64, 6, 512), 24), (S.MODE_ACO, (0, 64, 6, 512), 6)]


@pytest.mark.parametrize("neighbours", [5, 8])
def test_tile_order_keeps_results(pedsim, neighbours):
    scn = S.make_scenario(768, 768, 16000, 16000, band_a=48, seed=91, mode=S.MODE_ACO, obstacle_frac=0.02,
                          with_tau=True, neighbours=neighbours)
    sim = pedsim.Sim(scn, autotune=False)
    st = oracle.State.from_scenario(scn, threads=THREADS)
    done = 0
    for mode, tiling, n in PLAN:
        sim.set_tiling(mode, *tiling)
        print(f"[gpu-case] tile order: nb{neighbours} mode {mode} tiling {tiling} steps {done}..{done + n}",
              flush=True)
        sim.step(n, mode)
        moved = st.run(mode, n)
        done += n
        assert sim.stats()["moved_last"] == moved
        same(sim, st, f"after {done} steps (mode {mode}, tiling {tiling})")
    sim.close()


def test_tile_order_on_the_4096x2048_tiling(pedsim):
    scn = S.stress_4096x2048(S.MODE_ACO)
    sim = pedsim.Sim(scn, autotune=False)
    sim.set_tiling(S.MODE_ACO, 3, 62, 3, 256)
    st = oracle.State.from_scenario(scn, threads=THREADS)
    for n in (12, 9):
        print(f"[gpu-case] tile order: 4096x2048 ACO (3, 62, 3, 256), {n} steps", flush=True)
        sim.step(n, S.MODE_ACO)
        st.run(S.MODE_ACO, n)
    same(sim, st, "4096x2048 after 21 steps")
    sim.close()
