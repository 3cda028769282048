"""GPU parity: the HIP path against the CPU oracle, bit for bit.

Positions (id plane), occupancy (code plane), counters and both pheromone
planes must be identical (0 ULP): every pheromone value is produced by the
same binary32 operations in the same order on both sides, with no fused
multiply-add and with subnormals kept.
"""
import numpy as np
import pytest

import oracle
from paper_1412_4933_amd import scenarios as S

pytestmark = pytest.mark.gpu


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
    assert s["step"] == st.t


# One explicit tiling per engine (nw, rows, steps per launch, threads): the
# multi-wave engine, the row-lane engine and its streaming form.
ENGINES = {"multi": (1, 32, 2, 512), "rows": (0, 48, 2, 256), "stream": (3, 40, 3, 256)}


def run_both(pedsim, scn, mode, steps, chunks=(1,), tiling=None):
    """Advance GPU and oracle together, comparing after each chunk."""
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
        if c >= 1:
            assert sim.stats()["moved_last"] == moved
        assert_same(sim, st, f"after {done} steps")
    if done < steps:
        sim.step(steps - done, mode)
        moved = st.run(mode, steps - done)
        assert sim.stats()["moved_last"] == moved
        assert_same(sim, st, f"after {steps} steps")
    sim.close()


@pytest.mark.parametrize("mode", [S.MODE_LEM, S.MODE_ACO])
@pytest.mark.parametrize("engine", sorted(ENGINES))
def test_lem_200x100_full_run(pedsim, mode, engine):
    scn = S.lem_200x100()
    scn = S.make_scenario(200, 100, 1000, 1000, band_a=10, seed=1, mode=mode, steps=500,
                          with_tau=True)
    say("200x100", mode, engine)
    run_both(pedsim, scn, mode, 500, chunks=(1, 1, 1, 2, 5, 10, 30, 50, 100), tiling=ENGINES[engine])


@pytest.mark.parametrize("W,H,na,nb,obst,seed", [
    (67, 13, 90, 80, 0.0, 11),     # ragged in both tile dimensions
    (130, 37, 300, 280, 0.07, 12),
    (3, 40, 20, 0, 0.0, 13),       # narrower than a tile and than the halo
    (257, 9, 150, 160, 0.0, 14),
    (64, 8, 0, 0, 0.0, 15),        # no agents at all
])
@pytest.mark.parametrize("mode", [S.MODE_LEM, S.MODE_ACO])
@pytest.mark.parametrize("engine", sorted(ENGINES))
def test_ragged_grids(pedsim, W, H, na, nb, obst, seed, mode, engine):
    band = max(1, min(W // 2, 6))
    scn = S.make_scenario(W, H, na, nb, band_a=band, seed=seed, mode=mode,
                          obstacle_frac=obst, with_tau=True)
    say("ragged", W, H, mode, engine)
    run_both(pedsim, scn, mode, 60, chunks=(1, 1, 3, 10), tiling=ENGINES[engine])


@pytest.mark.parametrize("engine", sorted(ENGINES))
def test_full_grid_nobody_moves(pedsim, engine):
    code = S.wall_frame(70, 11)
    code[1:10, :35] = S.GROUP_A
    code[1:10, 35:] = S.GROUP_B
    scn = S.from_grid(code, seed=4, tau=np.ones((2, 11, 70), np.float32), mode=S.MODE_ACO)
    say("full grid")
    run_both(pedsim, scn, S.MODE_ACO, 5, chunks=(1,), tiling=ENGINES[engine])


@pytest.mark.parametrize("alpha,beta,rho,dtau", [(2, 3, 0.05, 0.5), (0, 1, 1.0, 2.0),
                                                 (3, 0, 0.3, 0.0)])
@pytest.mark.parametrize("engine", sorted(ENGINES))
def test_aco_parameters(pedsim, alpha, beta, rho, dtau, engine):
    scn = S.make_scenario(150, 60, 700, 650, band_a=8, seed=21, mode=S.MODE_ACO,
                          obstacle_frac=0.04, alpha=alpha, beta=beta, rho=rho, dtau=dtau)
    say("aco params", alpha, beta, rho, dtau)
    run_both(pedsim, scn, S.MODE_ACO, 120, chunks=(1, 10, 40), tiling=ENGINES[engine])


@pytest.mark.parametrize("engine", sorted(ENGINES))
def test_aco_subnormal_phase(pedsim, engine):
    """Run through the steps where unvisited cells reach the subnormal range
    and settle at the smallest fixed point (flush-to-zero would differ)."""
    scn = S.make_scenario(96, 24, 60, 60, band_a=4, seed=5, mode=S.MODE_ACO)
    say("subnormal phase")
    run_both(pedsim, scn, S.MODE_ACO, 1000, chunks=(500, 330, 100), tiling=ENGINES[engine])
    sim = pedsim.Sim(scn)
    sim.step(1000)
    _, _, tau = sim.state()
    assert np.any((tau > 0) & (tau < np.float32(2.0 ** -126)))
    sim.close()


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


@pytest.mark.parametrize("mode", [S.MODE_LEM, S.MODE_ACO])
@pytest.mark.parametrize("engine", sorted(ENGINES))
def test_bruteforce_all_4x4_grids_up_to_5_agents(pedsim, mode, engine):
    code, n = _mosaic_all_small_grids(5)
    assert n == 173889
    H, W = code.shape
    rng = np.random.default_rng(9)
    tau = rng.uniform(0.0, 2.0, size=(2, H, W)).astype(np.float32)
    scn = S.from_grid(code, seed=77, tau=tau, mode=mode)
    say("bruteforce", mode, W, H, engine)
    run_both(pedsim, scn, mode, 3, chunks=(1, 1, 1), tiling=ENGINES[engine])


@pytest.mark.parametrize("tiling", [None, ENGINES["rows"]])
def test_aco_1024x512_full_run(pedsim, tiling):
    """The 100K-agent ACO workload over all 2,000 steps."""
    scn = S.aco_1024x512()
    say("aco 1024x512 x2000", tiling)
    run_both(pedsim, scn, S.MODE_ACO, 2000, chunks=(1, 1, 8, 90, 400), tiling=tiling)


@pytest.mark.parametrize("mode", [S.MODE_LEM, S.MODE_ACO])
def test_stress_4096x2048_first_steps(pedsim, mode):
    """Full-size stress grid in the benchmark's launch configuration:
    bit-exact after 15 and after 100 steps, then invariants that hold at any
    size over a longer GPU run."""
    scn = S.stress_4096x2048(mode)
    say("stress 4096x2048", mode)
    sim = pedsim.Sim(scn)
    st = oracle.State.from_scenario(scn)
    for c in (1, 4, 10):
        sim.step(c, mode)
        st.run(mode, c)
    assert_same(sim, st, "stress after 15 steps")
    sim.step(85, mode)
    st.run(mode, 85)
    assert_same(sim, st, "stress after 100 steps")
    sim.step(300, mode)
    code, ids, tau = sim.state()
    assert np.array_equal(code == S.WALL, scn.code == S.WALL)
    occ = (code == 1) | (code == 2)
    assert np.array_equal(occ, ids != 0)
    assert np.count_nonzero(code == 1) == scn.n_a and np.count_nonzero(code == 2) == scn.n_b
    assert np.array_equal(np.sort(ids[occ]), np.arange(1, scn.agents + 1, dtype=np.uint32))
    assert np.all(tau >= 0) and np.all(np.isfinite(tau))
    sim.close()


def test_checkpoint_resume_is_exact(pedsim):
    scn = S.make_scenario(300, 80, 2000, 2000, band_a=12, seed=8, mode=S.MODE_ACO,
                          obstacle_frac=0.03)
    say("checkpoint")
    full = pedsim.Sim(scn)
    full.step(70)
    want = full.state()
    first = pedsim.Sim(scn)
    first.step(30)
    code, ids, tau = first.state()
    resumed_scn = scn.copy()
    resumed_scn.code, resumed_scn.ids, resumed_scn.tau = code, ids, tau
    second = pedsim.Sim(resumed_scn, step0=30)
    second.step(40)
    got = second.state()
    for w, g in zip(want, got):
        assert np.array_equal(w.view(np.uint8), g.view(np.uint8))
    assert second.stats()["step"] == 70
    for s in (full, first, second):
        s.close()


def test_result_independent_of_stream(pedsim):
    import torch
    scn = S.make_scenario(200, 64, 1500, 1500, band_a=12, seed=6, mode=S.MODE_ACO)
    say("streams")
    a = pedsim.Sim(scn)
    a.step(50)
    s = torch.cuda.Stream()
    b = pedsim.Sim(scn, stream=s)
    b.step(50)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
    a.close()
    b.close()


@pytest.mark.parametrize("what", ["dup_id", "bad_code", "id_on_empty", "missing_id", "neg_tau",
                                  "nan_tau", "id_too_big"])
def test_invalid_initial_state_rejected(pedsim, what):
    scn = S.make_scenario(64, 16, 40, 40, band_a=4, seed=2, mode=S.MODE_ACO)
    ys, xs = np.nonzero(scn.ids)
    if what == "dup_id":
        scn.ids[ys[1], xs[1]] = scn.ids[ys[0], xs[0]]
    elif what == "bad_code":
        scn.code[5, 30] = 7
    elif what == "id_on_empty":
        scn.ids[5, 30] = 3
    elif what == "missing_id":
        scn.ids[ys[0], xs[0]] = 0
    elif what == "neg_tau":
        scn.tau[1, 3, 3] = -1.0
    elif what == "nan_tau":
        scn.tau[0, 4, 4] = np.nan
    elif what == "id_too_big":
        scn.ids[ys[0], xs[0]] = 1000
    say("invalid state", what)
    with pytest.raises(pedsim.SimError) as e:
        pedsim.Sim(scn)
    assert e.value.code == pedsim.SIM_ESTATE


def test_aco_without_pheromone_refused(pedsim):
    scn = S.make_scenario(64, 16, 40, 40, band_a=4, seed=2, mode=S.MODE_LEM, with_tau=False)
    sim = pedsim.Sim(scn)
    with pytest.raises(pedsim.SimError) as e:
        sim.step(1, S.MODE_ACO)
    assert e.value.code == pedsim.SIM_ENOTAU
    sim.step(3, S.MODE_LEM)
    sim.close()


TILINGS = [(1, 32, 1, 256), (1, 48, 2, 512), (1, 64, 3, 1024), (2, 64, 2, 1024), (2, 64, 4, 1024),
           (1, 96, 2, 128), (1, 32, 1, 64),
           # row-lane engine: regions of 64 columns, at most 64 rows
           (0, 64, 1, 64), (0, 32, 1, 128), (0, 48, 2, 256), (0, 64, 3, 256), (0, 64, 2, 512),
           (0, 40, 4, 512), (0, 64, 8, 256),
           # streaming row-lane engine
           (3, 48, 2, 256), (3, 64, 3, 64), (3, 32, 1, 512), (3, 56, 4, 128)]


@pytest.mark.parametrize("mode", [S.MODE_LEM, S.MODE_ACO])
def test_results_do_not_depend_on_tiling(pedsim, mode):
    """Every allowed tile shape, region height, steps per launch and
    workgroup size gives the oracle's result bit for bit."""
    scn = S.make_scenario(333, 150, 2500, 2400, band_a=14, seed=19, mode=mode,
                          obstacle_frac=0.04, with_tau=True)
    st = oracle.State.from_scenario(scn)
    st.run(mode, 37)
    ran = 0
    for tl in TILINGS:
        sim = pedsim.Sim(scn)
        try:
            sim.set_tiling(mode, *tl)
        except pedsim.SimError:
            sim.close()
            continue  # shape not allowed on this device (LDS) or too small
        say("tiling", mode, tl)
        sim.step(10, mode)
        sim.step(27, mode)
        assert_same(sim, st, f"tiling {tl}")
        sim.close()
        ran += 1
    assert ran >= 8
