"""GPU parity of the tour variant (tour matrix and eq. 5's deposit): code,
ids, both pheromone planes and the tour matrix identical to the oracle's,
bit for bit, across tilings, ragged grids, parameters, initial tour lengths
and launch splits."""
import numpy as np
import pytest

import oracle
from paper_1412_4933_amd import scenarios as S

pytestmark = pytest.mark.gpu

TOUR = S.MODE_ACO_TOUR


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
    bad = tau.view(np.uint32) != st.tau.view(np.uint32)
    assert not bad.any(), f"pheromone differs {what}: {np.argwhere(bad)[:5]}"
    tour = sim.tour_lengths()
    badt = tour.view(np.uint32) != st.tour.view(np.uint32)
    assert not badt.any(), f"tour lengths differ {what}: {np.nonzero(badt)[0][:5]}"
    s = sim.stats()
    a, b, ca, cb = st.counts()
    assert (s["agents_a"], s["agents_b"], s["crossed_a"], s["crossed_b"]) == (a, b, ca, cb), what
    assert s["step"] == st.t


def run_both(pedsim, scn, steps, chunks=(1,), tiling=None):
    sim = pedsim.Sim(scn)
    if tiling is not None:
        sim.set_tiling(TOUR, *tiling)
    st = oracle.State.from_scenario(scn)
    done = 0
    for c in chunks:
        if done + c > steps:
            break
        sim.step(c, TOUR)
        moved = st.run(TOUR, c)
        done += c
        assert sim.stats()["moved_last"] == moved
        assert_same(sim, st, f"after {done} steps")
    if done < steps:
        sim.step(steps - done, TOUR)
        moved = st.run(TOUR, steps - done)
        assert sim.stats()["moved_last"] == moved
        assert_same(sim, st, f"after {steps} steps")
    sim.close()


TILINGS = [None, (0, 48, 2, 256), (0, 64, 8, 256), (0, 32, 1, 128), (0, 56, 4, 512),
           (0, 40, 3, 512), (0, 64, 1, 64)]


@pytest.mark.parametrize("tiling", TILINGS)
def test_tour_200x100_full_run(pedsim, tiling):
    scn = S.make_scenario(200, 100, 1000, 1000, band_a=10, seed=1, mode=TOUR, steps=500)
    say("tour 200x100", tiling)
    run_both(pedsim, scn, 500, chunks=(1, 1, 1, 2, 5, 10, 30, 50, 100), tiling=tiling)


@pytest.mark.parametrize("W,H,na,nb,obst,seed", [
    (67, 13, 90, 80, 0.0, 11),
    (130, 37, 300, 280, 0.07, 12),
    (3, 40, 20, 0, 0.0, 13),
    (257, 9, 150, 160, 0.0, 14),
    (64, 8, 0, 0, 0.0, 15),
])
@pytest.mark.parametrize("tiling", [None, (0, 48, 2, 256), (0, 40, 3, 512)])
def test_tour_ragged_grids(pedsim, W, H, na, nb, obst, seed, tiling):
    band = max(1, min(W // 2, 6))
    scn = S.make_scenario(W, H, na, nb, band_a=band, seed=seed, mode=TOUR, obstacle_frac=obst)
    say("tour ragged", W, H, tiling)
    run_both(pedsim, scn, 60, chunks=(1, 1, 3, 10), tiling=tiling)


@pytest.mark.parametrize("alpha,beta,rho,dtau,initial", [
    (2, 3, 0.05, 0.5, True), (0, 1, 1.0, 2.0, False), (3, 0, 0.3, 0.0, True),
    (1, 2, 0.9, 1.0, False)])  # rho 0.9: values reach the subnormal range within the run
@pytest.mark.parametrize("tiling", [None, (0, 64, 3, 256)])
def test_tour_parameters_and_initial_lengths(pedsim, alpha, beta, rho, dtau, initial, tiling):
    scn = S.make_scenario(150, 60, 700, 650, band_a=8, seed=21, mode=TOUR, obstacle_frac=0.04,
                          alpha=alpha, beta=beta, rho=rho, dtau=dtau)
    if initial:
        scn.tour = (np.random.default_rng(5).random(scn.agents) * 30).astype(np.float32)
    say("tour params", alpha, beta, rho, dtau, initial, tiling)
    run_both(pedsim, scn, 120, chunks=(1, 10, 40), tiling=tiling)


def test_tour_1024x512_default_tiling(pedsim):
    scn = S.aco_tour_1024x512()
    say("tour 1024x512")
    run_both(pedsim, scn, 200, chunks=(1, 7, 40))


def test_tour_resumes_from_a_checkpoint(pedsim):
    """Steps 0..n-1, then a fresh handle from the saved state (step0 = n, the
    saved tour lengths) continues exactly as the uninterrupted run."""
    scn = S.make_scenario(130, 37, 300, 280, band_a=6, seed=31, mode=TOUR, obstacle_frac=0.05)
    sim = pedsim.Sim(scn)
    sim.step(25, TOUR)
    code, ids, tau = sim.state()
    tour = sim.tour_lengths().copy()
    sim.close()
    resumed = scn.copy()
    resumed.code, resumed.ids, resumed.tau, resumed.tour = code, ids, tau, tour
    sim2 = pedsim.Sim(resumed, step0=25)
    sim2.step(35, TOUR)
    st = oracle.State.from_scenario(scn)
    st.run(TOUR, 60)
    assert_same(sim2, st, "after resume")
    sim2.close()


def test_tour_errors(pedsim):
    import torch
    scn = S.make_scenario(64, 32, 100, 100, band_a=6, seed=3, mode=S.MODE_ACO)
    sim = pedsim.Sim(scn)  # no tour array attached
    with pytest.raises(pedsim.SimError) as e:
        sim.step(1, TOUR)
    assert e.value.code == pedsim.SIM_ENOTOUR
    with pytest.raises(pedsim.SimError) as e:
        sim.set_tiling(TOUR, 3, 48, 2, 256)  # the streaming form has no tour variant
    assert e.value.code == pedsim.SIM_EINVAL
    bad = torch.full((scn.agents,), -1.0, device="cuda")
    shadow = torch.empty_like(bad)
    with pytest.raises(pedsim.SimError) as e:
        pedsim.sim_attach_tour(sim.h, bad, shadow)
    assert e.value.code == pedsim.SIM_ESTATE
    with pytest.raises(pedsim.SimError) as e:
        pedsim.sim_attach_tour(sim.h, shadow, shadow)
    assert e.value.code == pedsim.SIM_EINVAL
    sim.close()


def _batch_mix(neighbours):
    """Twelve scenarios of the 256-scenario batch's shapes; every third runs
    the tour variant (with initial tour lengths), the rest LEM or ACO."""
    scns = S.batched_256(count=12, steps=100)
    for i, s in enumerate(scns):
        s.neighbours = neighbours
        if i % 3 == 2:
            s.mode = TOUR
            if s.tau is None:
                s.tau = np.ones((2, s.H, s.W), np.float32)
            s.tour = (np.random.default_rng(i).random(s.agents) * 5).astype(np.float32)
    return scns


@pytest.mark.parametrize("neighbours", [5, 8])
def test_tour_in_a_batch_matches_oracle(pedsim, neighbours):
    scns = _batch_mix(neighbours)
    batch = pedsim.Batch(len(scns))
    if neighbours == 8:
        batch.set_neighbours(8)
    else:
        batch.set_tuning(0, 48, 3, 512, 2)
    slots = [batch.add(s) for s in scns]
    say("tour batch", neighbours)
    batch.step_slots({sl: 40 + 7 * i for i, sl in enumerate(slots)})
    batch.step(30)
    for i, (s, sl) in enumerate(zip(scns, slots)):
        st = oracle.State.from_scenario(s)
        st.run(s.mode, 40 + 7 * i + 30)
        code, ids, tau = batch.state(sl)
        assert np.array_equal(code, st.code) and np.array_equal(ids, st.ids), (i, s.mode)
        if s.mode != S.MODE_LEM:
            assert np.array_equal(tau.view(np.uint32), st.tau.view(np.uint32)), i
        if s.mode == TOUR:
            assert np.array_equal(batch.tour_lengths(sl).view(np.uint32), st.tour.view(np.uint32)), i
        got = batch.stats(sl)
        a, b, ca, cb = st.counts()
        assert (got["crossed_a"], got["crossed_b"], got["step"]) == (ca, cb, st.t)
    batch.close()


def test_tour_batch_needs_the_lds_form(pedsim):
    scn = S.make_scenario(64, 32, 100, 100, band_a=6, seed=3, mode=TOUR)
    batch = pedsim.Batch(2)  # default tuning: the streaming form
    with pytest.raises(pedsim.SimError) as e:
        batch.add(scn)
    assert e.value.code == pedsim.SIM_EINVAL
    batch.close()
