"""GPU parity of the population sweep's scenarios (Sec. VI shapes: 480 x 480,
2,560 k agents, LEM and ACO) run together through the batched path: every
scenario's planes and crossing counts equal the oracle's after the same
steps."""
import numpy as np
import pytest

import oracle
from paper_1412_4933_amd import scenarios as S

pytestmark = pytest.mark.gpu


def test_sweep_batch_matches_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_4933_amd import pedsim
    scns = S.paper_sweep([1, 8, 20], repeats=1, steps=300)
    batch = pedsim.Batch(len(scns))
    slots = [batch.add(s) for s in scns]
    print("[gpu-case] sweep batch", len(scns), flush=True)
    batch.step(300)
    for s, slot in zip(scns, slots):
        st = oracle.State.from_scenario(s)
        st.run(s.mode, 300)
        code, ids, tau = batch.state(slot)
        assert np.array_equal(code, st.code) and np.array_equal(ids, st.ids), (s.agents, s.mode)
        if s.mode == S.MODE_ACO:
            assert np.array_equal(tau.view(np.uint32), st.tau.view(np.uint32))
        got = batch.stats(slot)
        a, b, ca, cb = st.counts()
        assert (got["crossed_a"], got["crossed_b"]) == (ca, cb)
    batch.close()


def _batch_vs_oracle(pedsim, scns, steps, neighbours):
    batch = pedsim.Batch(len(scns))
    if neighbours != 5:
        batch.set_neighbours(neighbours)
    slots = [batch.add(s) for s in scns]
    batch.step(steps)
    for s, slot in zip(scns, slots):
        st = oracle.State.from_scenario(s)
        st.run(s.mode, steps)
        code, ids, tau = batch.state(slot)
        assert np.array_equal(code, st.code) and np.array_equal(ids, st.ids), (s.W, s.agents, s.mode)
        if s.mode == S.MODE_ACO:
            assert np.array_equal(tau.view(np.uint32), st.tau.view(np.uint32))
        got = batch.stats(slot)
        a, b, ca, cb = st.counts()
        assert (got["crossed_a"], got["crossed_b"], got["step"]) == (ca, cb, st.t)
    batch.close()


def test_sweep_batch_eight_neighbours_matches_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_4933_amd import pedsim
    scns = S.paper_sweep([1, 8], repeats=1, steps=300, neighbours=8)
    print("[gpu-case] sweep batch nb8", len(scns), flush=True)
    _batch_vs_oracle(pedsim, scns, 300, 8)


def test_uneven_batch_eight_neighbours_matches_oracle():
    """Scenarios of different sizes and modes (the first sixteen of the
    256-scenario batch) advanced together with the eight-neighbour set,
    split across several graph launches."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_4933_amd import pedsim
    scns = S.batched_256(count=16, steps=100)
    for s in scns:
        s.neighbours = 8
    print("[gpu-case] uneven batch nb8", len(scns), flush=True)
    _batch_vs_oracle(pedsim, scns, 100, 8)


def test_batch_rejects_a_scenario_of_another_candidate_set():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_4933_amd import pedsim
    s8 = S.make_scenario(64, 32, 50, 50, band_a=4, seed=2, mode=S.MODE_LEM, neighbours=8)
    s5 = S.make_scenario(64, 32, 50, 50, band_a=4, seed=2, mode=S.MODE_LEM)
    batch = pedsim.Batch(2)
    with pytest.raises(ValueError):
        batch.add(s8)
    batch.add(s5)
    with pytest.raises(ValueError):
        batch.set_neighbours(8)  # a resident scenario uses five candidates
    batch.close()
