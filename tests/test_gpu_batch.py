"""Batched form: many independent scenarios in shared launches of the
persistent batch kernel (captured in hipGraphs) give, scenario by scenario,
exactly the oracle's result and exactly the plain single-scenario result."""
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


def mixed_scenarios(n, seed0=100):
    """Small scenarios of uneven size, population and mode (oracle-sized)."""
    rng = np.random.default_rng(seed0)
    out = []
    for i in range(n):
        W = int(rng.integers(20, 300))
        H = int(rng.integers(8, 120))
        cap = max(1, (W // 4) * (H - 2))
        N = int(rng.integers(0, min(cap, 3000) + 1))
        mode = S.MODE_LEM if i % 2 == 0 else S.MODE_ACO
        out.append(S.make_scenario(W, H, N // 2, N - N // 2, band_a=max(1, W // 8), seed=seed0 + i,
                                   mode=mode, obstacle_frac=0.03 if i % 3 == 0 else 0.0,
                                   with_tau=(mode == S.MODE_ACO or i % 4 == 0)))
    return out


def check_slot(batch, slot, st, what):
    code, ids, tau = batch.state(slot)
    assert np.array_equal(code, st.code), f"code differs {what}"
    assert np.array_equal(ids, st.ids), f"ids differ {what}"
    if st.tau is not None and tau is not None and batch.members[slot].scenario.mode == S.MODE_ACO:
        assert np.array_equal(tau.view(np.uint32), st.tau.view(np.uint32)), f"tau differs {what}"
    s = batch.stats(slot)
    a, b, ca, cb = st.counts()
    assert (s["agents_a"], s["agents_b"], s["crossed_a"], s["crossed_b"]) == (a, b, ca, cb), what
    assert s["step"] == st.t, what


def test_batch_matches_oracle_per_scenario(pedsim):
    import torch
    scns = mixed_scenarios(24)
    batch = pedsim.Batch(32)
    slots = [batch.add(s) for s in scns]
    states = [oracle.State.from_scenario(s) for s in scns]
    rng = np.random.default_rng(5)
    for call in range(4):
        steps = [int(v) for v in rng.integers(0, 40, size=len(scns))]
        say("batch call", call, steps[:6])
        batch.step_slots({slot: k for slot, k in zip(slots, steps)})
        # unrelated eager work on the device between graph replays
        x = torch.ones(1 << 20, device="cuda")
        x.mul_(3.0).add_(1.0)
        for slot, st, k, scn in zip(slots, states, steps, scns):
            st.run(scn.mode, k)
        for slot, st in zip(slots, states):
            check_slot(batch, slot, st, f"slot {slot} after call {call}")
    batch.close()


def test_batch_alone_equals_in_the_mix(pedsim):
    scns = mixed_scenarios(10, seed0=300)
    batch = pedsim.Batch(16)
    slots = [batch.add(s) for s in scns]
    say("batch mix")
    batch.step(57)
    for slot, scn in zip(slots, scns):
        alone = pedsim.Sim(scn)
        alone.step(57)
        want = alone.state()
        got = batch.state(slot)
        assert np.array_equal(want[0], got[0]) and np.array_equal(want[1], got[1])
        if scn.mode == S.MODE_ACO:
            assert np.array_equal(want[2].view(np.uint32), got[2].view(np.uint32))
        alone.close()
    batch.close()


@pytest.mark.parametrize("tuning", [(1, 32, 1, 256, 1, 1), (1, 48, 2, 512, 2, 0), (2, 40, 2, 1024, 1, 1),
                                    (1, 64, 3, 512, 4, 1), (1, 32, 2, 64, 8, 1),
                                    (0, 64, 2, 256, 2, 1), (0, 48, 3, 64, 4, 0), (0, 64, 1, 512, 1, 1),
                                    (3, 48, 2, 256, 4, 1), (3, 32, 3, 128, 6, 0)])
def test_batch_results_do_not_depend_on_tuning(pedsim, tuning):
    scns = mixed_scenarios(8, seed0=500)
    states = [oracle.State.from_scenario(s) for s in scns]
    batch = pedsim.Batch(8)
    try:
        batch.set_tuning(*tuning)
    except pedsim.SimError:
        batch.close()
        pytest.skip(f"tuning {tuning} does not fit this device")
    slots = [batch.add(s) for s in scns]
    say("batch tuning", tuning)
    batch.step(23)
    batch.step(10)
    for slot, st, scn in zip(slots, states, scns):
        st.run(scn.mode, 33)
        check_slot(batch, slot, st, f"tuning {tuning}")
    batch.close()


def test_batch_long_call_splits_and_slots_are_reused(pedsim):
    scns = mixed_scenarios(6, seed0=700)
    batch = pedsim.Batch(4)
    batch.set_tuning(1, 32, 1, 256, 2, 1)
    slots = [batch.add(s) for s in scns[:4]]
    with pytest.raises(pedsim.SimError) as e:
        batch.add(scns[4])
    assert e.value.code == pedsim.SIM_EFULL
    say("batch long call")
    batch.step_slots({slots[0]: 300, slots[1]: 1, slots[2]: 0, slots[3]: 129})  # > 128 launches
    st = [oracle.State.from_scenario(s) for s in scns[:4]]
    for s_, k, scn in zip(st, (300, 1, 0, 129), scns[:4]):
        s_.run(scn.mode, k)
    for slot, s_ in zip(slots, st):
        check_slot(batch, slot, s_, "long call")
    batch.remove(slots[2])
    new_slot = batch.add(scns[4])
    assert new_slot == slots[2]
    batch.step_slots({new_slot: 44, slots[0]: 5})
    st4 = oracle.State.from_scenario(scns[4])
    st4.run(scns[4].mode, 44)
    st[0].run(scns[0].mode, 5)
    check_slot(batch, new_slot, st4, "reused slot")
    check_slot(batch, slots[0], st[0], "neighbour of reused slot")
    batch.close()


def test_full_256_scenario_batch_sampled_against_oracle(pedsim):
    """The benchmark's batch at full size (256 scenarios, 3.24M agents, the
    default tuning and graph replay): every counter is checked against the
    oracle's invariants, and sampled scenarios (the three largest, the three
    smallest and six others) bit for bit."""
    scns = S.batched_256(steps=60)
    batch = pedsim.Batch(len(scns))
    slots = [batch.add(s) for s in scns]
    say("full batch", len(scns), batch.tuning())
    batch.step(60)
    for s, slot in zip(scns, slots):
        got = batch.stats(slot)
        assert (got["agents_a"], got["agents_b"], got["step"]) == (s.n_a, s.n_b, 60)
    order = sorted(range(len(scns)), key=lambda i: scns[i].agents)
    rng = np.random.default_rng(7)
    sample = order[:3] + order[-3:] + [int(i) for i in rng.choice(order[3:-3], 6, replace=False)]
    for i in sample:
        st = oracle.State.from_scenario(scns[i])
        st.run(scns[i].mode, 60)
        check_slot(batch, slots[i], st, f"scenario {i} ({scns[i].W}x{scns[i].H}, {scns[i].agents} agents)")
    batch.close()
