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
