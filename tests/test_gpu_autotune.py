"""The autotuner on the GPU: tune_plain, tune_range and tune_batch each time a
few candidate launch shapes on a small workload from the same initial state,
and the winning shape, applied the way the binding applies the committed
cache, gives results identical to the oracle. The tuner's in-memory cache is
restored afterwards, so later tests see the committed tunings only."""
import numpy as np
import pytest

import oracle
from paper_1412_4933_amd import scenarios as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tuner():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_4933_amd import autotune, pedsim
    pedsim.lib()
    autotune._ensure_loaded()
    saved = dict(autotune._cache)
    yield autotune
    autotune._cache.clear()
    autotune._cache.update(saved)


def _same(code, ids, tau, st, what):
    assert np.array_equal(code, st.code), what
    assert np.array_equal(ids, st.ids), what
    if tau is not None and st.tau is not None:
        assert np.array_equal(tau.view(np.uint32), st.tau.view(np.uint32)), what


def test_tune_plain_winner_matches_oracle(tuner):
    from paper_1412_4933_amd import pedsim
    scn = S.make_scenario(300, 120, 3000, 3000, band_a=16, seed=61, mode=S.MODE_ACO, steps=60,
                          obstacle_frac=0.03)
    cands = [(0, 48, 2, 256), (0, 52, 4, 512), (3, 48, 2, 256), (1, 32, 2, 512)]
    best, timings = tuner.tune_plain(scn, S.MODE_ACO, candidates=cands)
    print("[gpu-case] tune_plain:", best, [(round(t * 1e3, 3), tl) for t, tl in timings], flush=True)
    assert best in cands and len(timings) == len(cands)
    assert tuner.cached_plain(scn, S.MODE_ACO) == best
    sim = pedsim.Sim(scn)  # reads the tuner's cache
    assert sim.tuned.get(S.MODE_ACO) == best and sim.tiling(S.MODE_ACO) == best
    sim.step(60)
    st = oracle.State.from_scenario(scn)
    st.run(S.MODE_ACO, 60)
    _same(*sim.state(), st, f"plain winner {best}")
    sim.close()


def test_tune_range_winner_matches_oracle(tuner):
    from paper_1412_4933_amd import pedsim
    scn = S.make_scenario(260, 90, 2000, 2000, band_a=14, seed=62, mode=S.MODE_ACO, steps=40,
                          ranges=(4, 2))
    cands = [(64, 16, 1, 256), (64, 32, 1, 256), (64, 32, 2, 512), (32, 16, 3, 128)]
    best, timings = tuner.tune_range(scn, S.MODE_ACO, candidates=cands)
    print("[gpu-case] tune_range:", best, [(round(t * 1e3, 3), tl) for t, tl in timings], flush=True)
    assert best in cands and len(timings) == len(cands)
    sim = pedsim.Sim(scn)
    assert sim.range_tuned == best and sim.range_tiling() == best
    sim.step(40)
    st = oracle.State.from_scenario(scn)
    st.run(S.MODE_ACO, 40)
    _same(*sim.state(), st, f"range winner {best}")
    sim.close()


def test_tune_batch_winner_matches_oracle(tuner):
    from paper_1412_4933_amd import pedsim
    scns = []
    for i, (W, n) in enumerate([(96, 400), (160, 1200), (256, 3000), (130, 800), (200, 2000), (70, 300)]):
        scns.append(S.make_scenario(W, W // 2, n, n, band_a=max(4, W // 16), seed=70 + i,
                                    mode=S.MODE_LEM if i % 2 == 0 else S.MODE_ACO, steps=50,
                                    with_tau=True))
    cands = [(3, 48, 2, 256, 4), (3, 62, 3, 256, 4), (0, 48, 3, 512, 2), (1, 32, 2, 512, 2)]
    best, timings = tuner.tune_batch(scns, candidates=cands)
    print("[gpu-case] tune_batch:", best, [(round(t * 1e3, 3), tu) for t, tu in timings], flush=True)
    assert best in cands and len(timings) == len(cands)
    assert tuner.cached_batch(scns) == best
    batch = pedsim.Batch(len(scns))
    slots = [batch.add(s) for s in scns]
    batch.step(50)
    assert tuple(batch.tuning()[:5]) == best and batch.tuning_source == "autotuner cache"
    for s, slot in zip(scns, slots):
        st = oracle.State.from_scenario(s)
        st.run(s.mode, 50)
        code, ids, tau = batch.state(slot)
        _same(code, ids, tau, st, f"batch winner {best}, scenario {s.W}x{s.H}")
    batch.close()
