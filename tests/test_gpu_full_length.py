"""GPU parity at full length on the large configurations.

  * the 4096x2048 stress grid (5% obstacles, 1M agents), LEM and ACO, through
    all 1,000 steps in the benchmark's launch configuration, compared bit for
    bit after 100, 500 and 1,000 steps;
  * the 256-scenario batch (widths 64-2048, half LEM half ACO) through all
    1,000 steps in one batch at its default tuning, every scenario compared
    bit for bit with the oracle;
  * sixteen requests of the served stream at full size (up to 2048x1024,
    200-2,000 steps) through the serving loop, each compared with the oracle.

The oracle runs on all the host cores this process may use: the OpenMP build
for one large grid, or the plain build on a thread pool (one scenario per
thread; the ctypes calls release the interpreter lock) for many scenarios.
"""
import time
from concurrent.futures import ThreadPoolExecutor

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


def same_state(code, ids, tau, st, what, tour=None):
    assert np.array_equal(code, st.code), f"code differs {what}: {np.argwhere(code != st.code)[:5]}"
    assert np.array_equal(ids, st.ids), f"ids differ {what}: {np.argwhere(ids != st.ids)[:5]}"
    if tau is not None and st.tau is not None:
        bad = tau.view(np.uint32) != st.tau.view(np.uint32)
        assert not bad.any(), f"pheromone differs {what}: {np.argwhere(bad)[:5]}"
    if tour is not None:
        assert np.array_equal(tour.view(np.uint32), st.tour.view(np.uint32)), f"tour differs {what}"


def same_stats(got, st, what):
    a, b, ca, cb = st.counts()
    assert (got["agents_a"], got["agents_b"], got["crossed_a"], got["crossed_b"]) == (a, b, ca, cb), what
    assert got["step"] == st.t, what


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", [S.MODE_LEM, S.MODE_ACO])
def test_stress_4096x2048_all_1000_steps(pedsim, mode):
    scn = S.stress_4096x2048(mode)
    sim = pedsim.Sim(scn)
    say("stress 4096x2048 x1000", mode, "tiling", sim.tiling(mode), "oracle threads", THREADS)
    st = oracle.State.from_scenario(scn, threads=THREADS)
    done = 0
    for chunk in (100, 400, 500):
        t0 = time.perf_counter()
        sim.step(chunk, mode)
        moved = st.run(mode, chunk)
        done += chunk
        code, ids, tau = sim.state()
        same_state(code, ids, tau if mode != S.MODE_LEM else None, st, f"after {done} steps")
        got = sim.stats()
        same_stats(got, st, f"after {done} steps")
        assert got["moved_last"] == moved
        say(f"  {done} steps equal ({time.perf_counter() - t0:.1f} s)")
    sim.close()


# ---------------------------------------------------------------------------
# The 256-scenario batch, every scenario through all 1,000 steps
# ---------------------------------------------------------------------------

BATCH_STEPS = 1000
BATCH_CHUNKS = 8


@pytest.fixture(scope="module")
def batch_result(pedsim):
    """Run the whole batch once on the GPU; keep every final state on the host."""
    scns = S.batched_256(steps=BATCH_STEPS)
    batch = pedsim.Batch(len(scns))
    slots = [batch.add(s) for s in scns]
    t0 = time.perf_counter()
    batch.step(BATCH_STEPS)
    out = []
    for s, slot in zip(scns, slots):
        code, ids, tau = batch.state(slot)
        out.append((code, ids, tau if s.mode != S.MODE_LEM else None, batch.stats(slot)))
    say("batch of", len(scns), "x", BATCH_STEPS, "steps, tuning", batch.tuning(), batch.tuning_source,
        f"({time.perf_counter() - t0:.1f} s with read-back)")
    batch.close()
    return scns, out


def _oracle_final(scn):
    st = oracle.State.from_scenario(scn)
    st.run(scn.mode, BATCH_STEPS)
    return st


@pytest.mark.timeout(900)
@pytest.mark.parametrize("part", range(BATCH_CHUNKS))
def test_batched_256_every_scenario_all_1000_steps(batch_result, part):
    scns, got = batch_result
    # interleave sizes across parts so that each part costs about the same
    order = sorted(range(len(scns)), key=lambda i: -scns[i].W * scns[i].H)
    mine = order[part::BATCH_CHUNKS]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(THREADS) as ex:
        states = list(ex.map(lambda i: _oracle_final(scns[i]), mine))
    for i, st in zip(mine, states):
        code, ids, tau, stats = got[i]
        what = f"scenario {i} ({scns[i].W}x{scns[i].H}, {scns[i].agents} agents, mode {scns[i].mode})"
        same_state(code, ids, tau, st, what)
        same_stats(stats, st, what)
    say(f"batch part {part}: {len(mine)} scenarios equal ({time.perf_counter() - t0:.1f} s, "
        f"{THREADS} oracle threads)")


# ---------------------------------------------------------------------------
# Served requests at full size
# ---------------------------------------------------------------------------

@pytest.mark.timeout(900)
def test_served_full_size_requests(pedsim):
    from paper_1412_4933_amd import serve
    specs = S.served_requests(16)
    reqs = serve.poisson_requests(specs, rate=540.0, seed=1)
    serve.prebuild(reqs)
    say("served", len(reqs), "full-size requests, largest",
        max((W * H, W, H) for W, H, *_ in specs)[1:], "steps", min(s[5] for s in specs), "..",
        max(s[5] for s in specs))
    srv = serve.Server(capacity=8, budget_bytes=2 << 30, quantum=100, keep_state=True)
    results = srv.run(reqs)
    srv.close()
    assert sorted(r.rid for r in results) == list(range(len(reqs)))
    overlapped = sum(1 for r in results if any(o.rid != r.rid and o.admitted < r.finished
                                               and o.finished > r.admitted for o in results))
    assert overlapped >= len(results) // 2

    def check(res):
        req = reqs[res.rid]
        st = oracle.State.from_scenario(req.build())
        st.run(req.mode, req.steps)
        return res, st

    t0 = time.perf_counter()
    with ThreadPoolExecutor(THREADS) as ex:
        pairs = list(ex.map(check, results))
    for res, st in pairs:
        code, ids, tau = res.state
        what = f"request {res.rid}"
        same_state(code, ids, tau if reqs[res.rid].mode != S.MODE_LEM else None, st, what)
        same_stats(res.stats, st, what)
    say(f"served: {len(pairs)} requests equal ({time.perf_counter() - t0:.1f} s)")
