"""The no-allocation entry point (sim_run_noalloc, for callers that cannot
allocate device memory) against the allocating path (sim_create with a
caller-owned scratch, sim_step_*, sim_stats) on the same inputs: identical
planes and counters, on two calls in a row, the second with a smaller input
(the static scratch keeps the first call's contents), and a scenario too large
for the static array is refused before any work."""
import numpy as np
import pytest

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


def _allocating(pedsim, scn, mode, steps):
    sim = pedsim.Sim(scn, autotune=False)
    sim.step(steps, mode)
    code, ids, tau = sim.state()
    stats = sim.stats()
    sim.close()
    return code, ids, tau, stats


def _noalloc(pedsim, scn, mode, steps):
    import torch
    dev = torch.device("cuda:0")
    code = torch.from_numpy(np.ascontiguousarray(scn.code)).to(dev)
    ids = torch.from_numpy(np.ascontiguousarray(scn.ids).view(np.int32)).to(dev)
    tau = torch.from_numpy(np.ascontiguousarray(scn.tau)).to(dev) if scn.tau is not None else None
    torch.cuda.synchronize(dev)
    stats = pedsim.sim_run_noalloc(pedsim.params_of(scn), mode, code, ids, tau, steps)
    out_tau = tau.cpu().numpy() if tau is not None else None
    return code.cpu().numpy(), ids.cpu().numpy().view(np.uint32), out_tau, stats


def _same(a, b, what):
    ca, ia, ta, sa = a
    cb, ib, tb, sb = b
    assert np.array_equal(ca, cb), f"code differs {what}"
    assert np.array_equal(ia, ib), f"ids differ {what}"
    if ta is not None:
        assert np.array_equal(ta.view(np.uint32), tb.view(np.uint32)), f"pheromone differs {what}"
    assert sa == sb, f"counters differ {what}: {sa} vs {sb}"


def test_noalloc_matches_allocating_path_twice(pedsim):
    big = S.make_scenario(700, 300, 9000, 9000, band_a=30, seed=31, mode=S.MODE_ACO, obstacle_frac=0.04)
    print("[gpu-case] noalloc call 1: 700x300 ACO, 37 steps", flush=True)
    _same(_noalloc(pedsim, big, S.MODE_ACO, 37), _allocating(pedsim, big, S.MODE_ACO, 37), "call 1")
    small = S.make_scenario(150, 44, 500, 480, band_a=8, seed=32, mode=S.MODE_LEM, with_tau=True)
    print("[gpu-case] noalloc call 2: 150x44 LEM, 23 steps", flush=True)
    _same(_noalloc(pedsim, small, S.MODE_LEM, 23), _allocating(pedsim, small, S.MODE_LEM, 23), "call 2")
    print("[gpu-case] noalloc call 3: 150x44 ACO, 0 steps", flush=True)
    _same(_noalloc(pedsim, small, S.MODE_ACO, 0), _allocating(pedsim, small, S.MODE_ACO, 0), "call 3")


def test_noalloc_refuses_what_does_not_fit(pedsim):
    import torch
    W, H = 4096, 2048  # 13 B per cell of scratch: far beyond the static array
    p = pedsim.SimParams(W, H, 1, 0, 0.1, 1.0, 1, 2, 4, 4)
    dev = torch.device("cuda:0")
    code = torch.zeros(8, dtype=torch.uint8, device=dev)  # never read: refused on the host first
    ids = torch.zeros(8, dtype=torch.int32, device=dev)
    with pytest.raises(pedsim.SimError) as e:
        pedsim.sim_run_noalloc(p, S.MODE_LEM, code, ids, None, 5)
    assert e.value.code == pedsim.SIM_ESCRATCH
