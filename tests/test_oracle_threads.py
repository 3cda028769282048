"""The OpenMP build of the oracle gives the plain build's results bit for bit.

Both builds come from the same source; the parallel loops write disjoint cells
and sum integers only, so every plane, every counter and the number of moves
must agree for any thread count.
"""
import numpy as np
import pytest

import oracle
from paper_1412_4933_amd import scenarios as S


def _same(a, b):
    assert np.array_equal(a.code, b.code)
    assert np.array_equal(a.ids, b.ids)
    if a.tau is not None:
        assert np.array_equal(a.tau.view(np.uint32), b.tau.view(np.uint32))
    if a.tour.size:
        assert np.array_equal(a.tour.view(np.uint32), b.tour.view(np.uint32))
    assert a.counts() == b.counts()


@pytest.mark.parametrize("threads", [2, 3, 8])
@pytest.mark.parametrize("mode,neighbours", [(S.MODE_LEM, 5), (S.MODE_ACO, 5), (S.MODE_ACO_TOUR, 5),
                                             (S.MODE_LEM, 8), (S.MODE_ACO, 8), (S.MODE_ACO_TOUR, 8)])
def test_threads_agree_with_one_thread(mode, neighbours, threads):
    scn = S.make_scenario(311, 97, 2600, 2500, band_a=14, seed=40 + mode, mode=mode,
                          obstacle_frac=0.05, neighbours=neighbours, with_tau=True)
    one = oracle.State.from_scenario(scn)
    many = oracle.State.from_scenario(scn, threads=threads)
    assert oracle.lib(parallel=True).oracle_set_threads(threads) == threads
    for chunk in (1, 7, 40):
        m1 = one.run(mode, chunk)
        m2 = many.run(mode, chunk)
        assert m1 == m2
        _same(one, many)
    m1, r1, w1 = one.step(mode, want_detail=True)
    m2, r2, w2 = many.step(mode, want_detail=True)
    assert m1 == m2 and np.array_equal(r1, r2) and np.array_equal(w1, w2)
    _same(one, many)


def test_plain_build_is_one_thread():
    assert oracle.lib().oracle_set_threads(8) == 1
