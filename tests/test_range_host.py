"""Host-side checks of the range step's heuristic weights (larger scanning and
moving ranges, Sec. VII): the library's table is the float nearest to
(f/S)^beta * D2^(-beta/2) for every scanning range S, moving range M, free run
f and beta, computed here with mpmath; and bad arguments are rejected."""
import numpy as np
import pytest

from paper_1412_4933_amd import pedsim


def _nearest(exact, mpmath):
    """The binary32 value nearest to an mpmath number (ties to even)."""
    f = np.float32(float(exact))
    best = f
    for cand in (np.nextafter(f, np.float32(0)), np.nextafter(f, np.float32(np.inf))):
        if abs(mpmath.mpf(float(cand)) - exact) < abs(mpmath.mpf(float(best)) - exact):
            best = cand
    return best


@pytest.mark.parametrize("S_", range(1, 9))
def test_library_range_weights_correctly_rounded(S_):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 60
    for M in range(1, S_ + 1):
        for beta in range(0, 9):
            diag, lat = pedsim.sim_range_weights(S_, M, beta)
            for f in range(1, 9):
                if f > S_:
                    assert diag[f - 1] == 0 and lat[f - 1] == 0
                    continue
                k = min(f, M)
                for a, got in ((1, diag[f - 1]), (0, lat[f - 1])):
                    d2 = (M + 1 - a * k) ** 2 + k * k
                    exact = mpmath.power(mpmath.mpf(f) / S_, beta) * mpmath.power(d2, -mpmath.mpf(beta) / 2)
                    want = _nearest(exact, mpmath)
                    assert np.float32(got).view(np.uint32) == want.view(np.uint32), (S_, M, beta, f, a)


def test_range_one_one_weights_are_the_base_weights():
    # with both ranges 1: diagonal D2 = 2, lateral D2 = 5 (the base heuristic)
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 60
    for beta in range(0, 9):
        diag, lat = pedsim.sim_range_weights(1, 1, beta)
        assert diag[0] == _nearest(mpmath.power(2, -mpmath.mpf(beta) / 2), mpmath)
        assert lat[0] == _nearest(mpmath.power(5, -mpmath.mpf(beta) / 2), mpmath)


@pytest.mark.parametrize("bad", [(0, 1, 2), (9, 1, 2), (2, 3, 2), (3, 0, 2), (3, 2, -1), (3, 2, 9)])
def test_range_weights_reject_bad_arguments(bad):
    with pytest.raises(pedsim.SimError):
        pedsim.sim_range_weights(*bad)
