"""Host checks of the population sweep's inputs (Sec. VI): 2,560 k agents on
a 480 x 480 grid, bands as narrow as the band rule allows, paired LEM/ACO
runs."""
import numpy as np

from paper_1412_4933_amd import scenarios as S


def test_sweep_bands_agree_with_the_papers_examples():
    # k = 1: three columns, the paper's example of an initial band; k = 5: a
    # crossing line at the 14th column from the far side, the paper's example
    # of where the opposite group counts as crossed
    s1, s5 = S.paper_sweep([1, 5], repeats=1, steps=10, modes=(S.MODE_LEM,))
    assert (s1.band_a, s1.band_b, s1.cross_a, s1.cross_b) == (3, 3, 3, 3)
    assert (s5.band_a, s5.band_b, s5.cross_a, s5.cross_b) == (14, 14, 14, 14)


def test_sweep_populations_and_pairing():
    scns = S.paper_sweep([2, 20], repeats=2, steps=25000)
    assert len(scns) == 2 * 2 * 2
    for i in range(0, len(scns), 2):
        lem, aco = scns[i], scns[i + 1]
        assert (lem.mode, aco.mode) == (S.MODE_LEM, S.MODE_ACO)
        assert lem.seed == aco.seed and np.array_equal(lem.code, aco.code)
        assert lem.W == lem.H == 480 and lem.steps == 25000
        assert lem.n_a == lem.n_b and lem.agents % 2560 == 0
        assert np.count_nonzero(lem.code == S.GROUP_A) == lem.n_a
        assert np.all(lem.code[:, lem.band_a:] != S.GROUP_A)
    assert scns[0].seed != scns[2].seed  # repeats differ
