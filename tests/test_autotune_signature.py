"""Host logic of the autotuner: workloads that run different kernels get
different cache keys."""
from paper_1412_4933_amd import autotune, scenarios as S


def test_signature_separates_candidate_sets_and_tour_variant():
    base = [S.make_scenario(64, 32, 50, 50, band_a=4, seed=1, mode=S.MODE_ACO)]
    nb8 = [S.make_scenario(64, 32, 50, 50, band_a=4, seed=1, mode=S.MODE_ACO, neighbours=8)]
    tour = [S.make_scenario(64, 32, 50, 50, band_a=4, seed=1, mode=S.MODE_ACO_TOUR)]
    keys = {autotune.signature(x, "batch") for x in (base, nb8, tour)}
    assert len(keys) == 3
    assert autotune.signature(base, "batch") == autotune.signature(
        [S.make_scenario(64, 32, 60, 40, band_a=4, seed=9, mode=S.MODE_ACO)], "batch")
