"""Pins of the oracle's larger scanning and moving ranges (the paper's future
work, Sec. VII; readings R18-R22 of the design notes): with both ranges 1 it is
the base model bit for bit; a lone agent walks M cells per step and stops at
obstacles; the LEM ranking and the ACO weights follow the scanned free runs
as computed by hand; every step keeps the invariants and every contested cell
goes to its lowest ticket; an independent Python implementation agrees."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import chisquare

import oracle
from oracle import ref
from paper_1412_4933_amd import scenarios as S

RAYS = {1: (1, 0), 2: (1, -1), 3: (1, 1), 4: (0, -1), 5: (0, 1)}


def _state(code, *, ranges, seed=1, tau=None, **kw):
    st = oracle.State.from_scenario(S.from_grid(code, seed=seed, tau=tau, **kw))
    st.ranges = ranges
    return st


@pytest.mark.parametrize("mode", [oracle.MODE_LEM, oracle.MODE_ACO])
@pytest.mark.parametrize("seed,obst", [(21, 0.0), (22, 0.07)])
def test_ranges_one_one_is_the_base_model(mode, seed, obst):
    scn = S.make_scenario(120, 40, 700, 650, band_a=10, seed=seed, mode=mode, obstacle_frac=obst,
                          with_tau=True)
    base = oracle.State.from_scenario(scn)
    rng = oracle.State.from_scenario(scn)
    rng.ranges = (1, 1)
    for _ in range(60):
        m1 = base.step(mode)
        m2 = rng.step(mode)
        assert m1 == m2
        assert np.array_equal(base.code, rng.code) and np.array_equal(base.ids, rng.ids)
        assert np.array_equal(base.tau.view(np.uint32), rng.tau.view(np.uint32))


@pytest.mark.parametrize("S_,M", [(1, 1), (2, 2), (3, 2), (5, 3), (8, 8)])
def test_range_weights_correctly_rounded(S_, M):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    for beta in range(0, 9):
        diag, lat = oracle.range_weights(S_, M, beta)
        for f in range(1, S_ + 1):
            k = min(f, M)
            for a, got in ((1, diag[f - 1]), (0, lat[f - 1])):
                d2 = (M + 1 - a * k) ** 2 + k * k
                exact = mpmath.power(mpmath.mpf(f) / S_, beta) * mpmath.power(d2, -mpmath.mpf(beta) / 2)
                # correctly rounded: no float lies strictly closer to the exact value
                g = float(got)
                below, above = np.nextafter(np.float32(g), np.float32(0)), np.nextafter(np.float32(g), np.float32(1e30))
                err = abs(mpmath.mpf(g) - exact)
                assert err <= abs(mpmath.mpf(float(below)) - exact), (S_, M, beta, f, a)
                assert err <= abs(mpmath.mpf(float(above)) - exact), (S_, M, beta, f, a)


@pytest.mark.parametrize("mode", [oracle.MODE_LEM, oracle.MODE_ACO])
@pytest.mark.parametrize("group", [S.GROUP_A, S.GROUP_B])
@pytest.mark.parametrize("S_,M", [(1, 1), (3, 2), (4, 4), (6, 3)])
def test_lone_agent_walks_m_cells_per_step(mode, group, S_, M):
    """Forward first along an open ray: M cells per step until the far column
    (W - 1 is reached after ceil((W - 1) / M) steps), then it stays there."""
    W, H, y0 = 40, 7, 3
    code = S.wall_frame(W, H)
    x0 = 0 if group == S.GROUP_A else W - 1
    code[y0, x0] = group
    st = _state(code, ranges=(S_, M), tau=np.ones((2, H, W), np.float32))
    for t in range(1, math.ceil((W - 1) / M) + 6):
        st.step(mode)
        ys, xs = np.nonzero(st.code == group)
        gone = min(t * M, W - 1)
        assert xs[0] == (x0 + gone if group == S.GROUP_A else x0 - gone), t
        if t * M < W - 1:
            assert ys[0] == y0


@pytest.mark.parametrize("S_,M", [(2, 1), (3, 2), (5, 5)])
def test_agent_stops_in_front_of_an_obstacle(S_, M):
    """A wall q cells ahead: the agent advances min(M, cells left) per step,
    stops next to the wall, then leaves the row sideways."""
    W, H, y0, q = 30, 9, 4, 11
    code = S.wall_frame(W, H)
    code[y0, 0] = S.GROUP_A
    code[y0, q] = S.WALL
    st = _state(code, ranges=(S_, M))
    x = 0
    while x < q - 1:
        st.step(oracle.MODE_LEM)
        x = min(x + M, q - 1)
        ys, xs = np.nonzero(st.code == S.GROUP_A)
        assert (xs[0], ys[0]) == (x, y0)
    st.step(oracle.MODE_LEM)
    ys, xs = np.nonzero(st.code == S.GROUP_A)
    assert ys[0] != y0


def _pocket_choices(S_, M, walls, tau_fn=None, n=4000, mode=oracle.MODE_LEM, beta=2):
    """Agent A at (5, 6) with the forward cell walled; `walls` shapes the side
    rays. Returns the requested rays over n seeds, one step each."""
    W, H = 14, 13
    counts = {}
    for seed in range(n):
        code = S.wall_frame(W, H)
        code[6, 6] = S.WALL  # forward blocked
        for (x, y) in walls:
            code[y, x] = S.WALL
        code[6, 5] = S.GROUP_A
        tau = None
        if mode == oracle.MODE_ACO:
            tau = np.ones((2, H, W), np.float32)
            if tau_fn:
                tau_fn(tau)
        st = _state(code, ranges=(S_, M), seed=seed + 1, tau=tau, beta=beta)
        _, req, length = st.step(mode, want_detail=True)
        r = int(req[6, 5])
        counts[r] = counts.get(r, 0) + 1
    return counts


PHI = [0.5 * math.erfc(-(j + 0.5) / math.sqrt(2)) for j in range(3)]


def _lem_expect(ranked, n):
    p = [PHI[0], PHI[1] - PHI[0], PHI[2] - PHI[1]]
    p = p[:len(ranked)]
    p[-1] += 1.0 - sum(p)
    return {r: q * n for r, q in zip(ranked, p)}


def test_lem_ranks_open_rays_by_scanned_free_run():
    """S = 3, M = 1: FD- (up-right) sees 1 free cell, FD+ (down-right) 3, L-
    (up) 3, L+ (down) none. Scores f^2/D2 with D2 = 2 (diagonal), 5
    (lateral): FD+ 9/2, L- 9/5, FD- 1/2, so the rank order is FD+, L-, FD-
    (the base model would rank both diagonals before the lateral)."""
    walls = [(7, 4), (5, 7)]  # ends the FD- ray after one cell; blocks L+
    n = 4000
    got = _pocket_choices(3, 1, walls, n=n)
    assert set(got) == {2, 3, 4}
    want = _lem_expect([3, 4, 2], n)
    assert chisquare([got[r] for r in (3, 4, 2)], [want[r] for r in (3, 4, 2)]).pvalue > 1e-4


def test_lem_lateral_ahead_of_a_short_diagonal_with_moving_range():
    """S = 3, M = 2 (reference point 3 cells ahead): FD- sees 1 free cell
    (D2 = 2^2 + 1 = 5, score 1/5), L- sees 3 and moves 2 (D2 = 3^2 + 2^2 =
    13, score 9/13), FD+ and L+ are closed: the lateral ray ranks first."""
    walls = [(7, 4), (6, 7), (7, 8), (5, 7)]  # FD- stops after 1; FD+ and L+ closed
    n = 3000
    got = _pocket_choices(3, 2, walls, n=n)
    assert set(got) == {2, 4}
    want = _lem_expect([4, 2], n)
    assert chisquare([got[4], got[2]], [want[4], want[2]]).pvalue > 1e-4


def test_aco_weights_use_landing_pheromone_and_visibility():
    """S = 4, M = 2, beta = 2: FD- sees 1 cell (k = 1), FD+ 4 (k = 2), L- 2
    (k = 2), L+ closed. eta^2 = (f/S)^2 / D2 with D2 from the landing cell to
    the point 3 cells ahead; the pheromone is read on the landing cell (set
    to 3 on FD+'s landing cell, 1 elsewhere)."""
    walls = [(7, 4), (5, 3), (5, 7)]  # FD- after 1 cell; L- after 2; L+ closed

    def tau_fn(tau):
        tau[0, 8, 7] = 3.0  # landing cell of FD+ (2 cells down-right of (5, 6))

    n = 6000
    got = _pocket_choices(4, 2, walls, tau_fn=tau_fn, n=n, mode=oracle.MODE_ACO)
    assert set(got) == {2, 3, 4}
    w = {2: Fraction(1, 16) / Fraction(2 ** 2 + 1), 3: 3 * Fraction(16, 16) / Fraction(1 + 4),
         4: Fraction(4, 16) / Fraction(9 + 4)}
    tot = sum(w.values())
    assert chisquare([got[r] for r in (2, 3, 4)], [float(w[r] / tot) * n for r in (2, 3, 4)]).pvalue > 1e-4


def _check_range_step(code0, ids0, code1, ids1, req, length, moved, S_, M, seed, t):
    H, W = code0.shape
    pos0 = {int(k): (int(x), int(y)) for y, x in zip(*np.nonzero(ids0)) for k in [ids0[y, x]]}
    pos1 = {int(k): (int(x), int(y)) for y, x in zip(*np.nonzero(ids1)) for k in [ids1[y, x]]}
    assert pos0.keys() == pos1.keys()
    assert np.array_equal(code0 == S.WALL, code1 == S.WALL)

    def empty(x, y):
        return 0 <= x < W and 0 <= y < H and code0[y, x] == 0

    requesters = {}
    for k, (x, y) in pos0.items():
        g = int(code0[y, x])
        d = 1 if g == 1 else -1
        run = {}
        for r, (a, b) in RAYS.items():
            n = 0
            while n < S_ and empty(x + (n + 1) * a * d, y + (n + 1) * b):
                n += 1
            run[r] = n
        r = int(req[y, x])
        if run[1] >= 1:  # forward first
            assert r == 1 and length[y, x] == min(run[1], M)
        if r == 0:
            assert all(run[q] == 0 for q in RAYS)
            assert pos1[k] == (x, y)
            continue
        a, b = RAYS[r]
        kk = int(length[y, x])
        assert 1 <= kk == min(run[r], M)
        tgt = (x + kk * a * d, y + kk * b)
        for i in range(1, kk + 1):  # the path and the landing cell are empty at t
            assert empty(x + i * a * d, y + i * b)
        requesters.setdefault(tgt, []).append((oracle.agent_words(seed, t, k - 1)[0], k - 1, k))
    winners = {min(v)[2]: tgt for tgt, v in requesters.items()}
    for k, (x, y) in pos0.items():
        assert pos1[k] == (winners[k] if k in winners else (x, y)), k
        if k in winners:  # monotone heading: no backward component
            g = int(code0[y, x])
            assert (pos1[k][0] - x) * (1 if g == 1 else -1) >= 0
    assert moved == len(winners)


@pytest.mark.parametrize("mode", [oracle.MODE_LEM, oracle.MODE_ACO])
@pytest.mark.parametrize("S_,M", [(2, 1), (3, 3), (5, 2)])
def test_invariants_and_lowest_ticket_every_step(mode, S_, M):
    scn = S.make_scenario(90, 30, 500, 480, band_a=9, seed=5 + S_ + M, mode=mode,
                          obstacle_frac=0.05, with_tau=True)
    st = oracle.State.from_scenario(scn)
    st.ranges = (S_, M)
    for t in range(25):
        code0, ids0 = st.code.copy(), st.ids.copy()
        moved, req, length = st.step(mode, want_detail=True)
        _check_range_step(code0, ids0, st.code, st.ids, req, length, moved, S_, M, scn.seed, t)
        assert np.all(st.tau >= 0)


@pytest.mark.parametrize("S_,M,mode,alpha,beta,seed", [
    (2, 1, 0, 1, 2, 31), (2, 2, 1, 1, 2, 32), (3, 2, 1, 2, 3, 33), (4, 4, 0, 1, 2, 34),
    (6, 3, 1, 0, 1, 35), (8, 5, 1, 1, 2, 36)])
def test_python_reference_agrees_with_ranges(S_, M, mode, alpha, beta, seed):
    scn = S.make_scenario(37, 15, 55, 50, band_a=5, seed=seed, mode=mode, obstacle_frac=0.08,
                          with_tau=True, alpha=alpha, beta=beta)
    st = oracle.State.from_scenario(scn)
    st.ranges = (S_, M)
    code, ids, tau = scn.code.copy(), scn.ids.copy(), scn.tau.copy()
    for t in range(15):
        moved, req, length = st.step(mode, want_detail=True)
        code, ids, tau, req2, len2, moved2 = ref.step_range(
            code, ids, tau, mode=mode, t=t, seed=scn.seed, rho=scn.rho, dtau=scn.dtau,
            alpha=alpha, beta=beta, S=S_, M=M)
        assert moved == moved2 and np.array_equal(req, req2) and np.array_equal(length, len2)
        assert np.array_equal(st.code, code) and np.array_equal(st.ids, ids)
        assert np.array_equal(st.tau.view(np.uint32), tau.view(np.uint32))


def test_bad_ranges_rejected():
    st = oracle.State.from_scenario(S.make_scenario(20, 8, 5, 5, band_a=2, seed=1, mode=0))
    for bad in ((0, 1), (2, 3), (9, 1), (3, 0)):
        st.ranges = bad
        with pytest.raises(ValueError):
            st.step(oracle.MODE_LEM)
