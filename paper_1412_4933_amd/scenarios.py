"""Seeded synthetic scenarios for the bi-directional pedestrian update.

This module only builds initial states (which cells are walls, where agents
stand, which id each agent carries, the initial pheromone value). It holds
none of the step's arithmetic, so the oracle tests and the HIP path can both
be fed from it.

Frame (the paper places its two groups at the top and bottom of the grid,
Sec. III and Sec. IV.a; here the frame is rotated so the groups walk along x):
  * x = column 0..W-1, y = row 0..H-1, cell (x, y) at flat index y*W + x;
  * rows 0 and H-1 are walls (code 3), anything outside the grid counts as wall;
  * group A (code 1) starts in the leftmost band and heads +x,
    group B (code 2) starts in the rightmost band and heads -x;
  * agents are placed uniformly at random without overlap inside their band
    (the paper confines each group's random initial placement to a fixed
    number of rows at its side, Sec. III and Sec. VI);
  * ids are 1..N assigned row-major over the initial grid; 0 marks a cell
    without an agent.

Band rule: a stated band that cannot hold its group is widened to the
narrowest band whose free cells can (the paper's own bands grow with the
population, Sec. VI).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Tuple, List, Optional

import numpy as np

EMPTY, GROUP_A, GROUP_B, WALL = 0, 1, 2, 3
MODE_LEM, MODE_ACO, MODE_ACO_TOUR = 0, 1, 2


@dataclasses.dataclass
class Scenario:
    """One initial state plus the parameters the step needs."""

    W: int
    H: int
    code: np.ndarray  # uint8 [H, W]
    ids: np.ndarray  # uint32 [H, W]
    tau: Optional[np.ndarray]  # float32 [2, H, W] (plane 0 = group A) or None
    seed: int
    band_a: int
    band_b: int
    n_a: int
    n_b: int
    mode: int = MODE_ACO
    steps: int = 0
    tau0: float = 1.0
    rho: float = 0.1
    dtau: float = 1.0
    alpha: int = 1
    beta: int = 2
    tour: Optional[np.ndarray] = None  # float32 [N] initial tour lengths (tour variant), None = zeros
    neighbours: int = 5  # 5: F, FD+-, L+- (no backward cells); 8: all eight neighbours
    ranges: Optional[Tuple[int, int]] = None  # (scanning range, moving range); None: the base step

    @property
    def cross_a(self) -> int:
        """B has crossed once x < cross_a (A's starting band)."""
        return self.band_a

    @property
    def cross_b(self) -> int:
        """A has crossed once x >= W - cross_b (B's starting band)."""
        return self.band_b

    @property
    def agents(self) -> int:
        return self.n_a + self.n_b

    def copy(self) -> "Scenario":
        return dataclasses.replace(
            self,
            code=self.code.copy(),
            ids=self.ids.copy(),
            tau=None if self.tau is None else self.tau.copy(),
            tour=None if self.tour is None else self.tour.copy(),
        )


def wall_frame(W: int, H: int) -> np.ndarray:
    code = np.zeros((H, W), dtype=np.uint8)
    code[0, :] = WALL
    code[H - 1, :] = WALL
    return code


def add_obstacles(code: np.ndarray, rng: np.random.Generator, frac: float,
                  min_side: int = 2, max_side: int = 16) -> None:
    """Random axis-aligned wall rectangles (sides uniform in
    [min_side, max_side], top-left uniform over the interior rows), added until
    at least `frac` of the interior cells are walls. Overlaps are allowed;
    rectangles are clipped to the interior."""
    H, W = code.shape
    interior = (H - 2) * W
    target = int(math.ceil(frac * interior))
    walls = int(np.count_nonzero(code[1:H - 1, :] == WALL))
    while walls < target:
        w = int(rng.integers(min_side, max_side + 1))
        h = int(rng.integers(min_side, max_side + 1))
        x0 = int(rng.integers(0, W))
        y0 = int(rng.integers(1, H - 1))
        x1, y1 = min(W, x0 + w), min(H - 1, y0 + h)
        code[y0:y1, x0:x1] = WALL
        walls = int(np.count_nonzero(code[1:H - 1, :] == WALL))


def _band_width(code: np.ndarray, n: int, stated: int, left: bool) -> int:
    H, W = code.shape
    free_per_col = np.count_nonzero(code == EMPTY, axis=0)
    if not left:
        free_per_col = free_per_col[::-1]
    cum = np.cumsum(free_per_col)
    if n > 0 and cum[-1] < n:
        raise ValueError(f"grid cannot hold {n} agents in one group")
    need = int(np.searchsorted(cum, n) + 1) if n > 0 else 0
    return max(stated, need)


def place_groups(code: np.ndarray, n_a: int, n_b: int, band_a: int,
                 band_b: int, rng: np.random.Generator):
    """Place n_a agents in columns [0, b_a) and n_b in [W-b_b, W), uniformly
    without replacement over each band's free cells; returns (ids, b_a, b_b)."""
    H, W = code.shape
    b_a = _band_width(code, n_a, band_a, left=True)
    b_b = _band_width(code, n_b, band_b, left=False)
    if b_a + b_b > W:
        raise ValueError(f"bands {b_a}+{b_b} overlap on a {W}-wide grid")
    for g, n, x0, x1 in ((GROUP_A, n_a, 0, b_a), (GROUP_B, n_b, W - b_b, W)):
        sub = code[:, x0:x1]
        ys, xs = np.nonzero(sub == EMPTY)
        pick = rng.choice(ys.size, size=n, replace=False)
        sub[ys[pick], xs[pick]] = g
    ids = np.zeros((H, W), dtype=np.uint32)
    occ = (code == GROUP_A) | (code == GROUP_B)
    ids[occ] = np.arange(1, int(np.count_nonzero(occ)) + 1, dtype=np.uint32)
    return ids, b_a, b_b


def make_scenario(W: int, H: int, n_a: int, n_b: int, *, band_a: int,
                  band_b: Optional[int] = None, seed: int = 1,
                  mode: int = MODE_ACO, steps: int = 0, obstacle_frac: float = 0.0,
                  tau0: float = 1.0, rho: float = 0.1, dtau: float = 1.0,
                  alpha: int = 1, beta: int = 2, with_tau: Optional[bool] = None,
                  neighbours: int = 5, ranges: Optional[Tuple[int, int]] = None) -> Scenario:
    """Build one seeded scenario; `seed` drives placement and is also the
    step's RNG key."""
    if band_b is None:
        band_b = band_a
    rng = np.random.default_rng(seed)
    code = wall_frame(W, H)
    if obstacle_frac > 0:
        add_obstacles(code, rng, obstacle_frac)
    ids, b_a, b_b = place_groups(code, n_a, n_b, band_a, band_b, rng)
    if with_tau is None:
        with_tau = mode in (MODE_ACO, MODE_ACO_TOUR)
    tau = np.full((2, H, W), np.float32(tau0), dtype=np.float32) if with_tau else None
    return Scenario(W=W, H=H, code=code, ids=ids, tau=tau, seed=seed, band_a=b_a,
                    band_b=b_b, n_a=n_a, n_b=n_b, mode=mode, steps=steps, tau0=tau0,
                    rho=rho, dtau=dtau, alpha=alpha, beta=beta, neighbours=neighbours,
                    ranges=ranges)


def from_grid(code: np.ndarray, *, seed: int = 1, band_a: int = 1, band_b: int = 1,
              tau: Optional[np.ndarray] = None, mode: int = MODE_LEM, **kw) -> Scenario:
    """Wrap a hand-built code grid (ids assigned row-major)."""
    code = np.ascontiguousarray(code, dtype=np.uint8)
    H, W = code.shape
    ids = np.zeros((H, W), dtype=np.uint32)
    occ = (code == GROUP_A) | (code == GROUP_B)
    ids[occ] = np.arange(1, int(np.count_nonzero(occ)) + 1, dtype=np.uint32)
    return Scenario(W=W, H=H, code=code, ids=ids, tau=tau, seed=seed, band_a=band_a,
                    band_b=band_b, n_a=int(np.count_nonzero(code == GROUP_A)),
                    n_b=int(np.count_nonzero(code == GROUP_B)), mode=mode, **kw)


# ---------------------------------------------------------------------------
# Named workloads (sizes follow the paper's 2K-100K-agent range, Sec. III).
# ---------------------------------------------------------------------------

def lem_200x100(seed: int = 1) -> Scenario:
    """LEM, 200x100, 1,000 agents per group in 10-column bands (widened by the
    band rule to 11), 500 steps."""
    return make_scenario(200, 100, 1000, 1000, band_a=10, seed=seed, mode=MODE_LEM,
                         steps=500)


def aco_1024x512(seed: int = 1) -> Scenario:
    """ACO, 1024x512, 50,000 agents per group in 64-column bands (widened to
    99), tau0=1, rho=0.1, dtau=1, alpha=1, beta=2, 2,000 steps."""
    return make_scenario(1024, 512, 50000, 50000, band_a=64, seed=seed, mode=MODE_ACO,
                         steps=2000)


def aco_tour_1024x512(seed: int = 1) -> Scenario:
    """The 1024x512 ACO workload run with the tour variant (eq. 5 deposits)."""
    return make_scenario(1024, 512, 50000, 50000, band_a=64, seed=seed, mode=MODE_ACO_TOUR,
                         steps=2000)


def aco_nb8_1024x512(seed: int = 1) -> Scenario:
    """The 1024x512 ACO workload with the paper's full eight-neighbour
    candidate set (backward cells ranked last)."""
    return make_scenario(1024, 512, 50000, 50000, band_a=64, seed=seed, mode=MODE_ACO,
                         steps=2000, neighbours=8)


def range_1024x512(mode: int = MODE_ACO, scan: int = 4, move: int = 2, seed: int = 1) -> Scenario:
    """The 1024x512 workload (50,000 agents per group, same ACO parameters,
    2,000 steps) with larger scanning and moving ranges (the paper's future
    work, Sec. VII): by default agents scan 4 cells along each ray and move up
    to 2 cells per step."""
    return make_scenario(1024, 512, 50000, 50000, band_a=64, seed=seed, mode=mode,
                         steps=2000, with_tau=True, ranges=(scan, move))


def stress_4096x2048(mode: int = MODE_ACO, seed: int = 1) -> Scenario:
    """4096x2048 with 5% of interior cells covered by 2..16-cell rectangles,
    500,000 agents per group, 1,000 steps."""
    return make_scenario(4096, 2048, 500000, 500000, band_a=64, seed=seed, mode=mode,
                         steps=1000, obstacle_frac=0.05, with_tau=True)


def paper_sweep(densities=range(1, 21), repeats: int = 10, steps: int = 25000,
                modes=(MODE_LEM, MODE_ACO), size: int = 480, neighbours: int = 5) -> List[Scenario]:
    """The population sweep of the paper's results (Sec. VI): a size x size
    grid, 1,280 k agents per group for density k (2,560 k in all), each group
    packed into the narrowest band that holds it (3 columns for k = 1), a
    crossing line at the opposite group's band, `steps` steps, `repeats`
    placements per density. The runs of one (k, repeat) in each of `modes`
    share their placement and random key (seed 100 k + repeat), so the
    comparison is paired. Returns the scenarios ordered by (k, repeat, mode)."""
    out = []
    for k in densities:
        for rep in range(repeats):
            for mode in modes:
                out.append(make_scenario(size, size, 1280 * k, 1280 * k, band_a=1, seed=100 * k + rep,
                                         mode=mode, steps=steps, neighbours=neighbours))
    return out


def batch_shapes(count: int = 256, rng_seed: int = 0):
    """(W, H, N, band, mode) for a batch of independent scenarios: widths
    log-uniform in [64, 2048] rounded to even, H = W/2, populations log-uniform
    in [500, 100000] rounded to even and capped so each band fits in a quarter
    of the width, stated band ceil(W/16), LEM for even index, ACO for odd."""
    rng = np.random.default_rng(rng_seed)
    out = []
    for i in range(count):
        W = int(2 * round(math.exp(rng.uniform(math.log(64), math.log(2048))) / 2))
        H = W // 2
        N = int(2 * round(math.exp(rng.uniform(math.log(500), math.log(100000))) / 2))
        N = min(N, 2 * (W // 4) * (H - 2))
        out.append((W, H, N, int(math.ceil(W / 16)), MODE_LEM if i % 2 == 0 else MODE_ACO))
    return out


def batched_256(count: int = 256, steps: int = 1000) -> List[Scenario]:
    """The batch of independent scenarios; scenario i uses seed i."""
    out = []
    for i, (W, H, N, band, mode) in enumerate(batch_shapes(count)):
        out.append(make_scenario(W, H, N // 2, N // 2, band_a=band, seed=i, mode=mode,
                                 steps=steps))
    return out


def served_requests(count: int = 512, rng_seed: int = 1):
    """Request stream for the serving loop: shapes drawn as in `batch_shapes`
    (own rng), step counts uniform in [200, 2000]. Returns a list of
    (W, H, N, band, mode, steps, seed)."""
    shapes = batch_shapes(count, rng_seed)
    rng = np.random.default_rng(rng_seed + 1000)
    out = []
    for i, (W, H, N, band, mode) in enumerate(shapes):
        out.append((W, H, N, band, mode, int(rng.integers(200, 2001)), 1000 + i))
    return out
