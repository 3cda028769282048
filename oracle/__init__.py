"""ctypes wrapper of the plain CPU oracle (pedsim_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may use this package; the library never does. It builds the
oracle with gcc (-O2 -ffp-contract=off, plain loops) on first use if a shared
object is missing, and `build()` rebuilds both unconditionally:
  libpedsim_oracle.so      the plain build, one thread;
  libpedsim_oracle_omp.so  the same source with -fopenmp, whose parallel loops
                           write disjoint cells, so its results are identical.
`State(..., threads=n)` runs on the OpenMP build with n threads; the default
(threads=None) is the plain build.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pedsim_oracle.c")
_LIB = os.path.join(_HERE, "libpedsim_oracle.so")
_LIB_OMP = os.path.join(_HERE, "libpedsim_oracle_omp.so")
# The mutation tests point this at a deliberately broken build of the oracle.
_LIB_OVERRIDE = os.environ.get("PEDSIM_ORACLE_LIB")

MODE_LEM, MODE_ACO, MODE_ACO_TOUR = 0, 1, 2


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("W", ctypes.c_int32), ("H", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("rho", ctypes.c_float), ("dtau", ctypes.c_float),
        ("alpha", ctypes.c_int32), ("beta", ctypes.c_int32),
        ("cross_a", ctypes.c_int32), ("cross_b", ctypes.c_int32),
        ("neighbours", ctypes.c_int32),
    ]


_FLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def _compile(out: str, extra) -> str:
    tmp = out + ".tmp"
    subprocess.run(["gcc", *_FLAGS, *extra, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, out)
    return out


def build() -> str:
    """Compile the oracle into oracle/libpedsim_oracle.so (one thread) and
    oracle/libpedsim_oracle_omp.so (OpenMP)."""
    _compile(_LIB_OMP, ["-fopenmp"])
    return _compile(_LIB, [])


_libs = {}


def cpu_threads() -> int:
    """Host threads this process may use (its CPU affinity), at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def lib(parallel: bool = False):
    """The plain oracle build, or with parallel=True the OpenMP build."""
    L = _libs.get(parallel)
    if L is None:
        target = _LIB_OMP if parallel else _LIB
        path = _LIB_OVERRIDE or target
        if not _LIB_OVERRIDE and not os.path.exists(target):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        L.oracle_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32),
                                           P(ctypes.c_uint32)]
        L.oracle_philox4x32_10.restype = None
        L.oracle_lem_thresholds.argtypes = [P(ctypes.c_uint32)]
        L.oracle_heuristic_weights.argtypes = [ctypes.c_int32, P(ctypes.c_float)]
        L.oracle_step.argtypes = [P(OracleParams), ctypes.c_int32, ctypes.c_uint64,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_step.restype = ctypes.c_int64
        L.oracle_run.argtypes = [P(OracleParams), ctypes.c_int32, ctypes.c_uint64,
                                 ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_run.restype = ctypes.c_int64
        L.oracle_step_tour.argtypes = [P(OracleParams), ctypes.c_uint64, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_step_tour.restype = ctypes.c_int64
        L.oracle_run_tour.argtypes = [P(OracleParams), ctypes.c_uint64, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_run_tour.restype = ctypes.c_int64
        L.oracle_counts.argtypes = [P(OracleParams), ctypes.c_void_p, P(ctypes.c_uint64)]
        L.oracle_step_range.argtypes = [P(OracleParams), ctypes.c_int32, ctypes.c_uint64,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_step_range.restype = ctypes.c_int64
        L.oracle_run_range.argtypes = [P(OracleParams), ctypes.c_int32, ctypes.c_uint64,
                                       ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]
        L.oracle_run_range.restype = ctypes.c_int64
        L.oracle_range_weights.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           P(ctypes.c_float), P(ctypes.c_float)]
        L.oracle_range_weights.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = ctypes.c_int
        _libs[parallel] = L
    return L


def philox4x32_10(ctr, key) -> Tuple[int, int, int, int]:
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return tuple(int(v) for v in o)


def agent_words(seed: int, t: int, k: int):
    """The four Philox words agent k draws in step t under `seed`."""
    return philox4x32_10((k, t & 0xFFFFFFFF, t >> 32, 0),
                         (seed & 0xFFFFFFFF, seed >> 32))


def lem_thresholds():
    o = (ctypes.c_uint32 * 6)()
    lib().oracle_lem_thresholds(o)
    return tuple(int(v) for v in o)


def range_weights(S: int, M: int, beta: int):
    """eta^beta of the side rays with ranges (S, M): (diagonal, lateral),
    each indexed by the free run f - 1 for f = 1..S."""
    d = (ctypes.c_float * 8)()
    la = (ctypes.c_float * 8)()
    lib().oracle_range_weights(int(S), int(M), int(beta), d, la)
    return ([np.float32(v) for v in d[:S]], [np.float32(v) for v in la[:S]])


def heuristic_weights(beta: int):
    """(eta^beta) for the forward, diagonal, lateral, backward and backward
    diagonal candidates."""
    o = (ctypes.c_float * 5)()
    lib().oracle_heuristic_weights(int(beta), o)
    return tuple(np.float32(v) for v in o)


class State:
    """Host copy of one scenario's planes, advanced by the oracle.

    `tour` is the tour matrix of the tour variant (one float per agent,
    index = agent number = id - 1); zeros when not given. `threads` (an int)
    runs every call on the OpenMP build with that many threads; None runs the
    plain one-thread build."""

    def __init__(self, code, ids, tau=None, *, seed: int, rho: float = 0.1,
                 dtau: float = 1.0, alpha: int = 1, beta: int = 2, cross_a: int = 1,
                 cross_b: int = 1, t: int = 0, tour=None, neighbours: int = 5,
                 threads: Optional[int] = None, ranges: Optional[Tuple[int, int]] = None):
        self.code = np.ascontiguousarray(code, dtype=np.uint8).copy()
        self.ids = np.ascontiguousarray(ids, dtype=np.uint32).copy()
        self.H, self.W = self.code.shape
        n = int(self.ids.max()) if self.ids.size else 0
        if tour is None:
            self.tour = np.zeros(n, np.float32)
        else:
            self.tour = np.ascontiguousarray(tour, dtype=np.float32).copy()
            assert self.tour.shape == (n,)
        if tau is None:
            self.tau = None
        else:
            self.tau = np.ascontiguousarray(tau, dtype=np.float32).copy()
            assert self.tau.shape == (2, self.H, self.W)
        self.p = OracleParams(self.W, self.H, seed, rho, dtau, alpha, beta, cross_a,
                              cross_b, neighbours)
        self.t = t
        self.threads = threads
        # (scanning range S, moving range M): steps follow the range model
        # (oracle_step_range), also for (1, 1); None: the base step
        self.ranges = None if ranges is None else (int(ranges[0]), int(ranges[1]))

    @classmethod
    def from_scenario(cls, s, threads: Optional[int] = None) -> "State":
        return cls(s.code, s.ids, s.tau, seed=s.seed, rho=s.rho, dtau=s.dtau,
                   alpha=s.alpha, beta=s.beta, cross_a=s.cross_a, cross_b=s.cross_b,
                   tour=getattr(s, "tour", None), neighbours=getattr(s, "neighbours", 5),
                   threads=threads, ranges=getattr(s, "ranges", None))

    def _lib(self):
        """The build this state runs on; the OpenMP build's thread count is a
        per-calling-thread setting, so it is set before every call."""
        if self.threads is None:
            return lib()
        L = lib(parallel=True)
        L.oracle_set_threads(int(self.threads))
        return L

    def _tau_ptrs(self, mode):
        if mode in (MODE_ACO, MODE_ACO_TOUR):
            if self.tau is None:
                raise ValueError("ACO step needs pheromone planes")
            return self.tau[0].ctypes.data, self.tau[1].ctypes.data
        return None, None

    def step(self, mode: int, want_detail: bool = False):
        """One step; returns moved, or (moved, req, win) with want_detail
        (with ranges: (moved, ray, length))."""
        ta, tb = self._tau_ptrs(mode)
        if self.ranges is not None:
            req = length = None
            if want_detail:
                req = np.zeros((self.H, self.W), dtype=np.uint8)
                length = np.zeros((self.H, self.W), dtype=np.uint8)
            moved = self._lib().oracle_step_range(
                ctypes.byref(self.p), mode, self.t, self.ranges[0], self.ranges[1],
                self.code.ctypes.data, self.ids.ctypes.data, ta, tb,
                None if req is None else req.ctypes.data,
                None if length is None else length.ctypes.data)
            if moved == -2:
                raise ValueError(f"bad ranges {self.ranges} or mode {mode}")
            if moved < 0:
                raise MemoryError("oracle step failed to allocate")
            self.t += 1
            return (moved, req, length) if want_detail else moved
        req = win = None
        if want_detail:
            req = np.zeros((self.H, self.W), dtype=np.uint8)
            win = np.zeros((self.H, self.W), dtype=np.uint8)
        rq = None if req is None else req.ctypes.data
        wn = None if win is None else win.ctypes.data
        if mode == MODE_ACO_TOUR:
            moved = self._lib().oracle_step_tour(ctypes.byref(self.p), self.t, self.code.ctypes.data,
                                           self.ids.ctypes.data, ta, tb,
                                           self.tour.ctypes.data if self.tour.size else None,
                                           rq, wn)
        else:
            moved = self._lib().oracle_step(ctypes.byref(self.p), mode, self.t, self.code.ctypes.data,
                                      self.ids.ctypes.data, ta, tb, rq, wn)
        if moved < 0:
            raise MemoryError("oracle step failed to allocate")
        self.t += 1
        return (moved, req, win) if want_detail else moved

    def run(self, mode: int, nsteps: int) -> int:
        ta, tb = self._tau_ptrs(mode)
        if self.ranges is not None:
            moved = self._lib().oracle_run_range(ctypes.byref(self.p), mode, self.t, nsteps,
                                                 self.ranges[0], self.ranges[1],
                                                 self.code.ctypes.data, self.ids.ctypes.data, ta, tb)
            if moved == -2:
                raise ValueError(f"bad ranges {self.ranges} or mode {mode}")
            if moved < 0:
                raise MemoryError("oracle step failed to allocate")
            self.t += nsteps
            return moved
        if mode == MODE_ACO_TOUR:
            moved = self._lib().oracle_run_tour(ctypes.byref(self.p), self.t, nsteps,
                                          self.code.ctypes.data, self.ids.ctypes.data, ta, tb,
                                          self.tour.ctypes.data if self.tour.size else None)
        else:
            moved = self._lib().oracle_run(ctypes.byref(self.p), mode, self.t, nsteps,
                                     self.code.ctypes.data, self.ids.ctypes.data, ta, tb)
        if moved < 0:
            raise MemoryError("oracle step failed to allocate")
        self.t += nsteps
        return moved

    def counts(self):
        """(agents_a, agents_b, crossed_a, crossed_b)."""
        o = (ctypes.c_uint64 * 4)()
        self._lib().oracle_counts(ctypes.byref(self.p), self.code.ctypes.data, o)
        return tuple(int(v) for v in o)
