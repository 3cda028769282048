"""Python binding of the pedsim C ABI (include/pedsim.h).

Argument marshalling only: every step runs in the HIP kernels of
libpedsim.so. PyTorch provides device memory (tensors) and streams. The
library must have been built (`python -m paper_1412_4933_amd.build` or
`__graft_entry__.build()`); if it is missing, loading fails loudly rather than
falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpedsim.so")

SIM_OK, SIM_EINVAL, SIM_ESTATE, SIM_ESCRATCH, SIM_EHIP, SIM_ENOTAU, SIM_EFULL = 0, -1, -2, -3, -4, -5, -6
SIM_ENOTOUR = -7
SIM_MODE_LEM, SIM_MODE_ACO, SIM_MODE_ACO_TOUR = 0, 1, 2
# A batch tuning (nw, rows, steps per launch, threads, workgroups per CU) of
# the row-lane engine with the pheromone in LDS, which tour-variant scenarios
# need before they can be added (the library's own default for that form).
LDS_BATCH_TUNING = (0, 48, 3, 512, 2)


class SimError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        detail = ""
        if code == SIM_EHIP:
            detail = " [" + lib().sim_last_error().decode(errors="replace") + "]"
        super().__init__(f"{what}: {sim_strerror(code)} ({code}){detail}")


class SimParams(ctypes.Structure):
    _fields_ = [
        ("W", ctypes.c_int32), ("H", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("step0", ctypes.c_uint64),
        ("rho", ctypes.c_float), ("dtau", ctypes.c_float),
        ("alpha", ctypes.c_int32), ("beta", ctypes.c_int32),
        ("cross_a", ctypes.c_int32), ("cross_b", ctypes.c_int32),
    ]


class SimStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("step", "agents_a", "agents_b", "crossed_a", "crossed_b", "moved_last")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        # torch's HIP runtime must be the one in the process before the library
        # is loaded: torch asks the dynamic linker for a runtime by a name that
        # does not match the versioned name the library links against, so the
        # library loaded first would leave two HIP runtimes side by side.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        P = ctypes.POINTER
        L.sim_strerror.argtypes = [ctypes.c_int]
        L.sim_strerror.restype = ctypes.c_char_p
        L.sim_last_error.argtypes = []
        L.sim_last_error.restype = ctypes.c_char_p
        L.sim_scratch_bytes.argtypes = [P(SimParams), P(sz)]
        L.sim_create.argtypes = [P(SimParams), vp, vp, vp, vp, sz, vp, P(vp)]
        L.sim_step_lem.argtypes = [vp, i32, vp]
        L.sim_step_aco.argtypes = [vp, i32, vp]
        L.sim_step_aco_tour.argtypes = [vp, i32, vp]
        L.sim_attach_tour.argtypes = [vp, vp, vp, vp]
        L.sim_set_neighbours.argtypes = [vp, i32]
        L.sim_set_ranges.argtypes = [vp, i32, i32]
        L.sim_set_range_tiling.argtypes = [vp, i32, i32, i32, i32]
        L.sim_get_range_tiling.argtypes = [vp, P(ctypes.c_int32)]
        L.sim_range_weights.argtypes = [i32, i32, i32, P(ctypes.c_float), P(ctypes.c_float)]
        L.sim_stats.argtypes = [vp, P(SimStats), vp]
        L.sim_run_noalloc.argtypes = [P(SimParams), i32, vp, vp, vp, i32, vp, P(SimStats)]
        L.sim_read_state.argtypes = [vp, vp, vp, vp, vp]
        L.sim_step_timed.argtypes = [vp, i32, i32, vp, P(ctypes.c_double), P(ctypes.c_int64), i32]
        L.sim_step_timed.restype = ctypes.c_int
        L.sim_set_tiling.argtypes = [vp, i32, i32, i32, i32, i32]
        L.sim_set_tiling.restype = ctypes.c_int
        L.sim_get_tiling.argtypes = [vp, i32, P(ctypes.c_int32)]
        L.sim_get_tiling.restype = ctypes.c_int
        L.sim_kernel_name.argtypes = [i32]
        L.sim_kernel_name.restype = ctypes.c_char_p
        L.sim_destroy.argtypes = [vp]
        L.sim_destroy.restype = None
        for name in ("sim_scratch_bytes", "sim_create", "sim_step_lem", "sim_step_aco",
                     "sim_step_aco_tour", "sim_attach_tour", "sim_set_neighbours", "sim_stats",
                     "sim_read_state", "sim_set_ranges", "sim_set_range_tiling", "sim_get_range_tiling",
                     "sim_range_weights", "sim_run_noalloc"):
            getattr(L, name).restype = ctypes.c_int
        _bind_batch(L)
        _lib = L
    return _lib


def _bind_batch(L):
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    P = ctypes.POINTER
    L.sim_batch_workspace_bytes.argtypes = [i32, P(sz)]
    L.sim_batch_create.argtypes = [i32, vp, sz, P(vp)]
    L.sim_batch_add.argtypes = [vp, P(SimParams), i32, vp, vp, vp, vp, sz, vp, P(i32)]
    L.sim_batch_remove.argtypes = [vp, i32]
    L.sim_batch_step.argtypes = [vp, i32, vp]
    L.sim_batch_step_slots.argtypes = [vp, P(i32), i32, vp]
    L.sim_batch_stats.argtypes = [vp, i32, P(SimStats), vp]
    L.sim_batch_set_tuning.argtypes = [vp, i32, i32, i32, i32, i32, i32]
    L.sim_batch_get_tuning.argtypes = [vp, P(i32)]
    L.sim_batch_set_neighbours.argtypes = [vp, i32]
    L.sim_batch_attach_tour.argtypes = [vp, i32, vp, vp, vp]
    L.sim_batch_destroy.argtypes = [vp]
    L.sim_batch_destroy.restype = None
    for name in ("sim_batch_workspace_bytes", "sim_batch_create", "sim_batch_add", "sim_batch_remove",
                 "sim_batch_step", "sim_batch_step_slots", "sim_batch_stats", "sim_batch_set_tuning",
                 "sim_batch_get_tuning", "sim_batch_set_neighbours", "sim_batch_attach_tour"):
        getattr(L, name).restype = ctypes.c_int


def _check(code: int, what: str) -> None:
    if code != SIM_OK:
        raise SimError(code, what)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# --- the C ABI, name for name -------------------------------------------------

def sim_strerror(code: int) -> str:
    return lib().sim_strerror(int(code)).decode()


def sim_scratch_bytes(params: SimParams) -> int:
    out = ctypes.c_size_t()
    _check(lib().sim_scratch_bytes(ctypes.byref(params), ctypes.byref(out)), "sim_scratch_bytes")
    return int(out.value)


def sim_create(params: SimParams, code, ids, tau, scratch, scratch_bytes: int, stream=None):
    h = ctypes.c_void_p()
    _check(lib().sim_create(ctypes.byref(params), _ptr(code), _ptr(ids), _ptr(tau), _ptr(scratch),
                            int(scratch_bytes), _stream(stream), ctypes.byref(h)), "sim_create")
    return h


def sim_step_lem(h, nsteps: int, stream=None) -> None:
    _check(lib().sim_step_lem(h, int(nsteps), _stream(stream)), "sim_step_lem")


def sim_step_aco(h, nsteps: int, stream=None) -> None:
    _check(lib().sim_step_aco(h, int(nsteps), _stream(stream)), "sim_step_aco")


def sim_attach_tour(h, tour, tour_shadow, stream=None) -> None:
    _check(lib().sim_attach_tour(h, _ptr(tour), _ptr(tour_shadow), _stream(stream)), "sim_attach_tour")


def sim_set_neighbours(h, n: int) -> None:
    _check(lib().sim_set_neighbours(h, int(n)), "sim_set_neighbours")


def sim_set_ranges(h, scan: int, move: int) -> None:
    _check(lib().sim_set_ranges(h, int(scan), int(move)), "sim_set_ranges")


def sim_set_range_tiling(h, cols: int, rows: int, steps_per_launch: int, threads: int) -> None:
    _check(lib().sim_set_range_tiling(h, int(cols), int(rows), int(steps_per_launch), int(threads)),
           "sim_set_range_tiling")


def sim_get_range_tiling(h):
    out = (ctypes.c_int32 * 4)()
    _check(lib().sim_get_range_tiling(h, out), "sim_get_range_tiling")
    return tuple(int(v) for v in out)


def sim_range_weights(scan: int, move: int, beta: int):
    """(diagonal[8], lateral[8]) heuristic weights of the range step (host only)."""
    d = (ctypes.c_float * 8)()
    la = (ctypes.c_float * 8)()
    _check(lib().sim_range_weights(int(scan), int(move), int(beta), d, la), "sim_range_weights")
    return np.array(d[:], np.float32), np.array(la[:], np.float32)


def sim_run_noalloc(params: SimParams, mode: int, code, ids, tau, nsteps: int, stream=None) -> dict:
    """Create, step and count in one call with the library's static scratch
    (no allocation); the planes hold the new state afterwards."""
    s = SimStats()
    _check(lib().sim_run_noalloc(ctypes.byref(params), int(mode), _ptr(code), _ptr(ids), _ptr(tau),
                                 int(nsteps), _stream(stream), ctypes.byref(s)), "sim_run_noalloc")
    return s.as_dict()


def sim_step_aco_tour(h, nsteps: int, stream=None) -> None:
    _check(lib().sim_step_aco_tour(h, int(nsteps), _stream(stream)), "sim_step_aco_tour")


def sim_stats(h, stream=None) -> dict:
    s = SimStats()
    _check(lib().sim_stats(h, ctypes.byref(s), _stream(stream)), "sim_stats")
    return s.as_dict()


def sim_read_state(h, code, ids, tau, stream=None) -> None:
    _check(lib().sim_read_state(h, _ptr(code), _ptr(ids), _ptr(tau), _stream(stream)),
           "sim_read_state")


def sim_step_timed(h, mode: int, nsteps: int, stream=None) -> dict:
    """Per-kernel-kind {name: (total_ms, launches)} over nsteps timed steps."""
    n = 8
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    rc = lib().sim_step_timed(h, int(mode), int(nsteps), _stream(stream), ms, cnt, n)
    if rc < 0:
        raise SimError(rc, "sim_step_timed")
    return {lib().sim_kernel_name(k).decode(): (float(ms[k]), int(cnt[k])) for k in range(rc)}


def sim_set_tiling(h, mode: int, nw: int, rows: int, steps_per_launch: int, threads: int) -> None:
    _check(lib().sim_set_tiling(h, int(mode), int(nw), int(rows), int(steps_per_launch), int(threads)),
           "sim_set_tiling")


def sim_get_tiling(h, mode: int):
    out = (ctypes.c_int32 * 4)()
    _check(lib().sim_get_tiling(h, int(mode), out), "sim_get_tiling")
    return tuple(int(v) for v in out)


def sim_kernel_name(kind: int) -> str:
    return lib().sim_kernel_name(int(kind)).decode()


def sim_destroy(h) -> None:
    if h:
        lib().sim_destroy(h)


def sim_batch_workspace_bytes(capacity: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().sim_batch_workspace_bytes(int(capacity), ctypes.byref(out)), "sim_batch_workspace_bytes")
    return int(out.value)


def sim_batch_create(capacity: int, workspace, workspace_bytes: int):
    b = ctypes.c_void_p()
    _check(lib().sim_batch_create(int(capacity), _ptr(workspace), int(workspace_bytes), ctypes.byref(b)),
           "sim_batch_create")
    return b


def sim_batch_add(b, params: SimParams, mode: int, code, ids, tau, scratch, scratch_bytes: int,
                  stream=None) -> int:
    slot = ctypes.c_int32()
    _check(lib().sim_batch_add(b, ctypes.byref(params), int(mode), _ptr(code), _ptr(ids), _ptr(tau),
                               _ptr(scratch), int(scratch_bytes), _stream(stream), ctypes.byref(slot)),
           "sim_batch_add")
    return int(slot.value)


def sim_batch_remove(b, slot: int) -> None:
    _check(lib().sim_batch_remove(b, int(slot)), "sim_batch_remove")


def sim_batch_step(b, nsteps: int, stream=None) -> None:
    _check(lib().sim_batch_step(b, int(nsteps), _stream(stream)), "sim_batch_step")


def sim_batch_step_slots(b, steps, stream=None) -> None:
    arr = (ctypes.c_int32 * len(steps))(*[int(v) for v in steps])
    _check(lib().sim_batch_step_slots(b, arr, len(steps), _stream(stream)), "sim_batch_step_slots")


def sim_batch_stats(b, slot: int, stream=None) -> dict:
    s = SimStats()
    _check(lib().sim_batch_stats(b, int(slot), ctypes.byref(s), _stream(stream)), "sim_batch_stats")
    return s.as_dict()


def sim_batch_set_tuning(b, nw: int, rows: int, steps_per_launch: int, threads: int, wgs_per_cu: int,
                         use_graph: int = 1) -> None:
    _check(lib().sim_batch_set_tuning(b, int(nw), int(rows), int(steps_per_launch), int(threads),
                                      int(wgs_per_cu), int(use_graph)), "sim_batch_set_tuning")


def sim_batch_get_tuning(b):
    out = (ctypes.c_int32 * 6)()
    _check(lib().sim_batch_get_tuning(b, out), "sim_batch_get_tuning")
    return tuple(int(v) for v in out)


def sim_batch_attach_tour(b, slot: int, tour, tour_shadow, stream=None) -> None:
    _check(lib().sim_batch_attach_tour(b, int(slot), _ptr(tour), _ptr(tour_shadow), _stream(stream)),
           "sim_batch_attach_tour")


def sim_batch_set_neighbours(b, n: int) -> None:
    _check(lib().sim_batch_set_neighbours(b, int(n)), "sim_batch_set_neighbours")


def sim_batch_destroy(b) -> None:
    if b:
        lib().sim_batch_destroy(b)


# --- convenience: a scenario resident in torch device tensors -------------------

def params_of(s, step0: int = 0) -> SimParams:
    """SimParams of a `scenarios.Scenario`."""
    return SimParams(s.W, s.H, s.seed, step0, s.rho, s.dtau, s.alpha, s.beta, s.cross_a,
                     s.cross_b)


class Sim:
    """One scenario resident on the GPU: device planes allocated with torch,
    stepped by the library. With autotune=True (the default) the tilings the
    autotuner's committed cache holds for this workload replace the library's
    defaults."""

    def __init__(self, scenario, device: str = "cuda", stream=None, step0: int = 0,
                 autotune: bool = True):
        import torch
        self.torch = torch
        self.scenario = scenario
        self.device = torch.device(device)
        self.stream = stream
        self.params = params_of(scenario, step0)
        self.code = torch.from_numpy(np.ascontiguousarray(scenario.code)).to(self.device)
        self.ids = torch.from_numpy(np.ascontiguousarray(scenario.ids).view(np.int32)).to(self.device)
        self.tau = None
        if scenario.tau is not None:
            self.tau = torch.from_numpy(np.ascontiguousarray(scenario.tau)).to(self.device)
        nbytes = sim_scratch_bytes(self.params)
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self.h = sim_create(self.params, self.code, self.ids, self.tau, self.scratch, nbytes,
                            stream)
        if getattr(scenario, "neighbours", 5) != 5:
            sim_set_neighbours(self.h, scenario.neighbours)
        self.ranges = getattr(scenario, "ranges", None)
        self.range_tuned = None
        if self.ranges is not None:
            sim_set_ranges(self.h, *self.ranges)
            if autotune:
                from . import autotune as tuner
                tl = tuner.cached_range(scenario, scenario.mode)
                if tl is not None:
                    try:
                        sim_set_range_tiling(self.h, *tl)
                        self.range_tuned = tuple(tl)
                    except SimError:  # not allowed on this device: keep the default
                        pass
        self.tuned = {}
        if autotune:
            from . import autotune as tuner
            for m in (SIM_MODE_LEM, SIM_MODE_ACO, SIM_MODE_ACO_TOUR):
                tl = tuner.cached_plain(scenario, m)
                if tl is None:
                    continue
                try:
                    sim_set_tiling(self.h, m, *tl)
                    self.tuned[m] = tuple(tl)
                except SimError:  # not allowed on this device: keep the default
                    pass
        # tour variant: the tour matrix (one float per agent) and its ping-pong half
        self.tour = self.tour_shadow = None
        if scenario.mode == SIM_MODE_ACO_TOUR or getattr(scenario, "tour", None) is not None:
            n = int(scenario.ids.max()) if scenario.ids.size else 0
            t0 = scenario.tour if getattr(scenario, "tour", None) is not None else np.zeros(n, np.float32)
            self.tour = torch.from_numpy(np.ascontiguousarray(t0, dtype=np.float32)).to(self.device)
            self.tour_shadow = torch.empty_like(self.tour)
            torch.cuda.synchronize(self.device)
            sim_attach_tour(self.h, self.tour if n else None, self.tour_shadow if n else None,
                            stream)

    def step(self, nsteps: int, mode: Optional[int] = None) -> None:
        mode = self.scenario.mode if mode is None else mode
        if mode == SIM_MODE_LEM:
            sim_step_lem(self.h, nsteps, self.stream)
        elif mode == SIM_MODE_ACO_TOUR:
            sim_step_aco_tour(self.h, nsteps, self.stream)
        else:
            sim_step_aco(self.h, nsteps, self.stream)

    def tour_lengths(self) -> np.ndarray:
        """The tour matrix (float32 [N], index = agent number) on the host."""
        s = self.stream if self.stream is not None else self.torch.cuda.current_stream(self.device)
        s.synchronize()
        return self.tour.cpu().numpy()

    def stats(self) -> dict:
        return sim_stats(self.h, self.stream)

    def set_tiling(self, mode: int, nw: int, rows: int, steps_per_launch: int, threads: int) -> None:
        sim_set_tiling(self.h, mode, nw, rows, steps_per_launch, threads)

    def tiling(self, mode: int):
        return sim_get_tiling(self.h, mode)

    def set_ranges(self, scan: int, move: int) -> None:
        """Scanning and moving ranges of later LEM/ACO steps ((0, 0): the base
        step); resets the range kernel's launch shape to the library default."""
        sim_set_ranges(self.h, scan, move)
        self.ranges = None if scan == 0 else (int(scan), int(move))
        self.range_tuned = None

    def set_range_tiling(self, cols: int, rows: int, steps_per_launch: int, threads: int) -> None:
        sim_set_range_tiling(self.h, cols, rows, steps_per_launch, threads)

    def range_tiling(self):
        return sim_get_range_tiling(self.h)

    def state(self):
        """(code, ids, tau) copied to host numpy arrays."""
        H, W = self.scenario.H, self.scenario.W
        code = np.empty((H, W), np.uint8)
        ids = np.empty((H, W), np.uint32)
        tau = np.empty((2, H, W), np.float32) if self.tau is not None else None
        sim_read_state(self.h, code.ctypes.data, ids.ctypes.data,
                       None if tau is None else tau.ctypes.data, self.stream)
        return code, ids, tau

    def close(self) -> None:
        if self.h:
            sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Resident:
    """Device planes and scratch of one scenario (torch tensors)."""

    def __init__(self, scenario, device, step0: int = 0):
        import torch
        self.scenario = scenario
        self.params = params_of(scenario, step0)
        self.code = torch.from_numpy(np.ascontiguousarray(scenario.code)).to(device)
        self.ids = torch.from_numpy(np.ascontiguousarray(scenario.ids).view(np.int32)).to(device)
        self.tau = None
        if scenario.tau is not None:
            self.tau = torch.from_numpy(np.ascontiguousarray(scenario.tau)).to(device)
        self.scratch_bytes = sim_scratch_bytes(self.params)
        self.scratch = torch.empty(self.scratch_bytes, dtype=torch.uint8, device=device)
        self.tour = self.tour_shadow = None
        if scenario.mode == SIM_MODE_ACO_TOUR:
            n = int(scenario.ids.max()) if scenario.ids.size else 0
            t0 = scenario.tour if getattr(scenario, "tour", None) is not None else np.zeros(n, np.float32)
            self.tour = torch.from_numpy(np.ascontiguousarray(t0, dtype=np.float32)).to(device)
            self.tour_shadow = torch.empty_like(self.tour)

    def clone(self) -> "_Resident":
        """A device copy of these planes (and tour arrays) with scratch of its
        own; nothing crosses PCIe."""
        out = _Resident.__new__(_Resident)
        out.scenario = self.scenario
        out.params = params_of(self.scenario, int(self.params.step0))
        out.code = self.code.clone()
        out.ids = self.ids.clone()
        out.tau = None if self.tau is None else self.tau.clone()
        out.scratch_bytes = self.scratch_bytes
        out.scratch = self.torch_empty_like(self.scratch)
        out.tour = None if self.tour is None else self.tour.clone()
        out.tour_shadow = None if self.tour_shadow is None else self.torch_empty_like(self.tour_shadow)
        return out

    @staticmethod
    def torch_empty_like(t):
        import torch
        return torch.empty_like(t)

    def nbytes(self) -> int:
        n = self.code.numel() + 4 * self.ids.numel() + self.scratch_bytes
        n += 8 * self.tour.numel() if self.tour is not None else 0
        return n + (4 * self.tau.numel() if self.tau is not None else 0)

    def state(self):
        code = self.code.cpu().numpy()
        ids = self.ids.cpu().numpy().view(np.uint32)
        tau = None if self.tau is None else self.tau.cpu().numpy()
        return code, ids, tau


class Batch:
    """Many scenarios resident on one GPU, advanced together by the batched
    kernel. Device memory comes from torch; slots are the library's.

    With autotune=True (the default), the first step call applies the
    autotuner's cached tuning for the resident scenarios if the committed
    cache holds one and no tuning was set explicitly; `tuning_source` says
    which tuning the batch runs ("library default", "autotuner cache" or
    "explicit")."""

    def __init__(self, capacity: int, device: str = "cuda", stream=None, autotune: bool = True):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream
        self.capacity = capacity
        nbytes = sim_batch_workspace_bytes(capacity)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.b = sim_batch_create(capacity, self.workspace, nbytes)
        self.members = {}
        self.neighbours = 5
        self.autotune = autotune
        self.tuning_source = "library default"

    def add(self, scenario, mode: Optional[int] = None, step0: int = 0) -> int:
        if getattr(scenario, "neighbours", 5) != self.neighbours:
            raise ValueError(f"scenario uses {scenario.neighbours} neighbours, the batch "
                             f"{self.neighbours} (set_neighbours first)")
        return self.add_resident(_Resident(scenario, self.device, step0), mode)

    def add_resident(self, res: "_Resident", mode: Optional[int] = None) -> int:
        """Add a scenario whose planes are already on the device."""
        mode = res.scenario.mode if mode is None else mode
        self.torch.cuda.synchronize(self.device)
        slot = sim_batch_add(self.b, res.params, mode, res.code, res.ids, res.tau, res.scratch,
                             res.scratch_bytes, self.stream)
        if res.tour is not None and res.tour.numel():
            sim_batch_attach_tour(self.b, slot, res.tour, res.tour_shadow, self.stream)
        self.members[slot] = res
        return slot

    def _autotune(self) -> None:
        if not self.autotune or self.tuning_source != "library default" or not self.members:
            return
        self.autotune = False  # looked up once, for the first call's residents
        from . import autotune as tuner
        tu = tuner.cached_batch([r.scenario for r in self.members.values()])
        if tu is not None:
            try:
                sim_batch_set_tuning(self.b, *tu, 1)
                self.tuning_source = "autotuner cache"
            except SimError:  # not allowed on this device or for these residents
                pass

    def remove(self, slot: int) -> None:
        sim_batch_remove(self.b, slot)
        self.members.pop(slot, None)

    def step(self, nsteps: int) -> None:
        self._autotune()
        sim_batch_step(self.b, nsteps, self.stream)

    def step_slots(self, steps) -> None:
        """steps: list indexed by slot, or {slot: steps}."""
        self._autotune()
        if isinstance(steps, dict):
            arr = [0] * self.capacity
            for k, v in steps.items():
                arr[k] = v
            steps = arr
        sim_batch_step_slots(self.b, steps, self.stream)

    def stats(self, slot: int) -> dict:
        return sim_batch_stats(self.b, slot, self.stream)

    def state(self, slot: int):
        s = self.stream if self.stream is not None else self.torch.cuda.current_stream(self.device)
        s.synchronize()
        return self.members[slot].state()

    def set_tuning(self, nw, rows, steps_per_launch, threads, wgs_per_cu, use_graph=1) -> None:
        sim_batch_set_tuning(self.b, nw, rows, steps_per_launch, threads, wgs_per_cu, use_graph)
        self.tuning_source = "explicit"

    def tuning(self):
        return sim_batch_get_tuning(self.b)

    def set_neighbours(self, n: int) -> None:
        for res in self.members.values():
            if getattr(res.scenario, "neighbours", 5) != n:
                raise ValueError("a resident scenario uses another candidate set")
        sim_batch_set_neighbours(self.b, n)  # resets the tuning to that set's default
        self.neighbours = n
        if self.tuning_source == "explicit":
            self.tuning_source = "library default"

    def tour_lengths(self, slot: int) -> np.ndarray:
        """The tour matrix of a tour-variant slot on the host."""
        s = self.stream if self.stream is not None else self.torch.cuda.current_stream(self.device)
        s.synchronize()
        return self.members[slot].tour.cpu().numpy()

    def close(self) -> None:
        if self.b:
            sim_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
