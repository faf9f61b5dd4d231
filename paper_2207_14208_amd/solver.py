"""Python front end of libbcmg: problems and batches on torch device memory.

torch supplies device buffers and the stream; every step of setup and of the
cycle runs in the HIP library (see _native).  Arrays are flat, (N+1)^d, x fastest.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N
from ._native import check, lib


def _dev_f64(a, device="cuda") -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)


def _ptr(t: torch.Tensor | None):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------- device memory
# In a torch process the library's device memory comes from torch's caching
# allocator (bcmg_set_allocator), so one pool owns HBM and torch's memory
# statistics include the solver's hierarchies.
_alloc_cbs = None
_exiting = False


def _torch_alloc(nbytes, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:
        return None  # the library reports BCMG_ERR_OOM


def _torch_free(ptr, nbytes, stream, ctx):
    try:
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


def use_torch_allocator(enable: bool = True) -> None:
    """Route the library's device allocations through torch's caching
    allocator (enable) or back to its private pool.  Handles keep the source
    they were created with."""
    global _alloc_cbs
    if enable:
        if _alloc_cbs is None:
            _alloc_cbs = (N.ALLOC_FN(_torch_alloc), N.FREE_FN(_torch_free))
        check(lib().bcmg_set_allocator(C.cast(_alloc_cbs[0], C.c_void_p), C.cast(_alloc_cbs[1], C.c_void_p), None))
    else:
        check(lib().bcmg_set_allocator(None, None, None))


def _mark_exit():
    # handles still alive at interpreter exit are not destroyed: their frees
    # would call back into a torch that is shutting down
    global _exiting
    _exiting = True


import atexit  # noqa: E402

atexit.register(_mark_exit)
_torch_allocator_on = False


def _ensure_torch_allocator():
    global _torch_allocator_on
    if not _torch_allocator_on:
        use_torch_allocator(True)
        _torch_allocator_on = True


@dataclass
class SolveStats:
    cycles: int
    status: int
    r0: float
    r_final: float
    rho_mean: float
    solve_ms: float

    @classmethod
    def from_c(cls, s: N.bcmg_solve_stats) -> "SolveStats":
        return cls(s.cycles, s.status, s.r0, s.r_final, s.rho_mean, s.solve_ms)


class Problem:
    """One level-set problem (bcmg_setup ... bcmg_destroy).

    Options are the fields of bcmg_options (include/bcmg.h), for example
    nu1, nu2, precision (N.FP64 / N.MIXED), dtau_mode, dtau_const, and
    bc = N.BC_NEUMANN with reaction = c for c u - Laplace u = f; the ghost
    data given to set_data is then the normal derivative at each Q.
    """

    def __init__(self, dim: int, N_: int, phi, options: N.bcmg_options | None = None, stream=None, **opt_kw):
        self.dim, self.N = dim, N_
        self.opts = options if options is not None else N.default_options(**opt_kw)
        self.stream = stream
        phi_d = _dev_f64(phi)
        if phi_d.numel() != (N_ + 1) ** dim:
            raise ValueError("phi has the wrong size")
        h = C.c_void_p()
        _ensure_torch_allocator()
        check(lib().bcmg_setup(dim, N_, _ptr(phi_d), C.byref(self.opts), _stream_handle(stream), C.byref(h)))
        self.h = h
        n = C.c_int32()
        check(lib().bcmg_num_levels(self.h, C.byref(n)))
        self.levels = n.value
        self.nodes = (N_ + 1) ** dim

    def close(self):
        if getattr(self, "h", None):
            if not _exiting:
                lib().bcmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- geometry
    def level_info(self, level: int = 0) -> dict:
        Nl = C.c_int32()
        ni, ng, nb, ns = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().bcmg_level_info(self.h, level, C.byref(Nl), C.byref(ni), C.byref(ng), C.byref(nb), C.byref(ns)))
        return dict(N=Nl.value, n_inside=ni.value, n_ghost=ng.value, n_band=nb.value, n_segments=ns.value)

    def level_nodes(self, level: int) -> int:
        return (self.level_info(level)["N"] + 1) ** self.dim

    def classes(self, level: int = 0) -> torch.Tensor:
        out = torch.empty(self.level_nodes(level), dtype=torch.uint8, device="cuda")
        check(lib().bcmg_classes(self.h, level, _ptr(out)))
        return out

    def ghost_info(self, level: int = 0) -> dict:
        ng = self.level_info(level)["n_ghost"]
        dev = "cuda"
        g = dict(idx=torch.empty(ng, dtype=torch.int32, device=dev), code=torch.empty(ng, dtype=torch.int32, device=dev),
                 eta=torch.empty(ng, dtype=torch.float64, device=dev), n=torch.empty(ng, 3, dtype=torch.float64, device=dev),
                 q=torch.empty(ng, 3, dtype=torch.float64, device=dev), tau=torch.empty(ng, 3, dtype=torch.float64, device=dev),
                 dtau=torch.empty(ng, dtype=torch.float64, device=dev), fb=torch.empty(ng, dtype=torch.int32, device=dev))
        if ng:
            check(lib().bcmg_ghost_info(self.h, level, *[_ptr(g[k]) for k in ("idx", "code", "eta", "n", "q", "tau", "dtau", "fb")]))
        return g

    def ghost_stats(self, level: int = 0) -> dict:
        """bcmg_ghost_stats: {"widths": {(a, b, c): rows, ...} (sorted widths,
        nonzero classes only), "root_fallback": n, "row_fallback": n}."""
        counts = (C.c_int64 * 27)()
        root, row = C.c_int64(), C.c_int64()
        check(lib().bcmg_ghost_stats(self.h, level, counts, C.byref(root), C.byref(row)))
        widths = {(3 - k // 9, 3 - (k // 3) % 3, 3 - k % 3): int(counts[k]) for k in range(27) if counts[k]}
        return {"widths": widths, "root_fallback": root.value, "row_fallback": row.value}

    # ---------------------------------------------------------------- data
    def set_data(self, f, gq):
        f_d = _dev_f64(f) if f is not None else None
        gq_d = _dev_f64(gq)
        check(lib().bcmg_set_data(self.h, _ptr(f_d), _ptr(gq_d) if gq_d.numel() else None))

    def fill_boundary(self, gbox, u: torch.Tensor):
        gb = _dev_f64(gbox) if gbox is not None else None
        check(lib().bcmg_fill_boundary(self.h, _ptr(gb), _ptr(u)))

    def initial_guess(self, gbox=None) -> torch.Tensor:
        u = torch.zeros(self.nodes, dtype=torch.float64, device="cuda")
        self.fill_boundary(gbox, u)
        return u

    # ---------------------------------------------------------------- solve
    def vcycle(self, u: torch.Tensor):
        check(lib().bcmg_vcycle(self.h, _ptr(u)))

    def residual_norm(self, u: torch.Tensor) -> float:
        v = C.c_double()
        check(lib().bcmg_residual_norm(self.h, _ptr(u), C.byref(v)))
        return v.value

    def solve(self, u: torch.Tensor, tol: float = 1e-10, raise_on_fail: bool = False):
        st = N.bcmg_solve_stats()
        hist = np.zeros(self.opts.max_cycles + 1)
        status = lib().bcmg_solve(self.h, _ptr(u), float(tol), C.byref(st),
                                  hist.ctypes.data_as(C.c_void_p))
        if raise_on_fail:
            check(status)
        elif status not in (N.OK, N.ERR_NOT_CONVERGED, N.ERR_DIVERGED):
            check(status)
        s = SolveStats.from_c(st)
        return s, hist[: s.cycles + 1].copy()

    # ----------------------------------------------------------- single steps
    def level_smooth(self, level, u, rhs, steps=1):
        check(lib().bcmg_level_smooth(self.h, level, _ptr(u), _ptr(rhs), steps))

    def level_residual(self, level, u, rhs, r, with_norm=False):
        v = C.c_double()
        check(lib().bcmg_level_residual(self.h, level, _ptr(u), _ptr(rhs), _ptr(r), C.byref(v) if with_norm else None))
        return v.value if with_norm else None

    def level_extend(self, level, v):
        check(lib().bcmg_level_extend(self.h, level, _ptr(v)))

    def level_restrict(self, level, rfine, rcoarse):
        check(lib().bcmg_level_restrict(self.h, level, _ptr(rfine), _ptr(rcoarse)))

    def level_prolong(self, level, ecoarse, ufine):
        check(lib().bcmg_level_prolong(self.h, level, _ptr(ecoarse), _ptr(ufine)))

    def coarse_solve(self, u, rhs):
        check(lib().bcmg_coarse_solve(self.h, _ptr(u), _ptr(rhs)))

    def timing_sweeps(self, u: torch.Tensor, reps: int) -> float:
        """ms for `reps` back-to-back red + black finest-level sweeps on a copy of u."""
        v = C.c_double()
        check(lib().bcmg_timing_sweeps(self.h, _ptr(u), int(reps), C.byref(v)))
        return v.value

    def device_bytes(self) -> int:
        b = C.c_int64()
        check(lib().bcmg_problem_bytes(self.h, C.byref(b)))
        return b.value


def estimate_bytes(dim: int, N_: int, precision: int = N.FP64) -> int:
    b = C.c_int64()
    check(lib().bcmg_estimate_bytes(dim, N_, precision, C.byref(b)))
    return b.value


class Batch:
    """Many problems advanced together by whole V-cycles (bcmg_batch_*)."""

    def __init__(self, capacity: int, stream=None):
        h = C.c_void_p()
        _ensure_torch_allocator()
        check(lib().bcmg_batch_create(capacity, _stream_handle(stream), C.byref(h)))
        self.h = h
        self.capacity = capacity
        self.slots: dict[int, tuple[Problem, torch.Tensor]] = {}

    def add(self, prob: Problem, u: torch.Tensor, tol: float) -> int:
        s = C.c_int32()
        check(lib().bcmg_batch_add(self.h, prob.h, _ptr(u), float(tol), C.byref(s)))
        self.slots[s.value] = (prob, u)
        return s.value

    def restart(self):
        check(lib().bcmg_batch_restart(self.h))

    def set_param(self, param: int, value: int):
        check(lib().bcmg_batch_set_param(self.h, param, int(value)))

    def remove(self, slot: int):
        check(lib().bcmg_batch_remove(self.h, slot))
        self.slots.pop(slot, None)

    def step(self, cycles: int = 1) -> np.ndarray:
        act = np.zeros(self.capacity, dtype=np.int32)
        check(lib().bcmg_batch_step(self.h, cycles, act.ctypes.data_as(C.c_void_p)))
        return act

    def run(self, cycles_per_step: int = 1, max_steps: int = 1000):
        check(lib().bcmg_batch_run(self.h, cycles_per_step, max_steps))

    def stats(self, slot: int, max_cycles: int = 1000):
        st = N.bcmg_solve_stats()
        hist = np.zeros(max_cycles + 1)
        check(lib().bcmg_batch_stats(self.h, slot, C.byref(st), hist.ctypes.data_as(C.c_void_p)))
        s = SolveStats.from_c(st)
        return s, hist[: s.cycles + 1].copy()

    def close(self):
        if getattr(self, "h", None):
            if not _exiting:
                lib().bcmg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def timing_enable(on: bool):
    check(lib().bcmg_timing_enable(1 if on else 0))


def timing_read():
    n, ms, nodes = C.c_int64(), C.c_double(), C.c_int64()
    check(lib().bcmg_timing_read(C.byref(n), C.byref(ms), C.byref(nodes)))
    return n.value, ms.value, nodes.value
