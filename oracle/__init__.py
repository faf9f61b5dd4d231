"""Oracle: a plain FP64 CPU implementation of the ghost-point multigrid.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never imports, links or calls it.

The arithmetic lives in ``bcmg_oracle.c`` (plain C, lexicographic loops over
the whole node box, no blocking or fusion); this module is a ctypes wrapper
that marshals numpy arrays.  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bcmg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OUTSIDE, INSIDE, GHOST, BOXDIR = 0, 1, 2, 3
DTAU_OPT_EXP, DTAU_OPT_POLY, DTAU_CONST = 0, 1, 2
RESTRICT_RENORM_FW, RESTRICT_PLAIN_MEAN = 0, 1
SMOOTH_RB, SMOOTH_LEX, SMOOTH_JAC = 0, 1, 2
CYCLE_V, CYCLE_TGCS, CYCLE_W = 0, 1, 2
BC_DIRICHLET, BC_NEUMANN = 0, 1


class _Opts(C.Structure):
    _fields_ = [
        ("nu1", C.c_int), ("nu2", C.c_int), ("coarsest_N", C.c_int), ("max_cycles", C.c_int),
        ("dtau_mode", C.c_int), ("dtau_const", C.c_double), ("ext_iters", C.c_int),
        ("restrict_mode", C.c_int), ("smoother", C.c_int), ("cycle", C.c_int),
        ("bc", C.c_int), ("reaction", C.c_double), ("ghost_dominance", C.c_int),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle into ``liboracle.so`` (gcc, -O2, FP64, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp, i, d, l = C.c_void_p, C.c_int, C.c_double, C.c_long
        L.or_setup.restype = vp
        L.or_setup.argtypes = [i, i, vp, C.POINTER(_Opts)]
        L.or_destroy.argtypes = [vp]
        L.or_default_options.argtypes = [C.POINTER(_Opts)]
        L.or_dtau.restype = d
        L.or_dtau.argtypes = [i, d, i, d]
        L.or_dtau_neumann.restype = d
        L.or_dtau_neumann.argtypes = [i, d, i, d]
        L.or_get_ghost_nd.argtypes = [vp, i, vp]
        L.or_classify.argtypes = [i, i, vp, vp]
        for name, args in [
            ("or_num_levels", [vp]), ("or_level_N", [vp, i]), ("or_coarse_singular", [vp]),
        ]:
            getattr(L, name).restype = i
            getattr(L, name).argtypes = args
        L.or_level_nodes.restype = l
        L.or_level_nodes.argtypes = [vp, i]
        L.or_coarse_fallbacks.restype = l
        L.or_coarse_fallbacks.argtypes = [vp]
        L.or_coarse_unknowns.restype = l
        L.or_coarse_unknowns.argtypes = [vp]
        L.or_counts.argtypes = [vp, i, C.POINTER(l), C.POINTER(l)]
        L.or_get_phi.argtypes = [vp, i, vp]
        L.or_get_classes.argtypes = [vp, i, vp]
        L.or_get_ghosts.argtypes = [vp, i] + [vp] * 9
        L.or_set_rhs.argtypes = [vp, vp, vp]
        L.or_get_rhs.argtypes = [vp, i, vp]
        L.or_set_level_rhs.argtypes = [vp, i, vp]
        L.or_apply_A.argtypes = [vp, i, vp, vp]
        L.or_residual.argtypes = [vp, i, vp, vp, vp]
        L.or_norm.restype = d
        L.or_norm.argtypes = [vp, i, vp]
        L.or_smooth_n.argtypes = [vp, i, vp, vp, i]
        L.or_extend.argtypes = [vp, i, vp]
        L.or_restrict.argtypes = [vp, i, vp, vp]
        L.or_prolong.argtypes = [vp, i, vp, vp]
        L.or_coarse_solve.argtypes = [vp, vp, vp]
        L.or_vcycle.argtypes = [vp, vp]
        L.or_vcycle_at.argtypes = [vp, i, vp, vp]
        L.or_solve.restype = i
        L.or_solve.argtypes = [vp, vp, d, i, vp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


@dataclass
class Options:
    nu1: int = 2
    nu2: int = 1
    coarsest_N: int = 4
    max_cycles: int = 100
    dtau_mode: int = DTAU_OPT_EXP
    dtau_const: float = 1.0
    ext_iters: int = 4
    restrict_mode: int = RESTRICT_RENORM_FW
    smoother: int = SMOOTH_RB
    cycle: int = CYCLE_V
    bc: int = BC_DIRICHLET
    reaction: float = 0.0
    ghost_dominance: int = 1   # 0: stencil widths by validity only (shows why the dominance test is needed)

    def _c(self) -> _Opts:
        return _Opts(self.nu1, self.nu2, self.coarsest_N, self.max_cycles, self.dtau_mode,
                     float(self.dtau_const), self.ext_iters, self.restrict_mode, self.smoother, self.cycle,
                     self.bc, float(self.reaction), int(self.ghost_dominance))


def dtau(d: int, theta: float, mode: int = DTAU_OPT_EXP, const: float = 1.0) -> float:
    return lib().or_dtau(d, float(theta), mode, float(const))


def dtau_neumann(d: int, theta: float, mode: int = DTAU_OPT_EXP, const: float = 1.0) -> float:
    """Delta tau / h of a Neumann ghost row."""
    return lib().or_dtau_neumann(d, float(theta), mode, float(const))


def classify(d: int, N: int, phi: np.ndarray) -> np.ndarray:
    phi = np.ascontiguousarray(phi, dtype=np.float64).ravel()
    cls = np.zeros(phi.size, dtype=np.uint8)
    lib().or_classify(d, N, _p(phi), _p(cls))
    return cls


class Problem:
    """Oracle hierarchy for phi sampled at the finest nodes (x fastest)."""

    def __init__(self, d: int, N: int, phi: np.ndarray, opts: Options | None = None):
        self.d, self.N = d, N
        self.opts = opts or Options()
        phi = np.ascontiguousarray(phi, dtype=np.float64).ravel()
        if phi.size != (N + 1) ** d:
            raise ValueError("phi has the wrong size")
        self._o = self.opts._c()
        self.h = lib().or_setup(d, N, _p(phi), C.byref(self._o))
        if not self.h:
            raise ValueError("oracle setup rejected the grid")
        self.L = lib().or_num_levels(self.h)

    def __del__(self):
        try:
            if getattr(self, "h", None) and _lib is not None:
                _lib.or_destroy(self.h)
        except Exception:
            pass
        self.h = None

    # --- geometry ---------------------------------------------------------
    def nodes(self, l: int = 0) -> int:
        return lib().or_level_nodes(self.h, l)

    def level_N(self, l: int) -> int:
        return lib().or_level_N(self.h, l)

    def counts(self, l: int = 0):
        ni, ng = C.c_long(), C.c_long()
        lib().or_counts(self.h, l, C.byref(ni), C.byref(ng))
        return ni.value, ng.value

    def phi(self, l: int = 0) -> np.ndarray:
        out = np.empty(self.nodes(l))
        lib().or_get_phi(self.h, l, _p(out))
        return out

    def classes(self, l: int = 0) -> np.ndarray:
        out = np.empty(self.nodes(l), dtype=np.uint8)
        lib().or_get_classes(self.h, l, _p(out))
        return out

    def ghosts(self, l: int = 0) -> dict:
        _, ng = self.counts(l)
        g = dict(idx=np.empty(ng, np.int64), w=np.empty((ng, 3), np.int32), s=np.empty((ng, 3), np.int32),
                 fb=np.empty(ng, np.int32), eta=np.empty(ng), n=np.empty((ng, 3)), q=np.empty((ng, 3)),
                 tau=np.empty((ng, 3)), dtau=np.empty(ng))
        g["nd"] = np.zeros((ng, 3))
        if ng:
            lib().or_get_ghosts(self.h, l, *[_p(g[k]) for k in ("idx", "w", "s", "fb", "eta", "n", "q", "tau", "dtau")])
            lib().or_get_ghost_nd(self.h, l, _p(g["nd"]))
        return g

    def coarse_singular(self) -> bool:
        return bool(lib().or_coarse_singular(self.h))

    def coarse_unknowns(self) -> int:
        return lib().or_coarse_unknowns(self.h)

    # --- data -------------------------------------------------------------
    def set_rhs(self, f: np.ndarray, gq: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64).ravel()
        gq = np.ascontiguousarray(gq, dtype=np.float64).ravel()
        assert f.size == self.nodes(0) and gq.size == self.counts(0)[1]
        lib().or_set_rhs(self.h, _p(f), _p(gq) if gq.size else None)

    def rhs(self, l: int = 0) -> np.ndarray:
        out = np.empty(self.nodes(l))
        lib().or_get_rhs(self.h, l, _p(out))
        return out

    def set_level_rhs(self, l: int, rhs: np.ndarray):
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        assert rhs.size == self.nodes(l)
        lib().or_set_level_rhs(self.h, l, _p(rhs))

    # --- operators (arrays are modified in place where noted) --------------
    def apply_A(self, l: int, u: np.ndarray) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.empty(self.nodes(l))
        lib().or_apply_A(self.h, l, _p(u), _p(out))
        return out

    def residual(self, l: int, u: np.ndarray, rhs: np.ndarray | None = None) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64)
        rhs = self.rhs(l) if rhs is None else np.ascontiguousarray(rhs, dtype=np.float64)
        out = np.empty(self.nodes(l))
        lib().or_residual(self.h, l, _p(u), _p(rhs), _p(out))
        return out

    def norm(self, l: int, r: np.ndarray) -> float:
        r = np.ascontiguousarray(r, dtype=np.float64)
        return lib().or_norm(self.h, l, _p(r))

    def smooth(self, l: int, u: np.ndarray, rhs: np.ndarray | None = None, steps: int = 1):
        """In place on u."""
        assert u.dtype == np.float64 and u.flags.c_contiguous
        rhs = self.rhs(l) if rhs is None else np.ascontiguousarray(rhs, dtype=np.float64)
        lib().or_smooth_n(self.h, l, _p(u), _p(rhs), steps)

    def extend(self, l: int, v: np.ndarray):
        """In place on v (OUTSIDE entries)."""
        assert v.dtype == np.float64 and v.flags.c_contiguous
        lib().or_extend(self.h, l, _p(v))

    def restrict(self, l: int, r_ext: np.ndarray) -> np.ndarray:
        r_ext = np.ascontiguousarray(r_ext, dtype=np.float64)
        out = np.empty(self.nodes(l + 1))
        lib().or_restrict(self.h, l, _p(r_ext), _p(out))
        return out

    def prolong(self, l: int, ec: np.ndarray, u: np.ndarray):
        """u += P e on fine INSIDE and GHOST nodes; ec is modified (extension)."""
        assert ec.dtype == np.float64 and ec.flags.c_contiguous
        assert u.dtype == np.float64 and u.flags.c_contiguous
        lib().or_prolong(self.h, l, _p(ec), _p(u))

    def coarse_solve(self, u: np.ndarray, rhs: np.ndarray):
        assert u.dtype == np.float64 and u.flags.c_contiguous
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        lib().or_coarse_solve(self.h, _p(u), _p(rhs))

    def vcycle(self, u: np.ndarray):
        assert u.dtype == np.float64 and u.flags.c_contiguous
        lib().or_vcycle(self.h, _p(u))

    def vcycle_at(self, l: int, u: np.ndarray, rhs: np.ndarray):
        assert u.dtype == np.float64 and u.flags.c_contiguous
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        lib().or_vcycle_at(self.h, l, _p(u), _p(rhs))

    def solve(self, u: np.ndarray, tol: float = 1e-10, max_cycles: int | None = None):
        """In place on u.  Returns (cycles or -1, residual history)."""
        assert u.dtype == np.float64 and u.flags.c_contiguous
        mc = self.opts.max_cycles if max_cycles is None else max_cycles
        hist = np.full(mc + 1, -1.0)  # norms are >= 0: -1 marks entries never written
        it = lib().or_solve(self.h, _p(u), float(tol), mc, _p(hist))
        n = (it + 1) if it >= 0 else int(np.argmax(hist == -1.0)) if np.any(hist == -1.0) else mc + 1
        return it, hist[: n]
