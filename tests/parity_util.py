"""Shared checks of the GPU-against-oracle solve parity tests.

Two FP64 evaluations of the same residual differ by rounding only.  The
bounds below follow from that and from the 1e-8 relative agreement of the
per-cycle norms; they decide when a stopping test may flip by one cycle.
"""
import numpy as np

import oracle


def unknowns(cls):
    return (cls == oracle.INSIDE) | (cls == oracle.GHOST)


def residual_floor(d, N, cls, u, rhs, reaction=0.0):
    """Rounding floor of the residual's 2-norm.  A computed row differs from
    the exact one by at most (2d + 2) eps times the sum of its terms'
    magnitudes, which is below ((4d / h^2) + c) max|u| + max|rhs| on an
    INSIDE row (ghost rows are smaller); the norm over n rows then moves by
    at most sqrt(n) times that, and two independent evaluations by twice it."""
    eps = np.finfo(np.float64).eps
    m = unknowns(cls)
    n = int(m.sum())
    h = 2.0 / N
    scale = (4 * d / h ** 2 + reaction) * np.abs(u).max() + np.abs(rhs[m]).max()
    return 2 * (2 * d + 2) * eps * np.sqrt(n) * scale


def histories_agree(hg, ho, floor):
    """Per-cycle residual norms within 1e-8 relative plus the rounding floor."""
    hg, ho = np.asarray(hg), np.asarray(ho)
    n = min(len(hg), len(ho))
    return bool(np.all(np.abs(hg[:n] - ho[:n]) <= 1e-8 * ho[:n] + floor))


def cycles_agree(cg, co, ho, tol, floor):
    """The same cycle count, unless the norm at the earlier stop lies within
    the two sides' disagreement (1e-8 relative plus the floor) of the
    threshold tol * r0, where rounding alone can flip the stopping test."""
    if cg == co:
        return True
    k = min(cg, co)
    return abs(cg - co) == 1 and abs(ho[k] - tol * ho[0]) <= 1e-8 * ho[k] + floor
