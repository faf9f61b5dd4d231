"""Convergence-factor engine: the estimator and the sweep specification
(host logic, no GPU)."""
import math

import numpy as np
import pytest

from paper_2207_14208_amd import _native as N
from paper_2207_14208_amd import experiments as X


def test_rho_of_a_geometric_history_is_its_ratio():
    h = 3.0 * 0.3 ** np.arange(17)
    assert X.rho_from_history(h) == pytest.approx(0.3, rel=1e-12)


def test_rho_averages_cycles_11_to_15_only():
    ratios = np.full(16, 0.9)
    ratios[10:15] = [0.1, 0.2, 0.3, 0.4, 0.5]  # rho^(11) .. rho^(15)
    h = np.concatenate([[1.0], np.cumprod(ratios)])
    assert X.rho_from_history(h) == pytest.approx(0.3, rel=1e-12)


@pytest.mark.parametrize("h", [
    np.ones(10),                                    # stopped before cycle 15 (diverged or converged)
    np.concatenate([np.ones(12), [np.nan], np.ones(4)]),
    2.0 ** np.arange(17),                           # growing: cut at 1
])
def test_rho_is_cut_at_one(h):
    assert X.rho_from_history(h) == 1.0


def test_spec_dtau_parsing_and_domains():
    assert X.Spec("circle", 64, "const:1.75").dtau_mode() == (N.DTAU_CONST, 1.75)
    assert X.Spec("circle", 64, "opt_poly").dtau_mode() == (N.DTAU_OPT_POLY, 1.0)
    assert X.Spec("ellipsoid", 32).dim == 3 and X.Spec("rectangle", 128).dim == 2


def test_rectangle_ghosts_sit_at_theta_h():
    """The rectangle x <= x_V = 1 - theta h: the only non-eliminated
    boundary is x = x_V, so the last column holds the ghosts, theta h away."""
    for theta in (0.1, 0.5, 0.9):
        n = 64
        phi = X.DOMAINS["rectangle"][1](n, theta)
        x = np.array([1.0 - 2.0 / n, 1.0])
        vals = phi(x, np.zeros(2))
        assert vals[0] < 0 < vals[1]
        assert vals[1] == pytest.approx(theta * 2.0 / n, rel=1e-12)


def test_initial_guess_only_on_unknowns():
    cls = np.array([N.OUTSIDE, N.INSIDE, N.GHOST, N.BOXDIR] * 50, dtype=np.uint8)
    u = X.initial_guess(cls, 3)
    unk = (cls == N.INSIDE) | (cls == N.GHOST)
    assert np.all(u[~unk] == 0.0) and np.all(np.abs(u[unk]) < 1.0) and np.all(u[unk] != 0.0)


def test_boundary_dft_of_a_pure_mode():
    """A cosine on one grid frequency alpha_m has amplitude 2|R_m| = 1 there
    and none elsewhere (the M frequencies are orthogonal over j = 1..M)."""
    m = 127
    alpha = -np.pi + np.arange(1, m + 1) * 2 * np.pi / m
    for k in (70, 110):  # a low and a high positive frequency
        a0 = alpha[k - 1]
        a, amp, ratio = X.boundary_dft(np.cos(a0 * np.arange(1, m + 1)))
        i = int(np.argmin(np.abs(a - a0)))
        assert amp[i] == pytest.approx(1.0, abs=1e-12)
        assert np.max(np.delete(amp, i)) < 1e-12
        assert (ratio > 1.0) == (a0 > np.pi / 2)
