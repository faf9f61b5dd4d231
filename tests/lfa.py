"""Local Fourier analysis of the two-grid method on the full box (test helper).

Written from the standard two-grid LFA (the analysis the paper cites for its
optimal factor, Sec. 3.2): the error of a low frequency theta and its 2^d
aliases theta + pi*alpha (alpha in {0,1}^d) span an invariant space of the
two-grid operator M = S^nu2 (I - P Lc^-1 R Lh) S^nu1 for the 2d+1-point
Laplacian, full weighting R and multilinear interpolation P.  The two-grid
factor is the largest spectral radius of M(theta) over the low frequencies.

Smoothers:
  'lex' lexicographic Gauss-Seidel: diagonal, symbol sum_k e^{i th_k} / (2d - sum_k e^{-i th_k})
  'jac' weighted Jacobi, omega = 2d/(2d+1): diagonal, symbol 1 - omega (1 - sum_k cos th_k / d)
  'rb'  red-black Gauss-Seidel: a red partial step is chi_R J + chi_B with J
        the Jacobi symbol and chi_R = (I + Pi)/2, chi_B = (I - Pi)/2, where Pi
        swaps each harmonic with its (pi,...,pi) shift (multiplication by
        (-1)^{i+j+k}); then the black step with the colours exchanged.

Shares nothing with the oracle; only numpy.
"""
from __future__ import annotations

import itertools

import numpy as np


def _harmonics(d):
    return [np.array(a) for a in itertools.product((0, 1), repeat=d)]


def two_grid_matrix(theta, d, smoother="rb", nu1=2, nu2=1):
    theta = np.asarray(theta, dtype=float)
    alphas = _harmonics(d)
    H = len(alphas)
    th = [theta + np.pi * a for a in alphas]
    # fine operator symbol (h = 1), coarse operator at 2*theta with H = 2
    Lh = np.array([sum(2 - 2 * np.cos(t[k]) for k in range(d)) for t in th], dtype=complex)
    Lc = sum(2 - 2 * np.cos(2 * theta[k]) for k in range(d)) / 4.0
    Rh = np.array([np.prod([(1 + np.cos(t[k])) / 2 for k in range(d)]) for t in th], dtype=complex)
    Ph = Rh.copy()
    K = np.eye(H, dtype=complex) - np.outer(Ph, Rh * Lh) / Lc
    if smoother == "lex":
        S = np.diag([sum(np.exp(1j * t[k]) for k in range(d)) / (2 * d - sum(np.exp(-1j * t[k]) for k in range(d)))
                     for t in th])
    elif smoother == "jac":
        om = 2.0 * d / (2.0 * d + 1.0)
        S = np.diag([1.0 - om * (1.0 - sum(np.cos(t[k]) for k in range(d)) / d) for t in th]).astype(complex)
    elif smoother == "rb":
        J = np.diag([sum(np.cos(t[k]) for k in range(d)) / d for t in th]).astype(complex)
        Pi = np.zeros((H, H))
        ones = np.ones(d, dtype=int)
        for i, a in enumerate(alphas):
            j = next(jj for jj, b in enumerate(alphas) if np.array_equal(b, (a + ones) % 2))
            Pi[j, i] = 1.0
        I = np.eye(H)
        chiR, chiB = (I + Pi) / 2, (I - Pi) / 2
        SR = chiR @ J + chiB
        SB = chiB @ J + chiR
        S = SB @ SR
    else:
        raise ValueError(smoother)
    return np.linalg.matrix_power(S, nu2) @ K @ np.linalg.matrix_power(S, nu1)


def two_grid_factor(d, smoother="rb", nu1=2, nu2=1, n=24):
    """sup over a grid of low frequencies (-pi/2, pi/2]^d, theta != 0."""
    grid = -np.pi / 2 + np.pi * (np.arange(1, n + 1)) / n
    best = 0.0
    for theta in itertools.product(grid, repeat=d):
        if np.allclose(theta, 0):
            continue
        M = two_grid_matrix(theta, d, smoother, nu1, nu2)
        best = max(best, max(abs(np.linalg.eigvals(M))))
    return best


def smoothing_factor(d, smoother="rb", nu=1, n=48):
    """Idealised-coarse-grid smoothing factor: spectral radius of Q S^nu with Q
    removing the low-frequency harmonic."""
    grid = -np.pi / 2 + np.pi * (np.arange(1, n + 1)) / n
    best = 0.0
    alphas = _harmonics(d)
    Q = np.diag([0.0 if not a.any() else 1.0 for a in alphas])
    for theta in itertools.product(grid, repeat=d):
        if np.allclose(theta, 0):
            continue
        M = two_grid_matrix(theta, d, smoother, nu, 0)
        # two_grid_matrix includes K; rebuild S alone via nu1=nu, K replaced by Q
        th = np.asarray(theta)
        del M
        Mq = _smoother_only(th, d, smoother, nu)
        best = max(best, max(abs(np.linalg.eigvals(Q @ Mq))))
    return best ** (1.0 / nu)


def _smoother_only(theta, d, smoother, nu):
    alphas = _harmonics(d)
    H = len(alphas)
    th = [theta + np.pi * a for a in alphas]
    if smoother == "lex":
        S = np.diag([sum(np.exp(1j * t[k]) for k in range(d)) / (2 * d - sum(np.exp(-1j * t[k]) for k in range(d)))
                     for t in th])
    else:
        J = np.diag([sum(np.cos(t[k]) for k in range(d)) / d for t in th]).astype(complex)
        Pi = np.zeros((H, H))
        ones = np.ones(d, dtype=int)
        for i, a in enumerate(alphas):
            j = next(jj for jj, b in enumerate(alphas) if np.array_equal(b, (a + ones) % 2))
            Pi[j, i] = 1.0
        I = np.eye(H)
        S = ((I - Pi) / 2 @ J + (I + Pi) / 2) @ ((I + Pi) / 2 @ J + (I - Pi) / 2)
    return np.linalg.matrix_power(S, nu)
