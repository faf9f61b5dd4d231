"""Pins for the ghost rows' stencil admissibility, the fallback distance and
the theta~ that sets Delta tau (oracle side, no GPU).

 * The dominance test on stencil blocks: with it, the Jacobi relaxation of
   the ghost rows alone (interior values fixed) has spectral radius below 1
   on domains whose ghost rows couple to each other (the flower's pole
   crease, unions of spheres); without it, two of those unions give a
   ghost block whose relaxation expands (spectral radius above 1).  The
   ghost block is read from the operator itself (A applied to unit vectors).
 * The first-order distance used when the interpolant has no root within
   one grid step of G: a hand-made level set with the expected eta written
   out from its node values.
 * theta~ is the distance, along the normal, from G to the point where its
   row interpolates.  That point is found by applying the row to the
   coordinate functions (the Lagrange weights reproduce linear functions),
   not from the stored widths or local coordinates.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2207_14208_amd import workloads as W


def _spheres(seed, count=20):
    cen = np.random.default_rng(seed).uniform(-0.7, 0.7, (count, 3))
    rad = np.random.default_rng(seed + 100).uniform(0.05, 0.2, count)
    return W.phi_spheres(cen, rad)


def _ghost_block(P, l=0):
    """A restricted to ghost rows and ghost columns, and the ghosts' dtau."""
    g = P.ghosts(l)
    idx = g["idx"]
    A = np.zeros((idx.size, idx.size))
    for j, p in enumerate(idx):
        e = np.zeros(P.nodes(l))
        e[p] = 1.0
        A[:, j] = P.apply_A(l, e)[idx]
    return A, g["dtau"]


def _jacobi_radius(P):
    A, dt = _ghost_block(P)
    E = np.eye(dt.size) - dt[:, None] * A
    return float(np.abs(np.linalg.eigvals(E)).max())


@pytest.mark.parametrize("name,N,phi_fn", [
    ("flower", 32, W.phi_flower3d()),
    ("spheres1", 32, _spheres(1)),
    ("spheres5", 32, _spheres(5)),
])
def test_ghost_relaxation_contracts_with_dominance(name, N, phi_fn):
    phi = W.sample(3, N, phi_fn)
    assert _jacobi_radius(oracle.Problem(3, N, phi)) < 1.0


@pytest.mark.parametrize("seed", [1, 5])
def test_ghost_relaxation_expands_without_dominance(seed):
    phi = W.sample(3, 32, _spheres(seed))
    assert _jacobi_radius(oracle.Problem(3, 32, phi, oracle.Options(ghost_dominance=0))) > 1.05


def _fallback_phi(phi_g):
    """N = 8, 2D: every node outside except (3,4) (phi = -0.1, just inside).
    The ghost G = (4,4) has phi_G = phi_g.  Its discrete gradient is
    ((1 - (-0.1)) / 2h, (10 - 1) / 2h): the normal points along +y, away
    from the only inside node, and the interpolant stays positive one grid
    step from G along the normal."""
    N = 8
    phi = np.ones((N + 1, N + 1))  # [j][i]
    phi[4, 3] = -0.1
    phi[4, 4] = phi_g
    phi[5, 4] = 10.0
    return N, phi.ravel()


@pytest.mark.parametrize("phi_g,eta_expected", [
    (0.5, 0.5 * 2.0 / math.hypot(1.1, 9.0)),   # phi_G / (h |grad_h phi|), |grad_h phi| = hypot(1.1, 9) / 2h
    (10.0, 1.0),                                 # the same estimate exceeds one step: eta = 1
])
def test_root_fallback_is_first_order_distance(phi_g, eta_expected):
    N, phi = _fallback_phi(phi_g)
    P = oracle.Problem(2, N, phi)
    g = P.ghosts(0)
    k = int(np.nonzero(g["idx"] == 4 + 9 * 4)[0][0])
    assert g["fb"][k] == 1
    assert abs(g["eta"][k] - eta_expected) <= 1e-15


@pytest.mark.parametrize("name,d,N,phi_fn", [
    ("flower", 3, 32, W.phi_flower3d()),
    ("spheres1", 3, 32, _spheres(1)),
    ("flower2d", 2, 64, W.phi_flower2d()),
])
def test_theta_is_normal_distance_to_row_point(name, d, N, phi_fn):
    P = oracle.Problem(d, N, W.sample(d, N, phi_fn))
    g = P.ghosts(0)
    h = 2.0 / N
    idx = g["idx"]
    X = [W.sample(d, N, (lambda k: (lambda *xs: xs[k] + 0.0 * xs[0]))(k)) for k in range(d)]
    xg = np.stack([Xk[idx] for Xk in X], axis=1)
    # the row's interpolation point: the row applied to each coordinate
    qhat = np.stack([P.apply_A(0, Xk)[idx] for Xk in X], axis=1)
    n = g["n"][:, :d]
    theta = np.einsum("ij,ij->i", xg - qhat, n) / h
    A, dt = _ghost_block(P)
    c0 = np.diag(A)
    expect = np.array([min(oracle.dtau(d, t), 1.0 / c) for t, c in zip(theta, c0)])
    assert np.allclose(dt, expect, rtol=1e-11, atol=0)
    full = np.all(g["w"][:, :d] >= 2, axis=1)
    short = ~full
    # a full-width row interpolates at Q itself: theta~ = eta
    assert np.allclose(qhat[full], g["q"][full, :d], rtol=0, atol=1e-13)
    assert np.allclose(theta[full], g["eta"][full], rtol=0, atol=1e-12)
    if name != "flower2d":
        # shortened rows exist here, and for them theta~ < eta
        assert short.sum() > 0
        assert np.all(theta[short] <= g["eta"][short] + 1e-12)
        assert np.any(theta[short] < g["eta"][short] - 0.05)
