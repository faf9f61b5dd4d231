"""Pins for the fictitious time step Delta tau_OPT (oracle side, no GPU).

The oracle evaluates the closed forms of Prop. opt / Prop. opt3D / the
d-dimensional remark (polynomial form) and of Remark exptheta2D (exponential
form).  These tests pin them to (i) closed forms written with e^{-acosh x} =
x - sqrt(x^2-1), and (ii) a brute-force minimax over the high tangential
frequencies, which is the definition eq. (def_dtau_opt) / (def_dtau_opt3D)
itself, computed numerically with no use of the oracle.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import oracle

SQ2, SQ3, SQ6 = math.sqrt(2), math.sqrt(3), math.sqrt(6)


def coeff(t):
    # eq. (coeff), written independently here from (BC1D) with s = 3
    return t * (t - 1) / 2, t * (2 - t), (1 - t) * (2 - t) / 2  # c_{-2}, c_{-1}, c_0


def high_p_values(d, n=161):
    """p over the high-frequency set: 2D alpha in [pi/2, pi]; 3D (a1,a2) in [0,pi]^2 minus [0,pi/2)^2."""
    if d == 2:
        a = np.linspace(np.pi / 2, np.pi, n)
        return np.arccosh(2 - np.cos(a))
    a = np.linspace(0, np.pi, n)
    A1, A2 = np.meshgrid(a, a, indexing="ij")
    high = (A1 >= np.pi / 2) | (A2 >= np.pi / 2)
    return np.arccosh(3 - np.cos(A1[high]) - np.cos(A2[high]))


def brute_dtau(d, theta, form):
    p = high_p_values(d)
    if form == "poly":
        cm2, cm1, c0 = coeff(theta)
        G0 = cm2 * np.exp(-2 * p) + cm1 * np.exp(-p) + c0
    else:
        G0 = np.exp(-p * theta)
    res = minimize_scalar(lambda dt: np.max(np.abs(1 - dt * G0)), bounds=(1e-3, 20), method="bounded",
                          options={"xatol": 1e-11})
    return res.x


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("form,mode", [("poly", oracle.DTAU_OPT_POLY), ("exp", oracle.DTAU_OPT_EXP)])
@pytest.mark.parametrize("theta", [0.0, 0.2, 0.5, 0.8, 0.95])
def test_dtau_matches_bruteforce_minimax(d, form, mode, theta):
    got = oracle.dtau(d, theta, mode)
    want = brute_dtau(d, theta, form)
    assert abs(got - want) <= 1e-6 * want


def test_dtau_closed_forms():
    # theta = 0: Gauss-Seidel on the ghost row, dtau = 1/c_0 = 1 (Sec. 2.1)
    for d in (1, 2, 3):
        for mode in (oracle.DTAU_OPT_POLY, oracle.DTAU_OPT_EXP):
            assert oracle.dtau(d, 0.0, mode) == pytest.approx(1.0, abs=1e-15)
    # theta = 1: G0 = e^{-p}, e^{-acosh x} = x - sqrt(x^2 - 1)
    want2 = 2 / ((2 - SQ3) + (3 - 2 * SQ2))
    want3 = 2 / ((2 - SQ3) + (5 - 2 * SQ6))
    for mode in (oracle.DTAU_OPT_POLY, oracle.DTAU_OPT_EXP):
        assert oracle.dtau(2, 1.0, mode) == pytest.approx(want2, rel=1e-14)
        assert oracle.dtau(3, 1.0, mode) == pytest.approx(want3, rel=1e-14)
    assert want2 == pytest.approx(4.5503972316, abs=1e-9)
    assert want3 == pytest.approx(5.4204991976, abs=1e-9)
    # exp form at theta = 1/2: 2 / ((2-sqrt3)^{1/2} + (2d-1 - sqrt((2d-1)^2-1))^{1/2})
    assert oracle.dtau(2, 0.5, oracle.DTAU_OPT_EXP) == pytest.approx(2 / (math.sqrt(2 - SQ3) + math.sqrt(3 - 2 * SQ2)), rel=1e-14)
    assert oracle.dtau(3, 0.5, oracle.DTAU_OPT_EXP) == pytest.approx(2 / (math.sqrt(2 - SQ3) + math.sqrt(5 - 2 * SQ6)), rel=1e-14)
    # 1D: no tangential direction, p = acosh(1) = 0 (Sec. 2.2: no special dtau needed)
    assert oracle.dtau(1, 0.7, oracle.DTAU_OPT_EXP) == 1.0


def test_dtau_poly_2d_scan_values():
    # brute-force scan values 1.2578 / 1.8744 / 3.0588 at theta = 0.2 / 0.5 / 0.8
    for th, want in [(0.2, 1.25776), (0.5, 1.87444), (0.8, 3.05884)]:
        assert oracle.dtau(2, th, oracle.DTAU_OPT_POLY) == pytest.approx(want, abs=2e-5)


def test_dtau_clamp_and_const():
    for d in (2, 3):
        assert oracle.dtau(d, 1.7, oracle.DTAU_OPT_EXP) == oracle.dtau(d, 1.0, oracle.DTAU_OPT_EXP)
    assert oracle.dtau(3, 0.3, oracle.DTAU_CONST, 1.75) == 1.75


def test_lemmas_g0_positive_and_monotone():
    """Lemmas fnostat / G0pos: G0 > 0 and has no interior extremum in alpha,
    so the sup over the high frequencies sits at the ends (checked on a grid)."""
    a = np.linspace(np.pi / 2, np.pi, 401)
    p = np.arccosh(2 - np.cos(a))
    for th in np.linspace(0, 0.999, 40):
        cm2, cm1, c0 = coeff(th)
        G0 = cm2 * np.exp(-2 * p) + cm1 * np.exp(-p) + c0
        assert np.all(G0 > 0)
        dG = np.diff(G0)
        assert np.all(dG <= 1e-15) or np.all(dG >= -1e-15)
