"""Seeded synthetic inputs: level sets, manufactured solutions, data draws.

This module is shared by the tests, the benchmark, the oracle checks and the
serving loop.  It holds none of the multigrid method's arithmetic: only the
problem definitions (level-set functions sampled at grid nodes, exact
solutions and their Laplacians, random draws).  Everything is FP64 numpy and
laid out with x fastest, the node order the solver uses.

Domains:
  * circle and flower of the 2D Dirichlet tests (Sec. 3.3, eqs. dom2D:circle,
    dom2D:flower), the ellipsoid of the 3D tests (Sec. 4.2);
  * the shifted circle (65^2), the 3D "flower" r - (0.5 + 0.1 sin 3t sin 4p)
    (257^3 / 513^3), the batched 2D stars and the served sphere unions of the
    benchmark workloads;
  * the full box (phi = -1), a half-space phi = x - x_V (rectangle case,
    Sec. 3.2) and a line for Test1N-like set-ups.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable

import numpy as np

Array = np.ndarray


def node_coords(d: int, N: int):
    """Coordinates of the (N+1)^d nodes x_i = -1 + i h, h = 2/N, as d arrays
    of shape (N+1,)*d indexed [z][y][x] so that ravel() is x fastest."""
    x = -1.0 + np.arange(N + 1, dtype=np.float64) * (2.0 / N)
    if d == 1:
        return (x.copy(),)
    if d == 2:
        Y, X = np.meshgrid(x, x, indexing="ij")
        return (X, Y)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return (X, Y, Z)


def sample(d: int, N: int, fn: Callable[..., Array]) -> Array:
    """fn(x[, y[, z]]) evaluated at every node, flattened x fastest."""
    return np.ascontiguousarray(fn(*node_coords(d, N)), dtype=np.float64).ravel()


def points_eval(fn: Callable[..., Array], q: Array, d: int) -> Array:
    """fn at points q (n x 3, first d columns used)."""
    q = np.asarray(q, dtype=np.float64)
    return np.ascontiguousarray(fn(*[q[:, k] for k in range(d)]), dtype=np.float64)


# ---------------------------------------------------------------- level sets
def phi_full_box(*xs):
    return -np.ones_like(xs[0])


def phi_halfspace(xv: float):
    """x < x_V is the domain (the rectangle of Sec. 3.2 seen in [-1,1]^d)."""
    return lambda *xs: xs[0] - xv


def phi_circle(x0=0.02, y0=0.03, R=0.5):
    return lambda x, y: np.sqrt((x - x0) ** 2 + (y - y0) ** 2) - R


def phi_circle_paper():
    """Circle of the 2D tests: (x-x0)^2+(y-y0)^2-R^2, x0=sqrt3/40, y0=-sqrt4/40, R=sqrt2/2."""
    x0, y0, R = math.sqrt(3) / 40, -math.sqrt(4) / 40, math.sqrt(2) / 2
    return lambda x, y: (x - x0) ** 2 + (y - y0) ** 2 - R * R


def phi_flower2d(x0=math.sqrt(3) / 40, y0=-math.sqrt(4) / 40, r1=0.5, r2=0.2):
    """Five-petal flower of the 2D tests (centre read as the circle's)."""
    def f(x, y):
        X, Y = x - x0, y - y0
        r = np.sqrt(X * X + Y * Y)
        rr = np.where(r == 0, 1.0, r)
        poly = Y ** 5 + 5 * X ** 4 * Y - 10 * X ** 2 * Y ** 3
        return np.where(r == 0, -r1, r - r1 - r2 * poly / rr ** 5)
    return f


def phi_ellipsoid():
    """Ellipsoid of the 3D Dirichlet tests (semi-axes 0.686, 0.386, 0.586)."""
    cx, cy, cz = math.sqrt(2) / 20, math.sqrt(3) / 40, -math.sqrt(2) / 50
    return lambda x, y, z: ((x - cx) / 0.686) ** 2 + ((y - cy) / 0.386) ** 2 + ((z - cz) / 0.586) ** 2 - 1.0


def phi_flower3d(c=0.01, r0=0.5, amp=0.1):
    """r - (r0 + amp sin(3 theta) sin(4 varphi)), theta polar angle, varphi
    azimuth, about the centre (c, c, c); both angles 0 at the centre."""
    def f(x, y, z):
        X, Y, Z = x - c, y - c, z - c
        r = np.sqrt(X * X + Y * Y + Z * Z)
        rr = np.where(r == 0, 1.0, r)
        th = np.where(r == 0, 0.0, np.arccos(np.clip(Z / rr, -1.0, 1.0)))
        ph = np.arctan2(Y, X)
        return r - (r0 + amp * np.sin(3 * th) * np.sin(4 * ph))
    return f


def phi_star(R0: float, a: float, k: int):
    def f(x, y):
        r = np.sqrt(x * x + y * y)
        return r - (R0 + a * np.cos(k * np.arctan2(y, x)))
    return f


def phi_spheres(centres: Array, radii: Array):
    """Union of balls: min_i(|x - c_i| - r_i)."""
    centres = np.asarray(centres, dtype=np.float64)
    radii = np.asarray(radii, dtype=np.float64)

    def f(x, y, z):
        out = np.full(x.shape, np.inf)
        for (cx, cy, cz), r in zip(centres, radii):
            out = np.minimum(out, np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) - r)
        return out
    return f


# ------------------------------------------------------ manufactured solutions
@dataclass
class Manufactured:
    """Exact solution u and right-hand side f = -Laplace(u)."""
    u: Callable[..., Array]
    f: Callable[..., Array]


def exp_sin_2d() -> Manufactured:
    return Manufactured(u=lambda x, y: np.exp(x) * np.sin(y), f=lambda x, y: np.zeros_like(x))


def exp_sum(d: int) -> Manufactured:
    return Manufactured(u=lambda *xs: np.exp(sum(xs)), f=lambda *xs: -d * np.exp(sum(xs)))


def sincos_xy() -> Manufactured:
    pi = math.pi
    return Manufactured(u=lambda x, y: np.sin(pi * x) * np.cos(pi * y) + x * y,
                        f=lambda x, y: 2 * pi * pi * np.sin(pi * x) * np.cos(pi * y))


def quadratic_2d() -> Manufactured:
    """x^2 - y^2 + 3xy: harmonic, reproduced exactly by the 5-point stencil
    and by tensor-quadratic boundary interpolation."""
    return Manufactured(u=lambda x, y: x * x - y * y + 3 * x * y, f=lambda x, y: np.zeros_like(x))


def constant(c: float) -> Manufactured:
    return Manufactured(u=lambda *xs: np.full_like(xs[0], c), f=lambda *xs: np.zeros_like(xs[0]))


def smooth_random_f(rng: np.random.Generator, d: int = 3, terms: int = 8) -> Callable[..., Array]:
    """sum_q a_q cos(pi k_q . x + psi_q), k_q in {0..3}^d, a_q ~ U[-1,1], psi_q ~ U[0, 2pi)."""
    ks = rng.integers(0, 4, size=(terms, d))
    amps = rng.uniform(-1.0, 1.0, size=terms)
    phases = rng.uniform(0.0, 2 * math.pi, size=terms)

    def f(*xs):
        out = np.zeros_like(xs[0])
        for q in range(terms):
            arg = phases[q] + sum(math.pi * ks[q, k] * xs[k] for k in range(d))
            out = out + amps[q] * np.cos(arg)
        return out
    return f


# ------------------------------------------------------------ problem bundles
@dataclass
class Case:
    """A ready-to-solve problem definition (all arrays FP64, x fastest)."""
    name: str
    d: int
    N: int
    phi: Array                     # (N+1)^d node samples of the level set
    f: Array                       # (N+1)^d right-hand side at nodes
    u_exact: Callable[..., Array] | None   # for g(Q), g_B and error measurement
    g: Callable[..., Array]        # Dirichlet data on the curved boundary
    gB: Array                      # (N+1)^d box-face Dirichlet data (used on BOXDIR nodes)
    meta: dict = field(default_factory=dict)


def make_case(name: str, d: int, N: int, phi_fn, sol: Manufactured | None, f_fn=None, g_fn=None, **meta) -> Case:
    phi = sample(d, N, phi_fn)
    if sol is not None:
        f = sample(d, N, sol.f)
        g = sol.u
        gB = sample(d, N, sol.u)
        ue = sol.u
    else:
        f = sample(d, N, f_fn) if f_fn is not None else np.zeros((N + 1) ** d)
        g = g_fn if g_fn is not None else (lambda *xs: np.zeros_like(xs[0]))
        gB = sample(d, N, g)
        ue = None
    return Case(name, d, N, phi, f, ue, g, gB, dict(meta))


def circle_65() -> Case:
    """2D Poisson on the circle of radius 0.5 about (0.02, 0.03), 65^2 nodes, u = e^x sin y."""
    return make_case("circle65", 2, 64, phi_circle(), exp_sin_2d())


def flower3d(N: int = 256) -> Case:
    """3D flower, u = exp(x+y+z); N = 256 (257^3) or 512 (513^3)."""
    return make_case(f"flower3d_{N + 1}", 3, N, phi_flower3d(), exp_sum(3))


def ellipsoid(N: int) -> Case:
    return make_case(f"ellipsoid_{N + 1}", 3, N, phi_ellipsoid(), exp_sum(3))


def star_batch(count: int = 512, seed: int = 2207, sides=(65, 129, 257, 513, 1025)) -> list[Case]:
    """Independent 2D star problems; per problem the draws are, in order:
    side, R0 ~ U[0.3,0.6], a ~ U[0,0.1], k ~ U{3..8}; u = sin(pi x) cos(pi y) + x y."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        side = int(sides[rng.integers(0, len(sides))])
        R0 = float(rng.uniform(0.3, 0.6))
        a = float(rng.uniform(0.0, 0.1))
        k = int(rng.integers(3, 9))
        out.append(make_case(f"star{i}", 2, side - 1, phi_star(R0, a, k), sincos_xy(), R0=R0, a=a, k=k))
    return out


def star_params(count: int = 512, seed: int = 2207, sides=(65, 129, 257, 513, 1025)):
    """The same draws as star_batch without sampling the grids."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        side = int(sides[rng.integers(0, len(sides))])
        R0 = float(rng.uniform(0.3, 0.6))
        a = float(rng.uniform(0.0, 0.1))
        k = int(rng.integers(3, 9))
        out.append((side, R0, a, k))
    return out


def star_case(i: int, side: int, R0: float, a: float, k: int) -> Case:
    return make_case(f"star{i}", 2, side - 1, phi_star(R0, a, k), sincos_xy(), R0=R0, a=a, k=k)


def sphere_request(rng: np.random.Generator, sides=(33, 65, 129, 257)) -> Case:
    """One served request: side ~ U{sides}; m ~ U{4..64} balls, centres ~ U[-0.7,0.7]^3,
    radii ~ U[0.05,0.2]; random smooth f; g = 0."""
    side = int(sides[rng.integers(0, len(sides))])
    m = int(rng.integers(4, 65))
    centres = rng.uniform(-0.7, 0.7, size=(m, 3))
    radii = rng.uniform(0.05, 0.2, size=m)
    f_fn = smooth_random_f(rng, 3)
    return make_case(f"spheres{side}_{m}", 3, side - 1, phi_spheres(centres, radii), None, f_fn=f_fn,
                     side=side, m=m)


def random_guess(n: int, seed: int = 0) -> Array:
    """U(-1, 1) initial guess (convergence-factor protocol, Sec. 2.2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=n)


# ------------------------------------------------------- device-side sampling
def sphere_request_params(rng: np.random.Generator, sides=(33, 65, 129, 257)) -> dict:
    """The draws of one served request, in order: side ~ U{sides}; m ~ U{4..64};
    centres ~ U[-0.7,0.7]^3; radii ~ U[0.05,0.2]; the 8 terms of the random
    smooth f (k ~ U{0..3}^3, a ~ U[-1,1], psi ~ U[0,2pi))."""
    side = int(sides[rng.integers(0, len(sides))])
    m = int(rng.integers(4, 65))
    centres = rng.uniform(-0.7, 0.7, size=(m, 3))
    radii = rng.uniform(0.05, 0.2, size=m)
    ks = rng.integers(0, 4, size=(8, 3))
    amps = rng.uniform(-1.0, 1.0, size=8)
    phases = rng.uniform(0.0, 2 * math.pi, size=8)
    return dict(side=side, m=m, centres=centres, radii=radii, ks=ks, amps=amps, phases=phases)


def sample_sphere_request_torch(p: dict, device="cuda"):
    """phi = min_i(|x - c_i| - r_i) and f = sum_q a_q cos(pi k_q . x + psi_q) on
    the (side)^3 nodes, FP64, evaluated with torch on `device` (x fastest)."""
    import torch
    n = p["side"]
    x = -1.0 + torch.arange(n, dtype=torch.float64, device=device) * (2.0 / (n - 1))
    Z, Y, X = torch.meshgrid(x, x, x, indexing="ij")
    phi = torch.full_like(X, float("inf"))
    for (cx, cy, cz), r in zip(p["centres"], p["radii"]):
        phi = torch.minimum(phi, torch.sqrt((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2) - r)
    f = torch.zeros_like(X)
    for q in range(len(p["amps"])):
        k = p["ks"][q]
        f = f + p["amps"][q] * torch.cos(math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + p["phases"][q])
    return phi.reshape(-1).contiguous(), f.reshape(-1).contiguous()


def sample_sphere_request_numpy(p: dict):
    """The same phi and f as sample_sphere_request_torch, with numpy on the host."""
    X, Y, Z = node_coords(3, p["side"] - 1)
    phi = np.full(X.shape, np.inf)
    for (cx, cy, cz), r in zip(p["centres"], p["radii"]):
        phi = np.minimum(phi, np.sqrt((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2) - r)
    f = np.zeros_like(X)
    for q in range(len(p["amps"])):
        k = p["ks"][q]
        f = f + p["amps"][q] * np.cos(math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + p["phases"][q])
    return phi.ravel(), f.ravel()
