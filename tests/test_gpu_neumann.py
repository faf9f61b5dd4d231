"""GPU parity of Neumann ghost rows and the reaction term (needs an MI355X).

The cases are the paper's Neumann tests (Sec. 3.3 Test1N: Neumann on the
oblique line, Dirichlet on the box; Test2N and Sec. 4.2: c u - Laplace u with
Neumann rows on the circle and the ellipsoid) plus a 1D half-line, each with a
manufactured solution whose boundary data is grad u(Q) . n at every ghost.

 * setup: classes, ghost lists, stencil codes and fallback flags bit-exact;
   eta, normal, Q, tau and dtau within 1e-13;
 * single steps on identical inputs within 1e-12 (relative);
 * whole FP64 solves: cycle counts within one, per-cycle norms within 1e-8,
   u after the GPU's cycle count within 1e-12 of the oracle's;
 * a batch mixing Dirichlet and Neumann problems gives each problem's
   results alone; LDS and HBM coarse workgroups agree bit for bit; the mixed
   precision solve reaches the FP64 solution to 1e-8.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2207_14208_amd import workloads as W
from parity_util import cycles_agree, histories_agree, residual_floor

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NEU = oracle.BC_NEUMANN


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


class NCase:
    def __init__(self, name, d, N, phi_fn, u, grad, lap, c):
        self.name, self.d, self.N, self.c = name, d, N, c
        self.phi = W.sample(d, N, phi_fn)
        self.u, self.grad = u, grad
        self.f = c * W.sample(d, N, u) - W.sample(d, N, lap)
        self.gB = W.sample(d, N, u)

    def gdata(self, q, n):
        q = np.asarray(q)
        n = np.asarray(n)
        cols = [q[:, k] for k in range(self.d)]
        gr = np.stack([gk(*cols) * np.ones(len(q)) for gk in self.grad], axis=1)
        return (gr * n[:, : self.d]).sum(axis=1)


def _exp_sin():
    u = lambda x, y: np.exp(x) * np.sin(y)
    return u, (u, lambda x, y: np.exp(x) * np.cos(y)), lambda x, y: np.zeros_like(x)


def _exp_sum3():
    u = lambda x, y, z: np.exp(x + y + z)
    return u, (u, u, u), lambda x, y, z: 3.0 * np.exp(x + y + z)


def _spheres():
    rng = np.random.Generator(np.random.PCG64(7))
    cen = rng.uniform(-0.7, 0.7, size=(30, 3))
    rad = rng.uniform(0.05, 0.2, size=30)
    return W.phi_spheres(cen, rad)


def _line(N):
    h = 2.0 / N
    return lambda x, y: 0.5 * (x + math.sqrt(3.0) * y - 1.0 + 0.7 * h)


CASES = {
    "test1n_65": lambda: NCase("test1n_65", 2, 64, _line(64), *_exp_sin(), 0.0),
    "circle_react_129": lambda: NCase("circle_react_129", 2, 128, W.phi_circle_paper(), *_exp_sin(), 1.0),
    "ellipsoid_react_33": lambda: NCase("ellipsoid_react_33", 3, 32, W.phi_ellipsoid(), *_exp_sum3(), 1.0),
    "ellipsoid_react_65": lambda: NCase("ellipsoid_react_65", 3, 64, W.phi_ellipsoid(), *_exp_sum3(), 1.0),
    # 30 spheres, some 3 nodes across: coarse levels hold Neumann rows with no
    # admissible block (the one-sided fallback); too under-resolved to solve
    "spheres_react_65": lambda: NCase("spheres_react_65", 3, 64, _spheres(), *_exp_sum3(), 1.0),
    "line1d_129": lambda: NCase("line1d_129", 1, 128, W.phi_halfspace(0.3137), lambda x: np.exp(x),
                                (lambda x: np.exp(x),), lambda x: np.exp(x), 0.5),
}


def build_pair(name, **opt):
    _gpu()
    from paper_2207_14208_amd.solver import Problem
    c = CASES[name]()
    oo = {k: v for k, v in opt.items() if k in ("dtau_mode", "dtau_const", "nu1", "nu2")}
    O = oracle.Problem(c.d, c.N, c.phi, oracle.Options(bc=NEU, reaction=c.c, **oo))
    G = Problem(c.d, c.N, c.phi, bc=NEU, reaction=c.c, **opt)
    return c, O, G


def set_data(c, O, G):
    og = O.ghosts(0)
    gg = G.ghost_info(0)
    O.set_rhs(c.f, c.gdata(og["q"], og["n"]))
    G.set_data(c.f, c.gdata(gg["q"].cpu().numpy(), gg["n"].cpu().numpy()))
    return O.rhs(0)


def unknowns(cls):
    return (cls == oracle.INSIDE) | (cls == oracle.GHOST)


def _close(a, b, tol=1e-12):
    scale = max(np.abs(a).max(), np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() <= tol * scale


@pytest.mark.parametrize("name", list(CASES))
def test_neumann_setup_parity(name):
    c, O, G = build_pair(name)
    assert G.levels == O.L
    for l in range(O.L):
        assert np.array_equal(O.classes(l), G.classes(l).cpu().numpy())
        og = O.ghosts(l)
        gg = {k: v.cpu().numpy() for k, v in G.ghost_info(l).items()}
        assert np.array_equal(og["idx"], gg["idx"].astype(np.int64))
        code = gg["code"]
        w = np.stack([(code >> (2 * k)) & 3 for k in range(3)], axis=1)
        s = np.stack([np.where((code >> (6 + k)) & 1, -1, 1) for k in range(3)], axis=1)
        assert np.array_equal(w, og["w"]), f"level {l}: widths differ"
        assert np.array_equal(s[:, : c.d], og["s"][:, : c.d]), f"level {l}: signs differ"
        assert np.array_equal(gg["fb"], og["fb"])
        for key in ("eta", "n", "q", "tau", "dtau"):
            assert np.allclose(og[key], gg[key], rtol=1e-13, atol=1e-13), (l, key, np.abs(og[key] - gg[key]).max())


@pytest.mark.parametrize("name,levels", [("test1n_65", (0, 1)), ("circle_react_129", (0, 1)),
                                         ("ellipsoid_react_33", (0, 1)), ("line1d_129", (0, 1)),
                                         ("spheres_react_65", (0, 2, 3))])
def test_neumann_step_parity(name, levels):
    c, O, G = build_pair(name)
    rhs0 = set_data(c, O, G)
    rng = np.random.default_rng(17)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    if name.startswith("spheres"):  # the levels below hold one-sided fallback rows
        assert all((O.ghosts(l)["fb"] & 2).any() for l in levels[1:])
    for l in levels:
        cls = O.classes(l)
        nn = cls.size
        rhs = rhs0 if l == 0 else np.where(unknowns(cls), rng.standard_normal(nn), 0.0)
        u = np.where(unknowns(cls), rng.uniform(-1, 1, nn), 0.0)
        if l == 0:  # box-face Dirichlet values, read by Neumann rows there
            u[cls == oracle.BOXDIR] = rng.uniform(-1, 1, (cls == oracle.BOXDIR).sum())
        uo = u.copy()
        O.smooth(l, uo, rhs, steps=3)
        ug = dev(u)
        G.level_smooth(l, ug, dev(rhs), 3)
        assert _close(uo, ug.cpu().numpy()), f"smooth level {l}"
        ro = O.residual(l, u, rhs)
        rg = torch.zeros(nn, dtype=torch.float64, device="cuda")
        ng = G.level_residual(l, dev(u), dev(rhs), rg, with_norm=True)
        assert _close(ro, rg.cpu().numpy()), f"residual level {l}"
        assert abs(ng - O.norm(l, ro)) <= 1e-12 * O.norm(l, ro)
    L = O.L - 1
    cls = O.classes(L)
    rhs = np.where(unknowns(cls), rng.standard_normal(cls.size), 0.0)
    uo = np.zeros(cls.size)
    O.coarse_solve(uo, rhs)
    ug = torch.zeros(cls.size, dtype=torch.float64, device="cuda")
    G.coarse_solve(ug, dev(rhs))
    assert _close(uo, ug.cpu().numpy(), 1e-11)


def _check_solve(c, O, it, ho, st, hg, ug, tol=1e-10):
    uo = oracle_after(c, O, st.cycles)
    floor = residual_floor(c.d, c.N, O.classes(0), uo, O.rhs(0), O.opts.reaction)
    assert cycles_agree(st.cycles, it, ho, tol, floor), (st.cycles, it)
    assert histories_agree(hg, ho, floor)
    assert _close(uo, ug, 1e-12)


def solve_pair(name, tol=1e-10, **opt):
    c, O, G = build_pair(name, **opt)
    set_data(c, O, G)
    cls = O.classes(0)
    uo = np.where(cls == oracle.BOXDIR, c.gB, 0.0)
    it, ho = O.solve(uo, tol)
    ug = G.initial_guess(torch.from_numpy(c.gB).cuda())
    st, hg = G.solve(ug, tol)
    return c, O, G, it, ho, st, hg, ug.cpu().numpy()


def oracle_after(c, O, cycles):
    cls = O.classes(0)
    u = np.where(cls == oracle.BOXDIR, c.gB, 0.0)
    O.solve(u, 0.0, cycles)
    return u


@pytest.mark.parametrize("name", ["test1n_65", "circle_react_129", "ellipsoid_react_33", "ellipsoid_react_65",
                                  "line1d_129"])
def test_neumann_solve_parity(name):
    c, O, G, it, ho, st, hg, ug = solve_pair(name)
    assert it > 0 and st.status == 0, (it, st)
    _check_solve(c, O, it, ho, st, hg, ug)


@pytest.mark.parametrize("mode,const", [(1, 1.0), (2, 0.75)])
def test_neumann_dtau_modes(mode, const):
    c, O, G, it, ho, st, hg, ug = solve_pair("test1n_65", dtau_mode=mode, dtau_const=const)
    assert it > 0 and st.status == 0, (it, st)
    _check_solve(c, O, it, ho, st, hg, ug)


def test_batch_mixing_dirichlet_and_neumann():
    """Dirichlet problems in a batch that also holds Neumann problems run the
    kernels with both row types compiled in; every problem matches its solve
    alone."""
    _gpu()
    from paper_2207_14208_amd.solver import Batch, Problem

    def make(kind):
        if kind == "dir":
            d = W.circle_65()
            G = Problem(d.d, d.N, d.phi)
            gg = G.ghost_info(0)
            G.set_data(d.f, W.points_eval(d.g, gg["q"].cpu().numpy(), d.d))
            return G, d.gB
        c = CASES[kind]()
        G = Problem(c.d, c.N, c.phi, bc=NEU, reaction=c.c)
        gg = G.ghost_info(0)
        G.set_data(c.f, c.gdata(gg["q"].cpu().numpy(), gg["n"].cpu().numpy()))
        return G, c.gB

    kinds = ["dir", "test1n_65", "circle_react_129", "dir"]
    alone = []
    for k in kinds:
        G, gB = make(k)
        u = G.initial_guess(torch.from_numpy(gB).cuda())
        st, _ = G.solve(u, 1e-10)
        assert st.status == 0
        alone.append((st.cycles, u.cpu().numpy()))
    B = Batch(4)
    items = []
    for k in kinds:
        G, gB = make(k)
        u = G.initial_guess(torch.from_numpy(gB).cuda())
        items.append((G, u, B.add(G, u, 1e-10)))
    B.run(1, 200)
    for (cyc, ua), (G, u, s) in zip(alone, items):
        st, _ = B.stats(s)
        assert st.status == 0 and st.cycles == cyc
        assert _close(ua, u.cpu().numpy(), 1e-13)


@pytest.mark.parametrize("name", ["circle_react_129", "ellipsoid_react_33"])
def test_neumann_coarse_levels_in_lds_same_as_in_hbm(name):
    _gpu()
    from paper_2207_14208_amd import _native as N
    from paper_2207_14208_amd.solver import Batch, Problem
    c = CASES[name]()
    out = []
    for lds in (N.LDS_DEFAULT, 0):
        G = Problem(c.d, c.N, c.phi, bc=NEU, reaction=c.c)
        gg = G.ghost_info(0)
        G.set_data(c.f, c.gdata(gg["q"].cpu().numpy(), gg["n"].cpu().numpy()))
        u = G.initial_guess(torch.from_numpy(c.gB).cuda())
        B = Batch(2)
        B.set_param(N.PARAM_COARSE_NODES, 1200)
        B.set_param(N.PARAM_LDS_BYTES, lds)
        s = B.add(G, u, 1e-10)
        B.run(1, 300)
        st, h = B.stats(s)
        out.append((st.status, st.cycles, h, u.cpu().numpy()))
        B.close()
        G.close()
    (s1, c1, h1, u1), (s2, c2, h2, u2) = out
    assert (s1, c1) == (s2, c2) and s1 == 0
    assert np.array_equal(h1, h2)
    assert np.array_equal(u1, u2)


@pytest.mark.parametrize("name", ["circle_react_129", "ellipsoid_react_65"])
def test_neumann_mixed_precision(name):
    _gpu()
    from paper_2207_14208_amd import _native as N
    c, O, G = build_pair(name, precision=N.MIXED)
    set_data(c, O, G)
    cls = O.classes(0)
    # the converged FP64 solution: the Neumann rows put the residual's
    # rounding floor near 1e-12 of r0, so a fixed 60 cycles rather than a
    # tolerance (the FP64 solve to 1e-10 is within 2e-11 of it)
    ustar = np.where(cls == oracle.BOXDIR, c.gB, 0.0)
    O.solve(ustar, 0.0, 60)
    u = G.initial_guess(torch.from_numpy(c.gB).cuda())
    st, _ = G.solve(u, 1e-10)
    assert st.status == 0, st
    m = unknowns(cls)
    err = np.abs(u.cpu().numpy()[m] - ustar[m]).max() / np.abs(ustar[m]).max()
    assert err <= 1e-8, err


@pytest.mark.parametrize("name", ["ellipsoid_react_65", "spheres_react_65", "circle_react_129", "flower_dirichlet_65"])
def test_memory_estimate_covers_the_problem(name):
    """bcmg_estimate_bytes (used for admission control) is at least what a
    problem of that size holds, for Dirichlet and Neumann rows alike."""
    _gpu()
    from paper_2207_14208_amd import _native as N
    from paper_2207_14208_amd.solver import Problem, estimate_bytes
    if name == "flower_dirichlet_65":
        c = W.flower3d(64)
        G = Problem(c.d, c.N, c.phi)
    else:
        c = CASES[name]()
        G = Problem(c.d, c.N, c.phi, bc=NEU, reaction=c.c)
    for prec in (N.FP64,):
        est = estimate_bytes(c.d, c.N, prec)
        assert G.device_bytes() <= est, (G.device_bytes(), est)
    G.close()


def test_pure_neumann_poisson_reports_not_converged():
    """Neumann rows on the whole boundary with c = 0 make the problem
    singular (Sec. 3.3): the coarsest operator is flagged singular and
    smoothed instead of inverted, the residual stalls, and the solve ends
    NOT_CONVERGED at max_cycles with finite norms that follow the oracle's."""
    _gpu()
    from paper_2207_14208_amd import _native as N
    from paper_2207_14208_amd.solver import Problem
    n = 64
    phi = W.sample(2, n, W.phi_circle_paper())
    f = W.sample(2, n, lambda x, y: np.cos(3 * x) * np.sin(2 * y) + 0.3)
    O = oracle.Problem(2, n, phi, oracle.Options(bc=NEU, reaction=0.0))
    assert O.coarse_singular()
    ng = O.counts(0)[1]
    O.set_rhs(f, np.zeros(ng))
    uo = np.zeros(O.nodes(0))
    it, ho = O.solve(uo, 1e-10, 20)
    assert it == -1
    G = Problem(2, n, phi, bc=NEU, reaction=0.0, max_cycles=20)
    G.set_data(f, np.zeros(ng))
    ug = G.initial_guess()
    st, hg = G.solve(ug, 1e-10)
    assert st.status == N.ERR_NOT_CONVERGED and st.cycles == 20, st
    hg = np.asarray(hg)
    assert np.all(np.isfinite(hg))
    assert histories_agree(hg, ho, residual_floor(2, n, O.classes(0), uo, O.rhs(0)))
