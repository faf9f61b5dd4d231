"""GPU tests of the mixed-precision solve and of batches (needs an MI355X).

Mixed precision (FP32 cycle on the correction, FP64 residual, update and
coarse solve): converges to the same relative residual as FP64 and stays
within 1e-8 (relative, max norm) of the oracle's FP64 solution solved to
1e-12.  Batches: every problem gives the same bits alone and in a batch of
different sizes, and matches the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2207_14208_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def oracle_solution(c, tol=1e-12):
    O = oracle.Problem(c.d, c.N, c.phi)
    og = O.ghosts(0)
    O.set_rhs(c.f, W.points_eval(c.g, og["q"], c.d))
    cls = O.classes(0)
    u = np.where(cls == oracle.BOXDIR, c.gB, 0.0)
    it, h = O.solve(u, tol, 300)
    return O, u, cls, it, h


def gpu_problem(c, **opt):
    from paper_2207_14208_amd.solver import Problem
    G = Problem(c.d, c.N, c.phi, **opt)
    gg = G.ghost_info(0)
    G.set_data(c.f, W.points_eval(c.g, gg["q"].cpu().numpy(), c.d))
    return G


@pytest.mark.parametrize("name", ["circle65", "ellipsoid33", "flower3d65"])
def test_mixed_precision_accuracy(name):
    _need_gpu()
    from paper_2207_14208_amd import _native as N
    c = {"circle65": W.circle_65, "ellipsoid33": lambda: W.ellipsoid(32), "flower3d65": lambda: W.flower3d(64)}[name]()
    O, ustar, cls, it, _ = oracle_solution(c)
    G = gpu_problem(c, precision=N.MIXED)
    u = G.initial_guess(torch.from_numpy(c.gB).cuda())
    st, hist = G.solve(u, 1e-10)
    assert st.status == 0, st
    Gd = gpu_problem(c)
    ud = Gd.initial_guess(torch.from_numpy(c.gB).cuda())
    std, _ = Gd.solve(ud, 1e-10)
    assert abs(st.cycles - std.cycles) <= 2, (st.cycles, std.cycles)
    m = (cls == oracle.INSIDE) | (cls == oracle.GHOST)
    err = np.abs(u.cpu().numpy()[m] - ustar[m]).max() / np.abs(ustar[m]).max()
    assert err <= 1e-8, err
    # the final residual is an FP64 residual of the FP64 iterate
    rn = O.norm(0, O.residual(0, u.cpu().numpy()))
    assert rn <= 1.01 * 1e-10 * st.r0


def test_batch_same_alone_and_in_mix():
    _need_gpu()
    from paper_2207_14208_amd.solver import Batch
    params = [(65, 0.45, 0.05, 3), (129, 0.35, 0.09, 7), (33, 0.55, 0.02, 4), (257, 0.5, 0.1, 8), (65, 0.3, 0.0, 5)]
    cases = [W.star_case(i, *p) for i, p in enumerate(params)]
    alone = []
    for c in cases:
        G = gpu_problem(c)
        u = G.initial_guess(torch.from_numpy(c.gB).cuda())
        st, h = G.solve(u, 1e-10)
        assert st.status == 0
        alone.append((st, u.cpu().numpy()))
    B = Batch(8)
    probs, us = [], []
    for c in cases:
        G = gpu_problem(c)
        u = G.initial_guess(torch.from_numpy(c.gB).cuda())
        probs.append(G)
        us.append(u)
    slots = [B.add(G, u, 1e-10) for G, u in zip(probs, us)]
    B.run(1, 200)
    for (st_a, u_a), s, u in zip(alone, slots, us):
        st, h = B.stats(s)
        assert st.status == 0 and st.cycles == st_a.cycles
        assert np.array_equal(u.cpu().numpy(), u_a)
    # and each matches the oracle after the same number of cycles
    for c, (st_a, u_a) in zip(cases[:3], alone[:3]):
        O = oracle.Problem(c.d, c.N, c.phi)
        og = O.ghosts(0)
        O.set_rhs(c.f, W.points_eval(c.g, og["q"], c.d))
        cls = O.classes(0)
        uo = np.where(cls == oracle.BOXDIR, c.gB, 0.0)
        O.solve(uo, 0.0, st_a.cycles)
        assert np.abs(uo - u_a).max() <= 1e-12 * np.abs(uo).max()


@pytest.mark.parametrize("name,coarse_nodes", [("circle65", 1200), ("flower3d65", 1200), ("star257", 300),
                                               ("star257", 5000), ("ellipsoid33", 1200)])
def test_coarse_levels_in_lds_same_as_in_hbm(name, coarse_nodes):
    """The per-problem coarse workgroup gives the same bits with its levels
    staged in LDS and kept in HBM."""
    _need_gpu()
    from paper_2207_14208_amd import _native as N
    from paper_2207_14208_amd.solver import Batch
    c = {"circle65": W.circle_65, "flower3d65": lambda: W.flower3d(64), "ellipsoid33": lambda: W.ellipsoid(32),
         "star257": lambda: W.star_case(0, 257, 0.45, 0.08, 5)}[name]()
    out = []
    for lds in (N.LDS_DEFAULT, 0):
        G = gpu_problem(c)
        u = G.initial_guess(torch.from_numpy(c.gB).cuda())
        B = Batch(2)
        B.set_param(N.PARAM_COARSE_NODES, coarse_nodes)
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


def test_mixed_precision_at_full_size():
    """The 513^3 flower in the benchmark's configuration (mixed precision,
    u0 = 0, g at the GPU's own projections, tolerance 1e-10), checked by
    properties the oracle can compute at this size: its FP64 residual of the
    final u meets the tolerance against its own r0, the GPU's r0 is the
    oracle's, u is within 1e-8 of the GPU's FP64 solve, and both carry the
    same discretisation error against the exact solution."""
    _need_gpu()
    from paper_2207_14208_amd import _native as N
    from paper_2207_14208_amd.solver import Problem
    c = W.flower3d(512)
    sols = {}
    for prec in (N.MIXED, N.FP64):
        G = Problem(3, c.N, torch.from_numpy(c.phi).cuda(), precision=prec)
        q = G.ghost_info(0)["q"]
        G.set_data(torch.from_numpy(c.f).cuda(), torch.exp(q[:, 0] + q[:, 1] + q[:, 2]))
        u = torch.zeros(G.nodes, dtype=torch.float64, device="cuda")
        st, _ = G.solve(u, 1e-10)
        assert st.status == 0, st
        sols[prec] = (st, u.cpu().numpy())
        G.close()
        del G, u, q
        torch.cuda.empty_cache()
    st, um = sols[N.MIXED]
    _, ud = sols[N.FP64]
    O = oracle.Problem(3, c.N, c.phi)
    og = O.ghosts(0)
    O.set_rhs(c.f, W.points_eval(c.g, og["q"], 3))
    cls = O.classes(0)
    m = (cls == oracle.INSIDE) | (cls == oracle.GHOST)
    r0 = O.norm(0, O.residual(0, np.zeros(cls.size)))
    assert abs(st.r0 - r0) <= 1e-10 * r0, (st.r0, r0)
    rn = O.norm(0, O.residual(0, um))
    assert rn <= 1.01 * 1e-10 * r0, (rn, r0)
    assert np.abs(um[m] - ud[m]).max() <= 1e-8 * np.abs(ud[m]).max()
    em = np.abs(um[m] - c.gB[m]).max()
    ed = np.abs(ud[m] - c.gB[m]).max()
    assert em <= 0.02 and abs(em - ed) <= 1e-8, (em, ed)


@pytest.mark.parametrize("name", ["flower3d65", "star1025", "flower3d513"])
def test_split_layout_same_bits_as_natural(name):
    """With BCMG_LAYOUT_SPLIT the FP32 arrays of the large levels of a
    mixed-precision problem are stored split by node parity (the finest
    level of all three cases; at 513^3 also the 257^3 level below it): the
    same arithmetic in another storage order, so the solve gives the same
    cycle count, history and u bits as with BCMG_LAYOUT_NATURAL, alone and
    in a batch with a problem too small to be split."""
    _need_gpu()
    from paper_2207_14208_amd import _native as N
    from paper_2207_14208_amd.solver import Batch
    c = {"flower3d65": lambda: W.flower3d(64), "star1025": lambda: W.star_case(0, 1025, 0.45, 0.08, 5),
         "flower3d513": lambda: W.flower3d(512)}[name]()
    small = W.star_case(1, 65, 0.35, 0.05, 3) if c.d == 2 else W.ellipsoid(32)
    out = []
    for layout in (N.LAYOUT_SPLIT, N.LAYOUT_NATURAL):
        G = gpu_problem(c, precision=N.MIXED, layout=layout)
        u = G.initial_guess(torch.from_numpy(c.gB).cuda())
        st, h = G.solve(u, 1e-10)
        assert st.status == 0, st
        out.append((st.cycles, h, u.cpu().numpy()))
        # in a batch beside a small problem (natural order)
        G2 = gpu_problem(c, precision=N.MIXED, layout=layout)
        u2 = G2.initial_guess(torch.from_numpy(c.gB).cuda())
        S = gpu_problem(small, precision=N.MIXED)
        us = S.initial_guess(torch.from_numpy(small.gB).cuda())
        B = Batch(2)
        s1 = B.add(G2, u2, 1e-10)
        B.add(S, us, 1e-10)
        B.run(1, 300)
        stb, hb = B.stats(s1)
        assert stb.cycles == st.cycles and np.array_equal(hb, h)
        assert np.array_equal(u2.cpu().numpy(), out[-1][2])
        B.close()
        for P in (G, G2, S):
            P.close()
    (c1, h1, u1), (c2, h2, u2) = out
    assert c1 == c2 and np.array_equal(h1, h2) and np.array_equal(u1, u2)


def test_paired_segment_sweep_same_bits():
    """FP32 sweeps of a split level with four row segments per wavefront
    and four nodes per lane (the default) give the same bits as one segment
    per wavefront (forced by a threshold above the level's segment count)."""
    _need_gpu()
    from paper_2207_14208_amd import _native as N
    from paper_2207_14208_amd.solver import Batch
    c = W.flower3d(128)
    out = []
    for pair_min in (1, 1 << 30):
        G = gpu_problem(c, precision=N.MIXED, layout=N.LAYOUT_SPLIT)
        u = G.initial_guess(torch.from_numpy(c.gB).cuda())
        B = Batch(1)
        B.set_param(N.PARAM_SWEEP_PAIR_SEGS, pair_min)
        s = B.add(G, u, 1e-10)
        B.run(1, 300)
        st, h = B.stats(s)
        assert st.status == 0, st
        out.append((st.cycles, h, u.cpu().numpy()))
        B.close()
        G.close()
    (c1, h1, u1), (c2, h2, u2) = out
    assert c1 == c2 and np.array_equal(h1, h2) and np.array_equal(u1, u2)


def test_stars512_batch_equals_solo_and_oracle():
    """The batched workload's own draw: 512 star problems (seed 2207, sides
    65..1025, mixed precision, tol 1e-10) solved in one batch with the
    workload's settings give every problem the same status, cycle count and
    u bits as its solve alone; one problem of each of three sides is within
    1e-8 of the oracle's FP64 solution."""
    _need_gpu()
    from paper_2207_14208_amd import _native as N
    from paper_2207_14208_amd.batching import BatchConfig, BatchSolver, make_problem
    params = W.star_params(512, seed=2207)
    cases = [W.star_case(i, *p) for i, p in enumerate(params)]
    cfg = BatchConfig(seg_len=128, coarse_nodes=5000, cycles_per_step=4, precision=N.MIXED)
    bs = BatchSolver(cases, cfg)
    r = bs.run()
    assert all(s == 0 for s in r.status), [s for s in r.status if s]
    batch_u = [u.cpu().numpy() for _, u, _ in bs.items]
    bs.close()
    checked = set()
    for i, c in enumerate(cases):
        G, u, _ = make_problem(c, cfg)
        st, _ = G.solve(u, cfg.tol)
        assert st.status == 0 and st.cycles == r.cycles[i], (i, st, r.cycles[i])
        ua = u.cpu().numpy()
        assert np.array_equal(ua, batch_u[i]), i
        G.close()
        if c.N in (64, 128, 256) and c.N not in checked:
            checked.add(c.N)
            O, ustar, cls, it, _ = oracle_solution(c)
            m = (cls == oracle.INSIDE) | (cls == oracle.GHOST)
            assert np.abs(ua[m] - ustar[m]).max() <= 1e-8 * np.abs(ustar[m]).max(), i
    assert checked == {64, 128, 256}


def test_coarse_workgroup_in_hbm_over_a_large_level():
    """The per-problem coarse workgroup in HBM (LDS off) over levels larger
    than those that keep an INSIDE list (the 65^3 flower's 33^3 level,
    35937 nodes): the batch builds no LDS programs or images then (the image
    copy once read the missing list), and the solve matches the oracle after
    the same cycles."""
    _need_gpu()
    from paper_2207_14208_amd import _native as N
    from paper_2207_14208_amd.solver import Batch
    c = W.flower3d(64)
    G = gpu_problem(c)
    u = G.initial_guess(torch.from_numpy(c.gB).cuda())
    B = Batch(1)
    B.set_param(N.PARAM_COARSE_NODES, 40000)
    B.set_param(N.PARAM_LDS_BYTES, 0)
    s = B.add(G, u, 1e-10)
    B.run(1, 300)
    st, _ = B.stats(s)
    assert st.status == 0, st
    O = oracle.Problem(c.d, c.N, c.phi)
    og = O.ghosts(0)
    O.set_rhs(c.f, W.points_eval(c.g, og["q"], c.d))
    cls = O.classes(0)
    uo = np.where(cls == oracle.BOXDIR, c.gB, 0.0)
    O.solve(uo, 0.0, st.cycles)
    assert np.abs(uo - u.cpu().numpy()).max() <= 1e-12 * np.abs(uo).max()
    B.close()
    G.close()


@pytest.mark.parametrize("d,N", [(3, 64), (2, 512)])
def test_split_sweep_with_ghosts_on_a_box_face(d, N):
    """The domain y > -1 + h/2: the whole face y = -1 is a row of ghosts next
    to INSIDE nodes, so segments of the split sweep lie on the box face and
    their lanes' neighbour reads start below the array (clamped, and never
    used).  Split and natural storage give the same bits, and the mixed
    solve meets the FP64 residual tolerance by the oracle's residual."""
    _need_gpu()
    from paper_2207_14208_amd import _native as N_
    h = 2.0 / N
    sol = W.Manufactured(u=(lambda x, y: np.sin(x) * np.cos(y)) if d == 2 else (lambda x, y, z: np.exp(x + y + z)),
                         f=(lambda x, y: 2 * np.sin(x) * np.cos(y)) if d == 2 else (lambda x, y, z: -3 * np.exp(x + y + z)))
    c = W.make_case("face", d, N, lambda *xs: (-1.0 + 0.5 * h) - xs[1], sol)
    O = oracle.Problem(c.d, c.N, c.phi)
    cls = O.classes(0)
    face_ghosts = int(np.count_nonzero(cls.reshape((N + 1,) * d)[(slice(None),) * (d - 2) + (0,)] == oracle.GHOST))
    assert face_ghosts > 0
    out = []
    for layout in (N_.LAYOUT_SPLIT, N_.LAYOUT_NATURAL):
        G = gpu_problem(c, precision=N_.MIXED, layout=layout)
        u = G.initial_guess(torch.from_numpy(c.gB).cuda())
        st, hist = G.solve(u, 1e-10)
        assert st.status == 0, st
        out.append((st.cycles, hist, u.cpu().numpy()))
        G.close()
    (c1, h1, u1), (c2, h2, u2) = out
    assert c1 == c2 and np.array_equal(h1, h2) and np.array_equal(u1, u2)
    O.set_rhs(c.f, W.points_eval(c.g, O.ghosts(0)["q"], c.d))
    u0 = np.where(cls == oracle.BOXDIR, c.gB, 0.0)
    r0 = O.norm(0, O.residual(0, u0))
    assert O.norm(0, O.residual(0, u1)) <= 1e-10 * r0 * 1.001


@pytest.mark.parametrize("mixed", [False, True])
def test_solve_into_another_array_same_as_fresh_problem(mixed):
    """A second solve of the same problem into another caller array (the
    descriptors that name u are rewritten in place, the work lists and graphs
    kept) gives the bits of a fresh problem solving into that array, and
    leaves the first array as its own solve left it."""
    _need_gpu()
    from paper_2207_14208_amd import _native as N
    c = W.flower3d(64)
    prec = N.MIXED if mixed else N.FP64
    G = gpu_problem(c, precision=prec, check_interval=4)
    gB = torch.from_numpy(c.gB).cuda()
    u1 = G.initial_guess(gB)
    st1, h1 = G.solve(u1, 1e-10)
    first = u1.clone()
    u2 = G.initial_guess(gB)
    st2, h2 = G.solve(u2, 1e-10)
    assert torch.equal(u1, first)
    F = gpu_problem(c, precision=prec, check_interval=4)
    u3 = F.initial_guess(gB)
    st3, h3 = F.solve(u3, 1e-10)
    assert st2.status == 0 and st2.cycles == st3.cycles
    assert np.array_equal(h2, h3, equal_nan=True)
    assert torch.equal(u2, u3)
    # and back into the first array: the same result again
    u1.copy_(G.initial_guess(gB))
    st4, _ = G.solve(u1, 1e-10)
    assert st4.cycles == st3.cycles and torch.equal(u1, u3)
    G.close()
    F.close()
