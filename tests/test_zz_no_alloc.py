"""bcmg_residual_norm_noalloc through the C ABI on an MI355X: the same norm
as bcmg_residual_norm, on two calls in a row (the second on a smaller
problem, so stale partial sums of the first would show), with no device
allocation by the call; and the size limit reported as an error."""
import ctypes as C

import numpy as np
import pytest

from paper_2207_14208_amd import _native as N
from paper_2207_14208_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _norms(G, u):
    L = N.lib()
    a, b = C.c_double(), C.c_double()
    N.check(L.bcmg_residual_norm(G.h, C.c_void_p(u.data_ptr()), C.byref(a)))
    N.check(L.bcmg_residual_norm_noalloc(G.h, C.c_void_p(u.data_ptr()), C.byref(b)))
    return a.value, b.value


def _problem(c):
    from paper_2207_14208_amd.solver import Problem
    G = Problem(c.d, c.N, c.phi)
    q = G.ghost_info(0)["q"].cpu().numpy()
    G.set_data(c.f, W.points_eval(c.g, q, c.d))
    rng = np.random.default_rng(3)
    u = torch.from_numpy(rng.uniform(-1, 1, G.nodes)).cuda()
    return G, u


def test_noalloc_norm_matches_and_allocates_nothing():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_14208_amd import solver
    big, small = W.flower3d(128), W.circle_65()
    Gb, ub = _problem(big)
    Gs, us = _problem(small)
    assert Gb.level_info(0)["n_segments"] > 4 * Gs.level_info(0)["n_segments"]
    # count allocations made while the no-allocation entry point runs
    calls = []
    cbs = (N.ALLOC_FN(lambda n, s, c: calls.append(n) or None), N.FREE_FN(lambda p, n, s, c: calls.append(-1)))
    N.check(N.lib().bcmg_set_allocator(C.cast(cbs[0], C.c_void_p), C.cast(cbs[1], C.c_void_p), None))
    try:
        before = torch.cuda.memory_allocated()
        for G, u in ((Gb, ub), (Gs, us), (Gb, ub)):
            a, b = _norms(G, u)
            assert a > 0 and b == a, (a, b)
        assert torch.cuda.memory_allocated() == before
    finally:
        solver.use_torch_allocator(True)
    # bcmg_residual_norm allocates nothing after setup either, so the counter
    # stays empty for both
    assert calls == []
    # after a solve, the converged residual's norm agrees too
    st, _ = Gs.solve(us, 1e-10)
    a, b = _norms(Gs, us)
    assert st.status == 0 and b == a and a <= 1e-10 * st.r0 * 1.01
    Gb.close()
    Gs.close()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    """A full 513^3 box has about 1.04e6 finest row segments, more than the
    static array holds: the call fails with BCMG_ERR_INVALID and names the
    limit; the allocating entry point still works."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_14208_amd.solver import Problem
    N_ = 512
    G = Problem(3, N_, -torch.ones((N_ + 1) ** 3, dtype=torch.float64, device="cuda"))
    assert G.level_info(0)["n_segments"] > (1 << 19)
    u = torch.zeros(G.nodes, dtype=torch.float64, device="cuda")
    G.set_data(torch.ones(G.nodes, dtype=torch.float64, device="cuda"),
               torch.zeros(0, dtype=torch.float64, device="cuda"))
    v = C.c_double(-1.0)
    st = N.lib().bcmg_residual_norm_noalloc(G.h, C.c_void_p(u.data_ptr()), C.byref(v))
    assert st == N.ERR_INVALID and b"at most" in N.lib().bcmg_last_error()
    assert v.value == -1.0
    assert G.residual_norm(u) > 0
    G.close()
