"""Device memory through the caller's allocator (bcmg_set_allocator), via the
C ABI on an MI355X: every byte a problem holds comes from the callbacks,
setup temporaries and batch tables included, and everything is returned."""
import ctypes as C

import numpy as np
import pytest

from paper_2207_14208_amd import _native as N
from paper_2207_14208_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


class Counting:
    """Callbacks over torch's caching allocator that record every block."""

    def __init__(self, fail_at=None):
        self.live, self.allocs, self.frees, self.peak, self.fail_at = {}, 0, 0, 0, fail_at
        self.calls = 0
        self.cbs = (N.ALLOC_FN(self._alloc), N.FREE_FN(self._free))

    def _alloc(self, nbytes, stream, ctx):
        self.calls += 1
        if self.fail_at is not None and self.calls == self.fail_at:
            return None
        p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        self.live[p] = int(nbytes)
        self.allocs += 1
        self.peak = max(self.peak, sum(self.live.values()))
        return p

    def _free(self, ptr, nbytes, stream, ctx):
        assert self.live.pop(ptr) == nbytes
        self.frees += 1
        torch.cuda.caching_allocator_delete(ptr)

    def install(self):
        N.check(N.lib().bcmg_set_allocator(C.cast(self.cbs[0], C.c_void_p), C.cast(self.cbs[1], C.c_void_p), None))

    def bytes(self):
        return sum(self.live.values())


@pytest.fixture
def counting():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_14208_amd import solver
    solver._ensure_torch_allocator()
    cnt = Counting()
    cnt.install()
    yield cnt
    solver.use_torch_allocator(True)


def test_problem_memory_comes_from_the_callbacks(counting):
    from paper_2207_14208_amd.solver import Problem
    c = W.flower3d(64)
    G = Problem(3, 64, c.phi)
    # after setup, what the callbacks hold is exactly what the problem reports
    assert counting.bytes() == G.device_bytes() > 0
    # setup temporaries went through them too (and were returned)
    assert counting.frees > 0 and counting.allocs == counting.frees + len(counting.live)
    q = G.ghost_info(0)["q"]
    G.set_data(c.f, torch.exp(q[:, 0] + q[:, 1] + q[:, 2]))
    u = G.initial_guess(torch.from_numpy(c.gB).cuda())
    st, _ = G.solve(u, 1e-10)
    assert st.status == 0
    # the solve's batch tables are the callbacks' too
    assert counting.bytes() > G.device_bytes()
    G.close()
    torch.cuda.synchronize()
    assert counting.bytes() == 0 and counting.allocs == counting.frees


@pytest.mark.parametrize("fail_at", [1, 4, 12, 30, 60])
def test_failed_allocation_is_oom_and_leaks_nothing(counting, fail_at):
    """The k-th allocation of a setup fails: setup reports BCMG_ERR_OOM and
    every block taken before it (arrays and temporaries) is returned."""
    from paper_2207_14208_amd.solver import Problem
    counting.fail_at = fail_at
    c = W.flower3d(64)
    try:
        G = Problem(3, 64, c.phi)
    except N.BcmgError as e:
        assert e.status == N.ERR_OOM, e
    else:  # fewer allocations than fail_at
        assert counting.calls < fail_at
        G.close()
    torch.cuda.synchronize()
    assert counting.bytes() == 0


def test_handles_keep_their_source(counting):
    """A problem set up under one allocator frees through it even after the
    allocator is changed."""
    from paper_2207_14208_amd.solver import Problem
    c = W.circle_65()
    G = Problem(2, 64, c.phi)
    held = counting.bytes()
    assert held == G.device_bytes()
    other = Counting()
    other.install()
    G2 = Problem(2, 64, c.phi)
    assert other.bytes() == G2.device_bytes() and counting.bytes() == held
    G.close()
    G2.close()
    torch.cuda.synchronize()
    assert counting.bytes() == 0 and other.bytes() == 0
