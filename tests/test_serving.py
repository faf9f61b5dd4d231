"""Scheduler of the continuous-batching server (admission, slot reuse,
retirement, rejection), driven by a CPU stand-in backend; and the seeded
request draws.  No GPU."""
import threading

import numpy as np
import pytest

from paper_2207_14208_amd import serving as S
from paper_2207_14208_amd import workloads as W


class FakeBackend:
    """Each request needs `cycles` V-cycles (drawn from its parameters); the
    batch has `capacity` slots and hands out the lowest free one."""

    def __init__(self, capacity, fail_side=None, bytes_per_node=100):
        self.capacity = capacity
        self.left = {}
        self.cycles = {}
        self.fail_side = fail_side
        self.bpn = bytes_per_node
        self.max_resident = 0
        self.lock = threading.Lock()
        self.prepared_threads = set()

    def estimate(self, req):
        return self.bpn * req.params["side"] ** 3

    def prepare(self, req):
        self.prepared_threads.add(threading.get_ident())
        if req.params["side"] == self.fail_side:
            raise RuntimeError("setup rejected")
        return (req.rid, 1 + req.params["m"] % 5)

    def add(self, handle):
        slot = min(set(range(self.capacity)) - set(self.left))
        self.left[slot] = handle[1]
        self.cycles[slot] = 0
        self.max_resident = max(self.max_resident, len(self.left))
        return slot

    def step(self, cycles):
        act = np.zeros(self.capacity, dtype=np.int32)
        for s in self.left:
            n = min(cycles, self.left[s])
            self.left[s] -= n
            self.cycles[s] += n
            act[s] = 1 if self.left[s] > 0 else 0
        return act

    def finish(self, slot):
        self.left.pop(slot)
        return 0, self.cycles.pop(slot), 1000


class FailingOnceBackend(FakeBackend):
    """Requests with an even sphere count fail (status 5) on their first solve."""
    retry_statuses = (5,)
    max_attempts = 2

    def prepare(self, req):
        rid, cyc = super().prepare(req)
        fail = req.attempts == 1 and req.params["m"] % 2 == 0
        return (rid, cyc, fail)

    def add(self, handle):
        slot = super().add(handle)
        self.fail = getattr(self, "fail", {})
        self.fail[slot] = handle[2]
        return slot

    def finish(self, slot):
        st, cyc, n = super().finish(slot)
        return (5 if self.fail.pop(slot) else st), cyc, n


def _requests(n, seed=3, rate=0.0, sides=(33, 65)):
    return S.make_requests(n, seed, rate, sides=sides)


def test_all_requests_complete_with_their_cycle_counts():
    be = FakeBackend(4)
    srv = S.Server(be, slots=4, budget_bytes=1 << 40, cycles_per_step=2)
    reqs = _requests(30)
    st = S.run(srv, reqs, max_seconds=30)
    srv.close()
    assert len(st.completed) == 30 and not st.rejected
    for r in st.completed:
        assert r.cycles == 1 + r.params["m"] % 5
        assert r.done >= r.admitted >= r.arrival
    assert be.max_resident <= 4
    assert st.peak_slots == 4
    # preparation runs off the main thread
    assert threading.get_ident() not in be.prepared_threads


def test_memory_budget_limits_residency():
    be = FakeBackend(16)
    big = 100 * 65 ** 3
    srv = S.Server(be, slots=16, budget_bytes=2 * big + 1, cycles_per_step=1)
    reqs = _requests(20, sides=(65,))
    st = S.run(srv, reqs, max_seconds=30)
    srv.close()
    assert len(st.completed) == 20
    assert st.peak_bytes <= 2 * big + 1
    assert be.max_resident <= 2
    assert srv.used_bytes == 0


def test_oversized_and_failed_requests_are_rejected_not_fatal():
    be = FakeBackend(4, fail_side=33)
    srv = S.Server(be, slots=4, budget_bytes=100 * 65 ** 3, cycles_per_step=2)
    reqs = _requests(24, sides=(33, 65, 129))
    st = S.run(srv, reqs, max_seconds=30)
    srv.close()
    sides = [r.params["side"] for r in reqs]
    assert len(st.completed) == sides.count(65)
    assert len(st.rejected) == sides.count(33) + sides.count(129)
    assert all(r.rejected for r in st.rejected)
    assert srv.used_bytes == 0


def test_poisson_arrivals_are_served_after_they_arrive():
    be = FakeBackend(8)
    srv = S.Server(be, slots=8, budget_bytes=1 << 40)
    reqs = _requests(40, rate=2000.0)
    st = S.run(srv, reqs, max_seconds=30)
    srv.close()
    assert len(st.completed) == 40
    assert all(r.admitted >= r.arrival for r in st.completed)
    assert np.isfinite(st.percentile_ms(99))


def test_arrival_process_rate():
    rng = np.random.Generator(np.random.PCG64(5))
    a = S.poisson_arrivals(20000, 50.0, rng)
    assert np.all(np.diff(a) > 0)
    assert a[-1] / 20000 == pytest.approx(1 / 50.0, rel=0.03)


def test_request_draws_are_seeded_and_in_range():
    a = _requests(50, seed=11, sides=(33, 65, 129, 257))
    b = _requests(50, seed=11, sides=(33, 65, 129, 257))
    for x, y in zip(a, b):
        assert x.params["side"] == y.params["side"]
        assert np.array_equal(x.params["centres"], y.params["centres"])
    for r in a:
        p = r.params
        assert p["side"] in (33, 65, 129, 257)
        assert 4 <= p["m"] <= 64
        assert np.all(np.abs(p["centres"]) <= 0.7) and np.all((p["radii"] >= 0.05) & (p["radii"] <= 0.2))


def test_sphere_request_phi_is_union_distance():
    rng = np.random.Generator(np.random.PCG64(2))
    p = W.sphere_request_params(rng, sides=(9,))
    X, Y, Z = W.node_coords(3, 8)
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    d = np.min(np.linalg.norm(x[:, None, :] - p["centres"][None], axis=2) - p["radii"][None], axis=1)
    phi, f = W.sample_sphere_request_numpy(p)
    assert np.allclose(phi, d, atol=1e-15)
    assert f.shape == phi.shape and np.all(np.isfinite(f))


def test_failed_solves_are_retried_once_with_fallback():
    be = FailingOnceBackend(4)
    srv = S.Server(be, slots=4, budget_bytes=1 << 40, cycles_per_step=2)
    reqs = _requests(20)
    st = S.run(srv, reqs, max_seconds=30)
    srv.close()
    assert len(st.completed) == 20 and all(r.status == 0 for r in st.completed)
    for r in st.completed:
        even = r.params["m"] % 2 == 0
        assert r.attempts == (2 if even else 1)
        assert r.cycles == (2 if even else 1) * (1 + r.params["m"] % 5)
    assert st.retried == sum(1 for r in reqs if r.params["m"] % 2 == 0)
    assert srv.used_bytes == 0
