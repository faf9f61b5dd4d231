"""GPU test of the continuous-batching server (needs an MI355X).

Requests are served through the real scheduler with fewer slots than
requests (slots are reused, problems join and leave the batch between
steps).  Every served request gives the same bits, status and cycle count as
the same problem solved alone with bcmg_solve, and matches the oracle after
the same number of cycles.
"""
import numpy as np
import pytest

import oracle
from paper_2207_14208_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_served_requests_match_solo_solves_and_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_14208_amd import _native as N
    from paper_2207_14208_amd import serving as S
    from paper_2207_14208_amd.solver import Problem

    reqs = S.make_requests(7, seed=21, rate=0.0, sides=(33, 65))
    be = S.GPUBackend(3, N.DTAU_OPT_POLY, keep_results=True)
    srv = S.Server(be, slots=3, budget_bytes=1 << 34, cycles_per_step=2)
    st = S.run(srv, reqs, max_seconds=120)
    srv.close()
    assert len(st.completed) == 7 and not st.rejected
    assert st.peak_slots <= 3
    for r in st.completed:
        p = r.params
        phi, f = W.sample_sphere_request_torch(p)
        opts = be.opts if r.attempts == 1 else be.fallback
        G = Problem(3, p["side"] - 1, phi, **opts)
        ng = G.level_info(0)["n_ghost"]
        G.set_data(f, torch.zeros(ng, dtype=torch.float64, device="cuda"))
        u = G.initial_guess()
        s, _ = G.solve(u, 1e-8)
        assert s.status == r.status, r.rid
        if r.attempts == 1:
            assert s.cycles == r.cycles, r.rid
        assert torch.equal(u, be.results[r.rid]), r.rid
    small = [r for r in st.completed if r.params["side"] == 33 and r.status == 0 and r.attempts == 1][:2]
    assert small
    for r in small:
        phi, f = W.sample_sphere_request_torch(r.params)
        O = oracle.Problem(3, 32, phi.cpu().numpy(), oracle.Options(dtau_mode=1))
        O.set_rhs(f.cpu().numpy(), np.zeros(O.counts(0)[1]))
        uo = np.zeros(33 ** 3)
        O.solve(uo, 0.0, r.cycles)
        ug = be.results[r.rid].cpu().numpy()
        assert np.abs(uo - ug).max() <= 1e-12 * np.abs(uo).max()
    be.close()


def test_served_large_requests_match_solo_solves():
    """The serving workload's large sides (129^3 and 257^3 sphere unions)
    through the scheduler with fewer slots than requests: the same bits,
    status and cycles as solo solves; one 129^3 request against the oracle
    after its cycle count."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_14208_amd import _native as N
    from paper_2207_14208_amd import serving as S
    from paper_2207_14208_amd.solver import Problem

    reqs = S.make_requests(4, seed=32, rate=0.0, sides=(129, 257))
    assert {r.params["side"] for r in reqs} == {129, 257}
    be = S.GPUBackend(2, N.DTAU_OPT_POLY, keep_results=True)
    srv = S.Server(be, slots=2, budget_bytes=1 << 36, cycles_per_step=2)
    st = S.run(srv, reqs, max_seconds=240)
    srv.close()
    assert len(st.completed) == 4 and not st.rejected
    for r in st.completed:
        p = r.params
        phi, f = W.sample_sphere_request_torch(p)
        opts = be.opts if r.attempts == 1 else be.fallback
        G = Problem(3, p["side"] - 1, phi, **opts)
        ng = G.level_info(0)["n_ghost"]
        G.set_data(f, torch.zeros(ng, dtype=torch.float64, device="cuda"))
        u = G.initial_guess()
        s, _ = G.solve(u, 1e-8)
        assert s.status == r.status, r.rid
        if r.attempts == 1:
            assert s.cycles == r.cycles, r.rid
        assert torch.equal(u, be.results[r.rid]), r.rid
        G.close()
    mid = [r for r in st.completed if r.params["side"] == 129 and r.status == 0 and r.attempts == 1][:1]
    for r in mid:
        phi, f = W.sample_sphere_request_torch(r.params)
        O = oracle.Problem(3, 128, phi.cpu().numpy(), oracle.Options(dtau_mode=1))
        O.set_rhs(f.cpu().numpy(), np.zeros(O.counts(0)[1]))
        uo = np.zeros(129 ** 3)
        O.solve(uo, 0.0, r.cycles)
        ug = be.results[r.rid].cpu().numpy()
        assert np.abs(uo - ug).max() <= 1e-12 * np.abs(uo).max()
    be.close()
