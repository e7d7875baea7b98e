"""Serving loop on the GPU: continuous batching of a small request trace.

Bar: every served result (force/torque at the step the request finished) is
bit for bit the result of the same solve run alone with lbm_step for the same
number of steps from the same uniform start (lbm_set_equilibrium), although requests joined and left the batch at different
times; converged requests meet the drag-change criterion.
"""
import numpy as np
import pytest

from paper_1906_05445_amd import serving as S
from paper_1906_05445_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_05445_amd import lbm as L

    return L


def test_served_results_match_lone_runs(lbm):
    trace = W.request_trace(count=7, rate=200.0, seed=7, edge=(24, 36), Re=(1.0, 2.0))
    reqs = S.requests_from_trace(trace, n_iter=3)
    fps = [S.footprint(lbm, r.case) for r in reqs]
    # room for about three of them at once, and at most four slots: the rest queue
    pool = lbm.lbm_batch_table_bytes(4) + int(3.2 * max(fps))
    srv = S.Server(pool_bytes=pool, max_slots=4, check_every=100, tol=1e-6, step_cap=4000)
    st = srv.run(reqs, wall_limit=240)
    srv.close()
    assert st["completed"] == len(reqs), st
    assert st["rejected"] == 0
    assert any(r.queue_time > 0 for r in reqs if r.admitted is not None)
    for r in reqs:
        assert r.steps % 100 == 0 and 0 < r.steps <= 4000
        if r.converged:
            assert 0.0 <= r.change < 1e-6
        c = r.case
        lone = lbm.Lattice(c.lattice, c.collision, c.storage, c.shape, c.tau, g=c.g, max_solids=1)
        lone.set_solids(c.solids, c.method, n_iter=3)
        u0 = S.initial_velocity(c)  # the server's warm start
        if u0 is not None:
            lone.set_equilibrium(1.0, u0)
        lone.step(r.steps)
        ft = lone.force_torque()
        lone.close()
        assert np.array_equal(ft.view(np.uint64), r.force.view(np.uint64)), f"request {r.rid}"


def test_diverging_request_ends_without_disturbing_the_others(lbm):
    """A request whose flow blows up (tau just above 1/2, a body force of 0.05 per
    step: the oracle grows by about 1e41 every 25 steps) ends as diverged at the
    first check that has a force change (step 200: the change over 100 steps
    needs 101 steps of history); the requests served beside it match their lone
    runs bit for bit."""
    import dataclasses

    trace = W.request_trace(count=3, rate=200.0, seed=7, edge=(24, 36), Re=(1.0, 2.0))
    reqs = S.requests_from_trace(trace, n_iter=3)
    bad = dataclasses.replace(reqs[0].case, name="blowup", tau=0.5001, g=(0.05, 0.0, 0.0), method="QUADRATIC",
                              meta={})
    reqs.insert(1, S.Request(99, reqs[0].arrival, bad, n_iter=3))
    srv = S.Server(pool_bytes=1 << 30, max_slots=4, check_every=100, tol=1e-6, step_cap=4000)
    st = srv.run(reqs, wall_limit=240)
    srv.close()
    assert st["completed"] == len(reqs) and st["diverged"] == 1, st
    assert reqs[1].diverged and reqs[1].steps == 200
    for r in reqs:
        if r.rid == 99:
            continue
        assert not r.diverged
        c = r.case
        lone = lbm.Lattice(c.lattice, c.collision, c.storage, c.shape, c.tau, g=c.g, max_solids=1)
        lone.set_solids(c.solids, c.method, n_iter=3)
        u0 = S.initial_velocity(c)
        if u0 is not None:
            lone.set_equilibrium(1.0, u0)
        lone.step(r.steps)
        ft = lone.force_torque()
        lone.close()
        assert np.array_equal(ft.view(np.uint64), r.force.view(np.uint64)), f"request {r.rid}"
