"""Host logic of the serving loop (no GPU): admission order, percentiles, summary."""
import numpy as np

from paper_1906_05445_amd import serving as S
from paper_1906_05445_amd import workloads as W


def _req(rid, arrival, size):
    r = S.Request(rid, arrival, case=None)
    r.footprint = size
    return r


def test_first_fit_admission_does_not_block_small_requests():
    free = {"bytes": 100, "slots": 3}

    def try_admit(req):
        if req.footprint > free["bytes"] or free["slots"] == 0:
            return None
        free["bytes"] -= req.footprint
        free["slots"] -= 1
        return object()

    adm = S.Admission(try_admit)
    for rid, size in enumerate([60, 70, 30, 20, 5]):
        adm.push(_req(rid, 0.1 * rid, size))
    got = adm.admit_all(now=1.0)
    # 60 fits, 70 does not, 30 fits, 20 no longer fits (10 left), 5 takes the last slot
    assert [r.rid for r, _ in got] == [0, 2, 4]
    assert [r.rid for r in adm.queue] == [1, 3]
    assert all(r.admitted == 1.0 for r, _ in got)
    free["bytes"] += 60  # request 0 leaves: 65 bytes, one slot
    free["slots"] += 1
    got = adm.admit_all(now=2.0)
    assert [r.rid for r, _ in got] == [3]  # 70 still does not fit; the next oldest that fits goes
    assert [r.rid for r in adm.queue] == [1]


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert S.percentile(v, 50) == 50
    assert S.percentile(v, 99) == 99
    assert S.percentile(v, 100) == 100
    assert S.percentile([3.0], 99) == 3.0
    assert S.percentile([], 50) is None
    assert S.percentile([5, 1, 3], 50) == 3


def test_stats_split_queue_and_service():
    reqs = []
    for k in range(4):
        r = _req(k, float(k), 1)
        r.admitted = k + 0.5
        r.finished = k + 2.0 if k < 3 else None
        r.converged = k < 2
        r.capped = k == 2
        r.steps = 100 * (k + 1)
        reqs.append(r)
    s = S.stats(reqs, wall=10.0, cell_steps=1e9, in_flight=[reqs[3]])
    assert s["completed"] == 3 and s["converged"] == 2 and s["capped"] == 1
    assert s["solves_per_s"] == 0.3
    assert s["latency_p50_s"] == 2.0 and s["queue_p50_s"] == 0.5 and s["service_p50_s"] == 1.5
    assert s["mlups"] == 100.0
    assert s["in_flight_at_end"] == 1 and s["in_flight_mean_steps"] == 400.0


def test_request_trace_is_poisson_and_seeded():
    a = W.request_trace(count=2000, rate=50.0, seed=5)
    b = W.request_trace(count=2000, rate=50.0, seed=5)
    assert [x["arrival"] for x in a] == [x["arrival"] for x in b]
    t = np.array([x["arrival"] for x in a])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 1 / 50.0) < 0.1 / 50.0  # mean gap 1/rate within 10%
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1  # exponential: coefficient of variation 1
    methods = [x["case"].method for x in a]
    assert 0.45 < methods.count("IBM") / len(methods) < 0.55
    for x in a[:50]:
        c = x["case"]
        assert 48 <= c.shape[0] <= 160 and c.solids[0]["radius"] == c.shape[0] / 8.0


def test_link_capacity_bound_holds_for_bounce_back_spheres():
    """The link capacity a bounce-back request reserves bounds the links the
    oracle's builder finds (Sec. 2.2), over radii and sub-cell centre offsets;
    IBM requests keep the library's bounds."""
    import oracle

    rng = np.random.default_rng(11)
    for R in (2.6, 4.0, 5.5, 8.0, 11.3, 16.2):
        L = int(2 * R + 10)
        for _ in range(2):
            c = tuple(L / 2.0 + rng.random(3))
            case = W.Case("cap", "D3Q19", "MRT", (L, L, L), 0.8, (1e-6, 0.0, 0.0), [W.solid("sphere", c, R)],
                          "QUADRATIC", 0, "F32")
            max_links, max_lag = S.capacities(case)
            assert max_lag == -1
            o = oracle.Oracle("D3Q19", "MRT", (L, L, L), 0.8)
            o.set_solids(case.solids, "QUADRATIC")
            n = len(o.links()["cell"])
            assert 0 < n <= max_links, (R, n, max_links)
    ibm = W.Case("cap", "D3Q19", "MRT", (40, 40, 40), 0.8, (1e-6, 0.0, 0.0), [W.solid("sphere", (20, 20, 20), 5.0)],
                 "IBM", 0, "F32")
    assert S.capacities(ibm) == (0, 0)


def test_workspace_without_ibm_space_is_smaller():
    """max_lagrangian < 0 drops the IBM arrays (points, shell, spread force
    field): at least 3 N force values less than the default capacity."""
    import ctypes
    from paper_1906_05445_amd import lbm

    p, _ = lbm.make_params("D3Q19", "MRT", "F32", (64, 64, 64), 0.8)
    N = 64 ** 3
    full = lbm.lbm_workspace_bytes(ctypes.byref(p), 1, 0, 0)
    none = lbm.lbm_workspace_bytes(ctypes.byref(p), 1, 0, -1)
    assert 0 < none and full - none >= 3 * N * 4
    # populations stay the bulk: two arrays of 19 values per cell
    assert none > 2 * 19 * N * 4


def test_check_outcome_of_a_running_request():
    nan = float("nan")
    # (change, time, cap, tol, nsolid) -> outcome
    assert S.outcome(5e-7, 300, 1000, 1e-6, 1) == "converged"
    assert S.outcome(0.0, 300, 1000, 1e-6, 1) == "converged"
    assert S.outcome(2e-6, 300, 1000, 1e-6, 1) is None
    assert S.outcome(-1.0, 100, 1000, 1e-6, 1) is None  # not enough history yet
    assert S.outcome(2e-6, 1000, 1000, 1e-6, 1) == "capped"
    assert S.outcome(-1.0, 100, 1000, 1e-6, 0) == "capped"  # nothing to converge
    assert S.outcome(nan, 100, 1000, 1e-6, 1) == "diverged"
    assert S.outcome(nan, 1000, 1000, 1e-6, 1) == "diverged"
    assert S.outcome(float("inf"), 300, 1000, 1e-6, 1) is None  # zero to non-zero force: keep running
    st = S.stats([], 1.0)
    assert st["diverged"] == 0


def test_array_body_force_inverts_the_periodic_array_estimate():
    """The benchmark's body force for a target Re is the force under which the periodic-array
    estimate (the serving warm start) gives U = Re nu / D; a lone sphere's Stokes force is smaller,
    since the array factor K(c) and the inertia factor both exceed one."""
    nu = W.nu_of_tau(0.8)
    for Re, D, box, n in ((20.0, 32.4, 128 ** 3, 1), (10.0, 16.0, 256 ** 3, 64), (1.0, 12.0, 48 ** 3, 1)):
        Vs = np.pi / 6.0 * D ** 3
        g, U = W.array_body_force(Re, nu, D, box / n, Vs)
        assert U == Re * nu / D
        assert abs(W.periodic_array_velocity(g, nu, D, box / n, Vs) - U) <= 1e-12 * U
        g_stokes, _ = W.stokes_body_force(Re, nu, D, box, n * Vs, n_spheres=n)
        assert g > g_stokes
    case = W.sphere_pack(drive="array")
    assert abs(case.meta["U_init"] - case.meta["U_ref"]) <= 1e-12 * case.meta["U_ref"]
    assert W.sphere_box().g[0] < W.sphere_box(drive="array").g[0]
