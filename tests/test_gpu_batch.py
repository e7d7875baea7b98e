"""Batched stepping (lbm_batch_*) through the C ABI.

Bar: a member of a batch computes bit for bit what the same context computes
stepped alone with lbm_step -- same populations, same per-step force/torque
history, same macroscopic fields, same links -- whatever else is in the batch,
whenever it was admitted, and whether its steps ran eagerly (sweep tuning),
from the one-step graph or from the multi-step graph.  One member is also
compared with the FP64 oracle directly (1e-12, as for single contexts).
"""
import numpy as np
import pytest

from paper_1906_05445_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_05445_amd import lbm as L

    return L


# (collision, shape, tau, g, solids, method, rates) of a mixed set of members
def _specs():
    return [
        ("MRT", (40, 36, 33), 0.8, (0.0, 0.0, 0.0),
         [W.solid("sphere", (18.2, 17.1, 15.4), 6.3, velocity=(0.018, -0.011, 0.007))], "QUADRATIC", None),
        ("MRT", (32, 32, 32), 0.7, (2e-6, 0.0, 0.0), [W.solid("sphere", (16.3, 15.8, 16.1), 5.1)], "QUADRATIC",
         None),
        ("MRT", (35, 30, 29), 0.9, (1e-6, 5e-7, 0.0), [W.solid("sphere", (17.1, 14.6, 14.2), 5.6)], "IBM", None),
        ("BGK", (27, 25, 23), 0.75, (1e-6, 0.0, 0.0),
         [W.solid("sphere", (13.4, 12.2, 11.9), 4.2, velocity=(-0.012, 0.009, 0.015))], "LINEAR", None),
        ("MRT", (26, 24, 22), 0.85, (1e-6, 0.0, 0.0), [], "QUADRATIC", None),
        ("MRT", (30, 28, 26), 0.8, (1.5e-6, 0.0, 0.0), [W.solid("sphere", (15.2, 13.9, 12.8), 4.9)], "QUADRATIC",
         np.array([0, 1.2, 1.4, 0, 1.1, 0, 1.1, 0, 1.1, 1.25, 1.3, 1.25, 1.3, 1.25, 1.25, 1.25, 1.5, 1.5, 1.5])),
        ("MRT", (34, 31, 28), 0.8, (0.0, 0.0, 0.0),
         [W.solid("sphere", (16.1, 15.3, 13.6), 5.8, velocity=(-0.015, 0.012, -0.009))], "ZHAO_YONG", None),
        ("MRT", (29, 33, 27), 0.75, (1e-6, 0.0, 5e-7), [W.solid("sphere", (14.3, 16.2, 13.1), 5.4)], "YU", None),
        # fixed: alone, the sweep evaluates these links; in the batch, the bounce-back kernel
        ("BGK", (31, 27, 30), 0.85, (2e-6, -1e-6, 0.0), [W.solid("sphere", (15.4, 13.2, 14.7), 5.9)], "ZHAO_YONG",
         None),
        # two translating spheres whose boxes overlap (the two classification phases run apart)
        ("MRT", (44, 30, 28), 0.8, (1e-6, 0.0, 0.0),
         [W.solid("sphere", (14.6, 15.2, 13.7), 4.6, velocity=(0.014, 0.006, -0.004)),
          W.solid("sphere", (27.9, 14.1, 14.3), 4.3, velocity=(-0.011, 0.008, 0.005))], "QUADRATIC", None),
    ]


def _configure(ctx, spec):
    _, shape, _, _, solids, method, _ = spec
    if solids:
        ctx.set_solids(solids, method, n_iter=3 if method == "IBM" else 5)


def _alone(lbm, storage, spec, steps_list):
    coll, shape, tau, g, solids, method, rates = spec
    ctx = lbm.Lattice("D3Q19", coll, storage, shape, tau, rates=rates, g=g, max_solids=max(1, len(solids)))
    _configure(ctx, spec)
    for n in steps_list:
        ctx.step(n)
    return ctx


def _same(a, b, what):
    assert a.shape == b.shape, what
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"{what} differs"


def _compare(member, ref, tag):
    assert member.time == ref.time
    _same(member.get_state(), ref.get_state(), f"{tag}: state")
    if member.nsolid:
        _same(member.history(), ref.history(), f"{tag}: force history")
    rb, ub, tb = member.macros()
    ra, ua, ta = ref.macros()
    _same(rb, ra, f"{tag}: rho")
    _same(ub, ua, f"{tag}: u")
    _same(tb, ta, f"{tag}: node types")
    if member.nsolid:
        lb, la = member.links(), ref.links()
        for k in ("cell", "dir", "sid", "q"):
            _same(np.asarray(lb[k]), np.asarray(la[k]), f"{tag}: links {k}")


@pytest.mark.parametrize("storage", ["F32", "F64"])
def test_batch_members_match_alone(lbm, storage):
    """Mixed members (translating and fixed spheres, IBB and IBM, BGK / two-rate /
    general-rate MRT, no solid), 45 steps in uneven calls with readouts between
    them: tuning steps, then graph replays (one-step and eight-step graphs)."""
    specs = _specs()
    calls = [1, 10, 3, 17, 8, 6]
    b = lbm.Batch("D3Q19", storage, max_slots=12, pool_bytes=1 << 30)
    members = []
    for spec in specs:
        coll, shape, tau, g, solids, _, rates = spec
        m = b.admit(coll, storage, shape, tau, rates=rates, g=g, max_solids=max(1, len(solids)))
        assert m is not None
        _configure(m, spec)
        members.append(m)
    done = 0
    for n in calls:
        b.step(n)
        done += n
        # eager readouts between replays
        for m in members:
            if m.nsolid:
                ft = m.force_torque()
                assert np.all(np.isfinite(ft))
    assert b.tune_info() is not None
    for k, (m, spec) in enumerate(zip(members, specs)):
        ref = _alone(lbm, storage, spec, [done])
        _compare(m, ref, f"member {k}")
        ref.close()
    b.close()


def test_batch_admission_release_and_late_member(lbm):
    """Admission by footprint: LBM_EAGAIN when the pool is full, room again after
    a release; a member admitted while others are mid-run matches its lone run."""
    specs = _specs()
    fp = [lbm.Batch.footprint("D3Q19", s[0], "F32", s[1], s[2], max_solids=max(1, len(s[4]))) for s in specs]
    table = lbm.lbm_batch_table_bytes(8)
    pool = table + fp[0] + fp[1] + fp[2] // 2 + 4096
    b = lbm.Batch("D3Q19", "F32", max_slots=8, pool_bytes=pool)
    m0 = b.admit(specs[0][0], "F32", specs[0][1], specs[0][2], g=specs[0][3], max_solids=1)
    m1 = b.admit(specs[1][0], "F32", specs[1][1], specs[1][2], g=specs[1][3], max_solids=1)
    assert m0 is not None and m1 is not None
    assert b.admit(specs[2][0], "F32", specs[2][1], specs[2][2], g=specs[2][3], max_solids=1) is None
    _configure(m0, specs[0])
    _configure(m1, specs[1])
    b.step(30)
    b.release(m1)
    info = b.info()
    assert info["members"] == 1 and info["largest_free"] >= fp[1]
    m3 = b.admit(specs[3][0], "F32", specs[3][1], specs[3][2], g=specs[3][3], max_solids=1)
    assert m3 is not None
    _configure(m3, specs[3])
    b.step(21)
    b.step(4)
    ref0 = _alone(lbm, "F32", specs[0], [55])
    _compare(m0, ref0, "first member")
    ref3 = _alone(lbm, "F32", specs[3], [25])
    _compare(m3, ref3, "late member")
    # a member may also be stepped alone in between; the batch picks up its new time
    m3.step(3)
    b.step(5)
    ref3.step(8)
    _compare(m3, ref3, "late member after a lone step")
    ref0.step(5)
    _compare(m0, ref0, "first member after the lone step of another")
    b.close()


@pytest.mark.parametrize("method", ["QUADRATIC", "ZHAO_YONG"])
def test_batch_member_matches_oracle_fp64(lbm, method):
    """FP64 batch: a translating sphere member against the FP64 oracle (1e-12)."""
    from oracle import Oracle

    shape = (30, 27, 25)
    solids = [W.solid("sphere", (14.2, 13.1, 12.4), 5.3, velocity=(0.07, -0.045, 0.03))]
    b = lbm.Batch("D3Q19", "F64", max_slots=4, pool_bytes=1 << 28)
    other = b.admit("MRT", "F64", (28, 26, 24), 0.8, g=(1e-6, 0.0, 0.0), max_solids=1)
    other.set_solids([W.solid("sphere", (14.0, 13.0, 12.0), 4.5)], "QUADRATIC")
    m = b.admit("MRT", "F64", shape, 0.8, max_solids=1)
    m.set_solids(solids, method)
    orc = Oracle("D3Q19", "MRT", shape, 0.8, form="h")
    orc.set_solids(solids, method)
    for n in (13, 20, 27):
        b.step(n)
        orc.step(n)
    fg, fo = m.get_f(), orc.get_f()
    fl = m.node_types() != 1
    assert np.max(np.abs(fg[:, fl] - fo[:, fl])) <= 1e-13
    hg, ho = m.history(), orc.history()
    scale = max(np.max(np.abs(ho[-1, :, :3])), 1e-300)
    assert np.max(np.abs(hg[:, :, :3] - ho[:, :, :3])) / scale <= 1e-12
    Lg, Lo = m.links(), orc.links()
    for k in ("cell", "dir", "sid"):
        assert np.array_equal(Lg[k], Lo[k]), k
    assert np.array_equal(Lg["q"].view(np.uint64), Lo["q"].view(np.uint64))
    b.close()


def test_batch_rejects_mismatched_members(lbm):
    b = lbm.Batch("D3Q19", "F32", max_slots=2, pool_bytes=1 << 26)
    with pytest.raises(lbm.LBMError):
        b.admit("MRT", "F64", (16, 16, 16), 0.8)
    a = b.admit("MRT", "F32", (16, 16, 16), 0.8)
    c = b.admit("MRT", "F32", (16, 16, 16), 0.8)
    assert a is not None and c is not None
    assert b.admit("MRT", "F32", (16, 16, 16), 0.8) is None  # every slot taken
    # a member cannot be destroyed behind the batch's back
    assert lbm.lbm_destroy(a.handle) == lbm.LBM_ESTATE
    b.step(3)
    assert a.time == 3 and c.time == 3
    b.close()


@pytest.mark.parametrize("storage", ["F16", "F16_SR", "F64"])
def test_batch_d2q9_members_match_alone(lbm, storage):
    """D2Q9 members (translating and fixed cylinders, IBM circle, BGK and MRT) match their lone runs."""
    specs = [
        ("BGK", (61, 47, 1), 0.8, (1e-6, 0.0, 0.0),
         [W.solid("cylinder", (30.4, 23.7, 0.0), 7.3, velocity=(0.013, -0.008, 0.0))], "LINEAR"),
        ("MRT", (64, 64, 1), 0.7, (1e-6, 0.0, 0.0), [W.solid("cylinder", (32.4, 31.7, 0.0), 8.3)], "QUADRATIC"),
        ("MRT", (50, 44, 1), 0.9, (2e-6, 0.0, 0.0), [W.solid("cylinder", (25.2, 21.9, 0.0), 6.1)], "IBM"),
    ]
    b = lbm.Batch("D2Q9", storage, max_slots=4, pool_bytes=1 << 27)
    members = []
    for coll, shape, tau, g, solids, method in specs:
        m = b.admit(coll, storage, shape, tau, g=g, max_solids=1)
        m.set_solids(solids, method, n_iter=3)
        members.append(m)
    for n in (7, 40, 13):
        b.step(n)
    for k, ((coll, shape, tau, g, solids, method), m) in enumerate(zip(specs, members)):
        ref = lbm.Lattice("D2Q9", coll, storage, shape, tau, g=g, max_solids=1)
        ref.set_solids(solids, method, n_iter=3)
        ref.step(60)
        _compare(m, ref, f"D2Q9 member {k}")
        ref.close()
    b.close()


def test_batch_ibm_delta_members_match_alone(lbm):
    """IBM members with the 3- and 2-point deltas (Sec. 3.1) next to a 4-point one."""
    specs = [((29, 27, 25), [W.solid("sphere", (14.2, 13.4, 12.1), 5.1)], 3, 0.3),
             ((31, 26, 24), [W.solid("sphere", (15.3, 12.6, 11.8), 4.8)], 2, 0.2),
             ((27, 27, 27), [W.solid("sphere", (13.6, 13.1, 13.9), 5.3)], 4, 0.0)]
    b = lbm.Batch("D3Q19", "F32", max_slots=4, pool_bytes=1 << 28)
    members = []
    for shape, solids, delta, rd in specs:
        m = b.admit("MRT", "F32", shape, 0.8, g=(2e-6, 0.0, 0.0), max_solids=1)
        m.set_solids(solids, "IBM", n_iter=3, delta=delta, retraction=rd)
        members.append(m)
    for n in (5, 12, 9):
        b.step(n)
    for k, ((shape, solids, delta, rd), m) in enumerate(zip(specs, members)):
        ref = lbm.Lattice("D3Q19", "MRT", "F32", shape, 0.8, g=(2e-6, 0.0, 0.0), max_solids=1)
        ref.set_solids(solids, "IBM", n_iter=3, delta=delta, retraction=rd)
        ref.step(26)
        _compare(m, ref, f"IBM member {k} ({delta}-point delta)")
        ref.close()
    b.close()


def test_batch_member_with_non_finite_state_is_isolated(lbm):
    """A member whose populations take a NaN mid-run: the batch steps on, the other
    members match their lone runs bit for bit, the member's own check reports the
    divergence and its force change is NaN (the serving loop ends such a request),
    and after its release the batch goes on as before."""
    specs = [_specs()[1], _specs()[0], _specs()[4]]  # fixed sphere (takes the NaN), translating sphere, no solid
    b = lbm.Batch("D3Q19", "F32", max_slots=4, pool_bytes=1 << 28)
    ms = []
    for spec in specs:
        coll, shape, tau, g, solids, _, rates = spec
        m = b.admit(coll, "F32", shape, tau, rates=rates, g=g, max_solids=max(1, len(solids)))
        _configure(m, spec)
        ms.append(m)
    b.step(6)
    h = ms[0].get_state().copy()
    h[3, 1234] = np.nan
    ms[0].set_state(h)
    b.step(30)
    assert not ms[0].check()
    assert ms[1].check() and ms[2].check()
    ch = b.force_change(10)
    assert np.isnan(ch[ms[0]])
    assert np.isfinite(ch[ms[1]]) and ch[ms[1]] >= 0.0
    assert ms[0] not in b.poll(10, tol=1e30)
    refs = [_alone(lbm, "F32", specs[k], [36]) for k in (1, 2)]
    for k, ref in zip((1, 2), refs):
        _compare(ms[k], ref, f"member {k} beside a diverged one")
    b.release(ms[0])
    b.step(4)
    for k, ref in zip((1, 2), refs):
        ref.step(4)
        _compare(ms[k], ref, f"member {k} after the diverged one left")
        ref.close()
    b.close()
