"""Edge cases through the C ABI.

* Invalid arguments give the documented status (LBM_EINVAL, LBM_EUNSUPPORTED) and leave the context
  usable; too many boundary links for the capacity gives LBM_ENOMEM; readouts out of range give
  LBM_EINVAL.
* Empty and degenerate inputs against the FP64 oracle: no solids, zero steps, periodic boxes one cell
  thick or of a single cell (every neighbour is the cell itself), at the FP64 parity bars.
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


def _oracle(*a, **k):
    from oracle import Oracle

    k.setdefault("form", "h")
    return Oracle(*a, **k)


def test_invalid_lattice_parameters(lbm):
    for shape, tau in (((8, 8, 8), 0.5), ((0, 8, 8), 0.8), ((8, 8, -1), 0.8)):
        with pytest.raises(lbm.LBMError) as e:
            lbm.Lattice("D3Q19", "MRT", "F64", shape, tau)
        assert e.value.status == lbm.LBM_EINVAL


@pytest.mark.parametrize("solids,method,status", [
    ([W.solid("sphere", (8.1, 7.9, 8.2), 0.0)], "QUADRATIC", "EINVAL"),             # radius
    ([W.solid("sphere", (8.1, 7.9, 8.2), 8.5)], "QUADRATIC", "EINVAL"),             # wider than the box
    ([W.solid("sphere", (18.0, 7.9, 8.2), 3.0)], "QUADRATIC", "EINVAL"),            # centre outside
    ([W.solid("sphere", (8.1, 7.9, 8.2), 3.0, velocity=(1.2, 0.0, 0.0))], "QUADRATIC", "EINVAL"),  # speed
    ([W.solid("sphere", (8.1, 7.9, 8.2), 3.0, inverted=True, velocity=(0.1, 0.0, 0.0))], "IBM",
     "EUNSUPPORTED"),                                                                # moving inverted IBM
    ([W.solid("plane", (0.0, 4.3, 0.0), axis=(0, 1, 0), velocity=(0.01, 0.0, 0.0))], "QUADRATIC",
     "EUNSUPPORTED"),
    ([W.solid("sphere", (8.1, 7.9, 8.2), 3.0, density=-1.0)], "QUADRATIC", "EINVAL"),
])
def test_invalid_solids(lbm, solids, method, status):
    g = lbm.Lattice("D3Q19", "MRT", "F64", (16, 16, 16), 0.8)
    with pytest.raises(lbm.LBMError) as e:
        g.set_solids(solids, method)
    assert e.value.status == getattr(lbm, "LBM_" + status)
    # the context stays usable
    g.set_solids([W.solid("sphere", (8.1, 7.9, 8.2), 3.0)], "QUADRATIC")
    g.step(3)
    assert g.check()
    g.close()


def test_link_capacity_overflow(lbm):
    g = lbm.Lattice("D3Q19", "MRT", "F64", (24, 24, 24), 0.8, max_links=200)
    with pytest.raises(lbm.LBMError) as e:
        g.set_solids([W.solid("sphere", (12.2, 11.8, 12.1), 6.0)], "QUADRATIC")
    assert e.value.status == lbm.LBM_ENOMEM
    g.close()


def test_history_and_readout_bounds(lbm):
    g = lbm.Lattice("D3Q19", "MRT", "F64", (16, 16, 16), 0.8, g=(1e-6, 0.0, 0.0))
    g.set_solids([W.solid("sphere", (8.1, 7.9, 8.2), 3.0)], "QUADRATIC")
    g.step(5)
    assert g.history(0, 5).shape == (5, 1, 6)
    for first, count in ((3, 5), (-1, 2), (6, 1)):
        with pytest.raises(lbm.LBMError) as e:
            g.history(first, count)
        assert e.value.status == lbm.LBM_EINVAL
    g.close()


def test_no_solids_and_zero_steps(lbm):
    shape, g = (13, 11, 9), (1e-6, 2e-6, -5e-7)
    gpu = lbm.Lattice("D3Q19", "MRT", "F64", shape, 0.8, g=g)
    gpu.set_solids([], "QUADRATIC")
    orc = _oracle("D3Q19", "MRT", shape, 0.8, g=g)
    orc.set_solids([], "QUADRATIC")
    f0 = gpu.get_f()
    gpu.step(0)
    assert gpu.time == 0 and np.array_equal(gpu.get_f(), f0)
    gpu.step(17)
    orc.step(17)
    rg, ug, _ = gpu.macros()
    ro, uo, _ = orc.macros()
    assert np.max(np.abs(ug - uo)) <= 1e-12 * np.max(np.abs(uo))
    assert np.max(np.abs(rg - ro)) <= 1e-12
    assert np.max(np.abs(gpu.get_f() - orc.get_f())) <= 1e-13
    gpu.close()


@pytest.mark.parametrize("lat,shape", [("D3Q19", (1, 1, 1)), ("D3Q19", (3, 1, 2)), ("D2Q9", (1, 5, 1)),
                                       ("D2Q9", (2, 2, 1))])
def test_degenerate_periodic_boxes(lbm, lat, shape):
    """Every pull wraps onto the cell itself or its one neighbour; general-rate MRT, body force."""
    Q = 9 if lat == "D2Q9" else 19
    rng = np.random.default_rng(61)
    rates = rng.uniform(0.7, 1.6, size=Q)
    g = (2e-6, -1e-6, 5e-7 if lat == "D3Q19" else 0.0)
    gpu = lbm.Lattice(lat, "MRT", "F64", shape, 0.8, rates=rates, g=g)
    orc = _oracle(lat, "MRT", shape, 0.8, rates=rates, g=g)
    _, w, _ = orc.lattice_tables()
    f0 = w[:, None] * (1.0 + 0.05 * rng.standard_normal((Q, orc.N)))
    gpu.set_f(f0)
    orc.set_f(f0)
    gpu.step(12)
    orc.step(12)
    assert np.max(np.abs(gpu.get_f() - orc.get_f())) <= 1e-13
    rg, ug, _ = gpu.macros()
    ro, uo, _ = orc.macros()
    assert np.max(np.abs(ug - uo)) <= 1e-12 * max(np.max(np.abs(uo)), 1e-300)
    assert np.max(np.abs(rg - ro)) <= 1e-12
    gpu.close()


def test_rejected_set_solids_leaves_the_context_unchanged(lbm):
    """An IBM set-up, then a call rejected on its options (a moving sphere with a 5-point delta): the
    context steps on bit for bit as one that never saw the rejected call."""
    shape, g = (26, 22, 20), (2e-6, 0.0, 0.0)
    fixed = [W.solid("sphere", (12.3, 10.6, 9.2), 4.7)]
    # body force on every node: a moving IBM sphere is allowed, so the 5-point delta is what is rejected
    a = lbm.Lattice("D3Q19", "MRT", "F64", shape, 0.8, g=g, g_fluid_only=False, max_lagrangian=600)
    b = lbm.Lattice("D3Q19", "MRT", "F64", shape, 0.8, g=g, g_fluid_only=False, max_lagrangian=600)
    for c in (a, b):
        c.set_solids(fixed, "IBM", n_iter=3)
        c.step(5)
    with pytest.raises(lbm.LBMError) as e:
        a.set_solids([W.solid("sphere", (12.3, 10.6, 9.2), 4.7, velocity=(0.01, 0.0, 0.0))], "IBM", delta=5)
    assert e.value.status == lbm.LBM_EINVAL
    a.step(10)
    b.step(10)
    assert np.array_equal(a.get_state().view(np.uint64), b.get_state().view(np.uint64))
    assert np.array_equal(a.history().view(np.uint64), b.history().view(np.uint64))
    a.close()
    b.close()


def test_failed_set_solids_leaves_a_plain_lattice(lbm):
    """A set-up that fails late (more links than max_links): the context has no solids, and steps as a
    lattice that never had any."""
    shape, g = (24, 24, 24), (1e-6, 0.0, 0.0)
    a = lbm.Lattice("D3Q19", "MRT", "F64", shape, 0.8, g=g, max_links=200)
    b = lbm.Lattice("D3Q19", "MRT", "F64", shape, 0.8, g=g, max_links=200)
    with pytest.raises(lbm.LBMError) as e:
        a.set_solids([W.solid("sphere", (12.2, 11.8, 12.1), 6.0)], "QUADRATIC")
    assert e.value.status == lbm.LBM_ENOMEM
    a.step(12)
    b.step(12)
    assert np.array_equal(a.get_state().view(np.uint64), b.get_state().view(np.uint64))
    assert np.all(a.node_types() != 1)
    a.close()
    b.close()


def test_context_without_ibm_space(lbm):
    """max_lagrangian < 0 reserves no IBM space: bounce-back solids step bit for bit as in a
    context with the default capacities, and an IBM set-up is refused (LBM_ENOMEM) without
    touching the context."""
    shape, g = (28, 26, 24), (1e-6, 0.0, 0.0)
    s = [W.solid("sphere", (13.6, 12.2, 11.9), 5.1)]
    a = lbm.Lattice("D3Q19", "MRT", "F32", shape, 0.8, g=g, max_lagrangian=-1)
    b = lbm.Lattice("D3Q19", "MRT", "F32", shape, 0.8, g=g)
    assert a.workspace.numel() < b.workspace.numel()
    with pytest.raises(lbm.LBMError) as e:
        a.set_solids(s, "IBM")
    assert e.value.status == lbm.LBM_ENOMEM
    for c in (a, b):
        c.set_solids(s, "QUADRATIC")
        c.step(40)
    assert np.array_equal(a.get_state().view(np.uint32), b.get_state().view(np.uint32))
    assert np.array_equal(a.history().view(np.uint64), b.history().view(np.uint64))
    a.close()
    b.close()
