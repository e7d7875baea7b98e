"""Lattices whose population arrays hold more than 2^32 values (64-bit offsets).

A box made of four copies of a smaller box along z, each copy with the same
sphere, holds by periodicity exactly the smaller box's flow in every copy:
every node of the large box computes from the same inputs as its image in the
small one.  The small box (640 x 640 x 140, 1.09e9 values per array) runs the
sweep with 32-bit offsets, the large one (640 x 640 x 560, 4.36e9) with 64-bit
offsets, so the two agree bit for bit only if the 64-bit path indexes every
node as the 32-bit one does.  Periodic, and open in x with stress-free planes
in y (periodic z), FP32 storage, quadratic bounce-back (its links evaluated in
the sweep from the second step of a call on), body force.
"""
import numpy as np
import pytest

from paper_1906_05445_amd import workloads as W

pytestmark = pytest.mark.gpu

NX, NY, NZ = 640, 640, 140
COPIES = 4


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_05445_amd import lbm as L

    return L


def _run(lbm, nz, copies, boundary, inflow, steps):
    import torch

    solids = [W.solid("sphere", (320.3, 319.7, 70.2 + k * NZ), 20.4) for k in range(copies)]
    g = lbm.Lattice("D3Q19", "MRT", "F32", (NX, NY, nz), 0.8, g=(2e-6, 0.0, 1e-6), max_solids=copies,
                    max_links=2_000_000, max_lagrangian=1024, boundary=boundary, inflow=inflow)
    g.set_solids(solids, "QUADRATIC")
    if inflow:
        g.set_equilibrium(1.0, (inflow, 0.0, 0.0))
    g.step(steps)
    rho, u, t = g.macros()
    hist = g.history()
    g.close()
    del g
    torch.cuda.empty_cache()
    return rho, u, t, hist


@pytest.mark.timeout(600)
@pytest.mark.parametrize("boundary,inflow", [(("periodic", "periodic", "periodic"), 0.0),
                                             (("open", "slip", "periodic"), 0.03)])
def test_large_box_equals_tiled_small_box(lbm, boundary, inflow):
    assert NX * NY * NZ * 19 < 2 ** 31 and NX * NY * NZ * COPIES * 19 > 2 ** 32
    print(f"small box {NX}x{NY}x{NZ}, {boundary}", flush=True)
    rs, us, ts, hs = _run(lbm, NZ, 1, boundary, inflow, 3)
    print(f"large box {NX}x{NY}x{NZ * COPIES}", flush=True)
    rb, ub, tb, hb = _run(lbm, NZ * COPIES, COPIES, boundary, inflow, 3)
    n = NX * NY * NZ
    for k in range(COPIES):
        sl = slice(k * n, (k + 1) * n)
        assert np.array_equal(tb[sl], ts), f"copy {k}: node types"
        assert np.array_equal(rb[sl].view(np.uint64), rs.view(np.uint64)), f"copy {k}: density"
        assert np.array_equal(ub[:, sl].view(np.uint64), us.view(np.uint64)), f"copy {k}: velocity"
    # every copy's sphere feels the small box's force (summed in the same link order)
    for k in range(COPIES):
        assert np.array_equal(hb[:, k, :3].view(np.uint64), hs[:, 0, :3].view(np.uint64)), f"copy {k}: force"
    assert np.max(np.abs(us)) > 0.0
