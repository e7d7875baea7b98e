"""Moving IBM solids on the GPU against the FP64 oracle, through the C ABI: a prescribed
translation, and free motion by Feng & Michaelides's discretisation (Eq. 23) under the IBM force
and torque of each step.

The solids cross several cell faces during each run, so the shell of stencil cells is shifted
(and the force of the old cells cleared) more than once.  Density ratios are chosen where the
explicit Eq. 23 update is stable at these small radii: with R = 4 and rho_p = 1.5 the rotation of
a sphere oscillates with growing amplitude (the diffuse IBM shell adds inertia beyond the solid's
volume that the inner-fluid term does not hold), while R = 7, or rho_p = 3 at R = 4, is stable.  The oracle
runs in its deviation form (pinned against the literal one in tests/test_oracle_forms.py).  Bars: FP64
storage, populations max|df| <= 1e-13 and velocities max|du| / max|u| <= 1e-12 over all cells (measured
about 1e-15), force and torque relative to their scale <= 1e-12 (torque scale: the larger of max|T| and the force scale
times the box edge, as a solid that does not spin has a torque of rounding size), solid centre, velocity and angular velocity <= 1e-12 (absolute;
centres of order 10, velocities of order 1e-2); FP32 storage, the bounds stated in the test.
"""
import math

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


def _run_pair(lbm, lat, shape, solid, steps, storage="F64", g=(0.0, 0.0, 0.0), fluid_only=False, n_iter=5,
              delta=4, tau=0.8, chunks=(1,)):
    from oracle import Oracle

    gpu = lbm.Lattice(lat, "MRT", storage, shape, tau, g=g, g_fluid_only=fluid_only)
    orc = Oracle(lat, "MRT", shape, tau, g=g, g_fluid_only=fluid_only, form="h")
    gpu.set_solids([solid], "IBM", n_iter=n_iter, delta=delta)
    orc.set_solids([solid], "IBM")
    orc.set_ibm_iters(n_iter)
    orc.set_ibm_delta(delta)
    X, dV = W.lagrangian_mesh(solid, lat, shape)
    gpu.set_lagrangian(0, X, dV)
    orc.set_lagrangian(0, X, dV)
    done, i = 0, 0
    while done < steps:  # lbm_step calls of varying length
        n = min(chunks[i % len(chunks)], steps - done)
        gpu.step(n)
        done += n
        i += 1
    orc.step(steps)
    return gpu, orc


def _compare(gpu, orc, tol_f=1e-13, tol_u=1e-12, tol_F=1e-12, tol_s=1e-12):
    df = np.max(np.abs(gpu.get_f() - orc.get_f()))
    _, ug, _ = gpu.macros()
    _, uo, _ = orc.macros()
    du = np.max(np.abs(ug - uo)) / max(np.max(np.abs(uo)), 1e-300)
    hg, ho = gpu.history(), orc.history()
    assert hg.shape == ho.shape
    scale = max(np.max(np.abs(ho[:, :, :3])), 1e-300)
    dF = np.max(np.abs(hg[:, :, :3] - ho[:, :, :3])) / scale
    tscale = max(np.max(np.abs(ho[:, :, 3:])), scale * max(gpu.shape), 1e-300)  # torque ~ force x lever
    dT = np.max(np.abs(hg[:, :, 3:] - ho[:, :, 3:])) / tscale
    sg, so = gpu.solid_state(), orc.solid_state()
    ds = np.max(np.abs(sg - so))
    print(f"df {df:.2e} du {du:.2e} dF {dF:.2e} dT {dT:.2e} dstate {ds:.2e}", flush=True)
    if tol_f is not None:
        assert df <= tol_f, f"population mismatch {df:.3e}"
    assert du <= tol_u, f"velocity mismatch {du:.3e}"
    assert dF <= tol_F, f"force mismatch {dF:.3e}"
    assert dT <= tol_F, f"torque mismatch {dT:.3e}"
    assert ds <= tol_s, f"solid state mismatch {ds:.3e}"
    return so


@pytest.mark.parametrize("lat,shape,solid,steps", [
    ("D2Q9", (47, 38, 1), W.solid("cylinder", (20.3, 18.6, 0.0), 5.2, velocity=(0.04, -0.03, 0.0),
                                  omega=(0.0, 0.0, 0.003)), 90),
    ("D3Q19", (26, 23, 21), W.solid("sphere", (12.4, 11.3, 10.2), 4.3, velocity=(0.03, -0.02, 0.025),
                                    omega=(0.001, -0.002, 0.0015)), 70),
])
def test_translating_ibm_against_oracle(lbm, lat, shape, solid, steps):
    gpu, orc = _run_pair(lbm, lat, shape, solid, steps, chunks=(1, 7, 30))
    st = _compare(gpu, orc)
    moved = np.abs(st[0, :3] - np.array(solid["centre"]))
    assert np.max(moved) > 2.0  # several whole-cell shifts of the shell


@pytest.mark.parametrize("lat,shape,solid,g,steps", [
    ("D2Q9", (44, 52, 1), W.solid("cylinder", (21.7, 30.4, 0.0), 5.0, velocity=(0.01, 0.0, 0.0),
                                  omega=(0.0, 0.0, 0.002), density=1.5, gravity=(0.0, -2e-4, 0.0)),
     (0.0, 0.0, 0.0), 600),
    ("D3Q19", (24, 26, 30), W.solid("sphere", (11.6, 12.7, 18.4), 4.0, velocity=(0.0, 0.005, 0.0),
                                    omega=(0.0, 0.0, 0.001), density=3.0, gravity=(0.0, 0.0, -3e-4)),
     (0.0, 0.0, 2e-6), 300),
])
def test_free_ibm_against_oracle(lbm, lat, shape, solid, g, steps):
    gpu, orc = _run_pair(lbm, lat, shape, solid, steps, g=g, chunks=(3, 40))
    st = _compare(gpu, orc)
    moved = st[0, :3] - np.array(solid["centre"])
    assert np.any(np.floor(moved) != 0.0)  # the whole-cell shift of the shell changed


@pytest.mark.parametrize("delta", [3, 2])
def test_free_ibm_narrow_deltas(lbm, delta):
    s = W.solid("cylinder", (20.2, 24.6, 0.0), 4.6, density=1.3, gravity=(1e-4, -2e-4, 0.0))
    gpu, orc = _run_pair(lbm, "D2Q9", (40, 48, 1), s, 120, delta=delta, chunks=(120,))
    _compare(gpu, orc)


def test_free_ibm_fp32(lbm):
    """FP32 deviation storage against the FP64 oracle: velocities within 2e-5 of max|u|, force and
    torque within 1e-3 of their scale (the drag of a settling solid is a small difference of large
    Lagrangian forces), solid state within 1e-6 absolute."""
    s = W.solid("sphere", (14.6, 15.3, 20.8), 6.0, density=2.0, gravity=(0.0, 0.0, -3e-4))
    gpu, orc = _run_pair(lbm, "D3Q19", (30, 31, 36), s, 100, storage="F32", chunks=(100,))
    _compare(gpu, orc, tol_f=None, tol_u=2e-5, tol_F=1e-3, tol_s=1e-6)


def test_moving_ibm_rules(lbm):
    g = lbm.Lattice("D3Q19", "MRT", "F64", (20, 20, 20), 0.8, g=(1e-6, 0.0, 0.0), g_fluid_only=True)
    s = W.solid("sphere", (9.6, 10.1, 9.8), 3.0, velocity=(0.02, 0.0, 0.0))
    with pytest.raises(lbm.LBMError) as e:  # a fluid-only body force would follow the moving solid
        g.set_solids([s], "IBM")
    assert e.value.status == lbm.LBM_EUNSUPPORTED
    g.close()
    g = lbm.Lattice("D3Q19", "MRT", "F64", (20, 20, 20), 0.8)
    g.set_solids([s], "IBM")
    g.step(2)
    X, dV = W.icosphere(s["centre"], 3.0)
    with pytest.raises(lbm.LBMError) as e:  # points are placed before the solid moves
        g.set_lagrangian(0, X, dV)
    assert e.value.status == lbm.LBM_EINVAL
    # a fixed IBM solid after a moving one: the shell cells of the moving one are cleared
    g.set_solids([W.solid("sphere", (9.6, 10.1, 9.8), 3.0)], "IBM")
    g.step(3)
    assert g.check()
    g.close()


def test_free_ibm_fp16(lbm):
    """FP16 deviation storage against the FP64 oracle, with the FP16 bars of the fixed-solid parity tests:
    velocities within 2e-2 of max|u|, force and torque within 5e-2 of their scale; solid state within 1e-4
    absolute (velocities of order 5e-3, centres of order 20)."""
    s = W.solid("sphere", (14.6, 15.3, 20.8), 6.0, density=2.0, gravity=(0.0, 0.0, -3e-4))
    gpu, orc = _run_pair(lbm, "D3Q19", (30, 31, 36), s, 100, storage="F16", chunks=(100,))
    _compare(gpu, orc, tol_f=None, tol_u=2e-2, tol_F=5e-2, tol_s=1e-4)


def test_free_ibm_without_points(lbm):
    """A free IBM solid with no Lagrangian points feels no fluid force: its motion is the Eq. 23 recurrence
    alone (whose closed form pins the oracle), and the fluid stays at rest."""
    from oracle import Oracle

    s = W.solid("sphere", (12.3, 11.8, 12.6), 4.0, velocity=(0.01, 0.0, -0.004), omega=(0.0, 2e-4, 1e-4),
                density=1.6, gravity=(1e-5, -2e-5, 4e-6))
    gpu = lbm.Lattice("D3Q19", "MRT", "F64", (24, 24, 24), 0.8)
    orc = Oracle("D3Q19", "MRT", (24, 24, 24), 0.8, form="h")
    gpu.set_solids([s], "IBM")
    gpu.set_lagrangian(0, np.zeros((0, 3)), 1.0)
    orc.set_solids([s], "IBM")
    for n in (1, 12, 27):
        gpu.step(n)
    orc.step(40)
    assert np.max(np.abs(gpu.solid_state() - orc.solid_state())) <= 1e-14
    assert np.max(np.abs(gpu.get_f() - orc.get_f())) == 0.0
    with pytest.raises(lbm.LBMError) as e:  # no forcing iterations for a moving IBM solid
        gpu.set_solids([s], "IBM", n_iter=0)
    assert e.value.status == lbm.LBM_EINVAL
