"""Pins of the oracle's freely moving solids (Eq. 20 with the Eq. 17 force and torque).

The paper's reference data for moving solids (the ALE sedimentation runs of Sec. 3.2) is not
available, so the free motion is pinned by the cases it must reduce to:
* a very heavy free solid is the fixed solid (same fields and forces);
* a very heavy free solid started with a velocity is the prescribed translation;
* from rest, without flow, the first step is the buoyant free fall (1 - 1/rho_p) g exactly: the
  rest-state part of Eq. 17 cancels over a closed body, link by opposite link;
* a free inner cylinder of circular Couette flow spins up to the outer wall's angular velocity
  (rigid rotation is the only steady state), and stays centred.
"""
import math

import numpy as np
import pytest

from oracle import Oracle
from paper_1906_05445_amd import workloads as W

SHAPE = (30, 27, 25)
G = (2e-6, 0.0, 1e-6)


def _fields(o):
    r, u, t = o.macros()
    return r, u, t


def _pair_runs(solid_fixed, solid_free, density, steps, gravity=(0.0, 0.0, 0.0)):
    a = Oracle("D3Q19", "MRT", SHAPE, 0.8, g=G)
    a.set_solids([solid_fixed], "QUADRATIC")
    b = Oracle("D3Q19", "MRT", SHAPE, 0.8, g=G)
    b.set_solids([solid_free], "QUADRATIC")
    b.set_free(0, density, gravity)
    a.step(steps)
    b.step(steps)
    return a, b


def test_heavy_free_solid_is_fixed():
    s = W.solid("sphere", (14.2, 13.1, 12.4), 5.3)
    a, b = _pair_runs(s, s, 1e15, 40)
    ra, ua, ta = _fields(a)
    rb, ub, tb = _fields(b)
    assert np.array_equal(ta, tb)
    fl = ta != 1
    assert np.max(np.abs(ua[:, fl] - ub[:, fl])) <= 1e-12 * np.max(np.abs(ua[:, fl]))
    assert np.max(np.abs(ra[fl] - rb[fl])) <= 1e-12
    Fa, Fb = a.history()[:, 0, :3], b.history()[:, 0, :3]
    assert np.max(np.abs(Fa - Fb)) <= 1e-12 * np.max(np.abs(Fa))
    st = b.solid_state()[0]
    assert np.max(np.abs(st[3:])) < 1e-15 and np.allclose(st[:3], s["centre"], atol=1e-14, rtol=0)


def test_heavy_free_solid_is_prescribed_translation():
    U = (0.03, -0.02, 0.025)
    moving = W.solid("sphere", (14.2, 13.1, 12.4), 5.3, velocity=U)
    a, b = _pair_runs(moving, moving, 1e15, 60)
    ra, ua, ta = _fields(a)
    rb, ub, tb = _fields(b)
    assert np.array_equal(ta, tb)
    fl = ta != 1
    assert np.max(np.abs(ua[:, fl] - ub[:, fl])) <= 1e-12 * np.max(np.abs(ua[:, fl]))
    La, Lb = a.links(), b.links()
    for k in ("cell", "dir", "sid"):
        assert np.array_equal(La[k], Lb[k]), k
    assert np.max(np.abs(La["q"] - Lb["q"])) < 1e-12
    st = b.solid_state()[0]
    assert np.max(np.abs(st[3:6] - np.array(U))) < 1e-15  # F / (rho_p V_p) ~ 1e-18
    want = (np.array(moving["centre"]) + 60 * np.array(U)) % np.array(SHAPE)
    assert np.max(np.abs(st[:3] - want)) < 1e-12


@pytest.mark.parametrize("density", [1.03, 2.5])
@pytest.mark.parametrize("form", ["f", "h"])
def test_first_step_is_buoyant_free_fall(density, form):
    g = np.array([0.0, -2e-5, 1e-5])
    o = Oracle("D3Q19", "MRT", SHAPE, 0.8, form=form)
    s = W.solid("sphere", (14.2, 13.1, 12.4), 5.3)
    o.set_solids([s], "QUADRATIC")
    o.set_free(0, density, g)
    o.step(1)
    # no flow: the exchange cancels over the closed surface, exactly in the
    # deviation form (the rest-state terms -2 w_i e_i are summed compensated);
    # the literal form sums ~1e3 terms of size 2 w_i with plain additions
    F0 = o.history()[0, 0, :3]
    if form == "h":
        assert np.all(F0 == 0.0)
    else:
        assert np.max(np.abs(F0)) < 1e-14
    st = o.solid_state()[0]
    v1 = (1.0 - 1.0 / density) * g
    # rho_p - 1 rounds at a few ulp; the literal form's rounding-size force adds F0 / (rho_p V_p)
    Vp = 4.0 / 3.0 * math.pi * s["radius"] ** 3
    assert np.max(np.abs(st[3:6] - v1)) <= 4e-15 * np.max(np.abs(v1)) + np.max(np.abs(F0)) / (density * Vp)
    assert np.max(np.abs(st[:3] - (np.array(s["centre"]) + 0.5 * v1))) < 1e-15
    o.step(30)  # then it keeps falling, along g
    st = o.solid_state()[0]
    assert st[4] < v1[1] < 0.0 and st[5] > v1[2] > 0.0


def test_free_inner_cylinder_spins_up_to_rigid_rotation():
    R1, R2, Om2 = 6.0, 14.0, 0.01 / 14.0
    n = int(2 * R2 + 6)
    c = (n / 2.0 + 0.31, n / 2.0 - 0.17, 0.0)
    o = Oracle("D2Q9", "MRT", (n, n, 1), 1.0, rates=np.full(9, 1.0))
    o.set_solids([W.solid("cylinder", c, R1), W.solid("cylinder", c, R2, inverted=True, omega=(0, 0, Om2))],
                 "QUADRATIC")
    o.set_free(0, 1.0)
    nu = 0.5 / 3.0
    steps = int(6.0 * R2 * R2 / nu)  # several spin-up times
    o.step(steps)
    st = o.solid_state()[0]
    assert abs(st[8] / Om2 - 1.0) < 1e-4, st[8] / Om2  # measured 2e-7
    assert np.max(np.abs(st[:2] - np.array(c[:2]))) < 0.01  # measured 7e-4 lattice units
