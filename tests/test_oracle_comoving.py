"""Closed-form pins of the moving-wall pieces and of the IBM coupling.

1. Galilean co-moving state.  A uniform flow f = f_eq(1, U) with a solid that
   translates at the same U is an exact steady state of the method: the
   collision leaves an equilibrium unchanged, streaming a uniform field keeps
   it, every bounce-back formula returns f_eq_i because its weights sum to one
   and the wall term 2 w_i rho0 e_i.u_w / c_s^2 (Eq. 10) is exactly
   f_eq_i(1, U) - f_eq_ibar(1, U), and a node uncovered by the moving solid is
   refilled with f_eq(rho_bar, u_w) = f_eq(1, U).  The momentum exchange of
   Eq. 17 then sums to zero over the closed surface: per direction, the links
   e_i and e_ibar are equal in number (each solid run along a lattice line has
   one entry and one exit), and every term is odd or even in e_i.  So this
   pins the refill rule (its density and velocity), the moving-wall term of the
   bounce-back schemes, the link rebuild as the solid crosses grid lines, and
   the wall velocity inside Eq. 17.  With the IBM and U^d = U the interpolated
   velocity equals U exactly (the delta functions sum to one), so no force
   arises and the flow stays uniform too.

2. One Lagrangian point in a uniform flow.  With u^0 = (j + g/2)/rho uniform,
   Eq. 5 interpolates U~^1 = u^0 exactly; Eq. 7-9 then give, with the sum of
   the squared delta weights s = sum_x delta_h(x - X)^2 h^3,
       U~^{k+1} - U^d = (U~^k - U^d)(1 - s dV),
   so the total point force after n iterations is
       F = (U^d - u^0) (1 - r^n) / (1 - r),  r = 1 - s dV.
   s is (3/8)^D for Peskin's 4-point function (Eq. 6), (1/2)^D for the
   3-point function of Roma et al., and prod_a [(1 - a_a)^2 + a_a^2] for the
   2-point hat (a_a the fractional part of X_a).  This fixes the reading of
   Sec. 2.1 that the oracle takes: which velocity is interpolated (half the
   body force, none of the boundary force), the force factor 1 of Eq. 7, the
   full spread force in the velocity update of Eq. 9, and the number of
   iterations; the force on the solid is -F dV and the collision at a stencil
   node uses u = (j + (g + f)/2)/rho with f = F delta_h(x - X) dV.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_1906_05445_amd import workloads as W

SHAPE = (21, 18, 16)


def _uniform(o, U, rho=1.0):
    f = np.tile(np.asarray(o.feq(rho, U))[:, None], (1, o.N))
    o.set_f(f)
    return f[:, 0]


@pytest.mark.parametrize("form", ["f", "h"])
@pytest.mark.parametrize("method", ["BB", "LINEAR", "QUADRATIC", "YU", "ZHAO_YONG"])
def test_comoving_translating_sphere_stays_uniform(method, form):
    U = (0.045, -0.03, 0.025)  # 2.7, 1.8 and 1.5 cells in 60 steps: the solid crosses grid lines
    s = W.solid("sphere", (10.3, 8.6, 7.9), 4.6, velocity=U)
    o = Oracle("D3Q19", "MRT", SHAPE, 0.8, form=form)
    o.set_solids([s], method)
    feq = _uniform(o, U)
    n0 = o.links()["cell"].size
    o.step(60)
    ex, _, _ = o.node_flags()
    f = o.get_f()[:, ex == 0]
    # the literal form rounds populations of ~0.3 (and rho, u from them) every step
    bar = 1e-15 if form == "f" else 1e-16
    assert np.max(np.abs(f - feq[:, None])) <= bar
    H = o.history()
    assert H.shape[0] == 60 and n0 > 0
    # Eq. 17 over the closed surface: zero up to the rounding of ~1.5e3 terms of size ~0.1 (each
    # rounded at ~1e-17; the literal form also adds them with plain additions)
    assert np.max(np.abs(H[:, 0, :3])) <= (1e-13 if form == "f" else 1e-14)
    # the fluid velocity of the last collision is U at every fluid node, and u_w = U at solid nodes
    _, u, t = o.macros()
    assert np.max(np.abs(u - np.asarray(U)[:, None])) <= 1e-14


@pytest.mark.parametrize("form", ["f", "h"])
def test_comoving_translating_ibm_sphere_stays_uniform(form):
    U = (0.045, -0.03, 0.025)
    s = W.solid("sphere", (10.3, 8.6, 7.9), 4.6, velocity=U)
    o = Oracle("D3Q19", "MRT", SHAPE, 0.8, g_fluid_only=False, form=form)
    o.set_solids([s], "IBM")
    X, dV = W.lagrangian_mesh(s, "D3Q19", SHAPE)
    o.set_lagrangian(0, X, dV)
    feq = _uniform(o, U)
    o.step(40)
    f = o.get_f()
    assert np.max(np.abs(f - feq[:, None])) <= (1e-15 if form == "f" else 1e-16)
    # U^d - U~ vanishes up to the rounding of the interpolation sums
    assert np.max(np.abs(o.lagrangian_force())) <= 1e-15
    assert np.max(np.abs(o.history()[:, 0, :3])) <= 1e-13


def _sum_phi_sq(delta, X):
    """sum over the stencil of the squared 1D weights, multiplied over the axes"""
    s = 1.0
    for x in X:
        if delta == 4:
            s *= 3.0 / 8.0
        elif delta == 3:
            s *= 0.5
        else:
            a = x - np.floor(x)
            s *= (1.0 - a) ** 2 + a ** 2
    return s


@pytest.mark.parametrize("form", ["f", "h"])
@pytest.mark.parametrize("lat,delta,n_iter", [("D3Q19", 4, 5), ("D3Q19", 4, 1), ("D3Q19", 3, 5), ("D3Q19", 2, 3),
                                              ("D2Q9", 4, 5), ("D2Q9", 2, 4)])
def test_single_point_direct_forcing_recurrence(lat, delta, n_iter, form):
    D = 2 if lat == "D2Q9" else 3
    shape = (17, 15, 1) if D == 2 else (17, 15, 13)
    c = (8.4, 7.3, 0.0) if D == 2 else (8.4, 7.3, 6.1)
    W_rot = (0.0, 0.0, 0.03) if D == 2 else (0.01, -0.02, 0.03)
    solid = W.solid("sphere", c, 2.0, omega=W_rot)  # fixed: U^d = omega x (X - centre)
    g = np.array([2e-5, -1e-5, 0.0 if D == 2 else 3e-5])
    rho0, U0 = 1.015, np.array([0.02, 0.01, 0.0 if D == 2 else -0.015])
    o = Oracle(lat, "MRT", shape, 0.8, g=g, g_fluid_only=False, form=form)
    o.set_solids([solid], "IBM")
    o.set_ibm_iters(n_iter)
    o.set_ibm_delta(delta)
    X = np.array([[c[0] + 1.37, c[1] - 0.82, 0.0 if D == 2 else c[2] + 0.55]])
    dV = 0.9
    o.set_lagrangian(0, X, dV)
    _uniform(o, U0, rho0)
    o.step(1)
    u0 = U0 + 0.5 * g / rho0
    r = X[0] - np.asarray(c)
    Ud = np.cross(np.asarray(W_rot), r)
    if D == 2:
        Ud[2] = 0.0
    s = _sum_phi_sq(delta, X[0][:D])
    rr = 1.0 - s * dV
    F = (Ud - u0) * (1.0 - rr ** n_iter) / (1.0 - rr)
    got = o.lagrangian_force()[0]
    assert np.max(np.abs(got - F)) <= 1e-14 * np.max(np.abs(F)), (got, F)
    # the force and torque on the solid
    H = o.history()[0, 0]
    assert np.max(np.abs(H[:3] + F * dV)) <= 1e-14 * np.max(np.abs(F))
    assert np.max(np.abs(H[3:] + np.cross(r, F * dV))) <= 1e-14 * np.max(np.abs(F))
    # the spread force is F dV times the delta weight: its sum over the box is F dV
    fib = o.ibm_force_field()
    assert np.max(np.abs(fib.sum(axis=1) - F * dV)) <= 1e-14 * np.max(np.abs(F))
    # collision velocity at every node: u = (j + (g + f)/2)/rho with j = rho0 U0
    _, u, _ = o.macros()
    expect = U0[:, None] + 0.5 * (g[:, None] + fib) / rho0
    assert np.max(np.abs(u - expect)) <= 1e-15


@pytest.mark.parametrize("form", ["f", "h"])
def test_comoving_cover_momentum(form):
    """Covering and uncovering momentum (R38) in the co-moving state.  Every
    fluid node holds f_eq(1, U), whose momentum is U, and a node the solid
    uncovers is refilled with f_eq(1, U) as well; Eq. 17 sums to zero force.
    So the force and torque a step reports with the correction, less those of
    the same run without it, are U times (nodes covered - nodes uncovered) by
    the move before it and the sum of r x U over them (r from the solid's
    centre after that move, shortest periodic image): counts taken from the
    node flags, the lever arms from the prescribed motion."""
    U = np.array([0.045, -0.03, 0.025])
    c0 = np.array([10.3, 8.6, 7.9])
    L = np.array(SHAPE, dtype=float)
    s = W.solid("sphere", tuple(c0), 4.6, velocity=tuple(U))
    o = Oracle("D3Q19", "MRT", SHAPE, 0.8, form=form)
    o.set_solids([s], "QUADRATIC")
    o.set_cover(True)
    _uniform(o, U)
    x, y, z = np.meshgrid(*(np.arange(n) for n in SHAPE), indexing="ij")
    pos = np.stack([a.transpose(2, 1, 0).ravel() for a in (x, y, z)], axis=1)  # cell n = x + nx (y + ny z)
    expect, moved = [], 0
    ex0, _, _ = o.node_flags()
    for t in range(40):
        o.step(1)
        ex1, _, _ = o.node_flags()
        cov, unc = (ex0 == 0) & (ex1 != 0), (ex0 != 0) & (ex1 == 0)
        moved += int(cov.sum() + unc.sum())
        Y = np.mod(c0 + (t + 1) * U, L)
        r = pos - Y
        r -= L * np.round(r / L)
        F = U * (cov.sum() - unc.sum())
        T = np.cross(r[cov], U).sum(axis=0) - np.cross(r[unc], U).sum(axis=0)
        expect.append(np.concatenate([F, T]))
        ex0 = ex1
    # off: the same run (the fluid does not depend on the setting) reports Eq. 17 alone, zero force
    o2 = Oracle("D3Q19", "MRT", SHAPE, 0.8, form=form)
    o2.set_solids([s], "QUADRATIC")
    _uniform(o2, U)
    o2.step(40)
    H0 = o2.history()
    assert np.max(np.abs(H0[:, 0, :3])) <= 1e-13
    H = o.history()
    assert moved > 50  # the solid covers and uncovers nodes on most steps
    got = H[1:, 0, :] - H0[1:, 0, :]  # the force of step t + 1 carries the move of step t
    want = np.array(expect[:-1])
    assert np.max(np.abs(got[:, :3] - want[:, :3])) <= 1e-13
    assert np.max(np.abs(got[:, 3:] - want[:, 3:])) <= 1e-12
    assert np.array_equal(H[0], H0[0])  # nothing moved before the first step
