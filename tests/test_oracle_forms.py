"""The oracle's two representations of one step agree within the literal form's rounding.

The literal form stores the populations f_i and evaluates Eq. 1 / Eq. 3, the
bounce-back formulas (Eq. 10-16) and the momentum exchange of Eq. 17 on them
with plain sums, as the paper writes them.  The deviation form stores
h_i = f_i - w_i: the same arithmetic after an exact change of variables
(every relation is linear in f apart from f_eq, and every bounce-back weight
set sums to one), with three decades less rounding.  The GPU library keeps the
deviation too, so the deviation form is checked here against the literal one
on every boundary scheme, the IBM, a translating solid (refill) and a free
solid.

Bars, from the largest difference measured over these cases.  The literal
form rounds populations of ~0.1-0.4 at 2^-53 each step, so its error has an
absolute floor whatever the flow: velocities ~4e-16, and the plain Eq. 17 sum,
which adds one term per link (each carrying its populations' rounding) and
cancels them down to the force, ~2e-16 per link here (4.6e-16 per link in the
GPU comparison of a 4170-link sphere).
  velocity    max|du| <= 1e-12 max|u| + 2e-15      measured <= 3.8e-16 abs, 3.7e-13 rel
  density     max|drho| <= 5e-13                   measured <= 1.4e-13
  populations max|df| <= 2e-13                     measured <= 6.2e-14
  force       max|dF| <= 1e-11 F_scale + 1e-15 n   measured <= 2.1e-13 abs, 4.4e-12 rel
(F_scale = max(|F(end)|, |g| V_fluid), as in the GPU parity tests; n the
number of links, or of Lagrangian points for the IBM.)

A mistake in either form's algebra (a dropped rest-state term, a wrong
offset in f_eq or in the refill density) is a difference proportional to the
flow, not to the rounding: the scaling test below drives the same case 16
times harder and requires the relative difference to fall.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_1906_05445_amd import workloads as W

# (relative, absolute floor) per quantity: |d| <= rel * scale + floor (the force floor per term)
BARS = {"u": (1e-12, 2e-15), "rho": (5e-13, 0.0), "f": (2e-13, 0.0), "F": (1e-11, 1e-15)}

SHAPE3 = (26, 22, 19)
SPHERE3 = W.solid("sphere", (12.3, 10.6, 9.2), 5.7)


def _run(form, lat, coll, shape, tau, g, solids, method, steps, fluid_only=True, free=None):
    o = Oracle(lat, coll, shape, tau, g=g, g_fluid_only=fluid_only, form=form)
    o.set_solids(solids, method)
    if method == "IBM":
        for k, s in enumerate(solids):
            X, dV = W.lagrangian_mesh(s, lat, shape)
            o.set_lagrangian(k, X, dV)
    if free is not None:
        o.set_free(0, *free)
    nterms = max(len(o.links()["cell"]), o.nlag, 1)  # at the start; moving solids keep about as many
    o.step(steps)
    rho, u, t = o.macros()
    return {"rho": rho, "u": u, "t": t, "H": o.history(), "f": o.get_f(), "ex": o.node_flags()[0], "n": nterms}


def _diff(a, b, g):
    """Absolute differences and the scale each is measured against."""
    assert np.array_equal(a["t"], b["t"])
    fl = a["t"] != 1
    now = a["ex"] != 1
    return {"u": (np.max(np.abs(a["u"][:, fl] - b["u"][:, fl])), np.max(np.abs(b["u"][:, fl]))),
            "rho": (np.max(np.abs(a["rho"][fl] - b["rho"][fl])), 1.0),
            "f": (np.max(np.abs(a["f"][:, now] - b["f"][:, now])), 1.0),
            "F": (np.max(np.abs(a["H"][..., :3] - b["H"][..., :3])),
                  max(np.max(np.abs(b["H"][-1, :, :3])), np.linalg.norm(g) * fl.sum()))}


def _check(lat, coll, shape, tau, g, solids, method, steps, **kw):
    lit = _run("f", lat, coll, shape, tau, g, solids, method, steps, **kw)
    dev = _run("h", lat, coll, shape, tau, g, solids, method, steps, **kw)
    d = _diff(lit, dev, g)
    for k, (rel, floor) in BARS.items():
        err, scale = d[k]
        if k == "F":
            floor *= lit["n"]
        assert err <= rel * scale + floor, f"{k}: {err:.3e} > {rel} * {scale:.3e} + {floor}"
    return {k: err / scale for k, (err, scale) in d.items()}


@pytest.mark.parametrize("method", ["BB", "LINEAR", "QUADRATIC", "YU", "ZHAO_YONG", "IBM"])
def test_forms_agree_d3q19_mrt(method):
    _check("D3Q19", "MRT", SHAPE3, 0.8, (3e-6, 1e-6, 0.0), [SPHERE3], method, 250)


@pytest.mark.parametrize("method", ["LINEAR", "QUADRATIC", "IBM"])
def test_forms_agree_d2q9_bgk(method):
    _check("D2Q9", "BGK", (48, 40), 0.8, (1e-6, 0.0), [W.solid("sphere", (23.6, 19.3), 6.4)], method, 1000)


def test_forms_agree_translating_sphere_with_refill():
    s = W.solid("sphere", (12.3, 10.6, 9.2), 5.7, velocity=(0.03, -0.02, 0.015))
    _check("D3Q19", "MRT", SHAPE3, 0.8, (0.0, 0.0, 0.0), [s], "QUADRATIC", 150)


def test_forms_agree_free_sphere():
    _check("D3Q19", "MRT", SHAPE3, 0.8, (0.0, 0.0, 0.0), [SPHERE3], "QUADRATIC", 150,
           free=(1.5, (0.0, -2e-5, 1e-5)))


def test_forms_agree_ibm_with_rotation():
    s = W.solid("sphere", (12.3, 10.6, 9.2), 5.7, omega=(0.0, 0.0, 0.004))
    _check("D3Q19", "MRT", SHAPE3, 0.8, (0.0, 0.0, 0.0), [s], "IBM", 200, fluid_only=False)


def test_form_difference_is_rounding_not_algebra():
    """16 times the forcing: 16 times the velocities, about the same absolute
    rounding, so the relative difference falls (a term of the algebra missing
    from one form would keep it, or make it grow)."""
    d1 = _check("D3Q19", "MRT", SHAPE3, 0.8, (3e-6, 1e-6, 0.0), [SPHERE3], "QUADRATIC", 200)
    d16 = _check("D3Q19", "MRT", SHAPE3, 0.8, (48e-6, 16e-6, 0.0), [SPHERE3], "QUADRATIC", 200)
    assert d16["u"] < d1["u"] / 4.0, (d1["u"], d16["u"])
    assert d16["F"] < d1["F"] / 4.0, (d1["F"], d16["F"])
