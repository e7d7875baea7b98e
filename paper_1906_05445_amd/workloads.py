"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no step of the lattice Boltzmann method: it only draws and
lays out inputs -- solid geometry, Lagrangian surface meshes, relaxation
times, body forces and request traces -- so that the GPU library and the FP64
oracle are fed identical data.  All randomness comes from
``numpy.random.default_rng(seed)``.

The paper's own flows (a rotating-cylinder Couette cell, a pipe, a settling
cylinder and a sphere in an open uniform stream; Sec. 3) are stood in for by
periodic boxes of the same lattice, similar D/dx and similar Reynolds
numbers: the open-domain inlet/outlet and the reference data of the settling
case are not reproduced.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PHI = (1.0 + math.sqrt(5.0)) / 2.0


def solid(kind="sphere", centre=(0.0, 0.0, 0.0), radius=1.0, axis=(0.0, 0.0, 1.0), inverted=False,
          velocity=(0.0, 0.0, 0.0), omega=(0.0, 0.0, 0.0), density=0.0, gravity=(0.0, 0.0, 0.0)):
    """Solid description understood by both the GPU binding and the oracle.  density > 0: a free solid
    with that density ratio to the fluid and external acceleration gravity (velocity, omega: initial)."""
    c = list(map(float, centre)) + [0.0] * (3 - len(centre))
    return {"kind": kind, "inverted": bool(inverted), "centre": tuple(c[:3]), "radius": float(radius),
            "axis": tuple(map(float, axis)), "velocity": tuple(map(float, velocity)),
            "omega": tuple(map(float, omega)), "density": float(density),
            "gravity": tuple(map(float, gravity))}


# --------------------------------------------------------------------------
# Lagrangian meshes (inputs of the direct-forcing IBM, Sec. 2.1)
# --------------------------------------------------------------------------
def _icosahedron():
    v = []
    for a in (-1.0, 1.0):
        for b in (-PHI, PHI):
            v.append((0.0, a, b))
            v.append((a, b, 0.0))
            v.append((b, 0.0, a))
    v = np.array(sorted(v), dtype=np.float64)
    n = len(v)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n)
             if abs(np.sum((v[i] - v[j]) ** 2) - 4.0) < 1e-9]
    adj = {e for e in edges}
    faces = [(i, j, k) for (i, j) in edges for k in range(j + 1, n) if (i, k) in adj and (j, k) in adj]
    return v, edges, faces


def icosphere_frequency(radius: float) -> int:
    """Subdivision frequency giving about one point per unit area."""
    return max(1, int(round(radius * math.sqrt(4.0 * math.pi / 10.0))))


def icosphere(centre, radius, freq=None):
    """Geodesic sphere: every icosahedron face split into freq^2 triangles.

    Points: the 12 vertices, then the interior points of the 30 edges, then the
    interior points of the 20 faces, each projected onto the sphere.  Returns
    (X [10 f^2 + 2, 3], dV) with dV = 4 pi R^2 h / N (h = 1).
    """
    n = icosphere_frequency(radius) if freq is None else int(freq)
    v, edges, faces = _icosahedron()
    pts = [p for p in v]
    for (a, b) in edges:
        for k in range(1, n):
            pts.append(((n - k) * v[a] + k * v[b]) / n)
    for (a, b, c) in faces:
        for i in range(1, n):
            for j in range(1, n - i):
                k = n - i - j
                pts.append((i * v[a] + j * v[b] + k * v[c]) / n)
    P = np.array(pts, dtype=np.float64)
    P = P / np.sqrt(np.sum(P * P, axis=1))[:, None]
    X = np.asarray(centre, dtype=np.float64)[None, :] + radius * P
    dV = 4.0 * math.pi * radius * radius / X.shape[0]
    return X, dV


def circle(centre, radius, z=0.0):
    """Evenly spaced points on a circle, spacing about h = 1; dV = arc * h."""
    n = max(3, int(round(2.0 * math.pi * radius)))
    ang = 2.0 * math.pi * np.arange(n) / n
    X = np.stack([centre[0] + radius * np.cos(ang), centre[1] + radius * np.sin(ang), np.full(n, z)], axis=1)
    return X, 2.0 * math.pi * radius / n


def cylinder_surface(centre, radius, nz):
    """Rings of circle() points on every z plane 0..nz-1 (cylinder along z)."""
    rings = [circle(centre, radius, z=float(k))[0] for k in range(nz)]
    n = rings[0].shape[0]
    return np.concatenate(rings, axis=0), 2.0 * math.pi * radius / n


def lagrangian_mesh(s, lattice, shape, retraction=0.0):
    """Mesh of one solid at radius R - R_d (Breugem's retraction, Sec. 3.1)."""
    R = s["radius"] - retraction if not s["inverted"] else s["radius"] + retraction
    if lattice == "D2Q9":
        return circle(s["centre"], R)
    if s["kind"] == "cylinder":
        return cylinder_surface(s["centre"], R, shape[2])
    return icosphere(s["centre"], R)


# --------------------------------------------------------------------------
# flow parameters
# --------------------------------------------------------------------------
def nu_of_tau(tau: float) -> float:
    return (tau - 0.5) / 3.0


def tau_of_nu(nu: float) -> float:
    return 3.0 * nu + 0.5


def stokes_body_force(Re, nu, D, box_cells, solid_volume, n_spheres=1):
    """Body force density driving a periodic array of spheres at about Re.

    U_ref = Re nu / D; the Stokes drag 3 pi nu D U_ref of every sphere balances
    g over the fluid volume.  The achieved Re is reported from the measured
    superficial velocity, not from this estimate.
    """
    U = Re * nu / D
    return 3.0 * math.pi * nu * D * U * n_spheres / (box_cells - solid_volume), U


def _array_drag_factor(c):
    # K(c) of Sangani & Acrivos (1982), simple cubic array at solid fraction c
    return 1.0 / (1.0 - 1.7601 * c ** (1.0 / 3.0) + c - 1.5593 * c ** 2 + 3.9799 * c ** (8.0 / 3.0)
                  - 3.0734 * c ** (10.0 / 3.0))


def array_body_force(Re, nu, D, box_cells, solid_volume):
    """Body force density under which the periodic-array estimate below gives the mean velocity
    U = Re nu / D: g = 3 pi nu D U K(c) (1 + 0.15 Re^0.687) / (box - V_s).  Returns (g, U)."""
    U = Re * nu / D
    c = solid_volume / box_cells
    return 3.0 * math.pi * nu * D * U * _array_drag_factor(c) * (1.0 + 0.15 * Re ** 0.687) / (
        box_cells - solid_volume), U


def periodic_array_velocity(g, nu, D, box_cells, solid_volume):
    """Estimate of the mean fluid velocity that a body force g drives through a
    simple cubic array of spheres (one sphere of diameter D per periodic box):
    the root of  g (box - V_s) = 3 pi nu D U K(c) (1 + 0.15 Re^0.687),
    with K(c) = 1 / (1 - 1.7601 c^(1/3) + c - 1.5593 c^2 + 3.9799 c^(8/3)
    - 3.0734 c^(10/3)) the drag factor of Sangani & Acrivos (1982) for the
    simple cubic array at solid fraction c, and the Schiller-Naumann factor
    for the inertia at Re = U D / nu.  An initial condition only (a warm
    start for solves run to a steady drag): the flow then relaxes to the
    method's own steady state."""
    K = _array_drag_factor(solid_volume / box_cells)
    total = g * (box_cells - solid_volume)
    U = total / (3.0 * math.pi * nu * D * K)
    for _ in range(50):  # fixed point on the inertial factor (a contraction for these Re)
        U = total / (3.0 * math.pi * nu * D * K * (1.0 + 0.15 * (U * D / nu) ** 0.687))
    return U


@dataclass
class Case:
    name: str
    lattice: str
    collision: str
    shape: tuple
    tau: float
    g: tuple
    solids: list
    method: str
    steps: int
    storage: str = "F64"
    ibm_iters: int = 5
    retraction: float = 0.0
    meta: dict = field(default_factory=dict)
    delta: int = 4
    g_fluid_only: bool = True
    boundary: tuple = ("periodic", "periodic", "periodic")
    inflow: float = 0.0


def cylinder_channel_2d(n=64, R=8.3, centre=(32.4, 31.7), g=1e-6, tau=0.8, steps=2000, method="LINEAR"):
    """Periodic array of fixed cylinders driven by a body force, D2Q9 BGK FP64."""
    return Case("cylinder_2d_64", "D2Q9", "BGK", (n, n, 1), tau, (g, 0.0, 0.0),
                [solid("cylinder", centre, R, axis=(0, 0, 1))], method, steps)


def sphere_box(n=128, R=16.2, Re=20.0, tau=0.8, seed=2, method="QUADRATIC", storage="F64", steps=5000,
               retraction=0.0, delta=4, drive="stokes"):
    """Fixed sphere at a seed-drawn sub-grid offset in a periodic cube, D3Q19 MRT.  Body force: the
    Stokes drag of one sphere at Re (drive="stokes"; the steady flow of the array is slower), or the
    periodic-array estimate that gives Re at steady state (drive="array").  meta["U_init"]: the
    periodic-array estimate of the mean velocity under that force (a warm start)."""
    rng = np.random.default_rng(seed)
    c = np.array([n / 2.0] * 3) + rng.random(3)
    nu = nu_of_tau(tau)
    Vs = 4.0 / 3.0 * math.pi * R ** 3
    force = array_body_force if drive == "array" else stokes_body_force
    g, U = force(Re, nu, 2 * R, n ** 3, Vs)
    U0 = periodic_array_velocity(g, nu, 2 * R, n ** 3, Vs)
    return Case(f"sphere_{n}", "D3Q19", "MRT", (n, n, n), tau, (g, 0.0, 0.0), [solid("sphere", c, R)],
                method, steps, storage, retraction=retraction, meta={"Re": Re, "U_ref": U, "U_init": U0},
                delta=delta)


def settling_sphere(n=128, R=16.2, density=1.03, U_set=0.01, tau=0.8, seed=2, storage="F32", steps=5000,
                    method="QUADRATIC"):
    """A free sphere settling under gravity in a periodic cube (the density ratio of the paper's
    sedimentation case, Sec. 3.2), quadratic IBB (Eq. 20) or the IBM (Eq. 23).  Gravity from the Stokes
    estimate of a settling speed U_set; the fluid carries the opposite body force, so that no net force
    drives the box: on the fluid outside the sphere with IBB, on every cell with the IBM (whose fluid
    fills the sphere)."""
    rng = np.random.default_rng(seed)
    c = np.array([n / 2.0] * 3) + rng.random(3)
    nu = nu_of_tau(tau)
    Vp = 4.0 / 3.0 * math.pi * R ** 3
    gz = -6.0 * math.pi * nu * R * U_set / ((density - 1.0) * Vp)
    ibm = method == "IBM"
    g_fluid = -(density - 1.0) * Vp * gz / (n ** 3 - (0.0 if ibm else Vp))
    return Case(f"settle_{n}", "D3Q19", "MRT", (n, n, n), tau, (0.0, 0.0, g_fluid),
                [solid("sphere", c, R, density=density, gravity=(0.0, 0.0, gz))], method, steps, storage,
                meta={"U_set": U_set, "density": density}, g_fluid_only=not ibm)


def open_sphere(D=16.0, Re=20.0, U=0.05, method="ZHAO_YONG", storage="F32", steps=20000, seed=6, nu=None):
    """The sphere of Sec. 3.4: diameter D fixed at (6D, 6D, 6D) (plus a seed-drawn sub-node offset) in a
    24D x 12D x 12D box, uniform inflow U at x = 0, stress-free sides, convective outflow; nu from
    Re_p = U D / nu, or, given nu (the paper keeps nu fixed as it refines), U from it.  D3Q19 MRT."""
    rng = np.random.default_rng(seed)
    n = (int(round(24 * D)), int(round(12 * D)), int(round(12 * D)))
    c = np.array([6 * D, 6 * D, 6 * D]) + 0.5 * rng.random(3)
    if nu is None:
        nu = U * D / Re
    else:
        U = Re * nu / D
    return Case(f"open_sphere_D{D:g}_Re{Re:g}", "D3Q19", "MRT", n, tau_of_nu(nu), (0.0, 0.0, 0.0),
                [solid("sphere", c, D / 2.0)], method, steps, storage, meta={"Re": Re, "U_ref": U, "D": D},
                boundary=("open", "slip", "slip"), inflow=U)


def drag_coefficient(F, Re, nu):
    """C_D = 8 F_D / (rho_f Re_p^2 pi nu^2) (Sec. 3.4), rho_f = 1."""
    return 8.0 * F / (Re * Re * math.pi * nu * nu)


def schiller_naumann(Re):
    """Standard drag correlation of a sphere, C_D = 24/Re (1 + 0.15 Re^0.687) (Re < 800): a sanity
    reference, not the paper's data."""
    return 24.0 / Re * (1.0 + 0.15 * Re ** 0.687)


def sphere_pack(n=256, count=64, R=8.0, gap=2.0, Re=10.0, tau=0.8, seed=3, storage="F64", steps=10000,
                method="QUADRATIC", drive="stokes"):
    """Random sequential addition of non-overlapping spheres (periodic gap >= gap).  Body force as in
    sphere_box (drive), each sphere taken with its share of the box; meta["U_init"]: the periodic-array
    estimate of the mean velocity under it."""
    rng = np.random.default_rng(seed)
    cs = []
    dmin = 2 * R + gap
    while len(cs) < count:
        c = rng.random(3) * n
        ok = True
        for d in cs:
            s = c - d
            s -= n * np.round(s / n)
            if np.sqrt(np.sum(s * s)) < dmin:
                ok = False
                break
        if ok:
            cs.append(c)
    nu = nu_of_tau(tau)
    Vs = 4.0 / 3.0 * math.pi * R ** 3
    if drive == "array":
        g, U = array_body_force(Re, nu, 2 * R, n ** 3 / count, Vs)
    else:
        g, U = stokes_body_force(Re, nu, 2 * R, n ** 3, count * Vs, n_spheres=count)
    U0 = periodic_array_velocity(g, nu, 2 * R, n ** 3 / count, Vs)
    return Case(f"pack_{n}_{count}", "D3Q19", "MRT", (n, n, n), tau, (g, 0.0, 0.0),
                [solid("sphere", c, R) for c in cs], method, steps, storage,
                meta={"Re": Re, "U_ref": U, "U_init": U0})


def moving_sphere_batch(count=512, seed=4, edge=(32, 96), radius=(4.0, 16.0), speed=(0.005, 0.02),
                        tau=0.8, steps=2000):
    """Independent cubic lattices, each with one sphere translating at constant velocity.

    Radius is drawn in [4, 16] and capped at edge/4 so that the sphere spans at
    most half of its box.
    """
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(count):
        L = int(rng.integers(edge[0], edge[1] + 1))
        R = float(rng.uniform(radius[0], radius[1]))
        R = min(R, L / 4.0)
        sp = float(rng.uniform(speed[0], speed[1]))
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        c = rng.random(3) * L
        cases.append(Case(f"moving_{k}", "D3Q19", "MRT", (L, L, L), tau, (0.0, 0.0, 0.0),
                          [solid("sphere", c, R, velocity=tuple(sp * d))], "QUADRATIC", steps, "F32"))
    return cases


def request_trace(count=256, rate=50.0, seed=5, edge=(48, 160), Re=(1.0, 100.0), U_ref=0.05):
    """Poisson arrivals of flow-past-sphere solves (edge, R = edge/8, Re, IBB or IBM)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    for k in range(count):
        L = int(rng.integers(edge[0], edge[1] + 1))
        R = L / 8.0
        re = float(rng.uniform(Re[0], Re[1]))
        method = "QUADRATIC" if rng.random() < 0.5 else "IBM"
        nu = U_ref * 2 * R / re
        tau = tau_of_nu(nu)
        c = np.array([L / 2.0] * 3) + rng.random(3)
        Vs = 4.0 / 3.0 * math.pi * R ** 3
        g, _ = stokes_body_force(re, nu, 2 * R, L ** 3, Vs)
        U0 = periodic_array_velocity(g, nu, 2 * R, L ** 3, Vs)
        out.append({"arrival": float(t[k]), "case": Case(f"req_{k}", "D3Q19", "MRT", (L, L, L), tau,
                                                          (g, 0.0, 0.0), [solid("sphere", c, R)], method,
                                                          0, "F32", meta={"Re": re, "U_init": U0})})
    return out


def random_populations(Q, N, seed, amplitude=0.01, weights=None):
    """Positive random populations around the rest state (for permutation tests)."""
    rng = np.random.default_rng(seed)
    base = np.ones((Q, 1)) / Q if weights is None else np.asarray(weights, dtype=np.float64)[:, None]
    return base * (1.0 + amplitude * rng.uniform(-1.0, 1.0, size=(Q, N)))
