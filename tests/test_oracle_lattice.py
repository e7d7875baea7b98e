"""Pins of the oracle's lattice, equilibrium, forcing and collision.

Each check is fixed by mathematics independent of the oracle's code: exact
rational moment identities of the velocity sets, the moments that the
equilibrium and the forcing term must have, MRT with one rate reducing to BGK
(Sec. 3.1 runs "MRT with identical rates"), and the exact permutation that a
step reduces to when nothing relaxes.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import Oracle

LATTICES = ["D2Q9", "D3Q19"]


def _mk(lat, coll="MRT", shape=None, **kw):
    if shape is None:
        shape = (6, 5, 1) if lat == "D2Q9" else (6, 5, 4)
    return Oracle(lat, coll, shape, kw.pop("tau", 0.8), **kw)


@pytest.mark.parametrize("lat", LATTICES)
def test_velocity_set_moments_exact(lat):
    o = _mk(lat)
    e, w, opp = o.lattice_tables()
    D = 2 if lat == "D2Q9" else 3
    W = [Fraction(x).limit_denominator(100) for x in w]
    for x, fx in zip(w, W):
        assert float(fx) == x  # the stored weight is the rational one, correctly rounded
    assert sum(W) == 1
    for a in range(D):
        assert sum(Wi * int(ei[a]) for Wi, ei in zip(W, e)) == 0
        for b in range(D):
            m2 = sum(Wi * int(ei[a]) * int(ei[b]) for Wi, ei in zip(W, e))
            assert m2 == (Fraction(1, 3) if a == b else 0)
            for c in range(D):
                assert sum(Wi * int(ei[a]) * int(ei[b]) * int(ei[c]) for Wi, ei in zip(W, e)) == 0
                for d in range(D):
                    m4 = sum(Wi * int(ei[a]) * int(ei[b]) * int(ei[c]) * int(ei[d]) for Wi, ei in zip(W, e))
                    iso = Fraction(int(a == b and c == d) + int(a == c and b == d) + int(a == d and b == c), 9)
                    assert m4 == iso
    for i in range(len(w)):
        assert np.all(e[opp[i]] == -e[i])
        if i > 0:
            assert opp[i] == (i + 1 if i % 2 == 1 else i - 1)


@pytest.mark.parametrize("lat", LATTICES)
def test_equilibrium_moments(lat):
    o = _mk(lat)
    e, w, _ = o.lattice_tables()
    rng = np.random.default_rng(11)
    D = 2 if lat == "D2Q9" else 3
    for _ in range(20):
        rho = 1.0 + 0.1 * rng.standard_normal()
        u = np.zeros(3)
        u[:D] = 0.05 * rng.standard_normal(D)
        feq = o.feq(rho, u)
        assert abs(feq.sum() - rho) < 1e-15
        assert np.max(np.abs(feq @ e - rho * u)) < 1e-15
        P = np.einsum("i,ia,ib->ab", feq, e, e)[:D, :D]
        assert np.max(np.abs(P - (rho / 3.0 * np.eye(D) + rho * np.outer(u[:D], u[:D])))) < 1e-15


@pytest.mark.parametrize("lat", LATTICES)
def test_forcing_moments(lat):
    o = _mk(lat)
    e, w, _ = o.lattice_tables()
    rng = np.random.default_rng(12)
    D = 2 if lat == "D2Q9" else 3
    for _ in range(20):
        u = np.zeros(3)
        F = np.zeros(3)
        u[:D] = 0.05 * rng.standard_normal(D)
        F[:D] = 1e-3 * rng.standard_normal(D)
        Fi = o.forcing(u, F)
        assert abs(Fi.sum()) < 1e-17
        assert np.max(np.abs(Fi @ e - F)) < 1e-17
        # second moment of Guo's term: u F + F u
        P = np.einsum("i,ia,ib->ab", Fi, e, e)[:D, :D]
        assert np.max(np.abs(P - (np.outer(u[:D], F[:D]) + np.outer(F[:D], u[:D])))) < 1e-17


@pytest.mark.parametrize("lat", LATTICES)
@pytest.mark.parametrize("coll", ["BGK", "MRT"])
def test_collision_adds_exactly_the_force(lat, coll):
    rng = np.random.default_rng(13)
    Q = 9 if lat == "D2Q9" else 19
    rates = None if coll == "BGK" else rng.uniform(0.3, 1.9, size=Q)
    o = _mk(lat, coll, rates=rates)
    e, w, _ = o.lattice_tables()
    D = 2 if lat == "D2Q9" else 3
    for _ in range(10):
        fin = w * (1.0 + 0.05 * rng.standard_normal(Q))
        F = np.zeros(3)
        F[:D] = 1e-4 * rng.standard_normal(D)
        fout = o.collide_node(fin, F)
        assert abs(fout.sum() - fin.sum()) < 1e-15
        assert np.max(np.abs(fout @ e - fin @ e - F)) < 1e-15


@pytest.mark.parametrize("lat", LATTICES)
def test_mrt_matrix_orthogonal_and_inverse(lat):
    o = _mk(lat)
    M, Mi = o.mrt_matrices()
    Q = M.shape[0]
    G = M @ M.T
    off = G - np.diag(np.diag(G))
    assert np.max(np.abs(off)) < 1e-12
    assert np.max(np.abs(Mi @ M - np.eye(Q))) < 1e-13
    assert np.max(np.abs(M @ Mi - np.eye(Q))) < 1e-13
    assert np.all(np.abs(M[0] - 1.0) < 1e-15)  # density row


@pytest.mark.parametrize("lat", LATTICES)
def test_default_rates_magic_parameter(lat):
    tau = 0.8
    o = _mk(lat, tau=tau)
    S = o.rates()
    odd = [4, 6] if lat == "D2Q9" else [4, 6, 8, 16, 17, 18]
    cons = [0, 3, 5] if lat == "D2Q9" else [0, 3, 5, 7]
    snu = 1.0 / tau
    for k in range(len(S)):
        if k in odd:
            assert abs((1.0 / snu - 0.5) * (1.0 / S[k] - 0.5) - 3.0 / 16.0) < 1e-15
        elif k not in cons:
            assert S[k] == snu


@pytest.mark.parametrize("lat", LATTICES)
def test_mrt_single_rate_equals_bgk(lat):
    tau = 0.77
    Q = 9 if lat == "D2Q9" else 19
    rng = np.random.default_rng(14)
    mrt = _mk(lat, "MRT", tau=tau, rates=np.full(Q, 1.0 / tau))
    bgk = _mk(lat, "BGK", tau=tau)
    e, w, _ = bgk.lattice_tables()
    D = 2 if lat == "D2Q9" else 3
    for _ in range(10):
        fin = w * (1.0 + 0.05 * rng.standard_normal(Q))
        F = np.zeros(3)
        F[:D] = 1e-4 * rng.standard_normal(D)
        assert np.max(np.abs(mrt.collide_node(fin, F) - bgk.collide_node(fin, F))) < 1e-15
    # and over many steps of a forced, perturbed periodic lattice
    shape = (8, 7, 1) if lat == "D2Q9" else (6, 5, 4)
    g = (1e-5, -2e-6, 3e-6)
    a = Oracle(lat, "MRT", shape, tau, rates=np.full(Q, 1.0 / tau), g=g)
    b = Oracle(lat, "BGK", shape, tau, g=g)
    f0 = w[:, None] * (1.0 + 0.01 * rng.standard_normal((Q, a.N)))
    a.set_f(f0)
    b.set_f(f0)
    a.step(1000)
    b.step(1000)
    assert np.max(np.abs(a.get_f() - b.get_f())) < 1e-12


@pytest.mark.parametrize("lat", LATTICES)
@pytest.mark.parametrize("form", ["f", "h"])
def test_no_relaxation_step_is_exact_streaming(lat, form):
    """With S = 0 and g = 0 a step is a pure periodic shift of each stored
    population (f in the literal form, h = f - w in the deviation form)."""
    Q = 9 if lat == "D2Q9" else 19
    shape = (7, 5, 1) if lat == "D2Q9" else (7, 5, 4)
    o = Oracle(lat, "MRT", shape, 0.8, rates=np.zeros(Q), form=form)
    e, w, _ = o.lattice_tables()
    rng = np.random.default_rng(15)
    h0 = w[:, None] * 0.1 * rng.uniform(-1, 1, size=(Q, o.N))
    x0 = w[:, None] + h0 if form == "f" else h0
    (o.set_f if form == "f" else o.set_h)(x0)
    o.step(3)
    nx, ny, nz = shape
    ref = x0.reshape(Q, nz, ny, nx).copy()
    for i in range(Q):
        ref[i] = np.roll(ref[i], shift=(3 * e[i][2], 3 * e[i][1], 3 * e[i][0]), axis=(0, 1, 2))
    got = o.get_f() if form == "f" else o.get_h()
    assert np.array_equal(got, ref.reshape(Q, -1))


@pytest.mark.parametrize("form", ["f", "h"])
def test_no_relaxation_with_halfway_walls_is_a_permutation(form):
    """S = 0, g = 0, u_w = 0 and halfway walls: streaming plus exact reversal
    of the stored populations, in either form."""
    Q = 9
    nx, ny = 5, 8
    o = Oracle("D2Q9", "MRT", (nx, ny, 1), 0.8, rates=np.zeros(Q), form=form)
    o.set_solids([{"kind": "plane", "centre": (0, 0.5, 0), "axis": (0, 1, 0)},
                  {"kind": "plane", "centre": (0, ny - 1.5, 0), "axis": (0, -1, 0)}], "QUADRATIC")
    e, w, opp = o.lattice_tables()
    rng = np.random.default_rng(16)
    f0 = w[:, None] * 0.1 * rng.uniform(-1, 1, size=(Q, o.N))  # deviations h = f - w
    if form == "f":
        f0 = w[:, None] + f0
    (o.set_f if form == "f" else o.set_h)(f0)
    o.step(1)
    fluid = lambda y: 1 <= y <= ny - 2
    ref = np.zeros_like(f0)
    for y in range(ny):
        if not fluid(y):
            continue
        for x in range(nx):
            n = x + nx * y
            for i in range(Q):
                sx, sy = (x - e[i][0]) % nx, y - e[i][1]
                if fluid(sy):
                    ref[i, n] = f0[i, sx + nx * sy]
                else:
                    ref[i, n] = f0[opp[i], n]
    got = o.get_f() if form == "f" else o.get_h()
    mask = np.array([fluid(n // nx) for n in range(o.N)])
    assert np.array_equal(got[:, mask], ref[:, mask])
