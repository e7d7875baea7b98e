"""Pins of the open-domain boundaries of Sec. 3.4 in the oracle.

The paper's sphere case has a uniform inflow at x = 0, four stress-free
sides and a convective outflow (Sec. 3.4).  Readings (the paper gives the
conditions, not their lattice form): the inlet is halfway bounce-back with
the inflow velocity as wall velocity (the form of Eq. 10), the stress-free
sides are specular reflection at planes halfway outside the first and last
node layers, the outflow is the convective condition taken for the
populations entering the last layer, first-order implicit in time and
upwind in x, with U_o the streamwise velocity of the last collision there.

1. A uniform stream f_eq(1, U) entering at U is an exact steady state: the
   collision keeps an equilibrium, specular reflection maps f_eq to itself
   (no normal velocity), the inlet returns f_eq,i = f_eq,ibar + 6 w_i e_i.U,
   and the outflow average of two equal values is that value.
2. Stress-free planes are mirrors: a run between them equals, up to
   rounding, the periodic run of the mirror-doubled box on mirror-symmetric
   data (the collision commutes with the reflection; streaming across the
   doubled box's mirror line is the specular reflection).  The periodic
   oracle is pinned on its own (test_oracle_lattice, test_oracle_flows).
3. Mass balance at the inlet and outlet: each inlet node adds exactly U per
   step (the wall terms 6 w_i e_ix U over the directions entering sum to U),
   so the total mass changes by A U minus what leaves through the last layer.
"""
import numpy as np
import pytest

from oracle import Oracle

U_IN = 0.04


@pytest.mark.parametrize("form", ["f", "h"])
@pytest.mark.parametrize("lat,coll", [("D2Q9", "BGK"), ("D3Q19", "MRT")])
def test_uniform_stream_is_steady(lat, coll, form):
    shape = (14, 9, 1) if lat == "D2Q9" else (12, 8, 7)
    o = Oracle(lat, coll, shape, 0.8, form=form)
    o.set_boundaries("open", "slip", "periodic" if lat == "D2Q9" else "slip", inflow=U_IN)
    feq = np.asarray(o.feq(1.0, (U_IN, 0.0, 0.0)))
    o.set_f(np.tile(feq[:, None], (1, o.N)))
    o.step(50)
    f = o.get_f()
    assert np.max(np.abs(f - feq[:, None])) <= (2e-15 if form == "f" else 1e-16)
    _, u, _ = o.macros()
    assert np.max(np.abs(u[0] - U_IN)) <= 1e-14 and np.max(np.abs(u[1:])) <= 1e-14


@pytest.mark.parametrize("form", ["f", "h"])
@pytest.mark.parametrize("lat,coll", [("D2Q9", "BGK"), ("D2Q9", "MRT"), ("D3Q19", "MRT")])
def test_slip_planes_are_mirrors(lat, coll, form):
    D3 = lat == "D3Q19"
    nx, ny, nz = (10, 7, 5) if D3 else (12, 9, 1)
    g = (3e-6, 0.0, 1e-6 if D3 else 0.0)
    slip = Oracle(lat, coll, (nx, ny, nz), 0.7, g=g, form=form)
    slip.set_boundaries("periodic", "slip", "periodic")
    dbl = Oracle(lat, coll, (nx, 2 * ny, nz), 0.7, g=g, form=form)
    e, w, _ = slip.lattice_tables()
    Q = len(w)
    mir = [next(k for k in range(Q) if e[k][0] == e[i][0] and e[k][1] == -e[i][1] and e[k][2] == e[i][2])
           for i in range(Q)]
    rng = np.random.default_rng(21)
    x, y, z = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ux = 0.02 * np.cos(np.pi * (y + 0.5) / ny) + 0.003 * np.sin(2 * np.pi * x / nx)
    uy = 0.01 * np.sin(np.pi * (y + 0.5) / ny) * np.cos(2 * np.pi * x / nx)  # zero at both planes
    uz = 0.004 * np.cos(2 * np.pi * z / nz) * np.cos(np.pi * (y + 0.5) / ny) if D3 else 0.0 * ux
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, size=ux.shape)
    f = np.empty((Q, nx, ny, nz))
    for xi in range(nx):
        for yi in range(ny):
            for zi in range(nz):
                f[:, xi, yi, zi] = slip.feq(rho[xi, yi, zi], (ux[xi, yi, zi], uy[xi, yi, zi], uz[xi, yi, zi]))
    # cell order n = x + nx (y + ny z): arrays [Q][nz][ny][nx]
    fs = np.transpose(f, (0, 3, 2, 1)).reshape(Q, -1)
    # doubled box: y in [0, ny) as is, y in [ny, 2 ny) the mirror of y' = 2 ny - 1 - y
    fd = np.empty((Q, nz, 2 * ny, nx))
    fq = np.transpose(f, (0, 3, 2, 1))
    fd[:, :, :ny, :] = fq
    fd[:, :, ny:, :] = fq[mir][:, :, ::-1, :]
    slip.set_f(fs)
    dbl.set_f(fd.reshape(Q, -1))
    slip.step(40)
    dbl.step(40)
    a = slip.get_f().reshape(Q, nz, ny, nx)
    b = dbl.get_f().reshape(Q, nz, 2 * ny, nx)
    assert np.max(np.abs(a - b[:, :, :ny, :])) <= 1e-14
    assert np.max(np.abs(b[:, :, ny:, :] - b[mir][:, :, ny - 1::-1, :])) <= 1e-14  # the doubled run stays mirrored


@pytest.mark.parametrize("form", ["f", "h"])
def test_inlet_outlet_mass_balance(form):
    """Per step: mass(t+1) = mass(t) + U A (inlet) - what the last layer's
    post-collision populations carry out + what the outflow condition sets
    entering there (collisions conserve mass; reflections and streaming move
    it)."""
    nx, ny, nz = 16, 8, 7
    g = (2e-5, 0.0, 0.0)
    o = Oracle("D3Q19", "MRT", (nx, ny, nz), 0.8, g=g, g_fluid_only=False, form=form)
    o.set_boundaries("open", "slip", "slip", inflow=U_IN)
    e, w, _ = o.lattice_tables()
    Q = len(w)
    out_dirs = [i for i in range(Q) if e[i][0] > 0]
    in_dirs = [i for i in range(Q) if e[i][0] < 0]
    for step in range(25):  # from rest: the inflow accelerates the box
        f0 = o.get_f().reshape(Q, nz, ny, nx)
        o.step(1)
        f1 = o.get_f().reshape(Q, nz, ny, nx)
        leaving = 0.0
        for z in range(nz):
            for y in range(ny):
                post = o.collide_node(f0[:, z, y, nx - 1], g)
                leaving += sum(post[i] for i in out_dirs)
        entering = sum(f1[i, :, :, nx - 1].sum() for i in in_dirs)
        balance = f1.sum() - f0.sum() - U_IN * ny * nz + leaving - entering
        assert abs(balance) <= 1e-12, (step, balance)
