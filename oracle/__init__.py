"""FP64 CPU oracle of the lattice Boltzmann hot path (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never links, loads or
calls it, and it shares no code with the GPU library.  The arithmetic lives
in ``lbm_oracle.c`` (plain C, FP64, compiled without floating-point
contraction); this module only marshals arguments through ctypes.

Solids are described by plain dicts, the same ones the GPU binding accepts::

    {"kind": "sphere" | "cylinder" | "plane", "inverted": bool,
     "centre": (x, y, z), "radius": R, "axis": (ax, ay, az),
     "velocity": (Ux, Uy, Uz), "omega": (Wx, Wy, Wz)}

``axis`` is the cylinder axis or, for a plane, its unit normal pointing into
the fluid; both must be coordinate axes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_SO = os.path.join(_HERE, "liblbm_oracle.so")

LATTICES = {"D2Q9": 0, "D3Q19": 1}
COLLISIONS = {"BGK": 0, "MRT": 1}
METHODS = {"BB": 0, "LINEAR": 1, "QUADRATIC": 2, "IBM": 3, "YU": 4, "ZHAO_YONG": 5}
KINDS = {"sphere": 0, "cylinder": 1, "plane": 2}


def build() -> str:
    """Compile the oracle into ``oracle/liblbm_oracle.so``."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
           "-o", _SO, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _SO


_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i = ctypes.POINTER(ctypes.c_int)
_l = ctypes.POINTER(ctypes.c_long)
_u8 = ctypes.POINTER(ctypes.c_uint8)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, _d, _d, ctypes.c_int]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_set_solids.argtypes = [ctypes.c_void_p, ctypes.c_int, _i, _i, _d, _d, _i, _i, _d, _d,
                                     ctypes.c_int]
        L.orc_set_lagrangian.argtypes = [ctypes.c_void_p, ctypes.c_int, _d, ctypes.c_long, ctypes.c_double]
        L.orc_clear_lagrangian.argtypes = [ctypes.c_void_p]
        L.orc_set_ibm_iters.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.orc_cells.argtypes = [ctypes.c_void_p]
        L.orc_cells.restype = ctypes.c_long
        L.orc_q.argtypes = [ctypes.c_void_p]
        L.orc_time.argtypes = [ctypes.c_void_p]
        L.orc_time.restype = ctypes.c_long
        L.orc_get_f.argtypes = [ctypes.c_void_p, _d]
        L.orc_set_f.argtypes = [ctypes.c_void_p, _d]
        L.orc_get_h.argtypes = [ctypes.c_void_p, _d]
        L.orc_set_h.argtypes = [ctypes.c_void_p, _d]
        L.orc_get_rates.argtypes = [ctypes.c_void_p, _d]
        L.orc_get_mrt.argtypes = [ctypes.c_void_p, _d, _d]
        L.orc_lattice.argtypes = [ctypes.c_void_p, _i, _d, _i]
        L.orc_feq.argtypes = [ctypes.c_void_p, ctypes.c_double, _d, _d]
        L.orc_forcing.argtypes = [ctypes.c_void_p, _d, _d, _d]
        L.orc_collide_node.argtypes = [ctypes.c_void_p, _d, _d, _d]
        L.orc_macros.argtypes = [ctypes.c_void_p, _d, _d, _u8]
        L.orc_force_torque.argtypes = [ctypes.c_void_p, _d]
        L.orc_history_len.argtypes = [ctypes.c_void_p]
        L.orc_history_len.restype = ctypes.c_long
        L.orc_history.argtypes = [ctypes.c_void_p, _d]
        L.orc_link_count.argtypes = [ctypes.c_void_p]
        L.orc_link_count.restype = ctypes.c_long
        L.orc_links.argtypes = [ctypes.c_void_p, _l, _i, _i, _d, _i, _i]
        L.orc_node_flags.argtypes = [ctypes.c_void_p, _u8, _u8, _i]
        L.orc_ibm_force_field.argtypes = [ctypes.c_void_p, _d]
        L.orc_lagrangian_force.argtypes = [ctypes.c_void_p, _d]
        L.orc_interpolate.argtypes = [ctypes.c_void_p, _d, _d]
        L.orc_spread.argtypes = [ctypes.c_void_p, _d, _d]
        L.orc_phi.argtypes = [ctypes.c_double]
        L.orc_phi.restype = ctypes.c_double
        L.orc_phi_n.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_phi_n.restype = ctypes.c_double
        L.orc_set_ibm_delta.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_set_ibm_inner.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_kempe_volume.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_kempe_volume.restype = ctypes.c_double
        L.orc_kempe_inner.argtypes = [ctypes.c_void_p, ctypes.c_int, _d]
        L.orc_strain.argtypes = [ctypes.c_void_p, _d, _d]
        L.orc_set_form.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_form.argtypes = [ctypes.c_void_p]
        L.orc_set_threads.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_set_boundaries.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.orc_set_cover.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_set_free.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _d]
        L.orc_solid_state.argtypes = [ctypes.c_void_p, _d]
        L.orc_ibb_value.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int] + \
            [ctypes.c_double] * 7
        L.orc_ibb_value.restype = ctypes.c_double
        L.orc_zhao_yong_value.argtypes = [ctypes.c_double] * 4
        L.orc_zhao_yong_value.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a, t=_d):
    return a.ctypes.data_as(t)


def zhao_yong_value(q, fi_post, fb_pre, B):
    """Unknown population of one boundary link by Zhao & Yong's scheme, Eq. 16."""
    return lib().orc_zhao_yong_value(float(q), float(fi_post), float(fb_pre), float(B))


def phi_n(points: int, r: float) -> float:
    """Delta function factor: 4 points (Eq. 6), 3 points (Roma et al.) or 2 points (linear)."""
    return lib().orc_phi_n(int(points), float(r))


def phi(r: float) -> float:
    """Peskin's 4-point delta factor, Eq. 6."""
    return lib().orc_phi(float(r))


def ibb_value(method, q, ff_ok, fff_ok, fb_f, fb_ff, fb_fff, fs_f, fi_ff_new, fi_fff_new, B):
    """Unknown population of one boundary link (Eq. 10, Eq. 11, Eq. 12-14, linear Bouzidi)."""
    return lib().orc_ibb_value(METHODS[method] if isinstance(method, str) else int(method), float(q),
                               int(ff_ok), int(fff_ok), float(fb_f), float(fb_ff), float(fb_fff),
                               float(fs_f), float(fi_ff_new), float(fi_fff_new), float(B))


def _axis_index(axis):
    a = np.asarray(axis, dtype=np.float64)
    k = int(np.argmax(np.abs(a)))
    return k, (1 if a[k] > 0 else -1)


class Oracle:
    """One periodic lattice stepped by the FP64 oracle.

    form: "f" stores the populations themselves, the equations as written
    (the default); "h" stores their deviations from the rest state, the same
    step with three decades less rounding (the two are pinned against each
    other in tests/test_oracle_forms.py).  threads: threads of the per-cell
    loops (results do not depend on it)."""

    def __init__(self, lattice="D3Q19", collision="MRT", shape=(16, 16, 16), tau=0.8, rates=None,
                 g=(0.0, 0.0, 0.0), g_fluid_only=True, form="f", threads=1):
        nx, ny, nz = (tuple(shape) + (1,))[:3] if len(shape) == 2 else tuple(shape)
        self.shape = (nx, ny, nz)
        self.lattice = lattice
        self.Q = 9 if lattice == "D2Q9" else 19
        r = None if rates is None else np.ascontiguousarray(rates, dtype=np.float64)
        gg = np.ascontiguousarray(g, dtype=np.float64)
        if gg.size == 2:
            gg = np.append(gg, 0.0)
        h = lib().orc_create(LATTICES[lattice], COLLISIONS[collision], nx, ny, nz, float(tau),
                             None if r is None else _p(r), _p(gg), int(bool(g_fluid_only)))
        if not h:
            raise ValueError("oracle rejected the lattice parameters")
        self._h = ctypes.c_void_p(h)
        if form not in ("f", "h"):
            raise ValueError(form)
        self.form = form
        lib().orc_set_form(self._h, 1 if form == "f" else 0)
        lib().orc_set_threads(self._h, int(threads))
        self.N = nx * ny * nz
        self.nsolid = 0
        self.nlag = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    # -- configuration -----------------------------------------------------
    def set_solids(self, solids, method="QUADRATIC"):
        n = len(solids)
        kind = np.array([KINDS[s["kind"]] for s in solids] or [0], dtype=np.int32)
        inv = np.array([int(bool(s.get("inverted", False))) for s in solids] or [0], dtype=np.int32)
        cen = np.array([list(s.get("centre", (0, 0, 0)))[:3] + [0.0] * (3 - len(s.get("centre", (0, 0, 0))))
                        for s in solids] or [[0, 0, 0]], dtype=np.float64)
        rad = np.array([float(s.get("radius", 0.0)) for s in solids] or [0.0], dtype=np.float64)
        axs = [_axis_index(s.get("axis", (0, 0, 1))) for s in solids] or [(2, 1)]
        ax = np.array([a for a, _ in axs], dtype=np.int32)
        sg = np.array([b for _, b in axs], dtype=np.int32)
        U = np.array([list(s.get("velocity", (0, 0, 0))) for s in solids] or [[0, 0, 0]], dtype=np.float64)
        W = np.array([list(s.get("omega", (0, 0, 0))) for s in solids] or [[0, 0, 0]], dtype=np.float64)
        st = lib().orc_set_solids(self._h, n, _p(kind, _i), _p(inv, _i), _p(cen), _p(rad), _p(ax, _i),
                                  _p(sg, _i), _p(U), _p(W), METHODS[method])
        if st != 0:
            raise ValueError(f"oracle rejected the solids (status {st})")
        self.nsolid = n
        lib().orc_clear_lagrangian(self._h)
        self.nlag = 0
        for k, s in enumerate(solids):  # free solids (a "density" entry, as the GPU binding reads it)
            if float(s.get("density", 0.0)) != 0.0:
                self.set_free(k, s["density"], s.get("gravity", (0.0, 0.0, 0.0)))

    def set_lagrangian(self, sid, X, dV):
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 3)
        lib().orc_set_lagrangian(self._h, int(sid), _p(X), X.shape[0], float(dV))
        self.nlag += X.shape[0]

    def set_ibm_iters(self, n_iter):
        lib().orc_set_ibm_iters(self._h, int(n_iter))

    def set_ibm_inner(self, mode):
        """Inner-fluid treatment of free IBM solids: "FENG" (Eq. 23) or "KEMPE" (Eq. 24-26)."""
        if lib().orc_set_ibm_inner(self._h, {"FENG": 0, "KEMPE": 1}[mode]) != 0:
            raise ValueError("inner-fluid mode")

    def kempe_volume(self, k):
        return lib().orc_kempe_volume(self._h, int(k))

    def kempe_inner(self, k):
        out = np.zeros(6)
        lib().orc_kempe_inner(self._h, int(k), _p(out))
        return out

    def set_ibm_delta(self, points):
        """Delta function of the IBM: 4 (Eq. 6, default), 3 (Roma et al.) or 2 (linear)."""
        if lib().orc_set_ibm_delta(self._h, int(points)) != 0:
            raise ValueError(points)

    # -- stepping ------------------------------------------------------------
    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    @property
    def time(self):
        return lib().orc_time(self._h)

    # -- state ---------------------------------------------------------------
    def get_f(self):
        out = np.empty((self.Q, self.N), dtype=np.float64)
        lib().orc_get_f(self._h, _p(out))
        return out

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.Q, self.N)
        lib().orc_set_f(self._h, _p(f))

    def set_threads(self, n):
        lib().orc_set_threads(self._h, int(n))

    def set_cover(self, on=True):
        """Covering / uncovering momentum of moving bounce-back solids: a node the
        solid covers gives its momentum to the solid, a node it uncovers (refilled at
        the wall velocity) takes its momentum from it; added to the next step's force."""
        lib().orc_set_cover(self._h, int(bool(on)))

    BCS = {"periodic": 0, "slip": 1, "open": 2}

    def set_boundaries(self, x="periodic", y="periodic", z="periodic", inflow=0.0):
        """Domain boundaries of Sec. 3.4 per axis: "periodic", "slip" (stress-free planes
        halfway outside the first and last layers) or, on x only, "open" (velocity inlet
        `inflow` before x = 0, convective outflow at the last layer)."""
        if lib().orc_set_boundaries(self._h, self.BCS[x], self.BCS[y], self.BCS[z], float(inflow)) != 0:
            raise ValueError((x, y, z))

    def get_h(self):
        """Deviations h = f - w (exact in the "h" form)."""
        out = np.empty((self.Q, self.N), dtype=np.float64)
        lib().orc_get_h(self._h, _p(out))
        return out

    def set_h(self, h):
        h = np.ascontiguousarray(h, dtype=np.float64).reshape(self.Q, self.N)
        lib().orc_set_h(self._h, _p(h))

    def macros(self):
        rho = np.empty(self.N)
        u = np.empty((3, self.N))
        t = np.empty(self.N, dtype=np.uint8)
        lib().orc_macros(self._h, _p(rho), _p(u), _p(t, _u8))
        return rho, u, t

    def force_torque(self):
        out = np.zeros((max(self.nsolid, 1), 6))
        lib().orc_force_torque(self._h, _p(out))
        return out[: self.nsolid]

    def history(self):
        n = lib().orc_history_len(self._h)
        out = np.zeros((max(n, 1) * max(self.nsolid, 1) * 6,))
        lib().orc_history(self._h, _p(out))
        return out[: n * self.nsolid * 6].reshape(n, self.nsolid, 6)

    def links(self):
        n = lib().orc_link_count(self._h)
        m = max(n, 1)
        cell = np.zeros(m, dtype=np.int64)
        d = np.zeros(m, dtype=np.int32)
        sid = np.zeros(m, dtype=np.int32)
        q = np.zeros(m)
        a = np.zeros(m, dtype=np.int32)
        b = np.zeros(m, dtype=np.int32)
        lib().orc_links(self._h, _p(cell, _l), _p(d, _i), _p(sid, _i), _p(q), _p(a, _i), _p(b, _i))
        return {"cell": cell[:n], "dir": d[:n], "sid": sid[:n], "q": q[:n], "ff_ok": a[:n], "fff_ok": b[:n]}

    def node_flags(self):
        ex = np.empty(self.N, dtype=np.uint8)
        ins = np.empty(self.N, dtype=np.uint8)
        own = np.empty(self.N, dtype=np.int32)
        lib().orc_node_flags(self._h, _p(ex, _u8), _p(ins, _u8), _p(own, _i))
        return ex, ins, own

    def ibm_force_field(self):
        out = np.empty((3, self.N))
        lib().orc_ibm_force_field(self._h, _p(out))
        return out

    def lagrangian_force(self):
        out = np.zeros((max(self.nlag, 1), 3))
        lib().orc_lagrangian_force(self._h, _p(out))
        return out[: self.nlag]

    # -- pieces for the pins --------------------------------------------------
    def lattice_tables(self):
        e = np.zeros((self.Q, 3), dtype=np.int32)
        w = np.zeros(self.Q)
        opp = np.zeros(self.Q, dtype=np.int32)
        lib().orc_lattice(self._h, _p(e, _i), _p(w), _p(opp, _i))
        return e, w, opp

    def rates(self):
        out = np.zeros(self.Q)
        lib().orc_get_rates(self._h, _p(out))
        return out

    def mrt_matrices(self):
        M = np.zeros((self.Q, self.Q))
        Mi = np.zeros((self.Q, self.Q))
        lib().orc_get_mrt(self._h, _p(M), _p(Mi))
        return M, Mi

    def feq(self, rho, u):
        u = np.ascontiguousarray(list(u) + [0.0] * (3 - len(u)), dtype=np.float64)
        out = np.zeros(self.Q)
        lib().orc_feq(self._h, float(rho), _p(u), _p(out))
        return out

    def forcing(self, u, F):
        u = np.ascontiguousarray(list(u) + [0.0] * (3 - len(u)), dtype=np.float64)
        F = np.ascontiguousarray(list(F) + [0.0] * (3 - len(F)), dtype=np.float64)
        out = np.zeros(self.Q)
        lib().orc_forcing(self._h, _p(u), _p(F), _p(out))
        return out

    def collide_node(self, fin, F=(0.0, 0.0, 0.0)):
        fin = np.ascontiguousarray(fin, dtype=np.float64)
        F = np.ascontiguousarray(list(F) + [0.0] * (3 - len(F)), dtype=np.float64)
        out = np.zeros(self.Q)
        lib().orc_collide_node(self._h, _p(fin), _p(F), _p(out))
        return out

    def set_free(self, k, density, gravity=(0.0, 0.0, 0.0)):
        """Make solid k move freely (Eq. 20): density ratio rho_p / rho_f, external acceleration."""
        g = np.asarray(gravity, dtype=np.float64)
        st = lib().orc_set_free(self._h, int(k), float(density), _p(g))
        if st != 0:
            raise ValueError(st)

    def solid_state(self):
        """[n][9]: centre, velocity and angular velocity of every solid now."""
        out = np.zeros((self.nsolid, 9))
        lib().orc_solid_state(self._h, _p(out))
        return out

    def strain(self):
        """Strain rate [6][N] (xx, yy, zz, xy, yz, xz) and dissipation rate [N] of the
        most recent collision, from the non-equilibrium moments (Sec. 3.1, Eq. 19)."""
        S = np.zeros((6, self.N))
        eps = np.zeros(self.N)
        if lib().orc_strain(self._h, _p(S), _p(eps)) != 0:
            raise RuntimeError("no collision yet")
        return S, eps

    def interpolate(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, self.N)
        out = np.zeros((max(self.nlag, 1), 3))
        lib().orc_interpolate(self._h, _p(u), _p(out))
        return out[: self.nlag]

    def spread(self, F):
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(-1, 3)
        out = np.zeros((3, self.N))
        lib().orc_spread(self._h, _p(F), _p(out))
        return out
