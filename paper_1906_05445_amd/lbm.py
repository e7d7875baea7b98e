"""ctypes binding of liblbm.so (include/lbm.h), argument marshalling only.

Every function named ``lbm_*`` here calls the C entry point of the same name;
all computation happens in the HIP library.  PyTorch provides the device
workspace and the stream.  If the library is missing this module raises at
import: there is no fallback path.

``Lattice`` is a small owner object: it allocates the workspace tensor,
creates the context and exposes numpy views of the readouts.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1906_05445_amd/build.py (no fallback exists)")

# torch ships its own HIP runtime (SONAME libamdhip64.so.7).  Loading torch
# first makes liblbm.so bind to that same runtime instead of pulling in a
# second copy (with a second HSA runtime) from /opt/rocm.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EDIVERGED, LBM_EUNSUPPORTED, LBM_ESTATE, LBM_EAGAIN = \
    0, -1, -2, -3, -4, -5, -6, -7
LATTICES = {"D2Q9": 0, "D3Q19": 1}
COLLISIONS = {"BGK": 0, "MRT": 1}
STORAGES = {"F64": 0, "F32": 1, "F16": 2, "F16_SR": 3}
METHODS = {"BB": 0, "LINEAR": 1, "QUADRATIC": 2, "IBM": 3, "YU": 4, "ZHAO_YONG": 5}
KINDS = {"sphere": 0, "cylinder": 1, "plane": 2}
STORAGE_DTYPES = {0: np.float64, 1: np.float32, 2: np.float16, 3: np.float16}


class lbm_params(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("collision", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("tau", ctypes.c_double), ("rates", ctypes.POINTER(ctypes.c_double)),
                ("body_force", ctypes.c_double * 3), ("body_force_fluid_only", ctypes.c_int32),
                ("boundary", ctypes.c_int32 * 3), ("inflow", ctypes.c_double), ("cover_momentum", ctypes.c_int32)]


class lbm_solid(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("inverted", ctypes.c_int32), ("centre", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("axis", ctypes.c_double * 3), ("velocity", ctypes.c_double * 3),
                ("omega", ctypes.c_double * 3), ("density", ctypes.c_double), ("gravity", ctypes.c_double * 3)]


class lbm_ibm_opts(ctypes.Structure):
    _fields_ = [("n_iter", ctypes.c_int32), ("delta", ctypes.c_int32), ("retraction", ctypes.c_double)]


_vp = ctypes.c_void_p
_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64
_st = ctypes.c_int32


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("lbm_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(lbm_params), ctypes.c_int32, _i64, _i64])
_sig("lbm_create", _st, [ctypes.POINTER(lbm_params), ctypes.c_int32, _i64, _i64, _vp, ctypes.c_size_t, _vp,
                         ctypes.POINTER(_vp)])
_sig("lbm_create_noalloc", _st, [ctypes.POINTER(lbm_params), ctypes.c_int32, _i64, _i64, _vp, ctypes.POINTER(_vp)])
_sig("lbm_noalloc_capacity", ctypes.c_size_t, [])
_sig("lbm_set_solids", _st, [_vp, ctypes.POINTER(lbm_solid), ctypes.c_int32, ctypes.c_int32,
                             ctypes.POINTER(lbm_ibm_opts)])
_sig("lbm_set_lagrangian", _st, [_vp, ctypes.c_int32, _d, _i64, ctypes.c_double])
_sig("lbm_step", _st, [_vp, _i64])
_sig("lbm_force_torque", _st, [_vp, _d, _d])
_sig("lbm_force_history", _st, [_vp, _i64, _i64, _d])
_sig("lbm_history_capacity", _i64, [])
_sig("lbm_macros", _st, [_vp, _d, _d, ctypes.POINTER(ctypes.c_uint8)])
_sig("lbm_strain", _st, [_vp, _d, _d])
_sig("lbm_solid_state", _st, [_vp, _d])
_sig("lbm_get_f", _st, [_vp, _d])
_sig("lbm_set_f", _st, [_vp, _d])
_sig("lbm_set_equilibrium", _st, [_vp, ctypes.c_double, _d])
_sig("lbm_get_state", _st, [_vp, _vp])
_sig("lbm_set_state", _st, [_vp, _vp])
_sig("lbm_link_list", _st, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_uint32),
                            ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32), _d])
_sig("lbm_node_types", _st, [_vp, ctypes.POINTER(ctypes.c_uint8)])
_sig("lbm_time", _i64, [_vp])
_sig("lbm_check", _st, [_vp])
_sig("lbm_destroy", _st, [_vp])
_sig("lbm_status_string", ctypes.c_char_p, [_st])
_sig("lbm_last_error", ctypes.c_char_p, [_vp])
_sig("lbm_copy_probe", _st, [_vp, _vp, ctypes.c_size_t, _vp])
_sig("lbm_profile", _st, [_vp, ctypes.c_int32])
_sig("lbm_profile_read", _st, [_vp, _d, ctypes.POINTER(_i64)])
_sig("lbm_autotune_info", _st, [_vp, ctypes.POINTER(ctypes.c_int32), _d, _d])
_sig("lbm_autotune_policy", _st, [_vp, ctypes.POINTER(ctypes.c_int32), _d])

_sig("lbm_batch_table_bytes", ctypes.c_size_t, [ctypes.c_int32])
_sig("lbm_batch_create", _st, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_size_t, _vp,
                               ctypes.POINTER(_vp)])
_sig("lbm_batch_admit", _st, [_vp, ctypes.POINTER(lbm_params), ctypes.c_int32, _i64, _i64, ctypes.POINTER(_vp)])
_sig("lbm_batch_release", _st, [_vp, _vp])
_sig("lbm_batch_step", _st, [_vp, _i64])
_sig("lbm_batch_sync", _st, [_vp])
_sig("lbm_batch_info", _st, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_size_t),
                             ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_i64)])
_sig("lbm_batch_tune_info", _st, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _d])
_sig("lbm_batch_time_sweep", _st, [_vp, _i64, _d])
_sig("lbm_batch_tune_table", ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32), _d])
_sig("lbm_batch_force_change", _st, [_vp, _i64, ctypes.POINTER(_vp), _d])
_sig("lbm_batch_poll", _st, [_vp, _i64, ctypes.c_double, ctypes.POINTER(_vp), ctypes.c_int32,
                             ctypes.POINTER(ctypes.c_int32)])
_sig("lbm_batch_stream", _vp, [_vp])
_sig("lbm_batch_last_error", ctypes.c_char_p, [_vp])
_sig("lbm_batch_destroy", _st, [_vp])

EXPORTED = ["lbm_workspace_bytes", "lbm_create", "lbm_create_noalloc", "lbm_noalloc_capacity", "lbm_set_solids", "lbm_set_lagrangian", "lbm_step",
            "lbm_force_torque", "lbm_force_history", "lbm_history_capacity", "lbm_macros", "lbm_strain", "lbm_solid_state", "lbm_get_f",
            "lbm_set_f", "lbm_set_equilibrium", "lbm_get_state", "lbm_set_state", "lbm_link_list", "lbm_node_types", "lbm_time",
            "lbm_check", "lbm_destroy", "lbm_status_string", "lbm_last_error", "lbm_copy_probe",
            "lbm_profile", "lbm_profile_read", "lbm_autotune_info", "lbm_autotune_policy", "lbm_batch_table_bytes", "lbm_batch_create",
            "lbm_batch_admit", "lbm_batch_release", "lbm_batch_step", "lbm_batch_sync", "lbm_batch_info",
            "lbm_batch_tune_info", "lbm_batch_tune_table", "lbm_batch_time_sweep", "lbm_batch_force_change", "lbm_batch_poll", "lbm_batch_stream", "lbm_batch_last_error",
            "lbm_batch_destroy"]
globals().update({n: getattr(_lib, n) for n in EXPORTED})


class LBMError(RuntimeError):
    def __init__(self, status, detail=""):
        self.status = status
        msg = _lib.lbm_status_string(status).decode()
        super().__init__(f"{msg} ({status})" + (f": {detail}" if detail else ""))


def _ptr(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


DOMAINS = {"periodic": 0, "slip": 1, "open": 2}


def make_params(lattice="D3Q19", collision="MRT", storage="F64", shape=(16, 16, 16), tau=0.8, rates=None,
                g=(0.0, 0.0, 0.0), g_fluid_only=True, boundary=("periodic", "periodic", "periodic"), inflow=0.0,
                cover_momentum=False):
    """boundary: per axis "periodic", "slip" (stress-free planes) or, on x, "open"
    (velocity inlet `inflow` at x = 0, convective outflow at the last layer): Sec. 3.4."""
    p = lbm_params()
    p.lattice = LATTICES[lattice]
    p.collision = COLLISIONS[collision]
    p.storage = STORAGES[storage]
    nx, ny, nz = (tuple(shape) + (1,))[:3]
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.tau = float(tau)
    keep = None
    if rates is not None:
        keep = np.ascontiguousarray(rates, dtype=np.float64)
        p.rates = _ptr(keep)
    gg = list(g) + [0.0] * (3 - len(g))
    for k in range(3):
        p.body_force[k] = float(gg[k])
    p.body_force_fluid_only = int(bool(g_fluid_only))
    bnd = list(boundary) + ["periodic"] * (3 - len(boundary))
    for k in range(3):
        p.boundary[k] = DOMAINS[bnd[k]]
    p.inflow = float(inflow)
    p.cover_momentum = int(bool(cover_momentum))
    return p, keep


def make_solids(solids):
    arr = (lbm_solid * max(1, len(solids)))()
    for k, s in enumerate(solids):
        arr[k].kind = KINDS[s["kind"]]
        arr[k].inverted = int(bool(s.get("inverted", False)))
        c = list(s.get("centre", (0, 0, 0))) + [0.0] * 3
        ax = list(s.get("axis", (0, 0, 1))) + [0.0] * 3
        v = list(s.get("velocity", (0, 0, 0))) + [0.0] * 3
        w = list(s.get("omega", (0, 0, 0))) + [0.0] * 3
        gr = list(s.get("gravity", (0, 0, 0))) + [0.0] * 3
        for a in range(3):
            arr[k].centre[a] = float(c[a])
            arr[k].axis[a] = float(ax[a])
            arr[k].velocity[a] = float(v[a])
            arr[k].omega[a] = float(w[a])
            arr[k].gravity[a] = float(gr[a])
        arr[k].density = float(s.get("density", 0.0))
        arr[k].radius = float(s.get("radius", 0.0))
    return arr


class _Context:
    """Calls on one context handle (readouts as numpy arrays)."""

    handle = None

    def _describe(self, lattice, params):
        self.params = params
        self.shape = (params.nx, params.ny, params.nz)
        self.N = self.shape[0] * self.shape[1] * self.shape[2]
        self.Q = 9 if lattice == "D2Q9" else 19
        self.storage = params.storage
        self.nsolid = 0

    def _check(self, st):
        if st != LBM_OK:
            raise LBMError(st, _lib.lbm_last_error(self.handle).decode())

    def set_solids(self, solids, method="QUADRATIC", n_iter=5, retraction=0.0, delta=4):
        arr = make_solids(solids)
        opts = lbm_ibm_opts(int(n_iter), int(delta), float(retraction))
        self._check(_lib.lbm_set_solids(self.handle, arr, len(solids), METHODS[method], ctypes.byref(opts)))
        self.nsolid = len(solids)

    def set_lagrangian(self, sid, X, dV):
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 3)
        self._check(_lib.lbm_set_lagrangian(self.handle, int(sid), _ptr(X), X.shape[0], float(dV)))

    def step(self, n=1):
        self._check(_lib.lbm_step(self.handle, int(n)))

    @property
    def time(self):
        return _lib.lbm_time(self.handle)

    def force_torque(self):
        F = np.zeros((max(self.nsolid, 1), 3))
        T = np.zeros((max(self.nsolid, 1), 3))
        self._check(_lib.lbm_force_torque(self.handle, _ptr(F), _ptr(T)))
        return np.concatenate([F, T], axis=1)[: self.nsolid]

    def history(self, first=None, count=None):
        """Per-step force/torque [count][nsolid][6]; by default every step still in the ring."""
        if first is None:
            first = max(0, self.time - int(_lib.lbm_history_capacity()))
        if count is None:
            count = self.time - first
        out = np.zeros((max(count, 1), max(self.nsolid, 1), 6))
        self._check(_lib.lbm_force_history(self.handle, int(first), int(count), _ptr(out)))
        return out[:count, : self.nsolid]

    def macros(self):
        rho = np.empty(self.N)
        u = np.empty((3, self.N))
        t = np.empty(self.N, dtype=np.uint8)
        self._check(_lib.lbm_macros(self.handle, _ptr(rho), _ptr(u), _ptr(t, ctypes.c_uint8)))
        return rho, u, t

    def solid_state(self):
        """[n][9]: centre, velocity and angular velocity of every solid now."""
        out = np.zeros((max(self.nsolid, 1), 9))
        self._check(_lib.lbm_solid_state(self.handle, _ptr(out)))
        return out[: self.nsolid]

    def strain(self):
        """Strain rate [6][N] (xx, yy, zz, xy, yz, xz) and dissipation [N] of the last collision (Eq. 19)."""
        S = np.empty((6, self.N))
        eps = np.empty(self.N)
        self._check(_lib.lbm_strain(self.handle, _ptr(S), _ptr(eps)))
        return S, eps

    def get_f(self):
        f = np.empty((self.Q, self.N))
        self._check(_lib.lbm_get_f(self.handle, _ptr(f)))
        return f

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.Q, self.N)
        self._check(_lib.lbm_set_f(self.handle, _ptr(f)))

    def set_equilibrium(self, rho=1.0, u=(0.0, 0.0, 0.0)):
        """Uniform flow f = f_eq(rho, u) everywhere (lbm_set_equilibrium)."""
        uu = np.ascontiguousarray((list(u) + [0.0, 0.0, 0.0])[:3], dtype=np.float64)
        self._check(_lib.lbm_set_equilibrium(self.handle, float(rho), _ptr(uu)))

    def get_state(self):
        out = np.empty((self.Q, self.N), dtype=STORAGE_DTYPES[self.storage])
        self._check(_lib.lbm_get_state(self.handle, out.ctypes.data_as(_vp)))
        return out

    def set_state(self, h):
        h = np.ascontiguousarray(h, dtype=STORAGE_DTYPES[self.storage]).reshape(self.Q, self.N)
        self._check(_lib.lbm_set_state(self.handle, h.ctypes.data_as(_vp)))

    def links(self):
        n = _i64(0)
        self._check(_lib.lbm_link_list(self.handle, ctypes.byref(n), None, None, None, None))
        m = max(n.value, 1)
        cell = np.zeros(m, dtype=np.uint32)
        d = np.zeros(m, dtype=np.uint8)
        sid = np.zeros(m, dtype=np.int32)
        q = np.zeros(m)
        cnt = _i64(m)
        self._check(_lib.lbm_link_list(self.handle, ctypes.byref(cnt), _ptr(cell, ctypes.c_uint32),
                                       _ptr(d, ctypes.c_uint8), _ptr(sid, ctypes.c_int32), _ptr(q)))
        k = cnt.value
        return {"cell": cell[:k].astype(np.int64), "dir": d[:k].astype(np.int32), "sid": sid[:k], "q": q[:k]}

    def node_types(self):
        t = np.empty(self.N, dtype=np.uint8)
        self._check(_lib.lbm_node_types(self.handle, _ptr(t, ctypes.c_uint8)))
        return t

    def check(self):
        st = _lib.lbm_check(self.handle)
        if st not in (LBM_OK, LBM_EDIVERGED):
            self._check(st)
        return st == LBM_OK


class Lattice(_Context):
    """One lattice on the current CUDA/HIP device, owning its workspace."""

    def __init__(self, lattice="D3Q19", collision="MRT", storage="F64", shape=(16, 16, 16), tau=0.8, rates=None,
                 g=(0.0, 0.0, 0.0), g_fluid_only=True, max_solids=1, max_links=0, max_lagrangian=0,
                 stream=None, device="cuda", boundary=("periodic", "periodic", "periodic"), inflow=0.0,
                 cover_momentum=False):
        import torch
        self._torch = torch
        params, self._rates = make_params(lattice, collision, storage, shape, tau, rates, g, g_fluid_only,
                                          boundary, inflow, cover_momentum)
        self._describe(lattice, params)
        nbytes = _lib.lbm_workspace_bytes(ctypes.byref(self.params), max_solids, max_links, max_lagrangian)
        if nbytes == 0:
            raise LBMError(LBM_EINVAL, "lattice parameters rejected")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = _vp()
        st = _lib.lbm_create(ctypes.byref(self.params), max_solids, max_links, max_lagrangian, _vp(aligned),
                             nbytes, _vp(self.stream.cuda_stream), ctypes.byref(h))
        if st != LBM_OK:
            raise LBMError(st, "lbm_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _lib.lbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable=True, every=1):
        """Time every `every`-th stream-collide launch with HIP events (enable=False: stop)."""
        self._check(_lib.lbm_profile(self.handle, int(every) if enable else 0))

    def profile_read(self):
        """(summed stream-collide milliseconds, launches) since the last read."""
        ms = ctypes.c_double(0.0)
        n = _i64(0)
        self._check(_lib.lbm_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def autotune_info(self):
        nt = ctypes.c_int32(-1)
        a, b = ctypes.c_double(0.0), ctypes.c_double(0.0)
        self._check(_lib.lbm_autotune_info(self.handle, ctypes.byref(nt), ctypes.byref(a), ctypes.byref(b)))
        pol = ctypes.c_int32(-1)
        us = (ctypes.c_double * 4)()
        self._check(_lib.lbm_autotune_policy(self.handle, ctypes.byref(pol), us))
        names = ["plain_linear", "nontemporal_linear", "plain_xcd", "nontemporal_xcd"]
        return {"nontemporal_stores": nt.value, "sweep_us_plain": a.value, "sweep_us_nontemporal": b.value,
                "policy": names[pol.value] if pol.value >= 0 else None,
                "sweep_us": {names[k]: us[k] for k in range(4)}}


class StaticLattice(_Context):
    """One lattice whose workspace is the library's static device array
    (lbm_create_noalloc): no device memory is allocated for it.  One per
    device at a time."""

    def __init__(self, lattice="D3Q19", collision="MRT", storage="F64", shape=(16, 16, 16), tau=0.8, rates=None,
                 g=(0.0, 0.0, 0.0), g_fluid_only=True, max_solids=1, max_links=0, max_lagrangian=0, stream=None):
        import torch
        params, self._rates = make_params(lattice, collision, storage, shape, tau, rates, g, g_fluid_only)
        self._describe(lattice, params)
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = _vp()
        st = _lib.lbm_create_noalloc(ctypes.byref(self.params), max_solids, max_links, max_lagrangian,
                                     _vp(self.stream.cuda_stream), ctypes.byref(h))
        if st != LBM_OK:
            raise LBMError(st, "lbm_create_noalloc")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _lib.lbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Member(_Context):
    """A lattice admitted into a Batch (its workspace lives in the batch pool)."""

    def __init__(self, batch, handle, lattice, params, rates_keep):
        self.batch = batch
        self.handle = handle
        self._rates = rates_keep
        self._describe(lattice, params)


class Batch:
    """Many lattices of one lattice type and storage advanced together
    (lbm_batch_*); the pool is a torch tensor owned by this object."""

    def __init__(self, lattice="D3Q19", storage="F32", max_slots=64, pool_bytes=1 << 30, device="cuda",
                 stream=None):
        import torch
        self._torch = torch
        self.lattice = lattice
        self.pool = torch.empty(int(pool_bytes) + 256, dtype=torch.uint8, device=device)
        aligned = (self.pool.data_ptr() + 255) // 256 * 256
        # the caller's stream (a torch stream of default priority unless one is given):
        # batched steps are captured as graphs on it, so it is never the null stream
        self.stream = torch.cuda.Stream() if stream is None else stream
        h = _vp()
        st = _lib.lbm_batch_create(LATTICES[lattice], STORAGES[storage], int(max_slots), _vp(aligned),
                                   int(pool_bytes), _vp(self.stream.cuda_stream), ctypes.byref(h))
        if st != LBM_OK:
            raise LBMError(st, "lbm_batch_create")
        self.handle = h
        self.max_slots = int(max_slots)
        self.members = []

    def _check(self, st):
        if st != LBM_OK:
            raise LBMError(st, _lib.lbm_batch_last_error(self.handle).decode())

    @staticmethod
    def footprint(lattice="D3Q19", collision="MRT", storage="F32", shape=(16, 16, 16), tau=0.8, max_solids=1,
                  max_links=0, max_lagrangian=0):
        p, _ = make_params(lattice, collision, storage, shape, tau)
        return int(_lib.lbm_workspace_bytes(ctypes.byref(p), max_solids, max_links, max_lagrangian))

    def admit(self, collision="MRT", storage="F32", shape=(16, 16, 16), tau=0.8, rates=None, g=(0.0, 0.0, 0.0),
              g_fluid_only=True, max_solids=1, max_links=0, max_lagrangian=0,
              boundary=("periodic", "periodic", "periodic"), inflow=0.0, cover_momentum=False):
        """A new Member, or None when the pool or the slots are full (LBM_EAGAIN)."""
        params, keep = make_params(self.lattice, collision, storage, shape, tau, rates, g, g_fluid_only,
                                   boundary, inflow, cover_momentum)
        h = _vp()
        st = _lib.lbm_batch_admit(self.handle, ctypes.byref(params), int(max_solids), int(max_links),
                                  int(max_lagrangian), ctypes.byref(h))
        if st == LBM_EAGAIN:
            return None
        self._check(st)
        m = Member(self, h, self.lattice, params, keep)
        self.members.append(m)
        return m

    def release(self, m):
        self._check(_lib.lbm_batch_release(self.handle, m.handle))
        m.handle = None
        self.members.remove(m)

    def step(self, n=1):
        self._check(_lib.lbm_batch_step(self.handle, int(n)))

    def sync(self):
        self._check(_lib.lbm_batch_sync(self.handle))

    def info(self):
        n = ctypes.c_int32(0)
        fr, big = ctypes.c_size_t(0), ctypes.c_size_t(0)
        cells = _i64(0)
        self._check(_lib.lbm_batch_info(self.handle, ctypes.byref(n), ctypes.byref(fr), ctypes.byref(big),
                                        ctypes.byref(cells)))
        return {"members": n.value, "bytes_free": fr.value, "largest_free": big.value, "cells": cells.value}

    def tune_info(self):
        nt, order, blocks, tpb = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        us = ctypes.c_double(0.0)
        st = _lib.lbm_batch_tune_info(self.handle, ctypes.byref(nt), ctypes.byref(order), ctypes.byref(blocks),
                                      ctypes.byref(tpb), ctypes.byref(us))
        if st == LBM_ESTATE:
            return None
        self._check(st)
        return {"nontemporal_stores": nt.value, "order": order.value, "blocks": blocks.value,
                "tiles_per_block": tpb.value, "sweep_us": us.value}

    def force_change(self, lag=100):
        """{Member: relative force change over `lag` steps} (-1: not available yet)."""
        cap = len(self._slots_buf) if hasattr(self, "_slots_buf") else 0
        if cap != self.max_slots:
            self._slots_buf = (_vp * self.max_slots)()
            self._change_buf = np.empty(self.max_slots)
        self._check(_lib.lbm_batch_force_change(self.handle, int(lag), self._slots_buf, _ptr(self._change_buf)))
        by_handle = {m.handle.value: m for m in self.members}
        out = {}
        for k in range(self.max_slots):
            h = self._slots_buf[k]
            if h and h in by_handle:
                out[by_handle[h]] = float(self._change_buf[k])
        return out

    def poll(self, lag=100, tol=1e-6):
        """Members whose relative force change over `lag` steps is below tol (lbm_batch_poll)."""
        buf = (_vp * self.max_slots)()
        n = ctypes.c_int32(0)
        self._check(_lib.lbm_batch_poll(self.handle, int(lag), float(tol), buf, self.max_slots, ctypes.byref(n)))
        by_handle = {m.handle.value: m for m in self.members}
        return [by_handle[buf[k]] for k in range(min(n.value, self.max_slots)) if buf[k] in by_handle]

    def tune_table(self):
        """Every sweep candidate of the tuner with its measured time (us; -1 before tuning)."""
        n = _lib.lbm_batch_tune_table(self.handle, 0, None, None, None, None, None)
        nt = (ctypes.c_int32 * n)()
        order = (ctypes.c_int32 * n)()
        blocks = (ctypes.c_int32 * n)()
        tpb = (ctypes.c_int32 * n)()
        us = np.zeros(n)
        _lib.lbm_batch_tune_table(self.handle, n, nt, order, blocks, tpb, _ptr(us))
        return [{"nontemporal_stores": nt[k], "order": order[k], "blocks": blocks[k], "tiles_per_block": tpb[k],
                 "sweep_us": float(us[k])} for k in range(n)]

    def time_sweep(self, n):
        us = ctypes.c_double(0.0)
        self._check(_lib.lbm_batch_time_sweep(self.handle, int(n), ctypes.byref(us)))
        return us.value

    def close(self):
        if getattr(self, "handle", None):
            _lib.lbm_batch_destroy(self.handle)
            self.handle = None
            for m in self.members:
                m.handle = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
