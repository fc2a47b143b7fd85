"""ctypes binding of the C interface in ``include/sel.h``.

Argument marshalling only: every step of the method runs in the HIP library
``lib/libsel.so``. PyTorch supplies the device workspace (one uint8 tensor)
and the HIP stream. Loading fails loudly when the library has not been built
(``python -m paper_2509_19171_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libsel.so")

SEL_OK = 0
SEL_EINVAL = -1
SEL_ENOMEM = -2
SEL_EDEVICE = -3
SEL_ENONFINITE = -4
SEL_ESTATE = -5
SEL_EUNSUPPORTED = -6
ERR_NAMES = {0: "SEL_OK", -1: "SEL_EINVAL", -2: "SEL_ENOMEM", -3: "SEL_EDEVICE", -4: "SEL_ENONFINITE",
             -5: "SEL_ESTATE", -6: "SEL_EUNSUPPORTED"}

SEL_FP64 = 0
SEL_FP32_DEV = 1
PRECISIONS = {"fp64": SEL_FP64, "fp32dev": SEL_FP32_DEV}
FILTERS = {None: 0, "none": 0, "quad": 1, "exp": 2}
RKS = {"ssprk3": 0, "printed4": 1}
OPS = {"rhs": 0, "rhs_local": 1, "collide": 2, "filter": 3}


class SelError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class sel_params(ctypes.Structure):
    _fields_ = [("Q", ctypes.c_int32), ("precision", ctypes.c_int32), ("rk", ctypes.c_int32),
                ("filter_type", ctypes.c_int32), ("filter_kc", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("filter_amp", ctypes.c_double), ("filter_order", ctypes.c_double), ("rho0", ctypes.c_double),
                ("nu", ctypes.c_double), ("dt", ctypes.c_double), ("accel", ctypes.c_double * 3),
                ("closure", ctypes.c_void_p), ("closure_len", ctypes.c_int64)]


_lib = None


def load():
    """Load ``libsel.so``; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2509_19171_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sigs = {
        "sel_mesh_create": [I32, I32, I64, P, P, P, I32, P, P],
        "sel_mesh_create_dg": [I32, I32, I64, P, P, P, I32, P, P],
        "sel_mesh_destroy": [P],
        "sel_mesh_info": [P, P],
        "sel_workspace_bytes": [P, P, P],
        "sel_init": [P, P, P, P, P, SZ, P, P],
        "sel_step": [P, I64],
        "sel_step_timed": [P, I64, P, P],
        "sel_sync": [P],
        "sel_moments": [P, P, P],
        "sel_moments_device": [P, P, P],
        "sel_reduce": [P, P],
        "sel_get_f": [P, P],
        "sel_set_f": [P, P],
        "sel_set_force": [P, P],
        "sel_velocity_gradient": [P, P],
        "sel_get_time": [P, P, P],
        "sel_radial_profile": [P, P, P, ctypes.c_double, I32, P],
        "sel_apply": [P, I32, P, P],
        "sel_geometry": [P, P, P],
        "sel_destroy": [P],
        "sel_closure_set": [P, P, I64],
        "sel_closure_features": [P, P],
        "sel_closure_dtau": [P, P],
        "sel_coarse_grain": [P, P],
        "sel_closure_targets": [P, P, P],
        "sel_mlp_forward": [P, P, I64, ctypes.c_double, P, P, P],
        "sel_mlp_gradient": [P, P, P, P, I64, P, P, P, P],
        "sel_mlp_train_step": [P, P, P, P, P, P, I64, I64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, P, P, P],
        "sel_mlp_train_step_noalloc": [P, P, P, P, P, P, I64, I64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, P, P],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.sel_last_error.restype = ctypes.c_char_p
    lib.sel_last_error.argtypes = []
    lib.sel_version.restype = ctypes.c_char_p
    lib.sel_version.argtypes = []
    lib.sel_stream.restype = ctypes.c_void_p
    lib.sel_stream.argtypes = [P]
    lib.sel_closure_len.restype = I64
    lib.sel_closure_len.argtypes = []
    lib.sel_mlp_work_floats.restype = I64
    lib.sel_mlp_work_floats.argtypes = [I64]
    _lib = lib
    return lib


def _check(rc: int):
    if rc != SEL_OK:
        raise SelError(rc, load().sel_last_error().decode())


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def version() -> str:
    return load().sel_version().decode()


class Mesh:
    """sel_mesh_create / sel_mesh_destroy."""

    def __init__(self, dim, N, xyz, gid, face_tag=None, wall_u=None, coupling="cg"):
        """coupling "cg" (sel_mesh_create) or "dg" (sel_mesh_create_dg)."""
        lib = load()
        self.dim, self.N = int(dim), int(N)
        self.np_ = (self.N + 1) ** self.dim
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.E = int(xyz.shape[0])
        gid = np.ascontiguousarray(gid, dtype=np.int64)
        ft = None if face_tag is None else np.ascontiguousarray(face_tag, dtype=np.int32)
        wu = np.zeros((0, self.dim)) if wall_u is None else np.ascontiguousarray(wall_u, dtype=np.float64)
        wu = wu.reshape(-1, self.dim)
        ntags = int(wu.shape[0])
        h = ctypes.c_void_p()
        create = {"cg": lib.sel_mesh_create, "dg": lib.sel_mesh_create_dg}[coupling]
        _check(create(self.dim, self.N, self.E, _ptr(xyz), _ptr(gid), _ptr(ft) if ft is not None else None,
                      ntags, _ptr(wu) if ntags else None, ctypes.byref(h)))
        self._h = h
        self._lib = lib

    @classmethod
    def from_inputs(cls, mesh, coupling="cg"):
        return cls(mesh.dim, mesh.N, mesh.xyz, mesh.gid, mesh.face_tag, mesh.wall_u, coupling)

    def info(self) -> dict:
        out = np.zeros(8, dtype=np.int64)
        _check(self._lib.sel_mesh_info(self._h, _ptr(out)))
        keys = ["dim", "N", "E", "np", "unique_nodes", "groups", "boundary_nodes_per_element", "wall_faces"]
        return dict(zip(keys, (int(v) for v in out)))

    def workspace_bytes(self, params: sel_params) -> int:
        n = ctypes.c_size_t()
        _check(self._lib.sel_workspace_bytes(self._h, ctypes.byref(params), ctypes.byref(n)))
        return int(n.value)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sel_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(Q, nu, dt, rho0=1.0, accel=(0.0, 0.0, 0.0), precision="fp64", filter=None, filter_kc=2,
                filter_amp=0.0, filter_order=2.0, rk="ssprk3", closure=None) -> sel_params:
    p = sel_params()
    p.Q = int(Q)
    p.precision = PRECISIONS[precision]
    p.rk = RKS[rk]
    p.filter_type = FILTERS[filter]
    p.filter_kc = int(filter_kc if filter_kc is not None else 0)
    p.filter_amp = float(filter_amp)
    p.filter_order = float(filter_order)
    p.rho0 = float(rho0)
    p.nu = float(nu)
    p.dt = float(dt)
    acc = list(accel) + [0.0] * (3 - len(accel))
    for k in range(3):
        p.accel[k] = float(acc[k])
    p.closure = None
    p.closure_len = 0
    if closure is not None:
        blob = np.ascontiguousarray(closure, dtype=np.float32).reshape(-1)
        p._closure_blob = blob  # kept alive with the struct; sel_init copies it
        p.closure = blob.ctypes.data
        p.closure_len = blob.size
    return p


class Sim:
    """One simulation on the GPU: sel_init ... sel_destroy.

    The workspace is a torch uint8 tensor on ``device``; work is enqueued on
    ``stream`` (a torch.cuda.Stream, default: the current stream)."""

    def __init__(self, mesh: Mesh, params: sel_params, rho, u, device="cuda:0", stream=None):
        import torch

        lib = load()
        self.mesh = mesh
        self.params = params
        self.dim, self.N, self.E, self.np_, self.Q = mesh.dim, mesh.N, mesh.E, mesh.np_, params.Q
        self.device = torch.device(device)
        nbytes = mesh.workspace_bytes(params)
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.E, self.np_)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.E, self.np_, self.dim)
        h = ctypes.c_void_p()
        _check(lib.sel_init(mesh._h, ctypes.byref(params), _ptr(rho), _ptr(u), ctypes.c_void_p(self.ws.data_ptr()),
                            nbytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sel_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nv(self):
        return self.E * self.Q * self.np_

    def step(self, n=1):
        _check(self._lib.sel_step(self._h, int(n)))

    def step_timed(self, n):
        """Run n steps with HIP events around every launch; returns
        {kind: (total ms, launches)} for the kernel kinds of sel_step_timed."""
        ms = np.zeros(6)
        cnt = np.zeros(6, dtype=np.int64)
        _check(self._lib.sel_step_timed(self._h, int(n), _ptr(ms), _ptr(cnt)))
        names = ["stage1", "stage23", "assembly", "filter", "features", "network"]
        return {names[k]: (float(ms[k]), int(cnt[k])) for k in range(6)}

    def sync(self):
        _check(self._lib.sel_sync(self._h))

    def moments(self):
        rho = np.zeros((self.E, self.np_))
        u = np.zeros((self.E, self.np_, self.dim))
        _check(self._lib.sel_moments(self._h, _ptr(rho), _ptr(u)))
        return rho, u

    def moments_device(self, d_rho, d_u):
        """Enqueue moments into FP64 torch tensors d_rho [E][np], d_u [E][np][dim] (no sync)."""
        _check(self._lib.sel_moments_device(self._h, ctypes.c_void_p(d_rho.data_ptr()),
                                            ctypes.c_void_p(d_u.data_ptr())))

    def reduce(self):
        out = np.zeros(self.dim + 3)
        _check(self._lib.sel_reduce(self._h, _ptr(out)))
        return out

    def velocity_gradient(self):
        """du_c/dx_q of the current state at every element node [E][np][dim][dim]."""
        out = np.zeros((self.E, self.np_, self.dim, self.dim))
        _check(self._lib.sel_velocity_gradient(self._h, _ptr(out)))
        return out

    def radial_profile(self, origin, axis, rmax, nbins):
        """Per radial bin of [0, rmax) around the line through origin along
        axis: (sum wJ u.n, sum wJ) over the element nodes of the bin
        (sel_radial_profile); their ratio is the bin's mean axial velocity."""
        o = np.zeros(self.dim)
        n = np.zeros(self.dim)
        o[:] = np.asarray(origin, dtype=np.float64)[:self.dim]
        n[:] = np.asarray(axis, dtype=np.float64)[:self.dim]
        out = np.zeros(2 * int(nbins))
        _check(self._lib.sel_radial_profile(self._h, _ptr(o), _ptr(n), float(rmax), int(nbins), _ptr(out)))
        return out[:nbins], out[nbins:]

    def set_force(self, F):
        """Force density per node [E][np][dim] added to rho g from the next
        step on (sel_set_force); None removes it."""
        if F is None:
            _check(self._lib.sel_set_force(self._h, None))
            return
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(self.E, self.np_, self.dim)
        _check(self._lib.sel_set_force(self._h, _ptr(F)))

    def get_f(self):
        f = np.zeros((self.E, self.Q, self.np_))
        _check(self._lib.sel_get_f(self._h, _ptr(f)))
        return f

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.E, self.Q, self.np_)
        _check(self._lib.sel_set_f(self._h, _ptr(f)))

    def apply(self, op: str, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.E, self.Q, self.np_)
        out = np.zeros_like(f)
        _check(self._lib.sel_apply(self._h, OPS[op], _ptr(f), _ptr(out)))
        return out

    def geometry(self):
        wJ = np.zeros((self.E, self.np_))
        J = np.zeros((self.E, self.np_))
        _check(self._lib.sel_geometry(self._h, _ptr(wJ), _ptr(J)))
        return wJ, J

    # ---- learned closure --------------------------------------------------
    def closure_set(self, blob):
        """Replace the closure blob (None: plain method until the next blob)."""
        if blob is None:
            _check(self._lib.sel_closure_set(self._h, None, 0))
            return
        b = np.ascontiguousarray(blob, dtype=np.float32).reshape(-1)
        _check(self._lib.sel_closure_set(self._h, _ptr(b), b.size))

    def closure_features(self):
        """Features of the current state as a float32 torch tensor [E][np][6]."""
        import torch

        X = torch.empty((self.E, self.np_, 6), dtype=torch.float32, device=self.device)
        _check(self._lib.sel_closure_features(self._h, ctypes.c_void_p(X.data_ptr())))
        return X

    @property
    def unique_nodes(self):
        return self.mesh.info()["unique_nodes"]

    def closure_dtau(self):
        """Increments the next step would use, per unique node id (float32 torch tensor)."""
        import torch

        d = torch.empty(self.unique_nodes, dtype=torch.float32, device=self.device)
        _check(self._lib.sel_closure_dtau(self._h, ctypes.c_void_p(d.data_ptr())))
        return d

    @property
    def time(self):
        t = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self._lib.sel_get_time(self._h, ctypes.byref(t), ctypes.byref(n)))
        return t.value

    @property
    def nstep(self):
        t = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self._lib.sel_get_time(self._h, ctypes.byref(t), ctypes.byref(n)))
        return n.value


def params_from_case(case, precision="fp64") -> sel_params:
    return make_params(case.Q, case.nu, case.dt, rho0=case.rho0, accel=case.g, precision=precision,
                       filter=case.filter, filter_kc=case.filter_kc, filter_amp=case.filter_amp,
                       filter_order=case.filter_order, rk=case.rk)


def from_case(case, precision="fp64", device="cuda:0", rho=None, u=None, stream=None, closure=None) -> Sim:
    """GPU simulation of a case from the seeded input generators."""
    mesh = Mesh.from_inputs(case.mesh, case.coupling)
    p = params_from_case(case, precision)
    if closure is not None:
        blob = np.ascontiguousarray(closure, dtype=np.float32).reshape(-1)
        p._closure_blob = blob
        p.closure = blob.ctypes.data
        p.closure_len = blob.size
    return Sim(mesh, p, case.rho if rho is None else rho, case.u if u is None else u, device=device, stream=stream)


# ---- learned closure: coarse graining, targets, network ----------------------
def closure_len() -> int:
    return int(load().sel_closure_len())


def coarse_grain(fine: Sim, coarse: Sim) -> None:
    """Project the fine state onto the coarse simulation (same elements)."""
    _check(load().sel_coarse_grain(fine._h, coarse._h))


def closure_targets(fine: Sim, coarse: Sim):
    """Targets dtau* = nu_t / (c_s^2 dt_coarse), the element value on every
    coarse node (float32 torch tensor [E][np_coarse])."""
    import torch

    y = torch.empty((coarse.E, coarse.np_), dtype=torch.float32, device=coarse.device)
    _check(load().sel_closure_targets(fine._h, coarse._h, ctypes.c_void_p(y.data_ptr())))
    return y


def _dp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_of(t, stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream(t.device)
    return ctypes.c_void_p(s.cuda_stream)


def mlp_forward(params, X, tau, stream=None):
    """z and dtau for feature rows X [n][6] (float32 torch tensors on the GPU)."""
    import torch

    X = X.reshape(-1, 6).contiguous()
    n = X.shape[0]
    z = torch.empty(n, dtype=torch.float32, device=X.device)
    d = torch.empty(n, dtype=torch.float32, device=X.device)
    _check(load().sel_mlp_forward(_dp(params), _dp(X), n, float(tau), _dp(z), _dp(d), _stream_of(X, stream)))
    return z, d


def mlp_work(n, device):
    import torch

    return torch.empty(int(load().sel_mlp_work_floats(int(n))), dtype=torch.float32, device=device)


def mlp_gradient(params, X, y, idx=None, work=None, stream=None):
    """(gradient of the trainable range [8833], loss) on the GPU; idx selects rows."""
    import torch

    X = X.reshape(-1, 6).contiguous()
    n = X.shape[0] if idx is None else idx.numel()
    work = mlp_work(n, X.device) if work is None else work
    g = torch.empty(8833, dtype=torch.float32, device=X.device)
    loss = ctypes.c_double()
    _check(load().sel_mlp_gradient(_dp(params), _dp(X), _dp(y), _dp(idx), n, _dp(work), _dp(g),
                                   ctypes.byref(loss), _stream_of(X, stream)))
    return g, loss.value


class MLPTrainer:
    """Adam training of a closure blob held in a float32 torch tensor."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        import torch

        self.params = params
        self.m = torch.zeros(8833, dtype=torch.float32, device=params.device)
        self.v = torch.zeros_like(self.m)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self._work = None

    def step(self, X, y, idx=None, stream=None, want_loss=True):
        """One Adam step on rows idx (int32 device tensor) of X, y (all rows if None)."""
        X = X.reshape(-1, 6).contiguous()
        n = X.shape[0] if idx is None else idx.numel()
        if self._work is None or self._work.numel() < load().sel_mlp_work_floats(n):
            self._work = mlp_work(n, X.device)
        self.t += 1
        loss = ctypes.c_double()
        _check(load().sel_mlp_train_step(_dp(self.params), _dp(self.m), _dp(self.v), _dp(X), _dp(y), _dp(idx), n,
                                         self.t,
                                         self.lr, self.b1, self.b2, self.eps, _dp(self._work),
                                         ctypes.byref(loss) if want_loss else None, _stream_of(X, stream)))
        return loss.value if want_loss else None
