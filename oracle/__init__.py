"""Python access to the FP64 CPU oracle (``sel_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers. The product path never
imports this package. Build with ``python -m oracle.build`` (or call
``build()``); the library is compiled with gcc, FP64, no fast-math.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sel_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FILTER_CODES = {None: 0, "none": 0, "quad": 1, "exp": 2}
RK_CODES = {"ssprk3": 0, "printed4": 1}
COUPLING_CODES = {"cg": 0, "dg": 1}


def build(force: bool = True, native: bool = False, path: str | None = None) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over elements, no fast-math).
    native=True adds -march=native, for timing on the machine that runs it
    (that build is written to ``path`` and is not portable to other hosts)."""
    out = path or _LIB_PATH
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2"] + (["-march=native"] if native else []) + \
              ["-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def use_library(path: str) -> None:
    """Load the oracle from another build of the same source (the native
    build used for CPU timing); later calls use it."""
    global _lib
    _lib = None
    _load(path)


def _load(path: str | None = None):
    global _lib
    if _lib is not None:
        return _lib
    path = path or _LIB_PATH
    if not os.path.exists(path):
        build(force=True, path=path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    D = ctypes.c_double
    I = ctypes.c_int
    I64 = ctypes.c_int64
    lib.oracle_create.restype = P
    lib.oracle_create.argtypes = [I, I, I64, P, P, P, I, P, I, D, D, D, P, I, I, D, D, I, I]
    lib.oracle_destroy.argtypes = [P]
    for name in ("oracle_init",):
        getattr(lib, name).argtypes = [P, P, P]
    lib.oracle_step.argtypes = [P, I64]
    lib.oracle_advect.argtypes = [P, I64]
    lib.oracle_moments.argtypes = [P, P, P]
    lib.oracle_reduce.argtypes = [P, P]
    lib.oracle_get_f.argtypes = [P, P]
    lib.oracle_set_f.argtypes = [P, P]
    lib.oracle_geometry.argtypes = [P, P, P, P]
    lib.oracle_mass.argtypes = [P, P]
    lib.oracle_set_force.argtypes = [P, P]
    for name in ("oracle_rhs_local", "oracle_rhs", "oracle_collide", "oracle_filter"):
        getattr(lib, name).argtypes = [P, P, P]
    lib.oracle_time.restype = D
    lib.oracle_time.argtypes = [P]
    lib.oracle_tau.restype = D
    lib.oracle_tau.argtypes = [P]
    lib.oracle_gll.argtypes = [I, P, P]
    lib.oracle_dmat.argtypes = [I, P, P]
    lib.oracle_lattice.argtypes = [I, I, P, P, P]
    lib.oracle_filter_sigma.argtypes = [I, I, I, D, D, P]
    lib.oracle_filter_matrix.argtypes = [I, P, I, I, D, D, P]
    lib.oracle_legendre.argtypes = [I, D, P, P]
    lib.oracle_rk_scalar.argtypes = [I, D, D, D, D, I64, P]
    lib.oracle_set_threads.argtypes = [I]
    lib.oracle_set_dtau.argtypes = [P, P]
    lib.oracle_get_threads.restype = I
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def gll(N: int):
    lib = _load()
    xi = np.zeros(N + 1)
    w = np.zeros(N + 1)
    if lib.oracle_gll(N, _ptr(xi), _ptr(w)):
        raise ValueError("bad N")
    return xi, w


def dmat(N: int, xi=None) -> np.ndarray:
    lib = _load()
    if xi is None:
        xi, _ = gll(N)
    xi = _f64(xi)
    D = np.zeros((N + 1, N + 1))
    if lib.oracle_dmat(N, _ptr(xi), _ptr(D)):
        raise ValueError("bad N")
    return D


def lattice(dim: int, Q: int):
    lib = _load()
    e = np.zeros((Q, 3))
    t = np.zeros(Q)
    opp = np.zeros(Q, dtype=np.int32)
    if lib.oracle_lattice(dim, Q, _ptr(e), _ptr(t), _ptr(opp)):
        raise ValueError("unsupported lattice")
    return e[:, :dim].copy(), t, opp


def filter_sigma(N, ftype, kc, amp, order=2.0):
    lib = _load()
    s = np.zeros(N + 1)
    if lib.oracle_filter_sigma(N, FILTER_CODES[ftype], int(kc), float(amp), float(order), _ptr(s)):
        raise ValueError("bad filter")
    return s


def filter_matrix(N, ftype, kc, amp, order=2.0, xi=None):
    lib = _load()
    if xi is None:
        xi, _ = gll(N)
    xi = _f64(xi)
    F = np.zeros((N + 1, N + 1))
    if lib.oracle_filter_matrix(N, _ptr(xi), FILTER_CODES[ftype], int(kc), float(amp),
                                float(order), _ptr(F)):
        raise ValueError("bad filter")
    return F


def legendre(n: int, x: float):
    lib = _load()
    L = np.zeros(1)
    dL = np.zeros(1)
    lib.oracle_legendre(n, float(x), _ptr(L), _ptr(dL))
    return float(L[0]), float(dL[0])


def rk_scalar(rk: str, lam: float, b: float, y0: float, dt: float, nsteps: int) -> float:
    lib = _load()
    y = np.zeros(1)
    if lib.oracle_rk_scalar(RK_CODES[rk], lam, b, y0, dt, nsteps, _ptr(y)):
        raise ValueError("bad rk")
    return float(y[0])


class OracleSim:
    """One oracle simulation on a mesh (FP64, host memory)."""

    def __init__(self, dim, N, xyz, gid, face_tag, wall_u, Q, rho0, nu, dt, g=(0.0, 0.0, 0.0),
                 filter=None, filter_kc=2, filter_amp=0.0, filter_order=2.0, rk="ssprk3", coupling="cg"):
        lib = _load()
        self.dim, self.N, self.Q = dim, N, Q
        self.nu, self.dt, self.rho0 = float(nu), float(dt), float(rho0)
        self.np_ = (N + 1) ** dim
        self._xyz = _f64(xyz)
        self.E = self._xyz.shape[0]
        self._gid = np.ascontiguousarray(gid, dtype=np.int64)
        self._ftag = np.ascontiguousarray(face_tag, dtype=np.int32)
        wall_u = np.zeros((0, dim)) if wall_u is None else _f64(wall_u).reshape(-1, dim)
        self._wall_u = _f64(wall_u) if wall_u.size else np.zeros((1, dim))
        ntags = wall_u.shape[0]
        gg = _f64(list(g) + [0.0] * (3 - len(g)))
        self._g = gg
        h = lib.oracle_create(dim, N, self.E, _ptr(self._xyz), _ptr(self._gid), _ptr(self._ftag),
                              ntags, _ptr(self._wall_u), Q, rho0, nu, dt, _ptr(gg),
                              FILTER_CODES[filter], int(filter_kc), float(filter_amp),
                              float(filter_order), RK_CODES[rk], COUPLING_CODES[coupling])
        if not h:
            raise ValueError("oracle_create rejected the mesh or parameters")
        self._h = ctypes.c_void_p(h)
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nv(self):
        return self.E * self.Q * self.np_

    def init(self, rho, u):
        rho = _f64(rho).reshape(self.E, self.np_)
        u = _f64(u).reshape(self.E, self.np_, self.dim)
        self._lib.oracle_init(self._h, _ptr(rho), _ptr(u))

    def step(self, n=1):
        self._lib.oracle_step(self._h, int(n))

    def advect(self, n=1):
        self._lib.oracle_advect(self._h, int(n))

    def moments(self):
        rho = np.zeros((self.E, self.np_))
        u = np.zeros((self.E, self.np_, self.dim))
        self._lib.oracle_moments(self._h, _ptr(rho), _ptr(u))
        return rho, u

    def reduce(self):
        out = np.zeros(self.dim + 2)
        self._lib.oracle_reduce(self._h, _ptr(out))
        return out

    def get_f(self):
        f = np.zeros((self.E, self.Q, self.np_))
        self._lib.oracle_get_f(self._h, _ptr(f))
        return f

    def set_f(self, f):
        f = _f64(f).reshape(self.E, self.Q, self.np_)
        self._lib.oracle_set_f(self._h, _ptr(f))

    def geometry(self):
        wJ = np.zeros((self.E, self.np_))
        G = np.zeros((self.E, self.np_, 3, 3))
        J = np.zeros((self.E, self.np_))
        self._lib.oracle_geometry(self._h, _ptr(wJ), _ptr(G), _ptr(J))
        return wJ, G, J

    def set_force(self, F):
        """Force density per node [E][np][dim] added to rho g from the next
        step on; None removes it."""
        if F is None:
            self._lib.oracle_set_force(self._h, None)
            return
        self._F = _f64(F).reshape(self.E, self.np_, self.dim)
        if self._lib.oracle_set_force(self._h, _ptr(self._F)):
            raise MemoryError("oracle_set_force")

    def mass(self):
        M = np.zeros((self.E, self.np_))
        self._lib.oracle_mass(self._h, _ptr(M))
        return M

    def _op(self, name, f):
        f = _f64(f).reshape(self.E, self.Q, self.np_)
        out = np.zeros_like(f)
        getattr(self._lib, name)(self._h, _ptr(f), _ptr(out))
        return out

    def rhs_local(self, f):
        return self._op("oracle_rhs_local", f)

    def rhs(self, f):
        return self._op("oracle_rhs", f)

    def collide(self, f):
        return self._op("oracle_collide", f)

    def filter(self, f):
        return self._op("oracle_filter", f)

    @property
    def time(self):
        return float(self._lib.oracle_time(self._h))

    @property
    def tau(self):
        return float(self._lib.oracle_tau(self._h))


def from_case(case, **over) -> OracleSim:
    """Oracle simulation for a case of the seeded input generators."""
    kw = dict(g=case.g, filter=case.filter, filter_kc=case.filter_kc, filter_amp=case.filter_amp,
              filter_order=case.filter_order, rk=case.rk, coupling=case.coupling)
    kw.update(over)
    sim = OracleSim(case.dim, case.N, case.xyz, case.gid, case.face_tag, case.wall_u, case.Q,
                    case.rho0, case.nu, case.dt, **kw)
    sim.init(case.rho, case.u)
    return sim
