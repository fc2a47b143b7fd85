"""Seeded synthetic inputs: meshes, initial fields and case parameters.

This module serves both the HIP library and the CPU oracle, so it holds none
of the method's arithmetic: it only places mesh nodes, numbers them, tags wall
faces and evaluates initial and analytic fields. Each side builds its own
quadrature, derivative, lattice and filter tables from these inputs.

Mesh nodes are placed at the Gauss-Lobatto-Legendre points returned by
``numpy.polynomial.legendre`` (the roots of P_N' plus the end points); the
solver treats whatever nodes it is given as the isoparametric map.

Conventions (the public interface states them too): node index
``i + (N+1) j + (N+1)^2 k`` with r fastest; ``xyz[E][np][dim]``;
``gid[E][np]`` global node ids in ``[0, E*np)``, copies of a shared or
periodic node carry the same id; ``face_tag[E][2 dim]`` over faces
``(r-, r+, s-, s+, t-, t+)``, 0 = interior or periodic, k >= 1 = wall k whose
velocity is ``wall_u[k-1]``. Lattice units: speed 1, c_s^2 = 1/3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

CS2 = 1.0 / 3.0
CS = math.sqrt(CS2)


def gll_points(N: int) -> np.ndarray:
    """GLL points on [-1, 1] from numpy's Legendre module (mesh placement only)."""
    from numpy.polynomial import legendre as npleg

    c = np.zeros(N + 1)
    c[N] = 1.0
    inner = np.sort(np.real(npleg.legroots(npleg.legder(c)))) if N >= 2 else np.zeros(0)
    return np.concatenate([[-1.0], inner, [1.0]])


@dataclass
class Mesh:
    dim: int
    N: int
    xyz: np.ndarray       # [E][np][dim]
    gid: np.ndarray       # [E][np] int64
    face_tag: np.ndarray  # [E][2dim] int32
    wall_u: np.ndarray    # [ntags][dim]

    @property
    def E(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def np_(self) -> int:
        return (self.N + 1) ** self.dim


def box_mesh(dim: int, N: int, nel, lo, hi, periodic, wall_tags=None, wall_u=None,
             warp: Optional[Callable[[np.ndarray], np.ndarray]] = None) -> Mesh:
    """Structured box of nel[0] x nel[1] (x nel[2]) elements, elements ordered
    with x fastest. ``wall_tags[m] = (tag_lo, tag_hi)`` for non-periodic
    directions. ``warp`` maps node coordinates [..., dim] to displaced ones
    (it must keep periodic copies consistent and walls in place)."""
    nel = tuple(int(n) for n in nel)
    lo = np.asarray(lo, dtype=float)
    hi = np.asarray(hi, dtype=float)
    n1 = N + 1
    ref = (gll_points(N) + 1.0) / 2.0
    h = (hi - lo) / np.asarray(nel, dtype=float)
    E = int(np.prod(nel))
    npn = n1 ** dim
    # element multi-index (x fastest) and node multi-index (r fastest)
    eidx = np.stack(np.unravel_index(np.arange(E), nel[::-1])[::-1], axis=1)      # [E][dim]
    nidx = np.stack(np.unravel_index(np.arange(npn), (n1,) * dim)[::-1], axis=1)  # [np][dim]
    xyz = np.zeros((E, npn, dim))
    gcoord = np.zeros((E, npn, dim), dtype=np.int64)
    gsize = []
    for m in range(dim):
        xyz[:, :, m] = lo[m] + (eidx[:, None, m] + ref[nidx[None, :, m]]) * h[m]
        Gm = nel[m] * N + (0 if periodic[m] else 1)
        gsize.append(Gm)
        gcoord[:, :, m] = (eidx[:, None, m] * N + nidx[None, :, m]) % Gm
    gid = np.zeros((E, npn), dtype=np.int64)
    stride = 1
    for m in range(dim):
        gid += gcoord[:, :, m] * stride
        stride *= gsize[m]
    if warp is not None:
        xyz = warp(xyz)
    face_tag = np.zeros((E, 2 * dim), dtype=np.int32)
    for m in range(dim):
        if periodic[m]:
            continue
        tl, th = wall_tags[m]
        face_tag[eidx[:, m] == 0, 2 * m] = tl
        face_tag[eidx[:, m] == nel[m] - 1, 2 * m + 1] = th
    ntags = int(face_tag.max()) if face_tag.size else 0
    wu = np.zeros((max(ntags, 0), dim))
    if wall_u is not None:
        wu[:] = np.asarray(wall_u, dtype=float).reshape(-1, dim)[:ntags]
    return Mesh(dim, N, xyz, gid, face_tag, wu)


def min_node_spacing(mesh: Mesh) -> float:
    """Smallest distance between neighbouring nodes along a reference line."""
    n1 = mesh.N + 1
    x = mesh.xyz.reshape((mesh.E,) + (n1,) * mesh.dim + (mesh.dim,))
    hmin = np.inf
    for m in range(mesh.dim):
        ax = mesh.dim - m  # r is the last spatial axis of the reshaped array
        dx = np.diff(x, axis=ax)
        hmin = min(hmin, float(np.sqrt((dx ** 2).sum(-1)).min()))
    return hmin


# ----------------------------------------------------------------------------
# Initial fields
# ----------------------------------------------------------------------------

def tgv2d_fields(xyz, u0, rho0=1.0, L0=1.0, t=0.0, nu=0.0):
    """2D Taylor-Green vortex: u = u0 e^{-2 nu t / L0^2}(sin x cos y, -cos x sin y),
    p = rho0 u0^2/4 (cos 2x + cos 2y) e^{-4 nu t}, rho = rho0 + p / c_s^2."""
    x = xyz[..., 0] / L0
    y = xyz[..., 1] / L0
    a = math.exp(-2.0 * nu * t / (L0 * L0))
    u = np.stack([u0 * a * np.sin(x) * np.cos(y), -u0 * a * np.cos(x) * np.sin(y)], axis=-1)
    p = rho0 * u0 * u0 / 4.0 * (np.cos(2 * x) + np.cos(2 * y)) * a * a
    return rho0 + p / CS2, u


def tgv3d_fields(xyz, u0, rho0=1.0, L0=1.0):
    """3D Taylor-Green vortex initial field, p = rho0 u0^2/16 (cos 2x + cos 2y)(cos 2z + 2)."""
    x, y, z = (xyz[..., k] / L0 for k in range(3))
    u = np.stack([u0 * np.sin(x) * np.cos(y) * np.cos(z),
                  -u0 * np.cos(x) * np.sin(y) * np.cos(z),
                  np.zeros_like(x)], axis=-1)
    p = rho0 * u0 * u0 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    return rho0 + p / CS2, u


def double_shear_fields(xyz, u0, kappa=80.0, delta=0.05, rho0=1.0):
    """Double shear layer on the unit square; the transverse perturbation is
    delta * u0 * sin(2 pi (x + 1/4))."""
    x = xyz[..., 0]
    y = xyz[..., 1]
    ux = np.where(y <= 0.5, u0 * np.tanh(kappa * (y - 0.25)), u0 * np.tanh(kappa * (0.75 - y)))
    uy = delta * u0 * np.sin(2 * np.pi * (x + 0.25))
    return np.full(x.shape, rho0), np.stack([ux, uy], axis=-1)


def rest_fields(xyz, rho0=1.0):
    dim = xyz.shape[-1]
    return np.full(xyz.shape[:-1], rho0), np.zeros(xyz.shape)


# ----------------------------------------------------------------------------
# Analytic references
# ----------------------------------------------------------------------------

def couette_profile(y, t, U, H, nu, nterms=400):
    """Start-up Couette flow between a wall at y = 0 and a plate at y = H moving at U."""
    y = np.asarray(y, dtype=float)
    u = U * y / H
    for n in range(1, nterms + 1):
        u = u - (2.0 * U / math.pi) * ((-1) ** (n + 1) / n) * np.sin(n * math.pi * y / H) * \
            math.exp(-n * n * math.pi * math.pi * nu * t / (H * H))
    return u


def poiseuille_profile(y, t, g, H, nu, nterms=400):
    """Start-up plane Poiseuille flow driven by body acceleration g (t = inf: steady)."""
    y = np.asarray(y, dtype=float)
    u = g * y * (H - y) / (2.0 * nu)
    if not math.isinf(t):
        for n in range(1, nterms + 1, 2):
            u = u - 4.0 * g * H * H / (nu * n ** 3 * math.pi ** 3) * np.sin(n * math.pi * y / H) * \
                math.exp(-n * n * math.pi * math.pi * nu * t / (H * H))
    return u


# ----------------------------------------------------------------------------
# Cases
# ----------------------------------------------------------------------------

@dataclass
class Case:
    name: str
    mesh: Mesh
    Q: int
    rho0: float
    nu: float
    dt: float
    rho: np.ndarray
    u: np.ndarray
    steps: int
    g: tuple = (0.0, 0.0, 0.0)
    filter: Optional[str] = None
    filter_kc: int = 2
    filter_amp: float = 0.0
    filter_order: float = 2.0
    rk: str = "ssprk3"
    coupling: str = "cg"  # "cg" (continuous, the paper's) or "dg" (discontinuous, upwind interface flux)
    meta: dict = field(default_factory=dict)

    # convenience views
    @property
    def dim(self):
        return self.mesh.dim

    @property
    def N(self):
        return self.mesh.N

    @property
    def xyz(self):
        return self.mesh.xyz

    @property
    def gid(self):
        return self.mesh.gid

    @property
    def face_tag(self):
        return self.mesh.face_tag

    @property
    def wall_u(self):
        return self.mesh.wall_u

    @property
    def E(self):
        return self.mesh.E

    @property
    def np_(self):
        return self.mesh.np_

    @property
    def nv(self):
        return self.E * self.np_ * self.Q


def stable_dt(mesh: Mesh, cfl: float = 0.5) -> float:
    """dt = cfl * h_min / max_a |e_a|_1, with |e_a|_1 = dim for the full lattices."""
    return cfl * min_node_spacing(mesh) / mesh.dim


FILTER_PAPER = dict(filter="quad", filter_kc=2, filter_amp=0.1, filter_order=2.0)
FILTER_EXP = dict(filter="exp", filter_kc=None, filter_amp=36.0, filter_order=16.0)


def _filter_kw(spec, N):
    if spec is None or spec == "none":
        return dict(filter=None)
    if spec == "quad":
        return dict(FILTER_PAPER)
    if spec == "exp":
        kw = dict(FILTER_EXP)
        kw["filter_kc"] = (2 * N) // 3
        return kw
    raise ValueError(spec)


def case_tgv2d(nel=8, N=5, Re=100.0, u0=0.05, steps=200, filt=None, cfl=0.5) -> Case:
    """2D Taylor-Green vortex, D2Q9, periodic [0, 2 pi]^2."""
    L = 2 * math.pi
    mesh = box_mesh(2, N, (nel, nel), (0, 0), (L, L), (True, True))
    nu = u0 * 1.0 / Re
    dt = stable_dt(mesh, cfl)
    rho, u = tgv2d_fields(mesh.xyz, u0)
    return Case("tgv2d", mesh, 9, 1.0, nu, dt, rho, u, steps, meta=dict(u0=u0, Re=Re),
                **_filter_kw(filt, N))


def case_double_shear(nel=32, N=7, Re=1.0e4, Ma=0.1, kappa=80.0, delta=0.05, steps=2000,
                      filt="exp", cfl=0.5) -> Case:
    """Double shear layer, D2Q9, periodic unit square."""
    mesh = box_mesh(2, N, (nel, nel), (0, 0), (1, 1), (True, True))
    u0 = Ma * CS
    nu = u0 * 1.0 / Re
    dt = stable_dt(mesh, cfl)
    rho, u = double_shear_fields(mesh.xyz, u0, kappa, delta)
    return Case("double_shear", mesh, 9, 1.0, nu, dt, rho, u, steps,
                meta=dict(u0=u0, Re=Re, kappa=kappa, delta=delta), **_filter_kw(filt, N))


def channel_warp(seed=2509, amp=0.0125, Lx=2.0, H=1.0, kx=1, ky=1):
    """Seeded sinusoidal displacement of channel nodes: zero on the walls,
    periodic in x with period Lx / k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ph = rng.uniform(0.0, 2 * math.pi, size=2)

    def warp(xyz):
        x = xyz[..., 0]
        y = xyz[..., 1]
        s = np.sin(math.pi * y / H)
        out = xyz.copy()
        out[..., 0] = x + amp * s * np.sin(2 * math.pi * kx * x / Lx + ph[0])
        out[..., 1] = y + amp * s * np.sin(2 * math.pi * ky * x / Lx + ph[1])
        return out

    return warp


def _channel_mesh(nelx, nely, N, Lx, H, curved, top_u, seed):
    warp = channel_warp(seed=seed, amp=0.1 * (H / nely), Lx=Lx, H=H) if curved else None
    return box_mesh(2, N, (nelx, nely), (0, 0), (Lx, H), (True, False),
                    wall_tags={1: (1, 2)}, wall_u=[[0.0, 0.0], [top_u, 0.0]], warp=warp)


def case_poiseuille(nelx=16, nely=8, N=7, Re=100.0, umax=0.1 / 3.0, Lx=2.0, H=1.0,
                    curved=False, steps=200, seed=2509, cfl=0.5, filt=None) -> Case:
    """Plane Poiseuille flow driven by a body acceleration g = 8 nu umax / H^2,
    FBB walls at y = 0 and y = H, periodic in x, starting from rest."""
    mesh = _channel_mesh(nelx, nely, N, Lx, H, curved, 0.0, seed)
    nu = umax * H / Re
    g = 8.0 * nu * umax / (H * H)
    dt = stable_dt(mesh, cfl)
    rho, u = rest_fields(mesh.xyz)
    return Case("poiseuille" + ("_curved" if curved else ""), mesh, 9, 1.0, nu, dt, rho, u, steps,
                g=(g, 0.0, 0.0), meta=dict(umax=umax, Re=Re, H=H, gx=g), **_filter_kw(filt, N))


def case_couette(nelx=16, nely=8, N=7, Re=10.0, Ma=0.1, Lx=2.0, H=1.0, curved=False, steps=200,
                 seed=2509, cfl=0.5, filt=None) -> Case:
    """Start-up Couette flow: wall at y = 0 at rest, wall at y = H moving at U."""
    U = Ma * CS
    mesh = _channel_mesh(nelx, nely, N, Lx, H, curved, U, seed)
    nu = U * H / Re
    dt = stable_dt(mesh, cfl)
    rho, u = rest_fields(mesh.xyz)
    return Case("couette" + ("_curved" if curved else ""), mesh, 9, 1.0, nu, dt, rho, u, steps,
                meta=dict(U=U, Re=Re, H=H), **_filter_kw(filt, N))


def case_tgv3d(nel=16, N=7, Q=27, Re=1600.0, Ma=0.1, steps=5000, filt="quad", cfl=0.5) -> Case:
    """3D Taylor-Green vortex, periodic [0, 2 pi]^3, L0 = 1."""
    L = 2 * math.pi
    mesh = box_mesh(3, N, (nel,) * 3, (0, 0, 0), (L, L, L), (True, True, True))
    u0 = Ma * CS
    nu = u0 * 1.0 / Re
    dt = stable_dt(mesh, cfl)
    rho, u = tgv3d_fields(mesh.xyz, u0)
    return Case("tgv3d", mesh, Q, 1.0, nu, dt, rho, u, steps, meta=dict(u0=u0, Re=Re),
                **_filter_kw(filt, N))


def random_state(case: Case, seed: int = 7, amp: float = 0.01):
    """Seeded perturbation of a case's initial fields, drawn per global node so
    that every copy of a shared node gets the same value (continuous fields)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ng = int(case.gid.max()) + 1
    dr = rng.standard_normal(ng)[case.gid]
    du = rng.standard_normal((ng, case.dim))[case.gid]
    return case.rho + amp * dr, case.u + amp * 0.1 * du


# ----------------------------------------------------------------------------
# Learned-closure initial network
# ----------------------------------------------------------------------------

CLOSURE_NF, CLOSURE_NH = 6, 64


def closure_blob(seed: int, mean, std, dtau_max: float = 100.0, b4: float = -3.0) -> np.ndarray:
    """Seeded initial parameter blob of the closure network (FP32, layout
    mean[6], std[6], W1[64][6], b1[64], W2[64][64], b2[64], W3[64][64], b3[64],
    w4[64], b4, dtau_max): Glorot-uniform weights, zero hidden biases, b4 < 0
    so that the untrained network starts near dtau = 0."""
    nf, nh = CLOSURE_NF, CLOSURE_NH
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [np.asarray(mean, float).reshape(nf), np.asarray(std, float).reshape(nf)]
    for fo, fi in ((nh, nf), (nh, nh), (nh, nh)):
        a = math.sqrt(6.0 / (fi + fo))
        parts.append(rng.uniform(-a, a, size=fo * fi))
        parts.append(np.zeros(nh))
    a = math.sqrt(6.0 / (nh + 1))
    parts.append(rng.uniform(-a, a, size=nh))
    parts.append(np.array([b4, dtau_max]))
    return np.concatenate(parts).astype(np.float32)


# ----------------------------------------------------------------------------
# O-grid pipe (turbulent pipe case)
# ----------------------------------------------------------------------------

def _pos1d(I, nel, N, x_gll, bounds=None):
    """Parameter of global node index I on a line of nel elements of order N:
    element e = min(I // N, nel - 1), GLL point i = I - e N inside it; element
    bounds default to a uniform split of [-1, 1]."""
    I = np.asarray(I)
    e = np.minimum(I // N, nel - 1)
    i = I - e * N
    if bounds is None:
        bounds = np.linspace(-1.0, 1.0, nel + 1)
    lo, hi = bounds[e], bounds[e + 1]
    return lo + (hi - lo) * (1.0 + x_gll[i]) / 2.0


def pipe_radial_bounds(nrad, a, R, h_wall):
    """Radial element bounds t_0 = 0 < ... < t_nrad = 1 of the shell blocks in
    geometric progression, the last element (at the wall) of height h_wall at
    the middle of each block face (shell thickness R - a there)."""
    last = h_wall / (R - a)
    if not 0.0 < last < 1.0:
        raise ValueError("h_wall must be below the shell thickness")

    def total(q):
        return sum(q ** -k for k in range(nrad)) * last  # elements from the wall inwards

    lo, hi = 1e-3, 1e3
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if total(mid) > 1.0:
            lo = mid
        else:
            hi = mid
    q = math.sqrt(lo * hi)
    sizes = np.array([last * q ** -(nrad - 1 - k) for k in range(nrad)])
    sizes /= sizes.sum()
    return np.concatenate([[0.0], np.cumsum(sizes)])


def pipe_mesh(N: int, nsq: int = 8, nrad: int = 8, nax: int = 64, R: float = 1.0, L: float = 10.0,
              a: float = 0.35, h_wall: float = 0.087) -> Mesh:
    """O-grid pipe of radius R and periodic length L along z.

    Cross-section: a central square [-a, a]^2 of nsq x nsq elements and four
    shell blocks of nsq (azimuthal) x nrad (radial) elements between the
    square's sides and the circle. Shell nodes come from the transfinite
    (Gordon-Hall) blend of the straight inner side and the exact circular
    arc; radial element bounds grow geometrically so that the wall element is
    h_wall high. nax elements along z. Wall faces (tag 1, at rest) are the r+
    faces of the outermost shell elements. Element node order: central
    elements (x, y, z); shell elements (radial, azimuthal, z), so every
    Jacobian is positive. Global ids are assigned from integer block
    coordinates, so shared nodes are identified exactly."""
    n1 = N + 1
    xg = gll_points(N)
    S = nsq * N  # global node intervals along a square side / an arc
    T = nrad * N
    tb = pipe_radial_bounds(nrad, a, R, h_wall)
    # ---- 2D cross-section: element node keys and coordinates
    keys2d = []   # per 2D element: list of n1*n1 hashable keys, r fastest
    xy2d = []     # per 2D element: [n1*n1][2]
    for ey in range(nsq):
        for ex in range(nsq):
            I = ex * N + np.arange(n1)[None, :].repeat(n1, 0)
            J = ey * N + np.arange(n1)[:, None].repeat(n1, 1)
            I, J = I.reshape(-1), J.reshape(-1)
            keys2d.append([("c", int(i), int(j)) for i, j in zip(I, J)])
            xy2d.append(np.stack([a * _pos1d(I, nsq, N, xg), a * _pos1d(J, nsq, N, xg)], -1))

    def shell_key(b, s, t):
        if t == 0:  # on the square's side, counter-clockwise along block b
            if b == 0:
                return ("c", S, s)
            if b == 1:
                return ("c", S - s, S)
            if b == 2:
                return ("c", 0, S - s)
            return ("c", s, 0)
        if s == S:
            return ("s", (b + 1) % 4, 0, t)
        return ("s", b, s, t)

    for b in range(4):
        c, sn = math.cos(b * math.pi / 2), math.sin(b * math.pi / 2)
        for ea in range(nsq):
            for er in range(nrad):
                # local r = radial (index t), local s = azimuthal (index s)
                tt = er * N + np.arange(n1)[None, :].repeat(n1, 0)
                ss = ea * N + np.arange(n1)[:, None].repeat(n1, 1)
                tt, ss = tt.reshape(-1), ss.reshape(-1)
                keys2d.append([shell_key(b, int(s_), int(t_)) for s_, t_ in zip(ss, tt)])
                sp = _pos1d(ss, nsq, N, xg)
                tp = _pos1d(tt, nrad, N, xg, bounds=tb)
                inner = np.stack([np.full_like(sp, a), a * sp], -1)
                th = sp * math.pi / 4
                outer = np.stack([R * np.cos(th), R * np.sin(th)], -1)
                p = (1.0 - tp)[:, None] * inner + tp[:, None] * outer
                xy2d.append(np.stack([c * p[:, 0] - sn * p[:, 1], sn * p[:, 0] + c * p[:, 1]], -1))
    E2 = len(keys2d)
    ids = {}
    id2d = np.zeros((E2, n1 * n1), dtype=np.int64)
    for e, kl in enumerate(keys2d):
        for q, k in enumerate(kl):
            id2d[e, q] = ids.setdefault(k, len(ids))
    n2d = len(ids)
    xy2d = np.stack(xy2d)
    # ---- extrude along z (periodic)
    zb = np.linspace(0.0, L, nax + 1)
    E = E2 * nax
    npn = n1 ** 3
    xyz = np.zeros((E, npn, 3))
    gid = np.zeros((E, npn), dtype=np.int64)
    face_tag = np.zeros((E, 6), dtype=np.int32)
    kz = np.arange(n1)
    Kglob = (np.arange(nax)[:, None] * N + kz[None, :]) % (nax * N)  # [nax][n1]
    zpos = zb[:-1, None] + (zb[1:] - zb[:-1])[:, None] * (1.0 + xg[None, :]) / 2.0
    for ez in range(nax):
        sl = slice(ez * E2, (ez + 1) * E2)
        xyz[sl, :, 0] = np.tile(xy2d[:, :, 0], (1, n1))
        xyz[sl, :, 1] = np.tile(xy2d[:, :, 1], (1, n1))
        xyz[sl, :, 2] = np.repeat(zpos[ez], n1 * n1)[None, :]
        gid[sl] = np.tile(id2d, (1, n1)) + n2d * np.repeat(Kglob[ez], n1 * n1)[None, :]
    shell_outer = np.zeros(E2, dtype=bool)
    for b in range(4):
        for ea in range(nsq):
            shell_outer[nsq * nsq + b * nsq * nrad + ea * nrad + (nrad - 1)] = True
    face_tag[np.tile(shell_outer, nax), 1] = 1
    return Mesh(3, N, xyz, gid, face_tag, np.zeros((1, 3)))


def pipe_perturbation(xyz, R, L, amp, seed=180, nmodes=16, scale=None):
    """Divergence-free perturbation u' = curl(phi A), phi = (1 - r^2/R^2)^2
    (zero with its gradient at the wall, so u' = 0 there), A a sum of seeded
    Fourier modes periodic in z; scaled so that max |u'| = amp over the given
    points, or multiplied by ``scale`` when that is given."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    r2 = (x * x + y * y) / (R * R)
    phi = (1.0 - r2) ** 2
    dphi = np.stack([-4.0 * (1.0 - r2) * x / (R * R), -4.0 * (1.0 - r2) * y / (R * R), np.zeros_like(x)], -1)
    A = np.zeros(xyz.shape)
    curlA = np.zeros(xyz.shape)
    for _ in range(nmodes):
        k = np.array([rng.integers(1, 5) * math.pi / R * rng.choice([-1, 1]),
                      rng.integers(1, 5) * math.pi / R * rng.choice([-1, 1]),
                      rng.integers(1, 5) * 2 * math.pi / L])
        av = rng.standard_normal(3)
        ph = rng.uniform(0, 2 * math.pi)
        arg = xyz @ k + ph
        A += np.sin(arg)[..., None] * av
        curlA += np.cos(arg)[..., None] * np.cross(k, av)
    u = phi[..., None] * curlA + np.cross(dphi, A)
    if scale is not None:
        return u * scale
    m = np.sqrt((u * u).sum(-1)).max()
    return u * (amp / m if m > 0 else 0.0)


def law_of_wall(yplus, kappa=0.41, Cplus=5.0):
    """Mean streamwise velocity in wall units (Sec. 3.5): u+ = y+ in the
    viscous sublayer and ln(y+)/kappa + C+ in the inertial sublayer, switched
    where the two meet (y+ = 11.4 for kappa = 0.41, C+ = 5), so that the
    profile is continuous."""
    yplus = np.asarray(yplus, dtype=np.float64)
    # crossing of y+ and ln(y+)/kappa + C+ above y+ = 1 (bisection)
    lo, hi = 1.0, 100.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid < math.log(mid) / kappa + Cplus:
            lo = mid
        else:
            hi = mid
    yc = 0.5 * (lo + hi)
    inertial = np.log(np.maximum(yplus, 1e-300)) / kappa + Cplus
    return np.where(yplus < yc, yplus, inertial)


def pipe_force(xyz, t, R, L, g, t0, kz=3, ktheta=4, B0=50.0, kappa=0.5, period=8.0, l0=0.2, lw=0.4):
    """Divergence-free perturbation force of the pipe case (Sec. 3.5): in
    cylindrical components, with S = sin(2 pi t / P), phi = 2 pi (R - r - l0)/l,
    Z = 2 pi k_z z / L and the region l0 <= R - r <= l0 + l (zero elsewhere),
      F_r = -g kappa B0 (R/r) (k_z l / L) S (1 - cos phi) cos Z cos(k_t theta),
      F_t = g (1 - kappa) B0 (k_z / k_t) (2 pi R / L) S sin phi cos Z sin(k_t theta),
      F_z = -g B0 (R/r) S sin phi sin Z cos(k_t theta),
    returned in Cartesian components [E][np][3] (per unit density). P is
    period * t0, l0 = l0 R, l = lw R. The paper leaves the wavenumbers k_z
    and k_theta open; they are parameters here. It applies the field for
    t < 3 t0."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    r = np.sqrt(x * x + y * y)
    th = np.arctan2(y, x)
    l0, l = l0 * R, lw * R
    inside = (R - r >= l0) & (R - r <= l0 + l)
    rs = np.where(inside, r, R)  # the region keeps r >= R - l0 - l > 0
    S = math.sin(2 * math.pi * t / (period * t0))
    ph = 2 * math.pi * (R - rs - l0) / l
    Zc, Zs = np.cos(kz * 2 * math.pi * z / L), np.sin(kz * 2 * math.pi * z / L)
    Fr = -g * kappa * B0 * (R / rs) * (kz * l / L) * S * (1 - np.cos(ph)) * Zc * np.cos(ktheta * th)
    Ft = g * (1 - kappa) * B0 * (kz / ktheta) * (2 * math.pi * R / L) * S * np.sin(ph) * Zc * np.sin(ktheta * th)
    Fz = -g * B0 * (R / rs) * S * np.sin(ph) * Zs * np.cos(ktheta * th)
    F = np.stack([Fr * np.cos(th) - Ft * np.sin(th), Fr * np.sin(th) + Ft * np.cos(th), Fz], axis=-1)
    return np.where(inside[..., None], F, 0.0)


def case_pipe(N=7, nsq=8, nrad=8, nax=64, R=1.0, L=10.0, Re_tau=180.0, Ma=0.1, pert=0.05, seed=180,
              steps=200, filt="quad", cfl=0.5, init="parabolic") -> Case:
    """Turbulent pipe flow: O-grid, FBB wall at rest, body acceleration
    g = 2 u_tau^2 / R along z. u_b = Ma c_s, u_tau = u_b / 14.7 (the
    bulk-to-friction ratio at Re_tau = 180), nu = u_tau R / Re_tau. Initial
    u_z: init "parabolic", 2 u_b (1 - r^2/R^2), or "law_of_wall", u_tau u+(y+)
    with y+ = (R - r) u_tau / nu (Sec. 3.5); plus a seeded divergence-free
    perturbation of pert * u_b. The perturbation force of Sec. 3.5 is
    pipe_force, set per node by the caller. The default filter is the
    paper's (Sec. 2.2.3): on this curved O-grid the weaker exponential filter
    with cut-off 2N/3 lets the density deviation grow exponentially (orders
    5 and 6 diverge within 2e4 steps of the reduced pipe, FP64 as FP32)."""
    mesh = pipe_mesh(N, nsq, nrad, nax, R, L)
    ub = Ma * CS
    utau = ub / 14.7
    nu = utau * R / Re_tau
    g = 2.0 * utau * utau / R
    dt = stable_dt(mesh, cfl)
    x = mesh.xyz
    r2 = (x[..., 0] ** 2 + x[..., 1] ** 2) / (R * R)
    u = np.zeros(x.shape)
    if init == "parabolic":
        u[..., 2] = 2.0 * ub * np.maximum(0.0, 1.0 - r2)
    elif init == "law_of_wall":
        yplus = np.maximum(R - np.sqrt(r2) * R, 0.0) * utau / nu
        u[..., 2] = utau * law_of_wall(yplus)
    else:
        raise ValueError(init)
    u += pipe_perturbation(x, R, L, pert * ub, seed=seed)
    rho = np.ones(x.shape[:2])
    return Case("pipe", mesh, 27, 1.0, nu, dt, rho, u, steps, g=(0.0, 0.0, g),
                meta=dict(R=R, L=L, ub=ub, utau=utau, Re_tau=Re_tau, g=g, t0=R / utau), **_filter_kw(filt, N))
