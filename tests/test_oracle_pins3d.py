"""Pins of oracle parts that only 3D or the printed time marching reach,
each against mathematics that does not run through the oracle itself:

- the printed four-stage field integrator (Sec. 2.2.2, stage formulas RK1-RK4
  with L applied linearly): pure periodic transport converges at fourth
  order in dt, and under a body force the momentum of a periodic affine mesh
  grows by exactly dt F per step;
- the 3D flux bounce-back area vectors (Sec. 2.2.1, the wall flux and its
  jump): a disturbed state keeps its total mass to round-off in straight and
  skewed affine boxes with walls on every face family and on the warped box
  of the 3D parity cases, to quadrature accuracy (falling spectrally with N)
  under a fully 3D warp, and start-up Couette flow with the moving
  wall normal to each of r, s and t follows the series solution;
- the kinetic-energy, mass and momentum integrals (Sec. 3.4): closed forms of
  the 2D and 3D Taylor-Green initial fields;
- the 3D tensor filter (Sec. 2.2.3): a separable mode phi_a(r) phi_b(s)
  phi_c(t) of the filter basis is scaled by sigma_a sigma_b sigma_c, which
  fails if any of the three directions is skipped, repeated or transposed."""
import math

import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

from conftest import nerr
from paper_2509_19171_amd import inputs as I

CS = 3 ** -0.5
SKEW = np.array([[1.0, 0.3, 0.1], [-0.2, 0.9, 0.2], [0.1, 0.05, 1.1]])


def _sim(oracle_mod, mesh, Q, nu=0.01, dt=0.01, **kw):
    return oracle_mod.OracleSim(mesh.dim, mesh.N, mesh.xyz, mesh.gid, mesh.face_tag, mesh.wall_u, Q,
                                1.0, nu, dt, **kw)


# ------------------------------------------------- printed four-stage form --
def test_printed4_transport_fourth_order_in_time(oracle_mod):
    """Streaming alone on a periodic box with the printed stages: the error of
    exact transport falls 16x per halving of dt (spatial error negligible at
    N = 12); SSPRK3 on the same case falls 8x."""
    mesh = I.box_mesh(2, 12, (2, 2), (0, 0), (2 * math.pi, 2 * math.pi), (True, True))
    e, _, _ = oracle_mod.lattice(2, 9)
    x = mesh.xyz
    T = 0.6

    def field(t):
        return np.stack([np.sin(x[..., 0] - e[a, 0] * t + x[..., 1] - e[a, 1] * t) for a in range(9)], axis=1)

    rates = {}
    for rk in ("printed4", "ssprk3"):
        errs = []
        for nst in (20, 40):
            s = _sim(oracle_mod, mesh, 9, dt=T / nst, rk=rk)
            s.set_f(field(0.0))
            s.advect(nst)
            errs.append(nerr(s.get_f(), field(T)))
        rates[rk] = math.log2(errs[0] / errs[1])
    assert 3.7 < rates["printed4"] < 4.3, rates
    assert 2.7 < rates["ssprk3"] < 3.3, rates


@pytest.mark.parametrize("dim,Q", [(2, 9), (3, 27)])
def test_printed4_momentum_gain_under_body_force(oracle_mod, dim, Q):
    """Printed stages with a body acceleration on a periodic affine mesh and a
    disturbed state: the streaming part adds no momentum and the constant part
    of L is weighted to one over the step, so sum wJ rho u grows by exactly
    dt g (total mass) per step and mass stays constant."""
    mesh = I.box_mesh(dim, 4, (3,) * dim, (0,) * dim, (1,) * dim, (True,) * dim)
    rng = np.random.Generator(np.random.PCG64(31))
    ng = int(mesh.gid.max()) + 1
    rho = 1 + 0.01 * rng.standard_normal(ng)[mesh.gid]
    u = 0.02 * rng.standard_normal((ng, dim))[mesh.gid]
    dt = 0.5 * I.min_node_spacing(mesh) / dim
    g = np.array([1e-3, 2e-3, -1e-3][:dim])
    s = _sim(oracle_mod, mesh, Q, nu=0.01, dt=dt, g=tuple(g), filter="quad", filter_kc=2, filter_amp=0.1,
             rk="printed4")
    s.init(rho, u)
    r0 = s.reduce()
    s.step(5)
    r1 = s.reduce()
    assert abs(r1[0] - r0[0]) < 1e-13 * r0[0]
    np.testing.assert_allclose(r1[1:1 + dim] - r0[1:1 + dim], 5 * dt * g * r0[0], rtol=1e-10, atol=1e-16)


# ------------------------------------------------------- 3D wall fluxes -----
def _disturbed_mass_drift(oracle_mod, mesh, Q, steps=30, seed=11, filt=True):
    rng = np.random.Generator(np.random.PCG64(seed))
    ng = int(mesh.gid.max()) + 1
    rho = 1 + 0.01 * rng.standard_normal(ng)[mesh.gid]
    u = 0.02 * rng.standard_normal((ng, mesh.dim))[mesh.gid]
    kw = dict(filter="quad", filter_kc=2, filter_amp=0.1) if filt else {}
    s = _sim(oracle_mod, mesh, Q, nu=0.01, dt=I.stable_dt(mesh), **kw)
    s.init(rho, u)
    m0 = s.reduce()[0]
    s.step(steps)
    return abs(s.reduce()[0] - m0) / m0


def _closed_box(N, warp=None):
    return I.box_mesh(3, N, (2, 2, 2), (0, 0, 0), (1, 1, 1), (False, False, False),
                      wall_tags={0: (1, 2), 1: (3, 4), 2: (5, 6)}, warp=warp)


@pytest.mark.parametrize("Q", [19, 27])
@pytest.mark.parametrize("kind", ["channel", "closed", "closed_skew"])
def test_3d_wall_flux_conserves_mass(oracle_mod, Q, kind):
    """On affine elements the incoming-only flux with the bounce-back jump
    sums, over the velocities at a wall node, to n.j, which cancels the
    boundary term of the GLL-exact streaming operator: total mass is constant
    to round-off. The closed boxes put walls on all six faces (r-, s- and
    t-face families, with edges and corners where walls meet); the skewed box
    makes every component of the area vector non-zero, so a wrong sign or
    cyclic order in any face family shows as a mass change of order 1e-3."""
    if kind == "channel":
        mesh = I.box_mesh(3, 4, (2, 3, 2), (0, 0, 0), (1, 1, 1), (True, False, True), wall_tags={1: (1, 2)},
                          wall_u=[[0, 0, 0], [0.03, 0, 0.01]])
    elif kind == "closed":
        mesh = _closed_box(4)
    else:
        mesh = _closed_box(4, warp=lambda x: x @ SKEW.T + 0.1)
    assert _disturbed_mass_drift(oracle_mod, mesh, Q) < 2e-14


def _warp_box3d(x):  # periodic in x and z, flat walls at y = 0, 1 (the mesh of the 3D parity cases)
    out = x.copy()
    out[..., 0] += 0.02 * np.sin(2 * math.pi * x[..., 2] / 1.5)
    out[..., 1] += 0.02 * np.sin(math.pi * x[..., 1]) * np.sin(2 * math.pi * x[..., 0])
    out[..., 2] += 0.02 * np.sin(2 * math.pi * x[..., 0])
    return out


def _warp_full3d(x):  # every displacement varies with all three coordinates; walls at y = 0, 1 stay flat
    out = x.copy()
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    out[..., 0] += 0.03 * np.sin(2 * math.pi * (X + Z / 1.5)) * (1 + 0.5 * Y)
    out[..., 1] += 0.03 * np.sin(math.pi * Y) * np.sin(2 * math.pi * X) * np.cos(2 * math.pi * Z / 1.5)
    out[..., 2] += 0.03 * np.sin(2 * math.pi * X) * np.cos(math.pi * Y)
    return out


def _curved_box(N, warp):
    return I.box_mesh(3, N, (2, 2, 3), (0, 0, 0), (1, 1, 1.5), (True, False, True), wall_tags={1: (1, 2)},
                      wall_u=[[0, 0, 0], [0.02, 0, 0.01]], warp=warp)


def test_3d_curved_walls_mass(oracle_mod):
    """Curved 3D elements, no filter (the filter keeps the reference-space
    integral, which equals the physical one only on affine elements). On the
    warped box of the 3D parity cases mass stays constant to round-off; under
    a warp in which every displacement varies with all three coordinates the
    discrete metric identity holds only to quadrature accuracy, and the
    drift falls spectrally with N. A wrong area vector would give a drift of
    order 1e-3 at every N."""
    for Q in (19, 27):
        assert _disturbed_mass_drift(oracle_mod, _curved_box(4, _warp_box3d), Q, filt=False) < 2e-14
    x = None
    drift = []
    for N in (3, 5, 7):
        mesh = _curved_box(N, _warp_full3d)
        x = mesh.xyz
        rho = 1 + 0.01 * np.sin(2 * math.pi * x[..., 0]) * np.cos(math.pi * x[..., 1]) * \
            np.cos(2 * math.pi * x[..., 2] / 1.5)
        u = np.stack([0.02 * np.cos(2 * math.pi * x[..., 2] / 1.5) * np.cos(math.pi * x[..., 1]),
                      0.01 * np.sin(2 * math.pi * x[..., 0]), 0.02 * np.sin(math.pi * x[..., 1])], -1)
        s = _sim(oracle_mod, mesh, 27, nu=0.01, dt=0.002)
        s.init(rho, u)
        m0 = s.reduce()[0]
        s.step(20)
        drift.append(abs(s.reduce()[0] - m0) / m0)
    assert drift[0] < 1e-7 and drift[1] < 0.1 * drift[0] and drift[2] < 0.05 * drift[1], drift


def _couette3d(axis, N=5, nel=4, Re=10.0, Ma=0.1):
    """Channel of height 1 between walls normal to axis 'axis' (periodic in
    the other two); the wall at the top moves along the next axis."""
    U = Ma * CS
    nels = [1, 1, 1]
    nels[axis] = nel
    per = [True, True, True]
    per[axis] = False
    hi = [0.5, 0.5, 0.5]
    hi[axis] = 1.0
    mv = (axis + 1) % 3
    ub = [0.0, 0.0, 0.0]
    ub[mv] = U
    mesh = I.box_mesh(3, N, nels, (0, 0, 0), hi, per, wall_tags={axis: (1, 2)}, wall_u=[[0, 0, 0], ub])
    return mesh, U, U / Re, mv


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_3d_couette_startup_each_face_family(oracle_mod, axis):
    """Start-up Couette flow (D3Q27, N = 5) with the moving wall on the r-,
    s- or t-faces follows the Fourier-series solution as closely as the 2D
    case does, and the flow stays in the wall's direction."""
    mesh, U, nu, mv = _couette3d(axis)
    s = _sim(oracle_mod, mesh, 27, nu=nu, dt=I.stable_dt(mesh))
    rho, u = I.rest_fields(mesh.xyz)
    s.init(rho, u)
    s.step(1000)
    _, uu = s.moments()
    ue = I.couette_profile(mesh.xyz[..., axis], s.time, U, 1.0, nu)
    assert nerr(uu[..., mv], ue) < 2.5e-3
    others = [k for k in range(3) if k != mv]
    assert np.abs(uu[..., others]).max() < 1e-12 * U


# --------------------------------------------------------- reductions ------
def test_reduce_closed_forms_tgv2d(oracle_mod):
    """2D Taylor-Green initial field on [0, 2 pi]^2: kinetic energy
    sum wJ rho0 |u|^2 / 2 = pi^2 u0^2 rho0, mass (2 pi)^2 rho0 (the pressure
    term has zero mean), momentum 0 (GLL quadrature of these trigonometric
    fields is exact to round-off here)."""
    c = I.case_tgv2d(filt="quad")
    r = oracle_mod.from_case(c).reduce()
    u0 = c.meta["u0"]
    assert abs(r[-1] - math.pi ** 2 * u0 ** 2 * c.rho0) < 1e-12 * math.pi ** 2 * u0 ** 2
    assert abs(r[0] - (2 * math.pi) ** 2 * c.rho0) < 1e-12 * (2 * math.pi) ** 2
    assert np.abs(r[1:3]).max() < 1e-14


def test_reduce_closed_forms_tgv3d(oracle_mod):
    """3D Taylor-Green initial field on [0, 2 pi]^3: kinetic energy
    pi^3 u0^2 rho0, mass (2 pi)^3 rho0, momentum 0."""
    c = I.case_tgv3d(nel=4, N=5, steps=0)
    r = oracle_mod.from_case(c).reduce()
    u0 = c.meta["u0"]
    assert abs(r[-1] - math.pi ** 3 * u0 ** 2 * c.rho0) < 1e-12 * math.pi ** 3 * u0 ** 2
    assert abs(r[0] - (2 * math.pi) ** 3 * c.rho0) < 1e-12 * (2 * math.pi) ** 3
    assert np.abs(r[1:4]).max() < 1e-14


def test_reduce_uses_reference_density_and_lumped_mass(oracle_mod):
    """A uniform state rho = 1.3, u = (0.1, -0.2, 0.05) on a skewed affine box
    of volume det A: mass 1.3 det A, momentum 1.3 u det A, and kinetic energy
    rho0 |u|^2 det A / 2 with the reference density rho0 = 1 (not rho)."""
    mesh = I.box_mesh(3, 3, (2, 1, 2), (0, 0, 0), (1, 1, 1), (True, True, True), warp=lambda x: x @ SKEW.T)
    s = _sim(oracle_mod, mesh, 27)
    u = np.array([0.1, -0.2, 0.05])
    s.init(np.full((mesh.E, mesh.np_), 1.3), np.tile(u, (mesh.E, mesh.np_, 1)))
    r = s.reduce()
    V = np.linalg.det(SKEW)
    np.testing.assert_allclose(r[0], 1.3 * V, rtol=1e-13)
    np.testing.assert_allclose(r[1:4], 1.3 * u * V, rtol=1e-12)
    np.testing.assert_allclose(r[4], 0.5 * (u @ u) * V, rtol=1e-12)


# ------------------------------------------------------- 3D tensor filter --
def _phi(k, x):
    """Filter basis phi_0 = L_0, phi_1 = L_1, phi_k = L_k - L_{k-2}."""
    c = np.zeros(k + 1)
    c[k] = 1.0
    if k >= 2:
        c[k - 2] = -1.0
    return npleg.legval(x, c)


@pytest.mark.parametrize("ftype,kc,amp,order", [("quad", 2, 0.1, 2.0), ("exp", 3, 36.0, 16.0)])
def test_3d_filter_scales_separable_modes(oracle_mod, ftype, kc, amp, order):
    """On every element of a 3D mesh and for every velocity, the nodal values
    of phi_a(r) phi_b(s) phi_c(t) come out scaled by sigma_a sigma_b sigma_c;
    the velocities carry different (a, b, c), so a skipped, doubled or
    transposed direction fails."""
    N = 5
    mesh = I.box_mesh(3, N, (2, 1, 1), (0, 0, 0), (1, 1, 1), (True, True, True))
    Q = 27
    s = _sim(oracle_mod, mesh, Q, filter=ftype, filter_kc=kc, filter_amp=amp, filter_order=order)
    xi = np.sort(np.concatenate([[-1.0, 1.0], npleg.Legendre.basis(N).deriv().roots().real]))
    sigma = oracle_mod.filter_sigma(N, ftype, kc, amp, order)
    n1 = N + 1
    p = np.arange(n1 ** 3)
    ii, jj, kk = p % n1, (p // n1) % n1, p // (n1 * n1)
    rng = np.random.Generator(np.random.PCG64(4))
    modes = rng.integers(0, N + 1, size=(Q, 3))
    modes[0] = (N, N - 1, kc + 1)
    modes[1] = (kc + 1, N, N - 1)
    modes[2] = (N - 1, kc + 1, N)
    f = np.zeros((mesh.E, Q, n1 ** 3))
    exp = np.zeros_like(f)
    for a, (ma, mb, mc) in enumerate(modes):
        v = _phi(ma, xi[ii]) * _phi(mb, xi[jj]) * _phi(mc, xi[kk])
        f[:, a, :] = v
        exp[:, a, :] = sigma[ma] * sigma[mb] * sigma[mc] * v
    out = s.filter(f)
    assert np.abs(out - exp).max() < 1e-13
    # the three test modes are changed by the filter (the check is not vacuous)
    assert np.abs(exp[:, :3] - f[:, :3]).max() > 1e-3
