"""Pins of the oracle's discontinuous-Galerkin coupling: element-local mass,
the upwind flux of the entering velocities on interface faces, flux
bounce-back on wall faces.

- A continuous field has no jumps, so the interface flux vanishes and the
  element contributions equal those of the continuous coupling exactly; a
  wrong coincident-node map would leave jumps and fail this.
- On periodic affine meshes the streaming operator satisfies the upwind
  energy identity  sum f.M.L f = -1/2 sum_faces sum_a |n.e_a| w_s J_s [f_a]^2
  (GLL summation by parts for the volume part), with the right-hand side
  computed here from the box geometry alone.
- Mass and momentum are conserved to round-off on periodic affine meshes.
- Pure transport of a smooth field converges spectrally with N.
- Faces that cannot be matched are rejected."""
import math

import numpy as np
import pytest

from conftest import nerr
from paper_2509_19171_amd import inputs as I


def _sim(oracle_mod, mesh, Q, nu=0.01, dt=0.01, **kw):
    return oracle_mod.OracleSim(mesh.dim, mesh.N, mesh.xyz, mesh.gid, mesh.face_tag, mesh.wall_u, Q,
                                1.0, nu, dt, **kw)


def _gll(N):
    """GLL nodes and weights from numpy's Legendre series (independent of the
    oracle's tables)."""
    P = np.polynomial.legendre.Legendre.basis(N)
    x = np.concatenate([[-1.0], np.sort(P.deriv().roots().real), [1.0]])
    w = 2.0 / (N * (N + 1) * P(x) ** 2)
    return x, w


def _curved_periodic(x):
    out = x.copy()
    out[..., 0] = x[..., 0] + 0.03 * np.sin(2 * math.pi * x[..., 1]) * np.sin(2 * math.pi * x[..., 0])
    out[..., 1] = x[..., 1] + 0.03 * np.sin(2 * math.pi * x[..., 0]) * np.cos(2 * math.pi * x[..., 1])
    return out


def _warp3(x):  # periodic in x and z, flat walls at y = 0, 1
    out = x.copy()
    out[..., 0] += 0.02 * np.sin(2 * math.pi * x[..., 2] / 1.5)
    out[..., 1] += 0.02 * np.sin(math.pi * x[..., 1]) * np.sin(2 * math.pi * x[..., 0])
    out[..., 2] += 0.02 * np.sin(2 * math.pi * x[..., 0])
    return out


def _meshes_with_walls():
    return {
        "channel2d": I.box_mesh(2, 6, (4, 3), (0, 0), (2, 1), (True, False), wall_tags={1: (1, 2)},
                                wall_u=[[0, 0], [0.05, 0]], warp=None),
        "curved2d": I.box_mesh(2, 5, (3, 3), (0, 0), (1, 1), (True, True), warp=_curved_periodic),
        "box3d": I.box_mesh(3, 4, (2, 2, 3), (0, 0, 0), (1, 1, 1.5), (True, False, True), wall_tags={1: (1, 2)},
                            wall_u=[[0, 0, 0], [0.02, 0, 0.01]], warp=_warp3),
    }


@pytest.mark.parametrize("name", list(_meshes_with_walls()))
def test_continuous_field_has_no_interface_flux(oracle_mod, name):
    mesh = _meshes_with_walls()[name]
    Q = 9 if mesh.dim == 2 else 19
    rng = np.random.Generator(np.random.PCG64(31))
    ng = int(mesh.gid.max()) + 1
    f = rng.standard_normal((ng, Q))[mesh.gid].transpose(0, 2, 1).copy()
    cg = _sim(oracle_mod, mesh, Q).rhs_local(f)
    dg = _sim(oracle_mod, mesh, Q, coupling="dg").rhs_local(f)
    assert np.abs(dg - cg).max() == 0.0
    # a discontinuous field does feel the interface flux
    g = f + 0.1 * rng.standard_normal(f.shape)
    assert nerr(_sim(oracle_mod, mesh, Q, coupling="dg").rhs_local(g), _sim(oracle_mod, mesh, Q).rhs_local(g)) > 1e-3


def _box_jump_energy(mesh, f, e, N):
    """-1/2 sum over interfaces of |n.e_a| w_s J_s (f_A - f_B)^2 on a periodic
    axis-aligned box mesh, from the node coordinates only."""
    dim = mesh.dim
    n1 = N + 1
    _, w = _gll(N)
    xyz = mesh.xyz
    E = xyz.shape[0]
    lo = xyz.reshape(-1, dim).min(axis=0)
    hi = xyz.reshape(-1, dim).max(axis=0)
    corner = xyz[:, 0, :]
    h = xyz[:, -1, :] - xyz[:, 0, :]
    nel = np.rint((hi - lo) / h[0]).astype(int)
    idx = np.rint((corner - lo) / h[0]).astype(int)
    where = {tuple(v): el for el, v in enumerate(idx)}
    shape = (n1,) * dim
    total = 0.0
    for el in range(E):
        fe = f[el].reshape((f.shape[1],) + shape[::-1])  # [Q][k][j][i] (r fastest)
        for m in range(dim):
            nb = idx[el].copy()
            nb[m] = (nb[m] + 1) % nel[m]
            fb = f[where[tuple(nb)]].reshape((f.shape[1],) + shape[::-1])
            ax = dim - m  # axis of index m in [Q][..][i]
            fa_face = np.take(fe, N, axis=ax)
            fb_face = np.take(fb, 0, axis=ax)
            tang = [t for t in range(dim) if t != m]
            wt = np.ones(fa_face.shape[1:])
            for t in tang:
                at = dim - 1 - t - (1 if t < m else 0)  # axis of index t in the face array (after dropping m)
                sh = [1] * wt.ndim
                sh[at] = n1
                wt = wt * (w * h[el][t] / 2).reshape(sh)
            for a in range(f.shape[1]):
                total += -0.5 * abs(e[a, m]) * np.sum(wt * (fa_face[a] - fb_face[a]) ** 2)
    return total


@pytest.mark.parametrize("dim,Q,N", [(2, 9, 4), (3, 27, 3), (3, 19, 4)])
def test_upwind_energy_identity(oracle_mod, dim, Q, N):
    mesh = I.box_mesh(dim, N, (3,) * dim if dim == 3 else (3, 4), (0,) * dim, (1.0, 1.5, 0.8)[:dim], (True,) * dim)
    rng = np.random.Generator(np.random.PCG64(41))
    f = rng.standard_normal((mesh.E, Q, (N + 1) ** dim))
    s = _sim(oracle_mod, mesh, Q, coupling="dg")
    rt = s.rhs_local(f)
    lhs = float(np.sum(f * rt))
    e, _, _ = oracle_mod.lattice(dim, Q)
    rhs = _box_jump_energy(mesh, f, e, N)
    assert rhs < 0
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)
    # with the continuous coupling the same sum vanishes for continuous fields
    # only; for this discontinuous field it differs
    assert abs(float(np.sum(f * _sim(oracle_mod, mesh, Q).rhs_local(f))) - rhs) > 1e-3 * abs(rhs)


@pytest.mark.parametrize("dim,Q", [(2, 9), (3, 27)])
def test_dg_conservation(oracle_mod, dim, Q):
    """Mass and momentum to round-off on periodic affine meshes from a
    discontinuous start (collision, upwind streaming, the k_c >= 2 filter)."""
    mesh = I.box_mesh(dim, 4, (3,) * dim, (0,) * dim, (1,) * dim, (True,) * dim)
    rng = np.random.Generator(np.random.PCG64(51))
    rho = 1 + 0.01 * rng.standard_normal((mesh.E, mesh.np_))
    u = 0.02 * rng.standard_normal((mesh.E, mesh.np_, dim))
    dt = 0.5 * I.min_node_spacing(mesh) / dim
    s = _sim(oracle_mod, mesh, Q, nu=0.01, dt=dt, filter="quad", filter_kc=2, filter_amp=0.1, coupling="dg")
    s.init(rho, u)
    r0 = s.reduce()
    s.step(10)
    r1 = s.reduce()
    assert abs(r1[0] - r0[0]) < 1e-13 * r0[0]
    assert np.abs(r1[1:1 + dim] - r0[1:1 + dim]).max() < 1e-14
    # the lumped mass is the element's own: every copy of a node counts once
    wJ, _, _ = s.geometry()
    np.testing.assert_array_equal(s.mass(), wJ)


def test_dg_transport_spectral_convergence(oracle_mod):
    errs = []
    for N in (3, 5, 7):
        mesh = I.box_mesh(2, N, (4, 4), (0, 0), (2 * math.pi, 2 * math.pi), (True, True))
        dt = 0.25 * I.min_node_spacing(mesh) / 2
        s = _sim(oracle_mod, mesh, 9, dt=dt, coupling="dg")
        e, _, _ = oracle_mod.lattice(2, 9)
        x = mesh.xyz

        def field(t):
            return np.stack([np.sin(x[..., 0] - e[a, 0] * t) * np.cos(x[..., 1] - e[a, 1] * t) + 0.3 *
                             np.cos(2 * (x[..., 0] - e[a, 0] * t)) for a in range(9)], axis=1)

        s.set_f(field(0.0))
        s.advect(int(round(0.5 / dt)))
        errs.append(nerr(s.get_f(), field(s.time)))
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    assert errs[2] < 2e-5


def test_dg_rejects_unmatched_faces(oracle_mod):
    # one element along a periodic direction: a face repeats node ids
    m1 = I.box_mesh(2, 4, (1, 3), (0, 0), (1, 1), (True, True))
    with pytest.raises(ValueError):
        _sim(oracle_mod, m1, 9, coupling="dg")
    # open boundary faces (tag 0, no partner)
    m2 = I.box_mesh(2, 4, (2, 2), (0, 0), (1, 1), (False, False), wall_tags={0: (0, 0), 1: (0, 0)})
    with pytest.raises(ValueError):
        _sim(oracle_mod, m2, 9, coupling="dg")
    # the continuous coupling accepts both
    _sim(oracle_mod, m1, 9)
    _sim(oracle_mod, m2, 9)


def test_dg_dissipates_more_than_cg(oracle_mod):
    """The upwind interface flux damps an under-resolved 2D Taylor-Green
    vortex more than the continuous coupling on the same mesh: the kinetic
    energy of the DG run ends below the CG run's, both below the start."""
    c = I.case_tgv2d(nel=4, N=4, Re=2000.0, steps=0)
    ke = {}
    for coupling in ("cg", "dg"):
        s = oracle_mod.from_case(c, coupling=coupling)
        k0 = s.reduce()[-1]
        s.step(300)
        ke[coupling] = s.reduce()[-1] / k0
    assert 0 < ke["dg"] < ke["cg"] < 1
