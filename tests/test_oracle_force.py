"""Pins of the oracle's force density per node (F = rho g + F_n, Sec. 2.1;
taken at the collision of each step and frozen for its stages):

- on a uniform state (rho = rho0 everywhere, which the scheme keeps), the
  per-node force rho0 g gives the same run as the body acceleration g;
- on periodic affine meshes streaming and the filter conserve momentum and F**
  carries none, so sum wJ rho u grows by exactly dt sum wJ F_n per step;
- a zero force field is the plain method, bit for bit."""
import math

import numpy as np
import pytest

from conftest import nerr
from paper_2509_19171_amd import inputs as I


def _sim(oracle_mod, mesh, Q, nu=0.01, dt=0.01, **kw):
    return oracle_mod.OracleSim(mesh.dim, mesh.N, mesh.xyz, mesh.gid, mesh.face_tag, mesh.wall_u, Q,
                                1.0, nu, dt, **kw)


def _force_field(mesh, amp=1e-3):
    """A smooth periodic force density, continuous across elements, with a
    mean part (so that its integral does not vanish)."""
    x = mesh.xyz
    comps = [0.3 + np.sin(2 * math.pi * x[..., 1]) * np.cos(2 * math.pi * x[..., 0]),
             -0.2 + np.cos(2 * math.pi * x[..., 0]) + 0.5 * np.sin(2 * math.pi * x[..., 1]),
             0.1 + np.sin(2 * math.pi * (x[..., 0] + x[..., -1]))]
    return amp * np.stack(comps[:mesh.dim], axis=-1)


@pytest.mark.parametrize("dim,Q", [(2, 9), (3, 19)])
def test_uniform_force_equals_body_force(oracle_mod, dim, Q):
    mesh = I.box_mesh(dim, 4, (3,) * dim, (0,) * dim, (1,) * dim, (True,) * dim)
    g = np.array([2e-3, -1e-3, 5e-4][:dim])
    rho = np.ones((mesh.E, mesh.np_))
    u = np.zeros((mesh.E, mesh.np_, dim))
    u[..., 0] = 0.02
    dt = 0.5 * I.min_node_spacing(mesh) / dim
    body = _sim(oracle_mod, mesh, Q, dt=dt, g=tuple(g), filter="quad", filter_kc=2, filter_amp=0.1)
    body.init(rho, u)
    node = _sim(oracle_mod, mesh, Q, dt=dt, filter="quad", filter_kc=2, filter_amp=0.1)
    node.init(rho, u)
    # the force acts from the next step on; start from the same f-bar (its
    # initial -dt F**/2 part includes the body force)
    node.set_f(body.get_f())
    node.set_force(np.broadcast_to(g, (mesh.E, mesh.np_, dim)))
    body.step(20)
    node.step(20)
    assert nerr(node.get_f(), body.get_f()) < 1e-14
    # and the force did act: the momentum grew by 20 dt g (total mass)
    r = body.reduce()
    wJ, _, _ = body.geometry()
    np.testing.assert_allclose(r[1:1 + dim], wJ.sum() * (0.02 * np.eye(dim)[0] + 20 * dt * g), rtol=1e-12)


@pytest.mark.parametrize("dim,Q", [(2, 9), (3, 27)])
def test_force_momentum_balance(oracle_mod, dim, Q):
    mesh = I.box_mesh(dim, 4, (3,) * dim, (0,) * dim, (1,) * dim, (True,) * dim)
    rng = np.random.Generator(np.random.PCG64(61))
    ng = int(mesh.gid.max()) + 1
    rho = 1 + 0.01 * rng.standard_normal(ng)[mesh.gid]
    u = 0.02 * rng.standard_normal((ng, dim))[mesh.gid]
    dt = 0.5 * I.min_node_spacing(mesh) / dim
    s = _sim(oracle_mod, mesh, Q, dt=dt, filter="quad", filter_kc=2, filter_amp=0.1)
    s.init(rho, u)
    F = _force_field(mesh)
    s.set_force(F)
    wJ, _, _ = s.geometry()
    r0 = s.reduce()
    n = 8
    s.step(n)
    r1 = s.reduce()
    expect = n * dt * np.einsum("ep,epk->k", wJ, F)
    assert np.abs(expect).max() > 1e-6
    np.testing.assert_allclose(r1[1:1 + dim] - r0[1:1 + dim], expect, rtol=1e-10, atol=1e-16)
    assert abs(r1[0] - r0[0]) < 1e-13 * r0[0]


def test_zero_force_is_plain(oracle_mod):
    mesh = I.box_mesh(2, 5, (3, 2), (0, 0), (1, 1), (True, True))
    rng = np.random.Generator(np.random.PCG64(62))
    ng = int(mesh.gid.max()) + 1
    rho = 1 + 0.01 * rng.standard_normal(ng)[mesh.gid]
    u = 0.02 * rng.standard_normal((ng, 2))[mesh.gid]
    a = _sim(oracle_mod, mesh, 9, g=(1e-3, 0.0))
    b = _sim(oracle_mod, mesh, 9, g=(1e-3, 0.0))
    a.init(rho, u)
    b.init(rho, u)
    b.set_force(np.zeros((mesh.E, mesh.np_, 2)))
    a.step(10)
    b.step(10)
    np.testing.assert_array_equal(a.get_f(), b.get_f())
    b.set_force(None)
    b.step(1)
    a.step(1)
    np.testing.assert_array_equal(a.get_f(), b.get_f())
