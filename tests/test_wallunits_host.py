"""Wall-unit conversion of the pipe statistics (Sec. 3.5), host side: the
wall shear stress of a Poiseuille profile from its exact gradient, and the
law of the wall mapped back onto itself."""
import math

import numpy as np
import pytest

from paper_2509_19171_amd import inputs as I
from paper_2509_19171_amd import wallunits as W


def _cylinder_nodes(R, nz=5, nth=16, rs=(0.3, 0.7, 1.0)):
    th = np.linspace(0, 2 * math.pi, nth, endpoint=False)
    pts = [(r * math.cos(t) + 0.2, r * math.sin(t) - 0.1, z) for r in rs for t in th for z in np.linspace(0, 2, nz)]
    return np.array(pts)[None, :, :] * np.array([R, R, 1.0])  # [1][np][3], axis through (0.2R, -0.1R)


def test_wall_shear_of_poiseuille_profile():
    """u_z = 2 u_b (1 - r^2 / R^2): -du_z/dr = 4 u_b / R at the wall, so
    tau_w = rho0 nu 4 u_b / R exactly (here with the axis off the origin)."""
    R, ub, rho0, nu = 1.5, 0.03, 1.0, 2e-3
    xyz = _cylinder_nodes(R)
    o = np.array([0.2 * R, -0.1 * R, 0.0])
    d = xyz - o
    grad = np.zeros(xyz.shape[:2] + (3, 3))
    grad[..., 2, 0] = -4 * ub * d[..., 0] / R ** 2
    grad[..., 2, 1] = -4 * ub * d[..., 1] / R ** 2
    tau = W.wall_shear(grad, xyz, o, (0, 0, 2.0), R, rho0, nu)
    assert abs(tau - rho0 * nu * 4 * ub / R) < 1e-14
    # the opposite axis orientation flips u_a and its gradient together
    tau2 = W.wall_shear(-grad, xyz, o, (0, 0, -1.0), R, rho0, nu)
    assert abs(tau2 - tau) < 1e-14


def test_wall_shear_needs_wall_nodes():
    xyz = _cylinder_nodes(1.0, rs=(0.5,))
    with pytest.raises(ValueError):
        W.wall_shear(np.zeros(xyz.shape[:2] + (3, 3)), xyz, (0, 0, 0), (0, 0, 1), 1.0, 1.0, 1e-3)


def test_law_of_wall_round_trip():
    """A profile u_tau u+(y+) of the law of the wall comes back as u+(y+)."""
    R, u_tau, nu, rho0 = 1.0, 0.01, 5e-5, 1.0
    r = np.linspace(0.05, 0.95, 10)
    yplus = (R - r) * u_tau / nu
    ubar = u_tau * I.law_of_wall(yplus)
    yp, up, ut = W.to_wall_units(r, ubar, rho0 * u_tau ** 2, rho0, nu, R)
    assert abs(ut - u_tau) < 1e-15
    np.testing.assert_allclose(yp, yplus, rtol=1e-14)
    np.testing.assert_allclose(up, I.law_of_wall(yplus), rtol=1e-14)
    with pytest.raises(ValueError):
        W.to_wall_units(r, ubar, 0.0, rho0, nu, R)


class _FakeSim:
    """radial_profile / velocity_gradient of a fixed state, for the averaging."""

    def __init__(self, s, w, grad):
        self.s, self.w, self.grad = s, w, grad

    def radial_profile(self, origin, axis, rmax, nbins):
        return self.s.copy(), self.w.copy()

    def velocity_gradient(self):
        return self.grad


def test_wall_profile_time_average():
    """Averages over calls: bin means are ratios of summed sums, tau_w the
    mean of the samples; empty bins are dropped."""
    R, ub, rho0, nu = 1.0, 0.02, 1.0, 1e-3
    xyz = _cylinder_nodes(R)
    o = (0.2, -0.1, 0.0)
    grad = np.zeros(xyz.shape[:2] + (3, 3))
    grad[..., 2, 0] = -4 * ub * (xyz[..., 0] - o[0])
    grad[..., 2, 1] = -4 * ub * (xyz[..., 1] - o[1])
    p = W.WallProfile(o, (0, 0, 1), R, 4, rho0, nu)
    p.add(_FakeSim(np.array([1.0, 2.0, 0.0, 3.0]), np.array([1.0, 1.0, 0.0, 2.0]), grad), xyz)
    p.add(_FakeSim(np.array([3.0, 2.0, 0.0, 1.0]), np.array([1.0, 3.0, 0.0, 2.0]), 3 * grad), xyz)
    yp, up, ut = p.result()
    tau = rho0 * nu * 4 * ub * (1 + 3) / 2
    assert abs(ut - math.sqrt(tau / rho0)) < 1e-15
    np.testing.assert_allclose(up * ut, [4.0 / 2.0, 4.0 / 4.0, 4.0 / 4.0], rtol=1e-15)
    np.testing.assert_allclose(yp, (R - np.array([0.125, 0.375, 0.875])) * ut / nu, rtol=1e-14)
