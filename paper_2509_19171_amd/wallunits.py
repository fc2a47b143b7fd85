"""Pipe statistics in wall units (Sec. 3.5): the wall shear stress from the
velocity gradient at the wall nodes, the friction velocity, and the time- and
space-averaged axial velocity as u+ against y+.

The per-node velocity gradient and the radial bin sums are computed on the
device (sel_velocity_gradient, sel_radial_profile); this module only
accumulates them over calls and converts the averages:
  tau_w = rho0 nu (-d u_a / d r) at r = R,   u_tau = sqrt(tau_w / rho0),
  y+ = (R - r) u_tau / nu,                   u+ = u_a / u_tau,
with u_a = u . n the axial velocity and r the distance from the pipe axis.
"""
from __future__ import annotations

import numpy as np


def _radial_frame(xyz, origin, axis):
    n = np.asarray(axis, dtype=np.float64)
    n = n / np.linalg.norm(n)
    d = np.asarray(xyz, dtype=np.float64) - np.asarray(origin, dtype=np.float64)
    rv = d - (d @ n)[..., None] * n
    r = np.linalg.norm(rv, axis=-1)
    return n, rv, r


def wall_shear(grad, xyz, origin, axis, R, rho0, nu, tol=1e-9):
    """Mean wall shear stress rho0 nu (-d u_a / d r) over the element copies of
    the nodes on the wall r = R. grad [E][np][dim][dim] holds du_c/dx_q (as
    sel_velocity_gradient returns it), xyz [E][np][dim] the node coordinates."""
    n, rv, r = _radial_frame(xyz, origin, axis)
    wall = np.abs(r - R) < tol * R
    if not wall.any():
        raise ValueError("no element node lies on the wall r = R")
    er = rv[wall] / r[wall][:, None]
    dua_dx = np.einsum("c,kcq->kq", n, np.asarray(grad)[wall])  # d u_a / d x_q
    dua_dr = np.einsum("kq,kq->k", dua_dx, er)
    return float(rho0 * nu * np.mean(-dua_dr))


def to_wall_units(r_centers, ubar, tau_w, rho0, nu, R):
    """(y+, u+, u_tau) of a mean axial velocity profile ubar at radii r_centers."""
    if not tau_w > 0.0:
        raise ValueError("wall units need a positive wall shear stress")
    u_tau = float(np.sqrt(tau_w / rho0))
    yplus = (R - np.asarray(r_centers, dtype=np.float64)) * u_tau / nu
    uplus = np.asarray(ubar, dtype=np.float64) / u_tau
    return yplus, uplus, u_tau


class WallProfile:
    """Time average of the pipe's axial velocity profile and wall shear stress
    over the calls of add(), in wall units. nbins equal radial bins of [0, R)
    (the wall nodes themselves, r = R, fall outside)."""

    def __init__(self, origin, axis, R, nbins, rho0, nu):
        self.origin, self.axis, self.R, self.nbins = origin, axis, float(R), int(nbins)
        self.rho0, self.nu = float(rho0), float(nu)
        self.sums = np.zeros(self.nbins)
        self.weights = np.zeros(self.nbins)
        self.tau_sum = 0.0
        self.count = 0

    def add(self, sim, xyz):
        """Accumulate the current state of sim (node coordinates xyz)."""
        s, w = sim.radial_profile(self.origin, self.axis, self.R, self.nbins)
        self.sums += s
        self.weights += w
        self.tau_sum += wall_shear(sim.velocity_gradient(), xyz, self.origin, self.axis, self.R, self.rho0, self.nu)
        self.count += 1

    def result(self):
        """(y+, u+, u_tau) at the centres of the bins that hold nodes."""
        if self.count == 0:
            raise ValueError("no samples")
        keep = self.weights > 0
        r_c = (np.arange(self.nbins) + 0.5) * self.R / self.nbins
        ubar = self.sums[keep] / self.weights[keep]
        return to_wall_units(r_c[keep], ubar, self.tau_sum / self.count, self.rho0, self.nu, self.R)
