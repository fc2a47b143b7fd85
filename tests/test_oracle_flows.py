"""End-to-end pins of the oracle against the mathematics: Runge-Kutta
amplification polynomials, analytic flows (Taylor-Green decay, start-up
Couette and Poiseuille with FBB walls, straight and curved) and the 3D
Taylor-Green initial dissipation rate."""
import math

import numpy as np
import pytest

from conftest import nerr
from paper_2509_19171_amd import inputs as I


# ------------------------------------------------------------ time marching --
@pytest.mark.parametrize("z", [-0.7, -0.3, 0.2, -1.5])
def test_rk_amplification(oracle_mod, z):
    """Linear ODE y' = lam y: SSPRK3 gives R(z) = 1 + z + z^2/2 + z^3/6; the
    printed four-stage form gives the fourth-order Taylor polynomial."""
    T3 = 1 + z + z * z / 2 + z ** 3 / 6
    T4 = T3 + z ** 4 / 24
    assert abs(oracle_mod.rk_scalar("ssprk3", z, 0.0, 1.0, 1.0, 1) - T3) < 1e-15
    assert abs(oracle_mod.rk_scalar("printed4", z, 0.0, 1.0, 1.0, 1) - T4) < 1e-15


@pytest.mark.parametrize("z", [-0.7, 0.0, -0.2])
def test_rk_affine_forcing(oracle_mod, z):
    """Affine ODE y' = lam y + b from y = 0 over dt = 1: the constant part is
    integrated with the Taylor polynomial of phi_1(z) = (e^z - 1)/z of the
    scheme's order (exact dt b when lam = 0)."""
    b = 0.37
    p3 = b * (1 + z / 2 + z * z / 6)
    p4 = p3 + b * z ** 3 / 24
    assert abs(oracle_mod.rk_scalar("ssprk3", z, b, 0.0, 1.0, 1) - p3) < 1e-15
    assert abs(oracle_mod.rk_scalar("printed4", z, b, 0.0, 1.0, 1) - p4) < 1e-15


def test_rk_convergence_order(oracle_mod):
    lam, T = -1.3, 1.0
    e3 = [abs(oracle_mod.rk_scalar("ssprk3", lam, 0.0, 1.0, T / n, n) - math.exp(lam * T)) for n in (10, 20)]
    e4 = [abs(oracle_mod.rk_scalar("printed4", lam, 0.0, 1.0, T / n, n) - math.exp(lam * T)) for n in (10, 20)]
    assert 2.8 < math.log2(e3[0] / e3[1]) < 3.2
    assert 3.8 < math.log2(e4[0] / e4[1]) < 4.2


# ------------------------------------------------------------------ flows ----
def test_tgv2d_decay(oracle_mod):
    """2D Taylor-Green vortex (D2Q9, 8x8 elements, N = 5, 200 steps): the
    velocity field follows u0 exp(-2 nu t) and the kinetic energy decays at
    the rate 4 nu; mass is conserved to round-off."""
    c = I.case_tgv2d()
    s = oracle_mod.from_case(c)
    m0 = s.reduce()[0]
    s.step(50)
    t1, k1 = s.time, s.reduce()[-1]
    s.step(150)
    t2, k2 = s.time, s.reduce()[-1]
    rate = -math.log(k2 / k1) / (t2 - t1)
    assert abs(rate / (4 * c.nu) - 1) < 0.02, rate
    _, u = s.moments()
    ue = I.tgv2d_fields(c.xyz, c.meta["u0"], t=s.time, nu=c.nu)[1]
    assert nerr(u, ue) < 2e-3
    assert abs(s.reduce()[0] - m0) < 1e-13 * m0


def test_tgv3d_initial_dissipation(oracle_mod):
    """3D Taylor-Green vortex: all initial modes have |k|^2 = 3, so the
    kinetic energy initially decays at 6 nu (no filter, Re = 100)."""
    c = I.case_tgv3d(nel=4, N=5, Re=100.0, steps=0, filt=None)
    s = oracle_mod.from_case(c)
    s.step(10)
    t1, k1 = s.time, s.reduce()[-1]
    s.step(30)
    t2, k2 = s.time, s.reduce()[-1]
    rate = -math.log(k2 / k1) / (t2 - t1)
    assert abs(rate / (6 * c.nu) - 1) < 0.05, rate


@pytest.mark.parametrize("curved", [False, True])
def test_couette_startup(oracle_mod, curved):
    """Start-up Couette flow with FBB walls (moving top wall) follows the
    Fourier-series solution; the curved mesh is about as accurate as the
    straight one."""
    c = I.case_couette(nelx=2, nely=4, N=6, curved=curved)
    s = oracle_mod.from_case(c)
    s.step(2000)
    _, u = s.moments()
    ue = I.couette_profile(c.xyz[..., 1], s.time, c.meta["U"], 1.0, c.nu)
    assert nerr(u[..., 0], ue) < 2e-3
    assert np.abs(u[..., 1]).max() < 2e-3 * c.meta["U"]


@pytest.mark.parametrize("curved", [False, True])
def test_poiseuille_startup(oracle_mod, curved):
    """Body-force driven plane Poiseuille start-up between FBB walls follows
    the series solution."""
    c = I.case_poiseuille(nelx=2, nely=4, N=6, curved=curved)
    s = oracle_mod.from_case(c)
    s.step(3000)
    _, u = s.moments()
    ue = I.poiseuille_profile(c.xyz[..., 1], s.time, c.g[0], 1.0, c.nu)
    assert nerr(u[..., 0], ue) < 4e-3


def test_couette_converges_with_order(oracle_mod):
    """The error against the analytic solution falls as N grows (until the
    time error saturates)."""
    errs = []
    for N in (2, 4):
        c = I.case_couette(nelx=1, nely=3, N=N, Re=10.0)
        s = oracle_mod.from_case(c)
        nst = int(round(1.0 / c.dt))
        s.step(nst)
        _, u = s.moments()
        ue = I.couette_profile(c.xyz[..., 1], s.time, c.meta["U"], 1.0, c.nu)
        errs.append(nerr(u[..., 0], ue))
    assert errs[1] < 0.5 * errs[0], errs
