"""Velocity-gradient diagnostics on the GPU (sel_velocity_gradient): parity
with the FP64 oracle, the initial dissipation of the 3D Taylor-Green vortex,
and the wall shear stress of channel and pipe profiles (Sec. 3.4, 3.5)."""
import math
import sys

import numpy as np
import pytest

from paper_2509_19171_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2509_19171_amd import sel

    sel.load()
    yield


def _warp(x):
    out = x.copy()
    out[..., 0] += 0.02 * np.sin(2 * math.pi * x[..., 2] / 1.5)
    out[..., 1] += 0.02 * np.sin(math.pi * x[..., 1]) * np.sin(2 * math.pi * x[..., 0])
    out[..., 2] += 0.02 * np.sin(2 * math.pi * x[..., 0])
    return out


def _box():
    m = I.box_mesh(3, 5, (2, 2, 3), (0, 0, 0), (1, 1, 1.5), (True, False, True), wall_tags={1: (1, 2)},
                   wall_u=[[0, 0, 0], [0.02, 0, 0.01]], warp=_warp)
    r, u = I.rest_fields(m.xyz)
    c = I.Case("box", m, 19, 1.0, 0.01, I.stable_dt(m), r, u, 0, filter="quad", filter_kc=2, filter_amp=0.1)
    c.rho, c.u = I.random_state(c, seed=8, amp=0.01)
    return c


CASES = {
    "channel_curved_N7": lambda: I.case_couette(nelx=4, nely=3, N=7, curved=True, filt="exp"),
    "box3d_q19_walls_N5": _box,
    "tgv3d_q27_N4": lambda: I.case_tgv3d(nel=3, N=4, Q=27, Re=200.0, steps=0, filt="quad"),
}


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32dev", 2e-5)])
@pytest.mark.parametrize("name", list(CASES))
def test_velocity_gradient_parity(name, prec, tol):
    import oracle
    from oracle import closure as C
    from paper_2509_19171_amd import sel

    c = CASES[name]()
    g = sel.from_case(c, prec)
    o = oracle.from_case(c)
    g.step(10)
    o.step(10)
    got = g.velocity_gradient()
    ref = C.velocity_gradient(o)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"  grad {name} {prec}: {err:.2e}")
    assert err < tol


def test_tgv3d_initial_dissipation():
    """Sec. 3.4: the initial field has only modes with |k|^2 = 3, so
    nu sum wJ |grad u|^2 = 6 nu KE_0 (KE = sum wJ |u|^2 / 2, rho0 = 1)."""
    from paper_2509_19171_amd import sel

    c = I.case_tgv3d(nel=4, N=7, Q=27, Re=1600.0, steps=0)
    g = sel.from_case(c, "fp64")
    A = g.velocity_gradient()
    wJ, _ = g.geometry()
    r = g.reduce()
    eps = c.nu * np.einsum("ep,epij->", wJ, A * A)
    ke = r[4]  # [mass, momentum (3), kinetic energy, non-finite count]
    say(f"  eps(0) = {eps:.6e}, 6 nu KE0 = {6 * c.nu * ke:.6e}")
    assert abs(eps - 6 * c.nu * ke) < 1e-6 * 6 * c.nu * ke


def test_channel_wall_shear_exact():
    """u_x = 4 U y (H - y) / H^2 is of degree 2 <= N: du_x/dy at the walls is
    +-4 U / H to rounding (tau_w = mu |du_x/dy|)."""
    from paper_2509_19171_amd import sel

    U, H = 0.05, 1.0
    m = I.box_mesh(2, 6, (4, 3), (0, 0), (2, H), (True, False), wall_tags={1: (1, 1)}, wall_u=[[0, 0]])
    rho = np.ones(m.xyz.shape[:2])
    u = np.zeros(m.xyz.shape)
    y = m.xyz[..., 1]
    u[..., 0] = 4 * U * y * (H - y) / H ** 2
    c = I.Case("channel", m, 9, 1.0, 0.01, I.stable_dt(m), rho, u, 0)
    A = sel.from_case(c, "fp64").velocity_gradient()
    lo, hi = np.abs(y) < 1e-12, np.abs(y - H) < 1e-12
    np.testing.assert_allclose(A[..., 0, 1][lo], 4 * U / H, rtol=1e-10)
    np.testing.assert_allclose(A[..., 0, 1][hi], -4 * U / H, rtol=1e-10)


def test_pipe_wall_shear_laminar():
    """Laminar pipe profile u_z = 2 u_b (1 - r^2/R^2) on the curved O-grid:
    -du_z/dr at the wall is 4 u_b / R (the wall shear stress of Sec. 3.5,
    tau_w = mu (sin theta du_z/dy + cos theta du_z/dx), up to sign)."""
    from paper_2509_19171_amd import sel

    c = I.case_pipe(N=6, nsq=2, nrad=2, nax=4, L=2.0, pert=0.0, filt=None)
    A = sel.from_case(c, "fp64").velocity_gradient()
    x, yy = c.mesh.xyz[..., 0], c.mesh.xyz[..., 1]
    r = np.hypot(x, yy)
    wall = r > 1 - 1e-12
    th = np.arctan2(yy, x)
    dudr = np.cos(th) * A[..., 2, 0] + np.sin(th) * A[..., 2, 1]
    tau = -dudr[wall].mean()
    say(f"  -du_z/dr at the wall: {tau:.6e} (4 u_b / R = {4 * c.meta['ub']:.6e})")
    assert abs(tau - 4 * c.meta["ub"]) < 1e-3 * 4 * c.meta["ub"]


def test_pipe_wall_units_laminar():
    """Wall units (Sec. 3.5) of the laminar profile u_z = 2 u_b (1 - r^2/R^2)
    on the curved O-grid (no body force, so the state's velocity is the
    profile itself): u_tau from the wall shear stress against
    sqrt(nu 4 u_b / R) to 5e-4 (the wall gradient is good to 1e-3), each bin's
    mean axial velocity u+ u_tau against the lumped-mass average of the exact
    profile over the bin's nodes to 1e-10 of u_b, and y+ = (R - r) u_tau / nu
    at the bin centres."""
    import dataclasses

    from paper_2509_19171_amd import sel
    from paper_2509_19171_amd import wallunits as W

    c = dataclasses.replace(I.case_pipe(N=6, nsq=2, nrad=2, nax=4, L=2.0, pert=0.0, filt=None), g=(0.0, 0.0, 0.0))
    R, ub, nb = c.meta["R"], c.meta["ub"], 7
    g = sel.from_case(c, "fp64")
    prof = W.WallProfile((0, 0, 0), (0, 0, 1), R, nb, c.rho0, c.nu)
    prof.add(g, c.mesh.xyz)
    yp, up, ut = prof.result()
    ut_ref = math.sqrt(c.nu * 4 * ub / R)
    say(f"  u_tau {ut:.6e} (exact {ut_ref:.6e}); u+ {np.round(up, 3)}")
    assert abs(ut - ut_ref) < 5e-4 * ut_ref
    wJ, _ = g.geometry()
    x, y = c.mesh.xyz[..., 0], c.mesh.xyz[..., 1]
    r = np.sqrt(x * x + y * y)  # the library's binning: sqrt(r^2) / rmax * nbins
    b = np.floor(r / R * nb).astype(int)
    uex = 2 * ub * (1 - (r / R) ** 2)
    ref = np.array([(wJ * uex)[b == k].sum() / wJ[b == k].sum() for k in range(nb) if (b == k).any()])
    assert up.shape == ref.shape
    assert np.abs(up * ut - ref).max() < 1e-10 * ub
    centres = (np.arange(nb) + 0.5) * R / nb
    np.testing.assert_allclose(yp, (R - centres[[k for k in range(nb) if (b == k).any()]]) * ut / c.nu, rtol=1e-14)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32dev", 1e-5)])
def test_radial_profile_parity(prec, tol):
    """sel_radial_profile (the pipe's averaged axial velocity profile, Sec.
    3.5) against the reference sums on the oracle's state and geometry after
    20 steps of the perturbed O-grid pipe; bin weights to 1e-12, velocity sums
    normwise to the storage form's tolerance; a repeated call returns the same
    values bit for bit, and a new binning replaces the old one."""
    import oracle
    from paper_2509_19171_amd import sel
    from radial_ref import radial_sums

    c = I.case_pipe(N=5, nsq=4, nrad=3, nax=3, L=3.0)
    g = sel.from_case(c, prec)
    o = oracle.from_case(c)
    g.step(20)
    o.step(20)
    wJ, _, _ = o.geometry()
    _, ou = o.moments()
    R = c.meta["R"] * (1 + 1e-9)
    for nb in (24, 7):
        s, w = g.radial_profile((0, 0, 0), (0, 0, 1), R, nb)
        rs, rw = radial_sums(c.mesh.xyz, wJ, ou, (0, 0, 0), (0, 0, 1), R, nb)
        es = np.abs(s - rs).max() / np.abs(rs).max()
        ew = np.abs(w - rw).max() / np.abs(rw).max()
        say(f"  {prec} nbins {nb}: sums {es:.2e} weights {ew:.2e}; profile {np.round(s / w, 5)}")
        assert ew < 1e-12 and es < tol
        s2, w2 = g.radial_profile((0, 0, 0), (0, 0, 1), R, nb)
        assert np.array_equal(s, s2) and np.array_equal(w, w2)
