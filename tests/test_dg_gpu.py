"""The discontinuous-Galerkin coupling on the GPU against the FP64 oracle
(element-local mass, upwind flux of the entering velocities on every face
that is not a wall, FBB on wall faces).

Tolerances as in the continuous-coupling parity tests (normwise relative
error): FP64 storage 1e-12 on single operators and whole runs; FP32 deviation
storage 2e-6 on single operators and 1e-5 on rho and u after 200 steps."""
import dataclasses
import math
import sys

import numpy as np
import pytest

from conftest import nerr
from paper_2509_19171_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def uerr(u, uref):
    """Velocity error normalised by max(max|u_ref|, 0.01 c), c = 1."""
    return float(np.abs(u - uref).max() / max(np.abs(uref).max(), 0.01))


def _warp(x):  # periodic in x and z, flat walls at y = 0, 1
    out = x.copy()
    out[..., 0] += 0.02 * np.sin(2 * math.pi * x[..., 2] / 1.5)
    out[..., 1] += 0.02 * np.sin(math.pi * x[..., 1]) * np.sin(2 * math.pi * x[..., 0])
    out[..., 2] += 0.02 * np.sin(2 * math.pi * x[..., 0])
    return out


def _walled_box(N, Q, nel, seed):
    m = I.box_mesh(3, N, nel, (0, 0, 0), (1, 1, 1.5), (True, False, True), wall_tags={1: (1, 2)},
                   wall_u=[[0, 0, 0], [0.02, 0, 0.01]], warp=_warp)
    r, u = I.rest_fields(m.xyz)
    c = I.Case(f"box3d_q{Q}_N{N}", m, Q, 1.0, 0.01, I.stable_dt(m), r, u, 0, g=(0.0, 0.0, 1e-3),
               filter="quad", filter_kc=2, filter_amp=0.1)
    c.rho, c.u = I.random_state(c, seed=seed, amp=0.01)
    return c


def _cases():
    out = {}
    c = I.case_tgv2d(nel=5, N=5, steps=0, filt="quad")
    c.mesh = I.box_mesh(2, 5, (5, 3), (0, 0), (2 * math.pi, 2 * math.pi), (True, True))
    c.rho, c.u = I.tgv2d_fields(c.mesh.xyz, 0.05)
    out["tgv2d_ragged_N5"] = c
    out["channel_curved_N7"] = I.case_poiseuille(nelx=4, nely=3, N=7, curved=True)
    out["tgv3d_q27_N4"] = I.case_tgv3d(nel=3, N=4, Q=27, Re=200.0, steps=0, filt="quad")
    out["box3d_q19_walls_N5"] = _walled_box(5, 19, (2, 2, 3), 8)
    out["box3d_q27_walls_N7"] = _walled_box(7, 27, (2, 2, 3), 9)
    return {k: dataclasses.replace(v, coupling="dg") for k, v in out.items()}


CASES = _cases()


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2509_19171_amd import sel

    sel.load()
    yield


def _discontinuous_f(case, seed=3, amp=1e-2):
    """An equilibrium-like state with independent values at every local node
    (the copies of a face node differ)."""
    import oracle

    rng = np.random.Generator(np.random.PCG64(seed))
    _, t, _ = oracle.lattice(case.dim, case.Q)
    np_ = (case.N + 1) ** case.dim
    return t[None, :, None] * (1.0 + amp * rng.standard_normal((case.mesh.E, case.Q, np_)))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32dev", 2e-6)])
@pytest.mark.parametrize("op", ["rhs_local", "rhs"])
@pytest.mark.parametrize("name", list(CASES))
def test_dg_operator_parity(name, op, prec, tol):
    import oracle
    from paper_2509_19171_amd import sel

    c = CASES[name]
    say(f"dg operator {op} {prec} {name}")
    g = sel.from_case(c, prec)
    o = oracle.from_case(c)
    f = _discontinuous_f(c)
    got = g.apply(op, f)
    ref = {"rhs_local": o.rhs_local, "rhs": o.rhs}[op](f)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"  {err:.2e}")
    assert err < tol


@pytest.mark.parametrize("name,steps", [("tgv2d_ragged_N5", 200), ("channel_curved_N7", 200),
                                        ("tgv3d_q27_N4", 40), ("box3d_q19_walls_N5", 40),
                                        ("box3d_q27_walls_N7", 20)])
def test_dg_step_parity_fp64(name, steps):
    import oracle
    from paper_2509_19171_amd import sel

    c = CASES[name]
    say(f"dg steps fp64 {name} x{steps}")
    g = sel.from_case(c, "fp64")
    o = oracle.from_case(c)
    g.step(steps)
    o.step(steps)
    rho, u = g.moments()
    orho, ou = o.moments()
    ef = nerr(g.get_f(), o.get_f())
    say(f"  f {ef:.2e} rho {nerr(rho, orho):.2e} u {uerr(u, ou):.2e}")
    assert ef < 1e-12
    assert nerr(rho, orho) < 1e-12
    assert uerr(u, ou) < 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_dg_step_parity_fp32dev(name):
    import oracle
    from paper_2509_19171_amd import sel

    c = CASES[name]
    say(f"dg steps fp32dev {name} x200")
    g = sel.from_case(c, "fp32dev")
    o = oracle.from_case(c)
    g.step(200)
    o.step(200)
    rho, u = g.moments()
    orho, ou = o.moments()
    er, eu = nerr(rho, orho), nerr(u, ou)
    say(f"  fp32dev error rho {er:.3e} u {eu:.3e}")
    assert er < 1e-5
    assert eu < 1e-5


def test_dg_printed4_parity():
    """The discontinuous coupling with the printed four-stage form."""
    import oracle
    from paper_2509_19171_amd import sel

    c = dataclasses.replace(CASES["channel_curved_N7"], rk="printed4")
    g = sel.from_case(c, "fp64")
    o = oracle.from_case(c)
    g.step(100)
    o.step(100)
    ef = nerr(g.get_f(), o.get_f())
    say(f"  dg printed4 f {ef:.2e}")
    assert ef < 1e-12


def test_dg_dissipates_more_than_cg_tgv3d():
    """The upwind interface flux damps the under-resolved 3D Taylor-Green
    vortex more than the continuous coupling (same mesh, same steps): the
    kinetic energy of the DG run ends below the CG run's."""
    from paper_2509_19171_amd import sel

    c = I.case_tgv3d(nel=4, N=5, Q=27, Re=1600.0, steps=0, filt="quad")
    nst = 1000
    ke = {}
    for coupling in ("cg", "dg"):
        g = sel.from_case(dataclasses.replace(c, coupling=coupling), "fp32dev")
        k0 = g.reduce()[4]  # [mass, momentum (3), kinetic energy, non-finite count]
        g.step(nst)
        r = g.reduce()
        assert r[5] == 0
        ke[coupling] = r[4] / k0
    say(f"  KE/KE0 after {nst} steps: cg {ke['cg']:.6f} dg {ke['dg']:.6f}")
    assert 0 < ke["dg"] < ke["cg"] < 1
