"""The four printed stage formulas of Sec. 2.2.2 (rk = printed4, L applied
linearly to the printed combinations) on the GPU against the FP64 oracle.

The device evaluates each stage as a two-state combination with the earlier
L values eliminated through the stages that define them; the oracle applies
the printed formulas as written, with the earlier L values kept. The two agree
in exact arithmetic (also with the body force, an affine part of L), so the
tolerances are those of the SSPRK3 parity tests: FP64 1e-12 normwise, FP32
deviation storage 1e-5 on rho and u after 200 steps."""
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
    # walls, a moving lid and the body force (the affine part of L)
    out["channel_curved_N7"] = I.case_poiseuille(nelx=4, nely=3, N=7, curved=True)
    out["box3d_q19_walls_N5"] = _walled_box(5, 19, (2, 2, 3), 8)
    out["box3d_q27_walls_N7"] = _walled_box(7, 27, (2, 2, 3), 9)
    return {k: dataclasses.replace(v, rk="printed4") for k, v in out.items()}


CASES = _cases()


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2509_19171_amd import sel

    sel.load()
    yield


def _run(c, prec, steps):
    from paper_2509_19171_amd import sel

    g = sel.from_case(c, prec)
    g.step(steps)
    return g


@pytest.mark.parametrize("name,steps", [("tgv2d_ragged_N5", 200), ("channel_curved_N7", 200),
                                        ("box3d_q19_walls_N5", 40), ("box3d_q27_walls_N7", 20)])
def test_printed4_parity_fp64(name, steps):
    import oracle

    c = CASES[name]
    say(f"printed4 fp64 {name} x{steps}")
    o = oracle.from_case(c)
    o.step(steps)
    g = _run(c, "fp64", steps)
    rho, u = g.moments()
    orho, ou = o.moments()
    ef = nerr(g.get_f(), o.get_f())
    say(f"  f {ef:.2e} rho {nerr(rho, orho):.2e} u {uerr(u, ou):.2e}")
    assert ef < 1e-12
    assert nerr(rho, orho) < 1e-12
    assert uerr(u, ou) < 1e-12
    assert abs(g.time - o.time) < 1e-12 * o.time


@pytest.mark.parametrize("name", list(CASES))
def test_printed4_parity_fp32dev(name):
    import oracle

    c = CASES[name]
    say(f"printed4 fp32dev {name} x200")
    o = oracle.from_case(c)
    o.step(200)
    g = _run(c, "fp32dev", 200)
    rho, u = g.moments()
    orho, ou = o.moments()
    er, eu = nerr(rho, orho), nerr(u, ou)
    say(f"  fp32dev error rho {er:.3e} u {eu:.3e}")
    assert er < 1e-5
    assert eu < 1e-5


def test_printed4_differs_from_ssprk3():
    """The form is really in use: after 50 steps of the forced channel the
    two time-marching forms differ by far more than the parity tolerance,
    and each matches its own oracle run."""
    import oracle

    c4 = CASES["channel_curved_N7"]
    c3 = dataclasses.replace(c4, rk="ssprk3")
    f4 = _run(c4, "fp64", 50).get_f()
    f3 = _run(c3, "fp64", 50).get_f()
    o3 = oracle.from_case(c3)
    o3.step(50)
    d = nerr(f4, f3)
    say(f"  printed4 vs ssprk3 after 50 steps: {d:.2e}")
    assert d > 1e-9
    assert nerr(f3, o3.get_f()) < 1e-12
