"""A force density per node (F = rho g + F_n, Sec. 2.1; sel_set_force) on the
GPU against the FP64 oracle: constant and time-dependent fields, with the
continuous and the discontinuous coupling and both time-marching forms.

Tolerances as in the other parity tests (normwise relative error): FP64 1e-12,
FP32 deviation storage 1e-5 on rho and u after 200 steps."""
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
    return float(np.abs(u - uref).max() / max(np.abs(uref).max(), 0.01))


def _warp(x):  # periodic in x and z, flat walls at y = 0, 1
    out = x.copy()
    out[..., 0] += 0.02 * np.sin(2 * math.pi * x[..., 2] / 1.5)
    out[..., 1] += 0.02 * np.sin(math.pi * x[..., 1]) * np.sin(2 * math.pi * x[..., 0])
    out[..., 2] += 0.02 * np.sin(2 * math.pi * x[..., 0])
    return out


def _box():
    m = I.box_mesh(3, 5, (2, 2, 3), (0, 0, 0), (1, 1, 1.5), (True, False, True), wall_tags={1: (1, 2)},
                   wall_u=[[0, 0, 0], [0.0, 0, 0.0]], warp=_warp)
    r, u = I.rest_fields(m.xyz)
    return I.Case("box3d_q19_N5", m, 19, 1.0, 0.01, I.stable_dt(m), r, u, 0, filter="quad", filter_kc=2,
                  filter_amp=0.1)


CASES = {
    # periods: channel x in [0, 2]; box x in [0, 1], z in [0, 1.5]; TGV [0, 2 pi]^3
    "channel_curved_N7": (I.case_poiseuille(nelx=4, nely=3, N=7, curved=True),
                          lambda x: np.stack([0.5 + np.sin(math.pi * x[..., 0]) * np.sin(math.pi * x[..., 1]),
                                              0.3 * np.cos(math.pi * x[..., 0])], -1)),
    "box3d_q19_walls_N5": (_box(),
                           lambda x: np.stack([0.4 + np.sin(2 * math.pi * x[..., 0]) * np.sin(math.pi * x[..., 1]),
                                               0.2 * np.sin(2 * math.pi * x[..., 2] / 1.5),
                                               -0.3 + np.cos(2 * math.pi * x[..., 0])], -1)),
    "tgv3d_q27_N4": (I.case_tgv3d(nel=3, N=4, Q=27, Re=200.0, steps=0, filt="quad"),
                     lambda x: np.stack([np.sin(x[..., 1]), 0.5 + np.cos(x[..., 2]), np.sin(x[..., 0] + x[..., 2])],
                                        -1)),
}


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2509_19171_amd import sel

    sel.load()
    yield


def _pair(c, prec, field, amp):
    import oracle
    from paper_2509_19171_amd import sel

    F = amp * field(c.mesh.xyz)
    g = sel.from_case(c, prec)
    o = oracle.from_case(c)
    g.set_force(F)
    o.set_force(F)
    return g, o


@pytest.mark.parametrize("name", list(CASES))
def test_force_parity_fp64(name):
    c, field = CASES[name]
    say(f"force fp64 {name}")
    g, o = _pair(c, "fp64", field, 1e-3)
    g.step(50)
    o.step(50)
    rho, u = g.moments()
    orho, ou = o.moments()
    ef = nerr(g.get_f(), o.get_f())
    say(f"  f {ef:.2e} rho {nerr(rho, orho):.2e} u {uerr(u, ou):.2e}")
    assert ef < 1e-12 and nerr(rho, orho) < 1e-12 and uerr(u, ou) < 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_force_parity_fp32dev(name):
    c, field = CASES[name]
    say(f"force fp32dev {name}")
    g, o = _pair(c, "fp32dev", field, 1e-3)
    g.step(200)
    o.step(200)
    rho, u = g.moments()
    orho, ou = o.moments()
    er, eu = nerr(rho, orho), nerr(u, ou)
    say(f"  fp32dev error rho {er:.3e} u {eu:.3e}")
    assert er < 1e-5 and eu < 1e-5


def test_time_dependent_force():
    """The force is set again between calls (a pulsating field), on both
    sides, every 10 steps."""
    c, field = CASES["channel_curved_N7"]
    g, o = _pair(c, "fp64", field, 0.0)
    for k in range(8):
        F = 1e-3 * math.cos(0.7 * k) * field(c.mesh.xyz)
        g.set_force(F)
        o.set_force(F)
        g.step(10)
        o.step(10)
    ef = nerr(g.get_f(), o.get_f())
    say(f"  time-dependent force f {ef:.2e}")
    assert ef < 1e-12


@pytest.mark.parametrize("variant", ["dg", "printed4"])
def test_force_with_other_forms(variant):
    c, field = CASES["channel_curved_N7"]
    c = dataclasses.replace(c, coupling="dg") if variant == "dg" else dataclasses.replace(c, rk="printed4")
    g, o = _pair(c, "fp64", field, 1e-3)
    g.step(50)
    o.step(50)
    ef = nerr(g.get_f(), o.get_f())
    say(f"  force with {variant}: f {ef:.2e}")
    assert ef < 1e-12


def test_zero_and_removed_force():
    """A zero field leaves the run as without it (to rounding of the split
    first stage), and removing the field restores the plain path."""
    from paper_2509_19171_amd import sel

    c, field = CASES["box3d_q19_walls_N5"]
    a = sel.from_case(c, "fp64")
    b = sel.from_case(c, "fp64")
    b.set_force(np.zeros((c.mesh.E, c.mesh.np_, 3)))
    a.step(20)
    b.step(20)
    assert nerr(b.get_f(), a.get_f()) < 1e-14
    b.set_force(None)
    a.step(5)
    b.step(5)
    assert nerr(b.get_f(), a.get_f()) < 1e-14
    with pytest.raises(sel.SelError):
        b.set_force(np.full((c.mesh.E, c.mesh.np_, 3), np.nan))
