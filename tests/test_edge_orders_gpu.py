"""Edge cases of the compiled range against the FP64 oracle: the lowest order
(N = 2: one interior node per line) in 2D and with both 3D lattices, the
highest 2D order (N = 10), and a call of zero steps, which leaves the state
and the clock unchanged.

Tolerances as in the other parity tests (normwise relative error): FP64 1e-12,
FP32 deviation storage 1e-5 on rho and u."""
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


def _warp3(x):  # periodic in x and z, flat walls at y = 0, 1
    out = x.copy()
    out[..., 0] += 0.02 * np.sin(2 * math.pi * x[..., 2])
    out[..., 1] += 0.02 * np.sin(math.pi * x[..., 1]) * np.sin(2 * math.pi * x[..., 0])
    return out


def _cases():
    out = {}
    c = I.case_tgv2d(nel=5, N=2, steps=0, filt=None)
    c.mesh = I.box_mesh(2, 2, (5, 4), (0, 0), (2 * math.pi, 2 * math.pi), (True, True))
    c.rho, c.u = I.tgv2d_fields(c.mesh.xyz, 0.05)
    c.dt = I.stable_dt(c.mesh)
    out["tgv2d_N2"] = c
    c = I.case_tgv2d(nel=3, N=10, steps=0, filt="quad")
    c.mesh = I.box_mesh(2, 10, (3, 2), (0, 0), (2 * math.pi, 2 * math.pi), (True, True))
    c.rho, c.u = I.tgv2d_fields(c.mesh.xyz, 0.05)
    c.dt = I.stable_dt(c.mesh)
    out["tgv2d_N10"] = c
    for Q in (19, 27):
        m = I.box_mesh(3, 2, (3, 2, 3), (0, 0, 0), (1, 1, 1), (True, False, True), wall_tags={1: (1, 2)},
                       wall_u=[[0, 0, 0], [0.02, 0, 0]], warp=_warp3)
        r, u = I.rest_fields(m.xyz)
        c = I.Case(f"box3d_q{Q}_N2", m, Q, 1.0, 0.01, I.stable_dt(m), r, u, 0, g=(1e-3, 0.0, 0.0))
        c.rho, c.u = I.random_state(c, seed=11, amp=0.01)
        out[f"box3d_q{Q}_N2_walls"] = c
    return out


CASES = _cases()


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2509_19171_amd import sel

    sel.load()
    yield


@pytest.mark.parametrize("name", list(CASES))
def test_edge_order_parity(name):
    import oracle
    from paper_2509_19171_amd import sel

    c = CASES[name]
    o = oracle.from_case(c)
    g64 = sel.from_case(c, "fp64")
    g32 = sel.from_case(c, "fp32dev")
    o.step(100)
    g64.step(100)
    g32.step(100)
    orho, ou = o.moments()
    ef = nerr(g64.get_f(), o.get_f())
    r32, u32 = g32.moments()
    er, eu = nerr(r32, orho), nerr(u32, ou)
    say(f"{name}: fp64 f {ef:.2e}; fp32dev rho {er:.2e} u {eu:.2e}")
    assert ef < 1e-12
    assert er < 1e-5 and eu < 1e-5


def test_zero_steps_is_a_no_op():
    from paper_2509_19171_amd import sel

    c = CASES["box3d_q27_N2_walls"]
    g = sel.from_case(c, "fp32dev")
    g.step(3)
    f0, t0, n0 = g.get_f(), g.time, g.nstep
    g.step(0)
    assert np.array_equal(g.get_f(), f0) and g.time == t0 and g.nstep == n0
