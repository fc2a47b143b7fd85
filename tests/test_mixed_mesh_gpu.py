"""A mesh whose elements are half straight (x < 0.5) and half curved, with
walls, against the FP64 oracle: every element reads its own per-node metric
(wJ dr_m/dx_k of Sec. 2.2), so straight and curved elements share one code
path.

Tolerances as in the other parity tests (normwise relative error): FP64 1e-12,
FP32 deviation storage 1e-5 on rho and u after 200 steps."""
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


def _half_warp(x):
    """Displaces y only where x > 0.5 (smoothly, zero at x = 0.5 and 1 and on
    the walls y = 0, 1): elements with x < 0.5 stay straight."""
    out = x.copy()
    s = np.where(x[..., 0] > 0.5, np.sin(2 * math.pi * (x[..., 0] - 0.5)) ** 2, 0.0)
    out[..., 1] += 0.03 * s * np.sin(math.pi * x[..., 1])
    return out


def _mixed_case(dim, N, Q):
    nel = (4, 3) if dim == 2 else (4, 3, 2)
    lo, hi = (0.0,) * dim, (1.0,) * dim
    per = (True, False) if dim == 2 else (True, False, True)
    wu = [[0.0] * dim, [0.02] + [0.0] * (dim - 1)]
    m = I.box_mesh(dim, N, nel, lo, hi, per, wall_tags={1: (1, 2)}, wall_u=wu, warp=_half_warp)
    r, u = I.rest_fields(m.xyz)
    c = I.Case(f"mixed{dim}d_q{Q}_N{N}", m, Q, 1.0, 0.01, I.stable_dt(m), r, u, 0,
               g=(1e-3,) + (0.0,) * (dim - 1), filter="quad", filter_kc=2, filter_amp=0.1)
    c.rho, c.u = I.random_state(c, seed=21, amp=0.01)
    return c


CASES = {"2d_q9_N7": (2, 7, 9), "3d_q27_N7": (3, 7, 27), "3d_q19_N5": (3, 5, 19)}


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2509_19171_amd import sel

    sel.load()
    yield


@pytest.mark.parametrize("op", ["rhs_local", "rhs"])
@pytest.mark.parametrize("name", list(CASES))
def test_mixed_operator_fp64(name, op):
    import oracle
    from paper_2509_19171_amd import sel

    c = _mixed_case(*CASES[name])
    g = sel.from_case(c, "fp64")
    o = oracle.from_case(c)
    # continuous across elements (one value per node id, as the GPU stores it)
    rng = np.random.Generator(np.random.PCG64(5))
    _, t, _ = oracle.lattice(c.dim, c.Q)
    ng = int(c.mesh.gid.max()) + 1
    base = t[None, :] * (1.0 + 1e-2 * rng.standard_normal((ng, c.Q)))
    f = base[c.mesh.gid].transpose(0, 2, 1).copy()
    got = g.apply(op, f)
    ref = {"rhs_local": o.rhs_local, "rhs": o.rhs}[op](f)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"mixed {name} {op}: {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_steps(name):
    import oracle
    from paper_2509_19171_amd import sel

    c = _mixed_case(*CASES[name])
    o = oracle.from_case(c)
    g64 = sel.from_case(c, "fp64")
    g32 = sel.from_case(c, "fp32dev")
    o.step(200)
    g64.step(200)
    g32.step(200)
    orho, ou = o.moments()
    r64, u64 = g64.moments()
    r32, u32 = g32.moments()
    e64 = nerr(g64.get_f(), o.get_f())
    er, eu = nerr(r32, orho), nerr(u32, ou)
    say(f"mixed {name}: fp64 f {e64:.2e}; fp32dev rho {er:.2e} u {eu:.2e}")
    assert e64 < 1e-12 and nerr(r64, orho) < 1e-12
    assert er < 1e-5 and eu < 1e-5
