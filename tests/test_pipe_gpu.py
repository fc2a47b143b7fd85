"""GPU parity on the O-grid pipe (curved hexahedra, exact circular FBB wall,
body force along the axis, exponential filter), FP64 and FP32 deviation
storage, at reduced size over many steps and at full size (20,480 hexes,
N = 7) over two steps; and the learned closure on the coarse (N = 5) pipe.
Tolerances as in the other parity tests: FP64 1e-12 (u normalised by
max(|u|, 0.01 c)), FP32 deviation storage normwise with no floor on u."""
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


def _sel():
    from paper_2509_19171_amd import sel

    sel.load()
    return sel


def _small(N=5):
    return I.case_pipe(N=N, nsq=4, nrad=3, nax=3, L=3.0)


def test_pipe_small_fp64_and_fp32():
    import oracle

    assert torch.cuda.is_available()
    c = _small()
    say(f"pipe small: E={c.E} N={c.N}, oracle 200 steps")
    o = oracle.from_case(c)
    o.step(20)
    f20 = o.get_f()
    rho20, u20 = o.moments()
    o.step(180)
    rho200, u200 = o.moments()
    sel = _sel()
    g = sel.from_case(c, "fp64")
    g.step(20)
    rho, u = g.moments()
    say(f"  fp64 20 steps: f {nerr(g.get_f(), f20):.2e} rho {nerr(rho, rho20):.2e} u {uerr(u, u20):.2e}")
    assert nerr(g.get_f(), f20) < 1e-12 and nerr(rho, rho20) < 1e-12 and uerr(u, u20) < 1e-12
    g = sel.from_case(c, "fp32dev")
    g.step(200)
    rho, u = g.moments()
    er, eu = nerr(rho, rho200), nerr(u, u200)
    say(f"  fp32dev 200 steps: rho {er:.2e} u {eu:.2e}")
    assert er < 1e-5 and eu < 1e-5


def test_pipe_full_size():
    """20,480 hexes at N = 7 (10.5 M element nodes, 283 M node-velocities)."""
    import oracle

    c = I.case_pipe()
    say(f"pipe full size: E={c.E}, oracle 2 steps")
    o = oracle.from_case(c)
    o.step(2)
    orho, ou = o.moments()
    of = o.get_f()
    del o
    sel = _sel()
    for prec, tol in (("fp64", 1e-12), ("fp32dev", 2e-6)):
        say(f"  {prec}")
        g = sel.from_case(c, prec)
        g.step(2)
        rho, u = g.moments()
        er, eu = nerr(rho, orho), (uerr(u, ou) if prec == "fp64" else nerr(u, ou))
        say(f"  {prec}: rho {er:.2e} u {eu:.2e}")
        assert er < tol and eu < tol, prec
        if prec == "fp64":
            assert nerr(g.get_f(), of) < 1e-12
        assert g.reduce()[-1] == 0
        del g
        torch.cuda.empty_cache()


def test_pipe_coarse_closure_run():
    """Closure inference every step on the coarse pipe, against the oracle."""
    import oracle
    from oracle import closure as C

    c = _small(5)
    o = oracle.from_case(c)
    X0 = C.features(o).reshape(-1, 6)
    p = C.init_params(4, mean=X0.mean(0), std=np.abs(X0).max(0) + 1e-30)
    p["b4"] = np.array([0.0])
    blob = C.pack(p).astype(np.float32)
    p = C.unpack(blob.astype(np.float64))
    sel = _sel()
    for prec, tol in (("fp64", 1e-8), ("fp32dev", 1e-5)):
        say(f"pipe coarse closure {prec}")
        o = oracle.from_case(c)
        C.step_with_closure(o, p, 8)
        orho, ou = o.moments()
        g = sel.from_case(c, prec, closure=blob)
        g.step(8)
        rho, u = g.moments()
        er, eu = nerr(rho, orho), (uerr(u, ou) if prec == "fp64" else nerr(u, ou))
        say(f"  rho {er:.2e} u {eu:.2e}")
        assert er < tol and eu < tol


@pytest.mark.parametrize("prec,steps,tol", [("fp64", 40, 1e-12), ("fp32dev", 200, 1e-5)])
def test_pipe_forced_law_of_wall(prec, steps, tol):
    """The paper's start of the pipe run (Sec. 3.5): law-of-the-wall initial
    profile and the time-dependent divergence-free perturbation force,
    re-set every 5 steps on both sides (sel_set_force), against the oracle."""
    import oracle
    from paper_2509_19171_amd import inputs as I
    from paper_2509_19171_amd import sel

    c = I.case_pipe(N=5, nsq=2, nrad=2, nax=4, L=2.0, init="law_of_wall", pert=0.0)
    m = c.meta
    g = sel.from_case(c, prec)
    o = oracle.from_case(c)
    t = 0.0
    t0 = steps * c.dt / 4  # short time scale: the forcing period 8 t0 spans the run twice over
    for k in range(steps // 5):
        F = c.rho0 * I.pipe_force(c.mesh.xyz, t, m["R"], m["L"], m["g"], t0, kz=1, ktheta=2)
        g.set_force(F)
        o.set_force(F)
        g.step(5)
        o.step(5)
        t += 5 * c.dt
    rho, u = g.moments()
    orho, ou = o.moments()
    er = np.abs(rho - orho).max() / np.abs(orho).max()
    eu = np.abs(u - ou).max() / (max(np.abs(ou).max(), 0.01) if prec == "fp64" else np.abs(ou).max())
    print(f"[gpu]   pipe forced {prec}: rho {er:.2e} u {eu:.2e}", flush=True)
    assert er < tol and eu < tol
