"""The learned closure against the plain filtered method (its fallback and
judge): a closure trained on GPU-generated data from perturbed 3D Taylor-Green
runs (fine N = 7, coarse-grained to N = 3 on the same 8^3 elements, Re = 400,
exponential filter) is judged on the unperturbed vortex. Both coarse runs
start from the coarse-grained fine initial state and are compared with the
coarse-grained fine run up to t u0 / L = 8.

Measured on MI355X: the closure reduces the mean kinetic-energy error by a
factor of about 1.27 and the mean relative L2 velocity error by about 1.05;
every kernel involved is deterministic, so the run repeats exactly. The test
asserts margins below those figures. At N = 7 -> 4 the same recipe gains
nothing (about 1.0), which is why the coarser pair is used here."""
import sys

import numpy as np
import pytest

from paper_2509_19171_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def _make(seed=None):
    def make(N):
        c = I.case_tgv3d(nel=8, N=N, Q=27, Re=400.0, steps=0, filt="exp")
        if seed is not None:
            c.rho, c.u = I.random_state(c, seed=seed, amp=0.002)
        return c
    return make


def test_closure_gain_tgv3d():
    assert torch.cuda.is_available()
    from paper_2509_19171_amd import closure_train as T

    tstar = 0.1 * I.CS  # u0 / L with L = 1
    cf = _make()(7)
    total = int(8.0 / tstar / cf.dt)
    every = total // 16
    say(f"gain test: dt {cf.dt:.4g}, {total} fine steps, snapshots every {every}")
    S = [T.generate(_make(seed), 7, 3, 16, every) for seed in (1, 2)]
    X = torch.cat([s.X for s in S])
    y = torch.cat([s.y for s in S])
    say(f"  {X.shape[0]} samples, mean target {float(y.mean()):.3e}")
    R = T.train(T.Samples(X, y), epochs=15, seed=0)
    say(f"  loss {R.train_loss[0]:.3e} -> {R.train_loss[-1]:.3e}, validation {R.val_loss[0]:.3e} -> "
        f"{R.val_loss[-1]:.3e} ({R.steps} Adam steps)")
    assert np.all(np.isfinite(R.blob))
    assert R.val_loss[-1] < 0.85 * R.val_loss[0]
    J = T.judge(_make(), 7, 3, R.blob, 16, every)
    for k in range(len(J.times)):
        say(f"  t*={J.times[k] * tstar:5.2f} L2 err plain {J.err_plain[k]:.4e} closure {J.err_closure[k]:.4e} "
            f"KE ref {J.ke_ref[k]:.5e} plain {J.ke_plain[k]:.5e} closure {J.ke_closure[k]:.5e}")
    say(f"  gain: kinetic energy {J.gain_ke:.4f}, velocity L2 {J.gain:.4f}")
    assert J.gain_ke > 1.15
    assert J.gain > 1.02
