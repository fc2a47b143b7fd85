"""The learned closure judged on a reduced O-grid pipe start-up (Sec. 3.5):
4 x 4 core and 4 x 4 x 3 shell elements per cross-section, 16 along the
periodic length L = 4R (1024 elements), Re_tau = 180, started from the
law-of-the-wall profile with a seeded 5% perturbation and driven by the
body force and the divergence-free perturbation force of Sec. 3.5 (set every
20 steps). The fine run is of order 7, the coarse runs of order 5 on the same
elements at the fine time step, all in FP32 deviation storage with the
paper's filter. 24000 fine steps (t u_tau / R = 0.068) are affordable here,
so the force's period is compressed to two such windows (it rises to its peak
and back). Training data: 16 snapshots each of two runs with other
perturbation seeds; the judge starts both coarse runs from the coarse-grained
fine state of a third seed and compares them with the coarse-grained fine run
every 1500 steps, on the space-averaged axial velocity u_z(r) in 12 radial
bins (sel_radial_profile), on the velocity field and on the kinetic energy.

Measured on MI355X: in this window the coarse-grained fine field carries
almost no subgrid stress (the mean target dtau*/tau is 4e-6), so the trained
network adds almost nothing and the gain is 1.000 on all three measures; the
coarse runs' own error (0.19% on u_z(r) at the end, 0.68% on u) comes from the
wall layer's resolution at order 5, which a non-negative eddy viscosity cannot
remove. The test asserts exactly that: the closure run stays finite, its
increments stay small and non-negative, and it neither gains nor loses more
than 0.1% against the plain run.

The second test trains on a-posteriori targets instead (closure_train,
target "a_posteriori"): at each snapshot a plain coarse run and one with a
uniform increment dtau/tau = 1 go 300 steps from the coarse-grained fine
state, and each element's target is the increment that best steers the plain
run's axial velocity towards the coarse-grained fine run over those steps
(linear, local response; clipped to [0, 10]). Measured on MI355X: the u_z(r)
error falls 1.029x, the velocity L2 error 1.008x and the kinetic-energy error
9.99x (the plain coarse run keeps too much energy). Fitting all three
velocity components instead gives 0.960 / 1.004 / 3.37, and a 600-step
horizon 0.90-0.91 on u_z(r) (the linear response no longer holds). Asserted
with margins: u_z(r) gain > 1.01, velocity gain > 1.0, KE gain > 5."""
import math
import sys

import numpy as np
import pytest

from paper_2509_19171_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOTAL = 24000
NCHK = 16


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def _make(seed):
    def make(N):
        return I.case_pipe(N=N, nsq=4, nrad=3, nax=16, L=4.0, init="law_of_wall", pert=0.05, seed=seed)
    return make


def _force(meta, dt):
    """Perturbation force with its period compressed to two judge windows;
    its spatial part is evaluated once per order (it is separable in t)."""
    window = TOTAL * dt
    t0f = 2.0 * window / 8.0   # the force's period is 8 t0
    cache = {}

    def force(c, t):
        if c.N not in cache:
            cache[c.N] = c.rho0 * I.pipe_force(c.mesh.xyz, 2.0 * t0f, meta["R"], meta["L"], meta["g"], t0f)
        return math.sin(2.0 * math.pi * t / (8.0 * t0f)) * cache[c.N]
    return force


def _judge(target):
    from paper_2509_19171_amd import closure_train as T

    cf = _make(180)(7)
    force = _force(cf.meta, cf.dt)
    every = TOTAL // NCHK
    say(f"pipe judge ({target} targets): E={cf.E}, dt {cf.dt:.4g}, {TOTAL} fine steps, snapshots every {every}")
    S = [T.generate(_make(seed), 7, 5, NCHK, every, force=force, force_every=20, target=target, horizon=300,
                    y_probe=1.0, y_max=10.0, components=(2,)) for seed in (181, 182)]
    X = torch.cat([s.X for s in S])
    y = torch.cat([s.y for s in S])
    say(f"  {X.shape[0]} samples, mean target {float(y.mean()):.3e}, max {float(y.max()):.3e}")
    assert float(y.min()) >= 0.0
    R = T.train(T.Samples(X, y), epochs=15, seed=0)
    say(f"  loss {R.train_loss[0]:.3e} -> {R.train_loss[-1]:.3e}, validation {R.val_loss[0]:.3e} -> "
        f"{R.val_loss[-1]:.3e} ({R.steps} Adam steps)")
    assert np.all(np.isfinite(R.blob))
    prof = ((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 1.0 + 1e-9, 12)
    J = T.judge(_make(180), 7, 5, R.blob, NCHK, every, force=force, force_every=20, profile=prof)
    ub = cf.meta["ub"]
    for k in range(len(J.times)):
        r = J.prof_ref[k]
        ep = np.linalg.norm(J.prof_plain[k] - r) / np.linalg.norm(r)
        ec = np.linalg.norm(J.prof_closure[k] - r) / np.linalg.norm(r)
        say(f"  t={J.times[k]:6.2f} u_z(r) err plain {ep:.4e} closure {ec:.4e}; L2 u plain {J.err_plain[k]:.4e} "
            f"closure {J.err_closure[k]:.4e}; KE ref {J.ke_ref[k]:.6e} plain {J.ke_plain[k]:.6e} "
            f"closure {J.ke_closure[k]:.6e}")
    say("  u_z(r)/u_b ref     " + " ".join(f"{v:.4f}" for v in J.prof_ref[-1] / ub))
    say("  u_z(r)/u_b plain   " + " ".join(f"{v:.4f}" for v in J.prof_plain[-1] / ub))
    say("  u_z(r)/u_b closure " + " ".join(f"{v:.4f}" for v in J.prof_closure[-1] / ub))
    say(f"  gain: u_z(r) {J.gain_profile:.5f}, velocity L2 {J.gain:.5f}, kinetic energy {J.gain_ke:.5f}")
    # the coarse runs follow the reference: profile error below 0.5%
    assert max(np.linalg.norm(p - r) / np.linalg.norm(r) for p, r in zip(J.prof_plain, J.prof_ref)) < 5e-3
    assert all(np.isfinite(J.err_closure))
    return J


def test_closure_gain_pipe():
    assert torch.cuda.is_available()
    J = _judge("a_priori")
    for g in (J.gain_profile, J.gain, J.gain_ke):
        assert 0.999 < g < 1.001


def test_closure_gain_pipe_a_posteriori():
    assert torch.cuda.is_available()
    J = _judge("a_posteriori")
    assert J.gain_profile > 1.01
    assert J.gain > 1.0
    assert J.gain_ke > 5.0
