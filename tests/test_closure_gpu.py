"""GPU parity of the learned-closure kernels against the FP64 closure oracle.

Tolerances:
  features: FP32 output of an FP64 computation (FP64 storage): 1e-6 of each
    feature's largest magnitude; FP32 deviation storage: 5e-3 (gradients
    and non-equilibrium moments of FP32 populations);
  network: FP32 MFMA / VALU against FP64 on the same FP32 weights:
    |dz| <= 2e-5 (1 + |z|), gradients 1e-4 normwise per parameter group;
  Adam: 1e-6 absolute on the parameters where the gradient sign is decided;
  coarse graining and targets: 1e-11 (FP64 state), 1e-6 (FP32 output);
  closure runs: the increments come from FP32 features and weights on both
    sides' inputs, so rho and u agree to 1e-8 (FP64 storage) and 1e-5
    (FP32 deviation storage) after the run.
"""
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


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2509_19171_amd import sel

    sel.load()
    yield


def _sel():
    from paper_2509_19171_amd import sel

    return sel


def _C():
    import oracle
    from oracle import closure

    oracle._load()
    return closure


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _blob(seed=1, b4=-1.0, mean=None, std=None, dtau_max=100.0):
    """Seeded FP32 blob and the oracle's parameters with the same FP32 values."""
    C = _C()
    r = _rng(seed + 100)
    p = C.init_params(seed, mean=mean, std=std, dtau_max=dtau_max)
    for b in ("b1", "b2", "b3"):
        p[b] = r.uniform(-0.3, 0.3, 64)
    p["b4"] = np.array([b4])
    blob = C.pack(p).astype(np.float32)
    return blob, C.unpack(blob.astype(np.float64))


def _case(name):
    if name == "couette_curved_N7":
        c = I.case_couette(nelx=4, nely=3, N=7, curved=True, filt="exp")
        c.rho, c.u = I.random_state(c, seed=3, amp=0.01)
        return c
    if name == "tgv3d_q27_N4":
        c = I.case_tgv3d(nel=3, N=4, Q=27, Re=200.0, steps=0, filt="quad")
        return c
    if name == "box3d_q19_N3":
        m = I.box_mesh(3, 3, (2, 3, 2), (0, 0, 0), (1, 1.5, 1), (True, True, False), wall_tags={2: (1, 2)},
                       wall_u=[[0, 0, 0], [0.03, 0.01, 0]])
        rho, u = I.rest_fields(m.xyz)
        c = I.Case("box3d_q19", m, 19, 1.0, 0.01, I.stable_dt(m), rho, u, 0, g=(1e-3, 0.0, 0.0), filter="quad",
                   filter_kc=2, filter_amp=0.1)
        c.rho, c.u = I.random_state(c, seed=5, amp=0.01)
        return c
    if name == "tgv2d_N5":
        return I.case_tgv2d(nel=4, N=5, steps=0, filt="quad")
    raise KeyError(name)


def _pair(case, prec, nsteps, closure=None, oracle_params=None):
    import oracle

    sel = _sel()
    g = sel.from_case(case, precision=prec, closure=closure)
    o = oracle.from_case(case)
    if nsteps:
        g.step(nsteps)
        if oracle_params is None:
            o.step(nsteps)
    return g, o


@pytest.mark.parametrize("name", ["couette_curved_N7", "tgv3d_q27_N4", "box3d_q19_N3"])
@pytest.mark.parametrize("prec", ["fp64", "fp32dev"])
def test_features(name, prec):
    C = _C()
    case = _case(name)
    say(f"features {name} {prec}")
    g, o = _pair(case, prec, 3)
    X = g.closure_features().cpu().numpy().astype(np.float64)
    Xo = C.features(o)
    tol = 1e-6 if prec == "fp64" else 5e-3
    for q in range(6):
        scale = np.abs(Xo[..., q]).max()
        err = np.abs(X[..., q] - Xo[..., q]).max() / max(scale, 1e-30)
        say(f"  feature {q}: scale {scale:.3e} err {err:.2e}")
        assert err < tol, (q, err)


@pytest.mark.parametrize("n", [1, 777, 530001])
def test_mlp_forward(n):
    C = _C()
    sel = _sel()
    blob, p = _blob(2, b4=0.3, mean=np.linspace(-0.2, 0.2, 6), std=np.linspace(0.5, 2.0, 6))
    X = _rng(n).normal(0, 1.5, size=(n, 6)).astype(np.float32)
    tau = 0.8
    say(f"mlp forward n={n}")
    zg, dg = sel.mlp_forward(torch.from_numpy(blob).cuda(), torch.from_numpy(X).cuda(), tau)
    torch.cuda.synchronize()
    z, _ = C.forward(p, X.astype(np.float64))
    d = C.dtau_of(p, X.astype(np.float64), tau)
    zg = zg.cpu().numpy()
    dg = dg.cpu().numpy()
    assert np.all(np.abs(zg - z) <= 2e-5 * (1 + np.abs(z))), np.abs(zg - z).max()
    assert np.all(np.abs(dg - d) <= 2e-5 * tau * (1 + np.abs(d / tau)))


def test_mlp_fallback():
    sel = _sel()
    blob, _ = _blob(3, b4=0.0, dtau_max=0.5)
    X = torch.from_numpy(_rng(1).normal(size=(300, 6)).astype(np.float32)).cuda()
    bad = blob.copy()
    bad[5000] = np.nan  # inside W2
    _, d = sel.mlp_forward(torch.from_numpy(bad).cuda(), X, 1.0)
    assert torch.all(d == 0)
    # softplus(z) above dtau_max -> 0; below -> kept
    _, d = sel.mlp_forward(torch.from_numpy(blob).cuda(), X, 1.0)
    z, _ = sel.mlp_forward(torch.from_numpy(blob).cuda(), X, 1.0)
    sp = torch.nn.functional.softplus(z)
    assert torch.all(d[sp > 0.5 + 1e-4] == 0)
    assert torch.all(d[sp < 0.5 - 1e-4] > 0)


@pytest.mark.parametrize("n,sub", [(3000, None), (5000, 1999)])
def test_mlp_gradient(n, sub):
    C = _C()
    sel = _sel()
    blob, p = _blob(4, b4=0.1, mean=np.linspace(-0.1, 0.3, 6), std=np.linspace(0.7, 1.5, 6))
    r = _rng(n)
    X = r.normal(0, 1.0, size=(n, 6)).astype(np.float32)
    y = r.uniform(0, 2, size=n).astype(np.float32)
    idx = None
    Xo, yo = X, y
    if sub is not None:
        idx = r.permutation(n)[:sub].astype(np.int32)
        Xo, yo = X[idx], y[idx]
    say(f"gradient n={n} sub={sub}")
    g, loss = sel.mlp_gradient(torch.from_numpy(blob).cuda(), torch.from_numpy(X).cuda(),
                               torch.from_numpy(y).cuda(), None if idx is None else torch.from_numpy(idx).cuda())
    g = g.cpu().numpy().astype(np.float64)
    lo, go = C.loss_and_grad(p, Xo.astype(np.float64), yo.astype(np.float64), 1.0)
    assert abs(loss - lo) <= 1e-5 * lo
    off = 0
    for k in C.TRAINABLE:
        sz = go[k].size
        e = np.abs(g[off:off + sz] - go[k].reshape(-1)).max() / np.abs(go[k]).max()
        say(f"  {k}: {e:.2e}")
        assert e < 1e-4, (k, e)
        off += sz


def test_adam_steps():
    C = _C()
    sel = _sel()
    blob, p = _blob(6, b4=0.0)
    r = _rng(9)
    n = 2048
    X = r.normal(0, 1.0, size=(n, 6)).astype(np.float32)
    y = r.uniform(0, 1, size=n).astype(np.float32)
    P = torch.from_numpy(blob.copy()).cuda()
    tr = sel.MLPTrainer(P, lr=1e-3)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    m = {k: np.zeros_like(p[k]) for k in C.TRAINABLE}
    v = {k: np.zeros_like(p[k]) for k in C.TRAINABLE}
    for t in (1, 2, 3):
        before = P.cpu().numpy().astype(np.float64)
        pc = C.unpack(before)
        _, go = C.loss_and_grad(pc, X.astype(np.float64), y.astype(np.float64), 1.0)
        C.adam(p, go, m, v, t)
        tr.step(Xd, yd)
        after = P.cpu().numpy().astype(np.float64)
        pg = C.pack(p)
        gflat = np.concatenate([go[k].reshape(-1) for k in C.TRAINABLE])
        sure = np.abs(gflat) > 1e-3 * np.abs(gflat).max()
        got = after[12:12 + 8833]
        exp = pg[12:12 + 8833]
        say(f"  adam t={t}: max err {np.abs(got - exp)[sure].max():.2e}")
        assert np.abs(got - exp)[sure].max() < 1e-6 * t
        if t == 1:  # |m-hat| / sqrt(v-hat) = 1 at the first step
            assert np.abs(got - before[12:12 + 8833]).max() <= 1e-3 * (1 + 1e-5)
        # non-trainable entries untouched
        np.testing.assert_array_equal(after[:12], before[:12])
        np.testing.assert_array_equal(after[-1:], before[-1:])
        p = C.unpack(after)  # continue both from the device parameters


def _coarse_pairs():
    return [("tgv3d", 3, 7, 5, 27), ("tgv3d", 3, 6, 3, 19), ("couette", 2, 7, 4, 9)]


def _make_fc(kind, nel, Nf, Nc, Q, prec):
    import oracle

    sel = _sel()
    if kind == "tgv3d":
        cf = I.case_tgv3d(nel=nel, N=Nf, Q=Q, Re=400.0, steps=0, filt="quad")
        cc = I.case_tgv3d(nel=nel, N=Nc, Q=Q, Re=400.0, steps=0, filt="quad")
        cc.dt = cf.dt
    else:
        cf = I.case_couette(nelx=4, nely=nel, N=Nf, curved=True, filt="quad")
        cc = I.case_couette(nelx=4, nely=nel, N=Nc, curved=True, filt="quad")
        cc.dt = cf.dt
    cf.rho, cf.u = I.random_state(cf, seed=11, amp=0.01)
    gf = sel.from_case(cf, precision=prec)
    gc = sel.from_case(cc, precision=prec)
    of = oracle.from_case(cf)
    oc = oracle.from_case(cc)
    gf.step(4)
    of.step(4)
    return cf, cc, gf, gc, of, oc


@pytest.mark.parametrize("kind,nel,Nf,Nc,Q", _coarse_pairs())
@pytest.mark.parametrize("prec", ["fp64", "fp32dev"])
def test_coarse_grain(kind, nel, Nf, Nc, Q, prec):
    C = _C()
    sel = _sel()
    say(f"coarse grain {kind} N{Nf}->N{Nc} Q{Q} {prec}")
    cf, cc, gf, gc, of, oc = _make_fc(kind, nel, Nf, Nc, Q, prec)
    sel.coarse_grain(gf, gc)
    fo = C.coarse_grain_f(of.get_f(), cf.dim, Nf, Nc)
    fg = gc.get_f()
    e = nerr(fg, fo)
    say(f"  err {e:.2e}")
    assert e < (1e-11 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("kind,nel,Nf,Nc,Q", _coarse_pairs())
@pytest.mark.parametrize("prec", ["fp64", "fp32dev"])
def test_targets(kind, nel, Nf, Nc, Q, prec):
    C = _C()
    sel = _sel()
    say(f"targets {kind} N{Nf}->N{Nc} Q{Q} {prec}")
    cf, cc, gf, gc, of, oc = _make_fc(kind, nel, Nf, Nc, Q, prec)
    y = sel.closure_targets(gf, gc).cpu().numpy().astype(np.float64)
    yo = C.targets(of, oc, cc.dt)
    scale = np.abs(yo).max()
    e = np.abs(y - yo).max() / max(scale, 1e-30)
    say(f"  scale {scale:.3e} err {e:.2e} nonzero {np.count_nonzero(yo[:, 0])}/{yo.shape[0]}")
    assert scale > 0
    # the targets are written as FP32 (0.5 ulp = 6e-8 of each value) from an
    # FP64 computation on the FP64 state
    assert e < (2e-7 if prec == "fp64" else 2e-3)


@pytest.mark.parametrize("name,prec,nsteps", [("tgv2d_N5", "fp64", 12), ("tgv3d_q27_N4", "fp64", 6),
                                              ("couette_curved_N7", "fp32dev", 10),
                                              ("tgv3d_q27_N4", "fp32dev", 6)])
def test_closure_run(name, prec, nsteps):
    """Closure on: every step infers increments from the current state."""
    import oracle

    C = _C()
    sel = _sel()
    case = _case(name)
    o = oracle.from_case(case)
    # normalisation from the initial features, so that the increments vary
    # from node to node
    X0 = C.features(o).reshape(-1, 6)
    blob, p = _blob(7, b4=0.5, mean=X0.mean(0), std=np.abs(X0).max(0) + 1e-30)
    say(f"closure run {name} {prec} {nsteps}")
    g = sel.from_case(case, precision=prec, closure=blob)
    g.step(nsteps)
    C.step_with_closure(o, p, nsteps)
    rho, u = g.moments()
    rho_o, u_o = o.moments()
    er = nerr(rho, rho_o)
    eu = float(np.abs(u - u_o).max() / max(np.abs(u_o).max(), 0.01))
    # the increments really act: the plain oracle differs
    plain = oracle.from_case(case)
    plain.step(nsteps)
    _, u_p = plain.moments()
    dp = float(np.abs(u_p - u_o).max() / max(np.abs(u_o).max(), 0.01))
    say(f"  rho {er:.2e} u {eu:.2e} (closure vs plain {dp:.2e})")
    tol = 1e-8 if prec == "fp64" else 1e-5
    assert er < tol and eu < tol
    assert dp > 10 * eu


def test_nan_weights_are_plain_bitwise():
    sel = _sel()
    case = _case("couette_curved_N7")
    blob, _ = _blob(8)
    blob[3000] = np.nan
    a = sel.from_case(case, precision="fp64")
    b = sel.from_case(case, precision="fp64", closure=blob)
    a.step(7)
    b.step(7)
    np.testing.assert_array_equal(a.get_f(), b.get_f())
    # switching the closure off gives the plain path
    good, _ = _blob(8)
    c = sel.from_case(case, precision="fp64", closure=good)
    c.closure_set(None)
    c.step(7)
    np.testing.assert_array_equal(a.get_f(), c.get_f())


def test_closure_set_requires_space():
    sel = _sel()
    case = _case("tgv2d_N5")
    a = sel.from_case(case, precision="fp64")
    blob, _ = _blob(1)
    with pytest.raises(sel.SelError) as ei:
        a.closure_set(blob)
    assert ei.value.code == sel.SEL_ESTATE
    with pytest.raises(sel.SelError):
        sel.from_case(case, precision="fp64", closure=blob[:-1])


def test_training_reduces_loss():
    """Adam on the device kernels fits a smooth synthetic target."""
    sel = _sel()
    blob, _ = _blob(12, b4=0.0)
    r = _rng(13)
    n = 16384
    X = r.normal(0, 1, size=(n, 6)).astype(np.float32)
    y = (0.5 + 0.4 * np.tanh(X[:, 0] - 0.5 * X[:, 3]) + 0.1 * X[:, 1] ** 2).astype(np.float32)
    P = torch.from_numpy(blob).cuda()
    tr = sel.MLPTrainer(P, lr=3e-3)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    gen = np.random.Generator(np.random.PCG64(0))
    first = tr.step(Xd, yd)
    for ep in range(30):
        perm = torch.from_numpy(gen.permutation(n).astype(np.int32)).cuda()
        for b in range(0, n, 4096):
            tr.step(Xd, yd, idx=perm[b:b + 4096], want_loss=False)
    _, last = sel.mlp_gradient(P, Xd, yd)
    say(f"  loss {first:.3e} -> {last:.3e}")
    assert last < 0.1 * first
