"""Pins of the closure oracle (network, gradient, Adam, features, projection,
targets, the relaxation-time hook) against closed forms, finite differences
and hand-computed cases. The closure is not in the paper; the projection
basis is the filter basis of Sec. 2.2.3 and the hook changes tau of Sec. 2.1."""
import math

import numpy as np
import pytest

from paper_2509_19171_amd import inputs as I


@pytest.fixture(scope="module")
def C(oracle_mod):
    from oracle import closure

    return closure


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _params(C, seed=1):
    r = _rng(seed + 100)
    p = C.init_params(seed, mean=r.normal(0, 0.5, 6), std=r.uniform(0.5, 2.0, 6))
    for b in ("b1", "b2", "b3"):
        p[b] = r.uniform(-0.3, 0.3, 64)
    p["b4"] = np.array([0.2])
    return p


def test_blob_layout(C):
    assert C.blob_size() == 8846
    p = _params(C)
    b = C.pack(p)
    q = C.unpack(b)
    for k in p:
        np.testing.assert_array_equal(p[k], q[k])
    # trainable range W1 .. b4 is contiguous from float 12, 8833 values
    assert sum(int(np.prod(s)) for n, s in C.SHAPES if n in C.TRAINABLE) == 8833
    assert C.SHAPES[2][0] == "W1" and C.SHAPES[9][0] == "b4"


def test_softplus_matches_logaddexp(C):
    z = np.concatenate([np.linspace(-40, 40, 801), [-1e3, 1e3, 0.0]])
    np.testing.assert_allclose(C.softplus(z), np.logaddexp(0.0, z), rtol=1e-15, atol=1e-300)


def test_forward_hand_network(C):
    """One path through the layers: z = 2 tanh(tanh(tanh(1.5 x2'))) + 0.1."""
    p = C.init_params(0)
    for k in ("W1", "W2", "W3", "w4", "b1", "b2", "b3"):
        p[k] = np.zeros_like(p[k])
    p["W1"][0, 2] = 1.5
    p["W2"][0, 0] = 1.0
    p["W3"][0, 0] = 1.0
    p["w4"][0] = 2.0
    p["b4"] = np.array([0.1])
    p["mean"] = np.array([0, 0, 0.3, 0, 0, 0.0])
    p["std"] = np.array([1, 1, 2.0, 1, 1, 1.0])
    X = _rng(3).normal(size=(5, 6))
    z, _ = C.forward(p, X)
    x2 = (X[:, 2] - 0.3) / 2.0
    np.testing.assert_allclose(z, 2 * np.tanh(np.tanh(np.tanh(1.5 * x2))) + 0.1, rtol=1e-14)
    # loss of a constant network
    for k in ("W1", "W2", "W3", "w4"):
        p[k] = np.zeros_like(p[k])
    y = np.array([0.1, 0.5, 2.0, 0.0, 1.0])
    loss, _ = C.loss_and_grad(p, X, y, 1.0)
    assert abs(loss - np.mean((np.log1p(np.exp(0.1)) - y) ** 2)) < 1e-15


def test_gradient_central_differences(C):
    """Backpropagated gradient against central differences (h = 1e-6)."""
    p = _params(C, 5)
    r = _rng(11)
    X = r.normal(0, 1.0, size=(9, 6))
    y = r.uniform(0, 2, size=9)
    _, g = C.loss_and_grad(p, X, y, 1.0)
    h = 1e-6
    for k in C.TRAINABLE:
        flat = p[k].reshape(-1)
        picks = r.choice(flat.size, size=min(flat.size, 24), replace=False)
        fd = np.zeros(picks.size)
        for i, q in enumerate(picks):
            old = flat[q]
            flat[q] = old + h
            lp, _ = C.loss_and_grad(p, X, y, 1.0)
            flat[q] = old - h
            lm, _ = C.loss_and_grad(p, X, y, 1.0)
            flat[q] = old
            fd[i] = (lp - lm) / (2 * h)
        an = g[k].reshape(-1)[picks]
        err = np.abs(an - fd).max() / max(np.abs(fd).max(), 1e-12)
        assert err < 1e-6, (k, err)


def test_adam_closed_forms(C):
    """Step 1 moves every parameter by -lr g / (|g| + eps); a second step with
    the same gradient moves it by the same amount again (m-hat = g, v-hat = g^2)."""
    p = _params(C, 2)
    r = _rng(4)
    g = {k: r.normal(size=p[k].shape) for k in C.TRAINABLE}
    m = {k: np.zeros_like(p[k]) for k in C.TRAINABLE}
    v = {k: np.zeros_like(p[k]) for k in C.TRAINABLE}
    p0 = {k: p[k].copy() for k in C.TRAINABLE}
    lr, eps = 1e-3, 1e-8
    C.adam(p, g, m, v, 1, lr=lr, eps=eps)
    for k in C.TRAINABLE:
        np.testing.assert_allclose(p[k], p0[k] - lr * g[k] / (np.abs(g[k]) + eps), rtol=1e-13, atol=1e-15)
    C.adam(p, g, m, v, 2, lr=lr, eps=eps)
    for k in C.TRAINABLE:
        np.testing.assert_allclose(p[k], p0[k] - 2 * lr * g[k] / (np.abs(g[k]) + eps), rtol=1e-12, atol=1e-14)


def test_dtau_fallback(C):
    p = C.init_params(0, dtau_max=5.0)
    for k in ("W1", "W2", "W3", "w4"):
        p[k] = np.zeros_like(p[k])
    X = _rng(1).normal(size=(4, 6))
    tau = 0.7
    p["b4"] = np.array([1.0])
    np.testing.assert_allclose(C.dtau_of(p, X, tau), tau * math.log1p(math.e), rtol=1e-15)
    p["b4"] = np.array([10.0])  # softplus(10) > dtau_max
    np.testing.assert_array_equal(C.dtau_of(p, X, tau), 0.0)
    p["b4"] = np.array([1.0])
    p["W2"][3, 3] = np.nan
    p["w4"][3] = 1.0
    np.testing.assert_array_equal(C.dtau_of(p, X, tau), 0.0)


def _feq(oracle_mod, dim, Q, rho, u):
    e, t, _ = oracle_mod.lattice(dim, Q)
    eu = np.einsum("ak,epk->epa", e, u)
    uu = (u * u).sum(-1)
    f = t * rho[..., None] * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * uu[..., None])
    return f.transpose(0, 2, 1).copy()


def _warp(dim):
    def w(x):
        out = x.copy()
        out[..., 0] = x[..., 0] + 0.05 * np.sin(math.pi * x[..., 1])
        out[..., 1] = x[..., 1] + 0.04 * np.sin(math.pi * x[..., 0])
        if dim == 3:
            out[..., 2] = x[..., 2] + 0.03 * np.sin(math.pi * x[..., 0]) * np.sin(math.pi * x[..., 1])
        return out
    return w


@pytest.mark.parametrize("dim,Q", [(2, 9), (3, 27), (3, 19)])
def test_features_linear_flow(oracle_mod, C, dim, Q):
    """u = A x on a curved mesh: the element-local gradient is exact, so
    S = sym A, W = skew A give the invariants in closed form; f = f^eq gives Pi = 0."""
    N = 4 if dim == 3 else 5
    mesh = I.box_mesh(dim, N, (2,) * dim, (0,) * dim, (1,) * dim, (False,) * dim,
                      wall_tags={m: (0, 0) for m in range(dim)}, warp=_warp(dim))
    nu = 0.02
    sim = oracle_mod.OracleSim(dim, N, mesh.xyz, mesh.gid, mesh.face_tag, mesh.wall_u, Q, 1.0, nu, 0.01)
    if dim == 2:
        A = np.array([[0.3, 0.7], [-0.2, -0.3]]) * 0.05
    else:
        A = np.array([[0.3, 0.7, 0.1], [-0.2, -0.1, 0.4], [0.25, -0.5, -0.2]]) * 0.05
    u = mesh.xyz @ A.T + 0.01
    rho = 1.0 + 0.02 * np.sin(3 * mesh.xyz[..., 0])
    X = C.features(sim, _feq(oracle_mod, dim, Q, rho, u))
    S = 0.5 * (A + A.T)
    W = 0.5 * (A - A.T)
    lam = 3 * nu
    exp = [lam ** 2 * (S * S).sum(), lam ** 2 * (W * W).sum(), lam ** 3 * np.trace(S @ S @ S),
           lam ** 3 * np.trace(S @ W @ W)]
    for q in range(4):
        np.testing.assert_allclose(X[..., q], exp[q], rtol=1e-9, atol=1e-12 * abs(exp[0]))
    assert np.abs(X[..., 4]).max() < 1e-24 and np.abs(X[..., 5]).max() < 1e-14 * abs(exp[0]) ** 0.5 + 1e-20


def test_features_nonequilibrium(oracle_mod, C):
    """f = f^eq + delta on +-x and -2 delta at rest: Pi_xx = 2 delta only, so
    Pi:Pi/(rho c_s^2)^2 = (6 delta / rho)^2 and lam Pi:S/(rho c_s^2) = 6 lam delta a / rho
    for u = (a x, -a y)."""
    N = 4
    mesh = I.box_mesh(2, N, (2, 2), (0, 0), (1, 1), (False, False), wall_tags={0: (0, 0), 1: (0, 0)})
    nu = 0.05
    sim = oracle_mod.OracleSim(2, N, mesh.xyz, mesh.gid, mesh.face_tag, mesh.wall_u, 9, 1.0, nu, 0.01)
    a = 0.02
    u = np.stack([a * mesh.xyz[..., 0], -a * mesh.xyz[..., 1]], -1)
    rho = np.full(u.shape[:2], 1.1)
    f = _feq(oracle_mod, 2, 9, rho, u)
    e, _, _ = oracle_mod.lattice(2, 9)
    ip = int(np.where((e[:, 0] == 1) & (e[:, 1] == 0))[0][0])
    im = int(np.where((e[:, 0] == -1) & (e[:, 1] == 0))[0][0])
    i0 = int(np.where((e[:, 0] == 0) & (e[:, 1] == 0))[0][0])
    d = 1e-3
    f[:, ip] += d
    f[:, im] += d
    f[:, i0] -= 2 * d
    X = C.features(sim, f)
    lam = 3 * nu
    np.testing.assert_allclose(X[..., 4], (6 * d / 1.1) ** 2, rtol=1e-9)
    np.testing.assert_allclose(X[..., 5], 6 * lam * d * a / 1.1, rtol=1e-9)
    np.testing.assert_allclose(X[..., 0], lam ** 2 * 2 * a * a, rtol=1e-9)


def test_owner_values(C):
    gid = np.array([[0, 1, 2], [2, 3, 0]])
    vals = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    np.testing.assert_array_equal(C.owner_values(gid, vals), [[1, 2, 3], [3, 5, 1]])


@pytest.mark.parametrize("Nf,Nc", [(7, 5), (7, 4), (6, 2), (5, 5)])
def test_projection(oracle_mod, C, Nf, Nc):
    """Identity for Nc = Nf, unit end rows, exact for degree <= Nc, and
    P(L_m) = L_Nc or L_(Nc-1) (by parity) for m > Nc: in the basis
    phi_k = L_k - L_(k-2) the coefficients of L_m are 1 at k = m, m-2, ...,
    and the truncated sum telescopes."""
    P = C.projection(Nf, Nc)
    xf, _ = oracle_mod.gll(Nf)
    xc, _ = oracle_mod.gll(Nc)
    if Nf == Nc:
        np.testing.assert_allclose(P, np.eye(Nf + 1), atol=1e-13)
    np.testing.assert_allclose(P[0], np.eye(Nf + 1)[0], atol=1e-13)
    np.testing.assert_allclose(P[-1], np.eye(Nf + 1)[-1], atol=1e-13)
    L = lambda m, x: np.array([oracle_mod.legendre(m, v)[0] for v in x])
    for m in range(Nf + 1):
        got = P @ L(m, xf)
        if m <= Nc:
            exp = L(m, xc)
        else:
            exp = L(Nc if (m - Nc) % 2 == 0 else Nc - 1, xc)
        np.testing.assert_allclose(got, exp, atol=1e-12)


def test_targets_zero_for_linear_flow(oracle_mod, C):
    """On affine elements a linear u has u u of degree 2 <= N_c: P is exact
    and tau_sgs vanishes. (On curved elements u(r) has the degree of the map.)"""
    dim, Nf, Nc = 2, 6, 3
    warp = lambda x: x @ np.array([[1.0, 0.3], [-0.2, 0.9]]).T
    mk = lambda N: I.box_mesh(dim, N, (2, 2), (0, 0), (1, 1), (False, False), wall_tags={0: (0, 0), 1: (0, 0)},
                              warp=warp)
    mf, mc = mk(Nf), mk(Nc)
    fine = oracle_mod.OracleSim(2, Nf, mf.xyz, mf.gid, mf.face_tag, mf.wall_u, 9, 1.0, 0.01, 0.01)
    coarse = oracle_mod.OracleSim(2, Nc, mc.xyz, mc.gid, mc.face_tag, mc.wall_u, 9, 1.0, 0.01, 0.02)
    u = mf.xyz @ np.array([[0.2, 0.5], [-0.4, -0.2]]).T * 0.05
    fine.set_f(_feq(oracle_mod, 2, 9, np.ones(u.shape[:2]), u))
    y = C.targets(fine, coarse, 0.02)
    assert np.abs(y).max() < 1e-12


def test_targets_hand_case(oracle_mod, C):
    """One element [-1,1]^2, fine N = 4, coarse N = 2, u = s (L2(y), c y).
    P(L2^2) = 1/5 + (4/5) L2 (so tau_xx = -0.45 s^2 at y = 0, 0 at y = +-1),
    P(y L2) = y (tau_xy = 0 at the coarse nodes), P(y^2) = y^2; S-bar_xy = 1.5 s y,
    S-bar_yy = s c. With GLL weights (1/3, 4/3, 1/3):
    <dev tau : S-bar> = 0.6 s^3 c, <2 S-bar : S-bar> = s^2 (12 + 8 c^2)."""
    mk = lambda N: I.box_mesh(2, N, (1, 1), (-1, -1), (1, 1), (False, False), wall_tags={0: (0, 0), 1: (0, 0)})
    mf, mc = mk(4), mk(2)
    nu = 0.01
    fine = oracle_mod.OracleSim(2, 4, mf.xyz, mf.gid, mf.face_tag, mf.wall_u, 9, 1.0, nu, 0.01)
    coarse = oracle_mod.OracleSim(2, 2, mc.xyz, mc.gid, mc.face_tag, mc.wall_u, 9, 1.0, nu, 0.02)
    for s, c in ((0.01, -1.0), (0.02, -0.5), (0.01, 1.0)):
        yy = mf.xyz[..., 1]
        u = s * np.stack([(3 * yy ** 2 - 1) / 2, c * yy], -1)
        fine.set_f(_feq(oracle_mod, 2, 9, np.ones(u.shape[:2]), u))
        y = C.targets(fine, coarse, 0.02)
        nut = max(0.0, -0.6 * s * c / (12 + 8 * c * c))
        np.testing.assert_allclose(y, nut / nu, rtol=1e-10, atol=1e-15)


def _tgv_small(oracle_mod, nu=None):
    case = I.case_tgv2d(nel=2, N=4, steps=10)
    nu = case.nu if nu is None else nu
    sim = oracle_mod.OracleSim(2, case.N, case.xyz, case.gid, case.face_tag, case.wall_u, 9, case.rho0, nu,
                               case.dt, filter="quad", filter_kc=2, filter_amp=0.1)
    sim.init(case.rho, case.u)
    return case, sim


def test_dtau_hook_equals_viscosity_change(oracle_mod, C):
    """A constant increment c acts as the viscosity c_s^2 dt (tau + c)."""
    case, a = _tgv_small(oracle_mod)
    c = 0.37 * a.tau
    C.set_dtau(a, np.full((a.E, a.np_), c))
    a.step(10)
    _, b = _tgv_small(oracle_mod, nu=(a.tau + c) * case.dt / 3.0)
    b.step(10)
    fa, fb = a.get_f(), b.get_f()
    assert np.abs(fa - fb).max() < 1e-13 * np.abs(fb).max()
    # zero increments are the plain method, bit for bit
    _, p = _tgv_small(oracle_mod)
    _, z = _tgv_small(oracle_mod)
    C.set_dtau(z, np.zeros((z.E, z.np_)))
    p.step(5)
    z.step(5)
    np.testing.assert_array_equal(p.get_f(), z.get_f())


def test_closure_with_nan_weights_is_plain(oracle_mod, C):
    _, p = _tgv_small(oracle_mod)
    _, q = _tgv_small(oracle_mod)
    prm = C.init_params(0)
    prm["W3"][0, 0] = np.nan
    p.step(4)
    C.step_with_closure(q, prm, 4)
    np.testing.assert_array_equal(p.get_f(), q.get_f())


@pytest.mark.parametrize("dim,Q", [(2, 9), (3, 19)])
def test_velocity_gradient_linear_flow(oracle_mod, C, dim, Q):
    """The velocity gradient of u = A x + b on a curved mesh is A exactly at
    every node (isoparametric elements reproduce linear fields)."""
    N = 4 if dim == 3 else 5
    mesh = I.box_mesh(dim, N, (2,) * dim, (0,) * dim, (1,) * dim, (False,) * dim,
                      wall_tags={m: (0, 0) for m in range(dim)}, warp=_warp(dim))
    sim = oracle_mod.OracleSim(dim, N, mesh.xyz, mesh.gid, mesh.face_tag, mesh.wall_u, Q, 1.0, 0.02, 0.01)
    A = (np.array([[0.3, 0.7, 0.1], [-0.2, -0.1, 0.4], [0.25, -0.5, -0.2]]) * 0.05)[:dim, :dim]
    u = mesh.xyz @ A.T + 0.01
    rho = 1.0 + 0.02 * np.sin(3 * mesh.xyz[..., 0])
    G = C.velocity_gradient(sim, _feq(oracle_mod, dim, Q, rho, u))
    np.testing.assert_allclose(G, np.broadcast_to(A, G.shape), rtol=0, atol=1e-12)
