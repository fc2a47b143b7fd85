"""FP64 oracle of the learned relaxation-time closure (test infrastructure).

The paper has no closure; the workload adds a per-node MLP that maps local
invariants to a relaxation-time increment for under-resolved runs. This
module is the plain definition the GPU kernels are checked against:

  features (per element node, from f-bar):
    u = sum e f / rho, A_ik = du_i/dx_k from element-local derivatives
    (du/dx_k = sum_m (dr_m/dx_k) D_m u), S = (A + A^T)/2, W = (A - A^T)/2,
    Pi = sum_a e e (f_a - f^eq_a), lam = tau dt = nu / c_s^2,
    x = [lam^2 S:S, lam^2 W:W, lam^3 tr(S^3), lam^3 tr(S W W),
         Pi:Pi / (rho c_s^2)^2, lam Pi:S / (rho c_s^2)]
    normalised as (x - mean) / std.
  network: h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), h3 = tanh(W3 h2 + b3),
    z = w4 . h3 + b4  (6 -> 64 -> 64 -> 64 -> 1);
  increment: dtau = tau softplus(z); a non-finite value, or one above
    dtau_max * tau, falls back to 0 (the plain method);
  shared nodes take the value of their lowest-numbered copy;
  collision: omega = 1 / (tau + dtau + 1/2).
  training target (per coarse element): the fine velocity is projected onto
    the coarse element (modal truncation in the basis phi_0 = L_0,
    phi_1 = L_1, phi_k = L_k - L_{k-2}, evaluated at the coarse GLL nodes),
    tau_sgs = P(u u) - P(u) P(u), S-bar from P(u),
    nu_t = max(0, -<dev(tau_sgs) : S-bar> / <2 S-bar : S-bar>) (wJ-weighted
    element means), dtau* = nu_t / (c_s^2 dt_coarse), target y = dtau* / tau;
  loss: mean squared error of dtau / tau against dtau* / tau;
  Adam (Kingma & Ba) with bias correction.

Parameter blob (float32, this order): mean[6], std[6], W1[64][6], b1[64],
W2[64][64], b2[64], W3[64][64], b3[64], w4[64], b4[1], dtau_max[1].
"""
from __future__ import annotations

import numpy as np

from . import _load, dmat, gll, lattice

NF, NH = 6, 64
CS2 = 1.0 / 3.0

SHAPES = [("mean", (NF,)), ("std", (NF,)), ("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)),
          ("b2", (NH,)), ("W3", (NH, NH)), ("b3", (NH,)), ("w4", (NH,)), ("b4", (1,)), ("dtau_max", (1,))]
TRAINABLE = ["W1", "b1", "W2", "b2", "W3", "b3", "w4", "b4"]


def blob_size() -> int:
    return int(sum(np.prod(s) for _, s in SHAPES))


def unpack(blob):
    blob = np.asarray(blob, dtype=np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = blob[o:o + n].reshape(shp)
        o += n
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def init_params(seed=0, mean=None, std=None, dtau_max=100.0):
    """Seeded Glorot-uniform initial network (float64 values)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {"mean": np.zeros(NF) if mean is None else np.asarray(mean, float),
         "std": np.ones(NF) if std is None else np.asarray(std, float)}
    for name, (fo, fi) in (("W1", (NH, NF)), ("W2", (NH, NH)), ("W3", (NH, NH))):
        a = np.sqrt(6.0 / (fi + fo))
        p[name] = rng.uniform(-a, a, size=(fo, fi))
    a = np.sqrt(6.0 / (NH + 1))
    p["w4"] = rng.uniform(-a, a, size=NH)
    for b in ("b1", "b2", "b3"):
        p[b] = np.zeros(NH)
    p["b4"] = np.array([-3.0])
    p["dtau_max"] = np.array([dtau_max])
    return p


# ---------------------------------------------------------------- network --
def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def forward(p, X):
    """Raw features X [n][6] -> (z [n], cache)."""
    Xn = (X - p["mean"]) / p["std"]
    h1 = np.tanh(Xn @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    h3 = np.tanh(h2 @ p["W3"].T + p["b3"])
    z = h3 @ p["w4"] + p["b4"][0]
    return z, (Xn, h1, h2, h3)


def dtau_of(p, X, tau):
    z, _ = forward(p, X)
    d = tau * softplus(z)
    bad = ~np.isfinite(d) | (d > p["dtau_max"][0] * tau) | (d < 0)
    return np.where(bad, 0.0, d)


def loss_and_grad(p, X, y, tau):
    """MSE of softplus(z) against y = dtau*/tau, and its gradient with respect
    to the trainable parameters (backpropagation through the layers)."""
    n = X.shape[0]
    z, (Xn, h1, h2, h3) = forward(p, X)
    sp = softplus(z)
    r = sp - y
    loss = float(np.mean(r * r))
    dz = (2.0 / n) * r / (1.0 + np.exp(-z))          # d loss / dz (softplus' = sigmoid)
    g = {"w4": h3.T @ dz, "b4": np.array([dz.sum()])}
    d3 = np.outer(dz, p["w4"]) * (1.0 - h3 * h3)
    g["W3"] = d3.T @ h2
    g["b3"] = d3.sum(0)
    d2 = (d3 @ p["W3"]) * (1.0 - h2 * h2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (1.0 - h1 * h1)
    g["W1"] = d1.T @ Xn
    g["b1"] = d1.sum(0)
    return loss, g


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t >= 1) on the trainable parameters, in place."""
    for k in TRAINABLE:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


# --------------------------------------------------------------- features --
def _grad_nodal(sim, fieldE):
    """Element-local physical gradient of a nodal field [E][np] -> [E][np][dim]."""
    dim, N = sim.dim, sim.N
    n1 = N + 1
    D = dmat(N)
    wJ, G, _ = sim.geometry()
    E = fieldE.shape[0]
    v = fieldE.reshape((E,) + (n1,) * dim)  # axes: (t, s, r) for 3D; (s, r) for 2D
    dref = []
    for m in range(dim):
        ax = dim - m  # r is the last axis
        dref.append(np.moveaxis(np.tensordot(D, v, axes=([1], [ax])), 0, ax).reshape(E, -1))
    drdx = G[..., :dim, :dim] / wJ[..., None, None]  # [E][np][m][k]
    return np.einsum("epmk,mep->epk", drdx, np.stack(dref))


def velocity_gradient(sim, f=None):
    """du_c/dx_q [E][np][dim][dim] of the state f (default: the oracle's
    state), element-local derivative with the metric (Sec. 2.2)."""
    dim, Q = sim.dim, sim.Q
    if f is None:
        f = sim.get_f()
    e, _, _ = lattice(dim, Q)
    u = np.einsum("eap,ak->epk", f, e) / f.sum(1)[..., None]
    return np.stack([_grad_nodal(sim, u[..., i]) for i in range(dim)], axis=2)


def features(sim, f=None):
    """Features [E][np][6] of the state f (default: the oracle's state)."""
    dim, Q = sim.dim, sim.Q
    if f is None:
        f = sim.get_f()
    e, t, _ = lattice(dim, Q)
    rho = f.sum(1)
    j = np.einsum("eap,ak->epk", f, e)
    u = j / rho[..., None]
    A = np.stack([_grad_nodal(sim, u[..., i]) for i in range(dim)], axis=2)  # [E][np][i][k]
    S = 0.5 * (A + np.swapaxes(A, -1, -2))
    W = 0.5 * (A - np.swapaxes(A, -1, -2))
    eu = np.einsum("ak,epk->epa", e, u)
    uu = (u * u).sum(-1)
    feq = t[None, None, :] * rho[..., None] * (1 + eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - uu[..., None] / (2 * CS2))
    fneq = f.transpose(0, 2, 1) - feq
    Pi = np.einsum("epa,ai,aj->epij", fneq, e, e)
    lam = sim.nu / CS2
    rc = rho * CS2
    x = np.stack([
        lam ** 2 * np.einsum("...ij,...ij", S, S),
        lam ** 2 * np.einsum("...ij,...ij", W, W),
        lam ** 3 * np.einsum("...ij,...jk,...ki", S, S, S),
        lam ** 3 * np.einsum("...ij,...jk,...ki", S, W, W),
        np.einsum("...ij,...ij", Pi, Pi) / rc ** 2,
        lam * np.einsum("...ij,...ij", Pi, S) / rc,
    ], axis=-1)
    return x


def owner_values(gid, vals):
    """Give every copy of a shared node the value of its lowest-numbered copy."""
    flat = vals.reshape(-1)
    g = gid.reshape(-1)
    first = np.full(int(g.max()) + 1, -1, dtype=np.int64)
    for i in range(g.size - 1, -1, -1):
        first[g[i]] = i
    return flat[first[g]].reshape(vals.shape)


# --------------------------------------------------------- coarse graining --
def _phi(N, x):
    """Filter/projection basis phi_k(x), k = 0..N, at points x."""
    from . import legendre
    P = np.zeros((len(x), N + 1))
    for i, xi in enumerate(x):
        for k in range(N + 1):
            Lk, _ = legendre(k, xi)
            if k >= 2:
                Lk2, _ = legendre(k - 2, xi)
                P[i, k] = Lk - Lk2
            else:
                P[i, k] = Lk
    return P


def projection(Nf, Nc):
    """1D map from Nf-nodal values to Nc-nodal values: modal truncation in the
    phi basis to k <= Nc, evaluated at the Nc GLL nodes."""
    xf, _ = gll(Nf)
    xc, _ = gll(Nc)
    Pf = _phi(Nf, xf)
    coef = np.linalg.solve(Pf, np.eye(Nf + 1))  # Pf^-1: nodal -> modal
    return _phi(Nc, xc)[:, :Nc + 1] @ coef[:Nc + 1, :]


def coarse_grain_field(v, dim, Nf, Nc):
    """Apply P (x) P (x) P to an element field [E][(Nf+1)^dim] (or with trailing axes)."""
    P = projection(Nf, Nc)
    E = v.shape[0]
    rest = v.shape[2:]
    a = v.reshape((E,) + (Nf + 1,) * dim + rest)
    for m in range(dim):
        ax = dim - m
        a = np.moveaxis(np.tensordot(P, a, axes=([1], [ax])), 0, ax)
    return a.reshape((E, (Nc + 1) ** dim) + rest)


def coarse_grain_f(f, dim, Nf, Nc):
    """f [E][Q][np_f] -> [E][Q][np_c]."""
    return coarse_grain_field(f.transpose(0, 2, 1), dim, Nf, Nc).transpose(0, 2, 1)


def targets(fine, coarse_sim, dt_coarse):
    """Per coarse node target y = dtau* / tau_coarse (the element value on every
    node) from the fine oracle state; coarse_sim supplies the coarse geometry
    and tau."""
    dim, Q = fine.dim, fine.Q
    f = fine.get_f()
    e, _, _ = lattice(dim, Q)
    rho = f.sum(1)
    u = np.einsum("eap,ak->epk", f, e) / rho[..., None]
    uu = np.einsum("epi,epj->epij", u, u)
    ub = coarse_grain_field(u, dim, fine.N, coarse_sim.N)
    uub = coarse_grain_field(uu.reshape(uu.shape[0], uu.shape[1], -1), dim, fine.N, coarse_sim.N)
    uub = uub.reshape(ub.shape + (dim,))
    tsgs = uub - np.einsum("epi,epj->epij", ub, ub)
    A = np.stack([_grad_nodal(coarse_sim, ub[..., i]) for i in range(dim)], axis=2)
    Sb = 0.5 * (A + np.swapaxes(A, -1, -2))
    tr = np.einsum("...ii", tsgs)
    td = tsgs - tr[..., None, None] * np.eye(dim) / dim
    wJ, _, _ = coarse_sim.geometry()
    num = (wJ * np.einsum("...ij,...ij", td, Sb)).sum(1)
    den = (wJ * 2.0 * np.einsum("...ij,...ij", Sb, Sb)).sum(1)
    nut = np.maximum(0.0, -num / np.where(den > 0, den, np.inf))
    d = nut / (CS2 * dt_coarse) / coarse_sim.tau
    return np.repeat(d[:, None], wJ.shape[1], axis=1)


# ------------------------------------------------------- oracle with closure --
def set_dtau(sim, dtau):
    """Per-node relaxation-time increments [E][np] for the oracle's next steps."""
    lib = _load()
    d = np.ascontiguousarray(dtau, dtype=np.float64)
    import ctypes

    lib.oracle_set_dtau(sim._h, ctypes.c_void_p(d.ctypes.data))


def step_with_closure(sim, p, nsteps):
    """Closure run of the oracle: before each step the increments are inferred
    from the current state (owner values at shared nodes)."""
    for _ in range(nsteps):
        x = features(sim)
        d = dtau_of(p, x.reshape(-1, NF), sim.tau).reshape(x.shape[:2])
        set_dtau(sim, owner_values(sim._gid, d))
        sim.step(1)
    set_dtau(sim, np.zeros((sim.E, sim.np_)))
