"""Training and judging the learned relaxation-time closure on the GPU.

Samples come from the solver itself: a fine plain run is coarse-grained onto
a coarser simulation over the same elements (``sel_coarse_grain``); the
features of the coarse-grained state (``sel_closure_features``) and the
per-element eddy-viscosity targets (``sel_closure_targets``) form one
snapshot. Training runs the library's forward, backward and Adam kernels
(``sel_mlp_train_step``) on seeded minibatches. The judge starts the coarse
case from the coarse-grained initial state, runs it with and without the
closure, and compares both with the coarse-grained fine run.

Only host-side orchestration lives here (loops, seeded permutations, small
statistics for the input normalisation); every step of the solver, the
coarse graining and the network runs in the HIP library.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np

from . import inputs as I
from . import sel


def _torch():
    import torch

    return torch


def coarse_pair(make_case: Callable[[int], "I.Case"], Nf: int, Nc: int):
    """Fine and coarse cases on the same elements with the fine time step
    (the coarse case's step is stable at the fine one)."""
    cf = make_case(Nf)
    cc = make_case(Nc)
    if cc.E != cf.E:
        raise ValueError("fine and coarse cases must have the same elements")
    cc.dt = cf.dt
    return cf, cc


@dataclass
class Samples:
    X: object            # float32 device tensor [M][6]
    y: object            # float32 device tensor [M] (dtau* / tau)
    times: List[float] = field(default_factory=list)


def _advance(sims, n: int, force=None, force_every: int = 5):
    """Step every (case, sim) pair n steps; with force(case, t) -> [E][np][dim],
    the force density is set again every force_every steps (sel_set_force)."""
    if force is None:
        for _, s in sims:
            s.step(n)
        return
    done = 0
    while done < n:
        k = min(force_every, n - done)
        for c, s in sims:
            s.set_force(force(c, s.time))
            s.step(k)
        done += k


def _run_from(sim, case, n: int, t0: float, force=None, force_every: int = 5):
    """n steps of a run started from a coarse-grained state at time t0 (its
    own clock is not the fine run's): the force is evaluated at t0 + elapsed."""
    done = 0
    while done < n:
        k = min(force_every, n - done) if force is not None else n - done
        if force is not None:
            sim.set_force(force(case, t0 + done * case.dt))
        sim.step(k)
        done += k


def constant_blob(y: float, dtau_max: float = 100.0) -> np.ndarray:
    """A closure blob whose network outputs the constant dtau / tau = y (output
    weights zero, output bias softplus^-1(y)): a uniform viscosity increase."""
    blob = I.closure_blob(0, np.zeros(6), np.ones(6), dtau_max=dtau_max)
    blob[-66:-2] = 0.0
    blob[-2] = np.float32(np.log(np.expm1(y)))
    return blob


def _posterior_targets(fine, cf, cc, probes, horizon: int, y_probe: float, y_max: float, wJ, force, force_every,
                       components=None):
    """A-posteriori targets of the current snapshot: from the coarse-grained
    fine state, a plain coarse run (u0) and one with the uniform increment
    dtau / tau = y_probe (u1) go horizon steps; the fine run goes on for the
    same steps and is coarse-grained (ur). Taking the response of u to an
    element's increment as linear and local over the horizon, the element's
    increment that best moves u0 towards ur in the wJ-weighted least-squares
    sense is y_probe <ur - u0, u1 - u0> / <u1 - u0, u1 - u0> over the element,
    clipped to [0, y_max]; it is the target of every node of the element."""
    p0, p1, ref = probes
    t = fine.time
    sel.coarse_grain(fine, p0)
    sel.coarse_grain(fine, p1)
    _run_from(p0, cc, horizon, t, force, force_every)
    _run_from(p1, cc, horizon, t, force, force_every)
    _advance([(cf, fine)], horizon, force, force_every)
    sel.coarse_grain(fine, ref)
    _, u0 = p0.moments()
    _, u1 = p1.moments()
    _, ur = ref.moments()
    return posterior_fit(u0, u1, ur, wJ, y_probe, y_max, components)


def posterior_fit(u0, u1, ur, wJ, y_probe: float, y_max: float, components=None) -> np.ndarray:
    """Per element (arrays [E][np][dim], wJ [E][np]): the increment y with
    u0 + (y / y_probe)(u1 - u0) closest to ur in the wJ-weighted norm over the
    velocity components given (all by default), clipped to [0, y_max] (0
    where the probe moved nothing); [E][np]."""
    if components is not None:
        idx = list(components)
        u0, u1, ur = u0[..., idx], u1[..., idx], ur[..., idx]
    d = u1 - u0
    num = (wJ * ((ur - u0) * d).sum(-1)).sum(1)
    den = (wJ * (d * d).sum(-1)).sum(1)
    ye = np.where(den > 0, y_probe * num / np.where(den > 0, den, 1.0), 0.0)
    ye = np.clip(ye, 0.0, y_max)
    return np.repeat(ye[:, None], wJ.shape[1], axis=1)


def generate(make_case, Nf: int, Nc: int, nsnap: int, every: int, warm: int = 0, precision: str = "fp32dev",
             device: str = "cuda:0", force=None, force_every: int = 5, target: str = "a_priori",
             horizon: int = 300, y_probe: float = 1.0, y_max: float = 10.0, components=None) -> Samples:
    """Features and targets from nsnap snapshots of a fine plain run, taken
    every ``every`` steps after ``warm`` steps (force: optional time-dependent
    force density per node, set every force_every steps). target "a_priori":
    the sub-filter stress targets of sel_closure_targets; "a_posteriori": the
    per-element increments that best steer a short coarse run (horizon steps
    < every) towards the coarse-grained fine run (_posterior_targets; over the
    velocity components given, all by default)."""
    torch = _torch()
    if target not in ("a_priori", "a_posteriori"):
        raise ValueError(target)
    post = target == "a_posteriori"
    if post and not 0 < horizon < every:
        raise ValueError("the a-posteriori horizon must be shorter than the snapshot interval")
    cf, cc = coarse_pair(make_case, Nf, Nc)
    fine = sel.from_case(cf, precision=precision, device=device)
    coarse = sel.from_case(cc, precision=precision, device=device)
    probes, wJ = None, None
    if post:
        probes = (sel.from_case(cc, precision=precision, device=device),
                  sel.from_case(cc, precision=precision, device=device, closure=constant_blob(y_probe)),
                  sel.from_case(cc, precision=precision, device=device))
        wJ, _ = coarse.geometry()
    Xs, ys, times = [], [], []
    if warm:
        _advance([(cf, fine)], warm, force, force_every)
    ahead = 0  # steps the fine run went on past the last snapshot (a-posteriori probe)
    for _ in range(nsnap):
        _advance([(cf, fine)], every - ahead, force, force_every)
        fine.sync()  # raises on a non-finite state
        sel.coarse_grain(fine, coarse)
        Xs.append(coarse.closure_features().reshape(-1, 6))
        times.append(fine.time)
        if post:
            y = _posterior_targets(fine, cf, cc, probes, horizon, y_probe, y_max, wJ, force, force_every, components)
            ys.append(torch.from_numpy(y.astype(np.float32).reshape(-1)).to(Xs[-1].device))
            ahead = horizon
        else:
            ys.append(sel.closure_targets(fine, coarse).reshape(-1))
    torch.cuda.synchronize()
    return Samples(torch.cat(Xs), torch.cat(ys), times)


@dataclass
class TrainResult:
    blob: np.ndarray
    train_loss: List[float]
    val_loss: List[float]
    steps: int


def train(samples: Samples, epochs: int = 20, batch: int = 4096, lr: float = 1e-3, seed: int = 0,
          val_frac: float = 0.1, dtau_max: float = 100.0) -> TrainResult:
    """Adam (lr, 0.9, 0.999, 1e-8) on seeded minibatches; a seeded hold-out
    of val_frac of the rows gives the validation loss after every epoch."""
    torch = _torch()
    X, y = samples.X, samples.y
    M = int(X.shape[0])
    gen = np.random.Generator(np.random.PCG64(seed))
    order = gen.permutation(M)
    nval = max(1, int(M * val_frac))
    tr_rows, val_rows = order[nval:], order[:nval]
    Xh = X.cpu().numpy().astype(np.float64)[tr_rows]
    mean = Xh.mean(0)
    std = Xh.std(0)
    std = np.where(std > 0, std, 1.0)
    blob = I.closure_blob(seed, mean, std, dtau_max=dtau_max)
    P = torch.from_numpy(blob).to(X.device)
    trainer = sel.MLPTrainer(P, lr=lr)
    val_idx = torch.from_numpy(val_rows.astype(np.int32)).to(X.device)
    tr_idx_h = tr_rows.astype(np.int32)
    hist_t, hist_v = [], []
    work = sel.mlp_work(max(batch, nval), X.device)
    for _ in range(epochs):
        perm = torch.from_numpy(tr_idx_h[gen.permutation(tr_idx_h.size)]).to(X.device)
        last = None
        for b in range(0, perm.numel(), batch):
            last = trainer.step(X, y, idx=perm[b:b + batch], want_loss=(b + batch >= perm.numel()))
        hist_t.append(float(last))
        _, vl = sel.mlp_gradient(P, X, y, idx=val_idx, work=work)
        hist_v.append(float(vl))
    return TrainResult(P.cpu().numpy(), hist_t, hist_v, trainer.t)


@dataclass
class Judgement:
    times: List[float]
    err_plain: List[float]
    err_closure: List[float]
    ke_ref: List[float]
    ke_plain: List[float]
    ke_closure: List[float]
    # averaged axial velocity profile (sel_radial_profile), when asked for
    prof_ref: List[np.ndarray] = field(default_factory=list)
    prof_plain: List[np.ndarray] = field(default_factory=list)
    prof_closure: List[np.ndarray] = field(default_factory=list)

    @property
    def gain_profile(self) -> float:
        """Mean relative error of the averaged profile, plain over closure."""
        ep = [np.linalg.norm(p - r) / np.linalg.norm(r) for p, r in zip(self.prof_plain, self.prof_ref)]
        ec = [np.linalg.norm(p - r) / np.linalg.norm(r) for p, r in zip(self.prof_closure, self.prof_ref)]
        return float(np.mean(ep) / max(np.mean(ec), 1e-300))

    @property
    def gain(self) -> float:
        """Mean velocity error of the plain coarse run over that of the closure run."""
        return float(np.mean(self.err_plain) / max(np.mean(self.err_closure), 1e-300))

    @property
    def gain_ke(self) -> float:
        """Mean kinetic-energy error of the plain coarse run over that of the closure run."""
        r = np.asarray(self.ke_ref)
        ep = np.abs(np.asarray(self.ke_plain) - r).mean()
        ec = np.abs(np.asarray(self.ke_closure) - r).mean()
        return float(ep / max(ec, 1e-300))


def _l2(u, uref, wJ):
    d = ((u - uref) ** 2).sum(-1)
    r = (uref ** 2).sum(-1)
    return float(np.sqrt((wJ * d).sum() / max((wJ * r).sum(), 1e-300)))


def judge(make_case, Nf: int, Nc: int, blob, nchk: int, every: int, precision: str = "fp32dev",
          device: str = "cuda:0", force=None, force_every: int = 5, profile=None) -> Judgement:
    """Coarse runs with and without the closure against the coarse-grained
    fine run, compared every ``every`` steps (relative wJ-weighted L2 error of
    u, and kinetic energy; with profile = (origin, axis, rmax, nbins) also the
    averaged axial velocity profile). force: optional time-dependent force
    density per node of every run, set every force_every steps."""
    cf, cc = coarse_pair(make_case, Nf, Nc)
    fine = sel.from_case(cf, precision=precision, device=device)
    ref = sel.from_case(cc, precision=precision, device=device)
    plain = sel.from_case(cc, precision=precision, device=device)
    clos = sel.from_case(cc, precision=precision, device=device, closure=blob)
    sel.coarse_grain(fine, plain)
    sel.coarse_grain(fine, clos)
    wJ, _ = ref.geometry()
    dim = cc.dim
    J = Judgement([], [], [], [], [], [])
    for _ in range(nchk):
        _advance([(cf, fine), (cc, plain), (cc, clos)], every, force, force_every)
        sel.coarse_grain(fine, ref)
        _, ur = ref.moments()
        _, up = plain.moments()
        _, uc = clos.moments()
        J.times.append(fine.time)
        J.err_plain.append(_l2(up, ur, wJ))
        J.err_closure.append(_l2(uc, ur, wJ))
        J.ke_ref.append(float(ref.reduce()[dim + 1]))
        J.ke_plain.append(float(plain.reduce()[dim + 1]))
        J.ke_closure.append(float(clos.reduce()[dim + 1]))
        if profile is not None:
            for sim, lst in ((ref, J.prof_ref), (plain, J.prof_plain), (clos, J.prof_closure)):
                s_un, s_w = sim.radial_profile(*profile)
                lst.append(s_un / np.where(s_w > 0, s_w, 1.0))
    return J
