"""End-to-end material inverse design: L-BFGS over the per-tet log Young's
moduli (the system-identification use of Sec. 5.4), with the gradient of a
whole rollout from the library's adjoint steps (Sec. 4.8, Alg. 2).

Every evaluation installs the candidate material, which makes the factor stale
and refactorizes it once (the refactorization policy of Sec. 4.6: A~ depends
on the material, not on the state), then rolls the scene forward and sweeps
the adjoint back.  The optimizer works on device tensors; each evaluation's
arithmetic runs in the HIP library.  The L-BFGS update is the standard
two-loop recursion (Nocedal and Wright, Numerical Optimization, Alg. 7.4) with
a backtracking Armijo line search and a cap on the largest change of any
log E per iteration.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Tuple

import numpy as np


@dataclass
class LbfgsResult:
    x: object
    f: float
    history: List[float] = field(default_factory=list)
    evaluations: int = 0
    iterations: int = 0


def lbfgs(fg: Callable[[object], Tuple[float, object]], x0, iters: int, memory: int = 8, c1: float = 1e-4,
          max_ls: int = 20, max_step: float = 1.0, gtol: float = 0.0) -> LbfgsResult:
    """Minimise f with L-BFGS.  fg(x) returns (f(x), grad f(x)) for a torch
    tensor x.  The search direction is the two-loop recursion over the last
    `memory` curvature pairs (s, y) with s.y > 0, scaled initially by
    s.y / y.y; the step starts at 1 (at the first iteration at 1/|g|_inf),
    is shortened so that no entry moves by more than `max_step`, and is halved
    until the Armijo condition f(x + a d) <= f(x) + c1 a g.d holds."""
    x = x0.detach().clone()
    f, g = fg(x)
    res = LbfgsResult(x=x, f=f, history=[f], evaluations=1)
    S, Y, R = [], [], []
    for it in range(iters):
        if float(g.abs().max()) <= gtol:
            break
        # two-loop recursion
        q = g.clone()
        alphas = []
        for s, y, rho in zip(reversed(S), reversed(Y), reversed(R)):
            a = rho * float((s * q).sum())
            alphas.append(a)
            q.add_(y, alpha=-a)
        if S:
            gamma = float((S[-1] * Y[-1]).sum() / (Y[-1] * Y[-1]).sum())
        else:
            gamma = 1.0 / max(float(g.abs().max()), 1e-300)
        r = q.mul_(gamma)
        for (s, y, rho), a in zip(zip(S, Y, R), reversed(alphas)):
            b = rho * float((y * r).sum())
            r.add_(s, alpha=a - b)
        d = -r
        slope = float((g * d).sum())
        if slope >= 0.0:  # not a descent direction: restart from the gradient
            S, Y, R = [], [], []
            d = -g / max(float(g.abs().max()), 1e-300)
            slope = float((g * d).sum())
        a = min(1.0, max_step / max(float(d.abs().max()), 1e-300))
        accepted = False
        for _ in range(max_ls):
            xn = x + a * d
            fn, gn = fg(xn)
            res.evaluations += 1
            if fn <= f + c1 * a * slope:
                accepted = True
                break
            a *= 0.5
        if not accepted:
            break
        s_, y_ = xn - x, gn - g
        sy = float((s_ * y_).sum())
        if sy > 1e-12 * float(s_.norm() * y_.norm()):
            S.append(s_)
            Y.append(y_)
            R.append(1.0 / sy)
            if len(S) > memory:
                S.pop(0), Y.pop(0), R.pop(0)
        x, f, g = xn, fn, gn
        res.history.append(f)
        res.iterations = it + 1
    res.x, res.f = x, f
    return res


def trajectory_objective(scene, sc, steps: int, observed, mass, torch, ckpt_every: int = 1):
    """The identification loss of one scene as a function of its per-tet log E:
    L(log E) = sum_{t=1..T} sum_v m_v |q_t,v - q^obs_t,v|^2 over a rollout of
    `steps` steps from the scene's initial state and load schedule, where
    `observed` holds q^obs_0..q^obs_T (device tensors) and `mass` the vertex
    masses.  Returns fg(log_E) -> (L, dL/dlog E) for lbfgs; each call
    refactorizes, rolls forward and sweeps the adjoint back through the
    library (autograd.rollout).  The mesh means of the local prox and
    mu_ref are frozen at their values for the scene's current material, so
    that L is exactly the function whose gradient the adjoint returns (the
    means are constants of the gradient)."""
    from . import autograd
    info = scene.info()
    scene.freeze_means((info["mu_bar"], info["lam_bar"], info["mu_ref"]))
    scene.factorize()
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    q0, v0 = dev(sc.q0()), dev(sc.v0())
    forces = torch.stack([dev(sc.f_ext(t)) for t in range(steps)])
    obs = torch.stack(list(observed[: steps + 1]))
    m = mass.reshape(1, -1, 1)

    def fg(log_E):
        le = log_E.detach().clone().requires_grad_(True)
        traj, _ = autograd.rollout(scene, q0, v0, forces=forces, log_E=le, steps=steps, ckpt_every=ckpt_every)
        loss = (m * (traj[1:] - obs[1:]) ** 2).sum()
        loss.backward()
        return float(loss.detach()), le.grad.detach()

    return fg


def batch_trajectory_objective(batch, scenes_, scs, steps: int, observed, masses, torch):
    """The identification loss of a whole batch as a function of every scene's per-tet log E, concatenated in
    the batch's scene order: L = sum over scenes of the trajectory loss of trajectory_objective.  Each call
    installs each scene's share and refactorizes it (the batch picks the new factors up at its next step),
    rolls all scenes forward together with checkpoints (pd_batch_step_forward) and sweeps them back together
    (pd_batch_step_backward), the loss gradient 2 m (q_t - q_t^obs) entering at every step.  `observed[s]`
    holds scene s's q^obs_0..q^obs_T and `masses[s]` its vertex masses (device tensors).  Means frozen per
    scene as in trajectory_objective.  Returns fg(x) -> (L, dL/dx) for lbfgs."""
    sizes = [sc.n_e for sc in scs]
    cuts = np.cumsum([0] + sizes)
    for g in scenes_:
        info = g.info()
        g.freeze_means((info["mu_bar"], info["lam_bar"], info["mu_ref"]))
        g.factorize()
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")  # noqa: E731
    q0 = [dev(sc.q0()) for sc in scs]
    v0 = [dev(sc.v0()) for sc in scs]
    forces = [[dev(sc.f_ext(t)) for sc in scs] for t in range(steps)]
    m2 = [(2.0 * m.reshape(-1, 1)).expand(sc.n_v, 3).contiguous() for m, sc in zip(masses, scs)]

    def fg(x):
        for s, g in enumerate(scenes_):
            g.set_material_device(x[cuts[s]:cuts[s + 1]].contiguous())
            g.factorize()
        q, v = q0, v0
        traj, cks = [q], []
        for t in range(steps):
            ck = [g.new_ckpt() for g in scenes_]
            q, v, _, rc = batch.step_forward(q, v, forces[t], ckpt=ck)
            if rc != 0:
                raise RuntimeError(f"batched forward step {t} did not converge")
            traj.append(q)
            cks.append(ck)
        loss = 0.0
        for t in range(1, steps + 1):
            for s in range(len(scs)):
                d = traj[t][s] - observed[s][t]
                loss += float((m2[s][:, :1] * 0.5 * d * d).sum())
        for g in scenes_:
            g.adjoint_reset()
        g_logE = [torch.zeros(n, dtype=torch.float64, device="cuda") for n in sizes]
        gq = [(traj[steps][s] - observed[s][steps]) * m2[s] for s in range(len(scs))]
        gv = [torch.zeros_like(a) for a in gq]
        for t in reversed(range(steps)):
            gq, gv, _, _, _, rc = batch.step_backward(cks[t], gq, gv, g_logE=g_logE)
            if rc != 0:
                raise RuntimeError(f"batched adjoint step {t} did not converge")
            if t > 0:
                gq = [gq[s] + (traj[t][s] - observed[s][t]) * m2[s] for s in range(len(scs))]
        return loss, torch.cat(g_logE)

    return fg


def activation_objective(scene, sc, steps: int, tip_mask, target, torch):
    """The muscle-driven reaching task of one scene as a function of its
    groups' activations a: L(a) = |mean of q_T over the tip vertices - target|^2
    after a rollout of `steps` steps from the scene's initial state.  Returns
    fg(a) -> (L, dL/da) for lbfgs; each call sets the activations (no
    refactorization: they change b, not A~), rolls forward with checkpoints
    and sweeps the adjoint back, the library adding dL/da into a device buffer
    (pd_scene_set_activation_grad)."""
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    q0, v0 = dev(sc.q0()), dev(sc.v0())
    forces = [dev(sc.f_ext(t)) for t in range(steps)]
    tip = torch.tensor(np.asarray(tip_mask, bool), device="cuda")
    tgt = dev(np.asarray(target, float))
    n_tip = int(tip.sum())
    g_act = torch.zeros(scene.n_groups, dtype=torch.float64, device="cuda")
    scene.set_activation_grad(g_act)

    def fg(a):
        scene.set_activation(a.detach().contiguous())
        q, v = q0, v0
        cks = []
        for t in range(steps):
            ck = scene.new_ckpt()
            q, v, _ = scene.step_forward(q, v, forces[t], ckpt=ck)
            cks.append(ck)
        d = q[tip].mean(dim=0) - tgt
        loss = float((d * d).sum())
        gq = torch.zeros_like(q)
        gq[tip] = 2.0 * d / n_tip
        gv = torch.zeros_like(q)
        g_act.zero_()
        scene.adjoint_reset()
        for ck in reversed(cks):
            gq, gv, _, _, _ = scene.step_backward(ck, gq, gv)
        torch.cuda.synchronize()
        return loss, g_act.clone()

    return fg
