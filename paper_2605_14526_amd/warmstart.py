"""Learned warm start: trajectories from the solver, training of the network
on the GPU, and rollouts that start each step from its prediction.

The network (pd_mpn_*) predicts q_{t+h} - (q_t + h v_t); the step still runs
the PD iteration to the same dual gate, so the prediction only moves the
starting point (Alg. 1 otherwise starts from q_t).  Every product of the
network, its gradient and the Adam update run in the HIP library; this module
orders the calls and keeps the samples as device tensors.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import List

import numpy as np

from .binding import Mpn, Scene


@dataclass
class Sample:
    q_t: object
    v_tm1: object
    v_t: object
    f: object
    q_next: object
    logw: object


def scene_inputs(sc, torch):
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")  # noqa: E731
    return dev


def generate(scenes_list, steps: int, torch, **solver_kw) -> List[Sample]:
    """Plain-start rollouts of each scene with the solver; one sample per step."""
    out = []
    for sc in scenes_list:
        dev = scene_inputs(sc, torch)
        g = Scene.from_scene(sc, **solver_kw)
        logw = dev(g.vertex_logw())
        q, v = dev(sc.q0()), dev(sc.v0())
        v_prev = v
        for t in range(steps):
            f = dev(sc.f_ext(t))
            qn, vn, st = g.step_forward(q, v, f)
            out.append(Sample(q, v_prev, v, f, qn, logw))
            v_prev, q, v = v, qn, vn
        g.close()
    return out


def generate_on(g: Scene, scenes_list, steps: int, torch) -> List[Sample]:
    """Plain-start rollouts of family members that share g's mesh and material (one factorization for all)."""
    out = []
    for sc in scenes_list:
        dev = scene_inputs(sc, torch)
        logw = dev(g.vertex_logw())
        q, v = dev(sc.q0()), dev(sc.v0())
        v_prev = v
        for t in range(steps):
            f = dev(sc.f_ext(t))
            qn, vn, st = g.step_forward(q, v, f)
            out.append(Sample(q, v_prev, v, f, qn, logw))
            v_prev, q, v = v, qn, vn
    return out


def output_scale(samples: List[Sample], h: float, pinned) -> float:
    """RMS of the correction q_{t+h} - q_t - h v_t over the samples' free vertices."""
    free = ~np.asarray(pinned, bool)
    acc, n = 0.0, 0
    for s in samples[:: max(1, len(samples) // 64)]:
        d = (s.q_next.cpu().numpy() - s.q_t.cpu().numpy() - h * s.v_t.cpu().numpy())[free]
        acc += float((d * d).sum())
        n += d.size
    return float(np.sqrt(acc / max(n, 1))) or 1.0


def fit_correction_scale(nets: List[Mpn], samples: List[List[Sample]], h: float, torch, stride: int = 4) -> float:
    """The factor alpha that scales the trained network's correction c = q0 - q_t - h v_t so that alpha c is
    closest (least squares over the samples' vertices) to the solver's correction q_{t+h} - q_t - h v_t:
    alpha = sum <c, y> / sum <c, c>.  A network that only partly predicts the correction then moves the start
    by the part it gets right instead of overshooting the inertial guess (alpha = 0 would give that guess
    back).  Every `stride`-th sample of each mesh; the network runs in the library, the two sums on the host."""
    num = den = 0.0
    for net, ss in zip(nets, samples):
        for smp in ss[::stride]:
            q0 = torch.empty_like(smp.q_t)
            net.forward(smp.q_t, smp.v_tm1, smp.v_t, smp.f, smp.logw, q0=q0)
            base = (smp.q_t + h * smp.v_t).cpu().numpy()
            c = q0.cpu().numpy() - base
            y = smp.q_next.cpu().numpy() - base
            num += float((c * y).sum())
            den += float((c * c).sum())
    return num / den if den > 0.0 else 0.0


def train(net: Mpn, samples: List[Sample], epochs: int, lr: float = 1e-3, seed: int = 0, log_every: int = 0,
          lr_decay: float = 1.0):
    """Adam over the samples in a seeded shuffled order; returns the loss of each epoch's last sample."""
    rng = np.random.Generator(np.random.PCG64(seed))
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(samples))
        rate = lr * (lr_decay ** ep)
        for j, i in enumerate(order):
            s = samples[i]
            last = j == len(order) - 1
            loss = net.loss_grad(s.q_t, s.v_tm1, s.v_t, s.f, s.logw, s.q_next, want_loss=last)
            net.adam_step(rate)
        hist.append(loss)
        if log_every and (ep + 1) % log_every == 0:
            print(f"[warmstart] epoch {ep + 1}: loss {loss:.4e}", flush=True)
    return hist


def rollout(g: Scene, sc, steps: int, torch, start: str = "plain", net: Mpn = None, logw=None, ckpts=None):
    """Forward rollout with q0 = q_t ("plain"), q_t + h v_t ("inertial": g must
    have been created with fwd_start = 1) or the network's prediction
    ("learned"); returns (q_T, v_T, iterations per step, seconds)."""
    dev = scene_inputs(sc, torch)
    q, v = dev(sc.q0()), dev(sc.v0())
    forces = [dev(sc.f_ext(t)) for t in range(steps)]
    v_prev = v
    q0 = torch.empty_like(q)
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(steps):
        # "inertial": the scene was created with fwd_start = 1, the library forms q_t + h v_t
        arg = None
        if start == "learned":
            net.forward(q, v_prev, v, forces[t], logw, q0=q0)
            arg = q0
        ck = ckpts[t] if ckpts is not None else None
        qn, vn, st = g.step_forward(q, v, forces[t], q0=arg, ckpt=ck)
        iters.append(st["iters"])
        v_prev, q, v = v, qn, vn
    torch.cuda.synchronize()
    return q, v, iters, time.perf_counter() - t0


def train_for(sc_family, n_train: int, steps: int, epochs: int, torch, seed: int = 0, compute: int = 0,
              lr: float = 1e-3, log_every: int = 0, edge_weight: float = 0.0):
    """Generate n_train family members' trajectories and train a fresh network on them."""
    train_scenes = [sc_family(k) for k in range(n_train)]
    samples = generate(train_scenes, steps, torch)
    net = Mpn.for_scene(train_scenes[0], compute=compute, edge_weight=edge_weight)
    net.init_params(seed)
    net.set_output_scale(output_scale(samples, train_scenes[0].h, train_scenes[0].pinned))
    t0 = time.perf_counter()
    hist = train(net, samples, epochs, lr=lr, seed=seed, log_every=log_every, lr_decay=0.9)
    torch.cuda.synchronize()
    return net, hist, time.perf_counter() - t0, len(samples)


def train_shared(master: Mpn, nets: List[Mpn], samples: List[List[Sample]], epochs: int, lr: float = 1e-3,
                 seed: int = 0, lr_decay: float = 1.0):
    """Adam over the samples of several meshes with one set of weights: nets[k] (sharing master's weights,
    gradient and moments) computes the gradient of a sample of mesh k, master takes the Adam step.  The
    samples of all meshes are visited in one seeded shuffled order; returns the loss of each epoch's last
    sample."""
    rng = np.random.Generator(np.random.PCG64(seed))
    flat = [(k, i) for k, ss in enumerate(samples) for i in range(len(ss))]
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(flat))
        rate = lr * (lr_decay ** ep)
        loss = None
        for j, idx in enumerate(order):
            k, i = flat[idx]
            s = samples[k][i]
            loss = nets[k].loss_grad(s.q_t, s.v_tm1, s.v_t, s.f, s.logw, s.q_next, want_loss=j == len(order) - 1)
            master.adam_step(rate)
        hist.append(loss)
    return hist
