"""torch.autograd wrapper of a PD rollout (differentiation through T time
steps by the adjoint method of Sec. 4.8, Alg. 2).

The forward pass keeps only the per-step checkpoint records written by the
library (q_t, q tilde, q*, q*-1; Alg. 1's outputs) and, with ``ckpt_every`` > 1,
only the states at segment starts: the reverse sweep then re-runs each
segment's forward steps to rebuild its records before stepping back through
it.  The backward pass recomputes every per-tet quantity it needs (the SVD, the
prox stretches and the filtered prox differential at q*) inside
``pd_step_backward``; nothing else is stored.  All arithmetic runs in the HIP
library; this module only orders the calls and hands tensors across.
"""
from __future__ import annotations

from typing import Optional

from .binding import Scene


def _sync_material(scene: Scene, log_E) -> None:
    """Refactorize when the caller's log E differs from the scene's (Sec. 4.6 policy)."""
    import torch
    if log_E is None:
        return
    le = log_E.detach().to(dtype=torch.float64).contiguous()
    cur = getattr(scene, "_logE_dev", None)
    if cur is None or cur.device != le.device:
        cur = torch.as_tensor(scene._logE, dtype=torch.float64, device=le.device)
    if le.shape != cur.shape or not torch.equal(le, cur):
        scene.set_material_device(le)
        scene.factorize()
    else:
        scene._logE_dev = cur


def _forward_steps(scene: Scene, q, v, forces, t0: int, t1: int, ckpts, keep_states):
    """Steps t0 .. t1-1 from (q, v); writes records into ckpts[t] and returns the states."""
    import torch
    states = []
    for t in range(t0, t1):
        ck = ckpts[t] if ckpts[t] is not None else scene.new_ckpt()
        ckpts[t] = ck
        q, v, st = scene.step_forward(q, v, forces[t] if forces is not None else None, ckpt=ck)
        if st["rc"] != 0:
            raise RuntimeError(f"forward step {t} did not converge: {st}")
        if keep_states:
            states.append(q)
    return q, v, states


def _make_function():
    import torch

    class PDRollout(torch.autograd.Function):
        """Differentiable T-step rollout: (q0, v0, forces, log E) -> (q_0..q_T, v_T)."""

        @staticmethod
        def forward(ctx, scene, steps, ckpt_every, q0, v0, forces, log_E):
            _sync_material(scene, log_E)
            T = int(steps)
            k = max(1, int(ckpt_every))
            q, v = q0.detach().contiguous(), v0.detach().contiguous()
            fr = forces.detach().contiguous() if forces is not None else None
            traj = torch.empty((T + 1,) + tuple(q.shape), dtype=q.dtype, device=q.device)
            traj[0] = q
            ckpts = [None] * T
            seg_states = {0: (q, v)}
            for t0 in range(0, T, k):
                t1 = min(T, t0 + k)
                q, v, states = _forward_steps(scene, q, v, fr, t0, t1, ckpts, True)
                for j, s in enumerate(states):
                    traj[t0 + 1 + j] = s
                if k > 1:
                    # keep only the segment's start state; records are rebuilt in backward
                    for t in range(t0, t1):
                        ckpts[t] = None
                    seg_states[t1] = (q, v)
            ctx.scene, ctx.T, ctx.k = scene, T, k
            ctx.ckpts, ctx.seg_states = ckpts, seg_states
            ctx.forces = fr
            ctx.has_forces = forces is not None
            ctx.has_logE = log_E is not None
            ctx.n_tets = scene.n_tets
            return traj, v

        @staticmethod
        def backward(ctx, g_traj, g_vT):
            scene, T, k = ctx.scene, ctx.T, ctx.k
            shape = ctx.seg_states[0][0].shape
            dev = ctx.seg_states[0][0].device
            g_traj = torch.zeros((T + 1,) + tuple(shape), dtype=torch.float64, device=dev) if g_traj is None else g_traj
            gq = g_traj[T].contiguous().clone()
            gv = torch.zeros(shape, dtype=torch.float64, device=dev) if g_vT is None else g_vT.contiguous().clone()
            g_logE = torch.zeros(ctx.n_tets, dtype=torch.float64, device=dev)
            g_forces = torch.zeros((T,) + tuple(shape), dtype=torch.float64, device=dev) if ctx.has_forces else None
            gq_t = torch.empty_like(gq)
            gv_t = torch.empty_like(gq)
            gf = torch.empty_like(gq)
            scene.adjoint_reset()
            ckpts = ctx.ckpts
            starts = list(range(0, T, k))
            for t0 in reversed(starts):
                t1 = min(T, t0 + k)
                if k > 1:  # rebuild this segment's records
                    q, v = ctx.seg_states[t0]
                    seg = [None] * T
                    _forward_steps(scene, q, v, ctx.forces, t0, t1, seg, False)
                    recs = seg
                else:
                    recs = ckpts
                for t in reversed(range(t0, t1)):
                    _, _, _, _, st = scene.step_backward(recs[t], gq, gv, g_logE=g_logE, gq_t=gq_t, gv_t=gv_t,
                                                         gf_ext=gf)
                    if st["rc"] != 0:
                        raise RuntimeError(f"adjoint step {t} did not converge: {st}")
                    if g_forces is not None:
                        g_forces[t].copy_(gf)
                    gq, gq_t = gq_t, gq
                    gv, gv_t = gv_t, gv
                    gq.add_(g_traj[t])
                if k > 1:
                    del recs
            return (None, None, None, gq, gv, g_forces, g_logE if ctx.has_logE else None)

    return PDRollout


_FN = None


def rollout(scene: Scene, q0, v0, forces=None, log_E=None, steps: Optional[int] = None, ckpt_every: int = 1):
    """Run ``steps`` PD time steps and return (q_0 .. q_T stacked, v_T), differentiable
    with respect to q0, v0, the per-step external forces (T x n_verts x 3) and
    log E (per tet).  Gradients come from the library's adjoint steps."""
    global _FN
    if _FN is None:
        _FN = _make_function()
    if steps is None:
        if forces is None:
            raise ValueError("steps is required without forces")
        steps = int(forces.shape[0])
    return _FN.apply(scene, int(steps), int(ckpt_every), q0, v0, forces, log_E)
