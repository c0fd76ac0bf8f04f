"""The torch.autograd rollout (per-step checkpoint records, optional segment
recomputation) against reverse sweeps of the FP64 CPU oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2605_14526_amd import scenes

pytestmark = pytest.mark.gpu

TOL_POS = 1e-9
TOL_GRAD = 1e-6


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.fixture(scope="module")
def th(torch_cuda):
    return torch_cuda


def oracle_grads(sc, logE, T, w_traj):
    """Reverse sweep of the oracle for L = |mean q_T - c*|^2 + w_traj sum_t |q_t|^2 / 2."""
    sc2 = scenes.Scene(**{**sc.__dict__, "log_E": logE})
    o = O.OracleScene(sc2)
    q, v, ck, _ = O.rollout(o, T)
    qs = [sc.q0()] + [c[3] for c in ck]
    _, gq = scenes.centroid_loss(q, sc.target_centroid)
    gq = gq + w_traj * qs[T]
    gv = np.zeros_like(gq)
    gl = np.zeros(sc.n_e)
    gf = [None] * T
    for t in reversed(range(T)):
        q_t, v_t, f, qsr, qsm1 = ck[t]
        gq, gv, gf[t], gl, _ = o.step_backward(q_t, v_t, f, qsr, qsm1, gq, gv, gl, adj_mode=1)
        gq = gq + w_traj * qs[t]
    return q, gq, gv, np.stack(gf), gl


def torch_grads(th, sc, logE, T, w_traj, ckpt_every):
    from paper_2605_14526_amd.autograd import rollout
    from paper_2605_14526_amd.binding import Scene
    g = Scene.from_scene(sc, eps_adj=1e-12, adj_warm=2)
    d = lambda a: th.tensor(np.ascontiguousarray(a), dtype=th.float64, device="cuda", requires_grad=True)  # noqa: E731
    q0, v0 = d(sc.q0()), d(sc.v0())
    forces = d(np.stack([sc.f_ext(t) for t in range(T)]))
    le = d(logE)
    traj, vT = rollout(g, q0, v0, forces, le, ckpt_every=ckpt_every)
    target = th.tensor(sc.target_centroid, dtype=th.float64, device="cuda")
    loss = ((traj[T].mean(dim=0) - target) ** 2).sum() + 0.5 * w_traj * (traj ** 2).sum()
    loss.backward()
    h = lambda t: t.detach().cpu().numpy()  # noqa: E731
    return h(traj[T]), h(q0.grad), h(v0.grad), h(forces.grad), h(le.grad)


@pytest.mark.parametrize("ckpt_every", [1, 3])
def test_autograd_rollout_matches_oracle(th, ckpt_every):
    sc = scenes.small_beam(7, 3, 3, seed=5, contrast=30.0, nu=0.49)
    T, w = 5, 1e-3
    ref = oracle_grads(sc, sc.log_E, T, w)
    got = torch_grads(th, sc, sc.log_E, T, w, ckpt_every)
    assert rel(got[0], ref[0]) < TOL_POS
    for a, b in zip(got[1:], ref[1:]):
        assert rel(a, b) < TOL_GRAD, rel(a, b)


def test_autograd_new_material_refactorizes(th):
    """A log E that differs from the scene's is installed (set_material +
    factorize) before stepping; its gradient is the oracle's for that material."""
    sc = scenes.small_beam(7, 3, 3, seed=5, contrast=30.0, nu=0.49)
    rng = np.random.Generator(np.random.PCG64(77))
    logE = sc.log_E + 0.3 * rng.standard_normal(sc.n_e)
    T = 4
    ref = oracle_grads(sc, logE, T, 0.0)
    got = torch_grads(th, sc, logE, T, 0.0, 1)
    assert rel(got[0], ref[0]) < TOL_POS
    assert rel(got[4], ref[4]) < TOL_GRAD


def test_segment_recompute_equals_full_records(th):
    sc = scenes.small_beam(10, 4, 3, seed=11, contrast=30.0, nu=0.49)
    T = 6
    a = torch_grads(th, sc, sc.log_E, T, 0.0, 1)
    b = torch_grads(th, sc, sc.log_E, T, 0.0, 4)
    for x, y in zip(a, b):
        assert rel(x, y) < 1e-9


def test_autograd_rollout_through_contact(th):
    """The autograd rollout through a landing (contact rows detected by the
    library each step, their records in the checkpoints, segments recomputed)
    against the oracle's reverse sweep with the active rows held fixed."""
    from paper_2605_14526_amd.autograd import rollout
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.drop_blob(res=6, with_box=True)
    osc = O.OracleScene(sc)
    q, v = sc.q0(), sc.v0()
    hist = []
    for t in range(200):  # the oracle's state two steps ahead of the landing
        hist.append((q, v))
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        q, v, _, lam, _ = O.step_forward_contact(osc, q, v, sc.f_ext(t), con)
        if (lam > 0).any():
            break
    q0, v0 = hist[-3]
    T, w_traj = 6, 0.05
    # oracle
    q, v, ck = q0.copy(), v0.copy(), []
    qs = [q0]
    for t in range(T):
        f = sc.f_ext(t)
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        qn, vn, qm1, lam, _ = O.step_forward_contact(osc, q, v, f, con)
        ck.append((q, v, f, qn, qm1, con, lam))
        q, v = qn, vn
        qs.append(q)
    assert sum(int((c[6] > 0).sum()) for c in ck) > 0
    _, gq = scenes.centroid_loss(q, sc.target_centroid)
    gq = gq + w_traj * qs[T]
    gv = np.zeros_like(gq)
    gl = np.zeros(sc.n_e)
    for t in reversed(range(T)):
        q_t, v_t, f, qsr, qsm1, con, lam = ck[t]
        gq, gv, _, gl, _ = O.step_backward_contact(osc, q_t, v_t, f, qsr, qsm1, gq, gv, con, lam, gl, adj_mode=1)
        gq = gq + w_traj * qs[t]
    for ckpt_every in (1, 3):
        g = Scene.from_scene(sc, eps_adj=1e-12, adj_warm=2)
        d = lambda a: th.tensor(np.ascontiguousarray(a), dtype=th.float64, device="cuda", requires_grad=True)  # noqa: E731
        tq0, tv0 = d(q0), d(v0)
        forces = d(np.stack([sc.f_ext(t) for t in range(T)]))
        le = d(sc.log_E)
        traj, vT = rollout(g, tq0, tv0, forces, le, ckpt_every=ckpt_every)
        target = th.tensor(sc.target_centroid, dtype=th.float64, device="cuda")
        loss = ((traj[T].mean(dim=0) - target) ** 2).sum() + 0.5 * w_traj * (traj ** 2).sum()
        loss.backward()
        assert rel(traj[T].detach().cpu().numpy(), q) < TOL_POS
        for a, b in [(tq0.grad, gq), (tv0.grad, gv), (le.grad, gl)]:
            assert rel(a.cpu().numpy(), b) < TOL_GRAD, (ckpt_every, rel(a.cpu().numpy(), b))
