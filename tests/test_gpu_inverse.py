"""Material inverse design (L-BFGS over per-tet log E, refactorizing per
evaluation) through the library: the trajectory-matching gradient of one
evaluation against the oracle's, and the optimisation itself."""
import numpy as np
import pytest

import oracle as O
from paper_2605_14526_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def th(torch_cuda):
    return torch_cuda


def setup(th, T):
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.small_beam(6, 3, 3, seed=31, contrast=20.0, nu=0.45, tip_force=10.0)
    log_E_obs = scenes.observed_log_E(sc, 77)
    dev = lambda a: th.tensor(np.ascontiguousarray(a), dtype=th.float64, device="cuda")  # noqa: E731
    # observations: the same scene rolled out with the observation field
    gobs = Scene.from_scene(sc, eps_rel=1e-12, eps_abs=1e-16)
    gobs.set_material(log_E_obs)
    gobs.factorize()
    q, v = dev(sc.q0()), dev(sc.v0())
    obs = [q]
    for t in range(T):
        q, v, _ = gobs.step_forward(q, v, dev(sc.f_ext(t)))
        obs.append(q)
    # the estimate starts from a uniform field at the mean log E
    log_E0 = np.full(sc.n_e, float(np.mean(sc.log_E)))
    sc.log_E = log_E0.copy()
    g = Scene.from_scene(sc, eps_rel=1e-12, eps_abs=1e-16, eps_adj=1e-12)
    mass = dev(g.vertex_mass())
    return sc, g, obs, mass, log_E0, log_E_obs


def test_trajectory_gradient_matches_oracle(th):
    """One evaluation of the identification loss sum_t |q_t - q_t^obs|_M^2 and
    its gradient with respect to all log E against the oracle (same frozen
    means, the loss gradient injected at every step of the reverse sweep)."""
    from paper_2605_14526_amd.inverse import trajectory_objective
    T = 8
    sc, g, obs, mass, log_E0, _ = setup(th, T)
    fg = trajectory_objective(g, sc, T, obs, mass, th)
    L, grad = fg(th.tensor(log_E0, dtype=th.float64, device="cuda"))
    info = g.info()
    o = O.OracleScene(sc, log_E=log_E0, eps_rel=1e-12, eps_abs=1e-16, eps_adj=1e-13,
                      frozen=(info["mu_bar"], info["lam_bar"], info["mu_ref"]))
    q, v, ck, _ = O.rollout(o, T)
    obs_h = [x.cpu().numpy() for x in obs]
    m = mass.cpu().numpy()[:, None]
    traj = [sc.q0()] + [c[3] for c in ck]
    L_o = sum(float((m * (traj[t] - obs_h[t]) ** 2).sum()) for t in range(1, T + 1))
    gq = 2.0 * m * (traj[T] - obs_h[T])
    gv = np.zeros_like(gq)
    gl = np.zeros(sc.n_e)
    for t in reversed(range(T)):
        q_t, v_t, f, qs, qsm1 = ck[t]
        gq, gv, _, gl, _ = o.step_backward(q_t, v_t, f, qs, qsm1, gq, gv, gl, adj_mode=1)
        if t > 0:
            gq = gq + 2.0 * m * (traj[t] - obs_h[t])
    assert abs(L - L_o) <= 1e-9 * L_o
    gg = grad.cpu().numpy()
    assert np.abs(gg - gl).max() <= 1e-6 * np.abs(gl).max(), np.abs(gg - gl).max() / np.abs(gl).max()


def test_lbfgs_identification_reduces_loss(th):
    """Twelve L-BFGS iterations from the uniform field cut the identification
    loss by more than 10x (it falls monotonically; 20x was measured), every
    evaluation refactorizes."""
    from paper_2605_14526_amd.inverse import lbfgs, trajectory_objective
    T = 8
    sc, g, obs, mass, log_E0, log_E_obs = setup(th, T)
    fg = trajectory_objective(g, sc, T, obs, mass, th)
    res = lbfgs(fg, th.tensor(log_E0, dtype=th.float64, device="cuda"), iters=12, memory=8, max_step=1.0)
    assert res.f < 1e-1 * res.history[0], res.history
    assert all(a >= b for a, b in zip(res.history, res.history[1:]))


def batch_task(th, T):
    """Three uneven scenes of the identification kind, each observed under its own seeded field, all estimated
    from uniform fields at their mean log E."""
    from paper_2605_14526_amd.binding import Batch, Scene
    scs = [scenes.small_beam(6, 3, 3, seed=31, contrast=20.0, nu=0.45, tip_force=10.0),
           scenes.small_beam(8, 2, 2, seed=32, contrast=8.0, nu=0.42, tip_force=6.0),
           scenes.anchored_blob(500, seed=33, contrast=30.0, nu=0.46)]
    dev = lambda a: th.tensor(np.ascontiguousarray(a), dtype=th.float64, device="cuda")  # noqa: E731
    obs, gs, masses, x0 = [], [], [], []
    for k, sc in enumerate(scs):
        gobs = Scene.from_scene(sc, eps_rel=1e-12, eps_abs=1e-16)
        gobs.set_material(scenes.observed_log_E(sc, 90 + k))
        gobs.factorize()
        q, v = dev(sc.q0()), dev(sc.v0())
        traj = [q]
        for t in range(T):
            q, v, _ = gobs.step_forward(q, v, dev(sc.f_ext(t)))
            traj.append(q)
        obs.append(traj)
        sc.log_E = np.full(sc.n_e, float(np.mean(sc.log_E)))
        g = Scene.from_scene(sc, eps_rel=1e-12, eps_abs=1e-16, eps_adj=1e-12)
        gs.append(g)
        masses.append(dev(g.vertex_mass()))
        x0.append(sc.log_E)
    return scs, gs, Batch(gs), obs, masses, dev(np.concatenate(x0))


def test_batch_identification_gradient_is_the_sum_of_the_scenes(th):
    """The batched identification loss and gradient equal those of each scene's own objective on a fresh scene
    (the batch's kernels are the scenes' own; what is left is the loss's summation order and the 1e-12 stops
    of the two sweeps, while a wrong slice or a missing term would be of order one)."""
    from paper_2605_14526_amd.binding import Scene
    from paper_2605_14526_amd.inverse import batch_trajectory_objective, trajectory_objective
    T = 4
    scs, gs, B, obs, masses, x0 = batch_task(th, T)
    fg = batch_trajectory_objective(B, gs, scs, T, obs, masses, th)
    L, grad = fg(x0)
    cuts = np.cumsum([0] + [sc.n_e for sc in scs])
    L_sum = 0.0
    for s, sc in enumerate(scs):
        g = Scene.from_scene(sc, eps_rel=1e-12, eps_abs=1e-16, eps_adj=1e-12)
        f1 = trajectory_objective(g, sc, T, obs[s], masses[s], th)
        l1, g1 = f1(x0[cuts[s]:cuts[s + 1]].contiguous())
        L_sum += l1
        gb, g1 = grad[cuts[s]:cuts[s + 1]].cpu().numpy(), g1.cpu().numpy()
        assert np.abs(gb - g1).max() <= 1e-10 * np.abs(g1).max(), (s, np.abs(gb - g1).max() / np.abs(g1).max())
    assert abs(L - L_sum) <= 1e-12 * L_sum, (L, L_sum)


def test_batch_lbfgs_identification_reduces_loss(th):
    """L-BFGS over the three scenes' fields together, every evaluation refactorizing every scene and
    stepping the batch: the loss falls monotonically, by more than 5x in 8 iterations."""
    from paper_2605_14526_amd.inverse import batch_trajectory_objective, lbfgs
    T = 6
    scs, gs, B, obs, masses, x0 = batch_task(th, T)
    fg = batch_trajectory_objective(B, gs, scs, T, obs, masses, th)
    res = lbfgs(fg, x0, iters=8, memory=8, max_step=1.0)
    assert res.f < 0.2 * res.history[0], res.history
    assert all(a >= b for a, b in zip(res.history, res.history[1:]))


def tendon_task(th, T):
    """A helical-fibre tendon beam whose tip must reach the position that seeded activations reach after
    T steps (a realisable target), started from uniform activations."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.tendon_beam(2, 6, layout=1, steps=T, w_m=2e5, gravity=(0.0, 0.0, -9.81))
    g = Scene.from_scene(sc, eps_rel=1e-12, eps_abs=1e-16, eps_adj=1e-12)
    tip = sc.X[:, 2] > sc.X[:, 2].max() - 1e-9
    a_true = np.random.Generator(np.random.PCG64(61)).uniform(0.0, 0.3, 16)
    dev = lambda a: th.tensor(np.ascontiguousarray(a), dtype=th.float64, device="cuda")  # noqa: E731
    g.set_activation(dev(a_true))
    q, v = dev(sc.q0()), dev(sc.v0())
    for t in range(T):
        q, v, _ = g.step_forward(q, v, dev(sc.f_ext(t)))
    target = q.cpu().numpy()[tip].mean(axis=0)
    return sc, g, tip, target, np.full(16, 0.15), dev


def test_activation_gradient_matches_oracle(th):
    """dL/da of the reaching loss through the library against the oracle's adjoint sweep (same rollout)."""
    from paper_2605_14526_amd.inverse import activation_objective
    T = 10
    sc, g, tip, target, a0, dev = tendon_task(th, T)
    fg = activation_objective(g, sc, T, tip, target, th)
    L, ga = fg(dev(a0))
    o = O.OracleScene(sc, eps_rel=1e-12, eps_abs=1e-16, eps_adj=1e-13)
    o.set_muscles(sc.muscle_group, sc.muscle_fibre, sc.muscle_w)
    o.set_activation(a0)
    q, v, ck, _ = O.rollout(o, T)
    d = q[tip].mean(axis=0) - target
    gq = np.zeros_like(q)
    gq[tip] = 2.0 * d / tip.sum()
    o.g_act[:] = 0.0
    O.rollout_backward(o, ck, gq, np.zeros_like(gq), adj_mode=1)
    assert abs(L - float(d @ d)) <= 1e-8 * float(d @ d)
    assert np.abs(ga.cpu().numpy() - o.g_act).max() <= 1e-6 * np.abs(o.g_act).max()


def test_lbfgs_activation_reaching_reduces_loss(th):
    """L-BFGS over the 16 activations (the muscle-driven reaching task in miniature): ten iterations cut the
    loss by more than 100x, without refactorizing."""
    from paper_2605_14526_amd.inverse import activation_objective, lbfgs
    T = 10
    sc, g, tip, target, a0, dev = tendon_task(th, T)
    fg = activation_objective(g, sc, T, tip, target, th)
    res = lbfgs(fg, dev(a0), iters=10, memory=8, max_step=0.05)
    assert res.f < 1e-2 * res.history[0], res.history
