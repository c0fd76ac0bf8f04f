"""Pins of the oracle's muscle actuation (fibre constraints with activations) against
mathematics fixed independently of the oracle: the fibre projection is the closest point
of a sphere, the muscle's part of A~ q - b(q) is the gradient of its energy, K is the
derivative of b, the activated free bar contracts to the fibre length 1 - a, the rest
state is a fixed point at zero activation, and dL/da and dL/dlog E match central
differences through a rollout.  CPU only."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2605_14526_amd import scenes


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def muscle_scene(sc, act=None, **kw):
    o = O.OracleScene(sc, **kw)
    o.set_muscles(sc.muscle_group, sc.muscle_fibre, sc.muscle_w)
    o.set_activation(sc.activation if act is None else act)
    return o


def def_grad(sc, q):
    Dm = np.stack([sc.X[sc.tets[:, k]] - sc.X[sc.tets[:, 0]] for k in (1, 2, 3)], axis=2)
    Ds = np.stack([q[sc.tets[:, k]] - q[sc.tets[:, 0]] for k in (1, 2, 3)], axis=2)
    return Ds @ np.linalg.inv(Dm), np.abs(np.linalg.det(Dm)) / 6.0


def muscle_energy(sc, q, act):
    """sum_e (w_m V_e / 2) dist(F_e m_e, sphere of radius 1 - a_g)^2, written from the definition."""
    F, V = def_grad(sc, q)
    f = np.einsum("eij,ej->ei", F, sc.muscle_fibre)
    ell = 1.0 - act[sc.muscle_group]
    return 0.5 * sc.muscle_w * np.sum(V * (np.linalg.norm(f, axis=1) - ell) ** 2)


def one_tet_scene(fibre):
    sc = scenes.tendon_beam(1, 1, layout=0, w_m=1.0, E=1e-9)
    t = sc.tets[:1]
    X = sc.X[t[0]].copy()
    return dataclasses.replace(sc, X=X, tets=np.arange(4, dtype=np.int32)[None, :], pinned=np.zeros(4, np.uint8),
                               log_E=sc.log_E[:1], muscle_group=np.zeros(1, np.int32),
                               muscle_fibre=np.asarray(fibre, float)[None, :], activation=np.zeros(1))


def test_fibre_projection_is_closest_point_of_sphere():
    """On one tet the muscle's b is w_m V (c (x) p) with c_a = Bhat_a . m: the p recovered from the
    oracle's b must be the point of the sphere |p| = 1 - a nearest to f = F m (brute force over
    sampled directions)."""
    r = rng(3)
    dirs = r.standard_normal((400000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    for trial in range(5):
        m = r.standard_normal(3)
        m /= np.linalg.norm(m)
        sc = one_tet_scene(m)
        a = r.uniform(0.0, 0.5)
        o = O.OracleScene(sc)
        o.set_muscles(sc.muscle_group, sc.muscle_fibre, 1.0)
        o.set_activation(np.array([a]))
        q = sc.X + 0.02 * r.standard_normal(sc.X.shape)
        bm = o.local_rhs(q) - O.OracleScene(sc).local_rhs(q)
        Dm = (sc.X[1:] - sc.X[0]).T
        V = abs(np.linalg.det(Dm)) / 6.0
        Bi = np.linalg.inv(Dm)
        grads = np.vstack([-Bi.sum(axis=0), Bi])  # shape gradients of the four vertices
        c = grads @ m
        p = (c @ bm) / (V * (c @ c))
        f = ((q[1:] - q[0]).T @ Bi) @ m
        ell = 1.0 - a
        assert abs(np.linalg.norm(p) - ell) < 1e-12
        best = np.min(np.linalg.norm(ell * dirs - f, axis=1))
        assert np.linalg.norm(p - f) <= best + 1e-12
        # and b is exactly that rank-one form
        assert np.allclose(bm, V * np.outer(c, p), rtol=0, atol=1e-12 * np.abs(bm).max())


def test_muscle_residual_is_energy_gradient():
    """(A~ q - b(q)) with muscles minus without = grad of the muscle energy (central differences of the
    energy written from its definition); nothing pinned, so A~ acts on every vertex."""
    sc = scenes.tendon_beam(2, 3, layout=1, w_m=2e5)
    sc = dataclasses.replace(sc, pinned=np.zeros_like(sc.pinned))
    act = sc.activation
    with_m = muscle_scene(sc)
    without = O.OracleScene(sc)
    q = sc.X + 4e-3 * rng(5).standard_normal(sc.X.shape)
    r_m = (with_m.apply_A(q) - with_m.local_rhs(q)) - (without.apply_A(q) - without.local_rhs(q))
    g = np.zeros_like(q)
    h = 1e-7
    for v in range(sc.n_v):
        for a in range(3):
            qp, qm = q.copy(), q.copy()
            qp[v, a] += h
            qm[v, a] -= h
            g[v, a] = (muscle_energy(sc, qp, act) - muscle_energy(sc, qm, act)) / (2 * h)
    assert np.allclose(r_m, g, rtol=1e-6, atol=1e-6 * np.abs(g).max())


def test_muscle_K_is_derivative_of_b():
    sc = scenes.tendon_beam(2, 3, layout=1, w_m=2e5)
    with_m = muscle_scene(sc)
    without = O.OracleScene(sc)
    r = rng(7)
    q = sc.X + 3e-3 * r.standard_normal(sc.X.shape)
    pin = sc.pinned.astype(bool)
    q[pin] = sc.X[pin]
    x, y = r.standard_normal(q.shape), r.standard_normal(q.shape)
    x[pin] = 0
    y[pin] = 0
    Km = lambda z: with_m.apply_K(q, 1.0, z) - without.apply_K(q, 1.0, z)  # noqa: E731
    Kx, Ky = Km(x), Km(y)
    assert np.isclose(np.sum(y * Kx), np.sum(x * Ky), rtol=1e-11)
    h = 1e-7
    bm = lambda z: with_m.local_rhs(z) - without.local_rhs(z)  # noqa: E731
    fd = (bm(q + h * x) - bm(q - h * x)) / (2 * h)
    assert np.allclose(Kx[~pin], fd[~pin], rtol=1e-5, atol=1e-6 * np.abs(Kx).max())


def test_activated_free_bar_contracts_to_fibre_length():
    """A free bar of fibres along its axis, negligible elastic stiffness, no gravity, strong mass
    damping: its rest state under activation a is |F m| = 1 - a in every tet."""
    sc = scenes.tendon_beam(1, 4, layout=0, E=1.0, w_m=1e5, h=0.01)
    sc = dataclasses.replace(sc, pinned=np.zeros_like(sc.pinned), alpha=20.0)
    o = muscle_scene(sc, np.full(16, 0.2), eps_rel=1e-12, eps_abs=1e-14)
    q, v = sc.X.copy(), np.zeros_like(sc.X)
    for _ in range(300):
        q, v, _, st = o.step_forward(q, v)
    F, _ = def_grad(sc, q)
    fm = np.linalg.norm(np.einsum("eij,ej->ei", F, sc.muscle_fibre), axis=1)
    assert np.abs(fm - 0.8).max() < 2e-4, (fm.min(), fm.max())
    assert np.abs(v).max() < 1e-3


def test_rest_state_is_fixed_point_at_zero_activation():
    sc = scenes.tendon_beam(2, 4, layout=1)
    o = muscle_scene(sc, np.zeros(16))
    qn, vn, qm1, st = o.step_forward(sc.X, np.zeros_like(sc.X), record=3)
    assert st["iters"] == 2 and np.abs(qn - sc.X).max() < 1e-14
    # an activation moves it
    o.set_activation(np.full(16, 0.1))
    qn, _, _, _ = o.step_forward(sc.X, np.zeros_like(sc.X))
    assert np.abs(qn - sc.X).max() > 1e-5


def loss_of(sc, act, log_E, steps, frozen, q_target):
    o = O.OracleScene(sc, log_E=log_E, frozen=frozen, eps_rel=1e-13, eps_abs=1e-15, eps_adj=1e-14)
    o.set_muscles(sc.muscle_group, sc.muscle_fibre, sc.muscle_w)
    o.set_activation(act)
    q, v = sc.X.copy(), np.zeros_like(sc.X)
    ck = []
    for t in range(steps):
        qn, vn, qm1, _ = o.step_forward(q, v)
        ck.append((q, v, qn, qm1))
        q, v = qn, vn
    d = q - q_target
    return float(np.sum(d * d)), 2.0 * d, ck, o


@pytest.mark.parametrize("layout", [0, 1])
def test_activation_and_material_gradients_central_differences(layout):
    sc = scenes.tendon_beam(2, 4, layout=layout, steps=3, w_m=2e5, gravity=(0.0, 0.0, -9.81))
    base = O.OracleScene(sc).info()
    frozen = (base["mu_bar"], base["lam_bar"], base["mu_ref"])
    steps = 3
    q_target = sc.X + 0.01 * rng(11).standard_normal(sc.X.shape)
    L, gq, ck, o = loss_of(sc, sc.activation, sc.log_E, steps, frozen, q_target)
    gv = np.zeros_like(gq)
    gl = np.zeros(sc.n_e)
    o.g_act[:] = 0.0
    for (q_t, v_t, qs, qsm1) in reversed(ck):
        gq, gv, _, gl, _ = o.step_backward(q_t, v_t, None, qs, qsm1, gq, gv, gl, adj_mode=1)
    ga = o.g_act.copy()
    h = 1e-6
    for g in (0, 5, 10, 15):
        ap, am = sc.activation.copy(), sc.activation.copy()
        ap[g] += h
        am[g] -= h
        fd = (loss_of(sc, ap, sc.log_E, steps, frozen, q_target)[0] -
              loss_of(sc, am, sc.log_E, steps, frozen, q_target)[0]) / (2 * h)
        assert np.isclose(ga[g], fd, rtol=2e-5, atol=1e-7 * np.abs(ga).max()), (g, ga[g], fd)
    for e in rng(13).choice(sc.n_e, 3, replace=False):
        lp, lm = sc.log_E.copy(), sc.log_E.copy()
        lp[e] += 1e-5
        lm[e] -= 1e-5
        fd = (loss_of(sc, sc.activation, lp, steps, frozen, q_target)[0] -
              loss_of(sc, sc.activation, lm, steps, frozen, q_target)[0]) / 2e-5
        assert np.isclose(gl[e], fd, rtol=2e-5, atol=1e-7 * np.abs(gl).max()), (e, gl[e], fd)
