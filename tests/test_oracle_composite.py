"""Pins of the oracle's corotated + volume composite (the paper's default
heterogeneous PD assembly: a corotated rotation step with weight 2 mu_e and a
volume step with weight lam_e, Sec. 4.1 and Sec. 7.2) against closed forms,
brute force, finite differences and the invariants of the PD iteration.  CPU
only."""
import copy

import numpy as np
import pytest
from scipy import linalg, optimize

import oracle as O
from paper_2605_14526_amd import scenes


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def rot(seed):
    q, r = np.linalg.qr(rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


MU, LAM = 1.0e5, 4.0e5


@pytest.mark.parametrize("seed", range(8))
def test_volume_step_is_the_closest_unit_determinant_point(seed):
    """Brute force: minimise |s - sF|^2 over s = exp(x), x1 + x2 + x3 = 0."""
    sF = rng(seed).uniform(0.6, 1.7, 3)
    s, _ = O.volume_project(sF)
    assert abs(np.prod(s) - 1.0) < 1e-14

    def obj(x2):
        x = np.array([x2[0], x2[1], -x2[0] - x2[1]])
        return float(np.sum((np.exp(x) - sF) ** 2))

    best = None
    for x0 in ([0.0, 0.0], list(np.log(sF[:2])), [0.3, -0.3], [-0.3, 0.3]):
        r = optimize.minimize(obj, x0, method="BFGS", options={"gtol": 1e-14})
        if best is None or r.fun < best.fun:
            best = r
    xb = np.array([best.x[0], best.x[1], -best.x[0] - best.x[1]])
    assert np.abs(np.exp(xb) - s).max() < 1e-7
    assert np.sum((s - sF) ** 2) <= best.fun + 1e-15


def test_volume_step_special_cases():
    """sF = t (1, 1, 1) projects to (1, 1, 1); a unit-determinant sF is fixed."""
    for t in (0.7, 1.0, 1.3):
        s, _ = O.volume_project(t * np.ones(3))
        assert np.abs(s - 1.0).max() < 1e-14
    sF = np.array([1.2, 0.9, 1.0 / (1.2 * 0.9)])
    s, _ = O.volume_project(sF)
    assert np.abs(s - sF).max() < 1e-14


@pytest.mark.parametrize("seed", range(5))
def test_volume_step_jacobian_fd(seed):
    sF = rng(10 + seed).uniform(0.7, 1.5, 3)
    D = O.volume_diff(sF)
    h = 1e-6
    Dfd = np.zeros((3, 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        Dfd[:, j] = (O.volume_project(sF + e)[0] - O.volume_project(sF - e)[0]) / (2 * h)
    assert np.abs(D - Dfd).max() < 1e-7
    assert np.allclose(D, D.T, atol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_rotation_step_is_the_polar_factor(seed):
    """With lam = 0 the composite is the rotation of the polar decomposition F = R S."""
    F = np.eye(3) + 0.3 * rng(20 + seed).standard_normal((3, 3))
    if np.linalg.det(F) < 0:
        F[:, 0] *= -1
    R, S = linalg.polar(F)
    assert np.abs(O.composite_map(F, MU, 0.0) - R).max() < 1e-13
    # with mu = 0 it is the volume step: determinant 1, same singular vectors
    P = O.composite_map(F, 0.0, LAM)
    assert abs(np.linalg.det(P) - 1.0) < 1e-13
    U, s, Vt = np.linalg.svd(F)
    sv, _ = O.volume_project(s)
    assert np.abs(P - U @ np.diag(sv) @ Vt).max() < 1e-12


@pytest.mark.parametrize("seed", range(5))
def test_composite_jacobian_fd_and_symmetry(seed):
    F = rot(30 + seed) @ np.diag(rng(40 + seed).uniform(0.8, 1.3, 3)) @ rot(50 + seed).T
    J = O.composite_jacobian(F, MU, LAM)
    h = 1e-6
    Jfd = np.zeros((9, 9))
    for c in range(9):
        E = np.zeros(9)
        E[c] = h
        Jfd[:, c] = ((O.composite_map(F + E.reshape(3, 3), MU, LAM) -
                      O.composite_map(F - E.reshape(3, 3), MU, LAM)) / (2 * h)).ravel()
    assert np.abs(J - Jfd).max() < 1e-7
    assert np.abs(J - J.T).max() < 1e-12


def test_composite_jacobian_at_rest():
    """At F = R: rotations pass unchanged, deviatoric symmetric strain is kept
    by the volume step only (factor lam/(2 mu + lam)), volumetric strain by
    neither."""
    th = LAM / (2 * MU + LAM)
    for R in (np.eye(3), rot(7)):
        J = O.composite_jacobian(R, MU, LAM)
        ap = lambda dF: (J @ dF.ravel()).reshape(3, 3)  # noqa: E731
        W = np.array([[0, 1, 0], [-1, 0, 0], [0, 0, 0.0]])
        S = np.array([[0, 1, 0], [1, 0, 0], [0, 0, 0.0]])
        Dv = np.diag([1.0, -1.0, 0.0])
        assert np.allclose(ap(W @ R), W @ R, atol=1e-12)
        assert np.allclose(ap(S @ R), th * S @ R, atol=1e-12)
        assert np.allclose(ap(Dv @ R), th * Dv @ R, atol=1e-12)
        assert np.allclose(ap(R), 0 * R, atol=1e-12)


def composite_scene(**kw):
    sc = copy.copy(scenes.small_beam(5, 2, 2, **kw))
    sc.energy = 1
    return sc


def test_composite_rest_state_zero_force():
    sc = composite_scene(seed=2, tip_force=0.0, gravity=(0.0, 0.0, 0.0))
    osc = O.OracleScene(sc)
    qn, vn, qm1, st = osc.step_forward(sc.X, np.zeros_like(sc.X), record=4)
    assert st["iters"] == 2 and st["status"] == 0
    assert np.abs(qn - sc.X).max() < 1e-14
    c, _ = osc.const_rhs(sc.X, np.zeros_like(sc.X))
    b = osc.local_rhs(sc.X) + c
    free = ~sc.pinned.astype(bool)
    AX = osc.apply_A(sc.X)
    assert np.abs(AX[free] - b[free]).max() <= 1e-14 * np.abs(b[free]).max()


def composite_energy(osc, sc, q, qt, qtil):
    """E(q) = inertia + dissipation + sum_e V_e (mu_e dist(F, SO(3))^2 + lam_e/2 dist(F, det = 1)^2)."""
    info = osc.info()
    h = sc.h
    m = info["mass"]
    free = ~sc.pinned.astype(bool)
    E = 0.5 / h ** 2 * np.sum(m[:, None] * (q - qtil) ** 2 * free[:, None])
    E += 0.5 / h * sc.alpha * np.sum(m[:, None] * (q - qt) ** 2 * free[:, None])
    for t in range(sc.n_e):
        Xs = sc.X[sc.tets[t]]
        Bi = np.linalg.inv((Xs[1:] - Xs[0]).T)
        F = (q[sc.tets[t]][1:] - q[sc.tets[t]][0]).T @ Bi
        Ft = (qt[sc.tets[t]][1:] - qt[sc.tets[t]][0]).T @ Bi
        Ee = np.exp(sc.log_E[t])
        mu, lam = Ee / (2 * (1 + sc.nu)), Ee * sc.nu / ((1 + sc.nu) * (1 - 2 * sc.nu))
        R, _ = linalg.polar(F)
        U, s, Vt = np.linalg.svd(F)
        Pv = U @ np.diag(O.volume_project(s)[0]) @ Vt
        V = info["vol"][t]
        E += V * (mu * np.sum((F - R) ** 2) + 0.5 * lam * np.sum((F - Pv) ** 2))
        E += 0.5 / h * info["beta"][t] * V * np.sum((F - Ft) ** 2)
    return E


def test_composite_monotone_energy_plain_iteration():
    """Plain local-global (AA off) alternates exact minimisations, so the
    composite's PD energy decreases at every iteration."""
    sc = composite_scene(seed=6, contrast=50.0, tip_force=40.0, nu=0.45)
    osc = O.OracleScene(sc, m=0)
    q, v = sc.X.copy(), np.zeros_like(sc.X)
    f = sc.f_ext(3)
    qn, vn, qm1, st = osc.step_forward(q, v, f, force_iters=25, m=0, record=26)
    _, qtil = osc.const_rhs(q, v, f)
    Es = [composite_energy(osc, sc, st["record"][k], q, qtil) for k in range(26)]
    d = np.diff(Es)
    assert np.all(d <= 1e-12 * abs(Es[0])), d
    assert Es[-1] < Es[0]


def test_composite_K_is_db_dq():
    """K x (Eq. db_dq with the composite's differentials) against central
    differences of b(q), and K symmetric."""
    sc = composite_scene(seed=12, contrast=20.0)
    osc = O.OracleScene(sc)
    r = rng(12)
    q = sc.X + 3e-3 * r.standard_normal(sc.X.shape)
    q[sc.pinned.astype(bool)] = sc.X[sc.pinned.astype(bool)]
    free = ~sc.pinned.astype(bool)
    x = r.standard_normal(sc.X.shape) * free[:, None]
    y = r.standard_normal(sc.X.shape) * free[:, None]
    Kx = osc.apply_K(q, 1.0, x)
    h = 1e-7
    fd = (osc.local_rhs(q + h * x) - osc.local_rhs(q - h * x)) / (2 * h)
    assert np.abs((Kx - fd)[free]).max() < 1e-6 * np.abs(Kx[free]).max()
    assert abs(np.sum(y * Kx) - np.sum(x * osc.apply_K(q, 1.0, y))) < 1e-10 * abs(np.sum(y * Kx))


def test_composite_gradients_match_central_differences():
    sc = composite_scene(seed=13, contrast=10.0, tip_force=20.0, alpha=0.2, beta_rel=0.02)
    base = O.OracleScene(sc).info()
    frozen = (base["mu_bar"], base["lam_bar"], base["mu_ref"])
    steps = 3

    def run(logE, q0, v0):
        osc = O.OracleScene(sc, log_E=logE, eps_rel=1e-14, eps_abs=1e-16, frozen=frozen, eps_adj=1e-14)
        q, v = q0.copy(), v0.copy()
        ck = []
        for t in range(steps):
            f = sc.f_ext(t)
            qn, vn, qm1, st = osc.step_forward(q, v, f)
            ck.append((q, v, f, qn, qm1))
            q, v = qn, vn
        L, gq = scenes.centroid_loss(q, sc.target_centroid)
        return L, gq, ck, osc

    q0 = sc.X + 1e-3 * rng(1).standard_normal(sc.X.shape)
    q0[sc.pinned.astype(bool)] = sc.X[sc.pinned.astype(bool)]
    v0 = 0.05 * rng(2).standard_normal(sc.X.shape)
    v0[sc.pinned.astype(bool)] = 0
    L, gq, ck, osc = run(sc.log_E, q0, v0)
    gv = np.zeros_like(gq)
    gl = np.zeros(sc.n_e)
    for (q_t, v_t, f, qs, qsm1) in reversed(ck):
        gq, gv, gf, gl, st = osc.step_backward(q_t, v_t, f, qs, qsm1, gq, gv, gl, adj_mode=1)
    for e in rng(3).choice(sc.n_e, 3, replace=False):
        h = 1e-4  # the bisection of the volume step leaves rounding noise of ~1e-16 in L
        lp, lm = sc.log_E.copy(), sc.log_E.copy()
        lp[e] += h
        lm[e] -= h
        fd = (run(lp, q0, v0)[0] - run(lm, q0, v0)[0]) / (2 * h)
        assert np.isclose(gl[e], fd, rtol=2e-5, atol=1e-9 * abs(L)), (e, gl[e], fd)
    free = np.where(~sc.pinned.astype(bool))[0]
    for (vtx, ax) in [(free[3], 1), (free[-1], 2)]:
        h = 1e-6
        for which, g in ((0, gq), (1, gv)):
            xp = [q0.copy(), v0.copy()]
            xm = [q0.copy(), v0.copy()]
            xp[which][vtx, ax] += h
            xm[which][vtx, ax] -= h
            fd = (run(sc.log_E, xp[0], xp[1])[0] - run(sc.log_E, xm[0], xm[1])[0]) / (2 * h)
            assert np.isclose(g[vtx, ax], fd, rtol=1e-4, atol=1e-8 * abs(L)), (which, g[vtx, ax], fd)
