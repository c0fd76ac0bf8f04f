"""Pins of the oracle's logarithmic volume-barrier variant (Sec. 4.1 Eq.
pd_log_volume: the barrier -mu sum ln s + lam/2 (sum ln s)^2 solved by the same
Newton on stretches, registered with weight lam_e next to the corotated
rotation step of weight 2 mu_e) against a closed form, brute force, finite
differences and the invariants of the PD iteration.  CPU only."""
import copy

import numpy as np
import pytest
from scipy import linalg, optimize

import oracle as O
from paper_2605_14526_amd import scenes

MU, LAM = 1.0e5, 4.0e5  # means of the barrier step; its penalty is LAM


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def rot(seed):
    q, r = np.linalg.qr(rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def barrier(s, mu=MU, lam=LAM):
    l = np.sum(np.log(s))
    return -mu * l + 0.5 * lam * l * l


def objective(s, sF, k=LAM):
    return 0.5 * k * np.sum((s - sF) ** 2) + barrier(s)


def isotropic_root(sv, k=LAM):
    """t with k (t - s) - mu/t + 3 lam ln t / t = 0 (stationarity on s = t (1, 1, 1)), by bisection"""
    f = lambda t: k * (t - sv) - MU / t + 3 * LAM * np.log(t) / t  # noqa: E731
    lo, hi = 1e-6, 10.0
    assert f(lo) < 0 < f(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) < 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("sv", [0.6, 1.0, 1.3])
def test_isotropic_closed_form(sv):
    s, it = O.logvol_stretch(sv * np.ones(3), MU, LAM, LAM)
    t = isotropic_root(sv)
    assert np.abs(s - t).max() < 1e-14 * max(1.0, t) and 0 < it < 50


def test_not_the_identity_at_rest():
    """As printed the barrier's gradient at s = 1 is -mu, so the step at rest
    dilates: s* = t (1, 1, 1) with t > 1 from the closed form."""
    s, _ = O.logvol_stretch(np.ones(3), MU, LAM, LAM)
    t = isotropic_root(1.0)
    assert t > 1.0 + 1e-3 and np.abs(s - t).max() < 1e-14


@pytest.mark.parametrize("seed", range(6))
def test_matches_brute_force_minimum(seed):
    sF = rng(seed).uniform(0.5, 1.8, 3)
    s, _ = O.logvol_stretch(sF, MU, LAM, LAM)
    best = None
    for x0 in (np.zeros(3), np.log(sF), np.array([0.3, -0.2, 0.1])):
        r = optimize.minimize(lambda x: objective(np.exp(x), sF) / LAM, x0, method="BFGS",
                              options={"gtol": 1e-13})
        if best is None or r.fun < best.fun:
            best = r
    assert np.abs(np.exp(best.x) - s).max() < 1e-6
    assert objective(s, sF) <= LAM * best.fun + 1e-9 * LAM


@pytest.mark.parametrize("sF", [(1.1, 0.02, 0.9), (1.0, 0.8, -0.3), (1e-4, 1e-4, 2.0)])
def test_barrier_keeps_stretches_positive(sF):
    s, it = O.logvol_stretch(np.array(sF), MU, LAM, LAM)
    assert (s > 0).all() and 0 < it < 50
    # stationarity at the returned point
    l = np.sum(np.log(s))
    g = LAM * (s - np.array(sF)) - MU / s + LAM * l / s
    assert np.abs(g).max() <= 1e-12 * LAM * max(1.0, np.abs(sF).max())


@pytest.mark.parametrize("seed", range(4))
def test_logvol_jacobian_fd_and_symmetry(seed):
    F = rot(30 + seed) @ np.diag(rng(40 + seed).uniform(0.8, 1.3, 3)) @ rot(50 + seed).T
    mu_e, lam_e = 2 * MU, 2 * LAM
    J = O.logvol_jacobian(F, MU, LAM, mu_e, lam_e)
    h = 1e-6
    Jfd = np.zeros((9, 9))
    for c in range(9):
        E = np.zeros(9)
        E[c] = h
        Jfd[:, c] = ((O.logvol_map(F + E.reshape(3, 3), MU, LAM, mu_e, lam_e) -
                      O.logvol_map(F - E.reshape(3, 3), MU, LAM, mu_e, lam_e)) / (2 * h)).ravel()
    assert np.abs(J - Jfd).max() < 1e-7
    assert np.abs(J - J.T).max() < 1e-12


def test_logvol_map_is_the_weighted_sum_of_the_steps():
    """(2 mu R + lam U diag(s*) V^T) / (2 mu + lam) with R the polar rotation"""
    F = rot(3) @ np.diag([1.2, 0.9, 0.7]) @ rot(4).T
    U, sF, Vt = np.linalg.svd(F)
    s, _ = O.logvol_stretch(sF, MU, LAM, LAM)
    R, _ = linalg.polar(F)
    ref = (2 * MU * R + LAM * U @ np.diag(s) @ Vt) / (2 * MU + LAM)
    assert np.abs(O.logvol_map(F, MU, LAM, MU, LAM) - ref).max() < 1e-13


def logvol_scene(**kw):
    sc = copy.copy(scenes.small_beam(5, 2, 2, **kw))
    sc.energy = 2
    return sc


def pd_energy(osc, sc, q, qt, qtil):
    """inertia + dissipation + sum_e V_e (mu_e |F - R|^2 + lam_e/2 |F - P_log|^2 + lam_e/lam_bar phi(s_log)),
    the PD surrogate that the local-global iteration minimises alternately"""
    info = osc.info()
    mu_bar, lam_bar = info["mu_bar"], info["lam_bar"]
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
        sl, _ = O.logvol_stretch(s, mu_bar, lam_bar, lam_bar)
        Pl = U @ np.diag(sl) @ Vt
        V = info["vol"][t]
        E += V * (mu * np.sum((F - R) ** 2) + 0.5 * lam * np.sum((F - Pl) ** 2)
                  + lam / lam_bar * barrier(sl, mu_bar, lam_bar))
        E += 0.5 / h * info["beta"][t] * V * np.sum((F - Ft) ** 2)
    return E


def test_same_system_matrix_as_the_other_energies():
    sc = logvol_scene(seed=3, contrast=30.0)
    a = O.OracleScene(sc).info()
    b = O.OracleScene(sc, energy=0).info()
    assert np.array_equal(a["w"], b["w"]) and np.array_equal(a["beta"], b["beta"])


def test_monotone_energy_plain_iteration():
    sc = logvol_scene(seed=6, contrast=50.0, tip_force=40.0, nu=0.45)
    osc = O.OracleScene(sc, m=0)
    q, v = sc.X.copy(), np.zeros_like(sc.X)
    f = sc.f_ext(3)
    qn, vn, qm1, st = osc.step_forward(q, v, f, force_iters=25, m=0, record=26)
    _, qtil = osc.const_rhs(q, v, f)
    Es = [pd_energy(osc, sc, st["record"][k], q, qtil) for k in range(26)]
    d = np.diff(Es)
    assert np.all(d <= 1e-12 * abs(Es[0])), d
    assert Es[-1] < Es[0]


def test_K_is_db_dq():
    sc = logvol_scene(seed=12, contrast=20.0)
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


def test_gradients_match_central_differences():
    sc = logvol_scene(seed=13, contrast=10.0, tip_force=20.0, alpha=0.2, beta_rel=0.02)
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
        h = 1e-4
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
