"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(closed forms, special cases, brute force, finite differences, textbook
properties) -- never against the oracle itself.  CPU only."""
import copy

import numpy as np
import pytest
from scipy import optimize

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
KB = 2 * MU + LAM


# ------------------------------------------------------------------ SVD
@pytest.mark.parametrize("seed", range(12))
def test_svd3_signed(seed):
    r = rng(seed)
    F = r.standard_normal((3, 3))
    if seed % 3 == 0:
        F = rot(seed) @ np.diag([1.2, 1.2, 0.7]) @ rot(seed + 50).T  # repeated singular value
    if seed % 4 == 1:
        F[:, 2] *= -1.0  # inverted
    U, s, V = O.svd3(F)
    assert np.allclose(U @ U.T, np.eye(3), atol=1e-14) and np.allclose(V @ V.T, np.eye(3), atol=1e-14)
    assert abs(np.linalg.det(U) - 1) < 1e-13 and abs(np.linalg.det(V) - 1) < 1e-13
    assert np.allclose(U @ np.diag(s) @ V.T, F, atol=1e-14 * np.abs(F).max() * 10)
    tol = 1e-14 * abs(s[0])
    assert s[0] >= s[1] - tol and s[1] >= abs(s[2]) - tol
    assert np.sign(s[2]) == np.sign(np.linalg.det(F))
    assert np.allclose(np.abs(s), np.linalg.svd(F, compute_uv=False), rtol=1e-13)


# ------------------------------------------------------------------ energy and stress
def pk1(F, mu, lam):
    """First Piola-Kirchhoff stress as printed in the paper (Eq. pkstress)."""
    Fit = np.linalg.inv(F).T
    return mu * (F - Fit) + lam * np.log(np.linalg.det(F)) * Fit


@pytest.mark.parametrize("seed", range(4))
def test_psi_gradient_is_pk1(seed):
    F = np.eye(3) + 0.2 * rng(seed).standard_normal((3, 3))
    G = np.zeros((3, 3))
    h = 1e-6
    for i in range(3):
        for j in range(3):
            E = np.zeros((3, 3))
            E[i, j] = h
            G[i, j] = (O.psi_nh(F + E, MU, LAM) - O.psi_nh(F - E, MU, LAM)) / (2 * h)
    assert np.allclose(G, pk1(F, MU, LAM), rtol=1e-6, atol=1e-3)
    assert O.psi_nh(np.eye(3), MU, LAM) == 0.0
    assert O.psi_nh(np.diag([1, 1, -1.0]), MU, LAM) == np.inf


# ------------------------------------------------------------------ prox (P5)
@pytest.mark.parametrize("s", [0.3, 0.7, 1.0, 1.25, 2.0])
def test_prox_isotropic_closed_form(s):
    """sigma_F = s 1 gives sigma* = t 1 with k(t - s) + mu(t - 1/t) + 3 lam ln(t)/t = 0."""
    f = lambda t: KB * (t - s) + MU * (t - 1 / t) + 3 * LAM * np.log(t) / t  # noqa: E731
    t = optimize.brentq(f, 1e-3, 10.0, xtol=1e-15, rtol=1e-15)
    out, it = O.prox_stretch(np.array([s, s, s]), MU, LAM, KB)
    assert it >= 0
    assert np.allclose(out, t, rtol=1e-12)


def matrix_prox_bruteforce(F, mu, lam, k):
    """argmin_p k/2 |F - p|^2 + psi(p) over all 3x3 matrices (BFGS, analytic gradient)."""

    def fun(x):
        p = x.reshape(3, 3)
        J = np.linalg.det(p)
        if J <= 0:
            return 1e30, np.zeros(9)
        lj = np.log(J)
        val = 0.5 * k * np.sum((F - p) ** 2) + 0.5 * mu * (np.sum(p * p) - 3) - mu * lj + 0.5 * lam * lj * lj
        grad = k * (p - F) + pk1(p, mu, lam)
        return val / k, grad.ravel() / k

    U, s, Vt = np.linalg.svd(F)
    x0 = (U @ np.diag(np.maximum(s, 0.5)) @ Vt)
    if np.linalg.det(x0) < 0:
        x0 = U @ np.diag([s[0], s[1], 0.3]) @ Vt
    res = optimize.minimize(fun, x0.ravel(), jac=True, method="BFGS", options=dict(gtol=1e-13, maxiter=20000))
    return res.x.reshape(3, 3)


@pytest.mark.parametrize("seed", range(6))
def test_prox_matrix_bruteforce(seed):
    """The SVD reduction of Eq. nh_prox: p* from the oracle equals the
    minimiser over all matrices (brute force)."""
    r = rng(100 + seed)
    F = rot(seed) @ np.diag(np.sort(r.uniform(0.6, 1.5, 3))[::-1]) @ rot(seed + 7).T
    P_or = O.prox_map(F, MU, LAM, KB)
    P_bf = matrix_prox_bruteforce(F, MU, LAM, KB)
    assert np.allclose(P_or, P_bf, atol=2e-8)
    # stationarity of the matrix objective at the oracle's answer
    g = KB * (P_or - F) + pk1(P_or, MU, LAM)
    assert np.abs(g).max() < 1e-6 * KB


def test_prox_inverted_input():
    """det F < 0: the prox lands on det p > 0 and is stationary there."""
    F = rot(3) @ np.diag([1.1, 0.9, -0.2]) @ rot(4).T
    P = O.prox_map(F, MU, LAM, KB)
    assert np.linalg.det(P) > 0
    g = KB * (P - F) + pk1(P, MU, LAM)
    assert np.abs(g).max() < 1e-6 * KB


# ------------------------------------------------------------------ prox differential (P6, P7)
def test_prox_jacobian_at_rest():
    """At F = R (a rotation): rotations pass unchanged, deviatoric symmetric
    strain is scaled by k/(2mu + k) and volumetric strain by k/(2mu + 3lam + k)."""
    for R in (np.eye(3), rot(5)):
        J = O.prox_jacobian(R, MU, LAM, KB, 0.5)
        ap = lambda dF: (J @ dF.ravel()).reshape(3, 3)  # noqa: E731
        W = np.array([[0, 1, 0], [-1, 0, 0], [0, 0, 0.0]])
        S = np.array([[0, 1, 0], [1, 0, 0], [0, 0, 0.0]])
        Dv = np.diag([1.0, -1.0, 0.0])
        I = np.eye(3)
        assert np.allclose(ap(W @ R), W @ R, atol=1e-12)
        assert np.allclose(ap(S @ R), KB / (2 * MU + KB) * S @ R, atol=1e-12)
        assert np.allclose(ap(Dv @ R), KB / (2 * MU + KB) * Dv @ R, atol=1e-12)
        assert np.allclose(ap(I @ R), KB / (2 * MU + 3 * LAM + KB) * R, atol=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_prox_jacobian_fd_and_symmetry(seed):
    r = rng(200 + seed)
    F = rot(seed) @ np.diag([1.3, 1.0, 0.8] + 0.05 * r.standard_normal(3)) @ rot(seed + 11).T
    J = O.prox_jacobian(F, MU, LAM, KB, 0.0)
    h = 1e-6
    Jfd = np.zeros((9, 9))
    for c in range(9):
        E = np.zeros(9)
        E[c] = h
        Jfd[:, c] = (O.prox_map(F + E.reshape(3, 3), MU, LAM, KB) - O.prox_map(F - E.reshape(3, 3), MU, LAM, KB)).ravel() / (2 * h)
    assert np.allclose(J, Jfd, atol=1e-7)
    assert np.allclose(J, J.T, atol=1e-12)
    # at a minimiser the filter is the identity: tau does not matter
    assert np.allclose(O.prox_jacobian(F, MU, LAM, KB, 1.0), J, atol=1e-12)
    assert np.allclose(O.prox_jacobian(F, MU, LAM, KB, 0.5), J, atol=1e-12)


# ------------------------------------------------------------------ TR filter (P8)
def test_tr_filter_special_cases():
    Q = rot(9)
    H = Q @ np.diag([3.0, -2.0, 0.5]) @ Q.T
    Ht0, _ = O.tr_filter(H, 0.0)
    Ht1, _ = O.tr_filter(H, 1.0)
    Hth, Dh = O.tr_filter(H, 0.5, k=7.0)
    assert np.allclose(Ht0, H, atol=1e-13)
    assert np.allclose(Ht1, Q @ np.diag([3.0, 2.0, 0.5]) @ Q.T, atol=1e-13)
    assert np.allclose(Hth, Q @ np.diag([3.0, 0.0, 0.5]) @ Q.T, atol=1e-13)  # eigenvalue clamping
    assert np.allclose(Dh, 7.0 * np.linalg.pinv(Q @ np.diag([3.0, 0.0, 0.5]) @ Q.T), atol=1e-12)
    P = Q @ np.diag([3.0, 2.0, 0.5]) @ Q.T
    for tau in (0.0, 0.25, 0.5, 1.0):
        assert np.allclose(O.tr_filter(P, tau)[0], P, atol=1e-13)


# ------------------------------------------------------------------ Anderson (P9)
def test_aa_affine_gmres_property():
    n = 4
    r = rng(5)
    M = r.standard_normal((n, n))
    M = 0.9 * M / np.abs(np.linalg.eigvals(M)).max()
    c = r.standard_normal(n)
    xs = np.linalg.solve(np.eye(n) - M, c)
    H = O.AAHistory(n, 5)
    x = np.zeros(n)
    errs = []
    for k in range(n + 3):
        x, reset, _ = H.step(x, M @ x + c)
        assert not reset
        errs.append(np.linalg.norm(x - xs) / np.linalg.norm(xs))
    assert errs[n + 1] < 1e-6, errs
    # m = 0 is the plain fixed-point iteration
    H0 = O.AAHistory(n, 0)
    x0 = np.zeros(n)
    y0 = np.zeros(n)
    for k in range(5):
        x0, _, _ = H0.step(x0, M @ x0 + c)
        y0 = M @ y0 + c
    assert np.array_equal(x0, y0)


def test_aa_reliability_guard():
    """Near-stagnant map: |gamma| > 10 drops the history and takes the plain step."""
    c = np.array([1.0, 2.0, -1.0])
    T = lambda x: 0.999 * x + c  # noqa: E731
    H = O.AAHistory(3, 1)
    x = np.zeros(3)
    x1, r1, _ = H.step(x, T(x))
    assert not r1 and np.array_equal(x1, T(x))
    x2, r2, _ = H.step(x1, T(x1))
    assert r2 and np.array_equal(x2, T(x1))
    assert H.hn.value == 0


# ------------------------------------------------------------------ system matrix and factor (P10)
def small():
    return scenes.small_beam(5, 2, 2, seed=4, contrast=20.0)


def dense_A(osc):
    n = osc.nv
    free = ~osc.pinned
    cols = []
    idx = [(v, a) for v in range(n) if free[v] for a in range(3)]
    for (v, a) in idx:
        e = np.zeros((n, 3))
        e[v, a] = 1.0
        y = osc.apply_A(e)
        cols.append(np.array([y[w, b] for (w, b) in idx]))
    return np.array(cols).T, idx


def test_system_matrix_properties():
    sc = small()
    osc = O.OracleScene(sc)
    info = osc.info()
    A, idx = dense_A(osc)
    assert np.allclose(A, A.T, rtol=0, atol=1e-9 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0
    # total lumped mass = rho * volume of the box
    ext = sc.X.max(axis=0) - sc.X.min(axis=0)
    assert np.isclose(info["mass"].sum(), sc.rho * np.prod(ext), rtol=1e-13)
    # translations are free of elastic stiffness: with every vertex displaced
    # by the same vector, A_ff 1 + A_fp 1 = (1 + alpha h) M / h^2 on free rows
    d = np.array([0.3, -0.2, 0.5])
    x = np.broadcast_to(d, sc.X.shape).copy()
    c_free, _ = osc.const_rhs(sc.X, np.zeros_like(sc.X))  # at rest: the pinned coupling only
    # a uniform dilation q = (1 + e) X gives sum_e w_e V_e |G q|^2 = 3 (1 + e)^2 sum_e w_e V_e
    e = 0.01
    q = (1 + e) * sc.X
    Gq2 = 0.0
    tets = sc.tets
    for t in range(sc.n_e):
        Xs = sc.X[tets[t]]
        Dm = (Xs[1:] - Xs[0]).T
        Ds = (q[tets[t]][1:] - q[tets[t]][0]).T
        F = Ds @ np.linalg.inv(Dm)
        Gq2 += info["w"][t] * info["vol"][t] * np.sum(F * F)
    assert np.isclose(Gq2, 3 * (1 + e) ** 2 * np.sum(info["w"] * info["vol"]), rtol=1e-12)
    h = sc.h
    free = ~osc.pinned
    Ax = osc.apply_A(x)  # free-free part
    # the free-pinned part of A applied to the constant field: -(pinned coupling at X shifted)
    # equals (c at q_t = X + d shifted rigidly) - (c at X); use linearity of the pinned term
    m = info["mass"]
    target = (1 + sc.alpha * h) * m[free, None] / h ** 2 * d
    # A_fp 1 d from the elementwise stiffness: assemble directly with the oracle's element data
    Afp = np.zeros_like(sc.X)
    for t in range(sc.n_e):
        Xs = sc.X[tets[t]]
        Bi = np.linalg.inv((Xs[1:] - Xs[0]).T)
        Bh = np.vstack([-Bi.sum(axis=0), Bi])
        K = (info["w"][t] + info["beta"][t] / h) * info["vol"][t] * (Bh @ Bh.T)
        for a in range(4):
            for b in range(4):
                if free[tets[t][a]] and not free[tets[t][b]]:
                    Afp[tets[t][a]] += K[a, b] * d
    assert np.allclose(Ax[free] + Afp[free], target, rtol=1e-10, atol=1e-8 * np.abs(target).max())
    _ = c_free


def test_factor_solve_matches_dense():
    sc = small()
    osc = O.OracleScene(sc)
    A, idx = dense_A(osc)
    r = rng(8).standard_normal(sc.X.shape)
    x = osc.apply_Ainv(r)
    rv = np.array([r[v, a] for (v, a) in idx])
    xv = np.linalg.solve(A, rv)
    assert np.allclose(np.array([x[v, a] for (v, a) in idx]), xv, rtol=1e-12, atol=1e-14 * np.abs(xv).max())


# ------------------------------------------------------------------ local-step Jacobian K
def test_K_symmetric_and_fd():
    sc = small()
    osc = O.OracleScene(sc)
    r = rng(12)
    q = sc.X + 2e-3 * r.standard_normal(sc.X.shape)
    q[sc.pinned.astype(bool)] = sc.X[sc.pinned.astype(bool)]
    x, y = r.standard_normal(sc.X.shape), r.standard_normal(sc.X.shape)
    free = ~sc.pinned.astype(bool)
    x[~free] = 0
    y[~free] = 0
    Kx, Ky = osc.apply_K(q, 1.0, x), osc.apply_K(q, 1.0, y)
    assert np.isclose(np.sum(y * Kx), np.sum(x * Ky), rtol=1e-11)
    h = 1e-7
    fd = (osc.local_rhs(q + h * x) - osc.local_rhs(q - h * x)) / (2 * h)
    assert np.allclose(Kx[free], fd[free], rtol=1e-5, atol=1e-6 * np.abs(Kx).max())


# ------------------------------------------------------------------ forward (P1, P2, P3, P12)
def test_rest_state_zero_force():
    sc = scenes.small_beam(6, 3, 3, seed=2, tip_force=0.0, gravity=(0.0, 0.0, 0.0))
    osc = O.OracleScene(sc)
    qn, vn, qm1, st = osc.step_forward(sc.X, np.zeros_like(sc.X), record=4)
    assert st["iters"] == 2 and st["status"] == 0
    assert np.abs(qn - sc.X).max() < 1e-14
    for k in range(3):
        assert np.abs(st["record"][k] - sc.X).max() < 1e-14
    # b(X) + c = A X on the free rows (zero elastic force at rest)
    c, _ = osc.const_rhs(sc.X, np.zeros_like(sc.X))
    b = osc.local_rhs(sc.X) + c
    AX = osc.apply_A(sc.X)
    free = ~sc.pinned.astype(bool)
    assert np.abs(AX[free] - b[free]).max() <= 1e-14 * np.abs(b[free]).max()


def surrogate_energy(osc, sc, q, qt, qtil):
    """E(q) = min_p L(q, p): inertia + dissipation + sum_e V_e [w_e/2 |G q - p*|^2 + psi_e(p*)]."""
    info = osc.info()
    h = sc.h
    m = info["mass"]
    free = ~sc.pinned.astype(bool)
    E = 0.5 / h ** 2 * np.sum(m[:, None] * (q - qtil) ** 2 * free[:, None])
    E += 0.5 / h * sc.alpha * np.sum(m[:, None] * (q - qt) ** 2 * free[:, None])
    mub, lamb, kb = info["mu_bar"], info["lam_bar"], info["k_bar"]
    nu = sc.nu
    for t in range(sc.n_e):
        Xs = sc.X[sc.tets[t]]
        Bi = np.linalg.inv((Xs[1:] - Xs[0]).T)
        F = (q[sc.tets[t]][1:] - q[sc.tets[t]][0]).T @ Bi
        Ft = (qt[sc.tets[t]][1:] - qt[sc.tets[t]][0]).T @ Bi
        P = O.prox_map(F, mub, lamb, kb)
        Ee = np.exp(sc.log_E[t])
        mu, lam = Ee / (2 * (1 + nu)), Ee * nu / ((1 + nu) * (1 - 2 * nu))
        w, V = info["w"][t], info["vol"][t]
        E += V * (0.5 * w * np.sum((F - P) ** 2) + O.psi_nh(P, mu, lam))
        E += 0.5 / h * info["beta"][t] * V * np.sum((F - Ft) ** 2)
    return E


def test_monotone_energy_plain_iteration():
    sc = scenes.small_beam(5, 2, 2, seed=6, contrast=50.0, tip_force=40.0, nu=0.45)
    osc = O.OracleScene(sc, m=0)
    q, v = sc.X.copy(), np.zeros_like(sc.X)
    f = sc.f_ext(3)
    qn, vn, qm1, st = osc.step_forward(q, v, f, force_iters=25, m=0, record=26)
    _, qtil = osc.const_rhs(q, v, f)
    Es = [surrogate_energy(osc, sc, st["record"][k], q, qtil) for k in range(26)]
    d = np.diff(Es)
    assert np.all(d <= 1e-12 * abs(Es[0])), d
    assert Es[-1] < Es[0]


def test_newton_agreement_tiny_mesh():
    """PD + AA reaches the root of r(q) = A q - b(q) - c found by Newton with a
    finite-difference Jacobian."""
    sc = scenes.small_beam(1, 1, 1, seed=3, contrast=1.0, tip_force=0.0, gravity=(0.0, 0.0, -9.81), h=0.02,
                           aa_window=5)
    sc = copy.copy(sc)
    sc.gravity = np.array([0.0, 0.0, -400.0])
    osc = O.OracleScene(sc, eps_rel=1e-15, eps_abs=1e-15)
    q_t, v_t = sc.X.copy(), np.zeros_like(sc.X)
    qn, vn, qm1, st = osc.step_forward(q_t, v_t)
    assert np.abs(qn - sc.X).max() > 1e-4
    c, _ = osc.const_rhs(q_t, v_t)
    free = ~sc.pinned.astype(bool)
    idx = [(v, a) for v in range(sc.n_v) if free[v] for a in range(3)]

    def res(x):
        q = q_t.copy()
        for i, (v, a) in enumerate(idx):
            q[v, a] = x[i]
        r = osc.apply_A(q) - osc.local_rhs(q) - c
        # apply_A covers the free block only; the pinned coupling sits in c
        return np.array([r[v, a] for (v, a) in idx])

    x = np.array([q_t[v, a] for (v, a) in idx])
    for it in range(30):
        r = res(x)
        if np.abs(r).max() < 1e-9:
            break
        J = np.zeros((len(x), len(x)))
        for j in range(len(x)):
            e = np.zeros(len(x))
            e[j] = 1e-7
            J[:, j] = (res(x + e) - res(x - e)) / 2e-7
        x = x - np.linalg.solve(J, r)
    qN = q_t.copy()
    for i, (v, a) in enumerate(idx):
        qN[v, a] = x[i]
    assert np.abs(qN - qn).max() < 1e-10 * np.abs(qn - q_t).max() * 1e3


def test_damping_residual():
    """At the converged q*, implicit Euler with the explicit Rayleigh force
    f_d = -(alpha M + B_beta)(q* - q_t)/h and the projected elastic force holds."""
    sc = scenes.small_beam(5, 2, 2, seed=9, contrast=10.0, alpha=0.5, beta_rel=0.05)
    osc = O.OracleScene(sc, eps_rel=1e-14, eps_abs=1e-15)
    info = osc.info()
    q_t = sc.X + 1e-3 * rng(3).standard_normal(sc.X.shape)
    q_t[sc.pinned.astype(bool)] = sc.X[sc.pinned.astype(bool)]
    v_t = 0.1 * rng(4).standard_normal(sc.X.shape)
    f = sc.f_ext(1)
    qs, vs, _, st = osc.step_forward(q_t, v_t, f)
    h = sc.h
    m = info["mass"][:, None]
    qtil = q_t + h * v_t + h * h * (f / m + sc.gravity)
    # elastic PD force and B_beta (q* - q_t), assembled here element by element
    fel = np.zeros_like(q_t)
    Bd = np.zeros_like(q_t)
    for t in range(sc.n_e):
        T = sc.tets[t]
        Bi = np.linalg.inv((sc.X[T][1:] - sc.X[T][0]).T)
        Bh = np.vstack([-Bi.sum(axis=0), Bi])
        F = (qs[T][1:] - qs[T][0]).T @ Bi
        P = O.prox_map(F, info["mu_bar"], info["lam_bar"], info["k_bar"])
        fel[T] -= info["w"][t] * info["vol"][t] * (Bh @ (F - P).T)
        Fd = (qs[T][1:] - qs[T][0] - (q_t[T][1:] - q_t[T][0])).T @ Bi
        Bd[T] += info["beta"][t] * info["vol"][t] * (Bh @ Fd.T)
    resid = m / h ** 2 * (qs - qtil) - fel + (sc.alpha * m * (qs - q_t) + Bd) / h
    free = ~sc.pinned.astype(bool)
    scale = np.abs(m / h ** 2 * (qs - qtil)).max()
    assert np.abs(resid[free]).max() < 1e-7 * scale


# ------------------------------------------------------------------ backward (P11)
def test_adjoint_iteration_matches_dense():
    sc = small()
    osc = O.OracleScene(sc, eps_adj=1e-13)
    q, v, ck, _ = O.rollout(osc, 2)
    r = rng(21)
    gq, gv = r.standard_normal(q.shape), r.standard_normal(q.shape)
    (q_t, v_t, f, qs, qsm1) = ck[-1]
    a = osc.step_backward(q_t, v_t, f, qs, qsm1, gq, gv, adj_mode=0)
    b = osc.step_backward(q_t, v_t, f, qs, qsm1, gq, gv, adj_mode=1)
    for x, y in zip(a[:4], b[:4]):
        assert np.allclose(x, y, rtol=1e-9, atol=1e-11 * np.abs(y).max())


def test_tr_ratio_matches_primal_objective():
    sc = small()
    osc = O.OracleScene(sc)
    q, v, ck, _ = O.rollout(osc, 2)
    (q_t, v_t, f, qs, qsm1) = ck[-1]
    _, qtil = osc.const_rhs(q_t, v_t, f)
    st = osc.step_backward(q_t, v_t, f, qs, qsm1, np.ones_like(q), np.zeros_like(q))[4]
    act = osc.phi(qsm1, qtil) - osc.phi(qs, qtil)
    assert np.isclose(st["dphi_act"], act, rtol=1e-6, atol=1e-12 * abs(osc.phi(qs, qtil)))
    dq = (qs - qsm1) * (~sc.pinned.astype(bool))[:, None]
    assert np.isclose(st["dphi_mod"], 0.5 * abs(np.sum(dq * osc.apply_A(dq))), rtol=1e-12)
    rho = 1.0 if st["dphi_mod"] < 1e-12 else st["dphi_act"] / st["dphi_mod"]
    assert st["tau"] == (0.5 if abs(rho - 1) <= 0.1 else 1.0)


def rollout_loss(sc, logE, q0, v0, fscale, steps, frozen):
    osc = O.OracleScene(sc, log_E=logE, eps_rel=1e-14, eps_abs=1e-16, frozen=frozen, eps_adj=1e-14)
    q, v = q0.copy(), v0.copy()
    ck = []
    for t in range(steps):
        f = fscale * sc.f_ext(t)
        qn, vn, qm1, st = osc.step_forward(q, v, f)
        ck.append((q, v, f, qn, qm1))
        q, v = qn, vn
    L, gq = scenes.centroid_loss(q, sc.target_centroid)
    L += 0.5 * float(np.sum(v * v)) * 1e-3
    gv = 1e-3 * v
    return L, gq, gv, ck, osc


def test_gradients_match_central_differences():
    sc = scenes.small_beam(4, 2, 2, seed=13, contrast=10.0, tip_force=20.0, alpha=0.2, beta_rel=0.02)
    base = O.OracleScene(sc).info()
    frozen = (base["mu_bar"], base["lam_bar"], base["mu_ref"])
    steps = 3
    q0 = sc.X + 1e-3 * rng(1).standard_normal(sc.X.shape)
    q0[sc.pinned.astype(bool)] = sc.X[sc.pinned.astype(bool)]
    v0 = 0.05 * rng(2).standard_normal(sc.X.shape)
    v0[sc.pinned.astype(bool)] = 0
    L, gq, gv, ck, osc = rollout_loss(sc, sc.log_E, q0, v0, 1.0, steps, frozen)
    gl = np.zeros(sc.n_e)
    for (q_t, v_t, f, qs, qsm1) in reversed(ck):
        gq, gv, gf, gl, st = osc.step_backward(q_t, v_t, f, qs, qsm1, gq, gv, gl, adj_mode=1)
    # log E of three tets
    for e in rng(3).choice(sc.n_e, 3, replace=False):
        h = 1e-5
        lp, lm = sc.log_E.copy(), sc.log_E.copy()
        lp[e] += h
        lm[e] -= h
        fd = (rollout_loss(sc, lp, q0, v0, 1.0, steps, frozen)[0] -
              rollout_loss(sc, lm, q0, v0, 1.0, steps, frozen)[0]) / (2 * h)
        assert np.isclose(gl[e], fd, rtol=2e-5, atol=1e-9 * abs(L)), (e, gl[e], fd)
    # initial position and velocity of two free vertices
    free = np.where(~sc.pinned.astype(bool))[0]
    for (vtx, ax) in [(free[3], 1), (free[-1], 2)]:
        h = 1e-6
        for which, g in ((0, gq), (1, gv)):
            xp = [q0.copy(), v0.copy()]
            xm = [q0.copy(), v0.copy()]
            xp[which][vtx, ax] += h
            xm[which][vtx, ax] -= h
            fd = (rollout_loss(sc, sc.log_E, xp[0], xp[1], 1.0, steps, frozen)[0] -
                  rollout_loss(sc, sc.log_E, xm[0], xm[1], 1.0, steps, frozen)[0]) / (2 * h)
            assert np.isclose(g[vtx, ax], fd, rtol=1e-4, atol=1e-8 * abs(L)), (which, g[vtx, ax], fd)


def test_force_gradient_central_difference():
    sc = scenes.small_beam(4, 2, 2, seed=17, contrast=5.0, tip_force=10.0)
    base = O.OracleScene(sc).info()
    frozen = (base["mu_bar"], base["lam_bar"], base["mu_ref"])
    L, gq, gv, ck, osc = rollout_loss(sc, sc.log_E, sc.X, np.zeros_like(sc.X), 1.0, 1, frozen)
    (q_t, v_t, f, qs, qsm1) = ck[0]
    _, _, gf, _, _ = osc.step_backward(q_t, v_t, f, qs, qsm1, gq, gv, adj_mode=1)
    # dL/d(scale of the force field) = <dL/df, f>
    h = 1e-6
    fd = (rollout_loss(sc, sc.log_E, sc.X, np.zeros_like(sc.X), 1 + h, 1, frozen)[0] -
          rollout_loss(sc, sc.log_E, sc.X, np.zeros_like(sc.X), 1 - h, 1, frozen)[0]) / (2 * h)
    assert np.isclose(np.sum(gf * f), fd, rtol=1e-5)


# ------------------------------------------------------------------ material setup (row a1)
def _stretch_hessian_diag_at_rest(mu, lam, eps=1e-4):
    """Diagonal of the Neo-Hookean stretch Hessian at sigma = (1, 1, 1), by
    second differences of the energy of Sec. 3.2 Eq. neohookean (pinned to
    its stress by test_psi_gradient_is_pk1): the rest tangent modulus that
    Eq. pd_weight asks the PD weight to match."""
    d = []
    for i in range(3):
        ep, em = np.ones(3), np.ones(3)
        ep[i] += eps
        em[i] -= eps
        d.append((O.psi_nh(np.diag(ep), mu, lam) - 2 * O.psi_nh(np.eye(3), mu, lam)
                  + O.psi_nh(np.diag(em), mu, lam)) / eps ** 2)
    return np.array(d)


@pytest.mark.parametrize("make", [lambda: scenes.small_beam(5, 2, 2, seed=4, contrast=20.0),
                                  lambda: scenes.small_beam(4, 3, 2, seed=9, contrast=100.0, nu=0.49)])
def test_material_setup_from_E_and_nu(make):
    """Sec. 3.1 Eq. lame gives mu_e, lam_e from E_e and nu; the PD weight is
    the rest tangent modulus (the stretch Hessian's diagonal at sigma = 1,
    Sec. 4.1/7.2), the local prox uses the element means and k_bar is the
    same modulus of the mean energy (Sec. 4.2); Rayleigh's beta_e scales with
    mu_e relative to the stiffest element (Sec. 4.5 Eq. rayleigh).  Every
    quantity is recomputed here from E, nu and the rest shape and compared
    with what the oracle set up."""
    sc = make()
    sc = copy.copy(sc)
    sc.beta0 = 3.0e2  # nonzero so beta_e is exercised
    osc = O.OracleScene(sc)
    info = osc.info()
    E = np.exp(sc.log_E)
    nu = sc.nu
    mu = E / (2 * (1 + nu))
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    # w_e: the stretch Hessian's diagonal at rest, per element (all three entries equal)
    w = np.array([_stretch_hessian_diag_at_rest(m_, l_) for (m_, l_) in zip(mu, lam)])
    assert np.allclose(w, w[:, :1], rtol=1e-6)
    assert np.allclose(info["w"], w[:, 0], rtol=1e-6)
    mu_bar, lam_bar = mu.mean(), lam.mean()
    k_bar = _stretch_hessian_diag_at_rest(mu_bar, lam_bar)[0]
    assert np.isclose(info["mu_bar"], mu_bar, rtol=1e-13)
    assert np.isclose(info["lam_bar"], lam_bar, rtol=1e-13)
    assert np.isclose(info["k_bar"], k_bar, rtol=1e-6)
    mu_ref = mu.max()
    assert np.isclose(info["mu_ref"], mu_ref, rtol=1e-15)
    assert np.allclose(info["beta"], sc.beta0 * mu / mu_ref, rtol=1e-13)
    # rest volumes and lumped masses
    Xt = sc.X[sc.tets]
    vol = np.abs(np.linalg.det(np.transpose(Xt[:, 1:] - Xt[:, :1], (0, 2, 1)))) / 6
    assert np.allclose(info["vol"], vol, rtol=1e-12)
    mass = np.zeros(sc.n_v)
    np.add.at(mass, sc.tets.ravel(), np.repeat(sc.rho * vol / 4, 4))
    assert np.allclose(info["mass"], mass, rtol=1e-12)


@pytest.mark.parametrize("kind", ["deviatoric", "shear", "volumetric", "rotation"])
def test_scene_prox_jacobian_at_rest_uses_mesh_means(kind):
    """Behavioural pin of k_bar: at rest every element's prox differential
    (Sec. 4.4 Eq. tr_ift at F = I) passes an infinitesimal rotation unchanged
    and scales deviatoric strain by k/(2 mu_bar + k) and volumetric strain by
    k/(2 mu_bar + 3 lam_bar + k), k = 2 mu_bar + lam_bar with the means
    computed here from E and nu.  On a mesh without pinned vertices and
    without damping, K x for an affine field x = A X is that factor times
    (A~ - M/h^2) x = sum_e w_e V_e G_e^T A."""
    sc = copy.copy(scenes.small_beam(4, 2, 2, seed=11, contrast=30.0, nu=0.45))
    sc.pinned = np.zeros_like(sc.pinned)
    sc.alpha, sc.beta0 = 0.0, 0.0
    osc = O.OracleScene(sc)
    E = np.exp(sc.log_E)
    mu_bar = (E / (2 * (1 + sc.nu))).mean()
    lam_bar = (E * sc.nu / ((1 + sc.nu) * (1 - 2 * sc.nu))).mean()
    k = 2 * mu_bar + lam_bar
    A = {"deviatoric": np.diag([1.0, -0.4, -0.6]), "shear": np.array([[0, 1, 0], [1, 0, 0.5], [0, 0.5, 0.0]]),
         "volumetric": np.eye(3), "rotation": np.array([[0, 1, -0.3], [-1, 0, 0.2], [0.3, -0.2, 0.0]])}[kind]
    fac = {"deviatoric": k / (2 * mu_bar + k), "shear": k / (2 * mu_bar + k),
           "volumetric": k / (2 * mu_bar + 3 * lam_bar + k), "rotation": 1.0}[kind]
    x = sc.X @ A.T
    Kx = osc.apply_K(sc.X, 1.0, x)
    m = osc.info()["mass"]
    elastic = osc.apply_A(x) - m[:, None] / sc.h ** 2 * x
    assert np.allclose(Kx, fac * elastic, rtol=0, atol=1e-10 * np.abs(elastic).max())


def test_thread_count_does_not_change_results():
    """The oracle's element loops run on several threads but add their
    contributions in a fixed (element) order, so one thread and four threads
    give bitwise the same forward step, backward step and gradients."""
    sc = scenes.small_beam(6, 3, 2, seed=21, contrast=30.0, tip_force=10.0)
    out = []
    n0 = O.get_threads()
    try:
        for n in (1, 4):
            O.set_threads(n)
            osc = O.OracleScene(sc, eps_adj=1e-10)
            qn, vn, qm1, st = osc.step_forward(sc.X, np.zeros_like(sc.X), sc.f_ext(2))
            gq = rng(5).standard_normal(sc.X.shape)
            res = osc.step_backward(sc.X, np.zeros_like(sc.X), sc.f_ext(2), qn, qm1, gq, 0 * gq, adj_mode=0)
            out.append([qn, qm1, *res[:4], osc.phi(qn, sc.X)])
    finally:
        O.set_threads(n0)
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
