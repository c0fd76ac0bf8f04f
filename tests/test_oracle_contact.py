"""Pins of the oracle's contact step (Sec. 4.7, frictionless reading) against
facts fixed by mathematics: brute-force enumeration of the complementarity
problem, the Delassus operator from a dense inverse, the contact KKT
conditions at a converged step, bitwise equality with the contact-free step
when no row activates, agreement of the two adjoint solvers, and central
finite differences through contact steps.  CPU only."""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_2605_14526_amd import scenes


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def lcp_bruteforce(W, d):
    """The unique solution of delta = d + W lam >= 0, lam >= 0, lam.delta = 0 (W SPD) by enumerating
    every active set."""
    K = len(d)
    sols = []
    for mask in itertools.product([0, 1], repeat=K):
        A = [i for i in range(K) if mask[i]]
        lam = np.zeros(K)
        if A:
            lam[A] = np.linalg.solve(W[np.ix_(A, A)], -d[A])
        delta = d + W @ lam
        if (lam >= -1e-12).all() and (delta >= -1e-12).all():
            sols.append(lam)
    assert len(sols) >= 1
    return sols[0]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_fb_newton_matches_enumeration(seed):
    r = rng(seed)
    K = 7
    B = r.standard_normal((K, K))
    W = B @ B.T + 0.1 * np.eye(K)
    d = r.standard_normal(K)
    lam, it, res = O.fb_lcp(W, d)
    ref = lcp_bruteforce(W, d)
    assert np.allclose(lam, ref, rtol=1e-10, atol=1e-12)
    assert res <= 1e-12 and it <= 30


def test_fb_newton_special_cases():
    W = np.diag([2.0, 3.0, 0.5])
    # all separated: lam = 0; all penetrating: lam = -d / W_cc
    lam, _, _ = O.fb_lcp(W, np.array([1.0, 0.1, 2.0]))
    assert np.array_equal(lam, np.zeros(3))
    d = np.array([-1.0, -0.3, -0.2])
    lam, _, _ = O.fb_lcp(W, d)
    assert np.allclose(lam, -d / np.diag(W), rtol=1e-13)


def tiny_drop(res=4, **kw):
    return scenes.drop_blob(res=res, **kw)


def test_delassus_equals_dense_inverse():
    sc = tiny_drop()
    osc = O.OracleScene(sc)
    nv = sc.n_v
    # dense A~ from its action on unit vectors of axis 0 (A is the same on every axis)
    A = np.zeros((nv, nv))
    for j in range(nv):
        e = np.zeros((nv, 3))
        e[j, 0] = 1.0
        A[:, j] = osc.apply_A(e)[:, 0]
    Ainv = np.linalg.inv(A)
    r = rng(5)
    cv = np.sort(r.choice(nv, 6, replace=False)).astype(np.int32)
    cv[1] = cv[0]  # two rows on one vertex
    cn = r.standard_normal((6, 3))
    cn /= np.linalg.norm(cn, axis=1)[:, None]
    W = O.contact_W(osc, cv, cn)
    ref = (cn @ cn.T) * Ainv[np.ix_(cv, cv)]
    assert np.allclose(W, ref, rtol=1e-11, atol=1e-14 * np.abs(ref).max())
    assert np.allclose(W, W.T, rtol=1e-12, atol=1e-16 * np.abs(W).max())
    assert np.linalg.eigvalsh(0.5 * (W + W.T)).min() > 0


def test_detection_rules():
    sc = tiny_drop()
    obs = {"planes": [((0.0, 0.0, 1.0), 0.0)], "boxes": [((0.0, 0.0, -1.0), (1.0, 1.0, 0.2))], "d_c": 0.05}
    q = np.array([[2.0, 2.0, 0.01],    # near the plane only
                  [0.5, 0.5, 0.23],     # above the box top, within d_c
                  [0.5, 0.5, 0.40],     # far from both
                  [1.02, 0.5, 0.1],     # beside the box (+x face) and within d_c of the plane? no: z = 0.1
                  [2.0, 2.0, 0.5]])     # far, but the inertial prediction crosses the plane
    v = np.zeros_like(q)
    v[4, 2] = -300.0
    pinned = np.zeros(5, np.uint8)
    cv, cn, cg = O.detect_contacts(q, v, 0.002, pinned, obs)
    assert list(cv) == [0, 1, 3, 4]
    assert np.allclose(cn[0], [0, 0, 1]) and cg[0] == 0.0
    assert np.allclose(cn[1], [0, 0, 1]) and cg[1] == 0.2
    assert np.allclose(cn[2], [1, 0, 0]) and cg[2] == 1.0
    assert np.allclose(cn[3], [0, 0, 1]) and cg[3] == 0.0
    pinned[0] = 1
    cv2, _, _ = O.detect_contacts(q, v, 0.002, pinned, obs)
    assert list(cv2) == [1, 3, 4]


def test_inactive_rows_are_bitwise_contact_free():
    sc = scenes.small_beam(4, 2, 2, seed=21, contrast=30.0, tip_force=10.0)
    osc = O.OracleScene(sc)
    q, v = sc.q0(), sc.v0()
    for t in range(3):
        f = sc.f_ext(t)
        qa, va, qma, sta = osc.step_forward(q, v, f)
        # rows on every free vertex against a plane far below: candidates that never activate
        free = np.where(sc.pinned == 0)[0].astype(np.int32)
        con = (free, np.tile([0.0, 0.0, 1.0], (len(free), 1)), np.full(len(free), -10.0))
        qb, vb, qmb, lam, stb = O.step_forward_contact(osc, q, v, f, con)
        assert np.array_equal(qa, qb) and np.array_equal(va, vb) and np.array_equal(qma, qmb)
        assert sta["iters"] == stb["iters"] and not lam.any()
        q, v = qa, va


def contact_window(res=4, before=1):
    """State of the tiny drop ``before`` steps ahead of its first step with an active contact."""
    sc = tiny_drop(res)
    osc = O.OracleScene(sc)
    q, v = sc.q0(), sc.v0()
    hist = []
    for t in range(200):
        hist.append((q, v))
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        q, v, _, lam, _ = O.step_forward_contact(osc, q, v, sc.f_ext(t), con)
        if (lam > 0).any():
            q, v = hist[max(0, t - before)]
            return sc, q, v
    raise AssertionError("the drop never lands")


def test_contact_step_kkt():
    sc, q, v = contact_window()
    osc = O.OracleScene(sc, eps_rel=1e-13, eps_abs=1e-16)
    n_act = 0
    for t in range(4):
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        f = sc.f_ext(t)
        qn, vn, qm1, lam, st = O.step_forward_contact(osc, q, v, f, con, fb_tol=1e-14)
        assert st["status"] == 0
        cv, cn, cg = con
        n_act += int((lam > 0).sum())
        # stationarity: A q - c - b_local(q) - J^T lam = 0
        c, _ = osc.const_rhs(q, v, f)
        res = osc.apply_A(qn) - c - osc.local_rhs(qn)
        for k in range(len(cv)):
            res[cv[k]] -= lam[k] * cn[k]
        scale = np.abs(osc.apply_A(qn)).max()
        assert np.abs(res).max() <= 1e-9 * scale
        # complementarity
        delta = (cn * qn[cv]).sum(axis=1) - cg
        assert (lam >= 0).all() and (delta >= -1e-10).all()
        assert np.abs(lam * delta).max() <= 1e-10 * max(1.0, lam.max())
        q, v = qn, vn
    assert n_act > 0


def test_contact_adjoint_dense_matches_fixed_point():
    sc, q, v = contact_window()
    osc = O.OracleScene(sc, eps_rel=1e-12, eps_abs=1e-16, eps_adj=1e-13)
    g = rng(9).standard_normal(q.shape)
    for t in range(3):
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        f = sc.f_ext(t)
        qn, vn, qm1, lam, st = O.step_forward_contact(osc, q, v, f, con)
        if (lam > 0).any():
            a = O.step_backward_contact(osc, q, v, f, qn, qm1, g, 0.1 * g, con, lam, adj_mode=1)
            b = O.step_backward_contact(osc, q, v, f, qn, qm1, g, 0.1 * g, con, lam, adj_mode=0)
            for x, y in zip(a[:4], b[:4]):
                assert np.allclose(x, y, rtol=1e-9, atol=1e-11 * np.abs(x).max())
            return
        q, v = qn, vn
    pytest.fail("no active contact in the window")


def contact_loss(sc, logE, q0, v0, cons, frozen):
    osc = O.OracleScene(sc, log_E=logE, eps_rel=1e-14, eps_abs=1e-16, frozen=frozen, eps_adj=1e-14)
    q, v = q0.copy(), v0.copy()
    ck = []
    for t, con in enumerate(cons):
        f = sc.f_ext(t)
        qn, vn, qm1, lam, st = O.step_forward_contact(osc, q, v, f, con, fb_tol=1e-15)
        ck.append((q, v, f, qn, qm1, con, lam))
        q, v = qn, vn
    L, gq = scenes.centroid_loss(q, sc.target_centroid)
    w = np.linspace(0.5, 1.5, q.shape[0])[:, None]
    L += float(np.sum(w * q * q)) + 1e-3 * float(np.sum(v * v))
    gq = gq + 2.0 * w * q
    gv = 2e-3 * v
    return L, gq, gv, ck, osc


def test_contact_gradients_match_central_differences():
    """Through four steps with active contacts (rows fixed to those of the unperturbed rollout, active sets
    unchanged by the perturbations), the adjoint gradients equal central differences."""
    sc, q0, v0 = contact_window(before=2)
    base = O.OracleScene(sc).info()
    frozen = (base["mu_bar"], base["lam_bar"], base["mu_ref"])
    steps = 4
    # rows detected on the unperturbed rollout, then held fixed
    osc = O.OracleScene(sc, eps_rel=1e-14, eps_abs=1e-16, frozen=frozen)
    cons, q, v = [], q0.copy(), v0.copy()
    for t in range(steps):
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        cons.append(con)
        q, v, _, _, _ = O.step_forward_contact(osc, q, v, sc.f_ext(t), con)
    L, gq, gv, ck, osc = contact_loss(sc, sc.log_E, q0, v0, cons, frozen)
    assert sum(int((c[6] > 0).sum()) for c in ck) > 0
    act = [c[6] > 0 for c in ck]
    gl = np.zeros(sc.n_e)
    for (q_t, v_t, f, qs, qsm1, con, lam) in reversed(ck):
        gq, gv, gf, gl, st = O.step_backward_contact(osc, q_t, v_t, f, qs, qsm1, gq, gv, con, lam, gl, adj_mode=1)
    # steps: the converged forward carries a noise of ~1e-14 relative, so central differences need a step
    # well above it; their O(h^2) truncation stays below the tolerance
    for e in rng(3).choice(sc.n_e, 3, replace=False):
        h = 1e-3
        lp, lm = sc.log_E.copy(), sc.log_E.copy()
        lp[e] += h
        lm[e] -= h
        Lp, _, _, ckp, _ = contact_loss(sc, lp, q0, v0, cons, frozen)
        Lm, _, _, ckm, _ = contact_loss(sc, lm, q0, v0, cons, frozen)
        assert all(np.array_equal(a, c[6] > 0) for a, c in zip(act, ckp))
        assert all(np.array_equal(a, c[6] > 0) for a, c in zip(act, ckm))
        fd = (Lp - Lm) / (2 * h)
        assert np.isclose(gl[e], fd, rtol=1e-4, atol=1e-7 * abs(gl).max()), (e, gl[e], fd)
    for (vtx, ax) in [(3, 2), (10, 0)]:
        h = 1e-5
        for which, g in ((0, gq), (1, gv)):
            xp = [q0.copy(), v0.copy()]
            xm = [q0.copy(), v0.copy()]
            xp[which][vtx, ax] += h
            xm[which][vtx, ax] -= h
            fd = (contact_loss(sc, sc.log_E, xp[0], xp[1], cons, frozen)[0] -
                  contact_loss(sc, sc.log_E, xm[0], xm[1], cons, frozen)[0]) / (2 * h)
            assert np.isclose(g[vtx, ax], fd, rtol=1e-4, atol=1e-7 * np.abs(g).max()), (which, g[vtx, ax], fd)
