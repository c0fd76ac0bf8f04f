"""Pins of the oracle's Coulomb friction (Sec. 4.7 with the friction disk;
Sec. 4.8 with the active set fixed) against facts fixed outside it: the
single-contact closed forms of Coulomb's law, a projected Gauss-Seidel solve
of the same law written here in world coordinates (a different algorithm
that shares nothing with the oracle's Newton), the frictionless LCP as the
zero-friction limit, the step's equilibrium and Coulomb conditions at
convergence, the dense adjoint against the fixed point, and central finite
differences through sticking and sliding steps.  CPU only."""
import numpy as np
import pytest

import oracle as O
from paper_2605_14526_amd import scenes

MU = 0.5


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


def test_frame_is_orthonormal_and_right_handed():
    t1, t2 = O.contact_frame(np.array([0.0, 0.0, 1.0]))
    assert np.array_equal(t1, [1.0, 0.0, 0.0]) and np.array_equal(t2, [0.0, 1.0, 0.0])
    for n in rng(0).standard_normal((20, 3)):
        n = unit(n)
        t1, t2 = O.contact_frame(n)
        F = np.stack([n, t1, t2])
        assert np.allclose(F @ F.T, np.eye(3), atol=1e-14)
        assert np.allclose(np.cross(t1, t2), n, atol=1e-14)


def world_impulse(n, lam):
    t1, t2 = O.contact_frame(n)
    return lam[0] * n + lam[1] * t1 + lam[2] * t2


def oracle_u0(normals, x, g):
    """gap and slip in the oracle's frames of world-frame free displacements x (K, 3)"""
    u0 = np.zeros_like(x)
    for c, n in enumerate(normals):
        t1, t2 = O.contact_frame(n)
        u0[c] = [n @ x[c] - g[c], t1 @ x[c], t2 @ x[c]]
    return u0


@pytest.mark.parametrize("n", [(0.0, 0.0, 1.0), (0.3, -0.5, 0.8), (-1.0, 0.0, 0.0)])
def test_single_contact_closed_forms(n):
    """One contact with w = G_cc: separated (lambda = 0); in contact the normal impulse closes the gap,
    lambda_n = -delta0/w; the trial tangential impulse -s0/w sticks inside the disk mu lambda_n and
    otherwise slides at its rim against the free slip."""
    n = unit(n)
    w = 0.7
    G = np.array([[w]])
    t1, t2 = O.contact_frame(n)
    for delta0, slip, kind in [(0.2, (0.1, 0.0), "sep"), (-0.3, (0.05, -0.02), "stick"),
                               (-0.3, (0.4, 0.25), "slide")]:
        x = delta0 * n + slip[0] * t1 + slip[1] * t2
        u0 = oracle_u0([n], x[None], [0.0])
        lam, it, res = O.friction_ncp(G, n[None], u0, MU)
        imp = world_impulse(n, lam[0])
        s0 = np.array(slip)
        if kind == "sep":
            assert np.array_equal(lam, np.zeros((1, 3)))
            continue
        ln = -delta0 / w
        trial = -s0 / w
        if kind == "stick":
            assert np.linalg.norm(trial) <= MU * ln
            ref = ln * n + trial[0] * t1 + trial[1] * t2
        else:
            assert np.linalg.norm(trial) > MU * ln
            d = -s0 / np.linalg.norm(s0)
            ref = ln * n + MU * ln * (d[0] * t1 + d[1] * t2)
        assert np.allclose(imp, ref, rtol=1e-13, atol=1e-15), (kind, imp, ref)
        assert res <= 1e-14 and it <= 10


def pgs_world(G, normals, x, g, mu, sweeps=4000):
    """Projected block Gauss-Seidel on Coulomb's law in world coordinates: contact c sees the
    displacement x_c + sum_d G_cd imp_d and its 3x3 diagonal block is G_cc I, so its local problem
    (every other impulse fixed) has the closed-form solution of the single-contact law."""
    K = len(G)
    imp = np.zeros((K, 3))
    for _ in range(sweeps):
        for c in range(K):
            n = normals[c]
            r = x[c] + G[c] @ imp - G[c, c] * imp[c]
            rn = n @ r - g[c]
            rt = r - (n @ r) * n
            w = G[c, c]
            ln = max(0.0, -rn / w)
            trial = -rt / w
            if np.linalg.norm(trial) <= mu * ln:
                f = trial
            else:
                f = -mu * ln * rt / np.linalg.norm(rt)
            imp[c] = ln * n + f
    return imp


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_newton_matches_projected_gauss_seidel(seed):
    r = rng(seed)
    K = 2 + seed
    B = r.standard_normal((K, K))
    G = 0.3 * B @ B.T / K + np.diag(r.uniform(1.0, 2.0, K))
    normals = np.array([unit(r.standard_normal(3) + [0, 0, 2.0]) for _ in range(K)])
    x = r.standard_normal((K, 3))
    g = np.zeros(K)
    lam, it, res = O.friction_ncp(G, normals, oracle_u0(normals, x, g), MU)
    imp = np.array([world_impulse(normals[c], lam[c]) for c in range(K)])
    ref = pgs_world(G, normals, x, g, MU)
    assert res <= 1e-14 and it < 50
    assert np.allclose(imp, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max()), (imp, ref)
    # both sticking and sliding contacts occur across the seeds
    ln = lam[:, 0]
    assert (ln >= 0).all()
    assert (np.linalg.norm(lam[:, 1:], axis=1) <= MU * ln * (1 + 1e-12) + 1e-300).all()


def test_mix_of_states_across_seeds():
    kinds = set()
    for seed in [1, 2, 3, 4, 5]:
        r = rng(seed)
        K = 2 + seed
        B = r.standard_normal((K, K))
        G = 0.3 * B @ B.T / K + np.diag(r.uniform(1.0, 2.0, K))
        normals = np.array([unit(r.standard_normal(3) + [0, 0, 2.0]) for _ in range(K)])
        x = r.standard_normal((K, 3))
        lam, _, _ = O.friction_ncp(G, normals, oracle_u0(normals, x, np.zeros(K)), MU)
        for c in range(K):
            if lam[c, 0] == 0:
                kinds.add("separated")
            elif np.linalg.norm(lam[c, 1:]) < MU * lam[c, 0] * (1 - 1e-9):
                kinds.add("stick")
            else:
                kinds.add("slide")
    assert kinds == {"separated", "stick", "slide"}


def test_vanishing_friction_is_the_frictionless_lcp():
    """mu -> 0 leaves no tangential impulse, and the normal impulses solve the frictionless LCP on
    W = (n_c . n_d) G_cd (the oracle's FB Newton, itself pinned by enumeration)."""
    r = rng(11)
    K = 6
    B = r.standard_normal((K, K))
    G = B @ B.T / K + np.eye(K)
    normals = np.array([unit(r.standard_normal(3) + [0, 0, 1.5]) for _ in range(K)])
    x = r.standard_normal((K, 3))
    u0 = oracle_u0(normals, x, np.zeros(K))
    lam, _, _ = O.friction_ncp(G, normals, u0, 1e-300)
    W = (normals @ normals.T) * G
    ref, _, _ = O.fb_lcp(W, u0[:, 0])
    assert np.abs(lam[:, 1:]).max() <= 1e-290
    assert np.allclose(lam[:, 0], ref, rtol=1e-11, atol=1e-14)


def sliding_drop(res=4, lateral=(0.2, 0.2 / 3)):
    return scenes.drop_blob(res=res, friction=MU, lateral=lateral)


def friction_window(sc, before=1, max_steps=300):
    osc = O.OracleScene(sc)
    q, v = sc.q0(), sc.v0()
    hist = []
    for t in range(max_steps):
        hist.append((q, v, t))
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles, one_per_vertex=True)
        q, v, _, lam, _ = O.step_forward_friction(osc, q, v, sc.f_ext(t), con, MU)
        if (lam[:, 0] > 0).any():
            return hist[max(0, t - before)]
    raise AssertionError("the drop never lands")


def classify(lam, slip, G_diag):
    ln = lam[:, 0]
    out = []
    for c in range(len(ln)):
        if ln[c] <= 0:
            out.append("sep")
        elif np.linalg.norm(slip[c]) / G_diag[c] > 1e-8 * MU * ln[c]:
            out.append("slide")
        else:
            out.append("stick")
    return out


def test_friction_step_conditions():
    """At converged steps through the landing: equilibrium A q - c - b(q) - sum_c impulse_c = 0, the
    Signorini conditions on the normal, |lambda_f| <= mu lambda_n, zero slip where the friction is
    inside the disk, and the friction opposite the slip at the rim where it slides."""
    sc = sliding_drop()
    q, v, t0 = friction_window(sc)
    osc = O.OracleScene(sc, eps_rel=1e-13, eps_abs=1e-16)
    seen = set()
    for t in range(t0, t0 + 12):
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles, one_per_vertex=True)
        f = sc.f_ext(t)
        qn, vn, qm1, lam, st = O.step_forward_friction(osc, q, v, f, con, MU, fb_tol=1e-14)
        assert st["status"] == 0
        cv, cn, cg = con
        c_rhs, _ = osc.const_rhs(q, v, f)
        res = osc.apply_A(qn) - c_rhs - osc.local_rhs(qn)
        for k in range(len(cv)):
            res[cv[k]] -= world_impulse(cn[k], lam[k])
        scale = np.abs(osc.apply_A(qn)).max()
        assert np.abs(res).max() <= 1e-9 * scale
        ln = lam[:, 0]
        delta = (cn * qn[cv]).sum(axis=1) - cg
        assert (ln >= 0).all() and (delta >= -1e-12).all()
        assert np.abs(ln * delta).max() <= 1e-12 * max(1.0, ln.max())
        lf = np.linalg.norm(lam[:, 1:], axis=1)
        assert (lf <= MU * ln * (1 + 1e-12)).all()
        for k in range(len(cv)):
            if ln[k] == 0:
                continue
            t1, t2 = O.contact_frame(cn[k])
            s = np.array([t1 @ (qn[cv[k]] - q[cv[k]]), t2 @ (qn[cv[k]] - q[cv[k]])])
            ns = np.linalg.norm(s)
            if lf[k] < MU * ln[k] * (1 - 1e-8):
                assert ns <= 1e-12, (k, ns)
                seen.add("stick")
            elif ns > 1e-9:
                assert np.allclose(lam[k, 1:], -MU * ln[k] * s / ns, rtol=1e-8, atol=1e-14 * ln[k])
                seen.add("slide")
        q, v = qn, vn
    assert seen == {"stick", "slide"}


def test_unreached_rows_are_bitwise_contact_free():
    sc = scenes.small_beam(4, 2, 2, seed=21, contrast=30.0, tip_force=10.0)
    osc = O.OracleScene(sc)
    q, v = sc.q0(), sc.v0()
    for t in range(3):
        f = sc.f_ext(t)
        qa, va, qma, sta = osc.step_forward(q, v, f)
        free = np.where(sc.pinned == 0)[0].astype(np.int32)
        con = (free, np.tile([0.0, 0.0, 1.0], (len(free), 1)), np.full(len(free), -10.0))
        qb, vb, qmb, lam, stb = O.step_forward_friction(osc, q, v, f, con, MU)
        assert np.array_equal(qa, qb) and np.array_equal(va, vb) and np.array_equal(qma, qmb)
        assert sta["iters"] == stb["iters"] and not lam.any()
        q, v = qa, va


def test_friction_adjoint_dense_matches_fixed_point():
    sc = sliding_drop()
    q, v, t0 = friction_window(sc)
    osc = O.OracleScene(sc, eps_rel=1e-12, eps_abs=1e-16, eps_adj=1e-13, kmax_bwd=20000)
    g = rng(9).standard_normal(q.shape)
    kinds = set()
    checked = 0
    for t in range(t0, t0 + 10):
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles, one_per_vertex=True)
        f = sc.f_ext(t)
        qn, vn, qm1, lam, st = O.step_forward_friction(osc, q, v, f, con, MU)
        if (lam[:, 0] > 0).any():
            a = O.step_backward_friction(osc, q, v, f, qn, qm1, g, 0.1 * g, con, MU, lam, adj_mode=1)
            b = O.step_backward_friction(osc, q, v, f, qn, qm1, g, 0.1 * g, con, MU, lam, adj_mode=0)
            assert a[4]["status"] == 0 and b[4]["status"] == 0
            for x, y in zip(a[:4], b[:4]):
                assert np.allclose(x, y, rtol=1e-8, atol=1e-10 * np.abs(x).max())
            lf = np.linalg.norm(lam[:, 1:], axis=1)
            kinds |= {"slide" if lf[k] >= MU * lam[k, 0] * (1 - 1e-8) else "stick"
                      for k in range(len(lam)) if lam[k, 0] > 0}
            checked += 1
        q, v = qn, vn
    assert checked >= 3 and kinds == {"stick", "slide"}


def friction_loss(sc, logE, q0, v0, cons, frozen, t0):
    osc = O.OracleScene(sc, log_E=logE, eps_rel=1e-14, eps_abs=1e-16, frozen=frozen, eps_adj=1e-14)
    q, v = q0.copy(), v0.copy()
    ck = []
    for k, con in enumerate(cons):
        f = sc.f_ext(t0 + k)
        qn, vn, qm1, lam, st = O.step_forward_friction(osc, q, v, f, con, MU, fb_tol=1e-15)
        ck.append((q, v, f, qn, qm1, con, lam))
        q, v = qn, vn
    L, gq = scenes.centroid_loss(q, sc.target_centroid)
    w = np.linspace(0.5, 1.5, q.shape[0])[:, None]
    L += float(np.sum(w * q * q)) + 1e-3 * float(np.sum(v * v))
    gq = gq + 2.0 * w * q
    gv = 2e-3 * v
    return L, gq, gv, ck, osc


def states(ck):
    out = []
    for (q_t, v_t, f, qs, qsm1, con, lam) in ck:
        cv, cn, cg = con
        st = []
        for k in range(len(cv)):
            if lam[k, 0] <= 0:
                st.append(0)
            else:
                st.append(2 if np.linalg.norm(lam[k, 1:]) >= MU * lam[k, 0] * (1 - 1e-8) else 1)
        out.append(st)
    return out


def test_friction_gradients_match_central_differences():
    """Through steps with sticking and sliding contacts (rows fixed to those of the unperturbed rollout,
    no contact changing state under the perturbations), the adjoint gradients with respect to log E,
    q0 and v0 equal central differences."""
    sc = sliding_drop()
    q0, v0, t0 = friction_window(sc, before=0)
    base = O.OracleScene(sc).info()
    frozen = (base["mu_bar"], base["lam_bar"], base["mu_ref"])
    steps = 5
    osc = O.OracleScene(sc, eps_rel=1e-14, eps_abs=1e-16, frozen=frozen)
    cons, q, v = [], q0.copy(), v0.copy()
    for k in range(steps):
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles, one_per_vertex=True)
        cons.append(con)
        q, v, _, _, _ = O.step_forward_friction(osc, q, v, sc.f_ext(t0 + k), con, MU)
    L, gq, gv, ck, osc = friction_loss(sc, sc.log_E, q0, v0, cons, frozen, t0)
    st0 = states(ck)
    flat = [s for st in st0 for s in st]
    assert 1 in flat and 2 in flat
    gl = np.zeros(sc.n_e)
    for (q_t, v_t, f, qs, qsm1, con, lam) in reversed(ck):
        gq, gv, gf, gl, st = O.step_backward_friction(osc, q_t, v_t, f, qs, qsm1, gq, gv, con, MU, lam, gl,
                                                      adj_mode=1)
        assert st["status"] == 0
    for e in rng(3).choice(sc.n_e, 3, replace=False):
        h = 1e-3
        lp, lm = sc.log_E.copy(), sc.log_E.copy()
        lp[e] += h
        lm[e] -= h
        Lp, _, _, ckp, _ = friction_loss(sc, lp, q0, v0, cons, frozen, t0)
        Lm, _, _, ckm, _ = friction_loss(sc, lm, q0, v0, cons, frozen, t0)
        assert states(ckp) == st0 and states(ckm) == st0
        fd = (Lp - Lm) / (2 * h)
        assert np.isclose(gl[e], fd, rtol=1e-4, atol=1e-7 * abs(gl).max()), (e, gl[e], fd)
    for (vtx, ax) in [(3, 2), (10, 0), (7, 1)]:
        h = 1e-6
        for which, g in ((0, gq), (1, gv)):
            xp = [q0.copy(), v0.copy()]
            xm = [q0.copy(), v0.copy()]
            xp[which][vtx, ax] += h
            xm[which][vtx, ax] -= h
            Lp, _, _, ckp, _ = friction_loss(sc, sc.log_E, xp[0], xp[1], cons, frozen, t0)
            Lm, _, _, ckm, _ = friction_loss(sc, sc.log_E, xm[0], xm[1], cons, frozen, t0)
            assert states(ckp) == st0 and states(ckm) == st0
            fd = (Lp - Lm) / (2 * h)
            assert np.isclose(g[vtx, ax], fd, rtol=1e-4, atol=1e-7 * np.abs(g).max()), (which, vtx, ax, g[vtx, ax], fd)
