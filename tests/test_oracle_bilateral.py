"""Pins of the oracle's bilateral rows (attachments held as equality constraints
with free multipliers, Sec. 4.7) and of the restitution post-correction
against facts fixed independently of the oracle: attaching a vertex to its rest
position reproduces the eliminated (pinned) vertex, forward and backward; the
attachment holds exactly; the gradient with respect to an attachment target and
the gradients through restitution steps match central differences; the
restitution rule's post-condition.  CPU only."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2605_14526_amd import scenes


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def attached_twin(sc):
    """The scene with its pinned vertices freed (they become attachment rows)."""
    return dataclasses.replace(sc, pinned=np.zeros_like(sc.pinned))


@pytest.mark.parametrize("seed", [3, 8])
def test_attachment_at_rest_equals_elimination(seed):
    """Rows tying each pinned vertex to its rest position give the Dirichlet solution: positions through a
    rollout, and the gradients w.r.t. log E and the other vertices' initial state."""
    sc = scenes.small_beam(5, 2, 2, seed=seed, tip_force=15.0, alpha=0.05, beta_rel=0.02)
    pin = np.where(sc.pinned)[0]
    kw = dict(eps_rel=1e-13, eps_abs=1e-16, eps_adj=1e-14)
    o_pin = O.OracleScene(sc, **kw)
    frozen = (o_pin.info()["mu_bar"], o_pin.info()["lam_bar"], o_pin.info()["mu_ref"])
    o_att = O.OracleScene(attached_twin(sc), frozen=frozen, **kw)
    steps = 4
    q, v, ck, _ = O.rollout(o_pin, steps)
    qa, va, cka, sta = O.rollout_contact_ext(o_att, steps, attach=(pin, lambda t: sc.X[pin]), fb_tol=1e-15)
    assert np.abs(qa[pin] - sc.X[pin]).max() < 1e-13  # the FB stop (1e-14) after Anderson mixing
    assert np.abs(q - qa).max() < 1e-10 * np.abs(q).max()
    assert np.abs(v - va).max() < 1e-8 * np.abs(v).max()
    _, gq = scenes.centroid_loss(q, sc.target_centroid)
    gv = 0.1 * rng(seed).standard_normal(q.shape)
    gq0, gv0, gl, _ = O.rollout_backward(o_pin, ck, gq, gv, adj_mode=1)
    gqa, gva, gla, ggs, _ = O.rollout_backward_contact_ext(o_att, cka, gq, gv, adj_mode=1)
    free = ~sc.pinned.astype(bool)
    assert np.abs(gla - gl).max() < 1e-8 * np.abs(gl).max()
    assert np.abs(gqa[free] - gq0[free]).max() < 1e-8 * np.abs(gq0).max()
    assert np.abs(gva[free] - gv0[free]).max() < 1e-8 * np.abs(gv0).max()
    # the projected fixed point gives the dense saddle point's gradients and target gradients
    gqf, gvf, glf, ggf, _ = O.rollout_backward_contact_ext(o_att, cka, gq, gv, adj_mode=0)
    assert np.abs(glf - gla).max() < 1e-7 * np.abs(gla).max()
    for a, b in zip(ggf, ggs):
        assert np.abs(a - b).max() < 1e-7 * max(np.abs(b).max(), 1e-300)


def moving_target_loss(sc, pin, targets, q0, v0, frozen, logE=None):
    o = O.OracleScene(sc, log_E=logE, eps_rel=1e-14, eps_abs=1e-16, frozen=frozen, eps_adj=1e-14)
    q, v, ck, _ = O.rollout_contact_ext(o, len(targets), attach=(pin, lambda t: targets[t]), fb_tol=1e-15,
                                        q0=q0, v0=v0)
    w = np.linspace(0.5, 1.5, q.shape[0])[:, None]
    L = float(np.sum(w * q * q)) + 1e-3 * float(np.sum(v * v))
    return L, 2.0 * w * q, 2e-3 * v, ck, o


def test_attachment_target_gradient_central_differences():
    """A beam whose end vertices are dragged along a path by attachment rows: dL/dg of each row at each step
    (and dL/dlog E) against central differences of the loss."""
    base = scenes.small_beam(4, 2, 2, seed=5, tip_force=0.0, alpha=0.02, beta_rel=0.01)
    pin = np.where(base.pinned)[0]
    sc = attached_twin(base)
    frozen = (O.OracleScene(sc).info()["mu_bar"], O.OracleScene(sc).info()["lam_bar"],
              O.OracleScene(sc).info()["mu_ref"])
    steps = 3
    targets = [base.X[pin] + np.array([0.0, 0.01 * (t + 1), -0.004 * (t + 1)]) for t in range(steps)]
    q0, v0 = sc.X.copy(), np.zeros_like(sc.X)
    L, gq, gv, ck, o = moving_target_loss(sc, pin, targets, q0, v0, frozen)
    gqa, gva, gla, ggs, _ = O.rollout_backward_contact_ext(o, ck, gq, gv, adj_mode=1)
    r = rng(9)
    for t in range(steps):
        for row in r.choice(3 * len(pin), 3, replace=False):
            h = 1e-6
            tp = [x.copy() for x in targets]
            tm = [x.copy() for x in targets]
            tp[t][row // 3, row % 3] += h
            tm[t][row // 3, row % 3] -= h
            fd = (moving_target_loss(sc, pin, tp, q0, v0, frozen)[0] -
                  moving_target_loss(sc, pin, tm, q0, v0, frozen)[0]) / (2 * h)
            assert np.isclose(ggs[t][row], fd, rtol=1e-5, atol=1e-8 * np.abs(ggs[t]).max()), (t, row, ggs[t][row], fd)
    for e in r.choice(sc.n_e, 2, replace=False):
        h = 1e-3  # the converged rollout carries noise of ~1e-14 of L: smaller steps see it
        lp, lm = sc.log_E.copy(), sc.log_E.copy()
        lp[e] += h
        lm[e] -= h
        fd = (moving_target_loss(sc, pin, targets, q0, v0, frozen, lp)[0] -
              moving_target_loss(sc, pin, targets, q0, v0, frozen, lm)[0]) / (2 * h)
        assert np.isclose(gla[e], fd, rtol=1e-4, atol=1e-8 * np.abs(gla).max()), (e, gla[e], fd)


def landing(res=4, e=0.5, before=1):
    """The tiny drop's state `before` steps ahead of its first landing step."""
    sc = scenes.drop_blob(res=res)
    osc = O.OracleScene(sc)
    q, v = sc.q0(), sc.v0()
    hist = []
    empty = (np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.uint8))
    for t in range(200):
        hist.append((q, v))
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        rows = O.join_rows(con, empty)
        qn, vn, _, lam, _ = O.step_forward_contact_ext(osc, q, v, sc.f_ext(t), rows, restitution=e)
        if (lam > 0).any():
            q, v = hist[max(0, t - before)]
            return sc, q, v, t - before
        q, v = qn, vn
    raise AssertionError("the drop never lands")


def test_restitution_post_condition():
    """At the landing step every active row whose vertex approached sets the vertex's outgoing normal
    velocity to -e times the incoming one, leaves its tangential velocity to the step, and moves no
    position; with no approaching active row the step is unchanged."""
    e = 0.4
    sc, q, v, t = landing(e=e, before=0)
    osc = O.OracleScene(sc)
    empty = (np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.uint8))
    rows = O.join_rows(O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles), empty)
    qe, ve, _, lam, _ = O.step_forward_contact_ext(osc, q, v, sc.f_ext(t), rows, restitution=e)
    q0_, v0_, _, lam0, _ = O.step_forward_contact_ext(osc, q, v, sc.f_ext(t), rows, restitution=None)
    assert np.array_equal(qe, q0_) and np.array_equal(lam, lam0)
    cv, cn = rows[0], rows[1]
    hit = 0
    for c in range(len(cv)):
        u = float(cn[c] @ v[cv[c]])
        if lam[c] > 1e-10 * lam.max() and u < 0.0:
            hit += 1
            assert abs(float(cn[c] @ ve[cv[c]]) + e * u) < 1e-14 * max(1.0, abs(u))
            tang = ve[cv[c]] - (cn[c] @ ve[cv[c]]) * cn[c]
            tang0 = v0_[cv[c]] - (cn[c] @ v0_[cv[c]]) * cn[c]
            assert np.abs(tang - tang0).max() < 1e-14 * max(1.0, np.abs(tang0).max())
    assert hit > 0
    moved = np.zeros(len(ve), bool)
    moved[cv[(lam > 1e-10 * lam.max())]] = True
    assert np.array_equal(ve[~moved], v0_[~moved])


def restitution_loss(sc, logE, q0, v0, rows_per_step, e, frozen):
    o = O.OracleScene(sc, log_E=logE, eps_rel=1e-14, eps_abs=1e-16, frozen=frozen, eps_adj=1e-14)
    q, v = q0.copy(), v0.copy()
    ck = []
    for t, rows in enumerate(rows_per_step):
        f = sc.f_ext(t)
        qn, vn, qm1, lam, _ = O.step_forward_contact_ext(o, q, v, f, rows, restitution=e, fb_tol=1e-15)
        ck.append((q, v, f, qn, qm1, rows, lam))
        q, v = qn, vn
    w = np.linspace(0.5, 1.5, q.shape[0])[:, None]
    L = float(np.sum(w * q * q)) + 0.3 * float(np.sum(w * v * v))
    return L, 2.0 * w * q, 0.6 * w * v, ck, o


@pytest.mark.parametrize("adj_mode", [0, 1])
def test_restitution_gradients_central_differences(adj_mode):
    """Through four steps around the landing with e = 0.5 (rows fixed to those of the unperturbed rollout,
    active and restitution sets unchanged by the perturbations): gradients w.r.t. log E, q0 and v0."""
    e = 0.5
    sc, q0, v0, t0 = landing(e=e, before=1)
    base = O.OracleScene(sc).info()
    frozen = (base["mu_bar"], base["lam_bar"], base["mu_ref"])
    empty = (np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.uint8))
    o = O.OracleScene(sc, eps_rel=1e-14, eps_abs=1e-16, frozen=frozen)
    rows_per_step, q, v = [], q0.copy(), v0.copy()
    for t in range(4):
        rows = O.join_rows(O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles), empty)
        rows_per_step.append(rows)
        q, v, _, _, _ = O.step_forward_contact_ext(o, q, v, sc.f_ext(t), rows, restitution=e)
    L, gq, gv, ck, o = restitution_loss(sc, sc.log_E, q0, v0, rows_per_step, e, frozen)
    bounced = sum(int(((c[6] > 1e-10 * max(c[6].max(), 1e-300)) &
                       (np.einsum("ij,ij->i", c[5][1], c[1][c[5][0]]) < 0)).sum()) for c in ck)
    assert bounced > 0
    gl = np.zeros(sc.n_e)
    for (q_t, v_t, f, qs, qsm1, rows, lam) in reversed(ck):
        gq, gv, _, gl, _, _ = O.step_backward_contact_ext(o, q_t, v_t, f, qs, qsm1, gq, gv, rows, lam,
                                                          restitution=e, g_logE=gl, adj_mode=adj_mode)
    tol = 1e-4 if adj_mode == 1 else 1e-3
    for ev in rng(3).choice(sc.n_e, 2, replace=False):
        h = 1e-3
        lp, lm = sc.log_E.copy(), sc.log_E.copy()
        lp[ev] += h
        lm[ev] -= h
        fd = (restitution_loss(sc, lp, q0, v0, rows_per_step, e, frozen)[0] -
              restitution_loss(sc, lm, q0, v0, rows_per_step, e, frozen)[0]) / (2 * h)
        assert np.isclose(gl[ev], fd, rtol=tol, atol=1e-6 * np.abs(gl).max()), (ev, gl[ev], fd)
    contact_v = int(rows_per_step[1][0][0]) if len(rows_per_step[1][0]) else 3
    for (vtx, ax) in [(contact_v, 2), (contact_v, 0), (10, 1)]:
        h = 1e-6
        for which, g in ((0, gq), (1, gv)):
            xp = [q0.copy(), v0.copy()]
            xm = [q0.copy(), v0.copy()]
            xp[which][vtx, ax] += h
            xm[which][vtx, ax] -= h
            fd = (restitution_loss(sc, sc.log_E, xp[0], xp[1], rows_per_step, e, frozen)[0] -
                  restitution_loss(sc, sc.log_E, xm[0], xm[1], rows_per_step, e, frozen)[0]) / (2 * h)
            assert np.isclose(g[vtx, ax], fd, rtol=tol, atol=1e-6 * np.abs(g).max()), (which, vtx, ax, g[vtx, ax], fd)
