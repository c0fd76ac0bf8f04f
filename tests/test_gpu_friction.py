"""Coulomb friction (Sec. 4.7 with the friction disk; Sec. 4.8 with the active
set fixed) on the GPU against the FP64 oracle: one contact per vertex with a
frame of three rows, the detected contacts (exact), positions and the three
impulse components step by step from the oracle's states through sliding and
sticking landings, reverse sweeps through frictional steps (the unsymmetric
adjoint), obstacles out of reach, and the contact drops at the benchmark's
sizes.  All calls go through the C ABI."""
import numpy as np
import pytest

import oracle as O
from paper_2605_14526_amd import scenes

pytestmark = pytest.mark.gpu

TOL_POS = 1e-9
TOL_GRAD = 1e-6
MU = 0.5


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.fixture(scope="module")
def th(torch_cuda):
    return torch_cuda


def dev(th, a):
    return th.tensor(np.ascontiguousarray(a), dtype=th.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def detect(sc, q, v):
    return O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles, one_per_vertex=True)


def oracle_until_landing(sc, before=1, max_steps=300):
    osc = O.OracleScene(sc)
    q, v = sc.q0(), sc.v0()
    hist = []
    for t in range(max_steps):
        hist.append((t, q, v))
        con = detect(sc, q, v)
        q, v, _, lam, _ = O.step_forward_friction(osc, q, v, sc.f_ext(t), con, MU)
        if (lam[:, 0] > 0).any():
            return hist[max(0, t - before)]
    raise AssertionError("no landing")


def row_key(v, n, g):
    return [(int(a), tuple(float(x) for x in b), float(c)) for a, b, c in zip(v, n, g)]


def kinds(lam):
    out = set()
    for l in lam:
        if l[0] <= 0:
            continue
        out.add("slide" if np.linalg.norm(l[1:]) >= MU * l[0] * (1 - 1e-8) else "stick")
    return out


@pytest.mark.parametrize("res,with_box,lateral", [(4, True, 0.2), (6, True, 0.3), (8, False, 0.5), (12, True, 0.4)])
def test_friction_stepwise(th, res, with_box, lateral):
    """From each oracle state through a sliding landing: the GPU's contacts
    equal the oracle's (one per vertex: vertex, normal, offset), iteration
    counts are equal, positions agree to 1e-9 and every impulse component to
    1e-6 of the largest, with sticking and sliding contacts both present."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.drop_blob(res=res, with_box=with_box, friction=MU, lateral=(lateral, lateral / 3))
    t0, q, v = oracle_until_landing(sc)
    osc = O.OracleScene(sc)
    g = Scene.from_scene(sc)
    seen = set()
    print(f"[friction] res {res} landing at step {t0}", flush=True)
    for t in range(t0, t0 + 10):
        f = sc.f_ext(t)
        con = detect(sc, q, v)
        qo, vo, _, lam_o, st_o = O.step_forward_friction(osc, q, v, f, con, MU)
        qg, vg, st = g.step_forward(dev(th, q), dev(th, v), dev(th, f))
        assert st["status"] == 0 and st_o["status"] == 0
        rv, rn, rg, _ = g.contact_rows()
        lg = g.contact_impulses()
        # the library lists contacts in its own vertex order: match them by key
        kg, ko = row_key(rv, rn, rg), row_key(*con)
        assert sorted(kg) == sorted(ko), t
        assert st["iters"] == st_o["iters"], (t, st["iters"], st_o["iters"])
        assert rel(host(qg), qo) < TOL_POS, (t, rel(host(qg), qo))
        if len(lam_o):
            lg = np.array([lg[kg.index(k)] for k in ko])
            scale = max(np.abs(lam_o).max(), 1e-300)
            assert np.abs(lg - lam_o).max() <= 1e-6 * scale, (t, np.abs(lg - lam_o).max() / scale)
            seen |= kinds(lam_o)
        q, v = qo, vo
    assert seen == {"stick", "slide"}, seen


def test_friction_out_of_reach_is_contact_free(th):
    """Obstacles that never come within reach leave the frictional step bitwise
    equal to the step without obstacles."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.small_beam(5, 2, 2, seed=8, contrast=10.0, tip_force=6.0)
    a = Scene.from_scene(sc)
    b = Scene.from_scene(sc)
    b.set_obstacles({"planes": [((0.0, 0.0, 1.0), -50.0)], "boxes": [], "d_c": 0.01}, max_contacts=16)
    b.set_friction(MU)
    q, v = dev(th, sc.q0()), dev(th, sc.v0())
    for t in range(3):
        f = dev(th, sc.f_ext(t))
        qa, va, sa = a.step_forward(q, v, f)
        qb, vb, sb = b.step_forward(q, v, f)
        assert th.equal(qa, qb) and th.equal(va, vb) and sa["iters"] == sb["iters"]
        q, v = qa, va


@pytest.mark.parametrize("res,lateral", [(4, 0.2), (6, 0.3)])
def test_friction_gradients_match_oracle(th, res, lateral):
    """Eight steps through a sliding and sticking landing forward, the loss
    gradient swept back to the start state and log E with the active contacts
    held fixed: the GPU's projected fixed point (the frictional adjoint is
    unsymmetric) matches the oracle's dense solves to 1e-6."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.drop_blob(res=res, with_box=True, friction=MU, lateral=(lateral, lateral / 3))
    t0, q0, v0 = oracle_until_landing(sc, before=1)
    T = 8
    osc = O.OracleScene(sc)
    q, v = q0.copy(), v0.copy()
    ck_o = []
    seen = set()
    for t in range(t0, t0 + T):
        f = sc.f_ext(t)
        con = detect(sc, q, v)
        qn, vn, qm1, lam, st = O.step_forward_friction(osc, q, v, f, con, MU)
        ck_o.append((q, v, f, qn, qm1, con, lam))
        seen |= kinds(lam)
        q, v = qn, vn
    assert seen == {"stick", "slide"}, seen
    g = Scene.from_scene(sc, eps_adj=1e-12, kmax_bwd=20000)
    qg, vg = dev(th, q0), dev(th, v0)
    cks = []
    for t in range(t0, t0 + T):
        ck = g.new_ckpt()
        qg, vg, st = g.step_forward(qg, vg, dev(th, sc.f_ext(t)), ckpt=ck)
        assert st["status"] == 0
        cks.append(ck)
    assert rel(host(qg), q) < TOL_POS
    _, gq = scenes.centroid_loss(q, sc.target_centroid)
    gv = 0.3 * np.ones_like(gq)
    gq0_o, gv0_o, gl_o, _ = O.rollout_backward_friction(osc, ck_o, gq, gv, MU, adj_mode=1)
    g.adjoint_reset()
    gqd, gvd = dev(th, gq), dev(th, gv)
    gl = th.zeros(sc.n_e, dtype=th.float64, device="cuda")
    n_act = 0
    for ck in reversed(cks):
        gqd, gvd, _, _, st = g.step_backward(ck, gqd, gvd, g_logE=gl)
        assert st["status"] == 0, st
        n_act += st["n_active"]
    assert n_act > 0
    for a, b in [(host(gqd), gq0_o), (host(gvd), gv0_o), (host(gl), gl_o)]:
        assert rel(a, b) < TOL_GRAD, rel(a, b)


def test_friction_drop_benchmark_size(th):
    """The frictional drop at the contact benchmark's size (res 27, about 28k
    tets, mu 0.5) in the benchmark's launch configuration, stepped from the
    oracle's own states through its landing, then one reverse step through
    its active contacts against the oracle's fixed point."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.drop_blob(res=27, friction=MU, lateral=(0.3, 0.1))
    t0, q, v = oracle_until_landing(sc, before=1)
    osc = O.OracleScene(sc, eps_adj=1e-11, kmax_bwd=20000)
    g = Scene.from_scene(sc, eps_adj=1e-11, kmax_bwd=20000)
    seen = set()
    for t in range(t0, t0 + 5):
        f = sc.f_ext(t)
        con = detect(sc, q, v)
        qo, vo, qm1, lam, st_o = O.step_forward_friction(osc, q, v, f, con, MU)
        ck = g.new_ckpt()
        qg, vg, st = g.step_forward(dev(th, q), dev(th, v), dev(th, f), ckpt=ck)
        assert st["n_contacts"] == len(con[0]) and st["iters"] == st_o["iters"], (t, st, st_o["iters"])
        assert rel(host(qg), qo) < TOL_POS, (t, rel(host(qg), qo))
        seen |= kinds(lam)
        last = (q, v, f, qo, qm1, con, lam, ck)
        q, v = qo, vo
    assert "slide" in seen or "stick" in seen
    q_t, v_t, f, qs, qsm1, con, lam, ck = last
    gq = np.random.Generator(np.random.PCG64(5)).standard_normal(q_t.shape)
    gv = 0.1 * gq
    a = O.step_backward_friction(osc, q_t, v_t, f, qs, qsm1, gq, gv, con, MU, lam, adj_mode=0)
    assert a[4]["status"] == 0
    b = g.step_backward(ck, dev(th, gq), dev(th, gv))
    assert b[4]["n_active"] == int((lam[:, 0] > 0).sum())
    for x, y in zip(b[:4], a[:4]):
        assert rel(host(x), y) < TOL_GRAD, rel(host(x), y)
