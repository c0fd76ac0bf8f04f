"""Contact (frictionless reading of Sec. 4.7) on the GPU against the FP64
oracle: the detected rows (exact), positions and impulses step by step from
the oracle's states through a landing on the ground and on a box, reverse
sweeps through contact steps with both adjoint solvers, obstacles that never
touch, and the drop at its benchmark size.  All calls go through the C ABI."""
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


def dev(th, a):
    return th.tensor(np.ascontiguousarray(a), dtype=th.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def oracle_until_landing(sc, before=2, max_steps=200):
    """Oracle state `before` steps ahead of the first step with a positive impulse."""
    osc = O.OracleScene(sc)
    q, v = sc.q0(), sc.v0()
    hist = []
    for t in range(max_steps):
        hist.append((t, q, v))
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        q, v, _, lam, _ = O.step_forward_contact(osc, q, v, sc.f_ext(t), con)
        if (lam > 0).any():
            return hist[max(0, t - before)]
    raise AssertionError("no landing")


def row_key(v, n, g):
    return [(int(a), tuple(float(x) for x in b), float(c)) for a, b, c in zip(v, n, g)]


@pytest.mark.parametrize("res,with_box,dc_scale", [(4, True, 1.0), (6, True, 1.0), (8, False, 1.0), (12, False, 8.0)])
def test_rows_positions_impulses_stepwise(th, res, with_box, dc_scale):
    """From each oracle state of a landing: the GPU's rows equal the oracle's
    (same vertices, normals, offsets), and its positions and impulses agree.
    The last case has more than 64 rows (the workgroup-wide Newton kernel; the
    others run the single-wave one)."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.drop_blob(res=res, with_box=with_box)
    sc.obstacles["d_c"] *= dc_scale
    t0, q, v = oracle_until_landing(sc)
    osc = O.OracleScene(sc)
    g = Scene.from_scene(sc)
    n_act = 0
    k_max = 0
    for t in range(t0, t0 + 8):
        f = sc.f_ext(t)
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        qo, vo, _, lam_o, st_o = O.step_forward_contact(osc, q, v, f, con)
        qg, vg, st = g.step_forward(dev(th, q), dev(th, v), dev(th, f))
        assert st["status"] == 0 and st_o["status"] == 0
        rv, rn, rg, rl = g.contact_rows()
        assert sorted(row_key(rv, rn, rg)) == sorted(row_key(*con)), t
        assert st["n_contacts"] == len(con[0])
        k_max = max(k_max, len(con[0]))
        assert st["iters"] == st_o["iters"], (t, st["iters"], st_o["iters"])
        assert rel(host(qg), qo) < TOL_POS, (t, rel(host(qg), qo))
        assert rel(host(vg), vo) < 1e-6, t
        if len(lam_o):
            ko = {k: l for k, l in zip(row_key(*con), lam_o)}
            kg = {k: l for k, l in zip(row_key(rv, rn, rg), rl)}
            scale = max(np.abs(lam_o).max(), 1e-300)
            for k in ko:
                assert abs(kg[k] - ko[k]) <= 1e-6 * scale, (t, k, kg[k], ko[k])
            n_act += int((lam_o > 0).sum())
        q, v = qo, vo
    assert n_act > 0
    assert dc_scale == 1.0 or k_max > 64


def gpu_rollout_from(th, g, sc, q0, v0, t0, T):
    q, v = dev(th, q0), dev(th, v0)
    cks, iters = [], []
    for t in range(t0, t0 + T):
        ck = g.new_ckpt()
        q, v, st = g.step_forward(q, v, dev(th, sc.f_ext(t)), ckpt=ck)
        assert st["status"] == 0, st
        cks.append(ck)
        iters.append(st["iters"])
    return q, v, cks, iters


@pytest.mark.parametrize("adj_method", [0, 1])
def test_contact_gradients_match_oracle(th, adj_method):
    """Six steps through a landing forward, the loss gradient swept back to
    the start state and log E with the active rows held fixed; the GPU's PCG
    (projected preconditioner) and fixed point both match the oracle's dense
    saddle-point solves."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.drop_blob(res=6, with_box=True)
    t0, q0, v0 = oracle_until_landing(sc, before=2)
    T = 6
    osc = O.OracleScene(sc)
    q, v = q0.copy(), v0.copy()
    ck_o = []
    for t in range(t0, t0 + T):
        f = sc.f_ext(t)
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        qn, vn, qm1, lam, st = O.step_forward_contact(osc, q, v, f, con)
        ck_o.append((q, v, f, qn, qm1, con, lam))
        q, v = qn, vn
    assert sum(int((c[6] > 0).sum()) for c in ck_o) > 0
    g = Scene.from_scene(sc, eps_adj=1e-12, adj_method=adj_method, kmax_bwd=4000)
    qg, vg, cks, iters = gpu_rollout_from(th, g, sc, q0, v0, t0, T)
    assert rel(host(qg), q) < TOL_POS
    _, gq = scenes.centroid_loss(q, sc.target_centroid)
    gv = 0.3 * np.ones_like(gq)
    gq0_o, gv0_o, gl_o, _ = O.rollout_backward_contact(osc, ck_o, gq, gv, adj_mode=1)
    g.adjoint_reset()
    a, b = dev(th, gq), dev(th, gv)
    gl = th.zeros(sc.n_e, dtype=th.float64, device="cuda")
    n_act = 0
    for ck in reversed(cks):
        a, b, _, _, st = g.step_backward(ck, a, b, g_logE=gl)
        assert st["status"] == 0, st
        n_act += st["n_active"]
    assert n_act > 0
    for x, y in [(host(a), gq0_o), (host(b), gv0_o), (host(gl), gl_o)]:
        assert rel(x, y) < TOL_GRAD, (adj_method, rel(x, y))


def test_obstacles_out_of_reach(th):
    """Obstacles with no rows give bitwise the contact-free step; rows that
    never carry an impulse change the results only by rounding."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.small_beam(6, 3, 3, seed=5, contrast=30.0, nu=0.49, aa_window=2)
    far = {"planes": [((0.0, 0.0, 1.0), -10.0)], "boxes": [((5.0, 5.0, 5.0), (6.0, 6.0, 6.0))], "d_c": 0.01}
    near = {"planes": [((0.0, 0.0, 1.0), -10.0)], "boxes": [], "d_c": 100.0}
    res = {}
    for name, obs in (("none", None), ("far", far), ("near", near)):
        g = Scene.from_scene(sc)
        if obs:
            g.set_obstacles(obs)
        q, v = dev(th, sc.q0()), dev(th, sc.v0())
        cks, its, nc = [], [], []
        for t in range(4):
            ck = g.new_ckpt()
            q, v, st = g.step_forward(q, v, dev(th, sc.f_ext(t)), ckpt=ck)
            cks.append(ck)
            its.append(st["iters"])
            nc.append(st["n_contacts"])
        a, b = dev(th, np.ones_like(sc.X)), dev(th, np.zeros_like(sc.X))
        gl = th.zeros(sc.n_e, dtype=th.float64, device="cuda")
        for ck in reversed(cks):
            a, b, _, _, _ = g.step_backward(ck, a, b, g_logE=gl)
        res[name] = (host(q), host(a), host(gl), its, nc)
    assert res["far"][4] == [0] * 4 and min(res["near"][4]) > 0
    for x, y in zip(res["none"][:3], res["far"][:3]):
        assert np.array_equal(x, y)
    assert res["none"][3] == res["far"][3] == res["near"][3]
    # rounding of the inactive rows' (zero) corrections, carried through four steps and the
    # reverse sweep's solves (condition ~1e4): far below what one active row would change
    for x, y in zip(res["none"][:3], res["near"][:3]):
        assert rel(x, y) < 1e-11


def test_contact_capacity_errors(th):
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.drop_blob(res=6, with_box=False)
    g = Scene.from_scene(sc)
    # every free vertex becomes a row against a plane far above: beyond the capacity
    g.set_obstacles({"planes": [((0.0, 0.0, -1.0), -100.0)], "boxes": [], "d_c": 1e3}, max_contacts=8)
    with pytest.raises(RuntimeError, match="PD_ERR_CONTACT"):
        g.step_forward(dev(th, sc.q0()), dev(th, sc.v0()))
    with pytest.raises(RuntimeError, match="PD_ERR_INVALID_ARG"):
        g.set_obstacles({"planes": [((0.0, 0.0, 2.0), 0.0)], "boxes": [], "d_c": 0.1})


def test_drop_benchmark_size_stepwise(th):
    """The drop at about 28k tets (the benchmark's contact workload), in the
    benchmark's launch configuration, stepped from the oracle's own states
    through its landing on the ground."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.drop_blob(res=27, with_box=False)
    osc = O.OracleScene(sc)
    g = Scene.from_scene(sc)
    q, v = sc.q0(), sc.v0()
    n_act = 0
    for t in range(10):
        f = sc.f_ext(t)
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        qo, vo, _, lam, st_o = O.step_forward_contact(osc, q, v, f, con)
        qg, vg, st = g.step_forward(dev(th, q), dev(th, v), dev(th, f))
        assert st["n_contacts"] == len(con[0])
        assert st["iters"] == st_o["iters"], (t, st["iters"], st_o["iters"])
        assert rel(host(qg), qo) < TOL_POS, (t, rel(host(qg), qo))
        n_act += int((lam > 0).sum())
        q, v = qo, vo
    assert n_act > 0


def test_drop_100k_tets_through_contact(th):
    """The drop at about 100k tets (99,730 tets; its 566 MB factor exceeds the
    Infinity Cache) in the benchmark's launch configuration, started with its
    lowest point half a detection distance above the obstacles so that it
    touches at once: four steps from the oracle's own states (rows, iteration
    counts and positions).  The gradient of such a step is the next test."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.drop_blob(res=41, with_box=True)
    (lo, hi) = sc.obstacles["boxes"][0]
    X = sc.X
    over = (X[:, 0] >= lo[0]) & (X[:, 0] <= hi[0]) & (X[:, 1] >= lo[1]) & (X[:, 1] <= hi[1])
    gap = min(X[:, 2].min(), (X[over, 2] - hi[2]).min())
    osc = O.OracleScene(sc)
    g = Scene.from_scene(sc, eps_adj=1e-6, adj_warm=3)
    q = X - np.array([0.0, 0.0, gap - 0.5 * sc.obstacles["d_c"]])
    v = sc.v0()
    n_act = 0
    for t in range(4):
        f = sc.f_ext(t)
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        qo, vo, _, lam, st_o = O.step_forward_contact(osc, q, v, f, con)
        qg, vg, st = g.step_forward(dev(th, q), dev(th, v), dev(th, f))
        assert st["n_contacts"] == len(con[0]) and st["iters"] == st_o["iters"], (t, st, st_o["iters"])
        assert rel(host(qg), qo) < TOL_POS, (t, rel(host(qg), qo))
        n_act = max(n_act, int((lam > 0).sum()))
        q, v = qo, vo
    assert n_act > 0


def test_drop_100k_tets_gradient_through_contact(th):
    """One backward step of the 99,730-tet drop at first touch (rows active),
    from the oracle's own checkpoint data, against the oracle's projected fixed
    point run to a 1e-9 step (its error, about 2e-8 at its contraction rate of
    0.95, is well inside the 1e-6 gradient tolerance)."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.drop_blob(res=41, with_box=True)
    (lo, hi) = sc.obstacles["boxes"][0]
    X = sc.X
    over = (X[:, 0] >= lo[0]) & (X[:, 0] <= hi[0]) & (X[:, 1] >= lo[1]) & (X[:, 1] <= hi[1])
    gap = min(X[:, 2].min(), (X[over, 2] - hi[2]).min())
    osc = O.OracleScene(sc, eps_adj=1e-9, kmax_bwd=5000)
    g = Scene.from_scene(sc, eps_adj=1e-10, adj_warm=3)
    q = X - np.array([0.0, 0.0, gap - 0.5 * sc.obstacles["d_c"]])
    v = sc.v0()
    for t in range(2):
        f = sc.f_ext(t)
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        qo, vo, qm1, lam, st_o = O.step_forward_contact(osc, q, v, f, con)
        ck = g.new_ckpt()
        qg, vg, st = g.step_forward(dev(th, q), dev(th, v), dev(th, f), ckpt=ck)
        assert st["iters"] == st_o["iters"] and rel(host(qg), qo) < TOL_POS, (t, st, st_o["iters"])
        q_t, v_t, qs, qsm1 = q, v, qo, qm1
        q, v = qo, vo
    n_act = int((lam > 0).sum())
    assert n_act > 0
    gq = np.random.Generator(np.random.PCG64(7)).standard_normal(q_t.shape)
    gv = 0.1 * gq
    a = O.step_backward_contact(osc, q_t, v_t, f, qs, qsm1, gq, gv, con, lam, adj_mode=0)
    assert a[4]["status"] == 0
    b = g.step_backward(ck, dev(th, gq), dev(th, gv))
    assert b[4]["n_active"] == n_act
    for x, y in zip(b[:4], a[:4]):
        assert rel(host(x), y) < TOL_GRAD, rel(host(x), y)


def slab_drop(n=14, nz=2, edge=0.02):
    """A flat slab of n x n x nz cubes landing flat on the ground: (n+1)^2 rows at once, more than the LDS
    factorization holds, so the Newton systems and the adjoint's W_AA are factored in the global scratch."""
    X, tets = scenes.box_tet_mesh(n, n, nz, edge)
    X = X + np.array([0.0, 0.0, 0.25 * edge])
    logE = np.full(tets.shape[0], np.log(1e5))
    return scenes.Scene("slab_drop", X, tets, np.zeros(X.shape[0], np.uint8), logE, nu=0.45, rho=1000.0,
                        alpha=0.01, beta0=1.0, h=0.002, gravity=np.array([0.0, 0.0, -9.81]), aa_window=1, steps=8,
                        force_fn=None, target_centroid=X.mean(axis=0) + 0.01,
                        obstacles={"planes": [((0.0, 0.0, 1.0), 0.0)], "boxes": [], "d_c": 0.5 * edge},
                        v_init=np.array([0.0, 0.0, -0.5]))


def test_large_contact_systems(th):
    """225 rows active at once: forward steps and a reverse sweep through them match the oracle."""
    from paper_2605_14526_amd.binding import Scene
    sc = slab_drop()
    osc = O.OracleScene(sc)
    g = Scene.from_scene(sc, eps_adj=1e-12)
    q, v = sc.q0(), sc.v0()
    T = 6
    ck_o, cks, n_act_max = [], [], 0
    for t in range(T):
        f = sc.f_ext(t)
        con = O.detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        qo, vo, qm1, lam, st_o = O.step_forward_contact(osc, q, v, f, con)
        ck = g.new_ckpt()
        qg, vg, st = g.step_forward(dev(th, q), dev(th, v), dev(th, f), ckpt=ck)
        assert st["n_contacts"] == len(con[0]) and st["iters"] == st_o["iters"], (t, st, st_o["iters"])
        assert rel(host(qg), qo) < TOL_POS, (t, rel(host(qg), qo))
        n_act_max = max(n_act_max, int((lam > 0).sum()))
        ck_o.append((q, v, f, qo, qm1, con, lam))
        cks.append(ck)
        q, v = qo, vo
    assert n_act_max > 176
    # one backward step at the last (fully landed) step, from the oracle's own checkpoint data
    q_t, v_t, f, qs, qsm1, con, lam = ck_o[-1]
    gq = np.random.Generator(np.random.PCG64(3)).standard_normal(q_t.shape)
    gv = 0.1 * gq
    a = O.step_backward_contact(osc, q_t, v_t, f, qs, qsm1, gq, gv, con, lam, adj_mode=1)
    b = g.step_backward(cks[-1], dev(th, gq), dev(th, gv))
    assert b[4]["n_active"] > 176
    for x, y in zip(b[:4], a[:4]):
        assert rel(host(x), y) < TOL_GRAD, rel(host(x), y)
