"""Muscle actuation on the GPU against the oracle (fibre constraints with
per-group activations, read from the paper's muscle-driven scenes whose
inverse problems route through db/da): local step, K apply, forward steps with
path parity through the gate, backward steps including dL/da, the rest state
at zero activation, a 2,500-tet tendon beam rollout and its reverse sweep, and
the argument checks.  All calls go through the C ABI."""
import numpy as np
import pytest

import oracle as O
from paper_2605_14526_amd import scenes

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.fixture(scope="module")
def th(torch_cuda):
    return torch_cuda


def dev(th, a):
    return th.tensor(np.ascontiguousarray(a), dtype=th.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


SMALL = [
    lambda: scenes.tendon_beam(2, 4, layout=0, w_m=2e5, gravity=(0.0, 0.0, -9.81)),
    lambda: scenes.tendon_beam(2, 4, layout=1, w_m=2e5, gravity=(0.0, 0.0, -9.81)),
    lambda: scenes.tendon_beam(3, 8, layout=1, w_m=3e5, aa_window=5, seed=6007),
]


def pair(th, sc, **kw):
    from paper_2605_14526_amd.binding import Scene
    g = Scene.from_scene(sc, **kw)
    o = O.OracleScene(sc, eps_adj=kw.get("eps_adj", 1e-6))
    o.set_muscles(sc.muscle_group, sc.muscle_fibre, sc.muscle_w)
    o.set_activation(sc.activation)
    return g, o


def perturbed(sc, amp, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    q = sc.X + amp * r.standard_normal(sc.X.shape)
    q[sc.pinned.astype(bool)] = sc.X[sc.pinned.astype(bool)]
    return q


@pytest.mark.parametrize("mk", SMALL)
def test_local_rhs_parity(th, mk):
    sc = mk()
    g, o = pair(th, sc)
    free = ~sc.pinned.astype(bool)
    for amp, seed in [(0.0, 1), (2e-3, 2), (1e-2, 3)]:
        q = perturbed(sc, amp, seed)
        b_g = host(g.debug_local_rhs(dev(th, q)))
        b_o = o.local_rhs(q)
        assert rel(b_g[free], b_o[free]) < 1e-11, (amp, rel(b_g[free], b_o[free]))


@pytest.mark.parametrize("mk", SMALL)
def test_apply_Ainv_and_K_parity(th, mk):
    sc = mk()
    g, o = pair(th, sc)
    r = np.random.Generator(np.random.PCG64(23))
    x = r.standard_normal(sc.X.shape)
    assert rel(host(g.debug_apply_Ainv(dev(th, x))), o.apply_Ainv(x)) < 1e-11
    q = perturbed(sc, 5e-3, 29)
    for tau in (0.5, 1.0):
        assert rel(host(g.debug_apply_K(dev(th, q), tau, dev(th, x))), o.apply_K(q, tau, x)) < 1e-10


def test_rest_state_zero_activation(th):
    sc = scenes.tendon_beam(2, 4, layout=1)
    sc.activation = np.zeros(16)
    g, o = pair(th, sc)
    qn, vn, st = g.step_forward(dev(th, sc.X), dev(th, np.zeros_like(sc.X)))
    assert st["iters"] == 2 and st["status"] == 0
    assert rel(host(qn), sc.X) < 1e-14


def forward_pair(th, sc, steps, **kw):
    """Library and oracle steps from the oracle's states, path parity through the gate."""
    g, o = pair(th, sc, **kw)
    q, v = sc.q0(), sc.v0()
    ck, worst, its = [], 0.0, []
    for t in range(steps):
        f = sc.f_ext(t)
        ckpt = g.new_ckpt()
        qg, _, stg = g.step_forward(dev(th, q), dev(th, v), dev(th, f), ckpt=ckpt)
        qo, vo, qm1, sto = o.step_forward(q, v, f)
        assert stg["status"] == 0 and sto["status"] == 0
        qc, qm1c = qo, qm1
        if stg["iters"] != sto["iters"]:
            kg, ko = stg["iters"], sto["iters"]
            qc, _, qm1c, stf = o.step_forward(q, v, f, force_iters=kg)
            gt = (stf if kg < ko else sto)["gate"]
            r = max(gt[0] / (sc.eps_rel * gt[1] + sc.eps_abs), gt[2] / (sc.eps_rel * gt[3] + sc.eps_abs))
            assert abs(r - 1.0) <= 1e-4, (t, kg, ko, r)
        its.append((stg["iters"], sto["iters"]))
        worst = max(worst, rel(host(qg), qc))
        ck.append((q, v, f, qc, qm1c, ckpt))
        q, v = qo, vo
    return g, o, ck, worst, its


@pytest.mark.parametrize("mk", SMALL)
def test_forward_parity(th, mk):
    sc = mk()
    g, o, ck, worst, its = forward_pair(th, sc, 4)
    assert worst < 1e-9, (worst, its)


@pytest.mark.parametrize("mk", SMALL)
@pytest.mark.parametrize("method", [0, 1])
def test_backward_parity_with_activation_gradient(th, mk, method):
    sc = mk()
    eps = 1e-12 if method == 0 else 1e-10
    g, o, ck, worst, its = forward_pair(th, sc, 3, adj_method=method, eps_adj=eps)
    ga = th.zeros(16, dtype=th.float64, device="cuda")
    g.set_activation_grad(ga)
    r = np.random.Generator(np.random.PCG64(31))
    for (q_t, v_t, f, qs, qsm1, ckpt) in ck:
        gq = r.standard_normal(q_t.shape)
        gv = r.standard_normal(q_t.shape)
        ga.zero_()
        o.g_act[:] = 0.0
        res_o = o.step_backward(q_t, v_t, f, qs, qsm1, gq, gv, adj_mode=1)
        res_g = g.step_backward(ckpt, dev(th, gq), dev(th, gv))
        assert res_g[4]["status"] == 0
        for a, b in zip(res_g[:4], res_o[:4]):
            assert rel(host(a), b) < 1e-6, rel(host(a), b)
        assert rel(host(ga), o.g_act) < 1e-6, (host(ga), o.g_act)


def test_tendon_beam_rollout_and_sweep(th):
    """The 2,500-tet tendon beam (16 groups, helical fibres, gravity): eight steps of the library's own
    rollout with the oracle on the same path, and the reverse sweep of a tip loss with dL/da and
    dL/dlog E against the oracle's adjoint run to 1e-13."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.tendon_beam(5, 20, layout=1, gravity=(0.0, 0.0, -9.81))
    T = 8
    g = Scene.from_scene(sc, eps_adj=1e-11, adj_warm=3)
    o = O.OracleScene(sc, eps_adj=1e-13)
    o.set_muscles(sc.muscle_group, sc.muscle_fibre, sc.muscle_w)
    o.set_activation(sc.activation)
    q, v = sc.q0(), sc.v0()
    qg, vg = dev(th, q), dev(th, v)
    cks, ck_o = [], []
    for t in range(T):
        f = sc.f_ext(t)
        ck = g.new_ckpt()
        qg, vg, stg = g.step_forward(qg, vg, dev(th, f), ckpt=ck)
        cks.append(ck)
        qo, vo, qm1, sto = o.step_forward(q, v, f)
        if stg["iters"] != sto["iters"]:
            qo, vo, qm1, _ = o.step_forward(q, v, f, force_iters=stg["iters"])
        assert rel(host(qg), qo) < 1e-9, t
        ck_o.append((q, v, f, qo, qm1))
        q, v = qo, vo
    tip = sc.X[:, 2] > sc.X[:, 2].max() - 1e-9
    gq = np.zeros_like(q)
    gq[tip] = 2.0 * (q[tip].mean(axis=0) - sc.target_centroid) / tip.sum()
    o.g_act[:] = 0.0
    gq0_o, gv0_o, gl_o, _ = O.rollout_backward(o, ck_o, gq, np.zeros_like(gq), adj_mode=0)
    g.adjoint_reset()
    ga = th.zeros(16, dtype=th.float64, device="cuda")
    g.set_activation_grad(ga)
    gqd, gvd = dev(th, gq), dev(th, np.zeros_like(gq))
    gl = th.zeros(sc.n_e, dtype=th.float64, device="cuda")
    for ck in reversed(cks):
        gqd, gvd, _, _, st = g.step_backward(ck, gqd, gvd, g_logE=gl)
        assert st["status"] == 0
    for a, b in [(host(gqd), gq0_o), (host(gvd), gv0_o), (host(gl), gl_o), (host(ga), o.g_act)]:
        assert rel(a, b) < 1e-6, rel(a, b)


def test_argument_checks(th):
    from paper_2605_14526_amd import binding
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.tendon_beam(2, 2, layout=0)
    g = Scene.from_scene(sc)
    bad = sc.muscle_fibre.copy()
    bad[3] *= 1.01
    with pytest.raises(RuntimeError, match="PD_ERR_INVALID_ARG"):
        g.set_muscles(sc.muscle_group, bad, sc.muscle_w)
    grp = sc.muscle_group.copy()
    grp[0] = 99
    with pytest.raises(RuntimeError, match="PD_ERR_INVALID_ARG"):
        binding.check(binding.lib().pd_scene_set_muscles(g.ptr, 16, 1e5, grp.ctypes.data, bad.ctypes.data), "x")
    with pytest.raises(RuntimeError, match="PD_ERR_INVALID_ARG"):
        g.set_muscles(sc.muscle_group, sc.muscle_fibre, -1.0)
    # a batch rejects scenes with muscles
    with pytest.raises(RuntimeError, match="PD_ERR_INVALID_ARG"):
        binding.Batch([Scene.from_scene(sc)])
    # removing the muscles restores the plain scene
    plain = scenes.small_beam(3, 2, 2, seed=1)
    gp = Scene.from_scene(plain)
    gp.set_muscles(np.full(plain.n_e, -1, np.int32), np.zeros((plain.n_e, 3)), 1.0)
    gp.factorize()
    o = O.OracleScene(plain)
    q = perturbed(plain, 1e-3, 5)
    free = ~plain.pinned.astype(bool)
    assert rel(host(gp.debug_local_rhs(dev(th, q)))[free], o.local_rhs(q)[free]) < 1e-11
