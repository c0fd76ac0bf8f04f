"""GPU parity of the HIP path against the FP64 CPU oracle (stage by stage, then
whole forward and backward steps).  All calls go through the C ABI."""
import copy

import numpy as np
import pytest

import oracle as O
from paper_2605_14526_amd import scenes

pytestmark = pytest.mark.gpu

# tolerances of the hot-path contract: positions 1e-9 relative, gradients 1e-6
# relative; single stages are held tighter (they differ only by rounding order).
TOL_STAGE = 1e-11
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


def make_pair(sc, **kw):
    from paper_2605_14526_amd.binding import Scene
    g = Scene.from_scene(sc, **kw)
    o = O.OracleScene(sc, eps_adj=kw.get("eps_adj", 1e-6), kmax_bwd=kw.get("kmax_bwd", 1000))
    return g, o


def perturbed(sc, amp, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    q = sc.X + amp * rng.standard_normal(sc.X.shape)
    q[sc.pinned.astype(bool)] = sc.X[sc.pinned.astype(bool)]
    return q


SMALL = [
    lambda: scenes.small_beam(4, 2, 2, seed=3),
    lambda: scenes.small_beam(7, 3, 3, seed=5, contrast=30.0, nu=0.49),
    lambda: scenes.small_beam(10, 4, 3, seed=11, contrast=1.0, aa_window=5, alpha=0.0, beta_rel=0.0),
]


@pytest.mark.parametrize("mk", SMALL)
@pytest.mark.parametrize("max_sub", [0, 16])
def test_local_rhs_parity(th, mk, max_sub):
    sc = mk()
    g, o = make_pair(sc, max_sub=max_sub)
    free = ~sc.pinned.astype(bool)
    for amp, seed in [(0.0, 1), (2e-3, 2), (1e-2, 3)]:
        q = perturbed(sc, amp, seed)
        b_g = host(g.debug_local_rhs(dev(th, q)))
        b_o = o.local_rhs(q)
        assert rel(b_g[free], b_o[free]) < TOL_STAGE, (amp, rel(b_g[free], b_o[free]))
        assert np.all(b_g[~free] == 0.0)


@pytest.mark.parametrize("mk", SMALL)
@pytest.mark.parametrize("max_sub", [0, 16, 7])
def test_apply_Ainv_parity(th, mk, max_sub):
    sc = mk()
    g, o = make_pair(sc, max_sub=max_sub)
    rng = np.random.Generator(np.random.PCG64(17))
    r = rng.standard_normal(sc.X.shape)
    x_g = host(g.debug_apply_Ainv(dev(th, r)))
    x_o = o.apply_Ainv(r)
    assert rel(x_g, x_o) < TOL_STAGE
    # A x = r on free vertices
    free = ~sc.pinned.astype(bool)
    assert rel(o.apply_A(x_g)[free], r[free]) < 1e-11


@pytest.mark.parametrize("mk", SMALL)
@pytest.mark.parametrize("tau", [0.5, 1.0])
def test_apply_K_parity(th, mk, tau):
    sc = mk()
    g, o = make_pair(sc)
    rng = np.random.Generator(np.random.PCG64(23))
    q = perturbed(sc, 5e-3, 29)
    x = rng.standard_normal(sc.X.shape)
    y_g = host(g.debug_apply_K(dev(th, q), tau, dev(th, x)))
    y_o = o.apply_K(q, tau, x)
    assert rel(y_g, y_o) < 1e-10


def test_rest_state(th):
    """At rest with no load every iterate equals X and the gate fires after two solves."""
    sc = scenes.small_beam(6, 3, 3, seed=2, tip_force=0.0, gravity=(0.0, 0.0, 0.0))
    g, o = make_pair(sc)
    qn, vn, st = g.step_forward(dev(th, sc.X), dev(th, np.zeros_like(sc.X)))
    assert st["iters"] == 2 and st["status"] == 0
    assert rel(host(qn), sc.X) < 1e-14


def run_pair(th, sc, steps, **kw):
    g, o = make_pair(sc, **kw)
    q, v = sc.q0(), sc.v0()
    qg, vg = dev(th, q), dev(th, v)
    ck = []
    worst = 0.0
    iters = []
    for t in range(steps):
        f = sc.f_ext(t)
        ckpt = g.new_ckpt()
        qg2, vg2, stg = g.step_forward(qg, vg, dev(th, f), ckpt=ckpt)
        qo, vo, qm1, sto = o.step_forward(q, v, f)
        iters.append((stg["iters"], sto["iters"]))
        assert stg["status"] == 0 and sto["status"] == 0
        ck.append((q, v, f, qo, qm1, ckpt))
        if stg["iters"] == sto["iters"]:
            worst = max(worst, rel(host(qg2), qo))
        q, v, qg, vg = qo, vo, dev(th, qo), dev(th, vo)
    return g, o, ck, worst, iters


@pytest.mark.parametrize("mk", SMALL)
def test_forward_parity(th, mk):
    sc = mk()
    g, o, ck, worst, iters = run_pair(th, sc, 4)
    same = sum(a == b for a, b in iters)
    assert same >= len(iters) - 1, iters
    assert worst < TOL_POS, worst


def test_forward_parity_c1(th):
    sc = scenes.cantilever_c1()
    g, o, ck, worst, iters = run_pair(th, sc, 5)
    assert sum(a == b for a, b in iters) >= 4, iters
    assert worst < TOL_POS, (worst, iters)


@pytest.mark.parametrize("mk", SMALL)
@pytest.mark.parametrize("method", [0, 1])
def test_backward_parity(th, mk, method):
    sc = mk()
    eps = 1e-12 if method == 0 else 1e-10
    g, o, ck, worst, iters = run_pair(th, sc, 3, adj_method=method, eps_adj=eps)
    rng = np.random.Generator(np.random.PCG64(31))
    for (q_t, v_t, f, qs, qsm1, ckpt) in ck:
        gq = rng.standard_normal(q_t.shape)
        gv = rng.standard_normal(q_t.shape)
        gq_o, gv_o, gf_o, gl_o, st_o = o.step_backward(q_t, v_t, f, qs, qsm1, gq, gv, adj_mode=1)
        gq_g, gv_g, gf_g, gl_g, st_g = g.step_backward(ckpt, dev(th, gq), dev(th, gv))
        assert st_g["status"] == 0, st_g
        assert st_g["tau"] == st_o["tau"]
        for a, b in [(gq_g, gq_o), (gv_g, gv_o), (gf_g, gf_o), (gl_g, gl_o)]:
            assert rel(host(a), b) < TOL_GRAD, (rel(host(a), b), st_g, st_o)
