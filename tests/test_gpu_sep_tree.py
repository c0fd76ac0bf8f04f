"""The interface solve over the separator tree (Sec. 4.6 in role: one factor,
applied by a forward and a backward sweep).  Every number of tree levels is an
exact solve of A~ x = r, so each is compared with the oracle's solve; a
rollout gives the same states and gradients with one level (one dense
interface inverse) and with eight; a batch whose scenes keep different level
counts gives every scene bitwise what it gives alone."""
import numpy as np
import pytest

import oracle as O
from paper_2605_14526_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def th(torch_cuda):
    return torch_cuda


def dev(th, a):
    return th.tensor(np.ascontiguousarray(a), dtype=th.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


TREE_SCENES = [lambda: scenes.small_beam(24, 3, 3, seed=5, contrast=30.0, nu=0.49),
               lambda: scenes.anchored_blob(2500, seed=31, contrast=50.0, nu=0.47)]


@pytest.mark.parametrize("mk", TREE_SCENES)
@pytest.mark.parametrize("max_sub", [16, 64])
def test_apply_Ainv_every_level_count(th, mk, max_sub):
    """x = A~^{-1} r for 1, 2, 3, 5 and 8 levels against the oracle's solve (1e-11),
    with the residual of A~ x = r on the free vertices."""
    from paper_2605_14526_amd.binding import Scene
    sc = mk()
    o = O.OracleScene(sc)
    rng = np.random.Generator(np.random.PCG64(41))
    r = rng.standard_normal(sc.X.shape)
    x_o = o.apply_Ainv(r)
    free = ~sc.pinned.astype(bool)
    for lv in (1, 2, 3, 5, 8):
        g = Scene.from_scene(sc, max_sub=max_sub, iface_levels=lv)
        print(f"[sep] {sc.name} max_sub {max_sub} levels {lv}", flush=True)
        x_g = host(g.debug_apply_Ainv(dev(th, r)))
        assert rel(x_g, x_o) < 1e-11, (lv, rel(x_g, x_o))
        assert rel(o.apply_A(x_g)[free], r[free]) < 1e-11
        del g


def _rollout(th, g, sc, T):
    q, v = dev(th, sc.q0()), dev(th, sc.v0())
    cks, its = [], []
    for t in range(T):
        ck = g.new_ckpt()
        q, v, st = g.step_forward(q, v, dev(th, sc.f_ext(t)), ckpt=ck)
        assert st["status"] == 0, st
        cks.append(ck)
        its.append(st["iters"])
    g.adjoint_reset()
    gq, gv = dev(th, np.ones_like(sc.X)), dev(th, np.zeros_like(sc.X))
    gl = th.zeros(sc.n_e, dtype=th.float64, device="cuda")
    for ck in reversed(cks):
        gq, gv, _, _, st = g.step_backward(ck, gq, gv, g_logE=gl)
        assert st["status"] == 0, st
    return host(q), host(gq), host(gl), its


def test_rollout_one_level_against_eight(th):
    """Three forward steps and their reverse sweep on a blob of about 2.5k tets cut
    into subdomains of at most 16 vertices: one dense interface inverse and the
    eight-level tree give the same iterations, positions (1e-11) and gradients
    (1e-9), and the tree's positions match the oracle's (1e-9)."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.anchored_blob(2500, seed=31, contrast=50.0, nu=0.47)
    T = 3
    kw = dict(max_sub=16, eps_adj=1e-12, adj_warm=0)
    a = _rollout(th, Scene.from_scene(sc, iface_levels=1, **kw), sc, T)
    b = _rollout(th, Scene.from_scene(sc, iface_levels=8, **kw), sc, T)
    assert a[3] == b[3]
    assert rel(b[0], a[0]) < 1e-11
    assert rel(b[1], a[1]) < 1e-9
    assert rel(b[2], a[2]) < 1e-9
    o = O.OracleScene(sc)
    q, v = sc.q0(), sc.v0()
    for t in range(T):  # the oracle takes the library's iteration count of each step
        q, v, _, _ = o.step_forward(q, v, sc.f_ext(t), force_iters=b[3][t])
    assert rel(b[0], q) < 1e-9


def test_batch_with_different_level_counts_is_bitwise(th):
    """Scenes with 1, 3 and 8 interface levels in one batch: each gives bitwise the
    states, iterations and gradients it gives alone."""
    from paper_2605_14526_amd.binding import Batch, Scene
    scs = [scenes.small_beam(12, 3, 3, seed=5, contrast=30.0, nu=0.49, aa_window=1),
           scenes.anchored_blob(1500, seed=21, contrast=50.0, nu=0.47),
           scenes.small_beam(16, 2, 2, seed=8, contrast=3.0, nu=0.45, aa_window=5)]
    levels = [1, 3, 8]
    T = 3
    alone = [_rollout(th, Scene.from_scene(sc, max_sub=32, iface_levels=lv, adj_warm=2), sc, T)
             for sc, lv in zip(scs, levels)]
    gs = [Scene.from_scene(sc, max_sub=32, iface_levels=lv, adj_warm=2) for sc, lv in zip(scs, levels)]
    B = Batch(gs)
    q = [dev(th, sc.q0()) for sc in scs]
    v = [dev(th, sc.v0()) for sc in scs]
    cks, its = [], []
    for t in range(T):
        ck = [g.new_ckpt() for g in gs]
        q, v, stats, rc = B.step_forward(q, v, [dev(th, sc.f_ext(t)) for sc in scs], ckpt=ck)
        assert rc == 0
        cks.append(ck)
        its.append([s_["iters"] for s_ in stats])
    for g in gs:
        g.adjoint_reset()
    gq = [dev(th, np.ones_like(sc.X)) for sc in scs]
    gv = [dev(th, np.zeros_like(sc.X)) for sc in scs]
    gl = [th.zeros(sc.n_e, dtype=th.float64, device="cuda") for sc in scs]
    for ck in reversed(cks):
        gq, gv, _, gl, _, rc = B.step_backward(ck, gq, gv, g_logE=gl)
        assert rc == 0
    for i, a in enumerate(alone):
        assert a[3] == [it[i] for it in its]
        assert np.array_equal(a[0], host(q[i]))
        assert np.array_equal(a[1], host(gq[i]))
        assert np.array_equal(a[2], host(gl[i]))


def test_iface_levels_out_of_range(th):
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.small_beam(4, 2, 2, seed=3)
    for lv in (-1, 9):
        with pytest.raises(RuntimeError, match="PD_ERR_INVALID_ARG"):
            Scene.from_scene(sc, iface_levels=lv)
