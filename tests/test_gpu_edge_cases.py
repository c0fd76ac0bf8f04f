"""Edge cases through the C ABI: invalid inputs are errors (empty mesh,
repeated vertex, zero-volume tet, stepping a stale factor, unit normals for
obstacles), the smallest mesh (one cube, five tets) and tets given with
negative orientation match the oracle forward and backward, the library's
vertex order, and steps stopped by the iteration cap alternated with
converging steps."""
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


def make(sc, **kw):
    from paper_2605_14526_amd.binding import Scene
    return Scene.from_scene(sc, **kw)


def test_invalid_inputs_are_errors(th):
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.small_beam(2, 1, 1)
    with pytest.raises(RuntimeError, match="PD_ERR_INVALID_ARG"):
        Scene(sc.X, np.zeros((0, 4), np.int32), sc.pinned, np.zeros(0), sc.nu, sc.rho, sc.alpha, sc.beta0, sc.h)
    bad = sc.tets.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(RuntimeError, match="PD_ERR_DEGENERATE_TET"):
        Scene(sc.X, bad, sc.pinned, sc.log_E, sc.nu, sc.rho, sc.alpha, sc.beta0, sc.h)
    X = sc.X.copy()
    t0 = sc.tets[0]
    X[t0[3]] = X[t0[0]] + 0.5 * (X[t0[1]] - X[t0[0]]) + 0.5 * (X[t0[2]] - X[t0[0]])  # flattened tet
    with pytest.raises(RuntimeError, match="PD_ERR_DEGENERATE_TET"):
        Scene(X, sc.tets, sc.pinned, sc.log_E, sc.nu, sc.rho, sc.alpha, sc.beta0, sc.h)
    g = make(sc)
    g.set_material(sc.log_E + 0.1)
    with pytest.raises(RuntimeError, match="PD_ERR_STALE_FACTOR"):
        g.step_forward(dev(th, sc.q0()), dev(th, sc.v0()))
    g.factorize()
    g.step_forward(dev(th, sc.q0()), dev(th, sc.v0()))
    with pytest.raises(RuntimeError, match="PD_ERR_INVALID_ARG"):
        g.set_obstacles({"planes": [((0.0, 0.0, 2.0), 0.0)], "boxes": [], "d_c": 0.1})
    with pytest.raises(RuntimeError, match="PD_ERR_INVALID_ARG"):
        g.set_obstacles({"planes": [], "boxes": [((1.0, 0.0, 0.0), (0.0, 1.0, 1.0))], "d_c": 0.1})


def step_pair(th, sc, T=3):
    """T forward steps and one backward step on the GPU and in the oracle, from the same states."""
    g = make(sc, eps_adj=1e-12)
    o = O.OracleScene(sc)
    q, v = sc.q0(), sc.v0()
    rng = np.random.Generator(np.random.PCG64(4))
    for t in range(T):
        f = sc.f_ext(t)
        ck = g.new_ckpt()
        qg, vg, st = g.step_forward(dev(th, q), dev(th, v), dev(th, f), ckpt=ck)
        qo, vo, qm1, st_o = o.step_forward(q, v, f)
        assert st["iters"] == st_o["iters"]
        assert rel(qg.cpu().numpy(), qo) < 1e-9
        gq, gv = rng.standard_normal(q.shape), rng.standard_normal(q.shape)
        a = g.step_backward(ck, dev(th, gq), dev(th, gv))
        b = o.step_backward(q, v, f, qo, qm1, gq, gv, adj_mode=1)
        for x, y in zip(a[:4], b[:4]):
            assert rel(x.cpu().numpy(), y) < 1e-6
        q, v = qo, vo


def test_single_cube(th):
    sc = scenes.small_beam(1, 1, 1, seed=3, contrast=10.0, tip_force=2.0)
    assert sc.n_e == 5 and sc.n_v == 8
    step_pair(th, sc)


def test_negatively_oriented_tets(th):
    sc = scenes.small_beam(4, 2, 2, seed=9, contrast=20.0, tip_force=5.0)
    flipped = sc.tets.copy()
    flipped[::3, [1, 2]] = flipped[::3, [2, 1]]  # every third tet given inside out
    sc2 = scenes.Scene(**{**sc.__dict__, "tets": flipped})
    step_pair(th, sc2)


def test_permutation_is_the_library_order(th):
    """pd_scene_get_permutation: a permutation of the vertices in which the
    free vertices precede the pinned ones, and the subdomain solve's rows
    precede the interface rows (n_free - n_interface of them)."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.small_beam(7, 3, 3, seed=5, contrast=30.0, nu=0.49)
    g = Scene.from_scene(sc, max_sub=16)
    info = g.info()
    perm = g.permutation()
    nv, nf = int(info["n_verts"]), int(info["n_free"])
    assert perm.shape == (nv,) and np.array_equal(np.sort(perm), np.arange(nv))
    pinned = sc.pinned.astype(bool)
    assert not pinned[perm[:nf]].any() and pinned[perm[nf:]].all()
    assert info["n_subdomains"] > 1 and 0 < info["n_interface"] < nf



def test_capped_step_leaves_no_state_behind(th):
    """A step stopped by the iteration cap (status 1) and a step that converges
    (status 0), alternated on one scene: each call starts from cleared control
    words, so iteration counts, status and positions equal the oracle's with the
    same cap (a loaded beam needs 13 iterations, the cap stops it earlier; the
    unloaded rest state converges under it)."""
    sc = scenes.small_beam(6, 3, 3, seed=2, tip_force=0.0, gravity=(0.0, 0.0, 0.0))
    g = make(sc, kmax_fwd=3)
    o = O.OracleScene(sc, kmax_fwd=3)
    X = sc.X
    z = np.zeros_like(X)
    f = np.zeros_like(X)
    tip = np.abs(X[:, 0] - X[:, 0].max()) < 1e-12
    f[tip, 2] = -40.0 / tip.sum()
    seen = set()
    for ff in (f, z, f, z):
        qo, vo, _, sto = o.step_forward(X, z, ff)
        qg, vg, stg = g.step_forward(dev(th, X), dev(th, z), dev(th, ff))
        assert (stg["iters"], stg["status"]) == (sto["iters"], sto["status"])
        assert rel(qg.cpu().numpy(), qo) < 1e-9
        # at rest both velocities are rounding noise: scale by at least 1 m/s
        # (the loaded step moves the tip at about 0.7 m/s)
        assert np.abs(vg.cpu().numpy() - vo).max() <= 1e-9 * max(np.abs(vo).max(), 1.0)
        seen.add(sto["status"])
    assert seen == {0, 1}
