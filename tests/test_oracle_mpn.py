"""Pins of the FP64 reference of the warm-start network (CPU): its gradient
against central differences, permutation equivariance, the edge set, and the
bfloat16 rounding used to feed it the GPU's rounded weights."""
import numpy as np
import pytest

from oracle import mpn as R
from paper_2605_14526_amd import scenes


def tiny_case(seed=0):
    sc = scenes.small_beam(2, 1, 1, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    src, dst = R.mesh_edges(sc.n_v, sc.tets)
    ell, L = R.mesh_constants(sc.X, src, dst)
    q_t = sc.X + 0.01 * rng.standard_normal(sc.X.shape)
    q_tm = sc.X + 0.01 * rng.standard_normal(sc.X.shape)
    v = rng.standard_normal(sc.X.shape)
    f = rng.standard_normal(sc.X.shape)
    mass = rng.uniform(0.5, 1.5, sc.n_v)
    logw = rng.standard_normal(sc.n_v)
    x = R.features(q_t, q_tm, v, f, sc.X, mass, logw, 0.01, ell, L, 1e-3)
    theta = R.init_params(seed + 7)
    # non-zero biases so every term of the gradient is exercised
    theta = theta + 0.05 * rng.standard_normal(theta.shape)
    return sc, x, q_t, src, dst, ell, theta, rng


def test_edges_of_one_tet():
    src, dst = R.mesh_edges(4, np.array([[0, 1, 2, 3]]))
    assert len(src) == 12
    assert set(zip(src.tolist(), dst.tolist())) == {(i, j) for i in range(4) for j in range(4) if i != j}
    assert np.all(np.diff(dst) >= 0)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -2.5, 3.0e-3])
    r = R.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # halfway: ties to even (1.0)
    assert r[2] == 1.0 + 2.0 ** -7           # above halfway rounds up
    assert r[3] == -2.5
    assert abs(r[4] - 3.0e-3) <= 3.0e-3 * 2.0 ** -8


def test_gradient_matches_central_differences():
    sc, x, q_t, src, dst, ell, theta, rng = tiny_case(1)
    c = rng.standard_normal((sc.n_v, 3))
    y, cache = R.forward(theta, x, q_t, sc.X, src, dst, ell)
    g = R.backward(theta, cache, c)
    idx = rng.choice(theta.size, 60, replace=False)
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fp = (R.forward(tp, x, q_t, sc.X, src, dst, ell)[0] * c).sum()
        fm = (R.forward(tm, x, q_t, sc.X, src, dst, ell)[0] * c).sum()
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


@pytest.mark.parametrize("kappa", [0.0, 3.0])
def test_loss_gradient_matches_differences(kappa):
    sc, x, q_t, src, dst, ell, theta, rng = tiny_case(2)
    y, cache = R.forward(theta, x, q_t, sc.X, src, dst, ell)
    tgt = rng.standard_normal(y.shape)
    free = ~sc.pinned.astype(bool)
    L0, dy = R.loss_and_dy(y, tgt, free, src, dst, kappa)
    eps = 1e-6
    for i in range(sc.n_v):
        for a in range(3):
            yp, ym = y.copy(), y.copy()
            yp[i, a] += eps
            ym[i, a] -= eps
            fd = (R.loss_and_dy(yp, tgt, free, src, dst, kappa)[0] - R.loss_and_dy(ym, tgt, free, src, dst, kappa)[0])
            assert abs(fd / (2 * eps) - dy[i, a]) < 1e-7 * max(1.0, abs(dy[i, a])), (i, a)
    # pinned vertices carry no gradient
    assert np.all(dy[~free] == 0.0)


def test_permutation_equivariance():
    sc, x, q_t, src, dst, ell, theta, rng = tiny_case(3)
    y, _ = R.forward(theta, x, q_t, sc.X, src, dst, ell)
    perm = rng.permutation(sc.n_v)          # new vertex k is old vertex perm[k]
    inv = np.argsort(perm)
    tets2 = inv[sc.tets]
    s2, d2 = R.mesh_edges(sc.n_v, tets2)
    y2, _ = R.forward(theta, x[perm], q_t[perm], sc.X[perm], s2, d2, ell)
    assert np.abs(y2 - y[perm]).max() <= 1e-12 * max(1.0, np.abs(y).max())
