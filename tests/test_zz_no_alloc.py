"""The allocation-free global solve (pd_apply_Ainv_noalloc) against the
solve it mirrors (pd_debug_apply_Ainv) through the C ABI: two calls in a row
on the 20,000-tet beam and then on a smaller beam (the shared static workspace
keeps the first call's contents), and the first scene again."""
import numpy as np
import pytest

from paper_2605_14526_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def th(torch_cuda):
    return torch_cuda


def test_noalloc_solve_matches_allocating_solve(th):
    from paper_2605_14526_amd.binding import Scene
    big = scenes.config("c2")
    small = scenes.small_beam(6, 3, 3, seed=5, contrast=20.0, tip_force=8.0)
    gb = Scene.from_scene(big)
    gs = Scene.from_scene(small)
    rng = np.random.Generator(np.random.PCG64(17))
    for g, sc in [(gb, big), (gs, small), (gb, big)]:
        r = th.tensor(rng.standard_normal((sc.n_v, 3)), dtype=th.float64, device="cuda")
        ref = g.debug_apply_Ainv(r)
        x = th.full_like(r, float("nan"))
        g.apply_Ainv_noalloc(r, x)
        th.cuda.synchronize()
        assert th.isfinite(x).all()
        assert th.equal(x, ref), float((x - ref).abs().max() / ref.abs().max())
        pinned = th.tensor(sc.pinned.astype(bool), device="cuda")
        assert (x[pinned] == 0).all()
