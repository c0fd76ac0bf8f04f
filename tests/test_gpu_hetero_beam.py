"""The heterogeneous beam (40x10x10 cubes, 20,000 tets) at the benchmark's own
solver settings against the oracle, and its material gradient against central
finite differences on the 16 seeded tets.  All calls go through the C ABI."""
import numpy as np
import pytest

import oracle as O
from paper_2605_14526_amd import scenes

pytestmark = pytest.mark.gpu

TOL_POS = 1e-9
TOL_GRAD = 1e-6
# see tests/test_gpu_parity.py: the gate ratio's rounding band
GATE_BAND = 1e-4


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.fixture(scope="module")
def th(torch_cuda):
    return torch_cuda


def dev(th, a):
    return th.tensor(np.ascontiguousarray(a), dtype=th.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def gate_ratio(gate, eps_rel, eps_abs):
    return max(gate[0] / (eps_rel * gate[1] + eps_abs), gate[2] / (eps_rel * gate[3] + eps_abs))


def test_benchmark_settings_gradients_match_oracle(th):
    """The benchmark's configuration of the beam: dual gate 1e-6, adjoint PCG
    to the benchmark's tolerance from the quadratically extrapolated start
    (a looser PCG stop left gradients 7e-4 away from the oracle), the 20
    timed steps and
    their reverse sweep with the centroid loss.  The library runs its own
    rollout; the oracle follows the same path (its step re-run at the
    library's iteration count where the gate decided one iteration apart,
    after checking that its gate was within rounding of the threshold) and
    runs its adjoint to 1e-13.  Positions agree to 1e-9, the gradients with
    respect to q0, v0 and all 20,000 log E to 1e-6."""
    import bench
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.config("c2")
    T = 20
    g = Scene.from_scene(sc, eps_adj=bench.ADJ_TOL, adj_warm=3)
    o = O.OracleScene(sc, eps_adj=1e-13)
    q, v = sc.q0(), sc.v0()
    qg, vg = dev(th, q), dev(th, v)
    cks, ck_o, mism = [], [], []
    worst = 0.0
    for t in range(T):
        f = sc.f_ext(t)
        ck = g.new_ckpt()
        qg, vg, stg = g.step_forward(qg, vg, dev(th, f), ckpt=ck)
        assert stg["status"] == 0, stg
        cks.append(ck)
        qo, vo, qm1, sto = o.step_forward(q, v, f)
        if stg["iters"] != sto["iters"]:
            kg, ko = stg["iters"], sto["iters"]
            qo, vo, qm1, stf = o.step_forward(q, v, f, force_iters=kg)
            r = gate_ratio((stf if kg < ko else sto)["gate"], sc.eps_rel, sc.eps_abs)
            assert abs(r - 1.0) <= GATE_BAND, (t, kg, ko, r)
            mism.append((t, kg, ko, r))
        worst = max(worst, rel(host(qg), qo))
        ck_o.append((q, v, f, qo, qm1))
        q, v = qo, vo
    assert worst < TOL_POS, (worst, mism)
    _, gq = scenes.centroid_loss(q, sc.target_centroid)
    gv = np.zeros_like(gq)
    gq0_o, gv0_o, gl_o, _ = O.rollout_backward(o, ck_o, gq, gv, adj_mode=0)
    g.adjoint_reset()
    gqd, gvd = dev(th, gq), dev(th, gv)
    gl = th.zeros(sc.n_e, dtype=th.float64, device="cuda")
    its = []
    for ck in reversed(cks):
        gqd, gvd, _, _, st = g.step_backward(ck, gqd, gvd, g_logE=gl)
        assert st["status"] == 0, st
        its.append(st["adj_iters"])
    for a, b in [(host(gqd), gq0_o), (host(gvd), gv0_o), (host(gl), gl_o)]:
        assert rel(a, b) < TOL_GRAD, (rel(a, b), its, mism)


def _rollout(th, g, sc, T):
    q, v = dev(th, sc.q0()), dev(th, sc.v0())
    cks = []
    for t in range(T):
        ck = g.new_ckpt()
        q, v, st = g.step_forward(q, v, dev(th, sc.f_ext(t)), ckpt=ck)
        assert st["status"] == 0, (t, st)
        cks.append(ck)
    return host(q), cks


def _sweep(th, g, sc, cks, gq):
    g.adjoint_reset()
    gqd, gvd = dev(th, gq), dev(th, np.zeros_like(gq))
    gl = th.zeros(sc.n_e, dtype=th.float64, device="cuda")
    for ck in reversed(cks):
        gqd, gvd, _, _, st = g.step_backward(ck, gqd, gvd, g_logE=gl)
        assert st["status"] == 0, st
    return host(gl)


def test_material_gradient_central_differences_16_tets(th):
    """Sec. 4.8 gradient routing (dL/dlog E_e) against central differences of
    the library's own forward rollout on the 16 seeded tets of the beam
    (step 1e-2 in log E), over the first 40 steps (the tip load's ramp and
    hold), with the mesh means held fixed (they are constants of the
    gradient) and the forward gate and the adjoint run to 1e-12.

    Two losses share the perturbed rollouts.  The centroid loss moves by
    about 1e-12 per perturbation of a single tet, so the rollout's own
    convergence error (gate 1e-12 relative, about 1e-14 in L) leaves an
    absolute noise near 5e-13 in each difference quotient: it is compared to
    1e-3 of the largest quotient and, where a quotient stands 2000 times above
    that noise, to 1e-3 relative.  The local loss <w, q_T> with seeded weights
    on the 16 tets' own vertices has gradients several orders larger than its
    noise: every tet is held to 2e-4 of its own quotient (the step leaves a
    truncation error near 2e-5) plus a noise floor of 3e-6 of the largest
    quotient (the rollout's convergence noise reaches about 1.3e-6 of it in
    the quotients of barely strained tets), and at least six quotients stand
    above 1e-2 of the largest, where the relative term decides."""
    from paper_2605_14526_amd.binding import Scene
    sc = scenes.config("c2")
    T = 40
    g = Scene.from_scene(sc, eps_rel=1e-12, eps_abs=1e-16, eps_adj=1e-12, kmax_fwd=5000, kmax_bwd=5000)
    inf = g.info()
    g.freeze_means((inf["mu_bar"], inf["lam_bar"], inf["mu_ref"]))
    g.set_material(sc.log_E)
    g.factorize()
    rng = np.random.Generator(np.random.PCG64(2005))
    w = np.zeros((sc.n_v, 3))
    verts = np.unique(sc.tets[sc.fd_tets].ravel())
    w[verts] = rng.standard_normal((len(verts), 3))
    qT, cks = _rollout(th, g, sc, T)
    _, gq_c = scenes.centroid_loss(qT, sc.target_centroid)
    ad_c = _sweep(th, g, sc, cks, gq_c)[sc.fd_tets]
    ad_l = _sweep(th, g, sc, cks, w)[sc.fd_tets]
    del cks
    hstep = 1e-2
    fd_c, fd_l = [], []
    for e in sc.fd_tets:
        vc, vl = [], []
        for s in (1.0, -1.0):
            le = sc.log_E.copy()
            le[e] += s * hstep
            g.set_material(le)
            g.factorize()
            q, _ = _rollout(th, g, sc, T)
            vc.append(scenes.centroid_loss(q, sc.target_centroid)[0])
            vl.append(float((w * q).sum()))
        fd_c.append((vc[0] - vc[1]) / (2 * hstep))
        fd_l.append((vl[0] - vl[1]) / (2 * hstep))
    fd_c, fd_l = np.array(fd_c), np.array(fd_l)
    print("fd check: tet, centroid adjoint / difference, local adjoint / difference, local rel. difference")
    for k, e in enumerate(sc.fd_tets.tolist()):
        print(f"  {e:6d} {ad_c[k]: .10e} {fd_c[k]: .10e} {ad_l[k]: .10e} {fd_l[k]: .10e} "
              f"{abs(ad_l[k] - fd_l[k]) / abs(fd_l[k]):.2e}")
    scale = np.abs(fd_c).max()
    assert scale > 0
    assert np.abs(ad_c - fd_c).max() <= 1e-3 * scale
    noise = 5e-13
    big = np.abs(fd_c) >= 2000 * noise
    assert big.sum() >= 1
    assert (np.abs(ad_c - fd_c)[big] <= 1e-3 * np.abs(fd_c)[big]).all()
    # tets in barely strained regions have local gradients 1e-4 of the largest, where the rollout's
    # convergence noise (up to about 1.3e-10 in a quotient here) dominates
    scale_l = np.abs(fd_l).max()
    assert (np.abs(fd_l) >= 1e-2 * scale_l).sum() >= 6
    bound = 2e-4 * np.abs(fd_l) + 3e-6 * scale_l
    assert (np.abs(ad_l - fd_l) <= bound).all(), np.abs(ad_l - fd_l) / bound
