"""ctypes binding of the plain FP64 CPU oracle (``pd_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  The product path (the HIP library and its
Python binding) never imports this package.

Position vectors are numpy arrays of shape (n_v, 3) in the scene's original
vertex order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pd_oracle.c")
_LIB = os.path.join(_HERE, "libpdoracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE FP64: no fast-math, no FMA contraction; OpenMP over
    elements with fixed summation orders)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.or_scene_create.restype = ctypes.c_void_p
        L.or_scene_create.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _ip, ctypes.c_char_p, _dp, _dp, _dp]
        L.or_scene_destroy.argtypes = [ctypes.c_void_p]
        L.or_scene_nfree.argtypes = [ctypes.c_void_p]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_get_threads.restype = ctypes.c_int
        L.or_scene_info.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp]
        L.or_scene_set_muscles.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _ip, _dp]
        L.or_scene_set_activation.argtypes = [ctypes.c_void_p, _dp]
        L.or_scene_set_act_grad.argtypes = [ctypes.c_void_p, _dp]
        L.or_svd3.argtypes = [_dp, _dp, _dp, _dp]
        L.or_prox_stretch.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        L.or_prox_map.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        L.or_prox_jacobian.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        L.or_psi_nh.restype = ctypes.c_double
        L.or_psi_nh.argtypes = [_dp, ctypes.c_double, ctypes.c_double]
        L.or_sym3_eig.argtypes = [_dp, _dp, _dp]
        L.or_volume_project.argtypes = [_dp, _dp]
        L.or_volume_diff.argtypes = [_dp, _dp]
        L.or_composite_map.argtypes = [_dp, ctypes.c_double, ctypes.c_double, _dp]
        L.or_composite_jacobian.argtypes = [_dp, ctypes.c_double, ctypes.c_double, _dp]
        L.or_logvol_stretch.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        L.or_logvol_map.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        L.or_logvol_jacobian.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         _dp]
        L.or_tr_filter.argtypes = [_dp, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.or_aa_step.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _ip, _dp, _dp, ctypes.c_char_p, _dp, _dp]
        L.or_local_rhs.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.or_const_rhs.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp]
        L.or_apply_Ainv.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.or_apply_A.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.or_apply_K.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, _dp, _dp]
        L.or_primal_phi.restype = ctypes.c_double
        L.or_primal_phi.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.or_step_forward.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, _dp, _ip, _dp]
        L.or_step_backward.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                       ctypes.c_int, ctypes.c_double, _ip, _dp]
        L.or_step_forward_contact.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, _ip,
                                              _dp, _dp, ctypes.c_double, _dp, _ip, _dp]
        L.or_step_backward_contact.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                               _dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _ip, _dp, _dp, _dp,
                                               _ip, _dp]
        L.or_contact_W.argtypes = [ctypes.c_void_p, ctypes.c_int, _ip, _dp, _dp]
        L.or_fb_lcp.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp]
        L.or_step_forward_friction.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int,
                                               _ip, _dp, _dp, ctypes.c_double, ctypes.c_double, _dp, ctypes.c_int,
                                               _ip, _dp]
        L.or_step_backward_friction.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                                _dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _ip, _dp, _dp,
                                                ctypes.c_double, _dp, _ip, _dp]
        L.or_contact_frame.argtypes = [_dp, _dp, _dp]
        L.or_step_forward_contact_ext.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int,
                                                  _ip, _dp, _dp, ctypes.c_char_p, ctypes.c_int, ctypes.c_double,
                                                  ctypes.c_double, ctypes.c_double, _dp, ctypes.c_int, _ip, _dp]
        L.or_step_backward_contact_ext.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                                   _dp, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _ip, _dp,
                                                   _dp, ctypes.c_char_p, ctypes.c_int, ctypes.c_double,
                                                   ctypes.c_double, _dp, _dp, _ip, _dp]
        L.or_friction_ncp.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, _dp, _dp]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's element loops (OpenMP); results are independent of it."""
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _f(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- element level
def svd3(F):
    F = _f(F).reshape(3, 3)
    U, S, V = np.zeros((3, 3)), np.zeros(3), np.zeros((3, 3))
    lib().or_svd3(_p(F), _p(U), _p(S), _p(V))
    return U, S, V


def prox_stretch(sF, mu, lam, k):
    sF = _f(sF)
    out = np.zeros(3)
    it = lib().or_prox_stretch(_p(sF), mu, lam, k, _p(out))
    return out, it


def prox_map(F, mu, lam, k):
    F = _f(F).reshape(3, 3)
    P = np.zeros((3, 3))
    lib().or_prox_map(_p(F), mu, lam, k, _p(P))
    return P


def prox_jacobian(F, mu, lam, k, tau):
    F = _f(F).reshape(3, 3)
    J = np.zeros((9, 9))
    lib().or_prox_jacobian(_p(F), mu, lam, k, tau, _p(J))
    return J


def psi_nh(F, mu, lam):
    return lib().or_psi_nh(_p(_f(F).reshape(3, 3)), mu, lam)


def volume_project(sF):
    s = np.zeros(3)
    it = lib().or_volume_project(_p(_f(sF)), _p(s))
    return s, it


def volume_diff(sF):
    D = np.zeros((3, 3))
    lib().or_volume_diff(_p(_f(sF)), _p(D))
    return D


def composite_map(F, mu, lam):
    P = np.zeros((3, 3))
    lib().or_composite_map(_p(_f(F).reshape(3, 3)), mu, lam, _p(P))
    return P


def composite_jacobian(F, mu, lam):
    J = np.zeros((9, 9))
    lib().or_composite_jacobian(_p(_f(F).reshape(3, 3)), mu, lam, _p(J))
    return J


def logvol_stretch(sF, mu, lam, k):
    s = np.zeros(3)
    it = lib().or_logvol_stretch(_p(_f(sF)), mu, lam, k, _p(s))
    return s, it


def logvol_map(F, mu_bar, lam_bar, mu, lam):
    P = np.zeros((3, 3))
    lib().or_logvol_map(_p(_f(F)), mu_bar, lam_bar, mu, lam, _p(P))
    return P


def logvol_jacobian(F, mu_bar, lam_bar, mu, lam):
    J = np.zeros((9, 9))
    lib().or_logvol_jacobian(_p(_f(F)), mu_bar, lam_bar, mu, lam, _p(J))
    return J


def sym3_eig(H):
    H = _f(H).reshape(3, 3)
    k, Q = np.zeros(3), np.zeros((3, 3))
    lib().or_sym3_eig(_p(H), _p(k), _p(Q))
    return k, Q


def tr_filter(H, tau, k=1.0):
    H = _f(H).reshape(3, 3)
    Ht, Dinv = np.zeros((3, 3)), np.zeros((3, 3))
    lib().or_tr_filter(_p(H), float(tau), float(k), _p(Ht), _p(Dinv))
    return Ht, Dinv


class AAHistory:
    """Anderson history for :func:`aa_step` on vectors of length n."""

    def __init__(self, n, m):
        self.n, self.m = n, m
        self.Hq = np.zeros((m + 1, n))
        self.Hg = np.zeros((m + 1, n))
        self.hn = ctypes.c_int(0)

    def step(self, q, qhat, mask=None):
        qn = np.zeros(self.n)
        gam = np.zeros(8)
        mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        reset = lib().or_aa_step(self.n, self.m, _p(self.Hq), _p(self.Hg), ctypes.byref(self.hn), _p(_f(q)),
                                 _p(_f(qhat)), mk.ctypes.data_as(ctypes.c_char_p) if mk is not None else None,
                                 _p(qn), _p(gam))
        return qn, bool(reset), gam


# ---------------------------------------------------------------- scene level
class OracleScene:
    """Oracle scene built from a :class:`paper_2605_14526_amd.scenes.Scene`-like object."""

    def __init__(self, sc, m=None, eps_rel=None, eps_abs=None, kmax_fwd=1000, kmax_bwd=1000, eps_adj=1e-6,
                 eps_tr=0.1, log_E=None, frozen=None, energy=None):
        L = lib()
        self.sc = sc
        self.nv = int(sc.X.shape[0])
        self.ne = int(sc.tets.shape[0])
        X = _f(sc.X)
        tets = np.ascontiguousarray(sc.tets, dtype=np.int32)
        pinned = np.ascontiguousarray(sc.pinned, dtype=np.uint8)
        logE = _f(sc.log_E if log_E is None else log_E)
        g = np.asarray(sc.gravity, float)
        params = _f([sc.nu, sc.rho, sc.alpha, sc.beta0, sc.h, g[0], g[1], g[2]])
        fr = (0.0, 0.0, 0.0) if frozen is None else tuple(frozen)
        solver = _f([sc.aa_window if m is None else m, sc.eps_rel if eps_rel is None else eps_rel,
                     sc.eps_abs if eps_abs is None else eps_abs, kmax_fwd, kmax_bwd, eps_adj, eps_tr,
                     fr[0], fr[1], fr[2], getattr(sc, "energy", 0) if energy is None else energy])
        self.h = float(sc.h)
        self._keep = (X, tets, pinned, logE, params, solver)
        self.ptr = L.or_scene_create(self.nv, self.ne, _p(X), tets.ctypes.data_as(_ip),
                                     pinned.ctypes.data_as(ctypes.c_char_p), _p(logE), _p(params), _p(solver))
        self.nf = L.or_scene_nfree(self.ptr)
        self.pinned = pinned.astype(bool)

    def set_muscles(self, group, fibre, w_m):
        """Muscle fibres (reading in pd_oracle.c): group per tet (-1 passive), unit fibre per tet, weight w_m.
        Reassembles and refactors A~; activations start at 0; the activation gradient accumulates into
        ``self.g_act`` (zeroed here)."""
        group = np.ascontiguousarray(group, dtype=np.int32)
        fibre = _f(fibre).reshape(self.ne, 3)
        self.n_groups = int(group.max()) + 1 if group.size and group.max() >= 0 else 0
        self._mkeep = (group, fibre)
        lib().or_scene_set_muscles(self.ptr, self.n_groups, float(w_m), group.ctypes.data_as(_ip), _p(fibre))
        self.g_act = np.zeros(max(self.n_groups, 1))
        lib().or_scene_set_act_grad(self.ptr, _p(self.g_act))

    def set_activation(self, a):
        self._akeep = _f(a)
        assert self._akeep.shape == (self.n_groups,)
        lib().or_scene_set_activation(self.ptr, _p(self._akeep))

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().or_scene_destroy(self.ptr)
            self.ptr = None

    def info(self):
        vol, w, beta, mass, means = np.zeros(self.ne), np.zeros(self.ne), np.zeros(self.ne), np.zeros(self.nv), np.zeros(4)
        lib().or_scene_info(self.ptr, _p(vol), _p(w), _p(beta), _p(mass), _p(means))
        return dict(vol=vol, w=w, beta=beta, mass=mass, mu_bar=means[0], lam_bar=means[1], k_bar=means[2],
                    mu_ref=means[3])

    def local_rhs(self, q):
        q = _f(q)
        b = np.zeros_like(q)
        lib().or_local_rhs(self.ptr, _p(q), _p(b))
        return b

    def const_rhs(self, q_t, v_t, f_ext=None):
        q_t, v_t = _f(q_t), _f(v_t)
        c, qt = np.zeros_like(q_t), np.zeros_like(q_t)
        lib().or_const_rhs(self.ptr, _p(q_t), _p(v_t), _p(_f(f_ext)) if f_ext is not None else None, _p(c), _p(qt))
        return c, qt

    def apply_Ainv(self, r):
        r = _f(r)
        x = np.zeros_like(r)
        lib().or_apply_Ainv(self.ptr, _p(r), _p(x))
        return x

    def apply_A(self, x):
        x = _f(x)
        y = np.zeros_like(x)
        lib().or_apply_A(self.ptr, _p(x), _p(y))
        return y

    def apply_K(self, q, tau, x):
        q, x = _f(q), _f(x)
        y = np.zeros_like(x)
        lib().or_apply_K(self.ptr, _p(q), tau, _p(x), _p(y))
        return y

    def phi(self, q, qtilde):
        return lib().or_primal_phi(self.ptr, _p(_f(q)), _p(_f(qtilde)))

    def step_forward(self, q_t, v_t, f_ext=None, q0=None, force_iters=0, m=-1, record=0):
        q_t, v_t = _f(q_t), _f(v_t)
        qn, vn, qm1 = np.zeros_like(q_t), np.zeros_like(q_t), np.zeros_like(q_t)
        ist = np.zeros(5, dtype=np.int32)
        dst = np.zeros(4)
        rec = np.zeros((record,) + q_t.shape) if record else None
        lib().or_step_forward(self.ptr, _p(q_t), _p(v_t), _p(_f(f_ext)) if f_ext is not None else None,
                              _p(_f(q0)) if q0 is not None else None, _p(qn), _p(vn), _p(qm1), int(force_iters),
                              int(m), int(record), _p(rec) if rec is not None else None,
                              ist.ctypes.data_as(_ip), _p(dst))
        st = dict(iters=int(ist[0]), resets=int(ist[1]), newton_capped=int(ist[2]), newton_max=int(ist[3]),
                  status=int(ist[4]), gate=dst.copy())
        if record:
            st["record"] = rec
        return qn, vn, qm1, st

    def step_backward(self, q_t, v_t, f_ext, q_star, q_star_m1, gq_next, gv_next, g_logE=None, adj_mode=0,
                      tau_force=-1.0):
        q_t, v_t = _f(q_t), _f(v_t)
        gq, gv, gf = np.zeros_like(q_t), np.zeros_like(q_t), np.zeros_like(q_t)
        gl = np.zeros(self.ne) if g_logE is None else g_logE
        ist = np.zeros(2, dtype=np.int32)
        dst = np.zeros(4)
        lib().or_step_backward(self.ptr, _p(q_t), _p(v_t), _p(_f(f_ext)) if f_ext is not None else None,
                               _p(_f(q_star)), _p(_f(q_star_m1)), _p(_f(gq_next)), _p(_f(gv_next)), _p(gq), _p(gv),
                               _p(gf), _p(gl), int(adj_mode), float(tau_force), ist.ctypes.data_as(_ip), _p(dst))
        st = dict(adj_iters=int(ist[0]), status=int(ist[1]), rho=dst[0], tau=dst[1], dphi_act=dst[2],
                  dphi_mod=dst[3])
        return gq, gv, gf, gl, st


# ---------------------------------------------------------------- contact
def _obstacle_faces(obs):
    """Half-spaces (n, o) with n.x - o = signed distance: every plane, then each box's six outward faces
    in the order -x, +x, -y, +y, -z, +z; returns (list of (n, o), list of obstacle ids)."""
    faces = []
    for (n, o) in obs.get("planes", []):
        faces.append([(np.asarray(n, float), float(o))])
    for (lo, hi) in obs.get("boxes", []):
        lo, hi = np.asarray(lo, float), np.asarray(hi, float)
        fl = []
        for a in range(3):
            e = np.zeros(3)
            e[a] = -1.0
            fl.append((e, -lo[a]))
            e = np.zeros(3)
            e[a] = 1.0
            fl.append((e, hi[a]))
        faces.append(fl)
    return faces


def detect_contacts(q_t, v_t, h, pinned, obs, one_per_vertex=False):
    """Contact rows for one step (frictionless reading of Sec. 4.7): for each free vertex (in vertex order)
    and each obstacle (planes first, then boxes), the obstacle's distance d(x) (a plane's signed distance;
    for a box the largest signed distance over its six faces) is evaluated at x0 = q_t and at the inertial
    prediction x1 = q_t + h v_t; the pair is a row if min(d(x0), d(x1)) < d_c.  Its normal and offset are
    those of the face that attains the maximum at x0 (the first such face on ties).  With
    one_per_vertex (the frictional reading: a contact carries a full frame, so two on one vertex would be
    redundant) a vertex keeps only the qualifying obstacle with the smallest distance at x0 (the first on
    ties).  Returns int32 vertex ids, normals (K, 3) and offsets (K,)."""
    dc = float(obs["d_c"])
    faces = _obstacle_faces(obs)
    cv, cn, cg = [], [], []
    for v in range(q_t.shape[0]):
        if pinned[v]:
            continue
        x0 = q_t[v]
        x1 = q_t[v] + h * v_t[v]
        best = None
        for fl in faces:
            d0 = [float(n[0] * x0[0] + n[1] * x0[1] + n[2] * x0[2] - o) for (n, o) in fl]
            d1 = [float(n[0] * x1[0] + n[1] * x1[1] + n[2] * x1[2] - o) for (n, o) in fl]
            i0 = int(np.argmax(d0))
            if min(max(d0), max(d1)) < dc:
                if one_per_vertex:
                    if best is None or max(d0) < best[0]:
                        best = (max(d0), fl[i0])
                    continue
                cv.append(v)
                cn.append(fl[i0][0])
                cg.append(fl[i0][1])
        if best is not None:
            cv.append(v)
            cn.append(best[1][0])
            cg.append(best[1][1])
    return (np.asarray(cv, dtype=np.int32), np.asarray(cn, dtype=np.float64).reshape(-1, 3),
            np.asarray(cg, dtype=np.float64))


def fb_lcp(W, dfree):
    """The oracle's FB-Newton solve of the LCP (delta = dfree + W lambda) alone."""
    W = _f(W)
    d = _f(dfree)
    K = d.shape[0]
    lam = np.zeros(K)
    res = ctypes.c_double(0.0)
    it = lib().or_fb_lcp(K, _p(W), _p(d), _p(lam), ctypes.byref(res))
    return lam, it, res.value


def contact_W(osc, cv, cn):
    cv = np.ascontiguousarray(cv, dtype=np.int32)
    cn = _f(cn)
    K = cv.shape[0]
    W = np.zeros((K, K))
    lib().or_contact_W(osc.ptr, K, cv.ctypes.data_as(_ip), _p(cn), _p(W))
    return W


def step_forward_contact(osc, q_t, v_t, f_ext, contacts, fb_tol=1e-10):
    """One forward step with a given contact set (cv, cn, cg); returns q, v, q*_-1, lambda, stats."""
    cv, cn, cg = contacts
    cv = np.ascontiguousarray(cv, dtype=np.int32)
    cn, cg = _f(cn), _f(cg)
    q_t, v_t = _f(q_t), _f(v_t)
    K = cv.shape[0]
    qn, vn, qm1 = np.zeros_like(q_t), np.zeros_like(q_t), np.zeros_like(q_t)
    lam = np.zeros(max(K, 1))
    ist = np.zeros(5, dtype=np.int32)
    dst = np.zeros(5)
    lib().or_step_forward_contact(osc.ptr, _p(q_t), _p(v_t), _p(_f(f_ext)) if f_ext is not None else None, None,
                                  _p(qn), _p(vn), _p(qm1), K, cv.ctypes.data_as(_ip), _p(cn), _p(cg),
                                  float(fb_tol), _p(lam), ist.ctypes.data_as(_ip), _p(dst))
    st = dict(iters=int(ist[0]), resets=int(ist[1]), newton_capped=int(ist[2]), newton_max=int(ist[3]),
              status=int(ist[4]), gate=dst[:4].copy(), fb_res=float(dst[4]), n_contacts=K,
              n_active=int((lam[:K] > 0).sum()))
    return qn, vn, qm1, lam[:K].copy(), st


def step_backward_contact(osc, q_t, v_t, f_ext, q_star, q_star_m1, gq_next, gv_next, contacts, lam, g_logE=None,
                          adj_mode=0, tau_force=-1.0):
    cv, cn, cg = contacts
    cv = np.ascontiguousarray(cv, dtype=np.int32)
    cn, cg = _f(cn), _f(cg)
    K = cv.shape[0]
    q_t, v_t = _f(q_t), _f(v_t)
    gq, gv, gf = np.zeros_like(q_t), np.zeros_like(q_t), np.zeros_like(q_t)
    gl = np.zeros(osc.ne) if g_logE is None else g_logE
    ist = np.zeros(2, dtype=np.int32)
    dst = np.zeros(4)
    lam = _f(lam if K else np.zeros(1))
    lib().or_step_backward_contact(osc.ptr, _p(q_t), _p(v_t), _p(_f(f_ext)) if f_ext is not None else None,
                                   _p(_f(q_star)), _p(_f(q_star_m1)), _p(_f(gq_next)), _p(_f(gv_next)), _p(gq),
                                   _p(gv), _p(gf), _p(gl), int(adj_mode), float(tau_force), K,
                                   cv.ctypes.data_as(_ip), _p(cn), _p(cg), _p(lam), ist.ctypes.data_as(_ip),
                                   _p(dst))
    st = dict(adj_iters=int(ist[0]), status=int(ist[1]), rho=dst[0], tau=dst[1], dphi_act=dst[2],
              dphi_mod=dst[3])
    return gq, gv, gf, gl, st


def contact_frame(n):
    """The oracle's tangent frame (t1, t2) of a unit normal."""
    n = _f(n)
    t1, t2 = np.zeros(3), np.zeros(3)
    lib().or_contact_frame(_p(n), _p(t1), _p(t2))
    return t1, t2


def friction_ncp(G, normals, u0, mu):
    """The oracle's friction Newton alone: G (K x K), normals (K, 3), free kinematics u0 (K, 3: gap, slip
    along t1, t2); returns impulses (K, 3: normal, t1, t2), Newton steps and the final residual."""
    G, normals, u0 = _f(G), _f(normals), _f(u0)
    K = G.shape[0]
    lam = np.zeros((max(K, 1), 3))
    res = ctypes.c_double(0.0)
    it = lib().or_friction_ncp(K, _p(G), _p(normals), _p(u0), float(mu), _p(lam), ctypes.byref(res))
    return lam[:K].copy(), it, res.value


def step_forward_friction(osc, q_t, v_t, f_ext, contacts, mu_f, fb_tol=1e-10, force_iters=0, q0=None):
    """One forward step with Coulomb friction on a given contact set; returns q, v, q*_-1, impulses (K, 3)
    and stats."""
    cv, cn, cg = contacts
    cv = np.ascontiguousarray(cv, dtype=np.int32)
    cn, cg = _f(cn), _f(cg)
    q_t, v_t = _f(q_t), _f(v_t)
    K = cv.shape[0]
    qn, vn, qm1 = np.zeros_like(q_t), np.zeros_like(q_t), np.zeros_like(q_t)
    lam = np.zeros((max(K, 1), 3))
    ist = np.zeros(5, dtype=np.int32)
    dst = np.zeros(6)
    lib().or_step_forward_friction(osc.ptr, _p(q_t), _p(v_t), _p(_f(f_ext)) if f_ext is not None else None,
                                   _p(_f(q0)) if q0 is not None else None, _p(qn), _p(vn), _p(qm1), K,
                                   cv.ctypes.data_as(_ip), _p(cn), _p(cg), float(mu_f), float(fb_tol), _p(lam),
                                   int(force_iters), ist.ctypes.data_as(_ip), _p(dst))
    st = dict(iters=int(ist[0]), resets=int(ist[1]), newton_capped=int(ist[2]), newton_max=int(ist[3]),
              status=int(ist[4]), gate=dst[:4].copy(), fb_res=float(dst[4]), fb_iters=int(dst[5]),
              n_contacts=K, n_active=int((lam[:K, 0] > 0).sum()))
    return qn, vn, qm1, lam[:K].copy(), st


def step_backward_friction(osc, q_t, v_t, f_ext, q_star, q_star_m1, gq_next, gv_next, contacts, mu_f, lam,
                           g_logE=None, adj_mode=0, tau_force=-1.0):
    cv, cn, cg = contacts
    cv = np.ascontiguousarray(cv, dtype=np.int32)
    cn, cg = _f(cn), _f(cg)
    K = cv.shape[0]
    q_t, v_t = _f(q_t), _f(v_t)
    gq, gv, gf = np.zeros_like(q_t), np.zeros_like(q_t), np.zeros_like(q_t)
    gl = np.zeros(osc.ne) if g_logE is None else g_logE
    ist = np.zeros(2, dtype=np.int32)
    dst = np.zeros(4)
    lam = _f(lam if K else np.zeros((1, 3)))
    lib().or_step_backward_friction(osc.ptr, _p(q_t), _p(v_t), _p(_f(f_ext)) if f_ext is not None else None,
                                    _p(_f(q_star)), _p(_f(q_star_m1)), _p(_f(gq_next)), _p(_f(gv_next)), _p(gq),
                                    _p(gv), _p(gf), _p(gl), int(adj_mode), float(tau_force), K,
                                    cv.ctypes.data_as(_ip), _p(cn), _p(cg), float(mu_f), _p(lam),
                                    ist.ctypes.data_as(_ip), _p(dst))
    st = dict(adj_iters=int(ist[0]), status=int(ist[1]), rho=dst[0], tau=dst[1], dphi_act=dst[2],
              dphi_mod=dst[3])
    return gq, gv, gf, gl, st


def rollout_friction(osc: OracleScene, steps: int, mu_f, fb_tol=1e-10, q0=None, v0=None):
    """Forward rollout with per-step contact detection (one contact per vertex) and Coulomb friction."""
    sc = osc.sc
    q = sc.q0() if q0 is None else q0.copy()
    v = sc.v0() if v0 is None else v0.copy()
    ckpts, stats = [], []
    for t in range(steps):
        f = sc.f_ext(t)
        con = detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles, one_per_vertex=True)
        qn, vn, qm1, lam, st = step_forward_friction(osc, q, v, f, con, mu_f, fb_tol)
        ckpts.append((q.copy(), v.copy(), f.copy(), qn.copy(), qm1.copy(), con, lam))
        stats.append(st)
        q, v = qn, vn
    return q, v, ckpts, stats


def rollout_backward_friction(osc: OracleScene, ckpts, gq_T, gv_T, mu_f, adj_mode=0):
    gq, gv = gq_T.copy(), gv_T.copy()
    gl = np.zeros(osc.ne)
    stats = []
    for (q_t, v_t, f, qs, qsm1, con, lam) in reversed(ckpts):
        gq, gv, _gf, gl, st = step_backward_friction(osc, q_t, v_t, f, qs, qsm1, gq, gv, con, mu_f, lam, gl,
                                                     adj_mode)
        stats.append(st)
    return gq, gv, gl, stats[::-1]


def rollout_contact(osc: OracleScene, steps: int, fb_tol=1e-10, q0=None, v0=None):
    """Forward rollout with per-step contact detection against the scene's obstacles."""
    sc = osc.sc
    q = sc.q0() if q0 is None else q0.copy()
    v = sc.v0() if v0 is None else v0.copy()
    ckpts, stats = [], []
    for t in range(steps):
        f = sc.f_ext(t)
        con = detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles)
        qn, vn, qm1, lam, st = step_forward_contact(osc, q, v, f, con, fb_tol)
        ckpts.append((q.copy(), v.copy(), f.copy(), qn.copy(), qm1.copy(), con, lam))
        stats.append(st)
        q, v = qn, vn
    return q, v, ckpts, stats


def rollout_backward_contact(osc: OracleScene, ckpts, gq_T, gv_T, adj_mode=0, tau_force=-1.0):
    gq, gv = gq_T.copy(), gv_T.copy()
    gl = np.zeros(osc.ne)
    stats = []
    for (q_t, v_t, f, qs, qsm1, con, lam) in reversed(ckpts):
        gq, gv, _gf, gl, st = step_backward_contact(osc, q_t, v_t, f, qs, qsm1, gq, gv, con, lam, gl, adj_mode,
                                                    tau_force)
        stats.append(st)
    return gq, gv, gl, stats[::-1]


def rollout(osc: OracleScene, steps: int, record_ckpt: bool = True, **kw):
    """Forward rollout of the scene; returns final (q, v), checkpoints and stats."""
    sc = osc.sc
    q, v = sc.q0(), sc.v0()
    ckpts, stats = [], []
    for t in range(steps):
        f = sc.f_ext(t)
        qn, vn, qm1, st = osc.step_forward(q, v, f, **kw)
        if record_ckpt:
            ckpts.append((q.copy(), v.copy(), f.copy(), qn.copy(), qm1.copy()))
        stats.append(st)
        q, v = qn, vn
    return q, v, ckpts, stats


def rollout_backward(osc: OracleScene, ckpts, gq_T, gv_T, adj_mode=0, tau_force=-1.0):
    """Reverse sweep over checkpoints; returns dL/dq0, dL/dv0, dL/dlogE and stats."""
    gq, gv = gq_T.copy(), gv_T.copy()
    gl = np.zeros(osc.ne)
    stats = []
    for (q_t, v_t, f, qs, qsm1) in reversed(ckpts):
        gq, gv, _gf, gl, st = osc.step_backward(q_t, v_t, f, qs, qsm1, gq, gv, gl, adj_mode, tau_force)
        stats.append(st)
    return gq, gv, gl, stats[::-1]


# ---------------------------------------------------------------- bilateral rows and restitution
def attachment_rows(verts, targets):
    """Bilateral rows pinning each vertex to its target point: three rows per vertex along x, y, z with
    offsets the target's coordinates (kind 1).  Returns (cv, cn, cg, kind)."""
    verts = np.asarray(verts, dtype=np.int32)
    targets = np.asarray(targets, float).reshape(-1, 3)
    cv = np.repeat(verts, 3).astype(np.int32)
    cn = np.tile(np.eye(3), (len(verts), 1))
    cg = targets.reshape(-1).copy()
    return cv, cn, cg, np.ones(cv.shape[0], dtype=np.uint8)


def join_rows(con, att):
    """Detected unilateral rows (cv, cn, cg) followed by bilateral rows (cv, cn, cg, kind)."""
    cv = np.concatenate([con[0], att[0]]).astype(np.int32)
    cn = np.concatenate([np.asarray(con[1]).reshape(-1, 3), att[1]])
    cg = np.concatenate([con[2], att[2]])
    kind = np.concatenate([np.zeros(len(con[0]), np.uint8), att[3]])
    return cv, cn, cg, kind


def step_forward_contact_ext(osc, q_t, v_t, f_ext, rows, restitution=None, mu_f=0.0, fb_tol=1e-10, force_iters=0,
                             q0=None):
    """One forward step with rows (cv, cn, cg, kind), the restitution post-correction (coefficient or None)
    and friction mu_f; returns q, v, q*_-1, impulses (K, or (K, 3) with friction) and stats."""
    cv, cn, cg, kind = rows
    cv = np.ascontiguousarray(cv, dtype=np.int32)
    cn, cg = _f(cn), _f(cg)
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    q_t, v_t = _f(q_t), _f(v_t)
    K = cv.shape[0]
    qn, vn, qm1 = np.zeros_like(q_t), np.zeros_like(q_t), np.zeros_like(q_t)
    w = 3 if mu_f > 0.0 else 1
    lam = np.zeros(max(K, 1) * w)
    ist = np.zeros(5, dtype=np.int32)
    dst = np.zeros(6)
    lib().or_step_forward_contact_ext(osc.ptr, _p(q_t), _p(v_t), _p(_f(f_ext)) if f_ext is not None else None,
                                      _p(_f(q0)) if q0 is not None else None, _p(qn), _p(vn), _p(qm1), K,
                                      cv.ctypes.data_as(_ip), _p(cn), _p(cg),
                                      kind.ctypes.data_as(ctypes.c_char_p) if K else None,
                                      int(restitution is not None), float(restitution or 0.0), float(mu_f),
                                      float(fb_tol), _p(lam), int(force_iters), ist.ctypes.data_as(_ip), _p(dst))
    st = dict(iters=int(ist[0]), resets=int(ist[1]), newton_capped=int(ist[2]), newton_max=int(ist[3]),
              status=int(ist[4]), gate=dst[:4].copy(), fb_res=float(dst[4]), n_contacts=K)
    lam = lam[:K * w].reshape(K, 3) if w == 3 else lam[:K].copy()
    return qn, vn, qm1, lam, st


def step_backward_contact_ext(osc, q_t, v_t, f_ext, q_star, q_star_m1, gq_next, gv_next, rows, lam,
                              restitution=None, mu_f=0.0, g_logE=None, adj_mode=0, tau_force=-1.0):
    """Backward of step_forward_contact_ext; also returns dL/dg per row (frictionless; zero off the active
    set)."""
    cv, cn, cg, kind = rows
    cv = np.ascontiguousarray(cv, dtype=np.int32)
    cn, cg = _f(cn), _f(cg)
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    K = cv.shape[0]
    q_t, v_t = _f(q_t), _f(v_t)
    gq, gv, gf = np.zeros_like(q_t), np.zeros_like(q_t), np.zeros_like(q_t)
    gl = np.zeros(osc.ne) if g_logE is None else g_logE
    gg = np.zeros(max(K, 1))
    ist = np.zeros(2, dtype=np.int32)
    dst = np.zeros(4)
    lam = _f(np.asarray(lam).reshape(-1) if K else np.zeros(3))
    lib().or_step_backward_contact_ext(osc.ptr, _p(q_t), _p(v_t), _p(_f(f_ext)) if f_ext is not None else None,
                                       _p(_f(q_star)), _p(_f(q_star_m1)), _p(_f(gq_next)), _p(_f(gv_next)), _p(gq),
                                       _p(gv), _p(gf), _p(gl), int(adj_mode), float(tau_force), K,
                                       cv.ctypes.data_as(_ip), _p(cn), _p(cg),
                                       kind.ctypes.data_as(ctypes.c_char_p) if K else None,
                                       int(restitution is not None), float(restitution or 0.0), float(mu_f), _p(lam),
                                       _p(gg), ist.ctypes.data_as(_ip), _p(dst))
    st = dict(adj_iters=int(ist[0]), status=int(ist[1]), rho=dst[0], tau=dst[1], dphi_act=dst[2],
              dphi_mod=dst[3])
    return gq, gv, gf, gl, gg[:K].copy(), st


def rollout_contact_ext(osc: OracleScene, steps: int, attach=None, restitution=None, mu_f=0.0, fb_tol=1e-10,
                        q0=None, v0=None):
    """Forward rollout with per-step detection against the scene's obstacles (if any), bilateral attachment
    rows appended (attach = (verts, targets(t)) or None) and the restitution post-correction."""
    sc = osc.sc
    q = sc.q0() if q0 is None else q0.copy()
    v = sc.v0() if v0 is None else v0.copy()
    ckpts, stats = [], []
    empty = (np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros(0))
    for t in range(steps):
        f = sc.f_ext(t)
        con = detect_contacts(q, v, sc.h, sc.pinned, sc.obstacles, one_per_vertex=mu_f > 0.0) \
            if sc.obstacles else empty
        att = attachment_rows(attach[0], attach[1](t)) if attach is not None else \
            (np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.uint8))
        rows = join_rows(con, att)
        qn, vn, qm1, lam, st = step_forward_contact_ext(osc, q, v, f, rows, restitution, mu_f, fb_tol)
        ckpts.append((q.copy(), v.copy(), f.copy(), qn.copy(), qm1.copy(), rows, lam))
        stats.append(st)
        q, v = qn, vn
    return q, v, ckpts, stats


def rollout_backward_contact_ext(osc: OracleScene, ckpts, gq_T, gv_T, restitution=None, mu_f=0.0, adj_mode=0):
    """Reverse sweep of rollout_contact_ext; returns dL/dq0, dL/dv0, dL/dlogE, per-step dL/dg and stats."""
    gq, gv = gq_T.copy(), gv_T.copy()
    gl = np.zeros(osc.ne)
    ggs, stats = [], []
    for (q_t, v_t, f, qs, qsm1, rows, lam) in reversed(ckpts):
        gq, gv, _gf, gl, gg, st = step_backward_contact_ext(osc, q_t, v_t, f, qs, qsm1, gq, gv, rows, lam,
                                                            restitution, mu_f, gl, adj_mode)
        ggs.append(gg)
        stats.append(st)
    return gq, gv, gl, ggs[::-1], stats[::-1]
