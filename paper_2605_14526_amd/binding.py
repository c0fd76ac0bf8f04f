"""ctypes binding of the pdhot C ABI (include/pdhot.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  PyTorch provides device memory (float64 tensors on ``cuda``) and the
stream.  Loading fails loudly when the compiled library is missing; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdhot.so")

PD_OK = 0
PD_NOT_CONVERGED = 1
ERRORS = {-1: "PD_ERR_INVALID_ARG", -2: "PD_ERR_DEGENERATE_TET", -3: "PD_ERR_NONFINITE",
          -4: "PD_ERR_STALE_FACTOR", -5: "PD_ERR_FACTOR_NOT_SPD", -6: "PD_ERR_HIP", -7: "PD_ERR_ALLOC",
          -8: "PD_ERR_CONTACT"}

EXPORTED = ["pd_scene_create", "pd_scene_destroy", "pd_scene_set_material", "pd_scene_set_material_device",
            "pd_scene_freeze_means", "pd_scene_vertex_mass", "pd_scene_factorize", "pd_scene_info",
            "pd_scene_get_permutation",
            "pd_ckpt_bytes", "pd_step_forward", "pd_step_backward", "pd_debug_local_rhs", "pd_debug_apply_Ainv",
            "pd_debug_apply_K", "pd_kernel_timer", "pd_kernel_timer_read", "pd_adjoint_reset", "pd_scene_vertex_logw",
            "pd_mpn_create", "pd_mpn_destroy", "pd_mpn_info", "pd_mpn_init_params", "pd_mpn_set_params",
            "pd_mpn_get_params", "pd_mpn_get_grads", "pd_mpn_set_output_scale", "pd_mpn_forward", "pd_mpn_loss_grad",
            "pd_mpn_adam_step", "pd_batch_create", "pd_batch_destroy", "pd_batch_config", "pd_batch_step_forward",
            "pd_batch_step_backward", "pd_scene_set_obstacles", "pd_contact_rows", "pd_last_error",
            "pd_scene_factor_nnz", "pd_batch_kernel_timer", "pd_batch_kernel_timer_read",
            "pd_scene_set_friction", "pd_contact_impulses", "pd_apply_Ainv_noalloc", "pd_scene_set_muscles",
            "pd_scene_set_activation", "pd_scene_set_activation_grad", "pd_scene_set_attachments",
            "pd_scene_set_restitution", "pd_contact_gap_grad", "pd_mpn_share_params", "pd_batch_capture_graph"]


class pd_mesh_desc(ctypes.Structure):
    _fields_ = [("n_verts", ctypes.c_int32), ("n_tets", ctypes.c_int32), ("rest_xyz", ctypes.c_void_p),
                ("tets", ctypes.c_void_p), ("pinned", ctypes.c_void_p)]


class pd_material_desc(ctypes.Structure):
    _fields_ = [("log_E", ctypes.c_void_p), ("nu", ctypes.c_double), ("rho", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta0", ctypes.c_double), ("energy", ctypes.c_int32)]


class pd_solver_opts(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("gravity", ctypes.c_double * 3), ("aa_window", ctypes.c_int32),
                ("eps_rel", ctypes.c_double), ("eps_abs", ctypes.c_double), ("kmax_fwd", ctypes.c_int32),
                ("kmax_bwd", ctypes.c_int32), ("eps_adj", ctypes.c_double), ("eps_tr", ctypes.c_double),
                ("adj_method", ctypes.c_int32), ("max_sub", ctypes.c_int32), ("iters_per_check", ctypes.c_int32),
                ("adj_warm", ctypes.c_int32), ("fwd_start", ctypes.c_int32), ("iface_levels", ctypes.c_int32)]


class pd_mpn_desc(ctypes.Structure):
    _fields_ = [("compute", ctypes.c_int32), ("h", ctypes.c_double), ("rho", ctypes.c_double),
                ("edge_weight", ctypes.c_double)]


class pd_fwd_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("aa_resets", ctypes.c_int32), ("status", ctypes.c_int32),
                ("newton_capped", ctypes.c_int32), ("gate", ctypes.c_double * 4), ("n_contacts", ctypes.c_int32),
                ("n_active", ctypes.c_int32), ("fb_res", ctypes.c_double)]


class pd_bwd_stats(ctypes.Structure):
    _fields_ = [("adj_iters", ctypes.c_int32), ("status", ctypes.c_int32), ("rho", ctypes.c_double),
                ("tau", ctypes.c_double), ("dphi_act", ctypes.c_double), ("dphi_mod", ctypes.c_double),
                ("residual", ctypes.c_double), ("n_active", ctypes.c_int32), ("pad", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libpdhot.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"pdhot: {LIB_PATH} is missing; build it with paper_2605_14526_amd/build.py "
                           "(there is no fallback path)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.pd_scene_create.argtypes = [ctypes.POINTER(pd_mesh_desc), ctypes.POINTER(pd_material_desc),
                                  ctypes.POINTER(pd_solver_opts), ctypes.POINTER(vp)]
    L.pd_scene_destroy.argtypes = [vp]
    L.pd_scene_set_material.argtypes = [vp, vp]
    L.pd_scene_set_material_device.argtypes = [vp, vp, vp]
    L.pd_scene_freeze_means.argtypes = [vp, vp]
    L.pd_scene_set_muscles.argtypes = [vp, i32, dbl, vp, vp]
    L.pd_scene_set_activation.argtypes = [vp, vp, vp]
    L.pd_scene_set_activation_grad.argtypes = [vp, vp]
    L.pd_scene_set_attachments.argtypes = [vp, i32, vp, vp, vp]
    L.pd_scene_set_restitution.argtypes = [vp, dbl]
    L.pd_contact_gap_grad.argtypes = [vp, vp, i32]
    L.pd_scene_vertex_mass.argtypes = [vp, vp]
    L.pd_scene_factorize.argtypes = [vp, vp]
    L.pd_scene_info.argtypes = [vp, vp, vp]
    L.pd_scene_get_permutation.argtypes = [vp, vp]
    L.pd_ckpt_bytes.argtypes = [vp]
    L.pd_ckpt_bytes.restype = ctypes.c_size_t
    L.pd_step_forward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(pd_fwd_stats), vp]
    L.pd_step_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(pd_bwd_stats), vp]
    L.pd_debug_local_rhs.argtypes = [vp, vp, vp, vp]
    L.pd_debug_apply_Ainv.argtypes = [vp, vp, vp, vp]
    L.pd_debug_apply_K.argtypes = [vp, vp, dbl, vp, vp, vp]
    L.pd_kernel_timer.argtypes = [vp, i32]
    L.pd_kernel_timer_read.argtypes = [vp, vp, vp, vp, vp]
    L.pd_adjoint_reset.argtypes = [vp]
    L.pd_scene_vertex_logw.argtypes = [vp, vp]
    L.pd_mpn_create.argtypes = [ctypes.POINTER(pd_mesh_desc), ctypes.POINTER(pd_mpn_desc), ctypes.POINTER(vp)]
    L.pd_mpn_destroy.argtypes = [vp]
    L.pd_mpn_info.argtypes = [vp, vp]
    L.pd_mpn_init_params.argtypes = [vp, ctypes.c_uint64]
    L.pd_mpn_set_params.argtypes = [vp, vp, ctypes.c_int64]
    L.pd_mpn_get_params.argtypes = [vp, vp, ctypes.c_int64]
    L.pd_mpn_share_params.argtypes = [vp, vp]
    L.pd_batch_capture_graph.argtypes = [vp, i32]
    L.pd_mpn_get_grads.argtypes = [vp, vp, ctypes.c_int64]
    L.pd_mpn_set_output_scale.argtypes = [vp, dbl]
    L.pd_mpn_forward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.pd_mpn_loss_grad.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.pd_mpn_adam_step.argtypes = [vp, dbl, dbl, dbl, dbl, vp]
    L.pd_batch_create.argtypes = [vp, i32, ctypes.POINTER(vp)]
    L.pd_batch_destroy.argtypes = [vp]
    L.pd_batch_config.argtypes = [vp, i32, i32, i32, i32]
    L.pd_batch_step_forward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.pd_batch_step_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.pd_scene_set_obstacles.argtypes = [vp, i32, vp, i32, vp, dbl, i32, dbl]
    L.pd_contact_rows.argtypes = [vp, vp, vp, vp, vp, vp, i32]
    L.pd_scene_set_friction.argtypes = [vp, dbl]
    L.pd_contact_impulses.argtypes = [vp, vp, i32]
    L.pd_apply_Ainv_noalloc.argtypes = [vp, vp, vp, vp]
    L.pd_scene_factor_nnz.argtypes = [vp, vp]
    L.pd_batch_kernel_timer.argtypes = [vp, i32]
    L.pd_batch_kernel_timer_read.argtypes = [vp, vp, vp, vp]
    L.pd_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        getattr(L, name)
    _ = i32
    _lib = L
    return L


def check(rc: int, what: str) -> int:
    if rc < 0:
        msg = lib().pd_last_error().decode()
        raise RuntimeError(f"{what} failed with {ERRORS.get(rc, rc)}: {msg}")
    return rc


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Scene:
    """A pdhot scene on the current GPU (wraps pd_scene_create ... pd_scene_destroy)."""

    def __init__(self, X, tets, pinned, log_E, nu, rho, alpha, beta0, h, gravity=(0.0, 0.0, 0.0), aa_window=1,
                 eps_rel=1e-6, eps_abs=1e-12, kmax_fwd=1000, kmax_bwd=1000, eps_adj=1e-6, eps_tr=0.1,
                 adj_method=0, max_sub=0, iters_per_check=0, adj_warm=0, fwd_start=0, energy=0, iface_levels=0):
        L = lib()
        self._X = np.ascontiguousarray(X, dtype=np.float64)
        self._tets = np.ascontiguousarray(tets, dtype=np.int32)
        self._pinned = np.ascontiguousarray(pinned, dtype=np.uint8)
        self._logE = np.ascontiguousarray(log_E, dtype=np.float64)
        self.n_verts = int(self._X.shape[0])
        self.n_tets = int(self._tets.shape[0])
        mesh = pd_mesh_desc(self.n_verts, self.n_tets, self._X.ctypes.data, self._tets.ctypes.data,
                            self._pinned.ctypes.data)
        mat = pd_material_desc(self._logE.ctypes.data, nu, rho, alpha, beta0, int(energy))
        opts = pd_solver_opts(h, (ctypes.c_double * 3)(*gravity), aa_window, eps_rel, eps_abs, kmax_fwd, kmax_bwd,
                              eps_adj, eps_tr, adj_method, max_sub, iters_per_check, adj_warm, fwd_start,
                              iface_levels)
        self.h = float(h)
        ptr = ctypes.c_void_p()
        check(L.pd_scene_create(ctypes.byref(mesh), ctypes.byref(mat), ctypes.byref(opts), ctypes.byref(ptr)),
              "pd_scene_create")
        self.ptr = ptr

    @classmethod
    def from_scene(cls, sc, **kw):
        args = dict(aa_window=sc.aa_window, eps_rel=sc.eps_rel, eps_abs=sc.eps_abs, energy=getattr(sc, "energy", 0))
        contact = kw.pop("contact", {})
        args.update(kw)
        g = cls(sc.X, sc.tets, sc.pinned, sc.log_E, sc.nu, sc.rho, sc.alpha, sc.beta0, sc.h,
                tuple(np.asarray(sc.gravity, float)), **args)
        if getattr(sc, "obstacles", None):
            g.set_obstacles(sc.obstacles, **contact)
            if getattr(sc, "friction", 0.0) > 0.0:
                g.set_friction(sc.friction)
        if getattr(sc, "muscle_group", None) is not None:
            import torch
            g.set_muscles(sc.muscle_group, sc.muscle_fibre, sc.muscle_w)
            g.factorize()
            g.set_activation(torch.tensor(sc.activation, dtype=torch.float64, device="cuda"))
        return g

    def set_muscles(self, group, fibre, w_m):
        """Muscle fibres (pd_scene_set_muscles): group per tet (-1 passive), unit fibre per tet, weight w_m.
        Marks the factor stale."""
        self._mgroup = np.ascontiguousarray(group, dtype=np.int32)
        self._mfib = np.ascontiguousarray(fibre, dtype=np.float64).reshape(-1, 3)
        self.n_groups = int(self._mgroup.max()) + 1 if self._mgroup.size and self._mgroup.max() >= 0 else 0
        check(lib().pd_scene_set_muscles(self.ptr, self.n_groups, float(w_m), self._mgroup.ctypes.data,
                                         self._mfib.ctypes.data), "pd_scene_set_muscles")

    def set_activation(self, a):
        """The groups' activations from a float64 device tensor (copied on the current stream)."""
        check(lib().pd_scene_set_activation(self.ptr, _ptr(a), _stream()), "pd_scene_set_activation")

    def set_activation_grad(self, g):
        """Device buffer (float64, n_groups) that every backward step adds dL/da into; None stops it."""
        self._g_act = g
        check(lib().pd_scene_set_activation_grad(self.ptr, _ptr(g) if g is not None else None),
              "pd_scene_set_activation_grad")

    def set_attachments(self, verts, normals, offsets):
        """Bilateral rows n . q_v = g (pd_scene_set_attachments): caller vertex ids, unit directions, offsets."""
        self._att = (np.ascontiguousarray(verts, dtype=np.int32),
                     np.ascontiguousarray(normals, dtype=np.float64).reshape(-1, 3),
                     np.ascontiguousarray(offsets, dtype=np.float64))
        n = int(self._att[0].shape[0])
        check(lib().pd_scene_set_attachments(self.ptr, n, self._att[0].ctypes.data if n else None,
                                             self._att[1].ctypes.data if n else None,
                                             self._att[2].ctypes.data if n else None), "pd_scene_set_attachments")

    def set_restitution(self, e):
        """Restitution coefficient of the contact rows (None or negative: off)."""
        check(lib().pd_scene_set_restitution(self.ptr, -1.0 if e is None else float(e)), "pd_scene_set_restitution")

    def contact_gap_grad(self, capacity=None):
        """dL/dg of the last backward step's rows (pd_contact_gap_grad)."""
        cap = int(capacity if capacity is not None else 4096)
        out = np.zeros(max(cap, 1))
        check(lib().pd_contact_gap_grad(self.ptr, out.ctypes.data, cap), "pd_contact_gap_grad")
        return out

    def set_friction(self, mu):
        """Coulomb coefficient of the obstacles (pd_scene_set_friction; 0 = frictionless)."""
        check(lib().pd_scene_set_friction(self.ptr, float(mu)), "pd_scene_set_friction")

    def contact_impulses(self):
        """Impulses of the last forward step's rows: (K, 3) normal, t1, t2 (pd_contact_impulses)."""
        K = ctypes.c_int()
        check(lib().pd_contact_rows(self.ptr, ctypes.byref(K), None, None, None, None, 0), "pd_contact_rows")
        n = K.value
        lam = np.zeros((max(n, 1), 3))
        check(lib().pd_contact_impulses(self.ptr, lam.ctypes.data, n), "pd_contact_impulses")
        return lam[:n]

    def set_obstacles(self, obs, max_contacts=512, fb_tol=1e-10):
        """Static obstacles {"planes": [(n, o)], "boxes": [(lo, hi)], "d_c": d} (pd_scene_set_obstacles)."""
        planes = np.ascontiguousarray([list(n) + [o] for (n, o) in obs.get("planes", [])] or np.zeros((0, 4)),
                                      dtype=np.float64)
        boxes = np.ascontiguousarray([list(lo) + list(hi) for (lo, hi) in obs.get("boxes", [])] or np.zeros((0, 6)),
                                     dtype=np.float64)
        self._obs = (planes, boxes)
        check(lib().pd_scene_set_obstacles(self.ptr, planes.shape[0], planes.ctypes.data if planes.size else None,
                                           boxes.shape[0], boxes.ctypes.data if boxes.size else None,
                                           float(obs["d_c"]), int(max_contacts), float(fb_tol)),
              "pd_scene_set_obstacles")

    def contact_rows(self):
        """Rows of the last forward step: caller's vertex ids, normals, offsets, impulses."""
        K = ctypes.c_int()
        check(lib().pd_contact_rows(self.ptr, ctypes.byref(K), None, None, None, None, 0), "pd_contact_rows")
        n = K.value
        v = np.zeros(max(n, 1), np.int32)
        nn = np.zeros((max(n, 1), 3))
        g = np.zeros(max(n, 1))
        lam = np.zeros(max(n, 1))
        check(lib().pd_contact_rows(self.ptr, ctypes.byref(K), v.ctypes.data, nn.ctypes.data, g.ctypes.data,
                                    lam.ctypes.data, n), "pd_contact_rows")
        return v[:n], nn[:n], g[:n], lam[:n]

    def close(self):
        if getattr(self, "ptr", None) is not None and self.ptr.value:
            lib().pd_scene_destroy(self.ptr)
        self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        info = (ctypes.c_double * 8)()
        means = (ctypes.c_double * 4)()
        check(lib().pd_scene_info(self.ptr, info, means), "pd_scene_info")
        keys = ["n_verts", "n_tets", "n_free", "n_subdomains", "n_interface", "aa_window", "factor_bytes",
                "max_couplings"]
        d = {k: info[i] for i, k in enumerate(keys)}
        d.update(mu_bar=means[0], lam_bar=means[1], k_bar=means[2], mu_ref=means[3])
        return d

    def permutation(self):
        """The library's vertex order: perm[i] = caller index of library vertex i."""
        n = int(self.info()["n_verts"])
        perm = np.empty(n, dtype=np.int32)
        check(lib().pd_scene_get_permutation(self.ptr, perm.ctypes.data), "pd_scene_get_permutation")
        return perm

    def set_material(self, log_E):
        self._logE = np.ascontiguousarray(log_E, dtype=np.float64)
        self._logE_dev = None
        check(lib().pd_scene_set_material(self.ptr, self._logE.ctypes.data), "pd_scene_set_material")

    def set_material_device(self, log_E):
        """log E from a float64 device tensor (copied on the current stream)."""
        check(lib().pd_scene_set_material_device(self.ptr, _ptr(log_E), _stream()), "pd_scene_set_material_device")
        self._logE_dev = log_E.detach().clone()
        self._logE = self._logE_dev.cpu().numpy()

    def freeze_means(self, means=None):
        """Hold (mu_bar, lam_bar, mu_ref) fixed across refactorizations (None: recompute each time)."""
        if means is None:
            check(lib().pd_scene_freeze_means(self.ptr, None), "pd_scene_freeze_means")
            return
        a = np.ascontiguousarray(means, dtype=np.float64)
        check(lib().pd_scene_freeze_means(self.ptr, a.ctypes.data), "pd_scene_freeze_means")

    def vertex_mass(self) -> np.ndarray:
        """Lumped vertex masses (caller's vertex order)."""
        out = np.zeros(self.n_verts)
        check(lib().pd_scene_vertex_mass(self.ptr, out.ctypes.data), "pd_scene_vertex_mass")
        return out

    def factorize(self):
        check(lib().pd_scene_factorize(self.ptr, _stream()), "pd_scene_factorize")

    def ckpt_bytes(self) -> int:
        return int(lib().pd_ckpt_bytes(self.ptr))

    def new_ckpt(self):
        import torch
        return torch.empty(self.ckpt_bytes() // 8, dtype=torch.float64, device="cuda")

    def step_forward(self, q_t, v_t, f_ext=None, q0=None, q_next=None, v_next=None, ckpt=None):
        import torch
        q_next = torch.empty_like(q_t) if q_next is None else q_next
        v_next = torch.empty_like(q_t) if v_next is None else v_next
        st = pd_fwd_stats()
        rc = check(lib().pd_step_forward(self.ptr, _ptr(q_t), _ptr(v_t), _ptr(f_ext), _ptr(q0), _ptr(q_next),
                                         _ptr(v_next), _ptr(ckpt), ctypes.byref(st), _stream()), "pd_step_forward")
        return q_next, v_next, dict(iters=st.iters, aa_resets=st.aa_resets, status=st.status, rc=rc,
                                    newton_capped=st.newton_capped, gate=list(st.gate), n_contacts=st.n_contacts,
                                    n_active=st.n_active, fb_res=st.fb_res)

    def step_backward(self, ckpt, gq_next, gv_next, g_logE=None, gq_t=None, gv_t=None, gf_ext=None):
        import torch
        gq_t = torch.empty_like(gq_next) if gq_t is None else gq_t
        gv_t = torch.empty_like(gq_next) if gv_t is None else gv_t
        gf_ext = torch.empty_like(gq_next) if gf_ext is None else gf_ext
        if g_logE is None:
            g_logE = torch.zeros(self.n_tets, dtype=torch.float64, device=gq_next.device)
        st = pd_bwd_stats()
        rc = check(lib().pd_step_backward(self.ptr, _ptr(ckpt), _ptr(gq_next), _ptr(gv_next), _ptr(gq_t),
                                          _ptr(gv_t), _ptr(gf_ext), _ptr(g_logE), ctypes.byref(st), _stream()),
                   "pd_step_backward")
        self.last_bwd_stats = dict(adj_iters=st.adj_iters, status=st.status, rho=st.rho, tau=st.tau,
                                   dphi_act=st.dphi_act, dphi_mod=st.dphi_mod, residual=st.residual, rc=rc,
                                   n_active=st.n_active)
        return gq_t, gv_t, gf_ext, g_logE, self.last_bwd_stats

    def factor_nnz(self) -> float:
        """Entries of a nested-dissection sparse Cholesky factor of A~ (the solve's algorithmic size)."""
        n = ctypes.c_double()
        check(lib().pd_scene_factor_nnz(self.ptr, ctypes.byref(n)), "pd_scene_factor_nnz")
        return n.value

    def vertex_logw(self) -> np.ndarray:
        """Per-vertex mean log(2 mu_e + lam_e) minus its mean (the warm-start network's material feature)."""
        out = np.zeros(self.n_verts)
        check(lib().pd_scene_vertex_logw(self.ptr, out.ctypes.data), "pd_scene_vertex_logw")
        return out

    def adjoint_reset(self):
        """Start the next backward step from zero (clears the adjoint warm-start history)."""
        check(lib().pd_adjoint_reset(self.ptr), "pd_adjoint_reset")

    def kernel_timer(self, kernel: int):
        check(lib().pd_kernel_timer(self.ptr, int(kernel)), "pd_kernel_timer")

    def kernel_timer_read(self):
        ms = ctypes.c_double()
        n, w = ctypes.c_int64(), ctypes.c_int64()
        b = ctypes.c_double()
        check(lib().pd_kernel_timer_read(self.ptr, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(w),
                                         ctypes.byref(b)), "pd_kernel_timer_read")
        self._last_bytes = b.value
        return ms.value, n.value, w.value

    def kernel_bytes(self, kernel: int) -> float:
        return getattr(self, "_last_bytes", 0.0)

    def debug_local_rhs(self, q):
        import torch
        b = torch.empty_like(q)
        check(lib().pd_debug_local_rhs(self.ptr, _ptr(q), _ptr(b), _stream()), "pd_debug_local_rhs")
        return b

    def debug_apply_Ainv(self, r):
        import torch
        x = torch.empty_like(r)
        check(lib().pd_debug_apply_Ainv(self.ptr, _ptr(r), _ptr(x), _stream()), "pd_debug_apply_Ainv")
        return x

    def apply_Ainv_noalloc(self, r, x):
        """x = A~^{-1} r into the caller's x, scratch from the library's static workspace
        (pd_apply_Ainv_noalloc; ordered on the current stream, no host wait)."""
        check(lib().pd_apply_Ainv_noalloc(self.ptr, _ptr(r), _ptr(x), _stream()), "pd_apply_Ainv_noalloc")
        return x

    def debug_apply_K(self, q, tau, x):
        import torch
        y = torch.empty_like(x)
        check(lib().pd_debug_apply_K(self.ptr, _ptr(q), float(tau), _ptr(x), _ptr(y), _stream()),
              "pd_debug_apply_K")
        return y


class Mpn:
    """The learned warm-start network on one mesh (wraps pd_mpn_create ... pd_mpn_destroy)."""

    def __init__(self, X, tets, pinned, h, rho, compute=0, edge_weight=0.0):
        L = lib()
        self._X = np.ascontiguousarray(X, dtype=np.float64)
        self._tets = np.ascontiguousarray(tets, dtype=np.int32)
        self._pinned = np.ascontiguousarray(pinned, dtype=np.uint8)
        mesh = pd_mesh_desc(int(self._X.shape[0]), int(self._tets.shape[0]), self._X.ctypes.data,
                            self._tets.ctypes.data, self._pinned.ctypes.data)
        desc = pd_mpn_desc(int(compute), float(h), float(rho), float(edge_weight))
        ptr = ctypes.c_void_p()
        check(L.pd_mpn_create(ctypes.byref(mesh), ctypes.byref(desc), ctypes.byref(ptr)), "pd_mpn_create")
        self.ptr = ptr
        self.n_params = int(self.info()["n_params"])

    @classmethod
    def for_scene(cls, sc, compute=0, edge_weight=0.0):
        return cls(sc.X, sc.tets, sc.pinned, sc.h, sc.rho, compute, edge_weight)

    def close(self):
        if getattr(self, "ptr", None) is not None and self.ptr.value:
            lib().pd_mpn_destroy(self.ptr)
        self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        info = (ctypes.c_double * 7)()
        check(lib().pd_mpn_info(self.ptr, info), "pd_mpn_info")
        keys = ["n_verts", "n_edges", "ell", "L", "n_params", "s_out", "compute"]
        return {k: info[i] for i, k in enumerate(keys)}

    def init_params(self, seed: int):
        check(lib().pd_mpn_init_params(self.ptr, int(seed)), "pd_mpn_init_params")

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        check(lib().pd_mpn_set_params(self.ptr, a.ctypes.data, a.size), "pd_mpn_set_params")

    def share_params(self, src: "Mpn"):
        """Use src's weights, gradient and Adam moments from now on (pd_mpn_share_params); src must outlive
        this network."""
        check(lib().pd_mpn_share_params(self.ptr, src.ptr), "pd_mpn_share_params")
        self._shared_src = src

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.n_params, dtype=np.float32)
        check(lib().pd_mpn_get_params(self.ptr, a.ctypes.data, a.size), "pd_mpn_get_params")
        return a

    def get_grads(self) -> np.ndarray:
        a = np.zeros(self.n_params, dtype=np.float32)
        check(lib().pd_mpn_get_grads(self.ptr, a.ctypes.data, a.size), "pd_mpn_get_grads")
        return a

    def set_output_scale(self, s_out: float):
        check(lib().pd_mpn_set_output_scale(self.ptr, float(s_out)), "pd_mpn_set_output_scale")

    def forward(self, q_t, v_tm1, v_t, f_ext, logw, q0=None):
        import torch
        q0 = torch.empty_like(q_t) if q0 is None else q0
        check(lib().pd_mpn_forward(self.ptr, _ptr(q_t), _ptr(v_tm1), _ptr(v_t), _ptr(f_ext), _ptr(logw), _ptr(q0),
                                   _stream()), "pd_mpn_forward")
        return q0

    def loss_grad(self, q_t, v_tm1, v_t, f_ext, logw, q_next, want_loss=True):
        loss = ctypes.c_double(0.0)
        check(lib().pd_mpn_loss_grad(self.ptr, _ptr(q_t), _ptr(v_tm1), _ptr(v_t), _ptr(f_ext), _ptr(logw),
                                     _ptr(q_next), ctypes.byref(loss) if want_loss else None, _stream()),
              "pd_mpn_loss_grad")
        return loss.value if want_loss else None

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        check(lib().pd_mpn_adam_step(self.ptr, float(lr), float(beta1), float(beta2), float(eps), _stream()),
              "pd_mpn_adam_step")


def _ptrs(ts):
    if ts is None:
        return None
    arr = (ctypes.c_void_p * len(ts))(*[(t.data_ptr() if t is not None else None) for t in ts])
    return arr


class Batch:
    """Several scenes stepped together (wraps pd_batch_*); the scenes must outlive it."""

    def __init__(self, scenes):
        self.scenes = list(scenes)
        arr = (ctypes.c_void_p * len(self.scenes))(*[sc.ptr.value for sc in self.scenes])
        ptr = ctypes.c_void_p()
        check(lib().pd_batch_create(arr, len(self.scenes), ctypes.byref(ptr)), "pd_batch_create")
        self.ptr = ptr
        self.cfg = dict(block_local=256, block_applyK=256, iters_per_check=0, use_graph=0)

    def close(self):
        if getattr(self, "ptr", None) is not None and self.ptr.value:
            lib().pd_batch_destroy(self.ptr)
        self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def config(self, block_local=256, block_applyK=256, iters_per_check=0, use_graph=0):
        check(lib().pd_batch_config(self.ptr, int(block_local), int(block_applyK), int(iters_per_check),
                                    int(use_graph)), "pd_batch_config")
        self.cfg = dict(block_local=block_local, block_applyK=block_applyK, iters_per_check=iters_per_check,
                        use_graph=use_graph)

    def capture_graph(self, iters_per_chunk: int):
        """Graph replay of chunks of iters_per_chunk iterations (pd_batch_capture_graph; 0: eager)."""
        check(lib().pd_batch_capture_graph(self.ptr, int(iters_per_chunk)), "pd_batch_capture_graph")
        self.cfg.update(iters_per_check=int(iters_per_chunk), use_graph=int(iters_per_chunk > 0))

    def kernel_timer(self, kernel: int):
        check(lib().pd_batch_kernel_timer(self.ptr, int(kernel)), "pd_batch_kernel_timer")

    def kernel_timer_read(self):
        """(summed launch ms, launches, algorithmic bytes of the work done)."""
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        check(lib().pd_batch_kernel_timer_read(self.ptr, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)),
              "pd_batch_kernel_timer_read")
        return ms.value, n.value, b.value

    def step_forward(self, q_t, v_t, f_ext=None, q0=None, q_next=None, v_next=None, ckpt=None):
        import torch
        n = len(self.scenes)
        q_next = [torch.empty_like(q) for q in q_t] if q_next is None else q_next
        v_next = [torch.empty_like(q) for q in q_t] if v_next is None else v_next
        st = (pd_fwd_stats * n)()
        keep = [_ptrs(q_t), _ptrs(v_t), _ptrs(f_ext), _ptrs(q0), _ptrs(q_next), _ptrs(v_next), _ptrs(ckpt)]
        rc = check(lib().pd_batch_step_forward(self.ptr, *keep, st, _stream()), "pd_batch_step_forward")
        stats = [dict(iters=x.iters, aa_resets=x.aa_resets, status=x.status, newton_capped=x.newton_capped,
                      gate=list(x.gate)) for x in st]
        return q_next, v_next, stats, rc

    def step_backward(self, ckpt, gq_next, gv_next, g_logE=None, gq_t=None, gv_t=None, gf_ext=None):
        import torch
        n = len(self.scenes)
        gq_t = [torch.empty_like(g) for g in gq_next] if gq_t is None else gq_t
        gv_t = [torch.empty_like(g) for g in gq_next] if gv_t is None else gv_t
        gf_ext = [torch.empty_like(g) for g in gq_next] if gf_ext is None else gf_ext
        if g_logE is None:
            g_logE = [torch.zeros(sc.n_tets, dtype=torch.float64, device="cuda") for sc in self.scenes]
        st = (pd_bwd_stats * n)()
        keep = [_ptrs(ckpt), _ptrs(gq_next), _ptrs(gv_next), _ptrs(gq_t), _ptrs(gv_t), _ptrs(gf_ext), _ptrs(g_logE)]
        rc = check(lib().pd_batch_step_backward(self.ptr, *keep, st, _stream()), "pd_batch_step_backward")
        stats = [dict(adj_iters=x.adj_iters, status=x.status, rho=x.rho, tau=x.tau, residual=x.residual)
                 for x in st]
        return gq_t, gv_t, gf_ext, g_logE, stats, rc
