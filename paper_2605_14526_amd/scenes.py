"""Seeded synthetic scene generators (inputs only).

This module builds the meshes, material fields, force schedules and loss
targets that stand in for the paper's scenes (Sec. 5, Table of examples: the
cantilever, the contact drops).  It holds none of the solver's arithmetic: no
Lame parameters, masses, weights or projections are computed here, only
geometry (vertex grids, the 5-tet cube split, orientation of each tet), random
fields and schedules.  Both the CPU oracle and the HIP library consume these
arrays, so it is the only code the two share.

Conventions
-----------
* ``X``      rest positions, float64, shape (n_v, 3), vertex-major.
* ``tets``   int32, shape (n_e, 4), positively oriented
             (det[x1-x0, x2-x0, x3-x0] > 0).
* ``pinned`` uint8, shape (n_v,), 1 for a Dirichlet vertex held at rest.
* ``log_E``  float64, shape (n_e,), natural log of Young's modulus in Pa.
* Seeds use ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
from typing import Tuple, Callable, Optional

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# The 5-tet split of a unit cube.  Corners are indexed by (i, j, k) in {0,1}^3.
# Even-parity cubes cut off the corners (0,0,0), (1,1,0), (1,0,1), (0,1,1) and
# keep the central tet on the other four corners; odd-parity cubes mirror that
# choice, so shared faces carry the same diagonal and the mesh is conforming.
_EVEN_CORNERS = [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
_ODD_CORNERS = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)]


def _cube_tets(parity: int):
    corners = _EVEN_CORNERS if parity == 0 else _ODD_CORNERS
    tets = []
    for c in corners:
        nb = [(c[0] ^ 1, c[1], c[2]), (c[0], c[1] ^ 1, c[2]), (c[0], c[1], c[2] ^ 1)]
        tets.append([c] + nb)
    # central tet: the four corners not cut off
    other = _ODD_CORNERS if parity == 0 else _EVEN_CORNERS
    tets.append(list(other))
    return tets


def _orient(X: np.ndarray, tets: np.ndarray) -> np.ndarray:
    d1 = X[tets[:, 1]] - X[tets[:, 0]]
    d2 = X[tets[:, 2]] - X[tets[:, 0]]
    d3 = X[tets[:, 3]] - X[tets[:, 0]]
    det = np.einsum("ij,ij->i", d1, np.cross(d2, d3))
    out = tets.copy()
    neg = det < 0
    out[neg, 1], out[neg, 2] = tets[neg, 2], tets[neg, 1]
    return out


def voxel_tet_mesh(occ: np.ndarray, edge: float, origin=(0.0, 0.0, 0.0)):
    """Tetrahedralise the occupied voxels of a boolean grid ``occ[nx, ny, nz]``.

    Each voxel is split into 5 tets with parity (i + j + k) mod 2.  Vertices
    are numbered with x the slowest index, then y, then z; vertices not used by
    any tet are dropped (numbering order is kept).
    """
    occ = np.asarray(occ, dtype=bool)
    nx, ny, nz = occ.shape
    vid = lambda i, j, k: (i * (ny + 1) + j) * (nz + 1) + k  # noqa: E731
    templ = [_cube_tets(0), _cube_tets(1)]
    tl = []
    idx = np.argwhere(occ)
    for (i, j, k) in idx:
        for t in templ[(i + j + k) & 1]:
            tl.append([vid(i + a, j + b, k + c) for (a, b, c) in t])
    tets = np.asarray(tl, dtype=np.int64).reshape(-1, 4)
    gi, gj, gk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    Xall = np.stack([gi.ravel(), gj.ravel(), gk.ravel()], axis=1).astype(np.float64) * edge
    Xall += np.asarray(origin, dtype=np.float64)
    used = np.zeros(Xall.shape[0], dtype=bool)
    used[tets.ravel()] = True
    remap = -np.ones(Xall.shape[0], dtype=np.int64)
    remap[used] = np.arange(int(used.sum()))
    X = Xall[used].copy()
    tets = remap[tets]
    tets = _orient(X, tets).astype(np.int32)
    return X, tets


def box_tet_mesh(nx: int, ny: int, nz: int, edge: float):
    return voxel_tet_mesh(np.ones((nx, ny, nz), dtype=bool), edge)


def gaussian_blob_field(points: np.ndarray, lo, hi, n_blobs: int, rng, sig_lo=0.1, sig_hi=0.3):
    """Sum of ``n_blobs`` isotropic Gaussians with uniform centres in [lo, hi]."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    field = np.zeros(points.shape[0])
    for _ in range(n_blobs):
        c = lo + (hi - lo) * rng.random(3)
        s = sig_lo + (sig_hi - sig_lo) * rng.random()
        r2 = ((points - c) ** 2).sum(axis=1)
        field += np.exp(-0.5 * r2 / (s * s))
    return field


def two_phase_log_E(field: np.ndarray, frac_stiff: float, E_soft: float, E_stiff: float) -> np.ndarray:
    """Exactly ``round(frac_stiff * n)`` entries with the largest field are stiff."""
    n = field.shape[0]
    n_stiff = int(round(frac_stiff * n))
    order = np.argsort(-field, kind="stable")
    logE = np.full(n, np.log(E_soft))
    logE[order[:n_stiff]] = np.log(E_stiff)
    return logE


@dataclasses.dataclass
class Scene:
    name: str
    X: np.ndarray
    tets: np.ndarray
    pinned: np.ndarray
    log_E: np.ndarray
    nu: float
    rho: float
    alpha: float
    beta0: float
    h: float
    gravity: np.ndarray
    aa_window: int
    steps: int
    force_fn: Optional[Callable[[int], np.ndarray]]
    target_centroid: np.ndarray
    fd_tets: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int64))
    eps_rel: float = 1e-6
    eps_abs: float = 1e-12
    # static obstacles: {"planes": [(normal, offset)], "boxes": [(lo, hi)], "d_c": candidate distance}
    obstacles: Optional[dict] = None
    v_init: Optional[np.ndarray] = None
    # identification tasks: the material field that generated the observed trajectory
    log_E_obs: Optional[np.ndarray] = None
    # energy model of the local step: 0 Neo-Hookean proximal map, 1 corotated + volume composite
    energy: int = 0
    # Coulomb friction coefficient of the obstacles (0: frictionless contact)
    friction: float = 0.0
    # muscle fibres: group per tet (-1 passive), unit fibre per tet (rest coordinates), fibre weight (Pa),
    # and the groups' activations
    muscle_group: Optional[np.ndarray] = None
    muscle_fibre: Optional[np.ndarray] = None
    muscle_w: float = 0.0
    activation: Optional[np.ndarray] = None

    @property
    def n_v(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_e(self) -> int:
        return int(self.tets.shape[0])

    def f_ext(self, t: int) -> np.ndarray:
        if self.force_fn is None:
            return np.zeros((self.n_v, 3))
        return self.force_fn(t)

    def q0(self) -> np.ndarray:
        return self.X.copy()

    def v0(self) -> np.ndarray:
        if self.v_init is not None:
            return np.broadcast_to(np.asarray(self.v_init, float), (self.n_v, 3)).copy()
        return np.zeros((self.n_v, 3))


def centroid_loss(q: np.ndarray, target: np.ndarray):
    """Loss ||mean_v q_v - target||^2 and its gradient w.r.t. q (harness, not solver)."""
    c = q.mean(axis=0)
    d = c - target
    g = np.broadcast_to(2.0 * d / q.shape[0], q.shape).copy()
    return float(d @ d), g


def cantilever_c1() -> Scene:
    """Plain PD beam: 16x4x4 unit cubes along x, edge 0.05 m, 1280 tets / 425 verts.

    Homogeneous E = 1e5 Pa, nu = 0.45, rho = 1000, x = 0 face pinned, gravity,
    h = 0.01 s, 20 steps, Anderson window 5, no damping.
    """
    X, tets = box_tet_mesh(16, 4, 4, 0.05)
    pinned = (np.abs(X[:, 0]) < 1e-12).astype(np.uint8)
    logE = np.full(tets.shape[0], np.log(1e5))
    rng = _rng(1001)
    target = X.mean(axis=0) + rng.uniform(-0.05, 0.05, 3)
    return Scene("c1_cantilever", X, tets, pinned, logE, nu=0.45, rho=1000.0, alpha=0.0, beta0=0.0,
                 h=0.01, gravity=np.array([0.0, 0.0, -9.81]), aa_window=5, steps=20, force_fn=None,
                 target_centroid=target)


def _tip_force_fn(X: np.ndarray, total: float, seed: int, ramp: int, hold: int):
    L = X[:, 0].max()
    face = np.abs(X[:, 0] - L) < 1e-12
    nface = int(face.sum())
    rng = _rng(seed)
    th = 2.0 * np.pi * rng.random()
    d = np.array([0.2, np.cos(th), np.sin(th)])
    d /= np.linalg.norm(d)
    base = np.zeros_like(X)
    base[face] = d * (total / nface)

    def fn(t: int) -> np.ndarray:
        if t < ramp:
            s = (t + 1) / ramp
        elif t < hold:
            s = 1.0
        else:
            s = 0.0
        return base * s

    return fn


def hetero_beam_c2(nx: int = 40, ny: int = 10, nz: int = 10, steps: int = 100, seeds=(2001, 2002, 2003, 2004),
                   name: str = "c2_hetero_beam") -> Scene:
    """Heterogeneous beam: 40x10x10 cubes (edge 0.05 m) = 20000 tets / 4961 verts.

    Two-phase E in {1e4, 1e6} Pa from 8 seeded Gaussian blobs (30 % stiff),
    nu = 0.49, rho = 1000, Rayleigh alpha = 0.01 and beta0 = 1e-2 s * E_max,
    x = 0 face pinned, no gravity, 50 N seeded tip force ramped over steps
    0-19, held to step 59, then released; h = 0.005 s, 100 steps, window 1.
    """
    edge = 0.05
    X, tets = box_tet_mesh(nx, ny, nz, edge)
    pinned = (np.abs(X[:, 0]) < 1e-12).astype(np.uint8)
    cen = X[tets].mean(axis=1)
    rng = _rng(seeds[0])
    field = gaussian_blob_field(cen, X.min(axis=0), X.max(axis=0), 8, rng)
    logE = two_phase_log_E(field, 0.3, 1e4, 1e6)
    force = _tip_force_fn(X, 50.0, seeds[1], 20, 60)
    rng3 = _rng(seeds[2])
    target = X.mean(axis=0) + rng3.uniform(-0.05, 0.05, 3)
    fd = _rng(seeds[3]).choice(tets.shape[0], size=16, replace=False)
    return Scene(name, X, tets, pinned, logE, nu=0.49, rho=1000.0, alpha=0.01,
                 beta0=1e-2 * 1e6, h=0.005, gravity=np.zeros(3), aa_window=1, steps=steps,
                 force_fn=force, target_centroid=target, fd_tets=fd)


def hetero_beam_family(k: int, steps: int = 100, nx: int = 40, ny: int = 10, nz: int = 10) -> Scene:
    """Member k of the heterogeneous-beam family: the benchmark beam's mesh,
    load schedule and materials drawn with seeds 2100 + 10 k + (1, 2, 3, 4)
    (another stiff-blob field and tip-force direction).  Training scenes of the
    learned warm start are members 0..; the benchmark beam itself is not a
    member."""
    b = 2100 + 10 * k
    return hetero_beam_c2(nx, ny, nz, steps, seeds=(b + 1, b + 2, b + 3, b + 4), name=f"hetero_beam_{k}")


def small_beam(nx: int, ny: int, nz: int, seed: int = 7, contrast: float = 100.0, nu: float = 0.45,
               alpha: float = 0.01, beta_rel: float = 1e-2, h: float = 0.01, gravity=(0.0, 0.0, -9.81),
               tip_force: float = 5.0, aa_window: int = 1, steps: int = 5) -> Scene:
    """Small heterogeneous beam for parity tests (C2-shaped, a few hundred tets)."""
    edge = 0.05
    X, tets = box_tet_mesh(nx, ny, nz, edge)
    pinned = (np.abs(X[:, 0]) < 1e-12).astype(np.uint8)
    cen = X[tets].mean(axis=1)
    rng = _rng(seed)
    field = gaussian_blob_field(cen, X.min(axis=0), X.max(axis=0), 3, rng, 0.03, 0.1)
    E_soft = 1e4
    logE = two_phase_log_E(field, 0.3, E_soft, E_soft * contrast)
    force = _tip_force_fn(X, tip_force, seed + 1, 2, 4) if tip_force else None
    target = X.mean(axis=0) + _rng(seed + 2).uniform(-0.05, 0.05, 3)
    fd = _rng(seed + 3).choice(tets.shape[0], size=min(4, tets.shape[0]), replace=False)
    return Scene(f"small_beam_{nx}x{ny}x{nz}", X, tets, pinned, logE, nu=nu, rho=1000.0, alpha=alpha,
                 beta0=beta_rel * E_soft * contrast, h=h, gravity=np.asarray(gravity, float),
                 aa_window=aa_window, steps=steps, force_fn=force, target_centroid=target, fd_tets=fd)


def beam_batch(n: int = 64, seed: int = 4000, steps: int = 50, ne_range=(1000, 30000)) -> list:
    """A batch of uneven beams: per scene, a tet count log-uniform in ne_range
    (square cross-section of 2-6 cubes, length to match, 5 tets per cube),
    two-phase stiffness contrast log-uniform in [1, 100], nu uniform in
    [0.40, 0.49], gravity plus a seeded tip force, h = 0.01 s; Anderson window
    5 below 10x contrast, else 1."""
    rng = _rng(seed)
    out = []
    for s in range(n):
        ne = float(np.exp(rng.uniform(np.log(ne_range[0]), np.log(ne_range[1]))))
        c = int(rng.integers(2, 7))
        nx = max(2, int(round(ne / (5 * c * c))))
        contrast = float(np.exp(rng.uniform(0.0, np.log(100.0))))
        nu = float(rng.uniform(0.40, 0.49))
        sc = small_beam(nx, c, c, seed=seed + 10 * (s + 1), contrast=contrast, nu=nu, tip_force=20.0,
                        aa_window=5 if contrast < 10.0 else 1, steps=steps)
        sc.name = f"batch_beam_{s}"
        out.append(sc)
    return out


def tendon_beam(nxy: int = 4, nz: int = 16, layout: int = 0, n_seg: int = 4, seed: int = 6001, E: float = 1e5,
                nu: float = 0.45, w_m: float = 3e5, h: float = 0.01, steps: int = 100, a_max: float = 0.3,
                gravity=(0.0, 0.0, 0.0), aa_window: int = 1) -> Scene:
    """Muscle-driven beam (the paper's tendon-routing scene in shape): a vertical beam of nxy x nxy x nz
    cubes of 0.05 m along z, its base (z = 0) pinned, homogeneous Young's modulus E.  Every tet belongs to
    one of 4 n_seg muscle groups: n_seg segments along z times the four quadrants of the cross-section
    around the beam's axis.  Fibres (unit, rest coordinates): layout 0 along z; layout 1 tilted 30 degrees
    from z toward the tangential direction around the axis (a helical routing through the same volume).
    Activations are seeded uniform in [0, a_max]; the target is the rest tip position shifted sideways."""
    edge = 0.05
    X, tets = box_tet_mesh(nxy, nxy, nz, edge)
    pinned = (np.abs(X[:, 2]) < 1e-12).astype(np.uint8)
    cen = X[tets].mean(axis=1)
    axis = np.array([0.5 * nxy * edge, 0.5 * nxy * edge])
    rel = cen[:, :2] - axis
    quad = (rel[:, 0] >= 0).astype(int) + 2 * (rel[:, 1] >= 0).astype(int)
    seg = np.minimum((cen[:, 2] / (nz * edge) * n_seg).astype(int), n_seg - 1)
    group = (seg * 4 + quad).astype(np.int32)
    fib = np.zeros((tets.shape[0], 3))
    if layout == 0:
        fib[:, 2] = 1.0
    else:
        r = np.maximum(np.hypot(rel[:, 0], rel[:, 1]), 1e-12)
        tang = np.stack([-rel[:, 1] / r, rel[:, 0] / r, np.zeros_like(r)], axis=1)
        th = np.deg2rad(30.0)
        fib = np.cos(th) * np.array([0.0, 0.0, 1.0]) + np.sin(th) * tang
        fib /= np.linalg.norm(fib, axis=1, keepdims=True)
    rng = _rng(seed)
    act = rng.uniform(0.0, a_max, 4 * n_seg)
    tip = X[:, 2] > nz * edge - 1e-9
    target = X[tip].mean(axis=0) + np.array([0.1, 0.05, -0.05])
    return Scene(f"tendon_beam_{nxy}x{nz}_l{layout}", X, tets, pinned, np.full(tets.shape[0], np.log(E)), nu=nu,
                 rho=1000.0, alpha=0.01, beta0=0.0, h=h, gravity=np.asarray(gravity, float),
                 aa_window=aa_window, steps=steps, force_fn=None, target_centroid=target,
                 muscle_group=group, muscle_fibre=fib, muscle_w=w_m, activation=act)


def shell_tets(tets: np.ndarray) -> np.ndarray:
    """Mask of the tets that have a vertex on the boundary surface (a face used by one tet)."""
    faces = {}
    for t in np.asarray(tets):
        for f in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
            key = tuple(sorted(int(t[i]) for i in f))
            faces[key] = faces.get(key, 0) + 1
    bnd = np.zeros(int(np.max(tets)) + 1, dtype=bool)
    for key, c in faces.items():
        if c == 1:
            bnd[list(key)] = True
    return bnd[np.asarray(tets)].any(axis=1)


def drop_blob(res: int = 8, seed: int = 3001, n_spheres: int = 6, r_lo: float = 0.1, r_hi: float = 0.3,
              contrast: float = 100.0, nu: float = 0.49, h: float = 0.002, steps: int = 200,
              drop_speed: float = 1.0, with_box: bool = True, aa_window: int = 1, friction: float = 0.0,
              lateral: Tuple[float, float] = (0.0, 0.0)) -> Scene:
    """Contact drop: a seeded implicit blob (union of ``n_spheres`` spheres with radii uniform in [r_lo, r_hi]
    and centres uniform in a 0.3 m cube), voxelised on a grid with ``res`` cells along its largest extent
    (largest face-connected component) and split 5 tets per cube.  The shell (tets touching the boundary
    surface) is ``contrast`` times stiffer than the interior (E 1e4 Pa inside).  Nothing is pinned; the
    blob starts half a cell above the ground plane z = 0, moving down at ``drop_speed``, under gravity;
    a static box under one half of the blob rises a quarter of the blob's height above the ground.
    ``friction`` is the Coulomb coefficient of both obstacles, ``lateral`` the horizontal start velocity.
    res = 27 gives about 1e5 tets."""
    import scipy.ndimage
    rng = _rng(seed)
    cen = rng.uniform(0.0, 0.3, (n_spheres, 3))
    rad = rng.uniform(r_lo, r_hi, n_spheres)
    lo = (cen - rad[:, None]).min(axis=0)
    hi = (cen + rad[:, None]).max(axis=0)
    edge = float((hi - lo).max()) / res
    dims = np.maximum(1, np.ceil((hi - lo) / edge).astype(int))
    gi = [lo[a] + edge * (np.arange(dims[a]) + 0.5) for a in range(3)]
    P = np.stack(np.meshgrid(*gi, indexing="ij"), axis=-1)
    occ = np.zeros(tuple(dims), dtype=bool)
    for c, r in zip(cen, rad):
        occ |= ((P - c) ** 2).sum(axis=-1) <= r * r
    lab, nlab = scipy.ndimage.label(occ)
    if nlab > 1:
        sizes = np.bincount(lab.ravel())[1:]
        occ = lab == (1 + int(np.argmax(sizes)))
    X, tets = voxel_tet_mesh(occ, edge)
    X = X - X.min(axis=0)
    ext = X.max(axis=0)
    X[:, 2] += 0.5 * edge
    shell = shell_tets(tets)
    E_in = 1e4
    logE = np.where(shell, np.log(E_in * contrast), np.log(E_in))
    obs = {"planes": [((0.0, 0.0, 1.0), 0.0)], "boxes": [], "d_c": 0.25 * edge}
    if with_box:
        # the box top sits a quarter of the blob height up, under the half x > ext_x / 2; the blob starts
        # above it by half a cell
        top = 0.25 * ext[2]
        obs["boxes"].append(((0.5 * ext[0], -0.5 * ext[1], -1.0), (1.5 * ext[0], 1.5 * ext[1], top)))
        X[:, 2] += top
    target = X.mean(axis=0) + _rng(seed + 1).uniform(-0.02, 0.02, 3)
    fd = _rng(seed + 2).choice(tets.shape[0], size=min(4, tets.shape[0]), replace=False)
    return Scene(f"drop_blob_r{res}", X, tets, np.zeros(X.shape[0], np.uint8), logE, nu=nu, rho=1000.0,
                 alpha=0.01, beta0=1e-3 * E_in * contrast, h=h, gravity=np.array([0.0, 0.0, -9.81]),
                 aa_window=aa_window, steps=steps, force_fn=None, target_centroid=target, fd_tets=fd,
                 obstacles=obs, v_init=np.array([lateral[0], lateral[1], -drop_speed]), friction=friction)


def drop_family(k: int, res: int = 27, steps: int = 100, friction: float = 0.0) -> Scene:
    """Member k of a family of drops of one blob (the contact benchmark's mesh and material): the initial velocity
    is drawn from seed 3100 + k (downward speed uniform in [0.5, 1.5] m/s, horizontal components uniform in
    [-0.5, 0.5] m/s), and so is the target centroid; ``friction`` is the obstacles' Coulomb coefficient.  Members
    with different k share the mesh, so one warm-start network serves all of them; the benchmark's drop (1 m/s
    down, (0.3, 0.1) m/s sideways) is not a member."""
    sc = drop_blob(res=res, steps=steps, friction=friction)
    rng = _rng(3100 + k)
    vz = rng.uniform(0.5, 1.5)
    vx, vy = rng.uniform(-0.5, 0.5, 2)
    sc.v_init = np.array([vx, vy, -vz])
    sc.target_centroid = sc.X.mean(axis=0) + rng.uniform(-0.02, 0.02, 3)
    sc.name = f"drop_family_r{res}_{k}"
    return sc


def shape_family(k: int, res: int = 27, steps: int = 100, friction: float = 0.0) -> Scene:
    """Member k of a family of drops of different blobs (the learned start's training and held-out scenes):
    the blob is drop_blob's with seed 5000 + k (another union of spheres, so another mesh), and the initial
    velocity is drawn as in drop_family from seed 3100 + k."""
    sc = drop_blob(res=res, seed=5000 + k, steps=steps, friction=friction)
    rng = _rng(3100 + k)
    vz = rng.uniform(0.5, 1.5)
    vx, vy = rng.uniform(-0.5, 0.5, 2)
    sc.v_init = np.array([vx, vy, -vz])
    sc.target_centroid = sc.X.mean(axis=0) + rng.uniform(-0.02, 0.02, 3)
    sc.name = f"shape_family_r{res}_{k}"
    return sc


def anchored_blob(ne: float, seed: int, contrast: float = 30.0, nu: float = 0.45, steps: int = 50,
                  h: float = 0.01, tip_force: float = 20.0) -> Scene:
    """A blob without obstacles for multi-scene identification: the implicit blob of drop_blob (shape from
    `seed`) voxelised to about `ne` tets, its bottom layer of vertices pinned (a jelly fixed to a table),
    two-phase stiffness from 4 Gaussian blobs (exactly 30 % stiff, E 1e4 and 1e4 * contrast), gravity plus a
    seeded force on its x-max vertices ramped over 2 steps and held to step 4; Anderson window 5 below 10x
    contrast, else 1."""
    res = max(3, int(round((float(ne) / 1.45) ** (1.0 / 3.0))))
    base = drop_blob(res=res, seed=seed, with_box=False)
    X = base.X - base.X.min(axis=0)
    tets = base.tets
    pinned = (np.abs(X[:, 2]) < 1e-12).astype(np.uint8)
    cen = X[tets].mean(axis=1)
    ext = X.max(axis=0)
    rng = _rng(seed + 1)
    field = gaussian_blob_field(cen, np.zeros(3), ext, 4, rng, 0.05 * ext.max(), 0.15 * ext.max())
    E_soft = 1e4
    logE = two_phase_log_E(field, 0.3, E_soft, E_soft * contrast)
    force = _tip_force_fn(X, tip_force, seed + 2, 2, 4) if tip_force else None
    target = X.mean(axis=0) + _rng(seed + 3).uniform(-0.05, 0.05, 3)
    return Scene(f"anchored_blob_{seed}", X, tets, pinned, logE, nu=nu, rho=1000.0, alpha=0.01,
                 beta0=1e-2 * E_soft * contrast, h=h, gravity=np.array([0.0, 0.0, -9.81]),
                 aa_window=5 if contrast < 10.0 else 1, steps=steps, force_fn=force, target_centroid=target)


def observed_log_E(sc: Scene, seed: int) -> np.ndarray:
    """Another two-phase field on the scene's mesh for a synthetic identification task: the same two moduli
    and stiff fraction (30 %) as the scene's own field, placed by 4 Gaussian blobs drawn with `seed`."""
    cen = sc.X[sc.tets].mean(axis=1)
    lo, hi = sc.X.min(axis=0), sc.X.max(axis=0)
    ext = float((hi - lo).max())
    field = gaussian_blob_field(cen, lo, hi, 4, _rng(seed), 0.05 * ext, 0.15 * ext)
    return two_phase_log_E(field, 0.3, float(np.exp(sc.log_E.min())), float(np.exp(sc.log_E.max())))


def sysid_batch(n: int = 64, seed: int = 4000, steps: int = 50, ne_range=(1000, 30000)) -> list:
    """A batch of uneven scenes for multi-scene identification: per scene a coin flip between a beam (as in
    beam_batch) and an anchored blob, a tet count log-uniform in ne_range, contrast log-uniform in [1, 100],
    nu uniform in [0.40, 0.49].  Each scene also carries `log_E_obs`, the field of its observed trajectory
    (observed_log_E with seed + 10 (s + 1) + 7)."""
    rng = _rng(seed)
    out = []
    for s in range(n):
        ne = float(np.exp(rng.uniform(np.log(ne_range[0]), np.log(ne_range[1]))))
        contrast = float(np.exp(rng.uniform(0.0, np.log(100.0))))
        nu = float(rng.uniform(0.40, 0.49))
        if rng.random() < 0.5:
            c = int(rng.integers(2, 7))
            nx = max(2, int(round(ne / (5 * c * c))))
            sc = small_beam(nx, c, c, seed=seed + 10 * (s + 1), contrast=contrast, nu=nu, tip_force=20.0,
                            aa_window=5 if contrast < 10.0 else 1, steps=steps)
            sc.name = f"sysid_beam_{s}"
        else:
            sc = anchored_blob(ne, seed=seed + 10 * (s + 1), contrast=contrast, nu=nu, steps=steps)
            sc.name = f"sysid_blob_{s}"
        sc.log_E_obs = observed_log_E(sc, seed + 10 * (s + 1) + 7)
        out.append(sc)
    return out


def config(name: str) -> Scene:
    if name in ("c1", "c1_cantilever"):
        return cantilever_c1()
    if name in ("c2", "c2_hetero_beam"):
        return hetero_beam_c2()
    if name == "tendon":
        # the actuated tendon at the heterogeneous beam's size: 10 x 10 x 40 cubes (20,000 tets), 16 muscle groups
        # along a 30 degree helix, seeded activations up to 0.3
        return tendon_beam(nxy=10, nz=40, layout=1, steps=100, gravity=(0.0, 0.0, -9.81))
    raise KeyError(name)
