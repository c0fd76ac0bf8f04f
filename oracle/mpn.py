"""FP64 reference of the learned warm-start network (message passing on mesh
edges), for the tests only.

TEST INFRASTRUCTURE.  Nothing in the GPU library imports, loads or calls this
module; the tests, the smoke check and the benchmark's CPU leg use it to check
the GPU network.  Plain numpy in FP64, written for clarity.

The network predicts, per vertex, the correction Delta = q_{t+h} - (q_t + h v_t)
of the inertial guess, so that the first PD iterate (Alg. 1 takes q^0 = q_t)
can start closer to the converged step.  The paper has no such network; its
specification is this project's (a graph network on the tetrahedral mesh):

  x_i    = 16 node features (below)
  h0_i   = silu(x_i W_enc + b_enc)                                  (H = 64)
  layer l = 1, 2 (message passing over directed edges j -> i):
    m_ij = silu([h_i, h_j, (q_j - q_i)/ell, (X_j - X_i)/ell] W_msg + b_msg)
    a_i  = sum_j m_ij
    h_i <- h_i + silu([h_i, a_i] W_node + b_node)
  y_i    = h_i W_dec + b_dec                                         (3)
  q0_i   = q_t,i + h v_t,i + s_out y_i   (free vertices; pinned keep q_t)

Node features: (q_t - X)/ell, h (v_t - v_{t-h})/s_out (the previous step's
correction of its inertial guess), h v_t/ell, h^2 f_ext/(m s_out),
(X - X_min)/L, and the vertex's mean log(2 mu_e + lam_e) over its tets minus
the mesh mean (ell = mean edge length, L = largest bounding-box extent, m =
lumped mass, s_out = the output scale).

Parameters are one flat FP32-compatible vector in the order
W_enc (16 x H, row-major), b_enc, then per layer W_msg ((2H + 6) x H), b_msg,
W_node (2H x H), b_node, then W_dec (H x 3), b_dec.
"""
from __future__ import annotations

import numpy as np

F = 16
H = 64
LAYERS = 2
KM = 2 * H + 6


def param_shapes(h: int = H, layers: int = LAYERS):
    km = 2 * h + 6
    shapes = [(F, h), (h,)]
    for _ in range(layers):
        shapes += [(km, h), (h,), (2 * h, h), (h,)]
    shapes += [(h, 3), (3,)]
    return shapes


def n_params(h: int = H, layers: int = LAYERS) -> int:
    return int(sum(np.prod(s) for s in param_shapes(h, layers)))


def unflatten(theta, h: int = H, layers: int = LAYERS):
    out, o = [], 0
    for s in param_shapes(h, layers):
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def mesh_edges(n_v: int, tets: np.ndarray):
    """Directed edges (src j, dst i) of the tet mesh, both directions, sorted by (dst, src)."""
    pairs = set()
    for t in np.asarray(tets):
        for a in range(4):
            for b in range(a + 1, 4):
                i, j = int(t[a]), int(t[b])
                pairs.add((i, j))
                pairs.add((j, i))
    e = np.array(sorted(pairs, key=lambda p: (p[1], p[0])), dtype=np.int64)
    return e[:, 0], e[:, 1]


def mesh_constants(X: np.ndarray, src, dst):
    ell = float(np.mean(np.linalg.norm(X[src] - X[dst], axis=1)))
    L = float(np.max(X.max(axis=0) - X.min(axis=0)))
    return ell, L


def vertex_logw(n_v: int, tets: np.ndarray, w_e: np.ndarray):
    """Mean log w_e over each vertex's tets, minus the mean over vertices."""
    s = np.zeros(n_v)
    c = np.zeros(n_v)
    lw = np.log(w_e)
    for t, l in zip(np.asarray(tets), lw):
        s[t] += l
        c[t] += 1
    v = s / np.maximum(c, 1)
    return v - v.mean()


def features(q_t, v_tm1, v_t, f_ext, X, mass, logw_v, h, ell, L, s_out):
    Xmin = X.min(axis=0)
    x = np.concatenate([(q_t - X) / ell, h * (v_t - v_tm1) / s_out, h * v_t / ell,
                        h * h * f_ext / (mass[:, None] * s_out), (X - Xmin) / L, logw_v[:, None]], axis=1)
    return x


def forward(theta, x, q_t, X, src, dst, ell, h_dim: int = H, layers: int = LAYERS):
    """Returns y (n_v x 3) and the cache for backward."""
    P = unflatten(theta, h_dim, layers)
    We, be = P[0], P[1]
    z0 = x @ We + be
    hcur = silu(z0)
    n = x.shape[0]
    dxe = (q_t[src] - q_t[dst]) / ell
    dXe = (X[src] - X[dst]) / ell
    cache = dict(x=x, z0=z0, layers=[], src=src, dst=dst, dxe=dxe, dXe=dXe, n=n)
    for l in range(layers):
        Wm, bm, Wn, bn = P[2 + 4 * l: 6 + 4 * l]
        ein = np.concatenate([hcur[dst], hcur[src], dxe, dXe], axis=1)
        zm = ein @ Wm + bm
        m = silu(zm)
        a = np.zeros((n, h_dim))
        np.add.at(a, dst, m)
        nin = np.concatenate([hcur, a], axis=1)
        zn = nin @ Wn + bn
        hn = hcur + silu(zn)
        cache["layers"].append(dict(h=hcur, ein=ein, zm=zm, nin=nin, zn=zn))
        hcur = hn
    Wd, bd = P[-2], P[-1]
    y = hcur @ Wd + bd
    cache["hL"] = hcur
    return y, cache


def backward(theta, cache, dy, h_dim: int = H, layers: int = LAYERS):
    """Gradient of sum(dy * y) with respect to the flat parameters."""
    P = unflatten(theta, h_dim, layers)
    G = [np.zeros_like(p) for p in P]
    Wd = P[-2]
    G[-2] = cache["hL"].T @ dy
    G[-1] = dy.sum(axis=0)
    dh = dy @ Wd.T
    src, dst = cache["src"], cache["dst"]
    for l in reversed(range(layers)):
        c = cache["layers"][l]
        Wm, bm, Wn, bn = P[2 + 4 * l: 6 + 4 * l]
        dzn = dh * dsilu(c["zn"])
        G[4 + 4 * l] = c["nin"].T @ dzn
        G[5 + 4 * l] = dzn.sum(axis=0)
        dnin = dzn @ Wn.T
        dh_new = dh + dnin[:, :h_dim]
        da = dnin[:, h_dim:]
        dzm = da[dst] * dsilu(c["zm"])
        G[2 + 4 * l] = c["ein"].T @ dzm
        G[3 + 4 * l] = dzm.sum(axis=0)
        dein = dzm @ Wm.T
        np.add.at(dh_new, dst, dein[:, :h_dim])
        np.add.at(dh_new, src, dein[:, h_dim:2 * h_dim])
        dh = dh_new
    dz0 = dh * dsilu(cache["z0"])
    G[0] = cache["x"].T @ dz0
    G[1] = dz0.sum(axis=0)
    return flatten(G)


def loss_and_dy(y, target, free_mask, src=None, dst=None, kappa=0.0):
    """L = sum over free vertices of |r|^2 / (3 n_free) + kappa sum over the
    directed edges of |r_src - r_dst|^2 / (3 n_edges), r = (y - target) on free
    vertices and 0 on pinned ones; returns L and dL/dy."""
    nf = int(free_mask.sum())
    r = (y - target) * free_mask[:, None]
    L = float((r * r).sum() / (3 * nf))
    dy = 2.0 * r / (3 * nf)
    if kappa > 0.0:
        ne = len(src)
        de = r[src] - r[dst]
        L += kappa * float((de * de).sum()) / (3 * ne)
        g = np.zeros_like(r)
        np.add.at(g, src, 2.0 * de)
        np.add.at(g, dst, -2.0 * de)
        dy = dy + kappa * g / (3 * ne) * free_mask[:, None]
    return L, dy


def init_params(seed: int, h_dim: int = H, layers: int = LAYERS):
    """Seeded initialisation (uniform +-1/sqrt(fan_in), zero biases, small decoder)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for s in param_shapes(h_dim, layers):
        if len(s) == 2:
            parts.append(rng.uniform(-1.0, 1.0, s) / np.sqrt(s[0]))
        else:
            parts.append(np.zeros(s))
    parts[-2] *= 0.1
    return flatten(parts)


def bf16_round(a):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
