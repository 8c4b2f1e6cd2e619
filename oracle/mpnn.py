"""FP64 reference of the learned correction to the monodomain preconditioner.

Not part of the paper: a small message-passing network delta(t) added to
the Schur-complement solve P_K^-1 t of Def. 2, so that the corrected block
approximates K^-1 t instead of K_m^-1 t (Sec. 5.2 replaces K by K_m; the
network learns part of the difference).  Because the correction is
nonlinear the outer iteration becomes flexible CG.

Graph: the heart vertices with the sparsity pattern of S_m (Sec. 5.2).
Edge weights a_ij = |S_m,ij| / sum_{k != i} |S_m,ik| for j != i.

Per-vertex input features (F = 16, zero padded):
  0            t_i / rms(t), rms(t) = |t|_2 / sqrt(N_H)   (the corrected vector)
  1..         mean over the incident heart elements of the entries of sigma_i
              then of sigma_e (2D: xx, xy, yy; 3D: xx, xy, xz, yy, yz, zz),
              divided by the largest diagonal conductivity value
  next        hop distance to the boundary of the heart sub-mesh / max hops

Network (hidden width 32, ReLU):
  m0 = A f,   h1 = relu(W1s f + W1n m0 + b1)
  m1 = A h1,  h2 = relu(W2s h1 + W2n m1 + b2)
  o  = w3 . h2 + b3,     delta = rms(t) * o

Loss of one sample (t, target), with r = o - target / rms(t):
  r^T W r,  W = K_m / mean(diag K_m)   (energy of the correction error)
or r^T r when no weight matrix is given.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

from . import fem

F = 16
HID = 32

PARAM_SHAPES = [("W1s", (HID, F)), ("W1n", (HID, F)), ("b1", (HID,)),
                ("W2s", (HID, HID)), ("W2n", (HID, HID)), ("b2", (HID,)),
                ("w3", (HID,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in PARAM_SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel()
                           for name, _ in PARAM_SHAPES])


def aggregation_matrix(Sm):
    """Row-normalised |off-diagonal| pattern of S_m."""
    A = abs(sp.csr_matrix(Sm)).tolil()
    A.setdiag(0.0)
    A = A.tocsr()
    A.eliminate_zeros()
    rs = np.asarray(A.sum(axis=1)).ravel()
    rs[rs == 0] = 1.0
    return sp.diags(1.0 / rs) @ A


def heart_boundary_vertices(cfg):
    """Vertices (heart-local ids) on facets that belong to one heart element."""
    heart = cfg["region"] == fem.REGION_HEART
    el = np.sort(cfg["elems"][heart].astype(np.int64), axis=1)
    k = el.shape[1]
    facets = np.concatenate([np.delete(el, j, axis=1) for j in range(k)], axis=0)
    uniq, counts = np.unique(facets, axis=0, return_counts=True)
    bverts = np.unique(uniq[counts == 1].ravel())
    hn = fem.heart_nodes(cfg)
    loc = -np.ones(len(cfg["xyz"]), dtype=np.int64)
    loc[hn] = np.arange(len(hn))
    return loc[bverts]


def static_features(cfg, Sm):
    """(N_H, F-1) static features: conductivity entries and boundary distance."""
    d = cfg["dim"]
    heart = cfg["region"] == fem.REGION_HEART
    hn = fem.heart_nodes(cfg)
    loc = -np.ones(len(cfg["xyz"]), dtype=np.int64)
    loc[hn] = np.arange(len(hn))
    si, se, _, _, _ = fem.tensors(cfg)
    iu = np.triu_indices(d)
    ent = np.concatenate([si[heart][:, iu[0], iu[1]], se[heart][:, iu[0], iu[1]]], axis=1)
    el = loc[cfg["elems"][heart].astype(np.int64)]
    NH = len(hn)
    acc = np.zeros((NH, ent.shape[1]))
    cnt = np.zeros(NH)
    for a in range(el.shape[1]):
        np.add.at(acc, el[:, a], ent)
        np.add.at(cnt, el[:, a], 1.0)
    acc /= cnt[:, None]
    scale = max(np.max(cfg["sigma_i"]), np.max(cfg["sigma_e"]))
    acc /= scale
    # hop distance to the heart boundary over the S_m graph
    G = abs(sp.csr_matrix(Sm))
    b = heart_boundary_vertices(cfg)
    dist = csg.dijkstra(G, unweighted=True, indices=b, min_only=True)
    dist = dist / max(dist.max(), 1.0)
    feats = np.zeros((NH, F - 1))
    feats[:, :ent.shape[1]] = acc
    feats[:, ent.shape[1]] = dist
    return feats


def features(t, static):
    """Input features and rms(t) (the output scale of delta)."""
    rms = np.linalg.norm(t) / np.sqrt(len(t))
    f = np.zeros((len(t), F))
    f[:, 0] = t / rms if rms > 0 else 0.0
    f[:, 1:] = static
    return f, rms


def forward(theta, A, f):
    p = unpack(theta)
    m0 = A @ f
    z1 = f @ p["W1s"].T + m0 @ p["W1n"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    m1 = A @ h1
    z2 = h1 @ p["W2s"].T + m1 @ p["W2n"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    o = h2 @ p["w3"] + p["b3"][0]
    cache = dict(f=f, m0=m0, z1=z1, h1=h1, m1=m1, z2=z2, h2=h2)
    return o, cache


def energy_weight(Km):
    """K_m scaled to unit mean diagonal: the norm of the training loss."""
    Km = sp.csr_matrix(Km)
    return Km / Km.diagonal().mean()


def loss_and_grad(theta, A, f, y, W=None):
    """Loss r^T W r (or r^T r), r = o - y, and its gradient w.r.t. theta."""
    p = unpack(theta)
    o, c = forward(theta, A, f)
    r = o - y
    Wr = r if W is None else W @ r
    loss = float(r @ Wr)
    do = 2.0 * Wr
    g = {}
    g["w3"] = c["h2"].T @ do
    g["b3"] = np.array([do.sum()])
    dh2 = np.outer(do, p["w3"])
    dz2 = dh2 * (c["z2"] > 0)
    g["W2s"] = dz2.T @ c["h1"]
    g["W2n"] = dz2.T @ c["m1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2s"] + A.T @ (dz2 @ p["W2n"])
    dz1 = dh1 * (c["z1"] > 0)
    g["W1s"] = dz1.T @ c["f"]
    g["W1n"] = dz1.T @ c["m0"]
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def init_params(seed):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in PARAM_SHAPES:
        if name.startswith("b"):
            p[name] = np.zeros(shape)
        else:
            fan_in = shape[-1] if len(shape) > 1 else HID
            p[name] = rng.normal(0.0, 1.0 / np.sqrt(fan_in), size=shape)
    return pack(p)


# ---------------------------------------------------------------------------
# Learned Schur-complement stencil: K_m + C ~ K
#
# The network of this module, fed a constant first channel (f0 = 1) and the
# static features, gives vertex embeddings h2.  On the sparsity pattern of
# S_m the symmetric correction is
#     C_ij = dbar * (sum_a w3_a h2_ia h2_ja + b3 [i == j])
# with dbar the mean diagonal of K_m, so that K_m + C is a symmetric sparse
# approximation of the Schur complement K of Prop. 2 (which K_m replaces
# in Sec. 5.2).  Exact Schur-complement solves z* = K^-1 t are available
# from converged solves (z* = V* - V_k for the residual t_k of iteration k),
# hence the regression  C z*_k ~ t_k - K_m z*_k,  in units of dbar * rms(z*_k):
#     loss = sum_k |C^ zh_k - bh_k|^2,  zh = z*/rms(z*),
#     bh = (t - K_m z*) / (dbar rms(z*)),  C^ = C / dbar.
# ---------------------------------------------------------------------------
def static_input(static):
    f = np.zeros((static.shape[0], F))
    f[:, 0] = 1.0
    f[:, 1:] = static
    return f


def stencil_values(theta, A, f, P):
    """C^ on the pattern P (CSR, with diagonal); returns (values, cache)."""
    p = unpack(theta)
    _, c = forward(theta, A, f)
    P = sp.csr_matrix(P)
    rows = np.repeat(np.arange(P.shape[0]), np.diff(P.indptr))
    cols = P.indices
    h2 = c["h2"]
    vals = np.einsum("ka,a,ka->k", h2[rows], p["w3"], h2[cols]) + p["b3"][0] * (rows == cols)
    return vals, (c, rows, cols)


def stencil_matrix(theta, A, f, P):
    vals, (c, rows, cols) = stencil_values(theta, A, f, P)
    return sp.csr_matrix((vals, (rows, cols)), shape=P.shape)


def stencil_loss_and_grad(theta, A, f, P, Zh, Bh):
    """Loss sum_k |C^ zh_k - bh_k|^2 over samples (rows of Zh, Bh) and its
    gradient with respect to theta."""
    p = unpack(theta)
    vals, (c, rows, cols) = stencil_values(theta, A, f, P)
    C = sp.csr_matrix((vals, (rows, cols)), shape=P.shape)
    R = (C @ Zh.T).T - Bh                       # (samples, n)
    loss = float(np.sum(R * R))
    # d loss / d C_ij on the pattern
    G = 2.0 * np.sum(R[:, rows] * Zh[:, cols], axis=0)
    h2 = c["h2"]
    g = {}
    g["w3"] = np.einsum("k,ka,ka->a", G, h2[rows], h2[cols])
    g["b3"] = np.array([np.sum(G[rows == cols])])
    # d loss / d h2_i = sum_j G_ij w3 h2_j + sum_j G_ji w3 h2_j
    dh2 = np.zeros_like(h2)
    np.add.at(dh2, rows, G[:, None] * p["w3"] * h2[cols])
    np.add.at(dh2, cols, G[:, None] * p["w3"] * h2[rows])
    dz2 = dh2 * (c["z2"] > 0)
    g["W2s"] = dz2.T @ c["h1"]
    g["W2n"] = dz2.T @ c["m1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2s"] + A.T @ (dz2 @ p["W2n"])
    dz1 = dh1 * (c["z1"] > 0)
    g["W1s"] = dz1.T @ c["f"]
    g["W1n"] = dz1.T @ c["m0"]
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)
