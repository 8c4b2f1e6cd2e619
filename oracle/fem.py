"""P1 finite elements: stiffness matrices and lumped mass (Sec. 3.1).

The paper's runs use CVFE with diagonal mass; on simplices its stiffness is
the P1 Galerkin stiffness with element-constant tensors, and the diagonal
mass is the row-sum lumped P1 mass.  Both are written out here directly.

Conductivity tensors follow Sec. 2: sigma_i and sigma_e are diagonal in the
local fibre frame Q (columns = fibre, sheet, normal), i.e. Q diag(g) Q^T in
the fixed basis; the torso tensor is k(x) Id, piecewise constant per organ.
The bidomain tensors of the weak form are sigma_1 = sigma_i + sigma_e in the
heart and sigma_T in the torso; Rem. 1 adds sigma_e (heart) / sigma_T
(torso) for S_e, and Sec. 5.2 defines the harmonic mean
sigma_m = (sigma_e^-1 + sigma_i^-1)^-1 for the monodomain matrix S_m.
"""
import math

import numpy as np
import scipy.sparse as sp

REGION_HEART = 1


def element_geometry(xyz, elems):
    """Per element: measure |e| and the (d+1, d) matrix G whose rows are the
    gradients of the barycentric coordinate functions."""
    x = xyz[elems]                       # (E, d+1, d)
    d = x.shape[2]
    J = np.transpose(x[:, 1:, :] - x[:, :1, :], (0, 2, 1))  # columns x_k - x_0
    det = np.linalg.det(J)
    vol = np.abs(det) / math.factorial(d)
    Jinv = np.linalg.inv(J)              # row k = grad of barycentric k (k>=1)
    G = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)
    return vol, G


def tensors(cfg, elements=None):
    """Per-element tensors (sigma_i, sigma_e, sigma_1, sigma_e_bar, sigma_m),
    for every element or for the listed `elements` only.

    sigma_i, sigma_e and sigma_m are only meaningful on heart elements; on
    torso elements they are returned as zero.
    """
    sel = slice(None) if elements is None else elements
    region = cfg["region"][sel]
    E = len(region)
    d = cfg["dim"]
    heart = region == REGION_HEART
    Q = cfg["fibre"][sel]
    si = np.einsum("eij,j,ekj->eik", Q, cfg["sigma_i"], Q)
    se = np.einsum("eij,j,ekj->eik", Q, cfg["sigma_e"], Q)
    kt = cfg["region_sigma"][region.astype(np.int64)]
    iso = kt[:, None, None] * np.eye(d)[None]
    sm = np.linalg.inv(np.linalg.inv(si) + np.linalg.inv(se))
    zero = np.zeros((E, d, d))
    h = heart[:, None, None]
    sig_i = np.where(h, si, zero)
    sig_e = np.where(h, se, zero)
    sig_1 = np.where(h, si + se, iso)
    sig_ebar = np.where(h, se, iso)
    sig_m = np.where(h, sm, zero)
    return sig_i, sig_e, sig_1, sig_ebar, sig_m


def stiffness(xyz, elems, sigma, n, index=None):
    """Assemble S_kl = sum_e |e| (G sigma G^T)_kl over the given elements.

    `index` maps global vertex ids to row/column ids of the result (default
    identity); `n` is the size of the result.
    """
    vol, G = element_geometry(xyz, elems)
    Ke = vol[:, None, None] * np.einsum("eai,eij,ebj->eab", G, sigma, G)
    v = elems if index is None else index[elems]
    k = elems.shape[1]
    rows = np.repeat(v, k, axis=1).ravel()
    cols = np.tile(v, (1, k)).ravel()
    return sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(n, n))


def lumped_mass(xyz, elems, n, index=None):
    """Row-sum lumped P1 mass: each vertex of e receives |e|/(d+1)."""
    vol, _ = element_geometry(xyz, elems)
    k = elems.shape[1]
    v = elems if index is None else index[elems]
    m = np.zeros(n)
    np.add.at(m, v.ravel(), np.repeat(vol / k, k))
    return m


def heart_nodes(cfg):
    """Heart vertices = vertices of heart elements, in ascending global id.

    This ascending order is the heart-local order of V used everywhere."""
    heart = cfg["region"] == REGION_HEART
    return np.unique(cfg["elems"][heart].ravel())


def assemble(cfg):
    """All matrices of Sec. 3.1 in global (not yet reordered) numbering.

    Returns dict with S1, Se (N x N), Si, Sm (N_H x N_H, heart-local order),
    m (lumped M diagonal, N), mH (lumped M_H diagonal, N_H), hn (heart ids).
    """
    xyz, el = cfg["xyz"], cfg["elems"].astype(np.int64)
    N = len(xyz)
    heart = cfg["region"] == REGION_HEART
    hn = heart_nodes(cfg)
    loc = -np.ones(N, dtype=np.int64)
    loc[hn] = np.arange(len(hn))
    sig_i, sig_e, sig_1, sig_ebar, sig_m = tensors(cfg)
    S1 = stiffness(xyz, el, sig_1, N)
    Se = stiffness(xyz, el, sig_ebar, N)
    Si = stiffness(xyz, el[heart], sig_i[heart], len(hn), loc)
    Sm = stiffness(xyz, el[heart], sig_m[heart], len(hn), loc)
    m = lumped_mass(xyz, el, N)
    mH = lumped_mass(xyz, el[heart], len(hn), loc)
    return dict(S1=S1, Se=Se, Si=Si, Sm=Sm, m=m, mH=mH, hn=hn, N=N,
                NH=len(hn))
