"""Pins for the oracle's P1 assembly (Sec. 3.1) against closed forms."""
import os

import numpy as np
import pytest

import workloads as w
from oracle import fem


def _read_golden(path):
    blocks, cur = {}, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] in ("tri", "tet"):
            cur = tok[0]
            blocks[cur] = (np.array(tok[1:], float), [])
        else:
            blocks[cur][1].append([float(t) for t in tok])
    return {k: (v[0], np.array(v[1])) for k, v in blocks.items()}


def test_reference_element_matrices(golden_dir):
    g = _read_golden(os.path.join(golden_dir, "p1_reference_elements.txt"))
    for key, d in (("tri", 2), ("tet", 3)):
        xyz = g[key][0].reshape(d + 1, d)
        el = np.arange(d + 1)[None]
        S = fem.stiffness(xyz, el, np.eye(d)[None], d + 1).toarray()
        np.testing.assert_allclose(S, g[key][1], atol=1e-15)


def test_anisotropic_reference_triangle():
    # integral of sigma grad(l_a).grad(l_b): with sigma = diag(a, b) on the
    # unit right triangle the entries are (a+b, -a, -b; a, 0; b) / 2
    a, b = 3.0, 0.31
    xyz = np.array([[0, 0], [1, 0], [0, 1]], float)
    S = fem.stiffness(xyz, np.array([[0, 1, 2]]), np.diag([a, b])[None], 3).toarray()
    ref = 0.5 * np.array([[a + b, -a, -b], [-a, a, 0], [-b, 0, b]])
    np.testing.assert_allclose(S, ref, atol=1e-15)


def _uniform_heart(cfg, theta):
    cfg = dict(cfg)
    E = len(cfg["elems"])
    d = cfg["dim"]
    cfg["region"] = np.full(E, w.REGION_HEART, np.int8)
    Q = np.eye(d)
    c, s = np.cos(theta), np.sin(theta)
    Q[0, 0], Q[1, 0], Q[0, 1], Q[1, 1] = c, s, -s, c
    cfg["fibre"] = np.broadcast_to(Q, (E, d, d)).copy()
    return cfg, Q


@pytest.mark.parametrize("mk", [lambda: w.square2d(n=10),
                                lambda: w.slab3d(n=4),
                                lambda: w.thorax2d(n_target=2500, seed=3)])
def test_patch_and_kernel(mk):
    """Patch test: for u = a.x the P1 energy u^T S u equals a^T sigma a |Omega|
    for a uniform tensor; the constants are in the kernel; S is symmetric."""
    cfg, Q = _uniform_heart(mk(), 0.4)
    d = cfg["dim"]
    sig = Q @ np.diag(cfg["sigma_i"]) @ Q.T
    A = fem.assemble(cfg)
    Si = A["Si"]
    hn = A["hn"]
    x = cfg["xyz"][hn]
    vol, _ = fem.element_geometry(cfg["xyz"], cfg["elems"].astype(np.int64))
    area = vol.sum()
    rng = np.random.default_rng(0)
    for _ in range(3):
        a = rng.normal(size=d)
        u = x @ a
        np.testing.assert_allclose(u @ (Si @ u), a @ sig @ a * area, rtol=1e-12)
    np.testing.assert_allclose(Si @ np.ones(len(hn)), 0.0, atol=1e-12 * abs(Si).max())
    assert abs(Si - Si.T).max() <= 1e-14 * abs(Si).max()


def test_mass_totals():
    cfg = w.square2d(n=16)
    A = fem.assemble(cfg)
    np.testing.assert_allclose(A["m"].sum(), 100.0, rtol=1e-13)
    n_heart = int((cfg["region"] == w.REGION_HEART).sum())
    h = 10.0 / 16
    np.testing.assert_allclose(A["mH"].sum(), n_heart * h * h / 2, rtol=1e-13)
    cfg3 = w.slab3d(n=5)
    A3 = fem.assemble(cfg3)
    np.testing.assert_allclose(A3["m"].sum(), 1.0, rtol=1e-13)
    np.testing.assert_allclose(A3["mH"].sum(), 1.0, rtol=1e-13)


def test_tensors_in_fibre_frame():
    cfg, Q = _uniform_heart(w.square2d(n=4), np.deg2rad(30.0))
    si, se, s1, sebar, sm = fem.tensors(cfg)
    f = Q[:, 0]
    # the fibre is an eigenvector with the longitudinal conductivity
    np.testing.assert_allclose(si[0] @ f, cfg["sigma_i"][0] * f, atol=1e-15)
    np.testing.assert_allclose(se[0] @ f, cfg["sigma_e"][0] * f, atol=1e-15)
    # harmonic mean along each frame axis: g_i g_e / (g_i + g_e)
    gi, ge = cfg["sigma_i"], cfg["sigma_e"]
    for k in range(2):
        ax = Q[:, k]
        np.testing.assert_allclose(ax @ sm[0] @ ax, gi[k] * ge[k] / (gi[k] + ge[k]),
                                   rtol=1e-14)
    np.testing.assert_allclose(s1[0], si[0] + se[0], rtol=1e-15)
    # torso elements are isotropic with the region conductivity
    cfg2 = w.square2d(n=4)
    _, _, s1t, sebt, _ = fem.tensors(cfg2)
    tor = np.nonzero(cfg2["region"] == w.REGION_TORSO)[0][0]
    np.testing.assert_allclose(s1t[tor], 2.0 * np.eye(2))
    np.testing.assert_allclose(sebt[tor], 2.0 * np.eye(2))


def test_thorax_regions_and_heart_nodes():
    cfg = w.thorax2d(n_target=20000, seed=5)
    A = fem.assemble(cfg)
    hn = A["hn"]
    assert np.all(np.diff(hn) > 0)
    assert len(hn) == A["Si"].shape[0]
    # every stimulated vertex is a heart vertex
    assert set(np.nonzero(cfg["stim_mask"])[0]) <= set(hn.tolist())
    assert (cfg["region"] == w.REGION_LUNG).any()
